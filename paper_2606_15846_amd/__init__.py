"""navsim: the batched bitmap navigation step of FlashNav (arXiv 2606.15846,
section 2.2) as HIP kernels for MI355X behind a C ABI (include/navsim.h).

``paper_2606_15846_amd.navsim`` is the Python binding of libnavsim.so.
"""
from . import navsim  # noqa: F401
from .navsim import NavSim, NavsimError  # noqa: F401
