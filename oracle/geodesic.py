"""Oracle side of the learned reset proposal: ctypes wrappers over
``geodesic_oracle.c`` (TEST INFRASTRUCTURE ONLY, like the rest of the package).

A ``ReachMap`` holds one map's C-free mask and C-free cell list (from the
oracle's free-cell lists, i.e. the circumscribed-disc clearance test at cell
centres) and answers geodesic, labelling, rejection and verification queries.
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import lib as _lib

P = C.POINTER
_DONE = False


def _L():
    global _DONE
    L = _lib()
    if not _DONE:
        i32, f64, u8p, i32p = C.c_int32, C.c_double, P(C.c_uint8), P(C.c_int32)
        L.orc_bfs_field.argtypes = [i32, i32, u8p, i32, i32, i32p]
        L.orc_bin_of.argtypes = [f64, i32, f64, f64, i32]
        L.orc_bin_of.restype = i32
        L.orc_max_hops.argtypes = [f64, f64, f64, i32]
        L.orc_max_hops.restype = i32
        L.orc_cell_dist.argtypes = [i32, f64, i32, i32]
        L.orc_cell_dist.restype = f64
        L.orc_label_start.argtypes = [i32, i32, f64, u8p, i32p, C.c_int64, P(C.c_uint32),
                                      C.c_uint32, f64, f64, i32, f64, i32p, i32p]
        L.orc_label_start.restype = i32
        L.orc_verify_pair.argtypes = [i32, i32, f64, u8p, i32, i32, i32, f64, f64, i32, f64, i32p]
        L.orc_verify_pair.restype = i32
        L.orc_reject_sample.argtypes = [i32, i32, f64, u8p, i32p, C.c_int64, P(C.c_uint32),
                                        C.c_uint32, C.c_uint32, i32, i32, f64, f64, i32, f64,
                                        i32p, i32p, i32p, P(C.c_float)]
        L.orc_reject_sample.restype = i32
        L.orc_snap_cell.argtypes = [i32, i32, u8p, i32]
        L.orc_snap_cell.restype = i32
        L.orc_pool32.argtypes = [i32, i32, u8p, P(C.c_float)]
        L.orc_decode_proposal.argtypes = [i32, i32, P(C.c_float), i32p, i32p, P(C.c_float)]
        _DONE = True
    return L


def _p(a, t):
    return a.ctypes.data_as(P(t))


def bin_of(s: float, hops: int, d_lo: float, d_hi: float, nbins: int) -> int:
    return int(_L().orc_bin_of(float(s), int(hops), float(d_lo), float(d_hi), int(nbins)))


def max_hops(s: float, d_lo: float, d_hi: float, nbins: int) -> int:
    return int(_L().orc_max_hops(float(s), float(d_lo), float(d_hi), int(nbins)))


def bfs_field(cfree: np.ndarray, a: int, max_hops_: int) -> np.ndarray:
    H, W = cfree.shape
    cf = np.ascontiguousarray(cfree, dtype=np.uint8)
    out = np.zeros(W * H, np.int32)
    _L().orc_bfs_field(W, H, _p(cf, C.c_uint8), int(a), int(max_hops_), _p(out, C.c_int32))
    return out.reshape(H, W)


def pool32(occ: np.ndarray) -> np.ndarray:
    H, W = occ.shape
    o = np.ascontiguousarray(occ, dtype=np.uint8)
    out = np.zeros(1024, np.float32)
    _L().orc_pool32(W, H, _p(o, C.c_uint8), _p(out, C.c_float))
    return out


def decode_proposal(W: int, H: int, y) -> tuple[int, int, float]:
    y = np.ascontiguousarray(y, dtype=np.float32)
    a, b, th = C.c_int32(), C.c_int32(), C.c_float()
    _L().orc_decode_proposal(W, H, _p(y, C.c_float), C.byref(a), C.byref(b), C.byref(th))
    return a.value, b.value, th.value


class ReachMap:
    """One map's reachability queries.  cfree: [H, W] uint8 mask of C-free
    cells; bins: nbins equal intervals of [d_lo, d_hi) metres."""

    def __init__(self, cfree: np.ndarray, res: float, seed: int, d_lo: float = 1.0,
                 d_hi: float = 12.0, nbins: int = 8, gmd: float = 1.0):
        self.cfree = np.ascontiguousarray(cfree, dtype=np.uint8)
        self.H, self.W = self.cfree.shape
        self.s = float(np.float32(res))
        self.free = np.ascontiguousarray(np.nonzero(self.cfree.ravel())[0].astype(np.int32))
        self.key = np.array([seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF], np.uint32)
        self.d_lo, self.d_hi, self.nbins = float(d_lo), float(d_hi), int(nbins)
        self.gmd = float(np.float32(gmd))
        self.depth = max_hops(self.s, self.d_lo, self.d_hi, self.nbins)

    def _args(self):
        return (self.W, self.H, self.s, _p(self.cfree, C.c_uint8))

    def label_start(self, sid: int):
        g = np.zeros(self.nbins, np.int32)
        h = np.zeros(self.nbins, np.int32)
        a = _L().orc_label_start(*self._args(), _p(self.free, C.c_int32), len(self.free),
                                 _p(self.key, C.c_uint32), int(sid) & 0xFFFFFFFF, self.d_lo,
                                 self.d_hi, self.nbins, self.gmd, _p(g, C.c_int32),
                                 _p(h, C.c_int32))
        return int(a), g, h

    def verify(self, a: int, b: int, k: int):
        h = C.c_int32()
        ok = _L().orc_verify_pair(*self._args(), int(a), int(b), int(k), self.d_lo, self.d_hi,
                                  self.nbins, self.gmd, C.byref(h))
        return bool(ok), h.value

    def reject(self, e: int, ep: int, k: int, max_tries: int, with_heading: bool = False):
        a, b, h, th = C.c_int32(), C.c_int32(), C.c_int32(), C.c_float()
        t = _L().orc_reject_sample(*self._args(), _p(self.free, C.c_int32), len(self.free),
                                   _p(self.key, C.c_uint32), int(e), int(ep), int(k),
                                   int(max_tries), self.d_lo, self.d_hi, self.nbins, self.gmd,
                                   C.byref(a), C.byref(b), C.byref(h), C.byref(th))
        if with_heading:
            return int(t), a.value, b.value, h.value, th.value
        return int(t), a.value, b.value, h.value

    def snap(self, c: int) -> int:
        return int(_L().orc_snap_cell(self.W, self.H, _p(self.cfree, C.c_uint8), int(c)))

    def centre(self, c: int) -> tuple[float, float]:
        """Cell centre in metres, float32 as the reset poses store it."""
        return (float(np.float32((c % self.W + 0.5) * self.s)),
                float(np.float32((c // self.W + 0.5) * self.s)))

    def bin_of(self, hops: int) -> int:
        return bin_of(self.s, hops, self.d_lo, self.d_hi, self.nbins)

    def cell_dist(self, a: int, b: int) -> float:
        return float(_L().orc_cell_dist(self.W, self.s, int(a), int(b)))
