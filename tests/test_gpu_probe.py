"""The LDS bandwidth probe (include/navsim_probe.h) reads what it says it
reads: the words each thread stores equal a host recomputation of the xor of
every 16-byte word its documented read pattern visits."""
import numpy as np
import pytest

from paper_2606_15846_amd import navsim


def _expected(threads: int, blocks: int, iters: int) -> np.ndarray:
    i = np.arange(4096, dtype=np.uint64)
    m = np.uint64(0xFFFFFFFF)
    f = (((i * np.uint64(2654435761)) & m) ^ (i ^ np.uint64(0x9E3779B9)) ^ ((i + np.uint64(7)) & m)
         ^ (~i & m)).astype(np.uint32)
    t = np.arange(threads)
    acc = np.zeros(threads, np.uint32)
    for it in range(iters):
        base = (t + 64 * it) & 255
        for k in range(16):
            acc ^= f[base + 256 * k]
    return np.tile(acc, blocks)


@pytest.mark.gpu
@pytest.mark.parametrize("threads,iters", [(256, 1), (512, 3), (1024, 7)])
def test_lds_probe_words_and_bytes(threads, iters):
    blocks = 300
    ms, nb, words = navsim.navsim_probe_lds_read(0, threads, blocks, iters, 2, want_words=True)
    assert ms > 0.0
    assert nb == blocks * threads * iters * 16 * 16
    np.testing.assert_array_equal(words, _expected(threads, blocks, iters))
