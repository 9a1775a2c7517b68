"""The proposer's allocation-free entry point (navsim_rp_propose_noalloc,
workspace in a fixed per-device array) against the allocating one
(navsim_rp_propose): same kernels, so every output must be bitwise equal, on
two calls in a row (the second smaller, leaving the first call's contents in
the array), with and without network draws; a call whose workspace would not
fit is refused before anything runs."""
import sys

import numpy as np
import pytest
import torch

from paper_2606_15846_amd import navsim as ns
from paper_2606_15846_amd.navsim import NavSim
from paper_2606_15846_amd.reset_proposal import ResetProposer
from workloads import configs

pytestmark = pytest.mark.gpu

KEYS = ("pose", "hops", "source", "checks")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _requests(n, seed):
    rng = np.random.default_rng(seed)
    return (rng.integers(0, 4, n), rng.integers(0, 8, n), rng.integers(0, 1 << 20, n),
            rng.integers(0, 50, n))


def _same(a, b, what):
    for k in KEYS + (("y",) if "y" in a else ()):
        x, y = a[k].cpu().numpy(), b[k].cpu().numpy()
        assert x.shape == y.shape, (what, k)
        assert np.array_equal(x.view(np.uint8), y.view(np.uint8)), (what, k)


def test_noalloc_propose_matches_allocating_entry_point():
    w = configs.build_workload("c5", num_envs=64)
    maps, res = w["maps"][:4], w["res"][:4]
    env_map = (np.arange(64) % 4).astype(np.int32)
    sim = NavSim(w["cfg"], maps, res, env_map, device=0)
    rp = ResetProposer(sim, **dict(w["proposer"], seed=0xBEEF))
    # a short training run so the table and weights are not the initial ones
    lab = rp.label(np.arange(64) % 4, first_sid=0)
    keep = lab["goal"] >= 0
    ids = torch.arange(64, device=sim.device, dtype=torch.int32)
    nb = rp.nb
    pairs = dict(map=(ids % 4)[:, None].expand(64, nb)[keep].contiguous(),
                 bin=torch.arange(nb, device=sim.device, dtype=torch.int32)[None, :]
                 .expand(64, nb)[keep].contiguous(),
                 start=lab["start"][:, None].expand(64, nb)[keep].contiguous(),
                 goal=lab["goal"][keep].contiguous())
    rp.train(pairs, steps=20, batch=256, samples=8)
    torch.cuda.synchronize()
    for n, M, tries, seed in ((96, 16, 60, 1), (40, 8, 30, 2), (33, 0, 80, 3)):
        say(f"noalloc propose: {n} requests x {M} draws, {tries} rejection tries (seed {seed})")
        mp, bins, env, ep = _requests(n, seed)
        a = rp.propose(mp, bins, env, ep, proposals=M, max_tries=tries, want_y=True)
        b = rp.propose(mp, bins, env, ep, proposals=M, max_tries=tries, want_y=True, noalloc=True)
        torch.cuda.synchronize()
        _same(a, b, (n, M))
        if M:
            assert (a["source"].cpu().numpy() >= 0).any()
    say("noalloc propose: a call that needs more than the fixed workspace")
    mp, bins, env, ep = _requests(4096, 4)
    with pytest.raises(ns.NavsimError, match="more than the fixed 16777216") as ei:
        rp.propose(mp, bins, env, ep, proposals=8, max_tries=1, noalloc=True)
    assert ei.value.status == -1  # NAVSIM_E_INVALID_ARG
    # the refused call launched nothing and the array still serves a call
    mp, bins, env, ep = _requests(12, 5)
    a = rp.propose(mp, bins, env, ep, proposals=4, max_tries=10)
    b = rp.propose(mp, bins, env, ep, proposals=4, max_tries=10, noalloc=True)
    torch.cuda.synchronize()
    _same(a, b, "after the refused call")
    rp.close()
    sim.close()
