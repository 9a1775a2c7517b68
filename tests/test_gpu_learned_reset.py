"""GPU parity of learned resets inside the step (navsim_rp_attach, the sparse
reset of section 2.2.3 drawn by the proposer): one navsim_step call defers
the resets of envs with a requested difficulty bin, proposes and verifies
their pairs and applies them in a masked reset pass.

Against the oracle (orc_step_defer, then orc_reset for the envs left to the
free-space sampler): flags, reward, hit ids, ranges, final observations and
the state of every other env as in the plain step parity.  A pair taken from
the network is one of many valid pairs (the network's float outputs decide
it), so it is checked for validity with the oracle's own geodesic search
(C-free cells, hop count in the requested bin, goal distance), and its state
and reset observation against orc_reset_to from that pair; a pair from a
rejection attempt is unique and must equal the oracle's rejection sampler
bitwise; requests past the per-step cap and requests with no valid pair
must equal the free-space sampler bitwise."""
import sys

import numpy as np
import pytest
import torch

import oracle
from oracle import geodesic as G
from paper_2606_15846_amd.navsim import NavSim, NavsimError
from paper_2606_15846_amd.reset_proposal import ResetProposer
from tests import parity
from workloads import configs

pytestmark = pytest.mark.gpu

N, NMAPS, PROPS, TRIES, CAP = 192, 4, 16, 60, 40


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def setup(n=N):
    w = configs.build_workload("c5", num_envs=n)
    maps, res = w["maps"][:NMAPS], w["res"][:NMAPS]
    env_map = (np.arange(n) % NMAPS).astype(np.int32)
    cfg = w["cfg"]
    sim = NavSim(cfg, maps, res, env_map, device=0)
    pcfg = dict(w["proposer"], seed=0xABCD)
    rp = ResetProposer(sim, **pcfg)
    ref = oracle.OracleSim(cfg, maps, res, env_map)
    reach = []
    M = ref.maps
    for k in range(NMAPS):
        cf = np.zeros(maps[k].size, np.uint8)
        cf[M.free_cells[M.free_off[k]:M.free_off[k] + M.free_cnt[k]]] = 1
        reach.append(G.ReachMap(cf.reshape(maps[k].shape), res[k], seed=pcfg["seed"],
                                d_lo=pcfg["d_lo_m"], d_hi=pcfg["d_hi_m"],
                                nbins=pcfg["num_bins"], gmd=cfg["goal_min_dist_m"]))
    # a short training run, so that some pairs come from the network
    lab = rp.label(np.arange(256) % NMAPS, first_sid=0)
    keep = lab["goal"] >= 0
    ids = torch.arange(256, device=sim.device, dtype=torch.int32)
    nb = rp.nb
    pairs = dict(map=(ids % NMAPS)[:, None].expand(256, nb)[keep].contiguous(),
                 bin=torch.arange(nb, device=sim.device, dtype=torch.int32)[None, :]
                 .expand(256, nb)[keep].contiguous(),
                 start=lab["start"][:, None].expand(256, nb)[keep].contiguous(),
                 goal=lab["goal"][keep].contiguous())
    rp.train(pairs, steps=300, batch=256, samples=8, lr=2e-3)
    torch.cuda.synchronize()
    return sim, rp, ref, reach


def apply_deferred(sim, rp, ref, reach, ref_out, deferred, bins, pre_ep, label):
    """Completes the oracle side of the deferred resets from what the GPU
    chose (validity-checked) and returns counters; ref_out's obs and
    fallback rows of the deferred envs are replaced by the oracle's."""
    src, hops = (t.cpu().numpy() for t in rp.attach_outputs())
    st = sim.get_state()
    n = sim.N
    order = np.nonzero(deferred)[0]
    assert np.all(src[order[CAP:]] == -1), f"{label}: envs past the cap got pairs"
    prop = np.zeros(n, bool)
    prop[order] = src[order] >= 0
    free = deferred & ~prop
    pose = np.zeros((n, 5), np.float32)
    n_net = n_rej = 0
    for e in np.nonzero(prop)[0]:
        R = reach[e % NMAPS]
        a = int(np.floor(st["y"][e] / R.s)) * R.W + int(np.floor(st["x"][e] / R.s))
        b = int(np.floor(st["gy"][e] / R.s)) * R.W + int(np.floor(st["gx"][e] / R.s))
        assert (st["x"][e], st["y"][e]) == R.centre(a), f"{label}: env {e} start off-centre"
        assert (st["gx"][e], st["gy"][e]) == R.centre(b), f"{label}: env {e} goal off-centre"
        ok, h = R.verify(a, b, int(bins[e]))
        assert ok and h == hops[e], f"{label}: env {e} pair invalid ({ok}, {h}, {hops[e]})"
        if src[e] >= PROPS:
            t, ra, rb, rh, th = R.reject(e, int(pre_ep[e]), int(bins[e]), TRIES,
                                         with_heading=True)
            assert (src[e], ra, rb, rh) == (PROPS + t, a, b, h), f"{label}: env {e} rejection"
            assert st["th"][e] == np.float32(th), f"{label}: env {e} heading"
            n_rej += 1
        else:
            assert -np.pi <= st["th"][e] <= np.pi
            n_net += 1
        pose[e] = (st["x"][e], st["y"][e], st["th"][e], st["gx"][e], st["gy"][e])
    obs_p = ref.reset_to(pose, prop.astype(np.uint8))
    obs_f, fb = ref.reset(free.astype(np.uint8))
    ref_out["obs"][prop] = obs_p[prop]
    ref_out["obs"][free] = obs_f[free]
    ref_out["fallback"][free] = fb[free]
    ref_out["fallback"][prop] = 0
    return dict(deferred=int(deferred.sum()), network=n_net, rejection=n_rej,
                free=int(free.sum()))


def test_learned_resets_inside_the_step_against_oracle():
    sim, rp, ref, reach = setup()
    sim.reset()
    ref.reset(threads=8)
    torch.cuda.synchronize()
    st = sim.get_state()
    for k in oracle.STATE_KEYS:
        assert np.array_equal(st[k], ref.state[k]), k
    bins = np.where(np.arange(N) % 5 != 4, np.arange(N) % 8, -1).astype(np.int32)
    rp.attach(bins, proposals=PROPS, max_tries=TRIES, max_per_step=CAP)
    acts = configs.uniform_actions(6, N, seed=17)
    tot = dict(deferred=0, network=0, rejection=0, free=0)
    for step in range(6):
        # the oracle's own state (bitwise the GPU's: compare_step asserts it)
        st = ref.get_state()
        if step % 2 == 0:
            st["t"][(np.arange(N) + step) % 3 == 0] = 199  # a third truncate now
            sim.set_state(st)
            ref.set_state(st)
        g, gst = parity.gpu_step(sim, acts[step], kernel=0)
        r = ref.step(acts[step], threads=8, defer_bin=bins)
        deferred = r["reset"].astype(bool) & (bins >= 0)
        c = apply_deferred(sim, rp, ref, reach, r, deferred, bins, st["ep"], f"step {step}")
        for k in tot:
            tot[k] += c[k]
        rep = parity.compare_step(g, r, gst, ref, label=f"step {step}")
        say(f"step {step}: {c}, resets {rep['resets']}, grazing {rep['grazing']}")
    stats = rp.attach_stats()
    say(f"totals {tot}; library stats {stats}")
    assert stats["deferred"] == tot["deferred"]
    assert stats["requests"] + stats["over_cap"] == stats["deferred"]
    assert stats["from_network"] == tot["network"]
    assert stats["from_rejection"] == tot["rejection"]
    assert stats["over_cap"] > 0 and tot["network"] > 0 and tot["rejection"] > 0
    rp.close()
    sim.close()


@pytest.mark.parametrize("n", [N, 200])  # 200: envs past the last 16-env block of the compaction
def test_learned_resets_in_masked_reset_and_detach(n):
    sim, rp, ref, reach = setup(n)
    sim.reset()
    ref.reset(threads=8)
    torch.cuda.synchronize()
    bins = (np.arange(n) % 8).astype(np.int32)
    rp.attach(bins, proposals=PROPS, max_tries=TRIES, max_per_step=CAP)
    mask = (np.arange(n) % 3 == 1).astype(np.uint8)
    pre = ref.get_state()
    g0 = sim.get_state()
    for k in oracle.STATE_KEYS:
        assert np.array_equal(g0[k], pre[k]), k
    obs = sim.reset(torch.from_numpy(mask).to(sim.device)).cpu().numpy()
    torch.cuda.synchronize()
    r = {"obs": np.zeros((n, sim.m + 4), np.float32), "fallback": np.zeros(n, np.uint8)}
    c = apply_deferred(sim, rp, ref, reach, r, mask.astype(bool), bins, pre["ep"], "reset")
    say(f"masked reset: {c}")
    gst = sim.get_state()
    for k in oracle.STATE_KEYS:
        assert np.array_equal(gst[k], ref.state[k]), k
    m = sim.m
    rows = np.nonzero(mask)[0]
    rg = parity.reset_scan_grazing(ref, rows)
    for e in rows:
        sg = rg[int(e)].reshape(m, -1).any(axis=1)
        d = np.abs(obs[e, :m] - r["obs"][e, :m])
        assert d[~sg].max(initial=0.0) <= parity.RANGE_TOL, (e, d.max())
        assert np.abs(obs[e, m:] - r["obs"][e, m:]).max() <= parity.SCALAR_TOL
    # while attached, the plain step and rollouts refuse; after detach the
    # step is the plain free-space one again
    act = torch.from_numpy(configs.uniform_actions(1, n, seed=3)[0]).to(sim.device)
    with pytest.raises(NavsimError, match="fused step only"):
        sim.step(act, plain=True)
    with pytest.raises(NavsimError, match="detach"):
        sim.rollout(4, first_step=0, buffers=sim.rollout_buffers(4), graph=False)
    rp.detach()
    g, gst = parity.gpu_step(sim, act.cpu().numpy(), kernel=0)
    r = ref.step(act.cpu().numpy(), threads=8)
    parity.compare_step(g, r, gst, ref, label="after detach")
    rp.close()
    sim.close()
