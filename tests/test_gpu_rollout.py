"""Device rollouts (navsim_rollout): in-kernel Philox actions and HIP-graph
replay, against the oracle and against single steps."""
import math
import sys

import numpy as np
import pytest
import torch

import oracle
from paper_2606_15846_amd.navsim import NAVSIM_KERNEL_FUSED, NAVSIM_KERNEL_PLAIN, NavSim
from tests.parity import compare_rollout
from workloads import configs

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def host(b: dict) -> dict:
    torch.cuda.synchronize()
    return {k: (v.cpu().numpy().copy() if v is not None else None) for k, v in b.items()}


def pair(w, num_envs=None):
    cfg = dict(w["cfg"])
    sim = NavSim(cfg, w["maps"], w["res"], w["env_map"], device=0, profiles=w["profiles"])
    ref = oracle.OracleSim(cfg, w["maps"], w["res"], w["env_map"], profiles=w["profiles"])
    return sim, ref


def start(sim, ref):
    sim.reset()
    ref.reset(threads=16)
    torch.cuda.synchronize()
    st = sim.get_state()
    for k in oracle.STATE_KEYS:
        assert np.array_equal(st[k], ref.state[k])
    return st


@pytest.mark.parametrize("graph", [True, False])
def test_c1_rollout_64_steps_against_oracle(graph):
    say(f"c1 rollout, 64 steps, graph={graph}")
    w = configs.build_workload("c1")
    sim, ref = pair(w)
    start(sim, ref)
    b = host(sim.rollout(64, first_step=1000, graph=graph))
    tot = compare_rollout(b, ref, 1000, label=f"c1 graph={graph}")
    st = sim.get_state()
    for k in oracle.STATE_KEYS:
        assert np.array_equal(st[k], ref.state[k]), k
    assert tot["resets"] > 0
    say(f"c1 rollout: {tot}")
    sim.close()


def test_rollout_equals_single_steps_and_graph_replays():
    say("c2 maps, 512 envs: graph rollout == eager rollout == single steps; 3 replays")
    w = configs.build_workload("c2", num_envs=512)
    sim, ref = pair(w)
    s0 = start(sim, ref)
    T = 16
    # single steps with the oracle's draws of the rollout actions
    singles = []
    for t in range(T):
        a = torch.from_numpy(ref.rollout_actions(77 + t)).to(sim.device)
        obs, rew, term, trunc, info = sim.step(a)
        torch.cuda.synchronize()
        singles.append(dict(obs=obs.cpu().numpy().copy(), reward=rew.cpu().numpy().copy(),
                            terminated=term.cpu().numpy().copy(),
                            truncated=trunc.cpu().numpy().copy()))
    s_end = sim.get_state()
    sim.set_state(s0)
    eager = host(sim.rollout(T, first_step=77, graph=False))
    assert all(np.array_equal(sim.get_state()[k], s_end[k]) for k in oracle.STATE_KEYS)
    for t in range(T):
        for k in singles[t]:
            assert np.array_equal(eager[k][t], singles[t][k]), (t, k)
    bufs = sim.rollout_buffers(T)
    for rep in range(3):
        sim.set_state(s0)
        junk = torch.randn(1 << 20, device=sim.device).sum()  # eager work between replays
        g = host(sim.rollout(T, first_step=77, buffers=bufs, graph=True))
        assert float(junk.item()) == float(junk.item())
        for k in eager:
            assert np.array_equal(g[k], eager[k]), (rep, k)
        st = sim.get_state()
        assert all(np.array_equal(st[k], s_end[k]) for k in oracle.STATE_KEYS), rep
    # the plain kernel's rollout gives the same results
    sim.set_state(s0)
    pl = host(sim.rollout(T, first_step=77, kernel=NAVSIM_KERNEL_PLAIN, graph=True))
    for k in eager:
        assert np.array_equal(pl[k], eager[k]), k
    sim.close()


def test_graph_recaptured_for_new_buffers_steps_and_tuning():
    say("graph cache: new buffers, new step count, new launch shape")
    w = configs.build_workload("c2", num_envs=300)
    sim, ref = pair(w)
    s0 = start(sim, ref)
    want = host(sim.rollout(8, first_step=5, graph=False))
    s8 = sim.get_state()
    for case in ("same", "new_buffers", "tuning", "persist", "threads", "claim", "first_step"):
        sim.set_state(s0)
        if case == "tuning":
            sim.set_tuning(8, 32, 2)
        if case == "persist":  # persistent workgroups, replayed from the graph
            sim.set_tuning(4, 48, 4, persist=2)
        if case == "threads":
            sim.set_tuning(16, 48, 4, threads=1024)
        if case == "claim":
            sim.set_tuning(4, 56, 8, walk=4, balance=1)
        if case == "first_step":
            sim.rollout(4, first_step=5, graph=True)
            torch.cuda.synchronize()
            got = host(sim.rollout(4, first_step=9, graph=True))
            for k in want:
                assert np.array_equal(got[k], want[k][4:] if want[k] is not None else None), k
        else:
            got = host(sim.rollout(8, first_step=5, graph=True))
            for k in want:
                assert np.array_equal(got[k], want[k]), (case, k)
        st = sim.get_state()
        assert all(np.array_equal(st[k], s8[k]) for k in oracle.STATE_KEYS), case
    sim.close()


def test_mixed_profiles_graph_rollout_against_oracle():
    say("c4 maps and profiles, 4096 envs, 16-step graph rollout")
    w = configs.build_workload("c4")
    # every 8th env, so all 128 maps and profiles appear
    keep = np.arange(0, w["cfg"]["num_envs"], 8)
    w["cfg"]["num_envs"] = len(keep)
    w["env_map"] = np.asarray(w["env_map"])[keep]
    sim, ref = pair(w)
    start(sim, ref)
    b = host(sim.rollout(16, first_step=(3 << 32) + 11, graph=True))
    tot = compare_rollout(b, ref, (3 << 32) + 11, label="c4-sub")
    st = sim.get_state()
    for k in oracle.STATE_KEYS:
        assert np.array_equal(st[k], ref.state[k]), k
    say(f"c4 rollout: {tot}")
    sim.close()


def test_rollout_argument_errors():
    w = configs.build_workload("c1")
    sim, _ = pair(w)
    from paper_2606_15846_amd import navsim
    b = sim.rollout_buffers(4)
    with pytest.raises(navsim.NavsimError):  # reset has not been called
        sim.rollout(4, 0, buffers=b)
    sim.reset()
    with pytest.raises(ValueError):
        sim.rollout(5, 0, buffers=b)
    lib = navsim.load_library()
    args = [b["act"].data_ptr(), b["obs"].data_ptr(), b["reward"].data_ptr(),
            b["terminated"].data_ptr(), b["truncated"].data_ptr(), None]
    assert lib.navsim_rollout(sim.h, 0, 0, *args, 0, 1, None) == -1
    assert lib.navsim_rollout(sim.h, 5000, 0, *args, 0, 1, None) == -1
    assert lib.navsim_rollout(sim.h, 4, 0, *args, 7, 1, None) == -1
    assert lib.navsim_rollout(sim.h, 4, 0, *args, 0, 8, None) == -1
    assert lib.navsim_rollout(sim.h, 4, 0, args[0], None, *args[2:], 0, 1, None) == -1
    assert lib.navsim_rollout(None, 4, 0, *args, 0, 1, None) == -2
    torch.cuda.synchronize()
    sim.close()
