"""Helpers for GPU-vs-oracle comparisons (imported by the GPU tests).

Acceptance, from identical float32 states:
  * bitwise: collision, goal, terminated, truncated, reset flags, the whole
    post-step state (including reset poses and goals), hit cell ids and cell
    visit counts of non-grazing rays;
  * |range_gpu - range_oracle| <= 1e-4 m on non-grazing rays, and on pooled
    sectors that contain no grazing ray;
  * goal distance / bearing within 1e-5 (float32 of the same double values);
  * reward within 1e-5.
A ray is grazing when the oracle finds it passes within 1e-6 m of a grid
corner, ends within 1e-6 m of r_max, or starts within 1e-6 m of a grid line;
such rays are counted and reported, not failed.
"""
from __future__ import annotations

import numpy as np
import torch

import oracle

RANGE_TOL = 1e-4
SCALAR_TOL = 1e-5


def env_beams(ref: oracle.OracleSim) -> np.ndarray:
    """Beam count of every env (per-map profiles, else the configuration's)."""
    if ref.maps.profiles is None:
        return np.full(ref.N, ref.K, dtype=np.int64)
    return ref.maps.p_beams.astype(np.int64)[ref.env_map]


def sectors_with_grazing(grazing: np.ndarray, m: int, kenv: np.ndarray) -> np.ndarray:
    """Per (env, sector): does the sector hold a grazing ray.  Env e's beams
    are the first kenv[e] entries of its row, kenv[e] / m per sector."""
    n = grazing.shape[0]
    out = np.zeros((n, m), dtype=bool)
    for k in np.unique(kenv):
        rows = kenv == k
        out[rows] = grazing[rows, :k].reshape(-1, m, k // m).any(axis=2)
    return out


def reset_scan_grazing(ref: oracle.OracleSim, rows) -> dict:
    """Grazing flags of the reset observation's scan, per reset env."""
    out = {}
    for e in rows:
        st = ref.state
        _, _, gr, _ = ref.scan(int(ref.env_map[e]), st["x"][e], st["y"][e], st["th"][e])
        out[int(e)] = gr.astype(bool)
    return out


def compare_step(gpu: dict, ref_out: dict, gpu_state: dict, ref: oracle.OracleSim,
                 label: str = "") -> dict:
    """Assert the acceptance rules; returns counters for reporting."""
    kenv = env_beams(ref)
    for key in ("collision", "goal", "reset", "terminated", "truncated", "fallback"):
        g = gpu[key]
        r = ref_out[key]
        bad = np.nonzero(g != r)[0]
        assert bad.size == 0, f"{label}: {key} differs at envs {bad[:8]} gpu={g[bad[:8]]} ref={r[bad[:8]]}"
    graze = ref_out["grazing"].astype(bool)
    live = ~graze
    hg, hr = gpu["hits"], ref_out["hits"]
    bad = np.argwhere((hg != hr) & live)
    assert bad.size == 0, f"{label}: hit cells differ at (env, beam) {bad[:8].tolist()}"
    vg, vr = gpu["visits"], ref_out["visits"]
    bad = np.argwhere((vg != vr) & live)
    assert bad.size == 0, f"{label}: visit counts differ at {bad[:8].tolist()}"
    dr = np.abs(gpu["ranges"] - ref_out["ranges"])
    assert dr[live].max(initial=0.0) <= RANGE_TOL, f"{label}: range diff {dr[live].max()}"
    for k in oracle.STATE_KEYS:
        bad = np.nonzero(gpu_state[k] != ref.state[k])[0]
        assert bad.size == 0, (f"{label}: state {k} differs at envs {bad[:8]} "
                               f"gpu={gpu_state[k][bad[:8]]} ref={ref.state[k][bad[:8]]}")
    n_reset_graze = compare_outputs(gpu, ref_out, ref, label)
    return dict(rays=int(kenv.sum()), grazing=int(graze.sum()),
                grazing_mismatch=int(((hg != hr) & graze).sum()),
                resets=int(ref_out["reset"].sum()), reset_grazing=n_reset_graze,
                visits=int(vr.sum()))


def compare_outputs(gpu: dict, ref_out: dict, ref: oracle.OracleSim, label: str = "") -> int:
    """Reward, terminated/truncated, O_{t+1} (final_obs of the envs that ended,
    obs otherwise) and the reset observations, against one oracle step whose
    post-step state ref holds.  Returns the reset scans' grazing ray count."""
    m = ref.m
    for key in ("terminated", "truncated"):
        bad = np.nonzero(gpu[key] != ref_out[key])[0]
        assert bad.size == 0, f"{label}: {key} differs at envs {bad[:8]}"
    graze = ref_out["grazing"].astype(bool)
    dreward = np.abs(gpu["reward"] - ref_out["reward"]).max()
    assert dreward <= SCALAR_TOL, f"{label}: reward diff {dreward}"
    # observations: O_{t+1} (final_obs rows for envs that ended, obs otherwise)
    done = ref_out["reset"].astype(bool)
    sec_g = sectors_with_grazing(graze, m, env_beams(ref))
    pre_g = np.where(done[:, None], gpu["final_obs"], gpu["obs"])
    pre_r = np.where(done[:, None], ref_out["final_obs"], ref_out["obs"])
    d = np.abs(pre_g[:, :m] - pre_r[:, :m])
    assert d[~sec_g].max(initial=0.0) <= RANGE_TOL, f"{label}: pooled obs diff {d[~sec_g].max()}"
    ds = np.abs(pre_g[:, m:m + 2] - pre_r[:, m:m + 2]).max(initial=0.0)
    assert ds <= SCALAR_TOL, f"{label}: goal features diff {ds}"
    assert np.array_equal(pre_g[:, m + 2:], pre_r[:, m + 2:]), f"{label}: velocity obs differ"
    # reset observations Õ of the envs that ended
    rows = np.nonzero(done)[0]
    rg = reset_scan_grazing(ref, rows)
    n_reset_graze = 0
    for e in rows:
        sg = rg[int(e)].reshape(m, -1).any(axis=1)
        n_reset_graze += int(rg[int(e)].sum())
        d = np.abs(gpu["obs"][e, :m] - ref_out["obs"][e, :m])
        assert d[~sg].max(initial=0.0) <= RANGE_TOL, f"{label}: reset obs env {e} diff {d.max()}"
        ds = np.abs(gpu["obs"][e, m:] - ref_out["obs"][e, m:]).max()
        assert ds <= SCALAR_TOL, f"{label}: reset obs scalars env {e} diff {ds}"
    return n_reset_graze


def gpu_step(sim, act_np: np.ndarray, kernel: int) -> tuple[dict, dict]:
    """One debug step on the GPU; returns host copies of outputs and state."""
    act = torch.from_numpy(np.ascontiguousarray(act_np)).to(sim.device)
    dbg = sim.step_debug(act, kernel=kernel)
    torch.cuda.synchronize(sim.device)
    out = {k: v.cpu().numpy() for k, v in dbg.items()}
    out.update(obs=sim.obs.cpu().numpy().copy(), final_obs=sim.final_obs.cpu().numpy().copy(),
               reward=sim.reward.cpu().numpy().copy(),
               terminated=sim.terminated.cpu().numpy().copy(),
               truncated=sim.truncated.cpu().numpy().copy())
    return out, sim.get_state()


def compare_rollout(bufs: dict, ref: oracle.OracleSim, first_step: int, label: str = "",
                    threads: int = 16) -> dict:
    """A device rollout (host copies of its [steps] buffers) against the oracle
    run free from the same start state under its own draws of the same
    actions.  Poses, goals, counters and flags do not depend on ranges, so the
    oracle's state stays bitwise on the device's path; ranges are held to the
    step tolerance outside grazing sectors."""
    steps = bufs["obs"].shape[0]
    tot = dict(resets=0, grazing=0, reset_grazing=0)
    for t in range(steps):
        a = ref.rollout_actions(first_step + t)
        assert np.array_equal(bufs["act"][t], a), f"{label}: actions of step {t} differ"
        r = ref.step(a, threads=threads)
        g = {k: bufs[k][t] for k in ("obs", "reward", "terminated", "truncated", "final_obs")}
        tot["reset_grazing"] += compare_outputs(g, r, ref, label=f"{label} step {t}")
        tot["resets"] += int(r["reset"].sum())
        tot["grazing"] += int(r["grazing"].sum())
    return tot
