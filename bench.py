"""Throughput of the batched navigation step on one MI355X.

Workload (default): 4096 envs over 16 seeded 128x128 maps at 0.05 m (rectangles
and rasterised discs, ~15 % occupancy), disc robot r = 0.18 m, 360 beams over
360 deg pooled to 30 sectors, r_max 6 m, dt 0.1 s, uniform random actions,
auto-reset.  Inputs are resident in HBM before the timed region.

One step = one navsim_step call over all envs = one launch of the fused step
kernel (action -> pose -> collision -> reward/flags -> reset draws -> 360-beam
scan of every new pose and every reset pose -> sector pooling -> observation
rows).  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

LDS_PEAK_GBS = 256 * 128 * 2.4  # 256 CUs x 128 B/clk x 2.4 GHz = 78643 GB/s
# the fused step's source: the kernel file and the headers it includes
KERNEL_SRCS = [os.path.join(ROOT, "paper_2606_15846_amd", "csrc", f)
               for f in ("navsim_kernels.hip", "navsim_internal.hpp", "philox.hpp")]
PMC_FILE = os.path.join(ROOT, "profiles", "fused_step_c2_hbm_traffic.txt")
SQ_FILE = os.path.join(ROOT, "profiles", "fused_step_c2_sq_counters.txt")
VALU_LANE_OPS_PEAK = 256 * 4 * 16 * 2.4e9  # 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz (int32 ops/s)


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SRCS:
        h.update(open(f, "rb").read())
    return h.hexdigest()[:16]


def profile_values(path: str):
    """`key: value` lines of a committed rocprofv3 summary, or None when absent
    or taken on a different kernel source."""
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    return vals


def hbm_traffic_from_profile():
    """HBM bytes per launch from the committed counter summary (or None)."""
    vals = profile_values(PMC_FILE)
    try:
        return float(vals["hbm_bytes_per_launch"]) if vals else None
    except (KeyError, ValueError):
        return None


def valu_from_profile(avg_launch_s: float, visits_per_launch: float):
    """VALU issue of the same launches from the committed SQ counter summary:
    wave instructions per launch, the share of the SIMDs' VALU issue they fill
    over the live launch time (4 cycles per wave64 instruction), and lane
    slots per cell visit; None when absent or stale."""
    vals = profile_values(SQ_FILE)
    if not vals:
        return None
    try:
        insts = float(vals["valu_wave_insts_per_launch"])
    except (KeyError, ValueError):
        return None
    lane_ops = insts * 64.0
    return {"wave_insts_per_launch": insts,
            "issue_frac": lane_ops / (VALU_LANE_OPS_PEAK * avg_launch_s),
            "lane_slots_per_visit": lane_ops / max(visits_per_launch, 1.0),
            "peak_lane_ops_per_s": VALU_LANE_OPS_PEAK}


def cpu_baseline(w, acts, rays_per_env_step: float, target_s: float = 10.0) -> dict:
    import oracle
    threads = min(len(os.sched_getaffinity(0)), 16)
    ref = oracle.OracleSim(w["cfg"], w["maps"], w["res"], w["env_map"], profiles=w["profiles"])
    ref.reset(threads=threads)
    N = ref.N
    t0 = time.perf_counter()
    ref.step(acts[0], debug=False, threads=threads)
    one = time.perf_counter() - t0
    steps = int(max(1, min(acts.shape[0] - 1, target_s / max(one, 1e-6))))
    t0 = time.perf_counter()
    for t in range(1, 1 + steps):
        ref.step(acts[t], debug=False, threads=threads)
    dt = time.perf_counter() - t0
    rate = N * steps / dt
    return {"value": rate, "unit": "env-steps/s", "cores": threads, "kind": "oracle",
            "rays_per_s": rate * rays_per_env_step,
            "sample": f"{steps} steps x {N} envs of the same workload (scalar FP64 C oracle, "
                      f"{threads} threads over env slices), {dt:.1f} s"}


def reset_proposal_gain(sim, w, args) -> dict:
    """Learned reset proposal against the plain rejection sampler on the
    workload's maps: label pairs with the GPU search, train the network, then
    answer the same requests (uniform over the bins) both ways and time them.
    Both return only pairs that passed the exact check."""
    import torch
    from paper_2606_15846_amd.reset_proposal import ResetProposer

    rp = ResetProposer(sim, **w["proposer"])
    nm = len(w["maps"])
    ns = args.label_starts
    t0 = time.perf_counter()
    lab = rp.label(np.arange(ns) % nm, first_sid=0)
    torch.cuda.synchronize()
    t_label = time.perf_counter() - t0
    nb = rp.nb
    keep = lab["goal"] >= 0
    ids = torch.arange(ns, device=sim.device, dtype=torch.int32)
    pairs = dict(map=(ids % nm)[:, None].expand(ns, nb)[keep].contiguous(),
                 bin=torch.arange(nb, device=sim.device, dtype=torch.int32)[None, :]
                 .expand(ns, nb)[keep].contiguous(),
                 start=lab["start"][:, None].expand(ns, nb)[keep].contiguous(),
                 goal=lab["goal"][keep].contiguous())
    loss = torch.zeros(args.train_steps, device=sim.device)
    t0 = time.perf_counter()
    rp.train(pairs, steps=args.train_steps, batch=1024, samples=16, lr=1e-3, weight_decay=1e-4,
             loss=loss)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    lv = loss.cpu().numpy() / 1024
    n = args.proposal_requests
    rng = np.random.default_rng(11)
    mp = rng.integers(0, nm, n)
    bins = np.arange(n) % nb
    env = np.arange(n)
    ep = rng.integers(0, 1 << 20, n)
    out = {"pairs": int(pairs["map"].numel()), "label_s": t_label, "train_steps": args.train_steps,
           "train_s": t_train, "loss_first_50": float(lv[:50].mean()),
           "loss_last_50": float(lv[-50:].mean()), "requests": n}
    for name, M, tries in (("learned", 32, 400), ("rejection", 0, 432)):
        rp.propose(mp, bins, env, ep, proposals=M, max_tries=tries)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        res = rp.propose(mp, bins, env, ep, proposals=M, max_tries=tries)
        e1.record()
        torch.cuda.synchronize()
        src = res["source"].cpu().numpy()
        ok = src >= 0
        # difficulty: geodesic length (hops x cell size) against the requested bin
        pc = w["proposer"]
        width = (pc["d_hi_m"] - pc["d_lo_m"]) / nb
        geo = res["hops"].cpu().numpy()[ok] * np.asarray(w["res"], np.float64)[mp[ok]]
        lo = pc["d_lo_m"] + bins[ok] * width
        out[name] = {"valid_fraction": float(ok.mean()),
                     "checks_per_request": float(res["checks"].float().mean().item()),
                     "resets_per_s": float(ok.sum() / (e0.elapsed_time(e1) / 1e3)),
                     "from_network": float(((src >= 0) & (src < M)).mean()) if M else 0.0,
                     "in_requested_bin": float(((geo >= lo) & (geo < lo + width)).mean()),
                     "difficulty_error_m": float(np.abs(geo - (lo + width / 2)).mean())}
    out["gain_resets_per_s"] = out["learned"]["resets_per_s"] / out["rejection"]["resets_per_s"]
    rp.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="c2")
    ap.add_argument("--plain-steps", type=int, default=50)
    ap.add_argument("--rollout-steps", type=int, default=64)
    ap.add_argument("--no-march", action="store_true")
    ap.add_argument("--no-proposal", action="store_true")
    ap.add_argument("--no-policy", action="store_true")
    ap.add_argument("--label-starts", type=int, default=131072)
    ap.add_argument("--train-steps", type=int, default=2000)
    ap.add_argument("--proposal-requests", type=int, default=8192)
    ap.add_argument("--march-step", type=float, default=0.03)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--tile-envs", type=int, default=None)
    ap.add_argument("--refill-at", type=int, default=None)
    ap.add_argument("--groups", type=int, default=None)
    ap.add_argument("--ray-slots", type=int, default=None)
    ap.add_argument("--walk", type=int, default=None)
    ap.add_argument("--persist", type=int, default=None)
    ap.add_argument("--threads", type=int, default=None)
    ap.add_argument("--balance", type=int, default=None)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run 5 device-to-device copies of 256 MiB (HBM counter scale)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU (asked for --gpus {args.gpus}): the step shards by "
              "env with no exchange between GPUs, so N GPUs run N independent shares",
              file=sys.stderr)
        sys.exit(2)

    import torch

    if args.calibrate_copy:
        a = torch.ones(64 << 20, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read_per_launch": a.numel() * 4,
                          "copy_bytes_written_per_launch": b.numel() * 4, "launches": 5}))
        return

    from paper_2606_15846_amd.navsim import NAVSIM_KERNEL_FUSED, NavSim
    from workloads import configs

    dev = torch.device("cuda", 0)
    w = configs.build_workload(args.workload)
    cfg = w["cfg"]
    N, K, m = cfg["num_envs"], cfg["num_beams"], cfg["num_sectors"]
    # beams cast per step (per-map beam counts when the workload has profiles)
    if w["profiles"] is None:
        rays_per_step = N * K
    else:
        kmap = np.array([q["num_beams"] for q in w["profiles"]], dtype=np.int64)
        rays_per_step = int(kmap[np.asarray(w["env_map"])].sum())
    total = args.warmup + args.steps
    acts_np = configs.uniform_actions(total, N, seed=42)
    acts = torch.from_numpy(acts_np).to(dev)
    sim = NavSim(cfg, w["maps"], w["res"], w["env_map"], device=0, profiles=w["profiles"])
    # launch shape: the autotuned one for this workload (paper_2606_15846_amd/
    # tuning.json) unless given on the command line; results do not depend on it
    from paper_2606_15846_amd import autotune
    tuning = autotune.best_for(autotune.workload_key(cfg, w["maps"], w["profiles"]))
    tuned = dict(tuning)
    for k in ("tile_envs", "refill_at", "groups", "ray_slots", "walk", "persist", "threads",
              "balance"):
        if getattr(args, k) is not None:
            tuning[k] = getattr(args, k)
    # the committed counter summaries cover the default workload in its tuned shape
    profiled = args.workload == "c2" and tuning == tuned
    sim.set_tuning(**tuning)
    sim.reset()
    for t in range(args.warmup):
        sim.step(acts[t])
    torch.cuda.synchronize()
    start_state = sim.get_state()
    stream = torch.cuda.current_stream(dev)
    resets = torch.zeros((), dtype=torch.int64, device=dev)
    # the timed steps: back to back, one event pair around all of them
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for t in range(args.steps):
        sim.step(acts[args.warmup + t])
    e1.record(stream)
    torch.cuda.synchronize()
    total_ms = e0.elapsed_time(e1)
    ms_per_step = total_ms / args.steps
    value = N * args.steps / (total_ms / 1e3)

    # algorithmic work of the timed steps: replay them with the per-ray visit
    # counts switched on (same state, same actions, results are bitwise equal)
    sim.set_state(start_state)
    visits = 0
    for t in range(args.steps):
        dbg = sim.step_debug(acts[args.warmup + t], kernel=NAVSIM_KERNEL_FUSED)
        visits += int(dbg["visits"].sum().item())
        resets += dbg["reset"].sum()
    reset_rate = float(resets.item()) / (N * args.steps)
    lds_bytes_per_launch = 4.0 * visits / args.steps
    # one launch per step, back to back: the timed region's time per step is
    # the launch's duration plus the dispatch gap (the roofline's denominator)
    avg_launch_s = ms_per_step / 1e3
    achieved = lds_bytes_per_launch / avg_launch_s / 1e9
    traffic = hbm_traffic_from_profile() if profiled else None
    valu = valu_from_profile(avg_launch_s, visits / args.steps) if profiled else None

    # the paper's fixed-step range query (0.03 m) on the same fused step
    march = None
    if not args.no_march:
        sim.set_state(start_state)
        sim.set_scan(1, args.march_step)
        for t in range(5):
            sim.step(acts[args.warmup + t])
        sim.set_state(start_state)
        torch.cuda.synchronize()
        m0, m1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        msteps = min(args.steps, 200)
        m0.record(stream)
        for t in range(msteps):
            sim.step(acts[args.warmup + t])
        m1.record(stream)
        torch.cuda.synchronize()
        mms = m0.elapsed_time(m1) / msteps
        # its error against the exact traversal: the same states and actions
        # (poses, collisions and resets do not depend on the scan), 5 steps
        if w["profiles"] is None:
            live = torch.ones(N, K, dtype=torch.bool, device=dev)
        else:  # beams past an env's own count are not cast
            kenv = torch.tensor([q["num_beams"] for q in w["profiles"]], device=dev)[
                torch.as_tensor(np.asarray(w["env_map"]), device=dev).long()]
            live = torch.arange(K, device=dev)[None, :] < kenv[:, None]
        stride = max(1, (5 * N * K) // 4_000_000)  # a bounded sample for the quantile
        sim.set_state(start_state)
        d_ray, d_sec = [], []
        for t in range(5):
            s0 = sim.get_state()
            rm = sim.step_debug(acts[args.warmup + t])["ranges"].clone()
            om = sim.obs[:, :m].clone()
            sim.set_scan(0, 0.03)
            sim.set_state(s0)
            re = sim.step_debug(acts[args.warmup + t])["ranges"].clone()
            oe = sim.obs[:, :m].clone()
            d_ray.append((rm - re).abs()[live][::stride].cpu())
            d_sec.append((om - oe).abs().flatten().cpu())
            sim.set_scan(1, args.march_step)
        sim.set_scan(0, 0.03)
        d_ray, d_sec = torch.cat(d_ray).double(), torch.cat(d_sec).double()
        cell = float(np.min(w["res"]))
        march_err = {"rays": int(d_ray.numel()),
                     "mean_abs_m": float(d_ray.mean()), "p99_abs_m": float(d_ray.quantile(0.99)),
                     "max_abs_m": float(d_ray.max()),
                     "rays_off_by_more_than_a_cell": float((d_ray > cell).double().mean()),
                     "sector_min_mean_abs_m": float(d_sec.mean()),
                     "sector_min_max_abs_m": float(d_sec.max())}
        march = {"value": N / (mms / 1e3), "unit": "env-steps/s", "ms_per_step": mms,
                 "steps": msteps, "step_m": args.march_step,
                 "traversal_speedup": mms / ms_per_step, "error_vs_traversal": march_err}

    # device rollouts: the same fused step under in-kernel actions, T steps
    # captured once as a HIP graph and replayed
    sim.set_state(start_state)
    T = args.rollout_steps
    bufs = sim.rollout_buffers(T, final_obs=True)
    sim.rollout(T, first_step=0, buffers=bufs, graph=True)  # capture + warm
    torch.cuda.synchronize()
    r0, r1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = max(1, args.steps // T)
    r0.record(stream)
    for r in range(reps):
        sim.rollout(T, first_step=(r + 1) * T, buffers=bufs, graph=True)
    r1.record(stream)
    torch.cuda.synchronize()
    rms = r0.elapsed_time(r1)
    rollout = {"value": N * T * reps / (rms / 1e3), "unit": "env-steps/s",
               "steps_per_rollout": T, "rollouts": reps, "ms_per_step": rms / (T * reps),
               "actions": "in-kernel Philox stream 4", "launch": "HIP graph of T fused steps"}
    # the paper's actor in front of every step (graph of T actor + step launches)
    policy = None
    if not args.no_policy:
        from paper_2606_15846_amd.policy import Policy
        pol = Policy(sim)
        pol.init_params(seed=3, beta=-0.1)
        sim.set_state(start_state)
        obs0 = sim.obs.clone()
        pol.rollout(T, 0, obs0, noise_std=0.1, buffers=bufs)  # capture + warm
        torch.cuda.synchronize()
        q0, q1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        q0.record(stream)
        for r in range(reps):
            pol.rollout(T, (r + 1) * T, obs0, noise_std=0.1, buffers=bufs)
        q1.record(stream)
        torch.cuda.synchronize()
        qms = q0.elapsed_time(q1)
        policy = {"value": N * T * reps / (qms / 1e3), "unit": "env-steps/s",
                  "ms_per_step": qms / (T * reps), "steps_per_rollout": T,
                  "actor": f"{pol.dims} leaky ReLU, tanh, bf16 matrix cores",
                  "launch": "HIP graph of T (actor + fused step)"}
        pol.close()
    del bufs

    plain = None
    if not args.no_plain:
        sim.set_state(start_state)
        torch.cuda.synchronize()
        p0, p1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        p0.record(stream)
        for t in range(args.plain_steps):
            sim.step(acts[args.warmup + t], plain=True)
        p1.record(stream)
        torch.cuda.synchronize()
        pms = p0.elapsed_time(p1)
        prate = N * args.plain_steps / (pms / 1e3)
        plain = {"value": prate, "rays_per_s": prate * rays_per_step / N, "steps": args.plain_steps,
                 "ms_per_step": pms / args.plain_steps,
                 "mapping": "one thread per env, beams in sequence, bitmap in HBM"}
    sim_tuning = sim.get_tuning()
    proposal = None
    if w.get("proposer") and not args.no_proposal:
        proposal = reset_proposal_gain(sim, w, args)
    sim.close()

    cpu = None if args.no_cpu else cpu_baseline(w, acts_np[args.warmup:], rays_per_step / N)
    out = {
        "metric": "env-steps/s + rays/s on 1 MI355X, fused-batched vs plain step; % LDS roofline",
        "value": value,
        "unit": "env-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32+f64",
        "data": "synthetic",
        "config": {"workload": w["name"], "envs": N, "sectors": m, "maps": len(w["maps"]),
                   "beams": K if w["profiles"] is None else "per map",
                   "beams_per_env_step": rays_per_step / N,
                   "map_cells": (f"{w['maps'][0].shape[1]}x{w['maps'][0].shape[0]}"
                                 if w["profiles"] is None else "per map"),
                   "res_m": w["res"][0], "max_range_m": cfg["max_range_m"],
                   "footprint": ("per map" if w["profiles"] is not None
                                 else "disc" if cfg["footprint"] == 0 else "rect")},
        "rays_per_s": value * rays_per_step / N,
        "graph_rollout": rollout,
        "policy_rollout": policy,
        "march_scan": march,
        "reset_proposal": proposal,
        "plain": plain,
        "speedup_vs_plain": (value / plain["value"]) if plain else None,
        "tuning": sim_tuning,
        "reset_rate_per_step": reset_rate,
        "cell_visits_per_env_step": visits / (N * args.steps),
        "roofline": {"bound": "lds", "achieved": achieved, "peak": LDS_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / LDS_PEAK_GBS, "traffic": traffic,
                     "kernel": "fused_step_kernel",
                     "avg_launch_us": avg_launch_s * 1e6,
                     "algorithmic_bytes_per_launch": lds_bytes_per_launch,
                     "bytes_per_unit": "4 B of bitmap word per DDA cell visit of the step's pre-reset scan",
                     "valu": valu},
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
