"""Throughput of the batched navigation step on one MI355X.

Headline workload (default, the fused-batched configuration): 32768 envs over
128 seeded maps whose sides are drawn from 96-512 cells at 0.05 m (rectangle +
disc maps and rooms maps alternating), each map with its own beam count from
{180, 360, 720, 1080} (pooled to 30 sectors) and its own footprint (disc
r 0.18 m or 0.70 x 0.31 m rectangle), r_max 8 m, dt 0.05 s, uniform random
actions with reverse, auto-reset, all envs in one launch per step.  A second
leg times the 4096-env workload (16 maps 128x128, 360 beams, r_max 6 m).

A third leg runs the learned reset proposal on its own workload (65,536
envs on 64 rooms maps 256x256, 8 difficulty bins): labelling, training, the
network against the rejection sampler on the same requests, and the step
with the proposer attached, so that every sparse reset takes a verified pair
at the env's requested difficulty, timed against the same step without it.

Before the warm-up an untimed burn-in of several episode horizons runs the
envs into their steady mix of episode ages, so the timed steps hold the steady
share of resets (auto-resets inside the step).  Inputs are resident in HBM
before the timed region.

One step = one navsim_step call over all envs = one launch of the fused step
kernel (action -> pose -> collision -> reward/flags -> reset draws -> scan of
every new pose and every reset pose -> sector pooling -> observation rows).
Prints one JSON line.
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

NOMINAL_LDS_GBS = 256 * 128 * 2.4  # 256 CUs x 128 B/clk x 2.4 GHz = 78643 GB/s
VALU_LANE_OPS_PEAK = 256 * 4 * 16 * 2.4e9  # 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz (int32 ops/s)
SIMDS = 256 * 4
XCDS = 8
CLOCK_HZ = 2.4e9
# the fused step's source: the kernel file and the headers it includes
KERNEL_SRCS = [os.path.join(ROOT, "paper_2606_15846_amd", "csrc", f)
               for f in ("navsim_kernels.hip", "navsim_internal.hpp", "philox.hpp")]
PROFILES = os.path.join(ROOT, "profiles")
# the paper's own headline, for context only (another GPU, and the whole
# training loop rather than the simulator step)
PAPER_CONTEXT = {
    "figure": "deployable navigation policy trained in under 20 s of wall-clock",
    "hardware": "one RTX 5090 (host Ryzen 9 9950X)",
    "what": "whole off-policy training loop (simulator + policy + learner), 1024 envs, "
            "1080 beams; not a simulator-step throughput",
    "source": "Abstract; section 3.4; table 2",
}


def log(msg: str) -> None:
    """Progress of the legs on stderr (the JSON line alone goes to stdout)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def plan_legs(steps: int, warmup: int, plain_steps: int, march_steps: int,
              march_err_steps: int = 5) -> dict:
    """Action rows and the [first, last) rows each leg reads.  Every leg
    starts at the first timed row (the same saved state); the action array
    holds as many rows as the longest leg needs."""
    if steps < 1 or warmup < 0 or plain_steps < 0 or march_steps < 0 or march_err_steps < 0:
        raise ValueError("steps must be >= 1 and the other counts >= 0")
    legs = {"warmup": (0, warmup), "timed": (warmup, warmup + steps),
            "replay": (warmup, warmup + steps), "plain": (warmup, warmup + plain_steps),
            "march": (warmup, warmup + march_steps),
            "march_error": (warmup, warmup + march_err_steps)}
    rows = max(b for _, b in legs.values())
    return {"rows": rows, "legs": legs}


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


def hbm_traffic_from_profile(workload: str):
    """HBM bytes per launch from the committed counter summary (or None)."""
    vals = profile_values(os.path.join(PROFILES, f"fused_step_{workload}_hbm_traffic.txt"))
    try:
        return float(vals["hbm_bytes_per_launch"]) if vals else None
    except (KeyError, ValueError):
        return None


def sq_from_profile(workload: str, avg_launch_s: float, visits_per_launch: float):
    """VALU issue and occupancy of the same launches from the committed SQ
    counter summary: wave instructions per launch, the share of the SIMDs'
    VALU issue they fill over the live launch time (4 cycles per wave64
    instruction), lane slots per cell visit, LDS bank-conflict cycles per LDS
    instruction, and resident wavefronts per SIMD (SQ_WAVE_CYCLES counts
    wave-cycles in units of 4 clocks, summed over the chip, over the busy span
    GRBM_GUI_ACTIVE / XCDs); None when absent or stale."""
    vals = profile_values(os.path.join(PROFILES, f"fused_step_{workload}_sq_counters.txt"))
    if not vals:
        return None
    try:
        insts = float(vals["valu_wave_insts_per_launch"])
    except (KeyError, ValueError):
        return None
    lane_ops = insts * 64.0
    out = {"wave_insts_per_launch": insts,
           "issue_frac": lane_ops / (VALU_LANE_OPS_PEAK * avg_launch_s),
           "lane_slots_per_visit": lane_ops / max(visits_per_launch, 1.0),
           "peak_lane_ops_per_s": VALU_LANE_OPS_PEAK}
    for k in ("lds_bank_conflict_cycles_per_lds_inst", "waves_per_simd"):
        if k in vals:
            out[k] = float(vals[k])
    return out


def measure_lds_peak(device: int) -> dict:
    """Conflict-free 16-byte LDS reads over the whole chip (two workgroups of
    1024 threads per CU, 64 KiB of LDS each): the measured LDS roof."""
    from paper_2606_15846_amd.navsim import navsim_probe_lds_read
    best = None
    for threads, per_cu in ((1024, 2), (512, 2), (256, 2)):
        ms, nb, _ = navsim_probe_lds_read(device, threads, 256 * per_cu * 8, 2048, 5)
        gbs = nb / (ms / 1e3) / 1e9
        row = {"threads": threads, "workgroups": 256 * per_cu * 8, "ms_per_launch": ms,
               "bytes_per_launch": nb, "gb_per_s": gbs}
        if best is None or gbs > best["gb_per_s"]:
            best = row
    best["bytes_per_clk_per_cu"] = best["gb_per_s"] * 1e9 / (256 * CLOCK_HZ)
    return best


def burn_in(sim, steps: int, seed: int):
    """Untimed steps under device-drawn uniform actions (seeded), so that the
    envs' episode ages reach their steady mix."""
    import torch
    g = torch.Generator(device=sim.device)
    g.manual_seed(seed)
    for _ in range(steps):
        a = torch.rand((sim.N, 2), generator=g, device=sim.device) * 2.0 - 1.0
        sim.step(a)
    torch.cuda.synchronize(sim.device)


def time_steps(sim, acts, first: int, count: int, plain: bool = False) -> float:
    """Milliseconds for `count` back-to-back steps, one HIP event pair on the
    stream the steps are launched on."""
    import torch
    stream = torch.cuda.current_stream(sim.device)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize(sim.device)
    e0.record(stream)
    for t in range(count):
        sim.step(acts[first + t], plain=plain)
    e1.record(stream)
    torch.cuda.synchronize(sim.device)
    return e0.elapsed_time(e1)


def replay_work(sim, acts, first: int, count: int, start_state, keep_first: bool):
    """Replay the timed steps from their saved state with the per-ray outputs
    on (results are bitwise those of the timed steps): cell visits, resets
    (start / goal free-list fallbacks) and, optionally, the first step's
    per-ray results and post-step state on the host."""
    import torch
    sim.set_state(start_state)
    visits = torch.zeros((), dtype=torch.int64, device=sim.device)
    resets = torch.zeros((), dtype=torch.int64, device=sim.device)
    fb_start = torch.zeros((), dtype=torch.int64, device=sim.device)
    fb_goal = torch.zeros((), dtype=torch.int64, device=sim.device)
    first_step = None
    for t in range(count):
        dbg = sim.step_debug(acts[first + t])
        visits += dbg["visits"].sum()
        resets += dbg["reset"].sum()
        fb = dbg["fallback"].to(torch.int64)
        fb_start += (fb & 1).sum()
        fb_goal += ((fb >> 1) & 1).sum()
        if keep_first and t == 0:
            first_step = {"ranges": dbg["ranges"].cpu().numpy(), "hits": dbg["hits"].cpu().numpy(),
                          "collision": dbg["collision"].cpu().numpy(),
                          "obs": sim.obs.cpu().numpy(), "reward": sim.reward.cpu().numpy(),
                          "terminated": sim.terminated.cpu().numpy(),
                          "truncated": sim.truncated.cpu().numpy(), "state": sim.get_state()}
    torch.cuda.synchronize(sim.device)
    return {"visits": int(visits.item()), "resets": int(resets.item()),
            "fallback_start": int(fb_start.item()), "fallback_goal": int(fb_goal.item()),
            "first_step": first_step}


def live_beams(w, N, K):
    """[N, K] mask of the beams each env casts (per-map beam counts)."""
    if w["profiles"] is None:
        return np.ones((N, K), bool)
    kmap = np.array([q["num_beams"] for q in w["profiles"]])
    kenv = kmap[np.asarray(w["env_map"])]
    return np.arange(K)[None, :] < kenv[:, None]


def cpu_baseline(w, acts_np, start_state, gpu_first, rays_per_env_step: float,
                 target_s: float = 15.0) -> dict:
    """The oracle on the machine's host cores, from the same steady state under
    the same actions: its first step (with per-ray outputs) is compared with
    the GPU's first timed step over every env -- a full-size parity sample
    that also counts grazing rays -- then steps are timed for ~target_s."""
    import oracle
    threads = len(os.sched_getaffinity(0))
    ref = oracle.OracleSim(w["cfg"], w["maps"], w["res"], w["env_map"], profiles=w["profiles"])
    ref.set_state(start_state)
    N = ref.N
    t0 = time.perf_counter()
    o = ref.step(acts_np[0], debug=True, threads=threads)
    one = time.perf_counter() - t0
    parity = None
    if gpu_first is not None:
        live = live_beams(w, N, ref.K)
        graze = o["grazing"].astype(bool) & live
        exact = live & ~graze
        dr = np.abs(gpu_first["ranges"] - o["ranges"])[exact]
        st_ok = all(np.array_equal(gpu_first["state"][k], ref.state[k]) for k in oracle.STATE_KEYS)
        parity = {"envs": N, "rays": int(live.sum()), "grazing_rays": int(graze.sum()),
                  "grazing_frac": float(graze.sum() / max(live.sum(), 1)),
                  "hit_mismatch_nongrazing": int((gpu_first["hits"] != o["hits"])[exact].sum()),
                  "max_range_err_nongrazing_m": float(dr.max()) if dr.size else 0.0,
                  "collision_equal": bool(np.array_equal(gpu_first["collision"], o["collision"])),
                  "flags_equal": bool(np.array_equal(gpu_first["terminated"], o["terminated"]) and
                                      np.array_equal(gpu_first["truncated"], o["truncated"])),
                  "max_reward_err": float(np.abs(gpu_first["reward"] - o["reward"]).max()),
                  "post_step_state_bitwise": bool(st_ok)}
    steps = int(max(1, min(200, target_s / max(one, 1e-6))))
    t0 = time.perf_counter()
    for t in range(1, 1 + steps):
        ref.step(acts_np[t % acts_np.shape[0]], debug=False, threads=threads)
    dt = time.perf_counter() - t0
    rate = N * steps / dt
    return {"value": rate, "unit": "env-steps/s", "cores": threads,
            "host_cpu_count": os.cpu_count(), "kind": "oracle",
            "rays_per_s": rate * rays_per_env_step,
            "sample": f"{steps} steps x {N} envs of the same workload from the same steady state "
                      f"(scalar FP64 C oracle, {threads} threads over env slices), {dt:.1f} s",
            "parity_sample": parity}


def reset_proposal_gain(sim, w, args, keep_proposer: bool = False) -> dict:
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
    rp.train(pairs, steps=args.train_steps, batch=1024, samples=args.train_samples, lr=1e-3,
             weight_decay=1e-4, loss=loss)
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
           "train_samples": args.train_samples, "train_s": t_train, "loss_first_50": float(lv[:50].mean()),
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
    if keep_proposer:
        out["_proposer"] = rp
    else:
        rp.close()
    return out


def learned_reset_leg(args) -> dict:
    """The learned reset proposal on its own workload (65,536 envs, 64 rooms
    maps 256x256, 8 difficulty bins over 1-12 m): label pairs, train the
    network, compare it with the rejection sampler on the same requests, then
    attach it to the step (every env asks for bin env mod 8) and time steps
    whose sparse resets take verified pairs from it, against the same step
    with the free-space sampler."""
    import torch
    from paper_2606_15846_amd.navsim import NavSim
    from workloads import configs

    w = configs.build_workload(args.proposal_workload)
    cfg = w["cfg"]
    N = cfg["num_envs"]
    sim = NavSim(cfg, w["maps"], w["res"], w["env_map"], device=0)
    tuning, _ = tuning_for(w, argparse.Namespace())
    sim.set_tuning(**tuning)
    sim.reset()
    log(f"learned resets: {N} envs built; burn-in of {args.burn_in} steps")
    burn_in(sim, args.burn_in, seed=77)
    g = torch.Generator(device=sim.device)
    g.manual_seed(78)

    def timed(k):
        acts = [torch.rand((N, 2), generator=g, device=sim.device) * 2.0 - 1.0 for _ in range(k)]
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        for a in acts:
            sim.step(a)
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / k

    steps = args.proposal_steps
    plain_ms = timed(steps)
    out = {"workload": w["name"], "steps": steps,
           "free_space_step": {"ms_per_step": plain_ms, "env_steps_per_s": N / (plain_ms / 1e3)}}
    log("learned resets: labelling and training")
    out["offline"] = reset_proposal_gain(sim, w, args, keep_proposer=True)
    rp = out["offline"].pop("_proposer")
    # in the step: 32 network draws, then at most 64 rejection attempts (a
    # request past that takes the free-space pose), at most 2,048 per step
    P, T, cap = 32, 64, min(N, 2048)
    rp.attach((np.arange(N) % rp.nb).astype(np.int32), proposals=P, max_tries=T,
              max_per_step=cap)
    timed(20)  # warm: the first resets of the attached proposer
    rp.attach_stats(clear=True)
    log("learned resets: attached steps")
    ms = timed(steps)
    st = rp.attach_stats()
    out["in_step"] = {
        "ms_per_step": ms, "env_steps_per_s": N / (ms / 1e3),
        "proposals": P, "max_tries": T, "max_per_step": cap,
        "bins": "env mod 8 (every env asks for a bin)",
        "resets_per_step": st["deferred"] / steps,
        "learned_resets_per_s": st["requests"] / (ms * steps / 1e3),
        "from_network": st["from_network"] / max(st["requests"], 1),
        "from_rejection": st["from_rejection"] / max(st["requests"], 1),
        "no_valid_pair": st["no_pair"] / max(st["requests"], 1),
        "over_cap": st["over_cap"] / max(st["deferred"], 1),
        "exact_checks_per_reset": st["checks"] / max(st["requests"], 1),
        "step_time_vs_free_space": ms / plain_ms}
    rp.close()
    sim.close()
    return out


def tuning_for(w, args) -> tuple[dict, bool]:
    """The autotuned launch shape of the workload (paper_2606_15846_amd/
    tuning.json) with command-line overrides; results do not depend on it.
    Also whether it is the tuned shape (the one the committed counters cover)."""
    from paper_2606_15846_amd import autotune
    tuned = autotune.best_for(autotune.workload_key(w["cfg"], w["maps"], w["profiles"]))
    tuning = dict(tuned)
    for k in autotune.FIELDS:
        if getattr(args, k, None) is not None:
            tuning[k] = getattr(args, k)
    return tuning, tuning == tuned


def roofline(workload: str, visits: int, steps: int, ms_per_step: float, lds_peak, profiled):
    lds_bytes_per_launch = 4.0 * visits / steps
    # one launch per step, back to back: the timed region's time per step is
    # the launch's duration plus the dispatch gap (the roofline's denominator)
    avg_launch_s = ms_per_step / 1e3
    achieved = lds_bytes_per_launch / avg_launch_s / 1e9
    out = {"bound": "lds", "achieved": achieved, "peak": NOMINAL_LDS_GBS, "unit": "GB/s",
           "frac": achieved / NOMINAL_LDS_GBS,
           "traffic": hbm_traffic_from_profile(workload) if profiled else None,
           "kernel": "fused_step_kernel", "avg_launch_us": avg_launch_s * 1e6,
           "algorithmic_bytes_per_launch": lds_bytes_per_launch,
           "bytes_per_unit": "4 B of bitmap word per grid-cell visit of the step's pre-reset scan",
           "peak_nominal": NOMINAL_LDS_GBS,
           "valu": sq_from_profile(workload, avg_launch_s, visits / steps) if profiled else None}
    if lds_peak:
        out["peak_measured"] = lds_peak["gb_per_s"]
        out["frac_measured"] = achieved / lds_peak["gb_per_s"]
    return out


def run_fused_leg(name: str, args, steps: int, warmup: int, lds_peak, full: bool) -> dict:
    """Build the workload, burn in, warm up, time `steps` fused steps and
    count their work.  With full=True also the march, rollout, policy, plain,
    proposal and CPU legs (the headline)."""
    import torch
    from paper_2606_15846_amd.navsim import NavSim
    from workloads import configs

    dev = torch.device("cuda", 0)
    w = configs.build_workload(name)
    cfg = w["cfg"]
    N, K, m = cfg["num_envs"], cfg["num_beams"], cfg["num_sectors"]
    live = live_beams(w, N, K)
    rays_per_step = int(live.sum())
    plan = plan_legs(steps, warmup, args.plain_steps if full and not args.no_plain else 0,
                     min(steps, 200) if full and not args.no_march else 0,
                     5 if full and not args.no_march else 0)
    legs = plan["legs"]
    acts_np = configs.uniform_actions(plan["rows"], N, seed=42)
    acts = torch.from_numpy(acts_np).to(dev)
    sim = NavSim(cfg, w["maps"], w["res"], w["env_map"], device=0, profiles=w["profiles"])
    tuning, profiled = tuning_for(w, args) if full else tuning_for(w, argparse.Namespace())
    sim.set_tuning(**tuning)
    sim.reset()
    log(f"{name}: {N} envs built; burn-in of {args.burn_in} steps")
    t_burn = time.perf_counter()
    burn_in(sim, args.burn_in, seed=4242)
    t_burn = time.perf_counter() - t_burn
    for t in range(*legs["warmup"]):
        sim.step(acts[t])
    torch.cuda.synchronize()
    start_state = sim.get_state()
    total_ms = time_steps(sim, acts, legs["timed"][0], steps)
    ms_per_step = total_ms / steps
    log(f"{name}: {steps} timed steps, {ms_per_step * 1e3:.1f} us per step")
    value = N * steps / (total_ms / 1e3)
    work = replay_work(sim, acts, legs["replay"][0], steps, start_state,
                       keep_first=full and not args.no_cpu)
    out = {"workload": w["name"], "value": value, "unit": "env-steps/s", "steps": steps,
           "warmup": warmup, "burn_in_steps": args.burn_in, "burn_in_s": t_burn,
           "ms_per_step": ms_per_step, "rays_per_s": value * rays_per_step / N,
           "beams_per_env_step": rays_per_step / N,
           "reset_rate_per_step": work["resets"] / (N * steps),
           "resets": work["resets"], "fallback_start": work["fallback_start"],
           "fallback_goal": work["fallback_goal"],
           "extra_rays_per_s": work["resets"] * (rays_per_step / N) / (total_ms / 1e3),
           "cell_visits_per_env_step": work["visits"] / (N * steps),
           "roofline": roofline(name, work["visits"], steps, ms_per_step, lds_peak, profiled),
           "tuning": sim.get_tuning()}
    if not full:
        sim.close()
        return out
    stream = torch.cuda.current_stream(dev)

    # the paper's fixed-step range query (0.03 m) on the same fused step
    if not args.no_march:
        log(f"{name}: fixed-step march leg")
        a0, a1 = legs["march"]
        sim.set_state(start_state)
        sim.set_scan(1, args.march_step)
        for t in range(a0, min(a1, a0 + 5)):
            sim.step(acts[t])
        sim.set_state(start_state)
        mms = time_steps(sim, acts, a0, a1 - a0) / (a1 - a0)
        # its error against the exact traversal: the same states and actions
        # (poses, collisions and resets do not depend on the scan)
        live_d = torch.from_numpy(live).to(dev)
        e0_, e1_ = legs["march_error"]
        stride = max(1, (5 * N * K) // 4_000_000)  # a bounded sample for the quantile
        sim.set_state(start_state)
        d_ray, d_sec = [], []
        for t in range(e0_, e1_):
            s0 = sim.get_state()
            rm = sim.step_debug(acts[t])["ranges"].clone()
            om = sim.obs[:, :m].clone()
            sim.set_scan(0, 0.03)
            sim.set_state(s0)
            re = sim.step_debug(acts[t])["ranges"].clone()
            oe = sim.obs[:, :m].clone()
            d_ray.append((rm - re).abs()[live_d][::stride].cpu())
            d_sec.append((om - oe).abs().flatten().cpu())
            sim.set_scan(1, args.march_step)
        sim.set_scan(0, 0.03)
        d_ray, d_sec = torch.cat(d_ray).double(), torch.cat(d_sec).double()
        cell = float(np.min(w["res"]))
        out["march_scan"] = {
            "value": N / (mms / 1e3), "unit": "env-steps/s", "ms_per_step": mms,
            "steps": a1 - a0, "step_m": args.march_step, "traversal_speedup": mms / ms_per_step,
            "error_vs_traversal": {
                "rays": int(d_ray.numel()), "mean_abs_m": float(d_ray.mean()),
                "p99_abs_m": float(d_ray.quantile(0.99)), "max_abs_m": float(d_ray.max()),
                "rays_off_by_more_than_a_cell": float((d_ray > cell).double().mean()),
                "sector_min_mean_abs_m": float(d_sec.mean()),
                "sector_min_max_abs_m": float(d_sec.max())}}

    # device rollouts: the same fused step under in-kernel actions, T steps
    # captured once as a HIP graph and replayed
    log(f"{name}: graph rollout leg")
    sim.set_state(start_state)
    T = args.rollout_steps
    bufs = sim.rollout_buffers(T, final_obs=True)
    sim.rollout(T, first_step=0, buffers=bufs, graph=True)  # capture + warm
    torch.cuda.synchronize()
    r0, r1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = max(1, steps // T)
    r0.record(stream)
    for r in range(reps):
        sim.rollout(T, first_step=(r + 1) * T, buffers=bufs, graph=True)
    r1.record(stream)
    torch.cuda.synchronize()
    rms = r0.elapsed_time(r1)
    out["graph_rollout"] = {"value": N * T * reps / (rms / 1e3), "unit": "env-steps/s",
                            "steps_per_rollout": T, "rollouts": reps,
                            "ms_per_step": rms / (T * reps),
                            "actions": "in-kernel Philox stream 4",
                            "launch": "HIP graph of T fused steps"}
    # the paper's actor in front of every step (graph of T actor + step launches)
    if not args.no_policy:
        log(f"{name}: policy rollout leg")
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
        out["policy_rollout"] = {"value": N * T * reps / (qms / 1e3), "unit": "env-steps/s",
                                 "ms_per_step": qms / (T * reps), "steps_per_rollout": T,
                                 "actor": f"{pol.dims} leaky ReLU, tanh, bf16 matrix cores",
                                 "launch": "HIP graph of T (actor + fused step)"}
        pol.close()
    del bufs

    if not args.no_plain:
        log(f"{name}: plain step leg")
        a0, a1 = legs["plain"]
        sim.set_state(start_state)
        pms = time_steps(sim, acts, a0, a1 - a0, plain=True)
        prate = N * (a1 - a0) / (pms / 1e3)
        out["plain"] = {"value": prate, "rays_per_s": prate * rays_per_step / N,
                        "steps": a1 - a0, "ms_per_step": pms / (a1 - a0),
                        "mapping": "one thread per env, beams in sequence, bitmap in HBM"}
        out["speedup_vs_plain"] = value / prate
    sim.close()
    if not args.no_cpu:
        log(f"{name}: oracle on the host cores")
        a0, a1 = legs["timed"]
        out["cpu_baseline"] = cpu_baseline(w, acts_np[a0:], start_state, work["first_step"],
                                           rays_per_step / N)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="c4")
    ap.add_argument("--secondary", default="c2",
                    help="a second workload timed the same way ('' for none)")
    ap.add_argument("--secondary-steps", type=int, default=1000)
    ap.add_argument("--burn-in", type=int, default=1000,
                    help="untimed steps before the warm-up (several 200-step horizons)")
    ap.add_argument("--plain-steps", type=int, default=50)
    ap.add_argument("--rollout-steps", type=int, default=64)
    ap.add_argument("--no-march", action="store_true")
    ap.add_argument("--no-proposal", action="store_true")
    ap.add_argument("--no-policy", action="store_true")
    ap.add_argument("--no-lds-peak", action="store_true")
    ap.add_argument("--label-starts", type=int, default=131072)
    ap.add_argument("--train-steps", type=int, default=2000)
    ap.add_argument("--train-samples", type=int, default=128,
                    help="noise draws per target in training (the closest one is fitted)")
    ap.add_argument("--proposal-requests", type=int, default=8192)
    ap.add_argument("--proposal-workload", default="c5",
                    help="workload of the learned reset leg (needs a proposer config)")
    ap.add_argument("--proposal-steps", type=int, default=50)
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
    ap.add_argument("--lds-probe-only", action="store_true",
                    help="only run the LDS read probe and print its best shape (profiling)")
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

    log("LDS read probe")
    lds_peak = None if args.no_lds_peak else measure_lds_peak(0)
    if args.lds_probe_only:
        print(json.dumps({"lds_peak_probe": lds_peak}))
        return
    head = run_fused_leg(args.workload, args, args.steps, args.warmup, lds_peak, full=True)
    learned = None
    if not args.no_proposal:
        learned = learned_reset_leg(args)
    second = None
    if args.secondary and args.secondary != args.workload:
        second = run_fused_leg(args.secondary, args, args.secondary_steps, args.warmup, lds_peak,
                               full=False)
    from workloads import configs
    w = configs.build_workload(args.workload)
    cfg = w["cfg"]
    out = {
        "metric": "env-steps/s + rays/s on 1 MI355X, fused-batched vs plain step; % LDS roofline",
        "value": head["value"],
        "unit": "env-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32+f64",
        "data": "synthetic",
        "config": {"workload": head["workload"], "envs": cfg["num_envs"],
                   "sectors": cfg["num_sectors"], "maps": len(w["maps"]),
                   "beams": cfg["num_beams"] if w["profiles"] is None else "per map",
                   "beams_per_env_step": head["beams_per_env_step"],
                   "map_cells": (f"{w['maps'][0].shape[1]}x{w['maps'][0].shape[0]}"
                                 if w["profiles"] is None else "per map"),
                   "res_m": w["res"][0], "max_range_m": cfg["max_range_m"],
                   "footprint": ("per map" if w["profiles"] is not None
                                 else "disc" if cfg["footprint"] == 0 else "rect"),
                   "launch": "one fused launch per step over all envs and maps"},
        "rays_per_s": head["rays_per_s"],
        "roofline": head["roofline"],
        "cpu_baseline": head.get("cpu_baseline"),
        "plain": head.get("plain"),
        "speedup_vs_plain": head.get("speedup_vs_plain"),
        "reset_rate_per_step": head["reset_rate_per_step"],
        "resets": {"count": head["resets"], "fallback_start": head["fallback_start"],
                   "fallback_goal": head["fallback_goal"],
                   "extra_rays_per_s": head["extra_rays_per_s"]},
        "burn_in_steps": head["burn_in_steps"],
        "cell_visits_per_env_step": head["cell_visits_per_env_step"],
        "graph_rollout": head.get("graph_rollout"),
        "policy_rollout": head.get("policy_rollout"),
        "march_scan": head.get("march_scan"),
        "learned_reset": learned,
        "tuning": head["tuning"],
        "lds_peak_probe": lds_peak,
        "secondary": second,
        "paper_context": PAPER_CONTEXT,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
