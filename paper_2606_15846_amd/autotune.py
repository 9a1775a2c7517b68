"""Launch-shape autotuner for the fused step.

The fused step's results do not depend on its launch shape (tile_envs,
refill_at, groups, ray_slots, walk, persist, threads; see navsim_set_tuning in
include/navsim.h), only its speed
does.  The tuner replays the same seeded steps from the same saved state under
every candidate shape, times them with HIP events on the simulator's stream,
and keeps the fastest.  Results are stored per workload key in tuning.json
next to this file; bench.py and NavSim users can load them with best_for().
"""
from __future__ import annotations

import argparse
import itertools
import json
import os
import sys

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
TUNING_FILE = os.path.join(HERE, "tuning.json")
DEFAULT = {"tile_envs": 8, "refill_at": 40, "groups": 8, "ray_slots": 0, "walk": 3, "persist": 0,
           "threads": 256, "balance": 0}
# walk = 1 (chunked run walk) measured about 2x slower than the group walk on
# every workload here, persistent workgroups 5-40 % slower, the chunked bitmap
# walk (walk 0) behind the byte and claim walks; --full-space includes them
SPACE = {"tile_envs": (1, 2, 4, 8, 16, 32), "refill_at": (24, 32, 40, 48), "groups": (8, 16),
         "ray_slots": (0,), "walk": (2, 3, 4, 5), "persist": (0,), "threads": (256, 512, 1024),
         "balance": (0, 1)}
FULL_SPACE = dict(SPACE, refill_at=(16, 24, 32, 40, 48, 56), groups=(2, 4, 8, 16, 32),
                  ray_slots=(0, 512, 1024, 2048), walk=(0, 1, 2, 3, 4, 5), persist=(0, 2))
FIELDS = tuple(DEFAULT)


def workload_key(cfg: dict, maps, profiles=None) -> str:
    w = max(m.shape[1] for m in maps)
    h = max(m.shape[0] for m in maps)
    key = (f"N{cfg['num_envs']}_K{cfg['num_beams']}_m{cfg['num_sectors']}_map{w}x{h}"
           f"_fp{cfg['footprint']}_r{cfg['max_range_m']:g}")
    if profiles is not None:
        key += f"_maps{len(maps)}_mixed{sum(q['num_beams'] for q in profiles)}"
    return key


def load_all() -> dict:
    if not os.path.exists(TUNING_FILE):
        return {}
    with open(TUNING_FILE) as f:
        return json.load(f)


def best_for(key: str) -> dict:
    entry = load_all().get(key)
    best = dict(DEFAULT)
    if entry:
        best.update(entry["best"])
    return best


def save(key: str, best: dict, table: list, device_name: str, path: str = TUNING_FILE,
         table_path: str | None = None):
    """Merge one workload's best shape into the JSON file at `path` (the
    product keeps only the winner); the whole sweep goes to `table_path`."""
    allt = {}
    if os.path.exists(path):
        with open(path) as f:
            allt = json.load(f)
    ok = [r for r in table if "ms_per_step" in r]
    allt[key] = {"best": best, "device": device_name,
                 "ms_per_step": min(r["ms_per_step"] for r in ok), "candidates": len(table)}
    with open(path, "w") as f:
        json.dump(allt, f, indent=1, sort_keys=True)
    if table_path:
        os.makedirs(os.path.dirname(os.path.abspath(table_path)), exist_ok=True)
        with open(table_path, "w") as f:
            json.dump({"key": key, "device": device_name, "table": table}, f, indent=1)


def time_steps(sim, acts, start_state, steps: int) -> float:
    """Mean milliseconds per step over `steps` steps from start_state."""
    sim.set_state(start_state)
    stream = torch.cuda.current_stream(sim.device)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize(sim.device)
    a.record(stream)
    for t in range(steps):
        sim.step(acts[t])
    b.record(stream)
    torch.cuda.synchronize(sim.device)
    return a.elapsed_time(b) / steps


def tune(sim, acts, steps: int = 50, space: dict | None = None, verbose: bool = False):
    space = space or SPACE
    start = sim.get_state()
    table = []
    for values in itertools.product(*(space[k] for k in FIELDS)):
        shape = dict(zip(FIELDS, values))
        try:
            sim.set_tuning(**shape)
        except Exception as exc:  # a shape the map does not fit (LDS)
            table.append(dict(shape, error=str(exc)))
            continue
        time_steps(sim, acts, start, min(5, steps))  # settle
        ms = time_steps(sim, acts, start, steps)
        table.append(dict(shape, ms_per_step=ms))
        if verbose:
            print(" ".join(f"{k}={v}" for k, v in shape.items()) + f" -> {ms * 1e3:8.1f} us/step",
                  flush=True)
    ok = [r for r in table if "ms_per_step" in r]
    best = min(ok, key=lambda r: r["ms_per_step"])
    best = {k: best[k] for k in FIELDS}
    sim.set_tuning(**best)
    sim.set_state(start)
    return best, table


def main():
    sys.path.insert(0, os.path.dirname(HERE))
    from paper_2606_15846_amd.navsim import NavSim
    from workloads import configs

    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="c2")
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--out", default=TUNING_FILE, help="JSON file the result is merged into")
    ap.add_argument("--table-out", default=None,
                    help="JSON file for the whole sweep table (not kept in the product)")
    ap.add_argument("--full-space", action="store_true")
    ap.add_argument("--burn-in", type=int, default=250,
                    help="steps run before timing, past the episode horizon, so that the timed "
                         "steps hold the steady mix of resets")
    args = ap.parse_args()
    w = configs.build_workload(args.workload)
    cfg = w["cfg"]
    dev = torch.device("cuda", 0)
    sim = NavSim(cfg, w["maps"], w["res"], w["env_map"], device=0, profiles=w["profiles"])
    sim.reset()
    N = cfg["num_envs"]
    acts = torch.from_numpy(configs.uniform_actions(args.steps, N, seed=7)).to(dev)
    burn = torch.from_numpy(configs.uniform_actions(min(args.burn_in, 64), N, seed=8)).to(dev)
    for t in range(args.burn_in):
        sim.step(burn[t % burn.shape[0]])
    best, table = tune(sim, acts, steps=args.steps, verbose=True,
                       space=FULL_SPACE if args.full_space else SPACE)
    key = workload_key(cfg, w["maps"], w["profiles"])
    save(key, best, table, torch.cuda.get_device_name(0), args.out, args.table_out)
    print(json.dumps({"key": key, "best": best}))
    sim.close()


if __name__ == "__main__":
    main()
