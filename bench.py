#!/usr/bin/env python3
"""Benchmark of the short-range non-bonded force path on one MI355X.

Workload: 92,224 atoms at 0.1 atoms/A^3 in a 108.86 x 108.86 x 77.76 A periodic box
(the ApoA1 benchmark's size and shape, synthetic jittered-lattice positions), 8 atom
types, cutoff 12 A with switching from 10 A, float32 positions; one step is one full
force evaluation (binning, cutoff filter and force over all cell pairs, per-atom sums
and energy) on inputs already resident in HBM.

Prints ONE JSON line: within-cutoff pair interactions per second, the roofline of the
pair kernel (algorithmic float32 FLOPs per launch / launch time measured with HIP
events on the launch stream), and the FP64 oracle timed on the host cores.

    python bench.py [--steps K] [--warmup W] [--gpus 1]
"""
import argparse
import json
import os
import statistics
import sys
import time

import numpy as np

PEAK_FP32_TFLOPS = 157.3       # MI355X published float32 vector peak
FLOP_PER_CANDIDATE = 8         # filter: 3 sub, 1 mul, 2 fma (fma = 2)
FLOP_PER_PAIR = 40             # force, switch, accumulation
METRIC = "within-cutoff pair-interactions/s @92k atoms; p50/p99 latency mixed batch"


def parse():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--mode", choices=["compact", "predicated"], default="compact")
    ap.add_argument("--accum", choices=["fixed64", "f32atomic"], default="fixed64")
    ap.add_argument("--workload", choices=["apoa1", "stmv"], default="apoa1")
    ap.add_argument("--cpu-seconds", type=float, default=10.0,
                    help="wall time budget of the oracle baseline (0 disables it)")
    ap.add_argument("--latency-reps", type=int, default=50)
    return ap.parse_args()


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(see DESIGN.md for how the path would shard)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1611_04474_amd import api
    from paper_1611_04474_amd import workloads as W

    dev = torch.device("cuda:0")
    s = W.apoa1_system() if args.workload == "apoa1" else W.stmv_system()
    flags = (api.PAIR_PREDICATED if args.mode == "predicated" else 0) | \
            (api.ACCUM_F32_ATOMIC if args.accum == "f32atomic" else 0)
    P = api.Params.from_dict(s.params(), flags)
    pos = torch.as_tensor(s.pos).to(dev)
    typ = torch.as_tensor(s.types).to(dev)
    q = torch.as_tensor(s.charges).to(dev)
    force = torch.empty((s.n, 3), dtype=torch.float32, device=dev)
    energy = torch.empty(1, dtype=torch.float64, device=dev)
    ws = api.alloc_workspace(P, s.n, dev)
    stream = torch.cuda.current_stream()

    # candidate and pair counts of this workload, from the kernel's own counters
    api.forces(P.with_flags(flags | api.DIAG_COUNTERS), pos, typ, q, force=force, energy=energy,
               workspace=ws)
    n_cand, n_filter, n_pairs, n_slots = api.read_diag(ws)
    flop_per_launch = FLOP_PER_CANDIDATE * n_cand + FLOP_PER_PAIR * n_pairs

    def step(evs=None):
        if evs is None:
            api.forces_stages(P, pos, typ, q, force, energy, ws, api.STAGE_ALL)
            return
        evs[0].record(stream)
        api.forces_stages(P, pos, typ, q, force, energy, ws, api.STAGE_BIN)
        evs[1].record(stream)
        api.forces_stages(P, pos, typ, q, force, energy, ws, api.STAGE_PAIR)
        evs[2].record(stream)
        api.forces_stages(P, pos, typ, q, force, energy, ws, api.STAGE_FINALIZE)
        evs[3].record(stream)

    for _ in range(args.warmup):
        step()
    events = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(events[k])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    if api.read_status(ws) != 0:
        raise SystemExit(f"device status {api.read_status(ws):#x}")
    bin_ms = [e[0].elapsed_time(e[1]) for e in events]
    pair_ms = [e[1].elapsed_time(e[2]) for e in events]
    fin_ms = [e[2].elapsed_time(e[3]) for e in events]
    ms_per_step = 1e3 * wall / args.steps
    pair_avg_s = statistics.mean(pair_ms) * 1e-3
    achieved = flop_per_launch / pair_avg_s / 1e12

    # single-call latency of the plain path (each call synchronised on its own)
    lat = []
    for _ in range(args.latency_reps):
        torch.cuda.synchronize()
        t = time.perf_counter()
        step()
        torch.cuda.synchronize()
        lat.append(1e3 * (time.perf_counter() - t))
    lat = np.array(lat)

    out = {
        "metric": METRIC,
        "value": n_pairs / (wall / args.steps),
        "unit": "pair-interactions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": ("ApoA1-sized periodic box: 92,224 atoms, 108.86x108.86x77.76 A"
                         if args.workload == "apoa1" else
                         "STMV-sized periodic cube: 1,066,628 atoms, 216.83 A"),
            "n_atoms": s.n, "density_per_A3": round(s.n / float(np.prod(s.box)), 5),
            "r_cut_A": 12.0, "r_switch_A": 10.0, "n_types": 8,
            "pair_mode": args.mode, "accumulation": args.accum,
            "candidates_per_step": n_cand, "filter_passes_per_step": n_filter,
            "pairs_per_step": n_pairs,
        },
        "stage_ms": {"bin": statistics.mean(bin_ms), "pair": statistics.mean(pair_ms),
                     "finalize": statistics.mean(fin_ms)},
        "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                       "kind": "plain path, one system per call"},
        "roofline": {
            "kernel": "pair (filter + force)",
            "bound": "alu",
            "achieved": achieved,
            "peak": PEAK_FP32_TFLOPS,
            "unit": "TFLOP/s",
            "frac": achieved / PEAK_FP32_TFLOPS,
            "flop_per_launch": flop_per_launch,
            "traffic": None,
        },
    }

    if args.cpu_seconds > 0:
        out["cpu_baseline"] = cpu_baseline(s, args.cpu_seconds)
        out["config"]["pairs_oracle_fp64"] = out["cpu_baseline"].pop("n_pairs")
    print(json.dumps(out), flush=True)


def cpu_baseline(s, budget_s):
    """The FP64 oracle's cell-list evaluation (Algorithm 1) on this host's cores."""
    import oracle
    threads = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or os.cpu_count()
    oracle.lib()
    runs = 0
    n_pairs = None
    t0 = time.perf_counter()
    while True:
        r = oracle.forces(s.params(), s.pos, s.types, s.charges, "celllist", n_threads=threads)
        n_pairs = r.n_pairs
        runs += 1
        if time.perf_counter() - t0 >= budget_s:
            break
    el = time.perf_counter() - t0
    return {"value": n_pairs * runs / el, "unit": "pair-interactions/s", "cores": threads,
            "kind": "oracle",
            "sample": f"{runs} full FP64 cell-list evaluations of the {s.n}-atom system "
                      f"in {el:.1f} s", "n_pairs": n_pairs}


if __name__ == "__main__":
    main()
