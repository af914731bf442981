#!/usr/bin/env python3
"""Benchmark of the short-range non-bonded force path on one MI355X.

Workload: 92,224 atoms at 0.1 atoms/A^3 in a 108.86 x 108.86 x 77.76 A periodic box
(the ApoA1 benchmark's size and shape, synthetic jittered-lattice positions), 8 atom
types, cutoff 12 A with switching from 10 A, float32 positions; one step is one full
force evaluation (binning, cutoff filter and force over all cell pairs, per-atom sums
and energy) on inputs already resident in HBM.

Prints ONE JSON line: within-cutoff pair interactions per second, the roofline of the
pair kernel (algorithmic float32 FLOPs per launch / launch time measured with HIP
events on the launch stream, against the published peak and against that peak scaled
to the shader clock the kernel's workgroups counted), the FP64 oracle timed on the host
cores, and two more
forms of the same path:
  serving  -- 512 requests of 2k-200k atoms (cubes at 0.1 atoms/A^3, Poisson arrivals
              at 200 req/s), continuous batching against the plain one-at-a-time path,
              plus a lowered HBM cap and saturating arrival rates;
  scaling  -- 1,066,628 atoms in a 216.83 A cube, 20 evaluations with positions
              perturbed by N(0, 0.01 A) between calls.

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
CLOCK_NOMINAL_GHZ = 2.4        # the clock that peak is quoted at
FLOP_PER_CANDIDATE = 8         # filter: 3 sub, 1 mul, 2 fma (fma = 2)
FLOP_PER_PAIR = 40             # force, switch, accumulation
# binning: x, y, z, q and type in; sorted (x, y, z, q), type and permutation out; the per-atom
# sums cleared; the pair kernel's prefilter constants out
BIN_BYTES_PER_ATOM = 20 + 24 + 24 + 32
METRIC = "within-cutoff pair-interactions/s @92k atoms; p50/p99 latency mixed batch"
# HBM bytes per launch of the pair kernel at 92,224 atoms, from the FETCH_SIZE and
# WRITE_SIZE counters scaled by a copy of known size (profiles/traffic_pair_fs_92k.md);
# valid only for the kernel code they were taken on (kernel_code_sha256)
PAIR_TRAFFIC = {"kernel_sha256": "4794194dfbde576d4c0a25f8e99242fba4680fe2e709ecfbaf35c35fdde40eef",
                "bytes": (15642 + 29421) * 1024}


def parse():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=100,
                    help="untimed evaluations first (about 17 ms at 92k atoms: after 5 the "
                         "timed steps still ran 4%% slower than after 100)")
    ap.add_argument("--mode", choices=["compact", "compact_full", "predicated"], default="compact",
                    help="compacted half shell (default), compacted full shell, or the "
                         "predicated (uncompacted) half shell")
    ap.add_argument("--accum", choices=["fixed64", "f32atomic"], default="fixed64")
    ap.add_argument("--workload", choices=["apoa1", "stmv"], default="apoa1")
    ap.add_argument("--cpu-seconds", type=float, default=10.0,
                    help="wall time budget of the oracle baseline (0 disables it)")
    ap.add_argument("--latency-reps", type=int, default=50)
    ap.add_argument("--serving-requests", type=int, default=512,
                    help="requests of the serving form (0 disables it)")
    ap.add_argument("--serving-max-batch", type=int, default=32,
                    help="most requests in one batched launch sequence")
    ap.add_argument("--serving-inflight", type=int, default=2,
                    help="most batches on the GPU at once")
    ap.add_argument("--md-steps", type=int, default=200,
                    help="velocity-Verlet steps of the motion-update run (0 disables it)")
    ap.add_argument("--scaling-evals", type=int, default=20,
                    help="evaluations of the 1,066,628-atom scaling shape (0 disables it)")
    ap.add_argument("--copy-calibration-mb", type=int, default=0,
                    help="run a plain copy kernel over this many MiB (read and write) before "
                         "the benchmark, as the reference point of HBM byte counters")
    ap.add_argument("--ewald-steps", type=int, default=5,
                    help="evaluations of the Ewald form at 92k atoms (0 skips it)")
    ap.add_argument("--ablation-steps", type=int, default=10,
                    help="pair-stage timings per data flow in the compacted vs predicated "
                         "comparison (0 disables it)")
    return ap.parse_args()


def kernel_code_sha256(path):
    """sha256 of a source file's code: comments removed and whitespace runs collapsed, so
    that counters stay tied to the code they were taken on and not to its comments."""
    import hashlib
    import re
    with open(path) as f:
        text = f.read()
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    text = " ".join(text.split())
    return hashlib.sha256(text.encode()).hexdigest()


def pair_traffic(args):
    """Counter-measured HBM bytes per pair-kernel launch, or None when the kernel code
    or the configuration differs from the one they were taken on."""
    if args.workload != "apoa1" or args.mode != "compact" or args.accum != "fixed64":
        return None
    src = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_1611_04474_amd",
                       "csrc", "md_pair_fs.hip")
    if kernel_code_sha256(src) != PAIR_TRAFFIC["kernel_sha256"]:
        return None
    return PAIR_TRAFFIC["bytes"]


def pct(v, q):
    return float(np.percentile(np.asarray(v), q)) if len(v) else None


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported: "
              "the path runs on one GPU, and a large system would shard by spatial "
              "decomposition of the cell grid with halo exchange", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1611_04474_amd import api
    from paper_1611_04474_amd import workloads as W

    dev = torch.device("cuda:0")
    if args.copy_calibration_mb > 0:
        # a plain elementwise copy (y = x + 0): reads and writes exactly this many bytes
        n_el = args.copy_calibration_mb * (1 << 20) // 4
        xc = torch.ones(n_el, dtype=torch.float32, device=dev)
        yc = torch.empty_like(xc)
        torch.add(xc, 0.0, out=yc)
        torch.cuda.synchronize()
        del xc, yc
    s = W.apoa1_system() if args.workload == "apoa1" else W.stmv_system()
    flags = {"compact": 0, "compact_full": api.PAIR_FULL_SHELL,
             "predicated": api.PAIR_PREDICATED}[args.mode] | \
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
    n_cand, n_filter, n_pairs, n_slots, n_lanes = api.read_diag(ws)
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
    # the K timed steps: whole evaluations, nothing recorded between their kernels
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        step()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    if api.read_status(ws) != 0:
        raise SystemExit(f"device status {api.read_status(ws):#x}")
    # then K more, with HIP events between the stages (the events themselves take time on
    # the stream, so the stage split and the pair kernel's rate come from this pass)
    events = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(args.steps)]
    for k in range(args.steps):
        step(events[k])
    torch.cuda.synchronize()
    # shader clock of the last pair launch, counted by its own workgroups
    clock_ghz = api.read_clock(ws)
    bin_ms = [e[0].elapsed_time(e[1]) for e in events]
    pair_ms = [e[1].elapsed_time(e[2]) for e in events]
    fin_ms = [e[2].elapsed_time(e[3]) for e in events]
    eval_ms = [e[0].elapsed_time(e[3]) for e in events]
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
            "candidates_examined_per_step": n_slots, "force_lanes_per_step": n_lanes,
            "force_lane_utilisation": n_pairs / n_lanes if n_lanes else None,
            "pairs_per_step": n_pairs,
        },
        "stage_ms": {"bin": statistics.mean(bin_ms), "pair": statistics.mean(pair_ms),
                     "finalize": statistics.mean(fin_ms)},
        "eval_ms": {"p10": pct(eval_ms, 10), "median": pct(eval_ms, 50), "p90": pct(eval_ms, 90)},
        "latency_ms": None,
        "latency_ms_plain_92k": {"p50": pct(lat, 50), "p99": pct(lat, 99),
                                 "kind": "plain path, one 92,224-atom system per call"},
        "roofline": {
            "kernel": "k_pair_fs (filter + force; half shell unless --mode says otherwise)",
            "bound": "alu",
            "achieved": achieved,
            "peak": PEAK_FP32_TFLOPS,
            "unit": "TFLOP/s",
            "frac": achieved / PEAK_FP32_TFLOPS,
            "clock_GHz_nominal": CLOCK_NOMINAL_GHZ,
            "clock_GHz_under_load": clock_ghz or None,
            "peak_at_clock_under_load": (PEAK_FP32_TFLOPS * clock_ghz / CLOCK_NOMINAL_GHZ
                                         if clock_ghz else None),
            "frac_at_clock_under_load": (achieved * CLOCK_NOMINAL_GHZ / (PEAK_FP32_TFLOPS * clock_ghz)
                                         if clock_ghz else None),
            "flop_per_launch": flop_per_launch,
            "traffic": pair_traffic(args),
        },
    }
    del ws, force, energy, pos, typ, q

    if args.serving_requests > 0:
        out["serving"] = serving(args.serving_requests, dev, args.serving_max_batch,
                                 args.serving_inflight)
        tr = out["serving"]["scenarios"]["trace_200hz"]["batched"]
        out["latency_ms"] = {"p50": tr["p50_ms"], "p99": tr["p99_ms"],
                             "kind": f"serving trace: {args.serving_requests} requests of "
                                     "2k-200k atoms at 200 req/s, continuous batching"}
    if args.scaling_evals > 0:
        out["scaling_1m"] = scaling(args.scaling_evals, dev)
    if args.md_steps > 0:
        out["md_vv_92k"] = md_loop(args.md_steps, dev)
    if args.ablation_steps > 0:
        out["ablation_data_flow"] = ablation(args.ablation_steps, dev)
    if args.ewald_steps > 0:
        out["ewald_92k"] = ewald(args.ewald_steps, dev)
    if args.cpu_seconds > 0:
        out["cpu_baseline"] = cpu_baseline(s, args.cpu_seconds)
        out["config"]["pairs_oracle_fp64"] = out["cpu_baseline"].pop("n_pairs")
    print(json.dumps(out), flush=True)


def serving(n_req, dev, max_batch, inflight):
    """The trace and saturating variants, continuous batching vs the plain path."""
    import torch
    from paper_1611_04474_amd import workloads as W
    from paper_1611_04474_amd import serving as S
    reqs, table = W.serving_trace(n_req=n_req)
    systems = [W.request_system(r, table) for r in reqs]
    items = S.prepare(systems, dev)
    pairs = np.array(S.count_pairs(items, dev), dtype=np.int64)
    arrivals = np.array([r.arrival_s for r in reqs])
    # every request's device buffers come from one pool allocated here, sized for the
    # largest budget below (64 GB, or all requests resident if that is less)
    backend = S.GpuBackend(dev, S.pool_bytes(items, 64 << 30), len(items), inflight)
    # warm both paths
    S.run_policy(items, np.zeros(len(items)), backend, 64 << 30, max_batch, inflight)
    S.replay_plain(items[:8], np.zeros(8), dev)
    torch.cuda.synchronize()
    import gc
    gc.collect()
    gc.disable()   # no collector pauses inside the timed replays
    rng = np.random.default_rng(6)
    gaps = rng.exponential(1.0, n_req)
    out = {"requests": n_req, "mean_atoms": float(np.mean([x.n for x in items])),
           "pairs_total": int(pairs.sum()), "max_batch": max_batch, "max_inflight": inflight,
           "scenarios": {}}

    def both(name, arr, budget, plain=True):
        res = {"batched": S.run_policy(items, arr, backend, budget, max_batch,
                                       inflight).summary(pairs)}
        if plain:
            res["plain"] = S.replay_plain(items, arr, dev).summary(pairs)
        res["budget_MB"] = budget / 2 ** 20
        out["scenarios"][name] = res

    both("trace_200hz", arrivals, 64 << 30)
    both("trace_200hz_cap_64MB", arrivals, 64 << 20, plain=False)
    both("all_at_t0", np.zeros(n_req), 64 << 30)
    for rate in (2000.0, 20000.0):
        arr = np.cumsum(gaps / rate)
        both(f"poisson_{int(rate)}hz", arr - arr[0], 64 << 30)
    gc.enable()
    return out


EWALD_ALPHA = 0.3              # 1/A: erfc(0.3 x 12) = 3.6e-7 at the cutoff
EWALD_TOL = 1e-6               # first omitted reciprocal term exp(-pi^2 h^2 / alpha^2)
FLOP_PER_ATOM_WAVEVECTOR = 24  # structure factor 8 (complex multiply-add), forces 16 (two)


def ewald(steps, dev):
    """Coulomb beyond the cutoff by Ewald summation at 92,224 atoms: the short-range call
    with the erfc-screened real-space term, and the reciprocal-space sum. Reports both times
    and the reciprocal kernels' algorithmic rate (24 FLOP per atom and half-space wave
    vector) against the float32 peak."""
    import math
    import torch
    from paper_1611_04474_amd import api
    from paper_1611_04474_amd import workloads as W
    s = W.apoa1_system()
    p = dict(s.params(), flags=api.COULOMB_EWALD, ewald_alpha=EWALD_ALPHA)
    P = api.Params.from_dict(p)
    h = EWALD_ALPHA * math.sqrt(-math.log(EWALD_TOL)) / math.pi
    kmax = [int(math.ceil(h * float(L))) for L in s.box]
    pos = torch.as_tensor(s.pos).to(dev)
    typ = torch.as_tensor(s.types).to(dev)
    q = torch.as_tensor(s.charges).to(dev)
    force = torch.empty((s.n, 3), dtype=torch.float32, device=dev)
    e_short = torch.empty(1, dtype=torch.float64, device=dev)
    e_rec = torch.empty(1, dtype=torch.float64, device=dev)
    ws = api.alloc_workspace(P, s.n, dev)
    _, _, ews = api.ewald_recip(P, pos, q, kmax, force=force, energy=e_rec)
    stream = torch.cuda.current_stream()
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(steps + 2)]
    for k in range(steps + 2):
        evs[k][0].record(stream)
        api.forces(P, pos, typ, q, force=force, energy=e_short, workspace=ws)
        evs[k][1].record(stream)
        api.ewald_recip(P, pos, q, kmax, force=force, energy=e_rec, accumulate=True, workspace=ews)
        evs[k][2].record(stream)
    torch.cuda.synchronize()
    short_ms = [e[0].elapsed_time(e[1]) for e in evs[2:]]
    rec_ms = [e[1].elapsed_time(e[2]) for e in evs[2:]]
    n_half = ((2 * kmax[0] + 1) * (2 * kmax[1] + 1) * (2 * kmax[2] + 1) - 1) // 2
    flop = FLOP_PER_ATOM_WAVEVECTOR * s.n * n_half
    rec_s = statistics.median(rec_ms) * 1e-3
    return {"alpha_per_A": EWALD_ALPHA, "kmax": kmax, "half_space_wavevectors": n_half,
            "short_range_ms_median": statistics.median(short_ms),
            "reciprocal_ms_median": statistics.median(rec_ms),
            "energy_short": float(e_short.item()), "energy_reciprocal_self_background": float(e_rec.item()),
            "reciprocal_flop": flop, "reciprocal_TFLOPs": flop / rec_s / 1e12,
            "reciprocal_frac_of_fp32_peak": flop / rec_s / 1e12 / PEAK_FP32_TFLOPS,
            "status": api.read_status(ws) | api.read_status(ews)}


def md_loop(steps, dev, dt=0.5):
    """The motion update around the force path: velocity Verlet (md_run_vv_f32) on 92,224
    atoms in the force benchmark's box and density, with LJ parameters that keep the
    dynamics bounded (workloads.liquid_system) and velocities of about 300 K. One call
    of `steps` steps is timed with HIP events after a 10-step warm-up, next to the force
    call alone on the same system; the energies of every step give the deviation of the
    total energy from its start."""
    import torch
    from paper_1611_04474_amd import api
    from paper_1611_04474_amd import workloads as W
    s = W.liquid_system(W.APOA1_N, W.APOA1_BOX)
    v, im = W.velocities(s.types)
    P = api.Params.from_dict(s.params())
    pos = torch.as_tensor(s.pos).to(dev)
    typ = torch.as_tensor(s.types).to(dev)
    q = torch.as_tensor(s.charges).to(dev)
    vel = torch.as_tensor(v).to(dev)
    inv_m = torch.as_tensor(im).to(dev)
    ws = api.alloc_workspace(P, s.n, dev)
    force, e0 = api.forces(P, pos, typ, q, workspace=ws)
    stream = torch.cuda.current_stream()
    api.run_vv(P, pos, vel, typ, q, inv_m, force, dt, 10, workspace=ws)
    en = torch.empty((steps, 2), dtype=torch.float64, device=dev)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    a.record(stream)
    api.run_vv(P, pos, vel, typ, q, inv_m, force, dt, steps, energies=en, workspace=ws)
    b.record(stream)
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / steps
    status = api.read_status(ws)
    # the force call alone on the final positions
    f2 = torch.empty_like(force)
    e2 = torch.empty(1, dtype=torch.float64, device=dev)
    fms = []
    for k in range(steps // 4 + 2):
        c, d = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        c.record(stream)
        api.forces(P, pos, typ, q, force=f2, energy=e2, workspace=ws)
        d.record(stream)
        torch.cuda.synchronize()
        if k >= 2:
            fms.append(c.elapsed_time(d))
    e = en.cpu().numpy()
    tot = e[:, 0] + e[:, 1]
    return {"n_atoms": s.n, "dt_fs": dt, "steps": steps, "ms_per_step": ms,
            "force_call_ms_median": pct(fms, 50), "ns_per_day": dt * 1e-6 * 86400e3 / ms,
            "energy_first": float(tot[0]), "energy_max_dev": float(np.abs(tot - tot[0]).max()),
            "kinetic_first": float(e[0, 1]), "kinetic_last": float(e[-1, 1]),
            "status": int(status)}


def scaling(n_eval, dev):
    """20 evaluations of the 1,066,628-atom cube, positions perturbed between calls."""
    import torch
    from paper_1611_04474_amd import api
    from paper_1611_04474_amd import workloads as W
    s = W.stmv_system()
    P = api.Params.from_dict(s.params())
    pos = torch.as_tensor(s.pos).to(dev)
    typ = torch.as_tensor(s.types).to(dev)
    q = torch.as_tensor(s.charges).to(dev)
    force = torch.empty((s.n, 3), dtype=torch.float32, device=dev)
    energy = torch.empty(1, dtype=torch.float64, device=dev)
    ws = api.alloc_workspace(P, s.n, dev)
    api.forces(P.with_flags(api.DIAG_COUNTERS), pos, typ, q, force=force, energy=energy,
               workspace=ws)
    n_cand, _, n_pairs, _, _ = api.read_diag(ws)
    stream = torch.cuda.current_stream()
    # positions of each evaluation: x += N(0, 0.01 A) per call, wrapped by the call; all
    # of them resident in HBM before the timing starts
    xs, x = [], s.pos
    for d in W.perturbation_stream(s.n, n_eval):
        x = W.perturb(x, d)
        xs.append(torch.as_tensor(x).to(dev))
    for _ in range(2):
        api.forces(P, pos, typ, q, force=force, energy=energy, workspace=ws)
    torch.cuda.synchronize()
    # no synchronisation between evaluations, so the host enqueues ahead of the GPU and the
    # events time kernels, not launch gaps; a device-to-device copy, outside the timed
    # spans, puts each evaluation's positions in place
    evs = []
    for k in range(n_eval):
        pos.copy_(xs[k])
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        ev[0].record(stream)
        api.forces_stages(P, pos, typ, q, force, energy, ws, api.STAGE_BIN)
        ev[1].record(stream)
        api.forces_stages(P, pos, typ, q, force, energy, ws, api.STAGE_PAIR | api.STAGE_FINALIZE)
        ev[2].record(stream)
        evs.append(ev)
    torch.cuda.synchronize()
    ms = [ev[0].elapsed_time(ev[2]) for ev in evs]
    bin_ms = [ev[0].elapsed_time(ev[1]) for ev in evs]
    del xs
    if api.read_status(ws) != 0:
        raise SystemExit(f"device status {api.read_status(ws):#x} (1M-atom system)")
    med = pct(ms, 50)
    flop = FLOP_PER_CANDIDATE * n_cand + FLOP_PER_PAIR * n_pairs
    bmed = pct(bin_ms, 50)
    return {"n_atoms": s.n, "evaluations": n_eval, "eval_ms_median": med,
            "bin_ms_median": bmed,
            # algorithmic binning bytes: read x, y, z, q, type (20 B), write the sorted
            # float4, type and permutation (24 B), clear the per-atom int64 sums (24 B)
            "bin_GBps_algorithmic": BIN_BYTES_PER_ATOM * s.n / (bmed * 1e-3) / 1e9,
            "eval_ms_p10": pct(ms, 10), "eval_ms_p90": pct(ms, 90),
            "pairs_first_eval": n_pairs, "candidates_first_eval": n_cand,
            "pairs_per_s": n_pairs / (med * 1e-3),
            "whole_eval_algorithmic_TFLOPs": flop / (med * 1e-3) / 1e12}


def ablation(steps, dev):
    """The paper's dynamic data flow on a GPU: the compacted kernel (cutoff filter feeding
    dense force passes through FIFOs), in its half-shell and full-shell forms, against the
    predicated one (every candidate through the force arithmetic under the cutoff
    predicate), on the 92,224-atom system: pair-stage time, force-stage lane utilisation
    (unique pairs / lanes through the force arithmetic; the full shell evaluates every
    pair twice, so its figure is at most 0.5). Then the half-shell kernel with 1 to 4
    candidate batches of 64 per force pass (the drain depth; 2 is the default): the GPU
    analog of the paper's sweep of distance PEs per force PE."""
    import torch
    from paper_1611_04474_amd import api
    from paper_1611_04474_amd import workloads as W
    s = W.apoa1_system()
    pos = torch.as_tensor(s.pos).to(dev)
    typ = torch.as_tensor(s.types).to(dev)
    q = torch.as_tensor(s.charges).to(dev)
    force = torch.empty((s.n, 3), dtype=torch.float32, device=dev)
    energy = torch.empty(1, dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream()
    out = {}
    for name, flags in (("compacted_half_shell", 0), ("compacted_full_shell", api.PAIR_FULL_SHELL),
                        ("predicated_half_shell", api.PAIR_PREDICATED)):
        P = api.Params.from_dict(s.params(), flags)
        ws = api.alloc_workspace(P, s.n, dev)
        api.forces(P.with_flags(flags | api.DIAG_COUNTERS), pos, typ, q, force=force,
                   energy=energy, workspace=ws)
        cand, _, pairs, _, lanes = api.read_diag(ws)
        ms = []
        for k in range(steps + 2):
            api.forces_stages(P, pos, typ, q, force, energy, ws, api.STAGE_BIN)
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            api.forces_stages(P, pos, typ, q, force, energy, ws, api.STAGE_PAIR)
            b.record(stream)
            api.forces_stages(P, pos, typ, q, force, energy, ws, api.STAGE_FINALIZE)
            torch.cuda.synchronize()
            if k >= 2:
                ms.append(a.elapsed_time(b))
        med = pct(ms, 50)
        out[name] = {"pair_ms_median": med, "pairs": pairs, "force_lanes": lanes,
                     "force_lane_utilisation": pairs / lanes if lanes else None,
                     "pairs_per_s_pair_stage": pairs / (med * 1e-3)}
    out["speedup_compacted"] = (out["predicated_half_shell"]["pair_ms_median"] /
                                out["compacted_half_shell"]["pair_ms_median"])
    # candidate batches per force pass: 64 d passing pairs drained together from a FIFO
    P0 = api.Params.from_dict(s.params())
    sweep = {}
    for d in (1, 2, 3, 4):
        P = P0.with_flags(api.PAIR_DRAIN(d))
        ws = api.alloc_workspace(P, s.n, dev)
        api.forces(P.with_flags(P.flags | api.DIAG_COUNTERS), pos, typ, q, force=force,
                   energy=energy, workspace=ws)
        _, _, pairs, _, lanes = api.read_diag(ws)
        ms = []
        for k in range(steps + 2):
            api.forces_stages(P, pos, typ, q, force, energy, ws, api.STAGE_BIN)
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            api.forces_stages(P, pos, typ, q, force, energy, ws, api.STAGE_PAIR)
            b.record(stream)
            api.forces_stages(P, pos, typ, q, force, energy, ws, api.STAGE_FINALIZE)
            torch.cuda.synchronize()
            if k >= 2:
                ms.append(a.elapsed_time(b))
        med = pct(ms, 50)
        sweep[str(d)] = {"pair_ms_median": med, "force_lanes": lanes,
                         "force_lane_utilisation": pairs / lanes if lanes else None,
                         "pairs_per_s_pair_stage": pairs / (med * 1e-3)}
    out["drain_depth_sweep_half_shell"] = sweep
    out["speedup_half_over_full_shell"] = (out["compacted_full_shell"]["pair_ms_median"] /
                                           out["compacted_half_shell"]["pair_ms_median"])
    # workgroups per home cell: the 92,224-atom system (486 cells) and a 20,000-atom cube
    # of 4^3 cells (a median serving request), whole evaluations
    split = {}
    for label, sysm in (("apoa1_92k_486_cells", s), ("cube_20k_64_cells",
                                                    W.gen_system(20000, (58.5, 58.5, 58.5), 12))):
        pos_s = torch.as_tensor(sysm.pos).to(dev)
        typ_s = torch.as_tensor(sysm.types).to(dev)
        q_s = torch.as_tensor(sysm.charges).to(dev)
        f_s = torch.empty((sysm.n, 3), dtype=torch.float32, device=dev)
        row = {}
        for sv in (1, 2, 4):
            P = api.Params.from_dict(sysm.params(), api.PAIR_SPLIT(sv))
            ws = api.alloc_workspace(P, sysm.n, dev)
            api.forces(P.with_flags(P.flags | api.DIAG_COUNTERS), pos_s, typ_s, q_s, force=f_s,
                       energy=energy, workspace=ws)
            pairs = api.read_diag(ws)[2]
            evs = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(steps + 2)]
            for k in range(steps + 2):
                evs[k][0].record(stream)
                api.forces_stages(P, pos_s, typ_s, q_s, f_s, energy, ws, api.STAGE_BIN)
                evs[k][1].record(stream)
                api.forces_stages(P, pos_s, typ_s, q_s, f_s, energy, ws, api.STAGE_PAIR)
                evs[k][2].record(stream)
                api.forces_stages(P, pos_s, typ_s, q_s, f_s, energy, ws, api.STAGE_FINALIZE)
            torch.cuda.synchronize()
            pair_ms = pct([e[1].elapsed_time(e[2]) for e in evs[2:]], 50)
            row[str(sv)] = {"pair_ms_median": pair_ms, "pairs_per_s_pair_stage": pairs / (pair_ms * 1e-3)}
        cells = int(np.prod(api.workspace_layout(sysm.params(), sysm.n)["dims"]))
        sa = 256 // cells
        row["automatic"] = 4 if sa >= 4 else 2 if sa >= 2 else 1
        split[label] = row
    out["workgroups_per_home_cell"] = split
    return out


def cpu_baseline(s, budget_s):
    """The FP64 oracle's cell-list evaluation (Algorithm 1) on this host's cores, timed over
    whole evaluations for about budget_s; then one evaluation on one thread (the paper's
    1-core vs 12-core comparison, Table 2) and one of the 1,066,628-atom cube on all."""
    import oracle
    from paper_1611_04474_amd import workloads as W
    threads = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or os.cpu_count()
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
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
    t1 = time.perf_counter()
    oracle.forces(s.params(), s.pos, s.types, s.charges, "celllist", n_threads=1)
    one = time.perf_counter() - t1
    big = W.stmv_system()
    t2 = time.perf_counter()
    rb = oracle.forces(big.params(), big.pos, big.types, big.charges, "celllist", n_threads=threads)
    el_big = time.perf_counter() - t2
    return {"value": n_pairs * runs / el, "unit": "pair-interactions/s", "cores": threads,
            "kind": "oracle",
            "sample": f"{runs} full FP64 cell-list evaluations of the {s.n}-atom system "
                      f"in {el:.1f} s", "n_pairs": n_pairs,
            "cpu_model": model, "nproc": os.cpu_count(),
            "one_thread_pairs_per_s": n_pairs / one,
            "stmv_1m_pairs_per_s": rb.n_pairs / el_big,
            "stmv_1m_sample": f"1 evaluation of the {big.n}-atom cube on {threads} threads "
                              f"in {el_big:.1f} s"}


if __name__ == "__main__":
    main()
