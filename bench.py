#!/usr/bin/env python3
"""PRISM benchmark on one MI355X.

Workload: PRISM f=4 on the 100 x 100 x 100 A nanoparticle-in-amorphous cell,
1024 x 1024 grid, 2 A slices (50), 200 keV, 20 mrad, 1245 beams, 128 x 128
probe scan, 1-mrad annular bins.  One step = the whole hot path on resident
inputs: compact S-matrix build (transmission, 50 x row/column propagation
passes, real-space store) followed by synthesis of all 16384 probes
(coefficients, windowed contraction, window FFT, detector sums).

Prints one JSON line.  `value` is probe positions per second of whole steps.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
PEAK_FP32_TFLOPS = 157.3          # published FP32 vector peak (packed FP32: 2 FMAs per lane per clock)
PEAK_FP32_UNPACKED_TFLOPS = 78.6  # 256 CUs x 4 SIMDs x 16 lanes x 2 (FMA) x 2.4 GHz, one FMA per lane per clock
PEAK_BF16_TFLOPS = 2500.0

# Kernel sources whose PMC traffic figures are recorded under profiles/; a
# recorded figure is used only while these files hash to the recorded value.
TRAFFIC_SOURCES = ("paper_1706_08563_amd/csrc/propagate.hip", "paper_1706_08563_amd/csrc/fft.hpp",
                   "paper_1706_08563_amd/csrc/kernels.hpp")


def source_hash(files=TRAFFIC_SOURCES):
    import hashlib
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def recorded_traffic(kernel, workload):
    """HBM bytes per launch recorded from FETCH_SIZE/WRITE_SIZE counters, or
    None when no record exists or the kernel sources changed since."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_pmc_traffic.md")
    if not os.path.exists(path):
        return None
    rec = {}
    with open(path) as fh:
        for line in fh:
            if line.startswith("- ") and ": " in line:
                k, v = line[2:].strip().split(": ", 1)
                rec[k] = v.strip("` ")
    if rec.get("source_sha256") != source_hash():
        return None
    try:
        return float(rec["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def copy_bandwidth(gib=2, reps=5):
    """Bytes read + written per second by the library's plain streaming copy
    (one 16-byte load and store per thread) of `gib` GiB: the practical HBM
    ceiling next to the 8 TB/s peak."""
    import torch

    import paper_1706_08563_amd as P
    x = torch.ones(gib << 28, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    P.prism_device_copy(x, y)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        P.prism_device_copy(x, y)
    b.record()
    torch.cuda.synchronize()
    gbs = 2.0 * x.numel() * 4 * reps / (a.elapsed_time(b) * 1e-3) / 1e9
    del x, y
    torch.cuda.empty_cache()
    return gbs


def pass_flops(n, B, rows):
    """Algorithmic FP32 flops of one propagation-pass launch over B beams:
    `rows` lines of two inverse and two forward (n/2)-point complex FFTs
    (5 m log2 m each), the pointwise product with the transmission or the
    propagator (6 n per line) and the band twiddles (7 n per line)."""
    m = n // 2
    return float(B) * rows * (4 * 5 * m * math.log2(m) + 13 * n)

METRIC = "probe positions/s + S-matrix beams/s @1024², ≤1e-4 rel err vs FP64; p99 latency"

GOLDEN = os.path.join(ROOT, "tests", "golden")
TOL = 1e-4


def load_fixture(name):
    """FP64 3D outputs of a workload's 16 x 16 probe subset, written by
    tests/golden/make_golden.py from the FP64 oracle; None when absent."""
    import numpy as np
    path = os.path.join(GOLDEN, f"{name}_fp64_subset.npz")
    if not os.path.exists(path):
        return None
    with np.load(path, allow_pickle=False) as z:
        return {k: z[k] for k in z.files}


def subset_index(scan, sub):
    """Indices, within a row-major (j, i) scan, of every sub-th probe per axis."""
    import numpy as np
    nx, ny = scan
    j, i = np.meshgrid(np.arange(0, ny, sub), np.arange(0, nx, sub), indexing="ij")
    return (j * nx + i).ravel()


def detector_errors(got, ref, dalpha=1e-3, adf_from=0.04):
    """Error of a 3D output against a reference: Frobenius relative error over
    probes x bins, relative error of the dark-field signal (bins from 40 mrad),
    and the worst per-bin relative error over probes (|dD| / max(|D_ref|,
    1e-3 max D_ref)); `within_1e-4` applies the element-wise gate
    |dD| <= 1e-4 |D_ref| + 1e-7 max D_ref with both norm-wise gates."""
    import numpy as np
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    rel_all = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
    b = np.arange(ref.shape[1])
    sel = b * dalpha >= adf_from - 1e-15
    ag, ar = got[:, sel].sum(1), ref[:, sel].sum(1)
    rel_adf = float(np.linalg.norm(ag - ar) / np.linalg.norm(ar))
    top = float(np.max(np.abs(ref)))
    pb = np.max(np.abs(got - ref) / np.maximum(np.abs(ref), 1e-3 * top), axis=0)
    elem = bool(np.all(np.abs(got - ref) <= TOL * np.abs(ref) + TOL * 1e-3 * top))
    return {"rel_all": rel_all, "rel_adf": rel_adf, "per_bin_max": float(pb.max()), "worst_bin": int(np.argmax(pb)),
            "within_1e-4": bool(elem and rel_all <= TOL and rel_adf <= TOL)}


def accuracy_report(w, d, S, out, ms_out, prec_name):
    """Accuracy of the benchmarked run on the workload's 16 x 16 probe subset
    against the FP64 fixture of the same cell: the timed step's own output,
    the three contraction precisions, plain multislice on the same probes
    (GPU against FP64), and PRISM against multislice (the method's own
    approximation at this f, GPU and FP64; reported, not gated)."""
    import numpy as np
    import torch

    import paper_1706_08563_amd as P
    fx = load_fixture(w.name)
    if fx is None:
        return {"fixture": None}
    sub = w.scan[0] // 16
    idx = subset_index(w.scan, sub)
    import workloads as W
    xy = W.scan_positions(w.cell, *w.scan, sub=sub)
    assert np.array_equal(xy, fx["probe_xy"]), "fixture positions differ from the scan subset"
    rep = {"fixture": os.path.relpath(os.path.join(GOLDEN, f"{w.name}_fp64_subset.npz"), ROOT),
           "probes": int(len(idx))}
    timed = out[torch.from_numpy(idx).to(out.device)].cpu().numpy()
    rep[f"timed_{prec_name}_vs_fp64"] = detector_errors(timed, fx["prism"])
    plan = P.prism_probe_plan_upload(d, xy)
    gpu = {}
    for name, prec in (("fp32", P.PRISM_FP32), ("bf16x3", P.PRISM_SPLIT_BF16X3), ("bf16", P.PRISM_BF16)):
        gpu[name] = P.prism_probe_outputs(d, S, plan, prec).cpu().numpy()
        rep[f"{name}_vs_fp64"] = detector_errors(gpu[name], fx["prism"])
    if ms_out is not None and "multislice" in fx:
        ms_w = W.WORKLOADS["multislice_np_1024"]
        assert ms_w.cell == w.cell and ms_w.seed == w.seed and ms_w.n == w.n
        midx = subset_index(ms_w.scan, ms_w.scan[0] // 16)
        ms = ms_out[torch.from_numpy(midx).to(ms_out.device)].cpu().numpy()
        rep["multislice_gpu_vs_fp64"] = detector_errors(ms, fx["multislice"])
        rep[f"prism_f{w.f}_vs_multislice_gpu_{prec_name}"] = detector_errors(timed, ms)
        rep[f"prism_f{w.f}_vs_multislice_fp64"] = detector_errors(fx["prism"], fx["multislice"])
    return rep


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--precision", choices=["fp32", "bf16x3", "bf16"], default="bf16x3")
    ap.add_argument("--workload", default="prism_f4_np_1024",
                    choices=["prism_f4_np_1024", "prism_f8_np_2048", "prism_f2_sc_256"],
                    help="PRISM workload (default: f = 4 at 1024^2)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-beams", type=int, default=3)
    ap.add_argument("--cpu-probes", type=int, default=12)
    ap.add_argument("--serve", action="store_true", help="serving benchmark (Poisson stream of mixed requests)")
    ap.add_argument("--requests", type=int, default=200)
    ap.add_argument("--loads", default="0.4,0.8,1.6",
                    help="offered loads, as fractions of the capacity measured by a saturation run")
    ap.add_argument("--grids", default="256,512,1024,2048", help="grid sizes of the serving requests")
    ap.add_argument("--capacity", type=float, default=None,
                    help="serving: requests/s measured by an earlier saturation run (skips the saturation run)")
    ap.add_argument("--saturation-only", action="store_true", help="serving: only the saturation run")
    ap.add_argument("--no-serving", action="store_true",
                    help="leave the bounded serving leg (16 requests, one offered load) out of the default run")
    ap.add_argument("--precision-study", action="store_true",
                    help="only the 2048^2 f=8 contraction precision study (part of the default run)")
    ap.add_argument("--no-precision-study", action="store_true",
                    help="leave the 2048^2 precision study out of the default run")
    ap.add_argument("--streaming-study", action="store_true",
                    help="single-transfer vs streaming memory model on the default workload: time and peak HBM")
    ap.add_argument("--budget-fraction", type=float, default=0.1,
                    help="streaming study: device budget as a fraction of the single-transfer footprint")
    ap.add_argument("--pmc-driver", action="store_true",
                    help="short program for hardware-counter runs: the default workload's build cut to 4 slices, "
                         "one synthesis of its probes, and a 256 MiB device copy for counter calibration")
    return ap.parse_args()


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def cpu_baseline(w, d, n_beams, n_probes, args):
    """Time the FP64 oracle on a bounded sample of the same workload.

    Multislice propagation and window synthesis cost does not depend on the
    values, so the sample uses seeded random inputs of the workload's shape:
    `cpu_beams` S-matrix layers (50 slices each) and `cpu_probes` probe
    syntheses over all beams; the step time is extrapolated to every beam and
    every probe of the scan.
    """
    import numpy as np
    import oracle as O
    import workloads as W

    rng = np.random.default_rng(1234)
    n, L = w.n, w.cell[0]
    V = rng.uniform(0.0, 60.0, size=(w.n_slices, n, n))
    t = O.transmission(V, d.sigma)
    Pp = O.propagator(n, L, d.lambda_, w.dz)
    beams = O.beam_set(n, L, d.lambda_, w.alpha_max, w.f)
    t0 = time.perf_counter()
    for b in range(args.cpu_beams):
        O.smatrix_layer(t, Pp, int(beams[b, 0]), int(beams[b, 1]))
    t_beam = (time.perf_counter() - t0) / args.cpu_beams
    M = d.m_win
    S = W.random_complex((len(beams), M, M), rng)
    xy = W.scan_positions(w.cell, *w.scan, sub=max(1, w.scan[0] // 4))[: args.cpu_probes]
    t0 = time.perf_counter()
    O.prism_outputs(S, beams, L, n, d.lambda_, w.f, xy)
    t_probe = (time.perf_counter() - t0) / len(xy)
    step = n_beams * t_beam + n_probes * t_probe
    return {"value": n_probes / step, "unit": "probe positions/s", "cores": os.cpu_count(), "kind": "oracle",
            "cpu_model": cpu_model(),
            "sample": f"{args.cpu_beams} S-matrix layers ({w.n_slices} slices, {n}^2, FP64) at "
                      f"{t_beam:.3f} s/beam and {len(xy)} probe syntheses ({n_beams} beams, {M}^2 window) at "
                      f"{t_probe:.3f} s/probe, extrapolated to {n_beams} beams + {n_probes} probes "
                      f"= {step:.0f} s per step",
            "beams_per_s": 1.0 / t_beam}


def device_info():
    """Name, architecture, compute units and memory of the benchmarked GPU."""
    import torch
    p = torch.cuda.get_device_properties(0)
    return {"name": p.name, "arch": getattr(p, "gcnArchName", None), "compute_units": p.multi_processor_count,
            "memory_GB": p.total_memory / 1e9}


def cpu_model():
    """The host CPU's model name (first processor in /proc/cpuinfo)."""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def serving_report(args, n_requests, grids, loads, seed=4, quiet=False, capacity=None, saturation_only=False):
    """Continuous-batching serving of a Poisson stream of mixed PRISM requests
    (`n_requests` requests of the stream seeded `seed`): a saturation run for
    the capacity, then one run per offered load (fraction of that capacity),
    alone-vs-mix for the three smallest requests and a sequential plain
    multislice baseline on the same GPU.  Returns the report."""
    import numpy as np
    import torch

    import paper_1706_08563_amd as P
    from paper_1706_08563_amd import serve as SV
    import workloads as W

    prec = {"fp32": P.PRISM_FP32, "bf16x3": P.PRISM_SPLIT_BF16X3, "bf16": P.PRISM_BF16}[args.precision]
    free, total = torch.cuda.mem_get_info()
    cap = int(0.8 * free)

    def run(rate, tag):
        """The request stream (same requests, arrivals scaled to `rate`)
        through a fresh scheduler and executor; returns (scheduler, wall s)."""
        reqs = []
        for p in W.serving_stream(n_requests, rate, seed=seed, grids=grids):
            r = SV.Request(**p)
            r.sample = W.serving_sample(r.cell, r.seed)
            reqs.append(r)
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
        log(f"[{tag}] serving {len(reqs)} requests at {rate:.3f}/s, budget {cap / 1e9:.1f} GB")
        ex = SV.GpuExecutor(prec, jobs_per_request=4)
        ex.reserve_arena()                 # the server's device arena, allocated before the stream starts
        torch.cuda.synchronize()
        # batch cost: 2.5e12 complex multiply-adds, ~50 ms of split-BF16 contraction
        sched = SV.Scheduler(cap, max_building=4, max_jobs=24, jobs_per_request=4, batch_cost=2.5e12)
        t0 = time.perf_counter()
        SV.serve(reqs, ex, sched, on_done=None if quiet else
                 lambda r: log(f"  [{tag}] done {r.rid} n={r.n} f={r.f} S={r.n_slices} P={r.n_probes} "
                               f"latency {r.latency:.2f} s, device free {torch.cuda.mem_get_info()[0] / 1e9:.0f} GB"))
        torch.cuda.synchronize()
        return sched, time.perf_counter() - t0

    # standalone capacity: every request present at t = 0 (saturation),
    # unless the caller gives it (from an earlier saturation run)
    sat_summary = None
    if capacity is None:
        sat, sat_wall = run(0.0, "saturation")
        capacity = len(sat.done) / sat_wall
        sat_summary = SV.summarize(sat, sat_wall)
        if saturation_only:
            return {"metric": "serving saturation run (all requests at t = 0)", "requests": sat_summary["requests"],
                    "rejected": sat_summary["rejected"], "wall_s": sat_wall, "capacity_requests_per_s": capacity,
                    "saturation_probes_per_s": sat_summary["probes_per_s"], "latency_by_grid": sat_summary["latency_by_grid"],
                    "stream_seed": seed, "grids": list(grids), "data": "synthetic"}
    sweep = {}
    for ld in loads:
        sc, wl = run(ld * capacity, f"load {ld}")
        sweep[ld] = (sc, wl, SV.summarize(sc, wl))
    ld0 = 0.8 if 0.8 in sweep else loads[0]
    sched, wall, summ = sweep[ld0]
    rate = ld0 * capacity
    # alone vs in the mix, for the three smallest requests
    small = sorted(sched.done, key=lambda r: r.n * r.n * r.n_slices)[:3]
    diffs = []
    for r in small:
        a = SV.Request(r.rid, 0.0, r.n, r.f, r.n_slices, r.scan, r.seed, sample=W.serving_sample(r.cell, r.seed))
        SV.serve([a], SV.GpuExecutor(prec), SV.Scheduler(cap, max_building=1, max_jobs=1))
        diffs.append(float(np.max(np.abs(a.result - r.result))))
    # sequential plain multislice on the same GPU, timed per (n, slices) class
    # on 8 probes and extrapolated to every request's scan
    ms_time = 0.0
    classes = {}
    for r in sched.done:
        classes.setdefault((r.n, r.n_slices), []).append(r)
    for (n, ns), rs in classes.items():
        r = rs[0]
        g = P.prism_grid_init(r.cell, 2.0, n)
        pos, sp, species = r.sample() if callable(r.sample) else W.serving_sample(r.cell, r.seed)()
        V = P.prism_project_potential(pos, sp, species, g)
        xy = W.scan_positions(r.cell, 8, 1)
        ws = torch.empty(P.multislice_workspace(g, 8, 8), dtype=torch.uint8, device="cuda")
        P.multislice_outputs(g, r.E0, r.alpha_max, V, xy, batch=8, ws=ws)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        P.multislice_outputs(g, r.E0, r.alpha_max, V, xy, batch=8, ws=ws)
        torch.cuda.synchronize()
        per_probe = (time.perf_counter() - t1) / 8
        ms_time += per_probe * sum(x.n_probes for x in rs)
    res = {"metric": "serving: aggregate probe positions/s, p50/p99 latency (mixed PRISM requests)",
           "value": summ["probes_per_s"], "unit": "probe positions/s", "n_gpus": 1,
           "p50_latency_s": summ["p50_latency_s"], "p99_latency_s": summ["p99_latency_s"],
           "latency_by_grid": summ["latency_by_grid"], "stream_seed": seed,
           "requests": summ["requests"], "rejected": summ["rejected"], "probes": summ["probes"],
           "wall_s": wall, "arrival_rate_per_s": rate, "offered_load": ld0,
           "capacity_requests_per_s": capacity,
           "saturation_probes_per_s": sat_summary["probes_per_s"] if sat_summary else None,
           "load_sweep": {str(k): {"probes_per_s": v[2]["probes_per_s"], "p50_latency_s": v[2]["p50_latency_s"],
                                   "p99_latency_s": v[2]["p99_latency_s"], "wall_s": v[1],
                                   "latency_by_grid": v[2]["latency_by_grid"]}
                          for k, v in sweep.items()},
           "hbm_budget_GB": cap / 1e9, "peak_reserved_GB": summ["peak_hbm_reserved"] / 1e9,
           "precision": args.precision, "grids": list(grids),
           "beam_chunked_requests": sum(1 for r in sched.done if r.info.get("beam_chunk")),
           "largest_request_beams": max((r.info.get("n_beams", 0) for r in sched.done), default=0),
           "alone_vs_mix_max_abs_diff": max(diffs) if diffs else None,
           "sequential_multislice_s_extrapolated": ms_time,
           "speedup_vs_sequential_multislice": ms_time / wall if wall > 0 else None,
           "data": "synthetic"}
    return res


def run_serving(args):
    """The serving benchmark alone (`--serve`)."""
    grids = tuple(int(x) for x in args.grids.split(","))
    loads = [float(x) for x in args.loads.split(",")]
    print(json.dumps(serving_report(args, args.requests, grids, loads, capacity=args.capacity,
                                    saturation_only=args.saturation_only)), flush=True)


def multislice_leg(args):
    """Plain multislice on the 1024^2 nanoparticle cell: 64 x 64 probes, 50
    slices, probes propagated 1024 at a time (the comparison method)."""
    import numpy as np
    import torch

    import paper_1706_08563_amd as P
    import workloads as W

    w = W.WORKLOADS["multislice_np_1024"]
    pos, sp = W.atoms_for(w)
    g = P.prism_grid_init(w.cell, w.dz, w.n)
    V = P.prism_project_potential(pos, sp, w.species, g)
    xy = W.scan_positions(w.cell, *w.scan)
    batch = 1024
    n_bins = P.prism_detector_default_bins(g, w.E0)[0]
    ws = torch.empty(P.multislice_workspace(g, batch, len(xy)), dtype=torch.uint8, device="cuda")
    out = torch.empty((len(xy), n_bins), dtype=torch.float32, device="cuda")
    P.multislice_outputs(g, w.E0, w.alpha_max, V, xy[:batch], batch=batch, ws=ws, out=out[:batch])
    torch.cuda.synchronize()
    P.prism_timing_reset()
    P.prism_timing_enable(True)
    t0 = time.perf_counter()
    P.multislice_outputs(g, w.E0, w.alpha_max, V, xy, batch=batch, ws=ws, out=out)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    P.prism_timing_enable(False)
    kt = {k: P.prism_timing_read(c) for k, c in P.TIMING_CLASSES.items()}
    N2 = float(w.n) ** 2
    a_ms = kt["pass_a"][0] / max(kt["pass_a"][1], 1)
    b_ms = kt["pass_b"][0] / max(kt["pass_b"][1], 1)
    return {"workload": w.name, "probes": len(xy), "slices": g.n_slices, "grid": w.n, "batch": batch,
            "seconds": dt, "probes_per_s": len(xy) / dt,
            "pass_a_avg_ms": a_ms, "pass_b_avg_ms": b_ms,
            "pass_a_GB_per_s": (batch * 8 * N2 + 8 * N2) / (a_ms * 1e-3) / 1e9,
            "pass_b_GB_per_s": batch * 8 * N2 / (b_ms * 1e-3) / 1e9}, out


def precision_study(args):
    """The contraction three ways (split-BF16, BF16, FP32) on the 2048^2, f = 8
    workload (200 x 200 x 100 A nanoparticle cell, 1245 beams, 50 slices,
    128^2 windows, 256 x 256 scan): the S-matrix is built on the GPU from the
    cell; device time per variant over the full scan, and each variant's error
    on the 16 x 16 probe subset against the FP64 fixture of the same cell
    (every beam through every slice in FP64, written by the oracle)."""
    import numpy as np
    import torch

    import paper_1706_08563_amd as P
    import workloads as W

    w = W.WORKLOADS["prism_f8_np_2048"]
    fx = load_fixture(w.name)
    pos, sp = W.atoms_for(w)
    g = P.prism_grid_init(w.cell, w.dz, w.n)
    V = P.prism_project_potential(pos, sp, w.species, g)
    d = P.prism_smatrix_plan(g, w.E0, w.alpha_max, w.f)
    log(f"precision study: building the {w.name} S-matrix ({d.n_beams} beams x {g.n_slices} slices)")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    S = P.prism_build_smatrix(d, V)
    torch.cuda.synchronize()
    build_s = time.perf_counter() - t0
    del V
    xy = W.scan_positions(w.cell, *w.scan)
    sub = W.scan_positions(w.cell, *w.scan, sub=w.scan[0] // 16)
    plan = P.prism_probe_plan_upload(d, xy)
    plan_s = P.prism_probe_plan_upload(d, sub)
    ws = torch.empty(plan.plan.ws_bytes, dtype=torch.uint8, device="cuda")
    res = {"workload": w.name, "probes_timed": len(xy), "probes_checked": len(sub), "beams": d.n_beams,
           "build_s": build_s, "smatrix": "built on the GPU from the cell",
           "fixture": None if fx is None else f"tests/golden/{w.name}_fp64_subset.npz"}
    if fx is not None:
        assert np.array_equal(sub, fx["probe_xy"]), "fixture positions differ from the scan subset"
    for name, prec in (("bf16x3", P.PRISM_SPLIT_BF16X3), ("bf16", P.PRISM_BF16), ("fp32", P.PRISM_FP32)):
        out = P.prism_probe_outputs(d, S, plan, prec, ws=ws)
        torch.cuda.synchronize()
        P.prism_timing_reset()
        P.prism_timing_enable(True)
        t0 = time.perf_counter()
        P.prism_probe_outputs(d, S, plan, prec, ws=ws, out=out)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        P.prism_timing_enable(False)
        cms, _ = P.prism_timing_read(P.TIMING_CLASSES["contract"])
        flops = 8.0 * d.n_beams * d.m_win ** 2 * len(xy)
        res[name] = {"synthesis_s": dt, "probes_per_s": len(xy) / dt, "contract_ms": cms,
                     "contract_useful_TFLOP_per_s": flops / (cms * 1e-3) / 1e12}
        if fx is not None:
            got = P.prism_probe_outputs(d, S, plan_s, prec).cpu().numpy()
            res[name]["vs_fp64"] = detector_errors(got, fx["prism"])
        log(f"  {name}: {dt * 1e3:.1f} ms, contract {cms:.1f} ms, {res[name].get('vs_fp64')}")
        del out
    del S, ws
    torch.cuda.empty_cache()
    return res


def streaming_study(args):
    """The paper's single-transfer vs streaming comparison ("Data
    Streaming/Single-Transfer Benchmark") on the default workload: the whole
    simulation (S-matrix build and synthesis of every probe) with the
    potential and S-matrix resident, then with both in page-locked host memory
    under a device budget of `budget_fraction` of the single-transfer
    footprint; wall time and peak device memory of each, and the difference
    of their outputs."""
    import numpy as np
    import torch

    import paper_1706_08563_amd as P
    from paper_1706_08563_amd import memory as MM
    import workloads as W

    prec = {"fp32": P.PRISM_FP32, "bf16x3": P.PRISM_SPLIT_BF16X3, "bf16": P.PRISM_BF16}[args.precision]
    w = W.WORKLOADS[args.workload]
    pos, sp = W.atoms_for(w)
    g = P.prism_grid_init(w.cell, w.dz, w.n)
    V = P.prism_project_potential(pos, sp, w.species, g)
    Vh = V.cpu().pin_memory()
    xy = W.scan_positions(w.cell, *w.scan)
    single = MM.plan_memory(g, w.E0, w.alpha_max, w.f, xy, 1 << 60)
    budget = int(args.budget_fraction * single.single_bytes)
    mp = MM.plan_memory(g, w.E0, w.alpha_max, w.f, xy, budget)
    log(f"streaming study: single transfer {single.single_bytes / 1e9:.2f} GB; budget {budget / 1e9:.2f} GB -> "
        f"{mp.mode}, beam batch {mp.desc.beam_batch}, beam chunk {mp.beam_chunk}, probe chunk {mp.probe_chunk}")

    def timed(fn):
        torch.cuda.synchronize()
        base = torch.cuda.memory_allocated()
        torch.cuda.reset_peak_memory_stats()
        t0 = time.perf_counter()
        out = fn()
        torch.cuda.synchronize()
        return out, time.perf_counter() - t0, torch.cuda.max_memory_allocated() - base

    MM.run_prism(single, V, xy, prec)            # warm-up (code objects, allocator)
    d_single, t_single, m_single = timed(lambda: MM.run_prism(single, V, xy, prec))
    del V
    torch.cuda.empty_cache()
    d_stream, t_stream, m_stream = timed(lambda: MM.run_prism(mp, Vh, xy, prec))
    a, b = d_single.cpu().numpy().astype(np.float64), d_stream.cpu().numpy().astype(np.float64)
    res = {"streaming_study": {
        "workload": w.name, "precision": args.precision, "probes": len(xy), "beams": single.desc.n_beams,
        "single_transfer": {"seconds": t_single, "peak_device_GB": m_single / 1e9,
                            "planned_GB": single.single_bytes / 1e9},
        "streaming": {"seconds": t_stream, "peak_device_GB": m_stream / 1e9, "planned_GB": mp.peak_bytes / 1e9,
                      "budget_GB": budget / 1e9, "beam_batch": mp.desc.beam_batch, "beam_chunk": mp.beam_chunk,
                      "probe_chunk": mp.probe_chunk},
        "time_ratio_streaming_over_single": t_stream / t_single,
        "peak_memory_ratio_single_over_streaming": m_single / max(m_stream, 1),
        "rel_diff_outputs": float(np.linalg.norm(a - b) / np.linalg.norm(a))}}
    print(json.dumps(res), flush=True)


def pmc_driver(args):
    """One launch of every kernel of the default workload at its real per-launch
    size (the build cut to 4 slices, on one stream as in the per-kernel timing:
    the first-slice gather, three interior row passes and four column passes
    over all beams),
    then a plain 256 MiB copy whose byte count calibrates the FETCH_SIZE /
    WRITE_SIZE counters."""
    import dataclasses

    import torch

    import paper_1706_08563_amd as P
    import workloads as W

    prec = {"fp32": P.PRISM_FP32, "bf16x3": P.PRISM_SPLIT_BF16X3, "bf16": P.PRISM_BF16}[args.precision]
    w = W.WORKLOADS[args.workload]
    w4 = dataclasses.replace(w, cell=(w.cell[0], w.cell[1], 4 * w.dz))
    pos, sp = W.atoms_for(w4)
    g = P.prism_grid_init(w4.cell, w4.dz, w4.n)
    V = P.prism_project_potential(pos, sp, w4.species, g)
    d = P.prism_smatrix_plan(g, w4.E0, w4.alpha_max, w4.f)
    P.prism_set_build_streams(1)
    S = P.prism_build_smatrix(d, V)
    plan = P.prism_probe_plan_upload(d, W.scan_positions(w4.cell, *w4.scan))
    P.prism_probe_outputs(d, S, plan, prec)
    x = torch.ones(64 * 1024 * 1024, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    y.copy_(x)
    torch.cuda.synchronize()
    log("pmc driver done")


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this implementation runs on a single GPU; --gpus must be 1",
                          "detail": "multi-GPU sharding is described in the design notes, not implemented"}))
        sys.exit(2)
    if args.serve:
        run_serving(args)
        return
    if args.precision_study:
        print(json.dumps({"precision_study": precision_study(args)}), flush=True)
        return
    if args.pmc_driver:
        pmc_driver(args)
        return
    if args.streaming_study:
        streaming_study(args)
        return

    import numpy as np
    import torch

    import paper_1706_08563_amd as P
    import workloads as W

    assert torch.cuda.is_available(), "bench needs a GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    prec = {"fp32": P.PRISM_FP32, "bf16x3": P.PRISM_SPLIT_BF16X3, "bf16": P.PRISM_BF16}[args.precision]

    w = W.WORKLOADS[args.workload]
    log(f"workload {w.name}: setup")
    pos, sp = W.atoms_for(w)
    g = P.prism_grid_init(w.cell, w.dz, w.n)
    V = P.prism_project_potential(pos, sp, w.species, g)
    d = P.prism_smatrix_plan(g, w.E0, w.alpha_max, w.f)
    xy = W.scan_positions(w.cell, *w.scan)
    t0 = time.perf_counter()
    plan = P.prism_probe_plan_upload(d, xy)
    plan_s = time.perf_counter() - t0
    B, n, nsl, M = d.n_beams, w.n, g.n_slices, d.m_win
    n_probes = len(xy)
    ws_build = torch.empty(d.build_ws_bytes, dtype=torch.uint8, device=dev)
    ws_probe = torch.empty(plan.plan.ws_bytes, dtype=torch.uint8, device=dev)
    S = torch.empty((B, d.ns, d.ns), dtype=torch.complex64, device=dev)
    out = torch.empty((n_probes, plan.plan.n_bins), dtype=torch.float32, device=dev)
    stream = torch.cuda.current_stream()

    def build():
        P.prism_build_smatrix(d, V, ws=ws_build, S=S)

    def synth():
        P.prism_probe_outputs(d, S, plan, prec, ws=ws_probe, out=out)

    log(f"warmup {args.warmup} (beams {B}, slices {nsl}, probes {n_probes}, window {M})")
    for _ in range(args.warmup):
        build()
        synth()
    torch.cuda.synchronize()

    def run_steps(k, kernel_timing):
        """k whole steps; returns (wall s, step ms, build ms, synthesis ms)."""
        if kernel_timing:
            P.prism_timing_reset()
            P.prism_timing_enable(True)
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True),
               torch.cuda.Event(enable_timing=True)) for _ in range(k)]
        torch.cuda.synchronize()
        t_wall = time.perf_counter()
        for i in range(k):
            ev[i][0].record(stream)
            build()
            ev[i][1].record(stream)
            synth()
            ev[i][2].record(stream)
        torch.cuda.synchronize()
        wall_s = time.perf_counter() - t_wall
        if kernel_timing:
            P.prism_timing_enable(False)
        return (wall_s, [a.elapsed_time(c) for a, b, c in ev], [a.elapsed_time(b) for a, b, c in ev],
                [b.elapsed_time(c) for a, b, c in ev])

    # headline: the library's default build streams (four overlapping beam
    # parts up to 1024^2, one stream above)
    log(f"timed {args.steps} steps")
    P.prism_set_build_streams(0)
    wall, step_ms, build_ms, synth_ms = run_steps(args.steps, False)
    log(f"steps done: wall {wall:.3f} s; step ms {step_ms}")
    # per-kernel times (roofline): one stream, so that launches do not overlap
    k_steps = max(1, min(args.steps, 2))
    log(f"kernel timing: {k_steps} one-stream steps")
    P.prism_set_build_streams(1)
    _, _, build_ms_1, _ = run_steps(k_steps, True)
    P.prism_set_build_streams(0)
    kt = {name: P.prism_timing_read(cls) for name, cls in P.TIMING_CLASSES.items()}
    # end to end with the probe planning in every step: the host plans the
    # scan and uploads its tables on a side stream while the GPU builds the
    # S-matrix; the synthesis then uses that step's plan
    k_plan = max(1, min(args.steps, 3))
    side = torch.cuda.Stream()
    plans = []
    log(f"end-to-end timing with planning: {k_plan} steps")
    torch.cuda.synchronize()
    t_wall = time.perf_counter()
    for _ in range(k_plan):
        build()
        with torch.cuda.stream(side):
            plans.append(P.prism_probe_plan_upload(d, xy))
        stream.wait_stream(side)
        P.prism_probe_outputs(d, S, plans[-1], prec, ws=ws_probe, out=out)
    torch.cuda.synchronize()
    planned_ms = (time.perf_counter() - t_wall) * 1e3 / k_plan
    del plans

    ms_per_step = wall * 1e3 / args.steps
    N2 = float(n) * n
    # algorithmic HBM bytes per launch of the propagation passes (band-limited
    # wave: 4 N^2 B per beam read and written, plus the slice's transmission;
    # the row pass runs on slices 2..S, the first slice being a gather from
    # the row spectrum, timed as "first")
    a_bytes = B * 8 * N2 + 8 * N2
    b_bytes = (B * 8 * N2 * (nsl - 1) + B * 6 * N2) / nsl
    c_flops = 8.0 * B * M * M * n_probes          # useful complex MACs x 8
    kernels = {}
    for name, (tot, cnt) in kt.items():
        if cnt:
            kernels[name] = {"ms_total": tot / k_steps, "launches_per_step": cnt // k_steps,
                             "avg_ms": tot / cnt}
    kernels["pass_a"]["GB_per_s"] = a_bytes / (kernels["pass_a"]["avg_ms"] * 1e-3) / 1e9
    kernels["pass_b"]["GB_per_s"] = b_bytes / (kernels["pass_b"]["avg_ms"] * 1e-3) / 1e9
    kernels["contract"]["TFLOP_per_s"] = c_flops / (kernels["contract"]["avg_ms"] * 1e-3) / 1e12
    if prec != P.PRISM_FP32:
        # MFMA work: three BF16 products per complex product in split mode, one in plain BF16
        mw = kernels["contract"]["TFLOP_per_s"] * (3 if prec == P.PRISM_SPLIT_BF16X3 else 1)
        kernels["contract"]["mfma_work_TFLOP_per_s"] = mw
        kernels["contract"]["mfma_frac_of_bf16_peak"] = mw / PEAK_BF16_TFLOPS
    kernels["pass_a"]["TFLOP_per_s"] = pass_flops(n, B, n) / (kernels["pass_a"]["avg_ms"] * 1e-3) / 1e12
    kernels["pass_b"]["TFLOP_per_s"] = pass_flops(n, B, n // 2) / (kernels["pass_b"]["avg_ms"] * 1e-3) / 1e12
    dom = max(["pass_a", "pass_b", "contract"], key=lambda k: kernels[k]["ms_total"])
    if dom == "contract":
        peak = PEAK_FP32_TFLOPS if prec == P.PRISM_FP32 else PEAK_BF16_TFLOPS
        ach = kernels["contract"]["TFLOP_per_s"]
        roof = {"kernel": "contract", "bound": "alu" if prec == P.PRISM_FP32 else "mfma", "achieved": ach,
                "peak": peak, "unit": "TFLOP/s", "frac": ach / peak, "traffic": None}
    else:
        # the propagation passes are bounded either by HBM or by FP32 VALU
        # issue (the library is built without packed FP32, so one FMA per
        # lane per clock is the ceiling); report the nearer bound
        k = kernels[dom]
        hbm_frac = k["GB_per_s"] / PEAK_HBM_GBS
        alu_frac = k["TFLOP_per_s"] / PEAK_FP32_UNPACKED_TFLOPS
        traffic = recorded_traffic(dom, w.name)
        if alu_frac > hbm_frac:
            roof = {"kernel": dom, "bound": "alu", "achieved": k["TFLOP_per_s"], "peak": PEAK_FP32_UNPACKED_TFLOPS,
                    "unit": "TFLOP/s", "frac": alu_frac, "traffic": traffic, "traffic_unit": "HBM bytes per launch",
                    "algorithmic_bytes_per_launch": a_bytes if dom == "pass_a" else b_bytes,
                    "peak_packed_fp32": PEAK_FP32_TFLOPS, "hbm_GB_per_s": k["GB_per_s"], "hbm_frac": hbm_frac}
        else:
            roof = {"kernel": dom, "bound": "hbm", "achieved": k["GB_per_s"], "peak": PEAK_HBM_GBS, "unit": "GB/s",
                    "frac": hbm_frac, "traffic": traffic, "traffic_unit": "HBM bytes per launch",
                    "algorithmic_bytes_per_launch": a_bytes if dom == "pass_a" else b_bytes, "alu_TFLOP_per_s": k["TFLOP_per_s"], "alu_frac": alu_frac}

    res = {
        "metric": METRIC,
        "value": n_probes / (ms_per_step * 1e-3),
        "unit": "probe positions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if prec == P.PRISM_FP32 else ("bf16x3/f32" if prec == P.PRISM_SPLIT_BF16X3 else "bf16/f32"),
        "data": "synthetic",
        "config": {"workload": w.name, "grid": n, "cell_A": list(w.cell), "slices": nsl, "E0_eV": w.E0,
                   "alpha_mrad": w.alpha_max * 1e3, "f": w.f, "beams": B, "probes": n_probes, "window": M,
                   "n_bins": plan.plan.n_bins, "precision": args.precision},
        "beams_per_s": B / (float(np.median(build_ms)) * 1e-3),
        "probes_per_s_synthesis": n_probes / (float(np.median(synth_ms)) * 1e-3),
        "p50_ms": float(np.percentile(step_ms, 50)),
        "p99_ms": float(np.percentile(step_ms, 99)),
        "build_ms": float(np.median(build_ms)),
        "build_ms_one_stream": float(np.median(build_ms_1)),
        "build_streams": 4 if n <= 1024 else 1,     # the library's default for this grid
        "synthesis_ms": float(np.median(synth_ms)),
        "probe_plan_host_s": plan_s,
        # whole steps that also plan the scan (window corners, work tiles,
        # bin tables) on the host and upload the plan, beside the build
        "probes_per_s_with_planning": n_probes / (planned_ms * 1e-3),
        "ms_per_step_with_planning": planned_ms,
        "kernels": kernels,
        "roofline": roof,
        "hbm_copy_GB_per_s": copy_bandwidth(),
        "device": device_info(),
    }
    res["multislice"], ms_out = multislice_leg(args)
    if w.name == "prism_f4_np_1024" and res["multislice"] and res["multislice"].get("probes_per_s"):
        res["speedup"] = {
            # both on this GPU; the multislice leg simulates the same cell
            "prism_vs_multislice_same_gpu": res["value"] / res["multislice"]["probes_per_s"],
            # the paper's figures on its own hardware (abstract; application
            # to a large oxide cell): context, not a target
            "paper_context": {
                "prism_vs_traditional_multislice": "up to ~1000x",
                "gpu_multislice_vs_traditional_multislice": "~15x",
                "prism_f4_vs_gpu_multislice": "2.7x (1024^2, 720^2 probes, oxide cell)",
                "hardware": "one machine: 4x Tesla K20 GPUs with multicore Xeon CPUs",
            },
        }
    if w.name == "prism_f4_np_1024":
        log("accuracy on the 16 x 16 probe subset against the FP64 fixture")
        res["accuracy"] = accuracy_report(w, d, S, out, ms_out, args.precision)
        acc = res["accuracy"].get(f"timed_{args.precision}_vs_fp64")
        if acc:
            res["rel_err_vs_fp64"] = acc["rel_all"]
            res["rel_adf_vs_fp64"] = acc["rel_adf"]
            res["per_bin_max_vs_fp64"] = acc["per_bin_max"]
    del ms_out
    if w.name == "prism_f4_np_1024" and not args.no_precision_study:
        del S, ws_build, ws_probe, out, V
        torch.cuda.empty_cache()
        res["precision_study"] = precision_study(args)
    if not args.no_serving:
        # bounded serving leg: 16 requests of the serving distribution (all
        # four grid sizes; the stream seeded 40 holds one 2048^2 f = 2
        # request of 19973 beams among small ones), offered load 0.8
        log("serving leg (16 requests, load 0.8)")
        torch.cuda.empty_cache()
        res["serving"] = serving_report(args, 16, (256, 512, 1024, 2048), [0.8], seed=40, quiet=True)
    if not args.no_cpu_baseline:
        log("cpu baseline (FP64 oracle, bounded sample)")
        res["cpu_baseline"] = cpu_baseline(w, d, B, n_probes, args)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
