"""Throughput benchmark of the NUFFT hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]

A step is one pass of the whole hot path over the workload's points: set the
points (FP64 fold + bin sort + subproblems) and execute each transform type
(spread / FFT / deconvolve for type 1; amplify / FFT / interpolate for type 2).
Where the workload runs both types on one point set, one type 1 plan sorts the
points once and runs type 2 as its adjoint (opposite sign) on the same sorted
points; the same step with one plan per type, each sorting for itself, is timed
too and reported under ``separate_plans``.  Plans (kernel parameters, the FP64
quadrature of the kernel's Fourier transform, rocFFT plans) are made once
before timing, as the paper times only calls after planning (Sec. 6).  All
inputs are resident in HBM before the timed region.  ``value`` = NU points
processed per second (M * ntransf per transform type, summed) over the timed
steps.

One JSON line is printed.  Besides the contract fields it carries
* ``roofline``: the dominant kernel's algorithmic work per launch divided by
  its mean duration, timed with HIP events on the kernel's own stream inside
  the timed region (the library's debug stage events);
* ``cpu_baseline``: the FP64 oracle (direct sums) timed on a bounded sample of
  the same workload on the host cores, scaled to the metric's unit;
* ``parity``: the GPU output's relative l2 error on that oracle sample;
* ``sort_ablation`` (both types on one point set): execute with the points
  left unsorted against the bin-sorted execute, alone and with the sort.
``stages`` holds the library's per-stage times; where the FFT runs as column
FFTs (3D single precision on column-FFT lengths, as the headline) it carries
the deconvolution / amplification, so ``fft_ms`` includes them and
``deconv_ms`` / ``amplify_ms`` are only the gaps between the stages.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from paper_1808_06736_amd import inputs as I  # noqa: E402

METRIC = "NU points/sec, 3D type1/2 at ε=1e-6; served p50/p99 latency vs plain"
HBM_PEAK_GBS = 8000.0
FP32_PEAK_TFLOPS = 157.3
FP64_PEAK_TFLOPS = 78.6


def progress(msg):
    """A line on stderr as each part of the run completes (the JSON result is
    the only line on stdout)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="3d_clustered", choices=sorted(I.WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true",
                    help="skip the oracle timing (profiling runs)")
    ap.add_argument("--cpu-sample", type=int, default=0,
                    help="modes per dim (type 1) in the oracle sample; 0 = default")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (5 times), the "
                         "reference for scaling HBM byte counters")
    ap.add_argument("--serve-requests", type=int, default=1000,
                    help="requests in the serving measurement (0: skip it)")
    ap.add_argument("--serve-load", type=float, nargs="+", default=[0.5, 0.8, 0.95],
                    help="offered loads as fractions of the plain serial throughput")
    ap.add_argument("--serve-slots", type=int, default=4)
    ap.add_argument("--no-sort-ablation", action="store_true",
                    help="skip the unsorted-points comparison (Sec. 5.1)")
    ap.add_argument("--traffic", default="",
                    help="JSON with measured HBM bytes per launch of the dominant "
                         "kernel ({\"kernel\": ..., \"bytes\": ...}) for roofline.traffic")
    return ap.parse_args()


def algorithmic_work(w, dim, M, ntr, nf, prec, kind):
    """Algorithmic bytes and flops of one spread or interp launch.

    Per point: d sorted coordinates (4 B fixed point or 8 B) + one complex
    strength per transform; per fine-grid cell: one complex write (spread) or
    nothing counted (interp reads only the cells the points touch, which the
    per-point figure already bounds).  Flops: 4 w^d per point per transform (a
    real weight times a complex value, accumulated) + the separable weights
    (w^(d-1) + ... products, ignored).
    """
    cb = 8 if prec == "f32" else 16
    coord_b = 4 if prec == "f32" else 8
    per_point = dim * coord_b + ntr * cb
    grid = math.prod(nf) * ntr * cb if kind == "spread" else 0
    bytes_ = M * per_point + grid
    flops = 4.0 * (w ** dim) * M * ntr
    return bytes_, flops


def measured_traffic(path, kernel, workload):
    """HBM bytes per launch measured with rocprofv3 (FETCH_SIZE, WRITE_SIZE scaled
    by a plain copy), from profiles/traffic_<workload>.json; None when missing or
    when the kernel's source changed since the counters were taken."""
    import hashlib
    path = path or os.path.join(ROOT, "profiles", f"traffic_{workload}.json")
    if not os.path.exists(path):
        return None
    tr = json.load(open(path))
    if tr.get("workload") != workload or kernel not in tr.get("kernels", {}):
        return None
    src = os.path.join(ROOT, tr.get("source_file", ""))
    if not os.path.isfile(src):
        return None
    if hashlib.sha256(open(src, "rb").read()).hexdigest()[:16] != tr.get("source_sha256_16"):
        return None
    return tr["kernels"][kernel]


def copy_calibration(mib):
    """A plain copy of a known size: each launch reads and writes mib MiB."""
    import torch
    n = mib * (1 << 20) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(5):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_mib": mib, "bytes_read": n * 4, "bytes_written": n * 4}))


def main():
    args = parse()
    if args.copy_calibration:
        copy_calibration(args.copy_calibration)
        return
    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU; --gpus {args.gpus} is not supported "
              "(this build has no multi-GPU path)", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_1808_06736_amd import binding as B

    wl = I.WORKLOADS[args.workload]
    torch.cuda.set_device(0)
    if wl.types == (3,):
        return bench_type3(args, wl)
    dim, M, ntr = wl.dim, wl.M, wl.ntransf
    N = wl.N[:dim]
    prec = wl.prec
    cdt = torch.complex64 if prec == "f32" else torch.complex128

    coords_np = wl.coords()
    coords = [torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in coords_np]
    c_np = wl.strengths()
    f_np = wl.coefficients()
    c_in = torch.from_numpy(c_np).cuda()
    f_in = torch.from_numpy(f_np).cuda()

    tuned = {}
    if wl.extra.get("autotune"):
        # bin / subproblem / fusion options picked by timing on these points,
        # before the timed region (like planning)
        from paper_1808_06736_amd import autotune
        for t in wl.types:
            tuned[t], _ = autotune.tune(t, N, wl.eps, coords, c_in if t == 1 else f_in,
                                        dtype=cdt, ntransf=ntr)
    # Both types on one point set (the 2D and 3D workloads): one plan of type 1
    # sorts the points once and runs type 1 and, by its adjoint, type 2 (the
    # opposite sign, isign -1, on the same sorted points).  Otherwise one plan
    # per type.
    shared = len(wl.types) == 2 and ntr == 1
    plans = {}
    outs = {}
    for t in wl.types:
        outs[t] = torch.empty_like(f_in) if t == 1 else torch.empty_like(c_in)
    for t in ([1] if shared else wl.types):
        plans[t] = B.Plan(t, N, wl.eps, dtype=cdt, ntransf=ntr, debug=1, **tuned.get(t, {}))
        plans[t].setpts(*coords)
    torch.cuda.synchronize()

    # Stage times come from the library's HIP events around each stage, recorded
    # on the plan's stream during the timed loop and read after it (no host
    # synchronisation inside the loop).
    def stage_rec(t, st_set, s):
        return (t, st_set, s.t_spread_or_interp, s.t_fft, s.t_deconv_or_amplify, s.t_execute)

    def step_shared():
        p = plans[1]
        p.setpts(*coords)
        p.execute(c_in, outs[1])
        p.execute_adjoint(outs[2], f_in)

    def step_separate(pl):
        for t in wl.types:
            p = pl[t]
            p.setpts(*coords)
            if t == 1:
                p.execute(c_in, outs[1])
            else:
                p.execute(outs[2], f_in)

    def history(p, calls_per_step, types_of_execs):
        """Per-step stage records from the plan's last steps: entries come as
        setpts then the step's executes."""
        h = p.stats_history(256)
        n = min(args.steps, len(h) // calls_per_step)
        h = h[len(h) - n * calls_per_step:]
        rec = []
        for k in range(n):
            grp = h[k * calls_per_step:(k + 1) * calls_per_step]
            for i, t in enumerate(types_of_execs):
                rec.append(stage_rec(t, grp[0].t_setpts if i == 0 else 0.0, grp[1 + i]))
        return rec

    def timed(step):
        for _ in range(args.warmup):
            step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            step()
        torch.cuda.synchronize()
        return time.perf_counter() - t0

    if shared:
        elapsed = timed(step_shared)
        rec = history(plans[1], 3, [1, 2])
    else:
        elapsed = timed(lambda: step_separate(plans))
        rec = [r for t in wl.types for r in history(plans[t], 2, [t])]
    ms_per_step = 1e3 * elapsed / args.steps
    pts_per_step = M * ntr * len(wl.types)
    value = pts_per_step / (elapsed / args.steps)

    # per-type stage means (ms)
    stages = {}
    for t in wl.types:
        r = np.array([x[1:] for x in rec if x[0] == t])
        stages[f"type{t}"] = {
            "setpts_ms": float(r[:, 0].mean()),
            ("spread_ms" if t == 1 else "interp_ms"): float(r[:, 1].mean()),
            "fft_ms": float(r[:, 2].mean()),
            ("deconv_ms" if t == 1 else "amplify_ms"): float(r[:, 3].mean()),
            "execute_ms": float(r[:, 4].mean()),
            "exec_pts_per_s": M * ntr / (r[:, 4].mean() * 1e-3),
        }

    separate = None
    if shared:
        # the same step with one plan per type, each sorting the points itself
        sep_plans = {t: B.Plan(t, N, wl.eps, dtype=cdt, ntransf=ntr, debug=1) for t in wl.types}
        for p in sep_plans.values():
            p.setpts(*coords)
        sep_elapsed = timed(lambda: step_separate(sep_plans))
        sep_rec = [r for t in wl.types for r in history(sep_plans[t], 2, [t])]
        separate = {"ms_per_step": 1e3 * sep_elapsed / args.steps,
                    "value": pts_per_step / (sep_elapsed / args.steps),
                    "setpts_ms": {f"type{t}": float(np.mean([x[1] for x in sep_rec if x[0] == t]))
                                  for t in wl.types},
                    "step": "per type: its own plan, setpts (fold+sort+subproblems) + execute"}
        for p in sep_plans.values():
            p.close()
        plans[2] = plans[1]

    # dominant kernel: the slower of spread / interp
    info = {t: plans[t].info() for t in wl.types}
    kern_t = {t: stages[f"type{t}"]["spread_ms" if t == 1 else "interp_ms"] for t in wl.types}
    tdom = max(kern_t, key=kern_t.get)
    inf = info[tdom]
    nf = [int(inf.nf[m]) for m in range(dim)]
    kind = "spread" if tdom == 1 else "interp"
    # per launch: a batched execute runs ceil(ntransf / chunk) launches of the
    # dominant kernel (chunk vectors each); the stage time covers them all
    chunk = max(1, int(inf.ntransf_chunk))
    nlaunch = -(-ntr // chunk)
    bytes_, flops = algorithmic_work(inf.w, dim, M, min(chunk, ntr), nf, prec, kind)
    dur_s = kern_t[tdom] * 1e-3 / nlaunch
    peak_alu = FP32_PEAK_TFLOPS if prec == "f32" else FP64_PEAK_TFLOPS
    intensity = flops / bytes_
    ridge = peak_alu * 1e12 / (HBM_PEAK_GBS * 1e9)
    method = inf.spread_method if tdom == 1 else inf.interp_method
    kname = {(1, 3): "spread_mfma_kernel", (2, 3): "interp_mfma_kernel",
             (1, 1): "spread_lds_kernel", (2, 1): "interp_lds_kernel",
             (1, 2): "spread_gm_kernel", (2, 2): "interp_gm_kernel"}[(tdom, method)]
    if method == 3 and dim == 2:
        kname = kname.replace("_mfma", "2d_mfma")
    if intensity >= ridge:
        # arithmetic-bound: on the matrix cores (method 3) against the dense
        # MFMA peak of the precision, otherwise against the vector ALU peak
        roof = {"bound": "mfma" if method == 3 else "alu",
                "achieved": flops / dur_s / 1e12, "peak": peak_alu, "unit": "TFLOP/s"}
    else:
        roof = {"bound": "hbm", "achieved": bytes_ / dur_s / 1e9, "peak": HBM_PEAK_GBS,
                "unit": "GB/s"}
    roof["frac"] = roof["achieved"] / roof["peak"]
    roof["traffic"] = None
    tname = "float" if prec == "f32" else "double"
    roof["kernel"] = (f"{kname}<{inf.w}>" if method == 3 and dim == 3 else
                      f"{kname}<{inf.w},{tname}>" if method == 3 else
                      f"{kname}<{dim},{inf.w},{tname}>")
    roof["traffic"] = measured_traffic(args.traffic, roof["kernel"], wl.name)
    roof["algorithmic_bytes"] = bytes_
    roof["algorithmic_flops"] = flops
    roof["mean_launch_ms"] = kern_t[tdom] / nlaunch
    roof["launches_per_execute"] = nlaunch
    roof["hbm_frac"] = bytes_ / dur_s / 1e9 / HBM_PEAK_GBS

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "NU pts/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": prec,
        "data": "synthetic",
        "config": {"workload": wl.name, "dim": dim, "N": list(N), "M": M, "ntransf": ntr,
                   "eps": wl.eps, "points": wl.points, "types": list(wl.types),
                   "w": int(inf.w), "nf": nf,
                   "step": ("setpts once (fold+sort+subproblems) on a type 1 plan, execute "
                            "type 1, execute its adjoint (type 2, isign -1) on the same sorted "
                            "points" if shared else
                            "per type: setpts (fold+sort+subproblems) + execute")},
        "stages": stages,
        "roofline": roof,
    }
    if separate is not None:
        out["separate_plans"] = separate

    if tuned:
        out["config"]["autotuned"] = {f"type{t}": {k: (list(v) if isinstance(v, tuple) else v)
                                                   for k, v in o.items()}
                                      for t, o in tuned.items()}
    if ntr > 1:
        out["batched_vs_plain"] = batched_vs_plain(wl, coords, c_in, f_in, plans, outs, cdt)
    if shared and not args.no_sort_ablation:
        out["sort_ablation"] = sort_ablation(wl, N, coords, c_in, f_in, outs, cdt, stages)
        progress("sort ablation done")

    progress(f"timed steps done: {ms_per_step:.3f} ms per step")
    if wl.name == "3d_clustered":
        out["batched_8_vectors"] = batched_headline(wl, coords, cdt)
        progress("batched 8-vector comparison done")

    if args.serve_requests > 0 and args.workload == "3d_clustered":
        out["serving"] = serve_bench(args.serve_requests, args.serve_load, args.serve_slots)
        progress("serving measurement done")

    if not args.no_cpu_baseline:
        out["cpu_baseline"], out["parity"] = cpu_baseline(wl, coords_np, c_np, f_np, plans,
                                                          outs, args.cpu_sample)
    if wl.name == "3d_clustered":
        out["paper_cpu_context"] = PAPER_CPU_CONTEXT
    for p in {id(p): p for p in plans.values()}.values():
        p.close()
    print(json.dumps(out))


# The paper's own 3D type 1 figure (Sec. 6.1, Table 2), quoted as context
# with its hardware: another machine, another problem size, FP64.
PAPER_CPU_CONTEXT = {
    "what": "3D type 1, N = 256^3 modes, M = 3e8 points clustered at the origin, tol 1e-6",
    "time_s": 14.6,
    "nu_pts_per_s": 3e8 / 14.6,
    "rel_l2": 1.4e-6,
    "hardware": "2 x Intel Xeon E5-2643 (3.4 GHz), 12 cores / 24 threads, FP64",
    "source": "Sec. 6.1, Table 2",
}


def bench_type3(args, wl):
    """Type 3 (eq. (3)): a step is setpts (bounds, grid choice, rescaling, sorts of
    the sources and of the targets, per-target factors) + execute (prephase,
    spread, inner type 2, correction).  ``value`` counts sources + targets."""
    import torch
    from oracle import oracle as O
    from paper_1808_06736_amd import binding as B
    prec = wl.prec
    cdt = torch.complex64 if prec == "f32" else torch.complex128
    xs_np, ss_np, c_np = wl.coords(), wl.targets(), wl.strengths()
    xs = [torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in xs_np]
    ss = [torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in ss_np]
    c_in = torch.from_numpy(c_np).cuda()
    M, N = wl.M, len(ss_np[0])
    p = B.Plan3(wl.dim, wl.eps, dtype=cdt, debug=1)
    p.setpts(xs, ss)
    out = torch.empty(N, dtype=cdt, device="cuda")
    torch.cuda.synchronize()

    def step(rec=None):
        p.setpts(xs, ss)
        st_set = p.stats().t_setpts
        p.execute(c_in, out)
        if rec is not None:
            s = p.stats()
            rec.append((st_set, s.t_spread_or_interp, s.t_fft, s.t_deconv_or_amplify,
                        s.t_execute))

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    rec = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step(rec)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    r = np.array(rec).mean(axis=0)
    info = p.info()
    nf = [int(info.nf[m]) for m in range(wl.dim)]
    stages = {"setpts_ms": float(r[0]), "spread_ms": float(r[1]), "inner_type2_ms": float(r[2]),
              "inner_interp_ms": float(r[3]), "execute_ms": float(r[4])}
    # dominant kernel: step 1 spreading (M sources onto the type 3 grid) or the
    # inner interpolation (N targets)
    if r[1] >= r[3]:
        kind, npts, dur, kname = "spread", M, r[1], "spread_mfma_kernel"
    else:
        kind, npts, dur, kname = "interp", N, r[3], "interp_mfma_kernel"
    bytes_, flops = algorithmic_work(int(info.w), wl.dim, npts, 1, nf, prec, kind)
    peak = FP32_PEAK_TFLOPS if prec == "f32" else FP64_PEAK_TFLOPS
    roof = {"bound": "mfma", "achieved": flops / (dur * 1e-3) / 1e12, "peak": peak,
            "unit": "TFLOP/s"}
    roof["frac"] = roof["achieved"] / roof["peak"]
    roof.update({"traffic": None, "kernel": f"{kname}<{int(info.w)}>", "algorithmic_bytes": bytes_,
                 "algorithmic_flops": flops, "mean_launch_ms": float(dur),
                 "hbm_frac": bytes_ / (dur * 1e-3) / 1e9 / HBM_PEAK_GBS})
    res = {
        "metric": "NU points/sec (sources + targets), 3D type 3 at eps=1e-6",
        "value": (M + N) / (elapsed / args.steps), "unit": "NU pts/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": prec,
        "data": "synthetic",
        "config": {"workload": wl.name, "dim": wl.dim, "M": M, "N_targets": N, "eps": wl.eps,
                   "sources": "uniform in [-pi, pi)^3",
                   "targets": f"uniform in [-{wl.extra['S']:g}, {wl.extra['S']:g})^3",
                   "w": int(info.w), "type3_grid": nf,
                   "step": "setpts (bounds, grid, rescaling, both sorts, factors) + execute"},
        "stages": stages, "roofline": roof}
    if not args.no_cpu_baseline:
        # the oracle on a bounded sample of targets (all sources)
        nt = 64 if args.cpu_sample <= 0 else args.cpu_sample
        idx = I.rng(7).choice(N, size=nt, replace=False)
        t1 = time.perf_counter()
        ref = O.type3(xs_np, c_np, [a[idx] for a in ss_np], 1)
        dt = time.perf_counter() - t1
        rate = nt * M / dt
        res["cpu_baseline"] = {"value": (M + N) / (N * M / rate), "unit": "NU pts/s",
                               "cores": O.default_threads(), "kind": "oracle",
                               "sample": f"{nt} targets x {M} sources ({dt:.1f} s); scaled to "
                                         f"all {N} targets of one step",
                               "cpu": _cpu_model()}
        e, lo, hi = O.rel_l2_interval(out.cpu().numpy()[idx], ref, seed=3)
        res["parity"] = {"rel_l2": e, "ci95": [lo, hi], "bar": 10 * wl.eps}
    p.close()
    print(json.dumps(res))


def sort_ablation(wl, N, coords, c_in, f_in, outs, cdt, stages, reps=3):
    """The bin sort's effect (Sec. 5.1): execute with the points in the caller's
    order (sort 0: one thread per point, global atomics for type 1, direct
    gathers for type 2) against the bin-sorted execute of the timed loop, alone
    and with the sort (setpts) added."""
    import torch
    from paper_1808_06736_amd import binding as B
    res = {}
    sort_ms = stages["type1"]["setpts_ms"]
    for t in wl.types:
        p = B.Plan(t, N, wl.eps, dtype=cdt, sort=0)
        p.setpts(*coords)
        out = torch.empty_like(outs[t])   # the timed loop's outputs stay for the parity check
        if t == 1:
            def run():
                p.execute(c_in, out)
        else:
            def run():
                p.execute(out, f_in)
        run()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            run()
        e1.record()
        e1.synchronize()
        unsorted = e0.elapsed_time(e1) / reps
        p.close()
        srt = stages[f"type{t}"]["execute_ms"]
        res[f"type{t}"] = {"unsorted_execute_ms": unsorted, "sorted_execute_ms": srt,
                           "sort_ms": sort_ms, "speedup_execute": unsorted / srt,
                           "speedup_with_sort": unsorted / (srt + sort_ms)}
    return res


def serve_bench(nreq, loads, nslots, seed=5):
    """Served vs plain latency on the serving mix (Poisson arrivals).

    The mix: type U{1,2}, d U{2,3}, N_i U[64,512] (2D) / U[64,160] (3D), M
    log-uniform in [1e5, 5e6], uniform or clustered points, eps U{1e-3, 1e-6
    (single), 1e-9 (double)} (inputs.serve_mix), every request with its own
    data.  Paths:
    * plain: one request at a time in arrival order, each planned, sorted,
      executed and freed (the paper's one-call interface, Sec. 2);
    * plain_reuse: one at a time with the plan already made (setpts + execute
      only: each plain request's time without its plan creation and
      destruction), which separates what the served path gains from plan
      caching from what it gains from overlap;
    * served_warm: the request loop with `nslots` worker streams and its plan
      cache filled by an untimed pass over the same requests;
    * served_cold: a fresh request loop (empty plan cache).
    Loads are taken against the plain path's serial throughput and, in
    ``loads_vs_plain_reuse``, against the plan-reusing path's.
    Both plain paths are serial, so their latency at an arrival sequence
    follows from each request's measured service time (single-server FIFO
    queue: start = max(arrival, previous finish)); the served paths are run
    with submissions at the arrival times.  Arrivals are Poisson at `loads` x
    the plain serial request rate.  Every shape is run once untimed first on
    both paths (rocFFT compiles kernels for new sizes).  Every served result is
    compared with the plain result of the same request on 256 sampled outputs.
    """
    import torch
    from paper_1808_06736_amd import binding as B
    reqs = I.serve_mix(nreq, seed=seed)
    data = []
    for k, wl in enumerate(reqs):
        cdt = torch.complex64 if wl.prec == "f32" else torch.complex128
        rdt = torch.float32 if wl.prec == "f32" else torch.float64
        xs = I.device_points(wl.M, wl.dim, 20_000 + k, wl.points, 0.3, rdt)
        N = wl.N[:wl.dim]
        if wl.types[0] == 1:
            c = I.device_complex((wl.M,), 30_000 + k, cdt)
            f = torch.empty(tuple(reversed(N)), dtype=cdt, device="cuda")
        else:
            c = torch.empty(wl.M, dtype=cdt, device="cuda")
            f = I.device_complex(tuple(reversed(N)), 30_000 + k, cdt)
        data.append((wl, xs, c, f))
    torch.cuda.synchronize()
    gsel = torch.Generator(device="cpu").manual_seed(seed)
    sample = []   # 256 output positions per request
    for wl, xs, c, f in data:
        out = f if wl.types[0] == 1 else c
        sample.append(torch.randint(0, out.numel(), (256,), generator=gsel).cuda())

    def output(d):
        wl, xs, c, f = d
        return (f if wl.types[0] == 1 else c).reshape(-1)

    def plain_one(wl, xs, c, f):
        """One plain request; returns (service time, time of setpts + execute)."""
        t0 = time.perf_counter()
        p = B.Plan(wl.types[0], wl.N[:wl.dim], wl.eps, dtype=c.dtype)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        p.setpts(*xs)
        p.execute(c, f)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        p.close()
        return time.perf_counter() - t0, t2 - t1

    progress(f"serving: data of {nreq} requests ready")
    # warm-up: every shape once on both paths
    for k, d in enumerate(data):
        plain_one(*d)
        if (k + 1) % 100 == 0:
            progress(f"serving: plain warm-up {k + 1}/{nreq}")
    warm = B.Server(nslots=nslots, hbm_budget_bytes=64 << 30)
    for tk in [warm.submit(wl.types[0], xs, c, f, wl.eps) for wl, xs, c, f in data]:
        warm.wait(tk)
    progress("serving: served warm-up done")

    # plain service times and the reference outputs; the plan-reusing path's
    # service time is the same request's setpts + execute (the plan made and
    # freed outside it), since holding a plan for each of the mix's shapes at
    # once would not fit the device
    times = np.array([plain_one(*d) for d in data])
    s_plain, s_reuse = times[:, 0], times[:, 1]
    progress(f"serving: plain service times measured ({times[:, 0].sum():.2f} s serial)")
    ref = [output(d)[sample[k]].clone() for k, d in enumerate(data)]
    serial = float(s_plain.sum())
    pts = np.array([float(wl.M) for wl, *_ in data])

    def fifo(arrive, svc):
        lat, fin = np.empty(len(svc)), 0.0
        for k in range(len(svc)):
            st = max(arrive[k], fin)
            fin = st + svc[k]
            lat[k] = fin - arrive[k]
        return lat, fin          # latencies, finish of the last request

    def wait_until(t_abs):
        while True:
            dt = t_abs - time.perf_counter()
            if dt <= 0:
                return
            time.sleep(dt - 2e-4 if dt > 1e-3 else 0)

    classes = sorted({(wl.types[0], wl.dim, wl.eps) for wl, *_ in data})
    cls_idx = {cl: [k for k, (wl, *_) in enumerate(data) if (wl.types[0], wl.dim, wl.eps) == cl]
               for cl in classes}

    def summary(lat, wall):
        out = {"p50_ms": 1e3 * float(np.percentile(lat, 50)),
               "p99_ms": 1e3 * float(np.percentile(lat, 99)),
               "pts_per_s": float(pts.sum() / wall)}
        out["per_class"] = {
            f"type{t} {d}d eps {e:g}": {
                "requests": len(ix), "p50_ms": 1e3 * float(np.percentile(lat[ix], 50)),
                "pts_per_s_per_request": float(np.mean(pts[ix] / lat[ix]))}
            for (t, d, e), ix in cls_idx.items()}
        return out

    def served_run(srv, arrive):
        srv.reset_stats()
        tickets = []
        start = time.perf_counter()
        for k, (wl, xs, c, f) in enumerate(data):
            wait_until(start + arrive[k])
            tickets.append(srv.submit(wl.types[0], xs, c, f, wl.eps))
        res = [srv.wait(t) for t in tickets]
        wall = time.perf_counter() - start
        torch.cuda.synchronize()
        lat = np.array([r[1] for r in res]) * 1e-3
        err = max(float(torch.linalg.vector_norm(output(d)[sample[k]] - ref[k]) /
                        torch.linalg.vector_norm(ref[k]).clamp_min(1e-300))
                  for k, d in enumerate(data))
        st = srv.stats()
        out = summary(lat, wall)
        out.update({"failed": int(sum(1 for r in res if r[0] >= 2)),
                    "plan_cache_hits": int(st.plan_cache_hits),
                    "plan_cache_misses": int(st.plan_cache_misses),
                    "hbm_peak_bytes": int(st.hbm_peak),
                    "max_rel_l2_vs_plain_on_samples": err})
        return out

    runs = []
    for load in loads:
        rate = load * nreq / serial
        gaps = np.random.Generator(np.random.PCG64(seed)).exponential(1.0 / rate, size=nreq)
        arrive = np.cumsum(gaps) - gaps[0]
        lp, wall_p = fifo(arrive, s_plain)
        lr, wall_r = fifo(arrive, s_reuse)
        plain = summary(lp, wall_p)
        reuse = summary(lr, wall_r)
        served_w = served_run(warm, arrive)
        cold = B.Server(nslots=nslots, hbm_budget_bytes=64 << 30)
        served_c = served_run(cold, arrive)
        cold.close()
        progress(f"serving: load {load} of the plain rate done")
        runs.append({"offered_load": load, "arrival_rate_per_s": rate, "plain": plain,
                     "plain_reuse": reuse, "served_warm": served_w, "served_cold": served_c,
                     "p50_speedup_warm_vs_plain": plain["p50_ms"] / max(served_w["p50_ms"], 1e-9),
                     "p99_speedup_warm_vs_plain": plain["p99_ms"] / max(served_w["p99_ms"], 1e-9),
                     "p50_speedup_warm_vs_plain_reuse": reuse["p50_ms"] / max(served_w["p50_ms"], 1e-9),
                     "p99_speedup_warm_vs_plain_reuse": reuse["p99_ms"] / max(served_w["p99_ms"], 1e-9)})
    # the same loads against the plain path that reuses plans: near its
    # capacity, what the worker streams' overlap adds
    runs_reuse = []
    serial_r = float(s_reuse.sum())
    for load in loads:
        rate = load * nreq / serial_r
        gaps = np.random.Generator(np.random.PCG64(seed + 1)).exponential(1.0 / rate, size=nreq)
        arrive = np.cumsum(gaps) - gaps[0]
        lr, wall_r = fifo(arrive, s_reuse)
        reuse = summary(lr, wall_r)
        served_w = served_run(warm, arrive)
        progress(f"serving: load {load} of the plan-reusing rate done")
        runs_reuse.append({"offered_load": load, "arrival_rate_per_s": rate, "plain_reuse": reuse,
                           "served_warm": served_w,
                           "p50_speedup": reuse["p50_ms"] / max(served_w["p50_ms"], 1e-9),
                           "p99_speedup": reuse["p99_ms"] / max(served_w["p99_ms"], 1e-9),
                           "throughput_ratio": served_w["pts_per_s"] / reuse["pts_per_s"]})
    warm.close()
    return {"requests": nreq, "slots": nslots, "plain_serial_s": serial,
            "loads_vs_plain_reuse": runs_reuse,
            "plain_reuse_serial_s": float(s_reuse.sum()),
            "plain_pts_per_s_serial": float(pts.sum() / serial),
            "plain_reuse_pts_per_s_serial": float(pts.sum() / s_reuse.sum()),
            "loads": runs}


def batched_headline(wl, coords, cdt, nvec=8, reps=3):
    """NU pts/s of nvec strength (type 1) or coefficient (type 2) vectors on
    the workload's points: one plan with ntransf = nvec (fused launches) against
    nvec executes on one ntransf = 1 plan; the points are sorted once either
    way (setpts not timed)."""
    import torch
    from paper_1808_06736_amd import binding as B
    N, M = wl.N[:wl.dim], wl.M
    res = {"vectors": nvec}

    def best(fn):
        fn()
        torch.cuda.synchronize()
        b = float("inf")
        for _ in range(reps):
            t0 = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            b = min(b, time.perf_counter() - t0)
        return b

    for t in (1, 2):
        pb = B.Plan(t, N, wl.eps, dtype=cdt, ntransf=nvec)
        pb.setpts(*coords)
        p1 = B.Plan(t, N, wl.eps, dtype=cdt)
        p1.setpts(*coords)
        if t == 1:
            cv = I.device_complex((nvec, M), 777, cdt)
            fv = torch.empty((nvec,) + tuple(reversed(N)), dtype=cdt, device="cuda")
            tb = best(lambda: pb.execute(cv, fv))
            tl = best(lambda: [p1.execute(cv[k], fv[k]) for k in range(nvec)])
        else:
            fv = I.device_complex((nvec,) + tuple(reversed(N)), 778, cdt)
            cv = torch.empty((nvec, M), dtype=cdt, device="cuda")
            tb = best(lambda: pb.execute(cv, fv))
            tl = best(lambda: [p1.execute(cv[k], fv[k]) for k in range(nvec)])
        info = pb.info()
        res[f"type{t}"] = {"batched_pts_per_s": M * nvec / tb, "plan_loop_pts_per_s": M * nvec / tl,
                           "batched_over_loop": tl / tb, "chunk": int(info.ntransf_chunk),
                           "method": int(info.spread_method if t == 1 else info.interp_method)}
        pb.close()
        p1.close()
        del cv, fv
    return res


def batched_vs_plain(wl, coords, c_in, f_in, plans, outs, cdt, reps=5):
    """NU pts/s of the fused batched execute against the same ntransf vectors
    run one at a time: on one plan (ntransf = 1, points already sorted), and as
    one-shot calls that plan, sort and execute per vector (the paper's plain
    interface, Sec. 2)."""
    import torch
    from paper_1808_06736_amd import binding as B
    N = wl.N[:wl.dim]
    ntr, M = wl.ntransf, wl.M
    res = {}

    def best(fn, reps=reps):
        fn()
        torch.cuda.synchronize()
        b = float("inf")
        for _ in range(reps):
            t0 = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            b = min(b, time.perf_counter() - t0)
        return b

    t = wl.types[0]
    pb = plans[t]
    tb = best(lambda: pb.execute(c_in, outs[1]) if t == 1 else pb.execute(outs[2], f_in))
    res["batched_pts_per_s"] = M * ntr / tb
    p1 = B.Plan(t, N, wl.eps, dtype=cdt)
    p1.setpts(*coords)
    if t == 1:
        o1 = torch.empty(tuple(reversed(N)), dtype=cdt, device="cuda")
        loop = lambda: [p1.execute(c_in[k], o1) for k in range(ntr)]
    else:
        o1 = torch.empty(M, dtype=cdt, device="cuda")
        loop = lambda: [p1.execute(o1, f_in[k]) for k in range(ntr)]
    tl = best(loop)
    p1.close()
    res["plan_loop_pts_per_s"] = M * ntr / tl

    def oneshots():
        for k in range(ntr):
            q = B.Plan(t, N, wl.eps, dtype=cdt)
            q.setpts(*coords)
            if t == 1:
                q.execute(c_in[k], o1)
            else:
                q.execute(o1, f_in[k])
            q.close()
    to = best(oneshots, reps=2)
    res["oneshot_pts_per_s"] = M * ntr / to
    res["speedup_vs_plan_loop"] = tl / tb
    res["speedup_vs_oneshot"] = to / tb
    return res


def cpu_baseline(wl, coords, c_np, f_np, plans, outs, cpu_sample):
    """Time the FP64 oracle on a bounded sample and scale to NU pts/s of a full step.

    type 1: a seeded product set of S modes per dim (incl. min, 0, max) for all M
    points -> extrapolated to all N modes.  type 2: seeded points (incl. the
    extreme ones; about 2e10 terms, at least 16384 points or all of them) over
    all N modes -> extrapolated to all M points.  For
    batched workloads only the first transform is timed and the time scaled
    by ntransf.
    """
    import torch
    from oracle import oracle as O
    threads = O.default_threads()
    dim, M, ntr = wl.dim, wl.M, wl.ntransf
    N = wl.N[:dim]
    Ntot = math.prod(N)
    S = cpu_sample or {1: 1000, 2: 100, 3: 24}[dim]
    t_full = 0.0
    parts = []
    parity = {}
    if 1 in wl.types:
        modes = [I.sample_modes(n, S, seed=31 + m) for m, n in enumerate(N)]
        c0 = c_np[0] if ntr > 1 else c_np
        t0 = time.perf_counter()
        ref = O.type1(coords, c0, +1, modes=modes, nthreads=threads)
        dt = time.perf_counter() - t0
        nsamp = math.prod(len(m) for m in modes)
        t_full += dt * (Ntot / nsamp) * ntr
        parts.append(f"type 1: {nsamp} modes x {M} points ({dt:.1f} s)")
        fg = outs[1].cpu().numpy()
        fg = fg[0] if ntr > 1 else fg
        idx = np.ix_(*[m + n // 2 for m, n in zip(reversed(modes), reversed(N))])
        e, lo, hi = O.rel_l2_interval(fg[idx], ref, seed=1)
        parity["type1_rel_l2"] = e
        parity["type1_ci95"] = [lo, hi]
    if 2 in wl.types:
        # about 2e10 oracle terms (all points when M is small)
        sel = I.sample_points(coords, max(16384, int(2e10 // Ntot)), seed=37)
        f0 = f_np[0] if ntr > 1 else f_np
        t0 = time.perf_counter()
        ref = O.type2([a[sel] for a in coords], f0, -1, nthreads=threads)
        dt = time.perf_counter() - t0
        t_full += dt * (M / len(sel)) * ntr
        parts.append(f"type 2: {len(sel)} points x {Ntot} modes ({dt:.1f} s)")
        cg = outs[2].cpu().numpy()
        cg = cg[0] if ntr > 1 else cg
        e, lo, hi = O.rel_l2_interval(cg[sel], ref, seed=2)
        parity["type2_rel_l2"] = e
        parity["type2_ci95"] = [lo, hi]
    parity["bar"] = 10 * wl.eps
    value = M * ntr * len(wl.types) / t_full
    return ({"value": value, "unit": "NU pts/s", "cores": threads, "kind": "oracle",
             "sample": "; ".join(parts) + "; scaled to all outputs of one step",
             "cpu": _cpu_model()}, parity)


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


if __name__ == "__main__":
    main()
