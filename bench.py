#!/usr/bin/env python3
"""Throughput of the DD-DLRA time step on one MI355X.

A step is one pass of Algorithm 6 over all subdomains (x stage, y stage,
collision stage) on synthetic inputs already resident in HBM.  The default
workload is the lattice configuration: 224 x 224 cells as 7 x 7 subdomains of
32 x 32, 256 directions (16 Gauss-Legendre polar x 16 azimuthal), fixed
rank 10, checkerboard absorber / scatterer blocks, source in the central
block.  Prints one JSON line.

  python bench.py [--steps K] [--warmup W] [--config C2] [--mode graph]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# dense matrix-core peaks (TFLOP/s) of the products in each precision mode:
# FP64 MFMA, FP32 MFMA, and BF16 MFMA for the split-BF16 mode (whose three
# products per multiply are counted once, as algorithmic flops)
MFMA_PEAK_TFLOPS = {"fp64": 78.6, "fp32": 157.3, "bf16": 2500.0}

WORKLOAD_NAMES = {
    "C1": "gaussian 32x32 cells, 2x2 subdomains, 64 directions, rank 5",
    "C2": "lattice 224x224 cells, 7x7 subdomains of 32x32, 256 directions, rank 10",
    "C3": "lattice 448x448 cells, 7x7 subdomains of 64x64, 1024 directions, rank 20",
    "C4cap": "thick/thin 512x512 cells, 8x8 subdomains of 64x64, 1024 directions, adaptive ranks 2..21",
}


def algorithmic_cost(wl, tmax, work_bytes=8.0):
    """Algorithmic HBM bytes and flops per launch of each kernel kind for one
    step, from the shapes the step must touch.  The stored factors U, V and
    the augmentation matrix are FP64 (8 bytes per element); the K-, L-step
    and V-hat working arrays take work_bytes per element (8 in FP64 mode, 4
    in the mixed modes).  t_s (intermediate rank) is taken as tmax[s]; r_s
    the stored rank."""
    import numpy as np
    N, M, ns = wl.N, wl.M, wl.n_sub
    r = np.asarray(wl.ranks(), float)
    t = np.minimum(np.asarray(tmax, float), wl.r_int_max)

    def m0(axis):
        out = []
        for s in range(ns):
            sx, sy = s % wl.px, s // wl.px
            k = r[s]
            for side in (-1, 1):
                if axis == 0 and 0 <= sx + side < wl.px:
                    k += r[sy * wl.px + sx + side]
                if axis == 1 and 0 <= sy + side < wl.py:
                    k += r[(sy + side) * wl.px + sx]
            out.append(k)
        return np.asarray(out)

    m = (m0(0) + m0(1)) / 2.0
    B, W = 8.0, float(work_bytes)
    cost = {}
    # per advection stage, summed over subdomains; 2 stages per step -> 2 launches
    cost["k_kstep"] = (N * np.sum(B * r + W * t), 2.0 * N * np.sum(3 * r * t + t * (t + 1) / 2), 2)
    # one product Gp = Q^T (Q_shift - Q); Gm = -Gp^T costs no pass
    cost["k_spatial_reduce"] = (W * N * np.sum(t), 2.0 * N * np.sum(t * t), 2)
    cost["k_aug_form"] = (B * M * np.sum(2 * m), 2.0 * M * np.sum(m * m), 2)
    cost["k_ang_reduce"] = (M * np.sum(W * t + B * m), 2.0 * M * np.sum(r * t + 3 * t * t + (m - r) * t), 2)
    cost["k_lstep"] = (W * M * np.sum(2 * t), 2.0 * M * np.sum(2 * t * t), 2)
    # the first Cholesky-QR product of K1 and of L1 per advection stage (t
    # columns, K1 -> Q1 out of place; 2 launches per step each), and the
    # out-of-place products of the collision stage (r columns; the first, and
    # the last, which writes the FP64 state).  The second and third passes
    # work in place and are timed under their own names ("... in place"); the
    # third exits at once when the second took the near-identity factor, so
    # it has no fixed byte count.
    cost["k_gemm[QR K1]"] = (W * N * np.sum(2 * t), 2.0 * N * np.sum(t * t), 2)
    cost["k_gemm[QR L1]"] = (W * M * np.sum(2 * t), 2.0 * M * np.sum(t * t), 2)
    cost["k_gemm[QR K1 collision]"] = (N * np.sum((3 * W + B) * r) / 2.0, 2.0 * N * np.sum(r * r), 2)
    cost["k_gemm[QR L1 collision]"] = (M * np.sum((3 * W + B) * r) / 2.0, 2.0 * M * np.sum(r * r), 2)
    cost["k_coll_kstep"] = (N * np.sum(B * (r + 3) + W * r), 2.0 * N * np.sum(r * r + 4 * r), 1)
    cost["k_coll_reduce"] = (B * N * np.sum(r + 3), 2.0 * N * np.sum(2 * r * r + r), 1)
    cost["k_gemm[U=Q*Bu]"] = (N * np.sum(W * t + B * r), 2.0 * N * np.sum(t * r), 2)
    cost["k_gemm[V=QL*Bv]"] = (M * np.sum(W * t + B * r), 2.0 * M * np.sum(t * r), 2)
    return cost


TS_SOURCES = ("paper_2602_14854_amd/csrc/dd_kernels_ts.hip", "paper_2602_14854_amd/csrc/dd_mfma.h")


def ts_source_hash():
    """Short hash of the tall-skinny kernel sources: traffic measured with
    hardware counters stays valid only while these are unchanged."""
    import hashlib
    h = hashlib.sha256()
    for rel in TS_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel, workload, precision):
    """HBM bytes per launch of `kernel` from the counter summaries committed
    under profiles/ (lines 'traffic kernel=.. workload=.. precision=..
    bytes_per_launch=.. source=..'), or None when there is none for the
    current kernel sources."""
    import glob
    import re
    src = ts_source_hash()
    pat = re.compile(r"\s*traffic kernel=(.+?) workload=(\S+) precision=(\S+) bytes_per_launch=(\S+) source=(\S+)")
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*.md"))):
        with open(path) as f:
            for line in f:
                m = pat.match(line)
                if m and m.group(1) == kernel and m.group(2) == workload and m.group(3) == precision \
                        and m.group(5) == src:
                    return float(m.group(4))
    return None


def precision_comparison(pkg, wl, base_prec, base_ms, steps, warmup, tune, flux_steps=2, wc_wl=None):
    """The metric's third part: the mixed-precision paths against the FP64
    path on the same workload -- time per step (graph mode, timed like the
    main line) and the scalar-flux error after flux_steps steps relative to
    the FP64 path's flux (which the parity tests hold within 1e-10 of the
    oracle).  A mixed path counts as equally accurate when its error is at
    most 1e-4 (the stated bar for mixed paths).  With wc_wl, the same flux
    errors on the well-conditioned variant of the workload (same geometry,
    generic factors with singular values 1 .. 1e-2), where the comparison is
    not dominated by noise-level singular directions."""
    import numpy as np
    import torch
    names = {"fp64": pkg.DD_PREC_FP64, "fp32": pkg.DD_PREC_MIXED_FP32, "bf16": pkg.DD_PREC_MIXED_BF16}

    def flux(prec, w=wl):
        eng = pkg.DDDLRA(w, exec_mode=pkg.DD_EXEC_BATCHED_GRAPH, precision=names[prec])
        eng.step(flux_steps)
        rho = eng.moments()
        eng.close()
        return rho

    def timed(prec):
        stream = torch.cuda.Stream()
        eng = pkg.DDDLRA(wl, exec_mode=pkg.DD_EXEC_BATCHED_GRAPH, precision=names[prec], stream=stream)
        tune(eng)
        eng.step(warmup)
        eng.sync()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        eng.step(steps)
        e1.record(stream)
        stream.synchronize()
        eng.close()
        return e0.elapsed_time(e1) / steps

    ref = flux("fp64")
    ms = {"fp64": base_ms if base_prec == "fp64" else timed("fp64")}
    out = {"reference": f"FP64 path, scalar flux after {flux_steps} steps", "fp64_ms_per_step": round(ms["fp64"], 4)}
    for prec in ("fp32", "bf16"):
        m = base_ms if base_prec == prec else timed(prec)
        err = float(np.linalg.norm(flux(prec) - ref) / np.linalg.norm(ref))
        out[prec] = {"ms_per_step": round(m, 4), "speedup_vs_fp64": round(ms["fp64"] / m, 4),
                     "flux_rel_err": err, "equal_accuracy": bool(err <= 1e-4)}
    if wc_wl is not None:
        ref_wc = flux("fp64", wc_wl)
        wc = {"workload": wc_wl.name}
        for prec in ("fp32", "bf16"):
            err = float(np.linalg.norm(flux(prec, wc_wl) - ref_wc) / np.linalg.norm(ref_wc))
            wc[prec] = {"flux_rel_err": err, "equal_accuracy": bool(err <= 1e-4)}
        out["well_conditioned"] = wc
    return out


def measured_mfma_busy(kernel, workload, precision):
    """Matrix-core busy fraction of `kernel` from the counter summaries under
    profiles/ (lines 'mfma kernel=.. workload=.. precision=.. busy=..
    source=..'), or None when there is none for the current kernel sources."""
    import glob
    import re
    src = ts_source_hash()
    pat = re.compile(r"\s*mfma kernel=(.+?) workload=(\S+) precision=(\S+) busy=(\S+) source=(\S+)")
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*.md"))):
        with open(path) as f:
            for line in f:
                m = pat.match(line)
                if m and m.group(1) == kernel and m.group(2) == workload and m.group(3) == precision \
                        and m.group(5) == src:
                    return float(m.group(4))
    return None


def cpu_baseline(wl, budget_s=12.0, max_steps=30):
    """The FP64 oracle on the host cores, on the first steps of the same
    workload until about budget_s seconds of work."""
    from oracle import ddlra as dd
    threads = None
    try:
        from threadpoolctl import threadpool_info
        info = threadpool_info()
        threads = max((i.get("num_threads", 1) for i in info), default=None)
    except Exception:
        pass
    prob = dd.Problem(wl)
    st = dd.initial_state(wl)
    st = dd.dd_step(st, prob)  # warm-up step
    n, t0 = 0, time.perf_counter()
    upd = 0.0
    while n < max_steps and time.perf_counter() - t0 < budget_s:
        upd += sum(prob.N * prob.M * s.shape[0] for _, s, _ in st)
        st = dd.dd_step(st, prob)
        n += 1
    el = time.perf_counter() - t0
    model = "unknown CPU"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"value": upd / el, "unit": "updates/s", "cores": threads or os.cpu_count(),
            "kind": "oracle",
            "sample": f"steps 2..{n + 1} of the same workload ({n} timed steps, {el:.1f} s, "
                      f"{el / n * 1e3:.0f} ms/step), NumPy/LAPACK FP64 on {model}, "
                      f"{os.cpu_count()} logical CPUs visible"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--config", default="C2")
    ap.add_argument("--mode", default="graph", choices=["graph", "batched", "per-subdomain"])
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32", "bf16"])
    ap.add_argument("--profile-steps", type=int, default=3)
    ap.add_argument("--profile-repeat", type=int, default=10,
                    help="repetitions (replayed as one graph) per timed tall-skinny phase")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-precision-compare", action="store_true")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--wg-per-subdomain", type=int, default=0,
                    help="fix the tall-skinny workgroups per subdomain instead of autotuning")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported by this build "
              "(the path would shard by blocks of subdomains with a halo exchange of low-rank traces)",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import workloads as wk
    import paper_2602_14854_amd as pkg

    torch.cuda.set_device(0)
    wl = wk.make_workload(args.config)
    mode = {"graph": pkg.DD_EXEC_BATCHED_GRAPH, "batched": pkg.DD_EXEC_BATCHED,
            "per-subdomain": pkg.DD_EXEC_PER_SUBDOMAIN}[args.mode]
    prec = {"fp64": pkg.DD_PREC_FP64, "fp32": pkg.DD_PREC_MIXED_FP32, "bf16": pkg.DD_PREC_MIXED_BF16}[args.precision]
    stream = torch.cuda.Stream()
    eng = pkg.DDDLRA(wl, exec_mode=mode, precision=prec, stream=stream)
    print(f"[bench] workload {args.config}: {wl.nx}x{wl.ny} cells, {wl.px}x{wl.py} subdomains, "
          f"M={wl.M}, rank {wl.r_fixed}, mode {args.mode}, precision {args.precision}", file=sys.stderr, flush=True)
    wg_choice, tune_ms = None, None
    if args.wg_per_subdomain:
        eng.set_tiling(args.wg_per_subdomain)
        wg_choice = args.wg_per_subdomain
    elif not args.no_autotune:
        wg_choice, tune_ms = eng.autotune(3)
        print(f"[bench] autotune: {wg_choice} workgroups per subdomain ({tune_ms:.3f} ms/step)",
              file=sys.stderr, flush=True)
    eng.step(args.warmup)
    eng.sync()
    r0, _, _ = eng.ranks()
    updates = float(np.sum(wl.N * wl.M * r0.astype(float)))
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record(stream)
    eng.step(args.steps)
    ev1.record(stream)
    stream.synchronize()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    eng.sync()
    ms_per_step = ev0.elapsed_time(ev1) / args.steps
    r1, tmax, clamps = eng.ranks()
    print(f"[bench] timed {args.steps} steps: {ms_per_step:.3f} ms/step (wall {wall:.3f} s)",
          file=sys.stderr, flush=True)

    # per-kernel timing: the same kernels, launched phase by phase with
    # hipEvent pairs on the engine's stream
    eng.profile(max(1, args.profile_repeat))
    for _ in range(args.profile_steps):
        for st in (0, 1, 2):
            eng.stage(st)
    stats = eng.kernel_stats()
    eng.profile(False)
    eng.close()
    prof_total = sum(ms for _, ms in stats.values())
    kern = {k: {"launches": n, "avg_us": 1e3 * ms / max(n, 1), "share": ms / prof_total}
            for k, (n, ms) in stats.items() if n > 0}
    costs = algorithmic_cost(wl, tmax, 8.0 if args.precision == "fp64" else 4.0)
    ts = {k: v for k, v in kern.items() if k in costs}
    dom = max(ts, key=lambda k: ts[k]["share"])
    nbytes, nflops, _ = costs[dom]
    avg_s = ts[dom]["avg_us"] * 1e-6
    gbs = nbytes / avg_s / 1e9
    tfl = nflops / avg_s / 1e12
    intensity = nflops / nbytes
    peak_tf = MFMA_PEAK_TFLOPS[args.precision]
    bound = "hbm" if intensity < peak_tf * 1e12 / (HBM_PEAK_GBS * 1e9) else "mfma"
    if bound == "hbm":
        roof = {"bound": "hbm", "achieved": round(gbs, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(gbs / HBM_PEAK_GBS, 4)}
    else:
        roof = {"bound": "mfma", "achieved": round(tfl, 3), "peak": peak_tf, "unit": "TFLOP/s",
                "frac": round(tfl / peak_tf, 4)}
    # attainable-roofline fraction: the time the kernel would take at the
    # binding roof (HBM for its bytes or the matrix cores for its flops)
    # over the time it takes
    attainable = max(nbytes / (HBM_PEAK_GBS * 1e9), nflops / (peak_tf * 1e12)) / avg_s
    traffic = measured_traffic(dom, args.config, args.precision)
    roof.update({"kernel": dom, "avg_us": round(ts[dom]["avg_us"], 3),
                 "algorithmic_bytes_per_launch": int(nbytes), "algorithmic_flops_per_launch": int(nflops),
                 "traffic": None if traffic is None else int(traffic),
                 "mfma_busy": measured_mfma_busy(dom, args.config, args.precision),
                 "attainable_frac": round(attainable, 4)})

    out = {
        "metric": "subdomain-cell·angle·rank updates/s per step",
        "value": updates / (ms_per_step * 1e-3),
        "unit": "updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f32+f64", "bf16": "bf16x3+f64"}[args.precision],
        "data": "synthetic",
        "config": {"workload": WORKLOAD_NAMES.get(args.config, args.config), "name": args.config,
                   "subdomains": wl.n_sub, "cells_per_subdomain": wl.N, "directions": wl.M,
                   "rank": int(wl.r_fixed), "r_int_max": int(wl.r_int_max), "exec_mode": args.mode,
                   "precision": args.precision,
                   "max_intermediate_rank": int(np.max(tmax)), "updates_per_step": updates,
                   "wg_per_subdomain": wg_choice},
        "phase_space_points_per_s": float(wl.n_sub * wl.N * wl.M) / (ms_per_step * 1e-3),
        "roofline": roof,
        "kernels": {k: {"avg_us": round(v["avg_us"], 2), "share": round(v["share"], 4), "launches": v["launches"]}
                    for k, v in sorted(kern.items(), key=lambda kv: -kv[1]["share"])},
    }
    if not args.no_precision_compare:
        print("[bench] mixed precision against FP64", file=sys.stderr, flush=True)
        def tune(e):
            if args.wg_per_subdomain:
                e.set_tiling(args.wg_per_subdomain)
            elif not args.no_autotune:
                e.autotune(3)
        try:
            wc_wl = wk.make_workload("wc-" + args.config)
        except KeyError:
            wc_wl = None
        out["mixed_vs_fp64"] = precision_comparison(pkg, wl, args.precision, ms_per_step, args.steps, args.warmup,
                                                    tune, wc_wl=wc_wl)
    if not args.no_cpu_baseline:
        print("[bench] timing the CPU oracle", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(wl)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
