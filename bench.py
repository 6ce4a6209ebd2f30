#!/usr/bin/env python3
"""Throughput of the DD-DLRA time step on one MI355X.

A step is one pass of Algorithm 6 over all subdomains (x stage, y stage,
collision stage) on synthetic inputs already resident in HBM.  The default
workload is the largest configuration: the point-source problem on
[-1,1]^2 with 1024 x 1024 cells as 16 x 16 subdomains of 64 x 64, 2048
directions (32 Gauss-Legendre polar x 64 azimuthal), adaptive ranks capped
at 64 (intermediate ranks at 128), sigma_s = 1, sigma_a = 0.1, 500 steps.
The timed region is steps W+1 .. W+K of that configured run from its
specified initial condition (default W = 5, K = 495: the rest of the run),
with the stored ranks read after every step (a synchronisation per step
inside the timed region, which only adds time) so that the rank-weighted
update count is exact.  The per-kernel figures (roofline of the dominant
kernel, kernel shares) come from a replay of the same steps with each
phase between hipEvent pairs.  Prints one JSON line.

  python bench.py [--steps K] [--warmup W] [--config C5] [--mode graph] [--precision fp64]
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
# FP64 vector ALU peak (256 CUs x 4 SIMDs x 16 FP64 lanes x 2 flops x 2.4 GHz)
ALU_PEAK_TFLOPS = 78.6

WORKLOAD_NAMES = {
    "C1": "gaussian 32x32 cells, 2x2 subdomains, 64 directions, rank 5",
    "C2": "lattice 224x224 cells, 7x7 subdomains of 32x32, 256 directions, rank 10",
    "C3": "lattice 448x448 cells, 7x7 subdomains of 64x64, 1024 directions, rank 20",
    "C4": "thick/thin 512x512 cells, 8x8 subdomains of 64x64, 1024 directions, adaptive ranks 2..40 "
          "(intermediate up to 80)",
    "C4cap": "thick/thin 512x512 cells, 8x8 subdomains of 64x64, 1024 directions, adaptive ranks 2..21",
    "C5": "point source 1024x1024 cells, 16x16 subdomains of 64x64, 2048 directions, adaptive ranks "
          "capped at 64 (intermediate up to 128)",
}
DEFAULT_STEPS = {"C5": 495, "C4": 95, "C4cap": 95}

# kernels of the small per-subdomain phases (one workgroup per subdomain,
# serial linear algebra: latency / vector-ALU bound, no HBM roofline)
SMALL = ("s_", "sw_")


def _m0(wl, ranks, axis):
    import numpy as np
    out = []
    for s in range(wl.n_sub):
        sx, sy = s % wl.px, s // wl.px
        k = ranks[s]
        for side in (-1, 1):
            if axis == 0 and 0 <= sx + side < wl.px:
                k += ranks[sy * wl.px + sx + side]
            if axis == 1 and 0 <= sy + side < wl.py:
                k += ranks[(sy + side) * wl.px + sx]
        out.append(k)
    return np.asarray(out, float)


def algorithmic_cost(wl, ranks, tdim, work_bytes=8.0):
    """Algorithmic HBM bytes and flops per launch of each kernel kind, from
    the shapes the step must touch at stored ranks r_s and intermediate
    ranks t_s (sums over subdomains).  The stored factors U, V and the
    augmentation matrix are FP64 (8 bytes per element); the K-, L-step and
    V-hat working arrays take work_bytes per element.  Small per-subdomain
    kernels get a flop count of their dense linear algebra (bytes: their
    inputs and outputs, negligible)."""
    import numpy as np
    N, M = wl.N, wl.M
    r = np.asarray(ranks, float)
    t = np.minimum(np.asarray(tdim, float), wl.r_int_max)
    m = (_m0(wl, r, 0) + _m0(wl, r, 1)) / 2.0
    B, W = 8.0, float(work_bytes)
    c = {}
    c["k_kstep"] = (N * np.sum(B * r + W * t), 2.0 * N * np.sum(3 * r * t + t * (t + 1) / 2))
    c["k_spatial_reduce"] = (W * N * np.sum(t), 2.0 * N * np.sum(t * t))
    c["kw_xgram[spatial]"] = c["k_spatial_reduce"]
    c["k_aug_form"] = (B * M * np.sum(2 * m), 2.0 * M * np.sum(m * m))
    c["kw_xgram[Gram A]"] = (B * M * np.sum(m), M * np.sum(m * (m + 1)))
    c["k_ang_reduce"] = (M * np.sum(W * t + B * m), 2.0 * M * np.sum(r * t + 3 * t * t + (m - r) * t))
    c["kw_xgram[angular]"] = c["k_ang_reduce"]
    c["k_lstep"] = (W * M * np.sum(2 * t), 2.0 * M * np.sum(2 * t * t))
    c["k_gemm[QR K1]"] = (W * N * np.sum(2 * t), 2.0 * N * np.sum(t * t))
    c["k_gemm[QR L1]"] = (W * M * np.sum(2 * t), 2.0 * M * np.sum(t * t))
    c["k_gemm[QR V-hat]"] = (W * M * np.sum(2 * t), 2.0 * M * np.sum(t * t))
    c["kw_xgram[Gram K1]"] = (W * N * np.sum(t), N * np.sum(t * (t + 1)))
    c["kw_xgram[Gram L1]"] = (W * M * np.sum(t), M * np.sum(t * (t + 1)))
    c["kw_xgram[Gram V-hat]"] = (W * M * np.sum(t), M * np.sum(t * (t + 1)))
    c["k_gemm[V-hat=A*Coef]"] = (M * np.sum(B * m + W * t), 2.0 * M * np.sum(m * t))
    c["k_gemm[QR K1 collision]"] = (N * np.sum((3 * W + B) * r) / 2.0, 2.0 * N * np.sum(r * r))
    c["k_gemm[QR L1 collision]"] = (M * np.sum((3 * W + B) * r) / 2.0, 2.0 * M * np.sum(r * r))
    c["k_coll_kstep"] = (N * np.sum(B * (r + 3) + W * r), 2.0 * N * np.sum(r * r + 4 * r))
    c["k_coll_reduce"] = (B * N * np.sum(r + 3), 2.0 * N * np.sum(2 * r * r + r))
    c["kw_xgram[collision]"] = c["k_coll_reduce"]
    c["kw_xgram[Gram K1 collision]"] = (W * N * np.sum(r), N * np.sum(r * (r + 1)))
    c["k_gemm[U=Q*Bu]"] = (N * np.sum(W * t + B * r), 2.0 * N * np.sum(t * r))
    c["k_gemm[V=QL*Bv]"] = (M * np.sum(W * t + B * r), 2.0 * M * np.sum(t * r))
    # small kernels: dense flop counts (Golub-Van Loan style; SVDs as 12 n^3,
    # Cholesky n^3 / 3 plus the triangular inverse n^3 / 3, the sign
    # iteration as 20 symmetric products of 2 t^3)
    c["s_aug_svd"] = (B * np.sum(m * m), np.sum(12.0 * m ** 3))
    c["s_trunc"] = (B * np.sum(t * t), np.sum(12.0 * t ** 3))
    c["s_adv_prep"] = (B * np.sum(3 * t * t), np.sum(40.0 * t ** 3 + 10.0 * r * t * t))
    c["s_adv_sstep"] = (B * np.sum(6 * t * t), np.sum(20.0 * t ** 3))
    c["s_chol"] = (B * np.sum(t * t), np.sum(2.0 * t ** 3 / 3.0))
    c["sw_chol"] = c["s_chol"]
    return c


def kernel_source_hash():
    """First 16 hex digits of the SHA-256 of the HIP sources (csrc/*.hip and
    *.h in name order): counter figures taken on other sources are stale."""
    import glob
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2602_14854_amd", "csrc")
    for path in sorted(glob.glob(os.path.join(csrc, "*.hip")) + glob.glob(os.path.join(csrc, "*.h"))):
        with open(path, "rb") as f:
            h.update(os.path.basename(path).encode() + b"\0" + f.read())
    return h.hexdigest()[:16]


def measured_value(tag, kernel, workload, precision, field):
    """A counter figure of `kernel` from the summaries committed under
    profiles/ (lines '<tag> kernel=.. workload=.. precision=.. <field>=..
    source=<kernel_source_hash()>'), or None when there is none for the
    current kernel sources."""
    import glob
    import re
    pat = re.compile(r"\s*" + tag + r" kernel=(.+?) workload=(\S+) precision=(\S+) " + field +
                     r"=(\S+) source=(\S+)")
    src = kernel_source_hash()
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*.md"))):
        with open(path) as f:
            for line in f:
                mm = pat.match(line)
                if (mm and mm.group(1) == kernel and mm.group(2) == workload and mm.group(3) == precision
                        and mm.group(5) == src):
                    return float(mm.group(4))
    return None


def run_timed(pkg, wl, mode, prec, warmup, steps, tiling, autotune):
    """Warm-up steps, then `steps` timed steps with the ranks read after each
    one.  Returns (engine, ms_per_step, updates, per-step ranks)."""
    import numpy as np
    import torch
    stream = torch.cuda.Stream()
    eng = pkg.DDDLRA(wl, exec_mode=mode, precision=prec, stream=stream)
    wg, tune_ms = None, None
    if tiling:
        eng.set_tiling(tiling)
        wg = tiling
    elif autotune:
        wg, tune_ms = eng.autotune(3)
    eng.step(warmup)
    r, _, _ = eng.ranks()
    torch.cuda.synchronize()
    updates = 0.0
    ranks = []
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    for _ in range(steps):
        updates += float(np.sum(wl.N * wl.M * r.astype(float)))
        eng.step(1)
        r, _, _ = eng.ranks()
        ranks.append(r.copy())
    e1.record(stream)
    stream.synchronize()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = e0.elapsed_time(e1) / steps
    return eng, ms, updates, ranks, wall, wg, tune_ms


def cpu_baseline(wl, budget_s=20.0):
    """The FP64 oracle on the host cores, on a bounded sample of the same
    workload: whole steps from its initial condition, computed only on the
    domain of dependence of the 2 x 2 subdomains at the centre (the source
    region), rated by the rank-weighted updates of the subdomains it
    advanced."""
    import numpy as np
    from oracle import ddlra as dd
    tests_dir = os.path.join(ROOT, "tests")
    if tests_dir not in sys.path:
        sys.path.insert(0, tests_dir)
    threads = None
    try:
        from threadpoolctl import threadpool_info
        threads = max((i.get("num_threads", 1) for i in threadpool_info()), default=None)
    except Exception:
        pass
    prob = dd.Problem(wl)
    st = dd.initial_state(wl)
    cx, cy = wl.px // 2, wl.py // 2
    sample = {sy * wl.px + sx for sy in range(max(0, cy - 3), min(wl.py, cy + 3))
              for sx in range(max(0, cx - 3), min(wl.px, cx + 3))}
    n, upd, el = 0, 0.0, 0.0
    while el < budget_s and n < 20:
        t0 = time.perf_counter()
        upd += sum(prob.N * prob.M * st[s][1].shape[0] for s in sample)
        st = dd.stage_advect(st, 0, prob, only=sample)
        st = dd.stage_advect(st, 1, prob, only=sample)
        st = dd.stage_collision(st, prob, only=sample)
        el += time.perf_counter() - t0
        n += 1
    model = "unknown CPU"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"value": upd / el, "unit": "updates/s", "cores": threads or os.cpu_count(), "kind": "oracle",
            "sample": f"steps 1..{n} of the same workload on {len(sample)} of its {wl.n_sub} subdomains "
                      f"(the 6 x 6 block at the centre), {el:.1f} s, {el / n * 1e3:.0f} ms/step for the block; "
                      f"NumPy/LAPACK FP64 on {model}, {os.cpu_count()} logical CPUs visible"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=0, help="timed steps (default: the rest of the configured run)")
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--config", default="C5")
    ap.add_argument("--mode", default="graph", choices=["graph", "batched", "per-subdomain"])
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32", "bf16"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-precision-compare", action="store_true")
    ap.add_argument("--no-per-subdomain", action="store_true")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--wg-per-subdomain", type=int, default=0,
                    help="fix the tall-skinny workgroups per subdomain instead of autotuning")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              "(the path would shard by blocks of subdomains with a halo exchange of low-rank traces)",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import workloads as wk
    import paper_2602_14854_amd as pkg

    torch.cuda.set_device(0)
    wl = wk.make_workload(args.config)
    steps = args.steps or DEFAULT_STEPS.get(args.config, 50)
    names = {"fp64": pkg.DD_PREC_FP64, "fp32": pkg.DD_PREC_MIXED_FP32, "bf16": pkg.DD_PREC_MIXED_BF16}
    mode = {"graph": pkg.DD_EXEC_BATCHED_GRAPH, "batched": pkg.DD_EXEC_BATCHED,
            "per-subdomain": pkg.DD_EXEC_PER_SUBDOMAIN}[args.mode]
    print(f"[bench] workload {args.config}: {wl.nx}x{wl.ny} cells, {wl.px}x{wl.py} subdomains, M={wl.M}, "
          f"rank cap {wl.r_max}, steps {args.warmup}+{steps}, mode {args.mode}, precision {args.precision}",
          file=sys.stderr, flush=True)
    tiling = args.wg_per_subdomain
    if not tiling and not args.no_autotune and wl.rank_mode == wk.RANK_ADAPTIVE:
        # adaptive ranks grow over the run: tune the tiling on the state half
        # way through the timed steps (a separate engine, advanced untimed)
        tune_at = args.warmup + steps // 2
        print(f"[bench] autotune on the state after {tune_at} steps", file=sys.stderr, flush=True)
        te = pkg.DDDLRA(wl, exec_mode=pkg.DD_EXEC_BATCHED_GRAPH, precision=names[args.precision])
        te.step(tune_at)
        tiling, tune_ms = te.autotune(3)
        te.close()
        print(f"[bench] autotune: {tiling} workgroups per subdomain ({tune_ms:.3f} ms/step there)",
              file=sys.stderr, flush=True)
    eng, ms_per_step, updates, ranks, wall, wg_choice, tune_ms = run_timed(
        pkg, wl, mode, names[args.precision], args.warmup, steps, tiling, not args.no_autotune)
    r_end, tmax, clamps = eng.ranks()
    print(f"[bench] timed {steps} steps: {ms_per_step:.3f} ms/step (wall {wall:.2f} s), "
          f"wg/subdomain {wg_choice}, final ranks {int(r_end.min())}..{int(r_end.max())}",
          file=sys.stderr, flush=True)

    eng.close()

    # per-kernel timing over the timed region: the same steps replayed from
    # the same initial condition (the state sequence is deterministic), each
    # phase launched on its own between hipEvent pairs on the engine's stream
    # (the timed run launches one graph per step, which hides the kernels);
    # the algorithmic cost of every launch from the ranks at the start of its
    # step (stored ranks) and the largest intermediate ranks reached so far
    print(f"[bench] per-kernel replay of steps {args.warmup + 1}..{args.warmup + steps}", file=sys.stderr,
          flush=True)
    wbytes = 8.0 if args.precision == "fp64" else 4.0
    pe = pkg.DDDLRA(wl, exec_mode=mode, precision=names[args.precision])
    if wg_choice:
        pe.set_tiling(wg_choice)
    pe.step(args.warmup)
    pe.profile(1)
    prev = pe.kernel_stats()
    cost_sum = {}
    for _ in range(steps):
        r0, _, _ = pe.ranks()
        for st in (0, 1, 2):
            pe.stage(st)
        cur = pe.kernel_stats()
        _, t1, _ = pe.ranks()
        c_step = algorithmic_cost(wl, r0, t1, wbytes)
        for k, (n, _) in cur.items():
            dn = n - prev.get(k, (0, 0.0))[0]
            if dn and k in c_step:
                b, f = cost_sum.get(k, (0.0, 0.0))
                cost_sum[k] = (b + dn * c_step[k][0], f + dn * c_step[k][1])
        prev = cur
    pe.profile(False)
    pe.close()
    stats = prev
    prof_total = sum(ms for _, ms in stats.values())
    kern = {k: {"launches": n, "avg_us": 1e3 * ms / max(n, 1), "share": ms / prof_total, "ms": ms}
            for k, (n, ms) in stats.items() if n > 0}
    # per-launch algorithmic cost averaged over the replayed launches
    costs = {k: (b / kern[k]["launches"], f / kern[k]["launches"]) for k, (b, f) in cost_sum.items()}
    peak_tf = MFMA_PEAK_TFLOPS[args.precision]

    def roofline(k):
        nbytes, nflops = costs[k]  # per launch (one launch covers all subdomains)
        avg_s = kern[k]["avg_us"] * 1e-6
        if k.startswith(SMALL):
            tf = nflops / avg_s / 1e12
            out = {"bound": "alu", "achieved": round(tf, 4), "peak": ALU_PEAK_TFLOPS, "unit": "TFLOP/s",
                   "frac": round(tf / ALU_PEAK_TFLOPS, 6)}
        else:
            gbs, tfl = nbytes / avg_s / 1e9, nflops / avg_s / 1e12
            if nflops / nbytes < peak_tf * 1e12 / (HBM_PEAK_GBS * 1e9):
                out = {"bound": "hbm", "achieved": round(gbs, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                       "frac": round(gbs / HBM_PEAK_GBS, 4)}
            else:
                out = {"bound": "mfma", "achieved": round(tfl, 3), "peak": peak_tf, "unit": "TFLOP/s",
                       "frac": round(tfl / peak_tf, 4)}
        tr = measured_value("traffic", k, args.config, args.precision, "bytes_per_launch")
        out.update({"kernel": k, "avg_us": round(kern[k]["avg_us"], 3),
                    "algorithmic_bytes_per_launch": int(nbytes), "algorithmic_flops_per_launch": int(nflops),
                    "traffic": None if tr is None else int(tr),
                    "mfma_busy": measured_value("mfma", k, args.config, args.precision, "busy")})
        return out

    known = [k for k in kern if k in costs]
    dom = max(known, key=lambda k: kern[k]["share"])
    ts_known = [k for k in known if not k.startswith(SMALL)]
    dom_ts = max(ts_known, key=lambda k: kern[k]["share"])
    small_share = sum(v["share"] for k, v in kern.items() if k.startswith(SMALL))
    # step-level algorithmic bytes over the step time (tall-skinny kernels)
    step_bytes = sum(cost_sum[k][0] for k in ts_known) / steps
    prof_step_ms = prof_total / steps

    out = {
        "metric": "subdomain-cell·angle·rank updates/s per step",
        "value": updates / (ms_per_step * 1e-3 * steps),
        "unit": "updates/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f32+f64", "bf16": "bf16x3+f64"}[args.precision],
        "data": "synthetic",
        "config": {"workload": WORKLOAD_NAMES.get(args.config, args.config)
                   + f"; steps {args.warmup + 1}..{args.warmup + steps} of the configured run from its "
                     "initial condition",
                   "name": args.config, "subdomains": wl.n_sub, "cells_per_subdomain": wl.N,
                   "directions": wl.M, "rank_cap": int(wl.r_max), "r_int_max": int(wl.r_int_max),
                   "exec_mode": args.mode, "precision": args.precision,
                   "final_ranks": [int(r_end.min()), int(r_end.max())],
                   "final_rank_histogram": np.bincount(r_end).tolist(),
                   "max_intermediate_rank": int(np.max(tmax)), "rank_clamp_events": int(clamps),
                   "updates_timed": updates, "wg_per_subdomain": wg_choice},
        "phase_space_points_per_s": float(wl.n_sub * wl.N * wl.M) / (ms_per_step * 1e-3),
        "roofline": roofline(dom),
        "roofline_tall_skinny": roofline(dom_ts),
        "step_level": {"algorithmic_bytes_per_step": step_bytes,
                       "algorithmic_GBps": round(step_bytes / (prof_step_ms * 1e-3) / 1e9, 2),
                       "frac_of_hbm_peak": round(step_bytes / (prof_step_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 5),
                       "profiled_ms_per_step": round(prof_step_ms, 3),
                       "small_kernel_time_share": round(small_share, 4)},
        "kernels": {k: {"avg_us": round(v["avg_us"], 2), "share": round(v["share"], 4), "launches": v["launches"]}
                    for k, v in sorted(kern.items(), key=lambda kv: -kv[1]["share"])},
    }

    if not args.no_per_subdomain:
        # the plain FP64 per-subdomain path (same kernels, one launch per
        # subdomain per phase, no graph) on the first steps of the same run,
        # against the batched graph on the same steps
        nps = min(10, steps)
        print(f"[bench] FP64 per-subdomain path, steps {args.warmup + 1}..{args.warmup + nps}",
              file=sys.stderr, flush=True)
        e, ms_ps, upd_ps, _, _, _, _ = run_timed(pkg, wl, pkg.DD_EXEC_PER_SUBDOMAIN, pkg.DD_PREC_FP64,
                                                  args.warmup, nps, wg_choice, False)
        e.close()
        e, ms_b, upd_b, _, _, _, _ = run_timed(pkg, wl, pkg.DD_EXEC_BATCHED_GRAPH, names[args.precision],
                                                args.warmup, nps, wg_choice, False)
        e.close()
        out["fp64_per_subdomain"] = {"steps": [args.warmup + 1, args.warmup + nps],
                                     "ms_per_step": round(ms_ps, 3), "batched_graph_ms_per_step": round(ms_b, 3),
                                     "speedup_batched": round(ms_ps / ms_b, 2)}
        out["vs_baseline"] = round(ms_ps / ms_b, 3)
        out["vs_baseline_definition"] = ("batched graph over the plain FP64 per-subdomain GPU path on the same "
                                         "GPU and steps (the comparison the hot path is measured against)")

    if not args.no_precision_compare:
        # mixed precision against FP64 over the same timed steps; the flux
        # of each at the end of the run against the FP64 path's (which the
        # parity tests tie to the oracle); equal accuracy: within 1e-4
        print("[bench] mixed precision against FP64", file=sys.stderr, flush=True)
        res = {"reference": f"FP64 batched path, scalar flux after step {args.warmup + steps}"}
        base = {}
        for prec in ("fp64", "fp32", "bf16"):
            e, ms, upd, _, _, _, _ = run_timed(pkg, wl, pkg.DD_EXEC_BATCHED_GRAPH, names[prec], args.warmup,
                                               steps, wg_choice, False)
            base[prec] = (ms, e.moments())
            e.close()
        ref = base["fp64"][1]
        res["fp64_ms_per_step"] = round(base["fp64"][0], 3)
        for prec in ("fp32", "bf16"):
            err = float(np.linalg.norm(base[prec][1] - ref) / np.linalg.norm(ref))
            res[prec] = {"ms_per_step": round(base[prec][0], 3),
                         "speedup_vs_fp64": round(base["fp64"][0] / base[prec][0], 4),
                         "flux_rel_err": err, "equal_accuracy": bool(err <= 1e-4)}
        out["mixed_vs_fp64"] = res

    if not args.no_cpu_baseline:
        print("[bench] timing the CPU oracle", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(wl)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
