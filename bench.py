#!/usr/bin/env python
"""Benchmark: adaptive randomized HSS compressions per second on one MI355X.

Workload (default): dense Laplace kernel A_ij = 1/(4 pi |x_i - x_j|),
A_ii = 1, n = 32768 points uniform on the unit sphere (seed 1), ordered by
recursive coordinate bisection with leaf size 128, entries generated on the
fly; incrementing strategy d0 = 128, delta_d = 64; rtol = 1e-6,
atol = 1e-12, per-node safety factor eta = 0.05 (one value for every
workload); FP64 throughout.  The points are resident in HBM before the
timed region; the Gaussian random matrix is drawn by the library on the
device from seed 0, inside the timed region.  One step = one full
hss_compress call (random columns, sampling, extraction, local samples,
stopping tests, IDs, reductions).

Other workloads (--workload): sphere Laplace n = 8192; Toeplitz n = 1024
(doubling strategy, d0 = 64); Gaussian kernel n = 65536 in the unit cube
(kd tree, leaf 256), with --precision fp32 / bf16x3 sampling and --rtol;
learned-* workloads time the learned d0 (predictor network) and, beside
it, the adaptive start d0 = 128 on Toeplitz n = 131072 and sphere Laplace
n = 65536.

Prints one JSON line.  `roofline` covers the kernel class with the largest
measured GPU time (HIP events around every launch of one extra profiled
compression); `cpu_baseline` times the CPU oracle on a bounded sample of
the same workload.
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

METRIC = "HSS compressions/s + sampling TFLOP/s at rel err≤1e-6; learned/mixed vs FP64"
PEAK_FP64_TFLOPS = 78.6
PEAK_FP32_TFLOPS = 157.3
PEAK_BF16_TFLOPS = 2500.0
PEAK_HBM_GBS = 8000.0
# Per-node safety factor on the tolerance (eps' = eta eps / level), frozen
# for every workload: the largest value that keeps every checked
# compression (the 256-matrix batch included) at or below rtol.
ETA = 0.05

# kernel class -> (HIP kernel name, bound)
KCLASS_INFO = {
    "SAMPLE": ("k_sample_f64", "mfma"),
    "GEMM": ("k_gemm_grouped+k_gemm_splitk_sum", "mfma"),
    "TEST_NORMS": ("k_fn_norms/k_cq_chol/k_fn_rtest", "hbm"),
    # block-pivoted ID (k_idb_select/gather/chol/rows1/small/rows2/norms and its GEMMs); one-step pivot
    # steps where a panel is too wide for it.  FP64-compute-bound by the ID's arithmetic intensity
    "QRCP_STEP": ("k_idb_* + block GEMMs (block-pivoted ID)", "mfma"),
    "TEST_QR": ("k_qrcp_step (stopping-test QR, no pivoting)", "hbm"),
    "RNG": ("k_randn", "hbm"),
    "QRCP_WG": ("k_qrcp_wg", "hbm"),
    "QFORM": ("k_qf_prep/k_qf_solve/k_qform", "hbm"),
    "GATHER": ("k_ls_gather/k_red_gather/k_fn_copy", "hbm"),
    "EXTRACT": ("k_extract_nodes", "hbm"),
    "TRSM": ("k_trsm_diag", "hbm"),
    "SAMPLE_REDUCE": ("k_splitk_reduce", "hbm"),
    "QRCP_OTHER": ("k_qrcp_plan/k_qrcp_init/k_qrcp_alive/k_qrcp_fin", "hbm"),
    "MISC": ("k_plan/k_finalize/...", "hbm"),
}

WORKLOADS = {
    "laplace-sphere-32768": dict(family="laplace", n=32768, leaf=128, method="rcb", points_seed=1,
                                 strategy="inc_fnorm", d0=128, delta_d=64, d_max=4096),
    "laplace-sphere-8192": dict(family="laplace", n=8192, leaf=128, method="rcb", points_seed=1,
                                strategy="inc_fnorm", d0=128, delta_d=64, d_max=2048),
    "toeplitz-1024": dict(family="toeplitz", n=1024, leaf=64, method="bisect", h=0.1,
                          strategy="dbl_fnorm", d0=64, delta_d=64, d_max=1024),
    # Gaussian kernel exp(-|x-y|^2 / 0.5) + 1e-2 I on uniform points in the unit cube
    "gauss-cube-65536": dict(family="gauss", n=65536, leaf=256, method="kd", points_seed=2, sigma=0.5,
                             strategy="inc_fnorm", d0=128, delta_d=64, d_max=2048),
    # 256 independent matrices (128 Toeplitz h ~ U[0.05, 0.5], 128 sphere Laplace), n log-uniform in
    # [2048, 16384], leaf 128, compressed together by hss_compress_batched
    "batch-256": dict(batch=256, seed=3, n_lo=2048, n_hi=16384, leaf=128, family="toeplitz+laplace",
                      method="bisect/rcb", strategy="dbl_fnorm", d0=64, delta_d=64, d_max=2048),
    # learned d0 against the adaptive start d0 = 128 (both incrementing, delta_d = 64)
    "learned-toeplitz-131072": dict(family="toeplitz", n=131072, leaf=128, method="bisect", h=0.1,
                                    strategy="inc_fnorm", d0=128, delta_d=64, d_max=2048, learned=True,
                                    r_seed=4),
    "learned-laplace-sphere-65536": dict(family="laplace", n=65536, leaf=128, method="rcb", points_seed=4,
                                         strategy="inc_fnorm", d0=128, delta_d=64, d_max=6144, learned=True,
                                         r_seed=4),
}


# HBM traffic of the dominant kernel, from two rocprofv3 --pmc passes
# (FETCH_SIZE, then WRITE_SIZE; KiB per dispatch, averaged over the
# kernel's dispatches in one compression of the workload) scaled by what the
# same counters read for a 1 GiB device copy (bench.py --copy-calibration).
# The figure is only reported while the kernel's source file is the one the
# counters were taken on (sha256); profiles/ holds the summaries.
TRAFFIC = {
    ("laplace-sphere-32768", "SAMPLE"): {
        "source": "paper_1810_04125_amd/csrc/k_sample.hip",
        "sha256": "aed9b951c64de8d3ef7a6981b256ef75861c7a2a900365e930d5300e75827d8b",
        "fetch_kib": 71851.3, "write_kib": 131072.0,               # k_sample_f64, 44 dispatches
        "fetch_scale": 1048576.0 / 524302.0, "write_scale": 1.0,   # 1 GiB copy: FETCH 524302 KiB, WRITE 1048576 KiB
    },
}

# Counters of the sampling kernel from rocprofv3 --pmc passes over one
# compression of the workload (profiles/ holds the summaries), averaged per
# dispatch: SQ_VALU_MFMA_BUSY_CYCLES and SQ_ACTIVE_INST_VALU over the SIMD
# cycles of the busy CUs (4 SQ_BUSY_CU_CYCLES); FP64 MFMA work from
# SQ_INSTS_VALU_MFMA_MOPS_F64 (512 flops per MOP).
SAMPLE_COUNTERS = {
    ("laplace-sphere-32768", "fp64"): {
        "source_sha256": "aed9b951c64de8d3ef7a6981b256ef75861c7a2a900365e930d5300e75827d8b",
        "mfma_busy_frac": round(4.39258e9 / (4 * 1.67249e9), 4),
        "valu_active_frac": round(4.39561e8 / (4 * 1.67249e9), 4),
        "mfma_valu_coexec_cycles": 0,
        "mfma_flops_per_dispatch": 2.74536e8 * 512,
        "valu_fp64_flops_per_dispatch": 3.08853e8,
        "avg_dispatch_us": 3033.249,
        "counter_tflops": round(2.74536e8 * 512 / 3033.249e-6 / 1e12, 2),
    },
}


def sample_counters(workload, precision):
    import hashlib
    c = SAMPLE_COUNTERS.get((workload, precision))
    src = os.path.join(ROOT, "paper_1810_04125_amd", "csrc", "k_sample.hip")
    if not c or hashlib.sha256(open(src, "rb").read()).hexdigest() != c["source_sha256"]:
        return None
    return {k: v for k, v in c.items() if k != "source_sha256"}


def traffic_bytes(workload, cls):
    import hashlib
    t = TRAFFIC.get((workload, cls))
    if not t:
        return None
    src = os.path.join(ROOT, t["source"])
    if not os.path.exists(src) or hashlib.sha256(open(src, "rb").read()).hexdigest() != t["sha256"]:
        return None
    return 1024.0 * (t["fetch_kib"] * t["fetch_scale"] + t["write_kib"] * t["write_scale"])


# launch-shape table from the autotuner (python -m paper_1810_04125_amd.autotune), loaded when present
TUNE_FILE = os.path.join(ROOT, "paper_1810_04125_amd", "data", "tunables_gfx950.txt")

# classes whose launches are one kernel each (the roofline is reported for
# the dominant one of these; the others mix kernels)
SINGLE_KERNEL = {"SAMPLE", "RNG", "QRCP_WG", "EXTRACT", "TRSM", "SAMPLE_REDUCE"}


def roofline(stats, precision="fp64"):
    name = max((k for k in stats if stats[k]["ms"] > 0 and k in SINGLE_KERNEL), key=lambda k: stats[k]["ms"])
    s = stats[name]
    kern, bound = KCLASS_INFO[name]
    sec = s["ms"] / 1e3
    if bound == "mfma":
        ach = s["flops"] / sec / 1e12
        peak, unit = PEAK_FP64_TFLOPS, "TFLOP/s"
        if name == "SAMPLE" and precision != "fp64":
            # FP32 MFMA, or bf16 MFMA (three bf16 products per algorithmic flop)
            kern = "k_sample_lp"
            peak = PEAK_FP32_TFLOPS if precision == "fp32" else PEAK_BF16_TFLOPS
    else:
        ach = s["bytes"] / sec / 1e9
        peak, unit = PEAK_HBM_GBS, "GB/s"
    return {"bound": bound, "achieved": round(ach, 3), "peak": peak, "unit": unit,
            "frac": round(ach / peak, 5), "traffic": None, "kernel": kern, "class": name,
            "launches": s["launches"], "avg_launch_us": round(1e3 * s["ms"] / max(1, s["launches"]), 3),
            "share_of_profiled_gpu_time": round(s["ms"] / sum(v["ms"] for v in stats.values()), 4),
            "largest_class": max(stats, key=lambda k: stats[k]["ms"])}


def cpu_baseline(W, d_final, budget_rows=16384):
    """The oracle's sampling of one 64-column increment on `budget_rows` of the
    n rows, scaled to a whole compression: n / budget_rows row blocks per
    increment, d_final / 64 increments.  Counts sampling only, so the figure
    is an upper bound on the oracle's compressions/s."""
    import numpy as np
    from threadpoolctl import threadpool_info

    from oracle.operators import Gauss, Laplace, PermutedOperator, Toeplitz
    from oracle.tree import build_tree
    from paper_1810_04125_amd import inputs

    n = W["n"]
    if W["family"] == "laplace":
        pts = inputs.sphere_points(n, W["points_seed"])
        ot = build_tree(n, W["leaf"], pts, W["method"])
        op = PermutedOperator(Laplace(pts), ot.perm, block=512)
    elif W["family"] == "gauss":
        pts = inputs.cube_points(n, W["points_seed"])
        ot = build_tree(n, W["leaf"], pts, W["method"])
        op = PermutedOperator(Gauss(pts, W["sigma"], 1e-2), ot.perm, block=512)
    else:
        ot = build_tree(n, W["leaf"])
        op = PermutedOperator(Toeplitz(n, W["h"]), ot.perm, block=512)
    rows = min(n, budget_rows)
    R = inputs.gaussian_matrix(n, 64, 0)
    cols = np.arange(n)
    t0 = time.perf_counter()
    for i0 in range(0, rows, op.block):
        blk = op.extract(np.arange(i0, min(rows, i0 + op.block)), cols)
        _ = blk @ R
    el = time.perf_counter() - t0
    est = el * (n / rows) * (d_final / 64.0)
    threads = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    return {"value": 1.0 / est, "unit": "compressions/s", "cores": threads, "kind": "oracle",
            "sample": ("oracle dense-block sampling of one 64-column increment on %d of %d rows "
                       "(%.1f s), scaled by %d/%d rows and d_final/64 = %d increments; sampling "
                       "only, so an upper bound on the oracle's rate" %
                       (rows, n, el, n, rows, d_final // 64))}


def setup(W):
    """(generator, tree, R) of a workload on the device; R = None: the
    library draws it from the seed (the workload's r_seed, else 0)."""
    import numpy as np
    import torch

    from paper_1810_04125_amd import hss, inputs

    n = W["n"]
    if W["family"] == "laplace":
        pts = inputs.sphere_points(n, W["points_seed"])
        T = hss.Tree(n, W["leaf"], pts, W["method"])
        gen = hss.laplace(torch.from_numpy(pts).cuda())
    elif W["family"] == "gauss":
        pts = inputs.cube_points(n, W["points_seed"])
        T = hss.Tree(n, W["leaf"], pts, W["method"])
        gen = hss.gauss(torch.from_numpy(pts).cuda(), W["sigma"], 1e-2)
    else:
        T = hss.Tree(n, W["leaf"])
        gen = hss.toeplitz(n, W["h"])
    return gen, T, None


def probe_error(gen, T, H, n):
    """(error, kind): exact ||A - H||_F / ||A||_F for n <= 8192, else the
    64-probe estimate ||(A - H) W||_F / ||A W||_F."""
    import numpy as np
    import torch

    from paper_1810_04125_amd import hss, inputs

    if n <= 8192:
        return H.rel_error(), "exact"
    Om = hss.colmajor(torch.from_numpy(np.ascontiguousarray(inputs.gaussian_matrix(n, 64, 7).T)).cuda().t())
    perm = torch.from_numpy(T.perm).cuda()
    inv = torch.empty_like(perm)
    inv[perm] = torch.arange(n, device=perm.device)
    AO = hss.sample(gen, perm, hss.colmajor(Om[perm]))[inv]      # A_hat (P Om), back to original order
    HO = H.matvec(Om)
    return float(torch.linalg.norm(AO - HO) / torch.linalg.norm(AO)), "64-probe estimate"


def timed(fn, steps, warmup, log, tag):
    import torch
    for i in range(warmup):
        fn()
        log("bench: %s warmup %d done" % (tag, i))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        out = fn()
    torch.cuda.synchronize()
    return out, time.perf_counter() - t0


def main_batch(args, W, log):
    """Throughput of hss_compress_batched over the 256-matrix batch."""
    import torch

    from paper_1810_04125_amd import hss, inputs

    specs = inputs.batch_problems(W["batch"], W["seed"], W["n_lo"], W["n_hi"])
    gens, trees = [], []
    for sp in specs:
        if sp["family"] == "toeplitz":
            gens.append(hss.toeplitz(sp["n"], sp["h"]))
            trees.append(hss.Tree(sp["n"], W["leaf"]))
        else:
            pts = inputs.sphere_points(sp["n"], sp["points_seed"])
            gens.append(hss.laplace(torch.from_numpy(pts).cuda()))
            trees.append(hss.Tree(sp["n"], W["leaf"], pts, "rcb"))
    Rs = None   # each problem draws R on the device from seed 0
    kw = dict(rtol=args.rtol, atol=1e-12, eta=ETA, strategy=W["strategy"], d0=W["d0"], delta_d=W["delta_d"],
              d_max=[min(W["d_max"], sp["n"]) for sp in specs], precision=args.precision)
    log("bench: batch of %d, sum n^2 = %.3e" % (len(specs), sum(sp["n"] ** 2 for sp in specs)))

    def step():
        return hss.compress_batched(gens, trees, Rs, **kw)

    (Hs, st), el = timed(step, args.steps, args.warmup, log, "batch")
    infos = [H.info() for H in Hs]
    pick = list(range(0, len(Hs), max(1, len(Hs) // 8)))
    errs = [Hs[i].rel_error() for i in pick]
    log("bench: %d steps in %.3f s; errors %s" % (args.steps, el, ["%.2e" % e for e in errs]))
    rl = None
    if not args.no_profile:
        del Hs
        Hp, _ = hss.compress_batched(gens, trees, Rs, profile=True, **kw)
        stats = Hp[0].kernel_stats()
        rl = roofline(stats, args.precision)
        rl["profiled_gpu_ms_by_class"] = {k: round(v["ms"], 2) for k, v in stats.items()}
        rl["note"] = "kernel statistics of the first memory group of the batch"
        del Hp
    cpu = None
    if not args.no_cpu:
        # oracle sampling rate on one Laplace problem of the batch, scaled to every problem's 2 n^2 d_final
        Wl = dict(family="laplace", n=8192, leaf=W["leaf"], method="rcb", points_seed=1)
        one = cpu_baseline(Wl, 64, budget_rows=8192)
        sec_per_flop = (1.0 / one["value"]) / (2.0 * 8192 * 8192 * 64)
        total = sum(2.0 * sp["n"] ** 2 * inf["d_final"] for sp, inf in zip(specs, infos)) * sec_per_flop
        cpu = {"value": len(specs) / total, "unit": "compressions/s", "cores": one["cores"], "kind": "oracle",
               "sample": "oracle dense-block Laplace sampling rate (one 64-column increment, n = 8192), "
                         "scaled to sum over the batch of 2 n^2 d_final; sampling only, an upper bound"}
    value = args.steps * len(specs) / el
    out = {
        "metric": METRIC, "value": round(value, 4), "unit": "compressions/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(1e3 * el / args.steps, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f64 (sampling %s)" % args.precision,
        "data": "synthetic",
        "config": {"workload": args.workload, "matrices": len(specs), "n_range": [W["n_lo"], W["n_hi"]],
                   "leaf": W["leaf"], "strategy": W["strategy"], "d0": W["d0"], "rtol": args.rtol,
                   "atol": 1e-12, "eta": ETA, "d_max": W["d_max"], "sampling": args.precision},
        "rel_err_max_of_8": max(errs), "rel_err_ok": bool(max(errs) <= args.rtol), "status": st,
        "rounds_max": max(i["rounds"] for i in infos), "d_final_max": max(i["d_final"] for i in infos),
        "roofline": rl, "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


def copy_calibration():
    """A plain copy of known size: 1 GiB read and 1 GiB written per launch.
    Under rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE its counters give the
    factor that turns the counters of other kernels into bytes."""
    import torch
    a = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": a.numel() * 8, "copy_bytes_written": b.numel() * 8, "launches": 3}))


def lowrank_plus_identity(n, r, seed):
    """A = I + U D V^T in HBM, column-major (the synthetic problem of the
    paper's adaptivity experiments, Sec. 5.3: alpha = beta = 1): U and V
    with orthonormal columns (QR of seeded Gaussian matrices, on the GPU)
    and D_kk = 2^(-53 (k-1) / r), k = 1..r."""
    import torch

    from paper_1810_04125_amd import hss, inputs

    U = torch.linalg.qr(torch.from_numpy(inputs.gaussian_matrix(n, r, seed)).cuda())[0]
    V = torch.linalg.qr(torch.from_numpy(inputs.gaussian_matrix(n, r, seed + 1)).cuda())[0]
    D = torch.pow(2.0, -53.0 * torch.arange(r, dtype=torch.float64, device="cuda") / r)
    At = (V * D) @ U.t()              # A^T row-major = A column-major
    At.diagonal().add_(1.0)
    del U, V
    return hss.dense(At.t(), symmetric=False)


def dense_sampling_rate(gen, T, R, log, reps=5):
    """The dense-matrix sampling kernel alone: S = A_hat R(:, 0:64), A read
    from HBM once per call (8 n^2 bytes, 2 n^2 64 flops), best of `reps`."""
    import torch

    from paper_1810_04125_amd import hss

    n = T.n
    perm = torch.from_numpy(T.perm).cuda()
    R64 = hss.colmajor(R[:, :64])
    hss.sample(gen, perm, R64)
    best = float("inf")
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        hss.sample(gen, perm, R64)
        torch.cuda.synchronize()
        best = min(best, time.perf_counter() - t0)
    gbs = 8.0 * n * n / best / 1e9
    tfs = 2.0 * n * n * 64 / best / 1e12
    log("bench: dense sampling n %d, 64 columns: %.3f ms, %.0f GB/s, %.1f TFLOP/s" % (n, best * 1e3, gbs, tfs))
    return {"columns": 64, "ms": round(best * 1e3, 4), "achieved_GBps": round(gbs, 1), "hbm_peak_GBps": 8000.0,
            "frac_hbm": round(gbs / 8000.0, 4), "achieved_tflops": round(tfs, 2), "fp64_peak_tflops": 78.6,
            "frac_fp64": round(tfs / 78.6, 4), "note": "host-timed single call, launch included"}


def table_run(gen, T, R, log, tag, exact, **kw):
    """One compression of a table cell: time, status, error, HSS rank, rounds."""
    import torch

    from paper_1810_04125_amd import hss

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    H, st = hss.compress(gen, T, R, **kw)
    torch.cuda.synchronize()
    sec = time.perf_counter() - t0
    inf = H.info()
    err, kind = (H.rel_error(), "exact") if exact else probe_error(gen, T, H, T.n)
    log("bench: %s %s: %.3g s, status %d, err %.3g, rank %d, rounds %d, d %d" % (
        tag, {k: kw[k] for k in ("strategy", "rtol", "atol", "d0", "d_max") if k in kw}, sec, st, err,
        inf["hss_rank"], inf["rounds"], inf["d_final"]))
    return {"sec": round(sec, 4), "status": st, "rel_err": err, "err_kind": kind, "hss_rank": inf["hss_rank"],
            "rounds": inf["rounds"], "d_final": inf["d_final"]}


def main_table(args, log):
    """Synthetic analogues of the paper's adaptivity tables on A = I + U D V^T
    (dense in HBM, sampled by the library's dense-matrix kernel).

    hmt: n = 20000, r = 200.  The F-norm test (incrementing, d0 = 128,
    delta_d = 64) over rtol x atol in {1e-2, 1e-6, 1e-10, 1e-14}^2 and the
    HMT-lemma test (eq. HMT_IQQH, alpha = 10, p = delta_d) over atol, with
    the paper's literal per-node tolerance (eta = 1) and d_max = 4096;
    exact errors ||A - H||_F / ||A||_F.

    adaptive-rank: n = 60000, r = 1200, rtol = atol = 1e-10 (with the
    literal per-node tolerance eps / level, 1e-14 lies below the FP64
    rounding floor of samples summed over 60000 terms, and 1e-12 within a
    few times of it, where test outcomes follow rounding).  "Known rank"
    (one round with d0 = the incrementing run's HSS rank + 64), the
    incrementing strategy (d0 = 128, delta_d = 64 and d0 = 512,
    delta_d = 128), and "hard restart" (compressions from scratch at
    d = d0, 2 d0, ... with d_max = d, until the error of one is within
    the requested tolerance); 64-probe error estimates.  With d_max = d0
    the stopping test of the first round fails at a few nodes and the
    second round accepts them (status NOT_CONVERGED): "known rank" and
    every restart sample once and include that test work."""
    import numpy as np
    import torch

    from paper_1810_04125_amd import hss, inputs

    out = {"table": args.table, "data": "synthetic", "matrix": "I + U D V^T, D_kk = 2^(-53(k-1)/r)"}
    if args.table == "hmt":
        n, r, dmax = 20000, 200, 4096
    else:
        n, r, dmax = 60000, 1200, 4096
    gen = lowrank_plus_identity(n, r, 11)
    T = hss.Tree(n, 128)
    Rh = inputs.gaussian_matrix(n, dmax, 12)
    R = hss.colmajor(torch.from_numpy(np.ascontiguousarray(Rh.T)).cuda().t())
    del Rh
    out.update({"n": n, "r": r, "leaf": 128, "tree": "bisect"})
    out["dense_sampling"] = dense_sampling_rate(gen, T, R, log)
    if args.table == "hmt":
        tols = [1e-2, 1e-6, 1e-10, 1e-14]
        base = dict(eta=1.0, d0=128, delta_d=64, d_max=dmax)
        grid = {}
        for rt in tols:
            for at in tols:
                grid["rtol=%g,atol=%g" % (rt, at)] = table_run(gen, T, R, log, "fnorm", True, rtol=rt, atol=at,
                                                               strategy="inc_fnorm", **base)
        hmt = {}
        for at in tols:
            hmt["atol=%g" % at] = table_run(gen, T, R, log, "hmt", True, rtol=0.0, atol=at, strategy="inc_hmt",
                                            hmt_alpha=10.0, **base)
        out.update({"strategy": "inc_fnorm d0=128 delta_d=64 eta=1", "fnorm": grid,
                    "hmt_lemma": hmt, "hmt_alpha": 10.0, "d_max": dmax})
    else:
        kw = dict(rtol=1e-10, atol=1e-10, eta=1.0)
        res = {}
        for d0, dd in ((128, 64), (512, 128)):
            key = "d0=%d,delta_d=%d" % (d0, dd)
            inc = table_run(gen, T, R, log, "inc " + key, False, strategy="inc_fnorm", d0=d0, delta_d=dd,
                            d_max=dmax, **kw)
            inc["adaptations"] = inc["rounds"] - 1
            dk = min(dmax, inc["hss_rank"] + 64)
            known = table_run(gen, T, R, log, "known rank", False, strategy="inc_fnorm", d0=dk, delta_d=dd,
                              d_max=dk, **kw)
            known["d"] = dk
            known["adaptations"] = 0
            hard, d, total = [], d0, 0.0
            while True:
                c = table_run(gen, T, R, log, "hard restart", False, strategy="inc_fnorm", d0=d, delta_d=dd,
                              d_max=d, **kw)
                c["d"] = d
                hard.append(c)
                total += c["sec"]
                if c["rel_err"] <= kw["rtol"] or d >= dmax:
                    break
                d = min(2 * d, dmax)
            res[key] = {"known_rank": known, "inc": inc,
                        "hard_restart": {"sec": round(total, 4), "adaptations": len(hard) - 1,
                                         "hss_rank": hard[-1]["hss_rank"], "rel_err": hard[-1]["rel_err"],
                                         "runs": hard}}
        out.update({"rtol": 1e-10, "atol": 1e-10, "eta": 1.0, "results": res})
    print(json.dumps(out))


def run_once(W, gen, T, kw, steps, warmup, log, tag):
    """Time `steps` compressions of one workload (after `warmup`), then check
    the error of the last one.  Returns (H, status, seconds, summary)."""
    from paper_1810_04125_amd import hss
    (H, st), el = timed(lambda: hss.compress(gen, T, None, **kw), steps, warmup, log, tag)
    info = H.info()
    err, kind = probe_error(gen, T, H, W["n"])
    summ = {"compressions_per_s": round(steps / el, 4), "ms_per_step": round(1e3 * el / steps, 3),
            "rel_err": err, "rel_err_kind": kind, "rel_err_ok": bool(err <= kw["rtol"]), "status": st,
            "rounds": info["rounds"], "d_final": info["d_final"], "hss_rank": info["hss_rank"]}
    log("bench: %s %s" % (tag, json.dumps(summ)))
    return H, st, el, summ


def mixed_leg(args, log):
    """Sampling in FP32 and BF16x3 against FP64 on the Gaussian-kernel
    workload (n = 65536, kd tree, leaf 256, incrementing d0 = 128), at rtol
    1e-6 and 1e-4: compressions/s, error and status of each."""
    W = WORKLOADS["gauss-cube-65536"]
    gen, T, _ = setup(W)
    out = {"workload": "gauss-cube-65536", "steps": args.leg_steps}
    for rtol in (1e-6, 1e-4):
        row = {}
        for prec in ("fp64", "fp32", "bf16x3"):
            kw = dict(rtol=rtol, atol=1e-12, eta=ETA, strategy=W["strategy"], d0=W["d0"], delta_d=W["delta_d"],
                      d_max=W["d_max"], precision=prec, seed=0)
            H, st, el, summ = run_once(W, gen, T, kw, args.leg_steps, 1, log, "mixed %s rtol %g" % (prec, rtol))
            row[prec] = summ
            del H
        for prec in ("fp32", "bf16x3"):
            row[prec]["speedup_vs_fp64"] = round(row[prec]["compressions_per_s"] / row["fp64"]["compressions_per_s"], 3)
        out["rtol=%g" % rtol] = row
    return out


def learned_leg(args, name, log):
    """Learned d0 (the predictor network run inside hss_compress) against the
    adaptive start d0 = 128 on one workload: compressions/s, rounds saved and
    the rank-prediction error per tree level."""
    import numpy as np

    from paper_1810_04125_amd import hss
    from paper_1810_04125_amd.learned import D0Predictor
    W = WORKLOADS[name]
    gen, T, _ = setup(W)
    n = W["n"]
    kw = dict(rtol=args.rtol, atol=1e-12, eta=ETA, strategy=W["strategy"], d0=W["d0"], delta_d=W["delta_d"],
              d_max=W["d_max"], seed=W.get("r_seed", 0))
    pred = D0Predictor()
    Hl, stl, ell, sl = run_once(W, gen, T, dict(kw, predictor=pred.handle()), args.leg_steps, 1, log,
                                "learned %s" % name)
    Hb, stb, elb, sb = run_once(W, gen, T, kw, args.leg_steps, 1, log, "adaptive %s" % name)
    param = W.get("h", W.get("sigma"))
    p = pred.predict(W["family"], param, n, T, args.rtol)
    act = np.zeros(int(T.level.max()) + 1)
    for node in range(T.num_nodes):
        ni = Hb.node_info(node)
        act[T.level[node]] = max(act[T.level[node]], ni["rank_r"], ni["rank_c"])
    lr_pred = np.array(p["level_rank"])
    return {"workload": name, "steps": args.leg_steps, "learned": sl, "adaptive": sb,
            "d0_learned": Hl.info()["d0"], "d0_adaptive": W["d0"],
            "speedup": round(sb["ms_per_step"] / sl["ms_per_step"], 3),
            "rounds_saved": sb["rounds"] - sl["rounds"],
            "d_final_predicted": round(p["d_final"], 1),
            "d_final_pred_rel_err": round(p["d_final"] / sb["d_final"] - 1.0, 4),
            "level_rank_predicted": [round(x, 1) for x in lr_pred],
            "level_rank_actual": [int(x) for x in act[1:]],
            "rank_pred_mae_log2": round(float(np.mean(np.abs(np.log2(1 + lr_pred) - np.log2(1 + act[1:])))), 4)}


def ulv_leg(H, T, args, log):
    """The direct factorization and solve of the bench's compressed matrix
    (hss_factor, hss_solve): time of one factorization, of solves with 1 and
    64 right-hand sides, algorithmic flops against the FP64 peak, and the
    residual through H.  Per node (m = leaf size or children's ranks, r its
    rank, k = m - r; the root r = 0): the basis transforms 4 r k (r + k)
    flops, the LU of the first k columns 2/3 (m^3 - (m - k)^3); a solve
    about 4 m k + 4 r k flops per right-hand side."""
    import torch

    from paper_1810_04125_amd import hss, inputs
    n = T.n
    ranks = [H.node_info(t)["rank_r"] if T.parent[t] >= 0 else 0 for t in range(T.num_nodes)]
    fflops = sflops = fbytes = 0.0
    for t in range(T.num_nodes):
        m = float(T.hi[t] - T.lo[t] if T.left[t] < 0 else ranks[T.left[t]] + ranks[T.right[t]])
        r = float(ranks[t])
        k = m - r
        fflops += 4.0 * r * k * (r + k) + 2.0 / 3.0 * (m ** 3 - (m - k) ** 3)
        sflops += 4.0 * m * k + 4.0 * r * k
        fbytes += 8.0 * m * m
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    H.factor()
    torch.cuda.synchronize()
    fsec = time.perf_counter() - t0
    out = {"factor_ms": round(1e3 * fsec, 2), "factor_alg_gflop": round(fflops / 1e9, 2),
           "factor_tflops": round(fflops / fsec / 1e12, 3),
           "factor_frac_fp64_peak": round(fflops / fsec / 1e12 / PEAK_FP64_TFLOPS, 4),
           "factor_gbytes": round(fbytes / 1e9, 3)}
    for nrhs in (1, 64):
        B = hss.colmajor(torch.from_numpy(inputs.gaussian_matrix(n, nrhs, 17)).cuda())
        X = H.solve(B)   # warm-up
        torch.cuda.synchronize()
        reps = 5
        t0 = time.perf_counter()
        for _ in range(reps):
            X = H.solve(B)
        torch.cuda.synchronize()
        ssec = (time.perf_counter() - t0) / reps
        res = float(torch.linalg.norm(H.matvec(X) - B) / torch.linalg.norm(B))
        out["solve_ms_nrhs%d" % nrhs] = round(1e3 * ssec, 3)
        out["solve_tflops_nrhs%d" % nrhs] = round(sflops * nrhs / ssec / 1e12, 4)
        out["residual_through_H_nrhs%d" % nrhs] = res
    log("bench: ulv %s" % json.dumps(out))
    return out


def id_roofline(stats):
    """The per-level ID (rows a6-a8 of the method): its algorithmic work as the
    method defines it (class ID: 4 d m r flops, 8 d m + 8 r (m - r) bytes per
    factored panel) over the GPU time of the kernels that ran it."""
    ms = sum(stats[c]["ms"] for c in ("QRCP_STEP", "QRCP_WG", "QRCP_OTHER", "TRSM"))
    idc = stats["ID"]
    sec = ms / 1e3
    if sec <= 0:
        return None
    tf = idc["flops"] / sec / 1e12
    gb = idc["bytes"] / sec / 1e9
    return {"kernels": "k_idb_* + block GEMMs, k_qrcp_wg/step (small or very wide panels), "
                       "k_qrcp_plan/init/alive/fin/count, k_trsm_diag",
            "id_calls": idc["launches"], "ms": round(ms, 2), "alg_tflop": round(idc["flops"] / 1e12, 4),
            "alg_gb": round(idc["bytes"] / 1e9, 3), "achieved_tflops": round(tf, 3),
            "frac_fp64_peak": round(tf / PEAK_FP64_TFLOPS, 5), "achieved_GBps": round(gb, 1),
            "frac_hbm_peak": round(gb / PEAK_HBM_GBS, 5)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=8)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="laplace-sphere-32768", choices=sorted(WORKLOADS))
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32", "bf16x3"],
                    help="arithmetic of the sampling product (everything else is FP64)")
    ap.add_argument("--rtol", type=float, default=1e-6)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-profile", action="store_true")
    ap.add_argument("--no-legs", action="store_true",
                    help="skip the factorization, mixed-precision and learned-d0 legs of the default line")
    ap.add_argument("--legs", default="all", choices=["all", "ulv", "none"],
                    help="legs of the default line: all, only the factorization and solve, or none")
    ap.add_argument("--leg-steps", type=int, default=3)
    ap.add_argument("--tunables", default=TUNE_FILE,
                    help="launch-shape table written by the autotuner ('none': the built-in shapes)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a device-to-device copy of 1 GiB three times (reference for HBM counters)")
    ap.add_argument("--table", choices=["hmt", "adaptive-rank"],
                    help="synthetic analogue of the paper's stopping-criterion or adaptivity-cost table "
                         "(one JSON line with the whole table instead of the bench line)")
    args = ap.parse_args()
    if args.copy_calibration:
        return copy_calibration()
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (run with --gpus 1)",
              file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1810_04125_amd import hss

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    if args.no_legs:
        args.legs = "none"
    W = WORKLOADS[args.workload]
    log = lambda m: print(m, file=sys.stderr, flush=True)
    tune_file = None
    if args.tunables != "none" and os.path.exists(args.tunables):
        hss.load_tunables(args.tunables)
        tune_file = os.path.relpath(args.tunables, ROOT)
        log("bench: launch shapes from %s" % tune_file)
    if args.table:
        return main_table(args, log)
    if W.get("batch"):
        return main_batch(args, W, log)
    if W.get("learned"):
        print(json.dumps(learned_leg(args, args.workload, log)), flush=True)
        return
    n = W["n"]
    log("bench: workload %s precision %s rtol %g" % (args.workload, args.precision, args.rtol))
    gen, T, _ = setup(W)
    kw = dict(rtol=args.rtol, atol=1e-12, eta=ETA, strategy=W["strategy"], d0=W["d0"], delta_d=W["delta_d"],
              d_max=W["d_max"], precision=args.precision, seed=W.get("r_seed", 0))
    (H, st), el = timed(lambda: hss.compress(gen, T, None, **kw), args.steps, args.warmup, log,
                        args.precision)
    info = H.info()
    log("bench: timed %d steps in %.3f s; info %s" % (args.steps, el, info))
    err, kind = probe_error(gen, T, H, n)
    log("bench: rel err %.3e (%s)" % (err, kind))
    ulv = None
    if args.legs in ("all", "ulv") and args.precision == "fp64" and args.workload == "laplace-sphere-32768":
        ulv = ulv_leg(H, T, args, log)
    del H

    rl = None
    if not args.no_profile:
        Hp, _ = hss.compress(gen, T, None, profile=True, **kw)
        stats = Hp.kernel_stats()
        rl = roofline(stats, args.precision)
        rl["traffic"] = traffic_bytes(args.workload, rl["class"])
        rl["traffic_unit"] = "bytes per launch (HBM, measured)"
        rl["algorithmic_per_launch"] = {"flops": round(stats[rl["class"]]["flops"] / max(1, rl["launches"]), 1),
                                        "bytes": round(stats[rl["class"]]["bytes"] / max(1, rl["launches"]), 1)}
        samp = stats["SAMPLE"]
        skern = "k_sample_f64" if args.precision == "fp64" else "k_sample_lp"
        speak = {"fp64": PEAK_FP64_TFLOPS, "fp32": PEAK_FP32_TFLOPS, "bf16x3": PEAK_BF16_TFLOPS}[args.precision]
        mult = 3.0 if args.precision == "bf16x3" else 1.0   # BF16x3: three bf16 products per product
        stf = samp["flops"] / (samp["ms"] / 1e3) / 1e12
        rl["sampling_kernel"] = {"kernel": skern, "launches": samp["launches"],
                                 "achieved_tflops": round(stf, 3),
                                 "mfma_tflops": round(mult * stf, 3),
                                 "frac_of_peak": round(mult * stf / speak, 4), "peak_tflops": speak,
                                 "avg_launch_us": round(1e3 * samp["ms"] / max(1, samp["launches"]), 3),
                                 "counters": sample_counters(args.workload, args.precision)}
        rl["id"] = id_roofline(stats)
        rl["profiled_gpu_ms_by_class"] = {k: round(v["ms"], 2) for k, v in stats.items()}
        log("bench: profile %s" % json.dumps(rl))
        del Hp

    legs = {}
    if args.legs == "all" and args.workload == "laplace-sphere-32768" and args.precision == "fp64":
        legs["mixed"] = mixed_leg(args, log)
        legs["learned"] = [learned_leg(args, nm, log) for nm in ("learned-laplace-sphere-65536",
                                                                 "learned-toeplitz-131072")]

    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(W, info["d_final"])
        log("bench: cpu baseline %s" % cpu)

    value = args.steps / el
    cfg = {"workload": args.workload, "n": n, "leaf": W["leaf"], "tree": W["method"],
           "strategy": W["strategy"], "d0": W["d0"], "delta_d": W["delta_d"],
           "rtol": args.rtol, "atol": 1e-12, "eta": ETA, "d_max": W["d_max"],
           "sampling": args.precision, "r": "device Philox4x64-10 + Box-Muller, seed %d" % W.get("r_seed", 0),
           "tunables": tune_file or "built-in"}
    out = {
        "metric": METRIC, "value": round(value, 4), "unit": "compressions/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(1e3 * el / args.steps, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f64 (sampling %s)" % args.precision,
        "data": "synthetic", "config": cfg,
        "rel_err": err, "rel_err_kind": kind, "rel_err_ok": bool(err <= args.rtol), "status": st,
        "sampling_tflops": round(info["sample_flops"] / (info["sample_ms"] / 1e3) / 1e12, 3),
        "rounds": info["rounds"], "d_final": info["d_final"], "hss_rank": info["hss_rank"],
        "roofline": rl, "cpu_baseline": cpu,
    }
    if ulv:
        out["ulv"] = ulv
    out.update(legs)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
