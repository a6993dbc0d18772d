#!/usr/bin/env python3
"""Benchmark of the leaf-level residual interaction on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload laplace_n1m]

One step = the forward (strength gather into the sorted order + pair kernel)
and the adjoint (cotangent gather + adjoint pair kernel, reusing the
forward's sorted strengths) of the whole workload, with the points already
binned and all inputs resident in HBM.  The binning (the paper's tree
construction, which its timings exclude) is timed on its own and reported as
bin_ms, and the end-to-end autograd step (bin + forward + backward through
DmkResidual) beside it.  The headline is the FP32-compensated path on
laplace_n1m; the FP64 path is timed the same way, and every other workload
of the metric's configuration list gets its own object in the line.

Metric: in-cutoff ordered pair interactions (0 < r < rc, P_in) per second of
forward + backward.  Prints ONE JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from paper_2606_27134_amd import workloads as W  # noqa: E402

METRIC = "residual pair-interactions/s fwd+bwd, FP32-compensated vs FP64 at stated rel err"

# Floating-point operations per in-cutoff pair of the pair step as compiled
# for gfx950 (distance from the staged coordinates, cutoff test, residual
# kernel or its adjoint with the Gaussian window): counted from the ISA of
# the kernels' pair arithmetic, FMA = 2, add / mul = 1, each rsq / rcp / exp
# = 1 (the FP64 exponential is a software sequence of adds and FMAs).  The
# FP64 accumulation into the target's sum runs in the LDS unit and is not
# counted.
FLOPS_PER_PAIR = {
    ("laplace", "fp32c", "fwd"): 44, ("laplace", "fp32c", "bwd"): 58,
    ("stokeslet", "fp32c", "fwd"): 67, ("stokeslet", "fp32c", "bwd"): 146,
    ("stresslet", "fp32c", "fwd"): 113, ("stresslet", "fp32c", "bwd"): 399,
    ("rotlet", "fp32c", "fwd"): 61, ("rotlet", "fp32c", "bwd"): 107,
    ("laplace", "fp64", "fwd"): 128, ("laplace", "fp64", "bwd"): 142,
    ("stokeslet", "fp64", "fwd"): 151, ("stokeslet", "fp64", "bwd"): 230,
    ("stresslet", "fp64", "fwd"): 196, ("stresslet", "fp64", "bwd"): 482,
    ("rotlet", "fp64", "fwd"): 145, ("rotlet", "fp64", "bwd"): 191,
}
# MI355X published vector peaks (TFLOP/s).  FP32 157.3 needs packed FP32
# instructions, which this build keeps out of the generated code; one
# unpacked FP32 (or FP64) instruction per lane per cycle is 78.6.
PEAK_TFLOPS = {"fp32c": 157.3, "fp64": 78.6}
PEAK_UNPACKED_TFLOPS = 78.6
# PSWF bandwidth c for a requested tolerance 1e-6 (the paper's parameter
# tables for the Laplace and Stokes kernels)
PSWF_C_1E6 = {"laplace": 14.5, "stokeslet": 17.80, "stresslet": 17.80, "rotlet": 13.61}
HBM_PEAK_GBS = 8000.0
# the workloads of the metric's configuration list, beside the headline:
# (label, workload, kernel)
CONFIGS = [("laplace_n2k", "laplace_n2k", None),
           ("stokeslet_n500k_clustered", "stokeslet_n500k_clustered", None),
           ("stresslet_n2m_rod", "stokes_n2m_rod", "stresslet"),
           ("rotlet_n2m_rod", "stokes_n2m_rod", "rotlet")]


def count_pairs(w, targets=None):
    """Ordered in-cutoff pairs (0 < r < rc) over the images of the first D axes."""
    from scipy.spatial import cKDTree
    L = np.asarray(w.L, dtype=np.float64)
    box = np.array([L[i] if i < w.D else 2.0 * L[i] + 4.0 * w.rc for i in range(3)])
    x = np.mod(w.x, L) if w.D == 3 else w.x.copy()
    for i in range(w.D):
        x[:, i] = np.mod(w.x[:, i], L[i])
        x[:, i] = np.where(x[:, i] >= L[i], 0.0, x[:, i])
    tree = cKDTree(x, boxsize=box)
    if targets is None:
        return int(tree.count_neighbors(tree, w.rc)) - len(x)
    q = cKDTree(x[targets], boxsize=box)
    return int(q.count_neighbors(tree, w.rc)) - len(targets)


def count_candidates(w):
    """Candidate pairs P_cand: for every target, the points of its own leaf box
    and its 26 neighbours (images across periodic faces), itself included --
    the stencil the pair kernels scan.  Box counts from the points on the
    host; a neighbour beyond a free face is empty."""
    L = np.asarray(w.L, dtype=np.float64)
    n = np.asarray(w.n)
    b = np.empty((w.N, 3), dtype=np.int64)
    for i in range(3):
        y = np.mod(w.x[:, i], L[i]) if i < w.D else w.x[:, i]
        b[:, i] = np.minimum(n[i] - 1, np.floor(y * (n[i] / L[i])).astype(np.int64))
    cnt = np.bincount((b[:, 0] * n[1] + b[:, 1]) * n[2] + b[:, 2], minlength=int(np.prod(n))).reshape(n)
    S = cnt.astype(np.int64)
    for i in range(3):
        T = S.copy()
        for d in (-1, 1):
            if i < w.D:
                T += np.roll(S, d, axis=i)
            else:
                sh = np.zeros_like(S)
                src = [slice(None)] * 3
                dst = [slice(None)] * 3
                src[i] = slice(max(0, -d), n[i] - max(0, d))
                dst[i] = slice(max(0, d), n[i] - max(0, -d))
                sh[tuple(dst)] = S[tuple(src)]
                T += sh
        S = T
    return int((cnt * S).sum())


def kernel_hash():
    """Hash of the sources that k_residual is built from (the counter-based
    traffic applies only while they are unchanged)."""
    h = hashlib.sha256()
    for f in ("paper_2606_27134_amd/csrc/dmk_residual.hip", "paper_2606_27134_amd/csrc/dmk_internal.h",
              "paper_2606_27134_amd/csrc/dmk_dpp.h",
              "paper_2606_27134_amd/csrc/erfcx_f32.h", "paper_2606_27134_amd/csrc/erfcx_f64.h", "include/dmk.h"):
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def read_traffic(workload, prec, khash, field=None):
    """HBM bytes per launch (or, with field, another per-launch counter figure)
    from the committed rocprofv3 counter summary, if it was taken on the
    current kernel sources."""
    path = os.path.join(ROOT, "profiles", "traffic_%s.json" % workload)
    if not os.path.exists(path):
        return None
    try:
        d = json.load(open(path))
    except Exception:
        return None
    if d.get("kernel_hash") != khash:
        return None
    if field is not None:
        return d.get(field, {}).get(prec)
    return d.get(prec)


def _omp_threads(n):
    """Set the OpenMP thread count of this process (the oracle's runtime)."""
    import ctypes
    try:
        ctypes.CDLL("libgomp.so.1").omp_set_num_threads(int(n))
        return True
    except OSError:
        return False


def cpu_baseline(w, budget_s=15.0):
    """The oracle (fwd + vjp, O(N^2) brute force) on a bounded sample of
    targets of the same workload, on all host cores and on one core."""
    import oracle
    oracle.build()
    rng = np.random.default_rng(123)
    G = W.cotangent(w.seed, w.N, W.M_OUT[w.kernel])
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    cores = min(cores, os.cpu_count() or cores)
    _omp_threads(cores)
    n_try = 2 * cores
    t = np.sort(rng.choice(w.N, size=n_try, replace=False))
    t0 = time.perf_counter()
    oracle.residual(w.kernel, w.D, w.L, w.sigma, w.rc, w.x, w.rho, targets=t)
    oracle.residual_vjp(w.kernel, w.D, w.L, w.sigma, w.rc, w.x, w.rho, G, targets=t)
    dt = time.perf_counter() - t0
    n = int(max(n_try, min(w.N, n_try * budget_s / max(dt, 1e-3))))
    n = max(cores, (n // cores) * cores)
    t = np.sort(rng.choice(w.N, size=n, replace=False))
    t0 = time.perf_counter()
    u = oracle.residual(w.kernel, w.D, w.L, w.sigma, w.rc, w.x, w.rho, targets=t)
    gr, gx = oracle.residual_vjp(w.kernel, w.D, w.L, w.sigma, w.rc, w.x, w.rho, G, targets=t)
    dt = time.perf_counter() - t0
    # one core, on a sixteenth of the sample
    n1 = max(1, n // 16)
    t1s = t[:n1]
    one = None
    if _omp_threads(1):
        t0 = time.perf_counter()
        oracle.residual(w.kernel, w.D, w.L, w.sigma, w.rc, w.x, w.rho, targets=t1s)
        oracle.residual_vjp(w.kernel, w.D, w.L, w.sigma, w.rc, w.x, w.rho, G, targets=t1s)
        one = time.perf_counter() - t0
        _omp_threads(cores)
    pin = count_pairs(w, targets=t)
    tests = 2.0 * n * w.N  # forward and vjp each test every (target, source) pair
    out = dict(value=pin / dt, unit="pair-interactions/s", cores=cores, kind="oracle",
               label="O(N^2) brute-force reference (long double, every source and image per target), "
                     "not a tuned CPU code",
               sample="%d seeded targets of %s (all %d sources, every image), fwd + vjp, %.1f s on %d cores, "
                      "P_in(sample)=%d" % (n, w.name, w.N, dt, cores, pin),
               pair_tests_per_s=tests / dt, seconds_all_cores=dt, targets=n)
    if one is not None:
        out.update(seconds_one_core=one, targets_one_core=n1,
                   pair_tests_per_s_one_core=2.0 * n1 * w.N / one,
                   seconds_one_core_per_target=one / n1, seconds_all_cores_per_target=dt / n)
    return out, (t, u, gr, gx, G)


def _time_ms(fn, reps, warm=3):
    import torch
    for _ in range(warm):
        fn()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    torch.cuda.synchronize()
    ev[0].record()
    for _ in range(reps):
        fn()
    ev[1].record()
    torch.cuda.synchronize()
    return ev[0].elapsed_time(ev[1]) / reps


def time_residual(w, bins, prec, steps, warmup, pswf_c=None):
    """Time `steps` forward + adjoint steps on the current stream.  Events
    bracket every call: the gathers and the pair kernels, so the pair
    kernels' durations are measured in the timed region itself."""
    import torch
    from paper_2606_27134_amd import residual as R
    k = w.kernel
    dev = "cuda"
    rho = torch.as_tensor(w.rho).to(dev)
    G = torch.as_tensor(W.cotangent(w.seed, w.N, W.M_OUT[k])).to(dev)
    rho_s = torch.empty((W.M_IN[k], w.N), dtype=torch.float64, device=dev)
    gu_s = torch.empty((W.M_OUT[k], w.N), dtype=torch.float64, device=dev)
    u = torch.empty((w.N, W.M_OUT[k]), dtype=torch.float64, device=dev)
    gr = torch.empty((w.N, W.M_IN[k]), dtype=torch.float64, device=dev)
    gx = torch.empty((w.N, 3), dtype=torch.float64, device=dev)
    sig = 0.0 if pswf_c else w.sigma

    def fwd():
        R.gather_sorted(bins, rho, out=rho_s)
        R.residual_eval_sorted(bins, k, prec, sig, w.rc, rho_s, out=u, pswf_c=pswf_c)

    def bwd():
        R.gather_sorted(bins, G, out=gu_s)
        R.residual_backward_sorted(bins, k, prec, sig, w.rc, rho_s, gu_s, out=(gr, gx), pswf_c=pswf_c)

    for _ in range(warmup):
        fwd()
        bwd()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(5)] for _ in range(steps)]
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t_wall = time.perf_counter()
    start.record(stream)
    for s in range(steps):
        e = ev[s]
        e[0].record(stream)
        R.gather_sorted(bins, rho, out=rho_s)
        e[1].record(stream)
        R.residual_eval_sorted(bins, k, prec, sig, w.rc, rho_s, out=u, pswf_c=pswf_c)
        e[2].record(stream)
        R.gather_sorted(bins, G, out=gu_s)
        e[3].record(stream)
        R.residual_backward_sorted(bins, k, prec, sig, w.rc, rho_s, gu_s, out=(gr, gx), pswf_c=pswf_c)
        e[4].record(stream)
    stop.record(stream)
    torch.cuda.synchronize()
    t_wall = time.perf_counter() - t_wall
    ms = start.elapsed_time(stop) / steps
    el = lambda a, b: float(np.mean([ev[s][a].elapsed_time(ev[s][b]) for s in range(steps)]))  # noqa: E731
    med = lambda a, b: float(np.median([ev[s][a].elapsed_time(ev[s][b]) for s in range(steps)]))  # noqa: E731
    res = dict(ms_per_step=ms, fwd_ms=el(0, 2), bwd_ms=el(2, 4), kernel_fwd_ms=el(1, 2), kernel_bwd_ms=el(3, 4),
               gather_fwd_ms=el(0, 1), gather_bwd_ms=el(2, 3), wall_s=t_wall,
               median_ms={"step": med(0, 4), "fwd": med(0, 2), "bwd": med(2, 4), "kernel_fwd": med(1, 2),
                          "kernel_bwd": med(3, 4)})
    outs = (u.cpu().numpy(), gr.cpu().numpy(), gx.cpu().numpy())
    return res, outs


def roofline(kernel, prec, P_in, r, khash=None, workload=None):
    """Roofline of the dominant pair-kernel launch of a step (the longer of
    forward and adjoint): algorithmic flops of the in-cutoff pairs over its
    measured duration, against the vector peak of the precision."""
    dom = "bwd" if r["kernel_bwd_ms"] >= r["kernel_fwd_ms"] else "fwd"
    dur_ms = r["kernel_%s_ms" % dom]
    fpp = FLOPS_PER_PAIR[(kernel, prec, dom)]
    achieved = fpp * P_in / (dur_ms * 1e-3) / 1e12
    roof = {"bound": "alu", "achieved": achieved, "peak": PEAK_TFLOPS[prec], "unit": "TFLOP/s",
            "frac": achieved / PEAK_TFLOPS[prec], "traffic": None,
            "kernel": "k_residual<%s,%s,%s>" % (kernel, prec, dom), "flops_per_pair": fpp, "launch_ms": dur_ms}
    if prec == "fp32c":
        roof["peak_unpacked"] = PEAK_UNPACKED_TFLOPS
        roof["frac_unpacked"] = achieved / PEAK_UNPACKED_TFLOPS
    if khash is not None and workload is not None:
        tr = read_traffic(workload, prec, khash)
        roof["traffic"] = None if tr is None else tr.get(dom)
        vi = read_traffic(workload, prec, khash, field="valu_issue")
        roof["valu_issue_frac"] = None if vi is None else vi.get(dom)
        ex = read_traffic(workload, prec, khash, field="valu_tflops")
        roof["valu_executed_tflops"] = None if ex is None else ex.get(dom)
        lu = read_traffic(workload, prec, khash, field="lane_utilisation")
        roof["valu_lane_utilisation"] = None if lu is None else lu.get(dom)
    return roof


def oracle_errors(w, outs, ntgt=64, seed=321):
    """rel l2 of every result on ntgt seeded targets against the oracle."""
    import oracle
    rng = np.random.default_rng(seed)
    t = np.sort(rng.choice(w.N, size=min(ntgt, w.N), replace=False))
    G = W.cotangent(w.seed, w.N, W.M_OUT[w.kernel])
    u_o = oracle.residual(w.kernel, w.D, w.L, w.sigma, w.rc, w.x, w.rho, targets=t)
    gr_o, gx_o = oracle.residual_vjp(w.kernel, w.D, w.L, w.sigma, w.rc, w.x, w.rho, G, targets=t)

    def rl2(a, b):
        return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))
    errs = {prec: {"u": rl2(u[t], u_o), "grad_rho": rl2(gr[t], gr_o), "grad_x": rl2(gx[t], gx_o)}
            for prec, (u, gr, gx) in outs.items()}
    errs["sample_targets"] = int(len(t))
    return errs


def bench_workload(w, precs, steps, warmup):
    """Binning, P_in and the timed fwd + adjoint steps of one workload."""
    import torch
    from paper_2606_27134_amd import residual as R
    x = torch.as_tensor(w.x).cuda()
    bins = R.Bins(w.L, w.D, w.n, w.N)
    for _ in range(2):
        bins.bin(x)
    torch.cuda.synchronize()
    tb = []  # host clock around each binning (it waits on its stream once)
    for _ in range(11):
        t0 = time.perf_counter()
        bins.bin(x)
        torch.cuda.synchronize()
        tb.append(time.perf_counter() - t0)
    res, outs = {}, {}
    for prec in precs:
        res[prec], outs[prec] = time_residual(w, bins, prec, steps, warmup)
    return bins, 1e3 * float(np.median(tb)), res, outs


def config_object(label, w, P_in, bin_ms, res, errs):
    P_cand = count_candidates(w)
    o = {"workload": "%s: %s D=%d L=%s n=%s N=%d sigma=%.6g rc=%.6g" % (
        w.name, w.kernel, w.D, list(w.L), list(w.n), w.N, w.sigma, w.rc), "P_in": P_in, "P_cand": P_cand,
        "bin_ms": bin_ms}
    for prec, r in res.items():
        o[prec] = {"value": P_in / (r["ms_per_step"] * 1e-3), "value_fwd": P_in / (r["fwd_ms"] * 1e-3),
                   "candidate_pairs_per_s": P_cand / (r["ms_per_step"] * 1e-3), "median_ms": r["median_ms"],
                   "ms_per_step": r["ms_per_step"], "fwd_ms": r["fwd_ms"], "bwd_ms": r["bwd_ms"],
                   "kernel_fwd_ms": r["kernel_fwd_ms"], "kernel_bwd_ms": r["kernel_bwd_ms"],
                   "roofline": roofline(w.kernel, prec, P_in, r)}
    if "fp32c" in res and "fp64" in res:
        o["fp32c_speedup_vs_fp64"] = res["fp64"]["ms_per_step"] / res["fp32c"]["ms_per_step"]
    if errs is not None:
        o["rel_l2_vs_oracle"] = errs
    return o


def autograd_step(w, prec, steps, warmup):
    """End to end through DmkResidual: bin + forward + backward of
    E = 1/2 sum rho . u w.r.t. positions and strengths."""
    import torch
    from paper_2606_27134_amd import residual as R
    x = torch.as_tensor(w.x).cuda().requires_grad_(True)
    rho = torch.as_tensor(w.rho).cuda().requires_grad_(True)
    spec = R.ResidualSpec(L=w.L, D=w.D, n=w.n, kernel=w.kernel, prec=prec, sigma=w.sigma, rc=w.rc)

    def step():
        u = R.dmk_residual(x, rho, spec)
        E = 0.5 * (rho * u).sum()
        torch.autograd.grad(E, (x, rho))

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    return 1e3 * (time.perf_counter() - t0) / steps


def _far_flops(M, p, K):
    """Algorithmic flops of one root-level far field on an exact tiling of
    M_i cubes, counting the form the library runs on each axis: the direct
    contraction over the grid index, or (8 or more cubes) the DFT over the
    cube index plus the fold over the Chebyshev index, the DFT as a dense
    product below 65 cubes (when it at least halves the terms) and as an FFT
    (5 M log2 M per transform) from 65 on.  Complex multiply-add 8, real by
    complex or real part only 4."""
    G = [m * p for m in M]
    Wn = [2 * k + 1 for k in K]
    fft = [m >= 65 for m in M]
    fac = [f or (8 <= m and 2 * (m * m + w) <= w * m) for f, m, w in zip(fft, M, Wn)]
    # (A, C) around each axis: axis 2 on [g0][g1][.], axis 1 on [g0][.][n2], axis 0 on [.][n1][n2]
    cols = {2: (G[0] * G[1], 1), 1: (G[0], Wn[2]), 0: (1, Wn[1] * Wn[2])}
    fl = 0.0
    for ax, first_or_last in ((2, True), (1, False), (0, False)):
        A, C = cols[ax]
        half = 4.0 if first_or_last else 8.0  # real input (forward) / real part (evaluation)
        if fft[ax]:
            fl += 2 * (5.0 * M[ax] * math.log2(M[ax]) * A * p * C + 8.0 * A * Wn[ax] * p * C)
        elif fac[ax]:
            fl += 2 * (half * A * M[ax] * M[ax] * p * C + 8.0 * A * Wn[ax] * p * C)
        else:
            fl += 2 * half * A * G[ax] * Wn[ax] * C
    return fl


def far_leaf_leg(args):
    """Root-level far field (dmk_far3p_eval) and leaf-grid anterpolation /
    evaluation (dmk_cheb_anterp / dmk_cheb_eval), FP64, at the Laplace
    parameters for 1e-12 (c = 29, p = 38, N_per from the table).  Algorithmic
    flops: the sum-factorized contractions (_far_flops) and, for the leaf
    grids, 4 per point and node (anterpolation) and 2 (evaluation)."""
    import torch
    from paper_2606_27134_amd import _lib as L
    from paper_2606_27134_amd import far as F
    from paper_2606_27134_amd import residual as R
    out = {}
    rng = np.random.default_rng(2026)
    for name, Lv, M in (("cube", (1.0, 1.0, 1.0), (1, 1, 1)), ("cuboid_32x1x1", (32.0, 1.0, 1.0), (32, 1, 1)),
                        ("cuboid_1x1x32", (1.0, 1.0, 32.0), (1, 1, 32)),
                        ("cuboid_128x1x1", (128.0, 1.0, 1.0), (128, 1, 1)),
                        ("cuboid_256x1x1", (256.0, 1.0, 1.0), (256, 1, 1)),
                        ("cuboid_1024x1x1", (1024.0, 1.0, 1.0), (1024, 1, 1)),
                        ("cuboid_4096x1x1", (4096.0, 1.0, 1.0), (4096, 1, 1)),
                        ("cuboid_1x1x256", (1.0, 1.0, 256.0), (1, 1, 256))):
        p, c = 38, 29.0
        K = F.table_modes(c, Lv, 1.0)
        G = [m * p for m in M]
        rho = torch.as_tensor(rng.normal(size=(1, *G))).cuda()
        u = torch.empty_like(rho)
        nb = L.dmk_far3p_ws_bytes(L.make_far_grid(Lv, M, p, K), 0)
        ws = torch.empty(nb // 8 + 32, dtype=torch.float64, device="cuda")
        ms = _time_ms(lambda: F.far3p_eval(Lv, M, p, K, "laplace", 1.0, rho, pswf_c=c, out=u, ws=ws),
                      20 if max(M) <= 256 else 5)
        fl = _far_flops(M, p, K)
        out["far3p_" + name] = {"L": list(Lv), "cubes": list(M), "p": p, "c": c, "K": list(K), "ms": ms,
                                "ms_per_cube": ms / (M[0] * M[1] * M[2]),
                                "gflops": fl / (ms * 1e-3) / 1e9, "frac_fp64_peak": fl / (ms * 1e-3) / 1e12 / 78.6}
        del rho, u, ws
        torch.cuda.empty_cache()
    # leaf grids: 100k uniform points on an 8^3 tiling, p = 20 (the 1e-6 order)
    N, n, p = 100_000, (8, 8, 8), 20
    x = torch.as_tensor(rng.random((N, 3))).cuda()
    q = torch.as_tensor(rng.normal(size=(N, 1))).cuda()
    b = R.tree_bin((1.0, 1.0, 1.0), 3, n, x)
    ws = F.cheb_workspace(b, p)
    rg = F.cheb_anterp(b, p, q, ws=ws)
    uu = torch.empty_like(q)
    ta = _time_ms(lambda: F.cheb_anterp(b, p, q, out=rg, ws=ws), 10)
    te = _time_ms(lambda: F.cheb_eval(b, p, rg, out=uu, ws=ws), 10)
    out["leaf_grid"] = {"N": N, "tiling": list(n), "p": p,
                        "anterp_ms": ta, "anterp_gflops": 4.0 * N * p ** 3 / (ta * 1e-3) / 1e9,
                        "eval_ms": te, "eval_gflops": 2.0 * N * p ** 3 / (te * 1e-3) / 1e9}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="laplace_n1m")
    ap.add_argument("--kernel", default=None)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--precs", default="fp32c,fp64")
    ap.add_argument("--pswf-c", type=float, default=None,
                    help="bandwidth of the PSWF-split leg (default: the paper's 1e-6 value for the kernel; 0 skips)")
    ap.add_argument("--no-far", action="store_true",
                    help="skip the root-level far field and leaf-grid leg")
    ap.add_argument("--configs", default="all",
                    help="comma-separated labels of the other configurations to time ('none' skips them)")
    ap.add_argument("--config-steps", type=int, default=10)
    ap.add_argument("--oracle-targets", type=int, default=64,
                    help="sampled targets per configuration for the error against the oracle (0 skips)")
    ap.add_argument("--headline-only", action="store_true",
                    help="only the headline workload's timed steps (for profiler runs)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run only a plain 1 GiB device copy (counter calibration)")
    args = ap.parse_args()

    ws_env = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or ws_env != 1:
        print("bench.py runs on exactly one GPU: this library has no multi-GPU path "
              "(--gpus %d requested)." % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    torch.cuda.set_device(0)

    if args.copy_calibration:
        n = 1 << 27  # 128 Mi doubles = 1 GiB
        a = torch.ones(n, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": n * 8, "copy_bytes_written": n * 8, "launches": 3}))
        return

    precs = [p for p in args.precs.split(",") if p]
    w = W.make(args.workload, kernel=args.kernel)
    bins, bin_ms, res, outs = bench_workload(w, precs, args.steps, args.warmup)
    print("headline %s timed" % w.name, file=sys.stderr, flush=True)
    if args.headline_only:
        r = res[precs[0]]
        print(json.dumps({"workload": w.name, "ms_per_step": r["ms_per_step"], "kernel_fwd_ms": r["kernel_fwd_ms"],
                          "kernel_bwd_ms": r["kernel_bwd_ms"]}), flush=True)
        return
    P_in = count_pairs(w)
    P_cand = count_candidates(w)

    # ---- PSWF split (Sec. 2.2) on the same points: support nu = rc, so the
    # same in-cutoff pairs; bandwidth c from the paper's parameter tables
    pswf = None
    pc = PSWF_C_1E6[w.kernel] if args.pswf_c is None else args.pswf_c
    if pc and pc > 0:
        pswf = {"c": pc, "nu": w.rc}
        for prec in precs:
            r, o = time_residual(w, bins, prec, max(5, args.steps // 2), args.warmup, pswf_c=pc)
            pswf[prec] = {"value": P_in / (r["ms_per_step"] * 1e-3), "fwd_ms": r["fwd_ms"], "bwd_ms": r["bwd_ms"],
                          "kernel_fwd_ms": r["kernel_fwd_ms"], "kernel_bwd_ms": r["kernel_bwd_ms"]}
            outs["pswf_" + prec] = o

    head = "fp32c" if "fp32c" in res else precs[0]
    r = res[head]
    khash = kernel_hash()
    roof = roofline(w.kernel, head, P_in, r, khash=khash, workload=w.name)
    line = {
        "metric": METRIC, "value": P_in / (r["ms_per_step"] * 1e-3), "unit": "pair-interactions/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": r["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32" if head == "fp32c" else "f64", "data": "synthetic",
        "config": {"workload": "%s: %s D=%d L=%s n=%s N=%d sigma=%.6g rc=%.6g" % (
            w.name, w.kernel, w.D, list(w.L), list(w.n), w.N, w.sigma, w.rc),
            "precision": head, "step": "residual forward + adjoint (points pre-binned)"},
        "P_in": P_in, "P_cand": P_cand, "candidate_pairs_per_s": P_cand / (r["ms_per_step"] * 1e-3),
        "bin_ms": bin_ms, "median_ms": r["median_ms"],
        "fwd_ms": r["fwd_ms"], "bwd_ms": r["bwd_ms"],
        "kernel_fwd_ms": r["kernel_fwd_ms"], "kernel_bwd_ms": r["kernel_bwd_ms"],
        "gather_fwd_ms": r["gather_fwd_ms"], "gather_bwd_ms": r["gather_bwd_ms"],
        "roofline": roof, "kernel_hash": khash,
    }
    # the paper's own timings, as context: it reports full-DMK runtimes of a
    # MATLAB code only in figures (normalized), none for the residual path
    line["paper_context"] = {
        "residual_path_timing": None,
        "platform": "MATLAB (not optimized for runtime), AMD EPYC 9655P 96-core CPU, FP64, full DMK",
        "published": "normalized runtimes (t(L)/N)/(t(unit cube)/N) within [0.9, 1.1] for cells [1,L2,L3], "
                     "L2,L3 in 1..5, 1e4 points per unit volume, tolerance 1e-6 (Sec. 6); achieved rel l2 "
                     "of the full method 1.0e-7 (Laplace) / 1.7e-7 (Stokeslet) at tolerance 1e-6"}
    if "fp64" in res and head != "fp64":
        f = res["fp64"]
        line["fp64"] = {"value": P_in / (f["ms_per_step"] * 1e-3), "ms_per_step": f["ms_per_step"],
                        "fwd_ms": f["fwd_ms"], "bwd_ms": f["bwd_ms"], "kernel_fwd_ms": f["kernel_fwd_ms"],
                        "kernel_bwd_ms": f["kernel_bwd_ms"],
                        "roofline": roofline(w.kernel, "fp64", P_in, f, khash=khash, workload=w.name)}
        line["fp32c_speedup_vs_fp64"] = f["ms_per_step"] / r["ms_per_step"]
    # end to end through the autograd function: bin + forward + backward
    line["autograd_step_ms"] = {p: autograd_step(w, p, max(5, args.steps // 5), 2) for p in precs}
    if pswf is not None:
        line["pswf"] = pswf

    # ---- the other workloads of the configuration list
    if args.configs != "none":
        want = None if args.configs == "all" else set(args.configs.split(","))
        cfg_out = {}
        pin_cache = {}
        for label, name, kern in CONFIGS:
            if want is not None and label not in want:
                continue
            wc = W.make(name, kernel=kern)
            _, cbin, cres, couts = bench_workload(wc, precs, args.config_steps, 3)
            key = (name, wc.D)
            if key not in pin_cache:
                pin_cache[key] = count_pairs(wc)
            errs = oracle_errors(wc, couts, args.oracle_targets) if args.oracle_targets > 0 else None
            cfg_out[label] = config_object(label, wc, pin_cache[key], cbin, cres, errs)
            print("config %s timed" % label, file=sys.stderr, flush=True)
            torch.cuda.empty_cache()
        line["configs"] = cfg_out

    if not args.no_far:
        line["far_leaf"] = far_leaf_leg(args)

    if not args.no_cpu_baseline:
        cb, (t, u_o, gr_o, gx_o, _) = cpu_baseline(w)
        line["cpu_baseline"] = cb

        def rl2(a, b):
            return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))
        errs = {}
        for prec, (u, gr, gx) in outs.items():
            if prec.startswith("pswf_"):
                continue
            errs[prec] = {"u": rl2(u[t], u_o), "grad_rho": rl2(gr[t], gr_o), "grad_x": rl2(gx[t], gx_o)}
        line["rel_l2_vs_oracle"] = errs
        if pswf is not None:
            # the PSWF leg against the oracle's own PSWF window on a small sample
            import oracle
            from oracle.pswf import PswfWindow
            ow = PswfWindow(pswf["c"])
            ts = t[: max(1, min(len(t), 64))]
            Gh = W.cotangent(w.seed, w.N, W.M_OUT[w.kernel])
            pu = oracle.residual(w.kernel, w.D, w.L, w.rc, w.rc, w.x, w.rho, targets=ts, window=ow)
            pgr, pgx = oracle.residual_vjp(w.kernel, w.D, w.L, w.rc, w.rc, w.x, w.rho, Gh, targets=ts, window=ow)
            pswf["rel_l2_vs_oracle"] = {
                prec: {"u": rl2(outs["pswf_" + prec][0][ts], pu), "grad_rho": rl2(outs["pswf_" + prec][1][ts], pgr),
                       "grad_x": rl2(outs["pswf_" + prec][2][ts], pgx)}
                for prec in precs}
            pswf["oracle_sample_targets"] = int(len(ts))
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
