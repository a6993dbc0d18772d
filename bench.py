#!/usr/bin/env python3
"""Benchmark of the leaf-level residual interaction on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload laplace_n1m]

One step = dmk_residual_eval (forward) + dmk_residual_backward (adjoint) of
the whole workload, with the points already binned and all inputs resident
in HBM (the binning, the paper's tree construction, is timed separately and
reported as bin_ms).  The headline is the FP32-compensated path; the FP64
path is timed the same way and reported beside it.

Metric: in-cutoff ordered pair interactions (0 < r < rc, P_in) per second of
forward + backward.  Prints ONE JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from paper_2606_27134_amd import workloads as W  # noqa: E402

METRIC = "residual pair-interactions/s fwd+bwd, FP32-compensated vs FP64 at stated rel err"

# Algorithmic flops per in-cutoff pair (add/mul = 1, fma = 2, each elementary
# function rsqrt/exp/erfc = 1), counted from the kernel formulas.
FLOPS_PER_PAIR = {
    ("laplace", "fwd"): 19, ("laplace", "bwd"): 34,
    ("stokeslet", "fwd"): 42, ("stokeslet", "bwd"): 95,
    ("stresslet", "fwd"): 68, ("stresslet", "bwd"): 190,
    ("rotlet", "fwd"): 33, ("rotlet", "bwd"): 70,
}
PEAK_TFLOPS = {"fp32c": 157.3, "fp64": 78.6}  # MI355X vector peaks
# PSWF bandwidth c for a requested tolerance 1e-6 (the paper's parameter
# tables for the Laplace and Stokes kernels)
PSWF_C_1E6 = {"laplace": 14.5, "stokeslet": 17.80, "stresslet": 17.80, "rotlet": 13.61}
HBM_PEAK_GBS = 8000.0


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


def kernel_hash():
    """Hash of the sources that k_residual is built from (the counter-based
    traffic applies only while they are unchanged)."""
    h = hashlib.sha256()
    for f in ("paper_2606_27134_amd/csrc/dmk_residual.hip", "paper_2606_27134_amd/csrc/dmk_internal.h",
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


def cpu_baseline(w, budget_s=15.0):
    """The oracle (fwd + vjp) on a bounded sample of targets of the same workload."""
    import oracle
    oracle.build()
    rng = np.random.default_rng(123)
    G = W.cotangent(w.seed, w.N, W.M_OUT[w.kernel])
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    cores = min(cores, os.cpu_count() or cores)
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
    pin = count_pairs(w, targets=t)
    return dict(value=pin / dt, unit="pair-interactions/s", cores=cores, kind="oracle",
                sample="%d seeded targets of %s (all %d sources, every image), fwd + vjp, %.1f s, "
                       "P_in(sample)=%d" % (n, w.name, w.N, dt, pin)), (t, u, gr, gx, G)


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


def _far_flops(M, p, K):
    """Algorithmic flops of one root-level far field on an exact tiling of
    M_i cubes, counting the form the library runs on each axis: the direct
    contraction over the grid index, or (8 or more cubes, when it at least
    halves the terms) the DFT over the cube index plus the fold over the
    Chebyshev index.  Complex multiply-add 8, real by complex or real part
    only 4."""
    G = [m * p for m in M]
    W = [2 * k + 1 for k in K]
    fac = [8 <= m <= 512 and 2 * (m * m + w) <= w * m for m, w in zip(M, W)]
    # (A, C) around each axis: axis 2 on [g0][g1][.], axis 1 on [g0][.][n2], axis 0 on [.][n1][n2]
    cols = {2: (G[0] * G[1], 1), 1: (G[0], W[2]), 0: (1, W[1] * W[2])}
    fl = 0.0
    for ax, first_or_last in ((2, True), (1, False), (0, False)):
        A, C = cols[ax]
        half = 4.0 if first_or_last else 8.0  # real input (forward) / real part (evaluation)
        if fac[ax]:
            fl += 2 * (half * A * M[ax] * M[ax] * p * C + 8.0 * A * W[ax] * p * C)
        else:
            fl += 2 * half * A * G[ax] * W[ax] * C
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
                        ("cuboid_128x1x1", (128.0, 1.0, 1.0), (128, 1, 1))):
        p, c = 38, 29.0
        K = F.table_modes(c, Lv, 1.0)
        G = [m * p for m in M]
        rho = torch.as_tensor(rng.normal(size=(1, *G))).cuda()
        u = torch.empty_like(rho)
        nb = L.dmk_far3p_ws_bytes(L.make_far_grid(Lv, M, p, K), 0)
        ws = torch.empty(nb // 8 + 32, dtype=torch.float64, device="cuda")
        ms = _time_ms(lambda: F.far3p_eval(Lv, M, p, K, "laplace", 1.0, rho, pswf_c=c, out=u, ws=ws), 20)
        fl = _far_flops(M, p, K)
        out["far3p_" + name] = {"L": list(Lv), "cubes": list(M), "p": p, "c": c, "K": list(K), "ms": ms,
                                "gflops": fl / (ms * 1e-3) / 1e9, "frac_fp64_peak": fl / (ms * 1e-3) / 1e12 / 78.6}
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

    from paper_2606_27134_amd import residual as R
    from paper_2606_27134_amd import _lib as L

    w = W.make(args.workload, kernel=args.kernel)
    stream = torch.cuda.current_stream()
    x = torch.as_tensor(w.x).cuda()
    rho = torch.as_tensor(w.rho).cuda()
    G = torch.as_tensor(W.cotangent(w.seed, w.N, W.M_OUT[w.kernel])).cuda()

    # binning (setup), timed on its own
    bins = R.Bins(w.L, w.D, w.n, w.N)
    bins.bin(x)
    torch.cuda.synchronize()
    tb = []
    for _ in range(3):
        t0 = time.perf_counter()
        bins.bin(x)
        torch.cuda.synchronize()
        tb.append(time.perf_counter() - t0)
    bin_ms = 1e3 * float(np.median(tb))

    P_in = count_pairs(w)
    precs = [p for p in args.precs.split(",") if p]
    res = {}
    outs = {}
    for prec in precs:
        ws_f = R.workspace(bins, w.kernel, prec, False)
        ws_b = R.workspace(bins, w.kernel, prec, True)
        u = torch.empty((w.N, W.M_OUT[w.kernel]), dtype=torch.float64, device="cuda")
        gr = torch.empty((w.N, W.M_IN[w.kernel]), dtype=torch.float64, device="cuda")
        gx = torch.empty((w.N, 3), dtype=torch.float64, device="cuda")

        def step():
            R.residual_eval(bins, w.kernel, prec, w.sigma, w.rc, rho, out=u, ws=ws_f)
            R.residual_backward(bins, w.kernel, prec, w.sigma, w.rc, rho, G, out=(gr, gx), ws=ws_b)

        for _ in range(args.warmup):
            step()
        torch.cuda.synchronize()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(3 * args.steps + 2)]
        start, stop = ev[-2], ev[-1]
        # events the library records around the pair kernel alone (the call
        # also gathers the strengths into the sorted order first)
        kev = [torch.cuda.Event(enable_timing=True) for _ in range(4 * args.steps)]
        for e in kev:
            e.record(stream)  # creates the device event
        torch.cuda.synchronize()
        t_wall = time.perf_counter()
        start.record(stream)
        for k in range(args.steps):
            ev[3 * k].record(stream)
            L.dmk_residual_set_kernel_events(kev[4 * k].cuda_event, kev[4 * k + 1].cuda_event)
            R.residual_eval(bins, w.kernel, prec, w.sigma, w.rc, rho, out=u, ws=ws_f)
            ev[3 * k + 1].record(stream)
            L.dmk_residual_set_kernel_events(kev[4 * k + 2].cuda_event, kev[4 * k + 3].cuda_event)
            R.residual_backward(bins, w.kernel, prec, w.sigma, w.rc, rho, G, out=(gr, gx), ws=ws_b)
            ev[3 * k + 2].record(stream)
        stop.record(stream)
        L.dmk_residual_set_kernel_events(0, 0)
        torch.cuda.synchronize()
        t_wall = time.perf_counter() - t_wall
        total_ms = start.elapsed_time(stop)
        fwd = [ev[3 * k].elapsed_time(ev[3 * k + 1]) for k in range(args.steps)]
        bwd = [ev[3 * k + 1].elapsed_time(ev[3 * k + 2]) for k in range(args.steps)]
        kfwd = [kev[4 * k].elapsed_time(kev[4 * k + 1]) for k in range(args.steps)]
        kbwd = [kev[4 * k + 2].elapsed_time(kev[4 * k + 3]) for k in range(args.steps)]
        ms_step = total_ms / args.steps
        res[prec] = dict(ms_per_step=ms_step, fwd_ms=float(np.mean(fwd)), bwd_ms=float(np.mean(bwd)),
                         fwd_ms_median=float(np.median(fwd)), bwd_ms_median=float(np.median(bwd)),
                         kernel_fwd_ms=float(np.mean(kfwd)), kernel_bwd_ms=float(np.mean(kbwd)),
                         value=P_in / (ms_step * 1e-3), wall_s=t_wall)
        outs[prec] = (u.cpu().numpy(), gr.cpu().numpy(), gx.cpu().numpy())

    # ---- PSWF split (Sec. 2.2) on the same points: support nu = rc, so the
    # same in-cutoff pairs; bandwidth c from the paper's parameter tables
    pswf = None
    pc = PSWF_C_1E6[w.kernel] if args.pswf_c is None else args.pswf_c
    if pc and pc > 0:
        pswf = {"c": pc, "nu": w.rc}
        for prec in precs:
            ws_f = R.workspace(bins, w.kernel, prec, False)
            ws_b = R.workspace(bins, w.kernel, prec, True)
            u = torch.empty((w.N, W.M_OUT[w.kernel]), dtype=torch.float64, device="cuda")
            gr = torch.empty((w.N, W.M_IN[w.kernel]), dtype=torch.float64, device="cuda")
            gx = torch.empty((w.N, 3), dtype=torch.float64, device="cuda")
            for _ in range(args.warmup):
                R.residual_eval(bins, w.kernel, prec, 0.0, w.rc, rho, out=u, ws=ws_f, pswf_c=pc)
                R.residual_backward(bins, w.kernel, prec, 0.0, w.rc, rho, G, out=(gr, gx), ws=ws_b, pswf_c=pc)
            torch.cuda.synchronize()
            ev = [torch.cuda.Event(enable_timing=True) for _ in range(3 * args.steps)]
            for k in range(args.steps):
                ev[3 * k].record(stream)
                R.residual_eval(bins, w.kernel, prec, 0.0, w.rc, rho, out=u, ws=ws_f, pswf_c=pc)
                ev[3 * k + 1].record(stream)
                R.residual_backward(bins, w.kernel, prec, 0.0, w.rc, rho, G, out=(gr, gx), ws=ws_b, pswf_c=pc)
                ev[3 * k + 2].record(stream)
            torch.cuda.synchronize()
            fwd = float(np.mean([ev[3 * k].elapsed_time(ev[3 * k + 1]) for k in range(args.steps)]))
            bwd = float(np.mean([ev[3 * k + 1].elapsed_time(ev[3 * k + 2]) for k in range(args.steps)]))
            pswf[prec] = {"value": P_in / ((fwd + bwd) * 1e-3), "fwd_ms": fwd, "bwd_ms": bwd}
            outs["pswf_" + prec] = (u.cpu().numpy(), gr.cpu().numpy(), gx.cpu().numpy())

    head = "fp32c" if "fp32c" in res else precs[0]
    r = res[head]
    # dominant kernel: the larger of the two launches of the headline step
    dom = "bwd" if r["kernel_bwd_ms"] >= r["kernel_fwd_ms"] else "fwd"
    dur_ms = r["kernel_%s_ms" % dom]  # average duration of that k_residual launch
    flops = FLOPS_PER_PAIR[(w.kernel, dom)] * P_in
    achieved = flops / (dur_ms * 1e-3) / 1e12
    khash = kernel_hash()
    tr = read_traffic(w.name, head, khash)
    traffic = None if tr is None else tr.get(dom)
    vi = read_traffic(w.name, head, khash, field="valu_issue")
    roof = {"bound": "alu", "achieved": achieved, "peak": PEAK_TFLOPS[head], "unit": "TFLOP/s",
            "frac": achieved / PEAK_TFLOPS[head], "traffic": traffic,
            # share of the SIMDs' VALU issue slots the launch used (SQ_INSTS_VALU
            # x 4 cycles over the launch's cycles), from the same counter runs
            "valu_issue_frac": None if vi is None else vi.get(dom),
            "kernel": "k_residual<%s,%s,%s>" % (w.kernel, head, dom),
            "flops_per_pair": FLOPS_PER_PAIR[(w.kernel, dom)], "launch_ms": dur_ms}

    line = {
        "metric": METRIC, "value": r["value"], "unit": "pair-interactions/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": r["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32" if head == "fp32c" else "f64", "data": "synthetic",
        "config": {"workload": "%s: %s D=%d L=%s n=%s N=%d sigma=%.6g rc=%.6g" % (
            w.name, w.kernel, w.D, list(w.L), list(w.n), w.N, w.sigma, w.rc),
            "precision": head, "step": "residual forward + adjoint (points pre-binned)"},
        "P_in": P_in, "bin_ms": bin_ms,
        "fwd_ms": r["fwd_ms"], "bwd_ms": r["bwd_ms"],
        "kernel_fwd_ms": r["kernel_fwd_ms"], "kernel_bwd_ms": r["kernel_bwd_ms"],
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
        line["fp64"] = {"value": f["value"], "ms_per_step": f["ms_per_step"], "fwd_ms": f["fwd_ms"],
                        "bwd_ms": f["bwd_ms"]}
        line["fp32c_speedup_vs_fp64"] = f["ms_per_step"] / r["ms_per_step"]

    if pswf is not None:
        line["pswf"] = pswf
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
