#!/usr/bin/env python3
"""Benchmark of the blocked multi-shift triangular solve on one MI355X.

Workload: complex128 multi-shift solve (U - l_j I) X = B at m = n = 4096,
plain FP64 (U off-diagonal CN(0,1)/64, diagonal on the annulus 0.5..2,
4096 shifts in the disk of radius 0.4, B iid CN(0,1); seeded synthetic data).
A step is one full solve of fresh right-hand sides already resident in HBM.
Metric: GFLOP/s = 4 m^2 n / t (complex multiply-add = 8 real flops).

Also reported on the same line:
  roofline      the substitution GEMM (the dominant kernel) timed live with
                HIP events around each of its launches, against the FP64
                matrix-core peak of MI355X (78.6 TFLOP/s);
  cpu_baseline  the CPU oracle (C, OpenMP over shifts) on a bounded sample of
                the same workload on this host's cores;
  secondary     the FP32-GEMM + FP64-refinement form of the same solve, its
                time to FP64 accuracy and its error against the FP64 result.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--workload solve|pencil|safe|triang_eig]

--workload pencil times the generalized solve (U - l_j V) X = B (appendix,
Alg 8) at the same size instead (8 m^2 n flops per solve); safe the safe
solve of the same inputs; triang_eig the triangular eigenvectors at m = 2048
(sum 4 j^2 flops). Each has its own roofline and CPU-oracle lines and no
secondary measurements.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64_MFMA_TF = 78.6
# HBM bytes per launch of the substitution GEMM at this workload, from rocprofv3
# FETCH_SIZE / WRITE_SIZE runs scaled by a 512 MiB copy (profiles/k_gemm_direct_solve_m4096_n4096.md).
# Valid only for the sources it was measured on: the GEMM kernel and the block
# loops that choose its launch shapes (sha1 prefix of csrc/kgemm.hip followed by
# csrc/api.hip).
GEMM_TRAFFIC = {"sources_sha1": "1010a805c6675784", "bytes_per_launch": 278.3e6, "m": 4096, "n": 4096,
                "nb": 16, "outer_nb": 0,
                # the pencil substitution (profiles/k_gemm_direct_pencil_m4096_n4096.md)
                "pencil_bytes_per_launch": 456.1e6}
# The same for the real substitution GEMM (all its tile variants, averaged over
# the 15 launches of a solve; profiles/real_solve_m4096_n4096.md), valid for the
# sources it was measured on (sha1 prefix of csrc/kreal.hip followed by csrc/api.hip).
REAL_GEMM_TRAFFIC = {"sources_sha1": "cf78bf470363a34f", "bytes_per_launch": 112.6e6, "m": 4096, "n": 4096,
                     "outer_nb": 0}
PEAK_FP32_MFMA_TF = 157.3
METRIC = "complex128 multi-shift solve GFLOP/s at m=n=4096 and % of MFMA peak vs plain FP64"
METRIC_PENCIL = "complex128 generalized multi-shift solve GFLOP/s (8 m^2 n) at m=n=4096"
METRIC_SAFE = "complex128 safe multi-shift solve GFLOP/s at m=n=4096"
METRIC_TEIG = "complex128 triangular eigenvectors GFLOP/s (sum 4 j^2) at m=2048"
METRIC_REAL = "float64 real multi-shift solve GFLOP/s (m^2 n) at m=n=4096"


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def dev(a, torch):
    import numpy as np
    a = np.asfortranarray(a)
    dt = torch.float64 if a.dtype == np.float64 else torch.complex128
    out = torch.empty_strided(a.shape, (1, a.shape[0]), dtype=dt, device="cuda")
    out.copy_(torch.from_numpy(a))
    return out


def sources_sha1(*names):
    """sha1 prefix of the named csrc files, read in order; None if one is missing."""
    import hashlib
    h = hashlib.sha1()
    try:
        for name in names:
            with open(os.path.join(ROOT, "paper_1607_01477_amd", "csrc", name), "rb") as f:
                h.update(f.read())
    except OSError:
        return None
    return h.hexdigest()[:16]


def gemm_traffic(m, n, nb, outer_nb, pencil=False):
    t = GEMM_TRAFFIC
    if (sources_sha1("kgemm.hip", "api.hip") != t["sources_sha1"]
            or (m, n, nb, outer_nb) != (t["m"], t["n"], t["nb"], t["outer_nb"])):
        return None
    return t["pencil_bytes_per_launch"] if pencil else t["bytes_per_launch"]


def real_gemm_traffic(m, n, outer_nb):
    t = REAL_GEMM_TRAFFIC
    if (sources_sha1("kreal.hip", "api.hip") != t["sources_sha1"]
            or (m, n, outer_nb) != (t["m"], t["n"], t["outer_nb"])):
        return None
    return t["bytes_per_launch"]


def _time(fn, torch, reps):
    fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) * 1e3 / reps


def other_workloads(P, W, torch, np) -> dict:
    """Triangular eigenvectors (safe solve, variable-length columns), inverse
    Lanczos on a 100x100 shift grid, forward + backward through the solve, the
    generalized (pencil) solve, generalized triangular eigenvectors, general
    eigenvectors after a host Schur decomposition, and the lower-triangular /
    transposed variants."""
    out = {}
    # triangular eigenvectors, m = 2048: sum_j 4 j^2 flops
    w = W.c2_triang_eig()
    T = dev(w.U, torch)
    ms = _time(lambda: P.triang_eig(T), torch, 3)
    ev, Z, k = P.triang_eig(T)
    fl = W.nominal_flops(w.m, w.n, w.col_len)
    out["c2_triang_eig_m2048"] = {"ms": round(ms, 3), "gflops": round(fl / (ms * 1e-3) / 1e9, 2),
                                  "rescaled_columns": int((k > 0).sum().item())}
    log("triangular eigenvectors m=2048: %.3f ms" % ms)
    del T, Z
    # pseudospectra: 15 Lanczos steps = 30 solves of 2000 x 10000
    w = W.c4_pseudospectra()
    Ud = dev(w.U, torch)
    z = torch.from_numpy(w.shifts).cuda()
    V0 = dev(w.B, torch)
    ms = _time(lambda: P.lanczos_sigma_min(Ud, z, V0, iters=15), torch, 2)
    fl = 30 * W.nominal_flops(w.m, w.n)
    out["c4_lanczos_m2000_N10000"] = {"ms": round(ms, 3), "gflops": round(fl / (ms * 1e-3) / 1e9, 2),
                                      "ms_per_shift_us": round(ms * 1e3 / w.n, 3)}
    log("pseudospectra 2000 x 10000 shifts, 15 steps: %.3f ms" % ms)
    # the same grid with thick-restart Lanczos to a relative residual of 1e-10
    res = {}

    def trl():
        res["r"] = P.lanczos_restarted_sigma_min(Ud, z, V0, tol=1e-10)
    ms = _time(trl, torch, 2)
    st = res["r"][2].cpu().numpy()
    cv = res["r"][3].cpu().numpy()
    fl = 2 * int(st.sum()) * 4.0 * w.m * w.m
    out["c4_lanczos_restarted_m2000_N10000"] = {
        "ms": round(ms, 3), "tol": 1e-10, "kdim": 20, "keep": 6, "converged": int(cv.sum()),
        "steps_min": int(st.min()), "steps_mean": round(float(st.mean()), 2), "steps_max": int(st.max()),
        "solve_gflops": round(fl / (ms * 1e-3) / 1e9, 2)}
    log("pseudospectra 2000 x 10000 shifts, thick restart to 1e-10: %.3f ms, steps %d..%d (mean %.1f), "
        "%d converged" % (ms, st.min(), st.max(), st.mean(), cv.sum()))
    del Ud, V0
    # forward + backward through the solve, m = 4096, n = 2048
    w = W.c5_adjoint()
    U = dev(w.U, torch).requires_grad_(True)
    s = torch.from_numpy(w.shifts).cuda().requires_grad_(True)
    B = dev(w.B, torch).requires_grad_(True)
    Wt = torch.from_numpy(np.asfortranarray(w.extra["W"])).cuda()

    def fwd_bwd():
        U.grad = s.grad = B.grad = None
        X = P.solve(U, s, B)
        (Wt * (X.real ** 2 + X.imag ** 2)).sum().backward()

    def fwd():
        with torch.no_grad():
            P.mstrsm(U.detach(), s.detach(), B.detach().clone())

    ms_f = _time(fwd, torch, 3)
    ms_fb = _time(fwd_bwd, torch, 3)
    ffl = W.nominal_flops(w.m, w.n)
    out["c5_fwd_bwd_m4096_n2048"] = {"fwd_ms": round(ms_f, 3), "fwd_bwd_ms": round(ms_fb, 3),
                                     "fwd_bwd_gflops": round(3 * ffl / (ms_fb * 1e-3) / 1e9, 2)}
    log("forward %.3f ms, forward+backward %.3f ms" % (ms_f, ms_fb))
    del U, s, B, Wt
    # generalized (pencil) solve, m = n = 4096: 8 m^2 n flops (U X and V (lambda X))
    w = W.c6_generalized()
    Ug, Vg = dev(w.U, torch), dev(w.extra["V"], torch)
    sg = torch.from_numpy(w.shifts).cuda()
    Bg = dev(w.B, torch)
    ms_g = _time(lambda: P.mstrsm_gen(Ug, Vg, sg, Bg), torch, 3)
    Bg.copy_(dev(w.B, torch))
    ms_gs = _time(lambda: P.mstrsm_safe_gen(Ug, Vg, sg, Bg), torch, 3)
    gfl = 2 * W.nominal_flops(w.m, w.n)
    out["c6_generalized_m4096_n4096"] = {
        "ms": round(ms_g, 3), "gflops": round(gfl / (ms_g * 1e-3) / 1e9, 2),
        "safe_ms": round(ms_gs, 3), "safe_gflops": round(gfl / (ms_gs * 1e-3) / 1e9, 2)}
    log("generalized solve 4096 x 4096: %.3f ms plain, %.3f ms safe" % (ms_g, ms_gs))
    del Ug, Vg, Bg
    # generalized triangular eigenvectors, m = 2048: sum_j 8 j^2 flops
    w = W.c7_gen_triang_eig()
    T, S = dev(w.U, torch), dev(w.extra["S"], torch)
    ms = _time(lambda: P.gen_triang_eig(T, S), torch, 3)
    ev, Z, k = P.gen_triang_eig(T, S)
    fl = 2 * W.nominal_flops(w.m, w.m, w.col_len)
    out["c7_gen_triang_eig_m2048"] = {"ms": round(ms, 3), "gflops": round(fl / (ms * 1e-3) / 1e9, 2),
                                      "rescaled_columns": int((k > 0).sum().item())}
    log("generalized triangular eigenvectors m=2048: %.3f ms" % ms)
    del T, S, Z
    # general eigenvectors (Eig, Alg 6), m = 2048: host Schur (context), then
    # TriangEig + X = Q Z (4 m^3 flops on the matrix cores) + unit columns on the GPU
    import scipy.linalg as sla
    A = W.c8_dense_eig().extra["A"]
    t0 = time.perf_counter()
    Th, Qh = sla.schur(A, output="complex")
    t_schur = time.perf_counter() - t0
    T, Q = dev(Th, torch), dev(Qh, torch)
    ms = _time(lambda: P.eig_schur(T, Q), torch, 3)
    ev, X, k = P.eig_schur(T, Q)
    Xh, evh = X.cpu().numpy(), ev.cpu().numpy()
    res = float(np.linalg.norm(A @ Xh - Xh * evh[None, :]) / np.linalg.norm(A))
    with P.profile() as pr:
        P.eig_schur(T, Q)
    bt = pr.result["resid"]
    out["c8_eig_m2048"] = {"gpu_ms": round(ms, 3), "host_schur_s": round(t_schur, 2),
                           "backtransform_ms": round(bt["ms"], 3),
                           "backtransform_tflops": round(bt["flops"] / (bt["ms"] * 1e-3) / 1e12, 2),
                           "rel_residual_F": res}
    log("eigenvectors m=2048: %.3f ms on the GPU (host Schur %.1f s), residual %.1e" % (ms, t_schur, res))
    del T, Q, X
    # lower-triangular and transposed variants, m = 4096, n = 2048 (4 m^2 n flops each)
    w = W.c5_adjoint()
    Ud = dev(w.U, torch)
    Ld = dev(np.asfortranarray(w.U.T.copy()), torch)
    sv = torch.from_numpy(w.shifts).cuda()
    Bv = dev(w.B, torch)
    fl = W.nominal_flops(w.m, w.n)
    var = {}
    for uplo, op in (("L", "N"), ("L", "T"), ("L", "C"), ("U", "T")):
        A = Ld if uplo == "L" else Ud
        msv = _time(lambda: P.mstrsm_op(A, sv, Bv, uplo=uplo, op=op), torch, 3)
        var[uplo + op] = {"ms": round(msv, 3), "gflops": round(fl / (msv * 1e-3) / 1e9, 2)}
    out["variants_m4096_n2048"] = var
    log("variants m=4096 n=2048: %s" % ", ".join("%s %.3f ms" % (k, v["ms"]) for k, v in var.items()))
    del Ud, Ld, Bv
    # real arithmetic, m = n = 4096 (m^2 n flops), solved in place repeatedly
    w = W.c10_real()
    Ur, sr, Br = dev(w.U, torch), torch.from_numpy(w.shifts).cuda(), dev(w.B, torch)
    msr = _time(lambda: P.mstrsm_real(Ur, sr, Br), torch, 5)
    fr = float(w.m) ** 2 * w.n
    out["c10_real_m4096_n4096"] = {"ms": round(msr, 3), "gflops": round(fr / (msr * 1e-3) / 1e9, 2)}
    # the lower forward variant (upper copy of the reversed matrix, rows of B reversed around the solve)
    Lr = dev(np.asfortranarray(w.U.T.copy()), torch)
    msl = _time(lambda: P.mstrsm_real_op(Lr, sr, Br, uplo="L", op="N"), torch, 5)
    out["c10_real_m4096_n4096"].update({"LN_ms": round(msl, 3), "LN_gflops": round(fr / (msl * 1e-3) / 1e9, 2)})
    log("real solve 4096 x 4096: %.3f ms (lower forward variant %.3f ms)" % (msr, msl))
    del Ur, Br, Lr
    return out


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=25)
    ap.add_argument("--m", type=int, default=4096)
    ap.add_argument("--n", type=int, default=4096)
    ap.add_argument("--nb", type=int, default=16)
    ap.add_argument("--outer-nb", type=int, default=0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-secondary", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--workload", choices=["solve", "pencil", "safe", "triang_eig", "real"], default="solve",
                    help="solve: (U - l_j I) X = B, the headline; pencil: the generalized "
                         "solve (U - l_j V) X = B at the same size (8 m^2 n flops); safe: the "
                         "safe solve of the headline inputs; triang_eig: triangular "
                         "eigenvectors at m = 2048 (sum 4 j^2 flops); real: the real-"
                         "arithmetic solve at the same size (m^2 n flops). All but the "
                         "first without the secondary measurements")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run 4 device copies of 512 MiB (reference for HBM byte counters)")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch
        src = torch.ones(64 << 20, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(4):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes_per_copy": src.numel() * 8 * 2}))
        return 0
    if args.gpus != 1:
        print("bench.py measures one GPU: there is no multi-GPU path (the shifts would be "
              "sharded across GPUs with U replicated and no communication)", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    import paper_1607_01477_amd as P
    import workloads as W

    pencil = args.workload == "pencil"
    safe = args.workload == "safe"
    teig = args.workload == "triang_eig"
    real = args.workload == "real"
    if args.workload != "solve":
        args.no_secondary = True
    if pencil:
        args.nb = 16
    if teig:
        args.m = args.n = min(args.m, 2048)
    m, n = args.m, args.n
    t_gen = time.perf_counter()
    if pencil:
        w = W.c6_generalized(m=m, n=n)
    elif teig:
        w = W.c2_triang_eig(m=m)
    elif real:
        w = W.c10_real(m=m, n=n)
    else:
        w = W.c3_mixed(m=m, n=n)
    log("inputs generated in %.1fs" % (time.perf_counter() - t_gen))
    torch.cuda.set_device(0)
    U = dev(w.U, torch)
    lam = torch.from_numpy(w.shifts).cuda()
    B0 = dev(w.B, torch)
    flops = (8.0 if pencil else 1.0 if real else 4.0) * m * m * n
    if teig:
        flops = W.nominal_flops(m, m, w.col_len)
    opts = dict(nb=args.nb, outer_nb=args.outer_nb)
    teig_out = {}
    if pencil:
        Vd = dev(w.extra["V"], torch)

        def solve(X):
            return P.mstrsm_gen(U, Vd, lam, X, outer_nb=args.outer_nb)
    elif safe:
        def solve(X):
            return P.mstrsm_safe(U, lam, X, **opts)
    elif real:
        def solve(X):
            return P.mstrsm_real(U, lam, X, outer_nb=args.outer_nb)
    elif teig:
        def solve(X):
            # X: unused placeholder (the eigenvector matrix is allocated by the call)
            teig_out["r"] = P.triang_eig(U, **opts)
    else:
        def solve(X):
            return P.mstrsm(U, lam, X, **opts)

    def fresh(k):
        return [B0.clone() for _ in range(k)]

    # ---- warmup
    for X in fresh(args.warmup):
        solve(X)
    torch.cuda.synchronize()
    log("warmup done")

    # ---- timed region: exactly `steps` solves on fresh resident inputs
    Xs = fresh(args.steps)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for X in Xs:
        solve(X)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    gflops = flops / (ms_per_step * 1e-3) / 1e9
    log("%s FP64: %.3f ms/solve, %.1f GFLOP/s" % (args.workload, ms_per_step, gflops))

    # accuracy of the timed result on sampled columns (true-modulus backward error)
    Xh = teig_out["r"][1].cpu().numpy() if teig else Xs[-1].cpu().numpy()
    cols = np.arange(0, n, max(1, n // 16))
    Ut = np.triu(w.U)
    if teig:
        ev = teig_out["r"][0].cpu().numpy()
        R = Ut @ Xh[:, cols] - Xh[:, cols] * ev[cols][None, :]
        nrm = np.full(len(cols), np.abs(Ut).sum(1).max())
    elif pencil:
        Vt = np.triu(w.extra["V"])
        R = Ut @ Xh[:, cols] - (Vt @ Xh[:, cols]) * w.shifts[cols][None, :] - w.B[:, cols]
        nrm = np.array([np.abs(Ut - w.shifts[j] * Vt).sum(1).max() for j in cols])
    else:
        R = Ut @ Xh[:, cols] - Xh[:, cols] * w.shifts[cols][None, :] - w.B[:, cols]
        offrow = np.abs(np.triu(w.U, 1)).sum(1)
        nrm = np.max(offrow[:, None] + np.abs(np.diag(w.U)[:, None] - w.shifts[cols][None, :]), axis=0)
    resid = float(np.max(np.max(np.abs(R), 0) / (nrm * np.max(np.abs(Xh[:, cols]), 0))))
    del Xs

    # ---- dominant kernel: same solves, each launch bracketed by HIP events
    Xs = fresh(args.steps)
    torch.cuda.synchronize()
    with P.profile() as pr:
        for X in Xs:
            solve(X)
    torch.cuda.synchronize()
    del Xs
    prof = pr.result
    g = prof["gemm_f64"]
    achieved = g["flops"] / (g["ms"] * 1e-3) / 1e12 if g["ms"] > 0 else 0.0
    split = {k: round(v["ms"] / args.steps, 4) for k, v in prof.items() if v["launches"]}
    launches = {k: v["launches"] // args.steps for k, v in prof.items() if v["launches"]}
    log("kernel ms/solve:", split, "launches/solve:", launches)
    roofline = {
        "bound": "mfma",
        "achieved": round(achieved, 3),
        "peak": PEAK_FP64_MFMA_TF,
        "unit": "TFLOP/s",
        "frac": round(achieved / PEAK_FP64_MFMA_TF, 4),
        "traffic": (real_gemm_traffic(m, n, args.outer_nb) if real
                    else gemm_traffic(m, n, args.nb, args.outer_nb, pencil)),
        "kernel": ("k_gemm_direct, pencil substitution C -= U X - V (lambda X) (FP64 MFMA 16x16x4)"
                   if pencil else "k_gemm_real (real substitution GEMM, FP64 MFMA 16x16x4)" if real
                   else "k_gemm_direct (substitution GEMM, FP64 MFMA 16x16x4)"),
        "avg_launch_us": round(g["ms"] * 1e3 / max(1, g["launches"]), 2),
        "flops_per_launch": g["flops"] / max(1, g["launches"]),
        "kernel_ms_per_solve": split,
        "launches_per_solve": launches,
    }

    line = {
        "metric": {"pencil": METRIC_PENCIL, "safe": METRIC_SAFE, "triang_eig": METRIC_TEIG,
                   "real": METRIC_REAL}.get(args.workload, METRIC),
        "value": round(gflops, 2),
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": ("complex128 generalized multi-shift solve (U - l_j V) X = B, FP64, "
                                "m=%d n=%d shifts (annulus-diagonal U, V diagonal in [0.5, 1.5], "
                                "shifts in disk r=0.2), inputs resident in HBM" % (m, n)) if pencil else
                               ("complex128 triangular eigenvectors (safe solve, variable-length "
                                "columns), m=%d, CN(0,1) entries with 5%% repeated eigenvalues" % m) if teig else
                               ("float64 real-arithmetic multi-shift solve, m=%d n=%d real shifts in "
                                "[-0.4, 0.4], inputs resident in HBM" % (m, n)) if real else
                               ("complex128 multi-shift solve, %s FP64, m=%d n=%d shifts (annulus-"
                                "diagonal U, shifts in disk r=0.4), inputs resident in HBM"
                                % ("safe" if safe else "plain", m, n)),
                   "m": m, "n": n, "nb": 64 if real else args.nb, "outer_nb": args.outer_nb},
        "pct_fp64_mfma_peak": round(100.0 * gflops / 1e3 / PEAK_FP64_MFMA_TF, 2),
        # the paper's own speedups, on its CPU hardware (context, not targets)
        "paper_context": {
            "multishift_vs_ztrsm": "within 1.5x of ZTRSM; 2x 4-core Xeon E5-2623 v3 (Haswell) 3.0 GHz, MKL",
            "triang_eig_vs_ztrevc": "60x at 32000^2; same Haswell, MKL",
            "eig_vs_zgeev": "3x at 32000^2; same Haswell, MKL",
            "pseudospectra_vs_eigtool": "9x at 3200^2 Fox/Li, 10000 grid points; Core i7-870 2.93 GHz, MKL",
        },
        "max_rel_residual_sampled": resid,
        "roofline": roofline,
    }

    # ---- FP32 GEMM + FP64 refinement: a fixed number of sweeps (0 = the
    # FP32-GEMM solve alone, stopped by refine_tol = 1e300; 1..3 with
    # refine_tol < 0, so no early stop), then the library's default stop
    # (refine_tol = 1e-14, at most 3 sweeps). Each row: time per solve, the
    # largest relative residual the library reports after each sweep, the
    # same measured here on sampled columns, and the difference to the FP64
    # solve; the forward error against the oracle is added by the CPU leg.
    mixed_cols = np.arange(0, n, 16)
    mixed_x = {}
    if not args.no_secondary:
        sec = {}
        Xref = P.mstrsm(U, lam, B0.clone(), **opts)
        offrow_m = np.abs(np.triu(w.U, 1)).sum(1)
        nrm_m = np.max(offrow_m[:, None] + np.abs(np.diag(w.U)[:, None] - w.shifts[mixed_cols][None, :]), axis=0)
        Ut_m = np.triu(w.U)
        for label, sweeps, tol in (("0", 1, 1e300), ("1", 1, -1.0), ("2", 2, -1.0), ("3", 3, -1.0),
                                   ("default", 3, 0.0)):
            Xs = fresh(max(2, args.steps // 2))
            rep = torch.zeros(sweeps + 1, dtype=torch.float64, device=U.device)
            P.mstrsm(U, lam, B0.clone(), precision=1, max_sweeps=sweeps, refine_tol=tol, **opts)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for X in Xs:
                P.mstrsm(U, lam, X, precision=1, max_sweeps=sweeps, refine_tol=tol, **opts)
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t0) * 1e3 / len(Xs)
            Xr = B0.clone()
            P.mstrsm(U, lam, Xr, precision=1, max_sweeps=sweeps, refine_tol=tol, refine_report=rep, **opts)
            torch.cuda.synchronize()
            fe = (torch.linalg.norm(Xs[-1] - Xref) / torch.linalg.norm(Xref)).item()
            Xh_m = Xs[-1][:, torch.from_numpy(mixed_cols).to(U.device)].cpu().numpy()
            mixed_x[label] = Xh_m
            R_m = Ut_m @ Xh_m - Xh_m * w.shifts[mixed_cols][None, :] - w.B[:, mixed_cols]
            rr_m = float(np.max(np.max(np.abs(R_m), 0) / (nrm_m * np.max(np.abs(Xh_m), 0))))
            rep_h = [float(v) for v in rep.cpu().numpy()]
            row = {"ms_per_solve": round(ms, 4), "effective_gflops": round(flops / (ms * 1e-3) / 1e9, 2),
                   "max_sweeps": sweeps, "refine_tol": tol if tol else 1e-14,
                   "report": rep_h, "sweeps_done": max(0, sum(1 for v in rep_h if v >= 0) - 1),
                   "max_rel_residual_sampled": rr_m, "rel_diff_vs_fp64": fe}
            if label in ("1", "2"):
                # executed work by kernel family: FP32 bulk against the FP32 peak,
                # residual and diagonal blocks against the FP64 peak
                Xp = B0.clone()
                torch.cuda.synchronize()
                with P.profile() as pr:
                    P.mstrsm(U, lam, Xp, precision=1, max_sweeps=sweeps, refine_tol=tol, **opts)
                torch.cuda.synchronize()
                del Xp
                brk = {}
                for k, peak in (("gemm_f32", PEAK_FP32_MFMA_TF), ("resid", PEAK_FP64_MFMA_TF),
                                ("diag", PEAK_FP64_MFMA_TF), ("aux", None)):
                    v = pr.result[k]
                    if not v["launches"]:
                        continue
                    tf = v["flops"] / (v["ms"] * 1e-3) / 1e12 if v["ms"] > 0 else 0.0
                    brk[k] = {"ms": round(v["ms"], 4), "tflops": round(tf, 2),
                              "frac_of_peak": round(tf / peak, 4) if peak else None}
                row["executed"] = brk
            sec["fp32_refine_%s" % label] = row
            del Xs, Xr
            log("fp32+%s sweeps: %.3f ms, report %s, sampled residual %.2e, rel diff vs fp64 %.2e"
                % (label, ms, rep_h, rr_m, fe))
        # context: the vendor triangular solve (one shift, lambda = 0) on the
        # same U and right-hand sides, the level-3 ceiling the method is measured against
        Ut = torch.triu(U)
        Bt = B0.clone()
        torch.linalg.solve_triangular(Ut, Bt, upper=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(3):
            torch.linalg.solve_triangular(Ut, Bt, upper=True)
        torch.cuda.synchronize()
        mt = (time.perf_counter() - t0) * 1e3 / 3
        sec["vendor_ztrsm_single_shift"] = {"ms": round(mt, 4), "gflops": round(flops / (mt * 1e-3) / 1e9, 2),
                                            "note": "torch.linalg.solve_triangular, lambda = 0 for all columns"}
        log("vendor ZTRSM (one shift): %.3f ms" % mt)
        del Ut, Bt
        # one GPU's share of a column-sharded solve: n = 512 of the 4096 shifts
        Xs = [B0[:, :512].clone() for _ in range(4)]
        ls = lam[:512].contiguous()
        P.mstrsm(U, ls, B0[:, :512].clone(), **opts)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for X in Xs:
            P.mstrsm(U, ls, X, **opts)
        torch.cuda.synchronize()
        ms5 = (time.perf_counter() - t0) * 1e3 / len(Xs)
        sec["shard_n512"] = {"ms": round(ms5, 4), "gflops": round(4.0 * m * m * 512 / (ms5 * 1e-3) / 1e9, 2)}
        log("shard shape m=%d n=512: %.3f ms" % (m, ms5))
        del Xs
        line["secondary"] = sec

    # ---- the other workloads of the path (each timed on inputs resident in HBM)
    if not args.no_secondary:
        line["workloads"] = other_workloads(P, W, torch, np)

    # ---- CPU oracle baseline on a bounded sample of the same workload
    if not args.no_cpu:
        import oracle
        cores = len(os.sched_getaffinity(0))
        env_threads = os.environ.get("OMP_NUM_THREADS")
        if env_threads and env_threads.isdigit():
            cores = min(cores, int(env_threads))
        oracle.set_num_threads(cores)
        if pencil:
            def osolve(k):
                return oracle.solve_gen(w.U, w.extra["V"], w.shifts[:k], w.B[:, :k])
        elif safe:
            def osolve(k):
                return oracle.solve_safe(w.U, w.shifts[:k], w.B[:, :k], nb=args.nb)
        elif real:
            def osolve(k):
                return oracle.solve_real(w.U, w.shifts[:k], w.B[:, :k])
        elif teig:
            def osolve(k):
                # the last k columns (the longest ones)
                sl = slice(n - k, n)
                return oracle.solve_safe(w.U, w.shifts[sl], w.B[:, sl], col_len=w.col_len[sl], nb=args.nb)
        else:
            def osolve(k):
                return oracle.solve(w.U, w.shifts[:k], w.B[:, :k])
        fpc = flops / n   # flops per shift

        def oflops(k):
            return W.nominal_flops(m, k, w.col_len[n - k:]) if teig else fpc * k
        probe = min(n, 2 * cores)
        t0 = time.perf_counter()
        osolve(probe)
        tp = time.perf_counter() - t0
        ncols = int(min(n, max(probe, probe * args.cpu_seconds / max(tp, 1e-3))))
        ncols = max(cores, (ncols // cores) * cores)
        t0 = time.perf_counter()
        osolve(ncols)
        tc = time.perf_counter() - t0
        cg = oflops(ncols) / tc / 1e9
        used = oracle.num_threads()
        # the same oracle on one thread, a smaller sample
        oracle.set_num_threads(1)
        n1 = max(1, min(ncols, int(ncols / max(1, cores) * 2)))
        t0 = time.perf_counter()
        osolve(n1)
        t1 = time.perf_counter() - t0
        oracle.set_num_threads(cores)
        line["cpu_baseline"] = {"value": round(cg, 3), "unit": "GFLOP/s", "cores": used,
                                "kind": "oracle", "cpu_model": cpu_model(),
                                "sample": "%d of %d shifts of the m=%d workload (%.1f s)" % (ncols, n, m, tc),
                                "one_thread": {"value": round(oflops(n1) / t1 / 1e9, 3),
                                               "sample": "%d shifts (%.1f s)" % (n1, t1)}}
        log("cpu oracle: %d cols in %.1fs = %.2f GFLOP/s on %d threads" % (ncols, tc, cg, cores))
        if mixed_x and not (pencil or safe or real or teig):
            # forward error of the mixed-precision rows against the oracle's FP64
            # solve on the same sampled columns
            Xo_m = oracle.solve(w.U, w.shifts[mixed_cols], w.B[:, mixed_cols])
            for label, Xh_m in mixed_x.items():
                line["secondary"]["fp32_refine_%s" % label]["forward_error_vs_oracle"] = float(
                    np.linalg.norm(Xh_m - Xo_m) / np.linalg.norm(Xo_m))
            log("mixed forward errors vs oracle:",
                {k: line["secondary"]["fp32_refine_%s" % k]["forward_error_vs_oracle"] for k in mixed_x})
        if not (pencil or safe or real or teig or args.no_secondary):
            # the oracle on the other workloads of the path, beside their GPU
            # times under "workloads": C1, C2 and the C5 forward solve in full, C4
            # on every 100th grid point (extrapolated to the whole grid)
            oc = {}

            def tm(f):
                t0 = time.perf_counter()
                f()
                return time.perf_counter() - t0
            w1 = W.c1_plain()
            t = tm(lambda: oracle.solve(w1.U, w1.shifts, w1.B))
            oc["c1_m256_n256"] = {"s": round(t, 4), "sample": "full",
                                  "gflops": round(W.nominal_flops(w1.m, w1.n) / t / 1e9, 2)}
            w2 = W.c2_triang_eig()
            t = tm(lambda: oracle.triang_eig(w2.U, nb=64))
            oc["c2_triang_eig_m2048"] = {"s": round(t, 3), "sample": "full (safe, nb = 64)",
                                         "gflops": round(W.nominal_flops(w2.m, w2.m, w2.col_len) / t / 1e9, 2)}
            w4 = W.c4_pseudospectra()
            sel = np.arange(0, w4.shifts.shape[0], 100)
            t = tm(lambda: oracle.lanczos_sigma_min(w4.U, w4.shifts[sel], w4.B[:, sel], iters=15))
            oc["c4_lanczos_m2000_N10000"] = {"s_subset": round(t, 3),
                                             "s_extrapolated": round(t * w4.shifts.shape[0] / sel.size, 2),
                                             "sample": "%d of %d shifts (every 100th), extrapolated"
                                                       % (sel.size, w4.shifts.shape[0])}
            w5 = W.c5_adjoint()
            t = tm(lambda: oracle.solve(w5.U, w5.shifts, w5.B))
            oc["c5_fwd_m4096_n2048"] = {"s": round(t, 3), "sample": "full",
                                        "gflops": round(W.nominal_flops(w5.m, w5.n) / t / 1e9, 2)}
            line["cpu_baseline"]["other_configs"] = oc
            log("cpu oracle, other configs:", oc)

    print(json.dumps(line), flush=True)
    return 0


def cpu_model() -> str:
    """The host CPU's model name (lscpu, else /proc/cpuinfo)."""
    import subprocess
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for ln in out.splitlines():
            if ln.strip().lower().startswith("model name"):
                return ln.split(":", 1)[1].strip()
    except (OSError, subprocess.SubprocessError):
        pass
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.lower().startswith("model name"):
                    return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


if __name__ == "__main__":
    sys.exit(main())
