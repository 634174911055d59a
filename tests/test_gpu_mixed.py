"""Mixed precision (FP32 substitution GEMMs, FP64 diagonal blocks, FP64
iterative refinement) on the GPU, through the C-ABI, against the FP64 oracle:
right-hand sides far outside FP32's range, the device-side stop test
(refine_tol), the per-sweep residual report, and the exact undo of a sweep
that raised the residual."""
import numpy as np
import pytest

import workloads as W
from gpu_util import announce, colerr, dev, host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1607_01477_amd as P
    P._lib.load()
    return P


def _bits(X):
    return np.ascontiguousarray(X).view(np.uint64)


def _report(P, sweeps):
    import torch
    return torch.zeros(sweeps + 1, dtype=torch.float64, device="cuda")


@pytest.mark.parametrize("log2_scale", [-140, 120, 0])
def test_mixed_rhs_outside_fp32_range(P, oracle_mod, log2_scale):
    """B scaled by 2^-140 (below FP32's normal range) or 2^120 (products
    beyond it), and a mix of column scales: each column is brought near 1
    by a power of two before rounding to FP32, so the result keeps FP64
    accuracy (forward error within 64 eps kappa of the oracle's solve of
    the same scaled B, relative residual <= 1e-13)."""
    w = W.c3_mixed(seed=81, m=600, n=96)
    B = np.asfortranarray(w.B * 2.0 ** log2_scale)
    B[:, ::3] *= 2.0 ** -60    # columns of another magnitude in the same call
    announce("mixed scaled rhs 2^%d" % log2_scale)
    X = host(P.mstrsm(dev(w.U), dev(w.shifts), dev(B), precision=1, max_sweeps=3))
    Xo = oracle_mod.solve(w.U, w.shifts, B)
    assert np.all(np.isfinite(X))
    rr = oracle_mod.relative_residual(w.U, w.shifts, X, B)
    assert rr.max() <= 1e-13, rr.max()
    assert colerr(X, Xo).max() <= 1e-11


def test_refine_report_and_oracle(P, oracle_mod):
    """Three sweeps that are never stopped early (refine_tol < 0): the report
    falls sweep by sweep to the FP64 level, its entries are the largest
    relative residual the oracle measures on the returned iterates, and the
    final solution meets the FP64 bars."""
    w = W.c3_mixed(seed=82, m=900, n=120)
    announce("mixed report m=900")
    rep = {}
    X = {}
    for sweeps in (1, 2, 3):
        r = _report(P, sweeps)
        X[sweeps] = host(P.mstrsm(dev(w.U), dev(w.shifts), dev(w.B), precision=1, max_sweeps=sweeps,
                                  refine_tol=-1.0, refine_report=r))
        rep[sweeps] = host(r)
    print("report", rep[3])
    # the same iterates whatever max_sweeps is: the shorter runs' reports are prefixes
    assert np.array_equal(rep[1], rep[3][:2]) and np.array_equal(rep[2], rep[3][:3])
    r3 = rep[3]
    assert 1e-10 < r3[0] < 1e-3           # the FP32-GEMM solve alone
    assert r3[1] < r3[0]
    for s in (1, 2, 3):
        ro = oracle_mod.relative_residual(w.U, w.shifts, X[s], w.B).max()
        # the device's value and the oracle's agree to a few units in their last
        # digits only where the residual is far above rounding level
        if rep[s][s] > 1e-12:
            assert abs(ro - rep[s][s]) <= 1e-3 * ro, (s, ro, rep[s][s])
        else:
            assert ro <= 1e-13 and rep[s][s] <= 1e-13, (s, ro, rep[s][s])
    Xo = oracle_mod.solve(w.U, w.shifts, w.B)
    assert np.linalg.norm(X[3] - Xo) / np.linalg.norm(Xo) <= 1e-13


def test_refine_tol_stop_equals_fewer_sweeps(P):
    """A tolerance met after one sweep skips the rest: the result equals the
    one-sweep run bit for bit, and the report marks the skipped sweeps -1.
    refine_tol = 1 stops before the first sweep (the FP32-GEMM solve alone)."""
    w = W.c3_mixed(seed=83, m=700, n=100)
    announce("mixed refine_tol stop")
    r1 = _report(P, 1)
    X1 = host(P.mstrsm(dev(w.U), dev(w.shifts), dev(w.B), precision=1, max_sweeps=1, refine_tol=-1.0,
                       refine_report=r1))
    r1 = host(r1)
    tol = 10.0 * r1[1]
    r3 = _report(P, 3)
    X3 = host(P.mstrsm(dev(w.U), dev(w.shifts), dev(w.B), precision=1, max_sweeps=3, refine_tol=tol,
                       refine_report=r3))
    r3 = host(r3)
    assert np.array_equal(_bits(X3), _bits(X1))
    assert np.array_equal(r3[:2], r1) and np.all(r3[2:] == -1.0)
    r0 = _report(P, 2)
    X0 = host(P.mstrsm(dev(w.U), dev(w.shifts), dev(w.B), precision=1, max_sweeps=2, refine_tol=1.0,
                       refine_report=r0))
    r0 = host(r0)
    assert r0[0] == r1[0] and np.all(r0[1:] == -1.0)
    assert not np.array_equal(_bits(X0), _bits(X1))


def test_refine_undo_is_exact(P):
    """With refine_tol < 0 the loop stops only when a sweep did not lower the
    largest relative residual, and that sweep is undone: the result must then
    equal, bit for bit, the run that stops right before it (max_sweeps = t - 1,
    or refine_tol = 1e300 for the FP32-GEMM solve alone), and the report shows
    the rise followed by -1. Near FP64 rounding level the residual of a further
    sweep rises or falls by chance, so several problems are solved (well
    conditioned, c3 recipe, and an unscaled CN(0,1) triangle far too
    ill-conditioned for the FP32 solve); at least one of them must undo."""
    import torch
    undone = 0
    cases = [("c3", s) for s in range(85, 91)] + [("growth", s) for s in range(91, 95)]
    for kind, seed in cases:
        if kind == "c3":
            w = W.c3_mixed(seed=seed, m=300, n=40)
            U, lam, B = w.U, w.shifts, w.B
        else:
            g = W.rng(seed)
            U = W.random_upper(g, 64, 1.0, W.cnormal(g, 64))
            lam = W.cnormal(g, 16)
            B = np.asfortranarray(W.cnormal(g, (64, 16)))
        r = _report(P, 3)
        X = host(P.mstrsm(dev(U), dev(lam), dev(B), precision=1, max_sweeps=3, refine_tol=-1.0,
                          refine_report=r))
        r = host(r)
        rise = [t for t in range(1, 4) if r[t] >= 0 and r[t] >= r[t - 1]]
        announce("undo %s seed %d report %s" % (kind, seed, np.array2string(r, precision=3)))
        if not rise:
            assert np.all(r >= 0) and np.all(np.diff(r) < 0)
            continue
        t = rise[0]
        undone += 1
        assert np.all(r[t + 1:] == -1.0)
        if t == 1:
            Xe = host(P.mstrsm(dev(U), dev(lam), dev(B), precision=1, max_sweeps=1, refine_tol=1e300))
        else:
            Xe = host(P.mstrsm(dev(U), dev(lam), dev(B), precision=1, max_sweeps=t - 1, refine_tol=-1.0))
        assert np.array_equal(_bits(X), _bits(Xe)), (kind, seed, t)
    assert undone >= 1
