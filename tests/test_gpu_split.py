"""K-split substitution GEMMs (mst_opts.gemm_split) against the oracle: each
forced split (1, 2, 4) and the automatic choice, on shapes that span several
tiles with ragged row, column and K edges, in the plain solve (K = 256 within
a group of outer blocks and the deferred K = 1024 above it), the adjoint
(conjugate-transposed A operand), the safe solve with and without
variable-length columns, mixed precision (FP32 substitution, FP64 residual)
and the triangular eigenvectors. A split fixes the order in which partial sums
are added, so two calls give the same bits; different splits agree to
rounding, each within the FP64 bars of the oracle comparison."""
import numpy as np
import pytest

import workloads as W
from gpu_util import announce, colerr, dev, host

pytestmark = pytest.mark.gpu

EPS = 2.0 ** -52
SPLITS = [1, 2, 4, 0]


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


def _kappa(U, lam, cols):
    Ut = np.triu(U)
    m = U.shape[0]
    out = []
    for j in cols:
        A = Ut - lam[j] * np.eye(m)
        out.append(np.linalg.norm(A, np.inf) * np.linalg.norm(np.linalg.inv(A), np.inf))
    return np.array(out)


@pytest.mark.parametrize("m,n", [(530, 140), (1300, 70)])
@pytest.mark.parametrize("split", SPLITS)
def test_split_plain(P, oracle_mod, m, n, split):
    announce("split plain m=%d n=%d split=%d" % (m, n, split))
    w = W.c1_plain(seed=300 + m + split, m=m, n=n)
    X = host(P.mstrsm(dev(w.U), dev(w.shifts), dev(w.B), nb=16, gemm_split=split))
    X2 = host(P.mstrsm(dev(w.U), dev(w.shifts), dev(w.B), nb=16, gemm_split=split))
    assert np.array_equal(_bits(X), _bits(X2))
    rr = oracle_mod.relative_residual(w.U, w.shifts, X, w.B)
    assert rr.max() <= 1e-13, rr.max()
    Xo = oracle_mod.solve(w.U, w.shifts, w.B)
    cols = np.arange(0, n, max(1, n // 12))
    kap = _kappa(w.U, w.shifts, cols)
    err = colerr(X[:, cols], Xo[:, cols])
    assert np.all(err <= 64 * EPS * kap), (err / (EPS * kap)).max()
    if split != 1:
        # another summation order of the same products: within two solves' bars
        X1 = host(P.mstrsm(dev(w.U), dev(w.shifts), dev(w.B), nb=16, gemm_split=1))
        assert np.all(colerr(X[:, cols], X1[:, cols]) <= 128 * EPS * kap)


@pytest.mark.parametrize("split", SPLITS)
def test_split_adjoint(P, oracle_mod, split):
    m, n = 530, 90
    announce("split adjoint split=%d" % split)
    w = W.c1_plain(seed=320 + split, m=m, n=n)
    Y = host(P.mstrsm_adjoint(dev(w.U), dev(w.shifts), dev(w.B), nb=16, gemm_split=split))
    Yo = oracle_mod.solve_adjoint(w.U, w.shifts, w.B)
    Ut = np.triu(w.U)
    for j in range(0, n, 7):
        A = (Ut - w.shifts[j] * np.eye(m)).conj().T
        r = np.abs(A @ Y[:, j] - w.B[:, j]).max()
        assert r <= 1e-13 * np.abs(A).sum(1).max() * np.abs(Y[:, j]).max()
    cols = np.arange(0, n, 9)
    kap = _kappa(w.U, w.shifts, cols)
    assert np.all(colerr(Y[:, cols], Yo[:, cols]) <= 64 * EPS * kap)


@pytest.mark.parametrize("split", SPLITS)
def test_split_safe_and_col_len(P, oracle_mod, split):
    """Safe solve of a fast-growing triangle (rescaling happens) with and
    without variable-length columns: the exponents equal the oracle's Alg 5
    and the solution agrees within the safe path's bars."""
    import torch
    g = W.rng(330)
    m, n = 450, 60
    U = W.random_upper(g, m, 1.0, W.cnormal(g, m))
    lam = W.cnormal(g, n)
    B = np.asfortranarray(W.cnormal(g, (m, n)))
    L = W.rng(331).integers(0, m + 1, n).astype(np.int32)
    announce("split safe split=%d" % split)
    X, s, k = P.mstrsm_safe(dev(U), dev(lam), dev(B), nb=16, omega_log2=40, gemm_split=split)
    Xo, so, ko = oracle_mod.solve_safe(U, lam, B, nb=16, omega_log2=40)
    X, s, k = host(X), host(s), host(k)
    assert np.array_equal(k, ko) and np.array_equal(s, so)
    assert np.any(k > 0)
    rr = oracle_mod.relative_residual(U, lam, X, B, k=k)
    assert rr.max() <= 1e-13, rr.max()
    X, s, k = P.mstrsm_safe(dev(U), dev(lam), dev(B), col_len=dev(L, dtype=torch.int32), nb=16,
                            omega_log2=40, gemm_split=split)
    Xo, so, ko = oracle_mod.solve_safe(U, lam, B, col_len=L, nb=16, omega_log2=40)
    X, k = host(X), host(k)
    assert np.array_equal(k, ko)
    for j in range(n):
        assert np.all(X[L[j]:, j] == B[L[j]:, j])   # rows past a column's length untouched
    # rows within the length: a solve of the leading L_j x L_j system
    for j in range(0, n, 5):
        lj = int(L[j])
        if lj == 0:
            continue
        A = np.triu(U[:lj, :lj]) - lam[j] * np.eye(lj)
        r = np.abs(A @ X[:lj, j] - 2.0 ** -k[j] * B[:lj, j]).max()
        assert r <= 1e-13 * np.abs(A).sum(1).max() * max(np.abs(X[:lj, j]).max(), 1e-300)


@pytest.mark.parametrize("split", SPLITS)
def test_split_mixed_precision(P, oracle_mod, split):
    """FP32 substitution GEMMs and the FP64 residual of the refinement, split
    alike: after two sweeps the FP64 bars hold."""
    w = W.c3_mixed(seed=340, m=700, n=150)
    announce("split mixed split=%d" % split)
    X = host(P.mstrsm(dev(w.U), dev(w.shifts), dev(w.B), precision=1, max_sweeps=2, refine_tol=-1.0,
                      gemm_split=split))
    X2 = host(P.mstrsm(dev(w.U), dev(w.shifts), dev(w.B), precision=1, max_sweeps=2, refine_tol=-1.0,
                       gemm_split=split))
    assert np.array_equal(_bits(X), _bits(X2))
    rr = oracle_mod.relative_residual(w.U, w.shifts, X, w.B)
    assert rr.max() <= 1e-13, rr.max()
    Xo = oracle_mod.solve(w.U, w.shifts, w.B)
    assert np.linalg.norm(X - Xo) / np.linalg.norm(Xo) <= 1e-13


@pytest.mark.parametrize("split", SPLITS)
def test_split_triang_eig(P, oracle_mod, split):
    w = W.c2_triang_eig(m=600)
    announce("split triang_eig m=600 split=%d" % split)
    ev, Z, k = P.triang_eig(dev(w.U), nb=16, gemm_split=split)
    ev, Z, k = host(ev), host(Z), host(k)
    lo, Zo, ko = oracle_mod.triang_eig(w.U, nb=16)
    assert np.array_equal(ev, lo)
    assert np.array_equal(k, ko)
    assert np.all(np.tril(Z, -1) == 0)
    T = w.U
    Tn = np.max(np.sum(np.abs(T), axis=1))
    R = T @ Z - Z * ev[None, :]
    rel = np.max(np.abs(R), axis=0) / (Tn * np.max(np.abs(Z), axis=0))
    assert rel.max() <= 1e-13, rel.max()
