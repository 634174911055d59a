"""Edge cases and full-size checks across the entry points (GPU): empty
problems leave every buffer untouched; the default launch configuration of the
triangular eigenvectors and of the safe solve at the benchmark size against
the oracle with the same decision block size."""
import ctypes

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


def test_empty_problems_touch_nothing(P):
    import torch
    lib = P._lib.load()
    s = P._stream()
    B = dev(W.cnormal(W.rng(1), (5, 3)))
    keep = host(B).copy()
    U = dev(W.random_upper(W.rng(2), 5, 1.0, np.ones(5)))
    lam = dev(np.zeros(3, dtype=np.complex128))
    p = P._p
    # n = 0: nothing is read or written
    assert lib.mstrsm(5, 0, p(U), 5, p(lam), p(B), 5, None, s) == 0
    assert lib.mstrsm_adjoint(5, 0, p(U), 5, p(lam), p(B), 5, None, s) == 0
    assert lib.mstrsm_gen(5, 0, p(U), 5, p(U), 5, p(lam), p(B), 5, None, s) == 0
    assert lib.mstrsm_op(ord("L"), ord("L"), ord("N"), 5, 0, p(U), 5, p(lam), p(B), 5, None, s) == 0
    # m = 0
    assert lib.mstrsm(0, 3, None, 1, p(lam), None, 1, None, s) == 0
    assert lib.mst_triang_eig(0, None, 1, None, 1, None, None, None, s) == 0
    assert lib.mst_gen_triang_eig(0, None, 1, None, 1, None, 1, None, None, None, s) == 0
    assert lib.mst_eig_schur(0, None, 1, None, 1, None, 1, None, None, None, s) == 0
    # safe with m = 0: s_j = 1, k_j = 0
    sc = torch.full((3,), -1.0, dtype=torch.float64, device="cuda")
    kl = torch.full((3,), -1, dtype=torch.int32, device="cuda")
    assert lib.mstrsm_safe(0, 3, None, 1, p(lam), None, 1, None, p(sc), p(kl), None, s) == 0
    assert lib.mstrsm_safe_gen(0, 3, None, 1, None, 1, p(lam), None, 1, None, p(sc), p(kl), None, s) == 0
    torch.cuda.synchronize()
    assert np.all(host(sc) == 1.0) and np.all(host(kl) == 0)
    assert np.array_equal(host(B), keep)


def test_triang_eig_c2_default_configuration(P, oracle_mod):
    # the benchmark's launch configuration (nb = 16, fused outer blocks)
    w = W.c2_triang_eig()
    announce("c2 triangular eigenvectors, nb = 16")
    ev, Z, k = P.triang_eig(dev(w.U))
    ev, Z, k = host(ev), host(Z), host(k)
    lo, Zo, ko = oracle_mod.triang_eig(w.U, nb=16)
    assert np.array_equal(ev, lo)
    assert np.array_equal(k, ko), np.nonzero(k != ko)[0][:10]
    T = w.U
    R = T @ Z - Z * ev[None, :]
    rel = np.max(np.abs(R), axis=0) / (np.abs(T).sum(1).max() * np.max(np.abs(Z), axis=0))
    assert rel.max() <= 1e-13


def test_safe_full_size_sampled(P, oracle_mod):
    w = W.c3_mixed()
    announce("c3 safe 4096x4096 (sampled columns)")
    X, s, k = P.mstrsm_safe(dev(w.U), dev(w.shifts), dev(w.B))
    X, k = host(X), host(k)
    cols = np.unique(np.concatenate([np.sort(W.rng(334).choice(w.n, 16, replace=False)), [0, w.n - 1]]))
    Xo, so, ko = oracle_mod.solve_safe(w.U, w.shifts[cols], w.B[:, cols], nb=16)
    assert np.array_equal(k[cols], ko) and np.all(k == 0)
    assert colerr(X[:, cols], Xo).max() <= 1e-12
    rr = oracle_mod.relative_residual(w.U, w.shifts, X, w.B, k=k, cols=cols)
    assert rr.max() <= 1e-13


def test_ragged_large_sizes(P, oracle_mod):
    # sizes that are multiples of nothing: every block, tile and outer block ragged
    w = W.c3_mixed(seed=31, m=3001, n=2999)
    announce("plain 3001 x 2999 (sampled columns)")
    X = host(P.mstrsm(dev(w.U), dev(w.shifts), dev(w.B)))
    cols = np.array([0, 1, 15, 16, 17, 1500, 2997, 2998])
    Xo = oracle_mod.solve(w.U, w.shifts[cols], w.B[:, cols])
    assert colerr(X[:, cols], Xo).max() <= 1e-12
    rr = oracle_mod.relative_residual(w.U, w.shifts, X, w.B, cols=cols)
    assert rr.max() <= 1e-13
    Y = host(P.mstrsm_adjoint(dev(w.U), dev(w.shifts), dev(w.B)))
    Yo = oracle_mod.solve_adjoint(w.U, w.shifts[cols], w.B[:, cols])
    assert colerr(Y[:, cols], Yo).max() <= 1e-12


def test_side_stream_and_determinism(P):
    # the library only uses the stream it is given (workspace included), and
    # repeated calls give identical bits (safe and pencil forms too)
    import torch
    w = W.c6_generalized(seed=32, m=700, n=300)
    U, V, lam = dev(w.U), dev(w.extra["V"]), dev(w.shifts)
    ref = host(P.mstrsm(U, lam, dev(w.B)))
    side = torch.cuda.Stream()
    B = dev(w.B)
    torch.cuda.synchronize()
    with torch.cuda.stream(side):
        X = P.mstrsm(U, lam, B)
    side.synchronize()
    assert np.array_equal(host(X), ref)
    # safe form on a growth problem (unscaled off-diagonal) with rescaling
    g = W.rng(33)
    Ug = dev(W.random_upper(g, 700, 1.0, W.cnormal(g, 700)))
    a = P.mstrsm_safe(Ug, lam, dev(w.B), omega_log2=30)
    b = P.mstrsm_safe(Ug, lam, dev(w.B), omega_log2=30)
    assert np.array_equal(host(a[0]), host(b[0])) and np.array_equal(host(a[2]), host(b[2]))
    assert np.any(host(a[2]) > 0)
    g1 = host(P.mstrsm_gen(U, V, lam, dev(w.B)))
    g2 = host(P.mstrsm_gen(U, V, lam, dev(w.B)))
    assert np.array_equal(g1, g2)


def test_offsets_beyond_two_gib(P, oracle_mod):
    # U and B of 2.4 GB each (complex, m = n = 12288): element offsets times 16
    # bytes pass 2^31, so any 32-bit index arithmetic would show here
    import torch
    m = n = 12288
    announce("complex m = n = %d (sampled columns)" % m)
    w = W.c3_mixed(seed=31, m=m, n=n)
    Ud, ld, Bd = dev(w.U), dev(w.shifts), dev(w.B)
    X = P.mstrsm(Ud, ld, Bd)
    torch.cuda.synchronize()
    cols = [0, 1, 6143, n - 2, n - 1]
    Xs = X[:, cols].cpu().numpy()
    del Ud, Bd, X
    Xo = oracle_mod.solve(w.U, w.shifts[cols], w.B[:, cols])
    assert colerr(Xs, Xo).max() <= 1e-12
    rows = np.abs(w.U).sum(1)
    for k, j in enumerate(cols):
        r = w.U @ Xs[:, k] - w.shifts[j] * Xs[:, k] - w.B[:, j]
        nrm = (rows + np.abs(np.diag(w.U) - w.shifts[j]) - np.abs(np.diag(w.U))).max()
        assert np.abs(r).max() <= 1e-13 * nrm * np.abs(Xs[:, k]).max()
    del w
    # real, m = n = 16384 (2 GB each)
    m = n = 16384
    announce("real m = n = %d (sampled columns)" % m)
    w = W.c10_real(seed=32, m=m, n=n)
    Ur = torch.from_numpy(w.U).cuda()   # Fortran-ordered: column-major on the device
    Br = torch.from_numpy(w.B).cuda()
    Xr = P.mstrsm_real(Ur, torch.from_numpy(w.shifts).cuda(), Br)
    torch.cuda.synchronize()
    Xs = Xr[:, cols].cpu().numpy()
    del Ur, Br, Xr
    Xo = oracle_mod.solve_real(w.U, w.shifts[cols], w.B[:, cols])
    assert colerr(Xs, Xo).max() <= 1e-12


def test_nonfinite_columns_stay_isolated(P):
    # NaN and Inf in single columns of B and an exactly zero pivot for one
    # shift: those columns turn non-finite, every other column is bit-identical
    # to the solve of the clean data (the plain solve, like xTRSM, reports
    # nothing; shifts never mix)
    import torch
    m, n = 600, 70
    bad = (3, 40, 55)
    w = W.c3_mixed(seed=41, m=m, n=n)
    clean = host(P.mstrsm(dev(w.U), dev(w.shifts), dev(w.B)))
    B = w.B.copy(order="F")
    B[100, 3] = np.nan
    B[5, 40] = np.inf
    lam = w.shifts.copy()
    lam[55] = w.U[300, 300]
    X = host(P.mstrsm(dev(w.U), dev(lam), dev(B)))
    for j in range(n):
        if j in bad:
            assert not np.all(np.isfinite(X[:, j])), j
        else:
            assert np.array_equal(X[:, j], clean[:, j]), j
    # the same for the real path
    w = W.c10_real(seed=42, m=m, n=n)
    rd = lambda a: torch.from_numpy(np.asfortranarray(a)).cuda()
    clean = P.mstrsm_real(rd(w.U), rd(w.shifts), rd(w.B)).cpu().numpy()
    B = w.B.copy(order="F")
    B[100, 3] = np.nan
    B[5, 40] = np.inf
    lam = w.shifts.copy()
    lam[55] = w.U[300, 300]
    X = P.mstrsm_real(rd(w.U), rd(lam), rd(B)).cpu().numpy()
    for j in range(n):
        if j in bad:
            assert not np.all(np.isfinite(X[:, j])), j
        else:
            assert np.array_equal(X[:, j], clean[:, j]), j
