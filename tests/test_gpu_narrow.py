"""Fused outer blocks with 4, 2 or 1 shifts per workgroup (mst_opts.fuse_blocks
= 2, 3 or 4, chosen automatically when 16-shift workgroups would leave compute
units idle) against the oracle: plain solves on shapes with partial outer and diagonal
blocks and shift counts that are not multiples of 4, the safe solve with
rescaling, variable-length columns and the triangular eigenvectors (exponents
equal to the oracle's Alg 5), mixed precision, the lower-triangular,
transposed and conjugated variants and the adjoint (forward substitution,
the other triangle filled with NaN), the automatic choice, agreement with
the 16-shift kernel to rounding, and the same bits at every narrow width."""
import numpy as np
import pytest

import workloads as W
from gpu_util import announce, colerr, dev, host

pytestmark = pytest.mark.gpu

EPS = 2.0 ** -52


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


@pytest.mark.parametrize("m,n,outer", [(1, 1, 256), (17, 5, 256), (256, 4, 256), (530, 70, 256),
                                       (1000, 37, 128), (700, 9, 64), (300, 11, 512), (530, 70, 512),
                                       (1100, 23, 512)])
@pytest.mark.parametrize("width", [4, 2, 1])
def test_narrow_plain(P, oracle_mod, m, n, outer, width):
    announce("narrow w%d " % width + "plain m=%d n=%d outer=%d" % (m, n, outer))
    w = W.c1_plain(seed=400 + m + n, m=m, n=n)
    X = host(P.mstrsm(dev(w.U), dev(w.shifts), dev(w.B), nb=16, outer_nb=outer, fuse_width=width))
    X2 = host(P.mstrsm(dev(w.U), dev(w.shifts), dev(w.B), nb=16, outer_nb=outer, fuse_width=width))
    assert np.array_equal(_bits(X), _bits(X2))
    rr = oracle_mod.relative_residual(w.U, w.shifts, X, w.B)
    assert rr.max() <= 1e-13, rr.max()
    Xo = oracle_mod.solve(w.U, w.shifts, w.B)
    cols = np.arange(0, n, max(1, n // 10))
    kap = _kappa(w.U, w.shifts, cols)
    assert np.all(colerr(X[:, cols], Xo[:, cols]) <= 64 * EPS * kap)
    X16 = host(P.mstrsm(dev(w.U), dev(w.shifts), dev(w.B), nb=16, outer_nb=outer, fuse_width=16))
    assert np.all(colerr(X[:, cols], X16[:, cols]) <= 128 * EPS * kap)


def test_narrow_automatic_choice(P):
    """Few shifts: the automatic width is a narrow one (same bits as forced 2,
    unlike 16), in the back and the forward substitution, with 512-row outer
    blocks in plain back substitutions; 4096 shifts fill the device with
    16-shift workgroups (same bits as forced 16)."""
    w = W.c1_plain(seed=410, m=300, n=40)
    args = (dev(w.U), dev(w.shifts))
    Xa = host(P.mstrsm(*args, dev(w.B), nb=16))
    X2 = host(P.mstrsm(*args, dev(w.B), nb=16, fuse_width=2))
    X16 = host(P.mstrsm(*args, dev(w.B), nb=16, fuse_width=16))
    assert np.array_equal(_bits(Xa), _bits(X2))
    assert not np.array_equal(_bits(Xa), _bits(X16))
    Ya = host(P.mstrsm_adjoint(*args, dev(w.B), nb=16))
    Y2 = host(P.mstrsm_adjoint(*args, dev(w.B), nb=16, fuse_width=2))
    Y16 = host(P.mstrsm_adjoint(*args, dev(w.B), nb=16, fuse_width=16))
    assert np.array_equal(_bits(Ya), _bits(Y2))
    assert not np.array_equal(_bits(Ya), _bits(Y16))
    # few shifts, plain FP64, outer block left to the library: 512 rows (the
    # same bits as forced 512; 256-row blocks group the products otherwise)
    w = W.c1_plain(seed=412, m=1100, n=23)
    args = (dev(w.U), dev(w.shifts))
    Xa = host(P.mstrsm(*args, dev(w.B), nb=16))
    X512 = host(P.mstrsm(*args, dev(w.B), nb=16, outer_nb=512, fuse_width=2))
    X256 = host(P.mstrsm(*args, dev(w.B), nb=16, outer_nb=256, fuse_width=2))
    assert np.array_equal(_bits(Xa), _bits(X512))
    assert not np.array_equal(_bits(Xa), _bits(X256))
    Ya = host(P.mstrsm_adjoint(*args, dev(w.B), nb=16))
    Y256 = host(P.mstrsm_adjoint(*args, dev(w.B), nb=16, outer_nb=256, fuse_width=1))
    assert np.array_equal(_bits(Ya), _bits(Y256))   # forward substitution keeps 256
    w = W.c1_plain(seed=411, m=300, n=4096)
    args = (dev(w.U), dev(w.shifts))
    Xa = host(P.mstrsm(*args, dev(w.B), nb=16))
    X16 = host(P.mstrsm(*args, dev(w.B), nb=16, fuse_width=16))
    assert np.array_equal(_bits(Xa), _bits(X16))


@pytest.mark.parametrize("omega_log2", [960, 40])
@pytest.mark.parametrize("width", [4, 2, 1])
def test_narrow_safe_growth(P, oracle_mod, omega_log2, width):
    g = W.rng(420)
    m, n = 450, 30
    U = W.random_upper(g, m, 1.0, W.cnormal(g, m))
    lam = W.cnormal(g, n)
    B = np.asfortranarray(W.cnormal(g, (m, n)))
    announce("narrow w%d " % width + "safe omega 2^%d" % omega_log2)
    X, s, k = P.mstrsm_safe(dev(U), dev(lam), dev(B), nb=16, omega_log2=omega_log2, fuse_width=width)
    X, s, k = host(X), host(s), host(k)
    Xo, so, ko = oracle_mod.solve_safe(U, lam, B, nb=16, omega_log2=omega_log2)
    assert np.array_equal(k, ko) and np.array_equal(s, so)
    if omega_log2 == 40:
        assert np.any(k > 0)
    assert np.all(np.isfinite(X))
    rr = oracle_mod.relative_residual(U, lam, X, B, k=k)
    assert rr.max() <= 1e-13, rr.max()
    # forced checked steps: the same bits
    Xf, sf, kf = P.mstrsm_safe(dev(U), dev(lam), dev(B), nb=16, omega_log2=omega_log2, fuse_width=width,
                               force_phase2=True)
    assert np.array_equal(_bits(host(Xf)), _bits(X)) and np.array_equal(host(kf), k)


@pytest.mark.parametrize("width", [4, 2, 1])
def test_narrow_col_len(P, oracle_mod, width):
    """Variable-length columns, including lengths 0, 1, m and columns whose
    workgroup has no column reaching an outer block (early exit)."""
    import torch
    g = W.rng(430)
    m, n = 600, 41
    U = W.random_upper(g, m, 1.0, W.cnormal(g, m))
    lam = W.cnormal(g, n)
    B = np.asfortranarray(W.cnormal(g, (m, n)))
    L = np.sort(W.rng(431).integers(0, m + 1, n)).astype(np.int32)
    L[:5] = [0, 1, 3, 16, 17]
    L[-1] = m
    announce("narrow w%d " % width + "col_len")
    X, s, k = P.mstrsm_safe(dev(U), dev(lam), dev(B), col_len=dev(L, dtype=torch.int32), nb=16,
                            omega_log2=50, fuse_width=width)
    X, k = host(X), host(k)
    Xo, so, ko = oracle_mod.solve_safe(U, lam, B, col_len=L, nb=16, omega_log2=50)
    assert np.array_equal(k, ko)
    for j in range(n):
        assert np.array_equal(X[L[j]:, j], B[L[j]:, j])
        if L[j] > 0:
            e = np.abs(X[:L[j], j] - Xo[:L[j], j]).max() / max(np.abs(Xo[:L[j], j]).max(), 1e-300)
            assert e <= 1e-8, (j, e)


@pytest.mark.parametrize("m", [600, 2048])
@pytest.mark.parametrize("width", [4, 2, 1])
def test_narrow_triang_eig(P, oracle_mod, m, width):
    w = W.c2_triang_eig(m=m)
    announce("narrow w%d " % width + "triang_eig m=%d" % m)
    ev, Z, k = P.triang_eig(dev(w.U), nb=16, fuse_width=width)
    ev, Z, k = host(ev), host(Z), host(k)
    lo, Zo, ko = oracle_mod.triang_eig(w.U, nb=16)
    assert np.array_equal(ev, lo)
    mism = np.nonzero(k != ko)[0]
    assert len(mism) == 0, (mism[:10], k[mism[:10]], ko[mism[:10]])
    if m == 2048:
        assert np.any(k > 0)   # the full-size recipe rescales (at m = 600 nothing does)
    assert np.all(np.tril(Z, -1) == 0)
    T = w.U
    Tn = np.max(np.sum(np.abs(T), axis=1))
    R = T @ Z - Z * ev[None, :]
    rel = np.max(np.abs(R), axis=0) / (Tn * np.max(np.abs(Z), axis=0))
    assert rel.max() <= 1e-13, rel.max()


@pytest.mark.parametrize("width", [4, 2, 1])
def test_narrow_mixed_precision(P, oracle_mod, width):
    w = W.c3_mixed(seed=440, m=700, n=60)
    announce("narrow w%d " % width + "mixed")
    X = host(P.mstrsm(dev(w.U), dev(w.shifts), dev(w.B), precision=1, max_sweeps=2, refine_tol=-1.0,
                      fuse_width=width))
    rr = oracle_mod.relative_residual(w.U, w.shifts, X, w.B)
    assert rr.max() <= 1e-13, rr.max()
    Xo = oracle_mod.solve(w.U, w.shifts, w.B)
    assert np.linalg.norm(X - Xo) / np.linalg.norm(Xo) <= 1e-13


def _operator(A, lam, uplo, op):
    T = np.triu(A) if uplo == "U" else np.tril(A)
    E = T - lam * np.eye(A.shape[0])
    return {"N": E, "T": E.T, "C": E.conj().T}[op]


@pytest.mark.parametrize("uplo,op", [(u, o) for u in "UL" for o in "NTC"])
@pytest.mark.parametrize("width", [4, 2, 1])
def test_narrow_variants(P, oracle_mod, uplo, op, width):
    """op(A - l_j I) x_j = b_j for A upper or lower and op N, T, C with 4-shift
    fused blocks (forward substitution for lower N and upper T/C): residual,
    oracle agreement, the unread triangle NaN, and agreement with the 16-shift
    kernel."""
    m, n = 530, 37
    w = W.c1_plain(seed=450 + ord(uplo) + ord(op), m=m, n=n)
    A = w.U if uplo == "U" else np.asfortranarray(w.U.T.copy())
    An = A.copy(order="F")
    if uplo == "U":
        An[np.tril_indices(m, -1)] = np.nan
    else:
        An[np.triu_indices(m, 1)] = np.nan
    announce("narrow w%d " % width + "variant %s%s" % (uplo, op))
    X = host(P.mstrsm_op(dev(An), dev(w.shifts), dev(w.B), uplo=uplo, op=op, nb=16, fuse_width=width))
    assert np.all(np.isfinite(X))
    Xo = oracle_mod.solve_op(A, w.shifts, w.B, uplo, op)
    X16 = host(P.mstrsm_op(dev(An), dev(w.shifts), dev(w.B), uplo=uplo, op=op, nb=16, fuse_width=16))
    for j in range(n):
        E = _operator(A, w.shifts[j], uplo, op)
        r = np.abs(E @ X[:, j] - w.B[:, j]).max()
        assert r <= 1e-13 * np.abs(E).sum(1).max() * np.abs(X[:, j]).max(), j
        if j % 6 == 0:
            kap = np.linalg.norm(E, np.inf) * np.linalg.norm(np.linalg.inv(E), np.inf)
            assert colerr(X[:, j:j + 1], Xo[:, j:j + 1])[0] <= 64 * EPS * kap
            assert colerr(X[:, j:j + 1], X16[:, j:j + 1])[0] <= 128 * EPS * kap


@pytest.mark.parametrize("width", [4, 2, 1])
def test_narrow_adjoint(P, oracle_mod, width):
    m, n = 600, 50
    w = W.c1_plain(seed=460, m=m, n=n)
    announce("narrow w%d " % width + "adjoint")
    Y = host(P.mstrsm_adjoint(dev(w.U), dev(w.shifts), dev(w.B), nb=16, fuse_width=width))
    Y2 = host(P.mstrsm_adjoint(dev(w.U), dev(w.shifts), dev(w.B), nb=16, fuse_width=width))
    assert np.array_equal(_bits(Y), _bits(Y2))
    Yo = oracle_mod.solve_adjoint(w.U, w.shifts, w.B)
    Ut = np.triu(w.U)
    for j in range(0, n, 5):
        A = (Ut - w.shifts[j] * np.eye(m)).conj().T
        r = np.abs(A @ Y[:, j] - w.B[:, j]).max()
        assert r <= 1e-13 * np.abs(A).sum(1).max() * np.abs(Y[:, j]).max()
    cols = np.arange(0, n, 7)
    kap = _kappa(w.U, w.shifts, cols)
    assert np.all(colerr(Y[:, cols], Yo[:, cols]) <= 64 * EPS * kap)


def test_narrow_widths_same_bits(P):
    """4-, 2- and 1-shift workgroups take the same steps for each shift: the
    same bits in the plain solve, the safe solve with rescaling (and the same
    exponents) and the adjoint at one outer block size (256 rows; 512 for the
    widths that take it)."""
    widths = (4, 2, 1)
    w = W.c1_plain(seed=470, m=1100, n=23)
    announce("narrow widths same bits")
    X = [host(P.mstrsm(dev(w.U), dev(w.shifts), dev(w.B), nb=16, outer_nb=256, fuse_width=c)) for c in widths]
    Y = [host(P.mstrsm_adjoint(dev(w.U), dev(w.shifts), dev(w.B), nb=16, outer_nb=256, fuse_width=c))
         for c in widths]
    X5 = [host(P.mstrsm(dev(w.U), dev(w.shifts), dev(w.B), nb=16, outer_nb=512, fuse_width=c)) for c in (2, 1)]
    Y5 = [host(P.mstrsm_adjoint(dev(w.U), dev(w.shifts), dev(w.B), nb=16, outer_nb=512, fuse_width=c))
          for c in (2, 1)]
    assert np.array_equal(_bits(X5[0]), _bits(X5[1]))
    assert np.array_equal(_bits(Y5[0]), _bits(Y5[1]))
    g = W.rng(471)
    m, n = 450, 19
    U = W.random_upper(g, m, 1.0, W.cnormal(g, m))
    lam = W.cnormal(g, n)
    B = np.asfortranarray(W.cnormal(g, (m, n)))
    R = [P.mstrsm_safe(dev(U), dev(lam), dev(B), nb=16, omega_log2=40, fuse_width=c) for c in widths]
    assert np.any(host(R[0][2]) > 0)
    for i in (1, 2):
        assert np.array_equal(_bits(X[0]), _bits(X[i]))
        assert np.array_equal(_bits(Y[0]), _bits(Y[i]))
        assert np.array_equal(_bits(host(R[0][0])), _bits(host(R[i][0])))
        assert np.array_equal(host(R[0][2]), host(R[i][2]))


@pytest.mark.parametrize("width", [2, 1])
def test_narrow_512_rows_forward_and_safe(P, oracle_mod, width):
    """512-row outer blocks forced in the forward substitution (adjoint; the
    library keeps 256 there unless asked) against the oracle, and a forced
    outer_nb = 512 in the safe solve, which the fused kernels do not take
    (per-block path), with exponents equal to the oracle's."""
    m, n = 1100, 23
    w = W.c1_plain(seed=480 + width, m=m, n=n)
    announce("narrow w%d 512-row adjoint and safe" % width)
    Y = host(P.mstrsm_adjoint(dev(w.U), dev(w.shifts), dev(w.B), nb=16, outer_nb=512, fuse_width=width))
    Yo = oracle_mod.solve_adjoint(w.U, w.shifts, w.B)
    cols = np.arange(0, n, 4)
    kap = _kappa(w.U, w.shifts, cols)
    assert np.all(colerr(Y[:, cols], Yo[:, cols]) <= 64 * EPS * kap)
    g = W.rng(490)
    U = W.random_upper(g, 600, 1.0, W.cnormal(g, 600))
    lam = W.cnormal(g, 17)
    B = np.asfortranarray(W.cnormal(g, (600, 17)))
    X, s, k = P.mstrsm_safe(dev(U), dev(lam), dev(B), nb=16, outer_nb=512, omega_log2=40, fuse_width=width)
    Xo, so, ko = oracle_mod.solve_safe(U, lam, B, nb=16, omega_log2=40)
    assert np.array_equal(host(k), ko) and np.array_equal(host(s), so)
    rr = oracle_mod.relative_residual(U, lam, host(X), B, k=host(k))
    assert rr.max() <= 1e-13, rr.max()
