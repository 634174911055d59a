"""GPU parity of the real-arithmetic solve against the oracle: relative
residual <= 1e-13, forward agreement within 64 eps kappa_inf(U - l_j I)."""
import numpy as np
import pytest
import torch

import workloads as W
from gpu_util import announce, colerr

pytestmark = pytest.mark.gpu

EPS = 2.0 ** -52


@pytest.fixture(scope="module")
def P():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1607_01477_amd as P
    P._lib.load()
    return P


def rdev(a):
    a = np.asfortranarray(np.asarray(a, dtype=np.float64))
    if a.ndim == 1:
        return torch.from_numpy(a.copy()).cuda()
    out = torch.empty_strided(a.shape, (1, max(1, a.shape[0])), dtype=torch.float64, device="cuda")
    out.copy_(torch.from_numpy(a))
    return out


def check(oracle_mod, U, lam, B, X, cols=None):
    n = B.shape[1]
    cols = np.arange(n) if cols is None else np.asarray(cols)
    Xo = oracle_mod.solve_real(U, lam[cols], B[:, cols])
    err = colerr(X[:, cols], Xo)
    for i, j in enumerate(cols):
        A = np.triu(U) - lam[j] * np.eye(U.shape[0])
        r = np.abs(A @ X[:, j] - B[:, j]).max()
        assert r <= 1e-13 * np.abs(A).sum(1).max() * np.abs(X[:, j]).max(), j
        if U.shape[0] <= 700 and i < 16:
            kap = np.linalg.norm(A, np.inf) * np.linalg.norm(np.linalg.inv(A), np.inf)
            assert err[i] <= 64 * EPS * kap, (j, err[i] / (EPS * kap))
    if U.shape[0] > 700:
        assert err.max() <= 1e-12


@pytest.mark.parametrize("m,n", [(1, 1), (2, 3), (63, 17), (64, 64), (65, 70), (200, 33), (257, 130),
                                 (600, 96)])
@pytest.mark.parametrize("outer", [64, 256])
def test_real_shapes(P, oracle_mod, m, n, outer):
    announce("real m=%d n=%d outer=%d" % (m, n, outer))
    w = W.c10_real(seed=1000 + m + n, m=m, n=n)
    Un = w.U.copy(order="F")
    Un[np.tril_indices(m, -1)] = np.nan   # never read
    X = P.mstrsm_real(rdev(Un), rdev(w.shifts), rdev(w.B), outer_nb=outer).cpu().numpy()
    check(oracle_mod, w.U, w.shifts, w.B, X)


def test_real_full_size_sampled(P, oracle_mod):
    w = W.c10_real()
    announce("real 4096 x 4096 (sampled columns)")
    X = P.mstrsm_real(rdev(w.U), rdev(w.shifts), rdev(w.B)).cpu().numpy()
    assert np.all(np.isfinite(X))
    check(oracle_mod, w.U, w.shifts, w.B, X, cols=[0, 1, 63, 64, 2048, 4094, 4095])


def test_real_matches_complex_path(P):
    w = W.c10_real(seed=1001, m=500, n=80)
    Xr = P.mstrsm_real(rdev(w.U), rdev(w.shifts), rdev(w.B)).cpu().numpy()
    cd = lambda a: torch.from_numpy(np.asfortranarray(a.astype(np.complex128))).cuda()
    Uc = torch.empty_strided((500, 500), (1, 500), dtype=torch.complex128, device="cuda")
    Uc.copy_(cd(w.U))
    Bc = torch.empty_strided((500, 80), (1, 500), dtype=torch.complex128, device="cuda")
    Bc.copy_(cd(w.B))
    Xc = P.mstrsm(Uc, cd(w.shifts), Bc).cpu().numpy()
    assert np.all(Xc.imag == 0)
    assert colerr(Xr, Xc.real).max() <= 1e-12


def test_real_empty_problems(P):
    # m = 0 or n = 0: nothing to do, no launch, B returned as is
    for m, n in [(0, 0), (0, 5), (7, 0)]:
        U = torch.zeros((m, m), dtype=torch.float64, device="cuda").t()
        B = torch.zeros((m, n), dtype=torch.float64, device="cuda").t().contiguous().t()
        s = torch.zeros(n, dtype=torch.float64, device="cuda")
        X = P.mstrsm_real(U, s, B)
        assert X.shape == (m, n)


def test_real_deterministic_side_stream_and_padding(P):
    # bitwise equal across calls, also on a non-default stream; rows of a padded
    # leading dimension stay untouched
    w = W.c10_real(seed=1003, m=777, n=301)
    X1 = P.mstrsm_real(rdev(w.U), rdev(w.shifts), rdev(w.B)).cpu().numpy()
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        X2 = P.mstrsm_real(rdev(w.U), rdev(w.shifts), rdev(w.B))
    st.synchronize()
    assert np.array_equal(X1, X2.cpu().numpy())
    ld = 800
    Bp = torch.full((301, ld), 7.25, dtype=torch.float64, device="cuda").t()   # ld x n, column-major
    Bp[:777].copy_(torch.from_numpy(w.B))
    Xp = P.mstrsm_real(rdev(w.U), rdev(w.shifts), Bp[:777])
    torch.cuda.synchronize()
    assert Xp.data_ptr() == Bp.data_ptr()
    assert np.array_equal(Xp.cpu().numpy(), X1)
    assert torch.all(Bp[777:] == 7.25)


def _real_operator(A, lam, uplo, op):
    T = np.triu(A) if uplo == "U" else np.tril(A)
    E = T - lam * np.eye(A.shape[0])
    return E if op == "N" else E.T


@pytest.mark.parametrize("uplo,op", [(u, o) for u in "UL" for o in "NTC"])
@pytest.mark.parametrize("m,n,outer", [(1, 2, 256), (33, 17, 64), (65, 33, 256), (257, 70, 128), (600, 96, 256)])
def test_real_variants(P, oracle_mod, uplo, op, m, n, outer):
    announce("real variant %s%s m=%d n=%d outer=%d" % (uplo, op, m, n, outer))
    w = W.c10_real(seed=1100 + m + n + ord(uplo) + ord(op), m=m, n=n)
    A = w.U if uplo == "U" else np.asfortranarray(w.U.T.copy())
    An = A.copy(order="F")
    if uplo == "U":
        An[np.tril_indices(m, -1)] = np.nan   # the triangle the variant must not read
    else:
        An[np.triu_indices(m, 1)] = np.nan
    X = P.mstrsm_real_op(rdev(An), rdev(w.shifts), rdev(w.B), uplo=uplo, op=op, outer_nb=outer).cpu().numpy()
    assert np.all(np.isfinite(X))
    # the complex oracle on the same real data (for real data 'C' is 'T')
    Xo = oracle_mod.solve_op(A.astype(np.complex128), w.shifts.astype(np.complex128),
                             w.B.astype(np.complex128), uplo, op)
    assert np.all(Xo.imag == 0)
    err = colerr(X, Xo.real)
    for j in range(n):
        E = _real_operator(A, w.shifts[j], uplo, op)
        r = np.abs(E @ X[:, j] - w.B[:, j]).max()
        assert r <= 1e-13 * np.abs(E).sum(1).max() * np.abs(X[:, j]).max(), j
        if j < 16:
            kap = np.linalg.norm(E, np.inf) * np.linalg.norm(np.linalg.inv(E), np.inf)
            assert err[j] <= 64 * EPS * kap, (j, err[j] / (EPS * kap))


@pytest.mark.parametrize("uplo", "UL")
@pytest.mark.parametrize("op", "NT")
def test_real_right_side(P, oracle_mod, uplo, op):
    # x op(A - l_j I) = b_j  <=>  op(A - l_j I)^T x_j^T = b_j^T
    w = W.c10_real(seed=1200 + ord(uplo) + ord(op), m=300, n=40)
    A = w.U if uplo == "U" else np.asfortranarray(w.U.T.copy())
    X = P.mstrsm_real_op(rdev(A), rdev(w.shifts), rdev(w.B), uplo=uplo, op=op, side="R").cpu().numpy()
    Xo = oracle_mod.solve_op(A.astype(np.complex128), w.shifts.astype(np.complex128),
                             w.B.astype(np.complex128), uplo, "T" if op == "N" else "N")
    assert colerr(X, Xo.real).max() <= 1e-12
    for j in range(40):
        E = _real_operator(A, w.shifts[j], uplo, op)
        r = np.abs(X[:, j] @ E - w.B[:, j]).max()
        assert r <= 1e-13 * np.abs(E).sum(0).max() * np.abs(X[:, j]).max()


def test_real_upper_n_is_mstrsm_real_and_full_size_lower(P, oracle_mod):
    w = W.c10_real(seed=1300, m=333, n=50)
    a = P.mstrsm_real_op(rdev(w.U), rdev(w.shifts), rdev(w.B), uplo="U", op="N").cpu().numpy()
    b = P.mstrsm_real(rdev(w.U), rdev(w.shifts), rdev(w.B)).cpu().numpy()
    assert np.array_equal(a, b)
    # 4096 x 4096 lower forward solve, sampled columns against the oracle
    w = W.c10_real()
    L = np.asfortranarray(w.U.T.copy())
    X = P.mstrsm_real_op(rdev(L), rdev(w.shifts), rdev(w.B), uplo="L", op="N").cpu().numpy()
    assert np.all(np.isfinite(X))
    cols = [0, 1, 63, 64, 2048, 4095]
    Xo = oracle_mod.solve_op(L.astype(np.complex128), w.shifts[cols].astype(np.complex128),
                             w.B[:, cols].astype(np.complex128), "L", "N")
    assert colerr(X[:, cols], Xo.real).max() <= 1e-12


@pytest.mark.parametrize("m,n", [(3002, 2500), (3001, 2499)])
def test_real_large_ragged_tiles(P, oracle_mod, m, n):
    # even m: the 16-byte row-pair loads of the GEMM, with ragged edge tiles;
    # odd m (odd leading dimension): the single-row loads
    announce("real ragged m=%d n=%d" % (m, n))
    w = W.c10_real(seed=1400 + m, m=m, n=n)
    X = P.mstrsm_real(rdev(w.U), rdev(w.shifts), rdev(w.B)).cpu().numpy()
    assert np.all(np.isfinite(X))
    cols = [0, 1, 31, 32, n // 2, n - 2, n - 1]
    Xo = oracle_mod.solve_real(w.U, w.shifts[cols], w.B[:, cols])
    assert colerr(X[:, cols], Xo).max() <= 1e-12
    for k, j in enumerate(cols):
        A = np.triu(w.U) - w.shifts[j] * np.eye(m)
        r = np.abs(A @ X[:, j] - w.B[:, j]).max()
        assert r <= 1e-13 * np.abs(A).sum(1).max() * np.abs(X[:, j]).max(), j


@pytest.mark.parametrize("outer", [128, 192, 320, 512, 1024])
def test_real_outer_block_sizes(P, oracle_mod, outer):
    # fused blocks of 128 or 192 rows (outer 128, 192), 64 (outer 320), and
    # several fused blocks per outer block (outer 512, 1024)
    m, n = 1100, 300
    announce("real outer=%d m=%d n=%d" % (outer, m, n))
    w = W.c10_real(seed=1500 + outer, m=m, n=n)
    X = P.mstrsm_real(rdev(w.U), rdev(w.shifts), rdev(w.B), outer_nb=outer).cpu().numpy()
    check(oracle_mod, w.U, w.shifts, w.B, X, cols=range(0, n, 23))
