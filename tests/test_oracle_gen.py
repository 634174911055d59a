"""Pins for the oracle's generalized multi-shift solves (appendix, Alg 8, 9, 10).

Problem: (U - lambda_j V) x_j = b_j with U, V upper triangular; the safe form
solves it with s_j b_j, s_j = 2^-k_j. Each test checks the oracle against
something other than its own formula: closed forms, dense and triangular
library solvers, an independent route through the standard problem (for
nonsingular V, (U V^-1 - lambda I)(V x) = b), reduction to the separately
pinned standard solves when V = I, exact rational arithmetic on dyadic
pencils, and a hand-traced scaling example for the pencil's growth bound.
"""
from fractions import Fraction

import numpy as np
import pytest
import scipy.linalg as sla

import workloads as W

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def _pencil(seed, m, n, off=None, shift_radius=0.2):
    g = W.rng(seed)
    s = (1.0 / np.sqrt(m)) if off is None else off
    U = W.random_upper(g, m, s, W.annulus_uniform(g, m, 0.5, 2.0))
    V = W.random_upper(g, m, s, (0.5 + g.random(m)).astype(np.complex128))
    lam = W.disk_uniform(g, n, shift_radius)
    B = np.asfortranarray(W.cnormal(g, (m, n)))
    return U, V, lam, B


# ---------------------------------------------------------------- plain (Alg 8)

def test_gen_diagonal_closed_form(oracle_mod):
    g = W.rng(31)
    m, n = 29, 7
    u = W.cnormal(g, m) + 2.0
    v = W.cnormal(g, m)
    lam = W.cnormal(g, n) * 0.3
    B = np.asfortranarray(W.cnormal(g, (m, n)))
    X = oracle_mod.solve_gen(np.diag(u), np.diag(v), lam, B)
    ref = B / (u[:, None] - lam[None, :] * v[:, None])
    np.testing.assert_allclose(X, ref, rtol=1e-15, atol=0)


def test_gen_identity_v_is_standard_solve(oracle_mod):
    # V = I: every coefficient u - lambda * 0 and pivot u - lambda * 1 is
    # formed exactly, so the generalized solve is the standard one bit for bit
    U, _, lam, B = _pencil(32, 90, 11, shift_radius=1.0)
    X = oracle_mod.solve_gen(U, np.eye(90), lam, B)
    assert np.array_equal(X, oracle_mod.solve(U, lam, B))


def test_gen_zero_shift_ignores_v(oracle_mod):
    U, V, _, B = _pencil(33, 70, 5)
    lam = np.zeros(5, dtype=np.complex128)
    X = oracle_mod.solve_gen(U, V, lam, B)
    ref = sla.solve_triangular(U, B, lower=False)
    np.testing.assert_allclose(X, ref, rtol=1e-12, atol=1e-13 * np.abs(ref).max())


@pytest.mark.parametrize("m", [1, 2, 3, 5, 8, 13, 16])
def test_gen_brute_force_small(oracle_mod, m):
    U, V, lam, B = _pencil(300 + m, m, 6, off=1.0, shift_radius=0.3)
    X = oracle_mod.solve_gen(U, V, lam, B)
    for j in range(6):
        A = np.triu(U) - lam[j] * np.triu(V)
        ref = np.linalg.solve(A, B[:, j])
        tol = 1e-15 * np.linalg.cond(A) * 20
        assert np.max(np.abs(X[:, j] - ref)) <= tol * max(1.0, np.abs(ref).max())


def test_gen_matches_triangular_solver_and_lower_ignored(oracle_mod):
    m, n = 160, 9
    U, V, lam, B = _pencil(34, m, n)
    X = oracle_mod.solve_gen(U, V, lam, B)
    for j in range(n):
        ref = sla.solve_triangular(U - lam[j] * V, B[:, j], lower=False)
        np.testing.assert_allclose(X[:, j], ref, rtol=1e-12, atol=1e-13 * np.abs(ref).max())
    # strict lower triangles are never read
    Un, Vn = U.copy(order="F"), V.copy(order="F")
    Un[np.tril_indices(m, -1)] = np.nan
    Vn[np.tril_indices(m, -1)] = np.nan
    assert np.array_equal(oracle_mod.solve_gen(Un, Vn, lam, B), X)


def test_gen_route_through_standard_problem(oracle_mod):
    # nonsingular V: (U V^-1 - lambda I)(V x) = b, solved by the standard
    # oracle on W = U V^-1 (upper triangular), then x = V^-1 y
    m, n = 120, 10
    U, V, lam, B = _pencil(35, m, n)
    Wm = np.triu(sla.solve_triangular(V.T, U.T, lower=True).T)
    Y = oracle_mod.solve(np.asfortranarray(Wm), lam, B)
    ref = sla.solve_triangular(V, Y, lower=False)
    X = oracle_mod.solve_gen(U, V, lam, B)
    np.testing.assert_allclose(X, ref, rtol=1e-10, atol=1e-11 * np.abs(ref).max())


def test_gen_residual(oracle_mod):
    m, n = 300, 16
    U, V, lam, B = _pencil(36, m, n)
    X = oracle_mod.solve_gen(U, V, lam, B)
    R = U @ X - (V @ X) * lam[None, :] - B
    nrm = np.abs(U).sum(axis=1).max() + np.abs(lam).max() * np.abs(V).sum(axis=1).max()
    assert np.abs(R).max() / (nrm * np.abs(X).max()) <= 1e-15 * 10


# ---------------------------------------------------------------- safe (Alg 9)

@pytest.mark.parametrize("nb", [0, 1, 16, 64])
@pytest.mark.parametrize("omega_log2", [960, 40])
def test_safe_gen_identity_v_is_safe_solve(oracle_mod, nb, omega_log2):
    # V = I: U' is formed exactly, V(I0, I1) = 0 so the bound's V term is
    # zero, and B(I0) += 0 * C leaves B unchanged; with max cabs1(U) >= 1 the
    # zero-pivot replacement is the same too. Result: Alg 5 bit for bit,
    # rescaling decisions included.
    g = W.rng(37)
    m, n = 200, 24
    U = W.random_upper(g, m, 1.0, W.cnormal(g, m))
    lam = W.cnormal(g, n)
    B = np.asfortranarray(W.cnormal(g, (m, n)))
    assert np.abs(U.real).max() + 0 >= 1.0
    Xs, ss, ks = oracle_mod.solve_safe(U, lam, B, nb=nb, omega_log2=omega_log2)
    Xg, sg, kg = oracle_mod.solve_safe_gen(U, np.eye(m), lam, B, nb=nb, omega_log2=omega_log2)
    assert np.array_equal(ks, kg) and np.array_equal(ss, sg)
    assert np.array_equal(Xs, Xg)
    if omega_log2 == 40:
        assert np.any(kg > 0)


def test_safe_gen_unblocked_is_alg4_on_shifted_matrix(oracle_mod):
    # one block: Alg 9 is Alg 4 on U - lambda_j V formed entry by entry
    U, V, lam, B = _pencil(38, 60, 8, off=1.0, shift_radius=1.0)
    Xg, sg, kg = oracle_mod.solve_safe_gen(U, V, lam, B, nb=0, omega_log2=30)
    for j in range(8):
        # U - lambda V with each real operation rounded separately (numpy's
        # complex product may round differently)
        lr, li = lam[j].real, lam[j].imag
        Uj = np.asfortranarray((U.real - (lr * V.real - li * V.imag))
                               + 1j * (U.imag - (lr * V.imag + li * V.real)))
        x, s, k = oracle_mod.solve_safe(Uj, np.zeros(1, dtype=np.complex128), B[:, j:j + 1], nb=0,
                                        omega_log2=30)
        assert kg[j] == k[0]
        assert np.array_equal(Xg[:, j], x[:, 0])
    assert np.any(kg > 0)


@pytest.mark.parametrize("lam", [2.0 ** 600, 1j * 2.0 ** 600])
@pytest.mark.parametrize("nb", [0, 1])
def test_safe_gen_hand_traced_pencil_bound(oracle_mod, lam, nb):
    # U = I, V = [[0, 1], [0, 0]], b = (0, 2^500), Omega = 2^960.
    # nb = 1: row 1 gives x1 = 2^500 (pivot 1 - lam * 0 = 1, no rescale);
    # the bound G = 2^500 + (0 + |lam| * 1) * 2^500 overflows; from the
    # exponents E = max(500, 600 + 500 + 1) + 1 = 1102, k = 1103 - 960 = 143,
    # so x1 = 2^357; then C = lam x1 (|C| = 2^957) and b0 = 0 - 0 * x1 + 1 * C.
    # Row 0: x0 = lam 2^357, below Omega. Without the |lam| ||V|| term of the
    # bound, C = lam 2^500 would overflow.
    # nb = 0: Alg 4 on [[1, -lam], [0, 1]] with column norm 2^600 reaches the
    # same k in its growth check.
    U = np.eye(2, dtype=np.complex128)
    V = np.array([[0, 1], [0, 0]], dtype=np.complex128)
    b = np.array([[0], [2.0 ** 500]], dtype=np.complex128)
    X, s, k = oracle_mod.solve_safe_gen(U, V, np.array([lam]), b, nb=nb)
    assert int(k[0]) == 143 and s[0] == 2.0 ** -143
    assert X[1, 0] == 2.0 ** 357
    assert X[0, 0] == lam * 2.0 ** 357


def _dyadic_pencil(seed, m, n):
    """Entries in {0, +-1, +-i}; diagonal of U chosen so that every pivot
    u - lambda v is +-2^-2 or +-i 2^-2 for the shift lambda in {+-1, +-i} of
    each column (one shift per column, same for all here); integer b.
    Every operation of back substitution is exact in binary64."""
    g = W.rng(seed)
    units = np.array([1, -1, 1j, -1j, 0], dtype=np.complex128)
    lamv = units[g.integers(0, 4)]
    U = np.zeros((m, m), dtype=np.complex128)
    V = np.zeros((m, m), dtype=np.complex128)
    for c in range(m):
        for r in range(c):
            U[r, c] = units[g.integers(0, 5)]
            V[r, c] = units[g.integers(0, 5)]
        V[c, c] = units[g.integers(0, 4)]
        U[c, c] = units[g.integers(0, 4)] * 0.25 + lamv * V[c, c]
    lam = np.full(n, lamv, dtype=np.complex128)
    B = (g.integers(-3, 4, (m, n)) + 1j * g.integers(-3, 4, (m, n))).astype(np.complex128)
    return np.asfortranarray(U), np.asfortranarray(V), lam, np.asfortranarray(B)


def _exact_solve(A, b):
    m = A.shape[0]
    F = lambda v: (Fraction(v.real), Fraction(v.imag))
    x = [None] * m
    bb = [F(v) for v in b]
    for i in range(m - 1, -1, -1):
        br, bi = bb[i]
        for k in range(i + 1, m):
            ur, ui = F(A[i, k])
            xr, xi = x[k]
            br -= ur * xr - ui * xi
            bi -= ur * xi + ui * xr
        dr, di = F(A[i, i])
        den = dr * dr + di * di
        x[i] = ((br * dr + bi * di) / den, (bi * dr - br * di) / den)
    return x


@pytest.mark.parametrize("nb", [0, 1, 3, 4, 16])
@pytest.mark.parametrize("omega_log2", [8, 14, 960])
@pytest.mark.parametrize("m", [10, 20])
def test_safe_gen_dyadic_exact(oracle_mod, nb, omega_log2, m):
    # (for larger m the exact solutions need more than 53 significant bits)
    n = 4
    U, V, lam, B = _dyadic_pencil(40 + omega_log2 + nb + m, m, n)
    X, s, k = oracle_mod.solve_safe_gen(U, V, lam, B, nb=nb, omega_log2=omega_log2)
    events = 0
    for j in range(n):
        xt = _exact_solve(U - lam[j] * V, B[:, j])
        kj = int(k[j])
        events += kj > 0
        for i in range(m):
            ex = complex(float(xt[i][0] * Fraction(2) ** (-kj)), float(xt[i][1] * Fraction(2) ** (-kj)))
            assert X[i, j] == ex, (j, i, kj)
        assert np.max(np.abs(X[:, j].real) + np.abs(X[:, j].imag)) < 2.0 ** (omega_log2 + 1)
    if omega_log2 <= 8:
        assert events > 0


@pytest.mark.parametrize("nb", [0, 16, 64])
def test_safe_gen_residual_and_phase2_invariance(oracle_mod, nb):
    # growth: unscaled off-diagonals; a small Omega forces rescaling
    U, V, lam, B = _pencil(41, 250, 16, off=1.0, shift_radius=1.0)
    for omega_log2 in (960, 60):
        X, s, k = oracle_mod.solve_safe_gen(U, V, lam, B, nb=nb, omega_log2=omega_log2)
        X2, s2, k2 = oracle_mod.solve_safe_gen(U, V, lam, B, nb=nb, omega_log2=omega_log2,
                                               force_phase2=True)
        assert np.array_equal(X, X2) and np.array_equal(k, k2)
        assert np.all(np.isfinite(X))
        Bs = B * np.ldexp(1.0, -k.astype(np.int64))[None, :]
        R = U @ X - (V @ X) * lam[None, :] - Bs
        for j in range(16):
            A = U - lam[j] * V
            den = np.abs(A).sum(axis=1).max() * np.abs(X[:, j]).max()
            assert np.abs(R[:, j]).max() <= 1e-13 * den
        if omega_log2 == 60:
            assert np.any(k > 0)
        else:
            np.testing.assert_allclose(X, oracle_mod.solve_gen(U, V, lam, B), rtol=1e-9,
                                       atol=1e-12 * np.abs(X).max())


def test_safe_gen_col_len_equals_zero_padded(oracle_mod):
    U, V, lam, B = _pencil(42, 130, 20, off=1.0, shift_radius=1.0)
    g = W.rng(420)
    L = g.integers(0, 131, 20).astype(np.int32)
    L[:3] = [0, 130, 64]
    Bz = B.copy(order="F")
    for j in range(20):
        Bz[L[j]:, j] = 0
    for nb in (0, 16, 64):
        Xa, sa, ka = oracle_mod.solve_safe_gen(U, V, lam, B, col_len=L, nb=nb)
        Xb, sb, kb = oracle_mod.solve_safe_gen(U, V, lam, Bz, nb=nb)
        assert np.array_equal(ka, kb)
        for j in range(20):
            assert np.array_equal(Xa[:L[j], j], Xb[:L[j], j])
            assert np.array_equal(Xa[L[j]:, j], B[L[j]:, j])


# ---------------------------------------------------------------- GeneralizedTriangEig (Alg 10)

def test_gen_triang_eig_identity_s_is_triang_eig(oracle_mod):
    w = W.c2_triang_eig(m=160, dup_frac=0.0)
    T = w.U
    assert np.abs(T).max() >= 1.0
    lam1, Z1, k1 = oracle_mod.triang_eig(T)
    lam2, Z2, k2 = oracle_mod.gen_triang_eig(T, np.eye(160))
    assert np.array_equal(lam1, lam2) and np.array_equal(k1, k2)
    assert np.array_equal(Z1, Z2)


def test_gen_triang_eig_eigenpairs(oracle_mod):
    w = W.c7_gen_triang_eig(m=120)
    T, S = w.U, w.extra["S"]
    lam, Z, k = oracle_mod.gen_triang_eig(T, S)
    assert np.all(np.tril(Z, -1) == 0)
    assert np.array_equal(np.diag(Z), np.ldexp(1.0, -k.astype(np.int64)))
    R = T @ Z - (S @ Z) * lam[None, :]
    nrm = np.abs(T).sum(axis=1).max() + np.abs(lam)[None, :] * np.abs(S).sum(axis=1).max()
    rel = np.abs(R).max(axis=0) / (nrm[0] * np.abs(Z).max(axis=0))
    assert rel.max() <= 1e-13
    # eigenvalues against the library's QZ-based solver
    ev = sla.eigvals(T, S)
    assert np.all(np.min(np.abs(ev[None, :] - lam[:, None]), axis=1) <= 1e-10 * np.abs(lam).max())
