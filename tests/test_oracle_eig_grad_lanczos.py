"""Pins for the oracle's triangular eigenvectors (Alg 6, Sec. 4), gradient of
the solve (not in the paper: reverse-mode rule of a linear solve) and inverse
Lanczos resolvent norms (Alg 7, Sec. 5)."""
import numpy as np
import pytest

import workloads as W


# ---------------------------------------------------------------- TriangEig

@pytest.mark.parametrize("nb", [0, 16, 64])
@pytest.mark.parametrize("omega_log2", [960, 100])
def test_triang_eig_eigen_relation(oracle_mod, nb, omega_log2):
    w = W.c2_triang_eig(seed=31, m=256)
    T = w.U
    lam, Z, k = oracle_mod.triang_eig(T, nb=nb, omega_log2=omega_log2)
    assert np.array_equal(lam, np.diag(T))
    assert np.all(np.isfinite(Z))
    # upper triangular with diag(Z) = s
    assert np.all(np.tril(Z, -1) == 0)
    np.testing.assert_array_equal(np.diag(Z).real, np.ldexp(1.0, -k.astype(np.int64)))
    Tn = np.max(np.sum(np.abs(T), axis=1))
    R = T @ Z - Z * lam[None, :]
    zn = np.max(np.abs(Z), axis=0)
    rel = np.max(np.abs(R), axis=0) / (Tn * np.where(zn > 0, zn, 1))
    assert rel.max() <= 1e-13
    if omega_log2 == 100:
        assert np.any(k > 0)  # growth of this workload passes 2^100


def test_triang_eig_direction_vs_numpy(oracle_mod):
    g = W.rng(32)
    m = 48
    d = W.disk_uniform(g, m, 1.0)
    T = W.random_upper(g, m, 1.0 / np.sqrt(m), d)
    lam, Z, k = oracle_mod.triang_eig(T, nb=16)
    ev, V = np.linalg.eig(T)
    for j in range(m):
        i = np.argmin(np.abs(ev - lam[j]))
        a = Z[:, j] / np.linalg.norm(Z[:, j])
        b = V[:, i] / np.linalg.norm(V[:, i])
        assert abs(np.vdot(a, b)) >= 1 - 1e-10


def test_triang_eig_repeated_eigenvalue(oracle_mod):
    # exact repeat: the pivot of column 2 at row 0 is exactly zero -> delta
    T = np.array([[1.0, 0.5, 0.25], [0, 2.0, 1.0], [0, 0, 1.0]], dtype=np.complex128)
    lam, Z, k = oracle_mod.triang_eig(np.asfortranarray(T))
    assert np.all(np.isfinite(Z))
    R = T @ Z - Z * lam[None, :]
    rel = np.max(np.abs(R), axis=0) / (np.max(np.sum(np.abs(T), 1)) * np.max(np.abs(Z), axis=0))
    assert rel.max() <= 1e-13
    # column 2 is (numerically) parallel to column 0 (defective pair)
    a = Z[:, 2] / np.linalg.norm(Z[:, 2])
    assert abs(abs(a[0]) - 1) < 1e-12


# ---------------------------------------------------------------- gradient

def _loss(U, lam, B, Wt, oracle_mod):
    X = oracle_mod.solve(np.triu(U), lam, B)
    return float(np.sum(Wt * np.abs(X) ** 2))


def test_gradient_finite_differences(oracle_mod):
    g = W.rng(33)
    m, n = 9, 4
    d = W.annulus_uniform(g, m, 0.5, 2.0)
    U = W.random_upper(g, m, 1.0 / np.sqrt(m), d)
    lam = W.disk_uniform(g, n, 0.4)
    B = np.asfortranarray(W.cnormal(g, (m, n)))
    Wt = g.standard_normal((m, n))
    X = oracle_mod.solve(U, lam, B)
    Y = oracle_mod.solve_adjoint(U, lam, 2.0 * Wt * X)
    gU, glam, gB = oracle_mod.gradient(U, lam, X, Y)
    h = 1e-6

    def fd(f, z):
        return ((f(z + h) - f(z - h)) + 1j * (f(z + 1j * h) - f(z - 1j * h))) / (2 * h)

    for (r, c) in [(0, 0), (1, 4), (3, 8), (8, 8), (2, 2), (0, 7)]:
        def f(v, r=r, c=c):
            U2 = U.copy()
            U2[r, c] = v
            return _loss(U2, lam, B, Wt, oracle_mod)
        ref = fd(f, U[r, c])
        assert abs(gU[r, c] - ref) <= 1e-6 * max(1.0, abs(ref)), (r, c)
    assert np.all(np.tril(gU, -1) == 0)
    for j in range(n):
        def f(v, j=j):
            l2 = lam.copy()
            l2[j] = v
            return _loss(U, l2, B, Wt, oracle_mod)
        ref = fd(f, lam[j])
        assert abs(glam[j] - ref) <= 1e-6 * max(1.0, abs(ref))
    for (r, c) in [(0, 0), (5, 1), (8, 3)]:
        def f(v, r=r, c=c):
            B2 = B.copy()
            B2[r, c] = v
            return _loss(U, lam, B2, Wt, oracle_mod)
        ref = fd(f, B[r, c])
        assert abs(gB[r, c] - ref) <= 1e-6 * max(1.0, abs(ref))


def test_gradient_diagonal_closed_form(oracle_mod):
    g = W.rng(34)
    m, n = 7, 3
    d = W.cnormal(g, m) + 2.0
    U = np.asfortranarray(np.diag(d))
    lam = W.cnormal(g, n) * 0.1
    B = np.asfortranarray(W.cnormal(g, (m, n)))
    Gx = np.asfortranarray(W.cnormal(g, (m, n)))
    X = oracle_mod.solve(U, lam, B)
    Y = oracle_mod.solve_adjoint(U, lam, Gx)
    gU, glam, gB = oracle_mod.gradient(U, lam, X, Y)
    A = d[:, None] - lam[None, :]
    np.testing.assert_allclose(Y, Gx / np.conj(A), rtol=1e-15)
    np.testing.assert_allclose(glam, np.sum(np.conj(B / A) * (Gx / np.conj(A)), axis=0), rtol=1e-13)
    np.testing.assert_allclose(np.diag(gU), -np.sum((Gx / np.conj(A)) * np.conj(B / A), axis=1),
                               rtol=1e-13)


# ---------------------------------------------------------------- Lanczos

def test_lanczos_diagonal_exact(oracle_mod):
    # normal (diagonal) U: sigma_min(U - zI) = min_i |d_i - z|; with m <= iters
    # the Krylov space is the whole space
    g = W.rng(35)
    m = 10
    d = W.disk_uniform(g, m, 1.0)
    U = np.asfortranarray(np.diag(d))
    z = W.disk_uniform(g, 40, 1.5)
    V0 = W.cnormal(g, (m, 40))
    sig, a, b, steps = oracle_mod.lanczos_sigma_min(U, z, V0, iters=15)
    ref = np.min(np.abs(d[:, None] - z[None, :]), axis=0)
    np.testing.assert_allclose(sig, ref, rtol=1e-8)


def test_lanczos_ritz_bound_and_svd(oracle_mod):
    w = W.c4_pseudospectra(seed=36, m=120, grid=4)
    sig, a, b, steps = oracle_mod.lanczos_sigma_min(w.U, w.shifts, w.B, iters=15)
    for j in range(w.n):
        smin = np.linalg.svd(np.triu(w.U) - w.shifts[j] * np.eye(w.m), compute_uv=False)[-1]
        assert sig[j] >= smin * (1 - 1e-10)
        assert sig[j] <= smin * 1.5  # 15 steps of Lanczos get close for this operator


def test_lanczos_first_alpha_is_rayleigh_quotient(oracle_mod):
    g = W.rng(37)
    m = 30
    U = W.random_upper(g, m, 0.2, W.disk_uniform(g, m, 1.0) + 2.0)
    z = np.array([0.1 + 0.2j, -0.3j])
    V0 = W.cnormal(g, (m, 2))
    sig, a, b, steps = oracle_mod.lanczos_sigma_min(U, z, V0, iters=3)
    for j in range(2):
        v = V0[:, j] / np.linalg.norm(V0[:, j])
        A = np.triu(U) - z[j] * np.eye(m)
        Ainv = np.linalg.inv(A)
        ref = np.real(np.vdot(v, Ainv.conj().T @ (Ainv @ v)))
        np.testing.assert_allclose(a[0, j], ref, rtol=1e-12)
