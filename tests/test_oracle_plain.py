"""Pins for the oracle's plain and adjoint multi-shift solves.

Each test checks the oracle against something other than itself: a closed
form, a library triangular or dense solver, or a mathematical identity.
Problem (2) of Sec. 2: (U - lambda_j I) x_j = b_j; the adjoint solves
(U - lambda_j I)^H y_j = g_j (lower-triangular variant, footnote to Sec. 2).
"""
import numpy as np
import pytest
import scipy.linalg as sla

import workloads as W

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def _rand_problem(seed, m, n, offscale=None, shift_radius=1.5):
    g = W.rng(seed)
    d = W.disk_uniform(g, m, 1.0)
    U = W.random_upper(g, m, (1.0 / np.sqrt(m)) if offscale is None else offscale, d)
    lam = W.disk_uniform(g, n, shift_radius)
    B = np.asfortranarray(W.cnormal(g, (m, n)))
    return U, lam, B


def test_diagonal_closed_form(oracle_mod):
    # diagonal U: x = b / (d - lambda), one rounding
    g = W.rng(11)
    m, n = 37, 9
    d = W.cnormal(g, m) + 2.0
    U = np.asfortranarray(np.diag(d))
    lam = W.cnormal(g, n)
    B = np.asfortranarray(W.cnormal(g, (m, n)))
    X = oracle_mod.solve(U, lam, B)
    ref = B / (d[:, None] - lam[None, :])
    np.testing.assert_allclose(X, ref, rtol=4e-16 * 4, atol=0)


def test_zero_shift_is_trsm(oracle_mod):
    # lambda = 0 reduces to the standard triangular solve (Alg 2)
    U, _, B = _rand_problem(12, 80, 7)
    lam = np.zeros(7, dtype=np.complex128)
    X = oracle_mod.solve(U, lam, B)
    ref = sla.solve_triangular(U, B, lower=False)
    np.testing.assert_allclose(X, ref, rtol=1e-12, atol=1e-13 * np.abs(ref).max())


@pytest.mark.parametrize("m", [1, 2, 3, 5, 8, 13, 16])
def test_brute_force_small(oracle_mod, m):
    U, lam, B = _rand_problem(100 + m, m, 6, offscale=1.0)
    X = oracle_mod.solve(U, lam, B)
    for j in range(6):
        A = np.triu(U) - lam[j] * np.eye(m)
        ref = np.linalg.solve(A, B[:, j])
        cond = np.linalg.cond(A)
        tol = 1e-15 * cond * 20
        assert np.max(np.abs(X[:, j] - ref)) <= tol * max(1.0, np.abs(ref).max())


def test_residual_and_lower_triangle_ignored(oracle_mod):
    U, lam, B = _rand_problem(13, 120, 11)
    Ugarbage = U.copy(order="F")
    il = np.tril_indices(120, -1)
    Ugarbage[il] = np.nan
    X = oracle_mod.solve(Ugarbage, lam, B)
    rr = oracle_mod.relative_residual(U, lam, X, B)
    assert rr.max() <= 1e-15 * 20
    X2 = oracle_mod.solve(U, lam, B)
    assert np.array_equal(X, X2)


def test_shift_equal_to_zero_matrix_identity(oracle_mod):
    # U = c I, lambda = c - 1 => x = b
    m, n = 10, 3
    U = np.asfortranarray(np.eye(m) * (0.75 + 0.5j))
    lam = np.full(n, (0.75 + 0.5j) - 1.0)
    B = np.asfortranarray(W.cnormal(W.rng(3), (m, n)))
    X = oracle_mod.solve(U, lam, B)
    np.testing.assert_allclose(X, B, rtol=1e-15)


def test_eigen_relation_via_plain_solve(oracle_mod):
    # Sec. 4: (T11 - lambda_k I) z = -u gives T [z; 1; 0] = lambda_k [z; 1; 0]
    U, _, _ = _rand_problem(14, 50, 1)
    k = 30
    lam = np.array([U[k, k]])
    T11 = np.asfortranarray(U[:k, :k])
    z = oracle_mod.solve(T11, lam, -U[:k, k:k + 1])
    v = np.zeros(50, dtype=np.complex128)
    v[:k] = z[:, 0]
    v[k] = 1.0
    r = np.triu(U) @ v - lam[0] * v
    assert np.abs(r).max() <= 1e-13 * np.abs(U).sum(axis=1).max() * np.abs(v).max()


def test_adjoint_matches_library(oracle_mod):
    U, lam, G = _rand_problem(15, 90, 8)
    Y = oracle_mod.solve_adjoint(U, lam, G)
    for j in range(8):
        A = np.triu(U) - lam[j] * np.eye(90)
        ref = sla.solve_triangular(A.conj().T, G[:, j], lower=True)
        np.testing.assert_allclose(Y[:, j], ref, rtol=1e-12, atol=1e-13 * np.abs(ref).max())


def test_adjoint_diagonal_closed_form(oracle_mod):
    g = W.rng(16)
    m, n = 21, 5
    d = W.cnormal(g, m) + 1.5j
    U = np.asfortranarray(np.diag(d))
    lam = W.cnormal(g, n)
    G = np.asfortranarray(W.cnormal(g, (m, n)))
    Y = oracle_mod.solve_adjoint(U, lam, G)
    ref = G / np.conj(d[:, None] - lam[None, :])
    np.testing.assert_allclose(Y, ref, rtol=1e-15)


def test_adjoint_duality(oracle_mod):
    # <y, b> = <g, x> when x = A^-1 b and y = A^-H g
    U, lam, B = _rand_problem(17, 64, 6)
    G = np.asfortranarray(W.cnormal(W.rng(170), (64, 6)))
    X = oracle_mod.solve(U, lam, B)
    Y = oracle_mod.solve_adjoint(U, lam, G)
    lhs = np.sum(Y.conj() * B, axis=0)
    rhs = np.sum(G.conj() * X, axis=0)
    np.testing.assert_allclose(lhs, rhs, rtol=1e-12)


def test_empty_shapes(oracle_mod):
    U = np.zeros((0, 0), dtype=np.complex128)
    X = oracle_mod.solve(U, np.zeros(0, complex), np.zeros((0, 0), complex))
    assert X.shape == (0, 0)
    U, lam, B = _rand_problem(18, 5, 0)
    assert oracle_mod.solve(U, lam, B).shape == (5, 0)
