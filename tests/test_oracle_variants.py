"""Pins for the oracle's lower-triangular and transposed variants (footnote to
Sec. 2): op(A - lambda_j I) x_j = b_j, A upper or lower triangular, op in
{N, T, C}. Checked against SciPy's triangular solver (its own trans and lower
options), dense solves, diagonal closed forms, and the identities between the
variants (a lower A is the transpose of an upper one)."""
import numpy as np
import pytest
import scipy.linalg as sla

import workloads as W

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")

CASES = [(u, o) for u in "UL" for o in "NTC"]


def _tri(seed, m, n, uplo):
    w = W.c1_plain(seed=seed, m=m, n=n)
    A = w.U if uplo == "U" else np.asfortranarray(w.U.T.copy())
    return A, w.shifts, w.B


def _dense_op(A, lam, uplo, op):
    T = np.triu(A) if uplo == "U" else np.tril(A)
    E = T - lam * np.eye(A.shape[0])
    return {"N": E, "T": E.T, "C": E.conj().T}[op]


@pytest.mark.parametrize("uplo,op", CASES)
def test_against_library_triangular_solver(oracle_mod, uplo, op):
    m, n = 150, 8
    A, lam, B = _tri(50 + ord(uplo) + ord(op), m, n, uplo)
    X = oracle_mod.solve_op(A, lam, B, uplo, op)
    trans = {"N": 0, "T": 1, "C": 2}[op]
    for j in range(n):
        T = (np.triu(A) if uplo == "U" else np.tril(A)) - lam[j] * np.eye(m)
        ref = sla.solve_triangular(T, B[:, j], lower=(uplo == "L"), trans=trans)
        np.testing.assert_allclose(X[:, j], ref, rtol=1e-12, atol=1e-13 * np.abs(ref).max())


@pytest.mark.parametrize("uplo,op", CASES)
@pytest.mark.parametrize("m", [1, 2, 5, 11])
def test_brute_force_small(oracle_mod, uplo, op, m):
    A, lam, B = _tri(60 + m, m, 4, uplo)
    X = oracle_mod.solve_op(A, lam, B, uplo, op)
    for j in range(4):
        E = _dense_op(A, lam[j], uplo, op)
        ref = np.linalg.solve(E, B[:, j])
        tol = 1e-15 * np.linalg.cond(E) * 20
        assert np.max(np.abs(X[:, j] - ref)) <= tol * max(1.0, np.abs(ref).max())


@pytest.mark.parametrize("uplo,op", CASES)
def test_diagonal_closed_form_and_other_triangle_unread(oracle_mod, uplo, op):
    g = W.rng(70)
    m, n = 20, 6
    d = W.cnormal(g, m) + 2.0
    lam = W.cnormal(g, n) * 0.5
    B = np.asfortranarray(W.cnormal(g, (m, n)))
    A = np.diag(d).astype(np.complex128)
    # the triangle the variant does not use is never read
    if uplo == "U":
        A[np.tril_indices(m, -1)] = np.nan
    else:
        A[np.triu_indices(m, 1)] = np.nan
    X = oracle_mod.solve_op(np.asfortranarray(A), lam, B, uplo, op)
    piv = d[:, None] - lam[None, :]
    ref = B / (piv.conj() if op == "C" else piv)
    np.testing.assert_allclose(X, ref, rtol=1e-15, atol=0)


def test_identities_between_variants(oracle_mod):
    # a lower L = U^T: (L - l I) = (U - l I)^T, (L - l I)^T = U - l I, and the
    # conjugate variants follow; the forward/back substitution order is the same
    U, lam, B = _tri(71, 90, 7, "U")
    L = np.asfortranarray(U.T.copy())
    assert np.array_equal(oracle_mod.solve_op(L, lam, B, "L", "N"), oracle_mod.solve_op(U, lam, B, "U", "T"))
    assert np.array_equal(oracle_mod.solve_op(L, lam, B, "L", "T"), oracle_mod.solve_op(U, lam, B, "U", "N"))
    Lc = np.asfortranarray(U.conj().T.copy())
    assert np.array_equal(oracle_mod.solve_op(Lc, lam.conj(), B, "L", "N"),
                          oracle_mod.solve_op(U, lam, B, "U", "C"))
    # the standard and adjoint solves of the oracle
    np.testing.assert_allclose(oracle_mod.solve_op(U, lam, B, "U", "N"), oracle_mod.solve(U, lam, B),
                               rtol=0, atol=0)
    np.testing.assert_allclose(oracle_mod.solve_op(U, lam, B, "U", "C"),
                               oracle_mod.solve_adjoint(U, lam, B), rtol=1e-13, atol=1e-14)


def test_right_side_through_transpose(oracle_mod):
    # x_j (A - l_j I) = b_j (row vectors) is (A - l_j I)^T x_j^T = b_j^T
    A, lam, B = _tri(72, 60, 5, "U")
    Xt = oracle_mod.solve_op(A, lam, B, "U", "T")
    for j in range(5):
        r = Xt[:, j] @ (np.triu(A) - lam[j] * np.eye(60)) - B[:, j]
        assert np.abs(r).max() <= 1e-13 * np.abs(np.triu(A)).sum(0).max() * np.abs(Xt[:, j]).max()
