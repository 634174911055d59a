"""Pins for the oracle's real-arithmetic solve: (U - l_j I) x_j = b_j with U,
the shifts and B real. Checked against SciPy's triangular solver, the diagonal
closed form, dense solves, and the complex oracle on the same (real) data."""
import numpy as np
import pytest
import scipy.linalg as sla

import workloads as W


def test_real_against_library(oracle_mod):
    w = W.c10_real(seed=101, m=180, n=12)
    X = oracle_mod.solve_real(w.U, w.shifts, w.B)
    assert X.dtype == np.float64
    for j in range(12):
        ref = sla.solve_triangular(w.U - w.shifts[j] * np.eye(180), w.B[:, j], lower=False)
        np.testing.assert_allclose(X[:, j], ref, rtol=1e-12, atol=1e-13 * np.abs(ref).max())


def test_real_diagonal_closed_form_and_lower_unread(oracle_mod):
    g = W.rng(102)
    d = g.standard_normal(25) + 3.0
    lam = g.standard_normal(6)
    B = np.asfortranarray(g.standard_normal((25, 6)))
    U = np.diag(d)
    U[np.tril_indices(25, -1)] = np.nan
    X = oracle_mod.solve_real(np.asfortranarray(U), lam, B)
    assert np.array_equal(X, B / (d[:, None] - lam[None, :]))


@pytest.mark.parametrize("m", [1, 2, 5, 16])
def test_real_brute_force(oracle_mod, m):
    w = W.c10_real(seed=103 + m, m=m, n=5)
    X = oracle_mod.solve_real(w.U, w.shifts, w.B)
    for j in range(5):
        A = w.U - w.shifts[j] * np.eye(m)
        ref = np.linalg.solve(A, w.B[:, j])
        assert np.max(np.abs(X[:, j] - ref)) <= 1e-14 * np.linalg.cond(A) * max(1.0, np.abs(ref).max())


def test_real_equals_complex_oracle_on_real_data(oracle_mod):
    w = W.c10_real(seed=104, m=140, n=9)
    X = oracle_mod.solve_real(w.U, w.shifts, w.B)
    Xc = oracle_mod.solve(w.U.astype(np.complex128), w.shifts.astype(np.complex128), w.B.astype(np.complex128))
    assert np.all(Xc.imag == 0)
    np.testing.assert_allclose(X, Xc.real, rtol=1e-12, atol=1e-13 * np.abs(X).max())
