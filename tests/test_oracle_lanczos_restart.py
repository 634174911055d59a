"""Pins of the oracle's thick-restart Lanczos (the Krylov part of Alg 7,
Sec. 5, with restarts and a per-shift tolerance) against what the
mathematics fixes: the closed form for a normal (diagonal) U, dense SVDs with
restarts forced by a small basis, the Ritz-value bound sigma_est >= sigma_min,
the true residual of the returned Ritz vector against the estimate the method
stops on, and equality with the plain 15-step Lanczos when one cycle of 15
steps runs without restarting."""
import numpy as np
import pytest

import workloads as W


def _dense_sigma_min(U, z):
    m = U.shape[0]
    Ut = np.triu(U)
    return np.array([np.linalg.svd(Ut - zz * np.eye(m), compute_uv=False)[-1] for zz in z])


def test_diagonal_closed_form(oracle_mod):
    # U normal: A_z = diag(1 / |d_i - z|^2), sigma_min = min_i |d_i - z|
    g = W.rng(3)
    d = W.cnormal(g, 60)
    z = np.linspace(-1.0, 1.0, 7) + 0.3j
    V0 = W.cnormal(W.rng(4), (60, 7))
    s, r, st, c = oracle_mod.lanczos_restarted_sigma_min(np.diag(d), z, V0, kdim=10, keep=3,
                                                          max_restarts=100, tol=1e-12)
    exact = np.array([np.min(np.abs(d - zz)) for zz in z])
    assert c.all()
    np.testing.assert_allclose(s, exact, rtol=1e-12)


@pytest.mark.parametrize("kdim,keep", [(8, 3), (12, 5), (20, 6)])
def test_dense_svd_with_restarts(oracle_mod, kdim, keep):
    w = W.c4_pseudospectra(m=120, grid=4)
    s, r, st, c = oracle_mod.lanczos_restarted_sigma_min(w.U, w.shifts, w.B, kdim=kdim, keep=keep,
                                                          max_restarts=200, tol=1e-11)
    sv = _dense_sigma_min(w.U, w.shifts)
    assert c.all() and np.all(r <= 1e-11)
    if kdim == 8:
        assert st.max() > kdim       # restarts did happen
    np.testing.assert_allclose(s, sv, rtol=1e-12)
    # a Ritz value never exceeds the largest eigenvalue: sigma_est >= sigma_min
    assert np.all(s >= sv * (1 - 1e-13))


def test_residual_estimate_is_the_true_residual(oracle_mod):
    # ||A y - theta y|| / theta of the returned Ritz vector equals the estimate
    # |beta S(k-1, 0)| / theta the method stops on (up to rounding level)
    m = 120
    w = W.c4_pseudospectra(m=m, grid=4)
    s, r, st, c, Y = oracle_mod.lanczos_restarted_sigma_min(w.U, w.shifts, w.B, kdim=8, keep=3,
                                                             max_restarts=200, tol=1e-9,
                                                             return_vectors=True)
    U = np.triu(w.U)
    for j, z in enumerate(w.shifts):
        A = U - z * np.eye(m)
        y = Y[:, j] / np.linalg.norm(Y[:, j])
        Ay = np.linalg.solve(A.conj().T, np.linalg.solve(A, y))
        th = s[j] ** -2
        true = np.linalg.norm(Ay - th * y) / th
        assert true <= 1.01 * r[j] + 1e-13, (j, true, r[j])
        assert r[j] <= 1e-9


def test_one_cycle_of_15_equals_plain_lanczos(oracle_mod):
    # without a restart the Krylov space and its projection are those of the
    # plain 15-step Lanczos; full reorthogonalisation only changes rounding
    for m in (150, 600):
        w = W.c4_pseudospectra(m=m, grid=5)
        s, r, st, c = oracle_mod.lanczos_restarted_sigma_min(w.U, w.shifts, w.B, kdim=15, keep=5,
                                                              max_restarts=0, tol=0.0)
        s15, _, _, _ = oracle_mod.lanczos_sigma_min(w.U, w.shifts, w.B, iters=15)
        assert np.all(st == 15)
        np.testing.assert_allclose(s, s15, rtol=1e-12)


def test_converged_estimate_beats_fixed_steps(oracle_mod):
    # on the pseudospectra recipe at m = 300 the fixed 15 steps stop short of
    # sigma_min for some shifts; the restarted method reaches it (dense SVD)
    w = W.c4_pseudospectra(m=300, grid=6)
    s, r, st, c = oracle_mod.lanczos_restarted_sigma_min(w.U, w.shifts, w.B, tol=1e-10)
    s15, _, _, _ = oracle_mod.lanczos_sigma_min(w.U, w.shifts, w.B, iters=15)
    sv = _dense_sigma_min(w.U, w.shifts)
    assert c.all()
    err_r = np.abs(s - sv) / sv
    err_15 = np.abs(s15 - sv) / sv
    assert err_r.max() <= 1e-10
    assert err_15.max() >= 10 * err_r.max()
