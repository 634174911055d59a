"""GPU pseudospectra drivers (Sec. 5; the window / portrait / cloud shapes):
the resolvent-norm grid against the oracle's Lanczos on the same grid and
start vectors, and the Ritz inequality against dense SVDs."""
import numpy as np
import pytest
import scipy.linalg as sla

import workloads as W
from gpu_util import announce, dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1607_01477_amd as P
    P._lib.load()
    return P


def test_portrait_triangular_against_oracle(P, oracle_mod):
    from paper_1607_01477_amd import pseudospectra as PS
    w = W.c4_pseudospectra(m=200, grid=2)
    announce("spectral portrait m=200 grid 10x12")
    xs, ys, sigma, eigs = PS.spectral_portrait(dev(w.U), nx=10, ny=12, triangular=True, seed=3)
    assert sigma.shape == (12, 10)
    z = oracle_mod.portrait_grid(np.diag(w.U), 10, 12)
    V0 = PS._start_vectors(200, 120, 3, "cpu").numpy()
    so, _, _, _ = oracle_mod.lanczos_sigma_min(w.U, z, V0, iters=15)
    np.testing.assert_allclose(sigma.reshape(-1), so, rtol=1e-8)


def test_portrait_dense_ritz_bound(P):
    from paper_1607_01477_amd import pseudospectra as PS
    A = W.c8_dense_eig(seed=83, m=120).extra["A"]
    xs, ys, sigma, eigs = PS.spectral_portrait(dev(A), nx=6, ny=6)
    # sigma_min(A - zI) = sigma_min(T - zI); the Lanczos value bounds it from above
    for iy in range(6):
        for ix in range(6):
            zz = xs[ix] + 1j * ys[iy]
            smin = np.linalg.svd(A - zz * np.eye(120), compute_uv=False)[-1]
            assert sigma[iy, ix] >= smin * (1 - 1e-10)
            assert sigma[iy, ix] <= 1.5 * smin
    ev = np.linalg.eigvals(A)
    assert np.max(np.min(np.abs(eigs[:, None] - ev[None, :]), axis=1)) < 1e-10


def test_window_and_cloud(P, oracle_mod):
    from paper_1607_01477_amd import pseudospectra as PS
    w = W.c4_pseudospectra(m=150, grid=2)
    xs, ys, sigma = PS.spectral_window(dev(w.U), 0.2 + 0.1j, 1.0, 0.5, nx=7, ny=5, seed=5)
    _, _, z = PS.window_grid(0.2 + 0.1j, 1.0, 0.5, 7, 5)
    V0 = PS._start_vectors(150, 35, 5, "cpu").numpy()
    so, _, _, _ = oracle_mod.lanczos_sigma_min(w.U, z, V0, iters=15)
    np.testing.assert_allclose(sigma.reshape(-1), so, rtol=1e-8)
    c = PS.spectral_cloud(dev(w.U), z[:4], V0=dev(V0[:, :4]))
    np.testing.assert_allclose(c.cpu().numpy(), so[:4], rtol=1e-8)


# ------------------------------------------------------------------ restarted Lanczos

def _host(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy()


@pytest.mark.parametrize("kdim,keep", [(8, 3), (20, 6)])
def test_restarted_against_oracle(P, oracle_mod, kdim, keep):
    """Thick-restart Lanczos on the GPU against the oracle's, same grid and
    start vectors: sigma to 1e-10 (both converge to 1e-11 in the residual),
    the same number of steps per shift, every shift converged; and against
    dense SVDs."""
    w = W.c4_pseudospectra(m=150, grid=6)
    announce("restarted lanczos m=150 kdim=%d keep=%d" % (kdim, keep))
    s, r, st, c = (_host(t) for t in P.lanczos_restarted_sigma_min(
        dev(w.U), dev(w.shifts), dev(w.B), kdim=kdim, keep=keep, max_restarts=200, tol=1e-11))
    so, ro, sto, co = oracle_mod.lanczos_restarted_sigma_min(w.U, w.shifts, w.B, kdim=kdim, keep=keep,
                                                             max_restarts=200, tol=1e-11)
    assert np.all(c == 1) and co.all() and np.all(r <= 1e-11)
    np.testing.assert_array_equal(st, sto)
    if kdim == 8:
        assert st.max() > kdim
    np.testing.assert_allclose(s, so, rtol=1e-10)
    Ut = np.triu(w.U)
    sv = np.array([sla.svdvals(Ut - z * np.eye(150))[-1] for z in w.shifts])
    np.testing.assert_allclose(s, sv, rtol=1e-10)


def test_restarted_one_cycle_equals_plain(P):
    """One cycle of 15 steps and no restart is the plain 15-step Lanczos (full
    reorthogonalisation changes rounding only)."""
    w = W.c4_pseudospectra(m=300, grid=5)
    announce("restarted lanczos, one cycle of 15 = plain 15 steps")
    s, r, st, c = (_host(t) for t in P.lanczos_restarted_sigma_min(
        dev(w.U), dev(w.shifts), dev(w.B), kdim=15, keep=5, max_restarts=0, tol=0.0))
    s15, _, _, _ = P.lanczos_sigma_min(dev(w.U), dev(w.shifts), dev(w.B), iters=15)
    assert np.all(st == 15)
    np.testing.assert_allclose(s, _host(s15), rtol=1e-12)
    # the workspace of a call starts from nothing the previous call left
    s2 = _host(P.lanczos_restarted_sigma_min(dev(w.U), dev(w.shifts), dev(w.B), kdim=15, keep=5,
                                             max_restarts=0, tol=0.0)[0])
    assert np.array_equal(s2, s)


def test_restarted_diagonal_closed_form(P):
    g = W.rng(3)
    d = W.cnormal(g, 60)
    z = np.linspace(-1.0, 1.0, 7) + 0.3j
    V0 = W.cnormal(W.rng(4), (60, 7))
    s, r, st, c = (_host(t) for t in P.lanczos_restarted_sigma_min(
        dev(np.diag(d)), dev(z), dev(V0), kdim=10, keep=3, max_restarts=100, tol=1e-12))
    exact = np.array([np.min(np.abs(d - zz)) for zz in z])
    assert np.all(c == 1)
    np.testing.assert_allclose(s, exact, rtol=1e-12)


def test_restarted_c4_config_sampled(P, oracle_mod):
    """The pseudospectra workload (2000 x 2000, 100 x 100 grid) to tol 1e-10:
    every shift converges, and every 100th agrees with the oracle (sigma to
    1e-9, the same number of Lanczos steps)."""
    import torch
    w = W.c4_pseudospectra()
    announce("restarted lanczos c4 2000 x 10000 shifts")
    V0 = dev(w.B)
    s, r, st, c = (_host(t) for t in P.lanczos_restarted_sigma_min(dev(w.U), dev(w.shifts), V0, tol=1e-10))
    assert np.array_equal(_host(V0), np.asarray(w.B))   # start vectors not modified
    assert np.all(c == 1) and np.all(r <= 1e-10) and np.all(np.isfinite(s)) and np.all(s > 0)
    print("steps: min %d mean %.1f max %d" % (st.min(), st.mean(), st.max()))
    cols = np.arange(0, w.n, 100)
    so, ro, sto, co = oracle_mod.lanczos_restarted_sigma_min(w.U, w.shifts[cols], w.B[:, cols], tol=1e-10)
    np.testing.assert_allclose(s[cols], so, rtol=1e-9)
    np.testing.assert_array_equal(st[cols], sto)


def test_cloud_with_tolerance_uses_the_restarted_method(P):
    from paper_1607_01477_amd import pseudospectra as PS
    w = W.c4_pseudospectra(m=120, grid=3)
    V0 = dev(w.B)
    s = PS.spectral_cloud(dev(w.U), w.shifts, V0=V0, tol=1e-11).cpu().numpy()
    s2 = _host(P.lanczos_restarted_sigma_min(dev(w.U), dev(w.shifts), V0, tol=1e-11)[0])
    assert np.array_equal(s, s2)
