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
