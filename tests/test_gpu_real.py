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
