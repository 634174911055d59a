"""GPU parity of the general eigensolvers after the Schur step (Alg 6 Eig,
appendix Alg 10 GeneralizedEig): TriangEig / GeneralizedTriangEig, the
back-transformation X = Q Z (resp. P Z) on the matrix cores and unit columns,
against the oracle on the same Schur factors (computed on the host with
SciPy's LAPACK). Bars: ||A X - X Lambda||_F / ||A||_F < 1e-13 (the paper's
validation), eigenvalues equal to diag(T) (resp. within 4 ulps of
T(j,j)/S(j,j)), columns equal to the oracle's to 1e-9 (unit columns, same
phase convention: Z(j,j) > 0).
"""
import numpy as np
import pytest
import scipy.linalg as sla

import workloads as W
from gpu_util import announce, dev, host

pytestmark = pytest.mark.gpu

EPS = 2.0 ** -52


@pytest.fixture(scope="module")
def P():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1607_01477_amd as P
    P._lib.load()
    return P


@pytest.mark.parametrize("m", [1, 2, 7, 33, 64, 65, 130, 300])
def test_eig_schur_shapes(P, oracle_mod, m):
    announce("eig_schur m=%d" % m)
    A = W.c8_dense_eig(seed=800 + m, m=m).extra["A"]
    T, Q = sla.schur(A, output="complex")
    ev, X, k = P.eig_schur(dev(T), dev(Q))
    ev, X = host(ev), host(X)
    assert np.array_equal(ev, np.diag(T))
    lo, Xo = oracle_mod.eig_schur(T, Q, nb=16)
    assert np.max(np.abs(X - Xo)) <= 1e-9, np.max(np.abs(X - Xo))
    res = np.linalg.norm(A @ X - X * ev[None, :]) / np.linalg.norm(A)
    assert res < 1e-13, res
    assert np.allclose(np.linalg.norm(X, axis=0), 1.0, rtol=1e-13, atol=0)


def test_eig_c8_m1024(P, oracle_mod):
    A = W.c8_dense_eig(m=1024).extra["A"]
    announce("eig m=1024")
    T, Q = sla.schur(A, output="complex")
    ev, X, k = P.eig_schur(dev(T), dev(Q))
    ev, X = host(ev), host(X)
    res = np.linalg.norm(A @ X - X * ev[None, :]) / np.linalg.norm(A)
    assert res < 1e-13, res
    lo, Xo = oracle_mod.eig_schur(T, Q, nb=16)
    assert np.max(np.abs(X - Xo)) <= 1e-9


def test_eig_end_to_end(P):
    # host Schur inside the driver; eigenvalues against the library's
    A = W.c8_dense_eig(seed=82, m=200).extra["A"]
    ev, X = P.eig(dev(A))
    ev, X = host(ev), host(X)
    ref = np.linalg.eigvals(A)
    idx = np.argmin(np.abs(ev[:, None] - ref[None, :]), axis=1)
    assert len(set(idx.tolist())) == 200
    assert np.max(np.abs(ev - ref[idx])) <= 1e-12
    assert np.linalg.norm(A @ X - X * ev[None, :]) / np.linalg.norm(A) < 1e-13


@pytest.mark.parametrize("m", [1, 5, 64, 200, 300])
def test_gen_eig_schur_shapes(P, oracle_mod, m):
    announce("gen_eig_schur m=%d" % m)
    w = W.c9_dense_pencil(seed=900 + m, m=m)
    A, B = w.extra["A"], w.extra["B"]
    T, S, _, Pz = sla.qz(A, B, output="complex")
    ev, X, k = P.gen_eig_schur(dev(T), dev(S), dev(Pz))
    ev, X = host(ev), host(X)
    lo, Xo = oracle_mod.gen_eig_schur(T, S, Pz, nb=16)
    np.testing.assert_allclose(ev, lo, rtol=4 * EPS, atol=0)
    R = A @ X - (B @ X) * ev[None, :]
    rel = np.linalg.norm(R, axis=0) / (np.linalg.norm(A, 2) + np.abs(ev) * np.linalg.norm(B, 2))
    assert rel.max() < 1e-13, rel.max()
    # eigenvectors with a tiny |S(j,j)| are ill-conditioned; compare the others
    ok = np.abs(np.diag(S)) > 1e-3 * np.abs(np.diag(S)).max()
    assert np.max(np.abs(X - Xo)[:, ok]) <= 1e-8


def test_gen_eig_end_to_end(P):
    w = W.c9_dense_pencil(seed=92, m=150)
    A, B = w.extra["A"], w.extra["B"]
    ev, X = P.gen_eig(dev(A), dev(B))
    ev, X = host(ev), host(X)
    R = A @ X - (B @ X) * ev[None, :]
    rel = np.linalg.norm(R, axis=0) / (np.linalg.norm(A, 2) + np.abs(ev) * np.linalg.norm(B, 2))
    assert rel.max() < 1e-13
