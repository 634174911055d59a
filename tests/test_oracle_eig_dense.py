"""Pins for the oracle's general eigensolvers after the Schur step.

Eig (Alg 6): A = Q T Q^H (host Schur), Z = TriangEig(T), X = Q Z; and
GeneralizedEig (appendix, Alg 10): A = Q T P^H, B = Q S P^H (host QZ),
Z = GeneralizedTriangEig(T, S), X = P Z. Columns of X have unit 2-norm.
Pinned against the eigen-relation the paper validates with
(||A X - X Lambda||_F / ||A||_F < 1e-13), the library eigensolvers, and
matrices built with known eigenvectors.
"""
import numpy as np
import pytest
import scipy.linalg as sla

import workloads as W

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def _match(lam, ref):
    """index into ref of the nearest value for each lam (one-to-one here)."""
    idx = np.argmin(np.abs(lam[:, None] - ref[None, :]), axis=1)
    assert len(set(idx.tolist())) == len(idx)
    return idx


def test_eig_relation_and_library_eigenvalues(oracle_mod):
    A = W.c8_dense_eig(seed=80, m=120).extra["A"]
    T, Q = sla.schur(A, output="complex")
    lam, X = oracle_mod.eig_schur(T, Q)
    res = np.linalg.norm(A @ X - X * lam[None, :]) / np.linalg.norm(A)
    assert res < 1e-13, res
    assert np.allclose(np.linalg.norm(X, axis=0), 1.0, rtol=1e-14, atol=0)
    ev = np.linalg.eigvals(A)
    idx = _match(lam, ev)
    assert np.max(np.abs(lam - ev[idx])) <= 1e-12
    # the paper's second diagnostic: a nonsingular eigenvector matrix
    assert np.linalg.cond(X) < 1e6


def test_eig_known_eigenvectors(oracle_mod):
    # A = V diag(d) V^-1 with well-separated d: X's columns are V's up to phase
    g = W.rng(81)
    m = 40
    V = np.eye(m) + 0.3 * W.cnormal(g, (m, m)) / np.sqrt(m)
    d = np.exp(2j * np.pi * np.arange(m) / m) * (1.0 + np.arange(m) / m)
    A = V @ np.diag(d) @ np.linalg.inv(V)
    T, Q = sla.schur(A, output="complex")
    lam, X = oracle_mod.eig_schur(T, Q)
    idx = _match(lam, d)
    Vn = V / np.linalg.norm(V, axis=0)[None, :]
    for j in range(m):
        c = abs(np.vdot(Vn[:, idx[j]], X[:, j]))
        assert abs(c - 1.0) < 1e-10, (j, c)


def test_gen_eig_relation_and_library_eigenvalues(oracle_mod):
    w = W.c9_dense_pencil(seed=90, m=100)
    A, B = w.extra["A"], w.extra["B"]
    T, S, Qq, P = sla.qz(A, B, output="complex")
    lam, X = oracle_mod.gen_eig_schur(T, S, P)
    R = A @ X - (B @ X) * lam[None, :]
    res = np.max(np.linalg.norm(R, axis=0) / (np.linalg.norm(A, 2) + np.abs(lam) * np.linalg.norm(B, 2)))
    assert res < 1e-13, res
    ev = sla.eigvals(A, B)
    idx = _match(lam, ev)
    assert np.max(np.abs(lam - ev[idx]) / np.maximum(1.0, np.abs(ev[idx]))) <= 1e-9


def test_gen_eig_known_eigenvectors(oracle_mod):
    # A = W diag(alpha) V^-1, B = W diag(beta) V^-1: eigenvectors V, eigenvalues alpha/beta
    g = W.rng(91)
    m = 30
    V = np.eye(m) + 0.3 * W.cnormal(g, (m, m)) / np.sqrt(m)
    Wm = np.eye(m) + 0.3 * W.cnormal(g, (m, m)) / np.sqrt(m)
    beta = 0.5 + g.random(m)
    alpha = np.exp(2j * np.pi * np.arange(m) / m) * (1.0 + np.arange(m) / m) * beta
    Vi = np.linalg.inv(V)
    A = Wm @ np.diag(alpha) @ Vi
    B = Wm @ np.diag(beta) @ Vi
    T, S, Qq, P = sla.qz(A, B, output="complex")
    lam, X = oracle_mod.gen_eig_schur(T, S, P)
    idx = _match(lam, alpha / beta)
    Vn = V / np.linalg.norm(V, axis=0)[None, :]
    for j in range(m):
        c = abs(np.vdot(Vn[:, idx[j]], X[:, j]))
        assert abs(c - 1.0) < 1e-9, (j, c)
