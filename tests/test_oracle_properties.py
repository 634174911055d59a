"""Property-based pins of the oracle on random small problems (m <= 16):
every solve against a dense brute-force solve of the same system
(numpy.linalg.solve on the full matrix), and the safe solve's defining
relation (U - l_j I) X_j = 2^-k_j B_j with k_j >= 0 and finite X, also under a
small overflow threshold that forces rescaling. Hypothesis draws the shapes,
seeds and threshold; the run is derandomized so that it is reproducible."""
import numpy as np
from hypothesis import given, settings, strategies as st

import workloads as W

SETTINGS = settings(max_examples=40, deadline=None, derandomize=True)


def _problem(seed, m, n, real=False):
    g = W.rng(seed)
    if real:
        U = np.triu(g.standard_normal((m, m)) / np.sqrt(m), 1)
        U[np.arange(m), np.arange(m)] = np.where(g.random(m) < 0.5, -1.0, 1.0) * (0.5 + 1.5 * g.random(m))
        lam = -0.4 + 0.8 * g.random(n)
        B = g.standard_normal((m, n))
    else:
        U = W.random_upper(g, m, 1.0 / np.sqrt(m), W.annulus_uniform(g, m, 0.5, 2.0))
        lam = W.disk_uniform(g, n, 0.4)
        B = W.cnormal(g, (m, n))
    return np.asfortranarray(U), lam, np.asfortranarray(B)


def _dense(E, b):
    return np.linalg.solve(E, b)


def _close(x, y):
    return np.abs(x - y).max() <= 1e-11 * max(1.0, np.abs(y).max())


shapes = dict(seed=st.integers(0, 2 ** 31 - 1), m=st.integers(1, 16), n=st.integers(1, 6))


@SETTINGS
@given(**shapes)
def test_plain_and_adjoint_against_dense(oracle_mod, seed, m, n):
    U, lam, B = _problem(seed, m, n)
    X = oracle_mod.solve(U, lam, B)
    Y = oracle_mod.solve_adjoint(U, lam, B)
    for j in range(n):
        E = U - lam[j] * np.eye(m)
        assert _close(X[:, j], _dense(E, B[:, j]))
        assert _close(Y[:, j], _dense(E.conj().T, B[:, j]))


@SETTINGS
@given(**shapes)
def test_real_against_dense(oracle_mod, seed, m, n):
    U, lam, B = _problem(seed, m, n, real=True)
    X = oracle_mod.solve_real(U, lam, B)
    for j in range(n):
        assert _close(X[:, j], _dense(U - lam[j] * np.eye(m), B[:, j]))


@SETTINGS
@given(uplo=st.sampled_from("UL"), op=st.sampled_from("NTC"), **shapes)
def test_variants_against_dense(oracle_mod, seed, m, n, uplo, op):
    U, lam, B = _problem(seed, m, n)
    A = U if uplo == "U" else np.asfortranarray(U.T.copy())
    X = oracle_mod.solve_op(A, lam, B, uplo, op)
    for j in range(n):
        E = A - lam[j] * np.eye(m)
        E = {"N": E, "T": E.T, "C": E.conj().T}[op]
        assert _close(X[:, j], _dense(E, B[:, j]))


@SETTINGS
@given(**shapes)
def test_pencil_against_dense(oracle_mod, seed, m, n):
    U, lam, B = _problem(seed, m, n)
    g = W.rng(seed + 1)
    V = np.triu(W.cnormal(g, (m, m), 1.0 / np.sqrt(m)), 1)
    V[np.arange(m), np.arange(m)] = 0.5 + g.random(m)
    V = np.asfortranarray(V)
    X = oracle_mod.solve_gen(U, V, lam, B)
    for j in range(n):
        assert _close(X[:, j], _dense(U - lam[j] * V, B[:, j]))


@SETTINGS
@given(omega_log2=st.sampled_from([8, 12, 20, 960]), nb=st.sampled_from([0, 1, 4, 16, 64]), **shapes)
def test_safe_relation(oracle_mod, seed, m, n, omega_log2, nb):
    # growth problem: small pivots make the solution grow, so small thresholds rescale
    g = W.rng(seed)
    U = W.random_upper(g, m, 1.0, 0.05 + 0.1 * g.random(m))
    lam = np.zeros(n, dtype=np.complex128)
    B = np.asfortranarray(W.cnormal(g, (m, n)))
    X, s, k = oracle_mod.solve_safe(np.asfortranarray(U), lam, B, nb=nb, omega_log2=omega_log2)
    assert np.all(np.isfinite(X))
    assert np.all(k >= 0)
    assert np.array_equal(s, np.ldexp(1.0, -k))
    for j in range(n):
        ref = _dense(U, B[:, j]) * s[j]
        assert np.abs(X[:, j] - ref).max() <= 1e-9 * max(np.abs(ref).max(), 2.0 ** -1000)
