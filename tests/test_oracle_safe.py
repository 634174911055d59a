"""Pins for the oracle's safe multi-shift solve (Alg 4 and Alg 5, Sec. 3).

Problem (6): (U - lambda_j I) x_j = s_j b_j with s_j in [0, 1]; here
s_j = 2^-k_j. The pins are: hand-traced examples (tests/golden), exact
dyadic problems whose true solution is known in rational arithmetic, the
identity with the plain solve when nothing rescales, invariance under the
phase-1 fast path, equality of Alg 4 and Alg 5 with nb = 1 where the two
growth quantities coincide, the growth-bound invariant, and the
triangular-eigenvector short-cut.
"""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "safe_scaling_examples.json")


def _p2(s):
    # "2^959" / "2^959 (1 + i)" / number
    if isinstance(s, (int, float)):
        return complex(s)
    s = s.strip()
    if s.startswith("2^"):
        head, _, tail = s.partition(" ")
        v = 2.0 ** int(head[2:])
        if tail:
            assert tail == "(1 + i)"
            return complex(v, v)
        return complex(v)
    raise ValueError(s)


def _golden_inputs(case):
    m = case["m"]
    if case["name"] == "growth_chain_m12":
        U = np.zeros((m, m), dtype=np.complex128)
        U[np.arange(m), np.arange(m)] = 2.0 ** -100
        U[np.arange(m - 1), np.arange(1, m)] = -1.0
        b = np.zeros((m, 1), dtype=np.complex128)
        b[-1, 0] = 1.0
    else:
        U = np.array(case["U"], dtype=np.complex128)
        b = np.array([[_p2(v)] for v in case["b"]], dtype=np.complex128)
    lam = np.array([complex(*case["shift"])])
    return np.asfortranarray(U), lam, np.asfortranarray(b)


def _golden_cases():
    with open(GOLDEN) as f:
        return json.load(f)["cases"]


@pytest.mark.parametrize("case", _golden_cases(), ids=lambda c: c["name"])
@pytest.mark.parametrize("force_phase2", [False, True])
def test_golden_examples(oracle_mod, case, force_phase2):
    U, lam, b = _golden_inputs(case)
    for nb in case["block_sizes"]:
        X, s, k = oracle_mod.solve_safe(U, lam, b, nb=nb, force_phase2=force_phase2)
        assert int(k[0]) == case["k"], (nb, k)
        assert s[0] == 2.0 ** -case["k"]
        if "log2_abs_x" in case:
            for i, (e, sg) in enumerate(zip(case["log2_abs_x"], case["x_sign"])):
                assert X[i, 0] == complex(sg * 2.0 ** e), (nb, i, X[i, 0])
        else:
            for i, (er, ei) in enumerate(case["x_re_im_log2"]):
                assert X[i, 0] == complex(2.0 ** er, 2.0 ** ei)


def _dyadic_problem(seed, m, n, complex_diag=True):
    """Upper-triangular U with diagonal +-2^-2 or +-i 2^-2 and off-diagonal
    entries in {0, +-1, +-i}; integer right-hand sides. Back substitution
    on these is exact in binary64 (every quotient is a power-of-two multiple)
    and the solution grows like 5^m, so small Omega forces rescaling."""
    g = W.rng(seed)
    U = np.zeros((m, m), dtype=np.complex128)
    units = np.array([1, -1, 1j, -1j, 0], dtype=np.complex128)
    for c in range(m):
        for r in range(c):
            U[r, c] = units[g.integers(0, 5)]
        U[c, c] = units[g.integers(0, 4 if complex_diag else 2)] * 0.25
    lam = np.zeros(n, dtype=np.complex128)
    B = (g.integers(-3, 4, (m, n)) + 1j * g.integers(-3, 4, (m, n))).astype(np.complex128)
    return np.asfortranarray(U), lam, np.asfortranarray(B)


def _exact_solve(U, b):
    """Rational back substitution (Gaussian rationals as Fraction pairs)."""
    m = U.shape[0]
    F = lambda v: (Fraction(v.real), Fraction(v.imag))
    x = [None] * m
    bb = [F(v) for v in b]
    for i in range(m - 1, -1, -1):
        br, bi = bb[i]
        for k in range(i + 1, m):
            ur, ui = F(U[i, k])
            xr, xi = x[k]
            br -= ur * xr - ui * xi
            bi -= ur * xi + ui * xr
        dr, di = F(U[i, i])
        den = dr * dr + di * di
        x[i] = ((br * dr + bi * di) / den, (bi * dr - br * di) / den)
    return x


@pytest.mark.parametrize("nb", [0, 1, 2, 3, 4, 16])
@pytest.mark.parametrize("omega_log2", [6, 9, 14, 960])
def test_dyadic_exact_scaling(oracle_mod, nb, omega_log2):
    m, n = 12, 5
    U, lam, B = _dyadic_problem(7 + omega_log2, m, n)
    X, s, k = oracle_mod.solve_safe(U, lam, B, nb=nb, omega_log2=omega_log2)
    events = 0
    for j in range(n):
        xt = _exact_solve(U, B[:, j])
        kj = int(k[j])
        events += kj > 0
        for i in range(m):
            exr = float(xt[i][0] * Fraction(2) ** (-kj))
            exi = float(xt[i][1] * Fraction(2) ** (-kj))
            assert X[i, j] == complex(exr, exi), (j, i, kj)
        # scaled solution stays below the overflow threshold (2x slack for cabs1)
        assert np.max(np.abs(X[:, j].real) + np.abs(X[:, j].imag)) < 2.0 ** (omega_log2 + 1)
    if omega_log2 <= 9:
        assert events > 0


def test_no_scaling_identity(oracle_mod):
    w = W.c1_plain(seed=21, m=200, n=40)
    Xp = oracle_mod.solve(w.U, w.shifts, w.B)
    for nb in (0, 1, 16, 64, 200):
        Xs, s, k = oracle_mod.solve_safe(w.U, w.shifts, w.B, nb=nb)
        assert np.all(k == 0)
        assert np.array_equal(Xs, Xp), nb


def _growth_problem(seed, m, n):
    # C2-like growth: unscaled CN(0,1) off-diagonal, CN(0,1) diagonal
    g = W.rng(seed)
    d = W.cnormal(g, m)
    U = W.random_upper(g, m, 1.0, d)
    lam = W.cnormal(g, n)
    B = np.asfortranarray(W.cnormal(g, (m, n)))
    return U, lam, B


@pytest.mark.parametrize("nb", [0, 16, 64])
def test_force_phase2_invariance(oracle_mod, nb):
    U, lam, B = _growth_problem(22, 300, 24)
    for omega_log2 in (960, 40):
        a = oracle_mod.solve_safe(U, lam, B, nb=nb, omega_log2=omega_log2)
        b = oracle_mod.solve_safe(U, lam, B, nb=nb, omega_log2=omega_log2, force_phase2=True)
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[2], b[2])
        if omega_log2 == 40:
            assert np.any(a[2] > 0)


def test_alg4_equals_alg5_nb1_with_power_of_two_pivots(oracle_mod):
    # With real power-of-two pivots cabs1(b/d) = cabs1(b)/cabs1(d) exactly, so
    # the growth quantities of Alg 4 (M) and Alg 5 with nb = 1 (||x_i||) agree.
    g = W.rng(23)
    m, n = 60, 10
    U = W.random_upper(g, m, 1.0, np.zeros(m))
    U[np.arange(m), np.arange(m)] = np.where(g.random(m) < 0.5, 1.0, -1.0) * 2.0 ** g.integers(-3, 1, m)
    lam = np.zeros(n, dtype=np.complex128)
    B = np.asfortranarray(W.cnormal(g, (m, n)))
    for omega_log2 in (960, 30, 60):
        a = oracle_mod.solve_safe(U, lam, B, nb=0, omega_log2=omega_log2)
        b = oracle_mod.solve_safe(U, lam, B, nb=1, omega_log2=omega_log2)
        assert np.array_equal(a[2], b[2])
        assert np.array_equal(a[0], b[0])


@pytest.mark.parametrize("nb", [8, 32])
def test_growth_bound_invariant(oracle_mod, nb):
    # After each block: G(j) >= max cabs1 of the rows above the block
    U, lam, B = _growth_problem(24, 256, 16)
    X, s, k, tr = oracle_mod.solve_safe(U, lam, B, nb=nb, trace=True)
    G = tr[:, :, 0]
    mx = tr[:, :, 1]
    ok = ~np.isnan(G)
    assert np.all(G[ok] * (1 + 1e-12) >= mx[ok])
    assert np.all(G[ok] < 2.0 ** 960)


@pytest.mark.parametrize("nb", [0, 16, 64])
def test_safe_residual_growth_problem(oracle_mod, nb):
    U, lam, B = _growth_problem(25, 400, 20)
    X, s, k = oracle_mod.solve_safe(U, lam, B, nb=nb)
    assert np.all(np.isfinite(X))
    assert np.all((s >= 0) & (s <= 1))
    rr = oracle_mod.relative_residual(U, lam, X, B, k=k)
    assert rr.max() <= 1e-13


def test_col_len_shortcut_equals_zero_padded_column(oracle_mod):
    U, lam, B = _growth_problem(26, 150, 30)
    g = W.rng(260)
    L = g.integers(0, 151, 30).astype(np.int32)
    L[:3] = [0, 150, 64]
    Bz = B.copy(order="F")
    for j in range(30):
        Bz[L[j]:, j] = 0
    for nb in (0, 16, 64):
        Xa, sa, ka = oracle_mod.solve_safe(U, lam, B, col_len=L, nb=nb)
        Xb, sb, kb = oracle_mod.solve_safe(U, lam, Bz, col_len=None, nb=nb)
        assert np.array_equal(ka, kb)
        for j in range(30):
            assert np.array_equal(Xa[:L[j], j], Xb[:L[j], j])
            assert np.all(Xb[L[j]:, j] == 0)
            # rows at and below col_len are not touched
            assert np.array_equal(Xa[L[j]:, j], B[L[j]:, j])


def test_scale_exponents_are_not_excessive(oracle_mod):
    # the scaled solution keeps its largest entry within a few binades of
    # Omega whenever a rescaling happened (rescaling is never gratuitous)
    U, lam, B = _growth_problem(27, 500, 24)
    for nb in (0, 64):
        X, s, k = oracle_mod.solve_safe(U, lam, B, nb=nb)
        for j in np.nonzero(k > 0)[0]:
            top = np.max(np.abs(X[:, j].real) + np.abs(X[:, j].imag))
            assert top > 2.0 ** (960 - 64), (j, math.log2(top))
