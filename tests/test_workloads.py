"""Seeded generators: determinism, shapes and the stated distributions."""
import numpy as np

import workloads as W


def test_deterministic():
    a = W.c1_plain()
    b = W.c1_plain()
    assert np.array_equal(a.U, b.U) and np.array_equal(a.B, b.B)
    assert np.array_equal(a.shifts, b.shifts)
    c = W.c1_plain(seed=99)
    assert not np.array_equal(a.U, c.U)


def test_c1_shapes_and_distribution():
    w = W.c1_plain()
    assert w.U.shape == (256, 256) and w.B.shape == (256, 256) and w.n == 256
    assert w.U.flags.f_contiguous and w.B.flags.f_contiguous
    assert np.all(np.tril(w.U, -1) == 0)
    assert np.all(np.abs(np.diag(w.U)) <= 1.0)
    assert np.all(np.abs(w.shifts) <= 1.5)
    # CN(0,1): E|z|^2 = 1, re and im each variance 1/2
    assert abs(np.mean(np.abs(w.B) ** 2) - 1.0) < 0.02
    assert abs(np.var(w.B.real) - 0.5) < 0.02
    off = w.U[np.triu_indices(256, 1)]
    assert abs(np.mean(np.abs(off) ** 2) * 256 - 1.0) < 0.03


def test_c2_duplicates_and_columns():
    w = W.c2_triang_eig(m=2048)
    d = np.diag(w.U)
    assert len(w.extra["dup_targets"]) == 102
    # every target equals some non-target value exactly
    t = set(w.extra["dup_targets"].tolist())
    nont = {complex(v) for i, v in enumerate(d) if i not in t}
    assert all(complex(d[i]) in nont for i in t)
    assert np.array_equal(w.shifts, d)
    assert np.array_equal(w.col_len, np.arange(2048))
    assert np.all(w.B[np.tril_indices(2048)] == 0)
    assert np.array_equal(w.B[:5, 5], -w.U[:5, 5])
    assert abs(W.nominal_flops(2048, 2048, w.col_len) / 1e9 - 11.44) < 0.01


def test_c3_c5_annulus_and_disk():
    w = W.c3_mixed(m=512, n=256)
    a = np.abs(np.diag(w.U))
    assert a.min() >= 0.5 and a.max() <= 2.0
    assert np.all(np.abs(w.shifts) <= 0.4)
    w5 = W.c5_adjoint(m=256, n=128)
    assert w5.extra["W"].shape == (256, 128) and w5.extra["W"].dtype == np.float64


def test_c4_grid():
    w = W.c4_pseudospectra(m=50, grid=100)
    z = w.shifts
    assert z.shape == (10000,)
    assert np.isclose(z.real.min(), -1.5) and np.isclose(z.real.max(), 1.5)
    assert np.isclose(z.imag.min(), -1.5) and np.isclose(z.imag.max(), 1.5)
    assert len(np.unique(np.round(z.real, 12))) == 100
    np.testing.assert_allclose(np.linalg.norm(w.B, axis=0), 1.0, rtol=1e-14)
    assert abs(W.nominal_flops(2000, 10000) * 30 / 1e12 - 4.8) < 0.01


def test_c6_c7_generalized_pencils():
    w = W.c6_generalized(m=256, n=64)
    V = w.extra["V"]
    assert V.shape == (256, 256) and V.flags.f_contiguous
    assert np.all(np.tril(V, -1) == 0) and np.all(np.tril(w.U, -1) == 0)
    dv = np.diag(V)
    assert np.all(dv.imag == 0) and dv.real.min() >= 0.5 and dv.real.max() <= 1.5
    assert np.all(np.abs(w.shifts) <= 0.2)
    # pivots of U - lambda V stay away from zero: |u| >= 0.5, |lambda v| <= 0.3
    piv = np.diag(w.U)[:, None] - w.shifts[None, :] * dv[:, None]
    assert np.abs(piv).min() >= 0.2
    w7 = W.c7_gen_triang_eig(m=128)
    S = w7.extra["S"]
    assert np.all(np.tril(S, -1) == 0) and np.all(np.diag(S).real >= 0.5)
    assert np.array_equal(w7.col_len, np.arange(128)) and w7.B is None


def test_c8_c9_dense_unit_disk():
    A = W.c8_dense_eig(m=200).extra["A"]
    assert A.shape == (200, 200) and A.flags.f_contiguous
    assert np.abs(A).max() <= 1.0
    # area-uniform in the unit disk: E|z|^2 = 1/2
    assert abs(np.mean(np.abs(A) ** 2) - 0.5) < 0.01
    w = W.c9_dense_pencil(m=64)
    assert w.extra["A"].shape == w.extra["B"].shape == (64, 64)
    assert not np.array_equal(w.extra["A"], w.extra["B"])


def test_c10_real():
    w = W.c10_real(m=300, n=50)
    assert w.U.dtype == np.float64 and w.B.dtype == np.float64 and w.shifts.dtype == np.float64
    assert np.all(np.tril(w.U, -1) == 0)
    d = np.abs(np.diag(w.U))
    assert d.min() >= 0.5 and d.max() <= 2.0 and np.abs(w.shifts).max() <= 0.4
