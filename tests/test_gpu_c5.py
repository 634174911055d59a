"""GPU parity of the gradient through the multi-shift solve at the size of the
loss-gradient workload (m = 4096, n = 2048 shifts; loss sum(W |X|^2)).

The gradient is not in the paper; the adjoint solve it rests on is the
conjugate-transposed (lower-triangular) variant of the footnote to Sec. 2.
Convention (torch's): grad z = dL/dRe z + i dL/dIm z, so with
Y = adjoint solve of 2 W X:  gB = Y, gU = -triu(Y X^H), gshift_j = x_j^H y_j.

Bars:
  * every gradient entry is a sum of products; GPU and oracle differ by the
    rounding of that sum plus the propagated difference of X and Y (both
    backward stable). Entry-wise: |g_gpu - g_or| <= 1e-11 * sum |terms|
    (the magnitude sum of the dot product, which bounds any such difference
    relative to the quantity's own conditioning);
  * central finite differences (h = 1e-6) of the loss, formed from the
    difference X+ - X- so that the loss's own rounding does not enter:
    |fd - analytic| <= 1e-6 |analytic| + 1e-9 ||grad||_inf.
"""
import numpy as np
import pytest

import workloads as W
from gpu_util import announce, colerr, dev, host

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


@pytest.fixture(scope="module")
def c5(oracle_mod):
    """The workload and its oracle solution X, adjoint Y and full gradient."""
    w = W.c5_adjoint()
    announce("c5 oracle: X, Y (4096 x 2048) and -triu(Y X^H)")
    Xo = oracle_mod.solve(w.U, w.shifts, w.B)
    Yo = oracle_mod.solve_adjoint(w.U, w.shifts, 2.0 * w.extra["W"] * Xo)
    gU, gl, gB = oracle_mod.gradient(w.U, w.shifts, Xo, Yo)
    return w, Xo, Yo, gU, gl, gB


# ------------------------------------------------------------------ -triu(Y X^H)

@pytest.mark.parametrize("m,n", [(960, 64), (1024, 200), (1000, 3), (1088, 33)])
def test_grad_u_xcd_tile_order(P, oracle_mod, m, n):
    """Square grids whose count of on/above-diagonal 64 x 64 tiles is a
    multiple of 8 (m = 960: 120 tiles; m = 1024 and the ragged m = 1000: 136),
    so that those tiles are dealt to the eight XCDs in contiguous ranges, and
    m = 1088 (153 tiles, dealt in launch order) beside them. Every entry
    against the oracle within the dot-product error bound."""
    announce("grad_u m=%d n=%d" % (m, n))
    g = W.rng(7000 + m + n)
    Y = W.cnormal(g, (m, n))
    X = W.cnormal(g, (m, n))
    gU, _, _ = oracle_mod.gradient(np.zeros((m, m), complex), np.zeros(n, complex), X, Y)
    gUd = host(P.grad_u(dev(Y), dev(X)))
    bound = np.triu(np.abs(Y) @ np.abs(X).T)
    assert np.all(np.tril(gUd, -1) == 0)
    assert np.all(np.abs(gUd - gU) <= 4.0 * n * EPS * bound + 1e-300)


def test_grad_u_c5_full(P, c5):
    """The U gradient of the loss-gradient workload: every upper entry of
    -triu(Y X^H) at 4096 x 4096 (K = 2048) against the oracle's."""
    w, Xo, Yo, gU, gl, gB = c5
    announce("grad_u c5 4096 x 4096, K = 2048")
    gUd = host(P.grad_u(dev(Yo), dev(Xo)))
    assert np.all(np.tril(gUd, -1) == 0)
    bound = np.triu(np.abs(Yo) @ np.abs(Xo).T)
    n = w.n
    err = np.abs(gUd - gU)
    assert np.all(err <= 4.0 * n * EPS * bound), (err / np.maximum(bound, 1e-300)).max()


# ------------------------------------------------------------------ autograd at full size

def _autograd(P, w, precision, max_sweeps):
    import torch
    U = dev(w.U).requires_grad_(True)
    s = dev(w.shifts).requires_grad_(True)
    B = dev(w.B).requires_grad_(True)
    Wt = torch.from_numpy(w.extra["W"]).cuda()
    X = P.solve(U, s, B, precision=precision, max_sweeps=max_sweeps)
    (Wt * X.abs() ** 2).sum().backward()
    return host(X), host(U.grad), host(s.grad), host(B.grad)


@pytest.mark.parametrize("precision,sweeps", [(0, 0), (1, 2)])
def test_autograd_c5_against_oracle(P, c5, precision, sweeps):
    """Forward (FP64, or FP32 substitution GEMMs + 2 FP64 refinement sweeps)
    and FP64 backward at 4096 x 2048: gshift on every column, gB on 16
    sampled columns, gU on 4096 sampled upper entries (corners included)."""
    w, Xo, Yo, gU, gl, gB = c5
    announce("c5 autograd precision=%d sweeps=%d" % (precision, sweeps))
    X, gUd, gld, gBd = _autograd(P, w, precision, sweeps or 2)
    m, n = w.m, w.n
    cols = np.unique(np.concatenate([np.sort(W.rng(501).choice(n, 14, replace=False)), [0, n - 1]]))
    assert colerr(X[:, cols], Xo[:, cols]).max() <= 1e-12
    # gB = Y: per column against the oracle's adjoint solve
    assert colerr(gBd[:, cols], gB[:, cols]).max() <= 1e-11
    # gshift_j = x_j^H y_j, every column
    lbound = np.sum(np.abs(Xo) * np.abs(Yo), axis=0)
    assert np.all(np.abs(gld - gl) <= 1e-11 * lbound)
    # gU on sampled upper entries, strict lower triangle zero
    g = W.rng(502)
    r = g.integers(0, m, 4096)
    c = g.integers(0, m, 4096)
    r, c = np.minimum(r, c), np.maximum(r, c)
    r = np.concatenate([r, [0, 0, m - 1, m - 64, 63]])
    c = np.concatenate([c, [0, m - 1, m - 1, m - 1, 64]])
    ubound = np.sum(np.abs(Yo[r]) * np.abs(Xo[c]), axis=1)
    assert np.all(np.abs(gUd[r, c] - gU[r, c]) <= 1e-11 * ubound)
    lr = np.tril_indices(m, -1)
    assert np.all(gUd[lr[0][::997], lr[1][::997]] == 0)


def test_finite_differences_c5(P, c5):
    """Central differences of the loss on 64 entries spread over U (upper
    triangle), B and the shifts, real and imaginary directions, at the full
    4096 x 2048 size, against the FP64 autograd gradient."""
    import torch
    w, Xo, Yo, gU, gl, gB = c5
    announce("c5 finite differences, 64 entries")
    _, gUd, gld, gBd = _autograd(P, w, 0, 2)
    gmax = max(np.abs(gUd).max(), np.abs(gld).max(), np.abs(gBd).max())
    Wt = torch.from_numpy(w.extra["W"]).cuda()
    Ud, sd, Bd = dev(w.U), dev(w.shifts), dev(w.B)
    m, n = w.m, w.n
    h = 1e-6

    def dloss(which, idx, d):
        # L(+h d) - L(-h d) from X+ - X- (exact subtraction of nearby values)
        Xs = []
        for sgn in (1.0, -1.0):
            t = {"U": Ud, "B": Bd, "s": sd}[which]
            old = t[idx].clone()
            t[idx] = old + sgn * h * d
            X = P.mstrsm(Ud, sd, Bd.clone())
            torch.cuda.synchronize()
            t[idx] = old
            Xs.append(X)
        D = Xs[0] - Xs[1]
        S = Xs[0] + Xs[1]
        return (Wt * (D * S.conj()).real).sum().item()

    g = W.rng(503)
    cases = []
    for _ in range(22):
        a, b = sorted(g.integers(0, m, 2))
        cases.append(("U", (int(a), int(b)), gUd[a, b]))
    for _ in range(21):
        a, b = int(g.integers(0, m)), int(g.integers(0, n))
        cases.append(("B", (a, b), gBd[a, b]))
    for _ in range(21):
        j = int(g.integers(0, n))
        cases.append(("s", j, gld[j]))
    worst = 0.0
    for which, idx, an in cases:
        for d in (1.0, 1j):
            fd = dloss(which, idx, d) / (2 * h)
            a = (np.conj(an) * d).real
            tol = 1e-6 * abs(a) + 1e-9 * gmax
            worst = max(worst, abs(fd - a) / tol)
            assert abs(fd - a) <= tol, (which, idx, d, fd, a)
    print("finite differences: worst error / tolerance = %.3g" % worst)
