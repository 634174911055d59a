"""Pseudospectra drivers around the inverse-Lanczos resolvent-norm kernel
(Sec. 5, Alg 7), in the shapes the paper lists for Elemental: the resolvent
norm at user shifts (a "cloud"), over a user grid (a "window"), and over a grid
chosen from the spectrum (a "portrait"), plus level-set segments for contour
output.

The GPU work is one call of `lanczos_sigma_min` (all grid points at once: one
upper and one adjoint multi-shift solve per Lanczos step, a fixed number of
steps), or, with a tolerance `tol`, of `lanczos_restarted_sigma_min` (thick
restart with a per-shift stopping test); the grid, the start vectors and the
contour extraction are host-side set-up and post-processing.

Automatic window (the paper gives no rule): the square centred on the midpoint
of the eigenvalues' bounding box, of side (1 + 2 pad) times the larger of its
two spans, but at least `min_side` times max(1, max |lambda|).
"""
from __future__ import annotations

import numpy as np
import torch

from . import lanczos_restarted_sigma_min, lanczos_sigma_min


def window_grid(center: complex, width: float, height: float, nx: int, ny: int):
    """Grid of nx x ny points over the rectangle centred at `center`,
    endpoints included. Returns (xs, ys, shifts) with shifts[iy * nx + ix] =
    xs[ix] + 1j * ys[iy]."""
    if nx < 1 or ny < 1:
        raise ValueError("nx, ny >= 1")
    c = complex(center)
    xs = c.real - 0.5 * width + width * (np.arange(nx) / max(nx - 1, 1))
    ys = c.imag - 0.5 * height + height * (np.arange(ny) / max(ny - 1, 1))
    if nx == 1:
        xs = np.array([c.real])
    if ny == 1:
        ys = np.array([c.imag])
    zr, zi = np.meshgrid(xs, ys, indexing="xy")
    return xs, ys, (zr + 1j * zi).reshape(-1).astype(np.complex128)


def portrait_window(eigs, pad: float = 0.2, min_side: float = 1e-2):
    """Automatic window for a spectral portrait: (center, width, height)."""
    ev = np.asarray(eigs, dtype=np.complex128).reshape(-1)
    if ev.size == 0:
        raise ValueError("no eigenvalues")
    lo_r, hi_r = ev.real.min(), ev.real.max()
    lo_i, hi_i = ev.imag.min(), ev.imag.max()
    center = complex(0.5 * (lo_r + hi_r), 0.5 * (lo_i + hi_i))
    span = max(hi_r - lo_r, hi_i - lo_i)
    side = max((1.0 + 2.0 * pad) * span, min_side * max(1.0, float(np.abs(ev).max())))
    return center, side, side


def _start_vectors(m: int, n: int, seed: int, device) -> torch.Tensor:
    g = torch.Generator(device="cpu").manual_seed(int(seed))
    re = torch.randn((n, m), generator=g, dtype=torch.float64)
    im = torch.randn((n, m), generator=g, dtype=torch.float64)
    v = torch.complex(re, im).t()   # m x n, column-major (start vector j = column j)
    return v.to(device)


def spectral_cloud(U, shifts, *, iters: int = 15, seed: int = 0, V0=None, tol=None, kdim: int = 20,
                   keep: int = 6, max_restarts: int = 30):
    """sigma_min(U - z I) estimates at arbitrary shifts z (U upper triangular,
    device tensor). tol None: `iters` plain Lanczos steps; otherwise thick-
    restart Lanczos until the relative residual of each shift's top Ritz pair
    is <= tol (basis kdim, keep Ritz vectors, at most max_restarts restarts).
    Returns a device tensor of len(shifts)."""
    dev = U.device
    z = torch.as_tensor(np.asarray(shifts, dtype=np.complex128)).to(dev)
    if V0 is None:
        V0 = _start_vectors(U.shape[0], z.numel(), seed, dev)
    if tol is not None:
        sigma, _, _, _ = lanczos_restarted_sigma_min(U, z, V0, kdim=kdim, keep=keep,
                                                     max_restarts=max_restarts, tol=tol)
        return sigma
    sigma, _, _, _ = lanczos_sigma_min(U, z, V0, iters=iters)
    return sigma


def spectral_window(U, center, width, height, nx: int = 100, ny: int = 100, *, iters: int = 15,
                    seed: int = 0, tol=None):
    """Resolvent-norm data over a user window: (xs, ys, sigma) with
    sigma[iy, ix] ~ sigma_min(U - (xs[ix] + i ys[iy]) I) on the host (tol as
    for spectral_cloud)."""
    xs, ys, z = window_grid(center, width, height, nx, ny)
    sigma = spectral_cloud(U, z, iters=iters, seed=seed, tol=tol)
    return xs, ys, sigma.cpu().numpy().reshape(ny, nx)


def spectral_portrait(A, nx: int = 100, ny: int = 100, *, iters: int = 15, seed: int = 0,
                      triangular: bool = False, pad: float = 0.2, tol=None):
    """Spectral portrait of A: the Schur form on the host unless `triangular`,
    an automatic window around the eigenvalues, then the resolvent-norm grid on
    the GPU. Returns (xs, ys, sigma, eigs)."""
    import scipy.linalg as sla
    if triangular:
        U = A if isinstance(A, torch.Tensor) else torch.as_tensor(np.asarray(A, dtype=np.complex128))
        U = U.to("cuda") if not U.is_cuda else U
        eigs = torch.diagonal(U).cpu().numpy()
    else:
        An = A.detach().cpu().numpy() if isinstance(A, torch.Tensor) else np.asarray(A)
        T, _ = sla.schur(An.astype(np.complex128), output="complex")
        U = torch.as_tensor(T).to("cuda")
        eigs = np.diag(T).copy()
    center, w, h = portrait_window(eigs, pad=pad)
    xs, ys, sigma = spectral_window(U, center, w, h, nx, ny, iters=iters, seed=seed, tol=tol)
    return xs, ys, sigma, eigs


def contour_segments(xs, ys, field, level: float) -> np.ndarray:
    """Line segments of the level set field = level on the grid (marching
    squares, linear interpolation along cell edges; the two ambiguous saddle
    cases are split by the cell-centre average). field[iy, ix] lives at
    (xs[ix], ys[iy]). Returns an array (k, 2, 2) of segment end points
    ((x0, y0), (x1, y1))."""
    F = np.asarray(field, dtype=np.float64)
    xs = np.asarray(xs, dtype=np.float64)
    ys = np.asarray(ys, dtype=np.float64)
    ny, nx = F.shape
    segs = []

    def cross(p, q, fp, fq):
        t = (level - fp) / (fq - fp)
        return (p[0] + t * (q[0] - p[0]), p[1] + t * (q[1] - p[1]))

    for iy in range(ny - 1):
        for ix in range(nx - 1):
            # corners counter-clockwise: (x0,y0), (x1,y0), (x1,y1), (x0,y1)
            P = [(xs[ix], ys[iy]), (xs[ix + 1], ys[iy]), (xs[ix + 1], ys[iy + 1]), (xs[ix], ys[iy + 1])]
            v = [F[iy, ix], F[iy, ix + 1], F[iy + 1, ix + 1], F[iy + 1, ix]]
            above = [x >= level for x in v]
            pts = []
            for e in range(4):
                a, b = e, (e + 1) % 4
                if above[a] != above[b]:
                    pts.append(cross(P[a], P[b], v[a], v[b]))
            if len(pts) == 2:
                segs.append((pts[0], pts[1]))
            elif len(pts) == 4:
                # saddle: pair the crossings so that the centre value decides
                # (pts[e] lies on edge e, between corners e and e + 1)
                mid_above = 0.25 * sum(v) >= level
                if mid_above == above[0]:
                    # corners 0 and 2 connect through the centre: cut off 1 and 3
                    segs.append((pts[0], pts[1]))
                    segs.append((pts[2], pts[3]))
                else:
                    # cut off corners 0 and 2
                    segs.append((pts[3], pts[0]))
                    segs.append((pts[1], pts[2]))
    return np.array(segs, dtype=np.float64).reshape(-1, 2, 2)
