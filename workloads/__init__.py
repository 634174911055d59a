"""Seeded synthetic inputs for the multi-shift triangular solve.

This module is the only code shared by the CPU oracle and the GPU path. It
draws random numbers and lays them out; it holds none of the solve's
arithmetic.

Conventions
-----------
* Every array is generated on the host in float64 / complex128 with
  ``numpy.random.Generator(PCG64(seed))``.
* "Complex normal" means CN(0,1): real and imaginary parts iid N(0, 1/2),
  so that E|z|^2 = 1.
* Matrices are returned in Fortran (column-major) order, the layout the C
  interfaces take. U is upper triangular; its strict lower triangle is zero
  here (the solvers never read it).

The workloads stand in for the paper's own test matrices (random
triangular factors with shifts near the spectrum, triangular eigenvectors,
a 100x100 grid of pseudospectra shifts), which are not available as data:
see the experimental-results section of the paper.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "rng", "cnormal", "disk_uniform", "random_upper",
    "Workload", "c1_plain", "c2_triang_eig", "c3_mixed", "c4_pseudospectra",
    "c5_adjoint", "c6_generalized", "c7_gen_triang_eig", "c8_dense_eig", "c9_dense_pencil", "c10_real",
    "WORKLOADS", "nominal_flops",
]


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def cnormal(g: np.random.Generator, shape, scale: float = 1.0) -> np.ndarray:
    """iid CN(0, scale^2): re, im ~ N(0, scale^2 / 2)."""
    s = scale / math.sqrt(2.0)
    re = g.standard_normal(shape)
    im = g.standard_normal(shape)
    return (re * s + 1j * (im * s)).astype(np.complex128)


def disk_uniform(g: np.random.Generator, n: int, radius: float = 1.0,
                 center: complex = 0.0) -> np.ndarray:
    """Area-uniform points in a disk: r = R sqrt(u), theta = 2 pi v."""
    u = g.random(n)
    v = g.random(n)
    r = radius * np.sqrt(u)
    th = 2.0 * math.pi * v
    return (center + r * np.cos(th) + 1j * r * np.sin(th)).astype(np.complex128)


def annulus_uniform(g: np.random.Generator, n: int, r0: float, r1: float) -> np.ndarray:
    """Area-uniform points on the annulus r0 <= |z| <= r1."""
    u = g.random(n)
    v = g.random(n)
    r = np.sqrt(r0 * r0 + (r1 * r1 - r0 * r0) * u)
    th = 2.0 * math.pi * v
    return (r * np.cos(th) + 1j * r * np.sin(th)).astype(np.complex128)


def random_upper(g: np.random.Generator, m: int, offdiag_scale: float,
                 diag: np.ndarray) -> np.ndarray:
    """Upper-triangular m x m, off-diagonal iid CN(0, offdiag_scale^2)."""
    U = cnormal(g, (m, m), offdiag_scale)
    U = np.triu(U, 1)
    U[np.arange(m), np.arange(m)] = diag
    return np.asfortranarray(U)


@dataclass
class Workload:
    name: str
    U: np.ndarray                 # m x m upper triangular, complex128, F-order
    shifts: np.ndarray            # n complex128
    B: np.ndarray | None          # m x n complex128, F-order (None: built by the driver)
    col_len: np.ndarray | None = None   # n int32, rows used by column j
    extra: dict = field(default_factory=dict)

    @property
    def m(self) -> int:
        return self.U.shape[0]

    @property
    def n(self) -> int:
        return self.shifts.shape[0]


def c1_plain(seed: int = 1, m: int = 256, n: int = 256) -> Workload:
    """Plain solve: off-diagonal CN(0,1)/sqrt(m), diagonal uniform in the unit
    disk; shifts uniform in the disk of radius 1.5; B iid CN(0,1)."""
    g = rng(seed)
    d = disk_uniform(g, m, 1.0)
    U = random_upper(g, m, 1.0 / math.sqrt(m), d)
    lam = disk_uniform(g, n, 1.5)
    B = np.asfortranarray(cnormal(g, (m, n)))
    return Workload("c1_plain", U, lam, B)


def c2_triang_eig(seed: int = 2, m: int = 2048, dup_frac: float = 0.05) -> Workload:
    """Triangular eigenvectors: off-diagonal CN(0,1) (unscaled), diagonal CN(0,1)
    with floor(dup_frac*m) target indices set equal to the value at a random
    non-target index (exact repeats). Shift j = T(j,j); column j holds
    -T(0:j, j) on rows 0..j-1 (col_len[j] = j)."""
    g = rng(seed)
    d = cnormal(g, m)
    ndup = int(math.floor(dup_frac * m))
    targets = g.choice(m, size=ndup, replace=False)
    mask = np.ones(m, dtype=bool)
    mask[targets] = False
    sources = np.nonzero(mask)[0]
    picks = g.choice(sources, size=ndup, replace=True)
    d[targets] = d[picks]
    T = random_upper(g, m, 1.0, d)
    lam = np.array(np.diag(T), dtype=np.complex128)
    Z = np.asfortranarray(np.triu(-T, 1))
    col_len = np.arange(m, dtype=np.int32)
    return Workload("c2_triang_eig", T, lam, Z, col_len,
                    extra={"dup_targets": targets, "dup_sources": picks})


def c3_mixed(seed: int = 3, m: int = 4096, n: int = 4096) -> Workload:
    """Off-diagonal CN(0,1)/sqrt(m), diagonal area-uniform on the annulus
    0.5 <= |d| <= 2; shifts uniform in the disk of radius 0.4; B iid CN(0,1)."""
    g = rng(seed)
    d = annulus_uniform(g, m, 0.5, 2.0)
    U = random_upper(g, m, 1.0 / math.sqrt(m), d)
    lam = disk_uniform(g, n, 0.4)
    B = np.asfortranarray(cnormal(g, (m, n)))
    return Workload("c3_mixed", U, lam, B)


def c4_pseudospectra(seed: int = 4, m: int = 2000, grid: int = 100,
                     lo: float = -1.5, hi: float = 1.5) -> Workload:
    """Off-diagonal CN(0,1)/sqrt(m), diagonal exp(i theta) + 1e-2 CN(0,1);
    shifts on a grid x grid lattice over [lo,hi]^2 (endpoints included);
    start vectors iid CN(0,1), normalised per shift."""
    g = rng(seed)
    th = 2.0 * math.pi * g.random(m)
    d = np.exp(1j * th) + cnormal(g, m, 1e-2)
    U = random_upper(g, m, 1.0 / math.sqrt(m), d)
    xs = lo + (hi - lo) * np.arange(grid) / (grid - 1)
    zr, zi = np.meshgrid(xs, xs, indexing="xy")
    z = (zr + 1j * zi).reshape(-1).astype(np.complex128)
    V0 = cnormal(g, (m, z.shape[0]))
    V0 = np.asfortranarray(V0 / np.linalg.norm(V0, axis=0, keepdims=True))
    return Workload("c4_pseudospectra", U, z, V0, extra={"grid": grid})


def c5_adjoint(seed: int = 5, m: int = 4096, n: int = 2048) -> Workload:
    """As the mixed-precision workload with n = 2048 shifts; real loss weights
    W iid N(0,1) for the loss sum(W * |X|^2)."""
    g = rng(seed)
    d = annulus_uniform(g, m, 0.5, 2.0)
    U = random_upper(g, m, 1.0 / math.sqrt(m), d)
    lam = disk_uniform(g, n, 0.4)
    B = np.asfortranarray(cnormal(g, (m, n)))
    W = np.asfortranarray(g.standard_normal((m, n)))
    return Workload("c5_adjoint", U, lam, B, extra={"W": W})


def c6_generalized(seed: int = 6, m: int = 4096, n: int = 4096) -> Workload:
    """Generalized solve (U - lambda_j V) x_j = b_j on a triangular pencil:
    U as the mixed-precision workload (off-diagonal CN(0,1)/sqrt(m), diagonal
    area-uniform on the annulus 0.5 <= |d| <= 2); V off-diagonal
    CN(0,1)/sqrt(m), diagonal real uniform in [0.5, 1.5] (the real
    non-negative diagonal a complex QZ factorisation gives); shifts uniform in
    the disk of radius 0.2; B iid CN(0,1). V is in extra["V"]."""
    g = rng(seed)
    d = annulus_uniform(g, m, 0.5, 2.0)
    U = random_upper(g, m, 1.0 / math.sqrt(m), d)
    V = random_upper(g, m, 1.0 / math.sqrt(m), (0.5 + g.random(m)).astype(np.complex128))
    lam = disk_uniform(g, n, 0.2)
    B = np.asfortranarray(cnormal(g, (m, n)))
    return Workload("c6_generalized", U, lam, B, extra={"V": V})


def c7_gen_triang_eig(seed: int = 7, m: int = 2048) -> Workload:
    """Generalized triangular eigenvectors of the pencil (T, S): T as the
    triangular-eigenvector workload without repeats (off-diagonal CN(0,1),
    diagonal CN(0,1)), S off-diagonal CN(0,1)/sqrt(m), diagonal real uniform in
    [0.5, 1.5]. Shifts and right-hand sides are formed by the solver from
    (T, S); S is in extra["S"]."""
    g = rng(seed)
    T = random_upper(g, m, 1.0, cnormal(g, m))
    S = random_upper(g, m, 1.0 / math.sqrt(m), (0.5 + g.random(m)).astype(np.complex128))
    return Workload("c7_gen_triang_eig", T, np.zeros(m, dtype=np.complex128), None,
                    np.arange(m, dtype=np.int32), extra={"S": S})


def c8_dense_eig(seed: int = 8, m: int = 2048) -> Workload:
    """General eigenproblem: A with iid entries area-uniform in the unit disk
    (the paper's dense test matrices have entries uniform in the unit ball).
    A is in extra["A"]; the Schur factors are computed by the caller."""
    g = rng(seed)
    A = np.asfortranarray(disk_uniform(g, m * m, 1.0).reshape(m, m))
    return Workload("c8_dense_eig", np.zeros((0, 0), dtype=np.complex128),
                    np.zeros(m, dtype=np.complex128), None, extra={"A": A})


def c9_dense_pencil(seed: int = 9, m: int = 1024) -> Workload:
    """Generalized eigenproblem A x = lambda B x with A and B iid entries
    area-uniform in the unit disk; extra["A"], extra["B"]."""
    g = rng(seed)
    A = np.asfortranarray(disk_uniform(g, m * m, 1.0).reshape(m, m))
    B = np.asfortranarray(disk_uniform(g, m * m, 1.0).reshape(m, m))
    return Workload("c9_dense_pencil", np.zeros((0, 0), dtype=np.complex128),
                    np.zeros(m, dtype=np.complex128), None, extra={"A": A, "B": B})


def c10_real(seed: int = 10, m: int = 4096, n: int = 4096) -> Workload:
    """Real arithmetic: U real upper triangular, off-diagonal N(0,1)/sqrt(m),
    diagonal of random sign with modulus uniform in [0.5, 2]; real shifts
    uniform in [-0.4, 0.4]; B iid N(0,1). Arrays are float64."""
    g = rng(seed)
    U = np.triu(g.standard_normal((m, m)) / math.sqrt(m), 1)
    U[np.arange(m), np.arange(m)] = np.where(g.random(m) < 0.5, -1.0, 1.0) * (0.5 + 1.5 * g.random(m))
    lam = -0.4 + 0.8 * g.random(n)
    B = np.asfortranarray(g.standard_normal((m, n)))
    return Workload("c10_real", np.asfortranarray(U), lam, B)


WORKLOADS = {
    "c1_plain": c1_plain,
    "c2_triang_eig": c2_triang_eig,
    "c3_mixed": c3_mixed,
    "c4_pseudospectra": c4_pseudospectra,
    "c5_adjoint": c5_adjoint,
    "c6_generalized": c6_generalized,
    "c7_gen_triang_eig": c7_gen_triang_eig,
    "c8_dense_eig": c8_dense_eig,
    "c9_dense_pencil": c9_dense_pencil,
    "c10_real": c10_real,
}


def nominal_flops(m: int, n: int, col_len=None) -> float:
    """Real flops of one multi-shift solve, counting a complex multiply-add as
    8 flops: 4 m^2 n, or sum_j 4 L_j^2 for variable-length columns."""
    if col_len is None:
        return 4.0 * m * m * n
    L = np.asarray(col_len, dtype=np.float64)
    return float(4.0 * np.sum(L * L))
