"""CPU oracle for the (safe) multi-shift triangular solve — TEST INFRASTRUCTURE.

Only ``tests/``, the smoke check and the benchmark's CPU-baseline leg may use
this package. The GPU library never imports it, and this package never imports
the GPU library: the two share no code. The only shared module is
``workloads`` (seeded input generators, no solver arithmetic).

What each function follows (T. Moon, J. Poulson, arXiv 1607.01477):

* :func:`solve` — back substitution, Alg 1 (Sec. 2) on ``U - lambda_j I``
  for each shift, the per-column content of Alg 3.
* :func:`solve_safe` — Alg 4 (Sec. 3) per column (``nb=0``), or Alg 5 (Sec. 3)
  with decision block size ``nb``; scale factors ``s_j = 2^-k_j``.
* :func:`solve_real` — the real-arithmetic solve (real U, shifts and B).
* :func:`solve_op` — the lower-triangular and (conjugate-)transposed variants
  of the footnote to Sec. 2, op(A - lambda_j I) x_j = b_j.
* :func:`solve_gen` — the generalized solve ``(U - lambda_j V) x_j = b_j``
  of the appendix (Alg 8), unblocked: back substitution on the shifted pencil.
* :func:`solve_safe_gen` — its safe form, Alg 9: Alg 4 on each shifted
  diagonal block U(I1,I1) - lambda_j V(I1,I1), column bound with both norms.
* :func:`solve_adjoint` — forward substitution with ``(U - lambda_j I)^H``, the
  lower-triangular variant noted in the footnote to Sec. 2.
* :func:`gradient` — gradients of a real loss through the solve (not in the
  paper): ``gB = Y``, ``gU = -triu(Y X^H)``, ``glambda_j = x_j^H y_j``.
* :func:`triang_eig` — TriangEig, Alg 6 (Sec. 4).
* :func:`gen_triang_eig` — GeneralizedTriangEig (appendix, Alg 10).
* :func:`eig_schur`, :func:`gen_eig_schur` — the rest of Eig (Alg 6) and of
  GeneralizedEig (Alg 10) after the (generalized) Schur decomposition: the
  back-transformation X = Q Z (resp. P Z), a library matmul, and columns
  scaled to unit 2-norm.
* :func:`portrait_grid` — the grid of the automatic pseudospectra window.
* :func:`lanczos_sigma_min` — second stage of the Van Loan/Lui method, Alg 7
  (Sec. 5): Lanczos on ``(U - zI)^{-H}(U - zI)^{-1}``.

The C part is built with gcc (``-O2 -fno-fast-math -ffp-contract=off
-fopenmp``) by :func:`build`.

Parity: pinned by ``tests/test_oracle_*.py`` (closed forms, library solvers,
brute force, hand-traced scaling examples, invariants). The Lanczos estimate
is pinned only through the diagonal closed form, the Ritz inequality and
dense SVDs; its agreement with any other Lanczos run is "parity unpinned"
beyond those.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import sys
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mstrsm_oracle.c")
_LIB = os.path.join(_HERE, "liboracle_mstrsm.so")
_lock = threading.Lock()
_lib = None

OMEGA_LOG2 = 960


def build(force: bool = False) -> str:
    """Compile the C oracle into oracle/liboracle_mstrsm.so."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-std=c11", "-O2", "-fno-fast-math", "-ffp-contract=off", "-fopenmp",
               "-fPIC", "-shared", "-Wall", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    with _lock:
        if _lib is None:
            build()
            lib = ctypes.CDLL(_LIB)
            P = ctypes.c_void_p
            I = ctypes.c_int
            lib.oracle_mstrsm.argtypes = [I, I, P, I, P, P, I]
            lib.oracle_mstrsm_adjoint.argtypes = [I, I, P, I, P, P, I]
            lib.oracle_mstrsm_safe.argtypes = [I, I, P, I, P, P, I, P, P, P, I, I, I, P]
            lib.oracle_mstrsm_gen.argtypes = [I, I, P, I, P, I, P, P, I]
            lib.oracle_mstrsm_safe_gen.argtypes = [I, I, P, I, P, I, P, P, I, P, P, P, I, I, I]
            lib.oracle_mstrsm_op.argtypes = [I, I, I, I, P, I, P, P, I]
            lib.oracle_mstrsm_real.argtypes = [I, I, P, I, P, P, I]
            for f in (lib.oracle_mstrsm, lib.oracle_mstrsm_adjoint, lib.oracle_mstrsm_safe,
                      lib.oracle_mstrsm_gen, lib.oracle_mstrsm_safe_gen, lib.oracle_mstrsm_op,
                      lib.oracle_mstrsm_real):
                f.restype = I
            lib.oracle_num_threads.restype = I
            lib.oracle_set_num_threads.argtypes = [I]
            _lib = lib
    return _lib


def num_threads() -> int:
    return _load().oracle_num_threads()


def set_num_threads(t: int) -> None:
    _load().oracle_set_num_threads(int(t))


def _cm(a) -> np.ndarray:
    return np.asfortranarray(np.asarray(a, dtype=np.complex128))


def _ptr(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data) if a is not None and a.size else None


def solve(U, lam, B) -> np.ndarray:
    """X with (U - lam[j] I) X[:, j] = B[:, j] (plain; singular systems give inf/NaN)."""
    U = _cm(U)
    lam = np.ascontiguousarray(lam, dtype=np.complex128)
    X = _cm(B).copy(order="F")
    m, n = X.shape
    if U.shape != (m, m) or lam.shape != (n,):
        raise ValueError("shape mismatch")
    rc = _load().oracle_mstrsm(m, n, _ptr(U), max(1, m), _ptr(lam), _ptr(X), max(1, m))
    if rc != 0:
        raise RuntimeError("oracle_mstrsm failed: %d" % rc)
    return X


def solve_real(U, lam, B) -> np.ndarray:
    """Real arithmetic: X with (U - lam[j] I) X[:, j] = B[:, j], U, lam, B real
    (back substitution, Alg 1, in float64)."""
    U = np.asfortranarray(np.asarray(U, dtype=np.float64))
    lam = np.ascontiguousarray(lam, dtype=np.float64)
    X = np.asfortranarray(np.asarray(B, dtype=np.float64)).copy(order="F")
    m, n = X.shape
    if U.shape != (m, m) or lam.shape != (n,):
        raise ValueError("shape mismatch")
    rc = _load().oracle_mstrsm_real(m, n, _ptr(U), max(1, m), _ptr(lam), _ptr(X), max(1, m))
    if rc != 0:
        raise RuntimeError("oracle_mstrsm_real failed: %d" % rc)
    return X


def solve_op(A, lam, B, uplo: str = "U", op: str = "N") -> np.ndarray:
    """X with op(A - lam[j] I) X[:, j] = B[:, j] for A upper ('U') or lower
    ('L') triangular and op 'N', 'T' (transpose) or 'C' (conjugate
    transpose): the variants of the footnote to Sec. 2 (back substitution when
    op(A) is upper triangular, forward substitution when it is lower)."""
    A = _cm(A)
    lam = np.ascontiguousarray(lam, dtype=np.complex128)
    X = _cm(B).copy(order="F")
    m, n = X.shape
    if A.shape != (m, m) or lam.shape != (n,):
        raise ValueError("shape mismatch")
    rc = _load().oracle_mstrsm_op(ord(uplo), ord(op), m, n, _ptr(A), max(1, m), _ptr(lam), _ptr(X),
                                  max(1, m))
    if rc != 0:
        raise RuntimeError("oracle_mstrsm_op failed: %d" % rc)
    return X


def solve_gen(U, V, lam, B) -> np.ndarray:
    """X with (U - lam[j] V) X[:, j] = B[:, j], U and V upper triangular
    (appendix, Alg 8; plain, singular systems give inf/NaN)."""
    U = _cm(U)
    V = _cm(V)
    lam = np.ascontiguousarray(lam, dtype=np.complex128)
    X = _cm(B).copy(order="F")
    m, n = X.shape
    if U.shape != (m, m) or V.shape != (m, m) or lam.shape != (n,):
        raise ValueError("shape mismatch")
    rc = _load().oracle_mstrsm_gen(m, n, _ptr(U), max(1, m), _ptr(V), max(1, m), _ptr(lam), _ptr(X),
                                   max(1, m))
    if rc != 0:
        raise RuntimeError("oracle_mstrsm_gen failed: %d" % rc)
    return X


def solve_adjoint(U, lam, G) -> np.ndarray:
    """Y with (U - lam[j] I)^H Y[:, j] = G[:, j]."""
    U = _cm(U)
    lam = np.ascontiguousarray(lam, dtype=np.complex128)
    Y = _cm(G).copy(order="F")
    m, n = Y.shape
    if U.shape != (m, m) or lam.shape != (n,):
        raise ValueError("shape mismatch")
    rc = _load().oracle_mstrsm_adjoint(m, n, _ptr(U), max(1, m), _ptr(lam), _ptr(Y), max(1, m))
    if rc != 0:
        raise RuntimeError("oracle_mstrsm_adjoint failed: %d" % rc)
    return Y


def solve_safe(U, lam, B, col_len=None, nb: int = 64, omega_log2: int = OMEGA_LOG2,
               force_phase2: bool = False, trace: bool = False):
    """Safe solve: returns (X, scale, k) with (U - lam_j I) X_j = 2^-k_j B_j.

    nb = 0 applies Alg 4 to each column unblocked; nb > 0 is Alg 5 with that
    decision block size. col_len[j] limits column j to rows [0, col_len[j]).
    With trace=True also returns an array (nblocks, n, 2) of (G(j) after the
    block's bound update, max cabs1 of the rows above after its substitution).
    """
    U = _cm(U)
    lam = np.ascontiguousarray(lam, dtype=np.complex128)
    X = _cm(B).copy(order="F")
    m, n = X.shape
    if U.shape != (m, m) or lam.shape != (n,):
        raise ValueError("shape mismatch")
    cl = None
    if col_len is not None:
        cl = np.ascontiguousarray(col_len, dtype=np.int32)
        if cl.shape != (n,):
            raise ValueError("col_len shape")
    scale = np.zeros(n, dtype=np.float64)
    k = np.zeros(n, dtype=np.int32)
    nbe = m if (nb <= 0 or nb >= m) else nb
    nblk = (m + nbe - 1) // nbe if m > 0 else 0
    tr = np.zeros((max(nblk, 1), n, 2), dtype=np.float64) if trace else None
    rc = _load().oracle_mstrsm_safe(m, n, _ptr(U), max(1, m), _ptr(lam), _ptr(X), max(1, m),
                                    _ptr(cl) if cl is not None else None,
                                    _ptr(scale), _ptr(k), int(nb), int(omega_log2),
                                    int(bool(force_phase2)), _ptr(tr) if tr is not None else None)
    if rc != 0:
        raise RuntimeError("oracle_mstrsm_safe failed: %d" % rc)
    if trace:
        return X, scale, k, tr[:nblk]
    return X, scale, k


def solve_safe_gen(U, V, lam, B, col_len=None, nb: int = 64, omega_log2: int = OMEGA_LOG2,
                   force_phase2: bool = False):
    """Safe generalized solve (appendix, Alg 9): returns (X, scale, k) with
    (U - lam_j V) X_j = 2^-k_j B_j. nb and col_len as in :func:`solve_safe`."""
    U = _cm(U)
    V = _cm(V)
    lam = np.ascontiguousarray(lam, dtype=np.complex128)
    X = _cm(B).copy(order="F")
    m, n = X.shape
    if U.shape != (m, m) or V.shape != (m, m) or lam.shape != (n,):
        raise ValueError("shape mismatch")
    cl = None
    if col_len is not None:
        cl = np.ascontiguousarray(col_len, dtype=np.int32)
        if cl.shape != (n,):
            raise ValueError("col_len shape")
    scale = np.zeros(n, dtype=np.float64)
    k = np.zeros(n, dtype=np.int32)
    rc = _load().oracle_mstrsm_safe_gen(m, n, _ptr(U), max(1, m), _ptr(V), max(1, m), _ptr(lam),
                                        _ptr(X), max(1, m), _ptr(cl) if cl is not None else None,
                                        _ptr(scale), _ptr(k), int(nb), int(omega_log2),
                                        int(bool(force_phase2)))
    if rc != 0:
        raise RuntimeError("oracle_mstrsm_safe_gen failed: %d" % rc)
    return X, scale, k


def gradient(U, lam, X, Y):
    """Gradients of a real loss L through X = solve(U, lam, B), given
    Y = solve_adjoint(U, lam, dL/dX) (PyTorch convention: the gradient of a
    complex input z is dL/dRe z + i dL/dIm z).

    gB = Y; gU = -triu(Y X^H); glam_j = sum_i conj(X_ij) Y_ij.
    """
    Y = np.asarray(Y)
    X = np.asarray(X)
    gU = -np.triu(Y @ X.conj().T)
    glam = np.sum(X.conj() * Y, axis=0)
    return gU, glam, Y.copy()


def triang_eig(T, nb: int = 64, omega_log2: int = OMEGA_LOG2, force_phase2: bool = False):
    """TriangEig (Alg 6): lam = diag(T); Z = -T with zero diagonal; safe
    multi-shift solve with column j limited to rows [0, j); diag(Z) = s.
    Returns (lam, Z, k) with T Z[:, j] = lam_j Z[:, j] and Z(j, j) = 2^-k_j."""
    T = _cm(T)
    m = T.shape[0]
    lam = np.array(np.diag(T), dtype=np.complex128)
    Z = np.asfortranarray(np.triu(-T, 1))
    col_len = np.arange(m, dtype=np.int32)
    Z, s, k = solve_safe(T, lam, Z, col_len=col_len, nb=nb, omega_log2=omega_log2,
                         force_phase2=force_phase2)
    Z[np.arange(m), np.arange(m)] = s
    return lam, Z, k


def gen_triang_eig(T, S, nb: int = 64, omega_log2: int = OMEGA_LOG2):
    """GeneralizedTriangEig (appendix, Alg 10): lam = diag(T) / diag(S);
    Z = -T + S diag(lam) with zero diagonal (upper triangular, so column j
    has rows [0, j) only); safe generalized solve; diag(Z) = s.
    Returns (lam, Z, k) with T Z[:, j] = lam_j S Z[:, j] and Z(j, j) = 2^-k_j.
    The diagonal of S must be nonzero (finite eigenvalues)."""
    T = _cm(T)
    S = _cm(S)
    m = T.shape[0]
    lam = np.array(np.diag(T) / np.diag(S), dtype=np.complex128)
    Z = np.asfortranarray(np.triu(-T + S * lam[None, :], 1))
    col_len = np.arange(m, dtype=np.int32)
    Z, s, k = solve_safe_gen(T, S, lam, Z, col_len=col_len, nb=nb, omega_log2=omega_log2)
    Z[np.arange(m), np.arange(m)] = s
    return lam, Z, k


def _unit_columns(X) -> np.ndarray:
    # every column scaled to unit 2-norm (columns that are zero stay zero)
    nrm = np.sqrt(np.sum(X.real ** 2 + X.imag ** 2, axis=0))
    return np.asfortranarray(X / np.where(nrm > 0, nrm, 1.0)[None, :])


def eig_schur(T, Q, nb: int = 64, omega_log2: int = OMEGA_LOG2):
    """Eig (Alg 6) after its Schur step: given A = Q T Q^H, lam, Z =
    TriangEig(T), X = Q Z (the back-transformation), columns scaled to unit
    2-norm. Returns (lam, X) with A X = X diag(lam)."""
    lam, Z, _ = triang_eig(T, nb=nb, omega_log2=omega_log2)
    return lam, _unit_columns(_cm(Q) @ Z)


def gen_eig_schur(T, S, P, nb: int = 64, omega_log2: int = OMEGA_LOG2):
    """GeneralizedEig (appendix, Alg 10) after its generalized Schur step:
    given A = Q T P^H, B = Q S P^H, lam, Z = GeneralizedTriangEig(T, S),
    X = P Z, columns scaled to unit 2-norm. Returns (lam, X) with
    A X = B X diag(lam)."""
    lam, Z, _ = gen_triang_eig(T, S, nb=nb, omega_log2=omega_log2)
    return lam, _unit_columns(_cm(P) @ Z)


def portrait_grid(eigs, nx: int, ny: int, pad: float = 0.2, min_side: float = 1e-2):
    """Grid of a spectral portrait (the automatic window of the pseudospectra
    driver): the square around the eigenvalues' bounding box, side
    (1 + 2 pad) max(re span, im span), at least min_side max(1, max|lambda|),
    nx x ny points with endpoints, point (ix, iy) at index iy nx + ix."""
    ev = np.asarray(eigs, dtype=np.complex128)
    re0, re1 = float(np.min(ev.real)), float(np.max(ev.real))
    im0, im1 = float(np.min(ev.imag)), float(np.max(ev.imag))
    side = (1.0 + 2.0 * pad) * max(re1 - re0, im1 - im0)
    side = max(side, min_side * max(1.0, float(np.max(np.abs(ev)))))
    cx, cy = (re0 + re1) / 2.0, (im0 + im1) / 2.0
    pts = np.empty(nx * ny, dtype=np.complex128)
    for iy in range(ny):
        y = cy - side / 2.0 + side * (iy / (ny - 1) if ny > 1 else 0.5)
        for ix in range(nx):
            x = cx - side / 2.0 + side * (ix / (nx - 1) if nx > 1 else 0.5)
            pts[iy * nx + ix] = complex(x, y)
    return pts


def relative_residual(U, lam, X, B, k=None, cols=None) -> np.ndarray:
    """Per column ||(U - lam_j I) x_j - 2^-k_j b_j||_inf / (||U - lam_j I||_inf ||x_j||_inf)
    with the true modulus; absolute residual where x_j = 0."""
    U = np.asarray(U)
    X = np.asarray(X)
    B = np.asarray(B)
    lam = np.asarray(lam)
    if cols is None:
        cols = np.arange(X.shape[1])
    cols = np.asarray(cols)
    Xc = X[:, cols]
    Bc = B[:, cols]
    if k is not None:
        Bc = Bc * np.ldexp(1.0, -np.asarray(k)[cols].astype(np.int64))[None, :]
    Ut = np.triu(U)
    R = Ut @ Xc - Xc * lam[cols][None, :] - Bc
    offrow = np.sum(np.abs(np.triu(U, 1)), axis=1)
    d = np.diag(U)
    unorm = np.max(offrow[:, None] + np.abs(d[:, None] - lam[cols][None, :]), axis=0)
    rn = np.max(np.abs(R), axis=0)
    xn = np.max(np.abs(Xc), axis=0)
    den = unorm * xn
    out = np.where(den > 0, rn / np.where(den > 0, den, 1.0), rn)
    return out


def _theta_max(alpha: np.ndarray, beta: np.ndarray) -> float:
    from scipy.linalg import eigvalsh_tridiagonal
    if alpha.size == 1:
        return float(alpha[0])
    return float(eigvalsh_tridiagonal(alpha, beta)[-1])


def lanczos_sigma_min(U, z, V0, iters: int = 15):
    """Inverse Lanczos estimate of sigma_min(U - z_j I) for every shift z_j.

    Plain Lanczos (no reorthogonalisation) on A_j = (U - z_j I)^{-H}(U - z_j I)^{-1}
    with start vector V0[:, j] (normalised here), each product computed as one
    upper and one adjoint multi-shift solve over all shifts at once:
      w = A v_k; alpha_k = Re(v_k^H w); w -= alpha_k v_k + beta_{k-1} v_{k-1};
      beta_k = ||w||_2; v_{k+1} = w / beta_k (stop early only if beta_k = 0).
    theta_max = largest eigenvalue of the k x k tridiagonal; sigma = theta^-1/2.
    Returns (sigma, alpha, beta, steps)."""
    U = _cm(U)
    z = np.ascontiguousarray(z, dtype=np.complex128)
    V = _cm(V0).copy(order="F")
    m, N = V.shape
    V = V / np.linalg.norm(V, axis=0, keepdims=True)
    Vprev = np.zeros_like(V)
    alpha = np.zeros((iters, N))
    beta = np.zeros((iters, N))
    steps = np.full(N, iters, dtype=np.int64)
    bprev = np.zeros(N)
    active = np.ones(N, dtype=bool)
    for it in range(iters):
        Y = solve(U, z, V)
        W = solve_adjoint(U, z, Y)
        a = np.real(np.sum(V.conj() * W, axis=0))
        W = W - a[None, :] * V - bprev[None, :] * Vprev
        b = np.linalg.norm(W, axis=0)
        alpha[it] = np.where(active, a, 0.0)
        beta[it] = np.where(active, b, 0.0)
        stop = active & (b == 0.0)
        steps[stop] = it + 1
        active = active & ~stop
        Vprev = V
        V = W / np.where(b > 0, b, 1.0)[None, :]
        bprev = b
    sigma = np.empty(N)
    for j in range(N):
        s = int(steps[j])
        th = _theta_max(alpha[:s, j], beta[:s - 1, j])
        sigma[j] = 1.0 / np.sqrt(th)
    return sigma, alpha, beta, steps


def lanczos_restarted_sigma_min(U, z, V0, kdim: int = 20, keep: int = 6, max_restarts: int = 30,
                                tol: float = 1e-10, return_vectors: bool = False):
    """Thick-restart Lanczos for sigma_min(U - z_j I) of every shift z_j: the
    largest eigenvalue theta of the Hermitian positive definite
    A_j = (U - z_j I)^{-H}(U - z_j I)^{-1} (Alg 7, Sec. 5, the Krylov part of its
    second stage; the paper's own runs used implicitly restarted Arnoldi, on a
    Hermitian operator the same Krylov spaces as thick-restart Lanczos, Wu and
    Simon 2000). Per shift, cycles of Lanczos steps with full
    reorthogonalisation (classical Gram-Schmidt applied twice) build a basis of
    kdim vectors; Rayleigh-Ritz on the projected matrix gives the Ritz pairs
    (theta_l, y_l), the top one's residual norm being |beta S(kdim-1, 0)|. A
    shift is done when that is <= tol * theta_0, or after max_restarts
    restarts; otherwise the next cycle starts from the keep largest Ritz
    vectors and the last Lanczos vector, whose projected matrix is
    diag(theta_0..theta_{keep-1}) bordered by beta S(kdim-1, l) (an arrowhead),
    and the first step of the cycle removes that border instead of the
    three-term predecessor. All shifts advance together: each Lanczos step is
    one upper and one adjoint multi-shift solve over the shifts still running.
    Start vectors V0 (normalised here).
    Returns (sigma, resid, steps, converged[, Y]) with sigma = theta_0^{-1/2},
    resid = |beta S(kdim-1, 0)| / theta_0 (relative residual of the top Ritz
    pair), steps the Lanczos steps taken per shift, and Y the top Ritz vectors."""
    U = _cm(U)
    z = np.ascontiguousarray(z, dtype=np.complex128)
    V = _cm(V0)
    m, N = V.shape
    if not (1 <= keep < kdim):
        raise ValueError("need 1 <= keep < kdim")
    Q = np.zeros((kdim + 1, m, N), dtype=np.complex128)
    Q[0] = V / np.linalg.norm(V, axis=0, keepdims=True)
    H = np.zeros((N, kdim, kdim))
    sigma = np.zeros(N)
    resid = np.zeros(N)
    steps = np.zeros(N, dtype=np.int64)
    conv = np.zeros(N, dtype=bool)
    Yout = np.zeros((m, N), dtype=np.complex128) if return_vectors else None
    act = np.arange(N)
    k0 = 0
    for cycle in range(max_restarts + 1):
        za = z[act]
        beta = np.zeros(act.size)
        for i in range(k0, kdim):
            qi = Q[i][:, act]
            W = solve_adjoint(U, za, solve(U, za, qi))
            if i == k0 and k0 > 0:
                # first step after a restart: remove the arrowhead border
                for l in range(k0):
                    W = W - H[act, l, k0][None, :] * Q[l][:, act]
            elif i > 0:
                W = W - H[act, i - 1, i][None, :] * Q[i - 1][:, act]
            alpha = np.real(np.sum(qi.conj() * W, axis=0))
            W = W - alpha[None, :] * qi
            for _ in range(2):
                Qb = Q[:i + 1][:, :, act]
                h = np.einsum("lmn,mn->ln", Qb.conj(), W)
                W = W - np.einsum("lmn,ln->mn", Qb, h)
                alpha = alpha + np.real(h[i])
            beta = np.linalg.norm(W, axis=0)
            H[act, i, i] = alpha
            if i + 1 < kdim:
                H[act, i, i + 1] = beta
                H[act, i + 1, i] = beta
            Q[i + 1][:, act] = W / np.where(beta > 0, beta, 1.0)[None, :]
            steps[act] += 1
        th, S = np.linalg.eigh(H[act])
        th = th[:, ::-1]
        S = S[:, :, ::-1]
        res = np.abs(beta * S[:, kdim - 1, 0])
        sigma[act] = 1.0 / np.sqrt(th[:, 0])
        resid[act] = res / th[:, 0]
        done = res <= tol * th[:, 0]
        conv[act[done]] = True
        if return_vectors:
            Yout[:, act] = np.einsum("lmn,nl->mn", Q[:kdim][:, :, act], S[:, :, 0])
        if cycle == max_restarts or np.all(done):
            break
        # thick restart of the shifts still running
        keep_idx = ~done
        R = act[keep_idx]
        Sk = S[keep_idx]
        newq = np.einsum("lmn,nlk->kmn", Q[:kdim][:, :, R], Sk[:, :, :keep])
        for l in range(keep):
            Q[l][:, R] = newq[l]
        Q[keep][:, R] = Q[kdim][:, R]
        H[R] = 0.0
        for l in range(keep):
            H[R, l, l] = th[keep_idx, l]
            H[R, l, keep] = beta[keep_idx] * Sk[:, kdim - 1, l]
            H[R, keep, l] = H[R, l, keep]
        act = R
        k0 = keep
    if return_vectors:
        return sigma, resid, steps, conv, Yout
    return sigma, resid, steps, conv


__all__ = ["build", "solve", "solve_safe", "solve_adjoint", "gradient", "triang_eig",
           "solve_gen", "solve_safe_gen", "gen_triang_eig", "eig_schur", "gen_eig_schur", "solve_op",
           "portrait_grid", "solve_real",
           "relative_residual", "lanczos_sigma_min", "lanczos_restarted_sigma_min", "num_threads",
           "set_num_threads",
           "OMEGA_LOG2"]

if __name__ == "__main__":  # pragma: no cover
    print(build(force="--force" in sys.argv))
