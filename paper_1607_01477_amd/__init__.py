"""Blocked multi-shift triangular solves on AMD MI355X (gfx950).

Python binding of ``libmstrsm.so`` (C-ABI declared in ``include/mstrsm.h``).
Keyword options left at 0 take the library's defaults (nb = 16; outer_nb = 256, or 512 in plain back substitutions with few shifts).
Every function here only marshals arguments: tensors must be complex128 (int32
for ``col_len``) on a ROCm device; matrices are passed column-major (a
Fortran-ordered view, ``t.stride(0) == 1``), copied into that layout if they
are not. All work is enqueued on the current torch stream.

Method: T. Moon, J. Poulson, "Accelerating eigenvector and pseudospectra
computation using blocked multi-shift triangular solves" (arXiv 1607.01477):
Alg 3 (multi-shift solve), Alg 4/5 (safe solve), Alg 6 (triangular
eigenvectors), Alg 7 (resolvent norms).
"""
from __future__ import annotations

import ctypes

import torch

from . import _lib
from ._lib import MstError, MstOpts

__all__ = ["mstrsm", "mstrsm_safe", "mstrsm_safe_noalloc", "mstrsm_adjoint", "grad_u", "grad_shift", "residual",
           "triang_eig", "lanczos_sigma_min", "lanczos_restarted_sigma_min", "mstrsm_gen", "mstrsm_safe_gen", "gen_triang_eig",
           "eig_schur", "gen_eig_schur", "eig", "gen_eig", "mstrsm_op", "mstrsm_real", "mstrsm_real_op",
           "solve", "MultiShiftSolve", "colmajor",
           "MstError", "version", "lib_path"]

lib_path = _lib.LIB_PATH


def version() -> str:
    return _lib.load().mst_version().decode()


def _opts(nb=0, outer_nb=0, precision=0, max_sweeps=0, omega_log2=0, force_phase2=0, fuse=True,
          staged=False, overlap=False, refine_tol=0.0, refine_report=None, gemm_split=0, fuse_width=0):
    o = MstOpts()
    o.gemm_split = int(gemm_split)
    o.refine_tol = float(refine_tol)
    o.refine_report = refine_report.data_ptr() if refine_report is not None else None
    o.overlap = 1 if overlap else 0
    o.gemm_staged = 1 if staged else 0
    o.nb, o.outer_nb, o.precision = int(nb), int(outer_nb), int(precision)
    o.max_sweeps, o.omega_log2, o.force_phase2 = int(max_sweeps), int(omega_log2), int(force_phase2)
    if fuse_width not in (0, 1, 2, 4, 16):
        raise ValueError("fuse_width must be 0 (automatic), 1, 2, 4 or 16")
    o.fuse_blocks = {0: 0, 16: 1, 4: 2, 2: 3, 1: 4}[fuse_width] if fuse else -1
    return o


def _stream() -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _is_colmajor(t: torch.Tensor) -> bool:
    if t.dim() != 2:
        return False
    m, n = t.shape
    if m <= 1 or n <= 1:
        return t.is_contiguous() or t.stride(0) == 1
    return t.stride(0) == 1 and t.stride(1) >= m


def colmajor(t: torch.Tensor, dtype=torch.complex128) -> torch.Tensor:
    """The same matrix as a column-major (Fortran-ordered) tensor of `dtype`;
    `t` itself when it already is one."""
    if t.dtype != dtype:
        t = t.to(dtype)
    if _is_colmajor(t):
        return t
    return t.t().contiguous().t()


def _ld(t: torch.Tensor) -> int:
    m, n = t.shape
    if n <= 1 or m <= 1:
        return max(1, m) if t.stride(0) == 1 or m <= 1 else t.stride(0)
    return t.stride(1)


def _dev(t: torch.Tensor, name: str) -> None:
    if not t.is_cuda:
        raise ValueError("%s must be on a ROCm device" % name)


def _vec(t: torch.Tensor, n: int, name: str, dtype=torch.complex128) -> torch.Tensor:
    t = t.reshape(-1)
    if t.dtype != dtype:
        t = t.to(dtype)
    t = t.contiguous()
    if t.numel() != n:
        raise ValueError("%s must have %d entries" % (name, n))
    _dev(t, name)
    return t


def _fcopy(t: torch.Tensor) -> torch.Tensor:
    """A fresh column-major complex128 copy of matrix t."""
    m, n = t.shape
    out = torch.empty_strided((m, n), (1, max(1, m)), dtype=torch.complex128, device=t.device)
    out.copy_(t)
    return out


def _p(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None and t.numel() > 0 else None


def _mat(t: torch.Tensor, name: str) -> torch.Tensor:
    if t.dim() != 2:
        raise ValueError("%s must be a matrix" % name)
    _dev(t, name)
    return colmajor(t)


def mstrsm(U, shifts, B, *, nb=0, outer_nb=0, precision=0, max_sweeps=2, fuse=True, staged=False,
           overlap=False, refine_tol=0.0, refine_report=None, gemm_split=0, fuse_width=0):
    """X with (U - shifts[j] I) X[:, j] = B[:, j]; B is overwritten when it is
    already column-major complex128 (the result is returned either way).
    precision=1: FP32 substitution GEMMs + FP64 refinement, at most max_sweeps
    sweeps, stopping once the largest relative residual is <= refine_tol (0:
    the library's default 1e-14; negative: never early). refine_report: an
    optional float64 device tensor of max_sweeps + 1 entries that receives the
    largest relative residual after each sweep (-1 where not evaluated)."""
    U = _mat(U, "U")
    X = _mat(B, "B")
    m, n = X.shape
    if U.shape != (m, m):
        raise ValueError("U must be %d x %d" % (m, m))
    s = _vec(shifts, n, "shifts")
    if refine_report is not None:
        if (refine_report.dtype != torch.float64 or not refine_report.is_contiguous()
                or refine_report.numel() != max_sweeps + 1 or not refine_report.is_cuda):
            raise ValueError("refine_report must be a contiguous float64 device tensor of %d entries"
                             % (max_sweeps + 1))
    o = _opts(nb=nb, outer_nb=outer_nb, precision=precision, max_sweeps=max_sweeps, fuse=fuse,
              staged=staged, overlap=overlap, refine_tol=refine_tol, refine_report=refine_report,
              gemm_split=gemm_split, fuse_width=fuse_width)
    rc = _lib.load().mstrsm(m, n, _p(U), _ld(U), _p(s), _p(X), _ld(X), ctypes.byref(o), _stream())
    _lib.check("mstrsm", rc)
    return X


def mstrsm_safe(U, shifts, B, col_len=None, *, nb=0, outer_nb=0, omega_log2=0, fuse=True,
                staged=False, overlap=False, force_phase2=False, gemm_split=0, fuse_width=0):
    """Safe solve: returns (X, scale, scale_log2) with
    (U - shifts[j] I) X[:, j] = scale[j] B[:, j], scale[j] = 2^-scale_log2[j]."""
    U = _mat(U, "U")
    X = _mat(B, "B")
    m, n = X.shape
    if U.shape != (m, m):
        raise ValueError("U must be %d x %d" % (m, m))
    s = _vec(shifts, n, "shifts")
    cl = _vec(col_len, n, "col_len", torch.int32) if col_len is not None else None
    scale = torch.empty(n, dtype=torch.float64, device=X.device)
    klog = torch.empty(n, dtype=torch.int32, device=X.device)
    o = _opts(nb=nb, outer_nb=outer_nb, omega_log2=omega_log2, fuse=fuse, staged=staged,
              overlap=overlap, force_phase2=force_phase2, gemm_split=gemm_split, fuse_width=fuse_width)
    rc = _lib.load().mstrsm_safe(m, n, _p(U), _ld(U), _p(s), _p(X), _ld(X), _p(cl), _p(scale),
                                 _p(klog), ctypes.byref(o), _stream())
    _lib.check("mstrsm_safe", rc)
    return X, scale, klog


def mstrsm_safe_noalloc(U, shifts, B, col_len=None, *, scale=None, scale_log2=None, nb=0, outer_nb=0,
                        omega_log2=0, fuse=True, staged=False, gemm_split=0, fuse_width=0):
    """mstrsm_safe without device allocation inside the library: the workspace
    is the library's static scratch (16 MiB per device; calls that overlap on
    one device race). scale (float64) and scale_log2 (int32) may be given as
    preallocated device vectors of n entries; otherwise they are created here.
    Returns (X, scale, scale_log2)."""
    U = _mat(U, "U")
    X = _mat(B, "B")
    m, n = X.shape
    if U.shape != (m, m):
        raise ValueError("U must be %d x %d" % (m, m))
    s = _vec(shifts, n, "shifts")
    cl = _vec(col_len, n, "col_len", torch.int32) if col_len is not None else None
    scale = torch.empty(n, dtype=torch.float64, device=X.device) if scale is None else \
        _vec(scale, n, "scale", torch.float64)
    klog = torch.empty(n, dtype=torch.int32, device=X.device) if scale_log2 is None else \
        _vec(scale_log2, n, "scale_log2", torch.int32)
    o = _opts(nb=nb, outer_nb=outer_nb, omega_log2=omega_log2, fuse=fuse, staged=staged,
              gemm_split=gemm_split, fuse_width=fuse_width)
    rc = _lib.load().mstrsm_safe_noalloc(m, n, _p(U), _ld(U), _p(s), _p(X), _ld(X), _p(cl), _p(scale),
                                         _p(klog), ctypes.byref(o), _stream())
    _lib.check("mstrsm_safe_noalloc", rc)
    return X, scale, klog


def mstrsm_adjoint(U, shifts, G, *, nb=0, outer_nb=0, fuse=True, overlap=False, staged=False, gemm_split=0,
                   fuse_width=0):
    """Y with (U - shifts[j] I)^H Y[:, j] = G[:, j] (G overwritten when column-major)."""
    U = _mat(U, "U")
    Y = _mat(G, "G")
    m, n = Y.shape
    if U.shape != (m, m):
        raise ValueError("U must be %d x %d" % (m, m))
    s = _vec(shifts, n, "shifts")
    o = _opts(nb=nb, outer_nb=outer_nb, fuse=fuse, overlap=overlap, staged=staged, gemm_split=gemm_split,
              fuse_width=fuse_width)
    rc = _lib.load().mstrsm_adjoint(m, n, _p(U), _ld(U), _p(s), _p(Y), _ld(Y), ctypes.byref(o),
                                    _stream())
    _lib.check("mstrsm_adjoint", rc)
    return Y


def mstrsm_op(A, shifts, B, *, uplo="U", op="N", side="L", nb=0, outer_nb=0, fuse=True,
              precision=0, max_sweeps=2, fuse_width=0):
    """Variants of the footnote to Sec. 2: X with op(A - shifts[j] I) X[:, j] = B[:, j]
    (side "L") or X[:, j]^T op(A - shifts[j] I) = B[:, j]^T (side "R"), A upper
    ("U") or lower ("L") triangular, op "N", "T" or "C" (side "R": "N" or "T").
    B is overwritten when it is already column-major complex128."""
    A = _mat(A, "A")
    X = _mat(B, "B")
    m, n = X.shape
    if A.shape != (m, m):
        raise ValueError("A must be %d x %d" % (m, m))
    s = _vec(shifts, n, "shifts")
    o = _opts(nb=nb, outer_nb=outer_nb, fuse=fuse, precision=precision, max_sweeps=max_sweeps,
              fuse_width=fuse_width)
    rc = _lib.load().mstrsm_op(ord(side), ord(uplo), ord(op), m, n, _p(A), _ld(A), _p(s), _p(X), _ld(X),
                               ctypes.byref(o), _stream())
    _lib.check("mstrsm_op", rc)
    return X


def mstrsm_real(U, shifts, B, *, outer_nb=0):
    """Real arithmetic: X with (U - shifts[j] I) X[:, j] = B[:, j] for real U,
    shifts and B (float64; B overwritten when it is already column-major
    float64). Fused blocks of up to 256 rows."""
    for t, name in ((U, "U"), (B, "B")):
        if t.dim() != 2:
            raise ValueError("%s must be a matrix" % name)
        _dev(t, name)
    U = colmajor(U, torch.float64)
    X = colmajor(B, torch.float64)
    m, n = X.shape
    if U.shape != (m, m):
        raise ValueError("U must be %d x %d" % (m, m))
    s = _vec(shifts, n, "shifts", torch.float64)
    o = _opts(outer_nb=outer_nb)
    rc = _lib.load().mstrsm_real(m, n, _p(U), _ld(U), _p(s), _p(X), _ld(X), ctypes.byref(o), _stream())
    _lib.check("mstrsm_real", rc)
    return X


def mstrsm_real_op(A, shifts, B, *, uplo="U", op="N", side="L", outer_nb=0):
    """The variants of `mstrsm_op` in real arithmetic (float64): X with
    op(A - shifts[j] I) X[:, j] = B[:, j] (side "L") or
    X[:, j]^T op(A - shifts[j] I) = B[:, j]^T (side "R"), A upper ("U") or lower
    ("L"), op "N", "T" or "C" (the same as "T" for real data). B is overwritten
    when it is already column-major float64."""
    for t, name in ((A, "A"), (B, "B")):
        if t.dim() != 2:
            raise ValueError("%s must be a matrix" % name)
        _dev(t, name)
    A = colmajor(A, torch.float64)
    X = colmajor(B, torch.float64)
    m, n = X.shape
    if A.shape != (m, m):
        raise ValueError("A must be %d x %d" % (m, m))
    s = _vec(shifts, n, "shifts", torch.float64)
    o = _opts(outer_nb=outer_nb)
    rc = _lib.load().mstrsm_real_op(ord(side), ord(uplo), ord(op), m, n, _p(A), _ld(A), _p(s), _p(X), _ld(X),
                                    ctypes.byref(o), _stream())
    _lib.check("mstrsm_real_op", rc)
    return X


def grad_u(Y, X):
    """-triu(Y X^H) (m x m, strict lower triangle zero)."""
    Y = _mat(Y, "Y")
    X = _mat(X, "X")
    m, n = Y.shape
    if X.shape != (m, n):
        raise ValueError("X and Y must have the same shape")
    gU = torch.empty_strided((m, m), (1, max(1, m)), dtype=torch.complex128, device=Y.device)
    rc = _lib.load().mst_grad_u(m, n, _p(Y), _ld(Y), _p(X), _ld(X), _p(gU), max(1, m), _stream())
    _lib.check("mst_grad_u", rc)
    return gU


def grad_shift(X, Y):
    """sum_i conj(X[i, j]) Y[i, j] for every column j."""
    X = _mat(X, "X")
    Y = _mat(Y, "Y")
    m, n = X.shape
    if Y.shape != (m, n):
        raise ValueError("X and Y must have the same shape")
    out = torch.empty(n, dtype=torch.complex128, device=X.device)
    rc = _lib.load().mst_grad_shift(m, n, _p(X), _ld(X), _p(Y), _ld(Y), _p(out), _stream())
    _lib.check("mst_grad_shift", rc)
    return out


def residual(U, shifts, X, B0):
    """B0 - (U X - X diag(shifts)) in FP64 on the matrix cores."""
    U = _mat(U, "U")
    X = _mat(X, "X")
    B0 = _mat(B0, "B0")
    m, n = X.shape
    s = _vec(shifts, n, "shifts")
    R = torch.empty_strided((m, n), (1, max(1, m)), dtype=torch.complex128, device=X.device)
    rc = _lib.load().mst_residual(m, n, _p(U), _ld(U), _p(s), _p(X), _ld(X), _p(B0), _ld(B0), _p(R),
                                  max(1, m), _stream())
    _lib.check("mst_residual", rc)
    return R


def triang_eig(T, *, nb=0, outer_nb=0, omega_log2=0, force_phase2=False, gemm_split=0, fuse_width=0):
    """TriangEig (Alg 6): returns (eigvals, Z, scale_log2) with T Z[:, j] =
    eigvals[j] Z[:, j], Z upper triangular, Z[j, j] = 2^-scale_log2[j]."""
    T = _mat(T, "T")
    m = T.shape[0]
    if T.shape != (m, m):
        raise ValueError("T must be square")
    Z = torch.empty_strided((m, m), (1, max(1, m)), dtype=torch.complex128, device=T.device)
    ev = torch.empty(m, dtype=torch.complex128, device=T.device)
    klog = torch.empty(m, dtype=torch.int32, device=T.device)
    o = _opts(nb=nb, outer_nb=outer_nb, omega_log2=omega_log2, force_phase2=force_phase2,
              gemm_split=gemm_split, fuse_width=fuse_width)
    rc = _lib.load().mst_triang_eig(m, _p(T), _ld(T), _p(Z), max(1, m), _p(ev), _p(klog),
                                    ctypes.byref(o), _stream())
    _lib.check("mst_triang_eig", rc)
    return ev, Z, klog


def mstrsm_gen(U, V, shifts, B, *, outer_nb=0, fuse=True, overlap=False):
    """Generalized solve (appendix, Alg 8): X with
    (U - shifts[j] V) X[:, j] = B[:, j] (nb = 16; B overwritten when column-major)."""
    U = _mat(U, "U")
    V = _mat(V, "V")
    X = _mat(B, "B")
    m, n = X.shape
    if U.shape != (m, m) or V.shape != (m, m):
        raise ValueError("U and V must be %d x %d" % (m, m))
    s = _vec(shifts, n, "shifts")
    o = _opts(outer_nb=outer_nb, fuse=fuse, overlap=overlap)
    rc = _lib.load().mstrsm_gen(m, n, _p(U), _ld(U), _p(V), _ld(V), _p(s), _p(X), _ld(X),
                                ctypes.byref(o), _stream())
    _lib.check("mstrsm_gen", rc)
    return X


def mstrsm_safe_gen(U, V, shifts, B, col_len=None, *, outer_nb=0, omega_log2=0, fuse=True,
                    overlap=False):
    """Safe generalized solve (appendix, Alg 9): returns (X, scale, scale_log2) with
    (U - shifts[j] V) X[:, j] = scale[j] B[:, j], scale[j] = 2^-scale_log2[j]."""
    U = _mat(U, "U")
    V = _mat(V, "V")
    X = _mat(B, "B")
    m, n = X.shape
    if U.shape != (m, m) or V.shape != (m, m):
        raise ValueError("U and V must be %d x %d" % (m, m))
    s = _vec(shifts, n, "shifts")
    cl = _vec(col_len, n, "col_len", torch.int32) if col_len is not None else None
    scale = torch.empty(n, dtype=torch.float64, device=X.device)
    klog = torch.empty(n, dtype=torch.int32, device=X.device)
    o = _opts(outer_nb=outer_nb, omega_log2=omega_log2, fuse=fuse, overlap=overlap)
    rc = _lib.load().mstrsm_safe_gen(m, n, _p(U), _ld(U), _p(V), _ld(V), _p(s), _p(X), _ld(X),
                                     _p(cl), _p(scale), _p(klog), ctypes.byref(o), _stream())
    _lib.check("mstrsm_safe_gen", rc)
    return X, scale, klog


def gen_triang_eig(T, S, *, outer_nb=0, omega_log2=0, fuse=True):
    """GeneralizedTriangEig (appendix, Alg 10): returns (eigvals, Z, scale_log2)
    with T Z[:, j] = eigvals[j] S Z[:, j], eigvals[j] = T[j, j] / S[j, j],
    Z upper triangular, Z[j, j] = 2^-scale_log2[j]."""
    T = _mat(T, "T")
    S = _mat(S, "S")
    m = T.shape[0]
    if T.shape != (m, m) or S.shape != (m, m):
        raise ValueError("T and S must be square and of one size")
    Z = torch.empty_strided((m, m), (1, max(1, m)), dtype=torch.complex128, device=T.device)
    ev = torch.empty(m, dtype=torch.complex128, device=T.device)
    klog = torch.empty(m, dtype=torch.int32, device=T.device)
    o = _opts(outer_nb=outer_nb, omega_log2=omega_log2, fuse=fuse)
    rc = _lib.load().mst_gen_triang_eig(m, _p(T), _ld(T), _p(S), _ld(S), _p(Z), max(1, m), _p(ev),
                                        _p(klog), ctypes.byref(o), _stream())
    _lib.check("mst_gen_triang_eig", rc)
    return ev, Z, klog


def eig_schur(T, Q, *, nb=0, outer_nb=0, omega_log2=0):
    """Eig (Alg 6) after the Schur step A = Q T Q^H: returns (eigvals, X,
    scale_log2) with A X = X diag(eigvals), columns of X of unit 2-norm."""
    T = _mat(T, "T")
    Q = _mat(Q, "Q")
    m = T.shape[0]
    if T.shape != (m, m) or Q.shape != (m, m):
        raise ValueError("T and Q must be square and of one size")
    X = torch.empty_strided((m, m), (1, max(1, m)), dtype=torch.complex128, device=T.device)
    ev = torch.empty(m, dtype=torch.complex128, device=T.device)
    klog = torch.empty(m, dtype=torch.int32, device=T.device)
    o = _opts(nb=nb, outer_nb=outer_nb, omega_log2=omega_log2)
    rc = _lib.load().mst_eig_schur(m, _p(T), _ld(T), _p(Q), _ld(Q), _p(X), max(1, m), _p(ev), _p(klog),
                                   ctypes.byref(o), _stream())
    _lib.check("mst_eig_schur", rc)
    return ev, X, klog


def gen_eig_schur(T, S, P, *, outer_nb=0, omega_log2=0):
    """GeneralizedEig (appendix, Alg 10) after A = Q T P^H, B = Q S P^H:
    returns (eigvals, X, scale_log2) with A X = B X diag(eigvals), unit columns."""
    T = _mat(T, "T")
    S = _mat(S, "S")
    P = _mat(P, "P")
    m = T.shape[0]
    if T.shape != (m, m) or S.shape != (m, m) or P.shape != (m, m):
        raise ValueError("T, S and P must be square and of one size")
    X = torch.empty_strided((m, m), (1, max(1, m)), dtype=torch.complex128, device=T.device)
    ev = torch.empty(m, dtype=torch.complex128, device=T.device)
    klog = torch.empty(m, dtype=torch.int32, device=T.device)
    o = _opts(outer_nb=outer_nb, omega_log2=omega_log2)
    rc = _lib.load().mst_gen_eig_schur(m, _p(T), _ld(T), _p(S), _ld(S), _p(P), _ld(P), _p(X), max(1, m),
                                       _p(ev), _p(klog), ctypes.byref(o), _stream())
    _lib.check("mst_gen_eig_schur", rc)
    return ev, X, klog


def eig(A, *, nb=0, outer_nb=0):
    """Eigenpairs of a general square A (Alg 6): the Schur decomposition
    A = Q T Q^H on the host (LAPACK through SciPy), then TriangEig, the
    back-transformation X = Q Z and unit columns on the GPU. Returns
    (eigvals, X) as device tensors."""
    import numpy as np
    import scipy.linalg as sla
    dev = A.device if isinstance(A, torch.Tensor) and A.is_cuda else torch.device("cuda")
    An = A.detach().cpu().numpy() if isinstance(A, torch.Tensor) else np.asarray(A)
    T, Q = sla.schur(An.astype(np.complex128), output="complex")
    ev, X, _ = eig_schur(torch.from_numpy(T).to(dev), torch.from_numpy(Q).to(dev), nb=nb,
                         outer_nb=outer_nb)
    return ev, X


def gen_eig(A, B, *, outer_nb=0):
    """Eigenpairs of the pencil A x = lambda B x (appendix, Alg 10): the QZ
    decomposition A = Q T P^H, B = Q S P^H on the host (LAPACK through SciPy),
    then GeneralizedTriangEig, X = P Z and unit columns on the GPU.
    Infinite eigenvalues (S(j,j) = 0) are not supported."""
    import numpy as np
    import scipy.linalg as sla
    dev = A.device if isinstance(A, torch.Tensor) and A.is_cuda else torch.device("cuda")
    An = A.detach().cpu().numpy() if isinstance(A, torch.Tensor) else np.asarray(A)
    Bn = B.detach().cpu().numpy() if isinstance(B, torch.Tensor) else np.asarray(B)
    T, S, _, P = sla.qz(An.astype(np.complex128), Bn.astype(np.complex128), output="complex")
    ev, X, _ = gen_eig_schur(torch.from_numpy(T).to(dev), torch.from_numpy(S).to(dev),
                             torch.from_numpy(P).to(dev), outer_nb=outer_nb)
    return ev, X


def lanczos_restarted_sigma_min(U, z, V0, *, kdim=20, keep=6, max_restarts=30, tol=1e-10, nb=0,
                                outer_nb=0):
    """Thick-restart Lanczos estimate of sigma_min(U - z_j I) for every shift
    (Alg 7 with restarts and a per-shift tolerance). V0 (m x N start vectors)
    is not modified. Returns (sigma, resid, steps, converged). Synchronises
    the current stream once per restart cycle."""
    U = _mat(U, "U")
    V = _mat(V0, "V0")
    m, N = V.shape
    if U.shape != (m, m):
        raise ValueError("U must be %d x %d" % (m, m))
    zz = _vec(z, N, "z")
    sigma = torch.empty(N, dtype=torch.float64, device=V.device)
    resid = torch.empty(N, dtype=torch.float64, device=V.device)
    steps = torch.empty(N, dtype=torch.int32, device=V.device)
    conv = torch.empty(N, dtype=torch.int32, device=V.device)
    o = _opts(nb=nb, outer_nb=outer_nb)
    rc = _lib.load().mst_lanczos_restart_sigma_min(m, N, _p(U), _ld(U), _p(zz), _p(V), _ld(V), int(kdim),
                                                   int(keep), int(max_restarts), float(tol), _p(sigma),
                                                   _p(resid), _p(steps), _p(conv), ctypes.byref(o), _stream())
    _lib.check("mst_lanczos_restart_sigma_min", rc)
    return sigma, resid, steps, conv


def lanczos_sigma_min(U, z, V0, iters=15, *, nb=0, outer_nb=0):
    """Inverse-Lanczos estimate of sigma_min(U - z_j I) for every shift
    (Alg 7, second stage). V0 (m x N start vectors) is not modified.
    Returns (sigma, alpha, beta, steps); alpha/beta are (N, iters)."""
    U = _mat(U, "U")
    V0 = _mat(V0, "V0")
    m, N = V0.shape
    V = _fcopy(V0)
    zz = _vec(z, N, "z")
    sigma = torch.empty(N, dtype=torch.float64, device=V.device)
    alpha = torch.empty((N, iters), dtype=torch.float64, device=V.device)
    beta = torch.empty((N, iters), dtype=torch.float64, device=V.device)
    steps = torch.empty(N, dtype=torch.int32, device=V.device)
    o = _opts(nb=nb, outer_nb=outer_nb)
    rc = _lib.load().mst_lanczos_sigma_min(m, N, _p(U), _ld(U), _p(zz), _p(V), _ld(V), int(iters),
                                           _p(sigma), _p(alpha), _p(beta), _p(steps),
                                           ctypes.byref(o), _stream())
    _lib.check("mst_lanczos_sigma_min", rc)
    return sigma, alpha, beta, steps


class MultiShiftSolve(torch.autograd.Function):
    """X = solve(U, shifts, B) with (U - shifts_j I) x_j = b_j, differentiable
    in U (upper triangle), shifts and B. Backward: Y = adjoint solve of dL/dX,
    gB = Y, gU = -triu(Y X^H), gshift_j = x_j^H y_j (gradient convention
    dL/dRe z + i dL/dIm z, as torch uses for complex tensors)."""

    @staticmethod
    def forward(ctx, U, shifts, B, nb, outer_nb, precision, max_sweeps, recompute):
        X = _fcopy(B)
        mstrsm(U, shifts, X, nb=nb, outer_nb=outer_nb, precision=precision, max_sweeps=max_sweeps)
        ctx.nb, ctx.outer_nb = nb, outer_nb
        ctx.precision, ctx.max_sweeps = precision, max_sweeps
        ctx.recompute = int(recompute)
        if ctx.recompute > 0:
            # X is not kept: the backward pass solves again, recompute columns at a time
            ctx.save_for_backward(U, shifts, B)
        else:
            ctx.save_for_backward(U, shifts, X)
        return X

    @staticmethod
    def backward(ctx, gX):
        if ctx.recompute <= 0:
            U, shifts, X = ctx.saved_tensors
            Y = _fcopy(gX)
            mstrsm_adjoint(U, shifts, Y, nb=ctx.nb, outer_nb=ctx.outer_nb)
            gU = grad_u(Y, X) if ctx.needs_input_grad[0] else None
            gs = grad_shift(X, Y) if ctx.needs_input_grad[1] else None
            gB = Y if ctx.needs_input_grad[2] else None
            return gU, gs, gB, None, None, None, None, None
        U, shifts, B = ctx.saved_tensors
        n = B.shape[1]
        gU = None
        gs = torch.empty(n, dtype=torch.complex128, device=B.device) if ctx.needs_input_grad[1] else None
        gB = torch.empty_strided(B.shape, (1, max(1, B.shape[0])), dtype=torch.complex128,
                                 device=B.device) if ctx.needs_input_grad[2] else None
        for c0 in range(0, n, ctx.recompute):
            c1 = min(n, c0 + ctx.recompute)
            sc = shifts[c0:c1].contiguous()
            Xc = _fcopy(B[:, c0:c1])
            mstrsm(U, sc, Xc, nb=ctx.nb, outer_nb=ctx.outer_nb, precision=ctx.precision,
                   max_sweeps=ctx.max_sweeps)
            Yc = _fcopy(gX[:, c0:c1])
            mstrsm_adjoint(U, sc, Yc, nb=ctx.nb, outer_nb=ctx.outer_nb)
            if ctx.needs_input_grad[0]:
                g = grad_u(Yc, Xc)
                gU = g if gU is None else gU.add_(g)
            if gs is not None:
                gs[c0:c1] = grad_shift(Xc, Yc)
            if gB is not None:
                gB[:, c0:c1] = Yc
        return gU, gs, gB, None, None, None, None, None


def solve(U, shifts, B, *, nb=0, outer_nb=0, precision=0, max_sweeps=2, recompute=0):
    """Differentiable multi-shift solve (see MultiShiftSolve). recompute > 0:
    X is not stored for the backward pass; it is solved again there, that many
    columns at a time, so the backward pass holds two m x recompute blocks
    instead of the m x n solution."""
    return MultiShiftSolve.apply(U, shifts, B, nb, outer_nb, precision, max_sweeps, recompute)


class profile:
    """Context manager timing every kernel the library launches from this
    thread (HIP events around each launch). After exit, `.result` maps a
    kernel family to {"ms", "flops", "launches"}."""

    def __enter__(self):
        _lib.check("mst_profile_start", _lib.load().mst_profile_start())
        return self

    def __exit__(self, *exc):
        k = len(_lib.PROF_KINDS)
        ms = (ctypes.c_double * k)()
        fl = (ctypes.c_double * k)()
        ln = (ctypes.c_longlong * k)()
        rc = _lib.load().mst_profile_stop(ms, fl, ln)
        self.result = {name: {"ms": ms[i], "flops": fl[i], "launches": ln[i]}
                       for i, name in enumerate(_lib.PROF_KINDS)}
        if exc[0] is None:
            _lib.check("mst_profile_stop", rc)
        return False
