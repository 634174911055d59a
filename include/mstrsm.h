/*
 * mstrsm.h — blocked multi-shift triangular solves on AMD Instinct MI355X (gfx950).
 *
 * Implements the method of T. Moon and J. Poulson, "Accelerating eigenvector
 * and pseudospectra computation using blocked multi-shift triangular solves"
 * (arXiv 1607.01477): one upper-triangular U, many shifts lambda_j, solved
 * together so that the bulk of the work is a matrix-matrix product.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - All matrix and vector pointers are DEVICE pointers (hipMalloc'd or
 *    equivalent) unless a parameter says otherwise.
 *  - Complex numbers are complex128, stored interleaved {double re, im}
 *    (hipDoubleComplex / std::complex<double> / torch.complex128 layout).
 *  - Matrices are column-major with a leading dimension >= max(1, rows).
 *  - The strict lower triangle of U is never read.
 *  - `stream` is a hipStream_t (NULL = the default stream). Every call only
 *    enqueues work on it and returns; the caller synchronises the stream
 *    before reading outputs. No pointer is retained after a call returns.
 *  - Workspace is allocated stream-ordered on `stream` (hipMallocAsync) and
 *    released the same way before the call returns.
 *  - Arguments are validated on the host before anything is enqueued. On
 *    MST_EARG, mst_last_bad_arg() gives the 1-based position of the first
 *    offending argument. m == 0 or n == 0 returns MST_OK with nothing enqueued.
 *  - Calls from several host threads are allowed; the error state
 *    (mst_last_bad_arg, mst_last_error) is per thread.
 *  - With the environment variable MSTRSM_LOG set (to anything but "0") each
 *    call is reported on stderr with its sizes, and so is each argument or HIP
 *    error with the name of the call; nothing is synchronised for it.
 */
#ifndef MSTRSM_H
#define MSTRSM_H

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    MST_OK = 0,
    MST_EARG = -1,          /* invalid argument, see mst_last_bad_arg() */
    MST_EHIP = -2,          /* a HIP runtime call failed, see mst_last_error() */
    MST_ENOMEM = -3,        /* workspace allocation failed */
    MST_EUNSUPPORTED = -4   /* valid but unsupported combination of options */
} mst_status;

/* Options. A NULL mst_opts* means all defaults; a zero field means its default. */
typedef struct {
    int nb;            /* diagonal-block (and scaling-decision) size: 16, 32 or 64; default 16 */
    int outer_nb;      /* rows per deferred substitution step, a multiple of nb; 0 (default):
                          256, or 512 in plain FP64 back substitutions whose fused blocks
                          run 1 or 2 shifts per workgroup with at most one workgroup per
                          compute unit (few shifts; see fuse_blocks).
                          Equal to nb gives the paper's right-looking order (Alg 3 / Alg 5). */
    int precision;     /* 0: all FP64.
                          1: substitution GEMMs in FP32 on MFMA (FP32 accumulation),
                             diagonal blocks in FP64, then FP64 iterative refinement
                             on the residual B - (U X - X diag(lambda)). mstrsm only. */
    int max_sweeps;    /* most refinement sweeps for precision 1: 1..3; default 2 (see
                          refine_tol for stopping earlier) */
    int omega_log2;    /* overflow threshold Omega = 2^omega_log2 for the safe solve;
                          default 960 (leaves 2^64 of headroom below DBL_MAX). Smaller
                          values force rescaling at small sizes (testing). Range 8..1000. */
    int force_phase2;  /* safe solves: 0 (default) or 1. Alg 4 has a fast path (phase 1)
                          that only decides whether the checked back substitution (phase 2)
                          can be skipped. Here each diagonal block first runs a speculative
                          pass with the checks of phase 2 evaluated beside the substitution
                          and runs the checked steps only when a check fires; 1 skips the
                          speculative pass so that every block runs the checked steps.
                          Results are the same bit for bit (tested). */
    int fuse_blocks;   /* 0 (default): an outer block of at most 256 rows is solved by one
                          fused kernel (diagonal blocks plus the substitution between them),
                          with 16 shifts per workgroup, or with 4, 2 or 1 where 16-shift
                          workgroups would leave compute units idle (nb = 16, standard
                          problem, at most 8 x (compute units) shifts; the safe, variable-
                          length and mixed forms in the upper op N solve); 1, 2, 3 or 4
                          force 16, 4, 2 or 1 shifts per workgroup (2, 3 and 4 fall back to
                          16 where the narrow kernel is not available). The 16-shift kernel
                          applies the in-block updates in another summation order than the
                          narrow ones, so results agree to rounding; 4, 2 and 1 give the
                          same bits.
                          -1: one kernel per diagonal block plus separate GEMMs (same
                          arithmetic, kept for testing and for outer blocks larger than the
                          fused kernel takes). */
    int gemm_staged;   /* 0 (default): substitution GEMM without LDS staging (each wavefront
                          streams its operands from L1/L2); 1: LDS-staged GEMM. Same results
                          up to summation order; kept for testing. */
    int overlap;       /* 0 (default): everything on the caller's stream.
                          1: with fused outer blocks, the substitution of an outer block's
                          solution into the rows of the next outer block up runs ahead on
                          a second stream of the library, together with that block's
                          diagonal solve, while the GEMM for all rows further up runs on
                          the caller's stream (ordered by events; the call stays
                          asynchronous on the caller's stream). The rows above each
                          outer block then receive one product with K = outer_nb per
                          outer block, where the default path groups four outer blocks
                          into one deeper product: the same arithmetic in another
                          summation order, so results agree to rounding, not bit for
                          bit (safe exponents are the same). On MI355X it pays off
                          for nb = 32 only. */
    int gemm_split;    /* 0 (default): the substitution and residual products split the K
                          range of each 32 x 32 tile over 2 or 4 wavefronts of a workgroup
                          when the launch has too few tiles to fill the device (decided per
                          launch from its shape and the device's compute-unit count);
                          1, 2 or 4 forces that split for every such product. Partial sums
                          are added in a fixed order, so a given shape and split give the
                          same bits on every call; different splits agree to rounding.
                          Other values: MST_EINVAL. */
    double refine_tol; /* precision 1: before each sweep the relative residual of every
                          column, ||(U - l_j I) x_j - b_j||_inf / (||U - l_j I||_inf
                          ||x_j||_inf) (true modulus), is evaluated on the device; the
                          remaining sweeps are skipped once the largest is <= refine_tol,
                          and when a sweep did not lower the largest one, that sweep is
                          undone and refinement stops. 0 = default 1e-14; negative: never
                          stop early (but still undo a sweep that raised the residual). */
    double* refine_report; /* precision 1, nullable device pointer to max_sweeps + 1
                          doubles: entry t receives the largest relative residual after t
                          sweeps (t = 0: the FP32-GEMM solve), -1 where not evaluated
                          (after a stop). When given, the residual after the last sweep
                          is evaluated too (one more FP64 residual product), so a last
                          sweep that raised it is also undone. */
} mst_opts;

/*
 * mstrsm — plain multi-shift solve, problem (2) of Sec. 2 with Alg 3:
 *     (U - shifts[j] I) X(:,j) = B(:,j),   j = 0..n-1.
 *   m, n      rows of U / number of shifts (= columns of B)
 *   U, ldu    m x m upper triangular, read only
 *   shifts    n complex, read only
 *   B, ldb    m x n; on entry the right-hand sides, on exit X
 *   opt       nullable
 * Like xTRSM it does not detect singular or overflowing systems: a zero or
 * subnormal pivot gives Inf/NaN in X. With opt->precision = 1 the substitution
 * GEMMs run in FP32 and FP64 iterative refinement on the residual brings the
 * result to FP64 accuracy (refine_tol, max_sweeps, refine_report). Each right-
 * hand side (and each residual) is scaled by an exact power of two before it
 * is rounded to FP32, so B of any magnitude is safe; U's entries must lie in
 * FP32's range (|Re|, |Im| < 2^128; smaller entries than 2^-126 lose digits in
 * the FP32 copy, which refinement makes up for). The refinement converges when
 * the FP32 solve is accurate to better than one digit, roughly when
 * cond(U - l_j I) < 10^6; otherwise it stops as described for refine_tol, and
 * refine_report shows the residual reached.
 */
mst_status mstrsm(int m, int n, const void* U, int ldu, const void* shifts,
                  void* B, int ldb, const mst_opts* opt, void* stream);

/*
 * mstrsm_safe — safe multi-shift solve, problem (6) of Sec. 3 with Alg 5:
 *     (U - shifts[j] I) X(:,j) = s_j B(:,j),  s_j = 2^-k_j in [0, 1],
 * with power-of-two scale factors chosen so that no intermediate quantity
 * reaches Omega, and exactly zero pivots replaced by delta = 2^-52 max|U|_1
 * (|z|_1 = |Re z| + |Im z|; delta = 2^-1022 when U = 0). Finite input gives
 * finite X. Scaling decisions are taken per diagonal block of nb rows, so
 * they depend on nb (any nb gives a valid answer).
 *   col_len   nullable, device, n int32: column j uses rows [0, col_len[j]) only;
 *             the rows below are neither read nor written and act as zero
 *             right-hand-side entries (the triangular-eigenvector short-cut,
 *             Sec. 4). Values are clamped to [0, m].
 *   scale     device, n doubles: s_j (0 when k_j > 1074)
 *   scale_log2 nullable, device, n int32: k_j (exact)
 */
mst_status mstrsm_safe(int m, int n, const void* U, int ldu, const void* shifts,
                       void* B, int ldb, const int* col_len, double* scale, int* scale_log2,
                       const mst_opts* opt, void* stream);

/*
 * mstrsm_safe_noalloc — mstrsm_safe for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc). Same arguments, kernels and results as mstrsm_safe
 * (bit for bit), but the workspace comes from a static device array of the
 * library (MST_SCRATCH_LIMIT bytes on each device, held until the process
 * ends) instead of stream-ordered allocations: the call makes no hipMalloc,
 * hipMallocAsync or hipFree. The caller still provides U, shifts, B, col_len,
 * scale and scale_log2.
 *   Workspace needed, each piece rounded up to 256 bytes: n doubles, n int32,
 *   ceil(m/nb) * n int32, three times m doubles, ceil(m/nb) doubles and one
 *   double (about 4.2 MiB at m = n = 4096, nb = 16). A problem that needs more
 *   than MST_SCRATCH_LIMIT returns MST_ENOMEM before anything is enqueued,
 *   with the sizes in mst_last_error().
 *   opt->overlap = 1 (a second stream) gives MST_EUNSUPPORTED.
 * All calls on one device share that device's array: calls that overlap in
 * time on one device (several streams or host threads) race and give wrong
 * results; serialise them. No part of the array needs to start at zero (each
 * call writes every entry before reading it).
 */
#define MST_SCRATCH_LIMIT (16u << 20)
mst_status mstrsm_safe_noalloc(int m, int n, const void* U, int ldu, const void* shifts,
                               void* B, int ldb, const int* col_len, double* scale,
                               int* scale_log2, const mst_opts* opt, void* stream);

/*
 * mstrsm_adjoint — conjugate-transposed multi-shift solve (the lower-triangular
 * forward-substitution variant noted in the footnote to Sec. 2):
 *     (U - shifts[j] I)^H Y(:,j) = G(:,j).
 *   G, ldg    m x n; on entry G, on exit Y.
 * Plain FP64 (no scaling); singular systems give Inf/NaN like mstrsm.
 */
mst_status mstrsm_adjoint(int m, int n, const void* U, int ldu, const void* shifts,
                          void* G, int ldg, const mst_opts* opt, void* stream);

/*
 * mstrsm_op — the lower-triangular and right-side variants the footnote to
 * Sec. 2 mentions, and the transposed ones:
 *   side 'L':  op(A - shifts[j] I) X(:,j) = B(:,j)
 *   side 'R':  X(:,j)^T op(A - shifts[j] I) = B(:,j)^T   (the row vector x_j is
 *              stored as the column X(:,j); op 'N' or 'T' only)
 * with A upper ('U') or lower ('L') triangular and op 'N' (identity), 'T'
 * (transpose) or 'C' (conjugate transpose, so the shift enters conjugated).
 * When op(A) is upper triangular the solve is back substitution (Alg 3),
 * when lower forward substitution (blocks top to bottom); the triangle of A
 * that the variant does not use is never read. (U, 'N') is mstrsm and honours
 * opt->precision; every other variant is FP64 only (precision 1 gives
 * MST_EUNSUPPORTED). Plain solves: no scaling, like mstrsm.
 *   side, uplo, op   the characters above (as int)
 *   A, lda           m x m triangular, read only
 *   B, ldb           m x n; on entry the right-hand sides, on exit X
 */
mst_status mstrsm_op(int side, int uplo, int op, int m, int n, const void* A, int lda,
                     const void* shifts, void* B, int ldb, const mst_opts* opt, void* stream);

/*
 * mstrsm_real — real-arithmetic multi-shift solve (named as future work in the
 * paper's conclusion, Sec. 8; here in its plainest form): U, the shifts and B
 * real (float64),
 *     (U - shifts[j] I) X(:,j) = B(:,j),
 * Alg 3 with real operands: fused blocks of up to 256 rows (64-row diagonal
 * blocks and the updates inside the block in one kernel), the substitution
 * between blocks on the FP64 matrix cores. Plain: no scaling, like mstrsm.
 *   U, ldu     m x m upper triangular float64, read only (strict lower triangle not read)
 *   shifts     n float64
 *   B, ldb     m x n float64; on entry B, on exit X
 *   opt        nullable; outer_nb (a multiple of 64, default 256) is used, nb is not;
 *              precision must be 0 (else MST_EUNSUPPORTED)
 * Errors: MST_EARG for m < 0, n < 0, a leading dimension below max(1, m), a
 * null pointer with a non-empty operand, or outer_nb not a multiple of 64
 * (mst_last_bad_arg names the argument); HIP errors as MST_EHIP.
 */
mst_status mstrsm_real(int m, int n, const double* U, int ldu, const double* shifts, double* B,
                       int ldb, const mst_opts* opt, void* stream);

/*
 * mstrsm_real_op — the variants of mstrsm_op (footnote to Sec. 2) in real
 * arithmetic: side 'L': op(A - shifts[j] I) X(:,j) = B(:,j); side 'R':
 * X(:,j)^T op(A - shifts[j] I) = B(:,j)^T; A upper ('U') or lower ('L'); op 'N',
 * 'T' or 'C' ('C' = 'T' for real data). (U, 'N') on the left is mstrsm_real.
 * Every other variant is reduced to the upper solve: a lower A transposed is
 * upper, and a forward substitution is a back substitution in reversed order,
 * (J E J)(J x) = J b with J the row reversal. The library forms that
 * upper-triangular copy of A (m x m doubles of stream-ordered workspace; only
 * A's own triangle is read) and, for the forward cases, reverses the rows of
 * B before and after the solve.
 *   side, uplo, op   the characters above (as int)
 *   A, lda           m x m triangular float64, read only
 *   shifts           n float64
 *   B, ldb           m x n float64; on entry B, on exit X
 *   opt              nullable; outer_nb (a multiple of 64, default 256); precision must be 0
 * Errors as mstrsm_op (MST_EARG names the argument; MST_EUNSUPPORTED for
 * precision 1; MST_ENOMEM when the copy of A cannot be allocated).
 */
mst_status mstrsm_real_op(int side, int uplo, int op, int m, int n, const double* A, int lda,
                          const double* shifts, double* B, int ldb, const mst_opts* opt, void* stream);

/*
 * Gradient pieces of a real loss L through X = solve(U, shifts, B), given
 * Y = adjoint solve of dL/dX (gradient convention dL/dRe z + i dL/dIm z).
 * The gradient of B is Y itself.
 *
 * mst_grad_u:     gU = -triu(Y X^H), m x m; the strict lower triangle is set to 0.
 *                 Y and X are m x n.
 * mst_grad_shift: gshift[j] = sum_i conj(X(i,j)) Y(i,j), n complex.
 */
mst_status mst_grad_u(int m, int n, const void* Y, int ldy, const void* X, int ldx,
                      void* gU, int ldgu, void* stream);
mst_status mst_grad_shift(int m, int n, const void* X, int ldx, const void* Y, int ldy,
                          void* gshift, void* stream);

/*
 * mst_residual — R = B0 - (U X - X diag(shifts)), the FP64 residual of the
 * multi-shift system (used by the mixed-precision refinement).
 * R may not alias X; it may alias B0 (then ldr must equal ldb0).
 */
mst_status mst_residual(int m, int n, const void* U, int ldu, const void* shifts,
                        const void* X, int ldx, const void* B0, int ldb0,
                        void* R, int ldr, void* stream);

/*
 * mst_triang_eig — TriangEig, Alg 6 (Sec. 4): eigenvectors of an upper
 * triangular T through one safe multi-shift solve with shifts diag(T):
 *   Z(:,j) = [z; s_j; 0] with (T(0:j,0:j) - T(j,j) I) z = -s_j T(0:j, j),
 * so that T Z(:,j) = T(j,j) Z(:,j) and Z(j,j) = s_j = 2^-k_j.
 *   T, ldt        m x m upper triangular, read only
 *   Z, ldz        m x m output (the strict lower triangle is set to 0)
 *   eigvals       m complex output (diag(T))
 *   scale_log2    nullable, m int32 output (k_j)
 */
mst_status mst_triang_eig(int m, const void* T, int ldt, void* Z, int ldz, void* eigvals,
                          int* scale_log2, const mst_opts* opt, void* stream);

/*
 * mstrsm_gen — generalized multi-shift solve, appendix (Alg 8):
 *     (U - shifts[j] V) X(:,j) = B(:,j),   j = 0..n-1,
 * with U and V upper triangular (e.g. the triangular pair of a generalized
 * Schur form). The diagonal blocks are solved with U' = U - shifts[j] V
 * formed per shift; the rows above receive U X and V (shifts * X) as two
 * matrix products.
 *   V, ldv    m x m upper triangular, read only (strict lower triangle not read)
 *   other arguments as for mstrsm
 * Supported: nb = 16 (the default), precision 0; otherwise MST_EUNSUPPORTED.
 * Singular systems give Inf/NaN like mstrsm.
 */
mst_status mstrsm_gen(int m, int n, const void* U, int ldu, const void* V, int ldv,
                      const void* shifts, void* B, int ldb, const mst_opts* opt, void* stream);

/*
 * mstrsm_safe_gen — safe generalized multi-shift solve, appendix (Alg 9):
 *     (U - shifts[j] V) X(:,j) = s_j B(:,j),  s_j = 2^-k_j,
 * as mstrsm_safe, with: the checked back substitution (Alg 4) run on each
 * shifted diagonal block U' = U - shifts[j] V (its pivots, and its column norms
 * above the diagonal inside the block, per shift); the column growth bound
 * adding sum_k (||U(I0,k)||_inf + |shifts[j]|_1 ||V(I0,k)||_inf) ||X(I1,j)||_inf
 * over the columns k of the block; exactly zero pivots replaced by
 * delta = 2^-52 max(max|U|_1, max|V|_1).
 *   arguments as for mstrsm_safe, plus V, ldv as for mstrsm_gen
 * Supported: nb = 16 (the default); otherwise MST_EUNSUPPORTED.
 */
mst_status mstrsm_safe_gen(int m, int n, const void* U, int ldu, const void* V, int ldv,
                           const void* shifts, void* B, int ldb, const int* col_len,
                           double* scale, int* scale_log2, const mst_opts* opt, void* stream);

/*
 * mst_gen_triang_eig — GeneralizedTriangEig, appendix (Alg 10): eigenvectors
 * of the upper triangular pencil (T, S) through one safe generalized solve:
 * eigvals[j] = T(j,j) / S(j,j); Z(:,j) = [z; s_j; 0] with
 *   (T - eigvals[j] S)(0:j,0:j) z = -s_j (T - eigvals[j] S)(0:j, j),
 * so that T Z(:,j) = eigvals[j] S Z(:,j) and Z(j,j) = s_j = 2^-k_j.
 *   T, ldt; S, lds   m x m upper triangular, read only; S(j,j) must be nonzero
 *                    (finite eigenvalues), otherwise the column is Inf/NaN
 *   Z, ldz           m x m output (the strict lower triangle is set to 0)
 *   eigvals          m complex output
 *   scale_log2       nullable, m int32 output (k_j)
 * Supported: nb = 16 (the default); otherwise MST_EUNSUPPORTED.
 */
mst_status mst_gen_triang_eig(int m, const void* T, int ldt, const void* S, int lds, void* Z,
                              int ldz, void* eigvals, int* scale_log2, const mst_opts* opt,
                              void* stream);

/*
 * mst_eig_schur — the rest of Eig, Alg 6 (Sec. 4), after the Schur
 * decomposition A = Q T Q^H (computed by the caller, e.g. LAPACK xGEES on the
 * host): eigenvalues diag(T), triangular eigenvectors Z = TriangEig(T), the
 * back-transformation X = Q Z as a triangular product on the matrix cores,
 * and every column of X scaled to unit 2-norm, so that A X = X diag(eigvals).
 *   T, ldt        m x m upper triangular Schur factor, read only
 *   Q, ldq        m x m unitary Schur vectors, read only
 *   X, ldx        m x m output (may not alias T or Q)
 *   eigvals       m complex output
 *   scale_log2    nullable, m int32 output: k_j of TriangEig (Z(j,j) = 2^-k_j)
 */
mst_status mst_eig_schur(int m, const void* T, int ldt, const void* Q, int ldq, void* X, int ldx,
                         void* eigvals, int* scale_log2, const mst_opts* opt, void* stream);

/*
 * mst_gen_eig_schur — the rest of GeneralizedEig, appendix (Alg 10), after the
 * generalized Schur decomposition A = Q T P^H, B = Q S P^H (the caller's, e.g.
 * LAPACK xGGES): eigenvalues T(j,j)/S(j,j), Z = GeneralizedTriangEig(T, S),
 * X = P Z on the matrix cores, columns scaled to unit 2-norm, so that
 * A X = B X diag(eigvals). S(j,j) must be nonzero.
 *   T, S          m x m upper triangular, read only; P, ldp  m x m, read only
 *   X, ldx        m x m output (may not alias the inputs)
 * Supported: nb = 16 (the default); otherwise MST_EUNSUPPORTED.
 */
mst_status mst_gen_eig_schur(int m, const void* T, int ldt, const void* S, int lds, const void* P, int ldp,
                             void* X, int ldx, void* eigvals, int* scale_log2, const mst_opts* opt,
                             void* stream);

/*
 * mst_lanczos_sigma_min — second stage of the Van Loan/Lui method (Alg 7,
 * Sec. 5): for every shift z_j, `iters` steps of plain Lanczos (no
 * reorthogonalisation) on (U - z_j I)^{-H} (U - z_j I)^{-1}, each product
 * being one mstrsm and one mstrsm_adjoint over all shifts at once;
 * sigma[j] = theta_max^{-1/2} with theta_max the largest eigenvalue of the
 * Lanczos tridiagonal (computed on the device by bisection).
 *   V, ldv     m x N start vectors (normalised here); overwritten (workspace)
 *   iters      1..64
 *   sigma      device, N doubles: estimate of sigma_min(U - z_j I)
 *   alpha,beta nullable, device, iters x N doubles each (column j at offset j*iters)
 *   steps      nullable, device, N int32: steps taken (< iters only if beta hit 0)
 */
mst_status mst_lanczos_sigma_min(int m, int N, const void* U, int ldu, const void* z,
                                 void* V, int ldv, int iters, double* sigma,
                                 double* alpha, double* beta, int* steps,
                                 const mst_opts* opt, void* stream);

/*
 * mst_lanczos_restart_sigma_min — the second stage of Alg 7 (Sec. 5) with a
 * restarted Krylov method and a per-shift tolerance (the paper's runs used
 * implicitly restarted Arnoldi; on the Hermitian positive definite operator
 * A_j = (U - z_j I)^{-H} (U - z_j I)^{-1} that is thick-restart Lanczos).
 * For every shift: cycles of Lanczos steps with full reorthogonalisation
 * (classical Gram-Schmidt, two passes) build a basis of kdim vectors, each
 * step one mstrsm and one mstrsm_adjoint over the shifts still running;
 * Rayleigh-Ritz on the kdim x kdim projection gives the largest Ritz value
 * theta and the residual norm of its Ritz vector, |beta S(kdim-1, 0)|. A shift
 * stops when that is <= tol * theta, or after max_restarts restarts;
 * otherwise the next cycle keeps its keep largest Ritz vectors and the last
 * Lanczos vector (thick restart). sigma[j] = theta^{-1/2}.
 *   V, ldv        m x N start vectors, read only (normalised copies are used)
 *   kdim          basis vectors per cycle, 2..32
 *   keep          Ritz vectors kept at a restart, 1..min(kdim - 1, 16)
 *   max_restarts  0..100000 (0: one cycle of kdim plain Lanczos steps)
 *   tol           >= 0: relative residual at which a shift stops
 *   sigma         device, N doubles: the estimate of sigma_min(U - z_j I)
 *   resid         nullable, device, N doubles: |beta S(kdim-1, 0)| / theta
 *   steps         nullable, device, N int32: Lanczos steps taken
 *   converged     nullable, device, N int32: 1 when resid <= tol
 * Unlike the other entry points this call synchronises `stream` once per
 * restart cycle (it reads the number of shifts still running, which sizes the
 * next cycle's solves), so it cannot be captured into a graph. Workspace:
 * (kdim + 1) m N + m N complex128 plus O(N kdim^2) doubles.
 */
mst_status mst_lanczos_restart_sigma_min(int m, int N, const void* U, int ldu, const void* z,
                                         const void* V, int ldv, int kdim, int keep,
                                         int max_restarts, double tol, double* sigma,
                                         double* resid, int* steps, int* converged,
                                         const mst_opts* opt, void* stream);

/*
 * Kernel timing (diagnostics). Between mst_profile_start() and
 * mst_profile_stop(), every kernel launch made by this thread is bracketed by
 * a pair of HIP events on its stream and attributed to one family. stop()
 * waits for the recorded events and returns, per family, the summed kernel
 * time in milliseconds, the nominal real flops those launches performed
 * (8 per complex multiply-add) and the launch count. Arrays have
 * MST_PROF_KINDS entries (any may be NULL).
 */
enum {
    MST_PROF_GEMM_F64 = 0,   /* substitution GEMM, FP64 matrix cores */
    MST_PROF_GEMM_F32 = 1,   /* substitution GEMM, FP32 matrix cores */
    MST_PROF_DIAG = 2,       /* diagonal-block solves */
    MST_PROF_RESID = 3,      /* residual, gradient and back-transformation products */
    MST_PROF_AUX = 4,        /* norms, rescaling, conversions, Lanczos vectors */
    MST_PROF_KINDS = 5
};
mst_status mst_profile_start(void);
mst_status mst_profile_stop(double* ms, double* flops, long long* launches);

/* Human-readable name of a status code (static storage). */
const char* mst_status_string(mst_status s);
/* 1-based position of the first bad argument of this thread's last MST_EARG. */
int mst_last_bad_arg(void);
/* Text of this thread's last MST_EHIP / MST_ENOMEM / MST_EUNSUPPORTED failure (static
   storage per thread); every call of the library clears it on entry. */
const char* mst_last_error(void);
/* Library version, e.g. "0.1.0". */
const char* mst_version(void);

#ifdef __cplusplus
}
#endif

#endif /* MSTRSM_H */
