// Internal declarations of the mstrsm HIP library (gfx950). Not installed.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mst {

struct zd { double re, im; };   // complex128, interleaved
struct zf { float re, im; };    // complex64, interleaved

// Safe-solve state kept on the device for one call.
struct SafeState {
    double* G;          // n: column growth bound G(j)
    int* kcur;          // n: current exponent k_j (s_j = 2^-k_j)
    int* kb;            // nblk x n: exponent of column j right after block q was solved
    const double* cn_in;      // m: max cabs1 of U above the diagonal inside the diagonal block
    const double* above_sum;  // nblk: sum over the block's columns of max cabs1 above the block
    const double* delta;      // 1: replacement for a zero pivot
    int omega_log2;
    int force_checked;        // 1: no speculative pass; every diagonal block runs the checked steps
    // pencil (U - lambda V): the same sums and replacement for V; the bound adds
    // cabs1(lambda_j) * above_sum_v and the zero-pivot replacement is max(delta, delta_v)
    const double* above_sum_v;
    const double* delta_v;
};

// ---------------------------------------------------------------- solve variants
// The triangular operator a solve substitutes with: E = op(A) for A upper or
// lower triangular (the variants of the footnote to Sec. 2). Bits:
//   1: forward substitution (E lower triangular; otherwise back substitution)
//   2: E(r, c) = A(c, r) (transposed storage access)
//   4: conjugated entries (and shifts)
enum SolveVariant : int {
    EV_UPPER_N = 0,   // (U - l I) x = b                     back substitution
    EV_LOWER_N = 1,   // (L - l I) x = b                     forward
    EV_LOWER_T = 2,   // (L - l I)^T x = b                   back
    EV_UPPER_T = 3,   // (U - l I)^T x = b                   forward
    EV_LOWER_C = 6,   // (L - l I)^H x = b                   back
    EV_UPPER_C = 7,   // (U - l I)^H x = b (the adjoint)     forward
};
constexpr bool ev_fwd(int ev) { return (ev & 1) != 0; }
constexpr bool ev_tr(int ev) { return (ev & 2) != 0; }
constexpr bool ev_cj(int ev) { return (ev & 4) != 0; }
// A is lower triangular exactly when the access is transposed for back
// substitution or direct for forward substitution
constexpr bool ev_lower_a(int ev) { return ev_tr(ev) != ev_fwd(ev); }

// ---------------------------------------------------------------- diagonal blocks
// Solves the nb-row diagonal block [i0, i0+bs) for all n shifts in place.
//   ev = EV_UPPER_N: (U(I1,I1) - lambda_j I) x = b        (back substitution, Alg 1)
//   ev = EV_UPPER_C: (U(I1,I1) - lambda_j I)^H y = g      (forward substitution)
//   other SolveVariant values: the lower and transposed variants (plain FP64 only)
// safe != nullptr: Alg 4 phase 2 with Alg 5's column bound and decisions, block index q.
// b32 != nullptr (mixed precision): the right-hand side is read from b32 (FP32),
// solved in FP64, and written both to B (FP64) and back to b32 (rounded).
// V != nullptr: the pencil U - lambda_j V (nb = 16, forward, FP64 only).
struct DiagArgs {
    int m, n, i0, bs, q;
    const zd* U; long ldu;
    const zd* V; long ldv;
    const zd* lam;
    zd* B; long ldb;
    zf* b32; long ldb32;
    const int* col_len;
    SafeState safe;
    int use_safe;
    const int* skip;   // mixed precision: nothing is done when *skip != 0 (nullable)
};
hipError_t launch_diag(int nb, int ev, const DiagArgs& a, hipStream_t s);

// Whole outer block [iS, iS+rows) (rows <= block_rows_for(...): 256, or 512 for
// the narrow kernel of a plain solve; iS a multiple of nb,
// first diagonal block index qa) for all n shifts: the diagonal blocks in
// order and the substitution between them, in one launch. V != nullptr: the
// pencil U - lambda_j V (nb = 16, forward, FP64 only).
struct BlockArgs {
    int m, n, nb, qa, iS, rows;
    const zd* U; long ldu;
    const zd* V; long ldv;
    const zd* lam;
    zd* B; long ldb;
    zf* b32; long ldb32;
    const int* col_len;
    SafeState safe;
    int use_safe;
    const int* skip;   // mixed precision: nothing is done when *skip != 0 (nullable)
    int width;         // shifts per workgroup: 16, 4, 2 or 1 (where available); 0 = chosen from n
};
// Rows an outer block may have in the fused kernel for n shifts at the given
// width (0 = automatic): 512 where the narrow kernel runs at most 2 shifts per
// workgroup, one workgroup per compute unit, in a plain FP64 solve (nb = 16),
// else 256.
int block_rows_for(int n, int nb, int width, bool plain);
bool block_fusable(int nb);   // nb handled by the fused kernel (16 or 32)
hipError_t launch_block(int ev, const BlockArgs& a, hipStream_t s);

// Compute units of the current device (read once per device; 256 if the
// query fails). Launch shapes that depend on it: the K split of the direct
// GEMM and the width of the fused outer-block kernel.
int device_cu_count();

// ---------------------------------------------------------------- tile order
// Workgroup -> output tile (tm, tn) of a TM x TN grid, shared by the GEMM
// kernels. The hardware deals workgroup w to XCD w % 8; when the tile count is
// a multiple of 8 each XCD gets one contiguous range of the order below, so
// the workgroups that run together on one XCD share operand panels in its L2.
// Within the order, row tiles go in groups of GROUP, column by column.
template <int GROUP = 8>
__device__ inline void tile_coords(int TM, int TN, int& tm, int& tn) {
    const int T = TM * TN;
    int w = blockIdx.x;
    if ((T & 7) == 0) w = (w & 7) * (T >> 3) + (w >> 3);   // one contiguous range per XCD
    const int per_group = GROUP * TN;
    const int gid = w / per_group;
    const int first = gid * GROUP;
    const int gsz = min(TM - first, GROUP);
    const int in = w - gid * per_group;
    tm = first + in % gsz;
    tn = in / gsz;
}

// ---------------------------------------------------------------- MFMA GEMM
// C(M x N) <- epilogue(acc), acc = A(M x K) * B(K x N), complex.
enum GemmOp : int {
    GOP_SUB = 0,      // C = 2^-dk_c * C - acc   (dk from the safe state, else 0)
    GOP_RESID = 1,    // C = B0 - acc + lam_c * Bop(row, c)   (A upper triangular, global indices)
    GOP_NEG_TRIU = 2, // C = -acc on and above the diagonal, 0 below
    GOP_GEN_SUB = 3,  // C = 2^-dk_c * C - A B + lam_c * (A2 B)   (pencil substitution)
    GOP_TRMM = 4,     // C = A B, B upper triangular (its strict lower triangle is not read)
};
struct GemmArgs {
    int M, N, K;
    const void* A; long lda; int a_ct;   // a_ct: 1 A(r,k) = conj(a[r*lda + k]); 2 a[r*lda + k];
                                         // 0 a[k*lda + r]
    const void* B; long ldb; int b_ct;   // b_ct: B(k,c) = conj(b[k*ldb + c]); else b[c*ldb + k]
    void* C; long ldc;
    int op;
    // GOP_RESID: A is U(0:M, 0:K) (square, upper triangular), Bop is X, B0/lam given
    const zd* B0; long ldb0; const zd* lam;
    // safe scaling (GOP_SUB): kb rows of the B operand belong to blocks (b_row0 + k)/nb,
    // scaled on load by 2^-(kb[q_cur] - kb[q(k)]); C scaled by 2^-(kb[q_cur] - kb[q_c])
    // (kb[-1] = 0, i.e. q_c < 0 means exponent 0).
    const int* kb; int n_kb; int q_cur; int q_c; int nb; int b_row0;
    // variable-length columns: column c uses rows < col_len[c] (global row of C row 0 = c_row0)
    const int* col_len; int c_row0;
    // substitution (GOP_SUB, plain operands): 1 = LDS-staged kernel, 0 = barrier-free kernel
    int staged;
    // GOP_GEN_SUB: second A operand (plain, same shape as A) and the shift of each column
    const void* A2; long lda2; const zd* glam;
    // FP32 substitution and FP64 residual (refinement): nothing is done when *skip != 0
    const int* skip;
    // GOP_SUB / GOP_RESID without staging: wavefronts per tile's K range (1, 2, 4),
    // 0 = chosen from the launch shape
    int split;
};
hipError_t launch_gemm_f64(const GemmArgs& g, hipStream_t s);
hipError_t launch_gemm_f32(const GemmArgs& g, hipStream_t s);

// ---------------------------------------------------------------- real arithmetic
// C(M x N) -= A(M x K) B(K x N), float64, column-major, A plain.
struct RealGemmArgs {
    int M, N, K;
    const double* A; long lda;
    const double* B; long ldb;
    double* C; long ldc;
};
hipError_t launch_gemm_real(const RealGemmArgs& g, hipStream_t s);
// Block [i0, i0 + bs) (bs <= 256) of the real solve (U - lambda_j I) x = b, all
// n shifts, in place in B: the 64-row diagonal blocks and the updates inside
// the block fused.
struct RealDiagArgs {
    int m, n, i0, bs;
    const double* U; long ldu;
    const double* lam;
    double* B; long ldb;
};
hipError_t launch_block_real(const RealDiagArgs& a, hipStream_t s);
// Upper-triangular copy Uh (m x m, leading dimension m; only the upper triangle
// is written) of a triangular A whose variant reduces to an upper solve:
//   REAL_T    Uh(i,j) = A(j,i)                  (A lower, transposed solve)
//   REAL_JJ   Uh(i,j) = A(m-1-i, m-1-j)         (A lower, forward solve)
//   REAL_JTJ  Uh(i,j) = A(m-1-j, m-1-i)         (A upper, transposed solve)
// Only A's own triangle is read.
enum RealCopyMode { REAL_T = 0, REAL_JJ = 1, REAL_JTJ = 2 };
hipError_t launch_real_upper_copy(int m, const double* A, long lda, int mode, double* Uh, hipStream_t s);
// Rows of B (m x n) in reverse order, in place.
hipError_t launch_reverse_rows(int m, int n, double* B, long ldb, hipStream_t s);

// ---------------------------------------------------------------- auxiliary kernels
hipError_t launch_norms(int m, const zd* U, long ldu, int nb, double* cn_in, double* above,
                        double* colmax, double* above_sum, double* delta, hipStream_t s);
hipError_t launch_colinit(int m, int n, const zd* B, long ldb, const int* col_len,
                          double* G, int* kcur, hipStream_t s);
hipError_t launch_finalize(int m, int n, int nb, zd* B, long ldb, const int* col_len,
                           const int* kcur, const int* kb, double* scale, int* klog,
                           hipStream_t s);
hipError_t launch_dot(int m, int n, const zd* X, long ldx, const zd* Y, long ldy, zd* out,
                      hipStream_t s);
hipError_t launch_to_f32(int rows, int cols, const zd* src, long lds, zf* dst, long ldd,
                         bool upper_only, hipStream_t s);
hipError_t launch_copy(int rows, int cols, const zd* src, long lds, zd* dst, long ldd,
                       hipStream_t s);
hipError_t launch_axpy_inplace(int rows, int cols, const zd* D, long ldd, zd* X, long ldx,
                               hipStream_t s);
hipError_t launch_triang_setup(int m, const zd* T, long ldt, zd* Z, long ldz, zd* eig,
                               int* col_len, hipStream_t s);
hipError_t launch_gen_triang_setup(int m, const zd* T, long ldt, const zd* S, long lds, zd* Z, long ldz,
                                   zd* eig, int* col_len, hipStream_t s);
hipError_t launch_triang_diag(int m, zd* Z, long ldz, const double* scale, hipStream_t s);
hipError_t launch_normalize_cols(int m, int n, zd* V, long ldv, hipStream_t s);
hipError_t launch_lanczos_step(int m, int n, int it, int iters, const zd* V, long ldv,
                               zd* W, long ldw, const zd* Vprev, long ldp,
                               double* alpha, double* beta, int* steps, hipStream_t s);
hipError_t launch_fill_int(int n, int v, int* p, hipStream_t s);

// ---------------------------------------------------------------- iterative refinement
// State of the refinement loop of the mixed-precision solve, kept on the device
// so that the stop test and the undo of a sweep run as kernels (the call stays
// asynchronous). stop: later sweeps do nothing; rb[t]: sweep t raised the
// residual and is undone; prev: residual of the last iterate tested.
constexpr int kMaxSweeps = 3;
struct RefineCtl {
    int stop;
    int rb[kMaxSweeps + 1];
    double prev;
};
constexpr int kRowChunk = 128;   // columns per partial row sum
// rowoff[i] = sum_{k > i} |U(i,k)| (true modulus; fixed order: chunks of kRowChunk
// columns, then the chunks in order); udiag[i] = U(i,i). part: ceil(m/kRowChunk) * m doubles.
hipError_t launch_rowabs(int m, const zd* U, long ldu, double* part, double* rowoff, zd* udiag,
                         hipStream_t s);
// Per column j of R (m x n): e[j] = ilogb(max_i |R(i,j)|_1) (0 for a zero or non-finite
// column), so that 2^-e[j] R(:,j) has entries below 2 in each part; with X given also
//   rel[j] = max_i |R(i,j)| / (max_i (rowoff[i] + |udiag[i] - lam_j|) max_i |X(i,j)|)
// (true modulus; the absolute residual where X(:,j) = 0; +inf where R or X holds a
// non-finite value). Nothing is done when skip && *skip.
hipError_t launch_colstats(int m, int n, const zd* R, long ldr, const zd* X, long ldx,
                           const double* rowoff, const zd* udiag, const zd* lam, int* e, double* rel,
                           const int* skip, hipStream_t s);
// dst(r, c) = fp32(2^-e[c] src(r, c)), unless skip && *skip
hipError_t launch_to_f32_cols(int rows, int cols, const zd* src, long lds, const int* e, zf* dst,
                              long ldd, const int* skip, hipStream_t s);
// X(r, c) += sign 2^e[c] D(r, c); nothing is done when skip && *skip, or when
// cond && *cond != 1
hipError_t launch_axpy_cols(int rows, int cols, const zd* D, long ldd, const int* e, double sign,
                            zd* X, long ldx, const int* skip, const int* cond, hipStream_t s);
// dst = src, unless skip && *skip, or cond && *cond != 1
hipError_t launch_copy_cond(int rows, int cols, const zd* src, long lds, zd* dst, long ldd,
                            const int* skip, const int* cond, hipStream_t s);
// X(r, c) = 2^e[c] X(r, c)
hipError_t launch_scale_cols(int rows, int cols, zd* X, long ldx, const int* e, hipStream_t s);
// ctl: stop = 0, rb = 0, prev = +inf; report[0..nrep) = -1 (report nullable)
hipError_t launch_refine_init(RefineCtl* ctl, double* report, int nrep, hipStream_t s);
// After the residual of iterate t (t = 0: the FP32 solve; rel from launch_colstats):
// res = max_j rel[j]; report[t] = res; stop when res <= tol; when t > 0 and res is
// not below the previous iterate's, stop and set rb[t] (undo sweep t). Nothing is
// done once stop is set.
hipError_t launch_refine_ctl(int n, int t, const double* rel, double tol, RefineCtl* ctl,
                             double* report, hipStream_t s);
hipError_t launch_zero(long count, zd* p, hipStream_t s);
hipError_t launch_tridiag_max(int n, int iters, const double* alpha, const double* beta,
                              const int* steps, double* sigma, hipStream_t s);

// ---------------------------------------------------------------- thick-restart Lanczos
// Kernels of the restarted resolvent-norm driver (klanczos.hip). Q holds kdim + 1
// basis blocks of m x N (block l at Q + l * qs, leading dimension ldq); H the
// kdim x kdim projected matrix of each shift (row-major); idx the running shifts.
int trl_max_kdim();
int trl_max_keep();
hipError_t launch_trl_init(int m, int N, int kdim, const zd* V, long ldv, zd* Q, long ldq, double* H, int* idx,
                           int* steps, hipStream_t s);
hipError_t launch_trl_gather(int m, int nact, const int* idx, const zd* Qi, long ldq, zd* W, long ldw,
                             const zd* z, zd* zact, hipStream_t s);
hipError_t launch_trl_orth(int m, int nact, int i, int k0, int kdim, const int* idx, zd* W, long ldw, zd* Q,
                           long ldq, long qs, double* H, double* beta, int* steps, hipStream_t s);
hipError_t launch_trl_ritz(int nact, int kdim, int keep, double tol, int last, const int* idx, double* H,
                           const double* beta, double* Sk, double* sigma, double* resid, int* conv, int* go,
                           hipStream_t s);
hipError_t launch_trl_restart(int m, int nact, int kdim, int keep, const int* idx, const int* go, zd* Q,
                              long ldq, long qs, const double* Sk, hipStream_t s);
hipError_t launch_trl_compact(int nact, const int* idx, const int* go, int* idx_out, int* count,
                              hipStream_t s);

}  // namespace mst
