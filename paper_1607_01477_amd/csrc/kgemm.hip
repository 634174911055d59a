// Complex GEMM on the matrix cores of gfx950 for the substitution step of the
// blocked multi-shift solve (the xGEMM of Alg 3 / Alg 5 of Moon & Poulson,
// arXiv 1607.01477), and for the residual and gradient products around it.
//
// A complex product is four real MFMA products on the same operands:
//   Re C += Re A Re B - Im A Im B,  Im C += Re A Im B + Im A Re B,
// exactly the 8 real flops per complex multiply-add of the nominal count.
// FP64 uses v_mfma_f64_16x16x4_f64, FP32 v_mfma_f32_16x16x4_f32.
//
// Workgroup tile 64 x 64 complex, 4 wavefronts of 32 x 32; K is staged
// through LDS 16 complex at a time, double buffered, rows padded by one
// element so that the transposing stores do not collide in one bank. Each
// thread keeps its share of the next K-chunk in registers while the matrix
// cores work on the current one. Interior tiles take an unmasked path. For
// the substitution (C = C - A B) the accumulators start from C itself, loaded
// before the K loop, so the C read latency hides behind the first chunks.
// Operands are read straight from interleaved column-major storage,
// optionally conjugate-transposed; no realified copy is formed in HBM. Tiles
// are ordered in groups of 8 row tiles and dealt out so that each XCD (own L2)
// receives a contiguous range of tiles.
#include "common.h"

#include <type_traits>

namespace mst {
namespace {

constexpr int BM = 64, BN = 64, BK = 16, NT = 256, PAD = 1;

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

// Output lane layout of the 16x16x4 products (measured on gfx950): lane l,
// item v holds column l % 16 and row (l / 16) + 4 v for FP64, row
// 4 (l / 16) + v for FP32. Inputs: A(i, k) at lane i + 16 k, B(k, j) at
// lane j + 16 k for both.
template <typename T> struct Traits;
template <> struct Traits<double> {
    using C = zd;
    using V = v4d;
    static __device__ inline int out_row(int lq, int v) { return lq + 4 * v; }
    static __device__ inline V mfma(double a, double b, V c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
};
template <> struct Traits<float> {
    using C = zf;
    using V = v4f;
    static __device__ inline int out_row(int lq, int v) { return 4 * lq + v; }
    static __device__ inline V mfma(float a, float b, V c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
};

// Tile order of -triu(A B^H) on a square grid of TM x TM tiles: the first
// TM (TM + 1) / 2 workgroups take the tiles on and above the diagonal (row
// major, dealt out to the XCDs in equal contiguous ranges, since the
// hardware places workgroup w on XCD w % 8), the rest the tiles below it,
// which only write zeros.
__device__ inline void tri_coords(int TM, int& tm, int& tn) {
    const int T_up = TM * (TM + 1) / 2;
    int w = blockIdx.x;
    if (w < T_up) {
        if ((T_up & 7) == 0) w = (w & 7) * (T_up >> 3) + (w >> 3);
        int r = 0;
        while (w >= TM - r) {
            w -= TM - r;
            ++r;
        }
        tm = r;
        tn = r + w;
    } else {
        int z = w - T_up, r = 1;
        while (z >= r) {
            z -= r;
            ++r;
        }
        tm = r;
        tn = z;
    }
}

template <typename CT>
__device__ inline CT cconj(CT v) {
    v.im = -v.im;
    return v;
}

template <typename T, bool A_CT, bool B_CT, int OP, bool SAFE, bool VARLEN>
__global__ __launch_bounds__(NT, 2) void k_gemm(GemmArgs g) {
    using Tr = Traits<T>;
    using CT = typename Tr::C;
    using V = typename Tr::V;
    __shared__ CT As[2][BK][BM + PAD];
    __shared__ CT Bs[2][BK][BN + PAD];

    if ((sizeof(T) == 4 || OP == GOP_RESID) && g.skip && *g.skip) return;   // refinement stopped
    const int TM = (g.M + BM - 1) / BM, TN = (g.N + BN - 1) / BN;
    int tm, tn;
    tile_coords(TM, TN, tm, tn);
    const int r0 = tm * BM, c0 = tn * BN;
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int wr = wave >> 1, wc = wave & 1;
    const int lr = lane & 15, lq = lane >> 4;
    const CT* __restrict__ A = (const CT*)g.A;
    const CT* __restrict__ B = (const CT*)g.B;
    CT* __restrict__ C = (CT*)g.C;

    if (OP == GOP_NEG_TRIU && r0 > c0 + BN - 1) {
        for (int e = t; e < BM * BN; e += NT) {
            const int rr = r0 + (e % BM), cc = c0 + (e / BM);
            if (rr < g.M && cc < g.N) C[(long)cc * g.ldc + rr] = CT{0, 0};
        }
        return;
    }
    if (VARLEN) {
        // a tile whose columns all end above the B operand's rows has nothing to do
        bool act = false;
        for (int c = 0; c < BN; ++c) {
            const int cc = c0 + c;
            if (cc < g.N && g.col_len[cc] > g.b_row0) act = true;
        }
        if (!act) return;
    }
    const bool full_mn = (r0 + BM <= g.M) && (c0 + BN <= g.N);

    // ---- accumulators (start from C for the substitution)
    V accR[2][2], accI[2][2];
    int clim0 = g.M, clim1 = g.M;
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        const int col = c0 + wc * 32 + j * 16 + lr;
        int csh = 0, clim = g.M;
        if (OP == GOP_SUB && col < g.N) {
            if (VARLEN) clim = min(g.M, g.col_len[col] - g.c_row0);
            if (SAFE && g.kb != nullptr) {
                const int kc = g.kb[(long)g.q_cur * g.n_kb + col];
                const int kq = (g.q_c >= 0) ? g.kb[(long)g.q_c * g.n_kb + col] : 0;
                csh = kc - kq;
            }
        }
        if (j == 0) clim0 = clim; else clim1 = clim;
#pragma unroll
        for (int i = 0; i < 2; ++i) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                accR[i][j][v] = 0;
                accI[i][j][v] = 0;
            }
            if (OP == GOP_SUB) {
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int row = r0 + wr * 32 + i * 16 + Tr::out_row(lq, v);
                    if (col < g.N && row < clim) {
                        CT c = C[(long)col * g.ldc + row];
                        if (SAFE) {
                            c.re = ldexp(c.re, -csh);
                            c.im = ldexp(c.im, -csh);
                        }
                        accR[i][j][v] = c.re;
                        accI[i][j][v] = c.im;
                    }
                }
            }
        }
    }

    // K range (the residual's A is upper triangular: rows r0.. need k >= r0)
    int kbeg = 0;
    if (OP == GOP_RESID) kbeg = (r0 / BK) * BK;
    const int nchunk = (g.K - kbeg + BK - 1) / BK;

    // per-thread staging coordinates
    //   A, plain:   k = t/16, rows 4*(t%16)..+3      A, conj-T: row = t/4, k = 4*(t%4)..+3
    //   B, plain:   col = t/4, k = 4*(t%4)..+3       B, conj-T: k = t/16, cols 4*(t%16)..+3
    const int a_k = A_CT ? 4 * (t & 3) : (t >> 4);
    const int a_r = A_CT ? (t >> 2) : 4 * (t & 15);
    const int b_k = B_CT ? (t >> 4) : 4 * (t & 3);
    const int b_c = B_CT ? 4 * (t & 15) : (t >> 2);
    int b_lim = g.K;
    if (VARLEN && !B_CT && c0 + b_c < g.N) b_lim = min(b_lim, g.col_len[c0 + b_c] - g.b_row0);
    CT ra0, ra1, ra2, ra3, rb0, rb1, rb2, rb3;

#define MST_LOAD_A(E, R)                                                                   \
    {                                                                                      \
        const int gk = k0 + a_k + (A_CT ? E : 0), gr = r0 + a_r + (A_CT ? 0 : E);          \
        R = CT{0, 0};                                                                      \
        if (fast || (gk < g.K && gr < g.M && (OP != GOP_RESID || gr <= gk))) {             \
            if (A_CT) R = cconj(A[(long)gr * g.lda + gk]);                                 \
            else R = A[(long)gk * g.lda + gr];                                             \
        }                                                                                  \
    }
#define MST_LOAD_B(E, R)                                                                   \
    {                                                                                      \
        const int gk = k0 + b_k + (B_CT ? 0 : E), gc = c0 + b_c + (B_CT ? E : 0);          \
        R = CT{0, 0};                                                                      \
        if (B_CT) {                                                                        \
            if (fast || (gk < g.K && gc < g.N)) R = cconj(B[(long)gk * g.ldb + gc]);       \
        } else if (fast || (gk < b_lim && gc < g.N)) {                                     \
            R = B[(long)gc * g.ldb + gk];                                                  \
            if (SAFE) {                                                                    \
                R.re = ldexp(R.re, -b_dsh);                                                \
                R.im = ldexp(R.im, -b_dsh);                                                \
            }                                                                              \
        }                                                                                  \
    }
#define MST_LOAD_CHUNK(K0)                                                                 \
    {                                                                                      \
        const int k0 = (K0);                                                               \
        const bool fast = full_mn && (k0 + BK <= g.K) && !VARLEN && !SAFE &&               \
                          (OP != GOP_RESID || k0 >= r0 + BM);                              \
        int b_dsh = 0;                                                                     \
        if (SAFE && !B_CT && g.kb != nullptr && c0 + b_c < g.N) {                          \
            const int q = (g.b_row0 + k0 + b_k) / g.nb;                                    \
            b_dsh = g.kb[(long)g.q_cur * g.n_kb + c0 + b_c] -                              \
                    g.kb[(long)q * g.n_kb + c0 + b_c];                                     \
        }                                                                                  \
        (void)b_dsh;                                                                       \
        MST_LOAD_A(0, ra0) MST_LOAD_A(1, ra1) MST_LOAD_A(2, ra2) MST_LOAD_A(3, ra3)        \
        MST_LOAD_B(0, rb0) MST_LOAD_B(1, rb1) MST_LOAD_B(2, rb2) MST_LOAD_B(3, rb3)        \
    }
#define MST_STORE_CHUNK(BUF)                                                               \
    {                                                                                      \
        const int bf = (BUF);                                                              \
        if (!A_CT) {                                                                       \
            As[bf][a_k][a_r + 0] = ra0; As[bf][a_k][a_r + 1] = ra1;                        \
            As[bf][a_k][a_r + 2] = ra2; As[bf][a_k][a_r + 3] = ra3;                        \
        } else {                                                                           \
            As[bf][a_k + 0][a_r] = ra0; As[bf][a_k + 1][a_r] = ra1;                        \
            As[bf][a_k + 2][a_r] = ra2; As[bf][a_k + 3][a_r] = ra3;                        \
        }                                                                                  \
        if (!B_CT) {                                                                       \
            Bs[bf][b_k + 0][b_c] = rb0; Bs[bf][b_k + 1][b_c] = rb1;                        \
            Bs[bf][b_k + 2][b_c] = rb2; Bs[bf][b_k + 3][b_c] = rb3;                        \
        } else {                                                                           \
            Bs[bf][b_k][b_c + 0] = rb0; Bs[bf][b_k][b_c + 1] = rb1;                        \
            Bs[bf][b_k][b_c + 2] = rb2; Bs[bf][b_k][b_c + 3] = rb3;                        \
        }                                                                                  \
    }

    if (nchunk > 0) {
        MST_LOAD_CHUNK(kbeg)
        MST_STORE_CHUNK(0)
        __syncthreads();
        // substitution: the accumulators start at C, so A B is subtracted (A negated)
        const T s = (OP == GOP_SUB) ? T(-1) : T(1);
        for (int kc = 0; kc < nchunk; ++kc) {
            const int buf = kc & 1;
            if (kc + 1 < nchunk) MST_LOAD_CHUNK(kbeg + (kc + 1) * BK)
#pragma unroll
            for (int ks = 0; ks < BK / 4; ++ks) {
                const int kk = ks * 4 + lq;
                const CT a0 = As[buf][kk][wr * 32 + lr];
                const CT a1 = As[buf][kk][wr * 32 + 16 + lr];
                const CT b0 = Bs[buf][kk][wc * 32 + lr];
                const CT b1 = Bs[buf][kk][wc * 32 + 16 + lr];
                const T a0r = s * a0.re, a0i = s * a0.im, a1r = s * a1.re, a1i = s * a1.im;
                accR[0][0] = Tr::mfma(a0r, b0.re, accR[0][0]);
                accR[0][1] = Tr::mfma(a0r, b1.re, accR[0][1]);
                accR[1][0] = Tr::mfma(a1r, b0.re, accR[1][0]);
                accR[1][1] = Tr::mfma(a1r, b1.re, accR[1][1]);
                accI[0][0] = Tr::mfma(a0r, b0.im, accI[0][0]);
                accI[0][1] = Tr::mfma(a0r, b1.im, accI[0][1]);
                accI[1][0] = Tr::mfma(a1r, b0.im, accI[1][0]);
                accI[1][1] = Tr::mfma(a1r, b1.im, accI[1][1]);
                accR[0][0] = Tr::mfma(-a0i, b0.im, accR[0][0]);
                accR[0][1] = Tr::mfma(-a0i, b1.im, accR[0][1]);
                accR[1][0] = Tr::mfma(-a1i, b0.im, accR[1][0]);
                accR[1][1] = Tr::mfma(-a1i, b1.im, accR[1][1]);
                accI[0][0] = Tr::mfma(a0i, b0.re, accI[0][0]);
                accI[0][1] = Tr::mfma(a0i, b1.re, accI[0][1]);
                accI[1][0] = Tr::mfma(a1i, b0.re, accI[1][0]);
                accI[1][1] = Tr::mfma(a1i, b1.re, accI[1][1]);
            }
            if (kc + 1 < nchunk) MST_STORE_CHUNK(buf ^ 1)
            __syncthreads();
        }
    }
#undef MST_LOAD_A
#undef MST_LOAD_B
#undef MST_LOAD_CHUNK
#undef MST_STORE_CHUNK

    // ---- epilogue
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        const int col = c0 + wc * 32 + j * 16 + lr;
        if (col >= g.N) continue;
        const int clim = (j == 0) ? clim0 : clim1;
        CT lamc{0, 0};
        if (OP == GOP_RESID) lamc = CT{(T)g.lam[col].re, (T)g.lam[col].im};
#pragma unroll
        for (int i = 0; i < 2; ++i) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int row = r0 + wr * 32 + i * 16 + Tr::out_row(lq, v);
                if (!full_mn && row >= g.M) continue;
                const T ar = accR[i][j][v], ai = accI[i][j][v];
                CT* p = &C[(long)col * g.ldc + row];
                if (OP == GOP_SUB) {
                    if (VARLEN && row >= clim) continue;
                    *p = CT{ar, ai};
                } else if (OP == GOP_RESID) {
                    const CT b0 = ((const CT*)g.B0)[(long)col * g.ldb0 + row];
                    const CT x = B[(long)col * g.ldb + row];
                    const T lr_ = lamc.re * x.re - lamc.im * x.im;
                    const T li_ = lamc.re * x.im + lamc.im * x.re;
                    *p = CT{(b0.re - ar) + lr_, (b0.im - ai) + li_};
                } else {
                    *p = (row <= col) ? CT{-ar, -ai} : CT{0, 0};
                }
            }
        }
    }
}

// ---------------------------------------------------------------- barrier-free GEMM
// OP = GOP_SUB: C -= A B, A plain (the forward substitution step) or
// conjugate-transposed (the adjoint's); FP64, or FP32 for the mixed-precision
// substitution (plain operands only).
// OP = GOP_NEG_TRIU: C = -triu(A B^H) (the U gradient): accumulators start at
// zero, B is read conjugate-transposed, entries below the diagonal are written
// as zero and wavefront tiles entirely below it skip the product.
// OP = GOP_RESID: C = B0 - A B + B diag(lam), A upper triangular (U): each
// wavefront's K range starts at its first row and U's strict lower triangle
// is never read.
// Every wavefront owns a 32 x 32 complex tile of C and reads its MFMA operands
// straight from global memory (L1/L2) in the lane layout of the matrix cores:
// A(row, k) at lane row%16 + 16 k, B(k, col) at lane col%16 + 16 k. Loads run
// DEPTH k-steps ahead of the matrix cores in a register ring, so no LDS staging
// and no workgroup barrier are needed and each wavefront keeps its matrix pipe
// fed on its own. The 4 wavefronts of a workgroup cover a 64 x 64 tile and
// share A rows / B columns through L1.
// AM: A operand access: 0 plain A(r,k) = a[k*lda + r]; 1 conjugate transpose
// A(r,k) = conj(a[r*lda + k]); 2 transpose A(r,k) = a[r*lda + k].
// KS: wavefronts per 32 x 32 tile. With KS = 1 the workgroup covers 64 x 64;
// launches with too few tiles to give every SIMD work split each tile's K
// range over KS = 2 (workgroup tile 64 x 32) or KS = 4 (32 x 32) wavefronts,
// whose partial sums meet in LDS and are added in a fixed order, so the
// result does not depend on timing.
template <typename T, int DEPTH, int OP, int AM, bool SAFE, bool VARLEN, int KS>
__global__ __launch_bounds__(NT) void k_gemm_direct(GemmArgs g) {
    constexpr bool A_TR = AM != 0, A_CJ = AM == 1;
    static_assert(OP == GOP_SUB || OP == GOP_NEG_TRIU || OP == GOP_RESID || OP == GOP_GEN_SUB ||
                      OP == GOP_TRMM,
                  "direct GEMM op");
    static_assert(OP == GOP_SUB || OP == GOP_GEN_SUB || (!A_TR && !SAFE && !VARLEN),
                  "triangular products: plain A only");
    static_assert(OP != GOP_GEN_SUB || (sizeof(T) == 8 && !A_TR), "pencil substitution: FP64, plain A");
    static_assert(sizeof(T) == 8 || (OP == GOP_SUB && !A_TR && !SAFE && !VARLEN),
                  "FP32: plain substitution only");
    static_assert(KS == 1 || ((KS == 2 || KS == 4) && (OP == GOP_SUB || OP == GOP_RESID)),
                  "K split: substitution and residual only");
    constexpr bool TRI = OP == GOP_NEG_TRIU;
    constexpr bool RES = OP == GOP_RESID;
    constexpr bool GEN = OP == GOP_GEN_SUB;
    constexpr bool TRM = OP == GOP_TRMM;
    using Tr = Traits<T>;
    using CT = typename Tr::C;
    using V = typename Tr::V;
    if ((sizeof(T) == 4 || RES) && g.skip && *g.skip) return;   // refinement stopped
    constexpr int TBM = KS == 4 ? 32 : 64, TBN = KS == 1 ? 64 : 32;   // workgroup tile
    const int TM = (g.M + TBM - 1) / TBM, TN = (g.N + TBN - 1) / TBN;
    int tm, tn;
    if (TRI) {
        tri_coords(TM, tm, tn);   // square: M = N
    } else if (RES) {
        // work falls with the tile row (K runs from the row to the end): row
        // major, heaviest rows first, each row spread over all XCDs (the
        // hardware deals workgroup w to XCD w % 8)
        tm = blockIdx.x / TN;
        tn = blockIdx.x - tm * TN;
    } else if (TRM) {
        // work grows with the tile column (K runs to the column): column
        // major, heaviest columns first, each column spread over all XCDs
        tn = TN - 1 - blockIdx.x / TM;
        tm = blockIdx.x - (TN - 1 - tn) * TM;
    } else {
        tile_coords(TM, TN, tm, tn);
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    // wavefront tile (wr, wc) of the workgroup's and the K slice it computes
    const int wr = KS == 1 ? wave >> 1 : (KS == 2 ? wave & 1 : 0);
    const int wc = KS == 1 ? wave & 1 : 0;
    const int ksl = KS == 1 ? 0 : (KS == 2 ? wave >> 1 : wave);
    const int lr = lane & 15, lq = lane >> 4;
    const int rw = tm * TBM + wr * 32, cw = tn * TBN + wc * 32;
    const CT* __restrict__ A = (const CT*)g.A;
    const CT* __restrict__ B = (const CT*)g.B;
    CT* __restrict__ C = (CT*)g.C;

    if (VARLEN) {
        // a wavefront whose columns all end above the B operand's rows has nothing to do
        const int cc = cw + (lane & 31);
        const bool act = cc < g.N && g.col_len[cc] > g.b_row0;
        if (!__any(act)) return;
    }
    if (TRI && rw > cw + 31) {
        // tile entirely below the diagonal: zeros
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int col = cw + j * 16 + lr;
            if (col >= g.N) continue;
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int row = rw + i * 16 + Tr::out_row(lq, v);
                    if (row < g.M) C[(long)col * g.ldc + row] = CT{0, 0};
                }
        }
        return;
    }
    const bool full = (rw + 32 <= g.M) && (cw + 32 <= g.N);

    // ---- accumulators start from C (SUB), from B0 + lam B (RESID), from zero
    // (TRI; GEN, whose C is added at the end; K slices after the first)
    V accR[2][2], accI[2][2];
    int clim0 = g.M, clim1 = g.M, blim0 = g.K, blim1 = g.K;
    int cshv[2] = {0, 0};
    zd lamv[2] = {{0.0, 0.0}, {0.0, 0.0}};
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        const int col = cw + j * 16 + lr;
        int csh = 0, cl = g.M, bl = g.K;
        zd lamc{0.0, 0.0};
        if (col < g.N) {
            if (VARLEN) {
                cl = min(g.M, g.col_len[col] - g.c_row0);
                bl = min(g.K, g.col_len[col] - g.b_row0);
            }
            if (SAFE && g.kb != nullptr) {
                const int kc = g.kb[(long)g.q_cur * g.n_kb + col];
                const int kq = (g.q_c >= 0) ? g.kb[(long)g.q_c * g.n_kb + col] : 0;
                csh = kc - kq;
            }
            if (RES) lamc = g.lam[col];
            if (GEN) lamv[j] = g.glam[col];
        } else {
            bl = 0;
        }
        if (j == 0) {
            clim0 = cl;
            blim0 = bl;
        } else {
            clim1 = cl;
            blim1 = bl;
        }
        cshv[j] = csh;
#pragma unroll
        for (int i = 0; i < 2; ++i) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int row = rw + i * 16 + Tr::out_row(lq, v);
                CT c{0, 0};
                if (!TRI && !GEN && !TRM && ksl == 0 && col < g.N && row < cl) {
                    if (RES) {
                        const zd b0 = g.B0[(long)col * g.ldb0 + row];
                        const CT x = B[(long)col * g.ldb + row];
                        c = CT{T(b0.re + (lamc.re * x.re - lamc.im * x.im)),
                               T(b0.im + (lamc.re * x.im + lamc.im * x.re))};
                    } else {
                        c = C[(long)col * g.ldc + row];
                        if (SAFE) {
                            c.re = ldexp(c.re, -csh);
                            c.im = ldexp(c.im, -csh);
                        }
                    }
                }
                accR[i][j][v] = c.re;
                accI[i][j][v] = c.im;
            }
        }
    }

    // Operand positions of this lane, clamped into the matrices so that every
    // load is in bounds and none needs a branch: with straight-line loads the
    // wait before each k-step covers only that step's loads, not the ones in
    // flight for later steps. Elements outside the product are zeroed where
    // they are consumed (the clamped load may return anything, even NaN).
    int nks = (g.K + 3) / 4;
    if (VARLEN) {
        // no k-step past the longest of the wavefront's columns: beyond it
        // every B element is masked to zero (triangular right-hand sides
        // such as the eigenvector solve's skip about half the products)
        int bm = max(blim0, blim1);
        for (int off = 32; off >= 1; off >>= 1) bm = max(bm, __shfl_xor(bm, off, 64));
        nks = min(nks, (max(bm, 0) + 3) / 4);
    }
    const int kfirst0 = RES ? (rw >> 2) : 0;   // U(row, k) = 0 for k < row
    const int nloc0 = nks - kfirst0;
    const int ra0 = min(rw + lr, g.M - 1), ra1 = min(rw + 16 + lr, g.M - 1);
    const int cb0 = min(cw + lr, g.N - 1), cb1 = min(cw + 16 + lr, g.N - 1);
    const bool oka0 = rw + lr < g.M, oka1 = rw + 16 + lr < g.M;
    // safe form: exponent of the current outer block per column; the B rows of
    // diagonal block q carry exponent kb[q] and are brought to it exactly
    int kq0 = 0, kq1 = 0;
    // The plain loop also serves the safe and variable-length forms of a
    // wavefront whose columns all cover the B rows (col_len >= b_row0 + K, so
    // no element is masked) and for which every diagonal block under the K
    // range kept the current exponent (rescaling is rare): then the masks and
    // the operand scaling are identities.
    bool plain_ok = true;
    if (VARLEN) plain_ok = __all(g.col_len[cb0] >= g.b_row0 + g.K && g.col_len[cb1] >= g.b_row0 + g.K);
    if (SAFE) {
        kq0 = g.kb[(long)g.q_cur * g.n_kb + cb0];
        kq1 = g.kb[(long)g.q_cur * g.n_kb + cb1];
        if (plain_ok) {
            // exponents only grow as blocks are solved (bottom to top), so the
            // block solved first under the K range (the lowest) carries the
            // smallest: equal to the current one means all are equal
            const int qhi = (g.b_row0 + g.K - 1) / g.nb;
            plain_ok = __all(g.kb[(long)qhi * g.n_kb + cb0] == kq0 && g.kb[(long)qhi * g.n_kb + cb1] == kq1);
        }
    }

    auto kloop = [&](auto mask_tag, const CT* __restrict__ A, long lda, int kfirst, int nloc)
        __attribute__((always_inline)) {
        constexpr bool MASK = decltype(mask_tag)::value;
        CT pa0[DEPTH], pa1[DEPTH], pb0[DEPTH], pb1[DEPTH];
        int qe0[DEPTH] = {}, qe1[DEPTH] = {};
        auto load = [&](int ks, CT& a0, CT& a1, CT& b0, CT& b1, int& e0, int& e1)
            __attribute__((always_inline)) {
            const int k = MASK ? min(ks * 4 + lq, g.K - 1) : ks * 4 + lq;
            if (RES) {
                // stay inside U's upper triangle: below it the element is never used
                a0 = A[(long)max(k, ra0) * lda + ra0];
                a1 = A[(long)max(k, ra1) * lda + ra1];
            } else if (!A_TR) {
                const CT* ap = A + (long)k * lda;
                a0 = ap[ra0];
                a1 = ap[ra1];
            } else {
                // A(r, k) = conj(a[r * lda + k]); conjugated where consumed
                a0 = A[(long)ra0 * lda + k];
                a1 = A[(long)ra1 * lda + k];
            }
            if (!TRI) {
                b0 = B[(long)cb0 * g.ldb + k];
                b1 = B[(long)cb1 * g.ldb + k];
            } else {
                // B(k, c) = conj(b[k * ldb + c]); conjugated where consumed
                b0 = B[(long)k * g.ldb + cb0];
                b1 = B[(long)k * g.ldb + cb1];
            }
            if (SAFE) {
                const int q = (g.b_row0 + k) / g.nb;
                e0 = g.kb[(long)q * g.n_kb + cb0];
                e1 = g.kb[(long)q * g.n_kb + cb1];
            }
        };
        auto mma = [&](int ks, CT a0, CT a1, CT b0, CT b1, int e0, int e1)
            __attribute__((always_inline)) {
            if (MASK) {
                const int k = ks * 4 + lq;
                const bool kin = k < g.K;
                bool u0 = kin && oka0, u1 = kin && oka1;
                if (RES) {
                    u0 = u0 && k >= rw + lr;
                    u1 = u1 && k >= rw + 16 + lr;
                }
                // (TRM: B(k, c) = 0 below the diagonal, k > c)
                const bool v0 = k < blim0 && (!TRM || k <= cw + lr);
                const bool v1 = k < blim1 && (!TRM || k <= cw + 16 + lr);
                a0.re = u0 ? a0.re : T(0); a0.im = u0 ? a0.im : T(0);
                a1.re = u1 ? a1.re : T(0); a1.im = u1 ? a1.im : T(0);
                b0.re = v0 ? b0.re : T(0); b0.im = v0 ? b0.im : T(0);
                b1.re = v1 ? b1.re : T(0); b1.im = v1 ? b1.im : T(0);
            }
            if (SAFE && MASK) {
                b0.re = ldexp(b0.re, e0 - kq0); b0.im = ldexp(b0.im, e0 - kq0);
                b1.re = ldexp(b1.re, e1 - kq1); b1.im = ldexp(b1.im, e1 - kq1);
            }
            if constexpr (sizeof(T) == 8) {
                // acc -= A' B' with A' = conj(A) for A_CJ, B' = conj(B) for TRI.
                // FP64: every sign is an MFMA source modifier (the last operand's
                // bit 0 negates A), so the loop spends no VALU on negation:
                //   Re -= ar br - a'i b'i,  Im -= ar b'i + a'i br
                // (TRM: acc += A B, i.e. Re += ar br - ai bi, Im += ar bi + ai br)
                constexpr int NRR = TRM ? 0 : 1;
                constexpr int NII = TRM ? 1 : ((A_CJ != TRI) ? 1 : 0);   // + sa sb ai bi
                constexpr int NRI = (TRI || TRM) ? 0 : 1;               // - sb ar bi
                constexpr int NIR = (A_CJ || TRM) ? 0 : 1;              // - sa ai br
                accR[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0.re, b0.re, accR[0][0], 0, 0, NRR);
                accR[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0.re, b1.re, accR[0][1], 0, 0, NRR);
                accR[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1.re, b0.re, accR[1][0], 0, 0, NRR);
                accR[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1.re, b1.re, accR[1][1], 0, 0, NRR);
                accI[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0.re, b0.im, accI[0][0], 0, 0, NRI);
                accI[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0.re, b1.im, accI[0][1], 0, 0, NRI);
                accI[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1.re, b0.im, accI[1][0], 0, 0, NRI);
                accI[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1.re, b1.im, accI[1][1], 0, 0, NRI);
                accR[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0.im, b0.im, accR[0][0], 0, 0, NII);
                accR[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0.im, b1.im, accR[0][1], 0, 0, NII);
                accR[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1.im, b0.im, accR[1][0], 0, 0, NII);
                accR[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1.im, b1.im, accR[1][1], 0, 0, NII);
                accI[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0.im, b0.re, accI[0][0], 0, 0, NIR);
                accI[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0.im, b1.re, accI[0][1], 0, 0, NIR);
                accI[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1.im, b0.re, accI[1][0], 0, 0, NIR);
                accI[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1.im, b1.re, accI[1][1], 0, 0, NIR);
            } else {
                // FP32 (plain operands): acc = C - A B with A negated
                const T a0r = -a0.re, a1r = -a1.re, a0i = -a0.im, a1i = -a1.im;
                accR[0][0] = Tr::mfma(a0r, b0.re, accR[0][0]);
                accR[0][1] = Tr::mfma(a0r, b1.re, accR[0][1]);
                accR[1][0] = Tr::mfma(a1r, b0.re, accR[1][0]);
                accR[1][1] = Tr::mfma(a1r, b1.re, accR[1][1]);
                accI[0][0] = Tr::mfma(a0r, b0.im, accI[0][0]);
                accI[0][1] = Tr::mfma(a0r, b1.im, accI[0][1]);
                accI[1][0] = Tr::mfma(a1r, b0.im, accI[1][0]);
                accI[1][1] = Tr::mfma(a1r, b1.im, accI[1][1]);
                accR[0][0] = Tr::mfma(-a0i, b0.im, accR[0][0]);
                accR[0][1] = Tr::mfma(-a0i, b1.im, accR[0][1]);
                accR[1][0] = Tr::mfma(-a1i, b0.im, accR[1][0]);
                accR[1][1] = Tr::mfma(-a1i, b1.im, accR[1][1]);
                accI[0][0] = Tr::mfma(a0i, b0.re, accI[0][0]);
                accI[0][1] = Tr::mfma(a0i, b1.re, accI[0][1]);
                accI[1][0] = Tr::mfma(a1i, b0.re, accI[1][0]);
                accI[1][1] = Tr::mfma(a1i, b1.re, accI[1][1]);
            }
        };
        if (nloc <= 0) return;
        if constexpr (!MASK) {
            // Interior tiles (plain, full, K a multiple of 4, at least DEPTH
            // k-steps): one running pointer per operand, advanced by a k-step
            // per refill, so the loop spends one address add per operand
            // instead of recomputing products; the main loop runs while every
            // refill lies inside K, a short guarded tail drains the ring.
            const long sA = A_TR ? 4 : 4L * lda, sB = TRI ? 4L * g.ldb : 4;
            const long k0 = 4L * kfirst + lq;
            const CT* qa0 = A_TR ? A + (long)ra0 * lda + k0 : A + k0 * lda + ra0;
            const CT* qa1 = A_TR ? A + (long)ra1 * lda + k0 : qa0 + 16;
            const CT* qb0 = TRI ? B + k0 * g.ldb + cb0 : B + (long)cb0 * g.ldb + k0;
            const CT* qb1 = TRI ? qb0 + 16 : B + (long)cb1 * g.ldb + k0;
            auto next = [&](CT& a0, CT& a1, CT& b0, CT& b1) __attribute__((always_inline)) {
                a0 = *qa0; a1 = *qa1; b0 = *qb0; b1 = *qb1;
                qa0 += sA; qa1 += sA; qb0 += sB; qb1 += sB;
            };
            // the prologue fills the ring in the loop body's order (fenced like
            // it): the wait counts at the loop header merge both paths, and a
            // prologue the scheduler reordered makes the first k-step of every
            // ring round wait for loads of later slots
#pragma unroll
            for (int d = 0; d < DEPTH; ++d) {
                __builtin_amdgcn_sched_barrier(0);
                next(pa0[d], pa1[d], pb0[d], pb1[d]);
                __builtin_amdgcn_sched_barrier(0);
            }
            int l0 = 0;
            for (; l0 + 2 * DEPTH <= nloc; l0 += DEPTH) {
#pragma unroll
                for (int d = 0; d < DEPTH; ++d) {
                    mma(l0 + d, pa0[d], pa1[d], pb0[d], pb1[d], 0, 0);
                    __builtin_amdgcn_sched_barrier(0);
                    next(pa0[d], pa1[d], pb0[d], pb1[d]);
                    __builtin_amdgcn_sched_barrier(0);
                }
            }
#pragma unroll
            for (int d = 0; d < DEPTH; ++d) {
                mma(l0 + d, pa0[d], pa1[d], pb0[d], pb1[d], 0, 0);
                if (l0 + d + DEPTH < nloc) next(pa0[d], pa1[d], pb0[d], pb1[d]);
            }
#pragma unroll
            for (int d = 0; d < DEPTH; ++d)
                if (l0 + DEPTH + d < nloc) mma(l0 + DEPTH + d, pa0[d], pa1[d], pb0[d], pb1[d], 0, 0);
            return;
        }
        // The ring is refilled without a condition (past the end the last
        // k-step is loaded again, in bounds and unused), so the main loop is
        // straight-line code; only the last nloc % DEPTH steps are guarded.
#pragma unroll
        for (int d = 0; d < DEPTH; ++d) {
            __builtin_amdgcn_sched_barrier(0);
            load(kfirst + min(d, nloc - 1), pa0[d], pa1[d], pb0[d], pb1[d], qe0[d], qe1[d]);
            __builtin_amdgcn_sched_barrier(0);
        }
        int l0 = 0;
        for (; l0 + DEPTH <= nloc; l0 += DEPTH) {
#pragma unroll
            for (int d = 0; d < DEPTH; ++d) {
                // Step d consumes ring slot d, then refills it. The scheduling
                // fences pin that order: hoisting the refill above the products
                // gives it other registers, and the copy back into the ring at
                // the loop's end then waits for every load in flight; left free,
                // the scheduler also gathers all refills at the end of the body.
                mma(kfirst + l0 + d, pa0[d], pa1[d], pb0[d], pb1[d], qe0[d], qe1[d]);
                __builtin_amdgcn_sched_barrier(0);
                load(kfirst + min(l0 + d + DEPTH, nloc - 1), pa0[d], pa1[d], pb0[d], pb1[d], qe0[d], qe1[d]);
                __builtin_amdgcn_sched_barrier(0);
            }
        }
#pragma unroll
        for (int d = 0; d < DEPTH; ++d)
            if (l0 + d < nloc) mma(kfirst + l0 + d, pa0[d], pa1[d], pb0[d], pb1[d], qe0[d], qe1[d]);
    };
    // interior tiles of the plain forms need no masking at all
    const bool unmasked = full && (g.K & 3) == 0 && nloc0 >= DEPTH && !RES && plain_ok;
    if (GEN) {
        // pencil: acc = -A2 B, then acc = lam_c * (A2 B) per column (once per
        // tile, not per k-step), then acc -= A B; C is added in the epilogue
        if (unmasked)
            kloop(std::false_type{}, (const CT*)g.A2, g.lda2, 0, nloc0);
        else
            kloop(std::true_type{}, (const CT*)g.A2, g.lda2, 0, nloc0);
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const double r = accR[i][j][v], im = accI[i][j][v];
                    accR[i][j][v] = lamv[j].im * im - lamv[j].re * r;
                    accI[i][j][v] = -(lamv[j].re * im + lamv[j].im * r);
                }
    }
    if (TRM) {
        // B upper triangular: column c needs k <= c. k-steps below the
        // wavefront's first column need no mask; the (at most 8) steps across
        // its 32 columns are masked, and nothing past its last column is read.
        const int nk = (min(g.K, cw + 32) + 3) / 4;
        const int nfree = min(cw / 4, nk);
        int done = 0;
        if (full && (g.K & 3) == 0 && nfree >= DEPTH) {
            kloop(std::false_type{}, A, g.lda, 0, nfree);
            done = nfree;
        }
        kloop(std::true_type{}, A, g.lda, done, nk - done);
    } else if (KS == 1) {
        if (unmasked)
            kloop(std::false_type{}, A, g.lda, kfirst0, nloc0);
        else
            kloop(std::true_type{}, A, g.lda, kfirst0, nloc0);
    } else {
        // this wavefront's K slice: consecutive k-steps, the last slice shorter
        const int per = (nloc0 + KS - 1) / KS;
        const int kf = kfirst0 + ksl * per, nl = min(per, nloc0 - ksl * per);
        if (full && (g.K & 3) == 0 && nl >= DEPTH && !RES && plain_ok)
            kloop(std::false_type{}, A, g.lda, kf, nl);
        else
            kloop(std::true_type{}, A, g.lda, kf, nl);
    }

    if constexpr (KS > 1) {
        // Partial sums through LDS, one 16 KB (FP64) slot per wavefront tile
        // and round: KS = 2 adds s0 + s1, KS = 4 (s0 + s2) + (s1 + s3). Every
        // wavefront reaches every barrier (the early returns above are taken
        // by the whole workgroup or not at all: its wavefronts share columns).
        __shared__ T red[2][32][64];
        auto put = [&](int slot) __attribute__((always_inline)) {
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j)
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        red[slot][(i * 2 + j) * 4 + v][lane] = accR[i][j][v];
                        red[slot][16 + (i * 2 + j) * 4 + v][lane] = accI[i][j][v];
                    }
        };
        auto add = [&](int slot) __attribute__((always_inline)) {
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j)
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        accR[i][j][v] += red[slot][(i * 2 + j) * 4 + v][lane];
                        accI[i][j][v] += red[slot][16 + (i * 2 + j) * 4 + v][lane];
                    }
        };
        if (KS == 2) {
            if (ksl == 1) put(wr);
            __syncthreads();
            if (ksl == 1) return;
            add(wr);
        } else {
            if (ksl >= 2) put(ksl - 2);
            __syncthreads();
            if (ksl < 2) add(ksl);
            __syncthreads();
            if (ksl == 1) put(0);
            __syncthreads();
            if (ksl != 0) return;
            add(0);
        }
    }

    // ---- epilogue
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        const int col = cw + j * 16 + lr;
        if (col >= g.N) continue;
#pragma unroll
        for (int i = 0; i < 2; ++i) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int row = rw + i * 16 + Tr::out_row(lq, v);
                if (!full && row >= g.M) continue;
                if (VARLEN && row >= (j == 0 ? clim0 : clim1)) continue;
                if (TRI && row > col) {
                    C[(long)col * g.ldc + row] = CT{0, 0};
                    continue;
                }
                if (GEN) {
                    CT c = C[(long)col * g.ldc + row];
                    if (SAFE) {
                        c.re = ldexp(c.re, -cshv[j]);
                        c.im = ldexp(c.im, -cshv[j]);
                    }
                    C[(long)col * g.ldc + row] = CT{c.re + accR[i][j][v], c.im + accI[i][j][v]};
                    continue;
                }
                C[(long)col * g.ldc + row] = CT{accR[i][j][v], accI[i][j][v]};
            }
        }
    }
}

template <typename T, bool A_CT, bool B_CT, int OP, bool SAFE, bool VARLEN>
hipError_t go(const GemmArgs& g, hipStream_t s) {
    const int TM = (g.M + BM - 1) / BM, TN = (g.N + BN - 1) / BN;
    hipLaunchKernelGGL((k_gemm<T, A_CT, B_CT, OP, SAFE, VARLEN>), dim3(TM * TN), dim3(NT), 0, s, g);
    return hipGetLastError();
}


// K split of the direct GEMM for a launch shape (the measured cost of the
// shapes of the blocked solve on MI355X, FP64 and FP32, N = 128 ... 4096):
//  * a wavefront alone on its SIMD keeps the matrix pipe nearly as busy as
//    two, so time follows the k-steps of the SIMD with the most wavefronts,
//    ceil(waves / SIMDs) x k-steps per wavefront, plus about 16 k-steps for
//    every round of resident workgroups (ring fill, C, the slices' sums);
//  * a split-2 launch needing more than one round lost everywhere it was
//    measured (the workgroups of the last round pile up on the CUs that
//    free up first), so it is used within one round only.
// A split must promise a tenth less than the best smaller one.
int pick_split(const GemmArgs& g, int occupancy) {
    const long simds = 4L * device_cu_count();
    const long nks = (g.K + 3) / 4;
    long best = 0;
    int best_ks = 1;
    for (int ks = 1; ks <= 4; ks *= 2) {
        const int tbm = ks == 4 ? 32 : 64, tbn = ks == 1 ? 64 : 32;
        const long waves = 4L * ((g.M + tbm - 1) / tbm) * ((g.N + tbn - 1) / tbn);
        const long rounds = (waves + occupancy * simds - 1) / (occupancy * simds);
        if (ks == 2 && rounds > 1) continue;
        const long t = (waves + simds - 1) / simds * ((nks + ks - 1) / ks) + 16 * rounds;
        if (ks == 1 || 10 * t < 9 * best) {
            best = t;
            best_ks = ks;
        }
    }
    return best_ks;
}

template <typename T, int OP, int AM, bool SAFE, bool VARLEN>
hipError_t go_direct(const GemmArgs& g, hipStream_t s) {
    // wavefronts per tile: two per SIMD fit in FP64, three in FP32 (registers)
    const int ks = (OP != GOP_SUB && OP != GOP_RESID) ? 1 : g.split ? g.split : pick_split(g, sizeof(T) == 8 ? 2 : 3);
    if constexpr (OP == GOP_SUB || OP == GOP_RESID) {
        if (ks == 2) {
            const int TM = (g.M + 63) / 64, TN = (g.N + 31) / 32;
            hipLaunchKernelGGL((k_gemm_direct<T, 4, OP, AM, SAFE, VARLEN, 2>), dim3(TM * TN), dim3(NT), 0, s, g);
            return hipGetLastError();
        }
        if (ks == 4) {
            const int TM = (g.M + 31) / 32, TN = (g.N + 31) / 32;
            hipLaunchKernelGGL((k_gemm_direct<T, 4, OP, AM, SAFE, VARLEN, 4>), dim3(TM * TN), dim3(NT), 0, s, g);
            return hipGetLastError();
        }
    }
    const int TM = (g.M + BM - 1) / BM, TN = (g.N + BN - 1) / BN;
    hipLaunchKernelGGL((k_gemm_direct<T, 4, OP, AM, SAFE, VARLEN, 1>), dim3(TM * TN), dim3(NT), 0, s, g);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_gemm_f64(const GemmArgs& g, hipStream_t s) {
    if (g.M <= 0 || g.N <= 0) return hipSuccess;
    const bool safe = g.kb != nullptr;
    const bool varlen = g.col_len != nullptr;
    switch (g.op) {
        case GOP_SUB:
            if (g.b_ct || g.a_ct < 0 || g.a_ct > 2) return hipErrorInvalidValue;
            if (g.a_ct == 2) {
                if (safe || varlen || g.staged) return hipErrorInvalidValue;
                return go_direct<double, GOP_SUB, 2, false, false>(g, s);
            }
            if (g.a_ct) {
                if (safe || varlen) return hipErrorInvalidValue;
                if (g.staged) return go<double, true, false, GOP_SUB, false, false>(g, s);
                return go_direct<double, GOP_SUB, 1, false, false>(g, s);
            }
            if (g.staged) {
                if (safe && varlen) return go<double, false, false, GOP_SUB, true, true>(g, s);
                if (safe) return go<double, false, false, GOP_SUB, true, false>(g, s);
                if (varlen) return hipErrorInvalidValue;
                return go<double, false, false, GOP_SUB, false, false>(g, s);
            }
            if (safe && varlen) return go_direct<double, GOP_SUB, 0, true, true>(g, s);
            if (safe) return go_direct<double, GOP_SUB, 0, true, false>(g, s);
            if (varlen) return hipErrorInvalidValue;
            return go_direct<double, GOP_SUB, 0, false, false>(g, s);
        case GOP_RESID:
            if (g.a_ct || g.b_ct || safe || varlen) return hipErrorInvalidValue;
            if (g.staged) return go<double, false, false, GOP_RESID, false, false>(g, s);
            return go_direct<double, GOP_RESID, 0, false, false>(g, s);
        case GOP_GEN_SUB:
            if (g.a_ct || g.b_ct || !g.A2 || !g.glam || g.staged) return hipErrorInvalidValue;
            if (safe && varlen) return go_direct<double, GOP_GEN_SUB, 0, true, true>(g, s);
            if (safe) return go_direct<double, GOP_GEN_SUB, 0, true, false>(g, s);
            if (varlen) return hipErrorInvalidValue;
            return go_direct<double, GOP_GEN_SUB, 0, false, false>(g, s);
        case GOP_TRMM:
            if (g.a_ct || g.b_ct || safe || varlen || g.staged) return hipErrorInvalidValue;
            return go_direct<double, GOP_TRMM, 0, false, false>(g, s);
        case GOP_NEG_TRIU:
            if (g.a_ct || !g.b_ct || safe || varlen) return hipErrorInvalidValue;
            if (g.staged) return go<double, false, true, GOP_NEG_TRIU, false, false>(g, s);
            if (g.M != g.N) return hipErrorInvalidValue;
            return go_direct<double, GOP_NEG_TRIU, 0, false, false>(g, s);
        default:
            return hipErrorInvalidValue;
    }
}

hipError_t launch_gemm_f32(const GemmArgs& g, hipStream_t s) {
    if (g.M <= 0 || g.N <= 0) return hipSuccess;
    if (g.op != GOP_SUB || g.a_ct || g.b_ct || g.kb != nullptr || g.col_len != nullptr)
        return hipErrorInvalidValue;
    if (g.staged) return go<float, false, false, GOP_SUB, false, false>(g, s);
    return go_direct<float, GOP_SUB, 0, false, false>(g, s);
}

}  // namespace mst
