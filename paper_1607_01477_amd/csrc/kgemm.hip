// Complex GEMM on the matrix cores of gfx950 for the substitution step of the
// blocked multi-shift solve (the xGEMM of Alg 3 / Alg 5 of Moon & Poulson,
// arXiv 1607.01477), and for the residual and gradient products around it.
//
// A complex product is four real MFMA products on the same operands:
//   Re C += Re A Re B - Im A Im B,  Im C += Re A Im B + Im A Re B,
// which is exactly the 8 real flops per complex multiply-add of the nominal
// count (no extra flops, same rounding as a plain complex dot product up to
// order). FP64 uses v_mfma_f64_16x16x4_f64, FP32 v_mfma_f32_16x16x4_f32.
//
// Workgroup tile 64 x 64 complex, 4 wavefronts of 32 x 32, K staged through
// LDS 16 complex at a time with double buffering. Operands are read straight
// from the interleaved column-major storage, optionally conjugate-transposed,
// so no realified copy of U or X is ever formed in HBM. Tiles are ordered in
// groups of 8 row tiles and dealt out so that each XCD (own L2) receives a
// contiguous range of tiles.
#include "common.h"

namespace mst {
namespace {

constexpr int BM = 64, BN = 64, BK = 16, NT = 256;

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

template <typename T> struct Traits;
// Output lane layout of the 16x16x4 products (measured on gfx950): lane l,
// item v holds column l % 16 and row (l / 16) + 4 v for FP64, row 4 (l / 16) + v
// for FP32.
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

__device__ inline void tile_coords(int TM, int TN, int& tm, int& tn) {
    const int T = TM * TN;
    int w = blockIdx.x;
    if ((T & 7) == 0) w = (w & 7) * (T >> 3) + (w >> 3);   // one contiguous range per XCD
    constexpr int GROUP = 8;
    const int per_group = GROUP * TN;
    const int gid = w / per_group;
    const int first = gid * GROUP;
    const int gsz = min(TM - first, GROUP);
    const int in = w - gid * per_group;
    tm = first + in % gsz;
    tn = in / gsz;
}

template <typename T, bool A_CT, bool B_CT, int OP, bool SAFE, bool VARLEN>
__global__ __launch_bounds__(NT) void k_gemm(GemmArgs g) {
    using Tr = Traits<T>;
    using CT = typename Tr::C;
    using V = typename Tr::V;
    __shared__ CT As[2][BK][BM];
    __shared__ CT Bs[2][BK][BN];

    const int TM = (g.M + BM - 1) / BM, TN = (g.N + BN - 1) / BN;
    int tm, tn;
    tile_coords(TM, TN, tm, tn);
    const int r0 = tm * BM, c0 = tn * BN;
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int wr = wave >> 1, wc = wave & 1;
    const CT* __restrict__ A = (const CT*)g.A;
    const CT* __restrict__ B = (const CT*)g.B;
    CT* __restrict__ C = (CT*)g.C;

    if (OP == GOP_NEG_TRIU && r0 > c0 + BN - 1) {
        // tile strictly below the diagonal: zeros
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

    // K range (the residual's A is upper triangular: rows r0.. need k >= r0)
    int kbeg = 0;
    if (OP == GOP_RESID) kbeg = (r0 / BK) * BK;
    const int nchunk = (g.K - kbeg + BK - 1) / BK;

    // per-thread load coordinates (4 complex of A and 4 of B per chunk)
    CT ra[4], rb[4];
    auto load_chunk = [&](int k0) {
        // ---- A
        if (!A_CT) {
            const int k = t >> 4, rr = (t & 15) * 4;
            const int gk = k0 + k;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int gr = r0 + rr + e;
                CT v{0, 0};
                if (gk < g.K && gr < g.M) {
                    if (OP != GOP_RESID || gr <= gk) v = A[(long)gk * g.lda + gr];
                }
                ra[e] = v;
            }
        } else {
            const int rr = t >> 2, kk = (t & 3) * 4;
            const int gr = r0 + rr;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int gk = k0 + kk + e;
                CT v{0, 0};
                if (gk < g.K && gr < g.M) {
                    v = A[(long)gr * g.lda + gk];
                    v.im = -v.im;
                }
                ra[e] = v;
            }
        }
        // ---- B
        if (!B_CT) {
            const int cc = t >> 2, kk = (t & 3) * 4;
            const int gc = c0 + cc;
            int dsh = 0;
            int lim = g.K;
            if (gc < g.N) {
                if (VARLEN) lim = min(lim, g.col_len[gc] - g.b_row0);
                if (SAFE && g.kb != nullptr) {
                    const int q = (g.b_row0 + k0 + kk) / g.nb;
                    dsh = g.kb[(long)g.q_cur * g.n_kb + gc] - g.kb[(long)q * g.n_kb + gc];
                }
            }
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int gk = k0 + kk + e;
                CT v{0, 0};
                if (gk < lim && gc < g.N) {
                    v = B[(long)gc * g.ldb + gk];
                    if (SAFE) {
                        v.re = ldexp(v.re, -dsh);
                        v.im = ldexp(v.im, -dsh);
                    }
                }
                rb[e] = v;
            }
        } else {
            const int k = t >> 4, cc = (t & 15) * 4;
            const int gk = k0 + k;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int gc = c0 + cc + e;
                CT v{0, 0};
                if (gk < g.K && gc < g.N) {
                    v = B[(long)gk * g.ldb + gc];
                    v.im = -v.im;
                }
                rb[e] = v;
            }
        }
    };
    auto store_chunk = [&](int buf) {
        if (!A_CT) {
            const int k = t >> 4, rr = (t & 15) * 4;
#pragma unroll
            for (int e = 0; e < 4; ++e) As[buf][k][rr + e] = ra[e];
        } else {
            const int rr = t >> 2, kk = (t & 3) * 4;
#pragma unroll
            for (int e = 0; e < 4; ++e) As[buf][kk + e][rr] = ra[e];
        }
        if (!B_CT) {
            const int cc = t >> 2, kk = (t & 3) * 4;
#pragma unroll
            for (int e = 0; e < 4; ++e) Bs[buf][kk + e][cc] = rb[e];
        } else {
            const int k = t >> 4, cc = (t & 15) * 4;
#pragma unroll
            for (int e = 0; e < 4; ++e) Bs[buf][k][cc + e] = rb[e];
        }
    };

    V accR[2][2], accI[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            accR[i][j] = V{0, 0, 0, 0};
            accI[i][j] = V{0, 0, 0, 0};
        }

    if (nchunk > 0) {
        load_chunk(kbeg);
        store_chunk(0);
        __syncthreads();
        const int lr = lane & 15, lk = lane >> 4;
        for (int kc = 0; kc < nchunk; ++kc) {
            const int buf = kc & 1;
            if (kc + 1 < nchunk) load_chunk(kbeg + (kc + 1) * BK);
#pragma unroll
            for (int ks = 0; ks < BK / 4; ++ks) {
                const int kk = ks * 4 + lk;
                CT a[2], b[2];
#pragma unroll
                for (int i = 0; i < 2; ++i) a[i] = As[buf][kk][wr * 32 + i * 16 + lr];
#pragma unroll
                for (int j = 0; j < 2; ++j) b[j] = Bs[buf][kk][wc * 32 + j * 16 + lr];
#pragma unroll
                for (int i = 0; i < 2; ++i) {
                    const T nai = -a[i].im;
#pragma unroll
                    for (int j = 0; j < 2; ++j) {
                        accR[i][j] = Tr::mfma(a[i].re, b[j].re, accR[i][j]);
                        accR[i][j] = Tr::mfma(nai, b[j].im, accR[i][j]);
                        accI[i][j] = Tr::mfma(a[i].re, b[j].im, accI[i][j]);
                        accI[i][j] = Tr::mfma(a[i].im, b[j].re, accI[i][j]);
                    }
                }
            }
            if (kc + 1 < nchunk) store_chunk(buf ^ 1);
            __syncthreads();
        }
    }

    // epilogue: lane holds column lane%16 of each 16x16 tile, rows per Traits::out_row
    const int lr = lane & 15, lq = lane >> 4;
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        const int col = c0 + wc * 32 + j * 16 + lr;
        if (col >= g.N) continue;
        int csh = 0;
        int lim = g.M;
        if (OP == GOP_SUB) {
            if (VARLEN) lim = min(lim, g.col_len[col] - g.c_row0);
            if (SAFE && g.kb != nullptr) {
                const int kc = g.kb[(long)g.q_cur * g.n_kb + col];
                const int kq = (g.q_c >= 0) ? g.kb[(long)g.q_c * g.n_kb + col] : 0;
                csh = kc - kq;
            }
        }
        CT lamc{0, 0};
        if (OP == GOP_RESID) lamc = CT{(T)g.lam[col].re, (T)g.lam[col].im};
#pragma unroll
        for (int i = 0; i < 2; ++i) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int row = r0 + wr * 32 + i * 16 + Tr::out_row(lq, v);
                if (row >= lim) continue;
                const T ar = accR[i][j][v], ai = accI[i][j][v];
                CT* p = &C[(long)col * g.ldc + row];
                if (OP == GOP_SUB) {
                    CT c = *p;
                    if (SAFE) {
                        c.re = ldexp(c.re, -csh);
                        c.im = ldexp(c.im, -csh);
                    }
                    *p = CT{c.re - ar, c.im - ai};
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

template <typename T, bool A_CT, bool B_CT, int OP, bool SAFE, bool VARLEN>
hipError_t go(const GemmArgs& g, hipStream_t s) {
    const int TM = (g.M + BM - 1) / BM, TN = (g.N + BN - 1) / BN;
    hipLaunchKernelGGL((k_gemm<T, A_CT, B_CT, OP, SAFE, VARLEN>), dim3(TM * TN), dim3(NT), 0, s, g);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_gemm_f64(const GemmArgs& g, hipStream_t s) {
    if (g.M <= 0 || g.N <= 0) return hipSuccess;
    const bool safe = g.kb != nullptr;
    const bool varlen = g.col_len != nullptr;
    switch (g.op) {
        case GOP_SUB:
            if (g.b_ct) return hipErrorInvalidValue;
            if (g.a_ct) {
                if (safe || varlen) return hipErrorInvalidValue;
                return go<double, true, false, GOP_SUB, false, false>(g, s);
            }
            if (safe && varlen) return go<double, false, false, GOP_SUB, true, true>(g, s);
            if (safe) return go<double, false, false, GOP_SUB, true, false>(g, s);
            if (varlen) return hipErrorInvalidValue;
            return go<double, false, false, GOP_SUB, false, false>(g, s);
        case GOP_RESID:
            if (g.a_ct || g.b_ct || safe || varlen) return hipErrorInvalidValue;
            return go<double, false, false, GOP_RESID, false, false>(g, s);
        case GOP_NEG_TRIU:
            if (g.a_ct || !g.b_ct || safe || varlen) return hipErrorInvalidValue;
            return go<double, false, true, GOP_NEG_TRIU, false, false>(g, s);
        default:
            return hipErrorInvalidValue;
    }
}

hipError_t launch_gemm_f32(const GemmArgs& g, hipStream_t s) {
    if (g.M <= 0 || g.N <= 0) return hipSuccess;
    if (g.op != GOP_SUB || g.a_ct || g.b_ct || g.kb != nullptr || g.col_len != nullptr)
        return hipErrorInvalidValue;
    return go<float, false, false, GOP_SUB, false, false>(g, s);
}

}  // namespace mst
