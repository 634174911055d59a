// Real-arithmetic multi-shift solve on gfx950: U, the shifts and the
// right-hand sides real (float64). The paper leaves real arithmetic to future
// work; this is its plainest form, the blocked back substitution of Alg 3 with
// real operands:
//   k_block_real - one block of up to 256 rows for all shifts: the 64-row
//                  diagonal blocks and the updates inside the block fused,
//                  lane r of a wavefront owning rows r + 64 g, the solution
//                  entry of each step broadcast with v_readlane, several
//                  shifts per wavefront interleaved;
//   k_gemm_real  - the substitution C -= A B between blocks on the FP64
//                  matrix cores (one v_mfma_f64_16x16x4_f64 per 16 x 16 x 4
//                  block), operands streamed from L1/L2 into registers a few
//                  k-steps ahead, the wavefront tile chosen by shape;
//   k_real_upper_copy, k_reverse_rows - the lower, transposed and right-side
//                  variants (footnote to Sec. 2) as this upper solve: an
//                  upper-triangular copy of A and the rows of B reversed.
#include <cstdint>

#include "common.h"

namespace mst {
namespace {

typedef double v4d __attribute__((ext_vector_type(4)));

constexpr int RNT = 256;            // threads per workgroup

// C(M x N) -= A(M x K) B(K x N), all column-major, K > 0. Four wavefronts in a
// 2 x 2 arrangement, each with a (16 TI) x (16 TJ) tile of C: TI x TJ products
// of 16 x 16 x 4 per k-step from TI + TJ operand loads, DEPTH k-steps of
// operands in flight. FP64 output layout of the 16 x 16 x 4 product: lane l,
// item v holds column l % 16, row l / 16 + 4 v; operands A(i, k) at lane
// i + 16 k, B(k, j) at lane j + 16 k. The first k-step takes C as its
// accumulator input, one column subtile at a time, so that C never occupies
// more than TI x 4 registers outside the accumulators.
template <int TI, int TJ, int DEPTH, bool PAIR = false>
__global__ __launch_bounds__(RNT) void k_gemm_real(RealGemmArgs g) {
    static_assert(!PAIR || TI % 2 == 0, "row pairs: even number of row subtiles");
    constexpr int WM = 16 * TI, WN = 16 * TJ, BM = 2 * WM, BN = 2 * WN;
    const int TM = (g.M + BM - 1) / BM, TN = (g.N + BN - 1) / BN;
    int tm, tn;
    tile_coords(TM, TN, tm, tn);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int lr = lane & 15, lq = lane >> 4;
    const int rw = tm * BM + (wave >> 1) * WM, cw = tn * BN + (wave & 1) * WN;
    const bool full = rw + WM <= g.M && cw + WN <= g.N;
    const double* __restrict__ A = g.A;
    const double* __restrict__ B = g.B;
    double* __restrict__ C = g.C;
    const int nks = (g.K + 3) / 4;
    // row r16 (0..15) of row subtile i: consecutive 16-row blocks, or with
    // PAIR the subtiles 2p and 2p + 1 interleaved over 32 rows (even and odd
    // rows), so that one 16-byte load gives a lane its rows of both
    auto rowmap = [&](int i, int r16) __attribute__((always_inline)) {
        return PAIR ? rw + 32 * (i >> 1) + 2 * r16 + (i & 1) : rw + 16 * i + r16;
    };

    v4d acc[TI][TJ];
    // acc -= a b: the negation is the MFMA's source modifier on A
    auto mma = [&](const double (&a)[TI], const double (&b)[TJ]) __attribute__((always_inline)) {
#pragma unroll
        for (int i = 0; i < TI; ++i)
#pragma unroll
            for (int j = 0; j < TJ; ++j)
                acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 1);
    };
    // the first k-step: acc = C - a b, column subtile by column subtile
    auto first = [&](const double (&a)[TI], const double (&b)[TJ]) __attribute__((always_inline)) {
#pragma unroll
        for (int j = 0; j < TJ; ++j) {
            const int col = cw + j * 16 + lr;
            v4d c[TI];
#pragma unroll
            for (int i = 0; i < TI; ++i)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int row = rowmap(i, lq + 4 * v);
                    c[i][v] = (col < g.N && row < g.M) ? C[(long)col * g.ldc + row] : 0.0;
                }
#pragma unroll
            for (int i = 0; i < TI; ++i)
                acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], c[i], 0, 0, 1);
            __builtin_amdgcn_sched_barrier(0);
        }
    };
    int ra[TI], cb[TJ];
#pragma unroll
    for (int i = 0; i < TI; ++i) ra[i] = min(rowmap(i, lr), g.M - 1);
#pragma unroll
    for (int j = 0; j < TJ; ++j) cb[j] = min(cw + 16 * j + lr, g.N - 1);
    double pa[DEPTH][TI], pb[DEPTH][TJ];
    // k-step l lives in ring slot l % DEPTH; fetch(l, slot) loads it,
    // consume(l, slot) multiplies it in
    auto ring = [&](auto fetch, auto consume, auto consume_first) __attribute__((always_inline)) {
#pragma unroll
        for (int d = 0; d < DEPTH; ++d) fetch(d, pa[d], pb[d]);
        consume_first(pa[0], pb[0]);
        if (DEPTH < nks) fetch(DEPTH, pa[0], pb[0]);
        int l0 = 1;
        for (; l0 + 2 * DEPTH <= nks; l0 += DEPTH) {
#pragma unroll
            for (int d = 0; d < DEPTH; ++d) {
                const int sl = (1 + d) % DEPTH;
                consume(l0 + d, pa[sl], pb[sl]);
                __builtin_amdgcn_sched_barrier(0);
                fetch(l0 + d + DEPTH, pa[sl], pb[sl]);
                __builtin_amdgcn_sched_barrier(0);
            }
        }
#pragma unroll
        for (int d = 0; d < DEPTH; ++d) {
            const int sl = (1 + d) % DEPTH;
            if (l0 + d < nks) {
                consume(l0 + d, pa[sl], pb[sl]);
                if (l0 + d + DEPTH < nks) fetch(l0 + d + DEPTH, pa[sl], pb[sl]);
            }
        }
#pragma unroll
        for (int d = 0; d < DEPTH; ++d) {
            const int sl = (1 + d) % DEPTH;
            if (l0 + DEPTH + d < nks) consume(l0 + DEPTH + d, pa[sl], pb[sl]);
        }
    };
    if (full && (g.K & 3) == 0 && nks >= DEPTH) {
        // interior tile: no masking, one running pointer per operand row / column
        const long sA = 4L * g.lda;
        const double* qa = A + (long)lq * g.lda + ra[0];
        const double* qb[TJ];
#pragma unroll
        for (int j = 0; j < TJ; ++j) qb[j] = B + (long)cb[j] * g.ldb + lq;
        auto next = [&](int, double (&a)[TI], double (&b)[TJ]) __attribute__((always_inline)) {
            if constexpr (PAIR) {
                // rows rw + 32 p + 2 lr and + 1: one 16-byte load (16-byte
                // alignment checked by the launcher)
#pragma unroll
                for (int p = 0; p < TI / 2; ++p) {
                    const double2 v = *(const double2*)(qa + 32 * p);
                    a[2 * p] = v.x;
                    a[2 * p + 1] = v.y;
                }
            } else {
#pragma unroll
                for (int i = 0; i < TI; ++i) a[i] = qa[16 * i];
            }
#pragma unroll
            for (int j = 0; j < TJ; ++j) { b[j] = *qb[j]; qb[j] += 4; }
            qa += sA;
        };
        auto use = [&](int, const double (&a)[TI], const double (&b)[TJ]) __attribute__((always_inline)) {
            mma(a, b);
        };
        ring(next, use, first);
    } else {
        // edge tile: clamped unconditional loads, values outside zeroed at use
        bool oka[TI], okb[TJ];
#pragma unroll
        for (int i = 0; i < TI; ++i) oka[i] = rowmap(i, lr) < g.M;
#pragma unroll
        for (int j = 0; j < TJ; ++j) okb[j] = cw + 16 * j + lr < g.N;
        auto load = [&](int ks, double (&a)[TI], double (&b)[TJ]) __attribute__((always_inline)) {
            const int k = min(ks * 4 + lq, g.K - 1);
            const double* ap = A + (long)k * g.lda;
#pragma unroll
            for (int i = 0; i < TI; ++i) a[i] = ap[ra[i]];
#pragma unroll
            for (int j = 0; j < TJ; ++j) b[j] = B[(long)cb[j] * g.ldb + k];
        };
        auto masked = [&](int ks, const double (&a)[TI], const double (&b)[TJ], double (&am)[TI],
                          double (&bm)[TJ]) __attribute__((always_inline)) {
            const bool kin = ks * 4 + lq < g.K;
#pragma unroll
            for (int i = 0; i < TI; ++i) am[i] = (kin && oka[i]) ? a[i] : 0.0;
#pragma unroll
            for (int j = 0; j < TJ; ++j) bm[j] = (kin && okb[j]) ? b[j] : 0.0;
        };
        auto use = [&](int ks, const double (&a)[TI], const double (&b)[TJ]) __attribute__((always_inline)) {
            double am[TI], bm[TJ];
            masked(ks, a, b, am, bm);
            mma(am, bm);
        };
        auto use_first = [&](const double (&a)[TI], const double (&b)[TJ]) __attribute__((always_inline)) {
            double am[TI], bm[TJ];
            masked(0, a, b, am, bm);
            first(am, bm);
        };
        ring(load, use, use_first);
    }
#pragma unroll
    for (int j = 0; j < TJ; ++j) {
        const int col = cw + j * 16 + lr;
        if (col >= g.N) continue;
#pragma unroll
        for (int i = 0; i < TI; ++i)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int row = rowmap(i, lq + 4 * v);
                if (row < g.M) C[(long)col * g.ldc + row] = acc[i][j][v];
            }
    }
}

template <int TI, int TJ, int DEPTH, bool PAIR = false>
hipError_t launch_gemm_real_t(const RealGemmArgs& g, hipStream_t s) {
    constexpr int BM = 32 * TI, BN = 32 * TJ;
    const int TM = (g.M + BM - 1) / BM, TN = (g.N + BN - 1) / BN;
    hipLaunchKernelGGL((k_gemm_real<TI, TJ, DEPTH, PAIR>), dim3(TM * TN), dim3(RNT), 0, s, g);
    return hipGetLastError();
}

// Value of lane i (wave-uniform) to every lane.
__device__ inline double readlane_d(double v, int i) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), i);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), i);
    return __hiloint2double(hi, lo);
}

// One block [i0, i0 + bs) of up to 256 rows for all shifts, in place in B.
// Each wavefront owns S shifts and all rows of the block: lane r holds rows
// r, r + 64, r + 128, r + 192 (row groups g = 0..3). The 64-row diagonal
// blocks are taken bottom-up; inside diagonal block C, step i broadcasts the
// finished x(64 C + i) with v_readlane and applies column 64 C + i of U both
// to the rows of block C above it and to all rows of the groups g < C. Rows
// of block C are scaled by their pivot reciprocals when the block starts:
// with b'(r) = b(r) / d(r) and u'(r, i) = u(r, i) / d(r), step i is
// x(i) = b'(i) (broadcast) and b'(r) -= u'(r, i) x(i); rows of the groups
// g < C take the unscaled update until their own diagonal block starts. No
// LDS and no barriers: the columns of U are read straight from memory, R
// steps ahead of their use.
template <int C, int S, int R>
__device__ __forceinline__ void block_real_sub(const RealDiagArgs& a, double (&b)[4][S], const double (&lam)[S],
                                               const bool (&jv)[S], int lane) {
    const int bs = a.bs;
    const int rc = 64 * C + lane;                      // local row of this lane in group C
    const int ie = min(63, bs - 64 * C - 1);            // last step of the (possibly partial) block
    const double* __restrict__ Ub = a.U + (long)a.i0 * a.ldu + a.i0;   // U(i0, i0)
    double p[S];
    {
        const bool on = rc < bs;
        const double d = on ? Ub[(long)rc * a.ldu + rc] : 1.0;
#pragma unroll
        for (int s = 0; s < S; ++s) {
            p[s] = (on && jv[s]) ? 1.0 / (d - lam[s]) : 0.0;
            b[C][s] *= p[s];
        }
    }
    // Steps ie + 1 .. T - 1 (T a multiple of R) only pad a partial block: lane
    // `step` then holds b = 0, so x = 0 and the step changes nothing; their
    // column is clamped into the block.
    const int T = (ie + R) / R * R;
    auto fetch = [&](int step, double (&u)[C + 1]) __attribute__((always_inline)) {
        const int cs = min(max(step, 0), ie);
        const double* col = Ub + (long)(64 * C + cs) * a.ldu;
#pragma unroll
        for (int g = 0; g < C; ++g) u[g] = col[64 * g + lane];
        // rows on or below the diagonal read the diagonal entry instead (the
        // value is discarded there): the strict lower triangle is never read
        u[C] = col[64 * C + min(lane, cs)];
    };
    double uq[R][C + 1];
    // issue order = use order (the load counter is waited on in order)
#pragma unroll
    for (int r = 0; r < R; ++r) {
        fetch(T - 1 - r, uq[r]);
        __builtin_amdgcn_sched_barrier(0);
    }
    // Software-pipelined steps: the rows of the groups g < C take the update of
    // step k + 1 while the readlane of step k and the pivot-block update of
    // step k are in flight.
    double xp[S], up[C > 0 ? C : 1];
#pragma unroll
    for (int s = 0; s < S; ++s) xp[s] = 0.0;
#pragma unroll
    for (int g = 0; g < (C > 0 ? C : 1); ++g) up[g] = 0.0;
    auto lagged = [&](int h) __attribute__((always_inline)) {
        // half h of the lagged update: shifts [h S / 2, (h + 1) S / 2)
#pragma unroll
        for (int s = h * S / 2; s < (h + 1) * S / 2; ++s)
#pragma unroll
            for (int g = 0; g < C; ++g) b[g][s] = fma(-up[g], xp[s], b[g][s]);
    };
    for (int i = T - 1; i >= 0; i -= R) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int step = i - r;
            const double uc = (lane < step) ? uq[r][C] : 0.0;
            double x[S];
#pragma unroll
            for (int s = 0; s < S; ++s) x[s] = readlane_d(b[C][s], step);
            __builtin_amdgcn_sched_barrier(0);
            lagged(0);
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int s = 0; s < S; ++s) b[C][s] = fma(-(uc * p[s]), x[s], b[C][s]);
            __builtin_amdgcn_sched_barrier(0);
            lagged(1);
#pragma unroll
            for (int s = 0; s < S; ++s) xp[s] = x[s];
#pragma unroll
            for (int g = 0; g < C; ++g) up[g] = uq[r][g];
            fetch(step - R, uq[r]);
            __builtin_amdgcn_sched_barrier(0);
        }
    }
    lagged(0);
    lagged(1);
}

template <int S, int R>
__global__ __launch_bounds__(RNT) void k_block_real(RealDiagArgs a) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int j0 = (blockIdx.x * (RNT / 64) + wave) * S;
    if (j0 >= a.n) return;
    const int nsub = (a.bs + 63) / 64;
    double b[4][S], lam[S];
    bool jv[S];
#pragma unroll
    for (int s = 0; s < S; ++s) {
        const int j = j0 + s;
        jv[s] = j < a.n;
        lam[s] = jv[s] ? a.lam[j] : 0.0;
        const double* bc = a.B + (long)(jv[s] ? j : j0) * a.ldb + a.i0;
#pragma unroll
        for (int g = 0; g < 4; ++g) {
            const int r = 64 * g + lane;
            b[g][s] = (jv[s] && r < a.bs) ? bc[r] : 0.0;
        }
    }
    if (nsub > 3) block_real_sub<3, S, R>(a, b, lam, jv, lane);
    if (nsub > 2) block_real_sub<2, S, R>(a, b, lam, jv, lane);
    if (nsub > 1) block_real_sub<1, S, R>(a, b, lam, jv, lane);
    block_real_sub<0, S, R>(a, b, lam, jv, lane);
#pragma unroll
    for (int s = 0; s < S; ++s) {
        if (!jv[s]) continue;
        double* bc = a.B + (long)(j0 + s) * a.ldb + a.i0;
#pragma unroll
        for (int g = 0; g < 4; ++g) {
            const int r = 64 * g + lane;
            if (r < a.bs) bc[r] = b[g][s];
        }
    }
}

template <int S, int R>
hipError_t launch_block_real_t(const RealDiagArgs& a, hipStream_t s) {
    constexpr int per_wg = (RNT / 64) * S;
    hipLaunchKernelGGL((k_block_real<S, R>), dim3((a.n + per_wg - 1) / per_wg), dim3(RNT), 0, s, a);
    return hipGetLastError();
}

// One 32 x 32 tile of Uh: the matching tile of A is read along its columns
// (coalesced), parked in LDS under Uh's coordinates, and written along Uh's
// columns. Elements outside A's own triangle or outside the matrix are never
// touched; Uh's strict lower triangle is left unwritten.
__global__ __launch_bounds__(256) void k_real_upper_copy(int m, const double* __restrict__ A, long lda, int mode,
                                                         double* __restrict__ Uh) {
    __shared__ double sh[32][33];
    const int i0 = blockIdx.x * 32, j0 = blockIdx.y * 32;
    if (i0 > j0 + 31) return;   // tile entirely below the diagonal
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    // origin of the source tile and the map (rl, cl) -> (il, jl)
    int p0, q0;
    if (mode == REAL_T) { p0 = j0; q0 = i0; }
    else if (mode == REAL_JJ) { p0 = m - 32 - i0; q0 = m - 32 - j0; }
    else { p0 = m - 32 - j0; q0 = m - 32 - i0; }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int rl = tx, cl = ty + 8 * k;
        int il, jl;
        if (mode == REAL_T) { il = cl; jl = rl; }
        else if (mode == REAL_JJ) { il = 31 - rl; jl = 31 - cl; }
        else { il = 31 - cl; jl = 31 - rl; }
        const int p = p0 + rl, q = q0 + cl, i = i0 + il, j = j0 + jl;
        double v = 0.0;
        if (p >= 0 && p < m && q >= 0 && q < m && i <= j) v = A[(long)q * lda + p];
        sh[il][jl] = v;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int il = tx, jl = ty + 8 * k;
        const int i = i0 + il, j = j0 + jl;
        if (i < m && j < m && i <= j) Uh[(long)j * m + i] = sh[il][jl];
    }
}

__global__ __launch_bounds__(256) void k_reverse_rows(int m, int n, double* __restrict__ B, long ldb) {
    const int half = m / 2;
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y;
    if (t >= half || j >= n) return;
    double* col = B + (long)j * ldb;
    const int i = (int)t, k = m - 1 - (int)t;
    const double a = col[i], b = col[k];
    col[i] = b;
    col[k] = a;
}

}  // namespace

hipError_t launch_real_upper_copy(int m, const double* A, long lda, int mode, double* Uh, hipStream_t s) {
    if (m <= 0) return hipSuccess;
    if (mode < REAL_T || mode > REAL_JTJ) return hipErrorInvalidValue;
    const int T = (m + 31) / 32;
    hipLaunchKernelGGL(k_real_upper_copy, dim3(T, T), dim3(256), 0, s, m, A, lda, mode, Uh);
    return hipGetLastError();
}

hipError_t launch_reverse_rows(int m, int n, double* B, long ldb, hipStream_t s) {
    if (m < 2 || n <= 0) return hipSuccess;
    if (n > 65535) {
        // grid.y limit: columns in chunks
        for (int j0 = 0; j0 < n; j0 += 65535) {
            hipError_t e = launch_reverse_rows(m, (n - j0 < 65535 ? n - j0 : 65535), B + (long)j0 * ldb, ldb, s);
            if (e != hipSuccess) return e;
        }
        return hipSuccess;
    }
    const int half = m / 2;
    hipLaunchKernelGGL(k_reverse_rows, dim3((half + 255) / 256, n), dim3(256), 0, s, m, n, B, ldb);
    return hipGetLastError();
}

hipError_t launch_gemm_real(const RealGemmArgs& g, hipStream_t s) {
    if (g.K < 0) return hipErrorInvalidValue;
    if (g.M <= 0 || g.N <= 0 || g.K == 0) return hipSuccess;
    // The largest wavefront tile that still gives the chip enough wavefronts:
    // 128 x 32 (16 products per 10 loads, or per 6 with row pairs) for the
    // deferred updates, 64 x 32 in between, 32 x 32 for thin updates. Two
    // k-steps in flight for 128 x 32 once there are two such wavefronts per
    // SIMD, more below. Row pairs (one 16-byte load for two rows of A) need A
    // 16-byte aligned with an even leading dimension.
    const long w8 = (long)((g.M + 127) / 128) * ((g.N + 31) / 32);
    const long w4 = (long)((g.M + 63) / 64) * ((g.N + 31) / 32);
    const bool pair = ((uintptr_t)g.A & 15) == 0 && (g.lda & 1) == 0;
    if (w8 >= 1536) return pair ? launch_gemm_real_t<8, 2, 2, true>(g, s) : launch_gemm_real_t<8, 2, 2>(g, s);
    if (w8 >= 768) return pair ? launch_gemm_real_t<8, 2, 4, true>(g, s) : launch_gemm_real_t<8, 2, 3>(g, s);
    if (w4 >= 1024) return pair ? launch_gemm_real_t<4, 2, 4, true>(g, s) : launch_gemm_real_t<4, 2, 4>(g, s);
    return launch_gemm_real_t<2, 2, 4>(g, s);
}

hipError_t launch_block_real(const RealDiagArgs& a, hipStream_t s) {
    if (a.bs <= 0 || a.bs > 256 || a.n <= 0) return hipErrorInvalidValue;
    return launch_block_real_t<4, 8>(a, s);
}

}  // namespace mst
