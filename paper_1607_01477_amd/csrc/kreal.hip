// Real-arithmetic multi-shift solve on gfx950: U, the shifts and the
// right-hand sides real (float64). The paper leaves real arithmetic to future
// work; this is its plainest form, the blocked back substitution of Alg 3 with
// real operands:
//   k_diag_real - one nb x nb diagonal block for all shifts: the block in LDS,
//                 lane r of a wavefront owns row r, the solution entry of
//                 each step broadcast with v_readlane; several shifts per
//                 wavefront interleaved to hide the step latency;
//   k_gemm_real - the substitution C -= A B on the FP64 matrix cores
//                 (one v_mfma_f64_16x16x4_f64 per 16 x 16 x 4 block), operands
//                 streamed from L1/L2 into registers a few k-steps ahead.
#include "common.h"

namespace mst {
namespace {

typedef double v4d __attribute__((ext_vector_type(4)));

constexpr int RNT = 256;            // threads per workgroup
constexpr int RBM = 64, RBN = 64;   // GEMM workgroup tile (four 32 x 32 wavefront tiles)
constexpr int RDEPTH = 4;           // k-steps of operands in flight

// Workgroup -> tile: groups of 8 row tiles, one contiguous range of tiles per
// XCD (the hardware deals workgroup w to XCD w % 8).
__device__ inline void real_tile(int TM, int TN, int& tm, int& tn) {
    const int T = TM * TN;
    int w = blockIdx.x;
    if ((T & 7) == 0) w = (w & 7) * (T >> 3) + (w >> 3);
    constexpr int GROUP = 8;
    const int per_group = GROUP * TN;
    const int gid = w / per_group;
    const int first = gid * GROUP;
    const int gsz = min(TM - first, GROUP);
    const int in = w - gid * per_group;
    tm = first + in % gsz;
    tn = in / gsz;
}

// C(M x N) -= A(M x K) B(K x N), all column-major. FP64 output layout of the
// 16 x 16 x 4 product: lane l, item v holds column l % 16, row l / 16 + 4 v;
// operands A(i, k) at lane i + 16 k, B(k, j) at lane j + 16 k.
__global__ __launch_bounds__(RNT) void k_gemm_real(RealGemmArgs g) {
    const int TM = (g.M + RBM - 1) / RBM, TN = (g.N + RBN - 1) / RBN;
    int tm, tn;
    real_tile(TM, TN, tm, tn);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int lr = lane & 15, lq = lane >> 4;
    const int rw = tm * RBM + (wave >> 1) * 32, cw = tn * RBN + (wave & 1) * 32;
    const bool full = rw + 32 <= g.M && cw + 32 <= g.N;
    const double* __restrict__ A = g.A;
    const double* __restrict__ B = g.B;
    double* __restrict__ C = g.C;

    v4d acc[2][2];
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        const int col = cw + j * 16 + lr;
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int row = rw + i * 16 + lq + 4 * v;
                acc[i][j][v] = (col < g.N && row < g.M) ? C[(long)col * g.ldc + row] : 0.0;
            }
    }
    // acc -= a b: the negation is the MFMA's source modifier on A
    auto mma = [&](double a0, double a1, double b0, double b1) __attribute__((always_inline)) {
        acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 1);
        acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 1);
        acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 1);
        acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 1);
    };
    const int nks = (g.K + 3) / 4;
    const int ra0 = min(rw + lr, g.M - 1), ra1 = min(rw + 16 + lr, g.M - 1);
    const int cb0 = min(cw + lr, g.N - 1), cb1 = min(cw + 16 + lr, g.N - 1);
    double pa0[RDEPTH], pa1[RDEPTH], pb0[RDEPTH], pb1[RDEPTH];
    if (full && (g.K & 3) == 0 && nks >= RDEPTH) {
        // interior tile: no masking, one running pointer per operand
        const long sA = 4L * g.lda;
        const double* qa0 = A + (long)lq * g.lda + ra0;
        const double* qa1 = qa0 + 16;
        const double* qb0 = B + (long)cb0 * g.ldb + lq;
        const double* qb1 = B + (long)cb1 * g.ldb + lq;
        auto next = [&](double& a0, double& a1, double& b0, double& b1) __attribute__((always_inline)) {
            a0 = *qa0; a1 = *qa1; b0 = *qb0; b1 = *qb1;
            qa0 += sA; qa1 += sA; qb0 += 4; qb1 += 4;
        };
#pragma unroll
        for (int d = 0; d < RDEPTH; ++d) next(pa0[d], pa1[d], pb0[d], pb1[d]);
        int l0 = 0;
        for (; l0 + 2 * RDEPTH <= nks; l0 += RDEPTH) {
#pragma unroll
            for (int d = 0; d < RDEPTH; ++d) {
                mma(pa0[d], pa1[d], pb0[d], pb1[d]);
                __builtin_amdgcn_sched_barrier(0);
                next(pa0[d], pa1[d], pb0[d], pb1[d]);
                __builtin_amdgcn_sched_barrier(0);
            }
        }
#pragma unroll
        for (int d = 0; d < RDEPTH; ++d) {
            mma(pa0[d], pa1[d], pb0[d], pb1[d]);
            if (l0 + d + RDEPTH < nks) next(pa0[d], pa1[d], pb0[d], pb1[d]);
        }
#pragma unroll
        for (int d = 0; d < RDEPTH; ++d)
            if (l0 + RDEPTH + d < nks) mma(pa0[d], pa1[d], pb0[d], pb1[d]);
    } else if (nks > 0) {
        // edge tile: clamped unconditional loads, values outside zeroed at use
        const bool oka0 = rw + lr < g.M, oka1 = rw + 16 + lr < g.M;
        const bool okb0 = cw + lr < g.N, okb1 = cw + 16 + lr < g.N;
        auto load = [&](int ks, double& a0, double& a1, double& b0, double& b1) __attribute__((always_inline)) {
            const int k = min(ks * 4 + lq, g.K - 1);
            const double* ap = A + (long)k * g.lda;
            a0 = ap[ra0];
            a1 = ap[ra1];
            b0 = B[(long)cb0 * g.ldb + k];
            b1 = B[(long)cb1 * g.ldb + k];
        };
        auto use = [&](int ks, double a0, double a1, double b0, double b1) __attribute__((always_inline)) {
            const bool kin = ks * 4 + lq < g.K;
            mma((kin && oka0) ? a0 : 0.0, (kin && oka1) ? a1 : 0.0, (kin && okb0) ? b0 : 0.0,
                (kin && okb1) ? b1 : 0.0);
        };
#pragma unroll
        for (int d = 0; d < RDEPTH; ++d) load(min(d, nks - 1), pa0[d], pa1[d], pb0[d], pb1[d]);
        int l0 = 0;
        for (; l0 + RDEPTH <= nks; l0 += RDEPTH) {
#pragma unroll
            for (int d = 0; d < RDEPTH; ++d) {
                use(l0 + d, pa0[d], pa1[d], pb0[d], pb1[d]);
                __builtin_amdgcn_sched_barrier(0);
                load(min(l0 + d + RDEPTH, nks - 1), pa0[d], pa1[d], pb0[d], pb1[d]);
                __builtin_amdgcn_sched_barrier(0);
            }
        }
#pragma unroll
        for (int d = 0; d < RDEPTH; ++d)
            if (l0 + d < nks) use(l0 + d, pa0[d], pa1[d], pb0[d], pb1[d]);
    }
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        const int col = cw + j * 16 + lr;
        if (col >= g.N) continue;
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int row = rw + i * 16 + lq + 4 * v;
                if (row < g.M) C[(long)col * g.ldc + row] = acc[i][j][v];
            }
    }
}

// Value of lane i (wave-uniform) to every lane.
__device__ inline double readlane_d(double v, int i) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), i);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), i);
    return __hiloint2double(hi, lo);
}

// One diagonal block [i0, i0 + bs) of U for all shifts, in place in B. Lane r
// of each wavefront owns row r (NB = 64); each wavefront solves SPW shifts at
// once. Rows are scaled by their pivot reciprocals first: with
// b'(r) = b(r) / d(r) and u'(r, i) = u(r, i) / d(r), step i is x(i) = b'(i)
// (broadcast) and b'(r) -= u'(r, i) x(i).
template <int NB, int SPW>
__global__ __launch_bounds__(RNT) void k_diag_real(RealDiagArgs a) {
    static_assert(NB == 64, "one row per lane");
    __shared__ double Us[NB * NB];   // Us[i * NB + r] = U(i0 + r, i0 + i) for r < i, else 0
    __shared__ double Ud[NB];
    const int bs = a.bs, i0 = a.i0;
    for (int t = threadIdx.x; t < NB * NB; t += RNT) {
        const int c = t / NB, rr = t - c * NB;
        const double v = (rr <= c && c < bs) ? a.U[(long)(i0 + c) * a.ldu + i0 + rr] : 0.0;
        if (rr == c) Ud[rr] = v;
        Us[t] = (rr < c) ? v : 0.0;
    }
    __syncthreads();
    const int r = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int j0 = (blockIdx.x * (RNT / 64) + wave) * SPW;
    if (j0 >= a.n) return;
    double b[SPW], p[SPW];
    bool jv[SPW];
#pragma unroll
    for (int s = 0; s < SPW; ++s) {
        const int j = j0 + s;
        jv[s] = j < a.n;
        const bool on = jv[s] && r < bs;
        const double d = on ? Ud[r] - a.lam[j] : 1.0;
        p[s] = 1.0 / d;
        b[s] = on ? a.B[(long)j * a.ldb + i0 + r] / d : 0.0;
    }
    double un = Us[(bs - 1) * NB + r];
    for (int i = bs - 1; i >= 0; --i) {
        const double u = un;
        un = Us[(i > 0 ? i - 1 : 0) * NB + r];
#pragma unroll
        for (int s = 0; s < SPW; ++s) {
            const double x = readlane_d(b[s], i);
            b[s] = fma(-(u * p[s]), x, b[s]);
        }
    }
#pragma unroll
    for (int s = 0; s < SPW; ++s)
        if (jv[s] && r < bs) a.B[(long)(j0 + s) * a.ldb + i0 + r] = b[s];
}

}  // namespace

hipError_t launch_gemm_real(const RealGemmArgs& g, hipStream_t s) {
    if (g.M <= 0 || g.N <= 0) return hipSuccess;
    if (g.K < 0) return hipErrorInvalidValue;
    const int TM = (g.M + RBM - 1) / RBM, TN = (g.N + RBN - 1) / RBN;
    hipLaunchKernelGGL(k_gemm_real, dim3(TM * TN), dim3(RNT), 0, s, g);
    return hipGetLastError();
}

hipError_t launch_diag_real(const RealDiagArgs& a, hipStream_t s) {
    constexpr int NB = 64, SPW = 4, per_wg = (RNT / 64) * SPW;
    if (a.bs <= 0 || a.bs > NB || a.n <= 0) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_diag_real<NB, SPW>), dim3((a.n + per_wg - 1) / per_wg), dim3(RNT), 0, s, a);
    return hipGetLastError();
}

}  // namespace mst
