// Diagonal-block step of the blocked multi-shift solve (the xTRSV call inside
// Alg 3 / Alg 5 of Moon & Poulson, arXiv 1607.01477), for gfx950.
//
// One workgroup stages the nb x nb diagonal block of U in LDS once and every
// wavefront of it solves a group of shifts against it: lane r of a group of nb
// lanes owns row r of the block, the pivot U(r,r) - lambda_j is formed on the
// fly, and each of the nb sequential steps broadcasts the new solution entry
// to the group (v_readlane for nb = 64, ds_bpermute otherwise) followed by one
// complex multiply-add per lane. Several shifts are interleaved per wavefront
// to hide the dependency latency of the step chain.
//
// Safe variant: Alg 4 phase 2 (checked back substitution) on the block, then
// the column growth bound and rescaling decision of Alg 5. All scale factors
// are powers of two 2^-k, tracked as integer exponents; rows outside the block
// are rescaled lazily (in the substitution GEMM epilogue and a final pass).
// The fast path of Alg 4 (phase 1) is not used: when it would apply, phase 2
// performs no rescaling and computes the same result.
#include "common.h"

namespace mst {
namespace {

constexpr int kWG = 256;

__device__ inline double cabs1(double re, double im) { return fabs(re) + fabs(im); }

// Smallest k >= 1 with 2^-k q < 2^w, for finite q >= 2^w.
__device__ inline int scale_exp(double q, int w) { return ilogb(q) - (w - 1); }

// g + a*b evaluated without contraction; returns the exponent k that brings
// the sum below Omega = 2^w (0 if already below) and the scaled sum. When the
// sum overflows, k comes from the exponents of the two terms (the sum is
// < 2^(E+1) with E = max(ilogb g, ilogb a + ilogb b + 1) + 1).
__device__ inline int bound_add(double g, double a, double b, int w, double omega, double* out) {
#pragma clang fp contract(off)
    double s = g + a * b;
    if (s < omega) {
        *out = s;
        return 0;
    }
    int k;
    if (isinf(s)) {
        int e1 = (g > 0.0) ? ilogb(g) : -100000;
        int e2 = ilogb(a) + ilogb(b) + 1;
        int E = (e1 > e2 ? e1 : e2) + 1;
        k = E + 1 - w;
        *out = ldexp(g, -k) + ldexp(a, -k) * b;
    } else {
        k = scale_exp(s, w);
        *out = ldexp(s, -k);
    }
    return k;
}

__device__ inline double quotient(double a, double b) {
#pragma clang fp contract(off)
    return a / b;
}

template <int NB>
__device__ inline double bcast(double v, int i, int base) {
    if constexpr (NB == 64) {
        int lo = __builtin_amdgcn_readlane(__double2loint(v), i);
        int hi = __builtin_amdgcn_readlane(__double2hiint(v), i);
        return __hiloint2double(hi, lo);
    } else {
        return __shfl(v, base + i, 64);
    }
}

template <int NB>
__device__ inline double group_max(double v) {
#pragma unroll
    for (int off = NB / 2; off >= 1; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    return v;
}

template <int NB, int SPW, bool ADJ, bool SAFE, bool MIXED, bool VARLEN>
__global__ __launch_bounds__(kWG) void k_diag(DiagArgs a) {
    __shared__ zd Us[NB * NB];
    const int bs = a.bs, i0 = a.i0;
    // Us[i*NB + r]: coefficient of unknown i in row r of the block system
    //   forward: U(i0+r, i0+i) for r <= i;  adjoint: conj(U(i0+i, i0+r)) for r >= i
    // all loads of this thread are issued before any LDS store, so their
    // latencies overlap
    constexpr int PER = (NB * NB) / kWG;
    zd stage[PER];
#pragma unroll
    for (int e = 0; e < PER; ++e) {
        const int t = threadIdx.x + e * kWG;
        const int c = t / NB, rr = t - c * NB;
        stage[e] = zd{0.0, 0.0};
        if (rr <= c && c < bs) stage[e] = a.U[(long)(i0 + c) * a.ldu + i0 + rr];
    }
#pragma unroll
    for (int e = 0; e < PER; ++e) {
        const int t = threadIdx.x + e * kWG;
        const int c = t / NB, rr = t - c * NB;
        if (!ADJ) {
            Us[c * NB + rr] = stage[e];
        } else {
            Us[rr * NB + c] = zd{stage[e].re, -stage[e].im};
        }
    }
    __syncthreads();

    constexpr int G = 64 / NB;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int grp = lane / NB, r = lane - grp * NB, base = grp * NB;
    const int jw = (blockIdx.x * (kWG / 64) + wave) * (G * SPW);
    if (jw >= a.n) return;

    const int w = a.safe.omega_log2;
    const double omega = ldexp(1.0, w);
    const double delta = SAFE ? *a.safe.delta : 0.0;
    const double cn_l = (SAFE && r < bs) ? a.safe.cn_in[i0 + r] : 0.0;

    double br[SPW], bi[SPW], pr[SPW], pi[SPW], cdl[SPW];
    int pe[SPW], jj[SPW], Lr[SPW];
    double Gs[SPW], Ms[SPW];
    int kblk[SPW];
    bool any_active = false;
#pragma unroll
    for (int s = 0; s < SPW; ++s) {
        const int j = jw + s * G + grp;
        jj[s] = j;
        int L = a.m;
        if (VARLEN && j < a.n) {
            L = a.col_len[j];
            L = L < 0 ? 0 : (L > a.m ? a.m : L);
        }
        Lr[s] = (j < a.n) ? L : 0;
        const bool rv = (r < bs) && (i0 + r < Lr[s]);
        any_active |= (j < a.n) && (i0 < Lr[s]);
        double xr = 0.0, xi = 0.0;
        if (rv) {
            if (MIXED) {
                const zf v = a.b32[(long)j * a.ldb32 + i0 + r];
                xr = v.re;
                xi = v.im;
            } else {
                const zd v = a.B[(long)j * a.ldb + i0 + r];
                xr = v.re;
                xi = v.im;
            }
        }
        br[s] = xr;
        bi[s] = xi;
        // pivot d = U(r,r) - lambda (forward) or its conjugate (adjoint)
        double dr = 1.0, di = 0.0;
        if (r < bs && j < a.n) {
            const zd l = a.lam[j];
            const zd u = Us[r * NB + r];
            dr = u.re - l.re;
            di = ADJ ? (u.im + l.im) : (u.im - l.im);
            if (SAFE && dr == 0.0 && di == 0.0) dr = delta;
        }
        cdl[s] = cabs1(dr, di);
        // scaled reciprocal: d = 2^e d', 1/d = 2^-e conj(d')/|d'|^2
        const double am = fmax(fabs(dr), fabs(di));
        const int e = (am > 0.0) ? ilogb(am) : 0;
        const double sr = ldexp(dr, -e), si = ldexp(di, -e);
        const double den = sr * sr + si * si;
        if (SAFE) {
            pr[s] = sr / den;
            pi[s] = -si / den;
            pe[s] = e;
        } else {
            // plain solve: 1/d itself (overflows only for |d| < 2^-1022, a
            // singular system for this solver)
            pr[s] = ldexp(sr / den, -e);
            pi[s] = ldexp(-si / den, -e);
            pe[s] = 0;
        }
        kblk[s] = 0;
        Ms[s] = 0.0;
        Gs[s] = 0.0;
    }

    if (SAFE && VARLEN) {
        // every shift of this wavefront has all its rows above the block: nothing
        // to solve; the exponent record of the block is the current exponent
        if (!__any(any_active)) {
#pragma unroll
            for (int s = 0; s < SPW; ++s) {
                const int j = jj[s];
                if (r == 0 && j < a.n) a.safe.kb[(long)a.q * a.n + j] = a.safe.kcur[j];
            }
            return;
        }
    }
    if (SAFE) {
#pragma unroll
        for (int s = 0; s < SPW; ++s) Gs[s] = group_max<NB>(cabs1(br[s], bi[s]));
    }

    auto step = [&](int i) {
        const zd u = Us[i * NB + r];
        const double cni = SAFE ? bcast<NB>(cn_l, i, base) : 0.0;
#pragma unroll
        for (int s = 0; s < SPW; ++s) {
            if (SAFE) {
                const double cb = bcast<NB>(cabs1(br[s], bi[s]), i, base);
                const double cd = bcast<NB>(cdl[s], i, base);
                double M = quotient(cb, cd);
                if (M >= omega) {
                    const bool ov = isinf(M);
                    const int kk = ov ? (ilogb(cb) - ilogb(cd) - (w - 1)) : scale_exp(M, w);
                    br[s] = ldexp(br[s], -kk);
                    bi[s] = ldexp(bi[s], -kk);
                    kblk[s] += kk;
                    Gs[s] = ldexp(Gs[s], -kk);
                    if (ov) {
                        M = quotient(bcast<NB>(cabs1(br[s], bi[s]), i, base), cd);
                    } else {
                        M = ldexp(M, -kk);
                    }
                }
                Ms[s] = M;
            }
            double xl_r = br[s] * pr[s] - bi[s] * pi[s];
            double xl_i = br[s] * pi[s] + bi[s] * pr[s];
            if (SAFE) {
                xl_r = ldexp(xl_r, -pe[s]);
                xl_i = ldexp(xl_i, -pe[s]);
            }
            double xr = bcast<NB>(xl_r, i, base);
            double xi = bcast<NB>(xl_i, i, base);
            if (SAFE) {
                double Gn;
                const int kk = bound_add(Gs[s], Ms[s], cni, w, omega, &Gn);
                if (kk > 0) {
                    br[s] = ldexp(br[s], -kk);
                    bi[s] = ldexp(bi[s], -kk);
                    xr = ldexp(xr, -kk);
                    xi = ldexp(xi, -kk);
                    kblk[s] += kk;
                }
                Gs[s] = Gn;
            }
            const double nr = br[s] - (u.re * xr - u.im * xi);
            const double ni = bi[s] - (u.re * xi + u.im * xr);
            const bool upd = ADJ ? (r > i) : (r < i);
            br[s] = upd ? nr : (r == i ? xr : br[s]);
            bi[s] = upd ? ni : (r == i ? xi : bi[s]);
        }
    };
    if (!ADJ) {
        for (int i = bs - 1; i >= 0; --i) step(i);
    } else {
        for (int i = 0; i < bs; ++i) step(i);
    }

    if (SAFE) {
        const double asum = a.safe.above_sum[a.q];
#pragma unroll
        for (int s = 0; s < SPW; ++s) {
            const int j = jj[s];
            const double xn = group_max<NB>(cabs1(br[s], bi[s]));
            if (j >= a.n) continue;
            if (i0 >= Lr[s]) {
                // the block lies below the column's rows: skipped, state unchanged
                if (r == 0) a.safe.kb[(long)a.q * a.n + j] = a.safe.kcur[j];
                continue;
            }
            double Gj = ldexp(a.safe.G[j], -kblk[s]);
            double Gn;
            const int k2 = bound_add(Gj, asum, xn, w, omega, &Gn);
            if (k2 > 0) {
                br[s] = ldexp(br[s], -k2);
                bi[s] = ldexp(bi[s], -k2);
            }
            if (r == 0) {
                const int kc = a.safe.kcur[j] + kblk[s] + k2;
                a.safe.G[j] = Gn;
                a.safe.kcur[j] = kc;
                a.safe.kb[(long)a.q * a.n + j] = kc;
            }
        }
    }
#pragma unroll
    for (int s = 0; s < SPW; ++s) {
        const int j = jj[s];
        if (j < a.n && r < bs && i0 + r < Lr[s]) {
            a.B[(long)j * a.ldb + i0 + r] = zd{br[s], bi[s]};
            if (MIXED) a.b32[(long)j * a.ldb32 + i0 + r] = zf{(float)br[s], (float)bi[s]};
        }
    }
}

template <int NB, int SPW, bool ADJ>
hipError_t launch_nb(const DiagArgs& a, hipStream_t s) {
    constexpr int per_wg = (kWG / 64) * (64 / NB) * SPW;
    const dim3 grid((a.n + per_wg - 1) / per_wg);
    const bool safe = a.use_safe != 0;
    const bool mixed = a.b32 != nullptr;
    const bool varlen = a.col_len != nullptr;
    if (ADJ) {
        if (safe || mixed || varlen) return hipErrorInvalidValue;
        hipLaunchKernelGGL((k_diag<NB, SPW, true, false, false, false>), grid, dim3(kWG), 0, s, a);
    } else if (safe) {
        if (mixed) return hipErrorInvalidValue;
        if (varlen)
            hipLaunchKernelGGL((k_diag<NB, SPW, false, true, false, true>), grid, dim3(kWG), 0, s, a);
        else
            hipLaunchKernelGGL((k_diag<NB, SPW, false, true, false, false>), grid, dim3(kWG), 0, s, a);
    } else {
        if (varlen) return hipErrorInvalidValue;
        if (mixed)
            hipLaunchKernelGGL((k_diag<NB, SPW, false, false, true, false>), grid, dim3(kWG), 0, s, a);
        else
            hipLaunchKernelGGL((k_diag<NB, SPW, false, false, false, false>), grid, dim3(kWG), 0, s, a);
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_diag(int nb, bool adjoint, const DiagArgs& a, hipStream_t s) {
    if (a.bs <= 0 || a.bs > nb || a.n <= 0) return hipErrorInvalidValue;
    switch (nb) {
        case 64: return adjoint ? launch_nb<64, 4, true>(a, s) : launch_nb<64, 4, false>(a, s);
        case 32: return adjoint ? launch_nb<32, 2, true>(a, s) : launch_nb<32, 2, false>(a, s);
        case 16: return adjoint ? launch_nb<16, 1, true>(a, s) : launch_nb<16, 1, false>(a, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace mst
