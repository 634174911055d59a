// Diagonal-block step of the blocked multi-shift solve (the xTRSV call inside
// Alg 3 / Alg 5 of Moon & Poulson, arXiv 1607.01477), for gfx950.
//
// Back substitution on one nb x nb diagonal block: a workgroup stages the block
// of U in LDS once and every wavefront solves a group of shifts against it.
// Lane r of a group of nb lanes owns row r of the block, the pivot
// U(r,r) - lambda_j is formed on the fly, and each of the nb sequential steps
// broadcasts the new solution entry to the group (v_readlane, or DPP
// row_newbcast for nb = 16) followed by one complex multiply-add per lane (the
// staged block is zero outside the rows a step updates, so no lane masking).
// Several shifts are interleaved per wavefront to hide the step latency.
//
// Safe variant: Alg 4 phase 2 (checked back substitution) on the block, then
// the column growth bound and rescaling decision of Alg 5. Scale factors are
// powers of two 2^-k tracked as integer exponents; rows outside the block are
// rescaled lazily (by the consumer of the block and a final pass). The fast
// path of Alg 4 (phase 1) is not used: where it applies, phase 2 performs no
// rescaling and computes the same result.
//
// Two kernels use this step:
//   k_diag  - one diagonal block for all shifts (the paper's loop order);
//   k_block - a whole outer block of up to 256 rows for 16 shifts per
//             workgroup of 8 wavefronts: the right-hand sides of the outer
//             block stay in LDS,
//             each diagonal block is solved as above and the rows of the
//             outer block still to be solved are updated right away with
//             FP64 MFMA products (U panel from L2, solution from LDS). This
//             fuses nb-row diagonal solves and their short substitution GEMMs
//             into one launch per outer block.
#include "common.h"


namespace mst {
namespace {

constexpr int kWG = 256;

typedef double v4d __attribute__((ext_vector_type(4)));

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

// g + a*b without contraction (the growth bound when it stays below Omega)
__device__ inline double bound_sum(double g, double a, double b) {
#pragma clang fp contract(off)
    return g + a * b;
}

__device__ inline double quotient(double a, double b) {
#pragma clang fp contract(off)
    return a / b;
}

// Entry u - lambda v of the shifted pencil, every operation rounded on its own
// (the xAXPY that forms U' in Alg 8 / Alg 9).
__device__ inline zd pencil(zd u, zd v, zd l) {
#pragma clang fp contract(off)
    return zd{u.re - (l.re * v.re - l.im * v.im), u.im - (l.re * v.im + l.im * v.re)};
}

// Column-bound increment of Alg 9 for one shift: sum_k ||U(I0,k)||_inf +
// |lambda| sum_k ||V(I0,k)||_inf, with |lambda| taken as cabs1.
__device__ inline double pencil_asum(double au, double av, zd l) {
#pragma clang fp contract(off)
    return au + (fabs(l.re) + fabs(l.im)) * av;
}

// Value of lane i of each group of NB lanes, to every lane of that group.
//   NB = 64: v_readlane into scalar registers (measured faster than a pair of
//            readlanes plus a select for NB = 32, which uses ds_bpermute);
//   NB = 16: DPP row_newbcast (one VALU move per 32-bit word) — needs i as an
//            immediate, see bcast16 and BlockSolve::run.
template <int NB>
__device__ inline double bcast(double v, int i, int base) {
    const int lo = __double2loint(v), hi = __double2hiint(v);
    if constexpr (NB == 64) {
        return __hiloint2double(__builtin_amdgcn_readlane(hi, i), __builtin_amdgcn_readlane(lo, i));
    } else {
        return __shfl(v, base + i, 64);
    }
}

// 64-bit DPP moves: one v_mov_b64_dpp each (gfx950's DP ALU takes DPP64 with
// row_newbcast). Plain functions with literal controls: inside a template the
// builtin's result type is not resolved to its 64-bit operand's (it reads as
// int), so the template below only dispatches.
#define MST_BCAST64_FN(I, CTL)                                                           \
    __device__ inline double bcast64_##I(double v) {                                     \
        const long r = __builtin_amdgcn_mov_dpp(__builtin_bit_cast(long, v), CTL, 0xF, 0xF, false); \
        return __builtin_bit_cast(double, r);                                            \
    }
MST_BCAST64_FN(0, 0x150)
MST_BCAST64_FN(1, 0x151)
MST_BCAST64_FN(2, 0x152)
MST_BCAST64_FN(3, 0x153)
MST_BCAST64_FN(4, 0x154)
MST_BCAST64_FN(5, 0x155)
MST_BCAST64_FN(6, 0x156)
MST_BCAST64_FN(7, 0x157)
MST_BCAST64_FN(8, 0x158)
MST_BCAST64_FN(9, 0x159)
MST_BCAST64_FN(10, 0x15A)
MST_BCAST64_FN(11, 0x15B)
MST_BCAST64_FN(12, 0x15C)
MST_BCAST64_FN(13, 0x15D)
MST_BCAST64_FN(14, 0x15E)
MST_BCAST64_FN(15, 0x15F)
#undef MST_BCAST64_FN

// Value of lane I of each row of 16 lanes, to every lane of that row
// (DPP row_newbcast writes every lane, so no previous value is needed).
template <int I>
__device__ inline double bcast16(double v) {
    static_assert(I >= 0 && I < 16, "lane of a row");
    if constexpr (I == 0) return bcast64_0(v);
    else if constexpr (I == 1) return bcast64_1(v);
    else if constexpr (I == 2) return bcast64_2(v);
    else if constexpr (I == 3) return bcast64_3(v);
    else if constexpr (I == 4) return bcast64_4(v);
    else if constexpr (I == 5) return bcast64_5(v);
    else if constexpr (I == 6) return bcast64_6(v);
    else if constexpr (I == 7) return bcast64_7(v);
    else if constexpr (I == 8) return bcast64_8(v);
    else if constexpr (I == 9) return bcast64_9(v);
    else if constexpr (I == 10) return bcast64_10(v);
    else if constexpr (I == 11) return bcast64_11(v);
    else if constexpr (I == 12) return bcast64_12(v);
    else if constexpr (I == 13) return bcast64_13(v);
    else if constexpr (I == 14) return bcast64_14(v);
    else return bcast64_15(v);
}
template <int I>
__device__ inline double bcast16m(double v) {
    return bcast16<I>(v);
}

template <int NB>
__device__ inline double group_max(double v) {
#pragma unroll
    for (int off = NB / 2; off >= 1; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    return v;
}

// Us[i*NB + r]: coefficient of unknown i in row r of the block system E, zero
// on and outside the triangle that the substitution uses (E = op(A) of the
// variant EV, see ev_fwd / ev_tr / ev_cj):
//   back substitution (E upper): E(i0+r, i0+i) for r < i;
//   forward substitution (E lower): E(i0+r, i0+i) for r > i;
// with E(r, c) = A(r, c), A(c, r) (transposed) or conj(A(c, r)).
// Ud[r]: the diagonal of E. The element pair (rr <= c) of the loop below is
// read from A's upper triangle, A(rr, c), when A is upper triangular and from
// its lower triangle, A(c, rr), when A is lower (EV transposes exactly when the
// substitution direction differs from A's triangle).
// All loads of a thread are issued before its LDS stores so their latencies overlap.
template <int NB, int EV>
__device__ inline void stage_diag(zd* Us, zd* Ud, const zd* U, long ldu, int i0, int bs) {
    constexpr bool FWD = ev_fwd(EV), CJ = ev_cj(EV), LOWA = ev_lower_a(EV);
    constexpr int PER = (NB * NB) / kWG;
    zd st[PER];
#pragma unroll
    for (int e = 0; e < PER; ++e) {
        const int t = threadIdx.x + e * kWG;
        const int c = t / NB, rr = t - c * NB;
        st[e] = zd{0.0, 0.0};
        if (rr <= c && c < bs)
            st[e] = LOWA ? U[(long)(i0 + rr) * ldu + i0 + c] : U[(long)(i0 + c) * ldu + i0 + rr];
    }
#pragma unroll
    for (int e = 0; e < PER; ++e) {
        const int t = threadIdx.x + e * kWG;
        const int c = t / NB, rr = t - c * NB;
        const zd v = CJ ? zd{st[e].re, -st[e].im} : st[e];
        if (rr == c) {
            Ud[rr] = v;
            Us[c * NB + rr] = zd{0.0, 0.0};
        } else if (!FWD) {
            Us[c * NB + rr] = v;
        } else {
            Us[rr * NB + c] = v;
        }
    }
}

// Per-wavefront solve of SPW interleaved shifts (per group of NB lanes) against
// the staged block. b holds the right-hand side rows (lane r = row r) and
// receives the solution; kblk the block's scale exponent (safe variant).
// GEN: the block of a pencil, U' = U - lambda V per shift (nb = 16, one shift
// per lane group): pivots and coefficients are formed from both staged blocks.
template <int NB, int SPW, int EV, bool SAFE, bool GEN = false>
struct BlockSolve {
    static_assert(!GEN || (NB == 16 && SPW == 1 && EV == 0), "pencil blocks: nb 16, upper, op N");
    static constexpr bool ADJ = ev_fwd(EV);   // forward substitution (E lower triangular)
    static constexpr bool CJ = ev_cj(EV);
    double br[SPW], bi[SPW], pr[SPW], pi[SPW], cdl[SPW], Gs[SPW], Ms[SPW];
    int pe[SPW], kblk[SPW];

    // The pivot of one row d = dr + i di (1 + 0i outside the block): cabs1(d)
    // and its scaled reciprocal (safe: 1/d = 2^-e (pr + i pi); plain: pr + i pi
    // = 1/d, e = 0).
    static __device__ __forceinline__ void pivot_entry(double dr, double di, double& pr_, double& pi_,
                                                       int& pe_, double& cd_) {
        cd_ = cabs1(dr, di);
        // scaled reciprocal: d = 2^e d', 1/d = 2^-e conj(d')/|d'|^2
        const double am = fmax(fabs(dr), fabs(di));
        const int e = (am > 0.0) ? ilogb(am) : 0;
        const double sr = ldexp(dr, -e), si = ldexp(di, -e);
        const double den = sr * sr + si * si;
        if (SAFE) {
            pr_ = sr / den;
            pi_ = -si / den;
            pe_ = e;
        } else {
            // plain solve: 1/d itself (overflows only for |d| < 2^-1022, a
            // singular system for this solver)
            pr_ = ldexp(sr / den, -e);
            pi_ = ldexp(-si / den, -e);
            pe_ = 0;
        }
    }

    // pivot d = U(r,r) - lambda (forward) or its conjugate (adjoint); exact
    // zeros replaced by delta in the safe variant
    // (GEN: d = U(r,r) - lambda V(r,r), V's diagonal in Vd)
    static __device__ __forceinline__ void pivot_value(zd u, zd l, double delta, double& dr, double& di,
                                                       const zd* vd = nullptr) {
        if constexpr (GEN) {
            const zd d = pencil(u, *vd, l);
            dr = d.re;
            di = d.im;
        } else {
            dr = u.re - l.re;
            di = CJ ? (u.im + l.im) : (u.im - l.im);
        }
        if (SAFE && dr == 0.0 && di == 0.0) dr = delta;
    }

    __device__ __forceinline__ void pivots(const zd* Ud, int r, int bs, const zd (&lam)[SPW],
                                           const bool (&jv)[SPW], double delta,
                                           const zd* Vd = nullptr) {
#pragma unroll
        for (int s = 0; s < SPW; ++s) {
            double dr = 1.0, di = 0.0;
            if (r < bs && jv[s]) pivot_value(Ud[r], lam[s], delta, dr, di, GEN ? Vd + r : nullptr);
            pivot_entry(dr, di, pr[s], pi[s], pe[s], cdl[s]);
        }
        reset();
    }

    // the pivots from values formed beforehand (pivot_entry)
    __device__ __forceinline__ void pivots_given(const double (&pr_)[SPW], const double (&pi_)[SPW],
                                                 const int (&pe_)[SPW], const double (&cd_)[SPW]) {
#pragma unroll
        for (int s = 0; s < SPW; ++s) {
            pr[s] = pr_[s];
            pi[s] = pi_[s];
            pe[s] = pe_[s];
            cdl[s] = cd_[s];
        }
        reset();
    }

    __device__ __forceinline__ void reset() {
#pragma unroll
        for (int s = 0; s < SPW; ++s) {
            kblk[s] = 0;
            Ms[s] = 0.0;
            Gs[s] = 0.0;
        }
        if (SAFE) {
#pragma unroll
            for (int s = 0; s < SPW; ++s) Gs[s] = group_max<NB>(cabs1(br[s], bi[s]));
        }
    }

    // u: coefficient of unknown i in this lane's row (zero outside the rows the step updates)
    template <typename BC>
    __device__ __forceinline__ void step(const zd u, int i, int r, double cn_l, int w,
                                         double omega, BC bc) {
        const double cni = SAFE ? bc(cn_l) : 0.0;
#pragma unroll
        for (int s = 0; s < SPW; ++s) {
            if (SAFE) {
                const double cb = bc(cabs1(br[s], bi[s]));
                const double cd = bc(cdl[s]);
                double M = quotient(cb, cd);
                if (M >= omega) {
                    const bool ov = isinf(M);
                    const int kk = ov ? (ilogb(cb) - ilogb(cd) - (w - 1)) : scale_exp(M, w);
                    br[s] = ldexp(br[s], -kk);
                    bi[s] = ldexp(bi[s], -kk);
                    kblk[s] += kk;
                    Gs[s] = ldexp(Gs[s], -kk);
                    if (ov) {
                        M = quotient(bc(cabs1(br[s], bi[s])), cd);
                    } else {
                        M = ldexp(M, -kk);
                    }
                }
                Ms[s] = M;
            }
            // every lane forms its own quotient b_r / d_r; lane i's is x_i
            double xl_r = fma(br[s], pr[s], -bi[s] * pi[s]);
            double xl_i = fma(br[s], pi[s], bi[s] * pr[s]);
            if (SAFE) {
                xl_r = ldexp(xl_r, -pe[s]);
                xl_i = ldexp(xl_i, -pe[s]);
            }
            double xr = bc(xl_r);
            double xi = bc(xl_i);
            if (SAFE) {
                double Gn;
                const int kk = bound_add(Gs[s], Ms[s], cni, w, omega, &Gn);
                if (kk > 0) {
                    br[s] = ldexp(br[s], -kk);
                    bi[s] = ldexp(bi[s], -kk);
                    xl_r = ldexp(xl_r, -kk);
                    xl_i = ldexp(xl_i, -kk);
                    xr = ldexp(xr, -kk);
                    xi = ldexp(xi, -kk);
                    kblk[s] += kk;
                }
                Gs[s] = Gn;
            }
            // u is zero outside the rows still to be updated (and on the pivot row)
            const double nr = fma(-u.re, xr, fma(u.im, xi, br[s]));
            const double ni = fma(-u.re, xi, fma(-u.im, xr, bi[s]));
            br[s] = (r == i) ? xl_r : nr;
            bi[s] = (r == i) ? xl_i : ni;
        }
    }

    // Safe step without its rescaling branches: the quotient M = |b_i|/|d_i|
    // and the bound G + M c_i of Alg 4 are evaluated beside the substitution
    // chain instead of gating it, and a step that would rescale (or meet a
    // non-finite value) raises flag. Where nothing rescales, every value equals
    // the checked step's; the caller redoes the block with the checked steps
    // when any flag is up.
    template <typename BC>
    __device__ __forceinline__ void step_spec(const zd u, int i, int r, double cn_l, double omega,
                                              BC bc, bool& flag) {
        const double cni = bc(cn_l);
#pragma unroll
        for (int s = 0; s < SPW; ++s) {
            const double cb = bc(cabs1(br[s], bi[s]));
            const double cd = bc(cdl[s]);
            double xl_r = fma(br[s], pr[s], -bi[s] * pi[s]);
            double xl_i = fma(br[s], pi[s], bi[s] * pr[s]);
            xl_r = ldexp(xl_r, -pe[s]);
            xl_i = ldexp(xl_i, -pe[s]);
            const double xr = bc(xl_r), xi = bc(xl_i);
            const double M = quotient(cb, cd);
            const double Gn = bound_sum(Gs[s], M, cni);
            flag = flag || !(M < omega) || !(Gn < omega);
            Gs[s] = Gn;
            const double nr = fma(-u.re, xr, fma(u.im, xi, br[s]));
            const double ni = fma(-u.re, xi, fma(-u.im, xr, bi[s]));
            br[s] = (r == i) ? xl_r : nr;
            bi[s] = (r == i) ? xl_i : ni;
        }
    }

    template <int I>
    __device__ __forceinline__ void run16spec(const zd (&uu)[16], int bs, int r, double cn_l,
                                              double omega, bool& flag) {
        constexpr int STEP = ADJ ? I : 15 - I;
        if (STEP < bs)
            step_spec(uu[STEP], STEP, r, cn_l, omega, [](double v) { return bcast16<STEP>(v); }, flag);
        if constexpr (I < 15) run16spec<I + 1>(uu, bs, r, cn_l, omega, flag);
    }

    template <int I>
    __device__ __forceinline__ void run16(const zd (&uu)[16], int bs, int r, double cn_l, int w,
                                          double omega) {
        // steps with compile-time lane index (DPP immediates): 15..0 forward, 0..15 adjoint
        constexpr int STEP = ADJ ? I : 15 - I;
        if (STEP < bs) step(uu[STEP], STEP, r, cn_l, w, omega, [](double v) { return bcast16<STEP>(v); });
        if constexpr (I < 15) run16<I + 1>(uu, bs, r, cn_l, w, omega);
    }

    // Plain solve, nb = 16, rows scaled by their pivot reciprocals first:
    // with b'(r) = b(r)/d(r) and u'(r,i) = u(r,i)/d(r) the substitution is
    // x(i) = b'(i), b'(r) -= u'(r,i) x(i) — the same quotients, computed off the
    // dependent chain, which is then one broadcast and one complex
    // multiply-add per step. Lane i keeps x(i) unchanged (u'(i,i) = 0), and
    // steps past a partial block move zeros (b = 0 there, u = 0), so all 16
    // steps run unconditionally.
    template <int I>
    __device__ __forceinline__ void run16s(const zd (&uu)[16]) {
        constexpr int STEP = ADJ ? I : 15 - I;
#pragma unroll
        for (int s = 0; s < SPW; ++s) {
            const double xr = bcast16m<STEP>(br[s]), xi = bcast16m<STEP>(bi[s]);
            br[s] = fma(-uu[STEP].re, xr, fma(uu[STEP].im, xi, br[s]));
            bi[s] = fma(-uu[STEP].re, xi, fma(-uu[STEP].im, xr, bi[s]));
        }
        if constexpr (I < 15) run16s<I + 1>(uu);
    }

    // The coefficients come from LDS ahead of the dependent chain of steps:
    // all nb of them for nb = 16, one step ahead otherwise. GEN: coefficient
    // U(r,i) - lambda V(r,i) from the two staged blocks (Vs, shift lg), and in
    // the safe form the column norms of the shifted block (Alg 4 on U') are
    // formed here per shift instead of taken from cn_l.
    // force (safe form): skip the speculative pass and run the checked steps
    // of Alg 4 directly (the results are the same; kept to test that claim)
    __device__ __forceinline__ void run(const zd* Us, int bs, int r, int base, double cn_l, int w,
                                        double omega, const zd* Vs = nullptr, zd lg = zd{0.0, 0.0},
                                        bool force = false) {
        auto coef = [&](int i) __attribute__((always_inline)) {
            if constexpr (GEN) return pencil(Us[i * NB + r], Vs[i * NB + r], lg);
            else return Us[i * NB + r];
        };
        if constexpr (NB == 16 && !SAFE && SPW == 1) {
            zd uu[16];
#pragma unroll
            for (int i = 0; i < 16; ++i) uu[i] = coef(i);
            // b' = b / d, u' = u / d (pr, pi: 1 / d of this lane's row)
            const double b_r = br[0], b_i = bi[0];
            br[0] = fma(b_r, pr[0], -b_i * pi[0]);
            bi[0] = fma(b_r, pi[0], b_i * pr[0]);
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                const double u_r = uu[i].re, u_i = uu[i].im;
                uu[i].re = fma(u_r, pr[0], -u_i * pi[0]);
                uu[i].im = fma(u_r, pi[0], u_i * pr[0]);
            }
            run16s<0>(uu);
        } else if constexpr (NB == 16) {
            if constexpr (GEN && SAFE) {
                // lane r: max cabs1 of column r of U' above the diagonal (the
                // staged blocks are zero on and below it)
                double cn = 0.0;
#pragma unroll
                for (int i = 0; i < 15; ++i) {
                    const zd e = pencil(Us[r * NB + i], Vs[r * NB + i], lg);
                    cn = fmax(cn, cabs1(e.re, e.im));
                }
                cn_l = cn;
            }
            zd uu[16];
#pragma unroll
            for (int i = 0; i < 16; ++i) uu[i] = coef(i);
            // keep the loads here: left alone the compiler sinks each into its
            // step's branch and every step then waits for LDS
#pragma unroll
            for (int i = 0; i < 16; ++i) asm volatile("" : "+v"(uu[i].re), "+v"(uu[i].im));
            if constexpr (SAFE) {
                // speculative pass first; the checked steps only when some
                // step of some shift in the wavefront would rescale
                double b0r[SPW], b0i[SPW], G0[SPW];
#pragma unroll
                for (int s = 0; s < SPW; ++s) {
                    b0r[s] = br[s];
                    b0i[s] = bi[s];
                    G0[s] = Gs[s];
                }
                bool flag = force;
                if (!force) run16spec<0>(uu, bs, r, cn_l, omega, flag);
                if (__any(flag)) {
#pragma unroll
                    for (int s = 0; s < SPW; ++s) {
                        br[s] = b0r[s];
                        bi[s] = b0i[s];
                        Gs[s] = G0[s];
                    }
                    run16<0>(uu, bs, r, cn_l, w, omega);
                }
            } else {
                run16<0>(uu, bs, r, cn_l, w, omega);
            }
        } else if (!ADJ) {
            bool redo = true;
            double b0r[SPW], b0i[SPW], G0[SPW];
            if constexpr (SAFE) {
                // speculative pass, as for nb = 16
#pragma unroll
                for (int s = 0; s < SPW; ++s) {
                    b0r[s] = br[s];
                    b0i[s] = bi[s];
                    G0[s] = Gs[s];
                }
                bool flag = force;
                if (!force) {
                    zd un = Us[(bs - 1) * NB + r];
                    for (int i = bs - 1; i >= 0; --i) {
                        const zd u = un;
                        un = Us[(i > 0 ? i - 1 : 0) * NB + r];
                        step_spec(u, i, r, cn_l, omega, [&](double v) { return bcast<NB>(v, i, base); }, flag);
                    }
                }
                redo = __any(flag);
                if (redo) {
#pragma unroll
                    for (int s = 0; s < SPW; ++s) {
                        br[s] = b0r[s];
                        bi[s] = b0i[s];
                        Gs[s] = G0[s];
                    }
                }
            }
            if (redo) {
                zd un = Us[(bs - 1) * NB + r];
                for (int i = bs - 1; i >= 0; --i) {
                    const zd u = un;
                    un = Us[(i > 0 ? i - 1 : 0) * NB + r];
                    step(u, i, r, cn_l, w, omega, [&](double v) { return bcast<NB>(v, i, base); });
                }
            }
        } else {
            zd un = Us[r];
            for (int i = 0; i < bs; ++i) {
                const zd u = un;
                un = Us[(i + 1 < bs ? i + 1 : i) * NB + r];
                step(u, i, r, cn_l, w, omega, [&](double v) { return bcast<NB>(v, i, base); });
            }
        }
    }

    // Column bound of Alg 5 for slot s after the block: G(j) = 2^-kblk G(j) +
    // above_sum * max cabs1 x; rescale when it reaches Omega. Returns the total
    // exponent change of the column in this block. All lanes of the group call it.
    __device__ __forceinline__ int column_bound(int s, bool active, double asum, double* G, int w,
                                                double omega) {
        const double xn = group_max<NB>(cabs1(br[s], bi[s]));
        if (!active) return 0;
        double Gn;
        const int k2 = bound_add(ldexp(*G, -kblk[s]), asum, xn, w, omega, &Gn);
        if (k2 > 0) {
            br[s] = ldexp(br[s], -k2);
            bi[s] = ldexp(bi[s], -k2);
        }
        Gs[s] = Gn;   // new G(j), returned to the caller through Gs
        return kblk[s] + k2;
    }
};

template <int NB, int SPW, int EV, bool SAFE, bool MIXED, bool VARLEN, bool GEN = false>
__global__ __launch_bounds__(kWG) void k_diag(DiagArgs a) {
    static_assert(!GEN || (NB == 16 && EV == 0 && !MIXED), "pencil: nb 16, upper, op N, FP64");
    if (MIXED && a.skip && *a.skip) return;   // refinement stopped
    __shared__ zd Us[NB * NB];
    __shared__ zd Ud[NB];
    __shared__ zd Vs[GEN ? NB * NB : 1];
    __shared__ zd Vd[GEN ? NB : 1];
    const int bs = a.bs, i0 = a.i0;
    stage_diag<NB, EV>(Us, Ud, a.U, a.ldu, i0, bs);
    if (GEN) stage_diag<NB, 0>(Vs, Vd, a.V, a.ldv, i0, bs);
    __syncthreads();

    constexpr int G = 64 / NB;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int grp = lane / NB, r = lane - grp * NB, base = grp * NB;
    const int jw = (blockIdx.x * (kWG / 64) + wave) * (G * SPW);
    if (jw >= a.n) return;

    const int w = a.safe.omega_log2;
    const double omega = ldexp(1.0, w);
    const double delta = SAFE ? (GEN ? fmax(*a.safe.delta, *a.safe.delta_v) : *a.safe.delta) : 0.0;
    const double cn_l = (SAFE && !GEN && r < bs) ? a.safe.cn_in[i0 + r] : 0.0;

    BlockSolve<NB, SPW, EV, SAFE, GEN> S;
    int jj[SPW], Lr[SPW];
    zd lam[SPW];
    bool jv[SPW];
    bool any_active = false;
#pragma unroll
    for (int s = 0; s < SPW; ++s) {
        const int j = jw + s * G + grp;
        jj[s] = j;
        jv[s] = j < a.n;
        int L = a.m;
        if (VARLEN && jv[s]) {
            L = a.col_len[j];
            L = L < 0 ? 0 : (L > a.m ? a.m : L);
        }
        Lr[s] = jv[s] ? L : 0;
        lam[s] = jv[s] ? a.lam[j] : zd{0.0, 0.0};
        any_active |= jv[s] && (i0 < Lr[s]);
        double xr = 0.0, xi = 0.0;
        if (r < bs && i0 + r < Lr[s]) {
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
        S.br[s] = xr;
        S.bi[s] = xi;
    }
    if (SAFE && VARLEN && !__any(any_active)) {
        // every shift of this wavefront has all its rows above the block:
        // nothing to solve; the exponent record of the block is the current one
#pragma unroll
        for (int s = 0; s < SPW; ++s)
            if (r == 0 && jv[s]) a.safe.kb[(long)a.q * a.n + jj[s]] = a.safe.kcur[jj[s]];
        return;
    }
    S.pivots(Ud, r, bs, lam, jv, delta, Vd);
    S.run(Us, bs, r, base, cn_l, w, omega, Vs, lam[0], SAFE && a.safe.force_checked);

    if (SAFE) {
        const double asum0 = a.safe.above_sum[a.q];
        const double asumv = GEN ? a.safe.above_sum_v[a.q] : 0.0;
#pragma unroll
        for (int s = 0; s < SPW; ++s) {
            const int j = jj[s];
            const bool active = jv[s] && (i0 < Lr[s]);
            double Gj = jv[s] ? a.safe.G[j] : 0.0;
            const double asum = GEN ? pencil_asum(asum0, asumv, lam[s]) : asum0;
            const int dk = S.column_bound(s, active, asum, &Gj, w, omega);
            if (r == 0 && jv[s]) {
                const int kc = a.safe.kcur[j] + dk;
                if (active) {
                    a.safe.G[j] = S.Gs[s];
                    a.safe.kcur[j] = kc;
                }
                a.safe.kb[(long)a.q * a.n + j] = kc;
            }
        }
    }
#pragma unroll
    for (int s = 0; s < SPW; ++s) {
        const int j = jj[s];
        if (jv[s] && r < bs && i0 + r < Lr[s]) {
            a.B[(long)j * a.ldb + i0 + r] = zd{S.br[s], S.bi[s]};
            if (MIXED) a.b32[(long)j * a.ldb32 + i0 + r] = zf{(float)S.br[s], (float)S.bi[s]};
        }
    }
}

// b(r) -= sum_k uo(k) x(k) for nb = 16, x(k) held by lane k of each 16-lane
// group (DPP broadcast); two partial sums per shift
template <int SPW, int K>
__device__ __forceinline__ void couple16(const zd (&uo)[16], const double (&xr)[SPW],
                                         const double (&xi)[SPW], double (&ar)[SPW][2],
                                         double (&ai)[SPW][2]) {
#pragma unroll
    for (int s = 0; s < SPW; ++s) {
        const double yr = bcast16<K>(xr[s]), yi = bcast16<K>(xi[s]);
        ar[s][K & 1] = fma(uo[K].re, yr, fma(-uo[K].im, yi, ar[s][K & 1]));
        ai[s][K & 1] = fma(uo[K].re, yi, fma(uo[K].im, yr, ai[s][K & 1]));
    }
    if constexpr (K < 15) couple16<SPW, K + 1>(uo, xr, xi, ar, ai);
}

// The same product for one shift with the Re u and Im u terms in separate
// partial sums, so no step holds a dependent pair of FMAs (the narrow kernel).
template <int K>
__device__ __forceinline__ void couple16s(const zd (&uo)[16], double xr, double xi, double (&ar)[4],
                                          double (&ai)[4]) {
    const double yr = bcast16<K>(xr), yi = bcast16<K>(xi);
    ar[K & 1] = fma(uo[K].re, yr, ar[K & 1]);
    ar[2 + (K & 1)] = fma(-uo[K].im, yi, ar[2 + (K & 1)]);
    ai[K & 1] = fma(uo[K].re, yi, ai[K & 1]);
    ai[2 + (K & 1)] = fma(uo[K].im, yr, ai[2 + (K & 1)]);
    if constexpr (K < 15) couple16s<K + 1>(uo, xr, xi, ar, ai);
}

// ---------------------------------------------------------------- fused outer block
constexpr int kRowsMax = 256;          // rows of one outer block
constexpr int kCols = 16;              // shifts per workgroup
constexpr int kSP = kRowsMax + 1;      // padded LDS column stride (bank spread)
// threads of the fused kernel: 4 solving wavefronts plus 8 updating ones for
// the plain solves with nb = 16 (three wavefronts per SIMD, two of them on the
// matrix cores); 4 plus 4 where the register use leaves room for two
// wavefronts per SIMD only (nb = 32, safe). The adjoint variant at 768 threads
// keeps four addresses of its final store loop in scratch (reloaded once).
constexpr int block_threads(int nb, bool adj, bool safe, bool gen = false) {
    return (nb == 16 && !safe && !gen) ? 768 : 512;
}
constexpr int kAW = 4;                 // wavefronts that solve diagonal blocks; the others update
// rounds of the matrix-core tiles a pass deals to the updating wavefronts (the
// rest go to the solving ones): all of the at most 15 tiles with 8 updating
// wavefronts; with 4, the solving ones take tiles 12 and beyond
constexpr int upd_rounds(int nuw) { return nuw >= 8 ? 2 : 3; }

// One outer block (rows [iS, iS+rows)) for kCols shifts, with the right-hand
// sides resident in LDS. Diagonal blocks are solved one per pass with a
// one-block lookahead: in the pass that solves block q, the solving
// wavefronts first apply the solution of the block solved in the pass before
// (block p, adjacent to q) to q's own rows (a short product with the coupling
// block U(q, p), staged in LDS) and then run the back substitution of q, while
// the other wavefronts apply the same solution of p to all rows of the outer
// block beyond q with FP64 MFMA products. The two parts touch disjoint rows, so
// each pass needs one barrier, and the matrix-core work runs beside the
// latency-bound substitution instead of after it. Diagonal and coupling blocks
// of the next pass are loaded during the current one (double-buffered LDS).
// Per element the updates keep the order of the blocks.
// GEN: the pencil U - lambda_j V (Alg 8 / Alg 9): the V blocks are staged
// beside U's, the solving wavefronts form U - lambda V per shift, and the
// matrix-core update adds V times lambda x to the subtraction of U x.
template <int NB, int EV, bool SAFE, bool MIXED, bool VARLEN, bool GEN = false>
__global__ __launch_bounds__(block_threads(NB, ev_fwd(EV), SAFE, GEN)) void k_block(BlockArgs a) {
    static_assert(NB == 16 || NB == 32, "fused outer block: nb 16 or 32");
    static_assert(!GEN || (NB == 16 && EV == 0 && !MIXED), "pencil: nb 16, upper, op N, FP64");
    constexpr bool ADJ = ev_fwd(EV);          // forward substitution (E lower triangular)
    constexpr bool TR = ev_tr(EV), CJ = ev_cj(EV), LOWA = ev_lower_a(EV);
    constexpr int G = 64 / NB;
    constexpr int kWGB = block_threads(NB, ADJ, SAFE, GEN);
    constexpr int NWAVE = kWGB / 64;
    constexpr int NUW = NWAVE - kAW;                     // updating wavefronts
    constexpr int kUpdRounds = upd_rounds(NUW);
    constexpr int SPW = kCols / (kAW * G);               // interleaved shifts per lane group
    constexpr int NBB = NB * NB;
    constexpr int NST = GEN ? 4 : 2;                     // staged blocks per pass
    constexpr int PERS = (NST * NBB + kWGB - 1) / kWGB;  // staged elements per thread
    constexpr int KS = NB / 4;
    static_assert(SPW * G * kAW == kCols, "column split");
    __shared__ zd Bl[kCols * kSP];
    __shared__ zd Us[2][NBB];      // diagonal block, strict triangle (see stage_diag)
    __shared__ zd Uo[2][NBB];      // coupling block: Uo[k*NB + r] = coefficient of x_p(k) in row r of q
    __shared__ zd Ud[2][NB];
    __shared__ zd Vs[GEN ? 2 : 1][GEN ? NBB : 1];   // the same three blocks of V (pencil)
    __shared__ zd Vo[GEN ? 2 : 1][GEN ? NBB : 1];
    __shared__ zd Vd[GEN ? 2 : 1][GEN ? NB : 1];
    __shared__ double Gl[kCols];
    __shared__ int kcl[kCols], dkl[2][kCols], Ll[kCols];

    if (MIXED && a.skip && *a.skip) return;   // refinement stopped
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int col0 = blockIdx.x * kCols;
    const int iS = a.iS, rows = a.rows;
    const int w = a.safe.omega_log2;
    const double omega = ldexp(1.0, w);
    const double delta = SAFE ? (GEN ? fmax(*a.safe.delta, *a.safe.delta_v) : *a.safe.delta) : 0.0;

    if (tid < kCols) {
        const int j = col0 + tid;
        int L = 0;
        if (j < a.n) {
            L = a.m;
            if (VARLEN) {
                L = a.col_len[j];
                L = L < 0 ? 0 : (L > a.m ? a.m : L);
            }
        }
        Ll[tid] = L;
        dkl[0][tid] = 0;
        dkl[1][tid] = 0;
        if (SAFE) {
            Gl[tid] = (j < a.n) ? a.safe.G[j] : 0.0;
            kcl[tid] = (j < a.n) ? a.safe.kcur[j] : 0;
        }
    }
    // right-hand sides of the outer block -> LDS (rows outside the column: 0)
    {
        constexpr int PER = (kCols * kRowsMax + kWGB - 1) / kWGB;
        zd st[PER];
#pragma unroll
        for (int e = 0; e < PER; ++e) {
            const int idx = tid + e * kWGB;
            const int c = idx / kRowsMax, rr = idx - c * kRowsMax;
            const int j = col0 + c;
            int L = 0;
            if (idx < kCols * kRowsMax && j < a.n) {
                L = a.m;
                if (VARLEN) {
                    L = a.col_len[j];
                    L = L < 0 ? 0 : (L > a.m ? a.m : L);
                }
            }
            st[e] = zd{0.0, 0.0};
            if (rr < rows && iS + rr < L) {
                if (MIXED) {
                    const zf v = a.b32[(long)j * a.ldb32 + iS + rr];
                    st[e] = zd{v.re, v.im};
                } else {
                    st[e] = a.B[(long)j * a.ldb + iS + rr];
                }
            }
        }
#pragma unroll
        for (int e = 0; e < PER; ++e) {
            const int idx = tid + e * kWGB;
            const int c = idx / kRowsMax, rr = idx - c * kRowsMax;
            if (idx < kCols * kRowsMax) Bl[c * kSP + rr] = st[e];
        }
    }

    // ---- geometry of pass stp: block ql solved, block qp (solved in the pass
    // before) applied; rows of the outer block relative to iS
    const int nsub = (rows + NB - 1) / NB;
    struct Pass {
        int lr0, bs;      // rows of the block solved in this pass
        int p0, bsp;      // rows of the block applied in this pass (bsp = 0: none)
        int ubeg, uend;   // rows updated by the matrix cores in this pass
    };
    auto pass_of = [&](int stp) __attribute__((always_inline)) {
        Pass g;
        const int ql = ADJ ? stp : nsub - 1 - stp;
        g.lr0 = ql * NB;
        g.bs = min(NB, rows - g.lr0);
        if (stp > 0) {
            const int qp = ADJ ? ql - 1 : ql + 1;
            g.p0 = qp * NB;
            g.bsp = min(NB, rows - g.p0);
            g.ubeg = ADJ ? g.lr0 + g.bs : 0;
            g.uend = ADJ ? rows : g.lr0;
        } else {
            g.p0 = g.lr0;
            g.bsp = 0;
            g.ubeg = g.uend = 0;
        }
        return g;
    };

    // ---- staging of the diagonal and coupling blocks of a pass: loads into
    // registers, stores to LDS later (the latency hides behind a pass's work).
    // Every thread issues exactly one unconditional load per element, from a
    // clamped address inside U's upper triangle; elements outside the blocks
    // are zeroed at the store. Conditional loads into shared registers make
    // the compiler wait for each load before the next (write-after-write).
    zd ust[PERS];
    bool usv[PERS];
    auto stage_load = [&](int stp) __attribute__((always_inline)) {
        const Pass g = pass_of(stp);
        const int i0 = iS + g.lr0, p0 = iS + g.p0;
#pragma unroll
        for (int e = 0; e < PERS; ++e) {
            const int t0 = tid + e * kWGB;
            // pencil: elements 2 NBB .. 4 NBB stage the same blocks of V
            const bool fv = GEN && t0 >= 2 * NBB;
            const int t = fv ? t0 - 2 * NBB : t0;
            const long ld = fv ? a.ldv : a.ldu;
            long off = (long)i0 * ld + i0;   // the block's first pivot: always valid
            bool v = false;
            if (t < NBB) {
                const int c = t / NB, rr = t - c * NB;
                v = rr <= c && c < g.bs;
                off = v ? (LOWA ? (long)(i0 + rr) * ld + i0 + c : (long)(i0 + c) * ld + i0 + rr) : off;
            } else if (t < 2 * NBB) {
                const int t2 = t - NBB;
                if (!TR) {
                    // coefficient of x_p(k) in row r: A(i0 + r, p0 + k)
                    const int k = t2 / NB, r = t2 - k * NB;
                    v = r < g.bs && k < g.bsp;
                    off = v ? (long)(p0 + k) * ld + i0 + r : off;
                } else {
                    // transposed: A(p0 + k, i0 + r) (conjugated at the store for CJ)
                    const int r = t2 / NB, k = t2 - r * NB;
                    v = r < g.bs && k < g.bsp;
                    off = v ? (long)(i0 + r) * ld + p0 + k : off;
                }
            }
            usv[e] = v;
            ust[e] = (fv ? a.V : a.U)[off];
        }
    };
    auto stage_store = [&](int buf) __attribute__((always_inline)) {
#pragma unroll
        for (int e = 0; e < PERS; ++e) {
            const int t0 = tid + e * kWGB;
            zd v = usv[e] ? ust[e] : zd{0.0, 0.0};
            if (CJ) v.im = -v.im;
            if (GEN && t0 >= 2 * NBB) {
                const int t = t0 - 2 * NBB;
                if (t < NBB) {
                    const int c = t / NB, rr = t - c * NB;
                    if (rr == c) {
                        Vd[buf][rr] = v;
                        Vs[buf][c * NB + rr] = zd{0.0, 0.0};
                    } else {
                        Vs[buf][c * NB + rr] = v;
                    }
                } else if (t < 2 * NBB) {
                    const int t2 = t - NBB;
                    const int k = t2 / NB, r = t2 - k * NB;
                    Vo[buf][k * NB + r] = v;
                }
                continue;
            }
            const int t = t0;
            if (t < NBB) {
                const int c = t / NB, rr = t - c * NB;
                if (rr == c) {
                    Ud[buf][rr] = v;
                    Us[buf][c * NB + rr] = zd{0.0, 0.0};
                } else if (!ADJ) {
                    Us[buf][c * NB + rr] = v;
                } else {
                    Us[buf][rr * NB + c] = v;
                }
            } else if (t < 2 * NBB) {
                const int t2 = t - NBB;
                int k, r;
                if (!TR) {
                    k = t2 / NB;
                    r = t2 - k * NB;
                } else {
                    r = t2 / NB;
                    k = t2 - r * NB;
                }
                Uo[buf][k * NB + r] = v;
            }
        }
    };
    stage_load(0);
    stage_store(0);
    __syncthreads();

    const int grp = lane / NB, r = lane - grp * NB, base = grp * NB;
    const int lr = lane & 15, lq = lane >> 4;
    // solving wavefronts: fixed column slots
    int cc[SPW];
    zd lam[SPW];
    bool jv[SPW];
#pragma unroll
    for (int s = 0; s < SPW; ++s) {
        const int c = ((wave % kAW) * SPW + s) * G + grp;
        cc[s] = c;
        jv[s] = col0 + c < a.n;
        lam[s] = (wave < kAW && jv[s]) ? a.lam[col0 + c] : zd{0.0, 0.0};
        // wait for the shifts here, once: the first use is inside the pass loop,
        // where the compiler cannot count the loads in flight and would wait for
        // all of them (the next pass's staging loads included) in every pass
        asm volatile("" : "+v"(lam[s].re), "+v"(lam[s].im));
    }
    // pencil: shift of this lane's column in the matrix-core tiles (column lane % 16)
    zd lamt{0.0, 0.0};
    if (GEN) {
        if (col0 + lr < a.n) lamt = a.lam[col0 + lr];
        asm volatile("" : "+v"(lamt.re), "+v"(lamt.im));
    }

    // U fragments of the matrix-core update: A(row, k) for row = ubeg + tile*16 +
    // lane%16, k = 4 ks + lane/16 (forward: U(iS+row, iS+p0+k); adjoint:
    // conj(U(iS+p0+k, iS+row)), conjugated where consumed). Loads are
    // unconditional from clamped positions inside U's upper triangle (needs
    // uend > ubeg and bsp > 0); positions outside the tile are zeroed where
    // consumed.
    // (pencil: the same positions of V into dstv)
    auto aload = [&](zd (&dst)[KS], zd (&dstv)[GEN ? KS : 1], const Pass& g, int tile)
        __attribute__((always_inline)) {
        const int arow = max(g.ubeg, min(g.ubeg + tile * 16 + lr, g.uend - 1));
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
            const int k = min(ks * 4 + lq, g.bsp - 1);
            if (!TR) dst[ks] = a.U[(long)(iS + g.p0 + k) * a.ldu + iS + arow];
            else dst[ks] = a.U[(long)(iS + arow) * a.ldu + iS + g.p0 + k];
            if constexpr (GEN) dstv[ks] = a.V[(long)(iS + g.p0 + k) * a.ldv + iS + arow];
        }
    };
    zd an[KS];   // first fragment of a pass, loaded at the end of the pass before
    zd vn[GEN ? KS : 1];
    double xpr[SPW], xpi[SPW];   // solving wavefronts: solution of the block of the pass before
#pragma unroll
    for (int s = 0; s < SPW; ++s) xpr[s] = xpi[s] = 0.0;

    for (int stp = 0; stp < nsub; ++stp) {
        const int buf = stp & 1;
        const Pass g = pass_of(stp);
        const int q = a.qa + (ADJ ? stp : nsub - 1 - stp);
        const int i0 = iS + g.lr0;
        // updating wavefronts: settle the first fragment of this pass (loaded in
        // the pass before) before the staging loads are issued, so that the
        // wait for it does not also cover them
        if (wave >= kAW) {
#pragma unroll
            for (int ks = 0; ks < KS; ++ks) asm volatile("" : "+v"(an[ks].re), "+v"(an[ks].im));
            if constexpr (GEN) {
#pragma unroll
                for (int ks = 0; ks < KS; ++ks) asm volatile("" : "+v"(vn[ks].re), "+v"(vn[ks].im));
            }
        }
        if (stp + 1 < nsub) stage_load(stp + 1);

        if (wave < kAW) {
            // ---- rows of block q: apply x of block p, then back substitution
            BlockSolve<NB, SPW, EV, SAFE, GEN> S;
            bool act[SPW];
#pragma unroll
            for (int s = 0; s < SPW; ++s) {
                const int c = cc[s];
                act[s] = jv[s] && (i0 < Ll[c]);
                zd b{0.0, 0.0};
                if (r < g.bs) b = Bl[c * kSP + g.lr0 + r];
                if (SAFE && g.bsp > 0) {
                    // the rows still carry the exponent from before block p
                    const int dk = dkl[buf ^ 1][c];
                    b.re = ldexp(b.re, -dk);
                    b.im = ldexp(b.im, -dk);
                }
                S.br[s] = b.re;
                S.bi[s] = b.im;
            }
            if (g.bsp > 0) {
                // b(r) -= sum_k Uo(r, k) x_p(k), two partial sums per shift
                double ar[SPW][2], ai[SPW][2];
#pragma unroll
                for (int s = 0; s < SPW; ++s) ar[s][0] = ar[s][1] = ai[s][0] = ai[s][1] = 0.0;
                if constexpr (NB == 16) {
                    // x_p(k) is still in lane k of each group from the pass before
                    zd uo[16];
#pragma unroll
                    for (int k = 0; k < 16; ++k) {
                        if constexpr (GEN) uo[k] = pencil(Uo[buf][k * NB + r], Vo[buf][k * NB + r], lam[0]);
                        else uo[k] = Uo[buf][k * NB + r];
                    }
                    couple16<SPW, 0>(uo, xpr, xpi, ar, ai);
                } else {
                    // x_p(k) from LDS: one address per lane group (a broadcast read)
#pragma unroll
                    for (int k = 0; k < NB; ++k) {
                        const zd u = Uo[buf][k * NB + r];
#pragma unroll
                        for (int s = 0; s < SPW; ++s) {
                            const zd x = Bl[cc[s] * kSP + g.p0 + k];
                            ar[s][k & 1] = fma(u.re, x.re, fma(-u.im, x.im, ar[s][k & 1]));
                            ai[s][k & 1] = fma(u.re, x.im, fma(u.im, x.re, ai[s][k & 1]));
                        }
                    }
                }
#pragma unroll
                for (int s = 0; s < SPW; ++s) {
                    S.br[s] -= ar[s][0] + ar[s][1];
                    S.bi[s] -= ai[s][0] + ai[s][1];
                }
            }
            const double cn_l = (SAFE && !GEN && r < g.bs) ? a.safe.cn_in[i0 + r] : 0.0;
            S.pivots(Ud[buf], r, g.bs, lam, jv, delta, Vd[buf]);
            S.run(Us[buf], g.bs, r, base, cn_l, w, omega, Vs[buf], lam[0], SAFE && a.safe.force_checked);
            if (SAFE) {
                const double asum0 = a.safe.above_sum[q];
                const double asumv = GEN ? a.safe.above_sum_v[q] : 0.0;
#pragma unroll
                for (int s = 0; s < SPW; ++s) {
                    const int c = cc[s];
                    const double asum = GEN ? pencil_asum(asum0, asumv, lam[s]) : asum0;
                    double Gj = Gl[c];
                    const int dk = S.column_bound(s, act[s], asum, &Gj, w, omega);
                    if (r == 0 && jv[s]) {
                        const int kc = kcl[c] + dk;
                        if (act[s]) {
                            Gl[c] = S.Gs[s];
                            kcl[c] = kc;
                        }
                        dkl[buf][c] = dk;
                        a.safe.kb[(long)q * a.n + col0 + c] = kc;
                    }
                }
            }
#pragma unroll
            for (int s = 0; s < SPW; ++s) {
                if (r < g.bs) Bl[cc[s] * kSP + g.lr0 + r] = zd{S.br[s], S.bi[s]};
                xpr[s] = S.br[s];
                xpi[s] = S.bi[s];
            }
        }
        // ---- rows beyond block q: C -= U_panel * x(block p) on the matrix cores.
        // Static round-robin: updating wavefront u takes tiles u, u + NUW, ...
        // below NUW * kUpdRounds (its first fragment prefetched in the pass
        // before, each next one during the tile before); tiles from there on go
        // to the solving wavefronts after their solve. (A shared claim counter
        // would put an LDS atomic round trip, about a thousand cycles when the
        // pass is busy, on both critical paths.)
        {
            const int ntile = (g.uend - g.ubeg + 15) / 16;
            const int dsh = (SAFE && g.bsp > 0) ? dkl[buf ^ 1][lr] : 0;
            auto do_tile = [&](int tile, const zd (&af)[KS], const zd (&vf)[GEN ? KS : 1])
                __attribute__((always_inline)) {
                const int rb = g.ubeg + tile * 16;
                const bool rowok = rb + lr < g.uend;   // this lane's A row inside the tile
                // Every LDS read below is in bounds (rows < 256) and needs no
                // branch: rows past the outer block are zero in Bl, and the
                // tiles never reach into the block being solved. Unguarded
                // reads issue together instead of one wait per branch.
                // Four accumulator chains (real and imaginary parts, each split
                // in two) keep dependent matrix-core products apart; the halves
                // are added at the end.
                v4d accR, accI, accR2, accI2;
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int row = rb + lq + 4 * v;
                    zd c = Bl[lr * kSP + row];
                    if (SAFE) {
                        c.re = ldexp(c.re, -dsh);
                        c.im = ldexp(c.im, -dsh);
                    }
                    accR[v] = c.re;
                    accI[v] = c.im;
                    accR2[v] = 0.0;
                    accI2[v] = 0.0;
                }
#pragma unroll
                for (int ks = 0; ks < KS; ++ks) {
                    // x(block p) fragment from LDS: row k = 4 ks + lane/16, column lane%16
                    const int k = ks * 4 + lq;
                    const zd xb = Bl[lr * kSP + g.p0 + k];
                    const bool ok = rowok && k < g.bsp;
                    const double ar = ok ? -af[ks].re : 0.0;
                    const double ai = ok ? (CJ ? af[ks].im : -af[ks].im) : 0.0;
                    accR = __builtin_amdgcn_mfma_f64_16x16x4f64(ar, xb.re, accR, 0, 0, 0);
                    accI = __builtin_amdgcn_mfma_f64_16x16x4f64(ar, xb.im, accI, 0, 0, 0);
                    accR2 = __builtin_amdgcn_mfma_f64_16x16x4f64(-ai, xb.im, accR2, 0, 0, 0);
                    accI2 = __builtin_amdgcn_mfma_f64_16x16x4f64(ai, xb.re, accI2, 0, 0, 0);
                    if constexpr (GEN) {
                        // + V(row, k) * (lambda_col x(k, col))
                        const double wr = lamt.re * xb.re - lamt.im * xb.im;
                        const double wi = lamt.re * xb.im + lamt.im * xb.re;
                        const double vr = ok ? vf[ks].re : 0.0;
                        const double vi = ok ? vf[ks].im : 0.0;
                        accR = __builtin_amdgcn_mfma_f64_16x16x4f64(vr, wr, accR, 0, 0, 0);
                        accI = __builtin_amdgcn_mfma_f64_16x16x4f64(vr, wi, accI, 0, 0, 0);
                        accR2 = __builtin_amdgcn_mfma_f64_16x16x4f64(-vi, wi, accR2, 0, 0, 0);
                        accI2 = __builtin_amdgcn_mfma_f64_16x16x4f64(vi, wr, accI2, 0, 0, 0);
                    }
                }
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int row = rb + lq + 4 * v;
                    if (row < g.uend) Bl[lr * kSP + row] = zd{accR[v] + accR2[v], accI[v] + accI2[v]};
                }
            };
            const int nt_upd = min(ntile, NUW * kUpdRounds);
            // wave-uniform tile indices (scalar loop control and addresses)
            const int wv = __builtin_amdgcn_readfirstlane(wave);
            int cur, stride, lim;
            if (wv >= kAW) {
                cur = wv - kAW;
                stride = NUW;
                lim = nt_upd;
            } else {
                cur = nt_upd + wv;
                stride = kAW;
                lim = ntile;
                if (cur < lim) aload(an, vn, g, cur);
            }
            cur = __builtin_amdgcn_readfirstlane(cur);
            lim = __builtin_amdgcn_readfirstlane(lim);
            zd af[KS];
            zd vf[GEN ? KS : 1];
            while (cur < lim) {
                const int nxt = cur + stride;
#pragma unroll
                for (int ks = 0; ks < KS; ++ks) af[ks] = an[ks];
                if constexpr (GEN) {
#pragma unroll
                    for (int ks = 0; ks < KS; ++ks) vf[ks] = vn[ks];
                }
                if (nxt < lim) aload(an, vn, g, nxt);
                do_tile(cur, af, vf);
                cur = nxt;
            }
        }
        if (stp + 1 < nsub) stage_store(buf ^ 1);
        // first fragment of the next pass, in flight across the barrier; issued
        // after the staging stores so that their wait does not cover it
        if (wave >= kAW && stp + 1 < nsub) {
            const Pass gn = pass_of(stp + 1);
            if (gn.uend > gn.ubeg) aload(an, vn, gn, wave - kAW);
        }
        __syncthreads();
    }

    // ---- solution of the outer block -> HBM; safe state back
    if (SAFE && tid < kCols && col0 + tid < a.n) {
        a.safe.G[col0 + tid] = Gl[tid];
        a.safe.kcur[col0 + tid] = kcl[tid];
    }
    {
        constexpr int PER = (kCols * kRowsMax + kWGB - 1) / kWGB;
#pragma unroll
        for (int e = 0; e < PER; ++e) {
            const int idx = tid + e * kWGB;
            const int c = idx / kRowsMax, rr = idx - c * kRowsMax;
            const int j = col0 + c;
            if (idx < kCols * kRowsMax && j < a.n && rr < rows && iS + rr < Ll[c]) {
                const zd v = Bl[c * kSP + rr];
                a.B[(long)j * a.ldb + iS + rr] = v;
                if (MIXED) a.b32[(long)j * a.ldb32 + iS + rr] = zf{(float)v.re, (float)v.im};
            }
        }
    }
}

// ---------------------------------------------------------------- narrow fused outer block
// The outer block of k_block for C = 4, 2 or 1 shifts per workgroup of 4
// wavefronts, for launches whose 16-shift workgroups would leave compute units
// idle (few shifts, or few columns reaching an outer block in the
// triangular-eigenvector solve), for every solve variant EV (safe,
// variable-length and mixed forms: upper, op N), over outer blocks of up to
// R = 256 rows (512 for plain solves at C <= 2). Wavefront 0 solves the
// diagonal blocks exactly as a solving wavefront of k_block (one shift per
// lane group). Wavefronts 1-3 apply each solved block to the rows still to be
// solved (above it for back substitution, below it for forward) with FP64
// FMAs, one row per lane and all C shifts: at four shifts or fewer a
// 16-column matrix-core tile would be mostly padding, and the substitution
// chain then shares its SIMD's FP64 pipeline with no matrix-core products
// (the four wavefronts of a workgroup run on four different SIMDs). Rows of
// the update go in 64-row chunks: wavefront u takes chunks u - 1, u + 2,
// u + 5, ..., its first chunk's U entries loaded during the pass before. Per
// element the updates keep the order of the blocks, as in k_block, and a
// shift's arithmetic does not depend on C.
constexpr int kWGN = 256;     // threads per narrow workgroup

// accumulators of a step of the narrow update, pinned after the step (see
// uapply in k_block_narrow)
template <int C>
__device__ __forceinline__ void pin_step(double (&sr)[C], double (&si)[C], double (&tr)[C], double (&ti)[C]) {
    if constexpr (C == 4) {
        asm volatile(""
                     : "+v"(sr[0]), "+v"(sr[1]), "+v"(sr[2]), "+v"(sr[3]), "+v"(si[0]), "+v"(si[1]), "+v"(si[2]),
                       "+v"(si[3]), "+v"(tr[0]), "+v"(tr[1]), "+v"(tr[2]), "+v"(tr[3]), "+v"(ti[0]), "+v"(ti[1]),
                       "+v"(ti[2]), "+v"(ti[3])
                     :
                     : "memory");
    } else if constexpr (C == 2) {
        asm volatile(""
                     : "+v"(sr[0]), "+v"(sr[1]), "+v"(si[0]), "+v"(si[1]), "+v"(tr[0]), "+v"(tr[1]), "+v"(ti[0]),
                       "+v"(ti[1])
                     :
                     : "memory");
    } else {
        static_assert(C == 1, "2^k shifts per narrow workgroup, k <= 2");
        asm volatile("" : "+v"(sr[0]), "+v"(si[0]), "+v"(tr[0]), "+v"(ti[0]) : : "memory");
    }
}
template <int EV, bool SAFE, bool MIXED, bool VARLEN, int C, int R>
__global__ __launch_bounds__(kWGN) void k_block_narrow(BlockArgs a) {
    static_assert(EV == EV_UPPER_N || (!SAFE && !MIXED && !VARLEN), "variants: plain FP64 solves");
    static_assert(R == kRowsMax || (R == 2 * kRowsMax && C <= 2 && !SAFE && !MIXED && !VARLEN),
                  "512-row outer blocks: plain FP64, at most 2 shifts");
    constexpr int SP = R + 1;   // padded LDS column stride
    constexpr bool ADJ = ev_fwd(EV);          // forward substitution (E lower triangular)
    constexpr bool TR = ev_tr(EV), CJ = ev_cj(EV), LOWA = ev_lower_a(EV);
    using BS = BlockSolve<16, 1, EV, SAFE>;
    constexpr int NB = 16, NBB = NB * NB;
    constexpr int PERS = 2 * NBB / kWGN;
    __shared__ zd Bl[C * SP];
    __shared__ zd Us[2][NBB];
    __shared__ zd Uo[2][NBB];
    __shared__ zd Ud[2][NB];
    __shared__ double Gl[C];
    __shared__ int kcl[C], dkl[2][C], Ll[C];
    // pivots of every row of the outer block and shift (formed in the prologue,
    // off the substitution chain): reciprocal, exponent (safe), cabs1 (safe)
    __shared__ double Ppr[C][R], Ppi[C][R];
    __shared__ int Ppe[SAFE ? C : 1][SAFE ? R : 1];
    __shared__ double Pcd[SAFE ? C : 1][SAFE ? R : 1];

    if (MIXED && a.skip && *a.skip) return;   // refinement stopped
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int col0 = blockIdx.x * C;
    const int iS = a.iS, rows = a.rows;
    const int w = a.safe.omega_log2;
    const double omega = ldexp(1.0, w);
    const double delta = SAFE ? *a.safe.delta : 0.0;
    const int nsub = (rows + NB - 1) / NB;

    // column lengths of the workgroup's shifts
    int Lmax = 0;
#pragma unroll
    for (int c = 0; c < C; ++c) {
        const int j = col0 + c;
        int L = 0;
        if (j < a.n) {
            L = a.m;
            if (VARLEN) {
                L = a.col_len[j];
                L = L < 0 ? 0 : (L > a.m ? a.m : L);
            }
        }
        Lmax = max(Lmax, L);
        if (tid == c) Ll[c] = L;
    }
    if (VARLEN && Lmax <= iS) {
        // no column reaches the outer block: nothing to solve, the exponents
        // after each of its diagonal blocks are the current ones
        if (SAFE && tid < C * nsub) {
            const int c = tid % C, q = a.qa + tid / C;
            if (col0 + c < a.n) a.safe.kb[(long)q * a.n + col0 + c] = a.safe.kcur[col0 + c];
        }
        return;
    }
    if (tid < C) {
        const int j = col0 + tid;
        dkl[0][tid] = 0;
        dkl[1][tid] = 0;
        if (SAFE) {
            Gl[tid] = (j < a.n) ? a.safe.G[j] : 0.0;
            kcl[tid] = (j < a.n) ? a.safe.kcur[j] : 0;
        }
    }
    // pivots: A(r, r) - lambda_j (conjugated for CJ) for every row of the
    // outer block and shift (1 + 0i outside the block or past the shifts)
    {
        constexpr int PER = C * R / kWGN;
#pragma unroll
        for (int e = 0; e < PER; ++e) {
            const int idx = tid + e * kWGN;
            const int c = idx / R, rr = idx - c * R;
            double dr = 1.0, di = 0.0;
            if (rr < rows && col0 + c < a.n) {
                zd u = a.U[(long)(iS + rr) * a.ldu + iS + rr];
                if (CJ) u.im = -u.im;   // as staged (E's diagonal)
                BS::pivot_value(u, a.lam[col0 + c], delta, dr, di);
            }
            double pr, pi, cd;
            int pe;
            BS::pivot_entry(dr, di, pr, pi, pe, cd);
            Ppr[c][rr] = pr;
            Ppi[c][rr] = pi;
            if (SAFE) {
                Ppe[c][rr] = pe;
                Pcd[c][rr] = cd;
            }
        }
    }
    // right-hand sides of the outer block -> LDS (rows outside the column: 0)
    {
        constexpr int PER = C * R / kWGN;
        zd st[PER];
#pragma unroll
        for (int e = 0; e < PER; ++e) {
            const int idx = tid + e * kWGN;
            const int c = idx / R, rr = idx - c * R;
            const int j = col0 + c;
            int L = 0;
            if (j < a.n) {
                L = a.m;
                if (VARLEN) {
                    L = a.col_len[j];
                    L = L < 0 ? 0 : (L > a.m ? a.m : L);
                }
            }
            st[e] = zd{0.0, 0.0};
            if (rr < rows && iS + rr < L) {
                if (MIXED) {
                    const zf v = a.b32[(long)j * a.ldb32 + iS + rr];
                    st[e] = zd{v.re, v.im};
                } else {
                    st[e] = a.B[(long)j * a.ldb + iS + rr];
                }
            }
        }
#pragma unroll
        for (int e = 0; e < PER; ++e) {
            const int idx = tid + e * kWGN;
            const int c = idx / R, rr = idx - c * R;
            Bl[c * SP + rr] = st[e];
        }
    }

    // pass stp solves block ql (from the bottom; from the top for forward
    // substitution) and applies block qp (solved in the pass before, adjacent
    // to ql) to the rows [ubeg, uend) still to be solved beyond ql
    struct Pass {
        int lr0, bs, p0, bsp, ubeg, uend;
    };
    auto pass_of = [&](int stp) __attribute__((always_inline)) {
        Pass g;
        const int ql = ADJ ? stp : nsub - 1 - stp;
        g.lr0 = ql * NB;
        g.bs = min(NB, rows - g.lr0);
        g.p0 = (ADJ ? ql - 1 : ql + 1) * NB;
        g.bsp = stp > 0 ? min(NB, rows - g.p0) : 0;
        g.ubeg = ADJ ? g.lr0 + g.bs : 0;
        g.uend = ADJ ? rows : g.lr0;
        return g;
    };

    // staging of the diagonal and coupling blocks of a pass, as in k_block
    zd ust[PERS];
    bool usv[PERS];
    auto stage_load = [&](int stp) __attribute__((always_inline)) {
        const Pass g = pass_of(stp);
        const int i0 = iS + g.lr0, p0 = iS + g.p0;
#pragma unroll
        for (int e = 0; e < PERS; ++e) {
            const int t = tid + e * kWGN;
            long off = (long)i0 * a.ldu + i0;   // the block's first pivot: always valid
            bool v = false;
            if (t < NBB) {
                const int c = t / NB, rr = t - c * NB;
                v = rr <= c && c < g.bs;
                off = v ? (LOWA ? (long)(i0 + rr) * a.ldu + i0 + c : (long)(i0 + c) * a.ldu + i0 + rr) : off;
            } else {
                const int t2 = t - NBB;
                if (!TR) {
                    // coefficient of x_p(k) in row r: A(i0 + r, p0 + k)
                    const int k = t2 / NB, r = t2 - k * NB;
                    v = r < g.bs && k < g.bsp;
                    off = v ? (long)(p0 + k) * a.ldu + i0 + r : off;
                } else {
                    // transposed: A(p0 + k, i0 + r) (conjugated at the store for CJ)
                    const int r = t2 / NB, k = t2 - r * NB;
                    v = r < g.bs && k < g.bsp;
                    off = v ? (long)(i0 + r) * a.ldu + p0 + k : off;
                }
            }
            usv[e] = v;
            ust[e] = a.U[off];
        }
    };
    auto stage_store = [&](int buf) __attribute__((always_inline)) {
#pragma unroll
        for (int e = 0; e < PERS; ++e) {
            const int t = tid + e * kWGN;
            zd v = usv[e] ? ust[e] : zd{0.0, 0.0};
            if (CJ) v.im = -v.im;
            if (t < NBB) {
                const int c = t / NB, rr = t - c * NB;
                if (rr == c) {
                    Ud[buf][rr] = v;
                    Us[buf][c * NB + rr] = zd{0.0, 0.0};
                } else if (!ADJ) {
                    Us[buf][c * NB + rr] = v;
                } else {
                    Us[buf][rr * NB + c] = v;
                }
            } else {
                const int t2 = t - NBB;
                int k, r;
                if (!TR) {
                    k = t2 / NB;
                    r = t2 - k * NB;
                } else {
                    r = t2 / NB;
                    k = t2 - r * NB;
                }
                Uo[buf][k * NB + r] = v;
            }
        }
    };
    stage_load(0);
    stage_store(0);
    __syncthreads();

    // updating wavefronts: E(row, p0 + k), k < 16, of one 64-row chunk (row =
    // ubeg + chunk * 64 + lane; E(r, c) = A(r, c), or A(c, r) conjugated for
    // CJ when transposed), from clamped positions (in bounds; rows outside the
    // update are never stored, entries past block p are never used)
    auto uload = [&](zd (&u)[NB], const Pass& g, int chunk) __attribute__((always_inline)) {
        const int row = max(min(g.ubeg + chunk * 64 + lane, g.uend - 1), 0);
        // one running pointer along block p (one 64-bit add per step), held
        // at its last column past it
        const zd* up = TR ? a.U + (long)(iS + row) * a.ldu + iS + g.p0 : a.U + (long)(iS + g.p0) * a.ldu + iS + row;
        const long st = TR ? 1 : a.ldu;
#pragma unroll
        for (int k = 0; k < NB; ++k) {
            u[k] = *up;
            if (CJ) u[k].im = -u[k].im;
            if (k + 1 < g.bsp) up += st;
        }
    };
    // rows of the chunk -= U(rows, block p) x(block p), all four shifts per
    // step k. The x of step k + 3 (four LDS broadcast reads) are issued with
    // the FMAs of step k, and rows are stored after the last step. An empty
    // asm statement after each step takes the accumulators as operands and
    // clobbers memory: it keeps the step's FMAs before it and later reads
    // after it, so the compiler neither sinks each read next to its FMAs (an
    // LDS round trip on every step) nor hoists all of them to the top (every
    // x live at once). Rows p0 + k for
    // k >= bsp lie past the outer block, where Bl holds zeros (p0 + 15 <=
    // R - 1; only the last block can be partial, and it is never block p of
    // forward substitution), so no step needs a mask. Each component keeps two accumulators
    // (the terms with Re u and with Im u), so a step's 16 FMAs are
    // independent. In the safe form the rows first take the exponent change
    // of block p.
    auto uapply = [&](const zd (&u)[NB], const Pass& g, int chunk, int buf) __attribute__((always_inline)) {
        const int row = g.ubeg + chunk * 64 + lane;   // < R where stored (row < uend)
        const bool ok = row < g.uend;
        const zd* xb = Bl + g.p0;
        double sr[C], si[C], tr[C], ti[C];
        zd x0[C], x1[C], x2[C], x3[C];
#pragma unroll
        for (int c = 0; c < C; ++c) {
            zd v = Bl[c * SP + min(row, R - 1)];
            x0[c] = xb[c * SP];
            x1[c] = xb[c * SP + 1];
            x2[c] = xb[c * SP + 2];
            if (SAFE) {
                const int dk = dkl[buf ^ 1][c];
                v.re = ldexp(v.re, -dk);
                v.im = ldexp(v.im, -dk);
            }
            sr[c] = v.re;
            si[c] = v.im;
            tr[c] = 0.0;
            ti[c] = 0.0;
        }
#pragma unroll
        for (int k = 0; k < NB; ++k) {
            if (k + 3 < NB) {
#pragma unroll
                for (int c = 0; c < C; ++c) x3[c] = xb[c * SP + k + 3];
            }
#pragma unroll
            for (int c = 0; c < C; ++c) {
                sr[c] = fma(-u[k].re, x0[c].re, sr[c]);
                si[c] = fma(-u[k].re, x0[c].im, si[c]);
                tr[c] = fma(u[k].im, x0[c].im, tr[c]);
                ti[c] = fma(-u[k].im, x0[c].re, ti[c]);
            }
            pin_step<C>(sr, si, tr, ti);
#pragma unroll
            for (int c = 0; c < C; ++c) {
                x0[c] = x1[c];
                x1[c] = x2[c];
                x2[c] = x3[c];
            }
        }
#pragma unroll
        for (int c = 0; c < C; ++c)
            if (ok) Bl[c * SP + row] = zd{sr[c] + tr[c], si[c] + ti[c]};
    };

    // The solving and the updating wavefronts run separate pass loops (the
    // branch is uniform per wavefront), each with one barrier per pass, so
    // neither holds the other's registers.
    const int wv = __builtin_amdgcn_readfirstlane(wave);
    if (wv == 0) {
        // shift slot grp = lane / 16, row r = lane % 16; with fewer than four
        // shifts the lane groups past them repeat the last shift's chain and
        // store nothing
        const int grp = lane >> 4, r = lane & 15, base = grp * NB;
        const bool own = grp < C;
        const int c = own ? grp : C - 1;
        const bool jv[1] = {own && col0 + grp < a.n};
        double xpr[1] = {0.0}, xpi[1] = {0.0};
        for (int stp = 0; stp < nsub; ++stp) {
            const int buf = stp & 1;
            const Pass g = pass_of(stp);
            const int q = a.qa + (ADJ ? stp : nsub - 1 - stp);
            const int i0 = iS + g.lr0;
            if (stp + 1 < nsub) stage_load(stp + 1);
            // ---- rows of block q: apply x of block p, then the substitution
            BS S;
            const bool act = jv[0] && (i0 < Ll[c]);
            zd b{0.0, 0.0};
            if (r < g.bs) b = Bl[c * SP + g.lr0 + r];
            if (SAFE && g.bsp > 0) {
                const int dk = dkl[buf ^ 1][c];
                b.re = ldexp(b.re, -dk);
                b.im = ldexp(b.im, -dk);
            }
            S.br[0] = b.re;
            S.bi[0] = b.im;
            if (g.bsp > 0) {
                double ar[4] = {0.0, 0.0, 0.0, 0.0}, ai[4] = {0.0, 0.0, 0.0, 0.0};
                zd uo[16];
#pragma unroll
                for (int k = 0; k < 16; ++k) uo[k] = Uo[buf][k * NB + r];
                couple16s<0>(uo, xpr[0], xpi[0], ar, ai);
                S.br[0] -= (ar[0] + ar[1]) + (ar[2] + ar[3]);
                S.bi[0] -= (ai[0] + ai[1]) + (ai[2] + ai[3]);
            }
            const double cn_l = (SAFE && r < g.bs) ? a.safe.cn_in[i0 + r] : 0.0;
            {
                // rows past a partial block take 1 + 0i, as the table holds
                // for rows past the outer block
                const int pr_row = g.lr0 + r;
                const bool in = r < g.bs && jv[0];
                const double ppr[1] = {in ? Ppr[c][pr_row] : 1.0};
                const double ppi[1] = {in ? Ppi[c][pr_row] : -0.0};   // pivot_entry(1, 0)
                const int ppe[1] = {SAFE && in ? Ppe[SAFE ? c : 0][SAFE ? pr_row : 0] : 0};
                const double pcd[1] = {SAFE && in ? Pcd[SAFE ? c : 0][SAFE ? pr_row : 0] : 1.0};
                S.pivots_given(ppr, ppi, ppe, pcd);
            }
            S.run(Us[buf], g.bs, r, base, cn_l, w, omega, nullptr, zd{0.0, 0.0}, SAFE && a.safe.force_checked);
            if (SAFE) {
                const double asum = a.safe.above_sum[q];
                double Gj = Gl[c];
                const int dk = S.column_bound(0, act, asum, &Gj, w, omega);
                if (r == 0 && jv[0]) {
                    const int kc = kcl[c] + dk;
                    if (act) {
                        Gl[c] = S.Gs[0];
                        kcl[c] = kc;
                    }
                    dkl[buf][c] = dk;
                    a.safe.kb[(long)q * a.n + col0 + c] = kc;
                }
            }
            if (own && r < g.bs) Bl[c * SP + g.lr0 + r] = zd{S.br[0], S.bi[0]};
            xpr[0] = S.br[0];
            xpi[0] = S.bi[0];
            if (stp + 1 < nsub) stage_store(buf ^ 1);
            __syncthreads();
        }
    } else {
        // ---- rows beyond the block being solved: chunks wv - 1, wv + 2, wv + 5, ...
        zd un[NB];   // first chunk of a pass, loaded during the pass before
        if (nsub > 1) uload(un, pass_of(1), wv - 1);
        for (int stp = 0; stp < nsub; ++stp) {
            const int buf = stp & 1;
            const Pass g = pass_of(stp);
            if (stp > 0) {
                // settle the first chunk before the staging loads are issued,
                // so that the wait for it does not also cover them
#pragma unroll
                for (int k = 0; k < NB; ++k) asm volatile("" : "+v"(un[k].re), "+v"(un[k].im));
            }
            if (stp + 1 < nsub) stage_load(stp + 1);
            if (g.bsp > 0) {
                // (further chunks exist in the first passes of a full outer
                // block only; their loads reuse the registers)
                const int nch = (g.uend - g.ubeg + 63) / 64;
                if (wv - 1 < nch) uapply(un, g, wv - 1, buf);
                for (int ch = wv + 2; ch < nch; ch += 3) {
                    uload(un, g, ch);
                    uapply(un, g, ch, buf);
                }
            }
            if (stp + 1 < nsub) stage_store(buf ^ 1);
            // first chunk of the next pass, in flight across the barrier
            if (stp + 1 < nsub) {
                const Pass gn = pass_of(stp + 1);
                if (wv - 1 < (gn.uend - gn.ubeg + 63) / 64) uload(un, gn, wv - 1);
            }
            __syncthreads();
        }
    }

    // ---- solution of the outer block -> HBM; safe state back
    if (SAFE && tid < C && col0 + tid < a.n) {
        a.safe.G[col0 + tid] = Gl[tid];
        a.safe.kcur[col0 + tid] = kcl[tid];
    }
    {
        constexpr int PER = C * R / kWGN;
#pragma unroll
        for (int e = 0; e < PER; ++e) {
            const int idx = tid + e * kWGN;
            const int c = idx / R, rr = idx - c * R;
            const int j = col0 + c;
            if (j < a.n && rr < rows && iS + rr < Ll[c]) {
                const zd v = Bl[c * SP + rr];
                a.B[(long)j * a.ldb + iS + rr] = v;
                if (MIXED) a.b32[(long)j * a.ldb32 + iS + rr] = zf{(float)v.re, (float)v.im};
            }
        }
    }
}


// Shifts per workgroup of the fused outer block when the caller leaves it
// open: 16 (k_block) unless that grid leaves compute units idle; then
// k_block_narrow with 1 shift per workgroup where that grid gives each compute
// unit at most one workgroup, else the narrowest of 2 and 4 whose grid runs in
// one round of two workgroups per compute unit. Narrower workgroups shorten
// each pass (fewer shifts per updating lane) and spread the chains over more
// compute units, until two of them share a compute unit.
int auto_width(const BlockArgs& a) {
    const int cus = device_cu_count();
    const int wide = (a.n + kCols - 1) / kCols, w4 = (a.n + 3) / 4, w2 = (a.n + 1) / 2;
    if (wide >= cus || w4 > 2 * cus) return 16;
    if (a.n <= cus) return 1;
    return w2 <= 2 * cus ? 2 : 4;
}

template <int EV, int C>
hipError_t launch_narrow(const BlockArgs& a, bool safe, bool mixed, bool varlen, hipStream_t s) {
    const dim3 gn((a.n + C - 1) / C), bn(kWGN);
    if (a.rows > kRowsMax) {
        // 512-row outer blocks: plain FP64 with at most 2 shifts per workgroup
        if constexpr (C <= 2) {
            if (safe || mixed || varlen) return hipErrorInvalidValue;
            hipLaunchKernelGGL((k_block_narrow<EV, false, false, false, C, 2 * kRowsMax>), gn, bn, 0, s, a);
            return hipGetLastError();
        } else {
            return hipErrorInvalidValue;
        }
    }
    if constexpr (EV == EV_UPPER_N) {
        if (safe && varlen) hipLaunchKernelGGL((k_block_narrow<EV, true, false, true, C, kRowsMax>), gn, bn, 0, s, a);
        else if (safe) hipLaunchKernelGGL((k_block_narrow<EV, true, false, false, C, kRowsMax>), gn, bn, 0, s, a);
        else if (mixed) hipLaunchKernelGGL((k_block_narrow<EV, false, true, false, C, kRowsMax>), gn, bn, 0, s, a);
        else hipLaunchKernelGGL((k_block_narrow<EV, false, false, false, C, kRowsMax>), gn, bn, 0, s, a);
    } else {
        hipLaunchKernelGGL((k_block_narrow<EV, false, false, false, C, kRowsMax>), gn, bn, 0, s, a);
    }
    return hipGetLastError();
}

template <int NB, int SPW, int EV>
hipError_t launch_nb(const DiagArgs& a, hipStream_t s) {
    constexpr int per_wg = (kWG / 64) * (64 / NB) * SPW;
    const dim3 grid((a.n + per_wg - 1) / per_wg);
    const bool safe = a.use_safe != 0;
    const bool mixed = a.b32 != nullptr;
    const bool varlen = a.col_len != nullptr;
    if (a.V != nullptr) {
        if constexpr (NB == 16 && EV == EV_UPPER_N) {
            if (mixed || (varlen && !safe)) return hipErrorInvalidValue;
            if (safe && varlen)
                hipLaunchKernelGGL((k_diag<16, SPW, 0, true, false, true, true>), grid, dim3(kWG), 0, s, a);
            else if (safe)
                hipLaunchKernelGGL((k_diag<16, SPW, 0, true, false, false, true>), grid, dim3(kWG), 0, s, a);
            else
                hipLaunchKernelGGL((k_diag<16, SPW, 0, false, false, false, true>), grid, dim3(kWG), 0, s, a);
            return hipGetLastError();
        } else {
            return hipErrorInvalidValue;
        }
    }
    if constexpr (EV != EV_UPPER_N) {
        // the other variants: plain FP64 solves only
        if (safe || mixed || varlen) return hipErrorInvalidValue;
        hipLaunchKernelGGL((k_diag<NB, SPW, EV, false, false, false>), grid, dim3(kWG), 0, s, a);
    } else if (safe) {
        if (mixed) return hipErrorInvalidValue;
        if (varlen)
            hipLaunchKernelGGL((k_diag<NB, SPW, 0, true, false, true>), grid, dim3(kWG), 0, s, a);
        else
            hipLaunchKernelGGL((k_diag<NB, SPW, 0, true, false, false>), grid, dim3(kWG), 0, s, a);
    } else {
        if (varlen) return hipErrorInvalidValue;
        if (mixed)
            hipLaunchKernelGGL((k_diag<NB, SPW, 0, false, true, false>), grid, dim3(kWG), 0, s, a);
        else
            hipLaunchKernelGGL((k_diag<NB, SPW, 0, false, false, false>), grid, dim3(kWG), 0, s, a);
    }
    return hipGetLastError();
}

template <int NB, int EV>
hipError_t launch_blk(const BlockArgs& a, hipStream_t s) {
    const dim3 grid((a.n + kCols - 1) / kCols);
    const bool safe = a.use_safe != 0;
    const bool mixed = a.b32 != nullptr;
    const bool varlen = a.col_len != nullptr;
    if constexpr (NB == 16) {
        // 4-shift workgroups where 16-shift ones would leave compute units idle
        const bool supported = a.V == nullptr && !(safe && mixed) && !(varlen && !safe) &&
                               (EV == EV_UPPER_N || (!safe && !mixed && !varlen));
        const int width = !supported ? 16 : a.width ? a.width : auto_width(a);
        if (width == 4 || width == 2 || width == 1) {
            if (width == 4) return launch_narrow<EV, 4>(a, safe, mixed, varlen, s);
            if (width == 2) return launch_narrow<EV, 2>(a, safe, mixed, varlen, s);
            return launch_narrow<EV, 1>(a, safe, mixed, varlen, s);
        }
        if (a.rows > kRowsMax) return hipErrorInvalidValue;
    }
    if (a.V != nullptr) {
        if constexpr (NB == 16 && EV == EV_UPPER_N) {
            if (mixed || (varlen && !safe)) return hipErrorInvalidValue;
            const dim3 blk(block_threads(16, false, safe, true));
            if (safe && varlen)
                hipLaunchKernelGGL((k_block<16, 0, true, false, true, true>), grid, blk, 0, s, a);
            else if (safe)
                hipLaunchKernelGGL((k_block<16, 0, true, false, false, true>), grid, blk, 0, s, a);
            else
                hipLaunchKernelGGL((k_block<16, 0, false, false, false, true>), grid, blk, 0, s, a);
            return hipGetLastError();
        } else {
            return hipErrorInvalidValue;
        }
    }
    if constexpr (EV != EV_UPPER_N) {
        // the other variants: plain FP64 solves only
        if (safe || mixed || varlen) return hipErrorInvalidValue;
        hipLaunchKernelGGL((k_block<NB, EV, false, false, false>), grid,
                           dim3(block_threads(NB, ev_fwd(EV), false)), 0, s, a);
    } else if (safe) {
        if (mixed) return hipErrorInvalidValue;
        if (varlen)
            hipLaunchKernelGGL((k_block<NB, 0, true, false, true>), grid, dim3(block_threads(NB, false, true)), 0, s, a);
        else
            hipLaunchKernelGGL((k_block<NB, 0, true, false, false>), grid, dim3(block_threads(NB, false, true)), 0, s, a);
    } else {
        if (varlen) return hipErrorInvalidValue;
        if (mixed)
            hipLaunchKernelGGL((k_block<NB, 0, false, true, false>), grid, dim3(block_threads(NB, false, false)), 0, s, a);
        else
            hipLaunchKernelGGL((k_block<NB, 0, false, false, false>), grid, dim3(block_threads(NB, false, false)), 0, s, a);
    }
    return hipGetLastError();
}

template <int NB, int SPW>
hipError_t launch_nb_ev(int ev, const DiagArgs& a, hipStream_t s) {
    switch (ev) {
        case EV_UPPER_N: return launch_nb<NB, SPW, EV_UPPER_N>(a, s);
        case EV_UPPER_C: return launch_nb<NB, SPW, EV_UPPER_C>(a, s);
        case EV_UPPER_T: return launch_nb<NB, SPW, EV_UPPER_T>(a, s);
        case EV_LOWER_N: return launch_nb<NB, SPW, EV_LOWER_N>(a, s);
        case EV_LOWER_T: return launch_nb<NB, SPW, EV_LOWER_T>(a, s);
        case EV_LOWER_C: return launch_nb<NB, SPW, EV_LOWER_C>(a, s);
        default: return hipErrorInvalidValue;
    }
}

template <int NB>
hipError_t launch_blk_ev(int ev, const BlockArgs& a, hipStream_t s) {
    switch (ev) {
        case EV_UPPER_N: return launch_blk<NB, EV_UPPER_N>(a, s);
        case EV_UPPER_C: return launch_blk<NB, EV_UPPER_C>(a, s);
        case EV_UPPER_T: return launch_blk<NB, EV_UPPER_T>(a, s);
        case EV_LOWER_N: return launch_blk<NB, EV_LOWER_N>(a, s);
        case EV_LOWER_T: return launch_blk<NB, EV_LOWER_T>(a, s);
        case EV_LOWER_C: return launch_blk<NB, EV_LOWER_C>(a, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace

hipError_t launch_diag(int nb, int ev, const DiagArgs& a, hipStream_t s) {
    if (a.bs <= 0 || a.bs > nb || a.n <= 0) return hipErrorInvalidValue;
    switch (nb) {
        case 64: return launch_nb_ev<64, 4>(ev, a, s);
        case 32: return launch_nb_ev<32, 2>(ev, a, s);
        case 16: return launch_nb_ev<16, 1>(ev, a, s);
        default: return hipErrorInvalidValue;
    }
}

int block_rows_for(int n, int nb, int width, bool plain) {
    if (nb != 16 || !plain) return kRowsMax;
    BlockArgs a{};
    a.n = n;
    const int w = width ? width : auto_width(a);
    // 512-row blocks where every narrow workgroup has a compute unit to itself
    // (measured: at two per compute unit they gain nothing, or lose at m = 1024)
    return ((w == 1 || w == 2) && (n + w - 1) / w <= device_cu_count()) ? 2 * kRowsMax : kRowsMax;
}

bool block_fusable(int nb) { return nb == 16 || nb == 32; }

hipError_t launch_block(int ev, const BlockArgs& a, hipStream_t s) {
    if (a.rows <= 0 || a.rows > 2 * kRowsMax || a.n <= 0 || a.iS % a.nb) return hipErrorInvalidValue;
    if (a.rows > kRowsMax && (a.nb != 16 || a.V != nullptr)) return hipErrorInvalidValue;
    switch (a.nb) {
        case 32: return launch_blk_ev<32>(ev, a, s);
        case 16: return launch_blk_ev<16>(ev, a, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace mst
