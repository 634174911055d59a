// Bandwidth-bound helper kernels around the multi-shift solve (gfx950):
// growth-bound norms (Sec. 3), column init and final rescaling of the safe
// solve, the per-column dot product of the gradient, precision conversions,
// the triangular-eigenvector setup (Alg 6), and the Lanczos recurrence and
// tridiagonal eigenvalue of the resolvent-norm driver (Alg 7).
//
// Reductions use a fixed order (per-thread strided partials, then a fixed tree
// over the workgroup) so results are bitwise reproducible run to run.
#include "common.h"

#include <atomic>

namespace mst {
namespace {

__device__ inline double cabs1(zd z) { return fabs(z.re) + fabs(z.im); }

template <int NT>
__device__ inline double block_max(double v, double* sh) {
    for (int off = 32; off >= 1; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) sh[wave] = v;
    __syncthreads();
    double r = sh[0];
    for (int i = 1; i < NT / 64; ++i) r = fmax(r, sh[i]);
    return r;
}

// Fixed-order sum over the workgroup: butterfly within each wavefront (the
// same pairing on every run), then wave partials in index order.
template <int NT>
__device__ inline double block_sum(double v, double* sh) {
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) sh[wave] = v;
    __syncthreads();
    double r = sh[0];
    for (int i = 1; i < NT / 64; ++i) r += sh[i];
    return r;
}

// one workgroup per column c of U
__global__ __launch_bounds__(256) void k_norms(int m, const zd* U, long ldu, int nb, double* cn_in,
                                               double* above, double* colmax) {
    __shared__ double sh[8];
    const int c = blockIdx.x;
    const int bs = (c / nb) * nb;
    const zd* col = U + (long)c * ldu;
    double a = 0.0, in = 0.0;
    for (int r = threadIdx.x; r < c; r += 256) {
        const double v = cabs1(col[r]);
        if (r < bs) a = fmax(a, v); else in = fmax(in, v);
    }
    a = block_max<256>(a, sh);
    in = block_max<256>(in, sh);
    if (threadIdx.x == 0) {
        above[c] = a;
        cn_in[c] = in;
        colmax[c] = fmax(fmax(a, in), cabs1(col[c]));
    }
}

// above_sum[q] = sum over the block's columns (ascending) of above[c]; delta
__global__ __launch_bounds__(256) void k_norms2(int m, int nb, const double* above,
                                                const double* colmax, double* above_sum,
                                                double* delta) {
    __shared__ double sh[8];
    const int nblk = (m + nb - 1) / nb;
    for (int q = threadIdx.x; q < nblk; q += 256) {
        const int c1 = min((q + 1) * nb, m);
        double s = 0.0;
        for (int c = q * nb; c < c1; ++c) s = s + above[c];
        above_sum[q] = s;
    }
    double um = 0.0;
    for (int c = threadIdx.x; c < m; c += 256) um = fmax(um, colmax[c]);
    um = block_max<256>(um, sh);
    if (threadIdx.x == 0) *delta = (um > 0.0) ? ldexp(um, -52) : ldexp(1.0, -1022);
}

__global__ __launch_bounds__(256) void k_colinit(int m, int n, const zd* B, long ldb,
                                                 const int* col_len, double* G, int* kcur) {
    __shared__ double sh[8];
    const int j = blockIdx.x;
    int L = col_len ? col_len[j] : m;
    L = L < 0 ? 0 : (L > m ? m : L);
    const zd* col = B + (long)j * ldb;
    double v = 0.0;
    for (int r = threadIdx.x; r < L; r += 256) v = fmax(v, cabs1(col[r]));
    v = block_max<256>(v, sh);
    if (threadIdx.x == 0) {
        G[j] = v;
        kcur[j] = 0;
    }
}

// X(rows of block q, j) *= 2^-(k_j - kb[q][j]); s_j = 2^-k_j
__global__ __launch_bounds__(256) void k_finalize(int m, int n, int nb, zd* B, long ldb,
                                                  const int* col_len, const int* kcur,
                                                  const int* kb, double* scale, int* klog) {
    const int nrb = (m + 255) / 256 > 0 ? (m + 255) / 256 : 1;
    const int j = blockIdx.x / nrb;
    const int rb = blockIdx.x - j * nrb;
    const int r = rb * 256 + threadIdx.x;
    const int kj = kcur[j];
    if (rb == 0 && threadIdx.x == 0) {
        scale[j] = ldexp(1.0, -kj);
        if (klog) klog[j] = kj;
    }
    int L = col_len ? col_len[j] : m;
    L = L < 0 ? 0 : (L > m ? m : L);
    if (r >= L) return;
    const int d = kj - kb[(long)(r / nb) * n + j];
    if (d != 0) {
        zd* p = &B[(long)j * ldb + r];
        zd v = *p;
        *p = zd{ldexp(v.re, -d), ldexp(v.im, -d)};
    }
}

__global__ __launch_bounds__(256) void k_dot(int m, const zd* X, long ldx, const zd* Y, long ldy,
                                             zd* out) {
    __shared__ double sh[8];
    const int j = blockIdx.x;
    const zd* x = X + (long)j * ldx;
    const zd* y = Y + (long)j * ldy;
    double sr = 0.0, si = 0.0;
    for (int r = threadIdx.x; r < m; r += 256) {
        const zd a = x[r], b = y[r];
        // conj(a) * b
        sr += a.re * b.re + a.im * b.im;
        si += a.re * b.im - a.im * b.re;
    }
    sr = block_sum<256>(sr, sh);
    si = block_sum<256>(si, sh);
    if (threadIdx.x == 0) out[j] = zd{sr, si};
}

__global__ __launch_bounds__(256) void k_to_f32(int rows, int cols, const zd* src, long lds, zf* dst,
                                                long ldd, int upper_only) {
    const long total = (long)rows * cols;
    for (long e = (long)blockIdx.x * 256 + threadIdx.x; e < total; e += (long)gridDim.x * 256) {
        const int c = (int)(e / rows), r = (int)(e - (long)c * rows);
        zf v{0.f, 0.f};
        if (!upper_only || r <= c) {
            const zd s = src[(long)c * lds + r];
            v = zf{(float)s.re, (float)s.im};
        }
        dst[(long)c * ldd + r] = v;
    }
}

__global__ __launch_bounds__(256) void k_copy(int rows, int cols, const zd* src, long lds, zd* dst,
                                              long ldd) {
    const long total = (long)rows * cols;
    for (long e = (long)blockIdx.x * 256 + threadIdx.x; e < total; e += (long)gridDim.x * 256) {
        const int c = (int)(e / rows), r = (int)(e - (long)c * rows);
        dst[(long)c * ldd + r] = src[(long)c * lds + r];
    }
}

__global__ __launch_bounds__(256) void k_axpy(int rows, int cols, const zd* D, long ldd, zd* X,
                                              long ldx) {
    const long total = (long)rows * cols;
    for (long e = (long)blockIdx.x * 256 + threadIdx.x; e < total; e += (long)gridDim.x * 256) {
        const int c = (int)(e / rows), r = (int)(e - (long)c * rows);
        const zd d = D[(long)c * ldd + r];
        zd* p = &X[(long)c * ldx + r];
        const zd x = *p;
        *p = zd{x.re + d.re, x.im + d.im};
    }
}

// Alg 6 setup: eig = diag(T); Z = -T above the diagonal, 0 on and below; col_len[j] = j
__global__ __launch_bounds__(256) void k_triang_setup(int m, const zd* T, long ldt, zd* Z, long ldz,
                                                      zd* eig, int* col_len) {
    const int nrb = (m + 255) / 256;
    const int j = blockIdx.x / nrb;
    const int r = (blockIdx.x - j * nrb) * 256 + threadIdx.x;
    if (r >= m) return;
    zd v{0.0, 0.0};
    if (r < j) {
        const zd t = T[(long)j * ldt + r];
        v = zd{-t.re, -t.im};
    }
    Z[(long)j * ldz + r] = v;
    if (r == j) {
        eig[j] = T[(long)j * ldt + j];
        col_len[j] = j;
    }
}

// GeneralizedTriangEig set-up (appendix, Alg 10): lambda_j = T(j,j) / S(j,j)
// (scaled complex division: S(j,j) = 2^e d', T/S = 2^-e T conj(d') / |d'|^2);
// Z(r, j) = -T(r, j) + lambda_j S(r, j) for r < j, zero elsewhere.
__global__ __launch_bounds__(256) void k_gen_triang_setup(int m, const zd* T, long ldt, const zd* S,
                                                          long lds, zd* Z, long ldz, zd* eig,
                                                          int* col_len) {
#pragma clang fp contract(off)
    const int nrb = (m + 255) / 256;
    const int j = blockIdx.x / nrb;
    const int r = (blockIdx.x - j * nrb) * 256 + threadIdx.x;
    if (r >= m) return;
    const zd t = T[(long)j * ldt + j], d = S[(long)j * lds + j];
    const double am = fmax(fabs(d.re), fabs(d.im));
    const int e = (am > 0.0) ? ilogb(am) : 0;
    const double sr = ldexp(d.re, -e), si = ldexp(d.im, -e);
    const double den = sr * sr + si * si;
    const zd lam{ldexp((t.re * sr + t.im * si) / den, -e), ldexp((t.im * sr - t.re * si) / den, -e)};
    zd v{0.0, 0.0};
    if (r < j) {
        const zd tr = T[(long)j * ldt + r], sv = S[(long)j * lds + r];
        v = zd{(lam.re * sv.re - lam.im * sv.im) - tr.re, (lam.re * sv.im + lam.im * sv.re) - tr.im};
    }
    Z[(long)j * ldz + r] = v;
    if (r == j) {
        eig[j] = lam;
        col_len[j] = j;
    }
}

__global__ __launch_bounds__(256) void k_triang_diag(int m, zd* Z, long ldz, const double* scale) {
    const int j = blockIdx.x * 256 + threadIdx.x;
    if (j < m) Z[(long)j * ldz + j] = zd{scale[j], 0.0};
}

__global__ __launch_bounds__(256) void k_normalize(int m, zd* V, long ldv) {
    __shared__ double sh[8];
    const int j = blockIdx.x;
    zd* v = V + (long)j * ldv;
    double s = 0.0;
    for (int r = threadIdx.x; r < m; r += 256) s += v[r].re * v[r].re + v[r].im * v[r].im;
    s = block_sum<256>(s, sh);
    const double inv = 1.0 / sqrt(s);
    for (int r = threadIdx.x; r < m; r += 256) v[r] = zd{v[r].re * inv, v[r].im * inv};
}

// One Lanczos step for column j, given W = A V:
//   alpha = Re(v^H w); w -= alpha v + beta_prev vprev; beta = ||w||; w /= beta
__global__ __launch_bounds__(256) void k_lanczos(int m, int it, int iters, const zd* V, long ldv,
                                                 zd* W, long ldw, const zd* Vp, long ldp,
                                                 double* alpha, double* beta, int* steps) {
    __shared__ double sh[8];
    const int j = blockIdx.x;
    const zd* v = V + (long)j * ldv;
    zd* w = W + (long)j * ldw;
    const zd* vp = Vp + (long)j * ldp;
    const bool stopped = steps[j] <= it;   // beta hit zero at an earlier step
    double a = 0.0;
    for (int r = threadIdx.x; r < m; r += 256) a += v[r].re * w[r].re + v[r].im * w[r].im;
    a = block_sum<256>(a, sh);
    const double bprev = (it > 0) ? beta[(long)j * iters + it - 1] : 0.0;
    double s = 0.0;
    for (int r = threadIdx.x; r < m; r += 256) {
        const zd x = w[r], y = v[r], z = vp[r];
        const zd o{x.re - a * y.re - bprev * z.re, x.im - a * y.im - bprev * z.im};
        w[r] = o;
        s += o.re * o.re + o.im * o.im;
    }
    s = block_sum<256>(s, sh);
    const double b = sqrt(s);
    const double inv = (b > 0.0) ? 1.0 / b : 0.0;
    for (int r = threadIdx.x; r < m; r += 256) w[r] = zd{w[r].re * inv, w[r].im * inv};
    if (threadIdx.x == 0) {
        alpha[(long)j * iters + it] = stopped ? 0.0 : a;
        beta[(long)j * iters + it] = stopped ? 0.0 : b;
        if (!stopped && b == 0.0) steps[j] = it + 1;
    }
}

// Largest eigenvalue of the Lanczos tridiagonal by bisection on the Sturm
// count (number of negative pivots of T - x I), then sigma = theta^-1/2.
__global__ __launch_bounds__(256) void k_tridiag(int n, int iters, const double* alpha,
                                                 const double* beta, const int* steps,
                                                 double* sigma) {
    const int j = blockIdx.x * 256 + threadIdx.x;
    if (j >= n) return;
    const double* a = alpha + (long)j * iters;
    const double* b = beta + (long)j * iters;
    const int s = steps[j];
    double lo = a[0], hi = a[0];
    for (int i = 0; i < s; ++i) {
        const double off = (i > 0 ? fabs(b[i - 1]) : 0.0) + (i + 1 < s ? fabs(b[i]) : 0.0);
        lo = fmin(lo, a[i] - off);
        hi = fmax(hi, a[i] + off);
    }
    double bmax = 0.0;
    for (int i = 0; i + 1 < s; ++i) bmax = fmax(bmax, fabs(b[i]));
    const double pivmin = fmax(1e-300, 2.2250738585072014e-308 * fmax(1.0, bmax * bmax));
    // count of eigenvalues < x
    auto count_below = [&](double x) {
        int c = 0;
        double d = a[0] - x;
        if (fabs(d) < pivmin) d = -pivmin;
        if (d < 0) ++c;
        for (int i = 1; i < s; ++i) {
            d = (a[i] - x) - (b[i - 1] * b[i - 1]) / d;
            if (fabs(d) < pivmin) d = -pivmin;
            if (d < 0) ++c;
        }
        return c;
    };
    const double span = fmax(hi - lo, fabs(hi)) + 1e-300;
    hi += 1e-14 * span;
    lo -= 1e-14 * span;
    for (int it = 0; it < 200; ++it) {
        const double mid = 0.5 * (lo + hi);
        if (mid <= lo || mid >= hi) break;
        if (count_below(mid) >= s) hi = mid; else lo = mid;
    }
    sigma[j] = 1.0 / sqrt(0.5 * (lo + hi));
}

__global__ __launch_bounds__(256) void k_fill_int(int n, int v, int* p) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ __launch_bounds__(256) void k_zero(long count, zd* p) {
    for (long e = (long)blockIdx.x * 256 + threadIdx.x; e < count; e += (long)gridDim.x * 256)
        p[e] = zd{0.0, 0.0};
}

// ---------------------------------------------------------------- iterative refinement

__device__ inline double cmod(zd z) { return hypot(z.re, z.im); }

// partial row sums of |U(i,k)|, k > i, over the column chunk blockIdx.y
__global__ __launch_bounds__(256) void k_rowabs_part(int m, const zd* U, long ldu, double* part) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= m) return;
    const int c0 = blockIdx.y * kRowChunk, c1 = min(m, c0 + kRowChunk);
    double acc = 0.0;
    for (int c = max(c0, i + 1); c < c1; ++c) acc += cmod(U[(long)c * ldu + i]);
    part[(long)blockIdx.y * m + i] = acc;
}

__global__ __launch_bounds__(256) void k_rowabs_sum(int m, int nch, const zd* U, long ldu,
                                                    const double* part, double* rowoff, zd* udiag) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= m) return;
    double acc = 0.0;
    for (int ch = 0; ch < nch; ++ch) acc += part[(long)ch * m + i];
    rowoff[i] = acc;
    udiag[i] = U[(long)i * ldu + i];
}

__global__ __launch_bounds__(256) void k_colstats(int m, const zd* R, long ldr, const zd* X, long ldx,
                                                  const double* rowoff, const zd* udiag, const zd* lam,
                                                  int* e, double* rel, const int* skip) {
    if (skip && *skip) return;
    __shared__ double sh[8];
    const int j = blockIdx.x;
    const zd* rc = R + (long)j * ldr;
    double c1 = 0.0, rm = 0.0, xm = 0.0, am = 0.0;
    bool bad = false;
    const zd lj = X ? lam[j] : zd{0.0, 0.0};
    for (int r = threadIdx.x; r < m; r += 256) {
        const zd v = rc[r];
        const double a = cabs1(v);
        bad = bad || !isfinite(a);
        c1 = fmax(c1, a);
        if (X) {
            const zd x = X[(long)j * ldx + r];
            bad = bad || !isfinite(cabs1(x));
            rm = fmax(rm, cmod(v));
            xm = fmax(xm, cmod(x));
            const zd d = udiag[r];
            am = fmax(am, rowoff[r] + cmod(zd{d.re - lj.re, d.im - lj.im}));
        }
    }
    c1 = block_max<256>(c1, sh);
    const double fb = block_max<256>(bad ? 1.0 : 0.0, sh);
    if (X) {
        rm = block_max<256>(rm, sh);
        xm = block_max<256>(xm, sh);
        am = block_max<256>(am, sh);
    }
    if (threadIdx.x == 0) {
        const bool ok = fb == 0.0;
        e[j] = (ok && c1 > 0.0) ? ilogb(c1) : 0;
        if (X) {
            double q = xm > 0.0 ? rm / (am * xm) : rm;
            if (!ok || !(q >= 0.0) || !isfinite(am)) q = INFINITY;
            rel[j] = q;
        }
    }
}

__global__ __launch_bounds__(256) void k_to_f32_cols(int rows, int cols, const zd* src, long lds,
                                                     const int* e, zf* dst, long ldd, const int* skip) {
    if (skip && *skip) return;
    const long total = (long)rows * cols;
    for (long t = (long)blockIdx.x * 256 + threadIdx.x; t < total; t += (long)gridDim.x * 256) {
        const int c = (int)(t / rows), r = (int)(t - (long)c * rows);
        const zd v = src[(long)c * lds + r];
        const int k = e[c];
        dst[(long)c * ldd + r] = zf{(float)ldexp(v.re, -k), (float)ldexp(v.im, -k)};
    }
}

__global__ __launch_bounds__(256) void k_axpy_cols(int rows, int cols, const zd* D, long ldd,
                                                   const int* e, double sign, zd* X, long ldx,
                                                   const int* skip, const int* cond) {
    if (skip && *skip) return;
    if (cond && *cond != 1) return;
    const long total = (long)rows * cols;
    for (long t = (long)blockIdx.x * 256 + threadIdx.x; t < total; t += (long)gridDim.x * 256) {
        const int c = (int)(t / rows), r = (int)(t - (long)c * rows);
        const zd d = D[(long)c * ldd + r];
        const int k = e[c];
        zd* p = &X[(long)c * ldx + r];
        const zd x = *p;
        *p = zd{x.re + sign * ldexp(d.re, k), x.im + sign * ldexp(d.im, k)};
    }
}

__global__ __launch_bounds__(256) void k_copy_cond(int rows, int cols, const zd* src, long lds, zd* dst,
                                                   long ldd, const int* skip, const int* cond) {
    if (skip && *skip) return;
    if (cond && *cond != 1) return;
    const long total = (long)rows * cols;
    for (long t = (long)blockIdx.x * 256 + threadIdx.x; t < total; t += (long)gridDim.x * 256) {
        const int c = (int)(t / rows), r = (int)(t - (long)c * rows);
        dst[(long)c * ldd + r] = src[(long)c * lds + r];
    }
}

__global__ __launch_bounds__(256) void k_scale_cols(int rows, int cols, zd* X, long ldx, const int* e) {
    const long total = (long)rows * cols;
    for (long t = (long)blockIdx.x * 256 + threadIdx.x; t < total; t += (long)gridDim.x * 256) {
        const int c = (int)(t / rows), r = (int)(t - (long)c * rows);
        zd* p = &X[(long)c * ldx + r];
        const zd x = *p;
        *p = zd{ldexp(x.re, e[c]), ldexp(x.im, e[c])};
    }
}

__global__ __launch_bounds__(64) void k_refine_init(RefineCtl* ctl, double* report, int nrep) {
    const int t = threadIdx.x;
    if (t == 0) {
        ctl->stop = 0;
        for (int i = 0; i <= kMaxSweeps; ++i) ctl->rb[i] = 0;
        ctl->prev = INFINITY;
    }
    if (report && t < nrep) report[t] = -1.0;
}

__global__ __launch_bounds__(256) void k_refine_ctl(int n, int t, const double* rel, double tol,
                                                    RefineCtl* ctl, double* report) {
    __shared__ double sh[8];
    if (ctl->stop) return;
    double v = 0.0;
    for (int j = threadIdx.x; j < n; j += 256) v = fmax(v, rel[j]);
    const double res = block_max<256>(v, sh);
    if (threadIdx.x == 0) {
        if (report) report[t] = res;
        if (res <= tol) {
            ctl->stop = 1;
        } else if (t > 0 && !(res < ctl->prev)) {
            ctl->stop = 1;
            ctl->rb[t] = 1;
        }
        ctl->prev = res;
    }
}

inline int grid_for(long total) {
    long g = (total + 255) / 256;
    return (int)(g > 65536 ? 65536 : (g < 1 ? 1 : g));
}

}  // namespace

hipError_t launch_fill_int(int n, int v, int* p, hipStream_t s) {
    hipLaunchKernelGGL(k_fill_int, dim3((n + 255) / 256), dim3(256), 0, s, n, v, p);
    return hipGetLastError();
}

hipError_t launch_zero(long count, zd* p, hipStream_t s) {
    hipLaunchKernelGGL(k_zero, dim3(grid_for(count)), dim3(256), 0, s, count, p);
    return hipGetLastError();
}

hipError_t launch_rowabs(int m, const zd* U, long ldu, double* part, double* rowoff, zd* udiag,
                         hipStream_t s) {
    const int nch = (m + kRowChunk - 1) / kRowChunk;
    hipLaunchKernelGGL(k_rowabs_part, dim3((m + 255) / 256, nch), dim3(256), 0, s, m, U, ldu, part);
    hipLaunchKernelGGL(k_rowabs_sum, dim3((m + 255) / 256), dim3(256), 0, s, m, nch, U, ldu, part, rowoff,
                       udiag);
    return hipGetLastError();
}

hipError_t launch_colstats(int m, int n, const zd* R, long ldr, const zd* X, long ldx,
                           const double* rowoff, const zd* udiag, const zd* lam, int* e, double* rel,
                           const int* skip, hipStream_t s) {
    hipLaunchKernelGGL(k_colstats, dim3(n), dim3(256), 0, s, m, R, ldr, X, ldx, rowoff, udiag, lam, e, rel,
                       skip);
    return hipGetLastError();
}

hipError_t launch_to_f32_cols(int rows, int cols, const zd* src, long lds, const int* e, zf* dst,
                              long ldd, const int* skip, hipStream_t s) {
    hipLaunchKernelGGL(k_to_f32_cols, dim3(grid_for((long)rows * cols)), dim3(256), 0, s, rows, cols, src,
                       lds, e, dst, ldd, skip);
    return hipGetLastError();
}

hipError_t launch_axpy_cols(int rows, int cols, const zd* D, long ldd, const int* e, double sign,
                            zd* X, long ldx, const int* skip, const int* cond, hipStream_t s) {
    hipLaunchKernelGGL(k_axpy_cols, dim3(grid_for((long)rows * cols)), dim3(256), 0, s, rows, cols, D, ldd,
                       e, sign, X, ldx, skip, cond);
    return hipGetLastError();
}

hipError_t launch_copy_cond(int rows, int cols, const zd* src, long lds, zd* dst, long ldd,
                            const int* skip, const int* cond, hipStream_t s) {
    hipLaunchKernelGGL(k_copy_cond, dim3(grid_for((long)rows * cols)), dim3(256), 0, s, rows, cols, src, lds,
                       dst, ldd, skip, cond);
    return hipGetLastError();
}

hipError_t launch_scale_cols(int rows, int cols, zd* X, long ldx, const int* e, hipStream_t s) {
    hipLaunchKernelGGL(k_scale_cols, dim3(grid_for((long)rows * cols)), dim3(256), 0, s, rows, cols, X, ldx,
                       e);
    return hipGetLastError();
}

hipError_t launch_refine_init(RefineCtl* ctl, double* report, int nrep, hipStream_t s) {
    hipLaunchKernelGGL(k_refine_init, dim3(1), dim3(64), 0, s, ctl, report, nrep);
    return hipGetLastError();
}

hipError_t launch_refine_ctl(int n, int t, const double* rel, double tol, RefineCtl* ctl,
                             double* report, hipStream_t s) {
    hipLaunchKernelGGL(k_refine_ctl, dim3(1), dim3(256), 0, s, n, t, rel, tol, ctl, report);
    return hipGetLastError();
}

hipError_t launch_norms(int m, const zd* U, long ldu, int nb, double* cn_in, double* above,
                        double* colmax, double* above_sum, double* delta, hipStream_t s) {
    if (m > 0) hipLaunchKernelGGL(k_norms, dim3(m), dim3(256), 0, s, m, U, ldu, nb, cn_in, above, colmax);
    hipLaunchKernelGGL(k_norms2, dim3(1), dim3(256), 0, s, m, nb, above, colmax, above_sum, delta);
    return hipGetLastError();
}

hipError_t launch_colinit(int m, int n, const zd* B, long ldb, const int* col_len, double* G,
                          int* kcur, hipStream_t s) {
    hipLaunchKernelGGL(k_colinit, dim3(n), dim3(256), 0, s, m, n, B, ldb, col_len, G, kcur);
    return hipGetLastError();
}

hipError_t launch_finalize(int m, int n, int nb, zd* B, long ldb, const int* col_len,
                           const int* kcur, const int* kb, double* scale, int* klog,
                           hipStream_t s) {
    const dim3 grid(((m + 255) / 256 > 0 ? (m + 255) / 256 : 1) * n);
    hipLaunchKernelGGL(k_finalize, grid, dim3(256), 0, s, m, n, nb, B, ldb, col_len, kcur, kb, scale, klog);
    return hipGetLastError();
}

hipError_t launch_dot(int m, int n, const zd* X, long ldx, const zd* Y, long ldy, zd* out,
                      hipStream_t s) {
    hipLaunchKernelGGL(k_dot, dim3(n), dim3(256), 0, s, m, X, ldx, Y, ldy, out);
    return hipGetLastError();
}

hipError_t launch_to_f32(int rows, int cols, const zd* src, long lds, zf* dst, long ldd,
                         bool upper_only, hipStream_t s) {
    hipLaunchKernelGGL(k_to_f32, dim3(grid_for((long)rows * cols)), dim3(256), 0, s, rows, cols, src,
                       lds, dst, ldd, upper_only ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_copy(int rows, int cols, const zd* src, long lds, zd* dst, long ldd, hipStream_t s) {
    hipLaunchKernelGGL(k_copy, dim3(grid_for((long)rows * cols)), dim3(256), 0, s, rows, cols, src, lds,
                       dst, ldd);
    return hipGetLastError();
}

hipError_t launch_axpy_inplace(int rows, int cols, const zd* D, long ldd, zd* X, long ldx,
                               hipStream_t s) {
    hipLaunchKernelGGL(k_axpy, dim3(grid_for((long)rows * cols)), dim3(256), 0, s, rows, cols, D, ldd,
                       X, ldx);
    return hipGetLastError();
}

hipError_t launch_triang_setup(int m, const zd* T, long ldt, zd* Z, long ldz, zd* eig, int* col_len,
                               hipStream_t s) {
    const dim3 grid(((m + 255) / 256) * m);
    hipLaunchKernelGGL(k_triang_setup, grid, dim3(256), 0, s, m, T, ldt, Z, ldz, eig, col_len);
    return hipGetLastError();
}

hipError_t launch_gen_triang_setup(int m, const zd* T, long ldt, const zd* S, long lds, zd* Z, long ldz,
                                   zd* eig, int* col_len, hipStream_t s) {
    const dim3 grid(((m + 255) / 256) * m);
    hipLaunchKernelGGL(k_gen_triang_setup, grid, dim3(256), 0, s, m, T, ldt, S, lds, Z, ldz, eig, col_len);
    return hipGetLastError();
}

hipError_t launch_triang_diag(int m, zd* Z, long ldz, const double* scale, hipStream_t s) {
    hipLaunchKernelGGL(k_triang_diag, dim3((m + 255) / 256), dim3(256), 0, s, m, Z, ldz, scale);
    return hipGetLastError();
}

hipError_t launch_normalize_cols(int m, int n, zd* V, long ldv, hipStream_t s) {
    hipLaunchKernelGGL(k_normalize, dim3(n), dim3(256), 0, s, m, V, ldv);
    return hipGetLastError();
}

hipError_t launch_lanczos_step(int m, int n, int it, int iters, const zd* V, long ldv, zd* W,
                               long ldw, const zd* Vprev, long ldp, double* alpha, double* beta,
                               int* steps, hipStream_t s) {
    hipLaunchKernelGGL(k_lanczos, dim3(n), dim3(256), 0, s, m, it, iters, V, ldv, W, ldw, Vprev, ldp,
                       alpha, beta, steps);
    return hipGetLastError();
}

hipError_t launch_tridiag_max(int n, int iters, const double* alpha, const double* beta,
                              const int* steps, double* sigma, hipStream_t s) {
    hipLaunchKernelGGL(k_tridiag, dim3((n + 255) / 256), dim3(256), 0, s, n, iters, alpha, beta, steps,
                       sigma);
    return hipGetLastError();
}

int device_cu_count() {
    static std::atomic<int> cus[64];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
    int c = cus[dev].load(std::memory_order_relaxed);
    if (c <= 0) {
        if (hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || c <= 0)
            c = 256;
        cus[dev].store(c, std::memory_order_relaxed);
    }
    return c;
}

}  // namespace mst
