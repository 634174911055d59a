// Thick-restart Lanczos for sigma_min(U - z_j I) of many shifts at once (the
// Krylov part of the second stage of Alg 7, Sec. 5, with restarts and a
// per-shift tolerance; Wu and Simon's thick restart), for gfx950. The
// operator products are multi-shift solves over the shifts still running
// (api.hip); the kernels here do the rest of each step and of each cycle:
//   k_trl_gather   the Lanczos vector q_i of every running shift into a
//                  dense block (the solves' right-hand sides);
//   k_trl_orth     one workgroup per running shift: removes the three-term
//                  predecessor (or, right after a restart, the arrowhead
//                  border), alpha, two passes of classical Gram-Schmidt
//                  against the whole basis, beta, q_{i+1};
//   k_trl_ritz     one wavefront per running shift: Jacobi eigensolver of the
//                  projected matrix in LDS, the top Ritz value, its residual
//                  estimate and the convergence test, the restart border;
//   k_trl_restart  the kept Ritz vectors Q S(:, 0:keep) and the last Lanczos
//                  vector as the first keep + 1 basis vectors;
//   k_trl_compact  the running shifts that did not converge, in order.
// Reductions have a fixed order, so results are reproducible run to run.
#include "common.h"

namespace mst {
namespace {

constexpr int kT = 256;     // threads of the per-shift workgroups
constexpr int kChunk = 8;   // basis vectors per reduction
constexpr int kMaxBasis = 33;   // kdim + 1 for the largest basis (kdim <= 32)
constexpr int kMaxKeep = 16;    // Ritz vectors kept at a restart

// Fixed-order sums of NV values over the workgroup: butterfly in each
// wavefront, then the wavefronts' partials in index order.
template <int NV>
__device__ inline void block_sums(double (&v)[NV], double* sh) {
#pragma unroll
    for (int k = 0; k < NV; ++k)
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) v[k] += __shfl_xor(v[k], off, 64);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0)
#pragma unroll
        for (int k = 0; k < NV; ++k) sh[wave * NV + k] = v[k];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        double r = sh[k];
        for (int w = 1; w < kT / 64; ++w) r += sh[w * NV + k];
        v[k] = r;
    }
}

// one workgroup per running shift
__global__ __launch_bounds__(kT) void k_trl_gather(int m, int nact, const int* idx, const zd* Qi, long ldq,
                                                   zd* W, long ldw, const zd* z, zd* zact) {
    const int c = blockIdx.x;
    const int j = idx[c];
    if (threadIdx.x == 0) zact[c] = z[j];
    for (int r = threadIdx.x; r < m; r += kT) W[(long)c * ldw + r] = Qi[(long)j * ldq + r];
}

// Column c of W holds A q_i of shift j = idx[c]. Q: kdim + 1 blocks of m x N
// (block l at Q + l * qs, leading dimension ldq); H: kdim x kdim per shift
// (row-major at H + j * kdim * kdim). Five passes over the vectors:
//   1. w -= the arrowhead border sum_{l<k0} H(l, k0) q_l (first step after a
//      restart) or beta_{i-1} q_{i-1}; alpha = Re(q_i^H w);
//   2. w -= alpha q_i; h = Q^H w over q_0..q_i (first Gram-Schmidt pass);
//   3. w -= Q h; h' = Q^H w (second pass);
//   4. w -= Q h'; beta^2 = ||w||^2;
//   5. q_{i+1} = w / beta;
// with alpha + Re(h_i) + Re(h'_i) the diagonal entry of the projection.
__global__ __launch_bounds__(kT) void k_trl_orth(int m, int i, int k0, int kdim, const int* idx, zd* W,
                                                 long ldw, zd* Q, long ldq, long qs, double* H,
                                                 double* beta_out, int* steps) {
    __shared__ double sh[(kT / 64) * 2 * kChunk];
    __shared__ double coef[2 * kMaxBasis];
    const int c = blockIdx.x, j = idx[c];
    zd* w = W + (long)c * ldw;
    const zd* qj = Q + (long)j * ldq;   // basis vector l of shift j at qj + l * qs
    double* Hj = H + (long)j * kdim * kdim;
    const int t = threadIdx.x;

    // v -= sum_l coef_l q_l over l = 0..i, in that order; the basis entries
    // are loaded four at a time so that each thread keeps several loads in
    // flight (one at a time leaves the stream short of HBM bandwidth)
    auto sub_basis = [&](zd& v, int r) __attribute__((always_inline)) {
        int l = 0;
        for (; l + 4 <= i + 1; l += 4) {
            zd q[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) q[u] = qj[(l + u) * qs + r];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const double hr = coef[2 * (l + u)], hi = coef[2 * (l + u) + 1];
                v.re -= hr * q[u].re - hi * q[u].im;
                v.im -= hr * q[u].im + hi * q[u].re;
            }
        }
        for (; l <= i; ++l) {
            const zd q = qj[l * qs + r];
            const double hr = coef[2 * l], hi = coef[2 * l + 1];
            v.re -= hr * q.re - hi * q.im;
            v.im -= hr * q.im + hi * q.re;
        }
    };

    // pass 1
    const bool border = (i == k0) && (k0 > 0);
    const int l0 = border ? 0 : i - 1, l1 = border ? k0 : i;   // vectors removed: [l0, l1)
    double a[1] = {0.0};
    for (int r = t; r < m; r += kT) {
        zd v = w[r];
        for (int l = (l0 > 0 ? l0 : 0); l < l1; ++l) {
            const double cl = border ? Hj[l * kdim + k0] : Hj[(i - 1) * kdim + i];
            const zd q = qj[l * qs + r];
            v.re -= cl * q.re;
            v.im -= cl * q.im;
        }
        w[r] = v;
        const zd q = qj[i * qs + r];
        a[0] += q.re * v.re + q.im * v.im;
    }
    block_sums<1>(a, sh);
    const double alpha = a[0];
    double diag = alpha;

    // passes 2 and 3: subtract (alpha q_i, then h), then the dot products with q_0..q_i
    for (int pass = 0; pass < 2; ++pass) {
        for (int ch = 0; ch <= i; ch += kChunk) {
            const int nl = min(kChunk, i + 1 - ch);
            double h[2 * kChunk];
#pragma unroll
            for (int k = 0; k < 2 * kChunk; ++k) h[k] = 0.0;
            for (int r = t; r < m; r += kT) {
                zd v = w[r];
                if (ch == 0) {
                    if (pass == 0) {
                        const zd q = qj[i * qs + r];
                        v.re -= alpha * q.re;
                        v.im -= alpha * q.im;
                    } else {
                        sub_basis(v, r);
                    }
                    w[r] = v;
                }
#pragma unroll
                for (int k = 0; k < kChunk; ++k) {
                    if (k < nl) {
                        const zd q = qj[(ch + k) * qs + r];
                        h[2 * k] += q.re * v.re + q.im * v.im;
                        h[2 * k + 1] += q.re * v.im - q.im * v.re;
                    }
                }
            }
            block_sums<2 * kChunk>(h, sh);
            // coef is read by every thread in this pass's subtraction (ch == 0):
            // all of them are past it once block_sums has synchronised
            if (t < 2 * nl) coef[2 * ch + t] = h[t];
            __syncthreads();
        }
        diag += coef[2 * i];
        __syncthreads();
    }

    // pass 4: w -= Q h'; beta
    double b2[1] = {0.0};
    for (int r = t; r < m; r += kT) {
        zd v = w[r];
        sub_basis(v, r);
        w[r] = v;
        b2[0] += v.re * v.re + v.im * v.im;
    }
    block_sums<1>(b2, sh);
    const double beta = sqrt(b2[0]);
    const double inv = beta > 0.0 ? 1.0 / beta : 1.0;

    // pass 5
    zd* qn = Q + (long)(i + 1) * qs + (long)j * ldq;
    for (int r = t; r < m; r += kT) {
        const zd v = w[r];
        qn[r] = zd{v.re * inv, v.im * inv};
    }
    if (t == 0) {
        Hj[i * kdim + i] = diag;
        if (i + 1 < kdim) {
            Hj[i * kdim + i + 1] = beta;
            Hj[(i + 1) * kdim + i] = beta;
        }
        beta_out[j] = beta;
        steps[j] += 1;
    }
}

// One wavefront per running shift: Jacobi eigensolver of the symmetric
// projected matrix (kdim <= 32, in LDS) in the parallel (tournament) order:
// each step rotates kdim/2 disjoint index pairs at once (the rows of all pairs,
// then their columns and the eigenvector columns), so a sweep is kdim - 1
// steps of two barriers; eigenvalues sorted descending with their vectors;
// sigma = theta_0^-1/2, resid = |beta S(kdim-1, 0)| / theta_0, the
// convergence test, and for a shift that goes on, the restart: H becomes
// diag(theta_0..theta_{keep-1}) bordered by beta S(kdim-1, l) in row and
// column keep, and S(:, 0:keep) is stored for k_trl_restart.
constexpr int kMaxK = kMaxBasis - 1;
__global__ __launch_bounds__(64) void k_trl_ritz(int kdim, int keep, double tol, int last, const int* idx,
                                                 double* H, const double* beta, double* Sout,
                                                 double* sigma, double* resid, int* conv, int* go) {
    __shared__ double A[kMaxK * kMaxK];
    __shared__ double S[kMaxK * kMaxK];
    __shared__ double th[kMaxK];
    __shared__ int ord[kMaxK];
    __shared__ double rc[kMaxK / 2], rs[kMaxK / 2];
    __shared__ int rp[kMaxK / 2], rq[kMaxK / 2];
    const int c = blockIdx.x, j = idx[c], t = threadIdx.x;
    double* Hj = H + (long)j * kdim * kdim;
    for (int e = t; e < kdim * kdim; e += 64) {
        A[e] = Hj[e];
        S[e] = ((e / kdim) == (e % kdim)) ? 1.0 : 0.0;
    }
    const int np = (kdim + 1) & ~1;   // players of the tournament (a dummy when kdim is odd)
    const int npair = np / 2;
    __syncthreads();
    double prev = -1.0;   // off-diagonal mass before the last sweep
    for (int sweep = 0; sweep < 60; ++sweep) {
        // off-diagonal and diagonal mass (fixed-order wavefront sums)
        double off = 0.0, dia = 0.0;
        for (int e = t; e < kdim * kdim; e += 64) {
            const double v = A[e] * A[e];
            if ((e / kdim) != (e % kdim)) off += v; else dia += v;
        }
        for (int o = 32; o >= 1; o >>= 1) {
            off += __shfl_xor(off, o, 64);
            dia += __shfl_xor(dia, o, 64);
        }
        // converged; or the off-diagonal mass has reached the rounding floor
        // (about (kdim eps)^2 of the diagonal's) and stopped falling, where
        // further sweeps only move rounding errors around
        if (!(off > 1e-32 * dia) || (off <= 1e-24 * dia && prev >= 0.0 && off >= 0.5 * prev)) break;
        prev = off;
        for (int step = 0; step < np - 1; ++step) {
            // pairs of this step: player 0 against rotating player step + 1, and
            // the others folded around the circle of players 1 .. np - 1
            if (t < npair) {
                int a, b;
                if (t == 0) {
                    a = 0;
                    b = 1 + step % (np - 1);
                } else {
                    a = 1 + (step + t) % (np - 1);
                    b = 1 + (step + np - 1 - t) % (np - 1);
                }
                const int p = a < b ? a : b, q = a < b ? b : a;
                double cs = 1.0, sn = 0.0;
                if (q < kdim) {
                    const double apq = A[p * kdim + q];
                    if (apq != 0.0) {
                        const double app = A[p * kdim + p], aqq = A[q * kdim + q];
                        const double tau = (aqq - app) / (2.0 * apq);
                        const double tt = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
                        cs = 1.0 / sqrt(1.0 + tt * tt);
                        sn = tt * cs;
                    }
                }
                rp[t] = p;
                rq[t] = q;
                rc[t] = cs;
                rs[t] = sn;
            }
            __syncthreads();
            // rows p and q of every pair (disjoint pairs: no element is touched twice)
            for (int e = t; e < npair * kdim; e += 64) {
                const int k = e / kdim, col = e - k * kdim;
                const int p = rp[k], q = rq[k];
                if (q >= kdim || rs[k] == 0.0) continue;
                const double cs = rc[k], sn = rs[k];
                const double a_p = A[p * kdim + col], a_q = A[q * kdim + col];
                A[p * kdim + col] = cs * a_p - sn * a_q;
                A[q * kdim + col] = sn * a_p + cs * a_q;
            }
            __syncthreads();
            // columns p and q of every pair, and of the eigenvector matrix
            for (int e = t; e < npair * kdim; e += 64) {
                const int k = e / kdim, row = e - k * kdim;
                const int p = rp[k], q = rq[k];
                if (q >= kdim || rs[k] == 0.0) continue;
                const double cs = rc[k], sn = rs[k];
                const double a_p = A[row * kdim + p], a_q = A[row * kdim + q];
                A[row * kdim + p] = cs * a_p - sn * a_q;
                A[row * kdim + q] = sn * a_p + cs * a_q;
                const double s_p = S[row * kdim + p], s_q = S[row * kdim + q];
                S[row * kdim + p] = cs * s_p - sn * s_q;
                S[row * kdim + q] = sn * s_p + cs * s_q;
            }
            __syncthreads();
        }
    }
    if (t < kdim) th[t] = A[t * kdim + t];
    __syncthreads();
    if (t == 0) {
        // order by descending eigenvalue (stable selection)
        bool used[kMaxK];
        for (int k = 0; k < kdim; ++k) used[k] = false;
        for (int k = 0; k < kdim; ++k) {
            int best = -1;
            for (int e = 0; e < kdim; ++e)
                if (!used[e] && (best < 0 || th[e] > th[best])) best = e;
            used[best] = true;
            ord[k] = best;
        }
    }
    __syncthreads();
    const double th0 = th[ord[0]];
    const double bj = beta[j];
    const double res = fabs(bj * S[(kdim - 1) * kdim + ord[0]]);
    const bool done = res <= tol * th0;
    if (t == 0) {
        sigma[j] = 1.0 / sqrt(th0);
        resid[j] = res / th0;
        conv[j] = done ? 1 : 0;
        go[c] = (!done && !last) ? 1 : 0;
    }
    if (done || last) return;
    for (int e = t; e < kdim * keep; e += 64) {
        const int r = e / keep, l = e % keep;
        Sout[(long)j * kdim * keep + e] = S[r * kdim + ord[l]];
    }
    for (int e = t; e < kdim * kdim; e += 64) Hj[e] = 0.0;
    __syncthreads();
    if (t < keep) {
        const int l = t;
        Hj[l * kdim + l] = th[ord[l]];
        const double b = bj * S[(kdim - 1) * kdim + ord[l]];
        Hj[l * kdim + keep] = b;
        Hj[keep * kdim + l] = b;
    }
}

// Q(:, l) <- Q(:, 0:kdim) S(:, l) for l < keep and Q(:, keep) <- Q(:, kdim), for
// the running shifts with go[c]; each thread owns one row of one shift
__global__ __launch_bounds__(kT) void k_trl_restart(int m, int kdim, int keep, const int* idx, const int* go,
                                                    zd* Q, long ldq, long qs, const double* Sk) {
    const int nrb = (m + kT - 1) / kT;   // row blocks per shift
    const int c = blockIdx.x / nrb;
    if (!go[c]) return;
    const int j = idx[c];
    const int r = (blockIdx.x - c * nrb) * kT + threadIdx.x;
    if (r >= m) return;
    const double* S = Sk + (long)j * kdim * keep;
    zd acc[kMaxKeep];
#pragma unroll
    for (int l = 0; l < kMaxKeep; ++l) acc[l] = zd{0.0, 0.0};
    for (int k = 0; k < kdim; ++k) {
        const zd q = Q[(long)k * qs + (long)j * ldq + r];
#pragma unroll
        for (int l = 0; l < kMaxKeep; ++l) {
            if (l < keep) {
                const double sv = S[k * keep + l];
                acc[l].re += sv * q.re;
                acc[l].im += sv * q.im;
            }
        }
    }
    const zd last = Q[(long)kdim * qs + (long)j * ldq + r];
#pragma unroll
    for (int l = 0; l < kMaxKeep; ++l)
        if (l < keep) Q[(long)l * qs + (long)j * ldq + r] = acc[l];
    Q[(long)keep * qs + (long)j * ldq + r] = last;
}

// idx_out <- idx[c] for the c with go[c], in order; *count_out <- their number
__global__ __launch_bounds__(kT) void k_trl_compact(int nact, const int* idx, const int* go, int* idx_out,
                                                    int* count_out) {
    __shared__ int sh[kT];
    int base = 0;
    for (int c0 = 0; c0 < nact; c0 += kT) {
        const int c = c0 + threadIdx.x;
        const int f = (c < nact && go[c]) ? 1 : 0;
        sh[threadIdx.x] = f;
        __syncthreads();
        // inclusive scan (Hillis-Steele)
        for (int off = 1; off < kT; off <<= 1) {
            const int v = threadIdx.x >= off ? sh[threadIdx.x - off] : 0;
            __syncthreads();
            sh[threadIdx.x] += v;
            __syncthreads();
        }
        if (f) idx_out[base + sh[threadIdx.x] - 1] = idx[c];
        base += sh[kT - 1];
        __syncthreads();
    }
    if (threadIdx.x == 0) *count_out = base;
}

// q_0 = v / ||v|| for every shift; the projected matrix starts at zero (the
// steps write only its tridiagonal band)
__global__ __launch_bounds__(kT) void k_trl_init(int m, int N, int kdim, const zd* V, long ldv, zd* Q, long ldq,
                                                 double* H, int* idx, int* steps) {
    for (int e = threadIdx.x; e < kdim * kdim; e += kT) H[(long)blockIdx.x * kdim * kdim + e] = 0.0;
    __shared__ double sh[(kT / 64) * 2];
    const int j = blockIdx.x;
    double s[2] = {0.0, 0.0};
    for (int r = threadIdx.x; r < m; r += kT) {
        const zd v = V[(long)j * ldv + r];
        s[0] += v.re * v.re + v.im * v.im;
    }
    block_sums<2>(s, sh);
    const double inv = s[0] > 0.0 ? 1.0 / sqrt(s[0]) : 0.0;
    for (int r = threadIdx.x; r < m; r += kT) {
        const zd v = V[(long)j * ldv + r];
        Q[(long)j * ldq + r] = zd{v.re * inv, v.im * inv};
    }
    if (threadIdx.x == 0) {
        idx[j] = j;
        steps[j] = 0;
    }
}

}  // namespace

int trl_max_kdim() { return kMaxK; }
int trl_max_keep() { return kMaxKeep; }

hipError_t launch_trl_init(int m, int N, int kdim, const zd* V, long ldv, zd* Q, long ldq, double* H, int* idx,
                           int* steps, hipStream_t s) {
    hipLaunchKernelGGL(k_trl_init, dim3(N), dim3(kT), 0, s, m, N, kdim, V, ldv, Q, ldq, H, idx, steps);
    return hipGetLastError();
}

hipError_t launch_trl_gather(int m, int nact, const int* idx, const zd* Qi, long ldq, zd* W, long ldw,
                             const zd* z, zd* zact, hipStream_t s) {
    hipLaunchKernelGGL(k_trl_gather, dim3(nact), dim3(kT), 0, s, m, nact, idx, Qi, ldq, W, ldw, z, zact);
    return hipGetLastError();
}

hipError_t launch_trl_orth(int m, int nact, int i, int k0, int kdim, const int* idx, zd* W, long ldw, zd* Q,
                           long ldq, long qs, double* H, double* beta, int* steps, hipStream_t s) {
    hipLaunchKernelGGL(k_trl_orth, dim3(nact), dim3(kT), 0, s, m, i, k0, kdim, idx, W, ldw, Q, ldq, qs, H,
                       beta, steps);
    return hipGetLastError();
}

hipError_t launch_trl_ritz(int nact, int kdim, int keep, double tol, int last, const int* idx, double* H,
                           const double* beta, double* Sk, double* sigma, double* resid, int* conv, int* go,
                           hipStream_t s) {
    hipLaunchKernelGGL(k_trl_ritz, dim3(nact), dim3(64), 0, s, kdim, keep, tol, last, idx, H, beta, Sk, sigma,
                       resid, conv, go);
    return hipGetLastError();
}

hipError_t launch_trl_restart(int m, int nact, int kdim, int keep, const int* idx, const int* go, zd* Q,
                              long ldq, long qs, const double* Sk, hipStream_t s) {
    const long blocks = (long)((m + kT - 1) / kT) * nact;
    if (blocks > 0x7fffffffL) return hipErrorInvalidConfiguration;
    hipLaunchKernelGGL(k_trl_restart, dim3((unsigned)blocks), dim3(kT), 0, s, m, kdim, keep, idx, go, Q, ldq, qs,
                       Sk);
    return hipGetLastError();
}

hipError_t launch_trl_compact(int nact, const int* idx, const int* go, int* idx_out, int* count,
                              hipStream_t s) {
    hipLaunchKernelGGL(k_trl_compact, dim3(1), dim3(kT), 0, s, nact, idx, go, idx_out, count);
    return hipGetLastError();
}

}  // namespace mst
