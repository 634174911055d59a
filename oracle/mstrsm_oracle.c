/*
 * CPU oracle for the (safe) multi-shift triangular solve.
 *
 * TEST INFRASTRUCTURE ONLY. This file is the slow, plain, obviously correct
 * reference that the GPU library is checked against. It shares no code with
 * the GPU path and must never be linked into it. Only the tests, the smoke
 * check and the benchmark's CPU-baseline leg load it.
 *
 * Paper: T. Moon, J. Poulson, "Accelerating eigenvector and pseudospectra
 * computation using blocked multi-shift triangular solves" (arXiv 1607.01477).
 *
 * Arithmetic is IEEE binary64 throughout. Build with -ffp-contract=off so that
 * every operation is rounded exactly as written.
 *
 * Data layout: column-major, complex numbers interleaved {re, im}; U is upper
 * triangular and its strict lower triangle is never read.
 *
 * Readings of points the paper leaves open (each written out where it is used):
 *   - modulus in growth bounds: cabs1(z) = |Re z| + |Im z|
 *   - overflow threshold Omega = 2^omega_log2 (default 2^960)
 *   - scaling factors are powers of two, t = 2^-k with k the smallest integer
 *     that brings the offending quantity below Omega
 *   - a pivot that is exactly zero is replaced by delta = 2^-52 * max cabs1(U)
 *     (2^-1022 if U is zero)
 *   - blocks are aligned from the top (row starts 0, nb, 2nb, ...), processed
 *     bottom to top; the bottom block may be partial
 * Parity: pinned (see tests/test_oracle_*.py).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct { double re, im; } zc;

#define AT(P, ld, r, c) ((P)[(size_t)(c) * (size_t)(ld) + (size_t)(r)])

static inline double cabs1(zc z) { return fabs(z.re) + fabs(z.im); }

static inline zc zsub(zc a, zc b) { zc r = { a.re - b.re, a.im - b.im }; return r; }

static inline zc zmul(zc a, zc b) {
    zc r = { a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re };
    return r;
}

static inline zc zconj(zc a) { zc r = { a.re, -a.im }; return r; }

/* b - u*x, each real operation rounded separately. */
static inline zc zaxpy_neg(zc b, zc u, zc x) { return zsub(b, zmul(u, x)); }

/* Complex division b/d: scale d by 2^-e (e = exponent of its larger part, an
 * exact operation), divide by the scaled d through its conjugate and squared
 * modulus, then undo the scaling. No intermediate overflows unless the quotient
 * itself does. d == 0 gives the IEEE 0/0 (NaN) pattern. */
static zc zdiv(zc b, zc d) {
    double a = fmax(fabs(d.re), fabs(d.im));
    int e = (a > 0.0) ? ilogb(a) : 0;
    double dr = ldexp(d.re, -e), di = ldexp(d.im, -e);
    double den = dr * dr + di * di;
    double qr = (b.re * dr + b.im * di) / den;
    double qi = (b.im * dr - b.re * di) / den;
    zc r = { ldexp(qr, -e), ldexp(qi, -e) };
    return r;
}

static inline zc zscale2(zc a, int k) { zc r = { ldexp(a.re, -k), ldexp(a.im, -k) }; return r; }

/* ------------------------------------------------------------------------ */
/* Plain solve: back substitution (Alg 1, Sec. 2) on U - lambda_j I, one     */
/* shift at a time. Row i: x_i = b_i / (U(i,i) - lambda_j), then            */
/* b(0:i) -= x_i * U(0:i, i). Blocking (Alg 3) changes only the order in    */
/* which shifts are grouped, not the arithmetic of one column, so the       */
/* unblocked form is the definition.                                        */
/* ------------------------------------------------------------------------ */
static void trsv_plain(int m, const zc* U, int ldu, zc lam, zc* b) {
    for (int i = m - 1; i >= 0; --i) {
        zc d = zsub(AT(U, ldu, i, i), lam);
        zc x = zdiv(b[i], d);
        b[i] = x;
        const zc* col = &AT(U, ldu, 0, i);
        for (int r = 0; r < i; ++r) b[r] = zaxpy_neg(b[r], col[r], x);
    }
}

int oracle_mstrsm(int m, int n, const double* Up, int ldu, const double* lamp,
                  double* Bp, int ldb) {
    if (m < 0 || n < 0 || ldu < (m > 1 ? m : 1) || ldb < (m > 1 ? m : 1)) return -1;
    const zc* U = (const zc*)Up;
    const zc* lam = (const zc*)lamp;
    zc* B = (zc*)Bp;
    #pragma omp parallel for schedule(static)
    for (int j = 0; j < n; ++j) trsv_plain(m, U, ldu, lam[j], &AT(B, ldb, 0, j));
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Generalized plain solve (appendix, Alg 8): (U - lambda_j V) x_j = b_j     */
/* with V upper triangular. Back substitution on the shifted matrix, whose   */
/* entries are formed as U(r,c) - lambda_j * V(r,c) (the xAXPY of Alg 8).   */
/* Alg 8 blocks the same arithmetic (its second GEMM adds V * (lambda x),    */
/* i.e. subtracts the -lambda V part of the shifted entries), so the         */
/* unblocked form is the definition. V's strict lower triangle is never read.*/
/* ------------------------------------------------------------------------ */
static void trsv_gen(int m, const zc* U, int ldu, const zc* V, int ldv, zc lam, zc* b) {
    for (int i = m - 1; i >= 0; --i) {
        zc d = zsub(AT(U, ldu, i, i), zmul(lam, AT(V, ldv, i, i)));
        zc x = zdiv(b[i], d);
        b[i] = x;
        const zc* ucol = &AT(U, ldu, 0, i);
        const zc* vcol = &AT(V, ldv, 0, i);
        for (int r = 0; r < i; ++r) b[r] = zaxpy_neg(b[r], zsub(ucol[r], zmul(lam, vcol[r])), x);
    }
}

int oracle_mstrsm_gen(int m, int n, const double* Up, int ldu, const double* Vp, int ldv,
                      const double* lamp, double* Bp, int ldb) {
    if (m < 0 || n < 0 || ldu < (m > 1 ? m : 1) || ldv < (m > 1 ? m : 1) || ldb < (m > 1 ? m : 1))
        return -1;
    const zc* U = (const zc*)Up;
    const zc* V = (const zc*)Vp;
    const zc* lam = (const zc*)lamp;
    zc* B = (zc*)Bp;
    #pragma omp parallel for schedule(static)
    for (int j = 0; j < n; ++j) trsv_gen(m, U, ldu, V, ldv, lam[j], &AT(B, ldb, 0, j));
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Variants of the footnote to Sec. 2: op(A - lambda_j I) x_j = b_j with A   */
/* upper (uplo 'U') or lower (uplo 'L') triangular and op the identity ('N'),*/
/* the transpose ('T') or the conjugate transpose ('C'). The operator        */
/* E = op(A - lambda I) is triangular: upper for (U,N), (L,T), (L,C), solved */
/* by back substitution; lower for (U,T), (U,C), (L,N), solved by forward    */
/* substitution. Entries: E(r,c) = A(r,c) for 'N', A(c,r) for 'T',           */
/* conj(A(c,r)) for 'C'; diagonal A(r,r) - lambda, conjugated for 'C'. The   */
/* other triangle of A is never read.                                        */
/* ------------------------------------------------------------------------ */
static inline zc opel(const zc* A, int lda, int trans, int conj, int r, int c) {
    zc a = trans ? AT(A, lda, c, r) : AT(A, lda, r, c);
    return conj ? zconj(a) : a;
}

static void trsv_op(int m, const zc* A, int lda, int upper_e, int trans, int conj, zc lam, zc* b) {
    if (upper_e) {
        for (int i = m - 1; i >= 0; --i) {
            zc d = zsub(opel(A, lda, trans, conj, i, i), conj ? zconj(lam) : lam);
            zc x = zdiv(b[i], d);
            b[i] = x;
            for (int r = 0; r < i; ++r) b[r] = zaxpy_neg(b[r], opel(A, lda, trans, conj, r, i), x);
        }
    } else {
        for (int i = 0; i < m; ++i) {
            zc d = zsub(opel(A, lda, trans, conj, i, i), conj ? zconj(lam) : lam);
            zc x = zdiv(b[i], d);
            b[i] = x;
            for (int r = i + 1; r < m; ++r) b[r] = zaxpy_neg(b[r], opel(A, lda, trans, conj, r, i), x);
        }
    }
}

int oracle_mstrsm_op(int uplo, int op, int m, int n, const double* Ap, int lda, const double* lamp,
                     double* Bp, int ldb) {
    if (m < 0 || n < 0 || lda < (m > 1 ? m : 1) || ldb < (m > 1 ? m : 1)) return -1;
    if ((uplo != 'U' && uplo != 'L') || (op != 'N' && op != 'T' && op != 'C')) return -2;
    const int trans = op != 'N', conj = op == 'C';
    const int upper_e = (uplo == 'U') == (op == 'N');
    const zc* A = (const zc*)Ap;
    const zc* lam = (const zc*)lamp;
    zc* B = (zc*)Bp;
    #pragma omp parallel for schedule(static)
    for (int j = 0; j < n; ++j) trsv_op(m, A, lda, upper_e, trans, conj, lam[j], &AT(B, ldb, 0, j));
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Real arithmetic (the paper's future work, in its plainest form): U, the    */
/* shifts and B real, (U - lambda_j I) x_j = b_j by back substitution, Alg 1: */
/* x_i = (b_i - sum_{k>i} U(i,k) x_k) / (U(i,i) - lambda_j), updates applied  */
/* column by column as in the complex solve.                                  */
/* ------------------------------------------------------------------------ */
int oracle_mstrsm_real(int m, int n, const double* U, int ldu, const double* lam, double* B, int ldb) {
    if (m < 0 || n < 0 || ldu < (m > 1 ? m : 1) || ldb < (m > 1 ? m : 1)) return -1;
    #pragma omp parallel for schedule(static)
    for (int j = 0; j < n; ++j) {
        double* b = &B[(size_t)j * ldb];
        for (int i = m - 1; i >= 0; --i) {
            double x = b[i] / (U[(size_t)i * ldu + i] - lam[j]);
            b[i] = x;
            const double* col = &U[(size_t)i * ldu];
            for (int r = 0; r < i; ++r) b[r] = b[r] - col[r] * x;
        }
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Adjoint solve: (U - lambda_j I)^H y_j = g_j. U^H is lower triangular, so */
/* this is forward substitution (the lower-triangular variant the paper     */
/* notes in its footnote to Sec. 2):                                        */
/*   y_i = (g_i - sum_{r<i} conj(U(r,i)) y_r) / conj(U(i,i) - lambda_j).    */
/* ------------------------------------------------------------------------ */
static void trsv_adjoint(int m, const zc* U, int ldu, zc lam, zc* g) {
    for (int i = 0; i < m; ++i) {
        const zc* col = &AT(U, ldu, 0, i);
        zc acc = g[i];
        for (int r = 0; r < i; ++r) acc = zaxpy_neg(acc, zconj(col[r]), g[r]);
        zc d = zconj(zsub(col[i], lam));
        g[i] = zdiv(acc, d);
    }
}

int oracle_mstrsm_adjoint(int m, int n, const double* Up, int ldu, const double* lamp,
                          double* Gp, int ldg) {
    if (m < 0 || n < 0 || ldu < (m > 1 ? m : 1) || ldg < (m > 1 ? m : 1)) return -1;
    const zc* U = (const zc*)Up;
    const zc* lam = (const zc*)lamp;
    zc* G = (zc*)Gp;
    #pragma omp parallel for schedule(static)
    for (int j = 0; j < n; ++j) trsv_adjoint(m, U, ldu, lam[j], &AT(G, ldg, 0, j));
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Safe solve (Sec. 3).                                                     */
/* ------------------------------------------------------------------------ */

typedef struct {
    int omega_log2;     /* Omega = 2^omega_log2 */
    double omega;
    int force_phase2;   /* skip the phase-1 fast path of Alg 4 */
    double delta;       /* replacement for an exactly zero pivot */
} safe_cfg;

/* Smallest k >= 1 with 2^-k * q < Omega, for finite q >= Omega (Omega = 2^w):
 * q in [2^e, 2^(e+1)) needs k = e - (w - 1). */
static inline int scale_exp(double q, int w) { return ilogb(q) - (w - 1); }

/* g + a*b for the growth bound, with the scale exponent that brings the sum
 * under Omega when it reaches Omega. When the sum overflows to infinity the
 * exponent comes from an upper bound on the exponents of its two terms:
 * g < 2^(ilogb g + 1), a*b < 2^(ilogb a + ilogb b + 2), so with
 * E = max(ilogb g, ilogb a + ilogb b + 1) + 1 the sum is < 2^(E+1) and
 * k = E + 1 - w suffices. Returns k (0 if no scaling is needed); *out is the
 * sum after scaling by 2^-k, recomputed from the scaled terms. */
static int bound_add(double g, double a, double b, int w, double omega, double* out) {
    double s = g + a * b;
    if (s < omega) { *out = s; return 0; }
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

/* Alg 4 (SafeTrsv) on the nb x nb block U(i0:i0+nb, i0:i0+nb) - lambda I with
 * right-hand side b (length nb), overwritten by x. cn[i] is the largest cabs1
 * entry of column i of the block above its diagonal. Returns the exponent k of
 * the factor t = 2^-k with (block - lambda I) x = t b.
 *
 * Phase 1 is only a fast path: it proves that phase 2 would not rescale, in
 * which case phase 2 reduces to the plain back substitution done here. The
 * bound recursion the paper prints uses |b(i)| <= G/|U(i,i)|, which holds for
 * the true modulus; with cabs1 the quotient can be up to twice larger, so the
 * recursion used here is G := G * (1 + 2 cn(i)/cabs1(d_i)) and the fast path
 * needs M < Omega/2 and G < Omega/2 (slack for rounding). */
static int safe_trsv(int nb, const zc* U, int ldu, int i0, zc lam, zc* b,
                     const double* cn, const safe_cfg* cfg) {
    const int w = cfg->omega_log2;
    const double omega = cfg->omega;
    /* pivots d_i = U(i,i) - lambda, with exact zeros replaced by delta */
    zc dpiv[nb > 0 ? nb : 1];
    for (int i = 0; i < nb; ++i) {
        zc d = zsub(AT(U, ldu, i0 + i, i0 + i), lam);
        if (d.re == 0.0 && d.im == 0.0) { d.re = cfg->delta; d.im = 0.0; }
        dpiv[i] = d;
    }
    double bnorm = 0.0;
    for (int i = 0; i < nb; ++i) bnorm = fmax(bnorm, cabs1(b[i]));

    if (!cfg->force_phase2) {
        double M1 = 0.0, G1 = bnorm;
        for (int i = nb - 1; i >= 0; --i) {
            double cd = cabs1(dpiv[i]);
            M1 = fmax(G1 / cd, M1);
            G1 = G1 * (1.0 + 2.0 * cn[i] / cd);
        }
        if (M1 < 0.5 * omega && G1 < 0.5 * omega) {
            for (int i = nb - 1; i >= 0; --i) {
                zc x = zdiv(b[i], dpiv[i]);
                b[i] = x;
                const zc* col = &AT(U, ldu, i0, i0 + i);
                for (int r = 0; r < i; ++r) b[r] = zaxpy_neg(b[r], col[r], x);
            }
            return 0;
        }
    }

    /* phase 2: checked back substitution */
    int k = 0;
    double G = bnorm;
    for (int i = nb - 1; i >= 0; --i) {
        double cd = cabs1(dpiv[i]);
        double cb = cabs1(b[i]);
        double M = cb / cd;
        if (M >= omega) {
            int kk = isinf(M) ? (ilogb(cb) - ilogb(cd) - (w - 1)) : scale_exp(M, w);
            for (int r = 0; r < nb; ++r) b[r] = zscale2(b[r], kk);
            k += kk;
            M = isinf(M) ? cabs1(b[i]) / cd : ldexp(M, -kk);
            G = ldexp(G, -kk);
        }
        zc x = zdiv(b[i], dpiv[i]);
        b[i] = x;
        double Gn;
        int kk = bound_add(G, M, cn[i], w, omega, &Gn);
        if (kk > 0) {
            for (int r = 0; r < nb; ++r) b[r] = zscale2(b[r], kk);
            k += kk;
            M = ldexp(M, -kk);
        }
        G = Gn;
        const zc* col = &AT(U, ldu, i0, i0 + i);
        x = b[i];
        for (int r = 0; r < i; ++r) b[r] = zaxpy_neg(b[r], col[r], x);
    }
    return k;
}

/* Column norms used by the bounds (the paper reuses them across all shifts):
 *   cn_in[c]   = max_{blockstart(c) <= r < c} cabs1(U(r,c))  (inside the diagonal block)
 *   above[c]   = max_{r < blockstart(c)} cabs1(U(r,c))       (above the diagonal block)
 *   umax       = max_{r <= c} cabs1(U(r,c))                   (for delta)
 * For the unblocked Alg 4 (nb >= m) the block is the whole matrix. */
static void column_norms(int m, const zc* U, int ldu, int nb, double* cn_in, double* above,
                         double* umax) {
    double um = 0.0;
    for (int c = 0; c < m; ++c) {
        int bs = (c / nb) * nb;
        double a = 0.0, in = 0.0;
        for (int r = 0; r < bs; ++r) a = fmax(a, cabs1(AT(U, ldu, r, c)));
        for (int r = bs; r < c; ++r) in = fmax(in, cabs1(AT(U, ldu, r, c)));
        cn_in[c] = in;
        above[c] = a;
        um = fmax(um, fmax(fmax(a, in), cabs1(AT(U, ldu, c, c))));
    }
    *umax = um;
}

/*
 * Safe multi-shift solve (U - lambda_j I) x_j = s_j b_j, s_j = 2^-k_j.
 *
 * nb <= 0 or nb >= m: Alg 4 applied to each column, unblocked.
 * otherwise: Alg 5 with decision block size nb, one column at a time (the
 * column's share of the block GEMM is written as its matrix-vector product,
 * accumulated over the block's columns from last to first).
 *
 * col_len (nullable): column j uses rows [0, col_len[j]) only; the other rows
 * are neither read nor written and stand for zero right-hand-side entries
 * (the triangular-eigenvector short-cut of Sec. 4). With zero rows below, a
 * block that lies entirely in them leaves x, s and the bounds unchanged, so
 * skipping it is exact; a block that straddles col_len[j] is solved whole
 * with zeros in its lower rows.
 *
 * trace (nullable, debugging the bound invariant): for block index bi and
 * column j, trace[2*(bi*n+j)] = G(j) after the block's bound update and
 * trace[2*(bi*n+j)+1] = max cabs1 over rows above the block after its
 * substitution step (NaN when the block was skipped).
 */
int oracle_mstrsm_safe(int m, int n, const double* Up, int ldu, const double* lamp,
                       double* Bp, int ldb, const int* col_len, double* scale, int* klog,
                       int nb, int omega_log2, int force_phase2, double* trace) {
    if (m < 0 || n < 0 || ldu < (m > 1 ? m : 1) || ldb < (m > 1 ? m : 1)) return -1;
    if (omega_log2 <= 0) omega_log2 = 960;
    if (omega_log2 < 2 || omega_log2 > 1000) return -2;
    const zc* U = (const zc*)Up;
    const zc* lam = (const zc*)lamp;
    zc* B = (zc*)Bp;
    int unblocked = (nb <= 0 || nb >= m);
    int nbe = unblocked ? (m > 0 ? m : 1) : nb;
    int nblk = (m + nbe - 1) / nbe;

    double* cn_in = (double*)malloc(sizeof(double) * (size_t)(m > 0 ? m : 1));
    double* above = (double*)malloc(sizeof(double) * (size_t)(m > 0 ? m : 1));
    double* above_sum = (double*)malloc(sizeof(double) * (size_t)(nblk > 0 ? nblk : 1));
    double umax = 0.0;
    column_norms(m, U, ldu, nbe, cn_in, above, &umax);
    /* sum_{k in block} ||U(rows above block, k)||_inf, in ascending k */
    for (int bi = 0; bi < nblk; ++bi) {
        double s = 0.0;
        int c1 = (bi + 1) * nbe < m ? (bi + 1) * nbe : m;
        for (int c = bi * nbe; c < c1; ++c) s = s + above[c];
        above_sum[bi] = s;
    }

    safe_cfg cfg;
    cfg.omega_log2 = omega_log2;
    cfg.omega = ldexp(1.0, omega_log2);
    cfg.force_phase2 = force_phase2;
    cfg.delta = (umax > 0.0) ? ldexp(umax, -52) : ldexp(1.0, -1022);

    const int w = omega_log2;
    const double omega = cfg.omega;

    #pragma omp parallel
    {
        zc* buf = (zc*)malloc(sizeof(zc) * (size_t)nbe);
        #pragma omp for schedule(static)
        for (int j = 0; j < n; ++j) {
            zc* b = &AT(B, ldb, 0, j);
            int L = col_len ? col_len[j] : m;
            if (L > m) L = m;
            if (L < 0) L = 0;
            int kj = 0;
            if (unblocked) {
                for (int r = 0; r < m; ++r) buf[r] = (r < L) ? b[r] : (zc){0.0, 0.0};
                kj = safe_trsv(m, U, ldu, 0, lam[j], buf, cn_in, &cfg);
                for (int r = 0; r < L; ++r) b[r] = buf[r];
            } else {
                double G = 0.0;
                for (int r = 0; r < L; ++r) G = fmax(G, cabs1(b[r]));
                for (int bi = nblk - 1; bi >= 0; --bi) {
                    int i0 = bi * nbe;
                    int i1 = (i0 + nbe < m) ? i0 + nbe : m;
                    int bs = i1 - i0;
                    if (i0 >= L) {
                        if (trace) { trace[2 * ((size_t)bi * n + j)] = NAN;
                                     trace[2 * ((size_t)bi * n + j) + 1] = NAN; }
                        continue;
                    }
                    /* diagonal block step */
                    for (int r = 0; r < bs; ++r) buf[r] = (i0 + r < L) ? b[i0 + r] : (zc){0.0, 0.0};
                    int kb = safe_trsv(bs, U, ldu, i0, lam[j], buf, &cn_in[i0], &cfg);
                    for (int r = 0; r < bs; ++r) if (i0 + r < L) b[i0 + r] = buf[r];
                    if (kb > 0) {
                        /* B(I0,j), B(I2,j) scaled by t; G(j) too */
                        for (int r = 0; r < i0; ++r) b[r] = zscale2(b[r], kb);
                        for (int r = i1; r < L; ++r) b[r] = zscale2(b[r], kb);
                        G = ldexp(G, -kb);
                        kj += kb;
                    }
                    /* column bound: G(j) += sum_k ||U(I0,k)||_inf * ||B(I1,j)||_inf */
                    double xn = 0.0;
                    for (int r = 0; r < bs; ++r) xn = fmax(xn, cabs1(buf[r]));
                    double Gn;
                    int k2 = bound_add(G, above_sum[bi], xn, w, omega, &Gn);
                    if (k2 > 0) {
                        for (int r = 0; r < L; ++r) b[r] = zscale2(b[r], k2);
                        kj += k2;
                    }
                    G = Gn;
                    if (trace) trace[2 * ((size_t)bi * n + j)] = G;
                    /* substitution step: B(I0,j) -= U(I0,I1) X(I1,j), columns of
                     * the block from last to first */
                    for (int c = i1 - 1; c >= i0; --c) {
                        if (c >= L) continue;   /* zero entries of x contribute nothing */
                        zc x = b[c];
                        const zc* col = &AT(U, ldu, 0, c);
                        for (int r = 0; r < i0; ++r) b[r] = zaxpy_neg(b[r], col[r], x);
                    }
                    if (trace) {
                        double mx = 0.0;
                        for (int r = 0; r < i0; ++r) mx = fmax(mx, cabs1(b[r]));
                        trace[2 * ((size_t)bi * n + j) + 1] = mx;
                    }
                }
            }
            klog[j] = kj;
            scale[j] = ldexp(1.0, -kj);
        }
        free(buf);
    }
    free(cn_in);
    free(above);
    free(above_sum);
    return 0;
}

/*
 * Safe generalized solve (appendix, Alg 9): (U - lambda_j V) x_j = s_j b_j,
 * s_j = 2^-k_j, U and V upper triangular.
 *
 * Per column and decision block (blocks as in the safe solve above):
 *   - the shifted diagonal block U' = U(I1,I1) - lambda_j V(I1,I1) is formed
 *     entry by entry (the xAXPY of Alg 9) and Alg 4 runs on it: its pivots
 *     are the diagonal of U', its column norms those of U' above the diagonal
 *     inside the block;
 *   - a rescale t < 1 from the block scales B(I0,j), B(I2,j), s_j and G(j);
 *   - the column bound adds sum_{k in I1} (||U(I0,k)||_inf +
 *     |lambda_j| ||V(I0,k)||_inf) * ||B(I1,j)||_inf, evaluated as
 *     above_sum_U + cabs1(lambda_j) * above_sum_V, then rescales B(:,j) when
 *     it reaches Omega;
 *   - substitution: C = lambda_j X(I1,j), B(I0,j) -= U(I0,I1) X(I1,j), then
 *     B(I0,j) += V(I0,I1) C (the two xGEMM steps of Alg 9, columns of the
 *     block from last to first).
 * nb <= 0 or nb >= m: one block, i.e. Alg 4 on the whole shifted matrix.
 * A pivot of U' that is exactly zero is replaced by
 * delta = 2^-52 * max(max cabs1(U), max cabs1(V)) (2^-1022 if both are zero).
 * col_len (nullable): as in the safe solve above.
 */
int oracle_mstrsm_safe_gen(int m, int n, const double* Up, int ldu, const double* Vp, int ldv,
                           const double* lamp, double* Bp, int ldb, const int* col_len,
                           double* scale, int* klog, int nb, int omega_log2, int force_phase2) {
    if (m < 0 || n < 0 || ldu < (m > 1 ? m : 1) || ldv < (m > 1 ? m : 1) || ldb < (m > 1 ? m : 1))
        return -1;
    if (omega_log2 <= 0) omega_log2 = 960;
    if (omega_log2 < 2 || omega_log2 > 1000) return -2;
    const zc* U = (const zc*)Up;
    const zc* V = (const zc*)Vp;
    const zc* lam = (const zc*)lamp;
    zc* B = (zc*)Bp;
    int unblocked = (nb <= 0 || nb >= m);
    int nbe = unblocked ? (m > 0 ? m : 1) : nb;
    int nblk = (m + nbe - 1) / nbe;
    size_t mm = (size_t)(m > 0 ? m : 1);

    double* scratch = (double*)malloc(sizeof(double) * (4 * mm + 2 * (size_t)(nblk > 0 ? nblk : 1)));
    double *cnU = scratch, *aboveU = scratch + mm, *cnV = scratch + 2 * mm, *aboveV = scratch + 3 * mm;
    double *asumU = scratch + 4 * mm, *asumV = asumU + (nblk > 0 ? nblk : 1);
    double umax = 0.0, vmax = 0.0;
    column_norms(m, U, ldu, nbe, cnU, aboveU, &umax);
    column_norms(m, V, ldv, nbe, cnV, aboveV, &vmax);
    for (int bi = 0; bi < nblk; ++bi) {
        double su = 0.0, sv = 0.0;
        int c1 = (bi + 1) * nbe < m ? (bi + 1) * nbe : m;
        for (int c = bi * nbe; c < c1; ++c) { su = su + aboveU[c]; sv = sv + aboveV[c]; }
        asumU[bi] = su;
        asumV[bi] = sv;
    }

    safe_cfg cfg;
    cfg.omega_log2 = omega_log2;
    cfg.omega = ldexp(1.0, omega_log2);
    cfg.force_phase2 = force_phase2;
    double mx = fmax(umax, vmax);
    cfg.delta = (mx > 0.0) ? ldexp(mx, -52) : ldexp(1.0, -1022);
    const int w = omega_log2;
    const double omega = cfg.omega;
    const zc zero = {0.0, 0.0};

    #pragma omp parallel
    {
        zc* Ub = (zc*)malloc(sizeof(zc) * (size_t)nbe * (size_t)nbe);
        zc* buf = (zc*)malloc(sizeof(zc) * (size_t)nbe);
        zc* Cb = (zc*)malloc(sizeof(zc) * (size_t)nbe);
        double* cnb = (double*)malloc(sizeof(double) * (size_t)nbe);
        #pragma omp for schedule(static)
        for (int j = 0; j < n; ++j) {
            zc* b = &AT(B, ldb, 0, j);
            const zc lj = lam[j];
            const double labs = cabs1(lj);
            int L = col_len ? col_len[j] : m;
            if (L > m) L = m;
            if (L < 0) L = 0;
            int kj = 0;
            double G = 0.0;
            for (int r = 0; r < L; ++r) G = fmax(G, cabs1(b[r]));
            for (int bi = nblk - 1; bi >= 0; --bi) {
                int i0 = bi * nbe;
                int i1 = (i0 + nbe < m) ? i0 + nbe : m;
                int bs = i1 - i0;
                if (i0 >= L) continue;
                /* U' = U(I1,I1) - lambda_j V(I1,I1) and its column norms */
                for (int c = 0; c < bs; ++c) {
                    double cm = 0.0;
                    for (int r = 0; r <= c; ++r) {
                        zc e = zsub(AT(U, ldu, i0 + r, i0 + c), zmul(lj, AT(V, ldv, i0 + r, i0 + c)));
                        AT(Ub, nbe, r, c) = e;
                        if (r < c) cm = fmax(cm, cabs1(e));
                    }
                    cnb[c] = cm;
                }
                /* diagonal block step: Alg 4 on U' (its shift is already applied) */
                for (int r = 0; r < bs; ++r) buf[r] = (i0 + r < L) ? b[i0 + r] : zero;
                int kb = safe_trsv(bs, Ub, nbe, 0, zero, buf, cnb, &cfg);
                for (int r = 0; r < bs; ++r) if (i0 + r < L) b[i0 + r] = buf[r];
                if (kb > 0) {
                    for (int r = 0; r < i0; ++r) b[r] = zscale2(b[r], kb);
                    for (int r = i1; r < L; ++r) b[r] = zscale2(b[r], kb);
                    G = ldexp(G, -kb);
                    kj += kb;
                }
                /* column bound with the pencil's two norms */
                double xn = 0.0;
                for (int r = 0; r < bs; ++r) xn = fmax(xn, cabs1(buf[r]));
                double a = asumU[bi] + labs * asumV[bi];
                double Gn;
                int k2 = bound_add(G, a, xn, w, omega, &Gn);
                if (k2 > 0) {
                    for (int r = 0; r < L; ++r) b[r] = zscale2(b[r], k2);
                    kj += k2;
                }
                G = Gn;
                /* substitution: C = lambda X(I1), B(I0) -= U(I0,I1) X(I1), B(I0) += V(I0,I1) C */
                int cend = (i1 < L) ? i1 : L;   /* zero entries of x contribute nothing */
                for (int c = i0; c < cend; ++c) Cb[c - i0] = zmul(lj, b[c]);
                for (int c = cend - 1; c >= i0; --c) {
                    zc x = b[c];
                    const zc* col = &AT(U, ldu, 0, c);
                    for (int r = 0; r < i0; ++r) b[r] = zaxpy_neg(b[r], col[r], x);
                }
                for (int c = cend - 1; c >= i0; --c) {
                    zc cc = Cb[c - i0];
                    const zc* col = &AT(V, ldv, 0, c);
                    for (int r = 0; r < i0; ++r) {
                        zc p = zmul(col[r], cc);
                        b[r].re = b[r].re + p.re;
                        b[r].im = b[r].im + p.im;
                    }
                }
            }
            klog[j] = kj;
            scale[j] = ldexp(1.0, -kj);
        }
        free(Ub);
        free(buf);
        free(Cb);
        free(cnb);
    }
    free(scratch);
    return 0;
}

/* Number of OpenMP threads a parallel region would use (for reporting). */
int oracle_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void oracle_set_num_threads(int t) {
#ifdef _OPENMP
    if (t > 0) omp_set_num_threads(t);
#else
    (void)t;
#endif
}
