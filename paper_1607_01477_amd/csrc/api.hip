// C-ABI of the mstrsm library: argument checking, workspace, and the block
// loops of the multi-shift solves (Moon & Poulson, arXiv 1607.01477).
//
// Block order. Diagonal blocks of nb rows are aligned from the top (row starts
// 0, nb, 2nb, ...; the bottom block may be partial) and solved bottom to top
// (top to bottom for the adjoint). Consecutive diagonal blocks are grouped into
// outer blocks of outer_nb rows: after each diagonal block only the rows of its
// own outer block are updated (a short GEMM with K = nb), and the rows above
// the outer block receive one GEMM with K = outer_nb once the whole outer block
// is solved. This is Alg 3 with the substitution of several consecutive
// diagonal blocks fused into one longer product: the same arithmetic in
// another order, with a deeper K per pass over B so the GEMM is not bound by
// re-reading and re-writing B. outer_nb = nb gives the paper's order exactly.
//
// Safe solve (Alg 5): per diagonal block the kernel records the column's
// exponent k_j after that block; a GEMM brings its B operand rows and its C
// rows to the current exponent on the fly (exact powers of two), and a final
// pass rescales each solved block to the final exponent, so scaling never
// costs an extra sweep over B while no rescaling happens.
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <mutex>
#include <vector>

#include "common.h"
#include "mstrsm.h"

using namespace mst;

// Device memory of the entry point that allocates nothing (mstrsm_safe_noalloc):
// one copy of this array per device, held until the process ends. Host code
// never uses its name as an address: the device address comes from
// hipGetSymbolAddress, once per device (scratch_ptr below).
#define MST_SCRATCH_BYTES MST_SCRATCH_LIMIT
static __device__ __align__(256) unsigned char scratch[MST_SCRATCH_BYTES];

namespace {

thread_local int t_bad_arg = 0;
thread_local char t_err[256] = "";

// MSTRSM_LOG set (and not "0"): every call and every error is reported on
// stderr (the call's name and sizes; nothing is synchronised)
bool log_on() {
    static const bool on = [] {
        const char* e = getenv("MSTRSM_LOG");
        return e != nullptr && *e != 0 && strcmp(e, "0") != 0;
    }();
    return on;
}
thread_local const char* t_entry = "";

void entry(const char* name, int m, int n) {
    t_bad_arg = 0;
    t_err[0] = 0;
    t_entry = name;
    if (log_on()) fprintf(stderr, "[mstrsm] %s m=%d n=%d\n", name, m, n);
}

mst_status bad(int pos) {
    t_bad_arg = pos;
    if (log_on()) fprintf(stderr, "[mstrsm] %s: invalid argument %d\n", t_entry, pos);
    return MST_EARG;
}

// a valid option combination this entry point does not offer
mst_status unsupported(const char* why) {
    snprintf(t_err, sizeof(t_err), "%s", why);
    if (log_on()) fprintf(stderr, "[mstrsm] %s: unsupported: %s\n", t_entry, why);
    return MST_EUNSUPPORTED;
}

mst_status fail_hip(hipError_t e, const char* what) {
    snprintf(t_err, sizeof(t_err), "%s: %s", what, hipGetErrorString(e));
    if (log_on()) fprintf(stderr, "[mstrsm] %s: %s\n", t_entry, t_err);
    return (e == hipErrorOutOfMemory) ? MST_ENOMEM : MST_EHIP;
}

#define HIPCHK(x)                                             \
    do {                                                      \
        hipError_t e_ = (x);                                  \
        if (e_ != hipSuccess) return fail_hip(e_, #x);        \
    } while (0)

// ---------------------------------------------------------------- kernel timing
struct ProfRec {
    int kind;
    hipEvent_t a, b;
    double flops;
};
thread_local bool t_prof = false;
thread_local std::vector<ProfRec> t_recs;
thread_local std::vector<hipEvent_t> t_pool;

hipEvent_t pool_event() {
    if (!t_pool.empty()) {
        hipEvent_t e = t_pool.back();
        t_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    (void)hipEventCreate(&e);
    return e;
}

// Runs launch() bracketed by events when profiling is on.
template <typename F>
hipError_t timed(int kind, double flops, hipStream_t s, F&& launch) {
    if (!t_prof) return launch();
    ProfRec r{kind, pool_event(), pool_event(), flops};
    (void)hipEventRecord(r.a, s);
    hipError_t e = launch();
    (void)hipEventRecord(r.b, s);
    t_recs.push_back(r);
    return e;
}

double gemm_flops(const GemmArgs& g) {
    return (g.op == GOP_GEN_SUB ? 16.0 : 8.0) * g.M * (double)g.N * g.K;
}

struct Opts {
    int nb = 16, outer = 256, precision = 0, sweeps = 2, omega_log2 = 960;
    bool outer_auto = true;   // outer_nb left to the library
    bool fuse = true;
    int fuse_width = 0;
    int staged = 0;
    int split = 0;
    bool overlap = false;
    bool force_checked = false;
    double refine_tol = 1e-14;
    double* report = nullptr;
    const int* skip = nullptr;   // set internally: the refinement loop's stop flag
};

// position of opt in the caller's argument list, for error reporting
mst_status read_opts(const mst_opts* o, Opts& r, int pos) {
    r = Opts();
    if (!o) return MST_OK;
    if (o->nb) r.nb = o->nb;
    if (r.nb != 16 && r.nb != 32 && r.nb != 64) return bad(pos);
    r.outer = o->outer_nb ? o->outer_nb : (r.nb > 256 ? r.nb : 256);
    r.outer_auto = o->outer_nb == 0;
    if (o->outer_nb == 0 && r.outer % r.nb) r.outer = r.nb;
    if (r.outer < r.nb || r.outer % r.nb || r.outer > 8192) return bad(pos);
    r.precision = o->precision;
    if (r.precision != 0 && r.precision != 1) return bad(pos);
    if (o->max_sweeps) r.sweeps = o->max_sweeps;
    if (r.sweeps < 1 || r.sweeps > 3) return bad(pos);
    if (o->omega_log2) r.omega_log2 = o->omega_log2;
    if (r.omega_log2 < 8 || r.omega_log2 > 1000) return bad(pos);
    if (o->fuse_blocks < -1 || o->fuse_blocks > 4) return bad(pos);
    r.fuse = o->fuse_blocks >= 0;
    r.fuse_width = o->fuse_blocks == 1 ? 16 : o->fuse_blocks == 2 ? 4 : o->fuse_blocks == 3 ? 2 : o->fuse_blocks == 4 ? 1 : 0;
    if (o->gemm_staged != 0 && o->gemm_staged != 1) return bad(pos);
    r.staged = o->gemm_staged;
    if (o->overlap != 0 && o->overlap != 1) return bad(pos);
    r.overlap = o->overlap == 1;
    if (o->force_phase2 != 0 && o->force_phase2 != 1) return bad(pos);
    r.force_checked = o->force_phase2 == 1;
    if (o->gemm_split != 0 && o->gemm_split != 1 && o->gemm_split != 2 && o->gemm_split != 4) return bad(pos);
    r.split = o->gemm_split;
    if (o->refine_tol != 0.0) r.refine_tol = o->refine_tol;
    if (r.refine_tol != r.refine_tol) return bad(pos);   // NaN
    r.report = o->refine_report;
    return MST_OK;
}

// Stream-ordered workspace, released on scope exit (also on error paths).
// With an arena (the static scratch of mstrsm_safe_noalloc) the pieces are
// carved from it in order, each aligned to 256 bytes, and nothing is
// allocated or freed.
constexpr size_t kWsAlign = 256;
inline size_t ws_round(size_t bytes) { return ((bytes > 0 ? bytes : 16) + kWsAlign - 1) & ~(kWsAlign - 1); }

struct Workspace {
    hipStream_t s;
    std::vector<void*> ptrs;
    char* arena = nullptr;
    size_t cap = 0, used = 0;
    explicit Workspace(hipStream_t st) : s(st) {}
    Workspace(hipStream_t st, void* base, size_t bytes) : s(st), arena((char*)base), cap(bytes) {}
    ~Workspace() {
        for (void* p : ptrs) (void)hipFreeAsync(p, s);
    }
    hipError_t get(size_t bytes, void** out) {
        if (arena) {
            const size_t sz = ws_round(bytes);
            if (used + sz > cap) return hipErrorOutOfMemory;
            *out = arena + used;
            used += sz;
            return hipSuccess;
        }
        void* p = nullptr;
        hipError_t e = hipMallocAsync(&p, bytes > 0 ? bytes : 16, s);
        if (e != hipSuccess) return e;
        ptrs.push_back(p);
        *out = p;
        return hipSuccess;
    }
};

template <typename T>
hipError_t ws_get(Workspace& w, size_t count, T** out) {
    return w.get(count * sizeof(T), (void**)out);
}

// ---------------------------------------------------------------- lookahead stream
// A second stream per thread and device for the lookahead chain, with events
// to order it against the caller's stream. Created on first use and kept until
// the process ends (default priority, non-blocking).
struct Aux {
    int dev = -1;
    hipStream_t stream = nullptr;
    std::vector<hipEvent_t> ev;
};
thread_local std::vector<Aux> t_aux;

hipError_t aux_get(int nev, Aux** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    Aux* ax = nullptr;
    for (Aux& a : t_aux)
        if (a.dev == dev) ax = &a;
    if (!ax) {
        Aux a;
        a.dev = dev;
        if ((e = hipStreamCreateWithFlags(&a.stream, hipStreamNonBlocking)) != hipSuccess) return e;
        t_aux.push_back(a);
        ax = &t_aux.back();
    }
    while ((int)ax->ev.size() < nev) {
        hipEvent_t ev = nullptr;
        if ((e = hipEventCreateWithFlags(&ev, hipEventDisableTiming)) != hipSuccess) return e;
        ax->ev.push_back(ev);
    }
    *out = ax;
    return hipSuccess;
}

// ---------------------------------------------------------------- forward block loop
// FP64 (b32 == nullptr) or mixed: the right-hand side lives in W32 (FP32) for the
// substitution GEMMs and the diagonal blocks write FP64 X into B.
// V != nullptr: the pencil U - lambda_j V (FP64, nb = 16): diagonal blocks of
// U - lambda_j V, substitution C -= U X - V (lambda X) (Alg 8 / Alg 9).
// rows per group of the two-level deferral in the one-stream forward loop
constexpr int kSuperRows = 1024;

// Outer block size of a back substitution: where the library chooses it and
// the fused kernel runs narrow workgroups of at most 2 shifts (plain FP64
// solves with few shifts), outer blocks of twice the rows: half the fused
// launches and half the substitution GEMMs, whose small launches are bound by
// their start-up rather than their flops at this n.
Opts outer_for(const Opts& o, int n, bool plain) {
    Opts r = o;
    if (o.outer_auto && o.fuse && !o.overlap && o.outer < block_rows_for(n, o.nb, o.fuse_width, plain))
        r.outer = block_rows_for(n, o.nb, o.fuse_width, plain);
    return r;
}

hipError_t forward_loop(int m, int n, const zd* U, long ldu, const zf* U32, long ldu32,
                        const zd* lam, zd* B, long ldb, zf* W32, long ldw, const Opts& oin,
                        const SafeState* safe, const int* col_len, hipStream_t s,
                        const zd* V = nullptr, long ldv = 0, int ev = EV_UPPER_N) {
    const bool plain = safe == nullptr && col_len == nullptr && W32 == nullptr && V == nullptr;
    const Opts o = outer_for(oin, n, plain);
    // ev: EV_UPPER_N, or EV_LOWER_T / EV_LOWER_C (plain FP64): back substitution
    // with E(r, c) = A(c, r) (conjugated for EV_LOWER_C) read from A's lower triangle
    const bool etr = ev_tr(ev);
    const int amode = etr ? (ev_cj(ev) ? 1 : 2) : 0;
    const int nb = o.nb, P = o.outer / o.nb;
    const int nblk = (m + nb - 1) / nb;
    const int nob = (nblk + P - 1) / P;
    const bool mixed = W32 != nullptr;
    const bool fused = o.fuse && o.outer <= block_rows_for(n, o.nb, o.fuse_width, plain) && block_fusable(o.nb);
    auto q_first = [&](int ob) { return ob * P; };
    auto q_last = [&](int ob) { return (ob * P + P < nblk ? ob * P + P : nblk) - 1; };
    auto row_end = [&](int ob) { return ((q_last(ob) + 1) * nb < m) ? (q_last(ob) + 1) * nb : m; };

    // B(r0:r1, :) -= U(r0:r1, x0:x1) X(x0:x1, :) with X the solved rows of outer
    // blocks ob_lo..ob_hi (x0:x1 are their rows); the safe form brings C from the
    // exponent of the outer block below ob_hi to that of ob_lo
    auto substitute_range = [&](int ob_lo, int ob_hi, int r0, int r1, hipStream_t st) -> hipError_t {
        if (r1 <= r0) return hipSuccess;
        const int qa = q_first(ob_lo), qb = q_last(ob_hi);
        const int x0 = qa * nb, x1 = row_end(ob_hi);
        GemmArgs g{};
        g.M = r1 - r0; g.N = n; g.K = x1 - x0;
        g.op = GOP_SUB; g.staged = o.staged; g.split = o.split;
        g.nb = nb; g.b_row0 = x0; g.c_row0 = r0; g.col_len = col_len;
        if (safe) {
            g.kb = safe->kb; g.n_kb = n; g.q_cur = qa; g.q_c = (qb + 1 < nblk) ? qb + 1 : -1;
        }
        if (!mixed) {
            g.A = etr ? U + (long)r0 * ldu + x0 : U + (long)x0 * ldu + r0; g.lda = ldu; g.a_ct = amode;
            g.B = B + x0; g.ldb = ldb;
            g.C = B + r0; g.ldc = ldb;
            if (V) {
                g.op = GOP_GEN_SUB;
                g.A2 = V + (long)x0 * ldv + r0; g.lda2 = ldv; g.glam = lam;
            }
            return timed(MST_PROF_GEMM_F64, gemm_flops(g), st, [&] { return launch_gemm_f64(g, st); });
        }
        g.A = U32 + (long)x0 * ldu32 + r0; g.lda = ldu32;
        g.B = W32 + x0; g.ldb = ldw;
        g.C = W32 + r0; g.ldc = ldw;
        g.skip = o.skip;
        return timed(MST_PROF_GEMM_F32, gemm_flops(g), st, [&] { return launch_gemm_f32(g, st); });
    };
    auto substitute = [&](int ob, int r0, int r1, hipStream_t st) -> hipError_t {
        return substitute_range(ob, ob, r0, r1, st);
    };
    // all diagonal blocks of outer block ob, with the substitution between them, in one kernel
    auto solve_outer = [&](int ob, hipStream_t st) -> hipError_t {
        const int qa = q_first(ob);
        BlockArgs b{};
        b.m = m; b.n = n; b.nb = nb; b.qa = qa; b.iS = qa * nb;
        b.rows = row_end(ob) - qa * nb;
        b.U = U; b.ldu = ldu; b.lam = lam; b.B = B; b.ldb = ldb;
        b.V = V; b.ldv = ldv;
        b.b32 = mixed ? W32 : nullptr; b.ldb32 = ldw;
        b.skip = mixed ? o.skip : nullptr;
        b.col_len = col_len;
        b.width = o.fuse_width;
        if (safe) {
            b.safe = *safe;
            b.use_safe = 1;
        } else {
            b.safe.omega_log2 = o.omega_log2;
        }
        const double fl = (V ? 8.0 : 4.0) * b.rows * (double)b.rows * n;
        return timed(MST_PROF_DIAG, fl, st, [&] { return launch_block(ev, b, st); });
    };

    if (fused && o.overlap && nob > 2) {
        // Lookahead. The library's second stream K carries the critical chain:
        // X of outer block ob+1 into the rows of ob, then the solve of ob. The
        // caller's stream S carries the bulk: X of ob into all rows above ob-1.
        // Per element the updates keep their order (outer blocks bottom to
        // top, one product of K = outer_nb each), so the result is that of a
        // one-stream loop with one substitution per outer block; the default
        // one-stream loop below groups outer blocks into deeper products and
        // therefore differs from this one in summation order (rounding only).
        //   K, substitute(ob+1 -> rows of ob): after S's GEMM of ob+2, the last
        //      earlier writer of those rows;
        //   S, GEMM of ob: after K's solve of ob (it reads X of ob).
        Aux* ax = nullptr;
        hipError_t e = aux_get(2 * nob + 2, &ax);
        if (e != hipSuccess) return e;
        hipStream_t k = ax->stream;
        hipEvent_t* evG = ax->ev.data();          // evG[ob]: S's GEMM of ob done
        hipEvent_t* evK = ax->ev.data() + nob;    // evK[ob]: K's solve of ob done
        hipEvent_t evFork = ax->ev[2 * nob], evJoin = ax->ev[2 * nob + 1];
        if ((e = hipEventRecord(evFork, s)) != hipSuccess) return e;
        if ((e = hipStreamWaitEvent(k, evFork, 0)) != hipSuccess) return e;
        for (int ob = nob - 1; ob >= 0; --ob) {
            if (ob + 1 < nob) {
                if (ob + 2 < nob && (e = hipStreamWaitEvent(k, evG[ob + 2], 0)) != hipSuccess) return e;
                if ((e = substitute(ob + 1, q_first(ob) * nb, row_end(ob), k)) != hipSuccess) return e;
            }
            if ((e = solve_outer(ob, k)) != hipSuccess) return e;
            if ((e = hipEventRecord(evK[ob], k)) != hipSuccess) return e;
            if (ob >= 2) {
                if ((e = hipStreamWaitEvent(s, evK[ob], 0)) != hipSuccess) return e;
                if ((e = substitute(ob, 0, q_first(ob - 1) * nb, s)) != hipSuccess) return e;
                if ((e = hipEventRecord(evG[ob], s)) != hipSuccess) return e;
            }
        }
        if ((e = hipEventRecord(evJoin, k)) != hipSuccess) return e;
        return hipStreamWaitEvent(s, evJoin, 0);
    }

    for (int ob = nob - 1; ob >= 0; --ob) {
        const int qa = q_first(ob), qb = q_last(ob);
        if (fused) {
            hipError_t e = solve_outer(ob, s);
            if (e != hipSuccess) return e;
        }
        for (int q = qb; q >= qa && !fused; --q) {
            const int i0 = q * nb, bs = (m - i0 < nb) ? m - i0 : nb;
            DiagArgs d{};
            d.m = m; d.n = n; d.i0 = i0; d.bs = bs; d.q = q;
            d.U = U; d.ldu = ldu; d.lam = lam; d.B = B; d.ldb = ldb;
            d.V = V; d.ldv = ldv;
            d.b32 = mixed ? W32 : nullptr; d.ldb32 = ldw;
            d.skip = mixed ? o.skip : nullptr;
            d.col_len = col_len;
            if (safe) {
                d.safe = *safe;
                d.use_safe = 1;
            } else {
                d.safe.omega_log2 = o.omega_log2;
            }
            hipError_t e = timed(MST_PROF_DIAG, (V ? 8.0 : 4.0) * bs * bs * (double)n, s, [&] { return launch_diag(nb, ev, d, s); });
            if (e != hipSuccess) return e;
            if (q > qa) {
                GemmArgs g{};
                g.M = i0 - qa * nb; g.N = n; g.K = bs;
                g.op = GOP_SUB; g.staged = o.staged; g.split = o.split;
                g.nb = nb; g.b_row0 = i0; g.c_row0 = qa * nb; g.col_len = col_len;
                if (safe) {
                    g.kb = safe->kb; g.n_kb = n; g.q_cur = q; g.q_c = (q + 1 < nblk) ? q + 1 : -1;
                }
                if (!mixed) {
                    g.A = etr ? U + (long)(qa * nb) * ldu + i0 : U + (long)i0 * ldu + qa * nb;
                    g.lda = ldu; g.a_ct = amode;
                    g.B = B + i0; g.ldb = ldb;
                    g.C = B + qa * nb; g.ldc = ldb;
                    if (V) {
                        g.op = GOP_GEN_SUB;
                        g.A2 = V + (long)i0 * ldv + qa * nb; g.lda2 = ldv; g.glam = lam;
                    }
                    e = timed(MST_PROF_GEMM_F64, gemm_flops(g), s, [&] { return launch_gemm_f64(g, s); });
                } else {
                    g.A = U32 + (long)i0 * ldu32 + qa * nb; g.lda = ldu32;
                    g.B = W32 + i0; g.ldb = ldw;
                    g.C = W32 + qa * nb; g.ldc = ldw;
                    g.skip = o.skip;
                    e = timed(MST_PROF_GEMM_F32, gemm_flops(g), s, [&] { return launch_gemm_f32(g, s); });
                }
                if (e != hipSuccess) return e;
            }
        }
        if (qa > 0) {
            // Two-level deferral: the rows above a group of outer blocks
            // (kSuperRows rows) get X of all its outer blocks in one GEMM once
            // the group is solved (K = its rows), so most of the substitution
            // runs as a few deep products. Inside the group the order is
            // binary: after the i-th outer block from the group's bottom is
            // solved, X of the last L = lowbit(i + 1) solved blocks goes into
            // the L blocks above them (of four: 1 into 1, 2 into 2, 1 into 1),
            // which gives every row each block's X exactly once, keeps the
            // next block's rows current, and makes the middle product twice
            // as deep as one outer block.
            const int G = (o.outer < kSuperRows) ? kSuperRows / o.outer : 1;   // outer blocks per group
            const int g_lo = (ob / G) * G;
            const int g_hi = (g_lo + G - 1 < nob - 1) ? g_lo + G - 1 : nob - 1;
            const int g0 = q_first(g_lo) * nb;
            hipError_t e = hipSuccess;
            if (ob == g_lo) {
                if (g0 > 0 && (e = substitute_range(g_lo, g_hi, 0, g0, s)) != hipSuccess) return e;
            } else {
                const int i = g_hi - ob, L = (i + 1) & -(i + 1);
                const int lo = (ob - L > g_lo) ? ob - L : g_lo;
                if ((e = substitute_range(ob, ob + L - 1, q_first(lo) * nb, qa * nb, s)) != hipSuccess) return e;
            }
        }
    }
    return hipSuccess;
}

// ---------------------------------------------------------------- adjoint block loop
// ev: EV_UPPER_C (the adjoint), EV_UPPER_T, or EV_LOWER_N (E(r, c) = A(r, c) from
// A's lower triangle): forward substitution, blocks top to bottom
hipError_t adjoint_loop(int m, int n, const zd* U, long ldu, const zd* lam, zd* G, long ldg,
                        const Opts& o, hipStream_t s, int ev = EV_UPPER_C) {
    // (outer blocks as given: 512-row blocks measured slower here than 256)
    const bool etr = ev_tr(ev);
    const int amode = etr ? (ev_cj(ev) ? 1 : 2) : 0;
    const int nb = o.nb, P = o.outer / o.nb;
    const int nblk = (m + nb - 1) / nb;
    const int nob = (nblk + P - 1) / P;
    const bool fused = o.fuse && o.outer <= block_rows_for(n, o.nb, o.fuse_width, true) && block_fusable(o.nb);
    for (int ob = 0; ob < nob; ++ob) {
        const int qa = ob * P, qb = (qa + P < nblk ? qa + P : nblk) - 1;
        const int end = ((qb + 1) * nb < m) ? (qb + 1) * nb : m;
        if (fused) {
            BlockArgs b{};
            b.m = m; b.n = n; b.nb = nb; b.qa = qa; b.iS = qa * nb; b.rows = end - qa * nb;
            b.U = U; b.ldu = ldu; b.lam = lam; b.B = G; b.ldb = ldg;
            b.width = o.fuse_width;
            b.safe.omega_log2 = o.omega_log2;
            const double fl = 4.0 * b.rows * (double)b.rows * n;
            hipError_t e = timed(MST_PROF_DIAG, fl, s, [&] { return launch_block(ev, b, s); });
            if (e != hipSuccess) return e;
        }
        for (int q = qa; q <= qb && !fused; ++q) {
            const int i0 = q * nb, bs = (m - i0 < nb) ? m - i0 : nb;
            const int i1 = i0 + bs;
            DiagArgs d{};
            d.m = m; d.n = n; d.i0 = i0; d.bs = bs; d.q = q;
            d.U = U; d.ldu = ldu; d.lam = lam; d.B = G; d.ldb = ldg;
            d.safe.omega_log2 = o.omega_log2;
            hipError_t e = timed(MST_PROF_DIAG, 4.0 * bs * bs * (double)n, s, [&] { return launch_diag(nb, ev, d, s); });
            if (e != hipSuccess) return e;
            if (q < qb) {
                // G(i1:end) -= E(i1:end, i0:i1) Y(i0:i1), E = U^H for the adjoint
                GemmArgs g{};
                g.M = end - i1; g.N = n; g.K = bs; g.op = GOP_SUB; g.staged = o.staged; g.split = o.split;
                g.A = etr ? U + (long)i1 * ldu + i0 : U + (long)i0 * ldu + i1; g.lda = ldu; g.a_ct = amode;
                g.B = G + i0; g.ldb = ldg;
                g.C = G + i1; g.ldc = ldg;
                e = timed(MST_PROF_GEMM_F64, gemm_flops(g), s, [&] { return launch_gemm_f64(g, s); });
                if (e != hipSuccess) return e;
            }
        }
        // Two-level deferral, as in the back-substitution loop: the rows below
        // a group of outer blocks (kSuperRows rows) get Y of all its outer
        // blocks in one product once the group is solved; inside the group,
        // after its i-th outer block from the top, Y of the last
        // L = lowbit(i + 1) solved blocks goes into the L blocks below them.
        const int Gp = (o.outer < kSuperRows) ? kSuperRows / o.outer : 1;
        const int g_lo = (ob / Gp) * Gp;
        const int g_hi = (g_lo + Gp - 1 < nob - 1) ? g_lo + Gp - 1 : nob - 1;
        const int g_end = ((g_hi * P + P) * nb < m) ? (g_hi * P + P) * nb : m;
        // rows [r1, r2) -= E(r1:r2, x0:x1) Y(x0:x1)
        auto below = [&](int x0, int x1, int r1, int r2) -> hipError_t {
            if (r2 <= r1) return hipSuccess;
            GemmArgs g{};
            g.M = r2 - r1; g.N = n; g.K = x1 - x0; g.op = GOP_SUB; g.staged = o.staged; g.split = o.split;
            g.A = etr ? U + (long)r1 * ldu + x0 : U + (long)x0 * ldu + r1; g.lda = ldu; g.a_ct = amode;
            g.B = G + x0; g.ldb = ldg;
            g.C = G + r1; g.ldc = ldg;
            return timed(MST_PROF_GEMM_F64, gemm_flops(g), s, [&] { return launch_gemm_f64(g, s); });
        };
        hipError_t e = hipSuccess;
        if (ob == g_hi) {
            if ((e = below(g_lo * P * nb, g_end, g_end, m)) != hipSuccess) return e;
        } else {
            const int i = ob - g_lo, L = (i + 1) & -(i + 1);
            const int hi = (ob + L < g_hi) ? ob + L : g_hi;   // last block that receives
            const int r2 = ((hi + 1) * P * nb < m) ? (hi + 1) * P * nb : m;
            if ((e = below((ob - L + 1) * P * nb, end, end, r2)) != hipSuccess) return e;
        }
    }
    return hipSuccess;
}

hipError_t residual(int m, int n, const zd* U, long ldu, const zd* lam, const zd* X, long ldx,
                    const zd* B0, long ldb0, zd* R, long ldr, hipStream_t s, int staged = 0,
                    const int* skip = nullptr, int split = 0) {
    GemmArgs g{};
    g.skip = skip;
    g.split = split;
    g.M = m; g.N = n; g.K = m; g.op = GOP_RESID; g.staged = staged;
    g.A = U; g.lda = ldu;
    g.B = X; g.ldb = ldx;
    g.C = R; g.ldc = ldr;
    g.B0 = B0; g.ldb0 = ldb0; g.lam = lam;
    return timed(MST_PROF_RESID, 4.0 * m * (double)m * n, s, [&] { return launch_gemm_f64(g, s); });
}

// Real-arithmetic solve: fused blocks of up to 256 rows (bottom to top; the
// 64-row diagonal blocks and the updates inside a fused block in one kernel),
// the rows of each outer block updated after each of its fused blocks, and
// the two-level deferral above the outer blocks as in forward_loop.
hipError_t real_loop(int m, int n, const double* U, long ldu, const double* lam, double* B, long ldb,
                     int outer, hipStream_t s) {
    // fused blocks: the largest of 256, 192, 128, 64 rows that divides the outer block
    const int nb = (outer % 256 == 0) ? 256 : (outer % 192 == 0) ? 192 : (outer % 128 == 0) ? 128 : 64;
    const int P = outer / nb;
    const int nblk = (m + nb - 1) / nb;
    const int nob = (nblk + P - 1) / P;
    auto q_first = [&](int ob) { return ob * P; };
    auto row_end = [&](int ob) {
        const int qe = (ob * P + P < nblk ? ob * P + P : nblk);
        return (qe * nb < m) ? qe * nb : m;
    };
    // B(r0:r1) -= U(r0:r1, x0:x1) X(x0:x1)
    auto gemm = [&](int r0, int r1, int x0, int x1) -> hipError_t {
        if (r1 <= r0 || x1 <= x0) return hipSuccess;
        RealGemmArgs g{};
        g.M = r1 - r0; g.N = n; g.K = x1 - x0;
        g.A = U + (long)x0 * ldu + r0; g.lda = ldu;
        g.B = B + x0; g.ldb = ldb;
        g.C = B + r0; g.ldc = ldb;
        return timed(MST_PROF_GEMM_F64, 2.0 * g.M * (double)g.N * g.K, s, [&] { return launch_gemm_real(g, s); });
    };
    for (int ob = nob - 1; ob >= 0; --ob) {
        const int qa = q_first(ob), qb = (ob * P + P < nblk ? ob * P + P : nblk) - 1;
        for (int q = qb; q >= qa; --q) {
            const int i0 = q * nb, bs = (m - i0 < nb) ? m - i0 : nb;
            RealDiagArgs d{};
            d.m = m; d.n = n; d.i0 = i0; d.bs = bs;
            d.U = U; d.ldu = ldu; d.lam = lam; d.B = B; d.ldb = ldb;
            hipError_t e = timed(MST_PROF_DIAG, 1.0 * bs * bs * (double)n, s, [&] { return launch_block_real(d, s); });
            if (e != hipSuccess) return e;
            if (q > qa && (e = gemm(qa * nb, i0, i0, i0 + bs)) != hipSuccess) return e;
        }
        if (qa > 0) {
            const int G = (outer < kSuperRows) ? kSuperRows / outer : 1;
            const int g_lo = (ob / G) * G;
            const int g_hi = (g_lo + G - 1 < nob - 1) ? g_lo + G - 1 : nob - 1;
            const int g0 = q_first(g_lo) * nb;
            hipError_t e = hipSuccess;
            if (ob == g_lo) {
                if (g0 > 0 && (e = gemm(0, g0, g0, row_end(g_hi))) != hipSuccess) return e;
            } else {
                // the same binary order as the complex solve's groups
                const int i = g_hi - ob, L = (i + 1) & -(i + 1);
                const int lo = (ob - L > g_lo) ? ob - L : g_lo;
                if ((e = gemm(q_first(lo) * nb, qa * nb, qa * nb, row_end(ob + L - 1))) != hipSuccess) return e;
            }
        }
    }
    return hipSuccess;
}

mst_status check_mat(const void* p, int ld, int rows, int cols, int ppos, int ldpos) {
    if (ld < (rows > 1 ? rows : 1)) return bad(ldpos);
    if ((long)rows * cols > 0 && p == nullptr) return bad(ppos);
    return MST_OK;
}

// Bytes safe_solve takes from its workspace (without V): the pieces it asks
// for below, in the same order, each rounded as Workspace rounds them.
size_t safe_ws_bytes(int m, int n, int nb) {
    const size_t nblk = (size_t)((m + nb - 1) / nb);
    return ws_round(n * sizeof(double)) + ws_round(n * sizeof(int)) + ws_round(nblk * n * sizeof(int)) +
           3 * ws_round(m * sizeof(double)) + ws_round(nblk * sizeof(double)) + ws_round(sizeof(double));
}

// safe solve into an existing workspace scope
mst_status safe_solve(int m, int n, const zd* U, long ldu, const zd* lam, zd* B, long ldb,
                      const int* col_len, double* scale, int* klog, const Opts& o, hipStream_t s,
                      Workspace& ws, const zd* V = nullptr, long ldv = 0) {
    const int nb = o.nb;
    const int nblk = (m + nb - 1) / nb;
    double *G, *cn_in, *above, *colmax, *above_sum, *delta;
    int *kcur, *kb;
    HIPCHK(ws_get(ws, (size_t)n, &G));
    HIPCHK(ws_get(ws, (size_t)n, &kcur));
    HIPCHK(ws_get(ws, (size_t)nblk * n, &kb));
    HIPCHK(ws_get(ws, (size_t)m, &cn_in));
    HIPCHK(ws_get(ws, (size_t)m, &above));
    HIPCHK(ws_get(ws, (size_t)m, &colmax));
    HIPCHK(ws_get(ws, (size_t)nblk, &above_sum));
    HIPCHK(ws_get(ws, (size_t)1, &delta));
    HIPCHK(timed(MST_PROF_AUX, 0.0, s, [&] { return launch_norms(m, U, ldu, nb, cn_in, above, colmax, above_sum, delta, s); }));
    HIPCHK(timed(MST_PROF_AUX, 0.0, s, [&] { return launch_colinit(m, n, B, ldb, col_len, G, kcur, s); }));
    SafeState st{};
    st.G = G; st.kcur = kcur; st.kb = kb; st.cn_in = cn_in; st.above_sum = above_sum;
    st.delta = delta; st.omega_log2 = o.omega_log2; st.force_checked = o.force_checked ? 1 : 0;
    if (V) {
        // the same sums and zero-pivot replacement for V (pencil bound of Alg 9)
        double *cn_v, *above_v, *colmax_v, *above_sum_v, *delta_v;
        HIPCHK(ws_get(ws, (size_t)m, &cn_v));
        HIPCHK(ws_get(ws, (size_t)m, &above_v));
        HIPCHK(ws_get(ws, (size_t)m, &colmax_v));
        HIPCHK(ws_get(ws, (size_t)nblk, &above_sum_v));
        HIPCHK(ws_get(ws, (size_t)1, &delta_v));
        HIPCHK(timed(MST_PROF_AUX, 0.0, s, [&] { return launch_norms(m, V, ldv, nb, cn_v, above_v, colmax_v, above_sum_v, delta_v, s); }));
        st.above_sum_v = above_sum_v;
        st.delta_v = delta_v;
    }
    HIPCHK(forward_loop(m, n, U, ldu, nullptr, 0, lam, B, ldb, nullptr, 0, o, &st, col_len, s, V, ldv));
    HIPCHK(timed(MST_PROF_AUX, 0.0, s, [&] { return launch_finalize(m, n, nb, B, ldb, col_len, kcur, kb, scale, klog, s); }));
    return MST_OK;
}

mst_status plain_solve(int m, int n, const zd* U, long ldu, const zd* lam, zd* B, long ldb,
                       const Opts& o, hipStream_t s, Workspace& ws) {
    if (o.precision == 0) {
        HIPCHK(forward_loop(m, n, U, ldu, nullptr, 0, lam, B, ldb, nullptr, 0, o, nullptr, nullptr, s));
        return MST_OK;
    }
    // FP32 substitution GEMMs, FP64 diagonal blocks, FP64 iterative refinement.
    // Every right-hand side is brought near 1 by an exact power of two per
    // column before it is rounded to FP32 (the solve is linear: the solution
    // carries the same factor, removed when it is added to X). The stop test
    // and the undo of a sweep that raised the residual run on the device
    // (RefineCtl), so the call stays asynchronous; the undo restores a copy of
    // the iterate taken before the sweep.
    const int S = o.sweeps;
    const int nch = (m + kRowChunk - 1) / kRowChunk;
    zf *U32, *W32;
    zd *B0, *R, *Xp, *udiag;
    double *part, *rowoff, *rel;
    int *einit, *ebuf;
    RefineCtl* ctl;
    HIPCHK(ws_get(ws, (size_t)m * m, &U32));
    HIPCHK(ws_get(ws, (size_t)m * n, &W32));
    HIPCHK(ws_get(ws, (size_t)m * n, &B0));
    HIPCHK(ws_get(ws, (size_t)m * n, &R));
    HIPCHK(ws_get(ws, (size_t)m * n, &Xp));
    HIPCHK(ws_get(ws, (size_t)m, &udiag));
    HIPCHK(ws_get(ws, (size_t)nch * m, &part));
    HIPCHK(ws_get(ws, (size_t)m, &rowoff));
    HIPCHK(ws_get(ws, (size_t)n, &rel));
    HIPCHK(ws_get(ws, (size_t)n, &einit));
    HIPCHK(ws_get(ws, (size_t)2 * n, &ebuf));
    HIPCHK(ws_get(ws, (size_t)1, &ctl));
    Opts om = o;
    om.skip = &ctl->stop;
    const int* stop = &ctl->stop;
    auto aux = [&](auto&& f) { return timed(MST_PROF_AUX, 0.0, s, f); };
    HIPCHK(aux([&] { return launch_refine_init(ctl, o.report, S + 1, s); }));
    HIPCHK(aux([&] { return launch_to_f32(m, m, U, ldu, U32, m, true, s); }));
    HIPCHK(aux([&] { return launch_rowabs(m, U, ldu, part, rowoff, udiag, s); }));
    HIPCHK(aux([&] { return launch_copy(m, n, B, ldb, B0, m, s); }));
    // X0: the FP32-GEMM solve of 2^-e B, then X0 = 2^e (that solution)
    HIPCHK(aux([&] { return launch_colstats(m, n, B, ldb, nullptr, 0, rowoff, udiag, lam, einit, rel, nullptr, s); }));
    HIPCHK(aux([&] { return launch_to_f32_cols(m, n, B, ldb, einit, W32, m, nullptr, s); }));
    HIPCHK(forward_loop(m, n, U, ldu, U32, m, lam, B, ldb, W32, m, o, nullptr, nullptr, s));
    HIPCHK(aux([&] { return launch_scale_cols(m, n, B, ldb, einit, s); }));
    // The residual of iterate t into R, its test, and the undo of sweep t when
    // it raised the residual. The exponents for the next correction go to the
    // half of ebuf that sweep t did not use.
    auto check = [&](int t) -> hipError_t {
        hipError_t e = residual(m, n, U, ldu, lam, B, ldb, B0, m, R, m, s, o.staged, stop, o.split);
        if (e != hipSuccess) return e;
        int* et = ebuf + (size_t)((t + 1) & 1) * n;
        if ((e = aux([&] { return launch_colstats(m, n, R, m, B, ldb, rowoff, udiag, lam, et, rel, stop, s); })) != hipSuccess)
            return e;
        if ((e = aux([&] { return launch_refine_ctl(n, t, rel, o.refine_tol, ctl, o.report, s); })) != hipSuccess)
            return e;
        if (t == 0) return hipSuccess;
        return aux([&] { return launch_copy_cond(m, n, Xp, m, B, ldb, nullptr, &ctl->rb[t], s); });
    };
    for (int sw = 1; sw <= S; ++sw) {
        HIPCHK(check(sw - 1));
        // correction: solve (U - lam I) D = R with 2^-e R in FP32 (D into R), X += 2^e D
        const int* es = ebuf + (size_t)(sw & 1) * n;
        HIPCHK(aux([&] { return launch_to_f32_cols(m, n, R, m, es, W32, m, stop, s); }));
        HIPCHK(forward_loop(m, n, U, ldu, U32, m, lam, R, m, W32, m, om, nullptr, nullptr, s));
        HIPCHK(aux([&] { return launch_copy_cond(m, n, B, ldb, Xp, m, stop, nullptr, s); }));
        HIPCHK(aux([&] { return launch_axpy_cols(m, n, R, m, es, 1.0, B, ldb, stop, nullptr, s); }));
    }
    if (o.report) HIPCHK(check(S));
    return MST_OK;
}

// Eigenvectors from a (generalized) Schur form: triangular eigenvectors Z into
// workspace, X = Qb Z on the matrix cores (Z upper triangular), columns of X
// scaled to unit 2-norm. S == nullptr: Alg 6; otherwise Alg 10.
mst_status eig_from_schur(int m, const zd* T, long ldt, const zd* S, long lds, const zd* Qb, long ldq,
                          zd* X, long ldx, zd* eig, int* klog, const Opts& o, hipStream_t s) {
    Workspace ws(s);
    zd* Z;
    int* col_len;
    double* scale;
    HIPCHK(ws_get(ws, (size_t)m * m, &Z));
    HIPCHK(ws_get(ws, (size_t)m, &col_len));
    HIPCHK(ws_get(ws, (size_t)m, &scale));
    if (S) {
        HIPCHK(timed(MST_PROF_AUX, 0.0, s, [&] { return launch_gen_triang_setup(m, T, ldt, S, lds, Z, m, eig, col_len, s); }));
    } else {
        HIPCHK(timed(MST_PROF_AUX, 0.0, s, [&] { return launch_triang_setup(m, T, ldt, Z, m, eig, col_len, s); }));
    }
    mst_status st = safe_solve(m, m, T, ldt, eig, Z, m, col_len, scale, klog, o, s, ws, S, lds);
    if (st != MST_OK) return st;
    HIPCHK(timed(MST_PROF_AUX, 0.0, s, [&] { return launch_triang_diag(m, Z, m, scale, s); }));
    GemmArgs g{};
    g.M = m; g.N = m; g.K = m; g.op = GOP_TRMM;
    g.A = Qb; g.lda = ldq;
    g.B = Z; g.ldb = m;
    g.C = X; g.ldc = ldx;
    HIPCHK(timed(MST_PROF_RESID, 4.0 * m * (double)m * m, s, [&] { return launch_gemm_f64(g, s); }));
    HIPCHK(timed(MST_PROF_AUX, 0.0, s, [&] { return launch_normalize_cols(m, m, X, ldx, s); }));
    return MST_OK;
}

// Device address of `scratch` on the current device, looked up once per
// device (each device holds its own copy of the array at its own address).
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

hipError_t scratch_ptr(void** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

}  // namespace

extern "C" {

mst_status mstrsm(int m, int n, const void* U, int ldu, const void* shifts, void* B, int ldb,
                  const mst_opts* opt, void* stream) {
    entry("mstrsm", m, n);
    if (m < 0) return bad(1);
    if (n < 0) return bad(2);
    mst_status st;
    if ((st = check_mat(U, ldu, m, n > 0 ? m : 0, 3, 4)) != MST_OK) return st;
    if (n > 0 && m > 0 && !shifts) return bad(5);
    if ((st = check_mat(B, ldb, m, n, 6, 7)) != MST_OK) return st;
    Opts o;
    if ((st = read_opts(opt, o, 8)) != MST_OK) return st;
    if (m == 0 || n == 0) return MST_OK;
    hipStream_t s = (hipStream_t)stream;
    Workspace ws(s);
    return plain_solve(m, n, (const zd*)U, ldu, (const zd*)shifts, (zd*)B, ldb, o, s, ws);
}

mst_status mstrsm_safe(int m, int n, const void* U, int ldu, const void* shifts, void* B, int ldb,
                       const int* col_len, double* scale, int* scale_log2, const mst_opts* opt,
                       void* stream) {
    entry("mstrsm_safe", m, n);
    if (m < 0) return bad(1);
    if (n < 0) return bad(2);
    mst_status st;
    if ((st = check_mat(U, ldu, m, n > 0 ? m : 0, 3, 4)) != MST_OK) return st;
    if (n > 0 && m > 0 && !shifts) return bad(5);
    if ((st = check_mat(B, ldb, m, n, 6, 7)) != MST_OK) return st;
    if (n > 0 && !scale) return bad(9);
    Opts o;
    if ((st = read_opts(opt, o, 11)) != MST_OK) return st;
    if (o.precision != 0) return unsupported("precision 1 is offered by the plain upper solve only");
    if (n == 0) return MST_OK;
    hipStream_t s = (hipStream_t)stream;
    Workspace ws(s);
    if (m == 0) {
        // no rows: s_j = 1, k_j = 0
        int* kcur;
        int* kb;
        HIPCHK(ws_get(ws, (size_t)n, &kcur));
        HIPCHK(ws_get(ws, (size_t)n, &kb));
        HIPCHK(launch_fill_int(n, 0, kcur, s));
        HIPCHK(timed(MST_PROF_AUX, 0.0, s, [&] { return launch_finalize(0, n, o.nb, (zd*)B, 1, nullptr, kcur, kb, scale, scale_log2, s); }));
        return MST_OK;
    }
    return safe_solve(m, n, (const zd*)U, ldu, (const zd*)shifts, (zd*)B, ldb, col_len, scale,
                      scale_log2, o, s, ws);
}

mst_status mstrsm_safe_noalloc(int m, int n, const void* U, int ldu, const void* shifts, void* B, int ldb,
                               const int* col_len, double* scale, int* scale_log2, const mst_opts* opt,
                               void* stream) {
    entry("mstrsm_safe_noalloc", m, n);
    if (m < 0) return bad(1);
    if (n < 0) return bad(2);
    mst_status st;
    if ((st = check_mat(U, ldu, m, n > 0 ? m : 0, 3, 4)) != MST_OK) return st;
    if (n > 0 && m > 0 && !shifts) return bad(5);
    if ((st = check_mat(B, ldb, m, n, 6, 7)) != MST_OK) return st;
    if (n > 0 && !scale) return bad(9);
    Opts o;
    if ((st = read_opts(opt, o, 11)) != MST_OK) return st;
    if (o.precision != 0) return unsupported("precision 1 is offered by the plain upper solve only");
    if (o.overlap) return unsupported("overlap = 1 needs a second stream; not offered without allocation");
    if (n == 0) return MST_OK;
    // m == 0 takes kcur and kb (n ints each) for the final pass
    const size_t need = (m == 0) ? 2 * ws_round((size_t)n * sizeof(int)) : safe_ws_bytes(m, n, o.nb);
    if (need > MST_SCRATCH_BYTES) {
        snprintf(t_err, sizeof(t_err), "scratch of %zu bytes needed, the limit is %u bytes", need,
                 (unsigned)MST_SCRATCH_BYTES);
        if (log_on()) fprintf(stderr, "[mstrsm] %s: %s\n", t_entry, t_err);
        return MST_ENOMEM;
    }
    void* base = nullptr;
    HIPCHK(scratch_ptr(&base));
    hipStream_t s = (hipStream_t)stream;
    Workspace ws(s, base, MST_SCRATCH_BYTES);
    if (m == 0) {
        int* kcur;
        int* kb;
        HIPCHK(ws_get(ws, (size_t)n, &kcur));
        HIPCHK(ws_get(ws, (size_t)n, &kb));
        HIPCHK(launch_fill_int(n, 0, kcur, s));
        HIPCHK(timed(MST_PROF_AUX, 0.0, s, [&] { return launch_finalize(0, n, o.nb, (zd*)B, 1, nullptr, kcur, kb, scale, scale_log2, s); }));
        return MST_OK;
    }
    return safe_solve(m, n, (const zd*)U, ldu, (const zd*)shifts, (zd*)B, ldb, col_len, scale,
                      scale_log2, o, s, ws);
}

mst_status mstrsm_adjoint(int m, int n, const void* U, int ldu, const void* shifts, void* G, int ldg,
                          const mst_opts* opt, void* stream) {
    entry("mstrsm_adjoint", m, n);
    if (m < 0) return bad(1);
    if (n < 0) return bad(2);
    mst_status st;
    if ((st = check_mat(U, ldu, m, n > 0 ? m : 0, 3, 4)) != MST_OK) return st;
    if (n > 0 && m > 0 && !shifts) return bad(5);
    if ((st = check_mat(G, ldg, m, n, 6, 7)) != MST_OK) return st;
    Opts o;
    if ((st = read_opts(opt, o, 8)) != MST_OK) return st;
    if (o.precision != 0) return unsupported("precision 1 is offered by the plain upper solve only");
    if (m == 0 || n == 0) return MST_OK;
    HIPCHK(adjoint_loop(m, n, (const zd*)U, ldu, (const zd*)shifts, (zd*)G, ldg, o, (hipStream_t)stream));
    return MST_OK;
}

mst_status mstrsm_op(int side, int uplo, int op, int m, int n, const void* A, int lda, const void* shifts,
                     void* B, int ldb, const mst_opts* opt, void* stream) {
    entry("mstrsm_op", m, n);
    if (side != 'L' && side != 'R') return bad(1);
    if (uplo != 'U' && uplo != 'L') return bad(2);
    if (op != 'N' && op != 'T' && op != 'C') return bad(3);
    if (m < 0) return bad(4);
    if (n < 0) return bad(5);
    mst_status st;
    if ((st = check_mat(A, lda, m, n > 0 ? m : 0, 6, 7)) != MST_OK) return st;
    if (n > 0 && m > 0 && !shifts) return bad(8);
    if ((st = check_mat(B, ldb, m, n, 9, 10)) != MST_OK) return st;
    Opts o;
    if ((st = read_opts(opt, o, 11)) != MST_OK) return st;
    // right side: x op(A - l I) = b for the row vector x, i.e. op(A - l I)^T x^T = b^T
    int eop = op;
    if (side == 'R') {
        if (op == 'C') return unsupported("right side with op C is not offered");
        eop = (op == 'N') ? 'T' : 'N';
    }
    if (o.precision != 0 && !(uplo == 'U' && eop == 'N')) return unsupported("precision 1 is offered by the plain upper solve only");
    if (m == 0 || n == 0) return MST_OK;
    hipStream_t s = (hipStream_t)stream;
    const zd* Az = (const zd*)A;
    const zd* lz = (const zd*)shifts;
    zd* Bz = (zd*)B;
    if (uplo == 'U' && eop == 'N') {
        Workspace ws(s);
        return plain_solve(m, n, Az, lda, lz, Bz, ldb, o, s, ws);
    }
    int ev;
    if (uplo == 'U') ev = (eop == 'T') ? EV_UPPER_T : EV_UPPER_C;
    else ev = (eop == 'N') ? EV_LOWER_N : (eop == 'T') ? EV_LOWER_T : EV_LOWER_C;
    if (ev_fwd(ev)) {
        HIPCHK(adjoint_loop(m, n, Az, lda, lz, Bz, ldb, o, s, ev));
    } else {
        HIPCHK(forward_loop(m, n, Az, lda, nullptr, 0, lz, Bz, ldb, nullptr, 0, o, nullptr, nullptr, s,
                            nullptr, 0, ev));
    }
    return MST_OK;
}

mst_status mstrsm_real(int m, int n, const double* U, int ldu, const double* shifts, double* B, int ldb,
                       const mst_opts* opt, void* stream) {
    entry("mstrsm_real", m, n);
    if (m < 0) return bad(1);
    if (n < 0) return bad(2);
    mst_status st;
    if ((st = check_mat(U, ldu, m, n > 0 ? m : 0, 3, 4)) != MST_OK) return st;
    if (n > 0 && m > 0 && !shifts) return bad(5);
    if ((st = check_mat(B, ldb, m, n, 6, 7)) != MST_OK) return st;
    Opts o;
    if ((st = read_opts(opt, o, 8)) != MST_OK) return st;
    if (o.precision != 0) return unsupported("precision 1 is offered by the plain upper solve only");
    const int outer = (opt && opt->outer_nb) ? opt->outer_nb : 256;
    if (outer < 64 || outer % 64) return bad(8);
    if (m == 0 || n == 0) return MST_OK;
    HIPCHK(real_loop(m, n, U, ldu, shifts, B, ldb, outer, (hipStream_t)stream));
    return MST_OK;
}

mst_status mstrsm_real_op(int side, int uplo, int op, int m, int n, const double* A, int lda,
                          const double* shifts, double* B, int ldb, const mst_opts* opt, void* stream) {
    entry("mstrsm_real_op", m, n);
    if (side != 'L' && side != 'R') return bad(1);
    if (uplo != 'U' && uplo != 'L') return bad(2);
    if (op != 'N' && op != 'T' && op != 'C') return bad(3);
    if (m < 0) return bad(4);
    if (n < 0) return bad(5);
    mst_status st;
    if ((st = check_mat(A, lda, m, n > 0 ? m : 0, 6, 7)) != MST_OK) return st;
    if (n > 0 && m > 0 && !shifts) return bad(8);
    if ((st = check_mat(B, ldb, m, n, 9, 10)) != MST_OK) return st;
    Opts o;
    if ((st = read_opts(opt, o, 11)) != MST_OK) return st;
    if (o.precision != 0) return unsupported("precision 1 is offered by the plain upper solve only");
    const int outer = (opt && opt->outer_nb) ? opt->outer_nb : 256;
    if (outer < 64 || outer % 64) return bad(11);
    // real data: the conjugate transpose is the transpose; the right side
    // x op(A - l I) = b is op(A - l I)^T x^T = b^T
    const bool tr = (op != 'N') != (side == 'R');
    if (m == 0 || n == 0) return MST_OK;
    hipStream_t s = (hipStream_t)stream;
    if (uplo == 'U' && !tr) {
        HIPCHK(real_loop(m, n, A, lda, shifts, B, ldb, outer, s));
        return MST_OK;
    }
    // Lower or transposed: an upper-triangular copy. A lower A transposed is
    // upper; a forward substitution becomes a back substitution on the
    // reversed order, (J E J)(J x) = J b with J the reversal permutation.
    const int mode = (uplo == 'L' && tr) ? REAL_T : (uplo == 'L') ? REAL_JJ : REAL_JTJ;
    const bool rev = mode != REAL_T;
    Workspace ws(s);
    double* Uh;
    HIPCHK(ws_get(ws, (size_t)m * m, &Uh));
    HIPCHK(timed(MST_PROF_AUX, 0.0, s, [&] { return launch_real_upper_copy(m, A, lda, mode, Uh, s); }));
    if (rev) HIPCHK(timed(MST_PROF_AUX, 0.0, s, [&] { return launch_reverse_rows(m, n, B, ldb, s); }));
    HIPCHK(real_loop(m, n, Uh, m, shifts, B, ldb, outer, s));
    if (rev) HIPCHK(timed(MST_PROF_AUX, 0.0, s, [&] { return launch_reverse_rows(m, n, B, ldb, s); }));
    return MST_OK;
}

mst_status mst_grad_u(int m, int n, const void* Y, int ldy, const void* X, int ldx, void* gU, int ldgu,
                      void* stream) {
    entry("mst_grad_u", m, n);
    if (m < 0) return bad(1);
    if (n < 0) return bad(2);
    mst_status st;
    if ((st = check_mat(Y, ldy, m, n, 3, 4)) != MST_OK) return st;
    if ((st = check_mat(X, ldx, m, n, 5, 6)) != MST_OK) return st;
    if ((st = check_mat(gU, ldgu, m, m, 7, 8)) != MST_OK) return st;
    if (m == 0) return MST_OK;
    GemmArgs g{};
    g.M = m; g.N = m; g.K = n; g.op = GOP_NEG_TRIU;
    g.A = Y; g.lda = ldy;
    g.B = X; g.ldb = ldx; g.b_ct = 1;
    g.C = gU; g.ldc = ldgu;
    HIPCHK(timed(MST_PROF_RESID, 4.0 * m * (double)m * n, (hipStream_t)stream, [&] { return launch_gemm_f64(g, (hipStream_t)stream); }));
    return MST_OK;
}

mst_status mst_grad_shift(int m, int n, const void* X, int ldx, const void* Y, int ldy, void* gshift,
                          void* stream) {
    entry("mst_grad_shift", m, n);
    if (m < 0) return bad(1);
    if (n < 0) return bad(2);
    mst_status st;
    if ((st = check_mat(X, ldx, m, n, 3, 4)) != MST_OK) return st;
    if ((st = check_mat(Y, ldy, m, n, 5, 6)) != MST_OK) return st;
    if (n > 0 && !gshift) return bad(7);
    if (n == 0) return MST_OK;
    HIPCHK(timed(MST_PROF_AUX, 8.0 * m * (double)n, (hipStream_t)stream, [&] { return launch_dot(m, n, (const zd*)X, ldx, (const zd*)Y, ldy, (zd*)gshift, (hipStream_t)stream); }));
    return MST_OK;
}

mst_status mst_residual(int m, int n, const void* U, int ldu, const void* shifts, const void* X, int ldx,
                        const void* B0, int ldb0, void* R, int ldr, void* stream) {
    entry("mst_residual", m, n);
    if (m < 0) return bad(1);
    if (n < 0) return bad(2);
    mst_status st;
    if ((st = check_mat(U, ldu, m, n > 0 ? m : 0, 3, 4)) != MST_OK) return st;
    if (n > 0 && m > 0 && !shifts) return bad(5);
    if ((st = check_mat(X, ldx, m, n, 6, 7)) != MST_OK) return st;
    if ((st = check_mat(B0, ldb0, m, n, 8, 9)) != MST_OK) return st;
    if ((st = check_mat(R, ldr, m, n, 10, 11)) != MST_OK) return st;
    if (R == X && (long)m * n > 0) return bad(10);
    if (R == B0 && ldr != ldb0) return bad(11);
    if (m == 0 || n == 0) return MST_OK;
    HIPCHK(residual(m, n, (const zd*)U, ldu, (const zd*)shifts, (const zd*)X, ldx, (const zd*)B0, ldb0,
                    (zd*)R, ldr, (hipStream_t)stream));
    return MST_OK;
}

mst_status mst_triang_eig(int m, const void* T, int ldt, void* Z, int ldz, void* eigvals, int* scale_log2,
                          const mst_opts* opt, void* stream) {
    entry("mst_triang_eig", m, m);
    if (m < 0) return bad(1);
    mst_status st;
    if ((st = check_mat(T, ldt, m, m, 2, 3)) != MST_OK) return st;
    if ((st = check_mat(Z, ldz, m, m, 4, 5)) != MST_OK) return st;
    if (m > 0 && !eigvals) return bad(6);
    Opts o;
    if ((st = read_opts(opt, o, 8)) != MST_OK) return st;
    if (o.precision != 0) return unsupported("precision 1 is offered by the plain upper solve only");
    if (m == 0) return MST_OK;
    hipStream_t s = (hipStream_t)stream;
    Workspace ws(s);
    int* col_len;
    double* scale;
    HIPCHK(ws_get(ws, (size_t)m, &col_len));
    HIPCHK(ws_get(ws, (size_t)m, &scale));
    HIPCHK(timed(MST_PROF_AUX, 0.0, s, [&] { return launch_triang_setup(m, (const zd*)T, ldt, (zd*)Z, ldz, (zd*)eigvals, col_len, s); }));
    st = safe_solve(m, m, (const zd*)T, ldt, (const zd*)eigvals, (zd*)Z, ldz, col_len, scale, scale_log2,
                    o, s, ws);
    if (st != MST_OK) return st;
    HIPCHK(timed(MST_PROF_AUX, 0.0, s, [&] { return launch_triang_diag(m, (zd*)Z, ldz, scale, s); }));
    return MST_OK;
}

mst_status mstrsm_gen(int m, int n, const void* U, int ldu, const void* V, int ldv, const void* shifts,
                      void* B, int ldb, const mst_opts* opt, void* stream) {
    entry("mstrsm_gen", m, n);
    if (m < 0) return bad(1);
    if (n < 0) return bad(2);
    mst_status st;
    if ((st = check_mat(U, ldu, m, n > 0 ? m : 0, 3, 4)) != MST_OK) return st;
    if ((st = check_mat(V, ldv, m, n > 0 ? m : 0, 5, 6)) != MST_OK) return st;
    if (n > 0 && m > 0 && !shifts) return bad(7);
    if ((st = check_mat(B, ldb, m, n, 8, 9)) != MST_OK) return st;
    Opts o;
    if ((st = read_opts(opt, o, 10)) != MST_OK) return st;
    if (o.nb != 16 || o.precision != 0) return unsupported("the pencil solves run with nb 16 and precision 0 only");
    if (m == 0 || n == 0) return MST_OK;
    HIPCHK(forward_loop(m, n, (const zd*)U, ldu, nullptr, 0, (const zd*)shifts, (zd*)B, ldb, nullptr, 0, o,
                        nullptr, nullptr, (hipStream_t)stream, (const zd*)V, ldv));
    return MST_OK;
}

mst_status mstrsm_safe_gen(int m, int n, const void* U, int ldu, const void* V, int ldv,
                           const void* shifts, void* B, int ldb, const int* col_len, double* scale,
                           int* scale_log2, const mst_opts* opt, void* stream) {
    entry("mstrsm_safe_gen", m, n);
    if (m < 0) return bad(1);
    if (n < 0) return bad(2);
    mst_status st;
    if ((st = check_mat(U, ldu, m, n > 0 ? m : 0, 3, 4)) != MST_OK) return st;
    if ((st = check_mat(V, ldv, m, n > 0 ? m : 0, 5, 6)) != MST_OK) return st;
    if (n > 0 && m > 0 && !shifts) return bad(7);
    if ((st = check_mat(B, ldb, m, n, 8, 9)) != MST_OK) return st;
    if (n > 0 && !scale) return bad(11);
    Opts o;
    if ((st = read_opts(opt, o, 13)) != MST_OK) return st;
    if (o.nb != 16 || o.precision != 0) return unsupported("the pencil solves run with nb 16 and precision 0 only");
    if (n == 0) return MST_OK;
    hipStream_t s = (hipStream_t)stream;
    Workspace ws(s);
    if (m == 0) {
        int* kcur;
        int* kb;
        HIPCHK(ws_get(ws, (size_t)n, &kcur));
        HIPCHK(ws_get(ws, (size_t)n, &kb));
        HIPCHK(launch_fill_int(n, 0, kcur, s));
        HIPCHK(timed(MST_PROF_AUX, 0.0, s, [&] { return launch_finalize(0, n, o.nb, (zd*)B, 1, nullptr, kcur, kb, scale, scale_log2, s); }));
        return MST_OK;
    }
    return safe_solve(m, n, (const zd*)U, ldu, (const zd*)shifts, (zd*)B, ldb, col_len, scale,
                      scale_log2, o, s, ws, (const zd*)V, ldv);
}

mst_status mst_gen_triang_eig(int m, const void* T, int ldt, const void* S, int lds, void* Z, int ldz,
                              void* eigvals, int* scale_log2, const mst_opts* opt, void* stream) {
    entry("mst_gen_triang_eig", m, m);
    if (m < 0) return bad(1);
    mst_status st;
    if ((st = check_mat(T, ldt, m, m, 2, 3)) != MST_OK) return st;
    if ((st = check_mat(S, lds, m, m, 4, 5)) != MST_OK) return st;
    if ((st = check_mat(Z, ldz, m, m, 6, 7)) != MST_OK) return st;
    if (m > 0 && !eigvals) return bad(8);
    Opts o;
    if ((st = read_opts(opt, o, 10)) != MST_OK) return st;
    if (o.nb != 16 || o.precision != 0) return unsupported("the pencil solves run with nb 16 and precision 0 only");
    if (m == 0) return MST_OK;
    hipStream_t s = (hipStream_t)stream;
    Workspace ws(s);
    int* col_len;
    double* scale;
    HIPCHK(ws_get(ws, (size_t)m, &col_len));
    HIPCHK(ws_get(ws, (size_t)m, &scale));
    HIPCHK(timed(MST_PROF_AUX, 0.0, s, [&] { return launch_gen_triang_setup(m, (const zd*)T, ldt, (const zd*)S, lds, (zd*)Z, ldz, (zd*)eigvals, col_len, s); }));
    st = safe_solve(m, m, (const zd*)T, ldt, (const zd*)eigvals, (zd*)Z, ldz, col_len, scale, scale_log2,
                    o, s, ws, (const zd*)S, lds);
    if (st != MST_OK) return st;
    HIPCHK(timed(MST_PROF_AUX, 0.0, s, [&] { return launch_triang_diag(m, (zd*)Z, ldz, scale, s); }));
    return MST_OK;
}

mst_status mst_eig_schur(int m, const void* T, int ldt, const void* Q, int ldq, void* X, int ldx,
                         void* eigvals, int* scale_log2, const mst_opts* opt, void* stream) {
    entry("mst_eig_schur", m, m);
    if (m < 0) return bad(1);
    mst_status st;
    if ((st = check_mat(T, ldt, m, m, 2, 3)) != MST_OK) return st;
    if ((st = check_mat(Q, ldq, m, m, 4, 5)) != MST_OK) return st;
    if ((st = check_mat(X, ldx, m, m, 6, 7)) != MST_OK) return st;
    if (m > 0 && !eigvals) return bad(8);
    Opts o;
    if ((st = read_opts(opt, o, 10)) != MST_OK) return st;
    if (o.precision != 0) return unsupported("precision 1 is offered by the plain upper solve only");
    if (m == 0) return MST_OK;
    return eig_from_schur(m, (const zd*)T, ldt, nullptr, 0, (const zd*)Q, ldq, (zd*)X, ldx, (zd*)eigvals,
                          scale_log2, o, (hipStream_t)stream);
}

mst_status mst_gen_eig_schur(int m, const void* T, int ldt, const void* S, int lds, const void* P, int ldp,
                             void* X, int ldx, void* eigvals, int* scale_log2, const mst_opts* opt,
                             void* stream) {
    entry("mst_gen_eig_schur", m, m);
    if (m < 0) return bad(1);
    mst_status st;
    if ((st = check_mat(T, ldt, m, m, 2, 3)) != MST_OK) return st;
    if ((st = check_mat(S, lds, m, m, 4, 5)) != MST_OK) return st;
    if ((st = check_mat(P, ldp, m, m, 6, 7)) != MST_OK) return st;
    if ((st = check_mat(X, ldx, m, m, 8, 9)) != MST_OK) return st;
    if (m > 0 && !eigvals) return bad(10);
    Opts o;
    if ((st = read_opts(opt, o, 12)) != MST_OK) return st;
    if (o.nb != 16 || o.precision != 0) return unsupported("the pencil solves run with nb 16 and precision 0 only");
    if (m == 0) return MST_OK;
    return eig_from_schur(m, (const zd*)T, ldt, (const zd*)S, lds, (const zd*)P, ldp, (zd*)X, ldx,
                          (zd*)eigvals, scale_log2, o, (hipStream_t)stream);
}

mst_status mst_lanczos_sigma_min(int m, int N, const void* U, int ldu, const void* z, void* V, int ldv,
                                 int iters, double* sigma, double* alpha, double* beta, int* steps,
                                 const mst_opts* opt, void* stream) {
    entry("mst_lanczos_sigma_min", m, N);
    if (m < 1) return bad(1);
    if (N < 0) return bad(2);
    mst_status st;
    if ((st = check_mat(U, ldu, m, N > 0 ? m : 0, 3, 4)) != MST_OK) return st;
    if (N > 0 && !z) return bad(5);
    if ((st = check_mat(V, ldv, m, N, 6, 7)) != MST_OK) return st;
    if (iters < 1 || iters > 64) return bad(8);
    if (N > 0 && !sigma) return bad(9);
    Opts o;
    if ((st = read_opts(opt, o, 13)) != MST_OK) return st;
    if (o.precision != 0) return unsupported("precision 1 is offered by the plain upper solve only");
    if (N == 0) return MST_OK;
    hipStream_t s = (hipStream_t)stream;
    Workspace ws(s);
    zd *W, *Vp;
    int* stp = steps;
    double *al = alpha, *be = beta;
    HIPCHK(ws_get(ws, (size_t)m * N, &W));
    HIPCHK(ws_get(ws, (size_t)m * N, &Vp));
    if (!stp) HIPCHK(ws_get(ws, (size_t)N, &stp));
    if (!al) HIPCHK(ws_get(ws, (size_t)iters * N, &al));
    if (!be) HIPCHK(ws_get(ws, (size_t)iters * N, &be));
    // steps = iters (no early stop yet); vprev = 0
    HIPCHK(launch_fill_int(N, iters, stp, s));
    HIPCHK(launch_zero((long)m * N, Vp, s));
    HIPCHK(timed(MST_PROF_AUX, 0.0, s, [&] { return launch_normalize_cols(m, N, (zd*)V, ldv, s); }));
    zd* bufs[3] = {(zd*)V, W, Vp};
    long lds[3] = {ldv, m, m};
    int iv = 0, iw = 1, ip = 2;
    const zd* Uz = (const zd*)U;
    const zd* zz = (const zd*)z;
    for (int it = 0; it < iters; ++it) {
        HIPCHK(timed(MST_PROF_AUX, 0.0, s, [&] { return launch_copy(m, N, bufs[iv], lds[iv], bufs[iw], lds[iw], s); }));
        HIPCHK(forward_loop(m, N, Uz, ldu, nullptr, 0, zz, bufs[iw], lds[iw], nullptr, 0, o, nullptr,
                            nullptr, s));
        HIPCHK(adjoint_loop(m, N, Uz, ldu, zz, bufs[iw], lds[iw], o, s));
        HIPCHK(timed(MST_PROF_AUX, 0.0, s, [&] {
            return launch_lanczos_step(m, N, it, iters, bufs[iv], lds[iv], bufs[iw], lds[iw], bufs[ip],
                                       lds[ip], al, be, stp, s);
        }));
        const int nv = iw, np = iv, nw = ip;
        iv = nv; ip = np; iw = nw;
    }
    HIPCHK(timed(MST_PROF_AUX, 0.0, s, [&] { return launch_tridiag_max(N, iters, al, be, stp, sigma, s); }));
    return MST_OK;
}

mst_status mst_lanczos_restart_sigma_min(int m, int N, const void* U, int ldu, const void* z, const void* V,
                                         int ldv, int kdim, int keep, int max_restarts, double tol,
                                         double* sigma, double* resid, int* steps, int* converged,
                                         const mst_opts* opt, void* stream) {
    entry("mst_lanczos_restart_sigma_min", m, N);
    if (m < 1) return bad(1);
    if (N < 0) return bad(2);
    mst_status st;
    if ((st = check_mat(U, ldu, m, N > 0 ? m : 0, 3, 4)) != MST_OK) return st;
    if (N > 0 && !z) return bad(5);
    if ((st = check_mat(V, ldv, m, N, 6, 7)) != MST_OK) return st;
    if (kdim < 2 || kdim > trl_max_kdim()) return bad(8);
    if (keep < 1 || keep >= kdim || keep > trl_max_keep()) return bad(9);
    if (max_restarts < 0 || max_restarts > 100000) return bad(10);
    if (!(tol >= 0.0)) return bad(11);
    if (N > 0 && !sigma) return bad(12);
    Opts o;
    if ((st = read_opts(opt, o, 16)) != MST_OK) return st;
    if (o.precision != 0) return unsupported("precision 1 is offered by the plain upper solve only");
    if (N == 0) return MST_OK;
    hipStream_t s = (hipStream_t)stream;
    Workspace ws(s);
    const long qs = (long)m * N;   // one basis block
    zd *Q, *Wb, *zact;
    double *H, *beta, *Sk, *res = resid;
    int *idx, *go, *cnt, *stp = steps, *cv = converged;
    HIPCHK(ws_get(ws, (size_t)(kdim + 1) * qs, &Q));
    HIPCHK(ws_get(ws, (size_t)qs, &Wb));
    HIPCHK(ws_get(ws, (size_t)N, &zact));
    HIPCHK(ws_get(ws, (size_t)N * kdim * kdim, &H));
    HIPCHK(ws_get(ws, (size_t)N, &beta));
    HIPCHK(ws_get(ws, (size_t)N * kdim * keep, &Sk));
    HIPCHK(ws_get(ws, (size_t)2 * N, &idx));
    HIPCHK(ws_get(ws, (size_t)N, &go));
    HIPCHK(ws_get(ws, (size_t)1, &cnt));
    if (!res) HIPCHK(ws_get(ws, (size_t)N, &res));
    if (!stp) HIPCHK(ws_get(ws, (size_t)N, &stp));
    if (!cv) HIPCHK(ws_get(ws, (size_t)N, &cv));
    const zd* Uz = (const zd*)U;
    const zd* zz = (const zd*)z;
    auto aux = [&](auto&& f) { return timed(MST_PROF_AUX, 0.0, s, f); };
    HIPCHK(aux([&] { return launch_trl_init(m, N, kdim, (const zd*)V, ldv, Q, m, H, idx, stp, s); }));
    int nact = N, cur = 0, k0 = 0;
    for (int cycle = 0; cycle <= max_restarts; ++cycle) {
        int* ic = idx + (size_t)cur * N;
        for (int i = k0; i < kdim; ++i) {
            // w = (U - z I)^{-H} (U - z I)^{-1} q_i for the running shifts, then the recurrence
            HIPCHK(aux([&] { return launch_trl_gather(m, nact, ic, Q + (long)i * qs, m, Wb, m, zz, zact, s); }));
            HIPCHK(forward_loop(m, nact, Uz, ldu, nullptr, 0, zact, Wb, m, nullptr, 0, o, nullptr, nullptr, s));
            HIPCHK(adjoint_loop(m, nact, Uz, ldu, zact, Wb, m, o, s));
            HIPCHK(aux([&] { return launch_trl_orth(m, nact, i, k0, kdim, ic, Wb, m, Q, m, qs, H, beta, stp, s); }));
        }
        const int last = cycle == max_restarts;
        HIPCHK(aux([&] { return launch_trl_ritz(nact, kdim, keep, tol, last, ic, H, beta, Sk, sigma, res, cv, go, s); }));
        if (last) break;
        HIPCHK(aux([&] { return launch_trl_restart(m, nact, kdim, keep, ic, go, Q, m, qs, Sk, s); }));
        HIPCHK(aux([&] { return launch_trl_compact(nact, ic, go, idx + (size_t)(1 - cur) * N, cnt, s); }));
        // the number of shifts still running sizes the next cycle's solves
        int h_cnt = 0;
        HIPCHK(hipMemcpyAsync(&h_cnt, cnt, sizeof(int), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        nact = h_cnt;
        cur = 1 - cur;
        k0 = keep;
        if (nact == 0) break;
    }
    return MST_OK;
}

mst_status mst_profile_start(void) {
    for (auto& r : t_recs) {
        t_pool.push_back(r.a);
        t_pool.push_back(r.b);
    }
    t_recs.clear();
    t_prof = true;
    return MST_OK;
}

mst_status mst_profile_stop(double* ms, double* flops, long long* launches) {
    t_prof = false;
    double tms[MST_PROF_KINDS] = {0}, tfl[MST_PROF_KINDS] = {0};
    long long tl[MST_PROF_KINDS] = {0};
    mst_status st = MST_OK;
    for (auto& r : t_recs) {
        float e = 0.f;
        hipError_t he = hipEventSynchronize(r.b);
        if (he == hipSuccess) he = hipEventElapsedTime(&e, r.a, r.b);
        if (he != hipSuccess) st = fail_hip(he, "hipEventElapsedTime");
        if (r.kind >= 0 && r.kind < MST_PROF_KINDS) {
            tms[r.kind] += e;
            tfl[r.kind] += r.flops;
            tl[r.kind] += 1;
        }
        t_pool.push_back(r.a);
        t_pool.push_back(r.b);
    }
    t_recs.clear();
    for (int k = 0; k < MST_PROF_KINDS; ++k) {
        if (ms) ms[k] = tms[k];
        if (flops) flops[k] = tfl[k];
        if (launches) launches[k] = tl[k];
    }
    return st;
}

const char* mst_status_string(mst_status s) {
    switch (s) {
        case MST_OK: return "MST_OK";
        case MST_EARG: return "MST_EARG: invalid argument";
        case MST_EHIP: return "MST_EHIP: HIP runtime error";
        case MST_ENOMEM: return "MST_ENOMEM: out of device memory";
        case MST_EUNSUPPORTED: return "MST_EUNSUPPORTED: unsupported option combination";
        default: return "unknown mst_status";
    }
}

int mst_last_bad_arg(void) { return t_bad_arg; }
const char* mst_last_error(void) { return t_err; }
const char* mst_version(void) { return "0.1.0"; }

}  // extern "C"
