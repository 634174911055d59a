"""The C oracle under AddressSanitizer and UndefinedBehaviorSanitizer (host
code only): a small C driver, compiled together with oracle/mstrsm_oracle.c,
calls every entry point on ragged shapes (m, n = 0 included), padded leading
dimensions, exact zero pivots, variable row counts, small overflow thresholds
and the trace output of the safe solve. Any out-of-bounds access or undefined
operation aborts the driver. Numerical results are pinned elsewhere."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

DRIVER = r"""
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int oracle_mstrsm(int, int, const double*, int, const double*, double*, int);
int oracle_mstrsm_gen(int, int, const double*, int, const double*, int, const double*, double*, int);
int oracle_mstrsm_op(int, int, int, int, const double*, int, const double*, double*, int);
int oracle_mstrsm_real(int, int, const double*, int, const double*, double*, int);
int oracle_mstrsm_adjoint(int, int, const double*, int, const double*, double*, int);
int oracle_mstrsm_safe(int, int, const double*, int, const double*, double*, int, const int*, double*, int*,
                       int, int, int, double*);
int oracle_mstrsm_safe_gen(int, int, const double*, int, const double*, int, const double*, double*, int,
                           const int*, double*, int*, int, int, int);

static unsigned long long st = 88172645463325252ULL;
static double rnd(void) {  /* xorshift64, uniform in [-1, 1) */
    st ^= st << 13; st ^= st >> 7; st ^= st << 17;
    return (double)(st >> 11) / 4503599627370496.0 - 1.0;
}
/* exact-size heap blocks, so that any access past them is caught */
static double* dalloc(size_t k) { return (double*)malloc((k ? k : 1) * sizeof(double)); }

int main(void) {
    const int ms[] = {0, 1, 2, 5, 17, 64, 65, 130};
    const int ns[] = {0, 1, 3, 7};
    int calls = 0;
    for (int a = 0; a < 8; ++a) for (int b = 0; b < 4; ++b) {
        const int m = ms[a], n = ns[b], ld = m + 3;
        double* U = dalloc((size_t)2 * ld * m);
        double* V = dalloc((size_t)2 * ld * m);
        double* Ur = dalloc((size_t)ld * m);
        double* lam = dalloc((size_t)2 * n);
        double* lr = dalloc((size_t)n);
        double* B0 = dalloc((size_t)2 * ld * n);
        double* B = dalloc((size_t)2 * ld * n);
        double* Br = dalloc((size_t)ld * n);
        double* scale = dalloc((size_t)n);
        int* klog = (int*)malloc((n ? n : 1) * sizeof(int));
        int* cl = (int*)malloc((n ? n : 1) * sizeof(int));
        for (long i = 0; i < 2L * ld * m; ++i) { U[i] = rnd(); V[i] = 0.1 * rnd(); }
        for (long i = 0; i < (long)ld * m; ++i) Ur[i] = rnd();
        for (int i = 0; i < m; ++i) {
            U[2 * ((long)i * ld + i)] = 2.0 + rnd(); U[2 * ((long)i * ld + i) + 1] = rnd();
            V[2 * ((long)i * ld + i)] = 1.0; V[2 * ((long)i * ld + i) + 1] = 0.0;
            Ur[(long)i * ld + i] = 2.0 + rnd();
        }
        for (int j = 0; j < n; ++j) {
            lam[2 * j] = 0.3 * rnd(); lam[2 * j + 1] = 0.3 * rnd(); lr[j] = 0.3 * rnd();
            cl[j] = m ? (j * 7) % (m + 1) : 0;
        }
        if (n > 1 && m > 0) {  /* an exact zero pivot for shift 1 */
            lam[2] = U[0]; lam[3] = U[1]; lr[1] = Ur[0];
        }
        for (long i = 0; i < 2L * ld * n; ++i) B0[i] = rnd();
        for (long i = 0; i < (long)ld * n; ++i) Br[i] = rnd();
#define FRESH() memcpy(B, B0, (size_t)2 * ld * n * sizeof(double))
        FRESH(); calls += oracle_mstrsm(m, n, U, ld, lam, B, ld) == 0;
        FRESH(); calls += oracle_mstrsm_gen(m, n, U, ld, V, ld, lam, B, ld) == 0;
        FRESH(); calls += oracle_mstrsm_adjoint(m, n, U, ld, lam, B, ld) == 0;
        calls += oracle_mstrsm_real(m, n, Ur, ld, lr, Br, ld) == 0;
        const char* uplos = "UL"; const char* ops = "NTC";
        for (int u = 0; u < 2; ++u) for (int o = 0; o < 3; ++o) {
            FRESH(); calls += oracle_mstrsm_op(uplos[u], ops[o], m, n, U, ld, lam, B, ld) == 0;
        }
        const int nbs[] = {0, 1, 16, 64};
        const int oms[] = {8, 960};
        for (int q = 0; q < 4; ++q) for (int w = 0; w < 2; ++w) for (int f = 0; f < 2; ++f) for (int c = 0; c < 2; ++c) {
            const int nb = nbs[q];
            const int nblk = nb > 0 ? (m + nb - 1) / nb : m;
            double* tr = dalloc((size_t)(nblk > 0 ? nblk : 1) * (n ? n : 1) * 2);
            FRESH();
            calls += oracle_mstrsm_safe(m, n, U, ld, lam, B, ld, c ? cl : NULL, scale, klog, nb, oms[w], f,
                                        nb > 0 ? tr : NULL) == 0;
            free(tr);
            FRESH();
            calls += oracle_mstrsm_safe_gen(m, n, U, ld, V, ld, lam, B, ld, c ? cl : NULL, scale, klog,
                                            nb, oms[w], f) == 0;
        }
        free(U); free(V); free(Ur); free(lam); free(lr); free(B0); free(B); free(Br);
        free(scale); free(klog); free(cl);
    }
    printf("calls ok: %d\n", calls);
    return 0;
}
"""


def test_oracle_under_sanitizers(tmp_path):
    cc = shutil.which("gcc")
    if cc is None:
        pytest.skip("no gcc")
    src = tmp_path / "driver.c"
    src.write_text(DRIVER)
    exe = tmp_path / "driver"
    cmd = [cc, "-std=c11", "-O1", "-g", "-fno-omit-frame-pointer", "-fopenmp", "-fno-fast-math",
           "-ffp-contract=off", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           str(src), os.path.join(ROOT, "oracle", "mstrsm_oracle.c"), "-lm", "-o", str(exe)]
    p = subprocess.run(cmd, capture_output=True, text=True)
    if p.returncode != 0 and "sanitize" in p.stderr and "cannot find" in p.stderr:
        pytest.skip("sanitizer runtime not installed")
    assert p.returncode == 0, p.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0", UBSAN_OPTIONS="print_stacktrace=1",
               OMP_NUM_THREADS="2")
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=600, env=env)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-4000:])
    assert "calls ok" in r.stdout
