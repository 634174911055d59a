"""The C-ABI from plain C: include/mstrsm.h compiles as pedantic C99 and a C
program links against libmstrsm.so and gets argument errors back (no GPU call
is made: every call below fails its argument check first)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

PROGRAM = r"""
#include <stdio.h>
#include "mstrsm.h"

int main(void) {
    mst_opts o = {0};
    double d = 0.0;
    int fails = 0;
    /* m < 0 */
    if (mstrsm(-1, 2, 0, 1, 0, 0, 1, &o, 0) != MST_EARG || mst_last_bad_arg() != 1) fails |= 1;
    /* leading dimension of B below m */
    if (mstrsm_real(3, 2, &d, 3, &d, &d, 2, 0, 0) != MST_EARG || mst_last_bad_arg() != 7) fails |= 2;
    /* unknown side character */
    if (mstrsm_real_op('X', 'U', 'N', 3, 2, &d, 3, &d, &d, 3, 0, 0) != MST_EARG || mst_last_bad_arg() != 1)
        fails |= 4;
    /* empty problems return at once */
    if (mstrsm_real(0, 5, 0, 1, 0, 0, 1, 0, 0) != MST_OK) fails |= 8;
    printf("%s %d\n", mst_version(), fails);
    return fails;
}
"""


def test_header_is_c99_and_links(tmp_path):
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    lib_dir = os.path.join(ROOT, "paper_1607_01477_amd")
    if not os.path.exists(os.path.join(lib_dir, "libmstrsm.so")):
        pytest.skip("library not built")
    src = tmp_path / "abi.c"
    src.write_text(PROGRAM)
    exe = tmp_path / "abi"
    cmd = [cc, "-std=c99", "-Wall", "-Wextra", "-pedantic", "-Werror", "-I", os.path.join(ROOT, "include"),
           str(src), "-L", lib_dir, "-lmstrsm", "-Wl,-rpath," + lib_dir, "-o", str(exe)]
    p = subprocess.run(cmd, capture_output=True, text=True)
    assert p.returncode == 0, p.stderr
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, (r.stdout, r.stderr)
