"""CPU-side checks of the C-ABI library: it loads and exports every symbol the
public header declares (no compute calls: there is no GPU here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    with open(os.path.join(ROOT, "include", "mstrsm.h")) as f:
        src = f.read()
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\*?\s+\**(mst\w+)\s*\(", src, re.M)))


def test_header_declares_the_boundary():
    syms = declared_symbols()
    for s in ("mstrsm", "mstrsm_safe", "mstrsm_adjoint"):
        assert s in syms


def test_library_exports_every_declared_symbol():
    from paper_1607_01477_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_1607_01477_amd import build
        build.build()
    lib = ctypes.CDLL(_lib.LIB_PATH)
    for s in declared_symbols():
        assert hasattr(lib, s), s
    assert sorted(_lib.EXPORTS) == declared_symbols()
    lib.mst_version.restype = ctypes.c_char_p
    assert lib.mst_version().decode().count(".") == 2


def test_argument_errors_without_gpu():
    # validation happens on the host before any HIP call
    from paper_1607_01477_amd import _lib
    lib = _lib.load()
    assert lib.mstrsm(-1, 1, None, 1, None, None, 1, None, None) == _lib.MST_EARG
    assert lib.mst_last_bad_arg() == 1
    assert lib.mstrsm(3, 2, None, 3, None, None, 3, None, None) == _lib.MST_EARG
    assert lib.mst_last_bad_arg() == 3
    assert lib.mstrsm_adjoint(3, 2, None, 2, None, None, 3, None, None) == _lib.MST_EARG
    assert lib.mst_last_bad_arg() == 4
    assert lib.mstrsm(0, 7, None, 1, None, None, 1, None, None) == _lib.MST_OK
    assert lib.mst_status_string(_lib.MST_EARG).decode().startswith("MST_EARG")


def test_option_errors_without_gpu():
    # mst_opts.gemm_split must be 0, 1, 2 or 4 and refine_tol must not be NaN
    # (checked on the host)
    from paper_1607_01477_amd import _lib
    lib = _lib.load()
    for bad in (3, -1, 8):
        o = _lib.MstOpts()
        o.gemm_split = bad
        assert lib.mstrsm(0, 7, None, 1, None, None, 1, ctypes.byref(o), None) == _lib.MST_EARG
        assert lib.mst_last_bad_arg() == 8
    for good in (0, 1, 2, 4):
        o = _lib.MstOpts()
        o.gemm_split = good
        assert lib.mstrsm(0, 7, None, 1, None, None, 1, ctypes.byref(o), None) == _lib.MST_OK
    # fuse_blocks: -1 (per block), 0 (automatic width), 1 / 2 / 3 / 4 (16 / 4 / 2 / 1 shifts per workgroup)
    for fb, want in ((-2, _lib.MST_EARG), (5, _lib.MST_EARG), (-1, _lib.MST_OK), (0, _lib.MST_OK),
                     (1, _lib.MST_OK), (2, _lib.MST_OK), (3, _lib.MST_OK), (4, _lib.MST_OK)):
        o = _lib.MstOpts()
        o.fuse_blocks = fb
        assert lib.mstrsm(0, 7, None, 1, None, None, 1, ctypes.byref(o), None) == want
    o = _lib.MstOpts()
    o.refine_tol = float("nan")
    assert lib.mstrsm(0, 7, None, 1, None, None, 1, ctypes.byref(o), None) == _lib.MST_EARG
    o = _lib.MstOpts()
    o.refine_tol = -1.0
    o.max_sweeps = 3
    assert lib.mstrsm(0, 7, None, 1, None, None, 1, ctypes.byref(o), None) == _lib.MST_OK
    o.max_sweeps = 4
    assert lib.mstrsm(0, 7, None, 1, None, None, 1, ctypes.byref(o), None) == _lib.MST_EARG


def test_generalized_argument_errors_without_gpu():
    from paper_1607_01477_amd import _lib
    lib = _lib.load()
    fake = ctypes.c_void_p(4096)   # never dereferenced: the calls return before any HIP call
    # V missing / its leading dimension too small
    assert lib.mstrsm_gen(3, 2, fake, 3, None, 3, fake, fake, 3, None, None) == _lib.MST_EARG
    assert lib.mst_last_bad_arg() == 5
    assert lib.mstrsm_gen(3, 2, fake, 3, fake, 2, fake, fake, 3, None, None) == _lib.MST_EARG
    assert lib.mst_last_bad_arg() == 6
    assert lib.mstrsm_safe_gen(3, 2, fake, 3, fake, 3, fake, fake, 3, None, None, None, None,
                               None) == _lib.MST_EARG
    assert lib.mst_last_bad_arg() == 11
    assert lib.mst_gen_triang_eig(3, fake, 3, None, 3, fake, 3, fake, None, None, None) == _lib.MST_EARG
    assert lib.mst_last_bad_arg() == 4
    # only nb = 16 is supported for the pencil
    o = _lib.MstOpts()
    o.nb = 32
    assert lib.mstrsm_gen(3, 2, fake, 3, fake, 3, fake, fake, 3, ctypes.byref(o), None) == \
        _lib.MST_EUNSUPPORTED
    assert lib.mstrsm_gen(0, 5, None, 1, None, 1, None, None, 1, None, None) == _lib.MST_OK


def test_variant_argument_errors_without_gpu():
    from paper_1607_01477_amd import _lib
    lib = _lib.load()
    fake = ctypes.c_void_p(4096)
    assert lib.mstrsm_op(ord("X"), ord("U"), ord("N"), 3, 2, fake, 3, fake, fake, 3, None, None) == _lib.MST_EARG
    assert lib.mst_last_bad_arg() == 1
    assert lib.mstrsm_op(ord("L"), ord("Q"), ord("N"), 3, 2, fake, 3, fake, fake, 3, None, None) == _lib.MST_EARG
    assert lib.mst_last_bad_arg() == 2
    assert lib.mstrsm_op(ord("L"), ord("U"), ord("H"), 3, 2, fake, 3, fake, fake, 3, None, None) == _lib.MST_EARG
    assert lib.mst_last_bad_arg() == 3
    assert lib.mstrsm_op(ord("L"), ord("L"), ord("T"), 3, 2, fake, 2, fake, fake, 3, None, None) == _lib.MST_EARG
    assert lib.mst_last_bad_arg() == 7
    # right side with the conjugate transpose is not offered
    assert lib.mstrsm_op(ord("R"), ord("U"), ord("C"), 3, 2, fake, 3, fake, fake, 3, None, None) == \
        _lib.MST_EUNSUPPORTED
    o = _lib.MstOpts()
    o.precision = 1
    assert lib.mstrsm_op(ord("L"), ord("L"), ord("N"), 3, 2, fake, 3, fake, fake, 3, ctypes.byref(o), None) == \
        _lib.MST_EUNSUPPORTED


def test_real_argument_errors_without_gpu():
    from paper_1607_01477_amd import _lib
    lib = _lib.load()
    fake = ctypes.c_void_p(4096)
    assert lib.mstrsm_real(3, 2, None, 3, fake, fake, 3, None, None) == _lib.MST_EARG
    assert lib.mst_last_bad_arg() == 3
    o = _lib.MstOpts()
    o.outer_nb = 96
    assert lib.mstrsm_real(3, 2, fake, 3, fake, fake, 3, ctypes.byref(o), None) == _lib.MST_EARG
    assert lib.mst_last_bad_arg() == 8
    assert lib.mstrsm_real(0, 4, None, 1, None, None, 1, None, None) == _lib.MST_OK


def test_real_op_argument_errors_without_gpu():
    from paper_1607_01477_amd import _lib
    lib = _lib.load()
    fake = ctypes.c_void_p(4096)
    c = ord
    assert lib.mstrsm_real_op(c("X"), c("U"), c("N"), 3, 2, fake, 3, fake, fake, 3, None, None) == _lib.MST_EARG
    assert lib.mst_last_bad_arg() == 1
    assert lib.mstrsm_real_op(c("L"), c("Q"), c("N"), 3, 2, fake, 3, fake, fake, 3, None, None) == _lib.MST_EARG
    assert lib.mst_last_bad_arg() == 2
    assert lib.mstrsm_real_op(c("L"), c("L"), c("Z"), 3, 2, fake, 3, fake, fake, 3, None, None) == _lib.MST_EARG
    assert lib.mst_last_bad_arg() == 3
    assert lib.mstrsm_real_op(c("L"), c("L"), c("N"), 3, 2, fake, 2, fake, fake, 3, None, None) == _lib.MST_EARG
    assert lib.mst_last_bad_arg() == 7
    assert lib.mstrsm_real_op(c("L"), c("L"), c("N"), 3, 2, fake, 3, None, fake, 3, None, None) == _lib.MST_EARG
    assert lib.mst_last_bad_arg() == 8
    o = _lib.MstOpts()
    o.outer_nb = 96
    assert lib.mstrsm_real_op(c("R"), c("L"), c("T"), 3, 2, fake, 3, fake, fake, 3, ctypes.byref(o), None) == \
        _lib.MST_EARG
    assert lib.mst_last_bad_arg() == 11
    o = _lib.MstOpts()
    o.precision = 1
    assert lib.mstrsm_real_op(c("L"), c("L"), c("N"), 3, 2, fake, 3, fake, fake, 3, ctypes.byref(o), None) == \
        _lib.MST_EUNSUPPORTED
    assert lib.mstrsm_real_op(c("L"), c("L"), c("C"), 0, 4, None, 1, None, None, 1, None, None) == _lib.MST_OK


def test_log_env_reports_calls_and_errors():
    # MSTRSM_LOG: each call and each argument error on stderr (no GPU call is made)
    import os
    import subprocess
    import sys
    code = ("import ctypes\n"
            "from paper_1607_01477_amd import _lib\n"
            "lib = _lib.load()\n"
            "lib.mstrsm_real(0, 4, None, 1, None, None, 1, None, None)\n"
            "lib.mstrsm_real(-1, 4, None, 1, None, None, 1, None, None)\n"
            "o = _lib.MstOpts(); o.precision = 1\n"
            "rc = lib.mstrsm_real(0, 4, None, 1, None, None, 1, ctypes.byref(o), None)\n"
            "assert rc == _lib.MST_EUNSUPPORTED, rc\n"
            "assert b'precision 1' in lib.mst_last_error(), lib.mst_last_error()\n"
            "assert lib.mstrsm_real(0, 4, None, 1, None, None, 1, None, None) == 0\n"
            "assert lib.mst_last_error() == b'', lib.mst_last_error()\n")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    env = dict(os.environ, MSTRSM_LOG="1", PYTHONPATH=root)
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, env=env, timeout=120)
    assert r.returncode == 0, r.stderr
    assert "[mstrsm] mstrsm_real m=0 n=4" in r.stderr
    assert "[mstrsm] mstrsm_real: invalid argument 1" in r.stderr
    assert "[mstrsm] mstrsm_real: unsupported: precision 1" in r.stderr
    env["MSTRSM_LOG"] = "0"
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, env=env, timeout=120)
    assert "[mstrsm]" not in r.stderr


def test_noalloc_rejections_without_gpu():
    # mstrsm_safe_noalloc checks its arguments and the size of its static
    # scratch on the host, before any HIP call
    from paper_1607_01477_amd import _lib
    lib = _lib.load()
    fake = ctypes.c_void_p(4096)   # never dereferenced: the calls return before any HIP call
    f = lib.mstrsm_safe_noalloc
    assert f(-1, 2, fake, 3, fake, fake, 3, None, fake, None, None, None) == _lib.MST_EARG
    assert lib.mst_last_bad_arg() == 1
    assert f(3, 2, fake, 3, fake, fake, 3, None, None, None, None, None) == _lib.MST_EARG
    assert lib.mst_last_bad_arg() == 9
    o = _lib.MstOpts()
    o.overlap = 1
    assert f(3, 2, fake, 3, fake, fake, 3, None, fake, None, ctypes.byref(o), None) == _lib.MST_EUNSUPPORTED
    o = _lib.MstOpts()
    o.precision = 1
    assert f(3, 2, fake, 3, fake, fake, 3, None, fake, None, ctypes.byref(o), None) == _lib.MST_EUNSUPPORTED
    # m = n = 8192, nb = 16: the per-block exponent record alone is 512 x 8192 int32 = 16 MiB
    assert f(8192, 8192, fake, 8192, fake, fake, 8192, None, fake, None, None, None) == _lib.MST_ENOMEM
    msg = lib.mst_last_error().decode()
    assert "scratch" in msg and str(_lib.SCRATCH_LIMIT) in msg, msg
    # nb = 64 needs a quarter of that record and fits
    nb64 = 128 * 8192 * 4 + 2 * 8192 * 8 + 3 * 8192 * 8 + 256 * 3
    assert nb64 < _lib.SCRATCH_LIMIT
    assert f(5, 0, fake, 5, fake, fake, 5, None, fake, None, None, None) == _lib.MST_OK


def test_restarted_lanczos_argument_errors_without_gpu():
    from paper_1607_01477_amd import _lib
    lib = _lib.load()
    fake = ctypes.c_void_p(4096)   # never dereferenced: the calls return before any HIP call
    f = lib.mst_lanczos_restart_sigma_min
    args = lambda kdim, keep, mr, tol: (5, 3, fake, 5, fake, fake, 5, kdim, keep, mr, tol, fake, None, None,
                                        None, None, None)
    assert f(*args(1, 1, 0, 0.0)) == _lib.MST_EARG and lib.mst_last_bad_arg() == 8
    assert f(*args(33, 1, 0, 0.0)) == _lib.MST_EARG and lib.mst_last_bad_arg() == 8
    assert f(*args(8, 8, 0, 0.0)) == _lib.MST_EARG and lib.mst_last_bad_arg() == 9
    assert f(*args(32, 17, 0, 0.0)) == _lib.MST_EARG and lib.mst_last_bad_arg() == 9
    assert f(*args(8, 3, -1, 0.0)) == _lib.MST_EARG and lib.mst_last_bad_arg() == 10
    assert f(*args(8, 3, 0, float("nan"))) == _lib.MST_EARG and lib.mst_last_bad_arg() == 11
    assert f(*args(8, 3, 0, -1.0)) == _lib.MST_EARG and lib.mst_last_bad_arg() == 11
    assert f(5, 0, fake, 5, None, fake, 5, 8, 3, 0, 0.0, None, None, None, None, None, None) == _lib.MST_OK
