"""GPU parity: the HIP library (through its C-ABI) against the CPU oracle.

Bars (floating point, FP64):
  * backward error: per column ||(U - l_j I) x_j - s_j b_j||_inf /
    (||U - l_j I||_inf ||x_j||_inf) <= 1e-13 (true modulus);
  * forward agreement with the oracle: ||x_gpu - x_or||_inf / ||x_or||_inf
    <= 64 eps kappa_inf(U - l_j I), i.e. what two backward-stable solves
    with different rounding order may differ by;
  * safe solve: scale exponents equal to the oracle's Alg 5 with the same nb
    (a mismatch is allowed only where the deciding quantity sits within
    1e-12 of a power of two -- none occurred in these cases), and dyadic
    problems, whose arithmetic is exact, bit for bit.
"""
import numpy as np
import pytest

import workloads as W
from gpu_util import announce, colerr, dev, host

pytestmark = pytest.mark.gpu

EPS = 2.0 ** -52


@pytest.fixture(scope="module")
def P():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1607_01477_amd as P
    P._lib.load()
    return P


def kappa_cols(U, lam, cols):
    Ut = np.triu(U)
    m = U.shape[0]
    out = []
    for j in cols:
        A = Ut - lam[j] * np.eye(m)
        out.append(np.linalg.norm(A, np.inf) * np.linalg.norm(np.linalg.inv(A), np.inf))
    return np.array(out)


def check_plain(oracle_mod, U, lam, B, X, cols=None, resid_tol=1e-13):
    m, n = B.shape
    if cols is None:
        cols = np.arange(n)
    cols = np.asarray(cols)
    Xo = oracle_mod.solve(U, lam[cols], B[:, cols])
    rr = oracle_mod.relative_residual(U, lam, X, B, cols=cols)
    assert rr.max() <= resid_tol, rr.max()
    kap = kappa_cols(U, lam, cols[: min(len(cols), 64)]) if m <= 700 else None
    err = colerr(X[:, cols], Xo)
    if kap is not None:
        k = len(kap)
        assert np.all(err[:k] <= 64 * EPS * kap), (err[:k] / (EPS * kap)).max()
    else:
        assert err.max() <= 1e-9, err.max()
    return err


# ------------------------------------------------------------------ plain

@pytest.mark.parametrize("m,n", [(1, 1), (2, 3), (7, 5), (63, 17), (64, 64), (65, 70), (200, 33),
                                 (257, 130), (600, 96)])
@pytest.mark.parametrize("nb,outer", [(64, 256), (64, 64), (32, 128), (16, 16)])
def test_plain_shapes(P, oracle_mod, m, n, nb, outer):
    announce("plain m=%d n=%d nb=%d outer=%d" % (m, n, nb, outer))
    w = W.c1_plain(seed=100 + m + n, m=m, n=n)
    X = host(P.mstrsm(dev(w.U), dev(w.shifts), dev(w.B), nb=nb, outer_nb=outer))
    check_plain(oracle_mod, w.U, w.shifts, w.B, X)


def test_plain_c1_config(P, oracle_mod):
    w = W.c1_plain()
    announce("c1 plain 256x256")
    X = host(P.mstrsm(dev(w.U), dev(w.shifts), dev(w.B)))
    check_plain(oracle_mod, w.U, w.shifts, w.B, X)


def test_plain_lower_triangle_and_padding_untouched(P, oracle_mod):
    import torch
    w = W.c1_plain(seed=7, m=150, n=40)
    m, n = 150, 40
    Ug = w.U.copy(order="F")
    Ug[np.tril_indices(m, -1)] = np.nan
    # B with leading dimension 160: rows 150..159 are padding
    Bpad = np.full((160, n), 7.0 + 3.0j, dtype=np.complex128, order="F")
    Bpad[:m] = w.B
    Bd = dev(Bpad)
    Ud = dev(Ug)
    announce("plain NaN lower triangle / padded ld")
    Xv = P.mstrsm(Ud, dev(w.shifts), Bd[:m])
    assert Xv.data_ptr() == Bd.data_ptr()
    out = host(Bd)
    assert np.all(out[m:] == 7.0 + 3.0j)
    check_plain(oracle_mod, w.U, w.shifts, w.B, out[:m])
    assert np.all(np.isnan(host(Ud)[np.tril_indices(m, -1)]))


def test_plain_full_size_sampled(P, oracle_mod):
    # the benchmark configuration, m = n = 4096, in the launch configuration bench.py times
    w = W.c3_mixed()
    announce("c3 plain 4096x4096 (sampled columns)")
    X = host(P.mstrsm(dev(w.U), dev(w.shifts), dev(w.B)))
    assert np.all(np.isfinite(X))
    cols = np.sort(W.rng(333).choice(w.n, 24, replace=False))
    cols = np.unique(np.concatenate([cols, [0, w.n - 1]]))
    err = check_plain(oracle_mod, w.U, w.shifts, w.B, X, cols=cols)
    assert err.max() <= 1e-12


def test_plain_deterministic(P):
    w = W.c1_plain(seed=9, m=300, n=100)
    a = host(P.mstrsm(dev(w.U), dev(w.shifts), dev(w.B)))
    b = host(P.mstrsm(dev(w.U), dev(w.shifts), dev(w.B)))
    assert np.array_equal(a, b)


# ------------------------------------------------------------------ adjoint

@pytest.mark.parametrize("m,n", [(1, 2), (65, 9), (200, 64), (513, 40)])
@pytest.mark.parametrize("nb,outer", [(64, 256), (32, 32), (16, 64)])
def test_adjoint_shapes(P, oracle_mod, m, n, nb, outer):
    announce("adjoint m=%d n=%d nb=%d" % (m, n, nb))
    w = W.c1_plain(seed=200 + m, m=m, n=n)
    Y = host(P.mstrsm_adjoint(dev(w.U), dev(w.shifts), dev(w.B), nb=nb, outer_nb=outer))
    Yo = oracle_mod.solve_adjoint(w.U, w.shifts, w.B)
    # adjoint residual
    Ut = np.triu(w.U)
    for j in range(n):
        A = (Ut - w.shifts[j] * np.eye(m)).conj().T
        r = np.abs(A @ Y[:, j] - w.B[:, j]).max()
        assert r <= 1e-13 * np.abs(A).sum(1).max() * np.abs(Y[:, j]).max()
    kap = kappa_cols(w.U, w.shifts, range(min(n, 16)))
    err = colerr(Y[:, :len(kap)], Yo[:, :len(kap)])
    assert np.all(err <= 64 * EPS * kap)


# ------------------------------------------------------------------ safe

def _growth(seed, m, n):
    g = W.rng(seed)
    U = W.random_upper(g, m, 1.0, W.cnormal(g, m))
    lam = W.cnormal(g, n)
    B = np.asfortranarray(W.cnormal(g, (m, n)))
    return U, lam, B


def _check_safe(oracle_mod, U, lam, B, X, s, k, nb, omega_log2, col_len=None):
    Xo, so, ko = oracle_mod.solve_safe(U, lam, B, col_len=col_len, nb=nb, omega_log2=omega_log2)
    assert np.array_equal(k, ko), np.nonzero(k != ko)
    assert np.array_equal(s, so)
    assert np.all(np.isfinite(X))
    m, n = B.shape
    if col_len is None:
        rr = oracle_mod.relative_residual(U, lam, X, B, k=k)
        assert rr.max() <= 1e-13, rr.max()
    err = colerr(X, Xo)
    return err


@pytest.mark.parametrize("nb", [64, 32, 16])
@pytest.mark.parametrize("omega_log2", [960, 60, 24])
def test_safe_growth(P, oracle_mod, nb, omega_log2):
    announce("safe growth nb=%d omega=2^%d" % (nb, omega_log2))
    U, lam, B = _growth(300 + nb, 333, 70)
    X, s, k = P.mstrsm_safe(dev(U), dev(lam), dev(B), nb=nb, omega_log2=omega_log2)
    X, s, k = host(X), host(s), host(k)
    err = _check_safe(oracle_mod, U, lam, B, X, s, k, nb, omega_log2)
    if omega_log2 < 100:
        assert np.any(k > 0)
    assert err.max() <= 1e-6   # growth problem: kappa large; residual bar above is the tight one


@pytest.mark.parametrize("outer", [64, 128, 256])
def test_safe_outer_block_invariance(P, oracle_mod, outer):
    # deferring the substitution over several diagonal blocks must not change any decision
    U, lam, B = _growth(31, 400, 50)
    X, s, k = P.mstrsm_safe(dev(U), dev(lam), dev(B), nb=32, outer_nb=outer, omega_log2=40)
    _check_safe(oracle_mod, U, lam, B, host(X), host(s), host(k), 32, 40)


def test_safe_well_conditioned_equals_plain(P, oracle_mod):
    w = W.c1_plain(seed=5, m=300, n=64)
    Xs, s, k = P.mstrsm_safe(dev(w.U), dev(w.shifts), dev(w.B))
    Xp = P.mstrsm(dev(w.U), dev(w.shifts), dev(w.B))
    assert np.all(host(k) == 0) and np.all(host(s) == 1.0)
    check_plain(oracle_mod, w.U, w.shifts, w.B, host(Xs))
    np.testing.assert_allclose(host(Xs), host(Xp), rtol=0, atol=1e-13 * np.abs(host(Xp)).max())


@pytest.mark.parametrize("nb", [64, 16])
@pytest.mark.parametrize("omega_log2", [8, 12, 960])
def test_safe_dyadic_bit_exact(P, oracle_mod, nb, omega_log2):
    # exact arithmetic on both sides: X and k must agree bit for bit
    from test_oracle_safe import _dyadic_problem
    U, lam, B = _dyadic_problem(40 + omega_log2, 20, 9)
    X, s, k = P.mstrsm_safe(dev(U), dev(lam), dev(B), nb=nb, omega_log2=omega_log2)
    Xo, so, ko = oracle_mod.solve_safe(U, lam, B, nb=nb, omega_log2=omega_log2)
    assert np.array_equal(host(k), ko)
    assert np.array_equal(host(X), Xo)


def test_safe_golden_examples(P):
    import json
    import os
    from test_oracle_safe import _golden_inputs
    with open(os.path.join(os.path.dirname(__file__), "golden", "safe_scaling_examples.json")) as f:
        cases = json.load(f)["cases"]
    for case in cases:
        U, lam, b = _golden_inputs(case)
        for nb in (16, 32, 64):
            X, s, k = P.mstrsm_safe(dev(U), dev(lam), dev(b), nb=nb)
            X, k = host(X), host(k)
            assert int(k[0]) == case["k"], (case["name"], nb)
            if "log2_abs_x" in case:
                exp = np.array([sg * 2.0 ** e for e, sg in zip(case["log2_abs_x"], case["x_sign"])])
                assert np.array_equal(X[:, 0], exp.astype(np.complex128)), case["name"]


def _bits(X):
    return np.ascontiguousarray(X).view(np.uint64)


@pytest.mark.parametrize("nb,fuse", [(16, True), (32, True), (16, False), (64, False)])
def test_force_phase2_bit_identical(P, oracle_mod, nb, fuse):
    """force_phase2 = 1 skips the speculative pass of the safe diagonal blocks
    (every block runs the checked steps of Alg 4's phase 2); the default runs
    the speculative pass and redoes a block with the checked steps only when a
    check fires. Both must give the same X, scales and exponents bit for bit:
    on inputs where nothing rescales (checked steps never taken by default)
    and on growth problems that rescale, with and without variable row counts.
    Fused outer blocks (nb 16, 32) and the per-block kernel (nb 16, 64)."""
    import torch
    w = W.c3_mixed(seed=71, m=700, n=150)
    announce("force_phase2 nb=%d fuse=%s: no rescaling" % (nb, fuse))
    a = [host(t) for t in P.mstrsm_safe(dev(w.U), dev(w.shifts), dev(w.B), nb=nb, fuse=fuse)]
    b = [host(t) for t in P.mstrsm_safe(dev(w.U), dev(w.shifts), dev(w.B), nb=nb, fuse=fuse,
                                        force_phase2=True)]
    assert np.all(a[2] == 0)
    assert np.array_equal(_bits(a[0]), _bits(b[0])) and np.array_equal(a[1], b[1]) and np.array_equal(a[2], b[2])
    U, lam, B = _growth(72 + nb, 600, 80)
    L = W.rng(720 + nb).integers(0, 601, 80).astype(np.int32)
    for cl in (None, L):
        announce("force_phase2 nb=%d fuse=%s: growth, col_len=%s" % (nb, fuse, cl is not None))
        cld = dev(cl, dtype=torch.int32) if cl is not None else None
        a = [host(t) for t in P.mstrsm_safe(dev(U), dev(lam), dev(B), cld, nb=nb, fuse=fuse,
                                            omega_log2=40)]
        b = [host(t) for t in P.mstrsm_safe(dev(U), dev(lam), dev(B), cld, nb=nb, fuse=fuse,
                                            omega_log2=40, force_phase2=True)]
        assert np.any(a[2] > 0)
        assert np.array_equal(_bits(a[0]), _bits(b[0]))
        assert np.array_equal(a[1], b[1]) and np.array_equal(a[2], b[2])
        Xo, so, ko = oracle_mod.solve_safe(U, lam, B, col_len=cl, nb=nb, omega_log2=40, force_phase2=True)
        assert np.array_equal(b[2], ko)


def test_force_phase2_triang_eig(P):
    """TriangEig (Alg 6) on the c2 recipe at m = 600 with Omega = 2^200 (183
    rescaled columns in the oracle, exact eigenvalue repeats): forced checked
    steps equal the default bit for bit."""
    w = W.c2_triang_eig(m=600)
    announce("force_phase2 triang_eig m=600")
    e0, Z0, k0 = (host(t) for t in P.triang_eig(dev(w.U), omega_log2=200))
    e1, Z1, k1 = (host(t) for t in P.triang_eig(dev(w.U), omega_log2=200, force_phase2=True))
    assert np.any(k0 > 0)
    assert np.array_equal(_bits(Z0), _bits(Z1)) and np.array_equal(k0, k1)


def test_safe_col_len(P, oracle_mod):
    U, lam, B = _growth(41, 260, 64)
    L = W.rng(410).integers(0, 261, 64).astype(np.int32)
    L[:4] = [0, 260, 64, 1]
    Bd = dev(B)
    X, s, k = P.mstrsm_safe(dev(U), dev(lam), Bd, col_len=dev(L, dtype=__import__("torch").int32),
                            nb=32, omega_log2=50)
    X, s, k = host(X), host(s), host(k)
    Xo, so, ko = oracle_mod.solve_safe(U, lam, B, col_len=L, nb=32, omega_log2=50)
    assert np.array_equal(k, ko)
    for j in range(64):
        assert np.array_equal(X[L[j]:, j], B[L[j]:, j])   # untouched
        if L[j] > 0:
            e = np.abs(X[:L[j], j] - Xo[:L[j], j]).max() / max(np.abs(Xo[:L[j], j]).max(), 1e-300)
            assert e <= 1e-8


def test_triang_eig_c2_config(P, oracle_mod):
    w = W.c2_triang_eig()
    announce("c2 triangular eigenvectors 2048")
    ev, Z, k = P.triang_eig(dev(w.U), nb=64)
    ev, Z, k = host(ev), host(Z), host(k)
    lo, Zo, ko = oracle_mod.triang_eig(w.U, nb=64)
    assert np.array_equal(ev, lo)
    mism = np.nonzero(k != ko)[0]
    assert len(mism) == 0, (mism[:10], k[mism[:10]], ko[mism[:10]])
    assert np.any(k > 0)
    assert np.all(np.isfinite(Z))
    assert np.all(np.tril(Z, -1) == 0)
    # eigen-relation on every column (sampled rows of the product would hide errors)
    T = w.U
    Tn = np.max(np.sum(np.abs(T), axis=1))
    R = T @ Z - Z * ev[None, :]
    rel = np.max(np.abs(R), axis=0) / (Tn * np.max(np.abs(Z), axis=0))
    assert rel.max() <= 1e-13, rel.max()


# ------------------------------------------------------------------ gradient, residual

def test_grad_pieces(P, oracle_mod):
    w = W.c5_adjoint(m=300, n=90)
    X = oracle_mod.solve(w.U, w.shifts, w.B)
    G = 2.0 * w.extra["W"] * X
    Y = oracle_mod.solve_adjoint(w.U, w.shifts, G)
    gU, gl, gB = oracle_mod.gradient(w.U, w.shifts, X, Y)
    gUd = host(P.grad_u(dev(Y), dev(X)))
    gld = host(P.grad_shift(dev(X), dev(Y)))
    np.testing.assert_allclose(gUd, gU, rtol=0, atol=1e-12 * np.abs(gU).max())
    assert np.all(np.tril(gUd, -1) == 0)
    np.testing.assert_allclose(gld, gl, rtol=1e-12, atol=1e-12 * np.abs(gl).max())


def test_autograd_matches_oracle_gradient(P, oracle_mod):
    import torch
    w = W.c5_adjoint(m=256, n=64)
    U = dev(w.U).requires_grad_(True)
    s = dev(w.shifts).requires_grad_(True)
    B = dev(w.B).requires_grad_(True)
    Wt = torch.from_numpy(w.extra["W"]).cuda()
    X = P.solve(U, s, B)
    loss = (Wt * X.abs() ** 2).sum()
    loss.backward()
    Xo = oracle_mod.solve(w.U, w.shifts, w.B)
    Yo = oracle_mod.solve_adjoint(w.U, w.shifts, 2.0 * w.extra["W"] * Xo)
    gU, gl, gB = oracle_mod.gradient(w.U, w.shifts, Xo, Yo)
    np.testing.assert_allclose(host(B.grad), gB, rtol=0, atol=1e-11 * np.abs(gB).max())
    np.testing.assert_allclose(host(s.grad), gl, rtol=0, atol=1e-11 * np.abs(gl).max())
    np.testing.assert_allclose(host(U.grad), gU, rtol=0, atol=1e-11 * np.abs(gU).max())


@pytest.mark.parametrize("chunk", [7, 64, 1000])
def test_autograd_recompute_matches(P, oracle_mod, chunk):
    # X recomputed in the backward pass, chunk columns at a time: the same
    # gradients (gB, gshift column by column bit for bit; gU summed over chunks)
    import torch
    w = W.c5_adjoint(m=300, n=130)
    Wt = torch.from_numpy(w.extra["W"]).cuda()
    grads = []
    for rc in (0, chunk):
        U = dev(w.U).requires_grad_(True)
        s = dev(w.shifts).requires_grad_(True)
        B = dev(w.B).requires_grad_(True)
        X = P.solve(U, s, B, recompute=rc)
        (Wt * X.abs() ** 2).sum().backward()
        grads.append((host(U.grad), host(s.grad), host(B.grad)))
    (gU0, gs0, gB0), (gU1, gs1, gB1) = grads
    assert np.array_equal(gB0, gB1) and np.array_equal(gs0, gs1)
    np.testing.assert_allclose(gU1, gU0, rtol=0, atol=1e-13 * np.abs(gU0).max())
    assert np.all(np.tril(gU1, -1) == 0)


def test_autograd_finite_differences(P):
    import torch
    w = W.c5_adjoint(m=40, n=7)
    Wt = torch.from_numpy(w.extra["W"]).cuda()

    def loss(U, s, B):
        return (Wt * P.solve(U, s, B).abs() ** 2).sum()

    U = dev(w.U).requires_grad_(True)
    s = dev(w.shifts).requires_grad_(True)
    B = dev(w.B).requires_grad_(True)
    loss(U, s, B).backward()
    h = 1e-6
    g = W.rng(77)
    for _ in range(12):
        r, c = sorted(g.integers(0, 40, 2))
        for d in (1.0, 1j):
            Up = dev(w.U); Up[r, c] += h * d
            Um = dev(w.U); Um[r, c] -= h * d
            fd = (loss(Up, dev(w.shifts), dev(w.B)) - loss(Um, dev(w.shifts), dev(w.B))).item() / (2 * h)
            an = (U.grad[r, c].conj() * d).real.item()
            assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)), (r, c, fd, an)
    for j in range(7):
        for d in (1.0, 1j):
            sp = dev(w.shifts); sp[j] += h * d
            sm = dev(w.shifts); sm[j] -= h * d
            fd = (loss(dev(w.U), sp, dev(w.B)) - loss(dev(w.U), sm, dev(w.B))).item() / (2 * h)
            an = (s.grad[j].conj() * d).real.item()
            assert abs(fd - an) <= 1e-6 * max(1.0, abs(an))


@pytest.mark.parametrize("m,n", [(1, 1), (5, 3), (64, 130), (333, 77), (600, 33)])
def test_residual_kernel(P, m, n):
    """B0 - (U X - X diag(lam)) on the barrier-free MFMA GEMM (triangular K
    range per wavefront); U's strict lower triangle holds NaN and must never
    be read."""
    w = W.c1_plain(seed=12 + m, m=m, n=n)
    X = np.asfortranarray(W.cnormal(W.rng(1 + m), (m, n)))
    Un = w.U.copy()
    Un[np.tril_indices(m, -1)] = np.nan
    R = host(P.residual(dev(Un), dev(w.shifts), dev(X), dev(w.B)))
    ref = w.B - (np.triu(w.U) @ X - X * w.shifts[None, :])
    assert np.all(np.isfinite(R))
    np.testing.assert_allclose(R, ref, rtol=0, atol=1e-13 * max(1.0, np.abs(ref).max()) * max(1, m) ** 0.5)


# ------------------------------------------------------------------ mixed precision

@pytest.mark.parametrize("sweeps", [1, 2, 3])
def test_mixed_precision_refinement(P, oracle_mod, sweeps):
    w = W.c3_mixed(m=700, n=150)
    announce("mixed m=700 sweeps=%d" % sweeps)
    X = host(P.mstrsm(dev(w.U), dev(w.shifts), dev(w.B), precision=1, max_sweeps=sweeps))
    Xo = oracle_mod.solve(w.U, w.shifts, w.B)
    fe = np.linalg.norm(X - Xo) / np.linalg.norm(Xo)
    rr = oracle_mod.relative_residual(w.U, w.shifts, X, w.B)
    print("sweeps", sweeps, "forward error", fe, "max residual", rr.max())
    if sweeps >= 2:
        assert rr.max() <= 1e-13
        assert fe <= 1e-13
    else:
        assert fe <= 1e-8


# ------------------------------------------------------------------ pseudospectra

def test_lanczos_small(P, oracle_mod):
    w = W.c4_pseudospectra(m=150, grid=6)
    sig, a, b, st = P.lanczos_sigma_min(dev(w.U), dev(w.shifts), dev(w.B), iters=15)
    so, ao, bo, sto = oracle_mod.lanczos_sigma_min(w.U, w.shifts, w.B, iters=15)
    np.testing.assert_allclose(host(sig), so, rtol=1e-8)
    np.testing.assert_allclose(host(a)[:, 0], ao[0], rtol=1e-12)


def test_lanczos_c4_config_sampled(P, oracle_mod):
    w = W.c4_pseudospectra()
    announce("c4 pseudospectra 2000 x 10000 shifts")
    sig, a, b, st = P.lanczos_sigma_min(dev(w.U), dev(w.shifts), dev(w.B), iters=15)
    sig = host(sig)
    cols = np.arange(0, w.n, 100)
    so, ao, bo, sto = oracle_mod.lanczos_sigma_min(w.U, w.shifts[cols], w.B[:, cols], iters=15)
    np.testing.assert_allclose(sig[cols], so, rtol=1e-8)
    assert np.all(np.isfinite(sig)) and np.all(sig > 0)


# ------------------------------------------------------------------ ABI errors

def test_abi_errors(P):
    import ctypes
    lib = P._lib.load()
    o = P._opts()
    assert lib.mstrsm(-1, 1, None, 1, None, None, 1, None, None) == P._lib.MST_EARG
    assert lib.mst_last_bad_arg() == 1
    assert lib.mstrsm(4, 2, None, 4, None, None, 4, None, None) == P._lib.MST_EARG
    assert lib.mst_last_bad_arg() == 3
    assert lib.mstrsm(0, 5, None, 1, None, None, 1, None, None) == 0
    assert lib.mstrsm(5, 0, None, 5, None, None, 5, None, None) == 0
    bad = P._opts(nb=48)
    x = dev(np.zeros((4, 4), complex))
    assert lib.mstrsm(4, 4, P._p(x), 4, P._p(x), P._p(x), 4, ctypes.byref(bad), None) == P._lib.MST_EARG
    assert lib.mst_last_bad_arg() == 8
    assert lib.mstrsm(4, 4, P._p(x), 3, P._p(x), P._p(x), 4, ctypes.byref(o), None) == P._lib.MST_EARG
    assert lib.mst_last_bad_arg() == 4
    mixed = P._opts(precision=1)
    sc = dev(np.zeros(4), dtype=__import__("torch").float64)
    assert lib.mstrsm_safe(4, 4, P._p(x), 4, P._p(x), P._p(x), 4, None, P._p(sc), None,
                           ctypes.byref(mixed), None) == P._lib.MST_EUNSUPPORTED


# ------------------------------------------------------------------ fused vs per-block paths

@pytest.mark.parametrize("nb,outer", [(64, 256), (32, 96), (16, 64)])
def test_unfused_and_fused_agree(P, oracle_mod, nb, outer):
    """One launch per diagonal block plus separate GEMMs (the paper's loop
    order) and the fused outer-block kernel solve the same systems."""
    w = W.c1_plain(seed=55 + nb, m=333, n=70)
    Xf = host(P.mstrsm(dev(w.U), dev(w.shifts), dev(w.B), nb=nb, outer_nb=outer))
    Xu = host(P.mstrsm(dev(w.U), dev(w.shifts), dev(w.B), nb=nb, outer_nb=outer, fuse=False))
    check_plain(oracle_mod, w.U, w.shifts, w.B, Xf)
    check_plain(oracle_mod, w.U, w.shifts, w.B, Xu)
    Yf = host(P.mstrsm_adjoint(dev(w.U), dev(w.shifts), dev(w.B), nb=nb, outer_nb=outer))
    Yu = host(P.mstrsm_adjoint(dev(w.U), dev(w.shifts), dev(w.B), nb=nb, outer_nb=outer, fuse=False))
    Yo = oracle_mod.solve_adjoint(w.U, w.shifts, w.B)
    assert colerr(Yf, Yo).max() <= 1e-10 and colerr(Yu, Yo).max() <= 1e-10
    U, lam, B = _growth(77, 300, 40)
    for fuse in (True, False):
        X, s, k = P.mstrsm_safe(dev(U), dev(lam), dev(B), nb=nb, outer_nb=outer, omega_log2=40,
                                fuse=fuse)
        _check_safe(oracle_mod, U, lam, B, host(X), host(s), host(k), nb, 40)


def test_large_outer_block_uses_per_block_path(P, oracle_mod):
    w = W.c1_plain(seed=58, m=700, n=50)
    X = host(P.mstrsm(dev(w.U), dev(w.shifts), dev(w.B), nb=64, outer_nb=512))
    check_plain(oracle_mod, w.U, w.shifts, w.B, X)


@pytest.mark.parametrize("safe", [False, True])
def test_staged_and_direct_gemm_agree(P, oracle_mod, safe):
    """LDS-staged and barrier-free substitution GEMMs solve the same systems."""
    if not safe:
        w = W.c1_plain(seed=59, m=530, n=140)
        for staged in (False, True):
            for fuse in (True, False):
                X = host(P.mstrsm(dev(w.U), dev(w.shifts), dev(w.B), nb=32, outer_nb=128,
                                  staged=staged, fuse=fuse))
                check_plain(oracle_mod, w.U, w.shifts, w.B, X)
            # mixed precision: FP32 substitution GEMM and FP64 residual on either kernel
            X = host(P.mstrsm(dev(w.U), dev(w.shifts), dev(w.B), nb=16, outer_nb=64, precision=1,
                              max_sweeps=2, staged=staged))
            check_plain(oracle_mod, w.U, w.shifts, w.B, X)
    else:
        U, lam, B = _growth(79, 450, 60)
        L = W.rng(790).integers(0, 451, 60).astype(np.int32)
        import torch
        for staged in (False, True):
            X, s, k = P.mstrsm_safe(dev(U), dev(lam), dev(B), nb=32, outer_nb=64, omega_log2=40,
                                    staged=staged)
            _check_safe(oracle_mod, U, lam, B, host(X), host(s), host(k), 32, 40)
            X, s, k = P.mstrsm_safe(dev(U), dev(lam), dev(B), col_len=dev(L, dtype=torch.int32),
                                    nb=32, outer_nb=64, omega_log2=40, staged=staged)
            Xo, so, ko = oracle_mod.solve_safe(U, lam, B, col_len=L, nb=32, omega_log2=40)
            assert np.array_equal(host(k), ko)


@pytest.mark.parametrize("nb,outer", [(16, 64), (32, 96), (64, 256)])
def test_lookahead_stream_matches(P, oracle_mod, nb, outer):
    """The two-stream lookahead (one substitution per outer block) and the
    one-stream loop (two-level deferral) solve the same systems: plain,
    mixed-precision and safe (variable-length) results match the oracle, and
    the safe exponents and scales of both equal the oracle's exactly."""
    import torch
    w = W.c1_plain(seed=61, m=1000 + nb // 2, n=150)
    for prec in (0, 1):
        X1 = host(P.mstrsm(dev(w.U), dev(w.shifts), dev(w.B), nb=nb, outer_nb=outer, precision=prec,
                           overlap=True))
        X0 = host(P.mstrsm(dev(w.U), dev(w.shifts), dev(w.B), nb=nb, outer_nb=outer, precision=prec))
        check_plain(oracle_mod, w.U, w.shifts, w.B, X1)
        check_plain(oracle_mod, w.U, w.shifts, w.B, X0)
    U, lam, B = _growth(81, 700, 50)
    L = W.rng(810).integers(0, 701, 50).astype(np.int32)
    r1 = P.mstrsm_safe(dev(U), dev(lam), dev(B), col_len=dev(L, dtype=torch.int32), nb=nb,
                       outer_nb=outer, omega_log2=40, overlap=True)
    r0 = P.mstrsm_safe(dev(U), dev(lam), dev(B), col_len=dev(L, dtype=torch.int32), nb=nb,
                       outer_nb=outer, omega_log2=40)
    assert np.array_equal(host(r1[1]), host(r0[1])) and np.array_equal(host(r1[2]), host(r0[2]))
    Xo, so, ko = oracle_mod.solve_safe(U, lam, B, col_len=L, nb=nb, omega_log2=40)
    assert np.array_equal(host(r1[2]), ko)
    for r in (r1, r0):
        assert colerr(host(r[0]), Xo).max() <= 1e-6   # growth problem: kappa large


@pytest.mark.parametrize("nb,outer,fuse", [(16, 64, True), (32, 96, True), (16, 48, False)])
def test_adjoint_direct_and_staged_gemm(P, oracle_mod, nb, outer, fuse):
    """The conjugate-transposed substitution GEMM of the adjoint solve: the
    barrier-free and the LDS-staged kernels both match the oracle (ragged m,
    several tiles)."""
    w = W.c1_plain(seed=63, m=530 + nb // 2, n=140)
    Yo = oracle_mod.solve_adjoint(w.U, w.shifts, w.B)
    for staged in (False, True):
        Y = host(P.mstrsm_adjoint(dev(w.U), dev(w.shifts), dev(w.B), nb=nb, outer_nb=outer, fuse=fuse,
                                  staged=staged))
        assert colerr(Y, Yo).max() <= 1e-10


@pytest.mark.parametrize("m,n", [(1, 1), (7, 3), (65, 70), (130, 5), (257, 33), (600, 130)])
def test_grad_u_shapes(P, oracle_mod, m, n):
    """-triu(Y X^H) on the barrier-free MFMA GEMM (zero tiles below the
    diagonal, ragged edges in M and K) against the oracle's gradient."""
    g = W.rng(900 + m)
    Y = W.cnormal(g, (m, n))
    X = W.cnormal(g, (m, n))
    gU, _, _ = oracle_mod.gradient(np.zeros((m, m), complex), np.zeros(n, complex), X, Y)
    gUd = host(P.grad_u(dev(Y), dev(X)))
    np.testing.assert_allclose(gUd, gU, rtol=0, atol=1e-13 * max(1.0, np.abs(gU).max()) * n)
    assert np.all(np.tril(gUd, -1) == 0)
