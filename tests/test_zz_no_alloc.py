"""The safe solve for callers that cannot allocate (mstrsm_safe_noalloc),
through the C-ABI: its workspace is the library's static scratch instead of
stream-ordered allocations, and its results must equal those of mstrsm_safe
(the same kernels) bit for bit, also on a call that follows a larger one and
so runs on the scratch contents that call left behind. Exponents are checked
against the oracle's Alg 5 as well. The call also replays inside a captured
HIP graph, which is what it is for."""
import numpy as np
import pytest

import workloads as W
from gpu_util import announce, dev, host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1607_01477_amd as P
    P._lib.load()
    return P


def _case(seed, m, n, varlen):
    g = W.rng(seed)
    U = W.random_upper(g, m, 1.0, W.cnormal(g, m))
    lam = W.cnormal(g, n)
    B = np.asfortranarray(W.cnormal(g, (m, n)))
    L = g.integers(0, m + 1, n).astype(np.int32) if varlen else None
    return U, lam, B, L


def _bits(X):
    return np.ascontiguousarray(X).view(np.uint64)


@pytest.mark.parametrize("nb", [16, 64])
def test_noalloc_equals_safe_on_consecutive_calls(P, oracle_mod, nb):
    import torch
    # the second and third calls are smaller than the first: they run on what
    # the earlier calls left in the scratch
    for seed, m, n, varlen in [(901, 2048, 512, False), (902, 1000, 300, True), (903, 300, 70, False)]:
        announce("noalloc vs safe nb=%d m=%d n=%d varlen=%s" % (nb, m, n, varlen))
        U, lam, B, L = _case(seed + nb, m, n, varlen)
        cl = dev(L, dtype=torch.int32) if L is not None else None
        Ud, ld = dev(U), dev(lam)
        X0, s0, k0 = P.mstrsm_safe(Ud, ld, dev(B), col_len=cl, nb=nb, omega_log2=40)
        X1, s1, k1 = P.mstrsm_safe_noalloc(Ud, ld, dev(B), col_len=cl, nb=nb, omega_log2=40)
        X0, s0, k0, X1, s1, k1 = (host(t) for t in (X0, s0, k0, X1, s1, k1))
        assert np.array_equal(k1, k0) and np.array_equal(s1, s0)
        assert np.array_equal(_bits(X1), _bits(X0))
        Xo, so, ko = oracle_mod.solve_safe(U, lam, B, col_len=L, nb=nb, omega_log2=40)
        assert np.array_equal(k1, ko) and np.any(ko > 0)
        if L is None:
            rr = oracle_mod.relative_residual(U, lam, X1, B, k=k1)
            assert rr.max() <= 1e-13, rr.max()


def test_noalloc_empty_and_benchmark_shape(P, oracle_mod):
    import torch
    announce("noalloc m=0 and the m=n=4096 nb=16 launch configuration (sampled columns)")
    # m = 0: s_j = 1, k_j = 0
    X, s, k = P.mstrsm_safe_noalloc(torch.zeros((0, 0), dtype=torch.complex128, device="cuda"),
                                    torch.ones(5, dtype=torch.complex128, device="cuda"),
                                    torch.zeros((0, 5), dtype=torch.complex128, device="cuda"))
    assert np.array_equal(host(s), np.ones(5)) and np.array_equal(host(k), np.zeros(5, np.int32))
    w = W.c3_mixed()
    Ud, ld = dev(w.U), dev(w.shifts)
    X0, s0, k0 = P.mstrsm_safe(Ud, ld, dev(w.B))
    X1, s1, k1 = P.mstrsm_safe_noalloc(Ud, ld, dev(w.B))
    assert np.array_equal(host(k1), host(k0)) and np.array_equal(host(s1), host(s0))
    assert torch.equal(torch.view_as_real(X1), torch.view_as_real(X0))
    cols = np.arange(0, w.n, 256)
    rr = oracle_mod.relative_residual(w.U, w.shifts[cols], host(X1)[:, cols], w.B[:, cols],
                                      k=host(k1)[cols])
    assert rr.max() <= 1e-13, rr.max()


def test_noalloc_replays_in_a_graph(P):
    import torch
    announce("noalloc in a captured graph m=700 n=130")
    U, lam, B, L = _case(905, 700, 130, True)
    Ud, ld, B0, cl = dev(U), dev(lam), dev(B), dev(L, dtype=torch.int32)
    scale = torch.empty(130, dtype=torch.float64, device="cuda")
    klog = torch.empty(130, dtype=torch.int32, device="cuda")
    Xe, se, ke = P.mstrsm_safe(Ud, ld, dev(B), col_len=cl, omega_log2=40)
    Xe, se, ke = host(Xe), host(se), host(ke)
    X = dev(B)

    def solve():
        X.copy_(B0)
        P.mstrsm_safe_noalloc(Ud, ld, X, col_len=cl, scale=scale, scale_log2=klog, omega_log2=40)

    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        solve()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        solve()
    U2, lam2, B2, _ = _case(906, 400, 50, False)
    for r in range(3):
        # another call on the same scratch between the replays
        P.mstrsm_safe_noalloc(dev(U2), dev(lam2), dev(B2), omega_log2=40)
        torch.cuda.synchronize()
        X.fill_(float("nan"))
        scale.fill_(-1.0)
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(_bits(host(X)), _bits(Xe)), r
        assert np.array_equal(host(scale), se) and np.array_equal(host(klog), ke), r
