"""The plain solves inside a captured HIP graph (through torch.cuda.graph):
the library enqueues only kernels on the caller's stream (no allocation, no
memset, no synchronisation on these paths), so a captured solve replays. Each
replay runs after unrelated eager work and a synchronisation and must equal
the eager solve bit for bit."""
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


def _capture_and_replay(solve, B0, X, eager, other):
    import torch
    # warm-up on a side stream before capture
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        X.copy_(B0)
        solve(X)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        X.copy_(B0)
        solve(X)
    for r in range(3):
        other()
        torch.cuda.synchronize()
        X.fill_(float("nan"))
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(X.cpu().numpy(), eager), r


def test_complex_solve_replays(P):
    import torch
    announce("graph: complex plain solve m=700 n=130")
    w = W.c3_mixed(seed=51, m=700, n=130)
    U, lam, B0 = dev(w.U), dev(w.shifts), dev(w.B)
    eager = host(P.mstrsm(U, lam, dev(w.B)))
    X = dev(w.B)
    w2 = W.c1_plain(seed=52, m=300, n=40)
    _capture_and_replay(lambda x: P.mstrsm(U, lam, x), B0, X, eager,
                        lambda: P.mstrsm(dev(w2.U), dev(w2.shifts), dev(w2.B)))


def test_real_solve_replays(P):
    import torch
    announce("graph: real solve m=700 n=130")
    w = W.c10_real(seed=53, m=700, n=130)
    rd = lambda a: torch.from_numpy(np.asfortranarray(a)).cuda()
    U, lam, B0 = rd(w.U), rd(w.shifts), rd(w.B)
    eager = P.mstrsm_real(U, lam, rd(w.B)).cpu().numpy()
    X = rd(w.B)
    _capture_and_replay(lambda x: P.mstrsm_real(U, lam, x), B0, X, eager,
                        lambda: P.mstrsm_real(U, lam, rd(w.B)))
