"""GPU parity of the lower-triangular, transposed and right-side variants
(footnote to Sec. 2) against the oracle: op(A - l_j I) x_j = b_j for A upper
or lower, op in {N, T, C}, and x_j^T op(A - l_j I) = b_j^T. Bars as for the
standard solves: relative residual <= 1e-13 (true modulus), forward agreement
with the oracle within 64 eps kappa_inf of the operator."""
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


def _problem(seed, m, n, uplo):
    w = W.c1_plain(seed=seed, m=m, n=n)
    A = w.U if uplo == "U" else np.asfortranarray(w.U.T.copy())
    return A, w.shifts, w.B


def _operator(A, lam, uplo, op):
    T = np.triu(A) if uplo == "U" else np.tril(A)
    E = T - lam * np.eye(A.shape[0])
    return {"N": E, "T": E.T, "C": E.conj().T}[op]


def _check(oracle_mod, A, lam, B, X, uplo, op):
    Xo = oracle_mod.solve_op(A, lam, B, uplo, op)
    err = colerr(X, Xo)
    n = B.shape[1]
    for j in range(n):
        E = _operator(A, lam[j], uplo, op)
        r = np.abs(E @ X[:, j] - B[:, j]).max()
        assert r <= 1e-13 * np.abs(E).sum(1).max() * np.abs(X[:, j]).max(), j
        if j < 16:
            kap = np.linalg.norm(E, np.inf) * np.linalg.norm(np.linalg.inv(E), np.inf)
            assert err[j] <= 64 * EPS * kap, (j, err[j] / (EPS * kap))


CASES = [(u, o) for u in "UL" for o in "NTC"]


@pytest.mark.parametrize("uplo,op", CASES)
@pytest.mark.parametrize("m,n", [(1, 2), (7, 5), (65, 33), (257, 70)])
@pytest.mark.parametrize("nb,outer,fuse", [(16, 64, True), (32, 96, True), (64, 128, False)])
def test_variant_shapes(P, oracle_mod, uplo, op, m, n, nb, outer, fuse):
    announce("variant %s%s m=%d n=%d nb=%d outer=%d fuse=%d" % (uplo, op, m, n, nb, outer, fuse))
    A, lam, B = _problem(500 + m + n + ord(uplo) + ord(op), m, n, uplo)
    # NaN in the triangle the variant must not read
    An = A.copy(order="F")
    if uplo == "U":
        An[np.tril_indices(m, -1)] = np.nan
    else:
        An[np.triu_indices(m, 1)] = np.nan
    X = host(P.mstrsm_op(dev(An), dev(lam), dev(B), uplo=uplo, op=op, nb=nb, outer_nb=outer, fuse=fuse))
    assert np.all(np.isfinite(X))
    _check(oracle_mod, A, lam, B, X, uplo, op)


@pytest.mark.parametrize("uplo,op", CASES)
def test_variant_default_config_600(P, oracle_mod, uplo, op):
    # default options (nb = 16, fused outer blocks of 256, the two-level deferral)
    A, lam, B = _problem(77, 600, 130, uplo)
    X = host(P.mstrsm_op(dev(A), dev(lam), dev(B), uplo=uplo, op=op))
    _check(oracle_mod, A, lam, B, X, uplo, op)


@pytest.mark.parametrize("uplo", "UL")
@pytest.mark.parametrize("op", "NT")
def test_right_side(P, oracle_mod, uplo, op):
    # x_j op(A - l_j I) = b_j  <=>  op(A - l_j I)^T x_j^T = b_j^T
    A, lam, B = _problem(78, 300, 40, uplo)
    X = host(P.mstrsm_op(dev(A), dev(lam), dev(B), uplo=uplo, op=op, side="R"))
    Xo = oracle_mod.solve_op(A, lam, B, uplo, "T" if op == "N" else "N")
    assert colerr(X, Xo).max() <= 1e-12
    for j in range(40):
        E = _operator(A, lam[j], uplo, op)
        r = np.abs(X[:, j] @ E - B[:, j]).max()
        assert r <= 1e-13 * np.abs(E).sum(0).max() * np.abs(X[:, j]).max()


def test_upper_n_is_mstrsm_and_upper_c_is_adjoint(P):
    A, lam, B = _problem(79, 333, 50, "U")
    a = host(P.mstrsm_op(dev(A), dev(lam), dev(B), uplo="U", op="N"))
    b = host(P.mstrsm(dev(A), dev(lam), dev(B)))
    assert np.array_equal(a, b)
    a = host(P.mstrsm_op(dev(A), dev(lam), dev(B), uplo="U", op="C"))
    b = host(P.mstrsm_adjoint(dev(A), dev(lam), dev(B)))
    assert np.array_equal(a, b)
