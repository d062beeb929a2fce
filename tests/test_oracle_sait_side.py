"""Pins of the oracle's right-multiplied Horner recursion W = M T~ + I, the
side it uses for the upper ILU factor (Sec. 2, Eq. Recursive; Sec. 4 for
why: its PCG needs a symmetric preconditioner).

What fixes it, independently of its own code:
  * an exact transposition identity with the (separately pinned)
    left-multiplied recursion: for an upper triangular U with d = diag(U),
    the unit lower triangular L' with L'_cl = fl(fl(1/d_l) U_lc) has
    T~(L') = T~(U)^T entry for entry, so the right recursion on U is the
    transpose of the left recursion on L', columns scaled by fl(1/d_c),
    bit for bit, under the threshold and the pattern rule alike;
  * without dropping, the series is the exact inverse (LAPACK);
  * one pass of M T~ + I from a given M, checked against dense products;
  * for a symmetric A (U = D L^T), M_U = M_L^T D^-1 up to rounding, so
    M_U M_L is symmetric positive definite;
  * the level-1 ratios and PCG iteration counts the paper prints
    (tests/test_oracle_iluk.py, tests/test_oracle_pcg.py).
"""

import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp

import oracle
from workloads import Csr, convdiff2d_upwind, poisson2d, poisson3d, random_diag_dominant, random_triangular


def _csr(M):
    M = sp.csr_matrix(M)
    M.sort_indices()
    return Csr(M.shape[0], M.indptr.astype(np.int32), M.indices.astype(np.int32), M.data.astype(np.float64))


def _mirror(U: Csr):
    """L' = I + strict lower part with L'_cl = fl(fl(1/d_l) * U_lc), and dinv."""
    Us = U.to_scipy().tocoo()
    d = U.to_scipy().diagonal()
    dinv = 1.0 / d
    off = Us.row != Us.col
    r, c, v = Us.row[off], Us.col[off], Us.data[off]
    vals = dinv[r] * v
    n = U.n
    Lp = sp.coo_matrix((np.concatenate([vals, np.ones(n)]), (np.concatenate([c, np.arange(n)]),
                                                              np.concatenate([r, np.arange(n)]))), shape=(n, n))
    return _csr(Lp), dinv


def _same(X: Csr, Y: Csr):
    return (np.array_equal(X.rp, Y.rp) and np.array_equal(X.ci, Y.ci)
            and np.array_equal(X.v.view(np.uint64), Y.v.view(np.uint64)))


def _upper_cases():
    yield "convdiff-ilu0", oracle.ilu0(convdiff2d_upwind(24, 10.0))[1]
    yield "rdd-ilu0", oracle.ilu0(random_diag_dominant(600, 8, band=80, seed=4))[1]
    yield "rdd-ilut", oracle.ilut(random_diag_dominant(500, 10, band=None, seed=5), 1e-3, 12)[1]
    yield "random-upper", random_triangular(300, 0.03, seed=7, lower=False)


@pytest.mark.parametrize("tau,m", [(0.0, 3), (1e-2, 4), (5e-2, 10), (1e-3, 2)])
def test_right_is_transposed_left_threshold(tau, m):
    for name, U in _upper_cases():
        Lp, dinv = _mirror(U)
        G = oracle.sait_thr(Lp, tau, m)                    # left recursion on L', d(L') = 1
        K = G.to_scipy().T.tocsr()
        K.sort_indices()
        K.data = K.data * dinv[K.indices]                  # M = K D^-1
        got = oracle.sait_thr(U, tau, m, side="right")
        assert _same(got, _csr(K)), name


@pytest.mark.parametrize("p,m", [(1, 3), (2, 5), (0, 2)])
def test_right_is_transposed_left_pattern(p, m):
    for name, U in _upper_cases():
        Lp, dinv = _mirror(U)
        K = oracle.sait_pat(Lp, p, m).to_scipy().T.tocsr()
        K.sort_indices()
        K.data = K.data * dinv[K.indices]
        assert _same(oracle.sait_pat(U, p, m, side="right"), _csr(K)), name


def test_no_dropping_gives_exact_inverse():
    for U in (random_triangular(120, 0.05, seed=9, lower=False), oracle.ilu0(poisson2d(9))[1]):
        Ud = U.to_scipy().toarray()
        Uinv = sla.solve_triangular(Ud, np.eye(U.n), lower=False)
        M = oracle.sait_thr(U, 0.0, U.n - 1, side="right").to_scipy().toarray()
        assert np.abs(M - Uinv).max() <= 1e-12 * np.abs(Uinv).max()


def test_one_pass_dense():
    # W = M T~ + I with T~ = I - D^-1 U, against dense products; then the mask.
    U = random_triangular(60, 0.1, seed=11, lower=False)
    Ud = U.to_scipy().toarray()
    d = np.diag(Ud)
    Tt = np.eye(60) - np.diag(1.0 / d) @ Ud
    M0 = oracle.sait_thr(U, 0.0, 2, side="right")      # some upper M, used as is
    W = M0.to_scipy().toarray() @ Tt + np.eye(60)
    for tau in (0.0, 0.05, 0.3):
        got = oracle.sait_step(U, M0, tau, side="right").to_scipy().toarray()
        want = np.where(np.abs(W) > tau, W, 0.0)
        np.fill_diagonal(want, np.diag(W))
        scale = max(1.0, np.abs(W).max())
        near = np.abs(np.abs(W) - tau) < 1e-12 * scale      # entries at the threshold may round either way
        assert np.all((np.abs(got - want) <= 1e-13 * scale) | near)


def test_left_and_right_differ_with_dropping():
    # the two sides are different recursions once entries are dropped
    U = oracle.ilu0(random_diag_dominant(600, 8, band=80, seed=4))[1]
    a = oracle.sait_thr(U, 1e-2, 4).to_scipy().toarray()
    b = oracle.sait_thr(U, 1e-2, 4, side="right").to_scipy().toarray()
    assert np.abs(a - b).max() > 1e-3


@pytest.mark.parametrize("level,tau", [(0, 2e-2), (1, 2e-2), (1, 5e-2)])
def test_symmetric_a_gives_transposed_lower(level, tau):
    A = poisson3d(12)
    L, U = oracle.ilu0(A) if level == 0 else oracle.iluk(A, level)
    ML, MU = oracle.sait_factors(L, U, 10, tau=tau)
    d = U.to_scipy().diagonal()
    X = (ML.to_scipy().T @ sp.diags(1.0 / d)).toarray()
    Y = MU.to_scipy().toarray()
    assert np.abs(X - Y).max() <= 1e-14 * np.abs(Y).max()
    P = (MU.to_scipy() @ ML.to_scipy()).toarray()
    assert np.abs(P - P.T).max() <= 1e-14 * np.abs(P).max()
    assert np.linalg.eigvalsh(0.5 * (P + P.T)).min() > 0


def test_bad_side_rejected():
    U = random_triangular(10, 0.2, seed=1, lower=False)
    with pytest.raises(ValueError):
        oracle.sait_thr(U, 0.1, 2, side="up")
