"""Pins of the oracle's fine-grained parallel ILU (Chow and Patel's fixed-
point iteration, cited in the paper's introduction as a way to build the ILU
factors in parallel), synchronous form:
  * enough sweeps reproduce the (separately pinned) row-wise ILU(0) and
    ILU(k) bit for bit: both evaluate the same formula with the products
    subtracted in increasing k;
  * zero sweeps return the start l_ij = a_ij / a_jj, u_ij = a_ij;
  * on a tridiagonal matrix one sweep has a closed form, and the pivots
    become final one row per two sweeps (u_ii needs l_(i,i-1) of the
    previous sweep, which needs u_(i-1,i-1) of the one before): after s
    sweeps exactly rows 0 .. (s + 1) // 2 are final;
  * the fixed point satisfies (L U)_ij = a_ij on the pattern.
"""

import numpy as np
import pytest
import scipy.sparse as sp

import oracle
from workloads import Csr, convdiff2d_upwind, poisson2d, poisson3d, random_diag_dominant


def _same(X, Y):
    return (np.array_equal(X.rp, Y.rp) and np.array_equal(X.ci, Y.ci)
            and np.array_equal(X.v.view(np.uint64), Y.v.view(np.uint64)))


@pytest.mark.parametrize("maker", [lambda: poisson2d(8), lambda: convdiff2d_upwind(9, 10.0),
                                   lambda: random_diag_dominant(120, 6, band=20, seed=3), lambda: poisson3d(4)])
def test_converges_to_ilu0_bitwise(maker):
    A = maker()
    L, U = oracle.parilu(A, A.n)
    L0, U0 = oracle.ilu0(A)
    assert _same(L, L0) and _same(U, U0)


@pytest.mark.parametrize("level", [1, 2])
def test_converges_to_iluk_bitwise(level):
    A = random_diag_dominant(150, 6, band=25, seed=4)
    L, U = oracle.parilu(A, A.n, level=level)
    Lk, Uk = oracle.iluk(A, level)
    assert _same(L, Lk) and _same(U, Uk)


def test_zero_sweeps_is_the_start():
    A = random_diag_dominant(60, 5, band=10, seed=5)
    L, U = oracle.parilu(A, 0)
    Ad = A.to_scipy().toarray()
    d = np.diag(Ad)
    np.testing.assert_array_equal(U.to_scipy().toarray(), np.triu(Ad))
    np.testing.assert_array_equal(L.to_scipy().toarray(), np.tril(Ad, -1) / d[None, :] + np.eye(A.n))


def _tridiag(n, seed):
    rng = np.random.default_rng(seed)
    lo, up = rng.uniform(-1, 1, n - 1), rng.uniform(-1, 1, n - 1)
    dg = 3 + rng.uniform(0, 1, n)
    return Csr.from_scipy(sp.diags([lo, dg, up], [-1, 0, 1], format="csr")), lo, dg, up


def test_tridiagonal_one_sweep_closed_form():
    A, lo, dg, up = _tridiag(40, 6)
    L, U = oracle.parilu(A, 1)
    Ld, Ud = L.to_scipy().toarray(), U.to_scipy().toarray()
    want_u = dg.copy()
    want_u[1:] = dg[1:] - (lo / dg[:-1]) * up
    np.testing.assert_allclose(np.diag(Ud), want_u, rtol=1e-15)
    np.testing.assert_allclose(np.diag(Ud, 1), up, rtol=0)
    np.testing.assert_allclose(np.diag(Ld, -1), lo / dg[:-1], rtol=1e-15)


@pytest.mark.parametrize("s", [1, 2, 3, 4, 7])
def test_tridiagonal_rows_final_one_per_two_sweeps(s):
    A, *_ = _tridiag(30, 7)
    L, U = oracle.parilu(A, s)
    L0, U0 = oracle.ilu0(A)
    u, u0 = np.diag(U.to_scipy().toarray()), np.diag(U0.to_scipy().toarray())
    f = (s + 1) // 2
    assert np.array_equal(u[: f + 1], u0[: f + 1])
    assert u[f + 1] != u0[f + 1]


def test_fixed_point_reproduces_a_on_pattern():
    A = poisson3d(6)
    L, U = oracle.parilu(A, 200)
    P = (L.to_scipy() @ U.to_scipy()).tocsr()
    As = A.to_scipy().tocoo()
    np.testing.assert_allclose(np.asarray(P[As.row, As.col]).ravel(), As.data, atol=1e-13)


def test_zero_diagonal_rejected():
    A = Csr(2, np.array([0, 2, 4], np.int32), np.array([0, 1, 0, 1], np.int32), np.array([0.0, 1.0, 1.0, 2.0]))
    with pytest.raises(Exception):
        oracle.parilu(A, 2)


# ---- symmetric (incomplete Cholesky) form ------------------------------------

def _sym_rdd(n, seed):
    B = random_diag_dominant(n, 5, band=30, seed=seed).to_scipy()
    S = (B + B.T).tocsr()
    S.setdiag(np.abs(S).sum(axis=1).A1 + 1.0)
    S.sort_indices()
    return Csr.from_scipy(S)


@pytest.mark.parametrize("maker", [lambda: poisson3d(6), lambda: poisson2d(12), lambda: _sym_rdd(200, 3)])
def test_paric_converges_to_ilu0(maker):
    A = maker()
    L, U = oracle.paric(A, 200)
    L0, U0 = oracle.ilu0(A)
    assert np.array_equal(L.ci, L0.ci) and np.array_equal(U.ci, U0.ci)
    np.testing.assert_allclose(U.v, U0.v, rtol=1e-13, atol=1e-14 * np.abs(U0.v).max())
    np.testing.assert_allclose(L.v, L0.v, rtol=1e-13, atol=1e-14)


@pytest.mark.parametrize("s", [0, 1, 3])
def test_paric_symmetric_after_every_sweep(s):
    A = _sym_rdd(150, 4)
    L, U = oracle.paric(A, s)
    Ld, Ud = L.to_scipy().toarray(), U.to_scipy().toarray()
    d = np.diag(Ud)
    # l_ji = fl(u_ij / u_ii): the unit-lower factor is D^-1 U transposed
    np.testing.assert_allclose(Ld.T, np.triu(Ud, 1) / d[:, None] + np.eye(A.n), rtol=1e-15, atol=0)


def test_paric_zero_sweeps_and_tridiagonal_one_sweep():
    A, lo, dg, up = _tridiag(30, 8)
    Ad = A.to_scipy().toarray()
    S = np.triu(Ad) + np.triu(Ad, 1).T            # the symmetric matrix of A's upper triangle
    L, U = oracle.paric(Csr.from_scipy(sp.csr_matrix(S)), 0)
    np.testing.assert_array_equal(U.to_scipy().toarray(), np.triu(S))
    L1, U1 = oracle.paric(Csr.from_scipy(sp.csr_matrix(S)), 1)
    want = dg.copy()
    want[1:] = dg[1:] - (up / dg[:-1]) * up       # u_ii = a_ii - (u_(i-1,i) / u_(i-1,i-1)) u_(i-1,i)
    np.testing.assert_allclose(np.diag(U1.to_scipy().toarray()), want, rtol=1e-15)


def test_paric_gives_symmetric_sait_preconditioner():
    # with the upper factor right-multiplied, the SAIT pair of the symmetric
    # factors is symmetric up to rounding even after a single sweep
    A = poisson3d(7)
    L, U = oracle.paric(A, 1)
    ML, MU = oracle.sait_factors(L, U, 4, tau=0.02)
    P = (MU.to_scipy() @ ML.to_scipy()).toarray()
    assert np.abs(P - P.T).max() <= 1e-13 * np.abs(P).max()
    assert np.linalg.eigvalsh(0.5 * (P + P.T)).min() > 0
