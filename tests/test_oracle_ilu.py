"""Pins of the oracle's ILU(0), ILUT and exact substitution.

Each check ties the oracle to something other than itself: the LU
factorisation computed by LAPACK (scipy.linalg.lu) where ILU must be exact,
the defining identity (LU)_ij = a_ij on the pattern of A, closed-form
limits of the pivots on Laplacian stencils, and scipy's triangular solver.
"""

import json

import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from workloads import Csr, poisson2d, poisson3d, random_diag_dominant, convdiff2d_upwind


def _col_dd_tridiag(n, seed):
    """Tridiagonal, strictly diagonally dominant by columns, so Gaussian
    elimination with partial pivoting performs no row interchange and
    LAPACK's LU is the unpivoted one."""
    rng = np.random.default_rng(seed)
    lo = rng.uniform(-1, 1, n - 1)
    up = rng.uniform(-1, 1, n - 1)
    colsum = np.zeros(n)
    colsum[:-1] += np.abs(lo)
    colsum[1:] += np.abs(up)
    d = (1.5 + colsum) * rng.choice([-1, 1], n)
    return Csr.from_scipy(sp.diags([lo, d, up], [-1, 0, 1], format="csr"))


def _col_dd_dense(n, seed, density=0.4):
    rng = np.random.default_rng(seed)
    A = rng.uniform(-1, 1, (n, n)) * (rng.random((n, n)) < density)
    np.fill_diagonal(A, 0.0)
    np.fill_diagonal(A, 1.0 + np.abs(A).sum(axis=0))
    return A


def _lapack_lu_nopivot(Ad):
    P, L, U = sla.lu(Ad)
    assert np.array_equal(P, np.eye(len(Ad))), "expected no pivoting on a column-dominant matrix"
    return L, U


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_ilu0_exact_on_tridiagonal(orc, seed):
    # ILU(0) of a tridiagonal matrix creates no fill, so it is the exact LU.
    A = _col_dd_tridiag(40, seed)
    L, U = orc.ilu0(A)
    Lr, Ur = _lapack_lu_nopivot(A.to_scipy().toarray())
    np.testing.assert_allclose(L.to_scipy().toarray(), Lr, rtol=0, atol=1e-14)
    np.testing.assert_allclose(U.to_scipy().toarray(), Ur, rtol=1e-14, atol=1e-14)


@pytest.mark.parametrize("maker", [lambda: poisson2d(12), lambda: poisson3d(6),
                                   lambda: random_diag_dominant(300, 6, band=40, seed=3),
                                   lambda: convdiff2d_upwind(10, 10.0)])
def test_ilu0_defining_identity(orc, maker):
    # ILU(0): L unit lower, U upper, pattern(L+U) = pattern(A), (LU)_ij = a_ij on pattern(A).
    A = maker()
    L, U = orc.ilu0(A)
    Ls, Us, As = L.to_scipy(), U.to_scipy(), A.to_scipy()
    assert sp.triu(Ls, 1).nnz == 0 and np.all(Ls.diagonal() == 1.0)
    assert sp.tril(Us, -1).nnz == 0
    def struct(M):
        return sp.csr_matrix((np.ones(M.nnz), M.ci, M.rp), shape=(M.n, M.n))
    pat = struct(A)
    lu_pat = sp.tril(struct(L), -1) + struct(U)
    assert abs(lu_pat - pat).nnz == 0
    LU = (Ls @ Us).tocsr()
    err = abs((LU - As).multiply(pat)).max()
    assert err <= 1e-13 * abs(As).max()


def test_ilu0_stencil_pivot_limits(orc):
    # Pivots of the 5-point (7-point) Laplacian satisfy d = 4 - 2/d (6 - 3/d)
    # in the interior; the fixed points are 2 + sqrt(2) and 3 + sqrt(6).
    L, U = orc.ilu0(poisson2d(32))
    assert abs(U.to_scipy().diagonal()[-1] - (2 + np.sqrt(2))) < 1e-12
    L, U = orc.ilu0(poisson3d(24))
    d = U.to_scipy().diagonal()
    s = 24
    c = s // 2
    assert abs(d[c + s * c + s * s * c] - (3 + np.sqrt(6))) < 1e-12
    # U's off-diagonals equal A's (no fill to modify them for these stencils)
    A = poisson3d(6)
    L, U = orc.ilu0(A)
    np.testing.assert_array_equal(sp.triu(U.to_scipy(), 1).toarray(), sp.triu(A.to_scipy(), 1).toarray())


def test_ilu0_errors(orc):
    A = Csr.from_scipy(sp.csr_matrix(np.array([[0.0, 1.0], [1.0, 2.0]])))
    with pytest.raises(orc.OracleError) as e:
        orc.ilu0(A)
    assert e.value.status == orc.E_ZERO_PIVOT


@pytest.mark.parametrize("seed", [0, 1])
def test_ilut_no_dropping_is_exact_lu(orc, seed):
    Ad = _col_dd_dense(30, seed)
    A = Csr.from_scipy(sp.csr_matrix(Ad))
    L, U = orc.ilut(A, 0.0, A.n)
    Lr, Ur = _lapack_lu_nopivot(Ad)
    np.testing.assert_allclose(L.to_scipy().toarray(), Lr, rtol=0, atol=1e-13)
    np.testing.assert_allclose(U.to_scipy().toarray(), Ur, rtol=0, atol=1e-12)


def test_ilut_limits(orc):
    A = random_diag_dominant(200, 6, band=30, seed=5)
    # tau = infinity: every off-diagonal is dropped -> L = I, U = diag(A)
    L, U = orc.ilut(A, 1e300, 10)
    assert L.nnz == A.n and U.nnz == A.n
    np.testing.assert_array_equal(U.to_scipy().diagonal(), A.to_scipy().diagonal())
    # p = 0: no off-diagonal survives either
    L, U = orc.ilut(A, 0.0, 0)
    assert L.nnz == A.n and U.nnz == A.n
    np.testing.assert_array_equal(U.to_scipy().diagonal(), A.to_scipy().diagonal())
    # tridiagonal with tau = 0 equals ILU(0) (= exact LU)
    T = _col_dd_tridiag(50, 7)
    L1, U1 = orc.ilut(T, 0.0, 5)
    L0, U0 = orc.ilu0(T)
    np.testing.assert_allclose(L1.to_scipy().toarray(), L0.to_scipy().toarray(), atol=1e-15)
    np.testing.assert_allclose(U1.to_scipy().toarray(), U0.to_scipy().toarray(), atol=1e-15)


def test_ilut_threshold_and_fill_bound(orc):
    # Every stored off-diagonal obeys |w| >= tau*||a_i||, at most p per side.
    A = convdiff2d_upwind(24, 10.0)
    tau, p = 1e-3, 3
    L, U = orc.ilut(A, tau, p)
    As = A.to_scipy()
    nrm = np.sqrt(np.asarray(As.multiply(As).sum(axis=1)).ravel())
    for M, strict in ((L.to_scipy(), -1), (U.to_scipy(), 1)):
        off = sp.tril(M, -1) if strict < 0 else sp.triu(M, 1)
        off = off.tocsr()
        assert np.diff(off.indptr).max() <= p
        rows = np.repeat(np.arange(A.n), np.diff(off.indptr))
        assert np.all(np.abs(off.data) >= tau * nrm[rows])


def test_triangular_substitution(orc):
    A = random_diag_dominant(400, 8, band=50, seed=11)
    L, U = orc.ilu0(A)
    b = np.random.default_rng(0).uniform(-1, 1, A.n)
    x = orc.lower_solve(L, b)
    xr = spla.spsolve_triangular(L.to_scipy(), b, lower=True)
    np.testing.assert_allclose(x, xr, rtol=1e-13, atol=1e-13)
    y = orc.upper_solve(U, b)
    yr = spla.spsolve_triangular(U.to_scipy(), b, lower=False)
    np.testing.assert_allclose(y, yr, rtol=1e-12, atol=1e-13)
    assert np.linalg.norm(U.to_scipy() @ y - b) <= 1e-13 * np.linalg.norm(b)
