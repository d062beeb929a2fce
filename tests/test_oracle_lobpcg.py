"""Pins of the oracle's LOBPCG (the eigenvalue solver of the paper's Sec. 4
experiment) against what the mathematics fixes:
  * the closed-form spectrum of the 7-point (3D) and 3-point (1D) Dirichlet
    Laplacians, including the triple second eigenvalue of the cube;
  * a dense LAPACK eigensolver on an anisotropic 2D problem;
  * Cauchy interlacing: every Ritz value bounds its eigenvalue from above,
    and the Ritz values never increase (each trial space holds the
    previous iterate);
  * the trial space [X_i, W_i, P_i] equals [X_i, W_i, X_(i-1)]: a
    test-side LOBPCG that keeps the previous iterate instead of P gives the
    same Ritz values step by step;
  * a trial space of full dimension gives the exact eigenpairs at once;
  * X is orthonormal and diagonalises A on exit;
  * on a clustered spectrum every Ritz value stays above lambda_min (the
    P-drop bound of 1e-8; with 1e-14 the iteration diverged).
"""

import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp

import oracle
from workloads import Csr, aniso2d, poisson2d, poisson3d


def _laplace3d_eigs(s, k):
    t = np.sin(np.arange(1, 5) * np.pi / (2 * (s + 1))) ** 2
    return np.sort([4 * (t[i] + t[j] + t[l]) for i in range(4) for j in range(4) for l in range(4)])[:k]


def _start(n, k, seed=0):
    return np.random.default_rng(seed).uniform(-1.0, 1.0, (n, k))


def _sait(A, tau=0.01, m=10, level=0):
    L, U = oracle.ilu0(A) if level == 0 else oracle.iluk(A, level)
    return ("sait64", *oracle.sait_factors(L, U, m, tau=tau))


@pytest.mark.parametrize("prec", ["none", "sait"])
def test_laplace3d_closed_form(prec):
    A = poisson3d(10)
    out = oracle.lobpcg(A, _start(A.n, 4), None if prec == "none" else _sait(A), tol=1e-10, maxit=2000)
    ev = _laplace3d_eigs(10, 4)
    assert ev[1] == ev[3] or abs(ev[1] - ev[3]) < 1e-15  # the triple eigenvalue
    assert out["status"] == 0
    np.testing.assert_allclose(out["lam"], ev, rtol=1e-11)


def test_laplace1d_exact_preconditioner():
    n = 200
    main, off = 2.0 * np.ones(n), -np.ones(n - 1)
    A = Csr.from_scipy(sp.diags([off, main, off], [-1, 0, 1], format="csr"))
    L, U = oracle.ilu0(A)  # tridiagonal: ILU(0) is the exact LU, T = A^-1
    out = oracle.lobpcg(A, _start(n, 3, 1), ("exact", L, U), tol=1e-10)
    ev = 2 - 2 * np.cos(np.arange(1, 4) * np.pi / (n + 1))
    assert out["status"] == 0
    np.testing.assert_allclose(out["lam"], ev, rtol=1e-11)


@pytest.mark.parametrize("prec", ["none", "sait", "jacobi"])
def test_aniso_against_dense_lapack(prec):
    A = aniso2d(24, 0.1)
    L, U = oracle.ilu0(A)
    p = {"none": None, "sait": _sait(A, 0.02, 6), "jacobi": ("jacobi", L, U, 3)}[prec]
    out = oracle.lobpcg(A, _start(A.n, 5, 2), p, tol=1e-9, maxit=3000)
    ev = sla.eigvalsh(A.to_scipy().toarray())[:5]
    assert out["status"] == 0
    np.testing.assert_allclose(out["lam"], ev, rtol=1e-10)
    X = out["X"]
    np.testing.assert_allclose(X.T @ X, np.eye(5), atol=1e-10)
    np.testing.assert_allclose(X.T @ (A.to_scipy() @ X), np.diag(out["lam"]), atol=1e-10 * ev[-1])


def test_ritz_values_interlace_and_decrease():
    A = poisson2d(20)
    ev = sla.eigvalsh(A.to_scipy().toarray())[:4]
    out = oracle.lobpcg(A, _start(A.n, 4, 3), _sait(A, 0.05, 4), tol=1e-10)
    th = out["theta_hist"]
    assert np.all(th >= ev - 1e-12 * ev)
    assert np.all(np.diff(th, axis=0) <= 1e-12 * th[:-1])


def _lobpcg_previous_iterate(A, X0, T, steps):
    """LOBPCG with the trial space [X_i, W_i, X_(i-1)] (the same space as
    [X_i, W_i, P_i] in exact arithmetic); Ritz values after every step."""
    As = A.to_scipy()
    k = X0.shape[1]

    def rr(S):
        GA, GB = S.T @ (As @ S), S.T @ S
        th, V = sla.eigh(0.5 * (GA + GA.T), GB)
        return th[:k], V[:, :k]

    th, V = rr(X0)
    X, Xprev, out = X0 @ V, None, []
    for _ in range(steps):
        R = As @ X - X * th
        W = T(R)
        S = np.hstack([X, W] + ([Xprev] if Xprev is not None else []))
        th, V = rr(S)
        Xprev, X = X, S @ V
        out.append(th)
    return np.array(out)


def test_p_spans_the_previous_iterate():
    A = aniso2d(16, 0.3)
    L, U = oracle.ilu0(A)
    prec = _sait(A, 0.02, 4)
    X0 = _start(A.n, 3, 4)
    steps = 6
    ref = _lobpcg_previous_iterate(A, X0, oracle.lobpcg_module.block_preconditioner(prec), steps)
    out = oracle.lobpcg(A, X0, prec, tol=0.0, maxit=steps)
    np.testing.assert_allclose(out["theta_hist"][1:steps + 1], ref, rtol=1e-9)


def test_full_trial_space_is_exact():
    rng = np.random.default_rng(5)
    B = sp.random(12, 12, density=0.4, random_state=7).toarray()
    Ad = B @ B.T + 12 * np.eye(12)
    A = Csr.from_scipy(sp.csr_matrix(Ad))
    out = oracle.lobpcg(A, rng.uniform(-1, 1, (12, 4)), None, tol=1e-12)
    assert out["status"] == 0 and out["iters"] <= 2  # [X, W, P] spans R^12 at step 2
    np.testing.assert_allclose(out["lam"], sla.eigvalsh(Ad)[:4], rtol=1e-12)


def test_rank_deficient_start_rejected():
    A = poisson2d(6)
    X0 = _start(A.n, 2)
    X0[:, 1] = X0[:, 0]
    with pytest.raises(ValueError):
        oracle.lobpcg(A, X0)


def test_clustered_spectrum_stays_above_lambda_min():
    # a symmetric diagonally dominant matrix whose 2nd..6th eigenvalues lie
    # within 5 % of each other, k = 4, SAIT_Thr(1e-3, 3): the trial basis
    # [X, W, P] becomes nearly dependent.  Cauchy interlacing forbids a Ritz
    # value below lambda_min; with P kept down to a pivot of 1e-14 the Ritz
    # values fell below it and the iteration diverged.  Dropping P below
    # 1e-8 keeps every Ritz value above lambda_min and converges to LAPACK's
    # eigenvalues.
    from workloads import random_diag_dominant

    R = random_diag_dominant(750, 4, band=73, seed=2).to_scipy()
    off = R - sp.diags(R.diagonal())
    S = (off + off.T).tocsr()
    S = S + sp.diags(1.0 + np.asarray(abs(S).sum(axis=1)).ravel())
    A = Csr.from_scipy(sp.csr_matrix(S))
    ev = sla.eigh(S.toarray(), eigvals_only=True)
    assert ev[5] - ev[1] < 0.05 * ev[1]
    L, U = oracle.ilu0(A)
    out = oracle.lobpcg(A, _start(A.n, 4, 12), ("sait64", *oracle.sait_factors(L, U, 3, tau=1e-3)), tol=1e-8,
                        maxit=3000)
    assert out["status"] == 0 and out["p_drops"] > 0
    assert np.all(np.asarray(out["theta_hist"])[:, 0] >= ev[0] * (1 - 1e-12))
    np.testing.assert_allclose(out["lam"], ev[:4], rtol=1e-10)
