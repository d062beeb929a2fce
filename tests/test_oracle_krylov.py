"""Pins of the oracle's preconditioner apply, storage roundings, (F)GMRES,
transpose and adjoint gradient.

Independent references: scipy sparse products and direct solves, numpy /
torch float conversions, the GMRES minimal-residual characterisation
computed by dense least squares over an explicit Krylov basis, closed
forms (A = I, exact preconditioner, diagonal A), and central finite
differences of the loss through a sparse LU solve.
"""

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla
import torch

from workloads import Csr, config, grf_diffusion2d, poisson2d, poisson3d, random_diag_dominant, uniform_vector


def _factors(orc, A, tau=1e-2, m=3):
    L, U = orc.ilu0(A)
    return (L, U, *orc.sait_factors(L, U, m, tau=tau))


def test_apply_f64_matches_scipy(orc):
    A = random_diag_dominant(3000, 8, band=200, seed=1)
    L, U, ML, MU = _factors(orc, A)
    r = uniform_vector(A.n, 3)
    z = orc.apply(ML, MU, r)
    zr = MU.to_scipy() @ (ML.to_scipy() @ r)
    np.testing.assert_allclose(z, zr, rtol=1e-13, atol=1e-14)


def test_roundings_bit_exact():
    import oracle as orc
    rng = np.random.default_rng(0)
    v = np.concatenate([rng.standard_normal(10000) * 10.0 ** rng.integers(-30, 30, 10000),
                        [0.0, -0.0, 1.0, 1e-40, 3.4e38, -2.5]])
    np.testing.assert_array_equal(orc.round_f32(v), v.astype(np.float32))
    # bf16 = RNE of the binary32 value: torch's float32 -> bfloat16 conversion
    b = orc.round_bf16(v)
    ref = torch.from_numpy(v.astype(np.float32)).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    np.testing.assert_array_equal(b, ref)
    # ties to even: 1 + 2^-8 is halfway between two bf16 neighbours
    t = np.array([1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8])
    np.testing.assert_array_equal(orc.bf16_to_f32(orc.round_bf16(t)), np.array([1.0, 1.0 + 2 * 2.0 ** -7], np.float32))


@pytest.mark.parametrize("prec", ["f32", "bf16"])
def test_mixed_apply_error_bound(orc, prec):
    # z from binary32 accumulation stays within 2 gamma_K |M_U| (|M_L| |r32|)
    # of the exact product of the rounded matrices (Higham, inner products).
    A = poisson3d(12)
    L, U, ML, MU = _factors(orc, A, 1e-3, 3)
    f1 = orc.storage_values(ML, prec)
    f2 = orc.storage_values(MU, prec)
    r = uniform_vector(A.n, 5)
    z = orc.apply_f32acc(ML, f1, MU, f2, r)
    r32 = r.astype(np.float32).astype(np.float64)
    M1 = sp.csr_matrix((f1.astype(np.float64), ML.ci, ML.rp), shape=(A.n, A.n))
    M2 = sp.csr_matrix((f2.astype(np.float64), MU.ci, MU.rp), shape=(A.n, A.n))
    zstar = M2 @ (M1 @ r32)
    K = max(np.diff(ML.rp).max(), np.diff(MU.rp).max()) + 1
    u = 2.0 ** -24
    gam = K * u / (1 - K * u)
    bound = 2 * gam * (abs(M2) @ (abs(M1) @ np.abs(r32))) * (1 + 4 * u)
    assert np.all(np.abs(z - zstar) <= bound)
    # and it is genuinely binary32, not FP64 in disguise
    assert np.abs(z - zstar).max() > 0


def test_gmres_identity_and_exact_preconditioner(orc):
    n = 50
    I = Csr(n, np.arange(n + 1, dtype=np.int32), np.arange(n, dtype=np.int32), np.ones(n))
    b = uniform_vector(n, 1)
    out = orc.gmres(I, b, None, restart=10, rtol=1e-12)
    assert out["iters"] == 1 and out["relres"] < 1e-15
    # tridiagonal A: ILU(0) = exact LU and SAIT(0, n-1) = exact inverses
    A = Csr.from_scipy(sp.diags([-np.ones(n - 1), 3 * np.ones(n), -np.ones(n - 1)], [-1, 0, 1], format="csr"))
    L, U = orc.ilu0(A)
    ML, MU = orc.sait_factors(L, U, n - 1, tau=0.0)
    out = orc.gmres(A, b, ("sait64", ML, MU), restart=10, rtol=1e-10)
    assert out["iters"] == 1 and out["relres"] < 1e-12
    out = orc.gmres(A, b, ("exact", L, U), restart=10, rtol=1e-10)
    assert out["iters"] == 1


def test_gmres_diagonal_distinct_values(orc):
    # A diagonal with d distinct eigenvalues: the minimal polynomial has
    # degree d, so unrestarted GMRES terminates in exactly d steps.
    d = np.repeat([1.0, 2.0, 5.0, 7.0, 11.0], 20)
    n = len(d)
    A = Csr(n, np.arange(n + 1, dtype=np.int32), np.arange(n, dtype=np.int32), d)
    b = uniform_vector(n, 2)
    out = orc.gmres(A, b, None, restart=50, rtol=1e-12)
    assert out["iters"] == 5
    np.testing.assert_allclose(out["x"], b / d, rtol=1e-11)


@pytest.mark.parametrize("flexible", [False, True])
def test_gmres_minimal_residual(orc, flexible):
    # GMRES step j minimises ||b - A M y|| over y in K_j(A M, b) (x0 = 0,
    # no restart): compare each estimate with dense least squares over an
    # orthonormalised Krylov basis.
    A = random_diag_dominant(60, 6, band=20, seed=4)
    A = Csr(A.n, A.rp, A.ci, A.v * np.where(np.arange(A.nnz) % 3 == 0, 0.3, 1.0))
    L, U, ML, MU = _factors(orc, A, 5e-2, 2)
    b = uniform_vector(A.n, 6)
    out = orc.gmres(A, b, ("sait64", ML, MU), restart=60, maxit=12, rtol=1e-30, flexible=flexible, history=True)
    As, M = A.to_scipy().toarray(), (MU.to_scipy() @ ML.to_scipy()).toarray()
    AM = As @ M
    K = [b / np.linalg.norm(b)]
    for j in range(1, 12):
        w = AM @ K[-1]
        for q in K:          # re-orthonormalise (twice) for a well-conditioned basis
            w -= (q @ w) * q
        for q in K:
            w -= (q @ w) * q
        K.append(w / np.linalg.norm(w))
    nb = np.linalg.norm(b)
    for j in range(1, 12):
        Q = np.array(K[:j]).T
        y, *_ = np.linalg.lstsq(AM @ Q, b, rcond=None)
        res = np.linalg.norm(b - AM @ Q @ y) / nb
        assert abs(out["hist"][j - 1] - res) <= 1e-9 * max(res, 1e-12) + 1e-14
    assert np.all(np.diff(out["hist"]) <= 1e-15)


def test_gmres_solution_and_flexible_equivalence(orc):
    c = config("c1", small=True)
    A, b = c["A"], c["b"]
    L, U, ML, MU = _factors(orc, A)
    g = orc.gmres(A, b, ("sait64", ML, MU), restart=8, rtol=1e-10)
    f = orc.gmres(A, b, ("sait64", ML, MU), restart=8, rtol=1e-10, flexible=True)
    assert g["status"] == 0 and g["relres"] <= 1e-10
    assert f["iters"] == g["iters"] and f["restarts"] == g["restarts"]
    x = spla.spsolve(A.to_scipy().tocsc(), b)
    cond = np.linalg.cond(A.to_scipy().toarray())
    assert np.linalg.norm(g["x"] - x) / np.linalg.norm(x) <= cond * 1e-10
    np.testing.assert_allclose(f["x"], g["x"], rtol=1e-9)
    np.testing.assert_allclose(g["x"], np.ones(A.n), rtol=1e-7)


def test_gmres_c1_reference_counts(orc):
    # Config c1 (64^2 Poisson, ILU(0), SAIT(1e-2, 3), GMRES(30), 1e-8):
    # the SAIT preconditioner must sit between the exact ILU(0) solves and
    # no preconditioning, and the true residual must meet the tolerance.
    c = config("c1")
    A, b = c["A"], c["b"]
    L, U, ML, MU = _factors(orc, A, c["tau"], c["m"])
    s = orc.gmres(A, b, ("sait64", ML, MU), restart=30, rtol=1e-8)
    e = orc.gmres(A, b, ("exact", L, U), restart=30, rtol=1e-8)
    o = orc.gmres(A, b, None, restart=30, rtol=1e-8)
    assert s["status"] == 0 and s["relres"] <= 1e-8
    assert e["iters"] < s["iters"] < o["iters"]


def test_gmres_maxit(orc):
    A = poisson2d(20)
    b = uniform_vector(A.n, 1)
    out = orc.gmres(A, b, None, restart=5, maxit=7, rtol=1e-14)
    assert out["status"] == orc.NOT_CONVERGED and out["iters"] == 7
    z = orc.gmres(A, np.zeros(A.n), None, restart=5, rtol=1e-8)
    assert z["iters"] == 0 and np.all(z["x"] == 0)


def test_transpose(orc):
    A = random_diag_dominant(500, 7, band=None, seed=2)
    At = orc.transpose(A)
    ref = Csr.from_scipy(A.to_scipy().T.tocsr())
    np.testing.assert_array_equal(At.rp, ref.rp)
    np.testing.assert_array_equal(At.ci, ref.ci)
    np.testing.assert_array_equal(At.v, ref.v)


def test_adjoint_gradient_dense_closed_form(orc):
    # loss = ||x - xt||^2, x = A^-1 b: dl/db = lambda = A^-T 2(x - xt),
    # dl/dA_ij = -lambda_i x_j.
    A = random_diag_dominant(40, 5, band=10, seed=3)
    Ad = A.to_scipy().toarray()
    b = uniform_vector(40, 1)
    xt = uniform_vector(40, 2)
    x = np.linalg.solve(Ad, b)
    lam = np.linalg.solve(Ad.T, 2 * (x - xt))
    g = orc.grad_values(A, lam, x)
    full = -np.outer(lam, x)
    rows = np.repeat(np.arange(A.n), np.diff(A.rp))
    np.testing.assert_allclose(g, full[rows, A.ci], rtol=1e-15)


def test_adjoint_gradient_finite_differences(orc):
    # The oracle's adjoint path (GMRES on A^T preconditioned by M_L^T M_U^T,
    # then grad_values) against central differences of the loss evaluated
    # with a sparse direct solve, 16 seeded unit directions, h = 1e-6.
    A, kap = grf_diffusion2d(16, seed=5)
    At_, _ = grf_diffusion2d(16, seed=5, kappa_log=np.log(kap.reshape(16, 16)).T * 1.05)
    b = np.ones(A.n)
    xt = spla.spsolve(At_.to_scipy().tocsc(), b)
    L, U, ML, MU = _factors(orc, A)

    def loss(vals, bb):
        Ap = sp.csr_matrix((vals, A.ci, A.rp), shape=(A.n, A.n)).tocsc()
        return float(np.sum((spla.splu(Ap).solve(bb) - xt) ** 2))

    fw = orc.gmres(A, b, ("sait64", ML, MU), restart=30, rtol=1e-14, maxit=2000)
    x = fw["x"]
    AT, MLT, MUT = orc.transpose(A), orc.transpose(ML), orc.transpose(MU)
    bw = orc.gmres(AT, 2 * (x - xt), ("sait64", MUT, MLT), restart=30, rtol=1e-14, maxit=2000)
    lam = bw["x"]
    gA = orc.grad_values(A, lam, x)
    gb = lam
    rng = np.random.default_rng(7)
    h = 1e-6
    for _ in range(16):
        # entry-relative Gaussian direction, normalised to unit 2-norm
        xi = rng.standard_normal(A.nnz) * np.abs(A.v)
        eta = rng.standard_normal(A.n) * np.abs(b)
        nrm = np.sqrt(xi @ xi + eta @ eta)
        xi, eta = xi / nrm, eta / nrm
        dfd = (loss(A.v + h * xi, b + h * eta) - loss(A.v - h * xi, b - h * eta)) / (2 * h)
        dan = gA @ xi + gb @ eta
        assert abs(dfd - dan) <= 1e-6 * max(abs(dfd), abs(dan))
