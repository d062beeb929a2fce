"""Randomised parity of the device solvers: seeded matrices of the kinds the
paper and its workloads use (random diagonally dominant, upwind
convection-diffusion, anisotropic diffusion, Poisson), each with random
solver settings, against the oracle's solver on the same factors.

GMRES / FGMRES (right preconditioning, Sec. 3.1): random restart, rtol,
m, tau, side of the upper recursion and storage precision; iteration counts
within one of the oracle's (two for the binary32 / bfloat16 factors, whose
oracle applies the same roundings), the true residual at most rtol.
PCG (the paper's solver, Sec. 4) on symmetric matrices with the SAIT,
Jacobi, exact and no preconditioner, level-0 or level-1 ILU: iteration
counts within one, the true residual at most 1.5 rtol (PCG stops on the
recursively updated residual).
Adjoint (the backward of the differentiable solve): A^T lam = g by
(F)GMRES with the transposed factors, iteration counts within one and the
gradient on A's pattern bit for bit the oracle's for the same lam."""

import numpy as np
import pytest
import scipy.sparse as sp

import oracle
from paper_2106_12836_amd import SaitPreconditioner
from workloads import Csr, aniso2d, convdiff2d_upwind, poisson2d, poisson3d, random_diag_dominant, spmv_rhs

pytestmark = pytest.mark.gpu


def _t(x):
    import torch

    return torch.tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda:0")


def _matrix(rng, seed):
    kind = str(rng.choice(["rdd", "rdd", "convdiff", "aniso", "poisson2d", "poisson3d"]))
    if kind == "rdd":
        n = int(rng.integers(200, 20000))
        band = None if rng.random() < 0.3 else int(rng.integers(8, max(9, n // 8)))
        return kind, random_diag_dominant(n, int(rng.integers(2, 10)), band=band, seed=seed)
    if kind == "convdiff":
        return kind, convdiff2d_upwind(int(rng.integers(12, 120)), float(rng.choice([0.5, 2.0, 10.0])))
    if kind == "aniso":
        return kind, aniso2d(int(rng.integers(12, 120)), float(rng.choice([0.05, 0.2, 1.0])))
    if kind == "poisson2d":
        return kind, poisson2d(int(rng.integers(12, 120)))
    return kind, poisson3d(int(rng.integers(6, 24)))


def _gmres_case(seed):
    rng = np.random.default_rng(2000 + seed)
    kind, A = _matrix(rng, seed)
    o = dict(restart=int(rng.choice([5, 10, 20, 30, 50])), rtol=float(rng.choice([1e-6, 1e-8, 1e-10])),
             flexible=bool(rng.random() < 0.5), m=int(rng.integers(1, 5)),
             tau=float(rng.choice([1e-3, 1e-2, 5e-2])), upper_side=str(rng.choice(["left", "right"])),
             precision=str(rng.choice(["f64", "f64", "f32", "bf16"])))
    x_true = rng.uniform(-1.0, 1.0, A.n)
    return kind, A, spmv_rhs(A, x_true), o


@pytest.mark.parametrize("seed", range(24))
def test_random_gmres_matches_oracle(seed):
    kind, A, b, o = _gmres_case(seed)
    print(f"[test_random_gmres_matches_oracle] seed={seed} {kind} n={A.n} {o}", flush=True)
    L, U = oracle.ilu0(A)
    ML, MU = oracle.sait_factors(L, U, o["m"], tau=o["tau"], upper_side=o["upper_side"])
    if o["precision"] == "f64":
        prec = ("sait64", ML, MU)
    else:
        prec = ("sait32", ML, oracle.storage_values(ML, o["precision"]), MU,
                oracle.storage_values(MU, o["precision"]))
    ref = oracle.gmres(A, b, prec, restart=o["restart"], rtol=o["rtol"], flexible=o["flexible"], maxit=5000)
    assert ref["status"] == 0, ref["iters"]
    pre = SaitPreconditioner(A, m=o["m"], tau=o["tau"], upper_side=o["upper_side"], precision=o["precision"])
    try:
        x, (info,) = pre.solve(_t(b), restart=o["restart"], rtol=o["rtol"], flexible=o["flexible"], maxit=5000)
        xs = x.cpu().numpy()
    finally:
        pre.close()
    print(f"  device {info.iterations} oracle {ref['iters']}", flush=True)
    assert info.status == 0
    slack = 1 if o["precision"] == "f64" else 2
    assert abs(info.iterations - ref["iters"]) <= slack, (info.iterations, ref["iters"])
    r = b - A.to_scipy() @ xs
    assert np.linalg.norm(r) <= o["rtol"] * np.linalg.norm(b) * (1 + 1e-7)


def _spd(rng, seed):
    kind = str(rng.choice(["sym-rdd", "aniso", "poisson2d", "poisson3d"]))
    if kind == "sym-rdd":
        n = int(rng.integers(200, 20000))
        R = random_diag_dominant(n, int(rng.integers(2, 8)), band=int(rng.integers(8, max(9, n // 8))),
                                 seed=seed).to_scipy()
        off = R - sp.diags(R.diagonal())
        S = (off + off.T).tocsr()
        S = S + sp.diags(1.0 + np.asarray(abs(S).sum(axis=1)).ravel())
        return kind, Csr.from_scipy(sp.csr_matrix(S))
    if kind == "aniso":
        return kind, aniso2d(int(rng.integers(12, 100)), float(rng.choice([0.05, 0.2, 1.0])))
    if kind == "poisson2d":
        return kind, poisson2d(int(rng.integers(12, 100)))
    return kind, poisson3d(int(rng.integers(6, 24)))


@pytest.mark.parametrize("seed", range(16))
def test_random_pcg_matches_oracle(seed):
    rng = np.random.default_rng(3000 + seed)
    kind, A = _spd(rng, seed)
    level = int(rng.integers(0, 2))
    pk = str(rng.choice(["sait", "sait", "jacobi", "exact", "none"]))
    sweeps = int(rng.integers(1, 5))
    m, tau = int(rng.integers(1, 8)), float(rng.choice([1e-3, 1e-2, 5e-2]))
    rtol = float(rng.choice([1e-6, 1e-8, 1e-10]))
    f = rng.uniform(0.0, 1.0, A.n)
    print(f"[test_random_pcg_matches_oracle] seed={seed} {kind} n={A.n} level={level} {pk} sweeps={sweeps} "
          f"m={m} tau={tau} rtol={rtol}", flush=True)
    L, U = oracle.ilu0(A) if level == 0 else oracle.iluk(A, level)
    if pk == "sait":
        prec = ("sait64", *oracle.sait_factors(L, U, m, tau=tau))
    elif pk == "jacobi":
        prec = ("jacobi", L, U, sweeps)
    elif pk == "exact":
        prec = ("exact", L, U)
    else:
        prec = None
    ref = oracle.pcg(A, f, prec, rtol=rtol, maxit=5000)
    assert ref["status"] == 0, ref["iters"]
    build = dict(m=m, tau=tau)
    if level:
        build.update(ilu_kind="iluk", ilu_level=level)
    pre = SaitPreconditioner(A, **build)
    try:
        if pk != "sait":
            pre.set_preconditioner(pk, sweeps)
        x, (info,) = pre.solve(_t(f), rtol=rtol, method="pcg", maxit=5000)
    finally:
        pre.close()
    print(f"  device {info.iterations} oracle {ref['iters']}", flush=True)
    assert info.status == 0
    assert abs(info.iterations - ref["iters"]) <= 1, (info.iterations, ref["iters"])
    assert info.true_relres <= 1.5 * rtol


@pytest.mark.parametrize("seed", range(12))
def test_random_adjoint_matches_oracle(seed):
    # the adjoint solve A^T lam = g with the transposed factors
    # (z = M_L^T (M_U^T r)) and the gradient on A's pattern, on seeded
    # nonsymmetric matrices and settings
    rng = np.random.default_rng(7000 + seed)
    kind, A = _matrix(rng, seed)
    m, tau = int(rng.integers(1, 5)), float(rng.choice([1e-3, 1e-2, 5e-2]))
    side = str(rng.choice(["left", "right"]))
    restart, flexible = int(rng.choice([10, 20, 30])), bool(rng.random() < 0.5)
    g = rng.uniform(-1.0, 1.0, A.n)
    print(f"[test_random_adjoint_matches_oracle] seed={seed} {kind} n={A.n} m={m} tau={tau} side={side} "
          f"restart={restart} flexible={flexible}", flush=True)
    L, U = oracle.ilu0(A)
    ML, MU = oracle.sait_factors(L, U, m, tau=tau, upper_side=side)
    ref = oracle.gmres(oracle.transpose(A), g, ("sait64", oracle.transpose(MU), oracle.transpose(ML)),
                       restart=restart, rtol=1e-10, flexible=flexible, maxit=5000)
    assert ref["status"] == 0
    pre = SaitPreconditioner(A, m=m, tau=tau, upper_side=side, build_transpose=1)
    try:
        lam, (info,) = pre.solve(_t(g), transpose=True, restart=restart, rtol=1e-10, flexible=flexible, maxit=5000)
        lam_np = lam.cpu().numpy()
        x = rng.uniform(-1.0, 1.0, A.n)
        gv = pre.grad_values(_t(lam_np), _t(x)).cpu().numpy()
    finally:
        pre.close()
    print(f"  device {info.iterations} oracle {ref['iters']}", flush=True)
    assert info.status == 0
    assert abs(info.iterations - ref["iters"]) <= 1, (info.iterations, ref["iters"])
    r = g - A.to_scipy().T @ lam_np
    assert np.linalg.norm(r) <= 1e-10 * np.linalg.norm(g) * (1 + 1e-7)
    np.testing.assert_array_equal(gv, oracle.grad_values(A, lam_np, x))
