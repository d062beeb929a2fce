"""GPU parity of the apply, the (F)GMRES solve, the transpose path and the
adjoint gradient against the CPU oracle.

Tolerances:
  * FP64 apply: |z - z_oracle| <= 4 K u (|M_U| (|M_L| |r|)) componentwise
    (K = longest row + 1, u = 2^-53): the two sides only differ in the
    order of the row sums and in fused multiply-adds, and 1e-12 relative
    in the 2-norm.
  * binary32 accumulation: within 2 gamma_K |M_U|(|M_L| |r32|) (u = 2^-24)
    of the exact product of the stored matrices.
  * GMRES: same iteration count as the oracle +- 1 and the true residual
    below rtol.
"""

import numpy as np
import pytest
import scipy.sparse as sp
import torch

import oracle
from paper_2106_12836_amd import SaitError, SaitPreconditioner, sait_solve_autograd
from workloads import Csr, config, grf_diffusion2d, poisson3d, random_diag_dominant, uniform_vector

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _t(x):
    return torch.tensor(np.ascontiguousarray(x), dtype=torch.float64, device=DEV)


def _sp(M: Csr, vals=None):
    return sp.csr_matrix((M.v if vals is None else vals, M.ci, M.rp), shape=(M.n, M.n))


def _factors(A, tau, m, ilu="ilu0"):
    L, U = oracle.ilu0(A) if ilu == "ilu0" else oracle.ilut(A, 1e-3, 10)
    return (L, U, *oracle.sait_factors(L, U, m, tau=tau))


APPLY_CASES = [
    ("c3-small", lambda: config("c3", small=True)["A"], 1e-3, 3),
    ("rdd", lambda: random_diag_dominant(5003, 8, band=500, seed=5), 1e-2, 3),
    ("c1", lambda: config("c1")["A"], 1e-2, 3),
]


# apply shapes: -64/-65 sliced ELL, -8/-16 LDS-staged CSR (all four exact
# column-order sums), > 0 lanes per row of the wavefront CSR kernel
SHAPES = [-64, -65, -8, -16, 1, 4, 8, 16, 64]


@pytest.mark.parametrize("name,maker,tau,m", APPLY_CASES, ids=[c[0] for c in APPLY_CASES])
@pytest.mark.parametrize("lanes", SHAPES)
def test_apply_f64(name, maker, tau, m, lanes):
    print(f"[test_apply_f64] {name} lanes={lanes}", flush=True)
    A = maker()
    L, U, ML, MU = _factors(A, tau, m)
    pre = SaitPreconditioner(A, m=m, tau=tau, build_transpose=1)
    try:
        from paper_2106_12836_amd import sait_set_apply_lanes
        sait_set_apply_lanes(pre.handle, lanes, lanes)
        r = uniform_vector(A.n, 7)
        z = pre.apply(_t(r)).cpu().numpy()
        zr = oracle.apply(ML, MU, r)
        if lanes < 0:
            # rounded products summed in column order: the oracle's arithmetic
            np.testing.assert_array_equal(z, zr)
        K = max(np.diff(ML.rp).max(), np.diff(MU.rp).max()) + 1
        bound = 4 * K * 2.0 ** -53 * (abs(_sp(MU)) @ (abs(_sp(ML)) @ np.abs(r)))
        assert np.all(np.abs(z - zr) <= bound + 1e-300)
        assert np.linalg.norm(z - zr) <= 1e-12 * np.linalg.norm(zr)
        # transpose apply: z = M_L^T (M_U^T r)
        zt = pre.apply(_t(r), transpose=True).cpu().numpy()
        ztr = oracle.apply(oracle.transpose(MU), oracle.transpose(ML), r)
        assert np.linalg.norm(zt - ztr) <= 1e-12 * np.linalg.norm(ztr)
        # operator products
        y = pre.matvec(_t(r)).cpu().numpy()
        assert np.linalg.norm(y - oracle.spmv(A, r)) <= 1e-13 * np.linalg.norm(y)
        yt = pre.matvec(_t(r), transpose=True).cpu().numpy()
        assert np.linalg.norm(yt - _sp(A).T @ r) <= 1e-13 * np.linalg.norm(yt)
    finally:
        pre.close()


@pytest.mark.parametrize("nrhs,shape", [(2, -64), (3, -64), (4, -64), (5, -65), (8, -64), (4, 8), (11, -64)])
def test_apply_block(nrhs, shape):
    # sliced-ELL blocks (2..5, 8 right-hand sides): every column bit for bit
    # the oracle's FP64 apply; other shapes / widths: the wavefront kernel
    print(f"[test_apply_block] nrhs={nrhs} shape={shape}", flush=True)
    from paper_2106_12836_amd import sait_set_apply_lanes
    A = config("c3", small=True)["A"]
    L, U, ML, MU = _factors(A, 1e-3, 3)
    pre = SaitPreconditioner(A, m=3, tau=1e-3)
    try:
        sait_set_apply_lanes(pre.handle, shape, shape)
        R = uniform_vector(A.n, 3, k=nrhs)
        Z = pre.apply(_t(R)).cpu().numpy()
        for k in range(nrhs):
            zr = oracle.apply(ML, MU, R[:, k])
            if shape < 0 and nrhs in (2, 3, 4, 5, 8):
                np.testing.assert_array_equal(Z[:, k], zr)
            else:
                assert np.linalg.norm(Z[:, k] - zr) <= 1e-12 * np.linalg.norm(zr)
    finally:
        pre.close()


def test_matvec_block_sliced():
    # A X with the sliced-ELL block kernel: each column equals scipy's
    # product up to rounding and the one-vector device product bit for bit
    print("[test_matvec_block_sliced]", flush=True)
    from paper_2106_12836_amd import sait_set_apply_lanes
    A = config("c3", small=True)["A"]
    pre = SaitPreconditioner(A, m=3, tau=1e-3)
    try:
        R = uniform_vector(A.n, 4, k=4)
        Y = pre.matvec(_t(R)).cpu().numpy()
        for k in range(4):
            y1 = pre.matvec(_t(np.ascontiguousarray(R[:, k]))).cpu().numpy()
            np.testing.assert_array_equal(Y[:, k], y1)
            ys = A.to_scipy() @ R[:, k]
            assert np.linalg.norm(Y[:, k] - ys) <= 1e-14 * np.linalg.norm(ys)
    finally:
        pre.close()


@pytest.mark.parametrize("prec", ["f32", "bf16"])
@pytest.mark.parametrize("nrhs,shape", [(1, -64), (1, -65), (1, -8), (1, -16), (4, -16), (4, -64), (3, -65)])
def test_apply_mixed_bound(prec, nrhs, shape):
    print(f"[test_apply_mixed_bound] {prec} nrhs={nrhs} shape={shape}", flush=True)
    A = config("c3", small=True)["A"]
    L, U, ML, MU = _factors(A, 1e-3, 3)
    pre = SaitPreconditioner(A, m=3, tau=1e-3, precision=prec)
    try:
        from paper_2106_12836_amd import sait_set_apply_lanes
        sait_set_apply_lanes(pre.handle, shape, shape)
        R = uniform_vector(A.n, 9, k=nrhs)
        Z = pre.apply(_t(R if nrhs > 1 else R[:, 0])).cpu().numpy().reshape(A.n, nrhs)
        f1 = oracle.storage_values(ML, prec).astype(np.float64)
        f2 = oracle.storage_values(MU, prec).astype(np.float64)
        K = max(np.diff(ML.rp).max(), np.diff(MU.rp).max()) + 1
        u = 2.0 ** -24
        gam = K * u / (1 - K * u)
        for k in range(nrhs):
            r32 = R[:, k].astype(np.float32).astype(np.float64)
            zstar = _sp(MU, f2) @ (_sp(ML, f1) @ r32)
            bound = 2 * gam * (abs(_sp(MU, f2)) @ (abs(_sp(ML, f1)) @ np.abs(r32))) * (1 + 4 * u)
            assert np.all(np.abs(Z[:, k] - zstar) <= bound)
            zo = oracle.apply_f32acc(ML, f1.astype(np.float32), MU, f2.astype(np.float32), R[:, k])
            if nrhs == 1 or shape < 0:
                # binary32 products and sums in the oracle's order
                np.testing.assert_array_equal(Z[:, k], zo)
            assert np.linalg.norm(Z[:, k] - zo) <= 1e-5 * np.linalg.norm(zo)
    finally:
        pre.close()


@pytest.mark.parametrize("cfg,flexible", [("c1", False), ("c1", True), ("c2s", False), ("c3s", True)])
def test_gmres_matches_oracle(cfg, flexible):
    print(f"[test_gmres_matches_oracle] {cfg} flexible={flexible}", flush=True)
    c = config({"c1": "c1", "c2s": "c2", "c3s": "c3"}[cfg], small=cfg.endswith("s"))
    A, b = c["A"], c["b"]
    L, U, ML, MU = _factors(A, c["tau"], c["m"], c["ilu"])
    ref = oracle.gmres(A, b, ("sait64", ML, MU), restart=c["restart"], rtol=c["rtol"], flexible=flexible)
    pre = SaitPreconditioner(A, m=c["m"], tau=c["tau"], ilu_kind=c["ilu"])
    try:
        x, info = pre.solve(_t(b), restart=c["restart"], rtol=c["rtol"], flexible=flexible)
        inf = info[0]
        assert inf.status == 0
        assert inf.true_relres <= c["rtol"]
        assert abs(inf.iterations - ref["iters"]) <= 1, (inf.iterations, ref["iters"])
        xs = x.cpu().numpy()
        r = b - _sp(A) @ xs
        assert np.linalg.norm(r) <= c["rtol"] * np.linalg.norm(b) * 1.0000001
        assert np.linalg.norm(xs - ref["x"]) <= 1e-5 * np.linalg.norm(ref["x"])
    finally:
        pre.close()


@pytest.mark.parametrize("prec", ["f32", "bf16"])
def test_fgmres_mixed(prec):
    print(f"[test_fgmres_mixed] {prec}", flush=True)
    c = config("c3", small=True)
    A, b = c["A"], c["b"]
    L, U, ML, MU = _factors(A, c["tau"], c["m"])
    f1 = oracle.storage_values(ML, prec)
    f2 = oracle.storage_values(MU, prec)
    ref = oracle.gmres(A, b, ("sait32", ML, f1, MU, f2), restart=40, rtol=1e-10, flexible=True)
    pre = SaitPreconditioner(A, m=3, tau=1e-3, precision=prec)
    try:
        x, info = pre.solve(_t(b), restart=40, rtol=1e-10, flexible=True)
        inf = info[0]
        assert inf.status == 0 and inf.true_relres <= 1e-10
        assert abs(inf.iterations - ref["iters"]) <= 2, (inf.iterations, ref["iters"])
        xs = x.cpu().numpy()
        assert np.linalg.norm(xs - c["x_true"]) <= 1e-6 * np.linalg.norm(c["x_true"])
    finally:
        pre.close()


def test_solve_edge_cases():
    print("[test_solve_edge_cases]", flush=True)
    A = config("c1", small=True)["A"]
    pre = SaitPreconditioner(A, m=3, tau=1e-2)
    try:
        # b = 0 -> x = 0, no iterations
        x, info = pre.solve(torch.zeros(A.n, dtype=torch.float64, device=DEV), x=_t(np.ones(A.n)))
        assert info[0].iterations == 0 and torch.all(x == 0)
        # x0 already the solution
        xt = uniform_vector(A.n, 1)
        b = A.to_scipy() @ xt
        x, info = pre.solve(_t(b), x=_t(xt), rtol=1e-8)
        assert info[0].iterations == 0
        # maxit reached
        x, info = pre.solve(_t(b), restart=5, maxit=3, rtol=1e-15)
        assert info[0].status == 1 and info[0].iterations == 3
        ref = oracle.gmres(A, b, ("sait64", *_factors(A, 1e-2, 3)[2:]), restart=5, maxit=3, rtol=1e-15)
        assert abs(info[0].true_relres - ref["relres"]) <= 1e-6 * ref["relres"]
        # restart 1
        x, info = pre.solve(_t(b), restart=1, rtol=1e-6, maxit=5000)
        assert info[0].status == 0 and info[0].true_relres <= 1e-6
        with pytest.raises(SaitError):
            pre.solve(_t(b), restart=0)
    finally:
        pre.close()


def test_adjoint_and_gradient():
    print("[test_adjoint_and_gradient]", flush=True)
    A, kap = grf_diffusion2d(24, seed=5)
    L, U, ML, MU = _factors(A, 1e-2, 3)
    b = np.ones(A.n)
    g = uniform_vector(A.n, 3)
    pre = SaitPreconditioner(A, m=3, tau=1e-2, build_transpose=1)
    try:
        lam, info = pre.solve(_t(g), transpose=True, restart=30, rtol=1e-12, flexible=True)
        ref = oracle.gmres(oracle.transpose(A), g, ("sait64", oracle.transpose(MU), oracle.transpose(ML)),
                           restart=30, rtol=1e-12, flexible=True)
        assert info[0].status == 0
        assert abs(info[0].iterations - ref["iters"]) <= 1
        lam_np = lam.cpu().numpy()
        assert np.linalg.norm(lam_np - ref["x"]) <= 1e-9 * np.linalg.norm(ref["x"])
        x = uniform_vector(A.n, 4)
        gv = pre.grad_values(_t(lam_np), _t(x)).cpu().numpy()
        np.testing.assert_array_equal(gv, oracle.grad_values(A, lam_np, x))
    finally:
        pre.close()


def test_autograd_finite_differences():
    # C5 structure at 32^2: loss = ||x - x_t||^2, x = A(vals)^-1 b; gradients
    # from the adjoint FGMRES against central differences of the loss
    # evaluated with the oracle's sparse direct path (scipy splu), 16 unit
    # directions, h = 1e-6, agreement 1e-6.
    print("[test_autograd_finite_differences]", flush=True)
    import scipy.sparse.linalg as spla

    c = config("c5", small=True)
    A, At_ = c["A"], c["A_target"]
    b = c["b"]
    xt = spla.spsolve(At_.to_scipy().tocsc(), b)
    pre = SaitPreconditioner(A, m=3, tau=1e-2, build_transpose=1)
    try:
        vals = _t(A.v).requires_grad_(True)
        bt = _t(b).requires_grad_(True)
        x = sait_solve_autograd(vals, bt, pre, restart=30, rtol=1e-13)
        loss = ((x - _t(xt)) ** 2).sum()
        loss.backward()
        gA = vals.grad.cpu().numpy()
        gb = bt.grad.cpu().numpy()

        def f(v, bb):
            M = sp.csr_matrix((v, A.ci, A.rp), shape=(A.n, A.n)).tocsc()
            return float(np.sum((spla.splu(M).solve(bb) - xt) ** 2))

        rng = np.random.default_rng(c["fd_seed"])
        h = 1e-6
        for _ in range(c["fd_dirs"]):
            xi = rng.standard_normal(A.nnz) * np.abs(A.v)
            eta = rng.standard_normal(A.n) * np.abs(b)
            nrm = np.sqrt(xi @ xi + eta @ eta)
            xi, eta = xi / nrm, eta / nrm
            dfd = (f(A.v + h * xi, b + h * eta) - f(A.v - h * xi, b - h * eta)) / (2 * h)
            dan = gA @ xi + gb @ eta
            assert abs(dfd - dan) <= 1e-6 * max(abs(dfd), abs(dan)), (dfd, dan)
    finally:
        pre.close()


def test_autograd_c5_full_size():
    """The differentiable workload at its full size (GRF diffusion 512^2,
    n = 262,144): loss = ||x - x_t||^2 with x from FGMRES(30) to 1e-10 and
    gradients from the adjoint FGMRES on A^T with the transposed SAIT factors
    (both converged).
    (1) Every entry against the FP64 adjoint gradient formed from sparse
    direct solves (scipy splu for x and lambda, the oracle's grad_values for
    A's pattern).  (2) Central differences of the loss (sparse direct solves)
    on 16 seeded unit directions, agreement 1e-6.  At this size the loss is
    ~6e9 and the rounding of the direct solves makes the h = 1e-6 quotient
    itself wrong by ~4e-6 (it is 4e-8 at h = 1e-4, measured against the
    exact directional derivative), so the step here is 1e-4."""
    print("[test_autograd_c5_full_size] setup", flush=True)
    import scipy.sparse.linalg as spla

    c = config("c5")
    A, At_, b = c["A"], c["A_target"], c["b"]
    lu_opts = dict(permc_spec="MMD_AT_PLUS_A")
    xt = spla.splu(At_.to_scipy().tocsc(), **lu_opts).solve(b)
    pre = SaitPreconditioner(A, m=c["m"], tau=c["tau"], build_transpose=1)
    try:
        vals = _t(A.v).requires_grad_(True)
        bt = _t(b).requires_grad_(True)
        x = sait_solve_autograd(vals, bt, pre, restart=c["restart"], rtol=c["rtol"])
        loss = ((x - _t(xt)) ** 2).sum()
        loss.backward()
        gA = vals.grad.cpu().numpy()
        gb = bt.grad.cpu().numpy()
        assert pre.last_forward_info.status == 0 and pre.last_adjoint_info.status == 0
    finally:
        pre.close()

    lu = spla.splu(A.to_scipy().tocsc(), **lu_opts)
    xd = lu.solve(b)
    lam = lu.solve(2 * (xd - xt), trans="T")
    gA_ref = oracle.grad_values(A, lam, xd)
    print(f"[test_autograd_c5_full_size] gradient vs direct adjoint: "
          f"{np.max(np.abs(gA - gA_ref)) / np.max(np.abs(gA_ref)):.3e} (A), "
          f"{np.max(np.abs(gb - lam)) / np.max(np.abs(lam)):.3e} (b)", flush=True)
    assert np.max(np.abs(gA - gA_ref)) <= 1e-6 * np.max(np.abs(gA_ref))
    assert np.max(np.abs(gb - lam)) <= 1e-6 * np.max(np.abs(lam))

    def f(v, bb):
        M = sp.csr_matrix((v, A.ci, A.rp), shape=(A.n, A.n)).tocsc()
        return float(np.sum((spla.splu(M, **lu_opts).solve(bb) - xt) ** 2))

    rng = np.random.default_rng(c["fd_seed"])
    h = 1e-4
    for d in range(c["fd_dirs"]):
        xi = rng.standard_normal(A.nnz) * np.abs(A.v)
        eta = rng.standard_normal(A.n) * np.abs(b)
        nrm = np.sqrt(xi @ xi + eta @ eta)
        xi, eta = xi / nrm, eta / nrm
        dfd = (f(A.v + h * xi, b + h * eta) - f(A.v - h * xi, b - h * eta)) / (2 * h)
        dan = gA @ xi + gb @ eta
        print(f"[test_autograd_c5_full_size] direction {d}: fd {dfd:.10e} adjoint {dan:.10e}", flush=True)
        assert abs(dfd - dan) <= 1e-6 * max(abs(dfd), abs(dan)), (d, dfd, dan)


def test_c3_full_size():
    # the headline workload at full size (3D Poisson 128^3, n = 2,097,152,
    # ILU(0) + SAIT_Thr(1e-3, 3)): factors bit for bit, the FP64 apply in the
    # autotuned launch shape the bench times bit for bit (sliced ELL) or
    # within the wavefront bound, and FGMRES(40) to a 1e-10 true residual in
    # the oracle's iteration count; FP32 / BF16 factors within 2 steps of it
    print("[test_c3_full_size] building", flush=True)
    c = config("c3")
    A = c["A"]
    L, U = oracle.ilu0(A)
    ML, MU = oracle.sait_factors(L, U, c["m"], tau=c["tau"])
    pre = SaitPreconditioner(A, m=c["m"], tau=c["tau"])
    try:
        for which, ref in (("ML", ML), ("MU", MU)):
            rp, ci, v, _ = pre.export(which)
            np.testing.assert_array_equal(rp, ref.rp)
            np.testing.assert_array_equal(ci, ref.ci)
            np.testing.assert_array_equal(v, ref.v)
        lanes = pre.autotune()
        print(f"[test_c3_full_size] apply shapes {lanes}", flush=True)
        r = uniform_vector(A.n, 11)
        z = pre.apply(_t(r)).cpu().numpy()
        zr = oracle.apply(ML, MU, r)
        if all(x in (-64, -65, -8, -16) for x in lanes):
            np.testing.assert_array_equal(z, zr)
        else:
            assert np.linalg.norm(z - zr) <= 1e-12 * np.linalg.norm(zr)
        print("[test_c3_full_size] solving", flush=True)
        b = _t(c["b"])
        x, (info,) = pre.solve(b, restart=c["restart"], rtol=c["rtol"], flexible=True)
        ref = oracle.gmres(A, c["b"], ("sait64", ML, MU), restart=c["restart"], rtol=c["rtol"], flexible=True)
        assert info.status == 0 and info.true_relres <= c["rtol"], info
        assert abs(info.iterations - ref["iters"]) <= 1, (info.iterations, ref["iters"])
    finally:
        pre.close()
    for prec in ("f32", "bf16"):
        p2 = SaitPreconditioner(A, m=c["m"], tau=c["tau"], precision=prec)
        try:
            x, (i2,) = p2.solve(b, restart=c["restart"], rtol=c["rtol"], flexible=True)
            assert i2.status == 0 and i2.true_relres <= c["rtol"], (prec, i2)
            assert abs(i2.iterations - ref["iters"]) <= 2, (prec, i2.iterations, ref["iters"])
        finally:
            p2.close()


def test_c2_full_size():
    # 2D upwind convection-diffusion 1024^2 with ILUT(1e-3, 10) +
    # SAIT_Thr(1e-3, 4) (n = 1,048,576): factors bit for bit, the autotuned
    # FP64 apply bit for bit (or within the wavefront bound), GMRES(50) to
    # 1e-8 within one step of the oracle
    print("[test_c2_full_size] building", flush=True)
    c = config("c2")
    A = c["A"]
    L, U = oracle.ilut(A, c["ilut_tau"], c["ilut_fill"])
    ML, MU = oracle.sait_factors(L, U, c["m"], tau=c["tau"])
    pre = SaitPreconditioner(A, m=c["m"], tau=c["tau"], ilu_kind="ilut", ilut_tau=c["ilut_tau"],
                             ilut_fill=c["ilut_fill"])
    try:
        for which, ref in (("ML", ML), ("MU", MU)):
            rp, ci, v, _ = pre.export(which)
            np.testing.assert_array_equal(rp, ref.rp)
            np.testing.assert_array_equal(ci, ref.ci)
            np.testing.assert_array_equal(v, ref.v)
        lanes = pre.autotune()
        r = uniform_vector(A.n, 12)
        z = pre.apply(_t(r)).cpu().numpy()
        zr = oracle.apply(ML, MU, r)
        if all(x in (-64, -65, -8, -16) for x in lanes):
            np.testing.assert_array_equal(z, zr)
        else:
            assert np.linalg.norm(z - zr) <= 1e-12 * np.linalg.norm(zr)
        x, (info,) = pre.solve(_t(c["b"]), restart=c["restart"], rtol=c["rtol"])
        ref = oracle.gmres(A, c["b"], ("sait64", ML, MU), restart=c["restart"], rtol=c["rtol"])
        assert info.status == 0 and info.true_relres <= c["rtol"], info
        assert abs(info.iterations - ref["iters"]) <= 1, (info.iterations, ref["iters"])
    finally:
        pre.close()
