"""Randomised parity of the SAIT apply z = M_U (M_L r) (Sec. 3.1): seeded
matrices of the workloads' kinds, random ILU (ILU(0), ILU(k), ILUT), m,
tau, side of the upper recursion, storage precision, kernel shape and
number of right-hand sides, against the oracle's apply of the oracle's
factors.

Exact shapes (sliced ELL, LDS-staged CSR; the sliced block kernel for 2-5
and 8 right-hand sides) sum the rounded products in column order, as the
oracle does: equal bit for bit, in FP64 and with binary32 accumulation.
The wavefront kernel (FMA, tree reduction) and other block widths: within
4 K u |M_U| (|M_L| |r|) (FP64, K = longest row + 1) or the binary32 bound
2 K u32 / (1 - K u32) of the products of the stored values."""

import numpy as np
import pytest
import scipy.sparse as sp

import oracle
from paper_2106_12836_amd import SaitPreconditioner, sait_set_apply_lanes
from workloads import aniso2d, convdiff2d_upwind, poisson2d, poisson3d, random_diag_dominant, uniform_vector

pytestmark = pytest.mark.gpu


def _t(x):
    import torch

    return torch.tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda:0")


def _sp(M, vals=None):
    return sp.csr_matrix((M.v if vals is None else vals, M.ci, M.rp), shape=(M.n, M.n))


def _case(seed):
    rng = np.random.default_rng(6000 + seed)
    kind = str(rng.choice(["rdd", "rdd", "convdiff", "aniso", "poisson2d", "poisson3d"]))
    if kind == "rdd":
        n = int(rng.integers(64, 9000))
        band = None if rng.random() < 0.3 else int(rng.integers(4, max(5, n // 4)))
        A = random_diag_dominant(n, int(rng.integers(1, 14)), band=band, seed=seed)
    elif kind == "convdiff":
        A = convdiff2d_upwind(int(rng.integers(8, 90)), float(rng.choice([0.5, 10.0])))
    elif kind == "aniso":
        A = aniso2d(int(rng.integers(8, 90)), float(rng.choice([0.01, 0.1, 1.0])))
    elif kind == "poisson2d":
        A = poisson2d(int(rng.integers(8, 90)))
    else:
        A = poisson3d(int(rng.integers(4, 20)))
    o = dict(m=int(rng.integers(0, 5)), tau=float(rng.choice([0.0, 1e-3, 1e-2, 5e-2])),
             upper_side=str(rng.choice(["left", "right"])), precision=str(rng.choice(["f64", "f64", "f32", "bf16"])),
             ilu_kind=str(rng.choice(["ilu0", "ilu0", "iluk", "ilut"])))
    if o["ilu_kind"] == "iluk":
        o["ilu_level"] = int(rng.integers(1, 3))
    elif o["ilu_kind"] == "ilut":
        o["ilut_tau"], o["ilut_fill"] = 1e-3, int(rng.integers(3, 12))
    nrhs = int(rng.choice([1, 1, 1, 2, 3, 4, 5, 8, 11]))
    shape = int(rng.choice([-64, -65, -8, -16, 1, 2, 4, 8, 16, 32, 64]))
    return kind, A, o, nrhs, shape


@pytest.mark.parametrize("seed", range(24))
def test_random_apply_matches_oracle(seed):
    kind, A, o, nrhs, shape = _case(seed)
    print(f"[test_random_apply_matches_oracle] seed={seed} {kind} n={A.n} {o} nrhs={nrhs} shape={shape}", flush=True)
    if o["ilu_kind"] == "iluk":
        L, U = oracle.iluk(A, o["ilu_level"])
    elif o["ilu_kind"] == "ilut":
        L, U = oracle.ilut(A, o["ilut_tau"], o["ilut_fill"])
    else:
        L, U = oracle.ilu0(A)
    ML, MU = oracle.sait_factors(L, U, o["m"], tau=o["tau"], upper_side=o["upper_side"])
    R = uniform_vector(A.n, 40 + seed, k=nrhs)
    exact = shape < 0 and nrhs in (1, 2, 3, 4, 5, 8)
    K = max(np.diff(ML.rp).max(), np.diff(MU.rp).max()) + 1
    pre = SaitPreconditioner(A, build_transpose=1 if o["precision"] == "f64" else 0, **o)
    try:
        sait_set_apply_lanes(pre.handle, shape, shape)
        Z = pre.apply(_t(R if nrhs > 1 else R[:, 0])).cpu().numpy().reshape(A.n, nrhs)
        if o["precision"] == "f64":
            for k in range(nrhs):
                zr = oracle.apply(ML, MU, R[:, k])
                if exact:
                    np.testing.assert_array_equal(Z[:, k], zr)
                bound = 4 * K * 2.0 ** -53 * (abs(_sp(MU)) @ (abs(_sp(ML)) @ np.abs(R[:, k])))
                assert np.all(np.abs(Z[:, k] - zr) <= bound + 1e-300)
            if nrhs == 1:
                zt = pre.apply(_t(R[:, 0]), transpose=True).cpu().numpy()
                ztr = oracle.apply(oracle.transpose(MU), oracle.transpose(ML), R[:, 0])
                assert np.linalg.norm(zt - ztr) <= 1e-12 * np.linalg.norm(ztr)
        else:
            f1 = oracle.storage_values(ML, o["precision"]).astype(np.float64)
            f2 = oracle.storage_values(MU, o["precision"]).astype(np.float64)
            u = 2.0 ** -24
            gam = K * u / (1 - K * u)
            for k in range(nrhs):
                r32 = R[:, k].astype(np.float32).astype(np.float64)
                zstar = _sp(MU, f2) @ (_sp(ML, f1) @ r32)
                bound = 2 * gam * (abs(_sp(MU, f2)) @ (abs(_sp(ML, f1)) @ np.abs(r32))) * (1 + 4 * u)
                assert np.all(np.abs(Z[:, k] - zstar) <= bound)
                if exact:
                    zo = oracle.apply_f32acc(ML, f1.astype(np.float32), MU, f2.astype(np.float32), R[:, k])
                    np.testing.assert_array_equal(Z[:, k], zo)
    finally:
        pre.close()


@pytest.mark.parametrize("seed", range(16))
def test_tiny_random_build_apply_solve(seed):
    # n from 1 to 130 (one partial slice, exactly 64 / 128 rows, one row
    # past a slice): factors bit for bit, the apply on every exact shape bit
    # for bit, GMRES within one iteration of the oracle
    rng = np.random.default_rng(9000 + seed)
    n = int(rng.choice([1, 2, 3, 63, 64, 65, 127, 128, 129, int(rng.integers(4, 130))]))
    A = random_diag_dominant(n, int(rng.integers(1, 6)), band=None, seed=seed)
    m, tau = int(rng.integers(0, 5)), float(rng.choice([0.0, 1e-2, 5e-2]))
    side = str(rng.choice(["left", "right"]))
    print(f"[test_tiny_random_build_apply_solve] seed={seed} n={n} nnz={A.nnz} m={m} tau={tau} side={side}",
          flush=True)
    L, U = oracle.ilu0(A)
    ML, MU = oracle.sait_factors(L, U, m, tau=tau, upper_side=side)
    r = uniform_vector(n, 60 + seed)
    pre = SaitPreconditioner(A, m=m, tau=tau, upper_side=side)
    try:
        for which, ref in (("ML", ML), ("MU", MU)):
            rp, ci, v, _ = pre.export(which)
            np.testing.assert_array_equal(rp, ref.rp)
            np.testing.assert_array_equal(ci, ref.ci)
            np.testing.assert_array_equal(v.view(np.uint64), ref.v.view(np.uint64))
        zr = oracle.apply(ML, MU, r)
        for shape in (-64, -65, -8, -16):
            sait_set_apply_lanes(pre.handle, shape, shape)
            np.testing.assert_array_equal(pre.apply(_t(r)).cpu().numpy(), zr)
        sait_set_apply_lanes(pre.handle, -64, -64)
        b = A.to_scipy() @ uniform_vector(n, 80 + seed)
        ref = oracle.gmres(A, b, ("sait64", ML, MU), restart=10, rtol=1e-10)
        x, (info,) = pre.solve(_t(b), restart=10, rtol=1e-10)
        assert info.status == 0 and ref["status"] == 0
        assert abs(info.iterations - ref["iters"]) <= 1, (info.iterations, ref["iters"])
        assert np.linalg.norm(b - A.to_scipy() @ x.cpu().numpy()) <= 1e-10 * np.linalg.norm(b) * (1 + 1e-7)
    finally:
        pre.close()
