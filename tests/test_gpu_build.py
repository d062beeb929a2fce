"""GPU parity of the SAIT construction against the CPU oracle.

The device builds M_L, M_U with the same summation order as the oracle
(products in increasing l, explicitly rounded), so patterns must be
identical and values agree to 1e-12 relative (bitwise in practice); the
binary32 / bfloat16 stored values must equal the oracle's roundings bit
for bit.  Host ILU factors of the library must equal the oracle's.
"""

import numpy as np
import pytest
import scipy.sparse as sp

import oracle
from paper_2106_12836_amd import SaitError, SaitPreconditioner, sait_debug_step
from workloads import (Csr, aniso2d, config, convdiff2d_upwind, poisson2d, poisson3d, random_diag_dominant,
                       random_triangular)

pytestmark = pytest.mark.gpu

RTOL = 1e-12


def _cmp_csr(rp, ci, v, ref: Csr, what):
    np.testing.assert_array_equal(rp, ref.rp, err_msg=f"{what}: row pointers")
    np.testing.assert_array_equal(ci, ref.ci, err_msg=f"{what}: columns")
    scale = np.maximum(np.abs(ref.v), 1e-300)
    err = np.abs(v - ref.v) / scale
    assert err.max(initial=0.0) <= RTOL, f"{what}: max rel err {err.max()}"


def _oracle_factors(A, ilu, m, tau, cap=0, p=-1, ilut=(1e-3, 10), level=1, upper_side="right", sweeps=3):
    if ilu == "ilu0":
        L, U = oracle.ilu0(A)
    elif ilu == "iluk":
        L, U = oracle.iluk(A, level)
    elif ilu == "parilu":
        L, U = oracle.parilu(A, sweeps, level)
    elif ilu == "paric":
        L, U = oracle.paric(A, sweeps, level)
    else:
        L, U = oracle.ilut(A, *ilut)
    if p >= 0:
        return (L, U, *oracle.sait_factors(L, U, m, p=p, upper_side=upper_side))
    return (L, U, *oracle.sait_factors(L, U, m, tau=tau, cap=cap, upper_side=upper_side))


CASES = [
    ("c1-small", lambda: config("c1", small=True)["A"], dict(m=3, tau=1e-2)),
    ("c1", lambda: config("c1")["A"], dict(m=3, tau=1e-2)),
    ("c3-small", lambda: config("c3", small=True)["A"], dict(m=3, tau=1e-3)),
    ("poisson3d-9-tau0-m6", lambda: poisson3d(9), dict(m=6, tau=0.0)),
    ("rdd-ragged", lambda: random_diag_dominant(3001, 8, band=300, seed=3), dict(m=3, tau=1e-2)),
    ("rdd-wide", lambda: random_diag_dominant(2000, 8, band=None, seed=4), dict(m=2, tau=0.0)),
    ("convdiff-ilut", lambda: convdiff2d_upwind(40, 10.0), dict(m=4, tau=1e-3, ilu_kind="ilut")),
    ("poisson3d-ilu1", lambda: poisson3d(10), dict(m=10, tau=0.02, ilu_kind="iluk", ilu_level=1)),
    ("rdd-ilu2", lambda: random_diag_dominant(1500, 8, band=120, seed=6), dict(m=3, tau=1e-2, ilu_kind="iluk",
                                                                                ilu_level=2)),
    ("p3d-parilu3", lambda: poisson3d(9), dict(m=3, tau=1e-2, ilu_kind="parilu", ilu_level=0, parilu_sweeps=3)),
    ("rdd-parilu0", lambda: random_diag_dominant(2000, 8, band=150, seed=11), dict(m=3, tau=1e-2, ilu_kind="parilu",
                                                                                  ilu_level=0, parilu_sweeps=0)),
    ("convdiff-parilu-l1", lambda: convdiff2d_upwind(30, 10.0), dict(m=4, tau=1e-3, ilu_kind="parilu", ilu_level=1,
                                                                      parilu_sweeps=2)),
    ("p3d-paric1", lambda: poisson3d(9), dict(m=4, tau=1e-2, ilu_kind="paric", ilu_level=0, parilu_sweeps=1)),
    ("p2d-paric-l1", lambda: poisson2d(24), dict(m=3, tau=1e-2, ilu_kind="paric", ilu_level=1, parilu_sweeps=2)),
    ("aniso-paric0", lambda: aniso2d(30, 0.05), dict(m=3, tau=1e-2, ilu_kind="paric", ilu_level=0, parilu_sweeps=0)),
    ("cap5", lambda: poisson3d(7), dict(m=4, tau=0.0, max_nnz_row=5)),
    ("rdd-cap6", lambda: random_diag_dominant(1200, 8, band=90, seed=8), dict(m=3, tau=1e-3, max_nnz_row=6)),
    ("pat2", lambda: poisson3d(8), dict(m=3, tau=0.0, pattern_p=2)),
    ("rdd-upper-left", lambda: random_diag_dominant(2500, 8, band=200, seed=9), dict(m=3, tau=1e-2,
                                                                                     upper_side="left")),
    ("rdd-pat2-upper-left", lambda: random_diag_dominant(900, 6, band=60, seed=10), dict(m=3, tau=0.0, pattern_p=2,
                                                                                         upper_side="left")),
    ("m0", lambda: poisson2d(9), dict(m=0, tau=0.1)),
    ("n1", lambda: Csr(1, np.array([0, 1], np.int32), np.array([0], np.int32), np.array([3.0])), dict(m=2, tau=0.1)),
    ("n1-parilu", lambda: Csr(1, np.array([0, 1], np.int32), np.array([0], np.int32), np.array([3.0])),
     dict(m=2, tau=0.1, ilu_kind="parilu", ilu_level=0, parilu_sweeps=2)),
    ("n1-paric", lambda: Csr(1, np.array([0, 1], np.int32), np.array([0], np.int32), np.array([3.0])),
     dict(m=2, tau=0.1, ilu_kind="paric", ilu_level=0, parilu_sweeps=2)),
]


@pytest.mark.parametrize("name,maker,opts", CASES, ids=[c[0] for c in CASES])
def test_factors_match_oracle(name, maker, opts):
    print(f"[test_factors_match_oracle] {name}", flush=True)
    A = maker()
    ilu = opts.get("ilu_kind", "ilu0")
    L, U, ML, MU = _oracle_factors(A, ilu, opts["m"], opts["tau"], opts.get("max_nnz_row", 0),
                                   opts.get("pattern_p", -1), level=opts.get("ilu_level", 1),
                                   upper_side=opts.get("upper_side", "right"), sweeps=opts.get("parilu_sweeps", 3))
    pre = SaitPreconditioner(A, **opts)
    try:
        for which, ref in (("L", L), ("U", U)):
            rp, ci, v = pre.export(which)
            np.testing.assert_array_equal(rp, ref.rp)
            np.testing.assert_array_equal(ci, ref.ci)
            np.testing.assert_array_equal(v, ref.v)  # same operations in the same order
        for which, ref in (("ML", ML), ("MU", MU)):
            rp, ci, v, _ = pre.export(which)
            _cmp_csr(rp, ci, v, ref, which)
        q = pre.query()
        assert q["nnz_ML"] == ML.nnz and q["nnz_MU"] == MU.nnz
        assert abs(q["ratio_L"] - ML.nnz / L.nnz) < 1e-15
    finally:
        pre.close()


@pytest.mark.parametrize("prec", ["f32", "bf16"])
def test_stored_values_bit_exact(prec):
    print(f"[test_stored_values_bit_exact] {prec}", flush=True)
    A = config("c3", small=True)["A"]
    L, U, ML, MU = _oracle_factors(A, "ilu0", 3, 1e-3)
    pre = SaitPreconditioner(A, m=3, tau=1e-3, precision=prec)
    try:
        for which, ref in (("ML", ML), ("MU", MU)):
            rp, ci, v, stored = pre.export(which)
            want = oracle.round_f32(ref.v) if prec == "f32" else oracle.round_bf16(ref.v)
            np.testing.assert_array_equal(stored.view(want.dtype), want)
    finally:
        pre.close()


def test_dense_rows_all_tiers():
    # tau = 0 with m = n-1 on a dense-ish triangular matrix: rows reach
    # thousands of candidate products (LDS tiers and the global fallback),
    # and the result must be the exact inverse (Eq. T_inverse).
    for lower in (True, False):
        T = random_triangular(160, 0.5, 11, lower=lower, diag_range=(2.0, 3.0))
        for side in ("left", "right"):
            print(f"[test_dense_rows_all_tiers] lower={lower} side={side}", flush=True)
            # one pass at a time through the debug entry point (T itself as input)
            Mk = oracle.identity(160)
            for k in range(12):
                rp, ci, v = sait_debug_step(160, (T.rp, T.ci, T.v), (Mk.rp, Mk.ci, Mk.v), 0.0, side=side)
                ref = oracle.sait_step(T, Mk, 0.0, side=side)
                _cmp_csr(rp, ci, v, ref, f"pass {k}")
                Mk = ref
        # after 159 passes the scaled series is the exact inverse
        Tinv = np.linalg.inv(T.to_scipy().toarray())
        assert np.abs(oracle.sait_thr(T, 0.0, 159).to_scipy().toarray() - Tinv).max() < 1e-10 * np.abs(Tinv).max()


def test_long_rows_apply():
    # rows longer than one LDS chunk (4088 entries) are processed chunk by
    # chunk; results stay bit-exact with the oracle for every exact shape
    print("[test_long_rows_apply]", flush=True)
    import torch
    from paper_2106_12836_amd import sait_set_apply_lanes
    n = 9000
    rng = np.random.default_rng(5)
    rows = [np.arange(n)]
    cols = [np.arange(n)]
    dense_rows = [4000, 8999]
    for r in dense_rows:
        c = np.arange(r)
        rows.append(np.full(r, r))
        cols.append(c)
    rr = np.concatenate(rows)
    cc = np.concatenate(cols)
    vals = np.where(rr == cc, 4.0, rng.uniform(-1, 1, rr.size) * 1e-3)
    A = Csr.from_scipy(sp.csr_matrix((vals, (rr, cc)), shape=(n, n)))
    L, U, ML, MU = _oracle_factors(A, "ilu0", 1, 0.0)
    assert max(np.diff(ML.rp)) > 4088
    pre = SaitPreconditioner(A, m=1, tau=0.0)
    try:
        r = np.random.default_rng(2).uniform(-1, 1, n)
        zr = oracle.apply(ML, MU, r)
        for shape in (-64, -65, -8, -16):
            sait_set_apply_lanes(pre.handle, shape, shape)
            z = pre.apply(torch.tensor(r, device="cuda:0")).cpu().numpy()
            np.testing.assert_array_equal(z, zr)
    finally:
        pre.close()


@pytest.mark.parametrize("side", ["left", "right"])
@pytest.mark.parametrize("tau,cap", [(0.0, 0), (1e-2, 0), (0.05, 0), (0.0, 4), (1e-3, 7)])
def test_stepwise_harness(tau, cap, side):
    # Each device pass is fed the oracle's previous M (never the reverse).
    print(f"[test_stepwise_harness] tau={tau} cap={cap} side={side}", flush=True)
    A = random_diag_dominant(1500, 8, band=100, seed=21)
    L, U = oracle.ilu0(A)
    for T in (L, U):
        M = oracle.identity(A.n)
        for k in range(4):
            rp, ci, v = sait_debug_step(A.n, (T.rp, T.ci, T.v), (M.rp, M.ci, M.v), tau, cap, side=side)
            ref = oracle.sait_step(T, M, tau, cap, side=side)
            _cmp_csr(rp, ci, v, ref, f"pass {k}")
            M = ref


@pytest.mark.parametrize("side", ["left", "right"])
def test_empty_operand_rows(side):
    # T diagonal (T~ = 0): in M T~ + I every product segment of a row of M is
    # empty, so a row has far more segments than candidates (rows of M up to
    # 2600 entries reach every size tier); the result is the identity.
    print(f"[test_empty_operand_rows] side={side}", flush=True)
    n = 2600
    T = Csr(n, np.arange(n + 1, dtype=np.int32), np.arange(n, dtype=np.int32), np.linspace(1.0, 2.0, n))
    M = Csr.from_scipy(sp.csr_matrix(np.tril(np.random.default_rng(3).uniform(0.5, 1.0, (n, n)))))
    rp, ci, v = sait_debug_step(n, (T.rp, T.ci, T.v), (M.rp, M.ci, M.v), 0.0, side=side)
    ref = oracle.sait_step(T, M, 0.0, side=side)
    assert ref.nnz == n
    _cmp_csr(rp, ci, v, ref, side)


def test_build_errors():
    print("[test_build_errors]", flush=True)
    A = Csr(2, np.array([0, 2, 4], np.int32), np.array([0, 1, 0, 1], np.int32), np.array([0.0, 1.0, 1.0, 2.0]))
    with pytest.raises(SaitError) as e:
        SaitPreconditioner(A)
    assert e.value.status == -2  # zero pivot
    with pytest.raises(SaitError) as e:
        SaitPreconditioner(poisson2d(4), tau=1.0)
    assert e.value.status == -1
    with pytest.raises(SaitError) as e:
        SaitPreconditioner(poisson2d(4), upper_side=2)
    assert e.value.status == -1
    bad = Csr(2, np.array([0, 2, 3], np.int32), np.array([1, 0, 1], np.int32), np.array([1.0, 1.0, 1.0]))
    with pytest.raises(SaitError) as e:
        SaitPreconditioner(bad)
    assert e.value.status == -1  # unsorted columns
    nanA = poisson2d(3)
    nanA.v[0] = np.nan
    with pytest.raises(SaitError) as e:
        SaitPreconditioner(nanA)
    assert e.value.status == -3


@pytest.mark.parametrize("level", [0, 1])
def test_parilu_reaches_the_ilu_factors(level):
    # enough synchronous sweeps on the device give the row-wise ILU(0) /
    # ILU(1) factors bit for bit (the same formula, products in the same order)
    print(f"[test_parilu_reaches_the_ilu_factors] level={level}", flush=True)
    A = random_diag_dominant(400, 6, band=40, seed=12)
    pre = SaitPreconditioner(A, m=2, tau=1e-2, ilu_kind="parilu", ilu_level=level, parilu_sweeps=A.n)
    try:
        L0, U0 = oracle.ilu0(A) if level == 0 else oracle.iluk(A, level)
        for which, ref in (("L", L0), ("U", U0)):
            rp, ci, v = pre.export(which)
            np.testing.assert_array_equal(rp, ref.rp)
            np.testing.assert_array_equal(ci, ref.ci)
            np.testing.assert_array_equal(v, ref.v)
    finally:
        pre.close()


def test_paric_needs_a_symmetric_pattern():
    print("[test_paric_needs_a_symmetric_pattern]", flush=True)
    with pytest.raises(SaitError) as e:
        SaitPreconditioner(random_diag_dominant(300, 6, band=40, seed=13), ilu_kind="paric", ilu_level=0)
    assert e.value.status == -1


def test_parilu_errors():
    print("[test_parilu_errors]", flush=True)
    with pytest.raises(SaitError):
        SaitPreconditioner(poisson2d(5), ilu_kind="parilu", parilu_sweeps=-1)
    A = Csr(2, np.array([0, 2, 4], np.int32), np.array([0, 1, 0, 1], np.int32), np.array([0.0, 1.0, 1.0, 2.0]))
    with pytest.raises(SaitError) as e:
        SaitPreconditioner(A, ilu_kind="parilu", ilu_level=0)
    assert e.value.status == -2
    # a matrix whose sweeps overflow: huge off-diagonals against tiny pivots
    B = Csr(3, np.array([0, 2, 5, 7], np.int32), np.array([0, 1, 0, 1, 2, 1, 2], np.int32),
            np.array([1e-300, 1e300, 1e300, 1e-300, 1e300, 1e300, 1e-300]))
    with pytest.raises(SaitError) as e:
        SaitPreconditioner(B, ilu_kind="parilu", ilu_level=0, parilu_sweeps=2)
    assert e.value.status == -3


@pytest.mark.parametrize("kind,sweeps", [("parilu", 3), ("paric", 1)])
def test_device_ilu_full_size(kind, sweeps):
    # the paper's 100^3 matrix (6.94 M entries): device factors bit for bit
    print(f"[test_device_ilu_full_size] {kind} sweeps={sweeps}", flush=True)
    A = poisson3d(100)
    L, U = (oracle.parilu if kind == "parilu" else oracle.paric)(A, sweeps)
    pre = SaitPreconditioner(A, m=0, tau=0.0, ilu_kind=kind, ilu_level=0, parilu_sweeps=sweeps)
    try:
        for which, ref in (("L", L), ("U", U)):
            rp, ci, v = pre.export(which)
            np.testing.assert_array_equal(rp, ref.rp)
            np.testing.assert_array_equal(ci, ref.ci)
            np.testing.assert_array_equal(v, ref.v)
    finally:
        pre.close()
