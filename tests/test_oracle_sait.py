"""Pins of the oracle's SAIT construction (Sec. 2-3, Alg. 1-3, Appendix A).

What fixes the oracle here, independently of its own code:
  * the exact inverse from a dense LAPACK inverse (Eq. T_inverse),
  * nilpotency of the strictly triangular iteration matrix: the series is
    exact from the level-schedule depth on and not before,
  * Jacobi sweeps from a zero start (Eq. Jacobi_iter / M_poly),
  * closed forms (bidiagonal matrices, m = 0, m = 1, large tau, scaling),
  * the inverse-pattern of the 5-point ILU(0) factor,
  * block-diagonal invariance,
  * the ratios the paper prints for the 3D Laplace problem (golden fixture).
"""

import json
import os

import numpy as np
import pytest
import scipy.sparse as sp

from workloads import Csr, block_diag, poisson2d, poisson3d, random_triangular

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _dense(M: Csr):
    return M.to_scipy().toarray()


def _depth(T: Csr):
    """Level-schedule depth of a triangular matrix: length of the longest
    dependency chain (number of levels)."""
    Ts = T.to_scipy().tocsr()
    n = T.n
    lower = sp.triu(Ts, 1).nnz == 0
    lev = np.zeros(n, dtype=int)
    order = range(n) if lower else range(n - 1, -1, -1)
    for i in order:
        cols = Ts.indices[Ts.indptr[i]:Ts.indptr[i + 1]]
        deps = cols[cols < i] if lower else cols[cols > i]
        lev[i] = 1 + (lev[deps].max() if len(deps) else 0)
    return int(lev.max())


@pytest.mark.parametrize("n,density,lower,unit,seed", [
    (12, 0.5, True, False, 0), (20, 0.3, False, False, 1), (33, 0.2, True, True, 2),
    (40, 0.15, False, True, 3), (1, 1.0, True, False, 4), (2, 1.0, False, False, 5)])
def test_series_exact_inverse(orc, n, density, lower, unit, seed):
    # Eq. T_inverse: with no dropping and m = n-1 the series is T^-1.
    T = random_triangular(n, density, seed, lower=lower, unit=unit)
    M = orc.sait_thr(T, 0.0, max(n - 1, 0))
    Tinv = np.linalg.inv(_dense(T))
    err = np.abs(_dense(M) - Tinv).max() / np.abs(Tinv).max()
    assert err < 1e-12


def test_nilpotency_depth(orc):
    # T~ is strictly triangular, so T~^k = 0 once k reaches the depth of the
    # dependency graph: M_m = T^-1 exactly for m >= depth-1 and not for m = depth-2.
    L, U = orc.ilu0(poisson2d(8))
    for T in (L, U):
        dep = _depth(T)
        assert dep == 2 * 8 - 1
        Tinv = np.linalg.inv(_dense(T))
        ok = _dense(orc.sait_thr(T, 0.0, dep - 1))
        short = _dense(orc.sait_thr(T, 0.0, dep - 2))
        assert np.abs(ok - Tinv).max() < 1e-14
        assert np.abs(short - Tinv).max() > 1e-8


@pytest.mark.parametrize("m", [0, 1, 2, 5])
def test_jacobi_sweeps(orc, m):
    # Eq. Jacobi_iter / M_poly with no dropping: M_m r = x^{m+1}, the
    # (m+1)-th Jacobi iterate for T x = r started from x^0 = 0.
    T = random_triangular(60, 0.1, 7, lower=True)
    r = np.random.default_rng(1).uniform(-1, 1, 60)
    Td = _dense(T)
    D = np.diag(Td)
    x = np.zeros(60)
    for _ in range(m + 1):
        x = ((np.diag(D) - Td) @ x + r) / D
    M = orc.sait_thr(T, 0.0, m)
    np.testing.assert_allclose(M.to_scipy() @ r, x, rtol=1e-13, atol=1e-13)


def test_scaling_invariance(orc):
    # T~ = I - D^-1 T is unchanged by T -> cT, so SAIT(cT) = SAIT(T) / c.
    L, U = orc.ilu0(poisson3d(5))
    for T in (L, U):
        c = 2.5
        Tc = Csr(T.n, T.rp, T.ci, T.v * c)
        M = orc.sait_thr(T, 1e-2, 3)
        Mc = orc.sait_thr(Tc, 1e-2, 3)
        np.testing.assert_array_equal(M.ci, Mc.ci)
        np.testing.assert_allclose(Mc.v, M.v / c, rtol=1e-15)


def test_small_m_closed_forms(orc):
    T = random_triangular(30, 0.3, 9, lower=False, diag_range=(2.0, 3.0))  # |T~_ij| <= 1/2
    Td = _dense(T)
    Dinv = np.diag(1.0 / np.diag(Td))
    # m = 0: M = D^-1
    np.testing.assert_allclose(_dense(orc.sait_thr(T, 0.0, 0)), Dinv, rtol=1e-15)
    # m = 1, tau = 0: M = (I + T~) D^-1 = (2I - D^-1 T) D^-1, pattern of T, ratio exactly 1
    M1 = orc.sait_thr(T, 0.0, 1)
    np.testing.assert_allclose(_dense(M1), (2 * np.eye(30) - Dinv @ Td) @ Dinv, rtol=1e-14, atol=1e-15)
    assert M1.nnz == T.nnz
    np.testing.assert_array_equal(M1.ci, T.ci)
    # tau >= max |T~_ij|: every product is dropped, M = D^-1 for any m
    Tt = np.eye(30) - Dinv @ Td
    M = orc.sait_thr(T, float(np.abs(Tt).max()), 4)
    np.testing.assert_allclose(_dense(M), Dinv, rtol=1e-15)


@pytest.mark.parametrize("c,d,tau,m", [(0.5, 2.0, 0.0, 6), (0.5, 2.0, 0.1, 10), (-0.8, 3.0, 0.3, 8),
                                       (0.9, 1.0, 0.5, 3)])
def test_bidiagonal_closed_form(orc, c, d, tau, m):
    # T = d (I - c S) (S the shift): T~ = c S, M_ij = c^(i-j) / d for
    # 0 <= i-j <= m with |c|^(i-j) > tau (drop is strict: keep iff > tau).
    n = 25
    T = Csr.from_scipy(sp.diags([np.full(n - 1, -c * d), np.full(n, d)], [-1, 0], format="csr"))
    M = _dense(orc.sait_thr(T, tau, m))
    i, j = np.indices((n, n))
    k = i - j
    expect = np.where((k >= 0) & (k <= m) & (np.abs(c) ** np.clip(k, 0, None) > tau),
                      np.power(c, np.clip(k, 0, None)) / d, 0.0)
    np.testing.assert_allclose(M, expect, rtol=1e-14, atol=0)


def test_drop_is_strict(orc):
    # Appendix A keeps abs(M) > tau: an entry equal to tau is dropped.
    n = 5
    T = Csr.from_scipy(sp.diags([np.full(n - 1, -0.5), np.ones(n)], [-1, 0], format="csr"))
    M = orc.sait_thr(T, 0.5, 3)
    assert M.nnz == n
    M = orc.sait_thr(T, np.nextafter(0.5, 0.0), 3)
    assert M.nnz == n + (n - 1)


def test_inverse_pattern_5pt(orc):
    # For the 5-point ILU(0) factor L on an s x s grid, L^-1 is nonzero
    # exactly where x_j <= x_i and y_j <= y_i.
    s = 6
    L, U = orc.ilu0(poisson2d(s))
    M = _dense(orc.sait_thr(L, 0.0, s * s - 1))
    idx = np.arange(s * s)
    x, y = idx % s, idx // s
    expect = (x[None, :] <= x[:, None]) & (y[None, :] <= y[:, None])
    np.testing.assert_array_equal(M != 0, expect)


def test_block_diagonal(orc):
    b1 = random_triangular(15, 0.3, 1)
    b2 = random_triangular(9, 0.5, 2)
    b3 = random_triangular(21, 0.2, 3)
    T, ptr = block_diag([b1, b2, b3])
    M = orc.sait_thr(T, 1e-2, 4)
    Md = _dense(M)
    for blk, (s, e) in zip((b1, b2, b3), zip(ptr[:-1], ptr[1:])):
        np.testing.assert_array_equal(Md[s:e, s:e], _dense(orc.sait_thr(blk, 1e-2, 4)))
    mask = np.zeros_like(Md, dtype=bool)
    for s, e in zip(ptr[:-1], ptr[1:]):
        mask[s:e, s:e] = True
    assert np.all(Md[~mask] == 0)


def test_cap_keeps_largest(orc):
    # One pass with cap K keeps the diagonal plus the K-1 largest magnitudes of
    # the uncapped pass (ties to the smaller column).
    T = random_triangular(60, 0.4, 5, lower=True)
    M0 = orc.sait_thr(T, 0.0, 2)  # some nontrivial previous M (scaled, used as is)
    full = orc.sait_step(T, M0, 0.0, 0)
    K = 4
    capped = orc.sait_step(T, M0, 0.0, K)
    Fs, Cs = full.to_scipy(), capped.to_scipy()
    for i in range(T.n):
        cols = Fs.indices[Fs.indptr[i]:Fs.indptr[i + 1]]
        vals = Fs.data[Fs.indptr[i]:Fs.indptr[i + 1]]
        off = [(-abs(v), c, v) for c, v in zip(cols, vals) if c != i]
        keep = sorted(off)[: K - 1]
        want = sorted([(c, v) for _, c, v in keep] + [(i, Fs[i, i])])
        got = list(zip(Cs.indices[Cs.indptr[i]:Cs.indptr[i + 1]], Cs.data[Cs.indptr[i]:Cs.indptr[i + 1]]))
        assert [c for c, _ in got] == [c for c, _ in want]
        np.testing.assert_array_equal([v for _, v in got], [v for _, v in want])


def test_step_matches_definition(orc):
    # One unscaled pass equals drop(T~ M + I) computed with scipy.
    T = random_triangular(50, 0.2, 8, lower=False)
    M = orc.sait_thr(T, 0.0, 2)
    Td = _dense(T)
    Dinv = np.diag(1.0 / np.diag(Td))
    Tt = np.eye(50) - Dinv @ Td
    np.fill_diagonal(Tt, 0.0)
    W = Tt @ _dense(M) + np.eye(50)
    tau = 0.05
    W[np.abs(W) <= tau] = 0.0
    got = _dense(orc.sait_step(T, M, tau, 0))
    np.testing.assert_allclose(got, W, rtol=1e-13, atol=1e-15)
    assert np.array_equal(got != 0, W != 0)


def test_errors(orc):
    T = random_triangular(10, 0.3, 1)
    for tau in (1.0, -0.1, float("nan")):
        with pytest.raises(orc.OracleError):
            orc.sait_thr(T, tau, 3)
    with pytest.raises(orc.OracleError):
        orc.sait_thr(T, 0.1, -1)
    bad = Csr(T.n, T.rp, T.ci, np.where(T.ci == np.repeat(np.arange(T.n), np.diff(T.rp)), 0.0, T.v))
    with pytest.raises(orc.OracleError) as e:
        orc.sait_thr(bad, 0.1, 2)
    assert e.value.status == orc.E_ZERO_PIVOT


def test_paper_ratios_level0(orc):
    # Table runtime_SAIT (level-0 ILU) and the SAIT_Pat legend ratios of
    # Sec. 4.1, on the 10^6-unknown 3D Laplace problem.
    g = json.load(open(os.path.join(GOLDEN, "paper_table_runtime_sait.json")))
    A = poisson3d(100)
    L, U = orc.ilu0(A)
    tau, m, printed = g["level0"]["thr"][0]
    for T in (L, U):  # both factors give the same ratio on this symmetric stencil
        r = orc.sait_thr(T, tau, m).nnz / T.nnz
        assert round(r, 2) == printed
    for tau, m, printed in g["level0"]["thr"][1:]:
        assert round(orc.sait_thr(L, tau, m).nnz / L.nnz, 2) == printed
    for p, m, printed in g["level0"]["pat"]:
        assert round(orc.sait_pat(L, p, m).nnz / L.nnz, 2) == printed


def test_pattern_variant_equals_power_pattern(orc):
    # Sec. 3: the pattern of T^p equals the pattern of M_{p+1} (no dropping).
    L, U = orc.ilu0(poisson2d(7))
    for T in (L, U):
        Td = _dense(T)
        for p in (1, 2, 3):
            Pp = np.linalg.matrix_power(np.abs(Td), p) != 0
            S = orc.sait_thr(T, 0.0, p)  # p passes = highest power p = M_{p+1}
            assert np.array_equal(_dense(S) != 0, Pp)
            # SAIT_Pat(p, m) never leaves that pattern
            Mp = orc.sait_pat(T, p, 5)
            assert not np.any((_dense(Mp) != 0) & ~Pp)


def test_interior_row_count_without_dropping(orc):
    # 3D 7-point stencil, tau = 0: an interior row of M_m (m passes) holds
    # every column reachable by at most m steps back along x, y or z, i.e.
    # (m+1)(m+2)(m+3)/6 entries (the tau = 0 curve of Sec. 4.1)
    s = 13
    A = poisson3d(s)
    L, U = orc.ilu0(A)
    c = (s // 2) * (1 + s + s * s)  # the centre point
    for m in range(1, 6):
        M = orc.sait_thr(L, 0.0, m)
        assert M.rp[c + 1] - M.rp[c] == (m + 1) * (m + 2) * (m + 3) // 6, m
