"""Pins of the oracle's ILU(p) by levels of fill (the "level-1 ILU" of the
paper's experiments, Sec. 4): with p = 0 it is ILU(0) bit for bit; the
level-1 pattern of the 5-point stencil is the stencil plus the two
diagonals at offsets -(s-1) (L) and +(s-1) (U); the product L U equals A on
the kept pattern; a level large enough keeps everything and gives the exact
LU; and the SAIT ratios the paper prints for its level-1 factors at 100^3
are reproduced, for M_L and (built with T~ from the right) M_U alike."""

import json
import os

import numpy as np
import pytest
import scipy.sparse as sp

import oracle
from workloads import Csr, poisson2d, poisson3d, random_diag_dominant

HERE = os.path.dirname(os.path.abspath(__file__))


def test_level0_is_ilu0():
    for A in (poisson3d(7), random_diag_dominant(500, 8, band=60, seed=2)):
        L0, U0 = oracle.ilu0(A)
        Lk, Uk = oracle.iluk(A, 0)
        for X, Y in ((L0, Lk), (U0, Uk)):
            assert np.array_equal(X.rp, Y.rp) and np.array_equal(X.ci, Y.ci) and np.array_equal(X.v, Y.v)


def test_level1_pattern_of_5_point():
    s = 9
    L, U = oracle.iluk(poisson2d(s), 1)
    for i in range(s * s):
        x, y = i % s, i // s
        lw = [i - s] * (y > 0) + [i - s + 1] * (y > 0 and x < s - 1) + [i - 1] * (x > 0) + [i]
        uw = [i] + [i + 1] * (x < s - 1) + [i + s - 1] * (x > 0 and y < s - 1) + [i + s] * (y < s - 1)
        assert list(L.ci[L.rp[i]:L.rp[i + 1]]) == sorted(lw), i
        assert list(U.ci[U.rp[i]:U.rp[i + 1]]) == sorted(uw), i


@pytest.mark.parametrize("p", [1, 2])
def test_product_matches_a_on_kept_pattern(p):
    for A in (poisson3d(8), random_diag_dominant(400, 8, band=50, seed=3)):
        L, U = oracle.iluk(A, p)
        P = (L.to_scipy() @ U.to_scipy()).toarray()
        Ad = A.to_scipy().toarray()
        kept = (L.to_scipy() + U.to_scipy()).toarray() != 0
        pat = np.zeros_like(kept)
        Ls, Us = L.to_scipy().tocoo(), U.to_scipy().tocoo()
        pat[Ls.row, Ls.col] = True
        pat[Us.row, Us.col] = True
        assert np.max(np.abs(P - Ad)[pat]) <= 1e-12 * np.max(np.abs(Ad))
        assert kept.sum() <= pat.sum()


def test_full_level_is_exact_lu():
    A = random_diag_dominant(60, 6, band=None, seed=4)
    L, U = oracle.iluk(A, 60)
    Ad = A.to_scipy().toarray()
    n = A.n
    Lx, Ux = np.eye(n), Ad.copy()
    for k in range(n):                       # Doolittle without pivoting
        for i in range(k + 1, n):
            Lx[i, k] = Ux[i, k] / Ux[k, k]
            Ux[i, k:] -= Lx[i, k] * Ux[k, k:]
    assert np.allclose(L.to_scipy().toarray(), Lx, rtol=0, atol=1e-12)
    assert np.allclose(U.to_scipy().toarray(), np.triu(Ux), rtol=0, atol=1e-12 * np.max(np.abs(Ad)))


@pytest.mark.parametrize("kind,param", [("thr", 0.05), ("thr", 0.02), ("thr", 0.01), ("pat", 1), ("pat", 2)])
def test_paper_level1_ratios(paper_level1, kind, param):
    L, U = paper_level1.L, paper_level1.U
    g = json.load(open(os.path.join(HERE, "golden", "paper_table_runtime_sait.json")))["level1"][kind]
    printed = {q: r for q, m, r in g}[param]
    ML, MU = paper_level1.sait(kind, param)
    assert round(ML.nnz / L.nnz, 2) == printed, (ML.nnz / L.nnz, printed)
    assert round(MU.nnz / U.nnz, 2) == printed, (MU.nnz / U.nnz, printed)
