"""Seeded generators for the matrices and vectors the SAIT path is run on.

Conventions shared by every generator:
  * CSR with int32 ``rp`` (row pointers, n+1) and int32 ``ci`` (column
    indices, sorted and unique within each row) and float64 ``v``;
  * grid unknowns in natural lexicographic order, x fastest;
  * Dirichlet boundary rows eliminated (only interior unknowns);
  * the h^2 factor of finite-difference stencils is dropped: SAIT and GMRES
    are both invariant under a scalar scaling of A;
  * randomness from ``numpy.random.default_rng(seed)``.

The 3D Laplace problem on a 102^3 mesh of the paper's numerical section
(10^6 interior unknowns, 7-point finite differences) is ``poisson3d(100)``.
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp


@dataclass
class Csr:
    """Square CSR matrix: int32 row pointers / columns, float64 values."""

    n: int
    rp: np.ndarray
    ci: np.ndarray
    v: np.ndarray

    @property
    def nnz(self) -> int:
        return int(self.rp[-1])

    def to_scipy(self) -> sp.csr_matrix:
        return sp.csr_matrix((self.v, self.ci, self.rp), shape=(self.n, self.n))

    @staticmethod
    def from_scipy(m) -> "Csr":
        m = sp.csr_matrix(m)
        m.sum_duplicates()
        m.sort_indices()
        return Csr(
            int(m.shape[0]),
            np.ascontiguousarray(m.indptr, dtype=np.int32),
            np.ascontiguousarray(m.indices, dtype=np.int32),
            np.ascontiguousarray(m.data, dtype=np.float64),
        )


def _grid_stencil(dims, diag, neighbours) -> Csr:
    """Assemble a grid operator.

    ``dims``: grid sizes (x fastest).  ``diag``: (n,) diagonal values.
    ``neighbours``: list of (offset tuple, values) where values is a scalar
    or an (n,) array giving A[i, i+offset] for every row i whose neighbour
    lies inside the grid (outside neighbours are Dirichlet and dropped).
    """
    dims = tuple(int(d) for d in dims)
    n = int(np.prod(dims))
    idx = np.arange(n, dtype=np.int64)
    coords = []
    rem = idx.copy()
    for d in dims:
        coords.append(rem % d)
        rem //= d
    strides = np.cumprod((1,) + dims[:-1])
    rows = [idx]
    cols = [idx]
    vals = [np.broadcast_to(np.asarray(diag, dtype=np.float64), (n,))]
    for off, val in neighbours:
        mask = np.ones(n, dtype=bool)
        lin = 0
        for ax, o in enumerate(off):
            if o:
                c = coords[ax] + o
                mask &= (c >= 0) & (c < dims[ax])
                lin += o * int(strides[ax])
        r = idx[mask]
        vv = np.broadcast_to(np.asarray(val, dtype=np.float64), (n,))[mask]
        rows.append(r)
        cols.append(r + lin)
        vals.append(vv)
    m = sp.coo_matrix(
        (np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(n, n)
    ).tocsr()
    return Csr.from_scipy(m)


def poisson2d(s: int) -> Csr:
    """5-point Laplacian [-1; -1 4 -1; -1] on an s x s interior grid."""
    nb = [((dx, dy), -1.0) for dx, dy in ((-1, 0), (1, 0), (0, -1), (0, 1))]
    return _grid_stencil((s, s), 4.0, nb)


def poisson3d(s: int) -> Csr:
    """7-point Laplacian (6 on the diagonal, -1 off) on an s^3 interior grid."""
    nb = []
    for ax in range(3):
        for o in (-1, 1):
            off = [0, 0, 0]
            off[ax] = o
            nb.append((tuple(off), -1.0))
    return _grid_stencil((s, s, s), 6.0, nb)


def convdiff2d_upwind(s: int, peclet: float = 10.0) -> Csr:
    """-Laplace(u) + v.grad(u), v = (1, 1), first-order upwind, mesh Peclet
    number ``peclet`` per direction (|v| h / nu), scaled by h^2/nu:
    diagonal 4 + 2 Pe, west/south -(1 + Pe), east/north -1."""
    pe = float(peclet)
    nb = [((-1, 0), -(1.0 + pe)), ((0, -1), -(1.0 + pe)), ((1, 0), -1.0), ((0, 1), -1.0)]
    return _grid_stencil((s, s), 4.0 + 2.0 * pe, nb)


def aniso2d(s: int, eps: float) -> Csr:
    """Anisotropic diffusion -eps u_xx - u_yy: diagonal 2 eps + 2,
    x-neighbours -eps, y-neighbours -1."""
    e = float(eps)
    nb = [((-1, 0), -e), ((1, 0), -e), ((0, -1), -1.0), ((0, 1), -1.0)]
    return _grid_stencil((s, s), 2.0 * e + 2.0, nb)


def block_diag(blocks) -> tuple[Csr, np.ndarray]:
    """Concatenate square CSR blocks block-diagonally; returns (A, sys_ptr)."""
    sys_ptr = np.zeros(len(blocks) + 1, dtype=np.int64)
    for k, b in enumerate(blocks):
        sys_ptr[k + 1] = sys_ptr[k] + b.n
    n = int(sys_ptr[-1])
    nnz = sum(b.nnz for b in blocks)
    rp = np.zeros(n + 1, dtype=np.int64)
    ci = np.empty(nnz, dtype=np.int32)
    v = np.empty(nnz, dtype=np.float64)
    pos = 0
    for k, b in enumerate(blocks):
        r0 = int(sys_ptr[k])
        rp[r0 + 1 : r0 + b.n + 1] = b.rp[1:].astype(np.int64) + pos
        ci[pos : pos + b.nnz] = b.ci + r0
        v[pos : pos + b.nnz] = b.v
        pos += b.nnz
    if nnz >= 2**31:
        raise ValueError("block-diagonal matrix exceeds int32 nnz")
    return Csr(n, rp.astype(np.int32), ci, v), sys_ptr


def batched_aniso2d(nsys: int = 256, smin: int = 32, smax: int = 512, seed: int = 3):
    """``nsys`` anisotropic systems, sides s ~ U{smin..smax}, log10(eps) ~
    U[-3, 0].  Returns (A block-diagonal, sys_ptr, sides, eps)."""
    rng = np.random.default_rng(seed)
    sides = rng.integers(smin, smax + 1, size=nsys)
    eps = 10.0 ** rng.uniform(-3.0, 0.0, size=nsys)
    blocks = [aniso2d(int(s), float(e)) for s, e in zip(sides, eps)]
    A, sys_ptr = block_diag(blocks)
    return A, sys_ptr, sides, eps


def gaussian_random_field(s: int, length: float = 0.1, variance: float = 1.0, seed: int = 5):
    """Stationary Gaussian field on the s x s cell centres of [0,1]^2 with
    covariance variance * exp(-r^2 / (2 length^2)), sampled exactly by
    circulant embedding on a periodic 2s x 2s torus (Dietrich & Newsam
    1997).  Negative embedding eigenvalues (round-off sized for this
    kernel) are clipped to zero."""
    rng = np.random.default_rng(seed)
    m = 2 * s
    h = 1.0 / s
    d = np.minimum(np.arange(m), m - np.arange(m)) * h
    r2 = d[:, None] ** 2 + d[None, :] ** 2
    c = variance * np.exp(-r2 / (2.0 * length * length))
    lam = np.fft.fft2(c).real
    lam = np.clip(lam, 0.0, None)
    xi = rng.standard_normal((m, m)) + 1j * rng.standard_normal((m, m))
    field = np.fft.fft2(np.sqrt(lam / (m * m)) * xi)
    return np.ascontiguousarray(field.real[:s, :s])


def grf_diffusion2d(s: int = 512, seed: int = 5, kappa_log=None) -> tuple[Csr, np.ndarray]:
    """Cell-centred finite volumes for -div(kappa grad u) on [0,1]^2, s x s
    cells, kappa = exp(g) with g a GRF (length 0.1, variance 1).  Interior
    faces use the harmonic mean of the two cell values; Dirichlet boundary
    faces use 2 kappa (ghost value at distance h/2).  Returns (A, kappa)."""
    g = gaussian_random_field(s, seed=seed) if kappa_log is None else kappa_log
    kap = np.exp(g)  # kap[ix, iy]
    n = s * s
    # flatten with x fastest: index = ix + s*iy  -> use kap.T ravel
    k = kap.T.ravel()  # k[iy*s + ix]
    kx = kap.T  # [iy, ix]
    hm_x = 2.0 * kx[:, 1:] * kx[:, :-1] / (kx[:, 1:] + kx[:, :-1])  # faces between ix, ix+1
    hm_y = 2.0 * kx[1:, :] * kx[:-1, :] / (kx[1:, :] + kx[:-1, :])  # faces between iy, iy+1
    east = np.zeros((s, s))
    west = np.zeros((s, s))
    north = np.zeros((s, s))
    south = np.zeros((s, s))
    east[:, :-1] = hm_x
    west[:, 1:] = hm_x
    north[:-1, :] = hm_y
    south[1:, :] = hm_y
    diag = east + west + north + south
    diag[:, 0] += 2.0 * kx[:, 0]
    diag[:, -1] += 2.0 * kx[:, -1]
    diag[0, :] += 2.0 * kx[0, :]
    diag[-1, :] += 2.0 * kx[-1, :]
    nb = [
        ((-1, 0), -west.ravel()),
        ((1, 0), -east.ravel()),
        ((0, -1), -south.ravel()),
        ((0, 1), -north.ravel()),
    ]
    A = _grid_stencil((s, s), diag.ravel(), nb)
    assert A.n == n
    return A, k


def random_diag_dominant(n: int, k_off: int = 8, band: int | None = 2**14, seed: int = 8) -> Csr:
    """Rows with ``k_off`` off-diagonal entries, values U[-1,1], columns
    uniform within +-band of the row (or over all of [0,n) when band is
    None); duplicates and the diagonal are redrawn away; the diagonal is
    1 + sum |off-diagonals| (strict diagonal dominance)."""
    rng = np.random.default_rng(seed)
    rows = np.repeat(np.arange(n, dtype=np.int64), k_off)
    if band is None:
        cols = rng.integers(0, n, size=n * k_off)
    else:
        cols = rows + rng.integers(-band, band + 1, size=n * k_off)
        cols = np.clip(cols, 0, n - 1)
    vals = rng.uniform(-1.0, 1.0, size=n * k_off)
    keep = cols != rows
    m = sp.coo_matrix((vals[keep], (rows[keep], cols[keep])), shape=(n, n)).tocsr()
    m.sum_duplicates()
    offsum = np.asarray(abs(m).sum(axis=1)).ravel()
    m = (m + sp.diags(1.0 + offsum)).tocsr()
    return Csr.from_scipy(m)


def random_triangular(n: int, density: float, seed: int, lower: bool = True,
                      unit: bool = False, diag_range=(0.5, 2.0)) -> Csr:
    """Random sparse triangular matrix with a nonzero diagonal (signs
    random, magnitudes in ``diag_range``) and off-diagonals U[-1,1]."""
    rng = np.random.default_rng(seed)
    dense = np.zeros((n, n))
    mask = rng.random((n, n)) < density
    vals = rng.uniform(-1.0, 1.0, size=(n, n))
    tri = np.tril(np.ones((n, n), dtype=bool), -1) if lower else np.triu(np.ones((n, n), dtype=bool), 1)
    dense[mask & tri] = vals[mask & tri]
    if unit:
        d = np.ones(n)
    else:
        d = rng.uniform(*diag_range, size=n) * rng.choice([-1.0, 1.0], size=n)
    dense[np.arange(n), np.arange(n)] = d
    return Csr.from_scipy(sp.csr_matrix(dense))


def uniform_vector(n: int, seed: int, lo: float = -1.0, hi: float = 1.0, k: int | None = None):
    rng = np.random.default_rng(seed)
    if k is None:
        return rng.uniform(lo, hi, size=n)
    return rng.uniform(lo, hi, size=(n, k))


def spmv_rhs(A: Csr, x: np.ndarray) -> np.ndarray:
    """b = A x for manufacturing right-hand sides (input synthesis only)."""
    return np.asarray(A.to_scipy() @ x)


def config(name: str, small: bool = False) -> dict:
    """Parameters and inputs of the named workload.

    c1  2D 5-point Poisson 64^2, ILU(0), SAIT(1e-2, 3), GMRES(30), 1e-8, b = A*1
    c2  2D upwind convection-diffusion 1024^2 (Pe 10), ILUT(1e-3, 10),
        SAIT(1e-3, 4), GMRES(50), 1e-8, b = A x_true, x_true ~ U[-1,1] seed 1
    c3  3D 7-point Poisson 128^3, ILU(0), SAIT(1e-3, 3) in f64/f32/bf16,
        FGMRES(40), 1e-10 true residual, b = A x_true (seed 2)
    c4  256 anisotropic 2D systems (s ~ U{32..512}, seed 3), 8 RHS each
        (seed 4), ILU(0) + SAIT(1e-2, 3), GMRES(30), 1e-8
    c5  GRF diffusion 512^2 (seed 5), ILU(0) + SAIT(1e-2, 3), FGMRES(30),
        1e-10 (1e-12 at the small size), f = 1, target from a perturbed kappa
        (seed 6)

    ``small=True`` shrinks the grid so the CPU oracle finishes in seconds
    while the structure (stencil, parameters) is unchanged.
    """
    name = name.lower()
    if name == "c1":
        A = poisson2d(16 if small else 64)
        b = spmv_rhs(A, np.ones(A.n))
        return dict(A=A, b=b, ilu="ilu0", m=3, tau=1e-2, restart=30, rtol=1e-8, flexible=False)
    if name == "c2":
        A = convdiff2d_upwind(64 if small else 1024, 10.0)
        xt = uniform_vector(A.n, 1)
        return dict(A=A, b=spmv_rhs(A, xt), x_true=xt, ilu="ilut", ilut_tau=1e-3, ilut_fill=10,
                    m=4, tau=1e-3, restart=50, rtol=1e-8, flexible=False)
    if name == "c3":
        A = poisson3d(24 if small else 128)
        xt = uniform_vector(A.n, 2)
        return dict(A=A, b=spmv_rhs(A, xt), x_true=xt, ilu="ilu0", m=3, tau=1e-3, restart=40,
                    rtol=1e-10, flexible=True)
    if name == "c4":
        if small:
            A, sys_ptr, sides, eps = batched_aniso2d(nsys=8, smin=8, smax=24, seed=3)
        else:
            A, sys_ptr, sides, eps = batched_aniso2d(seed=3)
        B = uniform_vector(A.n, 4, k=8)
        return dict(A=A, B=B, sys_ptr=sys_ptr, sides=sides, eps=eps, ilu="ilu0", m=3, tau=1e-2,
                    restart=30, rtol=1e-8, flexible=False, nrhs=8)
    if name == "c5":
        s = 32 if small else 512
        A, kap = grf_diffusion2d(s, seed=5)
        gp = gaussian_random_field(s, seed=6)
        g = gaussian_random_field(s, seed=5)
        A_t, _ = grf_diffusion2d(s, kappa_log=g + 0.1 * gp)
        # the FP64 true-residual floor of the 512^2 problem is ~8e-12, so the
        # full size solves to 1e-10
        return dict(A=A, A_target=A_t, b=np.ones(A.n), ilu="ilu0", m=3, tau=1e-2, restart=30,
                    rtol=1e-12 if small else 1e-10, flexible=True, fd_seed=7, fd_dirs=16)
    if name in ("rdd-b", "rdd-s"):
        n = 2**14 if small else 2**22
        A = random_diag_dominant(n, 8, band=(2**10 if small else 2**14) if name == "rdd-b" else None, seed=8)
        xt = uniform_vector(A.n, 9)
        return dict(A=A, b=spmv_rhs(A, xt), x_true=xt, ilu="ilu0", m=3, tau=1e-2)
    raise KeyError(name)
