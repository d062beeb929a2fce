"""LOBPCG for the k smallest eigenpairs of a symmetric positive definite A,
preconditioned by a symmetric positive definite T ~ A^-1 -- the solver of
the paper's eigenvalue experiment (Sec. 4, eigenvalue problem of Eq.
A_u_f), where T = M_U M_L is applied to the whole block of residuals (two
sparse matrix-matrix products).  Test infrastructure only: it checks the
device solver and is never called by the product path.

The method is Knyazev's locally optimal block preconditioned conjugate
gradient (SIAM J. Sci. Comput. 23 (2001)), written out plainly in FP64:

  X_0 given (n x k); Rayleigh-Ritz on span(X_0) gives theta, X, AX.
  repeat, it = 0, 1, ...:
      R = A X - X diag(theta)                       (block residual)
      stop if ||R_j|| <= tol * |theta_j| for every j   (||X_j|| = 1)
      W = T R                                       (preconditioning)
      S = [X, W, P]  ([X, W] in the first step)     (trial basis)
      Rayleigh-Ritz on span(S): Gram matrices G_A = S^T A S, G_B = S^T S,
          scaled to unit diagonal by D = diag(G_B)^-1/2, G_B = L L^T
          (Cholesky), eigenpairs of L^-1 G_A L^-T; the k smallest give
          theta and the coefficients c = D L^-T V
      X <- S c;  P <- [W, P] c_(W,P)  (the part of the update outside X)
  AX, AW, AP are carried along so that A multiplies only W.

If the scaled G_B of [X, W, P] has a Cholesky pivot L_jj^2 <= PIVOT_P (the
basis is close to dependent), that step is redone without P; if the pivot
of [X, W] falls to PIVOT_MIN the solve stops with status 2.
"""

import numpy as np
import scipy.linalg as sla

# Rayleigh-Ritz on a basis whose scaled Gram matrix has condition number c
# loses about log10(c) digits.  [X, W, P] is accepted only while its
# smallest pivot stays above PIVOT_P: with pivots near 1e-10 the Ritz values
# of a clustered spectrum drifted below the smallest eigenvalue of an SPD
# matrix and the iteration diverged.  [X, W] (and the start block) only has
# to stay above PIVOT_MIN: near convergence W is small and noisy, and a
# stricter bound there would stop the iteration one step short.
PIVOT_MIN = 1e-14
PIVOT_P = 1e-8


def _cholesky_lower(B, pivot_min=PIVOT_MIN):
    """Plain Cholesky B = L L^T (column by column); None when a pivot
    L_jj^2 <= pivot_min."""
    m = B.shape[0]
    L = np.zeros_like(B)
    for j in range(m):
        s = B[j, j] - L[j, :j] @ L[j, :j]
        if not s > pivot_min:
            return None
        L[j, j] = np.sqrt(s)
        for i in range(j + 1, m):
            L[i, j] = (B[i, j] - L[i, :j] @ L[j, :j]) / L[j, j]
    return L


def rayleigh_ritz(GA, GB, k, pivot_min=PIVOT_MIN):
    """k smallest Ritz pairs of the pencil (G_A, G_B): (theta, coefficients)
    or None when the scaled G_B has a Cholesky pivot <= pivot_min."""
    d = 1.0 / np.sqrt(np.diag(GB))
    Ah = 0.5 * (GA + GA.T) * np.outer(d, d)
    Bh = GB * np.outer(d, d)
    L = _cholesky_lower(Bh, pivot_min)
    if L is None:
        return None
    Cm = sla.solve_triangular(L, sla.solve_triangular(L, Ah, lower=True).T, lower=True)
    theta, V = np.linalg.eigh(0.5 * (Cm + Cm.T))
    coef = d[:, None] * sla.solve_triangular(L.T, V[:, :k], lower=False)
    return theta[:k], coef


def block_preconditioner(prec):
    """W = T R column by column: None (T = I) | ("sait64", M_L, M_U) |
    ("exact", L, U) | ("jacobi", L, U, sweeps), with the oracle's own
    applies and triangular solves."""
    import oracle

    if prec is None:
        return lambda R: R.copy()
    kind = prec[0]
    if kind == "sait64":
        f = lambda r: oracle.apply(prec[1], prec[2], r)
    elif kind == "exact":
        f = lambda r: oracle.upper_solve(prec[2], oracle.lower_solve(prec[1], r))
    elif kind == "jacobi":
        f = lambda r: oracle.jacobi_sweeps(prec[2], oracle.jacobi_sweeps(prec[1], r, prec[3]), prec[3])
    else:
        raise ValueError(f"unknown preconditioner {kind!r}")
    return lambda R: np.stack([f(np.ascontiguousarray(R[:, j])) for j in range(R.shape[1])], axis=1)


def lobpcg(A, X0, prec=None, tol=1e-8, maxit=1000):
    """A: workloads.Csr (symmetric positive definite); X0: n x k start block
    (full column rank).  Returns dict(lam, X, iters, status (0 converged,
    1 maxit, 2 breakdown), relres (max_j ||R_j|| / |theta_j| at the end),
    p_drops, hist (that maximum before every step), theta_hist)."""
    As = A.to_scipy()
    T = block_preconditioner(prec)
    X0 = np.array(X0, dtype=np.float64)
    k = X0.shape[1]
    AX0 = As @ X0
    out = rayleigh_ritz(X0.T @ AX0, X0.T @ X0, k)
    if out is None:
        raise ValueError("X0 is numerically rank deficient")
    theta, c = out
    X, AX = X0 @ c, AX0 @ c
    P = AP = None
    hist, theta_hist, p_drops, status, it = [], [theta.copy()], 0, 1, 0
    for it in range(maxit + 1):
        R = AX - X * theta
        res = np.linalg.norm(R, axis=0) / np.abs(theta)
        hist.append(res.max())
        if res.max() <= tol:
            status = 0
            break
        if it == maxit:
            break
        W = T(R)
        AW = As @ W
        step = None
        for use_p in ((True, False) if P is not None else (False,)):
            S = np.hstack([X, W, P] if use_p else [X, W])
            AS = np.hstack([AX, AW, AP] if use_p else [AX, AW])
            step = rayleigh_ritz(S.T @ AS, S.T @ S, k, PIVOT_P if use_p else PIVOT_MIN)
            if step is not None:
                break
            p_drops += 1
        if step is None:
            status = 2
            break
        theta, c = step
        X, AX = S @ c, AS @ c
        P, AP = S[:, k:] @ c[k:], AS[:, k:] @ c[k:]
        theta_hist.append(theta.copy())
    return dict(lam=theta, X=X, iters=it, status=status, relres=hist[-1], p_drops=p_drops,
                hist=np.array(hist), theta_hist=np.array(theta_hist))
