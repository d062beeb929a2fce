"""Python binding of the CPU oracle -- TEST INFRASTRUCTURE ONLY.

Argument marshalling around oracle/liboracle.so (plain C, FP64).  Only the
test-suite, the smoke check and the CPU-baseline leg of the benchmark may
import this package; the product library never does.
"""

from __future__ import annotations

import ctypes as C
import os

import numpy as np

from workloads import Csr

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None

OK, NOT_CONVERGED, E_INVALID, E_ZERO_PIVOT, E_NONFINITE, E_NOMEM = 0, 1, -1, -2, -3, -4

_i32p = C.POINTER(C.c_int32)
_f64p = C.POINTER(C.c_double)
_f32p = C.POINTER(C.c_float)
_u16p = C.POINTER(C.c_uint16)


class OracleError(RuntimeError):
    def __init__(self, status, what):
        super().__init__(f"oracle {what} failed with status {status}")
        self.status = status


class _Prec(C.Structure):
    _fields_ = [
        ("kind", C.c_int),
        ("rp1", _i32p), ("ci1", _i32p), ("v1", _f64p), ("f1", _f32p),
        ("rp2", _i32p), ("ci2", _i32p), ("v2", _f64p), ("f2", _f32p),
        ("sweeps", C.c_int),
    ]


def lib():
    global _LIB
    if _LIB is None:
        path = os.path.join(_HERE, "liboracle.so")
        if not os.path.exists(path):
            from . import build as _b
            _b.build()
        L = C.CDLL(path)
        I64, I32, D = C.c_int64, C.c_int32, C.c_double
        pp_i = C.POINTER(_i32p)
        pp_d = C.POINTER(_f64p)
        L.or_ilu0.argtypes = [I64, _i32p, _i32p, _f64p, pp_i, pp_i, pp_d, pp_i, pp_i, pp_d]
        L.or_ilut.argtypes = [I64, _i32p, _i32p, _f64p, D, C.c_int, pp_i, pp_i, pp_d, pp_i, pp_i, pp_d]
        L.or_iluk.argtypes = [I64, _i32p, _i32p, _f64p, C.c_int, pp_i, pp_i, pp_d, pp_i, pp_i, pp_d]
        L.or_iluk_pattern.argtypes = [I64, _i32p, _i32p, _f64p, C.c_int, pp_i, pp_i, pp_d]
        L.or_parilu.argtypes = [I64, _i32p, _i32p, _f64p, C.c_int, pp_i, pp_i, pp_d, pp_i, pp_i, pp_d]
        L.or_paric.argtypes = [I64, _i32p, _i32p, _f64p, C.c_int, pp_i, pp_i, pp_d, pp_i, pp_i, pp_d]
        L.or_lower_solve.argtypes = [I64, _i32p, _i32p, _f64p, _f64p, _f64p]
        L.or_upper_solve.argtypes = [I64, _i32p, _i32p, _f64p, _f64p, _f64p]
        L.or_sait_step.argtypes = [I64, _i32p, _i32p, _f64p, _i32p, _i32p, _f64p, D, C.c_int, C.c_int, pp_i, pp_i,
                                   pp_d]
        L.or_sait_thr.argtypes = [I64, _i32p, _i32p, _f64p, D, C.c_int, C.c_int, C.c_int, pp_i, pp_i, pp_d]
        L.or_sait_pat.argtypes = [I64, _i32p, _i32p, _f64p, C.c_int, C.c_int, C.c_int, pp_i, pp_i, pp_d]
        L.or_spmv.argtypes = [I64, _i32p, _i32p, _f64p, _f64p, _f64p]
        L.or_spmv.restype = None
        L.or_apply.argtypes = [I64, _i32p, _i32p, _f64p, _i32p, _i32p, _f64p, _f64p, _f64p]
        L.or_round_f32.argtypes = [I64, _f64p, _f32p]
        L.or_round_f32.restype = None
        L.or_round_bf16.argtypes = [I64, _f64p, _u16p]
        L.or_round_bf16.restype = None
        L.or_bf16_to_f32.argtypes = [I64, _u16p, _f32p]
        L.or_bf16_to_f32.restype = None
        L.or_apply_f32acc.argtypes = [I64, _i32p, _i32p, _f32p, _i32p, _i32p, _f32p, _f64p, _f64p]
        L.or_transpose.argtypes = [I64, _i32p, _i32p, _f64p, pp_i, pp_i, pp_d]
        L.or_grad_values.argtypes = [I64, _i32p, _i32p, _f64p, _f64p, _f64p]
        L.or_grad_values.restype = None
        L.or_gmres.argtypes = [I64, _i32p, _i32p, _f64p, C.POINTER(_Prec), _f64p, _f64p,
                               C.c_int, C.c_int, D, C.c_int,
                               C.POINTER(C.c_int), C.POINTER(C.c_int), _f64p, _f64p, _f64p]
        L.or_jacobi_sweeps.argtypes = [I64, _i32p, _i32p, _f64p, _f64p, C.c_int, _f64p]
        L.or_pcg.argtypes = [I64, _i32p, _i32p, _f64p, C.POINTER(_Prec), _f64p, _f64p, C.c_int, D,
                             C.POINTER(C.c_int), C.POINTER(C.c_double), _f64p]
        L.or_free.argtypes = [C.c_void_p]
        L.or_free.restype = None
        L.or_num_threads.restype = C.c_int
        _LIB = L
    return _LIB


def num_threads() -> int:
    return int(lib().or_num_threads())


def _p(a, t):
    return a.ctypes.data_as(t)


def _csr_args(M: Csr):
    rp = np.ascontiguousarray(M.rp, dtype=np.int32)
    ci = np.ascontiguousarray(M.ci, dtype=np.int32)
    v = np.ascontiguousarray(M.v, dtype=np.float64)
    return (rp, ci, v), (_p(rp, _i32p), _p(ci, _i32p), _p(v, _f64p))


def _take(n, rp, ci, v) -> Csr:
    """Copy a malloc'd CSR out of the library and free it."""
    L = lib()
    rpa = np.ctypeslib.as_array(rp, shape=(n + 1,)).copy()
    nnz = int(rpa[-1])
    cia = np.ctypeslib.as_array(ci, shape=(max(nnz, 1),))[:nnz].copy()
    va = np.ctypeslib.as_array(v, shape=(max(nnz, 1),))[:nnz].copy()
    for p in (rp, ci, v):
        L.or_free(C.cast(p, C.c_void_p))
    return Csr(n, rpa, cia, va)


def _out3():
    return _i32p(), _i32p(), _f64p()


def _check(st, what):
    if st < 0:
        raise OracleError(st, what)
    return st


def ilu0(A: Csr):
    """Level-0 ILU, A ~ L U (L unit lower with its diagonal stored)."""
    keep, (rp, ci, v) = _csr_args(A)
    Lo, Uo = _out3(), _out3()
    st = lib().or_ilu0(A.n, rp, ci, v, *(C.byref(x) for x in Lo), *(C.byref(x) for x in Uo))
    _check(st, "ilu0")
    return _take(A.n, *Lo), _take(A.n, *Uo)


def ilut(A: Csr, tau: float, p: int):
    keep, (rp, ci, v) = _csr_args(A)
    Lo, Uo = _out3(), _out3()
    st = lib().or_ilut(A.n, rp, ci, v, float(tau), int(p), *(C.byref(x) for x in Lo), *(C.byref(x) for x in Uo))
    _check(st, "ilut")
    return _take(A.n, *Lo), _take(A.n, *Uo)


def iluk(A: Csr, p: int):
    """ILU(p) by levels of fill: the ILU(0) elimination on the level-p pattern."""
    keep, (rp, ci, v) = _csr_args(A)
    Lo, Uo = _out3(), _out3()
    st = lib().or_iluk(A.n, rp, ci, v, int(p), *(C.byref(x) for x in Lo), *(C.byref(x) for x in Uo))
    _check(st, "iluk")
    return _take(A.n, *Lo), _take(A.n, *Uo)


def iluk_pattern(A: Csr, p: int) -> Csr:
    """The level-p pattern of A as a matrix: A's values, explicit zeros at
    the kept fill."""
    keep, (rp, ci, v) = _csr_args(A)
    E = _out3()
    _check(lib().or_iluk_pattern(A.n, rp, ci, v, int(p), *(C.byref(x) for x in E)), "iluk_pattern")
    return _take(A.n, *E)


def parilu(A: Csr, sweeps: int, level: int = 0):
    """Fine-grained parallel ILU (Chow and Patel), synchronous sweeps on the
    level-`level` pattern of A (0: A's own pattern).  Returns (L, U)."""
    E = A if level == 0 else iluk_pattern(A, level)
    keep, (rp, ci, v) = _csr_args(E)
    Lo, Uo = _out3(), _out3()
    st = lib().or_parilu(E.n, rp, ci, v, int(sweeps), *(C.byref(x) for x in Lo), *(C.byref(x) for x in Uo))
    _check(st, "parilu")
    return _take(E.n, *Lo), _take(E.n, *Uo)


def paric(A: Csr, sweeps: int, level: int = 0):
    """Symmetric (incomplete Cholesky) form of the synchronous fine-grained
    parallel ILU on the level-`level` pattern of a symmetric A (its upper
    triangle is read).  Returns (L, U) with l_ji = u_ij / u_ii."""
    E = A if level == 0 else iluk_pattern(A, level)
    keep, (rp, ci, v) = _csr_args(E)
    Lo, Uo = _out3(), _out3()
    st = lib().or_paric(E.n, rp, ci, v, int(sweeps), *(C.byref(x) for x in Lo), *(C.byref(x) for x in Uo))
    _check(st, "paric")
    return _take(E.n, *Lo), _take(E.n, *Uo)


def lower_solve(L: Csr, b):
    keep, (rp, ci, v) = _csr_args(L)
    b = np.ascontiguousarray(b, dtype=np.float64)
    x = np.empty(L.n)
    _check(lib().or_lower_solve(L.n, rp, ci, v, _p(b, _f64p), _p(x, _f64p)), "lower_solve")
    return x


def upper_solve(U: Csr, b):
    keep, (rp, ci, v) = _csr_args(U)
    b = np.ascontiguousarray(b, dtype=np.float64)
    x = np.empty(U.n)
    _check(lib().or_upper_solve(U.n, rp, ci, v, _p(b, _f64p), _p(x, _f64p)), "upper_solve")
    return x


def _side(side: str) -> int:
    if side not in ("left", "right"):
        raise ValueError("side must be 'left' (T~ M) or 'right' (M T~)")
    return int(side == "right")


def sait_step(T: Csr, M: Csr, tau: float, cap: int = 0, side: str = "left") -> Csr:
    """One unscaled pass: drop(T~ M + I), or drop(M T~ + I) with side="right"."""
    k1, (trp, tci, tv) = _csr_args(T)
    k2, (mrp, mci, mv) = _csr_args(M)
    O = _out3()
    st = lib().or_sait_step(T.n, trp, tci, tv, mrp, mci, mv, float(tau), int(cap), _side(side),
                            *(C.byref(x) for x in O))
    _check(st, "sait_step")
    return _take(T.n, *O)


def sait_thr(T: Csr, tau: float, m: int, cap: int = 0, side: str = "left") -> Csr:
    """SAIT_Thr(tau, m) (Alg. 2), optional per-row cap; side="right" runs
    every pass as M T~ + I."""
    keep, (rp, ci, v) = _csr_args(T)
    O = _out3()
    _check(lib().or_sait_thr(T.n, rp, ci, v, float(tau), int(m), int(cap), _side(side), *(C.byref(x) for x in O)),
           "sait_thr")
    return _take(T.n, *O)


def sait_pat(T: Csr, p: int, m: int, side: str = "left") -> Csr:
    """SAIT_Pat(p, m) (Alg. 3); side="right" runs every pass as M T~ + I."""
    keep, (rp, ci, v) = _csr_args(T)
    O = _out3()
    _check(lib().or_sait_pat(T.n, rp, ci, v, int(p), int(m), _side(side), *(C.byref(x) for x in O)), "sait_pat")
    return _take(T.n, *O)


def sait_factors(L: Csr, U: Csr, m: int, tau: float = 0.0, cap: int = 0, p: int = -1,
                 upper_side: str = "right"):
    """(M_L, M_U) of an ILU pair: M_L by the left-multiplied recursion of
    Alg. 1, M_U by the recursion multiplied from the right (the default; for
    a symmetric A this gives M_U = M_L^T D^-1 and a symmetric positive
    definite M_U M_L) or from the left (upper_side="left", Alg. 1 verbatim).
    p >= 0 selects SAIT_Pat(p, m), else SAIT_Thr(tau, m) with the cap."""
    if p >= 0:
        return sait_pat(L, p, m), sait_pat(U, p, m, side=upper_side)
    return sait_thr(L, tau, m, cap), sait_thr(U, tau, m, cap, side=upper_side)


def identity(n: int) -> Csr:
    return Csr(n, np.arange(n + 1, dtype=np.int32), np.arange(n, dtype=np.int32), np.ones(n))


def spmv(M: Csr, x):
    keep, (rp, ci, v) = _csr_args(M)
    x = np.ascontiguousarray(x, dtype=np.float64)
    y = np.empty(M.n)
    lib().or_spmv(M.n, rp, ci, v, _p(x, _f64p), _p(y, _f64p))
    return y


def apply(M1: Csr, M2: Csr, r):
    """z = M2 (M1 r) in FP64 (the preconditioner with M1 = M_L, M2 = M_U)."""
    k1, a1 = _csr_args(M1)
    k2, a2 = _csr_args(M2)
    r = np.ascontiguousarray(r, dtype=np.float64)
    z = np.empty(M1.n)
    _check(lib().or_apply(M1.n, *a1, *a2, _p(r, _f64p), _p(z, _f64p)), "apply")
    return z


def round_f32(v):
    v = np.ascontiguousarray(v, dtype=np.float64)
    out = np.empty(v.shape, dtype=np.float32)
    lib().or_round_f32(v.size, _p(v, _f64p), _p(out, _f32p))
    return out


def round_bf16(v):
    """bfloat16 encodings (uint16) of fl16(fl32(v))."""
    v = np.ascontiguousarray(v, dtype=np.float64)
    out = np.empty(v.shape, dtype=np.uint16)
    lib().or_round_bf16(v.size, _p(v, _f64p), _p(out, _u16p))
    return out


def bf16_to_f32(u):
    u = np.ascontiguousarray(u, dtype=np.uint16)
    out = np.empty(u.shape, dtype=np.float32)
    lib().or_bf16_to_f32(u.size, _p(u, _u16p), _p(out, _f32p))
    return out


def storage_values(M: Csr, precision: str):
    """Factor values as stored in the given precision, widened to float32
    (f32) or returned as float64 (f64)."""
    if precision == "f64":
        return np.asarray(M.v, dtype=np.float64)
    if precision == "f32":
        return round_f32(M.v)
    if precision == "bf16":
        return bf16_to_f32(round_bf16(M.v))
    raise ValueError(precision)


def apply_f32acc(M1: Csr, v1_f32, M2: Csr, v2_f32, r):
    """z = (double)(M2_32 (M1_32 fl32(r))) with binary32 accumulation."""
    rp1 = np.ascontiguousarray(M1.rp, dtype=np.int32)
    ci1 = np.ascontiguousarray(M1.ci, dtype=np.int32)
    rp2 = np.ascontiguousarray(M2.rp, dtype=np.int32)
    ci2 = np.ascontiguousarray(M2.ci, dtype=np.int32)
    f1 = np.ascontiguousarray(v1_f32, dtype=np.float32)
    f2 = np.ascontiguousarray(v2_f32, dtype=np.float32)
    r = np.ascontiguousarray(r, dtype=np.float64)
    z = np.empty(M1.n)
    _check(lib().or_apply_f32acc(M1.n, _p(rp1, _i32p), _p(ci1, _i32p), _p(f1, _f32p),
                                 _p(rp2, _i32p), _p(ci2, _i32p), _p(f2, _f32p),
                                 _p(r, _f64p), _p(z, _f64p)), "apply_f32acc")
    return z


def transpose(M: Csr) -> Csr:
    keep, (rp, ci, v) = _csr_args(M)
    O = _out3()
    _check(lib().or_transpose(M.n, rp, ci, v, *(C.byref(x) for x in O)), "transpose")
    return _take(M.n, *O)


def grad_values(A: Csr, lam, x):
    keep, (rp, ci, v) = _csr_args(A)
    lam = np.ascontiguousarray(lam, dtype=np.float64)
    x = np.ascontiguousarray(x, dtype=np.float64)
    g = np.empty(A.nnz)
    lib().or_grad_values(A.n, rp, ci, _p(lam, _f64p), _p(x, _f64p), _p(g, _f64p))
    return g


PREC_NONE, PREC_SAIT64, PREC_SAIT32, PREC_EXACT, PREC_JACOBI = 0, 1, 2, 3, 4


def _make_prec(prec):
    """or_prec for None | ("sait64", M1, M2) | ("sait32", M1, f1, M2, f2) |
    ("exact", L, U) | ("jacobi", L, U, sweeps); returns (struct, arrays to keep alive)."""
    P = _Prec()
    hold = []
    if prec is None:
        P.kind = PREC_NONE
    elif prec[0] in ("sait64", "exact", "jacobi"):
        P.kind = {"sait64": PREC_SAIT64, "exact": PREC_EXACT, "jacobi": PREC_JACOBI}[prec[0]]
        k1, a1 = _csr_args(prec[1])
        k2, a2 = _csr_args(prec[2])
        hold += [k1, k2]
        P.rp1, P.ci1, P.v1 = a1
        P.rp2, P.ci2, P.v2 = a2
        if prec[0] == "jacobi":
            P.sweeps = int(prec[3])
    elif prec[0] == "sait32":
        P.kind = PREC_SAIT32
        M1, f1, M2, f2 = prec[1:]
        arrs = [np.ascontiguousarray(M1.rp, dtype=np.int32), np.ascontiguousarray(M1.ci, dtype=np.int32),
                np.ascontiguousarray(f1, dtype=np.float32),
                np.ascontiguousarray(M2.rp, dtype=np.int32), np.ascontiguousarray(M2.ci, dtype=np.int32),
                np.ascontiguousarray(f2, dtype=np.float32)]
        hold += arrs
        P.rp1, P.ci1, P.f1 = _p(arrs[0], _i32p), _p(arrs[1], _i32p), _p(arrs[2], _f32p)
        P.rp2, P.ci2, P.f2 = _p(arrs[3], _i32p), _p(arrs[4], _i32p), _p(arrs[5], _f32p)
    else:
        raise ValueError(prec[0])
    return P, hold


def jacobi_sweeps(T: Csr, r, sweeps: int):
    """s Jacobi sweeps from zero for the triangular system T y = r (lower or
    upper): y_i <- (r_i - sum_{j != i} T_ij y_j) / T_ii from the previous iterate."""
    keep, (rp, ci, v) = _csr_args(T)
    r = np.ascontiguousarray(r, dtype=np.float64)
    y = np.empty(T.n)
    _check(lib().or_jacobi_sweeps(T.n, rp, ci, v, _p(r, _f64p), int(sweeps), _p(y, _f64p)), "jacobi_sweeps")
    return y


def pcg(A: Csr, b, prec=None, x0=None, maxit=10000, rtol=1e-10, history=False):
    """Preconditioned conjugate gradients (textbook form), stopping on the
    recursively updated relative residual; prec as for gmres.  Returns
    dict(x, iters, relres (true, at the end), status[, hist])."""
    keep, (rp, ci, v) = _csr_args(A)
    b = np.ascontiguousarray(b, dtype=np.float64)
    x = np.zeros(A.n) if x0 is None else np.array(x0, dtype=np.float64)
    P, hold = _make_prec(prec)
    it, rr = C.c_int(0), C.c_double(0)
    hist = np.zeros(max(maxit, 1)) if history else None
    st = lib().or_pcg(A.n, rp, ci, v, C.byref(P), _p(b, _f64p), _p(x, _f64p), int(maxit), float(rtol),
                      C.byref(it), C.byref(rr), _p(hist, _f64p) if history else None)
    _check(st, "pcg")
    out = dict(x=x, iters=it.value, relres=rr.value, status=st)
    if history:
        out["hist"] = hist[: it.value]
    return out


def gmres(A: Csr, b, prec=None, x0=None, restart=30, maxit=10000, rtol=1e-8, flexible=False,
          history=False):
    """Restarted right-preconditioned (F)GMRES.

    prec: None | ("sait64", M1, M2) | ("sait32", M1, f1, M2, f2) | ("exact", L, U)
    | ("jacobi", L, U, sweeps) where the preconditioner is z = M2 (M1 r) (for
    "exact": U^-1 (L^-1 r); "jacobi": s sweeps on L, then on U).
    Returns dict(x, iters, restarts, relres, est, status[, hist]).
    """
    keep, (rp, ci, v) = _csr_args(A)
    b = np.ascontiguousarray(b, dtype=np.float64)
    x = np.zeros(A.n) if x0 is None else np.array(x0, dtype=np.float64)
    P, hold = _make_prec(prec)
    it, rs = C.c_int(0), C.c_int(0)
    rr, est = C.c_double(0), C.c_double(0)
    hist = np.zeros(max(maxit, 1)) if history else None
    st = lib().or_gmres(A.n, rp, ci, v, C.byref(P), _p(b, _f64p), _p(x, _f64p), int(restart), int(maxit),
                        float(rtol), int(bool(flexible)), C.byref(it), C.byref(rs), C.byref(rr), C.byref(est),
                        _p(hist, _f64p) if history else None)
    _check(st, "gmres")
    out = dict(x=x, iters=it.value, restarts=rs.value, relres=rr.value, est=est.value, status=st)
    if history:
        out["hist"] = hist[: it.value]
    return out


from . import lobpcg as lobpcg_module  # noqa: E402  (LOBPCG of the eigenvalue experiment, Sec. 4)
from .lobpcg import lobpcg  # noqa: E402,F401
