"""Python binding of libsait (argument marshalling only).

Every function here forwards to the C ABI declared in include/sait.h; all
arithmetic of the SAIT path runs in the library's HIP kernels (or, for the
incomplete factorisation, in its host C++ code).  PyTorch is used only for
device memory (tensors) and streams.  There is no fallback: if the shared
library is missing or the GPU is unavailable the calls raise.
"""

from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libsait.so")
_LIB = None

SAIT_OK, SAIT_NOT_CONVERGED, SAIT_BREAKDOWN = 0, 1, 2
SAIT_E_INVALID, SAIT_E_ZERO_PIVOT, SAIT_E_NONFINITE, SAIT_E_NOMEM, SAIT_E_DEVICE = -1, -2, -3, -4, -5
SAIT_ILU0, SAIT_ILUT, SAIT_ILUK, SAIT_PARILU, SAIT_PARIC = 0, 1, 2, 3, 4
SAIT_SIDE_LEFT, SAIT_SIDE_RIGHT = 0, 1
SIDES = {"left": SAIT_SIDE_LEFT, "right": SAIT_SIDE_RIGHT}
SAIT_METHOD_GMRES, SAIT_METHOD_PCG = 0, 1
SAIT_PREC_SAIT, SAIT_PREC_JACOBI, SAIT_PREC_EXACT, SAIT_PREC_NONE = 0, 1, 2, 3
PREC_KINDS = {"sait": SAIT_PREC_SAIT, "jacobi": SAIT_PREC_JACOBI, "exact": SAIT_PREC_EXACT, "none": SAIT_PREC_NONE}
SAIT_F64, SAIT_F32, SAIT_BF16 = 0, 1, 2
SAIT_MAT_A, SAIT_MAT_L, SAIT_MAT_U, SAIT_MAT_ML, SAIT_MAT_MU = 0, 1, 2, 3, 4
PRECISIONS = {"f64": SAIT_F64, "f32": SAIT_F32, "bf16": SAIT_BF16}

EXPORTED = (
    "sait_default_build_opts", "sait_default_solve_opts", "sait_build", "sait_apply", "sait_matvec",
    "sait_solve", "sait_set_values", "sait_grad_values", "sait_query", "sait_export", "sait_destroy", "sait_last_error",
    "sait_autotune", "sait_set_apply_lanes", "sait_get_apply_lanes", "sait_time_apply", "sait_debug_step", "sait_copy",
    "sait_set_preconditioner", "sait_default_eig_opts", "sait_lobpcg",
)


class SaitError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"libsait status {status}: {msg}")
        self.status = status


class sait_allocator(C.Structure):
    _fields_ = [("alloc", C.c_void_p), ("free", C.c_void_p), ("ctx", C.c_void_p)]


class sait_build_opts(C.Structure):
    _fields_ = [
        ("ilu_kind", C.c_int), ("ilut_tau", C.c_double), ("ilut_fill", C.c_int),
        ("m", C.c_int), ("tau", C.c_double), ("max_nnz_row", C.c_int),
        ("pattern_p", C.c_int), ("precision", C.c_int), ("build_transpose", C.c_int),
        ("ilu_level", C.c_int),
        ("upper_side", C.c_int),
        ("parilu_sweeps", C.c_int),
    ]


class sait_solve_opts(C.Structure):
    _fields_ = [("restart", C.c_int), ("maxit", C.c_int), ("rtol", C.c_double), ("flexible", C.c_int),
                ("method", C.c_int)]


class sait_solve_info(C.Structure):
    _fields_ = [("iterations", C.c_int), ("restarts", C.c_int), ("status", C.c_int),
                ("est_relres", C.c_double), ("true_relres", C.c_double)]


class sait_eig_opts(C.Structure):
    _fields_ = [("maxit", C.c_int), ("tol", C.c_double)]


class sait_eig_info(C.Structure):
    _fields_ = [("iterations", C.c_int), ("status", C.c_int), ("p_drops", C.c_int), ("relres", C.c_double)]


def library_path() -> str:
    return _LIB_PATH


def lib():
    """Load libsait.so; raise if it has not been built."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(_LIB_PATH):
            raise ImportError(f"{_LIB_PATH} is missing: build it with `python __graft_entry__.py` "
                              "(or paper_2106_12836_amd/build.py)")
        L = C.CDLL(_LIB_PATH)
        vp, i64, i32p, f64p = C.c_void_p, C.c_int64, C.POINTER(C.c_int32), C.POINTER(C.c_double)
        L.sait_default_build_opts.argtypes = [C.POINTER(sait_build_opts)]
        L.sait_default_build_opts.restype = None
        L.sait_default_solve_opts.argtypes = [C.POINTER(sait_solve_opts)]
        L.sait_default_solve_opts.restype = None
        L.sait_default_eig_opts.argtypes = [C.POINTER(sait_eig_opts)]
        L.sait_default_eig_opts.restype = None
        L.sait_lobpcg.argtypes = [vp, vp, C.c_int, f64p, f64p, C.POINTER(sait_eig_opts), C.POINTER(sait_eig_info), vp]
        L.sait_build.argtypes = [i64, i32p, i32p, f64p, C.c_int, C.POINTER(C.c_int64),
                                 C.POINTER(sait_build_opts), C.POINTER(sait_allocator), vp, C.POINTER(vp)]
        L.sait_apply.argtypes = [vp, vp, vp, C.c_int, i64, C.c_int, vp]
        L.sait_matvec.argtypes = [vp, vp, vp, C.c_int, i64, C.c_int, vp]
        L.sait_solve.argtypes = [vp, vp, vp, C.c_int, i64, C.c_int, C.POINTER(sait_solve_opts),
                                 C.POINTER(sait_solve_info), vp]
        L.sait_grad_values.argtypes = [vp, vp, vp, vp, vp]
        L.sait_set_values.argtypes = [vp, vp, vp]
        L.sait_query.argtypes = [vp] + [C.POINTER(C.c_int64)] * 6
        L.sait_export.argtypes = [vp, C.c_int, i32p, i32p, f64p, vp]
        L.sait_destroy.argtypes = [vp]
        L.sait_destroy.restype = None
        L.sait_last_error.restype = C.c_char_p
        L.sait_autotune.argtypes = [vp, C.c_int, vp]
        L.sait_set_apply_lanes.argtypes = [vp, C.c_int, C.c_int]
        L.sait_get_apply_lanes.argtypes = [vp, C.POINTER(C.c_int), C.POINTER(C.c_int)]
        L.sait_time_apply.argtypes = [vp, vp, vp, C.c_int, vp, f64p, f64p, f64p]
        L.sait_copy.argtypes = [vp, vp, C.c_size_t, vp]
        L.sait_set_preconditioner.argtypes = [vp, C.c_int, C.c_int, vp]
        L.sait_debug_step.argtypes = [i64, i32p, i32p, f64p, i32p, i32p, f64p, C.c_double, C.c_int, C.c_int,
                                      i64, i32p, i32p, f64p, C.POINTER(C.c_int64)]
        _LIB = L
    return _LIB


def _check(st: int, allow_positive: bool = True) -> int:
    if st < 0 or (st > 0 and not allow_positive):
        raise SaitError(st, lib().sait_last_error().decode(errors="replace"))
    return st


def _ptr(a, t):
    return a.ctypes.data_as(C.POINTER(t))


def _stream(stream):
    import torch

    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def _dptr(t) -> C.c_void_p:
    """Device pointer of a torch tensor (must be CUDA/HIP, float64, contiguous)."""
    import torch

    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise TypeError("expected a device tensor")
    if t.dtype != torch.float64:
        raise TypeError("expected float64")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    return C.c_void_p(t.data_ptr())


def default_build_opts(**kw) -> sait_build_opts:
    o = sait_build_opts()
    lib().sait_default_build_opts(C.byref(o))
    for k, v in kw.items():
        if k == "precision" and isinstance(v, str):
            v = PRECISIONS[v]
        if k == "ilu_kind" and isinstance(v, str):
            v = {"ilu0": SAIT_ILU0, "ilut": SAIT_ILUT, "iluk": SAIT_ILUK, "parilu": SAIT_PARILU,
                 "paric": SAIT_PARIC}[v]
        if k == "upper_side" and isinstance(v, str):
            v = SIDES[v]
        setattr(o, k, v)
    return o


def default_solve_opts(**kw) -> sait_solve_opts:
    o = sait_solve_opts()
    lib().sait_default_solve_opts(C.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


# --------------------------------------------------------------------------
# Thin wrappers with the C names
# --------------------------------------------------------------------------

def sait_build(n, row_ptr, col_idx, val, nsys=1, sys_ptr=None, opts=None, stream=None) -> C.c_void_p:
    rp = np.ascontiguousarray(row_ptr, dtype=np.int32)
    ci = np.ascontiguousarray(col_idx, dtype=np.int32)
    v = np.ascontiguousarray(val, dtype=np.float64)
    sp = None if sys_ptr is None else np.ascontiguousarray(sys_ptr, dtype=np.int64)
    h = C.c_void_p()
    st = lib().sait_build(int(n), _ptr(rp, C.c_int32), _ptr(ci, C.c_int32), _ptr(v, C.c_double), int(nsys),
                          None if sp is None else _ptr(sp, C.c_int64),
                          C.byref(opts) if opts is not None else None, None, _stream(stream), C.byref(h))
    _check(st)
    return h


def sait_apply(h, r, z, nrhs=1, ld=None, transpose=0, stream=None):
    ld = nrhs if ld is None else ld
    return _check(lib().sait_apply(h, _dptr(r), _dptr(z), int(nrhs), int(ld), int(transpose), _stream(stream)))


def sait_matvec(h, x, y, nrhs=1, ld=None, transpose=0, stream=None):
    ld = nrhs if ld is None else ld
    return _check(lib().sait_matvec(h, _dptr(x), _dptr(y), int(nrhs), int(ld), int(transpose), _stream(stream)))


def sait_solve(h, b, x, nrhs=1, ld=None, transpose=0, opts=None, ninfo=1, stream=None):
    """Returns (status, list of info dicts)."""
    ld = nrhs if ld is None else ld
    infos = (sait_solve_info * max(int(ninfo), 1))()
    st = lib().sait_solve(h, _dptr(b), _dptr(x), int(nrhs), int(ld), int(transpose),
                          C.byref(opts) if opts is not None else None, infos, _stream(stream))
    _check(st)
    out = [dict(iterations=i.iterations, restarts=i.restarts, status=i.status, est_relres=i.est_relres,
                true_relres=i.true_relres) for i in infos]
    return st, out


def default_eig_opts(**kw) -> sait_eig_opts:
    o = sait_eig_opts()
    lib().sait_default_eig_opts(C.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def sait_lobpcg(h, X, k, opts=None, history=False, stream=None):
    """X: device n x k row-major block (start block in, Ritz vectors out).
    Returns (status, lambda (k,), info dict, history array or None)."""
    lam = np.zeros(int(k))
    o = opts if opts is not None else default_eig_opts()
    hist = np.zeros(o.maxit + 1) if history else None
    info = sait_eig_info()
    st = lib().sait_lobpcg(h, _dptr(X), int(k), _ptr(lam, C.c_double), _ptr(hist, C.c_double) if history else None,
                           C.byref(o), C.byref(info), _stream(stream))
    _check(st)
    out = dict(iterations=info.iterations, status=info.status, p_drops=info.p_drops, relres=info.relres)
    return st, lam, out, (hist[: info.iterations + 1] if history else None)


def sait_set_values(h, vals, stream=None):
    return _check(lib().sait_set_values(h, _dptr(vals), _stream(stream)))


def sait_grad_values(h, lam, x, grad, stream=None):
    return _check(lib().sait_grad_values(h, _dptr(lam), _dptr(x), _dptr(grad), _stream(stream)))


def sait_query(h) -> dict:
    vals = [C.c_int64() for _ in range(6)]
    _check(lib().sait_query(h, *[C.byref(v) for v in vals]))
    keys = ("n", "nnz_A", "nnz_L", "nnz_U", "nnz_ML", "nnz_MU")
    return {k: v.value for k, v in zip(keys, vals)}


def sait_export(h, which: int, stored: bool = False):
    """Returns (row_ptr, col_idx, fp64 values[, stored values]) as numpy arrays."""
    q = sait_query(h)
    nnz = {SAIT_MAT_A: q["nnz_A"], SAIT_MAT_L: q["nnz_L"], SAIT_MAT_U: q["nnz_U"],
           SAIT_MAT_ML: q["nnz_ML"], SAIT_MAT_MU: q["nnz_MU"]}[which]
    rp = np.empty(q["n"] + 1, dtype=np.int32)
    ci = np.empty(max(nnz, 1), dtype=np.int32)
    v = np.empty(max(nnz, 1), dtype=np.float64)
    sv = None
    if stored:
        sv = np.empty(max(nnz, 1) * 8, dtype=np.uint8)
    _check(lib().sait_export(h, int(which), _ptr(rp, C.c_int32), _ptr(ci, C.c_int32), _ptr(v, C.c_double),
                             None if sv is None else sv.ctypes.data_as(C.c_void_p)))
    out = (rp, ci[:nnz], v[:nnz])
    if stored:
        return out + (sv,)
    return out


def sait_export_row_ptr(h, which: int):
    """Row pointers only (no entries are copied)."""
    q = sait_query(h)
    rp = np.empty(q["n"] + 1, dtype=np.int32)
    _check(lib().sait_export(h, int(which), _ptr(rp, C.c_int32), None, None, None))
    return rp


def sait_destroy(h):
    if h:
        lib().sait_destroy(h)


def sait_set_preconditioner(h, kind, sweeps=1, stream=None):
    if isinstance(kind, str):
        kind = PREC_KINDS[kind]
    return _check(lib().sait_set_preconditioner(h, int(kind), int(sweeps), _stream(stream)))


def sait_last_error() -> str:
    return lib().sait_last_error().decode(errors="replace")


def sait_autotune(h, nrhs=1, stream=None):
    return _check(lib().sait_autotune(h, int(nrhs), _stream(stream)))


def sait_set_apply_lanes(h, lanes_L=0, lanes_U=0):
    return _check(lib().sait_set_apply_lanes(h, int(lanes_L), int(lanes_U)))


def sait_get_apply_lanes(h):
    a, b = C.c_int(), C.c_int()
    _check(lib().sait_get_apply_lanes(h, C.byref(a), C.byref(b)))
    return a.value, b.value


def sait_time_apply(h, r, z, reps=10, stream=None):
    a, b, c = C.c_double(), C.c_double(), C.c_double()
    _check(lib().sait_time_apply(h, _dptr(r), _dptr(z), int(reps), _stream(stream), C.byref(a), C.byref(b),
                                 C.byref(c)))
    return a.value, b.value, c.value


def sait_copy(src, dst, stream=None):
    """dst <- src with the library's streaming copy kernel (torch tensors)."""
    nbytes = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() < nbytes:
        raise ValueError("dst too small")
    return _check(lib().sait_copy(C.c_void_p(src.data_ptr()), C.c_void_p(dst.data_ptr()), nbytes, _stream(stream)))


def sait_debug_step(n, T, M, tau, max_nnz_row=0, side="left"):
    """T, M: (row_ptr, col_idx, val) host arrays; side "left" (T~ M + I) or
    "right" (M T~ + I).  Returns the device pass as (rp, ci, v)."""
    Trp, Tci, Tv = (np.ascontiguousarray(T[0], np.int32), np.ascontiguousarray(T[1], np.int32),
                    np.ascontiguousarray(T[2], np.float64))
    Mrp, Mci, Mv = (np.ascontiguousarray(M[0], np.int32), np.ascontiguousarray(M[1], np.int32),
                    np.ascontiguousarray(M[2], np.float64))
    cap = int(Mrp[-1]) * max(1, int(np.diff(Trp).max(initial=1))) + n + 1
    orp = np.empty(n + 1, np.int32)
    oci = np.empty(max(cap, 1), np.int32)
    ov = np.empty(max(cap, 1), np.float64)
    nnz = C.c_int64()
    st = lib().sait_debug_step(int(n), _ptr(Trp, C.c_int32), _ptr(Tci, C.c_int32), _ptr(Tv, C.c_double),
                               _ptr(Mrp, C.c_int32), _ptr(Mci, C.c_int32), _ptr(Mv, C.c_double), float(tau),
                               int(max_nnz_row), SIDES[side], int(cap), _ptr(orp, C.c_int32), _ptr(oci, C.c_int32),
                               _ptr(ov, C.c_double), C.byref(nnz))
    _check(st)
    return orp, oci[: nnz.value].copy(), ov[: nnz.value].copy()


# --------------------------------------------------------------------------
# Object interface
# --------------------------------------------------------------------------

@dataclass
class SolveResult:
    status: int
    iterations: int
    restarts: int
    est_relres: float
    true_relres: float


class SaitPreconditioner:
    """Owns a libsait handle built from a host CSR matrix.

    A: any object with ``n``, ``rp``, ``ci``, ``v`` (e.g. workloads.Csr) or
    a scipy sparse matrix.  Keyword options mirror sait_build_opts
    (ilu_kind, ilut_tau, ilut_fill, m, tau, max_nnz_row, pattern_p,
    precision, build_transpose, ilu_level, upper_side: "right" or "left",
    parilu_sweeps).
    """

    def __init__(self, A, nsys: int = 1, sys_ptr=None, stream=None, **opts):
        if hasattr(A, "indptr"):
            import scipy.sparse as sp

            A = sp.csr_matrix(A)
            A.sort_indices()
            n, rp, ci, v = A.shape[0], A.indptr, A.indices, A.data
        else:
            n, rp, ci, v = A.n, A.rp, A.ci, A.v
        self.n = int(n)
        self.nnz = int(rp[-1])
        self.opts = default_build_opts(**opts)
        self.nsys = int(nsys)
        self.handle = sait_build(n, rp, ci, v, nsys, sys_ptr, self.opts, stream)
        self._rows = None

    def close(self):
        if getattr(self, "handle", None):
            sait_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def precision(self) -> str:
        return {SAIT_F64: "f64", SAIT_F32: "f32", SAIT_BF16: "bf16"}[self.opts.precision]

    def query(self) -> dict:
        q = sait_query(self.handle)
        q["ratio_L"] = q["nnz_ML"] / q["nnz_L"] if q["nnz_L"] else 0.0
        q["ratio_U"] = q["nnz_MU"] / q["nnz_U"] if q["nnz_U"] else 0.0
        return q

    def apply(self, r, z=None, transpose=False, stream=None):
        import torch

        if z is None:
            z = torch.empty_like(r)
        nrhs = 1 if r.dim() == 1 else r.shape[1]
        sait_apply(self.handle, r, z, nrhs, nrhs, int(transpose), stream)
        return z

    def matvec(self, x, y=None, transpose=False, stream=None):
        import torch

        if y is None:
            y = torch.empty_like(x)
        nrhs = 1 if x.dim() == 1 else x.shape[1]
        sait_matvec(self.handle, x, y, nrhs, nrhs, int(transpose), stream)
        return y

    def set_preconditioner(self, kind="sait", sweeps=1, stream=None):
        """Preconditioner of later apply / solve calls: "sait" (default),
        "jacobi" (`sweeps` Jacobi sweeps on L, then on U), "exact" (the
        triangular solves with L and U) or "none"."""
        sait_set_preconditioner(self.handle, kind, sweeps, stream)

    def solve(self, b, x=None, transpose=False, restart=30, maxit=10000, rtol=1e-8, flexible=False, stream=None,
              method="gmres"):
        import torch

        if x is None:
            x = torch.zeros_like(b)
        nrhs = 1 if b.dim() == 1 else b.shape[1]
        o = default_solve_opts(restart=restart, maxit=maxit, rtol=rtol, flexible=int(bool(flexible)),
                               method={"gmres": SAIT_METHOD_GMRES, "pcg": SAIT_METHOD_PCG}[method])
        st, infos = sait_solve(self.handle, b, x, nrhs, nrhs, int(transpose), o, self.nsys * nrhs, stream)
        return x, [SolveResult(**i) for i in infos]

    def lobpcg(self, X0, tol=1e-8, maxit=1000, history=False, stream=None):
        """The k = X0.shape[1] smallest eigenpairs by LOBPCG with the current
        preconditioner.  X0: (n, k) float64 device tensor (copied).  Returns
        (lambda (numpy), X (tensor), info dict[, history])."""
        X = X0.contiguous().clone()
        st, lam, info, hist = sait_lobpcg(self.handle, X, X.shape[1], default_eig_opts(maxit=maxit, tol=tol),
                                          history, stream)
        return (lam, X, info, hist) if history else (lam, X, info)

    def export(self, which: str):
        idx = {"A": SAIT_MAT_A, "L": SAIT_MAT_L, "U": SAIT_MAT_U, "ML": SAIT_MAT_ML, "MU": SAIT_MAT_MU}[which]
        if which in ("ML", "MU"):
            rp, ci, v, sv = sait_export(self.handle, idx, stored=True)
            nnz = len(ci)
            if self.opts.precision == SAIT_F32:
                s = sv[: 4 * nnz].view(np.float32).copy()
            elif self.opts.precision == SAIT_BF16:
                s = sv[: 2 * nnz].view(np.uint16).copy()
            else:
                s = sv[: 8 * nnz].view(np.float64).copy()
            return rp, ci, v, s
        return sait_export(self.handle, idx)

    def row_ptr(self, which: str):
        idx = {"A": SAIT_MAT_A, "L": SAIT_MAT_L, "U": SAIT_MAT_U, "ML": SAIT_MAT_ML, "MU": SAIT_MAT_MU}[which]
        return sait_export_row_ptr(self.handle, idx)

    def autotune(self, nrhs: int = 1, stream=None):
        sait_autotune(self.handle, nrhs, stream)
        return sait_get_apply_lanes(self.handle)

    def grad_values(self, lam, x, grad=None, stream=None):
        import torch

        if grad is None:
            grad = torch.empty(self.nnz, dtype=torch.float64, device=lam.device)
        sait_grad_values(self.handle, lam, x, grad, stream)
        return grad
