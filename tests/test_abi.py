"""The C ABI library loads and exports every function include/sait.h
declares; host-side argument validation works without touching the GPU."""

import ctypes as C
import os
import re

import numpy as np
import pytest

import paper_2106_12836_amd as P
from paper_2106_12836_amd import sait as S

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sait.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sait_\w+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(P.library_path()):
        from paper_2106_12836_amd import build

        build.build()
    return P.lib()


def test_every_declared_symbol_is_exported(lib):
    names = _declared()
    assert len(names) >= 15
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(P.EXPORTED) == names


def test_defaults(lib):
    o = S.default_build_opts()
    assert (o.ilu_kind, o.m, o.tau, o.max_nnz_row, o.pattern_p, o.precision) == (0, 3, 1e-2, 0, -1, 0)
    so = S.default_solve_opts()
    assert (so.restart, so.maxit, so.rtol, so.flexible) == (30, 10000, 1e-8, 0)


def test_host_validation_without_gpu(lib):
    # Malformed inputs are rejected on the host before any device call.
    h = C.c_void_p()
    rp = np.array([0, 2, 3], np.int32)
    ci = np.array([1, 0, 1], np.int32)  # row 0 unsorted
    v = np.ones(3)
    st = lib.sait_build(2, rp.ctypes.data_as(C.POINTER(C.c_int32)), ci.ctypes.data_as(C.POINTER(C.c_int32)),
                        v.ctypes.data_as(C.POINTER(C.c_double)), 1, None, None, None, None, C.byref(h))
    assert st == S.SAIT_E_INVALID and not h.value
    assert "sorted" in P.sait_last_error()
    o = S.default_build_opts(tau=1.5)
    ci = np.array([0, 1, 1], np.int32)
    st = lib.sait_build(2, rp.ctypes.data_as(C.POINTER(C.c_int32)), ci.ctypes.data_as(C.POINTER(C.c_int32)),
                        v.ctypes.data_as(C.POINTER(C.c_double)), 1, None, C.byref(o), None, None, C.byref(h))
    assert st == S.SAIT_E_INVALID and "tau" in P.sait_last_error()
    v2 = np.array([1.0, np.inf, 1.0])
    st = lib.sait_build(2, rp.ctypes.data_as(C.POINTER(C.c_int32)), ci.ctypes.data_as(C.POINTER(C.c_int32)),
                        v2.ctypes.data_as(C.POINTER(C.c_double)), 1, None, None, None, None, C.byref(h))
    assert st == S.SAIT_E_NONFINITE
    # null handle
    assert lib.sait_apply(None, None, None, 1, 1, 0, None) == S.SAIT_E_INVALID
    assert lib.sait_query(None, None, None, None, None, None, None) == S.SAIT_E_INVALID
    lib.sait_destroy(None)
    # debug step: non-triangular T and missing diagonal are host errors
    T = (np.array([0, 2, 4], np.int32), np.array([0, 1, 0, 1], np.int32), np.ones(4))
    M = (np.array([0, 1, 2], np.int32), np.array([0, 1], np.int32), np.ones(2))
    with pytest.raises(P.SaitError) as e:
        P.sait_debug_step(2, T, M, 0.1)
    assert e.value.status == S.SAIT_E_INVALID
    T = (np.array([0, 1, 2], np.int32), np.array([0, 0], np.int32), np.ones(2))
    with pytest.raises(P.SaitError) as e:
        P.sait_debug_step(2, T, M, 0.1)
    assert e.value.status == S.SAIT_E_ZERO_PIVOT


def test_build_opts_layout_matches_header(lib):
    # the C defaults land in the Python struct field by field; a field
    # missing or out of order on either side shifts them
    o = S.default_build_opts()
    assert (o.ilu_kind, o.ilut_tau, o.ilut_fill, o.m, o.tau) == (S.SAIT_ILU0, 1e-3, 10, 3, 1e-2)
    assert (o.max_nnz_row, o.pattern_p, o.precision, o.build_transpose) == (0, -1, S.SAIT_F64, 0)
    assert (o.ilu_level, o.upper_side, o.parilu_sweeps) == (1, S.SAIT_SIDE_RIGHT, 3)
    s = S.default_solve_opts()
    assert (s.restart, s.maxit, s.rtol, s.flexible, s.method) == (30, 10000, 1e-8, 0, 0)
    assert S.default_build_opts(upper_side="left").upper_side == S.SAIT_SIDE_LEFT
