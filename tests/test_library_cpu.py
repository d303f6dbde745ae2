"""Host-side checks of the C ABI that need no GPU: the library loads, exports every entry point that
include/sgheat.h declares, validates descriptions before touching the device, and samples the
coefficient at the same Gauss points as the oracle."""
import ctypes
import os
import re

import numpy as np
import pytest

import sg_inputs
from oracle import fem

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    from paper_2605_21046_amd import sgheat
    return sgheat


def test_library_exports_every_declared_symbol():
    sgheat = _lib()
    header = open(os.path.join(ROOT, "include", "sgheat.h")).read()
    declared = set(re.findall(r"^\s*(?:sg_status|const char\*)\s+(\w+)\s*\(", header, re.M))
    assert declared == set(sgheat.EXPORTS)
    lib = ctypes.CDLL(sgheat.LIB_PATH)
    for name in declared:
        assert hasattr(lib, name), name


@pytest.mark.parametrize("name,level", [("c1", 0), ("c2", 1), ("t2q3", 0), ("t3q4", 0), ("c3", 2)])
def test_quadrature_points_match_oracle(name, level):
    sgheat = _lib()
    w = sg_inputs.WORKLOADS[name]
    spec = sgheat.Spec(w.dim, w.n_cells_1d, w.fe_degree, w.time_degree, w.tau, w.n_vars, w.chaos_degree,
                       w.n_levels)
    pts = sgheat.quadrature_points(spec, level)
    ref = fem.Mesh(w.dim, w.n_cells_1d >> level, w.fe_degree).qp_coords()
    assert np.abs(pts - ref).max() < 1e-15


def _desc(**kw):
    sgheat = _lib()
    spec = sgheat.Spec(2, 4, 2, 1, 0.1, 2, 2, 2)
    d = sgheat._desc(spec)
    mus = (ctypes.c_int * 6)(0, 0, 1, 0, 0, 1)
    coef = (ctypes.c_double * 1)(0.0)
    d.n_coef_modes = 3
    d.coef_mu = ctypes.cast(mus, ctypes.POINTER(ctypes.c_int))
    d.coef_qp = ctypes.cast(coef, ctypes.POINTER(ctypes.c_double))
    for k, v in kw.items():
        setattr(d, k, v)
    return d, (mus, coef)


@pytest.mark.parametrize("field,value", [("dim", 4), ("fe_degree", 0), ("fe_degree", 5), ("time_degree", 4),
                                         ("n_levels", 4), ("tau", 0.0), ("fgmres_restart", 65),
                                         ("precision", 7), ("n_coef_modes", 0), ("hi", -1.0)])
def test_create_rejects_invalid_descriptions(field, value):
    sgheat = _lib()
    d, keep = _desc(**{field: value})
    h = ctypes.c_void_p()
    st = sgheat._lib.sg_create(ctypes.byref(d), ctypes.byref(h))
    assert st == -1 and not h.value
    assert len(sgheat._lib.sg_last_error()) > 0


def test_null_arguments_are_rejected():
    sgheat = _lib()
    assert sgheat._lib.sg_create(None, None) == -1
    assert sgheat._lib.sg_destroy(None) == 0
    assert sgheat._lib.sg_operator_apply(None, None, None, None) == -1
    assert sgheat._lib.gmg_vcycle(None, None, None, None) == -1
    assert sgheat._lib.sg_vanka_smooth(None, 0, None, None, 1, None) == -1
    assert sgheat._lib.fgmres_solve_slab(None, None, None, 1e-8, 10, None, None) == -1
