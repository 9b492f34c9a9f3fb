"""CPU-side checks of the C ABI library: it loads, exports every function that
include/gfem.h declares, and its host-side validation reports bad meshes
without touching a device."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_2103_14870_amd import gfem

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(gfem.LIB_PATH):
        from paper_2103_14870_amd import build

        build.build()
    return gfem.load()


def declared_functions():
    txt = open(os.path.join(ROOT, "include", "gfem.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(gf_[a-z_]+)\s*\(", txt)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for need in ("gf_mesh_create", "gf_step", "gf_get_positions", "gf_get_edge_damage"):
        assert need in names


def test_library_exports_every_declared_symbol(lib):
    names = declared_functions()
    assert len(names) >= 15
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(gfem._SIGS), "binding and header disagree"


def _create(lib, X, tets, **kw):
    p = dict(youngs=1e5, poisson=0.3, density=1000.0, damage_strain=0.01, dt=1e-3, cg_rel_tol=1e-8)
    p.update(kw)
    par = gfem.make_params(p)
    h = C.c_void_p()
    X = np.ascontiguousarray(X, np.float64)
    tets = np.ascontiguousarray(tets, np.int32)
    st = lib.gf_mesh_create(gfem._dptr(X), X.shape[0], gfem._iptr(tets), tets.shape[0], C.byref(par), C.byref(h))
    if st == 0:
        lib.gf_mesh_destroy(h)
    return st, lib.gf_last_error().decode()


X1 = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]], float)


def test_host_validation_errors(lib):
    st, msg = _create(lib, X1, [[0, 1, 2, 4]])
    assert st == gfem.GF_EINVAL and "outside" in msg
    flat = X1.copy()
    flat[3] = [0.5, 0.5, 0.0]
    st, msg = _create(lib, flat, [[0, 1, 2, 3]])
    assert st == gfem.GF_EDEGENERATE
    st, _ = _create(lib, X1, [[0, 1, 1, 2]])
    assert st == gfem.GF_EDEGENERATE
    st, _ = _create(lib, X1, [[0, 1, 2, 3]], poisson=0.5)
    assert st == gfem.GF_EINVAL
    st, _ = _create(lib, X1, [[0, 1, 2, 3]], dt=0.0)
    assert st == gfem.GF_EINVAL
    st, _ = _create(lib, X1, np.zeros((0, 4), np.int32))
    assert st == gfem.GF_EINVAL


def test_null_arguments_are_rejected(lib):
    assert lib.gf_step(None, 1, None) == gfem.GF_EINVAL
    assert lib.gf_get_positions(None, None) == gfem.GF_EINVAL
    assert lib.gf_mesh_destroy(None) == gfem.GF_OK


def test_valid_mesh_without_device_reports_device_error(lib):
    import torch

    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    st, msg = _create(lib, X1, [[0, 1, 3, 2]])
    assert st == gfem.GF_EDEVICE, msg
