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
    return sorted(set(re.findall(r"\b(gf_[a-z_0-9]+)\s*\(", txt)))


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


def test_weight_blob_is_validated_on_the_host(lib):
    """The network's weights cross the boundary as a sized, versioned blob;
    every malformed variant is rejected with GF_EINVAL before any device work."""
    n = C.c_int32()
    assert lib.gf_net_num_params(C.byref(n)) == gfem.GF_OK
    good = gfem.weights_blob(np.linspace(-1, 1, n.value).astype(np.float32))
    assert len(good) == 16 + 4 * n.value
    assert gfem.check_weights(good) == gfem.GF_OK
    bad = {
        "short header": good[:12],
        "truncated": good[:-4],
        "trailing byte": good + b"\0",
        "magic": b"XXXX" + good[4:],
        "version": good[:4] + np.array([2], "<u4").tobytes() + good[8:],
        "count": gfem.weights_blob(np.zeros(n.value - 1, np.float32)) + b"\0\0\0\0",
        "dtype": good[:12] + np.array([1], "<u4").tobytes() + good[16:],
        "nan": good[:16] + np.array([np.nan], "<f4").tobytes() + good[20:],
    }
    for what, blob in bad.items():
        assert gfem.check_weights(blob) == gfem.GF_EINVAL, what
        assert lib.gf_last_error().decode(), what
    assert lib.gf_net_check_weights(None, 0) == gfem.GF_EINVAL
    # a null network is rejected before the blob is read
    buf = C.create_string_buffer(good, len(good))
    assert lib.gf_net_set_weights(None, buf, len(good)) == gfem.GF_EINVAL
    sz = C.c_size_t()
    assert lib.gf_net_get_weights(None, None, C.byref(sz)) == gfem.GF_EINVAL


def test_shipped_weights_pass_the_blob_check(lib):
    w = np.load(os.path.join(ROOT, "paper_2103_14870_amd", "weights", "precond_net.npy"))
    assert gfem.check_weights(gfem.weights_blob(w)) == gfem.GF_OK
