"""Thin ctypes binding of libgfem.so (include/gfem.h).

Argument marshalling only: every step of the method runs in the HIP library.
If the library is missing or cannot be loaded this module raises; there is no
CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgfem.so")

GF_OK, GF_EINVAL, GF_EDEGENERATE, GF_ENOMEM, GF_EDEVICE, GF_ENOTCONVERGED, GF_ESTATE = 0, -1, -2, -3, -4, -5, -6
STATUS_NAMES = {0: "GF_OK", -1: "GF_EINVAL", -2: "GF_EDEGENERATE", -3: "GF_ENOMEM", -4: "GF_EDEVICE",
                -5: "GF_ENOTCONVERGED", -6: "GF_ESTATE"}
PREC = {"fp64": 0, "split": 1}
PRECOND = {"block_jacobi": 0, "learned": 1}
ENERGY = {"stable_neo_hookean": 0, "stvk": 1}
REORDER = {"none": 0, "rcm": 1}
KERNEL_CATEGORIES = ("damage", "element", "assembly", "precond", "spmv", "pcg_vector", "residual", "integrate",
                     "precond_gt")


class GfParams(C.Structure):
    _fields_ = [("youngs", C.c_double), ("poisson", C.c_double), ("density", C.c_double),
                ("damage_strain", C.c_double), ("damage_radius", C.c_double), ("yield_strain", C.c_double),
                ("dt", C.c_double),
                ("rayleigh_alpha", C.c_double), ("rayleigh_beta", C.c_double), ("gravity", C.c_double * 3),
                ("cg_rel_tol", C.c_double), ("cg_max_iter", C.c_int32), ("precision", C.c_int32),
                ("precond", C.c_int32), ("net_every_n_steps", C.c_int32), ("energy", C.c_int32),
                ("reorder", C.c_int32)]


class GfStepStats(C.Structure):
    _fields_ = [("steps_done", C.c_int32), ("inner_iters", C.c_int32), ("outer_iters", C.c_int32),
                ("used_fallback", C.c_int32), ("new_broken", C.c_int32), ("total_broken", C.c_int32),
                ("near_threshold", C.c_int32), ("chi_zero_tets", C.c_int32), ("degenerate_tets", C.c_int32),
                ("fp64_steps", C.c_int32),
                ("n_launch", C.c_int32 * 9), ("rel_residual", C.c_double), ("kernel_us", C.c_double * 9)]

    def as_dict(self) -> dict:
        d = {f: getattr(self, f) for f, _ in self._fields_ if f not in ("n_launch", "kernel_us")}
        d["kernel_us"] = {k: float(self.kernel_us[i]) for i, k in enumerate(KERNEL_CATEGORIES)}
        d["n_launch"] = {k: int(self.n_launch[i]) for i, k in enumerate(KERNEL_CATEGORIES)}
        return d


class GfQsStats(C.Structure):
    _fields_ = [("steps_done", C.c_int32), ("newton_iters", C.c_int32), ("line_search_halvings", C.c_int32),
                ("inner_iters", C.c_int32), ("new_broken", C.c_int32), ("total_broken", C.c_int32),
                ("force_initial", C.c_double), ("force_residual", C.c_double), ("energy", C.c_double)]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_}


class GfemError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


_lib = None
_lib_path = None

_P = C.POINTER
_SIGS = {
    "gf_mesh_create": ([_P(C.c_double), C.c_int32, _P(C.c_int32), C.c_int32, _P(GfParams), _P(C.c_void_p)], C.c_int),
    "gf_mesh_destroy": ([C.c_void_p], C.c_int),
    "gf_set_stream": ([C.c_void_p, C.c_void_p], C.c_int),
    "gf_get_sizes": ([C.c_void_p, _P(C.c_int32), _P(C.c_int32), _P(C.c_int32), _P(C.c_int32)], C.c_int),
    "gf_get_edges": ([C.c_void_p, _P(C.c_int32)], C.c_int),
    "gf_set_dirichlet": ([C.c_void_p, _P(C.c_int32), C.c_int32, _P(C.c_double)], C.c_int),
    "gf_set_edge_damage": ([C.c_void_p, _P(C.c_uint8)], C.c_int),
    "gf_step": ([C.c_void_p, C.c_int32, _P(GfStepStats)], C.c_int),
    "gf_quasi_static_step": ([C.c_void_p, C.c_int32, C.c_double, C.c_int32, C.c_double, _P(GfQsStats)], C.c_int),
    "gf_quasi_static_step_noalloc": ([C.c_void_p, C.c_int32, C.c_double, C.c_int32, C.c_double, _P(GfQsStats)],
                                     C.c_int),
    "gf_get_visual_mesh": ([C.c_void_p, _P(C.c_double), _P(C.c_uint8)], C.c_int),
    "gf_get_positions": ([C.c_void_p, _P(C.c_double)], C.c_int),
    "gf_get_velocities": ([C.c_void_p, _P(C.c_double)], C.c_int),
    "gf_get_edge_damage": ([C.c_void_p, _P(C.c_uint8)], C.c_int),
    "gf_eval_forces": ([C.c_void_p, _P(C.c_double)], C.c_int),
    "gf_get_near_threshold_edges": ([C.c_void_p, _P(C.c_int32), C.c_int32, _P(C.c_int32)], C.c_int),
    "gf_get_system": ([C.c_void_p, _P(C.c_int32), _P(C.c_int32), _P(C.c_double), _P(C.c_double)], C.c_int),
    "gf_get_state": ([C.c_void_p, C.c_void_p, _P(C.c_size_t)], C.c_int),
    "gf_set_state": ([C.c_void_p, C.c_void_p, C.c_size_t], C.c_int),
    "gf_set_timing": ([C.c_void_p, C.c_int32], C.c_int),
    "gf_set_fp64_rerun": ([C.c_void_p, C.c_int32], C.c_int),
    "gf_bench_spmv": ([C.c_void_p, C.c_int32, _P(C.c_double), _P(C.c_double)], C.c_int),
    "gf_last_error": ([], C.c_char_p),
    "gf_net_create": ([C.c_uint64, _P(C.c_void_p)], C.c_int),
    "gf_net_destroy": ([C.c_void_p], C.c_int),
    "gf_net_num_params": ([_P(C.c_int32)], C.c_int),
    "gf_net_check_weights": ([C.c_void_p, C.c_size_t], C.c_int),
    "gf_net_get_weights": ([C.c_void_p, C.c_void_p, _P(C.c_size_t)], C.c_int),
    "gf_net_set_weights": ([C.c_void_p, C.c_void_p, C.c_size_t], C.c_int),
    "gf_set_precond_net": ([C.c_void_p, C.c_void_p], C.c_int),
    "gf_set_precond": ([C.c_void_p, C.c_int32], C.c_int),
    "gf_set_precond_normalise": ([C.c_void_p, C.c_int32], C.c_int),
    "gf_net_train_step": ([C.c_void_p, C.c_void_p, C.c_double, _P(C.c_double)], C.c_int),
    "gf_net_set_power_steps": ([C.c_void_p, C.c_int32], C.c_int),
    "gf_net_eval": ([C.c_void_p, C.c_void_p, _P(C.c_double), _P(C.c_double), _P(C.c_float), _P(C.c_float),
                     _P(C.c_float)], C.c_int),
}


def load(path: str | None = None):
    """Load libgfem.so, or the library at `path` (raises if it is not
    built).  A process holds one library: with no path the loaded one is
    returned, and naming another file once one is loaded raises."""
    global _lib, _lib_path
    if _lib is not None:
        if path is not None and os.path.realpath(path) != _lib_path:
            raise RuntimeError(f"{_lib_path} is already loaded; cannot also load {path}")
        return _lib
    path = LIB_PATH if path is None else path
    if not os.path.exists(path):
        raise FileNotFoundError(f"{path} is not built; run __graft_entry__.build() first")
    lib = C.CDLL(path)
    for name, (args, res) in _SIGS.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib, _lib_path = lib, os.path.realpath(path)
    return lib


def _check(status: int):
    if status != GF_OK:
        raise GfemError(status, (load().gf_last_error() or b"").decode())


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(_P(C.c_double))


def _iptr(a: np.ndarray):
    return a.ctypes.data_as(_P(C.c_int32))


def _u8ptr(a: np.ndarray):
    return a.ctypes.data_as(_P(C.c_uint8))


def make_params(p: dict) -> GfParams:
    g = p.get("gravity", (0.0, 0.0, 0.0))
    return GfParams(float(p["youngs"]), float(p["poisson"]), float(p["density"]), float(p["damage_strain"]),
                    float(p.get("damage_radius", 0.0)), float(p.get("yield_strain", 0.0)), float(p["dt"]),
                    float(p.get("rayleigh_alpha", 0.0)),
                    float(p.get("rayleigh_beta", 0.0)), (C.c_double * 3)(*[float(x) for x in g]),
                    float(p["cg_rel_tol"]), int(p.get("cg_max_iter", 5000)), PREC[p.get("precision", "fp64")],
                    PRECOND[p.get("precond", "block_jacobi")], int(p.get("net_every_n_steps", 1)),
                    ENERGY[p.get("energy", "stable_neo_hookean")], REORDER[p.get("reorder", "none")])


class Mesh:
    """One simulated mesh living on the current HIP device."""

    def __init__(self, X: np.ndarray, tets: np.ndarray, params: dict):
        lib = load()
        X = np.ascontiguousarray(X, dtype=np.float64)
        tets = np.ascontiguousarray(tets, dtype=np.int32)
        if X.ndim != 2 or X.shape[1] != 3 or tets.ndim != 2 or tets.shape[1] != 4:
            raise ValueError("X must be (n,3) and tets (m,4)")
        self._lib = lib
        self._h = C.c_void_p()
        self._params = make_params(params)
        _check(lib.gf_mesh_create(_dptr(X), X.shape[0], _iptr(tets), tets.shape[0], C.byref(self._params),
                                  C.byref(self._h)))
        n, m, ne, nb = C.c_int32(), C.c_int32(), C.c_int32(), C.c_int32()
        _check(lib.gf_get_sizes(self._h, C.byref(n), C.byref(m), C.byref(ne), C.byref(nb)))
        self.n_nodes, self.n_tets, self.n_edges, self.n_blocks = n.value, m.value, ne.value, nb.value
        self._edges = None

    def close(self):
        if self._h:
            self._lib.gf_mesh_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # -- inputs
    def set_stream(self, stream_handle: int | None):
        _check(self._lib.gf_set_stream(self._h, C.c_void_p(stream_handle or 0)))

    def set_dirichlet(self, nodes, vel):
        nodes = np.ascontiguousarray(nodes, dtype=np.int32)
        vel = np.ascontiguousarray(vel, dtype=np.float64).reshape(-1, 3)
        _check(self._lib.gf_set_dirichlet(self._h, _iptr(nodes), nodes.size, _dptr(vel)))

    def set_edge_damage(self, zeta):
        z = np.ascontiguousarray(zeta, dtype=np.uint8)
        if z.size != self.n_edges:
            raise ValueError("zeta must have n_edges entries")
        _check(self._lib.gf_set_edge_damage(self._h, _u8ptr(z)))

    def break_pairs(self, pairs):
        """OR-in damage for node pairs (i, j); each pair must be a mesh edge."""
        pairs = np.asarray(pairs, dtype=np.int64).reshape(-1, 2)
        if pairs.size == 0:
            return
        e = self.edges().astype(np.int64)
        key = e[:, 0] * (self.n_nodes + 1) + e[:, 1]
        ps = np.sort(pairs, axis=1)
        pk = ps[:, 0] * (self.n_nodes + 1) + ps[:, 1]
        idx = np.searchsorted(key, pk)
        if np.any(idx >= key.size) or np.any(key[np.minimum(idx, key.size - 1)] != pk):
            raise ValueError("a pair is not an edge of the mesh")
        z = np.zeros(self.n_edges, np.uint8)
        z[idx] = 1
        self.set_edge_damage(z)

    # -- stepping
    def step(self, n_steps: int = 1, raise_on_error: bool = True) -> dict:
        st = GfStepStats()
        s = self._lib.gf_step(self._h, int(n_steps), C.byref(st))
        d = st.as_dict()
        d["status"] = s
        if s != GF_OK and raise_on_error:
            _check(s)
        return d

    def quasi_static_step(self, n_steps: int = 1, newton_rel_tol: float = 1e-6, max_newton: int = 50,
                          armijo: float = 1e-4, raise_on_error: bool = True, noalloc: bool = False) -> dict:
        """Quasi-static load steps (Eq. 36): Newton with a backtracking line search.
        noalloc: the allocation-free entry point (fixed library scratch)."""
        st = GfQsStats()
        fn = self._lib.gf_quasi_static_step_noalloc if noalloc else self._lib.gf_quasi_static_step
        s = fn(self._h, int(n_steps), float(newton_rel_tol), int(max_newton), float(armijo), C.byref(st))
        d = st.as_dict()
        d["status"] = s
        if s != GF_OK and raise_on_error:
            _check(s)
        return d

    # -- outputs
    def edges(self) -> np.ndarray:
        if self._edges is None:
            e = np.zeros((self.n_edges, 2), np.int32)
            _check(self._lib.gf_get_edges(self._h, _iptr(e)))
            self._edges = e
        return self._edges

    def positions(self) -> np.ndarray:
        x = np.zeros((self.n_nodes, 3))
        _check(self._lib.gf_get_positions(self._h, _dptr(x)))
        return x

    def visual_mesh(self):
        """Split visualisation mesh (Sec. 4.1): sub-cell vertices (n_tets, 4, 8, 3)
        and corner groups (n_tets, 4)."""
        xyz = np.zeros((self.n_tets, 4, 8, 3))
        grp = np.zeros((self.n_tets, 4), np.uint8)
        _check(self._lib.gf_get_visual_mesh(self._h, _dptr(xyz), _u8ptr(grp)))
        return xyz, grp

    def velocities(self) -> np.ndarray:
        v = np.zeros((self.n_nodes, 3))
        _check(self._lib.gf_get_velocities(self._h, _dptr(v)))
        return v

    def edge_damage(self) -> np.ndarray:
        z = np.zeros(self.n_edges, np.uint8)
        _check(self._lib.gf_get_edge_damage(self._h, _u8ptr(z)))
        return z

    def near_threshold_edges(self) -> np.ndarray:
        """Canonical ids of the edges within 1e-6 of the threshold in the last damage pass."""
        n = C.c_int32()
        _check(self._lib.gf_get_near_threshold_edges(self._h, None, 0, C.byref(n)))
        ids = np.zeros(max(n.value, 1), np.int32)
        _check(self._lib.gf_get_near_threshold_edges(self._h, _iptr(ids), ids.size, C.byref(n)))
        return ids[: n.value]

    def eval_forces(self) -> np.ndarray:
        f = np.zeros((self.n_nodes, 3))
        _check(self._lib.gf_eval_forces(self._h, _dptr(f)))
        return f

    def get_system(self):
        """(bi, bj, blocks (nb,3,3), rhs (n,3)) of the next step's system."""
        bi = np.zeros(self.n_blocks, np.int32)
        bj = np.zeros(self.n_blocks, np.int32)
        vals = np.zeros((self.n_blocks, 3, 3))
        rhs = np.zeros((self.n_nodes, 3))
        _check(self._lib.gf_get_system(self._h, _iptr(bi), _iptr(bj), _dptr(vals), _dptr(rhs)))
        return bi, bj, vals, rhs

    def get_state(self) -> bytes:
        n = C.c_size_t()
        _check(self._lib.gf_get_state(self._h, None, C.byref(n)))
        buf = C.create_string_buffer(n.value)
        _check(self._lib.gf_get_state(self._h, buf, C.byref(n)))
        return buf.raw[: n.value]

    def set_state(self, blob: bytes):
        buf = C.create_string_buffer(blob, len(blob))
        _check(self._lib.gf_set_state(self._h, buf, len(blob)))

    def set_fp64_rerun(self, always: bool):
        """Test hook: re-run every split-precision step in FP64."""
        _check(self._lib.gf_set_fp64_rerun(self._h, int(bool(always))))

    def set_timing(self, on: bool):
        _check(self._lib.gf_set_timing(self._h, int(bool(on))))

    def bench_spmv(self, reps: int = 50):
        us, by = C.c_double(), C.c_double()
        _check(self._lib.gf_bench_spmv(self._h, int(reps), C.byref(us), C.byref(by)))
        return us.value, by.value


class Net:
    """Learned block preconditioner network (lives on the current HIP device)."""

    def __init__(self, seed: int = 0):
        self._lib = load()
        self._h = C.c_void_p()
        _check(self._lib.gf_net_create(C.c_uint64(seed), C.byref(self._h)))
        n = C.c_int32()
        _check(self._lib.gf_net_num_params(C.byref(n)))
        self.n_params = n.value

    def close(self):
        if self._h:
            self._lib.gf_net_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def get_weights(self) -> np.ndarray:
        n = C.c_size_t()
        _check(self._lib.gf_net_get_weights(self._h, None, C.byref(n)))
        buf = C.create_string_buffer(n.value)
        _check(self._lib.gf_net_get_weights(self._h, buf, C.byref(n)))
        return weights_from_blob(buf.raw[: n.value])

    def set_weights(self, w):
        """FP32 weights (n_params) or a weight blob (bytes)."""
        blob = w if isinstance(w, (bytes, bytearray)) else weights_blob(w)
        buf = C.create_string_buffer(bytes(blob), len(blob))
        _check(self._lib.gf_net_set_weights(self._h, buf, len(blob)))

    def set_power_steps(self, k: int):
        """Power steps on G A G^T applied to the training probe (0: Kaporin)."""
        _check(self._lib.gf_net_set_power_steps(self._h, int(k)))

    def train_step(self, mesh: "Mesh", lr: float) -> float:
        loss = C.c_double()
        _check(self._lib.gf_net_train_step(self._h, mesh._h, float(lr), C.byref(loss)))
        return loss.value

    def eval(self, mesh: "Mesh", probe=None):
        """(loss, diagonal factor blocks (n,3,3), lower blocks G_ji of the
        canonical edges (ne,3,3), weight gradient) on the mesh's next system.
        probe: (n,3) array of +-1 (caller order) or None for the generator's."""
        loss = C.c_double()
        gd = np.zeros((mesh.n_nodes, 3, 3), np.float32)
        gl = np.zeros((mesh.n_edges, 3, 3), np.float32)
        grad = np.zeros(self.n_params, np.float32)
        pv = None
        if probe is not None:
            pv = np.ascontiguousarray(probe, dtype=np.float64).reshape(mesh.n_nodes, 3)
        _check(self._lib.gf_net_eval(self._h, mesh._h, pv.ctypes.data_as(_P(C.c_double)) if pv is not None else None,
                                     C.byref(loss), gd.ctypes.data_as(_P(C.c_float)),
                                     gl.ctypes.data_as(_P(C.c_float)), grad.ctypes.data_as(_P(C.c_float))))
        return loss.value, gd, gl, grad


NET_BLOB_MAGIC, NET_BLOB_VERSION = 0x574E4647, 1


def weights_blob(w) -> bytes:
    """Header (magic, version, parameter count, type 0 = FP32) + FP32 weights."""
    w = np.ascontiguousarray(w, dtype=np.float32).ravel()
    hdr = np.array([NET_BLOB_MAGIC, NET_BLOB_VERSION, w.size, 0], dtype="<u4")
    return hdr.tobytes() + w.astype("<f4").tobytes()


def weights_from_blob(blob: bytes) -> np.ndarray:
    hdr = np.frombuffer(blob[:16], dtype="<u4")
    return np.frombuffer(blob[16:], dtype="<f4", count=int(hdr[2])).copy()


def check_weights(blob: bytes) -> int:
    """Host-only validation of a weight blob through the library (status)."""
    buf = C.create_string_buffer(bytes(blob), len(blob)) if blob is not None else None
    return load().gf_net_check_weights(buf, len(blob) if blob is not None else 0)


def attach_net(mesh: "Mesh", net: "Net | None", use: bool = True):
    _check(load().gf_set_precond_net(mesh._h, net._h if net is not None else None))
    _check(load().gf_set_precond(mesh._h, PRECOND["learned"] if (use and net is not None) else 0))


def set_precond_normalise(mesh: "Mesh", on: bool):
    """Row normalisation of the learned factor ((G A G^T)_ii = I per block row)."""
    _check(load().gf_set_precond_normalise(mesh._h, int(bool(on))))


def set_precond(mesh: "Mesh", name: str):
    _check(load().gf_set_precond(mesh._h, PRECOND[name]))


def mesh_from_problem(prob) -> Mesh:
    """Create a Mesh for a meshgen.Problem: Dirichlet set and pre-broken pairs applied."""
    m = Mesh(prob.X, prob.tets, prob.params)
    if prob.dir_nodes.size:
        m.set_dirichlet(prob.dir_nodes, prob.dir_vel)
    if prob.broken_pairs.size:
        m.break_pairs(prob.broken_pairs)
    return m


def state_blob_layout(n_nodes: int, n_edges: int, n_tets: int, plastic: bool):
    """Offsets of the checkpoint blob fields: header 32 B; U, V as (n,3) f64 in
    caller order; zeta (n_edges) u8 in canonical order; plastic Gram offsets
    (6, n_tets) f64 when present."""
    u = 32
    v = u + 24 * n_nodes
    z = v + 24 * n_nodes
    p = z + n_edges
    end = p + (48 * n_tets if plastic else 0)
    return dict(U=u, V=v, zeta=z, plastic=p, end=end)


def set_displacement(mesh: Mesh, U: np.ndarray, V: np.ndarray | None = None):
    """Overwrite the displacement (and optionally velocity) through the checkpoint blob."""
    blob = bytearray(mesh.get_state())
    plastic = len(blob) > 32 + 48 * mesh.n_nodes + mesh.n_edges
    lay = state_blob_layout(mesh.n_nodes, mesh.n_edges, mesh.n_tets, plastic)
    blob[lay["U"]:lay["V"]] = np.ascontiguousarray(U, dtype=np.float64).tobytes()
    if V is not None:
        blob[lay["V"]:lay["zeta"]] = np.ascontiguousarray(V, dtype=np.float64).tobytes()
    mesh.set_state(bytes(blob))
