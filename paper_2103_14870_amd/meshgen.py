"""Seeded synthetic inputs for the graph-based FEM fracture step.

This module only builds *inputs*: tetrahedral meshes, material/solver parameter
sets, prescribed-velocity (Dirichlet) node sets and pre-broken edge sets.  It
holds none of the method's arithmetic (no energy, force, stiffness, damage
criterion or solver), so both the HIP library and the CPU oracle can consume
its output without sharing any computation.

The meshes stand in for the paper's scanned models (Sec. 4.3, Table 2), which
are not available: structured grids of cubes, each cut into six tetrahedra
along the cube's main diagonal (Freudenthal/Kuhn split), optionally clipped to
an ellipsoid and jittered.  Tetrahedra are emitted in their natural vertex
order, so about half of them are negatively oriented; consumers reorient.
"""
from __future__ import annotations

import itertools
from dataclasses import dataclass, field

import numpy as np

# The six tets of a unit cube: walk from corner (0,0,0) to (1,1,1) along the
# axes in the order given by each permutation of (0, 1, 2).
_PERMS = list(itertools.permutations((0, 1, 2)))


@dataclass
class Problem:
    """One simulation input: mesh, parameters, boundary conditions."""

    name: str
    X: np.ndarray                 # (n_nodes, 3) float64 rest positions
    tets: np.ndarray              # (n_tets, 4) int32, any orientation
    params: dict                  # mirrors the library's parameter struct
    dir_nodes: np.ndarray         # (k,) int32 nodes with prescribed velocity
    dir_vel: np.ndarray           # (k, 3) float64 prescribed velocity [m/s]
    broken_pairs: np.ndarray      # (p, 2) int32 node pairs (i < j) pre-broken
    n_steps: int
    meta: dict = field(default_factory=dict)

    @property
    def n_nodes(self) -> int:
        return int(self.X.shape[0])

    @property
    def n_tets(self) -> int:
        return int(self.tets.shape[0])


def default_params(**kw) -> dict:
    p = dict(youngs=1e5, poisson=0.3, density=1000.0, damage_strain=0.01, damage_radius=0.0,
             yield_strain=0.0, dt=1e-3, rayleigh_alpha=0.0, rayleigh_beta=0.0,
             gravity=(0.0, 0.0, 0.0), cg_rel_tol=1e-8, cg_max_iter=5000,
             precision="fp64", precond="block_jacobi", net_every_n_steps=1, energy="stable_neo_hookean")
    p.update(kw)
    return p


def grid_nodes(nx: int, ny: int, nz: int, h: float, origin=(0.0, 0.0, 0.0)) -> np.ndarray:
    """Nodes of an (nx+1)x(ny+1)x(nz+1) lattice, id = i + (nx+1)*(j + (ny+1)*k)."""
    i, j, k = np.meshgrid(np.arange(nx + 1), np.arange(ny + 1), np.arange(nz + 1), indexing="ij")
    ijk = np.stack([i.ravel(order="F"), j.ravel(order="F"), k.ravel(order="F")], axis=1)
    return ijk.astype(np.float64) * h + np.asarray(origin, dtype=np.float64)


def freudenthal_tets(nx: int, ny: int, nz: int, keep: np.ndarray | None = None):
    """Six tets per kept cube (cube order i fastest, then j, then k).

    Returns (tets (m,4) int64 lattice node ids, cube_ijk (m,3) int64).
    `keep` is an optional boolean array of shape (nx, ny, nz)."""
    sx, sy = nx + 1, (nx + 1) * (ny + 1)
    ci, cj, ck = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    cubes = np.stack([ci.ravel(order="F"), cj.ravel(order="F"), ck.ravel(order="F")], axis=1)
    if keep is not None:
        cubes = cubes[keep.ravel(order="F")]
    base = cubes[:, 0] + sx * cubes[:, 1] + sy * cubes[:, 2]
    step = np.array([1, sx, sy])
    tets = np.empty((cubes.shape[0], 6, 4), dtype=np.int64)
    for t, perm in enumerate(_PERMS):
        off = np.zeros(4, dtype=np.int64)
        acc = 0
        for v, axis in enumerate(perm):
            acc += step[axis]
            off[v + 1] = acc
        tets[:, t, :] = base[:, None] + off[None, :]
    cube_ijk = np.repeat(cubes, 6, axis=0)
    return tets.reshape(-1, 4), cube_ijk


def compact(X: np.ndarray, tets: np.ndarray):
    """Drop unreferenced nodes, keeping the remaining ones in their order."""
    used = np.zeros(X.shape[0], dtype=bool)
    used[tets.ravel()] = True
    new_id = -np.ones(X.shape[0], dtype=np.int64)
    new_id[used] = np.arange(int(used.sum()))
    return X[used].copy(), new_id[tets], np.nonzero(used)[0]


def jitter(X: np.ndarray, amp: float, seed: int) -> np.ndarray:
    """Uniform per-component perturbation in (-amp, amp), canonical node order."""
    rng = np.random.default_rng(seed)
    return X + rng.uniform(-1.0, 1.0, size=X.shape) * amp


def unique_edges(tets: np.ndarray) -> np.ndarray:
    """All distinct node pairs (i < j) joined by a tet edge, lexicographic."""
    pairs = np.concatenate([tets[:, [a, b]] for a, b in itertools.combinations(range(4), 2)])
    pairs = np.sort(pairs, axis=1)
    return np.unique(pairs, axis=0)


def tet_pairs(tets: np.ndarray) -> np.ndarray:
    """All node pairs (i < j) of the given tets (duplicates removed)."""
    if tets.shape[0] == 0:
        return np.zeros((0, 2), dtype=np.int32)
    return unique_edges(tets).astype(np.int32)


# --------------------------------------------------------------------------
# Workloads
# --------------------------------------------------------------------------

def cube_block(nx=10, ny=10, nz=10, h=0.1, jitter_frac=0.05, seed=0, top_speed=5.0,
               **param_kw) -> Problem:
    """Unit-cube style block: bottom face fixed, top face moved along +z.

    Defaults are the 10x10x10 cube (6000 tets, 1331 nodes), E=1e5, nu=0.3,
    rho=1000, brittle Green-strain threshold 0.01, top face +5 m/s (0.5 % of
    the 1 m side per 1 ms step), FP64, block-Jacobi PCG to 1e-8, 50 steps."""
    X = grid_nodes(nx, ny, nz, h)
    tets, _ = freudenthal_tets(nx, ny, nz)
    if jitter_frac > 0:
        X = jitter(X, jitter_frac * h, seed)
    k = np.rint((grid_nodes(nx, ny, nz, 1.0))[:, 2]).astype(np.int64)
    bottom = np.nonzero(k == 0)[0]
    top = np.nonzero(k == nz)[0]
    nodes = np.concatenate([bottom, top]).astype(np.int32)
    vel = np.zeros((nodes.size, 3))
    vel[bottom.size:, 2] = top_speed
    params = default_params(youngs=1e5, poisson=0.3, density=1000.0, damage_strain=0.01,
                            dt=1e-3, cg_rel_tol=1e-8, precision="fp64")
    params.update(param_kw)
    return Problem(f"cube{nx}x{ny}x{nz}", X, tets.astype(np.int32), params, nodes, vel,
                   np.zeros((0, 2), np.int32), 50, dict(h=h, shape=(nx, ny, nz)))


def notched_beam(nx=80, ny=16, nz=16, h=0.01, notch_cells=4, notch_width=2,
                 crack_fraction=0.0, crack_seed=11, **param_kw) -> Problem:
    """Three-point bending of a notched beam (stand-in for the Charpy/Izod bars).

    Defaults: 80x16x16 cubes of h=1 cm (122,880 tets), E=3e9, nu=0.35,
    rho=1000, threshold 0.005, dt=1e-4, 200 steps, PCG to 1e-6, split
    precision.  The notch is a set of pre-broken edges: every edge of every
    tet in the `notch_width` cube columns at midspan, `notch_cells` cubes deep
    from the bottom face (the mesh itself is unchanged).  Supports: bottom node
    lines at x=0 and x=L fixed; load: top node line at midspan moved down by
    h/400 per step.  `crack_fraction` > 0 adds random planar cracks (seeded)
    until that fraction of all edges is broken."""
    X = grid_nodes(nx, ny, nz, h)
    tets, cube = freudenthal_tets(nx, ny, nz)
    lat = np.rint(grid_nodes(nx, ny, nz, 1.0)).astype(np.int64)
    mid = nx // 2
    n0 = mid - notch_width // 2
    in_notch = (cube[:, 0] >= n0) & (cube[:, 0] < n0 + notch_width) & (cube[:, 2] < notch_cells)
    broken = tet_pairs(tets[in_notch])
    sup = np.nonzero(((lat[:, 0] == 0) | (lat[:, 0] == nx)) & (lat[:, 2] == 0))[0]
    load = np.nonzero((lat[:, 0] == mid) & (lat[:, 2] == nz))[0]
    params = default_params(youngs=3e9, poisson=0.35, density=1000.0, damage_strain=0.005,
                            dt=1e-4, cg_rel_tol=1e-6, precision="split")
    params.update(param_kw)
    speed = (h / 400.0) / params["dt"]
    nodes = np.concatenate([sup, load]).astype(np.int32)
    vel = np.zeros((nodes.size, 3))
    vel[sup.size:, 2] = -speed
    if crack_fraction > 0:
        extra = planar_cracks(X, tets, crack_fraction, crack_seed, already=broken)
        broken = np.unique(np.concatenate([broken, extra]), axis=0).astype(np.int32)
    return Problem(f"beam{nx}x{ny}x{nz}", X, tets.astype(np.int32), params, nodes, vel,
                   broken.astype(np.int32), 200,
                   dict(h=h, shape=(nx, ny, nz), crack_fraction=crack_fraction))


def ellipsoid(h=0.02165, axes=(1.0, 0.5, 0.5), grid=(95, 49, 49), jitter_frac=0.10, seed=7,
              cap=0.9, pull_per_step=0.01, dt=1e-2, **param_kw) -> Problem:
    """Ductile ellipsoid pulled apart at both end caps (stand-in for the 620k-tet loaf).

    Defaults: semi-axes (1.0, 0.5, 0.5) m voxelised on a 95x49x49 lattice of
    h=2.165 cm; a cube is kept when its centre lies inside the ellipsoid,
    giving 103,305 cubes = 619,830 tets and 111,912 nodes.  Jitter +-10 % of h
    (seed 7), E=5e4, nu=0.45, rho=1000, yield strain 0.05, damage threshold
    0.3; nodes with |x| >= 0.9 m move apart at 1 cm per step each."""
    nx, ny, nz = grid
    ox = -(nx / 2.0) * h
    oy = -(ny / 2.0) * h
    oz = -(nz / 2.0) * h
    Xl = grid_nodes(nx, ny, nz, h, origin=(ox, oy, oz))
    ci, cj, ck = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    cx = ox + (ci + 0.5) * h
    cy = oy + (cj + 0.5) * h
    cz = oz + (ck + 0.5) * h
    keep = (cx / axes[0]) ** 2 + (cy / axes[1]) ** 2 + (cz / axes[2]) ** 2 < 1.0
    tets, _ = freudenthal_tets(nx, ny, nz, keep)
    X, tets, _ = compact(Xl, tets)
    if jitter_frac > 0:
        X = jitter(X, jitter_frac * h, seed)
    right = np.nonzero(X[:, 0] >= cap)[0]
    left = np.nonzero(X[:, 0] <= -cap)[0]
    params = default_params(youngs=5e4, poisson=0.45, density=1000.0, damage_strain=0.3,
                            yield_strain=0.05, dt=dt, cg_rel_tol=1e-6, precision="split")
    params.update(param_kw)
    speed = pull_per_step / params["dt"]
    nodes = np.concatenate([right, left]).astype(np.int32)
    vel = np.zeros((nodes.size, 3))
    vel[: right.size, 0] = speed
    vel[right.size:, 0] = -speed
    return Problem(f"ellipsoid{nx}x{ny}x{nz}", X, tets.astype(np.int32), params, nodes, vel,
                   np.zeros((0, 2), np.int32), 300, dict(h=h, grid=grid, cubes=int(keep.sum())))


def planar_cracks(X: np.ndarray, tets: np.ndarray, fraction: float, seed: int,
                  already: np.ndarray | None = None) -> np.ndarray:
    """Random planar crack discs until `fraction` of all edges are broken.

    Each crack is a disc: a centre drawn uniformly in the bounding box, a
    normal drawn uniformly on the sphere and a radius in [0.25, 0.5] of the box
    diagonal.  It breaks the edges whose endpoints lie on opposite sides of its
    plane and whose crossing point is inside the disc.  Cracks are added until
    the target count is reached; the last one is applied partially, crossing
    points nearest to its centre first.  Returns (p, 2) node pairs."""
    edges = unique_edges(tets)
    target = int(round(fraction * edges.shape[0]))
    rng = np.random.default_rng(seed)
    broken = np.zeros(edges.shape[0], dtype=bool)
    if already is not None and already.size:
        key = edges[:, 0] * (X.shape[0] + 1) + edges[:, 1]
        akey = already[:, 0].astype(np.int64) * (X.shape[0] + 1) + already[:, 1]
        broken |= np.isin(key, akey)
    base = int(broken.sum())
    target = base + target
    lo, hi = X.min(axis=0), X.max(axis=0)
    diag = float(np.linalg.norm(hi - lo))
    xa, xb = X[edges[:, 0]], X[edges[:, 1]]
    for _ in range(10000):
        if broken.sum() >= target:
            break
        c = rng.uniform(lo, hi)
        n = rng.normal(size=3)
        n /= np.linalg.norm(n)
        r = rng.uniform(0.25, 0.5) * diag
        da = (xa - c) @ n
        db = (xb - c) @ n
        cross = (da * db) < 0
        t = np.where(cross, da / np.where(cross, da - db, 1.0), 0.0)
        p = xa + t[:, None] * (xb - xa)
        dist = np.linalg.norm(p - c, axis=1)
        cand = np.nonzero(cross & (dist < r) & ~broken)[0]
        need = target - int(broken.sum())
        if cand.size > need:
            cand = cand[np.argsort(dist[cand], kind="stable")[:need]]
        broken[cand] = True
    return edges[broken].astype(np.int32)


def tiny_cube(n=1, h=1.0, jitter_frac=0.0, seed=0, **param_kw) -> Problem:
    """n x n x n cubes with the same boundary conditions as `cube_block`."""
    return cube_block(n, n, n, h, jitter_frac=jitter_frac, seed=seed, **param_kw)


def permute_nodes(prob: Problem, seed: int) -> Problem:
    """The same problem with its node ids randomly permuted (seeded): rest
    positions, tets, prescribed nodes and pre-broken pairs renumbered, so a
    mesh arrives in no particular order."""
    n = prob.n_nodes
    new = np.random.default_rng(seed).permutation(n)  # new id of each old node
    X = np.empty_like(prob.X)
    X[new] = prob.X
    pairs = np.sort(new[prob.broken_pairs], axis=1).astype(np.int32) if prob.broken_pairs.size else prob.broken_pairs
    return Problem(prob.name + f"-perm{seed}", X, new[prob.tets].astype(np.int32), dict(prob.params),
                   new[prob.dir_nodes].astype(np.int32), prob.dir_vel.copy(), pairs, prob.n_steps,
                   dict(prob.meta, node_permutation=new))


# Quasi-static blocks pulled from both ends (Sec. 5.1): material -> (Poisson
# ratio, Green-strain threshold, kernel support R_d in m).  R_d is the paper's
# per-material value; the paper gives no elastic constants or thresholds for
# these blocks, so brittle-to-soft values are chosen.  In a displacement-driven
# quasi-static run Young's modulus cancels except against the small mass
# regulariser, so one modulus serves all three.
BLOCK_MATERIALS = {
    "stone": (0.20, 0.004, 0.0),
    "wood": (0.30, 0.008, 0.1),
    "cheese": (0.45, 0.02, 0.5),
}


def pulled_block(material="stone", nx=22, ny=22, nz=58, h=0.18, jitter_frac=0.05, seed=3, pull=0.002,
                 notch_cells=5, dt=1.0, **param_kw) -> Problem:
    """Rectangular block pulled from both ends, quasi-statically (Sec. 5.1).

    Defaults: 22 x 22 x 58 cubes of 18 cm (168,432 tets, the size of the
    paper's blocks; 3.96 x 3.96 x 10.44 m, so that the cheese support of
    R_d = 0.5 m spans 2.8 cells); both end faces prescribed and moved apart
    by `pull` m each per load step (pseudo-timestep dt, velocity pull / dt);
    a notch seeds the crack: every edge of every tet in the mid-length cube
    layer, `notch_cells` cubes deep from the x = 0 face, is pre-broken;
    E = 1e7 Pa, rho = 1000, split precision, block-Jacobi PCG to 1e-6."""
    nu, thr, radius = BLOCK_MATERIALS[material]
    X = grid_nodes(nx, ny, nz, h)
    tets, cube = freudenthal_tets(nx, ny, nz)
    if jitter_frac > 0:
        X = jitter(X, jitter_frac * h, seed)
    in_notch = (cube[:, 2] == nz // 2) & (cube[:, 0] < notch_cells)
    broken = tet_pairs(tets[in_notch])
    k = np.rint((grid_nodes(nx, ny, nz, 1.0))[:, 2]).astype(np.int64)
    bottom = np.nonzero(k == 0)[0]
    top = np.nonzero(k == nz)[0]
    nodes = np.concatenate([bottom, top]).astype(np.int32)
    vel = np.zeros((nodes.size, 3))
    vel[:bottom.size, 2] = -pull / dt
    vel[bottom.size:, 2] = pull / dt
    params = default_params(youngs=1e7, poisson=nu, density=1000.0, damage_strain=thr, damage_radius=radius,
                            dt=dt, cg_rel_tol=1e-6, precision="split")
    params.update(param_kw)
    return Problem(f"{material}-block{nx}x{ny}x{nz}", X, tets.astype(np.int32), params, nodes, vel,
                   broken.astype(np.int32), 40, dict(h=h, shape=(nx, ny, nz), material=material))
