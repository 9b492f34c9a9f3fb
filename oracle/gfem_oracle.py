"""Plain FP64 CPU oracle of one timestep of the remeshing-free graph-based FEM.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import or call this
module: only the tests, the smoke check and the CPU-baseline leg of the
benchmark use it.  It shares no code with the HIP library; the only common
input is the seeded mesh generator, which holds none of the method's
arithmetic.

What is computed, and where it comes from (Mandal, Chaudhuri & Chaudhuri,
"Remeshing-Free Graph-Based Finite Element Method for Ductile and Brittle
Fracture"):

* Linear tetrahedra; consistent element mass (Sec. 3.1, Eq. 5); forces and
  tangent stiffness of the per-element energy (Eq. 7, 9, 10, 11).
* The element energy is the stable neo-Hookean density (Sec. 5.1, Eq. 35),
  or the Saint-Venant Kirchhoff density of the dynamic runs (Sec. 5.2,
  Eq. 37), evaluated from the six squared edge lengths of the tet (Sec. 3.5,
  Theorem 3.1, Eq. 27-31): the Gram matrix of the edge vectors is linear in
  the squared lengths, so I_C = tr(G G0^-1), II_C = tr((G G0^-1)^2) and
  J^2 = det G / det G0.  Nodal forces are sums along the tet's edges
  (Sec. 3.2, Eq. 12).
* Per-edge binary damage, irreversible (Sec. 3.3, Eq. 20-21), evaluated as a
  Green normal-strain threshold along the edge: locally (R_d = 0), or on the
  kernel-weighted average of the strain tensors of the tets whose rest
  centroids lie within R_d (Eq. 20's non-local support).
* Per-tet energy fraction chi (Sec. 3.4, Eq. 22-25), zero when the tet's
  unbroken edges no longer connect its four nodes.
* The fractured system f* = chi f, K* = sum chi k (Sec. 3.6, Eq. 32-34),
  mass unchanged, damping b* = alpha M + beta K*.
* One linearised backward-Euler step per timestep solved by conjugate
  gradients (Sec. 4.3 and Algorithm 1), here with a 3x3 block-Jacobi
  preconditioner; positions advance by dt * v.

Readings where the paper is silent or garbled are the ones listed in the
design notes (squared (J - alpha) term in Eq. 35, Smith's reparametrisation of
the Lame constants, rest-frame edge directions in Eq. 28, tensor projection
of the 2nd Piola-Kirchhoff stress for Eq. 16, (1 - zeta) for Eq. 22, a strain
threshold for Eq. 21, coefficient-clamped edge Hessian, multiplicative
volume-preserving plasticity with a radial return of the deviatoric Hencky
strain for the ductile case).

Parity unpinned: the value of chi at a stress-free state (0/0) and the load
and notch geometry of the inputs are readings that no passage of the paper
fixes.  The plasticity model is a reading too; its return mapping is pinned
by closed-form properties (yield norm, flow direction, volume, the uniaxial
plastic stretch), the choice of model is not.
"""
from __future__ import annotations

import itertools
from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp

# Local edge order of a tet: (0,1),(0,2),(0,3),(1,2),(1,3),(2,3) -- the
# 12,13,14,23,24,34 order of Eq. 15.
LOCAL_EDGES = ((0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3))
EDGE_A = np.array([a for a, _ in LOCAL_EDGES])
EDGE_B = np.array([b for _, b in LOCAL_EDGES])


# --------------------------------------------------------------------------
# Constants of the reference simplex
# --------------------------------------------------------------------------

def reference_edges() -> np.ndarray:
    """e_hat_k: edge k of the reference simplex, node 0 at the origin and
    node i at the i-th unit vector.  s_k = e_hat_k^T G e_hat_k."""
    e = np.zeros((6, 3))
    for k, (a, b) in enumerate(LOCAL_EDGES):
        if b > 0:
            e[k, b - 1] += 1.0
        if a > 0:
            e[k, a - 1] -= 1.0
    return e


def polarisation_basis() -> np.ndarray:
    """E_k = dG/ds_k, where G = Ds^T Ds is the Gram matrix of the edge vectors
    from node 0: G_ii = s_0i and G_ij = (s_0i + s_0j - s_ij)/2."""
    E = np.zeros((6, 3, 3))
    for k, (a, b) in enumerate(LOCAL_EDGES):
        if a == 0:
            i = b - 1
            E[k, i, i] = 1.0
            for j in range(3):
                if j != i:
                    E[k, i, j] += 0.5
                    E[k, j, i] += 0.5
        else:
            i, j = a - 1, b - 1
            E[k, i, j] -= 0.5
            E[k, j, i] -= 0.5
    return E


EHAT = reference_edges()
EK = polarisation_basis()


def disconnected_masks() -> np.ndarray:
    """LUT over the 64 broken-edge masks of a tet: True when the unbroken
    edges leave the four nodes in more than one connected piece (the
    'disjoint fragments' case of Sec. 3.4).  Brute-force graph search."""
    lut = np.zeros(64, dtype=bool)
    for mask in range(64):
        adj = {n: set() for n in range(4)}
        for k, (a, b) in enumerate(LOCAL_EDGES):
            if not (mask >> k) & 1:
                adj[a].add(b)
                adj[b].add(a)
        seen, stack = {0}, [0]
        while stack:
            n = stack.pop()
            for m in adj[n]:
                if m not in seen:
                    seen.add(m)
                    stack.append(m)
        lut[mask] = len(seen) < 4
    return lut


DISCONNECTED = disconnected_masks()


ENERGIES = ("stable_neo_hookean", "stvk")


def material(youngs: float, poisson: float, energy: str = "stable_neo_hookean"):
    """Lame constants of (E, nu).  Stable neo-Hookean (Eq. 35): the
    reparametrisation mu' = 4 mu / 3, lambda' = lambda + 5 mu / 6 (so that the
    small-strain response has the given E and nu) and alpha of Eq. 35.
    Saint-Venant Kirchhoff (Eq. 37): the plain constants (its small-strain
    response is linear elasticity with them); alpha unused (0)."""
    mu = youngs / (2.0 * (1.0 + poisson))
    lam = youngs * poisson / ((1.0 + poisson) * (1.0 - 2.0 * poisson))
    if energy == "stvk":
        return mu, lam, 0.0
    if energy != "stable_neo_hookean":
        raise ValueError(f"unknown energy {energy!r}")
    mu_s = 4.0 * mu / 3.0
    lam_s = lam + 5.0 * mu / 6.0
    alpha = 1.0 + mu_s / lam_s - mu_s / (4.0 * lam_s)
    return mu_s, lam_s, alpha


# --------------------------------------------------------------------------
# Mesh set-up
# --------------------------------------------------------------------------

@dataclass
class Mesh:
    X: np.ndarray            # (n,3) rest positions
    tets: np.ndarray         # (m,4) positively oriented
    edges: np.ndarray        # (ne,2) i<j, lexicographic
    tet_edge: np.ndarray     # (m,6) edge id of each local edge
    Dm: np.ndarray           # (m,3,3) rest edge vectors from node 0 (columns)
    Dm_inv: np.ndarray
    G0: np.ndarray
    G0_inv: np.ndarray
    detG0: np.ndarray
    V: np.ndarray            # (m,) rest volume
    S: np.ndarray            # (m,6) rest squared lengths per local edge
    c: np.ndarray            # (m,6) c_k = tr(E_k G0^-1) = dI_C/ds_k
    S_edge: np.ndarray       # (ne,) rest squared length per global edge
    M: sp.csr_matrix         # (3n,3n) consistent mass
    params: dict
    mu: float = 0.0
    lam: float = 0.0
    alpha: float = 0.0
    nonlocal_support: tuple | None = None   # (ptr, idx, w) of Eq. 20's support when R_d > 0
    energy: str = "stable_neo_hookean"      # or "stvk" (Eq. 37)


def setup(X: np.ndarray, tets: np.ndarray, params: dict) -> Mesh:
    X = np.asarray(X, dtype=np.float64)
    tets = np.asarray(tets, dtype=np.int64).copy()
    Dm = np.stack([X[tets[:, i]] - X[tets[:, 0]] for i in (1, 2, 3)], axis=2)
    neg = np.linalg.det(Dm) < 0
    tets[neg, 2], tets[neg, 3] = tets[neg, 3].copy(), tets[neg, 2].copy()
    Dm = np.stack([X[tets[:, i]] - X[tets[:, 0]] for i in (1, 2, 3)], axis=2)
    detDm = np.linalg.det(Dm)
    if np.any(detDm <= 0):
        raise ValueError("degenerate tetrahedron")
    V = detDm / 6.0
    G0 = np.einsum("tji,tjk->tik", Dm, Dm)
    G0_inv = np.linalg.inv(G0)
    pairs = np.stack([np.sort(tets[:, [a, b]], axis=1) for a, b in LOCAL_EDGES], axis=1)
    edges, inv = np.unique(pairs.reshape(-1, 2), axis=0, return_inverse=True)
    tet_edge = inv.reshape(-1, 6)
    S = np.stack([np.sum((X[tets[:, b]] - X[tets[:, a]]) ** 2, axis=1) for a, b in LOCAL_EDGES], 1)
    S_edge = np.sum((X[edges[:, 1]] - X[edges[:, 0]]) ** 2, axis=1)
    c = np.einsum("kij,tji->tk", EK, G0_inv)
    M = consistent_mass(X.shape[0], tets, V, params["density"])
    energy = params.get("energy", "stable_neo_hookean")
    mu, lam, alpha = material(params["youngs"], params["poisson"], energy)
    mesh = Mesh(X, tets, edges, tet_edge, Dm, np.linalg.inv(Dm), G0, G0_inv,
                np.linalg.det(G0), V, S, c, S_edge, M, params, mu, lam, alpha, energy=energy)
    radius = params.get("damage_radius", 0.0)
    if radius > 0:
        mesh.nonlocal_support = nonlocal_neighbours(mesh, radius)
    return mesh


def consistent_mass(n: int, tets: np.ndarray, V: np.ndarray, rho: float) -> sp.csr_matrix:
    """Eq. 5 for linear shape functions: m_ab = rho V (1 + delta_ab) / 20 I_3."""
    rows, cols, vals = [], [], []
    for a in range(4):
        for b in range(4):
            m = rho * V * (2.0 if a == b else 1.0) / 20.0
            for d in range(3):
                rows.append(3 * tets[:, a] + d)
                cols.append(3 * tets[:, b] + d)
                vals.append(m)
    return sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(3 * n, 3 * n)).tocsr()


# --------------------------------------------------------------------------
# State
# --------------------------------------------------------------------------

@dataclass
class State:
    x: np.ndarray                    # (n,3) positions
    v: np.ndarray                    # (n,3) velocities
    zeta: np.ndarray                 # (ne,) bool, True = broken
    Cp: np.ndarray                   # (m,3,3) plastic right Cauchy-Green tensor (material frame, det 1)
    step: int = 0


def initial_state(mesh: Mesh) -> State:
    n, m = mesh.X.shape[0], mesh.tets.shape[0]
    return State(mesh.X.copy(), np.zeros((n, 3)), np.zeros(mesh.edges.shape[0], bool),
                 np.tile(np.eye(3), (m, 1, 1)))


def break_pairs(mesh: Mesh, state: State, pairs: np.ndarray) -> None:
    """OR the given node pairs (i<j) into the damage labels."""
    if len(pairs) == 0:
        return
    n = mesh.X.shape[0] + 1
    key = mesh.edges[:, 0] * n + mesh.edges[:, 1]
    pk = np.sort(np.asarray(pairs, dtype=np.int64), axis=1)
    state.zeta |= np.isin(key, pk[:, 0] * n + pk[:, 1])


# --------------------------------------------------------------------------
# Damage (Eq. 20-21, local support)
# --------------------------------------------------------------------------

def edge_strain(mesh: Mesh, x: np.ndarray) -> np.ndarray:
    """Green normal strain along each edge: (s - S) / (2 S) = (lambda^2 - 1)/2
    with lambda the stretch of Eq. 27; by Eq. 28 it equals q^T E q."""
    s = np.sum((x[mesh.edges[:, 1]] - x[mesh.edges[:, 0]]) ** 2, axis=1)
    return (s - mesh.S_edge) / (2.0 * mesh.S_edge)


def damage_update(mesh: Mesh, x: np.ndarray, zeta: np.ndarray, near_tol: float = 1e-6,
                  override: dict | None = None):
    """zeta <- zeta OR (strain >= threshold); labels never revert (Sec. 3.3).
    Returns (new zeta, indices of edges within near_tol of the threshold).
    `override` maps edge id -> label for near-threshold edges only.
    With a non-local support (R_d > 0, Eq. 20) an edge breaks when the
    averaged normal strain along it reaches the threshold in any tet that
    contains it, and is near the threshold when it is so in any of them."""
    thr = mesh.params["damage_strain"]
    if mesh.nonlocal_support is not None:
        eps_t = nonlocal_edge_strain(mesh, x)
        ne = mesh.edges.shape[0]
        hit = np.zeros(ne, bool)
        np.logical_or.at(hit, mesh.tet_edge.ravel(), (eps_t >= thr).ravel())
        nr = np.zeros(ne, bool)
        np.logical_or.at(nr, mesh.tet_edge.ravel(), (np.abs(eps_t - thr) < near_tol).ravel())
        near = np.nonzero(nr)[0]
    else:
        eps = edge_strain(mesh, x)
        hit = eps >= thr
        near = np.nonzero(np.abs(eps - thr) < near_tol)[0]
    if override:
        near_set = set(near.tolist())
        for e, lab in override.items():
            if e in near_set:
                hit[e] = bool(lab)
    return zeta | hit, near


# --------------------------------------------------------------------------
# Non-local damage criterion (Eq. 20 with a support R_d > 0)
# --------------------------------------------------------------------------

def rest_centroids(mesh: Mesh) -> np.ndarray:
    return mesh.X[mesh.tets].mean(axis=1)


def nonlocal_neighbours(mesh: Mesh, radius: float):
    """Eq. 20's support: for each tet t the tets t' whose rest centroid lies
    within `radius` of t's, ascending, with the kernel weights
    w = (1 - (r / R_d)^2)^2 normalised to sum 1 over the support (r the
    centroid distance; the tet itself has w = 1 before normalisation).
    Returns CSR arrays (ptr (m+1), idx, w)."""
    from scipy.spatial import cKDTree

    c = rest_centroids(mesh)
    m = c.shape[0]
    lists = cKDTree(c).query_ball_point(c, r=radius)
    ptr = np.zeros(m + 1, np.int64)
    idx, wts = [], []
    for t in range(m):
        nb = np.array(sorted(lists[t]), np.int64)
        r2 = np.sum((c[nb] - c[t]) ** 2, axis=1) / (radius * radius)
        w = (1.0 - r2) ** 2
        idx.append(nb)
        wts.append(w / w.sum())
        ptr[t + 1] = ptr[t] + nb.size
    return ptr, np.concatenate(idx), np.concatenate(wts)


def nonlocal_edge_strain(mesh: Mesh, x: np.ndarray) -> np.ndarray:
    """Per tet and local edge, the normal strain q_k^T E* q_k of the weighted
    average E* of the Green strain tensors of the tets in the support
    (Eq. 20 with the strain reading of the criterion), q_k the rest unit
    direction of the edge.  (m,6)."""
    ptr, idx, w = mesh.nonlocal_support
    F = deformation_gradient(mesh, x)
    E = 0.5 * (np.einsum("tji,tjk->tik", F, F) - np.eye(3))
    m = E.shape[0]
    row = np.repeat(np.arange(m), np.diff(ptr))
    Eavg = np.zeros_like(E)
    np.add.at(Eavg, row, w[:, None, None] * E[idx])
    t = mesh.tets
    q = np.stack([mesh.X[t[:, b]] - mesh.X[t[:, a]] for a, b in LOCAL_EDGES], axis=1)
    q /= np.linalg.norm(q, axis=2, keepdims=True)
    return np.einsum("tki,tij,tkj->tk", q, Eavg, q)


# Below this |J| the volume terms of the energy are evaluated in cofactor form
# (the edge-length form of J divides by J: one over the volume of a flat
# tet), and plastic flow is not applied.
J_MIN = 0.05


# --------------------------------------------------------------------------
# Plasticity (ductile case): multiplicative, volume-preserving flow with an
# instant radial return of the deviatoric elastic Hencky strain
# --------------------------------------------------------------------------

def deformation_gradient(mesh: Mesh, x: np.ndarray) -> np.ndarray:
    t = mesh.tets
    Ds = np.stack([x[t[:, i]] - x[t[:, 0]] for i in (1, 2, 3)], axis=2)
    return Ds @ mesh.Dm_inv


def plastic_update(mesh: Mesh, x: np.ndarray, Cp: np.ndarray) -> np.ndarray:
    """F = Fe Fp with Cp = Fp^T Fp (det 1).  The elastic stretches are the
    generalised eigenvalues lam_i of C v = lam Cp v (C = F^T F); their Hencky
    strains h_i = log(lam_i) / 2 have deviator d = h - mean(h).  If |d| exceeds
    the yield strain, d is scaled back onto the yield surface and Cp is moved
    so that C has the returned elastic stretches over it; the mean (volumetric)
    part never flows, so det Cp stays 1.  Tets with det F < J_MIN (nearly flat
    or inverted) do not flow: C = F^T F cannot tell an inverted tet from its
    mirror image, so its stretches are no measure of plastic strain there."""
    ey = mesh.params.get("yield_strain", 0.0)
    if ey <= 0:
        return Cp
    F = deformation_gradient(mesh, x)
    J = np.linalg.det(F)
    C = np.einsum("tji,tjk->tik", F, F)
    # generalised symmetric eigenproblem through the Cholesky factor of Cp:
    # S = L^-1 C L^-T = W diag(lam) W^T, V = L^-T W
    L = np.linalg.cholesky(Cp)
    Li = np.linalg.inv(L)
    S = Li @ C @ np.swapaxes(Li, 1, 2)
    lam, W = np.linalg.eigh(0.5 * (S + np.swapaxes(S, 1, 2)))
    h = 0.5 * np.log(lam)
    hm = h.mean(axis=1, keepdims=True)
    d = h - hm
    nd = np.linalg.norm(d, axis=1)
    flow = (nd > ey) & (J >= J_MIN)
    h_new = hm + d * np.where(flow, ey / np.where(flow, nd, 1.0), 1.0)[:, None]
    # Cp' = L W diag(lam / lam') W^T L^T: C over Cp' has the returned stretches
    LW = L @ W
    Cp_new = np.einsum("tij,tj,tkj->tik", LW, lam / np.exp(2.0 * h_new), LW)
    return np.where(flow[:, None, None], Cp_new, Cp)


def gram_offset(mesh: Mesh, Cp: np.ndarray) -> np.ndarray:
    """The plastic rest shape on the Gram matrix: Gp = Dm^T Cp Dm = G0 + P,
    P = Dm^T (Cp - I) Dm (zero without plastic flow)."""
    return np.einsum("tji,tjk,tkl->til", mesh.Dm, Cp - np.eye(3), mesh.Dm)


# --------------------------------------------------------------------------
# Edge-length element (Theorem 3.1 + Eq. 12 + Eq. 35)
# --------------------------------------------------------------------------



@dataclass
class Element:
    s: np.ndarray        # (m,6) current squared edge lengths
    d: np.ndarray        # (m,6,3) current edge vectors x_b - x_a
    IC: np.ndarray       # elastic I_C = tr(G Gp^-1)
    J: np.ndarray        # det F
    G: np.ndarray
    c: np.ndarray        # (m,6) dI_C/ds_k = tr(E_k Gp^-1)
    g: np.ndarray        # (m,6) dPsi/ds_k (small tets: the I_C terms only)
    v: np.ndarray        # (m,6) tr(G^-1 E_k) (zero on small tets)
    Mkl: np.ndarray      # (m,6,6) (zero on small tets)
    coef: np.ndarray     # (m,3) unclamped edge-Hessian coefficients (small tets: a2 = a3 = 0)
    psi: np.ndarray
    small: np.ndarray    # |J| < J_MIN: volume terms in cofactor form
    gradJ: np.ndarray    # (m,4,3) dJ/dx_a (cofactor form; used on small tets)
    hessJ: np.ndarray    # (m,12,12) d^2 J/dx^2 (cofactor form; used on small tets, unclamped only)


def cofactor_gradient(Ds: np.ndarray, detDm: np.ndarray):
    """dJ/dx_a for J = det(Ds)/det(Dm), Ds = [x1-x0, x2-x0, x3-x0]: the
    cofactor columns x2'x x3', x3' x x1', x1' x x2' over det Dm (nodes 1-3) and
    minus their sum (node 0); and the 12x12 second derivative of the triple
    product (entries +-d_c, independent of the differentiated pair)."""
    d1, d2, d3 = Ds[:, :, 0], Ds[:, :, 1], Ds[:, :, 2]
    g = np.zeros((Ds.shape[0], 4, 3))
    g[:, 1] = np.cross(d2, d3)
    g[:, 2] = np.cross(d3, d1)
    g[:, 3] = np.cross(d1, d2)
    g[:, 0] = -(g[:, 1] + g[:, 2] + g[:, 3])
    g /= detDm[:, None, None]
    # d^2 (d1 . d2 x d3) / dd_a dd_b = [d_c]x-type blocks with the sign of the
    # permutation (a, b, c); the node-0 rows/columns follow from translation
    # invariance (d_i = x_i - x_0)
    eps = np.zeros((3, 3, 3))
    for i, j, k in itertools.permutations(range(3)):
        eps[i, j, k] = np.linalg.det(np.eye(3)[[i, j, k]])
    Hd = np.zeros((Ds.shape[0], 3, 3, 3, 3))      # [a, b] blocks over d_1..d_3
    dd = (d1, d2, d3)
    for a in range(3):
        for b in range(3):
            if a == b:
                continue
            c = 3 - a - b
            sgn = np.linalg.det(np.eye(3)[[a, b, c]])
            Hd[:, a, b] = sgn * np.einsum("ijk,tk->tij", eps, dd[c])
    T = np.zeros((4, 3))
    T[0] = -1.0
    T[1:] = np.eye(3)                              # d_i = sum_a T[a, i] x_a
    H = np.einsum("ai,bj,tijpq->tapbq", T, T, Hd).reshape(-1, 12, 12)
    return g, H / detDm[:, None, None]


def element(mesh: Mesh, x: np.ndarray, Cp: np.ndarray | None = None) -> Element:
    if mesh.energy == "stvk":
        return element_stvk(mesh, x, Cp)
    t = mesh.tets
    m = t.shape[0]
    d = np.stack([x[t[:, b]] - x[t[:, a]] for a, b in LOCAL_EDGES], axis=1)
    s = np.sum(d * d, axis=2)
    G = np.einsum("tk,kij->tij", s, EK)
    Gp = mesh.G0 if Cp is None else mesh.G0 + gram_offset(mesh, Cp)
    Gp_inv = np.linalg.inv(Gp)
    mu, lam, al = mesh.mu, mesh.lam, mesh.alpha
    IC = np.einsum("tij,tji->t", G, Gp_inv)
    c = np.einsum("kij,tji->tk", EK, Gp_inv)
    Ds = np.stack([x[t[:, i]] - x[t[:, 0]] for i in (1, 2, 3)], axis=2)
    detDm = np.linalg.det(mesh.Dm)
    J = np.linalg.det(Ds) / detDm                  # = sign(det Ds) sqrt(det G / det G0)
    small = np.abs(J) < J_MIN
    big = ~small
    v = np.zeros((m, 6))
    Mkl = np.zeros((m, 6, 6))
    if np.any(big):
        Ginv = np.linalg.inv(G[big])
        W = np.einsum("tij,kjl->tkil", Ginv, EK)   # G^-1 E_k
        v[big] = np.einsum("tkii->tk", W)
        Mkl[big] = np.einsum("tkij,tlji->tkl", W, W)
    gJ = np.where(big, 0.5 * lam * (J - al) * J, 0.0)
    g = 0.5 * mu * (1.0 - 1.0 / (IC + 1.0))[:, None] * c + gJ[:, None] * v
    coef = np.stack([0.5 * mu / (IC + 1.0) ** 2,
                     np.where(big, 0.25 * lam * (2.0 * J - al) * J, 0.0),
                     np.where(big, -0.5 * lam * (J - al) * J, 0.0)], axis=1)
    psi = 0.5 * mu * (IC - 3.0) + 0.5 * lam * (J - al) ** 2 - 0.5 * mu * np.log(IC + 1.0)
    gradJ, hessJ = cofactor_gradient(Ds, detDm)
    return Element(s, d, IC, J, G, c, g, v, Mkl, coef, psi, small, gradJ, hessJ)


def element_stvk(mesh: Mesh, x: np.ndarray, Cp: np.ndarray | None = None) -> Element:
    """Saint-Venant Kirchhoff density of Eq. 37 in edge form:
    Psi = lam/8 (I_C - 3)^2 + mu/4 (II_C - 2 I_C + 3) with A = Gp^-1,
    I_C = tr(G A), II_C = tr(G A G A).  Its edge derivatives:
    dPsi/ds_k = lam/4 (I_C - 3) c_k + mu/2 (t_k - c_k), c_k = tr(E_k A),
    t_k = tr(E_k A G A); d2Psi/ds_k ds_l = lam/4 c_k c_l + mu/2 N_kl,
    N_kl = tr(E_k A E_l A).  No J enters, so flat and inverted tets need no
    special form; the edge Hessian is PSD as it stands (returned as the
    coefficients (lam/4, 0, mu/2) on (c c^T, v v^T, N), with v = 0)."""
    t = mesh.tets
    m = t.shape[0]
    d = np.stack([x[t[:, b]] - x[t[:, a]] for a, b in LOCAL_EDGES], axis=1)
    s = np.sum(d * d, axis=2)
    G = np.einsum("tk,kij->tij", s, EK)
    Gp = mesh.G0 if Cp is None else mesh.G0 + gram_offset(mesh, Cp)
    A = np.linalg.inv(Gp)
    mu, lam = mesh.mu, mesh.lam
    GA = G @ A
    IC = np.einsum("tii->t", GA)
    II = np.einsum("tij,tji->t", GA, GA)
    c = np.einsum("kij,tji->tk", EK, A)
    AGA = A @ G @ A
    tk = np.einsum("kij,tji->tk", EK, AGA)
    g = 0.25 * lam * (IC - 3.0)[:, None] * c + 0.5 * mu * (tk - c)
    EA_ = np.einsum("kij,tjl->tkil", EK, A)          # E_k A
    N = np.einsum("tkij,tlji->tkl", EA_, EA_)
    coef = np.stack([np.full(m, 0.25 * lam), np.zeros(m), np.full(m, 0.5 * mu)], axis=1)
    psi = lam / 8.0 * (IC - 3.0) ** 2 + mu / 4.0 * (II - 2.0 * IC + 3.0)
    Ds = np.stack([x[t[:, i]] - x[t[:, 0]] for i in (1, 2, 3)], axis=2)
    J = np.linalg.det(Ds) / np.linalg.det(mesh.Dm)
    return Element(s, d, IC, J, G, c, g, np.zeros((m, 6)), N, coef, psi, np.zeros(m, bool),
                   np.zeros((m, 4, 3)), np.zeros((m, 12, 12)))


def edge_hessian(mesh: Mesh, el: Element, clamp: bool = True) -> np.ndarray:
    """d^2 Psi / ds_k ds_l = a1 c c^T + a2 v v^T + a3 M; clamped: each a_i >= 0
    (c c^T, v v^T and the Gram matrix M are PSD, so the result is PSD).  On
    small tets only the I_C term is in edge form."""
    a = np.maximum(el.coef, 0.0) if clamp else el.coef
    c, v = el.c, el.v
    return (a[:, 0, None, None] * c[:, :, None] * c[:, None, :]
            + a[:, 1, None, None] * v[:, :, None] * v[:, None, :]
            + a[:, 2, None, None] * el.Mkl)


def edge_jacobian(el: Element) -> np.ndarray:
    """Js (m,6,12): ds_k/dx, edge k=(a,b) gives +2 d_k at b and -2 d_k at a."""
    m = el.d.shape[0]
    Js = np.zeros((m, 6, 12))
    for k, (a, b) in enumerate(LOCAL_EDGES):
        Js[:, k, 3 * b:3 * b + 3] = 2.0 * el.d[:, k]
        Js[:, k, 3 * a:3 * a + 3] = -2.0 * el.d[:, k]
    return Js


LAPLACE = np.zeros((6, 12, 12))
for _k, (_a, _b) in enumerate(LOCAL_EDGES):
    _u = np.zeros(4)
    _u[_a], _u[_b] = 1.0, -1.0
    LAPLACE[_k] = np.kron(np.outer(_u, _u), np.eye(3))


def element_forces(mesh: Mesh, el: Element, chi: np.ndarray) -> np.ndarray:
    """Restoring nodal forces (m,4,3): f_a = 2 V chi sum_{k ∋ a} g_k (x_b - x_a)
    (Eq. 12 with the unit vector pointing from a to the other node, times the
    energy fraction of Eq. 32).  On small tets the volume term's force
    -V chi lambda (J - alpha) dJ/dx_a is added in cofactor form."""
    f = np.zeros((el.d.shape[0], 4, 3))
    w = 2.0 * (mesh.V * chi)[:, None] * el.g
    for k, (a, b) in enumerate(LOCAL_EDGES):
        f[:, a] += w[:, k, None] * el.d[:, k]
        f[:, b] -= w[:, k, None] * el.d[:, k]
    fJ = np.where(el.small, -mesh.V * chi * mesh.lam * (el.J - mesh.alpha), 0.0)
    return f + fJ[:, None, None] * el.gradJ


def element_stiffness(mesh: Mesh, el: Element, chi: np.ndarray, clamp: bool = True) -> np.ndarray:
    """k*_e = chi V [Js^T H Js + sum_k 2 g_k L_k]  (Eq. 10, 33), with the clamped
    H and g_k -> max(g_k, 0) for a PSD tangent.  On small tets the volume term
    adds lambda dJ dJ^T (PSD) and, unclamped only, lambda (J - alpha) d^2 J
    (indefinite, dropped by the clamp)."""
    H = edge_hessian(mesh, el, clamp)
    Js = edge_jacobian(el)
    gg = np.maximum(el.g, 0.0) if clamp else el.g
    K = np.einsum("tki,tkl,tlj->tij", Js, H, Js) + 2.0 * np.einsum("tk,kij->tij", gg, LAPLACE)
    gJ = el.gradJ.reshape(-1, 12)
    KJ = mesh.lam * gJ[:, :, None] * gJ[:, None, :]
    if not clamp:
        KJ = KJ + (mesh.lam * (el.J - mesh.alpha))[:, None, None] * el.hessJ
    K = K + np.where(el.small[:, None, None], KJ, 0.0)
    return (mesh.V * chi)[:, None, None] * K


# --------------------------------------------------------------------------
# Energy fraction chi (Eq. 22-25)
# --------------------------------------------------------------------------

def scaled_edge_stress(mesh: Mesh, x: np.ndarray, Cp: np.ndarray | None = None):
    """sigma_k = q_k^T S q_k: the 2nd Piola-Kirchhoff stress S = 2 dPsi/dC of
    Eq. 35 (or Eq. 37) projected on the rest unit direction q_k of each edge (Eq. 16-19,
    as a tensor projection).  With plastic flow the I_C term is taken relative
    to Cp: S = mu (1 - 1/(I_C + 1)) Cp^-1 + lambda (J - alpha) J C^-1.
    On small tets (|J| < J_MIN) every sigma_k is returned multiplied by |J|
    (J C^-1 = adj(C) / J), which leaves chi's ratios unchanged and keeps
    them finite on a flat tet.  Returns (sigma (m,6), small, J)."""
    F = deformation_gradient(mesh, x)
    C = np.einsum("tji,tjk->tik", F, F)
    m = C.shape[0]
    Cpi = np.tile(np.eye(3), (m, 1, 1)) if Cp is None else np.linalg.inv(Cp)
    mu, lam, al = mesh.mu, mesh.lam, mesh.alpha
    IC = np.einsum("tij,tji->t", C, Cpi)
    J = np.linalg.det(F)
    t = mesh.tets
    q = np.stack([mesh.X[t[:, b]] - mesh.X[t[:, a]] for a, b in LOCAL_EDGES], axis=1)
    q /= np.linalg.norm(q, axis=2, keepdims=True)
    if mesh.energy == "stvk":
        # S = 2 dPsi/dC = lam/2 (I_C - 3) Cp^-1 + mu (Cp^-1 C Cp^-1 - Cp^-1)
        Sst = (0.5 * lam * (IC - 3.0))[:, None, None] * Cpi + mu * (Cpi @ C @ Cpi - Cpi)
        return np.einsum("tki,tij,tkj->tk", q, Sst, q), np.zeros(m, bool), J
    small = np.abs(J) < J_MIN
    # adjugate of the symmetric C (its cofactor matrix)
    adj = np.empty_like(C)
    for i in range(3):
        for j in range(3):
            r = [k for k in range(3) if k != i]
            cl = [k for k in range(3) if k != j]
            adj[:, j, i] = (-1) ** (i + j) * (C[:, r[0], cl[0]] * C[:, r[1], cl[1]]
                                              - C[:, r[0], cl[1]] * C[:, r[1], cl[0]])
    sgn = np.where(J >= 0, 1.0, -1.0)
    scale = np.where(small, np.abs(J), 1.0)
    # J C^-1 = adj(C) / J on big tets; |J| J C^-1 = sign(J) adj(C) on small ones
    jc = np.where(small, sgn, 1.0 / np.where(small, 1.0, J))[:, None, None] * adj
    Sst = (scale * mu * (1.0 - 1.0 / (IC + 1.0)))[:, None, None] * Cpi \
        + (lam * (J - al))[:, None, None] * jc
    return np.einsum("tki,tij,tkj->tk", q, Sst, q), small, J


def edge_normal_stress(mesh: Mesh, x: np.ndarray, Cp: np.ndarray | None = None) -> np.ndarray:
    """The unscaled sigma_k (m,6) (infinite on an exactly flat tet)."""
    sig, small, J = scaled_edge_stress(mesh, x, Cp)
    with np.errstate(divide="ignore", invalid="ignore"):
        return np.where(small[:, None], sig / np.abs(J)[:, None], sig)


def energy_fraction(mesh: Mesh, x: np.ndarray, zeta: np.ndarray, Cp: np.ndarray | None = None):
    """chi of Eq. 25 with sigma' = (1 - zeta) sigma; 0 for disconnected tets;
    n_unbroken/6 when the stress is (numerically) zero.  Returns (chi, mask)."""
    zt = zeta[mesh.tet_edge]
    mask = np.sum(zt.astype(np.int64) << np.arange(6), axis=1)
    chi = np.ones(mesh.tets.shape[0])
    dmg = mask != 0
    if np.any(dmg):
        sig, small, J = scaled_edge_stress(mesh, x, Cp)
        sig = np.abs(sig)
        den = sig.sum(axis=1)
        num = np.where(zt, 0.0, sig).sum(axis=1)
        # the zero-stress test on the unscaled stresses: |J| sum|sigma| on small tets
        lim = 1e-12 * (mesh.mu + mesh.lam) * np.where(small, np.abs(J), 1.0)
        zero = den <= lim
        ratio = np.where(zero, (6 - zt.sum(axis=1)) / 6.0, num / np.where(zero, 1.0, den))
        chi = np.where(dmg, ratio, 1.0)
    chi = np.where(DISCONNECTED[mask], 0.0, chi)
    return chi, mask


# --------------------------------------------------------------------------
# Global system, solve and step
# --------------------------------------------------------------------------

def scatter_forces(n: int, tets: np.ndarray, fe: np.ndarray) -> np.ndarray:
    f = np.zeros((n, 3))
    for a in range(4):
        np.add.at(f, tets[:, a], fe[:, a])
    return f


def assemble_stiffness(n: int, tets: np.ndarray, Ke: np.ndarray) -> sp.csr_matrix:
    dof = (3 * tets[:, :, None] + np.arange(3)).reshape(-1, 12)
    rows = np.repeat(dof, 12, axis=1).ravel()
    cols = np.tile(dof, (1, 12)).ravel()
    return sp.coo_matrix((Ke.ravel(), (rows, cols)), shape=(3 * n, 3 * n)).tocsr()


def restoring_forces(mesh: Mesh, state: State) -> np.ndarray:
    """f* = sum_e chi_e f_e at the state's positions and labels (n,3)."""
    chi, _ = energy_fraction(mesh, state.x, state.zeta, state.Cp)
    el = element(mesh, state.x, state.Cp)
    return scatter_forces(mesh.X.shape[0], mesh.tets, element_forces(mesh, el, chi))


def total_energy(mesh: Mesh, x: np.ndarray, chi: np.ndarray, Cp=None) -> float:
    el = element(mesh, x, Cp)
    return float(np.sum(mesh.V * chi * el.psi))


@dataclass
class System:
    A: sp.csr_matrix
    b: np.ndarray          # (3n,)
    dv_c: np.ndarray       # (k,3) prescribed velocity increments
    chi: np.ndarray
    stats: dict = field(default_factory=dict)


def build_system(mesh: Mesh, state: State, dir_nodes, dir_vel, zeta: np.ndarray, Cp) -> System:
    """A = M + dt (aM + bK*) + dt^2 K*;
    b = dt (f_ext + f* - (aM + bK*) v) - dt^2 K* v; then Dirichlet elimination."""
    p = mesh.params
    n = mesh.X.shape[0]
    dt = p["dt"]
    chi, mask = energy_fraction(mesh, state.x, zeta, Cp)
    el = element(mesh, state.x, Cp)
    f = scatter_forces(n, mesh.tets, element_forces(mesh, el, chi)).ravel()
    K = assemble_stiffness(n, mesh.tets, element_stiffness(mesh, el, chi))
    M = mesh.M
    ra, rb = p.get("rayleigh_alpha", 0.0), p.get("rayleigh_beta", 0.0)
    D = ra * M + rb * K
    v = state.v.ravel()
    fext = M @ np.tile(np.asarray(p.get("gravity", (0, 0, 0)), float), n)
    A = (M + dt * D + dt * dt * K).tocsr()
    b = dt * (fext + f - D @ v) - dt * dt * (K @ v)
    dir_nodes = np.asarray(dir_nodes, dtype=np.int64)
    dv_c = np.asarray(dir_vel, float) - state.v[dir_nodes]
    if dir_nodes.size:
        cdof = (3 * dir_nodes[:, None] + np.arange(3)).ravel()
        xc = np.zeros(3 * n)
        xc[cdof] = dv_c.ravel()
        b = b - A @ xc
        keep = np.ones(3 * n)
        keep[cdof] = 0.0
        Dk = sp.diags(keep)
        A = (Dk @ A @ Dk + sp.diags(1.0 - keep)).tocsr()
        b[cdof] = dv_c.ravel()
    A.eliminate_zeros()
    stats = dict(chi_zero_tets=int(np.sum(chi == 0.0)),
                 degenerate_tets=int(np.sum(np.abs(el.J) < J_MIN)))
    return System(A, b, dv_c, chi, stats)


def block_jacobi(A: sp.csr_matrix) -> sp.csr_matrix:
    """Inverse of the 3x3 diagonal blocks of A, as a block-diagonal matrix."""
    n = A.shape[0] // 3
    blocks = np.zeros((n, 3, 3))
    for r in range(3):
        for c in range(3):
            blocks[:, r, c] = A.diagonal(c - r)[np.arange(n) * 3 + min(r, c)]
    inv = np.linalg.inv(blocks)
    return sp.bsr_matrix((inv, np.arange(n), np.arange(n + 1)), shape=(3 * n, 3 * n)).tocsr()


def pcg(A: sp.csr_matrix, b: np.ndarray, P: sp.csr_matrix, tol: float, max_iter: int):
    """Preconditioned conjugate gradients from x0 = 0.  Converged when the true
    residual satisfies |b - A x| <= tol |b|.  Returns (x, iters, rel_res, ok)."""
    bn = np.linalg.norm(b)
    x = np.zeros_like(b)
    if bn == 0.0:
        return x, 0, 0.0, True
    r = b.copy()
    z = P @ r
    p = z.copy()
    rz = r @ z
    it = 0
    while it < max_iter:
        q = A @ p
        pq = p @ q
        if pq <= 0:
            break
        al = rz / pq
        x += al * p
        r -= al * q
        it += 1
        if np.linalg.norm(r) <= tol * bn:
            rt = np.linalg.norm(b - A @ x)
            if rt <= tol * bn:
                return x, it, rt / bn, True
            r = b - A @ x
        z = P @ r
        rz_new = r @ z
        p = z + (rz_new / rz) * p
        rz = rz_new
    rt = np.linalg.norm(b - A @ x)
    return x, it, rt / bn, rt <= tol * bn


def step(mesh: Mesh, state: State, dir_nodes, dir_vel, override: dict | None = None,
         max_iter: int | None = None, solver: str = "pcg"):
    """One timestep of Algorithm 1 (without collisions and visualisation):
    damage -> plasticity -> build system -> solve -> update.  Returns
    (new_state, stats); on non-convergence returns (state unchanged, stats)."""
    p = mesh.params
    zeta, near = damage_update(mesh, state.x, state.zeta, override=override)
    Cp = plastic_update(mesh, state.x, state.Cp)
    sysm = build_system(mesh, state, dir_nodes, dir_vel, zeta, Cp)
    if solver == "direct":
        import scipy.sparse.linalg as spla
        dv = spla.spsolve(sysm.A.tocsc(), sysm.b)
        it, ok = 0, True
        rel = np.linalg.norm(sysm.b - sysm.A @ dv) / max(np.linalg.norm(sysm.b), 1e-300)
    else:
        P = block_jacobi(sysm.A)
        dv, it, rel, ok = pcg(sysm.A, sysm.b, P, p["cg_rel_tol"], max_iter or p["cg_max_iter"])
    stats = dict(iters=it, rel_residual=rel, converged=ok,
                 new_broken=int(np.sum(zeta & ~state.zeta)), total_broken=int(zeta.sum()),
                 near_threshold=near, **sysm.stats)
    if not ok:
        return state, stats
    v = state.v + dv.reshape(-1, 3)
    x = state.x + p["dt"] * v
    return State(x, v, zeta, Cp, state.step + 1), stats


def run(mesh: Mesh, state: State, dir_nodes, dir_vel, n_steps: int, overrides=None):
    """n_steps of `step`; overrides[i] is the label override for step i."""
    hist = []
    for i in range(n_steps):
        ov = overrides[i] if overrides is not None and i < len(overrides) else None
        state, st = step(mesh, state, dir_nodes, dir_vel, override=ov)
        hist.append(st)
        if not st["converged"]:
            break
    return state, hist


# --------------------------------------------------------------------------
# Quasi-static load step: Newton with a backtracking line search (Eq. 36)
# --------------------------------------------------------------------------

def energy_fixed_chi(mesh: Mesh, x: np.ndarray, chi: np.ndarray, Cp=None) -> float:
    """E(x) = sum_e chi_e V_e Psi_e(x) with chi held fixed: the potential whose
    negative gradient is the restoring force f* of Eq. 32 at that chi."""
    return float(np.sum(mesh.V * chi * element(mesh, x, Cp).psi))


def quasi_static_step(mesh: Mesh, state: State, dir_nodes, dir_vel, newton_rtol: float = 1e-6,
                      max_newton: int = 50, armijo: float = 1e-4, min_step: float = 2.0 ** -20,
                      override: dict | None = None):
    """One load step of the quasi-static problem of Eq. 36, sum chi k u =
    sum chi f, solved for equilibrium by Newton's method with a backtracking
    line search on the total energy (Sec. 4.3, Sec. 5.1):

    1. damage and plastic flow at the previous equilibrium x_n;
    2. the prescribed nodes move by dt * their prescribed velocity;
    3. chi is evaluated at that first iterate and held fixed, so that
       E(x) = sum chi V Psi is the potential of the forces;
    4. Newton: f = f*(x) on the free nodes; stop when |f| <= newton_rtol |f_0|
       (f_0: the out-of-balance force of the first iterate) or f = 0; else
       solve (M / dt^2 + K*) dx = f with the prescribed rows fixed (the mass
       term is a regulariser that vanishes as dt grows and keeps the rows of
       detached fragments definite), then take the largest alpha in
       1, 1/2, 1/4, ... with E(x + alpha dx) <= E(x) - armijo alpha f.dx
       (accepted outright once the energy change is below FP64 resolution,
       |E(x + alpha dx) - E(x)| <= 1e-14 |E(x)|), x += alpha dx.
    Velocities are zero after the step.  Returns (new_state, stats); on
    failure (no equilibrium within max_newton iterations, a step below
    min_step, or a linear solve that misses its tolerance) the state is
    returned unchanged.  `override` as in `step` (labels of near-threshold
    edges only)."""
    p = mesh.params
    dt = p["dt"]
    n = mesh.X.shape[0]
    zeta, near = damage_update(mesh, state.x, state.zeta, override=override)
    Cp = plastic_update(mesh, state.x, state.Cp)
    dir_nodes = np.asarray(dir_nodes, dtype=np.int64)
    x = state.x.copy()
    if dir_nodes.size:
        x[dir_nodes] += dt * np.asarray(dir_vel, float)
    chi, _ = energy_fraction(mesh, x, zeta, Cp)
    cdof = (3 * dir_nodes[:, None] + np.arange(3)).ravel()
    keep = np.ones(3 * n)
    keep[cdof] = 0.0
    Dk = sp.diags(keep)
    stats = dict(newton_iters=0, halvings=0, inner_iters=0, converged=False, energy=[], force=[],
                 new_broken=int(np.sum(zeta & ~state.zeta)), total_broken=int(zeta.sum()), near_threshold=near)
    f0 = None
    for it in range(max_newton + 1):
        el = element(mesh, x, Cp)
        f = scatter_forces(n, mesh.tets, element_forces(mesh, el, chi)).ravel() * keep
        fn = float(np.linalg.norm(f))
        stats["force"].append(fn)
        if f0 is None:
            f0 = fn
        if fn == 0.0 or fn <= newton_rtol * f0:
            stats["converged"] = True
            break
        if it == max_newton:
            break
        K = assemble_stiffness(n, mesh.tets, element_stiffness(mesh, el, chi))
        A = (Dk @ (mesh.M / (dt * dt) + K) @ Dk + sp.diags(1.0 - keep)).tocsr()
        dx, its, rel, ok = pcg(A, f, block_jacobi(A), p["cg_rel_tol"], p["cg_max_iter"])
        stats["inner_iters"] += its
        if not ok:
            break
        dx = dx.reshape(-1, 3)
        E0 = energy_fixed_chi(mesh, x, chi, Cp)
        slope = float(f @ dx.ravel())
        alpha = 1.0
        while True:
            E1 = energy_fixed_chi(mesh, x + alpha * dx, chi, Cp)
            if E1 <= E0 - armijo * alpha * slope or abs(E1 - E0) <= 1e-14 * abs(E0):
                break
            alpha *= 0.5
            stats["halvings"] += 1
            if alpha < min_step:
                break
        if alpha < min_step:
            break
        x = x + alpha * dx
        stats["energy"].append(E1)
        stats["newton_iters"] = it + 1
    if not stats["converged"]:
        return state, stats
    return State(x, np.zeros_like(state.v), zeta, Cp, state.step + 1), stats


# --------------------------------------------------------------------------
# Visualisation mesh (Sec. 4.1): node-associated four-split of each tet
# --------------------------------------------------------------------------

def _component(nodes, start, unbroken):
    """Nodes of `nodes` reachable from `start` through unbroken edges whose
    both ends lie in `nodes`."""
    comp, stack = {start}, [start]
    while stack:
        a = stack.pop()
        for b in nodes:
            if b not in comp and unbroken(a, b):
                comp.add(b)
                stack.append(b)
    return comp


def visual_mesh(X: np.ndarray, x: np.ndarray, tets: np.ndarray, edges: np.ndarray, zeta: np.ndarray):
    """The split visualisation mesh of Sec. 4.1, one sub-cell per tet corner
    (the node-associated four-split: the corner, the centroids of its three
    edges, of its three faces and of the tet).  Each split point has one
    child per group of the tet's corners that its unbroken edges connect
    within that edge, face or tet; the child of corner a sits at the split
    point's rest position plus the mean displacement of a's group (a broken
    edge: each child follows its own parent; the face of the paper's example
    with both edges at PF1 broken: SF1 follows PF1, SF2 and SF3 the average
    of PF2 and PF3).  Loops over tets: small meshes only.

    Returns (xyz (m,4,8,3): per tet (caller order) and corner (caller local
    order) the sub-cell vertices [corner, edge points towards the other
    corners b1 < b2 < b3, face points (b1,b2), (b1,b3), (b2,b3), tet point];
    group (m,4) uint8: the smallest local corner index connected to each
    corner through unbroken edges of the tet)."""
    X = np.asarray(X, float)
    u = np.asarray(x, float) - X
    key = {(int(i), int(j)): bool(z) for (i, j), z in zip(edges, zeta)}
    m = tets.shape[0]
    xyz = np.zeros((m, 4, 8, 3))
    group = np.zeros((m, 4), np.uint8)
    for t in range(m):
        nd = [int(v) for v in tets[t]]

        def unbroken(a, b):
            i, j = nd[a], nd[b]
            return not key[(min(i, j), max(i, j))]

        def child(simplex, a):
            comp = _component(simplex, a, unbroken)
            rest = np.mean([X[nd[c]] for c in simplex], axis=0)
            return rest + np.mean([u[nd[c]] for c in comp], axis=0)

        for a in range(4):
            others = [b for b in range(4) if b != a]
            verts = [X[nd[a]] + u[nd[a]]]
            verts += [child([a, b], a) for b in others]
            verts += [child([a, b, c], a) for b, c in ((others[0], others[1]), (others[0], others[2]),
                                                        (others[1], others[2]))]
            verts.append(child([0, 1, 2, 3], a))
            xyz[t, a] = verts
            group[t, a] = min(_component([0, 1, 2, 3], a, unbroken))
    return xyz, group

