"""FP64 CPU oracle of the learned block preconditioner (message-passing network).

TEST INFRASTRUCTURE ONLY (see gfem_oracle.py).  Not part of the paper: the
paper solves with plain conjugate gradients.  This network predicts, per mesh
node i, a lower-triangular 3x3 factor L_i (exponentiated diagonal) and the
preconditioner block B_i = L_i A_ii^-1 L_i^T, so L = I is exactly 3x3
block-Jacobi and every B_i is symmetric positive definite.

Architecture (all sizes fixed):
  edge features (per edge i-j): f = (rest length / mean rest length,
      current length / rest length - 1, zeta)
  node input a_i (8): 1, and means over the incident edges of
      f0, f1, f2, f1^2, |f1|, (1 - zeta) f1, plus degree / 16
  embedding:  h0 = relu(W0 a + b0)                         (8 -> 64)
  3 layers:   m = P h  (mean over unbroken incident edges, P_ij = w_ij / sum_j w_ij, w = 1 - zeta)
              h <- h + relu(Wl [h; m] + bl)                 (128 -> 64)
  head:       o = Wh h + bh                                 (64 -> 6)
  L = [[e^o0, 0, 0], [o3, e^o1, 0], [o4, o5, e^o2]]
Two losses for one system A dv* = b:
  "solution": sum over free nodes |B_i b_i - dv*_i|^2 / sum |dv*_i|^2;
  "cg_step" (scale-invariant): log of the A-norm error left by one optimal
      preconditioned conjugate-gradient step from zero,
      log(u^T A u) - 2 log(b^T u) + log(b^T dv*) with u = B b
      (B on prescribed nodes fixed to A_ii^-1).

The backward pass is written out by hand; tests pin it to finite differences.
"""
from __future__ import annotations

import numpy as np

HIDDEN = 64
N_IN = 8
N_LAYERS = 3
N_OUT = 6

# parameter order (flat vector): W0 (64x8), b0 (64), [Wl (64x128), bl (64)] x 3, Wh (6x64), bh (6)
SHAPES = [("W0", (HIDDEN, N_IN)), ("b0", (HIDDEN,))]
for _l in range(N_LAYERS):
    SHAPES += [(f"W{_l + 1}", (HIDDEN, 2 * HIDDEN)), (f"b{_l + 1}", (HIDDEN,))]
SHAPES += [("Wh", (N_OUT, HIDDEN)), ("bh", (N_OUT,))]
N_PARAMS = int(sum(np.prod(s) for _, s in SHAPES))


def unflatten(w: np.ndarray) -> dict:
    out, o = {}, 0
    for name, shp in SHAPES:
        k = int(np.prod(shp))
        out[name] = w[o:o + k].reshape(shp)
        o += k
    return out


def flatten(p: dict) -> np.ndarray:
    return np.concatenate([p[name].ravel() for name, _ in SHAPES])


def init_weights(seed: int, head_scale: float = 0.0) -> np.ndarray:
    """He-style initial weights; the head starts at head_scale (0 = block-Jacobi)."""
    rng = np.random.default_rng(seed)
    p = {}
    for name, shp in SHAPES:
        if name.startswith("W") and name != "Wh":
            p[name] = rng.normal(size=shp) * np.sqrt(2.0 / shp[1])
        elif name == "Wh":
            p[name] = rng.normal(size=shp) * head_scale
        else:
            p[name] = np.zeros(shp)
    return flatten(p)


def edge_features(X: np.ndarray, x: np.ndarray, edges: np.ndarray, zeta: np.ndarray) -> np.ndarray:
    """(ne, 3): rest length / mean rest length, stretch - 1, zeta."""
    L0 = np.linalg.norm(X[edges[:, 1]] - X[edges[:, 0]], axis=1)
    L = np.linalg.norm(x[edges[:, 1]] - x[edges[:, 0]], axis=1)
    return np.stack([L0 / L0.mean(), L / L0 - 1.0, zeta.astype(float)], axis=1)


def node_inputs(n: int, edges: np.ndarray, f: np.ndarray) -> np.ndarray:
    """(n, 8) node input vector built from the incident edges' features."""
    per_edge = np.stack([f[:, 0], f[:, 1], f[:, 2], f[:, 1] ** 2, np.abs(f[:, 1]), (1 - f[:, 2]) * f[:, 1]], 1)
    acc = np.zeros((n, per_edge.shape[1]))
    deg = np.zeros(n)
    for side in (0, 1):
        np.add.at(acc, edges[:, side], per_edge)
        np.add.at(deg, edges[:, side], 1.0)
    mean = acc / np.maximum(deg, 1.0)[:, None]
    return np.concatenate([np.ones((n, 1)), mean, (deg / 16.0)[:, None]], axis=1)


def mean_operator(n: int, edges: np.ndarray, zeta: np.ndarray):
    """Dense-free representation of P: returns a function h -> P h and its transpose."""
    w = 1.0 - zeta.astype(float)
    deg = np.zeros(n)
    np.add.at(deg, edges[:, 0], w)
    np.add.at(deg, edges[:, 1], w)
    inv = np.where(deg > 0, 1.0 / np.where(deg > 0, deg, 1.0), 0.0)

    def P(h):
        out = np.zeros_like(h)
        np.add.at(out, edges[:, 0], w[:, None] * h[edges[:, 1]])
        np.add.at(out, edges[:, 1], w[:, None] * h[edges[:, 0]])
        return inv[:, None] * out

    def PT(g):
        gs = inv[:, None] * g
        out = np.zeros_like(g)
        np.add.at(out, edges[:, 0], w[:, None] * gs[edges[:, 1]])
        np.add.at(out, edges[:, 1], w[:, None] * gs[edges[:, 0]])
        return out

    return P, PT


def lower_factor(o: np.ndarray) -> np.ndarray:
    L = np.zeros((o.shape[0], 3, 3))
    L[:, 0, 0] = np.exp(o[:, 0])
    L[:, 1, 1] = np.exp(o[:, 1])
    L[:, 2, 2] = np.exp(o[:, 2])
    L[:, 1, 0] = o[:, 3]
    L[:, 2, 0] = o[:, 4]
    L[:, 2, 1] = o[:, 5]
    return L


def forward(w: np.ndarray, a: np.ndarray, P) -> dict:
    p = unflatten(w)
    cache = {"a": a}
    z0 = a @ p["W0"].T + p["b0"]
    h = np.maximum(z0, 0.0)
    cache["z0"], cache["h"] = z0, [h]
    cache["m"], cache["z"] = [], []
    for l in range(N_LAYERS):
        m = P(h)
        z = np.concatenate([h, m], 1) @ p[f"W{l + 1}"].T + p[f"b{l + 1}"]
        h = h + np.maximum(z, 0.0)
        cache["m"].append(m)
        cache["z"].append(z)
        cache["h"].append(h)
    cache["o"] = h @ p["Wh"].T + p["bh"]
    return cache


def precond_blocks(o: np.ndarray, Aii: np.ndarray) -> np.ndarray:
    """B_i = L_i A_ii^-1 L_i^T."""
    L = lower_factor(o)
    C = np.linalg.inv(Aii)
    return L @ C @ np.transpose(L, (0, 2, 1))


def loss_and_grad(w: np.ndarray, a: np.ndarray, P, PT, Aii: np.ndarray, b: np.ndarray, dv: np.ndarray,
                  free: np.ndarray, A=None, kind: str = "solution"):
    """Loss of one system and its gradient with respect to the flat weights.
    kind "cg_step" needs the assembled matrix A (3n x 3n)."""
    p = unflatten(w)
    c = forward(w, a, P)
    o = c["o"]
    L = lower_factor(o)
    C = np.linalg.inv(Aii)
    B = L @ C @ np.transpose(L, (0, 2, 1))
    if kind == "solution":
        r = np.einsum("nij,nj->ni", B, b) - dv
        r = r * free[:, None]
        D = float(np.sum((dv * free[:, None]) ** 2))
        loss = float(np.sum(r * r)) / D
        # dloss/dB = 2 r b^T / D
        G = 2.0 * np.einsum("ni,nj->nij", r, b) / D
    else:
        Bf = np.where(free[:, None, None] > 0, B, C)
        u = np.einsum("nij,nj->ni", Bf, b)
        wv = (A @ u.ravel()).reshape(-1, 3)
        s_ = float(np.sum(b * u))
        q_ = float(np.sum(u * wv))
        loss = np.log(q_) - 2.0 * np.log(s_) + np.log(float(np.sum(b * dv)))
        # dloss/dB_i = (2/q) w_i b_i^T - (2/s) b_i b_i^T on free nodes
        G = (2.0 / q_) * np.einsum("ni,nj->nij", wv, b) - (2.0 / s_) * np.einsum("ni,nj->nij", b, b)
        G = G * free[:, None, None]
    # dloss/dL = (G + G^T) L C
    GL = np.einsum("nij,njk,nkl->nil", G + np.transpose(G, (0, 2, 1)), L, C)
    go = np.zeros_like(o)
    go[:, 0] = GL[:, 0, 0] * L[:, 0, 0]
    go[:, 1] = GL[:, 1, 1] * L[:, 1, 1]
    go[:, 2] = GL[:, 2, 2] * L[:, 2, 2]
    go[:, 3] = GL[:, 1, 0]
    go[:, 4] = GL[:, 2, 0]
    go[:, 5] = GL[:, 2, 1]
    g = {k: np.zeros_like(v) for k, v in p.items()}
    h = c["h"]
    g["Wh"] = go.T @ h[-1]
    g["bh"] = go.sum(0)
    gh = go @ p["Wh"]
    for l in reversed(range(N_LAYERS)):
        gz = gh * (c["z"][l] > 0)
        inp = np.concatenate([h[l], c["m"][l]], 1)
        g[f"W{l + 1}"] = gz.T @ inp
        g[f"b{l + 1}"] = gz.sum(0)
        gi = gz @ p[f"W{l + 1}"]
        gh = gh + gi[:, :HIDDEN] + PT(gi[:, HIDDEN:])
    gz0 = gh * (c["z0"] > 0)
    g["W0"] = gz0.T @ c["a"]
    g["b0"] = gz0.sum(0)
    return loss, flatten(g), B


def system_data(mesh, state, sysm, dv: np.ndarray, dir_nodes):
    """Per-node diagonal blocks, right-hand side, solution and free mask of an
    assembled oracle system (gfem_oracle.System)."""
    n = mesh.X.shape[0]
    A = sysm.A
    Aii = np.zeros((n, 3, 3))
    for r in range(3):
        for cc in range(3):
            Aii[:, r, cc] = A.diagonal(cc - r)[np.arange(n) * 3 + min(r, cc)]
    free = np.ones(n)
    free[np.asarray(dir_nodes, dtype=int)] = 0.0
    return Aii, sysm.b.reshape(-1, 3), dv.reshape(-1, 3), free
