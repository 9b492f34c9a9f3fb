"""FP64 CPU oracle of the learned preconditioner (message-passing network).

TEST INFRASTRUCTURE ONLY (see gfem_oracle.py).  Not part of the paper: the
paper solves with plain conjugate gradients.

Preconditioner family (factorised sparse approximate inverse): B = G^T G with
G block lower triangular on the lower block pattern of A (3x3 blocks, node
order):
    G_ii = L_i C_i,        C_i = inverse of the lower Cholesky factor of A_ii,
    G_ij = -L_i C_i W_ij A_ij A_jj^-1      for every stored block j < i,
L_i lower triangular with exponentiated diagonal and W_ij a 3x3 block, both
predicted by the network.  L = I, W = 0 gives B = blockdiag(A_ii^-1), i.e.
3x3 block-Jacobi; W = w I is a damped first-order (Neumann) approximation of
the inverse Cholesky factor.  Prescribed nodes keep G_ii = I (their rows and
columns of A are the identity).

Network (all sizes fixed):
  edge features (per edge i-j): f = (rest length / mean rest length,
      tanh(current length / rest length - 1), zeta)
  node input a_i (8): 1, and means over the incident edges of
      f0, f1, f2, f1^2, |f1|, (1 - zeta) f1, plus degree / 16
  embedding:  h0 = relu(W0 a + b0)                         (8 -> 64)
  3 layers:   m = P h  (mean over unbroken incident edges, P_ij = w_ij / sum_j w_ij, w = 1 - zeta)
              h <- h + relu(Wl [h; m] + bl)                 (128 -> 64)
  node head:  o = Wh h + bh                                 (64 -> 24)
      o[0:6]   -> L = [[e^b(o0), 0, 0], [b(o3), e^b(o1), 0], [b(o4), b(o5), e^b(o2)]]
      o[6:15]  -> s_i,  o[15:24] -> t_i
  edge term:  W_ij = b(s_i + t_j + We f_ij + be)  (9 values, row-major 3x3)
with the bounded map b(x) = 2 tanh(x / 2) (slope 1 at 0, range (-2, 2)), so
that no input drives the factor to overflow: the diagonal of L stays within
(e^-2, e^2) and every W entry within (-2, 2).  The pre-activation of the edge
term is linear in (h_i, h_j, f_ij), so it costs one node GEMM and a gather per
block.

Training objective (one system, one probe vector v with entries +-1):
Kaporin's condition number of G A G^T, K = (tr(GAG^T)/N)^N / det(GAG^T),
estimated with the probe (E[v^T X v] = tr X):
    loss = log(v^T G A G^T v / N) - (2/N) log det G     (N = 3n)
which is log K / N up to the constant log det A / N.  Its exact minimiser over
all G with this block pattern is the classical factorised sparse approximate
inverse (Kolotilina-Yeremin), so the network learns an approximation of that
preconditioner from local features.  The backward pass is written out by
hand; tests pin it to finite differences.

Power-weighted variant: the probe is first replaced by X^k v (X = G A G^T),
rescaled to |v|^2 = N, so that the first term is the Rayleigh quotient of
X^k v.  Over the eigen-decomposition of X it weighs eigenvalue lambda by
lambda^(2k) times the probe's component: k = 0 is the mean (Kaporin), and as
k grows it tends to the largest eigenvalue, the end of the spectrum that
conjugate gradients pays for and the mean hardly sees.  The gradient holds
the stepped probe fixed (loss_and_grad with that probe).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp
from scipy.linalg import solve_triangular

HIDDEN = 64
N_IN = 8
N_LAYERS = 3
N_HEAD = 24
N_EDGE_F = 3

# parameter order (flat vector): W0 (64x8), b0 (64), [Wl (64x128), bl (64)] x 3,
# Wh (24x64), bh (24), We (9x3), be (9)
SHAPES = [("W0", (HIDDEN, N_IN)), ("b0", (HIDDEN,))]
for _l in range(N_LAYERS):
    SHAPES += [(f"W{_l + 1}", (HIDDEN, 2 * HIDDEN)), (f"b{_l + 1}", (HIDDEN,))]
SHAPES += [("Wh", (N_HEAD, HIDDEN)), ("bh", (N_HEAD,)), ("We", (9, N_EDGE_F)), ("be", (9,))]
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


def offset(name: str) -> int:
    o = 0
    for nm, shp in SHAPES:
        if nm == name:
            return o
        o += int(np.prod(shp))
    raise KeyError(name)


def init_weights(seed: int, head_scale: float = 0.0) -> np.ndarray:
    """He-style hidden layers; head and edge term drawn with std head_scale
    (0 = block-Jacobi)."""
    rng = np.random.default_rng(seed)
    p = {}
    for name, shp in SHAPES:
        if name in ("Wh", "We"):
            p[name] = rng.normal(size=shp) * head_scale
        elif name.startswith("W"):
            p[name] = rng.normal(size=shp) * np.sqrt(2.0 / shp[1])
        else:
            p[name] = np.zeros(shp)
    return flatten(p)


def edge_features(X: np.ndarray, x: np.ndarray, edges: np.ndarray, zeta: np.ndarray) -> np.ndarray:
    """(ne, 3): rest length / mean rest length, tanh(stretch - 1), zeta."""
    L0 = np.linalg.norm(X[edges[:, 1]] - X[edges[:, 0]], axis=1)
    L = np.linalg.norm(x[edges[:, 1]] - x[edges[:, 0]], axis=1)
    return np.stack([L0 / L0.mean(), np.tanh(L / L0 - 1.0), zeta.astype(float)], axis=1)


def bound(x: np.ndarray) -> np.ndarray:
    """b(x) = 2 tanh(x / 2)."""
    return 2.0 * np.tanh(0.5 * x)


def bound_slope(x: np.ndarray) -> np.ndarray:
    """b'(x) = 1 - tanh(x / 2)^2."""
    return 1.0 - np.tanh(0.5 * x) ** 2


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
    bo = bound(o)
    L = np.zeros((o.shape[0], 3, 3))
    L[:, 0, 0] = np.exp(bo[:, 0])
    L[:, 1, 1] = np.exp(bo[:, 1])
    L[:, 2, 2] = np.exp(bo[:, 2])
    L[:, 1, 0] = bo[:, 3]
    L[:, 2, 0] = bo[:, 4]
    L[:, 2, 1] = bo[:, 5]
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


@dataclass
class Factor:
    """Lower block pattern of an assembled system and the fixed pieces of G."""
    n: int
    rows: np.ndarray     # (nb,) block row i of each stored block j < i
    cols: np.ndarray     # (nb,) block column j
    Ablk: np.ndarray     # (nb, 3, 3) A_ij
    K: np.ndarray        # (nb, 3, 3) A_ij A_jj^-1
    C: np.ndarray        # (n, 3, 3) inverse lower Cholesky factor of A_ii
    fb: np.ndarray       # (nb, 3) features of the block's edge
    free: np.ndarray     # (n,) 1 for free nodes, 0 for prescribed


def diagonal_blocks(A: sp.csr_matrix) -> np.ndarray:
    n = A.shape[0] // 3
    D = np.zeros((n, 3, 3))
    for r in range(3):
        for c in range(3):
            D[:, r, c] = A.diagonal(c - r)[np.arange(n) * 3 + min(r, c)]
    return D


def make_factor(A: sp.csr_matrix, edges: np.ndarray, f: np.ndarray, free: np.ndarray) -> Factor:
    """Stored lower blocks of A: every mesh edge (i, j), i < j, is block (j, i)."""
    n = A.shape[0] // 3
    D = diagonal_blocks(A)
    rows = edges[:, 1].astype(np.int64)
    cols = edges[:, 0].astype(np.int64)
    Ad = A.toarray() if n <= 3000 else None
    Ablk = np.zeros((len(rows), 3, 3))
    Acsr = A.tocsr()
    for k, (i, j) in enumerate(zip(rows, cols)):
        Ablk[k] = Ad[3 * i:3 * i + 3, 3 * j:3 * j + 3] if Ad is not None else \
            Acsr[3 * i:3 * i + 3, 3 * j:3 * j + 3].toarray()
    K = Ablk @ np.linalg.inv(D)[cols]
    C = np.linalg.inv(np.linalg.cholesky(D))
    return Factor(n, rows, cols, Ablk, K, C, f, free.astype(float))


def edge_preactivation(o: np.ndarray, w: np.ndarray, fac: Factor) -> np.ndarray:
    """(nb, 9): s_i + t_j + We f_ij + be for every stored lower block (i, j)."""
    p = unflatten(w)
    return o[fac.rows, 6:15] + o[fac.cols, 15:24] + fac.fb @ p["We"].T + p["be"]


def factor_blocks(o: np.ndarray, w: np.ndarray, fac: Factor):
    """(Gd (n,3,3), Gl (nb,3,3), W (nb,3,3)) for head outputs o (n,24)."""
    L = lower_factor(o[:, :6])
    L[fac.free == 0] = np.eye(3)
    M = L @ fac.C
    W = bound(edge_preactivation(o, w, fac)).reshape(-1, 3, 3)
    Gl = -np.einsum("bij,bjk,bkl->bil", M[fac.rows], W, fac.K)
    return M, Gl, W


def G_matrix(fac: Factor, Gd: np.ndarray, Gl: np.ndarray) -> sp.csr_matrix:
    """Assemble G as a sparse (3n x 3n) matrix."""
    rows = np.concatenate([np.arange(fac.n), fac.rows])
    cols = np.concatenate([np.arange(fac.n), fac.cols])
    blocks = np.concatenate([Gd, Gl])
    r = (3 * rows[:, None, None] + np.arange(3)[None, :, None]).repeat(3, 2).ravel()
    c = (3 * cols[:, None, None] + np.arange(3)[None, None, :]).repeat(3, 1).ravel()
    return sp.csr_matrix((blocks.ravel(), (r, c)), shape=(3 * fac.n, 3 * fac.n))


def apply(fac: Factor, Gd: np.ndarray, Gl: np.ndarray, r: np.ndarray) -> np.ndarray:
    """z = G^T G r (r and z of shape (n, 3))."""
    y = np.einsum("nij,nj->ni", Gd, r)
    np.add.at(y, fac.rows, np.einsum("bij,bj->bi", Gl, r[fac.cols]))
    z = np.einsum("nji,nj->ni", Gd, y)
    np.add.at(z, fac.cols, np.einsum("bji,bj->bi", Gl, y[fac.rows]))
    return z


def normalise_rows(fac: Factor, Gd: np.ndarray, Gl: np.ndarray, A: sp.csr_matrix):
    """Row normalisation: every block row of G is multiplied from the left by
    N_i, the inverse of the lower Cholesky factor of the diagonal block
    (G A G^T)_ii, so that block becomes I.  A row whose block is not positive
    definite is left as it is.  Returns the new (Gd, Gl)."""
    G = G_matrix(fac, Gd, Gl)
    Xd = diagonal_blocks((G @ A @ G.T).tocsr())
    N = np.empty_like(Xd)
    for i in range(fac.n):
        try:
            N[i] = solve_triangular(np.linalg.cholesky(Xd[i]), np.eye(3), lower=True)
        except np.linalg.LinAlgError:
            N[i] = np.eye(3)
    return N @ Gd, N[fac.rows] @ Gl


def power_probe(fac: Factor, Gd: np.ndarray, Gl: np.ndarray, A: sp.csr_matrix, v: np.ndarray, k: int) -> np.ndarray:
    """The probe after k power steps on X = G A G^T: v <- X v, rescaled to
    |v|^2 = N (N = 3n) after every step.  k = 0 returns v."""
    G = G_matrix(fac, Gd, Gl)
    N = 3 * fac.n
    x = np.array(v, dtype=float).ravel()
    for _ in range(k):
        y = G @ (A @ (G.T @ x))
        x = y * np.sqrt(N / (y @ y))
    return x.reshape(-1, 3)


def loss_and_grad_power(w: np.ndarray, a: np.ndarray, P, PT, fac: Factor, A: sp.csr_matrix, v: np.ndarray, k: int):
    """Power-weighted loss: loss_and_grad with the probe after k power steps
    on this network's X (held fixed in the gradient)."""
    Gd, Gl, _ = factor_blocks(forward(w, a, P)["o"], w, fac)
    return loss_and_grad(w, a, P, PT, fac, A, power_probe(fac, Gd, Gl, A, v, k))


def loss_and_grad(w: np.ndarray, a: np.ndarray, P, PT, fac: Factor, A: sp.csr_matrix, v: np.ndarray):
    """Kaporin probe loss of one system and its gradient w.r.t. the flat weights.
    v: (n, 3) probe.  Returns (loss, grad, (Gd, Gl))."""
    p = unflatten(w)
    c = forward(w, a, P)
    o = c["o"]
    Gd, Gl, W = factor_blocks(o, w, fac)
    N = 3 * fac.n
    # u = G^T v, w = A u, t = u.w
    u = np.einsum("nji,nj->ni", Gd, v)
    np.add.at(u, fac.cols, np.einsum("bji,bj->bi", Gl, v[fac.rows]))
    wv = (A @ u.ravel()).reshape(-1, 3)
    t = float(np.sum(u * wv))
    L = lower_factor(o[:, :6])
    logdet = float(np.sum(np.log(np.abs(np.linalg.det(Gd)))))
    slope_o = bound_slope(o[:, :6])
    slope_w = bound_slope(edge_preactivation(o, w, fac))
    loss = np.log(t / N) - 2.0 / N * logdet
    # dloss/dW_b = -(2/t) (M_i^T v_i)(K_b w_j)^T
    m = np.einsum("nji,nj->ni", Gd, v)                       # M_i^T v_i
    k = np.einsum("bij,bj->bi", fac.K, wv[fac.cols])         # K_b w_j
    dW = -(2.0 / t) * np.einsum("bi,bj->bij", m[fac.rows], k)
    # dloss/dL_i = (2/t) v_i rho_i^T - (2/N) L_i^-T, rho_i = C_i (w_i - sum_b W_b k_b)
    s = wv.copy()
    np.add.at(s, fac.rows, -np.einsum("bij,bj->bi", W, k))
    rho = np.einsum("nij,nj->ni", fac.C, s)
    dL = (2.0 / t) * np.einsum("ni,nj->nij", v, rho) - (2.0 / N) * np.transpose(np.linalg.inv(L), (0, 2, 1))
    go = np.zeros_like(o)
    go[:, 0] = dL[:, 0, 0] * L[:, 0, 0]
    go[:, 1] = dL[:, 1, 1] * L[:, 1, 1]
    go[:, 2] = dL[:, 2, 2] * L[:, 2, 2]
    go[:, 3] = dL[:, 1, 0]
    go[:, 4] = dL[:, 2, 0]
    go[:, 5] = dL[:, 2, 1]
    go[:, :6] *= slope_o
    go[fac.free == 0, :6] = 0.0
    dWv = dW.reshape(-1, 9) * slope_w
    np.add.at(go[:, 6:15], fac.rows, dWv)
    np.add.at(go[:, 15:24], fac.cols, dWv)
    g = {kk: np.zeros_like(vv) for kk, vv in p.items()}
    g["We"] = dWv.T @ fac.fb
    g["be"] = dWv.sum(0)
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
    return loss, flatten(g), (Gd, Gl)


def system_inputs(mesh, x: np.ndarray, zeta: np.ndarray, A: sp.csr_matrix, dir_nodes):
    """Network inputs and the factor pattern of an assembled oracle system."""
    n = mesh.X.shape[0]
    free = np.ones(n)
    free[np.asarray(dir_nodes, dtype=int)] = 0.0
    f = edge_features(mesh.X, x, mesh.edges, zeta)
    a = node_inputs(n, mesh.edges, f)
    P, PT = mean_operator(n, mesh.edges, zeta)
    fac = make_factor(A, mesh.edges, f, free)
    return a, P, PT, fac
