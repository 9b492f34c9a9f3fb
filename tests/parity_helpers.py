"""Shared helpers for the GPU-vs-oracle parity tests (test infrastructure)."""
from __future__ import annotations

import sys

import numpy as np
import scipy.sparse as sp

from oracle import gfem_oracle as O
from paper_2103_14870_amd import gfem


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def gpu_sparse(bi, bj, blocks, n):
    """COO 3x3 blocks -> (3n,3n) CSR."""
    r = (3 * bi[:, None, None] + np.arange(3)[None, :, None]).repeat(3, axis=2)
    c = (3 * bj[:, None, None] + np.arange(3)[None, None, :]).repeat(3, axis=1)
    return sp.coo_matrix((blocks.ravel(), (r.ravel(), c.ravel())), shape=(3 * n, 3 * n)).tocsr()


def rel(a, b):
    d = np.linalg.norm(np.asarray(a) - np.asarray(b))
    s = np.linalg.norm(np.asarray(b))
    return d / s if s > 0 else d


def rowrel(a, b, floor):
    """Largest per-row relative error: rows are nodes ((n,3) vectors) or
    blocks ((nb,3,3)); each row's error |a_i - b_i| is divided by
    max(|b_i|, floor * max_j |b_j|), so rows whose reference is tiny are
    measured against that floor instead of their own size."""
    a = np.asarray(a, float).reshape(np.shape(b)[0], -1)
    b = np.asarray(b, float).reshape(np.shape(b)[0], -1)
    nb = np.linalg.norm(b, axis=1)
    big = nb.max() if nb.size else 0.0
    if big == 0.0:
        return float(np.abs(a).max()) if a.size else 0.0
    d = np.linalg.norm(a - b, axis=1)
    return float((d / np.maximum(nb, floor * big)).max())


def block_rowrel(bi, bj, blocks, A_ref, floor):
    """rowrel over the stored 3x3 blocks of a GPU system against a (3n,3n)
    reference matrix."""
    A_ref = A_ref.tocsr()
    ref = np.zeros_like(blocks)
    for r in range(3):
        for c in range(3):
            ref[:, r, c] = np.asarray(A_ref[3 * bi + r, 3 * bj + c]).ravel()
    return rowrel(blocks, ref, floor)


def oracle_near(mesh, st):
    """Edges the oracle's next damage pass finds within 1e-6 of the threshold
    (local strain, or the non-local averaged strain in any tet of the edge)."""
    _, near = O.damage_update(mesh, st.x, st.zeta)
    return near


def lockstep(prob, n_steps, check_every=1, on_step=None):
    """Run the GPU library and the oracle side by side.  Near-threshold edges
    (|strain - threshold| < 1e-6) adopt the GPU's label in the oracle so that
    the trajectories stay comparable; every other label must agree exactly.
    Returns (gpu mesh, oracle mesh, oracle state, history)."""
    m = gfem.mesh_from_problem(prob)
    mesh = O.setup(prob.X, prob.tets, prob.params)
    st = O.initial_state(mesh)
    O.break_pairs(mesh, st, prob.broken_pairs)
    hist = []
    for i in range(n_steps):
        g = m.step(1)
        zg = m.edge_damage().astype(bool)
        near = oracle_near(mesh, st)
        st, h = O.step(mesh, st, prob.dir_nodes, prob.dir_vel, override={int(e): bool(zg[e]) for e in near})
        assert h["converged"], f"oracle did not converge at step {i}"
        mism = np.nonzero(zg != st.zeta)[0]
        # the GPU reports the same near-threshold edges (both evaluate the
        # strain in FP64, from the same displacement)
        gn = m.near_threshold_edges()
        rec = dict(step=i, gpu=g, oracle=h, label_mismatch=int(mism.size), near=int(near.size),
                   near_ids_match=bool(np.array_equal(np.sort(gn), np.sort(near))))
        if (i + 1) % check_every == 0 or i == n_steps - 1:
            x = m.positions()
            rec["pos_rel"] = rel(x, st.x)
            rec["disp_rel"] = rel(x - prob.X, st.x - prob.X)
            # per node, against max(|u_i|, 1e-3 max |u|)
            rec["disp_node"] = rowrel(x - prob.X, st.x - prob.X, 1e-3)
        hist.append(rec)
        if on_step:
            on_step(i, m, mesh, st)
        assert mism.size == 0, f"step {i}: {mism.size} labels differ away from the threshold"
    return m, mesh, st, hist
