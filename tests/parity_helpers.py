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
        eps = O.edge_strain(mesh, st.x)
        near = np.nonzero(np.abs(eps - prob.params["damage_strain"]) < 1e-6)[0]
        st, h = O.step(mesh, st, prob.dir_nodes, prob.dir_vel, override={int(e): bool(zg[e]) for e in near})
        assert h["converged"], f"oracle did not converge at step {i}"
        mism = np.nonzero(zg != st.zeta)[0]
        rec = dict(step=i, gpu=g, oracle=h, label_mismatch=int(mism.size), near=int(near.size))
        if (i + 1) % check_every == 0 or i == n_steps - 1:
            x = m.positions()
            rec["pos_rel"] = rel(x, st.x)
            rec["disp_rel"] = rel(x - prob.X, st.x - prob.X)
        hist.append(rec)
        if on_step:
            on_step(i, m, mesh, st)
        assert mism.size == 0, f"step {i}: {mism.size} labels differ away from the threshold"
    return m, mesh, st, hist
