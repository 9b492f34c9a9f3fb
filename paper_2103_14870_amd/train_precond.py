"""Train the learned block preconditioner on systems the method itself generates.

Each training system is the next timestep of a running simulation: the
library assembles it, runs the network forward, builds the factor G, draws a
+-1 probe and takes one Adam step on Kaporin's condition number of G A G^T
(forward and backward on the GPU); the simulation then advances one step.  Episodes are seeded
variants of the beam, cube and ellipsoid workloads (smaller meshes, varied
jitter, damage threshold, load rate and pre-cracked fraction).

    python -m paper_2103_14870_amd.train_precond --systems 20000 \\
        --out paper_2103_14870_amd/weights/precond_net.npy
"""
from __future__ import annotations

import argparse
import math
import os
import sys
import time

import numpy as np

if __package__ in (None, ""):
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    from paper_2103_14870_amd import gfem, meshgen  # noqa: E402
else:
    from . import gfem, meshgen

DEFAULT_WEIGHTS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "weights", "precond_net.npy")


def episode(rng: np.random.Generator, max_steps: int):
    """One seeded training problem (split precision) and its number of steps.
    Ellipsoid episodes run long enough to reach heavy ductile damage."""
    kind = rng.choice(["beam", "cube", "ellipsoid"], p=[0.4, 0.2, 0.4])
    thr_scale = rng.uniform(0.8, 1.2)
    rate = rng.uniform(0.5, 2.0)
    if kind == "beam":
        nx = int(rng.integers(12, 33))
        ny = int(rng.integers(3, 7))
        prob = meshgen.notched_beam(nx, ny, ny, h=0.01, notch_cells=max(1, ny // 4),
                                    crack_fraction=float(rng.uniform(0.0, 0.3)) * (rng.random() < 0.7),
                                    crack_seed=int(rng.integers(100, 10 ** 6)))
        steps = int(rng.integers(max_steps // 4, max_steps // 2 + 1))
    elif kind == "cube":
        n = int(rng.integers(4, 9))
        prob = meshgen.cube_block(n, n, n, h=0.1, jitter_frac=0.05, seed=int(rng.integers(1000, 10 ** 6)),
                                  precision="split", cg_rel_tol=1e-6)
        steps = int(rng.integers(max_steps // 4, max_steps // 2 + 1))
    else:
        h = float(rng.uniform(0.06, 0.1))
        grid = (int(math.ceil(2.1 / h)) | 1, int(math.ceil(1.1 / h)) | 1, int(math.ceil(1.1 / h)) | 1)
        prob = meshgen.ellipsoid(h=h, grid=grid, jitter_frac=0.1, seed=int(rng.integers(1000, 10 ** 6)), dt=1e-2)
        steps = int(rng.integers(max_steps // 4, max_steps + 1))
    prob.params["damage_strain"] *= thr_scale
    prob.dir_vel = prob.dir_vel * rate
    return prob, steps


def train(n_systems: int, seed: int, max_steps: int, lr0: float, lr1: float, log_every: int,
          net: "gfem.Net | None" = None, verbose: bool = True):
    rng = np.random.default_rng(seed)
    net = net or gfem.Net(seed=seed)
    done = 0
    hist = []
    t0 = time.time()
    while done < n_systems:
        prob, steps = episode(rng, max_steps)
        with gfem.mesh_from_problem(prob) as m:
            for _ in range(steps):
                if done >= n_systems:
                    break
                frac = done / max(1, n_systems - 1)
                lr = lr1 + 0.5 * (lr0 - lr1) * (1 + math.cos(math.pi * frac))
                try:
                    loss = net.train_step(m, lr)
                except gfem.GfemError:
                    break
                hist.append(loss)
                done += 1
                if verbose and done % log_every == 0:
                    print(f"train: {done}/{n_systems} systems, loss (last {log_every}) "
                          f"{np.mean(hist[-log_every:]):.4f}, lr {lr:.2e}, {time.time() - t0:.0f} s", flush=True)
                out = m.step(1, raise_on_error=False)
                if out["status"] != gfem.GF_OK:
                    break
    return net, np.array(hist)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--systems", type=int, default=20000)
    ap.add_argument("--seed", type=int, default=2024)
    ap.add_argument("--max-steps", type=int, default=100, help="longest episode (ellipsoids; others half)")
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--lr-final", type=float, default=1e-4)
    ap.add_argument("--log-every", type=int, default=500)
    ap.add_argument("--out", default=DEFAULT_WEIGHTS)
    args = ap.parse_args()
    gfem.load()
    net, hist = train(args.systems, args.seed, args.max_steps, args.lr, args.lr_final, args.log_every)
    os.makedirs(os.path.dirname(os.path.abspath(args.out)), exist_ok=True)
    np.save(args.out, net.get_weights())
    k = max(1, len(hist) // 10)
    print(f"train: saved {args.out}; mean loss first {k}: {hist[:k].mean():.4f}, last {k}: {hist[-k:].mean():.4f}",
          flush=True)


if __name__ == "__main__":
    main()
