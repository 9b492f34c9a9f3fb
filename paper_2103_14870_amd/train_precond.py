"""Train the learned block preconditioner on systems the method itself generates.

Each training system is the next timestep of a running simulation: the
library assembles it, runs the network forward, builds the factor G, draws a
+-1 probe, applies k power steps of G A G^T to it (default 16) and takes one
Adam step on the power-weighted Kaporin loss (forward and backward on the
GPU); the simulation then advances one step.  Plain Kaporin (k = 0) weighs
the spectrum of G A G^T by its mean and trains couplings that stretch its top
end on heavily damaged states; the power steps shift the weight towards the
largest eigenvalues.  Episodes are seeded variants of the beam, cube and
ellipsoid workloads (smaller meshes, varied jitter, damage threshold, load
rate and pre-cracked fraction).  The shipped weights come from the defaults:

    python -m paper_2103_14870_amd.train_precond --log-every 20000 \
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


def episode(rng: np.random.Generator, max_steps: int, fine_fraction: float = 0.0):
    """One seeded training problem (split precision) and its number of steps.
    Ellipsoid episodes run long enough to reach heavy ductile damage.  A
    fraction fine_fraction of the episodes are "fine" ellipsoids: cells of the
    620k-tet workload's size (2.165 cm, +-10 %) on a body scaled down to
    0.3-0.55 of it (semi-axes, end caps and pull per step scaled alike, so the
    same strain per step and the same stiffness-to-mass ratio per cell)."""
    base = np.array([0.4, 0.2, 0.4]) * (1.0 - fine_fraction)
    kind = rng.choice(["beam", "cube", "ellipsoid", "fine"], p=[*base, fine_fraction])
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
    elif kind == "fine":
        sc = float(rng.uniform(0.3, 0.55))
        h = 0.02165 * float(rng.uniform(0.9, 1.1))
        grid = (int(math.ceil(2.1 * sc / h)) | 1, int(math.ceil(1.1 * sc / h)) | 1, int(math.ceil(1.1 * sc / h)) | 1)
        prob = meshgen.ellipsoid(h=h, axes=(sc, 0.5 * sc, 0.5 * sc), grid=grid, jitter_frac=0.1,
                                 seed=int(rng.integers(1000, 10 ** 6)), cap=0.9 * sc, pull_per_step=0.01 * sc,
                                 dt=1e-2)
        steps = int(rng.integers(max_steps // 4, max_steps + 1))
    else:
        h = float(rng.uniform(0.06, 0.1))
        grid = (int(math.ceil(2.1 / h)) | 1, int(math.ceil(1.1 / h)) | 1, int(math.ceil(1.1 / h)) | 1)
        prob = meshgen.ellipsoid(h=h, grid=grid, jitter_frac=0.1, seed=int(rng.integers(1000, 10 ** 6)), dt=1e-2)
        steps = int(rng.integers(max_steps // 4, max_steps + 1))
    prob.params["damage_strain"] *= thr_scale
    prob.dir_vel = prob.dir_vel * rate
    return prob, steps


def train(n_systems: int, seed: int, max_steps: int, lr0: float, lr1: float, log_every: int,
          net: "gfem.Net | None" = None, verbose: bool = True, fine_fraction: float = 0.0):
    rng = np.random.default_rng(seed)
    net = net or gfem.Net(seed=seed)
    done = 0
    hist = []
    t0 = time.time()
    while done < n_systems:
        prob, steps = episode(rng, max_steps, fine_fraction)
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
    ap.add_argument("--systems", type=int, default=80000)
    ap.add_argument("--seed", type=int, default=2024)
    ap.add_argument("--max-steps", type=int, default=100, help="longest episode (ellipsoids; others half)")
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--lr-final", type=float, default=1e-4)
    ap.add_argument("--log-every", type=int, default=500)
    ap.add_argument("--out", default=DEFAULT_WEIGHTS)
    ap.add_argument("--power-steps", type=int, default=16,
                    help="power steps on G A G^T applied to each training probe (0: plain Kaporin)")
    ap.add_argument("--fine-fraction", type=float, default=0.0,
                    help="fraction of episodes on fine ellipsoids (cells of the 620k-tet workload's size)")
    ap.add_argument("--init-omega", type=float, default=None,
                    help="start from the constant member W = omega I (edge bias only) instead of block-Jacobi")
    ap.add_argument("--init-weights", default=None,
                    help="start from these weights (.npy, e.g. the shipped ones) instead of block-Jacobi")
    args = ap.parse_args()
    gfem.load()
    net = gfem.Net(seed=args.seed)
    net.set_power_steps(args.power_steps)
    if args.init_weights is not None:
        net.set_weights(np.load(args.init_weights))
    if args.init_omega is not None:
        if not 0.0 <= args.init_omega < 2.0:
            raise SystemExit("--init-omega must lie in [0, 2)")
        w = net.get_weights()  # the edge bias be (3x3, row-major) is the last 9 parameters
        w[-9:] = (2.0 * np.arctanh(args.init_omega / 2.0) * np.eye(3)).ravel()
        net.set_weights(w)
    if not 0.0 <= args.fine_fraction <= 1.0:
        raise SystemExit("--fine-fraction must lie in [0, 1]")
    net, hist = train(args.systems, args.seed, args.max_steps, args.lr, args.lr_final, args.log_every, net=net,
                      fine_fraction=args.fine_fraction)
    os.makedirs(os.path.dirname(os.path.abspath(args.out)), exist_ok=True)
    np.save(args.out, net.get_weights())
    k = max(1, len(hist) // 10)
    print(f"train: saved {args.out}; mean loss first {k}: {hist[:k].mean():.4f}, last {k}: {hist[-k:].mean():.4f}",
          flush=True)


if __name__ == "__main__":
    main()
