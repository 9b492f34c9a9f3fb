"""GPU parity of the quasi-static load step (Eq. 36; Newton with a
backtracking line search on the total energy, Sec. 4.3 / Sec. 5.1): blocks
pulled apart load step by load step, lockstep with the FP64 oracle -- labels
identical away from the threshold, positions, Newton iteration counts -- for
the stable neo-Hookean and StVK energies, the local and the non-local
criterion (the stone and wood settings of Sec. 5.1), FP64 and split
precision; a twisted block with a demanding Armijo constant so that the
line search acts; a failed load step leaves the state unchanged."""
import numpy as np
import pytest

from oracle import gfem_oracle as O
from paper_2103_14870_amd import gfem, meshgen

from parity_helpers import oracle_near, rel, rowrel, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _lib():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    gfem.load()


def pulled_block(prec, energy="stable_neo_hookean", radius=0.0, speed=0.004):
    """A 6 x 3 x 3 block of 5 cm cubes pulled along z, the top face moving by
    `speed` per load step (pseudo-timestep 1), brittle."""
    prob = meshgen.cube_block(3, 3, 6, h=0.05, jitter_frac=0.08, seed=9, top_speed=speed, dt=1.0,
                              precision=prec, cg_rel_tol=1e-10 if prec == "fp64" else 1e-6, damage_strain=0.03,
                              energy=energy)
    prob.params["damage_radius"] = radius
    return prob


def qs_lockstep(prob, n_steps, rtol, armijo=1e-4, max_newton=60):
    m = gfem.mesh_from_problem(prob)
    mesh = O.setup(prob.X, prob.tets, prob.params)
    st = O.initial_state(mesh)
    O.break_pairs(mesh, st, prob.broken_pairs)
    hist = []
    for i in range(n_steps):
        g = m.quasi_static_step(1, newton_rel_tol=rtol, max_newton=max_newton, armijo=armijo)
        zg = m.edge_damage().astype(bool)
        near = oracle_near(mesh, st)
        st, h = O.quasi_static_step(mesh, st, prob.dir_nodes, prob.dir_vel, newton_rtol=rtol, armijo=armijo,
                                    max_newton=max_newton, override={int(e): bool(zg[e]) for e in near})
        assert h["converged"], f"oracle load step {i} did not converge"
        mism = int(np.count_nonzero(zg != st.zeta))
        x = m.positions()
        hist.append(dict(step=i, gpu=g, oracle=h, mism=mism, disp=rel(x - prob.X, st.x - prob.X),
                         node=rowrel(x - prob.X, st.x - prob.X, 1e-3)))
        assert mism == 0, f"load step {i}: {mism} labels differ away from the threshold"
    return m, mesh, st, hist


@pytest.mark.parametrize("prec", ["fp64", "split"])
@pytest.mark.parametrize("energy,radius", [("stable_neo_hookean", 0.0), ("stable_neo_hookean", 0.08),
                                           ("stvk", 0.0)])
def test_quasi_static_pull_lockstep(prec, energy, radius):
    say(f"case quasi-static pull prec={prec} energy={energy} R_d={radius}")
    rtol = 1e-8 if prec == "fp64" else 1e-4
    prob = pulled_block(prec, energy, radius)
    m, mesh, st, hist = qs_lockstep(prob, 12, rtol)
    ng = [h["gpu"]["newton_iters"] for h in hist]
    no = [h["oracle"]["newton_iters"] for h in hist]
    last = hist[-1]
    say(f"  broken {int(st.zeta.sum())} newton gpu {ng} oracle {no} disp {last['disp']:.2e} node {last['node']:.2e}")
    assert st.zeta.sum() > 0
    bar, row = (1e-7, 1e-5) if prec == "fp64" else (1e-3, 1e-2)
    assert max(h["disp"] for h in hist) <= bar and last["node"] <= row
    if prec == "fp64":
        assert all(abs(a - b) <= 1 for a, b in zip(ng, no))
    assert all(h["gpu"]["force_residual"] <= rtol * h["gpu"]["force_initial"] for h in hist)
    assert not m.velocities().any()
    m.close()


def test_quasi_static_block_full_size():
    """Three load steps of the bench's 168,432-tet stone block (the size of the
    paper's blocks, Table 2), pulled 6 mm per end per load step so that edges
    break at the notch tip in the third: labels identical away from the
    threshold, displacements and Newton counts against the oracle."""
    say("case quasi-static stone block, full size (168,432 tets), 3 load steps")
    prob = meshgen.pulled_block("stone", pull=0.006)
    rtol = 1e-4
    m, mesh, st, hist = qs_lockstep(prob, 3, rtol)
    ng = [h["gpu"]["newton_iters"] for h in hist]
    no = [h["oracle"]["newton_iters"] for h in hist]
    last = hist[-1]
    say(f"  new broken {[h['gpu']['new_broken'] for h in hist]} newton gpu {ng} oracle {no} "
        f"disp {max(h['disp'] for h in hist):.2e} node {last['node']:.2e}")
    assert last["gpu"]["new_broken"] > 0
    assert max(h["disp"] for h in hist) <= 1e-3 and last["node"] <= 1e-2
    assert all(abs(a - b) <= 1 for a, b in zip(ng, no))
    assert all(h["gpu"]["force_residual"] <= rtol * h["gpu"]["force_initial"] for h in hist)
    m.close()


def test_quasi_static_line_search_acts():
    """Twist of the top face by 20 degrees per load step with Armijo constant
    0.9: the line search cuts steps on both sides and the equilibria agree."""
    say("case quasi-static twist, line search")
    prob = pulled_block("fp64", speed=0.0)
    X = prob.X
    top = X[prob.dir_nodes, 2] > X[:, 2].mean()
    c = X[prob.dir_nodes[top]].mean(axis=0)
    a = np.radians(20.0)
    R = np.array([[np.cos(a), -np.sin(a), 0], [np.sin(a), np.cos(a), 0], [0, 0, 1]])
    prob.dir_vel[:] = 0.0
    prob.dir_vel[top] = ((X[prob.dir_nodes[top]] - c) @ R.T + c) - X[prob.dir_nodes[top]]
    prob.params["damage_strain"] = 10.0
    m, mesh, st, hist = qs_lockstep(prob, 1, 1e-8, armijo=0.9, max_newton=200)
    h = hist[0]
    say(f"  halvings gpu {h['gpu']['line_search_halvings']} oracle {h['oracle']['halvings']} "
        f"newton {h['gpu']['newton_iters']} / {h['oracle']['newton_iters']} disp {h['disp']:.2e}")
    assert h["gpu"]["line_search_halvings"] > 0 and h["oracle"]["halvings"] > 0
    assert h["disp"] <= 1e-7
    m.close()


def test_failed_load_step_leaves_state_unchanged():
    say("case quasi-static failure path")
    prob = pulled_block("fp64")
    with gfem.mesh_from_problem(prob) as m:
        m.quasi_static_step(2, newton_rel_tol=1e-8)
        x0, z0 = m.positions(), m.edge_damage()
        r = m.quasi_static_step(1, newton_rel_tol=1e-8, max_newton=0, raise_on_error=False)
        assert r["status"] == gfem.GF_ENOTCONVERGED and r["steps_done"] == 0
        assert np.array_equal(m.positions(), x0) and np.array_equal(m.edge_damage(), z0)
        r = m.quasi_static_step(1, newton_rel_tol=1e-8)
        assert r["steps_done"] == 1
