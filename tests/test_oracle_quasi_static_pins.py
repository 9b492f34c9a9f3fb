"""Pins of the oracle's quasi-static load step (Eq. 36, Newton with a
backtracking line search on the total energy, Sec. 4.3 / Sec. 5.1):
  * the equilibrium it reaches is the minimiser of the total energy that
    scipy's quasi-Newton optimiser finds independently (same prescribed
    nodes, same chi), for a small and a large load increment, and with an
    Armijo constant that makes the line search cut the steps;
  * for a tiny increment it is the textbook linear-elastic solution
    u_f = -K_ff^-1 K_fc u_c with the rest stiffness (pinned to the textbook
    tet stiffness elsewhere);
  * the energy decreases at every Newton iterate and the out-of-balance force
    reaches the relative tolerance; prescribed nodes sit at X + dt v and the
    velocities are zero;
  * a fully detached fragment stays where it is and keeps the solve finite.
"""
import numpy as np
import pytest
import scipy.optimize as so

from oracle import gfem_oracle as O
from paper_2103_14870_amd import meshgen as mg

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def block(top_disp, energy="stable_neo_hookean", n=2, seed=4):
    prob = mg.cube_block(n, n, n, h=0.1, jitter_frac=0.08, seed=seed, top_speed=top_disp, dt=1.0,
                         damage_strain=10.0, cg_rel_tol=1e-12, energy=energy)
    mesh = O.setup(prob.X, prob.tets, prob.params)
    return prob, mesh


def minimise(mesh, prob, x_start, chi):
    """Energy minimum over the free nodes (prescribed nodes as in x_start),
    by BFGS with the restoring forces as the negative gradient."""
    free = np.setdiff1d(np.arange(mesh.X.shape[0]), prob.dir_nodes)

    def fun(z):
        x = x_start.copy()
        x[free] = z.reshape(-1, 3)
        el = O.element(mesh, x)
        f = O.scatter_forces(x.shape[0], mesh.tets, O.element_forces(mesh, el, chi))
        return O.energy_fixed_chi(mesh, x, chi), -f[free].ravel()

    r = so.minimize(fun, x_start[free].ravel(), jac=True, method="BFGS", options=dict(gtol=1e-10, maxiter=20000))
    x = x_start.copy()
    x[free] = r.x.reshape(-1, 3)
    return x


@pytest.mark.parametrize("energy", ["stable_neo_hookean", "stvk"])
@pytest.mark.parametrize("top,armijo", [(0.002, 1e-4), (0.04, 1e-4), (0.04, 0.9)])
def test_equilibrium_is_the_energy_minimiser(energy, top, armijo):
    """armijo = 0.9 demands more decrease than a full Newton step gives on a
    nearly quadratic energy, so the backtracking branch has to act."""
    prob, mesh = block(top, energy)
    st = O.initial_state(mesh)
    st1, h = O.quasi_static_step(mesh, st, prob.dir_nodes, prob.dir_vel, newton_rtol=1e-10, armijo=armijo,
                                 max_newton=200)
    assert h["converged"], h
    x_start = mesh.X.copy()
    x_start[prob.dir_nodes] += prob.params["dt"] * prob.dir_vel
    chi = np.ones(mesh.tets.shape[0])
    xm = minimise(mesh, prob, x_start, chi)
    u = st1.x - mesh.X
    assert np.linalg.norm(st1.x - xm) <= 1e-6 * np.linalg.norm(u)
    if armijo > 0.5:
        assert h["halvings"] > 0, "the demanding Armijo constant should cut the Newton step"
    else:
        assert h["halvings"] == 0
    e = h["energy"]
    assert all(b <= a + 1e-14 * abs(a) for a, b in zip(e, e[1:]))
    assert h["force"][-1] <= 1e-10 * h["force"][0]
    np.testing.assert_array_equal(st1.x[prob.dir_nodes], x_start[prob.dir_nodes])
    assert not st1.v.any()


def test_tiny_increment_is_linear_elastic():
    prob, mesh = block(1e-8, n=3)
    st = O.initial_state(mesh)
    st1, h = O.quasi_static_step(mesh, st, prob.dir_nodes, prob.dir_vel, newton_rtol=1e-7)
    assert h["converged"]
    n = mesh.X.shape[0]
    el = O.element(mesh, mesh.X)
    K = O.assemble_stiffness(n, mesh.tets, O.element_stiffness(mesh, el, np.ones(mesh.tets.shape[0]))).toarray()
    c = (3 * prob.dir_nodes[:, None] + np.arange(3)).ravel()
    f = np.setdiff1d(np.arange(3 * n), c)
    uc = (prob.params["dt"] * prob.dir_vel).ravel()
    uf = -np.linalg.solve(K[np.ix_(f, f)], K[np.ix_(f, c)] @ uc)
    u = (st1.x - mesh.X).ravel()
    assert np.linalg.norm(u[f] - uf) <= 1e-5 * np.linalg.norm(uf)


def test_detached_fragment_stays_and_solve_is_finite():
    prob, mesh = block(0.004, n=3)
    st = O.initial_state(mesh)
    # break every edge of the tets around one interior node of the middle layer
    node = 13
    on = np.any(mesh.edges == node, axis=1)
    st.zeta |= on
    st1, h = O.quasi_static_step(mesh, st, prob.dir_nodes, prob.dir_vel, newton_rtol=1e-10)
    assert h["converged"] and np.isfinite(st1.x).all()
    np.testing.assert_allclose(st1.x[node], mesh.X[node], rtol=0, atol=1e-14)
    assert np.linalg.norm(st1.x - mesh.X) > 1e-3
