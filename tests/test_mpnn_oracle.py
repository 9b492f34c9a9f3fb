"""Pins of the network oracle: its hand-written backward pass against central
finite differences of its own loss (FP64), the identity head against block
Jacobi, and the mean operator's transpose against a dense matrix."""
import numpy as np
import pytest

from oracle import gfem_oracle as O
from oracle import mpnn_oracle as N
from paper_2103_14870_amd import meshgen as mg


def small_system(seed=0):
    prob = mg.tiny_cube(2, h=0.1, jitter_frac=0.05, seed=seed, top_speed=0.4, damage_strain=0.05)
    mesh = O.setup(prob.X, prob.tets, prob.params)
    st = O.initial_state(mesh)
    rng = np.random.default_rng(seed + 1)
    st.x = prob.X + 0.002 * rng.normal(size=prob.X.shape)
    st.v = 0.1 * rng.normal(size=prob.X.shape)
    st.zeta = rng.random(mesh.edges.shape[0]) < 0.2
    zeta, _ = O.damage_update(mesh, st.x, st.zeta)
    sysm = O.build_system(mesh, st, prob.dir_nodes, prob.dir_vel, zeta, st.Ep)
    dv = np.linalg.solve(sysm.A.toarray(), sysm.b)
    Aii, b, d, free = N.system_data(mesh, st, sysm, dv, prob.dir_nodes)
    f = N.edge_features(prob.X, st.x, mesh.edges, zeta)
    a = N.node_inputs(prob.n_nodes, mesh.edges, f)
    P, PT = N.mean_operator(prob.n_nodes, mesh.edges, zeta)
    small_system.A = sysm.A
    return a, P, PT, Aii, b, d, free, mesh, zeta


def test_parameter_count():
    assert N.N_PARAMS == 64 * 8 + 64 + 3 * (64 * 128 + 64) + 6 * 64 + 6


def test_mean_operator_transpose_is_dense_transpose():
    a, P, PT, *_ , mesh, zeta = small_system(1)
    n = a.shape[0]
    Pd = np.stack([P(np.eye(n)[:, [i]])[:, 0] for i in range(n)], 1)
    rng = np.random.default_rng(2)
    g = rng.normal(size=(n, 4))
    np.testing.assert_allclose(PT(g), Pd.T @ g, rtol=1e-12, atol=1e-12)
    rows = Pd.sum(1)
    assert np.all((np.abs(rows - 1) < 1e-12) | (rows == 0))


def test_identity_head_is_block_jacobi():
    a, P, PT, Aii, b, d, free, *_ = small_system(3)
    w = N.init_weights(0, head_scale=0.0)
    B = N.precond_blocks(N.forward(w, a, P)["o"], Aii)
    np.testing.assert_allclose(B, np.linalg.inv(Aii), rtol=1e-12, atol=1e-14)


@pytest.mark.parametrize("kind", ["solution", "cg_step"])
def test_backward_matches_finite_differences(kind):
    a, P, PT, Aii, b, d, free, *_ = small_system(4)
    A = small_system.A
    w = N.init_weights(5, head_scale=0.05)
    lg = lambda ww: N.loss_and_grad(ww, a, P, PT, Aii, b, d, free, A=A, kind=kind)
    loss, g, _ = lg(w)
    rng = np.random.default_rng(6)
    idx = rng.choice(N.N_PARAMS, 40, replace=False)
    names = np.concatenate([[nm] * int(np.prod(s)) for nm, s in N.SHAPES])
    idx = np.unique(np.concatenate([idx, [np.nonzero(names == nm)[0][0] for nm, _ in N.SHAPES]]))
    h = 1e-6
    for i in idx:
        wp, wm = w.copy(), w.copy()
        wp[i] += h
        wm[i] -= h
        fd = (lg(wp)[0] - lg(wm)[0]) / (2 * h)
        assert g[i] == pytest.approx(fd, rel=1e-5, abs=1e-9 * max(1.0, abs(loss))), (i, names[i])


def test_loss_is_zero_for_the_exact_inverse_on_a_decoupled_system():
    # block-diagonal A: block Jacobi is the exact inverse, so the identity head has zero loss
    rng = np.random.default_rng(7)
    n = 5
    M = rng.normal(size=(n, 3, 3))
    Aii = M @ np.transpose(M, (0, 2, 1)) + 3 * np.eye(3)
    dv = rng.normal(size=(n, 3))
    b = np.einsum("nij,nj->ni", Aii, dv)
    edges = np.array([[0, 1], [1, 2], [2, 3], [3, 4]])
    zeta = np.zeros(4, bool)
    a = N.node_inputs(n, edges, np.zeros((4, 3)))
    P, PT = N.mean_operator(n, edges, zeta)
    loss, g, _ = N.loss_and_grad(N.init_weights(1), a, P, PT, Aii, b, dv, np.ones(n))
    assert loss < 1e-25


def test_cg_step_loss_is_the_one_step_energy_error():
    # log of |dv* - x1|_A^2 / |dv*|_A^2 for the optimal first step x1 = t B b
    a, P, PT, Aii, b, d, free, *_ = small_system(8)
    A = small_system.A
    w = N.init_weights(9, head_scale=0.05)
    loss, _, B = N.loss_and_grad(w, a, P, PT, Aii, b, d, free, A=A, kind="cg_step")
    Bf = np.where(free[:, None, None] > 0, B, np.linalg.inv(Aii))
    u = np.einsum("nij,nj->ni", Bf, b).ravel()
    x = d.ravel()
    t = (b.ravel() @ u) / (u @ (A @ u))
    e = x - t * u
    ratio = (e @ (A @ e)) / (x @ (A @ x))
    # one-step error energy = 1 - exp(-loss)... loss = log(q) - 2 log(s) + log(b.x) = -log(1 - ratio)
    assert loss == pytest.approx(-np.log(1 - ratio), rel=1e-10)
    assert 0 <= ratio < 1
