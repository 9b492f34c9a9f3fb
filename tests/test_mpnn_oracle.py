"""Pins of the network oracle: the factor G against a direct dense
construction, its log-determinant against a dense one, the zero network
against block-Jacobi, the Kaporin loss at the exact inverse, the hand-written
backward pass against central finite differences (FP64), and the mean
operator's transpose against a dense matrix."""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import gfem_oracle as O
from oracle import mpnn_oracle as N
from paper_2103_14870_amd import meshgen as mg


def small_system(seed=0, n=2):
    prob = mg.tiny_cube(n, h=0.1, jitter_frac=0.05, seed=seed, top_speed=0.4, damage_strain=0.05)
    mesh = O.setup(prob.X, prob.tets, prob.params)
    st = O.initial_state(mesh)
    rng = np.random.default_rng(seed + 1)
    st.x = prob.X + 0.002 * rng.normal(size=prob.X.shape)
    st.v = 0.1 * rng.normal(size=prob.X.shape)
    st.zeta = rng.random(mesh.edges.shape[0]) < 0.2
    zeta, _ = O.damage_update(mesh, st.x, st.zeta)
    sysm = O.build_system(mesh, st, prob.dir_nodes, prob.dir_vel, zeta, st.Cp)
    a, P, PT, fac = N.system_inputs(mesh, st.x, zeta, sysm.A, prob.dir_nodes)
    return a, P, PT, fac, sysm.A.tocsr(), sysm.b, mesh


def test_parameter_count():
    assert N.N_PARAMS == 64 * 8 + 64 + 3 * (64 * 128 + 64) + 24 * 64 + 24 + 9 * 3 + 9


def test_mean_operator_transpose_is_dense_transpose():
    a, P, PT, fac, *_ = small_system(1)
    n = a.shape[0]
    Pd = np.stack([P(np.eye(n)[:, [i]])[:, 0] for i in range(n)], 1)
    rng = np.random.default_rng(2)
    g = rng.normal(size=(n, 4))
    np.testing.assert_allclose(PT(g), Pd.T @ g, rtol=1e-12, atol=1e-12)
    rows = Pd.sum(1)
    assert np.all((np.abs(rows - 1) < 1e-12) | (rows == 0))


def test_zero_network_is_block_jacobi():
    a, P, PT, fac, A, b, _ = small_system(3)
    w = N.init_weights(0, head_scale=0.0)
    Gd, Gl, _ = N.factor_blocks(N.forward(w, a, P)["o"], w, fac)
    r = np.random.default_rng(4).normal(size=(fac.n, 3))
    Dinv = np.linalg.inv(N.diagonal_blocks(A))
    np.testing.assert_allclose(N.apply(fac, Gd, Gl, r), np.einsum("nij,nj->ni", Dinv, r), rtol=1e-11, atol=1e-13)


def test_constant_damping_matches_dense_construction():
    # W_ij = w I, L = I: G = blockdiag(C) (I - w E_L blockdiag(D^-1)), E_L the strictly block-lower part of A
    a, P, PT, fac, A, b, _ = small_system(5)
    wgt = N.init_weights(0, head_scale=0.0)
    om = 0.7
    wgt[N.offset("be"):N.offset("be") + 9] = 2.0 * np.arctanh(om / 2.0) * np.eye(3).ravel()
    Gd, Gl, _ = N.factor_blocks(N.forward(wgt, a, P)["o"], wgt, fac)
    G = N.G_matrix(fac, Gd, Gl).toarray()
    Ad = A.toarray()
    n3 = Ad.shape[0]
    blk = np.arange(n3) // 3
    EL = np.where(blk[:, None] > blk[None, :], Ad, 0.0)
    Dd = np.where(blk[:, None] == blk[None, :], Ad, 0.0)
    Lc = np.linalg.cholesky(Dd)
    Gref = np.linalg.inv(Lc) @ (np.eye(n3) - om * EL @ np.linalg.inv(Dd))
    np.testing.assert_allclose(G, Gref, rtol=1e-10, atol=1e-12)
    assert np.allclose(np.triu(G, 1)[blk[:, None] != blk[None, :]], 0.0)


def test_factor_is_lower_triangular_and_B_is_spd():
    a, P, PT, fac, A, b, _ = small_system(6)
    w = N.init_weights(7, head_scale=0.1)
    Gd, Gl, _ = N.factor_blocks(N.forward(w, a, P)["o"], w, fac)
    G = N.G_matrix(fac, Gd, Gl).toarray()
    blk = np.arange(G.shape[0]) // 3
    assert np.all(G[blk[:, None] < blk[None, :]] == 0.0)
    B = G.T @ G
    assert np.linalg.eigvalsh(B).min() > 0
    r = np.random.default_rng(8).normal(size=(fac.n, 3))
    np.testing.assert_allclose(N.apply(fac, Gd, Gl, r).ravel(), B @ r.ravel(), rtol=1e-10, atol=1e-12)
    # log det G from the diagonal blocks equals the dense log-determinant
    sign, ld = np.linalg.slogdet(G)
    assert ld == pytest.approx(np.sum(np.log(np.abs(np.linalg.det(Gd)))), rel=1e-10)


def test_kaporin_loss_at_the_exact_inverse():
    # block-diagonal A: G = blockdiag(C) is an exact inverse factor, G A G^T = I,
    # so K = 1 and loss = log K / N + log det A / N = log det A / N for any probe of +-1 entries
    rng = np.random.default_rng(9)
    n = 5
    Mx = rng.normal(size=(n, 3, 3))
    D = Mx @ np.transpose(Mx, (0, 2, 1)) + 3 * np.eye(3)
    A = sp.block_diag(list(D), format="csr")
    edges = np.array([[0, 1], [1, 2], [2, 3], [3, 4]])
    f = np.zeros((4, 3))
    a = N.node_inputs(n, edges, f)
    P, PT = N.mean_operator(n, edges, np.zeros(4, bool))
    fac = N.make_factor(A, edges, f, np.ones(n))
    v = rng.choice([-1.0, 1.0], size=(n, 3))
    w = N.init_weights(1, head_scale=0.0)
    w[N.offset("be"):N.offset("be") + 9] = rng.normal(size=9)  # W is irrelevant: A_ij = 0
    loss, _, _ = N.loss_and_grad(w, a, P, PT, fac, A, v)
    assert loss == pytest.approx(np.linalg.slogdet(A.toarray())[1] / (3 * n), rel=1e-12)


def test_bounded_maps():
    x = np.linspace(-30, 30, 601)
    assert np.all(np.abs(N.bound(x)) < 2.0) and N.bound(np.zeros(1))[0] == 0.0
    h = 1e-6
    np.testing.assert_allclose(N.bound_slope(x), (N.bound(x + h) - N.bound(x - h)) / (2 * h), atol=1e-8)
    # huge head outputs still give a finite, well-defined factor
    o = np.full((4, 6), 1e6)
    L = N.lower_factor(o)
    assert np.all(np.isfinite(L)) and np.allclose(np.diagonal(L, axis1=1, axis2=2), np.exp(2.0))


def test_backward_matches_finite_differences():
    a, P, PT, fac, A, b, _ = small_system(4)
    w = N.init_weights(5, head_scale=0.5)
    v = np.random.default_rng(6).choice([-1.0, 1.0], size=(fac.n, 3))
    lg = lambda ww: N.loss_and_grad(ww, a, P, PT, fac, A, v)
    loss, g, _ = lg(w)
    rng = np.random.default_rng(6)
    idx = rng.choice(N.N_PARAMS, 40, replace=False)
    names = np.concatenate([[nm] * int(np.prod(s)) for nm, s in N.SHAPES])
    idx = np.unique(np.concatenate([idx, [np.nonzero(names == nm)[0][0] for nm, _ in N.SHAPES],
                                    N.offset("Wh") + np.arange(0, 24 * 64, 64) + 3]))
    h = 1e-6
    for i in idx:
        wp, wm = w.copy(), w.copy()
        wp[i] += h
        wm[i] -= h
        fd = (lg(wp)[0] - lg(wm)[0]) / (2 * h)
        assert g[i] == pytest.approx(fd, rel=1e-5, abs=1e-9 * max(1.0, abs(loss))), (i, names[i])


def test_damped_factor_reduces_cg_iterations():
    # the family's constant member W = 0.75 I already needs far fewer PCG
    # iterations than block-Jacobi on a three-point-bending beam
    prob = mg.notched_beam(16, 4, 4, h=0.01, notch_cells=1)
    mesh = O.setup(prob.X, prob.tets, prob.params)
    st = O.initial_state(mesh)
    O.break_pairs(mesh, st, prob.broken_pairs)
    zeta, _ = O.damage_update(mesh, st.x, st.zeta)
    sysm = O.build_system(mesh, st, prob.dir_nodes, prob.dir_vel, zeta, st.Cp)
    a, P, PT, fac = N.system_inputs(mesh, st.x, zeta, sysm.A, prob.dir_nodes)
    w = N.init_weights(0)
    w[N.offset("be"):N.offset("be") + 9] = 2.0 * np.arctanh(0.75 / 2.0) * np.eye(3).ravel()
    Gd, Gl, _ = N.factor_blocks(N.forward(w, a, P)["o"], w, fac)
    G = N.G_matrix(fac, Gd, Gl)
    B = (G.T @ G).tocsr()
    _, it_f, _, ok_f = O.pcg(sysm.A, sysm.b, B, 1e-6, 5000)
    _, it_j, _, ok_j = O.pcg(sysm.A, sysm.b, O.block_jacobi(sysm.A), 1e-6, 5000)
    assert ok_f and ok_j
    assert it_f < 0.7 * it_j, (it_f, it_j)


def test_power_probe_is_the_normalised_matrix_power():
    # k power steps equal the dense X^k v, X = G A G^T, scaled to |v|^2 = N
    a, P, PT, fac, A, b, _ = small_system(7)
    w = N.init_weights(8, head_scale=0.2)
    Gd, Gl, _ = N.factor_blocks(N.forward(w, a, P)["o"], w, fac)
    G = N.G_matrix(fac, Gd, Gl).toarray()
    X = G @ A.toarray() @ G.T
    v = np.random.default_rng(9).choice([-1.0, 1.0], size=(fac.n, 3))
    for k in (0, 1, 3):
        ref = np.linalg.matrix_power(X, k) @ v.ravel()
        ref *= np.sqrt(3 * fac.n / (ref @ ref))
        np.testing.assert_allclose(N.power_probe(fac, Gd, Gl, A, v, k).ravel(), ref, rtol=1e-10, atol=1e-12)


def test_power_loss_rises_to_the_largest_eigenvalue():
    # loss + (2/N) log det G = log of the Rayleigh quotient of X^k v: it never
    # decreases with k, never exceeds log lambda_max(X), and reaches it
    a, P, PT, fac, A, b, _ = small_system(8)
    w = N.init_weights(10, head_scale=0.2)
    Gd, Gl, _ = N.factor_blocks(N.forward(w, a, P)["o"], w, fac)
    G = N.G_matrix(fac, Gd, Gl).toarray()
    lmax = np.linalg.eigvalsh(G @ A.toarray() @ G.T).max()
    Nn = 3 * fac.n
    ld = np.sum(np.log(np.abs(np.linalg.det(Gd))))
    v = np.random.default_rng(11).choice([-1.0, 1.0], size=(fac.n, 3))
    rq = []
    for k in (0, 1, 2, 4, 8, 16, 64, 400):
        loss, _, _ = N.loss_and_grad_power(w, a, P, PT, fac, A, v, k)
        rq.append(loss + 2.0 / Nn * ld)
    assert np.all(np.diff(rq) >= -1e-12)
    assert rq[-1] <= np.log(lmax) + 1e-12
    assert rq[-1] == pytest.approx(np.log(lmax), abs=1e-6)
    # k = 0 is the plain Kaporin probe loss
    assert N.loss_and_grad_power(w, a, P, PT, fac, A, v, 0)[0] == N.loss_and_grad(w, a, P, PT, fac, A, v)[0]


def test_row_normalisation_gives_unit_diagonal_blocks():
    # after normalisation the diagonal blocks of the dense G A G^T are I, and G
    # keeps its block lower triangular shape with lower-triangular G_ii
    a, P, PT, fac, A, b, _ = small_system(12)
    w = N.init_weights(13, head_scale=0.3)
    Gd, Gl, _ = N.factor_blocks(N.forward(w, a, P)["o"], w, fac)
    Gd2, Gl2 = N.normalise_rows(fac, Gd, Gl, A)
    G = N.G_matrix(fac, Gd2, Gl2).toarray()
    X = G @ A.toarray() @ G.T
    blk = np.arange(X.shape[0]) // 3
    np.testing.assert_allclose(np.where(blk[:, None] == blk[None, :], X, 0.0), np.eye(X.shape[0]), atol=1e-10)
    assert np.all(G[blk[:, None] < blk[None, :]] == 0.0)
    assert np.all(np.triu(Gd2, 1) == 0.0)


def test_row_normalisation_ignores_a_lower_triangular_row_scaling():
    # (L G)_i normalised equals G_i normalised for any lower-triangular L_i with
    # positive diagonal: chol(L X L^T) = L chol(X)
    a, P, PT, fac, A, b, _ = small_system(14)
    w = N.init_weights(15, head_scale=0.3)
    Gd, Gl, _ = N.factor_blocks(N.forward(w, a, P)["o"], w, fac)
    rng = np.random.default_rng(16)
    L = np.tril(rng.normal(size=(fac.n, 3, 3)), -1) + np.eye(3) * rng.uniform(0.3, 3.0, size=(fac.n, 1, 3))
    ref = N.normalise_rows(fac, Gd, Gl, A)
    got = N.normalise_rows(fac, L @ Gd, L[fac.rows] @ Gl, A)
    np.testing.assert_allclose(got[0], ref[0], rtol=1e-9, atol=1e-12)
    np.testing.assert_allclose(got[1], ref[1], rtol=1e-9, atol=1e-12)


def test_row_normalisation_leaves_block_jacobi_unchanged():
    a, P, PT, fac, A, b, _ = small_system(17)
    w = N.init_weights(0, head_scale=0.0)
    Gd, Gl, _ = N.factor_blocks(N.forward(w, a, P)["o"], w, fac)
    Gd2, Gl2 = N.normalise_rows(fac, Gd, Gl, A)
    np.testing.assert_allclose(Gd2, Gd, rtol=1e-12, atol=1e-14)
    assert np.all(Gl2 == 0.0)
