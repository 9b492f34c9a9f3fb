"""Pins of the oracle's Saint-Venant Kirchhoff energy (Sec. 5.2, Eq. 37) in
edge form, against the textbook deformation-gradient form
Psi = mu |E|^2 + lam/2 tr(E)^2, E = (F^T F - I)/2, written out here:
  * the edge-length energy equals it on random tets, inverted ones included;
  * forces equal -V P Dm^-T with P = F S, S = lam tr(E) I + 2 mu E, and central
    finite differences;
  * the rest stiffness is the textbook linear-elastic tet stiffness with the
    plain Lame constants (no reparametrisation for this energy);
  * the unclamped tangent equals the finite-difference Hessian; the clamped
    one is PSD, and equal to it when every edge is stretched;
  * the energy depends on C only: reflecting a node through the opposite
    face (an inverted tet with the same six edge lengths) keeps it;
  * chi's edge stresses are q^T S q of the same S.
"""
import numpy as np
import pytest

from oracle import gfem_oracle as O

from test_oracle_pins import lame, random_tets

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")

PARAMS = dict(youngs=1e5, poisson=0.3, density=1000.0, damage_strain=10.0, dt=1e-3,
              cg_rel_tol=1e-10, cg_max_iter=5000, energy="stvk")


def mesh_of(X, tets, **kw):
    return O.setup(X, tets, dict(PARAMS, **kw))


def stvk_psi_F(F, mu, lam):
    E = 0.5 * (F.T @ F - np.eye(3))
    return mu * np.sum(E * E) + 0.5 * lam * np.trace(E) ** 2


def stvk_S(F, mu, lam):
    E = 0.5 * (F.T @ F - np.eye(3))
    return lam * np.trace(E) * np.eye(3) + 2 * mu * E


def defgrads(mesh, X, x):
    out = []
    for idx in mesh.tets:
        Dm = (X[idx[1:]] - X[idx[0]]).T
        Ds = (x[idx[1:]] - x[idx[0]]).T
        out.append((Ds @ np.linalg.inv(Dm), Dm))
    return out


def inverted_copy(X, x, tets, every=3):
    """Reflect every `every`-th deformed tet through the plane of three of its
    nodes (det F < 0)."""
    x = x.copy()
    for t in range(0, tets.shape[0], every):
        a, b, c, d = tets[t]
        n = np.cross(x[b] - x[a], x[c] - x[a])
        n /= np.linalg.norm(n)
        x[d] -= 2.0 * np.dot(x[d] - x[a], n) * n
    return x


def test_energy_equals_F_form_including_inverted():
    X, x, tets = random_tets(150, seed=31)
    x = inverted_copy(X, x, tets)
    mesh = mesh_of(X, tets)
    mu, lam = lame(1e5, 0.3)
    assert mesh.mu == pytest.approx(mu) and mesh.lam == pytest.approx(lam)
    el = O.element(mesh, x)
    Fs = defgrads(mesh, X, x)
    assert sum(np.linalg.det(F) < 0 for F, _ in Fs) >= 40
    for t, (F, _) in enumerate(Fs):
        assert el.psi[t] == pytest.approx(stvk_psi_F(F, mu, lam), rel=1e-11, abs=1e-9 * mu)


def test_forces_equal_first_PK_and_finite_differences():
    X, x, tets = random_tets(40, seed=32)
    x = inverted_copy(X, x, tets, every=4)
    mesh = mesh_of(X, tets)
    mu, lam = mesh.mu, mesh.lam
    el = O.element(mesh, x)
    f = O.element_forces(mesh, el, np.ones(40))
    for t, (F, Dm) in enumerate(defgrads(mesh, X, x)):
        H = -mesh.V[t] * (F @ stvk_S(F, mu, lam)) @ np.linalg.inv(Dm).T
        fref = np.vstack([-H.sum(axis=1), H.T])
        np.testing.assert_allclose(f[t], fref, rtol=1e-9, atol=1e-9 * np.abs(fref).max())
    chi = np.ones(40)
    h = 1e-6
    for t in (0, 5, 17):
        for a in range(4):
            for d in range(3):
                node = mesh.tets[t, a]
                xp, xm = x.copy(), x.copy()
                xp[node, d] += h
                xm[node, d] -= h
                dE = (O.total_energy(mesh, xp, chi) - O.total_energy(mesh, xm, chi)) / (2 * h)
                assert -dE == pytest.approx(f[t, a, d], rel=1e-5, abs=1e-6 * np.abs(f[t]).max())


def test_rest_state_stress_free_and_rest_stiffness_is_linear_elastic():
    X, _, tets = random_tets(10, seed=33)
    E, nu = 2.5e4, 0.35
    mesh = mesh_of(X, tets, youngs=E, poisson=nu)
    el = O.element(mesh, X)
    assert np.abs(O.element_forces(mesh, el, np.ones(10))).max() < 1e-9 * E
    K = O.element_stiffness(mesh, el, np.ones(10))
    c = E / ((1 + nu) * (1 - 2 * nu))
    D = c * np.array([[1 - nu, nu, nu, 0, 0, 0], [nu, 1 - nu, nu, 0, 0, 0], [nu, nu, 1 - nu, 0, 0, 0],
                      [0, 0, 0, (1 - 2 * nu) / 2, 0, 0], [0, 0, 0, 0, (1 - 2 * nu) / 2, 0],
                      [0, 0, 0, 0, 0, (1 - 2 * nu) / 2]])
    for t in range(10):
        idx = mesh.tets[t]
        Dm = (X[idx[1:]] - X[idx[0]]).T
        grads = np.linalg.inv(Dm)
        grads = np.vstack([-grads.sum(axis=0), grads])
        B = np.zeros((6, 12))
        for a in range(4):
            bx, by, bz = grads[a]
            B[:, 3 * a:3 * a + 3] = [[bx, 0, 0], [0, by, 0], [0, 0, bz], [by, bx, 0], [0, bz, by], [bz, 0, bx]]
        Kref = mesh.V[t] * B.T @ D @ B
        np.testing.assert_allclose(K[t], Kref, rtol=1e-9, atol=1e-9 * np.abs(Kref).max())


def fd_stiffness(X4, x4):
    """Finite-difference tangent of one positively oriented tet (nodes in its
    local order)."""
    m1 = mesh_of(X4, np.arange(4)[None])
    assert np.array_equal(m1.tets[0], np.arange(4))
    h = 1e-6
    Kfd = np.zeros((12, 12))
    for j in range(12):
        xp, xm = x4.copy(), x4.copy()
        xp[j // 3, j % 3] += h
        xm[j // 3, j % 3] -= h
        fp = O.element_forces(m1, O.element(m1, xp), np.ones(1))[0].ravel()
        fm = O.element_forces(m1, O.element(m1, xm), np.ones(1))[0].ravel()
        Kfd[:, j] = -(fp - fm) / (2 * h)
    return Kfd


def test_tangent_unclamped_is_fd_hessian_clamped_is_psd():
    X, x, tets = random_tets(60, seed=34, deform=0.3)
    x = inverted_copy(X, x, tets, every=5)
    mesh = mesh_of(X, tets)
    el = O.element(mesh, x)
    Ku = O.element_stiffness(mesh, el, np.ones(60), clamp=False)
    Kc = O.element_stiffness(mesh, el, np.ones(60))
    for t in range(60):
        w = np.linalg.eigvalsh(0.5 * (Kc[t] + Kc[t].T))
        assert w.min() >= -1e-9 * w.max()
    for t in (0, 3, 10, 21):
        Kfd = fd_stiffness(X[mesh.tets[t]], x[mesh.tets[t]])
        np.testing.assert_allclose(Ku[t], Kfd, rtol=1e-5, atol=1e-6 * np.abs(Kfd).max())
    # every edge stretched: the clamp of g_k is inactive and the PSD tangent is exact
    rng = np.random.default_rng(35)
    X, _, tets = random_tets(50, seed=35)
    cen = X.reshape(-1, 4, 3).mean(axis=1).repeat(4, axis=0)
    x = cen + 1.05 * (X - cen) + 0.001 * rng.normal(size=X.shape)
    mesh = mesh_of(X, tets)
    el = O.element(mesh, x)
    ids = np.nonzero(np.all(el.g >= 0, axis=1))[0][:4]
    assert ids.size >= 2
    Kc = O.element_stiffness(mesh, el, np.ones(50))
    for t in ids:
        Kfd = fd_stiffness(X[mesh.tets[t]], x[mesh.tets[t]])
        np.testing.assert_allclose(Kc[t], Kfd, rtol=1e-5, atol=1e-6 * np.abs(Kfd).max())


def test_reflected_tet_has_the_energy_of_its_mirror_image():
    X, x, tets = random_tets(20, seed=36)
    mesh = mesh_of(X, tets)
    xr = inverted_copy(X, x, tets, every=1)
    e0 = O.element(mesh, x).psi
    e1 = O.element(mesh, xr).psi
    for t, ((F0, _), (F1, _)) in enumerate(zip(defgrads(mesh, X, x), defgrads(mesh, X, xr))):
        assert np.linalg.det(F1) < 0
        assert e1[t] == pytest.approx(stvk_psi_F(F1, mesh.mu, mesh.lam), rel=1e-11)
    # reflecting a node through the opposite face keeps all six edge lengths,
    # hence C and the energy: the edge form is defined on inverted tets
    np.testing.assert_allclose(e1, e0, rtol=1e-11)


def test_chi_edge_stresses_are_q_S_q():
    X, x, tets = random_tets(30, seed=37)
    mesh = mesh_of(X, tets)
    sig, small, _ = O.scaled_edge_stress(mesh, x)
    assert not small.any()
    for t, (F, _) in enumerate(defgrads(mesh, X, x)):
        S = stvk_S(F, mesh.mu, mesh.lam)
        idx = mesh.tets[t]
        for k, (a, b) in enumerate(O.LOCAL_EDGES):
            q = X[idx[b]] - X[idx[a]]
            q /= np.linalg.norm(q)
            assert sig[t, k] == pytest.approx(q @ S @ q, rel=1e-10, abs=1e-8 * mesh.mu)
