"""Pins of the oracle on nearly flat and inverted tets (|J| < J_MIN).

The edge-length form of the volume term divides by J (the edge Gram matrix
is singular on a flat tet), so below J_MIN = 0.05 the oracle evaluates the
volume term of Eq. 35 in cofactor form: the same energy, another formula.
Pinned here against the textbook deformation-gradient forms:
  * forces equal -V P(F) Dm^-T and central differences of the energy, on tets
    with J in (-0.05, 0.05), including J = +-1e-9;
  * the force is continuous through J = 0 and across J = J_MIN (same
    function on both sides of the switch);
  * a flattened tet of either orientation carries the finite restoring force
    of the energy, not the force of some other state;
  * the clamped tangent is PSD; the unclamped one equals the finite-difference
    Hessian;
  * chi's stress ratios are continuous across J_MIN and finite at J = 0.
"""
import numpy as np
import pytest

from oracle import gfem_oracle as O

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")

PARAMS = dict(youngs=5e4, poisson=0.45, density=1000.0, damage_strain=10.0, dt=1e-2,
              cg_rel_tol=1e-10, cg_max_iter=5000)


def tet_with_J(seed, J, scale=0.1):
    """A random rest tet (positively oriented) and a deformed copy with
    det F = J (F = Q1 diag(s1, s2, J/(s1 s2)) Q2)."""
    rng = np.random.default_rng(seed)
    base = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]], float)
    while True:
        X = (base + 0.2 * rng.normal(size=(4, 3))) * scale
        if np.linalg.det((X[1:] - X[0]).T) > 0.1 * scale ** 3:
            break
    Q1, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    Q2, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    Q1 *= np.sign(np.linalg.det(Q1))
    Q2 *= np.sign(np.linalg.det(Q2))
    s1, s2 = rng.uniform(0.7, 1.4, size=2)
    F = Q1 @ np.diag([s1, s2, J / (s1 * s2)]) @ Q2
    x = X @ F.T + rng.normal(size=3) * scale
    return X, x, F


def snh_P(F, mu, lam, alpha):
    IC = np.sum(F * F)
    J = np.linalg.det(F)
    cof = np.array([np.cross(F[:, 1], F[:, 2]), np.cross(F[:, 2], F[:, 0]), np.cross(F[:, 0], F[:, 1])]).T
    return mu * (1 - 1 / (IC + 1)) * F + lam * (J - alpha) * cof


def textbook_forces(X, F, mesh):
    Dm = (X[1:] - X[0]).T
    H = -mesh.V[0] * snh_P(F, mesh.mu, mesh.lam, mesh.alpha) @ np.linalg.inv(Dm).T
    return np.vstack([-H.sum(axis=1), H.T])



@pytest.mark.parametrize("J", [0.049, 0.02, 1e-3, 1e-9, 0.0, -1e-9, -1e-3, -0.03, -0.049])
@pytest.mark.parametrize("seed", [1, 2])
def test_small_J_forces_are_the_textbook_forces(J, seed):
    X, x, F = tet_with_J(seed, J)
    mesh = O.setup(X, np.arange(4)[None], PARAMS)
    assert np.array_equal(mesh.tets[0], [0, 1, 2, 3])
    el = O.element(mesh, x)
    assert el.small[0]
    assert el.J[0] == pytest.approx(J, abs=1e-12)
    f = O.element_forces(mesh, el, np.ones(1))[0]
    fref = textbook_forces(X, F, mesh)
    np.testing.assert_allclose(f, fref, rtol=1e-9, atol=1e-9 * np.abs(fref).max())
    assert np.all(np.isfinite(O.element_stiffness(mesh, el, np.ones(1))))


@pytest.mark.parametrize("J", [0.03, 1e-4, -1e-4, -0.03])
def test_small_J_forces_are_energy_gradients(J):
    X, x, _ = tet_with_J(5, J)
    mesh = O.setup(X, np.arange(4)[None], PARAMS)
    el = O.element(mesh, x)
    f = O.element_forces(mesh, el, np.ones(1))[0]
    h = 1e-7 * 0.1
    for a in range(4):
        for d in range(3):
            xp, xm = x.copy(), x.copy()
            xp[a, d] += h
            xm[a, d] -= h
            dE = (O.total_energy(mesh, xp, np.ones(1)) - O.total_energy(mesh, xm, np.ones(1))) / (2 * h)
            assert -dE == pytest.approx(f[a, d], rel=1e-5, abs=1e-6 * np.abs(f).max())


def test_force_continuous_through_flat_and_across_the_switch():
    for seed in (3, 4):
        fs = {}
        for J in (1e-9, -1e-9, O.J_MIN * (1 + 1e-9), O.J_MIN * (1 - 1e-9)):
            X, x, _ = tet_with_J(seed, J)
            mesh = O.setup(X, np.arange(4)[None], PARAMS)
            el = O.element(mesh, x)
            fs[J] = O.element_forces(mesh, el, np.ones(1))[0]
        a, b = fs[1e-9], fs[-1e-9]
        assert np.abs(a - b).max() <= 1e-6 * np.abs(a).max()
        c, d = fs[O.J_MIN * (1 + 1e-9)], fs[O.J_MIN * (1 - 1e-9)]
        assert np.abs(c - d).max() <= 1e-6 * np.abs(c).max()


def test_flattened_tet_of_either_orientation_has_the_finite_energy_force():
    """A tet flattened onto a plane (det Ds = +-1e-9 relative) feels the
    restoring force -V lambda (J - alpha) dJ/dx (plus the I_C term), of the
    size lambda V / h, on both sides of the plane.  (An evaluation at some
    other reference state, e.g. J = -1 at the rest Gram matrix, gives forces
    orders of magnitude larger and fails this.)"""
    for sign in (1.0, -1.0):
        X, x, F = tet_with_J(9, sign * 1e-9)
        mesh = O.setup(X, np.arange(4)[None], PARAMS)
        el = O.element(mesh, x)
        f = O.element_forces(mesh, el, np.ones(1))[0]
        fref = textbook_forces(X, F, mesh)
        np.testing.assert_allclose(f, fref, rtol=1e-9, atol=1e-9 * np.abs(fref).max())
        scale = mesh.lam * mesh.V[0] / 0.1
        assert np.abs(f).max() < 20 * scale
        assert abs(el.psi[0] - (0.5 * mesh.lam * mesh.alpha ** 2 + 0.5 * mesh.mu * (el.IC[0] - 3)
                                - 0.5 * mesh.mu * np.log(el.IC[0] + 1))) < 1e-6 * mesh.lam


@pytest.mark.parametrize("J", [0.04, 1e-3, -1e-3, -0.04])
def test_small_J_tangent_psd_and_unclamped_equals_fd_hessian(J):
    X, x, _ = tet_with_J(11, J)
    mesh = O.setup(X, np.arange(4)[None], PARAMS)
    el = O.element(mesh, x)
    K = O.element_stiffness(mesh, el, np.ones(1))[0]
    w = np.linalg.eigvalsh(0.5 * (K + K.T))
    assert w.min() >= -1e-9 * w.max()
    Ku = O.element_stiffness(mesh, el, np.ones(1), clamp=False)[0]
    h = 1e-7 * 0.1
    Kfd = np.zeros((12, 12))
    for j in range(12):
        xp, xm = x.copy(), x.copy()
        xp[j // 3, j % 3] += h
        xm[j // 3, j % 3] -= h
        fp = O.element_forces(mesh, O.element(mesh, xp), np.ones(1))[0].ravel()
        fm = O.element_forces(mesh, O.element(mesh, xm), np.ones(1))[0].ravel()
        Kfd[:, j] = -(fp - fm) / (2 * h)
    np.testing.assert_allclose(Ku, Kfd, rtol=1e-5, atol=1e-6 * np.abs(Kfd).max())


def test_chi_continuous_across_the_switch_and_finite_when_flat():
    """chi of a damaged tet (one broken edge) uses |J| times the stresses on
    small tets: the ratio is the same function on both sides of J_MIN and has
    a finite limit at J = 0."""
    out = {}
    for J in (O.J_MIN * (1 + 1e-9), O.J_MIN * (1 - 1e-9), 1e-12, -1e-12):
        X, x, _ = tet_with_J(13, J)
        mesh = O.setup(X, np.arange(4)[None], PARAMS)
        zeta = np.zeros(mesh.edges.shape[0], bool)
        zeta[mesh.tet_edge[0, 2]] = True
        chi, mask = O.energy_fraction(mesh, x, zeta)
        assert mask[0] == 4
        out[J] = chi[0]
    assert out[O.J_MIN * (1 + 1e-9)] == pytest.approx(out[O.J_MIN * (1 - 1e-9)], rel=1e-7)
    assert 0.0 < out[1e-12] < 1.0
    assert out[1e-12] == pytest.approx(out[-1e-12], rel=1e-6)
