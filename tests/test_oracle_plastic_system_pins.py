"""Pins of the oracle's plastic update and of its backward-Euler system.

The plastic update (the ductile reading: multiplicative, volume-preserving
plastic flow F = Fe Fp with an instant radial return of the deviatoric
elastic Hencky strain, no hardening, stored as the plastic rest shape
Gp = Dm^T Cp Dm on the Gram matrix) is checked against the properties that
define such a return, each computed here from the deformation gradient with
a different eigen-routine than the oracle's:
  * below yield the plastic state does not move;
  * after the return the deviatoric elastic Hencky strain has norm equal to
    the yield strain and points the same way as before, its volumetric part
    is untouched, and det Cp stays 1 (isochoric flow);
  * a nearly flat or inverted tet (det F < 0.05) does not flow;
  * a uniaxial isochoric stretch returns to the closed-form plastic stretch;
  * the plastic rest Gram matrix gives I_C = tr(C Cp^-1) and J = det F.
The system (one linearised backward-Euler step, Sec. 4.3, consistent mass of
Eq. 5, Dirichlet elimination) is checked against closed forms on a single
tetrahedron with three prescribed nodes: the textbook linear-elastic tet
stiffness and the textbook backward-Euler step of a linear oscillator, and
against a Dirichlet elimination done by hand with dense linear algebra.
"""
import numpy as np
import pytest

from oracle import gfem_oracle as O

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")

PARAMS = dict(youngs=2.0e4, poisson=0.3, density=900.0, damage_strain=10.0, dt=2e-3,
              cg_rel_tol=1e-13, cg_max_iter=5000)


def one_tet(seed, scale=0.1):
    rng = np.random.default_rng(seed)
    base = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]], float)
    while True:
        P = base + 0.25 * rng.normal(size=(4, 3))
        if np.linalg.det((P[1:] - P[0]).T) > 0.1:
            return P * scale


def defgrad(X, x):
    Dm = (X[1:] - X[0]).T
    Ds = (x[1:] - x[0]).T
    return Ds @ np.linalg.inv(Dm)


def random_Cp(rng, amp):
    """A random symmetric positive definite tensor with det 1."""
    A = rng.normal(size=(3, 3))
    w, V = np.linalg.eigh(0.5 * (A + A.T))
    w = amp * (w - w.mean())
    return V @ np.diag(np.exp(w)) @ V.T


def hencky(C, Cp):
    """Elastic Hencky strains (sorted) from the eigenvalues of Cp^-1 C,
    computed with the general (non-symmetric) eigen-solver."""
    lam = np.sort(np.linalg.eigvals(np.linalg.solve(Cp, C)).real)
    return 0.5 * np.log(lam)


# ---------------------------------------------------------------- plasticity

@pytest.mark.parametrize("seed", range(6))
def test_plastic_return_properties(seed):
    rng = np.random.default_rng(seed)
    X = one_tet(seed)
    ey = 0.05
    mesh = O.setup(X, np.arange(4)[None], dict(PARAMS, yield_strain=ey))
    X = mesh.X[mesh.tets[0]]
    F0 = np.eye(3) + 0.3 * rng.normal(size=(3, 3))
    x = X @ F0.T
    Cp = random_Cp(rng, 0.1)[None]
    F = defgrad(X, x)
    C = F.T @ F
    h0 = hencky(C, Cp[0])
    d0 = h0 - h0.mean()
    assert np.linalg.norm(d0) > ey, "case must start above yield"
    Cp1 = O.plastic_update(mesh, x, Cp)
    h1 = hencky(C, Cp1[0])
    d1 = h1 - h1.mean()
    # on the yield surface, same direction, volumetric part untouched
    assert np.linalg.norm(d1) == pytest.approx(ey, rel=1e-10)
    np.testing.assert_allclose(d1, d0 * (ey / np.linalg.norm(d0)), rtol=0, atol=1e-11)
    assert h1.mean() == pytest.approx(h0.mean(), rel=1e-10, abs=1e-13)
    # isochoric, symmetric positive definite
    assert np.linalg.det(Cp1[0]) == pytest.approx(1.0, rel=1e-12)
    np.testing.assert_allclose(Cp1[0], Cp1[0].T, rtol=0, atol=1e-14)
    assert np.linalg.eigvalsh(Cp1[0]).min() > 0
    # a second return at the same state does not move it (on the surface)
    np.testing.assert_allclose(O.plastic_update(mesh, x, Cp1), Cp1, rtol=0, atol=1e-12)


@pytest.mark.parametrize("seed", range(4))
def test_plastic_no_flow_below_yield(seed):
    rng = np.random.default_rng(100 + seed)
    X = one_tet(seed)
    mesh = O.setup(X, np.arange(4)[None], dict(PARAMS, yield_strain=0.05))
    X = mesh.X[mesh.tets[0]]
    Cp = random_Cp(rng, 0.3)[None]
    # elastic stretch with a deviatoric Hencky strain of norm 0.04 (< yield)
    # and any volume change, on top of the plastic state: C = Cp^1/2 Be Cp^1/2
    w, V = np.linalg.eigh(Cp[0])
    Ch = V @ np.diag(np.sqrt(w)) @ V.T
    dh = rng.normal(size=3)
    dh -= dh.mean()
    dh *= 0.04 / np.linalg.norm(dh)
    Q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    Be = Q @ np.diag(np.exp(2 * (dh + 0.07))) @ Q.T
    C = Ch @ Be @ Ch
    wc, Vc = np.linalg.eigh(C)
    F = Vc @ np.diag(np.sqrt(wc)) @ Vc.T          # F^T F = C
    x = X @ F.T
    np.testing.assert_array_equal(O.plastic_update(mesh, x, Cp), Cp)
    # plasticity switched off: never moves
    mesh0 = O.setup(X, np.arange(4)[None], dict(PARAMS, yield_strain=0.0))
    np.testing.assert_array_equal(O.plastic_update(mesh0, x * 3.0, Cp), Cp)


@pytest.mark.parametrize("J", [0.04, 1e-3, -0.2, -1.5])
def test_no_flow_in_flat_or_inverted_tets(J):
    """A tet far above yield whose det F is below 0.05 (nearly flat, or
    inverted) keeps its plastic state; the same shear with det F = 1 flows."""
    X = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]], float) * 0.1
    mesh = O.setup(X, np.arange(4)[None], dict(PARAMS, yield_strain=0.05))
    X = mesh.X[mesh.tets[0]]
    shear = np.eye(3) + np.array([[0, 0.8, 0], [0, 0, 0], [0, 0, 0]])
    Cp = np.eye(3)[None]
    flows = O.plastic_update(mesh, X @ shear.T, Cp)
    assert np.abs(flows - Cp).max() > 0.1
    F = shear @ np.diag([1.0, 1.0, J])  # det F = J
    np.testing.assert_array_equal(O.plastic_update(mesh, X @ F.T, Cp), Cp)


def test_uniaxial_isochoric_stretch_closed_form():
    """F = diag(a, a^-1/2, a^-1/2) from Cp = I: Hencky strains (1, -1/2, -1/2) log a
    have deviator norm sqrt(3/2) log a; the returned elastic strain is that
    direction at norm ey, so Cp = diag(a^2 e^-2 h1, ...) with
    h = (1, -1/2, -1/2) ey / sqrt(3/2)."""
    X = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]], float) * 0.1
    ey = 0.05
    mesh = O.setup(X, np.arange(4)[None], dict(PARAMS, yield_strain=ey))
    a = 1.3
    st = np.array([a, a ** -0.5, a ** -0.5])
    x = X * st
    Cp = O.plastic_update(mesh, x, np.eye(3)[None])[0]
    h = np.array([1.0, -0.5, -0.5]) * ey / np.sqrt(1.5)
    np.testing.assert_allclose(Cp, np.diag(st ** 2 * np.exp(-2 * h)), rtol=1e-12, atol=1e-14)


def test_plastic_rest_gram_gives_the_elastic_invariants():
    rng = np.random.default_rng(7)
    for seed in range(5):
        X = one_tet(seed)
        mesh = O.setup(X, np.arange(4)[None], dict(PARAMS, yield_strain=0.05))
        X = mesh.X[mesh.tets[0]]
        x = X @ (np.eye(3) + 0.2 * rng.normal(size=(3, 3))).T
        Cp = random_Cp(rng, 0.3)[None]
        el = O.element(mesh, x, Cp)
        Dm = (X[1:] - X[0]).T
        F = defgrad(X, x)
        Gp = mesh.G0[0] + O.gram_offset(mesh, Cp)[0]
        np.testing.assert_allclose(np.linalg.inv(Dm).T @ Gp @ np.linalg.inv(Dm), Cp[0], rtol=1e-12, atol=1e-13)
        assert el.IC[0] == pytest.approx(np.trace(F.T @ F @ np.linalg.inv(Cp[0])), rel=1e-12)
        assert el.J[0] == pytest.approx(np.linalg.det(F), rel=1e-12)
        # the plastic rest shape is stress-free
        elr = O.element(mesh, X @ np.linalg.cholesky(Cp[0]), Cp)
        f = O.element_forces(mesh, elr, np.ones(1))
        assert np.abs(f).max() <= 1e-9 * mesh.mu * 0.01


# ---------------------------------------------------------------- backward Euler system

def textbook_tet_stiffness(X, E, nu):
    """V B^T D B of linear elasticity for one tet (12 x 12)."""
    Dm = (X[1:] - X[0]).T
    V = np.linalg.det(Dm) / 6.0
    grads = np.linalg.inv(Dm)
    grads = np.vstack([-grads.sum(axis=0), grads])
    c = E / ((1 + nu) * (1 - 2 * nu))
    D = c * np.array([[1 - nu, nu, nu, 0, 0, 0], [nu, 1 - nu, nu, 0, 0, 0], [nu, nu, 1 - nu, 0, 0, 0],
                      [0, 0, 0, (1 - 2 * nu) / 2, 0, 0], [0, 0, 0, 0, (1 - 2 * nu) / 2, 0],
                      [0, 0, 0, 0, 0, (1 - 2 * nu) / 2]])
    B = np.zeros((6, 12))
    for a in range(4):
        bx, by, bz = grads[a]
        B[:, 3 * a:3 * a + 3] = [[bx, 0, 0], [0, by, 0], [0, 0, bz], [by, bx, 0], [0, bz, by], [bz, 0, bx]]
    return V * B.T @ D @ B, V


@pytest.mark.parametrize("seed", range(3))
def test_single_free_node_step_is_textbook_backward_euler(seed):
    """Three nodes held at rest, the fourth displaced by a tiny u0 with
    velocity v0.  In the linear regime the method's step is backward Euler on
    the oscillator m v' = -K u (m = 2 rho V / 20, K the textbook 3x3 block of
    the free node): v1 = (m I + dt^2 K)^-1 (m v0 - dt K u0), x1 = x0 + dt v1."""
    rng = np.random.default_rng(seed)
    X = one_tet(seed)
    p = dict(PARAMS)
    mesh = O.setup(X, np.arange(4)[None], p)
    X = mesh.X
    free = 3
    fixed = [0, 1, 2]
    K, V = textbook_tet_stiffness(X, p["youngs"], p["poisson"])
    Kff = K[3 * free:3 * free + 3, 3 * free:3 * free + 3]
    m = 2.0 * p["density"] * V / 20.0
    dt = p["dt"]
    u0 = 1e-7 * rng.normal(size=3)
    v0 = rng.normal(size=3)
    st = O.initial_state(mesh)
    st.x[free] += u0
    st.v[free] = v0
    new, stats = O.step(mesh, st, fixed, np.zeros((3, 3)))
    assert stats["converged"]
    v1 = np.linalg.solve(m * np.eye(3) + dt * dt * Kff, m * v0 - dt * Kff @ u0)
    np.testing.assert_allclose(new.v[free], v1, rtol=2e-6, atol=1e-9 * np.abs(v1).max())
    np.testing.assert_allclose(new.x[free], st.x[free] + dt * new.v[free], rtol=0, atol=1e-15)
    # prescribed nodes move exactly at their prescribed velocity (zero)
    np.testing.assert_array_equal(new.v[fixed], 0.0)
    np.testing.assert_array_equal(new.x[fixed], X[fixed])
    # the assembled 3x3 system of the free node: A = m I + dt^2 K, b = -dt K u0 - dt^2 K v0
    sysm = O.build_system(mesh, st, fixed, np.zeros((3, 3)), st.zeta, st.Cp)
    A = sysm.A.toarray()
    f3 = slice(3 * free, 3 * free + 3)
    Aref = m * np.eye(3) + dt * dt * Kff
    np.testing.assert_allclose(A[f3, f3], Aref, rtol=0, atol=1e-6 * np.abs(Aref).max())
    np.testing.assert_allclose(sysm.b[f3], -dt * Kff @ u0 - dt * dt * Kff @ v0, rtol=1e-5,
                               atol=1e-9 * np.abs(dt * dt * Kff @ v0).max())


def test_dirichlet_elimination_equals_dense_partition():
    """Eliminate prescribed velocity increments by hand from the unconstrained
    system (dense partition A_ff dv_f = b_f - A_fc dv_c) and compare with the
    oracle's eliminated system and its solution."""
    rng = np.random.default_rng(3)
    X = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1], [1, 1, 1]], float) * 0.1
    X += 0.01 * rng.normal(size=X.shape)
    tets = np.array([[0, 1, 2, 3], [1, 2, 3, 4]])
    mesh = O.setup(X, tets, dict(PARAMS))
    st = O.initial_state(mesh)
    st.x = mesh.X + 0.004 * rng.normal(size=X.shape)
    st.v = rng.normal(size=X.shape)
    fixed = np.array([0, 4])
    vpres = rng.normal(size=(2, 3))
    full = O.build_system(mesh, st, [], np.zeros((0, 3)), st.zeta, st.Cp)
    elim = O.build_system(mesh, st, fixed, vpres, st.zeta, st.Cp)
    A, b = full.A.toarray(), full.b
    cd = np.concatenate([3 * c + np.arange(3) for c in fixed])
    fd = np.setdiff1d(np.arange(3 * X.shape[0]), cd)
    dvc = (vpres - st.v[fixed]).ravel()
    dvf = np.linalg.solve(A[np.ix_(fd, fd)], b[fd] - A[np.ix_(fd, cd)] @ dvc)
    Ae = elim.A.toarray()
    np.testing.assert_allclose(Ae[np.ix_(fd, fd)], A[np.ix_(fd, fd)], rtol=0, atol=0)
    np.testing.assert_array_equal(Ae[np.ix_(cd, cd)], np.eye(cd.size))
    np.testing.assert_array_equal(Ae[np.ix_(cd, fd)], 0.0)
    np.testing.assert_array_equal(Ae[np.ix_(fd, cd)], 0.0)
    np.testing.assert_allclose(elim.b[cd], dvc, rtol=0, atol=0)
    dv = np.linalg.solve(Ae, elim.b)
    np.testing.assert_allclose(dv[fd], dvf, rtol=1e-10, atol=1e-12)
    np.testing.assert_allclose(dv[cd], dvc, rtol=0, atol=1e-14)


def test_rayleigh_damping_enters_as_backward_euler_of_the_damped_oscillator():
    """Same single free node with Rayleigh damping b = a M + c K: backward
    Euler of m v' = -K u - (a m + c K) v gives
    v1 = (m(1 + dt a) I + (dt^2 + dt c) K)^-1 (m v0 - dt K u0)."""
    rng = np.random.default_rng(11)
    X = one_tet(4)
    a_, c_ = 3.0, 2e-4
    p = dict(PARAMS, rayleigh_alpha=a_, rayleigh_beta=c_)
    mesh = O.setup(X, np.arange(4)[None], p)
    X = mesh.X
    K, V = textbook_tet_stiffness(X, p["youngs"], p["poisson"])
    Kff = K[9:12, 9:12]
    m = 2.0 * p["density"] * V / 20.0
    dt = p["dt"]
    u0 = 1e-7 * rng.normal(size=3)
    v0 = rng.normal(size=3)
    st = O.initial_state(mesh)
    st.x[3] += u0
    st.v[3] = v0
    new, stats = O.step(mesh, st, [0, 1, 2], np.zeros((3, 3)))
    assert stats["converged"]
    v1 = np.linalg.solve(m * (1 + dt * a_) * np.eye(3) + (dt * dt + dt * c_) * Kff, m * v0 - dt * Kff @ u0)
    np.testing.assert_allclose(new.v[3], v1, rtol=2e-6, atol=1e-9 * np.abs(v1).max())


def test_gravity_enters_as_body_force():
    """All four nodes free, at rest, undeformed, with gravity g: every node
    falls at v1 = dt g (M is consistent, so M^-1 (M g) = g node-wise)."""
    X = one_tet(2)
    g = np.array([0.0, -9.81, 1.5])
    mesh = O.setup(X, np.arange(4)[None], dict(PARAMS, gravity=g))
    st = O.initial_state(mesh)
    new, stats = O.step(mesh, st, [], np.zeros((0, 3)))
    assert stats["converged"]
    np.testing.assert_allclose(new.v, np.tile(PARAMS["dt"] * g, (4, 1)), rtol=1e-10, atol=1e-13)
