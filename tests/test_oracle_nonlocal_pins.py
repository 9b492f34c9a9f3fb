"""Pins of the oracle's non-local damage criterion (Eq. 20 with R_d > 0).

Reading: the support of Eq. 20 is the set of tets whose rest centroids lie
within R_d of the reference tet's; the weights are (1 - (r / R_d)^2)^2
normalised to sum 1; the averaged quantity is the Green strain tensor (the
strain reading of the criterion); an edge breaks when the averaged normal
strain along it reaches the threshold in any tet that contains it.
Pinned against:
  * a support smaller than the centroid spacing: the local criterion (Eq. 28
    makes q^T E q the edge's own strain);
  * an affine deformation (uniform strain): averaging changes nothing;
  * brute-force neighbour search and a brute-force weighted average;
  * the paper's statement that a larger support diffuses cracks (Sec. 5.1):
    a single stretched node breaks edges beyond its own under R_d > 0.
"""
import numpy as np
import pytest

from oracle import gfem_oracle as O
from paper_2103_14870_amd import meshgen as mg

H = 0.1


def block(radius, seed=0, thr=0.02):
    prob = mg.cube_block(4, 4, 3, h=H, jitter_frac=0.08, seed=seed, damage_strain=thr)
    prob.params["damage_radius"] = radius
    return prob, O.setup(prob.X, prob.tets, prob.params)


def local_labels(mesh, x):
    eps = O.edge_strain(mesh, x)
    return eps >= mesh.params["damage_strain"], eps


def test_tiny_support_is_the_local_criterion():
    prob, mesh = block(1e-6 * H)
    rng = np.random.default_rng(1)
    x = mesh.X + 0.01 * rng.normal(size=mesh.X.shape)
    ptr, idx, w = mesh.nonlocal_support
    assert np.array_equal(np.diff(ptr), np.ones(mesh.tets.shape[0]))
    eps_t = O.nonlocal_edge_strain(mesh, x)
    _, eps = local_labels(mesh, x)
    np.testing.assert_allclose(eps_t, eps[mesh.tet_edge], rtol=1e-11, atol=1e-13)
    z, _ = O.damage_update(mesh, x, np.zeros(mesh.edges.shape[0], bool))
    zl, _ = local_labels(mesh, x)
    assert np.array_equal(z, zl) and zl.any() and not zl.all()


@pytest.mark.parametrize("radius", [1.5 * H, 3.0 * H])
def test_uniform_strain_is_unchanged_by_averaging(radius):
    prob, mesh = block(radius, thr=0.03)
    rng = np.random.default_rng(2)
    F = np.eye(3) + 0.05 * rng.normal(size=(3, 3))
    x = mesh.X @ F.T + 0.3
    eps_t = O.nonlocal_edge_strain(mesh, x)
    _, eps = local_labels(mesh, x)
    np.testing.assert_allclose(eps_t, eps[mesh.tet_edge], rtol=1e-10, atol=1e-13)
    z, _ = O.damage_update(mesh, x, np.zeros(mesh.edges.shape[0], bool))
    zl, _ = local_labels(mesh, x)
    assert np.array_equal(z, zl)


def test_support_and_weights_against_brute_force():
    radius = 1.7 * H
    prob, mesh = block(radius)
    ptr, idx, w = mesh.nonlocal_support
    c = mesh.X[mesh.tets].mean(axis=1)
    m = c.shape[0]
    for t in range(0, m, 7):
        d = np.sqrt(np.sum((c - c[t]) ** 2, axis=1))
        ref = np.nonzero(d <= radius)[0]
        got = idx[ptr[t]:ptr[t + 1]]
        assert np.array_equal(got, ref)
        wt = w[ptr[t]:ptr[t + 1]]
        raw = np.array([(1 - (d[j] / radius) ** 2) ** 2 for j in ref])
        np.testing.assert_allclose(wt, raw / raw.sum(), rtol=1e-9, atol=1e-14)
        assert wt[list(ref).index(t)] == wt.max()
    # the averaged strain of one tet, summed by hand
    rng = np.random.default_rng(3)
    x = mesh.X + 0.01 * rng.normal(size=mesh.X.shape)
    t = 17
    Eavg = np.zeros((3, 3))
    for j, wj in zip(idx[ptr[t]:ptr[t + 1]], w[ptr[t]:ptr[t + 1]]):
        a, b, cc, dd = mesh.tets[j]
        Dm = np.stack([mesh.X[b] - mesh.X[a], mesh.X[cc] - mesh.X[a], mesh.X[dd] - mesh.X[a]], axis=1)
        Ds = np.stack([x[b] - x[a], x[cc] - x[a], x[dd] - x[a]], axis=1)
        F = Ds @ np.linalg.inv(Dm)
        Eavg += wj * 0.5 * (F.T @ F - np.eye(3))
    eps_t = O.nonlocal_edge_strain(mesh, x)
    for k, (a, b) in enumerate(O.LOCAL_EDGES):
        q = mesh.X[mesh.tets[t, b]] - mesh.X[mesh.tets[t, a]]
        q /= np.linalg.norm(q)
        assert eps_t[t, k] == pytest.approx(q @ Eavg @ q, rel=1e-12, abs=1e-15)


def test_larger_support_diffuses_the_crack():
    """One interior node pulled out: locally only its own edges are strained.
    With R_d = 2h the averaged strain reaches edges that do not touch it, and
    a threshold below that level breaks some of them (Sec. 5.1: crack
    diffusion grows with the kernel support)."""
    radius = 2.0 * H
    prob, mesh = block(radius)
    n = int(np.argmin(np.sum((mesh.X - mesh.X.mean(axis=0)) ** 2, axis=1)))
    x = mesh.X.copy()
    x[n] += np.array([0.03, 0.02, 0.01])
    eps_t = O.nonlocal_edge_strain(mesh, x)
    _, eps = local_labels(mesh, x)
    touch = np.any(mesh.edges == n, axis=1)
    assert np.all(eps[~touch] == 0.0)
    far = ~touch[mesh.tet_edge]
    thr = 0.5 * eps_t[far].max()
    mesh.params["damage_strain"] = thr
    z, _ = O.damage_update(mesh, x, np.zeros(mesh.edges.shape[0], bool))
    assert np.any(z & ~touch)
    zl, _ = local_labels(mesh, x)
    assert not np.any(zl & ~touch)


def test_nonlocal_labels_never_revert():
    prob, mesh = block(1.5 * H)
    rng = np.random.default_rng(4)
    zeta = rng.random(mesh.edges.shape[0]) < 0.2
    z, _ = O.damage_update(mesh, mesh.X.copy(), zeta)
    assert np.array_equal(z, zeta)
