"""Pins of the oracle's split visualisation mesh (Sec. 4.1, node-associated
four-split of each tet):
  * no broken edge: every sub-cell is the image of its rest sub-cell under the
    tet's affine deformation (children at the current centroids), and the four
    sub-cells tile the deformed tet (volumes sum to the tet's);
  * every edge broken: every sub-cell is its rest sub-cell translated by its
    corner's displacement (each child follows its own parent);
  * the paper's face example: both edges at PF1 broken and PF2-PF3 not: SF1
    follows PF1, SF2 and SF3 the average movement of PF2 and PF3;
  * the copies of a split point that two tets share agree (same parent group,
    same position), and group labels follow the tet's unbroken-edge graph.
"""
import itertools

import numpy as np
import pytest

from oracle import gfem_oracle as O
from paper_2103_14870_amd import meshgen as mg


def hexa_volume(v):
    """Volume of a sub-cell [corner, e1, e2, e3, f12, f13, f23, c] split into
    six tets around the diagonal corner -> c (a hexahedron with planar or
    twisted faces: the sum of these six signed volumes)."""
    a, e1, e2, e3, f12, f13, f23, c = v
    tets = [(a, e1, f12, c), (a, f12, e2, c), (a, e2, f23, c), (a, f23, e3, c), (a, e3, f13, c), (a, f13, e1, c)]
    return sum(abs(np.linalg.det(np.stack([q - p, r - p, s_ - p]))) / 6.0 for p, q, r, s_ in tets)


def block(seed=2):
    prob = mg.cube_block(2, 2, 2, h=0.1, jitter_frac=0.08, seed=seed)
    edges = mg.unique_edges(prob.tets)
    return prob, edges


def test_undamaged_subcells_follow_the_affine_map_and_tile_the_tet():
    prob, edges = block()
    rng = np.random.default_rng(3)
    F = np.eye(3) + 0.2 * rng.normal(size=(3, 3))
    x = prob.X @ F.T + 0.01
    zeta = np.zeros(edges.shape[0], bool)
    xyz, group = O.visual_mesh(prob.X, x, prob.tets, edges, zeta)
    rest, _ = O.visual_mesh(prob.X, prob.X, prob.tets, edges, zeta)
    np.testing.assert_allclose(xyz, rest @ F.T + 0.01, rtol=0, atol=1e-14)
    assert not group.any()
    for t in range(prob.tets.shape[0]):
        P = x[prob.tets[t]]
        V = abs(np.linalg.det(P[1:] - P[0])) / 6.0
        vols = [hexa_volume(xyz[t, a]) for a in range(4)]
        assert sum(vols) == pytest.approx(V, rel=1e-12)
        np.testing.assert_allclose(vols, V / 4.0, rtol=1e-12)


def test_all_broken_subcells_move_with_their_corner():
    prob, edges = block()
    rng = np.random.default_rng(4)
    x = prob.X + 0.02 * rng.normal(size=prob.X.shape)
    zeta = np.ones(edges.shape[0], bool)
    xyz, group = O.visual_mesh(prob.X, x, prob.tets, edges, zeta)
    rest, _ = O.visual_mesh(prob.X, prob.X, prob.tets, edges, np.zeros_like(zeta))
    for t in range(prob.tets.shape[0]):
        for a in range(4):
            u = x[prob.tets[t, a]] - prob.X[prob.tets[t, a]]
            np.testing.assert_allclose(xyz[t, a], rest[t, a] + u, rtol=0, atol=1e-14)
    assert np.array_equal(group, np.tile(np.arange(4, dtype=np.uint8), (prob.tets.shape[0], 1)))


def test_the_papers_face_example():
    X = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]], float)
    tets = np.array([[0, 1, 2, 3]])
    edges = np.array(list(itertools.combinations(range(4), 2)))
    rng = np.random.default_rng(5)
    x = X + 0.1 * rng.normal(size=X.shape)
    u = x - X
    # face (0, 1, 2) = (PF1, PF2, PF3): edges 0-1 and 0-2 broken, 1-2 not; edges to node 3 unbroken
    zeta = np.array([e in ((0, 1), (0, 2)) for e in map(tuple, edges)])
    xyz, group = O.visual_mesh(X, x, tets, edges, zeta)
    fc = X[[0, 1, 2]].mean(axis=0)
    # corner 0's face point (1, 2) is its vertex 4; corner 1's face point (0, 2) is its vertex 4;
    # corner 2's face point (0, 1) is its vertex 4
    np.testing.assert_allclose(xyz[0, 0, 4], fc + u[0], atol=1e-15)
    np.testing.assert_allclose(xyz[0, 1, 4], fc + (u[1] + u[2]) / 2, atol=1e-15)
    np.testing.assert_allclose(xyz[0, 2, 4], fc + (u[1] + u[2]) / 2, atol=1e-15)
    # in the whole tet node 0 still connects to 3 and through it to 1 and 2
    assert np.array_equal(group[0], [0, 0, 0, 0])


def test_shared_split_points_agree():
    prob, edges = block(seed=6)
    rng = np.random.default_rng(7)
    x = prob.X + 0.02 * rng.normal(size=prob.X.shape)
    zeta = rng.random(edges.shape[0]) < 0.4
    xyz, group = O.visual_mesh(prob.X, x, prob.tets, edges, zeta)
    seen = {}
    for t in range(prob.tets.shape[0]):
        nd = prob.tets[t]
        for a in range(4):
            others = [b for b in range(4) if b != a]
            for j, b in enumerate(others):
                k = ("e", nd[a], frozenset((nd[a], nd[b])))
                if k in seen:
                    np.testing.assert_allclose(xyz[t, a, 1 + j], seen[k], atol=1e-15)
                seen[k] = xyz[t, a, 1 + j]
            for j, (b, c) in enumerate(((others[0], others[1]), (others[0], others[2]), (others[1], others[2]))):
                k = ("f", nd[a], frozenset((nd[a], nd[b], nd[c])))
                if k in seen:
                    np.testing.assert_allclose(xyz[t, a, 4 + j], seen[k], atol=1e-15)
                seen[k] = xyz[t, a, 4 + j]
    # group labels: corners with the same label are joined by an unbroken path
    for t in range(prob.tets.shape[0]):
        lut_mask = 0
        for k, (a, b) in enumerate(O.LOCAL_EDGES):
            i, j = sorted((prob.tets[t, a], prob.tets[t, b]))
            e = np.nonzero((edges[:, 0] == i) & (edges[:, 1] == j))[0][0]
            lut_mask |= int(zeta[e]) << k
        assert O.DISCONNECTED[lut_mask] == (len(set(group[t].tolist())) > 1)
