"""Host logic of the training driver (no GPU): the seeded episode generator
gives valid split-precision problems of every kind, reproducibly."""
import numpy as np
import pytest

from paper_2103_14870_amd import meshgen, train_precond


def tet_volumes(X, tets):
    d = X[tets[:, 1:]] - X[tets[:, :1]]
    return np.linalg.det(d) / 6.0


@pytest.mark.parametrize("fine", [0.0, 1.0])
def test_episodes_are_valid_and_seeded(fine):
    kinds = set()
    for seed in range(6):
        p1, n1 = train_precond.episode(np.random.default_rng(seed), 40, fine)
        p2, n2 = train_precond.episode(np.random.default_rng(seed), 40, fine)
        assert n1 == n2 and np.array_equal(p1.X, p2.X) and np.array_equal(p1.tets, p2.tets)
        assert 10 <= n1 <= 40
        assert p1.params["precision"] == "split" and p1.params["cg_rel_tol"] == 1e-6
        v = np.abs(tet_volumes(p1.X, p1.tets))
        assert v.min() > 0
        assert p1.dir_nodes.size > 0 and p1.dir_vel.shape == (p1.dir_nodes.size, 3)
        kinds.add(p1.name.split()[0])
        if fine == 1.0:
            # cells of the 620k-tet workload's size on a scaled-down body
            e = meshgen.unique_edges(p1.tets)
            med = np.median(np.linalg.norm(p1.X[e[:, 1]] - p1.X[e[:, 0]], axis=1))
            assert 0.015 < med < 0.04
    assert kinds
