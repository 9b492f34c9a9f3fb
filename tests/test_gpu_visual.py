"""GPU parity of the split visualisation mesh (Sec. 4.1): the library's
sub-cells and corner groups against the oracle's, on the library's own
positions and labels (so the comparison is of the split alone): a damaged,
jittered block whose input tets have both orientations, and the 122,880-tet
beam (two device chunks) on a sample of tets."""
import numpy as np
import pytest

from oracle import gfem_oracle as O
from paper_2103_14870_amd import gfem, meshgen

from parity_helpers import say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _lib():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    gfem.load()


def compare(m, prob, sample=None):
    xyz, grp = m.visual_mesh()
    x, z = m.positions(), m.edge_damage().astype(bool)
    tets = prob.tets if sample is None else prob.tets[sample]
    oxyz, ogrp = O.visual_mesh(prob.X, x, tets, m.edges(), z)
    gx = xyz if sample is None else xyz[sample]
    gg = grp if sample is None else grp[sample]
    err = np.abs(gx - oxyz).max() / np.abs(x).max()
    return err, np.array_equal(gg, ogrp), int((gg != np.arange(4)).sum()), z.sum()


def test_visual_mesh_damaged_block():
    say("case visual mesh, damaged block")
    prob = meshgen.cube_block(4, 3, 3, h=0.1, jitter_frac=0.08, seed=2, top_speed=2.0, damage_strain=0.01)
    tets = prob.tets.copy()
    X = prob.X
    det = np.linalg.det(np.stack([X[tets[:, i]] - X[tets[:, 0]] for i in (1, 2, 3)], axis=2))
    assert (det < 0).any() and (det > 0).any()
    with gfem.mesh_from_problem(prob) as m:
        for _ in range(12):
            m.step(1)
        err, same, _, nb = compare(m, prob)
        say(f"  broken {nb}: max |xyz - oracle| / max |x| = {err:.2e}, groups equal {same}")
        assert nb > 0 and same and err <= 1e-14


def test_visual_mesh_full_size_beam_sample():
    say("case visual mesh, 122,880-tet beam with 30 % cracks (sample)")
    prob = meshgen.notched_beam(crack_fraction=0.3)
    with gfem.mesh_from_problem(prob) as m:
        m.step(2)
        rng = np.random.default_rng(1)
        sample = np.sort(rng.choice(prob.n_tets, 3000, replace=False))
        sample = np.concatenate([sample, [0, 65535, 65536, prob.n_tets - 1]])
        err, same, split, nb = compare(m, prob, sample)
        say(f"  broken {nb}, split corners in sample {split}: err {err:.2e}, groups equal {same}")
        assert same and err <= 1e-14 and split > 0
