"""The allocation-free quasi-static entry point (scratch in a fixed device
array of the library) against the allocating one, through the C ABI: two
calls in a row on meshes of decreasing size, FP64 and split precision --
positions, labels and statistics must agree exactly (same kernels, same
order of operations); a mesh beyond the fixed scratch is refused."""
import numpy as np
import pytest

from paper_2103_14870_amd import gfem, meshgen

from parity_helpers import say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _lib():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    gfem.load()


def block(prec, nx, nz, seed):
    return meshgen.cube_block(nx, 3, nz, h=0.05, jitter_frac=0.08, seed=seed, top_speed=0.004, dt=1.0,
                              precision=prec, cg_rel_tol=1e-10 if prec == "fp64" else 1e-6, damage_strain=0.03)


@pytest.mark.parametrize("prec", ["fp64", "split"])
def test_noalloc_equals_the_allocating_entry_point(prec):
    rtol = 1e-8 if prec == "fp64" else 1e-4
    for nx, nz, seed, steps in ((5, 8, 11, 6), (3, 5, 12, 4)):  # second call: smaller mesh
        say(f"case no-alloc quasi-static prec={prec} mesh {nx}x3x{nz} steps {steps}")
        prob = block(prec, nx, nz, seed)
        with gfem.mesh_from_problem(prob) as ma, gfem.mesh_from_problem(prob) as mb:
            ra = ma.quasi_static_step(steps, newton_rel_tol=rtol)
            rb = mb.quasi_static_step(steps, newton_rel_tol=rtol, noalloc=True)
            xa, xb = ma.positions(), mb.positions()
            say(f"  newton {ra['newton_iters']} / {rb['newton_iters']} broken {ra['total_broken']} / "
                f"{rb['total_broken']} max |dx| {np.abs(xa - xb).max():.1e}")
            assert ra["steps_done"] == rb["steps_done"] == steps
            assert np.array_equal(xa, xb)
            assert np.array_equal(ma.edge_damage(), mb.edge_damage())
            for k in ("newton_iters", "line_search_halvings", "inner_iters", "total_broken", "force_residual"):
                assert ra[k] == rb[k], k
            assert ra["total_broken"] > 0


def test_noalloc_refuses_a_mesh_beyond_its_scratch():
    say("case no-alloc size limit")
    # 16,385 separate tets: 65,540 nodes, one more record than the scratch holds
    base = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]], float) * 0.1
    k = 16385
    X = (base[None, :, :] + 0.5 * np.arange(k)[:, None, None] * np.array([1.0, 0, 0])).reshape(-1, 3)
    tets = np.arange(4 * k, dtype=np.int32).reshape(k, 4)
    p = meshgen.default_params(dt=1.0, damage_strain=10.0)
    with gfem.Mesh(X, tets, p) as m:
        r = m.quasi_static_step(1, noalloc=True, raise_on_error=False)
        assert r["status"] == gfem.GF_EINVAL and r["steps_done"] == 0
        assert b"exceeds the fixed scratch" in gfem.load().gf_last_error()
        # the allocating entry point still works on it
        assert m.quasi_static_step(1)["steps_done"] == 1
