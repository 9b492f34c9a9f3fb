"""GPU parity of the Saint-Venant Kirchhoff energy of the dynamic runs
(Sec. 5.2, Eq. 37) in edge form: forces, blocks and right-hand side on a
deformed, damaged block with flat and inverted tets (norm-wise and per node /
per block), a lockstep run of a pulled brittle block, and the learned
preconditioner on a StVK beam against block-Jacobi at the same residual."""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import gfem_oracle as O
from paper_2103_14870_amd import gfem, meshgen

from parity_helpers import block_rowrel, gpu_sparse, lockstep, rel, rowrel, say
from test_gpu_parity_more import WEIGHTS, flattened_problem

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _lib():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    gfem.load()


@pytest.mark.parametrize("prec", ["fp64", "split"])
@pytest.mark.parametrize("seed", [21, 23])
def test_stvk_forces_and_system_match_oracle(prec, seed):
    say(f"case StVK forces/system prec={prec} seed={seed}")
    prob, U, V, picked = flattened_problem(prec, seed)
    prob.params["energy"] = "stvk"
    mesh = O.setup(prob.X, prob.tets, prob.params)
    st = O.initial_state(mesh)
    st.x = mesh.X + U
    st.v = V
    O.break_pairs(mesh, st, prob.broken_pairs)
    el = O.element(mesh, st.x)
    assert (el.J[picked] < 0).sum() >= 3
    fo = O.restoring_forces(mesh, st)
    zeta, _ = O.damage_update(mesh, st.x, st.zeta)
    so = O.build_system(mesh, st, prob.dir_nodes, prob.dir_vel, zeta, st.Cp)
    with gfem.mesh_from_problem(prob) as m:
        gfem.set_displacement(m, U, V)
        f = m.eval_forces()
        bi, bj, blocks, rhs = m.get_system()
        s = m.step(1)
    ef, efn = rel(f, fo), rowrel(f, fo, 1e-3)
    ea = sp.linalg.norm(gpu_sparse(bi, bj, blocks, prob.n_nodes) - so.A) / sp.linalg.norm(so.A)
    ean = block_rowrel(bi, bj, blocks, so.A, 1e-3)
    eb, ebn = rel(rhs.ravel(), so.b), rowrel(rhs, so.b.reshape(-1, 3), 1e-3)
    say(f"  forces {ef:.2e} / node {efn:.2e}  A {ea:.2e} / block {ean:.2e}  b {eb:.2e} / node {ebn:.2e}  "
        f"degenerate {s['degenerate_tets']} (oracle {so.stats['degenerate_tets']})")
    tol, tol_row = (1e-10, 1e-8) if prec == "fp64" else (1e-5, 1e-3)
    assert ef <= tol and ea <= tol and eb <= tol
    assert efn <= tol_row and ean <= tol_row and ebn <= tol_row
    assert s["degenerate_tets"] == so.stats["degenerate_tets"]


@pytest.mark.parametrize("prec", ["fp64", "split"])
def test_stvk_lockstep(prec):
    """40 steps of a pulled jittered brittle block with the StVK energy."""
    say(f"case StVK lockstep prec={prec}")
    prob = meshgen.cube_block(5, 5, 4, h=0.1, jitter_frac=0.08, seed=7, top_speed=0.8, precision=prec,
                              cg_rel_tol=1e-9 if prec == "fp64" else 1e-6, damage_strain=0.02, energy="stvk")
    m, mesh, st, hist = lockstep(prob, 40, check_every=20)
    last = hist[-1]
    say(f"  broken {int(st.zeta.sum())} disp rel {last['disp_rel']:.2e} per node {last['disp_node']:.2e}")
    assert st.zeta.sum() > 0
    bar, row = (1e-8, 1e-6) if prec == "fp64" else (1e-4, 1e-3)
    assert last["disp_rel"] <= bar and last["disp_node"] <= row
    assert all(h["near_ids_match"] for h in hist)
    m.close()


def test_stvk_learned_preconditioner():
    """The shipped network (trained on neo-Hookean systems) on a cracked StVK
    beam: same residual and trajectory as block-Jacobi, fewer iterations."""
    say("case StVK learned vs block-Jacobi beam")
    prob = meshgen.notched_beam(32, 6, 6, h=0.01, crack_fraction=0.1, crack_seed=5, dt=1e-4, energy="stvk")
    prob.params["net_every_n_steps"] = 4
    net = gfem.Net(seed=0)
    net.set_weights(np.load(WEIGHTS))
    mj = gfem.mesh_from_problem(prob)
    ml = gfem.mesh_from_problem(prob)
    gfem.attach_net(ml, net)
    ij = il = 0
    for _ in range(10):
        sj, sl = mj.step(1), ml.step(1)
        assert sj["rel_residual"] <= 1e-6 and sl["rel_residual"] <= 1e-6 and sl["used_fallback"] == 0
        ij += sj["inner_iters"]
        il += sl["inner_iters"]
    d = rel(ml.positions() - prob.X, mj.positions() - prob.X)
    say(f"  iterations block-Jacobi {ij} learned {il} ({il / ij:.2f}x) disp diff {d:.2e}")
    assert il < ij and d <= 1e-4
    for mm in (mj, ml):
        mm.close()
    net.close()
