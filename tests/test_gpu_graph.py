"""The GMRES iterations replayed from captured HIP graphs in blocks (mlq_set_gmres_block) against
the same solve launched and steered one iteration at a time: the same kernels run in the same order
on the same data, and converged samples skip the extra iterations of a block, so quantities of
interest, states, statuses and iteration counts agree bit for bit (3D boxes in both precisions and
both lane layouts, a 2D box, a tetrahedral shell), also over repeated solves that replay the graphs."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2105_02007_amd import mlq
    return torch, mlq


def _check_blocks(torch, mlq, level, theta, blocks=(1, 3, 8)):
    level.set_gmres_block(0)
    ref = level.solve(theta, want_state=True)
    torch.cuda.synchronize()
    assert ref["code"] == mlq.MLQ_OK
    for J in blocks:
        level.set_gmres_block(J)
        for rep in range(2):  # the second solve replays the captured graphs
            print(f"gmres block {J}, solve {rep}", flush=True)
            got = level.solve(theta, want_state=True)
            torch.cuda.synchronize()
            assert got["code"] == mlq.MLQ_OK
            for k in ("qoi", "status", "iters", "u", "act"):
                assert torch.equal(got[k], ref[k]), (J, rep, k)
    level.set_gmres_block(0)
    return ref


@pytest.mark.parametrize("prec,lanes", [(0, 8), (1, 16), (1, 8), (0, 16)])
def test_box3d_graph_blocks_match_steered_solve(env, prec, lanes):
    torch, mlq = env
    phys = W.physics(3)
    lv = dict(dim=3, n=[49, 7, 9], lo=[0.0] * 3, hi=[1.0, 0.3, 0.4], n_steps=12)
    desc, keep = mlq.make_desc(lv, phys, prec=prec, qoi=mlq.MLQ_QOI_MEAN_ACT_TIME,
                               newton_tol=1e-13 if prec == 0 else 1e-10, inner_tol=1e-6, max_batch=5,
                               newton_guess=mlq.MLQ_GUESS_EXTRAPOLATE)
    level = mlq.Level(desc, keep)
    level.set_lane_layout(lanes)
    tdt = torch.float32 if prec else torch.float64
    theta = torch.as_tensor(W.random_angles(31, 5, level.n_elems), dtype=tdt, device="cuda")
    ref = _check_blocks(torch, mlq, level, theta)
    assert int(ref["iters"][:, 1].min()) > 12  # GMRES ran several iterations per step


def test_box2d_graph_blocks_match_steered_solve(env):
    torch, mlq = env
    phys = W.physics(2)
    lv = dict(dim=2, n=[21, 17], lo=[0.0] * 2, hi=[1.0, 1.0], n_steps=10)
    desc, keep = mlq.make_desc(lv, phys, prec=0, max_batch=3, newton_tol=1e-13)
    level = mlq.Level(desc, keep)
    theta = torch.as_tensor(W.random_angles(32, 3, level.n_elems), device="cuda")
    _check_blocks(torch, mlq, level, theta, blocks=(2, 5))


def test_shell_graph_blocks_match_steered_solve(env):
    torch, mlq = env
    cfg = W.config("c5")
    lvl = dict(cfg["levels"][0], cells=[2, 12, 24], n_steps=8)
    mesh = W.tet_mesh(lvl)
    desc, keep = mlq.make_desc(dict(lvl, mesh=mesh), cfg["physics"], prec=1, max_batch=4, newton_tol=1e-10,
                               inner_tol=1e-5, qoi=mlq.MLQ_QOI_MEAN_ACT_TIME)
    level = mlq.Level(desc, keep)
    theta = torch.as_tensor(mesh["theta0"][None, :] + 0.3 * W.random_nodal(33, 4, level.n_elems), dtype=torch.float32,
                            device="cuda")
    _check_blocks(torch, mlq, level, theta, blocks=(4,))
