"""The solve entry point without allocation (mlq_solve_batch_static: the library's static device
workspace) against the ordinary entry point (mlq_solve_batch_ex with a caller's workspace), through
the C ABI: two calls in a row on one level, the second with a smaller batch and other fields, and a
batch too large for the static workspace refused on the host.  Both entry points run the same
kernels on the same inputs, so every output must agree bit for bit."""
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


@pytest.mark.parametrize("prec", [0, 1])
def test_static_workspace_solve_matches_solve(env, prec):
    torch, mlq = env
    phys = W.physics(3)
    lv = dict(dim=3, n=[9, 9, 9], lo=[0.0] * 3, hi=[1.0] * 3, n_steps=16)
    desc, keep = mlq.make_desc(lv, phys, prec=prec, qoi=mlq.MLQ_QOI_MEAN_ACT_TIME,
                               newton_tol=1e-13 if prec == 0 else 1e-10, max_batch=64,
                               newton_guess=mlq.MLQ_GUESS_EXTRAPOLATE)
    level = mlq.Level(desc, keep)
    tdt = torch.float32 if prec == 1 else torch.float64
    for call, (B, seed) in enumerate([(6, 21), (3, 22)]):
        print(f"static workspace solve: prec {prec}, call {call}, batch {B}", flush=True)
        theta = torch.as_tensor(W.random_angles(seed, B, level.n_elems), dtype=tdt, device="cuda")
        ref = level.solve(theta)
        got = level.solve_static(theta)
        torch.cuda.synchronize()
        assert ref["code"] == mlq.MLQ_OK and got["code"] == mlq.MLQ_OK
        assert torch.equal(got["status"], ref["status"])
        assert torch.equal(got["iters"], ref["iters"])
        assert torch.equal(got["qoi"], ref["qoi"]), (got["qoi"] - ref["qoi"]).abs().max()
        assert int(ref["iters"][:, 1].min()) > 0


def test_static_workspace_refuses_large_batches(env):
    torch, mlq = env
    import ctypes as C
    phys = W.physics(3)
    lv = dict(dim=3, n=[33, 33, 33], lo=[0.0] * 3, hi=[1.0] * 3, n_steps=8)
    desc, keep = mlq.make_desc(lv, phys, prec=0, max_batch=64)
    level = mlq.Level(desc, keep)
    nbytes = C.c_size_t()
    mlq.check(mlq.lib.mlq_workspace_bytes(level.handle, 64, C.byref(nbytes)))
    assert nbytes.value > mlq.STATIC_WS_BYTES
    theta = torch.zeros((64, level.n_elems), dtype=torch.float64, device="cuda")
    with pytest.raises(mlq.MlqError) as e:
        level.solve_static(theta)
    assert e.value.code == mlq.MLQ_ESIZE
