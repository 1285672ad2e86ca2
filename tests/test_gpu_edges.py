"""Edge cases of the solve on the GPU against the oracle: one-element meshes (the smallest
grids the library accepts), a solve stopped after zero steps (quantities of interest of the
initial state), invalid batch sizes refused on the host, and a sample whose field is NaN,
which is reported and leaves the other samples of its batch untouched."""
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


def _level(mlq, n, steps, B, qoi, hi=None, prec=None):
    phys = W.physics(len(n))
    lv = dict(dim=len(n), n=list(n), lo=[0.0] * len(n), hi=hi or [0.2] * len(n), n_steps=steps)
    desc, keep = mlq.make_desc(lv, phys, qoi=qoi, max_batch=B, prec=prec if prec is not None else mlq.MLQ_FP64)
    return mlq.Level(desc, keep), lv, phys


@pytest.mark.parametrize("n", [[2, 2, 2], [2, 2], [3, 2, 2]])
def test_one_element_meshes_match_oracle(env, n):
    torch, mlq = env
    from oracle import fem, stepper
    from oracle.mesh import BoxMesh
    steps, B = 12, 2
    L, lv, phys = _level(mlq, n, steps, B, mlq.MLQ_QOI_MEAN_U_FINAL)
    mesh = BoxMesh(n, hi=lv["hi"])
    th = W.random_angles(3, B, mesh.n_elems)
    out = L.solve(torch.as_tensor(th, device="cuda"), want_state=True)
    assert out["code"] == mlq.MLQ_OK
    u = out["u"].cpu().numpy()
    for b in range(B):
        G = fem.conductivity_from_angle(th[b], len(n), phys["sigma_l"], phys["sigma_t"])
        r = stepper.solve(mesh, G, phys, steps, tol=1e-13)
        assert np.abs(u[b] - r["u"]).max() <= 1e-10 * np.abs(r["u"]).max()
        assert abs(float(out["qoi"][b]) - r["mean_u_final"]) <= 1e-10 * abs(r["mean_u_final"])


@pytest.mark.parametrize("qoi", [0, 1])
def test_zero_steps_give_the_initial_state(env, qoi):
    torch, mlq = env
    L, lv, phys = _level(mlq, [9, 7, 5], 16, 2, qoi)
    th = torch.as_tensor(W.random_angles(4, 2, 8 * 6 * 4), device="cuda")
    out = L.solve(th, n_steps=0, want_state=True)
    assert out["code"] == mlq.MLQ_OK
    assert not out["u"].any() and not out["qoi"].any()  # u_0 = 0; activation censored at t = 0
    assert (out["act"] < 0).all() and not out["iters"].any()


def test_invalid_batches_are_refused(env):
    torch, mlq = env
    L, lv, phys = _level(mlq, [9, 7, 5], 8, 2, 1)
    th = torch.zeros((3, 8 * 6 * 4), dtype=torch.float64, device="cuda")
    with pytest.raises(mlq.MlqError):
        L.solve(th)              # more samples than the level's max_batch
    with pytest.raises(mlq.MlqError):
        L.solve(th[:0])          # no samples


@pytest.mark.parametrize("prec", [0, 1])
def test_nan_sample_is_reported_and_isolated(env, prec):
    torch, mlq = env
    from oracle import fem, stepper
    from oracle.mesh import BoxMesh
    n, steps = [9, 7, 5], 10
    L, lv, phys = _level(mlq, n, steps, 3, mlq.MLQ_QOI_MEAN_ACT_TIME, prec=prec)
    mesh = BoxMesh(n, hi=lv["hi"])
    th = W.random_angles(5, 3, mesh.n_elems)
    th[1, 7] = np.nan
    tdt = torch.float32 if prec == mlq.MLQ_MIXED else torch.float64
    out = L.solve(torch.as_tensor(th, dtype=tdt, device="cuda"))
    assert out["code"] == mlq.MLQ_ENOCONV
    st = out["status"].cpu().numpy()
    assert st[1] == 2 and st[0] == 0 and st[2] == 0  # MLQ_SAMPLE_NAN for sample 1 only
    q = out["qoi"].cpu().numpy()
    for b in (0, 2):
        thb = th[b].astype(np.float32).astype(np.float64) if prec == mlq.MLQ_MIXED else th[b]
        G = fem.conductivity_from_angle(thb, 3, phys["sigma_l"], phys["sigma_t"])
        r = stepper.solve(mesh, G, phys, steps, tol=1e-13)
        tol = 1e-10 if prec == mlq.MLQ_FP64 else 1e-6
        assert abs(q[b] - r["mean_act"]) <= tol * abs(r["mean_act"]), b
