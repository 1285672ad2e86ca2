"""Persistent per-sample solves (mlq_set_persistent) against the FP64 CPU oracle and the batched path.

Section 3.3's time stepping with Newton-GMRES, one workgroup per sample for the whole time loop.
Bars as for every solve: FP64 per sample and per node within 1e-10 relative of the oracle; mixed
precision QoIs within 1e-6 relative (and the batched mixed path within the same bar).
"""
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


def _setup(env, n, steps, B, prec, qoi, n_modes=8, seed=21, hi=None, guess=1):
    torch, mlq = env
    from oracle import fem, kl
    from oracle.mesh import BoxMesh
    phys = W.physics(3)
    hi = hi or [1.0, 1.0, 1.0]
    mesh = BoxMesh(n, hi=hi)
    M = fem.assemble_mass(mesh)
    lam, psi = kl.kl_modes(mesh, M, 0.3, 0.2, n_modes)
    sl, phi = np.sqrt(lam), kl.level_basis(mesh, psi, mesh)
    Y = W.mc_normals(seed, 0, B, n_modes)
    lv = dict(dim=3, n=list(n), lo=[0.0] * 3, hi=hi, n_steps=steps)
    desc, keep = mlq.make_desc(lv, phys, n_modes=n_modes, phi=phi, sqrt_lambda=sl, prec=prec, qoi=qoi,
                               newton_tol=W.NEWTON_TOL[prec], inner_tol=W.INNER_TOL[prec], max_batch=B,
                               newton_guess=guess)
    L = mlq.Level(desc, keep)
    theta = L.sample_fields(torch.as_tensor(Y, device="cuda"))
    th = kl.field(np.zeros(mesh.n_elems), phi, sl, Y)
    return L, theta, th, mesh, phys


def _oracle(mesh, th, phys, steps, stop=None):
    from oracle import fem, stepper
    out = []
    for b in range(th.shape[0]):
        G = fem.conductivity_from_angle(th[b], 3, phys["sigma_l"], phys["sigma_t"])
        out.append(stepper.solve(mesh, G, phys, steps, tol=1e-13, stop_after=stop))
    return out


@pytest.mark.parametrize("n,steps,qoi", [
    ([9, 9, 9], 32, W.QOI_MEAN_ACT_TIME),
    ([9, 7, 5], 24, W.QOI_MEAN_U_FINAL),     # ragged box: every axis a different length
    ([17, 17, 17], 16, W.QOI_MEAN_ACT_TIME),
])
def test_persistent_fp64_matches_oracle(env, n, steps, qoi):
    torch, mlq = env
    B = 5
    L, theta, th, mesh, phys = _setup(env, n, steps, B, W.PREC_FP64, qoi, hi=[1.0, 0.8, 1.3] if n[1] != n[0] else None)
    L.set_persistent(True)
    out = L.solve(theta, want_state=True)
    torch.cuda.synchronize()
    assert out["code"] == mlq.MLQ_OK
    assert int(out["status"].abs().sum()) == 0
    q = out["qoi"].cpu().numpy()
    u = out["u"].cpu().numpy()
    act = out["act"].cpu().numpy()
    key = "mean_u_final" if qoi == W.QOI_MEAN_U_FINAL else "mean_act"
    for b, r in enumerate(_oracle(mesh, th, phys, steps)):
        assert abs(q[b] - r[key]) <= 1e-10 * abs(r[key]), (b, q[b], r[key])
        assert np.abs(u[b] - r["u"]).max() <= 1e-10 * np.abs(r["u"]).max(), b
        ra = np.where(np.isnan(r["act"]), -1.0, r["act"])
        assert np.array_equal(ra < 0, act[b] < 0), b
        on = ra >= 0
        assert np.abs(act[b][on] - ra[on]).max(initial=0.0) <= 1e-10 * r["t_stop"], b
    it = out["iters"].cpu().numpy()
    assert (it[:, 0] >= steps).all() and (it[:, 1] >= it[:, 0]).all()


def test_persistent_equals_batched_within_tolerance_and_truncated_runs(env):
    """Same samples through both paths (FP64), also stopped after a few steps."""
    torch, mlq = env
    B = 7
    L, theta, th, mesh, phys = _setup(env, [9, 9, 9], 32, B, W.PREC_FP64, W.QOI_MEAN_ACT_TIME, seed=5)
    ref = L.solve(theta, want_state=True)
    L.set_persistent(True)
    for stop in (None, 3, 0):
        out = L.solve(theta, n_steps=stop, want_state=True)
        base = ref if stop is None else (L.set_persistent(False), L.solve(theta, n_steps=stop, want_state=True))[1]
        L.set_persistent(True)
        torch.cuda.synchronize()
        qa, qb = out["qoi"].cpu().numpy(), base["qoi"].cpu().numpy()
        assert np.abs(qa - qb).max() <= 1e-10 * np.abs(qb).max(), stop
        ua, ub = out["u"].cpu().numpy(), base["u"].cpu().numpy()
        assert np.abs(ua - ub).max() <= 1e-10 * max(np.abs(ub).max(), 1e-300), stop


def test_persistent_mixed_precision(env):
    torch, mlq = env
    B = 6
    L, theta, th, mesh, phys = _setup(env, [17, 17, 17], 16, B, W.PREC_MIXED, W.QOI_MEAN_ACT_TIME, seed=9)
    L.set_persistent(True)
    out = L.solve(theta)
    torch.cuda.synchronize()
    assert int(out["status"].abs().sum()) == 0
    q = out["qoi"].cpu().numpy()
    refs = _oracle(mesh, th, phys, 16)
    ref = np.array([r["mean_act"] for r in refs])
    assert np.abs(q - ref).max() <= 1e-6 * np.abs(ref).max()
    assert abs(q.mean() - ref.mean()) <= 1e-6 * abs(ref.mean())
    # and the batched mixed path on the same fields
    L.set_persistent(False)
    qb = L.solve(theta)["qoi"].cpu().numpy()
    assert np.abs(q - qb).max() <= 1e-6 * np.abs(qb).max()


def test_persistent_more_samples_than_resident_workgroups(env):
    """Workgroups walk the batch: 2600 samples (more than the GPU holds at once) all agree with
    the batched path."""
    torch, mlq = env
    B = 2600
    L, theta, th, mesh, phys = _setup(env, [9, 9, 9], 8, B, W.PREC_FP64, W.QOI_MEAN_U_FINAL, seed=3)
    qb = L.solve(theta)["qoi"].cpu().numpy()
    L.set_persistent(True)
    out = L.solve(theta)
    q = out["qoi"].cpu().numpy()
    assert int(out["status"].abs().sum()) == 0
    assert np.abs(q - qb).max() <= 1e-10 * np.abs(qb).max()


def test_persistent_nan_sample_reported(env):
    torch, mlq = env
    B = 4
    L, theta, th, mesh, phys = _setup(env, [9, 9, 9], 8, B, W.PREC_FP64, W.QOI_MEAN_U_FINAL, seed=4)
    qb = L.solve(theta)["qoi"].cpu().numpy()
    theta = theta.clone()
    theta[2, 5] = float("nan")
    L.set_persistent(True)
    out = L.solve(theta)
    torch.cuda.synchronize()
    assert out["code"] == mlq.MLQ_OK  # enqueue only: the status carries the failure
    st = out["status"].cpu().numpy()
    assert st[2] == mlq.MLQ_SAMPLE_NAN and (np.delete(st, 2) == 0).all()
    assert mlq.check_status(st) == mlq.MLQ_ENOCONV
    q = out["qoi"].cpu().numpy()
    for b in (0, 1, 3):
        assert abs(q[b] - qb[b]) <= 1e-10 * abs(qb[b])


def test_persistent_refused_where_it_does_not_apply(env):
    torch, mlq = env
    phys = W.physics(3)
    desc, keep = mlq.make_desc(dict(dim=3, n=[33, 33, 33], lo=[0.0] * 3, hi=[1.0] * 3, n_steps=4), phys, max_batch=2)
    L = mlq.Level(desc, keep)
    with pytest.raises(mlq.MlqError):
        L.set_persistent(True)   # 33^3 x 8 bytes is more than 64 KiB
    desc, keep = mlq.make_desc(dict(dim=2, n=[9, 9], lo=[0.0] * 2, hi=[1.0] * 2, n_steps=4), W.physics(2), max_batch=2)
    with pytest.raises(mlq.MlqError):
        mlq.Level(desc, keep).set_persistent(True)


def test_persistent_solve_captured_in_a_graph_replays_bit_identical(env):
    """An enqueue-only solve can be captured: the whole persistent solve (field coefficients and the
    one solver launch) recorded into a HIP graph through torch, replayed several times with eager
    work and synchronisations in between, every replay equal to the eager solve bit for bit."""
    torch, mlq = env
    B = 6
    L, theta, th, mesh, phys = _setup(env, [9, 9, 9], 16, B, W.PREC_MIXED, W.QOI_MEAN_ACT_TIME, seed=12)
    L.set_persistent(True)
    eager = L.solve(theta, want_state=True)  # also sizes the level's workspace outside the capture
    torch.cuda.synchronize()
    q0, u0 = eager["qoi"].clone(), eager["u"].clone()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        L.solve(theta, want_state=True)  # warm-up on the capture stream
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        cap = L.solve(theta, want_state=True)
    for rep in range(3):
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(cap["qoi"], q0), rep
        assert torch.equal(cap["u"], u0), rep
        assert int(cap["status"].abs().sum()) == 0
        # eager work between the replays
        again = L.solve(theta)
        torch.cuda.synchronize()
        assert torch.equal(again["qoi"], q0)
