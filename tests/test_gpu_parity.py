"""GPU parity: the HIP path through the C ABI against the FP64 CPU oracle.

Bars: FP64 mode, per element / per sample within 1e-10 relative (operator
applies within 1e-13 of the row scale); mixed mode, QoI statistics within 1e-6
relative of the FP64 oracle.
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


def _level(dim, n, steps, lo=None, hi=None):
    return dict(dim=dim, n=list(n), lo=lo or [0.0] * dim, hi=hi or [1.0] * dim, n_steps=steps)


def _kl(mesh, n_modes, ell=0.2):
    from oracle import fem, kl
    M = fem.assemble_mass(mesh)
    lam, psi = kl.kl_modes(mesh, M, 0.3, ell, n_modes)
    return np.sqrt(lam), kl.level_basis(mesh, psi, mesh)


def _oracle_apply(mesh, theta, x, d, phys, dt):
    from oracle import fem
    G = fem.conductivity_from_angle(theta, mesh.d, phys["sigma_l"], phys["sigma_t"])
    M, K = fem.assemble(mesh, G)
    y = M @ ((1.0 + d) * x) + 0.5 * dt * (K @ x)
    scale = abs(M) @ np.abs((1.0 + d) * x) + 0.5 * dt * (abs(K) @ np.abs(x))
    return y, scale


@pytest.mark.parametrize("dim,n,mixed", [
    (3, [9, 7, 5], False), (3, [17, 17, 17], False), (2, [33, 33], False), (2, [13, 30], False),
    (3, [9, 7, 5], True), (3, [17, 17, 17], True), (2, [33, 33], True),
    # x-extent >= 48: the 16 x 4 lane layout of the 3D kernels, ragged in every direction
    (3, [49, 7, 5], False), (3, [61, 11, 13], True), (3, [64, 4, 12], False),
])
def test_apply_matches_assembled_jacobian(env, dim, n, mixed):
    torch, mlq = env
    from oracle.mesh import BoxMesh
    phys = W.physics(dim)
    lv_desc = _level(dim, n, 16, hi=[1.0, 0.8, 1.3][:dim])
    B = 3
    desc, keep = mlq.make_desc(lv_desc, phys, prec=mlq.MLQ_MIXED if mixed else mlq.MLQ_FP64, max_batch=B)
    lv = mlq.Level(desc, keep)
    mesh = BoxMesh(n, hi=lv_desc["hi"])
    dt = phys["t_end"] / 16
    theta = W.random_angles(3, B, mesh.n_elems)
    x = W.random_nodal(4, B, mesh.n_nodes)
    dv = W.random_nodal(5, B, mesh.n_nodes, -0.05, 0.14)
    tdt = torch.float32 if mixed else torch.float64
    th_d = torch.as_tensor(theta, dtype=tdt, device="cuda")
    x_d = torch.as_tensor(x, dtype=tdt, device="cuda")
    d_d = torch.as_tensor(dv, dtype=tdt, device="cuda")
    y = lv.apply(th_d, x_d, d_d).double().cpu().numpy()
    for b in range(B):
        # the oracle sees exactly the inputs the GPU saw (rounded to FP32 in mixed mode)
        tb = th_d[b].double().cpu().numpy()
        xb = x_d[b].double().cpu().numpy()
        db = d_d[b].double().cpu().numpy()
        ref, scale = _oracle_apply(mesh, tb, xb, db, phys, dt)
        tol = (2e-6 if mixed else 3e-14) * scale.max()
        assert np.abs(y[b] - ref).max() <= tol, (b, np.abs(y[b] - ref).max() / scale.max())


def _solve_pair(env, dim, n, steps, B, qoi, prec, n_modes=8, seed=7, phys=None, stop=None, guess=0):
    torch, mlq = env
    from oracle import fem, kl, stepper
    from oracle.mesh import BoxMesh
    phys = phys or W.physics(dim)
    mesh = BoxMesh(n)
    sl, phi = _kl(mesh, n_modes)
    Y = W.mc_normals(seed, 0, B, n_modes)
    tol = W.NEWTON_TOL[prec]
    desc, keep = mlq.make_desc(_level(dim, n, steps), phys, n_modes=n_modes, phi=phi, sqrt_lambda=sl, prec=prec,
                               qoi=qoi, newton_tol=tol, inner_tol=W.INNER_TOL[prec], max_batch=B,
                               newton_guess=guess)
    lv = mlq.Level(desc, keep)
    theta = lv.sample_fields(torch.as_tensor(Y, device="cuda"))
    out = lv.solve(theta, n_steps=stop, want_state=True)
    torch.cuda.synchronize()
    th = kl.field(np.zeros(mesh.n_elems), phi, sl, Y)
    refs = []
    for b in range(B):
        G = fem.conductivity_from_angle(th[b], dim, phys["sigma_l"], phys["sigma_t"])
        refs.append(stepper.solve(mesh, G, phys, steps, tol=1e-13, stop_after=stop))
    return out, refs, mesh


def test_solve_fp64_2d_mean_u(env):
    torch, mlq = env
    out, refs, mesh = _solve_pair(env, 2, [17, 17], 32, 4, W.QOI_MEAN_U_FINAL, W.PREC_FP64)
    assert int(out["status"].abs().sum()) == 0
    q = out["qoi"].cpu().numpy()
    u = out["u"].cpu().numpy()
    for b, r in enumerate(refs):
        assert abs(q[b] - r["mean_u_final"]) <= 1e-10 * abs(r["mean_u_final"])
        assert np.abs(u[b] - r["u"]).max() <= 1e-10 * np.abs(r["u"]).max()
    it = out["iters"].cpu().numpy()
    assert (it[:, 0] >= 32).all() and (it[:, 1] >= it[:, 0]).all()


def test_solve_fp64_3d_activation(env):
    torch, mlq = env
    out, refs, mesh = _solve_pair(env, 3, [9, 9, 9], 32, 3, W.QOI_MEAN_ACT_TIME, W.PREC_FP64)
    assert int(out["status"].abs().sum()) == 0
    q = out["qoi"].cpu().numpy()
    act = out["act"].cpu().numpy()
    u = out["u"].cpu().numpy()
    for b, r in enumerate(refs):
        assert abs(q[b] - r["mean_act"]) <= 1e-10 * abs(r["mean_act"])
        assert np.abs(u[b] - r["u"]).max() <= 1e-10 * np.abs(r["u"]).max()
        ra = np.where(np.isnan(r["act"]), -1.0, r["act"])
        assert np.array_equal(ra < 0, act[b] < 0)
        on = ra >= 0
        assert np.abs(act[b][on] - ra[on]).max(initial=0.0) <= 1e-10 * r["t_stop"]
    # the mass-inverse preconditioner keeps GMRES short (mass-dominated Jacobian)
    it = out["iters"].cpu().numpy()
    assert (it[:, 1] / it[:, 0]).max() < 12, it


def test_solve_fp64_ragged_3d_truncated(env):
    """A ragged box spanning several blocks, stopped after 6 of 64 steps."""
    torch, mlq = env
    out, refs, mesh = _solve_pair(env, 3, [19, 13, 11], 64, 2, W.QOI_MEAN_U_FINAL, W.PREC_FP64, stop=6)
    u = out["u"].cpu().numpy()
    for b, r in enumerate(refs):
        assert np.abs(u[b] - r["u"]).max() <= 1e-10 * np.abs(r["u"]).max()


def test_solve_fp64_ragged_wide_3d_truncated(env):
    """A box wide enough in x for the 16 x 4 lane layout (ragged tiles in x, y and z), with
    the fused projections of the apply kernel, stopped after 5 of 64 steps."""
    torch, mlq = env
    out, refs, mesh = _solve_pair(env, 3, [53, 8, 6], 64, 2, W.QOI_MEAN_U_FINAL, W.PREC_FP64, stop=5)
    assert int(out["status"].abs().sum()) == 0
    u = out["u"].cpu().numpy()
    for b, r in enumerate(refs):
        assert np.abs(u[b] - r["u"]).max() <= 1e-10 * np.abs(r["u"]).max()


@pytest.mark.parametrize("prec", [W.PREC_FP64, W.PREC_MIXED])
def test_solve_extrapolated_newton_guess(env, prec):
    """Newton started from 2 u_k - u_{k-1}: the same discrete solution as the oracle's Newton
    from u_k (FP64 per node and per QoI 1e-10; mixed within its stopping test), in fewer
    Newton iterations."""
    torch, mlq = env
    out, refs, mesh = _solve_pair(env, 3, [9, 9, 9], 32, 3, W.QOI_MEAN_ACT_TIME, prec, guess=1)
    out0, _, _ = _solve_pair(env, 3, [9, 9, 9], 32, 3, W.QOI_MEAN_ACT_TIME, prec, guess=0)
    assert int(out["status"].abs().sum()) == 0
    u = out["u"].cpu().numpy()
    q = out["qoi"].cpu().numpy()
    tol = 1e-10 if prec == W.PREC_FP64 else 1e-6
    for b, r in enumerate(refs):
        assert np.abs(u[b] - r["u"]).max() <= tol * np.abs(r["u"]).max()
        assert abs(q[b] - r["mean_act"]) <= tol * abs(r["mean_act"])
    n1 = int(out["iters"][:, 0].sum())
    n0 = int(out0["iters"][:, 0].sum())
    assert n1 < n0, (n1, n0)


def test_solve_mixed_statistics(env):
    torch, mlq = env
    out, refs, mesh = _solve_pair(env, 3, [9, 9, 9], 32, 4, W.QOI_MEAN_ACT_TIME, W.PREC_MIXED)
    assert int(out["status"].abs().sum()) == 0
    q = out["qoi"].cpu().numpy()
    ref = np.array([r["mean_act"] for r in refs])
    assert abs(q.mean() - ref.mean()) <= 1e-6 * abs(ref.mean())
    assert np.abs(q - ref).max() <= 1e-6 * np.abs(ref).max()
    out2, refs2, _ = _solve_pair(env, 2, [17, 17], 32, 4, W.QOI_MEAN_U_FINAL, W.PREC_MIXED)
    q2 = out2["qoi"].cpu().numpy()
    ref2 = np.array([r["mean_u_final"] for r in refs2])
    assert abs(q2.mean() - ref2.mean()) <= 1e-6 * abs(ref2.mean())


def test_isotropic_samples_are_bitwise_identical(env):
    torch, mlq = env
    phys = W.physics(3)
    phys["sigma_t"] = phys["sigma_l"]
    B = 5
    desc, keep = mlq.make_desc(_level(3, [9, 9, 9], 16), phys, qoi=W.QOI_MEAN_ACT_TIME, max_batch=B)
    lv = mlq.Level(desc, keep)
    theta = torch.as_tensor(W.random_angles(9, B, 512), device="cuda")
    out = lv.solve(theta, want_state=True)
    u = out["u"].cpu().numpy()
    for b in range(1, B):
        assert np.array_equal(u[b], u[0])
    q = out["qoi"].cpu().numpy()
    assert np.all(q == q[0])


def test_sample_fields_matches_oracle(env):
    torch, mlq = env
    from oracle import kl
    from oracle.mesh import BoxMesh
    for prec in (W.PREC_FP64, W.PREC_MIXED):
        mesh = BoxMesh([17, 17, 17])
        sl, phi = _kl(mesh, 12)
        th0 = np.linspace(-0.2, 0.3, mesh.n_elems)
        B = 19
        Y = W.mc_normals(2, 1, B, 12)
        desc, keep = mlq.make_desc(_level(3, [17, 17, 17], 8), W.physics(3), n_modes=12, phi=phi, sqrt_lambda=sl,
                                   theta0=th0, prec=prec, max_batch=B)
        lv = mlq.Level(desc, keep)
        th = lv.sample_fields(torch.as_tensor(Y, device="cuda")).double().cpu().numpy()
        ref = kl.field(th0, phi, sl, Y)
        tol = 1e-14 if prec == W.PREC_FP64 else 1e-6
        assert np.abs(th - ref).max() <= tol * np.abs(ref).max()


@pytest.mark.parametrize("n,n_modes,B", [([10, 7, 6], 13, 70), ([9, 9, 9], 150, 5), ([33, 33, 33], 64, 128)])
def test_sample_fields_ragged_shapes(env, n, n_modes, B):
    """The synthesis contraction on shapes that leave partial tiles in every dimension
    (elements, modes past one LDS stage, samples) against eq. (KLlowrank) in FP64."""
    torch, mlq = env
    from oracle import kl
    from oracle.mesh import BoxMesh
    mesh = BoxMesh(n)
    phi = W.random_nodal(41, n_modes, mesh.n_elems).T.copy()
    sl = W.random_nodal(42, 1, n_modes, 0.01, 0.3)[0]
    th0 = W.random_nodal(43, 1, mesh.n_elems, -0.5, 0.5)[0]
    Y = W.mc_normals(3, 0, B, n_modes)
    ref = kl.field(th0, phi, sl, Y)
    for prec in (W.PREC_FP64, W.PREC_MIXED):
        desc, keep = mlq.make_desc(_level(3, n, 8), W.physics(3), n_modes=n_modes, phi=phi, sqrt_lambda=sl,
                                   theta0=th0, prec=prec, max_batch=B)
        lv = mlq.Level(desc, keep)
        th = lv.sample_fields(torch.as_tensor(Y, device="cuda")).double().cpu().numpy()
        # a dot product of n terms summed in precision u errs by at most ~n u sum|terms|;
        # FP32 also rounds the basis, the scaled coordinates and the result once each
        u = 2.0 ** -53 if prec == W.PREC_FP64 else 2.0 ** -24
        bound = (n_modes + 4) * u * (np.abs(th0)[None, :] + (np.abs(phi) @ (sl[:, None] * np.abs(Y))).T)
        assert (np.abs(th - ref) <= bound).all(), (prec, (np.abs(th - ref) / bound).max())


def test_lattice_normals_match_oracle(env):
    torch, mlq = env
    from oracle import qmc
    N, s = 64, 20
    gamma = 0.8 ** np.arange(s)
    z = mlq.cbc(N, s, gamma)
    assert np.array_equal(z, qmc.cbc(N, s, gamma))
    shift = W.lattice_shifts(4, 2, 1, s)[0]
    Y = mlq.lattice_normals(z, shift, N, 0, N).cpu().numpy()
    ref = qmc.lattice_normals(z, N, shift)
    assert np.abs(Y - ref).max() <= 1e-13 * np.abs(ref).max()
    Y2 = mlq.lattice_normals(z, shift, N, 10, 7).cpu().numpy()
    assert np.array_equal(Y2, Y[:, 10:17])


def test_accumulate_matches_host(env):
    torch, mlq = env
    rng = np.random.default_rng(0)
    ff, fc = rng.normal(size=1000), rng.normal(size=1000)
    acc = torch.zeros(3, dtype=torch.float64, device="cuda")
    mlq.accumulate(torch.as_tensor(ff, device="cuda"), torch.as_tensor(fc, device="cuda"), acc)
    mlq.accumulate(torch.as_tensor(ff[:10], device="cuda"), None, acc)
    a = acc.cpu().numpy()
    y = ff - fc
    assert a[0] == 1010
    assert abs(a[1] - (y.sum() + ff[:10].sum())) < 1e-12
    assert abs(a[2] - ((y * y).sum() + (ff[:10] ** 2).sum())) < 1e-10


@pytest.mark.parametrize("dim,n", [(3, [7, 6, 5]), (2, [12, 9])])
def test_kl_modes_match_oracle_full_rank(env, dim, n):
    torch, mlq = env
    from oracle import fem, kl
    from oracle.mesh import BoxMesh
    mesh = BoxMesh(n)
    M = fem.assemble_mass(mesh)
    k = 8
    lam_ref, V_ref = kl.kl_dense(mesh.nodes, M, 0.3, 0.2, k)
    kd = mlq.kl_desc(dim, n, [0.0] * dim, [1.0] * dim, 0.3, 0.2, k, max_rank=mesh.n_nodes, eps=0.0)
    lam, psi, rank, resid = mlq.kl_modes(kd)
    assert rank == mesh.n_nodes and resid < 1e-12
    assert np.allclose(lam, lam_ref, rtol=1e-10, atol=0)
    P = psi.cpu().numpy().T  # (n, k)
    assert np.abs(P.T @ (M @ P) - np.eye(k)).max() < 1e-10
    gaps = np.abs(np.diff(lam_ref)) > 1e-6 * lam_ref[0]
    for j in range(k - 1):
        if gaps[j] and (j == 0 or gaps[j - 1]):  # simple eigenvalue: same mode and sign
            ref = V_ref[:, j] / np.sqrt(lam_ref[j])
            assert np.abs(P[:, j] - ref).max() < 1e-8 * np.abs(ref).max()


def test_kl_truncated_and_transfer_match_oracle(env):
    torch, mlq = env
    from oracle import fem, kl
    from oracle.mesh import BoxMesh
    fine = BoxMesh([17, 17, 17])
    M = fem.assemble_mass(fine)
    k, R = 12, 40
    L, _ = kl.pivoted_cholesky(fine.nodes, 0.3, 0.1, R)
    lam_ref, V_ref = kl.kl_from_cholesky(L, M, k)
    kd = mlq.kl_desc(3, [17] * 3, [0.0] * 3, [1.0] * 3, 0.3, 0.1, k, max_rank=R, eps=0.0)
    lam, psi, rank, resid = mlq.kl_modes(kd)
    assert rank == R
    assert np.allclose(lam, lam_ref, rtol=1e-9, atol=0)
    tr = 0.09 * fine.n_nodes
    assert abs(resid - (tr - np.sum(L * L)) / tr) < 1e-10
    # midpoint transfer of the oracle's own modes to a nested coarse level and to the KL grid itself
    psi_ref = V_ref / np.sqrt(lam_ref)
    psi_d = torch.as_tensor(np.ascontiguousarray(psi_ref.T), device="cuda")
    for nc in (5, 9, 17):
        coarse = BoxMesh([nc] * 3)
        lv = dict(dim=3, n=[nc] * 3, lo=[0.0] * 3, hi=[1.0] * 3)
        phi = mlq.kl_transfer(kd, psi_d, lv).cpu().numpy()
        ref = kl.level_basis(fine, psi_ref, coarse)
        assert np.abs(phi - ref).max() <= 1e-14 * np.abs(ref).max()


@pytest.mark.parametrize("n,mixed", [([9, 9, 9], False), ([23, 11, 7], True), ([50, 13, 6], False)])
def test_lane_layouts_give_identical_operators(env, n, mixed):
    """The operator apply is bitwise the same in both lane layouts of the 3D kernels (each node
    sums its element contributions in one fixed order), and the tuner keeps one of them."""
    torch, mlq = env
    phys = W.physics(3)
    lv = dict(dim=3, n=n, lo=[0.0] * 3, hi=[1.0, 0.8, 0.6], n_steps=16)
    B = 3
    desc, keep = mlq.make_desc(lv, phys, prec=mlq.MLQ_MIXED if mixed else mlq.MLQ_FP64, max_batch=B)
    level = mlq.Level(desc, keep)
    P = int(np.prod([a - 1 for a in n]))
    tdt = torch.float32 if mixed else torch.float64
    th = torch.as_tensor(W.random_angles(5, B, P), dtype=tdt, device="cuda")
    x = torch.as_tensor(W.random_nodal(6, B, level.n_nodes), dtype=tdt, device="cuda")
    d = torch.as_tensor(W.random_nodal(7, B, level.n_nodes, -0.05, 0.14), dtype=tdt, device="cuda")
    ys = []
    for lx in (8, 16):
        level.set_lane_layout(lx)
        ys.append(level.apply(th, x, d).cpu().numpy())
    assert np.array_equal(ys[0], ys[1])
    times = level.tune_lane_layout()
    assert set(times) == {8, 16} and level.lanes_x in (8, 16)
    assert np.array_equal(level.apply(th, x, d).cpu().numpy(), ys[0])
    with pytest.raises(mlq.MlqError):
        level.set_lane_layout(32)


def test_lane_layout_solves_agree(env):
    """A solve in either layout agrees within the stopping test (the fused projections are
    summed over other partitions)."""
    torch, mlq = env
    phys = W.physics(3)
    lv = dict(dim=3, n=[17, 17, 17], lo=[0.0] * 3, hi=[1.0] * 3, n_steps=16)
    desc, keep = mlq.make_desc(lv, phys, qoi=mlq.MLQ_QOI_MEAN_ACT_TIME, max_batch=2)
    level = mlq.Level(desc, keep)
    th = torch.as_tensor(W.random_angles(9, 2, 16 ** 3), device="cuda")
    q = []
    for lx in (8, 16):
        level.set_lane_layout(lx)
        out = level.solve(th, want_state=True)
        q.append((out["qoi"].cpu().numpy(), out["u"].cpu().numpy()))
    assert np.abs(q[0][0] - q[1][0]).max() <= 1e-10 * np.abs(q[0][0]).max()
    assert np.abs(q[0][1] - q[1][1]).max() <= 1e-10 * np.abs(q[0][1]).max()
