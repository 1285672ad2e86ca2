"""GPU parity of the isotropic scalar conductivity model (G = v I per element, the paper's
cube model of Section 5.1) and of the squared-exponential KL kernel against the oracle.

Bars as elsewhere: FP64 apply within 3e-14 of the row scale, FP32 within 2e-6; FP64 solves
within 1e-10 relative per node and per QoI; KL eigenvalues 1e-10, simple modes 1e-8."""
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


def _level(n, steps, hi=None):
    return dict(dim=3, n=list(n), lo=[0.0] * 3, hi=hi or [1.0] * 3, n_steps=steps)


def _positive_field(seed, B, P, mean=3.325e-3, amp=0.3):
    return mean * (1.0 + amp * (2.0 * W.random_nodal(seed, B, P, 0.0, 1.0) - 1.0))


@pytest.mark.parametrize("n,mixed", [([9, 7, 5], False), ([9, 7, 5], True), ([53, 6, 7], False),
                                     ([61, 5, 9], True)])
def test_iso_apply_matches_assembled_jacobian(env, n, mixed):
    torch, mlq = env
    from oracle import fem
    from oracle.mesh import BoxMesh
    phys = W.physics(3)
    lv = _level(n, 16, hi=[1.0, 0.8, 1.3])
    B = 3
    desc, keep = mlq.make_desc(lv, phys, prec=mlq.MLQ_MIXED if mixed else mlq.MLQ_FP64, max_batch=B,
                               diffusion=mlq.MLQ_DIFF_ISO)
    level = mlq.Level(desc, keep)
    mesh = BoxMesh(n, hi=lv["hi"])
    dt = phys["t_end"] / 16
    v = _positive_field(3, B, mesh.n_elems)
    x = W.random_nodal(4, B, mesh.n_nodes)
    dv = W.random_nodal(5, B, mesh.n_nodes, -0.05, 0.14)
    tdt = torch.float32 if mixed else torch.float64
    v_d, x_d, d_d = (torch.as_tensor(a, dtype=tdt, device="cuda") for a in (v, x, dv))
    y = level.apply(v_d, x_d, d_d).double().cpu().numpy()
    for b in range(B):
        vb, xb, db = (a[b].double().cpu().numpy() for a in (v_d, x_d, d_d))
        M, K = fem.assemble(mesh, fem.conductivity_iso(vb, 3))
        ref = M @ ((1.0 + db) * xb) + 0.5 * dt * (K @ xb)
        scale = abs(M) @ np.abs((1.0 + db) * xb) + 0.5 * dt * (abs(K) @ np.abs(xb))
        tol = (2e-6 if mixed else 3e-14) * scale.max()
        assert np.abs(y[b] - ref).max() <= tol, (b, np.abs(y[b] - ref).max() / scale.max())


def test_iso_solve_fp64_matches_oracle(env):
    torch, mlq = env
    from oracle import fem, stepper
    from oracle.mesh import BoxMesh
    phys = W.physics(3)
    n, steps, B = [9, 9, 9], 32, 3
    desc, keep = mlq.make_desc(_level(n, steps), phys, qoi=mlq.MLQ_QOI_MEAN_ACT_TIME, newton_tol=1e-13,
                               max_batch=B, diffusion=mlq.MLQ_DIFF_ISO, newton_guess=mlq.MLQ_GUESS_EXTRAPOLATE)
    level = mlq.Level(desc, keep)
    mesh = BoxMesh(n)
    v = _positive_field(8, B, mesh.n_elems)
    out = level.solve(torch.as_tensor(v, device="cuda"), want_state=True)
    assert int(out["status"].abs().sum()) == 0
    u = out["u"].cpu().numpy()
    q = out["qoi"].cpu().numpy()
    for b in range(B):
        r = stepper.solve(mesh, fem.conductivity_iso(v[b], 3), phys, steps, tol=1e-13)
        assert np.abs(u[b] - r["u"]).max() <= 1e-10 * np.abs(r["u"]).max()
        assert abs(q[b] - r["mean_act"]) <= 1e-10 * abs(r["mean_act"])


@pytest.mark.parametrize("mixed", [False, True])
def test_iso_floor_clips_the_field(env, mixed):
    """A field that crosses the lower bound: G = max(v, sigma_t) I element by element (values
    down to -0.5 E[V] and up to 2.5 E[V], the floor at 0.1 E[V])."""
    torch, mlq = env
    from oracle import fem
    from oracle.mesh import BoxMesh
    phys = W.physics(3)
    phys["sigma_t"] = 0.1 * 3.325e-3
    n = [17, 9, 6]
    lv = _level(n, 16, hi=[1.0, 0.6, 0.4])
    B = 2
    desc, keep = mlq.make_desc(lv, phys, prec=mlq.MLQ_MIXED if mixed else mlq.MLQ_FP64, max_batch=B,
                               diffusion=mlq.MLQ_DIFF_ISO)
    level = mlq.Level(desc, keep)
    mesh = BoxMesh(n, hi=lv["hi"])
    dt = phys["t_end"] / 16
    v = _positive_field(13, B, mesh.n_elems, amp=1.5)
    assert (v < phys["sigma_t"]).mean() > 0.1
    x = W.random_nodal(14, B, mesh.n_nodes)
    dv = W.random_nodal(15, B, mesh.n_nodes, -0.05, 0.14)
    tdt = torch.float32 if mixed else torch.float64
    v_d, x_d, d_d = (torch.as_tensor(a, dtype=tdt, device="cuda") for a in (v, x, dv))
    y = level.apply(v_d, x_d, d_d).double().cpu().numpy()
    for b in range(B):
        vb, xb, db = (a[b].double().cpu().numpy() for a in (v_d, x_d, d_d))
        M, K = fem.assemble(mesh, fem.conductivity_iso(vb, 3, phys["sigma_t"]))
        ref = M @ ((1.0 + db) * xb) + 0.5 * dt * (K @ xb)
        scale = abs(M) @ np.abs((1.0 + db) * xb) + 0.5 * dt * (abs(K) @ np.abs(xb))
        tol = (2e-6 if mixed else 3e-14) * scale.max()
        assert np.abs(y[b] - ref).max() <= tol, (b, np.abs(y[b] - ref).max() / scale.max())


def test_c2i_pipeline_small_matches_oracle(env):
    """The cube model end to end at small size through the driver: squared-exponential KL
    relative to E[V] with uniform coordinates, midpoint transfer, v = E[V] + W bounded below,
    nested box levels, MLMC estimator eq. (StandardML), against the oracle's own pipeline (FP64).
    The box is not a cube, so the KL eigenvalues are simple and the modes comparable; the
    standard deviation is raised so that the floor is reached."""
    torch, mlq = env
    from oracle import estimators, run
    from paper_2105_02007_amd.driver import ConfigRunner
    cfg = W.config("c2i")
    hi = [1.0, 0.8, 1.3]
    cfg["levels"] = [dict(dim=3, n=[n] * 3, lo=[0.0] * 3, hi=hi, n_steps=m) for n, m in zip([5, 9], [8, 16])]
    cfg["kl"].update(n_modes=5, grid_level=1, std=1.5)
    cfg["sampling"]["n_per_level"] = [4, 2]
    M = cfg["kl"]["n_modes"]
    meshes = run.level_meshes(cfg)
    factor = meshes[-1].n_nodes // M  # near-full-rank Cholesky on both sides, same rank
    runner = ConfigRunner(cfg, prec=W.PREC_FP64, kl_rank_factor=factor, kl_eps=0.0, kl_method="cholesky")
    Ys = [W.mc_uniforms(cfg["seed"], l, n, M) for l, n in enumerate(cfg["sampling"]["n_per_level"])]
    res = runner.run_mlmc([torch.as_tensor(Y, device="cuda") for Y in Ys])
    B = run.kl_basis(cfg, meshes, max_rank=factor * M, eps=0.0)
    ph = cfg["physics"]
    floor_hit = False

    def qois(l, Y):
        nonlocal floor_hit
        th = run.sample_theta(B["phi"][l], B["sqrt_lam"], Y, run.level_theta0(cfg, meshes[l]))
        floor_hit |= bool((th < ph["sigma_t"]).any())
        return np.array([run.qoi_of(run.solve_theta(meshes[l], th[b], ph, cfg["levels"][l]["n_steps"],
                                                    model="iso"), cfg["qoi"]) for b in range(th.shape[0])])
    ff = [qois(l, Ys[l]) for l in range(2)]
    fc = [None, qois(0, Ys[1])]
    assert floor_hit
    for l in range(2):
        assert np.abs(res["f_fine"][l] - ff[l]).max() <= 1e-10 * np.abs(ff[l]).max(), l
    assert np.abs(res["f_coarse"][1] - fc[1]).max() <= 1e-10 * np.abs(fc[1]).max()
    est = estimators.standard_ml(ff, fc)[0]
    assert abs(res["estimate"] - est) <= 1e-10 * abs(est)


@pytest.mark.parametrize("mixed", [False, True])
def test_iso_model_on_tetrahedra_matches_assembled_jacobian(env, mixed):
    """The isotropic model on a shell (the idealised-ventricle analogue): G = max(v, sigma_t) I
    per tetrahedron, with part of the field below the floor."""
    torch, mlq = env
    from oracle import fem
    from oracle.tetfem import TetMesh
    from workloads import tetshell
    xyz, tets, ec, el, _ = tetshell.shell_mesh((3, 8, 16), seed=5)
    mesh_d = dict(xyz=xyz, tets=tets, e_circ=ec, e_long=el)
    phys = W.physics(3)
    c, r = tetshell.stimulus_ball(0.3)
    phys.update(stim_center=c.tolist(), stim_radius=float(r), sigma_t=0.1 * 3.325e-3)
    steps, B = 16, 2
    desc, keep = mlq.make_desc(dict(kind="tet", dim=3, n_steps=steps, mesh=mesh_d), phys,
                               prec=mlq.MLQ_MIXED if mixed else mlq.MLQ_FP64, max_batch=B, diffusion=mlq.MLQ_DIFF_ISO)
    lv = mlq.Level(desc, keep)
    mesh = TetMesh(xyz, tets)
    dt = phys["t_end"] / steps
    v = _positive_field(41, B, mesh.n_elems, amp=1.5)
    assert (v < phys["sigma_t"]).any()
    x = W.random_nodal(42, B, mesh.n_nodes)
    dv = W.random_nodal(43, B, mesh.n_nodes, -0.05, 0.14)
    tdt = torch.float32 if mixed else torch.float64
    v_d, x_d, d_d = (torch.as_tensor(a, dtype=tdt, device="cuda") for a in (v, x, dv))
    y = lv.apply(v_d, x_d, d_d).double().cpu().numpy()
    for b in range(B):
        vb, xb, db = (a[b].double().cpu().numpy() for a in (v_d, x_d, d_d))
        M, K = mesh.assemble(fem.conductivity_iso(vb, 3, phys["sigma_t"]))
        ref = M @ ((1.0 + db) * xb) + 0.5 * dt * (K @ xb)
        scale = abs(M) @ np.abs((1.0 + db) * xb) + 0.5 * dt * (abs(K) @ np.abs(xb))
        tol = (2e-6 if mixed else 1e-13) * scale.max()
        assert np.abs(y[b] - ref).max() <= tol, (b, np.abs(y[b] - ref).max() / scale.max())


@pytest.mark.parametrize("n", [[7, 6, 5], [9, 8, 1]])
def test_kl_squared_exponential_matches_oracle(env, n):
    torch, mlq = env
    from oracle import fem, kl
    from oracle.mesh import BoxMesh
    dim = 3 if n[2] > 1 else 2
    n = n[:dim]
    mesh = BoxMesh(n)
    M = fem.assemble_mass(mesh)
    k = 8
    lam_ref, V_ref = kl.kl_dense(mesh.nodes, M, 0.3, 0.25, k, kernel="sqexp")
    # full rank (the factorisation stops early only if a pivot's remaining variance is zero)
    kd = mlq.kl_desc(dim, n, [0.0] * dim, [1.0] * dim, 0.3, 0.25, k, max_rank=mesh.n_nodes, eps=0.0,
                     cov_kernel=mlq.MLQ_COV_SQEXP)
    lam, psi, rank, resid = mlq.kl_modes(kd)
    assert resid < 1e-12
    assert np.allclose(lam, lam_ref, rtol=1e-9, atol=0)
    P = psi.cpu().numpy().T
    assert np.abs(P.T @ (M @ P) - np.eye(k)).max() < 1e-9
    gaps = np.abs(np.diff(lam_ref)) > 1e-3 * lam_ref[0]
    for j in range(k - 1):
        if gaps[j] and (j == 0 or gaps[j - 1]):
            ref = V_ref[:, j] / np.sqrt(lam_ref[j])
            assert np.abs(P[:, j] - ref).max() < 1e-5 * np.abs(ref).max()


@pytest.mark.parametrize("n,kernel,corr", [([17, 17, 17], "sqexp", 0.25), ([13, 11, 9], "sqexp", 0.5)])
def test_stochastic_dimension_from_tolerance_matches_oracle(env, n, kernel, corr):
    """n_modes = 0 asks the library for the rank at which the pivoted Cholesky meets the
    truncation tolerance (the paper's way of fixing M); bit-exact integer against the oracle's
    factorisation, and 65 on the paper's cube set-up (which reports M = 66)."""
    torch, mlq = env
    from oracle import kl
    from oracle.mesh import BoxMesh
    mesh = BoxMesh(n)
    cov = mlq.MLQ_COV_SQEXP if kernel == "sqexp" else mlq.MLQ_COV_EXP
    kd = mlq.kl_desc(3, n, [0.0] * 3, [1.0] * 3, 0.3, corr, 8, max_rank=300, eps=1e-2, cov_kernel=cov)
    rank, resid = mlq.kl_dimension(kd)
    L, _ = kl.pivoted_cholesky(mesh.nodes, 0.3, corr, 300, eps=1e-2, kernel=kernel)
    assert rank == L.shape[1] and resid <= 1e-2
    assert abs(resid - (1.0 - (L ** 2).sum() / (0.09 * mesh.n_nodes))) <= 1e-10
    if corr == 0.25:  # the cube of Section 5.1
        assert rank == 65
    assert kd.n_modes == 8


def test_driver_fixes_the_dimension_from_the_tolerance(env):
    """A workload with n_modes = 0 takes M from the truncation tolerance."""
    torch, mlq = env
    from oracle import kl
    from oracle.mesh import BoxMesh
    from paper_2105_02007_amd.driver import ConfigRunner
    cfg = W.scaled_config("c2i", nodes=[5, 9], steps=[4, 8], n_per_level=[2, 1], n_modes=0)
    runner = ConfigRunner(cfg, prec=W.PREC_FP64)
    L, _ = kl.pivoted_cholesky(BoxMesh([9, 9, 9]).nodes, 0.3 * cfg["kl"]["mean"], 0.25, 300, eps=1e-2,
                               kernel="sqexp")
    assert runner.n_modes == L.shape[1] == runner.kd.n_modes
    assert runner.levels[0].desc.n_modes == runner.n_modes
