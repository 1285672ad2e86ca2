"""GPU parity of the Halton rule (the paper's QMC points) and of MLQMC with shifted Halton
points on the cube model against the oracle.

Bars: the uniform coordinates are bit-exact (the radical inverse is the exact rational rounded
once on both sides, the shift and 2x - 1 are single IEEE operations); the Gaussian map within
1e-13 of the largest coordinate (two implementations of Phi^-1); QoIs and the estimate within
1e-10 relative (FP64)."""
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


@pytest.mark.parametrize("s,first,count", [(20, 1, 50), (3, 0, 729), (1024, 1, 3), (40, 2 ** 32 - 5, 5)])
def test_halton_matches_oracle(env, s, first, count):
    torch, mlq = env
    from oracle import qmc
    Y = mlq.halton(s, first, count, None, uniform=True).cpu().numpy()
    assert np.array_equal(Y, qmc.halton_coordinates(s, first, count, None, uniform=True))
    shift = W.lattice_shifts(9, 0, 1, s)[0]
    Ys = mlq.halton(s, first, count, shift, uniform=True).cpu().numpy()
    assert np.array_equal(Ys, qmc.halton_coordinates(s, first, count, shift, uniform=True))
    Yn = mlq.halton(s, first, count, shift, uniform=False).cpu().numpy()
    ref = qmc.halton_coordinates(s, first, count, shift, uniform=False)
    assert np.abs(Yn - ref).max() <= 1e-13 * np.abs(ref).max()


def test_halton_subranges_are_consistent(env):
    torch, mlq = env
    shift = W.lattice_shifts(9, 1, 1, 7)[0]
    Y = mlq.halton(7, 1, 100, shift).cpu().numpy()
    assert np.array_equal(mlq.halton(7, 31, 9, shift).cpu().numpy(), Y[:, 30:39])
    assert mlq.halton(7, 1, 0, shift).shape == (7, 0)


def test_c4i_pipeline_small_matches_oracle(env):
    """MLQMC with randomly shifted Halton points on the cube model through the driver (library
    KL relative to E[V], uniform coordinates, clamped isotropic solves, eq. (StandardML) over
    shifts) against the oracle's pipeline, FP64, on a non-cubic box (simple KL eigenvalues)."""
    torch, mlq = env
    from oracle import estimators, qmc, run
    from paper_2105_02007_amd.driver import ConfigRunner
    cfg = W.config("c4i")
    hi = [1.0, 0.8, 1.3]
    cfg["levels"] = [dict(dim=3, n=[n] * 3, lo=[0.0] * 3, hi=hi, n_steps=m) for n, m in zip([5, 9], [8, 16])]
    cfg["kl"].update(n_modes=5, grid_level=1, std=1.5)
    cfg["sampling"].update(n_per_level=[4, 2], n_shifts=3)
    cfg["prec"] = W.PREC_FP64
    M, S = cfg["kl"]["n_modes"], 3
    meshes = run.level_meshes(cfg)
    factor = meshes[-1].n_nodes // M
    runner = ConfigRunner(cfg, prec=W.PREC_FP64, kl_rank_factor=factor, kl_eps=0.0, kl_method="cholesky")
    shifts = [W.lattice_shifts(cfg["seed"], l, S, M) for l in range(2)]
    res = runner.run_mlqmc(shifts)
    B = run.kl_basis(cfg, meshes, max_rank=factor * M, eps=0.0)
    ph = cfg["physics"]

    def qois(l, Y):
        th = run.sample_theta(B["phi"][l], B["sqrt_lam"], Y, run.level_theta0(cfg, meshes[l]))
        return [run.qoi_of(run.solve_theta(meshes[l], th[b], ph, cfg["levels"][l]["n_steps"], model="iso"),
                           cfg["qoi"]) for b in range(th.shape[0])]
    ff, fc = [], [None]
    for l, N in enumerate(cfg["sampling"]["n_per_level"]):
        Ys = [qmc.halton_coordinates(M, 1, N, shifts[l][s], uniform=True) for s in range(S)]
        ff.append([qois(l, Y) for Y in Ys])
        if l > 0:
            fc.append([qois(l - 1, Y) for Y in Ys])
    for l in range(2):
        ref = np.concatenate(ff[l])  # shift-major
        assert np.abs(res["f_fine"][l] - ref).max() <= 1e-10 * np.abs(ref).max(), l
    ref = np.concatenate(fc[1])
    assert np.abs(res["f_coarse"][1] - ref).max() <= 1e-10 * np.abs(ref).max()
    est, rmse, _ = estimators.standard_mlqmc(ff, fc)
    assert abs(res["estimate"] - est) <= 1e-10 * abs(est)
    assert abs(res["rmse"] - rmse) <= 1e-9 * abs(est)


def test_lattice_uniform_coordinates_match_oracle(env):
    """Shifted lattice points in the uniform map y = 2x - 1 (bit-exact: the same exact fraction,
    one rounded addition of the shift, an exact doubling and one rounded subtraction), and the
    driver's QMC points of a uniform-coordinate workload with the lattice rule."""
    torch, mlq = env
    from oracle import qmc
    from paper_2105_02007_amd.driver import ConfigRunner
    N, s = 61, 12
    gamma = 0.7 ** np.arange(s)
    z = qmc.cbc(N, s, gamma)
    shift = W.lattice_shifts(3, 0, 1, s)[0]
    Y = mlq.lattice_points(z, shift, N, 0, N, uniform=True).cpu().numpy()
    assert np.array_equal(Y, qmc.lattice_uniforms(z, N, shift))
    Yn = mlq.lattice_points(z, shift, N, 0, N, uniform=False).cpu().numpy()
    assert np.array_equal(Yn, mlq.lattice_normals(z, shift, N, 0, N).cpu().numpy())
    cfg = W.scaled_config("c4i", nodes=[5, 9], steps=[4, 8], n_per_level=[8, 2], n_modes=5)
    cfg["sampling"].update(rule="lattice", n_shifts=2)
    cfg["prec"] = W.PREC_FP64
    runner = ConfigRunner(cfg, prec=W.PREC_FP64)
    shifts = W.lattice_shifts(cfg["seed"], 0, 2, 5)
    P = runner.qmc_points(0, shifts).cpu().numpy()
    zr = qmc.cbc(8, 5, runner.lam / runner.lam[0])
    ref = np.concatenate([qmc.lattice_uniforms(zr, 8, shifts[k]) for k in range(2)], axis=1)
    assert np.array_equal(P, ref)
    res = runner.run_mlqmc([W.lattice_shifts(cfg["seed"], l, 2, 5) for l in range(2)])
    assert np.isfinite(res["estimate"]) and res["rmse"] >= 0
