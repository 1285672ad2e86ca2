"""The benchmarked estimators end to end through the driver against the oracle's pipeline, at a
size the oracle finishes in seconds: the MLQMC workload c4 (fibre-angle model with the exponential
kernel, randomly shifted rank-1 lattices with Gaussian coordinates, eq. (StandardML) over shifts)
in FP64 and in mixed precision, and the MLMC workload c2 (independent Monte Carlo normals per level)
in FP64.  The box is 48 elements long, so the finest level runs the 16-lane layout of the 3D kernels
with the Gram-Schmidt projections fused into the apply; three nested levels, three shifts.

Bars: FP64 per sample, level means and estimate within 1e-10 relative of the oracle; mixed
precision (FP32 KL synthesis and Krylov, FP64 residual) level means and estimate within 1e-6
relative of the FP64 oracle.  The activation-time QoI is censored at T, so the messages also give
the mixed error relative to the informative part T - QoI."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

HI = [0.6, 0.1, 0.08]
NODES = [[13, 2, 2], [25, 3, 3], [49, 5, 5]]
STEPS = [8, 16, 32]
M = 25  # divides the 1225 KL-grid nodes: both sides factorise at full rank


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2105_02007_amd import mlq
    return torch, mlq


def _cfg(name, n_per_level, n_shifts=None):
    cfg = W.config(name)
    cfg["levels"] = [dict(dim=3, n=list(n), lo=[0.0] * 3, hi=list(HI), n_steps=m) for n, m in zip(NODES, STEPS)]
    cfg["kl"].update(n_modes=M, grid_level=len(NODES) - 1)
    cfg["sampling"]["n_per_level"] = list(n_per_level)
    if n_shifts is not None:
        cfg["sampling"]["n_shifts"] = n_shifts
    return cfg


def _oracle_qois(cfg, B, l, Y):
    from oracle import run
    th = run.sample_theta(B["phi"][l], B["sqrt_lam"], Y, run.level_theta0(cfg, B["meshes"][l]))
    return np.array([run.qoi_of(run.solve_theta(B["meshes"][l], th[b], cfg["physics"], cfg["levels"][l]["n_steps"]),
                                cfg["qoi"]) for b in range(th.shape[0])])


def _oracle_basis(cfg):
    from oracle import run
    meshes = run.level_meshes(cfg)
    n = meshes[-1].n_nodes
    B = run.kl_basis(cfg, meshes, max_rank=n, eps=0.0)  # full rank: the exact eigenpairs
    B["meshes"] = meshes
    return B


@pytest.fixture(scope="module")
def c4_oracle():
    """The oracle's MLQMC pipeline: its own KL, CBC vectors from its own eigenvalues, shifted lattice
    normals, solves; f[l][s] per level and shift."""
    from oracle import qmc
    cfg = _cfg("c4", [4, 2, 1], n_shifts=3)
    B = _oracle_basis(cfg)
    S = 3
    shifts = [W.lattice_shifts(cfg["seed"], l, S, M) for l in range(3)]
    ff, fc = [], []
    for l, N in enumerate(cfg["sampling"]["n_per_level"]):
        z = qmc.cbc(N, M, B["lam"] / B["lam"][0])
        Ys = [qmc.lattice_normals(z, N, shifts[l][s]) for s in range(S)]
        ff.append([_oracle_qois(cfg, B, l, Y) for Y in Ys])
        fc.append([_oracle_qois(cfg, B, l - 1, Y) for Y in Ys] if l > 0 else [None] * S)
    return cfg, shifts, ff, fc


def _run_c4(env, cfg, shifts, prec):
    from paper_2105_02007_amd.driver import ConfigRunner
    n = int(np.prod(NODES[-1]))
    runner = ConfigRunner(cfg, prec=prec, kl_rank_factor=n // M, kl_eps=0.0, kl_method="cholesky", tune_layout=False)
    assert runner.levels[-1].desc.n[0] >= 48
    return runner.run_mlqmc(shifts)


def test_c4_mlqmc_fp64_matches_oracle(env, c4_oracle):
    from oracle import estimators
    cfg, shifts, ff, fc = c4_oracle
    res = _run_c4(env, cfg, shifts, W.PREC_FP64)
    for l in range(3):
        ref = np.concatenate(ff[l])  # shift-major
        assert np.abs(res["f_fine"][l] - ref).max() <= 1e-10 * np.abs(ref).max(), l
        if l > 0:
            ref = np.concatenate(fc[l])
            assert np.abs(res["f_coarse"][l] - ref).max() <= 1e-10 * np.abs(ref).max(), l
    est, rmse, means = estimators.standard_mlqmc(ff, fc)
    assert abs(res["estimate"] - est) <= 1e-10 * abs(est)
    assert abs(res["rmse"] - rmse) <= 1e-10 * abs(est)
    for l in range(3):
        assert abs(res["level_mean"][l] - means[l]) <= 1e-10 * abs(est), l
    assert rmse > 0 and abs(means[1]) > 0


def test_c4_mlqmc_mixed_matches_oracle(env, c4_oracle):
    from oracle import estimators
    cfg, shifts, ff, fc = c4_oracle
    res = _run_c4(env, cfg, shifts, W.PREC_MIXED)
    est, rmse, means = estimators.standard_mlqmc(ff, fc)
    T = cfg["physics"]["t_end"]
    err = abs(res["estimate"] - est)
    assert err <= 1e-6 * abs(est), (err / abs(est), err / abs(T - est))
    for l in range(3):
        e = abs(res["level_mean"][l] - means[l])
        assert e <= 1e-6 * abs(means[l]), (l, e / abs(means[l]), e / abs(T - est))
    assert abs(res["rmse"] - rmse) <= 1e-6 * rmse
    # per sample, for the record: FP32 fields and Krylov, FP64 residual
    worst = max(np.abs(res["f_fine"][l] - np.concatenate(ff[l])).max() for l in range(3))
    assert worst <= 1e-6 * T


def test_c2_mlmc_fp64_matches_oracle(env):
    from oracle import estimators
    from paper_2105_02007_amd.driver import ConfigRunner
    torch, mlq = env
    cfg = _cfg("c2", [6, 3, 2])
    B = _oracle_basis(cfg)
    Ys = [W.mc_normals(cfg["seed"], l, N, M) for l, N in enumerate(cfg["sampling"]["n_per_level"])]
    n = int(np.prod(NODES[-1]))
    runner = ConfigRunner(cfg, prec=W.PREC_FP64, kl_rank_factor=n // M, kl_eps=0.0, kl_method="cholesky", tune_layout=False)
    res = runner.run_mlmc([torch.as_tensor(Y, device="cuda") for Y in Ys])
    ff = [_oracle_qois(cfg, B, l, Ys[l]) for l in range(3)]
    fc = [None] + [_oracle_qois(cfg, B, l - 1, Ys[l]) for l in (1, 2)]
    for l in range(3):
        assert np.abs(res["f_fine"][l] - ff[l]).max() <= 1e-10 * np.abs(ff[l]).max(), l
        if l > 0:
            assert np.abs(res["f_coarse"][l] - fc[l]).max() <= 1e-10 * np.abs(fc[l]).max(), l
    est, rmse, means, _ = estimators.standard_ml(ff, fc)
    assert abs(res["estimate"] - est) <= 1e-10 * abs(est)
    assert abs(res["rmse"] - rmse) <= 1e-10 * abs(est)
    assert rmse > 0
