"""Synthetic workloads and seeded random draws shared by the oracle and the HIP path.

This module is deliberately free of the method's arithmetic: it only holds
workload descriptions (mesh sizes, time steps, physical constants printed in
the paper, KL settings, sample plans) and seeded random numbers (standard
normals for Monte Carlo, uniform shifts for randomly shifted lattice rules,
random test fields).  Both the oracle under ``oracle/`` and the HIP path read
their inputs from here; neither imports the other.

Physical constants are those of the paper's experiment set-up (Section 5.1,
"Parameters for the monodomain equation"; mean / perpendicular diffusion from
the KL parameter list of Section 5.1).  The end time T = 0.32 is not printed;
it is the value for which every row of the cube and heart level tables
satisfies DOF = (spatial unknowns) * T / dt.
"""
from __future__ import annotations

import copy
import numpy as np

from . import tetshell

# --- physical constants (Section 5.1) --------------------------------------
ALPHA = 1.4e-3          # mV^-2 ms^-1
U_REST = 0.0            # mV
U_TH = 28.0             # mV
U_PEAK = 115.0          # mV
SIGMA_L = 3.325e-3      # mm^2/ms, along the fibre (mean diffusion of Section 5.1)
SIGMA_T = 1.625e-3      # mm^2/ms, across the fibre (g of eq. (AdmV), heart set-up)
T_END = 0.32            # ms, implied by the level tables of Section 5

# stimulus: corner box [0, 0.1]^d during the first 2 % of [0, T]; the amplitude
# is chosen so that the time integral of the stimulus equals u_peak (reading S2:
# the printed amplitude is a potential in mV, the PDE needs a rate in mV/ms)
STIM_FRAC_T = 0.02
STIM_BOX = 0.1

QOI_MEAN_U_FINAL = 0
QOI_MEAN_ACT_TIME = 1

PREC_FP64 = 0
PREC_MIXED = 1


def physics(dim: int) -> dict:
    """Model parameters shared by every configuration."""
    t_off = STIM_FRAC_T * T_END
    return dict(
        alpha=ALPHA, u_rest=U_REST, u_th=U_TH, u_peak=U_PEAK,
        sigma_l=SIGMA_L, sigma_t=SIGMA_T, t_end=T_END,
        stim_lo=[0.0] * dim, stim_hi=[STIM_BOX] * dim,
        stim_t_on=0.0, stim_t_off=t_off, stim_amp=U_PEAK / t_off,
    )


def _box_levels(dim, nodes, steps):
    return [dict(dim=dim, n=[int(n)] * dim, lo=[0.0] * dim, hi=[1.0] * dim,
                 n_steps=int(m)) for n, m in zip(nodes, steps)]


def _tet_levels(cells, steps, seed):
    """Non-nested tetrahedral shells (workloads/tetshell.py), one mesh seed per level."""
    return [dict(kind="tet", dim=3, cells=list(c), mesh_seed=int(100 * seed + l), n_steps=int(m))
            for l, (c, m) in enumerate(zip(cells, steps))]


def tet_mesh(level: dict) -> dict:
    """Vertices, tetrahedra, fibre frame and rule-based base angle of a tetrahedral level."""
    xyz, tets, ec, el, th0 = tetshell.shell_mesh(level["cells"], level["mesh_seed"])
    return dict(xyz=xyz, tets=tets, e_circ=ec, e_long=el, theta0=th0)


# the three non-nested shells (n_mu, n_nu, n_phi cells; vertices (n_mu + 1)(n_nu + 1) n_phi):
# 24,960 / 198,702 / 1,602,352 vertices, the configured 25k / 200k / 1.6M, with about the same
# cell aspect on every level
SHELL_CELLS = [(4, 38, 128), (8, 82, 266), (16, 171, 548)]

# --- the five synthetic workloads -------------------------------------------
CONFIGS = {
    "c1": dict(
        name="c1", title="plain FP64 MC, 2D unit square, Q1 33x33, 64 steps, 16 samples",
        dim=2, levels=_box_levels(2, [33], [64]),
        kl=dict(n_modes=16, corr_len=0.2, std=0.3, grid_level=0, method="exact"),
        sampling=dict(kind="mc", n_per_level=[16]),
        qoi=QOI_MEAN_U_FINAL, prec=PREC_FP64, seed=1),
    "c2": dict(
        name="c2", title="FP64 batched MLMC, 3D cube, Q1 9^3..65^3, 32..256 steps",
        dim=3, levels=_box_levels(3, [9, 17, 33, 65], [32, 64, 128, 256]),
        kl=dict(n_modes=64, corr_len=0.1, std=0.3, grid_level=3, method="exact"),
        sampling=dict(kind="mlmc", n_per_level=[2048, 512, 128, 32]),
        qoi=QOI_MEAN_ACT_TIME, prec=PREC_FP64, seed=2),
    "c3": dict(
        name="c3", title="mixed single level, 3D cube, Q1 129^3, 512 steps, 64 lattice points",
        dim=3, levels=_box_levels(3, [129], [512]),
        kl=dict(n_modes=128, corr_len=0.1, std=0.3, grid_level=0, method="exact"),
        sampling=dict(kind="qmc", n_per_level=[64], n_shifts=1),
        qoi=QOI_MEAN_ACT_TIME, prec=PREC_MIXED, seed=3),
    "c4": dict(
        name="c4", title="batched uneven MLQMC, 3D cube, Q1 9^3..129^3, 32..512 steps, 16 shifts",
        dim=3, levels=_box_levels(3, [9, 17, 33, 65, 129], [32, 64, 128, 256, 512]),
        kl=dict(n_modes=128, corr_len=0.1, std=0.3, grid_level=4, method="exact"),
        sampling=dict(kind="mlqmc", n_per_level=[256, 64, 16, 4, 1], n_shifts=16),
        qoi=QOI_MEAN_ACT_TIME, prec=PREC_MIXED, seed=4),
    # combination form eq. (PimpedML): Q_0, Q_1, Q_2 with 16, 64, 256 nested Monte Carlo
    # points (prefixes of one stream) on the fine, middle and coarse shell
    "c5": dict(
        name="c5", title="non-nested multilevel, prolate-ellipsoidal shell, P1 tetrahedra 25k/199k/1.6M "
                         "vertices, 512 steps, 256-mode KL, combination estimator",
        dim=3, levels=_tet_levels(SHELL_CELLS, [512, 512, 512], 5),
        kl=dict(n_modes=256, corr_len=0.1 * tetshell.LONG_AXIS, std=0.3, grid_level=2),
        sampling=dict(kind="combination", n_per_level=[16, 64, 256]),
        qoi=QOI_MEAN_ACT_TIME, prec=PREC_MIXED, seed=5),
    # the paper's cube model (Section 5.1): isotropic G = v I with v = E[V] (1 + W), W a KL field
    # with the squared-exponential covariance 0.3^2 exp(-|x - x'|^2 / 0.25) relative to
    # E[V] = 3.325e-3, 66 modes with uniform coordinates (modes scaled by sqrt(3 lambda)),
    # bounded below by 0.1 E[V]; the nested levels and sample plan of c2
    "c2i": dict(
        name="c2i", title="the paper's cube model: isotropic random scalar diffusion, MLMC 9^3..65^3",
        dim=3, levels=_box_levels(3, [9, 17, 33, 65], [32, 64, 128, 256]),
        kl=dict(n_modes=66, corr_len=0.25, std=0.3, grid_level=3, kernel="sqexp", variables="uniform",
                mean=SIGMA_L, floor=0.1),
        model="iso",
        sampling=dict(kind="mlmc", n_per_level=[2048, 512, 128, 32]),
        qoi=QOI_MEAN_ACT_TIME, prec=PREC_FP64, seed=7),
    # the cube model with the paper's QMC rule: MLQMC with Halton points (randomly shifted,
    # 16 shifts, for the error estimate) on the c4 hierarchy, N_l = 2^(2(L - l)) points
    "c4i": dict(
        name="c4i", title="the paper's cube model, MLQMC with shifted Halton points, Q1 9^3..129^3",
        dim=3, levels=_box_levels(3, [9, 17, 33, 65, 129], [32, 64, 128, 256, 512]),
        kl=dict(n_modes=66, corr_len=0.25, std=0.3, grid_level=4, kernel="sqexp", variables="uniform",
                mean=SIGMA_L, floor=0.1),
        model="iso",
        sampling=dict(kind="mlqmc", rule="halton", n_per_level=[256, 64, 16, 4, 1], n_shifts=16),
        qoi=QOI_MEAN_ACT_TIME, prec=PREC_MIXED, seed=8),
    # the paper's own heart model (Section 5.1) on the c5 shells: eq. (AdmV) with a random
    # vector field V = sigma_l f0 + W, f0 the rule-based fibre, W three independent components
    # with the squared-exponential covariance (0.3 sigma_l)^2 exp(-|x - x'|^2 / sigma_KL),
    # uniform coordinates on [-1, 1] (modes scaled by sqrt(3 lambda)), 45 modes per component
    "c5v": dict(
        name="c5v", title="non-nested shells with the paper's heart model: random fibre vector field, "
                          "uniform coordinates, 3 x 45 modes, combination estimator",
        dim=3, levels=_tet_levels(SHELL_CELLS, [512, 512, 512], 5),
        kl=dict(n_modes=45, corr_len=0.16 * (tetshell.LONG_AXIS / 1.0) ** 2, std=0.3, grid_level=2,
                kernel="sqexp", components=3, variables="uniform"),
        model="vector",
        sampling=dict(kind="combination", n_per_level=[16, 64, 256]),
        qoi=QOI_MEAN_ACT_TIME, prec=PREC_MIXED, seed=6),
    # the paper's idealised-ventricle model (Section 5.1) on the c5 shells: isotropic G = v I,
    # v = E[V] (1 + W) with W squared-exponential, theta = 0.3 relative to E[V] = 3.325e-3,
    # sigma_KL = 0.5 (the ventricle's bounding box, about 2 x 2.5 x 2, matches the shell's size),
    # 87 uniform coordinates, bounded below by 0.1 E[V]
    "c5i": dict(
        name="c5i", title="non-nested shells with the paper's ventricle model: isotropic random diffusion, "
                          "87 uniform coordinates, combination estimator",
        dim=3, levels=_tet_levels(SHELL_CELLS, [512, 512, 512], 5),
        kl=dict(n_modes=87, corr_len=0.5, std=0.3, grid_level=2,
                kernel="sqexp", variables="uniform", mean=SIGMA_L, floor=0.1),
        model="iso",
        sampling=dict(kind="combination", n_per_level=[16, 64, 256]),
        qoi=QOI_MEAN_ACT_TIME, prec=PREC_MIXED, seed=9),
}

# solver tolerances: normwise backward error of the nonlinear step equation
NEWTON_TOL = {PREC_FP64: 1e-13, PREC_MIXED: 1e-10}
INNER_TOL = {PREC_FP64: 1e-6, PREC_MIXED: 1e-5}
MAX_NEWTON = 20
MAX_INNER = 30


def config(name: str) -> dict:
    cfg = copy.deepcopy(CONFIGS[name])
    cfg["physics"] = physics(cfg["dim"])
    if cfg.get("model") == "iso":  # sigma_t is the lower bound of the isotropic conductivity
        cfg["physics"]["sigma_t"] = cfg["kl"]["floor"] * cfg["kl"]["mean"]
    if cfg["levels"][0].get("kind") == "tet":
        # stimulus: the ball around the epicardial apex (radius 1/8 of the long axis)
        c, r = tetshell.stimulus_ball()
        cfg["physics"].update(stim_center=c.tolist(), stim_radius=float(r))
    return cfg


def scaled_config(name: str, nodes=None, steps=None, n_per_level=None, n_modes=None) -> dict:
    """A smaller copy of a workload (same physics, KL settings and plan shape)."""
    cfg = config(name)
    d = cfg["dim"]
    if nodes is not None:
        steps = steps if steps is not None else [lv["n_steps"] for lv in cfg["levels"]][:len(nodes)]
        cfg["levels"] = _box_levels(d, nodes, steps)
        cfg["kl"]["grid_level"] = len(nodes) - 1
    elif steps is not None:
        for lv, m in zip(cfg["levels"], steps):
            lv["n_steps"] = int(m)
    if n_per_level is not None:
        cfg["sampling"]["n_per_level"] = list(n_per_level)
    if n_modes is not None:
        cfg["kl"]["n_modes"] = int(n_modes)
    return cfg


# --- seeded random draws ------------------------------------------------------
def _gen(*key) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([int(k) for k in key])))


def mc_normals(seed: int, level: int, n_samples: int, n_modes: int, stream: int = 0) -> np.ndarray:
    """Standard normal KL coordinates, shape (n_modes, n_samples), column i = sample i.

    Sample i of (seed, level, stream) does not depend on how many samples are
    drawn: column i is always the i-th row of one fixed stream.
    """
    g = _gen(seed, level, stream, 0x4D43)
    return np.ascontiguousarray(g.standard_normal((n_samples, n_modes)).T)


def mc_uniforms(seed: int, level: int, n_samples: int, n_dims: int, stream: int = 0) -> np.ndarray:
    """Uniform coordinates on [-1, 1], shape (n_dims, n_samples), column i = sample i (drawn
    as for mc_normals: sample i does not depend on how many samples are drawn)."""
    g = _gen(seed, level, stream, 0x4D55)
    return np.ascontiguousarray(g.uniform(-1.0, 1.0, (n_samples, n_dims)).T)


def lattice_shifts(seed: int, level: int, n_shifts: int, n_dims: int) -> np.ndarray:
    """Uniform random shifts in [0,1)^n_dims for a randomly shifted lattice rule, shape (n_shifts, n_dims)."""
    g = _gen(seed, level, 0x5348)
    return g.random((n_shifts, n_dims))


def random_angles(seed: int, n_samples: int, n_elems: int, scale: float = 0.6) -> np.ndarray:
    """Random per-element fibre angles (B, P): a smooth-free stress test for the operator."""
    g = _gen(seed, 0x414E)
    return scale * g.standard_normal((n_samples, n_elems))


def random_nodal(seed: int, n_samples: int, n_nodes: int, lo: float = -1.0, hi: float = 1.0,
                 tag: int = 0) -> np.ndarray:
    """Uniform random nodal vectors (B, n)."""
    g = _gen(seed, 0x4E44, tag)
    return g.uniform(lo, hi, (n_samples, n_nodes))


def random_potential(seed: int, n_samples: int, n_nodes: int, tag: int = 0) -> np.ndarray:
    """Random transmembrane potentials spanning rest..peak (B, n), in mV."""
    g = _gen(seed, 0x5550, tag)
    return g.uniform(-5.0, 120.0, (n_samples, n_nodes))
