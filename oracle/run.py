"""Per-sample and per-workload driver of the oracle (test infrastructure).

One sample omega (KL coordinates y) on level l (Section 4, Section 5.1):
  1. theta at the level's element centres from eq. (KLlowrank) and the midpoint transfer;
  2. G_e from eq. (AdmV) with the rule-based fibre angle, or the isotropic model of the
     cube experiment, G_e = max(v_e, b_min) I with v = E[V] + W (the floor b_min is sigma_t);
  3. the space-time solve (``stepper``);
  4. the quantity of interest: mean u at the final time, or the mean activation
     time (first crossing of u_th, Section 2.4, linear in time between nodes,
     censored at the end time) -- both as integrals of the nodal interpolant
     over D divided by |D|.
"""
from __future__ import annotations

import numpy as np

from . import fem, kl, stepper
from .mesh import BoxMesh


def level_meshes(cfg):
    return [BoxMesh(lv["n"], lv["lo"], lv["hi"]) for lv in cfg["levels"]]


def kl_basis(cfg, meshes=None, max_rank=None, eps=1e-2):
    """KL modes on the grid of level ``kl.grid_level`` and their midpoint transfer to every level.

    The isotropic model states its standard deviation relative to E[V].  Uniform coordinates on
    [-1, 1] have variance 1/3, so each mode is weighted by sqrt(3 lambda) to keep the field's
    covariance; normal coordinates take sqrt(lambda) (eq. (KLlowrank))."""
    meshes = meshes or level_meshes(cfg)
    kcfg = cfg["kl"]
    kmesh = meshes[kcfg["grid_level"]]
    M = fem.assemble_mass(kmesh)
    std = kcfg["std"] * (kcfg["mean"] if cfg.get("model") == "iso" else 1.0)
    lam, psi = kl.kl_modes(kmesh, M, std, kcfg["corr_len"], kcfg["n_modes"],
                           max_rank=max_rank, eps=eps, kernel=kcfg.get("kernel", "exp"))
    phis = [kl.level_basis(kmesh, psi, m) for m in meshes]
    w = 3.0 if kcfg.get("variables") == "uniform" else 1.0
    return dict(lam=lam, sqrt_lam=np.sqrt(w * lam), psi=psi, phi=phis, kl_mesh=kmesh)


def level_theta0(cfg, mesh):
    """The field's mean per element: E[V] for the isotropic model, 0 for the fibre angle."""
    mean = cfg["kl"]["mean"] if cfg.get("model") == "iso" else 0.0
    return np.full(mesh.n_elems, float(mean))


def sample_theta(phi_l, sqrt_lam, Y, theta0=None):
    theta0 = np.zeros(phi_l.shape[0]) if theta0 is None else theta0
    return kl.field(theta0, phi_l, sqrt_lam, Y)


def solve_theta(mesh, theta_e, phys, n_steps, tol=1e-13, stop_after=None, model=None, keep_all=False):
    if model == "iso":
        G = fem.conductivity_iso(theta_e, mesh.d, phys["sigma_t"])
    else:
        G = fem.conductivity_from_angle(theta_e, mesh.d, phys["sigma_l"], phys["sigma_t"])
    return stepper.solve(mesh, G, phys, n_steps, tol=tol, stop_after=stop_after, keep_all=keep_all)


def qoi_of(out, qoi):
    return stepper.qoi_value(out, qoi)
