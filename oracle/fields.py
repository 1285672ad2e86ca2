"""Field quantities of interest and their multilevel estimate (test infrastructure; see
``oracle/__init__``).

Section 2.4 names three quantities of interest besides scalar summaries: the transmembrane
potential u itself (the identity functional on the space-time solution), the action potential
u(x0, t) at a location x0, and the activation map a(x) (first time u reaches u_th).  Their
multilevel estimate (eq. (StandardML)) needs the level-l field on the finest level's space-time
grid; the paper transfers it with the tensor product of the space and time interpolations
(Section 5, the paragraph on the error measures).  Here:

* space: the nodal Q1 interpolant of the coarse field evaluated at the fine nodes (nested boxes);
* time: the piecewise linear interpolant in t on the coarse time grid evaluated at the fine
  time nodes;
* the field estimate: sum over levels of the sample means of P_l^L u_l - P_(l-1)^L u_(l-1), the
  same estimator as for scalars applied to every space-time node.

Readings: the initial state u_0 is part of the space-time field (row k = 0); never-activated
nodes enter the activation map at the stop time, as for the scalar mean activation time.
"""
from __future__ import annotations

import numpy as np

from . import kl
from .mesh import BoxMesh


def space_time_field(out):
    """(m + 1, n): the nodal states u_0 .. u_m of one sample (``stepper.solve(keep_all=True)``)."""
    return np.asarray(out["history"])


def action_potential(mesh: BoxMesh, out, pts):
    """(P, m + 1): the Q1 interpolant of u(., t_k) at the points, for every time node."""
    H = space_time_field(out)
    return np.asarray(kl.interpolate(mesh, H.T, np.atleast_2d(pts)))


def activation_map(out):
    """(n,): activation times with never-activated nodes at the stop time."""
    return np.asarray(out["act_censored"])


def prolongate_space(mesh_c: BoxMesh, values_c, mesh_f: BoxMesh):
    """Coarse nodal values (n_c, ...) -> their Q1 interpolant at the fine nodes (n_f, ...)."""
    return np.asarray(kl.interpolate(mesh_c, values_c, mesh_f.nodes))


def prolongate_time(series_c, m_c, m_f, t_end):
    """Rows of values on the coarse time nodes (..., m_c + 1) -> the linear interpolant at the
    fine time nodes (..., m_f + 1)."""
    tc = np.linspace(0.0, t_end, m_c + 1)
    tf = np.linspace(0.0, t_end, m_f + 1)
    S = np.asarray(series_c, dtype=np.float64)
    flat = S.reshape(-1, m_c + 1)
    res = np.stack([np.interp(tf, tc, row) for row in flat])
    return res.reshape(S.shape[:-1] + (m_f + 1,))


def prolongate_space_time(mesh_c, m_c, field_c, mesh_f, m_f, t_end):
    """(m_c + 1, n_c) -> (m_f + 1, n_f): space interpolation, then time interpolation."""
    Fs = prolongate_space(mesh_c, np.asarray(field_c).T, mesh_f)       # (n_f, m_c + 1)
    return np.ascontiguousarray(prolongate_time(Fs, m_c, m_f, t_end).T)


def mlmc_field(fine_sums, coarse_sums, n_per_level, transfer):
    """eq. (StandardML) for a field: fine_sums[l] = sum over the level-l samples of the level-l
    field, coarse_sums[l] = the same samples' level-(l-1) field summed (None for l = 0);
    transfer(j, F) maps a level-j field to the finest grid."""
    est = 0.0
    for l, N in enumerate(n_per_level):
        est = est + transfer(l, fine_sums[l]) / N
        if l > 0:
            est = est - transfer(l - 1, coarse_sums[l]) / N
    return est
