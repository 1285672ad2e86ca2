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


def space_time_norm2(mesh: BoxMesh, field, t_end, q=0):
    """||f||^2 in L^2((0, T); H^q(D)) (eq. (space-time-error)) of the space-time interpolant of
    the nodal values field ((m + 1, n): Q1 in space, linear in time), integrated exactly:
    on [t_k, t_(k+1)], dt/3 (f_k' A f_k + f_k' A f_(k+1) + f_(k+1)' A f_(k+1)) with A = M (q = 0)
    or M + K (q = 1, K the Laplacian stiffness, so the H^1 norm includes its L^2 part)."""
    from . import fem
    F = np.asarray(field, dtype=np.float64)
    m = F.shape[0] - 1
    Mm, K = fem.assemble(mesh, fem.conductivity_iso(np.ones(mesh.n_elems), mesh.d))
    A = Mm if q == 0 else Mm + K
    AF = np.stack([A @ F[k] for k in range(m + 1)])
    dt = t_end / m
    total = 0.0
    for k in range(m):
        total += dt / 3.0 * (F[k] @ AF[k] + F[k] @ AF[k + 1] + F[k + 1] @ AF[k + 1])
    return float(total)


def time_norm2(series, t_end, q=0):
    """||f||^2 in H^q(0, T) (eq. (point-error)) of the linear interpolant of each row of series
    (..., m + 1): sum_k dt/3 (a^2 + a b + b^2), plus sum_k (b - a)^2 / dt for q = 1."""
    S = np.asarray(series, dtype=np.float64)
    m = S.shape[-1] - 1
    dt = t_end / m
    a, b = S[..., :-1], S[..., 1:]
    out = (dt / 3.0 * (a * a + a * b + b * b)).sum(axis=-1)
    if q == 1:
        out = out + ((b - a) ** 2 / dt).sum(axis=-1)
    return out
