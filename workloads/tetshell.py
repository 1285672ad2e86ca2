"""Seeded heart-like geometry: a truncated prolate-ellipsoidal shell split into tetrahedra.

This is an input description only (node coordinates, connectivity, a local
fibre frame and a rule-based base angle per element); it holds none of the
method's arithmetic.

Geometry.  Prolate spheroidal coordinates (mu, nu, phi) with focal distance a:
    x = a sinh(mu) sin(nu) cos(phi),  y = a sinh(mu) sin(nu) sin(phi),  z = a cosh(mu) cos(nu).
The epicardium is the spheroid with semi-axes (1, 1, 2) (a = sqrt(3)); the
endocardium is the confocal spheroid whose short semi-axis is 0.85 (a wall of
0.15 short-axis units).  nu runs from NU_APEX (a small apical opening) to pi / 2
(the base, cut at the equator); phi covers the full circle.  A structured grid of
n_mu x n_nu x n_phi cells (periodic in phi) is split into the six tetrahedra of
the Kuhn triangulation per cell, and every vertex off the endo-, epicardial,
apical and basal surfaces is moved by a seeded offset of up to +-JITTER/2 cell
widths in each parametric direction, so that the levels are not nested.

Per tetrahedron: the unit circumferential direction e_circ = (-sin phi, cos phi, 0)
and the unit longitudinal direction e_long (along d x / d nu, from the apex to the
base), both evaluated at the centroid and tangent to the confocal spheroids, and
the base fibre angle theta0 = +60 deg at the epicardium to -60 deg at the
endocardium, linear in the transmural coordinate of the centroid.
"""
from __future__ import annotations

import numpy as np

A_FOCAL = float(np.sqrt(3.0))
MU_EPI = float(np.arcsinh(1.0 / A_FOCAL))
MU_ENDO = float(np.arcsinh(0.85 / A_FOCAL))
NU_APEX = 0.1
NU_BASE = 0.5 * np.pi
JITTER = 0.3
APEX = np.array([0.0, 0.0, A_FOCAL * np.cosh(MU_EPI)])  # epicardial apex (0, 0, 2)
LONG_AXIS = float(APEX[2])                              # apex-to-base length (base at z = 0)

# Kuhn split of a cell with corners c[i][j][k] (i: mu, j: nu, k: phi offsets)
_KUHN = [((0, 0, 0), (1, 0, 0), (1, 1, 0), (1, 1, 1)),
         ((0, 0, 0), (1, 0, 0), (1, 0, 1), (1, 1, 1)),
         ((0, 0, 0), (0, 1, 0), (1, 1, 0), (1, 1, 1)),
         ((0, 0, 0), (0, 1, 0), (0, 1, 1), (1, 1, 1)),
         ((0, 0, 0), (0, 0, 1), (1, 0, 1), (1, 1, 1)),
         ((0, 0, 0), (0, 0, 1), (0, 1, 1), (1, 1, 1))]


def spheroidal_to_xyz(mu, nu, phi):
    s = A_FOCAL * np.sinh(mu) * np.sin(nu)
    return np.stack([s * np.cos(phi), s * np.sin(phi), A_FOCAL * np.cosh(mu) * np.cos(nu)], axis=-1)


def xyz_to_spheroidal(p):
    """Inverse map (closed form through the distances to the two foci)."""
    p = np.asarray(p, dtype=np.float64)
    rho = np.hypot(p[..., 0], p[..., 1])
    d1 = np.hypot(rho, p[..., 2] + A_FOCAL)
    d2 = np.hypot(rho, p[..., 2] - A_FOCAL)
    mu = np.arccosh(np.maximum((d1 + d2) / (2.0 * A_FOCAL), 1.0))
    nu = np.arccos(np.clip((d1 - d2) / (2.0 * A_FOCAL), -1.0, 1.0))
    phi = np.arctan2(p[..., 1], p[..., 0])
    return mu, nu, phi


def shell_mesh(cells, seed, jitter=JITTER):
    """Vertices (V, 3), tetrahedra (T, 4) int32 (positively oriented), e_circ (T, 3),
    e_long (T, 3), theta0 (T,) for n_mu x n_nu x n_phi = cells."""
    n_mu, n_nu, n_phi = (int(c) for c in cells)
    mu = np.linspace(MU_ENDO, MU_EPI, n_mu + 1)
    nu = np.linspace(NU_APEX, NU_BASE, n_nu + 1)
    phi = np.arange(n_phi) * (2.0 * np.pi / n_phi)
    M, N, F = np.meshgrid(mu, nu, phi, indexing="ij")  # (n_mu+1, n_nu+1, n_phi)
    g = np.random.Generator(np.random.PCG64(np.random.SeedSequence([int(seed), n_mu, n_nu, n_phi, 0x5445])))
    off = g.uniform(-0.5, 0.5, M.shape + (3,)) * jitter
    interior = np.zeros(M.shape, dtype=bool)
    interior[1:-1, 1:-1, :] = True
    M = M + np.where(interior, off[..., 0] * (mu[1] - mu[0]), 0.0)
    N = N + np.where(interior, off[..., 1] * (nu[1] - nu[0]), 0.0)
    F = F + np.where(interior, off[..., 2] * (2.0 * np.pi / n_phi), 0.0)
    # vertices numbered longitudinal index slowest, then transmural, circumferential fastest: the
    # rows of a wave are consecutive around a ring (their slot gathers coalesce), and a row's
    # transmural neighbours are one ring (n_phi rows) away, its longitudinal ones one ring of rings
    xyz = np.transpose(spheroidal_to_xyz(M, N, F), (1, 0, 2, 3)).reshape(-1, 3)

    def vid(i, j, k):
        return (j * (n_mu + 1) + i) * n_phi + (k % n_phi)

    J, I, K = np.meshgrid(np.arange(n_nu), np.arange(n_mu), np.arange(n_phi), indexing="ij")
    I, J, K = I.ravel(), J.ravel(), K.ravel()
    tets = np.concatenate([np.stack([vid(I + a[0], J + a[1], K + a[2]) for a in t], axis=1) for t in _KUHN])
    # positive orientation
    p = xyz[tets]
    vol6 = np.einsum("ij,ij->i", np.cross(p[:, 1] - p[:, 0], p[:, 2] - p[:, 0]), p[:, 3] - p[:, 0])
    neg = vol6 < 0
    tets[neg, 2], tets[neg, 3] = tets[neg, 3].copy(), tets[neg, 2].copy()
    # local frame and rule-based angle at the centroids
    c = xyz[tets].mean(axis=1)
    cmu, cnu, cphi = xyz_to_spheroidal(c)
    e_circ = np.stack([-np.sin(cphi), np.cos(cphi), np.zeros_like(cphi)], axis=1)
    dnu = np.stack([np.sinh(cmu) * np.cos(cnu) * np.cos(cphi), np.sinh(cmu) * np.cos(cnu) * np.sin(cphi),
                    -np.cosh(cmu) * np.sin(cnu)], axis=1)
    e_long = dnu / np.linalg.norm(dnu, axis=1, keepdims=True)
    t = np.clip((cmu - MU_ENDO) / (MU_EPI - MU_ENDO), 0.0, 1.0)
    theta0 = np.deg2rad(-60.0 + 120.0 * t)
    return xyz, tets.astype(np.int32), e_circ, e_long, theta0


def stimulus_ball(radius_frac=0.125):
    """Stimulus region: the ball around the epicardial apex of radius radius_frac * long axis."""
    return APEX.copy(), radius_frac * LONG_AXIS
