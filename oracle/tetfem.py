"""P1 finite elements on tetrahedral meshes (test infrastructure; see ``oracle/__init__``).

Section 3.1: the Galerkin semi-discretisation eq. (semi-disc) with the
piecewise-linear space on a shape-regular tetrahedral mesh, G constant per
element (Section 4, element midpoint rule), read at the element centroid.

* mass      M_ij = int phi_i phi_j = |T| (1 + delta_ij) / 20 on each tetrahedron T;
* stiffness K_ij = |T| grad phi_i . G_T grad phi_j, with constant gradients;
* fibres    eq. (AdmV) with V = sigma_l f and f = cos(theta) e_circ + sin(theta) e_long,
            the unit circumferential / longitudinal directions of the element;
* stimulus  F = M chi, chi the indicator of the vertices inside the stimulus ball
            (reading: the stimulated region enters through its nodal interpolant);
* transfer  the value at a point of the P1 interpolant on another (non-nested)
            mesh: the point is assigned the tetrahedron with the largest smallest
            barycentric coordinate (lowest index on ties within 1e-12), whose
            barycentric coordinates, clipped at 0 and renormalised, are the weights.
            Inside the mesh this is the containing tetrahedron; a point just
            outside a curved boundary takes the nearest one.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .fem import conductivity


class TetMesh:
    def __init__(self, xyz, tets):
        self.nodes = np.asarray(xyz, dtype=np.float64)
        self.elems = np.asarray(tets, dtype=np.int64)
        self.d = 3
        self.n_nodes = self.nodes.shape[0]
        self.n_elems = self.elems.shape[0]
        p = self.nodes[self.elems]                       # (T, 4, 3)
        E = (p[:, 1:, :] - p[:, :1, :])                  # edge vectors, rows
        det = np.linalg.det(E)
        self.vol = det / 6.0
        if (self.vol <= 0).any():
            raise ValueError("tetrahedra must be positively oriented")
        # grad phi_a: rows of inv(E)^T give grad of phi_1..3; grad phi_0 = -sum
        inv = np.linalg.inv(E)                           # (T, 3, 3): columns map to barycentric
        g = np.zeros((self.n_elems, 4, 3))
        g[:, 1:, :] = np.transpose(inv, (0, 2, 1))
        g[:, 0, :] = -g[:, 1:, :].sum(axis=1)
        self.grad = g
        self.centres = p.mean(axis=1)

    @property
    def volume(self) -> float:
        return float(self.vol.sum())

    def _scatter(self, Ke):
        nl = 4
        rows = np.repeat(self.elems, nl, axis=1).ravel()
        cols = np.tile(self.elems, (1, nl)).ravel()
        n = self.n_nodes
        return sp.coo_matrix((Ke.reshape(self.n_elems, -1).ravel(), (rows, cols)), shape=(n, n)).tocsr()

    def assemble(self, G):
        """Global mass and stiffness for per-element conductivities G (T, 3, 3)."""
        Me = (np.ones((4, 4)) + np.eye(4)) / 20.0
        M = self._scatter(self.vol[:, None, None] * Me[None])
        Ke = self.vol[:, None, None] * np.einsum("tam,tmn,tbn->tab", self.grad, G, self.grad)
        K = self._scatter(Ke)
        return M, K

    def conductivity(self, theta, e_circ, e_long, sigma_l, sigma_t):
        th = np.asarray(theta, dtype=np.float64)
        f = np.cos(th)[:, None] * e_circ + np.sin(th)[:, None] * e_long
        return conductivity(sigma_l * f, sigma_t)

    def stim_load(self, p):
        M, _ = self.assemble(np.zeros((self.n_elems, 3, 3)))
        chi = (np.linalg.norm(self.nodes - np.asarray(p["stim_center"]), axis=1) < p["stim_radius"]).astype(float)
        return M @ chi

    def barycentric(self, pts, tet_ids):
        """Barycentric coordinates (P, 4) of points in the given tetrahedra."""
        pts = np.atleast_2d(pts)
        p0 = self.nodes[self.elems[tet_ids, 0]]
        lam = np.einsum("pam,pm->pa", self.grad[tet_ids, 1:, :], pts - p0)
        return np.concatenate([1.0 - lam.sum(axis=1, keepdims=True), lam], axis=1)

    def locate(self, pts, chunk=256):
        """Tetrahedron of each point (largest smallest barycentric coordinate, lowest index
        on ties within 1e-12) and its clipped, renormalised barycentric weights.  Brute force."""
        pts = np.atleast_2d(np.asarray(pts, dtype=np.float64))
        tet = np.zeros(pts.shape[0], dtype=np.int64)
        w = np.zeros((pts.shape[0], 4))
        p0 = self.nodes[self.elems[:, 0]]
        G = self.grad[:, 1:, :]
        for s in range(0, pts.shape[0], chunk):
            q = pts[s:s + chunk]
            lam = np.einsum("tam,ptm->pta", G, q[:, None, :] - p0[None, :, :])   # (p, T, 3)
            lam0 = 1.0 - lam.sum(axis=2)
            score = np.minimum(lam0, lam.min(axis=2))                              # (p, T)
            best = score.max(axis=1, keepdims=True)
            cand = score >= best - 1e-12
            t = np.argmax(cand, axis=1)                                            # lowest index
            tet[s:s + chunk] = t
            b = np.concatenate([lam0[np.arange(q.shape[0]), t][:, None], lam[np.arange(q.shape[0]), t]], axis=1)
            b = np.maximum(b, 0.0)
            w[s:s + chunk] = b / b.sum(axis=1, keepdims=True)
        return tet, w

    def interpolate(self, values, pts):
        """P1 interpolant of nodal ``values`` (n, ...) at points (P, 3)."""
        tet, w = self.locate(pts)
        v = np.asarray(values)[self.elems[tet]]                 # (P, 4, ...)
        return np.einsum("pa,pa...->p...", w, v)


def node_weights(M):
    """w = M 1 (integrates the P1 interpolant of nodal values)."""
    return np.asarray(M @ np.ones(M.shape[0])).ravel()
