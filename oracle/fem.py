"""Finite elements on Q1 box meshes (test infrastructure; see ``oracle/__init__``).

* ``conductivity``  -- eq. (AdmV): G = g I + (|V| - g) V V^T / (V^T V), with the
  fibre field V = sigma_l f, f the unit fibre direction of the element.
* ``assemble``      -- mass M_ij = int phi_j phi_i and anisotropic stiffness
  K_ij = int G grad phi_j . grad phi_i of the Galerkin semi-discretisation,
  eq. (semi-disc) of Section 3.1, with G constant per element (the element
  midpoint rule of Section 4).  Integrals use the 2-point Gauss rule per axis,
  which is exact for the Q1 products involved.
* ``box_load``      -- F_i = int chi_box(x) phi_i(x) dx, integrated exactly.
* ``source_load``   -- F_i = int f(x) phi_i(x) dx by a 4-point Gauss rule per axis
  (only used for manufactured solutions).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .mesh import BoxMesh, local_offsets

_G2 = np.array([0.5 - 0.5 / np.sqrt(3.0), 0.5 + 0.5 / np.sqrt(3.0)])
_W2 = np.array([0.5, 0.5])


def fibre_direction(theta, d):
    """Unit fibre direction from an angle: rotation in the x-y plane, (cos, sin[, 0])."""
    theta = np.asarray(theta, dtype=np.float64)
    f = np.zeros(theta.shape + (d,))
    f[..., 0] = np.cos(theta)
    f[..., 1] = np.sin(theta)
    return f


def conductivity(V, g):
    """eq. (AdmV): G = g I + (|V| - g) V V^T / (V^T V), for V of shape (..., d)."""
    V = np.asarray(V, dtype=np.float64)
    d = V.shape[-1]
    vtv = np.einsum("...i,...i->...", V, V)
    nv = np.sqrt(vtv)
    outer = np.einsum("...i,...j->...ij", V, V)
    eye = np.broadcast_to(np.eye(d), V.shape[:-1] + (d, d))
    return g * eye + ((nv - g) / vtv)[..., None, None] * outer


def conductivity_from_angle(theta, d, sigma_l, sigma_t):
    """Per-element conductivity for fibre angle theta: V = sigma_l f(theta), g = sigma_t."""
    return conductivity(sigma_l * fibre_direction(theta, d), sigma_t)


def conductivity_iso(v, d, floor=0.0):
    """Isotropic scalar conductivity G = max(v, floor) I per element (the paper's cube model,
    Section 5.1; the floor is the lower bound b_min the model assumes)."""
    v = np.maximum(np.asarray(v, dtype=np.float64), floor)
    return v[..., None, None] * np.broadcast_to(np.eye(d), v.shape + (d, d))


def _ref_basis(d, xi):
    """Q1 reference basis values (2^d,) and reference gradients (2^d, d) at xi in [0,1]^d."""
    offs = local_offsets(d)
    vals = np.ones(2 ** d)
    grads = np.ones((2 ** d, d))
    for a, off in enumerate(offs):
        for k in range(d):
            lin = xi[k] if off[k] else 1.0 - xi[k]
            dlin = 1.0 if off[k] else -1.0
            vals[a] *= lin
            for m in range(d):
                grads[a, m] *= dlin if m == k else lin
    return vals, grads


def _gauss_points(d, pts, wts):
    grids = np.meshgrid(*([pts] * d), indexing="ij")
    wg = np.meshgrid(*([wts] * d), indexing="ij")
    P = np.stack([g.ravel() for g in grids], axis=1)
    W = np.prod(np.stack([w.ravel() for w in wg], axis=1), axis=1)
    return P, W


def element_matrices(mesh: BoxMesh, G):
    """Element mass (2^d, 2^d) and per-element stiffness (E, 2^d, 2^d) for G of shape (E, d, d)."""
    d = mesh.d
    P, W = _gauss_points(d, _G2, _W2)
    detJ = float(np.prod(mesh.h))
    nl = 2 ** d
    Me = np.zeros((nl, nl))
    Ke = np.zeros((G.shape[0], nl, nl))
    for q in range(P.shape[0]):
        v, gr = _ref_basis(d, P[q])
        gphys = gr / mesh.h  # (nl, d): d phi_a / d x_m
        Me += W[q] * detJ * np.outer(v, v)
        # K_e[a,b] = int (G grad phi_b) . grad phi_a
        Ke += W[q] * detJ * np.einsum("am,emn,bn->eab", gphys, G, gphys)
    return Me, Ke


def assemble(mesh: BoxMesh, G):
    """Global mass and stiffness (CSR) for per-element conductivities G (E, d, d)."""
    Me, Ke = element_matrices(mesh, G)
    conn = mesh.elems
    nl = conn.shape[1]
    rows = np.repeat(conn, nl, axis=1).ravel()
    cols = np.tile(conn, (1, nl)).ravel()
    n = mesh.n_nodes
    M = sp.coo_matrix((np.tile(Me.ravel(), mesh.n_elems), (rows, cols)), shape=(n, n)).tocsr()
    K = sp.coo_matrix((Ke.reshape(mesh.n_elems, -1).ravel(), (rows, cols)), shape=(n, n)).tocsr()
    return M, K


def assemble_mass(mesh: BoxMesh):
    G = np.zeros((mesh.n_elems, mesh.d, mesh.d))
    M, _ = assemble(mesh, G)
    return M


def _hat_integral_1d(xn, h, a, b, i, n):
    """Exact int_{[a,b]} phi_i over the 1D hat of node i (coordinate xn)."""
    total = 0.0
    # left half: [xn - h, xn], phi rises 0 -> 1 ; right half: [xn, xn + h], falls 1 -> 0
    for lo, hi, rising in ((xn - h, xn, True), (xn, xn + h, False)):
        if (rising and i == 0) or ((not rising) and i == n - 1):
            continue
        s, t = max(lo, a), min(hi, b)
        if t <= s:
            continue
        mid = 0.5 * (s + t)
        val = (mid - lo) / h if rising else (hi - mid) / h
        total += (t - s) * val  # midpoint rule is exact for linear integrands
    return total


def box_load(mesh: BoxMesh, box_lo, box_hi):
    """F_i = int_D chi_[box_lo, box_hi](x) phi_i(x) dx for the tensor-product Q1 basis (exact)."""
    one_d = []
    for k in range(mesh.d):
        xs = mesh.lo[k] + mesh.h[k] * np.arange(mesh.n[k])
        one_d.append(np.array([_hat_integral_1d(xs[i], mesh.h[k], box_lo[k], box_hi[k], i, mesh.n[k])
                               for i in range(mesh.n[k])]))
    F = one_d[0]
    for k in range(1, mesh.d):
        F = np.kron(one_d[k], F)  # axis k varies slower than the axes before it
    return F


def source_load(mesh: BoxMesh, f):
    """F_i = int f(x) phi_i(x) dx with a 4-point Gauss rule per axis; f maps (N, d) -> (N,)."""
    g4, w4 = np.polynomial.legendre.leggauss(4)
    pts, wts = _gauss_points(mesh.d, 0.5 * (g4 + 1.0), 0.5 * w4)
    detJ = float(np.prod(mesh.h))
    base = mesh.lo + mesh.elem_index * mesh.h  # (E, d) lower corners
    F = np.zeros(mesh.n_nodes)
    for q in range(pts.shape[0]):
        v, _ = _ref_basis(mesh.d, pts[q])
        fx = f(base + pts[q] * mesh.h)  # (E,)
        contrib = wts[q] * detJ * fx[:, None] * v[None, :]
        np.add.at(F, mesh.elems.ravel(), contrib.ravel())
    return F


def node_weights(M):
    """w = M 1: integrating the FE interpolant of nodal values gives w . values."""
    return np.asarray(M @ np.ones(M.shape[0])).ravel()


def row_products(mesh: BoxMesh, theta, sigma_l, sigma_t, rows, vecs):
    """Rows of M v and K v for the listed nodes only, each from the (up to 2^d)
    elements around the node, with K for per-element fibre angles theta (E,).

    The same element matrices as ``assemble``; meant for meshes too large to
    assemble.  Returns (Mv, Kv), each of shape (len(vecs), len(rows)).
    """
    d = mesh.d
    rows = np.asarray(rows, dtype=np.int64)
    ijk = np.zeros((rows.size, d), dtype=np.int64)
    r = rows.copy()
    for a in range(d):
        ijk[:, a] = r % mesh.n[a]
        r //= mesh.n[a]
    Mv = np.zeros((len(vecs), rows.size))
    Kv = np.zeros((len(vecs), rows.size))
    ne = np.array(mesh.ne)
    for a, off in enumerate(local_offsets(d)):
        e = ijk - np.array(off)
        ok = np.all((e >= 0) & (e < ne), axis=1)
        if not ok.any():
            continue
        ek = e[ok]
        eid = ek[:, 0].copy()
        stride = 1
        for k in range(1, d):
            stride *= ne[k - 1]
            eid += stride * ek[:, k]
        G = conductivity_from_angle(np.asarray(theta)[eid], d, sigma_l, sigma_t)
        Me, Ke = element_matrices(mesh, G)
        conn = mesh.node_id(ek[:, None, :] + np.array(local_offsets(d))[None, :, :])
        for v, vec in enumerate(vecs):
            vals = np.asarray(vec)[conn]  # (k, 2^d)
            Mv[v, ok] += vals @ Me[a]
            Kv[v, ok] += np.einsum("kb,kb->k", Ke[:, a, :], vals)
    return Mv, Kv


def stiffness_row_bound(mesh: BoxMesh, sigma_l, sigma_t):
    """An upper bound of max_i sum_j |K_ij| over every fibre field.

    K_e depends on the angle only through (cos 2t, sin 2t) linearly, K_e = A + cos 2t Bc
    + sin 2t Bs, so |K_e[a, b]| <= |A[a, b]| + sqrt(Bc[a, b]^2 + Bs[a, b]^2); a node
    touches at most 2^d elements.
    """
    d = mesh.d
    th = np.array([0.0, 0.5 * np.pi, 0.25 * np.pi])
    _, Ke = element_matrices(mesh, conductivity_from_angle(th, d, sigma_l, sigma_t))
    A = 0.5 * (Ke[0] + Ke[1])
    Bc = 0.5 * (Ke[0] - Ke[1])
    Bs = Ke[2] - A
    per_elem = (np.abs(A) + np.sqrt(Bc ** 2 + Bs ** 2)).sum(axis=1).max()
    return (2 ** d) * per_elem
