"""Discrete Karhunen-Loeve expansion of the fibre-angle field (test infrastructure).

Section 2.3 of the paper: with the covariance interpolated on the nodal basis of
the finest mesh, the KL eigenproblem becomes the generalised problem
eq. (algEig)   M C M v = lambda M v.
A pivoted Cholesky factor C ~ L L^T (greedy largest-diagonal pivoting, columns
of C computed on demand) turns it into eq. (approxEig), equivalent to the small
eq. (redEig)   L^T M L v~ = lambda v~,   v = L v~,
and then v_i^T M v_j = lambda_i delta_ij, so v_k = sqrt(lambda_k) psi_k with
M-orthonormal modes psi_k.  The discrete field is eq. (KLlowrank); here it is
the scalar fibre angle  theta(x) = theta0(x) + sum_k sqrt(lambda_k) psi_k(x) y_k.

Readings (where the paper leaves a choice):
* kernel C(x, x') = s^2 exp(-|x - x'|_2 / l) (exponential, Euclidean distance), or the
  paper's squared-exponential s^2 exp(-|x - x'|_2^2 / l) (Section 5.1, l = sigma_KL);
* y_k standard normal (the workloads' fibre-angle model) or uniform on [-1, 1] with the
  modes scaled by sqrt(3 lambda_k) (the paper's model, Section 5.1): the field is linear
  in y either way, see ``field``;
* pivoted Cholesky stops when trace(C - L L^T) <= eps trace(C) or at rank r_max;
* sign of each mode: its first entry of largest magnitude is positive (entries
  within a relative 1e-9 of the maximum count as ties);
* fine -> coarse transfer (Section 4, element midpoint rule): a level-l element
  takes the value of the finest-mesh nodal interpolant at its centre.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from .mesh import BoxMesh, local_offsets


def exp_cov(X, Y, std, corr_len, kernel="exp"):
    """s^2 exp(-|x - y|_2 / l) (kernel "exp"), or s^2 exp(-|x - y|_2^2 / l) (kernel "sqexp",
    the paper's squared-exponential kernel of Section 5.1 with l = sigma_KL)."""
    d2 = np.maximum(((X[:, None, :] - Y[None, :, :]) ** 2).sum(-1), 0.0)
    if kernel == "sqexp":
        return std * std * np.exp(-d2 / corr_len)
    return std * std * np.exp(-np.sqrt(d2) / corr_len)


def pivoted_cholesky(nodes, std, corr_len, max_rank, eps=0.0, kernel="exp"):
    """Greedy pivoted Cholesky of C_ij = k(x_i, x_j).  Returns L (n, r) and pivots."""
    n = nodes.shape[0]
    diag = np.full(n, std * std)
    tr0 = diag.sum()
    L = np.zeros((n, max_rank))
    piv = []
    for r in range(max_rank):
        p = int(np.argmax(diag))
        if diag[p] <= 0.0:
            break
        col = exp_cov(nodes, nodes[p:p + 1], std, corr_len, kernel)[:, 0]
        col = col - L[:, :r] @ L[p, :r]
        L[:, r] = col / np.sqrt(diag[p])
        diag = diag - L[:, r] ** 2
        diag[p] = 0.0
        piv.append(p)
        if diag.sum() <= eps * tr0:
            r += 1
            return L[:, :r], np.array(piv)
    return L[:, :len(piv)], np.array(piv)


def fix_signs(V):
    """Make the first entry of (numerically) largest magnitude of each column positive.

    Symmetric meshes produce modes whose extreme entries come in +/- pairs of
    equal magnitude; entries within a relative 1e-9 of the maximum count as tied
    and the lowest index decides.
    """
    V = V.copy()
    for k in range(V.shape[1]):
        a = np.abs(V[:, k])
        j = int(np.argmax(a >= a.max() * (1.0 - 1e-9)))
        if V[j, k] < 0:
            V[:, k] = -V[:, k]
    return V


def kl_from_cholesky(L, M, n_modes):
    """eq. (redEig): eigenpairs of L^T M L, largest first; returns lambda (n_modes,), v = L v~ (n, n_modes)."""
    S = L.T @ (M @ L)
    S = 0.5 * (S + S.T)
    lam, Vt = np.linalg.eigh(S)
    order = np.argsort(lam)[::-1][:n_modes]
    lam, Vt = lam[order], Vt[:, order]
    V = fix_signs(L @ Vt)
    return lam, V


def kl_dense(nodes, M, std, corr_len, n_modes, kernel="exp"):
    """Direct solution of eq. (algEig) on small meshes: M C M v = lambda M v."""
    Md = M.toarray() if hasattr(M, "toarray") else np.asarray(M)
    C = exp_cov(nodes, nodes, std, corr_len, kernel)
    lam, V = sla.eigh(Md @ C @ Md, Md)
    order = np.argsort(lam)[::-1][:n_modes]
    lam, V = lam[order], V[:, order]  # V^T M V = I
    return lam, fix_signs(V * np.sqrt(np.maximum(lam, 0.0)))


def kl_modes(mesh: BoxMesh, M, std, corr_len, n_modes, max_rank=None, eps=1e-2, kernel="exp"):
    """KL on the nodes of ``mesh``: returns lambda (n_modes,) and unit modes psi (n, n_modes)."""
    if max_rank is None:
        max_rank = 2 * n_modes
    L, _ = pivoted_cholesky(mesh.nodes, std, corr_len, max(max_rank, n_modes), eps, kernel)
    if L.shape[1] < n_modes:
        L, _ = pivoted_cholesky(mesh.nodes, std, corr_len, n_modes, 0.0, kernel)
    lam, V = kl_from_cholesky(L, M, n_modes)
    return lam, V / np.sqrt(lam)


def interpolate(mesh: BoxMesh, values, pts):
    """Evaluate the Q1 nodal interpolant of ``values`` (n, ...) at points (P, d)."""
    e, xi = mesh.locate(pts)
    d = mesh.d
    out = 0.0
    for a, off in enumerate(local_offsets(d)):
        w = np.ones(e.shape[0])
        for k in range(d):
            w = w * (xi[:, k] if off[k] else 1.0 - xi[:, k])
        nid = mesh.node_id(e + np.array(off))
        out = out + w.reshape((-1,) + (1,) * (np.ndim(values) - 1)) * values[nid]
    return out


def level_basis(kl_mesh: BoxMesh, psi, level_mesh: BoxMesh):
    """Phi_l: the KL modes at the element centres of a level (midpoint transfer)."""
    return interpolate(kl_mesh, psi, level_mesh.centres)


def field(theta0, phi, sqrt_lam, Y):
    """eq. (KLlowrank) for the angle: theta (B, P) = theta0 + Phi diag(sqrt(lambda)) Y, Y (M, B)."""
    return (np.asarray(theta0)[None, :] + (phi @ (sqrt_lam[:, None] * Y)).T)
