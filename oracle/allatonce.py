"""All-at-once space-time Newton on tiny meshes (test infrastructure; see ``oracle/__init__``).

Builds the block lower-bidiagonal matrix C of eq. (system_C), blocks
A = M + dt/2 K on the diagonal and B = -M + dt/2 K below it, adds the reaction
term r(U) = (dt I (x) M) I_ion(U) of eq. (mono_disc) and solves
C U + r(U) = I_app for all unknown time levels at once by Newton's method with
the Jacobian C + (dt I (x) M) diag(I_ion'(U)) (Section 3.2) and a sparse LU.

The unknowns are u_1..u_m; u_0 = 0 is the initial condition, so the first block
row reads A u_1 = dt/2 (F(t_1) + F(t_0)).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .ionic import i_ion, di_ion
from .stepper import Problem


def solve_all_at_once(mesh, G, p, n_steps, tol=1e-13, max_newton=50):
    prob = Problem(mesh, G, p, n_steps)
    m, n, dt = prob.n_steps, mesh.n_nodes, prob.dt
    C = sp.kron(sp.eye(m), prob.A) + sp.kron(sp.eye(m, k=-1), -prob.B)
    C = C.tocsr()
    R = sp.kron(sp.eye(m), dt * prob.M).tocsr()
    rhs = np.concatenate([0.5 * dt * (prob.load((k + 1) * dt) + prob.load(k * dt)) for k in range(m)])
    U = np.zeros(m * n)
    for _ in range(max_newton):
        GU = C @ U + R @ i_ion(U, p)
        F = GU - rhs
        den = np.linalg.norm(GU) + np.linalg.norm(rhs)
        if den == 0.0 or np.linalg.norm(F) / den <= tol:
            return U.reshape(m, n)
        J = (C + R @ sp.diags(di_ion(U, p))).tocsc()
        U = U + spla.splu(J).solve(-F)
    raise RuntimeError("all-at-once Newton did not converge")
