"""Space-time solve of the monodomain equation (test infrastructure; see ``oracle/__init__``).

Crank-Nicolson in time, eq. (st-system):
    (M + dt/2 K) u_{k+1} + (-M + dt/2 K) u_k = dt/2 (F(t_{k+1}) + F(t_k)),
extended by the reaction term of eq. (mono_disc), r(u) = (dt I (x) M) I_ion(u),
i.e. for every unknown time level dt * M * I_ion(u_{k+1}) is added to the left
side.  The all-at-once matrix eq. (system_C) is block lower bidiagonal and the
reaction term is block diagonal, so the whole space-time system decouples into
one nonlinear equation per time level, solved in order with u_0 = 0 (the
initial condition of eq. (monodomain)).  This is the multiple-time-blocks
strategy of Section 3.3 with one step per block; ``allatonce`` checks the
equivalence on tiny meshes.

Each step is solved by Newton's method with the Jacobian of Section 3.2,
J = M + dt/2 K + dt M diag(I_ion'(u)), starting from u_k, until the normwise
backward error ||G(u) - b|| / (||G(u)|| + ||b||) <= tol, where
G(u) = (M + dt/2 K) u + dt M I_ion(u) and b is the right-hand side of the step.
Linear systems are solved exactly (sparse LU) on small meshes and by
Jacobi-preconditioned GMRES to a relative residual of 1e-14 on larger ones;
either way Newton stops on the same true residual test.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import fem
from .ionic import i_ion, di_ion
from .mesh import BoxMesh

DIRECT_MAX_NODES = 1500


def stim_rate(t, p):
    """Time profile of the stimulus: amplitude on [t_on, t_off), zero elsewhere."""
    return p["stim_amp"] if (p["stim_t_on"] <= t < p["stim_t_off"]) else 0.0


class Problem:
    """One sample's discrete problem on one mesh: matrices and load vectors."""

    def __init__(self, mesh: BoxMesh, G, p, n_steps, source=None):
        self.mesh, self.p, self.n_steps = mesh, p, int(n_steps)
        self.dt = p["t_end"] / self.n_steps
        if isinstance(mesh, BoxMesh):
            self.M, self.K = fem.assemble(mesh, G)
            self.F_box = fem.box_load(mesh, p["stim_lo"], p["stim_hi"])
        else:  # P1 tetrahedra (oracle/tetfem.py): own assembly, ball stimulus
            self.M, self.K = mesh.assemble(G)
            self.F_box = mesh.stim_load(p)
        self.A = (self.M + 0.5 * self.dt * self.K).tocsr()
        self.B = (self.M - 0.5 * self.dt * self.K).tocsr()
        self.source = source  # optional callable t -> load vector (manufactured solutions)
        self.w = fem.node_weights(self.M)
        self.lin_iters = 0  # linear-solver iterations (a direct solve counts as one)

    def load(self, t):
        F = stim_rate(t, self.p) * self.F_box
        if self.source is not None:
            F = F + self.source(t)
        return F

    def rhs(self, k, u_k):
        t0, t1 = k * self.dt, (k + 1) * self.dt
        return self.B @ u_k + 0.5 * self.dt * (self.load(t1) + self.load(t0))

    def G(self, u):
        return self.A @ u + self.dt * (self.M @ i_ion(u, self.p))

    def jacobian(self, u):
        return (self.A + self.dt * (self.M @ sp.diags(di_ion(u, self.p)))).tocsc()

    def linsolve(self, J, r):
        n = r.shape[0]
        if n <= DIRECT_MAX_NODES:
            self.lin_iters += 1
            return spla.splu(J).solve(r)
        dinv = 1.0 / J.diagonal()
        pre = spla.LinearOperator(J.shape, matvec=lambda v: dinv * v)

        def count(_):
            self.lin_iters += 1

        x, _ = spla.gmres(J, r, M=pre, rtol=1e-14, atol=0.0, restart=200, maxiter=5, callback=count,
                          callback_type="pr_norm")
        return x  # Newton's own residual test decides convergence


def backward_error(Gu, b, F):
    den = np.linalg.norm(Gu) + np.linalg.norm(b)
    return 0.0 if den == 0.0 else np.linalg.norm(F) / den


def newton_step(prob: Problem, b, u0, tol, max_newton=30):
    u = u0.copy()
    for it in range(max_newton + 1):
        Gu = prob.G(u)
        F = Gu - b
        if backward_error(Gu, b, F) <= tol:
            return u, it
        if it == max_newton:
            break
        u = u + prob.linsolve(prob.jacobian(u), -F)
    raise RuntimeError("oracle Newton did not converge")


def solve(mesh: BoxMesh, G, p, n_steps, tol=1e-13, source=None, keep_all=False, max_newton=30,
          stop_after=None, u0=None):
    """Time-step one sample.  Returns a dict with the final state, activation times and QoIs.

    ``stop_after`` truncates the run after that many steps (used for timing samples
    and for parity checks on large meshes); QoIs then refer to that time.
    ``u0`` replaces the zero initial state (only for manufactured solutions and
    invariance checks).
    """
    prob = Problem(mesh, G, p, n_steps, source=source)
    n, dt = mesh.n_nodes, prob.dt
    steps = prob.n_steps if stop_after is None else min(int(stop_after), prob.n_steps)
    u_k = np.zeros(n) if u0 is None else np.array(u0, dtype=np.float64)
    act = np.full(n, np.nan)
    act[u_k >= p["u_th"]] = 0.0
    newton_its = []
    history = [u_k.copy()] if keep_all else None
    for k in range(steps):
        b = prob.rhs(k, u_k)
        u, its = newton_step(prob, b, u_k, tol, max_newton)
        newton_its.append(its)
        # activation: first crossing of u_th, linear in time between the two nodes
        cross = np.isnan(act) & (u_k < p["u_th"]) & (u >= p["u_th"])
        act[cross] = k * dt + dt * (p["u_th"] - u_k[cross]) / (u[cross] - u_k[cross])
        u_k = u
        if keep_all:
            history.append(u_k.copy())
    t_stop = steps * dt
    act_c = np.where(np.isnan(act), t_stop, act)
    vol = float(prob.w.sum())
    out = dict(u=u_k, act=act, act_censored=act_c, dt=dt, t_stop=t_stop,
               mean_u_final=float(prob.w @ u_k) / vol,
               mean_act=float(prob.w @ act_c) / vol,
               newton_iters=np.array(newton_its), lin_iters=prob.lin_iters, w=prob.w)
    if keep_all:
        out["history"] = np.array(history)
    return out


def qoi_value(out, qoi):
    return out["mean_u_final"] if qoi == 0 else out["mean_act"]
