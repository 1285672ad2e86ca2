"""Pins of the oracle's space-time solve (Sections 3.1-3.3) and QoIs (Section 2.4).

* constant states of the zero-current model and the rest / threshold / peak
  fixed points of eq. (ionic_term);
* a spatially uniform stimulus reduces eq. (mono_disc) to a scalar recurrence,
  solved here by bisection;
* alpha = 0: Crank-Nicolson in the generalised eigenbasis of (K, M);
* the all-at-once Newton on eq. (system_C) + eq. (mono_disc) equals time stepping;
* manufactured solutions: spatial order 2, temporal order 2 (alpha = 0) and 1
  (alpha > 0, the reaction sits at the new time level);
* isotropy (sigma_l = sigma_t) makes the solution independent of the angle;
  theta and theta + pi give the same conductivity.
"""
import numpy as np
import pytest
import scipy.linalg as sla

import workloads as W
from oracle import allatonce, fem, stepper
from oracle.ionic import di_ion, i_ion
from oracle.mesh import BoxMesh


def phys(d=2, **kw):
    p = W.physics(d)
    p.update(kw)
    return p


def G_of(mesh, theta, p):
    return fem.conductivity_from_angle(theta, mesh.d, p["sigma_l"], p["sigma_t"])


def test_ionic_roots_and_derivative():
    p = phys()
    for r in (p["u_rest"], p["u_th"], p["u_peak"]):
        assert i_ion(np.array([r]), p)[0] == 0.0
    u = np.linspace(-20, 140, 33)
    cs = np.imag(i_ion(u + 1e-30j, p)) / 1e-30  # complex-step derivative, exact to rounding
    assert np.allclose(di_ion(u, p), cs, rtol=1e-14, atol=1e-16)
    # the minimum of I_ion' (non-uniqueness bound of the step equation) is about -5.035
    umin = (p["u_rest"] + p["u_th"] + p["u_peak"]) / 3.0
    assert abs(di_ion(np.array([umin]), p)[0] + 5.0353) < 1e-3


@pytest.mark.parametrize("alpha,c", [(0.0, 3.7), (W.ALPHA, 0.0), (W.ALPHA, W.U_TH), (W.ALPHA, W.U_PEAK)])
def test_constant_states(alpha, c):
    mesh = BoxMesh([5, 6])
    p = phys(alpha=alpha, stim_amp=0.0)
    theta = np.random.default_rng(0).normal(size=mesh.n_elems)
    out = stepper.solve(mesh, G_of(mesh, theta, p), p, 10, u0=np.full(mesh.n_nodes, c))
    assert np.abs(out["u"] - c).max() <= 1e-12 * max(1.0, c)


def _scalar_recurrence(p, n_steps, amp_fn):
    """u_{k+1} + dt I(u_{k+1}) = u_k + dt/2 (s_k + s_{k+1}), root by bisection."""
    dt = p["t_end"] / n_steps
    us = [0.0]
    for k in range(n_steps):
        rhs = us[-1] + 0.5 * dt * (amp_fn(k * dt) + amp_fn((k + 1) * dt))
        f = lambda v: v + dt * float(i_ion(np.array([v]), p)[0]) - rhs
        lo, hi = -50.0, 200.0
        for _ in range(200):
            mid = 0.5 * (lo + hi)
            if f(mid) > 0:
                hi = mid
            else:
                lo = mid
        us.append(0.5 * (lo + hi))
    return np.array(us)


def test_uniform_stimulus_scalar_recurrence_and_activation():
    mesh = BoxMesh([4, 5])
    n_steps = 64
    p = phys(stim_lo=[-1, -1], stim_hi=[2, 2], stim_amp=W.U_PEAK * 0.4 / (0.02 * W.T_END))
    theta = np.random.default_rng(5).normal(size=mesh.n_elems)
    out = stepper.solve(mesh, G_of(mesh, theta, p), p, n_steps, keep_all=True)
    ref = _scalar_recurrence(p, n_steps, lambda t: stepper.stim_rate(t, p))
    assert np.abs(out["history"] - ref[:, None]).max() < 2e-12 * np.abs(ref).max()
    # activation: first k with u_k < u_th <= u_{k+1}, linear interpolation in time
    dt = p["t_end"] / n_steps
    k = int(np.argmax(ref >= p["u_th"])) - 1
    assert k >= 0
    t_act = k * dt + dt * (p["u_th"] - ref[k]) / (ref[k + 1] - ref[k])
    assert np.allclose(out["act"], t_act, rtol=1e-9)
    assert abs(out["mean_act"] - t_act) < 1e-9


def test_linear_case_matches_generalised_eigen_cn():
    mesh = BoxMesh([6, 5], hi=[1.0, 0.8])
    n_steps = 20
    p = phys(alpha=0.0, sigma_l=0.05, sigma_t=0.01)
    theta = np.random.default_rng(6).normal(size=mesh.n_elems)
    G = G_of(mesh, theta, p)
    out = stepper.solve(mesh, G, p, n_steps)
    M, K = fem.assemble(mesh, G)
    lam, Phi = sla.eigh(K.toarray(), M.toarray())  # K Phi = M Phi diag(lam), Phi^T M Phi = I
    F = fem.box_load(mesh, p["stim_lo"], p["stim_hi"])
    dt = p["t_end"] / n_steps
    xi = np.zeros(mesh.n_nodes)
    g = Phi.T @ F
    for k in range(n_steps):
        c = 0.5 * dt * (stepper.stim_rate((k + 1) * dt, p) + stepper.stim_rate(k * dt, p))
        xi = ((1 - 0.5 * dt * lam) * xi + c * g) / (1 + 0.5 * dt * lam)
    u_ref = Phi @ xi
    assert np.abs(out["u"] - u_ref).max() < 1e-11 * np.abs(u_ref).max()


def test_all_at_once_equals_time_stepping():
    mesh = BoxMesh([5, 5], hi=[0.2, 0.2])
    n_steps = 8
    p = phys(sigma_l=0.01, sigma_t=0.004, t_end=0.04, stim_t_off=0.01, stim_amp=W.U_PEAK / 0.01)
    theta = np.random.default_rng(7).normal(size=mesh.n_elems)
    G = G_of(mesh, theta, p)
    ts = stepper.solve(mesh, G, p, n_steps, keep_all=True)["history"][1:]
    aa = allatonce.solve_all_at_once(mesh, G, p, n_steps)
    assert np.abs(ts).max() > W.U_TH  # the reaction is active
    assert np.abs(ts - aa).max() < 1e-11 * np.abs(ts).max()


def _mms(n, n_steps, alpha, t_end=0.2):
    """u* = (1 + t) cos(pi x) cos(pi y) on [0,1]^2, G = diag(sigma_l, sigma_t) (theta = 0)."""
    p = phys(alpha=alpha, u_rest=0.0, u_th=0.5, u_peak=1.0, sigma_l=0.3, sigma_t=0.1,
             t_end=t_end, stim_amp=0.0)
    mesh = BoxMesh([n, n])
    G = G_of(mesh, np.zeros(mesh.n_elems), p)
    cc = lambda X: np.cos(np.pi * X[:, 0]) * np.cos(np.pi * X[:, 1])
    ustar = lambda X, t: (1.0 + t) * cc(X)

    def f(X, t):
        u = ustar(X, t)
        return cc(X) + np.pi ** 2 * (p["sigma_l"] + p["sigma_t"]) * u + i_ion(u, p)

    source = lambda t: fem.source_load(mesh, lambda X: f(X, t))
    out = stepper.solve(mesh, G, p, n_steps, source=source, u0=ustar(mesh.nodes, 0.0))
    M = fem.assemble_mass(mesh)
    e = out["u"] - ustar(mesh.nodes, t_end)
    return np.sqrt(e @ (M @ e)), out["u"], mesh


def test_mms_spatial_order_two():
    errs = [_mms(n, 200, 0.0)[0] for n in (5, 9, 17)]
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(rates > 1.85), rates


@pytest.mark.parametrize("alpha,order", [(0.0, 2), (2.0, 1)])
def test_mms_temporal_order(alpha, order):
    us = [_mms(9, m, alpha, t_end=0.5)[1] for m in (4, 8, 16, 32)]
    d = [np.abs(us[i] - us[i + 1]).max() for i in range(3)]
    rates = np.log2(np.array(d[:-1]) / np.array(d[1:]))
    assert np.all(np.abs(rates - order) < 0.25), rates


def test_isotropic_field_gives_identical_samples():
    mesh = BoxMesh([5, 5, 4])
    p = phys(3, sigma_t=W.SIGMA_L)
    rng = np.random.default_rng(8)
    outs = [stepper.solve(mesh, G_of(mesh, rng.normal(size=mesh.n_elems), p), p, 12) for _ in range(3)]
    for o in outs[1:]:
        assert np.abs(o["u"] - outs[0]["u"]).max() < 1e-13 * np.abs(outs[0]["u"]).max()
        assert o["mean_act"] == pytest.approx(outs[0]["mean_act"], rel=1e-13)


def test_angle_shift_by_pi_is_a_symmetry():
    mesh = BoxMesh([6, 5])
    p = phys()
    th = np.random.default_rng(9).normal(size=mesh.n_elems)
    a = stepper.solve(mesh, G_of(mesh, th, p), p, 16)
    b = stepper.solve(mesh, G_of(mesh, th + np.pi, p), p, 16)
    assert np.abs(a["u"] - b["u"]).max() < 1e-11 * np.abs(a["u"]).max()
