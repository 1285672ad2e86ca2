"""Pins of the oracle's field quantities of interest and transfers (Section 2.4; Section 5,
error measures).

* the space-time transfer reproduces exactly every function that is trilinear (bilinear) in
  space times linear in time, at several refinement ratios, and is the identity onto the same
  grids;
* the action potential at a node is that node's history, at a cell centre the mean of the
  corners;
* with one level, the field estimate is the sample mean; with a second level whose fine and
  coarse fields coincide after transfer, the correction vanishes;
* the activation map is the per-node activation time, censored at the stop time.
"""
import numpy as np
import pytest

from oracle import fields, stepper
from oracle.fem import conductivity_iso
from oracle.mesh import BoxMesh


def _affine_st(nodes, t, c):
    """A function trilinear in space times linear in time (products of coordinates included)."""
    x = nodes[:, 0]
    y = nodes[:, 1]
    z = nodes[:, 2] if nodes.shape[1] > 2 else 0.0 * x
    sp = c[0] + c[1] * x + c[2] * y + c[3] * z + c[4] * x * y + c[5] * y * z + c[6] * x * z + c[7] * x * y * z
    sp2 = c[8] + c[9] * x - c[10] * x * y * z
    return np.outer(np.ones_like(t), sp) + np.outer(t, sp2)


@pytest.mark.parametrize("nc,nf,mc,mf", [([3, 4, 2], [5, 7, 3], 2, 6), ([5, 5, 5], [9, 9, 9], 4, 8),
                                         ([4, 3], [10, 5], 3, 9)])
def test_space_time_transfer_exact_for_multilinear_times_linear(nc, nf, mc, mf):
    rng = np.random.default_rng(1)
    d = len(nc)
    hi = [1.0, 0.7, 1.3][:d]
    Mc, Mf = BoxMesh(nc, hi=hi), BoxMesh(nf, hi=hi)
    T = 0.32
    c = rng.normal(size=11)
    Fc = _affine_st(Mc.nodes, np.linspace(0, T, mc + 1), c)
    Ff = _affine_st(Mf.nodes, np.linspace(0, T, mf + 1), c)
    P = fields.prolongate_space_time(Mc, mc, Fc, Mf, mf, T)
    assert P.shape == Ff.shape
    assert np.abs(P - Ff).max() <= 1e-13 * np.abs(Ff).max()
    same = fields.prolongate_space_time(Mc, mc, Fc, Mc, mc, T)
    assert np.abs(same - Fc).max() <= 1e-15 * np.abs(Fc).max()


def test_transfer_detects_a_nonlinear_time_profile():
    """A quadratic in t is not reproduced between the coarse time nodes (the pin above is not
    satisfied by an operator that ignores time)."""
    Mc = BoxMesh([3, 3, 3])
    t = np.linspace(0, 1, 3)
    Fc = np.outer(t ** 2, np.ones(Mc.n_nodes))
    P = fields.prolongate_space_time(Mc, 2, Fc, Mc, 4, 1.0)
    assert np.allclose(P[1], 0.125) and np.allclose(P[2], 0.25) and np.allclose(P[3], 0.625)


def _solve(n=5, steps=12):
    from workloads import physics
    mesh = BoxMesh([n] * 3)
    ph = physics(3)
    v = np.full(mesh.n_elems, 3.325e-2)
    return mesh, ph, stepper.solve(mesh, conductivity_iso(v, 3), ph, steps, tol=1e-13, keep_all=True)


def test_action_potential_and_activation_map():
    mesh, ph, out = _solve()
    H = fields.space_time_field(out)
    assert H.shape == (13, mesh.n_nodes) and np.all(H[0] == 0.0)
    ap = fields.action_potential(mesh, out, mesh.nodes[[0, 7, 30]])
    assert np.allclose(ap, H[:, [0, 7, 30]].T, rtol=0, atol=1e-15)
    centre = mesh.lo + 0.5 * mesh.h
    ap_c = fields.action_potential(mesh, out, centre[None, :])[0]
    corners = [mesh.node_id(np.array([[i, j, k]]))[0] for i in (0, 1) for j in (0, 1) for k in (0, 1)]
    assert np.allclose(ap_c, H[:, corners].mean(axis=1), rtol=0, atol=1e-14 * np.abs(H).max())
    a = fields.activation_map(out)
    assert np.all((a > 0) & (a <= out["t_stop"]))
    hit = ~np.isnan(out["act"])
    assert hit.any() and (~hit).any()
    assert np.array_equal(a[~hit], np.full((~hit).sum(), out["t_stop"]))
    # the first crossing lies between the two time nodes that bracket it
    for i in np.flatnonzero(hit)[:20]:
        k = int(np.floor(a[i] / out["dt"] - 1e-12))
        assert H[k, i] < ph["u_th"] <= H[k + 1, i]


def test_field_estimator_mean_and_vanishing_correction():
    rng = np.random.default_rng(2)
    Mc, Mf = BoxMesh([3, 3, 3]), BoxMesh([5, 5, 5])
    T = 1.0

    def tr(j, F):
        return F if j == 1 else fields.prolongate_space_time(Mc, 2, F, Mf, 4, T)
    f0 = [rng.normal(size=(3, Mc.n_nodes)) for _ in range(4)]
    est1 = fields.mlmc_field([sum(f0)], [None], [4], lambda j, F: F)
    assert np.allclose(est1, np.mean(f0, axis=0), rtol=1e-15, atol=1e-15)
    # level-1 fine fields equal to the transferred coarse ones: the correction is zero
    g = [rng.normal(size=(3, Mc.n_nodes)) for _ in range(2)]
    fine = sum(fields.prolongate_space_time(Mc, 2, x, Mf, 4, T) for x in g)
    est2 = fields.mlmc_field([sum(f0), fine], [None, sum(g)], [4, 2], tr)
    assert np.allclose(est2, tr(0, sum(f0)) / 4, rtol=0, atol=1e-14)


@pytest.mark.parametrize("n,hi", [([4, 5, 3], [1.0, 0.7, 1.3]), ([6, 4], [0.5, 2.0])])
def test_space_time_norms_closed_forms(n, hi):
    """Exact integrals of functions the space-time interpolant reproduces: a constant c gives
    c^2 |D| T in both norms; f = t gives |D| T^3 / 3; f = g . x (constant in time) gives
    T (int (g.x)^2 + |g|^2 |D|) in H^1; the L^2 part of that by the 1D integrals of x^2."""
    mesh = BoxMesh(n, hi=hi)
    d = mesh.d
    vol = float(np.prod(hi))
    T, m = 0.32, 7
    t = np.linspace(0, T, m + 1)
    c = 1.7
    F = np.full((m + 1, mesh.n_nodes), c)
    for q in (0, 1):
        assert np.isclose(fields.space_time_norm2(mesh, F, T, q), c * c * vol * T, rtol=1e-13)
    F = np.outer(t, np.ones(mesh.n_nodes))
    assert np.isclose(fields.space_time_norm2(mesh, F, T, 1), vol * T ** 3 / 3, rtol=1e-13)
    g = np.array([0.3, -1.1, 0.7])[:d]
    F = np.outer(np.ones(m + 1), mesh.nodes @ g)
    # int_D (g.x)^2 over a box [0, L]: sum_a g_a^2 L_a^3/3 prod_{b != a} L_b + sum_{a<b} g_a g_b L_a^2 L_b^2/2 prod_rest
    L = np.array(hi)
    l2 = 0.0
    for a in range(d):
        l2 += g[a] ** 2 * L[a] ** 3 / 3 * np.prod(np.delete(L, a))
        for b in range(a + 1, d):
            l2 += 2 * g[a] * g[b] * (L[a] ** 2 / 2) * (L[b] ** 2 / 2) * np.prod(np.delete(L, [a, b]))
    # Q1 interpolates g.x exactly but the mass of Q1 integrates (g.x)^2 exactly too (it is in Q2)
    assert np.isclose(fields.space_time_norm2(mesh, F, T, 0), T * l2, rtol=1e-12)
    assert np.isclose(fields.space_time_norm2(mesh, F, T, 1), T * (l2 + (g @ g) * vol), rtol=1e-12)


def test_time_norms_closed_forms():
    T, m = 0.32, 9
    t = np.linspace(0, T, m + 1)
    S = np.stack([np.full(m + 1, 2.0), t, 3.0 - 5.0 * t])
    l2 = fields.time_norm2(S, T, 0)
    h1 = fields.time_norm2(S, T, 1)
    assert np.allclose(l2, [4 * T, T ** 3 / 3, 9 * T - 15 * T ** 2 + 25 * T ** 3 / 3], rtol=1e-13)
    assert np.allclose(h1 - l2, [0.0, T, 25 * T], rtol=1e-13, atol=1e-15)
