"""Pins of the P1 tetrahedral oracle (oracle/tetfem.py) and the shell generator.

Each check is fixed by mathematics independent of the formulas under test:
quadrature of polynomials, exact reproduction of linear functions, the patch test,
energy identities and brute-force point location.
"""
import numpy as np
import pytest

import workloads as W
from workloads import tetshell
from oracle import kl, stepper
from oracle.tetfem import TetMesh


@pytest.fixture(scope="module")
def shell():
    xyz, tets, ec, el, th0 = tetshell.shell_mesh((2, 6, 12), seed=5)
    return TetMesh(xyz, tets), ec, el, th0


def _quad_tet(p, f):
    """Integral of f over the tetrahedron with vertices p (4, 3) by the 5-point degree-3
    rule (Keast): -4/5 at the centroid, 9/20 at the points (1/2, 1/6, 1/6, 1/6)."""
    vol = abs(np.linalg.det(p[1:] - p[0])) / 6.0
    pts = [(0.25, 0.25, 0.25, 0.25, -0.8)]
    for k in range(4):
        b = [1.0 / 6.0] * 4
        b[k] = 0.5
        pts.append((*b, 0.45))
    return vol * sum(w * f(np.array(b) @ p) for *b, w in pts)


def test_shell_generator(shell):
    mesh, ec, el, th0 = shell
    assert mesh.vol.min() > 0
    # the frame is orthonormal and tangent to the confocal spheroid through the centroid
    assert np.allclose(np.einsum("ij,ij->i", ec, el), 0.0, atol=1e-14)
    assert np.allclose(np.linalg.norm(ec, axis=1), 1.0) and np.allclose(np.linalg.norm(el, axis=1), 1.0)
    mu, nu, phi = tetshell.xyz_to_spheroidal(mesh.centres)
    back = tetshell.spheroidal_to_xyz(mu, nu, phi)
    assert np.allclose(back, mesh.centres, atol=1e-12)
    # rule-based angle within [-60, 60] degrees, +60 near the epicardium
    assert th0.min() >= np.deg2rad(-60) - 1e-12 and th0.max() <= np.deg2rad(60) + 1e-12
    # the volume approaches the analytic shell volume as the mesh is refined
    from scipy import integrate
    a = tetshell.A_FOCAL
    V, _ = integrate.dblquad(lambda nu, mu: 2 * np.pi * a ** 3 * np.sinh(mu) * np.sin(nu)
                             * (np.sinh(mu) ** 2 + np.sin(nu) ** 2),
                             tetshell.MU_ENDO, tetshell.MU_EPI, tetshell.NU_APEX, tetshell.NU_BASE)
    fine = TetMesh(*tetshell.shell_mesh((3, 16, 32), seed=5)[:2])
    assert abs(fine.volume - V) < abs(mesh.volume - V) and abs(fine.volume - V) < 0.02 * V


def test_levels_are_not_nested():
    c = TetMesh(*tetshell.shell_mesh((2, 6, 12), seed=5)[:2])
    f = TetMesh(*tetshell.shell_mesh((4, 12, 24), seed=5)[:2])
    d = np.linalg.norm(c.nodes[:, None, :] - f.nodes[None, :, :], axis=2).min(axis=1)
    interior = np.ones(c.n_nodes, dtype=bool)
    mu, nu, _ = tetshell.xyz_to_spheroidal(c.nodes)
    interior &= (mu > tetshell.MU_ENDO + 1e-9) & (mu < tetshell.MU_EPI - 1e-9)
    interior &= (nu > tetshell.NU_APEX + 1e-9) & (nu < tetshell.NU_BASE - 1e-9)
    assert (d[interior] > 1e-6).all()


def test_mass_matches_quadrature(shell):
    mesh, *_ = shell
    M, _ = mesh.assemble(np.zeros((mesh.n_elems, 3, 3)))
    for t in (0, 17, mesh.n_elems - 1):
        # a one-element mesh: its assembled mass is the element matrix; phi_a phi_b is
        # quadratic, so the degree-3 rule integrates it exactly
        p = mesh.nodes[mesh.elems[t]]
        one_tet = TetMesh(p, np.array([[0, 1, 2, 3]]))
        Ms = one_tet.assemble(np.zeros((1, 3, 3)))[0].toarray()
        Me = np.array([[_quad_tet(p, lambda x, a=a, b=b: np.prod(one_tet.barycentric(x, np.array([0]))[0][[a, b]]))
                        for b in range(4)] for a in range(4)])
        assert np.abs(Ms - Me).max() < 1e-13 * Me.max()  # the rule has a negative weight: mild cancellation
    # total mass integrates 1; x^T M x integrates a linear function squared exactly
    one = np.ones(mesh.n_nodes)
    assert abs(one @ M @ one - mesh.volume) < 1e-13 * mesh.volume
    c = np.array([0.3, -0.7, 1.1])
    u = mesh.nodes @ c + 0.2
    exact = sum(_quad_tet(mesh.nodes[mesh.elems[t]], lambda x: (x @ c + 0.2) ** 2) for t in range(mesh.n_elems))
    assert abs(u @ M @ u - exact) < 1e-12 * exact


def test_stiffness_energy_and_patch_test(shell):
    mesh, ec, el, th0 = shell
    ph = W.physics(3)
    G = mesh.conductivity(th0, ec, el, ph["sigma_l"], ph["sigma_t"])
    _, K = mesh.assemble(G)
    assert np.abs(K @ np.ones(mesh.n_nodes)).max() < 1e-14 * abs(K).max()   # constants in the kernel
    assert abs(K - K.T).max() < 1e-16
    c = np.array([0.5, 0.25, -1.0])
    u = mesh.nodes @ c
    energy = sum(mesh.vol[t] * c @ G[t] @ c for t in range(mesh.n_elems))
    assert abs(u @ K @ u - energy) < 1e-12 * energy
    # patch test: a linear field has zero flux imbalance at interior vertices (isotropic G)
    _, K1 = mesh.assemble(np.broadcast_to(np.eye(3), (mesh.n_elems, 3, 3)).copy())
    mu, nu, _ = tetshell.xyz_to_spheroidal(mesh.nodes)
    inner = (mu > tetshell.MU_ENDO + 1e-9) & (mu < tetshell.MU_EPI - 1e-9) & \
            (nu > tetshell.NU_APEX + 1e-9) & (nu < tetshell.NU_BASE - 1e-9)
    assert inner.any()
    assert np.abs((K1 @ u)[inner]).max() < 1e-13


def test_fibre_conductivity_eigenstructure(shell):
    mesh, ec, el, _ = shell
    ph = W.physics(3)
    th = np.full(mesh.n_elems, 0.4)
    G = mesh.conductivity(th, ec, el, ph["sigma_l"], ph["sigma_t"])
    f = np.cos(0.4) * ec + np.sin(0.4) * el
    n = np.cross(ec, el)
    assert np.allclose(np.einsum("tij,tj->ti", G, f), ph["sigma_l"] * f, atol=1e-18)
    assert np.allclose(np.einsum("tij,tj->ti", G, n), ph["sigma_t"] * n, atol=1e-18)


def test_locate_and_interpolate(shell):
    mesh, *_ = shell
    rng = np.random.default_rng(3)
    t = rng.integers(0, mesh.n_elems, 40)
    b = rng.dirichlet(np.ones(4), 40)
    pts = np.einsum("pa,pam->pm", b, mesh.nodes[mesh.elems[t]])
    # brute force: a tetrahedron containing the point (all barycentric >= -1e-12)
    tet, w = mesh.locate(pts)
    for q in range(pts.shape[0]):
        lam = mesh.barycentric(pts[q], np.array([tet[q]]))[0]
        assert lam.min() >= -1e-12
    # linear functions are reproduced exactly
    c = np.array([1.0, -2.0, 0.5])
    vals = mesh.interpolate(mesh.nodes @ c + 3.0, pts)
    assert np.allclose(vals, pts @ c + 3.0, atol=1e-12)
    # a point outside the mesh takes the best tetrahedron, with clipped weights
    out = np.array([[0.0, 0.0, tetshell.LONG_AXIS + 0.05]])
    to, wo = mesh.locate(out)
    assert wo.min() >= 0 and abs(wo.sum() - 1) < 1e-15


def test_tet_solve_isotropic_invariance_and_kl(shell):
    mesh, ec, el, th0 = shell
    ph = W.physics(3)
    c, r = tetshell.stimulus_ball(0.3)
    ph.update(stim_center=c.tolist(), stim_radius=float(r))
    ph["sigma_t"] = ph["sigma_l"]
    outs = []
    for seed in (1, 2):
        th = W.random_angles(seed, 1, mesh.n_elems)[0]
        G = mesh.conductivity(th, ec, el, ph["sigma_l"], ph["sigma_t"])
        outs.append(stepper.solve(mesh, G, ph, 8))
    assert np.allclose(outs[0]["u"], outs[1]["u"], rtol=0, atol=1e-12 * np.abs(outs[0]["u"]).max())
    assert np.abs(outs[0]["u"]).max() > 0
    # KL on the tetrahedral nodes: M-orthonormal modes
    M, _ = mesh.assemble(np.zeros((mesh.n_elems, 3, 3)))
    lam, psi = kl.kl_modes(mesh, M, 0.3, 0.5, 6)
    assert np.allclose(psi.T @ (M @ psi), np.eye(6), atol=1e-10)
    assert (np.diff(lam) <= 0).all()
