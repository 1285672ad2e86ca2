"""Pins of the oracle's finite-element pieces against facts fixed by the mathematics.

Conductivity: eq. (AdmV) and its ellipticity lemma (eigenvalues g and |V|).
Mass / stiffness: Section 3.1 (semi-disc); closed Kronecker forms on uniform
Q1 boxes, zero row sums (Neumann problem), exact energy of linear functions.
"""
import numpy as np
import pytest

import workloads as W
from oracle import fem
from oracle.mesh import BoxMesh


def _m1(n, h):
    """1D Q1 mass: h/6 tridiag(1, 4, 1) with 2 on the two end diagonals."""
    M = np.diag(np.full(n, 4.0)) + np.diag(np.ones(n - 1), 1) + np.diag(np.ones(n - 1), -1)
    M[0, 0] = M[-1, -1] = 2.0
    return M * h / 6.0


def _k1(n, h):
    K = np.diag(np.full(n, 2.0)) - np.diag(np.ones(n - 1), 1) - np.diag(np.ones(n - 1), -1)
    K[0, 0] = K[-1, -1] = 1.0
    return K / h


def _c1(n):
    """1D C[i, j] = int phi_i phi_j' : 1/2 (e_{i,i+1} - e_{i,i-1}), -1/2 / +1/2 at the ends."""
    C = 0.5 * (np.diag(np.ones(n - 1), 1) - np.diag(np.ones(n - 1), -1))
    C[0, 0] = -0.5
    C[-1, -1] = 0.5
    return C


def _kron(mats):
    """Kronecker product with axis 0 fastest: mats = [A_x, A_y, (A_z)]."""
    out = mats[0]
    for A in mats[1:]:
        out = np.kron(A, out)
    return out


@pytest.mark.parametrize("d,n", [(2, [5, 4]), (3, [4, 3, 5])])
def test_stiffness_row_sums_symmetry_psd(d, n):
    mesh = BoxMesh(n)
    theta = np.random.default_rng(1).normal(size=mesh.n_elems)
    G = fem.conductivity_from_angle(theta, d, W.SIGMA_L, W.SIGMA_T)
    M, K = fem.assemble(mesh, G)
    K = K.toarray()
    assert np.abs(K @ np.ones(mesh.n_nodes)).max() < 1e-16
    assert np.abs(K - K.T).max() < 1e-18
    ev = np.linalg.eigvalsh(K)
    assert ev.min() > -1e-16 and np.sum(ev < 1e-14) == 1  # kernel = constants only
    assert abs(M.sum() - mesh.volume) < 1e-15


@pytest.mark.parametrize("d", [2, 3])
def test_mass_is_kronecker_of_1d_masses(d):
    n = [5, 4, 3][:d]
    mesh = BoxMesh(n, hi=[1.0, 0.5, 2.0][:d])
    M = fem.assemble_mass(mesh).toarray()
    ref = _kron([_m1(n[a], mesh.h[a]) for a in range(d)])
    assert np.abs(M - ref).max() < 1e-16


@pytest.mark.parametrize("theta", [0.0, 0.3, np.pi / 4, 1.2, -2.0])
def test_stiffness_closed_form_uniform_angle_3d(theta):
    n = [4, 5, 3]
    mesh = BoxMesh(n, hi=[1.0, 1.5, 0.75])
    h = mesh.h
    G1 = fem.conductivity_from_angle(np.array([theta]), 3, W.SIGMA_L, W.SIGMA_T)[0]
    _, K = fem.assemble(mesh, np.broadcast_to(G1, (mesh.n_elems, 3, 3)))
    M1 = [_m1(n[a], h[a]) for a in range(3)]
    K1 = [_k1(n[a], h[a]) for a in range(3)]
    C1 = [_c1(n[a]) for a in range(3)]
    ref = np.zeros((mesh.n_nodes, mesh.n_nodes))
    # int d_q phi_j d_p phi_i : factor per axis a is K1 if a == p == q, C1^T if a == p != q,
    # C1 if a == q != p, M1 otherwise
    for p in range(3):
        for q in range(3):
            mats = []
            for a in range(3):
                if a == p and a == q:
                    mats.append(K1[a])
                elif a == p:
                    mats.append(C1[a].T)
                elif a == q:
                    mats.append(C1[a])
                else:
                    mats.append(M1[a])
            ref += G1[p, q] * _kron(mats)
    assert np.abs(K.toarray() - ref).max() < 1e-17


@pytest.mark.parametrize("d", [2, 3])
def test_energy_of_linear_functions(d):
    """Q1 contains linear u = g.x, so u^T K u = |D| g^T G g exactly for uniform G."""
    mesh = BoxMesh([4, 6, 3][:d], lo=[-0.5] * d, hi=[0.5, 1.0, 0.7][:d])
    rng = np.random.default_rng(3)
    for theta in (0.0, 0.7, 2.5):
        G1 = fem.conductivity_from_angle(np.array([theta]), d, W.SIGMA_L, W.SIGMA_T)[0]
        _, K = fem.assemble(mesh, np.broadcast_to(G1, (mesh.n_elems, d, d)))
        g = rng.normal(size=d)
        u = mesh.nodes @ g
        assert np.isclose(u @ (K @ u), mesh.volume * g @ G1 @ g, rtol=1e-13, atol=0)


def test_conductivity_ellipticity_lemma():
    """eq. (AdmV): eigenvalues g (d-1 times) and |V|, eigenvector of |V| along V."""
    rng = np.random.default_rng(4)
    for d in (2, 3):
        for _ in range(20):
            V = rng.normal(size=d)
            g = rng.uniform(0.1, 2.0)
            G = fem.conductivity(V, g)
            ev = np.sort(np.linalg.eigvalsh(G))
            ref = np.sort(np.r_[np.full(d - 1, g), np.linalg.norm(V)])
            assert np.allclose(ev, ref, rtol=1e-13, atol=0)
            assert np.allclose(G @ V, np.linalg.norm(V) * V, rtol=1e-13)
    # the angle form: fibre direction has eigenvalue sigma_l, its normal sigma_t
    th = 0.83
    G = fem.conductivity_from_angle(np.array([th]), 2, 2.0, 0.5)[0]
    f, nrm = np.array([np.cos(th), np.sin(th)]), np.array([-np.sin(th), np.cos(th)])
    assert np.allclose(G @ f, 2.0 * f, rtol=1e-14) and np.allclose(G @ nrm, 0.5 * nrm, rtol=1e-14)


def test_box_load_exact():
    mesh = BoxMesh([5, 3], hi=[1.0, 1.0])  # h = 0.25, 0.5
    F = fem.box_load(mesh, [0.0, 0.0], [0.1, 0.3])
    assert np.isclose(F.sum(), 0.1 * 0.3, rtol=1e-14)
    # 1D hat integrals over [0, 0.1] with h = 0.25: node 0: 0.1 - 0.01/0.5 = 0.08, node 1: 0.02
    # over [0, 0.3] with h = 0.5: node 0: 0.3 - 0.09 = 0.21, node 1: 0.09
    fx = np.array([0.08, 0.02, 0, 0, 0])
    fy = np.array([0.21, 0.09, 0.0])
    assert np.allclose(F, np.kron(fy, fx), rtol=1e-14, atol=1e-18)
    # a box covering the domain gives w = M 1
    M = fem.assemble_mass(mesh)
    assert np.allclose(fem.box_load(mesh, [-1, -1], [2, 2]), fem.node_weights(M), rtol=1e-14)


def test_source_load_reproduces_mass_action():
    mesh = BoxMesh([4, 3, 3])
    M = fem.assemble_mass(mesh)
    g = np.array([0.3, -1.0, 2.0])
    F = fem.source_load(mesh, lambda X: X @ g + 0.5)
    assert np.allclose(F, M @ (mesh.nodes @ g + 0.5), rtol=1e-13, atol=1e-16)


def test_row_products_match_assembled():
    """Row-wise products (used on meshes too large to assemble) equal the assembled rows."""
    from oracle.fem import row_products
    for n in ([7, 6, 5], [9, 8]):
        mesh = BoxMesh(n, hi=[1.0, 0.7, 1.2][:len(n)])
        ph = W.physics(len(n))
        th = W.random_angles(11, 1, mesh.n_elems)[0]
        G = fem.conductivity_from_angle(th, mesh.d, ph["sigma_l"], ph["sigma_t"])
        M, K = fem.assemble(mesh, G)
        v1 = W.random_nodal(12, 1, mesh.n_nodes)[0]
        v2 = W.random_nodal(13, 1, mesh.n_nodes)[0]
        rows = np.unique(np.concatenate([[0, mesh.n_nodes - 1, n[0] - 1], np.arange(3, mesh.n_nodes, 7)]))
        Mv, Kv = row_products(mesh, th, ph["sigma_l"], ph["sigma_t"], rows, [v1, v2])
        for k, v in enumerate((v1, v2)):
            np.testing.assert_allclose(Mv[k], (M @ v)[rows], rtol=0, atol=1e-15 * np.abs(M @ v).max())
            np.testing.assert_allclose(Kv[k], (K @ v)[rows], rtol=0, atol=1e-14 * np.abs(K @ v).max())


def test_stiffness_row_bound_holds_for_any_field():
    from oracle.fem import stiffness_row_bound
    mesh = BoxMesh([6, 5, 4], hi=[1.0, 0.7, 1.2])
    ph = W.physics(3)
    bound = stiffness_row_bound(mesh, ph["sigma_l"], ph["sigma_t"])
    worst = 0.0
    for seed in range(6):
        th = W.random_angles(20 + seed, 1, mesh.n_elems)[0]
        if seed == 0:
            th[:] = 0.3  # a uniform field
        G = fem.conductivity_from_angle(th, 3, ph["sigma_l"], ph["sigma_t"])
        _, K = fem.assemble(mesh, G)
        worst = max(worst, np.asarray(abs(K).sum(axis=1)).max())
    assert worst <= bound <= 3.0 * worst


def test_isotropic_scalar_model_equals_isotropic_fibre_model():
    """G = v I (the paper's cube model) equals eq. (AdmV) with sigma_l = sigma_t = v for any
    fibre direction; its assembled stiffness is v times the Laplacian stiffness."""
    from oracle import fem
    mesh = BoxMesh([5, 4, 6])
    rng = np.random.default_rng(2)
    v = 3.3e-3 * (1.0 + 0.3 * rng.uniform(-1, 1, mesh.n_elems))
    th = rng.uniform(0, np.pi, mesh.n_elems)
    Gi = fem.conductivity_iso(v, 3)
    Gf = np.stack([fem.conductivity_from_angle(th[e:e + 1], 3, v[e], v[e])[0] for e in range(mesh.n_elems)])
    assert np.abs(Gi - Gf).max() <= 1e-14 * v.max()  # |V| = v up to rounding
    _, K = fem.assemble(mesh, Gi)
    _, K1 = fem.assemble(mesh, fem.conductivity_iso(np.ones(mesh.n_elems), 3))
    # element by element: K = sum_e v_e K1_e, so a uniform v scales the Laplacian stiffness
    _, Ku = fem.assemble(mesh, fem.conductivity_iso(np.full(mesh.n_elems, 2.5), 3))
    assert abs(Ku - 2.5 * K1).max() < 1e-14 * abs(Ku).max()
    assert np.abs(K @ np.ones(mesh.n_nodes)).max() < 1e-14 * abs(K).max()


def test_isotropic_model_floor():
    """The lower bound b_min of the cube model: a field entirely below it gives b_min times the
    Laplacian stiffness, a field entirely above it is untouched, and the stiffness of a mixed
    field is positive semi-definite with the constants as its only null space (all element
    conductivities positive)."""
    from oracle import fem
    mesh = BoxMesh([4, 5, 3])
    rng = np.random.default_rng(6)
    b = 3.3e-4
    _, K1 = fem.assemble(mesh, fem.conductivity_iso(np.ones(mesh.n_elems), 3))
    _, Klow = fem.assemble(mesh, fem.conductivity_iso(rng.uniform(-2e-3, 0.9 * b, mesh.n_elems), 3, b))
    assert abs(Klow - b * K1).max() <= 1e-14 * b * abs(K1).max()
    v = rng.uniform(1.1 * b, 5e-3, mesh.n_elems)
    assert np.array_equal(fem.conductivity_iso(v, 3, b), fem.conductivity_iso(v, 3))
    vm = 3.3e-3 * (1.0 + 1.5 * rng.uniform(-1, 1, mesh.n_elems))
    assert (vm < 0).any()
    _, Km = fem.assemble(mesh, fem.conductivity_iso(vm, 3, b))
    ev = np.linalg.eigvalsh(Km.toarray() if hasattr(Km, "toarray") else Km)
    assert abs(ev[0]) < 1e-12 * ev[-1] and ev[1] > 1e-6 * ev[-1]


def test_vector_field_conductivity_eigenstructure():
    """eq. (AdmV) for a general vector field: G V = |V| V and G n = g n for n orthogonal to V,
    so G is SPD with eigenvalues g (twice) and |V| whenever V != 0."""
    from oracle import fem
    rng = np.random.default_rng(4)
    V = rng.normal(size=(50, 3)) * 3e-3
    g = 1.625e-3
    G = fem.conductivity(V, g)
    nv = np.linalg.norm(V, axis=1)
    assert np.allclose(np.einsum("eij,ej->ei", G, V), nv[:, None] * V, rtol=0, atol=1e-15 * nv.max() ** 2)
    n = np.cross(V, rng.normal(size=(50, 3)))
    assert np.allclose(np.einsum("eij,ej->ei", G, n), g * n, rtol=0, atol=1e-15 * np.abs(n).max())
    assert np.allclose(G, np.transpose(G, (0, 2, 1)), rtol=0, atol=0)
