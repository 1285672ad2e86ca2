"""Host-side checks of the C ABI (no GPU): the library loads, exports every
symbol of include/mlq.h, validates descriptors, and its host-only routines
(lattice construction, estimators) agree with the oracle."""
import os
import re

import numpy as np
import pytest

import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def mlq():
    lib = os.path.join(ROOT, "paper_2105_02007_amd", "libmlq.so")
    if not os.path.exists(lib):
        pytest.fail("libmlq.so is not built: run __graft_entry__.build()")
    from paper_2105_02007_amd import mlq as m
    return m


def test_exports_every_declared_symbol(mlq):
    header = open(os.path.join(ROOT, "include", "mlq.h")).read()
    declared = set(re.findall(r"\b(mlq_[a-z_0-9]+)\s*\(", header))
    assert declared >= set(mlq.EXPORTED) and len(declared) >= 15
    for name in declared:
        assert hasattr(mlq.lib, name), name


def _desc(mlq, **kw):
    lv = dict(dim=3, n=[9, 9, 9], lo=[0, 0, 0], hi=[1, 1, 1], n_steps=32)
    lv.update({k: v for k, v in kw.items() if k in lv})
    phys = W.physics(3)
    phys.update({k: v for k, v in kw.items() if k in phys})
    rest = {k: v for k, v in kw.items() if k not in lv and k not in phys}
    return mlq.make_desc(lv, phys, **rest)


def _bytes(mlq, d):
    import ctypes as C
    n = C.c_size_t()
    return mlq.lib.mlq_level_bytes(C.byref(d), C.byref(n)), n.value


def test_descriptor_validation(mlq):
    d, _ = _desc(mlq)
    code, nbytes = _bytes(mlq, d)
    assert code == 0 and nbytes >= 2 * 729 * 8
    for bad in (dict(dim=4), dict(n_steps=0), dict(sigma_l=-1.0), dict(max_inner=1000), dict(prec=7),
                dict(qoi=5), dict(newton_tol=0.0), dict(max_batch=0)):
        d, _ = _desc(mlq, **bad)
        assert _bytes(mlq, d)[0] == mlq.MLQ_EINVAL, bad
    # dt * |min I_ion'| >= 1 admits several roots of the step equation
    d, _ = _desc(mlq, n_steps=1, t_end=0.25)
    assert _bytes(mlq, d)[0] == mlq.MLQ_EINVAL
    assert b"several roots" in mlq.lib.mlq_last_error()
    d, _ = _desc(mlq, n_steps=2, t_end=0.25)
    assert _bytes(mlq, d)[0] == 0


@pytest.mark.parametrize("N,s", [(1, 4), (4, 20), (16, 128), (64, 32), (256, 128)])
def test_cbc_bit_exact_with_oracle(mlq, N, s):
    from oracle import qmc
    gamma = 1.0 / (1.0 + np.arange(s)) ** 1.5
    assert np.array_equal(mlq.cbc(N, s, gamma), qmc.cbc(N, s, gamma))


def test_halton_argument_validation(mlq):
    """Invalid Halton requests are refused on the host before anything is enqueued (run where no
    GPU is visible: the pointer below is a placeholder that must never be dereferenced)."""
    import torch
    if torch.cuda.is_available():
        pytest.skip("host-side checks only")
    lib = mlq.lib
    fake = 4096
    assert lib.mlq_halton(4, 1, 8, None, mlq.MLQ_MAP_UNIFORM, None, None) == mlq.MLQ_EINVAL
    for s, first, count, m in [(0, 1, 8, 1), (1025, 1, 8, 1), (4, -1, 8, 1), (4, 1, -1, 1),
                               (4, 2 ** 32 - 3, 4, 1), (4, 1, 8, 2)]:
        assert lib.mlq_halton(s, first, count, None, m, fake, None) == mlq.MLQ_EINVAL, (s, first, count, m)
    assert lib.mlq_halton(4, 5, 0, None, mlq.MLQ_MAP_UNIFORM, fake, None) == mlq.MLQ_OK


def test_estimators_match_oracle(mlq):
    from oracle import estimators as E
    rng = np.random.default_rng(3)
    f = rng.normal(size=50)
    r = mlq.estimate(mlq.MLQ_EST_MC, [f])
    m, s = E.single_level(list(f))
    assert np.isclose(r["estimate"], m, rtol=1e-14) and np.isclose(r["rmse"], s, rtol=1e-13)
    ff = [rng.normal(size=n) for n in (64, 16, 4)]
    fc = [None] + [rng.normal(size=n) for n in (16, 4)]
    r = mlq.estimate(mlq.MLQ_EST_MLMC, ff, fc)
    est, rmse, means, vars_ = E.standard_ml([list(a) for a in ff], [None] + [list(a) for a in fc[1:]])
    assert np.isclose(r["estimate"], est, rtol=1e-14) and np.isclose(r["rmse"], rmse, rtol=1e-13)
    assert np.allclose(r["level_var"], vars_, rtol=1e-13)
    S = 5
    ff = [rng.normal(size=S * n) for n in (8, 2)]
    fc = [None, rng.normal(size=S * 2)]
    r = mlq.estimate(mlq.MLQ_EST_MLQMC, ff, fc, n_per_level=[8, 2], n_shifts=S)
    of = [[list(a[s * n:(s + 1) * n]) for s in range(S)] for a, n in zip(ff, (8, 2))]
    oc = [None, [list(fc[1][s * 2:(s + 1) * 2]) for s in range(S)]]
    est, rmse, _ = E.standard_mlqmc(of, [[None] * S, oc[1]])
    assert np.isclose(r["estimate"], est, rtol=1e-14) and np.isclose(r["rmse"], rmse, rtol=1e-13)
    npts = [4, 8, 16]
    F = [rng.normal(size=16) for _ in range(3)]
    fj = [F[j][:npts[2 - j]] for j in range(3)]
    r = mlq.estimate(mlq.MLQ_EST_COMBINATION, fj, n_per_level=npts)
    assert np.isclose(r["estimate"], E.combination(fj, npts), rtol=1e-14)


def test_tet_locate_matches_oracle(mlq):
    """mlq_tet_locate (host): the P1 interpolant of a random nodal field at the vertices of a
    finer non-nested shell (points inside the coarse mesh and boundary points outside it)
    equals the oracle's brute-force location (1e-12)."""
    from oracle.tetfem import TetMesh
    from workloads import tetshell
    xyz_c, tets_c, _, _, _ = tetshell.shell_mesh((2, 6, 12), seed=3)
    xyz_f, _, _, _, _ = tetshell.shell_mesh((3, 9, 18), seed=4)
    node, w = mlq.tet_locate(dict(xyz=xyz_c, tets=tets_c), xyz_f)
    assert np.allclose(w.sum(axis=1), 1.0) and (w >= 0).all()
    vals = np.random.default_rng(2).normal(size=xyz_c.shape[0])
    got = (w * vals[node]).sum(axis=1)
    ref = TetMesh(xyz_c, tets_c).interpolate(vals, xyz_f)
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(vals).max()


def test_estimator_edge_cases(mlq):
    """A level with one sample contributes no variance (as the oracle's estimator); a level
    without samples, non-nested combination point sets and a multi-level MC call are refused."""
    from oracle import estimators as E
    rng = np.random.default_rng(8)
    ff = [rng.normal(size=5), rng.normal(size=1)]
    fc = [None, rng.normal(size=1)]
    r = mlq.estimate(mlq.MLQ_EST_MLMC, ff, fc)
    est, rmse, _, vars_ = E.standard_ml([list(a) for a in ff], [None, list(fc[1])])
    assert np.isclose(r["estimate"], est, rtol=1e-14) and np.isclose(r["rmse"], rmse, rtol=1e-13)
    assert vars_[1] == 0.0 and r["level_var"][1] == 0.0
    for args in ((mlq.MLQ_EST_MLMC, [np.zeros(0)], None), (mlq.MLQ_EST_MC, [np.ones(3), np.ones(3)], None)):
        with pytest.raises(mlq.MlqError):
            mlq.estimate(*args)
    with pytest.raises(mlq.MlqError):
        mlq.estimate(mlq.MLQ_EST_COMBINATION, [np.ones(4), np.ones(2)], None, n_per_level=[4, 2])


def test_header_is_plain_c_and_the_library_links_from_c(mlq, tmp_path):
    """include/mlq.h compiles as C99 and a C program linked against libmlq.so calls the host-only
    entry points: the CBC construction (against the oracle) and an argument check."""
    import shutil
    import subprocess
    from oracle import qmc
    if shutil.which("gcc") is None:
        pytest.skip("no C compiler")
    src = tmp_path / "use_mlq.c"
    src.write_text(r'''
#include <stdio.h>
#include "mlq.h"
int main(void) {
  double gamma[3] = {1.0, 0.5, 0.25};
  int64_t z[3];
  if (mlq_cbc(31, 3, gamma, z) != MLQ_OK) return 1;
  printf("%lld %lld %lld\n", (long long)z[0], (long long)z[1], (long long)z[2]);
  double y[4];
  printf("%d\n", (int)mlq_halton(0, 1, 2, NULL, MLQ_MAP_UNIFORM, y, NULL));
  return 0;
}
''')
    libdir = os.path.join(ROOT, "paper_2105_02007_amd")
    exe = tmp_path / "use_mlq"
    subprocess.run(["gcc", "-std=c99", "-Wall", "-Werror", "-pedantic", "-I", os.path.join(ROOT, "include"),
                    str(src), "-L", libdir, "-lmlq", "-Wl,-rpath," + libdir, "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    assert [int(v) for v in out[0].split()] == list(qmc.cbc(31, 3, [1.0, 0.5, 0.25]))
    assert int(out[1]) == mlq.MLQ_EINVAL


@pytest.mark.parametrize("uniform", [False, True])
def test_kl_weights_reproduce_the_covariance(mlq, uniform):
    """The library's mode weights (sqrt(lambda) for normal, sqrt(3 lambda) for uniform coordinates on
    [-1, 1], Section 5.1) with the oracle's full-rank eigenpairs: the exact covariance of the field,
    sum_k w_k^2 psi_k psi_k^T E[y^2] (E[y^2] from a Gauss rule exact for quadratics), is the kernel."""
    from oracle import fem, kl
    from oracle.mesh import BoxMesh
    mesh = BoxMesh([4, 3, 3])
    n = mesh.n_nodes
    lam, psi = kl.kl_modes(mesh, fem.assemble_mass(mesh), 0.3, 0.2, n, max_rank=n, eps=0.0)
    w = mlq.kl_weights(lam, uniform=uniform)
    y, q = np.polynomial.legendre.leggauss(2) if uniform else np.polynomial.hermite_e.hermegauss(2)
    ey2 = float((q * y * y).sum() / q.sum())
    cov = (psi * w ** 2) @ psi.T * ey2
    d = np.sqrt(((mesh.nodes[:, None, :] - mesh.nodes[None, :, :]) ** 2).sum(-1))
    assert np.abs(cov - 0.09 * np.exp(-d / 0.2)).max() <= 1e-10 * 0.09
    with pytest.raises(mlq.MlqError):
        mlq.kl_weights(np.array([1.0, -1.0]))


def test_lattice_weights_and_fibre_field(mlq):
    lam = np.array([2.0, 1.0, 0.5, 0.0])
    g = mlq.lattice_weights(lam, components=3)
    assert np.array_equal(g, np.tile(lam / 2.0, 3))
    rng = np.random.default_rng(3)
    n = 50
    a = rng.normal(size=(n, 3))
    ec = a / np.linalg.norm(a, axis=1)[:, None]
    b = rng.normal(size=(n, 3))
    b -= (b * ec).sum(1)[:, None] * ec
    el = b / np.linalg.norm(b, axis=1)[:, None]
    th = rng.uniform(-np.pi, np.pi, n)
    v = mlq.fibre_field(th, ec, el, 3.325e-3)
    # |V| = sigma_l and V makes the angle theta with e_circ in the (e_circ, e_long) plane
    assert np.allclose(np.linalg.norm(v, axis=1), 3.325e-3, rtol=1e-14)
    assert np.allclose(np.arctan2((v * el).sum(1), (v * ec).sum(1)), th, atol=1e-13)
