"""Pins of the oracle's randomly shifted rank-1 lattice rules and normal map.

* an unshifted lattice is a group under addition mod 1;
* a lattice rule integrates exp(2 pi i h.x) exactly: the mean is 1 (times the
  shift phase) when h.z = 0 mod N and 0 otherwise;
* the shift-averaged worst-case error of the 1D N-point grid is gamma/(6 N^2);
* each CBC component is the argmin of the error formula evaluated directly;
* Phi^-1 maps the lattice to N(0,1) coordinates with the clamp at 2^-53.
"""
import numpy as np

from oracle import qmc


def test_lattice_group_and_exact_trig_integration():
    N, z = 16, np.array([1, 5, 7])
    X = qmc.lattice_points(z, N, np.zeros(3))
    keys = {tuple(np.round(x * N).astype(int) % N) for x in X}
    for a in X:
        for b in X:
            assert tuple(np.round(((a + b) % 1.0) * N).astype(int) % N) in keys
    shift = np.array([0.13, 0.71, 0.42])
    Xs = qmc.lattice_points(z, N, shift)
    rng = np.random.default_rng(0)
    for _ in range(30):
        h = rng.integers(-20, 21, size=3)
        val = np.mean(np.exp(2j * np.pi * Xs @ h))
        if (h @ z) % N == 0:
            assert abs(val - np.exp(2j * np.pi * shift @ h)) < 1e-12
        else:
            assert abs(val) < 1e-12


def test_worst_case_error_closed_form_1d():
    for N in (1, 4, 16, 64):
        assert np.isclose(qmc.worst_case_error2([1], N, [0.7]), 0.7 / (6 * N * N), rtol=1e-12)


def test_cbc_components_are_greedy_minimisers():
    N, s = 32, 5
    gamma = 0.9 ** np.arange(s)
    z = qmc.cbc(N, s, gamma)
    assert z[0] == 1
    cands = [c for c in range(1, N) if np.gcd(c, N) == 1]
    for j in range(1, s):
        errs = [qmc.worst_case_error2(list(z[:j]) + [c], N, gamma) for c in cands]
        best = min(errs)
        assert qmc.worst_case_error2(z[:j + 1], N, gamma) <= best * (1 + 1e-12)
    # a good lattice beats a bad one (all components equal)
    assert qmc.worst_case_error2(z, N, gamma) < qmc.worst_case_error2(np.ones(s, int), N, gamma)


def test_normal_map():
    x = np.array([0.0, 0.5, 0.975, 1.0 - 2.0 ** -53, 1.0])
    y = qmc.to_normal(x)
    assert y[1] == 0.0 and abs(y[2] - 1.959963984540054) < 1e-13
    assert np.isfinite(y).all() and y[0] < -8 and y[-1] > 8
    Y = qmc.lattice_normals(np.array([1, 3]), 8, np.array([0.25, 0.5]))
    assert Y.shape == (2, 8)
