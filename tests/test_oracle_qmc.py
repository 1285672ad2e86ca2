"""Pins of the oracle's QMC rules: randomly shifted rank-1 lattices, Halton points, normal map.

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


def test_first_primes():
    """The prime-counting landmarks pi(541) = 100 and pi(7919) = 1000, and the first ten."""
    ps = qmc.first_primes(1000)
    assert ps[:10] == [2, 3, 5, 7, 11, 13, 17, 19, 23, 29]
    assert ps[99] == 541 and ps[999] == 7919
    assert all(b > a for a, b in zip(ps, ps[1:]))


def test_van_der_corput_values():
    """The base-2 and base-3 radical inverses of the first integers (digit reversal)."""
    assert [qmc.radical_inverse(i, 2) for i in range(8)] == [0, 0.5, 0.25, 0.75, 0.125, 0.625, 0.375, 0.875]
    third = [qmc.radical_inverse(i, 3) for i in range(10)]
    assert third == [0, 1 / 3, 2 / 3, 1 / 9, 4 / 9, 7 / 9, 2 / 9, 5 / 9, 8 / 9, 1 / 27]
    # a digit string and its reversal: 1234 in base 10 <-> 0.4321
    assert qmc.radical_inverse(1234, 10) == 0.4321


def test_halton_stratification():
    """The first p^m points of the base-p radical inverse are exactly the grid {j / p^m}; the
    first 2^a 3^b points of the 2D Halton set (bases 2 and 3) put one point in each cell of the
    2^a x 3^b grid (a = b = 3: 216 points, 8 x 27 cells)."""
    for p, m in [(2, 6), (3, 4), (7, 2)]:
        x = sorted(qmc.radical_inverse(i, p) for i in range(p ** m))
        assert x == [j / p ** m for j in range(p ** m)]
    X = qmc.halton_points(2, 0, 216, None)
    cells = {(int(x * 8), int(y * 27)) for x, y in X}
    assert len(cells) == 216


def test_halton_shift_and_maps():
    """A shift moves every point mod 1; the uniform map lands in [-1, 1); the Gaussian map is
    Phi^-1 of the same points; points do not depend on how many are drawn."""
    rng = np.random.default_rng(3)
    sh = rng.random(5)
    X = qmc.halton_points(5, 1, 40, None)
    Xs = qmc.halton_points(5, 1, 40, sh)
    d = (Xs - X - sh[None, :]) % 1.0
    assert np.all(np.minimum(d, 1.0 - d) < 1e-15)
    assert np.all((Xs >= 0) & (Xs < 1))
    Yu = qmc.halton_coordinates(5, 1, 40, sh, uniform=True)
    assert np.all((Yu >= -1) & (Yu < 1)) and np.array_equal(Yu, (2.0 * Xs - 1.0).T)
    Yn = qmc.halton_coordinates(5, 1, 40, sh, uniform=False)
    assert np.allclose(Yn, qmc.to_normal(Xs).T)
    assert np.array_equal(qmc.halton_points(5, 11, 7, sh), Xs[10:17])


def test_lattice_uniform_map():
    """The uniform map of a shifted lattice: 2x - 1 of the same points, in [-1, 1)."""
    z, N = np.array([1, 5, 7]), 16
    sh = np.array([0.1, 0.5, 0.9])
    U = qmc.lattice_uniforms(z, N, sh)
    assert np.array_equal(U, (2.0 * qmc.lattice_points(z, N, sh) - 1.0).T)
    assert U.shape == (3, N) and np.all((U >= -1) & (U < 1))
