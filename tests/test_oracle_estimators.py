"""Pins of the oracle's estimators, eqs. (SL), (StandardML), (PimpedML).

* a single-level MLMC is plain MC;
* with common samples on all levels the telescoping sum equals the mean of F_L;
* eq. (StandardML) and eq. (PimpedML) are the same linear functional
  (regrouping the double sum), checked with nested point sets;
* shifted-lattice RMSE is the standard error of the shift means.
"""
import math

import numpy as np

from oracle import estimators as E


def test_single_level_mlmc_is_mc():
    f = list(np.random.default_rng(0).normal(size=37))
    est, rmse, means, vars_ = E.standard_ml([f], [None])
    m, r = E.single_level(f)
    assert est == m and rmse == r and vars_[0] == E.var(f)
    assert math.isclose(E.var(f), np.var(f, ddof=1), rel_tol=1e-13)


def test_telescoping_with_common_samples():
    rng = np.random.default_rng(1)
    F = [rng.normal(size=20) + l for l in range(4)]
    fine = [F[l] for l in range(4)]
    coarse = [None] + [F[l - 1] for l in range(1, 4)]
    est, *_ = E.standard_ml(fine, coarse)
    assert math.isclose(est, E.mean(F[3]), rel_tol=1e-13)


def test_standard_ml_equals_combination_form():
    """sum_l Q_{L-l}(F_l - F_{l-1}) = sum_l (Q_l - Q_{l-1}) F_{L-l} with nested rules Q_l."""
    rng = np.random.default_rng(2)
    L = 3
    n_points = [4, 8, 16, 32]  # Q_l uses the first n_points[l] points of one sequence
    F = [rng.normal(size=32) * 0.1 + np.sin(l) for l in range(L + 1)]  # F_j at all points
    std = 0.0
    for l in range(L + 1):
        N = n_points[L - l]
        y = F[l][:N] - (F[l - 1][:N] if l > 0 else 0.0)
        std += E.mean(y)
    comb = E.combination([F[j][:n_points[L - j]] for j in range(L + 1)], n_points)
    assert math.isclose(std, comb, rel_tol=1e-13, abs_tol=1e-15)


def test_shifted_lattice_rmse():
    vals = [[1.0, 2.0], [2.0, 4.0], [0.0, 1.0]]
    m, r = E.shifted_lattice(vals)
    q = np.array([1.5, 3.0, 0.5])
    assert math.isclose(m, q.mean(), rel_tol=1e-15)
    assert math.isclose(r, np.std(q, ddof=1) / np.sqrt(3), rel_tol=1e-13)
    est, rmse, means = E.standard_mlqmc([vals], [[None, None, None]])
    assert math.isclose(est, m) and math.isclose(rmse, r)
