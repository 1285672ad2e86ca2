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


def test_mlqmc_common_points_telescope_and_rmse():
    """eq. (StandardML) with shifted QMC rules over three levels, every level evaluated at the
    same points per shift: the telescoping sum is the shift average of the finest level's
    means.  When the coarser levels do not vary between shifts (constant F_0, F_1), only the
    last level difference does, and the RMSE estimate is the standard error of the finest
    level's shift means."""
    rng = np.random.default_rng(5)
    S, N = 5, 6
    F0 = np.full((S, N), 0.25)
    F1 = np.full((S, N), 0.125)
    F2 = 0.3 + rng.normal(size=(S, N))
    F = [F0, F1, F2]
    fine = [[list(F[l][s]) for s in range(S)] for l in range(3)]
    coarse = [[None] * S] + [[list(F[l - 1][s]) for s in range(S)] for l in range(1, 3)]
    est, rmse, means = E.standard_mlqmc(fine, coarse)
    q = F2.mean(axis=1)  # shift means of the finest level
    assert math.isclose(est, q.mean(), rel_tol=1e-13)
    assert math.isclose(rmse, np.std(q, ddof=1) / np.sqrt(S), rel_tol=1e-12)
    assert math.isclose(means[0], 0.25) and math.isclose(means[1], -0.125)
    assert math.isclose(means[2], q.mean() - 0.125, rel_tol=1e-13)


def test_mlqmc_estimate_unbiased_and_rmse_consistent():
    """Independent synthetic level data (level l: fine values mu_l + a_l z, coarse values
    nu_l + b_l z', z, z' standard normal, S shifts of N_l points): over many repetitions the
    estimate averages sum_l (mu_l - nu_l), its variance is sum_l (a_l^2 + b_l^2) / (S N_l), and
    the squared RMSE estimate averages to that same variance (the shift-variance estimator is
    unbiased).  A dropped level, a coarse value added instead of subtracted, or a wrong
    normalisation of the shift variance fails one of the three checks."""
    rng = np.random.default_rng(6)
    S, Nl = 4, [8, 4, 2]
    mu, nu = [0.5, 0.2, -0.1], [0.0, 0.15, -0.12]
    a, b = [1.0, 0.6, 0.5], [0.0, 0.5, 0.4]
    R = 4000
    ests, ms = np.empty(R), np.empty(R)
    for r in range(R):
        fine, coarse = [], []
        for l, N in enumerate(Nl):
            fine.append([list(mu[l] + a[l] * rng.normal(size=N)) for _ in range(S)])
            coarse.append([list(nu[l] + b[l] * rng.normal(size=N)) for _ in range(S)] if l else [None] * S)
        est, rmse, _ = E.standard_mlqmc(fine, coarse)
        ests[r], ms[r] = est, rmse * rmse
    var = sum((a[l] ** 2 + (b[l] ** 2 if l else 0.0)) / (S * Nl[l]) for l in range(3))
    mean_ref = mu[0] + sum(mu[l] - nu[l] for l in (1, 2))
    assert abs(ests.mean() - mean_ref) < 4.0 * math.sqrt(var / R)
    # the sample variance of R normal estimates has relative standard deviation sqrt(2 / (R - 1))
    assert abs(ests.var(ddof=1) / var - 1.0) < 4.0 * math.sqrt(2.0 / (R - 1))
    # each level's squared RMSE term is var_l chi^2_(S-1) / (S - 1): relative sd sqrt(2 / (S - 1))
    assert abs(ms.mean() / var - 1.0) < 4.0 * math.sqrt(2.0 / (S - 1)) / math.sqrt(R)
