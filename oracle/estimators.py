"""Single- and multilevel quadrature estimators (test infrastructure; see ``oracle/__init__``).

* eq. (SL):          QoI_L = Q_L(F_L).
* eq. (StandardML):  QoI_L = sum_{l=0}^{L} Q_{L-l}(F_l - F_{l-1}),  F_{-1} = 0.
* eq. (PimpedML):    QoI_L = sum_{l=0}^{L} (Q_l - Q_{l-1})(F_{L-l}),  Q_{-1} = 0.

Q is a Monte Carlo mean or the shift average of randomly shifted lattice rules.
RMSE estimates: Monte Carlo sum_l V_l / N_l (unbiased sample variances);
shifted lattices sum_l sum_s (Q_{l,s} - mean_s Q_{l,s})^2 / (S (S - 1)).
All sums are plain Python loops in sample order.
"""
from __future__ import annotations

import math


def mean(xs):
    s = 0.0
    for x in xs:
        s += float(x)
    return s / len(xs)


def var(xs):
    if len(xs) < 2:
        return 0.0
    m = mean(xs)
    s = 0.0
    for x in xs:
        s += (float(x) - m) ** 2
    return s / (len(xs) - 1)


def single_level(f):
    """eq. (SL) with Monte Carlo: estimate and RMSE estimate."""
    return mean(f), math.sqrt(var(f) / len(f))


def standard_ml(f_fine, f_coarse):
    """eq. (StandardML) with independent Monte Carlo sample sets per level.

    f_fine[l][i] = F_l(omega_{l,i}), f_coarse[l][i] = F_{l-1}(omega_{l,i}) (ignored for l = 0).
    Returns (estimate, rmse, level means, level variances).
    """
    est, mse, means, vars_ = 0.0, 0.0, [], []
    for l in range(len(f_fine)):
        y = [f_fine[l][i] - (f_coarse[l][i] if l > 0 else 0.0) for i in range(len(f_fine[l]))]
        m, v = mean(y), var(y)
        means.append(m)
        vars_.append(v)
        est += m
        mse += v / len(y)
    return est, math.sqrt(mse), means, vars_


def shifted_lattice(per_shift_values):
    """Shift-averaged lattice rule: values[s][i] for shift s, point i.  Returns (estimate, rmse)."""
    q = [mean(v) for v in per_shift_values]
    S = len(q)
    m = mean(q)
    mse = 0.0 if S < 2 else sum((x - m) ** 2 for x in q) / (S * (S - 1))
    return m, math.sqrt(mse)


def standard_mlqmc(f_fine, f_coarse):
    """eq. (StandardML) with randomly shifted QMC rules (lattice or Halton): f_fine[l][s][i],
    f_coarse[l][s][i]."""
    est, mse, means = 0.0, 0.0, []
    for l in range(len(f_fine)):
        q = []
        for s in range(len(f_fine[l])):
            y = [f_fine[l][s][i] - (f_coarse[l][s][i] if l > 0 else 0.0) for i in range(len(f_fine[l][s]))]
            q.append(mean(y))
        S = len(q)
        m = mean(q)
        means.append(m)
        est += m
        if S > 1:
            mse += sum((x - m) ** 2 for x in q) / (S * (S - 1))
    return est, math.sqrt(mse), means


def combination(f_on_mesh, n_points):
    """eq. (PimpedML) with nested point sets.

    n_points[l] = number of points of Q_l (increasing, nested prefixes of one sequence);
    f_on_mesh[j] = values of F_j at the first n_points[L - j] points.
    """
    L = len(n_points) - 1
    est = 0.0
    for l in range(L + 1):
        F = f_on_mesh[L - l]
        q_l = mean(F[:n_points[l]])
        q_lm1 = mean(F[:n_points[l - 1]]) if l > 0 else 0.0
        est += q_l - q_lm1
    return est
