"""Randomly shifted rank-1 lattice rules (test infrastructure; see ``oracle/__init__``).

The paper uses quasi-Monte Carlo quadrature (Section 5.1, Halton points); the
workloads use randomly shifted rank-1 lattice rules instead, whose shift
average gives an error estimate.  Points: x_i = frac(i z / N + Delta),
i = 0..N-1, mapped to Gaussian coordinates y = Phi^-1(x).

Generating vector: component-by-component (CBC) construction minimising the
shift-averaged worst-case error in the weighted unanchored Sobolev space of
first order with product weights gamma_j,
    e^2(z) = -1 + (1/N) sum_{k<N} prod_j (1 + gamma_j B2(frac(k z_j / N))),
    B2(x) = x^2 - x + 1/6.
Candidates are the integers in [1, N) coprime to N; ties (criteria within a
relative 1e-12 of the minimum, i.e. equal up to rounding) go to the smallest.
The sum over k runs in increasing k with one accumulator so that the decision
is reproducible bit for bit by any implementation doing the same operations.
"""
from __future__ import annotations

from math import gcd

import numpy as np
from scipy.special import ndtri


def b2(x):
    return x * x - x + 1.0 / 6.0


def cbc(N, s, gamma):
    N = int(N)
    gamma = np.asarray(gamma, dtype=np.float64)
    if N == 1:
        return np.ones(s, dtype=np.int64)
    cands = np.array([z for z in range(1, N) if gcd(z, N) == 1], dtype=np.int64)
    k = np.arange(N, dtype=np.int64)
    P = np.ones(N)
    z = np.zeros(s, dtype=np.int64)
    for j in range(s):
        acc = np.zeros(cands.shape[0])
        for kk in range(N):
            r = (kk * cands) % N
            acc = acc + P[kk] * (1.0 + gamma[j] * b2(r / N))
        err = -1.0 + acc / N
        # exact ties (equal up to rounding) go to the smallest candidate
        best = int(np.argmax(err <= err.min() + 1e-12 * abs(err.min())))
        z[j] = cands[best]
        P = P * (1.0 + gamma[j] * b2(((k * z[j]) % N) / N))
    return z


def worst_case_error2(z, N, gamma):
    """Shift-averaged squared worst-case error of the lattice with generating vector z."""
    k = np.arange(N, dtype=np.int64)
    prod = np.ones(N)
    for j, zj in enumerate(z):
        prod = prod * (1.0 + gamma[j] * b2(((k * int(zj)) % N) / N))
    return -1.0 + prod.mean()


def lattice_points(z, N, shift):
    """Shifted lattice points (N, s) in [0, 1)."""
    i = np.arange(N, dtype=np.int64)[:, None]
    x = ((i * np.asarray(z, dtype=np.int64)[None, :]) % N) / N + np.asarray(shift)[None, :]
    return np.where(x >= 1.0, x - 1.0, x)


def to_normal(x):
    """y = Phi^-1(x) with x clamped to [2^-53, 1 - 2^-53]."""
    eps = 2.0 ** -53
    return ndtri(np.clip(x, eps, 1.0 - eps))


def lattice_normals(z, N, shift):
    """Gaussian KL coordinates (s, N) of a shifted lattice rule."""
    return np.ascontiguousarray(to_normal(lattice_points(z, N, shift)).T)
