"""Quasi-Monte Carlo point sets (test infrastructure; see ``oracle/__init__``).

Halton points (the paper's QMC rule, Section 5.1 and its quadrature-methods
paragraph): coordinate k of point i is the radical inverse of i in the base of
the (k+1)-th prime, optionally shifted at random mod 1 (randomised QMC, which
gives an error estimate over independent shifts), mapped to the uniform
coordinates y = 2x - 1 of the parametrisation on [-1, 1]^M or to Gaussian ones.
The radical inverse is formed as an exact rational and rounded once.

Randomly shifted rank-1 lattice rules, the other QMC rule of the workloads:
x_i = frac(i z / N + Delta), i = 0..N-1, mapped to Gaussian coordinates
y = Phi^-1(x).

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

from fractions import Fraction
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


def lattice_uniforms(z, N, shift):
    """Uniform coordinates y = 2x - 1 on [-1, 1] (s, N) of a shifted lattice rule."""
    return np.ascontiguousarray((2.0 * lattice_points(z, N, shift) - 1.0).T)


def first_primes(n):
    """The first n primes, by trial division against the primes found so far."""
    ps = []
    c = 2
    while len(ps) < n:
        if all(c % q for q in ps if q * q <= c):
            ps.append(c)
        c += 1
    return ps


def radical_inverse(i, p):
    """phi_p(i) = sum_j d_j p^(-j-1) for i = sum_j d_j p^j, rounded once from the exact rational."""
    x, scale = Fraction(0), Fraction(1, p)
    while i > 0:
        i, d = divmod(i, p)
        x += d * scale
        scale /= p
    return float(x)


def halton_points(s, first, count, shift=None):
    """Points i = first .. first + count - 1 of the s-dimensional Halton sequence, (count, s) in
    [0, 1); with a shift, x = frac(phi + shift) (the sum rounded in FP64, then 1 subtracted
    once if it reached 1)."""
    ps = first_primes(s)
    X = np.array([[radical_inverse(first + i, p) for p in ps] for i in range(count)]).reshape(count, s)
    if shift is not None:
        X = X + np.asarray(shift, dtype=np.float64)[None, :]
        X = np.where(X >= 1.0, X - 1.0, X)
    return X


def halton_coordinates(s, first, count, shift=None, uniform=True):
    """KL coordinates (s, count): y = 2x - 1 in [-1, 1] (uniform) or y = Phi^-1(x) (Gaussian)."""
    X = halton_points(s, first, count, shift)
    Y = 2.0 * X - 1.0 if uniform else to_normal(X)
    return np.ascontiguousarray(Y.T)
