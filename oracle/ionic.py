"""Cubic ionic current, eq. (ionic_term) (test infrastructure; see ``oracle/__init__``).

I_ion(u) = alpha (u - u_rest)(u - u_th)(u - u_peak), applied node-wise; the
reaction term of eq. (mono_disc) multiplies the nodal values by dt * M.
"""
from __future__ import annotations

import numpy as np


def i_ion(u, p):
    return p["alpha"] * (u - p["u_rest"]) * (u - p["u_th"]) * (u - p["u_peak"])


def di_ion(u, p):
    """d I_ion / du by the product rule."""
    a, b, c = u - p["u_rest"], u - p["u_th"], u - p["u_peak"]
    return p["alpha"] * (b * c + a * c + a * b)
