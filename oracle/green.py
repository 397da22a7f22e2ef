"""Green's function table (oracle; test infrastructure only).

Paper, Sec. 1: the free-space Green's function is G(x) = (i/4) H0^(1)(omega|x|)
in 2D and exp(i omega |x|) / (4 pi |x|) in 3D.
Paper, Sec. 2.1 (Nystrom discretisation, eq. LS_d): k_i = G(p_i) h^d for
i != 0, and k_0 is a quadrature correction at the singular point whose value
the paper does not print (reading G1 below).
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import hankel1


def green(d: int, omega: float, r: np.ndarray) -> np.ndarray:
    """G(r) for r > 0 (Sec. 1)."""
    r = np.asarray(r, dtype=np.float64)
    if d == 2:
        return 0.25j * hankel1(0, omega * r)
    if d == 3:
        return np.exp(1j * omega * r) / (4.0 * math.pi * r)
    raise ValueError("d must be 2 or 3")


def central_weight(d: int, omega: float, h: float) -> complex:
    """k_0, reading G1: the integral of G over the disk (2D) or ball (3D) of
    the same measure as one grid cell, h^d, in closed form.

    2D, a = h / sqrt(pi):       k0 = (i pi a / (2 omega)) H1^(1)(omega a) - 1/omega^2
    3D, a = h (3/(4 pi))^(1/3): k0 = (exp(i omega a)(1 - i omega a) - 1) / omega^2
    """
    if d == 2:
        a = h / math.sqrt(math.pi)
        return complex(1j * math.pi * a / (2.0 * omega) * hankel1(1, omega * a) - 1.0 / omega ** 2)
    if d == 3:
        a = h * (3.0 / (4.0 * math.pi)) ** (1.0 / 3.0)
        return complex((np.exp(1j * omega * a) * (1.0 - 1j * omega * a) - 1.0) / omega ** 2)
    raise ValueError("d must be 2 or 3")


def green_table(d: int, n: int, omega: float) -> np.ndarray:
    """k_delta for delta in [-(n+1), n+1]^d; array index delta + (n+1).

    k_delta = G(|delta| h) h^d for delta != 0, k_0 per G1 (Sec. 2.1)."""
    h = 1.0 / (n + 1)
    off = np.arange(-(n + 1), n + 2, dtype=np.float64)
    grids = np.meshgrid(*([off] * d), indexing="ij")
    r = np.sqrt(sum(g * g for g in grids)) * h
    centre = (n + 1,) * d
    r[centre] = 1.0  # placeholder, overwritten below
    k = green(d, omega, r) * h ** d
    k[centre] = central_weight(d, omega, h)
    return k


def wrapped_table(table: np.ndarray, n: int, d: int) -> np.ndarray:
    """The table laid out for a length P = 2(n+1) cyclic convolution: entry q
    holds k_delta with delta = q for q <= P/2 and delta = q - P otherwise.
    Every offset |delta| <= n-1 used by the product on the interior lands on
    its own slot, so the cyclic product equals the linear one there."""
    P = 2 * (n + 1)
    q = np.arange(P)
    delta = np.where(q <= P // 2, q, q - P)
    idx = delta + (n + 1)
    return table[np.ix_(*([idx] * d))]
