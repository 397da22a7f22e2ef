"""Pins for the oracle's Green's function table (Sec. 1 and Sec. 2.1).

The oracle evaluates H0^(1) through scipy (AMOS); the pins compare against
mpmath at 30 digits, an independent implementation, and check the central
weight's closed form (reading G1) against adaptive quadrature of G over the
cell-measure disk / ball.
"""
import math

import mpmath as mp
import numpy as np
import pytest

from oracle import green, central_weight, green_table, wrapped_table

mp.mp.dps = 30


@pytest.mark.parametrize("x", [0.05, 0.39, 1.0, 3.7, 12.5, 40.0, 402.1, 569.0])
def test_hankel_against_mpmath(x):
    omega = 1.0
    got = complex(green(2, omega, np.array([x]))[0])
    ref = complex(0.25j * mp.hankel1(0, x))
    env = 0.25 * math.sqrt(2.0 / (math.pi * x)) + abs(ref)
    assert abs(got - ref) <= 1e-14 * env


def test_green_solves_helmholtz_away_from_origin():
    # radial Helmholtz ODE G'' + (d-1)/r G' + omega^2 G = 0, evaluated with
    # mpmath derivatives of the 30-digit reference functions
    omega = 7.3
    for d, f in [(2, lambda r: 0.25j * mp.hankel1(0, omega * r)),
                 (3, lambda r: mp.exp(1j * omega * r) / (4 * mp.pi * r))]:
        for r in [0.1, 0.37, 1.4]:
            res = mp.diff(f, r, 2) + (d - 1) / r * mp.diff(f, r, 1) + omega ** 2 * f(r)
            assert abs(res) < 1e-12 * omega ** 2 * abs(f(r))
            assert abs(complex(green(d, omega, np.array([r]))[0]) - complex(f(r))) < 1e-14 * abs(f(r))


@pytest.mark.parametrize("d,n,ppw", [(2, 63, 4.0), (2, 1023, 64.0), (3, 127, 8.0), (3, 15, 2.0)])
def test_central_weight_is_disk_integral(d, n, ppw):
    omega = 2 * math.pi * ppw
    h = 1.0 / (n + 1)
    if d == 2:
        a = h / mp.sqrt(mp.pi)
        integral = 2 * mp.pi * mp.quad(lambda r: 0.25j * mp.hankel1(0, omega * r) * r, [0, a])
    else:
        a = h * (3 / (4 * mp.pi)) ** (mp.mpf(1) / 3)
        integral = 4 * mp.pi * mp.quad(lambda r: mp.exp(1j * omega * r) / (4 * mp.pi * r) * r * r, [0, a])
    k0 = central_weight(d, omega, h)
    assert abs(k0 - complex(integral)) <= 1e-12 * abs(complex(integral))


def test_central_weight_small_cell_limit():
    # the disk average of G differs from G at the disk's rim by a bounded
    # log term: k0 / h^2 must track G(a) - (i/4)(2/pi)(1/2) as h -> 0 (2D)
    omega = 2 * math.pi * 4
    for n in [255, 1023, 4095]:
        h = 1.0 / (n + 1)
        a = h / math.sqrt(math.pi)
        k0 = central_weight(2, omega, h)
        # small-argument forms: Y0 ~ (2/pi)(ln(x/2)+gamma), integral of r ln r
        approx = 0.25j * (1 + 2j / math.pi * (math.log(omega * a / 2) + np.euler_gamma - 0.5)) * math.pi * a * a
        assert abs(k0 - approx) < 5e-3 * abs(approx)


def test_table_symmetry_and_layout():
    n, d, omega = 15, 2, 2 * math.pi * 2
    t = green_table(d, n, omega)
    assert t.shape == (2 * n + 3, 2 * n + 3)
    np.testing.assert_array_equal(t, t[::-1, :])
    np.testing.assert_array_equal(t, t[:, ::-1])
    np.testing.assert_array_equal(t, t.T)
    h = 1.0 / (n + 1)
    # offset (3, 4): |delta| = 5 h
    assert t[n + 1 + 3, n + 1 + 4] == pytest.approx(complex(0.25j * mp.hankel1(0, omega * 5 * h)) * h * h, rel=1e-14)
    w = wrapped_table(t, n, d)
    P = 2 * (n + 1)
    assert w.shape == (P, P)
    assert w[0, 0] == t[n + 1, n + 1]
    assert w[P - 1, 2] == t[n + 1 - 1, n + 1 + 2]
