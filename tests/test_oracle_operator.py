"""Pins for the oracle's dense operator (eq. LS_d, eq. LS_d_c).

The FFT product is checked against the O(N^2) sum that defines it; the
symmetry of K and the m = 0 identity are closed-form facts.
"""
import math

import numpy as np
import pytest

import workloads
from oracle import DenseOperator, brute_force_K, green_table


@pytest.mark.parametrize("d,n,ppw", [(2, 7, 1.0), (2, 15, 2.0), (2, 31, 2.0), (3, 7, 1.0)])
def test_fft_product_equals_direct_sum(d, n, ppw):
    rng = np.random.default_rng(11)
    omega = 2 * math.pi * ppw
    m = rng.uniform(-0.3, 0.3, (n,) * d)
    op = DenseOperator(d, n, omega, m)
    x = rng.standard_normal((n,) * d) + 1j * rng.standard_normal((n,) * d)
    ref = brute_force_K(op.table, n, d, x)
    got = op.apply_K(x)
    assert np.linalg.norm(got - ref) <= 1e-13 * np.linalg.norm(ref)
    # A = I + omega^2 K M
    refA = x + omega ** 2 * brute_force_K(op.table, n, d, m * x)
    assert np.linalg.norm(op.apply_A(x) - refA) <= 1e-13 * np.linalg.norm(refA)


def test_K_is_complex_symmetric():
    n, d = 15, 2
    rng = np.random.default_rng(3)
    op = DenseOperator(d, n, 2 * math.pi * 2, np.zeros((n, n)))
    x = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    y = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    lhs = np.sum(x * op.apply_K(y))
    rhs = np.sum(y * op.apply_K(x))
    assert abs(lhs - rhs) <= 1e-13 * abs(lhs)


def test_zero_medium_gives_identity_and_zero_rhs():
    n, d = 15, 2
    op = DenseOperator(d, n, 2 * math.pi * 2, np.zeros((n, n)))
    x = np.random.default_rng(0).standard_normal((n, n)) + 0j
    np.testing.assert_allclose(op.apply_A(x), x, atol=0, rtol=0)
    uinc = workloads.plane_waves(n, 2, op.omega, np.array([[1.0, 0.0]]))[0]
    assert np.abs(op.rhs_incident(uinc)).max() == 0.0


def test_incident_rhs_is_minus_omega2_K_m_uI():
    n, d = 15, 2
    wl = workloads.workload("C0").scaled(n)
    m = wl.medium_array()
    op = DenseOperator(d, n, wl.omega, m)
    uinc = wl.incident()[0]
    ref = -wl.omega ** 2 * brute_force_K(op.table, n, d, m * uinc)
    got = op.rhs_incident(uinc)
    assert np.linalg.norm(got - ref) <= 1e-13 * np.linalg.norm(ref)


def test_sampled_direct_sum_equals_full_direct_sum():
    """brute_force_K_at (one output at a time, for large grids) agrees with the
    full O(N^2) definition at random points, in 2D and 3D."""
    from oracle import green_table, brute_force_K, brute_force_K_at
    for n, d in [(9, 2), (5, 3)]:
        t = green_table(d, n, 7.0)
        rng = np.random.default_rng(0)
        x = rng.standard_normal((n,) * d) + 1j * rng.standard_normal((n,) * d)
        full = brute_force_K(t, n, d, x)
        pts = rng.integers(0, n, size=(8, d))
        s = brute_force_K_at(t, n, d, x, pts)
        assert np.abs(s - full[tuple(pts.T)]).max() <= 1e-14 * np.abs(full).max()
