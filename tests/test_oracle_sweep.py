"""Pins for the oracle's sparse system and sweep (eq. Huf, eq. Hwv_approx,
Algorithms 1 and 2).

* With one slice the sweep is the exact solve of H (T~_1 = T_1, Sec. 2.3).
* With the exact Schur-complement inverses T_k (restrictions of
  H_[1:k,1:k]^{-1}, Sec. 2.3) the forward/backward sweep is block Gaussian
  elimination, hence equals H^{-1} f for any slicing.
* H itself discretises eq. LS_d: its solution restricted to I is close to the
  dense solution (accuracy parity unpinned; the paper prints no number).
"""
import math

import numpy as np
import pytest
import scipy.sparse.linalg as spla

import workloads
from oracle import (OracleSolver, SparseSystem, Sweep, alpha_beta, green_table, DenseOperator,
                    dense_A)


def small_case(n=23, ppw=2.0, b=6, d=2):
    wl = workloads.workload("C0").scaled(n, ppw_omega=ppw)
    if d == 3:
        m = workloads.single_gaussian_medium(n, 3)
    else:
        m = wl.medium_array()
    omega = wl.omega
    t = green_table(d, n, omega)
    alpha, beta, _ = alpha_beta(t, n, d)
    system = SparseSystem(d, n, omega, m, alpha, beta, b, 10.0)
    return system, m, omega


@pytest.mark.parametrize("d", [2, 3])
def test_single_slice_sweep_is_exact_solve(d):
    n = 23 if d == 2 else 7
    system, m, omega = small_case(n=n, d=d, b=4 if d == 3 else 6)
    sw = Sweep(system, n + 2, m)
    assert sw.nslices == 1
    rng = np.random.default_rng(1)
    r = rng.standard_normal((n,) * d) + 1j * rng.standard_normal((n,) * d)
    f = system.apply_Q(r)
    ref = system.restrict(spla.spsolve(system.H.tocsc(), f))
    got = sw.apply(r)
    assert np.linalg.norm(got - ref) <= 1e-12 * np.linalg.norm(ref)


@pytest.mark.parametrize("w", [3, 4, 7])
def test_exact_T_sweep_is_block_elimination(w):
    n = 23
    system, m, omega = small_case(n=n)
    sw = Sweep(system, w, m, exact=True)
    assert sw.nslices == (n + 2) // w
    rng = np.random.default_rng(2)
    f = rng.standard_normal(system.npts) + 1j * rng.standard_normal(system.npts)
    ref = spla.spsolve(system.H.tocsc(), f)
    got = sw.sweep(f)
    assert np.linalg.norm(got - ref) <= 1e-11 * np.linalg.norm(ref)


def test_slices_partition_the_extended_grid():
    n, b = 23, 6
    system, m, omega = small_case(n=n, b=b)
    sw = Sweep(system, 4, m)
    lines = np.concatenate([np.arange(lo, hi + 1) for lo, hi in sw.bounds])
    np.testing.assert_array_equal(lines, np.arange(-b, n + 2 + b))
    assert sw.bounds[0] == (-b, 3)
    assert sw.bounds[-1][1] == n + 1 + b
    # the last slice absorbs the remainder (reading G8)
    assert sw.bounds[-1][0] == (sw.nslices - 1) * 4
    assert sw.aux_count[0] == 0 and all(c == b * system.L for c in sw.aux_count[1:])


def test_first_subproblem_is_leading_block():
    n = 23
    system, m, omega = small_case(n=n)
    sw = Sweep(system, 4, m)
    pts = sw.points(0)
    v = np.random.default_rng(5).standard_normal(len(pts)) + 0j
    ref = spla.spsolve(system.H[pts][:, pts].tocsc(), v)
    assert np.linalg.norm(sw.solve_slice(0, v) - ref) <= 1e-12 * np.linalg.norm(ref)


def test_type1_rows_match_local_equation():
    # row i in I^h: alpha^* u_mu + omega^2 beta^* (m u)_mu (eq. local_c_approx)
    n = 23
    system, m, omega = small_case(n=n)
    b, L = system.b, system.L
    u = np.random.default_rng(7).standard_normal(system.npts) + 1j
    Hu = system.H @ u
    for (i1, i2) in [(0, 0), (5, 9), (n + 1, 3), (1, n)]:
        p = (i1 + b) * L + (i2 + b)
        acc = 0
        for o, (d1, d2) in enumerate(system.mu):
            q = (i1 + d1 + b) * L + (i2 + d2 + b)
            acc += np.conj(system.alpha[o]) * u[q] + omega ** 2 * np.conj(system.beta[o]) * system.m_ext[q] * u[q]
        assert abs(Hu[p] - acc) < 1e-12 * abs(acc)


def test_sparse_system_discretises_ls_equation():
    # parity unpinned: the paper gives no accuracy number for H; this checks
    # only that its solution is a close approximation of the dense one
    wl = workloads.workload("C0")
    n = wl.n
    s = OracleSolver(2, n, wl.omega, wl.medium_array(), 12, 4)
    g = s.op.rhs_incident(wl.incident()[0])
    ud = np.linalg.solve(dense_A(s.op.table, n, 2, wl.omega, s.m), g.reshape(-1)).reshape(g.shape)
    ut = s.system.restrict(spla.spsolve(s.system.H.tocsc(), s.system.apply_Q(g)))
    assert np.linalg.norm(ut - ud) < 1e-2 * np.linalg.norm(ud)


def test_exact_T_sweep_is_block_elimination_3d():
    # three slabs of the extended cube (Sec. 3.1): with the exact Schur
    # complements the slab-by-slab sweep is block Gaussian elimination
    n = 7
    system, m, omega = small_case(n=n, d=3, b=3)
    sw = Sweep(system, 3, m, exact=True)
    assert sw.nslices == 3
    rng = np.random.default_rng(21)
    f = rng.standard_normal(system.npts) + 1j * rng.standard_normal(system.npts)
    ref = spla.spsolve(system.H.tocsc(), f)
    got = sw.sweep(f)
    assert np.linalg.norm(got - ref) <= 1e-11 * np.linalg.norm(ref)
