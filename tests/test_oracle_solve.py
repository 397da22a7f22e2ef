"""Pins for the oracle's GMRES and end-to-end solve.

* against an explicit dense LU solve of (I + omega^2 K M) u = g (the closed
  definition of the discrete problem), at tolerance 1e-12;
* m = 0 gives g = 0, hence u = 0 after zero iterations;
* GMRES on a plain dense system with the identity preconditioner matches
  numpy.linalg.solve, and its residual estimates never increase within a cycle.
"""
import math

import numpy as np
import pytest

import workloads
from oracle import OracleSolver, dense_A, fgmres
from oracle.gmres import givens


@pytest.mark.parametrize("n,ppw", [(7, 1.0), (15, 2.0), (31, 2.0)])
def test_solve_matches_dense_lu(n, ppw):
    wl = workloads.workload("C0").scaled(n, ppw_omega=ppw)
    m = wl.medium_array()
    b = 6 if n > 7 else 4
    s = OracleSolver(2, n, wl.omega, m, b, 4)
    g = s.op.rhs_incident(wl.incident()[0])
    res = s.solve_rhs(g, tol=1e-12)
    ref = np.linalg.solve(dense_A(s.op.table, n, 2, wl.omega, m), g.reshape(-1)).reshape(g.shape)
    assert res.converged
    assert np.linalg.norm(res.x - ref) <= 1e-9 * np.linalg.norm(ref)
    assert res.rel_residual <= 1e-12


def test_zero_medium_zero_solution():
    n = 15
    wl = workloads.workload("C0").scaled(n, ppw_omega=2.0)
    s = OracleSolver(2, n, wl.omega, np.zeros((n, n)), 6, 4)
    g = s.op.rhs_incident(wl.incident()[0])
    assert np.abs(g).max() == 0
    res = s.solve_rhs(g, 1e-6)
    assert res.iterations == 0 and res.converged and np.abs(res.x).max() == 0


def test_gmres_plain_dense():
    rng = np.random.default_rng(4)
    N = 60
    A = np.eye(N) * 4 + rng.standard_normal((N, N)) * 0.2 + 1j * rng.standard_normal((N, N)) * 0.2
    g = rng.standard_normal(N) + 1j * rng.standard_normal(N)
    res = fgmres(lambda x: A @ x, lambda x: x, g, 1e-12, restart=10, max_iters=500)
    ref = np.linalg.solve(A, g)
    assert res.converged
    assert np.linalg.norm(res.x - ref) <= 1e-10 * np.linalg.norm(ref)
    # within each cycle the estimate is non-increasing
    est = np.array(res.estimates)
    for c in range(0, len(est), 10):
        cyc = est[c:c + 10]
        assert np.all(np.diff(cyc) <= 1e-15)


def test_gmres_nonconvergence_is_reported():
    rng = np.random.default_rng(6)
    N = 40
    A = rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N))
    g = rng.standard_normal(N) + 0j
    res = fgmres(lambda x: A @ x, lambda x: x, g, 1e-300, restart=5, max_iters=3)
    assert not res.converged and res.iterations == 3


def test_givens_convention():
    for f, g in [(1 + 2j, 3 - 1j), (0.0, 2j), (1.5, 0.0), (-2 + 0j, 1e-3j)]:
        c, s, r = givens(f, g)
        G = np.array([[c, s], [-np.conj(s), c]])
        out = G @ np.array([f, g])
        assert abs(out[1]) < 1e-15 * (abs(f) + abs(g))
        assert abs(out[0] - r) < 1e-15 * (abs(f) + abs(g))
        assert abs(abs(c) ** 2 + abs(s) ** 2 - 1) < 1e-15


def test_preconditioned_solve_c0():
    # the full C0 case: a handful of iterations (qualitatively as in the
    # paper's tables), true residual below the tolerance
    wl = workloads.workload("C0")
    s = OracleSolver(2, wl.n, wl.omega, wl.medium_array(), 12, 4)
    res = s.solve_rhs(s.op.rhs_incident(wl.incident()[0]), 1e-6)
    assert res.converged and res.rel_residual <= 1e-6
    assert 2 <= res.iterations <= 12
