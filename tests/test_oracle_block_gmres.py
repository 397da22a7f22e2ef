"""Pins for the oracle's block flexible GMRES (a shared block Krylov space for
a batch of right-hand sides; reading G20).

* With one right-hand side the block method is GMRES: stopped after the same
  number of steps, its iterate equals fgmres's.
* On a small dense system it reaches the direct solution, every column's true
  residual below the tolerance, and its residual estimates never increase
  (each step minimises over a larger space). A zero column stays out of the
  block (x = 0 after no step); columns that converge leave it at a restart.
* Finite termination: with B columns on a system of order N = B s, s block
  steps span the whole space, and the residual is zero up to rounding.
* On the Lippmann-Schwinger problem with the sweeping preconditioner it needs
  no more block steps than the slowest column needs GMRES steps alone (the
  block space contains every column's own Krylov space), here fewer.
"""
import numpy as np
import pytest

import workloads
from oracle import OracleSolver, block_fgmres, fgmres


def dense_case(n=40, seed=0):
    rng = np.random.default_rng(seed)
    A = np.eye(n) * 4 + (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) / np.sqrt(n)
    Pm = np.linalg.inv(A + 0.3 * (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) / np.sqrt(n))
    return A, (lambda x: A @ x), (lambda x: Pm @ x), rng


@pytest.mark.parametrize("k", [1, 3, 6])
def test_single_column_is_gmres(k):
    A, fA, fP, rng = dense_case()
    g = rng.standard_normal(40) + 1j * rng.standard_normal(40)
    one = fgmres(fA, fP, g, 1e-300, restart=30, max_iters=k)
    blk = block_fgmres(fA, fP, g[None], 1e-300, restart=30, max_iters=k)
    assert one.iterations == blk.iterations == k
    assert np.linalg.norm(blk.x[0] - one.x) <= 1e-12 * np.linalg.norm(one.x)


def test_dense_system_block_solution():
    A, fA, fP, rng = dense_case(seed=1)
    G = rng.standard_normal((5, 40)) + 1j * rng.standard_normal((5, 40))
    G[2] = 0.0
    res = block_fgmres(fA, fP, G, 1e-12, restart=2)
    assert res.converged and res.rel_residuals.max() <= 1e-12
    X = np.linalg.solve(A, G.T).T
    assert np.linalg.norm(res.x - X) <= 1e-10 * np.linalg.norm(X)
    assert not np.any(res.x[2]) and res.col_iterations[2] == 0
    est = res.estimates
    assert est[1] <= est[0] * (1 + 1e-12)                                # within the first cycle
    # several cycles, and some column left the block before the last one
    assert res.iterations > 2 and res.col_iterations.max() == res.iterations
    assert res.col_iterations[[0, 1, 3, 4]].min() < res.iterations


def test_finite_termination():
    n, B = 40, 5
    rng = np.random.default_rng(7)
    A = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    G = rng.standard_normal((B, n)) + 1j * rng.standard_normal((B, n))
    ident = lambda x: x
    res = block_fgmres(lambda x: A @ x, ident, G, 1e-300, restart=n // B, max_iters=n // B)
    assert res.iterations == n // B
    assert res.rel_residuals.max() <= 1e-9
    early = block_fgmres(lambda x: A @ x, ident, G, 1e-300, restart=n // B, max_iters=n // B - 1)
    assert early.rel_residuals.min() > 1e-6


def test_block_steps_on_the_lippmann_schwinger_problem():
    wl = workloads.workload("C0").scaled(47, ppw_omega=3.0)
    m = wl.medium_array()
    s = OracleSolver(2, wl.n, wl.omega, m, 8, 4, fronts=2)
    uinc = workloads.plane_waves(wl.n, 2, wl.omega, workloads.angle_directions(8, 2))
    G = np.stack([s.op.rhs_incident(uinc[j]) for j in range(8)])
    single = [s.solve_rhs(G[j], 1e-6).iterations for j in range(8)]
    blk = s.solve_block(G, 1e-6)
    print(f"per column {single}, block {blk.iterations}")
    assert blk.converged and blk.rel_residuals.max() <= 1e-6
    assert blk.iterations <= max(single)
    tight = [s.solve_rhs(G[j], 1e-12).x for j in range(8)]
    for j in range(8):
        assert np.linalg.norm(blk.x[j] - tight[j]) <= 1e-4 * np.linalg.norm(tight[j])
