"""The largest 2D grid a handle accepts, and the first one it refuses.

In 2D n <= 2047: the zero-padded FFT length P = 2^k >= 2(n+1) is then at
most 4096, and one complex128 sequence of that length plus its twiddles
fills a compute unit's LDS. n = 2048 (P = 8192) must be refused at setup
with LS_E_INVALID rather than fail inside a launch.

At n = 2047 (32 Gaussian bumps with C1's distributions, omega = 2 pi 32,
b = 12, w = 4, mixed precision, one plane wave) the checks are properties
that hold at any size:
* the operator A x (float64) at sampled points, by the oracle's direct sum
  of the definition (1e-11 of the largest sampled value);
* the solve's residual u + omega^2 K(m (u + u_I)) at sampled points,
  bounded entrywise by the tolerance times ||g||_2, with
  g = -omega^2 K(m u_I) from the oracle's FFT product.
"""
import math
import sys

import numpy as np
import pytest

import oracle
import workloads

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

N_MAX = 2047


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def test_first_refused_size():
    from paper_1705_09443_amd import LSSolver, LsError, _lib
    m = torch.zeros((N_MAX + 1, N_MAX + 1), dtype=torch.float64, device="cuda")
    with pytest.raises(LsError) as ei:
        LSSolver(m, 2 * math.pi * 4.0, 12, 4, precision="mixed")
    assert ei.value.status == _lib.LS_E_INVALID


def test_largest_2d_grid():
    from paper_1705_09443_amd import LSSolver
    n, omega, tol = N_MAX, 2 * math.pi * 32.0, 1e-6
    m = workloads.gaussian_bump_medium(n, 2, 32, (0.2, 0.8), (0.02, 0.05), (-0.4, 0.4), seed=0)
    uinc = workloads.plane_waves(n, 2, omega, workloads.angle_directions(1, 2))
    rng = np.random.default_rng(3)
    pts = rng.integers(0, n, size=(8, 2))
    pts[0] = (0, 0)
    pts[1] = (n - 1, n - 1)
    say(f"[max] setup n={n}, mixed")
    with LSSolver(torch.as_tensor(m).cuda(), omega, 12, 4, precision="mixed") as s:
        x = rng.standard_normal((1, n, n)) + 1j * rng.standard_normal((1, n, n))
        ya = s.apply_A(torch.as_tensor(x).cuda(), precision="fp64").cpu().numpy()[0]
        say("[max] solve, one plane wave")
        u, info = s.solve(torch.as_tensor(uinc).cuda(), "incident", tol)
        u = u.cpu().numpy()[0]
    assert info[0].converged and info[0].rel_residual <= tol
    say(f"[max] {info[0].iterations} iterations; oracle table and direct sums")
    op = oracle.DenseOperator(2, n, omega, m, workers=8)
    want = x[0][tuple(pts.T)] + omega ** 2 * oracle.brute_force_K_at(op.table, n, 2, m * x[0], pts)
    err = np.abs(ya[tuple(pts.T)] - want).max() / np.abs(want).max()
    say(f"[max] A x at {len(pts)} points: relative {err:.2e}")
    assert err <= 1e-11
    g = op.rhs_incident(uinc[0])
    r = u[tuple(pts.T)] + omega ** 2 * oracle.brute_force_K_at(op.table, n, 2, m * (u + uinc[0]), pts)
    bound = 1.01 * tol * np.linalg.norm(g)
    say(f"[max] residual at {len(pts)} points: max {np.abs(r).max():.3e}, bound {bound:.3e}")
    assert np.abs(r).max() <= bound
