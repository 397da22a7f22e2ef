"""The 3D workload at full size: 127^3 interior points, omega = 2 pi 8, PML
b = 8, slabs of w = 4 planes, 16 Gaussian bumps, four incident directions,
mixed precision (complex64 factors and sweep inside float64 FGMRES).

The oracle's setup cannot factor this size within a test, so the check is a
property that holds at any size: every right-hand side converges, and the
whole residual of the returned field, g - A u with A = I + omega^2 K M
(eq. LS_d_c) applied by the oracle's own FFT convolution and
g = -omega^2 K (m u_I), is at most the tolerance times ||g||_2. Sampled
entries are also recomputed by the oracle's direct sum (no FFT at all).
"""
import sys

import numpy as np
import pytest

import oracle
import workloads

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def test_c3_full_size_solve():
    from paper_1705_09443_amd import LSSolver
    wl = workloads.workload("C3")
    n, omega = wl.n, wl.omega
    m = wl.medium_array()
    uinc = wl.incident()
    say(f"[c3] setup n={n} b={wl.pml_width} w={wl.layer_thickness}")
    g = LSSolver(torch.as_tensor(m).cuda(), omega, pml_width=wl.pml_width,
                 layer_thickness=wl.layer_thickness, precision="mixed", schedule="sequential")
    assert g.dim == 3 and g.nslices == (n + 2) // wl.layer_thickness
    say("[c3] solve, 4 incident waves, tol 1e-6")
    u, info = g.solve(torch.as_tensor(uinc).cuda(), "incident", 1e-6)
    u = u.cpu().numpy()
    g.close()
    for i in info:
        assert i.converged and i.rel_residual <= 1e-6 and 0 < i.iterations <= 20
    say("[c3] oracle residual, whole grid (FFT operator) and sampled points (direct sum)")
    op = oracle.DenseOperator(3, n, omega, m, workers=8)
    rng = np.random.default_rng(5)
    pts = rng.integers(0, n, size=(10, 3))
    pts[0] = (0, 0, 0)
    pts[1] = (n - 1, n - 1, n - 1)
    pts[2] = (n // 2, n // 2, n // 2)
    for j in range(wl.nrhs):
        gj = op.rhs_incident(uinc[j])
        whole = np.linalg.norm(gj - op.apply_A(u[j])) / np.linalg.norm(gj)
        total = m * (u[j] + uinc[j])
        r = u[j][tuple(pts.T)] + omega ** 2 * oracle.brute_force_K_at(op.table, n, 3, total, pts)
        bound = 1.01e-6 * np.linalg.norm(gj)
        say(f"[c3]   rhs {j}: iterations {info[j].iterations}, library residual {info[j].rel_residual:.3e}, "
            f"oracle whole-grid residual {whole:.3e}, max sampled residual entry {np.abs(r).max():.3e} "
            f"(||g|| tol {bound:.3e})")
        assert whole <= 1.01e-6
        assert abs(whole - info[j].rel_residual) <= 1e-3 * whole
        assert np.abs(r).max() <= bound
