"""Parity at the full 2D workload size: 1023^2, omega = 2 pi 64, b = 12, w = 4,
the seeded 32-bump medium, in the launch configurations the benchmark times
(one float64 wave; 64 mixed-precision waves in one batch).

The oracle cannot run the whole path at this size within test time, so the
library is checked on outputs the oracle computes one at a time and on
properties that hold at any size:
* A x at sampled points by direct summation (eq. LS_d_c), float64 and mixed;
* single slice solves T~_k v (eq. Hwv_approx) for the first, a middle and
  the last (32-line) slice against the oracle's sparse LU of that subproblem;
* the solves: every right-hand side's true residual, recomputed with the
  oracle's FFT operator, meets the tolerance, and the float64 iteration
  count is within one of the oracle's on the same wave (parity rule P2).
"""
import os

import numpy as np
import pytest
import torch

import oracle
import workloads
from oracle.sparse import SparseSystem, Sweep

pytestmark = pytest.mark.gpu

SLICES = (0, 128, 255)


def _cores():
    return max(1, min(16, len(os.sched_getaffinity(0))))


@pytest.fixture(scope="module")
def c1():
    wl = workloads.workload("C1")
    m = wl.medium_array()
    op = oracle.DenseOperator(2, wl.n, wl.omega, m, workers=_cores())
    return wl, m, op


@pytest.fixture(scope="module")
def gpu_fp64(c1):
    from paper_1705_09443_amd import LSSolver
    wl, m, _ = c1
    s = LSSolver(torch.as_tensor(m, device="cuda:0"), wl.omega, wl.pml_width, wl.layer_thickness,
                 precision="fp64")
    yield s
    s.close()


@pytest.fixture(scope="module")
def gpu_mixed(c1):
    from paper_1705_09443_amd import LSSolver
    wl2 = workloads.workload("C2")
    _, m, _ = c1
    s = LSSolver(torch.as_tensor(m, device="cuda:0"), wl2.omega, wl2.pml_width, wl2.layer_thickness,
                 precision="mixed", restart=wl2.restart)
    yield s
    s.close()


@pytest.mark.parametrize("precision,bound", [("fp64", 1e-11), ("mixed", 2e-5)])
def test_apply_A_sampled(c1, gpu_fp64, precision, bound):
    wl, m, op = c1
    n = wl.n
    rng = np.random.default_rng(5)
    x = rng.standard_normal((2, n, n)) + 1j * rng.standard_normal((2, n, n))
    y = gpu_fp64.apply_A(torch.as_tensor(x.astype(np.complex128 if precision == "fp64" else np.complex64),
                                         device="cuda:0"), precision=precision).cpu().numpy()
    pts = np.concatenate([rng.integers(0, n, size=(20, 2)), [[0, 0], [n - 1, n - 1], [0, n - 1], [n // 2, n // 2]]])
    for r in range(2):
        yo = x[r][tuple(pts.T)] + op.omega ** 2 * oracle.brute_force_K_at(op.table, n, 2, m * x[r], pts)
        err = np.linalg.norm(y[r][tuple(pts.T)] - yo) / np.linalg.norm(yo)
        print(f"[A {precision} col {r}] sampled relative error {err:.2e}", flush=True)
        assert err <= bound


@pytest.fixture(scope="module")
def oracle_slices(c1):
    wl, m, op = c1
    alpha, beta, _ = oracle.alpha_beta(op.table, wl.n, 2)
    system = SparseSystem(2, wl.n, wl.omega, m, alpha, beta, wl.pml_width, oracle.DEFAULT_PML_C)
    return Sweep(system, wl.layer_thickness, m, only=list(SLICES))


@pytest.mark.parametrize("precision,bound", [("fp64", 1e-10), ("mixed", 1e-4)])
def test_slice_solves_sampled_slices(c1, gpu_fp64, gpu_mixed, oracle_slices, precision, bound):
    wl, _, _ = c1
    sw = oracle_slices
    gpu = gpu_fp64 if precision == "fp64" else gpu_mixed
    assert gpu.nslices == sw.nslices
    rng = np.random.default_rng(11)
    for k in SLICES:
        lo, hi, naux = gpu.slice_bounds(k)
        assert (lo, hi) == sw.bounds[k] and naux * gpu.L == sw.aux_count[k]
        v = rng.standard_normal((2, hi - lo + 1, gpu.L)) + 1j * rng.standard_normal((2, hi - lo + 1, gpu.L))
        dt = np.complex128 if precision == "fp64" else np.complex64
        w = gpu.slice_solve(k, torch.as_tensor(v.astype(dt), device="cuda:0"), precision=precision)
        w = w.cpu().numpy()
        for r in range(2):
            wo = sw.solve_slice(k, v[r].reshape(-1)).reshape(v[r].shape)
            err = np.linalg.norm(w[r] - wo) / np.linalg.norm(wo)
            print(f"[slice {k} {precision} col {r}] t={hi - lo + 1 + naux} relative error {err:.2e}", flush=True)
            assert err <= bound


def _true_residuals(op, wl_nrhs_uinc, u):
    out = []
    for j in range(u.shape[0]):
        g = op.rhs_incident(wl_nrhs_uinc[j])
        out.append(np.linalg.norm(g - op.apply_A(u[j])) / np.linalg.norm(g))
    return np.array(out)


def test_fp64_solve_residual_and_iterations(c1, gpu_fp64):
    wl, m, op = c1
    uinc = wl.incident()
    u, info = gpu_fp64.solve(torch.as_tensor(uinc, device="cuda:0"), "incident", wl.tol)
    res = _true_residuals(op, uinc, u.cpu().numpy())
    print(f"[C1 fp64] iterations {info[0].iterations}, library residual {info[0].rel_residual:.2e}, "
          f"oracle-operator residual {res[0]:.2e}", flush=True)
    assert info[0].converged and res[0] <= wl.tol * 1.01
    o = oracle.OracleSolver(2, wl.n, wl.omega, m, wl.pml_width, wl.layer_thickness, workers=_cores())
    ro = o.solve_incident(uinc, tol=wl.tol)[0]
    print(f"[C1 oracle] iterations {ro.iterations}, residual {ro.rel_residual:.2e}", flush=True)
    assert abs(ro.iterations - info[0].iterations) <= 1


def test_mixed_batched_solve_residuals(c1, gpu_mixed):
    wl2 = workloads.workload("C2")
    _, m, op = c1
    uinc = wl2.incident()
    u, info = gpu_mixed.solve(torch.as_tensor(uinc, device="cuda:0"), "incident", wl2.tol)
    u = u.cpu().numpy()
    res = _true_residuals(op, uinc, u)
    its = [i.iterations for i in info]
    print(f"[C2 mixed] 64 waves, iterations {min(its)}..{max(its)}, oracle-operator residual max {res.max():.2e}",
          flush=True)
    assert all(i.converged for i in info)
    assert res.max() <= wl2.tol * 1.01
