"""GPU adjoint gradient of a receiver misfit with respect to m.

The paper has no adjoint; the gradient follows from eq. LS_d_c: with
psi = u + u_I and A nu_j = K conj(r_j), dJ/dm = -omega^2 Re sum_j psi_j nu_j
for J = 1/2 sum_j |R u_j - d_j|^2 and r_j = R^T (R u_j - d_j).

Checked through the C ABI (ls_solve then ls_adjoint) against
* the oracle's gradient on the same inputs (float64 1e-8, mixed 1e-5),
* central finite differences of J computed with GPU solves (1e-5),
* the torch.autograd.Function path, and gradcheck on a 7 x 7 grid.
"""
import numpy as np
import pytest
import torch

import workloads
from oracle import OracleSolver

pytestmark = pytest.mark.gpu

N, PPW, B, W = 31, 2.0, 6, 3
NDIR = 3
TOL = 1e-12


def _case():
    wl = workloads.workload("C4").scaled(N, ppw_omega=PPW)
    m = workloads.gaussian_bump_medium(N, 2, 6, (0.25, 0.75), (0.05, 0.1), (-0.3, 0.3), seed=0)
    md = workloads.gaussian_bump_medium(N, 2, 6, (0.25, 0.75), (0.05, 0.1), (-0.3, 0.3), seed=1)
    dirs = workloads.angle_directions(NDIR, 2)
    uinc = workloads.plane_waves(N, 2, wl.omega, dirs)
    rec = workloads.circle_receivers(N, 0.4)
    return wl.omega, m, md, uinc, rec


@pytest.fixture(scope="module")
def case():
    omega, m, md, uinc, rec = _case()
    # data: the oracle's fields for the second medium
    od = OracleSolver(2, N, omega, md, B, W)
    data = np.array([r.x[rec] for r in od.solve_incident(uinc, tol=TOL)])
    o = OracleSolver(2, N, omega, m, B, W)
    uo = np.array([r.x for r in o.solve_incident(uinc, tol=TOL)])
    ro = np.zeros_like(uo)
    for j in range(NDIR):
        ro[j][rec] = uo[j][rec] - data[j]
    grad_o = o.gradient(uo, ro, uinc, tol=TOL)
    return dict(omega=omega, m=m, uinc=uinc, rec=rec, data=data, grad_o=grad_o)


def _gpu_misfit_and_grad(c, m, precision, with_grad=True):
    from paper_1705_09443_amd import LSSolver
    dev = torch.device("cuda:0")
    s = LSSolver(torch.as_tensor(m, device=dev), c["omega"], B, W, precision=precision)
    try:
        u, info = s.solve(torch.as_tensor(c["uinc"], device=dev), "incident", TOL)
        assert all(i.converged for i in info)
        u = u.cpu().numpy()
        rec = c["rec"]
        r = np.zeros_like(u)
        J = 0.0
        for j in range(NDIR):
            r[j][rec] = u[j][rec] - c["data"][j]
            J += 0.5 * np.sum(np.abs(r[j][rec]) ** 2)
        if not with_grad:
            return J, None
        g, ginfo = s.adjoint(torch.as_tensor(r, device=dev), TOL)
        assert all(i.converged for i in ginfo)
        return J, g.cpu().numpy()
    finally:
        s.close()


@pytest.mark.parametrize("precision,bound", [("fp64", 1e-8), ("mixed", 1e-5)])
def test_adjoint_matches_oracle(case, precision, bound):
    _, g = _gpu_misfit_and_grad(case, case["m"], precision)
    go = case["grad_o"]
    err = np.linalg.norm(g - go) / np.linalg.norm(go)
    print(f"[adjoint {precision}] relative L2 vs oracle gradient {err:.2e}", flush=True)
    assert err <= bound


def test_adjoint_central_differences(case):
    J0, g = _gpu_misfit_and_grad(case, case["m"], "fp64")
    eps = 1e-6
    for k, dm in enumerate(workloads.fd_directions(N, 2, 3, seed=2)):
        jp, _ = _gpu_misfit_and_grad(case, case["m"] + eps * dm, "fp64", with_grad=False)
        jm, _ = _gpu_misfit_and_grad(case, case["m"] - eps * dm, "fp64", with_grad=False)
        fd = (jp - jm) / (2 * eps)
        an = float(np.sum(g * dm))
        rel = abs(fd - an) / abs(an)
        print(f"[fd {k}] fd {fd:.10e} adjoint {an:.10e} rel {rel:.2e} (J {J0:.3e})", flush=True)
        assert rel <= 1e-5


def test_autograd_function_matches_oracle(case):
    from paper_1705_09443_amd import LSSolve
    dev = torch.device("cuda:0")
    m = torch.as_tensor(case["m"], device=dev).clone().requires_grad_(True)
    uinc = torch.as_tensor(case["uinc"], device=dev)
    u = LSSolve.apply(m, uinc, case["omega"], B, W, "fp64", TOL, TOL)
    rec = torch.as_tensor(case["rec"], device=dev)
    d = torch.as_tensor(case["data"], device=dev)
    J = 0.5 * sum(((u[j][rec] - d[j]).abs() ** 2).sum() for j in range(NDIR))
    J.backward()
    g = m.grad.cpu().numpy()
    go = case["grad_o"]
    err = np.linalg.norm(g - go) / np.linalg.norm(go)
    print(f"[autograd] relative L2 vs oracle gradient {err:.2e}", flush=True)
    assert err <= 1e-8


def test_gradcheck_tiny_grid():
    from paper_1705_09443_amd import LSSolve
    dev = torch.device("cuda:0")
    n = 7
    omega = 2 * np.pi * 1.0
    m0 = workloads.gaussian_bump_medium(n, 2, 2, (0.3, 0.7), (0.1, 0.2), (-0.3, 0.3), seed=3)
    uinc = torch.as_tensor(workloads.plane_waves(n, 2, omega, workloads.angle_directions(2, 2)), device=dev)
    m = torch.as_tensor(m0, device=dev).clone().requires_grad_(True)
    fn = lambda mm: LSSolve.apply(mm, uinc, omega, 3, 2, "fp64", 1e-13, 1e-13)
    assert torch.autograd.gradcheck(fn, (m,), eps=1e-6, atol=1e-7, rtol=1e-5)
