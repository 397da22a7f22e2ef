"""ls_solve with the output written over the input (u_dev == rhs_dev).

The solve reads the right-hand side (or incident wave) when it forms g and
once more when it writes u and the total field psi = u + u_I kept for
ls_adjoint; each element is read before u is written. So an in-place call
must give the same u, bit for bit, as a call with separate arrays, and the
adjoint gradient that follows must be the same too (it reads psi). Checked
through the C ABI for both kinds of right-hand side, float64 and mixed.
"""
import numpy as np
import pytest
import torch

import workloads

pytestmark = pytest.mark.gpu

N, PPW, B, W, NRHS = 31, 4.0, 6, 4, 3


def say(msg):
    print(msg, flush=True)


def _solve_into(s, buf, kind, tol):
    from paper_1705_09443_amd import _lib
    from paper_1705_09443_amd._lib import LS_RHS_INCIDENT, LS_RHS_SOURCE, LsRhsInfo
    k = buf.shape[0]
    infos = (LsRhsInfo * k)()
    st = s._lib.ls_solve(s._h, buf.data_ptr(), k, LS_RHS_INCIDENT if kind == "incident" else LS_RHS_SOURCE,
                         float(tol), buf.data_ptr(), infos)
    _lib.check(st, "ls_solve")
    return [i.iterations for i in infos]


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("kind", ["incident", "source"])
def test_in_place_solve_matches(precision, kind):
    from paper_1705_09443_amd import LSSolver
    wl = workloads.workload("C2").scaled(N, ppw_omega=PPW)
    m = workloads.gaussian_bump_medium(N, 2, 6, (0.25, 0.75), (0.05, 0.1), (-0.3, 0.3), seed=0)
    rhs = workloads.plane_waves(N, 2, wl.omega, workloads.angle_directions(NRHS, 2))
    rng = np.random.default_rng(5)
    resid = torch.as_tensor(rng.standard_normal((NRHS, N, N)) + 1j * rng.standard_normal((NRHS, N, N))).cuda()
    tol = 1e-10 if precision == "fp64" else 1e-6
    say(f"[inplace] {kind} {precision}: n={N}, {NRHS} rhs")
    with LSSolver(torch.as_tensor(m).cuda(), wl.omega, B, W, precision=precision) as s:
        x = torch.as_tensor(rhs).cuda()
        u_ref, info = s.solve(x, kind, tol)
        g_ref, _ = s.adjoint(resid, 1e-10)
        buf = x.clone()
        iters = _solve_into(s, buf, kind, tol)
        g_in, _ = s.adjoint(resid, 1e-10)
    assert iters == [i.iterations for i in info]
    assert torch.equal(buf, u_ref)
    assert torch.equal(g_in, g_ref)
    say(f"[inplace] {kind} {precision}: iterations {iters}, u and the gradient bitwise equal")
