"""Error paths of the C ABI, each forced from the host with valid arguments:

* LS_E_NOCONV: a tolerance no solve reaches (1e-300) with max_iters = 3. The
  best iterate and the per-right-hand-side info are still written, and the
  iterate equals the oracle's after the same three Arnoldi steps.
* LS_E_NUMERIC: a NaN in a right-hand side (its norm is not finite).
* LS_E_SINGULAR: a PML so strong (pml_C = 1e3, Sec. 2.2.2) that the modified
  plane waves of eq. gamma overflow, so the PML stencils and the first slice
  block are not finite; the slice factorization meets a non-finite pivot, in
  2D and in 3D.

Every kernel still runs to completion on well-formed (if non-finite) data:
nothing here faults or waits on the device.
"""
import math
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


def test_noconv_returns_the_best_iterate():
    from paper_1705_09443_amd import LSSolver, _lib
    n, b, w = 31, 6, 3
    omega = 2 * math.pi * 2.0
    m = workloads.gaussian_bump_medium(n, 2, 6, (0.25, 0.75), (0.05, 0.1), (-0.3, 0.3), seed=0)
    uinc = workloads.plane_waves(n, 2, omega, workloads.angle_directions(2, 2))
    ref = oracle.OracleSolver(2, n, omega, m, b, w)
    say("[error paths] LS_E_NOCONV: tol 1e-300, max_iters 3, fp64")
    with LSSolver(torch.as_tensor(m).cuda(), omega, b, w, precision="fp64", max_iters=3) as s:
        lib = _lib.load()
        rhs = torch.as_tensor(uinc).cuda()
        u = torch.empty_like(rhs)
        infos = (_lib.LsRhsInfo * 2)()
        st = lib.ls_solve(s._h, rhs.data_ptr(), 2, _lib.LS_RHS_INCIDENT, 1e-300, u.data_ptr(), infos)
        assert st == _lib.LS_E_NOCONV, _lib.STATUS_NAMES[st]
        assert "max_iters" in lib.ls_last_error().decode()
        u = u.cpu().numpy()
        for j in range(2):
            assert infos[j].iterations == 3 and not infos[j].converged
            res = ref.solve_rhs(ref.op.rhs_incident(uinc[j]), 1e-300, max_iters=3)
            assert res.iterations == 3 and not res.converged
            err = np.linalg.norm(u[j] - res.x) / np.linalg.norm(res.x)
            say(f"  rhs {j}: residual {infos[j].rel_residual:.3e} (oracle {res.rel_residual:.3e}), "
                f"iterate vs oracle {err:.2e}")
            assert err <= 1e-10
            assert abs(infos[j].rel_residual - res.rel_residual) <= 1e-8 * res.rel_residual
        # the handle stays usable: the next solve runs normally (at most 3 steps)
        v, info = s.solve(torch.as_tensor(uinc).cuda(), "incident", 1e-6, allow_noconv=True)
        assert all(1 <= i.iterations <= 3 for i in info) and bool(torch.isfinite(v).all())


def test_numeric_on_a_nan_right_hand_side():
    from paper_1705_09443_amd import LSSolver, _lib
    n, b, w = 31, 6, 3
    omega = 2 * math.pi * 2.0
    m = workloads.gaussian_bump_medium(n, 2, 6, (0.25, 0.75), (0.05, 0.1), (-0.3, 0.3), seed=0)
    lib = _lib.load()
    for prec in ("fp64", "mixed"):
        say(f"[error paths] LS_E_NUMERIC: NaN in the right-hand side, {prec}")
        with LSSolver(torch.as_tensor(m).cuda(), omega, b, w, precision=prec) as s:
            g = torch.zeros((2, n, n), dtype=torch.complex128, device="cuda")
            g[1, 5, 7] = complex(float("nan"), 0.0)
            g[0, 3, 3] = 1.0
            u = torch.empty_like(g)
            st = lib.ls_solve(s._h, g.data_ptr(), 2, _lib.LS_RHS_SOURCE, 1e-6, u.data_ptr(), None)
            assert st == _lib.LS_E_NUMERIC, _lib.STATUS_NAMES[st]
            assert "non-finite" in lib.ls_last_error().decode()
            # a finite batch on the same handle is solved as usual
            g[1, 5, 7] = 0.0
            v, info = s.solve(g, "source", 1e-6)
            assert info[0].converged and info[1].iterations == 0


@pytest.mark.parametrize("d", [2, 3])
def test_singular_slice_factorization(d):
    from paper_1705_09443_amd import LSSolver, _lib
    n, b, w = (15, 4, 4) if d == 2 else (9, 3, 3)
    omega = 2 * math.pi * 2.0
    m = np.zeros((n,) * d)
    say(f"[error paths] LS_E_SINGULAR: pml_C = 1e3, {d}D n={n}")
    with pytest.raises(_lib.LsError) as ei:
        LSSolver(torch.as_tensor(m).cuda(), omega, b, w, precision="fp64", pml_C=1e3)
    assert ei.value.status == _lib.LS_E_SINGULAR
    assert "pivot" in str(ei.value)
    # the same grid with the default PML sets up and solves
    with LSSolver(torch.as_tensor(m).cuda(), omega, b, w, precision="fp64") as s:
        u, info = s.solve(torch.zeros((1,) + (n,) * d, dtype=torch.complex128, device="cuda"), "source", 1e-6)
        assert info[0].iterations == 0
