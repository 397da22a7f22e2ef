"""The sparsifying stencils as a direct Helmholtz scheme (Sec. 4) on the GPU:
H of a handle with m = 0 solved by ls_solve_H (flexible GMRES, the sweep as
preconditioner) for the right-hand side beta^* f of a point source
(ls_apply_B), against the oracle's sparse direct solve, and, at the largest
grid the library sets up (2047^2 at 3 points per wavelength, 683 wavelengths
across), the far-field phase error against the Green's function that Sec. 4
reports (about 2.3e-4 per wavelength of distance at 3 points per wavelength:
a phase shift of about 1/6 at the corners of a 1024-wavelength square).
"""
import math
import sys

import numpy as np
import pytest

from oracle import alpha_beta, green_table
from oracle import direct

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(b))


def point_source(n):
    h = 1.0 / (n + 1)
    f = np.zeros((1, n, n), dtype=np.complex128)
    c = direct.centre_index(n) - 1
    f[0, c, c] = 1.0 / (h * h)
    return f


@pytest.mark.parametrize("n,ppw,fronts", [(63, 3, 1), (63, 3, 2), (127, 3, 2), (127, 5, 1)])
def test_direct_scheme_matches_the_oracle(n, ppw, fronts):
    from paper_1705_09443_amd import LSSolver
    b, C = 12, 10.0
    omega = 2 * math.pi * (n + 1) / ppw
    st = alpha_beta(green_table(2, n, omega), n, 2)
    uo, system = direct.sparsifying_solve(n, omega, b, C, st)
    md = torch.zeros((n, n), dtype=torch.float64, device="cuda")
    f = torch.as_tensor(point_source(n), device="cuda")
    for prec, tol, bound in (("fp64", 1e-12, 1e-8), ("mixed", 1e-10, 1e-7)):
        with LSSolver(md, omega, b, 4, precision=prec, pml_C=C, fronts=fronts) as s:
            rhs = s.apply_B(f, "fp64")
            ro = direct.beta_rhs(system, point_source(n)[0].real)
            assert rel(rhs.cpu().numpy()[0].reshape(-1), ro) <= 1e-13
            u, info = s.solve_H(rhs, tol)
            ui = u.cpu().numpy()[0][b + 1:b + 1 + n, b + 1:b + 1 + n]
            e = rel(ui, uo)
            say(f"[direct n={n} {ppw} ppw, {fronts} front(s), {prec}] iterations {info[0].iterations}, "
                f"residual {info[0].rel_residual:.2e}, vs oracle {e:.2e}")
            assert info[0].converged and e <= bound
            # the same handle still solves the Lippmann-Schwinger equation
            # (here with m = 0: g = 0 and u = 0 after no iteration)
            z, zi = s.solve(torch.zeros((1, n, n), dtype=torch.complex128, device="cuda"), "source", 1e-6)
            assert zi[0].iterations == 0


@pytest.mark.timeout(900)
def test_phase_error_at_the_largest_grid():
    from paper_1705_09443_amd import LSSolver
    n, ppw, b, C = 2047, 3, 12, 10.0
    omega = 2 * math.pi * (n + 1) / ppw
    say(f"[direct 2047^2] setup: omega/2pi = {omega / (2 * math.pi):.1f}, two fronts, mixed precision")
    md = torch.zeros((n, n), dtype=torch.float64, device="cuda")
    with LSSolver(md, omega, b, 4, precision="mixed", pml_C=C, fronts=2) as s:
        rhs = s.apply_B(torch.as_tensor(point_source(n), device="cuda"), "fp64")
        u, info = s.solve_H(rhs, 1e-8)
    ui = u.cpu().numpy()[0][b + 1:b + 1 + n, b + 1:b + 1 + n]
    shift, relerr = direct.far_field_phase_error(ui, n, omega)
    dphi, rl = direct.phase_error(ui, n, omega)
    corner = float(np.mean([dphi[0, 0], dphi[0, -1], dphi[-1, 0], dphi[-1, -1]]))
    say(f"[direct 2047^2] iterations {info[0].iterations}, residual {info[0].rel_residual:.2e}; far-field shift "
        f"{shift:.4f} wavelengths, {relerr:.2e} per wavelength of distance; corners {corner:.4f} "
        f"({corner / (math.sqrt(0.5) * omega / (2 * math.pi)):.2e} per wavelength)")
    assert info[0].converged
    assert 1e-4 <= relerr <= 5e-4
