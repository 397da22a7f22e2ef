"""The sparsifying stencils as a direct discretisation of the Helmholtz
equation, and the quasi-stabilised FEM stencil it is compared with (Sec. 4;
oracle; test infrastructure only).

Problem (eq. 2D_Helm_comparison): (-Laplacian - omega^2) u = f on the plane, f
a point source at the centre of the unit square, whose solution is the
free-space Green's function G(r) = (i/4) H0(omega r) about that centre.

Sparsifying scheme: at every point i of I^h the 9-point equation
alpha^* u_{mu_i} = beta^* f_{mu_i} with the stencils alpha, beta of eqs.
alpha and beta (those of the Lippmann-Schwinger sparsification: u = K f with
k_delta = G(|delta| h) h^2, so the discrete point source is f = delta / h^2),
and the PML rows gamma_i^* u_{mu_i} = 0 outside it (eq. gamma, the PML of
Sec. 2.2.2). This is the sparse system H of eq. Huf with m = 0 and the
right-hand side formed with beta in place of alpha.

QSFEM (Babuska et al., as quoted in Sec. 4; reading G17 for its typos and
G19 for A2): the 9-point stencil [A2 A1 A2; A1 A0 A1; A2 A1 A2], A0 = 4, on the
same points, with the same PML rows, and the point source at the centre.

Phase error: with u = A exp(2 pi i phi), the difference phi - phi_G, taken as
arg(u / G) / (2 pi) (no unwrapping needed while it stays below half a
wavelength); relative to the distance in wavelengths omega r / (2 pi).
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .green import green, green_table
from .stencils import alpha_beta
from .sparse import SparseSystem


def qsfem_coefficients(kappa: float):
    """(A0, A1, A2) of the QSFEM stencil at kappa = omega h (Sec. 4).

    A1 as printed. A2 (reading G19): the printed A2 carries a factor 2 that
    the stencil's defining property does not allow; QSFEM is the 9-point
    stencil with A0 = 4 whose symbol A0 + 2 A1 (cos(kappa cos t) + cos(kappa
    sin t)) + 4 A2 cos(kappa cos t) cos(kappa sin t) vanishes at t = pi/16 and
    3 pi/16. Solving those two conditions reproduces the printed A1 exactly
    and gives A2 = (c2 + s2 - c1 - s1) / D with the printed denominator D."""
    c1, s1 = math.cos(kappa * math.cos(math.pi / 16)), math.cos(kappa * math.sin(math.pi / 16))
    c2, s2 = math.cos(kappa * math.cos(3 * math.pi / 16)), math.cos(kappa * math.sin(3 * math.pi / 16))
    den = c2 * s2 * (c1 + s1) - c1 * s1 * (c2 + s2)
    return 4.0, 2.0 * (c1 * s1 - c2 * s2) / den, (c2 + s2 - c1 - s1) / den


def centre_index(n: int) -> int:
    """Grid index of the point (1/2, 1/2): n must be odd."""
    if n % 2 == 0:
        raise ValueError("n must be odd so that (1/2, 1/2) is a grid point")
    return (n + 1) // 2


def _point_source(n: int) -> np.ndarray:
    f = np.zeros((n, n))
    c = centre_index(n) - 1
    f[c, c] = 1.0
    return f


def sparsifying_system(n: int, omega: float, b: int, C: float, stencils=None) -> SparseSystem:
    """H of eq. Huf with m = 0 (type-1 rows alpha^*, PML rows gamma^*)."""
    if stencils is None:
        stencils = alpha_beta(green_table(2, n, omega), n, 2)
    alpha, beta, _ = stencils
    return SparseSystem(2, n, omega, np.zeros((n, n)), alpha, beta, b, C)


def beta_rhs(system: SparseSystem, f: np.ndarray) -> np.ndarray:
    """beta^* f_{mu_i} on I^h, 0 on the PML: the right-hand side of the
    scheme, f given on the interior grid."""
    L, b, n = system.L, system.b, system.n
    x = system.extend(f).reshape(L, L)
    out = np.zeros_like(x)
    core = (slice(b, b + n + 2),) * 2
    for o, off in enumerate(system.mu):
        src = tuple(slice(b + off[k], b + n + 2 + off[k]) for k in range(2))
        out[core] += np.conj(system.beta[o]) * x[src]
    return out.reshape(-1)


def sparsifying_solve(n: int, omega: float, b: int, C: float, stencils=None):
    """The scheme's field on the interior grid for the point source
    f = delta / h^2 at the centre (so that it approximates G)."""
    s = sparsifying_system(n, omega, b, C, stencils)
    h = 1.0 / (n + 1)
    rhs = beta_rhs(s, _point_source(n) / (h * h))
    return s.restrict(spla.spsolve(s.H.tocsc(), rhs)), s


def qsfem_solve(n: int, omega: float, b: int, C: float, stencils=None):
    """QSFEM on I^h with the same PML rows; the point source at the centre
    (unit weight: the phase does not depend on the source's scale)."""
    s = sparsifying_system(n, omega, b, C, stencils)
    h = 1.0 / (n + 1)
    A0, A1, A2 = qsfem_coefficients(omega * h)
    coef = {(0, 0): A0}
    for d in ((0, 1), (0, -1), (1, 0), (-1, 0)):
        coef[d] = A1
    for d in ((1, 1), (1, -1), (-1, 1), (-1, -1)):
        coef[d] = A2
    L = s.L
    H = s.H.tolil()
    gi = s.gi
    for p in np.nonzero(s.type1)[0]:
        i1, i2 = gi[p]
        H.rows[p] = []
        H.data[p] = []
        for (d1, d2), v in coef.items():
            H[p, (i1 + d1 + s.b) * L + (i2 + d2 + s.b)] = v
    H = H.tocsc()
    rhs = s.extend(_point_source(n).astype(np.complex128))
    return s.restrict(spla.spsolve(H, rhs)), s


def green_field(n: int, omega: float) -> np.ndarray:
    """G(|x - (1/2, 1/2)|) on the interior grid (the centre itself excluded:
    set to 1)."""
    h = 1.0 / (n + 1)
    x = np.arange(1, n + 1) * h - 0.5
    r = np.sqrt(x[:, None] ** 2 + x[None, :] ** 2)
    out = np.ones((n, n), dtype=np.complex128)
    nz = r > 0
    out[nz] = green(2, omega, r[nz])
    return out


def phase_error(u: np.ndarray, n: int, omega: float):
    """(phi - phi_G, r / lambda) on the interior grid: the phase difference in
    wavelengths and the distance from the source in wavelengths."""
    h = 1.0 / (n + 1)
    x = np.arange(1, n + 1) * h - 0.5
    r = np.sqrt(x[:, None] ** 2 + x[None, :] ** 2)
    dphi = np.angle(u / green_field(n, omega)) / (2 * math.pi)
    return dphi, r * omega / (2 * math.pi)


def far_field_phase_error(u: np.ndarray, n: int, omega: float, rmin: float = 0.6):
    """Mean phase shift (wavelengths) over the points at least rmin from the
    source, and the same relative to their mean distance in wavelengths."""
    dphi, rl = phase_error(u, n, omega)
    h = 1.0 / (n + 1)
    x = np.arange(1, n + 1) * h - 0.5
    r = np.sqrt(x[:, None] ** 2 + x[None, :] ** 2)
    sel = r >= rmin
    shift = float(np.mean(dphi[sel]))
    return shift, shift / float(np.mean(rl[sel]))
