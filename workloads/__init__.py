"""Seeded synthetic inputs for the Lippmann-Schwinger solver: media, incident
waves, receiver masks and perturbation directions.

This module holds only input generation. It performs none of the method's
arithmetic (no Green's function, no stencils, no solves), so both the CPU
oracle and the GPU library may consume what it produces.

Grid convention (Section 2.1 of the paper): the unit cube (0,1)^d carries n
interior points per axis, h = 1/(n+1), point p_i = i*h for i in [1, n]^d.
Arrays are C-ordered [n]^d with array index a_k = i_k - 1; axis 0 is x1, the
sweep direction.

The paper describes its velocity fields only in words (converging and
diverging Gaussians, many narrow Gaussians). The media below are seeded sums
of Gaussian bumps that stand in for them; draws use numpy's default_rng in
the order centres (K x d), widths (K), amplitudes (K).
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional, Sequence

import numpy as np

__all__ = [
    "grid_points",
    "single_gaussian_medium",
    "gaussian_bump_medium",
    "plane_waves",
    "circle_receivers",
    "fd_directions",
    "Workload",
    "WORKLOADS",
    "workload",
]


def grid_points(n: int, d: int) -> list[np.ndarray]:
    """Coordinates of the interior points, one array of shape [n]^d per axis."""
    h = 1.0 / (n + 1)
    x = np.arange(1, n + 1, dtype=np.float64) * h
    return list(np.meshgrid(*([x] * d), indexing="ij"))


def _threshold(m: np.ndarray, cut: float) -> np.ndarray:
    m = m.copy()
    m[np.abs(m) < cut] = 0.0
    return m


def single_gaussian_medium(n: int, d: int = 2, amplitude: float = 0.3,
                           width: float = 0.1, cut: float = 1e-8) -> np.ndarray:
    """m(x) = amplitude * exp(-|x - c|^2 / (2 width^2)), c the cube centre,
    set to zero where it falls below ``cut``."""
    xs = grid_points(n, d)
    r2 = sum((x - 0.5) ** 2 for x in xs)
    return _threshold(amplitude * np.exp(-r2 / (2.0 * width * width)), cut)


def gaussian_bump_medium(n: int, d: int, count: int, centre: tuple[float, float],
                         width: tuple[float, float], amplitude: tuple[float, float],
                         seed: int, cut: float = 1e-8) -> np.ndarray:
    """Sum of ``count`` Gaussian bumps with uniformly drawn centres, widths and
    amplitudes (seeded). Values below ``cut`` in modulus are set to zero."""
    rng = np.random.default_rng(seed)
    centres = rng.uniform(centre[0], centre[1], size=(count, d))
    widths = rng.uniform(width[0], width[1], size=count)
    amps = rng.uniform(amplitude[0], amplitude[1], size=count)
    xs = grid_points(n, d)
    m = np.zeros((n,) * d, dtype=np.float64)
    for k in range(count):
        r2 = sum((xs[a] - centres[k, a]) ** 2 for a in range(d))
        m += amps[k] * np.exp(-r2 / (2.0 * widths[k] ** 2))
    m = _threshold(m, cut)
    if m.max() >= 1.0:
        raise ValueError("medium has m >= 1 somewhere: the local frequency would not be real")
    return m


def plane_waves(n: int, d: int, omega: float, directions: np.ndarray) -> np.ndarray:
    """Incident plane waves u_I(x) = exp(i omega r.x) sampled at the interior
    points, one per row of ``directions`` (unit vectors, shape [k, d]).
    Returns complex128 [k][n]^d."""
    xs = grid_points(n, d)
    out = np.empty((len(directions),) + (n,) * d, dtype=np.complex128)
    for j, r in enumerate(np.asarray(directions, dtype=np.float64)):
        phase = sum(r[a] * xs[a] for a in range(d))
        out[j] = np.exp(1j * omega * phase)
    return out


def angle_directions(count: int, d: int = 2, full_turn: bool = True) -> np.ndarray:
    """Unit vectors (cos t_j, sin t_j[, 0]) with t_j = 2 pi j / count (or
    pi j / 2 steps for the four 3D directions when full_turn is False)."""
    if full_turn:
        t = 2.0 * math.pi * np.arange(count) / count
    else:
        t = 0.5 * math.pi * np.arange(count)
    dirs = np.zeros((count, d))
    dirs[:, 0] = np.cos(t)
    dirs[:, 1] = np.sin(t)
    return dirs


def circle_receivers(n: int, radius: float = 0.45) -> np.ndarray:
    """Boolean [n, n] mask of the grid points within h/2 of the circle of the
    given radius about (0.5, 0.5)."""
    h = 1.0 / (n + 1)
    x1, x2 = grid_points(n, 2)
    dist = np.sqrt((x1 - 0.5) ** 2 + (x2 - 0.5) ** 2)
    return np.abs(dist - radius) <= 0.5 * h


def fd_directions(n: int, d: int, count: int, seed: int) -> np.ndarray:
    """``count`` seeded perturbation directions, N(0,1) per point, each scaled
    to max-norm 1. Shape [count][n]^d float64."""
    rng = np.random.default_rng(seed)
    dm = rng.standard_normal((count,) + (n,) * d)
    for k in range(count):
        dm[k] /= np.abs(dm[k]).max()
    return dm


@dataclasses.dataclass(frozen=True)
class Workload:
    """One benchmark / parity configuration: grid, frequency, medium recipe,
    incident directions and solver parameters."""
    name: str
    d: int
    n: int
    ppw_omega: float          # omega / (2 pi)
    pml_width: int            # b
    layer_thickness: int      # w
    nrhs: int
    precision: str            # "fp64" or "mixed"
    medium: str               # "single" or "bumps"
    bump_count: int = 0
    bump_centre: tuple = (0.0, 0.0)
    bump_width: tuple = (0.0, 0.0)
    bump_amp: tuple = (0.0, 0.0)
    seed: int = 0
    restart: int = 30
    tol: float = 1e-6
    adjoint: bool = False

    @property
    def omega(self) -> float:
        return 2.0 * math.pi * self.ppw_omega

    @property
    def h(self) -> float:
        return 1.0 / (self.n + 1)

    def medium_array(self, seed: Optional[int] = None) -> np.ndarray:
        if self.medium == "single":
            return single_gaussian_medium(self.n, self.d)
        return gaussian_bump_medium(self.n, self.d, self.bump_count, self.bump_centre,
                                    self.bump_width, self.bump_amp,
                                    self.seed if seed is None else seed)

    def directions(self) -> np.ndarray:
        if self.d == 3:
            dirs = angle_directions(self.nrhs, 3, full_turn=False)
        else:
            dirs = angle_directions(self.nrhs, 2, full_turn=True)
        return dirs

    def incident(self) -> np.ndarray:
        return plane_waves(self.n, self.d, self.omega, self.directions())

    def scaled(self, n: int, ppw_omega: Optional[float] = None, nrhs: Optional[int] = None,
               name: Optional[str] = None) -> "Workload":
        """Same recipe on another grid (keeps points per wavelength unless
        ``ppw_omega`` is given)."""
        if ppw_omega is None:
            ppw_omega = self.ppw_omega * (n + 1) / (self.n + 1)
        return dataclasses.replace(self, n=n, ppw_omega=ppw_omega,
                                   nrhs=self.nrhs if nrhs is None else nrhs,
                                   name=name or f"{self.name}@{n}")


_BUMPS_2D = dict(medium="bumps", bump_centre=(0.2, 0.8), bump_width=(0.02, 0.05),
                 bump_amp=(-0.4, 0.4))

WORKLOADS = {
    # 2D, 63^2, one Gaussian, FP64, one plane wave: the small parity case.
    "C0": Workload("C0", 2, 63, 4.0, 12, 4, 1, "fp64", "single"),
    # 2D, 1023^2, 32 bumps, FP64, one plane wave.
    "C1": Workload("C1", 2, 1023, 64.0, 12, 4, 1, "fp64", bump_count=32, seed=0, **_BUMPS_2D),
    # Same medium, 64 plane waves as one batch, mixed precision.
    "C2": Workload("C2", 2, 1023, 64.0, 12, 4, 64, "mixed", bump_count=32, seed=0, **_BUMPS_2D),
    # 3D, 127^3, 16 bumps, four directions, mixed precision.
    "C3": Workload("C3", 3, 127, 8.0, 8, 4, 4, "mixed", "bumps", bump_count=16,
                   bump_centre=(0.25, 0.75), bump_width=(0.03, 0.06), bump_amp=(-0.3, 0.3), seed=0),
    # 2D, 511^2, 16 bumps, 32 plane waves, adjoint gradient.
    "C4": Workload("C4", 2, 511, 32.0, 12, 4, 32, "mixed", bump_count=16, seed=0,
                   adjoint=True, **_BUMPS_2D),
}


def workload(name: str) -> Workload:
    return WORKLOADS[name]
