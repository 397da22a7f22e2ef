"""Local stencils of the sparsified system (oracle; test infrastructure only).

Type 1 (interior points), Sec. 2.2.1, eqs. alpha and beta:
    alpha minimises ||alpha^* K_{mu,mu^c}||_2 over unit vectors, with
    mu = {j : |j|_inf <= 1} and mu^c = [-n, n]^d minus mu; beta^* = alpha^* K_{mu,mu}.
Type 2 (PML points), Sec. 2.2.2, eq. gamma: gamma_i spans the left null
space of the modified plane waves F^sigma(x) = exp(i omega r . x^sigma)
sampled on mu_i, for the 8 compass directions in 2D (Sec. 2.2.2) or the 26
neighbour directions in 3D (Sec. 3.1).
Local frequency samples for the auxiliary PML, Sec. 2.3.

Neighbourhood order: offsets in {-1,0,1}^d, lexicographic with axis 0
slowest; the centre is index (3^d - 1) / 2.
"""
from __future__ import annotations

import itertools
import math

import numpy as np


def neighbourhood(d: int) -> np.ndarray:
    """Offsets of mu, shape [3^d, d], lexicographic (axis 0 slowest)."""
    return np.array(list(itertools.product((-1, 0, 1), repeat=d)), dtype=np.int64)


def plane_wave_directions(d: int) -> np.ndarray:
    """r = v/|v| for v in {-1,0,1}^d minus 0 (reading G7): the 8 compass
    directions in 2D (Sec. 2.2.2), the 26 neighbour directions in 3D (Sec. 3.1)."""
    v = np.array([o for o in itertools.product((-1, 0, 1), repeat=d) if any(o)], dtype=np.float64)
    return v / np.linalg.norm(v, axis=1, keepdims=True)


def normalise_phase(v: np.ndarray) -> np.ndarray:
    """Reading G5: unit 2-norm, centre coefficient real and positive (if the
    centre is below 1e-12 in modulus, the first largest-modulus entry instead).
    The paper fixes the stencils only up to a scalar."""
    v = v / np.linalg.norm(v)
    j = (len(v) - 1) // 2
    if abs(v[j]) < 1e-12:
        j = int(np.argmax(np.abs(v)))
    c = v[j]
    v = v * (np.conj(c) / abs(c))
    v[j] = abs(c)          # exactly real, free of the rotation's rounding
    return v


def alpha_beta(table: np.ndarray, n: int, d: int, chunk_rows: int = 1 << 16):
    """Type-1 stencils alpha, beta (eqs. alpha, beta; readings G4, G5, G6).

    alpha is the right singular vector of K_{mu,mu^c}^H for its smallest
    singular value, found by a tall-skinny QR of K_{mu,mu^c}^H (rows stream
    over l in [-n,n]^d minus mu) followed by the SVD of the small R factor.
    Returns (alpha, beta, singular_values_of_K_mu_muc)."""
    mu = neighbourhood(d)
    c = n + 1  # table centre
    # Enumerate l over [-n, n]^d in row-major order, one axis-0 slab at a time.
    R = None
    tail = (2 * n + 1,) * (d - 1)
    rest = np.indices(tail).reshape(d - 1, -1).T - n   # offsets of the remaining axes
    for l0 in range(-n, n + 1):
        l = np.concatenate([np.full((len(rest), 1), l0), rest], axis=1)
        keep = np.abs(l).max(axis=1) > 1                 # l not in mu
        l = l[keep]
        # rows of K_{mu,mu^c}^H: conj(k_{j-l}) for j in mu
        off = mu[None, :, :] - l[:, None, :] + c
        block = np.conj(table[tuple(off[..., a] for a in range(d))])
        for s in range(0, len(block), chunk_rows):
            part = block[s:s + chunk_rows]
            stacked = part if R is None else np.vstack([R, part])
            R = np.linalg.qr(stacked, mode="r")
    _, sv, Vh = np.linalg.svd(R)
    alpha = normalise_phase(np.conj(Vh[-1]))
    # beta^* = alpha^* K_{mu,mu}:  beta_l = sum_j conj(k_{j-l}) alpha_j
    off = mu[:, None, :] - mu[None, :, :] + c                      # [j, l]
    Kmm = table[tuple(off[..., a] for a in range(d))]
    beta = Kmm.conj().T @ alpha
    return alpha, beta, sv


def sigma_global(i, n: int, b: int, C: float, omega: float):
    """Global PML stretch sigma(x) at x = i h (Sec. 2.2.2), per axis index i.

    sigma = -(C/omega)((x+h)/eta)^2 for x <= -h, (C/omega)((x-1-h)/eta)^2 for
    x >= 1+h, 0 in between, with eta = b h. In index form: q = -1-i on the
    low side and q = i-n-2 on the high side give -/+ (C/omega)(q/b)^2. At the
    Dirichlet points i = -(b+1) and n+2+b the formula is continued (G3)."""
    i = np.asarray(i, dtype=np.float64)
    lo = np.where(i <= -1, -(C / omega) * ((-1.0 - i) / b) ** 2, 0.0)
    hi = np.where(i >= n + 2, (C / omega) * ((i - n - 2.0) / b) ** 2, 0.0)
    return lo + hi


def sigma_aux(line, first_line: int, b: int, C: float, omega: float):
    """Auxiliary x1 stretch left of a slice starting at ``first_line`` (moving
    PML, Sec. 2.3; readings G8, G10): zero from first_line-1 on, and
    -(C/omega)(q/b)^2 at first_line-1-q, q = 0..b (q = b is the Dirichlet line)."""
    line = np.asarray(line, dtype=np.float64)
    q = (first_line - 1.0) - line
    return np.where(q > 0, -(C / omega) * (q / b) ** 2, 0.0)


def sigma_aux_right(line, last_line: int, b: int, C: float, omega: float):
    """Auxiliary x1 stretch right of a slice ending at ``last_line`` (the
    two-front sweep's bottom front and middle slice, remark 1 closing Sec. 2.4):
    the mirror image of sigma_aux, zero up to last_line+1 and
    +(C/omega)(q/b)^2 at last_line+1+q, q = 0..b (q = b is the Dirichlet line)."""
    line = np.asarray(line, dtype=np.float64)
    q = line - (last_line + 1.0)
    return np.where(q > 0, (C / omega) * (q / b) ** 2, 0.0)


def pml_stencil(kappa: float, h: float, sig: np.ndarray, dirs: np.ndarray) -> np.ndarray:
    """gamma for one point (eq. gamma).

    ``sig`` has shape [d, 3]: sigma of axis k at offsets -1, 0, +1 from the
    centre. Column r of the sampled modified plane wave exp(i kappa r.x^sigma)
    on mu is scaled by its value at the centre, which leaves its left null
    space unchanged:
        F'_{o,r} = exp(i kappa h r.o) exp(-kappa sum_k r_k (sig_k[o_k] - sig_k[0])).
    gamma is the right singular vector of F'^H for the smallest singular value."""
    d = sig.shape[0]
    mu = neighbourhood(d)
    phase = np.exp(1j * kappa * h * (mu @ dirs.T))                     # [3^d, |R|]
    dsig = np.stack([sig[k, mu[:, k] + 1] - sig[k, 1] for k in range(d)], axis=1)  # [3^d, d]
    damp = np.exp(-kappa * (dsig @ dirs.T))
    F = phase * damp
    _, _, Vh = np.linalg.svd(F.conj().T)
    return normalise_phase(np.conj(Vh[-1]))


class FrequencySamples:
    """Squared local frequencies sampled on [omega^2(1-max m), omega^2(1-min m)]
    (Sec. 2.3; reading G9): n_s = n samples with both endpoints (1 if the
    range is a point); a point takes the sample nearest to omega^2 (1 - m(x)),
    with m = 0 off the interior grid."""

    def __init__(self, m: np.ndarray, omega: float, count: int):
        w2 = omega * omega
        mmax = float(m.max())
        mmin = float(m.min())
        if not (1.0 - mmax > 0.0):
            raise ValueError("1 - max m must be positive")
        self.lo = w2 * (1.0 - mmax)
        self.hi = w2 * (1.0 - mmin)
        self.count = count if self.hi > self.lo else 1
        self.delta = (self.hi - self.lo) / (self.count - 1) if self.count > 1 else 0.0
        self.w2 = w2

    def index(self, m_at_point: np.ndarray) -> np.ndarray:
        m_at_point = np.asarray(m_at_point, dtype=np.float64)
        if self.count == 1:
            return np.zeros(m_at_point.shape, dtype=np.int64)
        v = self.w2 * (1.0 - m_at_point)
        t = (v - self.lo) / self.delta + 0.5
        k = np.floor(t).astype(np.int64)
        return np.clip(k, 0, self.count - 1)

    def kappa(self, k: np.ndarray) -> np.ndarray:
        return np.sqrt(self.lo + np.asarray(k, dtype=np.float64) * self.delta)
