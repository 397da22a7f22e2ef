"""The dense Lippmann-Schwinger operator (oracle; test infrastructure only).

Paper, Sec. 2.1, eq. LS_d and its compact form eq. LS_d_c:
    u_i + omega^2 sum_{j in I} k_{i-j} m_j u_j = g_i,   i in I,
    g_i = -omega^2 sum_{j in I} k_{i-j} m_j [u_I]_j.
The rows are Toeplitz, so K is applied by a zero-padded FFT (Sec. 2.1, the
remark that the uniform grid allows the convolution to be evaluated by FFT).
"""
from __future__ import annotations

import numpy as np
import scipy.fft as sfft

from .green import green_table, wrapped_table


class DenseOperator:
    """A = I + omega^2 K M on the interior grid [n]^d (eq. LS_d_c)."""

    def __init__(self, d: int, n: int, omega: float, m: np.ndarray, workers: int = 1):
        self.d, self.n, self.omega = d, n, float(omega)
        self.m = np.asarray(m, dtype=np.float64)
        assert self.m.shape == (n,) * d
        self.table = green_table(d, n, omega)
        self.P = 2 * (n + 1)
        self.workers = workers
        self.khat = sfft.fftn(wrapped_table(self.table, n, d), workers=workers)

    def apply_K(self, x: np.ndarray) -> np.ndarray:
        """(K x)_i = sum_j k_{i-j} x_j over the interior, by zero-padded FFT."""
        n, d, P = self.n, self.d, self.P
        pad = np.zeros((P,) * d, dtype=np.complex128)
        pad[(slice(0, n),) * d] = x
        y = sfft.ifftn(self.khat * sfft.fftn(pad, workers=self.workers), workers=self.workers)
        return y[(slice(0, n),) * d]

    def apply_A(self, u: np.ndarray) -> np.ndarray:
        """(I + omega^2 K M) u."""
        return u + self.omega ** 2 * self.apply_K(self.m * u)

    def rhs_incident(self, u_inc: np.ndarray) -> np.ndarray:
        """g = -omega^2 K (m u_I) (eq. LS_d)."""
        return -self.omega ** 2 * self.apply_K(self.m * u_inc)


def brute_force_K(table: np.ndarray, n: int, d: int, x: np.ndarray) -> np.ndarray:
    """Direct O(N^2) evaluation of sum_j k_{i-j} x_j: the definition itself."""
    idx = np.indices((n,) * d).reshape(d, -1).T          # [N, d] array indices
    diff = idx[:, None, :] - idx[None, :, :] + (n + 1)    # offsets into the table
    K = table[tuple(diff[..., a] for a in range(d))]
    return (K @ x.reshape(-1)).reshape((n,) * d)


def brute_force_K_at(table: np.ndarray, n: int, d: int, x: np.ndarray, points: np.ndarray) -> np.ndarray:
    """sum_j k_{i-j} x_j at the output points i (array indices, [npoints, d]) by
    direct summation over all j: the definition, one output at a time, for
    checking sampled outputs on grids too large for the full O(N^2) product."""
    out = np.empty(len(points), dtype=np.complex128)
    for p, i in enumerate(points):
        # i - j + (n + 1) runs over [i + 2, i + n + 1] as j runs over n-1..0
        sl = tuple(slice(i[a] + 2, i[a] + n + 2) for a in range(d))
        block = table[sl][(slice(None, None, -1),) * d]
        out[p] = np.sum(block * x)
    return out


def dense_A(table: np.ndarray, n: int, d: int, omega: float, m: np.ndarray) -> np.ndarray:
    """The explicit dense matrix I + omega^2 K M (small n only)."""
    idx = np.indices((n,) * d).reshape(d, -1).T
    diff = idx[:, None, :] - idx[None, :, :] + (n + 1)
    K = table[tuple(diff[..., a] for a in range(d))]
    return np.eye(n ** d, dtype=np.complex128) + omega ** 2 * K * m.reshape(-1)[None, :]
