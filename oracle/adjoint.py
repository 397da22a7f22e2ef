"""Gradient of a receiver misfit with respect to m (oracle; test infrastructure only).

The paper has no adjoint; this is derived from eq. LS_d_c. With
A(m) = I + omega^2 K M and psi = u + u_I one has A psi = u_I, so
delta u = -A^{-1} omega^2 K diag(delta m) psi. For J = 1/2 sum_j |R u_j - d_j|^2
and r_j = R^T (R u_j - d_j), K = K^T (k depends on |delta| only) gives
    dJ/dm = -omega^2 Re sum_j psi_j * nu_j,   A nu_j = K conj(r_j),
i.e. one more solve with the same A and preconditioner, one K product and a
pointwise product. The gradient is taken with respect to the grid vector m
(not the L^2 gradient; divide by h^d for that). When the right-hand side g is
given directly and held fixed, psi_j = u_j.
"""
from __future__ import annotations

from typing import Callable

import numpy as np


def misfit_gradient(op, solve: Callable, u: np.ndarray, resid: np.ndarray,
                    u_inc: np.ndarray | None = None) -> np.ndarray:
    """op: DenseOperator; solve(b) -> A^{-1} b; u, resid (r_j), u_inc: [k][n]^d."""
    grad = np.zeros(op.m.shape)
    for j in range(u.shape[0]):
        psi = u[j] if u_inc is None else u[j] + u_inc[j]
        nu = solve(op.apply_K(np.conj(resid[j])))
        grad += np.real(psi * nu)
    return -op.omega ** 2 * grad
