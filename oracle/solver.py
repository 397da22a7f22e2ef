"""End-to-end oracle solve (test infrastructure only).

Setup follows Algorithm 1 (stencils alpha, beta; PML stencils gamma for the
global PML and the sampled local frequencies; slices; one exact sparse LU
per subproblem), the solve is right-preconditioned GMRES on eq. LS_d_c with
the preconditioner of Algorithm 2.
"""
from __future__ import annotations

import numpy as np

from .lsop import DenseOperator
from .stencils import alpha_beta
from .sparse import SparseSystem, Sweep
from .gmres import fgmres, GmresResult, block_fgmres
from .adjoint import misfit_gradient

#: PML strength C (reading G2: the paper only says C = Theta(1)).
DEFAULT_PML_C = 10.0


class OracleSolver:
    def __init__(self, d: int, n: int, omega: float, m: np.ndarray, pml_width: int = 12,
                 layer_thickness: int = 4, pml_C: float = DEFAULT_PML_C, restart: int = 30,
                 exact_sweep: bool = False, workers: int = 1, stencils=None, fronts: int = 1):
        self.d, self.n, self.omega = d, n, float(omega)
        self.m = np.asarray(m, dtype=np.float64)
        self.restart = restart
        self.op = DenseOperator(d, n, omega, self.m, workers=workers)
        if stencils is None:
            alpha, beta, sv = alpha_beta(self.op.table, n, d)
        else:
            alpha, beta, sv = stencils
        self.alpha, self.beta, self.alpha_sv = alpha, beta, sv
        self.system = SparseSystem(d, n, omega, self.m, alpha, beta, pml_width, pml_C)
        self.sweep = Sweep(self.system, layer_thickness, self.m, exact=exact_sweep, fronts=fronts)

    def precondition(self, r: np.ndarray) -> np.ndarray:
        return self.sweep.apply(r)

    def solve_rhs(self, g: np.ndarray, tol: float = 1e-6, max_iters: int = 1000) -> GmresResult:
        return fgmres(self.op.apply_A, self.precondition, g, tol, self.restart, max_iters)

    def solve_block(self, G: np.ndarray, tol: float = 1e-6, restart: int = 10, max_iters: int = 200):
        """All right-hand sides G [B][n]^d in one shared block Krylov space."""
        return block_fgmres(self.op.apply_A, self.precondition, G, tol, restart, max_iters)

    def solve_incident(self, u_inc: np.ndarray, tol: float = 1e-6, max_iters: int = 1000):
        """Scattered fields for a batch of incident waves [k][n]^d."""
        out = []
        for j in range(u_inc.shape[0]):
            out.append(self.solve_rhs(self.op.rhs_incident(u_inc[j]), tol, max_iters))
        return out

    def gradient(self, u: np.ndarray, resid: np.ndarray, u_inc=None, tol: float = 1e-12):
        solve = lambda b: self.solve_rhs(b, tol).x
        return misfit_gradient(self.op, solve, u, resid, u_inc)
