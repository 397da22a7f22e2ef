"""CPU oracle for the sparsify-and-sweep preconditioned GMRES solve of the
discretized Lippmann-Schwinger equation (Liu & Ying, "Sparsify and sweep: an
efficient preconditioner for the Lippmann-Schwinger equation").

TEST INFRASTRUCTURE ONLY. This package is a plain, slow, float64 restatement
of what the paper defines, written to check the GPU library against. Only the
test-suite, the smoke check and the CPU-baseline leg of the benchmark may
import it; the library never does, and this package imports nothing from the
library. The two share no code: only the seeded input generators in
``workloads`` serve both.

Each function cites the passage of the paper it follows (section, equation or
algorithm). Where the paper is silent or garbled the oracle takes one
documented reading; every such reading carries a tag G1..G17 in the
docstring that implements it.

Modules
-------
green     Green's function table, central weight, FFT spectrum (Sec. 2.1)
lsop      the dense operator I + omega^2 K M and its right-hand side (eq. LS_d_c)
stencils  alpha, beta (eqs. alpha, beta), PML stretch and gamma (eq. gamma),
          local-frequency samples (Sec. 2.3)
sparse    the sparse system H u = f (eq. Huf), slices, moving-PML subproblems
          (eq. Hwv_approx) and the sweep (Algorithms 1 and 2)
gmres     right-preconditioned restarted (flexible) GMRES
adjoint   gradient of a receiver misfit with respect to m
solver    end-to-end driver tying the above together
direct    the sparsifying stencils as a direct Helmholtz scheme, QSFEM, and
          the phase error against the Green's function (Sec. 4)
"""
from .green import green, central_weight, green_table, wrapped_table
from .lsop import DenseOperator, brute_force_K, brute_force_K_at, dense_A
from .stencils import (neighbourhood, plane_wave_directions, normalise_phase,
                       alpha_beta, sigma_global, pml_stencil, FrequencySamples)
from .sparse import SparseSystem, Sweep
from .gmres import fgmres, GmresResult, block_fgmres, BlockGmresResult
from .adjoint import misfit_gradient
from .solver import OracleSolver, DEFAULT_PML_C

__all__ = [
    "green", "central_weight", "green_table", "wrapped_table",
    "DenseOperator", "brute_force_K", "dense_A",
    "neighbourhood", "plane_wave_directions", "normalise_phase", "alpha_beta",
    "sigma_global", "pml_stencil", "FrequencySamples",
    "SparseSystem", "Sweep", "fgmres", "GmresResult", "block_fgmres", "BlockGmresResult", "misfit_gradient",
    "OracleSolver", "DEFAULT_PML_C", "brute_force_K_at",
]
