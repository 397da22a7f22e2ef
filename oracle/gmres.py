"""Restarted GMRES with right preconditioning (oracle; test infrastructure only).

The paper pairs its preconditioner with "standard GMRES" at relative
tolerance 1e-6 (Sec. 2.5). Reading G11: right preconditioning in the flexible
form (the preconditioned directions z_j = P v_j are stored and the iterate is
x = x0 + Z y), x0 = 0, tolerance relative to ||g||_2, modified Gram-Schmidt
Arnoldi, complex Givens rotations in the LAPACK zlartg convention. A cycle
ends when the residual estimate meets the tolerance, on breakdown, or after
``restart`` steps; the true residual g - A x then decides whether to stop or
restart from it. The iteration count is the number of Arnoldi steps over all
cycles.
"""
from __future__ import annotations

import dataclasses
from typing import Callable

import numpy as np


@dataclasses.dataclass
class GmresResult:
    x: np.ndarray
    iterations: int
    converged: bool
    rel_residual: float                 # true ||g - A x|| / ||g||
    estimates: list                     # residual estimate after every step, relative


def givens(f: complex, g: complex):
    """(c, s, r) with [c s; -conj(s) c] [f; g] = [r; 0] (zlartg convention)."""
    if g == 0:
        return 1.0, 0.0 + 0.0j, f
    if f == 0:
        return 0.0, np.conj(g) / abs(g), abs(g)
    af, ag = abs(f), abs(g)
    rho = np.hypot(af, ag)
    c = af / rho
    s = (f / af) * np.conj(g) / rho
    return c, s, (f / af) * rho


def fgmres(apply_A: Callable, apply_P: Callable, g: np.ndarray, tol: float,
           restart: int = 30, max_iters: int = 1000) -> GmresResult:
    shape = g.shape
    g = g.reshape(-1)
    beta0 = float(np.linalg.norm(g))
    x = np.zeros_like(g)
    if beta0 == 0.0:
        return GmresResult(x.reshape(shape), 0, True, 0.0, [])
    iters = 0
    estimates = []
    r = g.copy()
    while True:
        beta = float(np.linalg.norm(r))
        V = [r / beta]
        Z = []
        H = np.zeros((restart + 1, restart), dtype=np.complex128)
        cs = np.zeros(restart)
        sn = np.zeros(restart, dtype=np.complex128)
        s = np.zeros(restart + 1, dtype=np.complex128)
        s[0] = beta
        j_end = 0
        for j in range(restart):
            z = apply_P(V[j].reshape(shape)).reshape(-1)
            Z.append(z)
            w = apply_A(z.reshape(shape)).reshape(-1)
            for k in range(j + 1):                       # modified Gram-Schmidt
                H[k, j] = np.vdot(V[k], w)
                w = w - H[k, j] * V[k]
            H[j + 1, j] = np.linalg.norm(w)
            for k in range(j):                           # previous rotations
                a, bb = H[k, j], H[k + 1, j]
                H[k, j] = cs[k] * a + sn[k] * bb
                H[k + 1, j] = -np.conj(sn[k]) * a + cs[k] * bb
            c, sgn, rr = givens(H[j, j], H[j + 1, j])
            cs[j], sn[j] = c, sgn
            H[j, j] = rr
            hnext = H[j + 1, j]
            H[j + 1, j] = 0.0
            s[j + 1] = -np.conj(sgn) * s[j]
            s[j] = c * s[j]
            iters += 1
            j_end = j + 1
            estimates.append(abs(s[j + 1]) / beta0)
            if abs(s[j + 1]) <= tol * beta0 or iters >= max_iters:
                break
            # breakdown: w is (numerically) zero, the Krylov space is invariant
            wn = float(np.linalg.norm(w))
            if wn == 0.0:
                break
            V.append(w / wn)
            del hnext
        y = np.zeros(j_end, dtype=np.complex128)
        for i in range(j_end - 1, -1, -1):               # back substitution
            y[i] = (s[i] - H[i, i + 1:j_end] @ y[i + 1:j_end]) / H[i, i]
        for i in range(j_end):
            x = x + y[i] * Z[i]
        r = g - apply_A(x.reshape(shape)).reshape(-1)
        rel = float(np.linalg.norm(r)) / beta0
        if rel <= tol:
            return GmresResult(x.reshape(shape), iters, True, rel, estimates)
        if iters >= max_iters:
            return GmresResult(x.reshape(shape), iters, False, rel, estimates)


@dataclasses.dataclass
class BlockGmresResult:
    x: np.ndarray                       # [B][shape]
    iterations: int                     # block Arnoldi steps over all cycles
    converged: bool
    rel_residuals: np.ndarray           # true ||g_c - A x_c|| / ||g_c|| per column
    estimates: list                     # largest column residual estimate after every step
    col_iterations: np.ndarray          # block steps taken while column c was in the block


def block_fgmres(apply_A: Callable, apply_P: Callable, G: np.ndarray, tol: float, restart: int = 10,
                 max_iters: int = 200) -> BlockGmresResult:
    """Block flexible GMRES with right preconditioning: one shared block
    Krylov space for a batch of right-hand sides (a batch of the problem of
    Sec. 2.5; reading G20). The block holds the columns not yet converged
    (zero right-hand sides never enter it: x = 0). Cycle: R = G - A X over the
    block's columns, R = V_0 S (QR), then per step the block Arnoldi step
    Z_j = P V_j (each column), W = A Z_j, two passes of block Gram-Schmidt
    against V_0..V_j (H_ij = V_i^H W), W = V_{j+1} H_{j+1,j} (QR); Y minimises
    ||E S - Hbar Y||_F column by column (E the first block of the identity)
    and X = X + [Z_0 .. Z_j] Y at the cycle's end. The cycle ends when every
    column's residual estimate meets tol ||g_c|| (or after ``restart`` steps);
    the true residuals then decide which columns stay in the block for the
    next cycle."""
    B = G.shape[0]
    shape = G.shape[1:]
    Gm = G.reshape(B, -1).T.astype(np.complex128)            # N x B
    gn = np.linalg.norm(Gm, axis=0)
    X = np.zeros_like(Gm)
    rel = np.zeros(B)
    col_its = np.zeros(B, dtype=int)
    act = np.nonzero(gn > 0.0)[0]
    if act.size == 0:
        return BlockGmresResult(X.T.reshape(G.shape), 0, True, rel, [], col_its)
    cols = lambda f, M: np.stack([f(M[:, c].reshape(shape)).reshape(-1) for c in range(M.shape[1])], axis=1)
    its = 0
    estimates = []
    R = Gm[:, act].copy()
    while True:
        b = act.size
        V0, S = np.linalg.qr(R)
        V, Z = [V0], []
        Hbar = np.zeros(((restart + 1) * b, restart * b), dtype=np.complex128)
        E = np.zeros(((restart + 1) * b, b), dtype=np.complex128)
        E[:b] = S
        Y = None
        for j in range(restart):
            Zj = cols(apply_P, V[j])
            Z.append(Zj)
            W = cols(apply_A, Zj)
            for _ in range(2):                                   # block Gram-Schmidt, twice
                for i in range(j + 1):
                    Hij = V[i].conj().T @ W
                    Hbar[i * b:(i + 1) * b, j * b:(j + 1) * b] += Hij
                    W = W - V[i] @ Hij
            Vn, Rn = np.linalg.qr(W)
            Hbar[(j + 1) * b:(j + 2) * b, j * b:(j + 1) * b] = Rn
            V.append(Vn)
            its += 1
            col_its[act] += 1
            k = (j + 1) * b
            Y = np.linalg.lstsq(Hbar[:k + b, :k], E[:k + b], rcond=None)[0]
            est = np.linalg.norm(E[:k + b] - Hbar[:k + b, :k] @ Y, axis=0) / gn[act]
            estimates.append(float(est.max()))
            if est.max() <= tol or its >= max_iters:
                break
        X[:, act] = X[:, act] + np.concatenate(Z, axis=1) @ Y
        Ra = Gm[:, act] - cols(apply_A, X[:, act])
        rel[act] = np.linalg.norm(Ra, axis=0) / gn[act]
        if rel.max() <= tol:
            return BlockGmresResult(X.T.reshape(G.shape), its, True, rel, estimates, col_its)
        if its >= max_iters:
            return BlockGmresResult(X.T.reshape(G.shape), its, False, rel, estimates, col_its)
        keep = rel[act] > tol
        act, R = act[keep], Ra[:, keep]
