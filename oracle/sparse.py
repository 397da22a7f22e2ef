"""Sparsified system and moving-PML sweep (oracle; test infrastructure only).

Sparse system H u~ = f on the PML-extended grid (Sec. 2.2.3, eqs. sp_stc and
Huf): rows i in I^h = [0, n+1]^d use the type-1 stencil
    alpha^* u~_{mu_i} + omega^2 beta^* [m u~]_{mu_i} = alpha^* g_{mu_i},
rows in I^{h+eta} minus I^h = [-b, n+1+b]^d minus I^h use the type-2
stencil gamma_i^* u~_{mu_i} = 0, and u~ vanishes on the Dirichlet ring.

Sweep (Sec. 2.3, eq. Hwv_approx, Algorithms 1 and 2): the extended grid is cut
into slices D_1..D_l along x1; the approximate Schur-complement inverse of
slice i is the D_i part of the solution of a subproblem on (auxiliary PML
left of D_i) union D_i, with zero right-hand side on the auxiliary part.

Extended-grid arrays are flat C-order [L]^d with L = n + 2 + 2b and array
index e = i + b; axis 0 is x1, so a slice is a contiguous range.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .stencils import (neighbourhood, plane_wave_directions, pml_stencil,
                       sigma_global, sigma_aux, sigma_aux_right, FrequencySamples)


def axis_class(i: np.ndarray, n: int, b: int) -> np.ndarray:
    """Per-axis stretch class of grid index i: 0 where the three sigma values
    around i vanish (i in [0, n+1]), 1..b for i = -b..-1 and b+1..2b for
    i = n+2..n+1+b. Points with equal classes get equal stencils (the
    translation invariance noted in Sec. 2.2.2)."""
    i = np.asarray(i)
    c = np.zeros(i.shape, dtype=np.int64)
    c = np.where(i < 0, i + b + 1, c)
    c = np.where(i > n + 1, i - (n + 2) + b + 1, c)
    return c


def class_index(c: int, n: int, b: int) -> int:
    """A representative grid index of per-axis class c."""
    if c == 0:
        return 0
    if c <= b:
        return c - 1 - b
    return n + 2 + (c - b - 1)


class SparseSystem:
    """H and Q on the extended grid (Sec. 2.2.3)."""

    def __init__(self, d, n, omega, m, alpha, beta, b, C):
        self.d, self.n, self.omega, self.b, self.C = d, n, float(omega), b, float(C)
        self.h = 1.0 / (n + 1)
        self.L = L = n + 2 + 2 * b
        self.alpha, self.beta = alpha, beta
        self.dirs = plane_wave_directions(d)
        mu = neighbourhood(d)
        self.mu = mu
        shape = (L,) * d
        gi = np.indices(shape).reshape(d, -1).T - b          # grid index i of each point
        self.gi = gi
        self.npts = len(gi)
        inner = np.all((gi >= 1) & (gi <= n), axis=1)       # I
        self.inner = inner
        type1 = np.all((gi >= 0) & (gi <= n + 1), axis=1)   # I^h
        self.type1 = type1
        m_ext = np.zeros(self.npts)
        m_ext[inner] = np.asarray(m, dtype=np.float64).reshape(-1)
        self.m_ext = m_ext
        # gamma for every PML point, through the per-axis class key
        cls = axis_class(gi, n, b)
        gam = np.zeros((self.npts, len(mu)), dtype=np.complex128)
        keys = {}
        for p in np.nonzero(~type1)[0]:
            key = tuple(cls[p])
            g = keys.get(key)
            if g is None:
                g = self._global_gamma(key)
                keys[key] = g
            gam[p] = g
        self.gamma_by_class = keys
        self.gamma = gam
        rows, cols, vals = [], [], []
        for o, off in enumerate(mu):
            nb = gi + off
            ok = np.all((nb >= -b) & (nb <= n + 1 + b), axis=1)
            nbf = np.ravel_multi_index(tuple((nb[ok] + b).T), shape)
            p = np.nonzero(ok)[0]
            v1 = np.conj(alpha[o]) + self.omega ** 2 * np.conj(beta[o]) * m_ext[nbf]
            v2 = np.conj(gam[p, o])
            rows.append(p)
            cols.append(nbf)
            vals.append(np.where(type1[p], v1, v2))
        self.H = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                               shape=(self.npts, self.npts))

    def _global_gamma(self, key) -> np.ndarray:
        n, b, C, w = self.n, self.b, self.C, self.omega
        sig = np.zeros((self.d, 3))
        for k, c in enumerate(key):
            i = class_index(c, n, b)
            sig[k] = sigma_global(np.array([i - 1, i, i + 1]), n, b, C, w)
        return pml_stencil(w, self.h, sig, self.dirs)

    def extend(self, r: np.ndarray) -> np.ndarray:
        """Zero-extend an interior array [n]^d to the flat extended grid."""
        x = np.zeros(self.npts, dtype=np.complex128)
        x[self.inner] = np.asarray(r).reshape(-1)
        return x

    def restrict(self, x: np.ndarray) -> np.ndarray:
        return x[self.inner].reshape((self.n,) * self.d)

    def apply_Q(self, r: np.ndarray) -> np.ndarray:
        """f_i = alpha^* r_{mu_i} on I^h, 0 on the PML (eq. Huf)."""
        L, b, d, n = self.L, self.b, self.d, self.n
        x = self.extend(r).reshape((L,) * d)
        f = np.zeros_like(x)
        core = tuple(slice(b, b + n + 2) for _ in range(d))   # I^h
        for o, off in enumerate(self.mu):
            src = tuple(slice(b + off[k], b + n + 2 + off[k]) for k in range(d))
            f[core] += np.conj(self.alpha[o]) * x[src]
        return f.reshape(-1)

    def apply_H(self, u: np.ndarray) -> np.ndarray:
        return self.H @ u


def slice_partition(n: int, b: int, w: int, fronts: int = 1):
    """Slices of the extended grid along x1, in grid order, as (lo, hi) line
    ranges, and the order in which they are eliminated.

    One front (Algorithms 1 and 2; reading G8): l = floor((n+2)/w) slices
    (at least 1), D_1 = [-b, w-1], D_k = [(k-1)w, kw-1], the last slice
    D_l = [(l-1)w, n+1+b] absorbs the remainder; eliminated left to right.

    Two fronts (the first remark after Algorithm 2, Sec. 2.4; reading G18):
    p = floor((n+1)/(2w)) slices of w lines from each end, the outermost of
    each front also holding the b PML lines of its side, and one middle slice
    of the remaining n+2-2pw lines (1..2w); the left front is eliminated left
    to right, the right front right to left, the middle slice last. With
    p = 0 the single slice is the whole extended grid."""
    if fronts == 1:
        nl = max(1, (n + 2) // w)
        bounds = []
        for k in range(nl):
            lo = -b if k == 0 else k * w
            hi = n + 1 + b if k == nl - 1 else (k + 1) * w - 1
            bounds.append((lo, hi))
        return bounds, list(range(nl))
    if fronts != 2:
        raise ValueError("fronts must be 1 or 2")
    p = (n + 1) // (2 * w)
    if p == 0:
        return [(-b, n + 1 + b)], [0]
    left = [(-b if k == 0 else k * w, (k + 1) * w - 1) for k in range(p)]
    right = [(n + 2 - (k + 1) * w, n + 1 + b if k == 0 else n + 1 - k * w) for k in range(p)]
    bounds = left + [(p * w, n + 1 - p * w)] + right[::-1]
    order = list(range(p)) + [2 * p - k for k in range(p)] + [p]
    return bounds, order


class Sweep:
    """Moving-PML sweeping preconditioner (Sec. 2.3; Algorithms 1 and 2).

    The extended grid is cut into slices along x1 (slice_partition) and the
    slices are eliminated in an order: the sparse system H, block tridiagonal
    in the slices, is factored block by block, with the exact Schur-complement
    inverse of each slice replaced by the approximation T~ of eq. Hwv_approx:
    the D part of the solution of a subproblem on D plus b auxiliary PML lines
    on each side whose neighbouring slice was eliminated before it (left of
    D_k for the one-front sweep; right of D_k for the right front of the
    two-front sweep; both sides for its middle slice), zero right-hand side on
    the auxiliary lines. Auxiliary lines are stretched in x1 by the moved
    profile and in the other axes by the global one, with stencils built from
    the sampled local frequency at each point (Sec. 2.3; G9, G10). The apply
    is the block forward and backward substitution of that factorization
    (sweep()). ``exact=True`` replaces every subproblem by H on the slice and
    every slice connected to it through slices eliminated earlier (its exact
    Schur-complement inverse), for checking the bookkeeping."""

    def __init__(self, system: SparseSystem, w: int, m: np.ndarray, exact: bool = False,
                 samples: FrequencySamples | None = None, only: list | None = None, fronts: int = 1):
        """only: factor just these slices (for checking single slice solves on
        large grids); sweep() and apply() then refuse to run."""
        s = system
        self.s = s
        d, n, b, L = s.d, s.n, s.b, s.L
        self.T = L ** (d - 1)
        self.fronts = fronts
        self.bounds, self.order = slice_partition(n, b, w, fronts)
        nl = len(self.bounds)
        self.nslices = nl
        self.pos = [0] * nl
        for i, k in enumerate(self.order):
            self.pos[k] = i
        self.samples = samples if samples is not None else FrequencySamples(np.asarray(m), s.omega, n)
        self.exact = exact
        self.lu = [None] * nl
        self.aux_count = [0] * nl          # auxiliary unknowns left of D_k
        self.aux_count_right = [0] * nl    # auxiliary unknowns right of D_k
        self.aux_gamma = {}                # left auxiliary stencils by (q, classes, sample)
        self.aux_gamma_right = {}          # right auxiliary stencils by (q, classes, sample)
        self.complete = only is None
        for k in (range(nl) if only is None else only):
            A, naux, nauxr = self._subproblem(k)
            self.aux_count[k] = naux
            self.aux_count_right[k] = nauxr
            self.lu[k] = spla.splu(A.tocsc())
        # couplings H_[k,k-1] and H_[k,k+1]
        self.Hm, self.Hp = [None] * nl, [None] * nl
        for k in range(nl):
            rk = self.points(k)
            if k > 0:
                self.Hm[k] = s.H[rk][:, self.points(k - 1)]
            if k < nl - 1:
                self.Hp[k] = s.H[rk][:, self.points(k + 1)]

    def points(self, k: int) -> np.ndarray:
        lo, hi = self.bounds[k]
        b = self.s.b
        return np.arange((lo + b) * self.T, (hi + b + 1) * self.T)

    def earlier(self, k: int):
        """Neighbouring slices eliminated before slice k."""
        return [j for j in (k - 1, k + 1) if 0 <= j < self.nslices and self.pos[j] < self.pos[k]]

    def later(self, k: int):
        """Neighbouring slices eliminated after slice k."""
        return [j for j in (k - 1, k + 1) if 0 <= j < self.nslices and self.pos[j] > self.pos[k]]

    def subproblem_lines(self, k: int):
        """(first, last) grid lines of slice k's subproblem."""
        lo, hi = self.bounds[k]
        first, last = lo, hi
        if self.exact:
            j = k - 1
            while j >= 0 and self.pos[j] < self.pos[k]:
                first = self.bounds[j][0]
                j -= 1
            j = k + 1
            while j < self.nslices and self.pos[j] < self.pos[k]:
                last = self.bounds[j][1]
                j += 1
        else:
            if k - 1 in self.earlier(k):
                first = lo - self.s.b
            if k + 1 in self.earlier(k):
                last = hi + self.s.b
        return first, last

    def _subproblem(self, k: int):
        s = self.s
        b, T = s.b, self.T
        lo, hi = self.bounds[k]
        first, last = self.subproblem_lines(k)
        base = (first + b) * T
        nloc = (last - first + 1) * T
        naux = (lo - first) * T
        nauxr = (last - hi) * T
        if self.exact:
            return s.H[base:base + nloc][:, base:base + nloc].tocoo(), naux, nauxr
        # rows of D_k come from H, restricted to the subproblem's lines
        Hsub = s.H[(lo + b) * T:(hi + b + 1) * T][:, base:base + nloc].tocoo()
        rows = [Hsub.row + naux]
        cols = [Hsub.col]
        vals = [Hsub.data]
        if naux:
            r, c, v = self._aux_rows(k, first, last, "left")
            rows.append(r)
            cols.append(c)
            vals.append(v)
        if nauxr:
            r, c, v = self._aux_rows(k, first, last, "right")
            rows.append(r)
            cols.append(c)
            vals.append(v)
        A = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                          shape=(nloc, nloc))
        return A, naux, nauxr

    def _aux_rows(self, k, first, last, side):
        """gamma rows of the auxiliary PML of slice k on one side (eq.
        Hwv_approx, the auxiliary block), in the subproblem's numbering."""
        s = self.s
        d, n, b, L, T = s.d, s.n, s.b, s.L, self.T
        lo, hi = self.bounds[k]
        mu = s.mu
        tshape = (L,) * (d - 1)
        tgi = np.indices(tshape).reshape(d - 1, -1).T - b if d > 1 else np.zeros((1, 0), int)
        tcls = axis_class(tgi, n, b)
        lines = range(first, lo) if side == "left" else range(hi + 1, last + 1)
        table = self.aux_gamma if side == "left" else self.aux_gamma_right
        rows, cols, vals = [], [], []
        for line in lines:
            a = line - first                   # local line
            q = lo - 1 - line if side == "left" else line - hi - 1   # depth into the auxiliary PML
            pts = (line + b) * T + np.arange(T)
            kstar = self.samples.index(s.m_ext[pts])
            gam = np.empty((T, len(mu)), dtype=np.complex128)
            for t in range(T):
                key = (q,) + tuple(tcls[t]) + (int(kstar[t]),)
                g = table.get(key)
                if g is None:
                    g = self._aux_gamma(q, tcls[t], int(kstar[t]), lo, hi, side)
                    table[key] = g
                gam[t] = g
            for o, off in enumerate(mu):
                nl_ = a + off[0]
                if nl_ < 0 or nl_ > last - first:
                    continue                   # the Dirichlet line beyond the auxiliary PML
                nt = tgi + off[1:]
                ok = np.all((nt >= -b) & (nt <= n + 1 + b), axis=1)
                tflat = np.ravel_multi_index(tuple((nt[ok] + b).T), tshape) if d > 1 else np.zeros(ok.sum(), int)
                t_ok = np.nonzero(ok)[0]
                rows.append(a * T + t_ok)
                cols.append(nl_ * T + tflat)
                vals.append(np.conj(gam[t_ok, o]))
        return np.concatenate(rows), np.concatenate(cols), np.concatenate(vals)

    def _aux_gamma(self, q, tcls, kstar, lo, hi, side):
        s = self.s
        n, b, C, w = s.n, s.b, s.C, s.omega
        sig = np.zeros((s.d, 3))
        if side == "left":
            line = lo - 1 - q
            sig[0] = sigma_aux(np.array([line - 1, line, line + 1]), lo, b, C, w)
        else:
            line = hi + 1 + q
            sig[0] = sigma_aux_right(np.array([line - 1, line, line + 1]), hi, b, C, w)
        for k, c in enumerate(tcls):
            i = class_index(int(c), n, b)
            sig[k + 1] = sigma_global(np.array([i - 1, i, i + 1]), n, b, C, w)
        kappa = float(self.samples.kappa(kstar))
        return pml_stencil(kappa, s.h, sig, s.dirs)

    def solve_slice(self, k: int, v: np.ndarray) -> np.ndarray:
        """T~_k v: pad v with zeros on the auxiliary lines, solve, restrict to D_k."""
        naux, nauxr = self.aux_count[k], self.aux_count_right[k]
        rhs = np.zeros(naux + len(v) + nauxr, dtype=np.complex128)
        rhs[naux:naux + len(v)] = v
        return self.lu[k].solve(rhs)[naux:naux + len(v)]

    def coupling(self, k: int, j: int):
        """H_[k,j] for a neighbouring slice j."""
        return self.Hm[k] if j == k - 1 else self.Hp[k]

    def sweep(self, f: np.ndarray) -> np.ndarray:
        """Algorithm 2, steps 3-8, as the block substitutions of the
        factorization above, on the flat extended grid: forward, slices in
        elimination order, u_k = T~_k (f_k - sum of H_[k,j] u_j over the
        neighbours j eliminated earlier); backward, in reverse order,
        u_k -= T~_k (sum of H_[k,j] u_j over the neighbours eliminated later)."""
        if not self.complete:
            raise RuntimeError("sweep needs every slice factored")
        u = np.zeros_like(f)
        for k in self.order:
            rhs = f[self.points(k)].copy()
            for j in self.earlier(k):
                rhs -= self.coupling(k, j) @ u[self.points(j)]
            u[self.points(k)] = self.solve_slice(k, rhs)
        for k in reversed(self.order):
            later = self.later(k)
            if later:
                corr = sum(self.coupling(k, j) @ u[self.points(j)] for j in later)
                u[self.points(k)] -= self.solve_slice(k, corr)
        return u

    def apply(self, r: np.ndarray) -> np.ndarray:
        """Algorithm 2: f = Q r, sweep, extract on the interior grid."""
        return self.s.restrict(self.sweep(self.s.apply_Q(r)))
