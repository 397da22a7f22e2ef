"""Pins for the oracle's two-front sweep (the first remark after Algorithm 2,
Sec. 2.4: sweep from both ends toward a middle slice, exchange there, then
sweep back; reading G18 for the partition).

* The slices partition the extended grid, mirror symmetrically, with a middle
  slice of 1..2w lines eliminated last.
* With exact Schur-complement inverses the two-front substitutions are block
  Gaussian elimination in that order, hence equal H^{-1} f.
* The left front's subproblems are the one-front sweep's first slices.
* The right front is the one-front sweep of the grid reversed along x1: each
  of its slice solves equals the reversed one-front solve on the reversed
  medium (its auxiliary PML, right of each slice, mirrors the left one).
* Every right auxiliary row (right front and middle slice) equals the
  conjugated null vector of the plane waves with the x1 stretch of Sec. 2.2.2
  moved to the slice's right edge, at the row's own sampled wavenumber.
* For a medium symmetric in x1 the two-front preconditioner commutes with the
  reflection (the one-front sweep does not).
* Preconditioned GMRES with it reaches the dense LU solution.
"""
import itertools
import math

import numpy as np
import pytest
import scipy.sparse.linalg as spla

import workloads
from oracle import (OracleSolver, SparseSystem, Sweep, alpha_beta, green_table, dense_A)
from oracle.sparse import slice_partition


def system_for(d, n, omega, m, b, C=10.0):
    alpha, beta, _ = alpha_beta(green_table(d, n, omega), n, d)
    return SparseSystem(d, n, omega, m, alpha, beta, b, C)


@pytest.mark.parametrize("n,b,w", [(23, 6, 4), (40, 6, 3), (63, 12, 4), (7, 3, 3), (5, 2, 4)])
def test_partition(n, b, w):
    bounds, order = slice_partition(n, b, w, fronts=2)
    lines = np.concatenate([np.arange(lo, hi + 1) for lo, hi in bounds])
    np.testing.assert_array_equal(lines, np.arange(-b, n + 2 + b))
    nl = len(bounds)
    assert sorted(order) == list(range(nl))
    if nl == 1:
        return
    p = (nl - 1) // 2
    assert nl == 2 * p + 1 and order[-1] == p
    mid = bounds[p][1] - bounds[p][0] + 1
    assert 1 <= mid <= 2 * w
    for k in range(nl):     # mirror symmetric about the centre line (n+1)/2
        lo, hi = bounds[k]
        lo2, hi2 = bounds[nl - 1 - k]
        assert (lo, hi) == (n + 1 - hi2, n + 1 - lo2)
    # each front is eliminated outward-in
    assert order[:p] == list(range(p)) and order[p:2 * p] == list(range(nl - 1, p, -1))


@pytest.mark.parametrize("n,w", [(23, 3), (23, 4), (31, 5)])
def test_exact_two_front_sweep_is_block_elimination(n, w):
    wl = workloads.workload("C0").scaled(n, ppw_omega=2.0)
    m = wl.medium_array()
    system = system_for(2, n, wl.omega, m, 6)
    sw = Sweep(system, w, m, exact=True, fronts=2)
    assert sw.nslices >= 5
    rng = np.random.default_rng(2)
    f = rng.standard_normal(system.npts) + 1j * rng.standard_normal(system.npts)
    ref = spla.spsolve(system.H.tocsc(), f)
    assert np.linalg.norm(sw.sweep(f) - ref) <= 1e-11 * np.linalg.norm(ref)


def test_exact_two_front_sweep_is_block_elimination_3d():
    n = 9
    m = workloads.gaussian_bump_medium(n, 3, 3, (0.25, 0.75), (0.1, 0.2), (-0.3, 0.3), seed=4)
    system = system_for(3, n, 2 * math.pi, m, 3)
    sw = Sweep(system, 2, m, exact=True, fronts=2)
    assert sw.nslices == 5
    rng = np.random.default_rng(21)
    f = rng.standard_normal(system.npts) + 1j * rng.standard_normal(system.npts)
    ref = spla.spsolve(system.H.tocsc(), f)
    assert np.linalg.norm(sw.sweep(f) - ref) <= 1e-11 * np.linalg.norm(ref)


def _media(n):
    return workloads.gaussian_bump_medium(n, 2, 6, (0.2, 0.8), (0.04, 0.1), (-0.4, 0.4), seed=3)


def test_left_front_is_the_one_front_sweep():
    n, b, w = 40, 6, 3
    omega = 2 * math.pi * 2.5
    m = _media(n)
    system = system_for(2, n, omega, m, b)
    two = Sweep(system, w, m, fronts=2)
    one = Sweep(system, w, m)
    p = (two.nslices - 1) // 2
    rng = np.random.default_rng(5)
    for k in range(p):
        assert two.bounds[k] == one.bounds[k]
        assert two.aux_count[k] == one.aux_count[k] and two.aux_count_right[k] == 0
        v = rng.standard_normal(len(two.points(k))) + 1j
        a, c = two.solve_slice(k, v), one.solve_slice(k, v)
        assert np.linalg.norm(a - c) <= 1e-14 * np.linalg.norm(c)


@pytest.mark.parametrize("d", [2, 3])
def test_right_front_is_the_one_front_sweep_of_the_reversed_grid(d):
    if d == 2:
        n, b, w, omega = 40, 6, 3, 2 * math.pi * 2.5
        m = _media(n)
    else:
        n, b, w, omega = 9, 3, 2, 2 * math.pi
        m = workloads.gaussian_bump_medium(n, 3, 3, (0.25, 0.75), (0.1, 0.2), (-0.3, 0.3), seed=4)
    mr = m[::-1].copy()
    two = Sweep(system_for(d, n, omega, m, b), w, m, fronts=2)
    sysr = system_for(d, n, omega, mr, b)
    one_r = Sweep(sysr, w, mr)
    L = two.s.L
    nl = two.nslices
    p = (nl - 1) // 2
    rng = np.random.default_rng(6)
    for j in range(p):
        k = nl - 1 - j                    # right-front slice j (outermost first)
        lo, hi = two.bounds[k]
        assert (n + 1 - hi, n + 1 - lo) == one_r.bounds[j]
        assert two.aux_count_right[k] == one_r.aux_count[j] and two.aux_count[k] == 0
        lines = hi - lo + 1
        v = rng.standard_normal((lines,) + (L,) * (d - 1)) + 1j * rng.standard_normal((lines,) + (L,) * (d - 1))
        a = two.solve_slice(k, v.reshape(-1)).reshape(v.shape)
        c = one_r.solve_slice(j, v[::-1].reshape(-1)).reshape(v.shape)[::-1]
        err = np.linalg.norm(a - c) / np.linalg.norm(c)
        assert err <= 1e-12, (j, err)


def _sigma_moved_right(x, edge, h, b, C, omega):
    """The high-side profile of Sec. 2.2.2 moved so that it vanishes up to
    ``edge``: (C/omega)((x - edge)/eta)^2 for x > edge, eta = b h."""
    eta = b * h
    x = np.asarray(x, dtype=np.float64)
    return np.where(x > edge, (C / omega) * ((x - edge) / eta) ** 2, 0.0)


def _sigma_paper(x, h, b, C, omega):
    eta = b * h
    x = np.asarray(x, dtype=np.float64)
    out = np.zeros_like(x)
    lo, hi = x <= -h, x >= 1 + h
    out[lo] = -(C / omega) * ((x[lo] + h) / eta) ** 2
    out[hi] = (C / omega) * ((x[hi] - 1 - h) / eta) ** 2
    return out


def _null_stencil(kappa, h, centre, sig_axes, d):
    offs = np.array(list(itertools.product((-1, 0, 1), repeat=d)))
    dirs = np.array([v for v in itertools.product((-1, 0, 1), repeat=d) if any(v)], dtype=np.float64)
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    xs = np.zeros((len(offs), d), dtype=np.complex128)
    for k in range(d):
        idx = centre[k] + offs[:, k]
        xs[:, k] = idx * h + 1j * sig_axes[k](idx * h)
    F = np.exp(1j * kappa * (xs @ dirs.T))
    c0 = (len(offs) - 1) // 2
    _, s, Vh = np.linalg.svd((F / F[c0]).conj().T)
    g = np.conj(Vh[-1])
    g /= np.linalg.norm(g)
    g *= np.conj(g[c0]) / abs(g[c0])
    return g, F


def test_right_auxiliary_rows_follow_depth_and_local_wavenumber():
    n, b, w, omega, C = 23, 5, 3, 2 * math.pi * 2.5, 10.0
    m = workloads.gaussian_bump_medium(n, 2, 6, (0.2, 0.8), (0.05, 0.1), (-0.35, 0.35), seed=3)
    h = 1.0 / (n + 1)
    system = system_for(2, n, omega, m, b, C)
    sw = Sweep(system, w, m, fronts=2)
    L = system.L
    w2 = omega * omega
    lo_s, hi_s = w2 * (1 - m.max()), w2 * (1 - m.min())
    count = n
    m_ext = np.zeros((L, L))
    m_ext[b + 1:b + 1 + n, b + 1:b + 1 + n] = m
    glob = lambda x: _sigma_paper(x, h, b, C, omega)
    offs = list(itertools.product((-1, 0, 1), repeat=2))
    p = (sw.nslices - 1) // 2
    checked = 0
    for k in range(p, sw.nslices - 1):       # the middle slice and the right front's inner slices
        lo, hi = sw.bounds[k]
        first, last = sw.subproblem_lines(k)
        assert last == hi + b
        A, naux, nauxr = sw._subproblem(k)
        A = A.tocsr()
        assert nauxr == b * L and naux == (b * L if k == p else 0)
        moved = lambda x, edge=(hi + 1) * h: _sigma_moved_right(x, edge, h, b, C, omega)
        for line in range(hi + 1, last + 1):
            a = line - first
            for t in range(L):
                pt = (line, t - b)
                mv = m_ext[line + b, t]
                if count == 1:
                    ks = 0
                else:
                    delta = (hi_s - lo_s) / (count - 1)
                    ks = int(min(max(math.floor((w2 * (1 - mv) - lo_s) / delta + 0.5), 0), count - 1))
                kappa = math.sqrt(lo_s + ks * (hi_s - lo_s) / (count - 1))
                g, F = _null_stencil(kappa, h, pt, [moved, glob], 2)
                row = A.getrow(a * L + t)
                want = {}
                for o, (d1, d2) in enumerate(offs):
                    if line + d1 > last or not (-b <= pt[1] + d2 <= n + 1 + b):
                        continue
                    want[(line + d1 - first) * L + (pt[1] + d2 + b)] = np.conj(g[o])
                got = dict(zip(row.indices.tolist(), row.data.tolist()))
                assert set(got) == set(want), (k, line, t)
                assert max(abs(got[c] - want[c]) for c in want) <= 1e-12, (k, line, t)
                checked += 1
    assert checked >= 2 * b * L


def test_symmetric_medium_commutes_with_reflection():
    n, b, w = 31, 6, 4
    omega = 2 * math.pi * 2.0
    m = workloads.gaussian_bump_medium(n, 2, 4, (0.2, 0.8), (0.05, 0.1), (-0.3, 0.3), seed=9)
    m = 0.5 * (m + m[::-1])                  # symmetric in x1
    system = system_for(2, n, omega, m, b)
    two = Sweep(system, w, m, fronts=2)
    one = Sweep(system, w, m)
    rng = np.random.default_rng(3)
    r = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    z = two.apply(r)
    zr = two.apply(r[::-1].copy())[::-1]
    assert np.linalg.norm(z - zr) <= 1e-11 * np.linalg.norm(z)
    z1 = one.apply(r)
    z1r = one.apply(r[::-1].copy())[::-1]
    assert np.linalg.norm(z1 - z1r) > 1e-6 * np.linalg.norm(z1)


def test_two_front_preconditioned_solve_reaches_dense_solution():
    wl = workloads.workload("C0").scaled(31, ppw_omega=2.0)
    m = wl.medium_array()
    s = OracleSolver(2, wl.n, wl.omega, m, 8, 4, fronts=2)
    assert s.sweep.fronts == 2
    g = s.op.rhs_incident(wl.incident()[0])
    res = s.solve_rhs(g, 1e-10)
    ud = np.linalg.solve(dense_A(s.op.table, wl.n, 2, wl.omega, s.m), g.reshape(-1)).reshape(g.shape)
    assert res.converged and res.iterations <= 15
    assert np.linalg.norm(res.x - ud) <= 1e-8 * np.linalg.norm(ud)
