"""Pins for the oracle's moving-PML auxiliary stencils (Sec. 2.3, eq. Hwv_approx).

The auxiliary rows of slice k >= 2 are PML rows whose x1 stretch starts at the
left edge of D_k (the profile of Sec. 2.2.2, moved) and whose plane waves use
the local wavenumber sqrt(s_k*) of the point's frequency sample (Sec. 2.3),
not omega. These tests rebuild what each assembled row must be from the
paper's definitions, in coordinates and independently of the oracle's own
helpers:

* sigma(x) of Sec. 2.2.2 (global, and moved to the slice edge) written out in
  coordinates, checked against the oracle's index-form stretch values;
* with m = 0 the auxiliary stencil at depth q is the global PML stencil of the
  same depth (same stretch, same frequency);
* with m = m0 != 0 every stored auxiliary stencil annihilates
  exp(i omega sqrt(1 - m0) r . x^sigma) with x^sigma built here; omega in
  place of the local wavenumber fails this;
* for a variable medium every assembled auxiliary row of every subproblem
  equals the conjugated null vector of the modified plane waves at that
  row's own depth and sampled wavenumber (sample rule written out here), with
  the entries toward the Dirichlet line dropped and no other entries.
"""
import itertools
import math

import numpy as np
import pytest

import workloads
from oracle import SparseSystem, Sweep, alpha_beta, green_table
from oracle.stencils import sigma_aux, sigma_global


def sigma_paper(x, h, b, C, omega):
    """Sec. 2.2.2: sigma(x) = -(C/omega)((x + h)/eta)^2 left of -h,
    (C/omega)((x - 1 - h)/eta)^2 right of 1 + h, zero between; eta = b h.
    (The Dirichlet points take the formula's continuation, reading G3.)"""
    eta = b * h
    x = np.asarray(x, dtype=np.float64)
    out = np.zeros_like(x)
    lo = x <= -h
    hi = x >= 1 + h
    out[lo] = -(C / omega) * ((x[lo] + h) / eta) ** 2
    out[hi] = (C / omega) * ((x[hi] - 1 - h) / eta) ** 2
    return out


def sigma_moved(x, edge, h, b, C, omega):
    """The low-side profile of Sec. 2.2.2 moved so that it vanishes from
    ``edge`` on: -(C/omega)((x - edge)/eta)^2 for x < edge (Sec. 2.3: the
    auxiliary PML left of D_k; ``edge`` is the last auxiliary line, one
    line left of D_k's first line)."""
    eta = b * h
    x = np.asarray(x, dtype=np.float64)
    return np.where(x < edge, -(C / omega) * ((x - edge) / eta) ** 2, 0.0)


def null_stencil(kappa, h, centre, sig_axes, d):
    """Conjugated left null vector of F_{o,r} = exp(i kappa r . x^sigma(p+o))
    over the 3^d neighbourhood, r = v/|v| for the 3^d - 1 unit directions;
    unit 2-norm, centre real positive (reading G5)."""
    offs = np.array(list(itertools.product((-1, 0, 1), repeat=d)))
    dirs = np.array([v for v in itertools.product((-1, 0, 1), repeat=d) if any(v)], dtype=np.float64)
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    xs = np.zeros((len(offs), d), dtype=np.complex128)
    for k in range(d):
        idx = centre[k] + offs[:, k]
        xs[:, k] = idx * h + 1j * sig_axes[k](idx * h)
    F = np.exp(1j * kappa * (xs @ dirs.T))
    # gamma^* F = 0: gamma spans the null space of F^H. Each column is divided
    # by its value at the centre first (same null space, far better scaled:
    # the stretched waves grow by orders of magnitude across the PML).
    c0 = (len(offs) - 1) // 2
    _, s, Vh = np.linalg.svd((F / F[c0]).conj().T)
    g = np.conj(Vh[-1])
    g /= np.linalg.norm(g)
    c = g[(len(g) - 1) // 2]
    g *= np.conj(c) / abs(c)
    return g, F, s


def build(d, n, omega, m, b, w, C=10.0):
    alpha, beta, _ = alpha_beta(green_table(d, n, omega), n, d)
    system = SparseSystem(d, n, omega, m, alpha, beta, b, C)
    return system, Sweep(system, w, m)


@pytest.mark.parametrize("q", [0, 1, 5, 8])
def test_stretch_values_against_formula(q):
    n, b, C, omega = 31, 8, 10.0, 2 * math.pi * 4
    h = 1.0 / (n + 1)
    # global PML: index -1-q and n+2+q (q = b is the Dirichlet point)
    for i in (-1 - q, n + 2 + q):
        ref = sigma_paper(np.array([i * h]), h, b, C, omega)[0]
        assert sigma_global(np.array([i]), n, b, C, omega)[0] == pytest.approx(ref, rel=1e-14, abs=1e-300)
    assert abs(sigma_global(np.array([-1 - q]), n, b, C, omega)[0]) == pytest.approx(
        (C / omega) * (q / b) ** 2, rel=1e-14, abs=1e-300)
    # moved PML left of a slice whose first line is s: zero at s-1, depth q at s-1-q
    s = 20
    got = sigma_aux(np.array([s - 1 - q, s - 1, s]), s, b, C, omega)
    ref = sigma_moved(np.array([s - 1 - q, s - 1, s]) * h, (s - 1) * h, h, b, C, omega)
    np.testing.assert_allclose(got, ref, rtol=1e-14, atol=1e-300)
    assert got[1] == 0.0 and got[2] == 0.0
    assert got[0] == pytest.approx(-(C / omega) * (q / b) ** 2, rel=1e-14, abs=1e-300)


def test_aux_stencil_is_global_stencil_of_same_depth_when_m_vanishes():
    n, b, w = 21, 6, 4
    omega = 2 * math.pi * 2.5
    m = np.zeros((n, n))
    system, sw = build(2, n, omega, m, b, w)
    assert sw.samples.count == 1
    assert len(sw.aux_gamma) > 0
    depths = set()
    for (q, c2, ks), g in sw.aux_gamma.items():
        assert ks == 0
        depths.add(q)
        # aux depth q sits where the global PML has index -1-q, i.e. class b - q
        ref = system.gamma_by_class[(b - q, c2)]
        assert np.abs(g - ref).max() <= 1e-14, (q, c2)
    assert depths == set(range(b))


@pytest.mark.parametrize("d", [2, 3])
def test_aux_stencils_annihilate_local_plane_waves_constant_medium(d):
    n, b, w, C = (21, 5, 4, 10.0) if d == 2 else (7, 3, 3, 10.0)
    omega = 2 * math.pi * (2.5 if d == 2 else 1.0)
    m0 = 0.36
    h = 1.0 / (n + 1)
    m = np.full((n,) * d, m0)
    system, sw = build(d, n, omega, m, b, w, C)
    kappa = omega * math.sqrt(1.0 - m0)
    glob = lambda x: sigma_paper(x, h, b, C, omega)
    # the stored stencils are keyed by depth and transverse class, shared by
    # every slice: check them at the edge of slice 2
    assert sw.nslices >= 2 and sw.samples.count == 1
    lo = sw.bounds[1][0]
    moved = lambda x: sigma_moved(x, (lo - 1) * h, h, b, C, omega)
    checked = 0
    for (q, *tcls, ks), g in sw.aux_gamma.items():
        centre = [lo - 1 - q] + [rep_index(c, n, b) for c in tcls]
        _, F, _ = null_stencil(kappa, h, centre, [moved] + [glob] * (d - 1), d)
        res = np.linalg.norm(g.conj() @ F) / np.linalg.norm(F)
        assert res <= 1e-12, (q, tcls, res)
        checked += 1
    assert checked >= b


def rep_index(c, n, b):
    """A transverse grid index whose 3-point stretch class is c (0: the three
    points unstretched; 1..b: low PML at depth b+1-c; b+1..2b: high side)."""
    if c == 0:
        return 3
    if c <= b:
        return c - 1 - b
    return n + 2 + (c - b - 1)


def sample_index(mv, lo, hi, count, omega):
    """Sec. 2.3 with reading G9: the nearest of ``count`` equispaced samples of
    the squared local frequency on [lo, hi], both endpoints included."""
    if count == 1 or hi == lo:
        return 0
    delta = (hi - lo) / (count - 1)
    v = omega * omega * (1.0 - mv)
    return int(min(max(math.floor((v - lo) / delta + 0.5), 0), count - 1))


@pytest.mark.parametrize("d", [2, 3])
def test_assembled_aux_rows_follow_depth_and_local_wavenumber(d):
    if d == 2:
        n, b, w, omega = 23, 5, 4, 2 * math.pi * 2.5
        m = workloads.gaussian_bump_medium(n, 2, 6, (0.2, 0.8), (0.05, 0.1), (-0.35, 0.35), seed=3)
    else:
        n, b, w, omega = 7, 3, 3, 2 * math.pi * 1.0
        m = workloads.gaussian_bump_medium(n, 3, 3, (0.25, 0.75), (0.1, 0.2), (-0.3, 0.3), seed=4)
    C = 10.0
    h = 1.0 / (n + 1)
    system, sw = build(d, n, omega, m, b, w, C)
    L = system.L
    T = L ** (d - 1)
    w2 = omega * omega
    lo_s, hi_s = w2 * (1 - m.max()), w2 * (1 - m.min())
    count = n
    assert sw.samples.count == count
    m_ext = np.zeros((L,) * d)
    m_ext[(slice(b + 1, b + 1 + n),) * d] = m
    glob = lambda x: sigma_paper(x, h, b, C, omega)
    offs = np.array(list(itertools.product((-1, 0, 1), repeat=d)))
    tpos = np.array(list(itertools.product(range(-b, n + 2 + b), repeat=d - 1)))
    kappas_seen = set()
    for k in range(1, sw.nslices):
        lo = sw.bounds[k][0]
        A, naux, nauxr = sw._subproblem(k)
        assert nauxr == 0
        A = A.tocsr()
        assert naux == b * T
        moved = lambda x, edge=(lo - 1) * h: sigma_moved(x, edge, h, b, C, omega)
        for a in range(b):
            line = lo - b + a                       # grid line of local aux line a
            for t, tp in enumerate(tpos):
                p = (line,) + tuple(tp)
                mv = m_ext[tuple(np.array(p) + b)]
                ks = sample_index(mv, lo_s, hi_s, count, omega)
                kappa = math.sqrt(lo_s + ks * (hi_s - lo_s) / (count - 1))
                kappas_seen.add(ks)
                g, F, s = null_stencil(kappa, h, p, [moved] + [glob] * (d - 1), d)
                assert s[-1] >= 1e-6 * s[0]         # 3^d - 1 independent waves: a 1-D null space
                assert np.linalg.norm(g.conj() @ F) <= 1e-12 * np.linalg.norm(F)
                row = A.getrow(a * T + t)
                want = {}
                for o, off in enumerate(offs):
                    nb = np.array(p) + off
                    if nb[0] < lo - b:
                        continue                    # the Dirichlet line left of the auxiliary PML
                    if np.any(nb[1:] < -b) or np.any(nb[1:] > n + 1 + b):
                        continue                    # the transverse Dirichlet ring
                    loc = (nb[0] - (lo - b)) * T + int(np.ravel_multi_index(tuple(nb[1:] + b), (L,) * (d - 1)))
                    want[loc] = np.conj(g[o])
                got = dict(zip(row.indices.tolist(), row.data.tolist()))
                assert set(got) == set(want), (k, a, t)
                err = max(abs(got[c] - want[c]) for c in want)
                assert err <= 1e-12, (k, a, t, err)
    assert len(kappas_seen) > 2          # the rows really use several samples
