"""Parity of the library's float64 host setup (own Bessel functions, streamed
QR + one-sided Jacobi SVD for alpha, Householder null vectors for gamma)
against the oracle (scipy AMOS Hankel, numpy QR + LAPACK SVD): the stencil
tables agree to 1e-12 after the phase normalisation (reading G5), the sample
map is bit-exact (an integer decided in float64 by the same expression)."""
import math

import numpy as np
import pytest

import workloads
import oracle
from oracle.sparse import class_index
from oracle.stencils import sigma_global, FrequencySamples
from paper_1705_09443_amd import host_tables


def _oracle_setup(wl, m, b, w, C=10.0):
    return oracle.OracleSolver(2, wl.n, wl.omega, m, b, w, pml_C=C)


@pytest.fixture(scope="module")
def c0():
    wl = workloads.workload("C0")
    m = wl.medium_array()
    ref = _oracle_setup(wl, m, 12, 4)
    got = host_tables(m, wl.omega, 12, 4)
    return wl, m, ref, got


def test_green_quadrant(c0):
    wl, m, ref, got = c0
    n = wl.n
    t = ref.op.table[n + 1:, n + 1:]
    env = np.abs(t).max()
    assert np.abs(got["green"] - t).max() <= 1e-14 * env
    # away from the centre, relative to the local size of G h^2
    h = 1.0 / (n + 1)
    r = np.hypot(*np.meshgrid(np.arange(n + 2), np.arange(n + 2), indexing="ij")) * h
    r[0, 0] = 1
    scale = 0.25 * np.sqrt(2 / (math.pi * wl.omega * r)) * h * h
    assert (np.abs(got["green"] - t) / scale)[1:, 1:].max() < 1e-13


def test_alpha_beta(c0):
    wl, m, ref, got = c0
    assert np.abs(got["alpha"] - ref.alpha).max() <= 1e-12
    assert np.abs(got["beta"] - ref.beta).max() <= 1e-12 * np.abs(ref.beta).max()


def test_global_gamma(c0):
    wl, m, ref, got = c0
    b = 12
    for key, g in ref.system.gamma_by_class.items():
        assert np.abs(got["gamma"][key] - g).max() <= 1e-12, key


def test_sample_map_bit_exact(c0):
    wl, m, ref, got = c0
    s = ref.system
    km = ref.sweep.samples.index(s.m_ext).reshape(s.L, s.L)
    np.testing.assert_array_equal(got["kmap"], km)


def test_aux_gamma(c0):
    wl, m, ref, got = c0
    assert len(ref.sweep.aux_gamma) > 100
    for (q, c2, ks), g in ref.sweep.aux_gamma.items():
        assert np.abs(got["aux"][q, c2, ks] - g).max() <= 1e-12, (q, c2, ks)
    # every table entry the library filled is one some auxiliary point uses
    used = set(ref.sweep.aux_gamma)
    filled = set(map(tuple, np.argwhere(np.abs(got["aux"]).sum(-1) > 0)))
    assert filled == used


@pytest.mark.parametrize("n,ppw", [(255, 16.0), (31, 2.0)])
def test_alpha_other_sizes(n, ppw):
    omega = 2 * math.pi * ppw
    t = oracle.green_table(2, n, omega)
    alpha, beta, sv = oracle.alpha_beta(t, n, 2)
    m = np.zeros((n, n))
    got = host_tables(m, omega, 8, 4)
    assert np.abs(got["alpha"] - alpha).max() <= 1e-12
    assert np.abs(got["beta"] - beta).max() <= 1e-12 * np.abs(beta).max()
    # constant medium: one frequency sample, index 0 everywhere
    assert got["aux"].shape[2] == 1 and got["kmap"].max() == 0


def test_invalid_inputs_raise():
    from paper_1705_09443_amd import LsError
    with pytest.raises(LsError):
        host_tables(np.full((7, 7), 1.0), 10.0, 4, 2)        # m >= 1
    with pytest.raises(LsError):
        host_tables(np.zeros((7, 7)), 1000.0, 4, 2)          # < 2 points per wavelength
    bad = np.zeros((7, 7))
    bad[3, 3] = np.nan
    with pytest.raises(LsError):
        host_tables(bad, 10.0, 4, 2)


@pytest.mark.parametrize("n,ppw", [(1, 0.5), (15, 2.0), (31, 2.0)])
def test_green3_octant(n, ppw):
    """The library's 3D table (Sec. 1 Green's function, k_0 over the ball of
    volume h^3) against the oracle's, 1e-14 of its largest entry and 1e-13
    relative to the local size of G h^3 away from the centre."""
    from paper_1705_09443_amd import host_green3
    omega = 2.0 * math.pi * ppw
    t = oracle.green_table(3, n, omega)[n + 1:, n + 1:, n + 1:]
    got = host_green3(n, omega)
    assert got.shape == (n + 2,) * 3
    assert np.abs(got - t).max() <= 1e-14 * np.abs(t).max()
    h = 1.0 / (n + 1)
    r = np.sqrt(sum(g * g for g in np.meshgrid(*([np.arange(n + 2)] * 3), indexing="ij"))) * h
    r[0, 0, 0] = 1.0
    scale = h ** 3 / (4 * math.pi * r)
    err = np.abs(got - t) / scale
    err[0, 0, 0] = 0.0
    assert err.max() < 1e-13


def test_green3_rejects_bad_arguments():
    from paper_1705_09443_amd import _lib
    lib = _lib.load()
    buf = np.zeros(2 * 27)
    for n, om in [(0, 1.0), (1024, 1.0), (1, 0.0), (1, float("nan"))]:
        assert lib.ls_host_green3(n, om, buf.ctypes.data) == _lib.LS_E_INVALID
    assert lib.ls_host_green3(1, 1.0, None) == _lib.LS_E_INVALID


@pytest.mark.parametrize("n,ppw,b,w", [(9, 1.0, 3, 3), (15, 2.0, 4, 4)])
def test_tables3_match_oracle(n, ppw, b, w):
    """3D setup (Sec. 3.1): alpha, beta to 1e-12 of the oracle's (numpy QR +
    LAPACK SVD), gamma of every global and used auxiliary class to 1e-12
    after the phase normalisation (reading G5), the sample map bit-exact."""
    from paper_1705_09443_amd import host_tables3
    omega = 2 * math.pi * ppw
    m = workloads.gaussian_bump_medium(n, 3, 5, (0.25, 0.75), (0.05, 0.1), (-0.3, 0.3), seed=1)
    got = host_tables3(m, omega, b, w)
    ref = oracle.OracleSolver(3, n, omega, m, b, w)
    assert np.abs(got["alpha"] - ref.alpha).max() < 1e-12
    assert np.abs(got["beta"] - ref.beta).max() < 1e-12 * np.abs(ref.beta).max()
    for key, g in ref.system.gamma_by_class.items():
        assert np.abs(got["gamma"][key] - g).max() < 1e-12, key
    assert len(ref.sweep.aux_gamma) > 0
    for (q, c2, c3, ks), g in ref.sweep.aux_gamma.items():
        assert np.abs(got["aux"][q, c2, c3, ks] - g).max() < 1e-12
    assert np.array_equal(got["kmap"].reshape(-1), FrequencySamples(m, omega, n).index(ref.system.m_ext))


def test_tables3_refuse_oversized_slabs_at_once():
    # slab limits (32 lines, blocks of 4800 unknowns) are checked before the
    # O(n^3) host setup: these grids would take minutes to tabulate
    from paper_1705_09443_amd import _lib
    import time
    lib = _lib.load()
    n = 200
    m = np.zeros((n, n, n))
    t0 = time.time()
    # b = 8, w = 8: the last slab has 8 + 18 lines of L = 218 -> 5668 unknowns per block
    st = lib.ls_host_tables3(n, 2 * math.pi * 8, m.ctypes.data, 8, 8, 10.0, 0, None, None, None, None, None)
    assert st == _lib.LS_E_INVALID
    assert b"4800" in lib.ls_last_error()
    # w = 40: slabs of 48 lines
    st = lib.ls_host_tables3(n, 2 * math.pi * 8, m.ctypes.data, 8, 40, 10.0, 0, None, None, None, None, None)
    assert st == _lib.LS_E_INVALID
    assert b"32" in lib.ls_last_error()
    assert time.time() - t0 < 5.0


def test_stencil_cache_reuses_velocity_independent_tables():
    """The 2D stencil cache: a second setup with the same (n, omega, b, C)
    and another medium and layer thickness reuses the Green table, alpha,
    beta and the global PML stencils. It returns bitwise what a fresh
    computation gives. A change of any key computes them anew, and the
    medium-dependent tables (aux stencils, sample map) always follow m."""
    import numpy as np
    import workloads
    from paper_1705_09443_amd import host_tables, stencil_cache
    n, omega, b = 40, 2 * np.pi * 2.5, 6
    m1 = workloads.gaussian_bump_medium(n, 2, 6, (0.2, 0.8), (0.04, 0.1), (-0.4, 0.4), seed=3)
    m2 = workloads.gaussian_bump_medium(n, 2, 6, (0.2, 0.8), (0.04, 0.1), (-0.4, 0.4), seed=4)
    stencil_cache(clear=True)
    fresh = host_tables(m1, omega, b, 3)                  # computes and caches
    assert stencil_cache() == (0, 1)
    again = host_tables(m2, omega, b, 4)                  # same key: a hit
    assert stencil_cache() == (1, 1)
    for k in ("alpha", "beta", "gamma", "green"):
        assert np.array_equal(again[k], fresh[k]), k
    # the medium-dependent tables follow m2, not m1
    stencil_cache(clear=True)
    ref2 = host_tables(m2, omega, b, 4)
    assert np.array_equal(again["aux"], ref2["aux"]) and np.array_equal(again["kmap"], ref2["kmap"])
    assert not np.array_equal(again["aux"], fresh["aux"])
    # every key component misses: omega, b, C, n
    stencil_cache(clear=True)
    host_tables(m1, omega, b, 3)
    host_tables(m1, omega * (1 + 1e-12), b, 3)
    host_tables(m1, omega, b - 1, 3)
    host_tables(m1, omega, b, 3, pml_C=9.0)
    host_tables(m1[:-1, :-1], omega, b, 3)
    assert stencil_cache() == (0, 5)
    # at most four entries are kept: the first key has been evicted
    host_tables(m1, omega, b, 3)
    assert stencil_cache() == (0, 6)
    stencil_cache(clear=True)


def test_stencil_cache_3d():
    """The same cache in 3D: a second 3D setup with another medium and layer
    thickness reuses the m-independent tables bitwise, and a 2D setup of the
    same n, omega, b and C does not match a 3D entry."""
    import numpy as np
    import workloads
    from paper_1705_09443_amd import host_tables, host_tables3, stencil_cache
    n, omega, b = 9, 2 * np.pi * 1.0, 3
    m1 = workloads.gaussian_bump_medium(n, 3, 5, (0.25, 0.75), (0.05, 0.1), (-0.3, 0.3), seed=1)
    m2 = workloads.gaussian_bump_medium(n, 3, 5, (0.25, 0.75), (0.05, 0.1), (-0.3, 0.3), seed=2)
    stencil_cache(clear=True)
    fresh = host_tables3(m1, omega, b, 3)
    again = host_tables3(m2, omega, b, 4)
    assert stencil_cache() == (1, 1)
    for k in ("alpha", "beta", "gamma"):
        assert np.array_equal(again[k], fresh[k]), k
    host_tables(m1[0], omega, b, 3)                        # 2D, same n, omega, b, C
    assert stencil_cache() == (1, 2)
    stencil_cache(clear=True)
