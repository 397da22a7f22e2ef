"""Pins for the oracle's stencils (eqs. alpha, beta, gamma; Sec. 2.3 sampling).

alpha is checked against a full SVD of the explicit K_{mu,mu^c} (a different
route from the oracle's streamed QR), beta against its definition with a
directly evaluated K_{mu,mu}, gamma against the paper's unscaled modified
plane waves exp(i kappa r . x^sigma) in absolute coordinates, and the
stencils against the grid symmetries noted in Sec. 2.2.
"""
import itertools
import math

import numpy as np
import pytest

from oracle import (alpha_beta, green, central_weight, green_table, neighbourhood,
                    plane_wave_directions, pml_stencil, sigma_global, normalise_phase,
                    FrequencySamples)
from oracle.stencils import sigma_aux


def explicit_K_mu_muc(d, n, omega):
    h = 1.0 / (n + 1)
    mu = neighbourhood(d)
    ls = [l for l in itertools.product(range(-n, n + 1), repeat=d) if max(abs(v) for v in l) > 1]
    ls = np.array(ls)
    off = mu[:, None, :] - ls[None, :, :]
    r = np.sqrt((off ** 2).sum(-1)) * h
    return green(d, omega, r) * h ** d


@pytest.mark.parametrize("d,n,ppw", [(2, 15, 2.0), (2, 63, 4.0), (3, 7, 1.0)])
def test_alpha_is_smallest_left_singular_vector(d, n, ppw):
    omega = 2 * math.pi * ppw
    t = green_table(d, n, omega)
    alpha, beta, sv = alpha_beta(t, n, d, chunk_rows=97)
    K = explicit_K_mu_muc(d, n, omega)
    U, S, _ = np.linalg.svd(K, full_matrices=False)
    ref = normalise_phase(U[:, -1])
    assert np.linalg.norm(alpha - ref) <= 1e-12
    assert np.linalg.norm(alpha.conj() @ K) == pytest.approx(S[-1], rel=1e-10)
    np.testing.assert_allclose(sv, S, rtol=1e-11)
    assert S[-2] / S[-1] > 10            # reading G6: the minimiser is unique
    assert abs(np.linalg.norm(alpha) - 1) < 1e-14


def test_alpha_beta_symmetry_2d():
    n, omega = 63, 2 * math.pi * 4
    alpha, beta, _ = alpha_beta(green_table(2, n, omega), n, 2)
    for v in (alpha, beta):
        a = v.reshape(3, 3)
        for g in (a.T, a[::-1, :], a[:, ::-1]):
            assert np.abs(g - a).max() < 1e-12 * np.abs(a).max()
    assert alpha[4].imag == 0 and alpha[4].real > 0


def test_alpha_symmetry_3d():
    n, omega = 7, 2 * math.pi
    alpha, beta, _ = alpha_beta(green_table(3, n, omega), n, 3)
    a = alpha.reshape(3, 3, 3)
    for perm in itertools.permutations(range(3)):
        assert np.abs(np.transpose(a, perm) - a).max() < 1e-12
    assert np.abs(a[::-1] - a).max() < 1e-12


def test_beta_definition():
    d, n, omega = 2, 31, 2 * math.pi * 2
    h = 1.0 / (n + 1)
    alpha, beta, _ = alpha_beta(green_table(d, n, omega), n, d)
    mu = neighbourhood(d)
    off = mu[:, None, :] - mu[None, :, :]
    r = np.sqrt((off ** 2).sum(-1)) * h
    with np.errstate(divide="ignore", invalid="ignore"):
        Kmm = np.where(r > 0, green(d, omega, np.where(r > 0, r, 1.0)) * h * h, central_weight(d, omega, h))
    # beta^* = alpha^* K_{mu,mu}
    np.testing.assert_allclose(np.conj(beta), alpha.conj() @ Kmm, rtol=0, atol=1e-15)


def paper_F(kappa, h, centre, sig_of_axis, dirs):
    """exp(i kappa r . x^sigma) on mu_i in absolute coordinates, x^sigma = x + i sigma(x)."""
    d = len(centre)
    mu = neighbourhood(d)
    cols = []
    for r in dirs:
        ph = np.zeros(len(mu), dtype=np.complex128)
        for k in range(d):
            idx = centre[k] + mu[:, k]
            ph += r[k] * (idx * h + 1j * sig_of_axis[k](idx))
        cols.append(np.exp(1j * kappa * ph))
    return np.array(cols).T


@pytest.mark.parametrize("d", [2, 3])
def test_gamma_annihilates_modified_plane_waves(d):
    n, b, C = 31, 8, 10.0
    omega = 2 * math.pi * 4
    h = 1.0 / (n + 1)
    dirs = plane_wave_directions(d)
    assert len(dirs) == 3 ** d - 1
    sg = lambda i: sigma_global(i, n, b, C, omega)
    positions = [(-1,) + (5,) * (d - 1), (-b,) + (0,) * (d - 1), (n + 2,) + (n + 1 + b,) * (d - 1),
                 (-3,) + (-b,) * (d - 1), (4,) + (n + 5,) * (d - 1)]
    for pos in positions:
        sig = np.array([sg(np.array([p - 1, p, p + 1])) for p in pos])
        g = pml_stencil(omega, h, sig, dirs)
        F = paper_F(omega, h, pos, [sg] * d, dirs)
        assert np.linalg.norm(g.conj() @ F) <= 1e-12 * np.linalg.norm(F)
        assert abs(np.linalg.norm(g) - 1) < 1e-14
    # auxiliary PML left of a slice starting at line s, at a sampled local wavenumber
    s = 12
    kappa = omega * math.sqrt(1 - 0.23)
    sa = lambda i: sigma_aux(i, s, b, C, omega)
    for q in range(b):
        pos = (s - 1 - q,) + (-2,) * (d - 1)
        sig = np.array([sa(np.array([pos[0] - 1, pos[0], pos[0] + 1]))] +
                       [sg(np.array([p - 1, p, p + 1])) for p in pos[1:]])
        g = pml_stencil(kappa, h, sig, dirs)
        F = paper_F(kappa, h, pos, [sa] + [sg] * (d - 1), dirs)
        assert np.linalg.norm(g.conj() @ F) <= 1e-12 * np.linalg.norm(F)


def test_gamma_mirror_symmetry():
    # the stretch is mirror symmetric (Sec. 2.2.2): the stencil at the mirrored
    # position is the mirrored stencil
    n, b, C, omega = 31, 8, 10.0, 2 * math.pi * 4
    h = 1.0 / (n + 1)
    dirs = plane_wave_directions(2)
    sg = lambda i: sigma_global(i, n, b, C, omega)
    for p1, p2 in [(-1, 7), (-b, -3), (-5, -b)]:
        q1, q2 = n + 1 - p1, n + 1 - p2
        s1 = np.array([sg(np.array([p1 - 1, p1, p1 + 1])), sg(np.array([p2 - 1, p2, p2 + 1]))])
        s2 = np.array([sg(np.array([q1 - 1, q1, q1 + 1])), sg(np.array([q2 - 1, q2, q2 + 1]))])
        g1 = pml_stencil(omega, h, s1, dirs).reshape(3, 3)
        g2 = pml_stencil(omega, h, s2, dirs).reshape(3, 3)
        assert np.abs(g1[::-1, ::-1] - g2).max() < 1e-12


def test_gamma_without_stretch_is_translation_invariant_plane_wave_stencil():
    n, b, C, omega = 31, 8, 10.0, 2 * math.pi * 4
    h = 1.0 / (n + 1)
    dirs = plane_wave_directions(2)
    g = pml_stencil(omega, h, np.zeros((2, 3)), dirs)
    pw = np.exp(1j * omega * h * (neighbourhood(2) @ dirs.T))
    assert np.linalg.norm(g.conj() @ pw) < 1e-13
    # symmetric like the free-space problem it discretises
    a = g.reshape(3, 3)
    assert np.abs(a - a.T).max() < 1e-12 and np.abs(a - a[::-1]).max() < 1e-12


def test_frequency_samples():
    m = np.array([[0.0, 0.2], [-0.1, 0.35]])
    omega = 10.0
    fs = FrequencySamples(m, omega, 8)
    assert fs.lo == pytest.approx(100 * 0.65) and fs.hi == pytest.approx(100 * 1.1)
    ks = fs.index(np.array([0.35, -0.1, 0.0, 0.2]))
    assert ks[0] == 0 and ks[1] == 7
    grid = fs.lo + np.arange(8) * fs.delta
    for mv, k in zip([0.0, 0.2], ks[2:]):
        v = 100 * (1 - mv)
        assert k == int(np.argmin(np.abs(grid - v)))
    assert fs.kappa(0) == pytest.approx(math.sqrt(65.0))
    # constant medium: one sample
    fs1 = FrequencySamples(np.full((3, 3), 0.1), omega, 8)
    assert fs1.count == 1 and fs1.index(np.array([0.1, 0.0]))[1] == 0
    with pytest.raises(ValueError):
        FrequencySamples(np.array([1.0, 0.0]), omega, 4)
