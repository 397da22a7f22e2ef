"""Pins for the oracle's misfit gradient (derived from eq. LS_d_c).

* brute force: on a tiny grid every component dJ/dm_k is formed from the
  dense matrices directly, du/dm_k = -A^{-1} omega^2 K e_k e_k^T psi;
* central finite differences of J along seeded directions;
* the dot-product identity <A x, y> = <x, A^H y> behind the adjoint solve.
"""
import math

import numpy as np

import workloads
from oracle import OracleSolver, dense_A, DenseOperator


def setup_case(n=9, ppw=1.5, ndir=3):
    wl = workloads.workload("C4").scaled(n, ppw_omega=ppw)
    m = workloads.gaussian_bump_medium(n, 2, 4, (0.3, 0.7), (0.1, 0.2), (-0.3, 0.3), seed=0)
    md = workloads.gaussian_bump_medium(n, 2, 4, (0.3, 0.7), (0.1, 0.2), (-0.3, 0.3), seed=1)
    dirs = workloads.angle_directions(ndir, 2)
    uinc = workloads.plane_waves(n, 2, wl.omega, dirs)
    rec = workloads.circle_receivers(n, 0.35)
    return wl.omega, m, md, uinc, rec


def misfit(op, m, uinc, rec, data):
    A = dense_A(op.table, op.n, 2, op.omega, m)
    J = 0.0
    us = []
    for j in range(uinc.shape[0]):
        g = -op.omega ** 2 * op.apply_K(m * uinc[j])
        u = np.linalg.solve(A, g.reshape(-1)).reshape(g.shape)
        us.append(u)
        J += 0.5 * np.sum(np.abs(u[rec] - data[j]) ** 2)
    return J, np.array(us)


def test_gradient_matches_brute_force_and_fd():
    n = 9
    omega, m, md, uinc, rec = setup_case(n)
    op_d = DenseOperator(2, n, omega, md)
    _, ud = misfit(op_d, md, uinc, rec, np.zeros((uinc.shape[0], rec.sum())))
    data = np.array([u[rec] for u in ud])
    s = OracleSolver(2, n, omega, m, 4, 3)
    J0, us = misfit(s.op, m, uinc, rec, data)
    resid = np.zeros_like(us)
    for j in range(us.shape[0]):
        resid[j][rec] = us[j][rec] - data[j]
    grad = s.gradient(us, resid, uinc, tol=1e-13)
    # brute force with dense matrices
    A = dense_A(s.op.table, n, 2, omega, m)
    # K itself: the dense operator with m = 1, minus I, over omega^2
    Kfull = (dense_A(s.op.table, n, 2, omega, np.ones((n, n))) - np.eye(n * n)) / omega ** 2
    Ainv_K = np.linalg.solve(A, Kfull)
    bf = np.zeros(n * n)
    for j in range(us.shape[0]):
        psi = (us[j] + uinc[j]).reshape(-1)
        r = resid[j].reshape(-1)
        # dJ/dm_k = Re r^H du/dm_k, du/dm_k = -omega^2 A^{-1} K e_k psi_k
        bf += np.real(np.conj(r) @ (-omega ** 2 * Ainv_K * psi[None, :]))
    assert np.linalg.norm(grad.reshape(-1) - bf) <= 1e-9 * np.linalg.norm(bf)
    # central differences along seeded directions
    dms = workloads.fd_directions(n, 2, 3, seed=2)
    eps = 1e-6
    for dm in dms:
        Jp, _ = misfit(s.op, m + eps * dm, uinc, rec, data)
        Jm, _ = misfit(s.op, m - eps * dm, uinc, rec, data)
        fd = (Jp - Jm) / (2 * eps)
        assert abs(fd - np.sum(grad * dm)) <= 1e-6 * abs(fd)


def test_dot_product_identity():
    n = 11
    omega, m, _, _, _ = setup_case(n)
    op = DenseOperator(2, n, omega, m)
    A = dense_A(op.table, n, 2, omega, m)
    rng = np.random.default_rng(8)
    x = rng.standard_normal(n * n) + 1j * rng.standard_normal(n * n)
    y = rng.standard_normal(n * n) + 1j * rng.standard_normal(n * n)
    Ax = op.apply_A(x.reshape(n, n)).reshape(-1)
    np.testing.assert_allclose(Ax, A @ x, rtol=1e-12)
    # A^H y = y + omega^2 M conj(K) y, using K = K^T
    AHy = y + omega ** 2 * m.reshape(-1) * np.conj(op.apply_K(np.conj(y).reshape(n, n))).reshape(-1)
    assert abs(np.vdot(Ax, y) - np.vdot(x, AHy)) <= 1e-12 * abs(np.vdot(Ax, y))
