"""GPU: the autotuned setup (layer thickness and kernel choice chosen by
timing on the device) lists every candidate it timed, keeps the fastest, and
solves to the same answers as the oracle set up with the thickness it chose.

The layer thickness is free in the method (the remarks closing Sec. 2.3), so
the oracle at the chosen w is the reference; the protocol of the other solve
tests applies (mixed form within 1e-5 of the oracle's tight solution at tol
1e-6, true residual with the oracle's operator).
"""
import math
import sys

import numpy as np
import pytest
import torch

import oracle
import workloads

pytestmark = pytest.mark.gpu

N, PPW, B, K = 40, 2.5, 6, 4


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(b), 1e-300))


@pytest.fixture(scope="module")
def medium():
    wl = workloads.workload("C0").scaled(N, ppw_omega=PPW)
    m = workloads.gaussian_bump_medium(N, 2, 6, (0.2, 0.8), (0.04, 0.1), (-0.4, 0.4), seed=3)
    return wl.omega, m


def candidates(n, b, fronts):
    """Layer thicknesses whose slice subproblems (the oracle's partition, b
    auxiliary lines on each side facing an earlier-eliminated slice) all have
    at most 32 lines; the tuner times the four thinnest."""
    from oracle.sparse import slice_partition
    out = []
    for w in range(2, n + 3):
        bounds, order = slice_partition(n, b, w, fronts)
        pos = {k: i for i, k in enumerate(order)}
        tmax = 0
        for k, (lo, hi) in enumerate(bounds):
            aux = sum(b for j in (k - 1, k + 1) if 0 <= j < len(bounds) and pos[j] < pos[k])
            tmax = max(tmax, hi - lo + 1 + aux)
        if tmax <= 32:
            out.append((w, len(bounds)))
    return out


@pytest.mark.parametrize("fronts", [1, 2])
def test_autotuned_setup_matches_the_oracle(medium, fronts):
    from paper_1705_09443_amd import LSSolver, layer_candidates
    omega, m = medium
    cands = candidates(N, B, fronts)
    if fronts == 1:
        assert [w for w, _ in cands] == layer_candidates(N, B)
    cands = cands[:4]
    say(f"[autotune] n={N} b={B}, {fronts} front(s), probe batch {K}, candidates timed {cands}")
    with LSSolver(torch.as_tensor(m).cuda(), omega, B, None, precision="mixed", autotune=K, fronts=fronts) as s:
        t = s.tuning()
        for row in t["layers"]:
            say(f"[autotune] w={row[0]} slices={row[1]} iterations={row[2]} setup {row[3]:.1f} ms "
                f"solve {row[4]:.2f} ms")
        for row in t["kernels"]:
            say(f"[autotune] batch {row[0]}: slice kernel {row[1]}, interface kernel {row[2]}, {row[3]:.3f} ms")
        assert [(r[0], r[1]) for r in t["layers"]] == cands
        for w, nl, its, sms, ms in t["layers"]:
            assert its >= 1 and sms > 0 and ms > 0
        assert s.layer_thickness == min(t["layers"], key=lambda r: r[4])[0]
        assert s.nslices == dict(cands)[s.layer_thickness]
        assert [r[0] for r in t["kernels"]] == [1, 2, 3, 4]
        for nb, sk, ik, ms in t["kernels"]:
            assert sk in (1, 4, 8, 16) and ik in (0, 1) and ms > 0
        uinc = workloads.plane_waves(N, 2, omega, workloads.angle_directions(K, 2))
        u, info = s.solve(torch.as_tensor(uinc).cuda(), "incident", 1e-6)
        u = u.cpu().numpy()
        w = s.layer_thickness
    ref = oracle.OracleSolver(2, N, omega, m, B, w, fronts=fronts)
    for j in range(K):
        g = ref.op.rhs_incident(uinc[j])
        assert info[j].converged and info[j].rel_residual <= 1e-6
        assert rel(ref.op.apply_A(u[j]), g) <= 1.01e-6
        assert rel(u[j], ref.solve_rhs(g, 1e-12).x) <= 1e-5


def test_fixed_thickness_tunes_kernels_only(medium):
    from paper_1705_09443_amd import LSSolver
    omega, m = medium
    rng = np.random.default_rng(7)
    r = rng.standard_normal((3, N, N)) + 1j * rng.standard_normal((3, N, N))
    md = torch.as_tensor(m).cuda()
    with LSSolver(md, omega, B, 3, precision="fp64", autotune=3) as s, \
            LSSolver(md, omega, B, 3, precision="fp64") as d:
        t = s.tuning()
        assert t["layers"] == [] and [row[0] for row in t["kernels"]] == [1, 2, 3]
        assert s.layer_thickness == 3
        # the tuned and the default choices compute the same preconditioner
        zt = s.apply_precond(torch.as_tensor(r).cuda()).cpu().numpy()
        zd = d.apply_precond(torch.as_tensor(r).cuda()).cpu().numpy()
        assert rel(zt, zd) <= 1e-12
