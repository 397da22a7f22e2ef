"""GPU parity of the 3D method (Sec. 3.1 with Sec. 2.2-2.3 and Algorithms 1-2
in d = 3): stencils through the handle, Q and H, single slab solves, the
sweeping preconditioner and whole solves, against the oracle (SuperLU slab
factorizations, scipy FFTs), through the C ABI.

Tolerances as in 2D: float64 applies and slab solves 1e-11 relative (the
library inverts the dense Schur complements of each slab block, the oracle
factors the sparse slab; both are backward stable, the slabs are
well-conditioned); complex64 slab solves and preconditioner 1e-5 (P5);
whole solves per the same protocol (iteration counts within one in both
precisions, the true residual below the tolerance, and float64 solutions
equal to 1e-10 with both sides stopped after the oracle's count, P1).
"""
import math
import sys

import numpy as np
import pytest

import oracle
import workloads

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def to_dev(x, dtype=torch.complex128):
    return torch.as_tensor(np.ascontiguousarray(x)).to(device="cuda", dtype=dtype)


def crand(rng, shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


FP32_BOUND = 1e-5   # P5


CASES3 = {
    # name: (n, omega/2pi, b, w); slabs of 6, 6 and 11 lines (nb = 102..187,
    # a ragged last Gauss-Jordan panel)
    "small": (9, 1.0, 3, 3),
    # four slabs, the last of 13 lines (nb = 325)
    "ragged": (15, 2.0, 4, 4),
    # eight slabs on L = 41: seven of 8 lines (nb = 328) and a last of 13
    # (nb = 533: 17 Gauss-Jordan panels, the last of 21 columns, and ragged
    # 64 x 64 update tiles), 8 points per wavelength
    "mid": (31, 4.0, 4, 4),
    # even L = 18: the top chain (blocks 0..8) is one block longer than the
    # bottom chain (17..10), so the last inward step carries one block
    "even": (10, 1.0, 3, 3),
}


@pytest.fixture(scope="module", params=list(CASES3))
def case3(request):
    from paper_1705_09443_amd import LSSolver
    n, ppw, b, w = CASES3[request.param]
    omega = 2 * math.pi * ppw
    m = workloads.gaussian_bump_medium(n, 3, 5, (0.25, 0.75), (0.05, 0.1), (-0.3, 0.3), seed=n)
    say(f"[{request.param}] oracle setup 3D n={n} b={b} w={w}")
    ref = oracle.OracleSolver(3, n, omega, m, b, w)
    md = torch.as_tensor(m).cuda()
    say(f"[{request.param}] library setup fp64 and mixed")
    g64 = LSSolver(md, omega, pml_width=b, layer_thickness=w, precision="fp64", schedule="sequential")
    g32 = LSSolver(md, omega, pml_width=b, layer_thickness=w, precision="mixed", schedule="sequential")
    yield request.param, n, omega, m, ref, g64, g32
    g64.close()
    g32.close()


def test_tables_through_handle(case3):
    name, n, omega, m, ref, g64, g32 = case3
    assert g64.dim == 3 and g64.nslices == ref.sweep.nslices
    al, be, gg, ga = g64.stencils()
    assert np.abs(al - ref.alpha).max() < 1e-12
    assert np.abs(be - ref.beta).max() < 1e-12 * np.abs(ref.beta).max()
    for key, g in ref.system.gamma_by_class.items():
        assert np.abs(gg[key] - g).max() < 1e-12
    for (q, c2, c3, ks), g in ref.sweep.aux_gamma.items():
        assert np.abs(ga[q, c2, c3, ks] - g).max() < 1e-12


def test_apply_A_Q_H(case3):
    name, n, omega, m, ref, g64, g32 = case3
    rng = np.random.default_rng(11)
    s = ref.system
    x = crand(rng, (2, n, n, n))
    u = crand(rng, (2,) + (s.L,) * 3)
    say(f"[{name}] apply A, Q, H")
    yA = g64.apply_A(to_dev(x)).cpu().numpy()
    f = g64.apply_Q(to_dev(x)).cpu().numpy()
    y = g64.apply_H(to_dev(u)).cpu().numpy()
    f32 = g32.apply_Q(to_dev(x, torch.complex64)).cpu().numpy()
    y32 = g32.apply_H(to_dev(u, torch.complex64)).cpu().numpy()
    for j in range(2):
        assert rel(yA[j], ref.op.apply_A(x[j])) <= 1e-12
        assert rel(f[j].reshape(-1), s.apply_Q(x[j])) <= 1e-12
        assert rel(y[j].reshape(-1), s.apply_H(u[j].reshape(-1))) <= 1e-12
        assert rel(f32[j].reshape(-1), s.apply_Q(x[j])) <= 1e-6
        assert rel(y32[j].reshape(-1), s.apply_H(u[j].reshape(-1))) <= 1e-6


def test_slab_solves(case3):
    name, n, omega, m, ref, g64, g32 = case3
    sw = ref.sweep
    L = sw.s.L
    rng = np.random.default_rng(12)
    for k in range(sw.nslices):
        lo, hi, naux = g64.slice_bounds(k)
        assert (lo, hi) == sw.bounds[k]
        lines = hi - lo + 1
        v = crand(rng, (3, lines, L, L))
        say(f"[{name}] slab_solve k={k} lines={lines} aux={naux}")
        w = g64.slice_solve(k, to_dev(v)).cpu().numpy()
        w32 = g32.slice_solve(k, to_dev(v, torch.complex64)).cpu().numpy()
        for j in range(3):
            ref_w = sw.solve_slice(k, v[j].reshape(-1))
            e64, e32 = rel(w[j].reshape(-1), ref_w), rel(w32[j].reshape(-1), ref_w)
            if j == 0:
                say(f"[{name}]   slab {k}: fp64 {e64:.2e} fp32 {e32:.2e}")
            assert e64 <= 1e-11, (k, j, e64)
            assert e32 <= FP32_BOUND, (k, j, e32)


def test_preconditioner(case3):
    name, n, omega, m, ref, g64, g32 = case3
    rng = np.random.default_rng(13)
    r = crand(rng, (3, n, n, n))
    say(f"[{name}] apply_precond fp64, fp32")
    z = g64.apply_precond(to_dev(r)).cpu().numpy()
    z32 = g32.apply_precond(to_dev(r, torch.complex64)).cpu().numpy()
    for j in range(3):
        zr = ref.precondition(r[j])
        e64, e32 = rel(z[j], zr), rel(z32[j], zr)
        say(f"[{name}]   rhs {j}: fp64 {e64:.2e} fp32 {e32:.2e}")
        assert e64 <= 1e-11
        assert e32 <= FP32_BOUND


def test_solves(case3):
    name, n, omega, m, ref, g64, g32 = case3
    uinc = workloads.plane_waves(n, 3, omega, workloads.angle_directions(2, 3, full_turn=False))
    say(f"[{name}] ls_solve fp64 and mixed, 2 rhs")
    u, info = g64.solve(to_dev(uinc), "incident", 1e-8)
    u32, info32 = g32.solve(to_dev(uinc), "incident", 1e-8)
    u, u32 = u.cpu().numpy(), u32.cpu().numpy()
    for j in range(uinc.shape[0]):
        g = ref.op.rhs_incident(uinc[j])
        res = ref.solve_rhs(g, 1e-8)
        say(f"[{name}]   rhs {j}: iterations lib {info[j].iterations} / {info32[j].iterations}, "
            f"oracle {res.iterations}")
        assert abs(info[j].iterations - res.iterations) <= 1
        assert info[j].converged and info32[j].converged
        assert rel(ref.op.apply_A(u[j]), g) <= 1.01e-8
        assert rel(ref.op.apply_A(u32[j]), g) <= 1.01e-8
        assert abs(info32[j].iterations - res.iterations) <= 1
        # P1: both stopped after the oracle's count k (a handle with
        # max_iters = k and an unreachable tolerance)
        from paper_1705_09443_amd import LSSolver
        k = res.iterations
        b, w = CASES3[name][2], CASES3[name][3]
        with LSSolver(torch.as_tensor(m).cuda(), omega, pml_width=b, layer_thickness=w, precision="fp64",
                      schedule="sequential", max_iters=k) as gk:
            uk, ik = gk.solve(to_dev(uinc[j][None]), "incident", 1e-300, allow_noconv=True)
        assert ik[0].iterations == k
        xk = ref.solve_rhs(g, 1e-300, max_iters=k).x
        e = rel(uk.cpu().numpy()[0], xk)
        say(f"[{name}]   rhs {j}: P1 after {k} steps {e:.2e}")
        assert e <= 1e-10


def test_preconditioner_batch_of_ten(case3):
    # ten right-hand sides: the products take them as one chunk of eight and
    # one of two (both right-hand-side widths of the product kernel)
    name, n, omega, m, ref, g64, g32 = case3
    rng = np.random.default_rng(14)
    r = crand(rng, (10, n, n, n))
    z = g64.apply_precond(to_dev(r)).cpu().numpy()
    z32 = g32.apply_precond(to_dev(r, torch.complex64)).cpu().numpy()
    w64 = w32 = 0.0
    for j in range(10):
        zr = ref.precondition(r[j])
        w64, w32 = max(w64, rel(z[j], zr)), max(w32, rel(z32[j], zr))
    say(f"[{name}] apply_precond, 10 rhs: worst fp64 {w64:.2e}, fp32 {w32:.2e}")
    assert w64 <= 1e-11
    assert w32 <= FP32_BOUND


def test_single_slab_preconditioner_is_exact_solve():
    """One slab (w >= n + 2) covers the whole extended cube: the sweep is the
    exact solve of H (Sec. 2.3), checked against a sparse LU of the oracle's H."""
    import scipy.sparse.linalg as spla
    from paper_1705_09443_amd import LSSolver
    n, b = 7, 2
    omega = 2 * math.pi * 1.0
    m = workloads.gaussian_bump_medium(n, 3, 4, (0.25, 0.75), (0.05, 0.1), (-0.3, 0.3), seed=7)
    ref = oracle.OracleSolver(3, n, omega, m, b, n + 2)
    assert ref.sweep.nslices == 1
    s = ref.system
    rng = np.random.default_rng(15)
    r = crand(rng, (2, n, n, n))
    g = LSSolver(torch.as_tensor(m).cuda(), omega, pml_width=b, layer_thickness=n + 2, precision="fp64")
    try:
        assert g.nslices == 1
        z = g.apply_precond(to_dev(r)).cpu().numpy()
    finally:
        g.close()
    lu = spla.splu(s.H.tocsc())
    for j in range(2):
        exact = s.restrict(lu.solve(s.apply_Q(r[j])))
        assert rel(z[j], exact) <= 1e-11


def test_source_kind_sample_map_and_refusals(case3):
    name, n, omega, m, ref, g64, g32 = case3
    if name != "small":
        pytest.skip("one case suffices")
    from paper_1705_09443_amd import LSSolver, LsError, _lib
    from oracle.stencils import FrequencySamples
    # the sample map through the handle (bit-exact, reading G9)
    km = g64.sample_map()
    assert np.array_equal(km.reshape(-1), FrequencySamples(m, omega, n).index(ref.system.m_ext))
    # a right-hand side g given directly (source kind)
    rng = np.random.default_rng(16)
    gsrc = crand(rng, (1, n, n, n))
    u, info = g64.solve(to_dev(gsrc), "source", 1e-10)
    res = ref.solve_rhs(gsrc[0], 1e-10)
    assert abs(info[0].iterations - res.iterations) <= 1
    assert rel(ref.op.apply_A(u.cpu().numpy()[0]), gsrc[0]) <= 1.01e-10
    # zero medium: g = 0, so u = 0 after no iterations
    z = LSSolver(torch.zeros((n, n, n), dtype=torch.float64, device="cuda"), omega, pml_width=3,
                 layer_thickness=3)
    try:
        uinc = workloads.plane_waves(n, 3, omega, workloads.angle_directions(1, 3, full_turn=False))
        u0, info0 = z.solve(to_dev(uinc), "incident", 1e-8)
        assert info0[0].iterations == 0 and torch.count_nonzero(u0).item() == 0
        with pytest.raises(LsError):
            z.set_kernels(4, 16, 1)
    finally:
        z.close()
    md = torch.as_tensor(m).cuda()
    with pytest.raises(LsError):
        LSSolver(md, omega, pml_width=3, layer_thickness=3, autotune=4)
    with pytest.raises(LsError):
        LSSolver(md, omega, pml_width=3, layer_thickness=0)
