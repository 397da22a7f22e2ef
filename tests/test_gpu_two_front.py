"""GPU parity of the two-front sweep (ls_options.fronts = 2; the first remark
after Algorithm 2, Sec. 2.4; reading G18) against the oracle's two-front
Sweep, through the C ABI: the slice partition, the auxiliary stencil tables
(left of the left front's slices, right of the right front's, both sides of
the middle slice), every slice solve, the preconditioner for every kernel
choice and batch shape, graph replays, and whole solves (P1, P2, P3).

Tolerances as for one front: float64 1e-12, complex64 slice solves and
preconditioner 1e-5 (P5); solves: iteration counts within one of the
two-front oracle's, P1 at 1e-10 with both sides stopped after the oracle's
count, the mixed path within 1e-6 of the oracle's tight solution (P3).
"""
import math
import sys

import numpy as np
import pytest

import oracle
import workloads

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

FP32_BOUND = 1e-5


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


CASES = {
    # name: (n, omega/2pi, b, w); middle slice of 1 line (t = 25), 8 slices per front
    "c0": (63, 4.0, 12, 4),
    # 6 slices of 3 lines per front, a middle slice of 6 lines (t = 18)
    "ragged": (40, 2.5, 6, 3),
    # one slice per front and a middle slice of 3 lines (t = 9)
    "short": (9, 1.0, 3, 4),
}


def medium(name, n):
    if name == "c0":
        return workloads.workload("C0").scaled(n, ppw_omega=CASES[name][1]).medium_array()
    return workloads.gaussian_bump_medium(n, 2, 6, (0.2, 0.8), (0.04, 0.1), (-0.4, 0.4), seed=3)


@pytest.fixture(scope="module", params=list(CASES))
def case(request):
    from paper_1705_09443_amd import LSSolver
    name = request.param
    n, ppw, b, w = CASES[name]
    omega = 2 * math.pi * ppw
    m = medium(name, n)
    say(f"[two fronts {name}] oracle setup n={n} b={b} w={w}")
    ref = oracle.OracleSolver(2, n, omega, m, b, w, fronts=2)
    md = torch.as_tensor(m).cuda()
    g64 = LSSolver(md, omega, b, w, precision="fp64", fronts=2)
    g32 = LSSolver(md, omega, b, w, precision="mixed", fronts=2)
    yield name, n, omega, m, ref, g64, g32
    g64.close()
    g32.close()


def test_partition_and_tables(case):
    name, n, omega, m, ref, g64, g32 = case
    sw = ref.sweep
    assert g64.info.fronts == 2 and g64.nslices == sw.nslices
    L = sw.s.L
    for k in range(sw.nslices):
        lo, hi, naux = g64.slice_bounds(k)
        assert (lo, hi) == sw.bounds[k], k
        assert naux * L == sw.aux_count[k] + sw.aux_count_right[k], k
    a, be, gam, aux = g64.stencils()
    for (q, c2, ks), g in sw.aux_gamma.items():
        assert np.abs(aux[q, c2, ks] - g).max() <= 1e-12
    # a right auxiliary stencil is the left one of the same depth, class and
    # sample with the x1 offsets mirrored
    for (q, c2, ks), g in sw.aux_gamma_right.items():
        lib = aux[q, c2, ks].reshape(3, 3)[::-1, :].reshape(-1)
        assert np.abs(lib - g).max() <= 1e-12, (q, c2, ks)
    say(f"[{name}] {sw.nslices} slices, {len(sw.aux_gamma)} left and {len(sw.aux_gamma_right)} right "
        f"auxiliary stencils")


@pytest.mark.parametrize("nb", [2, 20])
def test_every_slice_solve(case, nb):
    # 2 columns: the vector-ALU slice solves; 20: the matrix cores (two tiles)
    name, n, omega, m, ref, g64, g32 = case
    sw = ref.sweep
    L = sw.s.L
    rng = np.random.default_rng(40 + nb)
    w64 = w32 = 0.0
    for k in range(sw.nslices):
        lo, hi, _ = g64.slice_bounds(k)
        v = crand(rng, (nb, hi - lo + 1, L))
        x = g64.slice_solve(k, to_dev(v)).cpu().numpy()
        x32 = g32.slice_solve(k, to_dev(v, torch.complex64)).cpu().numpy()
        for j in range(nb):
            r = sw.solve_slice(k, v[j].reshape(-1))
            w64 = max(w64, rel(x[j].reshape(-1), r))
            w32 = max(w32, rel(x32[j].reshape(-1), r))
    say(f"[{name}] every slice, batch {nb}: worst fp64 {w64:.2e}, fp32 {w32:.2e}")
    assert w64 <= 1e-12 and w32 <= FP32_BOUND


@pytest.mark.parametrize("nb", [1, 3, 6, 17])
def test_preconditioner_every_kernel_choice(case, nb):
    name, n, omega, m, ref, g64, g32 = case
    rng = np.random.default_rng(60 + nb)
    r = crand(rng, (nb, n, n))
    zr = [ref.precondition(r[j]) for j in range(nb)]
    choices = [(sk, ik) for sk in (1, 4, 8, 16) for ik in ((0, 1) if nb <= 4 else (1,))]
    if nb == 17:
        choices = [(0, 0)]          # the defaults
    try:
        for sk, ik in choices:
            for g in (g64, g32):
                g.set_kernels(nb, sk, ik)
            z = g64.apply_precond(to_dev(r)).cpu().numpy()
            z32 = g32.apply_precond(to_dev(r, torch.complex64)).cpu().numpy()
            e64 = max(rel(z[j], zr[j]) for j in range(nb))
            e32 = max(rel(z32[j], zr[j]) for j in range(nb))
            say(f"[{name}] P r, batch {nb}, slice kernel {sk}, interface kernel {ik}: fp64 {e64:.2e}, fp32 {e32:.2e}")
            assert e64 <= 1e-12 and e32 <= FP32_BOUND
    finally:
        for g in (g64, g32):
            g.set_kernels(nb, 0, 0)


def test_graph_replays_agree(case):
    # both fronts' recurrences are branches of one captured graph: replays
    # with eager work and synchronisations in between all give the first result
    name, n, omega, m, ref, g64, g32 = case
    rng = np.random.default_rng(11)
    r = to_dev(crand(rng, (9, n, n)))
    outs = []
    for _ in range(4):
        outs.append(g64.apply_precond(r).cpu().numpy())
        g64.apply_A(r)
        torch.cuda.synchronize()
    zr = [ref.precondition(r[j].cpu().numpy()) for j in range(9)]
    for z in outs:
        assert max(rel(z[j], zr[j]) for j in range(9)) <= 1e-12
        assert np.array_equal(z, outs[0])


def test_solves(case):
    from paper_1705_09443_amd import LSSolver
    name, n, omega, m, ref, g64, g32 = case
    b, w = CASES[name][2], CASES[name][3]
    uinc = workloads.plane_waves(n, 2, omega, workloads.angle_directions(2, 2))
    u, info = g64.solve(to_dev(uinc), "incident", 1e-6)
    u32, info32 = g32.solve(to_dev(uinc), "incident", 1e-6)
    u, u32 = u.cpu().numpy(), u32.cpu().numpy()
    for j in range(2):
        g = ref.op.rhs_incident(uinc[j])
        res = ref.solve_rhs(g, 1e-6)
        tight = ref.solve_rhs(g, 1e-12).x
        k = res.iterations
        with LSSolver(torch.as_tensor(m).cuda(), omega, b, w, precision="fp64", fronts=2, max_iters=k) as sk:
            uk, ik = sk.solve(to_dev(uinc[j][None]), "incident", 1e-300, allow_noconv=True)
        assert ik[0].iterations == k
        e1 = rel(uk.cpu().numpy()[0], ref.solve_rhs(g, 1e-300, max_iters=k).x)
        e3, e_ref = rel(u32[j], tight), rel(res.x, tight)
        say(f"[{name}] rhs {j}: iterations fp64 {info[j].iterations}, mixed {info32[j].iterations}, oracle {k}; "
            f"P1 after {k} steps {e1:.2e}; P3 at tol 1e-6 {e3:.2e} (oracle float64 {e_ref:.2e})")
        assert abs(info[j].iterations - k) <= 1 and abs(info32[j].iterations - k) <= 1      # P2
        assert info[j].converged and info32[j].converged
        assert rel(ref.op.apply_A(u[j]), g) <= 1.01e-6 and rel(ref.op.apply_A(u32[j]), g) <= 1.01e-6
        assert e1 <= 1e-10                                                                   # P1
        assert e3 <= max(1e-6, 3 * e_ref)                                                    # P3


def test_refusals():
    # two fronts need a 2D grid and the interface schedule
    from paper_1705_09443_amd import LSSolver, _lib
    n = 15
    md = torch.zeros((n, n), dtype=torch.float64, device="cuda")
    with pytest.raises(_lib.LsError) as ei:
        LSSolver(md, 2 * math.pi, 4, 4, fronts=2, schedule="sequential")
    assert ei.value.status == _lib.LS_E_INVALID and "fronts" in str(ei.value)
    with pytest.raises(_lib.LsError):
        LSSolver(md, 2 * math.pi, 4, 4, fronts=3)
    m3 = torch.zeros((9, 9, 9), dtype=torch.float64, device="cuda")
    with pytest.raises(_lib.LsError):
        LSSolver(m3, 2 * math.pi, 3, 3, fronts=2, schedule="sequential")
