"""Benchmark: unknowns x right-hand sides solved per second to a 1e-6 relative
residual on one MI355X, mixed precision with a batch of 64 incident waves,
beside the plain float64 form with one incident wave.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

One step = one ls_solve of the whole batch: every FGMRES iteration applies
the preconditioner (Q stencil, slice solves, interface recurrences, slice
solves, extraction) and the FFT operator to every right-hand side still
running, until every right-hand side meets the tolerance. Inputs are resident
in HBM before the timed region; setup (Algorithm 1) is timed separately and
excluded. The batched setup is autotuned (the layer thickness and the kernel
choice per batch size timed on the device for this batch; it keeps w = 4,
132 ms against 146 for w = 5); its setup time includes the tuning.
--no-autotune keeps the workload's w = 4 and the default kernel table (the
configuration of the committed profiles: under a kernel tracer the tuner's
ranking of w = 4 and w = 5 flips).

A 3D leg (object "c3") times the 127^3 workload the same way: four incident
waves, mixed precision, the slab-by-slab sweep captured as one graph; its
roofline is the sweep's factor bytes per apply over the apply's event-timed
duration.

Prints one JSON line. Besides the contract fields it carries the float64
form (same medium, one wave), per-kind kernel times from HIP events recorded
on the library's stream inside the timed region, rooflines by the method's
algorithmic bytes (the sweep apply as "roofline"; the FFT convolution and the
Q stencil under "roofline_parts", with the interface form's dense map
products as an overhead figure), the CPU oracle timed on a bounded sample of
the same workload (one of the 64 right-hand sides, solved in full), and the
errors of the GPU results on that wave against the oracle.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "unknowns*RHS solved/s to 1e-6 residual, mixed+batched vs plain FP64 on 1 GPU"
HBM_PEAK_GBS = 8000.0


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=3)
    p.add_argument("--warmup", type=int, default=1)
    p.add_argument("--fp64-steps", type=int, default=2)
    p.add_argument("--n", type=int, default=None, help="grid override (default: the workload's)")
    p.add_argument("--nrhs", type=int, default=None)
    p.add_argument("--no-fp64", action="store_true")
    p.add_argument("--no-cpu", action="store_true")
    p.add_argument("--no-accuracy", action="store_true",
                   help="skip the oracle's tol-1e-12 solve that the errors of the mixed results are measured against")
    p.add_argument("--no-3d", action="store_true", help="skip the 3D leg (127^3, four waves, mixed)")
    p.add_argument("--steps-3d", type=int, default=2)
    p.add_argument("--no-adjoint", action="store_true",
                   help="skip the adjoint leg (511^2, 32 waves, mixed: forward solve plus adjoint solve)")
    p.add_argument("--steps-adjoint", type=int, default=3)
    p.add_argument("--no-direct", action="store_true",
                   help="skip the direct-scheme leg (Sec. 4: 2047^2 point source at 3 points per wavelength)")
    p.add_argument("--steps-direct", type=int, default=2)
    p.add_argument("--block-size", type=int, default=64,
                   help="block flexible GMRES leg: columns per block (0: skip the leg)")
    p.add_argument("--steps-block", type=int, default=2)
    p.add_argument("--no-autotune", action="store_true",
                   help="batched leg at the workload's w = 4 and the default kernels instead of autotuned ones")
    p.add_argument("--fronts", type=int, default=2, choices=(1, 2),
                   help="sweeping fronts of the 2D legs: 2 (default) from both ends toward a middle slice, "
                        "as the paper's 2D experiments; 1 the single front of Algorithms 1-2")
    p.add_argument("--copy-gib", type=float, default=0.0,
                   help="first run one plain device copy of this many GiB (a known-size dispatch that "
                        "calibrates hardware byte counters in a profile of this command)")
    return p.parse_args()


def fft_len(n: int) -> int:
    P = 1
    while P < 2 * (n + 1):
        P <<= 1
    return P


def sweep_method_bytes(solver, cbytes: int):
    """Algorithmic bytes of one preconditioner sweep (Algorithm 2) by the
    method's count: the 2l-1 slice solves (every slice forward, every slice but
    the last backward) each read their factors once, 2 L t^2 complex values
    for a t-line subproblem, shared by the whole batch; per right-hand-side
    column each solve reads its slice right-hand side and writes its field,
    (2 w_k + 2 t) L complex values (w_k lines of D_k). Returns (shared bytes,
    bytes per column)."""
    L, nl = solver.L, solver.nslices
    shared = col = 0.0
    for k in range(nl):
        lo, hi, naux = solver.slice_bounds(k)
        tw = hi - lo + 1
        t = tw + naux
        solves = 2 if k < nl - 1 else 1
        shared += solves * 2.0 * L * t * t * cbytes
        col += solves * (2.0 * tw + 2.0 * t) * L * cbytes
    return shared, col


def fft_method_bytes(n: int, cbytes: int):
    """One zero-padded FFT convolution: read x and m, write y ((2s + s/2) N with
    a float32 m), and the three passes over the n x P row transforms of the
    pruned two-dimensional FFT (4 n P s); the (P/2+1)^2 spectrum once per
    launch. Returns (shared, per column)."""
    P = fft_len(n)
    N = n * n
    return float((P // 2 + 1) ** 2 * cbytes), float((2 * cbytes + cbytes / 2) * N + 4 * n * P * cbytes)


def stencil_method_bytes(n: int, L: int, cbytes: int):
    """Q: read the interior field, write the extended one (s N + s N_ext) per column."""
    return 0.0, float(cbytes * (n * n + L * L))


def interface_map_flops(solver):
    """The interface form's own work, beyond the method's count: 3l - 5 dense
    L x L complex products per column and apply (the lambda chain, the fused P
    terms and the mu chain), 8 flop per complex multiply-add, and the maps'
    bytes once per apply."""
    L, nl = solver.L, solver.nslices
    steps = max(0, 3 * nl - 5)
    return 8.0 * steps * L * L, float(steps * L * L)


# HBM bytes per launch from hardware counters (FETCH_SIZE + WRITE_SIZE, each
# calibrated on a plain copy of known size) for the 1023^2 64-wave mixed
# workload at w = 4 with two fronts and the default kernel table (the tuned
# run keeps w = 4 and may pick other kernels at some batch sizes), keyed by
# (part, complex bytes of the part's launches, w, fronts); valid only for the
# kernels as they were when measured (profiles/c2_mixed_64rhs_hbm_counters.md).
# Per launch at the run's mean columns per launch: sweep 56.3 (one apply:
# every slice-solve, interface-product and coupling kernel), FFT 56.3
# (complex64 launches) and 32 (the complex128 launches of the true
# residuals), Q 56.3.
# Each entry: (bytes per launch, mean columns per launch of the counter run);
# a run with another mean is charged the shared bytes of the method's count
# plus the measured per-column remainder times its own mean.
MEASURED_TRAFFIC = {
    ("sweep", 8, 4, 2): (2.2748e10, 56.29),
    ("fft_convolve", 8, 4, 2): (5.8404e9, 56.29),
    ("fft_convolve_c128", 16, 4, 2): (6.2019e9, 32.0),
    ("stencil_Q", 8, 4, 2): (1.8362e9, 56.29),
}

# published MI355X dense matrix-core peaks (TFLOP/s): fp32 157.3, fp64 78.6
MFMA_PEAK = {8: 157.3, 16: 78.6}


def hbm_roofline(label, formula, shared, per_col, cols, avg_ms, traffic=None):
    nbytes = shared + per_col * cols
    achieved = nbytes / (avg_ms * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": traffic, "kernel": label, "avg_launch_ms": avg_ms,
            "mean_columns_per_launch": cols, "algorithmic_bytes_per_launch": nbytes, "formula": formula}


def rooflines(solver, prof, cbytes: int, n: int, fronts: int = 1):
    """The sweep apply (the dominant part of the step), the FFT convolution and
    the Q stencil against the HBM peak, each from the method's algorithmic
    bytes (sweep_method_bytes, fft_method_bytes, stencil_method_bytes) over the
    mean event-timed duration of one launch; plus the interface form's dense
    map products as an overhead figure against the matrix-core peak.

    A sweep "launch" is one preconditioner apply on the main stream: its two
    slice-solve phases and its interface graph (recurrences and coupling);
    the last slice's solves run on the second stream, overlapped."""
    L = solver.L
    out = {}

    def traffic(part, shared, cols, cb=cbytes):
        if n != 1023:
            return None
        t = MEASURED_TRAFFIC.get((part, cb, solver.layer_thickness, fronts))
        if t is None:
            return None
        return shared + (t[0] - shared) * cols / t[1]

    it = prof.get("interface")
    ss = prof.get("slice_solves")
    if it and ss:
        applies = it[0]
        cols = it[2] / applies
        avg = (it[1] + ss[1]) / applies
        sh, pc = sweep_method_bytes(solver, cbytes)
        out["sweep"] = hbm_roofline(
            "sweep apply (Algorithm 2: slice solves, phases A and C, plus the interface graph)",
            "sum over the 2l-1 slice solves of 2 L t^2 s (factors) + columns x (2 w_k + 2 t) L s",
            sh, pc, cols, avg, traffic("sweep", sh, cols))
        fl, mb = interface_map_flops(solver)
        t_if = it[1] / applies
        out["interface_dense_maps"] = {
            "note": "work of the interface form beyond the method's count (not a roofline of the method)",
            "flops_per_apply": fl * cols, "map_bytes_per_apply": mb * cbytes, "avg_ms": t_if,
            "achieved_tflops": fl * cols / (t_if * 1e-3) / 1e12, "mfma_peak_tflops": MFMA_PEAK[cbytes],
            "frac_of_mfma_peak": fl * cols / (t_if * 1e-3) / 1e12 / MFMA_PEAK[cbytes]}
    # operator applies in each precision: complex64 (the Arnoldi steps of the
    # mixed path) and complex128 (true residuals, the float64 path)
    for part, cb in (("fft_convolve", 8), ("fft_convolve_c128", 16)):
        f = prof.get(part)
        if f and f[0]:
            sh, pc = fft_method_bytes(n, cb)
            out[part] = hbm_roofline(
                f"FFT convolution, complex{8 * cb} launches (row forward, column convolve, row inverse)",
                "(P/2+1)^2 s + columns x ((2s + s/2) N + 4 n P s)", sh, pc, f[2] / f[0], f[1] / f[0],
                traffic(part, sh, f[2] / f[0], cb))
    q = prof.get("stencil_Q")
    if q:
        sh, pc = stencil_method_bytes(n, L, cbytes)
        out["stencil_Q"] = hbm_roofline(
            "Q stencil", "columns x (s N + s N_ext)", sh, pc, q[2] / q[0], q[1] / q[0],
            traffic("stencil_Q", sh, q[2] / q[0]))
        # the mixed Arnoldi step hands Q the float64 basis vector: 16-byte reads
        out["stencil_Q"]["frac_at_io_width"] = (
            (q[2] / q[0]) * (16.0 * n * n + cbytes * L * L) / (q[1] / q[0] * 1e-3) / 1e9 / HBM_PEAK_GBS)
    return out


def sweep3_bytes(solver, cbytes: int) -> float:
    """Factor bytes one 3D preconditioner apply streams: every slab solve reads
    S_j^{-1} (nb x nb complex) once per block in its forward pass (L blocks)
    and once more in its backward pass (L - 1 blocks); the sweep solves every
    slab forward and every slab but the last backward."""
    L, b, w, n = solver.L, solver.pml_width, solver.layer_thickness, solver.n
    total = 0.0
    for k in range(solver.nslices):
        lo, hi, naux = solver.slice_bounds(k)
        nb = (hi - lo + 1 + naux) * L
        per = (2 * L - 1) * nb * nb * cbytes
        total += per * (2 if k < solver.nslices - 1 else 1)
    return total


def leg_3d(args, dev):
    """The 3D workload (127^3, 16 bumps, four plane waves, mixed precision,
    b = 8, w = 4): setup timed apart, then whole solves; the sweep's roofline
    from its event-timed graph launches."""
    import torch
    import workloads
    from paper_1705_09443_amd import LSSolver
    wl = workloads.workload("C3")
    n = wl.n
    m = torch.as_tensor(wl.medium_array(), device=dev)
    uinc = torch.as_tensor(wl.incident(), device=dev)
    t0 = time.perf_counter()
    s3 = LSSolver(m, wl.omega, wl.pml_width, wl.layer_thickness, precision="mixed", restart=wl.restart,
                  schedule="sequential")
    torch.cuda.synchronize()
    setup = time.perf_counter() - t0
    print(f"[bench] 3D setup {setup:.2f} s (n={n}, slabs={s3.nslices})", file=sys.stderr, flush=True)
    u, info = s3.solve(uinc, "incident", wl.tol)  # warm-up (graph capture)
    torch.cuda.synchronize()
    s3.profile(True)
    t0 = time.perf_counter()
    for i in range(args.steps_3d):
        u, info = s3.solve(uinc, "incident", wl.tol)
    torch.cuda.synchronize()
    t = (time.perf_counter() - t0) / args.steps_3d
    s3.profile(False)
    prof = s3.profile_read()
    assert all(x.converged and x.rel_residual <= wl.tol for x in info), "a 3D right-hand side did not converge"
    launches, total_ms, cols = prof["slice_solves"]
    avg_ms = total_ms / launches
    nbytes = sweep3_bytes(s3, 8)
    achieved = nbytes / (avg_ms * 1e-3) / 1e9
    out = {"value": wl.nrhs * n ** 3 / t, "unit": "unknowns*RHS/s", "ms_per_step": t * 1e3,
           "steps": args.steps_3d, "setup_s": setup,
           "iterations": [x.iterations for x in info],
           "config": {"workload": (f"3D {n}^3, omega=2pi*{wl.ppw_omega:g}, 16 Gaussian bumps (seed 0), "
                                   f"{wl.nrhs} plane waves, mixed precision, b={wl.pml_width}, "
                                   f"w={wl.layer_thickness}, restart {wl.restart}, tol {wl.tol}"),
                      "n": n, "nrhs": wl.nrhs},
           "kernels": {k: {"launches": v[0], "avg_ms": v[1] / v[0]} for k, v in prof.items()},
           "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": achieved / HBM_PEAK_GBS, "traffic": None, "kernel": "sweep (slab solves)",
                        "avg_launch_ms": avg_ms, "algorithmic_bytes_per_launch": nbytes,
                        "note": ("bytes of this build's slab factors (dense block inverses, every block "
                                 "streamed once per pass), not the method's count: the paper factors each "
                                 "slab by nested dissection, whose apply streams far fewer bytes; the figure "
                                 "rates the streaming of the factors this build keeps")}}
    s3.close()
    return out


def leg_adjoint(args, dev):
    """The adjoint workload (511^2, 16 bumps, 32 plane waves, mixed precision):
    one step is one gradient of the receiver misfit, that is the forward
    solve (ls_solve) and the adjoint solve with the gradient product
    (ls_adjoint), both to 1e-10. The receiver residual comes from the
    warm-up's field against data from a second medium (bump seed 1), formed
    before the timed region; the timed region holds only the two C-ABI calls
    per step."""
    import torch
    import workloads
    from paper_1705_09443_amd import LSSolver
    wl = workloads.workload("C4")
    n, tol = wl.n, 1e-10
    uinc = torch.as_tensor(wl.incident(), device=dev)
    rec = torch.as_tensor(workloads.circle_receivers(n, 0.45), device=dev)
    with LSSolver(torch.as_tensor(wl.medium_array(seed=1), device=dev), wl.omega, wl.pml_width,
                  wl.layer_thickness, precision="mixed") as sd:
        ud, _ = sd.solve(uinc, "incident", tol)
        data = ud[:, rec].clone()
        del ud
    t0 = time.perf_counter()
    s = LSSolver(torch.as_tensor(wl.medium_array(), device=dev), wl.omega, wl.pml_width, wl.layer_thickness,
                 precision="mixed")
    torch.cuda.synchronize()
    setup = time.perf_counter() - t0
    u, info = s.solve(uinc, "incident", tol)  # warm-up: graphs, and the residual
    r = torch.zeros_like(u)
    r[:, rec] = u[:, rec] - data
    g, ginfo = s.adjoint(r, tol)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps_adjoint):
        u, info = s.solve(uinc, "incident", tol)
        g, ginfo = s.adjoint(r, tol)
    torch.cuda.synchronize()
    t = (time.perf_counter() - t0) / args.steps_adjoint
    assert all(x.converged for x in info) and all(x.converged for x in ginfo), "an adjoint-leg solve did not converge"
    assert bool(torch.isfinite(g).all()), "non-finite gradient"
    s.close()
    return {"value": wl.nrhs * n * n / t, "unit": "unknowns*RHS/s (forward + adjoint solve per RHS)",
            "ms_per_step": t * 1e3, "steps": args.steps_adjoint, "setup_s": setup,
            "iterations": {"forward": [x.iterations for x in info], "adjoint": [x.iterations for x in ginfo]},
            "config": {"workload": (f"2D {n}^2, omega=2pi*{wl.ppw_omega:g}, 16 Gaussian bumps (seed 0), "
                                    f"{wl.nrhs} plane waves, receivers on the circle r=0.45, data from bump "
                                    f"seed 1, mixed precision, b={wl.pml_width}, w={wl.layer_thickness}, "
                                    f"restart {wl.restart}, tol {tol}: one gradient = ls_solve + ls_adjoint"),
                       "n": n, "nrhs": wl.nrhs}}


def block_gemm_flops(N: int, b: int, s: int):
    """Algorithmic float64 flops of block GMRES's GEMMs for one block of b
    columns over one cycle of s block steps (8 real flops per complex
    multiply-add): Gram products (N x K)^H (N x b) of two classical passes per
    step (K = j b at step j) plus the two Cholesky-QR Gram matrices of every
    block QR (s + 1 of them, the initial one included); updates W -= V C of
    both passes, the two triangular multiplies of every block QR and
    X += Z Y at the cycle's end."""
    gram = 8.0 * N * b * b * (s * (s + 1) + 2 * (s + 1))
    update = 8.0 * N * b * b * (s * (s + 1) + 2 * (s + 1) + s)
    return gram, update


def leg_block(args, dev, md, wl2, w: int):
    """Block flexible GMRES (one shared block Krylov space per group of
    columns) on the headline workload: the same medium, waves, layer thickness
    and precision, restart 30 block steps, groups of args.block_size columns.
    Reports the time per solve and the block steps, and for the GEMMs of the
    block Gram-Schmidt and QR the float64 rate against the matrix-core peak
    (78.6 TFLOP/s)."""
    import torch
    from paper_1705_09443_amd import LSSolver
    bs = args.block_size
    uinc = torch.as_tensor(wl2.incident(), device=dev)
    s = LSSolver(md, wl2.omega, wl2.pml_width, w, precision="mixed", restart=min(30, 2048 // bs),
                 fronts=args.fronts, block_size=bs)
    u, info = s.solve(uinc, "incident", wl2.tol)  # warm-up
    torch.cuda.synchronize()
    s.profile(True)
    t0 = time.perf_counter()
    for _ in range(args.steps_block):
        u, info = s.solve(uinc, "incident", wl2.tol)
    torch.cuda.synchronize()
    t = (time.perf_counter() - t0) / args.steps_block
    s.profile(False)
    prof = s.profile_read()
    s.close()
    assert all(x.converged and x.rel_residual <= wl2.tol for x in info), "a block-GMRES column did not converge"
    its = [x.iterations for x in info]
    N = wl2.n * wl2.n
    out = {"value": wl2.nrhs * N / t, "unit": "unknowns*RHS/s", "ms_per_step": t * 1e3, "steps": args.steps_block,
           "block_size": bs, "block_steps": {"min": min(its), "max": max(its)},
           "kernels_ms_per_solve": {k: v[1] / args.steps_block for k, v in prof.items()},
           "config": {"workload": f"the headline workload with block flexible GMRES, groups of {bs} columns, "
                                  f"restart {min(30, 2048 // bs)} block steps"}}
    if min(its) == max(its) and wl2.nrhs % bs == 0:
        # one cycle per block, every block the same number of steps: the
        # flop counts hold exactly
        nb = wl2.nrhs // bs
        g, upd = block_gemm_flops(N, bs, its[0])
        for key, fl in (("block_gram", g * nb), ("block_update", upd * nb)):
            if key in prof:
                ms = prof[key][1] / args.steps_block
                out[key] = {"bound": "mfma", "achieved": fl / (ms * 1e-3) / 1e12, "peak": 78.6, "unit": "TFLOP/s",
                            "frac": fl / (ms * 1e-3) / 1e12 / 78.6, "flops_per_solve": fl, "ms_per_solve": ms}
    return out


def leg_direct(args, dev):
    """The sparsifying stencils as a direct Helmholtz scheme (Sec. 4): a point
    source at the centre of the largest grid the library sets up, 2047^2 at 3
    points per wavelength (omega/2pi = 682.7), m = 0, b = 12, two fronts,
    mixed precision; one step is one ls_solve_H of H u = beta^* f to a 1e-8
    residual. Reports the far-field phase error against the Green's function
    (the paper: about 2.3e-4 per wavelength of distance at 3 points per
    wavelength), computed from the field after the timed region."""
    import math
    import numpy as np
    import torch
    from paper_1705_09443_amd import LSSolver
    n, b, ppw = 2047, 12, 3
    omega = 2 * math.pi * (n + 1) / ppw
    h = 1.0 / (n + 1)
    f = torch.zeros((1, n, n), dtype=torch.complex128, device=dev)
    c = (n + 1) // 2 - 1
    f[0, c, c] = 1.0 / (h * h)
    t0 = time.perf_counter()
    s = LSSolver(torch.zeros((n, n), dtype=torch.float64, device=dev), omega, b, 4, precision="mixed", fronts=2)
    rhs = s.apply_B(f, "fp64")
    torch.cuda.synchronize()
    setup = time.perf_counter() - t0
    u, info = s.solve_H(rhs, 1e-8)  # warm-up (graph capture, workspaces)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps_direct):
        u, info = s.solve_H(rhs, 1e-8)
    torch.cuda.synchronize()
    t = (time.perf_counter() - t0) / args.steps_direct
    s.close()
    assert info[0].converged, "the direct scheme's solve did not converge"
    # phase of u / G over the interior, far field r >= 0.6 and the corners
    from scipy.special import hankel1
    ui = u[0, b + 1:b + 1 + n, b + 1:b + 1 + n].cpu().numpy()
    x = np.arange(1, n + 1) * h - 0.5
    r = np.sqrt(x[:, None] ** 2 + x[None, :] ** 2)
    r[c, c] = 1.0
    dphi = np.angle(ui * np.conj(0.25j * hankel1(0, omega * r))) / (2 * math.pi)
    far = r >= 0.6
    shift = float(np.mean(dphi[far]))
    per = shift / float(np.mean(r[far] * omega / (2 * math.pi)))
    corner = float(np.mean([dphi[0, 0], dphi[0, -1], dphi[-1, 0], dphi[-1, -1]]))
    return {"value": n * n / t, "unit": "unknowns/s (one point source)", "ms_per_step": t * 1e3,
            "steps": args.steps_direct, "setup_s": setup, "iterations": info[0].iterations,
            "phase_error": {"far_field_shift_wavelengths": shift, "per_wavelength_of_distance": per,
                            "corner_shift_wavelengths": corner,
                            "paper": "about 1/6 at the corners of a 1024-wavelength square: 2.3e-4 per wavelength"},
            "config": {"workload": (f"direct Helmholtz scheme (Sec. 4), {n}^2, omega=2pi*{omega / (2 * math.pi):.1f} "
                                    f"({ppw} points per wavelength), point source at the centre, m = 0, b={b}, "
                                    f"w=4, two fronts, mixed precision, ls_solve_H to 1e-8"), "n": n}}


def cpu_baseline(wl, m, uinc, mixed0, fp64, accuracy: bool, fronts: int = 1):
    """The float64 oracle on the machine's host cores: its setup (not timed into
    the value, like the GPU's), then one full FGMRES solve of the first
    incident wave of the batch (theta = 0) at the full grid, timed.

    The same leg states the error of the GPU results against the oracle on
    that wave: the float64 GPU solve against the oracle's solve at the same
    tolerance (their iteration counts beside it: at equal counts this is the
    P1 comparison), and the mixed batched GPU solve against the oracle's
    tol-1e-12 solution (P3; the oracle's own tol-1e-6 solution's distance to
    it beside it, the spread any tol-1e-6 solve has)."""
    import numpy as np
    cores = len(os.sched_getaffinity(0))
    os.environ.setdefault("OMP_NUM_THREADS", str(cores))
    try:
        import threadpoolctl
        threadpoolctl.threadpool_limits(cores)
    except Exception:
        pass
    import oracle
    t0 = time.perf_counter()
    s = oracle.OracleSolver(2, wl.n, wl.omega, m, wl.pml_width, wl.layer_thickness, workers=cores,
                            fronts=fronts)
    t_setup = time.perf_counter() - t0
    t0 = time.perf_counter()
    res = s.solve_incident(uinc[:1], tol=wl.tol)[0]
    t_solve = time.perf_counter() - t0
    iters = res.iterations
    base = {
        "value": wl.n ** 2 / t_solve,
        "unit": "unknowns*RHS/s",
        "cores": cores,
        "kind": "oracle",
        "sample": (f"1 of the {wl.nrhs} right-hand sides (theta=0), full {wl.n}^2 grid, solved to {wl.tol} by the "
                   f"float64 oracle (FGMRES, Algorithm-2 sweep with SuperLU slice factors, scipy FFT operator) in "
                   f"{t_solve:.1f} s, {iters} iterations; oracle setup {t_setup:.1f} s excluded like the GPU "
                   f"setup; SuperLU single-threaded, FFT and BLAS on {cores} threads"),
    }
    rel = lambda a, b: float(np.linalg.norm(a - b) / np.linalg.norm(b))
    err = {"wave": "theta=0", "oracle_iterations_tol_1e-6": iters}
    if fp64 is not None:
        err["fp64_1rhs_vs_oracle_same_tol"] = {"rel_l2": rel(fp64[0], res.x), "gpu_iterations": fp64[1],
                                               "oracle_iterations": iters}
    if accuracy:
        g = s.op.rhs_incident(uinc[0])
        tight = s.solve_rhs(g, 1e-12)
        err["mixed_64rhs_vs_oracle_tol_1e-12"] = {"rel_l2": rel(mixed0[0], tight.x), "gpu_iterations": mixed0[1],
                                                  "oracle_tol_1e-6_vs_tol_1e-12": rel(res.x, tight.x)}
        if fp64 is not None:
            err["fp64_1rhs_vs_oracle_tol_1e-12"] = rel(fp64[0], tight.x)
    return base, err


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path (its natural shard "
              "would be the incident directions across GPUs). Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)
    import dataclasses
    import torch
    import workloads
    from paper_1705_09443_amd import LSSolver

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    if args.copy_gib > 0:
        nel = int(args.copy_gib * 2 ** 30) // 8
        src = torch.ones(nel, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        print(f"[bench] calibration copy of {nel * 8} bytes", file=sys.stderr, flush=True)
        del src, dst
    wl2 = workloads.workload("C2")
    wl1 = workloads.workload("C1")
    if args.n:
        wl2 = wl2.scaled(args.n)
        wl1 = wl1.scaled(args.n)
    if args.nrhs:
        wl2 = dataclasses.replace(wl2, nrhs=args.nrhs)
    m = wl2.medium_array()
    md = torch.as_tensor(m, device=dev)
    n = wl2.n
    N = n * n

    # ---- mixed precision, batched (the headline) ----
    uinc2 = torch.as_tensor(wl2.incident(), device=dev)
    t0 = time.perf_counter()
    if args.no_autotune:
        mixed = LSSolver(md, wl2.omega, wl2.pml_width, wl2.layer_thickness, precision="mixed",
                         restart=wl2.restart, fronts=args.fronts)
    else:
        # w and the kernel choice per batch size timed on the device for this batch
        mixed = LSSolver(md, wl2.omega, wl2.pml_width, None, precision="mixed", restart=wl2.restart,
                         autotune=wl2.nrhs, fronts=args.fronts)
    torch.cuda.synchronize()
    setup_mixed = time.perf_counter() - t0
    wl2 = dataclasses.replace(wl2, layer_thickness=mixed.layer_thickness)
    tuning = mixed.tuning()
    print(f"[bench] mixed setup {setup_mixed:.2f} s (n={n}, w={mixed.layer_thickness}, slices={mixed.nslices})",
          file=sys.stderr, flush=True)
    for i in range(args.warmup):
        u, info = mixed.solve(uinc2, "incident", wl2.tol)
        print(f"[bench] warmup {i}: iterations {sorted(set(x.iterations for x in info))}", file=sys.stderr,
              flush=True)
    torch.cuda.synchronize()
    mixed.profile(True)
    t0 = time.perf_counter()
    for i in range(args.steps):
        u, info = mixed.solve(uinc2, "incident", wl2.tol)
        print(f"[bench] step {i} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t_mixed = (time.perf_counter() - t0) / args.steps
    mixed.profile(False)
    prof = mixed.profile_read()
    iters = [x.iterations for x in info]
    assert all(x.converged and x.rel_residual <= wl2.tol for x in info), "a right-hand side did not converge"
    value = wl2.nrhs * N / t_mixed
    roofs = rooflines(mixed, prof, 8, n, args.fronts)
    roof = roofs.get("sweep")
    kernels = {k: {"launches": v[0], "avg_ms": v[1] / v[0], "columns_per_launch": v[2] / v[0],
                   "share_of_step": v[1] / (t_mixed * 1e3 * args.steps)} for k, v in prof.items()}

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "unknowns*RHS/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": t_mixed * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64 applies (f32) in a c128 (f64) FGMRES loop",
        "data": "synthetic: seeded Gaussian-bump medium and plane waves",
        "config": {"workload": (f"2D {n}^2, omega=2pi*{wl2.ppw_omega:g}, 32 Gaussian bumps (seed 0), {wl2.nrhs} "
                                f"plane waves theta_j=2pi j/{wl2.nrhs}, mixed precision, b={wl2.pml_width}, "
                                f"w={wl2.layer_thickness}{'' if args.no_autotune else ' (autotuned)'}, "
                                f"{args.fronts} sweeping front{'s' if args.fronts > 1 else ''}, "
                                f"restart {wl2.restart}, tol {wl2.tol}"),
                   "n": n, "nrhs": wl2.nrhs, "omega": wl2.omega, "precision": "mixed"},
        "iterations": {"min": min(iters), "max": max(iters), "mean": sum(iters) / len(iters)},
        "setup_s": {"mixed": setup_mixed},
        "autotune": None if args.no_autotune else {
            "layers": [{"w": r[0], "slices": r[1], "iterations": r[2], "setup_ms": r[3], "solve_ms": r[4]}
                       for r in tuning["layers"]],
            "kernels": [{"nrhs": r[0], "slice_kernel": r[1], "iface_kernel": r[2], "apply_ms": r[3]}
                        for r in tuning["kernels"]]},
        "kernels": kernels,
        "roofline": roof,
        "roofline_parts": {k: v for k, v in roofs.items() if k != "sweep"},
    }
    u_mixed0 = u[0].cpu().numpy()
    mixed.close()
    del mixed

    # ---- block flexible GMRES on the same workload ----
    if args.block_size > 1:
        out["block_gmres"] = leg_block(args, dev, md, wl2, wl2.layer_thickness)
        print(f"[bench] block GMRES ({args.block_size} columns per block) {out['block_gmres']['ms_per_step']:.1f} ms",
              file=sys.stderr, flush=True)

    # ---- plain float64, one wave ----
    u_f64 = None
    if not args.no_fp64:
        uinc1 = torch.as_tensor(wl1.incident(), device=dev)
        t0 = time.perf_counter()
        f64 = LSSolver(md, wl1.omega, wl1.pml_width, wl1.layer_thickness, precision="fp64", restart=wl1.restart,
                       fronts=args.fronts)
        torch.cuda.synchronize()
        setup_f64 = time.perf_counter() - t0
        print(f"[bench] fp64 setup {setup_f64:.2f} s", file=sys.stderr, flush=True)
        u1, info1 = f64.solve(uinc1, "incident", wl1.tol)  # warm-up (graph capture)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(args.fp64_steps):
            u1, info1 = f64.solve(uinc1, "incident", wl1.tol)
        torch.cuda.synchronize()
        t_f64 = (time.perf_counter() - t0) / args.fp64_steps
        print(f"[bench] fp64 solve {t_f64 * 1e3:.1f} ms", file=sys.stderr, flush=True)
        v64 = wl1.nrhs * N / t_f64
        out["fp64"] = {"value": v64, "ms_per_step": t_f64 * 1e3, "iterations": info1[0].iterations,
                       "rel_residual": info1[0].rel_residual, "setup_s": setup_f64, "nrhs": wl1.nrhs}
        u_f64 = (u1[0].cpu().numpy(), info1[0].iterations)
        out["ratio_vs_fp64"] = value / v64
        f64.close()
        del f64

    # ---- 3D ----
    if not args.no_3d:
        out["c3"] = leg_3d(args, dev)
        print(f"[bench] 3D solve {out['c3']['ms_per_step']:.1f} ms", file=sys.stderr, flush=True)

    # ---- adjoint (gradient) ----
    if not args.no_adjoint:
        out["c4_adjoint"] = leg_adjoint(args, dev)
        print(f"[bench] adjoint gradient {out['c4_adjoint']['ms_per_step']:.1f} ms", file=sys.stderr, flush=True)

    # ---- the sparsifying stencils as a direct Helmholtz scheme ----
    if not args.no_direct:
        out["direct_scheme"] = leg_direct(args, dev)
        print(f"[bench] direct scheme solve {out['direct_scheme']['ms_per_step']:.1f} ms", file=sys.stderr, flush=True)

    # ---- CPU oracle on a bounded sample ----
    if not args.no_cpu:
        print("[bench] cpu oracle sample", file=sys.stderr, flush=True)
        out["cpu_baseline"], out["error_vs_oracle"] = cpu_baseline(
            wl2, m, wl2.incident(), (u_mixed0, info[0].iterations), u_f64, not args.no_accuracy, args.fronts)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
