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
choice per batch size timed on the device for this batch; --no-autotune keeps
the workload's w = 4 and the default kernels); its setup time includes the
tuning.

A 3D leg (object "c3") times the 127^3 workload the same way: four incident
waves, mixed precision, the slab-by-slab sweep captured as one graph; its
roofline is the sweep's factor bytes per apply over the apply's event-timed
duration.

Prints one JSON line. Besides the contract fields it carries the float64
form (same medium, one wave), per-kind kernel times from HIP events recorded
on the library's stream inside the timed region, the roofline of the
dominant kind, and the CPU oracle timed on a bounded sample of the same
workload (one of the 64 right-hand sides, solved in full).
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
# published MI355X vector peaks (TFLOP/s): fp32 157.3, fp64 78.6
ALU_PEAK = {8: 157.3, 16: 78.6}


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
    p.add_argument("--no-3d", action="store_true", help="skip the 3D leg (127^3, four waves, mixed)")
    p.add_argument("--steps-3d", type=int, default=2)
    p.add_argument("--no-adjoint", action="store_true",
                   help="skip the adjoint leg (511^2, 32 waves, mixed: forward solve plus adjoint solve)")
    p.add_argument("--steps-adjoint", type=int, default=3)
    p.add_argument("--no-autotune", action="store_true",
                   help="batched leg at the workload's w and the default kernels instead of autotuned ones")
    p.add_argument("--copy-gib", type=float, default=0.0,
                   help="first run one plain device copy of this many GiB (a known-size dispatch that "
                        "calibrates hardware byte counters in a profile of this command)")
    return p.parse_args()


def fstride(t: int, tw: int) -> int:
    return (t * t + t * tw + 1) & ~1


def work_per_column(solver, kind: str, cbytes: int, n: int):
    """(flops, shared_bytes, column_bytes) of one launch of a kind, per
    right-hand-side column: flops and the bytes every column moves, plus the
    bytes the launch reads once whatever its batch (factors, maps, spectrum).

    slice_solves: forward y_j = S_j^-1 r_j - W_j y_{j-1} (t^2 + t tw complex
      multiply-adds per transverse step) and backward x_j = y_j - G_j x_{j+1}
      (t^2), all slices; reads the factors once; per column reads the slice
      right-hand sides, writes and reads back the forward results and writes
      the solution.
    interface: 3l-5 dense L x L products (lambda chain, P term, mu chain).
    fft_convolve: read x and m, three passes over the n x P row transforms
      (written and read), write y; the (P/2+1)^2 spectrum once.
    stencil_Q: read n^2, write L^2.
    """
    L, nl = solver.L, solver.nslices
    if kind in ("slice_solves", "slice_solves_last"):
        # the last slice runs on its own stream beside the others when l > 2
        ks = range(nl)
        if nl > 2:
            ks = [nl - 1] if kind == "slice_solves_last" else range(nl - 1)
        fl = sh = col = 0.0
        for k in ks:
            lo, hi, naux = solver.slice_bounds(k)
            tw = hi - lo + 1
            t = tw + naux
            fl += 8.0 * L * (2 * t * t + t * tw)
            sh += cbytes * L * (fstride(t, tw) + fstride(t, 0))
            col += cbytes * L * (2 * tw + 2 * t)
        return fl, sh, col
    if kind == "interface":
        steps = max(0, 3 * nl - 5)
        return 8.0 * steps * L * L, float(cbytes * steps * L * L), float(cbytes * 3 * nl * L)
    if kind == "fft_convolve":
        P = 1
        while P < 2 * (n + 1):
            P <<= 1
        col = 2 * n * n * cbytes + n * n * 4 + 4 * n * P * cbytes + n * n * cbytes
        return 10.0 * P * P * (2 * P.bit_length() - 2), float((P // 2 + 1) ** 2 * cbytes), float(col)
    if kind == "stencil_Q":
        return 8.0 * 9 * n * n, 0.0, float(cbytes * (n * n + L * L))
    if kind == "extract":
        return 0.0, 0.0, float(cbytes * 2 * n * n)
    return 0.0, 0.0, 0.0


# HBM bytes per launch from hardware counters (FETCH_SIZE + WRITE_SIZE, each
# calibrated on a plain copy of known size), for the 1023^2 64-wave mixed
# workload: see profiles/c2_mixed_64rhs_hbm_counters.md. Keyed by kind and
# precision; valid only for the kernels as they were when measured.
MEASURED_TRAFFIC = {("interface", 8): 9.45e9}

# kinds that run on the second stream, overlapped with the main one
CONCURRENT = ("slice_solves_last",)
# published MI355X dense matrix-core peaks (TFLOP/s): fp32 157.3, fp64 78.6
MFMA_PEAK = {8: 157.3, 16: 78.6}


def roofline(solver, prof, cbytes: int, n: int):
    """Roofline entry of the main-stream kind with the largest total time:
    algorithmic work per launch (mean columns per launch x per-column work +
    shared work) over the mean event-timed launch duration, against the HBM
    peak or the arithmetic peak of the units the kernel runs on (matrix cores
    for the batched interface products and slice solves, else vector ALU),
    whichever bounds the work at that intensity."""
    dominant = max((k for k in prof if k not in CONCURRENT), key=lambda k: prof[k][1])
    launches, total_ms, columns = prof[dominant]
    avg_ms = total_ms / launches
    cols = columns / launches
    fl, sh, colb = work_per_column(solver, dominant, cbytes, n)
    flops = fl * cols
    nbytes = sh + colb * cols
    mfma = (dominant == "interface" and cols > 4) or (dominant.startswith("slice_solves") and cols > 8)
    peak = MFMA_PEAK[cbytes] if mfma else ALU_PEAK[cbytes]
    ridge = peak * 1e12 / (HBM_PEAK_GBS * 1e9)
    intensity = flops / nbytes if nbytes else float("inf")
    if intensity > ridge:
        achieved = flops / (avg_ms * 1e-3) / 1e12
        out = {"bound": "mfma" if mfma else "alu", "achieved": achieved, "peak": peak, "unit": "TFLOP/s"}
    else:
        achieved = nbytes / (avg_ms * 1e-3) / 1e9
        out = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s"}
    out["frac"] = out["achieved"] / out["peak"]
    out["traffic"] = MEASURED_TRAFFIC.get((dominant, cbytes)) if n == 1023 else None
    out.update({"kernel": dominant, "avg_launch_ms": avg_ms, "mean_columns_per_launch": cols,
                "algorithmic_flops_per_launch": flops, "algorithmic_bytes_per_launch": nbytes,
                "flop_per_byte": intensity})
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
                        "avg_launch_ms": avg_ms, "algorithmic_bytes_per_launch": nbytes}}
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


def cpu_baseline(wl, m, uinc):
    """The float64 oracle on the machine's host cores: its setup (not timed into
    the value, like the GPU's), then one full FGMRES solve of the first
    incident wave of the batch at the full grid."""
    cores = len(os.sched_getaffinity(0))
    os.environ.setdefault("OMP_NUM_THREADS", str(cores))
    try:
        import threadpoolctl
        threadpoolctl.threadpool_limits(cores)
    except Exception:
        pass
    import oracle
    t0 = time.perf_counter()
    s = oracle.OracleSolver(2, wl.n, wl.omega, m, wl.pml_width, wl.layer_thickness, workers=cores)
    t_setup = time.perf_counter() - t0
    t0 = time.perf_counter()
    res = s.solve_incident(uinc[:1], tol=wl.tol)[0]
    t_solve = time.perf_counter() - t0
    iters = res.iterations
    return {
        "value": wl.n ** 2 / t_solve,
        "unit": "unknowns*RHS/s",
        "cores": cores,
        "kind": "oracle",
        "sample": (f"1 of the {wl.nrhs} right-hand sides (theta=0), full {wl.n}^2 grid, solved to {wl.tol} by the "
                   f"float64 oracle (FGMRES, Algorithm-2 sweep with SuperLU slice factors, scipy FFT operator) in "
                   f"{t_solve:.1f} s, {iters} iterations; oracle setup {t_setup:.1f} s excluded like the GPU "
                   f"setup; SuperLU single-threaded, FFT and BLAS on {cores} threads"),
    }


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
                         restart=wl2.restart)
    else:
        # w and the kernel choice per batch size timed on the device for this batch
        mixed = LSSolver(md, wl2.omega, wl2.pml_width, None, precision="mixed", restart=wl2.restart,
                         autotune=wl2.nrhs)
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
    roof = roofline(mixed, prof, 8, n)
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
    }
    mixed.close()
    del mixed

    # ---- plain float64, one wave ----
    if not args.no_fp64:
        uinc1 = torch.as_tensor(wl1.incident(), device=dev)
        t0 = time.perf_counter()
        f64 = LSSolver(md, wl1.omega, wl1.pml_width, wl1.layer_thickness, precision="fp64", restart=wl1.restart)
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

    # ---- CPU oracle on a bounded sample ----
    if not args.no_cpu:
        print("[bench] cpu oracle sample", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(wl2, m, wl2.incident())
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
