"""Benchmark: M(s)stab(l) time-stepping sequence on one MI355X.

One step = one whole sequence of the 128^3 convection-diffusion workload
(N = 2,097,152, 7-point upwind, Pe = 100, implicit Euler dt = 1e-3,
50 right-hand sides b^(k+1) = x^(k)/dt + f, x^(0) = 0), solved by M(s)stab(l)
to relative residual 1e-8 with the recycle data carried from system to system.
Every step starts from x = 0 with the recycle data dropped, so each step does
the same work.  value = systems per second over the timed steps.

Also reported on the same line: MVs per system; IDR(s)stab(l) on the same
sequence (no recycling); the FP32+FP64-replacement form and the form with an
FP32 copy of the matrix; the kernel roofline of
the dominant kernel class (HIP events on the solver's stream over the timed
steps); and the CPU oracle on a bounded sample.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--s 4] [--ell 2]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("systems/sec + MVs/system at rel-res 1e-8; SpMV HBM GB/s vs peak, "
          "M(s)stab vs IDRstab")
PMC_RECORD = os.path.join(ROOT, "profiles", "solver_convdiff128_pmc.json")
HBM_PEAK_GBS = 8000.0
EVENT_PERIOD = 16
CLASS_NAMES = ["spmv", "gamma", "eta", "gram", "poly"]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def run_sequence(torch, ms, solver, cd, f, systems):
    x = torch.zeros(cd.N, dtype=torch.float64, device="cuda")
    b = torch.empty_like(x)
    solver.recycle_reset()
    mv = 0
    infos = []
    for _ in range(systems):
        ms.mstab_rhs_step(x, cd.inv_dt, f, b)
        info = solver.solve_next(b, x)
        if not info["converged"]:
            raise RuntimeError(f"system did not converge: {info}")
        mv += info["mv_total"]
        infos.append(info)
    return x, mv, infos


def timed(torch, fn, steps, warmup):
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    outs = [fn() for _ in range(steps)]
    torch.cuda.synchronize()
    return time.perf_counter() - t0, outs


def cpu_baseline(cd, s, ell, mvs_per_system):
    """The FP64 oracle on the first two systems of the same sequence (single
    thread, recycling as on the GPU), scaled to systems/s at the sequence's
    mean MVs per system (the first systems cost several times the mean)."""
    import numpy as np
    import oracle
    from paper_1604_06043_amd import inputs as I
    A = oracle.assemble_convdiff(cd.dim, cd.n, cd.beta, cd.inv_dt, cd.kappa)
    P = I.p_dense(0, cd.N, s)
    x = np.zeros(cd.N)
    rec = oracle.Recycle.empty(cd.N, s)
    mv = 0
    t0 = time.perf_counter()
    for _ in range(2):
        b = oracle.rhs_step(x, cd.inv_dt, cd.f)
        x, info, rec, _ = oracle.solve(A, b, x, s, ell, P, recycle=rec)
        mv += info.mv_total
    dt = time.perf_counter() - t0
    rate = mv / dt
    return {"value": rate / mvs_per_system, "unit": "systems/s", "cores": 1, "kind": "oracle",
            "sample": f"systems 1-2 of the 128^3 sequence ({mv} MVs in {dt:.1f} s, single-threaded C "
                      f"FP64, {rate:.1f} MVs/s), scaled to the sequence mean of "
                      f"{mvs_per_system:.2f} MVs/system",
            "mvs_per_s": rate}


def class_kernels(cls: str, s: int, ell: int):
    """The kernels of one timing class of the FP64 solver."""
    return {"spmv": [f"k_spmv_dia<double, {s}, double, true>", f"k_spmv_dia<double, {s}, double, false>",
                     f"k_spmv<double, {s}, double>"],
            "eta": [f"k_eta<double, {s}>", f"k_eta_low<double, {s}>"],
            "gamma": [f"k_gamma<double, {s}>"],
            "poly": [f"k_poly<double, {s}, {ell}>"],
            "gram": [f"k_gram<double, {ell}>"]}[cls]


def measured_traffic(name_parts):
    """HBM bytes per dispatch, averaged over the dispatches of the named
    kernels, from the committed counter record, if it was taken with the
    current kernel sources (else None)."""
    from paper_1604_06043_amd import prof
    if not os.path.exists(PMC_RECORD):
        return None
    rec = json.load(open(PMC_RECORD))
    if rec.get("sources_sha256") != prof.sources_digest():
        return None
    tot, disp = 0.0, 0
    for name, t in rec["traffic"].items():
        if any(p + "(" in name for p in name_parts):
            tot += t["traffic_bytes"] * t["dispatches"]
            disp += t["dispatches"]
    return tot / disp if disp else None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--s", type=int, default=4)
    ap.add_argument("--ell", type=int, default=2)
    ap.add_argument("--systems", type=int, default=50)
    ap.add_argument("--n", type=int, default=128)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--no-events", action="store_true",
                    help="time the steps without per-kernel HIP events (no roofline)")
    ap.add_argument("--matrix-format", choices=["auto", "diagonal", "sliced"], default="auto",
                    help="device copy of A for the timed method (auto: constant diagonals when "
                         "the matrix has them)")
    ap.add_argument("--calib", action="store_true",
                    help="first copy 256 MiB device-to-device with a plain copy kernel "
                         "(reference for the HBM byte counters)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported "
              f"(the solve is a single-GPU kernel path)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1604_06043_amd import inputs as I
    from paper_1604_06043_amd import mstab as ms

    if not torch.cuda.is_available():
        raise SystemExit("bench.py needs a GPU")
    torch.cuda.set_device(0)
    ms.load()
    if args.calib:
        src = torch.ones(32 * 1024 * 1024, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    s, ell = args.s, args.ell
    cd = I.config("c2", seed=0, n=args.n)
    A = ms.mstab_assemble_convdiff(cd.dim, cd.n, cd.beta, cd.inv_dt)
    f = torch.tensor(cd.f, device="cuda")
    torch.cuda.synchronize()
    log(f"[bench] N={cd.N} nnz={A.nnz} s={s} ell={ell} systems/step={args.systems}")

    fmt = {"auto": ms.FORMAT_AUTO, "diagonal": ms.FORMAT_DIAGONAL, "sliced": ms.FORMAT_SLICED}[args.matrix_format]
    solver = ms.Solver(A, s, ell, p_seed=0, method=ms.METHOD_MSTAB, matrix_format=fmt)
    state = {}

    def step():
        x, mv, infos = run_sequence(torch, ms, solver, cd, f, args.systems)
        state["mv"] = mv
        state["infos"] = infos
        return mv

    for _ in range(args.warmup):
        step()
        log(f"[bench] warmup step done, MVs/system {state['mv'] / args.systems:.1f}")
    torch.cuda.synchronize()
    # one launch in EVENT_PERIOD of each class is timed with HIP events (timing
    # every launch costs the sequence ~18% of its throughput)
    solver.set_profiling(not args.no_events, EVENT_PERIOD)
    t, mvs = timed(torch, step, args.steps, 0)
    stats = {c: solver.kernel_stats(i) for i, c in enumerate(CLASS_NAMES)}
    solver.set_profiling(False)
    log(f"[bench] timed {args.steps} steps in {t:.3f} s")
    systems = args.steps * args.systems
    value = systems / t
    mv_per_system = sum(mvs) / systems

    kernels = {}
    for c, (n, msec, by) in stats.items():
        if n:
            kernels[c] = {"timed_launches": n, "ms_total_timed": round(msec, 3),
                          "us_per_launch": round(1e3 * msec / n, 2),
                          "GBs": round(by / (msec * 1e-3) / 1e9, 1)}
    # which device copy the products read, from their counted bytes per launch
    device_matrix = None
    if stats["spmv"][0]:
        per_row = stats["spmv"][2] / stats["spmv"][0] / cd.N
        device_matrix = ("diagonal storage, one value per diagonal (constant coefficients, detected "
                         "bit for bit from the CSR values)" if per_row < 30 else
                         "diagonal storage, values streamed")
    roofline = None
    if not args.no_events:
        dom = max(stats, key=lambda c: stats[c][1])
        n, msec, by = stats[dom]
        achieved = by / (msec * 1e-3) / 1e9
        names = class_kernels(dom, s, ell)
        traffic = measured_traffic(names)
        roofline = {"bound": "hbm", "kernel": dom, "kernels": names, "achieved": round(achieved, 1),
                    "timed": f"1 launch in {EVENT_PERIOD} of each kernel class, HIP events on the solver stream",
                    "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(achieved / HBM_PEAK_GBS, 4),
                    "traffic": None if traffic is None else round(traffic),
                    "bytes_per_launch": round(by / n), "us_per_launch": round(1e3 * msec / n, 2)}

    variants = {}
    if not args.no_variants:
        idr = ms.Solver(A, s, ell, p_seed=0, method=ms.METHOD_IDRSTAB)
        ti, (mvi,) = timed(torch, lambda: run_sequence(torch, ms, idr, cd, f, args.systems)[1], 1, 0)
        idr.close()
        variants["idrstab"] = {"systems_per_s": args.systems / ti,
                               "mvs_per_system": mvi / args.systems}
        log(f"[bench] IDR(s)stab(l): {args.systems / ti:.2f} systems/s")
        # the same method with the diagonal values streamed from HBM instead of
        # kept as one constant per diagonal (bit-identical iterates)
        dg = ms.Solver(A, s, ell, p_seed=0, method=ms.METHOD_MSTAB, matrix_format=ms.FORMAT_DIAGONAL)
        td, (mvd,) = timed(torch, lambda: run_sequence(torch, ms, dg, cd, f, args.systems)[1], 1, 0)
        dg.close()
        variants["diagonal_values_streamed"] = {"systems_per_s": args.systems / td,
                                                "mvs_per_system": mvd / args.systems}
        log(f"[bench] diagonal values streamed: {args.systems / td:.2f} systems/s")
        mix = ms.Solver(A, s, ell, p_seed=0, method=ms.METHOD_MSTAB, precision=ms.PREC_F32_REFINE)
        x64, _, _ = run_sequence(torch, ms, solver, cd, f, args.systems)
        holder = {}

        def mixed_step():
            x, mv, infos = run_sequence(torch, ms, mix, cd, f, args.systems)
            holder["x"] = x
            return mv
        tm, (mvm,) = timed(torch, mixed_step, 1, 0)
        err = float(torch.linalg.norm(holder["x"] - x64) / torch.linalg.norm(x64))
        mix.close()
        variants["f32_refine"] = {"systems_per_s": args.systems / tm,
                                  "mvs_per_system": mvm / args.systems,
                                  "rel_err_vs_f64_path_last_system": err}
        log(f"[bench] FP32+refinement: {args.systems / tm:.2f} systems/s, err {err:.2e}")
        low = ms.Solver(A, s, ell, p_seed=0, method=ms.METHOD_MSTAB, precision=ms.PREC_F32_MATRIX)

        def low_step():
            x, mv, infos = run_sequence(torch, ms, low, cd, f, args.systems)
            holder["x"] = x
            return mv
        tl, (mvl,) = timed(torch, low_step, 1, 0)
        errl = float(torch.linalg.norm(holder["x"] - x64) / torch.linalg.norm(x64))
        low.close()
        variants["f32_matrix"] = {"systems_per_s": args.systems / tl,
                                  "mvs_per_system": mvl / args.systems,
                                  "rel_err_vs_f64_path_last_system": errl}
        log(f"[bench] FP32 matrix copy: {args.systems / tl:.2f} systems/s, err {errl:.2e}")

    cpu = None
    if not args.no_cpu_baseline:
        log("[bench] CPU oracle sample ...")
        cpu = cpu_baseline(cd, s, ell, mv_per_system)
        log(f"[bench] CPU oracle: {cpu['value']:.4f} systems/s")

    out = {
        "metric": METRIC,
        "value": round(value, 4),
        "unit": "systems/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * t / args.steps, 2),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"convdiff3d_{cd.n}cubed_pe100_dt1e-3_{args.systems}rhs",
                   "N": cd.N, "nnz": A.nnz, "s": s, "ell": ell, "tol": 1e-8,
                   "method": "M(s)stab(l)", "systems_per_step": args.systems, "format": "csr_int32_f64",
                   "device_matrix": device_matrix},
        "mvs_per_system": round(mv_per_system, 2),
        "roofline": roofline,
        "kernels": kernels,
        "variants": variants,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
