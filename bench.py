"""Benchmark: M(s)stab(l) time-stepping sequence on one MI355X.

One step = one whole sequence of the 128^3 convection-diffusion workload
(N = 2,097,152, 7-point upwind, Pe = 100, implicit Euler dt = 1e-3,
50 right-hand sides b^(k+1) = x^(k)/dt + f, x^(0) = 0), solved by M(s)stab(l)
to relative residual 1e-8 with the recycle data carried from system to system.
Every step starts from x = 0 with the recycle data dropped, so each step does
the same work.  value = systems per second over the timed steps.

Also reported on the same line, each timed over the same warmup and timed
steps with no kernel timing: IDR(s)stab(l) on the same sequence (no
recycling), the same method with the diagonal values streamed, the
FP32+FP64-replacement form and the form with an FP32 copy of the matrix.
Then: the kernel roofline of the dominant kernel class (HIP events on the
solver's stream in one extra, untimed step); the 256^3 lognormal-kappa
workload at s = 8, l = 4 in FP64 and both FP32 forms, with and without the
split diagonal preconditioning; and the CPU oracle on the host cores.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--s 4] [--ell 2]
       [--no-variants] [--no-c3] [--no-cpu-baseline] [--no-events]
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


def cpu_baseline(cd, s, ell, mvs_per_system, threads):
    """The FP64 oracle on the host cores: `threads` independent copies of the
    first system of the same sequence (the oracle is sequential C; ctypes
    releases the GIL, so the copies run on separate cores), their summed MVs
    over the wall time, scaled to systems/s at the GPU sequence's mean MVs per
    system (the first system costs several times the mean)."""
    import numpy as np
    from concurrent.futures import ThreadPoolExecutor
    import oracle
    from paper_1604_06043_amd import inputs as I
    A = oracle.assemble_convdiff(cd.dim, cd.n, cd.beta, cd.inv_dt, cd.kappa)
    P = I.p_dense(0, cd.N, s)
    b = oracle.rhs_step(np.zeros(cd.N), cd.inv_dt, cd.f)

    def one(_):
        rec = oracle.Recycle.empty(cd.N, s)
        _, info, _, _ = oracle.solve(A, b, np.zeros(cd.N), s, ell, P, recycle=rec)
        return info.mv_total
    t0 = time.perf_counter()
    with ThreadPoolExecutor(threads) as ex:
        mvs = list(ex.map(one, range(threads)))
    dt = time.perf_counter() - t0
    rate = sum(mvs) / dt
    return {"value": rate / mvs_per_system, "unit": "systems/s", "cores": threads, "kind": "oracle",
            "sample": f"system 1 of the 128^3 sequence solved by {threads} independent copies of the "
                      f"single-threaded C FP64 oracle at once, one per host core ({sum(mvs)} MVs in "
                      f"{dt:.1f} s, {rate:.1f} MVs/s), scaled to the GPU sequence mean of "
                      f"{mvs_per_system:.2f} MVs/system",
            "mvs_per_s": rate}


def class_kernels(cls: str, s: int, ell: int):
    """The kernels of one timing class of the FP64 solver."""
    return {"spmv": [f"k_spmv_dia_pair<double, {s}, double, {c}, {nd}, 0>" for c in ("true", "false") for nd in (7, 5)]
            + [f"k_spmv_dia_const<double, {s}, {nd}, 0>" for nd in (7, 5)]
            + [f"k_spmv_dia<double, {s}, double, {c}, 0>" for c in ("true", "false")]
            + [f"k_spmv<double, {s}, double, 0>"],
            "eta": [f"k_eta<double, {s}>", f"k_eta_low<double, {s}>", f"k_eta_low_gamma<double, {s}>"],
            "gamma": [f"k_gamma<double, {s}>"],
            "poly": [f"k_poly<double, {s}, {ell}, 0>"],
            "gram": [f"k_gram<double, {ell}>", f"k_eta_low_gram<double, {s}, {ell}>"]}[cls]


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


def c3_leg(torch, ms, n, systems):
    """The 256^3 variable-coefficient workload (Pe = 200, kappa = exp(N(0,1))
    per node, s = 8, l = 4): the first `systems` systems of its sequence in
    FP64 and in the two FP32 forms, each with and without the split diagonal
    preconditioning that Section 5.1 pairs with the method; error of each
    FP32 form's last x against the FP64 path's, and the FP64 path with the
    ILU(0) splitting of a multicolour order (the FP64 oracle needs hours
    at this size; the tests state the error against it on the same workload
    at 14^3-48^3)."""
    from paper_1604_06043_amd import inputs as I
    cd = I.config("c3", seed=0, n=n)
    kappa = torch.tensor(cd.kappa, device="cuda")
    A = ms.mstab_assemble_convdiff(cd.dim, cd.n, cd.beta, cd.inv_dt, kappa)
    f = torch.tensor(cd.f, device="cuda")
    s, ell = 8, 4
    out = {"workload": f"convdiff3d_{n}cubed_pe200_lognormal_kappa_{systems}rhs", "N": cd.N, "s": s,
           "ell": ell, "tol": 1e-8, "systems_per_step": systems}
    for pc_name, pc in (("none", ms.PRECOND_NONE), ("jacobi", ms.PRECOND_JACOBI), ("ilu0", ms.PRECOND_ILU0)):
        x64 = None
        forms = (("f64", ms.PREC_F64), ("f32_matrix", ms.PREC_F32_MATRIX), ("f32_refine", ms.PREC_F32_REFINE))
        # the ILU(0) splitting runs in FP64 only
        for key, prec in forms[:1] if pc == ms.PRECOND_ILU0 else forms:
            sv = ms.Solver(A, s, ell, p_seed=0, precision=prec, precond=pc)
            run_sequence(torch, ms, sv, cd, f, 1)             # warm-up
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            x, mv, infos = run_sequence(torch, ms, sv, cd, f, systems)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            sv.close()
            rec = {"systems_per_s": systems / dt, "mvs_per_system": mv / systems,
                   "max_relres_true": max(i["relres_true"] for i in infos)}
            if x64 is None:
                x64 = x.clone()
            else:
                rec["rel_err_vs_f64_path_last_system"] = float(torch.linalg.norm(x - x64) /
                                                               torch.linalg.norm(x64))
            out[f"{key}_{pc_name}"] = rec
            log(f"[bench] c3 {key} precond={pc_name}: {rec['systems_per_s']:.3f} systems/s, "
                f"{rec['mvs_per_system']:.1f} MVs/system")
    return out


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
    ap.add_argument("--no-c3", action="store_true",
                    help="skip the 256^3 lognormal-kappa mixed-precision leg")
    ap.add_argument("--c3-n", type=int, default=256)
    ap.add_argument("--c3-systems", type=int, default=3)
    ap.add_argument("--cpu-threads", type=int, default=16,
                    help="host cores for the oracle baseline (at most the available ones)")
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
    # the timed steps run with no kernel timing at all
    t, mvs = timed(torch, step, args.steps, 0)
    log(f"[bench] timed {args.steps} steps in {t:.3f} s")
    systems = args.steps * args.systems
    value = systems / t
    mv_per_system = sum(mvs) / systems

    # a separate pass with HIP events on the solver's stream gives the kernel
    # classes' durations for the roofline (1 launch in EVENT_PERIOD timed)
    stats = {c: (0, 0.0, 0.0) for c in CLASS_NAMES}
    if not args.no_events:
        solver.set_profiling(True, EVENT_PERIOD)
        step()
        torch.cuda.synchronize()
        stats = {c: solver.kernel_stats(i) for i, c in enumerate(CLASS_NAMES)}
        solver.set_profiling(False)

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
                    "timed": f"1 launch in {EVENT_PERIOD} of each kernel class, HIP events on the solver "
                             f"stream, in one extra untimed step",
                    "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(achieved / HBM_PEAK_GBS, 4),
                    "traffic": None if traffic is None else round(traffic),
                    "bytes_per_launch": round(by / n), "us_per_launch": round(1e3 * msec / n, 2)}

    variants = {}
    if not args.no_variants:
        # every variant: the same warmup and timed steps as the main line,
        # no kernel timing
        def variant(name, **opt):
            sv = ms.Solver(A, s, ell, p_seed=0, **opt)
            holder = {}

            def vstep():
                x, mv, infos = run_sequence(torch, ms, sv, cd, f, args.systems)
                holder["x"] = x
                return mv
            for _ in range(args.warmup):
                vstep()
            tv, mvv = timed(torch, vstep, args.steps, 0)
            sv.close()
            rec = {"systems_per_s": systems / tv, "mvs_per_system": sum(mvv) / systems}
            log(f"[bench] {name}: {rec['systems_per_s']:.2f} systems/s, {rec['mvs_per_system']:.2f} MVs/system")
            return rec, holder["x"]

        x64, _, _ = run_sequence(torch, ms, solver, cd, f, args.systems)
        variants["idrstab"], _ = variant("IDR(s)stab(l)", method=ms.METHOD_IDRSTAB)
        # the fetch point estimated from the previous solve's convergence
        # (Section 5, how to choose the fetching point) instead of sqrt(tol)
        variants["mstab_fetch_estimate"], _ = variant("M(s)stab(l), estimated fetch point",
                                                      method=ms.METHOD_MSTAB, fetch=ms.FETCH_ESTIMATE)
        # the same method with the diagonal values streamed from HBM instead of
        # kept as one constant per diagonal (bit-identical iterates)
        variants["diagonal_values_streamed"], _ = variant("values streamed", method=ms.METHOD_MSTAB,
                                                          matrix_format=ms.FORMAT_DIAGONAL)
        for key, prec in (("f32_refine", ms.PREC_F32_REFINE), ("f32_matrix", ms.PREC_F32_MATRIX)):
            rec, xv = variant(key, method=ms.METHOD_MSTAB, precision=prec)
            rec["rel_err_vs_f64_path_last_system"] = float(torch.linalg.norm(xv - x64) / torch.linalg.norm(x64))
            log(f"[bench] {key}: |x - x64| {float(torch.linalg.norm(xv - x64)):.3e}, |x64| "
                f"{float(torch.linalg.norm(x64)):.3e}, max |x - x64| {float((xv - x64).abs().max()):.3e}")
            variants[key] = rec
    c3 = None
    if not args.no_c3:
        c3 = c3_leg(torch, ms, args.c3_n, args.c3_systems)

    cpu = None
    if not args.no_cpu_baseline:
        threads = min(len(os.sched_getaffinity(0)), args.cpu_threads)
        log(f"[bench] CPU oracle sample on {threads} cores ...")
        cpu = cpu_baseline(cd, s, ell, mv_per_system, threads)
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
        "c3_mixed_precision": c3,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
