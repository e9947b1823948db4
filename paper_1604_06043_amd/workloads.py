"""Measurements of the solver on the sequence workloads beside the main bench.

    python -m paper_1604_06043_amd.workloads sweep   # 128^3, s in {2,4,8}, l in {1,2,4}
    python -m paper_1604_06043_amd.workloads c1      # 64^2 (latency-bound), s=4, l=2, 10 RHS
    python -m paper_1604_06043_amd.workloads c3      # 256^3, lognormal kappa, s=8, l=4, 20 RHS
    python -m paper_1604_06043_amd.workloads c5      # 4M-row random geometric graph, 100 RHS
    python -m paper_1604_06043_amd.workloads fetch   # fetch policies of M(s)stab on 128^3 and 64^2
    python -m paper_1604_06043_amd.workloads jacobi  # split diagonal preconditioning on c3 and c5
    python -m paper_1604_06043_amd.workloads ilu     # split ILU(0) (multicolour order) against it
    python -m paper_1604_06043_amd.workloads batch   # B independent 64^2 sequences solved together
    python -m paper_1604_06043_amd.workloads reorder # c5 with reverse Cuthill-McKee reordering

Each prints one JSON line per measurement (systems/s and MVs/system of
M(s)stab(l) and IDR(s)stab(l), FP64 and FP32 + FP64 refinement, and the
error of the mixed form against the FP64 path).  Inputs come from
:mod:`inputs`; every arithmetic step runs in the library's kernels.
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np

from . import inputs as I
from . import mstab as M


def log(*a):
    print(*a, file=sys.stderr, flush=True)


class Sequence:
    """A matrix on the device and the forcing of b^(k+1) = x^(k) inv_dt + f^(k)."""

    def __init__(self, A: M.CSR, inv_dt: float, forcing, name: str):
        self.A, self.inv_dt, self.forcing, self.name = A, inv_dt, forcing, name
        self.N = A.n

    def f(self, k):
        return self.forcing(k)


def run(seq: Sequence, systems: int, s: int, ell: int, method: int = M.METHOD_MSTAB,
        precision: int = M.PREC_F64, seed: int = 0, keep_x: bool = False, **opt):
    """Solve the sequence once; returns (seconds, MVs per system, infos, xs)."""
    import torch
    solver = M.Solver(seq.A, s, ell, p_seed=seed, method=method, precision=precision, **opt)
    x = torch.zeros(seq.N, dtype=torch.float64, device="cuda")
    b = torch.empty_like(x)
    infos, xs = [], []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(systems):
        M.mstab_rhs_step(x, seq.inv_dt, seq.f(k), b)
        info = solver.solve_next(b, x)
        if not info["converged"]:
            raise RuntimeError(f"{seq.name}: system {k} did not converge: {info}")
        infos.append(info)
        if keep_x:
            xs.append(x.clone())
    torch.cuda.synchronize()
    sec = time.perf_counter() - t0
    solver.close()
    mv = sum(i["mv_total"] for i in infos) / systems
    return sec, mv, infos, xs


def compare(seq: Sequence, systems: int, s: int, ell: int, seed: int = 0, idr: bool = True,
            mixed: bool = True, **opt):
    """M(s)stab FP64 (and IDR(s)stab, FP32+refinement) on one sequence."""
    import torch
    out = {"workload": seq.name, "N": seq.N, "nnz": seq.A.nnz, "s": s, "ell": ell,
           "systems": systems, "tol": 1e-8}
    # warm-up: first launches and allocator
    run(seq, 1, s, ell, seed=seed)
    t, mv, infos, xs = run(seq, systems, s, ell, seed=seed, keep_x=mixed, **opt)
    out["mstab_f64"] = {"systems_per_s": systems / t, "mvs_per_system": mv}
    log(f"[{seq.name}] M({s})stab({ell}) FP64: {systems / t:.2f} systems/s, {mv:.1f} MVs/system")
    if idr:
        t, mv, _, _ = run(seq, systems, s, ell, method=M.METHOD_IDRSTAB, seed=seed, **opt)
        out["idrstab_f64"] = {"systems_per_s": systems / t, "mvs_per_system": mv}
        log(f"[{seq.name}] IDR({s})stab({ell}) FP64: {systems / t:.2f} systems/s, {mv:.1f} MVs/system")
    if mixed:
        for name, method in (("mstab_f32_matrix", M.METHOD_MSTAB), ("idrstab_f32_matrix", M.METHOD_IDRSTAB)):
            tl, mvl, il, xl = run(seq, systems, s, ell, method=method, precision=M.PREC_F32_MATRIX,
                                  seed=seed, keep_x=True, **opt)
            errs = [float(torch.linalg.vector_norm(a - b) / torch.linalg.vector_norm(b))
                    for a, b in zip(xl, xs)]
            out[name] = {"systems_per_s": systems / tl, "mvs_per_system": mvl,
                         "f64_mvs_per_system": sum(i["mv_f64"] for i in il) / systems,
                         "max_true_relres": max(i["relres_true"] for i in il),
                         "rel_err_vs_f64_path_max": max(errs)}
            log(f"[{seq.name}] {name}: {systems / tl:.2f} systems/s, {mvl:.1f} MVs/system, "
                f"max err vs FP64 path {max(errs):.2e}")
            del xl
        tm, mvm, im, xm = run(seq, systems, s, ell, precision=M.PREC_F32_REFINE, seed=seed,
                              keep_x=True, **opt)
        errs = [float(torch.linalg.vector_norm(a - b) / torch.linalg.vector_norm(b))
                for a, b in zip(xm, xs)]
        out["mstab_f32_refine"] = {
            "systems_per_s": systems / tm, "mvs_per_system": mvm,
            "f64_mvs_per_system": sum(i["mv_f64"] for i in im) / systems,
            "refinements_per_system": sum(i["refinements"] for i in im) / systems,
            "max_true_relres": max(i["relres_true"] for i in im),
            "rel_err_vs_f64_path_max": max(errs), "rel_err_vs_f64_path_last": errs[-1]}
        log(f"[{seq.name}] M({s})stab({ell}) FP32+refinement: {systems / tm:.2f} systems/s, "
            f"{mvm:.1f} MVs/system, max err vs FP64 path {max(errs):.2e}")
    return out


def jacobi_compare(seq: Sequence, systems: int, s: int, ell: int, seed: int = 0):
    """M(s)stab and IDR(s)stab with and without the split diagonal preconditioning."""
    out = {"workload": seq.name, "N": seq.N, "nnz": seq.A.nnz, "s": s, "ell": ell,
           "systems": systems, "tol": 1e-8}
    run(seq, 1, s, ell, seed=seed)
    runs = [("mstab", M.METHOD_MSTAB, M.PREC_F64), ("idrstab", M.METHOD_IDRSTAB, M.PREC_F64),
            ("mstab_f32_matrix", M.METHOD_MSTAB, M.PREC_F32_MATRIX),
            ("idrstab_f32_matrix", M.METHOD_IDRSTAB, M.PREC_F32_MATRIX)]
    for name, method, prec in runs:
        variants = [(M.PRECOND_NONE, 0, "plain"), (M.PRECOND_JACOBI, 0, "jacobi")]
        if prec == M.PREC_F64:
            variants.append((M.PRECOND_JACOBI, 1, "jacobi_replace1"))
        for pc, every, tag in variants:
            t, mv, infos, _ = run(seq, systems, s, ell, method=method, precision=prec, seed=seed,
                                  precond=pc, replace_every=every)
            out[f"{name}_{tag}"] = {"systems_per_s": systems / t, "mvs_per_system": mv,
                                    "max_relres_true": max(i["relres_true"] for i in infos)}
            log(f"[{seq.name}] {name} {tag}: {systems / t:.2f} systems/s, {mv:.1f} MVs/system")
    return out


def ilu_compare(seq: Sequence, systems: int, s: int, ell: int, seed: int = 0):
    """M(s)stab and IDR(s)stab (FP64) with the split diagonal and the split
    ILU(0) preconditioning (Section 5.1's form), per-cycle replacement off."""
    out = {"workload": seq.name, "N": seq.N, "nnz": seq.A.nnz, "s": s, "ell": ell,
           "systems": systems, "tol": 1e-8}
    run(seq, 1, s, ell, seed=seed, precond=M.PRECOND_ILU0)
    for name, method in (("mstab", M.METHOD_MSTAB), ("idrstab", M.METHOD_IDRSTAB)):
        for tag, pc in (("jacobi", M.PRECOND_JACOBI), ("ilu0", M.PRECOND_ILU0)):
            t, mv, infos, _ = run(seq, systems, s, ell, method=method, seed=seed, precond=pc)
            out[f"{name}_{tag}"] = {"systems_per_s": systems / t, "mvs_per_system": mv,
                                    "max_relres_true": max(i["relres_true"] for i in infos)}
            log(f"[{seq.name}] {name} {tag}: {systems / t:.3f} systems/s, {mv:.1f} MVs/system")
    return out


def batch_throughput(B: int, systems: int = 10, n: int = 64, s: int = 4, ell: int = 2):
    """B independent c1-type sequences (seeds 0..B-1), each on its own handle
    and stream, advanced together by mstab_solve_batch; aggregate systems/s."""
    import torch
    cds = [I.config("c1", seed=k, n=n) for k in range(B)]
    mats = []
    for cd in cds:
        mats.append(M.mstab_assemble_convdiff(cd.dim, cd.n, cd.beta, cd.inv_dt, None))
    streams = [torch.cuda.Stream() for _ in range(B)]
    solvers = [M.Solver(A, s, ell, p_seed=0, stream=st) for A, st in zip(mats, streams)]
    fs = [torch.tensor(cd.f, device="cuda") for cd in cds]
    xs = [torch.zeros(cd.N, dtype=torch.float64, device="cuda") for cd in cds]
    bs = [torch.empty_like(x) for x in xs]
    torch.cuda.synchronize()
    mv, t0 = 0, time.perf_counter()
    for _ in range(systems):
        for i in range(B):
            M.mstab_rhs_step(xs[i], cds[i].inv_dt, fs[i], bs[i])
        infos = M.solve_batch(solvers, bs, xs)
        if not all(i["converged"] for i in infos):
            raise RuntimeError("a batched system did not converge")
        mv += sum(i["mv_total"] for i in infos)
    torch.cuda.synchronize()
    sec = time.perf_counter() - t0
    for sv in solvers:
        sv.close()
    return {"workload": f"c1_n{n}", "sequences": B, "systems_each": systems, "s": s, "ell": ell,
            "systems_per_s": B * systems / sec, "mvs_per_system": mv / (B * systems)}


def gmres_compare(seq: Sequence, systems: int, s: int, ell: int, restarts=(10, 30), seed: int = 0, **opt):
    """Section 5.1's comparison on one sequence: M(s)stab(l) and IDR(s)stab(l)
    against restarted GMRES(m), each with the same options (a splitting)."""
    out = {"workload": seq.name, "N": seq.N, "systems": systems, "s": s, "ell": ell, "tol": 1e-8}
    run(seq, 1, s, ell, seed=seed, **opt)   # warm-up
    rows = [("mstab", dict(method=M.METHOD_MSTAB), s, ell), ("idrstab", dict(method=M.METHOD_IDRSTAB), s, ell)]
    rows += [(f"gmres_{m}", dict(method=M.METHOD_GMRES, gmres_restart=m), 1, 1) for m in restarts]
    for name, mopt, ss, ll in rows:
        t, mv, infos, _ = run(seq, systems, ss, ll, seed=seed, **mopt, **opt)
        out[name] = {"systems_per_s": systems / t, "mvs_per_system": mv,
                     "max_relres_true": max(i["relres_true"] for i in infos)}
        log(f"[{seq.name}] {name}: {systems / t:.3f} systems/s, {mv:.1f} MVs/system")
    return out


def batch_workgroup(B: int, systems: int = 10, n: int = 64, s: int = 4, ell: int = 2):
    """B independent c1-type sequences (seeds 0..B-1) on handles of the
    one-workgroup engine: each step forms every right-hand side with one
    mstab_rhs_step over the B x N block, then one mstab_solve_batch launch
    solves all B systems (one workgroup each).  Aggregate systems/s."""
    import torch
    cds = [I.config("c1", seed=k, n=n) for k in range(B)]
    N = cds[0].N
    inv_dt = cds[0].inv_dt
    assert all(cd.inv_dt == inv_dt for cd in cds)
    mats = [M.mstab_assemble_convdiff(cd.dim, cd.n, cd.beta, cd.inv_dt, None) for cd in cds]
    solvers = [M.Solver(A, s, ell, p_seed=0, engine=M.ENGINE_WORKGROUP) for A in mats]
    F = torch.tensor(np.stack([cd.f for cd in cds]), device="cuda")
    X = torch.zeros((B, N), dtype=torch.float64, device="cuda")
    Bv = torch.empty_like(X)
    xs, bs = [X[i] for i in range(B)], [Bv[i] for i in range(B)]
    batch = M.Batch(solvers, bs, xs)
    torch.cuda.synchronize()
    mv, t0 = 0, time.perf_counter()
    for _ in range(systems):
        M.mstab_rhs_step(X.view(-1), inv_dt, F.view(-1), Bv.view(-1))
        batch.run()
        if not batch.field("converged").all():
            raise RuntimeError("a batched system did not converge")
        mv += int(batch.field("mv").sum() + batch.field("mv_check").sum())
    torch.cuda.synchronize()
    sec = time.perf_counter() - t0
    for sv in solvers:
        sv.close()
    return {"workload": f"c1_n{n}", "engine": "workgroup", "sequences": B, "systems_each": systems,
            "s": s, "ell": ell, "systems_per_s": B * systems / sec, "mvs_per_system": mv / (B * systems)}


def reorder_compare(seq: Sequence, systems: int, s: int, ell: int, seed: int = 0):
    """M(s)stab and IDR(s)stab on the caller's order and on the RCM order,
    with and without the split diagonal preconditioning."""
    out = {"workload": seq.name, "N": seq.N, "nnz": seq.A.nnz, "s": s, "ell": ell,
           "systems": systems, "tol": 1e-8}
    run(seq, 1, s, ell, seed=seed, reorder=M.REORDER_RCM)
    for name, method, prec in (("mstab", M.METHOD_MSTAB, M.PREC_F64),
                               ("idrstab", M.METHOD_IDRSTAB, M.PREC_F64),
                               ("mstab_f32_matrix", M.METHOD_MSTAB, M.PREC_F32_MATRIX),
                               ("idrstab_f32_matrix", M.METHOD_IDRSTAB, M.PREC_F32_MATRIX)):
        for ro, pc, tag in ((M.REORDER_RCM, M.PRECOND_NONE, "rcm"),
                            (M.REORDER_RCM, M.PRECOND_JACOBI, "rcm_jacobi")):
            t, mv, infos, _ = run(seq, systems, s, ell, method=method, precision=prec, seed=seed,
                                  reorder=ro, precond=pc)
            out[f"{name}_{tag}"] = {"systems_per_s": systems / t, "mvs_per_system": mv,
                                    "max_relres_true": max(i["relres_true"] for i in infos)}
            log(f"[{seq.name}] {name} {tag}: {systems / t:.2f} systems/s, {mv:.1f} MVs/system")
    return out


def convdiff_sequence(name: str, n: int | None = None, seed: int = 0) -> Sequence:
    import torch
    cd = I.config(name, seed=seed, n=n)
    kappa = None if cd.kappa is None else torch.tensor(cd.kappa, device="cuda")
    A = M.mstab_assemble_convdiff(cd.dim, cd.n, cd.beta, cd.inv_dt, kappa)
    f = torch.tensor(cd.f, device="cuda")
    del kappa
    return Sequence(A, cd.inv_dt, lambda k: f, f"{name}_n{cd.n}")


def rgg_sequence(N: int, seed: int = 0, systems: int = 100) -> Sequence:
    """b^(k+1) = x^(k) + 0.1 xi^(k) on the graph matrix (inv_dt = 1, f = 0.1 xi)."""
    import torch
    t0 = time.perf_counter()
    g = I.rgg(N, seed)
    log(f"[rgg] N={N} nnz={g.nnz} generated in {time.perf_counter() - t0:.1f} s")
    A = M.CSR(torch.tensor(g.row_ptr, device="cuda"), torch.tensor(g.col, device="cuda"),
              torch.tensor(g.val, device="cuda"))
    del g
    F = torch.empty((systems, N), dtype=torch.float64, device="cuda")
    for k in range(systems):
        F[k] = torch.tensor(0.1 * I.white_noise(seed, k, N), device="cuda")
    return Sequence(A, 1.0, lambda k: F[k], f"rgg_N{N}")


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("which", choices=["sweep", "c1", "c3", "c5", "c2", "fetch", "jacobi", "ilu", "batch",
                                      "wgbatch", "reorder", "fetchsweep", "gmres"])
    ap.add_argument("--n", type=int, default=None)
    ap.add_argument("--N", type=int, default=1 << 22)
    ap.add_argument("--systems", type=int, default=None)
    ap.add_argument("--B", type=int, default=None, help="wgbatch: one batch size only")
    a = ap.parse_args()
    import torch
    torch.cuda.set_device(0)
    M.load()
    if a.which == "sweep":
        seq = convdiff_sequence("c2", a.n)
        systems = a.systems or 50
        for s in (2, 4, 8):
            for ell in (1, 2, 4):
                print(json.dumps(compare(seq, systems, s, ell, mixed=False)), flush=True)
    elif a.which == "reorder":
        systems = a.systems or 100
        seq = rgg_sequence(a.N, 0, systems)
        print(json.dumps(reorder_compare(seq, systems, 4, 2)), flush=True)
    elif a.which == "batch":
        import os
        for B in (1, 2, 4, 8, 16, 32):
            batch_throughput(B, 2)   # warm-up
            r = batch_throughput(B, a.systems or 10)
            r["gpu_max_hw_queues"] = os.environ.get("GPU_MAX_HW_QUEUES", "default")
            log(f"[batch] {B} sequences: {r['systems_per_s']:.0f} systems/s, {r['mvs_per_system']:.1f} MVs/system")
            print(json.dumps(r), flush=True)
    elif a.which == "wgbatch":
        for B in ((a.B,) if a.B else (1, 8, 64, 256, 512, 1024, 2048)):
            batch_workgroup(min(B, 64), 1)   # warm-up
            r = batch_workgroup(B, a.systems or 10)
            log(f"[wgbatch] {B} sequences: {r['systems_per_s']:.0f} systems/s, "
                f"{r['mvs_per_system']:.1f} MVs/system")
            print(json.dumps(r), flush=True)
    elif a.which == "c1":
        seq = convdiff_sequence("c1", a.n)
        print(json.dumps(compare(seq, a.systems or 10, 4, 2, mixed=False)), flush=True)
    elif a.which == "c2":
        seq = convdiff_sequence("c2", a.n)
        print(json.dumps(compare(seq, a.systems or 50, 4, 2)), flush=True)
    elif a.which == "c3":
        seq = convdiff_sequence("c3", a.n)
        print(json.dumps(compare(seq, a.systems or 20, 8, 4)), flush=True)
    elif a.which == "fetch":
        policies = {"threshold": M.FETCH_THRESHOLD, "once": M.FETCH_ONCE, "at_end": M.FETCH_AT_END,
                    "estimate": M.FETCH_ESTIMATE}
        for name, n, systems in (("c1", 64, 10), ("c2", 64, 30), ("c2", 128, 50)):
            seq = convdiff_sequence(name, n)
            row = {"workload": seq.name, "systems": systems, "s": 4, "ell": 2}
            t, mv, infos, _ = run(seq, systems, 4, 2, method=M.METHOD_IDRSTAB)
            row["idrstab"] = {"systems_per_s": systems / t, "mvs_per_system": mv,
                              "mvs": [i["mv_total"] for i in infos]}
            for pname, pol in policies.items():
                t, mv, infos, _ = run(seq, systems, 4, 2, fetch=pol)
                row[f"mstab_{pname}"] = {"systems_per_s": systems / t, "mvs_per_system": mv,
                                         "mvs": [i["mv_total"] for i in infos]}
                log(f"[{seq.name}] fetch {pname}: {mv:.1f} MVs/system (IDR {row['idrstab']['mvs_per_system']:.1f})")
            print(json.dumps(row), flush=True)
    elif a.which == "gmres":
        print(json.dumps(gmres_compare(convdiff_sequence("c2", a.n), a.systems or 10, 4, 2)), flush=True)
        print(json.dumps(gmres_compare(convdiff_sequence("c3", a.n), a.systems or 5, 8, 4,
                                       precond=M.PRECOND_JACOBI)), flush=True)
        print(json.dumps(gmres_compare(rgg_sequence(a.N, 0, a.systems or 10), a.systems or 10, 4, 2,
                                       reorder=M.REORDER_RCM, precond=M.PRECOND_JACOBI)), flush=True)
    elif a.which == "fetchsweep":
        # the bench sequence under every fetch policy and THRESHOLD level
        seq = convdiff_sequence("c2", a.n)
        systems = a.systems or 50
        run(seq, 2, 4, 2)   # warm-up
        rows = {"idrstab": dict(method=M.METHOD_IDRSTAB)}
        for lvl in (1e-1, 1e-2, 1e-3, 1e-4, 1e-5, 1e-6):
            rows[f"threshold_{lvl:g}"] = dict(fetch_rel=lvl)
        rows["estimate"] = dict(fetch=M.FETCH_ESTIMATE)
        rows["at_end"] = dict(fetch=M.FETCH_AT_END)
        rows["threshold_orth"] = dict(orthonormalize_recycle=1)
        rows["estimate_orth"] = dict(fetch=M.FETCH_ESTIMATE, orthonormalize_recycle=1)
        out = {"workload": seq.name, "systems": systems, "s": 4, "ell": 2}
        for name, opt in rows.items():
            t, mv, infos, _ = run(seq, systems, 4, 2, **opt)
            out[name] = {"systems_per_s": systems / t, "mvs_per_system": mv,
                         "mvs": [i["mv_total"] for i in infos]}
            log(f"[fetchsweep] {name}: {mv:.2f} MVs/system, {systems / t:.1f} systems/s")
        print(json.dumps(out), flush=True)
    elif a.which == "c5":
        systems = a.systems or 100
        seq = rgg_sequence(a.N, 0, systems)
        print(json.dumps(compare(seq, systems, 4, 2)), flush=True)
    elif a.which == "ilu":
        for seq, systems, s, ell in ((convdiff_sequence("c3", a.n), a.systems or 20, 8, 4),
                                     (rgg_sequence(a.N, 0, a.systems or 100), a.systems or 100, 4, 2)):
            print(json.dumps(ilu_compare(seq, systems, s, ell)), flush=True)
            del seq
    elif a.which == "jacobi":
        for seq, systems, s, ell in ((convdiff_sequence("c3", a.n), a.systems or 20, 8, 4),
                                     (rgg_sequence(a.N, 0, a.systems or 100), a.systems or 100, 4, 2)):
            print(json.dumps(jacobi_compare(seq, systems, s, ell)), flush=True)
            del seq


if __name__ == "__main__":
    main()
