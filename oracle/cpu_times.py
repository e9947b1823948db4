"""Time the CPU oracle on bounded samples of the measured workloads.

TEST INFRASTRUCTURE: this times the oracle (single-threaded C, FP64) as a
reference beside the GPU figures; nothing in the library imports it.

    python -m oracle.cpu_times c1 c3 c5

Each workload prints one JSON line: the sample, the products with A it took,
its seconds, and the oracle's rate in MVs/s (every product and every vector
pass of Algorithm 1 included).  Systems/s follow by dividing the rate by a
sequence's MVs per system.
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import time

import numpy as np

import oracle
from paper_1604_06043_amd import inputs as I


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor()


def run_sequence(A, first_b, next_b, s, ell, systems, max_mv=10 ** 9, seed=0):
    P = I.p_dense(seed, A.n, s)
    x = np.zeros(A.n)
    rec = oracle.Recycle.empty(A.n, s)
    mv, t0 = 0, time.perf_counter()
    for k in range(systems):
        b = first_b if k == 0 else next_b(x, k)
        x, info, rec, _ = oracle.solve(A, b, x, s, ell, P, recycle=rec, max_mv=max_mv)
        mv += info.mv_total
    return mv, time.perf_counter() - t0


def time_c1():
    cd = I.config("c1", seed=0)
    A = oracle.assemble_convdiff(cd.dim, cd.n, cd.beta, cd.inv_dt)
    mv, sec = run_sequence(A, cd.f, lambda x, k: oracle.rhs_step(x, cd.inv_dt, cd.f), 4, 2, 10)
    return {"workload": "c1 64^2, M(4)stab(2)", "sample": "the whole 10-system sequence", "mvs": mv,
            "seconds": sec, "systems_per_s": 10 / sec}


def time_c3(cycles=5):
    cd = I.config("c3", seed=0)
    A = oracle.assemble_convdiff(cd.dim, cd.n, cd.beta, cd.inv_dt, cd.kappa)
    s, ell = 8, 4
    cap = 1 + s + cycles * ell * (s + 1)
    mv, sec = run_sequence(A, cd.f, None, s, ell, 1, max_mv=cap)
    return {"workload": "c3 256^3 lognormal kappa, M(8)stab(4)",
            "sample": f"the first {cycles} cycles of system 1 ({cap} MVs)", "mvs": mv, "seconds": sec}


def time_c5(systems=2):
    N = 1 << 22
    g = I.rgg(N, 0)
    A = oracle.CSR(g.row_ptr, g.col, g.val)
    del g
    xi = [0.1 * I.white_noise(0, k, N) for k in range(systems)]
    mv, sec = run_sequence(A, xi[0], lambda x, k: x + xi[k], 4, 2, systems)
    return {"workload": "c5 graph N=4.2M, M(4)stab(2)", "sample": f"systems 1-{systems}", "mvs": mv,
            "seconds": sec}


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("which", nargs="+", choices=["c1", "c3", "c5"])
    a = ap.parse_args()
    host = {"cpu": cpu_model(), "nproc": os.cpu_count(), "threads_used": 1}
    for w in a.which:
        r = {"c1": time_c1, "c3": time_c3, "c5": time_c5}[w]()
        r["mvs_per_s"] = r["mvs"] / r["seconds"]
        r.update(host)
        print(json.dumps(r), flush=True)


if __name__ == "__main__":
    main()
