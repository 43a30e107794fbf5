"""Times the oracle on a bounded sample of a workload (CPU baseline).

Test infrastructure: run as a child process by the benchmark's CPU-baseline
leg, with the BLAS/OpenMP thread counts pinned to one so the measurement is
single-core. Prints one JSON object.

  python -m oracle.baseline [--mesh lshape|paper] --level 6 [--repeat R] [--solve]
  python -m oracle.baseline --mesh paper --level 9 --repeat 5 --assembly-only

The sample is the L-shaped domain (12 * 4^level triangles) or the paper's
unit-square mesh with Dirichlet sides x = 0, 1 (4^(level+1) triangles),
red-refined `level` times, with the data and per-triangle coefficient of
the elliptic benchmark workloads. Stages: topology + boundary (edge tables),
assembly (K, M, D, C, F, b_D into CSR), saddle matrix, and optionally the
sparse LU solve. --assembly-only builds the tables once and times the
assembly `repeat` times (median reported). The oracle is used as it stands;
nothing here tunes it.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--mesh", choices=("lshape", "paper"), default="lshape")
    ap.add_argument("--level", type=int, default=6)
    ap.add_argument("--repeat", type=int, default=3)
    ap.add_argument("--solve", action="store_true")
    ap.add_argument("--assembly-only", action="store_true")
    a = ap.parse_args()
    import numpy as np
    from oracle import oracle as O
    from paper_2401_15557_amd import meshgen as G
    O.build(force=False)
    m = G.lshape(a.level) if a.mesh == "lshape" else G.paper_square(a.level, bc="x_sides")
    aT = G.per_triangle_coefficient(m.nE, 0)
    f = O.fn(O.FN_SIN_COS, 2 * np.pi * np.pi, 0)
    g = O.fn(O.FN_CONST, 1.0)
    uD = O.fn(O.FN_CONST, 1.0)
    if a.assembly_only:
        t0 = time.perf_counter()
        tab = O.mesh_tables(m)
        t1 = time.perf_counter()
        runs = []
        for _ in range(a.repeat):
            s0 = time.perf_counter()
            O.assemble(m, tab, aT=aT, f=f, g=g, uD=uD)
            runs.append(time.perf_counter() - s0)
        print(json.dumps(dict(nE=m.nE, mesh=a.mesh, level=a.level, topology_s=t1 - t0,
                              assembly_runs_s=runs,
                              assembly_median_s=float(np.median(runs)),
                              threads=int(os.environ.get("OMP_NUM_THREADS", "0") or 0))))
        return
    best = None
    for _ in range(a.repeat):
        t0 = time.perf_counter()
        tab = O.mesh_tables(m)
        t1 = time.perf_counter()
        asm = O.assemble(m, tab, aT=aT, f=f, g=g, uD=uD)
        t2 = time.perf_counter()
        O.saddle(asm)
        t3 = time.perf_counter()
        t4 = t3
        if a.solve:
            O.solve_saddle(asm)
            t4 = time.perf_counter()
        cur = dict(topology_s=t1 - t0, assembly_s=t2 - t1, saddle_s=t3 - t2, solve_s=t4 - t3,
                   total_s=t4 - t0)
        if best is None or cur["total_s"] < best["total_s"]:
            best = cur
    best.update(nE=m.nE, mesh=a.mesh, level=a.level, repeat=a.repeat, solve=bool(a.solve),
                threads=int(os.environ.get("OMP_NUM_THREADS", "0") or 0))
    print(json.dumps(best))


if __name__ == "__main__":
    main()
