"""Benchmark of the primal hybrid FEM hot path on one MI355X.

  python bench.py [--gpus 1] [--steps K] [--warmup W]

Headline workload (the paper's largest run): the unit square with the
paper's four-triangle criss-cross start mesh, red-refined 10 times on the
device = 4,194,304 triangles, fp64, per-triangle coefficient a_T ~ U[0.5, 2]
(seed 0), Dirichlet u_D = 1 on x = 0 and x = 1, Neumann g = 1 on y = 0 and
y = 1, f = 2 pi^2 sin(pi x) cos(pi y). Inputs are synthetic and resident in
device memory before timing starts; the mesh, its edge tables and CSR
patterns are built once (the paper times topology and assembly separately).

One timed step = one numeric assembly of that mesh (phf_assemble): K, M, C,
F = b + LN and b_D written into their CSR value arrays. `value` is assembled
elements per second (Melem/s); `roofline` is that kernel's algorithmic
bytes (268 B per triangle) over its average launch time, from HIP events the
library records on its own stream during the timed steps.

The JSON line also carries, measured in the same process:
  pipeline   the whole elliptic path on the same workload per step: the
             4-triangle base mesh uploaded and validated with its edge
             tables (phf_mesh_create), 10 device red refinements with edge
             tables, boundary classification and patterns
             (phf_mesh_refine), the assembly, and the saddle solve by
             multigrid-preconditioned conjugate gradients to rtol 1e-10 (and
             once to 1e-13); stage times from events on the library stream;
  lshape     the L-shaped configuration (12 triangles refined 9 times,
             3,145,728 triangles, Dirichlet u_D = 1 on the re-entrant edges,
             Neumann g = 1 elsewhere): assembly alone and the whole path;
  kernels_traced_step  every kernel of one fully traced pipeline step, and
             the dominant one (the finest multigrid sweep, whose operator
             largely stays in the 256 MB last-level cache: its fraction is
             labelled cache-assisted);
  copy_probe a plain 512 MiB device-to-device copy (read + write bytes / time)
             next to the 8 TB/s peak;
  scatter    segment-length histogram of the scatter (source terms summed
             into each output entry);
  cn         Crank-Nicolson steps/s (unit square, 1,048,576 triangles,
             k = 1e-3, 200 steps), replaying captured HIP graphs and eagerly;
  batch      256 uneven meshes in one launch vs one launch per mesh;
  cn_batch   16 uneven Crank-Nicolson problems advanced together (two graph
             launches per step) vs one stepper at a time;
  serve      mixed elliptic / Crank-Nicolson requests at Poisson rates,
             one slot vs continuous batching, p50/p99 latency;
  cpu_baseline  the CPU oracle, one core, assembly alone on a bounded sample
             of the headline workload (median of 5), plus the whole path with
             sparse LU on a smaller sample.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "assembled Melem/s + HBM GB/s (4M tris); CN steps/s; served p50/p99 latency"


def algorithmic_bytes(info, has_aT=True, level_nf=None, level_nE=None, jacobi=False):
    """Bytes a kernel must move at least, per launch, by kernel name.

    k_assemble: read coordinates once (16 B/node), element vertices
    (12 B/elem), a_T (8 B/elem), 8 B per multiplier row (the row's edge:
    |E|/2, or its two end nodes); write K and M (72 B/elem each), F
    (24 B/elem), C (8 B/nnz) and b_D (8 B/row).
    V-cycle kernels (single precision) on level l with n unknowns
    (level_nf[l]), operator rows scaled by the inverse diagonal with four
    off-diagonal (int32 column, fp32 value) slots = 32 B/row: smoothing sweep
    32 + 4 (D^-1 b) + 4 (x) + 4 (y) = 44 B/row; first sweep from zero on the
    finest level (rounds the fp64 residual once; only for the first cycle,
    later ones get it from the CG update) 8 + 4 (dinv) + 4 (D^-1 b) = 16
    B/row, the second sweep forming the first from D^-1 b 32 + 4 + 4 = 40;
    last finest sweep, which also writes z (fp32 for CG) and reduces r.z,
    32 + 4 + 4 + 8 (r) + 4 (z) = 52 B/row; residual 32 + 4 (diag) + 4 + 4 +
    4 (r) = 48 B/row; prolongation 20 (five int32 columns) + 4 (five 4-bit
    weight codes) + 8 (x in and out) = 32 B/fine row + 4 B/coarse row;
    restriction from level l: per coarse triangle 36 B of fine row ids, 4 B
    code word, 12 B of sums written, plus the fine residual once (4 B/fine
    row), then per coarse row 8 (positions) + 8 (two sums) + 4 (dinv) in,
    4 (D^-1 b) + 4 (first sweep) out = 28 B.
    """
    nE, nC, L = info.nE, info.nC, info.L
    nf, nnzR = info.n_free, info.nnz_reduced
    asm = (16 * nC + 12 * nE + (8 * nE if has_aT else 0) + 8 * L +
           8 * (9 * nE) * 2 + 8 * 3 * nE + 8 * info.nnz_C + 8 * L)
    mg = {}
    top = len(level_nf or []) - 1
    for l, n in enumerate(level_nf or []):
        mg[f"k_mg_smooth.L{l}"] = 44 * n
        if l == top:
            mg[f"k_mg_smooth0.L{l}"] = 16 * n
            # second sweep, the first formed from D^-1 b: 16 + 16 + 4 + 4
            mg[f"k_mg_smooth1.L{l}"] = 40 * n
            mg[f"k_mg_smooth_z.L{l}"] = 52 * n
        mg[f"k_mg_resid.L{l}"] = 48 * n
        if l > 0:
            mg[f"k_mg_prolong.L{l}"] = 32 * n + 4 * level_nf[l - 1]
            if level_nE:
                mg[f"k_mg_restrict.L{l}"] = 52 * level_nE[l - 1] + 4 * n
            mg[f"k_mg_collect.L{l}"] = 28 * level_nf[l - 1]
    return {
        **mg,
        "k_assemble": asm,
        # reduced operator: column + value of each off-diagonal entry (12 B),
        # the diagonal value (8 B/row); z in (fp64 with Jacobi, the cycle's
        # fp32 result with multigrid); p, q in and out
        "k_cg_dir": 12 * (nnzR - nf) + 8 * nf + (40 if jacobi else 36) * nf,
        # read p, q, w, r; write w, r; Jacobi: dinv in, z out (fp64);
        # multigrid: dinv (fp32) in, D^-1 r out (fp32; the first sweep is
        # formed by the second)
        "k_cg_upd": (64 if jacobi else 56) * nf,
    }


def sources_hash(files):
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_2401_15557_amd", "csrc")
    for n in files:
        h.update(open(os.path.join(d, n), "rb").read())
    return h.hexdigest()[:16]


def traffic_for(kernel, workload_key=None):
    """HBM traffic per launch from the committed counter summary, if it was
    taken on the current sources of that kernel (and on this workload, when
    a key is given); otherwise None."""
    p = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        rec = json.load(open(p))
    except (OSError, ValueError):
        return None
    k = rec.get("kernels", {}).get(workload_key or kernel)
    if not k:
        return None
    try:
        if k.get("hash") != sources_hash(k.get("sources", [])):
            return None
    except OSError:
        return None
    return k.get("bytes_per_launch")


def cpu_model():
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=20).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                return line.split(":", 1)[1].strip()
    except (OSError, subprocess.SubprocessError):
        pass
    return None


def cpu_baseline(level, repeat, pipeline_level):
    """The oracle on the host, one thread: assembly alone on the paper mesh
    at `level` (median of `repeat`), and the whole path with sparse LU on the
    L-shape at `pipeline_level`."""
    env = dict(os.environ, OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1", MKL_NUM_THREADS="1")

    def run(args):
        r = subprocess.run([sys.executable, "-m", "oracle.baseline", *args], cwd=ROOT, env=env,
                           capture_output=True, text=True, timeout=900)
        if r.returncode != 0:
            return {"error": r.stderr[-500:]}
        return json.loads(r.stdout.strip().splitlines()[-1])

    a = run(["--mesh", "paper", "--level", str(level), "--repeat", str(repeat),
             "--assembly-only"])
    p = run(["--mesh", "lshape", "--level", str(pipeline_level), "--repeat", "2", "--solve"])
    if "error" in a:
        return a
    out = {"value": round(a["nE"] / a["assembly_median_s"] / 1e6, 4), "unit": "Melem/s",
           "cores": 1, "kind": "oracle",
           "sample": (f"assembly alone (K, M, C, F, b_D into CSR) on the headline workload's mesh "
                      f"at level {level} ({a['nE']} triangles, same data), median of {repeat} "
                      f"runs {[round(x, 3) for x in a['assembly_runs_s']]} s, one thread; "
                      f"topology {a['topology_s']:.3f} s"),
           "cpu_model": cpu_model(), "nproc": os.cpu_count()}
    if "error" not in p:
        out["pipeline"] = {
            "value": round(p["nE"] / p["total_s"] / 1e6, 4), "unit": "Melem/s",
            "sample": (f"L-shape level {pipeline_level} ({p['nE']} triangles): topology + "
                       f"assembly + saddle CSR + sparse LU solve, best of 2"),
            "stage_s": {k: round(p[k], 4) for k in ("topology_s", "assembly_s", "saddle_s",
                                                      "solve_s")}}
    return out


def scatter_histogram(topo, nE):
    """Segment lengths of the scatter: how many source terms are summed into
    each output entry. K, M (element blocks), C (one per edge side and
    vertex) and b_D (one per Dirichlet row) have exactly one; F gets the
    element's body load plus |E| g / 2 from each Neumann edge of that element
    through the vertex (local edges other than the vertex's own)."""
    import numpy as np
    et = topo["edge_type"].astype(np.int64)
    ee = topo["elem_edges"].reshape(nE, 3)
    neu = et[ee] == 2                         # local edge i of element m is Neumann
    cnt = np.ones((nE, 3), np.int64)
    for j in range(3):
        for i in range(3):
            if i != j:
                cnt[:, j] += neu[:, i]
    hist = np.bincount(cnt.reshape(-1))
    f = {str(k): int(v) for k, v in enumerate(hist) if v}
    # b_D: one term on a Dirichlet row, none (an explicit zero) on an
    # interior row
    return {"K": {"1": 9 * nE}, "M": {"1": 9 * nE}, "F": f,
            "C": {"1": int(4 * (et == 0).sum() + 2 * (et == 1).sum())},
            "bD": {"0": int((et == 0).sum()), "1": int((et == 1).sum())}}


def serve_requests(G, phfem, count, seed):
    """Mixed request stream: 70% elliptic on refined structured unit squares,
    30% Crank-Nicolson on the refined paper mesh with 10-100 steps; final
    sizes log-uniform in [1e3, 1e6] triangles."""
    import numpy as np
    rng = np.random.default_rng(seed)
    pi = np.pi
    reqs = []
    for _ in range(count):
        target = np.exp(rng.uniform(np.log(1e3), np.log(1e6)))
        if rng.uniform() < 0.7:
            r = max(0, int(round(np.log(target / 32.0) / np.log(4.0))))
            n = max(2, int(round(np.sqrt(target / (2.0 * 4 ** r)))))
            a = rng.uniform(0.5, 2.0)
            d = phfem.make_data(phfem.make_fn(phfem.PHF_FN_SIN_COS, 2 * pi * pi, 0),
                                phfem.make_fn(phfem.PHF_FN_GRAD_SIN_COS, 1, 0),
                                phfem.make_fn(phfem.PHF_FN_SIN_COS, 1, 0))
            reqs.append(phfem.make_request(phfem.PHF_REQ_ELLIPTIC, G.unit_square_structured(n),
                                           refine=r, coeffs=phfem.make_coeffs(A=(a, 0, 0, a)),
                                           data=d, rtol=1e-10))
        else:
            lev = int(min(9, max(4, round(np.log(target / 4.0) / np.log(4.0)))))
            steps = int(rng.integers(10, 101))
            d = phfem.make_data(phfem.make_fn(phfem.PHF_FN_SIN_SIN, 2 * pi * pi - 1, -1),
                                phfem.make_fn(phfem.PHF_FN_GRAD_SIN_SIN, 1, -1),
                                phfem.make_fn(phfem.PHF_FN_SIN_SIN, 1, -1))
            reqs.append(phfem.make_request(phfem.PHF_REQ_CN, G.paper_square(0, bc="x_sides"),
                                           refine=lev, data=d,
                                           u0=phfem.make_fn(phfem.PHF_FN_SIN_SIN, 1, -1),
                                           rtol=1e-10, k=1e-3, steps=steps))
    return reqs


def serve_run(phfem, reqs, rate, slots, seed):
    """Open-loop Poisson arrivals at `rate` requests/s into a server with
    `slots` slots; returns latency percentiles and throughput."""
    import threading
    import numpy as np
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, size=len(reqs))
    srv = phfem.phf_server_create(0, slots=slots)
    ids = [None] * len(reqs)
    t0 = time.perf_counter()

    def submit():
        t = t0
        for q, r in enumerate(reqs):
            t += gaps[q]
            dt = t - time.perf_counter()
            if dt > 0:
                time.sleep(dt)
            ids[q] = phfem.phf_server_submit(srv, r)

    th = threading.Thread(target=submit)
    th.start()
    th.join()
    res = [phfem.phf_server_wait(srv, i) for i in ids]
    t1 = time.perf_counter()
    st = phfem.phf_server_query(srv)
    phfem.phf_server_destroy(srv)
    bad = [r.status for r in res if r.status != 0]
    lat = np.array([r.latency_ms for r in res])
    q = np.array([r.queue_ms for r in res])
    return dict(rate_per_s=rate, slots=slots, requests=len(reqs), failed=len(bad),
                p50_ms=round(float(np.percentile(lat, 50)), 3),
                p99_ms=round(float(np.percentile(lat, 99)), 3),
                mean_ms=round(float(lat.mean()), 3),
                mean_queue_ms=round(float(q.mean()), 3),
                solves_per_s=round(len(reqs) / (t1 - t0), 2),
                peak_concurrent=int(st.peak_running),
                triangles_per_s=round(sum(r.nE for r in res) / (t1 - t0), 1))




def build_chain(phfem, h, base, levels):
    """Device mesh chain: the base mesh (device arrays) and `levels` red
    refinements; returns the handles, coarsest first."""
    chain = [phfem.phf_mesh_create(h, *base, phfem.PHF_DEVICE)]
    for _ in range(levels):
        chain.append(phfem.phf_mesh_refine(chain[-1]))
    return chain


def release(phfem, chain):
    for c in reversed(chain):
        phfem.phf_mesh_destroy(c)


def time_assembly(phfem, torch, h, mh, co, data, sysd, reps, warmup):
    """`reps` back-to-back assemblies after `warmup` untimed ones: wall time
    per call (stream synchronised on both sides) and the kernel's per-launch
    times from the library's HIP events on its stream."""
    for _ in range(warmup):
        phfem.phf_assemble(mh, co, data, sysd)
    torch.cuda.synchronize()
    phfem.phf_trace_enable(h, True)
    phfem.phf_trace_filter(h, "k_assemble")
    phfem.phf_trace_reset(h)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        phfem.phf_assemble(mh, co, data, sysd)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    samples = phfem.phf_trace_samples(h, "k_assemble")
    phfem.phf_trace_filter(h, None)
    phfem.phf_trace_enable(h, False)
    return 1e3 * (t1 - t0) / reps, samples


def time_assembly_cold(phfem, torch, h, mh, co, data, sysd, reps, dev):
    """Per-launch kernel times of assemblies that each follow a read of 1 GiB
    (a sum), which evicts the inputs from the last-level cache and leaves it
    holding clean lines only (a copy would leave dirty lines there for the
    assembly to write back)."""
    fa = torch.ones(1 << 27, dtype=torch.float64, device=dev)
    acc = torch.zeros((), dtype=torch.float64, device=dev)
    phfem.phf_trace_enable(h, True)
    phfem.phf_trace_filter(h, "k_assemble")
    phfem.phf_trace_reset(h)
    for _ in range(reps):
        acc += fa.sum()
        phfem.phf_assemble(mh, co, data, sysd)
    torch.cuda.synchronize()
    samples = phfem.phf_trace_samples(h, "k_assemble")
    phfem.phf_trace_filter(h, None)
    phfem.phf_trace_enable(h, False)
    del fa, acc
    return samples


def assembly_summary(info, ms_call, samples, traffic_key, cold=None, has_aT=True):
    ab = algorithmic_bytes(info, has_aT=has_aT)["k_assemble"]
    avg_us = 1e3 * sum(samples) / len(samples)
    gbs = ab / (avg_us * 1e-6) / 1e9
    cold_s = None
    if cold:
        cus = 1e3 * sum(cold) / len(cold)
        cgbs = ab / (cus * 1e-6) / 1e9
        cold_s = {"kernel_us": round(cus, 2), "GB_per_s": round(cgbs, 1),
                  "frac_of_hbm_peak": round(cgbs / HBM_PEAK_GBS, 4), "launches": len(cold),
                  "note": "each launch after reading 1 GiB (inputs evicted from the cache)"}
    return {"Melem_per_s": round(info.nE / (ms_call * 1e3), 1),
            "kernel_us": round(avg_us, 2), "kernel_us_min": round(1e3 * min(samples), 2),
            "kernel_us_max": round(1e3 * max(samples), 2), "call_us": round(ms_call * 1e3, 2),
            "kernel_Melem_per_s": round(info.nE / avg_us, 1),
            "algorithmic_bytes": ab, "bytes_per_elem": round(ab / info.nE, 1),
            "GB_per_s": round(gbs, 1), "frac_of_hbm_peak": round(gbs / HBM_PEAK_GBS, 4),
            "traffic": traffic_for("k_assemble", traffic_key), "launches": len(samples),
            "cold": cold_s}


def pipeline_steps(phfem, torch, h, base, levels, co, data, sysd, U, Lam, rtol, steps, pc):
    """Whole elliptic path per step, with events on the library's stream
    between the stages (device times, idle gaps while the host waits on a
    read-back included)."""
    rows = []
    for _ in range(steps):
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(5)]
        t0 = time.perf_counter()
        ev[0].record()
        chain = build_chain(phfem, h, base, levels)
        ev[1].record()
        phfem.phf_assemble(chain[-1], co, data, sysd)
        ev[2].record()
        st = phfem.phf_solve(chain[-1], co, sysd, U, Lam, rtol=rtol, max_iter=200000,
                             check_every=32 if pc == phfem.PHF_PRECOND_JACOBI else 0,
                             precond=pc)
        ev[3].record()
        release(phfem, chain)
        ev[4].record()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        rows.append(dict(step_ms=1e3 * (t1 - t0), mesh_ms=ev[0].elapsed_time(ev[1]),
                         assembly_ms=ev[1].elapsed_time(ev[2]),
                         solve_ms=ev[2].elapsed_time(ev[3]),
                         release_ms=ev[3].elapsed_time(ev[4]),
                         iterations=st.iterations, rel_residual=st.rel_residual,
                         converged=bool(st.converged)))
    return rows


def summarise_pipeline(rows, nE):
    import numpy as np
    med = {k: float(np.median([r[k] for r in rows])) for k in rows[0] if k != "converged"}
    return {"steps": len(rows), "ms_per_step": round(med["step_ms"], 3),
            "Melem_per_s": round(nE / (med["step_ms"] * 1e3), 2),
            "device_stage_ms": {k[:-3]: round(med[k], 3)
                                for k in ("mesh_ms", "assembly_ms", "solve_ms", "release_ms")},
            "iterations": int(med["iterations"]), "rel_residual": med["rel_residual"],
            "all_converged": all(r["converged"] for r in rows)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100, help="timed assemblies")
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--level", type=int, default=10, help="paper-mesh refinement level")
    ap.add_argument("--pipeline-steps", type=int, default=3)
    ap.add_argument("--lshape-level", type=int, default=9)
    ap.add_argument("--cn-level", type=int, default=9)
    ap.add_argument("--cn-steps", type=int, default=200)
    ap.add_argument("--cn-chunk", type=int, default=8,
                    help="expected CG iterations of the first time step")
    ap.add_argument("--cpu-level", type=int, default=9,
                    help="paper-mesh level of the CPU oracle's assembly sample")
    ap.add_argument("--cpu-repeat", type=int, default=5)
    ap.add_argument("--no-lshape", action="store_true")
    ap.add_argument("--no-pipeline", action="store_true")
    ap.add_argument("--no-cn", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--rtol", type=float, default=1e-10)
    ap.add_argument("--mode", choices=("full", "assembly", "batch", "pipeline"), default="full",
                    help="counter runs: assembly = the numeric assembly alone (headline mesh, or "
                         "the L-shape with --workload lshape); batch = the batched assembly at "
                         "tile 128; pipeline = one whole elliptic step on the headline mesh; "
                         "each followed by one plain device copy of --copy-mib MiB")
    ap.add_argument("--workload", choices=("paper", "lshape"), default="paper")
    ap.add_argument("--asm-reps", type=int, default=2)
    ap.add_argument("--copy-mib", type=int, default=512)
    ap.add_argument("--precond", choices=("multigrid", "jacobi"), default="multigrid")
    ap.add_argument("--serve-requests", type=int, default=120)
    ap.add_argument("--serve-rates", type=str, default="20,40,80",
                    help="Poisson arrival rates (requests/s) to sweep")
    ap.add_argument("--serve-slots", type=int, default=4)
    ap.add_argument("--batch-count", type=int, default=256)
    ap.add_argument("--batch-reps", type=int, default=20)
    ap.add_argument("--cn-batch-count", type=int, default=16)
    ap.add_argument("--batch-tile", type=int, default=128, help="--mode batch: tile")
    ap.add_argument("--batch-gather", type=int, default=0, help="--mode batch: gathered coordinates")
    ap.add_argument("--cn-batch-steps", type=int, default=50)
    a = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if a.gpus != 1 or world != 1:
        print("bench.py runs on exactly one GPU: the library has no multi-GPU path; "
              "every figure is one GPU's.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2401_15557_amd import meshgen as G
    from paper_2401_15557_amd import phfem

    dev = torch.device("cuda", 0)
    pi = np.pi
    pc = phfem.PHF_PRECOND_MULTIGRID if a.precond == "multigrid" else phfem.PHF_PRECOND_JACOBI
    ctx = phfem.Context(0)
    h = ctx.handle

    def dev_mesh(m):
        return tuple(torch.tensor(x, device=dev) for x in
                     (m.coords, m.elements, m.dirichlet, m.neumann))

    # data of the elliptic workloads: f = 2 pi^2 sin(pi x) cos(pi y), g = 1, u_D = 1
    data = phfem.make_data(phfem.make_fn(phfem.PHF_FN_SIN_COS, 2 * pi * pi, 0),
                           phfem.make_fn(phfem.PHF_FN_CONST, 1.0),
                           phfem.make_fn(phfem.PHF_FN_CONST, 1.0))
    paper_base = dev_mesh(G.paper_square(0, bc="x_sides"))
    lshape_base = dev_mesh(G.lshape(0))

    if a.mode == "assembly":
        base, lev = ((paper_base, a.level) if a.workload == "paper"
                     else (lshape_base, a.lshape_level))
        chain = build_chain(phfem, h, base, lev)
        info = phfem.phf_mesh_get_info(chain[-1])
        aT_d = torch.tensor(G.per_triangle_coefficient(info.nE, 0), device=dev)
        co = phfem.make_coeffs(a_T=aT_d)
        sysd, t = phfem.alloc_system_for(info, dev)
        for _ in range(a.asm_reps):
            phfem.phf_assemble(chain[-1], co, data, sysd)
        src = torch.ones(a.copy_mib << 17, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        release(phfem, chain)
        print(json.dumps({"mode": "assembly", "workload": a.workload, "nE": info.nE,
                          "launches": a.asm_reps,
                          "algorithmic_bytes_per_launch": algorithmic_bytes(info)["k_assemble"],
                          "copy_bytes_each_way": src.numel() * 8}))
        return

    if a.mode == "batch":
        inst = G.batch_instances(a.batch_count, 1)
        bm = [phfem.phf_mesh_create(h, mm.coords, mm.elements, mm.dirichlet, mm.neumann)
              for mm, _ in inst]
        binfo = [phfem.phf_mesh_get_info(x) for x in bm]
        bco = [phfem.make_coeffs(A=(av, 0.0, 0.0, av)) for _, av in inst]
        bdat = [phfem.make_data(phfem.make_fn(phfem.PHF_FN_SIN_COS, 2 * pi * pi * av, 0),
                                phfem.make_fn(phfem.PHF_FN_GRAD_SIN_COS, av, 0),
                                phfem.make_fn(phfem.PHF_FN_SIN_COS, 1, 0)) for _, av in inst]
        bsys = [phfem.alloc_system_for(bi, dev)[0] for bi in binfo]
        batch = phfem.phf_batch_create(h, bm)
        phfem.phf_batch_set_config(batch, a.batch_tile, 0, 1, 0, a.batch_gather)
        for _ in range(a.asm_reps):
            phfem.phf_batch_assemble(batch, bco, bdat, bsys)
        src = torch.ones(a.copy_mib << 17, dtype=torch.float64, device=dev)
        torch.empty_like(src).copy_(src)
        torch.cuda.synchronize()
        phfem.phf_batch_destroy(batch)
        for x in bm:
            phfem.phf_mesh_destroy(x)
        print(json.dumps({"mode": "batch", "nE_total": sum(bi.nE for bi in binfo),
                          "launches": a.asm_reps,
                          "algorithmic_bytes_per_launch": sum(
                              algorithmic_bytes(bi, has_aT=False)["k_assemble"] for bi in binfo),
                          "copy_bytes_each_way": src.numel() * 8}))
        return

    if a.mode == "pipeline":
        chain = build_chain(phfem, h, paper_base, a.level)
        info = phfem.phf_mesh_get_info(chain[-1])
        aT_d = torch.tensor(G.per_triangle_coefficient(info.nE, 0), device=dev)
        co = phfem.make_coeffs(a_T=aT_d)
        sysd, t = phfem.alloc_system_for(info, dev)
        U = torch.empty(info.N, dtype=torch.float64, device=dev)
        Lam = torch.empty(info.L, dtype=torch.float64, device=dev)
        release(phfem, chain)
        rows = pipeline_steps(phfem, torch, h, paper_base, a.level, co, data, sysd, U, Lam, a.rtol,
                              1, pc)
        src = torch.ones(a.copy_mib << 17, dtype=torch.float64, device=dev)
        torch.empty_like(src).copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"mode": "pipeline", "nE": info.nE, "step": rows[0],
                          "copy_bytes_each_way": src.numel() * 8}))
        return

    # ---- headline: numeric assembly of the 4,194,304-triangle mesh ----------
    print(f"[bench] building the paper mesh, {a.level} device refinements", file=sys.stderr,
          flush=True)
    chain = build_chain(phfem, h, paper_base, a.level)
    mh = chain[-1]
    info = phfem.phf_mesh_get_info(mh)
    nE = info.nE
    aT_d = torch.tensor(G.per_triangle_coefficient(nE, 0), device=dev)
    co = phfem.make_coeffs(a_T=aT_d)
    sysd, sys_t = phfem.alloc_system_for(info, dev)
    U = torch.empty(info.N, dtype=torch.float64, device=dev)
    Lam = torch.empty(info.L, dtype=torch.float64, device=dev)
    print(f"[bench] headline: {a.warmup} warm-up + {a.steps} timed assemblies, nE={nE}",
          file=sys.stderr, flush=True)
    ms_call, samples = time_assembly(phfem, torch, h, mh, co, data, sysd, a.steps, a.warmup)
    cold = time_assembly_cold(phfem, torch, h, mh, co, data, sysd, 20, dev)
    head = assembly_summary(info, ms_call, samples, f"k_assemble@paper_L{a.level}", cold)
    print(f"[bench] assembly: {head}", file=sys.stderr, flush=True)
    topo = {k: np.empty(n, dt) for k, n, dt in (("edge_type", info.n_edges, np.int8),
                                                ("elem_edges", 3 * nE, np.int32))}
    phfem.phf_mesh_topology(mh, elem_edges=topo["elem_edges"], edge_type=topo["edge_type"],
                            memspace=phfem.PHF_HOST)
    scatter = scatter_histogram(topo, nE)
    del topo
    roof = {"bound": "hbm", "kernel": "k_assemble", "achieved": head["GB_per_s"],
            "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": head["frac_of_hbm_peak"],
            "traffic": head["traffic"], "avg_launch_us": head["kernel_us"],
            "launches": head["launches"], "algorithmic_bytes_per_launch": head["algorithmic_bytes"],
            "bytes_per_elem": head["bytes_per_elem"]}
    release(phfem, chain)

    # ---- the whole elliptic path on the same workload ------------------------
    out_pipe = None
    kern = {}
    if not a.no_pipeline:
        print("[bench] pipeline: warm-up step", file=sys.stderr, flush=True)
        pipeline_steps(phfem, torch, h, paper_base, a.level, co, data, sysd, U, Lam, a.rtol, 1,
                       pc)
        rows = pipeline_steps(phfem, torch, h, paper_base, a.level, co, data, sysd, U, Lam,
                              a.rtol, a.pipeline_steps, pc)
        print(f"[bench] pipeline rows {rows}", file=sys.stderr, flush=True)
        tight = pipeline_steps(phfem, torch, h, paper_base, a.level, co, data, sysd, U, Lam,
                               1e-13, 1, pc)
        print(f"[bench] pipeline rtol 1e-13 {tight}", file=sys.stderr, flush=True)
        # one fully traced step: every kernel, per-kernel breakdown
        phfem.phf_trace_enable(h, True)
        phfem.phf_trace_reset(h)
        chain = build_chain(phfem, h, paper_base, a.level)
        level_nf = [phfem.phf_mesh_get_info(c).n_free for c in chain]
        level_nE = [phfem.phf_mesh_get_info(c).nE for c in chain]
        phfem.phf_assemble(chain[-1], co, data, sysd)
        phfem.phf_solve(chain[-1], co, sysd, U, Lam, rtol=a.rtol, precond=pc)
        release(phfem, chain)
        kern = phfem.phf_trace_dump(h)
        phfem.phf_trace_enable(h, False)
        ab = algorithmic_bytes(info, level_nf=level_nf, level_nE=level_nE,
                               jacobi=pc == phfem.PHF_PRECOND_JACOBI)
        dname = max(kern.items(), key=lambda kv: kv[1][1])[0]
        dom = None
        if dname in ab:
            us = kern[dname][1] / kern[dname][0] * 1e3
            gbs = ab[dname] / (us * 1e-6) / 1e9
            dom = {"kernel": dname, "avg_launch_us": round(us, 3), "launches": kern[dname][0],
                   "algorithmic_bytes_per_launch": ab[dname], "GB_per_s": round(gbs, 1),
                   "frac_of_hbm_peak": round(gbs / HBM_PEAK_GBS, 4),
                   "cache_assisted": dname.startswith("k_mg_")}
        out_pipe = {
            "workload": (f"paper mesh refined {a.level} times on the device ({nE} triangles); "
                         f"step = base upload + {a.level} refinements with topology and "
                         f"patterns + assembly + saddle solve (CG + {a.precond}, rtol {a.rtol})"),
            **summarise_pipeline(rows, nE),
            "rtol_1e-13": summarise_pipeline(tight, nE),
            "kernels_traced_step": {
                "total_kernel_ms": round(sum(v[1] for v in kern.values()), 3),
                "launches": int(sum(v[0] for v in kern.values())),
                "dominant": dom,
                "top": {k: {"ms": round(v[1], 3), "launches": v[0],
                            "GB_per_s": (round(ab[k] / (v[1] / v[0] * 1e-3) / 1e9, 1)
                                         if k in ab else None)}
                        for k, v in sorted(kern.items(), key=lambda kv: -kv[1][1])[:14]}}}
    del sysd, sys_t, U, Lam, aT_d

    # ---- L-shaped configuration ----------------------------------------------
    out_l = None
    if not a.no_lshape:
        print(f"[bench] L-shape level {a.lshape_level}", file=sys.stderr, flush=True)
        chain = build_chain(phfem, h, lshape_base, a.lshape_level)
        li = phfem.phf_mesh_get_info(chain[-1])
        laT = torch.tensor(G.per_triangle_coefficient(li.nE, 0), device=dev)
        lco = phfem.make_coeffs(a_T=laT)
        lsys, lt = phfem.alloc_system_for(li, dev)
        lU = torch.empty(li.N, dtype=torch.float64, device=dev)
        lL = torch.empty(li.L, dtype=torch.float64, device=dev)
        ms_l, samp_l = time_assembly(phfem, torch, h, chain[-1], lco, data, lsys, 30, 3)
        cold_l = time_assembly_cold(phfem, torch, h, chain[-1], lco, data, lsys, 20, dev)
        release(phfem, chain)
        out_l = {"nE": li.nE,
                 "assembly": assembly_summary(li, ms_l, samp_l,
                                              f"k_assemble@lshape_L{a.lshape_level}", cold_l)}
        if not a.no_pipeline:
            pipeline_steps(phfem, torch, h, lshape_base, a.lshape_level, lco, data, lsys, lU, lL,
                           a.rtol, 1, pc)
            rows = pipeline_steps(phfem, torch, h, lshape_base, a.lshape_level, lco, data, lsys,
                                  lU, lL, a.rtol, a.pipeline_steps, pc)
            out_l["pipeline"] = summarise_pipeline(rows, li.nE)
        print(f"[bench] L-shape {out_l}", file=sys.stderr, flush=True)
        del lsys, lt, lU, lL, laT

    # ---- plain copy probe -------------------------------------------------------
    src = torch.ones(a.copy_mib << 17, dtype=torch.float64, device=dev)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(10):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    cms = e0.elapsed_time(e1) / 10
    nbytes = 2 * src.numel() * 8
    # write-only: the assembly's traffic is mostly writes (956 of 1,124 MB at
    # the headline size), so a plain fill is the closer practical bound
    dst.fill_(2.0)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(10):
        dst.fill_(2.0)
    e1.record()
    torch.cuda.synchronize()
    fms = e0.elapsed_time(e1) / 10
    fill_gbs = dst.numel() * 8 / (fms * 1e-3) / 1e9
    copy_probe = {"MiB_each_way": a.copy_mib, "ms": round(cms, 4),
                  "GB_per_s": round(nbytes / (cms * 1e-3) / 1e9, 1),
                  "frac_of_hbm_peak": round(nbytes / (cms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                  "kernel_vs_copy": round(head["GB_per_s"] / (nbytes / (cms * 1e-3) / 1e9), 4),
                  "fill_GB_per_s": round(fill_gbs, 1),
                  "kernel_vs_fill": round(head["GB_per_s"] / fill_gbs, 4)}
    del src, dst
    print(f"[bench] copy probe {copy_probe}", file=sys.stderr, flush=True)

    # ---- Crank-Nicolson on the parabolic configuration ------------------------
    out_cn = None
    if not a.no_cn:
        print(f"[bench] Crank-Nicolson (paper mesh level {a.cn_level})", file=sys.stderr,
              flush=True)
        mc = G.paper_square(a.cn_level, bc="x_sides")
        mb = G.paper_square(0, bc="x_sides")
        cchain = [phfem.phf_mesh_create(h, mb.coords, mb.elements, mb.dirichlet, mb.neumann)]
        for _ in range(a.cn_level):
            cchain.append(phfem.phf_mesh_refine(cchain[-1]))
        dmc = cchain[-1]
        ic = phfem.phf_mesh_get_info(dmc)
        k = 1e-3
        cn = phfem.phf_cn_create(dmc, phfem.make_coeffs(), k, rtol=1e-10,
                                 iters_per_step=a.cn_chunk, precond=pc)
        # initial state: P1 values through u0 at the edge midpoints (exact
        # for the discrete constraint), Lambda = 0
        P = mc.coords[mc.elements]
        mids = np.stack([(P[:, 1] + P[:, 2]) / 2, (P[:, 2] + P[:, 0]) / 2,
                         (P[:, 0] + P[:, 1]) / 2], axis=1)
        um = np.sin(pi * mids[..., 0]) * np.sin(pi * mids[..., 1])
        U0 = np.stack([um[:, 1] + um[:, 2] - um[:, 0], um[:, 2] + um[:, 0] - um[:, 1],
                       um[:, 0] + um[:, 1] - um[:, 2]], axis=1).reshape(-1)
        U0d = torch.tensor(U0, device=dev)
        L0d = torch.zeros(ic.L, dtype=torch.float64, device=dev)
        cdata = phfem.make_data(phfem.make_fn(phfem.PHF_FN_SIN_SIN, 2 * pi * pi - 1, -1),
                                phfem.make_fn(phfem.PHF_FN_GRAD_SIN_SIN, 1, -1),
                                phfem.make_fn(phfem.PHF_FN_SIN_SIN, 1, -1))
        res = {}
        for mode, nst in (("eager", max(a.cn_steps // 10, 5)), ("graph", a.cn_steps)):
            phfem.phf_cn_set_state(cn, U0d, L0d, 0.0)
            st0 = phfem.phf_cn_run(cn, cdata, 2, use_graph=(mode == "graph"),
                                   raise_on_noconv=False)  # warm-up / capture
            print(f"[bench] cn {mode} warm-up: iters={st0.iterations} conv={st0.converged} "
                  f"rel={st0.rel_residual:.2e}", file=sys.stderr, flush=True)
            phfem.phf_cn_set_state(cn, U0d, L0d, 0.0)
            torch.cuda.synchronize()
            c0 = time.perf_counter()
            st = phfem.phf_cn_run(cn, cdata, nst, use_graph=(mode == "graph"),
                                  raise_on_noconv=False)
            torch.cuda.synchronize()
            c1 = time.perf_counter()
            res[mode] = dict(steps=nst, steps_per_s=round(nst / (c1 - c0), 1),
                             cg_iters_per_step=round(st.iterations / nst, 2),
                             all_converged=bool(st.converged),
                             worst_rel_residual=st.rel_residual)
            print(f"[bench] cn {mode}: {res[mode]}", file=sys.stderr, flush=True)
        # accuracy at t = 0.2 after the graph run: max nodal error
        Ud = torch.empty(ic.N, dtype=torch.float64, device=dev)
        phfem.phf_cn_set_state(cn, U0d, L0d, 0.0)
        phfem.phf_cn_run(cn, cdata, a.cn_steps, use_graph=True, raise_on_noconv=False)
        tf = phfem.phf_cn_get_state(cn, Ud, None)
        torch.cuda.synchronize()
        ue = np.exp(-tf) * np.sin(pi * P[..., 0]) * np.sin(pi * P[..., 1])
        err = float(np.abs(Ud.cpu().numpy().reshape(-1, 3) - ue).max())
        h1, l2 = phfem.phf_error_norms(dmc, Ud, phfem.make_fn(phfem.PHF_FN_SIN_SIN, 1, -1), tf)
        phfem.phf_cn_destroy(cn)
        for c in reversed(cchain):
            phfem.phf_mesh_destroy(c)
        out_cn = dict(workload=f"unit square, paper mesh level {a.cn_level} ({ic.nE} triangles, "
                               f"device-refined), u = exp(-t) sin(pi x) sin(pi y), k = {k}, "
                               f"CG + {a.precond}",
                      t_final=tf, max_nodal_error=err, h1_error=h1, l2_error=l2, **res)

    # ---- batched assembly (many uneven meshes in one launch) -----------------
    out_batch = None
    if not a.no_batch:
        print(f"[bench] batched assembly ({a.batch_count} instances)", file=sys.stderr,
              flush=True)
        inst = G.batch_instances(a.batch_count, 1)
        bm = [phfem.phf_mesh_create(h, mm.coords, mm.elements, mm.dirichlet, mm.neumann)
              for mm, _ in inst]
        binfo = [phfem.phf_mesh_get_info(x) for x in bm]
        bco = [phfem.make_coeffs(A=(av, 0.0, 0.0, av)) for _, av in inst]
        bdat = [phfem.make_data(phfem.make_fn(phfem.PHF_FN_SIN_COS, 2 * pi * pi * av, 0),
                                phfem.make_fn(phfem.PHF_FN_GRAD_SIN_COS, av, 0),
                                phfem.make_fn(phfem.PHF_FN_SIN_COS, 1, 0)) for _, av in inst]
        bsys = [phfem.alloc_system_for(bi, dev)[0] for bi in binfo]
        nE_tot = sum(bi.nE for bi in binfo)
        bytes_tot = sum(algorithmic_bytes(bi, has_aT=False)["k_assemble"] for bi in binfo)
        batch = phfem.phf_batch_create(h, bm)
        tuning = phfem.phf_batch_tune(batch, bco, bdat, bsys, reps=5)
        cfg = phfem.phf_batch_get_config(batch)

        def timed(fn):
            fn()
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            w0 = time.perf_counter()
            e0.record()
            for _ in range(a.batch_reps):
                fn()
            e1.record()
            torch.cuda.synchronize()
            w1 = time.perf_counter()
            return e0.elapsed_time(e1) / a.batch_reps, 1e3 * (w1 - w0) / a.batch_reps

        def per_mesh():
            for x, co_i, d_i, s_i in zip(bm, bco, bdat, bsys):
                phfem.phf_assemble(x, co_i, d_i, s_i)

        ms_b, wall_b = timed(lambda: phfem.phf_batch_assemble(batch, bco, bdat, bsys))
        ms_p, wall_p = timed(per_mesh)
        phfem.phf_batch_destroy(batch)
        for x in bm:
            phfem.phf_mesh_destroy(x)
        del bsys
        out_batch = dict(
            workload=(f"{a.batch_count} jittered unit squares, triangles log-uniform in "
                      f"[2e3, 2e5] (seed 1), {nE_tot} triangles in total, per-instance "
                      f"coefficient a ~ U[0.5, 2], fp64"),
            nE_total=nE_tot, config={"tile": cfg[0], "blocks_per_cu": cfg[1], "lanes": cfg[2],
                                     "direct": cfg[3], "gather": cfg[4]},
            batched=dict(ms=round(ms_b, 4), Melem_per_s=round(nE_tot / ms_b / 1e3, 1),
                         GB_per_s=round(bytes_tot / ms_b / 1e6, 1),
                         frac_of_hbm_peak=round(bytes_tot / ms_b / 1e6 / HBM_PEAK_GBS, 4),
                         host_wall_ms=round(wall_b, 4)),
            one_launch_per_mesh=dict(ms=round(ms_p, 4), Melem_per_s=round(nE_tot / ms_p / 1e3, 1),
                                     host_wall_ms=round(wall_p, 4)),
            speedup=round(ms_p / ms_b, 2),
            algorithmic_bytes=bytes_tot,
            # counters were taken with the staged tile of 128
            traffic=(traffic_for("k_assemble_batch", "k_assemble_batch@256_meshes")
                     if tuple(cfg) == (128, 0, 1, 0, 0) and a.batch_count == 256 else None),
            tuning=[{"tile": t_, "blocks_per_cu": b_, "lanes": l_, "direct": d_, "gather": g_,
                     "ms": round(m_, 4)} for t_, b_, l_, d_, g_, m_ in tuning])
        print(f"[bench] batch: {out_batch['batched']} vs per mesh {out_batch['one_launch_per_mesh']}",
              file=sys.stderr, flush=True)

    # ---- batched Crank-Nicolson (many uneven problems per graph launch) ------
    out_cnb = None
    if not a.no_batch:
        print(f"[bench] batched Crank-Nicolson ({a.cn_batch_count} steppers)", file=sys.stderr,
              flush=True)
        rng = np.random.default_rng(4)
        levels = rng.integers(3, 8, size=a.cn_batch_count)
        chains, steppers, states = [], [], []
        cdata = phfem.make_data(phfem.make_fn(phfem.PHF_FN_SIN_SIN, 2 * pi * pi - 1, -1),
                                phfem.make_fn(phfem.PHF_FN_GRAD_SIN_SIN, 1, -1),
                                phfem.make_fn(phfem.PHF_FN_SIN_SIN, 1, -1))
        for lev in levels:
            ch = build_chain(phfem, h, paper_base, int(lev))
            chains.append(ch)
            ii = phfem.phf_mesh_get_info(ch[-1])
            xy = np.empty((ii.nC, 2)); el = np.empty((ii.nE, 3), np.int32)
            phfem.phf_mesh_geometry(ch[-1], xy, el, None, None, phfem.PHF_HOST)
            P = xy[el]
            um = np.sin(pi * (P[:, [1, 2, 0], 0] + P[:, [2, 0, 1], 0]) / 2) * \
                np.sin(pi * (P[:, [1, 2, 0], 1] + P[:, [2, 0, 1], 1]) / 2)
            U0 = (um[:, [1, 2, 0]] + um[:, [2, 0, 1]] - um).reshape(-1)
            states.append((torch.tensor(U0, device=dev),
                           torch.zeros(ii.L, dtype=torch.float64, device=dev)))
            steppers.append(phfem.phf_cn_create(ch[-1], phfem.make_coeffs(), 1e-3, rtol=1e-10,
                                                iters_per_step=8, precond=pc))
        sizes = [phfem.phf_mesh_get_info(ch[-1]).nE for ch in chains]

        def reset():
            for cn, (u0, l0) in zip(steppers, states):
                phfem.phf_cn_set_state(cn, u0, l0, 0.0)

        nst = a.cn_batch_steps
        # one launch per stepper and step (captured graphs), steppers in turn
        reset()
        for cn in steppers:
            phfem.phf_cn_run(cn, cdata, 2, use_graph=True)
        reset()
        torch.cuda.synchronize()
        w0 = time.perf_counter()
        for cn in steppers:
            phfem.phf_cn_run(cn, cdata, nst, use_graph=True)
        torch.cuda.synchronize()
        w1 = time.perf_counter()
        cb = phfem.phf_cn_batch_create(steppers)
        reset()
        phfem.phf_cn_batch_run(cb, [cdata] * len(steppers), 2)
        reset()
        torch.cuda.synchronize()
        w2 = time.perf_counter()
        bst = phfem.phf_cn_batch_run(cb, [cdata] * len(steppers), nst)
        torch.cuda.synchronize()
        w3 = time.perf_counter()
        phfem.phf_cn_batch_destroy(cb)
        for cn in steppers:
            phfem.phf_cn_destroy(cn)
        for ch in chains:
            release(phfem, ch)
        tot = len(steppers) * nst
        out_cnb = dict(
            workload=(f"{len(steppers)} Crank-Nicolson problems on the paper mesh refined 3-7 "
                      f"times (seed 4; {min(sizes)}-{max(sizes)} triangles, {sum(sizes)} in "
                      f"total), k = 1e-3, {nst} steps each, CG + {a.precond}"),
            sizes=sizes,
            batched=dict(s=round(w3 - w2, 4), stepper_steps_per_s=round(tot / (w3 - w2), 1),
                         steps_per_s=round(nst / (w3 - w2), 1),
                         cg_iters_per_step=round(sum(x.iterations for x in bst) / tot, 2),
                         all_converged=all(bool(x.converged) for x in bst)),
            one_stepper_at_a_time=dict(s=round(w1 - w0, 4),
                                       stepper_steps_per_s=round(tot / (w1 - w0), 1)),
            speedup=round((w1 - w0) / (w3 - w2), 2))
        print(f"[bench] cn batch {out_cnb}", file=sys.stderr, flush=True)

    # ---- serving: continuous batching against one request at a time ----------
    out_serve = None
    if not a.no_serve:
        print(f"[bench] serving ({a.serve_requests} requests)", file=sys.stderr, flush=True)
        reqs = serve_requests(G, phfem, a.serve_requests, 2)
        w = phfem.phf_server_create(0, slots=2)  # warm-up (code objects, pools)
        for r in reqs[:4]:
            phfem.phf_server_wait(w, phfem.phf_server_submit(w, r))
        phfem.phf_server_destroy(w)
        runs = []
        for rate in [float(x) for x in a.serve_rates.split(",") if x]:
            for slots in (1, a.serve_slots):
                rr = serve_run(phfem, reqs, rate, slots, 3)
                print(f"[bench] serve {rr}", file=sys.stderr, flush=True)
                runs.append(rr)
        out_serve = dict(
            workload=(f"{a.serve_requests} requests (seed 2): 70% elliptic on refined structured "
                      f"unit squares, 30% Crank-Nicolson (paper mesh, k = 1e-3, 10-100 steps); "
                      f"final sizes log-uniform in [1e3, 1e6] triangles; Poisson arrivals; "
                      f"slots = 1 is one request at a time, slots = {a.serve_slots} continuous "
                      f"batching"),
            runs=runs)

    cpu = None
    if not a.no_cpu:
        print("[bench] CPU oracle baseline", file=sys.stderr, flush=True)
        cpu = cpu_baseline(a.cpu_level, a.cpu_repeat, 7)

    line = {
        "metric": METRIC,
        "value": head["Melem_per_s"],
        "unit": "Melem/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(ms_call, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": (f"numeric assembly (K, M, C, F, b_D into CSR) of the paper's "
                                f"unit-square mesh red-refined {a.level} times on the device, "
                                f"{nE} triangles, fp64, a_T~U[0.5,2] seed 0, Dirichlet x=0,1, "
                                f"Neumann y=0,1; mesh tables built before timing"),
                   "nE": nE, "n_edges": info.n_edges, "L": info.L, "N": info.N,
                   "nnz_C": info.nnz_C},
        "assembly": {**head, "HBM_GB_per_s": head["GB_per_s"]},
        "roofline": roof,
        "copy_probe": copy_probe,
        "scatter": scatter,
        "pipeline": out_pipe,
        "lshape": out_l,
        "cn": out_cn,
        "batch": out_batch,
        "cn_batch": out_cnb,
        "serve": out_serve,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
