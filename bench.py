"""Benchmark of the primal hybrid FEM hot path on one MI355X.

  python bench.py [--gpus 1] [--steps K] [--warmup W]

Workload (the elliptic benchmark configuration): L-shaped domain
[-1,1]^2 minus [0,1]x[-1,0], 12 triangles red-refined 9 times =
3,145,728 triangles, fp64, per-triangle coefficient a_T ~ U[0.5, 2]
(seed 0), Dirichlet u_D = 1 on the two re-entrant edges, Neumann g = 1 on
the rest, f = 2 pi^2 sin(pi x) cos(pi y). Inputs are synthetic and resident
in device memory before timing starts.

One step = one pass of the elliptic hot path: the 12-triangle L-shape
(device-resident) is validated and given its edge tables (phf_mesh_create),
red-refined 9 times on the device, each level getting its edge tables,
boundary classification and CSR patterns (phf_mesh_refine); the numeric
assembly of K, M, C, F, b_D runs on the finest mesh (phf_assemble), and the
saddle-point system is solved to a relative residual of 1e-10 by
conjugate gradients preconditioned with a V-cycle over the refinement levels
(phf_solve); then the meshes are released. `value` is finest-mesh elements
per second through that step (Melem/s). `--precond jacobi` solves with the
Jacobi preconditioner instead.

The JSON line also carries, measured in the same process:
  rows      host-observed milliseconds between the calls of the step (the
            library's calls return before their GPU work ends, so the mesh
            build and the assembly run on in the next rows; the last row,
            the release, waits for the solve's final kernels) and solver
            iterations;
  assembly  the numeric assembly alone (the paper's timed computation):
            Melem/s, algorithmic GB/s and fraction of the HBM peak;
  cn        Crank-Nicolson steps/s on the parabolic configuration (unit
            square, 1,048,576 triangles, k = 1e-3, 200 steps), replaying one
            captured HIP graph per step, and eagerly;
  roofline  the dominant kernel of the step, from HIP events on the
            library's stream over the timed region;
  cpu_baseline  the CPU oracle on a bounded sample, one core.
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
    (12 B/elem), a_T (8 B/elem), the two end nodes of each multiplier row
    (8 B/row); write K and M (72 B/elem each), F (24 B/elem), C (8 B/nnz)
    and b_D (8 B/row).
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
    weight codes) + 8 (x in and out) = 32 B/fine row + 4 B/coarse row; restriction from level l: per coarse triangle 36 B of fine
    row ids, 4 B code word, 12 B of sums written, plus the fine residual once
    (4 B/fine row), then per coarse row 8 (positions) + 8 (two sums) + 4
    (dinv) in, 4 (D^-1 b) + 4 (first sweep) out = 28 B.
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


def traffic_for(kernel):
    """HBM traffic per launch from the committed counter summary, if it was
    taken on the current sources of that kernel; otherwise None."""
    p = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        rec = json.load(open(p))
    except (OSError, ValueError):
        return None
    k = rec.get("kernels", {}).get(kernel)
    if not k:
        return None
    try:
        if k.get("hash") != sources_hash(k.get("sources", [])):
            return None
    except OSError:
        return None
    return k.get("bytes_per_launch")


def cpu_baseline(level=7, repeat=2):
    env = dict(os.environ, OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1", MKL_NUM_THREADS="1")
    r = subprocess.run([sys.executable, "-m", "oracle.baseline", "--level", str(level),
                        "--repeat", str(repeat), "--solve"], cwd=ROOT, env=env,
                       capture_output=True, text=True, timeout=600)
    if r.returncode != 0:
        return {"error": r.stderr[-500:]}
    o = json.loads(r.stdout.strip().splitlines()[-1])
    return {"value": o["nE"] / o["total_s"] / 1e6, "unit": "Melem/s", "cores": 1,
            "kind": "oracle",
            "sample": (f"L-shape level {level} ({o['nE']} triangles), same data; topology + "
                       f"assembly + saddle CSR + sparse LU solve, best of {repeat}; "
                       f"stage s: topo {o['topology_s']:.3f} asm {o['assembly_s']:.3f} "
                       f"saddle {o['saddle_s']:.3f} solve {o['solve_s']:.3f}")}


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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--level", type=int, default=9, help="L-shape refinement level")
    ap.add_argument("--asm-reps", type=int, default=30)
    ap.add_argument("--cn-level", type=int, default=9)
    ap.add_argument("--cn-steps", type=int, default=200)
    ap.add_argument("--cn-chunk", type=int, default=8,
                    help="expected CG iterations of the first time step")
    ap.add_argument("--no-cn", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--rtol", type=float, default=1e-10)
    ap.add_argument("--mode", choices=("full", "assembly"), default="full",
                    help="assembly: only the numeric assembly on the benchmark mesh plus one "
                         "plain device copy of --copy-mib MiB (for hardware-counter runs)")
    ap.add_argument("--copy-mib", type=int, default=None,
                    help="size of the plain device copy run for counter calibration "
                         "(default 512 in assembly mode, none in full mode)")
    ap.add_argument("--precond", choices=("multigrid", "jacobi"), default="multigrid")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--serve-requests", type=int, default=120)
    ap.add_argument("--serve-rates", type=str, default="20,40,80",
                    help="Poisson arrival rates (requests/s) to sweep")
    ap.add_argument("--serve-slots", type=int, default=4)
    ap.add_argument("--batch-count", type=int, default=256)
    ap.add_argument("--batch-reps", type=int, default=20)
    a = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if a.gpus != 1 or world != 1:
        print("bench.py runs on exactly one GPU: this build has no multi-GPU path "
              "(how the path would shard is described in DESIGN.md).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2401_15557_amd import meshgen as G
    from paper_2401_15557_amd import phfem

    dev = torch.device("cuda", 0)
    pi = np.pi
    print(f"[bench] building inputs (L-shape level {a.level})", file=sys.stderr, flush=True)
    m = G.lshape(a.level)
    base = G.lshape(0)
    aT = G.per_triangle_coefficient(m.nE, 0)
    xy_d = torch.tensor(m.coords, device=dev)
    el_d = torch.tensor(m.elements, device=dev)
    D_d = torch.tensor(m.dirichlet, device=dev)
    N_d = torch.tensor(m.neumann, device=dev)
    bxy_d = torch.tensor(base.coords, device=dev)
    bel_d = torch.tensor(base.elements, device=dev)
    bD_d = torch.tensor(base.dirichlet, device=dev)
    bN_d = torch.tensor(base.neumann, device=dev)
    aT_d = torch.tensor(aT, device=dev)
    pc = phfem.PHF_PRECOND_MULTIGRID if a.precond == "multigrid" else phfem.PHF_PRECOND_JACOBI
    ctx = phfem.Context(0)
    co = phfem.make_coeffs(a_T=aT_d)
    data = phfem.make_data(phfem.make_fn(phfem.PHF_FN_SIN_COS, 2 * pi * pi, 0),
                           phfem.make_fn(phfem.PHF_FN_CONST, 1.0),
                           phfem.make_fn(phfem.PHF_FN_CONST, 1.0))
    h = ctx.handle
    out = {}

    if a.mode == "assembly":
        mh = phfem.phf_mesh_create(h, xy_d, el_d, D_d, N_d, phfem.PHF_DEVICE)
        info = phfem.phf_mesh_get_info(mh)
        sysd, t = phfem.alloc_system_for(info, dev)
        for _ in range(a.asm_reps):
            phfem.phf_assemble(mh, co, data, sysd)
        src = torch.ones((a.copy_mib or 512) << 17, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        phfem.phf_mesh_destroy(mh)
        ab = algorithmic_bytes(info)
        print(json.dumps({"mode": "assembly", "nE": info.nE, "launches": a.asm_reps,
                          "algorithmic_bytes_per_launch": ab["k_assemble"],
                          "copy_bytes_each_way": src.numel() * 8}))
        return

    def one_step(rows):
        t0 = time.perf_counter()
        chain = [phfem.phf_mesh_create(h, bxy_d, bel_d, bD_d, bN_d, phfem.PHF_DEVICE)]
        for _ in range(a.level):
            chain.append(phfem.phf_mesh_refine(chain[-1]))
        mh = chain[-1]
        t1 = time.perf_counter()
        if "sys" not in out:
            # sizes for the caller-owned outputs, allocated once (the mesh is
            # the same every step)
            info = phfem.phf_mesh_get_info(mh)
            sysd = phfem.phf_system()
            t = dict(K=torch.empty(info.nnz_K, dtype=torch.float64, device=dev),
                     M=torch.empty(info.nnz_K, dtype=torch.float64, device=dev),
                     C=torch.empty(info.nnz_C, dtype=torch.float64, device=dev),
                     F=torch.empty(info.N, dtype=torch.float64, device=dev),
                     bD=torch.empty(info.L, dtype=torch.float64, device=dev),
                     U=torch.empty(info.N, dtype=torch.float64, device=dev),
                     Lam=torch.empty(info.L, dtype=torch.float64, device=dev))
            for k in ("K", "M", "C", "F", "bD"):
                setattr(sysd, k, t[k].data_ptr())
            out["sys"], out["t"], out["info"] = sysd, t, info
            out["level_nf"] = [phfem.phf_mesh_get_info(c).n_free for c in chain]
            out["level_nE"] = [phfem.phf_mesh_get_info(c).nE for c in chain]
        sysd, t = out["sys"], out["t"]
        phfem.phf_assemble(mh, co, data, sysd)
        t2 = time.perf_counter()
        st = phfem.phf_solve(mh, co, sysd, t["U"], t["Lam"], rtol=a.rtol, max_iter=200000,
                             check_every=32 if pc == phfem.PHF_PRECOND_JACOBI else 0,
                             precond=pc)
        t3 = time.perf_counter()
        for c in reversed(chain):
            phfem.phf_mesh_destroy(c)
        t4 = time.perf_counter()
        rows.append(dict(mesh_ms=1e3 * (t1 - t0), assemble_ms=1e3 * (t2 - t1),
                         solve_ms=1e3 * (t3 - t2), release_ms=1e3 * (t4 - t3),
                         iterations=st.iterations, rel_residual=st.rel_residual))

    print(f"[bench] warmup {a.warmup} step(s), nE={m.nE}", file=sys.stderr, flush=True)
    warm = []
    for _ in range(a.warmup):
        one_step(warm)
        print(f"[bench] warmup step {warm[-1]}", file=sys.stderr, flush=True)
    # one untimed step with every launch traced: per-kernel breakdown and the
    # dominant kernel
    phfem.phf_trace_enable(h, True)
    phfem.phf_trace_reset(h)
    prof = []
    one_step(prof)
    kern = phfem.phf_trace_dump(h)
    info = out["info"]
    nE = info.nE
    ab = algorithmic_bytes(info, level_nf=out["level_nf"], level_nE=out["level_nE"],
                           jacobi=pc == phfem.PHF_PRECOND_JACOBI)
    dname = max(kern.items(), key=lambda kv: kv[1][1])[0]
    print(f"[bench] traced step {prof[-1]}; dominant kernel {dname}", file=sys.stderr, flush=True)
    # timed steps; only the dominant kernel carries events
    phfem.phf_trace_filter(h, dname)
    phfem.phf_trace_reset(h)
    rows = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(a.steps):
        one_step(rows)
        print(f"[bench] step {s}: {rows[-1]}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    samples = phfem.phf_trace_samples(h, dname)
    phfem.phf_trace_filter(h, None)
    phfem.phf_trace_enable(h, False)
    ms_step = 1e3 * (t1 - t0) / a.steps
    # The launches queued behind the iteration that converges return at once
    # on the device (a few microseconds, no bytes moved): they are not part of
    # the kernel's average.
    med = sorted(samples)[len(samples) // 2] if samples else 0.0
    work = [d for d in samples if d >= 0.25 * med]

    roof = None
    if dname in ab and work:
        avg_s = sum(work) / len(work) / 1e3
        ach = ab[dname] / avg_s / 1e9
        tr = traffic_for(dname)
        roof = {"bound": "hbm", "kernel": dname, "achieved": round(ach, 1),
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4),
                "traffic": tr, "avg_launch_us": round(avg_s * 1e6, 3), "launches": len(work),
                "skipped_launches": len(samples) - len(work),
                "algorithmic_bytes_per_launch": ab[dname]}

    # numeric assembly alone (the computation the paper times)
    print("[bench] assembly-only timing", file=sys.stderr, flush=True)
    mh = phfem.phf_mesh_create(h, xy_d, el_d, D_d, N_d, phfem.PHF_DEVICE)
    sysd = out["sys"]
    for _ in range(3):
        phfem.phf_assemble(mh, co, data, sysd)
    phfem.phf_synchronize(h)
    phfem.phf_trace_enable(h, True)
    phfem.phf_trace_reset(h)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(a.asm_reps):
        phfem.phf_assemble(mh, co, data, sysd)
    ev1.record()
    torch.cuda.synchronize()
    cnt, tot = phfem.phf_trace_query(h, "k_assemble")
    phfem.phf_trace_enable(h, False)
    asm_us = tot / cnt * 1e3
    wall_us = ev0.elapsed_time(ev1) / a.asm_reps * 1e3
    asm_gbs = ab["k_assemble"] / (asm_us * 1e-6) / 1e9
    out_asm = {"Melem_per_s": round(nE / asm_us, 1), "kernel_us": round(asm_us, 2),
               "stream_us_per_call": round(wall_us, 2),
               "algorithmic_bytes": ab["k_assemble"],
               "bytes_per_elem": round(ab["k_assemble"] / nE, 1),
               "GB_per_s": round(asm_gbs, 1), "frac_of_hbm_peak": round(asm_gbs / HBM_PEAK_GBS, 4),
               "traffic": traffic_for("k_assemble"), "launches": cnt}
    phfem.phf_mesh_destroy(mh)

    # Crank-Nicolson on the parabolic configuration
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
        phfem.phf_cn_destroy(cn)
        for c in reversed(cchain):
            phfem.phf_mesh_destroy(c)
        out_cn = dict(workload=f"unit square, paper mesh level {a.cn_level} ({ic.nE} triangles, "
                               f"device-refined), u = exp(-t) sin(pi x) sin(pi y), k = {k}, "
                               f"CG + {a.precond}",
                      t_final=tf, max_nodal_error=err, **res)

    # batched assembly (many uneven meshes in one launch) against one
    # phf_assemble launch per mesh
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
            nE_total=nE_tot, config={"tile": cfg[0], "blocks_per_cu": cfg[1]},
            batched=dict(ms=round(ms_b, 4), Melem_per_s=round(nE_tot / ms_b / 1e3, 1),
                         GB_per_s=round(bytes_tot / ms_b / 1e6, 1),
                         frac_of_hbm_peak=round(bytes_tot / ms_b / 1e6 / HBM_PEAK_GBS, 4),
                         host_wall_ms=round(wall_b, 4)),
            one_launch_per_mesh=dict(ms=round(ms_p, 4), Melem_per_s=round(nE_tot / ms_p / 1e3, 1),
                                     host_wall_ms=round(wall_p, 4)),
            speedup=round(ms_p / ms_b, 2),
            algorithmic_bytes=bytes_tot,
            tuning=[{"tile": t_, "blocks_per_cu": b_, "ms": round(m_, 4)} for t_, b_, m_ in tuning])
        print(f"[bench] batch: {out_batch['batched']} vs per mesh {out_batch['one_launch_per_mesh']}",
              file=sys.stderr, flush=True)

    # serving: continuous batching against one request at a time
    out_serve = None
    if not a.no_serve:
        print(f"[bench] serving ({a.serve_requests} requests)", file=sys.stderr, flush=True)
        reqs = serve_requests(G, phfem, a.serve_requests, 2)
        # warm-up (code objects, pools)
        w = phfem.phf_server_create(0, slots=2)
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

    if a.copy_mib:
        # a plain copy of known size: the reference for hardware byte counters
        src = torch.ones(a.copy_mib << 17, dtype=torch.float64, device=dev)
        torch.empty_like(src).copy_(src)
        torch.cuda.synchronize()
        del src

    cpu = None
    if not a.no_cpu:
        print("[bench] CPU oracle baseline", file=sys.stderr, flush=True)
        cpu = cpu_baseline()

    mean = {k: float(np.mean([r[k] for r in rows])) for k in rows[0]}
    line = {
        "metric": METRIC,
        "value": round(nE / (ms_step * 1e-3) / 1e6, 3),
        "unit": "Melem/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(ms_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": (f"elliptic L-shape, {nE} triangles (12 x 4^{a.level}), fp64, "
                                f"a_T~U[0.5,2] seed 0, mixed BCs; step = base mesh upload + "
                                f"{a.level} device red refinements with topology and patterns + "
                                f"assembly + saddle solve (CG + {a.precond}, rtol {a.rtol})"),
                   "nE": nE, "n_edges": info.n_edges, "L": info.L, "N": info.N},
        "rows": {"refine_topology_patterns_ms": round(mean["mesh_ms"], 3),
                 "assembly_ms": round(mean["assemble_ms"], 3),
                 "solve_ms": round(mean["solve_ms"], 3),
                 "release_ms": round(mean["release_ms"], 3),
                 "solve_iterations": int(mean["iterations"]),
                 "solve_rel_residual": mean["rel_residual"]},
        "assembly": out_asm,
        "cn": out_cn,
        "batch": out_batch,
        "serve": out_serve,
        "roofline": roof,
        # from the one fully traced (untimed) step
        "kernels_traced_step": {
            "total_kernel_ms": round(sum(v[1] for v in kern.values()), 3),
            "launches": int(sum(v[0] for v in kern.values())),
            "top": {k: {"ms": round(v[1], 3), "launches": v[0],
                        "GB_per_s": (round(ab[k] / (v[1] / v[0] * 1e-3) / 1e9, 1)
                                     if k in ab else None)}
                    for k, v in sorted(kern.items(), key=lambda kv: -kv[1][1])[:14]},
            "all": {k: [v[0], round(v[1], 4)]
                    for k, v in sorted(kern.items(), key=lambda kv: -kv[1][1])}},
        "cpu_baseline": cpu,
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
