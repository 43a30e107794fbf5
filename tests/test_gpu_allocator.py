"""The context's allocator hook: every device block the library holds comes
from the caller's allocator (here torch's caching allocator behind a
counting wrapper), through mesh builds, refinement, assembly, the
multigrid solve, Crank-Nicolson with graphs, error norms and batches; all of
it goes back on release, and results equal those of a context on the
library's own hipMalloc bit for bit."""
import numpy as np
import pytest

from paper_2401_15557_amd import meshgen as G
from parity_util import NAN, nan_vec

pytestmark = pytest.mark.gpu
PI = np.pi


class Counting:
    def __init__(self, dev, stream):
        import torch
        self.torch = torch
        self.dev, self.stream = dev, stream
        self.live = {}
        self.calls = 0
        self.total = 0

    def alloc(self, n):
        p = self.torch.cuda.caching_allocator_alloc(n, self.dev, self.stream)
        self.live[p] = n
        self.calls += 1
        self.total += n
        return p

    def free(self, p):
        assert p in self.live, hex(p)
        del self.live[p]
        self.torch.cuda.caching_allocator_delete(p)

    def live_bytes(self):
        return sum(self.live.values())


def _workload(ctx, phfem):
    """Refined L-shape, assembly, multigrid CG; refined paper square, CN with
    graphs, error norms; a batch of two meshes. Returns host copies."""
    import torch
    out = {}
    chain = [phfem.Mesh(ctx, G.lshape(0))]
    for _ in range(4):
        chain.append(chain[-1].refine())
    dm = chain[-1]
    aT = torch.tensor(G.per_triangle_coefficient(dm.info.nE, 0), device=ctx.device)
    co = phfem.make_coeffs(a_T=aT)
    d = phfem.make_data(phfem.make_fn(phfem.PHF_FN_SIN_COS, 2 * PI * PI, 0),
                        phfem.make_fn(phfem.PHF_FN_CONST, 1), phfem.make_fn(phfem.PHF_FN_CONST, 1))
    s, t = phfem.alloc_system(dm, fill=NAN)
    phfem.phf_assemble(dm.handle, co, d, s)
    U = nan_vec(dm.info.N, ctx.device)
    Lam = nan_vec(dm.info.L, ctx.device)
    st = phfem.phf_solve(dm.handle, co, s, U, Lam, rtol=1e-12,
                         precond=phfem.PHF_PRECOND_MULTIGRID)
    assert st.converged
    out["K"], out["U"], out["Lam"] = t["K"].cpu().numpy(), U.cpu().numpy(), Lam.cpu().numpy()

    cchain = [phfem.Mesh(ctx, G.paper_square(0, bc="x_sides"))]
    for _ in range(4):
        cchain.append(cchain[-1].refine())
    cm = cchain[-1]
    cd = phfem.make_data(phfem.make_fn(phfem.PHF_FN_SIN_SIN, 2 * PI * PI - 1, -1),
                         phfem.make_fn(phfem.PHF_FN_GRAD_SIN_SIN, 1, -1),
                         phfem.make_fn(phfem.PHF_FN_SIN_SIN, 1, -1))
    cn = phfem.phf_cn_create(cm.handle, phfem.make_coeffs(), 1e-2, rtol=1e-12,
                             precond=phfem.PHF_PRECOND_MULTIGRID)
    U0 = torch.zeros(cm.info.N, dtype=torch.float64, device=ctx.device)
    L0 = torch.zeros(cm.info.L, dtype=torch.float64, device=ctx.device)
    phfem.phf_cn_set_state(cn, U0, L0, 0.0)
    phfem.phf_cn_run(cn, cd, 6, use_graph=True)
    Uc = nan_vec(cm.info.N, ctx.device)
    phfem.phf_cn_get_state(cn, Uc, None)
    out["Ucn"] = Uc.cpu().numpy()
    out["norms"] = phfem.phf_error_norms(cm.handle, Uc, phfem.make_fn(phfem.PHF_FN_SIN_SIN, 1, -1),
                                         0.06)
    phfem.phf_cn_destroy(cn)

    b = phfem.phf_batch_create(ctx.handle, [chain[2].handle, cchain[3].handle])
    bs = [phfem.alloc_system(x, fill=NAN) for x in (chain[2], cchain[3])]
    phfem.phf_batch_assemble(b, [phfem.make_coeffs()] * 2, [d, cd], [x[0] for x in bs])
    out["batchK"] = np.concatenate([x[1]["K"].cpu().numpy() for x in bs])
    phfem.phf_batch_destroy(b)
    for c in reversed(cchain):
        c.close()
    for c in reversed(chain):
        c.close()
    return out


def test_every_device_byte_through_the_allocator():
    import torch
    from paper_2401_15557_amd import phfem
    dev = torch.device("cuda", 0)
    stream = torch.cuda.current_stream(dev)
    cnt = Counting(dev, stream)
    al = phfem.make_allocator(cnt.alloc, cnt.free)
    ctx = phfem.Context(0, allocator=al)
    h = ctx.handle
    live, cached = phfem.phf_mem_stats(h)
    assert cnt.calls >= 1 and live + cached == cnt.live_bytes()  # the context's flag words
    got = _workload(ctx, phfem)
    live, cached = phfem.phf_mem_stats(h)
    print(f"allocator calls {cnt.calls}, bytes {cnt.total}; pool live {live} cached {cached}",
          flush=True)
    assert cnt.calls > 50 and cnt.total > 2**20
    # everything the pool holds (live or cached) is exactly what the caller's
    # allocator handed out and has not had back
    assert live + cached == cnt.live_bytes()
    phfem.phf_release_cache(h)
    live, cached = phfem.phf_mem_stats(h)
    assert cached == 0 and live == cnt.live_bytes()
    ctx.close()
    assert cnt.live == {}

    # the same work on the library's own hipMalloc gives identical results
    ref_ctx = phfem.Context(0, allocator=False)
    ref = _workload(ref_ctx, phfem)
    ref_ctx.close()
    for k in ("K", "U", "Lam", "Ucn", "batchK"):
        assert got[k].tobytes() == ref[k].tobytes(), k
    assert got["norms"] == ref["norms"]


def test_allocator_failure_reports_enomem():
    import torch
    from paper_2401_15557_amd import phfem
    dev = torch.device("cuda", 0)
    cnt = Counting(dev, torch.cuda.current_stream(dev))
    budget = {"left": 4 << 20}

    def alloc(n):
        if n > budget["left"]:
            return 0
        budget["left"] -= n
        return cnt.alloc(n)

    def free(p):
        budget["left"] += cnt.live[p]
        cnt.free(p)

    al = phfem.make_allocator(alloc, free)
    ctx = phfem.Context(0, allocator=al)
    with pytest.raises(phfem.PhfError) as ei:
        phfem.Mesh(ctx, G.lshape(6))
    assert ei.value.code == phfem.PHF_ENOMEM
    # the context is still usable with a mesh that fits
    dm = phfem.Mesh(ctx, G.lshape(1))
    assert dm.info.nE == 48
    dm.close()
    ctx.close()
    assert cnt.live == {}
