"""phf_error_norms_noalloc (the entry point for callers that cannot
allocate) against phf_error_norms on two calls in a row, the second on a
smaller mesh: equal norms, no device allocation through the context's
allocator, and the output written on the stream without a wait."""
import numpy as np
import pytest

from paper_2401_15557_amd import meshgen as G
from parity_util import nan_vec

pytestmark = pytest.mark.gpu
PI = np.pi


def test_noalloc_norms_match_and_allocate_nothing():
    import torch
    from paper_2401_15557_amd import phfem
    dev = torch.device("cuda", 0)
    calls = {"n": 0}

    def alloc(n):
        calls["n"] += 1
        return torch.cuda.caching_allocator_alloc(n, dev, torch.cuda.current_stream(dev))

    ctx = phfem.Context(0, allocator=phfem.make_allocator(alloc,
                                                          torch.cuda.caching_allocator_delete))
    u = phfem.make_fn(phfem.PHF_FN_SIN_SIN, 1.0, -1.0)
    rng = np.random.default_rng(5)
    meshes = []
    for level in (5, 3):  # second call on a smaller mesh
        dm = phfem.Mesh(ctx, G.paper_square(level, bc="x_sides"))
        meshes.append(dm)
        # a discontinuous P1 function near u at t = 0.3: vertex values plus noise
        P = G.paper_square(level, bc="x_sides")
        xy = P.coords[P.elements]
        Uh = (np.exp(-0.3) * np.sin(PI * xy[..., 0]) * np.sin(PI * xy[..., 1])
              + 1e-3 * rng.normal(size=xy.shape[:2])).reshape(-1)
        U = torch.tensor(Uh, device=dev)
        h1, l2 = phfem.phf_error_norms(dm.handle, U, u, 0.3)
        out = nan_vec(2, dev)
        torch.cuda.synchronize()
        before = calls["n"]
        live0 = phfem.phf_mem_stats(ctx.handle)
        phfem.phf_error_norms_noalloc(dm.handle, U, u, 0.3, out)
        assert calls["n"] == before and phfem.phf_mem_stats(ctx.handle) == live0
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        print(f"level {level}: nE={dm.info.nE} h1 {h1:.16e} / {got[0]:.16e}, "
              f"l2 {l2:.16e} / {got[1]:.16e}", flush=True)
        # same partial sums in the same order; the square root is taken on the
        # device here and on the host there (both correctly rounded)
        assert abs(got[0] - h1) <= 1e-15 * h1 and abs(got[1] - l2) <= 1e-15 * l2
        assert h1 > 0 and l2 > 0
    for dm in reversed(meshes):
        dm.close()
    ctx.close()


def test_noalloc_rejects_bad_arguments():
    import torch
    from paper_2401_15557_amd import phfem
    ctx = phfem.Context(0)
    dm = phfem.Mesh(ctx, G.paper_square(1))
    U = torch.zeros(dm.info.N, dtype=torch.float64, device=ctx.device)
    out = nan_vec(2, ctx.device)
    with pytest.raises(phfem.PhfError) as ei:
        phfem.phf_error_norms_noalloc(dm.handle, U, phfem.make_fn(phfem.PHF_FN_PAPER_F, 1, 0),
                                      0.0, out)
    assert ei.value.code == phfem.PHF_EINVAL
    assert phfem.load().phf_error_norms_noalloc(dm.handle, None, None, 0.0, None) == \
        phfem.PHF_EINVAL
    dm.close()
    ctx.close()
