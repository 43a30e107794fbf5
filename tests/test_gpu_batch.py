"""Batched assembly: many meshes of uneven size in one launch. Every launch
shape gives outputs bit-identical to one phf_assemble per mesh, and those
match the oracle."""
import numpy as np
import pytest

from paper_2401_15557_amd import meshgen as G
from parity_util import NAN, assert_close_scaled, assert_written, block_scale, row_scale_fast

pytestmark = pytest.mark.gpu
PI = np.pi
KEYS = ("K", "M", "C", "F", "bD")


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_2401_15557_amd import phfem
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    c = phfem.Context(0)
    yield c
    c.close()


def _instances(phfem, ctx, count, seed, tmin=200, tmax=6000):
    inst = G.batch_instances(count, seed, tmin=tmin, tmax=tmax)
    meshes = [phfem.Mesh(ctx, m) for m, _ in inst]
    coeffs = [phfem.make_coeffs(A=(a, 0.0, 0.0, a)) for _, a in inst]
    data = [phfem.make_data(phfem.make_fn(phfem.PHF_FN_SIN_COS, 2 * PI * PI * a, 0),
                            phfem.make_fn(phfem.PHF_FN_GRAD_SIN_COS, a, 0),
                            phfem.make_fn(phfem.PHF_FN_SIN_COS, 1, 0)) for _, a in inst]
    return inst, meshes, coeffs, data


def _host(t):
    return {k: t[k].cpu().numpy().copy() for k in KEYS}


def test_batch_bit_identical_all_shapes(ctx):
    from paper_2401_15557_amd import phfem
    inst, meshes, coeffs, data = _instances(phfem, ctx, 12, 11)
    print("sizes", [m.nE for m, _ in inst], flush=True)
    ref = []
    for dm, co, d in zip(meshes, coeffs, data):
        s, t = phfem.alloc_system(dm, fill=NAN)
        phfem.phf_assemble(dm.handle, co, d, s)
        assert_written(t, dm.info)
        ref.append(_host(t))
    outs = [phfem.alloc_system(dm, fill=NAN) for dm in meshes]
    b = phfem.phf_batch_create(ctx.handle, [dm.handle for dm in meshes])
    shapes = [(tile, bpc, 1, 0, 0) for tile in (64, 128, 256) for bpc in (0, 1, 4)]
    shapes += [(tile, 0, 1, 1, 0) for tile in (64, 128, 256)]  # per-thread stores
    shapes += [(tile, 0, 4, 0, 0) for tile in (64, 128, 256)]  # four lanes per triangle
    shapes += [(tile, 0, 1, 0, 1) for tile in (64, 128, 256)]  # gathered coordinates
    try:
        for shape in shapes:
            for s, t in outs:  # poison the outputs
                for k in KEYS:
                    t[k].fill_(np.nan)
            phfem.phf_batch_set_config(b, *shape)
            assert phfem.phf_batch_get_config(b) == shape
            phfem.phf_batch_assemble(b, coeffs, data, [s for s, _ in outs])
            for i, (s, t) in enumerate(outs):
                got = _host(t)
                for k in KEYS:
                    assert got[k].tobytes() == ref[i][k].tobytes(), (shape, i, k)
        with pytest.raises(phfem.PhfError):
            phfem.phf_batch_set_config(b, 128, 2, 4, 0)  # persistent grids stage in LDS
        with pytest.raises(phfem.PhfError):
            phfem.phf_batch_set_config(b, 128, 0, 1, 1, 1)  # one form at a time
        res = phfem.phf_batch_tune(b, coeffs, data, [s for s, _ in outs], reps=2)
        print("tuning", res, "->", phfem.phf_batch_get_config(b), flush=True)
        assert len(res) == 21 and all(r[5] > 0 for r in res)
        best = min(res, key=lambda r: r[5])
        assert phfem.phf_batch_get_config(b) == best[:5]
        for i, (s, t) in enumerate(outs):
            got = _host(t)
            for k in KEYS:
                assert got[k].tobytes() == ref[i][k].tobytes()
    finally:
        phfem.phf_batch_destroy(b)
    for dm in meshes:
        dm.close()


def test_batch_with_D_and_aT_and_oracle(ctx, oracle):
    import torch
    from paper_2401_15557_amd import phfem
    inst, meshes, _, data = _instances(phfem, ctx, 5, 12)
    aTs = [G.per_triangle_coefficient(m.nE, 20 + i) for i, (m, _) in enumerate(inst)]
    aT_d = [torch.tensor(a, device=ctx.device) for a in aTs]
    coeffs = [phfem.make_coeffs(p=(0.5, -1.0), delta=1.0, a_T=a) for a in aT_d]
    outs = [phfem.alloc_system(dm, with_D=True, fill=NAN) for dm in meshes]
    b = phfem.phf_batch_create(ctx.handle, [dm.handle for dm in meshes])
    try:
        single = []
        for dm, co, d in zip(meshes, coeffs, data):
            s, t = phfem.alloc_system(dm, with_D=True, fill=NAN)
            phfem.phf_assemble(dm.handle, co, d, s)
            assert_written(t, dm.info)
            single.append({k: t[k].cpu().numpy() for k in KEYS + ("D",)})
        # staged persistent grid, four lanes per triangle, per-thread stores
        for shape in ((128, 2, 1, 0, 0), (64, 0, 4, 0, 0), (256, 0, 1, 1, 0), (128, 0, 1, 0, 1)):
            for _, t in outs:
                for k in KEYS + ("D",):
                    t[k].fill_(np.nan)
            phfem.phf_batch_set_config(b, *shape)
            phfem.phf_batch_assemble(b, coeffs, data, [s for s, _ in outs])
            for i in range(len(meshes)):
                for k in KEYS + ("D",):
                    gb, gs = outs[i][1][k].cpu().numpy(), single[i][k]
                    nd = int((gb != gs).sum())
                    assert nd == 0, (shape, i, k, nd, gb.size, float(np.nanmax(np.abs(gb - gs))),
                                     float(np.abs(gs).max()))
        # one instance against the oracle (values per scaled tolerance)
        m, a = inst[0]
        asm = oracle.assemble(m, oracle.mesh_tables(m), p=(0.5, -1.0), aT=aTs[0],
                              f=oracle.fn(oracle.FN_SIN_COS, 2 * PI * PI * a, 0),
                              g=oracle.fn(oracle.FN_GRAD_SIN_COS, a, 0),
                              uD=oracle.fn(oracle.FN_SIN_COS, 1, 0))
        t0 = outs[0][1]
        for key in ("K", "M", "D"):
            o = asm[key]
            assert_close_scaled(t0[key].cpu().numpy(), o, block_scale(o, 9), key)
        nc = len(asm["C"])
        assert_close_scaled(t0["C"].cpu().numpy()[:nc], asm["C"],
                            row_scale_fast(asm["C"], asm["C_rowptr"]), "C")
        for key in ("F", "bD"):
            o = asm[key]
            sc = np.full(len(o), np.abs(o).max() if len(o) else 1.0)
            assert_close_scaled(t0[key].cpu().numpy()[:len(o)], o, sc, key)
        # a_T for some instances only is rejected
        coeffs_mixed = list(coeffs)
        coeffs_mixed[1] = phfem.make_coeffs(p=(0.5, -1.0), delta=1.0)
        with pytest.raises(phfem.PhfError) as ei:
            phfem.phf_batch_assemble(b, coeffs_mixed, data, [s for s, _ in outs])
        assert ei.value.code == phfem.PHF_EINVAL
    finally:
        phfem.phf_batch_destroy(b)
    for dm in meshes:
        dm.close()
