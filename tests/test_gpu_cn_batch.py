"""Batched Crank-Nicolson (Section 4.1 for many problems at once): uneven
steppers advanced together by two HIP graphs per step give, bit for bit, the
states phf_cn_run gives each of them alone; one of them is checked against
the oracle's Crank-Nicolson (sparse LU of M+)."""
import numpy as np
import pytest

from paper_2401_15557_amd import meshgen as G
from parity_util import nan_vec

pytestmark = pytest.mark.gpu
PI = np.pi


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_2401_15557_amd import phfem
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    c = phfem.Context(0)
    yield c
    c.close()


def _rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def _instances():
    """Eight uneven problems: paper mesh (Dirichlet x = 0, 1) refined 1-5
    times with multigrid, the L-shape refined 1-3 times with Jacobi; time
    steps, coefficients, reaction and data scales differ."""
    out = []
    for i, lev in enumerate((1, 2, 3, 4, 5)):
        out.append(dict(base=G.paper_square(0, bc="x_sides"), levels=lev, k=[0.02, 0.01, 0.005,
                                                                          0.01, 0.002][i],
                        A=1.0 + 0.25 * i, delta=0.5 * (i % 2), scale=1.0 + i, mg=True))
    for j, lev in enumerate((1, 2, 3)):
        out.append(dict(base=G.lshape(0), levels=lev, k=[0.01, 0.02, 0.005][j], A=1.0,
                        delta=0.0, scale=0.5 + j, mg=False))
    return out


def _make(ctx, phfem, torch, inst):
    """Device mesh chain, one stepper, its data and initial state."""
    chain = [phfem.Mesh(ctx, inst["base"])]
    for _ in range(inst["levels"]):
        chain.append(chain[-1].refine())
    dm = chain[-1]
    co = phfem.make_coeffs(A=(inst["A"], 0, 0, inst["A"]), delta=inst["delta"])
    pc = phfem.PHF_PRECOND_MULTIGRID if inst["mg"] else phfem.PHF_PRECOND_JACOBI
    xy, el, _, _ = dm.geometry()
    P = xy[el]
    mids = np.stack([(P[:, 1] + P[:, 2]) / 2, (P[:, 2] + P[:, 0]) / 2, (P[:, 0] + P[:, 1]) / 2], 1)
    um = inst["scale"] * np.sin(PI * mids[..., 0]) * np.sin(PI * mids[..., 1])
    U0 = np.stack([um[:, 1] + um[:, 2] - um[:, 0], um[:, 2] + um[:, 0] - um[:, 1],
                   um[:, 0] + um[:, 1] - um[:, 2]], axis=1).reshape(-1)
    a = inst["A"]
    data = phfem.make_data(
        phfem.make_fn(phfem.PHF_FN_SIN_SIN, inst["scale"] * (2 * PI * PI * a - 1 + inst["delta"]), -1),
        phfem.make_fn(phfem.PHF_FN_GRAD_SIN_SIN, inst["scale"] * a, -1),
        phfem.make_fn(phfem.PHF_FN_SIN_SIN, inst["scale"], -1))

    def stepper():
        cn = phfem.phf_cn_create(dm.handle, co, inst["k"], rtol=1e-12, iters_per_step=6,
                                 precond=pc)
        phfem.phf_cn_set_state(cn, torch.tensor(U0, device=ctx.device),
                               torch.zeros(dm.info.L, dtype=torch.float64, device=ctx.device), 0.0)
        return cn

    return chain, dm, data, U0, stepper


def _state(ctx, phfem, cn, dm):
    import torch
    U = nan_vec(dm.info.N, ctx.device)
    L = nan_vec(dm.info.L, ctx.device)
    t = phfem.phf_cn_get_state(cn, U, L)
    torch.cuda.synchronize()
    return U.cpu().numpy(), L.cpu().numpy(), t


def test_cn_batch_equals_single_steppers(ctx, oracle):
    import torch
    from paper_2401_15557_amd import phfem
    insts = _instances()
    made = [_make(ctx, phfem, torch, inst) for inst in insts]
    print("sizes", [m[1].info.nE for m in made], flush=True)
    batch_cns = [m[4]() for m in made]
    alone_cns = [m[4]() for m in made]
    data = [m[2] for m in made]
    b = phfem.phf_cn_batch_create(batch_cns)
    try:
        for nst in (7, 4):  # two runs: budgets from the first carry into the second
            st = phfem.phf_cn_batch_run(b, data, nst)
            assert all(s.converged for s in st), [(s.iterations, s.rel_residual) for s in st]
            for cn, d in zip(alone_cns, data):
                s1 = phfem.phf_cn_run(cn, d, nst, use_graph=True)
                assert s1.converged
            for i, (m, cb, ca) in enumerate(zip(made, batch_cns, alone_cns)):
                Ub, Lb, tb = _state(ctx, phfem, cb, m[1])
                Ua, La, ta = _state(ctx, phfem, ca, m[1])
                assert tb == ta
                assert not np.isnan(Ub).any() and not np.isnan(Lb).any()
                assert Ub.tobytes() == Ua.tobytes() and Lb.tobytes() == La.tobytes(), (nst, i)
            print(f"{nst} steps: iterations per stepper {[s.iterations for s in st]}", flush=True)
        # a stepper in a batch cannot be destroyed before the batch
        with pytest.raises(phfem.PhfError) as ei:
            phfem.phf_cn_destroy(batch_cns[0])
        assert ei.value.code == phfem.PHF_ESTATE
    finally:
        phfem.phf_cn_batch_destroy(b)
    # one instance (paper mesh refined three times, multigrid) against the
    # oracle's Crank-Nicolson over the same 11 steps
    i = 2
    inst, (chain, dm, _, U0, _) = insts[i], made[i]
    Ub, Lb, tb = _state(ctx, phfem, batch_cns[i], dm)
    xy, el, dd, nn = dm.geometry()
    m = G.Mesh(xy, el, dd, nn)
    tables = oracle.mesh_tables(m)
    a, sc, de = inst["A"], inst["scale"], inst["delta"]
    od = dict(f=oracle.fn(oracle.FN_SIN_SIN, sc * (2 * PI * PI * a - 1 + de), -1),
              g=oracle.fn(oracle.FN_GRAD_SIN_SIN, sc * a, -1),
              uD=oracle.fn(oracle.FN_SIN_SIN, sc, -1))
    Uo, Lo, to = oracle.cn_run(m, tables, inst["k"], 11, U0, np.zeros(tables["L"]),
                               A=(a, 0, 0, a), delta=de, **od)
    assert tb == pytest.approx(to)
    assert _rel(Ub, Uo) < 1e-9, _rel(Ub, Uo)
    assert _rel(Lb, Lo) < 1e-8, _rel(Lb, Lo)
    for cn in batch_cns + alone_cns:
        phfem.phf_cn_destroy(cn)
    for m in made:
        for c in reversed(m[0]):
            c.close()
