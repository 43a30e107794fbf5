"""Request server: concurrent elliptic and Crank-Nicolson requests give the
same results as when each runs alone, admission respects the memory budget,
and results agree with the oracle."""
import numpy as np
import pytest

from paper_2401_15557_amd import meshgen as G

pytestmark = pytest.mark.gpu
PI = np.pi


def _elliptic(phfem, base, refine, a=1.0):
    d = phfem.make_data(phfem.make_fn(phfem.PHF_FN_SIN_COS, 2 * PI * PI, 0),
                        phfem.make_fn(phfem.PHF_FN_GRAD_SIN_COS, 1, 0),
                        phfem.make_fn(phfem.PHF_FN_SIN_COS, 1, 0))
    nE = base.nE * 4 ** refine
    U = np.zeros(3 * nE)
    r = phfem.make_request(phfem.PHF_REQ_ELLIPTIC, base, refine=refine,
                           coeffs=phfem.make_coeffs(A=(a, 0, 0, a)), data=d,
                           exact=phfem.make_fn(phfem.PHF_FN_SIN_COS, 1, 0), rtol=1e-12, U_out=U)
    return r, U


def _cn(phfem, level_refine, steps):
    base = G.paper_square(0, bc="x_sides")
    d = phfem.make_data(phfem.make_fn(phfem.PHF_FN_SIN_SIN, 2 * PI * PI - 1, -1),
                        phfem.make_fn(phfem.PHF_FN_GRAD_SIN_SIN, 1, -1),
                        phfem.make_fn(phfem.PHF_FN_SIN_SIN, 1, -1))
    nE = base.nE * 4 ** level_refine
    U = np.zeros(3 * nE)
    r = phfem.make_request(phfem.PHF_REQ_CN, base, refine=level_refine, data=d,
                           u0=phfem.make_fn(phfem.PHF_FN_SIN_SIN, 1, -1),
                           exact=phfem.make_fn(phfem.PHF_FN_SIN_SIN, 1, -1), rtol=1e-11, k=1e-3,
                           steps=steps, U_out=U)
    return r, U


def _mix(phfem):
    out = []
    for q in range(4):
        out.append(_elliptic(phfem, G.unit_square_structured(4 + q), 2 + (q % 3), a=0.5 + 0.3 * q))
    for q in range(3):
        out.append(_cn(phfem, 3 + q, 10 + 7 * q))
    out.append(_elliptic(phfem, G.lshape(0), 4))
    return out


def test_same_alone_and_in_mix():
    from paper_2401_15557_amd import phfem
    alone = []
    s1 = phfem.phf_server_create(0, slots=1)
    try:
        for r, U in _mix(phfem):
            res = phfem.phf_server_wait(s1, phfem.phf_server_submit(s1, r))
            assert res.status == 0, res.status
            alone.append((U.copy(), res.h1, res.l2, res.iterations))
    finally:
        phfem.phf_server_destroy(s1)
    s4 = phfem.phf_server_create(0, slots=4)
    try:
        reqs = _mix(phfem)
        ids = [phfem.phf_server_submit(s4, r) for r, _ in reqs]
        results = [phfem.phf_server_wait(s4, i) for i in ids]
        st = phfem.phf_server_query(s4)
        print(f"peak concurrent {st.peak_running}, completed {st.completed}", flush=True)
        assert st.completed == len(reqs) and st.peak_running >= 2
        for (r, U), res, (Ua, h1, l2, its) in zip(reqs, results, alone):
            assert res.status == 0
            assert U.tobytes() == Ua.tobytes()
            assert (res.h1, res.l2, res.iterations) == (h1, l2, its)
            assert res.latency_ms >= res.run_ms > 0
        assert len({res.slot for res in results}) >= 2
    finally:
        phfem.phf_server_destroy(s4)


def test_results_against_oracle_and_accuracy(oracle):
    from paper_2401_15557_amd import phfem
    s = phfem.phf_server_create(0, slots=2)
    try:
        base = G.unit_square_structured(4)
        r, U = _elliptic(phfem, base, 2)
        rc, Uc = _cn(phfem, 5, 40)
        i1, i2 = phfem.phf_server_submit(s, r), phfem.phf_server_submit(s, rc)
        res1, res2 = phfem.phf_server_wait(s, i1), phfem.phf_server_wait(s, i2)
        assert res1.status == 0 and res2.status == 0
        # elliptic: the oracle's LU solution on the same refined mesh
        m = base
        for _ in range(2):
            m = oracle.red_refine(m)
        asm = oracle.assemble(m, oracle.mesh_tables(m), f=oracle.fn(oracle.FN_SIN_COS, 2 * PI * PI, 0),
                              g=oracle.fn(oracle.FN_GRAD_SIN_COS, 1, 0),
                              uD=oracle.fn(oracle.FN_SIN_COS, 1, 0))
        Uo, _ = oracle.solve_saddle(asm)
        assert np.linalg.norm(U - Uo) / np.linalg.norm(Uo) < 1e-9
        # Crank-Nicolson: 40 steps of k = 1e-3 on 4096 triangles; the error is
        # the spatial one (O(h^2) in L2)
        assert res2.nE == 4096 and 0 < res2.l2 < 3e-3, res2.l2
        assert res2.iterations > 0
    finally:
        phfem.phf_server_destroy(s)


def test_admission_budget_and_errors():
    from paper_2401_15557_amd import phfem
    # a budget below one request's footprint: every request runs alone
    s = phfem.phf_server_create(0, slots=4, memory_bytes=1024)
    try:
        reqs = [_elliptic(phfem, G.unit_square_structured(4), 2) for _ in range(4)]
        ids = [phfem.phf_server_submit(s, r) for r, _ in reqs]
        for i in ids:
            assert phfem.phf_server_wait(s, i).status == 0
        st = phfem.phf_server_query(s)
        assert st.peak_running == 1 and st.completed == 4
        # a result is collected once
        with pytest.raises(phfem.PhfError):
            phfem.phf_server_wait(s, ids[0])
        # per-triangle coefficient arrays are not accepted (the pointer is
        # rejected before any use)
        r, _ = _elliptic(phfem, G.unit_square_structured(4), 1)
        keep = np.ones(10)
        r.coeffs.a_T = keep.ctypes.data
        with pytest.raises(phfem.PhfError) as ei:
            phfem.phf_server_submit(s, r)
        assert ei.value.code == phfem.PHF_EINVAL
    finally:
        phfem.phf_server_destroy(s)
