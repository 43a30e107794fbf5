"""The benchmark's algorithmic byte model of the assembly (CPU).

The roofline fraction the benchmark reports divides these bytes by the
kernel time, so the model is pinned here against sizes derived
independently of the library: for the paper's unit-square mesh refined n
times (4^(n+1) triangles, 2^(n+2) boundary edges, Dirichlet on x = 0, 1 and
Neumann on y = 0, 1), the edge count follows from 3 nE = 2 E - E_b, the
node count from Euler's formula V - E + T = 1, the multiplier rows are the
non-Neumann edges, and C holds 4 entries per interior row and 2 per
Dirichlet row. At n = 10 the model is 268 bytes per triangle
(1,124,073,488 B), 260 without a_T.
"""
import importlib.util
import os
from types import SimpleNamespace

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_model_under_test",
                                                  os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def _paper_sizes(n):
    nE = 4 ** (n + 1)
    Eb = 2 ** (n + 2)              # boundary edges, 2^n per side
    E = (3 * nE + Eb) // 2
    V = 1 + E - nE                 # simply connected: V - E + T = 1
    nD = nN = Eb // 2              # x = 0, 1 Dirichlet; y = 0, 1 Neumann
    L = E - nN
    nnzC = 4 * (L - nD) + 2 * nD
    return SimpleNamespace(nE=nE, nC=V, L=L, nnz_C=nnzC, n_free=E - nD, nnz_reduced=0)


def test_headline_assembly_bytes():
    B = _bench()
    info = _paper_sizes(10)
    assert (info.nE, info.nC, info.L, info.nnz_C) == (4194304, 2099201, 6291456, 25161728)
    b = B.algorithmic_bytes(info)["k_assemble"]
    assert b == 1124073488
    assert abs(b / info.nE - 268.0) < 1e-5
    assert B.algorithmic_bytes(info, has_aT=False)["k_assemble"] == b - 8 * info.nE


def test_model_per_triangle_over_levels():
    """Per triangle the model tends to 268 B as the boundary share vanishes:
    16 V/T -> 8, rows 1.5 per triangle (8 B read + 8 B written each),
    C 6 entries per triangle (48 B), K, M, F 168 B, vertices 12, a_T 8."""
    B = _bench()
    prev = None
    for n in range(3, 11):
        info = _paper_sizes(n)
        per = B.algorithmic_bytes(info)["k_assemble"] / info.nE
        assert 267.9 < per < 268.5
        if prev is not None:
            assert abs(per - 268.0) <= abs(prev - 268.0)
        prev = per
