"""Helpers of the GPU parity tests: run the HIP path through the C ABI and
the oracle on the same seeded inputs and compare with the stated tolerance.

Tolerance for floating-point values: |gpu - oracle| <= RTOL * s per entry,
with s the largest magnitude of the entry's element block (K, M, D: the 9
values of one element), of its row (C) or of the whole vector (F, b_D).
Both sides evaluate the same closed forms in fp64; they differ only by
rounding order and fused multiply-adds (a few units in the last place of
the block scale), so 1e-12 leaves three orders of margin while a wrong
term, sign or index is off by O(1) of the scale.
"""
import numpy as np

RTOL = 1e-12
# Every device output of a parity test starts as NaN: an entry the library
# does not write stays NaN and fails the comparison (torch's caching
# allocator would otherwise hand back the previous case's values).
NAN = float("nan")


def nan_vec(n, dev):
    import torch
    return torch.full((max(int(n), 1),), NAN, dtype=torch.float64, device=dev)


def assert_written(t, info):
    """Every entry of the outputs of one assembly (dict of NaN-filled device
    tensors, as from alloc_system(fill=NAN)) was written: none is NaN."""
    size = dict(K=info.nnz_K, M=info.nnz_K, D=info.nnz_K, C=info.nnz_C, F=info.N, bD=info.L,
                S=info.nnz_saddle)
    for k, v in t.items():
        n = size.get(k, v.numel())
        bad = int(v[:n].isnan().sum().item())
        assert bad == 0, f"{k}: {bad} of {n} entries not written"


def block_scale(v, width):
    return np.repeat(np.abs(v.reshape(-1, width)).max(axis=1), width)


def row_scale(v, rowptr):
    s = np.zeros(len(v))
    for r in range(len(rowptr) - 1):
        a, b = rowptr[r], rowptr[r + 1]
        if b > a:
            s[a:b] = np.abs(v[a:b]).max()
    return s


def row_scale_fast(v, rowptr):
    n = len(rowptr) - 1
    lens = np.diff(rowptr)
    rows = np.repeat(np.arange(n), lens)
    mx = np.zeros(n)
    np.maximum.at(mx, rows, np.abs(v))
    return mx[rows]


def assert_close_scaled(g, o, scale, what, rtol=RTOL):
    g = np.asarray(g, np.float64)
    o = np.asarray(o, np.float64)
    assert g.shape == o.shape, (what, g.shape, o.shape)
    err = np.abs(g - o)
    bad = err > rtol * np.maximum(scale, np.finfo(float).tiny)
    if bad.any():
        i = int(np.flatnonzero(bad)[0])
        raise AssertionError(f"{what}: {int(bad.sum())} entries differ; first at {i}: "
                             f"gpu={g[i]!r} oracle={o[i]!r} scale={scale[i]!r}")


def gpu_tables(ctx, mesh):
    """Builds the device mesh and returns (Mesh, topology dict, patterns)."""
    from paper_2401_15557_amd import phfem
    dm = phfem.Mesh(ctx, mesh)
    return dm, dm.topology(), dm.patterns()


def compare_topology(topo_g, topo_o):
    for k in ("edge_nodes", "edge_elems", "elem_edges", "led", "ledTN", "edge_type",
              "edge_row", "dir_edges", "neu_edges"):
        np.testing.assert_array_equal(np.asarray(topo_g[k]), np.asarray(topo_o[k]), err_msg=k)
