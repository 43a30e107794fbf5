"""Segment lengths of the assembly's scatter (how many source terms are summed
into each output entry), as the benchmark reports them, against a brute-force
count from the mesh's element list and Neumann pairs: K, M, C and b_D have one
producer per entry; an F entry takes the element's body load plus one term
per Neumann edge of that element through the vertex."""
import numpy as np
import pytest

from paper_2401_15557_amd import meshgen as G


def _brute(m):
    cnt = np.ones((m.nE, 3), np.int64)
    where = {}
    for e, tri in enumerate(m.elements):
        for j in range(3):
            a, b = int(tri[j]), int(tri[(j + 1) % 3])
            where.setdefault((min(a, b), max(a, b)), []).append(e)
    for a, b in m.neumann:
        (e,) = where[(min(a, b), max(a, b))]  # a boundary edge has one element
        tri = list(m.elements[e])
        cnt[e, tri.index(a)] += 1
        cnt[e, tri.index(b)] += 1
    h = np.bincount(cnt.reshape(-1))
    return {str(k): int(v) for k, v in enumerate(h) if v}


def _corner_fan():
    """A corner triangle with two Neumann edges: its corner vertex DOF sums
    three terms."""
    xy = np.array([[0.0, 0.0], [1.0, 0.0], [0.0, 1.0], [1.0, 1.0]])
    el = np.array([[0, 1, 2], [1, 3, 2]], np.int32)
    return G.Mesh(xy, el, [[1, 3], [3, 2]], [[0, 1], [2, 0]], name="corner")


@pytest.mark.parametrize("mesh", [G.unit_square_structured(8), G.lshape(3),
                                  G.paper_square(3, bc="paper"), _corner_fan(),
                                  G.jittered_square(9, np.random.default_rng(3))],
                         ids=["c1", "lshape3", "paper3", "corner", "jitter9"])
def test_scatter_histogram(oracle, mesh):
    import bench
    t = oracle.mesh_tables(mesh)
    h = bench.scatter_histogram({"edge_type": t["edge_type"][:t["n_edges"]],
                                 "elem_edges": np.asarray(t["elem_edges"]).reshape(-1)}, mesh.nE)
    assert h["F"] == _brute(mesh)
    assert h["K"] == h["M"] == {"1": 9 * mesh.nE}
    asm = oracle.assemble(mesh, t)
    assert h["C"] == {"1": len(asm["C"])}
    assert h["bD"]["1"] == len(mesh.dirichlet) and sum(h["bD"].values()) == t["L"]
    assert max(int(k) for k in h["F"]) <= 3
    if mesh.name == "corner":
        assert h["F"] == {"1": 3, "2": 2, "3": 1}
