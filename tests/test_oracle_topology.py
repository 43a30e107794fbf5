"""Pins of the oracle's edge tables (Section 2.2) against the paper's worked
example, brute force and mesh invariants."""
import numpy as np
import pytest

from conftest import read_golden
from paper_2401_15557_amd import meshgen as G


def test_paper_worked_example(oracle):
    gold = read_golden("paper_sec2_example.txt")
    m = G.paper_square(0)
    t = oracle.topology(m.elements, m.nC)
    assert t["n_edges"] == 8
    # nodes2edge: symmetric, entry (k,l) = edge number (1-based)
    n2ed = np.zeros((5, 5), int)
    for e, (k, l) in enumerate(t["edge_nodes"]):
        n2ed[k, l] = n2ed[l, k] = e + 1
    np.testing.assert_array_equal(n2ed, np.array(gold["nodes2edge"], int))
    # edge2element: [k l T+ T-] 1-based, 0 for a missing T-
    ed2el = np.concatenate([t["edge_nodes"] + 1, t["edge_elems"] + 1], axis=1)
    np.testing.assert_array_equal(ed2el, np.array(gold["edge2element"], int))
    # nodes2element: directed edge (k,l) -> element; recovered from the tables
    n2el = np.zeros((5, 5), int)
    for e, (k, l) in enumerate(t["edge_nodes"]):
        tp, tm = t["edge_elems"][e]
        n2el[k, l] = tp + 1
        if tm >= 0:
            n2el[l, k] = tm + 1
    np.testing.assert_array_equal(n2el, np.array(gold["nodes2element"], int))
    # local edge numbers: led / ledTN are the vertex of T+ / T- opposite e
    for e, (k, l) in enumerate(t["edge_nodes"]):
        for T, le in ((t["edge_elems"][e, 0], t["led"][e]), (t["edge_elems"][e, 1], t["ledTN"][e])):
            if T < 0:
                continue
            assert m.elements[T, le] not in (k, l)


def brute_force_edges(elements):
    """Dictionary-based edge table (independent of the oracle's sort)."""
    seen = {}
    for m, tri in enumerate(elements.tolist()):
        for j in range(3):
            a, b = tri[j], tri[(j + 1) % 3]
            seen.setdefault((max(a, b), min(a, b)), []).append((m, j, a, b))
    keys = sorted(seen)
    return keys, seen


def _random_mesh(seed, n=7):
    rng = np.random.default_rng(seed)
    m = G.jittered_square(n, rng, 0.2)
    # relabel nodes and shuffle element order (orientation preserved)
    perm = rng.permutation(m.nC)
    inv = np.empty_like(perm)
    inv[perm] = np.arange(m.nC)
    coords = m.coords[perm]
    el = inv[m.elements]
    order = rng.permutation(m.nE)
    el = el[order]
    rot = rng.integers(0, 3, size=m.nE)
    el = np.stack([np.roll(r, -k) for r, k in zip(el, rot)])
    return G.Mesh(coords, el, inv[m.dirichlet], inv[m.neumann])


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_brute_force_random(oracle, seed):
    m = _random_mesh(seed)
    t = oracle.topology(m.elements, m.nC)
    keys, seen = brute_force_edges(m.elements)
    assert t["n_edges"] == len(keys)
    for e, key in enumerate(keys):
        occ = sorted(seen[key])
        k, l = t["edge_nodes"][e]
        assert (max(k, l), min(k, l)) == key
        assert t["edge_elems"][e, 0] == occ[0][0]
        assert (k, l) == (occ[0][2], occ[0][3])
        if len(occ) == 2:
            assert t["edge_elems"][e, 1] == occ[1][0]
            assert t["ledTN"][e] == (occ[1][1] + 2) % 3
        else:
            assert t["edge_elems"][e, 1] == -1
            assert t["ledTN"][e] == t["led"][e]
        assert t["led"][e] == (occ[0][1] + 2) % 3
        for (mm, j, a, b) in occ:
            assert t["elem_edges"][mm, (j + 2) % 3] == e


@pytest.mark.parametrize("level", [0, 1, 2, 3])
def test_invariants(oracle, level):
    for m in (G.paper_square(level), G.lshape(level)):
        t = oracle.topology(m.elements, m.nC)
        nb = int(np.sum(t["edge_elems"][:, 1] < 0))
        assert 2 * t["n_edges"] == 3 * m.nE + nb
        # Euler characteristic of a simply connected planar triangulation
        assert m.nC - t["n_edges"] + m.nE == 1
        assert np.all(t["edge_elems"][:, 1][t["edge_elems"][:, 1] >= 0] >
                      t["edge_elems"][:, 0][t["edge_elems"][:, 1] >= 0])
        # boundary edges are exactly the listed D and N pairs
        assert nb == len(m.dirichlet) + len(m.neumann)


def test_boundary_rows(oracle):
    m = G.paper_square(0)
    t = oracle.mesh_tables(m)
    # Dirichlet [1 2],[2 4] -> edges 1, 3; Neumann [4 3],[3 1] -> 4, 2 (1-based)
    np.testing.assert_array_equal(t["dir_edges"] + 1, [1, 3])
    np.testing.assert_array_equal(t["neu_edges"] + 1, [4, 2])
    # Redges = setdiff(1:8, Nbed) = [1 3 5 6 7 8]
    rows = np.flatnonzero(t["edge_row"] >= 0) + 1
    np.testing.assert_array_equal(rows, [1, 3, 5, 6, 7, 8])
    assert t["L"] == 6


def test_errors(oracle):
    m = G.paper_square(0)
    el = m.elements.copy()
    with pytest.raises(oracle.OracleError):  # index out of range
        bad = el.copy(); bad[0, 0] = 99
        oracle.topology(bad, m.nC)
    with pytest.raises(oracle.OracleError):  # repeated vertex
        bad = el.copy(); bad[0, 1] = bad[0, 0]
        oracle.topology(bad, m.nC)
    with pytest.raises(oracle.OracleError):  # edge in three elements
        bad = np.concatenate([el, [[4, 0, 1]]])
        oracle.topology(bad, m.nC)
    with pytest.raises(oracle.OracleError):  # same direction in both neighbours
        bad = el.copy(); bad[1] = bad[1][::-1]
        oracle.topology(bad, m.nC)
    t = oracle.topology(el, m.nC)
    with pytest.raises(oracle.OracleError):  # boundary edge in no list
        oracle.boundary(t, m.dirichlet[:1], m.neumann)
    with pytest.raises(oracle.OracleError):  # listed twice
        oracle.boundary(t, m.dirichlet, np.concatenate([m.neumann, m.dirichlet[:1]]))
    with pytest.raises(oracle.OracleError):  # interior edge listed
        oracle.boundary(t, np.concatenate([m.dirichlet, [[4, 0]]]), m.neumann)
