"""Pins of the oracle's red refinement (Section 2.3, Listing 4)."""
import numpy as np
import pytest

from paper_2401_15557_amd import meshgen as G


def _area(P):
    return 0.5 * ((P[..., 1, 0] - P[..., 0, 0]) * (P[..., 2, 1] - P[..., 0, 1]) -
                  (P[..., 2, 0] - P[..., 0, 0]) * (P[..., 1, 1] - P[..., 0, 1]))


@pytest.mark.parametrize("base", ["paper", "lshape", "jitter"])
def test_refine_structure(oracle, base):
    m = {"paper": lambda: G.paper_square(0), "lshape": lambda: G.lshape(0),
         "jitter": lambda: G.jittered_square(5, np.random.default_rng(2))}[base]()
    for lev in range(1, 4):
        t = oracle.mesh_tables(m)
        f = oracle.red_refine(m, t)
        nE, nC = m.nE, m.nC
        assert f.nE == 4 * nE and f.nC == nC + t["n_edges"]
        if base == "paper":
            assert f.nE == 4 ** (lev + 1)  # level n has 4^(n+1) triangles (Section 2.4)
        Pp = m.coords[m.elements]
        Pf = f.coords[f.elements]
        # every child counter-clockwise with a quarter of its parent's area
        par = np.concatenate([np.arange(nE), np.repeat(np.arange(nE), 3)])
        np.testing.assert_allclose(_area(Pf), _area(Pp)[par] / 4, rtol=1e-13)
        # vertices: corners keep the parent vertex, midpoints sit on parent edges
        for m_ in range(0, nE, max(1, nE // 7)):
            v = m.elements[m_]
            mids = [f.coords[nC + t["elem_edges"][m_, i]] for i in range(3)]
            for i in range(3):
                a, b = m.coords[v[(i + 1) % 3]], m.coords[v[(i + 2) % 3]]
                np.testing.assert_allclose(mids[i], (a + b) / 2, rtol=0, atol=1e-15)
            np.testing.assert_array_equal(f.elements[m_], nC + t["elem_edges"][m_])
            for i in range(3):
                assert f.elements[nE + 3 * m_ + i, 0] == v[i]
        # refined boundary lists cover the refined boundary (the oracle's
        # boundary classification of the fine mesh accepts them)
        tf = oracle.mesh_tables(f)
        assert tf["n_edges"] - (3 * f.nE - len(f.dirichlet) - len(f.neumann)) // 2 \
            == len(f.dirichlet) + len(f.neumann)
        assert f.nC - tf["n_edges"] + f.nE == m.nC - t["n_edges"] + m.nE
        m = f


def test_refine_matches_vectorised_generator(oracle):
    """The plain-loop oracle and the vectorised input generator implement
    Listing 4 independently and agree bit for bit."""
    m = G.lshape(1)
    for _ in range(3):
        a = oracle.red_refine(m)
        b = G.red_refine(m)
        np.testing.assert_array_equal(a.coords, b.coords)
        np.testing.assert_array_equal(a.elements, b.elements)
        np.testing.assert_array_equal(a.dirichlet, b.dirichlet)
        np.testing.assert_array_equal(a.neumann, b.neumann)
        m = a
