"""Pins of the oracle's Crank-Nicolson workload data (Section 4): the source,
flux and Dirichlet kinds with the exp(c1 t) factor that drive the parabolic
configuration (u = exp(-t) sin(pi x) sin(pi y) on the unit square, Dirichlet
on x = 0, 1, Neumann on y = 0, 1), and the edge-midpoint start value.

What fixes them here, independently of the oracle's own code:
  * the exact solution: the L2 error at t = 0.2 falls as h^2 (and the broken
    H1 error as h) over four levels of the paper's mesh, which a wrong sign,
    factor or time dependence in f, g or u_D would stop;
  * the time discretisation: successive differences of the final state
    shrink by 4 per halving of k (second order of the scheme of Section 4);
  * the Neumann flux kind against a central finite difference of the numpy
    u at each Neumann edge midpoint, with the outward normal of that edge;
  * the start value: the P1 function through u0 at the three edge midpoints
    of each element satisfies the discrete constraint -C U = b_D exactly when
    u_D = u0 (both sides of every interior edge agree at its midpoint, and a
    Dirichlet edge's two vertex values average to u0 there).
"""
import numpy as np
import pytest
import scipy.sparse as sp

from paper_2401_15557_amd import meshgen as G

PI = np.pi


def _u(x, y, t):
    return np.exp(-t) * np.sin(PI * x) * np.sin(PI * y)


def _grad_u(x, y, t):
    e = np.exp(-t)
    return e * PI * np.cos(PI * x) * np.sin(PI * y), e * PI * np.sin(PI * x) * np.cos(PI * y)


def _data(oracle):
    # u_t - div grad u = f with f = (2 pi^2 - 1) u, g = grad u . nu, u_D = u
    return dict(f=oracle.fn(oracle.FN_SIN_SIN, 2 * PI * PI - 1, -1),
                g=oracle.fn(oracle.FN_GRAD_SIN_SIN, 1, -1),
                uD=oracle.fn(oracle.FN_SIN_SIN, 1, -1))


def _run(oracle, m, t, k, nst):
    U0 = oracle.cr_interpolant(m, _u, 0.0)
    U, _, tf = oracle.cn_run(m, t, k, nst, U0, np.zeros(t["L"]), **_data(oracle))
    return U, tf


def test_cn_sinsin_space_orders(oracle):
    """k = 1e-3 (k^2 far below the spatial error), t = 0.2, paper mesh
    levels 2-5: L2 order 2 +- 0.1 and broken H1 order 1 +- 0.05 against the
    exact solution at the final time."""
    res = []
    for lev in range(2, 6):
        m = G.paper_square(lev, bc="x_sides")
        t = oracle.mesh_tables(m)
        U, tf = _run(oracle, m, t, 1e-3, 200)
        assert tf == pytest.approx(0.2)
        h1, l2 = oracle.error_norms(m, U, _u, _grad_u, t=tf)
        res.append((h1, l2))
    e = np.array(res)
    o = np.log2(e[:-1] / e[1:])
    assert np.all(np.abs(o[:, 1] - 2.0) < 0.1), o
    assert np.all(np.abs(o[:, 0] - 1.0) < 0.05), o
    # the finest error is of the size of the interpolation error, not of a
    # wrong problem (1/h^2 = 1024 times smaller than u's scale)
    assert e[-1, 1] < 1e-3


def test_cn_sinsin_dt_halving(oracle):
    """Fixed mesh (level 3), k = 0.2/200 ... 0.2/1600: the differences of
    successive final states fall by 4 per halving of k."""
    m = G.paper_square(3, bc="x_sides")
    t = oracle.mesh_tables(m)
    Us = [_run(oracle, m, t, 0.2 / n, n)[0] for n in (200, 400, 800, 1600)]
    d = [np.linalg.norm(Us[q] - Us[q + 1]) for q in range(3)]
    ratios = [d[q] / d[q + 1] for q in range(2)]
    assert ratios[0] == pytest.approx(4.0, rel=0.02), ratios
    assert ratios[1] == pytest.approx(4.0, rel=0.01), ratios


@pytest.mark.parametrize("tt", [0.0, 0.3])
def test_grad_sinsin_flux(oracle, tt):
    """The Neumann load of FN_GRAD_SIN_SIN is |E| g(m_E) / 2 on the two
    vertices of each Neumann edge, g = grad u . nu (outward), u carrying
    exp(-t): checked against central differences of the numpy u."""
    m = G.paper_square(2, bc="x_sides")
    t = oracle.mesh_tables(m)
    asm = oracle.assemble(m, t, g=oracle.fn(oracle.FN_GRAD_SIN_SIN, 1, -1), t=tt)
    F = np.zeros(3 * m.nE)
    hh = 1e-6
    for e in t["neu_edges"]:
        T = t["edge_elems"][e, 0]
        i = t["led"][e]  # local edge = opposite local vertex i
        a, b = (i + 1) % 3, (i + 2) % 3  # counter-clockwise a -> b
        Pa, Pb = m.coords[m.elements[T, a]], m.coords[m.elements[T, b]]
        d = Pb - Pa
        ln = np.hypot(*d)
        nu = np.array([d[1], -d[0]]) / ln
        x, y = 0.5 * (Pa + Pb)
        gx = (_u(x + hh, y, tt) - _u(x - hh, y, tt)) / (2 * hh)
        gy = (_u(x, y + hh, tt) - _u(x, y - hh, tt)) / (2 * hh)
        w = ln * (gx * nu[0] + gy * nu[1]) / 2
        F[3 * T + a] += w
        F[3 * T + b] += w
    assert np.abs(F).max() > 0.1
    np.testing.assert_allclose(asm["F"], F, rtol=0, atol=1e-8)


@pytest.mark.parametrize("tt", [0.0, 0.3])
def test_cr_start_satisfies_constraint(oracle, tt):
    """-C U0 = b_D(t) to 1e-13 when U0 is the edge-midpoint interpolant of
    u_D(., t); on a mesh whose Dirichlet data are not zero (Dirichlet on
    y = 0 and y = 1 of the square shifted by 1/4 in y, so that sin(pi y) is
    not zero there)."""
    m0 = G.paper_square(3, bc="y_sides")
    xy = m0.coords + np.array([0.0, 0.25])
    m = G.Mesh(xy, m0.elements, m0.dirichlet, m0.neumann, name="shifted")
    t = oracle.mesh_tables(m)
    asm = oracle.assemble(m, t, uD=oracle.fn(oracle.FN_SIN_SIN, 1, -1), t=tt)
    C = sp.csr_matrix((asm["C"], asm["C_col"], asm["C_rowptr"]), shape=(asm["L"], asm["N"]))
    U0 = oracle.cr_interpolant(m, _u, tt)
    r = -(C @ U0) - asm["bD"]
    assert np.abs(asm["bD"]).max() > 0.05
    assert np.abs(r).max() <= 1e-13 * np.abs(asm["bD"]).max()
    # and with a start value off by a P1 bump the constraint fails
    U1 = U0.copy()
    U1[0] += 1e-3
    assert np.abs(-(C @ U1) - asm["bD"]).max() > 1e-6
