"""Pins of the oracle's local matrices and loads (Definition 3.1, Section 3.4)
against closed forms, brute-force quadrature and invariants."""
import numpy as np
import pytest

from paper_2401_15557_amd import meshgen as G


def _tri(seed):
    rng = np.random.default_rng(seed)
    while True:
        P = rng.uniform(-1, 1, size=(3, 2))
        area = 0.5 * ((P[1, 0] - P[0, 0]) * (P[2, 1] - P[0, 1]) -
                      (P[2, 0] - P[0, 0]) * (P[1, 1] - P[0, 1]))
        if abs(area) > 0.05:
            if area < 0:
                P = P[[0, 2, 1]]
            return P


def _single(P):
    return G.Mesh(P, np.array([[0, 1, 2]]), np.zeros((0, 2)), np.zeros((0, 2)))


def _rot_grad(P):
    """grad lambda_i = (y_{i+1} - y_{i+2}, x_{i+2} - x_{i+1}) / (2|T|)."""
    area = 0.5 * ((P[1, 0] - P[0, 0]) * (P[2, 1] - P[0, 1]) -
                  (P[2, 0] - P[0, 0]) * (P[1, 1] - P[0, 1]))
    g = np.empty((3, 2))
    for i in range(3):
        a, b = P[(i + 1) % 3], P[(i + 2) % 3]
        g[i] = [(a[1] - b[1]) / (2 * area), (b[0] - a[0]) / (2 * area)]
    return g, area


def _quad(P, fun, n=6):
    """Integral over triangle P of fun(lam) with lam the barycentric coords,
    by a tensor Gauss rule on the square collapsed onto the triangle."""
    z, w = np.polynomial.legendre.leggauss(n)
    s, ws = 0.5 * (z + 1), 0.5 * w
    area = 0.5 * abs((P[1, 0] - P[0, 0]) * (P[2, 1] - P[0, 1]) -
                     (P[2, 0] - P[0, 0]) * (P[1, 1] - P[0, 1]))
    tot = 0.0
    for a, wa in zip(s, ws):
        for b, wb in zip(s, ws):
            l1, l2 = a * (1 - b), b
            lam = np.array([1 - l1 - l2, l1, l2])
            tot += wa * wb * (1 - b) * fun(lam, lam @ P)
    return 2 * area * tot


@pytest.mark.parametrize("seed", range(6))
def test_stiffness_cotangent(oracle, seed):
    P = _tri(seed)
    K, D, M, b = oracle.element(_single(P), 0, aT=1.7)
    # K_ij = -(a/2) cot(theta_k) for i != j, theta_k the angle at the third vertex
    for i in range(3):
        for j in range(3):
            if i == j:
                continue
            k = 3 - i - j
            u, v = P[i] - P[k], P[j] - P[k]
            cot = (u @ v) / abs(u[0] * v[1] - u[1] * v[0])
            assert K[i, j] == pytest.approx(-0.85 * cot, rel=1e-12, abs=1e-14)
    np.testing.assert_allclose(K.sum(axis=1), 0, atol=1e-13)
    np.testing.assert_allclose(K, K.T, rtol=1e-14, atol=1e-15)
    assert np.all(np.linalg.eigvalsh(K) > -1e-12)


@pytest.mark.parametrize("seed", range(4))
def test_stiffness_anisotropic(oracle, seed):
    P = _tri(seed + 10)
    A = np.array([[2.0, 0.7], [0.7, 1.3]])
    K, _, _, _ = oracle.element(_single(P), 0, A=A.ravel(), aT=0.6)
    g, area = _rot_grad(P)
    ref = 0.6 * area * (g @ A @ g.T)
    np.testing.assert_allclose(K, ref, rtol=1e-12, atol=1e-14)


@pytest.mark.parametrize("seed", range(4))
def test_mass_and_convection_quadrature(oracle, seed):
    P = _tri(seed + 20)
    p = np.array([0.3, -1.2])
    K, D, M, b = oracle.element(_single(P), 0, p=p)
    g, area = _rot_grad(P)
    for j in range(3):
        for i in range(3):
            mq = _quad(P, lambda lam, x: lam[j] * lam[i])
            assert M[j, i] == pytest.approx(mq, rel=1e-13)
            dq = _quad(P, lambda lam, x: lam[j] * (p @ g[i]))
            assert D[j, i] == pytest.approx(dq, rel=1e-12, abs=1e-14)


@pytest.mark.parametrize("seed", range(4))
def test_load_exact_for_linear_source(oracle, seed):
    """Midpoint rule b_j is exact for int_T f lambda_j when f is linear."""
    P = _tri(seed + 30)
    m = _single(P)
    t = oracle.topology(m.elements, m.nC)
    cf = np.array([0.4, -1.1, 2.3])
    mids = 0.5 * (P[t["edge_nodes"][:, 0]] + P[t["edge_nodes"][:, 1]])
    fvals = cf[0] + cf[1] * mids[:, 0] + cf[2] * mids[:, 1]
    f = oracle.fn(edge_values=fvals)
    _, _, _, b = oracle.element(m, 0, f=f, elem_edges=t["elem_edges"])
    for j in range(3):
        ref = _quad(P, lambda lam, x: (cf[0] + cf[1] * x[0] + cf[2] * x[1]) * lam[j])
        assert b[j] == pytest.approx(ref, rel=1e-12)


def test_load_total_quadratic(oracle):
    """Sum_j F_j = int_Omega f exactly for quadratic f (midpoint rule)."""
    m = G.paper_square(3, bc="all_dirichlet")
    t = oracle.mesh_tables(m)
    mids = 0.5 * (m.coords[t["edge_nodes"][:, 0]] + m.coords[t["edge_nodes"][:, 1]])
    x, y = mids[:, 0], mids[:, 1]
    f = oracle.fn(edge_values=1 + x * x - 3 * x * y + 2 * y * y)
    asm = oracle.assemble(m, t, f=f)
    exact = 1 + 1 / 3 - 3 / 4 + 2 / 3
    assert asm["F"].sum() == pytest.approx(exact, rel=1e-13)
    # total of the unit mass = |Omega|
    assert asm["M"].sum() == pytest.approx(1.0, rel=1e-13)
    np.testing.assert_allclose(np.add.reduceat(asm["K"], np.arange(0, len(asm["K"]), 3)), 0,
                               atol=1e-12)


def test_coupling_matrix(oracle):
    """C entries = sigma int_E lambda_j (1-D Gauss), row sums +-|E|."""
    m = G.lshape(1)
    t = oracle.mesh_tables(m)
    asm = oracle.assemble(m, t)
    L, N = asm["L"], asm["N"]
    C = np.zeros((L, N))
    for r in range(L):
        for q in range(asm["C_rowptr"][r], asm["C_rowptr"][r + 1]):
            C[r, asm["C_col"][q]] = asm["C"][q]
    z, w = np.polynomial.legendre.leggauss(3)
    for e in range(t["n_edges"]):
        r = t["edge_row"][e]
        if r < 0:
            continue
        k, l = t["edge_nodes"][e]
        a, b = m.coords[k], m.coords[l]
        length = np.linalg.norm(b - a)
        for side, sigma in ((0, 1.0), (1, -1.0)):
            T = t["edge_elems"][e, side]
            if T < 0:
                continue
            P = m.coords[m.elements[T]]
            V = np.c_[np.ones(3), P]
            coef = np.linalg.solve(V, np.eye(3))  # column i: lambda_i coefficients
            for j in range(3):
                vals = []
                for s in 0.5 * (z + 1):
                    X = a + s * (b - a)
                    vals.append(coef[0, j] + coef[1, j] * X[0] + coef[2, j] * X[1])
                integ = 0.5 * length * np.dot(w, vals)
                assert C[r, 3 * T + j] == pytest.approx(sigma * integ, abs=1e-13)
        tp = t["edge_elems"][e, 0]
        assert C[r, 3 * tp:3 * tp + 3].sum() == pytest.approx(length, rel=1e-13)
    # nnz: 4 per interior row, 2 per Dirichlet row
    n_int = int(np.sum(t["edge_type"] == 0))
    n_dir = int(np.sum(t["edge_type"] == 1))
    assert len(asm["C"]) == 4 * n_int + 2 * n_dir


def test_neumann_and_dirichlet_data(oracle):
    m = G.paper_square(2)
    t = oracle.mesh_tables(m)
    gv = np.zeros(t["n_edges"]); ud = np.zeros(t["n_edges"])
    rng = np.random.default_rng(5)
    gv[t["neu_edges"]] = rng.normal(size=len(t["neu_edges"]))
    ud[t["dir_edges"]] = rng.normal(size=len(t["dir_edges"]))
    asm = oracle.assemble(m, t, g=oracle.fn(edge_values=gv), uD=oracle.fn(edge_values=ud))
    lens = np.linalg.norm(m.coords[t["edge_nodes"][:, 0]] - m.coords[t["edge_nodes"][:, 1]], axis=1)
    # f = 0: F is the Neumann load only; its total is sum |E| g(m_E)
    assert asm["F"].sum() == pytest.approx(np.sum(lens * gv), rel=1e-13)
    # each Neumann edge adds |E| g / 2 to the two vertex DOFs of T+
    F = np.zeros_like(asm["F"])
    for e in t["neu_edges"]:
        T = t["edge_elems"][e, 0]
        for j in range(3):
            if m.elements[T, j] in t["edge_nodes"][e]:
                F[3 * T + j] += 0.5 * lens[e] * gv[e]
    np.testing.assert_allclose(asm["F"], F, rtol=1e-13, atol=1e-15)
    bD = np.zeros(t["L"])
    bD[t["edge_row"][t["dir_edges"]]] = -lens[t["dir_edges"]] * ud[t["dir_edges"]]
    np.testing.assert_allclose(asm["bD"], bD, rtol=1e-14)


def test_clockwise_rejected(oracle):
    P = _tri(3)[[0, 2, 1]]
    with pytest.raises(oracle.OracleError):
        oracle.element(_single(P), 0)
