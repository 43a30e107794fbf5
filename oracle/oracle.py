"""Python driver of the CPU oracle (test infrastructure only).

The oracle is the plain statement of what the primal hybrid FEM hot path
computes (arXiv:2401.15557). It is used by the test suite, by the smoke check
and by the benchmark's CPU-baseline leg, and by nothing else: the product
path never imports it.

Contents:
  * ``build()``                  -- compile ``phfem_oracle.c`` with gcc;
  * ``topology / boundary``      -- Section 2.2 edge tables, boundary lookup;
  * ``assemble / saddle``        -- Sections 3.3-3.5 global matrices and loads;
  * ``solve_saddle``             -- the exact solution of the saddle system
                                    (sparse LU, SciPy SuperLU);
  * ``cn_matrices / cn_run``     -- the Crank-Nicolson system of Section 4;
  * ``error_norms``              -- broken H^1 seminorm and L^2 error by a
                                    collapsed Gauss-Legendre rule.
Parity status of each function is stated in its docstring.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "phfem_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

FN_ZERO, FN_CONST, FN_SIN_COS, FN_SIN_SIN = 0, 1, 2, 3
FN_GRAD_SIN_COS, FN_GRAD_SIN_SIN = 4, 5
FN_PAPER_U, FN_PAPER_F, FN_PAPER_FLUX = 6, 7, 8
FN_EDGE_ARRAY = 100

ERRORS = {-1: "EINVAL", -2: "EORIENT", -3: "EMESH", -4: "EBOUNDARY", -5: "ENOMEM"}


class OracleError(RuntimeError):
    def __init__(self, code, where):
        super().__init__(f"oracle {where}: {ERRORS.get(code, code)}")
        self.code = code


def build(force=True):
    """Compile the oracle shared library with gcc (-O2, single thread)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-o", tmp, _SRC,
                               "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Fn(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("pad", ctypes.c_int32),
                ("c", ctypes.c_double * 4), ("edge_values", ctypes.c_void_p)]


def fn(kind=FN_ZERO, *c, edge_values=None):
    """Problem-data function descriptor (kind, parameters, optional edge array)."""
    s = _Fn()
    s.kind = int(kind)
    for q, v in enumerate(c[:4]):
        s.c[q] = float(v)
    s._keep = None
    if edge_values is not None:
        arr = np.ascontiguousarray(edge_values, dtype=np.float64)
        s._keep = arr
        s.edge_values = arr.ctypes.data
        s.kind = FN_EDGE_ARRAY
    return s


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        _lib = ctypes.CDLL(_LIB)
    return _lib


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def _check(rc, where):
    if rc != 0:
        raise OracleError(rc, where)


def topology(elements, nC):
    """Edge tables of Section 2.2 (first-occurrence reading of Listing 3).

    Parity pinned: the paper's worked example (Section 2.2) and brute force.
    """
    e = np.ascontiguousarray(elements, dtype=np.int32)
    nE = e.shape[0]
    cap = max(3 * nE, 1)
    edge_nodes = np.empty((cap, 2), np.int32)
    edge_elems = np.empty((cap, 2), np.int32)
    elem_edges = np.empty((max(nE, 1), 3), np.int32)
    led = np.empty(cap, np.int8)
    ledTN = np.empty(cap, np.int8)
    ne = ctypes.c_int32(0)
    rc = lib().orc_topology(ctypes.c_int32(nC), ctypes.c_int32(nE), _p(e), ctypes.byref(ne),
                            _p(edge_nodes), _p(edge_elems), _p(elem_edges), _p(led), _p(ledTN))
    _check(rc, "topology")
    n = ne.value
    return dict(n_edges=n, edge_nodes=edge_nodes[:n].copy(), edge_elems=edge_elems[:n].copy(),
                elem_edges=elem_edges[:nE].copy(), led=led[:n].copy(), ledTN=ledTN[:n].copy())


def boundary(topo, dirichlet, neumann):
    """Dirichlet / Neumann edge ids and multiplier rows (Main.m lookups)."""
    n = topo["n_edges"]
    D = np.ascontiguousarray(dirichlet, dtype=np.int32).reshape(-1, 2)
    N = np.ascontiguousarray(neumann, dtype=np.int32).reshape(-1, 2)
    edge_type = np.empty(max(n, 1), np.int8)
    dir_edges = np.empty(max(len(D), 1), np.int32)
    neu_edges = np.empty(max(len(N), 1), np.int32)
    edge_row = np.empty(max(n, 1), np.int32)
    L = ctypes.c_int32(0)
    rc = lib().orc_boundary(ctypes.c_int32(n), _p(topo["edge_nodes"]), _p(topo["edge_elems"]),
                            ctypes.c_int32(len(D)), _p(D), ctypes.c_int32(len(N)), _p(N),
                            _p(edge_type), _p(dir_edges), _p(neu_edges), _p(edge_row),
                            ctypes.byref(L))
    _check(rc, "boundary")
    return dict(edge_type=edge_type[:n].copy(), dir_edges=dir_edges[:len(D)].copy(),
                neu_edges=neu_edges[:len(N)].copy(), edge_row=edge_row[:n].copy(), L=L.value)


def mesh_tables(mesh):
    """Topology + boundary classification of a meshgen.Mesh."""
    topo = topology(mesh.elements, mesh.nC)
    topo.update(boundary(topo, mesh.dirichlet, mesh.neumann))
    return topo


def _coeff_arrays(A, p):
    A = np.ascontiguousarray(np.asarray(A, dtype=np.float64).reshape(4))
    p = np.ascontiguousarray(np.asarray(p, dtype=np.float64).reshape(2))
    return A, p


def element(mesh, m, A=(1, 0, 0, 1), aT=1.0, p=(0, 0), f=None, t=0.0, elem_edges=None):
    """Local K, D, M (row-major 3x3) and b of one element (Definition 3.1)."""
    A, p = _coeff_arrays(A, p)
    f = f if f is not None else fn(FN_ZERO)
    K = np.empty(9); D = np.empty(9); M = np.empty(9); b = np.empty(3)
    ee = None if elem_edges is None else np.ascontiguousarray(elem_edges, dtype=np.int32)
    rc = lib().orc_element(_p(mesh.coords), _p(mesh.elements), ctypes.c_int32(int(m)), _p(A),
                           ctypes.c_double(float(aT)), _p(p), ctypes.byref(f), ctypes.c_double(t),
                           _p(ee), _p(K), _p(D), _p(M), _p(b))
    _check(rc, "element")
    return K.reshape(3, 3), D.reshape(3, 3), M.reshape(3, 3), b


def assemble(mesh, tables, A=(1, 0, 0, 1), p=(0, 0), aT=None, f=None, g=None, uD=None, t=0.0):
    """Global K, D, M (CSR, N x N), C (CSR, L x N), F = b + LN and b_D.

    Parity pinned: closed forms, brute-force quadrature, invariants and the
    paper's Table 4 (through ``solve_saddle``).
    """
    A, p = _coeff_arrays(A, p)
    f = f if f is not None else fn(FN_ZERO)
    g = g if g is not None else fn(FN_ZERO)
    uD = uD if uD is not None else fn(FN_ZERO)
    nE, L = mesh.nE, tables["L"]
    N = 3 * nE
    aTa = None if aT is None else np.ascontiguousarray(aT, dtype=np.float64)
    K_rowptr = np.empty(N + 1, np.int32)
    K_col = np.empty(max(9 * nE, 1), np.int32)
    K_val = np.empty(max(9 * nE, 1)); D_val = np.empty_like(K_val); M_val = np.empty_like(K_val)
    C_rowptr = np.empty(L + 1, np.int32)
    C_col = np.empty(max(4 * L, 1), np.int32)
    C_val = np.empty(max(4 * L, 1))
    nnzC = ctypes.c_int64(0)
    F = np.empty(max(N, 1)); bD = np.zeros(max(L, 1))
    rc = lib().orc_assemble(
        ctypes.c_int32(mesh.nC), _p(mesh.coords), ctypes.c_int32(nE), _p(mesh.elements),
        ctypes.c_int32(tables["n_edges"]), _p(tables["edge_nodes"]), _p(tables["edge_elems"]),
        _p(tables["elem_edges"]), _p(tables["edge_type"]), _p(tables["edge_row"]),
        ctypes.c_int32(L), _p(A), _p(p), _p(aTa), ctypes.byref(f), ctypes.byref(g),
        ctypes.byref(uD), ctypes.c_double(t), _p(K_rowptr), _p(K_col), _p(K_val), _p(D_val),
        _p(M_val), _p(C_rowptr), _p(C_col), _p(C_val), ctypes.byref(nnzC), _p(F), _p(bD))
    _check(rc, "assemble")
    nc = nnzC.value
    return dict(N=N, L=L, K_rowptr=K_rowptr, K_col=K_col[:9 * nE], K=K_val[:9 * nE],
                D=D_val[:9 * nE], M=M_val[:9 * nE], C_rowptr=C_rowptr, C_col=C_col[:nc].copy(),
                C=C_val[:nc].copy(), F=F[:N], bD=bD[:L])


def saddle(asm, delta=0.0):
    """CSR of M_vec = [K + D + delta M, -C^T; -C, 0] (Section 3.5)."""
    N, L = asm["N"], asm["L"]
    nE = N // 3
    cap = max(9 * nE + 2 * len(asm["C"]), 1)
    rowptr = np.empty(N + L + 1, np.int32)
    col = np.empty(cap, np.int32)
    val = np.empty(cap)
    nnz = ctypes.c_int64(0)
    rc = lib().orc_saddle(ctypes.c_int32(nE), ctypes.c_int32(L), _p(asm["K_rowptr"]),
                          _p(asm["K_col"]), _p(asm["K"]), _p(asm["D"]), _p(asm["M"]),
                          ctypes.c_double(delta), _p(asm["C_rowptr"]), _p(asm["C_col"]),
                          _p(asm["C"]), _p(rowptr), _p(col), _p(val), ctypes.byref(nnz))
    _check(rc, "saddle")
    n = nnz.value
    return rowptr, col[:n].copy(), val[:n].copy()


def csr_matvec(rowptr, col, val, x):
    """y = A x with the plain row loop."""
    y = np.empty(len(rowptr) - 1)
    xx = np.ascontiguousarray(x, dtype=np.float64)
    lib().orc_csr_matvec(ctypes.c_int32(len(rowptr) - 1), _p(rowptr), _p(col), _p(val), _p(xx),
                         _p(y))
    return y


def _scipy_csr(rowptr, col, val, n):
    import scipy.sparse as sp
    return sp.csr_matrix((val, col, rowptr), shape=(n, n))


def solve_saddle(asm, delta=0.0):
    """Exact solution (U, Lambda) of M_vec W = (F; b_D) by sparse LU.

    Library routine: SciPy SuperLU. Parity pinned by the paper's Table 4 and
    the linear patch test.
    """
    import scipy.sparse.linalg as spla
    N, L = asm["N"], asm["L"]
    rowptr, col, val = saddle(asm, delta)
    A = _scipy_csr(rowptr, col, val, N + L).tocsc()
    rhs = np.concatenate([asm["F"], asm["bD"]])
    w = spla.splu(A, permc_spec="COLAMD").solve(rhs)
    return w[:N].copy(), w[N:].copy()


def cn_matrices(asm, k, delta=0.0):
    """CSR of M+ and M- of the Crank-Nicolson system (Section 4.1).

    M(+/-) = [(1 +/- k delta/2) M +/- (k/2)(K + D), -/+ (k/2) C^T;
              -/+ (1/2) C, 0], with M the unit mass.
    """
    import scipy.sparse as sp
    N, L = asm["N"], asm["L"]
    Kc = _scipy_csr(asm["K_rowptr"], asm["K_col"], asm["K"], N)
    Dc = _scipy_csr(asm["K_rowptr"], asm["K_col"], asm["D"], N)
    Mc = _scipy_csr(asm["K_rowptr"], asm["K_col"], asm["M"], N)
    C = sp.csr_matrix((asm["C"], asm["C_col"], asm["C_rowptr"]), shape=(L, N))
    out = []
    for s in (+1.0, -1.0):
        A11 = (1.0 + s * k * delta / 2.0) * Mc + s * (k / 2.0) * (Kc + Dc)
        Mx = sp.bmat([[A11, -s * (k / 2.0) * C.T], [-s * 0.5 * C, None]], format="csr")
        out.append(Mx)
    return out[0], out[1]


def cn_run(mesh, tables, k, nsteps, U0, Lam0, t0=0.0, A=(1, 0, 0, 1), p=(0, 0), aT=None,
           delta=0.0, f=None, g=None, uD=None):
    """Crank-Nicolson time stepping M+ W^n = M- W^{n-1} + F (Section 4.1).

    The load is the average of its evaluations at t_{n-1} and t_n (4.1), for
    F (= b + LN) and for b_D. M+ is factorized once. Returns the final
    (U, Lambda) and the list of times.
    """
    import scipy.sparse.linalg as spla
    asm0 = assemble(mesh, tables, A=A, p=p, aT=aT, f=f, g=g, uD=uD, t=t0)
    N, L = asm0["N"], asm0["L"]
    Mp, Mm = cn_matrices(asm0, k, delta)
    lu = spla.splu(Mp.tocsc(), permc_spec="COLAMD")
    w = np.concatenate([np.asarray(U0, np.float64), np.asarray(Lam0, np.float64)])
    F_prev, bD_prev = asm0["F"], asm0["bD"]
    t = t0
    for n in range(1, nsteps + 1):
        tn = t0 + n * k
        asm_n = assemble(mesh, tables, A=A, p=p, aT=aT, f=f, g=g, uD=uD, t=tn)
        rhs = Mm @ w + np.concatenate([k * 0.5 * (F_prev + asm_n["F"]),
                                       0.5 * (bD_prev + asm_n["bD"])])
        w = lu.solve(rhs)
        F_prev, bD_prev = asm_n["F"], asm_n["bD"]
        t = tn
    return w[:N].copy(), w[N:].copy(), t


def cr_interpolant(mesh, u0, t=0.0):
    """Per-element P1 values matching u0 at the three edge midpoints.

    Vertex i gets u0(m_j) + u0(m_k) - u0(m_i), m_i the midpoint of the edge
    opposite vertex i (the P1 function through the three midpoint values).
    ``u0(x, y, t)`` is a numpy-vectorised callable.
    """
    P = mesh.coords[mesh.elements]  # nE x 3 x 2
    mids = np.stack([(P[:, 1] + P[:, 2]) / 2, (P[:, 2] + P[:, 0]) / 2, (P[:, 0] + P[:, 1]) / 2],
                    axis=1)
    um = u0(mids[..., 0], mids[..., 1], t)
    U = np.empty_like(um)
    for i in range(3):
        j, k = (i + 1) % 3, (i + 2) % 3
        U[:, i] = um[:, j] + um[:, k] - um[:, i]
    return U.reshape(-1)


def gauss_triangle_rule(n=5):
    """Collapsed (Duffy) Gauss-Legendre rule on the reference triangle.

    Built from the n-point 1-D rule (numpy.polynomial.legendre.leggauss):
    (s, r) in [0,1]^2 -> (x, y) = (s (1 - r), r) with Jacobian (1 - r).
    Exact for polynomials of degree <= 2n - 2 in (x, y). Returns points
    (n^2, 2) and weights summing to 1/2.
    """
    z, w = np.polynomial.legendre.leggauss(n)
    s = 0.5 * (z + 1.0)
    ws = 0.5 * w
    S, R = np.meshgrid(s, s, indexing="ij")
    WS, WR = np.meshgrid(ws, ws, indexing="ij")
    x = S * (1.0 - R)
    y = R
    wt = WS * WR * (1.0 - R)
    return np.stack([x.ravel(), y.ravel()], axis=1), wt.ravel()


def error_norms(mesh, U, u, grad_u, t=0.0, n=5):
    """Broken H^1 seminorm and L^2 norm of u - u_h (u_h = per-element P1 U).

    ``u(x, y, t)`` and ``grad_u(x, y, t) -> (ux, uy)`` are vectorised.
    The P1 gradient comes from the vertex values through the Vandermonde
    system; integrals use ``gauss_triangle_rule(n)`` mapped affinely.
    """
    P = mesh.coords[mesh.elements]  # nE x 3 x 2
    Ue = np.asarray(U, np.float64).reshape(-1, 3)
    q, w = gauss_triangle_rule(n)
    p0, p1, p2 = P[:, 0], P[:, 1], P[:, 2]
    J = np.stack([p1 - p0, p2 - p0], axis=2)  # nE x 2 x 2 (columns = edge vectors)
    det = J[:, 0, 0] * J[:, 1, 1] - J[:, 0, 1] * J[:, 1, 0]
    X = p0[:, None, :] + np.einsum("eij,qj->eqi", J, q)  # nE x nq x 2
    lam = np.stack([1.0 - q[:, 0] - q[:, 1], q[:, 0], q[:, 1]], axis=1)  # nq x 3
    uh = Ue @ lam.T  # nE x nq
    V = np.concatenate([np.ones((Ue.shape[0], 3, 1)), P], axis=2)  # rows [1 x y]
    coef = np.linalg.solve(V, Ue[..., None])[..., 0]  # uh = c0 + c1 x + c2 y
    ux, uy = grad_u(X[..., 0], X[..., 1], t)
    ue = u(X[..., 0], X[..., 1], t)
    wa = np.abs(det)[:, None] * w[None, :]
    l2 = np.sqrt(np.sum(wa * (ue - uh) ** 2))
    h1 = np.sqrt(np.sum(wa * ((ux - coef[:, 1:2]) ** 2 + (uy - coef[:, 2:3]) ** 2)))
    return h1, l2


def red_refine(mesh, tables=None):
    """One uniform red refinement with the paper's numbering (Section 2.3).

    Parity pinned: element counts 4^(level+1), counter-clockwise children of
    exactly a quarter of the parent area, the midpoint and vertex structure of
    every child, boundary lists covering the refined boundary, and the edge
    table of the refined mesh (Euler characteristic).
    """
    from paper_2401_15557_amd import meshgen as G
    t = tables if tables is not None else mesh_tables(mesh)
    nC, nE, ne = mesh.nC, mesh.nE, t["n_edges"]
    nD, nN = len(mesh.dirichlet), len(mesh.neumann)
    xy_f = np.empty((nC + ne, 2))
    el_f = np.empty((4 * nE, 3), np.int32)
    d_f = np.empty((max(2 * nD, 1), 2), np.int32)
    n_f = np.empty((max(2 * nN, 1), 2), np.int32)
    rc = lib().orc_red_refine(
        ctypes.c_int32(nC), _p(mesh.coords), ctypes.c_int32(nE), _p(mesh.elements),
        ctypes.c_int32(ne), _p(t["edge_nodes"]), _p(t["elem_edges"]), ctypes.c_int32(nD),
        _p(mesh.dirichlet), _p(np.ascontiguousarray(t["dir_edges"])), ctypes.c_int32(nN),
        _p(mesh.neumann), _p(np.ascontiguousarray(t["neu_edges"])), _p(xy_f), _p(el_f),
        _p(d_f), _p(n_f))
    _check(rc, "red_refine")
    return G.Mesh(xy_f, el_f, d_f[:2 * nD], n_f[:2 * nN], name=mesh.name + "+r")
