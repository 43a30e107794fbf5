"""Seeded synthetic mesh generators (inputs only).

This module builds triangulations and boundary-edge lists and nothing else:
it holds no finite-element arithmetic, so both the GPU path and the CPU
oracle can take their inputs from it.

Conventions (shared by every generator):
  * indices are 0-based int32; coordinates are float64 with shape (nC, 2);
  * every element lists its vertices counter-clockwise;
  * boundary edges are node pairs listed counter-clockwise along the domain
    boundary (domain on the left), split into a Dirichlet and a Neumann list.

Recipes:
  * ``unit_square_structured(n)``  -- n x n cells, each cut by the
    (i,j)->(i+1,j+1) diagonal, lower triangle first, cells row-major.
  * ``paper_square(level)`` -- the four-triangle criss-cross start mesh of the
    paper's Table 1, red-refined ``level`` times with the node and element
    numbering of the paper's red-refinement routine (Section 2.3): the new
    midpoint of edge e gets number nC + e with edges numbered by ascending
    (larger node, smaller node); the interior child [M1 M2 M3] keeps the
    parent's index and the three corner children follow at nE + 3m + {0,1,2};
    each boundary edge is split into its first halves (rows 0..n-1) followed by
    its second halves (rows n..2n-1).
  * ``lshape(level)`` -- L-shaped domain [-1,1]^2 minus [0,1]x[-1,0] made of
    three unit squares, each cut into four triangles around its centre, then
    red-refined ``level`` times.
  * ``jittered_square(n, rng, jitter)`` -- the structured square with interior
    nodes moved uniformly inside a disk of radius jitter*h.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "Mesh",
    "unit_square_structured",
    "paper_square",
    "lshape",
    "jittered_square",
    "red_refine",
    "per_triangle_coefficient",
    "batch_instances",
]


class Mesh:
    """A triangulation plus its Dirichlet / Neumann boundary node pairs."""

    __slots__ = ("coords", "elements", "dirichlet", "neumann", "name")

    def __init__(self, coords, elements, dirichlet, neumann, name=""):
        self.coords = np.ascontiguousarray(coords, dtype=np.float64).reshape(-1, 2)
        self.elements = np.ascontiguousarray(elements, dtype=np.int32).reshape(-1, 3)
        self.dirichlet = np.ascontiguousarray(dirichlet, dtype=np.int32).reshape(-1, 2)
        self.neumann = np.ascontiguousarray(neumann, dtype=np.int32).reshape(-1, 2)
        self.name = name

    @property
    def nE(self):
        return int(self.elements.shape[0])

    @property
    def nC(self):
        return int(self.coords.shape[0])

    def __repr__(self):
        return (f"Mesh({self.name!r}, nC={self.nC}, nE={self.nE}, "
                f"nD={len(self.dirichlet)}, nN={len(self.neumann)})")


def _square_boundary(n, node, dirichlet_sides):
    """Counter-clockwise boundary pairs of the structured n x n square.

    ``node(i, j)`` maps grid indices to node ids. Sides are named
    'bottom' (y=0), 'right' (x=1), 'top' (y=1), 'left' (x=0).
    """
    sides = {
        "bottom": [(node(i, 0), node(i + 1, 0)) for i in range(n)],
        "right": [(node(n, j), node(n, j + 1)) for j in range(n)],
        "top": [(node(i + 1, n), node(i, n)) for i in range(n - 1, -1, -1)],
        "left": [(node(0, j + 1), node(0, j)) for j in range(n - 1, -1, -1)],
    }
    D, N = [], []
    for name in ("bottom", "right", "top", "left"):
        (D if name in dirichlet_sides else N).extend(sides[name])
    return (np.array(D, dtype=np.int32).reshape(-1, 2),
            np.array(N, dtype=np.int32).reshape(-1, 2))


def unit_square_structured(n, dirichlet_sides=("left", "right"), h_scale=1.0):
    """Structured n x n grid on the unit square, 2 n^2 right triangles.

    Node (i, j) sits at (i/n, j/n) with id (n+1) j + i. Each cell is cut by the
    (i,j)->(i+1,j+1) diagonal into [(i,j),(i+1,j),(i+1,j+1)] and
    [(i,j),(i+1,j+1),(i,j+1)] (lower triangle first), cells row-major.
    """
    n = int(n)
    if n < 1:
        raise ValueError("n must be >= 1")
    ii, jj = np.meshgrid(np.arange(n + 1), np.arange(n + 1), indexing="xy")
    coords = np.stack([ii.ravel() / n, jj.ravel() / n], axis=1) * h_scale

    def node(i, j):
        return (n + 1) * j + i

    ci, cj = np.meshgrid(np.arange(n), np.arange(n), indexing="xy")
    ci, cj = ci.ravel(), cj.ravel()
    a = node(ci, cj)
    b = node(ci + 1, cj)
    c = node(ci + 1, cj + 1)
    d = node(ci, cj + 1)
    lower = np.stack([a, b, c], axis=1)
    upper = np.stack([a, c, d], axis=1)
    elements = np.empty((2 * n * n, 3), dtype=np.int32)
    elements[0::2] = lower
    elements[1::2] = upper
    D, N = _square_boundary(n, node, dirichlet_sides)
    return Mesh(coords, elements, D, N, name=f"square{n}x{n}")


def red_refine(mesh: Mesh) -> Mesh:
    """One uniform red refinement with the paper's numbering (Section 2.3)."""
    coords, elems = mesh.coords, mesh.elements.astype(np.int64)
    nC, nE = coords.shape[0], elems.shape[0]
    # undirected edges numbered by ascending (larger node, smaller node)
    a = elems
    b = elems[:, [1, 2, 0]]
    hi = np.maximum(a, b).ravel()
    lo = np.minimum(a, b).ravel()
    key = hi * np.int64(nC) + lo
    ukey, inv = np.unique(key, return_inverse=True)
    inv = inv.reshape(nE, 3)  # inv[m, j]: edge id of directed local edge j
    e_hi = ukey // nC
    e_lo = ukey % nC
    mid = 0.5 * (coords[e_hi] + coords[e_lo])
    new_coords = np.concatenate([coords, mid], axis=0)
    # local edge j runs v_j -> v_{j+1}; M1 = mid(v2,v3) is edge j=1,
    # M2 = mid(v3,v1) is j=2, M3 = mid(v1,v2) is j=0.
    M1 = nC + inv[:, 1]
    M2 = nC + inv[:, 2]
    M3 = nC + inv[:, 0]
    out = np.empty((4 * nE, 3), dtype=np.int64)
    out[:nE] = np.stack([M1, M2, M3], axis=1)
    out[nE + 0::3] = np.stack([elems[:, 0], M3, M2], axis=1)
    out[nE + 1::3] = np.stack([elems[:, 1], M1, M3], axis=1)
    out[nE + 2::3] = np.stack([elems[:, 2], M2, M1], axis=1)

    def refine_pairs(pairs):
        if len(pairs) == 0:
            return pairs
        p = pairs.astype(np.int64)
        k = np.maximum(p[:, 0], p[:, 1]) * np.int64(nC) + np.minimum(p[:, 0], p[:, 1])
        pos = np.searchsorted(ukey, k)
        if np.any(pos >= len(ukey)) or np.any(ukey[np.minimum(pos, len(ukey) - 1)] != k):
            raise ValueError("boundary pair is not an edge of the mesh")
        m = nC + pos
        first = np.stack([p[:, 0], m], axis=1)
        second = np.stack([m, p[:, 1]], axis=1)
        return np.concatenate([first, second], axis=0)

    if new_coords.shape[0] > np.iinfo(np.int32).max:
        raise ValueError("mesh too large for int32 node ids")
    return Mesh(new_coords, out.astype(np.int32), refine_pairs(mesh.dirichlet),
                refine_pairs(mesh.neumann), name=mesh.name)


def _paper_base(bc="paper"):
    """The paper's Table 1 start mesh, converted to 0-based indices.

    bc='paper': Dirichlet = {y=0, x=1}, Neumann = {y=1, x=0} (as in Table 1).
    bc='x_sides': Dirichlet = {x=0, x=1}, Neumann = {y=0, y=1}.
    bc='y_sides': Dirichlet = {y=0, y=1}, Neumann = {x=0, x=1}.
    """
    coords = np.array([[0, 0], [1, 0], [0, 1], [1, 1], [0.5, 0.5]], dtype=np.float64)
    elements = np.array([[5, 1, 2], [5, 3, 1], [5, 4, 3], [5, 2, 4]], dtype=np.int32) - 1
    bottom, right, top, left = [1, 2], [2, 4], [4, 3], [3, 1]
    if bc == "paper":
        D, N = [bottom, right], [top, left]
    elif bc == "x_sides":
        D, N = [right, left], [bottom, top]
    elif bc == "y_sides":
        D, N = [bottom, top], [right, left]
    elif bc == "all_dirichlet":
        D, N = [bottom, right, top, left], []
    else:
        raise ValueError(bc)
    D = np.array(D, dtype=np.int32).reshape(-1, 2) - 1
    N = np.array(N, dtype=np.int32).reshape(-1, 2) - 1
    return Mesh(coords, elements, D, N, name=f"paper_square[{bc}]")


def paper_square(level, bc="paper"):
    """Paper start mesh red-refined ``level`` times: 4^(level+1) triangles."""
    m = _paper_base(bc)
    for _ in range(int(level)):
        m = red_refine(m)
    m.name = f"paper_square_L{level}[{bc}]"
    return m


def _lshape_base():
    """Three unit squares, four CCW triangles each around the square centre.

    Re-entrant edges {x=0, y<=0} and {y=0, x>=0} form the Dirichlet list;
    the rest of the boundary is Neumann.
    """
    corners = {
        (-1, -1): 0, (0, -1): 1, (-1, 0): 2, (0, 0): 3, (1, 0): 4,
        (-1, 1): 5, (0, 1): 6, (1, 1): 7,
    }
    coords = [None] * 11
    for (x, y), k in corners.items():
        coords[k] = (float(x), float(y))
    squares = [(-1, -1), (-1, 0), (0, 0)]  # lower-left corners
    elements = []
    for s, (x0, y0) in enumerate(squares):
        c = 8 + s
        coords[c] = (x0 + 0.5, y0 + 0.5)
        bl = corners[(x0, y0)]
        br = corners[(x0 + 1, y0)]
        tr = corners[(x0 + 1, y0 + 1)]
        tl = corners[(x0, y0 + 1)]
        elements += [[c, bl, br], [c, br, tr], [c, tr, tl], [c, tl, bl]]
    k = corners
    # counter-clockwise boundary walk starting at (-1,-1)
    walk = [(-1, -1), (0, -1), (0, 0), (1, 0), (1, 1), (0, 1), (-1, 1), (-1, 0), (-1, -1)]
    D, N = [], []
    for p, q in zip(walk[:-1], walk[1:]):
        pair = [k[p], k[q]]
        reentrant = (p[0] == 0 and q[0] == 0 and max(p[1], q[1]) <= 0) or \
                    (p[1] == 0 and q[1] == 0 and min(p[0], q[0]) >= 0)
        (D if reentrant else N).append(pair)
    return Mesh(np.array(coords), np.array(elements, dtype=np.int32),
                np.array(D, dtype=np.int32), np.array(N, dtype=np.int32), name="lshape")


def lshape(level):
    """L-shaped domain, 12 * 4^level triangles."""
    m = _lshape_base()
    for _ in range(int(level)):
        m = red_refine(m)
    m.name = f"lshape_L{level}"
    return m


def jittered_square(n, rng, jitter=0.2, dirichlet_sides=("left", "right")):
    """Structured square whose interior nodes move uniformly in a disk.

    The disk radius is ``jitter * h`` with h = 1/n. For jitter < 1/(2 sqrt 2)
    every triangle stays counter-clockwise.
    """
    m = unit_square_structured(n, dirichlet_sides)
    xy = m.coords.copy()
    interior = (xy[:, 0] > 0) & (xy[:, 0] < 1) & (xy[:, 1] > 0) & (xy[:, 1] < 1)
    k = int(interior.sum())
    r = jitter / n * np.sqrt(rng.uniform(0.0, 1.0, size=k))
    th = rng.uniform(0.0, 2.0 * np.pi, size=k)
    xy[interior, 0] += r * np.cos(th)
    xy[interior, 1] += r * np.sin(th)
    m.coords = xy
    m.name = f"jitter{n}"
    return m


def per_triangle_coefficient(nE, seed, lo=0.5, hi=2.0):
    """Piecewise-constant coefficient a_T ~ U[lo, hi] per triangle."""
    rng = np.random.default_rng(seed)
    return rng.uniform(lo, hi, size=int(nE))


def batch_instances(count, seed, tmin=2e3, tmax=2e5, jitter=0.2):
    """Independent jittered unit-square instances of log-uniform size.

    Returns a list of (Mesh, a) with a ~ U[0.5, 2] per instance.
    """
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(int(count)):
        t = np.exp(rng.uniform(np.log(tmin), np.log(tmax)))
        n = max(2, int(round(np.sqrt(t / 2.0))))
        a = rng.uniform(0.5, 2.0)
        out.append((jittered_square(n, rng, jitter), float(a)))
    return out
