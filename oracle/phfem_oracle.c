/*
 * CPU oracle for the lowest-order primal hybrid FEM (Nagula Mallesham, Porwal,
 * Valdman, Acharya, "Vectorized implementation of primal hybrid FEM in
 * MATLAB", arXiv:2401.15557).
 *
 * TEST INFRASTRUCTURE ONLY. This file is the slow, plain, single-threaded
 * fp64 statement of what the GPU path must compute. Only the test suite, the
 * smoke check and the benchmark's CPU-baseline leg may load it. It shares no
 * code, header, table or helper with the HIP library.
 *
 * Conventions: 0-based indices. Local vertex i of element m is elem[3m+i];
 * "local edge i" is the edge opposite local vertex i (the paper's E_{i+1});
 * the directed local edge j runs v_j -> v_{(j+1)%3}, so it is local edge
 * (j+2)%3. Degrees of freedom: DOF 3m+i is the P1 basis function of element m
 * equal to the barycentric coordinate of its local vertex i (Section 3.3).
 *
 * Every function returns 0 on success and a negative code on error:
 *   -1 bad argument / index out of range, -2 element not counter-clockwise
 *   or degenerate, -3 edge shared by more than two elements or traversed in
 *   the same direction by both, -4 boundary lists inconsistent with the mesh,
 *   -5 out of memory.
 *
 * parity: pinned (see the oracle tests) except where a function says
 * otherwise.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_EINVAL -1
#define ORC_EORIENT -2
#define ORC_EMESH -3
#define ORC_EBOUNDARY -4
#define ORC_ENOMEM -5

/* ------------------------------------------------------------------------ */
/* Topology: the edge numbering and edge-to-element table of Section 2.2.    */
/* ------------------------------------------------------------------------ */

typedef struct {
    int32_t hi, lo; /* larger / smaller node id of the undirected edge */
    int32_t m, j;   /* element and directed local edge index */
} edge_rec;

static int cmp_edge_rec(const void* pa, const void* pb)
{
    const edge_rec* a = (const edge_rec*)pa;
    const edge_rec* b = (const edge_rec*)pb;
    if (a->hi != b->hi) return a->hi < b->hi ? -1 : 1;
    if (a->lo != b->lo) return a->lo < b->lo ? -1 : 1;
    if (a->m != b->m) return a->m < b->m ? -1 : 1;
    if (a->j != b->j) return a->j < b->j ? -1 : 1;
    return 0;
}

/*
 * Edges are numbered in ascending (larger node, smaller node) order, which is
 * the column-major order of the upper triangle of the node adjacency matrix
 * used to build nodes2edge (Section 2.2.2). For each edge:
 *   edge_elems = [T+, T-] where T+ is the element of the first occurrence in
 *     element order and T- the other element (-1 on the boundary) (2.2.3);
 *   edge_nodes = [k, l] = the edge traversed as in T+ (initial, end node);
 *   led   = local edge number (opposite local vertex, 0..2) in T+;
 *   ledTN = local edge number in T- (equal to led on the boundary).
 * elem_edges[3m+i] = global id of the edge opposite local vertex i of m.
 * Capacity of the edge arrays: 3*nE entries.
 */
int orc_topology(int32_t nC, int32_t nE, const int32_t* elem, int32_t* n_edges_out,
                 int32_t* edge_nodes, int32_t* edge_elems, int32_t* elem_edges,
                 int8_t* led, int8_t* ledTN)
{
    if (nC < 0 || nE < 0 || (nE > 0 && !elem) || !n_edges_out) return ORC_EINVAL;
    for (int64_t q = 0; q < 3 * (int64_t)nE; ++q)
        if (elem[q] < 0 || elem[q] >= nC) return ORC_EINVAL;
    int64_t nrec = 3 * (int64_t)nE;
    edge_rec* r = (edge_rec*)malloc((size_t)(nrec > 0 ? nrec : 1) * sizeof(edge_rec));
    if (!r) return ORC_ENOMEM;
    for (int32_t m = 0; m < nE; ++m) {
        for (int j = 0; j < 3; ++j) {
            int32_t a = elem[3 * (int64_t)m + j];
            int32_t b = elem[3 * (int64_t)m + (j + 1) % 3];
            if (a == b) { free(r); return ORC_EORIENT; }
            edge_rec* e = &r[3 * (int64_t)m + j];
            e->hi = a > b ? a : b;
            e->lo = a > b ? b : a;
            e->m = m;
            e->j = j;
        }
    }
    qsort(r, (size_t)nrec, sizeof(edge_rec), cmp_edge_rec);
    int32_t ne = 0;
    int64_t s = 0;
    while (s < nrec) {
        int64_t t = s + 1;
        while (t < nrec && r[t].hi == r[s].hi && r[t].lo == r[s].lo) ++t;
        if (t - s > 2) { free(r); return ORC_EMESH; }
        const edge_rec* p = &r[s];
        int32_t k = elem[3 * (int64_t)p->m + p->j];
        int32_t l = elem[3 * (int64_t)p->m + (p->j + 1) % 3];
        edge_nodes[2 * (int64_t)ne] = k;
        edge_nodes[2 * (int64_t)ne + 1] = l;
        edge_elems[2 * (int64_t)ne] = p->m;
        led[ne] = (int8_t)((p->j + 2) % 3);
        elem_edges[3 * (int64_t)p->m + (p->j + 2) % 3] = ne;
        if (t - s == 2) {
            const edge_rec* q = &r[s + 1];
            int32_t k2 = elem[3 * (int64_t)q->m + q->j];
            /* both neighbours counter-clockwise => opposite traversal */
            if (k2 == k || q->m == p->m) { free(r); return ORC_EMESH; }
            edge_elems[2 * (int64_t)ne + 1] = q->m;
            ledTN[ne] = (int8_t)((q->j + 2) % 3);
            elem_edges[3 * (int64_t)q->m + (q->j + 2) % 3] = ne;
        } else {
            edge_elems[2 * (int64_t)ne + 1] = -1;
            ledTN[ne] = led[ne];
        }
        ++ne;
        s = t;
    }
    free(r);
    *n_edges_out = ne;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Boundary classification (the Dbed / Nbed / Redges lookups of Main.m).     */
/* ------------------------------------------------------------------------ */

static int32_t find_edge(int32_t n_edges, const int32_t* edge_nodes, int32_t a, int32_t b)
{
    int32_t hi = a > b ? a : b, lo = a > b ? b : a;
    int32_t L = 0, R = n_edges - 1;
    while (L <= R) {
        int32_t mid = L + (R - L) / 2;
        int32_t k = edge_nodes[2 * (int64_t)mid], l = edge_nodes[2 * (int64_t)mid + 1];
        int32_t h2 = k > l ? k : l, l2 = k > l ? l : k;
        if (h2 == hi && l2 == lo) return mid;
        if (h2 < hi || (h2 == hi && l2 < lo)) L = mid + 1;
        else R = mid - 1;
    }
    return -1;
}

/*
 * edge_type[e] = 0 interior, 1 Dirichlet, 2 Neumann.
 * dir_edges / neu_edges: edge id of each listed pair (list order).
 * edge_row[e] = multiplier row of edge e: its rank among the non-Neumann
 * edges in ascending id order (the Redges enumeration), -1 for Neumann.
 * Every boundary edge must appear in exactly one list; listed pairs must be
 * boundary edges. *L_out = number of multiplier rows.
 */
int orc_boundary(int32_t n_edges, const int32_t* edge_nodes, const int32_t* edge_elems,
                 int32_t nD, const int32_t* dir, int32_t nN, const int32_t* neu,
                 int8_t* edge_type, int32_t* dir_edges, int32_t* neu_edges,
                 int32_t* edge_row, int32_t* L_out)
{
    if (n_edges < 0 || nD < 0 || nN < 0) return ORC_EINVAL;
    int8_t* listed = (int8_t*)calloc((size_t)(n_edges > 0 ? n_edges : 1), 1);
    if (!listed) return ORC_ENOMEM;
    for (int32_t e = 0; e < n_edges; ++e) edge_type[e] = 0;
    for (int pass = 0; pass < 2; ++pass) {
        int32_t n = pass == 0 ? nD : nN;
        const int32_t* pairs = pass == 0 ? dir : neu;
        int32_t* out = pass == 0 ? dir_edges : neu_edges;
        for (int32_t q = 0; q < n; ++q) {
            int32_t e = find_edge(n_edges, edge_nodes, pairs[2 * (int64_t)q],
                                  pairs[2 * (int64_t)q + 1]);
            if (e < 0 || edge_elems[2 * (int64_t)e + 1] >= 0 || listed[e]) {
                free(listed);
                return ORC_EBOUNDARY;
            }
            listed[e] = 1;
            edge_type[e] = (int8_t)(pass + 1);
            out[q] = e;
        }
    }
    for (int32_t e = 0; e < n_edges; ++e) {
        if (edge_elems[2 * (int64_t)e + 1] < 0 && !listed[e]) {
            free(listed);
            return ORC_EBOUNDARY;
        }
    }
    free(listed);
    int32_t L = 0;
    for (int32_t e = 0; e < n_edges; ++e) edge_row[e] = edge_type[e] == 2 ? -1 : L++;
    *L_out = L;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Problem data: the analytic source, flux and boundary functions used by    */
/* the paper's examples and by the synthetic workloads.                      */
/* ------------------------------------------------------------------------ */

enum {
    FN_ZERO = 0,
    FN_CONST = 1,       /* c0 */
    FN_SIN_COS = 2,     /* c0 exp(c1 t) sin(pi x) cos(pi y) */
    FN_SIN_SIN = 3,     /* c0 exp(c1 t) sin(pi x) sin(pi y) */
    FN_GRAD_SIN_COS = 4,/* flux vector c0 exp(c1 t) grad(sin(pi x) cos(pi y)) */
    FN_GRAD_SIN_SIN = 5,/* flux vector c0 exp(c1 t) grad(sin(pi x) sin(pi y)) */
    FN_PAPER_U = 6,     /* (c0 + c1 t)(x - x^2)(y - y^2) */
    FN_PAPER_F = 7,     /* source of the paper's examples 1 and 2 */
    FN_PAPER_FLUX = 8,  /* flux vector of the paper's examples 1 and 2 */
    FN_EDGE_ARRAY = 100 /* value given per global edge id (edge midpoint) */
};

typedef struct {
    int32_t kind;
    int32_t pad;
    double c[4];
    const double* edge_values;
} orc_fn;

/* Scalar value at (x, y, t); for a flux kind, the flux dotted with nu. */
static double fn_eval(const orc_fn* f, double x, double y, double t, double nx, double ny,
                      int32_t edge)
{
    const double pi = 3.14159265358979323846;
    switch (f->kind) {
    case FN_ZERO: return 0.0;
    case FN_CONST: return f->c[0];
    case FN_SIN_COS: return f->c[0] * exp(f->c[1] * t) * sin(pi * x) * cos(pi * y);
    case FN_SIN_SIN: return f->c[0] * exp(f->c[1] * t) * sin(pi * x) * sin(pi * y);
    case FN_GRAD_SIN_COS: {
        double gx = pi * cos(pi * x) * cos(pi * y);
        double gy = -pi * sin(pi * x) * sin(pi * y);
        return f->c[0] * exp(f->c[1] * t) * (gx * nx + gy * ny);
    }
    case FN_GRAD_SIN_SIN: {
        double gx = pi * cos(pi * x) * sin(pi * y);
        double gy = pi * sin(pi * x) * cos(pi * y);
        return f->c[0] * exp(f->c[1] * t) * (gx * nx + gy * ny);
    }
    case FN_PAPER_U: return (f->c[0] + f->c[1] * t) * (x - x * x) * (y - y * y);
    case FN_PAPER_F: {
        double tau = f->c[0] + f->c[1] * t;
        double sx = x - x * x, sy = y - y * y;
        double s = sx * sy;
        return f->c[1] * s +
               tau * (2.0 * sy + 2.0 * sx + (1.0 - 2.0 * x) * sy + sx * (1.0 - 2.0 * y) + s);
    }
    case FN_PAPER_FLUX: {
        double tau = f->c[0] + f->c[1] * t;
        double qx = (1.0 - x - x * x) * (y - y * y);
        double qy = (x - x * x) * (1.0 - y - y * y);
        return tau * (qx * nx + qy * ny);
    }
    case FN_EDGE_ARRAY: return f->edge_values[edge];
    default: return NAN;
    }
}

/* ------------------------------------------------------------------------ */
/* Element quantities (Definition 3.1 and Section 3.4).                     */
/* ------------------------------------------------------------------------ */

/*
 * Barycentric coordinates lambda_i(x, y) = c[i][0] + c[i][1] x + c[i][2] y,
 * obtained by solving V c_i = e_i with V = [1 x_k y_k] (rows k = vertices),
 * i.e. c = V^{-1} by Gauss-Jordan elimination with partial pivoting.
 * Returns the signed area (positive for counter-clockwise vertices).
 */
static double barycentric(const double x[3], const double y[3], double c[3][3])
{
    double a[3][6];
    for (int k = 0; k < 3; ++k) {
        a[k][0] = 1.0; a[k][1] = x[k]; a[k][2] = y[k];
        for (int q = 0; q < 3; ++q) a[k][3 + q] = (k == q) ? 1.0 : 0.0;
    }
    for (int col = 0; col < 3; ++col) {
        int piv = col;
        for (int k = col + 1; k < 3; ++k)
            if (fabs(a[k][col]) > fabs(a[piv][col])) piv = k;
        if (piv != col)
            for (int q = 0; q < 6; ++q) { double t = a[col][q]; a[col][q] = a[piv][q]; a[piv][q] = t; }
        double d = a[col][col];
        if (d == 0.0) return 0.0;
        for (int q = 0; q < 6; ++q) a[col][q] /= d;
        for (int k = 0; k < 3; ++k) {
            if (k == col) continue;
            double f = a[k][col];
            for (int q = 0; q < 6; ++q) a[k][q] -= f * a[col][q];
        }
    }
    /* V^{-1}: column i holds the coefficients of lambda_i */
    for (int i = 0; i < 3; ++i)
        for (int q = 0; q < 3; ++q) c[i][q] = a[q][3 + i];
    return 0.5 * ((x[1] - x[0]) * (y[2] - y[0]) - (x[2] - x[0]) * (y[1] - y[0]));
}

/*
 * Local matrices of element m (Definition 3.1), row = test function index j,
 * column = trial index i, stored row-major [3][3]:
 *   K[j][i] = a_T |T| (A grad lambda_j) . grad lambda_i        (stiffness)
 *   D[j][i] = int_T lambda_j (p . grad lambda_i)              (convection)
 *   M[j][i] = int_T lambda_j lambda_i = |T|/12 (1 + delta_ij)  (unit mass)
 * b[j] = (|T|/3) sum_i f(m_{E_i}) lambda_j(m_{E_i})  (midpoint rule, 3.4).
 * The mass is returned without the reaction coefficient delta.
 */
static int element_local(const double x[3], const double y[3], const double A[4], double aT,
                         const double p[2], const orc_fn* f, double t,
                         const int32_t* edges_of_m, double K[9], double D[9], double M[9],
                         double b[3])
{
    double c[3][3];
    double area = barycentric(x, y, c);
    if (!(area > 0.0)) return ORC_EORIENT;
    for (int j = 0; j < 3; ++j) {
        double gj[2] = {c[j][1], c[j][2]};
        double Agj[2] = {A[0] * gj[0] + A[1] * gj[1], A[2] * gj[0] + A[3] * gj[1]};
        for (int i = 0; i < 3; ++i) {
            double gi[2] = {c[i][1], c[i][2]};
            K[3 * j + i] = aT * area * (Agj[0] * gi[0] + Agj[1] * gi[1]);
            /* int_T lambda_j = |T|/3 */
            D[3 * j + i] = (area / 3.0) * (p[0] * gi[0] + p[1] * gi[1]);
            M[3 * j + i] = area / 12.0 * (i == j ? 2.0 : 1.0);
        }
    }
    if (b) {
        for (int j = 0; j < 3; ++j) b[j] = 0.0;
        for (int ei = 0; ei < 3; ++ei) {
            /* edge E_ei is opposite vertex ei: its midpoint */
            int v1 = (ei + 1) % 3, v2 = (ei + 2) % 3;
            double mx = 0.5 * (x[v1] + x[v2]), my = 0.5 * (y[v1] + y[v2]);
            double fv = fn_eval(f, mx, my, t, 0.0, 0.0, edges_of_m ? edges_of_m[ei] : -1);
            for (int j = 0; j < 3; ++j) {
                double lam = c[j][0] + c[j][1] * mx + c[j][2] * my;
                b[j] += (area / 3.0) * fv * lam;
            }
        }
    }
    return 0;
}

/* Single-element evaluation for sampled checks at large sizes. */
int orc_element(const double* xy, const int32_t* elem, int32_t m, const double* A, double aT,
                const double* p, const orc_fn* f, double t, const int32_t* elem_edges,
                double* K, double* D, double* M, double* b)
{
    double x[3], y[3];
    for (int k = 0; k < 3; ++k) {
        int32_t v = elem[3 * (int64_t)m + k];
        x[k] = xy[2 * (int64_t)v];
        y[k] = xy[2 * (int64_t)v + 1];
    }
    return element_local(x, y, A, aT, p, f, t, elem_edges ? elem_edges + 3 * (int64_t)m : NULL,
                         K, D, M, b);
}

/* ------------------------------------------------------------------------ */
/* Triplet -> CSR: the plain definition of global assembly (sum of local    */
/* contributions at equal (row, column)), with structural zeros kept.        */
/* ------------------------------------------------------------------------ */

typedef struct {
    int32_t i, j;
    double v;
} trip;

static int cmp_trip(const void* pa, const void* pb)
{
    const trip* a = (const trip*)pa;
    const trip* b = (const trip*)pb;
    if (a->i != b->i) return a->i < b->i ? -1 : 1;
    if (a->j != b->j) return a->j < b->j ? -1 : 1;
    /* tie-break on value so the summation order is fixed */
    if (a->v != b->v) return a->v < b->v ? -1 : 1;
    return 0;
}

typedef struct {
    trip* t;
    int64_t n, cap;
} trip_list;

static int tl_push(trip_list* l, int32_t i, int32_t j, double v)
{
    if (l->n == l->cap) {
        int64_t nc = l->cap ? 2 * l->cap : 1024;
        trip* nt = (trip*)realloc(l->t, (size_t)nc * sizeof(trip));
        if (!nt) return ORC_ENOMEM;
        l->t = nt;
        l->cap = nc;
    }
    l->t[l->n].i = i;
    l->t[l->n].j = j;
    l->t[l->n].v = v;
    l->n++;
    return 0;
}

/* Sorts the triplets and merges duplicates. Writes rowptr[nrows+1]; col and
 * val must hold at least l->n entries. Returns nnz. */
static int64_t tl_to_csr(trip_list* l, int32_t nrows, int32_t* rowptr, int32_t* col, double* val)
{
    qsort(l->t, (size_t)l->n, sizeof(trip), cmp_trip);
    int64_t nnz = 0;
    for (int32_t r = 0; r <= nrows; ++r) rowptr[r] = 0;
    for (int64_t q = 0; q < l->n;) {
        int64_t s = q;
        double sum = 0.0;
        while (q < l->n && l->t[q].i == l->t[s].i && l->t[q].j == l->t[s].j) sum += l->t[q++].v;
        col[nnz] = l->t[s].j;
        val[nnz] = sum;
        rowptr[l->t[s].i + 1]++;
        nnz++;
    }
    for (int32_t r = 0; r < nrows; ++r) rowptr[r + 1] += rowptr[r];
    return nnz;
}

/*
 * Global assembly (Sections 3.3-3.5):
 *   K, D, M: N x N (N = 3 nE), 9 structural entries per element;
 *   C: L x N, row edge_row[e] of each non-Neumann edge e, with entries
 *      C[row(e), 3T + j] = sigma |E| / 2 for the two vertices j of e in each
 *      neighbour T (sigma = +1 in T+, -1 in T-); the integral of a barycentric
 *      coordinate over an edge through its vertex is |E|/2;
 *   F = b + LN: N, LN adds |E| g(m_E) lambda_j(m_E) for each Neumann edge in
 *      its element (g = flux dotted with the outward normal of that element);
 *   bD: L, bD[row(e)] = -|E| u_D(m_E) for Dirichlet edges, 0 otherwise.
 * Output CSR arrays must be sized: K/D/M col,val 9 nE, rowptr N+1;
 * C col,val 4 L (upper bound), rowptr L+1. *nnzC_out receives nnz(C).
 */
int orc_assemble(int32_t nC, const double* xy, int32_t nE, const int32_t* elem,
                 int32_t n_edges, const int32_t* edge_nodes, const int32_t* edge_elems,
                 const int32_t* elem_edges, const int8_t* edge_type, const int32_t* edge_row,
                 int32_t L, const double* A, const double* p, const double* aT,
                 const orc_fn* f, const orc_fn* g, const orc_fn* uD, double t,
                 int32_t* K_rowptr, int32_t* K_col, double* K_val, double* D_val, double* M_val,
                 int32_t* C_rowptr, int32_t* C_col, double* C_val, int64_t* nnzC_out,
                 double* F, double* bD)
{
    (void)nC;
    int32_t N = 3 * nE;
    trip_list lk = {0}, ld = {0}, lm = {0}, lc = {0};
    int rc = 0;
    for (int32_t r = 0; r < N; ++r) F[r] = 0.0;
    for (int32_t m = 0; m < nE && rc == 0; ++m) {
        double K[9], D[9], M[9], b[3];
        rc = orc_element(xy, elem, m, A, aT ? aT[m] : 1.0, p, f, t, elem_edges, K, D, M, b);
        if (rc) break;
        for (int j = 0; j < 3; ++j) {
            for (int i = 0; i < 3; ++i) {
                int32_t row = 3 * m + j, colx = 3 * m + i;
                if (tl_push(&lk, row, colx, K[3 * j + i]) || tl_push(&ld, row, colx, D[3 * j + i]) ||
                    tl_push(&lm, row, colx, M[3 * j + i])) {
                    rc = ORC_ENOMEM;
                }
            }
            F[3 * m + j] += b[j];
        }
    }
    /* coupling matrix and boundary data, edge by edge */
    for (int32_t e = 0; e < n_edges && rc == 0; ++e) {
        int32_t k = edge_nodes[2 * (int64_t)e], l = edge_nodes[2 * (int64_t)e + 1];
        double dx = xy[2 * (int64_t)l] - xy[2 * (int64_t)k];
        double dy = xy[2 * (int64_t)l + 1] - xy[2 * (int64_t)k + 1];
        double len = sqrt(dx * dx + dy * dy);
        double mx = 0.5 * (xy[2 * (int64_t)k] + xy[2 * (int64_t)l]);
        double my = 0.5 * (xy[2 * (int64_t)k + 1] + xy[2 * (int64_t)l + 1]);
        if (edge_type[e] == 2) {
            /* Neumann: k -> l is counter-clockwise in T+, outward normal on the right */
            double nx = dy / len, ny = -dx / len;
            double gv = fn_eval(g, mx, my, t, nx, ny, e);
            int32_t T = edge_elems[2 * (int64_t)e];
            for (int j = 0; j < 3; ++j) {
                int32_t v = elem[3 * (int64_t)T + j];
                double lam = (v == k || v == l) ? 0.5 : 0.0; /* lambda_j at m_E */
                F[3 * T + j] += len * gv * lam;
            }
            continue;
        }
        int32_t row = edge_row[e];
        for (int side = 0; side < 2; ++side) {
            int32_t T = edge_elems[2 * (int64_t)e + side];
            if (T < 0) continue;
            double sigma = side == 0 ? 1.0 : -1.0;
            for (int j = 0; j < 3; ++j) {
                int32_t v = elem[3 * (int64_t)T + j];
                if (v == k || v == l) {
                    if (tl_push(&lc, row, 3 * T + j, sigma * len * 0.5)) rc = ORC_ENOMEM;
                }
            }
        }
        bD[row] = edge_type[e] == 1 ? -len * fn_eval(uD, mx, my, t, 0.0, 0.0, e) : 0.0;
    }
    if (rc == 0) {
        int32_t* tmp_rp = (int32_t*)malloc(sizeof(int32_t) * ((size_t)N + 1));
        int32_t* tmp_col = (int32_t*)malloc(sizeof(int32_t) * ((size_t)lk.n + 1));
        if (!tmp_rp || !tmp_col) rc = ORC_ENOMEM;
        if (rc == 0) {
            tl_to_csr(&lk, N, K_rowptr, K_col, K_val);
            tl_to_csr(&ld, N, tmp_rp, tmp_col, D_val);
            tl_to_csr(&lm, N, tmp_rp, tmp_col, M_val);
            *nnzC_out = tl_to_csr(&lc, L, C_rowptr, C_col, C_val);
        }
        free(tmp_rp);
        free(tmp_col);
    }
    free(lk.t); free(ld.t); free(lm.t); free(lc.t);
    return rc;
}

/*
 * Saddle-point matrix M_vec = [Kc + D + delta M, -C^T; -C, 0] of the global
 * system (Section 3.5), (N+L) x (N+L), from the assembled pieces. The
 * (1,1) block keeps all 9 structural entries per element. Capacity of
 * col/val: 9 nE + 2 nnz(C). Returns nnz through *nnz_out.
 */
int orc_saddle(int32_t nE, int32_t L, const int32_t* K_rowptr, const int32_t* K_col,
               const double* K_val, const double* D_val, const double* M_val, double delta,
               const int32_t* C_rowptr, const int32_t* C_col, const double* C_val,
               int32_t* rowptr, int32_t* col, double* val, int64_t* nnz_out)
{
    int32_t N = 3 * nE;
    trip_list l = {0};
    int rc = 0;
    for (int32_t r = 0; r < N && rc == 0; ++r)
        for (int32_t q = K_rowptr[r]; q < K_rowptr[r + 1]; ++q)
            rc = tl_push(&l, r, K_col[q], K_val[q] + D_val[q] + delta * M_val[q]);
    for (int32_t r = 0; r < L && rc == 0; ++r)
        for (int32_t q = C_rowptr[r]; q < C_rowptr[r + 1] && rc == 0; ++q) {
            rc = tl_push(&l, N + r, C_col[q], -C_val[q]);
            if (!rc) rc = tl_push(&l, C_col[q], N + r, -C_val[q]);
        }
    if (rc == 0) *nnz_out = tl_to_csr(&l, N + L, rowptr, col, val);
    free(l.t);
    return rc;
}

/* Plain CSR matrix-vector product y = A x (for residual checks). */
void orc_csr_matvec(int32_t nrows, const int32_t* rowptr, const int32_t* col, const double* val,
                    const double* x, double* y)
{
    for (int32_t r = 0; r < nrows; ++r) {
        double s = 0.0;
        for (int32_t q = rowptr[r]; q < rowptr[r + 1]; ++q) s += val[q] * x[col[q]];
        y[r] = s;
    }
}

/* ------------------------------------------------------------------------ */
/* Uniform red refinement (Section 2.3, Listing 4).                          */
/* ------------------------------------------------------------------------ */

/*
 * One red refinement with the paper's numbering, given the coarse edge table
 * of orc_topology: the midpoint of edge e becomes node nC + e; element m is
 * replaced by its interior child [M1 M2 M3] (M_i = midpoint of the edge
 * opposite vertex i) and the corner children [v1 M3 M2], [v2 M1 M3],
 * [v3 M2 M1] are appended at nE + 3m, nE + 3m + 1, nE + 3m + 2. Each listed
 * boundary pair (a, b) of edge e becomes (a, M_e) in the first half of the new
 * list and (M_e, b) in the second half. Output sizes: xy_f 2 (nC + n_edges),
 * elem_f 3 * 4 nE, dir_f 2 * 2 nD, neu_f 2 * 2 nN.
 */
int orc_red_refine(int32_t nC, const double* xy, int32_t nE, const int32_t* elem,
                   int32_t n_edges, const int32_t* edge_nodes, const int32_t* elem_edges,
                   int32_t nD, const int32_t* dir, const int32_t* dir_edges, int32_t nN,
                   const int32_t* neu, const int32_t* neu_edges, double* xy_f, int32_t* elem_f,
                   int32_t* dir_f, int32_t* neu_f)
{
    for (int64_t q = 0; q < 2 * (int64_t)nC; ++q) xy_f[q] = xy[q];
    for (int32_t e = 0; e < n_edges; ++e) {
        int32_t k = edge_nodes[2 * (int64_t)e], l = edge_nodes[2 * (int64_t)e + 1];
        xy_f[2 * ((int64_t)nC + e)] = 0.5 * (xy[2 * (int64_t)k] + xy[2 * (int64_t)l]);
        xy_f[2 * ((int64_t)nC + e) + 1] = 0.5 * (xy[2 * (int64_t)k + 1] + xy[2 * (int64_t)l + 1]);
    }
    for (int32_t m = 0; m < nE; ++m) {
        int32_t v[3], M[3];
        for (int i = 0; i < 3; ++i) {
            v[i] = elem[3 * (int64_t)m + i];
            M[i] = nC + elem_edges[3 * (int64_t)m + i];
        }
        int32_t* c = elem_f + 3 * (int64_t)m;
        c[0] = M[0]; c[1] = M[1]; c[2] = M[2];
        for (int i = 0; i < 3; ++i) {
            /* corner child at vertex i: [v_i, M_(i+2), M_(i+1)] */
            int32_t* d = elem_f + 3 * ((int64_t)nE + 3 * (int64_t)m + i);
            d[0] = v[i];
            d[1] = M[(i + 2) % 3];
            d[2] = M[(i + 1) % 3];
        }
    }
    for (int pass = 0; pass < 2; ++pass) {
        int32_t n = pass == 0 ? nD : nN;
        const int32_t* pr = pass == 0 ? dir : neu;
        const int32_t* ed = pass == 0 ? dir_edges : neu_edges;
        int32_t* out = pass == 0 ? dir_f : neu_f;
        for (int32_t q = 0; q < n; ++q) {
            int32_t mid = nC + ed[q];
            out[2 * (int64_t)q] = pr[2 * (int64_t)q];
            out[2 * (int64_t)q + 1] = mid;
            out[2 * ((int64_t)n + q)] = mid;
            out[2 * ((int64_t)n + q) + 1] = pr[2 * (int64_t)q + 1];
        }
    }
    return 0;
}
