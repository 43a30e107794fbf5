// Numeric assembly (Definition 3.1, Sections 3.4-3.5): one fused launch with
// element tiles (K, M, optional D, F = b + LN) and multiplier-row tiles (C,
// b_D). Every output entry has exactly one producer, so there are no atomics
// and no reductions across threads: the CSR "scatter" of the block-diagonal
// K, M, D is the identity map (element m owns values 9m..9m+8), and C rows
// are written in place at their precomputed row pointers.
//
// Memory layout: element tiles read element-major vertex coordinates
// (three double2 per triangle, streamed), not the node array through vertex
// ids: with the paper's red-refinement numbering consecutive triangles are
// far apart, and three scattered 16-byte gathers per triangle cost more than
// streaming 48 bytes. On a mesh refined by phf_mesh_refine the tiles form
// each child's vertices from its parent's record (24 bytes per element
// instead of 48); other meshes read their own. An element tile of 256
// triangles computes its 9 K values per element into LDS and the whole tile
// then streams out as one contiguous 18 KB block with 16-byte non-temporal
// stores; M is regenerated from the staged areas; F from a staged 3-value
// record. Multiplier rows gather their two end nodes (rows are in edge-id
// order, so the larger end node is monotone).
#include <algorithm>
#include <cstring>

#include "phf_device.h"
#include "phf_internal.h"

namespace {

constexpr int TILE = 256;

struct AsmArgs {
    int32_t nE, L, nbE, nbR;
    int32_t nEp, pad_;      // refined meshes: elements of the coarse mesh (nE = 4 nEp)
    const double2* exy;
    const double2* pexy;    // coarse mesh's element-major coordinates, or null
    const int4* elem4;      // vertex ids (and code) of each element
    const int32_t* ecode;
    const double2* xy;
    const double* aT;
    const int32_t* elem_edges;
    const double* row_hs;
    const int2* row_nodes;
    const int32_t* row_edge;
    const int32_t* C_tile;   // row pointer of every 256th row
    const int32_t* C_rowptr;
    const uint64_t* neu_mask;
    double A00, A01, A10, A11, p0, p1;
    phf_fn_dev f, g, uD;
    double t;
    const int64_t* t_step;
    double t0, dt;
    double* K;
    double* M;
    double* D;
    double* C;
    double* F;
    double* bD;
};

// Splits the fused grid between element tiles and row tiles in proportion,
// so that both kinds run side by side over the whole launch: block b is an
// element tile iff floor((b+1) nbE / T) > floor(b nbE / T), T = nbE + nbR.
// (Dealing contiguous ranges to each XCD measured slower.)
__device__ inline void fused_tile(int32_t b, int32_t nbE, int32_t nbR, bool* is_elem,
                                  int32_t* tile)
{
    const int32_t T = nbE + nbR;
    const int32_t e0 = (int32_t)(((int64_t)b * nbE) / T);
    const int32_t e1 = (int32_t)(((int64_t)(b + 1) * nbE) / T);
    if (e1 > e0) {
        *is_elem = true;
        *tile = e0;
    } else {
        *is_elem = false;
        *tile = b - e0;
    }
}

// f, g or u_D at one point. OOL = false inlines the evaluation (the
// single-mesh kernel); OOL = true calls one out-of-line copy: the batched
// kernel has 120 instantiations, and inlining the fp64 sine, cosine and
// exponential at its seven call sites grows the library from 2 to 15 MB for
// about 1% of its time. The evaluation contracts no multiply-adds, so both
// forms round alike.
__device__ __noinline__ double fn_eval_call(int32_t kind, double c0, double c1, double c2,
                                           double c3, const double* ev, double x, double y,
                                           double t, double nx, double ny, int32_t edge)
{
    phf_fn_dev f;
    f.kind = kind;
    f.c0 = c0;
    f.c1 = c1;
    f.c2 = c2;
    f.c3 = c3;
    f.ev = ev;
    return phf_fn_eval(f, x, y, t, nx, ny, edge);
}

template <bool OOL>
__device__ inline double fn_at(const phf_fn_dev& f, double x, double y, double t, double nx,
                               double ny, int32_t edge)
{
    if (OOL) return fn_eval_call(f.kind, f.c0, f.c1, f.c2, f.c3, f.ev, x, y, t, nx, ny, edge);
    return phf_fn_eval(f, x, y, t, nx, ny, edge);
}

// Element m with vertices P0, P1, P2 (counter-clockwise): its K (9 values,
// row-major), |T|/12 (M is regenerated from it), D and F = b + LN (3 values)
// into LDS slot `slot`.
template <bool HAS_AT, bool MATS, bool WITH_D, bool GEN_A, bool OOL = false>
__device__ inline void element_values(const AsmArgs& a, int32_t m, const double2 P0,
                                      const double2 P1, const double2 P2, int slot, double* shK,
                                      double* shD, double* shA, double* shF)
{
    // No contraction into fused multiply-adds here: element and parent tiles
    // (different instantiations, scheduled differently) then round every
    // value the same way and give bit-identical outputs.
#pragma clang fp contract(off)
    // g_i = 2|T| grad lambda_i (the edge opposite vertex i turned by 90 deg)
    const double g0x = P1.y - P2.y, g0y = P2.x - P1.x;
    const double g1x = P2.y - P0.y, g1y = P0.x - P2.x;
    const double g2x = P0.y - P1.y, g2y = P1.x - P0.x;
    const double det = (P1.x - P0.x) * (P2.y - P0.y) - (P2.x - P0.x) * (P1.y - P0.y);
    const double area = 0.5 * det;
    if (MATS) {
        const double aT = HAS_AT ? a.aT[m] : 1.0;
        const double s = aT / (2.0 * det);
        double k00, k01, k02, k11, k12, k22, k10, k20, k21;
        if (GEN_A) {
            // K[j][i] = aT |T| (A grad lambda_j) . grad lambda_i
            double a0x = a.A00 * g0x + a.A01 * g0y, a0y = a.A10 * g0x + a.A11 * g0y;
            double a1x = a.A00 * g1x + a.A01 * g1y, a1y = a.A10 * g1x + a.A11 * g1y;
            double a2x = a.A00 * g2x + a.A01 * g2y, a2y = a.A10 * g2x + a.A11 * g2y;
            k00 = s * (a0x * g0x + a0y * g0y);
            k01 = s * (a0x * g1x + a0y * g1y);
            k02 = s * (a0x * g2x + a0y * g2y);
            k10 = s * (a1x * g0x + a1y * g0y);
            k11 = s * (a1x * g1x + a1y * g1y);
            k12 = s * (a1x * g2x + a1y * g2y);
            k20 = s * (a2x * g0x + a2y * g0y);
            k21 = s * (a2x * g1x + a2y * g1y);
            k22 = s * (a2x * g2x + a2y * g2y);
        } else {
            k00 = s * (g0x * g0x + g0y * g0y);
            k11 = s * (g1x * g1x + g1y * g1y);
            k22 = s * (g2x * g2x + g2y * g2y);
            k01 = s * (g0x * g1x + g0y * g1y);
            k02 = s * (g0x * g2x + g0y * g2y);
            k12 = s * (g1x * g2x + g1y * g2y);
            k10 = k01;
            k20 = k02;
            k21 = k12;
        }
        double* kk = shK + slot * 9;
        kk[0] = k00; kk[1] = k01; kk[2] = k02;
        kk[3] = k10; kk[4] = k11; kk[5] = k12;
        kk[6] = k20; kk[7] = k21; kk[8] = k22;
        shA[slot] = area / 12.0;
        if (WITH_D) {
            // D[j][i] = (|T|/3) p . grad lambda_i = p . g_i / 6
            double h0 = (a.p0 * g0x + a.p1 * g0y) / 6.0;
            double h1 = (a.p0 * g1x + a.p1 * g1y) / 6.0;
            double h2 = (a.p0 * g2x + a.p1 * g2y) / 6.0;
            double* dd = shD + slot * 9;
            dd[0] = h0; dd[1] = h1; dd[2] = h2;
            dd[3] = h0; dd[4] = h1; dd[5] = h2;
            dd[6] = h0; dd[7] = h1; dd[8] = h2;
        }
    }
    // source load: midpoint rule over the three edge midpoints; the
    // midpoint of edge i (opposite vertex i) has lambda_j = 1/2, j != i
    int32_t ed0 = -1, ed1 = -1, ed2 = -1;
    const bool fe = a.f.kind == PHF_FN_EDGE_ARRAY;
    if (fe) {
        ed0 = a.elem_edges[3 * (int64_t)m];
        ed1 = a.elem_edges[3 * (int64_t)m + 1];
        ed2 = a.elem_edges[3 * (int64_t)m + 2];
    }
    double b0 = 0.0, b1 = 0.0, b2 = 0.0;
    if (a.f.kind != PHF_FN_ZERO) {
        const double f0 = fn_at<OOL>(a.f, 0.5 * (P1.x + P2.x), 0.5 * (P1.y + P2.y), a.t, 0, 0, ed0);
        const double f1 = fn_at<OOL>(a.f, 0.5 * (P2.x + P0.x), 0.5 * (P2.y + P0.y), a.t, 0, 0, ed1);
        const double f2 = fn_at<OOL>(a.f, 0.5 * (P0.x + P1.x), 0.5 * (P0.y + P1.y), a.t, 0, 0, ed2);
        const double c = area / 6.0;
        b0 = c * (f1 + f2);
        b1 = c * (f0 + f2);
        b2 = c * (f0 + f1);
    }
    // Neumann load: |E| g(m_E) / 2 on the two vertices of each Neumann
    // edge, for the (boundary) elements flagged in the mask
    if ((a.neu_mask[m >> 6] >> (m & 63)) & 1) {
        const int code = a.ecode[m];
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            if (PHF_CODE_TYPE(code, i) != 2) continue;
            const double2 Pa = i == 0 ? P1 : (i == 1 ? P2 : P0);
            const double2 Pb = i == 0 ? P2 : (i == 1 ? P0 : P1);
            const double dx = Pb.x - Pa.x, dy = Pb.y - Pa.y;
            const double len = sqrt(dx * dx + dy * dy);
            const int32_t eid =
                a.g.kind == PHF_FN_EDGE_ARRAY ? a.elem_edges[3 * (int64_t)m + i] : -1;
            // outward normal of the counter-clockwise edge Pa -> Pb
            const double gv = fn_at<OOL>(a.g, 0.5 * (Pa.x + Pb.x), 0.5 * (Pa.y + Pb.y), a.t,
                                         dy / len, -dx / len, eid);
            const double w = len * gv * 0.5;
            if (i == 0) { b1 += w; b2 += w; }
            if (i == 1) { b2 += w; b0 += w; }
            if (i == 2) { b0 += w; b1 += w; }
        }
    }
    shF[3 * slot] = b0;
    shF[3 * slot + 1] = b1;
    shF[3 * slot + 2] = b2;
}

typedef double phf_v2d __attribute__((ext_vector_type(2)));

// Output stores. NT: non-temporal (streamed to memory without displacing
// cached lines): the outputs are written once and not read again by the
// kernel, so that back-to-back assemblies of one mesh keep its inputs (the
// coarse coordinates, a_T, row records, about 40 bytes per element) in the
// last-level cache instead of the previous launch's outputs.
template <bool NT>
__device__ inline void put2(phf_v2d* p, double x, double y)
{
    phf_v2d w;
    w.x = x;
    w.y = y;
    if (NT) __builtin_nontemporal_store(w, p);
    else *p = w;
}

template <bool NT>
__device__ inline void put1(double* p, double x)
{
    if (NT) __builtin_nontemporal_store(x, p);
    else *p = x;
}

// Streams cnt values v(0..cnt-1) to dst with 16-byte stores where dst allows
// (dst is 8-byte aligned; a leading odd word is stored alone).
template <int TN, bool NT, typename F>
__device__ inline void store_run(double* dst, int32_t cnt, F v)
{
    const int tid = threadIdx.x;
    const int32_t head = (((uintptr_t)dst & 15) != 0 && cnt > 0) ? 1 : 0;
    if (head && tid == 0) put1<NT>(dst, v(0));
    const int32_t pairs = (cnt - head) >> 1;
    phf_v2d* d2 = reinterpret_cast<phf_v2d*>(dst + head);
    for (int32_t q = tid; q < pairs; q += TN) put2<NT>(d2 + q, v(head + 2 * q), v(head + 2 * q + 1));
    if (((cnt - head) & 1) && tid == 0) put1<NT>(dst + cnt - 1, v(cnt - 1));
}

// Stores elements m0 .. m0+cnt-1 from LDS slots 0 .. cnt-1: K, M, (D) as 9
// contiguous values per element, F as 3.
template <int TN, bool NT, bool MATS, bool WITH_D>
__device__ inline void store_elements(const AsmArgs& a, int32_t m0, int32_t cnt, const double* shK,
                                      const double* shD, const double* shA, const double* shF)
{
    if (MATS) {
        store_run<TN, NT>(a.K + 9 * (int64_t)m0, 9 * cnt, [&](int32_t v) { return shK[v]; });
        store_run<TN, NT>(a.M + 9 * (int64_t)m0, 9 * cnt, [&](int32_t v) {
            const int32_t el = v / 9, r = v - 9 * el;
            return shA[el] * ((r & 3) == 0 ? 2.0 : 1.0);
        });
        if (WITH_D)
            store_run<TN, NT>(a.D + 9 * (int64_t)m0, 9 * cnt, [&](int32_t v) { return shD[v]; });
    }
    store_run<TN, NT>(a.F + 3 * (int64_t)m0, 3 * cnt, [&](int32_t v) { return shF[v]; });
}

// An element tile: TN consecutive elements, vertices from the element-major
// coordinate copy (GATHER: through the vertex ids from the node array, 16
// bytes per element plus cached gathers, which pays on meshes numbered so
// that neighbouring elements share nodes, e.g. structured ones; the values
// are the same).
template <int TN, bool NT, bool HAS_AT, bool MATS, bool WITH_D, bool GEN_A, bool GATHER = false,
          bool OOL = false>
__device__ inline void element_tile(const AsmArgs& a, int32_t tile, double* shK, double* shD,
                                    double* shA, double* shF)
{
    const int tid = threadIdx.x;
    const int32_t m0 = tile * TN;
    const int32_t nt = min(TN, a.nE - m0);
    if (tid < nt) {
        const int32_t m = m0 + tid;
        double2 P0, P1, P2;
        if (GATHER) {
            const int4 v = a.elem4[m];
            P0 = a.xy[v.x];
            P1 = a.xy[v.y];
            P2 = a.xy[v.z];
        } else {
            P0 = a.exy[3 * (int64_t)m];
            P1 = a.exy[3 * (int64_t)m + 1];
            P2 = a.exy[3 * (int64_t)m + 2];
        }
        element_values<HAS_AT, MATS, WITH_D, GEN_A, OOL>(a, m, P0, P1, P2, tid, shK, shD, shA,
                                                         shF);
    }
    __syncthreads();
    store_elements<TN, NT, MATS, WITH_D>(a, m0, nt, shK, shD, shA, shF);
}

// An element tile of a red-refined mesh: TN consecutive elements whose
// vertices follow from their parent's (the coarse mesh's element-major
// coordinates) exactly as the refinement forms them: Q_i = 0.5 (P_{i+1} +
// P_{i+2}); element p < nEp is the interior child [Q0 Q1 Q2] of parent p and
// element nEp + 3p + i the corner child [P_i Q_{i+2} Q_{i+1}] of its vertex
// i. An interior child reads its parent's 48 bytes, the three corner
// children of a parent (neighbouring lanes) share one read: 24 bytes per
// element on average instead of the 48 of the element's own record. Each
// tile still writes one contiguous run of every output (a tile covering
// interior and corner children of different parents would split its writes
// between two distant runs, which measured slower).
template <int TN, bool NT, bool HAS_AT, bool MATS, bool WITH_D, bool GEN_A>
__device__ inline void child_tile(const AsmArgs& a, int32_t tile, double* shK, double* shD,
                                  double* shA, double* shF)
{
    const int tid = threadIdx.x;
    const int32_t m0 = tile * TN;
    const int32_t nt = min(TN, a.nE - m0);
    if (tid < nt) {
        const int32_t m = m0 + tid;
        const bool interior = m < a.nEp;
        const int32_t j = m - a.nEp;
        const int32_t p = interior ? m : j / 3;
        const int c = interior ? 3 : j - 3 * p;  // corner vertex, or 3 for the interior child
        const double2 P0 = a.pexy[3 * (int64_t)p], P1 = a.pexy[3 * (int64_t)p + 1];
        const double2 P2 = a.pexy[3 * (int64_t)p + 2];
        const double2 Q0 = make_double2(0.5 * (P1.x + P2.x), 0.5 * (P1.y + P2.y));
        const double2 Q1 = make_double2(0.5 * (P2.x + P0.x), 0.5 * (P2.y + P0.y));
        const double2 Q2 = make_double2(0.5 * (P0.x + P1.x), 0.5 * (P0.y + P1.y));
        double2 V0, V1, V2;
        if (c == 3) { V0 = Q0; V1 = Q1; V2 = Q2; }
        else if (c == 0) { V0 = P0; V1 = Q2; V2 = Q1; }
        else if (c == 1) { V0 = P1; V1 = Q0; V2 = Q2; }
        else { V0 = P2; V1 = Q1; V2 = Q0; }
        element_values<HAS_AT, MATS, WITH_D, GEN_A>(a, m, V0, V1, V2, tid, shK, shD, shA, shF);
    }
    __syncthreads();
    store_elements<TN, NT, MATS, WITH_D>(a, m0, nt, shK, shD, shA, shF);
}

// A row tile: TN consecutive multiplier rows. Their C values are one
// contiguous run starting at the tile's base pointer; each row's offset in it
// is an exclusive scan of the row lengths (4 interior, 2 Dirichlet). The rows
// put their values into LDS at those offsets and the tile streams the run out
// with 16-byte stores, so that every store instruction covers whole lines
// (rows writing their own 16 or 32 bytes leave lines split between two
// instructions, which non-temporal stores send to memory as two partial
// writes). A row reads its edge's half-length |E|/2 from the mesh's row
// records (negated on Dirichlet rows); only a Dirichlet row with data reads
// its end nodes, for the midpoint of u_D. shC: 4 TN doubles.
template <int TN, bool NT, bool MATS, bool OOL = false>
__device__ inline void row_tile(const AsmArgs& a, int32_t tile, int32_t* shs, double* shC)
{
    const int32_t r = tile * TN + threadIdx.x;
    const bool live = r < a.L;
    const double hs = live ? a.row_hs[r] : 0.0;
    const int32_t len = live ? (hs < 0.0 ? 2 : 4) : 0;
    int32_t tot;
    const int32_t off = phf_block_exscan_i32<TN>(len, shs, &tot);
    const bool dirichlet = hs < 0.0;
    const double h = fabs(hs);
    if (MATS) {
        if (live) {
            shC[off] = h;
            shC[off + 1] = h;
            if (!dirichlet) {
                shC[off + 2] = -h;
                shC[off + 3] = -h;
            }
        }
        __syncthreads();
        const int32_t c0 = TN == 256 ? a.C_tile[tile] : a.C_rowptr[tile * TN];
        store_run<TN, NT>(a.C + c0, tot, [&](int32_t v) { return shC[v]; });
    }
    if (!live) return;
    double v = 0.0;
    if (dirichlet && a.uD.kind != PHF_FN_ZERO) {
        const int2 kl = a.row_nodes[r];
        const double2 Pk = a.xy[~kl.x], Pl = a.xy[kl.y];
        const int32_t eid = a.uD.kind == PHF_FN_EDGE_ARRAY ? a.row_edge[r] : -1;
        v = -(2.0 * h) * fn_at<OOL>(a.uD, 0.5 * (Pk.x + Pl.x), 0.5 * (Pk.y + Pl.y), a.t, 0, 0, eid);
    }
    put1<NT>(a.bD + r, v);
}

template <bool PARENT, bool HAS_AT, bool MATS, bool WITH_D, bool GEN_A>
__global__ __launch_bounds__(TILE) void k_assemble(AsmArgs a)
{
    if (a.t_step) a.t = a.t0 + (double)(*a.t_step) * a.dt;
    __shared__ __align__(16) double shK[MATS ? TILE * 9 : 2];
    __shared__ __align__(16) double shD[WITH_D ? TILE * 9 : 2];
    __shared__ double shA[MATS ? TILE : 1];
    __shared__ __align__(16) double shF[TILE * 3];
    __shared__ int32_t shs[TILE / 64 + 1];
    bool is_elem;
    int32_t tile;
    fused_tile(blockIdx.x, a.nbE, a.nbR, &is_elem, &tile);
    if (is_elem) {
        if (PARENT)
            child_tile<TILE, true, HAS_AT, MATS, WITH_D, GEN_A>(a, tile, shK, shD, shA, shF);
        else
            element_tile<TILE, true, HAS_AT, MATS, WITH_D, GEN_A>(a, tile, shK, shD, shA, shF);
    } else {
        row_tile<TILE, true, MATS>(a, tile, shs, shK);
    }
}

// An element tile without the cooperative store: each thread computes its
// triangle (into its own LDS slot) and stores its own 9 + 9 (+ 9) + 3 values
// with 8-byte stores (no barrier; a launch-shape variant of the tuner).
template <int TN, bool NT, bool HAS_AT, bool WITH_D, bool GEN_A>
__device__ inline void element_direct(const AsmArgs& a, int32_t tile, double* shK, double* shD,
                                      double* shA, double* shF)
{
    const int tid = threadIdx.x;
    const int32_t m = tile * TN + tid;
    if (m >= a.nE) return;
    const double2 P0 = a.exy[3 * (int64_t)m], P1 = a.exy[3 * (int64_t)m + 1];
    const double2 P2 = a.exy[3 * (int64_t)m + 2];
    element_values<HAS_AT, true, WITH_D, GEN_A, true>(a, m, P0, P1, P2, tid, shK, shD, shA, shF);
    const double* k = shK + 9 * tid;
    for (int q = 0; q < 9; ++q) {
        put1<NT>(a.K + 9 * (int64_t)m + q, k[q]);
        put1<NT>(a.M + 9 * (int64_t)m + q, shA[tid] * ((q & 3) == 0 ? 2.0 : 1.0));
        if (WITH_D) put1<NT>(a.D + 9 * (int64_t)m + q, shD[9 * tid + q]);
    }
    for (int q = 0; q < 3; ++q) put1<NT>(a.F + 3 * (int64_t)m + q, shF[3 * tid + q]);
}

// An element tile with four lanes per triangle: lane i < 3 computes row i of
// K, M (and D) and F_i, lane 3 idles, and the lanes of a triangle exchange
// their midpoint values of f and Neumann terms through cross-lane moves; the
// rows go out with 8-byte stores, consecutive lanes writing consecutive 24
// bytes (no LDS, no barrier). The arithmetic and its order are those of
// element_values, so the outputs are bit-identical to the other tiles.
template <int TN, bool NT, bool HAS_AT, bool WITH_D, bool GEN_A>
__device__ inline void element_quad(const AsmArgs& a, int32_t tile)
{
#pragma clang fp contract(off)
    const int tid = threadIdx.x;
    const int i = tid & 3;
    const int base = (tid & 63) & ~3;  // the triangle's first lane in the wavefront
    const int32_t m = tile * (TN / 4) + (tid >> 2);
    const bool act = m < a.nE;
    double2 P0 = make_double2(0.0, 0.0), P1 = make_double2(1.0, 0.0), P2 = make_double2(0.0, 1.0);
    if (act) {
        P0 = a.exy[3 * (int64_t)m];
        P1 = a.exy[3 * (int64_t)m + 1];
        P2 = a.exy[3 * (int64_t)m + 2];
    }
    const double g0x = P1.y - P2.y, g0y = P2.x - P1.x;
    const double g1x = P2.y - P0.y, g1y = P0.x - P2.x;
    const double g2x = P0.y - P1.y, g2y = P1.x - P0.x;
    const double det = (P1.x - P0.x) * (P2.y - P0.y) - (P2.x - P0.x) * (P1.y - P0.y);
    const double area = 0.5 * det;
    const bool row = act && i < 3;
    // this lane's edge (opposite vertex i): midpoint value of f, Neumann term
    const double2 Pa = i == 0 ? P1 : (i == 1 ? P2 : P0);
    const double2 Pb = i == 0 ? P2 : (i == 1 ? P0 : P1);
    double fv = 0.0, wv = 0.0;
    int nv = 0;
    if (row && a.f.kind != PHF_FN_ZERO) {
        const int32_t ed = a.f.kind == PHF_FN_EDGE_ARRAY ? a.elem_edges[3 * (int64_t)m + i] : -1;
        fv = fn_at<true>(a.f, 0.5 * (Pa.x + Pb.x), 0.5 * (Pa.y + Pb.y), a.t, 0, 0, ed);
    }
    if (row && ((a.neu_mask[m >> 6] >> (m & 63)) & 1)) {
        const int code = a.ecode[m];
        if (PHF_CODE_TYPE(code, i) == 2) {
            const double dx = Pb.x - Pa.x, dy = Pb.y - Pa.y;
            const double len = sqrt(dx * dx + dy * dy);
            const int32_t eid =
                a.g.kind == PHF_FN_EDGE_ARRAY ? a.elem_edges[3 * (int64_t)m + i] : -1;
            const double gv = fn_at<true>(a.g, 0.5 * (Pa.x + Pb.x), 0.5 * (Pa.y + Pb.y), a.t,
                                          dy / len, -dx / len, eid);
            wv = len * gv * 0.5;
            nv = 1;
        }
    }
    const double f0 = __shfl(fv, base), f1 = __shfl(fv, base + 1), f2 = __shfl(fv, base + 2);
    const double w0 = __shfl(wv, base), w1 = __shfl(wv, base + 1), w2 = __shfl(wv, base + 2);
    const int n0 = __shfl(nv, base), n1 = __shfl(nv, base + 1), n2 = __shfl(nv, base + 2);
    if (!row) return;
    double b = 0.0;
    if (a.f.kind != PHF_FN_ZERO) {
        const double c = area / 6.0;
        b = i == 0 ? c * (f1 + f2) : (i == 1 ? c * (f0 + f2) : c * (f0 + f1));
    }
    // the Neumann terms in the order of element_values' edge loop
    if (i == 0) { if (n1) b += w1; if (n2) b += w2; }
    if (i == 1) { if (n0) b += w0; if (n2) b += w2; }
    if (i == 2) { if (n0) b += w0; if (n1) b += w1; }
    put1<NT>(a.F + 3 * (int64_t)m + i, b);
    const double gix = i == 0 ? g0x : (i == 1 ? g1x : g2x);
    const double giy = i == 0 ? g0y : (i == 1 ? g1y : g2y);
    const double aT = HAS_AT ? a.aT[m] : 1.0;
    const double s = aT / (2.0 * det);
    double k0, k1, k2;
    if (GEN_A) {
        const double aix = a.A00 * gix + a.A01 * giy, aiy = a.A10 * gix + a.A11 * giy;
        k0 = s * (aix * g0x + aiy * g0y);
        k1 = s * (aix * g1x + aiy * g1y);
        k2 = s * (aix * g2x + aiy * g2y);
    } else {
        // the symmetric entries as element_values forms them (lower index first)
        k0 = s * (g0x * gix + g0y * giy);
        k1 = i == 0 ? s * (g0x * g1x + g0y * g1y) : s * (g1x * gix + g1y * giy);
        k2 = i == 2 ? s * (g2x * g2x + g2y * g2y) : s * (gix * g2x + giy * g2y);
    }
    const int64_t o = 9 * (int64_t)m + 3 * i;
    put1<NT>(a.K + o, k0);
    put1<NT>(a.K + o + 1, k1);
    put1<NT>(a.K + o + 2, k2);
    const double a12 = area / 12.0;
    put1<NT>(a.M + o, a12 * (i == 0 ? 2.0 : 1.0));
    put1<NT>(a.M + o + 1, a12 * (i == 1 ? 2.0 : 1.0));
    put1<NT>(a.M + o + 2, a12 * (i == 2 ? 2.0 : 1.0));
    if (WITH_D) {
        put1<NT>(a.D + o, (a.p0 * g0x + a.p1 * g0y) / 6.0);
        put1<NT>(a.D + o + 1, (a.p0 * g1x + a.p1 * g1y) / 6.0);
        put1<NT>(a.D + o + 2, (a.p0 * g2x + a.p1 * g2y) / 6.0);
    }
}

// ---- batched assembly -------------------------------------------------------
// A pointer field of a record in device memory, read as a global-memory
// pointer. The compiler cannot tell where a pointer loaded from memory
// points and would address through it with flat instructions (which also
// count against the LDS wait counter); read this way the tile code keeps
// global loads and stores, as with the single-mesh kernel's by-value
// argument (measured: 6-8% of the batched launch).
template <class T>
__device__ inline T* as_global(T* const& field)
{
    typedef __attribute__((address_space(1))) T* GT;
    return (T*)*static_cast<const GT*>(static_cast<const void*>(&field));
}

__device__ inline AsmArgs global_record(const AsmArgs& g)
{
    AsmArgs a = g;
    a.exy = as_global(g.exy);
    a.pexy = as_global(g.pexy);
    a.elem4 = as_global(g.elem4);
    a.ecode = as_global(g.ecode);
    a.xy = as_global(g.xy);
    a.aT = as_global(g.aT);
    a.elem_edges = as_global(g.elem_edges);
    a.row_hs = as_global(g.row_hs);
    a.row_nodes = as_global(g.row_nodes);
    a.row_edge = as_global(g.row_edge);
    a.C_tile = as_global(g.C_tile);
    a.C_rowptr = as_global(g.C_rowptr);
    a.neu_mask = as_global(g.neu_mask);
    a.t_step = as_global(g.t_step);
    a.K = as_global(g.K);
    a.M = as_global(g.M);
    a.D = as_global(g.D);
    a.C = as_global(g.C);
    a.F = as_global(g.F);
    a.bD = as_global(g.bD);
    a.f.ev = as_global(g.f.ev);
    a.g.ev = as_global(g.g.ev);
    a.uD.ev = as_global(g.uD.ev);
    return a;
}

// One launch over a work list of (instance, tile) items of many meshes:
// item.y >= 0 is element tile item.y of instance item.x, item.y < 0 row tile
// ~item.y. PERSIST = false: one workgroup per item; PERSIST = true: each
// workgroup takes items blockIdx.x, blockIdx.x + gridDim.x, ... (the loop
// costs about 25 more VGPRs, one wave per SIMD of occupancy). MODE: the
// element tile's form, 0 staged through LDS (TN triangles), 1 per-thread
// stores (TN triangles), 2 four lanes per triangle (TN / 4 triangles), 3
// staged with coordinates gathered through the vertex ids. The
// instance record is read with scalar loads (the work item and the record
// are uniform over the workgroup). The tile code is the single-mesh kernel's
// (element tiles read each mesh's own element records; f, g and u_D are
// evaluated out of line), so the outputs are bit-identical to it.
template <int TN, int MODE, bool PERSIST, bool HAS_AT, bool WITH_D, bool GEN_A>
__global__ __launch_bounds__(TN) void k_assemble_batch(const AsmArgs* __restrict__ args,
                                                       const int2* __restrict__ work,
                                                       int32_t nwork)
{
    constexpr bool LDS = MODE != 2;
    __shared__ __align__(16) double shK[LDS ? TN * 9 : TN * 4];  // row tiles stage C here
    __shared__ __align__(16) double shD[LDS && WITH_D ? TN * 9 : 2];
    __shared__ double shA[LDS ? TN : 1];
    __shared__ __align__(16) double shF[LDS ? TN * 3 : 2];
    __shared__ int32_t shs[TN / 64 + 1];
    for (int32_t w = blockIdx.x; w < nwork; w += gridDim.x) {
        const int2 item = work[w];
        const AsmArgs a = global_record(args[item.x]);
        if (item.y < 0)
            row_tile<TN, true, true, true>(a, ~item.y, shs, shK);
        else if (MODE == 0)
            element_tile<TN, true, HAS_AT, true, WITH_D, GEN_A, false, true>(a, item.y, shK, shD,
                                                                            shA, shF);
        else if (MODE == 3)
            element_tile<TN, true, HAS_AT, true, WITH_D, GEN_A, true, true>(a, item.y, shK, shD,
                                                                           shA, shF);
        else if (MODE == 1)
            element_direct<TN, true, HAS_AT, WITH_D, GEN_A>(a, item.y, shK, shD, shA, shF);
        else
            element_quad<TN, true, HAS_AT, WITH_D, GEN_A>(a, item.y);
        if (!PERSIST) break;
        __syncthreads();  // the next item reuses the shared arrays
    }
}

// ---- saddle-matrix values -------------------------------------------------
struct SaddleArgs {
    int32_t nE, L, nbE, nbR;
    const double2* exy;
    const int32_t* ecode;
    const double2* xy;
    const double* aT;
    const int32_t* S_rowptr;
    const double* row_hs;
    double A00, A01, A10, A11, p0, p1, delta;
    double* S;
};

__global__ __launch_bounds__(TILE) void k_saddle_values(SaddleArgs a)
{
    bool is_elem;
    int32_t tile;
    fused_tile(blockIdx.x, a.nbE, a.nbR, &is_elem, &tile);
    const int32_t N = 3 * a.nE;
    if (is_elem) {
        const int32_t m = tile * TILE + threadIdx.x;
        if (m >= a.nE) return;
        const double2 P[3] = {a.exy[3 * (int64_t)m], a.exy[3 * (int64_t)m + 1],
                              a.exy[3 * (int64_t)m + 2]};
        double gx[3], gy[3];
        for (int i = 0; i < 3; ++i) {
            const double2 Pa = P[(i + 1) % 3], Pb = P[(i + 2) % 3];
            gx[i] = Pa.y - Pb.y;
            gy[i] = Pb.x - Pa.x;
        }
        const double det = (P[1].x - P[0].x) * (P[2].y - P[0].y) - (P[2].x - P[0].x) * (P[1].y - P[0].y);
        const double area = 0.5 * det;
        const double aT = a.aT ? a.aT[m] : 1.0;
        const double s = aT / (2.0 * det);
        double len[3];
        for (int i = 0; i < 3; ++i)  // as the row records round them: S = -C exactly
            len[i] = 2.0 * phf_half_length(P[(i + 1) % 3], P[(i + 2) % 3]);
        const int code = a.ecode[m];
        for (int j = 0; j < 3; ++j) {
            int32_t q = a.S_rowptr[3 * (int64_t)m + j];
            const double ajx = a.A00 * gx[j] + a.A01 * gy[j], ajy = a.A10 * gx[j] + a.A11 * gy[j];
            for (int i = 0; i < 3; ++i) {
                double v = s * (ajx * gx[i] + ajy * gy[i]);
                v += (a.p0 * gx[i] + a.p1 * gy[i]) / 6.0;
                v += a.delta * (area / 12.0) * (i == j ? 2.0 : 1.0);
                a.S[q + i] = v;
            }
            q += 3;
            int l1 = j == 0 ? 1 : 0, l2 = j == 2 ? 1 : 2;
            if (PHF_CODE_SWAP(code, j)) {
                int t = l1;
                l1 = l2;
                l2 = t;
            }
            if (PHF_CODE_TYPE(code, l1) != 2)
                a.S[q++] = -(PHF_CODE_TPLUS(code, l1) ? 0.5 : -0.5) * len[l1];
            if (PHF_CODE_TYPE(code, l2) != 2)
                a.S[q++] = -(PHF_CODE_TPLUS(code, l2) ? 0.5 : -0.5) * len[l2];
        }
    } else {
        const int32_t r = tile * TILE + threadIdx.x;
        if (r >= a.L) return;
        const double hs = a.row_hs[r];
        const double h = fabs(hs);
        const int32_t q = a.S_rowptr[N + r];
        a.S[q] = -h;
        a.S[q + 1] = -h;
        if (hs > 0.0) {  // interior row: the T- half too
            a.S[q + 2] = h;
            a.S[q + 3] = h;
        }
    }
}

template <bool HAS_AT, bool MATS, bool WITH_D, bool GEN_A>
int launch_assemble(phf_ctx* ctx, const AsmArgs& a)
{
    if (a.pexy)
        PHF_LAUNCH(ctx, "k_assemble", (k_assemble<true, HAS_AT, MATS, WITH_D, GEN_A>),
                   a.nbE + a.nbR, TILE, 0, a);
    else
        PHF_LAUNCH(ctx, "k_assemble", (k_assemble<false, HAS_AT, MATS, WITH_D, GEN_A>),
                   a.nbE + a.nbR, TILE, 0, a);
    return PHF_OK;
}

bool aligned16(const void* p) { return ((uintptr_t)p & 15) == 0; }

#define TRY(x)               \
    do {                     \
        int rc_ = (x);       \
        if (rc_) return rc_; \
    } while (0)

}  // namespace

namespace {
// Checks the arguments of one assembly and fills its kernel record.
int make_args(phf_mesh* mesh, const phf_coeffs* co, const phf_data* data, const phf_system* out,
              const char* fn, AsmArgs* pa)
{
    phf_ctx* ctx = mesh->ctx;
    if (!co || !data || !out) return phf_set_error(ctx, PHF_EINVAL, "%s: null argument", fn);
    if (!phf_fn_valid(data->f) || !phf_fn_valid(data->g) || !phf_fn_valid(data->uD))
        return phf_set_error(ctx, PHF_EINVAL, "%s: unknown function kind or missing edge array", fn);
    const bool mats = out->K || out->M || out->C;
    if (mats && !(out->K && out->M && out->C))
        return phf_set_error(ctx, PHF_EINVAL, "%s: K, M and C are written together", fn);
    if (!out->F || !out->bD)
        return phf_set_error(ctx, PHF_EINVAL, "%s: F and bD are required", fn);
    const void* ptrs[] = {out->K, out->M, out->D, out->C, out->F, out->bD};
    for (const void* p : ptrs)
        if (p && !aligned16(p))
            return phf_set_error(ctx, PHF_EINVAL, "%s: output buffers must be 16-byte aligned", fn);
    if (out->D && !mats) return phf_set_error(ctx, PHF_EINVAL, "%s: D needs K, M and C", fn);
    AsmArgs& a = *pa;
    a.nE = mesh->nE;
    a.L = mesh->L;
    a.nbE = (mesh->nE + TILE - 1) / TILE;
    a.nbR = (mesh->L + TILE - 1) / TILE;
    a.nEp = 0;
    a.pad_ = 0;
    a.exy = mesh->exy;
    a.pexy = nullptr;
    a.elem4 = mesh->elem4;
    a.ecode = mesh->ecode;
    a.xy = mesh->xy;
    a.aT = co->a_T;
    a.elem_edges = mesh->elem_edges;
    a.row_hs = mesh->row_hs;
    a.row_nodes = mesh->row_nodes;
    a.row_edge = mesh->row_edge;
    a.C_tile = mesh->C_tile;
    a.C_rowptr = mesh->C_rowptr;
    a.neu_mask = mesh->neu_mask;
    a.A00 = co->A[0];
    a.A01 = co->A[1];
    a.A10 = co->A[2];
    a.A11 = co->A[3];
    a.p0 = co->p[0];
    a.p1 = co->p[1];
    a.f = phf_fn_to_dev(data->f);
    a.g = phf_fn_to_dev(data->g);
    a.uD = phf_fn_to_dev(data->uD);
    a.t = data->t;
    a.t_step = nullptr;
    a.t0 = 0.0;
    a.dt = 0.0;
    a.K = out->K;
    a.M = out->M;
    a.D = out->D;
    a.C = out->C;
    a.F = out->F;
    a.bD = out->bD;
    return PHF_OK;
}

bool general_A(const phf_coeffs* co)
{
    return !(co->A[0] == 1.0 && co->A[1] == 0.0 && co->A[2] == 0.0 && co->A[3] == 1.0);
}
}  // namespace

int phf_assemble_impl(phf_mesh* mesh, const phf_coeffs* co, const phf_data* data,
                      const phf_system* out, const int64_t* t_step, double t0, double dt)
{
    phf_ctx* ctx = mesh->ctx;
    AsmArgs a;
    TRY(make_args(mesh, co, data, out, "phf_assemble", &a));
    if (mesh->parent && mesh->parent->exy && mesh->nE == 4 * mesh->parent->nE) {
        // red-refined: element tiles read the coarse mesh's coordinates
        a.pexy = mesh->parent->exy;
        a.nEp = mesh->parent->nE;
    }
    a.t_step = t_step;
    a.t0 = t0;
    a.dt = dt;
    const bool mats = out->K != nullptr;
    const bool genA = general_A(co);
    const bool hasAT = co->a_T != nullptr;
    const bool withD = out->D != nullptr;
    int rc;
    if (!mats) rc = launch_assemble<false, false, false, false>(ctx, a);
    else if (withD || genA) {
        if (hasAT) rc = withD ? launch_assemble<true, true, true, true>(ctx, a)
                              : launch_assemble<true, true, false, true>(ctx, a);
        else rc = withD ? launch_assemble<false, true, true, true>(ctx, a)
                        : launch_assemble<false, true, false, true>(ctx, a);
    } else {
        rc = hasAT ? launch_assemble<true, true, false, false>(ctx, a)
                   : launch_assemble<false, true, false, false>(ctx, a);
    }
    if (rc) return rc;
    if (out->S) {
        SaddleArgs s;
        s.nE = mesh->nE;
        s.L = mesh->L;
        s.nbE = a.nbE;
        s.nbR = a.nbR;
        s.exy = mesh->exy;
        s.ecode = mesh->ecode;
        s.xy = mesh->xy;
        s.aT = co->a_T;
        s.S_rowptr = mesh->S_rowptr;
        s.row_hs = mesh->row_hs;
        s.A00 = co->A[0];
        s.A01 = co->A[1];
        s.A10 = co->A[2];
        s.A11 = co->A[3];
        s.p0 = co->p[0];
        s.p1 = co->p[1];
        s.delta = co->delta;
        s.S = out->S;
        PHF_LAUNCH(ctx, "k_saddle_values", k_saddle_values, s.nbE + s.nbR, TILE, 0, s);
    }
    return PHF_OK;
}

extern "C" int phf_assemble(phf_mesh* mesh, const phf_coeffs* coeffs, const phf_data* data,
                            const phf_system* out)
{
    if (!mesh) return PHF_EINVAL;
    return phf_assemble_impl(mesh, coeffs, data, out);
}

// ---------------------------------------------------------------------------
// batched assembly
// ---------------------------------------------------------------------------

struct phf_batch {
    phf_ctx* ctx = nullptr;
    std::vector<phf_mesh*> meshes;
    AsmArgs* h_args = nullptr;  // pinned staging of the per-instance records
    AsmArgs* d_args = nullptr;
    hipEvent_t args_ev = nullptr;  // the last upload of h_args
    bool args_pending = false;
    std::vector<AsmArgs> last;     // records of the last upload (skipped when unchanged)
    // work lists for tiles of 64, 128, 256 threads with as many triangles
    // ([0..2]) or a quarter as many ([3..5], four lanes per triangle)
    int2* d_work[6] = {};
    int32_t nwork[6] = {};
    int32_t tile = 256, blocks_per_cu = 0, ncu = 256, lanes = 1, direct = 0, gather = 0;
    bool counted = false;  // registered with the meshes and context
};

namespace {
int tile_index(int32_t tile) { return tile == 64 ? 0 : (tile == 128 ? 1 : (tile == 256 ? 2 : -1)); }

// Work list for one tile size: per instance its element and row tiles,
// interleaved in proportion as in the single-mesh launch. wi = ti: element
// tiles of 64 << ti triangles; wi = 3 + ti: a quarter of that.
int batch_work(phf_batch* b, int wi)
{
    if (b->d_work[wi]) return PHF_OK;
    const int32_t tn = 64 << (wi % 3), te = wi >= 3 ? tn / 4 : tn;
    std::vector<int2> w;
    for (size_t i = 0; i < b->meshes.size(); ++i) {
        const phf_mesh* m = b->meshes[i];
        const int64_t ne = (m->nE + te - 1) / te, nr = (m->L + tn - 1) / tn, T = ne + nr;
        for (int64_t q = 0; q < T; ++q) {
            const int64_t e0 = q * ne / T, e1 = (q + 1) * ne / T;
            w.push_back(make_int2((int32_t)i, e1 > e0 ? (int32_t)e0 : ~(int32_t)(q - e0)));
        }
    }
    phf_ctx* ctx = b->ctx;
    TRY(phf_dmalloc(ctx, &b->d_work[wi], std::max<size_t>(w.size(), 1), "batch work list"));
    PHF_HIP(ctx, hipMemcpyAsync(b->d_work[wi], w.data(), sizeof(int2) * w.size(),
                                hipMemcpyHostToDevice, ctx->stream));
    PHF_HIP(ctx, hipStreamSynchronize(ctx->stream));  // w is released on return
    b->nwork[wi] = (int32_t)w.size();
    return PHF_OK;
}

template <int TN, int MODE, bool HAS_AT, bool WITH_D, bool GEN_A>
int launch_batch_t(phf_batch* b, int wi)
{
    phf_ctx* ctx = b->ctx;
    const int32_t nw = b->nwork[wi];
    if (nw == 0) return PHF_OK;
    if constexpr (MODE == 0) {  // persistent grids only for the staged tile
        if (b->blocks_per_cu > 0) {
            const int64_t grid = std::min<int64_t>(nw, (int64_t)b->blocks_per_cu * b->ncu);
            PHF_LAUNCH(ctx, "k_assemble_batch",
                       (k_assemble_batch<TN, MODE, true, HAS_AT, WITH_D, GEN_A>), (unsigned)grid,
                       TN, 0, b->d_args, b->d_work[wi], nw);
            return PHF_OK;
        }
    }
    PHF_LAUNCH(ctx, "k_assemble_batch",
               (k_assemble_batch<TN, MODE, false, HAS_AT, WITH_D, GEN_A>), (unsigned)nw, TN, 0,
               b->d_args, b->d_work[wi], nw);
    return PHF_OK;
}

template <int TN, int MODE>
int launch_batch_mode(phf_batch* b, int wi, bool hasAT, bool withD, bool genA)
{
    if (hasAT) {
        if (withD) return genA ? launch_batch_t<TN, MODE, true, true, true>(b, wi)
                               : launch_batch_t<TN, MODE, true, true, false>(b, wi);
        return genA ? launch_batch_t<TN, MODE, true, false, true>(b, wi)
                    : launch_batch_t<TN, MODE, true, false, false>(b, wi);
    }
    if (withD) return genA ? launch_batch_t<TN, MODE, false, true, true>(b, wi)
                           : launch_batch_t<TN, MODE, false, true, false>(b, wi);
    return genA ? launch_batch_t<TN, MODE, false, false, true>(b, wi)
                : launch_batch_t<TN, MODE, false, false, false>(b, wi);
}

template <int TN>
int launch_batch_tn(phf_batch* b, int wi, int mode, bool hasAT, bool withD, bool genA)
{
    if (mode == 3) return launch_batch_mode<TN, 3>(b, wi, hasAT, withD, genA);
    if (mode == 2) return launch_batch_mode<TN, 2>(b, wi, hasAT, withD, genA);
    if (mode == 1) return launch_batch_mode<TN, 1>(b, wi, hasAT, withD, genA);
    return launch_batch_mode<TN, 0>(b, wi, hasAT, withD, genA);
}

// Validates and uploads the per-instance records; returns the variant flags.
int batch_prepare(phf_batch* b, const phf_coeffs* co, const phf_data* data, const phf_system* out,
                  bool* hasAT, bool* withD, bool* genA)
{
    phf_ctx* ctx = b->ctx;
    if (!co || !data || !out) return phf_set_error(ctx, PHF_EINVAL, "phf_batch_assemble: null argument");
    const size_t n = b->meshes.size();
    *hasAT = n > 0 && co[0].a_T != nullptr;
    *withD = n > 0 && out[0].D != nullptr;
    *genA = false;
    std::vector<AsmArgs> rec(n);
    for (size_t i = 0; i < n; ++i) {
        TRY(make_args(b->meshes[i], &co[i], &data[i], &out[i], "phf_batch_assemble", &rec[i]));
        if (!out[i].K)
            return phf_set_error(ctx, PHF_EINVAL, "phf_batch_assemble: instance %zu: K, M, C required", i);
        if ((co[i].a_T != nullptr) != *hasAT || (out[i].D != nullptr) != *withD)
            return phf_set_error(ctx, PHF_EINVAL,
                                 "phf_batch_assemble: a_T and D must be given for all instances or none");
        *genA = *genA || general_A(&co[i]);
    }
    // the variant choice of phf_assemble (D implies the general-A form), so
    // that the outputs are bit-identical to it
    *genA = *genA || *withD;
    // the records go up only when they differ from the last upload (repeated
    // assemblies of one batch with the same buffers and data reuse them)
    if (b->last.size() == n && std::memcmp(b->last.data(), rec.data(), sizeof(AsmArgs) * n) == 0)
        return PHF_OK;
    if (b->args_pending) {
        PHF_HIP(ctx, hipEventSynchronize(b->args_ev));  // h_args is free again
        b->args_pending = false;
    }
    std::memcpy(b->h_args, rec.data(), sizeof(AsmArgs) * n);
    PHF_HIP(ctx, hipMemcpyAsync(b->d_args, b->h_args, sizeof(AsmArgs) * n, hipMemcpyHostToDevice,
                                ctx->stream));
    PHF_HIP(ctx, hipEventRecord(b->args_ev, ctx->stream));
    b->args_pending = true;
    b->last = rec;
    return PHF_OK;
}

int batch_launch(phf_batch* b, bool hasAT, bool withD, bool genA)
{
    const int ti = tile_index(b->tile);
    const int mode = b->lanes == 4 ? 2 : (b->direct ? 1 : (b->gather ? 3 : 0));
    const int wi = mode == 2 ? 3 + ti : ti;
    TRY(batch_work(b, wi));
    switch (b->tile) {
    case 64: return launch_batch_tn<64>(b, wi, mode, hasAT, withD, genA);
    case 128: return launch_batch_tn<128>(b, wi, mode, hasAT, withD, genA);
    default: return launch_batch_tn<256>(b, wi, mode, hasAT, withD, genA);
    }
}
}  // namespace

extern "C" int phf_batch_destroy(phf_batch* b)
{
    if (!b) return PHF_EINVAL;
    (void)hipStreamSynchronize(b->ctx->stream);
    if (b->counted) {
        for (phf_mesh* m : b->meshes) m->n_users--;
        b->ctx->n_objects--;
    }
    for (auto& w : b->d_work) phf_dfree(w);
    phf_dfree(b->d_args);
    if (b->h_args) (void)hipHostFree(b->h_args);
    if (b->args_ev) (void)hipEventDestroy(b->args_ev);
    delete b;
    return PHF_OK;
}

extern "C" int phf_batch_create(phf_ctx* ctx, phf_mesh* const* meshes, int32_t n, phf_batch** out)
{
    if (!ctx || !out || n < 1 || !meshes) return PHF_EINVAL;
    *out = nullptr;
    for (int32_t i = 0; i < n; ++i)
        if (!meshes[i] || meshes[i]->ctx != ctx)
            return phf_set_error(ctx, PHF_EINVAL,
                                 "phf_batch_create: mesh %d is null or of another context", i);
    phf_batch* b = new (std::nothrow) phf_batch;
    if (!b) return phf_set_error(ctx, PHF_ENOMEM, "host allocation failed");
    b->ctx = ctx;
    b->meshes.assign(meshes, meshes + n);
    int ncu = 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, ctx->device) ==
            hipSuccess && ncu > 0)
        b->ncu = ncu;
    auto body = [&]() -> int {
        PHF_HIP(ctx, hipHostMalloc((void**)&b->h_args, sizeof(AsmArgs) * n, hipHostMallocDefault));
        TRY(phf_dmalloc(ctx, &b->d_args, (size_t)n, "batch records"));
        PHF_HIP(ctx, hipEventCreateWithFlags(&b->args_ev, hipEventDisableTiming));
        return PHF_OK;
    };
    int rc = body();
    if (rc) {
        phf_batch_destroy(b);
        return rc;
    }
    b->counted = true;
    for (phf_mesh* m : b->meshes) m->n_users++;
    ctx->n_objects++;
    *out = b;
    return PHF_OK;
}

extern "C" int phf_batch_assemble(phf_batch* b, const phf_coeffs* co, const phf_data* data,
                                  const phf_system* out)
{
    if (!b) return PHF_EINVAL;
    bool hasAT, withD, genA;
    TRY(batch_prepare(b, co, data, out, &hasAT, &withD, &genA));
    return batch_launch(b, hasAT, withD, genA);
}

extern "C" int phf_batch_get_config(const phf_batch* b, phf_batch_config* cfg)
{
    if (!b || !cfg) return PHF_EINVAL;
    cfg->tile = b->tile;
    cfg->blocks_per_cu = b->blocks_per_cu;
    cfg->ms = -1.0;
    cfg->lanes = b->lanes;
    cfg->direct = b->direct;
    cfg->gather = b->gather;
    cfg->reserved_ = 0;
    return PHF_OK;
}

extern "C" int phf_batch_set_config(phf_batch* b, const phf_batch_config* cfg)
{
    if (!b || !cfg) return PHF_EINVAL;
    const int32_t lanes = cfg->lanes == 0 ? 1 : cfg->lanes;
    if (tile_index(cfg->tile) < 0 || cfg->blocks_per_cu < 0 || cfg->blocks_per_cu > 64 ||
        (lanes != 1 && lanes != 4) || (cfg->direct != 0 && cfg->direct != 1) ||
        (cfg->gather != 0 && cfg->gather != 1) ||
        ((lanes == 4 || cfg->direct || cfg->gather) && cfg->blocks_per_cu != 0) ||
        (lanes == 4 && (cfg->direct || cfg->gather)) || (cfg->direct && cfg->gather))
        return phf_set_error(b->ctx, PHF_EINVAL,
                             "phf_batch_set_config: tile must be 64, 128 or 256, blocks_per_cu "
                             "0..64 (0 unless the tile is staged from element records), lanes 1 "
                             "or 4, direct and gather 0 or 1, at most one of lanes = 4, direct, "
                             "gather");
    b->tile = cfg->tile;
    b->blocks_per_cu = cfg->blocks_per_cu;
    b->lanes = lanes;
    b->direct = cfg->direct;
    b->gather = cfg->gather;
    return PHF_OK;
}

extern "C" int phf_batch_tune(phf_batch* b, const phf_coeffs* co, const phf_data* data,
                              const phf_system* out, int32_t reps, phf_batch_config* results,
                              int32_t max_results, int32_t* n_results)
{
    if (!b) return PHF_EINVAL;
    phf_ctx* ctx = b->ctx;
    if (reps < 1) reps = 5;
    bool hasAT, withD, genA;
    TRY(batch_prepare(b, co, data, out, &hasAT, &withD, &genA));
    // candidate shapes: staged element tiles with one workgroup per item or a
    // persistent grid; per-thread stores; four lanes per triangle
    struct shape {
        int32_t tile, bpc, lanes, direct, gather;
    };
    std::vector<shape> shapes;
    for (int32_t tile : {64, 128, 256})
        for (int32_t bpc : {0, 2, 4, 8}) shapes.push_back({tile, bpc, 1, 0, 0});
    for (int32_t tile : {64, 128, 256}) shapes.push_back({tile, 0, 1, 1, 0});
    for (int32_t tile : {64, 128, 256}) shapes.push_back({tile, 0, 4, 0, 0});
    for (int32_t tile : {64, 128, 256}) shapes.push_back({tile, 0, 1, 0, 1});
    hipEvent_t e0 = nullptr, e1 = nullptr;
    PHF_HIP(ctx, hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return phf_set_error(ctx, PHF_EHIP, "phf_batch_tune: event creation failed");
    }
    const shape keep{b->tile, b->blocks_per_cu, b->lanes, b->direct, b->gather};
    shape bestc = keep;
    int32_t cnt = 0;
    double best = 1e300;
    int rc = PHF_OK;
    for (const shape& sh : shapes) {
        b->tile = sh.tile;
        b->blocks_per_cu = sh.bpc;
        b->lanes = sh.lanes;
        b->direct = sh.direct;
        b->gather = sh.gather;
        rc = batch_launch(b, hasAT, withD, genA);  // warm-up (and work list)
        if (rc) break;
        if (hipEventRecord(e0, ctx->stream) != hipSuccess) {
            rc = phf_set_error(ctx, PHF_EHIP, "phf_batch_tune: event record failed");
            break;
        }
        for (int32_t r = 0; r < reps && !rc; ++r) rc = batch_launch(b, hasAT, withD, genA);
        if (rc) break;
        float ms = 0.f;
        if (hipEventRecord(e1, ctx->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
            rc = phf_set_error(ctx, PHF_EHIP, "phf_batch_tune: timing failed");
            break;
        }
        const double avg = (double)ms / reps;
        if (results && cnt < max_results)
            results[cnt] = {sh.tile, sh.bpc, avg, sh.lanes, sh.direct, sh.gather, 0};
        ++cnt;
        if (avg < best) {
            best = avg;
            bestc = sh;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) {
        b->tile = keep.tile;
        b->blocks_per_cu = keep.bpc;
        b->lanes = keep.lanes;
        b->direct = keep.direct;
        b->gather = keep.gather;
        return rc;
    }
    b->tile = bestc.tile;
    b->blocks_per_cu = bestc.bpc;
    b->lanes = bestc.lanes;
    b->direct = bestc.direct;
    b->gather = bestc.gather;
    if (n_results) *n_results = std::min(cnt, max_results);
    return PHF_OK;
}
