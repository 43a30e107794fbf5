// Mesh upload, validation, edge topology (Section 2.2), boundary
// classification and CSR patterns (Section 3.5) on the device.
//
// Edge numbering: an edge {a, b} has key (max, min); edges are numbered in
// ascending key order. The build is a counting sort of the 3 nE directed
// local edges by their larger node (integer atomics count bucket sizes and
// hand out slots; the order inside a bucket is then fixed by sorting on
// (smaller node, position 3m+j)), so every output is independent of atomic
// ordering. T+ of an edge is its first occurrence in element order.
#include <cstring>

#include "phf_device.h"
#include "phf_internal.h"

namespace {

enum : int { FLAG_RANGE = 1, FLAG_ORIENT = 2, FLAG_MESH = 4, FLAG_BOUNDARY = 8 };

// Numbers of Dirichlet (d) and Neumann (n) edges.
struct phf_cnt2 {
    int32_t d, n;
};
__host__ __device__ inline phf_cnt2 operator+(phf_cnt2 a, phf_cnt2 b)
{
    return phf_cnt2{a.d + b.d, a.n + b.n};
}

__device__ inline void raise_flag(int* flags, int bit, int32_t where)
{
    atomicOr(&flags[0], bit);
    atomicMin(&flags[1], where);
}

// Validates element m, stores its record and counts its directed edges.
__global__ __launch_bounds__(256) void k_elem_init(const int32_t* __restrict__ raw, int32_t nE,
                                                   int32_t nC, const double2* __restrict__ xy,
                                                   int4* __restrict__ elem4,
                                                   int32_t* __restrict__ bucket_count,
                                                   int* flags)
{
    int32_t m = blockIdx.x * 256 + threadIdx.x;
    if (m >= nE) return;
    int32_t v0 = raw[3 * (int64_t)m], v1 = raw[3 * (int64_t)m + 1], v2 = raw[3 * (int64_t)m + 2];
    if (v0 < 0 || v0 >= nC || v1 < 0 || v1 >= nC || v2 < 0 || v2 >= nC) {
        raise_flag(flags, FLAG_RANGE, m);
        return;
    }
    if (v0 == v1 || v1 == v2 || v0 == v2) {
        raise_flag(flags, FLAG_ORIENT, m);
        return;
    }
    double2 p0 = xy[v0], p1 = xy[v1], p2 = xy[v2];
    double det = (p1.x - p0.x) * (p2.y - p0.y) - (p2.x - p0.x) * (p1.y - p0.y);
    if (!(det > 0.0)) raise_flag(flags, FLAG_ORIENT, m);
    elem4[m] = make_int4(v0, v1, v2, 0);
    atomicAdd(&bucket_count[max(v0, v1)], 1);
    atomicAdd(&bucket_count[max(v1, v2)], 1);
    atomicAdd(&bucket_count[max(v2, v0)], 1);
}

__global__ __launch_bounds__(256) void k_fill(const int4* __restrict__ elem4, int32_t nE,
                                              const int32_t* __restrict__ bucket_off,
                                              int32_t* __restrict__ cursor,
                                              uint64_t* __restrict__ keys)
{
    int32_t m = blockIdx.x * 256 + threadIdx.x;
    if (m >= nE) return;
    int4 e = elem4[m];
    int32_t v[3] = {e.x, e.y, e.z};
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        int32_t a = v[j], b = v[(j + 1) % 3];
        int32_t hi = max(a, b), lo = min(a, b);
        int32_t slot = bucket_off[hi] + atomicAdd(&cursor[hi], 1);
        keys[slot] = ((uint64_t)(uint32_t)lo << 32) | (uint32_t)(3 * m + j);
    }
}

__device__ inline int32_t start_node(const int4* elem4, uint32_t pos)
{
    int4 e = elem4[pos / 3];
    int j = pos % 3;
    return j == 0 ? e.x : (j == 1 ? e.y : e.z);
}

// Sorts bucket v by (smaller node, position) and counts its distinct edges.
__global__ __launch_bounds__(256) void k_bucket_sort(uint64_t* __restrict__ keys,
                                                     const int32_t* __restrict__ bucket_off,
                                                     int32_t nC, const int4* __restrict__ elem4,
                                                     int32_t* __restrict__ ucount, int* flags)
{
    int32_t v = blockIdx.x * 256 + threadIdx.x;
    if (v >= nC) return;
    int32_t b0 = bucket_off[v], b1 = bucket_off[v + 1];
    // insertion sort in place (buckets hold ~2 x the lower-neighbour count)
    for (int32_t q = b0 + 1; q < b1; ++q) {
        uint64_t k = keys[q];
        int32_t s = q - 1;
        while (s >= b0 && keys[s] > k) {
            keys[s + 1] = keys[s];
            --s;
        }
        keys[s + 1] = k;
    }
    int32_t n = 0;
    int32_t q = b0;
    while (q < b1) {
        uint32_t lo = (uint32_t)(keys[q] >> 32);
        int32_t t = q + 1;
        while (t < b1 && (uint32_t)(keys[t] >> 32) == lo) ++t;
        if (t - q > 2) {
            raise_flag(flags, FLAG_MESH, (int32_t)((uint32_t)keys[q] / 3));
        } else if (t - q == 2) {
            uint32_t p0 = (uint32_t)keys[q], p1 = (uint32_t)keys[q + 1];
            if (start_node(elem4, p0) == start_node(elem4, p1))
                raise_flag(flags, FLAG_MESH, (int32_t)(p1 / 3));
        }
        ++n;
        q = t;
    }
    ucount[v] = n;
}

// Writes the edge tables of bucket v (edges eoff[v] .. eoff[v+1]-1).
__global__ __launch_bounds__(256) void k_emit(const uint64_t* __restrict__ keys,
                                              const int32_t* __restrict__ bucket_off,
                                              const int32_t* __restrict__ eoff, int32_t nC,
                                              const int4* __restrict__ elem4,
                                              int2* __restrict__ edge_nodes,
                                              int2* __restrict__ edge_elems,
                                              int32_t* __restrict__ elem_edges,
                                              int8_t* __restrict__ led, int8_t* __restrict__ ledTN)
{
    int32_t v = blockIdx.x * 256 + threadIdx.x;
    if (v >= nC) return;
    int32_t b0 = bucket_off[v], b1 = bucket_off[v + 1];
    int32_t e = eoff[v];
    int32_t q = b0;
    while (q < b1) {
        uint32_t lo = (uint32_t)(keys[q] >> 32);
        int32_t t = q + 1;
        while (t < b1 && (uint32_t)(keys[t] >> 32) == lo) ++t;
        uint32_t p = (uint32_t)keys[q];
        int32_t m = (int32_t)(p / 3), j = (int32_t)(p % 3);
        int4 el = elem4[m];
        int32_t vv[3] = {el.x, el.y, el.z};
        edge_nodes[e] = make_int2(vv[j], vv[(j + 1) % 3]);
        int8_t lp = (int8_t)((j + 2) % 3);
        led[e] = lp;
        elem_edges[3 * (int64_t)m + lp] = e;
        if (t - q >= 2) {
            uint32_t p2 = (uint32_t)keys[q + 1];
            int32_t m2 = (int32_t)(p2 / 3), j2 = (int32_t)(p2 % 3);
            int8_t ln = (int8_t)((j2 + 2) % 3);
            edge_elems[e] = make_int2(m, m2);
            ledTN[e] = ln;
            elem_edges[3 * (int64_t)m2 + ln] = e;
        } else {
            edge_elems[e] = make_int2(m, -1);
            ledTN[e] = lp;
        }
        ++e;
        q = t;
    }
}

__device__ inline int32_t find_edge(int32_t a, int32_t b, const int32_t* eoff,
                                    const int2* edge_nodes)
{
    int32_t hi = max(a, b), lo = min(a, b);
    int32_t L = eoff[hi], R = eoff[hi + 1] - 1;
    while (L <= R) {
        int32_t mid = L + (R - L) / 2;
        int2 kl = edge_nodes[mid];
        int32_t l2 = min(kl.x, kl.y);
        if (l2 == lo) return mid;
        if (l2 < lo) L = mid + 1;
        else R = mid - 1;
    }
    return -1;
}

// One thread per listed boundary pair (Dirichlet first, then Neumann).
__global__ __launch_bounds__(256) void k_boundary_mark(
    const int32_t* __restrict__ dir, int32_t nD, const int32_t* __restrict__ neu, int32_t nN,
    int32_t nC, const int32_t* __restrict__ eoff, const int2* __restrict__ edge_nodes,
    const int2* __restrict__ edge_elems, int32_t* __restrict__ mark, int8_t* __restrict__ etype,
    int32_t* __restrict__ dir_edges, int32_t* __restrict__ neu_edges, int* flags)
{
    int32_t q = blockIdx.x * 256 + threadIdx.x;
    if (q >= nD + nN) return;
    bool isD = q < nD;
    const int32_t* pr = isD ? dir + 2 * (int64_t)q : neu + 2 * (int64_t)(q - nD);
    int32_t a = pr[0], b = pr[1];
    if (a < 0 || a >= nC || b < 0 || b >= nC || a == b) {
        raise_flag(flags, FLAG_BOUNDARY, q);
        return;
    }
    int32_t e = find_edge(a, b, eoff, edge_nodes);
    if (e < 0 || edge_elems[e].y >= 0) {
        raise_flag(flags, FLAG_BOUNDARY, q);
        return;
    }
    if (atomicAdd(&mark[e], 1) != 0) {
        raise_flag(flags, FLAG_BOUNDARY, q);
        return;
    }
    etype[e] = isD ? 1 : 2;
    if (isD) dir_edges[q] = e;
    else neu_edges[q - nD] = e;
}

// Per-tile (256 edges) numbers of Dirichlet and Neumann edges; with `mark`
// (a mesh given by the caller) also checks that every boundary edge was
// listed.
__device__ inline void d_rows_count(int32_t bid, int32_t n_edges, const int8_t* __restrict__ etype,
                                                    const int2* __restrict__ edge_elems,
                                                    const int32_t* __restrict__ mark,
                                                    phf_cnt2* __restrict__ tiles, int* flags)
{
    __shared__ phf_cnt2 sh[4];
    const int32_t e = bid * 256 + threadIdx.x;
    int t = 0;
    if (e < n_edges) {
        t = etype[e];
        if (mark && edge_elems[e].y < 0 && mark[e] == 0) raise_flag(flags, FLAG_BOUNDARY, e);
    }
    const uint64_t bd = __ballot(t == 1), bn = __ballot(t == 2);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = phf_cnt2{(int32_t)__popcll(bd), (int32_t)__popcll(bn)};
    __syncthreads();
    if (threadIdx.x == 0) tiles[bid] = sh[0] + sh[1] + sh[2] + sh[3];
}

// Exclusive prefix sums, in place, of n per-tile values by one workgroup of
// 1024 threads (each a contiguous run of tiles); *total (nullable) = the sum.
template <typename T>
__device__ inline void d_tile_exscan(int32_t n, T* __restrict__ v, T* __restrict__ total)
{
    __shared__ T sh[1024];
    const int32_t tid = threadIdx.x;
    const int32_t per = (n + 1023) / 1024;
    const int32_t b0 = min(n, tid * per), b1 = min(n, b0 + per);
    T s{};
    for (int32_t i = b0; i < b1; ++i) s = s + v[i];
    sh[tid] = s;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {  // inclusive scan of the runs
        const T a = tid >= off ? sh[tid - off] : T{};
        __syncthreads();
        sh[tid] = sh[tid] + a;
        __syncthreads();
    }
    T run = tid > 0 ? sh[tid - 1] : T{};
    for (int32_t i = b0; i < b1; ++i) {
        const T x = v[i];
        v[i] = run;
        run = run + x;
    }
    if (tid == 1023 && total) *total = sh[1023];
}

// Multiplier-row tables and the C pattern. With D(e), N(e) the Dirichlet and
// Neumann edges before e (tile base plus ballot prefix): multiplier row
// e - N(e), free row e - D(e), C row pointer 4 (e - D(e) - N(e)) + 2 D(e).
__device__ inline void d_rows(int32_t bid, 
    int32_t n_edges, const int8_t* __restrict__ etype, const phf_cnt2* __restrict__ tiles,
    const int2* __restrict__ edge_nodes, const int2* __restrict__ edge_elems,
    const int8_t* __restrict__ led, const int8_t* __restrict__ ledTN,
    int32_t* __restrict__ edge_row, int32_t* __restrict__ red_row,
    int32_t* __restrict__ red_edge, int32_t* __restrict__ row_edge,
    int2* __restrict__ row_nodes, const double2* __restrict__ xy, double* __restrict__ row_hs,
    int32_t* __restrict__ C_rowptr, int32_t* __restrict__ C_col,
    int32_t L, int32_t nnzC, int32_t nnz_dof, int32_t* __restrict__ S_rowptr_m,
    int32_t* __restrict__ S_col_m)
{
    __shared__ phf_cnt2 sh[4];
    const int32_t e = bid * 256 + threadIdx.x;
    if (e == 0) {  // the closing row pointers
        C_rowptr[L] = nnzC;
        S_rowptr_m[L] = nnz_dof + nnzC;
    }
    const int t = e < n_edges ? etype[e] : 0;
    const uint64_t bd = __ballot(t == 1), bn = __ballot(t == 2);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) sh[wid] = phf_cnt2{(int32_t)__popcll(bd), (int32_t)__popcll(bn)};
    __syncthreads();
    phf_cnt2 before = tiles[bid];
    for (int w = 0; w < wid; ++w) before = before + sh[w];
    const uint64_t below = lane == 0 ? 0ull : (1ull << lane) - 1ull;
    const int32_t nd = before.d + (int32_t)__popcll(bd & below),
                  nn = before.n + (int32_t)__popcll(bn & below);
    if (e >= n_edges) return;
    if (t == 1) {
        red_row[e] = -1;
    } else {
        const int32_t rr = e - nd;
        red_row[e] = rr;
        red_edge[rr] = e;
    }
    if (t == 2) {
        edge_row[e] = -1;
        return;
    }
    const int32_t r = e - nn;
    edge_row[e] = r;
    row_edge[r] = e;
    const int2 kl = edge_nodes[e];
    row_nodes[r] = make_int2(t == 1 ? ~kl.x : kl.x, kl.y);
    const double h = phf_half_length(xy[kl.x], xy[kl.y]);
    row_hs[r] = t == 1 ? -h : h;
    const int32_t c = 4 * (e - nd - nn) + 2 * nd;
    C_rowptr[r] = c;
    // saddle multiplier row r = C's row r, after the DOF rows' entries
    S_rowptr_m[r] = nnz_dof + c;
    int2 tt = edge_elems[e];
    // vertex DOFs of the edge in T+ (the two local vertices != led), ascending
    int lp = led[e];
    int a = lp == 0 ? 1 : 0, b = lp == 2 ? 1 : 2;
    int32_t cc[4] = {3 * tt.x + a, 3 * tt.x + b, 0, 0};
    int nc = 2;
    if (t == 0) {
        int ln = ledTN[e];
        int a2 = ln == 0 ? 1 : 0, b2 = ln == 2 ? 1 : 2;
        cc[2] = 3 * tt.y + a2;
        cc[3] = 3 * tt.y + b2;
        nc = 4;
    }
    for (int k = 0; k < nc; ++k) {
        C_col[c + k] = cc[k];
        S_col_m[c + k] = cc[k];
    }
}

// Element code words, the element-major coordinate copy, and per tile (256
// elements) the number of Neumann edge incidences.
// Element codes. On a refined mesh (ecode_c: the parent's codes) the edge
// types and T+ flags follow from the parent's code (numbering Section 2.3):
// the centre child m < nE_c has three interior edges and is their T+ side; the
// corner child nE_c + 3T + i has the interior edge shared with the centre
// child as local edge 0 (its T- side) and, as local edges 1 and 2, the halves
// of the parent's edges i+1 and i+2 at vertex i, with their parent's type and
// on the T+ side exactly where T is. Otherwise they are gathered from the
// edge tables.
__device__ inline void d_elem_codes(int32_t bid, int32_t nE, int4* __restrict__ elem4,
                                                    const int32_t* __restrict__ elem_edges,
                                                    const int8_t* __restrict__ etype,
                                                    const int2* __restrict__ edge_elems,
                                                    const int32_t* __restrict__ ecode_c,
                                                    int32_t nE_c,
                                                    const double2* __restrict__ xy,
                                                    double2* __restrict__ exy,
                                                    int32_t* __restrict__ ecode,
                                                    int32_t* __restrict__ tiles)
{
    __shared__ int32_t sh[256 / 64];
    const int32_t m = bid * 256 + threadIdx.x;
    int32_t nneu = 0;
    if (m < nE) {
        int32_t ed[3];
        int code = 0;
#pragma unroll
        for (int i = 0; i < 3; ++i) ed[i] = elem_edges[3 * (int64_t)m + i];
        if (ecode_c) {
            if (m < nE_c) {
                code = 7 << 6;
            } else {
                const int32_t q = m - nE_c, ci = q % 3;
                const int pc = ecode_c[q / 3];
                const int e1 = (ci + 1) % 3, e2 = (ci + 2) % 3;
                const int t1 = PHF_CODE_TYPE(pc, e1), t2 = PHF_CODE_TYPE(pc, e2);
                nneu = (t1 == 2) + (t2 == 2);
                code = (t1 << 2) | (t2 << 4) | (PHF_CODE_TPLUS(pc, e1) << 7) |
                       (PHF_CODE_TPLUS(pc, e2) << 8);
            }
        } else {
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                const int tp = etype[ed[i]];
                nneu += tp == 2;
                code |= tp << (2 * i);
                if (edge_elems[ed[i]].x == m) code |= 1 << (6 + i);
            }
        }
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            int l1 = i == 0 ? 1 : 0, l2 = i == 2 ? 1 : 2;
            if (ed[l1] > ed[l2]) code |= 1 << (9 + i);
        }
        int4 e = elem4[m];
        e.w = code;
        elem4[m] = e;
        ecode[m] = code;
        if (xy) {  // (a refined mesh has its element coordinates already)
            exy[3 * (int64_t)m] = xy[e.x];
            exy[3 * (int64_t)m + 1] = xy[e.y];
            exy[3 * (int64_t)m + 2] = xy[e.z];
        }
    }
    const int32_t tot = phf_block_sum_i32<256>(nneu, sh);
    if (threadIdx.x == 0) tiles[bid] = tot;
}

// Saddle pattern, DOF rows of element m: 3 + (non-Neumann edges of m at
// vertex i) entries in row 3m+i, the rows of m starting at 15 m - 2 (Neumann
// incidences before m) (tile base plus block prefix). Columns: the element's
// three DOFs, then the multiplier rows of its non-Neumann edges at vertex i
// in ascending edge order. The block's rows and columns are contiguous in
// S_rowptr and S_col: they are assembled in LDS and stored coalesced.
__device__ inline void d_saddle_dof(int32_t bid, int32_t nE, const int32_t* __restrict__ ecode,
                                                    const int32_t* __restrict__ tiles,
                                                    const int32_t* __restrict__ elem_edges,
                                                    const int32_t* __restrict__ edge_row,
                                                    const int32_t* __restrict__ red_row,
                                                    int32_t* __restrict__ S_rowptr,
                                                    int32_t* __restrict__ S_col,
                                                    int32_t* __restrict__ elem_row,
                                                    int32_t* __restrict__ elem_red)
{
    __shared__ int32_t sh[256 / 64 + 1];
    __shared__ int32_t scol[256 * 15];
    __shared__ int32_t srow[256 * 3];
    const int32_t m0 = bid * 256, m = m0 + threadIdx.x;
    const int32_t cnt = min(256, nE - m0);
    const int code = m < nE ? ecode[m] : 0;
    int nneu = 0;
#pragma unroll
    for (int l = 0; l < 3; ++l) nneu += PHF_CODE_TYPE(code, l) == 2;
    int32_t tot;
    const int32_t ex = phf_block_exscan_i32<256>(nneu, sh, &tot);
    const int32_t base = 15 * m0 - 2 * tiles[bid];  // first entry of the block
    if (m < nE) {
        const int32_t N = 3 * nE;
        // the rows of the three local edges, gathered once (also kept per
        // element for the solver)
        int32_t er[3];
#pragma unroll
        for (int l = 0; l < 3; ++l) {
            const int32_t e = elem_edges[3 * (int64_t)m + l];
            er[l] = edge_row[e];
            elem_row[3 * (int64_t)m + l] = er[l];
            elem_red[3 * (int64_t)m + l] = red_row[e];
        }
        int32_t s = 15 * (int32_t)threadIdx.x - 2 * ex;  // offset in the block
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            srow[3 * threadIdx.x + i] = base + s;
            scol[s] = 3 * m;
            scol[s + 1] = 3 * m + 1;
            scol[s + 2] = 3 * m + 2;
            int l1 = i == 0 ? 1 : 0, l2 = i == 2 ? 1 : 2;
            if (PHF_CODE_SWAP(code, i)) {
                int t = l1;
                l1 = l2;
                l2 = t;
            }
            int32_t k = s + 3;
            if (PHF_CODE_TYPE(code, l1) != 2) scol[k++] = N + er[l1];
            if (PHF_CODE_TYPE(code, l2) != 2) scol[k++] = N + er[l2];
            s = k;
        }
    }
    __syncthreads();
    const int32_t len = 15 * cnt - 2 * tot;
    for (int32_t q = threadIdx.x; q < len; q += 256) S_col[(int64_t)base + q] = scol[q];
    for (int32_t q = threadIdx.x; q < 3 * cnt; q += 256) S_rowptr[3 * (int64_t)m0 + q] = srow[q];
}


// Off-diagonal entries of the reduced (edge-midpoint) operator: each
// element couples its f free (non-Dirichlet) edges pairwise, f (f - 1)
// entries; two distinct edges share at most one element, so the count is
// exact. Per-block sums go to *total with integer atomics (order-independent;
// a bounded grid keeps the atomics few).
__device__ inline void d_reduced_count(int32_t bid, int32_t nblocks, int32_t nE, const int32_t* __restrict__ ecode,
                                                       unsigned long long* total)
{
    __shared__ int32_t sh[256 / 64 + 1];
    int32_t n = 0;  // at most 6 per element, 6 nE < 2^31 per block
    for (int32_t m = bid * 256 + threadIdx.x; m < nE; m += nblocks * 256) {
        const int32_t code = ecode[m];
        int f = 0;
        for (int i = 0; i < 3; ++i) f += PHF_CODE_TYPE(code, i) != 1;
        n += f * (f - 1);
    }
    int32_t tot;
    (void)phf_block_exscan_i32<256>(n, sh, &tot);
    if (threadIdx.x == 0 && tot) atomicAdd(total, (unsigned long long)tot);
}


__device__ inline void d_c_tiles(int32_t bid, int32_t L, const int32_t* __restrict__ C_rowptr,
                                                 int32_t* __restrict__ C_tile)
{
    int32_t t = bid * 256 + threadIdx.x;
    int32_t nt = (L + 255) / 256;
    if (t > nt) return;
    C_tile[t] = C_rowptr[min(256 * t, L)];
}

// One bit per element: does it own a Neumann edge? Each wavefront packs the
// bits of 64 consecutive elements with a ballot.
__device__ inline void d_neu_mask(int32_t bid, int32_t nE, const int32_t* __restrict__ ecode,
                                                  uint64_t* __restrict__ mask)
{
    const int64_t m = (int64_t)bid * 256 + threadIdx.x;
    const bool f = m < nE && (ecode[m] & 0x2A) != 0;
    const uint64_t b = __ballot(f);
    if ((threadIdx.x & 63) == 0 && m < nE) mask[m >> 6] = b;
}

}  // namespace

// ---------------------------------------------------------------------------

namespace {
__device__ inline void d_refine_nodes(int32_t bid, int32_t nC, int32_t ne,
                                                      const double2* __restrict__ xy,
                                                      const int2* __restrict__ edge_nodes,
                                                      double2* __restrict__ xy_f)
{
    const int64_t g = (int64_t)bid * 256 + threadIdx.x;
    if (g < nC) {
        xy_f[g] = xy[g];
    } else if (g < (int64_t)nC + ne) {
        const int2 kl = edge_nodes[g - nC];
        const double2 a = xy[kl.x], b = xy[kl.y];
        xy_f[g] = make_double2(0.5 * (a.x + b.x), 0.5 * (a.y + b.y));
    }
}

// Children of element m: [M0 M1 M2] at m and [v_i, M_(i+2), M_(i+1)] at
// nE + 3m + i, with M_i = nC + (edge opposite vertex i).
// Also the children's element-major coordinates from the parent's: the
// midpoint of the edge opposite v_i is 0.5 (P_(i+1) + P_(i+2)), the value the
// refined node gets (the sum is the same in either order).
__device__ inline void d_refine_elems(int32_t bid, int32_t nC, int32_t nE,
                                                      const int4* __restrict__ elem4,
                                                      const int32_t* __restrict__ elem_edges,
                                                      const double2* __restrict__ exy,
                                                      int4* __restrict__ el_f,
                                                      double2* __restrict__ exy_f)
{
    const int32_t m = bid * 256 + threadIdx.x;
    if (m >= nE) return;
    const int4 e = elem4[m];
    const int32_t v[3] = {e.x, e.y, e.z};
    int32_t M[3];
    for (int i = 0; i < 3; ++i) M[i] = nC + elem_edges[3 * (int64_t)m + i];
    el_f[m] = make_int4(M[0], M[1], M[2], 0);
    for (int i = 0; i < 3; ++i)
        el_f[(int64_t)nE + 3 * (int64_t)m + i] = make_int4(v[i], M[(i + 2) % 3], M[(i + 1) % 3], 0);
    double2 P[3], Q[3];
    for (int i = 0; i < 3; ++i) P[i] = exy[3 * (int64_t)m + i];
    for (int i = 0; i < 3; ++i) {
        const double2 a = P[(i + 1) % 3], b = P[(i + 2) % 3];
        Q[i] = make_double2(0.5 * (a.x + b.x), 0.5 * (a.y + b.y));
    }
    for (int i = 0; i < 3; ++i) exy_f[3 * (int64_t)m + i] = Q[i];
    for (int i = 0; i < 3; ++i) {
        const int64_t c = 3 * ((int64_t)nE + 3 * (int64_t)m + i);
        exy_f[c] = P[i];
        exy_f[c + 1] = Q[(i + 2) % 3];
        exy_f[c + 2] = Q[(i + 1) % 3];
    }
}

// Listed pair q of edge e: (a, M_e) at q and (M_e, b) at n + q.
__device__ inline void d_refine_pairs(int32_t bid, int32_t nC, int32_t n,
                                                      const int2* __restrict__ pairs,
                                                      const int32_t* __restrict__ edges,
                                                      int2* __restrict__ out)
{
    const int32_t q = bid * 256 + threadIdx.x;
    if (q >= n) return;
    const int2 ab = pairs[q];
    const int32_t mid = nC + edges[q];
    out[q] = make_int2(ab.x, mid);
    out[n + q] = make_int2(mid, ab.y);
}

// ---- topology of a red-refined mesh from its parent's tables ----------------
// Every fine edge has a midpoint node M_e = nC + e of a parent edge e as its
// larger node (the parent's nodes keep their numbers, midpoints come after
// them). Sorting by (larger node, smaller node) therefore groups the fine
// edges by parent edge, in parent-edge order; within group e come first the
// two halves of e (smaller node: the parent end nodes, in increasing order),
// then the inner edges (M_e, M_e') of the parent triangles at e with e' < e,
// in increasing e'. The children of parent p are p = [M0 M1 M2] and
// nE + 3p + i = [v_i, M_(i+2), M_(i+1)]; an element's local edge l runs from
// its vertex l+1 to vertex l+2. The fine element of lower number on a fine
// edge (its T+) is the centre child for inner edges and the corner child of
// the parent's T+ for halves.

// Fine edges of group e (2 halves + inner edges with e' < e).
// Fine edges in the group of parent edge e, summed over each tile of 256
// parent edges (tiles[bid]) and as the exclusive prefix inside the tile
// (pre[e]); the group's offset is the tile base (one scan over the tiles)
// plus pre[e].
__device__ inline void d_rt_count(int32_t bid, int32_t ne_c, const int2* __restrict__ edge_elems_c,
                                                  const int8_t* __restrict__ led_c,
                                                  const int8_t* __restrict__ ledTN_c,
                                                  const int32_t* __restrict__ elem_edges_c,
                                                  int32_t* __restrict__ pre,
                                                  int32_t* __restrict__ tiles)
{
    __shared__ int32_t sh[256 / 64 + 1];
    const int32_t e = bid * 256 + threadIdx.x;
    int32_t c = 0;
    if (e < ne_c) {
        const int2 tt = edge_elems_c[e];
        c = 2;
        for (int side = 0; side < 2; ++side) {
            const int32_t T = side ? tt.y : tt.x;
            if (T < 0) continue;
            const int le = side ? ledTN_c[e] : led_c[e];
            for (int d = 1; d <= 2; ++d)
                if (elem_edges_c[3 * (int64_t)T + (le + d) % 3] < e) ++c;
        }
    }
    int32_t tot;
    const int32_t ex = phf_block_exscan_i32<256>(c, sh, &tot);
    if (e < ne_c) pre[e] = ex;
    if (threadIdx.x == 0) tiles[bid] = tot;
}

__device__ inline void d_rt_emit(int32_t bid, 
    int32_t ne_c, int32_t nC_c, int32_t nE_c, const int2* __restrict__ edge_nodes_c,
    const int2* __restrict__ edge_elems_c, const int8_t* __restrict__ led_c,
    const int8_t* __restrict__ ledTN_c, const int32_t* __restrict__ elem_edges_c,
    const int4* __restrict__ elem4_c, const int8_t* __restrict__ etype_c,
    const int32_t* __restrict__ pre, const int32_t* __restrict__ tiles,
    int2* __restrict__ edge_nodes, int2* __restrict__ edge_elems,
    int32_t* __restrict__ elem_edges, int8_t* __restrict__ led, int8_t* __restrict__ ledTN,
    int8_t* __restrict__ etype)
{
    const int32_t e = bid * 256 + threadIdx.x;
    if (e >= ne_c) return;
    const int32_t base = tiles[bid] + pre[e], Me = nC_c + e;
    const int2 tt = edge_elems_c[e];
    const int2 kl = edge_nodes_c[e];
    const int32_t lo = min(kl.x, kl.y);
    const int8_t ty = etype_c[e];
    // halves: per side the corner children at the two end vertices of e
    int32_t he[2][2], hl[2][2];  // [half 0: at lo, 1: at hi][side]: fine element, local edge
    int2 hdir[2] = {make_int2(0, 0), make_int2(0, 0)};  // direction in the T+ side's child
    he[0][1] = he[1][1] = -1;
    hl[0][1] = hl[1][1] = 0;
    he[0][0] = he[1][0] = -1;
    hl[0][0] = hl[1][0] = 0;
    // inner edges of this group
    int32_t ie[4], it[4], il[4];
    int ni = 0;
    for (int side = 0; side < 2; ++side) {
        const int32_t T = side ? tt.y : tt.x;
        if (T < 0) continue;
        const int le = side ? ledTN_c[e] : led_c[e];
        const int4 v4 = elem4_c[T];
        const int32_t v[3] = {v4.x, v4.y, v4.z};
        // vertex i1 = le+1: its corner child has e's half as local edge 2,
        // running v_i1 -> M_e; vertex i2 = le+2: local edge 1, M_e -> v_i2
        const int i1 = (le + 1) % 3, i2 = (le + 2) % 3;
        const int h1 = v[i1] == lo ? 0 : 1, h2 = v[i2] == lo ? 0 : 1;
        he[h1][side] = nE_c + 3 * T + i1;
        hl[h1][side] = 2;
        he[h2][side] = nE_c + 3 * T + i2;
        hl[h2][side] = 1;
        if (side == 0) {
            hdir[h1] = make_int2(v[i1], Me);
            hdir[h2] = make_int2(Me, v[i2]);
        }
        for (int d = 1; d <= 2; ++d) {
            const int o = (le + d) % 3;
            const int32_t e2 = elem_edges_c[3 * (int64_t)T + o];
            if (e2 < e) {
                ie[ni] = e2;
                it[ni] = T;
                il[ni] = 3 - le - o;  // the centre child's edge joining M_e and M_e2
                ++ni;
            }
        }
    }
    for (int h = 0; h < 2; ++h) {
        const int32_t f = base + h;
        edge_nodes[f] = hdir[h];
        edge_elems[f] = make_int2(he[h][0], he[h][1]);
        led[f] = (int8_t)hl[h][0];
        ledTN[f] = (int8_t)(he[h][1] >= 0 ? hl[h][1] : hl[h][0]);
        etype[f] = ty;
        elem_edges[3 * (int64_t)he[h][0] + hl[h][0]] = f;
        if (he[h][1] >= 0) elem_edges[3 * (int64_t)he[h][1] + hl[h][1]] = f;
    }
    // inner edges in increasing e'
    for (int a = 1; a < ni; ++a) {
        const int32_t k0 = ie[a], k1 = it[a], k2 = il[a];
        int b = a - 1;
        while (b >= 0 && ie[b] > k0) {
            ie[b + 1] = ie[b];
            it[b + 1] = it[b];
            il[b + 1] = il[b];
            --b;
        }
        ie[b + 1] = k0;
        it[b + 1] = k1;
        il[b + 1] = k2;
    }
    for (int r = 0; r < ni; ++r) {
        const int32_t f = base + 2 + r, T = it[r];
        const int ls = il[r];
        const int32_t corner = nE_c + 3 * T + ls;
        edge_nodes[f] = make_int2(nC_c + elem_edges_c[3 * (int64_t)T + (ls + 1) % 3],
                                  nC_c + elem_edges_c[3 * (int64_t)T + (ls + 2) % 3]);
        edge_elems[f] = make_int2(T, corner);
        led[f] = (int8_t)ls;
        ledTN[f] = 0;
        etype[f] = 0;
        elem_edges[3 * (int64_t)T + ls] = f;
        elem_edges[3 * (int64_t)corner] = f;
    }
}

// Refined boundary edges in the refined pair order: pair q = (a, b) of parent
// edge e becomes (a, M_e) at q and (M_e, b) at n + q.
__device__ inline void d_rt_bnd(int32_t bid, int32_t n, const int2* __restrict__ pairs_c,
                                                const int32_t* __restrict__ edges_c,
                                                const int2* __restrict__ edge_nodes_c,
                                                const int32_t* __restrict__ pre,
                                                const int32_t* __restrict__ tiles,
                                                int32_t* __restrict__ edges_f)
{
    const int32_t q = bid * 256 + threadIdx.x;
    if (q >= n) return;
    const int32_t e = edges_c[q];
    const int2 ab = pairs_c[q], kl = edge_nodes_c[e];
    const int32_t lo = min(kl.x, kl.y);
    const int32_t off = tiles[e >> 8] + pre[e];
    edges_f[q] = off + (ab.x == lo ? 0 : 1);
    edges_f[n + q] = off + (ab.y == lo ? 0 : 1);
}
}  // namespace

static void mesh_free(phf_mesh* m)
{
    if (m->ns) phf_ns_destroy(m->ns);
    m->ns = nullptr;
    phf_dfree(m->xy);
    phf_dfree(m->elem4);
    phf_dfree(m->exy);
    phf_dfree(m->ecode);
    phf_dfree(m->edge_nodes);
    phf_dfree(m->edge_elems);
    phf_dfree(m->elem_edges);
    phf_dfree(m->led);
    phf_dfree(m->ledTN);
    phf_dfree(m->edge_type);
    phf_dfree(m->edge_row);
    phf_dfree(m->dir_edges);
    phf_dfree(m->neu_edges);
    phf_dfree(m->dir_pairs);
    phf_dfree(m->neu_pairs);
    phf_dfree(m->row_edge);
    phf_dfree(m->row_nodes);
    phf_dfree(m->row_hs);
    phf_dfree(m->C_tile);
    phf_dfree(m->neu_mask);
    phf_dfree(m->C_rowptr);
    phf_dfree(m->C_col);
    phf_dfree(m->S_rowptr);
    phf_dfree(m->S_col);
    phf_dfree(m->red_row);
    phf_dfree(m->red_edge);
    phf_dfree(m->elem_row);
    phf_dfree(m->elem_red);
    phf_dfree(m->d_nnzR);
}

namespace {
// Temporaries of the mesh build, freed on every exit path.
// ---- launches ---------------------------------------------------------------
// Steps of a build level that do not depend on each other share one launch:
// consecutive block ranges run different steps, each block one step (so
// block-level barriers inside a step stay uniform). On the small levels of a
// refinement chain the launches, not the bytes, are the cost.

// Refinement, first launch: child coordinates, children, refined boundary
// pairs, and the fine-edge group sizes (all from the parent's tables).
struct refine_a_args {
    int32_t nC_c, ne_c, nE_c, nD_c, nN_c;
    int32_t b1, b2, b3, b4;  // block range ends: nodes, elements, Dirichlet, Neumann
    const double2* xy_c;
    const int2* edge_nodes_c;
    double2* xy_f;
    const int4* elem4_c;
    const int32_t* elem_edges_c;
    const double2* exy_c;
    int4* elem4_f;
    double2* exy_f;
    const int2 *dir_pairs_c, *neu_pairs_c;
    const int32_t *dir_edges_c, *neu_edges_c;
    int2 *dir_pairs_f, *neu_pairs_f;
    const int2* edge_elems_c;
    const int8_t *led_c, *ledTN_c;
    int32_t* ucount;
    int32_t* utiles;
};
__global__ __launch_bounds__(256) void k_refine_a(refine_a_args a)
{
    const int32_t b = blockIdx.x;
    if (b < a.b1) d_refine_nodes(b, a.nC_c, a.ne_c, a.xy_c, a.edge_nodes_c, a.xy_f);
    else if (b < a.b2)
        d_refine_elems(b - a.b1, a.nC_c, a.nE_c, a.elem4_c, a.elem_edges_c, a.exy_c, a.elem4_f,
                       a.exy_f);
    else if (b < a.b3) d_refine_pairs(b - a.b2, a.nC_c, a.nD_c, a.dir_pairs_c, a.dir_edges_c, a.dir_pairs_f);
    else if (b < a.b4) d_refine_pairs(b - a.b3, a.nC_c, a.nN_c, a.neu_pairs_c, a.neu_edges_c, a.neu_pairs_f);
    else d_rt_count(b - a.b4, a.ne_c, a.edge_elems_c, a.led_c, a.ledTN_c, a.elem_edges_c, a.ucount,
                    a.utiles);
}

// Refinement, second launch: the fine topology and the boundary edge lists.
struct refine_b_args {
    int32_t ne_c, nC_c, nE_c, nD_c, nN_c;
    int32_t b1, b2;  // block range ends: topology, Dirichlet
    const int2 *edge_nodes_c, *edge_elems_c;
    const int8_t *led_c, *ledTN_c, *etype_c;
    const int32_t* elem_edges_c;
    const int4* elem4_c;
    const int32_t *pre, *tiles;  // in-tile prefixes of the group sizes, scanned tile sums
    int2 *edge_nodes, *edge_elems;
    int32_t* elem_edges;
    int8_t *led, *ledTN, *etype;
    const int2 *dir_pairs_c, *neu_pairs_c;
    const int32_t *dir_edges_c, *neu_edges_c;
    int32_t *dir_edges, *neu_edges;
};
__global__ __launch_bounds__(256) void k_refine_b(refine_b_args a)
{
    const int32_t b = blockIdx.x;
    if (b < a.b1)
        d_rt_emit(b, a.ne_c, a.nC_c, a.nE_c, a.edge_nodes_c, a.edge_elems_c, a.led_c, a.ledTN_c,
                  a.elem_edges_c, a.elem4_c, a.etype_c, a.pre, a.tiles, a.edge_nodes, a.edge_elems,
                  a.elem_edges, a.led, a.ledTN, a.etype);
    else if (b < a.b2)
        d_rt_bnd(b - a.b1, a.nD_c, a.dir_pairs_c, a.dir_edges_c, a.edge_nodes_c, a.pre, a.tiles,
                 a.dir_edges);
    else
        d_rt_bnd(b - a.b2, a.nN_c, a.neu_pairs_c, a.neu_edges_c, a.edge_nodes_c, a.pre, a.tiles,
                 a.neu_edges);
}

// Per-tile boundary counts of the edges (blocks [0, nt)) and the element codes
// with their per-tile Neumann incidences (the rest).
struct counts_args {
    int32_t ne, nE, nt;
    const int8_t* etype;
    const int2* edge_elems;
    const int32_t* mark;
    phf_cnt2* tiles;
    int* flags;
    int4* elem4;
    const int32_t* elem_edges;
    const int32_t* ecode_c;  // refined mesh: the parent's element codes
    int32_t nE_c;
    const double2* xy;
    double2* exy;
    int32_t* ecode;
    int32_t* etiles;
};
__global__ __launch_bounds__(256) void k_counts(counts_args a)
{
    const int32_t b = blockIdx.x;
    if (b < a.nt) d_rows_count(b, a.ne, a.etype, a.edge_elems, a.mark, a.tiles, a.flags);
    else d_elem_codes(b - a.nt, a.nE, a.elem4, a.elem_edges, a.etype, a.edge_elems, a.ecode_c,
                      a.nE_c, a.xy, a.exy, a.ecode, a.etiles);
}

// Exclusive scan of n tile sums in place (one workgroup).
__global__ __launch_bounds__(1024) void k_tile_scan1(int32_t n, int32_t* __restrict__ tiles)
{
    d_tile_exscan<int32_t>(n, tiles, nullptr);
}

// Both tile scans: block 0 the edge tiles, block 1 the element tiles.
__global__ __launch_bounds__(1024) void k_tile_scans(int32_t nt, phf_cnt2* __restrict__ tiles,
                                                     phf_cnt2* __restrict__ total, int32_t ntE,
                                                     int32_t* __restrict__ etiles)
{
    if (blockIdx.x == 0) d_tile_exscan<phf_cnt2>(nt, tiles, total);
    else d_tile_exscan<int32_t>(ntE, etiles, nullptr);
}

struct rows_args {
    int32_t ne, L, nnzC, nnz_dof;
    const int8_t* etype;
    const phf_cnt2* tiles;
    const int2 *edge_nodes, *edge_elems;
    const int8_t *led, *ledTN;
    int32_t *edge_row, *red_row, *red_edge, *row_edge;
    int2* row_nodes;
    const double2* xy;
    double* row_hs;
    int32_t *C_rowptr, *C_col, *S_rowptr_m, *S_col_m;
};
__global__ __launch_bounds__(256) void k_rows(rows_args a)
{
    d_rows(blockIdx.x, a.ne, a.etype, a.tiles, a.edge_nodes, a.edge_elems, a.led, a.ledTN,
           a.edge_row, a.red_row, a.red_edge, a.row_edge, a.row_nodes, a.xy, a.row_hs,
           a.C_rowptr, a.C_col, a.L, a.nnzC, a.nnz_dof, a.S_rowptr_m, a.S_col_m);
}

// The saddle DOF rows (blocks [0, ntE)), the C tile bases, the Neumann
// element mask and the reduced-operator size (a bounded range of blocks).
struct tail_args {
    int32_t nE, L, ntE, b1, b2, nred;  // range ends: saddle rows, C tiles, Neumann mask; reduced-count blocks
    const int32_t *ecode, *etiles, *elem_edges, *edge_row, *red_row, *C_rowptr;
    int32_t *S_rowptr, *S_col, *C_tile, *elem_row, *elem_red;
    uint64_t* neu_mask;
    unsigned long long* nnzR;
};
__global__ __launch_bounds__(256) void k_build_tail(tail_args a)
{
    const int32_t b = blockIdx.x;
    if (b < a.ntE)
        d_saddle_dof(b, a.nE, a.ecode, a.etiles, a.elem_edges, a.edge_row, a.red_row, a.S_rowptr,
                     a.S_col, a.elem_row, a.elem_red);
    else if (b < a.b1) d_c_tiles(b - a.ntE, a.L, a.C_rowptr, a.C_tile);
    else if (b < a.b2) d_neu_mask(b - a.b1, a.nE, a.ecode, a.neu_mask);
    else d_reduced_count(b - a.b2, a.nred, a.nE, a.ecode, a.nnzR);
}

struct build_tmp {
    int32_t* raw = nullptr;
    int32_t* bcount = nullptr;
    int32_t* boff = nullptr;
    uint64_t* keys = nullptr;
    int32_t* ucount = nullptr;
    int32_t* eoff = nullptr;
    int32_t* mark = nullptr;
    phf_cnt2* tiles = nullptr;
    phf_cnt2* tile_total = nullptr;
    int32_t* etiles = nullptr;
    int32_t* totals = nullptr;
    ~build_tmp()
    {
        phf_dfree(raw); phf_dfree(bcount); phf_dfree(boff); phf_dfree(keys);
        phf_dfree(ucount); phf_dfree(eoff); phf_dfree(mark); phf_dfree(tiles);
        phf_dfree(tile_total); phf_dfree(etiles); phf_dfree(totals);
    }
};

// The validation flags and, in the same synchronisation, `bytes` (at most 64)
// from device address d into h (through the context's pinned words).
int read_flags(phf_ctx* ctx, int* code, int* where, const void* d = nullptr, void* h = nullptr,
               size_t bytes = 0)
{
    int64_t* p = ctx->h_pinned;
    PHF_HIP(ctx, hipMemcpyAsync(p, ctx->d_flags, 2 * sizeof(int), hipMemcpyDeviceToHost,
                                ctx->stream));
    if (bytes)
        PHF_HIP(ctx, hipMemcpyAsync(p + 1, d, bytes, hipMemcpyDeviceToHost, ctx->stream));
    PHF_HIP(ctx, hipStreamSynchronize(ctx->stream));
    const int* f = reinterpret_cast<const int*>(p);
    *code = f[0];
    *where = f[1];
    if (bytes) memcpy(h, p + 1, bytes);
    return PHF_OK;
}

int flags_to_status(phf_ctx* ctx, int bits, int where, const char* stage)
{
    if (bits & FLAG_RANGE)
        return phf_set_error(ctx, PHF_EINVAL, "%s: element %d has a node index out of range",
                             stage, where);
    if (bits & FLAG_ORIENT)
        return phf_set_error(ctx, PHF_EORIENT,
                             "%s: element %d is clockwise, degenerate or has zero area", stage,
                             where);
    if (bits & FLAG_MESH)
        return phf_set_error(ctx, PHF_EMESH,
                             "%s: an edge of element %d is shared by more than two elements or "
                             "traversed in the same direction by both neighbours",
                             stage, where);
    if (bits & FLAG_BOUNDARY)
        return phf_set_error(ctx, PHF_EBOUNDARY,
                             "%s: boundary pair/edge %d is not a boundary edge, is listed twice "
                             "or a boundary edge is in neither list",
                             stage, where);
    return PHF_OK;
}

__global__ void k_flags_reset(int* flags)
{
    flags[0] = 0;
    flags[1] = 0x7fffffff;
}

int reset_flags(phf_ctx* ctx)
{
    PHF_LAUNCH(ctx, "k_flags_reset", k_flags_reset, 1, 1, 0, ctx->d_flags);
    return PHF_OK;
}

inline unsigned nblk(int64_t n) { return (unsigned)((n + 255) / 256); }

#define TRY(x)                 \
    do {                       \
        int rc_ = (x);         \
        if (rc_) return rc_;   \
    } while (0)

// Coordinates, elements, boundary pairs, edge tables and edge types of the
// red refinement of `P` (sizes already set in M), straight from P's tables.
int refined_tables(phf_mesh* M, const phf_mesh* P, build_tmp* T, int32_t* ne_out)
{
    phf_ctx* ctx = M->ctx;
    const int32_t ne_c = P->n_edges, nC_c = P->nC, nE_c = P->nE;
    const int32_t nE = M->nE, nD = M->nD, nN = M->nN;
    const int32_t ne = 2 * ne_c + 3 * nE_c;
    TRY(phf_dmalloc(ctx, &M->xy, M->nC, "coordinates"));
    TRY(phf_dmalloc(ctx, &M->elem4, nE, "elements"));
    TRY(phf_dmalloc(ctx, &M->exy, 3 * (size_t)nE, "element coordinates"));
    TRY(phf_dmalloc(ctx, &M->dir_pairs, nD, "Dirichlet pairs"));
    TRY(phf_dmalloc(ctx, &M->neu_pairs, nN, "Neumann pairs"));
    TRY(phf_dmalloc(ctx, &T->ucount, (size_t)ne_c + 1, "group size prefixes"));
    TRY(phf_dmalloc(ctx, &T->eoff, (size_t)nblk(ne_c) + 1, "group tile sums"));
    {
        refine_a_args a{};
        a.nC_c = nC_c;
        a.ne_c = ne_c;
        a.nE_c = nE_c;
        a.nD_c = P->nD;
        a.nN_c = P->nN;
        a.b1 = (int32_t)nblk((int64_t)M->nC);
        a.b2 = a.b1 + (int32_t)nblk(nE_c);
        a.b3 = a.b2 + (int32_t)nblk(P->nD);
        a.b4 = a.b3 + (int32_t)nblk(P->nN);
        a.xy_c = P->xy;
        a.edge_nodes_c = P->edge_nodes;
        a.xy_f = M->xy;
        a.elem4_c = P->elem4;
        a.elem_edges_c = P->elem_edges;
        a.exy_c = P->exy;
        a.elem4_f = M->elem4;
        a.exy_f = M->exy;
        a.dir_pairs_c = P->dir_pairs;
        a.neu_pairs_c = P->neu_pairs;
        a.dir_edges_c = P->dir_edges;
        a.neu_edges_c = P->neu_edges;
        a.dir_pairs_f = M->dir_pairs;
        a.neu_pairs_f = M->neu_pairs;
        a.edge_elems_c = P->edge_elems;
        a.led_c = P->led;
        a.ledTN_c = P->ledTN;
        a.ucount = T->ucount;
        a.utiles = T->eoff;
        PHF_LAUNCH(ctx, "k_refine_a", k_refine_a, a.b4 + (int32_t)nblk(ne_c), 256, 0, a);
    }
    // edge groups per parent edge: exclusive scan of the tile sums
    PHF_LAUNCH(ctx, "k_tile_scan1", k_tile_scan1, 1, 1024, 0, (int32_t)nblk(ne_c), T->eoff);
    M->n_edges = ne;
    TRY(phf_dmalloc(ctx, &M->edge_nodes, ne, "edge nodes"));
    TRY(phf_dmalloc(ctx, &M->edge_elems, ne, "edge elements"));
    TRY(phf_dmalloc(ctx, &M->elem_edges, 3 * (size_t)nE, "element edges"));
    TRY(phf_dmalloc(ctx, &M->led, ne, "led"));
    TRY(phf_dmalloc(ctx, &M->ledTN, ne, "ledTN"));
    TRY(phf_dmalloc(ctx, &M->edge_type, ne, "edge types"));
    TRY(phf_dmalloc(ctx, &M->dir_edges, nD, "Dirichlet edges"));
    TRY(phf_dmalloc(ctx, &M->neu_edges, nN, "Neumann edges"));
    {
        refine_b_args a{};
        a.ne_c = ne_c;
        a.nC_c = nC_c;
        a.nE_c = nE_c;
        a.nD_c = P->nD;
        a.nN_c = P->nN;
        a.b1 = (int32_t)nblk(ne_c);
        a.b2 = a.b1 + (int32_t)nblk(P->nD);
        a.edge_nodes_c = P->edge_nodes;
        a.edge_elems_c = P->edge_elems;
        a.led_c = P->led;
        a.ledTN_c = P->ledTN;
        a.etype_c = P->edge_type;
        a.elem_edges_c = P->elem_edges;
        a.elem4_c = P->elem4;
        a.pre = T->ucount;
        a.tiles = T->eoff;
        a.edge_nodes = M->edge_nodes;
        a.edge_elems = M->edge_elems;
        a.elem_edges = M->elem_edges;
        a.led = M->led;
        a.ledTN = M->ledTN;
        a.etype = M->edge_type;
        a.dir_pairs_c = P->dir_pairs;
        a.neu_pairs_c = P->neu_pairs;
        a.dir_edges_c = P->dir_edges;
        a.neu_edges_c = P->neu_edges;
        a.dir_edges = M->dir_edges;
        a.neu_edges = M->neu_edges;
        PHF_LAUNCH(ctx, "k_refine_b", k_refine_b, a.b2 + (int32_t)nblk(P->nN), 256, 0, a);
    }
    phf_dfree(T->ucount);
    phf_dfree(T->eoff);
    *ne_out = ne;
    return PHF_OK;
}

// `parent`: the mesh this one is the red refinement of, or null. A refinement
// of a valid mesh is valid, and its edge and boundary counts follow from the
// parent's, so that path skips the validation read-backs.
int mesh_build(phf_mesh* M, const double* xy, const int32_t* elem, const int32_t* dir,
               const int32_t* neu, phf_memspace ms, const phf_mesh* parent)
{
    phf_ctx* ctx = M->ctx;
    build_tmp T;
    const int32_t nC = M->nC, nE = M->nE, nD = M->nD, nN = M->nN;
    hipMemcpyKind kind = ms == PHF_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice;
    int bits = 0, where = 0;

    int32_t ne = 0;
    if (parent) {
        TRY(refined_tables(M, parent, &T, &ne));
    } else {
        TRY(phf_dmalloc(ctx, &M->xy, nC, "coordinates"));
        TRY(phf_dmalloc(ctx, &M->elem4, nE, "elements"));
        TRY(phf_dmalloc(ctx, &T.raw, 3 * (size_t)nE, "element input"));
        TRY(phf_dmalloc(ctx, &T.bcount, (size_t)nC + 1, "bucket counts"));
        TRY(phf_dmalloc(ctx, &T.boff, (size_t)nC + 1, "bucket offsets"));
        TRY(phf_dmalloc(ctx, &T.totals, 8, "totals"));
        PHF_HIP(ctx, hipMemcpyAsync(M->xy, xy, sizeof(double2) * nC, kind, ctx->stream));
        PHF_HIP(ctx, hipMemcpyAsync(T.raw, elem, sizeof(int32_t) * 3 * (size_t)nE, kind, ctx->stream));
        PHF_HIP(ctx, hipMemsetAsync(T.bcount, 0, sizeof(int32_t) * ((size_t)nC + 1), ctx->stream));
        TRY(reset_flags(ctx));

        // a1: validation + bucket counts by larger node
        PHF_LAUNCH(ctx, "k_elem_init", k_elem_init, nblk(nE), 256, 0, T.raw, nE, nC, M->xy, M->elem4,
                   T.bcount, ctx->d_flags);
        TRY(read_flags(ctx, &bits, &where));
        TRY(flags_to_status(ctx, bits, where, "validation"));
        phf_dfree(T.raw);

        // a2: counting sort of directed edges, per-bucket sort, unique count
        TRY(phf_scan_i32(ctx, T.bcount, T.boff, nC + 1, nullptr));
        TRY(phf_dmalloc(ctx, &T.keys, 3 * (size_t)nE, "edge keys"));
        PHF_HIP(ctx, hipMemsetAsync(T.bcount, 0, sizeof(int32_t) * ((size_t)nC + 1), ctx->stream));
        PHF_LAUNCH(ctx, "k_fill", k_fill, nblk(nE), 256, 0, M->elem4, nE, T.boff, T.bcount, T.keys);
        TRY(phf_dmalloc(ctx, &T.ucount, (size_t)nC + 1, "unique counts"));
        TRY(phf_dmalloc(ctx, &T.eoff, (size_t)nC + 1, "edge offsets"));
        PHF_LAUNCH(ctx, "k_bucket_sort", k_bucket_sort, nblk(nC), 256, 0, T.keys, T.boff, nC,
                   M->elem4, T.ucount, ctx->d_flags);
        // (the scan only reads the bucket counts, which stay in range even
        // when the topology check fails; the edge count comes back with the
        // flags)
        PHF_HIP(ctx, hipMemsetAsync(T.ucount + nC, 0, sizeof(int32_t), ctx->stream));
        TRY(phf_scan_i32(ctx, T.ucount, T.eoff, nC + 1, T.totals));
        TRY(read_flags(ctx, &bits, &where, T.totals, &ne, sizeof(int32_t)));
        TRY(flags_to_status(ctx, bits, where, "topology"));
        M->n_edges = ne;
        TRY(phf_dmalloc(ctx, &M->edge_nodes, ne, "edge nodes"));
        TRY(phf_dmalloc(ctx, &M->edge_elems, ne, "edge elements"));
        TRY(phf_dmalloc(ctx, &M->elem_edges, 3 * (size_t)nE, "element edges"));
        TRY(phf_dmalloc(ctx, &M->led, ne, "led"));
        TRY(phf_dmalloc(ctx, &M->ledTN, ne, "ledTN"));
        PHF_LAUNCH(ctx, "k_emit", k_emit, nblk(nC), 256, 0, T.keys, T.boff, T.eoff, nC, M->elem4,
                   M->edge_nodes, M->edge_elems, M->elem_edges, M->led, M->ledTN);
        phf_dfree(T.keys);
        phf_dfree(T.bcount);
        phf_dfree(T.boff);
        phf_dfree(T.ucount);

        // a3: boundary classification
        TRY(phf_dmalloc(ctx, &M->edge_type, ne, "edge types"));
        TRY(phf_dmalloc(ctx, &M->dir_edges, nD, "Dirichlet edges"));
        TRY(phf_dmalloc(ctx, &M->neu_edges, nN, "Neumann edges"));
        TRY(phf_dmalloc(ctx, &T.mark, ne, "edge marks"));
        TRY(phf_dmalloc(ctx, &M->dir_pairs, nD, "Dirichlet pairs"));
        TRY(phf_dmalloc(ctx, &M->neu_pairs, nN, "Neumann pairs"));
        if (nD) PHF_HIP(ctx, hipMemcpyAsync(M->dir_pairs, dir, sizeof(int32_t) * 2 * (size_t)nD, kind, ctx->stream));
        if (nN) PHF_HIP(ctx, hipMemcpyAsync(M->neu_pairs, neu, sizeof(int32_t) * 2 * (size_t)nN, kind, ctx->stream));
        PHF_HIP(ctx, hipMemsetAsync(M->edge_type, 0, ne, ctx->stream));
        PHF_HIP(ctx, hipMemsetAsync(T.mark, 0, sizeof(int32_t) * ne, ctx->stream));
        TRY(reset_flags(ctx));
        if (nD + nN > 0)
            PHF_LAUNCH(ctx, "k_boundary_mark", k_boundary_mark, nblk(nD + nN), 256, 0,
                       (const int32_t*)M->dir_pairs, nD, (const int32_t*)M->neu_pairs, nN, nC, T.eoff, M->edge_nodes, M->edge_elems, T.mark, M->edge_type,
                       M->dir_edges, M->neu_edges, ctx->d_flags);
    }
    // a3: multiplier rows, free rows and C row pointers from the numbers of
    // Dirichlet and Neumann edges before each edge (per-tile counts, their
    // exclusive scan, then per-edge ballots inside the tile). The element
    // codes and their per-tile Neumann incidences (for the saddle pattern:
    // the DOF rows of element m start at 15 m - 2 (incidences before m)) go in
    // the same launches.
    const int32_t nt = (ne + 255) / 256, ntE = (nE + 255) / 256;
    TRY(phf_dmalloc(ctx, &T.tiles, (size_t)nt, "row tile counts"));
    TRY(phf_dmalloc(ctx, &T.tile_total, 1, "row totals"));
    TRY(phf_dmalloc(ctx, &T.etiles, (size_t)ntE, "element tile counts"));
    if (!parent) TRY(phf_dmalloc(ctx, &M->exy, 3 * (size_t)nE, "element coordinates"));
    TRY(phf_dmalloc(ctx, &M->ecode, nE, "element codes"));
    {
        counts_args a{};
        a.ne = ne;
        a.nE = nE;
        a.nt = nt;
        a.etype = M->edge_type;
        a.edge_elems = M->edge_elems;
        a.mark = parent ? nullptr : T.mark;
        a.tiles = T.tiles;
        a.flags = ctx->d_flags;
        a.elem4 = M->elem4;
        a.elem_edges = M->elem_edges;
        a.ecode_c = parent ? parent->ecode : nullptr;
        a.nE_c = parent ? parent->nE : 0;
        a.xy = parent ? nullptr : M->xy;  // refined: built with the children
        a.exy = M->exy;
        a.ecode = M->ecode;
        a.etiles = T.etiles;
        PHF_LAUNCH(ctx, "k_counts", k_counts, nt + ntE, 256, 0, a);
    }
    phf_dfree(T.eoff);
    phf_dfree(T.mark);
    PHF_LAUNCH(ctx, "k_tile_scans", k_tile_scans, 2, 1024, 0, nt, T.tiles, T.tile_total, ntE,
               T.etiles);
    phf_cnt2 cnt{nD, nN};
    if (!parent) {
        // boundary check and the boundary edge counts in one read-back (the
        // tile scans only read the counts); every boundary edge of a refined
        // mesh is listed exactly once: the parent was checked
        TRY(read_flags(ctx, &bits, &where, T.tile_total, &cnt, sizeof(cnt)));
        TRY(flags_to_status(ctx, bits, where, "boundary"));
    }
    M->L = ne - cnt.n;                          // multiplier rows
    M->n_free = ne - cnt.d;                     // free edges
    M->n_int = ne - cnt.d - cnt.n;              // interior edges
    M->nnz_C = 4 * M->n_int + 2 * cnt.d;        // C entries
    const int32_t L = M->L, N = 3 * nE;
    if ((int64_t)9 * nE + 2 * M->nnz_C > 0x7fffffffLL)
        return phf_set_error(ctx, PHF_EINVAL, "saddle matrix too large for int32 indices");
    M->nnz_S = (int64_t)9 * nE + 2 * M->nnz_C;
    const int32_t nnz_dof = 9 * nE + M->nnz_C;  // entries of the saddle DOF rows

    TRY(phf_dmalloc(ctx, &M->edge_row, ne, "edge rows"));
    TRY(phf_dmalloc(ctx, &M->red_row, ne, "reduced rows"));
    TRY(phf_dmalloc(ctx, &M->red_edge, M->n_free, "reduced edges"));
    TRY(phf_dmalloc(ctx, &M->row_edge, L, "row edges"));
    TRY(phf_dmalloc(ctx, &M->row_nodes, L, "row nodes"));
    TRY(phf_dmalloc(ctx, &M->row_hs, L, "row half-lengths"));
    TRY(phf_dmalloc(ctx, &M->C_rowptr, (size_t)L + 1, "C rowptr"));
    TRY(phf_dmalloc(ctx, &M->C_col, M->nnz_C, "C columns"));
    TRY(phf_dmalloc(ctx, &M->S_rowptr, (size_t)N + L + 1, "saddle rowptr"));
    TRY(phf_dmalloc(ctx, &M->S_col, M->nnz_S, "saddle columns"));
    {
        rows_args a{};
        a.ne = ne;
        a.L = L;
        a.nnzC = (int32_t)M->nnz_C;
        a.nnz_dof = nnz_dof;
        a.etype = M->edge_type;
        a.tiles = T.tiles;
        a.edge_nodes = M->edge_nodes;
        a.edge_elems = M->edge_elems;
        a.led = M->led;
        a.ledTN = M->ledTN;
        a.edge_row = M->edge_row;
        a.red_row = M->red_row;
        a.red_edge = M->red_edge;
        a.row_edge = M->row_edge;
        a.row_nodes = M->row_nodes;
        a.xy = M->xy;
        a.row_hs = M->row_hs;
        a.C_rowptr = M->C_rowptr;
        a.C_col = M->C_col;
        a.S_rowptr_m = M->S_rowptr + N;
        a.S_col_m = M->S_col + nnz_dof;
        PHF_LAUNCH(ctx, "k_rows", k_rows, nt, 256, 0, a);
    }
    phf_dfree(T.tiles);

    // saddle DOF rows, tile bases of the C row pointers, the Neumann element
    // mask and the size of the reduced operator (read when the mesh info is
    // asked for)
    const int32_t nf = M->n_free;
    TRY(phf_dmalloc(ctx, &M->C_tile, (size_t)(L + 255) / 256 + 1, "C tile bases"));
    TRY(phf_dmalloc(ctx, &M->neu_mask, ((size_t)nE + 63) / 64, "Neumann element mask"));
    TRY(phf_dmalloc(ctx, &M->d_nnzR, 1, "reduced count"));
    TRY(phf_dmalloc(ctx, &M->elem_row, (size_t)N, "element multiplier rows"));
    TRY(phf_dmalloc(ctx, &M->elem_red, (size_t)N, "element reduced rows"));
    PHF_HIP(ctx, hipMemsetAsync(M->d_nnzR, 0, sizeof(unsigned long long), ctx->stream));
    {
        tail_args a{};
        a.nE = nE;
        a.L = L;
        a.ntE = ntE;
        a.b1 = ntE + (int32_t)nblk((L + 255) / 256 + 1);
        a.b2 = a.b1 + (int32_t)nblk(nE);
        a.nred = (int32_t)std::min<int64_t>(nblk(nE), 1024);
        a.ecode = M->ecode;
        a.etiles = T.etiles;
        a.elem_edges = M->elem_edges;
        a.edge_row = M->edge_row;
        a.red_row = M->red_row;
        a.elem_row = M->elem_row;
        a.elem_red = M->elem_red;
        a.C_rowptr = M->C_rowptr;
        a.S_rowptr = M->S_rowptr;
        a.S_col = M->S_col;
        a.C_tile = M->C_tile;
        a.neu_mask = M->neu_mask;
        a.nnzR = M->d_nnzR;
        PHF_LAUNCH(ctx, "k_build_tail", k_build_tail, a.b2 + a.nred, 256, 0, a);
    }
    phf_dfree(T.etiles);
    M->nnz_R = -1;
    // later work on the mesh runs in stream order behind these kernels (the
    // caller's input arrays were consumed before the first read-back)
    M->bytes = (int64_t)nC * 16 + (int64_t)nE * (16 + 48 + 4 + 24) + (int64_t)ne * (8 + 8 + 1 + 1 + 1 + 4 + 4) +
               (int64_t)nE * 12 + (int64_t)(nD + nN) * 4 + (int64_t)L * (4 + 8 + 4) +
               M->nnz_C * 4 + ((int64_t)N + L + 1) * 4 + M->nnz_S * 4 + (int64_t)nf * 8;
    return PHF_OK;
}
}  // namespace

namespace {
int mesh_create(phf_ctx* ctx, const double* xy, int32_t nC, const int32_t* elem, int32_t nE,
                const int32_t* dir, int32_t nD, const int32_t* neu, int32_t nN, phf_memspace ms,
                const phf_mesh* parent, phf_mesh** out)
{
    PHF_HIP(ctx, hipSetDevice(ctx->device));
    phf_mesh* M = new (std::nothrow) phf_mesh;
    if (!M) return phf_set_error(ctx, PHF_ENOMEM, "host allocation failed");
    M->ctx = ctx;
    M->nC = nC;
    M->nE = nE;
    M->nD = nD;
    M->nN = nN;
    int rc = mesh_build(M, xy, elem, dir, neu, ms, parent);
    if (rc) {
        (void)hipStreamSynchronize(ctx->stream);
        mesh_free(M);
        delete M;
        return rc;
    }
    ctx->n_objects++;
    *out = M;
    return PHF_OK;
}
}  // namespace

extern "C" int phf_mesh_create(phf_ctx* ctx, const double* xy, int32_t nC, const int32_t* elem,
                               int32_t nE, const int32_t* dir, int32_t nD, const int32_t* neu,
                               int32_t nN, phf_memspace ms, phf_mesh** out)
{
    if (!ctx || !out) return PHF_EINVAL;
    *out = nullptr;
    if (nC < 3 || nE < 1 || nE > 80000000 || nD < 0 || nN < 0 || !xy || !elem ||
        (nD > 0 && !dir) || (nN > 0 && !neu) || (ms != PHF_HOST && ms != PHF_DEVICE))
        return phf_set_error(ctx, PHF_EINVAL, "phf_mesh_create: invalid sizes or null arrays");
    return mesh_create(ctx, xy, nC, elem, nE, dir, nD, neu, nN, ms, nullptr, out);
}

extern "C" int phf_mesh_destroy(phf_mesh* mesh)
{
    if (!mesh) return PHF_EINVAL;
    if (mesh->n_children > 0 || mesh->n_users > 0)
        return phf_set_error(mesh->ctx, PHF_ESTATE,
                             "phf_mesh_destroy: %d refined meshes and %d steppers or batches "
                             "still refer to this mesh",
                             mesh->n_children, mesh->n_users);
    (void)hipStreamSynchronize(mesh->ctx->stream);
    if (mesh->parent) mesh->parent->n_children--;
    mesh->ctx->n_objects--;
    mesh_free(mesh);
    delete mesh;
    return PHF_OK;
}

// ---------------------------------------------------------------------------
// uniform red refinement (Section 2.3, Listing 4); the kernels are with the
// refined-mesh tables above
// ---------------------------------------------------------------------------

extern "C" int phf_mesh_refine(phf_mesh* coarse, phf_mesh** out)
{
    if (!coarse || !out) return PHF_EINVAL;
    *out = nullptr;
    phf_ctx* ctx = coarse->ctx;
    const int64_t nCf = (int64_t)coarse->nC + coarse->n_edges, nEf = 4 * (int64_t)coarse->nE;
    if (nCf > 0x7fffffffLL || nEf > 80000000LL)
        return phf_set_error(ctx, PHF_EINVAL, "phf_mesh_refine: refined mesh too large");
    // every table of the refined mesh is built on the device from the parent's
    TRY(mesh_create(ctx, nullptr, (int32_t)nCf, nullptr, (int32_t)nEf, nullptr, 2 * coarse->nD,
                    nullptr, 2 * coarse->nN, PHF_DEVICE, coarse, out));
    (*out)->parent = coarse;
    coarse->n_children++;
    return PHF_OK;
}

extern "C" int phf_mesh_get_info(const phf_mesh* m, phf_mesh_info* o)
{
    if (!m || !o) return PHF_EINVAL;
    if (m->nnz_R < 0) {
        // counted on the device during the build; read once (waits for it)
        unsigned long long v = 0;
        phf_mesh* mm = const_cast<phf_mesh*>(m);
        PHF_HIP(mm->ctx, hipMemcpyAsync(&v, m->d_nnzR, sizeof(v), hipMemcpyDeviceToHost,
                                        mm->ctx->stream));
        PHF_HIP(mm->ctx, hipStreamSynchronize(mm->ctx->stream));
        mm->nnz_R = (int64_t)v + m->n_free;  // the diagonal of every free row
    }
    o->nC = m->nC;
    o->nE = m->nE;
    o->n_edges = m->n_edges;
    o->N = 3 * m->nE;
    o->L = m->L;
    o->nD = m->nD;
    o->nN = m->nN;
    o->n_interior = m->n_int;
    o->n_free = m->n_free;
    o->nnz_K = 9 * (int64_t)m->nE;
    o->nnz_C = m->nnz_C;
    o->nnz_saddle = m->nnz_S;
    o->nnz_reduced = m->nnz_R;
    o->device_bytes = m->bytes;
    return PHF_OK;
}

namespace {
__global__ void k_split_pairs(const int2* __restrict__ in, int32_t n, int32_t* __restrict__ out)
{
    int32_t q = blockIdx.x * 256 + threadIdx.x;
    if (q >= n) return;
    int2 v = in[q];
    out[2 * (int64_t)q] = v.x;
    out[2 * (int64_t)q + 1] = v.y;
}

__global__ void k_k_pattern(int32_t nE, int32_t* __restrict__ rowptr, int32_t* __restrict__ col)
{
    int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x;
    int64_t N = 3 * (int64_t)nE;
    if (g > N) return;
    if (rowptr) rowptr[g] = (int32_t)(3 * g);
    if (g < N && col) {
        int32_t m = (int32_t)(g / 3);
        col[3 * g] = 3 * m;
        col[3 * g + 1] = 3 * m + 1;
        col[3 * g + 2] = 3 * m + 2;
    }
}

int copy_out(phf_ctx* ctx, void* dst, const void* src, size_t bytes, phf_memspace ms)
{
    if (!dst || bytes == 0) return PHF_OK;
    PHF_HIP(ctx, hipMemcpyAsync(dst, src, bytes,
                                ms == PHF_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice,
                                ctx->stream));
    return PHF_OK;
}
}  // namespace

extern "C" int phf_mesh_topology(const phf_mesh* m, int32_t* edge_nodes, int32_t* edge_elems,
                                 int32_t* elem_edges, int8_t* led, int8_t* ledTN,
                                 int8_t* edge_type, int32_t* edge_row, int32_t* dir_edges,
                                 int32_t* neu_edges, phf_memspace ms)
{
    if (!m || (ms != PHF_HOST && ms != PHF_DEVICE)) return PHF_EINVAL;
    phf_ctx* ctx = m->ctx;
    size_t ne = (size_t)m->n_edges;
    // int2 arrays are laid out as interleaved pairs already
    TRY(copy_out(ctx, edge_nodes, m->edge_nodes, ne * 8, ms));
    TRY(copy_out(ctx, edge_elems, m->edge_elems, ne * 8, ms));
    TRY(copy_out(ctx, elem_edges, m->elem_edges, (size_t)m->nE * 12, ms));
    TRY(copy_out(ctx, led, m->led, ne, ms));
    TRY(copy_out(ctx, ledTN, m->ledTN, ne, ms));
    TRY(copy_out(ctx, edge_type, m->edge_type, ne, ms));
    TRY(copy_out(ctx, edge_row, m->edge_row, ne * 4, ms));
    TRY(copy_out(ctx, dir_edges, m->dir_edges, (size_t)m->nD * 4, ms));
    TRY(copy_out(ctx, neu_edges, m->neu_edges, (size_t)m->nN * 4, ms));
    if (ms == PHF_HOST) PHF_HIP(ctx, hipStreamSynchronize(ctx->stream));
    return PHF_OK;
}

namespace {
__global__ __launch_bounds__(256) void k_elem_xyz(int32_t nE, const int4* __restrict__ elem4,
                                                  int32_t* __restrict__ out)
{
    const int32_t m = blockIdx.x * 256 + threadIdx.x;
    if (m >= nE) return;
    const int4 e = elem4[m];
    out[3 * (int64_t)m] = e.x;
    out[3 * (int64_t)m + 1] = e.y;
    out[3 * (int64_t)m + 2] = e.z;
}
}  // namespace

extern "C" int phf_mesh_geometry(const phf_mesh* m, double* xy, int32_t* elem, int32_t* dir,
                                 int32_t* neu, phf_memspace ms)
{
    if (!m || (ms != PHF_HOST && ms != PHF_DEVICE)) return PHF_EINVAL;
    phf_ctx* ctx = m->ctx;
    TRY(copy_out(ctx, xy, m->xy, (size_t)m->nC * 16, ms));
    if (elem) {
        int32_t* tmp = nullptr;
        if (ms == PHF_DEVICE) {
            tmp = elem;
        } else {
            TRY(phf_dmalloc(ctx, &tmp, 3 * (size_t)m->nE, "element copy"));
        }
        PHF_LAUNCH(ctx, "k_elem_xyz", k_elem_xyz, nblk(m->nE), 256, 0, m->nE, m->elem4, tmp);
        if (ms == PHF_HOST) {
            TRY(copy_out(ctx, elem, tmp, 12 * (size_t)m->nE, ms));
            PHF_HIP(ctx, hipStreamSynchronize(ctx->stream));
            phf_dfree(tmp);
        }
    }
    TRY(copy_out(ctx, dir, m->dir_pairs, (size_t)m->nD * 8, ms));
    TRY(copy_out(ctx, neu, m->neu_pairs, (size_t)m->nN * 8, ms));
    if (ms == PHF_HOST) PHF_HIP(ctx, hipStreamSynchronize(ctx->stream));
    return PHF_OK;
}

extern "C" int phf_mesh_pattern(const phf_mesh* m, int32_t* K_rowptr, int32_t* K_col,
                                int32_t* C_rowptr, int32_t* C_col, int32_t* S_rowptr,
                                int32_t* S_col, phf_memspace ms)
{
    if (!m || (ms != PHF_HOST && ms != PHF_DEVICE)) return PHF_EINVAL;
    phf_ctx* ctx = m->ctx;
    if (K_rowptr || K_col) {
        const int32_t N = 3 * m->nE;
        int32_t *rp = nullptr, *cl = nullptr;
        if (ms == PHF_DEVICE) {
            rp = K_rowptr;
            cl = K_col;
        } else {
            if (K_rowptr) TRY(phf_dmalloc(ctx, &rp, (size_t)N + 1, "K rowptr"));
            if (K_col) TRY(phf_dmalloc(ctx, &cl, 9 * (size_t)m->nE, "K columns"));
        }
        PHF_LAUNCH(ctx, "k_k_pattern", k_k_pattern, nblk((int64_t)N + 1), 256, 0, m->nE, rp, cl);
        if (ms == PHF_HOST) {
            if (K_rowptr) TRY(copy_out(ctx, K_rowptr, rp, ((size_t)N + 1) * 4, ms));
            if (K_col) TRY(copy_out(ctx, K_col, cl, 9 * (size_t)m->nE * 4, ms));
            PHF_HIP(ctx, hipStreamSynchronize(ctx->stream));
            phf_dfree(rp);
            phf_dfree(cl);
        }
    }
    TRY(copy_out(ctx, C_rowptr, m->C_rowptr, ((size_t)m->L + 1) * 4, ms));
    TRY(copy_out(ctx, C_col, m->C_col, (size_t)m->nnz_C * 4, ms));
    TRY(copy_out(ctx, S_rowptr, m->S_rowptr, (3 * (size_t)m->nE + m->L + 1) * 4, ms));
    TRY(copy_out(ctx, S_col, m->S_col, (size_t)m->nnz_S * 4, ms));
    if (ms == PHF_HOST) PHF_HIP(ctx, hipStreamSynchronize(ctx->stream));
    return PHF_OK;
}
