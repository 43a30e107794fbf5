// Multilevel (V-cycle) preconditioner over a chain of red-refined meshes; see
// phf_mg.h for the construction.
#include <algorithm>
#include <cmath>
#include <cstdio>

#include "phf_device.h"
#include "phf_mg.h"

namespace {

constexpr int NT = 256;
inline unsigned nblk(int64_t n) { return (unsigned)((n + NT - 1) / NT); }

#define TRY(x)               \
    do {                     \
        int rc_ = (x);       \
        if (rc_) return rc_; \
    } while (0)

// Parent of element m of a mesh refined from a coarse mesh with nEc elements.
__device__ inline int32_t parent_of(int32_t m, int32_t nEc)
{
    return m < nEc ? m : (m - nEc) / 3;
}


// Prolongation row of fine free edge rf: the coarse CR function at the fine
// edge midpoint, averaged over the (one or two) coarse triangles containing it.
// With psi_l = 1 - 2 lambda_l, the values at the fine midpoints are fixed by
// the red-refinement numbering (centre child p = [M0 M1 M2], corner child
// nEc + 3p + i = [v_i M_(i+2) M_(i+1)], local edge l opposite local vertex l):
//   - an edge of the centre child, local edge l, is parallel to coarse edge l
//     and has lambda = 1/2 at v_l and 1/4 at the other two vertices: psi = 0
//     on edge l, 1/2 on the other two;
//   - local edge l (1 or 2) of corner child i is the half of coarse edge
//     E = (i + l) mod 3 at v_i, lambda = 3/4 at v_i and 1/4 at the other end
//     of E: psi = 1 on E, -1/2 on edge i, 1/2 on the third edge.
// The fine edge's two triangles give the sides (a half of an interior coarse
// edge lies in two coarse triangles, weighted 1/2 each); columns are merged
// in side, then coarse-local-edge order.
__device__ inline void d_mg_prolong_build(int32_t rf, 
    int32_t nf_f, int32_t nEc, const int32_t* __restrict__ red_edge_f,
    const int2* __restrict__ edge_elems_f, const int8_t* __restrict__ led_f,
    const int8_t* __restrict__ ledTN_f, const int32_t* __restrict__ elem_red_c,
    int32_t* __restrict__ P_col, uint32_t* __restrict__ P_code)
{
    if (rf >= nf_f) return;
    const int32_t e = red_edge_f[rf];
    const int2 tt = edge_elems_f[e];
    const int32_t fine[2] = {tt.x, tt.y};
    const int lloc[2] = {led_f[e], tt.y >= 0 ? (int)ledTN_f[e] : 0};
    int32_t par[2] = {parent_of(tt.x, nEc), tt.y >= 0 ? parent_of(tt.y, nEc) : -1};
    if (par[1] == par[0]) par[1] = -1;
    const float scale = par[1] < 0 ? 1.0f : 0.5f;
    int32_t col[6];
    float val[6];
    int n = 0;
    for (int s = 0; s < 2; ++s) {
        const int32_t p = par[s];
        if (p < 0) continue;
        float w[3];
        const int l = lloc[s];
        if (fine[s] < nEc) {  // centre child: edge parallel to coarse edge l
            w[l] = 0.0f;
            w[(l + 1) % 3] = 0.5f;
            w[(l + 2) % 3] = 0.5f;
        } else {  // corner child i: half of coarse edge E at v_i
            const int i = (fine[s] - nEc) % 3;
            const int E = (i + l) % 3;
            w[E] = 1.0f;
            w[i] = -0.5f;
            w[3 - E - i] = 0.5f;
        }
        for (int k = 0; k < 3; ++k) {
            if (w[k] == 0.0f) continue;
            const int32_t rc = elem_red_c[3 * (int64_t)p + k];
            if (rc < 0) continue;
            int q = 0;
            while (q < n && col[q] != rc) ++q;
            if (q == n) {
                col[n] = rc;
                val[n] = 0.0f;
                ++n;
            }
            val[q] += scale * w[k];
        }
    }
    // every weight is a multiple of 1/4 in [-1, 1]: four bits per slot
    uint32_t code = 0;
    for (int k = 0; k < 5; ++k) {
        const int64_t slot = (int64_t)k * nf_f + rf;
        P_col[slot] = k < n ? col[k] : 0;
        code |= (uint32_t)((int)((k < n ? val[k] : 0.0f) * 4.0f) + 4) << (4 * k);
    }
    P_code[rf] = code;
}

// Weight of slot k of a prolongation row from its code (exact).
__device__ inline float prolong_weight(uint32_t code, int k)
{
    return (float)((int)((code >> (4 * k)) & 15u) - 4) * 0.25f;
}

// Fine rows of the nine fine edges inside coarse triangle p (-1 where the
// fine edge is Dirichlet), stored slot-major (slot k at k * nEc + p):
//   slot j      (j < 3) edge of the centre child parallel to coarse edge j;
//   slot 3 + 2i         half of coarse edge i+1 at vertex v_i;
//   slot 4 + 2i         half of coarse edge i+2 at vertex v_i.
// The centre child of p is element p = [M0 M1 M2], corner child i is
// nEc + 3p + i = [v_i M_(i+2) M_(i+1)] (M_j the midpoint of coarse edge j).
__device__ inline void d_mg_rows9(int32_t p, int32_t nEc, const int32_t* __restrict__ elem_red_f,
                                  int32_t* __restrict__ rows9)
{
    if (p >= nEc) return;
    for (int j = 0; j < 3; ++j) rows9[(int64_t)j * nEc + p] = elem_red_f[3 * (int64_t)p + j];
    for (int i = 0; i < 3; ++i) {
        const int64_t ch = (int64_t)nEc + 3 * (int64_t)p + i;
        rows9[(int64_t)(3 + 2 * i) * nEc + p] = elem_red_f[3 * ch + 1];
        rows9[(int64_t)(4 + 2 * i) * nEc + p] = elem_red_f[3 * ch + 2];
    }
}

// For coarse free row c: positions in the per-triangle restriction sums of
// its edge seen from T+ and from T- (-1 on the boundary).
__device__ inline void d_mg_sel(int32_t c, int32_t nc, const int32_t* __restrict__ red_edge_c,
                                               const int2* __restrict__ edge_elems_c,
                                               const int8_t* __restrict__ led_c,
                                               const int8_t* __restrict__ ledTN_c,
                                               int2* __restrict__ sel)
{
    if (c >= nc) return;
    const int32_t e = red_edge_c[c];
    const int2 tt = edge_elems_c[e];
    sel[c] = make_int2(3 * tt.x + led_c[e], tt.y >= 0 ? 3 * tt.y + ledTN_c[e] : -1);
}

__global__ __launch_bounds__(NT) void k_mg_dense(int32_t n, const int32_t* __restrict__ col,
                                                 const double* __restrict__ val,
                                                 double* __restrict__ A)
{
    const int32_t r = blockIdx.x * NT + threadIdx.x;
    if (r >= n) return;
    for (int32_t j = 0; j < n; ++j) A[(int64_t)r * n + j] = 0.0;
    for (int k = 0; k < 5; ++k) {
        const int64_t slot = (int64_t)k * n + r;
        A[(int64_t)r * n + col[slot]] += val[slot];
    }
}

// In-place Gauss-Jordan inversion of an SPD matrix (no pivoting needed) by
// one workgroup: A (n x n) becomes its inverse; W is n x n scratch.
__global__ __launch_bounds__(1024) void k_mg_gj(int32_t n, double* __restrict__ A,
                                                double* __restrict__ W)
{
    const int tid = threadIdx.x, nth = blockDim.x;
    for (int64_t q = tid; q < (int64_t)n * n; q += nth) W[q] = ((q / n) == (q % n)) ? 1.0 : 0.0;
    __syncthreads();
    for (int32_t c = 0; c < n; ++c) {
        const double piv = A[(int64_t)c * n + c];
        __syncthreads();
        for (int32_t j = tid; j < n; j += nth) {
            A[(int64_t)c * n + j] /= piv;
            W[(int64_t)c * n + j] /= piv;
        }
        __syncthreads();
        for (int64_t q = tid; q < (int64_t)n * n; q += nth) {
            const int32_t i = (int32_t)(q / n), j = (int32_t)(q % n);
            if (i == c) continue;
            const double f = A[(int64_t)i * n + c];
            if (j != c) A[q] -= f * A[(int64_t)c * n + j];
            W[q] -= f * W[(int64_t)c * n + j];
        }
        __syncthreads();
        for (int32_t i = tid; i < n; i += nth)
            if (i != c) A[(int64_t)i * n + c] = 0.0;
        __syncthreads();
    }
    for (int64_t q = tid; q < (int64_t)n * n; q += nth) A[q] = W[q];
}

// Tables and vectors that a per-step kernel reads once and nothing reads
// again before they are rewritten (prolongation and restriction tables, the
// outer iteration's residual) are loaded non-temporally with PHF_NT_MG, so
// that they displace less of the operator rows and iterates that the next
// sweep reads again.
#ifndef PHF_NT_MG
#define PHF_NT_MG 1
#endif
template <bool NTL, typename P, typename I>
__device__ inline auto ldx(P p, I i) -> std::remove_cv_t<std::remove_reference_t<decltype(p[i])>>
{
    if constexpr (NTL) return __builtin_nontemporal_load(&p[i]);
    else return p[i];
}

// The per-row helpers take their pointers as template parameters, so that a
// caller can pass pointers typed as device memory or local data share and the
// compiler emits the matching (not flat) loads and stores.
template <typename T>
using gmem_ptr = __attribute__((address_space(1))) T*;

// Row r of a row-major ELL-4 array (four consecutive entries, 16-byte
// aligned) in one 16-byte load.
__device__ inline phf_i4 ld_row4(const int32_t* p, int32_t r) { return *(const phf_i4*)(p + 4 * (int64_t)r); }
__device__ inline phf_f4 ld_row4(const float* p, int32_t r) { return *(const phf_f4*)(p + 4 * (int64_t)r); }
__device__ inline phf_i4 ld_row4(gmem_ptr<const int32_t> p, int32_t r)
{
    return *(gmem_ptr<const phf_i4>)(p + 4 * (int64_t)r);
}
__device__ inline phf_f4 ld_row4(gmem_ptr<const float> p, int32_t r)
{
    return *(gmem_ptr<const phf_f4>)(p + 4 * (int64_t)r);
}

// The cycle's operator rows are scaled by the inverse diagonal: four
// off-diagonal entries of D^-1 A (ELL-4, row-major: the row's four columns,
// then in a second array its four values; unused entries hold column r and
// value 0) and an implicit unit diagonal; right-hand sides are kept as
// D^-1 b. sres is then the scaled residual D^-1 (b - A x) of row i.
template <typename PC, typename PV, typename PB, typename PX>
__device__ inline float sres(int32_t i, int32_t n, PC __restrict__ col, PV __restrict__ val,
                             PB __restrict__ bh, PX __restrict__ x)
{
    (void)n;
    const phf_i4 c = ld_row4(col, i);
    const phf_f4 v = ld_row4(val, i);
    float s = 0.0f;
    s = fmaf(v.x, x[c.x], s);
    s = fmaf(v.y, x[c.y], s);
    s = fmaf(v.z, x[c.z], s);
    s = fmaf(v.w, x[c.w], s);
    return bh[i] - x[i] - s;
}

// Per-row (per-triangle) steps of the cycle, shared by the one-launch-per-step
// kernels of the large levels and the single-workgroup kernel of the small
// ones, so both compute the same values.
__device__ inline void row_smooth(int32_t i, int32_t n, const int32_t* __restrict__ col,
                                  const float* __restrict__ val, const float* __restrict__ bh,
                                  float omega, const float* __restrict__ x, float* __restrict__ y)
{
    y[i] = x[i] + omega * sres(i, n, col, val, bh, x);
}

// Unscaled residual b - A x = D (D^-1 b - D^-1 A x).
template <typename PC, typename PV, typename PD, typename PB, typename PX, typename PR>
__device__ inline void row_resid(int32_t i, int32_t n, PC __restrict__ col, PV __restrict__ val,
                                 PD __restrict__ diag, PB __restrict__ bh, PX __restrict__ x,
                                 PR __restrict__ r)
{
    r[i] = diag[i] * sres(i, n, col, val, bh, x);
}

// Restriction, first half: for coarse triangle p and each of its edges l, the
// sum over the nine fine edges e inside p of s_e psi_l(m_e) r[e], where
// psi_l = 1 - 2 lambda_l is the coarse edge-midpoint basis function, m_e the
// fine edge midpoint and s_e = 1/2 on halves of a coarse edge shared with a
// second coarse triangle (the prolongation averages the two sides there), 1
// otherwise. The barycentric coordinates of the fine midpoints do not depend
// on the shape of p, so the weights are the constants below. rf must hold at
// least one element (the gathers read a clamped index, so that all nine row
// loads are issued before the first gather waits).
template <typename PT>
__device__ inline void tri_combine(int32_t p, int32_t code, const float (&v)[9], PT __restrict__ t)
{
    float s[3];
#pragma unroll
    for (int e = 0; e < 3; ++e) s[e] = PHF_CODE_TYPE(code, e) == 0 ? 0.5f : 1.0f;
    float acc[3];
#pragma unroll
    for (int l = 0; l < 3; ++l) {
        // centre edges: parallel to l -> 0, the other two -> 1/2
        float a = 0.5f * (v[(l + 1) % 3] + v[(l + 2) % 3]);
        // halves at vertex i of edge e: psi_e = 1, psi_i = -1/2, psi_(third) = 1/2
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            const int e1 = (i + 1) % 3, e2 = (i + 2) % 3;
            const float h1 = s[e1] * v[3 + 2 * i], h2 = s[e2] * v[4 + 2 * i];
            if (l == i) a += -0.5f * (h1 + h2);
            else if (l == e1) a += h1 + 0.5f * h2;
            else a += 0.5f * h1 + h2;
        }
        acc[l] = a;
    }
    t[3 * (int64_t)p] = acc[0];
    t[3 * (int64_t)p + 1] = acc[1];
    t[3 * (int64_t)p + 2] = acc[2];
}

template <bool NTL = false, typename PR9, typename PE, typename PF, typename PT>
__device__ inline void tri_restrict(int32_t p, int32_t nEc, PR9 __restrict__ rows9,
                                    PE __restrict__ ecode_c, PF __restrict__ rf,
                                    PT __restrict__ t)
{
    int32_t row[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) row[k] = ldx<NTL>(rows9, (int64_t)k * nEc + p);
    float v[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        const float g = rf[row[k] >= 0 ? row[k] : 0];
        v[k] = row[k] >= 0 ? g : 0.0f;
    }
    tri_combine(p, ldx<NTL>(ecode_c, p), v, t);
}

// Restriction, second half: coarse row c sums its edge's entries from T+ and
// T- (in that order), keeps the scaled right-hand side D^-1 b and takes the
// coarse level's first sweep from zero, x = omega D^-1 b.
// Entry c of a gather map, given as int2 or (in device memory) as int32 pairs.
__device__ inline int2 sel_at(const int2* __restrict__ sel, int32_t c) { return sel[c]; }
template <typename PS>
__device__ inline int2 sel_at(PS __restrict__ sel, int32_t c)
{
    return make_int2(sel[2 * c], sel[2 * c + 1]);
}

template <typename PS, typename PT, typename PD, typename PB, typename PX>
__device__ inline void row_collect(int32_t c, PS __restrict__ sel, PT __restrict__ t,
                                   PD __restrict__ dinv, float omega, PB __restrict__ bh,
                                   PX __restrict__ x)
{
    const int2 q = sel_at(sel, c);
    const float tx = t[q.x], ty = t[q.y >= 0 ? q.y : q.x];
    const float b = q.y >= 0 ? tx + ty : tx;
    const float h = b * dinv[c];
    bh[c] = h;
    x[c] = omega * h;
}

// Prolongation of row r: sum over its five slots of weight times the coarse
// value (unused slots: column 0, weight 0).
template <bool NTL = false, typename PC, typename PW, typename PX>
__device__ inline float prolong_sum(int32_t r, int32_t n, PC __restrict__ col, PW __restrict__ code,
                                    PX __restrict__ xc)
{
    const uint32_t c = ldx<NTL>(code, r);
    float s = 0.0f;
#pragma unroll
    for (int k = 0; k < 5; ++k)
        s = fmaf(prolong_weight(c, k), xc[ldx<NTL>(col, (int64_t)k * n + r)], s);
    return s;
}

__device__ inline void row_prolong(int32_t i, int32_t n, const int32_t* __restrict__ P_col,
                                   const uint32_t* __restrict__ P_code,
                                   const float* __restrict__ xc, float* __restrict__ x)
{
    x[i] += prolong_sum<PHF_NT_MG>(i, n, P_col, P_code, xc);
}

// Coarsest level: x = A^-1 b with b = D (D^-1 b).
template <typename PA, typename PD, typename PB, typename PX>
__device__ inline void row_coarse(int32_t i, int32_t n, PA __restrict__ Ainv, PD __restrict__ diag,
                                  PB __restrict__ bh, PX __restrict__ x)
{
    double s = 0.0;
    for (int32_t j = 0; j < n; ++j)
        s = fma(Ainv[(int64_t)i * n + j], (double)diag[j] * (double)bh[j], s);
    x[i] = (float)s;
}

// Element blocks of a coarse level's re-discretised operator,
// B_T = P^T (cK K_T + cM M_T) P with K_T = a_T |T| (A grad lambda_j) . grad
// lambda_i and the unit mass M_T = |T|/12 (1 + delta_ij) (Definition 3.1),
// straight from the element coordinates, written as the level's half-row
// records (phf_hrec_element; staged in LDS, stored as one run per tile).
// aT_f: the next finer level's triangle coefficient (null: 1); the level's
// own, the average over the four children, is written to aT.
__global__ __launch_bounds__(NT) void k_mg_cblocks(int32_t nE, const double2* __restrict__ exy,
                                                   const int32_t* __restrict__ elem_red,
                                                   const double* __restrict__ aT_f,
                                                   double* __restrict__ aT, double A00,
                                                   double A01, double A10, double A11, double cK,
                                                   double cM, phf_i4* __restrict__ rec)
{
    __shared__ __align__(16) phf_i4 srec[6 * NT];
    const int tid = threadIdx.x;
    const int64_t m0 = (int64_t)blockIdx.x * NT;
    const int32_t nt = (int32_t)min((int64_t)NT, (int64_t)nE - m0);
    if (tid < nt) {
        const int64_t m = m0 + tid;
        const double2 P0 = exy[3 * m], P1 = exy[3 * m + 1], P2 = exy[3 * m + 2];
        // g_i = 2|T| grad lambda_i (the edge opposite vertex i turned by 90 deg)
        const double gx[3] = {P1.y - P2.y, P2.y - P0.y, P0.y - P1.y};
        const double gy[3] = {P2.x - P1.x, P0.x - P2.x, P1.x - P0.x};
        const double det = (P1.x - P0.x) * (P2.y - P0.y) - (P2.x - P0.x) * (P1.y - P0.y);
        double a = 1.0;
        if (aT_f) {
            const int64_t c = nE + 3 * m;
            a = 0.25 * (aT_f[m] + aT_f[c] + aT_f[c + 1] + aT_f[c + 2]);
            aT[m] = a;
        }
        const double s = a / (2.0 * det);
        const double mass = det / 24.0;  // |T| / 12
        double A[9];
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            const double ax = A00 * gx[j] + A01 * gy[j], ay = A10 * gx[j] + A11 * gy[j];
#pragma unroll
            for (int i = 0; i < 3; ++i)
                A[3 * j + i] = cK * s * (ax * gx[i] + ay * gy[i]) + cM * mass * (i == j ? 2.0 : 1.0);
        }
        double Bm[9];
        phf_reduce_block(A, Bm);
        const int32_t red[3] = {elem_red[3 * m], elem_red[3 * m + 1], elem_red[3 * m + 2]};
        phf_hrec_element(srec, tid, red, Bm);
    }
    __syncthreads();
    for (int32_t q = tid; q < 6 * nt; q += NT) rec[6 * m0 + q] = srec[q];
}

// Coarse-level rows of the reduced operator: the five (column, value) slots
// of row r from its half-row records, scaled straight into the cycle's rows
// by phf_scale_row (off-diagonals of D^-1 A in ELL-4, the diagonal and its
// inverse); returns the row's Gershgorin sum. With col64 and val64 (the
// coarsest level) also the double-precision ELL-5 rows.
__device__ inline float d_mg_crows(int32_t r, int32_t nf, const int32_t* __restrict__ red_edge,
                                   const int2* __restrict__ edge_elems,
                                   const int8_t* __restrict__ led, const int8_t* __restrict__ ledTN,
                                   const phf_i4* __restrict__ rec,
                                   int32_t* __restrict__ col4, float* __restrict__ val4,
                                   float* __restrict__ diag, float* __restrict__ dinv,
                                   int32_t* __restrict__ col64, double* __restrict__ val64)
{
    if (r >= nf) return 0.0f;
    int32_t col[5];
    double v[5];
    const int32_t e = red_edge[r];
    phf_hrec_row(r, edge_elems[e], led[e], ledTN[e], rec, col, v);
    if (col64) {
#pragma unroll
        for (int k = 0; k < 5; ++k) {
            col64[(int64_t)k * nf + r] = col[k];
            val64[(int64_t)k * nf + r] = v[k];
        }
    }
    return phf_scale_row(r, nf, col, v, col4, val4, diag, dinv);
}

// Row order of the per-step kernels (phf_for_rows): XCD-contiguous chunks
// where the rows gather from neighbouring rows of the same vector.
constexpr bool XCD_SMOOTH = PHF_XCD_BITS & 1, XCD_RESID = PHF_XCD_BITS & 2,
               XCD_PROLONG = PHF_XCD_BITS & 4, XCD_RESTRICT = PHF_XCD_BITS & 8,
               XCD_COLLECT = PHF_XCD_BITS & 16, XCD_SMOOTHZ = PHF_XCD_BITS & 32;

// First sweep from x = 0 on the finest level: also rounds the right-hand side
// (the double-precision residual of the outer iteration) once, scaled.
__global__ __launch_bounds__(NT) void k_mg_smooth0_top(int32_t n, const float* __restrict__ dinv,
                                                       const double* __restrict__ b64,
                                                       const float* __restrict__ w,
                                                       float* __restrict__ bh,
                                                       float* __restrict__ x, const int* iflags)
{
    if (iflags && iflags[0]) return;
    const float omega = w[0];
    phf_for_rows<XCD_SMOOTH, NT>(n, [&](int32_t i) {
        const float h = (float)ldx<PHF_NT_MG>(b64, i) * dinv[i];
        bh[i] = h;
        if (x) x[i] = omega * h;
    });
}

// Second sweep on the finest level. The first one, from zero, is
// x = w[0] D^-1 b; it is formed here from D^-1 b where it is read (the same
// rounded product), so the first sweep need not store it. Same arithmetic as
// row_smooth.
__global__ __launch_bounds__(NT) void k_mg_smooth1_top(int32_t n, const int32_t* __restrict__ col,
                                                       const float* __restrict__ val,
                                                       const float* __restrict__ bh,
                                                       const float* __restrict__ w,
                                                       float* __restrict__ y, const int* iflags)
{
    if (iflags && iflags[0]) return;
    const float w0 = w[0], omega = w[1];
    phf_for_rows<XCD_SMOOTH, NT>(n, [&](int32_t i) {
        const phf_i4 c = ld_row4(col, i);
        const phf_f4 v = ld_row4(val, i);
        float s = 0.0f;
        s = fmaf(v.x, __fmul_rn(w0, bh[c.x]), s);
        s = fmaf(v.y, __fmul_rn(w0, bh[c.y]), s);
        s = fmaf(v.z, __fmul_rn(w0, bh[c.z]), s);
        s = fmaf(v.w, __fmul_rn(w0, bh[c.w]), s);
        const float bi = bh[i];
        float xi = __fmul_rn(w0, bi);
        // (opaque to the compiler, so that bi - xi is not contracted with the
        // product into one fused operation: the first sweep is a stored value)
        __asm__ volatile("" : "+v"(xi));
        y[i] = xi + omega * (bi - xi - s);
    });
}

// FINEST only separates the finest level's launches under their own symbol
// (profilers aggregate by symbol); the code is the same.
template <bool FINEST>
__global__ __launch_bounds__(NT) void k_mg_smooth(int32_t n, const int32_t* __restrict__ col,
                                                  const float* __restrict__ val,
                                                  const float* __restrict__ bh,
                                                  const float* __restrict__ w, int32_t k,
                                                  const float* __restrict__ x,
                                                  float* __restrict__ y, const int* iflags)
{
    if (iflags && iflags[0]) return;
    const float omega = w[k];
    phf_for_rows<XCD_SMOOTH, NT>(n, [&](int32_t i) { row_smooth(i, n, col, val, bh, omega, x, y); });
}

// Last sweep on the finest level, which also hands the cycle's result to the
// outer iteration: z = y (stored as ZT) and per-block partial sums of r.z
// (fixed order within the block; the grid is the outer iteration's).
template <typename ZT>
__global__ __launch_bounds__(NT) void k_mg_smooth_z(int32_t n, const int32_t* __restrict__ col,
                                                    const float* __restrict__ val,
                                                    const float* __restrict__ bh,
                                                    const float* __restrict__ w, int32_t k,
                                                    const float* __restrict__ x,
                                                    const double* __restrict__ r,
                                                    ZT* __restrict__ z,
                                                    double* __restrict__ part, const int* iflags)
{
    if (iflags && iflags[0]) return;
    __shared__ double sh[NT / 64];
    const float omega = w[k];
    double s = 0.0;
    phf_for_rows<XCD_SMOOTHZ, NT>(n, [&](int32_t i) {
        const float zi = x[i] + omega * sres(i, n, col, val, bh, x);
        z[i] = (ZT)zi;
        s = fma(ldx<PHF_NT_MG>(r, i), (double)zi, s);
    });
    const double t = phf_block_sum_f64<NT>(s, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = t;
}

__global__ __launch_bounds__(NT) void k_mg_resid(int32_t n, const int32_t* __restrict__ col,
                                                 const float* __restrict__ val,
                                                 const float* __restrict__ diag,
                                                 const float* __restrict__ bh,
                                                 const float* __restrict__ x,
                                                 float* __restrict__ r, const int* iflags)
{
    if (iflags && iflags[0]) return;
    phf_for_rows<XCD_RESID, NT>(n, [&](int32_t i) { row_resid(i, n, col, val, diag, bh, x, r); });
}

__global__ __launch_bounds__(NT) void k_mg_restrict(int32_t nEc, const int32_t* __restrict__ rows9,
                                                    const int32_t* __restrict__ ecode_c,
                                                    const float* __restrict__ rf,
                                                    float* __restrict__ t, const int* iflags)
{
    if (iflags && iflags[0]) return;
    phf_for_rows<XCD_RESTRICT, NT>(nEc, [&](int32_t p) { tri_restrict<PHF_NT_MG>(p, nEc, rows9, ecode_c, rf, t); });
}

__global__ __launch_bounds__(NT) void k_mg_collect(int32_t nc, const int2* __restrict__ sel,
                                                   const float* __restrict__ t,
                                                   const float* __restrict__ dinv,
                                                   const float* __restrict__ w, int32_t k,
                                                   float* __restrict__ bh, float* __restrict__ x,
                                                   const int* iflags)
{
    if (iflags && iflags[0]) return;
    const float omega = w[k];
    phf_for_rows<XCD_COLLECT, NT>(nc, [&](int32_t c) { row_collect(c, sel, t, dinv, omega, bh, x); });
}

__global__ __launch_bounds__(NT) void k_mg_prolong(int32_t n, const int32_t* __restrict__ P_col,
                                                   const uint32_t* __restrict__ P_code,
                                                   const float* __restrict__ xc,
                                                   float* __restrict__ x, const int* iflags)
{
    if (iflags && iflags[0]) return;
    phf_for_rows<XCD_PROLONG, NT>(n, [&](int32_t i) { row_prolong(i, n, P_col, P_code, xc, x); });
}

// On the levels whose launches are bound by latency rather than bytes, two
// pairs of steps run as one launch each; every value is the one the separate
// launches compute (the same expressions on the same operands), so the cycle
// is bit-identical either way.
// Residual and the restriction's first half: a lane per fine row of each
// coarse triangle (nine lanes per triangle, RR_TRI triangles per workgroup)
// forms the row's residual into LDS; lanes 0..RR_TRI-1 then combine one
// triangle's nine values each. Rows on an edge shared by two coarse triangles are formed
// twice; the residual vector is neither written nor read back. Workgroups
// are dealt to the XCDs in contiguous ranges of triangles, as the row
// kernels are.
constexpr int RR_TRI = NT / 9;
__global__ __launch_bounds__(NT) void k_mg_resid_restrict(
    int32_t nEc, const int32_t* __restrict__ rows9, const int32_t* __restrict__ ecode_c, int32_t n,
    const int32_t* __restrict__ col, const float* __restrict__ val, const float* __restrict__ diag,
    const float* __restrict__ bh, const float* __restrict__ x, float* __restrict__ t,
    const int* iflags)
{
    if (iflags && iflags[0]) return;
    __shared__ float sv[RR_TRI * 9];
    // block b takes tile (the XCD permutation of the blocks, one tile each)
    const int32_t nb = gridDim.x, b = blockIdx.x, xcd = b % 8, q = nb / 8, rem = nb % 8;
    const int32_t tile = xcd * q + min(xcd, rem) + b / 8;
    const int32_t lane = threadIdx.x, tl = lane / 9, k = lane - 9 * tl;
    const int32_t p0 = tile * RR_TRI;
    if (tl < RR_TRI && p0 + tl < nEc) {
        const int32_t row = ldx<PHF_NT_MG>(rows9, (int64_t)k * nEc + p0 + tl);
        float v = 0.0f;
        if (row >= 0)  // the product rounded on its own, as row_resid stores it
            v = __fmul_rn(diag[row], sres(row, n, col, val, bh, x));
        sv[lane] = v;
    }
    __syncthreads();
    const int32_t p = p0 + lane;
    if (lane < RR_TRI && p < nEc) {
        float v[9];
#pragma unroll
        for (int j = 0; j < 9; ++j) v[j] = sv[9 * lane + j];
        tri_combine(p, ldx<PHF_NT_MG>(ecode_c, p), v, t);
    }
}

// Prolongation and the first sweep after it: row i forms the corrected
// iterate x + P x_c at itself and at its four neighbours (each as row_prolong
// would store it) and takes the sweep from those values into y; the
// corrected iterate itself is not stored (the next sweep reads only y).
__global__ __launch_bounds__(NT) void k_mg_prolong_smooth(
    int32_t n, const int32_t* __restrict__ P_col, const uint32_t* __restrict__ P_code,
    const float* __restrict__ xc, const int32_t* __restrict__ col, const float* __restrict__ val,
    const float* __restrict__ bh, const float* __restrict__ w, int32_t k,
    const float* __restrict__ x, float* __restrict__ y, const int* iflags)
{
    if (iflags && iflags[0]) return;
    const float omega = w[k];
    phf_for_rows<XCD_SMOOTH, NT>(n, [&](int32_t i) {
        const auto xp = [&](int32_t j) {
            float u = x[j];
            u += prolong_sum<PHF_NT_MG>(j, n, P_col, P_code, xc);
            return u;
        };
        const phf_i4 c = ld_row4(col, i);
        const phf_f4 v = ld_row4(val, i);
        const float xi = xp(i);
        float s = 0.0f;
        s = fmaf(v.x, xp(c.x), s);
        s = fmaf(v.y, xp(c.y), s);
        s = fmaf(v.z, xp(c.z), s);
        s = fmaf(v.w, xp(c.w), s);
        y[i] = xi + omega * (bh[i] - xi - s);
    });
}

// The whole V-cycle on levels 0..top of the descriptor table in one
// workgroup: every step is a loop over its rows followed by a workgroup
// barrier. The levels' vectors (two iterates, D^-1 b, the restriction sums)
// live in the workgroup's local data share, so a step reads only its
// operator rows and transfer tables from memory; the residual of a level
// takes the iterate buffer that is free at that point. On entry the top
// level's D^-1 b and first sweep from zero are in memory (L.b and L.y; level
// 0: L.x), written by the restriction from the level above; lower levels
// receive theirs the same way inside the kernel. Every level then takes
// 2 nu - 1 more sweeps, an odd number; the coarsest level solves directly, or
// takes an even number of further sweeps (csweeps) from its first one. The top
// level's result is stored to L.x.
constexpr int TAIL_NT = 1024;
// The level descriptor as the single-workgroup kernel uses it: device-memory
// pointers typed as such, so that their loads are global (not flat) loads,
// whose counter is separate from the local data share's; a step can then
// issue all its memory loads before it waits for any.
struct tail_lv {
    int32_t n, nEc, sx, sy, sb, st;
    gmem_ptr<const int32_t> col;
    gmem_ptr<const float> val, diag, dinv;
    gmem_ptr<float> x;
    gmem_ptr<const float> y, b;
    gmem_ptr<const int32_t> P_col;
    gmem_ptr<const uint32_t> P_code;
    gmem_ptr<const int32_t> rows9, ecode_c;
    gmem_ptr<const int32_t> sel;  // int2 entries as int32 pairs
    gmem_ptr<const float> w;
};
__device__ inline tail_lv tail_level(const phf_mg_dev_level* __restrict__ lv, int32_t l)
{
    const phf_mg_dev_level& L = lv[l];
    return tail_lv{L.n,
                   L.nEc,
                   L.sx,
                   L.sy,
                   L.sb,
                   L.st,
                   (gmem_ptr<const int32_t>)L.col,
                   (gmem_ptr<const float>)L.val,
                   (gmem_ptr<const float>)L.diag,
                   (gmem_ptr<const float>)L.dinv,
                   (gmem_ptr<float>)L.x,
                   (gmem_ptr<const float>)L.y,
                   (gmem_ptr<const float>)L.b,
                   (gmem_ptr<const int32_t>)L.P_col,
                   (gmem_ptr<const uint32_t>)L.P_code,
                   (gmem_ptr<const int32_t>)L.rows9,
                   (gmem_ptr<const int32_t>)L.ecode_c,
                   (gmem_ptr<const int32_t>)L.sel,
                   (gmem_ptr<const float>)L.w};
}
// Rows 0..n-1 of one step of the single-workgroup cycle: row i gets
// st(i, f(i)).
template <typename F, typename S>
__device__ inline void tail_rows(int32_t n, int32_t tid, F f, S st)
{
    for (int32_t i = tid; i < n; i += TAIL_NT) st(i, f(i));
}

__global__ __launch_bounds__(TAIL_NT) void k_mg_tail(const phf_mg_dev_level* __restrict__ lv,
                                                     int32_t top, int32_t nu,
                                                     const double* __restrict__ cinv,
                                                     int32_t dense, int32_t csweeps,
                                                     const int* iflags)
{
    if (iflags && iflags[0]) return;
    extern __shared__ float lds[];
    const int32_t tid = threadIdx.x;
    {
        const tail_lv T = tail_level(lv, top);
        const gmem_ptr<const float> first = top == 0 ? T.x : T.y;
        float* u0 = lds + (top == 0 ? T.sx : T.sy);
        for (int32_t i = tid; i < T.n; i += TAIL_NT) {
            lds[T.sb + i] = T.b[i];
            u0[i] = first[i];
        }
        __syncthreads();
    }
    // down: pre-smoothing, residual, restriction (with the coarse first sweep)
    for (int32_t l = top; l >= 1; --l) {
        const tail_lv L = tail_level(lv, l);
        const tail_lv C = tail_level(lv, l - 1);
        const float* bh = lds + L.sb;
        float *u = lds + L.sy, *v = lds + L.sx;
        for (int32_t s = 1; s < nu; ++s) {
            const float omega = L.w[s];
            tail_rows(
                L.n, tid, [&](int32_t i) { return u[i] + omega * sres(i, L.n, L.col, L.val, bh, u); },
                [&](int32_t i, float y) { v[i] = y; });
            __syncthreads();
            float* q = u;
            u = v;
            v = q;
        }
        // residual into the free iterate buffer (unused until the way up)
        float* r = v;
        tail_rows(
            L.n, tid, [&](int32_t i) { return L.diag[i] * sres(i, L.n, L.col, L.val, bh, u); },
            [&](int32_t i, float y) { r[i] = y; });
        __syncthreads();
        float* t = lds + L.st;
        for (int32_t p = tid; p < L.nEc; p += TAIL_NT) {
            if (L.n > 0) {
                tri_restrict(p, L.nEc, L.rows9, L.ecode_c, r, t);
            } else {  // no fine unknowns: the sums are zero
                t[3 * p] = 0.0f;
                t[3 * p + 1] = 0.0f;
                t[3 * p + 2] = 0.0f;
            }
        }
        __syncthreads();
        const float wc = l - 1 == 0 ? C.w[PHF_MG_MAX_SWEEPS] : C.w[0];
        float* xc = lds + (l - 1 == 0 ? C.sx : C.sy);
        for (int32_t c = tid; c < C.n; c += TAIL_NT)
            row_collect(c, C.sel, t, C.dinv, wc, lds + C.sb, xc);
        __syncthreads();
    }
    // coarsest level: the solution ends in sx
    {
        const tail_lv L = tail_level(lv, 0);
        float* x = lds + L.sx;
        const float* bh = lds + L.sb;
        if (dense) {
            for (int32_t i = tid; i < L.n; i += TAIL_NT) row_coarse(i, L.n, (gmem_ptr<const double>)cinv, L.diag, bh, x);
            __syncthreads();
        } else {
            float *u = x, *v = lds + L.sy;
            const float omega = L.w[PHF_MG_MAX_SWEEPS];
            for (int32_t s = 0; s < csweeps; ++s) {
                tail_rows(
                    L.n, tid,
                    [&](int32_t i) { return u[i] + omega * sres(i, L.n, L.col, L.val, bh, u); },
                    [&](int32_t i, float y) { v[i] = y; });
                __syncthreads();
                float* q = u;
                u = v;
                v = q;
            }
        }
    }
    // up: prolongation, post-smoothing; each level's result ends in sx
    for (int32_t l = 1; l <= top; ++l) {
        const tail_lv L = tail_level(lv, l);
        const tail_lv C = tail_level(lv, l - 1);
        const float* bh = lds + L.sb;
        // the pre-smoothing (from sy) ended nu - 1 swaps away
        float* u = lds + (((nu - 1) & 1) ? L.sx : L.sy);
        float* v = lds + (((nu - 1) & 1) ? L.sy : L.sx);
        if (C.n > 0) {  // (uniform branch) no coarse unknowns: no correction
            const float* xc = lds + C.sx;
            tail_rows(
                L.n, tid, [&](int32_t i) { return u[i] + prolong_sum(i, L.n, L.P_col, L.P_code, xc); },
                [&](int32_t i, float y) { u[i] = y; });
            __syncthreads();
        }
        for (int32_t s = 0; s < nu; ++s) {
            const float omega = L.w[s];
            tail_rows(
                L.n, tid, [&](int32_t i) { return u[i] + omega * sres(i, L.n, L.col, L.val, bh, u); },
                [&](int32_t i, float y) { v[i] = y; });
            __syncthreads();
            float* q = u;
            u = v;
            v = q;
        }
        if (l == top)
            for (int32_t i = tid; i < L.n; i += TAIL_NT) L.x[i] = u[i];
    }
    if (top == 0) {
        const tail_lv T = tail_level(lv, 0);
        for (int32_t i = tid; i < T.n; i += TAIL_NT) T.x[i] = lds[T.sx + i];
    }
}


__global__ void k_mg_lmax_clear(int32_t nlev, uint32_t* __restrict__ lmax)
{
    if ((int32_t)threadIdx.x < nlev) lmax[threadIdx.x] = 0u;
}

// Sweep weights of every level (one thread per level): Jacobi -> omega for
// every sweep; Chebyshev -> 1 / (c + h cos((2k + 1) pi / (2 nu))), the roots
// of the degree-nu Chebyshev polynomial mapped to [lo, hi] = [lmax / range,
// lmax] (c, h its centre and half-width), and 1 / c (the best single weight
// for that interval) for the plain sweeps of an iterative coarsest solve.
// Sweeps per side on the levels between the finest and the single-workgroup
// tail: one fewer than on those two. Measured with nu = 4 on the paper mesh
// (levels of 24,576-1,572,864 rows between them): 3 sweeps there kept the
// iterations (elliptic solve at 4,194,304 triangles 7, Crank-Nicolson 3.04 ->
// 3.06 per step) and took the solve from 7.49 to 7.10 ms and the stepper
// from 657 to 689 steps/s; 2 sweeps raised the iterations to 10 and 4.07.
// With a per-triangle coefficient the level-10 solve went 9.40 -> 8.93 ms (9
// iterations) and the 3,145,728-triangle L-shape 7.34 -> 7.58 ms (9 -> 10
// iterations); keeping 4 on the level below the finest helped neither.
__host__ __device__ constexpr int32_t mid_sweeps(int32_t nu) { return nu > 1 ? nu - 1 : 1; }

__global__ void k_mg_weights(int32_t nlev, int32_t tail_top, int32_t nu0, int32_t cheb,
                             float omega, float range, const uint32_t* __restrict__ lmax,
                             float* __restrict__ wts)
{
    const int32_t l = threadIdx.x;
    if (l >= nlev) return;
    const int32_t nu = l > tail_top && l < nlev - 1 ? mid_sweeps(nu0) : nu0;
    float* w = wts + (int64_t)l * PHF_MG_WSTRIDE;
    if (!cheb) {
        for (int k = 0; k < PHF_MG_WSTRIDE; ++k) w[k] = omega;
        return;
    }
    float hi = __uint_as_float(lmax[l]);
    if (!(hi > 0.0f)) hi = 1.0f;  // level without unknowns
    const double lo = (double)hi / range;
    const double c = 0.5 * ((double)hi + lo), h = 0.5 * ((double)hi - lo);
    for (int k = 0; k < PHF_MG_MAX_SWEEPS; ++k)
        w[k] = k < nu ? (float)(1.0 / (c + h * cos(M_PI * (2 * k + 1) / (2.0 * nu)))) : 0.0f;
    w[PHF_MG_MAX_SWEEPS] = (float)(1.0 / c);
}

// ---- set-up launches over all levels ------------------------------------
// Every level's prolongation, restriction rows and coarse gather map (one
// launch), and every level's scaled single-precision rows with the Gershgorin
// bound (one launch): consecutive block ranges per level and table, found by
// each block from the level table.
__device__ inline int find_level(const phf_mg_setup_level* lv, int32_t nlev, int32_t b, int part)
{
    int l = nlev - 1;
    while (l > 0 && b < lv[l].b[part]) --l;
    return l;
}

__global__ __launch_bounds__(NT) void k_mg_setup_tables(const phf_mg_setup_level* __restrict__ lv,
                                                        int32_t nlev)
{
    const int32_t b = blockIdx.x;
    // ranges in order: level 1..nlev-1, each prolongation | rows9 | gather map
    const int l = find_level(lv, nlev, b, 0);
    const phf_mg_setup_level& L = lv[l];
    if (l == 0) return;
    const int32_t t = threadIdx.x;
    if (b < L.b[1]) {
        d_mg_prolong_build((b - L.b[0]) * NT + t, L.nf, L.nEc, L.red_edge, L.edge_elems, L.led,
                           L.ledTN, L.elem_red_c, L.P_col, L.P_code);
    } else if (b < L.b[2]) {
        d_mg_rows9((b - L.b[1]) * NT + t, L.nEc, L.elem_red, L.rows9);
    } else {
        d_mg_sel((b - L.b[2]) * NT + t, L.nc, L.red_edge_c, L.edge_elems_c, L.led_c, L.ledTN_c,
                 L.sel_c);
    }
}

__global__ __launch_bounds__(NT) void k_mg_setup_rows(const phf_mg_setup_level* __restrict__ lv,
                                                      int32_t nlev, int32_t gersh,
                                                      uint32_t* __restrict__ lmax)
{
    __shared__ float sh[NT];
    const int l = find_level(lv, nlev, blockIdx.x, 3);
    const phf_mg_setup_level& L = lv[l];
    // a level's blocks loop over its rows
    const int32_t nb = (l + 1 < nlev ? lv[l + 1].b[3] : gridDim.x) - L.b[3];
    float m = 0.0f;  // Gershgorin bound of D^-1 A over this block's rows
    for (int32_t r = (blockIdx.x - L.b[3]) * NT + threadIdx.x; r < L.nf; r += nb * NT) {
        float s;  // 1 + sum_j |a_ij| / a_ii
        if (L.rec) {
            s = d_mg_crows(r, L.nf, L.red_edge, L.edge_elems, L.led, L.ledTN,
                           reinterpret_cast<const phf_i4*>(L.rec), L.col4, L.val4, L.diag,
                           L.dinv, L.col64, L.val64);
        } else {  // the finest level, from the caller's double-precision rows
            // (diagonal, then the four off-diagonal entries; the columns are
            // shared with the caller and already in place)
            const phf_i4 c4 = *(const phf_i4*)(L.ell_col + 4 * (int64_t)r);
            const double* v4 = L.ell_val + 4 * (int64_t)r;
            const int32_t c[5] = {r, c4.x, c4.y, c4.z, c4.w};
            const double v[5] = {L.ell_val[4 * (int64_t)L.nf + r], v4[0], v4[1], v4[2], v4[3]};
            s = phf_scale_row(r, L.nf, c, v, nullptr, L.val4, L.diag, L.dinv);
        }
        m = fmaxf(m, s);
    }
    if (!gersh) return;
    // merged into lmax[l] as the bits of a non-negative float (which order
    // like unsigned integers)
    sh[threadIdx.x] = m;
    __syncthreads();
    for (int h = NT / 2; h > 0; h >>= 1) {
        if (threadIdx.x < h) sh[threadIdx.x] = fmaxf(sh[threadIdx.x], sh[threadIdx.x + h]);
        __syncthreads();
    }
    // (only where it raises the value already there: the bound only grows,
    // so a stale read costs at most an unneeded atomic)
    if (threadIdx.x == 0) {
        const uint32_t bits = __float_as_uint(sh[0]);
        if (bits > __hip_atomic_load(lmax + l, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
            atomicMax(lmax + l, bits);
    }
}

// Levels of at most this many rows take the fused launches (residual with
// restriction, prolongation with the first sweep after it). There the
// launches are bound by latency and the fused forms' extra work costs less
// than the launch they save (measured, µs per cycle on the levels of 24,576
// and 98,304 rows: 4.5 / 5.7 fused against 8.9 / 8.1 for residual and
// restriction, 5.3 / 9.2 against 8.4 / 9.4 for prolongation and sweep). On
// larger levels the fused residual's scattered row loads (nine rows of a
// coarse triangle per group of lanes) and the five prolongations per row cost
// more: 15.5 against 10 µs at 393,216 rows.
#ifndef PHF_MG_FUSE_RR_MAX
#define PHF_MG_FUSE_RR_MAX 120000
#endif
#ifndef PHF_MG_FUSE_PS_MAX
#define PHF_MG_FUSE_PS_MAX 50000
#endif

#ifndef PHF_MG_GRID_MAX
#define PHF_MG_GRID_MAX (1 << 30)
#endif
// Grid of a per-step kernel over n rows (grid-stride beyond the cap), and of
// the last finest sweep, whose per-block partial sums must match the outer
// iteration's grid (at most PHF_PART_MAX blocks).
unsigned grid_for(int32_t n)
{
    return (unsigned)std::min<int64_t>(std::max<int64_t>(nblk(n), 1), PHF_MG_GRID_MAX);
}
unsigned part_grid(int32_t n)
{
    return (unsigned)std::min<int64_t>(std::max<int64_t>(nblk(n), 1), PHF_PART_MAX);
}

// Trace names carry the level ("k_mg_smooth.L9"), counted from the coarsest
// mesh, so per-launch byte counts can be attributed to a level.
enum {
    NM_SMOOTH0, NM_SMOOTH, NM_SMOOTHZ, NM_RESID, NM_RESTRICT, NM_COLLECT, NM_PROLONG, NM_SMOOTH1,
    NM_RESID_RESTRICT, NM_PROLONG_SMOOTH, NM_COUNT
};
struct mg_names {
    char s[NM_COUNT][PHF_MG_MAX_LEVELS][32];
    mg_names()
    {
        static const char* base[NM_COUNT] = {"k_mg_smooth0", "k_mg_smooth", "k_mg_smooth_z",
                                             "k_mg_resid", "k_mg_restrict", "k_mg_collect",
                                             "k_mg_prolong", "k_mg_smooth1",
                                             "k_mg_resid_restrict", "k_mg_prolong_smooth"};
        for (int k = 0; k < NM_COUNT; ++k)
            for (int l = 0; l < PHF_MG_MAX_LEVELS; ++l)
                snprintf(s[k][l], sizeof(s[k][l]), "%s.L%d", base[k], l);
    }
};
const char* mg_name(int kind, int level)
{
    static const mg_names names;  // initialised once, thread-safe
    return names.s[kind][level];
}

}  // namespace

int32_t phf_mg_levels(const phf_mesh* mesh)
{
    int32_t n = 0;
    for (const phf_mesh* m = mesh; m; m = m->parent) ++n;
    return n;
}

void phf_mg_destroy(phf_mg* mg)
{
    if (!mg) return;
    for (int l = 0; l < mg->nlev; ++l) {
        phf_mg_level& L = mg->lev[l];
        phf_dfree(L.aT);
        phf_dfree(L.rec);
        float* f[] = {L.val4, L.diag32, L.dinv32, L.x, L.y, L.b, L.r, L.t};
        for (float* p : f) phf_dfree(p);
        phf_dfree(L.P_code);
        if (l < mg->nlev - 1) phf_dfree(L.col4);  // (the finest level's is the operator's)
        phf_dfree(L.P_col);
        if (l == mg->nlev - 1) phf_dfree(mg->z32);
        phf_dfree(L.rows9);
        phf_dfree(L.sel);
    }
    phf_dfree(mg->cinv);
    phf_dfree(mg->cwork);
    phf_dfree(mg->col64);
    phf_dfree(mg->val64);
    phf_dfree(mg->d_lv);
    phf_dfree(mg->d_setup);
    phf_dfree(mg->lmax);
    phf_dfree(mg->wts);
    delete mg;
}

int phf_mg_create(phf_ns* fine, phf_mg** out, int32_t drop_coarse)
{
    phf_mesh* fm = fine->mesh;
    phf_ctx* ctx = fm->ctx;
    *out = nullptr;
    const int32_t chain = phf_mg_levels(fm);
    if (chain < 2 || chain > PHF_MG_MAX_LEVELS)
        return phf_set_error(ctx, PHF_EINVAL,
                             "multigrid needs a mesh made by phf_mesh_refine (1..%d refinements)",
                             PHF_MG_MAX_LEVELS - 1);
    // at least two levels stay
    const int32_t drop = std::max<int32_t>(0, std::min<int32_t>(drop_coarse, chain - 2));
    const int32_t nlev = chain - drop;
    phf_mg* mg = new (std::nothrow) phf_mg;
    if (!mg) return phf_set_error(ctx, PHF_ENOMEM, "host allocation failed");
    mg->nlev = nlev;
    if (drop > 0) mg->coarse_sweeps = 8;
    auto body = [&]() -> int {
        phf_mesh* m = fm;
        for (int l = nlev - 1; l >= 0; --l, m = m->parent) mg->lev[l].mesh = m;
        for (int l = 0; l < nlev; ++l) {
            phf_mg_level& L = mg->lev[l];
            phf_mesh* ms = L.mesh;
            if (l == nlev - 1) {
                L.ns = fine;
            } else {
                TRY(phf_dmalloc(ctx, &L.rec, 24 * (size_t)std::max<int32_t>(ms->nE, 1),
                                "multigrid half-row records"));
                TRY(phf_dmalloc(ctx, &L.aT, (size_t)ms->nE, "multigrid coefficient"));
            }
            L.nf = ms->n_free;
            const size_t nf = std::max<int32_t>(L.nf, 1);
            // (the finest level shares the operator's columns)
            if (l == nlev - 1) L.col4 = fine->ell_col;
            else TRY(phf_dmalloc(ctx, &L.col4, 4 * nf, "multigrid operator columns"));
            TRY(phf_dmalloc(ctx, &L.val4, 4 * nf, "multigrid operator (single)"));
            TRY(phf_dmalloc(ctx, &L.diag32, nf, "multigrid diagonal (single)"));
            TRY(phf_dmalloc(ctx, &L.dinv32, nf, "multigrid inverse diagonal (single)"));
            TRY(phf_dmalloc(ctx, &L.x, nf, "multigrid x"));
            TRY(phf_dmalloc(ctx, &L.y, nf, "multigrid y"));
            TRY(phf_dmalloc(ctx, &L.b, nf, "multigrid b"));
            TRY(phf_dmalloc(ctx, &L.r, nf, "multigrid r"));
            if (l == nlev - 1) TRY(phf_dmalloc(ctx, &mg->z32, nf, "multigrid result (single)"));
            if (l == 0) continue;
            // prolongation from level l-1
            phf_mg_level& Cl = mg->lev[l - 1];
            TRY(phf_dmalloc(ctx, &L.P_col, 5 * nf, "multigrid P columns"));
            TRY(phf_dmalloc(ctx, &L.P_code, (size_t)nf, "multigrid P weights"));
            // restriction tables
            const int32_t nEc = Cl.mesh->nE, nc = Cl.mesh->n_free;
            TRY(phf_dmalloc(ctx, &L.rows9, 9 * (size_t)nEc, "multigrid restriction rows"));
            TRY(phf_dmalloc(ctx, &L.t, 3 * (size_t)nEc, "multigrid restriction sums"));
            TRY(phf_dmalloc(ctx, &Cl.sel, (size_t)std::max(nc, 1), "multigrid restriction map"));
        }
        mg->n0 = mg->lev[0].nf;
        if (mg->n0 > 0 && mg->n0 <= PHF_MG_DENSE_MAX && drop == 0) {  // (else: sweeps)
            TRY(phf_dmalloc(ctx, &mg->cinv, (size_t)mg->n0 * mg->n0, "coarse inverse"));
            TRY(phf_dmalloc(ctx, &mg->cwork, (size_t)mg->n0 * mg->n0, "coarse work"));
            TRY(phf_dmalloc(ctx, &mg->col64, 5 * (size_t)mg->n0, "coarse operator columns"));
            TRY(phf_dmalloc(ctx, &mg->val64, 5 * (size_t)mg->n0, "coarse operator values"));
        }
        // the small levels below the finest: one workgroup runs their cycle,
        // with their vectors in its local data share (two iterates and D^-1 b
        // per row, three sums per triangle of the next coarser mesh)
        auto tail_floats = [&](int l) {
            return 3 * (int64_t)mg->lev[l].nf + (l > 0 ? 3 * (int64_t)mg->lev[l - 1].mesh->nE : 0);
        };
        // (a coarsest level too large for it runs with one launch per step)
        mg->tail_top = -1;
        int64_t lds_floats = 0;
        while (mg->tail_top + 1 < nlev - 1 && mg->lev[mg->tail_top + 1].nf <= PHF_MG_TAIL_MAX &&
               (lds_floats + tail_floats(mg->tail_top + 1)) * (int64_t)sizeof(float) <= PHF_MG_TAIL_LDS) {
            ++mg->tail_top;
            lds_floats += tail_floats(mg->tail_top);
        }
        mg->tail_lds = (int32_t)(lds_floats * (int64_t)sizeof(float));
        if (mg->tail_top >= 0)
            PHF_HIP(ctx, hipFuncSetAttribute(reinterpret_cast<const void*>(&k_mg_tail),
                                             hipFuncAttributeMaxDynamicSharedMemorySize,
                                             mg->tail_lds));
        int32_t lds_off = 0;
        for (int l = 0; l <= mg->tail_top; ++l) {
            const phf_mg_level& L = mg->lev[l];
            phf_mg_dev_level& d = mg->h_lv[l];
            d.n = L.nf;
            d.col = L.col4;
            d.val = L.val4;
            d.diag = L.diag32;
            d.dinv = L.dinv32;
            d.x = L.x;
            d.y = L.y;
            d.b = L.b;
            d.r = L.r;
            d.sel = L.sel;
            d.sx = lds_off;
            d.sy = lds_off + L.nf;
            d.sb = lds_off + 2 * L.nf;
            lds_off += 3 * L.nf;
            if (l > 0) {
                d.nEc = mg->lev[l - 1].mesh->nE;
                d.P_col = L.P_col;
                d.P_code = L.P_code;
                d.rows9 = L.rows9;
                d.t = L.t;
                d.ecode_c = mg->lev[l - 1].mesh->ecode;
                d.st = lds_off;
                lds_off += 3 * d.nEc;
            }
        }
        TRY(phf_dmalloc(ctx, &mg->lmax, (size_t)nlev, "multigrid spectral bounds"));
        TRY(phf_dmalloc(ctx, &mg->wts, (size_t)nlev * PHF_MG_WSTRIDE, "multigrid sweep weights"));
        for (int l = 0; l <= mg->tail_top; ++l) mg->h_lv[l].w = mg->wts + (size_t)l * PHF_MG_WSTRIDE;
        if (mg->tail_top >= 0) {
            TRY(phf_dmalloc(ctx, &mg->d_lv, (size_t)mg->tail_top + 1, "multigrid level table"));
            PHF_HIP(ctx, hipMemcpyAsync(mg->d_lv, mg->h_lv,
                                        sizeof(phf_mg_dev_level) * (mg->tail_top + 1),
                                        hipMemcpyHostToDevice, ctx->stream));
        }
        // set-up table: per level the mesh tables, outputs and block ranges
        int32_t blk = 0;
        for (int l = 0; l < nlev; ++l) {
            const phf_mg_level& L = mg->lev[l];
            const phf_mesh* ms = L.mesh;
            phf_mg_setup_level& d = mg->h_setup[l];
            d.nf = L.nf;
            d.red_edge = ms->red_edge;
            d.edge_elems = ms->edge_elems;
            d.led = ms->led;
            d.ledTN = ms->ledTN;
            d.elem_red = ms->elem_red;
            d.col4 = L.col4;
            d.val4 = L.val4;
            d.diag = L.diag32;
            d.dinv = L.dinv32;
            if (l == nlev - 1) {
                d.ell_col = fine->ell_col;
                d.ell_val = fine->ell_val;
            } else {
                d.rec = L.rec;
            }
            if (l == 0 && mg->cinv) {
                d.col64 = mg->col64;
                d.val64 = mg->val64;
            }
            if (l == 0) {
                d.b[0] = d.b[1] = d.b[2] = blk;
                continue;
            }
            const phf_mg_level& Cl = mg->lev[l - 1];
            const phf_mesh* mc = Cl.mesh;
            d.nEc = mc->nE;
            d.nc = Cl.nf;
            d.elem_red_c = mc->elem_red;
            d.red_edge_c = mc->red_edge;
            d.edge_elems_c = mc->edge_elems;
            d.led_c = mc->led;
            d.ledTN_c = mc->ledTN;
            d.P_col = L.P_col;
            d.P_code = L.P_code;
            d.rows9 = L.rows9;
            d.sel_c = Cl.sel;
            d.b[0] = blk;
            blk += (int32_t)nblk(L.nf);
            d.b[1] = blk;
            blk += (int32_t)nblk(d.nEc);
            d.b[2] = blk;
            blk += (int32_t)nblk(d.nc);
        }
        mg->setup_table_blocks = blk;
        blk = 0;
        for (int l = 0; l < nlev; ++l) {
            mg->h_setup[l].b[3] = blk;
            blk += (int32_t)nblk(mg->lev[l].nf);
        }
        mg->setup_row_blocks = blk;
        TRY(phf_dmalloc(ctx, &mg->d_setup, (size_t)nlev, "multigrid set-up table"));
        PHF_HIP(ctx, hipMemcpyAsync(mg->d_setup, mg->h_setup, sizeof(phf_mg_setup_level) * nlev,
                                    hipMemcpyHostToDevice, ctx->stream));
        if (mg->setup_table_blocks > 0)
            PHF_LAUNCH(ctx, "k_mg_setup_tables", k_mg_setup_tables, mg->setup_table_blocks, NT, 0,
                       mg->d_setup, nlev);
        return PHF_OK;
    };
    int rc = body();
    if (rc) {
        (void)hipStreamSynchronize(ctx->stream);
        phf_mg_destroy(mg);
        return rc;
    }
    *out = mg;
    return PHF_OK;
}

int phf_mg_numeric(phf_mg* mg, const phf_coeffs* co, double cK, double cM)
{
    phf_ctx* ctx = mg->lev[0].mesh->ctx;
    const int top = mg->nlev - 1;
    // coarse levels, finest to coarsest: the triangle coefficient averaged
    // over the four children and the element blocks of the re-discretised
    // operator (no convection)
    const double* aT_prev = co->a_T;
    for (int l = top - 1; l >= 0; --l) {
        phf_mg_level& L = mg->lev[l];
        const phf_mesh* ms = L.mesh;
        PHF_LAUNCH(ctx, "k_mg_cblocks", k_mg_cblocks, nblk(ms->nE), NT, 0, ms->nE, ms->exy,
                   ms->elem_red, aT_prev, L.aT, co->A[0], co->A[1], co->A[2], co->A[3], cK, cM,
                   reinterpret_cast<phf_i4*>(L.rec));
        if (aT_prev) aT_prev = L.aT;
    }
    // every level's scaled single-precision rows (coarse levels from their
    // blocks, the finest from the operator the caller built) and, for the
    // Chebyshev weights, their Gershgorin bounds
    // (the finest level's come with the operator when phf_mg_fine_rows was
    // used for it: its row blocks, the last ones, are then left out)
    const bool cheb = mg->smoother == PHF_MG_SMOOTH_CHEBYSHEV;
    const int32_t row_blocks = mg->fine_rows_ready ? mg->h_setup[top].b[3] : mg->setup_row_blocks;
    if (!mg->fine_rows_ready)
        PHF_LAUNCH(ctx, "k_mg_lmax_clear", k_mg_lmax_clear, 1, PHF_MG_MAX_LEVELS, 0, mg->nlev,
                   mg->lmax);
    mg->fine_rows_ready = false;
    if (row_blocks > 0)
        PHF_LAUNCH(ctx, "k_mg_setup_rows", k_mg_setup_rows, row_blocks, NT, 0, mg->d_setup,
                   mg->nlev, cheb ? 1 : 0, mg->lmax);
    PHF_LAUNCH(ctx, "k_mg_weights", k_mg_weights, 1, PHF_MG_MAX_LEVELS, 0, mg->nlev,
               mg->tail_top, mg->nu,
               cheb ? 1 : 0, (float)mg->omega, (float)mg->range, mg->lmax, mg->wts);
    if (mg->cinv) {
        const int32_t n0 = mg->n0;
        PHF_LAUNCH(ctx, "k_mg_dense", k_mg_dense, nblk(n0), NT, 0, n0, mg->col64, mg->val64,
                   mg->cinv);
        PHF_LAUNCH(ctx, "k_mg_gj", k_mg_gj, 1, 1024, 0, n0, mg->cinv, mg->cwork);
    }
    return PHF_OK;
}

namespace {
const float* level_weights(const phf_mg* mg, int l) { return mg->wts + (size_t)l * PHF_MG_WSTRIDE; }

// One sweep with weight k of level l, from L.x into L.y (then swapped).
int smooth(phf_mg* mg, int l, int k, const int* iflags)
{
    phf_mg_level& L = mg->lev[l];
    phf_ctx* ctx = L.mesh->ctx;
    const int32_t n = L.nf;
    const unsigned g = grid_for(n);
    const float* w = level_weights(mg, l);
    if (l == mg->nlev - 1)
        PHF_LAUNCH(ctx, mg_name(NM_SMOOTH, l), k_mg_smooth<true>, g, NT, 0, n, L.col4, L.val4,
                   L.b, w, k, L.x, L.y, iflags);
    else
        PHF_LAUNCH(ctx, mg_name(NM_SMOOTH, l), k_mg_smooth<false>, g, NT, 0, n, L.col4, L.val4,
                   L.b, w, k, L.x, L.y, iflags);
    std::swap(L.x, L.y);
    return PHF_OK;
}

// Cycle on level l > tail_top. On entry L.b holds D^-1 b and L.x the first
// sweep from zero (a coarsest level outside the single-workgroup kernel then
// takes coarse_sweeps further plain sweeps, an even number, so its result is in L.x),
// except on the finest level (r_top != null), where this
// function starts from the double-precision residual r_top (unless
// first_done) and the last sweep writes z (z64 or z32) and the partial sums
// of r.z instead of x.
int vcycle(phf_mg* mg, int l, const double* r_top, bool first_done, double* z64, float* z32,
           double* part_rz, const int* iflags)
{
    phf_mg_level& L = mg->lev[l];
    phf_ctx* ctx = L.mesh->ctx;
    if (l <= mg->tail_top) {
        // this level and all below in one workgroup; the result is in L.x
        PHF_LAUNCH(ctx, "k_mg_tail", k_mg_tail, 1, TAIL_NT, mg->tail_lds, mg->d_lv, (int32_t)l,
                   mg->nu, mg->cinv, mg->cinv ? 1 : 0, mg->coarse_sweeps, iflags);
        return PHF_OK;
    }
    const int32_t n = L.nf;
    if (n == 0) return PHF_OK;
    if (l == 0) {
        for (int s = 0; s < mg->coarse_sweeps; ++s)
            TRY(smooth(mg, 0, PHF_MG_MAX_SWEEPS, iflags));
        return PHF_OK;
    }
    const unsigned g = grid_for(n);
    const float* w = level_weights(mg, l);
    const int nu = r_top ? mg->nu : mid_sweeps(mg->nu);  // sweeps per side on this level
    // (on the finest level the second sweep forms the first from D^-1 b, which
    // is then not stored, unless it is the only sweep)
    const bool form1 = r_top && mg->nu >= 2;
    if (r_top && !first_done)
        PHF_LAUNCH(ctx, mg_name(NM_SMOOTH0, l), k_mg_smooth0_top, g, NT, 0, n, L.dinv32, r_top, w,
                   L.b, form1 ? nullptr : L.x, iflags);
    for (int s = 1; s < nu; ++s) {
        if (s == 1 && form1) {
            PHF_LAUNCH(ctx, mg_name(NM_SMOOTH1, l), k_mg_smooth1_top, g, NT, 0, n, L.col4, L.val4,
                       L.b, w, L.y, iflags);
            std::swap(L.x, L.y);
        } else {
            TRY(smooth(mg, l, s, iflags));
        }
    }
    phf_mg_level& C = mg->lev[l - 1];
    const int last = r_top ? nu - 1 : nu;
    bool swept = false;  // the first sweep after the correction is taken
    if (C.nf > 0) {
        if (n <= PHF_MG_FUSE_RR_MAX) {
            const int32_t nEc = C.mesh->nE;
            PHF_LAUNCH(ctx, mg_name(NM_RESID_RESTRICT, l), k_mg_resid_restrict,
                       (unsigned)((nEc + RR_TRI - 1) / RR_TRI), NT, 0, nEc, L.rows9,
                       C.mesh->ecode, n, L.col4, L.val4, L.diag32, L.b, L.x, L.t, iflags);
        } else {
            PHF_LAUNCH(ctx, mg_name(NM_RESID, l), k_mg_resid, g, NT, 0, n, L.col4, L.val4,
                       L.diag32, L.b, L.x, L.r, iflags);
            PHF_LAUNCH(ctx, mg_name(NM_RESTRICT, l), k_mg_restrict, grid_for(C.mesh->nE), NT, 0,
                       C.mesh->nE, L.rows9, C.mesh->ecode, L.r, L.t, iflags);
        }
        // the coarse level's first sweep lands where its cycle expects it:
        // the single-workgroup kernel in y (the coarsest level in x), the
        // per-step launches in the current x
        const bool in_tail = l - 1 <= mg->tail_top;
        float* xc = in_tail && l - 1 > 0 ? C.y : C.x;
        const int32_t kc = l - 1 == 0 ? PHF_MG_MAX_SWEEPS : 0;
        PHF_LAUNCH(ctx, mg_name(NM_COLLECT, l), k_mg_collect, grid_for(C.nf), NT, 0, C.nf, C.sel,
                   L.t, C.dinv32, level_weights(mg, l - 1), kc, C.b, xc, iflags);
        TRY(vcycle(mg, l - 1, nullptr, false, nullptr, nullptr, nullptr, iflags));
        if (n <= PHF_MG_FUSE_PS_MAX && last > 0) {
            PHF_LAUNCH(ctx, mg_name(NM_PROLONG_SMOOTH, l), k_mg_prolong_smooth, g, NT, 0, n,
                       L.P_col, L.P_code, C.x, L.col4, L.val4, L.b, w, 0, L.x, L.y, iflags);
            std::swap(L.x, L.y);
            swept = true;
        } else {
            PHF_LAUNCH(ctx, mg_name(NM_PROLONG, l), k_mg_prolong, g, NT, 0, n, L.P_col, L.P_code,
                       C.x, L.x, iflags);
        }
    }
    for (int s = swept ? 1 : 0; s < last; ++s) TRY(smooth(mg, l, s, iflags));
    if (r_top && z32)
        PHF_LAUNCH(ctx, mg_name(NM_SMOOTHZ, l), k_mg_smooth_z<float>, part_grid(n), NT, 0, n,
                   L.col4, L.val4,
                   L.b, w, mg->nu - 1, L.x, r_top, z32, part_rz, iflags);
    else if (r_top)
        PHF_LAUNCH(ctx, mg_name(NM_SMOOTHZ, l), k_mg_smooth_z<double>, part_grid(n), NT, 0, n,
                   L.col4,
                   L.val4, L.b, w, mg->nu - 1, L.x, r_top, z64, part_rz, iflags);
    return PHF_OK;
}
}  // namespace

int phf_mg_apply(phf_mg* mg, const double* r, double* z, double* part_rz, const int* iflags)
{
    const int top = mg->nlev - 1;
    phf_mg_level& F = mg->lev[top];
    if (F.nf == 0) return PHF_OK;
    // the finest right-hand side is the residual of the outer iteration
    return vcycle(mg, top, r, false, z, nullptr, part_rz, iflags);
}

int phf_mg_apply32(phf_mg* mg, const double* r, bool first_done, double* part_rz,
                   const int* iflags)
{
    const int top = mg->nlev - 1;
    if (mg->lev[top].nf == 0) return PHF_OK;
    return vcycle(mg, top, r, first_done, nullptr, mg->z32, part_rz, iflags);
}

int phf_mg_fine_rows(phf_mg* mg, phf_mg_rows* out)
{
    phf_ctx* ctx = mg->lev[0].mesh->ctx;
    const int top = mg->nlev - 1;
    phf_mg_level& F = mg->lev[top];
    PHF_LAUNCH(ctx, "k_mg_lmax_clear", k_mg_lmax_clear, 1, PHF_MG_MAX_LEVELS, 0, mg->nlev, mg->lmax);
    // (no columns: the finest level shares the operator's)
    *out = phf_mg_rows{nullptr, F.val4, F.diag32, F.dinv32, mg->lmax + top};
    mg->fine_rows_ready = true;
    return PHF_OK;
}

phf_mg_top phf_mg_top_view(phf_mg* mg)
{
    const int top = mg->nlev - 1;
    phf_mg_level& F = mg->lev[top];
    return phf_mg_top{F.b, mg->nu >= 2 ? nullptr : F.x, F.dinv32, level_weights(mg, top)};
}
