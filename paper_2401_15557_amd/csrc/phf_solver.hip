// Null-space conjugate-gradient solve of the saddle system of Section 3.5
// (see phf_solver.h for the reduction) and the phf_solve entry point.
#include "phf_device.h"
#include "phf_mg.h"
#include "phf_solver.h"

namespace {

constexpr int NT = 256;
constexpr int MAXB = PHF_PART_MAX;  // max blocks of the vector kernels = partial-sum slots

inline unsigned nblk(int64_t n) { return (unsigned)((n + NT - 1) / NT); }

// U_i = (w0 + w1 + w2) - 2 w_i ;  (P^T v)_l = (v0 + v1 + v2) - 2 v_l
__device__ inline void apply_P(const double w[3], double U[3])
{
    const double s = w[0] + w[1] + w[2];
    U[0] = s - 2.0 * w[0];
    U[1] = s - 2.0 * w[1];
    U[2] = s - 2.0 * w[2];
}

// A_T = cK K_T + cM M_T + cD D_T (M, D nullable) for a tile of NT elements,
// staged in LDS so that the 9-value element blocks are read (and, with Ablk,
// stored) with coalesced accesses; then each element's B_T = P^T A_T P
// (A_T need not be symmetric) and its half-row records of the reduced
// operator (phf_hrec_element), staged in LDS as well and stored as one
// contiguous run per tile. (A Dirichlet local edge's record is not formed;
// its slot is stored unset and never read.)
__global__ __launch_bounds__(NT) void k_ns_elem(int32_t nE, const double* __restrict__ K,
                                                const double* __restrict__ M,
                                                const double* __restrict__ D, double cK,
                                                double cM, double cD,
                                                const int32_t* __restrict__ elem_red,
                                                double* __restrict__ Ablk,
                                                phf_i4* __restrict__ rec)
{
    // the tile's blocks A_T, then (same space) its records, 6 units each
    __shared__ __align__(16) phf_i4 smem[6 * NT];
    double* sA = reinterpret_cast<double*>(smem);
    const int tid = threadIdx.x;
    const int64_t m0 = (int64_t)blockIdx.x * NT;
    const int32_t nt = (int32_t)min((int64_t)NT, (int64_t)nE - m0);
    for (int32_t q = tid; q < 9 * nt; q += NT) {
        const int64_t g = 9 * m0 + q;
        double a = M ? cK * K[g] + cM * M[g] : cK * K[g];
        if (D) a += cD * D[g];
        sA[q] = a;
    }
    __syncthreads();
    if (Ablk)
        for (int32_t q = tid; q < 9 * nt; q += NT) Ablk[9 * m0 + q] = sA[q];
    double Bm[9];
    int32_t red[3] = {-1, -1, -1};
    if (tid < nt) {
        const int64_t m = m0 + tid;
        phf_reduce_block(sA + 9 * tid, Bm);
#pragma unroll
        for (int l = 0; l < 3; ++l) red[l] = elem_red[3 * m + l];
    }
    __syncthreads();  // (the records overwrite the blocks)
    if (tid < nt) phf_hrec_element(smem, tid, red, Bm);
    __syncthreads();
    for (int32_t q = tid; q < 6 * nt; q += NT) rec[6 * m0 + q] = smem[q];
}

// Rows of the reduced operator from the half-row records: the diagonal, and
// the off-diagonal entries in ascending column order as ELL-4, row-major
// (ell_col[4r..4r+3] int32, ell_val[4r..4r+3] double; unused entries column
// r, value 0), the diagonal values behind them at ell_val[4 nf + r], and
// either the inverse diagonal (1 where it is not positive) or, with FINE,
// the multigrid preconditioner's finest-level rows (phf_scale_row, from the
// same values; they share the columns) and their Gershgorin bound.
template <bool FINE>
__global__ __launch_bounds__(NT) void k_ns_ellrows(int32_t nf, const int32_t* __restrict__ red_edge,
                                                   const int2* __restrict__ edge_elems,
                                                   const int8_t* __restrict__ led,
                                                   const int8_t* __restrict__ ledTN,
                                                   const phf_i4* __restrict__ rec,
                                                   int32_t* __restrict__ ell_col,
                                                   double* __restrict__ ell_val,
                                                   double* __restrict__ dinv, phf_mg_rows fr)
{
    const int32_t r = blockIdx.x * NT + threadIdx.x;
    float gs = 0.0f;  // Gershgorin sum of the row (FINE)
    if (r < nf) {
        int32_t col[5];
        double v[5];
        const int32_t e = red_edge[r];
        const int n = phf_hrec_row(r, edge_elems[e], led[e], ledTN[e], rec, col, v);
        double d = 0.0;
#pragma unroll
        for (int k = 0; k < 5; ++k)
            if (k < n && col[k] == r) d = v[k];
        int32_t c4[4] = {r, r, r, r};
        double v4[4] = {0.0, 0.0, 0.0, 0.0};
        int q = 0;
#pragma unroll
        for (int k = 0; k < 5; ++k)
            if (col[k] != r && q < 4) {
                c4[q] = col[k];
                v4[q] = v[k];
                ++q;
            }
        *(phf_i4*)(ell_col + 4 * (int64_t)r) = phf_i4{c4[0], c4[1], c4[2], c4[3]};
        *(phf_d2*)(ell_val + 4 * (int64_t)r) = phf_d2{v4[0], v4[1]};
        *(phf_d2*)(ell_val + 4 * (int64_t)r + 2) = phf_d2{v4[2], v4[3]};
        ell_val[4 * (int64_t)nf + r] = d;
        // (the Jacobi preconditioner's; the multigrid one scales its own rows)
        if (!FINE) dinv[r] = d > 0.0 ? 1.0 / d : 1.0;
        if (FINE) gs = phf_scale_row(r, nf, col, v, fr.col4, fr.val4, fr.diag, fr.dinv);
    }
    if (FINE) {
        // block maximum; merged into the bound only where it raises the value
        // already there (the bound only grows, so a stale read costs at most
        // an unneeded atomic)
        __shared__ float wm[NT / 64];
        float m = gs;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o));
        if ((threadIdx.x & 63) == 0) wm[threadIdx.x >> 6] = m;
        __syncthreads();
        if (threadIdx.x == 0) {
            float b = wm[0];
#pragma unroll
            for (int w = 1; w < NT / 64; ++w) b = fmaxf(b, wm[w]);
            const uint32_t bits = __float_as_uint(b);
            if (bits > __hip_atomic_load(fr.lmax, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
                atomicMax(fr.lmax, bits);
        }
    }
}

// Element records of a tile of NT elements (W values each, element-major)
// copied between global memory and LDS with coalesced accesses.
template <int W, typename T>
__device__ inline void tile_load(const T* __restrict__ g, int64_t m0, int32_t nt, T* s)
{
    for (int32_t q = threadIdx.x; q < W * nt; q += NT) s[q] = g[W * m0 + q];
}
template <int W, typename T>
__device__ inline void tile_store(T* __restrict__ g, int64_t m0, int32_t nt, const T* s)
{
    for (int32_t q = threadIdx.x; q < W * nt; q += NT) g[W * m0 + q] = s[q];
}

// Raises *jflag when an interior (non-Dirichlet) multiplier row has a
// non-zero constraint right-hand side, i.e. when k_ns_known has jumps to
// gather; it never lowers it (k_ns_gather does, after use), so a flag left
// raised only costs the gathers. One store per block at most.
__global__ __launch_bounds__(NT) void k_ns_jumpflag(int32_t L, const int2* __restrict__ row_nodes,
                                                    const double* __restrict__ rhs2,
                                                    int* __restrict__ jflag)
{
    int any = 0;
    for (int32_t r = blockIdx.x * NT + threadIdx.x; r < L; r += gridDim.x * NT)
        if (rhs2[r] != 0.0) any |= row_nodes[r].x >= 0;
    if (__syncthreads_or(any) && threadIdx.x == 0) *jflag = 1;
}

// Known midpoint values (Dirichlet) and T+-side jumps (interior rows with a
// non-zero right-hand side; gathered only when *jflag is raised), and the
// element part of the reduced rhs,
// c_T = P^T (rhs1_T - A_T P kv_T). Where kv_T = 0 (in an elliptic solve most
// elements: no known value on their edges) the product is zero and A_T is
// not read. The element rows of rhs1, kv and c go through LDS.
__global__ __launch_bounds__(NT) void k_ns_known(int32_t nE, const int32_t* __restrict__ ecode,
                                                 const int32_t* __restrict__ elem_row,
                                                 const double* __restrict__ row_hs,
                                                 const double* __restrict__ rhs1,
                                                 const double* __restrict__ rhs2,
                                                 const double* __restrict__ A,
                                                 const int* __restrict__ jflag, int all_jumps,
                                                 const double* __restrict__ hs_elem,
                                                 double* __restrict__ kv, double* __restrict__ cs)
{
    __shared__ double sR[3 * NT], sK[3 * NT], sC[3 * NT];
    const bool jumps = all_jumps || *jflag != 0;
    const int tid = threadIdx.x;
    const int64_t m0 = (int64_t)blockIdx.x * NT;
    const int32_t nt = (int32_t)min((int64_t)NT, (int64_t)nE - m0);
    tile_load<3>(rhs1, m0, nt, sR);
    __syncthreads();
    if (tid < nt) {
        const int64_t m = m0 + tid;
        const int code = ecode[m];
        double k3[3];
        bool known = false;
#pragma unroll
        for (int l = 0; l < 3; ++l) {
            const int t = PHF_CODE_TYPE(code, l);
            double v = 0.0;
            if (t == 1 || (jumps && t == 0 && PHF_CODE_TPLUS(code, l))) {
                const int32_t r = elem_row[3 * m + l];
                // |E|/2 per element edge when given (a stream), else by row
                const double h = hs_elem ? hs_elem[3 * m + l] : row_hs[r];
                v = -rhs2[r] / (2.0 * fabs(h));
                known |= v != 0.0;
            }
            k3[l] = v;
            sK[3 * tid + l] = v;
        }
        double res[3] = {sR[3 * tid], sR[3 * tid + 1], sR[3 * tid + 2]};
        if (known) {
            double Ub[3];
            apply_P(k3, Ub);
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                const double* a = A + 9 * m + 3 * i;
                res[i] -= a[0] * Ub[0] + a[1] * Ub[1] + a[2] * Ub[2];
            }
        }
        double c[3];
        apply_P(res, c);  // P is symmetric, so P^T v = P v
#pragma unroll
        for (int l = 0; l < 3; ++l) sC[3 * tid + l] = c[l];
    }
    __syncthreads();
    tile_store<3>(kv, m0, nt, sK);
    tile_store<3>(cs, m0, nt, sC);
}

__global__ __launch_bounds__(NT) void k_ns_gather(int32_t nf, const int32_t* __restrict__ red_edge,
                                                  const int2* __restrict__ edge_elems,
                                                  const int8_t* __restrict__ led,
                                                  const int8_t* __restrict__ ledTN,
                                                  const double* __restrict__ cs,
                                                  double* __restrict__ b, int* __restrict__ jflag)
{
    int32_t r = blockIdx.x * NT + threadIdx.x;
    if (r == 0) *jflag = 0;  // the jumps of this right-hand side are used
    if (r >= nf) return;
    int32_t e = red_edge[r];
    int2 tt = edge_elems[e];
    double v = cs[3 * (int64_t)tt.x + led[e]];
    if (tt.y >= 0) v += cs[3 * (int64_t)tt.y + ledTN[e]];
    b[r] = v;
}

// ---- conjugate gradients with device-side scalars --------------------------
//
// Two kernels per iteration i (i = 0, 1, ...):
//   dir(i):    beta = rz_i / rz_{i-1} (0 for i = 0); p = z + beta p;
//              q = A z + beta q  (= A p by linearity); partial sums of p.q.
//              For i > 0 it first tests the residual of iteration i: if
//              ||r||^2 <= tol^2 ||b||^2 every block exits and block 0 raises
//              the done flag.
//   upd(i):    alpha = rz_i / p.q; w += alpha p; r -= alpha q; z = D^-1 r;
//              partial sums of r.z (into the slot of parity i+1) and r.r.
//   check(i):  ||r|| of the update against the tolerance (one block); with
//              the multigrid preconditioner it runs before the V-cycle, so the
//              cycle of a converged iterate is skipped.
// Every block reduces the partial-sum arrays itself in the same fixed order,
// so all blocks see bitwise identical scalars and no kernel writes a value
// that another block of the same launch reads. The iteration index arrives as
// a kernel argument, so an unrolled chain can be captured in a graph; once
// done is set, the remaining kernels of the chain return immediately.

#ifndef PHF_NT_CG
#define PHF_NT_CG 1
#endif
// Streamed loads and stores of the conjugate-gradient vectors and operator,
// marked non-temporal with PHF_NT_CG: the cycle's sweeps between them then
// find more of their operator rows still in the caches.
template <typename T>
__device__ inline T ntl(const T* p)
{
#if PHF_NT_CG
    return __builtin_nontemporal_load(p);
#else
    return *p;
#endif
}
template <typename T>
__device__ inline void nts(T* p, T v)
{
#if PHF_NT_CG
    __builtin_nontemporal_store(v, p);
#else
    *p = v;
#endif
}

// Row r of the reduced operator times x (layout as k_ns_ellrows writes it).
// The terms are summed in ascending column order, the diagonal in its place
// (unused entries add an exact zero), so that the rounding does not depend on
// the storage layout.
template <typename XT>
__device__ inline double ell_row(int32_t r, int32_t nf, const int32_t* __restrict__ col,
                                 const double* __restrict__ val, const XT* __restrict__ x)
{
    const phf_i4 c = ntl(reinterpret_cast<const phf_i4*>(col + 4 * (int64_t)r));
    const phf_d2 v01 = ntl(reinterpret_cast<const phf_d2*>(val + 4 * (int64_t)r));
    const phf_d2 v23 = ntl(reinterpret_cast<const phf_d2*>(val + 4 * (int64_t)r + 2));
    const double dv = ntl(val + 4 * (int64_t)nf + r);
    const int32_t cc[4] = {c.x, c.y, c.z, c.w};
    const double vv[4] = {v01.x, v01.y, v23.x, v23.y};
    double s = 0.0;
    bool dd = false;  // diagonal term added
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        if (!dd && cc[k] > r) {
            s = fma(dv, (double)x[r], s);
            dd = true;
        }
        s = fma(vv[k], (double)x[cc[k]], s);
    }
    if (!dd) s = fma(dv, (double)x[r], s);
    return s;
}

// Partial-sum layout in phf_ns::part (MAXB slots each).
enum {
    P_RZ0 = 0, P_RZ1 = 1, P_PQ = 2, P_RR = 3, P_BB = 4,
    // BiCGSTAB: two parities each of (rh, r), (rh, v), (t, s), (t, t); scratch
    P_RHO0 = 5, P_RV0 = 7, P_TS0 = 9, P_TT0 = 11, P_SCR = 13,
    P_NARR = 14
};

// Sum of nb partials in a fixed order, broadcast to the whole block.
__device__ inline double block_reduce_partials(const double* __restrict__ part, int32_t nb,
                                               double* sh)
{
    double s = 0.0;
    for (int q = threadIdx.x; q < nb; q += NT) s += part[q];
    return phf_block_sum_f64<NT>(s, sh);
}

// K partial-sum slots reduced together, behind one pair of barriers; each in
// the same order as block_reduce_partials, so the results are identical. sh
// holds K * NT / 64 doubles.
template <int K>
__device__ inline void block_reduce_slots(const double* __restrict__ part, const int (&slot)[K],
                                          int32_t nb, double* sh, double (&out)[K])
{
    double s[K];
#pragma unroll
    for (int k = 0; k < K; ++k) s[k] = 0.0;
    for (int q = threadIdx.x; q < nb; q += NT) {
#pragma unroll
        for (int k = 0; k < K; ++k) s[k] += part[slot[k] * MAXB + q];
    }
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const double x = phf_wave_sum(s[k]);
        if (lane == 0) sh[k * (NT / 64) + wid] = x;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < K; ++k) {
        double t = 0.0;
#pragma unroll
        for (int w = 0; w < NT / 64; ++w) t += sh[k * (NT / 64) + w];
        out[k] = t;
    }
    __syncthreads();
}

// ZERO: the iteration starts from w = 0, which the kernel writes; r = b
// without a product.
template <bool JAC, bool ZERO>
__global__ __launch_bounds__(NT) void k_cg_init(int32_t nf, const int32_t* __restrict__ col,
                                                const double* __restrict__ val,
                                                const double* __restrict__ dinv,
                                                const double* __restrict__ b,
                                                double* __restrict__ w,
                                                double* __restrict__ r, double* __restrict__ z,
                                                double* __restrict__ p, double* __restrict__ q,
                                                double* __restrict__ part)
{
    __shared__ double sh[NT / 64];
    double s_rz = 0.0, s_rr = 0.0, s_bb = 0.0;
    for (int32_t i = blockIdx.x * NT + threadIdx.x; i < nf; i += gridDim.x * NT) {
        double ri;
        if (ZERO) {
            w[i] = 0.0;
            ri = b[i];
        } else {
            ri = b[i] - ell_row(i, nf, col, val, w);
        }
        r[i] = ri;
        p[i] = 0.0;
        q[i] = 0.0;
        if (JAC) {
            double zi = dinv[i] * ri;
            z[i] = zi;
            s_rz = fma(ri, zi, s_rz);
        }
        s_rr = fma(ri, ri, s_rr);
        s_bb = fma(b[i], b[i], s_bb);
    }
    double t0 = phf_block_sum_f64<NT>(s_rz, sh);
    double t1 = phf_block_sum_f64<NT>(s_rr, sh);
    double t2 = phf_block_sum_f64<NT>(s_bb, sh);
    if (threadIdx.x == 0) {
        if (JAC) part[P_RZ0 * MAXB + blockIdx.x] = t0;
        part[P_RR * MAXB + blockIdx.x] = t1;
        part[P_BB * MAXB + blockIdx.x] = t2;
    }
}

__global__ __launch_bounds__(NT) void k_cg_init_final(const double* __restrict__ part, int32_t nb,
                                                      double tol2, double* scal, int* iflags)
{
    __shared__ double sh[NT / 64];
    double rr = block_reduce_partials(part + P_RR * MAXB, nb, sh);
    double bb = block_reduce_partials(part + P_BB * MAXB, nb, sh);
    if (threadIdx.x == 0) {
        scal[NS_RR] = rr;
        scal[NS_BB] = bb;
        scal[NS_TOL2] = tol2;
        iflags[0] = (rr <= tol2 * bb) ? 1 : 0;
        iflags[1] = 0;
        iflags[2] = 0;
    }
}


// ZT: double, or float where z is the multigrid cycle's single-precision
// result (converted exactly).
template <typename ZT>
__global__ __launch_bounds__(NT) void k_cg_dir(int32_t nf, int32_t it, int32_t nb,
                                               const int32_t* __restrict__ col,
                                               const double* __restrict__ val,
                                               const ZT* __restrict__ z,
                                               double* __restrict__ p, double* __restrict__ q,
                                               double* __restrict__ part, double* scal,
                                               int* iflags)
{
    if (iflags[0]) return;
    __shared__ double sh[3 * NT / 64];
    double beta = 0.0;
    if (it > 0) {
        // r.r (convergence test), r.z of this and of the previous iteration
        double red[3];
        block_reduce_slots<3>(part, {P_RR, (it & 1) ? P_RZ1 : P_RZ0, (it & 1) ? P_RZ0 : P_RZ1},
                              nb, sh, red);
        const double rr = red[0];
        const double bb = scal[NS_BB], tol2 = scal[NS_TOL2];
        if (rr <= tol2 * bb) {
            if (blockIdx.x == 0 && threadIdx.x == 0) {
                iflags[0] = 1;
                scal[NS_RR] = rr;
            }
            return;
        }
        beta = red[1] / red[2];
        if (blockIdx.x == 0 && threadIdx.x == 0) scal[NS_RR] = rr;
    }
    double s = 0.0;
    phf_for_rows<(PHF_XCD_BITS & 64) != 0, NT>(nf, [&](int32_t i) {
        const double pi = fma(beta, ntl(p + i), (double)z[i]);
        const double qi = fma(beta, ntl(q + i), ell_row(i, nf, col, val, z));
        nts(p + i, pi);
        nts(q + i, qi);
        s = fma(pi, qi, s);
    });
    const double t = phf_block_sum_f64<NT>(s, sh);
    if (threadIdx.x == 0) part[P_PQ * MAXB + blockIdx.x] = t;
}

template <bool JAC>
__global__ __launch_bounds__(NT) void k_cg_upd(int32_t nf, int32_t it, int32_t nb,
                                               double* __restrict__ w, double* __restrict__ r,
                                               double* __restrict__ z,
                                               const double* __restrict__ p,
                                               const double* __restrict__ q,
                                               const double* __restrict__ dinv,
                                               double* __restrict__ part, int* iflags)
{
    if (iflags[0]) return;
    __shared__ double sh[2 * NT / 64];
    double red[2];  // r.z, p.q
    block_reduce_slots<2>(part, {(it & 1) ? P_RZ1 : P_RZ0, P_PQ}, nb, sh, red);
    const double alpha = red[0] / red[1];
    double s_rz = 0.0, s_rr = 0.0;
    for (int32_t i = blockIdx.x * NT + threadIdx.x; i < nf; i += gridDim.x * NT) {
        w[i] = fma(alpha, p[i], w[i]);
        const double ri = fma(-alpha, q[i], r[i]);
        r[i] = ri;
        if (JAC) {
            const double zi = dinv[i] * ri;
            z[i] = zi;
            s_rz = fma(ri, zi, s_rz);
        }
        s_rr = fma(ri, ri, s_rr);
    }
    const double t0 = phf_block_sum_f64<NT>(s_rz, sh);
    const double t1 = phf_block_sum_f64<NT>(s_rr, sh);
    if (threadIdx.x == 0) {
        if (JAC) part[((it & 1) ? P_RZ0 : P_RZ1) * MAXB + blockIdx.x] = t0;
        part[P_RR * MAXB + blockIdx.x] = t1;
        if (blockIdx.x == 0) iflags[1] += 1;
    }
}

// The update with the multigrid preconditioner, which also takes the cycle's
// first sweep from zero on the finest level: bh = D^-1 r rounded to single
// precision, x = w[0] bh (the cycle then continues from its second sweep; x
// null: that sweep forms x from bh itself).
__global__ __launch_bounds__(NT) void k_cg_upd_mg(int32_t nf, int32_t it, int32_t nb,
                                                  double* __restrict__ w, double* __restrict__ r,
                                                  const double* __restrict__ p,
                                                  const double* __restrict__ q,
                                                  double* __restrict__ part, int* iflags,
                                                  const float* __restrict__ dinv32,
                                                  const float* __restrict__ wts,
                                                  float* __restrict__ bh, float* __restrict__ x)
{
    if (iflags[0]) return;
    __shared__ double sh[2 * NT / 64];
    double red[2];  // r.z, p.q
    block_reduce_slots<2>(part, {(it & 1) ? P_RZ1 : P_RZ0, P_PQ}, nb, sh, red);
    const double alpha = red[0] / red[1];
    const float w0 = wts[0];
    double s_rr = 0.0;
    for (int32_t i = blockIdx.x * NT + threadIdx.x; i < nf; i += gridDim.x * NT) {
        nts(w + i, fma(alpha, ntl(p + i), ntl(w + i)));
        const double ri = fma(-alpha, ntl(q + i), ntl(r + i));
        nts(r + i, ri);
        s_rr = fma(ri, ri, s_rr);
        const float h = (float)ri * ntl(dinv32 + i);
        bh[i] = h;
        if (x) x[i] = w0 * h;
    }
    const double t1 = phf_block_sum_f64<NT>(s_rr, sh);
    if (threadIdx.x == 0) {
        part[P_RR * MAXB + blockIdx.x] = t1;
        if (blockIdx.x == 0) iflags[1] += 1;
    }
}

// Convergence test after the last iteration of a chain.
__global__ __launch_bounds__(NT) void k_cg_check(int32_t nb, const double* __restrict__ part,
                                                 double* scal, int* iflags)
{
    if (iflags[0]) return;
    __shared__ double sh[NT / 64];
    const double rr = block_reduce_partials(part + P_RR * MAXB, nb, sh);
    if (threadIdx.x == 0) {
        scal[NS_RR] = rr;
        if (rr <= scal[NS_TOL2] * scal[NS_BB]) iflags[0] = 1;
    }
}

// ---- recovery -------------------------------------------------------------

// U_T = P (w_T + kv_T) and (MU) the element residual P^T (A_T U_T - rhs1_T)
// from which the multipliers follow.
template <bool MU>
__global__ __launch_bounds__(NT) void k_ns_recover_u(int32_t nE, const int32_t* __restrict__ elem_red,
                                                     const double* __restrict__ w,
                                                     const double* __restrict__ kv,
                                                     const double* __restrict__ A,
                                                     const double* __restrict__ rhs1,
                                                     double* __restrict__ U,
                                                     double* __restrict__ cs)
{
    int32_t m = blockIdx.x * NT + threadIdx.x;
    if (m >= nE) return;
    double wt[3];
#pragma unroll
    for (int l = 0; l < 3; ++l) {
        int32_t rr = elem_red[3 * (int64_t)m + l];
        wt[l] = (rr >= 0 ? w[rr] : 0.0) + kv[3 * (int64_t)m + l];
    }
    double u[3];
    apply_P(wt, u);
#pragma unroll
    for (int i = 0; i < 3; ++i) U[3 * (int64_t)m + i] = u[i];
    if (!MU) return;
    double res[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        const double* a = A + 9 * (int64_t)m + 3 * i;
        res[i] = (a[0] * u[0] + a[1] * u[1] + a[2] * u[2]) - rhs1[3 * (int64_t)m + i];
    }
    double s[3];
    apply_P(res, s);
#pragma unroll
    for (int l = 0; l < 3; ++l) cs[3 * (int64_t)m + l] = s[l];
}

__global__ __launch_bounds__(NT) void k_ns_recover_mu(int32_t L, const int32_t* __restrict__ row_edge,
                                                      const int2* __restrict__ edge_elems,
                                                      const int8_t* __restrict__ led,
                                                      const double* __restrict__ row_hs,
                                                      const double* __restrict__ cs, double scale,
                                                      double* __restrict__ mu)
{
    int32_t r = blockIdx.x * NT + threadIdx.x;
    if (r >= L) return;
    int32_t e = row_edge[r];
    int32_t T = edge_elems[e].x;
    mu[r] = scale * cs[3 * (int64_t)T + led[e]] / (2.0 * fabs(row_hs[r]));
}

#define TRY(x)               \
    do {                     \
        int rc_ = (x);       \
        if (rc_) return rc_; \
    } while (0)


// ---- BiCGSTAB (right-preconditioned), for nonsymmetric reduced operators ---
//
// Iteration i with parity k = i & 1; slot X[k] holds a partial sum of
// iteration i, X[k ^ 1] the one of iteration i - 1:
//   dir(i): (i > 0) test ||r_i||; rho_i = (rh, r_i) from RHO[k]; beta =
//           (rho_i / rho_{i-1}) (alpha_{i-1} / omega_{i-1}); p = r + beta (p -
//           omega_{i-1} v); with Jacobi ph = D^-1 p (else the V-cycle follows).
//   v(i):   v = A ph; partial (rh, v) -> RV[k].
//   s(i):   alpha_i = rho_i / (rh, v); s = r - alpha_i v; with Jacobi sh = D^-1 s.
//   t(i):   t = A sh; partials (t, s) -> TS[k], (t, t) -> TT[k].
//   x(i):   omega_i = (t, s) / (t, t); w += alpha_i ph + omega_i sh;
//           r = s - omega_i t; partials (rh, r) -> RHO[k ^ 1], (r, r) -> RR.
// A zero rho, (rh, v) or omega is a breakdown: every block sees the same
// scalars, block 0 raises done and iflags[2], and the chain stops.

__global__ __launch_bounds__(NT) void k_bi_init(int32_t nf, const int32_t* __restrict__ col,
                                                const double* __restrict__ val,
                                                const double* __restrict__ b,
                                                const double* __restrict__ w,
                                                double* __restrict__ r, double* __restrict__ rh,
                                                double* __restrict__ p, double* __restrict__ v,
                                                double* __restrict__ part)
{
    __shared__ double sh[NT / 64];
    double s_rr = 0.0, s_bb = 0.0;
    for (int32_t i = blockIdx.x * NT + threadIdx.x; i < nf; i += gridDim.x * NT) {
        const double ri = b[i] - ell_row(i, nf, col, val, w);
        r[i] = ri;
        rh[i] = ri;
        p[i] = 0.0;
        v[i] = 0.0;
        s_rr = fma(ri, ri, s_rr);
        s_bb = fma(b[i], b[i], s_bb);
    }
    const double t1 = phf_block_sum_f64<NT>(s_rr, sh);
    const double t2 = phf_block_sum_f64<NT>(s_bb, sh);
    if (threadIdx.x == 0) {
        part[P_RHO0 * MAXB + blockIdx.x] = t1;
        part[P_RR * MAXB + blockIdx.x] = t1;
        part[P_BB * MAXB + blockIdx.x] = t2;
    }
}

template <bool JAC>
__global__ __launch_bounds__(NT) void k_bi_dir(int32_t nf, int32_t it, int32_t nb,
                                               const double* __restrict__ r,
                                               double* __restrict__ p, const double* __restrict__ v,
                                               const double* __restrict__ dinv,
                                               double* __restrict__ ph, const double* __restrict__ part,
                                               double* scal, int* iflags)
{
    if (iflags[0]) return;
    __shared__ double shm[NT / 64];
    const int k = it & 1;
    double beta = 0.0, om = 0.0;
    const double rho = block_reduce_partials(part + (P_RHO0 + k) * MAXB, nb, shm);
    bool brk = rho == 0.0;
    if (it > 0) {
        const double rr = block_reduce_partials(part + P_RR * MAXB, nb, shm);
        const double bb = scal[NS_BB], tol2 = scal[NS_TOL2];
        if (rr <= tol2 * bb) {
            if (blockIdx.x == 0 && threadIdx.x == 0) {
                iflags[0] = 1;
                scal[NS_RR] = rr;
            }
            return;
        }
        const double rho_o = block_reduce_partials(part + (P_RHO0 + (k ^ 1)) * MAXB, nb, shm);
        const double rv_o = block_reduce_partials(part + (P_RV0 + (k ^ 1)) * MAXB, nb, shm);
        const double ts_o = block_reduce_partials(part + (P_TS0 + (k ^ 1)) * MAXB, nb, shm);
        const double tt_o = block_reduce_partials(part + (P_TT0 + (k ^ 1)) * MAXB, nb, shm);
        om = tt_o != 0.0 ? ts_o / tt_o : 0.0;
        brk = brk || om == 0.0 || rho_o == 0.0 || rv_o == 0.0;
        if (!brk) beta = (rho / rho_o) * ((rho_o / rv_o) / om);
        if (blockIdx.x == 0 && threadIdx.x == 0) scal[NS_RR] = rr;
    }
    if (brk) {
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            iflags[0] = 1;
            iflags[2] = 1;
        }
        return;
    }
    for (int32_t i = blockIdx.x * NT + threadIdx.x; i < nf; i += gridDim.x * NT) {
        const double pi = it > 0 ? fma(beta, fma(-om, v[i], p[i]), r[i]) : r[i];
        p[i] = pi;
        if (JAC) ph[i] = dinv[i] * pi;
    }
}

// y = A x with one partial inner product (a, y) -> slot0, and optionally
// (c, y) -> slot1 and (y, y) -> slot2.
__global__ __launch_bounds__(NT) void k_bi_spmv(int32_t nf, const int32_t* __restrict__ col,
                                                const double* __restrict__ val,
                                                const double* __restrict__ x,
                                                double* __restrict__ y, const double* __restrict__ a,
                                                double* __restrict__ part, int slot0, int slot1,
                                                const int* iflags)
{
    if (iflags[0]) return;
    __shared__ double sh[NT / 64];
    double s0 = 0.0, s1 = 0.0;
    for (int32_t i = blockIdx.x * NT + threadIdx.x; i < nf; i += gridDim.x * NT) {
        const double yi = ell_row(i, nf, col, val, x);
        y[i] = yi;
        s0 = fma(a[i], yi, s0);
        s1 = fma(yi, yi, s1);
    }
    const double t0 = phf_block_sum_f64<NT>(s0, sh);
    const double t1 = phf_block_sum_f64<NT>(s1, sh);
    if (threadIdx.x == 0) {
        part[slot0 * MAXB + blockIdx.x] = t0;
        if (slot1 >= 0) part[slot1 * MAXB + blockIdx.x] = t1;
    }
}

template <bool JAC>
__global__ __launch_bounds__(NT) void k_bi_s(int32_t nf, int32_t it, int32_t nb,
                                             const double* __restrict__ r,
                                             const double* __restrict__ v,
                                             const double* __restrict__ dinv,
                                             double* __restrict__ s, double* __restrict__ sh,
                                             const double* __restrict__ part, int* iflags)
{
    if (iflags[0]) return;
    __shared__ double shm[NT / 64];
    const int k = it & 1;
    const double rho = block_reduce_partials(part + (P_RHO0 + k) * MAXB, nb, shm);
    const double rv = block_reduce_partials(part + (P_RV0 + k) * MAXB, nb, shm);
    if (rv == 0.0) {
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            iflags[0] = 1;
            iflags[2] = 1;
        }
        return;
    }
    const double alpha = rho / rv;
    for (int32_t i = blockIdx.x * NT + threadIdx.x; i < nf; i += gridDim.x * NT) {
        const double si = fma(-alpha, v[i], r[i]);
        s[i] = si;
        if (JAC) sh[i] = dinv[i] * si;
    }
}

__global__ __launch_bounds__(NT) void k_bi_x(int32_t nf, int32_t it, int32_t nb,
                                             double* __restrict__ w, double* __restrict__ r,
                                             const double* __restrict__ rh,
                                             const double* __restrict__ ph,
                                             const double* __restrict__ s,
                                             const double* __restrict__ sh,
                                             const double* __restrict__ t,
                                             double* __restrict__ part, int* iflags)
{
    if (iflags[0]) return;
    __shared__ double shm[NT / 64];
    const int k = it & 1;
    const double rho = block_reduce_partials(part + (P_RHO0 + k) * MAXB, nb, shm);
    const double rv = block_reduce_partials(part + (P_RV0 + k) * MAXB, nb, shm);
    const double ts = block_reduce_partials(part + (P_TS0 + k) * MAXB, nb, shm);
    const double tt = block_reduce_partials(part + (P_TT0 + k) * MAXB, nb, shm);
    const double alpha = rho / rv, om = tt != 0.0 ? ts / tt : 0.0;
    double s_rho = 0.0, s_rr = 0.0;
    for (int32_t i = blockIdx.x * NT + threadIdx.x; i < nf; i += gridDim.x * NT) {
        w[i] = fma(om, sh[i], fma(alpha, ph[i], w[i]));
        const double ri = fma(-om, t[i], s[i]);
        r[i] = ri;
        s_rho = fma(rh[i], ri, s_rho);
        s_rr = fma(ri, ri, s_rr);
    }
    const double t0 = phf_block_sum_f64<NT>(s_rho, shm);
    const double t1 = phf_block_sum_f64<NT>(s_rr, shm);
    if (threadIdx.x == 0) {
        part[(P_RHO0 + (k ^ 1)) * MAXB + blockIdx.x] = t0;
        part[P_RR * MAXB + blockIdx.x] = t1;
        if (blockIdx.x == 0) iflags[1] += 1;
    }
}

}  // namespace

// ---------------------------------------------------------------------------

void phf_ns_destroy(phf_ns* ns)
{
    if (!ns) return;
    if (ns->mg) phf_mg_destroy(ns->mg);
    phf_dfree(ns->ell_col);
    phf_dfree(ns->rec); phf_dfree(ns->Ablk);
    phf_dfree(ns->ell_val); phf_dfree(ns->dinv); phf_dfree(ns->kv); phf_dfree(ns->cs);
    phf_dfree(ns->b); phf_dfree(ns->w); phf_dfree(ns->r); phf_dfree(ns->z);
    phf_dfree(ns->p); phf_dfree(ns->q); phf_dfree(ns->part);
    phf_dfree(ns->scal);  // (the flags share its allocation)
    phf_dfree(ns->jflag);
    phf_dfree(ns->rh); phf_dfree(ns->s); phf_dfree(ns->sh); phf_dfree(ns->t);
    delete ns;
}

int phf_ns_create(phf_mesh* mesh, phf_ns** out)
{
    phf_ctx* ctx = mesh->ctx;
    phf_ns* ns = new (std::nothrow) phf_ns;
    if (!ns) return phf_set_error(ctx, PHF_ENOMEM, "host allocation failed");
    ns->mesh = mesh;
    ns->nE = mesh->nE;
    ns->nf = mesh->n_free;
    ns->L = mesh->L;
    ns->nbv = (int32_t)std::min<int64_t>(std::max<int64_t>(nblk(ns->nf), 1), MAXB);
    ns->elem_red = mesh->elem_red;
    ns->elem_row = mesh->elem_row;
    const size_t e3 = 3 * (size_t)ns->nE, nf = ns->nf;
    int rc = 0;
    rc = rc ? rc : phf_dmalloc(ctx, &ns->ell_col, 4 * nf, "solver ELL columns");
    rc = rc ? rc : phf_dmalloc(ctx, &ns->rec, 24 * std::max<size_t>(ns->nE, 1),
                               "solver half-row records");
    rc = rc ? rc : phf_dmalloc(ctx, &ns->ell_val, 5 * nf, "solver ELL values");
    rc = rc ? rc : phf_dmalloc(ctx, &ns->dinv, nf, "solver diagonal");
    rc = rc ? rc : phf_dmalloc(ctx, &ns->kv, e3, "solver known values");
    rc = rc ? rc : phf_dmalloc(ctx, &ns->cs, e3, "solver element rhs");
    rc = rc ? rc : phf_dmalloc(ctx, &ns->b, nf, "solver rhs");
    rc = rc ? rc : phf_dmalloc(ctx, &ns->w, nf, "solver x");
    rc = rc ? rc : phf_dmalloc(ctx, &ns->r, nf, "solver r");
    rc = rc ? rc : phf_dmalloc(ctx, &ns->z, nf, "solver z");
    rc = rc ? rc : phf_dmalloc(ctx, &ns->p, nf, "solver p");
    rc = rc ? rc : phf_dmalloc(ctx, &ns->q, nf, "solver q");
    rc = rc ? rc : phf_dmalloc(ctx, &ns->part, P_NARR * MAXB, "solver partials");
    // the scalars and, behind them, the flags: one block, read back at once
    rc = rc ? rc : phf_dmalloc(ctx, &ns->scal, NS_NSCAL + 2, "solver scalars and flags");
    if (!rc) ns->iflags = reinterpret_cast<int*>(ns->scal + NS_NSCAL);
    rc = rc ? rc : phf_dmalloc(ctx, &ns->jflag, 1, "solver jump flag");
    if (rc) {
        phf_ns_destroy(ns);
        return rc;
    }
    auto launch = [&]() -> int {
        PHF_HIP(ctx, hipMemsetAsync(ns->w, 0, sizeof(double) * std::max<size_t>(nf, 1), ctx->stream));
        PHF_HIP(ctx, hipMemsetAsync(ns->jflag, 0, sizeof(int), ctx->stream));
        PHF_HIP(ctx, hipMemsetAsync(ns->iflags, 0, 4 * sizeof(int), ctx->stream));
        return PHF_OK;
    };
    rc = launch();
    if (rc) {
        phf_ns_destroy(ns);
        return rc;
    }
    *out = ns;
    return PHF_OK;
}

int phf_ns_operator(phf_ns* ns, const double* K, const double* M, double cK, double cM,
                    const double* D, double cD, bool borrow_K)
{
    phf_mesh* mesh = ns->mesh;
    phf_ctx* ctx = mesh->ctx;
    // A = K: the element blocks are K's own (no copy)
    const bool alias = borrow_K && cK == 1.0 && cM == 0.0 && !D;
    if (!alias && !ns->Ablk) TRY(phf_dmalloc(ctx, &ns->Ablk, 9 * (size_t)ns->nE, "solver blocks"));
    ns->A = alias ? K : ns->Ablk;
    auto* rec = reinterpret_cast<phf_i4*>(ns->rec);
    PHF_LAUNCH(ctx, "k_ns_elem", k_ns_elem, nblk(ns->nE), NT, 0, ns->nE, K, alias ? nullptr : M, D,
               cK, cM, cD, mesh->elem_red, alias ? nullptr : ns->Ablk, rec);
    // with a multigrid preconditioner about to be set up for this operator,
    // its finest-level rows are written in the same pass
    const bool fine = ns->mg && ns->fuse_fine_rows && ns->nf > 0;
    ns->fuse_fine_rows = false;
    phf_mg_rows fr{};
    if (fine) TRY(phf_mg_fine_rows(ns->mg, &fr));
    else if (ns->mg) ns->mg->fine_rows_ready = false;
    if (ns->nf > 0)
        PHF_LAUNCH(ctx, "k_ns_ellrows", fine ? k_ns_ellrows<true> : k_ns_ellrows<false>,
                   nblk(ns->nf), NT, 0, ns->nf, mesh->red_edge, mesh->edge_elems, mesh->led,
                   mesh->ledTN, rec, ns->ell_col, ns->ell_val, ns->dinv, fr);
    return PHF_OK;
}

int phf_ns_rhs(phf_ns* ns, const double* rhs1, const double* rhs2, bool all_jumps,
               const double* hs_elem)
{
    phf_mesh* mesh = ns->mesh;
    phf_ctx* ctx = mesh->ctx;
    if (ns->L > 0 && !all_jumps)
        PHF_LAUNCH(ctx, "k_ns_jumpflag", k_ns_jumpflag,
                   (unsigned)std::min<int64_t>(nblk(ns->L), 1024), NT, 0, ns->L, mesh->row_nodes,
                   rhs2, ns->jflag);
    PHF_LAUNCH(ctx, "k_ns_known", k_ns_known, nblk(ns->nE), NT, 0, ns->nE, mesh->ecode,
               ns->elem_row, mesh->row_hs, rhs1, rhs2, ns->A, ns->jflag, all_jumps ? 1 : 0,
               hs_elem, ns->kv, ns->cs);
    if (ns->nf > 0)
        PHF_LAUNCH(ctx, "k_ns_gather", k_ns_gather, nblk(ns->nf), NT, 0, ns->nf, mesh->red_edge,
                   mesh->edge_elems, mesh->led, mesh->ledTN, ns->cs, ns->b, ns->jflag);
    return PHF_OK;
}

int phf_ns_zero_w(phf_ns* ns)
{
    phf_ctx* ctx = ns->mesh->ctx;
    PHF_HIP(ctx, hipMemsetAsync(ns->w, 0, sizeof(double) * std::max<int32_t>(ns->nf, 1), ctx->stream));
    return PHF_OK;
}

int phf_ns_cg_start(phf_ns* ns, double rtol, bool zero_start)
{
    phf_ctx* ctx = ns->mesh->ctx;
    ns->next_it = 0;
    if (ns->nf == 0) {
        PHF_HIP(ctx, hipMemsetAsync(ns->iflags, 0, 4 * sizeof(int), ctx->stream));
        return PHF_OK;
    }
    const bool mg = ns->mg && ns->mg_on;
    auto init = mg ? (zero_start ? k_cg_init<false, true> : k_cg_init<false, false>)
                   : (zero_start ? k_cg_init<true, true> : k_cg_init<true, false>);
    PHF_LAUNCH(ctx, "k_cg_init", init, ns->nbv, NT, 0, ns->nf, ns->ell_col, ns->ell_val, ns->dinv,
               ns->b, ns->w, ns->r, ns->z, ns->p, ns->q, ns->part);
    PHF_LAUNCH(ctx, "k_cg_init_final", k_cg_init_final, 1, NT, 0, ns->part, ns->nbv, rtol * rtol,
               ns->scal, ns->iflags);
    if (ns->mg && ns->mg_on)
        TRY(phf_mg_apply32(ns->mg, ns->r, false, ns->part + P_RZ0 * MAXB, ns->iflags));
    return PHF_OK;
}

int phf_ns_cg_iterate(phf_ns* ns, int32_t iters)
{
    phf_ctx* ctx = ns->mesh->ctx;
    if (ns->nf == 0) return PHF_OK;
    for (int32_t k = 0; k < iters; ++k) {
        // only the parity and "first or not" of the index matter to the kernels
        const int32_t it = ns->next_it;
        ns->next_it = it + 1 >= 2 ? 2 + ((it + 1) & 1) : it + 1;
        if (ns->mg && ns->mg_on) {
            PHF_LAUNCH(ctx, "k_cg_dir", k_cg_dir<float>, ns->nbv, NT, 0, ns->nf, it, ns->nbv,
                       ns->ell_col, ns->ell_val, ns->mg->z32, ns->p, ns->q, ns->part, ns->scal,
                       ns->iflags);
            const phf_mg_top top = phf_mg_top_view(ns->mg);
            PHF_LAUNCH(ctx, "k_cg_upd", k_cg_upd_mg, ns->nbv, NT, 0, ns->nf, it, ns->nbv, ns->w,
                       ns->r, ns->p, ns->q, ns->part, ns->iflags, top.dinv, top.w, top.bh,
                       top.x);
            PHF_LAUNCH(ctx, "k_cg_check", k_cg_check, 1, NT, 0, ns->nbv, ns->part, ns->scal,
                       ns->iflags);
            TRY(phf_mg_apply32(ns->mg, ns->r, true, ns->part + ((it & 1) ? P_RZ0 : P_RZ1) * MAXB,
                               ns->iflags));
        } else {
            PHF_LAUNCH(ctx, "k_cg_dir", k_cg_dir<double>, ns->nbv, NT, 0, ns->nf, it, ns->nbv,
                       ns->ell_col, ns->ell_val, ns->z, ns->p, ns->q, ns->part, ns->scal,
                       ns->iflags);
            PHF_LAUNCH(ctx, "k_cg_upd", k_cg_upd<true>, ns->nbv, NT, 0, ns->nf, it, ns->nbv, ns->w,
                       ns->r, ns->z, ns->p, ns->q, ns->dinv, ns->part, ns->iflags);
        }
    }
    if (!(ns->mg && ns->mg_on))
        PHF_LAUNCH(ctx, "k_cg_check", k_cg_check, 1, NT, 0, ns->nbv, ns->part, ns->scal,
                   ns->iflags);
    return PHF_OK;
}

int phf_ns_recover(phf_ns* ns, const double* rhs1, double* U, double* mu, double mu_scale)
{
    phf_mesh* mesh = ns->mesh;
    phf_ctx* ctx = mesh->ctx;
    const bool with_mu = mu && ns->L > 0;
    PHF_LAUNCH(ctx, "k_ns_recover_u", with_mu ? k_ns_recover_u<true> : k_ns_recover_u<false>,
               nblk(ns->nE), NT, 0, ns->nE, ns->elem_red, ns->w, ns->kv, ns->A, rhs1, U, ns->cs);
    if (mu && ns->L > 0)
        PHF_LAUNCH(ctx, "k_ns_recover_mu", k_ns_recover_mu, nblk(ns->L), NT, 0, ns->L,
                   mesh->row_edge, mesh->edge_elems, mesh->led, mesh->row_hs, ns->cs, mu_scale,
                   mu);
    return PHF_OK;
}

// Iterations to issue before the next convergence test when the caller leaves
// the period to the solver (multigrid): from the mean reduction of the
// residual norm per iteration so far, the number m still needed to reach the
// tolerance, less one, so that at most about one iteration runs past
// convergence; 1 until there is a rate to go by. rr0, rr: squared residual
// norms at the start and now; goal: the squared norm to reach.
static int32_t predicted_block(int32_t done, double rr0, double rr, double goal)
{
    if (done <= 0 || !(rr0 > 0.0) || !(rr > 0.0) || !(rr < rr0) || !(goal > 0.0) || rr <= goal)
        return 1;
    const double q = std::pow(rr / rr0, 0.5 / done);  // per-iteration factor on the norm
    if (!(q < 0.95)) return 1;
    const double m = std::ceil(0.5 * std::log(goal / rr) / std::log(q));
    return (int32_t)std::min(std::max(m - 1.0, 1.0), 16.0);
}

// Host-side convergence loop of phf_solve. check_every > 0: test after every
// check_every iterations; 0: the predicted schedule above. Each test reads the
// solver's scalars and flags back in one copy into pinned memory.
int phf_ns_cg_solve(phf_ns* ns, double rtol, int32_t max_iter, int32_t check_every,
                    int32_t* iters_out, double* relres_out, int* converged, bool zero_start)
{
    phf_ctx* ctx = ns->mesh->ctx;
    TRY(phf_ns_cg_start(ns, rtol, zero_start));
    if (ns->nf == 0) {
        // no free unknowns: the reduced system is empty and solved as it is
        // (nothing was launched that writes the scalars read below)
        if (iters_out) *iters_out = 0;
        if (relres_out) *relres_out = 0.0;
        if (converged) *converged = 1;
        return PHF_OK;
    }
    double* h = reinterpret_cast<double*>(ctx->h_pinned);
    const int* hf = reinterpret_cast<const int*>(h + NS_NSCAL);
    auto read_back = [&]() -> int {
        PHF_HIP(ctx, hipMemcpyAsync(h, ns->scal, (NS_NSCAL + 2) * sizeof(double),
                                    hipMemcpyDeviceToHost, ctx->stream));
        PHF_HIP(ctx, hipStreamSynchronize(ctx->stream));
        return PHF_OK;
    };
    TRY(read_back());
    const double rr0 = h[NS_RR];
    int32_t done_iters = 0;
    while (!hf[0] && done_iters < max_iter) {
        int32_t n = check_every > 0 ? check_every
                                    : predicted_block(done_iters, rr0, h[NS_RR], h[NS_TOL2] * h[NS_BB]);
        n = std::min(n, max_iter - done_iters);
        TRY(phf_ns_cg_iterate(ns, n));
        done_iters += n;
        TRY(read_back());
    }
    if (iters_out) *iters_out = hf[1];
    if (relres_out) *relres_out = h[NS_BB] > 0 ? std::sqrt(h[NS_RR] / h[NS_BB]) : 0.0;
    if (converged) *converged = hf[0];
    return PHF_OK;
}

namespace {
int bicg_start(phf_ns* ns, double rtol)
{
    phf_ctx* ctx = ns->mesh->ctx;
    ns->next_it = 0;
    if (ns->nf == 0) {
        PHF_HIP(ctx, hipMemsetAsync(ns->iflags, 0, 4 * sizeof(int), ctx->stream));
        return PHF_OK;
    }
    const size_t nf = ns->nf;
    if (!ns->rh) {
        TRY(phf_dmalloc(ctx, &ns->rh, nf, "solver shadow residual"));
        TRY(phf_dmalloc(ctx, &ns->s, nf, "solver s"));
        TRY(phf_dmalloc(ctx, &ns->sh, nf, "solver preconditioned s"));
        TRY(phf_dmalloc(ctx, &ns->t, nf, "solver t"));
    }
    // p -> ns->p, ph -> ns->z, v -> ns->q
    PHF_LAUNCH(ctx, "k_bi_init", k_bi_init, ns->nbv, NT, 0, ns->nf, ns->ell_col, ns->ell_val,
               ns->b, ns->w, ns->r, ns->rh, ns->p, ns->q, ns->part);
    PHF_LAUNCH(ctx, "k_cg_init_final", k_cg_init_final, 1, NT, 0, ns->part, ns->nbv, rtol * rtol,
               ns->scal, ns->iflags);
    return PHF_OK;
}

int bicg_iterate(phf_ns* ns, int32_t iters)
{
    phf_ctx* ctx = ns->mesh->ctx;
    if (ns->nf == 0) return PHF_OK;
    const bool mg = ns->mg && ns->mg_on;
    for (int32_t q = 0; q < iters; ++q) {
        const int32_t it = ns->next_it;
        ns->next_it = it + 1 >= 2 ? 2 + ((it + 1) & 1) : it + 1;
        const int k = it & 1;
        if (mg)
            PHF_LAUNCH(ctx, "k_bi_dir", k_bi_dir<false>, ns->nbv, NT, 0, ns->nf, it, ns->nbv,
                       ns->r, ns->p, ns->q, ns->dinv, ns->z, ns->part, ns->scal, ns->iflags);
        else
            PHF_LAUNCH(ctx, "k_bi_dir", k_bi_dir<true>, ns->nbv, NT, 0, ns->nf, it, ns->nbv,
                       ns->r, ns->p, ns->q, ns->dinv, ns->z, ns->part, ns->scal, ns->iflags);
        if (mg) TRY(phf_mg_apply(ns->mg, ns->p, ns->z, ns->part + P_SCR * MAXB, ns->iflags));
        PHF_LAUNCH(ctx, "k_bi_spmv", k_bi_spmv, ns->nbv, NT, 0, ns->nf, ns->ell_col, ns->ell_val,
                   ns->z, ns->q, ns->rh, ns->part, P_RV0 + k, -1, ns->iflags);
        if (mg)
            PHF_LAUNCH(ctx, "k_bi_s", k_bi_s<false>, ns->nbv, NT, 0, ns->nf, it, ns->nbv, ns->r,
                       ns->q, ns->dinv, ns->s, ns->sh, ns->part, ns->iflags);
        else
            PHF_LAUNCH(ctx, "k_bi_s", k_bi_s<true>, ns->nbv, NT, 0, ns->nf, it, ns->nbv, ns->r,
                       ns->q, ns->dinv, ns->s, ns->sh, ns->part, ns->iflags);
        if (mg) TRY(phf_mg_apply(ns->mg, ns->s, ns->sh, ns->part + P_SCR * MAXB, ns->iflags));
        PHF_LAUNCH(ctx, "k_bi_spmv", k_bi_spmv, ns->nbv, NT, 0, ns->nf, ns->ell_col, ns->ell_val,
                   ns->sh, ns->t, ns->s, ns->part, P_TS0 + k, P_TT0 + k, ns->iflags);
        PHF_LAUNCH(ctx, "k_bi_x", k_bi_x, ns->nbv, NT, 0, ns->nf, it, ns->nbv, ns->w, ns->r,
                   ns->rh, ns->z, ns->s, ns->sh, ns->t, ns->part, ns->iflags);
    }
    PHF_LAUNCH(ctx, "k_cg_check", k_cg_check, 1, NT, 0, ns->nbv, ns->part, ns->scal, ns->iflags);
    return PHF_OK;
}
}  // namespace

// Runs after a breakdown at most: each restarts the iteration from the
// current iterate, with its residual (recomputed) as the new shadow residual.
constexpr int BICG_RESTARTS = 8;

int phf_ns_bicg_solve(phf_ns* ns, double rtol, int32_t max_iter, int32_t check_every,
                      int32_t* iters_out, double* relres_out, int* converged, int* breakdown)
{
    phf_ctx* ctx = ns->mesh->ctx;
    int32_t prior = 0;  // iterations of the runs that broke down
    int hf[3] = {0, 0, 0};
    for (int run = 0;; ++run) {
        TRY(bicg_start(ns, rtol));
        PHF_HIP(ctx, hipMemcpyAsync(hf, ns->iflags, 3 * sizeof(int), hipMemcpyDeviceToHost,
                                    ctx->stream));
        PHF_HIP(ctx, hipStreamSynchronize(ctx->stream));
        int32_t done_iters = prior;
        while (!hf[0] && done_iters < max_iter) {
            int32_t n = std::min(check_every, max_iter - done_iters);
            TRY(bicg_iterate(ns, n));
            done_iters += n;
            PHF_HIP(ctx, hipMemcpyAsync(hf, ns->iflags, 3 * sizeof(int), hipMemcpyDeviceToHost,
                                        ctx->stream));
            PHF_HIP(ctx, hipStreamSynchronize(ctx->stream));
        }
        if (!hf[2] || run == BICG_RESTARTS || prior + hf[1] >= max_iter) break;
        prior += hf[1];
    }
    double sc[NS_NSCAL] = {0};
    if (ns->nf > 0) {
        PHF_HIP(ctx, hipMemcpyAsync(sc, ns->scal, sizeof(sc), hipMemcpyDeviceToHost, ctx->stream));
        PHF_HIP(ctx, hipStreamSynchronize(ctx->stream));
    }
    if (iters_out) *iters_out = prior + hf[1];
    if (relres_out) *relres_out = sc[NS_BB] > 0 ? std::sqrt(sc[NS_RR] / sc[NS_BB]) : 0.0;
    if (breakdown) *breakdown = ns->nf == 0 ? 0 : hf[2];
    if (converged) *converged = ns->nf == 0 ? 1 : (hf[0] && !hf[2]);
    return PHF_OK;
}

int phf_ns_prepare_precond(phf_ns* ns, int32_t precond, const phf_mg_params& mp)
{
    if (precond != PHF_PRECOND_MULTIGRID) return PHF_OK;
    phf_ctx* ctx = ns->mesh->ctx;
    if (mp.sweeps < 0 || mp.sweeps > PHF_MG_MAX_SWEEPS)
        return phf_set_error(ctx, PHF_EINVAL, "multigrid sweeps %d outside 0..%d", mp.sweeps,
                             PHF_MG_MAX_SWEEPS);
    if (mp.smoother != PHF_MG_SMOOTH_DEFAULT && mp.smoother != PHF_MG_SMOOTH_JACOBI &&
        mp.smoother != PHF_MG_SMOOTH_CHEBYSHEV)
        return phf_set_error(ctx, PHF_EINVAL, "unknown multigrid smoother %d", mp.smoother);
    if (mp.range != 0.0 && !(mp.range > 1.0))
        return phf_set_error(ctx, PHF_EINVAL, "Chebyshev range must exceed 1 (got %g)", mp.range);
    if (!(mp.omega >= 0.0))
        return phf_set_error(ctx, PHF_EINVAL, "negative Jacobi damping %g", mp.omega);
    if (!ns->mg) TRY(phf_mg_create(ns, &ns->mg, mp.drop_coarse));
    const bool jacobi = mp.smoother == PHF_MG_SMOOTH_JACOBI;
    ns->mg->smoother = jacobi ? PHF_MG_SMOOTH_JACOBI : PHF_MG_SMOOTH_CHEBYSHEV;
    ns->mg->nu = mp.sweeps > 0 ? mp.sweeps : jacobi ? 2 : 4;
    ns->mg->omega = mp.omega > 0 ? mp.omega : 0.8;
    ns->mg->range = mp.range > 0 ? mp.range : 10.0;
    return PHF_OK;
}

int phf_ns_set_precond(phf_ns* ns, int32_t precond, const phf_mg_params& mp,
                       const phf_coeffs* co, double cK, double cM)
{
    ns->mg_on = false;
    if (precond != PHF_PRECOND_MULTIGRID) return PHF_OK;
    TRY(phf_ns_prepare_precond(ns, precond, mp));
    TRY(phf_mg_numeric(ns->mg, co, cK, cM));
    ns->mg_on = true;
    return PHF_OK;
}

int phf_ns_get(phf_mesh* mesh, phf_ns** out)
{
    if (!mesh->ns) TRY(phf_ns_create(mesh, &mesh->ns));
    *out = mesh->ns;
    return PHF_OK;
}

namespace {
__global__ __launch_bounds__(NT) void k_concat(const double* __restrict__ a, int32_t na,
                                               const double* __restrict__ b, int32_t nbn,
                                               double* __restrict__ out)
{
    int64_t g = (int64_t)blockIdx.x * NT + threadIdx.x;
    if (g < na) out[g] = a[g];
    else if (g < (int64_t)na + nbn) out[g] = b[g - na];
}
}  // namespace

extern "C" int phf_solve(phf_mesh* mesh, const phf_coeffs* co, const phf_system* sys,
                         const phf_solver_opts* opts, double* U, double* Lambda,
                         phf_solve_stats* stats)
{
    if (!mesh) return PHF_EINVAL;
    phf_ctx* ctx = mesh->ctx;
    if (!co || !sys || !U || !sys->K || !sys->M || !sys->C || !sys->F || !sys->bD)
        return phf_set_error(ctx, PHF_EINVAL, "phf_solve: K, M, C, F, bD and U are required");
    const bool conv_term = co->p[0] != 0.0 || co->p[1] != 0.0;
    phf_solver_opts o{};
    o.method = PHF_SOLVER_NULLSPACE_CG;
    if (opts) o = *opts;
    if (o.max_iter <= 0) o.max_iter = 20000;
    if (o.rtol <= 0) o.rtol = 1e-10;
    // with the multigrid preconditioner, conjugate gradients predict how many
    // iterations to issue between tests (0); BiCGSTAB tests after each one
    if (o.check_every <= 0)
        o.check_every = o.precond == PHF_PRECOND_MULTIGRID && o.method == PHF_SOLVER_NULLSPACE_CG ? 0
                        : o.precond == PHF_PRECOND_MULTIGRID                                      ? 1
                                                                                                  : 8;
    if (o.method != PHF_SOLVER_NULLSPACE_CG && o.method != PHF_SOLVER_NULLSPACE_BICGSTAB)
        return phf_set_error(ctx, PHF_EINVAL, "phf_solve: unknown method %d", o.method);
    if (conv_term && o.method == PHF_SOLVER_NULLSPACE_CG)
        return phf_set_error(ctx, PHF_EINVAL,
                             "phf_solve: p != 0 makes the system nonsymmetric; use "
                             "PHF_SOLVER_NULLSPACE_BICGSTAB");
    if (conv_term && !sys->D)
        return phf_set_error(ctx, PHF_EINVAL, "phf_solve: p != 0 needs the assembled D");
    if (o.precond != PHF_PRECOND_JACOBI && o.precond != PHF_PRECOND_MULTIGRID)
        return phf_set_error(ctx, PHF_EINVAL, "phf_solve: unknown preconditioner %d", o.precond);
    if (o.saddle_rtol < 0 || (o.saddle_rtol > 0 && (!sys->S || !Lambda)))
        return phf_set_error(ctx, PHF_EINVAL,
                             "phf_solve: saddle_rtol must be >= 0 and needs S and Lambda");
    if (o.saddle_rtol > 0 && o.method != PHF_SOLVER_NULLSPACE_CG)
        return phf_set_error(ctx, PHF_EINVAL, "phf_solve: saddle_rtol needs conjugate gradients");
    phf_ns* ns = nullptr;
    TRY(phf_ns_get(mesh, &ns));
    // the operator below may read the element blocks from the caller's K;
    // the cached workspace does not keep that pointer past this call
    struct forget_A {
        phf_ns* ns;
        ~forget_A() { ns->A = nullptr; }
    } forget{ns};
    phf_mg_params mp;
    mp.sweeps = o.mg_sweeps;
    mp.smoother = o.mg_smoother;
    mp.omega = o.mg_omega;
    mp.range = o.mg_range;
    // the multigrid hierarchy exists before the operator, so that the
    // operator kernel writes its finest rows too
    TRY(phf_ns_prepare_precond(ns, o.precond, mp));
    ns->fuse_fine_rows = o.precond == PHF_PRECOND_MULTIGRID;
    // (K stays the caller's until the recovery below, so A = K is not copied)
    TRY(phf_ns_operator(ns, sys->K, sys->M, 1.0, co->delta, conv_term ? sys->D : nullptr, 1.0,
                        true));
    TRY(phf_ns_set_precond(ns, o.precond, mp, co, 1.0, co->delta));
    TRY(phf_ns_rhs(ns, sys->F, sys->bD));
    // both iterations start from w = 0 (the CG initialisation writes it)
    if (o.method == PHF_SOLVER_NULLSPACE_BICGSTAB) TRY(phf_ns_zero_w(ns));
    int32_t iters = 0;
    double relres = 0;
    int conv = 0, brk = 0;
    if (o.method == PHF_SOLVER_NULLSPACE_BICGSTAB)
        TRY(phf_ns_bicg_solve(ns, o.rtol, o.max_iter, o.check_every, &iters, &relres, &conv, &brk));
    else
        TRY(phf_ns_cg_solve(ns, o.rtol, o.max_iter, o.check_every, &iters, &relres, &conv, true));
    TRY(phf_ns_recover(ns, sys->F, U, Lambda, 1.0));
    double srel = -1.0;
    if ((o.saddle_residual || o.saddle_rtol > 0) && sys->S && Lambda) {
        const int32_t N = 3 * mesh->nE, L = mesh->L;
        double *W = nullptr, *Fv = nullptr, *R = nullptr;
        TRY(phf_dmalloc(ctx, &W, (size_t)N + L, "residual W"));
        int rc = phf_dmalloc(ctx, &Fv, (size_t)N + L, "residual F");
        if (!rc) rc = phf_dmalloc(ctx, &R, 2, "residual norms");
        double* part = ns->part;
        // ||F_vec - M_vec W|| / ||F_vec|| of the current U, Lambda
        auto saddle = [&]() -> int {
            PHF_LAUNCH(ctx, "k_concat", k_concat, nblk((int64_t)N + L), NT, 0, U, N, Lambda, L, W);
            PHF_LAUNCH(ctx, "k_concat", k_concat, nblk((int64_t)N + L), NT, 0, sys->F, N, sys->bD, L, Fv);
            // Fv <- M_vec W - F_vec
            TRY(phf_spmv(ctx, N + L, mesh->S_rowptr, mesh->S_col, sys->S, 1.0, W, -1.0, Fv));
            TRY(phf_dot(ctx, Fv, Fv, N + L, part, R));
            PHF_LAUNCH(ctx, "k_concat", k_concat, nblk((int64_t)N + L), NT, 0, sys->F, N, sys->bD, L, W);
            TRY(phf_dot(ctx, W, W, N + L, part, R + 1));
            double h[2];
            PHF_HIP(ctx, hipMemcpyAsync(h, R, sizeof(h), hipMemcpyDeviceToHost, ctx->stream));
            PHF_HIP(ctx, hipStreamSynchronize(ctx->stream));
            srel = h[1] > 0 ? std::sqrt(h[0] / h[1]) : std::sqrt(h[0]);
            return PHF_OK;
        };
        if (!rc) rc = saddle();
        // Saddle-residual target: the reduced residual appears in the first
        // block row of the saddle system, scaled by ||b_red|| / ||F_vec||,
        // which need not be near 1 (loads scale with |T|, the reduced
        // right-hand side with a_T u_D next to Dirichlet edges). Tighten the
        // reduced tolerance by the observed ratio and continue conjugate
        // gradients from the current iterate until the saddle residual meets
        // the target (at most SADDLE_PASSES more passes).
        // The saddle residual cannot fall below the rounding of its own
        // evaluation, about eps ||(|M_vec| |W|)|| / ||F_vec||, which grows
        // like 1/h: a pass that does not halve it stops the loop.
        constexpr int SADDLE_PASSES = 6;
        for (int pass = 0; !rc && o.saddle_rtol > 0 && srel > o.saddle_rtol && !brk &&
                           o.method == PHF_SOLVER_NULLSPACE_CG && pass < SADDLE_PASSES;
             ++pass) {
            const double r_next = relres > 0 ? 0.5 * relres * o.saddle_rtol / srel : 0.1 * o.rtol;
            const double before = srel;
            int32_t it2 = 0;
            rc = phf_ns_cg_solve(ns, r_next, std::max(o.max_iter - iters, 1), o.check_every, &it2,
                                 &relres, &conv, false);
            iters += it2;
            if (!rc) rc = phf_ns_recover(ns, sys->F, U, Lambda, 1.0);
            if (!rc) rc = saddle();
            if (!conv || srel > 0.5 * before) break;
        }
        (void)hipStreamSynchronize(ctx->stream);
        phf_dfree(W);
        phf_dfree(Fv);
        phf_dfree(R);
        if (rc) return rc;
        if (o.saddle_rtol > 0 && srel > o.saddle_rtol) conv = 0;
    }
    if (stats) {
        stats->iterations = iters;
        stats->converged = conv;
        stats->rel_residual = relres;
        stats->saddle_rel_residual = srel;
    }
    if (brk)
        return phf_set_error(ctx, PHF_ENOCONV,
                             "phf_solve: BiCGSTAB breakdown after %d iterations, relative "
                             "residual %.3e",
                             iters, relres);
    if (!conv && o.saddle_rtol > 0 && srel > o.saddle_rtol)
        return phf_set_error(ctx, PHF_ENOCONV,
                             "phf_solve: saddle residual %.3e above %.3e after %d iterations "
                             "(reduced residual %.3e)",
                             srel, o.saddle_rtol, iters, relres);
    if (!conv)
        return phf_set_error(ctx, PHF_ENOCONV, "phf_solve: %d iterations, relative residual %.3e",
                             iters, relres);
    return PHF_OK;
}
