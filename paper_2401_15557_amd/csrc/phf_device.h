// Device-side helpers of libphfem: wavefront/block reductions and scans
// (wave64), and the problem-data function catalogue.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "phf_internal.h"

#define PHF_PI 3.14159265358979323846

// Inclusive sum over the 64 lanes of a wavefront (lane order fixed).
template <typename T>
__device__ inline T phf_wave_inclusive_scan(T x)
{
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        T y = __shfl_up(x, d, 64);
        if (lane >= d) x += y;
    }
    return x;
}

// Exclusive block scan of one int32 per thread; *total = block sum.
// sh needs NT/64 + 1 ints. Contains barriers: call from all threads.
template <int NT>
__device__ inline int32_t phf_block_exscan_i32(int32_t v, int32_t* sh, int32_t* total)
{
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    int32_t x = phf_wave_inclusive_scan(v);
    if (lane == 63) sh[wid] = x;
    __syncthreads();
    int32_t woff = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < NT / 64; ++w) {
        int32_t s = sh[w];
        woff += (w < wid) ? s : 0;
        tot += s;
    }
    __syncthreads();
    *total = tot;
    return woff + x - v;
}

// Tree sum over a wavefront with a fixed pairing (bitwise reproducible).
template <typename T>
__device__ inline T phf_wave_sum(T x)
{
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) x += __shfl_xor(x, d, 64);
    return x;
}

template <int NT>
__device__ inline int32_t phf_block_sum_i32(int32_t v, int32_t* sh)
{
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    int32_t x = phf_wave_sum(v);
    if (lane == 0) sh[wid] = x;
    __syncthreads();
    int32_t tot = 0;
#pragma unroll
    for (int w = 0; w < NT / 64; ++w) tot += sh[w];
    __syncthreads();
    return tot;
}

// Block sum of doubles in a fixed order: wave trees, then waves in order.
template <int NT>
__device__ inline double phf_block_sum_f64(double v, double* sh)
{
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    double x = phf_wave_sum(v);
    if (lane == 0) sh[wid] = x;
    __syncthreads();
    double tot = 0.0;
#pragma unroll
    for (int w = 0; w < NT / 64; ++w) tot += sh[w];
    __syncthreads();
    return tot;
}

// Problem data (phfem.h PHF_FN_*): value at (x, y, t); flux kinds return the
// flux vector dotted with (nx, ny); PHF_FN_EDGE_ARRAY reads ev[edge].
// |E| / 2 of the edge a -> b, rounded the same way in every kernel (the mesh
// build's row records and the assembly's element-side edge lengths).
__device__ inline double phf_half_length(const double2 a, const double2 b)
{
#pragma clang fp contract(off)
    const double dx = b.x - a.x, dy = b.y - a.y;
    return 0.5 * sqrt(dx * dx + dy * dy);
}

__device__ inline double phf_fn_eval(const phf_fn_dev& f, double x, double y, double t, double nx,
                                     double ny, int32_t edge)
{
    // evaluated without fused multiply-adds, so that every kernel that
    // inlines it rounds the same way
#pragma clang fp contract(off)
    switch (f.kind) {
    case PHF_FN_ZERO: return 0.0;
    case PHF_FN_CONST: return f.c0;
    case PHF_FN_SIN_COS:
        return f.c0 * exp(f.c1 * t) * sin(PHF_PI * x) * cos(PHF_PI * y);
    case PHF_FN_SIN_SIN:
        return f.c0 * exp(f.c1 * t) * sin(PHF_PI * x) * sin(PHF_PI * y);
    case PHF_FN_GRAD_SIN_COS: {
        double sx = sin(PHF_PI * x), cx = cos(PHF_PI * x);
        double sy = sin(PHF_PI * y), cy = cos(PHF_PI * y);
        return f.c0 * exp(f.c1 * t) * (PHF_PI * cx * cy * nx - PHF_PI * sx * sy * ny);
    }
    case PHF_FN_GRAD_SIN_SIN: {
        double sx = sin(PHF_PI * x), cx = cos(PHF_PI * x);
        double sy = sin(PHF_PI * y), cy = cos(PHF_PI * y);
        return f.c0 * exp(f.c1 * t) * (PHF_PI * cx * sy * nx + PHF_PI * sx * cy * ny);
    }
    case PHF_FN_PAPER_U: return (f.c0 + f.c1 * t) * (x - x * x) * (y - y * y);
    case PHF_FN_PAPER_F: {
        double a = x - x * x, b = y - y * y, tau = f.c0 + f.c1 * t;
        return f.c1 * a * b +
               tau * (2.0 * b + 2.0 * a + (1.0 - 2.0 * x) * b + a * (1.0 - 2.0 * y) + a * b);
    }
    case PHF_FN_PAPER_FLUX: {
        double tau = f.c0 + f.c1 * t;
        double qx = (1.0 - x - x * x) * (y - y * y);
        double qy = (x - x * x) * (1.0 - y - y * y);
        return tau * (qx * nx + qy * ny);
    }
    case PHF_FN_EDGE_ARRAY: return f.ev[edge];
    default: return 0.0;
    }
}

// Gradient of the kinds that have one in closed form (ZERO, CONST, SIN_COS,
// SIN_SIN, PAPER_U); the error norms accept only these.
__device__ inline void phf_fn_grad(const phf_fn_dev& f, double x, double y, double t, double* gx,
                                   double* gy)
{
    switch (f.kind) {
    case PHF_FN_SIN_COS: {
        const double a = f.c0 * exp(f.c1 * t) * PHF_PI;
        *gx = a * cos(PHF_PI * x) * cos(PHF_PI * y);
        *gy = -a * sin(PHF_PI * x) * sin(PHF_PI * y);
        return;
    }
    case PHF_FN_SIN_SIN: {
        const double a = f.c0 * exp(f.c1 * t) * PHF_PI;
        *gx = a * cos(PHF_PI * x) * sin(PHF_PI * y);
        *gy = a * sin(PHF_PI * x) * cos(PHF_PI * y);
        return;
    }
    case PHF_FN_PAPER_U: {
        const double tau = f.c0 + f.c1 * t;
        *gx = tau * (1.0 - 2.0 * x) * (y - y * y);
        *gy = tau * (x - x * x) * (1.0 - 2.0 * y);
        return;
    }
    default:
        *gx = 0.0;
        *gy = 0.0;
    }
}

// Four-lane vectors for 16-byte row loads and stores.
typedef int32_t phf_i4 __attribute__((ext_vector_type(4)));
typedef float phf_f4 __attribute__((ext_vector_type(4)));
typedef double phf_d2 __attribute__((ext_vector_type(2)));

// Half-row records of the reduced (edge-midpoint) operator. Row r (a free
// edge) couples with the other free edges of its two triangles; each
// triangle T contributes one record to it, stored in element order at
// 3 T + l (l the row edge's local index in T): the reduced columns of T's
// two other local edges o1 < o2 (-1 where Dirichlet), the entries
// B_T[l][o1], B_T[l][o2] of T's block B_T = P^T A_T P, and B_T[l][l], its
// part of the diagonal. Layout, 32 bytes: two int32 columns and the first
// value as one 16-byte unit, the second value and the diagonal part as the
// next.
__device__ inline void phf_hrec_store(phf_i4* __restrict__ rec, int64_t slot, int32_t c1,
                                      int32_t c2, double v1, double v2, double d)
{
    const long long b = __double_as_longlong(v1);
    rec[2 * slot] = phf_i4{c1, c2, (int32_t)(b & 0xffffffffLL), (int32_t)(b >> 32)};
    *reinterpret_cast<phf_d2*>(rec + 2 * slot + 1) = phf_d2{v2, d};
}

// The records of element m (its block Bm, row-major, and the reduced rows
// red[] of its local edges; none for a Dirichlet local edge).
__device__ inline void phf_hrec_element(phf_i4* __restrict__ rec, int64_t m, const int32_t red[3],
                                        const double Bm[9])
{
#pragma unroll
    for (int l = 0; l < 3; ++l) {
        if (red[l] < 0) continue;
        const int o1 = l == 0 ? 1 : 0, o2 = l == 2 ? 1 : 2;
        phf_hrec_store(rec, 3 * m + l, red[o1], red[o2], Bm[3 * l + o1], Bm[3 * l + o2],
                       Bm[4 * l]);
    }
}

// Row r (free edge e) from the records of its T+ and T- (tt, with the edge's
// local indices lp, ln; no T-: a boundary edge) as five (column, value)
// slots: the diagonal (the two parts summed) and the off-diagonal entries,
// sorted by column, then the unused slots (column r, value 0); returns the
// number of entries. An off-diagonal value is its one source plus zero, and
// a boundary row's diagonal its T+ part plus zero, as when each entry sums
// its sources over both sides with zero for an absent one. The columns are
// distinct, so a fixed five-input sorting network gives the unique order.
__device__ inline int phf_hrec_row(int32_t r, int2 tt, int lp, int ln,
                                   const phf_i4* __restrict__ rec, int32_t col[5], double v[5])
{
    const int64_t pa = 2 * (3 * (int64_t)tt.x + lp);
    const phf_i4 a0 = rec[pa];
    const phf_d2 a1 = *reinterpret_cast<const phf_d2*>(rec + pa + 1);
    phf_i4 b0 = phf_i4{-1, -1, 0, 0};
    phf_d2 b1 = phf_d2{0.0, 0.0};
    if (tt.y >= 0) {
        const int64_t pb = 2 * (3 * (int64_t)tt.y + ln);
        b0 = rec[pb];
        b1 = *reinterpret_cast<const phf_d2*>(rec + pb + 1);
    }
    auto first = [](const phf_i4 u) {
        return __longlong_as_double(((long long)u.w << 32) | (long long)(uint32_t)u.z);
    };
    constexpr int32_t NONE = 0x7fffffff;  // sorts after every column
    const int32_t cc[4] = {a0.x, a0.y, b0.x, b0.y};
    const double vv[4] = {first(a0), a1.x, first(b0), b1.x};
    col[0] = r;
    v[0] = a1.y + b1.y;
    int n = 1;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const bool used = cc[k] >= 0;
        col[k + 1] = used ? cc[k] : NONE;
        v[k + 1] = used ? vv[k] + 0.0 : 0.0;
        n += used ? 1 : 0;
    }
    auto cx = [&](int i, int j) {
        if (col[i] > col[j]) {
            const int32_t c = col[i];
            col[i] = col[j];
            col[j] = c;
            const double x = v[i];
            v[i] = v[j];
            v[j] = x;
        }
    };
    cx(0, 1); cx(3, 4); cx(2, 4); cx(2, 3); cx(1, 4); cx(0, 3); cx(0, 2); cx(1, 3); cx(1, 2);
#pragma unroll
    for (int k = 0; k < 5; ++k)
        if (col[k] == NONE) col[k] = r;
    return n;
}

// Single-precision scaled copy of row r of a reduced operator given as five
// (column, value) slots, unused ones holding column r and value 0: the
// off-diagonal entries of D^-1 A in slot order (a free edge has at most four
// neighbours; the remaining slots get column r and value 0), the diagonal
// a_rr and its inverse (1 where a_rr <= 0, as for the double-precision
// inverse diagonal), stored row-major (the row's four columns at col4[4r..],
// its four values at val4[4r..]; n is unused; col4 null: the columns are
// already there). Returns the row's Gershgorin sum 1 + sum_j |a_ij| / a_ii in
// single precision.
__device__ inline float phf_scale_row(int32_t r, int32_t n, const int32_t* c, const double* v,
                                      int32_t* __restrict__ col4, float* __restrict__ val4,
                                      float* __restrict__ diag, float* __restrict__ dinv)
{
    double d = 0.0;
    int32_t c4[4] = {r, r, r, r};
    double v4[4] = {0.0, 0.0, 0.0, 0.0};
    int cnt = 0;
#pragma unroll
    for (int k = 0; k < 5; ++k) {
        if (c[k] == r) {
            d += v[k];  // the diagonal (unused slots add zero)
        } else if (cnt < 4) {
            c4[cnt] = c[k];
            v4[cnt] = v[k];
            ++cnt;
        }
    }
    const double di = d > 0.0 ? 1.0 / d : 1.0;
    (void)n;
    float s = 1.0f;
    phf_f4 f4;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const float f = (float)(v4[k] * di);
        f4[k] = f;
        s += fabsf(f);
    }
    if (col4) *(phf_i4*)(col4 + 4 * (int64_t)r) = phf_i4{c4[0], c4[1], c4[2], c4[3]};
    *(phf_f4*)(val4 + 4 * (int64_t)r) = f4;
    diag[r] = d > 0.0 ? (float)d : 1.0f;
    dinv[r] = (float)di;
    return s;
}

// ---- XCD-aware row blocks ----------------------------------------------------
// Workgroups are dealt to the eight XCDs of the device in turn, and each XCD
// has its own L2. Row kernels whose rows gather neighbouring values of the
// same vector therefore give the workgroups of one XCD one contiguous range
// of row tiles, through which they stride together (so each XCD streams one
// window of rows at a time): the lines that neighbouring rows share are then
// fetched into one L2 only. With one block per tile this is a permutation of
// the blocks.
template <int NT, typename F>
__device__ inline void phf_for_rows_xcd(int32_t n, F f)
{
    const int32_t nb = gridDim.x, b = blockIdx.x, x = b % 8, q = nb / 8, rem = nb % 8;
    const int32_t nbx = q + (x < rem ? 1 : 0);             // blocks on this XCD
    const int64_t first = (int64_t)x * q + min(x, rem);     // blocks on lower XCDs
    const int64_t tiles = ((int64_t)n + NT - 1) / NT;
    const int64_t t0 = tiles * first / nb, t1 = tiles * (first + nbx) / nb;
    for (int64_t t = t0 + b / 8; t < t1; t += nbx) {
        const int64_t i = t * NT + threadIdx.x;
        if (i < n) f((int32_t)i);
    }
}
// Calls f(i) for the rows of this workgroup: XCD ranges (XCD) or the plain
// grid-stride order.
template <bool XCD, int NT, typename F>
__device__ inline void phf_for_rows(int32_t n, F f)
{
    if (XCD) {
        phf_for_rows_xcd<NT>(n, f);
    } else {
        for (int32_t i = blockIdx.x * NT + threadIdx.x; i < n; i += gridDim.x * NT) f(i);
    }
}
