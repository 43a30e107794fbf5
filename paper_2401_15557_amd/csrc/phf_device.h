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

// Row of free edge e of the reduced (edge-midpoint) operator: e couples with
// the other free edges of T+ and T-. Writes the columns (ascending) and, per
// entry, up to two sources in the element blocks B (9T + 3 a + b, -1 none);
// returns the number of entries (at most 5).
__device__ inline int phf_reduced_entries(int32_t e, const int2* edge_elems, const int8_t* led,
                                      const int8_t* ledTN, const int32_t* elem_edges,
                                      const int32_t* red_row, int32_t* col, int32_t* s0,
                                      int32_t* s1)
{
    int n = 0;
    int2 tt = edge_elems[e];
    int lp = led[e];
    // diagonal: block (lp, lp) of T+ plus (ln, ln) of T-
    col[n] = red_row[e];
    s0[n] = 9 * tt.x + 4 * lp;
    s1[n] = tt.y >= 0 ? 9 * tt.y + 4 * ledTN[e] : -1;
    ++n;
    for (int side = 0; side < 2; ++side) {
        int32_t T = side == 0 ? tt.x : tt.y;
        if (T < 0) continue;
        int le = side == 0 ? lp : ledTN[e];
        for (int o = 0; o < 3; ++o) {
            if (o == le) continue;
            int32_t e2 = elem_edges[3 * (int64_t)T + o];
            int32_t r2 = red_row[e2];
            if (r2 < 0) continue;
            col[n] = r2;
            s0[n] = 9 * T + 3 * le + o;
            s1[n] = -1;
            ++n;
        }
    }
    // sort by column (at most 5 entries)
    for (int a = 1; a < n; ++a) {
        int32_t c = col[a], x0 = s0[a], x1 = s1[a];
        int b = a - 1;
        while (b >= 0 && col[b] > c) {
            col[b + 1] = col[b];
            s0[b + 1] = s0[b];
            s1[b + 1] = s1[b];
            --b;
        }
        col[b + 1] = c;
        s0[b + 1] = x0;
        s1[b + 1] = x1;
    }
    return n;
}

// Four-lane vectors for 16-byte row loads and stores.
typedef int32_t phf_i4 __attribute__((ext_vector_type(4)));
typedef float phf_f4 __attribute__((ext_vector_type(4)));
typedef double phf_d2 __attribute__((ext_vector_type(2)));

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
