// Multilevel preconditioner for the reduced (edge-midpoint) operator on a
// chain of red-refined meshes (internal to libphfem).
//
// Level l has the reduced operator R_l = sum_T P^T A_T P of its own mesh (the
// coarse ones re-discretised with the triangle coefficient averaged over the
// four children). The spaces of edge-midpoint (Crouzeix-Raviart) functions on
// nested meshes are not nested; the prolongation evaluates the coarse function
// at the midpoint of each fine edge: inside a coarse triangle (the three
// interior edges of its children) from that triangle, on a coarse edge as the
// average of the two coarse triangles sharing it. With ψ_l = 1 - 2 λ_l the CR
// basis of the coarse triangle, the weights are 1 - 2 λ_l(m_e); the
// barycentric coordinates of the fine midpoints are the same in every coarse
// triangle, so the weights are constants. Restriction is the transpose,
// applied as per-coarse-triangle sums over its nine fine edges followed by a
// sum over the two triangles of each coarse edge. Smoothing is damped Jacobi, the coarsest level is solved
// exactly (dense inverse), and the V-cycle with equal pre- and post-smoothing
// is symmetric, so it can precondition conjugate gradients. The cycle runs in
// single precision (operator copies, vectors, transfer weights; the coarsest
// solve accumulates in double): it only has to approximate the inverse, while
// the outer conjugate-gradient iteration keeps double precision, so the
// reached residual is unaffected and the cycle moves about 40% fewer bytes.
//
// Each sweep is x += w_k D^-1 (b - A x). With the Jacobi smoother every w_k
// is the damping omega; with the Chebyshev smoother the nu weights of a side
// are the reciprocal roots of the degree-nu Chebyshev polynomial on
// [lmax / range, lmax], lmax the Gershgorin bound max_i sum_j |a_ij| / a_ii of
// the level (computed on the device), so the nu sweeps together minimise the
// largest error factor over that upper part of the spectrum. Both are
// polynomials in D^-1 A, so the cycle stays symmetric.
#pragma once

#include "phf_solver.h"

#define PHF_MG_MAX_LEVELS 20
#define PHF_MG_DENSE_MAX 256
// Levels with at most this many unknowns (below the finest) run their part of
// the cycle in one single-workgroup launch, as long as their vectors fit in
// that workgroup's local data share (PHF_MG_TAIL_LDS bytes; gfx950 gives one
// workgroup up to 160 KiB).
#ifndef PHF_MG_TAIL_MAX
#define PHF_MG_TAIL_MAX 8192
#endif
#ifndef PHF_MG_TAIL_LDS
#define PHF_MG_TAIL_LDS (160 * 1024)
#endif
// Sweeps per side at most; each level keeps PHF_MG_MAX_SWEEPS sweep weights
// and, last, the weight of the plain sweeps of an iterative coarsest solve.
#define PHF_MG_MAX_SWEEPS 8
#define PHF_MG_WSTRIDE (PHF_MG_MAX_SWEEPS + 1)

// Device view of one level, for the single-workgroup cycle.
struct phf_mg_dev_level {
    int32_t n = 0, nEc = 0;  // unknowns; elements of the next coarser mesh
    const int32_t* col = nullptr;  // scaled operator (ELL-4 of D^-1 A off the diagonal)
    const float *val = nullptr, *diag = nullptr, *dinv = nullptr;
    float *x = nullptr, *y = nullptr, *b = nullptr, *r = nullptr;  // b holds D^-1 b
    const int32_t* P_col = nullptr;  // prolongation from the next coarser level
    const uint32_t* P_code = nullptr;
    const int32_t* rows9 = nullptr;  // restriction to the next coarser level
    float* t = nullptr;
    const int32_t* ecode_c = nullptr;  // element codes of the next coarser mesh
    const int2* sel = nullptr;         // own gather map (from the finer level's sums)
    const float* w = nullptr;          // sweep weights (PHF_MG_WSTRIDE)
    // offsets (in floats) of the level's vectors in the workgroup's local
    // data share: the two iterates, D^-1 b, and the restriction sums
    int32_t sx = 0, sy = 0, sb = 0, st = 0;
};

// One level's entry in the table that drives the set-up launches over all
// levels (built once per hierarchy).
struct phf_mg_setup_level {
    int32_t nf = 0, nEc = 0, nc = 0;  // own free rows; next coarser level's elements, free rows
    // first blocks: prolongation, restriction rows, gather map (levels >= 1);
    // scaled rows (every level)
    int32_t b[4] = {0, 0, 0, 0};
    const int32_t* red_edge = nullptr;  // this level's mesh tables
    const int2* edge_elems = nullptr;
    const int8_t *led = nullptr, *ledTN = nullptr;
    const int32_t* elem_red = nullptr;  // reduced rows of the elements' local edges
    const int32_t *elem_red_c = nullptr, *red_edge_c = nullptr;  // coarser
    const int2* edge_elems_c = nullptr;
    const int8_t *led_c = nullptr, *ledTN_c = nullptr;
    int32_t* P_col = nullptr;  // outputs of the tables
    uint32_t* P_code = nullptr;
    int32_t* rows9 = nullptr;
    int2* sel_c = nullptr;
    const int32_t* rec = nullptr;  // operator: half-row records (coarse levels) or
    // the caller's double-precision rows (finest): off-diagonal columns and
    // values as row-major ELL-4, then the nf diagonal values behind the values
    const int32_t* ell_col = nullptr;
    const double* ell_val = nullptr;
    int32_t* col4 = nullptr;  // the cycle's scaled rows
    float *val4 = nullptr, *diag = nullptr, *dinv = nullptr;
    int32_t* col64 = nullptr;  // coarsest level with a dense inverse
    double* val64 = nullptr;
};

struct phf_mg_level {
    phf_mesh* mesh = nullptr;
    phf_ns* ns = nullptr;       // the caller's operator (finest level only)
    int32_t nf = 0;
    // coarse levels: triangle coefficient (averaged from the finer level)
    // and the half-row records of the re-discretised operator (24 nE)
    double* aT = nullptr;
    int32_t* rec = nullptr;
    // single-precision scaled operator: the off-diagonal entries of D^-1 A
    // (ELL-4, row-major; unused slots hold the row itself and 0), the
    // diagonal D and its inverse. The finest level's columns are the caller's
    // operator columns (not owned).
    int32_t* col4 = nullptr;
    float *val4 = nullptr, *diag32 = nullptr, *dinv32 = nullptr;
    // V-cycle vectors (single precision); b holds the scaled D^-1 b
    float *x = nullptr, *y = nullptr, *b = nullptr, *r = nullptr;
    // prolongation from the next coarser level: ELL-5 columns over this
    // level's rows and per row the five weights, each a multiple of 1/4 in
    // [-1, 1], as 4-bit codes c (weight (c - 4) / 4, slot k in bits 4k..4k+3)
    int32_t* P_col = nullptr;
    uint32_t* P_code = nullptr;
    // restriction to the next coarser level: fine rows of the nine fine edges
    // in each coarse triangle (slot-major, 9 x nE_coarse), per-triangle sums
    // (3 x nE_coarse)
    int32_t* rows9 = nullptr;
    float* t = nullptr;
    // on coarse levels: positions of each row's edge in the sums of the finer
    // level (T+ side, T- side or -1)
    int2* sel = nullptr;
};

struct phf_mg {
    int32_t nlev = 0;  // lev[0] coarsest ... lev[nlev-1] finest
    phf_mg_level lev[PHF_MG_MAX_LEVELS];
    double* cinv = nullptr;  // dense inverse of the coarsest operator (n0 <= DENSE_MAX)
    double* cwork = nullptr;
    int32_t* col64 = nullptr;  // coarsest operator in double precision (ELL-5), for cinv
    double* val64 = nullptr;
    int32_t n0 = 0;
    int32_t tail_top = -1;   // levels 0..tail_top run in the single-workgroup kernel
    int32_t tail_lds = 0;    // its local data share (bytes)
    phf_mg_dev_level h_lv[PHF_MG_MAX_LEVELS];
    phf_mg_dev_level* d_lv = nullptr;
    phf_mg_setup_level h_setup[PHF_MG_MAX_LEVELS];
    phf_mg_setup_level* d_setup = nullptr;
    int32_t setup_table_blocks = 0, setup_row_blocks = 0;
    int32_t nu = 2;          // sweeps before and after the coarse correction
    // plain sweeps of the coarsest level when it has no dense inverse (even,
    // so that the result ends where the first sweep started): 40, or 8 when
    // the coarsest levels were left out for a mass-dominated operator
    int32_t coarse_sweeps = 40;
    int32_t smoother = 0;    // PHF_MG_SMOOTH_JACOBI or PHF_MG_SMOOTH_CHEBYSHEV
    double omega = 0.8;      // Jacobi damping
    double range = 4.0;      // Chebyshev: smoothing range [lmax / range, lmax]
    uint32_t* lmax = nullptr;  // per level: Gershgorin bound (float bits)
    float* wts = nullptr;      // per level: PHF_MG_WSTRIDE sweep weights
    float* z32 = nullptr;      // finest-level result for conjugate gradients
    bool fine_rows_ready = false;  // the finest scaled rows came with the operator
};

// Finest-level outputs that the kernel building the double-precision rows of
// the finest operator can fill at the same time: the scaled single-precision
// rows, the diagonal and its inverse (phf_scale_row), and the level's
// Gershgorin bound (float bits, merged with atomicMax; cleared beforehand).
struct phf_mg_rows {
    int32_t* col4;
    float* val4;
    float* diag;
    float* dinv;
    uint32_t* lmax;
};

// Finest-level buffers through which the outer iteration's update can take
// the cycle's first sweep from zero itself: bh = D^-1 r (single precision),
// x = w[0] bh. Valid until the next cycle is queued.
struct phf_mg_top {
    float* bh;
    float* x;  // null: the cycle's second sweep forms x from bh (not stored)
    const float* dinv;
    const float* w;
};

// Builds the hierarchy below the finest operator `fine` (whose mesh must come
// from phf_mesh_refine). Symbolic part only; call phf_mg_numeric next.
int phf_mg_create(phf_ns* fine, phf_mg** out, int32_t drop_coarse = 0);
void phf_mg_destroy(phf_mg* mg);
// Coarse operators for A = cK K + cM M with the finest-level triangle
// coefficient aT (nullable, constant A from coeffs), prolongations, coarse
// inverse. The finest operator is the one already built in `fine`.
int phf_mg_numeric(phf_mg* mg, const phf_coeffs* coeffs, double cK, double cM);
// z = V-cycle(r) on the finest level; writes partial sums of r.z into
// part (slot layout of the CG kernels). Skipped when *iflags (done) is set.
int phf_mg_apply(phf_mg* mg, const double* r, double* z, double* part_rz, const int* iflags);
// The same with the result in single precision in mg->z32 (it is the cycle's
// single-precision iterate, so nothing is lost); first_done: the caller has
// already written the first sweep through phf_mg_top_view.
int phf_mg_apply32(phf_mg* mg, const double* r, bool first_done, double* part_rz,
                   const int* iflags);
phf_mg_top phf_mg_top_view(phf_mg* mg);
// Queues the clearing of the spectral bounds and hands out the finest-level
// outputs for the operator kernel; the next phf_mg_numeric then takes the
// finest rows as written and builds only the coarser levels.
int phf_mg_fine_rows(phf_mg* mg, phf_mg_rows* out);
// Number of hierarchy levels below and including `mesh`.
int32_t phf_mg_levels(const phf_mesh* mesh);
