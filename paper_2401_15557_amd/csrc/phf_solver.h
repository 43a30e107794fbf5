// Null-space conjugate-gradient solver of the primal hybrid saddle system
// (internal to libphfem).
//
// System: A U - C^T mu = rhs1, -C U = rhs2, with A block diagonal (element
// blocks A_T = cK K_T + cM M_T read from assembled K and M arrays) and C the
// coupling matrix (row of edge e: +h on the vertex DOFs of T+, -h on those of
// T-, h = |E|/2).
//
// Reduction: on each element the P1 function is determined by its values at
// the three edge midpoints, U_T = P w_T with P[i][l] = -1 if l == i else +1
// (local edge l opposite vertex l). Taking w_e shared by both neighbours of
// every edge satisfies the interior constraints; Dirichlet rows fix w_e; a
// non-zero interior right-hand side is carried as a jump added on the T+
// side. The free unknowns are the midpoint values of non-Dirichlet edges and
// the projected operator R = sum_T P^T A_T P is symmetric positive definite
// when A is (plus at least one Dirichlet edge when A = K). mu follows element
// by element from the first block row: C_T^T mu_T = A_T U_T - rhs1_T, whose
// solution on T+ is mu_e = (P^T (A_T U_T - rhs1_T))_e / |E|.
#pragma once

#include "phf_internal.h"

struct phf_mg;

// B = P^T A P for one element (3 x 3, row-major; A need not be symmetric),
// with P[i][l] = -1 if l == i else 1: AP[i][l] = rowsum_i(A) - 2 A[i][l],
// then B[l][l'] = colsum_l'(AP) - 2 AP[l][l'].
__device__ inline void phf_reduce_block(const double* A, double B[9])
{
    double AP[9];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        const double rs = A[3 * i] + A[3 * i + 1] + A[3 * i + 2];
#pragma unroll
        for (int l = 0; l < 3; ++l) AP[3 * i + l] = rs - 2.0 * A[3 * i + l];
    }
#pragma unroll
    for (int lp = 0; lp < 3; ++lp) {
        const double cs = AP[lp] + AP[3 + lp] + AP[6 + lp];
#pragma unroll
        for (int l = 0; l < 3; ++l) B[3 * l + lp] = cs - 2.0 * AP[3 * l + lp];
    }
}

// Blocks of the solver's vector kernels at most, i.e. partial-sum slots per
// reduced quantity (each block writes one and every block of the next kernel
// reduces all of them in the same order).
// Row order of the row kernels (bit set: XCD-contiguous chunks): 1 sweeps,
// 2 residual, 4 prolongation, 8 restriction, 16 gather, 32 last finest sweep,
// 64 the conjugate-gradient direction.
#ifndef PHF_XCD_BITS
#define PHF_XCD_BITS 0x33
#endif
#ifndef PHF_PART_MAX
#define PHF_PART_MAX 1024
#endif

struct phf_ns {
    phf_mesh* mesh = nullptr;
    phf_mg* mg = nullptr;         // multilevel preconditioner (owned)
    bool mg_on = false;           // use it (else Jacobi)
    bool fuse_fine_rows = false;  // the next operator build also writes mg's finest rows
    int32_t nE = 0, nf = 0, L = 0, nbv = 0;
    // symbolic (per mesh; the element tables are the mesh's)
    const int32_t* elem_red = nullptr;  // 3 nE: reduced row of local edge l (-1 Dirichlet)
    const int32_t* elem_row = nullptr;  // 3 nE: multiplier row of local edge l (-1 Neumann)
    int32_t* ell_col = nullptr;   // 4 nf: off-diagonal columns of R, row-major ELL-4
    // numeric
    int32_t* rec = nullptr;       // 24 nE: half-row records of the reduced operator
                                  // (32 bytes per element and local edge, phf_hrec_row)
    double* Ablk = nullptr;       // 9 nE: A_T (allocated when A is not K itself)
    const double* A = nullptr;    // the element blocks A_T of the current operator
    double* ell_val = nullptr;    // 5 nf: the 4 nf off-diagonal values, then the diagonal
    double* dinv = nullptr;       // nf
    double* kv = nullptr;         // 3 nE known midpoint values / jumps
    double* cs = nullptr;         // 3 nE element right-hand side / residual
    double* b = nullptr;
    double* w = nullptr;
    double* r = nullptr;
    double* z = nullptr;
    double* p = nullptr;
    double* q = nullptr;
    double* part = nullptr;       // P_NARR x 1024 partial sums
    // BiCGSTAB only (allocated on first use): shadow residual, s, the
    // preconditioned s, t
    double *rh = nullptr, *s = nullptr, *sh = nullptr, *t = nullptr;
    double* scal = nullptr;       // device scalars
    int* iflags = nullptr;        // [0] done, [1] iterations
    int* jflag = nullptr;         // raised: interior constraint rows with a right-hand side
    int32_t next_it = 0;          // index of the next CG iteration issued
};

// Scalar slots in phf_ns::scal.
enum { NS_RR = 0, NS_BB, NS_TOL2, NS_NSCAL = 8 };

int phf_ns_create(phf_mesh* mesh, phf_ns** out);
void phf_ns_destroy(phf_ns* ns);
// Builds A_T, the half-row records, the ELL values and the Jacobi diagonal
// for A = cK K + cD D + cM M. borrow_K: with A = K (cK = 1, no M or D term)
// the solver reads the element blocks from K itself, which the caller keeps
// unchanged until the last phf_ns_rhs / phf_ns_recover of this operator.
// The multiplier scaling |E|/2 is the mesh's (the value phf_assemble writes
// into C).
int phf_ns_operator(phf_ns* ns, const double* K, const double* M, double cK, double cM,
                    const double* D = nullptr, double cD = 0.0, bool borrow_K = false);
// Right-hand side reduction (rhs2 is the right-hand side of -C U = rhs2).
// all_jumps: take the T+-side jumps of every interior row without testing
// rhs2 for them (a caller whose constraint right-hand side has them anyway).
// hs_elem: optional 3 nE values whose magnitude is |E|/2 of each element's
// local edge (read as a stream instead of the row's half-length by row).
int phf_ns_rhs(phf_ns* ns, const double* rhs1, const double* rhs2, bool all_jumps = false,
               const double* hs_elem = nullptr);
// Starts CG from the current w, or with zero_start from w = 0 (written by
// the start itself).
int phf_ns_cg_start(phf_ns* ns, double rtol, bool zero_start = false);
// Issues `iters` CG iterations (skipped on the device once converged).
int phf_ns_cg_iterate(phf_ns* ns, int32_t iters);
// U = P (w + kv); mu = mu_scale * element-local multiplier recovery.
int phf_ns_recover(phf_ns* ns, const double* rhs1, double* U, double* mu, double mu_scale);
int phf_ns_zero_w(phf_ns* ns);
// Right-preconditioned BiCGSTAB on the same reduced system (any A, also
// nonsymmetric), with the same device-side scalars and convergence flag;
// iflags[2] is set on a breakdown, after which the iteration restarts from
// the current iterate (a bounded number of times; *breakdown reports the
// last run's).
int phf_ns_bicg_solve(phf_ns* ns, double rtol, int32_t max_iter, int32_t check_every,
                      int32_t* iters_out, double* relres_out, int* converged, int* breakdown);
// Host convergence loop: cg_start + batches of check_every iterations.
int phf_ns_cg_solve(phf_ns* ns, double rtol, int32_t max_iter, int32_t check_every,
                    int32_t* iters_out, double* relres_out, int* converged,
                    bool zero_start = false);
// Multigrid smoothing as the public options give it (0 = default).
struct phf_mg_params {
    int32_t sweeps = 0, smoother = 0;
    double omega = 0.0, range = 0.0;
    // coarsest levels of the refinement chain left out of the hierarchy when
    // it is built (first use); the new coarsest level is then smoothed
    // instead of solved
    int32_t drop_coarse = 0;
};
// Checks the multigrid options and builds the hierarchy (first use) without
// its numeric part; nothing for Jacobi.
int phf_ns_prepare_precond(phf_ns* ns, int32_t precond, const phf_mg_params& mp);
// Chooses Jacobi or the multilevel preconditioner (built on first use, its
// coarse operators recomputed for A = cK K + cM M and coeffs' a_T).
int phf_ns_set_precond(phf_ns* ns, int32_t precond, const phf_mg_params& mp,
                       const phf_coeffs* co, double cK, double cM);
// The mesh's cached workspace (created on first use).
int phf_ns_get(phf_mesh* mesh, phf_ns** out);
