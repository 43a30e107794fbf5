/*
 * phfem.h -- C ABI of libphfem.so, the MI355X (gfx950) hot path of the
 * lowest-order primal hybrid finite element method for 2-D second-order
 * elliptic problems and their Crank-Nicolson parabolic counterpart with mixed
 * boundary conditions (Nagula Mallesham, Porwal, Valdman, Acharya,
 * arXiv:2401.15557).
 *
 * General rules
 *  - Every call returns PHF_OK (0) or a negative PHF_E* code; no exception or
 *    signal crosses the ABI. After an error, phf_last_error() describes it.
 *  - Indices are 0-based int32. Element vertices must be counter-clockwise.
 *    Boundary node pairs may be listed in either orientation.
 *  - A context owns one HIP stream (the caller's, or the null stream); every
 *    kernel of every call on objects of that context is launched on it, in
 *    call order. Calls return without synchronising unless stated.
 *  - Handles are not thread-safe: one host thread per context at a time.
 *  - Pointers tagged "device" must be HIP device (or managed) memory on the
 *    context's device; "host" pointers are ordinary host memory. Output
 *    buffers are owned by the caller and must stay valid until the stream
 *    has executed the call. Input arrays are copied; the caller keeps them.
 *  - Sizes are limited by int32 indexing: nE <= 80,000,000 elements.
 *
 * Notation (Sections 2-4 of the paper): nE elements, nC nodes, nrEdges
 * edges, N = 3 nE primal unknowns (discontinuous P1: DOF 3m+i is the
 * barycentric coordinate of local vertex i of element m), L = number of
 * interior + Dirichlet edges (multiplier unknowns, one per edge, in ascending
 * edge id order). "Local edge i" of an element is the edge opposite its local
 * vertex i.
 */
#ifndef PHFEM_H
#define PHFEM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
#define PHF_OK 0
#define PHF_EINVAL -1    /* null pointer, size, index out of range, bad option */
#define PHF_EORIENT -2   /* element clockwise, degenerate or zero area        */
#define PHF_EMESH -3     /* edge in > 2 elements or same direction in both    */
#define PHF_EBOUNDARY -4 /* boundary edge in no list or in two; listed pair
                            not a boundary edge of the mesh                    */
#define PHF_ENOMEM -5    /* device or host allocation failed                   */
#define PHF_ENOCONV -6   /* Krylov solver hit max_iter before rtol             */
#define PHF_EHIP -7      /* a HIP runtime call failed                          */
#define PHF_ESTATE -8    /* call out of order (e.g. solve before assemble)     */
#define PHF_ETIMEDOUT -9 /* phf_server_wait: the request is not finished yet  */

typedef struct phf_ctx phf_ctx;
typedef struct phf_mesh phf_mesh;
typedef struct phf_cn phf_cn;

typedef enum { PHF_HOST = 0, PHF_DEVICE = 1 } phf_memspace;

/* ---- context ----------------------------------------------------------- */

/* Source of the library's device memory. alloc returns `bytes` of device
 * memory on the context's device (NULL on failure; the library then frees
 * its cached blocks through `free` and asks once more), usable in the order
 * of the context's stream; free returns a block obtained from alloc, once
 * no work issued on that stream before the call uses it any longer (the
 * allocator may hand it out again for later work on the same stream).
 * `user` is passed back unchanged. Both are called from the host thread
 * that makes the library call (phf_destroy and phf_release_cache included).
 * A caller that keeps a caching allocator of its own (torch's, from
 * Python) passes it here, so that every device byte of the context comes
 * from it. */
typedef struct {
    void* (*alloc)(size_t bytes, void* user);
    void (*free)(void* ptr, void* user);
    void* user;
} phf_allocator;

/* Creates a context on HIP device `device` whose kernels run on `hip_stream`
 * (a hipStream_t; NULL = the null stream). *out receives the handle.
 * `alloc` (copied; may be NULL) supplies every device block the context
 * holds: mesh tables, solver and time-stepper state, temporaries and the
 * context's own flag words. NULL: hipMalloc / hipFree. Either way the
 * context keeps released blocks in its cache (phf_release_cache). */
int phf_create(phf_ctx** out, int device, void* hip_stream, const phf_allocator* alloc);
/* Synchronises the stream and frees the context. Returns PHF_ESTATE (and
 * frees nothing) while meshes, Crank-Nicolson steppers or batches created on
 * it are alive: destroy those first. */
int phf_destroy(phf_ctx* ctx);
/* Redirects later launches to another stream of the same device; waits for
 * the old stream first (cached device blocks were last used in its order). */
int phf_set_stream(phf_ctx* ctx, void* hip_stream);

/* ---- device memory -------------------------------------------------------
 * All device memory the library owns (mesh tables, solver and time-stepper
 * state, temporaries) comes from a caching pool of the context, which takes
 * its blocks from the context's allocator (phf_create): a released block is
 * kept and handed out again for a request of the same rounded size (512 B
 * granules up to 1 MiB, 2 MiB granules above), so rebuilding meshes of the
 * same sizes makes no allocator calls. The library runs all its work in order
 * on the context's stream, which makes reuse safe. Cached blocks go back to
 * the allocator on phf_release_cache, when an allocation fails (then it is
 * retried once), and in phf_destroy; blocks of objects that outlive their
 * context go back when those objects are destroyed. Not thread-safe per
 * context. */
/* Bytes held by live library objects / kept in the cache (either nullable). */
int phf_mem_stats(phf_ctx* ctx, int64_t* live_bytes, int64_t* cached_bytes);
/* Waits for the stream, then frees every cached block. */
int phf_release_cache(phf_ctx* ctx);
/* Blocks until all work issued on the context's stream has finished. */
int phf_synchronize(phf_ctx* ctx);
/* Static text of a status code / the last error recorded on ctx. */
const char* phf_status_str(int code);
const char* phf_last_error(const phf_ctx* ctx);
/* Library version as "major.minor.patch". */
const char* phf_version(void);

/* ---- kernel timing (tracing) -------------------------------------------
 * With tracing on, every kernel the library launches is bracketed by HIP
 * events on the context's stream; phf_trace_query() synchronises and returns
 * the launch count and total milliseconds of the kernels whose name equals
 * `kernel` (NULL: all kernels). phf_trace_reset() clears the record.
 * phf_trace_dump() writes "name count total_ms" lines into buf (truncated to
 * len bytes, NUL-terminated) and returns the number of kernel names.
 * phf_trace_filter() limits tracing to the launches named `kernel` (NULL or
 * "": every launch), so that timing one kernel adds no events to the rest. */
int phf_trace_enable(phf_ctx* ctx, int on);
int phf_trace_filter(phf_ctx* ctx, const char* kernel);
int phf_trace_reset(phf_ctx* ctx);
int phf_trace_query(phf_ctx* ctx, const char* kernel, int64_t* count, double* total_ms);
int phf_trace_dump(phf_ctx* ctx, char* buf, size_t len);
/* Per-launch milliseconds of the traced launches named `kernel` (required),
 * in launch order: up to `cap` values into the host array ms (may be NULL
 * when cap = 0); *count receives the number recorded since the last reset.
 * Launches of an iteration that had already converged return at once on the
 * device and show up here as near-empty launches. */
int phf_trace_samples(phf_ctx* ctx, const char* kernel, float* ms, int64_t cap, int64_t* count);

/* ---- mesh: upload, validation, topology, patterns ----------------------
 * Section 2.1 (data of Table 1) and Section 2.2 (edge_vec): builds on the
 * device
 *  - the edge numbering: edges in ascending (larger node, smaller node)
 *    order, i.e. the column-major upper-triangle order of nodes2edge;
 *  - edge2element: T+ = the element of the first occurrence of the edge in
 *    element order, T- the other one (-1 on the boundary); [k,l] = the edge
 *    as traversed by T+; led / ledTN = local edge number in T+ / T-;
 *  - the Dirichlet / Neumann edge ids of the listed pairs (Main.m, Dbed and
 *    Nbed) and the multiplier row of every non-Neumann edge (Redges);
 *  - the CSR patterns of K, M (3x3 element blocks), C (L x N) and of the
 *    saddle matrix [A, -C^T; -C, 0] (Section 3.5).
 * xy: nC x 2 (x, y) float64; elem: nE x 3; dir: nD x 2; neu: nN x 2, all in
 * memory space `ms`. Synchronises the stream (sizes are read back).
 * Errors: PHF_EINVAL (sizes, indices), PHF_EORIENT, PHF_EMESH,
 * PHF_EBOUNDARY, PHF_ENOMEM, PHF_EHIP. */
int phf_mesh_create(phf_ctx* ctx, const double* xy, int32_t nC, const int32_t* elem, int32_t nE,
                    const int32_t* dir, int32_t nD, const int32_t* neu, int32_t nN,
                    phf_memspace ms, phf_mesh** out);
/* Frees a mesh. PHF_ESTATE while meshes refined from it, Crank-Nicolson
 * steppers or batches built on it are alive. */
int phf_mesh_destroy(phf_mesh* mesh);

/* One uniform red refinement on the device with the paper's numbering
 * (Section 2.3, Listing 4): the midpoint of edge e becomes node nC + e;
 * element m is replaced by its interior child [M1 M2 M3] (M_i = midpoint of
 * the edge opposite vertex i) and the corner children [v1 M3 M2],
 * [v2 M1 M3], [v3 M2 M1] follow at nE + 3m + {0, 1, 2}; each listed boundary
 * pair (a, b) becomes (a, M) in the first half of its list and (M, b) in the
 * second. The new mesh is built as by phf_mesh_create and keeps a reference
 * to `coarse` (the multilevel preconditioner uses the chain), so `coarse`
 * must outlive it. Synchronises the stream. */
int phf_mesh_refine(phf_mesh* coarse, phf_mesh** fine);

typedef struct {
    int32_t nC, nE, n_edges;   /* nodes, elements, edges (nrEdges)         */
    int32_t N, L;              /* 3 nE primal unknowns; multiplier rows      */
    int32_t nD, nN;            /* Dirichlet / Neumann edges                  */
    int32_t n_interior;        /* interior edges                             */
    int32_t n_free;            /* non-Dirichlet edges (reduced unknowns)     */
    int64_t nnz_K;             /* 9 nE: nnz of K, M and D                    */
    int64_t nnz_C;             /* 4 n_interior + 2 nD                        */
    int64_t nnz_saddle;        /* 9 nE + 2 nnz_C                             */
    int64_t nnz_reduced;       /* nnz of the edge-midpoint (reduced) operator */
    int64_t device_bytes;      /* device memory held by the mesh             */
} phf_mesh_info;

/* Sizes of a mesh. (Named _get_info because C does not allow a function
 * and the struct typedef above to share the name phf_mesh_info.) */
int phf_mesh_get_info(const phf_mesh* mesh, phf_mesh_info* out);

/* Copies topology tables into caller buffers in memory space `ms` (device
 * copies are stream-ordered; host copies synchronise). Any pointer may be
 * NULL to skip it. Sizes: edge_nodes, edge_elems 2 n_edges; elem_edges
 * 3 nE (entry 3m+i = edge opposite local vertex i); led, ledTN, edge_type
 * (0 interior, 1 Dirichlet, 2 Neumann), edge_row (-1 for Neumann) n_edges;
 * dir_edges nD; neu_edges nN (list order). */
int phf_mesh_topology(const phf_mesh* mesh, int32_t* edge_nodes, int32_t* edge_elems,
                      int32_t* elem_edges, int8_t* led, int8_t* ledTN, int8_t* edge_type,
                      int32_t* edge_row, int32_t* dir_edges, int32_t* neu_edges,
                      phf_memspace ms);

/* Copies the mesh arrays out (memory space `ms`; NULL skips): xy nC x 2,
 * elem nE x 3, dir nD x 2, neu nN x 2, as given to phf_mesh_create or as
 * produced by phf_mesh_refine. Host copies synchronise. */
int phf_mesh_geometry(const phf_mesh* mesh, double* xy, int32_t* elem, int32_t* dir,
                      int32_t* neu, phf_memspace ms);

/* Copies CSR patterns (rowptr int32 rows+1, col int32 nnz). K/M/D: N rows,
 * columns 3m..3m+2 ascending; C: L rows, the two vertex columns of T+ then
 * those of T-; saddle: N + L rows, columns ascending. NULL skips. */
int phf_mesh_pattern(const phf_mesh* mesh, int32_t* K_rowptr, int32_t* K_col,
                     int32_t* C_rowptr, int32_t* C_col, int32_t* S_rowptr, int32_t* S_col,
                     phf_memspace ms);

/* ---- problem data -------------------------------------------------------
 * Coefficients of -div(A grad u + u p) + delta u = f (Section 3.1):
 * A constant 2x2 symmetric positive definite (row-major), scaled per element
 * by a_T (device array of nE, or NULL for 1); p constant; delta constant.
 * The convection block follows the listing's convention
 * D[j][i] = int_T lambda_j (p . grad lambda_i). */
typedef struct {
    double A[4];
    double p[2];
    double delta;
    const double* a_T;
} phf_coeffs;

/* Source f, Neumann flux g and Dirichlet value u_D (Section 3.1).
 * kind: */
#define PHF_FN_ZERO 0          /* 0                                           */
#define PHF_FN_CONST 1         /* c0                                          */
#define PHF_FN_SIN_COS 2       /* c0 exp(c1 t) sin(pi x) cos(pi y)            */
#define PHF_FN_SIN_SIN 3       /* c0 exp(c1 t) sin(pi x) sin(pi y)            */
#define PHF_FN_GRAD_SIN_COS 4  /* c0 exp(c1 t) grad(sin(pi x)cos(pi y)) . nu  */
#define PHF_FN_GRAD_SIN_SIN 5  /* c0 exp(c1 t) grad(sin(pi x)sin(pi y)) . nu  */
#define PHF_FN_PAPER_U 6       /* (c0 + c1 t)(x - x^2)(y - y^2)               */
#define PHF_FN_PAPER_F 7       /* source of the paper's Examples 1 (c0=1,c1=0)
                                  and 2 (c0=0, c1=1)                          */
#define PHF_FN_PAPER_FLUX 8    /* (c0 + c1 t)[(1-x-x^2)(y-y^2),
                                  (x-x^2)(1-y-y^2)] . nu (Examples 1, 2)      */
#define PHF_FN_EDGE_ARRAY 100  /* edge_values[e] (device, n_edges doubles) is
                                  the value at the midpoint of edge e (for g:
                                  the normal flux, outward from T+)            */
typedef struct {
    int32_t kind;
    int32_t pad_;
    double c[4];
    const double* edge_values;
} phf_fn;

/* f is evaluated at the three edge midpoints of each element, g and u_D
 * at the midpoint of each Neumann / Dirichlet edge (Section 3.4);
 * nu is the outward unit normal of the edge's element. t is the time. */
typedef struct {
    phf_fn f, g, uD;
    double t;
} phf_data;

/* ---- numeric assembly ---------------------------------------------------
 * Definition 3.1 and Sections 3.4-3.5, one pass over elements and one over
 * multiplier rows in a single launch. Device output buffers (NULL skips):
 *   K  nnz_K  stiffness a_T |T| (A grad lambda_j) . grad lambda_i, CSR order
 *              (element m: 9 values row-major at 9m)
 *   M  nnz_K  unit mass |T|/12 (1 + delta_ij) (without the reaction delta)
 *   D  nnz_K  convection (only if p != 0 is wanted)
 *   C  nnz_C  coupling: row of edge e = [|E|/2, |E|/2] on the vertex DOFs of
 *              T+ followed by [-|E|/2, -|E|/2] on those of T- (interior)
 *   F  N      b + LN (midpoint-rule source load + Neumann load)
 *   bD L      -|E| u_D(m_E) on Dirichlet rows, 0 on interior rows
 *   S  nnz_saddle  values of [K + D + delta M, -C^T; -C, 0]
 * Stream-ordered, deterministic (no floating-point atomics), no host sync. */
typedef struct {
    double* K;
    double* M;
    double* D;
    double* C;
    double* F;
    double* bD;
    double* S;
} phf_system;

int phf_assemble(phf_mesh* mesh, const phf_coeffs* coeffs, const phf_data* data,
                 const phf_system* out);

/* ---- batched assembly --------------------------------------------------
 * Many independent meshes of one context assembled in one launch (the
 * per-triangle work of Definition 3.1 and Sections 3.4-3.5 is independent
 * across meshes). The launch walks a work list of (mesh, tile) items, element
 * tiles then multiplier-row tiles of each mesh; its shape is the batch's
 * configuration: the tile size (64, 128 or 256 triangles or rows per
 * workgroup), the grid (blocks_per_cu = 0: one workgroup per item; k > 0:
 * a persistent grid of k workgroups per compute unit striding over the list),
 * the lanes per triangle, whether element tiles are staged in LDS, and where
 * their vertex coordinates come from.
 * phf_batch_assemble: coeffs[i], data[i], out[i] as for phf_assemble of
 * meshes[i] (K, M, C, F, bD required; D and a_T given for all instances or
 * none; S is not written). The outputs are bit-identical to phf_assemble of
 * each mesh. phf_batch_tune times every candidate shape on the given
 * arguments (a warm-up and `reps` launches each, HIP events on the context's
 * stream), keeps the fastest as the batch's configuration and returns the
 * candidates' average milliseconds in results (up to max_results; 21
 * candidates: tile x {one workgroup per item, 2, 4, 8 per CU} staged, tile x
 * per-thread stores, tile x four lanes per triangle, tile x staged with
 * gathered coordinates); it writes the outputs as phf_batch_assemble does.
 * Every shape gives bit-identical outputs. The meshes
 * must outlive the batch; the caller keeps ownership. */
typedef struct phf_batch phf_batch;
typedef struct {
    int32_t tile;          /* 64, 128 or 256 threads per workgroup; element
                              tiles of that many triangles (a quarter with
                              lanes = 4), row tiles of that many rows        */
    int32_t blocks_per_cu; /* 0 = one workgroup per work item; else 1..64
                              (lanes = 1 and direct = 0 only)                */
    double ms;             /* tuning: average milliseconds per launch        */
    int32_t lanes;         /* threads per triangle: 1 (0 reads as 1), or 4
                              (three compute one row of the element block
                              each, exchanging f and Neumann terms across
                              lanes, and store it directly; no LDS)          */
    int32_t direct;        /* lanes = 1: 0 = element tile staged in LDS and
                              streamed out with 16-byte stores, 1 = each
                              thread stores its own triangle's values        */
    int32_t gather;        /* staged tiles: 1 = vertex coordinates gathered
                              from the node array through the vertex ids
                              (16 bytes per triangle plus cached gathers)
                              instead of the element-major copy (48 bytes)   */
    int32_t reserved_;     /* 0                                              */
} phf_batch_config;
int phf_batch_create(phf_ctx* ctx, phf_mesh* const* meshes, int32_t n, phf_batch** out);
/* (the meshes cannot be destroyed while the batch is alive: PHF_ESTATE) */
int phf_batch_destroy(phf_batch* batch);
int phf_batch_assemble(phf_batch* batch, const phf_coeffs* coeffs, const phf_data* data,
                       const phf_system* out);
int phf_batch_tune(phf_batch* batch, const phf_coeffs* coeffs, const phf_data* data,
                   const phf_system* out, int32_t reps, phf_batch_config* results,
                   int32_t max_results, int32_t* n_results);
int phf_batch_get_config(const phf_batch* batch, phf_batch_config* cfg);
int phf_batch_set_config(phf_batch* batch, const phf_batch_config* cfg);

/* y = alpha * A x + beta * y for a CSR matrix (device arrays, int32 rowptr /
 * col, nrows rows). Used for residuals of the assembled operators. */
int phf_spmv(phf_ctx* ctx, int32_t nrows, const int32_t* rowptr, const int32_t* col,
             const double* val, double alpha, const double* x, double beta, double* y);

/* ---- saddle-point solve -------------------------------------------------
 * Solves M_vec W = F_vec, i.e. (K + D + delta M) U - C^T Lambda = F and
 * -C U = b_D (Section 3.5), for the system assembled into `sys` (K, M, C, F,
 * bD required; D as well when p != 0). The method is the null-space
 * reduction of the saddle system: the constraint -C U = b_D is parametrised
 * by edge-midpoint values (the lowest-order primal hybrid space is the
 * Crouzeix-Raviart space, Section 1), the projected operator is assembled as
 * a sparse matrix with five entries per row, and Lambda is recovered element
 * by element. With p = 0 the projected operator is symmetric positive
 * definite and conjugate gradients apply; p != 0 (convection) makes it
 * nonsymmetric and needs BiCGSTAB (right-preconditioned). The element
 * blocks are read from K (and M, D) during the call; the multipliers'
 * scaling |E|/2 is the mesh's, the value phf_assemble writes into C.
 * U, Lambda: device, N and L doubles; Lambda may be NULL. Synchronises the
 * stream. Returns
 * PHF_ENOCONV if rtol is not reached in max_iter iterations or BiCGSTAB
 * still breaks down after its restarts (a breakdown restarts it from the
 * current iterate, at most 8 times; the iterate is still written),
 * PHF_EINVAL for CG with p != 0 or p != 0 without D. */
#define PHF_SOLVER_NULLSPACE_CG 0
#define PHF_SOLVER_NULLSPACE_BICGSTAB 1
/* Preconditioners of the reduced operator: Jacobi (any mesh), or a V-cycle
 * over the chain of meshes the mesh was refined from by phf_mesh_refine
 * (edge-midpoint prolongation averaged across coarse edges, polynomial
 * smoothing, coarse operators re-discretised with the triangle coefficient
 * averaged over children, exact solve on the coarsest mesh). */
#define PHF_PRECOND_JACOBI 0
#define PHF_PRECOND_MULTIGRID 1
/* Multigrid smoothers. Each sweep is x += w_k D^-1 (b - A x). JACOBI: every
 * w_k = mg_omega. CHEBYSHEV: the mg_sweeps weights of a side are the
 * reciprocal roots of the Chebyshev polynomial of that degree on
 * [lmax / mg_range, lmax], lmax the level's Gershgorin bound of D^-1 A
 * (computed on the device); with one sweep this is the damping
 * 2 / (lmax (1 + 1 / mg_range)). Errors: mg_sweeps outside 0..8, an unknown
 * smoother, 0 < mg_range <= 1 or mg_omega < 0 give PHF_EINVAL. 0 selects
 * CHEBYSHEV. */
#define PHF_MG_SMOOTH_DEFAULT 0
#define PHF_MG_SMOOTH_JACOBI 1
#define PHF_MG_SMOOTH_CHEBYSHEV 2
typedef struct {
    int32_t method;      /* PHF_SOLVER_*                                   */
    int32_t max_iter;    /* 0 = 20000                                      */
    double rtol;         /* relative residual of the reduced system; 0 = 1e-10 */
    int32_t check_every; /* host convergence test period (iterations); 0 = 8,
                            or with the multigrid preconditioner: CG predicts
                            from the residual decay so far how many to issue
                            before the next test (about one at most past
                            convergence), BiCGSTAB tests after each */
    int32_t saddle_residual; /* 1: compute the saddle residual into stats   */
    int32_t precond;     /* PHF_PRECOND_*                                  */
    int32_t mg_sweeps;   /* sweeps before and after the coarse correction,
                            1..8; 0 = 4 (Chebyshev) or 2 (Jacobi)           */
    double mg_omega;     /* Jacobi damping; 0 = 0.8                         */
    int32_t mg_smoother; /* PHF_MG_SMOOTH_*                                 */
    int32_t reserved_;   /* 0                                               */
    double mg_range;     /* Chebyshev: lmax / lower end of the range (> 1);
                            0 = 10                                          */
    double saddle_rtol;  /* > 0: also require ||F_vec - M_vec W|| / ||F_vec||
                            <= saddle_rtol for the saddle system itself
                            (Section 3.5; needs sys->S and Lambda, CG only):
                            after rtol is met, conjugate gradients continue
                            from the iterate with the reduced tolerance
                            tightened by the observed ratio of the two
                            residuals (at most 6 passes, stopping early when
                            a pass does not halve the saddle residual; not
                            met: the result is written and PHF_ENOCONV
                            returned). Targets below the rounding of the
                            residual itself, about eps || |M_vec| |W| || /
                            ||F_vec|| (growing like 1/h), cannot be met.
                            0: off                                          */
} phf_solver_opts;

typedef struct {
    int32_t iterations;
    int32_t converged;
    double rel_residual;        /* reduced-system ||r|| / ||b||             */
    double saddle_rel_residual; /* ||F_vec - M_vec W|| / ||F_vec|| (if asked) */
} phf_solve_stats;

int phf_solve(phf_mesh* mesh, const phf_coeffs* coeffs, const phf_system* sys,
              const phf_solver_opts* opts, double* U, double* Lambda, phf_solve_stats* stats);

/* ---- error norms ------------------------------------------------------------
 * Broken H^1 seminorm and L^2 norm of u - U_h (the error columns of the
 * tables of Sections 3.7 and 4.2): U_h is the discontinuous piecewise-linear
 * function with vertex values U (device, N doubles; element m at 3m..3m+2),
 * u the exact solution given by `u` at time t, of a kind with a closed-form
 * gradient (PHF_FN_ZERO, CONST, SIN_COS, SIN_SIN, PAPER_U; others give
 * PHF_EINVAL). Each triangle is integrated with a collapsed Gauss-Legendre
 * rule of 5 x 5 points (exact for degree 8); the sums are reduced in a fixed
 * order (deterministic). h1, l2: host outputs. Synchronises the stream. */
int phf_error_norms(phf_mesh* mesh, const double* U, const phf_fn* u, double t, double* h1,
                    double* l2);
/* The same norms for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid allocation):
 * the same kernels and reduction order as phf_error_norms, with its block
 * partial sums in a 16 KiB device array of the library (one per device,
 * shared by every call on that device and kept until the process ends)
 * instead of a pool block. Writes norms[0] = H^1 seminorm, norms[1] = L^2
 * norm into `norms` (device, 2 doubles) on the context's stream and returns
 * without waiting: no allocation, no host copy, no memset, no event. The
 * partial sums of any mesh fit (at most 1024 blocks stride over the
 * elements); a larger count would give PHF_EINVAL. Calls that overlap on one
 * device (other streams or host threads) race on the shared array: order
 * them. The first call on a device resolves the array's address there. */
int phf_error_norms_noalloc(phf_mesh* mesh, const double* U, const phf_fn* u, double t,
                            double* norms);

/* ---- Crank-Nicolson (Section 4) -----------------------------------------
 * M+ W^n = M- W^{n-1} + [k F^{n-1/2}; b_D^{n-1/2}] with
 * M(+/-) = [(1 +/- k delta/2) M +/- (k/2)(K + D), -/+ (k/2) C^T;
 *           -/+ (1/2) C, 0], M the unit mass, and F^{n-1/2}, b_D^{n-1/2} the
 * averages of their evaluations at t_{n-1} and t_n (Section 4.1).
 * phf_cn_create assembles K, M, C once (coeffs as for phf_assemble, p = 0),
 * k > 0. set_state copies U (N) and Lambda (L) device arrays and sets t.
 * phf_cn_run advances nsteps steps with the time-dependent data `data`
 * (data->t is ignored). Each step runs all but the last one or two of the
 * CG iterations it expects (the previous step's count, `iters_per_step` for
 * the first) without reading the device-side convergence flag, then tests it
 * after every further pair (iterations after convergence are skipped on the device). use_graph = 1
 * captures the step as HIP graphs (loads, right-hand side and the first
 * iteration; 2, 4 and 8 further iterations; recovery and state update) and
 * replays them in that pattern. get_state
 * copies the current state out (device) and returns t. stats (may be NULL)
 * receives the total CG iterations and the worst final reduced residual over
 * the steps. */
typedef struct {
    double rtol;            /* 0 = 1e-10                                   */
    int32_t max_iter;       /* per step, eager mode; 0 = 5000             */
    int32_t iters_per_step; /* expected CG iterations of the first step; 0 = 8 */
    int32_t precond;        /* PHF_PRECOND_* (multigrid needs a refined mesh) */
    int32_t mg_sweeps;      /* as for phf_solve                            */
    double mg_omega;        /* 0 = 0.8                                     */
    int32_t mg_smoother;    /* PHF_MG_SMOOTH_*                             */
    int32_t reserved_;      /* 0                                           */
    double mg_range;        /* 0 = 10                                      */
} phf_cn_opts;

int phf_cn_create(phf_mesh* mesh, const phf_coeffs* coeffs, double k, const phf_cn_opts* opts,
                  phf_cn** out);
int phf_cn_set_state(phf_cn* cn, const double* U, const double* Lambda, double t);
int phf_cn_run(phf_cn* cn, const phf_data* data, int32_t nsteps, int32_t use_graph,
               phf_solve_stats* stats);
int phf_cn_get_state(phf_cn* cn, double* U, double* Lambda, double* t);
int phf_cn_destroy(phf_cn* cn);

/* ---- batched Crank-Nicolson (Section 4.1, many problems at once) ---------
 * A batch of n steppers of one context (distinct; meshes of any sizes)
 * advanced together. Each step of each stepper is replayed from its captured
 * HIP graphs (as phf_cn_run with use_graph = 1); the steppers are spread over
 * min(n, 4) streams the batch creates (default priority), so that the small
 * launches of different problems overlap. Per step every stepper runs its
 * head (loads, right-hand side, CG start, first iteration) and CG iterations
 * up to its budget (the smallest odd count >= its last steps' mean count);
 * the context's stream joins them and the convergence flags come back in one
 * read; a stepper that has not converged gets further pairs of iterations
 * (tested after each, and a larger budget from then on); then every
 * stepper's tail (recovery, state update) runs, joined again. Iterations
 * past convergence return at once on the device, so each stepper's state
 * after phf_cn_batch_run equals, bit for bit, the state phf_cn_run would
 * give it. Each stepper must have a state (phf_cn_set_state); data: n
 * entries (as for phf_cn_run, per stepper); stats: n entries or NULL. A
 * stepper in a batch cannot be destroyed (PHF_ESTATE) until the batch is.
 * PHF_ENOCONV if a stepper had a step that did not reach rtol within its
 * max_iter. Returns after the last step has finished. */
typedef struct phf_cn_batch phf_cn_batch;
int phf_cn_batch_create(phf_cn* const* steppers, int32_t n, phf_cn_batch** out);
int phf_cn_batch_run(phf_cn_batch* batch, const phf_data* data, int32_t nsteps,
                     phf_solve_stats* stats);
int phf_cn_batch_destroy(phf_cn_batch* batch);

/* ---- serving ---------------------------------------------------------------
 * A request server on one device: continuous batching of elliptic solves
 * (Section 3) and Crank-Nicolson runs (Section 4) from independent callers.
 * The server has `slots` workers, each with its own context (HIP stream and
 * device memory pool) and host thread. A submitted request is copied (the
 * caller may free its arrays on return) and waits until a slot is free and
 * its estimated device footprint (about 1.4 KB per triangle of the refined
 * mesh for an elliptic solve, 1.8 KB for Crank-Nicolson) fits the memory
 * budget beside the running requests; the first waiting request in arrival
 * order that fits is admitted (a request larger than the budget runs alone).
 * Admitted requests run concurrently on their slots' streams. A request:
 * the base mesh (host arrays, as phf_mesh_create) refined `refine` times on
 * the device; the elliptic kind assembles (coeffs with a_T = NULL, analytic
 * data) and solves by CG (multigrid preconditioner when refine > 0, else
 * Jacobi) to rtol; the Crank-Nicolson kind starts from the edge-midpoint
 * interpolant of u0 at data.t with Lambda = 0 and runs `steps` steps of size
 * k with captured graphs. Optional outputs: U (host buffer of 3 nE 4^refine
 * doubles, written before the request completes) and the error norms of
 * phf_error_norms against `exact` at the final time (when exact is not ZERO
 * or want_norms is set). The result records the status, the triangles of the
 * solved mesh, CG iterations, final relative residual, the slot, and the
 * queueing, running and total (submit to completion) milliseconds. A
 * request's kernels and reductions do not depend on the other requests: its
 * result is the same alone and in a mix. phf_server_wait blocks up to
 * timeout_ms (negative: no limit) and returns PHF_ETIMEDOUT if the request is
 * still unfinished; a result is collected once. phf_server_destroy finishes
 * the queued requests first. */
#define PHF_REQ_ELLIPTIC 0
#define PHF_REQ_CN 1
typedef struct phf_server phf_server;
typedef struct {
    int32_t slots;         /* concurrent requests (1..16); 0 = 4             */
    int32_t reserved_;
    int64_t memory_bytes;  /* admission budget; 0 = half the free device memory */
} phf_server_opts;
typedef struct {
    int32_t kind;          /* PHF_REQ_*                                      */
    int32_t refine;        /* device red refinements of the base mesh (0..12) */
    const double* xy;      /* base mesh, host arrays as for phf_mesh_create  */
    const int32_t* elem;
    const int32_t* dir;
    const int32_t* neu;
    int32_t nC, nE, nD, nN;
    phf_coeffs coeffs;     /* a_T must be NULL                               */
    phf_data data;         /* analytic kinds; data.t: start time              */
    phf_fn u0;             /* Crank-Nicolson initial value                   */
    phf_fn exact;          /* exact solution for the error norms             */
    double rtol;           /* solver tolerance; 0 = 1e-10                    */
    double k;              /* Crank-Nicolson time step                       */
    int32_t steps;         /* Crank-Nicolson steps                           */
    int32_t want_norms;
    double* U_out;         /* optional host output                           */
} phf_request;
typedef struct {
    int32_t status;        /* PHF_OK or the failing call's code              */
    int32_t nE;
    int32_t iterations;
    int32_t slot;
    double rel_residual;
    double h1, l2;         /* -1 when not computed                           */
    double queue_ms, run_ms, latency_ms;
} phf_result;
typedef struct {
    int32_t slots, running, peak_running, queued;
    int64_t completed;
    double budget_bytes, reserved_bytes, peak_reserved_bytes;
} phf_server_stats;
int phf_server_create(int device, const phf_server_opts* opts, phf_server** out);
int phf_server_destroy(phf_server* server);
int phf_server_submit(phf_server* server, const phf_request* req, int64_t* id);
int phf_server_wait(phf_server* server, int64_t id, double timeout_ms, phf_result* result);
int phf_server_query(phf_server* server, phf_server_stats* stats);

#ifdef __cplusplus
}
#endif
#endif /* PHFEM_H */
