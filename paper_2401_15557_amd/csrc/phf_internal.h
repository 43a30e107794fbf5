// Internal declarations of libphfem (not part of the ABI).
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

#include "phfem.h"

// ---------------------------------------------------------------------------
// Context, tracing, errors
// ---------------------------------------------------------------------------

struct phf_trace_rec {
    const char* name;
    hipEvent_t start, stop;
    bool marker;  // events recorded on the stream (else stamped by the launch)
};

struct phf_pool;

struct phf_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    char last_error[512] = {0};
    bool trace = false;
    std::string trace_only;                   // if set, the one kernel name traced
    std::vector<phf_trace_rec> pending;       // recorded, not yet read
    std::vector<hipEvent_t> event_pool;       // reusable events
    std::vector<std::pair<std::string, std::pair<int64_t, double>>> totals;
    std::vector<std::pair<std::string, std::vector<float>>> samples;  // per launch, ms
    int* d_flags = nullptr;                   // small device scratch for checks
    int64_t* h_pinned = nullptr;              // pinned host words for readback
    phf_pool* pool = nullptr;                 // caching device allocator
    int64_t n_objects = 0;                    // live meshes, steppers, batches
};

int phf_set_error(phf_ctx* ctx, int code, const char* fmt, ...);

#define PHF_HIP(ctx, call)                                                          \
    do {                                                                            \
        hipError_t e_ = (call);                                                     \
        if (e_ != hipSuccess)                                                       \
            return phf_set_error((ctx), PHF_EHIP, "%s failed: %s (%s:%d)", #call,   \
                                 hipGetErrorString(e_), __FILE__, __LINE__);         \
    } while (0)

// Launch bracket for tracing: every kernel launch goes through PHF_LAUNCH so
// that an enabled trace times it. A traced launch hands its event pair to
// hipExtLaunchKernelGGL, which stamps them from the kernel's own dispatch
// (the interval a profiler reports, without the queueing around it); an
// untraced launch is a plain launch. phf_trace_begin/end with marker = true
// instead record the events around whatever is issued in between.
void phf_trace_begin(phf_ctx* ctx, const char* name, phf_trace_rec* rec, bool marker = true);
void phf_trace_end(phf_ctx* ctx, phf_trace_rec* rec);

#define PHF_LAUNCH(ctx, name, kernel, grid, block, shmem, ...)                          \
    do {                                                                                \
        phf_trace_rec rec_;                                                             \
        phf_trace_begin((ctx), (name), &rec_, false);                                   \
        if (rec_.start)                                                                 \
            hipExtLaunchKernelGGL(kernel, dim3(grid), dim3(block), (shmem), (ctx)->stream, \
                                  rec_.start, rec_.stop, 0, __VA_ARGS__);               \
        else                                                                            \
            hipLaunchKernelGGL(kernel, dim3(grid), dim3(block), (shmem), (ctx)->stream, \
                               __VA_ARGS__);                                            \
        hipError_t le_ = hipGetLastError();                                             \
        if (le_ != hipSuccess)                                                          \
            return phf_set_error((ctx), PHF_EHIP, "launch of %s failed: %s", (name),    \
                                 hipGetErrorString(le_));                                \
        phf_trace_end((ctx), &rec_);                                                    \
    } while (0)

// Device memory comes from the context's caching pool: a freed block goes
// back to the pool of the context that allocated it and is handed out again
// for a request of the same rounded size. All library work of a context runs
// in order on its one stream, so a block reused there never overlaps work
// that still reads its previous contents. Blocks are returned to HIP by
// phf_release_cache, when an allocation fails, and at phf_destroy.
int phf_dmalloc_bytes(phf_ctx* ctx, void** p, size_t bytes, const char* what);
void phf_dfree_ptr(void* p);

template <typename T>
int phf_dmalloc(phf_ctx* ctx, T** p, size_t count, const char* what)
{
    if (count == 0) count = 1;
    return phf_dmalloc_bytes(ctx, (void**)p, count * sizeof(T), what);
}

template <typename T>
void phf_dfree(T*& p)
{
    if (p) phf_dfree_ptr((void*)p);
    p = nullptr;
}

// ---------------------------------------------------------------------------
// Mesh
// ---------------------------------------------------------------------------

// Per-element code word (fourth int of the element record):
//   bits 2i..2i+1  type of local edge i (0 interior, 1 Dirichlet, 2 Neumann)
//   bit  6+i       element is T+ of local edge i
//   bit  9+i       of the two edges through vertex i (local indices l1 < l2,
//                  both != i), edge l1 has the larger global id
#define PHF_CODE_TYPE(code, i) (((code) >> (2 * (i))) & 3)
#define PHF_CODE_TPLUS(code, i) (((code) >> (6 + (i))) & 1)
#define PHF_CODE_SWAP(code, i) (((code) >> (9 + (i))) & 1)

struct phf_ns;
void phf_ns_destroy(phf_ns* ns);

struct phf_mesh {
    phf_ctx* ctx = nullptr;
    phf_ns* ns = nullptr;          // cached solver workspace (lazy)
    phf_mesh* parent = nullptr;    // coarse mesh this one was refined from
    int32_t n_children = 0;        // meshes refined from this one, still alive
    int32_t n_users = 0;           // Crank-Nicolson steppers and batches using it
    int32_t nC = 0, nE = 0, n_edges = 0, L = 0, nD = 0, nN = 0, n_int = 0, n_free = 0;
    int64_t nnz_C = 0, nnz_S = 0, nnz_R = 0;
    int64_t bytes = 0;
    // geometry and elements
    double2* xy = nullptr;         // nC
    int4* elem4 = nullptr;         // nE: v0, v1, v2, code
    double2* exy = nullptr;        // 3 nE: vertex coordinates of each element, element-major
    int32_t* ecode = nullptr;      // nE: the code word alone
    // edge tables
    int2* edge_nodes = nullptr;    // n_edges: (k, l) as traversed by T+
    int2* edge_elems = nullptr;    // n_edges: (T+, T-)
    int32_t* elem_edges = nullptr; // 3 nE: edge opposite local vertex i
    int8_t* led = nullptr;         // n_edges
    int8_t* ledTN = nullptr;       // n_edges
    int8_t* edge_type = nullptr;   // n_edges
    int32_t* edge_row = nullptr;   // n_edges (-1 Neumann)
    int32_t* dir_edges = nullptr;  // nD
    int32_t* neu_edges = nullptr;  // nN
    int2* dir_pairs = nullptr;     // nD: listed node pairs, as given
    int2* neu_pairs = nullptr;     // nN
    // multiplier rows
    int32_t* row_edge = nullptr;   // L
    double* row_hs = nullptr;      // L: |E|/2 of the row's edge, negated on Dirichlet rows
    int2* row_nodes = nullptr;     // L: (k, l) of the row's edge; k stored as ~k
                                   // (negative) on Dirichlet rows
    int32_t* C_tile = nullptr;     // L/256 + 1: C row pointer of every 256th row
    uint64_t* neu_mask = nullptr;  // nE/64: bit m%64 of word m/64 set iff element m
                                   // has a Neumann edge
    int32_t* C_rowptr = nullptr;   // L + 1
    int32_t* C_col = nullptr;      // nnz_C
    int32_t* S_rowptr = nullptr;   // N + L + 1
    int32_t* S_col = nullptr;      // nnz_S
    // reduced (edge-midpoint) operator: rows = non-Dirichlet edges
    int32_t* red_row = nullptr;    // n_edges: reduced index, -1 for Dirichlet
    int32_t* red_edge = nullptr;   // n_free: edge of reduced row
    // per element, the rows of its local edges l (3 nE, element-major)
    int32_t* elem_row = nullptr;   // multiplier row (-1 Neumann)
    int32_t* elem_red = nullptr;   // reduced row (-1 Dirichlet)
    unsigned long long* d_nnzR = nullptr;  // entries of the reduced operator (device)
};

// Exclusive scan of n int32 values (in may alias out); total -> *d_total.
int phf_scan_i32(phf_ctx* ctx, const int32_t* in, int32_t* out, int32_t n, int32_t* d_total);

// Device function catalogue (problem data), see phfem.h PHF_FN_*.
struct phf_fn_dev {
    int32_t kind;
    double c0, c1, c2, c3;
    const double* ev;
};

inline phf_fn_dev phf_fn_to_dev(const phf_fn& f)
{
    phf_fn_dev d;
    d.kind = f.kind;
    d.c0 = f.c[0];
    d.c1 = f.c[1];
    d.c2 = f.c[2];
    d.c3 = f.c[3];
    d.ev = f.edge_values;
    return d;
}

bool phf_fn_valid(const phf_fn& f);
bool phf_fn_needs_edge(const phf_fn& f);

// Assembly entry used by the solver and Crank-Nicolson modules. With
// t_step non-null the kernels read the time as t0 + (*t_step) * dt from
// device memory instead of data->t (for graph-captured time loops).
int phf_assemble_impl(phf_mesh* mesh, const phf_coeffs* coeffs, const phf_data* data,
                      const phf_system* out, const int64_t* t_step = nullptr, double t0 = 0.0,
                      double dt = 0.0);

// Small device helpers shared by the solver modules.
int phf_dot(phf_ctx* ctx, const double* x, const double* y, int32_t n, double* d_partials,
            double* d_out);
