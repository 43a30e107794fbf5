// Crank-Nicolson time stepping of the parabolic problem (Section 4.1):
//   M+ W^n = M- W^{n-1} + [k F^{n-1/2}; b_D^{n-1/2}],
// solved each step by the null-space CG of phf_solver with the constant
// operator A+ = (1 + k delta/2) M + (k/2) K. With mu = (k/2) Lambda^n the
// step is A+ U^n - C^T mu = r1, -C U^n = r2 where
//   r1 = A- U^{n-1} + (k/2) C^T Lambda^{n-1} + (k/2)(F^{n-1} + F^n),
//   r2 = C U^{n-1} + b_D^{n-1} + b_D^n,  A- = (1 - k delta/2) M - (k/2) K.
// One step is a fixed kernel sequence whose only time input is a device step
// counter, so it can be captured once in a HIP graph and replayed.
#include <algorithm>
#include <cmath>
#include <vector>

#include "phf_device.h"
#include "phf_solver.h"

struct phf_cn {
    phf_mesh* mesh = nullptr;
    phf_ns* ns = nullptr;
    double k = 0, delta = 0;
    phf_coeffs co{};
    phf_cn_opts opts{};
    // K and M are assembled once; after the operator A+ is built only
    // A- = (1 - k delta/2) M - (k/2) K is kept (9 values per element)
    double *K = nullptr, *M = nullptr, *Am = nullptr, *C = nullptr, *Fs = nullptr, *bs = nullptr;
    double *U = nullptr, *Lam = nullptr;
    double *F0 = nullptr, *F1 = nullptr, *bD0 = nullptr, *bD1 = nullptr;
    double *r1 = nullptr, *r2 = nullptr;
    // per element and local edge: sigma_l |E_l| / 2 (+ on T+, - on T-), 0 on
    // Neumann edges; the weights of the multipliers in C^T Lambda
    double* sgh = nullptr;
    int64_t* d_step = nullptr;  // index n of the step being (or next) computed
    // reduced solutions of the last four steps (a ring of four vectors of
    // n_free values) and, on the device, {solves since set_state capped at 4,
    // ring slot of the latest}
    double* wr = nullptr;
    int32_t* d_nsol = nullptr;
    double* d_stats = nullptr;  // [0] CG iterations, [1] worst relres, [2] unconverged steps
    double t0 = 0;
    int64_t n = 0;              // completed steps since set_state
    bool have_state = false;
    // CG iterations of the previous step: the next step launches one fewer
    // without a convergence read-back, then tests after every pair
    int32_t predict = 0;
    // graph mode: [0] head (loads, right-hand side, CG start, first
    // iteration), [1..3] 2, 4, 8 further iterations, [4] tail
    static constexpr int NG = 5;
    hipGraphExec_t gx[NG] = {};
    hipGraph_t g[NG] = {};
    phf_data gdata{};           // data the graphs were captured with
    bool counted = false;       // registered with the mesh and context
    int32_t n_batches = 0;      // batches (phf_cn_batch) this stepper is part of
};

namespace {
constexpr int NT = 256;
inline unsigned nblk(int64_t n) { return (unsigned)((n + NT - 1) / NT); }

#define TRY(x)               \
    do {                     \
        int rc_ = (x);       \
        if (rc_) return rc_; \
    } while (0)

// Initial CG guess from the reduced solutions of the last time levels, w1
// (latest) to w4. Crank-Nicolson leaves the stiff error modes undamped (their
// amplification factor tends to -1), so beside its smooth part the sequence
// of solutions alternates in sign from step to step; a smooth extrapolation
// (2 w1 - w2) errs by four times that component and needs as many
// iterations as starting from w1. With four levels the guess is exact for a
// quadratic trend plus a constant alternation, 2 (w1 - w3) + w4; with three,
// for a linear trend plus the alternation, w2 + (w1 - w3); with one or two,
// w1; with none, 0.
constexpr int CN_RING = 4;
__global__ __launch_bounds__(NT) void k_cn_guess(int32_t nf, const int32_t* __restrict__ nsol,
                                                 const double* __restrict__ wr,
                                                 double* __restrict__ w)
{
    const int32_t c = nsol[0], h = nsol[1];
    const double* w1 = wr + (int64_t)h * nf;
    const double* w2 = wr + (int64_t)((h + 3) % CN_RING) * nf;
    const double* w3 = wr + (int64_t)((h + 2) % CN_RING) * nf;
    const double* w4 = wr + (int64_t)((h + 1) % CN_RING) * nf;
    for (int32_t i = blockIdx.x * NT + threadIdx.x; i < nf; i += gridDim.x * NT) {
        double g = 0.0;
        if (c >= 4) g = 2.0 * (w1[i] - w3[i]) + w4[i];
        else if (c == 3) g = w2[i] + (w1[i] - w3[i]);
        else if (c >= 1) g = w1[i];
        w[i] = g;
    }
}

// The step's solution into the next ring slot (one vector written, none
// moved); k_cn_close then advances the counters.
__global__ __launch_bounds__(NT) void k_cn_keep(int32_t nf, const int32_t* __restrict__ nsol,
                                                const double* __restrict__ w,
                                                double* __restrict__ wr)
{
    double* dst = wr + (int64_t)((nsol[1] + 1) % CN_RING) * nf;
    for (int32_t i = blockIdx.x * NT + threadIdx.x; i < nf; i += gridDim.x * NT) dst[i] = w[i];
}

// Area of the domain of a mesh: the sum of its element areas in one
// workgroup, in a fixed order.
__global__ __launch_bounds__(1024) void k_cn_area(int32_t nE, const double2* __restrict__ exy,
                                                  double* __restrict__ out)
{
    __shared__ double sh[1024];
    double s = 0.0;
    for (int32_t m = threadIdx.x; m < nE; m += 1024) {
        const double2 a = exy[3 * (int64_t)m], b = exy[3 * (int64_t)m + 1],
                      c = exy[3 * (int64_t)m + 2];
        s += 0.5 * ((b.x - a.x) * (c.y - a.y) - (c.x - a.x) * (b.y - a.y));
    }
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int h = 512; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) sh[threadIdx.x] += sh[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = sh[0];
}

// A- = cM M - cK K per element block, once per stepper.
// (Am may be K itself: each element is read before it is written.)
__global__ __launch_bounds__(NT) void k_cn_aminus(int64_t n, const double* K,
                                                  const double* __restrict__ M, double cM,
                                                  double cK, double* Am)
{
    const int64_t q = (int64_t)blockIdx.x * NT + threadIdx.x;
    if (q < n) Am[q] = cM * M[q] - cK * K[q];
}

// sigma_l |E_l| / 2 per element and local edge, once per stepper (the
// factor k_cn_rhs_elem applies to each multiplier, as a stream instead of a
// gather of the row's half-length).
__global__ __launch_bounds__(NT) void k_cn_sgh(int32_t nE, const int32_t* __restrict__ ecode,
                                               const int32_t* __restrict__ elem_row,
                                               const double* __restrict__ row_hs,
                                               double* __restrict__ sgh)
{
    const int64_t q = (int64_t)blockIdx.x * NT + threadIdx.x;
    if (q >= 3 * (int64_t)nE) return;
    const int64_t m = q / 3;
    const int l = (int)(q - 3 * m);
    const int code = ecode[m];
    double v = 0.0;
    if (PHF_CODE_TYPE(code, l) != 2)
        v = (PHF_CODE_TPLUS(code, l) ? 1.0 : -1.0) * fabs(row_hs[elem_row[q]]);
    sgh[q] = v;
}

// r1 per element (see file comment); the tile's A- blocks go through LDS so
// that they are read with coalesced accesses. F0 (the load at t_{n-1}) then
// takes F1's values, the next step's F0.
__global__ __launch_bounds__(NT) void k_cn_rhs_elem(
    int32_t nE, const double* __restrict__ Am, const double* __restrict__ U,
    const double* __restrict__ Lam, const int32_t* __restrict__ elem_row,
    const double* __restrict__ sgh, double* __restrict__ F0, const double* __restrict__ F1,
    double hk, double* __restrict__ r1)
{
    __shared__ double sA[9 * NT];
    const int tid = threadIdx.x;
    const int64_t m0 = (int64_t)blockIdx.x * NT;
    const int32_t nt = (int32_t)min((int64_t)NT, (int64_t)nE - m0);
    for (int32_t q = tid; q < 9 * nt; q += NT) sA[q] = Am[9 * m0 + q];
    __syncthreads();
    if (tid >= nt) return;
    const int64_t m = m0 + tid;
    double u[3], lt[3];
#pragma unroll
    for (int l = 0; l < 3; ++l) {
        u[l] = U[3 * m + l];
        // sigma_l h_l Lambda_row(l) for non-Neumann local edges (row -1)
        const int32_t r = elem_row[3 * m + l];
        lt[l] = r >= 0 ? sgh[3 * m + l] * Lam[r] : 0.0;
    }
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        const double* a = sA + 9 * tid + 3 * i;
        double au = 0.0;
#pragma unroll
        for (int j = 0; j < 3; ++j) au += a[j] * u[j];
        // (C^T Lambda)_i = sum over the two edges through vertex i
        double ctl = 0.0;
#pragma unroll
        for (int l = 0; l < 3; ++l) ctl += (l == i) ? 0.0 : lt[l];
        const double f0 = F0[3 * m + i], f1 = F1[3 * m + i];
        r1[3 * m + i] = au + hk * ctl + hk * (f0 + f1);
        F0[3 * m + i] = f1;
    }
}

// r2 per multiplier row: (C U)_r + b_D^{n-1} + b_D^n; bD0 then takes bD1's
// value, the next step's b_D^{n-1}.
__global__ __launch_bounds__(NT) void k_cn_rhs_row(int32_t L, const int32_t* __restrict__ C_rowptr,
                                                   const int32_t* __restrict__ C_col,
                                                   const double* __restrict__ C,
                                                   const double* __restrict__ U,
                                                   double* __restrict__ bD0,
                                                   const double* __restrict__ bD1,
                                                   double* __restrict__ r2)
{
    int32_t r = blockIdx.x * NT + threadIdx.x;
    if (r >= L) return;
    double s = 0.0;
    for (int32_t q = C_rowptr[r]; q < C_rowptr[r + 1]; ++q) s += C[q] * U[C_col[q]];
    const double b0 = bD0[r], b1 = bD1[r];
    r2[r] = s + b0 + b1;
    bD0[r] = b1;
}

// The step's scalars, in one thread after the step: the solve statistics
// (iterations, worst relative residual, unconverged steps), the ring
// counters of k_cn_keep (when there are free unknowns) and the step index
// the next step's loads are evaluated at.
__global__ void k_cn_close(const int* __restrict__ iflags, const double* __restrict__ scal,
                           double* __restrict__ st, int32_t* __restrict__ nsol,
                           int64_t* __restrict__ step)
{
    st[0] += iflags[1];
    double rel = scal[NS_BB] > 0 ? sqrt(scal[NS_RR] / scal[NS_BB]) : 0.0;
    st[1] = fmax(st[1], rel);
    st[2] += iflags[0] ? 0.0 : 1.0;
    if (nsol) {
        nsol[0] = min(nsol[0] + 1, CN_RING);
        nsol[1] = (nsol[1] + 1) % CN_RING;
    }
    *step += 1;
}

// Coarsest levels of the refinement chain to leave out of the step
// operator's multigrid hierarchy: level l (mean triangle area |Omega| / nE_l)
// counts as mass-dominated when cK a nE_l <= cM |Omega|, with a the larger
// diagonal entry of the constant coefficient A (with a per-element a_T
// nothing is left out). The stiffness part of an element block is of the
// order cK a, its mass part cM |T| / 12, so on such a level smoothing alone
// reduces every component and the levels below it add launches but little
// correction; the hierarchy starts at the finest mass-dominated level.
// Measured on the paper mesh refined 9 times with k = 1e-3 (cK a nE_l /
// (cM |Omega|) = 0.5 on the level of 1,024 triangles, 2.0 on the next):
// levels 0-3 left out, 689 -> 712 steps/s at 3.06 CG iterations per step;
// leaving out the next level as well raised them to 4.2.
int domain_area(const phf_mesh* m, double* d_area, double* area)
{
    phf_ctx* ctx = m->ctx;
    PHF_LAUNCH(ctx, "k_cn_area", k_cn_area, 1, 1024, 0, m->nE, (const double2*)m->exy, d_area);
    PHF_HIP(ctx, hipMemcpyAsync(area, d_area, sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    PHF_HIP(ctx, hipStreamSynchronize(ctx->stream));
    return PHF_OK;
}

int mass_levels(phf_mesh* mesh, const phf_coeffs* co, double cK, double cM, int32_t* out)
{
    *out = 0;
    if (!(cM > 0.0) || co->a_T) return PHF_OK;
    std::vector<phf_mesh*> chain;  // finest first
    for (phf_mesh* m = mesh; m; m = m->parent) chain.push_back(m);
    if (chain.size() < 3) return PHF_OK;
    phf_ctx* ctx = mesh->ctx;
    double* d_area = nullptr;
    TRY(phf_dmalloc(ctx, &d_area, 1, "domain area"));
    double area = 0.0;
    const int rc = domain_area(chain.back(), d_area, &area);  // the coarsest mesh: fewest elements
    phf_dfree(d_area);
    TRY(rc);
    const double a = std::max(std::fabs(co->A[0]), std::fabs(co->A[3]));
    int32_t drop = 0;
    for (size_t q = chain.size(); q-- > 0;) {  // coarsest first
        const int32_t l = (int32_t)(chain.size() - 1 - q);
        if (cK * a * (double)chain[q]->nE <= cM * area) drop = l;
        else break;
    }
    *out = drop;
    return PHF_OK;
}

int cn_loads(phf_cn* cn, const phf_data* data, double* F, double* bD, bool from_device)
{
    phf_system s{};
    s.F = F;
    s.bD = bD;
    if (from_device) return phf_assemble_impl(cn->mesh, &cn->co, data, &s, cn->d_step, cn->t0, cn->k);
    phf_data d = *data;
    d.t = cn->t0 + (double)cn->n * cn->k;
    return phf_assemble_impl(cn->mesh, &cn->co, &d, &s);
}

// Everything of one step before the CG iterations.
int cn_step_head(phf_cn* cn, const phf_data* data)
{
    phf_mesh* mesh = cn->mesh;
    phf_ctx* ctx = mesh->ctx;
    const int32_t nE = mesh->nE, L = mesh->L;
    TRY(cn_loads(cn, data, cn->F1, cn->bD1, true));
    const double hk = 0.5 * cn->k;
    PHF_LAUNCH(ctx, "k_cn_rhs_elem", k_cn_rhs_elem, nblk(nE), NT, 0, nE, cn->Am, cn->U,
               cn->Lam, cn->ns->elem_row, cn->sgh, cn->F0, cn->F1, hk, cn->r1);
    if (L > 0)
        PHF_LAUNCH(ctx, "k_cn_rhs_row", k_cn_rhs_row, nblk(L), NT, 0, L, mesh->C_rowptr,
                   mesh->C_col, cn->C, cn->U, cn->bD0, cn->bD1, cn->r2);
    // (C U + b_D has interior jumps; the edge weights give |E|/2 per element edge)
    TRY(phf_ns_rhs(cn->ns, cn->r1, cn->r2, true, cn->sgh));
    if (cn->ns->nf > 0)
        PHF_LAUNCH(ctx, "k_cn_guess", k_cn_guess, cn->ns->nbv, NT, 0, cn->ns->nf, cn->d_nsol,
                   cn->wr, cn->ns->w);
    TRY(phf_ns_cg_start(cn->ns, cn->opts.rtol));
    return PHF_OK;
}

int cn_step_tail(phf_cn* cn)
{
    phf_mesh* mesh = cn->mesh;
    phf_ctx* ctx = mesh->ctx;
    TRY(phf_ns_recover(cn->ns, cn->r1, cn->U, cn->Lam, 2.0 / cn->k));
    const bool keep = cn->ns->nf > 0;
    if (keep)
        PHF_LAUNCH(ctx, "k_cn_keep", k_cn_keep, cn->ns->nbv, NT, 0, cn->ns->nf, cn->d_nsol,
                   cn->ns->w, cn->wr);
    PHF_LAUNCH(ctx, "k_cn_close", k_cn_close, 1, 1, 0, cn->ns->iflags, cn->ns->scal, cn->d_stats,
               keep ? cn->d_nsol : nullptr, cn->d_step);
    return PHF_OK;
}

void cn_drop_graph(phf_cn* cn)
{
    for (int q = 0; q < phf_cn::NG; ++q) {
        if (cn->gx[q]) (void)hipGraphExecDestroy(cn->gx[q]);
        if (cn->g[q]) (void)hipGraphDestroy(cn->g[q]);
        cn->gx[q] = nullptr;
        cn->g[q] = nullptr;
    }
}

bool same_fn(const phf_fn& a, const phf_fn& b)
{
    return a.kind == b.kind && a.c[0] == b.c[0] && a.c[1] == b.c[1] && a.c[2] == b.c[2] &&
           a.c[3] == b.c[3] && a.edge_values == b.edge_values;
}

// Captures part q of a step (0: head with the first iteration; 1, 2, 3:
// 2, 4, 8 iterations; 4: tail). The kernels of an iteration only depend on
// whether it is the first and on its parity; every iteration graph starts at
// an odd index and has an even length, so they can follow each other freely.
int cn_capture_part(phf_cn* cn, const phf_data* data, int q, hipStream_t cap)
{
    phf_ctx* ctx = cn->mesh->ctx;
    int rc = PHF_OK;
    hipError_t e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess)
        return phf_set_error(ctx, PHF_EHIP, "begin capture failed: %s", hipGetErrorString(e));
    if (q == 0) {
        rc = cn_step_head(cn, data);
        if (!rc) rc = phf_ns_cg_iterate(cn->ns, 1);
    } else if (q < phf_cn::NG - 1) {
        cn->ns->next_it = 1;
        rc = phf_ns_cg_iterate(cn->ns, 1 << q);
    } else {
        rc = cn_step_tail(cn);
    }
    hipGraph_t g = nullptr;
    hipError_t e2 = hipStreamEndCapture(cap, &g);
    if (!rc && e2 != hipSuccess)
        rc = phf_set_error(ctx, PHF_EHIP, "graph capture failed: %s", hipGetErrorString(e2));
    if (!rc) {
        cn->g[q] = g;
        e2 = hipGraphInstantiate(&cn->gx[q], g, nullptr, nullptr, 0);
        if (e2 != hipSuccess)
            rc = phf_set_error(ctx, PHF_EHIP, "graph instantiation failed: %s",
                               hipGetErrorString(e2));
    } else if (g) {
        (void)hipGraphDestroy(g);
    }
    return rc;
}

int cn_capture(phf_cn* cn, const phf_data* data)
{
    phf_ctx* ctx = cn->mesh->ctx;
    hipStream_t cap = nullptr;
    PHF_HIP(ctx, hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
    hipStream_t saved = ctx->stream;
    bool saved_trace = ctx->trace;
    ctx->stream = cap;
    ctx->trace = false;
    int rc = PHF_OK;
    for (int q = 0; q < phf_cn::NG && !rc; ++q) rc = cn_capture_part(cn, data, q, cap);
    ctx->stream = saved;
    ctx->trace = saved_trace;
    (void)hipStreamDestroy(cap);
    if (rc) cn_drop_graph(cn);
    else cn->gdata = *data;
    return rc;
}
}  // namespace

extern "C" int phf_cn_destroy(phf_cn* cn)
{
    if (!cn) return PHF_EINVAL;
    if (cn->n_batches > 0)
        return phf_set_error(cn->mesh->ctx, PHF_ESTATE,
                             "phf_cn_destroy: the stepper is part of %d batches", cn->n_batches);
    (void)hipStreamSynchronize(cn->mesh->ctx->stream);
    if (cn->counted) {
        cn->mesh->n_users--;
        cn->mesh->ctx->n_objects--;
    }
    cn_drop_graph(cn);
    if (cn->ns) phf_ns_destroy(cn->ns);
    double* bufs[] = {cn->K, cn->M, cn->Am, cn->C, cn->Fs, cn->bs, cn->U, cn->Lam, cn->F0,
                      cn->F1, cn->bD0, cn->bD1, cn->r1, cn->r2, cn->sgh, cn->d_stats};
    for (double* b : bufs) phf_dfree(b);
    phf_dfree(cn->d_step);
    phf_dfree(cn->wr);
    phf_dfree(cn->d_nsol);
    delete cn;
    return PHF_OK;
}

extern "C" int phf_cn_create(phf_mesh* mesh, const phf_coeffs* co, double k,
                             const phf_cn_opts* opts, phf_cn** out)
{
    if (!mesh || !co || !out) return PHF_EINVAL;
    phf_ctx* ctx = mesh->ctx;
    *out = nullptr;
    if (!(k > 0.0) || co->p[0] != 0.0 || co->p[1] != 0.0)
        return phf_set_error(ctx, PHF_EINVAL, "phf_cn_create: need k > 0 and p = 0");
    phf_cn* cn = new (std::nothrow) phf_cn;
    if (!cn) return phf_set_error(ctx, PHF_ENOMEM, "host allocation failed");
    cn->mesh = mesh;
    cn->k = k;
    cn->delta = co->delta;
    cn->co = *co;
    cn->opts.rtol = opts && opts->rtol > 0 ? opts->rtol : 1e-10;
    cn->opts.max_iter = opts && opts->max_iter > 0 ? opts->max_iter : 5000;
    cn->opts.iters_per_step = opts && opts->iters_per_step > 0 ? opts->iters_per_step : 8;
    cn->predict = cn->opts.iters_per_step;
    cn->opts.precond = opts ? opts->precond : PHF_PRECOND_JACOBI;
    cn->opts.mg_sweeps = opts ? opts->mg_sweeps : 0;
    cn->opts.mg_omega = opts ? opts->mg_omega : 0.0;
    cn->opts.mg_smoother = opts ? opts->mg_smoother : 0;
    cn->opts.mg_range = opts ? opts->mg_range : 0.0;
    if (cn->opts.precond != PHF_PRECOND_JACOBI && cn->opts.precond != PHF_PRECOND_MULTIGRID) {
        delete cn;
        return phf_set_error(ctx, PHF_EINVAL, "phf_cn_create: unknown preconditioner");
    }
    const size_t N = 3 * (size_t)mesh->nE, L = mesh->L, nnzK = 9 * (size_t)mesh->nE;
    auto body = [&]() -> int {
        TRY(phf_dmalloc(ctx, &cn->K, nnzK, "CN K"));
        TRY(phf_dmalloc(ctx, &cn->M, nnzK, "CN M"));
        TRY(phf_dmalloc(ctx, &cn->C, mesh->nnz_C, "CN C"));
        TRY(phf_dmalloc(ctx, &cn->Fs, N, "CN F"));
        TRY(phf_dmalloc(ctx, &cn->bs, L, "CN bD"));
        TRY(phf_dmalloc(ctx, &cn->U, N, "CN U"));
        TRY(phf_dmalloc(ctx, &cn->Lam, L, "CN Lambda"));
        TRY(phf_dmalloc(ctx, &cn->F0, N, "CN F0"));
        TRY(phf_dmalloc(ctx, &cn->F1, N, "CN F1"));
        TRY(phf_dmalloc(ctx, &cn->bD0, L, "CN bD0"));
        TRY(phf_dmalloc(ctx, &cn->bD1, L, "CN bD1"));
        TRY(phf_dmalloc(ctx, &cn->r1, N, "CN r1"));
        TRY(phf_dmalloc(ctx, &cn->sgh, N, "CN edge weights"));
        TRY(phf_dmalloc(ctx, &cn->r2, L, "CN r2"));
        TRY(phf_dmalloc(ctx, &cn->d_stats, 4, "CN stats"));
        TRY(phf_dmalloc(ctx, &cn->d_step, 1, "CN step"));
        TRY(phf_dmalloc(ctx, &cn->wr, CN_RING * (size_t)std::max<int32_t>(mesh->n_free, 1),
                        "CN solution ring"));
        TRY(phf_dmalloc(ctx, &cn->d_nsol, 2, "CN solves"));
        // K, M, C once (the coefficient is time independent)
        phf_system s{};
        s.K = cn->K;
        s.M = cn->M;
        s.C = cn->C;
        s.F = cn->Fs;
        s.bD = cn->bs;
        phf_data d{};
        TRY(phf_assemble_impl(mesh, co, &d, &s));
        TRY(phf_ns_create(mesh, &cn->ns));
        if (N > 0)
            PHF_LAUNCH(ctx, "k_cn_sgh", k_cn_sgh, nblk((int64_t)N), NT, 0, mesh->nE, mesh->ecode,
                       cn->ns->elem_row, mesh->row_hs, cn->sgh);
        TRY(phf_ns_operator(cn->ns, cn->K, cn->M, 0.5 * k, 1.0 + 0.5 * k * co->delta));
        phf_mg_params mp;
        mp.sweeps = cn->opts.mg_sweeps;
        mp.smoother = cn->opts.mg_smoother;
        mp.omega = cn->opts.mg_omega;
        mp.range = cn->opts.mg_range;
        if (cn->opts.precond == PHF_PRECOND_MULTIGRID)
            TRY(mass_levels(mesh, co, 0.5 * k, 1.0 + 0.5 * k * co->delta, &mp.drop_coarse));
        TRY(phf_ns_set_precond(cn->ns, cn->opts.precond, mp, co, 0.5 * k,
                               1.0 + 0.5 * k * co->delta));
        // A- in K's place; M is no longer needed
        PHF_LAUNCH(ctx, "k_cn_aminus", k_cn_aminus, nblk((int64_t)nnzK), NT, 0, (int64_t)nnzK,
                   cn->K, cn->M, 1.0 - 0.5 * k * co->delta, 0.5 * k, cn->K);
        PHF_HIP(ctx, hipStreamSynchronize(ctx->stream));
        cn->Am = cn->K;
        cn->K = nullptr;
        phf_dfree(cn->M);
        return PHF_OK;
    };
    int rc = body();
    if (rc) {
        phf_cn_destroy(cn);
        return rc;
    }
    // the per-element coefficient is consumed by the assembly above
    cn->co.a_T = nullptr;
    cn->counted = true;
    mesh->n_users++;
    ctx->n_objects++;
    *out = cn;
    return PHF_OK;
}

extern "C" int phf_cn_set_state(phf_cn* cn, const double* U, const double* Lambda, double t)
{
    if (!cn || !U || !Lambda) return PHF_EINVAL;
    phf_ctx* ctx = cn->mesh->ctx;
    const size_t N = 3 * (size_t)cn->mesh->nE, L = cn->mesh->L;
    PHF_HIP(ctx, hipMemcpyAsync(cn->U, U, N * 8, hipMemcpyDeviceToDevice, ctx->stream));
    if (L) PHF_HIP(ctx, hipMemcpyAsync(cn->Lam, Lambda, L * 8, hipMemcpyDeviceToDevice, ctx->stream));
    cn->t0 = t;
    cn->n = 0;
    cn->have_state = true;
    TRY(phf_ns_zero_w(cn->ns));
    PHF_HIP(ctx, hipMemsetAsync(cn->d_nsol, 0, 2 * sizeof(int32_t), ctx->stream));
    return PHF_OK;
}

extern "C" int phf_cn_get_state(phf_cn* cn, double* U, double* Lambda, double* t)
{
    if (!cn) return PHF_EINVAL;
    phf_ctx* ctx = cn->mesh->ctx;
    const size_t N = 3 * (size_t)cn->mesh->nE, L = cn->mesh->L;
    if (U) PHF_HIP(ctx, hipMemcpyAsync(U, cn->U, N * 8, hipMemcpyDeviceToDevice, ctx->stream));
    if (Lambda && L)
        PHF_HIP(ctx, hipMemcpyAsync(Lambda, cn->Lam, L * 8, hipMemcpyDeviceToDevice, ctx->stream));
    if (t) *t = cn->t0 + (double)cn->n * cn->k;
    return PHF_OK;
}

extern "C" int phf_cn_run(phf_cn* cn, const phf_data* data, int32_t nsteps, int32_t use_graph,
                          phf_solve_stats* stats)
{
    if (!cn || !data || nsteps < 0) return PHF_EINVAL;
    phf_ctx* ctx = cn->mesh->ctx;
    if (!cn->have_state) return phf_set_error(ctx, PHF_ESTATE, "phf_cn_run: call phf_cn_set_state first");
    if (!phf_fn_valid(data->f) || !phf_fn_valid(data->g) || !phf_fn_valid(data->uD))
        return phf_set_error(ctx, PHF_EINVAL, "phf_cn_run: unknown function kind or missing edge array");
    // loads at the current time and the device step counter
    TRY(cn_loads(cn, data, cn->F0, cn->bD0, false));
    int64_t n_host = cn->n + 1;  // index of the next step
    PHF_HIP(ctx, hipMemcpyAsync(cn->d_step, &n_host, sizeof(int64_t), hipMemcpyHostToDevice, ctx->stream));
    PHF_HIP(ctx, hipMemsetAsync(cn->d_stats, 0, 4 * sizeof(double), ctx->stream));
    PHF_HIP(ctx, hipStreamSynchronize(ctx->stream));
    if (use_graph) {
        if (cn->gx[0] && !(same_fn(cn->gdata.f, data->f) && same_fn(cn->gdata.g, data->g) &&
                           same_fn(cn->gdata.uD, data->uD)))
            cn_drop_graph(cn);
        if (!cn->gx[0]) TRY(cn_capture(cn, data));
    }
    for (int32_t s = 0; s < nsteps; ++s) {
        phf_trace_rec rec;
        phf_trace_begin(ctx, use_graph ? "cn_graph_step" : "cn_step", &rec);
        // head and first iteration, then the rest of the predicted count
        // (the last step's) rounded down to pairs without reading the flag,
        // then pairs until converged: a step that needs as many iterations as
        // the last one reads the flag once (measured: 640 -> 648 steps/s
        // against holding back one more iteration)
        int32_t it = 1;
        const int32_t blind = std::max<int32_t>(cn->predict - 1, 0) & ~1;
        if (use_graph) {
            PHF_HIP(ctx, hipGraphLaunch(cn->gx[0], ctx->stream));
            for (int q = phf_cn::NG - 2; q >= 1; --q)
                while (it - 1 + (1 << q) <= blind) {
                    PHF_HIP(ctx, hipGraphLaunch(cn->gx[q], ctx->stream));
                    it += 1 << q;
                }
        } else {
            TRY(cn_step_head(cn, data));
            TRY(phf_ns_cg_iterate(cn->ns, 1));
            cn->ns->next_it = 1;
            if (blind > 0) TRY(phf_ns_cg_iterate(cn->ns, blind));
            it += blind;
        }
        int hf[2] = {0, 0};
        for (;;) {
            PHF_HIP(ctx, hipMemcpyAsync(hf, cn->ns->iflags, 2 * sizeof(int), hipMemcpyDeviceToHost,
                                        ctx->stream));
            PHF_HIP(ctx, hipStreamSynchronize(ctx->stream));
            if (hf[0] || it >= cn->opts.max_iter) break;
            if (use_graph) {
                PHF_HIP(ctx, hipGraphLaunch(cn->gx[1], ctx->stream));
            } else {
                cn->ns->next_it = 1;
                TRY(phf_ns_cg_iterate(cn->ns, 2));
            }
            it += 2;
        }
        cn->predict = hf[1];
        if (use_graph)
            PHF_HIP(ctx, hipGraphLaunch(cn->gx[phf_cn::NG - 1], ctx->stream));
        else
            TRY(cn_step_tail(cn));
        phf_trace_end(ctx, &rec);
    }
    double st[4] = {0, 0, 0, 0};
    PHF_HIP(ctx, hipMemcpyAsync(st, cn->d_stats, sizeof(st), hipMemcpyDeviceToHost, ctx->stream));
    PHF_HIP(ctx, hipStreamSynchronize(ctx->stream));
    cn->n += nsteps;
    if (stats) {
        stats->iterations = (int32_t)st[0];
        stats->converged = st[2] == 0.0;
        stats->rel_residual = st[1];
        stats->saddle_rel_residual = -1.0;
    }
    if (st[2] != 0.0)
        return phf_set_error(ctx, PHF_ENOCONV, "phf_cn_run: %d of %d steps did not reach rtol (worst %.3e)",
                             (int)st[2], nsteps, st[1]);
    return PHF_OK;
}

// ---------------------------------------------------------------------------
// Batched Crank-Nicolson: the steps of many independent steppers of one
// context, each step of each stepper replayed from its captured HIP graphs
// (head with the first CG iteration, iteration chunks, tail), the steppers
// spread over a few streams of their own so that the small launches of
// different problems overlap on the device. Per step: every stepper's head
// and its CG iterations up to its budget go to its stream; the context's
// stream joins them and one kernel gathers every convergence flag for a
// single read-back; a stepper that has not converged gets further pairs of
// iterations (tested after each); then every stepper's tail, joined again.
// Iterations after a stepper's convergence return at once on the device, so
// every stepper does exactly the work of phf_cn_run and its state is
// bit-identical to it. (One graph holding every stepper as a branch was
// measured too: its nodes ran one after another, no faster than stepping
// the problems in turn.)
// ---------------------------------------------------------------------------

struct phf_cn_batch {
    phf_ctx* ctx = nullptr;
    std::vector<phf_cn*> cns;
    std::vector<int32_t> budget;     // CG iterations per step before the flag read-back
    std::vector<hipStream_t> streams;
    std::vector<hipEvent_t> done;    // one per stream
    hipEvent_t fork = nullptr;
    const int** d_flagp = nullptr;   // each stepper's convergence flag word
    int* d_conv = nullptr;           // gathered flags
    int* h_conv = nullptr;           // pinned copy
    bool counted = false;
};

namespace {
constexpr int CNB_STREAMS = 4;

__global__ void k_cnb_gather(int32_t n, const int* const* __restrict__ flagp,
                             int* __restrict__ conv)
{
    for (int32_t i = threadIdx.x; i < n; i += blockDim.x) conv[i] = *flagp[i];
}

// Iteration budget: the head's one plus an even number of chunk iterations,
// at least the stepper's last step count.
int32_t cnb_budget(int32_t predicted) { return 1 + (std::max(predicted, 2) & ~1); }

// Forks the batch streams off the context's stream.
int cnb_fork(phf_cn_batch* b)
{
    phf_ctx* ctx = b->ctx;
    PHF_HIP(ctx, hipEventRecord(b->fork, ctx->stream));
    for (hipStream_t st : b->streams) PHF_HIP(ctx, hipStreamWaitEvent(st, b->fork, 0));
    return PHF_OK;
}

// Joins the batch streams back into the context's stream.
int cnb_join(phf_cn_batch* b)
{
    phf_ctx* ctx = b->ctx;
    for (size_t p = 0; p < b->streams.size(); ++p) {
        PHF_HIP(ctx, hipEventRecord(b->done[p], b->streams[p]));
        PHF_HIP(ctx, hipStreamWaitEvent(ctx->stream, b->done[p], 0));
    }
    return PHF_OK;
}
}  // namespace

extern "C" int phf_cn_batch_destroy(phf_cn_batch* b)
{
    if (!b) return PHF_EINVAL;
    (void)hipStreamSynchronize(b->ctx->stream);
    for (hipStream_t st : b->streams) {
        (void)hipStreamSynchronize(st);
        (void)hipStreamDestroy(st);
    }
    for (hipEvent_t e : b->done) (void)hipEventDestroy(e);
    if (b->fork) (void)hipEventDestroy(b->fork);
    if (b->counted) {
        for (phf_cn* cn : b->cns) cn->n_batches--;
        b->ctx->n_objects--;
    }
    phf_dfree(b->d_flagp);
    phf_dfree(b->d_conv);
    if (b->h_conv) (void)hipHostFree(b->h_conv);
    delete b;
    return PHF_OK;
}

extern "C" int phf_cn_batch_create(phf_cn* const* steppers, int32_t n, phf_cn_batch** out)
{
    if (!steppers || n < 1 || !out || !steppers[0]) return PHF_EINVAL;
    *out = nullptr;
    phf_ctx* ctx = steppers[0]->mesh->ctx;
    for (int32_t i = 0; i < n; ++i) {
        if (!steppers[i] || steppers[i]->mesh->ctx != ctx)
            return phf_set_error(ctx, PHF_EINVAL,
                                 "phf_cn_batch_create: stepper %d is null or of another context", i);
        for (int32_t j = 0; j < i; ++j)
            if (steppers[j] == steppers[i])
                return phf_set_error(ctx, PHF_EINVAL, "phf_cn_batch_create: stepper %d repeated", i);
    }
    phf_cn_batch* b = new (std::nothrow) phf_cn_batch;
    if (!b) return phf_set_error(ctx, PHF_ENOMEM, "host allocation failed");
    b->ctx = ctx;
    b->cns.assign(steppers, steppers + n);
    b->budget.assign(n, 0);
    auto body = [&]() -> int {
        PHF_HIP(ctx, hipSetDevice(ctx->device));
        const int ns = std::min(n, CNB_STREAMS);
        for (int p = 0; p < ns; ++p) {
            hipStream_t st = nullptr;
            PHF_HIP(ctx, hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
            b->streams.push_back(st);
            hipEvent_t e = nullptr;
            PHF_HIP(ctx, hipEventCreateWithFlags(&e, hipEventDisableTiming));
            b->done.push_back(e);
        }
        PHF_HIP(ctx, hipEventCreateWithFlags(&b->fork, hipEventDisableTiming));
        TRY(phf_dmalloc(ctx, &b->d_flagp, (size_t)n, "batch flag pointers"));
        TRY(phf_dmalloc(ctx, &b->d_conv, (size_t)n, "batch flags"));
        PHF_HIP(ctx, hipHostMalloc((void**)&b->h_conv, sizeof(int) * n, hipHostMallocDefault));
        std::vector<const int*> fp(n);
        for (int32_t i = 0; i < n; ++i) fp[i] = b->cns[i]->ns->iflags;
        PHF_HIP(ctx, hipMemcpyAsync(b->d_flagp, fp.data(), sizeof(int*) * n,
                                    hipMemcpyHostToDevice, ctx->stream));
        PHF_HIP(ctx, hipStreamSynchronize(ctx->stream));
        return PHF_OK;
    };
    int rc = body();
    if (rc) {
        phf_cn_batch_destroy(b);
        return rc;
    }
    b->counted = true;
    for (phf_cn* cn : b->cns) cn->n_batches++;
    ctx->n_objects++;
    *out = b;
    return PHF_OK;
}

extern "C" int phf_cn_batch_run(phf_cn_batch* b, const phf_data* data, int32_t nsteps,
                                phf_solve_stats* stats)
{
    if (!b || !data || nsteps < 0) return PHF_EINVAL;
    phf_ctx* ctx = b->ctx;
    const int32_t n = (int32_t)b->cns.size();
    const int32_t P = (int32_t)b->streams.size();
    for (int32_t i = 0; i < n; ++i) {
        phf_cn* cn = b->cns[i];
        const phf_data& d = data[i];
        if (!cn->have_state)
            return phf_set_error(ctx, PHF_ESTATE, "phf_cn_batch_run: stepper %d has no state", i);
        if (!phf_fn_valid(d.f) || !phf_fn_valid(d.g) || !phf_fn_valid(d.uD))
            return phf_set_error(ctx, PHF_EINVAL,
                                 "phf_cn_batch_run: stepper %d: unknown function kind", i);
        if (cn->gx[0] && !(same_fn(cn->gdata.f, d.f) && same_fn(cn->gdata.g, d.g) &&
                           same_fn(cn->gdata.uD, d.uD)))
            cn_drop_graph(cn);
        if (!cn->gx[0]) TRY(cn_capture(cn, &d));
        b->budget[i] = std::max(b->budget[i], cnb_budget(cn->predict));
        // loads at the current time, the device step counter, the statistics
        TRY(cn_loads(cn, &d, cn->F0, cn->bD0, false));
        int64_t n_host = cn->n + 1;  // index of the next step
        PHF_HIP(ctx, hipMemcpyAsync(cn->d_step, &n_host, sizeof(int64_t), hipMemcpyHostToDevice,
                                    ctx->stream));
        PHF_HIP(ctx, hipMemsetAsync(cn->d_stats, 0, 4 * sizeof(double), ctx->stream));
    }
    PHF_HIP(ctx, hipStreamSynchronize(ctx->stream));
    for (int32_t s = 0; s < nsteps; ++s) {
        phf_trace_rec rec;
        phf_trace_begin(ctx, "cn_batch_step", &rec);
        TRY(cnb_fork(b));
        for (int32_t i = 0; i < n; ++i) {
            phf_cn* cn = b->cns[i];
            hipStream_t st = b->streams[i % P];
            PHF_HIP(ctx, hipGraphLaunch(cn->gx[0], st));
            int32_t left = b->budget[i] - 1;  // the head runs the first iteration
            for (int q = phf_cn::NG - 2; q >= 1; --q)
                while (left >= (1 << q)) {
                    PHF_HIP(ctx, hipGraphLaunch(cn->gx[q], st));
                    left -= 1 << q;
                }
        }
        TRY(cnb_join(b));
        hipLaunchKernelGGL(k_cnb_gather, dim3(1), dim3(256), 0, ctx->stream, n,
                           (const int* const*)b->d_flagp, b->d_conv);
        PHF_HIP(ctx, hipGetLastError());
        PHF_HIP(ctx, hipMemcpyAsync(b->h_conv, b->d_conv, sizeof(int) * n, hipMemcpyDeviceToHost,
                                    ctx->stream));
        PHF_HIP(ctx, hipStreamSynchronize(ctx->stream));
        for (int32_t i = 0; i < n; ++i) {
            if (b->h_conv[i]) continue;
            // beyond the budget: pairs of iterations until this stepper
            // converges; it gets a larger budget from the next step on
            phf_cn* cn = b->cns[i];
            int32_t it = b->budget[i];
            int hf[2] = {0, 0};
            while (it < cn->opts.max_iter) {
                PHF_HIP(ctx, hipGraphLaunch(cn->gx[1], ctx->stream));
                it += 2;
                PHF_HIP(ctx, hipMemcpyAsync(hf, cn->ns->iflags, 2 * sizeof(int),
                                            hipMemcpyDeviceToHost, ctx->stream));
                PHF_HIP(ctx, hipStreamSynchronize(ctx->stream));
                if (hf[0]) break;
            }
            b->budget[i] = std::max(b->budget[i], cnb_budget(it));
        }
        TRY(cnb_fork(b));
        for (int32_t i = 0; i < n; ++i)
            PHF_HIP(ctx, hipGraphLaunch(b->cns[i]->gx[phf_cn::NG - 1], b->streams[i % P]));
        TRY(cnb_join(b));
        phf_trace_end(ctx, &rec);
    }
    // statistics and host step counts
    int bad = 0;
    std::vector<double> st(4 * (size_t)n, 0.0);
    for (int32_t i = 0; i < n; ++i)
        PHF_HIP(ctx, hipMemcpyAsync(&st[4 * (size_t)i], b->cns[i]->d_stats, 4 * sizeof(double),
                                    hipMemcpyDeviceToHost, ctx->stream));
    PHF_HIP(ctx, hipStreamSynchronize(ctx->stream));
    for (int32_t i = 0; i < n; ++i) {
        phf_cn* cn = b->cns[i];
        const double* q = &st[4 * (size_t)i];
        cn->n += nsteps;
        if (nsteps > 0) cn->predict = std::max<int32_t>((int32_t)(q[0] / nsteps + 0.5), 1);
        if (stats) {
            stats[i].iterations = (int32_t)q[0];
            stats[i].converged = q[2] == 0.0;
            stats[i].rel_residual = q[1];
            stats[i].saddle_rel_residual = -1.0;
        }
        bad += q[2] != 0.0;
    }
    if (bad)
        return phf_set_error(ctx, PHF_ENOCONV,
                             "phf_cn_batch_run: %d of %d steppers had steps that did not reach "
                             "rtol", bad, n);
    return PHF_OK;
}
