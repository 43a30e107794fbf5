// Request server: continuous batching of elliptic and Crank-Nicolson solves
// on one GPU. Each slot owns a library context (its own HIP stream and
// device memory pool) and a worker thread; waiting requests are admitted in
// arrival order as soon as a slot is free and their estimated device
// footprint fits the memory budget (a smaller request behind one that does
// not fit may go first). Admitted requests run concurrently on their slots'
// streams, so their kernels overlap on the device. Every request runs the
// same kernel sequence whether alone or in a mix, so its result does not
// depend on what else is running.
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "phf_device.h"
#include "phf_internal.h"

namespace {

using clk = std::chrono::steady_clock;

double ms_between(clk::time_point a, clk::time_point b)
{
    return std::chrono::duration<double, std::milli>(b - a).count();
}

// Device bytes per triangle of the finest mesh, including the coarser
// refinement levels, the system, the solver and the multigrid hierarchy
// (measured peaks of the library's pool are below these; on the paper mesh,
// mesh chain included, through the context's allocator: an elliptic request
// (system, multigrid solve) 1,288 / 1,281 / 992 B per triangle at 16,384 /
// 262,144 / 1,048,576 triangles, a Crank-Nicolson stepper 1,735 / 1,556 at
// the first two; the pool's size rounding weighs more on small meshes).
constexpr double BYTES_PER_ELEM_ELLIPTIC = 1400.0;
constexpr double BYTES_PER_ELEM_CN = 1800.0;

// Crank-Nicolson initial state: per element, the P1 values whose edge
// midpoint values are u0 at the midpoints (vertex i gets u0(m_j) + u0(m_k) -
// u0(m_i), m_i the midpoint of the edge opposite vertex i).
__global__ __launch_bounds__(256) void k_cr_interpolant(int32_t nE, const double2* __restrict__ exy,
                                                        phf_fn_dev u0, double t, double* __restrict__ U)
{
    const int32_t m = blockIdx.x * 256 + threadIdx.x;
    if (m >= nE) return;
    const double2 P0 = exy[3 * (int64_t)m], P1 = exy[3 * (int64_t)m + 1], P2 = exy[3 * (int64_t)m + 2];
    const double v0 = phf_fn_eval(u0, 0.5 * (P1.x + P2.x), 0.5 * (P1.y + P2.y), t, 0, 0, -1);
    const double v1 = phf_fn_eval(u0, 0.5 * (P2.x + P0.x), 0.5 * (P2.y + P0.y), t, 0, 0, -1);
    const double v2 = phf_fn_eval(u0, 0.5 * (P0.x + P1.x), 0.5 * (P0.y + P1.y), t, 0, 0, -1);
    U[3 * (int64_t)m] = v1 + v2 - v0;
    U[3 * (int64_t)m + 1] = v2 + v0 - v1;
    U[3 * (int64_t)m + 2] = v0 + v1 - v2;
}

struct job {
    int64_t id = 0;
    phf_request req{};
    std::vector<double> xy;
    std::vector<int32_t> elem, dir, neu;
    int64_t nE_final = 0;
    double bytes = 0;
    clk::time_point t_submit, t_start, t_done;
    phf_result res{};
    bool done = false;
};

}  // namespace

struct phf_server {
    int device = 0;
    int32_t slots = 1;
    double budget = 0;   // bytes
    double reserved = 0; // estimated bytes of running requests
    double peak_reserved = 0;
    int32_t running = 0, peak_running = 0;
    int64_t next_id = 1, completed = 0;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<job*> queue;
    std::unordered_map<int64_t, job*> jobs;
    std::vector<std::thread> workers;
    std::vector<phf_ctx*> ctxs;
    std::vector<hipStream_t> streams;
    bool stop = false;
};

namespace {

#define TRY(x)               \
    do {                     \
        int rc_ = (x);       \
        if (rc_) return rc_; \
    } while (0)

// Runs one request on a slot's context; fills j->res.
int run_job(phf_ctx* ctx, job* j)
{
    const phf_request& r = j->req;
    std::vector<phf_mesh*> chain;
    double *K = nullptr, *M = nullptr, *C = nullptr, *F = nullptr, *bD = nullptr, *U = nullptr;
    phf_cn* cn = nullptr;
    auto body = [&]() -> int {
        phf_mesh* m = nullptr;
        TRY(phf_mesh_create(ctx, j->xy.data(), r.nC, j->elem.data(), r.nE,
                            j->dir.empty() ? nullptr : j->dir.data(), r.nD,
                            j->neu.empty() ? nullptr : j->neu.data(), r.nN, PHF_HOST, &m));
        chain.push_back(m);
        for (int32_t q = 0; q < r.refine; ++q) {
            TRY(phf_mesh_refine(chain.back(), &m));
            chain.push_back(m);
        }
        m = chain.back();
        const int32_t N = 3 * m->nE;
        j->res.nE = m->nE;
        const int32_t pc = r.refine > 0 ? PHF_PRECOND_MULTIGRID : PHF_PRECOND_JACOBI;
        TRY(phf_dmalloc(ctx, &U, (size_t)N, "request U"));
        double t_final = r.data.t;
        if (r.kind == PHF_REQ_ELLIPTIC) {
            const size_t n9 = 9 * (size_t)m->nE;
            TRY(phf_dmalloc(ctx, &K, n9, "request K"));
            TRY(phf_dmalloc(ctx, &M, n9, "request M"));
            TRY(phf_dmalloc(ctx, &C, (size_t)m->nnz_C, "request C"));
            TRY(phf_dmalloc(ctx, &F, (size_t)N, "request F"));
            TRY(phf_dmalloc(ctx, &bD, (size_t)m->L, "request bD"));
            phf_system s{};
            s.K = K;
            s.M = M;
            s.C = C;
            s.F = F;
            s.bD = bD;
            TRY(phf_assemble_impl(m, &r.coeffs, &r.data, &s));
            phf_solver_opts o{};
            o.method = PHF_SOLVER_NULLSPACE_CG;
            o.rtol = r.rtol;
            o.precond = pc;
            phf_solve_stats st{};
            TRY(phf_solve(m, &r.coeffs, &s, &o, U, nullptr, &st));
            j->res.iterations = st.iterations;
            j->res.rel_residual = st.rel_residual;
        } else {
            phf_cn_opts o{};
            o.rtol = r.rtol;
            o.precond = pc;
            TRY(phf_cn_create(m, &r.coeffs, r.k, &o, &cn));
            double* L0 = nullptr;
            TRY(phf_dmalloc(ctx, &L0, (size_t)std::max(m->L, 1), "request Lambda0"));
            PHF_HIP(ctx, hipMemsetAsync(L0, 0, sizeof(double) * std::max(m->L, 1), ctx->stream));
            PHF_LAUNCH(ctx, "k_cr_interpolant", k_cr_interpolant, (m->nE + 255) / 256, 256, 0,
                       m->nE, m->exy, phf_fn_to_dev(r.u0), r.data.t, U);
            int rc = phf_cn_set_state(cn, U, L0, r.data.t);
            phf_dfree(L0);
            TRY(rc);
            phf_solve_stats st{};
            TRY(phf_cn_run(cn, &r.data, r.steps, 1, &st));
            TRY(phf_cn_get_state(cn, U, nullptr, &t_final));
            j->res.iterations = st.iterations;
            j->res.rel_residual = st.rel_residual;
        }
        j->res.h1 = j->res.l2 = -1.0;
        if (r.exact.kind != PHF_FN_ZERO || r.want_norms)
            TRY(phf_error_norms(m, U, &r.exact, t_final, &j->res.h1, &j->res.l2));
        if (r.U_out) {
            PHF_HIP(ctx, hipMemcpyAsync(r.U_out, U, sizeof(double) * N, hipMemcpyDeviceToHost,
                                        ctx->stream));
        }
        PHF_HIP(ctx, hipStreamSynchronize(ctx->stream));
        return PHF_OK;
    };
    int rc = body();
    (void)hipStreamSynchronize(ctx->stream);
    if (cn) phf_cn_destroy(cn);
    for (double* p : {K, M, C, F, bD, U}) {
        double* q = p;
        phf_dfree(q);
    }
    for (auto it = chain.rbegin(); it != chain.rend(); ++it) phf_mesh_destroy(*it);
    return rc;
}

void worker(phf_server* s, int slot)
{
    (void)hipSetDevice(s->device);
    phf_ctx* ctx = s->ctxs[slot];
    for (;;) {
        job* j = nullptr;
        {
            std::unique_lock<std::mutex> lk(s->mu);
            for (;;) {
                if (s->stop && s->queue.empty()) return;
                // first request in arrival order whose footprint fits
                for (auto it = s->queue.begin(); it != s->queue.end(); ++it) {
                    if (s->reserved + (*it)->bytes <= s->budget || s->running == 0) {
                        j = *it;
                        s->queue.erase(it);
                        break;
                    }
                }
                if (j) break;
                s->cv_work.wait(lk);
            }
            s->reserved += j->bytes;
            s->peak_reserved = std::max(s->peak_reserved, s->reserved);
            ++s->running;
            s->peak_running = std::max(s->peak_running, s->running);
            j->t_start = clk::now();
        }
        const int rc = run_job(ctx, j);
        {
            std::lock_guard<std::mutex> lk(s->mu);
            j->t_done = clk::now();
            j->res.status = rc;
            j->res.slot = slot;
            j->res.queue_ms = ms_between(j->t_submit, j->t_start);
            j->res.run_ms = ms_between(j->t_start, j->t_done);
            j->res.latency_ms = ms_between(j->t_submit, j->t_done);
            j->done = true;
            s->reserved -= j->bytes;
            --s->running;
            ++s->completed;
        }
        s->cv_done.notify_all();
        s->cv_work.notify_all();
    }
}

void server_stop(phf_server* s)
{
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->cv_work.notify_all();
    for (auto& t : s->workers)
        if (t.joinable()) t.join();
    for (phf_ctx* c : s->ctxs)
        if (c) phf_destroy(c);
    for (hipStream_t st : s->streams)
        if (st) (void)hipStreamDestroy(st);
    // the workers drained the queue before returning; every job not yet
    // collected by phf_server_wait is in the map
    for (auto& kv : s->jobs) delete kv.second;
    s->jobs.clear();
}

}  // namespace

extern "C" int phf_server_create(int device, const phf_server_opts* opts, phf_server** out)
{
    if (!out) return PHF_EINVAL;
    *out = nullptr;
    const int32_t slots = opts && opts->slots > 0 ? opts->slots : 4;
    if (slots > 16) return PHF_EINVAL;
    if (hipSetDevice(device) != hipSuccess) {
        (void)hipGetLastError();
        return PHF_EINVAL;
    }
    phf_server* s = new (std::nothrow) phf_server;
    if (!s) return PHF_ENOMEM;
    s->device = device;
    s->slots = slots;
    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) {
        (void)hipGetLastError();
        free_b = 0;
    }
    s->budget = opts && opts->memory_bytes > 0 ? (double)opts->memory_bytes : 0.5 * (double)free_b;
    for (int32_t q = 0; q < slots; ++q) {
        hipStream_t st = nullptr;
        phf_ctx* c = nullptr;
        if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess ||
            phf_create(&c, device, st, nullptr) != PHF_OK) {
            (void)hipGetLastError();
            if (st) (void)hipStreamDestroy(st);
            server_stop(s);
            delete s;
            return PHF_EHIP;
        }
        s->streams.push_back(st);
        s->ctxs.push_back(c);
    }
    for (int32_t q = 0; q < slots; ++q) s->workers.emplace_back(worker, s, q);
    *out = s;
    return PHF_OK;
}

extern "C" int phf_server_destroy(phf_server* s)
{
    if (!s) return PHF_EINVAL;
    server_stop(s);
    delete s;
    return PHF_OK;
}

extern "C" int phf_server_submit(phf_server* s, const phf_request* r, int64_t* id)
{
    if (!s || !r || !id) return PHF_EINVAL;
    if ((r->kind != PHF_REQ_ELLIPTIC && r->kind != PHF_REQ_CN) || !r->xy || !r->elem ||
        r->nC < 3 || r->nE < 1 || r->nD < 0 || r->nN < 0 || (r->nD > 0 && !r->dir) ||
        (r->nN > 0 && !r->neu) || r->refine < 0 || r->refine > 12 || r->coeffs.a_T ||
        (r->kind == PHF_REQ_CN && (r->k <= 0 || r->steps < 1)))
        return PHF_EINVAL;
    const phf_fn* fns[] = {&r->data.f, &r->data.g, &r->data.uD, &r->u0, &r->exact};
    for (const phf_fn* f : fns)
        if (f->kind == PHF_FN_EDGE_ARRAY || !phf_fn_valid(*f)) return PHF_EINVAL;
    job* j = new (std::nothrow) job;
    if (!j) return PHF_ENOMEM;
    j->req = *r;
    j->xy.assign(r->xy, r->xy + 2 * (size_t)r->nC);
    j->elem.assign(r->elem, r->elem + 3 * (size_t)r->nE);
    if (r->nD) j->dir.assign(r->dir, r->dir + 2 * (size_t)r->nD);
    if (r->nN) j->neu.assign(r->neu, r->neu + 2 * (size_t)r->nN);
    j->nE_final = (int64_t)r->nE << (2 * r->refine);
    j->bytes = (double)j->nE_final *
               (r->kind == PHF_REQ_CN ? BYTES_PER_ELEM_CN : BYTES_PER_ELEM_ELLIPTIC);
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->stop) {
            delete j;
            return PHF_ESTATE;
        }
        j->id = s->next_id++;
        j->t_submit = clk::now();
        s->jobs[j->id] = j;
        s->queue.push_back(j);
        *id = j->id;
    }
    s->cv_work.notify_all();
    return PHF_OK;
}

extern "C" int phf_server_wait(phf_server* s, int64_t id, double timeout_ms, phf_result* res)
{
    if (!s || !res) return PHF_EINVAL;
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->jobs.find(id);
    if (it == s->jobs.end()) return PHF_EINVAL;
    job* j = it->second;
    auto ready = [&] { return j->done; };
    if (timeout_ms < 0) {
        s->cv_done.wait(lk, ready);
    } else if (!s->cv_done.wait_for(lk, std::chrono::duration<double, std::milli>(timeout_ms),
                                    ready)) {
        return PHF_ETIMEDOUT;
    }
    *res = j->res;
    s->jobs.erase(it);
    delete j;
    return PHF_OK;
}

extern "C" int phf_server_query(phf_server* s, phf_server_stats* st)
{
    if (!s || !st) return PHF_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    st->slots = s->slots;
    st->running = s->running;
    st->peak_running = s->peak_running;
    st->queued = (int32_t)s->queue.size();
    st->completed = s->completed;
    st->budget_bytes = s->budget;
    st->reserved_bytes = s->reserved;
    st->peak_reserved_bytes = s->peak_reserved;
    return PHF_OK;
}
