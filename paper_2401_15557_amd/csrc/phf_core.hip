// Context, error reporting, kernel tracing, integer scan, SpMV and dot
// products of libphfem.
#include <cstdarg>
#include <cstring>
#include <map>
#include <mutex>
#include <unordered_map>

#include "phf_internal.h"
#include "phf_device.h"

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------

int phf_set_error(phf_ctx* ctx, int code, const char* fmt, ...)
{
    if (ctx) {
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(ctx->last_error, sizeof(ctx->last_error), fmt, ap);
        va_end(ap);
    }
    return code;
}

extern "C" const char* phf_status_str(int code)
{
    switch (code) {
    case PHF_OK: return "ok";
    case PHF_EINVAL: return "invalid argument";
    case PHF_EORIENT: return "element not counter-clockwise or degenerate";
    case PHF_EMESH: return "non-manifold or inconsistently oriented mesh";
    case PHF_EBOUNDARY: return "boundary lists inconsistent with the mesh";
    case PHF_ENOMEM: return "out of memory";
    case PHF_ENOCONV: return "solver did not converge";
    case PHF_EHIP: return "HIP runtime error";
    case PHF_ESTATE: return "call out of order";
    case PHF_ETIMEDOUT: return "timed out";
    default: return "unknown status";
    }
}

extern "C" const char* phf_last_error(const phf_ctx* ctx)
{
    return ctx ? ctx->last_error : "null context";
}

extern "C" const char* phf_version(void) { return "0.1.0"; }

// ---------------------------------------------------------------------------
// caching device allocator
// ---------------------------------------------------------------------------

struct phf_pool {
    std::multimap<size_t, void*> free_blocks;  // rounded size -> block
    int64_t live_bytes = 0, cached_bytes = 0;
    phf_allocator al{};                        // the context's allocator (alloc null: HIP)
};

namespace {
std::mutex g_pool_mu;

// Where a block came from, so that it goes back there even after its
// context is gone: the owning pool (null once that context is destroyed),
// the rounded size and the allocator.
struct block_rec {
    phf_pool* pool;
    size_t size;
    phf_allocator al;
};
std::unordered_map<void*, block_rec> g_blocks;

size_t round_block(size_t bytes)
{
    const size_t small = 512, large = size_t(2) << 20;
    return bytes <= (size_t(1) << 20) ? (bytes + small - 1) / small * small
                                      : (bytes + large - 1) / large * large;
}

void* raw_alloc(const phf_allocator& al, size_t bytes)
{
    if (al.alloc) return al.alloc(bytes, al.user);
    void* p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    return p;
}

void raw_free(const phf_allocator& al, void* p)
{
    if (al.alloc) {
        if (al.free) al.free(p, al.user);
        return;
    }
    (void)hipFree(p);
}

// Frees every cached block of the pool (caller holds the lock).
void pool_trim(phf_pool* pl)
{
    for (auto& kv : pl->free_blocks) {
        g_blocks.erase(kv.second);
        raw_free(pl->al, kv.second);
    }
    pl->free_blocks.clear();
    pl->cached_bytes = 0;
}
}  // namespace

int phf_dmalloc_bytes(phf_ctx* ctx, void** p, size_t bytes, const char* what)
{
    *p = nullptr;
    const size_t sz = round_block(bytes);
    std::lock_guard<std::mutex> lk(g_pool_mu);
    phf_pool* pl = ctx->pool;
    // best fit among cached blocks, at most 1/8 larger than asked for
    auto it = pl->free_blocks.lower_bound(sz);
    if (it != pl->free_blocks.end() && it->first <= sz + sz / 8) {
        *p = it->second;
        pl->cached_bytes -= (int64_t)it->first;
        pl->live_bytes += (int64_t)it->first;
        pl->free_blocks.erase(it);
        return PHF_OK;
    }
    *p = raw_alloc(pl->al, sz);
    if (!*p) {
        pool_trim(pl);
        *p = raw_alloc(pl->al, sz);
    }
    if (!*p)
        return phf_set_error(ctx, PHF_ENOMEM, "device allocation of %s (%zu bytes) failed", what,
                             bytes);
    g_blocks[*p] = block_rec{pl, sz, pl->al};
    pl->live_bytes += (int64_t)sz;
    return PHF_OK;
}

void phf_dfree_ptr(void* p)
{
    std::lock_guard<std::mutex> lk(g_pool_mu);
    auto it = g_blocks.find(p);
    if (it == g_blocks.end()) {
        (void)hipFree(p);
        return;
    }
    phf_pool* pl = it->second.pool;
    const size_t sz = it->second.size;
    if (!pl) {
        const phf_allocator al = it->second.al;
        g_blocks.erase(it);
        raw_free(al, p);
        return;
    }
    pl->live_bytes -= (int64_t)sz;
    pl->cached_bytes += (int64_t)sz;
    pl->free_blocks.emplace(sz, p);
}

extern "C" int phf_mem_stats(phf_ctx* ctx, int64_t* live_bytes, int64_t* cached_bytes)
{
    if (!ctx) return PHF_EINVAL;
    std::lock_guard<std::mutex> lk(g_pool_mu);
    if (live_bytes) *live_bytes = ctx->pool->live_bytes;
    if (cached_bytes) *cached_bytes = ctx->pool->cached_bytes;
    return PHF_OK;
}

extern "C" int phf_release_cache(phf_ctx* ctx)
{
    if (!ctx) return PHF_EINVAL;
    PHF_HIP(ctx, hipStreamSynchronize(ctx->stream));
    std::lock_guard<std::mutex> lk(g_pool_mu);
    pool_trim(ctx->pool);
    return PHF_OK;
}

// ---------------------------------------------------------------------------
// context
// ---------------------------------------------------------------------------

extern "C" int phf_create(phf_ctx** out, int device, void* hip_stream, const phf_allocator* alloc)
{
    if (!out) return PHF_EINVAL;
    *out = nullptr;
    if (alloc && (!alloc->alloc || !alloc->free)) return PHF_EINVAL;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) {
        (void)hipGetLastError();
        return PHF_EINVAL;
    }
    phf_ctx* ctx = new (std::nothrow) phf_ctx;
    if (!ctx) return PHF_ENOMEM;
    ctx->device = device;
    ctx->stream = (hipStream_t)hip_stream;
    ctx->pool = new (std::nothrow) phf_pool;
    if (!ctx->pool) {
        delete ctx;
        return PHF_ENOMEM;
    }
    if (alloc) ctx->pool->al = *alloc;
    if (hipSetDevice(device) != hipSuccess) {
        delete ctx->pool;
        delete ctx;
        return PHF_EHIP;
    }
    if (phf_dmalloc(ctx, &ctx->d_flags, 64, "context flags") != PHF_OK ||
        hipHostMalloc((void**)&ctx->h_pinned, 64 * sizeof(int64_t), hipHostMallocDefault) !=
            hipSuccess) {
        (void)hipGetLastError();
        phf_dfree(ctx->d_flags);
        {
            std::lock_guard<std::mutex> lk(g_pool_mu);
            pool_trim(ctx->pool);
        }
        delete ctx->pool;
        delete ctx;
        return PHF_ENOMEM;
    }
    *out = ctx;
    return PHF_OK;
}

extern "C" int phf_destroy(phf_ctx* ctx)
{
    if (!ctx) return PHF_EINVAL;
    if (ctx->n_objects > 0)
        return phf_set_error(ctx, PHF_ESTATE,
                             "phf_destroy: %lld meshes, steppers or batches of this context are "
                             "still alive",
                             (long long)ctx->n_objects);
    (void)hipSetDevice(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
    for (auto& r : ctx->pending) {
        ctx->event_pool.push_back(r.start);
        ctx->event_pool.push_back(r.stop);
    }
    for (auto e : ctx->event_pool) (void)hipEventDestroy(e);
    phf_dfree(ctx->d_flags);
    if (ctx->h_pinned) (void)hipHostFree(ctx->h_pinned);
    {
        std::lock_guard<std::mutex> lk(g_pool_mu);
        pool_trim(ctx->pool);
        // blocks still held by objects of this context go back to the
        // allocator directly when those objects are destroyed
        for (auto& kv : g_blocks)
            if (kv.second.pool == ctx->pool) kv.second.pool = nullptr;
        delete ctx->pool;
    }
    delete ctx;
    return PHF_OK;
}

extern "C" int phf_set_stream(phf_ctx* ctx, void* hip_stream)
{
    if (!ctx) return PHF_EINVAL;
    // cached blocks were last used in the order of the old stream
    if (hip_stream != (void*)ctx->stream) PHF_HIP(ctx, hipStreamSynchronize(ctx->stream));
    ctx->stream = (hipStream_t)hip_stream;
    return PHF_OK;
}

extern "C" int phf_synchronize(phf_ctx* ctx)
{
    if (!ctx) return PHF_EINVAL;
    PHF_HIP(ctx, hipStreamSynchronize(ctx->stream));
    return PHF_OK;
}

// ---------------------------------------------------------------------------
// tracing
// ---------------------------------------------------------------------------

static hipEvent_t take_event(phf_ctx* ctx)
{
    if (!ctx->event_pool.empty()) {
        hipEvent_t e = ctx->event_pool.back();
        ctx->event_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    return e;
}

void phf_trace_begin(phf_ctx* ctx, const char* name, phf_trace_rec* rec, bool marker)
{
    rec->name = name;
    rec->start = rec->stop = nullptr;
    rec->marker = marker;
    if (!ctx->trace) return;
    if (!ctx->trace_only.empty() && ctx->trace_only != name) return;
    rec->start = take_event(ctx);
    rec->stop = take_event(ctx);
    if (!rec->start || !rec->stop) {
        if (rec->start) ctx->event_pool.push_back(rec->start);
        if (rec->stop) ctx->event_pool.push_back(rec->stop);
        rec->start = rec->stop = nullptr;
        return;
    }
    if (marker) (void)hipEventRecord(rec->start, ctx->stream);
}

static int trace_collect(phf_ctx* ctx);

void phf_trace_end(phf_ctx* ctx, phf_trace_rec* rec)
{
    if (!ctx->trace || !rec->start || !rec->stop) return;
    if (rec->marker) (void)hipEventRecord(rec->stop, ctx->stream);
    ctx->pending.push_back(*rec);
    // bound the number of events in flight; reading them waits for the stream
    if (ctx->pending.size() >= 16384) (void)trace_collect(ctx);
}

static int trace_collect(phf_ctx* ctx)
{
    if (ctx->pending.empty()) return PHF_OK;
    PHF_HIP(ctx, hipEventSynchronize(ctx->pending.back().stop));
    for (auto& r : ctx->pending) {
        float ms = 0.f;
        PHF_HIP(ctx, hipEventElapsedTime(&ms, r.start, r.stop));
        bool found = false;
        for (auto& t : ctx->totals) {
            if (t.first == r.name) {
                t.second.first += 1;
                t.second.second += ms;
                found = true;
                break;
            }
        }
        if (!found) ctx->totals.push_back({std::string(r.name), {1, (double)ms}});
        found = false;
        for (auto& t : ctx->samples) {
            if (t.first == r.name) {
                t.second.push_back(ms);
                found = true;
                break;
            }
        }
        if (!found) ctx->samples.push_back({std::string(r.name), std::vector<float>(1, ms)});
        ctx->event_pool.push_back(r.start);
        ctx->event_pool.push_back(r.stop);
    }
    ctx->pending.clear();
    return PHF_OK;
}

extern "C" int phf_trace_enable(phf_ctx* ctx, int on)
{
    if (!ctx) return PHF_EINVAL;
    ctx->trace = on != 0;
    // create the events up front so that tracing adds no creation cost later
    while (ctx->trace && ctx->event_pool.size() + 2 * ctx->pending.size() < 2 * 16384 + 64) {
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) {
            (void)hipGetLastError();
            break;
        }
        ctx->event_pool.push_back(e);
    }
    return PHF_OK;
}

extern "C" int phf_trace_filter(phf_ctx* ctx, const char* kernel)
{
    if (!ctx) return PHF_EINVAL;
    ctx->trace_only = kernel ? kernel : "";
    return PHF_OK;
}

extern "C" int phf_trace_reset(phf_ctx* ctx)
{
    if (!ctx) return PHF_EINVAL;
    int rc = trace_collect(ctx);
    ctx->totals.clear();
    ctx->samples.clear();
    return rc;
}

extern "C" int phf_trace_samples(phf_ctx* ctx, const char* kernel, float* ms, int64_t cap,
                                 int64_t* count)
{
    if (!ctx || !kernel || cap < 0 || (cap > 0 && !ms)) return PHF_EINVAL;
    int rc = trace_collect(ctx);
    if (rc) return rc;
    int64_t n = 0;
    for (auto& t : ctx->samples) {
        if (t.first != kernel) continue;
        n = (int64_t)t.second.size();
        for (int64_t i = 0; i < n && i < cap; ++i) ms[i] = t.second[i];
    }
    if (count) *count = n;
    return PHF_OK;
}

extern "C" int phf_trace_query(phf_ctx* ctx, const char* kernel, int64_t* count, double* total_ms)
{
    if (!ctx) return PHF_EINVAL;
    int rc = trace_collect(ctx);
    if (rc) return rc;
    int64_t c = 0;
    double ms = 0;
    for (auto& t : ctx->totals) {
        if (!kernel || t.first == kernel) {
            c += t.second.first;
            ms += t.second.second;
        }
    }
    if (count) *count = c;
    if (total_ms) *total_ms = ms;
    return PHF_OK;
}

extern "C" int phf_trace_dump(phf_ctx* ctx, char* buf, size_t len)
{
    if (!ctx || (!buf && len)) return PHF_EINVAL;
    int rc = trace_collect(ctx);
    if (rc) return rc;
    std::string s;
    char line[256];
    for (auto& t : ctx->totals) {
        snprintf(line, sizeof(line), "%s %lld %.6f\n", t.first.c_str(),
                 (long long)t.second.first, t.second.second);
        s += line;
    }
    if (len) {
        size_t n = s.size() < len - 1 ? s.size() : len - 1;
        memcpy(buf, s.data(), n);
        buf[n] = 0;
    }
    return (int)ctx->totals.size();
}

// ---------------------------------------------------------------------------
// exclusive scan of int32 (three passes: block sums, scan of sums, block scan)
// ---------------------------------------------------------------------------

namespace {
constexpr int SCAN_THREADS = 256;
constexpr int SCAN_ITEMS = 8;
constexpr int SCAN_TILE = SCAN_THREADS * SCAN_ITEMS;

__global__ __launch_bounds__(SCAN_THREADS) void k_scan_reduce(const int32_t* __restrict__ in,
                                                              int32_t n, int32_t* bsum)
{
    __shared__ int32_t sh[SCAN_THREADS / 64];
    int64_t base = (int64_t)blockIdx.x * SCAN_TILE;
    int32_t s = 0;
    for (int k = 0; k < SCAN_ITEMS; ++k) {
        int64_t q = base + (int64_t)k * SCAN_THREADS + threadIdx.x;
        if (q < n) s += in[q];
    }
    int32_t tot = phf_block_sum_i32<SCAN_THREADS>(s, sh);
    if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

__global__ __launch_bounds__(SCAN_THREADS) void k_scan_sums(int32_t* bsum, int32_t nb,
                                                            int32_t* d_total)
{
    __shared__ int32_t sh[SCAN_THREADS / 64 + 1];
    int32_t carry = 0;
    for (int32_t base = 0; base < nb; base += SCAN_THREADS) {
        int32_t q = base + threadIdx.x;
        int32_t v = q < nb ? bsum[q] : 0;
        int32_t tot;
        int32_t ex = phf_block_exscan_i32<SCAN_THREADS>(v, sh, &tot);
        if (q < nb) bsum[q] = carry + ex;
        carry += tot;
        __syncthreads();
    }
    if (threadIdx.x == 0 && d_total) *d_total = carry;
}

__global__ __launch_bounds__(SCAN_THREADS) void k_scan_apply(const int32_t* in, int32_t* out,
                                                             int32_t n, const int32_t* bsum)
{
    __shared__ int32_t sh[SCAN_THREADS / 64 + 1];
    int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_ITEMS;
    int32_t v[SCAN_ITEMS];
    int32_t s = 0;
    for (int k = 0; k < SCAN_ITEMS; ++k) {
        int64_t q = base + k;
        v[k] = q < n ? in[q] : 0;
        s += v[k];
    }
    int32_t tot;
    int32_t ex = phf_block_exscan_i32<SCAN_THREADS>(s, sh, &tot) + bsum[blockIdx.x];
    for (int k = 0; k < SCAN_ITEMS; ++k) {
        int64_t q = base + k;
        if (q < n) out[q] = ex;
        ex += v[k];
    }
}
// Whole scan in one workgroup, for n <= SCAN_TILE.
__global__ __launch_bounds__(SCAN_THREADS) void k_scan_single(const int32_t* in, int32_t* out,
                                                              int32_t n, int32_t* d_total)
{
    __shared__ int32_t sh[SCAN_THREADS / 64 + 1];
    const int32_t base = threadIdx.x * SCAN_ITEMS;
    int32_t v[SCAN_ITEMS];
    int32_t s = 0;
    for (int k = 0; k < SCAN_ITEMS; ++k) {
        v[k] = base + k < n ? in[base + k] : 0;
        s += v[k];
    }
    int32_t tot;
    int32_t ex = phf_block_exscan_i32<SCAN_THREADS>(s, sh, &tot);
    for (int k = 0; k < SCAN_ITEMS; ++k) {
        if (base + k < n) out[base + k] = ex;
        ex += v[k];
    }
    if (threadIdx.x == 0 && d_total) *d_total = tot;
}
}  // namespace

int phf_scan_i32(phf_ctx* ctx, const int32_t* in, int32_t* out, int32_t n, int32_t* d_total)
{
    if (n <= 0) {
        if (d_total) PHF_HIP(ctx, hipMemsetAsync(d_total, 0, sizeof(int32_t), ctx->stream));
        return PHF_OK;
    }
    int32_t nb = (n + SCAN_TILE - 1) / SCAN_TILE;
    if (nb == 1) {
        PHF_LAUNCH(ctx, "k_scan", k_scan_single, 1, SCAN_THREADS, 0, in, out, n, d_total);
        return PHF_OK;
    }
    int32_t* bsum = nullptr;
    int rc = phf_dmalloc(ctx, &bsum, nb, "scan block sums");
    if (rc) return rc;
    phf_trace_rec rec;
    phf_trace_begin(ctx, "k_scan", &rec);
    hipLaunchKernelGGL(k_scan_reduce, dim3(nb), dim3(SCAN_THREADS), 0, ctx->stream, in, n, bsum);
    hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(SCAN_THREADS), 0, ctx->stream, bsum, nb,
                       d_total);
    hipLaunchKernelGGL(k_scan_apply, dim3(nb), dim3(SCAN_THREADS), 0, ctx->stream, in, out, n,
                       bsum);
    phf_trace_end(ctx, &rec);
    hipError_t e = hipGetLastError();
    // back to the pool: later users of the block run after these kernels
    phf_dfree(bsum);
    if (e != hipSuccess)
        return phf_set_error(ctx, PHF_EHIP, "scan launch failed: %s", hipGetErrorString(e));
    return PHF_OK;
}

// ---------------------------------------------------------------------------
// problem-data function validation
// ---------------------------------------------------------------------------

bool phf_fn_valid(const phf_fn& f)
{
    switch (f.kind) {
    case PHF_FN_ZERO:
    case PHF_FN_CONST:
    case PHF_FN_SIN_COS:
    case PHF_FN_SIN_SIN:
    case PHF_FN_GRAD_SIN_COS:
    case PHF_FN_GRAD_SIN_SIN:
    case PHF_FN_PAPER_U:
    case PHF_FN_PAPER_F:
    case PHF_FN_PAPER_FLUX: return true;
    case PHF_FN_EDGE_ARRAY: return f.edge_values != nullptr;
    default: return false;
    }
}

bool phf_fn_needs_edge(const phf_fn& f) { return f.kind == PHF_FN_EDGE_ARRAY; }

// ---------------------------------------------------------------------------
// CSR SpMV and deterministic dot products
// ---------------------------------------------------------------------------

namespace {
__global__ __launch_bounds__(256) void k_spmv(int32_t nrows, const int32_t* __restrict__ rowptr,
                                              const int32_t* __restrict__ col,
                                              const double* __restrict__ val, double alpha,
                                              const double* __restrict__ x, double beta,
                                              double* __restrict__ y)
{
    int32_t r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nrows) return;
    double s = 0.0;
    for (int32_t q = rowptr[r]; q < rowptr[r + 1]; ++q) s = fma(val[q], x[col[q]], s);
    y[r] = beta == 0.0 ? alpha * s : fma(alpha, s, beta * y[r]);
}
}  // namespace

extern "C" int phf_spmv(phf_ctx* ctx, int32_t nrows, const int32_t* rowptr, const int32_t* col,
                        const double* val, double alpha, const double* x, double beta, double* y)
{
    if (!ctx || nrows < 0 || (nrows > 0 && (!rowptr || !col || !val || !x || !y)))
        return PHF_EINVAL;
    if (nrows == 0) return PHF_OK;
    PHF_LAUNCH(ctx, "k_spmv", k_spmv, (nrows + 255) / 256, 256, 0, nrows, rowptr, col, val, alpha,
               x, beta, y);
    return PHF_OK;
}

namespace {
constexpr int DOT_BLOCKS = 512;
__global__ __launch_bounds__(256) void k_dot_partial(const double* __restrict__ x,
                                                     const double* __restrict__ y, int32_t n,
                                                     double* partials)
{
    __shared__ double sh[4];
    double s = 0.0;
    for (int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x; q < n;
         q += (int64_t)gridDim.x * 256)
        s = fma(x[q], y[q], s);
    double t = phf_block_sum_f64<256>(s, sh);
    if (threadIdx.x == 0) partials[blockIdx.x] = t;
}

__global__ __launch_bounds__(256) void k_dot_final(const double* partials, int32_t np,
                                                   double* out)
{
    __shared__ double sh[4];
    double s = 0.0;
    for (int q = threadIdx.x; q < np; q += 256) s += partials[q];
    double t = phf_block_sum_f64<256>(s, sh);
    if (threadIdx.x == 0) *out = t;
}
}  // namespace

int phf_dot(phf_ctx* ctx, const double* x, const double* y, int32_t n, double* d_partials,
            double* d_out)
{
    PHF_LAUNCH(ctx, "k_dot_partial", k_dot_partial, DOT_BLOCKS, 256, 0, x, y, n, d_partials);
    PHF_LAUNCH(ctx, "k_dot_final", k_dot_final, 1, 256, 0, d_partials, DOT_BLOCKS, d_out);
    return PHF_OK;
}
