// Broken H^1 seminorm and L^2 norm of u - U_h on the device (the error
// columns of Section 3.7's tables), for a discontinuous piecewise-linear U_h.
#include <cmath>
#include <mutex>

#include "phf_device.h"

namespace {

constexpr int NT = 256;
constexpr int MAXB = 1024;
constexpr int NG = 5;  // Gauss-Legendre points per direction

struct quad_rule {
    double x[NG * NG], y[NG * NG], w[NG * NG];  // reference triangle, weights sum to 1/2
};

// Gauss-Legendre nodes and weights on [0, 1]: Newton's method on the
// Legendre polynomial P_n from the Chebyshev-like starting guesses, with the
// three-term recurrence for P_n and its derivative.
void gauss_legendre01(int n, double* x, double* w)
{
    for (int i = 0; i < n; ++i) {
        double z = std::cos(M_PI * (i + 0.75) / (n + 0.5));
        double dp = 1.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= n; ++k) {
                const double pk = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = pk;
            }
            dp = n * (z * p1 - p0) / (z * z - 1.0);
            const double dz = p1 / dp;
            z -= dz;
            if (std::fabs(dz) < 1e-16) break;
        }
        x[i] = 0.5 * (1.0 - z);
        w[i] = 1.0 / ((1.0 - z * z) * dp * dp);  // = 2/((1-z^2)P'^2) on [-1,1], halved
    }
}

// Collapsed (Duffy) product rule on {x, y >= 0, x + y <= 1}: y = r,
// x = s (1 - r), weight w_s w_r (1 - r) for Gauss points s, r on [0, 1];
// exact for polynomials of total degree 2 NG - 2 = 8 (the Jacobian adds one
// degree in r).
quad_rule make_rule()
{
    double a[NG], wa[NG];
    gauss_legendre01(NG, a, wa);
    quad_rule q;
    for (int i = 0; i < NG; ++i)      // s
        for (int j = 0; j < NG; ++j) {  // r
            q.x[NG * i + j] = a[i] * (1.0 - a[j]);
            q.y[NG * i + j] = a[j];
            q.w[NG * i + j] = wa[i] * wa[j] * (1.0 - a[j]);
        }
    return q;
}

__global__ __launch_bounds__(NT) void k_err(int32_t nE, const double2* __restrict__ exy,
                                            const double* __restrict__ U, phf_fn_dev u, double t,
                                            quad_rule q, double* __restrict__ part)
{
    __shared__ double sh[NT / 64];
    double s_h1 = 0.0, s_l2 = 0.0;
    for (int32_t m = blockIdx.x * NT + threadIdx.x; m < nE; m += gridDim.x * NT) {
        const double2 P0 = exy[3 * (int64_t)m], P1 = exy[3 * (int64_t)m + 1],
                      P2 = exy[3 * (int64_t)m + 2];
        const double u0 = U[3 * (int64_t)m], u1 = U[3 * (int64_t)m + 1], u2 = U[3 * (int64_t)m + 2];
        const double d1x = P1.x - P0.x, d1y = P1.y - P0.y, d2x = P2.x - P0.x, d2y = P2.y - P0.y;
        const double det = d1x * d2y - d1y * d2x;  // 2 |T|
        // grad of U_h = u0 + (u1 - u0) l1 + (u2 - u0) l2 with
        // grad l1 = (d2y, -d2x)/det, grad l2 = (-d1y, d1x)/det
        const double gx = ((u1 - u0) * d2y - (u2 - u0) * d1y) / det;
        const double gy = (-(u1 - u0) * d2x + (u2 - u0) * d1x) / det;
        double e_h1 = 0.0, e_l2 = 0.0;
        for (int k = 0; k < NG * NG; ++k) {
            const double l1 = q.x[k], l2 = q.y[k];
            const double x = P0.x + l1 * d1x + l2 * d2x, y = P0.y + l1 * d1y + l2 * d2y;
            const double uh = u0 + (u1 - u0) * l1 + (u2 - u0) * l2;
            const double ue = phf_fn_eval(u, x, y, t, 0.0, 0.0, -1);
            double ex, ey;
            phf_fn_grad(u, x, y, t, &ex, &ey);
            e_l2 = fma(q.w[k], (ue - uh) * (ue - uh), e_l2);
            e_h1 = fma(q.w[k], (ex - gx) * (ex - gx) + (ey - gy) * (ey - gy), e_h1);
        }
        s_l2 = fma(fabs(det), e_l2, s_l2);
        s_h1 = fma(fabs(det), e_h1, s_h1);
    }
    const double a = phf_block_sum_f64<NT>(s_h1, sh);
    const double b = phf_block_sum_f64<NT>(s_l2, sh);
    if (threadIdx.x == 0) {
        part[blockIdx.x] = a;
        part[MAXB + blockIdx.x] = b;
    }
}

// Sums the block partials in a fixed order; ROOT: writes the square roots
// (the norms) instead of the squared norms.
template <bool ROOT>
__global__ __launch_bounds__(NT) void k_err_final(const double* __restrict__ part, int32_t nb,
                                                  double* __restrict__ out)
{
    __shared__ double sh[NT / 64];
    double a = 0.0, b = 0.0;
    for (int q = threadIdx.x; q < nb; q += NT) {
        a += part[q];
        b += part[MAXB + q];
    }
    a = phf_block_sum_f64<NT>(a, sh);
    b = phf_block_sum_f64<NT>(b, sh);
    if (threadIdx.x == 0) {
        out[0] = ROOT ? sqrt(a) : a;
        out[1] = ROOT ? sqrt(b) : b;
    }
}

bool norm_kind_ok(int k)
{
    return k == PHF_FN_ZERO || k == PHF_FN_CONST || k == PHF_FN_SIN_COS || k == PHF_FN_SIN_SIN ||
           k == PHF_FN_PAPER_U;
}

int32_t norm_blocks(int32_t nE)
{
    return (int32_t)std::min<int64_t>(std::max<int64_t>((nE + NT - 1) / NT, 1), MAXB);
}

#define TRY(x)               \
    do {                     \
        int rc_ = (x);       \
        if (rc_) return rc_; \
    } while (0)

}  // namespace

extern "C" int phf_error_norms(phf_mesh* mesh, const double* U, const phf_fn* u, double t,
                               double* h1, double* l2)
{
    if (!mesh || !U || !u || !h1 || !l2) return PHF_EINVAL;
    phf_ctx* ctx = mesh->ctx;
    if (!norm_kind_ok(u->kind))
        return phf_set_error(ctx, PHF_EINVAL,
                             "phf_error_norms: kind %d has no device gradient", u->kind);
    static const quad_rule rule = make_rule();
    const int32_t nb = norm_blocks(mesh->nE);
    double* part = nullptr;
    TRY(phf_dmalloc(ctx, &part, 2 * MAXB + 2, "norm partials"));
    int rc = PHF_OK;
    auto body = [&]() -> int {
        PHF_LAUNCH(ctx, "k_err", k_err, nb, NT, 0, mesh->nE, mesh->exy, U, phf_fn_to_dev(*u), t,
                   rule, part);
        PHF_LAUNCH(ctx, "k_err_final", k_err_final<false>, 1, NT, 0, part, nb, part + 2 * MAXB);
        double h[2];
        PHF_HIP(ctx, hipMemcpyAsync(h, part + 2 * MAXB, sizeof(h), hipMemcpyDeviceToHost,
                                    ctx->stream));
        PHF_HIP(ctx, hipStreamSynchronize(ctx->stream));
        *h1 = std::sqrt(h[0]);
        *l2 = std::sqrt(h[1]);
        return PHF_OK;
    };
    rc = body();
    phf_dfree(part);
    return rc;
}

// ---- the variant that allocates nothing ----------------------------------
// The block partials of k_err (MAXB for each norm) live in this file-scope
// device array instead of a pool block: 16 KiB, one copy per device, held
// until the process ends. Every call on a device writes all the partials it
// reads, so nothing needs clearing; calls that overlap on one device (two
// streams, or two host threads) race on it.
static __device__ __align__(256) double scratch[2 * MAXB];

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
double* g_scratch[MAX_DEVICES];  // device address of `scratch`, per device, once resolved

// Address of the scratch array on `device` (current), resolved on the first
// call for that device. In host code the array's name is only a stand-in
// for its symbol; kernels are given this address.
int scratch_address(phf_ctx* ctx, double** out)
{
    const int dev = ctx->device;
    if (dev < 0 || dev >= MAX_DEVICES)
        return phf_set_error(ctx, PHF_EINVAL, "phf_error_norms_noalloc: device %d >= %d", dev,
                             MAX_DEVICES);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return phf_set_error(ctx, PHF_EHIP,
                                 "phf_error_norms_noalloc: hipGetSymbolAddress failed: %s",
                                 hipGetErrorString(e));
        g_scratch[dev] = static_cast<double*>(p);
    }
    *out = g_scratch[dev];
    return PHF_OK;
}
}  // namespace

extern "C" int phf_error_norms_noalloc(phf_mesh* mesh, const double* U, const phf_fn* u, double t,
                                       double* norms)
{
    if (!mesh || !U || !u || !norms) return PHF_EINVAL;
    phf_ctx* ctx = mesh->ctx;
    if (!norm_kind_ok(u->kind))
        return phf_set_error(ctx, PHF_EINVAL,
                             "phf_error_norms_noalloc: kind %d has no device gradient", u->kind);
    static const quad_rule rule = make_rule();
    const int32_t nb = norm_blocks(mesh->nE);
    if (2 * (int64_t)nb > (int64_t)(sizeof(scratch) / sizeof(double)))
        return phf_set_error(ctx, PHF_EINVAL,
                             "phf_error_norms_noalloc: %d partial pairs exceed the %d the scratch "
                             "array holds", nb, MAXB);
    PHF_HIP(ctx, hipSetDevice(ctx->device));
    double* part = nullptr;
    TRY(scratch_address(ctx, &part));
    // plain launches: no trace events, nothing allocated, nothing waited for
    hipLaunchKernelGGL(k_err, dim3(nb), dim3(NT), 0, ctx->stream, mesh->nE, mesh->exy, U,
                       phf_fn_to_dev(*u), t, rule, part);
    hipLaunchKernelGGL(k_err_final<true>, dim3(1), dim3(NT), 0, ctx->stream, part, nb, norms);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return phf_set_error(ctx, PHF_EHIP, "phf_error_norms_noalloc: launch failed: %s",
                             hipGetErrorString(e));
    return PHF_OK;
}
