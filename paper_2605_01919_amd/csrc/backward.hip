// Gradient of sum_j g_j v_j with respect to the samples, through the forest
// of active parents left by the greedy interpolation.  With the decisions
// fixed every value depends on one parent constraint t:
//   HI: v = s_t + |q - p_t|, LO: v = s_t - |q - p_t|, COINCIDENT: v = s_t,
//   RMIN_T: v = sign * ||q - p_t| - |s_t||;  ZERO / RMIN_D / RMIN_U: no parent.
// A query whose parent is an earlier query passes its adjoint on (times
// dv/ds_parent); the chains are collapsed by pointer jumping (log2 depth
// rounds), then each chain's last link scatters into its sample.
#include <hip/hip_runtime.h>

#include "common.h"

namespace sdfi {

namespace {

__device__ inline int sgn_class(double s) { return s > 1e-9 ? 1 : (s < -1e-9 ? -1 : 0); }

// per query: link factor ds (dv/ds_parent), position factor dp (dv/dp_parent),
// next query up the chain (self when the parent is a sample or missing)
__global__ void links_kernel(const double *samples, int64_t n, const double *queries, int64_t m,
                             const double *values, const int64_t *active, const uint8_t *kind, double *ds,
                             double *dp, int64_t *nxt, double *mul) {
    int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (j >= m) return;
    int k = kind[j];
    int64_t t = active[j];
    double f = 0.0, g[3] = {0.0, 0.0, 0.0};
    bool link = (k == SDFI_KIND_HI || k == SDFI_KIND_LO || k == SDFI_KIND_COINCIDENT || k == SDFI_KIND_RMIN_T) &&
                t >= 0 && t < n + m;
    if (link) {
        double pt[3], st;
        if (t < n) {
            pt[0] = samples[4 * t]; pt[1] = samples[4 * t + 1]; pt[2] = samples[4 * t + 2]; st = samples[4 * t + 3];
        } else {
            int64_t u = t - n;
            pt[0] = queries[3 * u]; pt[1] = queries[3 * u + 1]; pt[2] = queries[3 * u + 2]; st = values[u];
        }
        const double *q = queries + 3 * j;
        double e[3] = {pt[0] - q[0], pt[1] - q[1], pt[2] - q[2]};
        double d = sqrt(e[0] * e[0] + e[1] * e[1] + e[2] * e[2]);
        double unit[3] = {0.0, 0.0, 0.0};
        if (d > 0.0) for (int a = 0; a < 3; ++a) unit[a] = e[a] / d;  // d|q - p_t| / dp_t
        if (k == SDFI_KIND_HI) {
            f = 1.0;
            for (int a = 0; a < 3; ++a) g[a] = unit[a];
        } else if (k == SDFI_KIND_LO) {
            f = 1.0;
            for (int a = 0; a < 3; ++a) g[a] = -unit[a];
        } else if (k == SDFI_KIND_COINCIDENT) {
            f = 1.0;
        } else {
            double sigma = values[j] > 0.0 ? 1.0 : (values[j] < 0.0 ? -1.0 : 0.0);
            double se = d - fabs(st) > 0.0 ? 1.0 : -1.0;
            f = sigma * se * (-(double)sgn_class(st));
            for (int a = 0; a < 3; ++a) g[a] = sigma * se * unit[a];
        }
    }
    ds[j] = f;
    for (int a = 0; a < 3; ++a) dp[3 * j + a] = g[a];
    if (link && t >= n) {
        nxt[j] = t - n;
        mul[j] = f;
    } else {
        nxt[j] = j;
        mul[j] = 1.0;
    }
}

__global__ void jump_kernel(const int64_t *nxt, const double *mul, int64_t *nxt2, double *mul2, int64_t m) {
    int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (j >= m) return;
    int64_t u = nxt[j];
    nxt2[j] = nxt[u];
    mul2[j] = mul[j] * mul[u];
}

__global__ void collect_kernel(const double *gv, const int64_t *root, const double *mul, double *G, int64_t m) {
    int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (j >= m) return;
    double c = gv[j] * mul[j];
    if (c != 0.0) atomicAdd(&G[root[j]], c);
}

__global__ void scatter_kernel(const double *G, const int64_t *active, const uint8_t *kind, const double *ds,
                               const double *dp, int64_t n, int64_t m, double *grad_s, double *grad_p) {
    int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (j >= m) return;
    int64_t t = active[j];
    if (t < 0 || t >= n || (ds[j] == 0.0 && dp[3 * j] == 0.0 && dp[3 * j + 1] == 0.0 && dp[3 * j + 2] == 0.0)) return;
    int k = kind[j];
    if (!(k == SDFI_KIND_HI || k == SDFI_KIND_LO || k == SDFI_KIND_COINCIDENT || k == SDFI_KIND_RMIN_T)) return;
    double g = G[j];
    if (g == 0.0) return;
    atomicAdd(&grad_s[t], g * ds[j]);
    for (int a = 0; a < 3; ++a) atomicAdd(&grad_p[3 * t + a], g * dp[3 * j + a]);
}

}  // namespace

size_t backward_ws(int64_t n, int64_t m) {
    Carver c(nullptr, 0, true);
    c.take<double>(m + 1);
    c.take<double>(3 * (m + 1));
    c.take<int64_t>(2 * (m + 1));
    c.take<double>(2 * (m + 1));
    c.take<double>(m + 1);
    return c.used + 1024;
}

}  // namespace sdfi

extern "C" sdfi_status sdfi_greedy_backward(const double *grad_values, const double *samples, int64_t n,
                                            const double *queries, int64_t m, const double *values,
                                            const int64_t *active, const uint8_t *kind, double *grad_s,
                                            double *grad_p, void *ws, size_t ws_bytes, sdfi_stream stream) {
    using namespace sdfi;
    SDFI_CHECK_ARG(n >= 1 && m >= 0 && n + m < (int64_t(1) << 31), "sizes out of range");
    SDFI_CHECK_ARG(grad_s && grad_p && samples, "null array argument");
    SDFI_CHECK_ARG(m == 0 || (grad_values && queries && values && active && kind), "null array argument");
    if (ws_bytes < backward_ws(n, m) || !ws) {
        set_error("workspace of %zu bytes is below the %zu required", ws_bytes, backward_ws(n, m));
        return SDFI_ERR_WORKSPACE;
    }
    hipStream_t st = to_hip(stream);
    SDFI_HIP(hipMemsetAsync(grad_s, 0, sizeof(double) * n, st));
    SDFI_HIP(hipMemsetAsync(grad_p, 0, sizeof(double) * 3 * n, st));
    if (m == 0) return SDFI_OK;
    Carver c(ws, ws_bytes);
    double *ds = c.take<double>(m + 1);
    double *dp = c.take<double>(3 * (m + 1));
    int64_t *nxt = c.take<int64_t>(2 * (m + 1));
    double *mul = c.take<double>(2 * (m + 1));
    double *G = c.take<double>(m + 1);
    unsigned blocks = (unsigned)((m + 255) / 256);
    links_kernel<<<blocks, 256, 0, st>>>(samples, n, queries, m, values, active, kind, ds, dp, nxt, mul);
    // pointer jumping: after r rounds every query points 2^r links up its chain
    int rounds = 1;
    while ((int64_t(1) << rounds) < m + 1) ++rounds;
    int64_t *a = nxt, *b = nxt + (m + 1);
    double *ma = mul, *mb = mul + (m + 1);
    for (int r = 0; r < rounds; ++r) {
        jump_kernel<<<blocks, 256, 0, st>>>(a, ma, b, mb, m);
        std::swap(a, b);
        std::swap(ma, mb);
    }
    SDFI_HIP(hipMemsetAsync(G, 0, sizeof(double) * m, st));
    collect_kernel<<<blocks, 256, 0, st>>>(grad_values, a, ma, G, m);
    scatter_kernel<<<blocks, 256, 0, st>>>(G, active, kind, ds, dp, n, m, grad_s, grad_p);
    SDFI_HIP(hipGetLastError());
    return SDFI_OK;
}
