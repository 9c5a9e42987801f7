// Certificate of Prop. 1 over a final sample set (pairwise cone + witnesses).
//
// Every pair is screened in float32; pairs whose float32 margin is within
// eps of the threshold are decided in float64, so the counts equal a pure
// float64 evaluation.  eps comes from the data on the device: with u the
// float32 unit roundoff, Mc the largest |coordinate| (points and witnesses)
// and Ms the largest |value|, a float32 distance errs by at most 28 u Mc
// (inputs rounded: 2 sqrt3 u Mc; differences: sqrt3 u Mc; squares, sum and
// sqrt: 6 u d with d <= 2 sqrt3 Mc), a difference of two values by 4 u Ms
// and the final subtraction by u (2 sqrt3 Mc + 2 Ms), so a margin errs by
// less than u (32 Mc + 6 Ms); eps is twice that.  Rows whose value is NaN
// (queries the greedy left without a value) are not part of the set: every
// comparison with them is false and their witness is not checked.
#include "common.h"

#include <cmath>

namespace sdfi {

namespace {

constexpr int BT = 256;
constexpr int TILE = 256;
constexpr int RPT = 2;  // rows per thread

struct Cnt {
    unsigned long long pair;
    unsigned long long wit;
};

// largest finite |coordinate| of points and witnesses and largest finite |value|
// (as float bits: non-negative floats order like their bit patterns); the
// counters start at zero here (a kernel, not a memset)
__global__ void mag_init_kernel(unsigned *mag, Cnt *cnt) {
    if (threadIdx.x == 0) {
        mag[0] = mag[1] = 0u;
        cnt->pair = cnt->wit = 0ull;
    }
}

__global__ void mag_kernel(const double *__restrict__ pv, const double *__restrict__ wit, int64_t N, unsigned *mag) {
    float mc = 0.0f, ms = 0.0f;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < N; i += stride) {
        for (int k = 0; k < 3; ++k) {
            const double x = fabs(pv[4 * i + k]), w = fabs(wit[3 * i + k]);
            if (isfinite(x)) mc = fmaxf(mc, (float)x);
            if (isfinite(w)) mc = fmaxf(mc, (float)w);
        }
        const double v = fabs(pv[4 * i + 3]);
        if (isfinite(v)) ms = fmaxf(ms, (float)v);
    }
    for (int o = 32; o > 0; o >>= 1) {
        mc = fmaxf(mc, __shfl_xor(mc, o, 64));
        ms = fmaxf(ms, __shfl_xor(ms, o, 64));
    }
    if ((threadIdx.x & 63) == 0) {
        atomicMax(&mag[0], __float_as_uint(mc));
        atomicMax(&mag[1], __float_as_uint(ms));
    }
}

__global__ void pack_kernel(const double *__restrict__ pv, float4 *__restrict__ out, int64_t N) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < N) out[i] = make_float4((float)pv[4 * i], (float)pv[4 * i + 1], (float)pv[4 * i + 2], (float)pv[4 * i + 3]);
}

__device__ inline double d64(const double *a, const double *b) {
#pragma clang fp contract(off)
    double dx = a[0] - b[0], dy = a[1] - b[1], dz = a[2] - b[2];
    return sqrt(dx * dx + dy * dy + dz * dz);
}

__global__ __launch_bounds__(BT) void certify_kernel(const float4 *__restrict__ pf, const double *__restrict__ pv,
                                                     const double *__restrict__ wit, int64_t N, double tol,
                                                     const unsigned *__restrict__ mag, Cnt *out) {
    __shared__ float4 tile[TILE];
    __shared__ unsigned long long red[2][BT];
    const int tid = threadIdx.x;
    const int64_t base = (int64_t)blockIdx.x * BT * RPT;
    float px[RPT], py[RPT], pz[RPT], ps[RPT], wx[RPT], wy[RPT], wz[RPT];
    bool wcov[RPT];
    unsigned long long npair = 0;
#pragma unroll
    for (int k = 0; k < RPT; ++k) {
        int64_t x = base + k * BT + tid;
        int64_t xc = x < N ? x : N - 1;
        float4 p = pf[xc];
        px[k] = p.x; py[k] = p.y; pz[k] = p.z; ps[k] = p.w;
        wx[k] = (float)wit[3 * xc]; wy[k] = (float)wit[3 * xc + 1]; wz[k] = (float)wit[3 * xc + 2];
        wcov[k] = false;
    }
    const float ftol = (float)tol;
    constexpr float U = 5.9604645e-8f;  // float32 unit roundoff
    const float eps = 2.0f * U * (32.0f * __uint_as_float(mag[0]) + 6.0f * __uint_as_float(mag[1]));
    for (int64_t t0 = 0; t0 < N; t0 += TILE) {
        const int cnt = (int)min((int64_t)TILE, N - t0);
        __syncthreads();
        if (tid < cnt) tile[tid] = pf[t0 + tid];
        __syncthreads();
        for (int j = 0; j < cnt; ++j) {
            const float4 q = tile[j];
            const int64_t y = t0 + j;
#pragma unroll
            for (int k = 0; k < RPT; ++k) {
                const int64_t x = base + k * BT + tid;
                if (x >= N || y == x) continue;
                float dx = px[k] - q.x, dy = py[k] - q.y, dz = pz[k] - q.z;
                float d = __builtin_amdgcn_sqrtf(dx * dx + dy * dy + dz * dz);
                float marg = d - fabsf(ps[k] - q.w);
                if (y > x && marg < -ftol + eps) {
                    double dd = d64(pv + 4 * x, pv + 4 * y);
                    if (fabs(pv[4 * x + 3] - pv[4 * y + 3]) > dd + tol) ++npair;
                }
                float ex = wx[k] - q.x, ey = wy[k] - q.y, ez = wz[k] - q.z;
                float dw = __builtin_amdgcn_sqrtf(ex * ex + ey * ey + ez * ez);
                if (!wcov[k] && dw - fabsf(q.w) < -ftol + eps) {
                    double ddw = d64(wit + 3 * x, pv + 4 * y);
                    if (ddw < fabs(pv[4 * y + 3]) - tol - 1e-9) wcov[k] = true;
                }
            }
        }
    }
    unsigned long long nw = 0;
#pragma unroll
    for (int k = 0; k < RPT; ++k) {
        const int64_t x = base + k * BT + tid;
        if (x >= N || isnan(pv[4 * x + 3])) continue;  // a row without a value is not in the set
        double w[3] = {wit[3 * x], wit[3 * x + 1], wit[3 * x + 2]};
        bool off = !(fabs(d64(w, pv + 4 * x) - fabs(pv[4 * x + 3])) <= tol);  // NaN counts as off
        if (wcov[k] || off) ++nw;
    }
    red[0][tid] = npair;
    red[1][tid] = nw;
    __syncthreads();
    for (int s = BT / 2; s > 0; s >>= 1) {
        if (tid < s) {
            red[0][tid] += red[0][tid + s];
            red[1][tid] += red[1][tid + s];
        }
        __syncthreads();
    }
    if (tid == 0) {
        atomicAdd(&out->pair, red[0][0]);
        atomicAdd(&out->wit, red[1][0]);
    }
}

}  // namespace

size_t certify_ws(int64_t N, const sdfi_options &) {
    Carver c(nullptr, 0, true);
    c.take<float4>(N > 0 ? N : 1);
    c.take<Cnt>(1);
    c.take<unsigned>(2);
    return c.used + 256;
}

sdfi_status run_certify(const double *pv, const double *wit, int64_t N, int64_t *pair_viol, int64_t *wit_viol,
                        Carver &ws, const sdfi_options &o, hipStream_t st) {
    float4 *pf = ws.take<float4>(N > 0 ? N : 1);
    Cnt *cnt = ws.take<Cnt>(1);
    unsigned *mag = ws.take<unsigned>(2);
    if (!ws.ok()) {
        set_error("workspace too small for the certificate");
        return SDFI_ERR_WORKSPACE;
    }
    mag_init_kernel<<<1, 64, 0, st>>>(mag, cnt);
    if (N > 0) {
        mag_kernel<<<(unsigned)std::min<int64_t>((N + 255) / 256, 1024), 256, 0, st>>>(pv, wit, N, mag);
        pack_kernel<<<(unsigned)((N + 255) / 256), 256, 0, st>>>(pv, pf, N);
        const int64_t per = (int64_t)BT * RPT;
        KernelTimer tm("certify", st);
        certify_kernel<<<(unsigned)((N + per - 1) / per), BT, 0, st>>>(pf, pv, wit, N, o.tol, mag, cnt);
        tm.stop();
        SDFI_HIP(hipGetLastError());
    }
    Cnt h;
    SDFI_HIP(hipMemcpyAsync(&h, cnt, sizeof(Cnt), hipMemcpyDeviceToHost, st));
    SDFI_HIP(hipStreamSynchronize(st));
    *pair_viol = (int64_t)h.pair;
    *wit_viol = (int64_t)h.wit;
    return SDFI_OK;
}

}  // namespace sdfi

extern "C" sdfi_status sdfi_certify(const double *pts_values, const double *witness, int64_t N, sdfi_report *report,
                                    void *ws, size_t ws_bytes, const sdfi_options *opt, sdfi_stream stream) {
    using namespace sdfi;
    sdfi_options o;
    sdfi_status s = read_options(opt, &o);
    if (s != SDFI_OK) return s;
    SDFI_CHECK_ARG(N >= 0 && N < (int64_t(1) << 31), "N must be in [0, 2^31)");
    SDFI_CHECK_ARG(report != nullptr, "report is required");
    SDFI_CHECK_ARG(N == 0 || (pts_values && witness), "null array argument");
    if (ws_bytes < certify_ws(N, o) || !ws) {
        set_error("workspace of %zu bytes is below the %zu required", ws_bytes, certify_ws(N, o));
        return SDFI_ERR_WORKSPACE;
    }
    Carver c(ws, ws_bytes);
    int64_t pv = 0, wv = 0;
    s = run_certify(pts_values, witness, N, &pv, &wv, c, o, to_hip(stream));
    if (s != SDFI_OK) return s;
    report->n_violations_pairwise = pv;
    report->n_violations_witness = wv;
    report->pairs_evaluated = N * (N - 1) / 2 + N * (N - 1);
    return SDFI_OK;
}
