// Dense pairwise bound sweep: lo = max_i(s_i - d_i), hi = min_i(s_i + d_i)
// over all samples for every query (Sec. 4.3 bounds), with argmax/argmin
// resolved exactly in float64 (smallest index within tie_tol).
//
// Pass 1 (sweep): a work-group owns BT*QPT queries and streams the samples
// through LDS in tiles of TILE.  Every thread keeps, per query, the running
// extreme and the extreme of the current tile; after each tile it records
// the tile in a short per-query candidate list when the tile extreme comes
// within `eps` of the running extreme.  eps bounds the float32 error of a
// pair value (2 x 5e-7) plus tie_tol, so every sample whose float64 value
// can reach the tie band of the true extreme sits in a listed tile.  In
// float64 mode eps is tie_tol plus one ulp-scale margin and the list is
// exact.  A list that would hold more than LIST near-extreme tiles marks the
// query for a full float64 rescan.
//
// Pass 2 (resolve): one wavefront per query recomputes its listed tiles in
// float64 (or all samples after an overflow), takes the exact extreme and
// the smallest index within tie_tol of it, and writes the flags.
#include "common.h"

#include <cfloat>
#include <cmath>

namespace sdfi {

namespace {

constexpr int BT = 256;    // threads per sweep work-group
constexpr int TILE = 256;  // samples per LDS tile
constexpr int LIST = 8;    // candidate tiles kept per query and side
constexpr uint32_t OVERFLOW_BIT = 0x80000000u;

template <typename T>
struct Pt4 {
    T x, y, z, s;
};

__global__ void pack_f32_kernel(const double *__restrict__ samples, float4 *__restrict__ out, int64_t n) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) {
        const double *p = samples + 4 * i;
        out[i] = make_float4((float)p[0], (float)p[1], (float)p[2], (float)p[3]);
    }
}

__device__ inline float fsqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ inline double fsqrt(double x) { return sqrt(x); }

template <typename T>
__device__ inline T inf_of() { return (T)INFINITY; }

template <typename T>
struct SweepOut {
    T *run;            // m x 2 (lo, hi) running extremes
    uint32_t *count;   // m x 2 list lengths (| OVERFLOW_BIT)
    int32_t *tiles;    // m x 2 x LIST
    T *vals;           // m x 2 x LIST tile extremes
};

template <typename T>
__device__ inline void note_tile(int side, int64_t qi, int tile, T tv, T &run, uint32_t &cnt, T eps,
                                 const SweepOut<T> &o) {
    // side 0: tile max vs running max; side 1: tile min vs running min (mirrored)
    bool near = side == 0 ? (tv >= run - eps) : (tv <= run + eps);
    if (!near) return;
    if (side == 0 ? tv > run : tv < run) run = tv;
    if (cnt & OVERFLOW_BIT) return;
    int64_t base = (qi * 2 + side) * LIST;
    if (cnt == LIST) {
        // drop entries that fell out of the band of the new extreme
        uint32_t k = 0;
        for (uint32_t e = 0; e < LIST; ++e) {
            T v = o.vals[base + e];
            bool keep = side == 0 ? (v >= run - eps) : (v <= run + eps);
            if (keep) {
                o.vals[base + k] = v;
                o.tiles[base + k] = o.tiles[base + e];
                ++k;
            }
        }
        cnt = k;
        if (cnt == LIST) {
            cnt = OVERFLOW_BIT;
            return;
        }
    }
    o.tiles[base + cnt] = tile;
    o.vals[base + cnt] = tv;
    ++cnt;
}

template <typename T, int QPT>
__global__ __launch_bounds__(BT) void sweep_kernel(const Pt4<T> *__restrict__ samples, int n,
                                                   const double *__restrict__ queries, int64_t m, T eps,
                                                   SweepOut<T> o) {
    __shared__ Pt4<T> tile[TILE];
    const int tid = threadIdx.x;
    const int64_t base = (int64_t)blockIdx.x * BT * QPT;
    T qx[QPT], qy[QPT], qz[QPT], lo_run[QPT], hi_run[QPT];
    uint32_t clo[QPT], chi[QPT];
#pragma unroll
    for (int k = 0; k < QPT; ++k) {
        int64_t qi = base + k * BT + tid;
        int64_t qc = qi < m ? qi : m - 1;
        qx[k] = (T)queries[3 * qc];
        qy[k] = (T)queries[3 * qc + 1];
        qz[k] = (T)queries[3 * qc + 2];
        lo_run[k] = -inf_of<T>();
        hi_run[k] = inf_of<T>();
        clo[k] = 0;
        chi[k] = 0;
    }
    const int ntiles = (n + TILE - 1) / TILE;
    for (int t = 0; t < ntiles; ++t) {
        const int cnt = min(TILE, n - t * TILE);
        __syncthreads();
        if (tid < cnt) tile[tid] = samples[(int64_t)t * TILE + tid];
        __syncthreads();
        T lo_t[QPT], hi_t[QPT];
#pragma unroll
        for (int k = 0; k < QPT; ++k) {
            lo_t[k] = -inf_of<T>();
            hi_t[k] = inf_of<T>();
        }
        if (cnt == TILE) {
#pragma unroll 4
            for (int j = 0; j < TILE; ++j) {
                const Pt4<T> p = tile[j];
#pragma unroll
                for (int k = 0; k < QPT; ++k) {
                    T dx = qx[k] - p.x, dy = qy[k] - p.y, dz = qz[k] - p.z;
                    T d = fsqrt(dx * dx + dy * dy + dz * dz);
                    lo_t[k] = fmax(lo_t[k], p.s - d);
                    hi_t[k] = fmin(hi_t[k], p.s + d);
                }
            }
        } else {
            for (int j = 0; j < cnt; ++j) {
                const Pt4<T> p = tile[j];
#pragma unroll
                for (int k = 0; k < QPT; ++k) {
                    T dx = qx[k] - p.x, dy = qy[k] - p.y, dz = qz[k] - p.z;
                    T d = fsqrt(dx * dx + dy * dy + dz * dz);
                    lo_t[k] = fmax(lo_t[k], p.s - d);
                    hi_t[k] = fmin(hi_t[k], p.s + d);
                }
            }
        }
#pragma unroll
        for (int k = 0; k < QPT; ++k) {
            int64_t qi = base + k * BT + tid;
            if (qi < m) {
                note_tile<T>(0, qi, t, lo_t[k], lo_run[k], clo[k], eps, o);
                note_tile<T>(1, qi, t, hi_t[k], hi_run[k], chi[k], eps, o);
            }
        }
    }
#pragma unroll
    for (int k = 0; k < QPT; ++k) {
        int64_t qi = base + k * BT + tid;
        if (qi < m) {
            o.run[2 * qi] = lo_run[k];
            o.run[2 * qi + 1] = hi_run[k];
            o.count[2 * qi] = clo[k];
            o.count[2 * qi + 1] = chi[k];
        }
    }
}

// float64 pair value of side 0 (s - d) or side 1 (s + d); no contraction so the
// arithmetic is sqrt((dx*dx + dy*dy) + dz*dz) exactly
__device__ inline double pair_val(const double *__restrict__ s4, const double q[3], int side) {
#pragma clang fp contract(off)
    double dx = q[0] - s4[0], dy = q[1] - s4[1], dz = q[2] - s4[2];
    double d = sqrt(dx * dx + dy * dy + dz * dz);
    return side == 0 ? s4[3] - d : s4[3] + d;
}

__device__ inline double wave_max(double v) {
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    return v;
}
__device__ inline double wave_min(double v) {
    for (int off = 32; off > 0; off >>= 1) v = fmin(v, __shfl_xor(v, off, 64));
    return v;
}
__device__ inline int64_t wave_min_i64(int64_t v) {
    for (int off = 32; off > 0; off >>= 1) {
        int64_t o = __shfl_xor(v, off, 64);
        v = o < v ? o : v;
    }
    return v;
}
__device__ inline int wave_sum(int v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__device__ inline int sign_class(double s, double tie) { return s > tie ? 1 : (s < -tie ? -1 : 0); }

template <typename T>
__global__ __launch_bounds__(256) void resolve_kernel(const double *__restrict__ samples, int64_t n,
                                                      const double *__restrict__ queries, int64_t m, T eps,
                                                      SweepOut<T> o, double tol, double tie, double *lo_out,
                                                      double *hi_out, int32_t *argmax, int32_t *argmin,
                                                      uint32_t *flags, int64_t *overflows) {
    const int lane = threadIdx.x & 63;
    const int64_t qi = (int64_t)blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
    if (qi >= m) return;
    const double q[3] = {queries[3 * qi], queries[3 * qi + 1], queries[3 * qi + 2]};
    double ext[2];
    int64_t arg[2];
    int tied[2];
    for (int side = 0; side < 2; ++side) {
        uint32_t cnt = o.count[2 * qi + side];
        const bool full = (cnt & OVERFLOW_BIT) != 0;
        const T run = o.run[2 * qi + side];
        const int64_t lb = (qi * 2 + side) * LIST;
        const int nt = full ? (int)((n + TILE - 1) / TILE) : (int)cnt;
        // exact extreme over the candidate tiles
        double best = side == 0 ? -INFINITY : INFINITY;
        for (int e = 0; e < nt; ++e) {
            int t;
            if (full) {
                t = e;
            } else {
                T v = o.vals[lb + e];
                bool keep = side == 0 ? (v >= run - eps) : (v <= run + eps);
                if (!keep) continue;
                t = o.tiles[lb + e];
            }
            for (int j = lane; j < TILE; j += 64) {
                int64_t i = (int64_t)t * TILE + j;
                if (i < n) {
                    double v = pair_val(samples + 4 * i, q, side);
                    best = side == 0 ? fmax(best, v) : fmin(best, v);
                }
            }
        }
        best = side == 0 ? wave_max(best) : wave_min(best);
        // smallest index within the tie band, and the band's population
        int64_t first = INT64_MAX;
        int inband = 0;
        for (int e = 0; e < nt; ++e) {
            int t;
            if (full) {
                t = e;
            } else {
                T v = o.vals[lb + e];
                bool keep = side == 0 ? (v >= run - eps) : (v <= run + eps);
                if (!keep) continue;
                t = o.tiles[lb + e];
            }
            for (int j = lane; j < TILE; j += 64) {
                int64_t i = (int64_t)t * TILE + j;
                if (i < n) {
                    double v = pair_val(samples + 4 * i, q, side);
                    bool in = side == 0 ? (v >= best - tie) : (v <= best + tie);
                    if (in) {
                        inband++;
                        first = i < first ? i : first;
                    }
                }
            }
        }
        ext[side] = best;
        arg[side] = wave_min_i64(first);
        tied[side] = wave_sum(inband);
        if (full && lane == 0) atomicAdd((unsigned long long *)overflows, 1ull);
    }
    if (lane == 0) {
        double lo = ext[0], hi = ext[1];
        // no candidate at all only happens with NaN inputs: report index -1
        const bool have_a = arg[0] >= 0 && arg[0] < n, have_b = arg[1] >= 0 && arg[1] < n;
        lo_out[qi] = lo;
        hi_out[qi] = hi;
        argmax[qi] = have_a ? (int32_t)arg[0] : -1;
        argmin[qi] = have_b ? (int32_t)arg[1] : -1;
        uint32_t f = 0;
        if (lo > hi + tol) f |= SDFI_FLAG_INFEASIBLE;
        if (lo > tol) f |= SDFI_FLAG_INSIDE_POS;
        if (hi < -tol) f |= SDFI_FLAG_INSIDE_NEG;
        if (tied[0] > 1) f |= SDFI_FLAG_TIE_LO;
        if (tied[1] > 1) f |= SDFI_FLAG_TIE_HI;
        if (have_b && sign_class(hi, tie) * sign_class(samples[4 * arg[1] + 3], tie) < 0) f |= SDFI_FLAG_HI_OPPOSITE;
        if (have_a && sign_class(lo, tie) * sign_class(samples[4 * arg[0] + 3], tie) < 0) f |= SDFI_FLAG_LO_OPPOSITE;
        flags[qi] = f;
    }
}

template <typename T>
struct SweepBufs {
    SweepOut<T> o;
    Pt4<T> *pts;
    int64_t *overflows;
};

template <typename T>
SweepBufs<T> carve_sweep(Carver &c, int64_t n, int64_t m) {
    SweepBufs<T> b;
    b.pts = std::is_same<T, float>::value ? c.take<Pt4<T>>(n) : nullptr;
    b.o.run = c.take<T>(2 * m);
    b.o.count = c.take<uint32_t>(2 * m);
    b.o.tiles = c.take<int32_t>(2 * m * LIST);
    b.o.vals = c.take<T>(2 * m * LIST);
    b.overflows = c.take<int64_t>(1);
    return b;
}

template <typename T, int QPT>
sdfi_status launch(const double *samples, int64_t n, const double *queries, int64_t m, double *lo, double *hi,
                   int32_t *argmax, int32_t *argmin, uint32_t *flags, Carver &ws, const sdfi_options &opt,
                   hipStream_t st, T eps, int64_t *overflow_count) {
    SweepBufs<T> b = carve_sweep<T>(ws, n, m);
    if (!ws.ok()) {
        set_error("workspace too small for the bound sweep");
        return SDFI_ERR_WORKSPACE;
    }
    const Pt4<T> *pts;
    if (std::is_same<T, float>::value) {
        pack_f32_kernel<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(samples, (float4 *)b.pts, n);
        pts = b.pts;
    } else {
        pts = reinterpret_cast<const Pt4<T> *>(samples);
    }
    SDFI_HIP(hipMemsetAsync(b.overflows, 0, sizeof(int64_t), st));
    const int64_t per = (int64_t)BT * QPT;
    KernelTimer t1("sweep", st);
    sweep_kernel<T, QPT><<<(unsigned)((m + per - 1) / per), BT, 0, st>>>(pts, (int)n, queries, m, eps, b.o);
    t1.stop();
    SDFI_HIP(hipGetLastError());
    KernelTimer t2("resolve", st);
    resolve_kernel<T><<<(unsigned)((m + 3) / 4), 256, 0, st>>>(samples, n, queries, m, eps, b.o, opt.tol,
                                                                opt.tie_tol, lo, hi, argmax, argmin, flags,
                                                                b.overflows);
    t2.stop();
    SDFI_HIP(hipGetLastError());
    if (overflow_count) {
        SDFI_HIP(hipMemcpyAsync(overflow_count, b.overflows, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    }
    return SDFI_OK;
}

}  // namespace

// float32 pair value error: inputs rounded (<= 2^-24 relative each), three
// subtractions, the squared sum and v_sqrt_f32 (1 ulp): well under 5e-7 for
// coordinates and values of magnitude <= 2; two values may err in opposite
// directions, hence 2 x 5e-7 plus the tie band.
static double eps_f32(const sdfi_options &o) { return 2.0 * 5e-7 + o.tie_tol + 1e-6; }
static double eps_f64(const sdfi_options &o) { return o.tie_tol * 1.001 + 1e-15; }

size_t bounds_ws(int64_t n, int64_t m, const sdfi_options &o) {
    Carver c(nullptr, 0, true);
    if (o.precision == SDFI_PREC_FP32_FP64_RECHECK)
        carve_sweep<float>(c, n, m);
    else
        carve_sweep<double>(c, n, m);
    return c.used + 256;
}

sdfi_status run_bounds(const double *samples, int64_t n, const double *queries, int64_t m, double *lo,
                       double *hi, int32_t *argmax, int32_t *argmin, uint32_t *flags, Carver &ws,
                       const sdfi_options &o, hipStream_t st, int64_t *overflow_count) {
    if (m == 0) return SDFI_OK;
    if (o.precision == SDFI_PREC_FP32_FP64_RECHECK)
        return launch<float, 4>(samples, n, queries, m, lo, hi, argmax, argmin, flags, ws, o, st,
                                (float)eps_f32(o), overflow_count);
    return launch<double, 2>(samples, n, queries, m, lo, hi, argmax, argmin, flags, ws, o, st, eps_f64(o),
                             overflow_count);
}

}  // namespace sdfi

extern "C" sdfi_status sdfi_bounds(const double *samples, int64_t n, const double *queries, int64_t m, double *lo,
                                   double *hi, int32_t *argmax, int32_t *argmin, uint32_t *flags, void *ws,
                                   size_t ws_bytes, const sdfi_options *opt, sdfi_stream stream) {
    using namespace sdfi;
    sdfi_options o;
    sdfi_status s = read_options(opt, &o);
    if (s != SDFI_OK) return s;
    SDFI_CHECK_ARG(n >= 1 && n < (int64_t(1) << 31), "n must be in [1, 2^31), got %lld", (long long)n);
    SDFI_CHECK_ARG(m >= 0 && m < (int64_t(1) << 31), "m must be in [0, 2^31), got %lld", (long long)m);
    if (m == 0) return SDFI_OK;
    SDFI_CHECK_ARG(samples && queries && lo && hi && argmax && argmin && flags, "null array argument");
    SDFI_CHECK_ARG(ws || ws_bytes == 0, "null workspace with nonzero size");
    if (ws_bytes < bounds_ws(n, m, o)) {
        set_error("workspace of %zu bytes is below the %zu required", ws_bytes, bounds_ws(n, m, o));
        return SDFI_ERR_WORKSPACE;
    }
    Carver c(ws, ws_bytes);
    return run_bounds(samples, n, queries, m, lo, hi, argmax, argmin, flags, c, o, to_hip(stream), nullptr);
}
