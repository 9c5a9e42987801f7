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
// Pass 2 (resolve): the listed tiles are recomputed in float64 (after an
// overflow every tile that can reach the band), giving the exact extreme and
// the smallest index within tie_tol of it, and the flags.  The float64 mode
// does this with one wavefront per query; the sorted float32 sweep resolves
// its own queries at its end, one lane per query, and leaves only the
// queries whose lists overflowed to a wavefront each.
//
// float32 mode runs pass 1 on spatially sorted data (Morton order of samples
// and of queries, so a tile and a work-group's 256 queries are compact
// boxes).  For a tile whose box is far from the work-group's query box the
// squared distances come from the matrix cores as one product per 16x16
// block, |p - q|^2 = |a|^2 - 2 a.b + |b|^2 with a = p - c, b = q - c and c the
// query box centre (v_mfma_f32_16x16x4f32: A = (-2a, |a|^2) per sample,
// B = (b, 1) per query, C = |b|^2); near tiles use the direct float32
// formula.  The far tiles' extra rounding is bounded from the data's extent
// and the box separation, and the candidate band eps (computed on the device
// from the data's magnitudes) covers both paths, so the float64 resolve sees
// every sample that can reach the tie band.
#include "common.h"

#include <hipcub/hipcub.hpp>

#include <cfloat>
#include <mutex>
#include <cmath>

namespace sdfi {

namespace {

constexpr int BT = 256;    // threads per sweep work-group
constexpr int TILE = 256;  // samples per LDS tile
constexpr int LIST = 8;    // candidate tiles kept per query and side
constexpr int BLK = 16;    // samples per block (one 16-row slice of a tile's matrix product)
constexpr uint32_t OVERFLOW_BIT = 0x80000000u;

template <typename T>
struct Pt4 {
    T x, y, z, s;
};


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

// note_tile on a work-group's lists kept in LDS: entry e of side `side` of
// local query `lq` at [side][e][lq]
__device__ inline void note_tile_lds(int side, int lq, int tile, float tv, float &run, uint32_t &cnt, float eps,
                                     int32_t (*lt)[LIST][256], float (*lv)[LIST][256]) {
    bool near = side == 0 ? (tv >= run - eps) : (tv <= run + eps);
    if (!near) return;
    if (side == 0 ? tv > run : tv < run) run = tv;
    if (cnt & OVERFLOW_BIT) return;
    if (cnt == LIST) {
        uint32_t k = 0;
        for (uint32_t e = 0; e < LIST; ++e) {
            const float v = lv[side][e][lq];
            const bool keep = side == 0 ? (v >= run - eps) : (v <= run + eps);
            if (keep) {
                lv[side][k][lq] = v;
                lt[side][k][lq] = lt[side][e][lq];
                ++k;
            }
        }
        cnt = k;
        if (cnt == LIST) {
            cnt = OVERFLOW_BIT;
            return;
        }
    }
    lt[side][cnt][lq] = tile;
    lv[side][cnt][lq] = tv;
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

struct BoundsOut {
    double *lo, *hi;
    int32_t *argmax, *argmin;
    uint32_t *flags;
};

// Outputs of query qi from its exact extremes, the smallest indices within
// their tie bands (INT64_MAX: none), the bands' populations and the values of
// the two indexed samples.
__device__ inline void write_query(int64_t qi, double lo, double hi, int64_t a, int64_t b, int tied_lo, int tied_hi,
                                   double s_a, double s_b, int64_t n, double tol, double tie, const BoundsOut &out) {
    // no candidate at all only happens with NaN inputs: report index -1
    const bool have_a = a >= 0 && a < n, have_b = b >= 0 && b < n;
    out.lo[qi] = lo;
    out.hi[qi] = hi;
    out.argmax[qi] = have_a ? (int32_t)a : -1;
    out.argmin[qi] = have_b ? (int32_t)b : -1;
    uint32_t f = 0;
    if (lo > hi + tol) f |= SDFI_FLAG_INFEASIBLE;
    if (lo > tol) f |= SDFI_FLAG_INSIDE_POS;
    if (hi < -tol) f |= SDFI_FLAG_INSIDE_NEG;
    if (tied_lo > 1) f |= SDFI_FLAG_TIE_LO;
    if (tied_hi > 1) f |= SDFI_FLAG_TIE_HI;
    if (have_b && sign_class(hi, tie) * sign_class(s_b, tie) < 0) f |= SDFI_FLAG_HI_OPPOSITE;
    if (have_a && sign_class(lo, tie) * sign_class(s_a, tie) < 0) f |= SDFI_FLAG_LO_OPPOSITE;
    out.flags[qi] = f;
}

// float32 value of one pair (the sweep's direct formula) within eps of the
// float32 extreme `run` of its side
__device__ inline bool near32(float4 p, const float *qf, int side, float run, float eps) {
    const float dx = qf[0] - p.x, dy = qf[1] - p.y, dz = qf[2] - p.z;
    const float d = __builtin_amdgcn_sqrtf(dx * dx + dy * dy + dz * dz);
    return side == 0 ? (p.w - d >= run - eps) : (p.w + d <= run + eps);
}

// Float64 mode, one wavefront per query: the listed tiles (every tile after
// an overflow) in float64, the exact extreme, the smallest index within the
// tie band and the band's population.
template <typename T>
__global__ __launch_bounds__(256) void resolve_kernel(const double *__restrict__ samples, int64_t n,
                                                      const double *__restrict__ queries, int64_t m, T eps,
                                                      SweepOut<T> o, double tol, double tie, BoundsOut out,
                                                      int64_t *overflows) {
    const int64_t qi = (int64_t)blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
    if (qi >= m) return;
    const int lane = threadIdx.x & 63;
    const double q[3] = {queries[3 * qi], queries[3 * qi + 1], queries[3 * qi + 2]};
    double ext[2];
    int64_t arg[2];
    int tied[2];
    for (int side = 0; side < 2; ++side) {
        const uint32_t cnt = o.count[2 * qi + side];
        const bool full = (cnt & OVERFLOW_BIT) != 0;
        const T run = o.run[2 * qi + side];
        const int64_t lb = (qi * 2 + side) * LIST;
        const int nt = full ? (int)((n + TILE - 1) / TILE) : (int)cnt;
        auto for_samples = [&](auto &&fn) {
            for (int e = 0; e < nt; ++e) {
                int t = e;
                if (!full) {
                    const T v = o.vals[lb + e];
                    if (!(side == 0 ? (v >= run - eps) : (v <= run + eps))) continue;
                    t = o.tiles[lb + e];
                }
                for (int r = 0; r < TILE / 64; ++r) {
                    const int64_t i = (int64_t)t * TILE + lane + 64 * r;
                    if (i < n) fn(i, pair_val(samples + 4 * i, q, side));
                }
            }
        };
        double best = side == 0 ? -INFINITY : INFINITY;
        for_samples([&](int64_t, double v) { best = side == 0 ? fmax(best, v) : fmin(best, v); });
        best = side == 0 ? wave_max(best) : wave_min(best);
        int64_t first = INT64_MAX;
        int inband = 0;
        for_samples([&](int64_t i, double v) {
            if (side == 0 ? (v >= best - tie) : (v <= best + tie)) {
                ++inband;
                first = i < first ? i : first;
            }
        });
        ext[side] = best;
        arg[side] = wave_min_i64(first);
        tied[side] = wave_sum(inband);
        if (full && lane == 0) atomicAdd((unsigned long long *)overflows, 1ull);
    }
    if (lane == 0) {
        const double s_a = arg[0] >= 0 && arg[0] < n ? samples[4 * arg[0] + 3] : 0.0;
        const double s_b = arg[1] >= 0 && arg[1] < n ? samples[4 * arg[1] + 3] : 0.0;
        write_query(qi, ext[0], ext[1], arg[0], arg[1], tied[0], tied[1], s_a, s_b, n, tol, tie, out);
    }
}

constexpr int RL_W = 16;  // wavefronts per query of the overflow resolve

// The slots listed by the sorted sweep (queries whose candidate lists
// overflowed), one work-group of RL_W wavefronts per query: the tiles of a
// side (its list, or after an overflow every tile that can reach the band by
// the tile test) are dealt out to the wavefronts, and the extreme, the
// smallest index within the tie band and the band's population are reduced
// over the work-group.  A fixed grid strides over the list, whose length is
// read on the device (zero: every work-group exits at once).
__global__ __launch_bounds__(RL_W * 64) void resolve_list_kernel(
    const double *__restrict__ samples, int64_t n, const double *__restrict__ queries,
    const float *__restrict__ eps_dev, SweepOut<float> o, double tol, double tie, BoundsOut out, int64_t *overflows,
    const int32_t *__restrict__ list, const unsigned long long *__restrict__ list_len,
    const int32_t *__restrict__ sperm, const int32_t *__restrict__ qperm, const float4 *__restrict__ ps32,
    const float4 *__restrict__ tbox) {
    __shared__ double rd[RL_W];
    __shared__ int64_t ri[RL_W];
    __shared__ int rc[RL_W];
    const int64_t len = (int64_t)*list_len;
    const float eps = *eps_dev;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int ntiles = (int)((n + TILE - 1) / TILE);
    for (int64_t k = blockIdx.x; k < len; k += gridDim.x) {
        const int64_t li = list[k];
        const int64_t qi = qperm[li];
        const float qf[3] = {(float)queries[3 * qi], (float)queries[3 * qi + 1], (float)queries[3 * qi + 2]};
        const double q[3] = {queries[3 * qi], queries[3 * qi + 1], queries[3 * qi + 2]};
        double ext[2];
        int64_t arg[2];
        int tied[2];
        for (int side = 0; side < 2; ++side) {
            const uint32_t cnt = o.count[2 * li + side];
            const bool full = (cnt & OVERFLOW_BIT) != 0;
            const float run = o.run[2 * li + side];
            const int64_t lb = (li * 2 + side) * LIST;
            // this wavefront's share of the side's tiles
            auto for_tiles = [&](auto &&fn) {
                if (!full) {
                    for (int e = w; e < (int)cnt; e += RL_W) {
                        const float v = o.vals[lb + e];
                        if (side == 0 ? (v >= run - eps) : (v <= run + eps)) fn(o.tiles[lb + e]);
                    }
                } else {
                    for (int c0 = 64 * w; c0 < ntiles; c0 += 64 * RL_W) {
                        const int t = c0 + lane;
                        bool reach = false;
                        if (t < ntiles) {
                            const float4 tl = tbox[2 * t], th = tbox[2 * t + 1];
                            const float gx = fmaxf(0.0f, fmaxf(tl.x - qf[0], qf[0] - th.x));
                            const float gy = fmaxf(0.0f, fmaxf(tl.y - qf[1], qf[1] - th.y));
                            const float gz = fmaxf(0.0f, fmaxf(tl.z - qf[2], qf[2] - th.z));
                            const float gap = sqrtf(gx * gx + gy * gy + gz * gz) * (1.0f - 8.0f * 5.9604645e-8f);
                            reach = side == 0 ? !(th.w - gap < run - 2.0f * eps) : !(tl.w + gap > run + 2.0f * eps);
                        }
                        for (unsigned long long mk = __ballot(reach); mk; mk &= mk - 1)
                            fn(c0 + __builtin_ctzll(mk));
                    }
                }
            };
            double best = side == 0 ? -INFINITY : INFINITY;
            for_tiles([&](int t) {
                for (int r = 0; r < TILE / 64; ++r) {
                    const int64_t i = (int64_t)t * TILE + lane + 64 * r;
                    if (i < n && near32(ps32[i], qf, side, run, eps)) {
                        const double v = pair_val(samples + 4 * (int64_t)sperm[i], q, side);
                        best = side == 0 ? fmax(best, v) : fmin(best, v);
                    }
                }
            });
            best = side == 0 ? wave_max(best) : wave_min(best);
            if (lane == 0) rd[w] = best;
            __syncthreads();
            best = rd[0];
            for (int j = 1; j < RL_W; ++j) best = side == 0 ? fmax(best, rd[j]) : fmin(best, rd[j]);
            int64_t first = INT64_MAX;
            int inband = 0;
            for_tiles([&](int t) {
                for (int r = 0; r < TILE / 64; ++r) {
                    const int64_t i = (int64_t)t * TILE + lane + 64 * r;
                    if (i < n && near32(ps32[i], qf, side, run, eps)) {
                        const int64_t oi = sperm[i];
                        const double v = pair_val(samples + 4 * oi, q, side);
                        if (side == 0 ? (v >= best - tie) : (v <= best + tie)) {
                            ++inband;
                            first = oi < first ? oi : first;
                        }
                    }
                }
            });
            first = wave_min_i64(first);
            inband = wave_sum(inband);
            if (lane == 0) {
                ri[w] = first;
                rc[w] = inband;
            }
            __syncthreads();
            first = ri[0];
            inband = rc[0];
            for (int j = 1; j < RL_W; ++j) {
                first = ri[j] < first ? ri[j] : first;
                inband += rc[j];
            }
            __syncthreads();  // rd, ri, rc are reused
            ext[side] = best;
            arg[side] = first;
            tied[side] = inband;
            if (full && threadIdx.x == 0) atomicAdd((unsigned long long *)overflows, 1ull);
        }
        if (threadIdx.x == 0) {
            const double s_a = arg[0] >= 0 && arg[0] < n ? samples[4 * arg[0] + 3] : 0.0;
            const double s_b = arg[1] >= 0 && arg[1] < n ? samples[4 * arg[1] + 3] : 0.0;
            write_query(qi, ext[0], ext[1], arg[0], arg[1], tied[0], tied[1], s_a, s_b, n, tol, tie, out);
        }
    }
}

// ---- float32 sweep over spatially sorted data ----

constexpr int MQ = 256;             // queries per work-group of the sorted sweep (4 wavefronts x 64)
static_assert(MQ == 256, "the LDS candidate lists are laid out for 256 queries");
constexpr int EXT_BLOCKS = 256;     // partial reductions of the extent
constexpr int RESOLVE_LIST_BLOCKS = 256;  // work-groups of the overflow resolve
constexpr float U32 = 5.9604645e-8f;  // unit roundoff of float32

// Extent of samples and queries and the constants derived from it.
struct Extent {
    float lo[4], hi[4];  // bounding box (float32 coordinates)
    float mc, ms;        // largest |coordinate| and |value|
    float eps;           // candidate band of the sweep
    float rho_cap;       // largest query-box radius that may use the matrix path
    float delta0;        // smallest box gap of a matrix-path tile
    float pad[3];
};

struct ExtPart {
    float lo[3], hi[3], mc, ms;
};

__device__ inline float wred_min(float v) {
    for (int o = 32; o > 0; o >>= 1) v = fminf(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ inline float wred_max(float v) {
    for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
    return v;
}

// per-block partial extents over samples (n x 4) and queries (m x 3)
__global__ __launch_bounds__(256) void extent_partial_kernel(const double *__restrict__ samples, int64_t n,
                                                             const double *__restrict__ queries, int64_t m,
                                                             ExtPart *parts) {
    __shared__ float red[8][4];
    float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    float mc = 0.0f, ms = 0.0f;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n + m; i += stride) {
        const double *p = i < n ? samples + 4 * i : queries + 3 * (i - n);
        for (int k = 0; k < 3; ++k) {
            const float x = (float)p[k];
            lo[k] = fminf(lo[k], x);
            hi[k] = fmaxf(hi[k], x);
            mc = fmaxf(mc, fabsf(x));
        }
        if (i < n) ms = fmaxf(ms, fabsf((float)p[3]));
    }
    float v[8] = {lo[0], lo[1], lo[2], hi[0], hi[1], hi[2], mc, ms};
    for (int k = 0; k < 8; ++k) v[k] = k < 3 ? wred_min(v[k]) : wred_max(v[k]);
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    __shared__ float wv[4][8];
    if (lane == 0)
        for (int k = 0; k < 8; ++k) wv[w][k] = v[k];
    __syncthreads();
    if (threadIdx.x == 0) {
        ExtPart e;
        for (int k = 0; k < 3; ++k) {
            e.lo[k] = fminf(fminf(wv[0][k], wv[1][k]), fminf(wv[2][k], wv[3][k]));
            e.hi[k] = fmaxf(fmaxf(wv[0][3 + k], wv[1][3 + k]), fmaxf(wv[2][3 + k], wv[3][3 + k]));
        }
        e.mc = fmaxf(fmaxf(wv[0][6], wv[1][6]), fmaxf(wv[2][6], wv[3][6]));
        e.ms = fmaxf(fmaxf(wv[0][7], wv[1][7]), fmaxf(wv[2][7], wv[3][7]));
        parts[blockIdx.x] = e;
    }
    (void)red;
}

// Final extent and the band.  Error of one float32 pair value s - d or s + d
// against its float64 value (u the unit roundoff, Mc/Ms the largest
// coordinate/value magnitudes, E the extent's diagonal):
//   direct formula: inputs rounded (2 sqrt3 u Mc on d, u Ms on s), three
//     differences, squares and sum (5u relative on d^2), sqrt (1 ulp) and the
//     final add: at most u (2 Ms + 23 Mc);
//   matrix path: the same input rounding plus the product form of d^2, whose
//     error is at most 8u (|a| + |b|)^2 <= 8u (d + 2 rho)^2 with rho the query
//     box radius; for a tile at box gap d >= max(delta0, 2 rho) and d <= E it
//     perturbs d by at most 8u (E + 6 rho) (+ rounding of the centring and of
//     the sqrt), so with rho <= rho_cap = E/16 the value errs by at most
//     u (11 E + 50 rho_cap + 7 Mc + 2 Ms).
// Two values may err in opposite directions: eps = tie + 2.5 x the larger.
__global__ void extent_final_kernel(const ExtPart *parts, int np, double tie, Extent *out) {
    if (threadIdx.x != 0) return;
    Extent e;
    for (int k = 0; k < 3; ++k) {
        e.lo[k] = INFINITY;
        e.hi[k] = -INFINITY;
    }
    e.lo[3] = e.hi[3] = 0.0f;
    e.mc = e.ms = 0.0f;
    for (int i = 0; i < np; ++i) {
        for (int k = 0; k < 3; ++k) {
            e.lo[k] = fminf(e.lo[k], parts[i].lo[k]);
            e.hi[k] = fmaxf(e.hi[k], parts[i].hi[k]);
        }
        e.mc = fmaxf(e.mc, parts[i].mc);
        e.ms = fmaxf(e.ms, parts[i].ms);
    }
    float d2 = 0.0f;
    for (int k = 0; k < 3; ++k) d2 += (e.hi[k] - e.lo[k]) * (e.hi[k] - e.lo[k]);
    const float E = sqrtf(d2) * 1.0001f;
    e.rho_cap = E / 16.0f;
    e.delta0 = E / 64.0f;
    const float near_err = U32 * (2.0f * e.ms + 23.0f * e.mc);
    const float far_err = U32 * (11.0f * E + 50.0f * e.rho_cap + 7.0f * e.mc + 2.0f * e.ms);
    e.eps = (float)tie + 2.5f * fmaxf(near_err, far_err);
    e.pad[0] = e.pad[1] = e.pad[2] = 0.0f;
    *out = e;
}

__device__ inline uint32_t spread10(uint32_t v) {
    v &= 1023u;
    v = (v | (v << 16)) & 0x030000FFu;
    v = (v | (v << 8)) & 0x0300F00Fu;
    v = (v | (v << 4)) & 0x030C30C3u;
    v = (v | (v << 2)) & 0x09249249u;
    return v;
}

// Morton keys (10 bits per axis over the extent's box) of rows of `pts`
// (stride 3 or 4 doubles) and the identity permutation.
__global__ void morton_kernel(const double *__restrict__ pts, int stride, int64_t k, const Extent *ext,
                              uint32_t *keys, int32_t *idx) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= k) return;
    uint32_t c[3];
    for (int a = 0; a < 3; ++a) {
        const float span = ext->hi[a] - ext->lo[a];
        const float t = span > 0.0f ? ((float)pts[stride * i + a] - ext->lo[a]) / span : 0.0f;
        const float f = fminf(fmaxf(t * 1024.0f, 0.0f), 1023.0f);  // NaN -> 0
        c[a] = (uint32_t)f;
    }
    keys[i] = spread10(c[0]) | (spread10(c[1]) << 1) | (spread10(c[2]) << 2);
    idx[i] = (int32_t)i;
}

// float32 copy of the samples in sorted order
__global__ void pack_sorted_kernel(const double *__restrict__ samples, const int32_t *__restrict__ perm, int64_t n,
                                   float4 *__restrict__ out, double *__restrict__ out64) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) {
        const double *p = samples + 4 * (int64_t)perm[i];
        const double x = p[0], y = p[1], z = p[2], v = p[3];
        out[i] = make_float4((float)x, (float)y, (float)z, (float)v);
        out64[4 * i] = x;
        out64[4 * i + 1] = y;
        out64[4 * i + 2] = z;
        out64[4 * i + 3] = v;
    }
}

// What the sorted sweep needs to resolve its queries itself.
struct Fused {
    const double *ps64;    // float64 samples in tile order (x, y, z, s)
    const int32_t *sperm;  // tile order -> input index
    double tol, tie;
    BoundsOut out;
    int32_t *ovf_list;               // slots whose lists overflowed, for resolve_list_kernel
    unsigned long long *ovf_len;
};

// Exact extreme of one side of one query by one lane, over the tiles its list
// keeps (entries within eps of the float32 extreme `run`): samples whose
// float32 value (the direct formula) is within eps of `run` get their
// float64 value; the smallest input index within `tie` of the float64
// extreme, the band's population and that sample's value follow.  The first
// two survivors are kept in registers for the band count; with more, the
// kept tiles are screened again.
// List entries are tile indices, or with `packed` tile | (block mask << 16):
// the blocks of BLK samples that can hold a survivor.
__device__ inline int64_t entry_tile(int32_t ent, bool packed) { return packed ? (ent & 0xFFFF) : ent; }
__device__ inline uint32_t entry_blocks(int32_t ent, bool packed) {
    return packed ? ((uint32_t)ent >> 16) : 0xFFFFu;
}

__device__ inline void resolve_lane(int side, const float *qf, const double *q, float run, float eps, uint32_t cnt,
                                    int lq, const int32_t (*lt)[LIST][256], const float (*lv)[LIST][256],
                                    bool packed, const float4 *__restrict__ ps, const float4 *__restrict__ bbox,
                                    int64_t n, const Fused &F, double &best, int64_t &first, int &inband,
                                    double &s_first) {
    best = side == 0 ? -INFINITY : INFINITY;
    int nc = 0;
    int64_t c0 = 0, c1 = 0;
    for (uint32_t e = 0; e < cnt; ++e) {
        const float v = lv[side][e][lq];
        if (!(side == 0 ? (v >= run - eps) : (v <= run + eps))) continue;
        const int32_t ent = lt[side][e][lq];
        const int64_t tb = entry_tile(ent, packed) * TILE;
        const int tlen = (int)min((int64_t)TILE, n - tb);
        for (uint32_t bm = entry_blocks(ent, packed) & ((1u << ((tlen + BLK - 1) / BLK)) - 1u); bm; bm &= bm - 1) {
            const int bk = __builtin_ctz(bm);
            if (!packed) {
                // without the sweep's block mask: a block whose box and value
                // range keep every pair with q out of the screen's band is
                // skipped (it holds no survivor)
                const int64_t k = tb / BLK + bk;
                const float4 bl = bbox[2 * k], bh = bbox[2 * k + 1];
                const float gx = fmaxf(0.0f, fmaxf(bl.x - qf[0], qf[0] - bh.x));
                const float gy = fmaxf(0.0f, fmaxf(bl.y - qf[1], qf[1] - bh.y));
                const float gz = fmaxf(0.0f, fmaxf(bl.z - qf[2], qf[2] - bh.z));
                const float g = sqrtf(gx * gx + gy * gy + gz * gz) * (1.0f - 8.0f * 5.9604645e-8f);
                if (side == 0 ? (bh.w - g < run - 2.0f * eps) : (bl.w + g > run + 2.0f * eps)) continue;
            }
            const int64_t base = tb + bk * BLK;
            const int len = (int)min((int64_t)BLK, n - base);
        for (int j0 = 0; j0 < len; j0 += 4) {
            float4 p4[4];  // four loads in flight
#pragma unroll
            for (int r = 0; r < 4; ++r) p4[r] = ps[base + min(j0 + r, len - 1)];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                if (j0 + r >= len || !near32(p4[r], qf, side, run, eps)) continue;
                const int64_t i = base + j0 + r;
                const double v64 = pair_val(F.ps64 + 4 * i, q, side);
                best = side == 0 ? fmax(best, v64) : fmin(best, v64);
                if (nc == 0) c0 = i;
                if (nc == 1) c1 = i;
                ++nc;
            }
        }
        }
    }
    first = INT64_MAX;
    inband = 0;
    s_first = 0.0;
    auto band = [&](int64_t i) {
        const double v64 = pair_val(F.ps64 + 4 * i, q, side);
        if (side == 0 ? (v64 >= best - F.tie) : (v64 <= best + F.tie)) {
            ++inband;
            const int64_t oi = F.sperm[i];
            if (oi < first) {
                first = oi;
                s_first = F.ps64[4 * i + 3];
            }
        }
    };
    if (nc <= 2) {
        if (nc > 0) band(c0);
        if (nc > 1) band(c1);
        return;
    }
    for (uint32_t e = 0; e < cnt; ++e) {
        const float v = lv[side][e][lq];
        if (!(side == 0 ? (v >= run - eps) : (v <= run + eps))) continue;
        const int64_t base = entry_tile(lt[side][e][lq], packed) * TILE;
        const int len = (int)min((int64_t)TILE, n - base);
        for (int j = 0; j < len; ++j)
            if (near32(ps[base + j], qf, side, run, eps)) band(base + j);
    }
}

// box and value range of each tile of the sorted samples: tbox[2t] = (low
// corner, smallest value), tbox[2t+1] = (high corner, largest value)
__global__ __launch_bounds__(TILE) void tile_box_kernel(const float4 *__restrict__ ps, int64_t n, float4 *tbox) {
    __shared__ float wv[TILE / 64][8];
    const int64_t i = (int64_t)blockIdx.x * TILE + threadIdx.x;
    float v[8] = {INFINITY, INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY, -INFINITY};
    if (i < n) {
        const float4 p = ps[i];
        v[0] = v[4] = p.x;
        v[1] = v[5] = p.y;
        v[2] = v[6] = p.z;
        v[3] = v[7] = p.w;
    }
    for (int k = 0; k < 8; ++k) v[k] = k < 4 ? wred_min(v[k]) : wred_max(v[k]);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0)
        for (int k = 0; k < 8; ++k) wv[w][k] = v[k];
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int ww = 1; ww < TILE / 64; ++ww)
            for (int k = 0; k < 8; ++k) wv[0][k] = k < 4 ? fminf(wv[0][k], wv[ww][k]) : fmaxf(wv[0][k], wv[ww][k]);
        tbox[2 * blockIdx.x] = make_float4(wv[0][0], wv[0][1], wv[0][2], wv[0][3]);
        tbox[2 * blockIdx.x + 1] = make_float4(wv[0][4], wv[0][5], wv[0][6], wv[0][7]);
    }
}

// box and value range of each block of BLK sorted samples, laid out like tbox
__global__ void block_box_kernel(const float4 *__restrict__ ps, int64_t n, float4 *bbox) {
    const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (k * BLK >= n) return;
    float4 lo = make_float4(INFINITY, INFINITY, INFINITY, INFINITY);
    float4 hi = make_float4(-INFINITY, -INFINITY, -INFINITY, -INFINITY);
    const int cnt = (int)min((int64_t)BLK, n - k * BLK);
    for (int j = 0; j < cnt; ++j) {
        const float4 p = ps[k * BLK + j];
        lo = make_float4(fminf(lo.x, p.x), fminf(lo.y, p.y), fminf(lo.z, p.z), fminf(lo.w, p.w));
        hi = make_float4(fmaxf(hi.x, p.x), fmaxf(hi.y, p.y), fmaxf(hi.z, p.z), fmaxf(hi.w, p.w));
    }
    bbox[2 * k] = lo;
    bbox[2 * k + 1] = hi;
}

// Can a pair of a point in box [ql, qh] with a sample of the box/range
// (bl, bh) have s - d >= lo - 2 eps or s + d <= hi + 2 eps?  False only when
// every such pair is below lo - 2 eps and above hi + 2 eps (the gap is taken
// a few float32 roundings short, so the test errs towards true).
__device__ inline bool box_reach(const float *ql, const float *qh, float4 bl, float4 bh, float lo, float hi,
                                 float eps) {
    const float gx = fmaxf(0.0f, fmaxf(bl.x - qh[0], ql[0] - bh.x));
    const float gy = fmaxf(0.0f, fmaxf(bl.y - qh[1], ql[1] - bh.y));
    const float gz = fmaxf(0.0f, fmaxf(bl.z - qh[2], ql[2] - bh.z));
    const float g = sqrtf(gx * gx + gy * gy + gz * gz) * (1.0f - 8.0f * 5.9604645e-8f);
    return !((bh.w - g < lo - 2.0f * eps) && (bl.w + g > hi + 2.0f * eps));
}

typedef float f32x4 __attribute__((ext_vector_type(4)));

// One work-group: 256 consecutive queries of the sorted order (lane l of
// wavefront w owns sorted query 256 b + 64 w + l), all sample tiles.
__global__ __launch_bounds__(MQ) void sweep_sorted_kernel(const float4 *__restrict__ ps, int n,
                                                          const float4 *__restrict__ tbox,
                                                          const double *__restrict__ queries,
                                                          const int32_t *__restrict__ qperm, int64_t m,
                                                          const Extent *__restrict__ ext, SweepOut<float> o,
                                                          unsigned long long *__restrict__ skipped, Fused F,
                                                          const float4 *__restrict__ bbox) {
    // a tile is either near (raw samples (x, y, z, s)) or far ((-2 a, |a|^2) with
    // a = p - c, values apart): the two layouts share one LDS array
    __shared__ float4 tilebuf[TILE];
    __shared__ float sv[TILE];    // tile values (far tiles)
    float4 *const raw = tilebuf;
    float4 *const cen = tilebuf;
    __shared__ float wbox[MQ / 64][6];
    __shared__ unsigned long long wneed[2][MQ / 64];  // far tiles of a chunk each wavefront needs (two phases)
    __shared__ int32_t ltile[2][LIST][MQ];  // candidate lists of the work-group's queries
    __shared__ float lval[2][LIST][MQ];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int64_t sq = (int64_t)blockIdx.x * MQ + tid;
    const bool valid = sq < m;
    const int64_t qi = qperm[valid ? sq : (int64_t)blockIdx.x * MQ];  // original index (a stand-in when past m)
    const float qx = (float)queries[3 * qi], qy = (float)queries[3 * qi + 1], qz = (float)queries[3 * qi + 2];
    // the work-group's query box, its centre and radius
    float v[6] = {qx, qy, qz, qx, qy, qz};
    for (int k = 0; k < 6; ++k) v[k] = k < 3 ? wred_min(v[k]) : wred_max(v[k]);
    if (lane == 0)
        for (int k = 0; k < 6; ++k) wbox[w][k] = v[k];
    __syncthreads();
    float qlo[3], qhi[3];
    for (int k = 0; k < 3; ++k) {
        qlo[k] = fminf(fminf(wbox[0][k], wbox[1][k]), fminf(wbox[2][k], wbox[3][k]));
        qhi[k] = fmaxf(fmaxf(wbox[0][3 + k], wbox[1][3 + k]), fmaxf(wbox[2][3 + k], wbox[3][3 + k]));
    }
    const float cx = 0.5f * (qlo[0] + qhi[0]), cy = 0.5f * (qlo[1] + qhi[1]), cz = 0.5f * (qlo[2] + qhi[2]);
    float r2 = 0.0f;
    for (int k = 0; k < 3; ++k) r2 += (qhi[k] - qlo[k]) * (qhi[k] - qlo[k]);
    const float rho = 0.5f * sqrtf(r2) * 1.0001f;
    const float eps = ext->eps;
    const bool far_ok = rho <= ext->rho_cap;
    const float delta = fmaxf(ext->delta0, 2.0f * rho);
    // matrix operands of this wave's queries: column block cb holds local
    // queries 16 cb + (lane & 15); this lane supplies component lane >> 4
    const float bx = qx - cx, by = qy - cy, bz = qz - cz;
    const float bb = bx * bx + by * by + bz * bz;
    float B[4];
    f32x4 C[4];
#pragma unroll
    for (int cb = 0; cb < 4; ++cb) {
        const int src = 16 * cb + (lane & 15);
        const float x_ = __shfl(bx, src, 64), y_ = __shfl(by, src, 64), z_ = __shfl(bz, src, 64);
        const float b2 = __shfl(bb, src, 64);
        const int k = lane >> 4;
        B[cb] = k == 0 ? x_ : (k == 1 ? y_ : (k == 2 ? z_ : 1.0f));
        C[cb] = f32x4{b2, b2, b2, b2};
    }
    float run_lo = -INFINITY, run_hi = INFINITY;
    uint32_t clo = 0, chi = 0;
    const int ntiles = (n + TILE - 1) / TILE;
    float wlo_all = -INFINITY, whi_all = INFINITY;  // the wavefront's lowest / highest running extremes
    // list entries carry a mask of the tile's blocks that can hold a sample of
    // the final band (packed with the tile index when that fits 16 bits)
    const bool packed = ntiles <= 65536;
    // valid queries of this wavefront (stand-in lanes past m are not counted)
    const int vl = (int)min((int64_t)64, max((int64_t)0, m - ((int64_t)blockIdx.x * MQ + 64 * w)));
    unsigned long long nskipped = 0;  // query x sample pairs this wavefront ruled out
    float wql[3], wqh[3];             // this wavefront's query box
    for (int k = 0; k < 3; ++k) {
        wql[k] = wbox[w][k];
        wqh[k] = wbox[w][3 + k];
    }
    int phase = 0;       // alternates per chunk, so that need masks are not rewritten before all waves read them
    // One tile: stage it in LDS, reduce it (the matrix path for far tiles, the
    // direct formula for near ones), note it in the candidate lists.  `act`:
    // this wavefront needs the tile (a far tile it ruled out is not reduced).
    // Called with the same (t, far) by all wavefronts of the work-group.
    auto sweep_tile = [&](int t, bool far, bool act) {
        const int cnt = min(TILE, n - t * TILE);
        // blocks of a far tile this wavefront needs: one test per lane, the
        // tile test at block size
        unsigned long long bneed = 0;
        if (far && act) {
            bool nb = false;
            if (lane < TILE / BLK) {
                const int64_t k = (int64_t)t * (TILE / BLK) + lane;
                nb = box_reach(wql, wqh, bbox[2 * k], bbox[2 * k + 1], wlo_all, whi_all, eps);
            }
            bneed = __ballot(nb);
            nskipped += (unsigned long long)(TILE / BLK - __popcll(bneed)) * BLK * vl;
        } else if (!far) {
            // the same for a near tile (possibly the short last one), against
            // the extremes as they stand
            const int nblk = (cnt + BLK - 1) / BLK;
            bool nb = false;
            if (lane < nblk) {
                const int64_t k = (int64_t)t * (TILE / BLK) + lane;
                nb = box_reach(wql, wqh, bbox[2 * k], bbox[2 * k + 1], wlo_all, whi_all, eps);
            }
            bneed = __ballot(nb);
            int used = __popcll(bneed) * BLK;
            if ((bneed >> (nblk - 1)) & 1ull) used -= nblk * BLK - cnt;
            nskipped += (unsigned long long)(cnt - used) * vl;
        }
        __syncthreads();
        if (tid < cnt) {
            const float4 p = ps[(int64_t)t * TILE + tid];
            if (far) {
                const float ax = p.x - cx, ay = p.y - cy, az = p.z - cz;
                cen[tid] = make_float4(-2.0f * ax, -2.0f * ay, -2.0f * az, ax * ax + ay * ay + az * az);
                sv[tid] = p.w;
            } else {
                raw[tid] = p;
            }
        }
        __syncthreads();
        float tlo = -INFINITY, thi = INFINITY;
        // blocks that can hold a sample within 2 eps of this tile's extreme for
        // this lane's query (a superset: the final screen keeps only samples
        // within eps of the final extreme, which is at least the tile's)
        uint32_t mlo = 0, mhi = 0;
        if (far && act) {
            // Running extremes of the four query columns this lane holds, widened
            // by 2 eps.  A pair with d >= max(s - rl, rh - s) has s - d <= rl and
            // s + d >= rh: it can neither be near either extreme nor move it, so a
            // 16 x 16 block where every lane has min d^2 >= T^2 (T built from its
            // four samples' largest and smallest value) needs no square root.
            float rl[4], rh[4];
#pragma unroll
            for (int cb = 0; cb < 4; ++cb) {
                const int src = 16 * cb + (lane & 15);
                rl[cb] = __shfl(run_lo, src, 64) - 2.0f * eps;
                rh[cb] = __shfl(run_hi, src, 64) + 2.0f * eps;
            }
            float lo4[4] = {-INFINITY, -INFINITY, -INFINITY, -INFINITY};
            float hi4[4] = {INFINITY, INFINITY, INFINITY, INFINITY};
            const float *cenf = reinterpret_cast<const float *>(cen);
#pragma unroll 2
            for (unsigned long long bm = bneed; bm; bm &= bm - 1) {
                const int b = __builtin_ctzll(bm);
                // A[i][k]: sample 16 b + i, component k (this lane: i = lane & 15, k = lane >> 4)
                const float a = cenf[4 * (16 * b + (lane & 15)) + (lane >> 4)];
                // rows of the product held by this lane: samples 16 b + 4 (lane >> 4) + 0..3
                const float4 s4 = *reinterpret_cast<const float4 *>(&sv[16 * b + 4 * (lane >> 4)]);
                f32x4 D[4];
#pragma unroll
                for (int cb = 0; cb < 4; ++cb)
                    D[cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, B[cb], C[cb], 0, 0, 0);
                const float smax = fmaxf(fmaxf(s4.x, s4.y), fmaxf(s4.z, s4.w));
                const float smin = fminf(fminf(s4.x, s4.y), fminf(s4.z, s4.w));
                int need = 0;
#pragma unroll
                for (int cb = 0; cb < 4; ++cb) {
                    const float dmin2 = fminf(fminf(D[cb][0], D[cb][1]), fminf(D[cb][2], D[cb][3]));
                    const float T = fmaxf(fmaxf(smax - rl[cb], rh[cb] - smin), 0.0f);
                    need |= dmin2 < T * T;
                }
                if (__any(need)) {
                    // a block the group test passes over holds no sample of
                    // either band; the computed ones are kept for both sides
                    mlo |= 1u << b;
                    mhi |= 1u << b;
#pragma unroll
                    for (int cb = 0; cb < 4; ++cb) {
                        const float d0 = __builtin_amdgcn_sqrtf(fabsf(D[cb][0]));
                        const float d1 = __builtin_amdgcn_sqrtf(fabsf(D[cb][1]));
                        const float d2 = __builtin_amdgcn_sqrtf(fabsf(D[cb][2]));
                        const float d3 = __builtin_amdgcn_sqrtf(fabsf(D[cb][3]));
                        lo4[cb] = fmaxf(fmaxf(lo4[cb], s4.x - d0), s4.y - d1);
                        lo4[cb] = fmaxf(fmaxf(lo4[cb], s4.z - d2), s4.w - d3);
                        hi4[cb] = fminf(fminf(hi4[cb], s4.x + d0), s4.y + d1);
                        hi4[cb] = fminf(fminf(hi4[cb], s4.z + d2), s4.w + d3);
                    }
                }
            }
            // combine the four row groups holding each query column
#pragma unroll
            for (int cb = 0; cb < 4; ++cb) {
                lo4[cb] = fmaxf(lo4[cb], __shfl_xor(lo4[cb], 16, 64));
                lo4[cb] = fmaxf(lo4[cb], __shfl_xor(lo4[cb], 32, 64));
                hi4[cb] = fminf(hi4[cb], __shfl_xor(hi4[cb], 16, 64));
                hi4[cb] = fminf(hi4[cb], __shfl_xor(hi4[cb], 32, 64));
            }
            // this lane's own query is local query `lane`: column block lane >> 4
            const int mine = lane >> 4;
            tlo = mine == 0 ? lo4[0] : (mine == 1 ? lo4[1] : (mine == 2 ? lo4[2] : lo4[3]));
            thi = mine == 0 ? hi4[0] : (mine == 1 ? hi4[1] : (mine == 2 ? hi4[2] : hi4[3]));
        } else if (!far) {
            for (unsigned long long bm = bneed; bm; bm &= bm - 1) {
                const int bk = __builtin_ctzll(bm);
                const int j0 = bk * BLK, j1 = min(j0 + BLK, cnt);
                float blo = -INFINITY, bhi = INFINITY;
                for (int j = j0; j < j1; ++j) {
                    const float4 p = raw[j];
                    const float dx = qx - p.x, dy = qy - p.y, dz = qz - p.z;
                    const float d = __builtin_amdgcn_sqrtf(dx * dx + dy * dy + dz * dz);
                    blo = fmaxf(blo, p.w - d);
                    bhi = fminf(bhi, p.w + d);
                }
                // bits set against the tile extreme so far stay valid as it grows
                tlo = fmaxf(tlo, blo);
                thi = fminf(thi, bhi);
                if (blo >= tlo - 2.0f * eps) mlo |= 1u << bk;
                if (bhi <= thi + 2.0f * eps) mhi |= 1u << bk;
            }
        }
        note_tile_lds(0, tid, packed ? (t | (int)(mlo << 16)) : t, tlo, run_lo, clo, eps, ltile, lval);
        note_tile_lds(1, tid, packed ? (t | (int)(mhi << 16)) : t, thi, run_hi, chi, eps, ltile, lval);
        if (!far) {  // the near tiles settle the extremes: keep the block test current
            wlo_all = wred_min(run_lo);
            whi_all = wred_max(run_hi);
        }
    };
    // The near tiles first (direct formula), so that
    // the running extremes are already close to final when the far tiles are
    // swept on the matrix path and its group test can skip most square roots.
    // Tiles are classified 64 at a time, one per lane.
    //
    // A far tile can be ruled out by a wavefront when every pair with its
    // queries has s - d < (lowest running lower extreme) - 2 eps and s + d >
    // (highest running upper extreme) + 2 eps: by the box gap g of the wave's
    // queries and the tile, when smax - g and smin + g clear those.  Such pairs
    // can neither move an extreme nor enter its band (the same margin as the
    // group test), so the results are those of the full sweep.  The work-group
    // stages only the tiles that one of its wavefronts needs, and a wavefront
    // reduces only the blocks of BLK samples that pass the same test at block
    // size (near tiles included, against the extremes as they stand: the
    // first near tiles are reduced whole).
    // Pass 0 takes the near tiles overlapping the work-group's box, pass 1 the
    // other near tiles (by then the block test prunes most of them), pass 2 the
    // far tiles.
    for (int pass = 0; pass < 3; ++pass) {
        for (int c0 = 0; c0 < ntiles; c0 += 64) {
            const int t = c0 + lane;
            bool in_pass = false, need = false;
            if (t < ntiles) {
                const int cnt = min(TILE, n - t * TILE);
                const float4 tl = tbox[2 * t], th = tbox[2 * t + 1];
                const float gx = fmaxf(0.0f, fmaxf(tl.x - qhi[0], qlo[0] - th.x));
                const float gy = fmaxf(0.0f, fmaxf(tl.y - qhi[1], qlo[1] - th.y));
                const float gz = fmaxf(0.0f, fmaxf(tl.z - qhi[2], qlo[2] - th.z));
                const float gap = sqrtf(gx * gx + gy * gy + gz * gz);
                const bool far = far_ok && cnt == TILE && gap > 0.0f && gap >= delta;
                in_pass = pass == 2 ? far : (!far && ((gap > 0.0f) == (pass == 1)));
                need = in_pass;
                if (in_pass && far) {
                    const float wx = fmaxf(0.0f, fmaxf(tl.x - wbox[w][3], wbox[w][0] - th.x));
                    const float wy = fmaxf(0.0f, fmaxf(tl.y - wbox[w][4], wbox[w][1] - th.y));
                    const float wz = fmaxf(0.0f, fmaxf(tl.z - wbox[w][5], wbox[w][2] - th.z));
                    const float wgap = sqrtf(wx * wx + wy * wy + wz * wz) * (1.0f - 8.0f * U32);
                    need = !((th.w - wgap < wlo_all - 2.0f * eps) && (tl.w + wgap > whi_all + 2.0f * eps));
                }
            }
            const unsigned long long inpass = __ballot(in_pass);  // the same in every wavefront
            const unsigned long long mine = __ballot(need);
            unsigned long long todo = inpass;
            if (pass == 2) {
                nskipped += (unsigned long long)__popcll(inpass & ~mine) * TILE * vl;
                if (lane == 0) wneed[phase][w] = mine;
                __syncthreads();
                todo = wneed[phase][0] | wneed[phase][1] | wneed[phase][2] | wneed[phase][3];
                phase ^= 1;
            }
            for (; todo; todo &= todo - 1) {
                const int k = __builtin_ctzll(todo);
                sweep_tile(c0 + k, pass == 2, ((mine >> k) & 1ull) != 0);
            }
            if (pass == 2) {
                wlo_all = wred_min(run_lo);
                whi_all = wred_max(run_hi);
            }
        }
    }
    // pairs ruled out without evaluation (stand-in lanes past m not counted)
    if (lane == 0 && nskipped) atomicAdd(skipped, nskipped);
    // Resolve here, one lane per query, unless a list overflowed: then the
    // lists and extremes leave in sorted order (slot sq) for resolve_list_kernel.
    if (valid) {
        if (((clo | chi) & OVERFLOW_BIT) == 0) {
            const float qf[3] = {qx, qy, qz};
            const double q[3] = {queries[3 * qi], queries[3 * qi + 1], queries[3 * qi + 2]};
            double lo, hi, s_a, s_b;
            int64_t a, b;
            int ta, tb;
            resolve_lane(0, qf, q, run_lo, eps, clo, tid, ltile, lval, packed, ps, bbox, n, F, lo, a, ta, s_a);
            resolve_lane(1, qf, q, run_hi, eps, chi, tid, ltile, lval, packed, ps, bbox, n, F, hi, b, tb, s_b);
            write_query(qi, lo, hi, a, b, ta, tb, s_a, s_b, n, F.tol, F.tie, F.out);
        } else {
            o.run[2 * sq] = run_lo;
            o.run[2 * sq + 1] = run_hi;
            for (int side = 0; side < 2; ++side) {
                const uint32_t c = side == 0 ? clo : chi;
                const float run = side == 0 ? run_lo : run_hi;
                // entries noted before the extreme settled may have left its band: drop them
                uint32_t k = 0;
                if (!(c & OVERFLOW_BIT)) {
                    for (uint32_t e = 0; e < c; ++e) {
                        const float v = lval[side][e][tid];
                        if (side == 0 ? (v >= run - eps) : (v <= run + eps)) {
                            o.tiles[(sq * 2 + side) * LIST + k] = (int32_t)entry_tile(ltile[side][e][tid], packed);
                            o.vals[(sq * 2 + side) * LIST + k] = v;
                            ++k;
                        }
                    }
                }
                o.count[2 * sq + side] = (c & OVERFLOW_BIT) ? c : k;
            }
            F.ovf_list[atomicAdd(F.ovf_len, 1ull)] = (int32_t)sq;
        }
    }
}

// the sweeps' counters start at zero (a kernel rather than a memset node, so a
// caller may capture the launches in a graph)
__global__ void zero_i64_kernel(int64_t *p, int k) {
    if ((int)threadIdx.x < k) p[threadIdx.x] = 0;
}

// workspace of the sorted float32 path
struct SortedBufs {
    ExtPart *parts;
    Extent *ext;
    uint32_t *keys_in, *keys_out;
    int32_t *idx_in, *sperm, *qperm;
    float4 *ps, *tbox, *bbox;
    double *ps64;
    int32_t *ovf_list;
    void *cub;
    size_t cub_bytes;
};

size_t cub_sort_bytes(int64_t k) {
    size_t bytes = 0;
    (void)hipcub::DeviceRadixSort::SortPairs(nullptr, bytes, (const uint32_t *)nullptr, (uint32_t *)nullptr,
                                            (const int32_t *)nullptr, (int32_t *)nullptr, (int)k, 0, 30);
    return bytes;
}

SortedBufs carve_sorted(Carver &c, int64_t n, int64_t m) {
    SortedBufs b;
    const int64_t k = n > m ? n : m;
    b.parts = c.take<ExtPart>(EXT_BLOCKS);
    b.ext = c.take<Extent>(1);
    b.keys_in = c.take<uint32_t>(k);
    b.keys_out = c.take<uint32_t>(k);
    b.idx_in = c.take<int32_t>(k);
    b.sperm = c.take<int32_t>(n);
    b.qperm = c.take<int32_t>(m);
    b.ps = c.take<float4>(n);
    b.ps64 = c.take<double>(4 * n);
    b.ovf_list = c.take<int32_t>(m);
    b.tbox = c.take<float4>(2 * ((n + TILE - 1) / TILE));
    b.bbox = c.take<float4>(2 * ((n + BLK - 1) / BLK));
    b.cub_bytes = std::max(cub_sort_bytes(n), cub_sort_bytes(m));
    b.cub = c.take<char>(b.cub_bytes);
    return b;
}

template <typename T>
struct SweepBufs {
    SweepOut<T> o;
    int64_t *overflows;  // [0] list overflows, [1] pairs the sorted sweep skipped, [2] its overflowed slots
};

template <typename T>
SweepBufs<T> carve_sweep(Carver &c, int64_t n, int64_t m) {
    SweepBufs<T> b;
    b.o.run = c.take<T>(2 * m);
    b.o.count = c.take<uint32_t>(2 * m);
    b.o.tiles = c.take<int32_t>(2 * m * LIST);
    b.o.vals = c.take<T>(2 * m * LIST);
    b.overflows = c.take<int64_t>(3);
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
    static_assert(std::is_same<T, double>::value, "the unsorted sweep serves the float64 mode");
    const Pt4<T> *pts = reinterpret_cast<const Pt4<T> *>(samples);
    zero_i64_kernel<<<1, 64, 0, st>>>(b.overflows, 3);
    const int64_t per = (int64_t)BT * QPT;
    KernelTimer t1("sweep", st);
    sweep_kernel<T, QPT><<<(unsigned)((m + per - 1) / per), BT, 0, st>>>(pts, (int)n, queries, m, eps, b.o);
    t1.stop();
    SDFI_HIP(hipGetLastError());
    KernelTimer t2("resolve", st);
    resolve_kernel<T><<<(unsigned)((m + 3) / 4), 256, 0, st>>>(samples, n, queries, m, eps, b.o, opt.tol,
                                                                opt.tie_tol, BoundsOut{lo, hi, argmax, argmin, flags},
                                                                b.overflows);
    t2.stop();
    SDFI_HIP(hipGetLastError());
    if (overflow_count) {
        SDFI_HIP(hipMemcpyAsync(overflow_count, b.overflows, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    }
    return SDFI_OK;
}

sdfi_status launch_sorted(const double *samples, int64_t n, const double *queries, int64_t m, double *lo,
                          double *hi, int32_t *argmax, int32_t *argmin, uint32_t *flags, Carver &ws,
                          const sdfi_options &opt, hipStream_t st, int64_t *overflow_count) {
    SweepBufs<float> b = carve_sweep<float>(ws, n, m);
    SortedBufs sb = carve_sorted(ws, n, m);
    if (!ws.ok()) {
        set_error("workspace too small for the bound sweep");
        return SDFI_ERR_WORKSPACE;
    }
    // extent, band, and the Morton orders of samples and queries
    extent_partial_kernel<<<EXT_BLOCKS, 256, 0, st>>>(samples, n, queries, m, sb.parts);
    extent_final_kernel<<<1, 64, 0, st>>>(sb.parts, EXT_BLOCKS, opt.tie_tol, sb.ext);
    morton_kernel<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(samples, 4, n, sb.ext, sb.keys_in, sb.idx_in);
    SDFI_HIP(hipcub::DeviceRadixSort::SortPairs(sb.cub, sb.cub_bytes, sb.keys_in, sb.keys_out, sb.idx_in, sb.sperm,
                                                (int)n, 0, 30, st));
    pack_sorted_kernel<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(samples, sb.sperm, n, sb.ps, sb.ps64);
    tile_box_kernel<<<(unsigned)((n + TILE - 1) / TILE), TILE, 0, st>>>(sb.ps, n, sb.tbox);
    block_box_kernel<<<(unsigned)(((n + BLK - 1) / BLK + 255) / 256), 256, 0, st>>>(sb.ps, n, sb.bbox);
    morton_kernel<<<(unsigned)((m + 255) / 256), 256, 0, st>>>(queries, 3, m, sb.ext, sb.keys_in, sb.idx_in);
    SDFI_HIP(hipcub::DeviceRadixSort::SortPairs(sb.cub, sb.cub_bytes, sb.keys_in, sb.keys_out, sb.idx_in, sb.qperm,
                                                (int)m, 0, 30, st));
    SDFI_HIP(hipGetLastError());
    zero_i64_kernel<<<1, 64, 0, st>>>(b.overflows, 3);
    const BoundsOut out{lo, hi, argmax, argmin, flags};
    const Fused fused{sb.ps64, sb.sperm, opt.tol, opt.tie_tol, out, sb.ovf_list,
                      reinterpret_cast<unsigned long long *>(b.overflows + 2)};
    KernelTimer t1("sweep", st);
    sweep_sorted_kernel<<<(unsigned)((m + MQ - 1) / MQ), MQ, 0, st>>>(sb.ps, (int)n, sb.tbox, queries, sb.qperm, m,
                                                                       sb.ext, b.o,
                                                                       reinterpret_cast<unsigned long long *>(b.overflows + 1),
                                                                       fused, sb.bbox);
    t1.stop();
    note_count("sweep_pairs_skipped", b.overflows + 1, st);
    SDFI_HIP(hipGetLastError());
    // the queries whose candidate lists overflowed (usually none)
    KernelTimer t2("resolve", st);
    resolve_list_kernel<<<RESOLVE_LIST_BLOCKS, RL_W * 64, 0, st>>>(samples, n, queries, &sb.ext->eps, b.o, opt.tol,
                                                             opt.tie_tol, out, b.overflows, sb.ovf_list,
                                                             reinterpret_cast<const unsigned long long *>(b.overflows + 2),
                                                             sb.sperm, sb.qperm, sb.ps, sb.tbox);
    t2.stop();
    note_count("bounds_list_overflows", b.overflows, st);
    SDFI_HIP(hipGetLastError());
    if (overflow_count) {
        SDFI_HIP(hipMemcpyAsync(overflow_count, b.overflows, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    }
    return SDFI_OK;
}

}  // namespace

static double eps_f64(const sdfi_options &o) { return o.tie_tol * 1.001 + 1e-15; }

size_t bounds_ws(int64_t n, int64_t m, const sdfi_options &o) {
    Carver c(nullptr, 0, true);
    if (o.precision == SDFI_PREC_FP32_FP64_RECHECK) {
        carve_sweep<float>(c, n, m);
        carve_sorted(c, n, m);
    } else {
        carve_sweep<double>(c, n, m);
    }
    return c.used + 256;
}

sdfi_status run_bounds(const double *samples, int64_t n, const double *queries, int64_t m, double *lo,
                       double *hi, int32_t *argmax, int32_t *argmin, uint32_t *flags, Carver &ws,
                       const sdfi_options &o, hipStream_t st, int64_t *overflow_count) {
    if (m == 0) return SDFI_OK;
    if (o.precision == SDFI_PREC_FP32_FP64_RECHECK)
        return launch_sorted(samples, n, queries, m, lo, hi, argmax, argmin, flags, ws, o, st, overflow_count);
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

// ---- the bound sweep without allocation ----
//
// A file-scope device array serves as the workspace of sdfi_bounds_noalloc.
// Host code never passes the array's name to a kernel or a copy (on the host
// it is a stand-in, not a device address): the device address is looked up
// once per device with hipGetSymbolAddress, with that device current, and
// kept in g_scratch_ptr.
namespace sdfi {
namespace {

constexpr size_t NOALLOC_SCRATCH_BYTES = size_t(64) << 20;
constexpr int MAX_DEVICES = 64;

__device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

std::mutex g_scratch_mu;
void *g_scratch_ptr[MAX_DEVICES] = {};

sdfi_status scratch_of_current_device(void **out) {
    int dev = 0;
    SDFI_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= MAX_DEVICES) {
        set_error("device ordinal %d beyond the %d supported by the allocation-free entry point", dev, MAX_DEVICES);
        return SDFI_ERR_UNSUPPORTED;
    }
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        SDFI_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) {
            set_error("hipGetSymbolAddress returned a null address for the scratch array");
            return SDFI_ERR_DEVICE;
        }
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return SDFI_OK;
}

}  // namespace
}  // namespace sdfi

extern "C" sdfi_status sdfi_bounds_noalloc(const double *samples, int64_t n, const double *queries, int64_t m,
                                           double *lo, double *hi, int32_t *argmax, int32_t *argmin,
                                           uint32_t *flags, const sdfi_options *opt, sdfi_stream stream) {
    using namespace sdfi;
    NoAllocScope no_alloc;
    sdfi_options o;
    sdfi_status s = read_options(opt, &o);
    if (s != SDFI_OK) return s;
    SDFI_CHECK_ARG(n >= 1 && n < (int64_t(1) << 31), "n must be in [1, 2^31), got %lld", (long long)n);
    SDFI_CHECK_ARG(m >= 0 && m < (int64_t(1) << 31), "m must be in [0, 2^31), got %lld", (long long)m);
    if (m == 0) return SDFI_OK;
    SDFI_CHECK_ARG(samples && queries && lo && hi && argmax && argmin && flags, "null array argument");
    const size_t need = bounds_ws(n, m, o);
    if (need > NOALLOC_SCRATCH_BYTES) {
        set_error("n = %lld, m = %lld need %zu bytes of scratch, beyond the %zu of the allocation-free entry point "
                  "(use sdfi_bounds with a workspace)",
                  (long long)n, (long long)m, need, NOALLOC_SCRATCH_BYTES);
        return SDFI_ERR_UNSUPPORTED;
    }
    void *ws = nullptr;
    s = scratch_of_current_device(&ws);
    if (s != SDFI_OK) return s;
    Carver c(ws, NOALLOC_SCRATCH_BYTES);
    return run_bounds(samples, n, queries, m, lo, hi, argmax, argmin, flags, c, o, to_hip(stream), nullptr);
}
