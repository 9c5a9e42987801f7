// Work-group helpers (reductions, ordered compaction) and the work-group
// minimum valid radius used by the greedy fallback and by the repair.
#pragma once

#include "geom_dev.h"

namespace sdfi {
namespace blk {

using geom::Balls;
using geom::Cap;

constexpr int NRAY = 15;  // rays of the minimum valid radius' upper bound
constexpr int RAYMAX = 16;

// Optional device-clock profile of rmin_block (slots of a counter array,
// written by thread 0 / lane 0 only): time in the containment scans, the ray
// bound, the candidate list builds and the sphere searches, and the number
// of calls, passes, listed candidates, local-set balls and sphere searches.
enum {
    RP_T_SCAN = 0, RP_T_RAY, RP_T_LIST, RP_T_SEARCH, RP_CALLS, RP_PASSES, RP_LIST_LEN, RP_LOCAL_LEN, RP_SEARCHES,
    // sphere searches (geom::lazy_nearest) that end before any cover scan,
    // right after the first one, and that enter the refinement rounds; rounds
    // run; searches that reach the exhaustive walk; wave ticks in the first
    // cover scan and in the rounds
    RP_LN_EARLY, RP_LN_FIRST, RP_LN_LOOP, RP_LN_ROUNDS, RP_LN_FALLBACK, RP_LN_T_FIRST, RP_LN_T_LOOP,
    // wave ticks in the exhaustive walks and the caps they walked; rounds that
    // ended because the covering cap was already in the subset; wave ticks in
    // the searches that ended early (holder or bound)
    RP_LN_T_FALLBACK, RP_LN_FALLBACK_CAPS, RP_LN_STALLED, RP_LN_T_EARLY,
    // passes run with the widened bound and with no bound; candidates that
    // the recent holders settled before any search; wave ticks in the
    // candidate pulls as a whole (searches included, waits at the end of the
    // pass excluded)
    RP_PASS_WIDE, RP_PASS_OPEN, RP_PRE_HELD, RP_T_PULL,
    RP_COUNT
};

template <int NW>
struct Shared {
    double rd[NW];
    double rv[NW][RAYMAX];
    int64_t ri[NW];
    int cnt[NW];
    int cnt2[NW];
    int counter;
    // minimum valid radius result slots, one per wave
    double wd[NW];
    double wlb[NW];
    int64_t wi[NW];
    int wk[NW];
    int wnd[NW];
    double wx[NW][3];
    unsigned long long bound_bits;
    double wlow[NW];
    int64_t hball[geom::NHOLD];  // balls that held whole search regions (this pass's local numbering)
    int hnext;
    // group_exist: each wave's part of the first cover test, and the result
    double gmx[NW];
    int64_t garg[NW], gpos[NW];
    int gwhole[NW], gcnt[NW], gecap[NW];
    int gst;
    double gx[3];
    // group_exist's rounds: wave 0's candidate directions (one per lane), the
    // rim each lies on and its cap's ball, their cover margins and covering
    // balls (found by all waves), the round's state
    double cv[64][3];
    double cmx[64];
    int64_t carg[64], cself[64];
    int crim[64];
    unsigned long long cfound;
    int gctl, gend, gfin;  // state after the walks, at the round's end, after the fallback
};

// Several work-groups on one instance (a team; all groups of a cooperative
// launch are resident at once): the team's first group runs the greedy and
// posts the steps whose work is many independent sphere searches (the
// minimum-radius candidate pulls, the re-validations) as jobs on a board in
// global memory; every group of the team takes items of a job from the
// shared counter.  A barrier of the team's groups opens and closes each job.
enum { J_RMIN = 1, J_REVAL = 2, J_EXIT = 3 };

struct Job {
    int type;
    int counter;                    // next item: candidate (pull at a time) or threatened sphere
    int fail;                       // re-validation: a sphere has no uncovered point left
    int keep_going;                 // re-validation: search every sphere even after a failure
    unsigned long long bound_bits;  // minimum radius: best distance so far (bits of a double >= 0)
    double q[3];
    double s;                       // re-validation: value of the new ball
    double Rdeep, tie;
    int64_t N, len, nl, deepest, nthr;
    // the holder ring of the minimum-radius searches, shared by the team
    int64_t hring[geom::NHOLD];
    int hnext;
    // the team's barrier: arrivals, generation; abort = a barrier waited past
    // its bound (the run is then reported as failed)
    unsigned bar_count, bar_gen;
    int abort;
};

// one group's best minimum-radius answer of a pass
struct GroupBest {
    double d, lb, low, x[3];
    int64_t i;
    int kind, nd;
};

struct Team {
    Job *job;
    GroupBest *best;  // one slot per group of the team
    int groups;       // groups in the team (1: none)
    int first;        // the launch's block index of the team's first group
};

// this group's rank in its team (0: the group that runs the greedy)
__device__ inline int team_rank(const Team &T) { return (int)blockIdx.x - T.first; }

// Barrier of the team's groups (every thread of each group calls it).  Each
// wave publishes its stores device-wide first; the last group to arrive
// starts the next generation.  A wait past 2^26 polls (about a minute) sets
// J->abort and returns, and later barriers of the team return at once, so
// every wave still reaches the kernel's end.
__device__ inline void team_sync(const Team &T) {
    Job *J = T.job;
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0 && !__hip_atomic_load(&J->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
        const unsigned gen = __hip_atomic_load(&J->bar_gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (atomicAdd(&J->bar_count, 1u) == (unsigned)T.groups - 1u) {
            __hip_atomic_store(&J->bar_count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __threadfence();
            atomicAdd(&J->bar_gen, 1u);
        } else {
            for (uint64_t spin = 0;; ++spin) {
                if (__hip_atomic_load(&J->bar_gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != gen) break;
                if (__hip_atomic_load(&J->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) break;
                if (spin > (uint64_t(1) << 26)) {
                    __hip_atomic_store(&J->abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    break;
                }
                __builtin_amdgcn_s_sleep(2);
            }
        }
    }
    __syncthreads();
    __threadfence();
}

__device__ inline int wid() { return threadIdx.x >> 6; }

// geom::lazy_exist_rest for a whole work-group: wave 0 walks the subset's
// rims as the one-wave search does; the cover tests of its candidate points
// (one per lane that found a gap) are shared out over all waves; wave 0 then
// takes them in lane order exactly as the one-wave search would (the first
// uncovered one is the answer, else each covering cap joins the subset).
// Every thread gets the status and the point.
template <int NW>
__device__ int group_exist_rest(const Balls &B0, const double *o, double r, const double *vh, Cap *kp, int64_t *kid,
                                int32_t *cl, int ccap, double *x, unsigned long long *walks, double mx, int64_t arg,
                                int whole, int ncl, int ecap, int64_t argpos, Shared<NW> &S) {
    const int w = threadIdx.x >> 6, ln = threadIdx.x & 63;
    if (whole) return geom::ST_NONE;
    if (!(mx > geom::COVER_EPS)) {
        for (int j = 0; j < 3; ++j) x[j] = o[j] + r * vh[j];
        return geom::ST_FOUND;
    }
    const bool compact = ncl <= ccap;
    const Balls B = geom::search_balls(B0, cl, ncl, ccap, ecap);
    if (compact) arg = argpos;
    if (threadIdx.x == 0) {
        kid[0] = arg;
        geom::cap_of(B, arg, o, r, kp[0]);
    }
    int k = 1;  // wave 0's subset size
    __syncthreads();
    // state: 0 next round, 1 found (S.gx), 2 covered, 3 fall back
    int state = 3;
    for (int round = 0; round < (B.walk_only ? 0 : 4 * geom::KMAX); ++round) {
        if (w == 0) {
            int found, numeric, frim;
            double mxp, myp;
            geom::Rim R;
            geom::subset_gap(kp, k, found, numeric, frim, R, mxp, myp);
            const unsigned long long fm = __ballot(found);
            const int anynum = geom::wor(numeric);
            if (found) {
                double v[3];
                geom::rim_dir(R, mxp, myp, v);
                S.cv[ln][0] = v[0];
                S.cv[ln][1] = v[1];
                S.cv[ln][2] = v[2];
                S.crim[ln] = frim;
                S.cself[ln] = kid[frim];
            }
            if (ln == 0) {
                S.cfound = fm;
                S.gctl = fm ? 0 : (anynum ? 3 : 2);
            }
        }
        __syncthreads();
        state = S.gctl;
        const unsigned long long fm = S.cfound;
        if (state) break;
        for (int c = w; c < 64; c += NW) {
            if (!((fm >> c) & 1ull)) continue;
            const double v[3] = {S.cv[c][0], S.cv[c][1], S.cv[c][2]};
            double m;
            int64_t a;
            int wh;
            geom::wave_cover(B, o, r, v, S.cself[c], &m, &a, &wh);
            if (ln == 0) {
                S.cmx[c] = m;
                S.carg[c] = a;
            }
        }
        __syncthreads();
        if (w == 0) {
            int st = 0, added = 0;
            for (int c = 0; c < 64 && !st; ++c) {
                if (!((fm >> c) & 1ull)) continue;
                if (!(S.cmx[c] > geom::COVER_EPS)) {
                    double v[3] = {S.cv[c][0], S.cv[c][1], S.cv[c][2]};
                    geom::nudge_off_rim(B, o, r, kp[S.crim[c]], v);
                    if (ln == 0)
                        for (int j = 0; j < 3; ++j) S.gx[j] = o[j] + r * v[j];
                    st = 1;
                    break;
                }
                const int64_t a = S.carg[c];
                bool have = false;
                for (int e = 0; e < k; ++e) have |= (kid[e] == a);
                if (!have && k < geom::KMAX) {
                    if (ln == 0) {
                        kid[k] = a;
                        geom::cap_of(B, a, o, r, kp[k]);
                    }
                    geom::wave_sync_lds();
                    ++k;
                    ++added;
                }
            }
            if (!st && !added) st = 3;  // subset full or no progress: fall back
            if (ln == 0) S.gend = st;
        }
        __syncthreads();
        state = S.gend;
        if (state) break;
        state = 3;
    }
    if (state == 2) return geom::ST_NONE;
    if (state == 3) {
        if (w == 0) {
            double xf[3];
            const int st = geom::exist_fallback(B, o, r, cl, ccap, compact, xf, walks);
            if (ln == 0) {
                S.gfin = st == geom::ST_FOUND ? 1 : (st == geom::ST_NONE ? 2 : 4);
                if (st == geom::ST_FOUND)
                    for (int j = 0; j < 3; ++j) S.gx[j] = xf[j];
            }
        }
        __syncthreads();
        state = S.gfin;
    }
    // state 1: found at S.gx; 2: covered; 4: numeric
    for (int j = 0; j < 3; ++j) x[j] = S.gx[j];
    __syncthreads();
    return state == 1 ? geom::ST_FOUND : (state == 2 ? geom::ST_NONE : geom::ST_NUMERIC);
}

// geom::lazy_exist for a whole work-group: the waves split the first cover
// test (which also lists the balls that meet the sphere) over slices of the
// balls, the slices' lists are joined in ball order, and wave 0 goes on
// alone, exactly as lazy_exist would.  cl: NW lists of ccap entries (one per
// wave; wave 0's receives the joined list).  Every thread gets the status
// and the point.
template <int NW>
__device__ __noinline__ int group_exist(const Balls &B, const double *o, double r, const double *hint, Cap *kp, int64_t *kid,
                           int32_t *cl, int ccap, double *x, unsigned long long *walks, Shared<NW> &S) {
    const int w = threadIdx.x >> 6;
    if (!(r > 0.0)) {
        // a point sphere: one wave's test
        if (w == 0) {
            const int st = geom::lazy_exist(B, o, r, hint, kp, kid, cl, ccap, x, walks);
            if ((threadIdx.x & 63) == 0) {
                S.gst = st;
                S.gx[0] = x[0];
                S.gx[1] = x[1];
                S.gx[2] = x[2];
            }
        }
        __syncthreads();
        const int st = S.gst;
        x[0] = S.gx[0];
        x[1] = S.gx[1];
        x[2] = S.gx[2];
        __syncthreads();
        return st;
    }
    double vh[3] = {1.0, 0.0, 0.0};
    if (hint) {
        double g[3] = {hint[0] - o[0], hint[1] - o[1], hint[2] - o[2]};
        double gn = sqrt(geom::dot3(g, g));
        if (gn > 0.0) {
            vh[0] = g[0] / gn;
            vh[1] = g[1] / gn;
            vh[2] = g[2] / gn;
        }
    }
    const int64_t n = geom::ball_count(B);
    const int64_t chunk = ((n + NW - 1) / NW + 63) / 64 * 64;
    const int64_t fb = min(n, (int64_t)w * chunk), fe = min(n, fb + chunk);
    double mx;
    int64_t arg, pos;
    int whole, cnt, ecap;
    geom::wave_cover_list(B, o, r, vh, &mx, &arg, &whole, cl + (int64_t)w * ccap, ccap, &cnt, &ecap, &pos, fb, fe);
    if ((threadIdx.x & 63) == 0) {
        S.gmx[w] = mx;
        S.garg[w] = arg;
        S.gpos[w] = pos;
        S.gwhole[w] = whole;
        S.gcnt[w] = cnt;
        S.gecap[w] = ecap;
    }
    __syncthreads();
    // join: the largest margin (lowest ball index among equals: the first such
    // slice), the list in ball order, its position there
    int total = 0, fits = 1, bw = 0, off_bw = 0, off_w = 0;
    whole = 0;
    ecap = 0;
    mx = -INFINITY;
    for (int v = 0; v < NW; ++v) {
        if (v == w) off_w = total;
        whole |= S.gwhole[v];
        ecap |= S.gecap[v];
        fits &= S.gcnt[v] <= ccap;
        if (S.gmx[v] > mx) {
            mx = S.gmx[v];
            bw = v;
            off_bw = total;
        }
        total += S.gcnt[v];
    }
    fits &= total <= ccap;
    arg = S.garg[bw];
    pos = arg >= B.N ? (int64_t)total : off_bw + S.gpos[bw];  // the extra ball sits after the rows
    if (fits && w > 0) {
        const int c = S.gcnt[w];
        for (int k = threadIdx.x & 63; k < c; k += 64) cl[off_w + k] = cl[(int64_t)w * ccap + k];
    }
    __threadfence_block();
    __syncthreads();
    return group_exist_rest<NW>(B, o, r, vh, kp, kid, cl, ccap, x, walks, mx, arg, whole, fits ? total : ccap + 1,
                                ecap, pos, S);
}
__device__ inline int lane() { return threadIdx.x & 63; }

template <int NW>
__device__ inline double bmax(double v, Shared<NW> &S) {
    v = geom::wmax(v);
    if (lane() == 0) S.rd[wid()] = v;
    __syncthreads();
    double r = S.rd[0];
    for (int w = 1; w < NW; ++w) r = fmax(r, S.rd[w]);
    __syncthreads();
    return r;
}

// element-wise block maximum of v[0..K) (K <= RAYMAX)
template <int NW, int K>
__device__ inline void bmax_n(double *v, Shared<NW> &S) {
    for (int k = 0; k < K; ++k) {
        const double r = geom::wmax(v[k]);
        if (lane() == 0) S.rv[wid()][k] = r;
    }
    __syncthreads();
    for (int k = 0; k < K; ++k) {
        double r = S.rv[0][k];
        for (int w = 1; w < NW; ++w) r = fmax(r, S.rv[w][k]);
        v[k] = r;
    }
    __syncthreads();
}

template <int NW>
__device__ inline double bmin(double v, Shared<NW> &S) {
    v = geom::wmin(v);
    if (lane() == 0) S.rd[wid()] = v;
    __syncthreads();
    double r = S.rd[0];
    for (int w = 1; w < NW; ++w) r = fmin(r, S.rd[w]);
    __syncthreads();
    return r;
}

template <int NW>
__device__ inline int64_t bmin_i64(int64_t v, Shared<NW> &S) {
    v = geom::wmin_i64(v);
    if (lane() == 0) S.ri[wid()] = v;
    __syncthreads();
    int64_t r = S.ri[0];
    for (int w = 1; w < NW; ++w) r = S.ri[w] < r ? S.ri[w] : r;
    __syncthreads();
    return r;
}

template <int NW>
__device__ inline int bor(int v, Shared<NW> &S) {
    v = geom::wor(v);
    if (lane() == 0) S.cnt[wid()] = v;
    __syncthreads();
    int r = 0;
    for (int w = 0; w < NW; ++w) r |= S.cnt[w];
    __syncthreads();
    return r;
}

// Append flagged items of one chunk (item base + threadIdx.x) to out[], in
// index order; returns the new length.  All threads call it.
// Ordered compaction of the rows c of [0, N) for which pred(c, f1, f2) sets
// f1 (into out1) or f2 (into out2), each list in row order, without a
// barrier per row block: wave w takes the contiguous slice w of the rows and
// stages its items in stage[w * scap ...] (first list from the front, second
// from the middle), then the slices' lists are concatenated.  Returns false,
// having written nothing, when a slice does not fit (2 x slice > scap).
// With `map`, position c stands for row map[c] (an index list in row order),
// which is what the lists receive.
template <int NW, class Pred>
__device__ bool bcompact2(int64_t N, Pred pred, int64_t *out1, int64_t cap1, int64_t *len1, int64_t *out2,
                          int64_t cap2, int64_t *len2, int32_t *stage, int scap, Shared<NW> &S,
                          const int64_t *map = nullptr) {
    const int64_t chunk = ((N + NW - 1) / NW + 63) / 64 * 64;
    if (2 * chunk > scap) return false;  // uniform
    const int w = wid(), ln = lane();
    const int64_t fb = min(N, (int64_t)w * chunk), fe = min(N, fb + chunk);
    int32_t *st1 = stage + (int64_t)w * scap, *st2 = st1 + chunk;
    int c1 = 0, c2 = 0;
    const unsigned long long below = (1ull << ln) - 1ull;
    for (int64_t f0 = fb; f0 < fe; f0 += 64) {
        const int64_t j = f0 + ln;
        const int64_t c = j < fe && map ? map[j] : j;
        bool f1 = false, f2 = false;
        if (j < fe) pred(c, f1, f2);
        const unsigned long long m1 = __ballot(f1), m2 = __ballot(f2);
        if (f1) st1[c1 + __popcll(m1 & below)] = (int32_t)c;
        if (f2) st2[c2 + __popcll(m2 & below)] = (int32_t)c;
        c1 += __popcll(m1);
        c2 += __popcll(m2);
    }
    if (ln == 0) {
        S.cnt[w] = c1;
        S.cnt2[w] = c2;
    }
    __threadfence_block();
    __syncthreads();
    int64_t o1 = 0, o2 = 0, t1 = 0, t2 = 0;
    for (int v = 0; v < NW; ++v) {
        if (v < w) {
            o1 += S.cnt[v];
            o2 += S.cnt2[v];
        }
        t1 += S.cnt[v];
        t2 += S.cnt2[v];
    }
    for (int k = ln; k < c1; k += 64)
        if (o1 + k < cap1) out1[o1 + k] = st1[k];
    for (int k = ln; k < c2; k += 64)
        if (o2 + k < cap2) out2[o2 + k] = st2[k];
    __syncthreads();
    *len1 = t1;
    *len2 = t2;
    return true;
}

template <int NW>
__device__ inline int64_t bappend(bool flag, int64_t item, int64_t len, int64_t *out, int64_t cap, Shared<NW> &S) {
    unsigned long long m = __ballot(flag);
    int before = __popcll(m & ((1ull << lane()) - 1ull));
    if (lane() == 0) S.cnt[wid()] = __popcll(m);
    __syncthreads();
    int off = 0, tot = 0;
    for (int w = 0; w < NW; ++w) {
        if (w < wid()) off += S.cnt[w];
        tot += S.cnt[w];
    }
    if (flag && len + off + before < cap) out[len + off + before] = item;
    __syncthreads();
    return len + tot;
}

__device__ inline int sign_class(double s, double tie) { return s > tie ? 1 : (s < -tie ? -1 : 0); }

// lexicographic (distance, not-deepest, lower bound, index) comparison
__device__ inline bool better(double d, int nd, double lb, int64_t i, double d2, int nd2, double lb2, int64_t i2) {
    if (d != d2) return d < d2;
    if (nd != nd2) return nd < nd2;
    if (lb != lb2) return lb < lb2;
    return i < i2;
}

// Lower bound of the distance from q to the points of sphere (p, r) that lie
// outside the open ball (pa, Ra) (INFINITY when there are none): every
// uncovered point of the sphere is such a point.  The points outside the ball
// are the sphere minus the cap v.u > c (u towards pa, c = (r^2 + D^2 -
// Ra^2)/(2 r D)); the nearest to q is the radial foot point when it lies
// outside the cap, else the rim point nearest to q, at distance
// sqrt(r^2 + d^2 - 2 r d (c g.u + sqrt(1 - c^2) sqrt(1 - (g.u)^2))) with g the
// direction from p to q.  The result is taken slightly short (relative
// 1e-12), so rounding never makes it exceed the true distance.
__device__ inline double dist_outside_ball(const double *q, const double *p, double r, const double *pa, double Ra) {
#pragma clang fp contract(off)
    const double g0 = q[0] - p[0], g1 = q[1] - p[1], g2 = q[2] - p[2];
    const double d = sqrt(g0 * g0 + g1 * g1 + g2 * g2);
    const double foot = fabs(d - r);
    const double u0 = pa[0] - p[0], u1 = pa[1] - p[1], u2 = pa[2] - p[2];
    const double D = sqrt(u0 * u0 + u1 * u1 + u2 * u2);
    if (!(Ra > 0.0) || !(r > 0.0) || !(D > 0.0) || !(d > 0.0)) return foot;
    if (D + r < Ra * (1.0 - 1e-12) - 1e-15) return INFINITY;  // the whole sphere is inside the ball
    if (!(D < r + Ra) || !(D + Ra > r)) return foot;           // the ball misses the sphere
    const double c = (r * r + D * D - Ra * Ra) / (2.0 * r * D);
    if (!(c > -1.0 && c < 1.0)) return foot;
    const double gu = (g0 * u0 + g1 * u1 + g2 * u2) / (d * D);
    if (!(gu > c)) return foot;                                 // the foot point is outside the ball
    const double vg = c * gu + sqrt(fmax(0.0, 1.0 - c * c)) * sqrt(fmax(0.0, 1.0 - gu * gu));
    const double rim = sqrt(fmax(0.0, r * r + d * d - 2.0 * r * d * vg));
    return fmax(foot, rim * (1.0 - 1e-12) - 1e-15);
}

// Upper bound of the minimum valid radius from ray exits (see rmin_block);
// out of line so that its per-ray state does not weigh on the caller's
// registers.  All threads of the work-group call it.
template <int NW>
__device__ __noinline__ double ray_bound(const double *q, int sigma, const double *p4, int64_t N, double tie,
                                         int64_t deepest, double depth, double known, Shared<NW> &S,
                                         const int64_t *idx, int64_t nr) {
    const int tid = threadIdx.x;
    const int BS = NW * 64;
    // A ray stops at `known` (an upper bound of the answer already), so only
    // balls that can hold a ray point nearer than that matter: the rows
    // idx[0..nr) when given (a superset of those, in row order), else all N.
    if (!idx) nr = N;
    {
        double dir[NRAY][3];
        {
            const double *pd = p4 + 4 * deepest;
            double u[3] = {q[0] - pd[0], q[1] - pd[1], q[2] - pd[2]};
            const double un = sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
            for (int j = 0; j < 3; ++j) dir[0][j] = un > 0.0 ? u[j] / un : (j == 0 ? 1.0 : 0.0);
            for (int k = 1; k < 7; ++k)
                for (int j = 0; j < 3; ++j) dir[k][j] = (j == (k - 1) / 2) ? ((k & 1) ? 1.0 : -1.0) : 0.0;
            const double is3 = 0.57735026918962576451;
            for (int k = 7; k < NRAY; ++k)
                for (int j = 0; j < 3; ++j) dir[k][j] = (((k - 7) >> j) & 1) ? -is3 : is3;
        }
        double t[NRAY];
        // the ray away from the deepest centre first; the others only when the
        // best bound so far (its exit, or `known` from elsewhere) is well beyond
        // the depth of the deepest ball (a lower bound of the answer), i.e. when
        // that bound may be loose
        unsigned live = 1u;
        bool widened = false;
        for (int k = 0; k < NRAY; ++k) t[k] = 0.0;
        double nearest = INFINITY;
        int wide_steps = 0;
        for (int it = 0; it < 128; ++it) {
            if (!live) {
                if (widened || !(fmin(nearest, known) > 1.25 * depth)) break;
                widened = true;
                live = ((1u << NRAY) - 1u) & ~1u;
            }
            // an extra ray that has not left the union after a few steps runs
            // through a long chain of balls: its exit is far and cannot help
            if (widened && ++wide_steps > 6) break;
            double step[NRAY];
            for (int k = 0; k < NRAY; ++k) step[k] = 0.0;
            for (int64_t c = tid; c < nr; c += BS) {
                const double *p = p4 + 4 * (idx ? idx[c] : c);
                if (sign_class(p[3], tie) != sigma) continue;
                const double R = fabs(p[3]) - tie;
                if (!(R > 0.0)) continue;
                for (int k = 0; k < NRAY; ++k) {
                    if (!((live >> k) & 1u)) continue;
                    const double w[3] = {q[0] + t[k] * dir[k][0] - p[0], q[1] + t[k] * dir[k][1] - p[1],
                                         q[2] + t[k] * dir[k][2] - p[2]};
                    const double cc = w[0] * w[0] + w[1] * w[1] + w[2] * w[2] - R * R;
                    if (!(cc < 0.0)) continue;
                    const double bb = dir[k][0] * w[0] + dir[k][1] * w[1] + dir[k][2] * w[2];
                    step[k] = fmax(step[k], -bb + sqrt(bb * bb - cc));
                }
            }
            bmax_n<NW, NRAY>(step, S);
            for (int k = 0; k < NRAY; ++k) {
                if (!((live >> k) & 1u)) continue;
                if (!(step[k] > 0.0)) {
                    nearest = fmin(nearest, t[k]);
                    live &= ~(1u << k);
                } else {
                    t[k] += step[k] + 1e-12;  // strictly past the exit of the ball left behind
                }
            }
            for (int k = 0; k < NRAY; ++k)
                if (((live >> k) & 1u) && !(t[k] < fmin(nearest, known))) live &= ~(1u << k);
        }
        // the exit may lie in a tol-thin overlap with an opposite-sign ball,
        // whose uncovered edge is within sqrt(2 R tol) of it: a margin of 2e-3
        // keeps the bound above the answer for radii up to 2
        return nearest < INFINITY ? nearest * (1.0 + 1e-12) + 2e-3 : INFINITY;
    }
}

// Minimum valid radius of q for sign sigma against balls rows [0, N) of p4
// (x, y, z, s) with known uncovered points W (rows may be NaN).  The contour
// is that of the balls shrunk by the uniqueness tolerance `tie` only, so the
// contact point clears every tol-shrunk ball by tol - tie while exactly
// tangent spheres leave non-degenerate gaps; q counts as inside a ball when
// d < |s| - tol.  Returns kind 0 (q in no sigma ball: radius 0),
// 1 T, 2 D, 3 U, -1 nothing found, -2 a search hit its cap (no answer).  list: scratch of 2 (N + 1) entries;
// kp/kid: per wave LDS scratch; flist: NW lists of fcap entries (global) for exhaustive searches.
// candidates a wave of a team takes at a time (a group alone takes 16)
constexpr int TEAM_PULL = 1;

// The candidate pulls of one minimum-radius pass, for every wave of the
// calling work-group: candidates list[0..len) (ball rows of p4, list[0] the
// deepest ball), local set lset[0..nl) (the balls that can cover a point
// within the pass bound of q), shared pull counter and best-distance bits
// (LDS for one group, the job board for a team).  Each wave's best ends in
// S.wd/wnd/wlb/wi/wk/wx/wlow[w].  ring/ring_next: the holder ring (null:
// this group's own, cleared here; else a team's, cleared by the poster).
template <int NW>
__device__ __noinline__ void rmin_pull(const double *q, const double *p4, double tie, const int64_t *list, int64_t len,
                          const int64_t *lset, int64_t nl, int64_t deepest, double Rdeep, int *counter,
                          unsigned long long *bound_bits, Cap (*kp)[geom::KMAX], int64_t (*kid)[geom::KMAX],
                          int32_t *flist, int fcap, Shared<NW> &S, unsigned long long *prof, int walk_only,
                          int64_t *ring = nullptr, int *ring_next = nullptr) {
    const double *pdeep = p4 + 4 * deepest;
    Balls L;
    L.p4 = p4;
    L.N = nl;
    L.idx = lset;
    L.has_extra = 0;
    L.tol = tie;  // contour of the balls shrunk by the uniqueness tolerance only
    L.skip = -1;
    L.lq[0] = q[0];
    L.lq[1] = q[1];
    L.lq[2] = q[2];
    L.lb = INFINITY;  // already applied by the index list
    L.use_region = 0;
    L.walk_only = walk_only;
    if (!ring) {
        ring = S.hball;
        ring_next = &S.hnext;
        if (threadIdx.x == 0) S.hnext = 0;
        if (threadIdx.x < geom::NHOLD) S.hball[threadIdx.x] = -1;
    }
    __syncthreads();
    // each wave pulls spheres and keeps its own best
    double wd = INFINITY, wlb = INFINITY, wx[3] = {0.0, 0.0, 0.0};
    int64_t wi = INT64_MAX;
    int wk = 0, wnd = 1;
    double wlow = INFINITY;
    geom::Holders hold{ring, ring_next, prof ? prof + RP_LN_EARLY : nullptr};  // shared by the waves, reset each pass
    const int w = wid();
    // each wave takes `pull` candidates at a time: lanes load them and their
    // lower bounds together, then the survivors are searched in list order
    // (re-pruned against the bound as it shrinks)
    const int pull = ring_next == &S.hnext ? 16 : TEAM_PULL;  // a team spreads the list thinner
    const unsigned long long t_pull = prof ? wall_clock64() : 0ull;
    for (int guard = 0; guard < (1 << 30); ++guard) {
        int k0 = 0;
        if (lane() == 0) k0 = atomicAdd(counter, pull);
        k0 = __shfl(k0, 0, 64);
        if (k0 >= len) break;
        const int64_t kl = (int64_t)k0 + lane();
        const bool have = lane() < pull && kl < len;
        const int64_t myi = have ? list[kl] : 0;
        double mylb = INFINITY, myprune = INFINITY;  // tie-break key, pruning bound
        if (have) {
            const double *pp = p4 + 4 * myi;
            mylb = fabs(geom::dist3(q, pp) - fabs(pp[3]));
            myprune = myi == deepest ? mylb : dist_outside_ball(q, pp, fabs(pp[3]), pdeep, Rdeep);
        }
        unsigned long long pending = __ballot(have);
        int ring_seen = -1;
        while (pending) {
            {
                // the recent holders first, for the pending candidates together,
                // whenever the ring has taken new entries: lane l tests candidate
                // l % pull against holder share l / pull of the ring (a holder
                // proves that the sphere has no uncovered point within the
                // bound; the bound only shrinks afterwards)
                const int shares = 64 / pull, per = (geom::NHOLD + shares - 1) / shares;
                int rn = 0;
                if (lane() == 0) rn = __hip_atomic_load(ring_next, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                rn = __shfl(rn, 0, 64);
                if (rn != ring_seen) {
                    ring_seen = rn;
                    unsigned long long cb = 0;
                    if (lane() == 0) cb = __hip_atomic_load(bound_bits, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    const double cur = __longlong_as_double((long long)__shfl(cb, 0, 64));
                    const int cj = lane() % pull, hg = lane() / pull;
                    const int64_t ci = __shfl(myi, cj, 64);
                    int hit = 0;
                    if ((pending >> cj) & 1ull) {
                        const double *pc = p4 + 4 * ci;
                        const double oc[3] = {pc[0], pc[1], pc[2]};
                        const double rc = fabs(pc[3]);
                        Balls Rg = L;
                        if (!geom::set_region(Rg, oc, rc, q, cur * (1.0 + 1e-12) + 1e-15))
                            hit = 1;
                        else
                            hit = geom::held_by(Rg, oc, rc, ring + hg * per,
                                                max(0, min(per, geom::NHOLD - hg * per)));
                    }
                    const unsigned long long hb = __ballot(hit);
                    unsigned long long held = 0;
                    for (int k = 0; k < shares; ++k) held |= hb >> (k * pull);
                    held &= (1ull << pull) - 1ull;
                    if (prof && lane() == 0 && (pending & held))
                        atomicAdd(&prof[RP_PRE_HELD], (unsigned long long)__popcll(pending & held));
                    pending &= ~held;
                    if (!pending) break;
                }
            }
            unsigned long long cb = 0;
            if (lane() == 0) cb = __hip_atomic_load(bound_bits, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            const double cur = __longlong_as_double((long long)__shfl(cb, 0, 64));  // wave-uniform
            // prune only clearly worse spheres: exact ties must reach the tie-break
            pending &= __ballot(!(myprune > cur * (1.0 + 1e-12) + 1e-15));
            if (!pending) break;
            const int src = __ffsll((long long)pending) - 1;
            pending &= pending - 1ull;
            const int64_t i = __shfl(myi, src, 64);
            const double lbi = __shfl(mylb, src, 64);
            const double *p = p4 + 4 * i;
            double d, x[3];
            if (prof && lane() == 0) atomicAdd(&prof[RP_SEARCHES], 1ull);
            int kk = geom::lazy_nearest(L, p, fabs(p[3]), q, cur * (1.0 + 1e-12) + 1e-15, kp[w], kid[w],
                                        flist + (int64_t)w * fcap, fcap, &d, x, &hold);
            if (kk < 0) {
                // a capped search proved only that this sphere has no uncovered
                // point nearer than d (a lower bound); it matters only if the
                // final answer is farther than that
                wlow = fmin(wlow, d);
                continue;
            }
            if (kk && better(d, i != deepest, lbi, i, wd, wnd, wlb, wi)) {
                wd = d;
                wnd = i != deepest;
                wlb = lbi;
                wi = i;
                wk = kk;
                wx[0] = x[0];
                wx[1] = x[1];
                wx[2] = x[2];
                if (lane() == 0)
                    atomicMin(bound_bits, (unsigned long long)__double_as_longlong(d));
            }
        }
    }
    if (prof && lane() == 0) atomicAdd(&prof[RP_T_PULL], wall_clock64() - t_pull);
    if (lane() == 0) {
        S.wlow[w] = wlow;
        S.wd[w] = wd;
        S.wnd[w] = wnd;
        S.wlb[w] = wlb;
        S.wi[w] = wi;
        S.wk[w] = wk;
        S.wx[w][0] = wx[0];
        S.wx[w][1] = wx[1];
        S.wx[w][2] = wx[2];
    }
}

// The best of the waves' answers (kind 0: none) and their lowest capped bound.
template <int NW>
__device__ inline GroupBest group_best(const Shared<NW> &S) {
    GroupBest gb;
    gb.kind = 0;
    gb.low = INFINITY;
    int bw = -1;
    for (int v = 0; v < NW; ++v) {
        gb.low = fmin(gb.low, S.wlow[v]);
        if (!S.wk[v]) continue;
        if (bw < 0 || better(S.wd[v], S.wnd[v], S.wlb[v], S.wi[v], S.wd[bw], S.wnd[bw], S.wlb[bw], S.wi[bw])) bw = v;
    }
    if (bw >= 0) {
        gb.d = S.wd[bw];
        gb.nd = S.wnd[bw];
        gb.lb = S.wlb[bw];
        gb.i = S.wi[bw];
        gb.kind = S.wk[bw];
        gb.x[0] = S.wx[bw][0];
        gb.x[1] = S.wx[bw][1];
        gb.x[2] = S.wx[bw][2];
    }
    return gb;
}

// a = the better of a and b (by `better`), lowest capped bound of both
__device__ inline void merge_best(GroupBest &a, const GroupBest &b) {
    a.low = fmin(a.low, b.low);
    if (b.kind && (!a.kind || better(b.d, b.nd, b.lb, b.i, a.d, a.nd, a.lb, a.i))) {
        const double low = a.low;
        a = b;
        a.low = low;
    }
}

// A helper group's part of a posted minimum-radius pass (job J): pull, then
// store the group's best in its slot.
template <int NW>
__device__ void rmin_pull_job(Job *J, const double *p4, const int64_t *list, Cap (*kp)[geom::KMAX],
                              int64_t (*kid)[geom::KMAX], int32_t *flist, int fcap, Shared<NW> &S, GroupBest *slot,
                              unsigned long long *prof, int walk_only) {
    const double q[3] = {J->q[0], J->q[1], J->q[2]};
    const int64_t N = J->N;
    rmin_pull<NW>(q, p4, J->tie, list, J->len, list + (N + 1), J->nl, J->deepest, J->Rdeep, &J->counter,
                  &J->bound_bits, kp, kid, flist, fcap, S, prof, walk_only, J->hring, &J->hnext);
    __syncthreads();
    const GroupBest gb = group_best(S);
    if (threadIdx.x == 0) *slot = gb;
}

template <int NW>
__device__ __noinline__ int rmin_block(const double *q, int sigma, const double *p4, const double *W, int64_t N, double tol,
                                 double tie, int64_t *list, Cap (*kp)[geom::KMAX], int64_t (*kid)[geom::KMAX],
                                 int32_t *flist, int fcap,
                                 Shared<NW> &S, double *r_out, double *x_out, int64_t *sphere_out,
                                 unsigned long long *prof = nullptr, int walk_only = 0,
                                 const Team *team = nullptr, int64_t *near = nullptr) {
    const int tid = threadIdx.x;
    const int BS = NW * 64;
    unsigned long long tmark = (prof && tid == 0) ? wall_clock64() : 0ull;
    auto lap = [&](int slot) {
        if (prof && tid == 0) {
            const unsigned long long t = wall_clock64();
            prof[slot] += t - tmark;
            tmark = t;
        }
    };
    if (prof && tid == 0) prof[RP_CALLS] += 1;
    // inside test, deepest sigma ball, and the nearest known contour point
    double depth = -INFINITY, wbest = INFINITY;
    int inside = 0;
    for (int64_t c = tid; c < N; c += BS) {
        const double *p = p4 + 4 * c;
        if (sign_class(p[3], tie) != sigma) continue;
        double d = geom::dist3(q, p);
        double R = fabs(p[3]);
        if (d < R - tol) inside = 1;
        depth = fmax(depth, R - d);
        if (W && !isnan(W[3 * c])) wbest = fmin(wbest, geom::dist3(W + 3 * c, q));
    }
    inside = bor(inside, S);
    if (!inside) {
        *r_out = 0.0;
        x_out[0] = q[0];
        x_out[1] = q[1];
        x_out[2] = q[2];
        *sphere_out = -1;
        return 0;
    }
    depth = bmax(depth, S);
    wbest = bmin(wbest, S);
    const double wbound = isinf(wbest) ? INFINITY : wbest * (1.0 + 1e-12) + 1e-15;
    // The balls near q, in row order: those that can cover a point within the
    // witness bound of q (d <= |s| + wbound).  Every ball the first pass
    // lists, every ball a ray meets before that bound, and the deepest ball
    // (it holds q) are among them; wider passes scan all rows.
    int64_t nn = N;
    const int64_t *nidx = nullptr;
    if (near && wbound < INFINITY) {
        auto sel = [&](int64_t c, bool &f, bool &) {
            const double *p = p4 + 4 * c;
            f = geom::dist3(q, p) <= fabs(p[3]) + wbound;
        };
        int64_t none = 0;
        if (bcompact2<NW>(N, sel, near, N, &nn, near, 0, &none, flist, fcap, S)) nidx = near;
        else nn = N;
    }
    int64_t deepest = INT64_MAX;
    for (int64_t j = tid; j < nn; j += BS) {
        const int64_t c = nidx ? nidx[j] : j;
        const double *p = p4 + 4 * c;
        if (sign_class(p[3], tie) != sigma) continue;
        if (fabs(p[3]) - geom::dist3(q, p) == depth) deepest = deepest < c ? deepest : c;
    }
    deepest = bmin_i64(deepest, S);
    lap(RP_T_SCAN);
    if (deepest == INT64_MAX) return -2;  // no ball attains the depth (only with NaN data): no answer
    double bound = wbound, rbound = INFINITY;
    // A second upper bound: the nearest exit of NRAY rays from q (away from the
    // deepest centre, along the axes and the diagonals).  At each point of a
    // ray, jump to the farthest exit among the balls (shrunk by tie) holding
    // it; the first point no ball holds is off the union, so the contour is no
    // farther from q than that point.  The rays advance together, one block
    // scan per step; a ray stops once it is past the nearest exit found.
    rbound = ray_bound<NW>(q, sigma, p4, N, tie, deepest, depth, wbound, S, nidx, nn);
    bound = fmin(bound, rbound);
    lap(RP_T_RAY);
    int64_t *lset = list + (N + 1);
    // Both bounds can fall just short of the answer: a cached witness is only
    // uncovered w.r.t. the tol-shrunk balls, and the ray may leave the sigma
    // union inside a tol-thin overlap with an opposite-sign ball, whose
    // uncovered edge lies within sqrt(2 R tol) of it.  A pass that finds
    // nothing within its bound moves on to that bound plus a margin of twice
    // that size, then to no bound at all; what a pass finds within its bound
    // is exact.
    const double looser = bound + 4e-3;
    const double *pdeep = p4 + 4 * deepest;
    const double Rdeep = fabs(pdeep[3]) - tie;  // the contour's balls are shrunk by tie
    for (int pass = 0; pass < 3; ++pass) {
        // candidate spheres: sigma spheres with points outside the deepest ball
        // within `bound` of q (deepest first): a sphere's uncovered points lie
        // outside every other ball, the deepest one included
        int64_t len = 0, nl = 0;
        auto select = [&](int64_t c, bool &f, bool &inl) {
            const double *p = p4 + 4 * c;
            double d = geom::dist3(q, p);
            if (c != deepest && sign_class(p[3], tie) == sigma && fabs(d - fabs(p[3])) <= bound)
                f = dist_outside_ball(q, p, fabs(p[3]), pdeep, Rdeep) <= bound;
            // the local set: balls that can cover a point within `bound` of q
            inl = isinf(bound) || d < fabs(p[3]) + bound;
        };
        // the first pass's bound is at most the witness bound: the near rows hold its lists
        const bool from_near = nidx && bound <= wbound;
        if (!bcompact2<NW>(from_near ? nn : N, select, list + 1, N, &len, lset, N, &nl, flist, fcap, S,
                           from_near ? nidx : nullptr)) {
            for (int64_t base = 0; base < N; base += BS) {
                int64_t c = base + tid;
                bool f = false, inl = false;
                if (c < N) select(c, f, inl);
                len = bappend(f, c, len, list + 1, N, S);
                nl = bappend(inl, c, nl, lset, N, S);
            }
        }
        if (tid == 0) list[0] = deepest;
        ++len;
        lap(RP_T_LIST);
        if (prof && tid == 0) {
            prof[RP_PASSES] += 1;
            if (pass == 1) prof[isinf(bound) ? RP_PASS_OPEN : RP_PASS_WIDE] += 1;
            if (pass == 2) prof[RP_PASS_OPEN] += 1;
            prof[RP_LIST_LEN] += (unsigned long long)len;
            prof[RP_LOCAL_LEN] += (unsigned long long)nl;
        }
        int *counter = &S.counter;
        unsigned long long *bbits = &S.bound_bits;
        if (tid == 0) {
            S.counter = 0;
            S.bound_bits = __double_as_longlong(bound);
        }
        const bool post = team && len > 32;  // a short list stays with this group
        if (post) {
            // post the pass on the board; every group pulls from its counter
            Job *J = team->job;
            if (tid == 0) {
                J->type = J_RMIN;
                J->counter = 0;
                J->bound_bits = __double_as_longlong(bound);
                J->q[0] = q[0];
                J->q[1] = q[1];
                J->q[2] = q[2];
                J->Rdeep = Rdeep;
                J->tie = tie;
                J->N = N;
                J->len = len;
                J->nl = nl;
                J->deepest = deepest;
                J->hnext = 0;
            }
            if (tid < geom::NHOLD) J->hring[tid] = -1;
            counter = &J->counter;
            bbits = &J->bound_bits;
            team_sync(*team);
        }
        rmin_pull<NW>(q, p4, tie, list, len, lset, nl, deepest, Rdeep, counter, bbits, kp, kid, flist, fcap, S, prof,
                      walk_only, post ? team->job->hring : nullptr, post ? &team->job->hnext : nullptr);
        __syncthreads();
        GroupBest gb = group_best(S);
        if (post) {
            if (tid == 0) team->best[0] = gb;
            team_sync(*team);  // every group has stored its best
            for (int g = 1; g < team->groups; ++g) merge_best(gb, team->best[g]);
        }
        int res = -1;
        const int numeric = gb.kind ? (gb.low < gb.d) : (gb.low < INFINITY);
        if (gb.kind && !numeric) {
            *r_out = gb.d;
            x_out[0] = gb.x[0];
            x_out[1] = gb.x[1];
            x_out[2] = gb.x[2];
            *sphere_out = gb.i;
            res = gb.kind;
        }
        __syncthreads();
        lap(RP_T_SEARCH);
        if (numeric) return -2;
        if (res > 0) return res;
        if (isinf(bound)) break;
        bound = (pass == 0 && looser > bound && !(isinf(wbound) && isinf(rbound))) ? looser : INFINITY;
    }
    return -1;
}

}  // namespace blk
}  // namespace sdfi
