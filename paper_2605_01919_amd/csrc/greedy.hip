// Greedy sequential interpolation (Sec. 3.3 interpolate_sdf_to applied in the
// refinement order of Sec. 4) and the per-sample witness search.
//
// One work-group of 1024 threads owns one instance and assigns its queries
// one after another, exactly as the sequential definition: for query q the
// work-group reduces the cone bounds over every constraint accepted so far
// (samples, then earlier queries), ranks the candidates hi and lo by the
// paper's score sign_score * |s|, and accepts the first one that keeps the
// set valid (Prop. 1):
//   - the new sphere keeps an uncovered point: its tangent point if no ball
//     covers it, else an exact search on the new sphere (one wavefront);
//   - every existing sphere keeps an uncovered point: spheres whose cached
//     witness falls inside the new ball are re-searched exactly with the new
//     ball added (wavefronts in parallel).
// Otherwise it takes 0 (outside every ball) or the minimum valid radius
// (all 16 wavefronts).  Batched instances run as independent work-groups of
// the same launch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <vector>

#include "block_dev.h"
#include "common.h"

namespace sdfi {

namespace {

// Wavefronts per greedy work-group: 8 by default, 4 with block_size 256 (one
// wavefront per SIMD, so the kernel may use twice the registers).
constexpr int NW_DEFAULT = 8;

enum {
    C_HI = 0, C_LO, C_ZERO, C_RMIN, C_COINC, C_INFEAS, C_UNRES, C_SEARCH, C_NUMERIC,
    C_WALKS,  // existence searches that reached the exhaustive walk over all listed caps
    // device wall-clock ticks per sub-phase: bounds, candidates, r_min, record
    C_T_BOUNDS, C_T_CAND, C_T_RMIN, C_T_RECORD,
    // finer split of the candidate checks: the cover test of the tangent point,
    // the new sphere's exact search, the threatened-witness scan, the
    // re-searches; number of threatened spheres
    C_T_COVER, C_T_VNEW, C_T_THREAT, C_T_REVAL, C_THREAT_LEN,
    C_RP0,  // blk::RP_COUNT slots of the minimum valid radius profile
    C_NCOUNT = C_RP0 + blk::RP_COUNT
};

struct GInst {
    const double *samples;   // n x 4
    const double *queries;   // m x 3
    const int64_t *order;    // m
    const double *w_in;      // n x 3 sample witnesses (NaN = none)
    double *values;
    int64_t *active;
    uint8_t *kind;
    double *witness;         // m x 3
    double *sample_witness;  // n x 3 or null
    int64_t *order_out;
    double *CP;              // (n + m) x 4 constraints
    double *CW;              // (n + m) x 3 witnesses
    int64_t *CSRC;           // (n + m) query index of each appended constraint
    int64_t *list;           // 2 (n + m + 1) scratch
    int32_t *flist;          // one cap list of fcap entries per wavefront, for the exhaustive searches
    int fcap;
    double *pend;            // (n + m) x 3 pending witness updates (the minimum radius's near rows meanwhile)
    unsigned long long *counts;  // C_NCOUNT
    int64_t n, m;
    int profile;             // record the finer sub-phase split (while timing is enabled)
    int walk_only;           // exact searches take the exhaustive rim walk (SDFI_OPT_EXHAUSTIVE)
    blk::Team team;          // several groups on this instance (team.groups > 1, a cooperative launch)
};

// the cap lists of this group's waves for the exhaustive searches (NW lists
// of fcap entries per group), and this wave's own
template <int NW>
__device__ inline int32_t *group_flist(const GInst &I) {
    const int g = I.team.groups > 1 ? blk::team_rank(I.team) : 0;
    return I.flist + (int64_t)g * NW * I.fcap;
}
template <int NW>
__device__ inline int32_t *wave_flist(const GInst &I) {
    return group_flist<NW>(I) + (int64_t)blk::wid() * I.fcap;
}

template <int NW>
struct StepShared {
    blk::Shared<NW> S;
    geom::Cap kp[NW][geom::KMAX];
    int64_t kid[NW][geom::KMAX];
    double x[3];
    int status;
    int fail;
    int counter;
    int rt, rfail;  // reval_group: the sphere taken, the failure flag seen
};

__device__ inline bool in_domain(const double *w, const double *dlo, const double *dhi, double tol) {
    for (int j = 0; j < 3; ++j)
        if (!(w[j] >= dlo[j] - tol && w[j] <= dhi[j] + tol)) return false;
    return true;
}

// indices c with |W_c - q| < rn, in index order, into I.list; returns the count
template <int NW>
__device__ int64_t threatened(const GInst &I, int64_t N, const double *q, double rn, int64_t n, int64_t m,
                              StepShared<NW> &SH) {
    constexpr int GBS = NW * 64;
    int64_t cnt = 0;
    if (rn > 0.0) {
        auto select = [&](int64_t c, bool &f, bool &) { f = geom::dist3(I.CW + 3 * c, q) < rn; };
        int64_t none = 0;
        if (!blk::bcompact2<NW>(N, select, I.list, n + m + 1, &cnt, I.list, 0, &none, group_flist<NW>(I), I.fcap,
                                SH.S)) {
            for (int64_t base = 0; base < N; base += GBS) {
                int64_t c = base + threadIdx.x;
                bool f = c < N && geom::dist3(I.CW + 3 * c, q) < rn;
                cnt = blk::bappend(f, c, cnt, I.list, n + m + 1, SH.S);
            }
        }
    }
    return cnt > n + m ? n + m : cnt;
}

// First guess for a threatened sphere (o, r) whose witness W lies inside the
// new ball (q, R): the point just outside that ball's cap on the sphere,
// nearest to W (the old uncovered region most likely straddles the cap's
// rim there).  Only orders the search.
__device__ inline void rim_hint(const double *o, double r, const double *q, double R, const double *W, double *h) {
    for (int j = 0; j < 3; ++j) h[j] = W[j];
    double u[3] = {q[0] - o[0], q[1] - o[1], q[2] - o[2]};
    const double D = sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
    if (!(D > 0.0) || !(R > 0.0) || !(r > 0.0)) return;
    for (int j = 0; j < 3; ++j) u[j] /= D;
    const double c0 = (r * r + D * D - R * R) / (2.0 * r * D);
    if (!(c0 > -1.0 && c0 < 1.0)) return;
    double w[3] = {(W[0] - o[0]) / r, (W[1] - o[1]) / r, (W[2] - o[2]) / r};
    const double wu = w[0] * u[0] + w[1] * u[1] + w[2] * u[2];
    double t[3] = {w[0] - wu * u[0], w[1] - wu * u[1], w[2] - wu * u[2]};
    double tn = sqrt(t[0] * t[0] + t[1] * t[1] + t[2] * t[2]);
    if (!(tn > 1e-12)) {  // W on the axis: any direction across it
        geom::basis(u, t, w);
        tn = 1.0;
    }
    const double c1 = c0 - 1e-7 * sqrt(1.0 - c0 * c0);  // just outside the cap
    const double r1 = sqrt(fmax(0.0, 1.0 - c1 * c1));
    for (int j = 0; j < 3; ++j) h[j] = o[j] + r * (c1 * u[j] + r1 * t[j] / tn);
}

// The calling group's share of the exact re-searches of the threatened
// spheres I.list[0..nthr) with the ball (q, s) added: waves take spheres from
// *counter; results into I.pend; *fail set if a sphere has no uncovered point
// left (without `keep_going` the waves then stop taking spheres; with it such
// spheres keep their old witness).
template <int NW>
__device__ __noinline__ void reval_part(const GInst &I, int64_t N, const double *q, double s, int64_t nthr, double tol,
                           StepShared<NW> &SH, bool keep_going, int *counter, int *fail) {
    const int w = blk::wid(), ln = blk::lane();
    geom::Balls B;
    B.p4 = I.CP;
    B.N = N;
    B.extra[0] = q[0];
    B.extra[1] = q[1];
    B.extra[2] = q[2];
    B.extra[3] = s;
    B.has_extra = 1;
    B.tol = tol;
    B.lb = INFINITY;
    B.idx = nullptr;
    B.use_region = 0;
    B.walk_only = I.walk_only;
    int32_t *fl = wave_flist<NW>(I);
    for (int64_t guard = 0; guard <= nthr; ++guard) {
        int t = 0;
        if (ln == 0) t = atomicAdd(counter, 1);
        t = __shfl(t, 0, 64);
        if (t >= nthr) break;
        int fv = 0;
        if (ln == 0) fv = __hip_atomic_load(fail, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (__shfl(fv, 0, 64) && !keep_going) break;  // wave-uniform
        int64_t c = I.list[t];
        B.skip = c;
        const double *p = I.CP + 4 * c;
        double x[3], hint[3];
        rim_hint(p, fabs(p[3]), q, fabs(s) - tol, I.CW + 3 * c, hint);
        int st = geom::lazy_exist_call(B, p, fabs(p[3]), hint, SH.kp[w], SH.kid[w], fl, I.fcap, x,
                                       &I.counts[C_WALKS]);
        if (ln == 0) {
            atomicAdd(&I.counts[C_SEARCH], 1ull);
            if (st == geom::ST_NUMERIC) atomicAdd(&I.counts[C_NUMERIC], 1ull);
            bool ok = st == geom::ST_FOUND;
            if (!ok) atomicOr(fail, 1);
            for (int j = 0; j < 3; ++j) I.pend[3 * t + j] = ok ? x[j] : I.CW[3 * c + j];
        }
    }
}

// A team group's share of the re-searches: the group takes one threatened
// sphere at a time from *counter and searches it with all its waves
// (group_exist); otherwise as reval_part.
template <int NW>
__device__ __noinline__ void reval_group(const GInst &I, int64_t N, const double *q, double s, int64_t nthr,
                                         double tol, StepShared<NW> &SH, bool keep_going, int *counter, int *fail) {
    geom::Balls B;
    B.p4 = I.CP;
    B.N = N;
    B.extra[0] = q[0];
    B.extra[1] = q[1];
    B.extra[2] = q[2];
    B.extra[3] = s;
    B.has_extra = 1;
    B.tol = tol;
    B.lb = INFINITY;
    B.idx = nullptr;
    B.use_region = 0;
    B.walk_only = I.walk_only;
    for (int64_t guard = 0; guard <= nthr; ++guard) {
        if (threadIdx.x == 0) {
            SH.rt = atomicAdd(counter, 1);
            SH.rfail = __hip_atomic_load(fail, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        __syncthreads();
        const int t = SH.rt, fv = SH.rfail;
        __syncthreads();
        if (t >= nthr || (fv && !keep_going)) break;  // group-uniform
        const int64_t c = I.list[t];
        B.skip = c;
        const double *p = I.CP + 4 * c;
        double x[3], hint[3];
        rim_hint(p, fabs(p[3]), q, fabs(s) - tol, I.CW + 3 * c, hint);
        const int st = blk::group_exist<NW>(B, p, fabs(p[3]), hint, SH.kp[0], SH.kid[0], group_flist<NW>(I), I.fcap,
                                            x, &I.counts[C_WALKS], SH.S);
        if (threadIdx.x == 0) {
            atomicAdd(&I.counts[C_SEARCH], 1ull);
            if (st == geom::ST_NUMERIC) atomicAdd(&I.counts[C_NUMERIC], 1ull);
            const bool ok = st == geom::ST_FOUND;
            if (!ok) atomicOr(fail, 1);
            for (int j = 0; j < 3; ++j) I.pend[3 * t + j] = ok ? x[j] : I.CW[3 * c + j];
        }
    }
}

// Exact re-search of the threatened spheres with the ball (q, s) added:
// several spheres go to the team's groups (each searched by a whole group);
// without a team, a few spheres are searched one after another by the whole
// group, more by the waves in parallel.  Results into I.pend, SH.fail = 1 if
// some sphere has no uncovered point left.
template <int NW>
__device__ __noinline__ void revalidate(const GInst &I, int64_t N, const double *q, double s, int64_t nthr, double tol,
                           StepShared<NW> &SH, bool keep_going) {
    if (threadIdx.x == 0) {
        SH.fail = 0;
        SH.counter = 0;
    }
    __syncthreads();
    if (nthr <= 0) return;
    if (I.team.groups > 1 && nthr > 1) {
        blk::Job *J = I.team.job;
        if (threadIdx.x == 0) {
            J->type = blk::J_REVAL;
            J->counter = 0;
            J->fail = 0;
            J->keep_going = keep_going ? 1 : 0;
            J->q[0] = q[0];
            J->q[1] = q[1];
            J->q[2] = q[2];
            J->s = s;
            J->N = N;
            J->nthr = nthr;
        }
        blk::team_sync(I.team);
        reval_group<NW>(I, N, q, s, nthr, tol, SH, keep_going, &J->counter, &J->fail);
        blk::team_sync(I.team);
        if (threadIdx.x == 0) SH.fail = __hip_atomic_load(&J->fail, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    } else if (nthr <= NW / 4 || I.team.groups > 1) {
        reval_group<NW>(I, N, q, s, nthr, tol, SH, keep_going, &SH.counter, &SH.fail);
    } else {
        reval_part<NW>(I, N, q, s, nthr, tol, SH, keep_going, &SH.counter, &SH.fail);
    }
    __syncthreads();
}

// A helper group of a team: work on the jobs group 0 posts until it posts
// J_EXIT.
template <int NW>
__device__ __noinline__ void helper_loop(const GInst &I, double tol, StepShared<NW> &SH) {
    blk::Job *J = I.team.job;
    for (;;) {
        blk::team_sync(I.team);
        const int type = __hip_atomic_load(&J->type, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (type == blk::J_EXIT || __hip_atomic_load(&J->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return;
        if (type == blk::J_RMIN) {
            blk::rmin_pull_job<NW>(J, I.CP, I.list, SH.kp, SH.kid, group_flist<NW>(I), I.fcap, SH.S,
                                   I.team.best + blk::team_rank(I.team), I.profile ? I.counts + C_RP0 : nullptr,
                                   I.walk_only);
        } else if (type == blk::J_REVAL) {
            const double q[3] = {J->q[0], J->q[1], J->q[2]};
            reval_group<NW>(I, J->N, q, J->s, J->nthr, tol, SH, J->keep_going != 0, &J->counter, &J->fail);
        }
        blk::team_sync(I.team);
    }
}

template <int NW>
__global__ __launch_bounds__(NW * 64) void greedy_kernel(const GInst *insts, double tol, double tie, double dlo0,
                                                         double dlo1, double dlo2, double dhi0, double dhi1,
                                                         double dhi2, int teams) {
    constexpr int GBS = NW * 64;
    __shared__ StepShared<NW> SH;
    // teams > 0: a team launch of that many instances, each on the groups
    // [team.first, team.first + team.groups); else one group per instance
    int ii = blockIdx.x;
    if (teams > 0) {
        int lo = 0, hi = teams - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (insts[mid].team.first <= (int)blockIdx.x) lo = mid;
            else hi = mid - 1;
        }
        ii = lo;
    }
    const GInst I = insts[ii];
    const bool team = I.team.groups > 1;
    if (team && blk::team_rank(I.team) > 0) {
        helper_loop<NW>(I, tol, SH);
        return;
    }
    const int tid = threadIdx.x;
    const int w = blk::wid(), ln = blk::lane();
    const double dlo[3] = {dlo0, dlo1, dlo2}, dhi[3] = {dhi0, dhi1, dhi2};
    const int64_t n = I.n, m = I.m;
    for (int64_t c = tid; c < n; c += GBS) {
        for (int j = 0; j < 4; ++j) I.CP[4 * c + j] = I.samples[4 * c + j];
        for (int j = 0; j < 3; ++j) I.CW[3 * c + j] = I.w_in[3 * c + j];
        I.CSRC[c] = -1;
    }
    if (tid < C_NCOUNT) I.counts[tid] = 0;
    __syncthreads();
    __threadfence_block();
    int64_t N = n;
    for (int64_t k = 0; k < m; ++k) {
        const int64_t j = I.order[k];
        const double q[3] = {I.queries[3 * j], I.queries[3 * j + 1], I.queries[3 * j + 2]};
        unsigned long long t_mark = tid == 0 ? wall_clock64() : 0;
        // ---- cone bounds over all constraints (Sec. 4.3) ----
        double lo = -INFINITY, hi = INFINITY;
        for (int64_t c = tid; c < N; c += GBS) {
            const double *p = I.CP + 4 * c;
            double d = geom::dist3(q, p);
            lo = fmax(lo, p[3] - d);
            hi = fmin(hi, p[3] + d);
        }
        lo = blk::bmax(lo, SH.S);
        hi = blk::bmin(hi, SH.S);
        int64_t a = INT64_MAX, b = INT64_MAX;
        for (int64_t c = tid; c < N; c += GBS) {
            const double *p = I.CP + 4 * c;
            double d = geom::dist3(q, p);
            if (p[3] - d >= lo - tie && c < a) a = c;
            if (p[3] + d <= hi + tie && c < b) b = c;
        }
        a = blk::bmin_i64(a, SH.S);
        b = blk::bmin_i64(b, SH.S);
        if (a == INT64_MAX || b == INT64_MAX) lo = NAN;  // only with NaN inputs
        if (tid == 0) {
            unsigned long long t = wall_clock64();
            I.counts[C_T_BOUNDS] += t - t_mark;
            t_mark = t;
        }
        double val = NAN, wq[3] = {q[0], q[1], q[2]};
        int kindv = 0;
        int64_t act = -1;
        int accepted = 0;
        int npend = 0;
        int64_t nthr = 0;
        if (!(lo <= hi + tol)) {
            kindv = SDFI_KIND_INFEASIBLE;
        } else {
            const double *pa = I.CP + 4 * a, *pb = I.CP + 4 * b;
            const double da = geom::dist3(q, pa), db = geom::dist3(q, pb);
            if (da <= tie || db <= tie) {
                int64_t c = da <= tie ? a : b;
                val = I.CP[4 * c + 3];
                kindv = SDFI_KIND_COINCIDENT;
                act = c;
                for (int jj = 0; jj < 3; ++jj) wq[jj] = I.CW[3 * c + jj];
                accepted = 2;
            } else {
                // candidates: hi tangent to b at p_b - s_b u_b, lo tangent to a at p_a + s_a u_a
                double cs[2], cw[2][3];
                int64_t ct[2];
                int ck[2];
                double sh = (hi > 0.0 ? 1.0 : 2.0) * fabs(hi), sl = (lo > 0.0 ? 1.0 : 2.0) * fabs(lo);
                bool hi_first;
                if (fabs(sh - sl) <= tie)
                    hi_first = !(lo < 0.0 && hi >= 0.0);
                else
                    hi_first = sh > sl;
                for (int e = 0; e < 2; ++e) {
                    bool is_hi = (e == 0) == hi_first;
                    const double *pt = is_hi ? pb : pa;
                    double dt = is_hi ? db : da;
                    double s = is_hi ? hi : lo;
                    double sgn = is_hi ? -1.0 : 1.0;
                    for (int jj = 0; jj < 3; ++jj) cw[e][jj] = pt[jj] + sgn * pt[3] * (q[jj] - pt[jj]) / dt;
                    cs[e] = s;
                    ct[e] = is_hi ? b : a;
                    ck[e] = is_hi ? SDFI_KIND_HI : SDFI_KIND_LO;
                }
                unsigned long long t_sub = (tid == 0 && I.profile) ? wall_clock64() : 0ull;
                auto sub = [&](int slot) {
                    if (tid == 0 && I.profile) {
                        const unsigned long long t = wall_clock64();
                        I.counts[slot] += t - t_sub;
                        t_sub = t;
                    }
                };
                for (int e = 0; e < 2 && !accepted; ++e) {
                    if (!in_domain(cw[e], dlo, dhi, tol)) continue;
                    const double s = cs[e], r = fabs(s);
                    // new sphere: tangent point uncovered?
                    int cov = 0;
                    for (int64_t c = tid; c < N; c += GBS) {
                        const double *p = I.CP + 4 * c;
                        if (geom::dist3(cw[e], p) < fabs(p[3]) - tol) cov = 1;
                    }
                    cov = blk::bor(cov, SH.S);
                    sub(C_T_COVER);
                    double nw[3] = {cw[e][0], cw[e][1], cw[e][2]};
                    if (cov) {
                        // the whole group runs the new sphere's exact search
                        geom::Balls B;
                        B.p4 = I.CP;
                        B.N = N;
                        B.has_extra = 0;
                        B.tol = tol;
                        B.skip = -1;
                        B.lb = INFINITY;
                        B.idx = nullptr;
                        B.use_region = 0;
                        B.walk_only = I.walk_only;
                        const int st = blk::group_exist<NW>(B, q, r, cw[e], SH.kp[0], SH.kid[0], group_flist<NW>(I),
                                                            I.fcap, nw, &I.counts[C_WALKS], SH.S);
                        if (tid == 0) {
                            atomicAdd(&I.counts[C_SEARCH], 1ull);
                            if (st == geom::ST_NUMERIC) atomicAdd(&I.counts[C_NUMERIC], 1ull);
                        }
                        sub(C_T_VNEW);
                        if (st != geom::ST_FOUND) continue;
                    }
                    // existing spheres whose witness lies in the new open (shrunk) ball
                    nthr = threatened(I, N, q, r - tol, n, m, SH);
                    sub(C_T_THREAT);
                    if (tid == 0 && I.profile) I.counts[C_THREAT_LEN] += (unsigned long long)nthr;
                    revalidate(I, N, q, s, nthr, tol, SH, false);
                    __syncthreads();
                    int failed = SH.fail;
                    __syncthreads();
                    sub(C_T_REVAL);
                    if (failed) continue;
                    accepted = 1;
                    val = s;
                    kindv = ck[e];
                    act = ct[e];
                    wq[0] = nw[0];
                    wq[1] = nw[1];
                    wq[2] = nw[2];
                    npend = 1;
                }
                if (tid == 0) {
                    unsigned long long t = wall_clock64();
                    I.counts[C_T_CAND] += t - t_mark;
                    t_mark = t;
                }
                if (!accepted) {
                    if (lo <= tol && hi >= -tol) {
                        val = 0.0;
                        kindv = SDFI_KIND_ZERO;
                        act = -1;
                        accepted = 3;
                    } else {
                        int sigma = lo > tol ? 1 : -1;
                        double rr, x[3];
                        int64_t sph;
                        int kk = blk::rmin_block<NW>(q, sigma, I.CP, I.CW, N, tol, tie, I.list, SH.kp, SH.kid, I.flist,
                                                     I.fcap, SH.S, &rr, x, &sph, I.profile ? I.counts + C_RP0 : nullptr,
                                                     I.walk_only, team ? &I.team : nullptr,
                                                     reinterpret_cast<int64_t *>(I.pend));
                        if (kk == -2 && tid == 0) atomicAdd(&I.counts[C_NUMERIC], 1ull);
                        if (kk > 0) {
                            val = sigma * rr;
                            kindv = kk == 1 ? SDFI_KIND_RMIN_T : (kk == 2 ? SDFI_KIND_RMIN_D : SDFI_KIND_RMIN_U);
                            act = sph;
                            wq[0] = x[0];
                            wq[1] = x[1];
                            wq[2] = x[2];
                            accepted = 4;
                            // Corollary 1: the minimal sphere covers no contour point; a cached
                            // witness is only uncovered w.r.t. the shrunk balls and may sit just
                            // inside the union, so witnesses inside the new ball are re-searched
                            nthr = threatened(I, N, q, rr - tol, n, m, SH);
                            revalidate(I, N, q, val, nthr, tol, SH, true);
                            npend = 1;
                        } else if (kk == 0) {
                            val = 0.0;
                            kindv = SDFI_KIND_ZERO;
                            accepted = 3;
                        } else {
                            kindv = SDFI_KIND_UNRESOLVED;
                        }
                        if (tid == 0) {
                            unsigned long long t = wall_clock64();
                            I.counts[C_T_RMIN] += t - t_mark;
                            t_mark = t;
                        }
                    }
                }
            }
        }
        // ---- record and append ----
        __syncthreads();
        if (npend) {
            for (int64_t t = tid; t < nthr; t += GBS) {
                int64_t c = I.list[t];
                for (int jj = 0; jj < 3; ++jj) I.CW[3 * c + jj] = I.pend[3 * t + jj];
            }
        }
        if (tid == 0) {
            I.values[j] = val;
            I.kind[j] = (uint8_t)kindv;
            I.active[j] = act < 0 ? -1 : (act < n ? act : n + I.CSRC[act]);
            I.order_out[k] = j;
            int ci = kindv == SDFI_KIND_HI ? C_HI
                   : kindv == SDFI_KIND_LO ? C_LO
                   : kindv == SDFI_KIND_ZERO ? C_ZERO
                   : kindv == SDFI_KIND_COINCIDENT ? C_COINC
                   : kindv == SDFI_KIND_INFEASIBLE ? C_INFEAS
                   : kindv == SDFI_KIND_UNRESOLVED ? C_UNRES : C_RMIN;
            atomicAdd(&I.counts[ci], 1ull);
            if (accepted) {
                I.CP[4 * N] = q[0];
                I.CP[4 * N + 1] = q[1];
                I.CP[4 * N + 2] = q[2];
                I.CP[4 * N + 3] = val;
                I.CW[3 * N] = wq[0];
                I.CW[3 * N + 1] = wq[1];
                I.CW[3 * N + 2] = wq[2];
                I.CSRC[N] = j;
            } else {
                I.witness[3 * j] = NAN;
                I.witness[3 * j + 1] = NAN;
                I.witness[3 * j + 2] = NAN;
            }
        }
        if (accepted) ++N;
        __threadfence_block();
        __syncthreads();
        if (tid == 0) I.counts[C_T_RECORD] += wall_clock64() - t_mark;
    }
    if (team) {
        // release the helper groups
        if (tid == 0) __hip_atomic_store(&I.team.job->type, blk::J_EXIT, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        blk::team_sync(I.team);
    }
    // final witnesses of the query spheres and of the samples
    for (int64_t c = n + tid; c < N; c += GBS) {
        int64_t jq = I.CSRC[c];
        for (int jj = 0; jj < 3; ++jj) I.witness[3 * jq + jj] = I.CW[3 * c + jj];
    }
    if (I.sample_witness)
        for (int64_t c = tid; c < n; c += GBS)
            for (int jj = 0; jj < 3; ++jj) I.sample_witness[3 * c + jj] = I.CW[3 * c + jj];
}

// One wavefront per sample: an uncovered point of its sphere, or none.  The
// rows [0, n) of p4 form nseg independent sets [seg[k], seg[k+1]) (seg null:
// one set); a sample's sphere is tested against its own set only.
__global__ __launch_bounds__(256) void witness_kernel(const double *p4_all, int64_t n, const int64_t *seg, int nseg,
                                                      double tol, double tie, double *wout_all, uint8_t *status_all) {
    __shared__ geom::Cap kp[4][geom::KMAX];
    __shared__ int64_t kid[4][geom::KMAX];
    __shared__ int32_t cl[4][geom::FALLBACK_LDS];
    const int w = threadIdx.x >> 6, ln = threadIdx.x & 63;
    for (int64_t ig = (int64_t)blockIdx.x * 4 + w; ig < n; ig += (int64_t)gridDim.x * 4) {
        // the set holding row ig (binary search over the segment starts)
        int64_t s0 = 0, s1 = n;
        if (seg) {
            int lo = 0, hi = nseg - 1;
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (seg[mid] <= ig) lo = mid;
                else hi = mid - 1;
            }
            s0 = seg[lo];
            s1 = seg[lo + 1];
        }
        const double *p4 = p4_all + 4 * s0;
        const int64_t i = ig - s0, n = s1 - s0;
        double *wout = wout_all + 3 * s0;
        uint8_t *status = status_all + s0;
        const double *pi = p4 + 4 * i;
        int sg = blk::sign_class(pi[3], tie);
        double sg1 = sg != 0 ? (double)sg : 1.0;
        // hint: the neighbour e minimising sign(s_i) s_e + d_ie (towards the surface)
        double best = INFINITY;
        int64_t be = INT64_MAX;
        for (int64_t e = ln; e < n; e += 64) {
            if (e == i) continue;
            double d = geom::dist3(pi, p4 + 4 * e);
            if (!(d > 0.0)) continue;
            double key = sg1 * p4[4 * e + 3] + d;
            if (key < best) {
                best = key;
                be = e;
            }
        }
        double g = geom::wmin(best);
        int64_t cand = best == g ? be : INT64_MAX;
        be = geom::wmin_i64(cand);
        geom::Balls B;
        B.p4 = p4;
        B.N = n;
        B.has_extra = 0;
        B.tol = tol;
        B.skip = i;
        B.lb = INFINITY;
        B.idx = nullptr;
        B.use_region = 0;
        double x[3];
        int st = geom::lazy_exist(B, pi, fabs(pi[3]), be != INT64_MAX ? p4 + 4 * be : nullptr, kp[w], kid[w], cl[w], geom::FALLBACK_LDS, x);
        if (ln == 0) {
            status[i] = st == geom::ST_FOUND ? 1 : 0;
            for (int j = 0; j < 3; ++j) wout[3 * i + j] = st == geom::ST_FOUND ? x[j] : NAN;
        }
    }
}

struct GBufs {
    double *CP, *CW, *pend, *win;
    int64_t *CSRC, *list;
    int32_t *flist;
    uint8_t *wstat;
    unsigned long long *counts;
    int64_t *order;
    int64_t *seg;
    GInst *inst;
    blk::Job *job;
    blk::GroupBest *best;
};

// Work-groups of the greedy kernel with nw waves that the current device
// keeps resident at once (occupancy x compute units), looked up once per
// device.
int resident_groups(int nw) {
    static std::mutex mu;
    static std::map<std::pair<int, int>, int> cache;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    std::lock_guard<std::mutex> lock(mu);
    auto it = cache.find({dev, nw});
    if (it != cache.end()) return it->second;
    int per_cu = 0, cus = 0;
    hipError_t e = nw == 4 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, greedy_kernel<4>, 256, 0)
                           : hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, greedy_kernel<NW_DEFAULT>,
                                                                          NW_DEFAULT * 64, 0);
    if (e != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return 0;
    return cache[{dev, nw}] = per_cu * cus;
}

// Wavefronts per greedy work-group.  block_size 256 or 512 fixes it; 0 picks
// 8 waves while every instance of the launch can hold a resident work-group
// of 8 waves, else 4 waves, which keeps more instances in flight.
int greedy_waves(const sdfi_options &o, int ninst = 1) {
    if (o.block_size == 256) return 4;
    if (o.block_size == 512 || ninst <= 1) return NW_DEFAULT;
    const int slots = resident_groups(NW_DEFAULT);
    return slots > 0 && ninst > slots ? 4 : NW_DEFAULT;
}

// Groups that share a single instance: o.groups, else 16; at most what the
// device keeps resident (a cooperative launch needs every group resident).
constexpr int TEAM_DEFAULT = 16;
int team_request(const sdfi_options &o) { return o.groups > 0 ? o.groups : TEAM_DEFAULT; }

// whether the current device takes cooperative launches (teams need them)
bool cooperative_ok() {
    int dev = 0, on = 0;
    if (hipGetDevice(&dev) != hipSuccess) return false;
    return hipDeviceGetAttribute(&on, hipDeviceAttributeCooperativeLaunch, dev) == hipSuccess && on != 0;
}

int team_groups(const sdfi_options &o, int nw) {
    if (!cooperative_ok()) return 1;
    const int slots = resident_groups(nw);
    return std::max(1, std::min(team_request(o), slots));
}

// groups: the most work-groups any instance gets (a team when > 1)
GBufs carve_greedy(Carver &c, int64_t n, int64_t m, int ninst, int nw, int groups) {
    GBufs b;
    int64_t cap = n + m + 1;
    b.CP = c.take<double>(4 * cap);
    b.CW = c.take<double>(3 * cap);
    b.pend = c.take<double>(3 * cap);
    b.win = c.take<double>(3 * (n + 1));
    b.CSRC = c.take<int64_t>(cap);
    b.list = c.take<int64_t>(2 * (cap + ninst) + 2);
    b.flist = c.take<int32_t>((int64_t)groups * nw * (cap + ninst));
    b.wstat = c.take<uint8_t>(n + 1);
    b.counts = c.take<unsigned long long>(C_NCOUNT * ninst);
    b.order = c.take<int64_t>(m + 1);
    b.seg = c.take<int64_t>(ninst + 1);
    b.inst = c.take<GInst>(ninst);
    b.job = c.take<blk::Job>(ninst);
    b.best = c.take<blk::GroupBest>((int64_t)groups * ninst);
    return b;
}

}  // namespace

size_t witness_ws(int64_t, const sdfi_options &) { return 256; }

// what each further instance of a batched launch takes: counters, its
// descriptor, offsets, job board and group slots (with the alignment of
// each carved array)
size_t greedy_instance_ws(const sdfi_options &o) {
    return sizeof(unsigned long long) * C_NCOUNT + sizeof(GInst) + sizeof(int64_t) + sizeof(blk::Job) +
           sizeof(blk::GroupBest) * (size_t)team_request(o) + 2 * sizeof(int64_t);
}

sdfi_status run_witnesses(const double *samples, int64_t n, double *w, uint8_t *st, const sdfi_options &o,
                          hipStream_t s, const int64_t *seg, int nseg) {
    if (n == 0) return SDFI_OK;
    int blocks = (int)std::min<int64_t>((n + 3) / 4, 4096);
    KernelTimer tm("witness", s);
    witness_kernel<<<blocks, 256, 0, s>>>(samples, n, seg, nseg, o.tol, o.tie_tol, w, st);
    tm.stop();
    SDFI_HIP(hipGetLastError());
    return SDFI_OK;
}

size_t greedy_ws(int64_t n, int64_t m, const sdfi_options &o) {
    Carver c(nullptr, 0, true);
    carve_greedy(c, n + 1, m, 1, greedy_waves(o), team_request(o));  // as greedy_common carves one instance
    Carver c2(nullptr, 0, true);
    size_t ord = order_ws(n, m, o);
    size_t cert = (o.flags & SDFI_OPT_CERTIFY) ? certify_ws(n + m, o) + 4 * (n + m) * 8 + 3 * (n + m) * 8 + 1024 : 0;
    size_t incheck = (o.flags & SDFI_OPT_INPUT_CHECK) ? certify_ws(n, o) : 0;
    return c.used + std::max({ord, cert, incheck, check_ws(m)}) + 1024;
}

sdfi_status run_order(const double *samples, int64_t n, const double *queries, int64_t m, int64_t *order_out,
                      Carver &ws, const sdfi_options &o, hipStream_t st);
sdfi_status run_order_batched(int ninst, const int64_t *soff, const int32_t *grids, const double *samples,
                              int64_t *order_out, Carver &ws, const sdfi_options &o, hipStream_t st);

static double now_ms() {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

__global__ void zero_words_kernel(unsigned *p, int64_t k) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < k) p[i] = 0u;
}

__global__ void pack_set_kernel(const double *samples, int64_t n, const double *queries, const double *values,
                                int64_t m, const double *sw, const double *qw, double *pv, double *wall) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) {
        for (int j = 0; j < 4; ++j) pv[4 * i + j] = samples[4 * i + j];
        for (int j = 0; j < 3; ++j) wall[3 * i + j] = sw[3 * i + j];
    } else if (i < n + m) {
        int64_t q = i - n;
        for (int j = 0; j < 3; ++j) pv[4 * i + j] = queries[3 * q + j];
        pv[4 * i + 3] = values[q];
        for (int j = 0; j < 3; ++j) wall[3 * i + j] = qw[3 * q + j];
    }
}

}  // namespace sdfi

using namespace sdfi;

extern "C" sdfi_status sdfi_sample_witnesses(const double *samples, int64_t n, double *witness_out,
                                             uint8_t *status_out, void *, size_t, const sdfi_options *opt,
                                             sdfi_stream stream) {
    sdfi_options o;
    sdfi_status s = read_options(opt, &o);
    if (s != SDFI_OK) return s;
    SDFI_CHECK_ARG(n >= 0 && n < (int64_t(1) << 31), "n out of range");
    if (n == 0) return SDFI_OK;
    SDFI_CHECK_ARG(samples && witness_out && status_out, "null array argument");
    return run_witnesses(samples, n, witness_out, status_out, o, to_hip(stream));
}

static sdfi_status greedy_common(int ninst, const int64_t *soff, const int64_t *qoff, const int32_t *grids,
                                 const double *samples, const double *queries, const int64_t *order_in,
                                 double *values, int64_t *order_out, int64_t *active, uint8_t *kind, double *witness,
                                 double *sample_witness, sdfi_report *report, void *ws, size_t ws_bytes,
                                 const sdfi_options &o, hipStream_t st) {
    const int64_t n = soff[ninst], m = qoff[ninst];
    Carver c(ws, ws_bytes);
    const int nw = greedy_waves(o, ninst);
    // work-groups per instance: a team when more than one (all resident: a
    // cooperative launch); a batch shares the resident groups out by pair
    // count when there are at least two per instance
    std::vector<int> G(ninst, 1);
    {
        const int slots = resident_groups(nw);
        const int cap = team_request(o);
        if (ninst == 1) {
            G[0] = team_groups(o, nw);
        } else if (cap > 1 && slots >= 2 * ninst && cooperative_ok()) {
            const int total = std::min<int64_t>(slots, (int64_t)cap * ninst);
            double wsum = 0.0;
            std::vector<double> wk(ninst);
            for (int i = 0; i < ninst; ++i) {
                const double ni = (double)(soff[i + 1] - soff[i]), mi = (double)(qoff[i + 1] - qoff[i]);
                wk[i] = ni * mi + 0.5 * mi * mi;
                wsum += wk[i];
            }
            int used = 0;
            for (int i = 0; i < ninst; ++i) {
                G[i] = std::max(1, std::min(cap, (int)(total * (wsum > 0.0 ? wk[i] / wsum : 1.0 / ninst))));
                used += G[i];
            }
            while (used > total) {  // trim the largest teams
                int big = 0;
                for (int i = 1; i < ninst; ++i)
                    if (G[i] > G[big]) big = i;
                if (G[big] <= 1) break;
                --G[big];
                --used;
            }
        }
    }
    const int gmax = *std::max_element(G.begin(), G.end());
    const bool teams = gmax > 1;
    GBufs b = carve_greedy(c, n + ninst, m, ninst, nw, team_request(o));
    if (!c.ok()) {
        set_error("workspace too small for the greedy interpolation");
        return SDFI_ERR_WORKSPACE;
    }
    double t0 = now_ms();
    char *rest_base = c.base + c.used + 256;
    const size_t rest_bytes = ws_bytes > c.used + 256 ? ws_bytes - c.used - 256 : 0;
    // 0. inputs: finite, inside the domain box (Appendix B), grid samples and
    //    refinement queries where the order is derived, order_in a permutation;
    //    all instances checked together, one read-back
    {
        std::vector<CheckJob> jobs(ninst);
        for (int i = 0; i < ninst; ++i) {
            const int g = order_in ? 0 : (grids ? grids[i] : o.grid);
            jobs[i] = CheckJob{samples + 4 * soff[i], soff[i + 1] - soff[i], queries + 3 * qoff[i],
                               qoff[i + 1] - qoff[i], order_in ? order_in + qoff[i] : nullptr, g, 2 * g};
        }
        sdfi_status s = validate_jobs(jobs.data(), ninst, true, rest_base, rest_bytes, o, st);
        if (s != SDFI_OK) return s;
    }
    // 1. witnesses of the input spheres, each instance against its own
    //    samples, one launch
    SDFI_HIP(hipMemsetAsync(b.wstat, 0, n + 1, st));
    {
        const int64_t *seg = nullptr;
        if (ninst > 1) {
            SDFI_HIP(hipMemcpyAsync(b.seg, soff, sizeof(int64_t) * (ninst + 1), hipMemcpyHostToDevice, st));
            seg = b.seg;
        }
        sdfi_status s = run_witnesses(samples, n, b.win, b.wstat, o, st, seg, ninst);
        if (s != SDFI_OK) return s;
    }
    if (o.flags & SDFI_OPT_INPUT_CHECK) {
        // Prop. 1 on the inputs: every sphere has an uncovered point (the
        // witness search) and no pair breaks the cone (the certificate's
        // pairwise count on the samples)
        std::vector<uint8_t> h(n);
        SDFI_HIP(hipMemcpyAsync(h.data(), b.wstat, n, hipMemcpyDeviceToHost, st));
        SDFI_HIP(hipStreamSynchronize(st));
        for (int64_t i = 0; i < n; ++i)
            if (!h[i]) {
                set_error("input sample %lld has no uncovered point (Prop. 1 (ii) violated)", (long long)i);
                return SDFI_ERR_INVALID_INPUT;
            }
        for (int i = 0; i < ninst; ++i) {
            Carver cc(rest_base, rest_bytes);
            int64_t pv = 0, wv = 0;
            sdfi_status s = run_certify(samples + 4 * soff[i], b.win + 3 * soff[i], soff[i + 1] - soff[i], &pv, &wv,
                                        cc, o, st);
            if (s != SDFI_OK) return s;
            if (pv > 0) {
                set_error("instance %d: %lld pairs of input samples break the cone |s_x - s_y| <= |p_x - p_y| "
                          "(opposite-sign spheres intersect or a sphere lies in another's ball, Prop. 1)",
                          i, (long long)pv);
                return SDFI_ERR_INVALID_INPUT;
            }
        }
    }
    double t1 = now_ms();
    // 2. order
    const int64_t *ord = order_in;
    if (!ord && ninst > 1) {
        Carver rest(rest_base, rest_bytes);
        sdfi_status s = run_order_batched(ninst, soff, grids, samples, b.order, rest, o, st);
        if (s != SDFI_OK) return s;
        ord = b.order;
    } else if (!ord) {
        for (int i = 0; i < ninst; ++i) {
            sdfi_options oi = o;
            oi.grid = grids ? grids[i] : o.grid;
            if (oi.grid <= 0) {
                set_error("order_in is NULL and no grid resolution was given");
                return SDFI_ERR_INVALID_ARGUMENT;
            }
            Carver rest(c.base + c.used + 256, ws_bytes > c.used + 256 ? ws_bytes - c.used - 256 : 0);
            sdfi_status s = run_order(samples + 4 * soff[i], soff[i + 1] - soff[i], nullptr, qoff[i + 1] - qoff[i],
                                      b.order + qoff[i], rest, oi, st);
            if (s != SDFI_OK) return s;
        }
        ord = b.order;
    }
    double t2 = now_ms();
    // 3. greedy, one work-group per instance
    std::vector<GInst> hi(ninst);
    int64_t cpos = 0, fpos = 0;
    for (int i = 0; i < ninst; ++i) {
        GInst &g = hi[i];
        int64_t ni = soff[i + 1] - soff[i], mi = qoff[i + 1] - qoff[i];
        g.samples = samples + 4 * soff[i];
        g.queries = queries + 3 * qoff[i];
        g.order = ord + qoff[i];
        g.w_in = b.win + 3 * soff[i];
        g.values = values + qoff[i];
        g.active = active + qoff[i];
        g.kind = kind + qoff[i];
        g.witness = witness + 3 * qoff[i];
        // final sample witnesses go to the caller, else back into the workspace copy
        // (the certificate below reads them from there)
        g.sample_witness = sample_witness ? sample_witness + 3 * soff[i] : b.win + 3 * soff[i];
        g.order_out = order_out + qoff[i];
        g.CP = b.CP + 4 * cpos;
        g.CW = b.CW + 3 * cpos;
        g.pend = b.pend + 3 * cpos;
        g.CSRC = b.CSRC + cpos;
        g.list = b.list + 2 * (cpos + i);
        // each wave's cap list holds every ball of a small instance, FALLBACK_GLOBAL otherwise
        g.fcap = (int)std::min<int64_t>(geom::FALLBACK_GLOBAL, ni + mi + 1);
        g.flist = b.flist + fpos;
        fpos += (int64_t)G[i] * nw * g.fcap;
        g.counts = b.counts + C_NCOUNT * i;
        g.profile = timing_enabled() ? 1 : 0;
        g.walk_only = (o.flags & SDFI_OPT_EXHAUSTIVE) ? 1 : 0;
        g.team.job = b.job + i;
        g.team.best = b.best + (int64_t)team_request(o) * i;
        g.team.groups = G[i];
        g.team.first = 0;  // set below, in launch order
        g.n = ni;
        g.m = mi;
        cpos += ni + mi;
    }
    // longest first: work-groups start roughly in launch order, so the
    // instances with the most pairs to scan (n m + m^2 / 2) start earliest and
    // the short ones fill in behind them
    std::stable_sort(hi.begin(), hi.end(), [](const GInst &x, const GInst &y) {
        return x.n * x.m + x.m * x.m / 2 > y.n * y.m + y.m * y.m / 2;
    });
    // teams take consecutive blocks in launch order
    int nblocks = 0;
    for (int k = 0; k < ninst; ++k) {
        hi[k].team.first = nblocks;
        nblocks += hi[k].team.groups;
    }
    SDFI_HIP(hipMemcpyAsync(b.inst, hi.data(), sizeof(GInst) * ninst, hipMemcpyHostToDevice, st));
    if (teams) {
        const int64_t words = (int64_t)(sizeof(blk::Job) * ninst / sizeof(unsigned));
        zero_words_kernel<<<(unsigned)((words + 255) / 256), 256, 0, st>>>(reinterpret_cast<unsigned *>(b.job), words);
    }
    KernelTimer tm("greedy", st);
    if (teams) {
        // every group resident at once: a cooperative launch
        const GInst *ip = b.inst;
        double tol = o.tol, tie = o.tie_tol;
        double d0 = o.domain_lo[0], d1 = o.domain_lo[1], d2 = o.domain_lo[2];
        double d3 = o.domain_hi[0], d4 = o.domain_hi[1], d5 = o.domain_hi[2];
        int nt = ninst;
        void *args[] = {&ip, &tol, &tie, &d0, &d1, &d2, &d3, &d4, &d5, &nt};
        const void *fn = nw == 4 ? (const void *)greedy_kernel<4> : (const void *)greedy_kernel<NW_DEFAULT>;
        SDFI_HIP(hipLaunchCooperativeKernel(fn, dim3(nblocks), dim3(nw * 64), args, 0, st));
    } else if (nw == 4) {
        greedy_kernel<4><<<ninst, 4 * 64, 0, st>>>(b.inst, o.tol, o.tie_tol, o.domain_lo[0], o.domain_lo[1],
                                                   o.domain_lo[2], o.domain_hi[0], o.domain_hi[1], o.domain_hi[2], 0);
    } else {
        greedy_kernel<NW_DEFAULT><<<ninst, NW_DEFAULT * 64, 0, st>>>(b.inst, o.tol, o.tie_tol, o.domain_lo[0],
                                                                     o.domain_lo[1], o.domain_lo[2], o.domain_hi[0],
                                                                     o.domain_hi[1], o.domain_hi[2], 0);
    }
    tm.stop();
    SDFI_HIP(hipGetLastError());
    std::vector<unsigned long long> cnt(C_NCOUNT * ninst);
    SDFI_HIP(hipMemcpyAsync(cnt.data(), b.counts, sizeof(unsigned long long) * cnt.size(), hipMemcpyDeviceToHost, st));
    std::vector<blk::Job> jobs(teams ? ninst : 0);
    if (teams) SDFI_HIP(hipMemcpyAsync(jobs.data(), b.job, sizeof(blk::Job) * ninst, hipMemcpyDeviceToHost, st));
    SDFI_HIP(hipStreamSynchronize(st));
    for (int i = 0; i < (int)jobs.size(); ++i)
        if (jobs[i].abort) {
            set_error("instance %d: a barrier of its work-groups waited past its bound; the results are not valid", i);
            return SDFI_ERR_DEVICE;
        }
    double t3 = now_ms();
    if (report) {
        std::memset(report, 0, sizeof(*report));
        int dev = 0, khz = 0;
        SDFI_HIP(hipGetDevice(&dev));
        SDFI_HIP(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev));
        const double wall_khz = khz > 0 ? (double)khz : 1e5;
        int64_t pairs = 0;
        for (int i = 0; i < ninst; ++i) {
            int64_t ni = soff[i + 1] - soff[i], mi = qoff[i + 1] - qoff[i];
            pairs += mi * ni + mi * (mi - 1) / 2;
            const unsigned long long *cc = cnt.data() + C_NCOUNT * i;
            report->n_hi += cc[C_HI];
            report->n_lo += cc[C_LO];
            report->n_zero += cc[C_ZERO];
            report->n_rmin += cc[C_RMIN];
            report->n_coincident += cc[C_COINC];
            report->n_infeasible += cc[C_INFEAS];
            report->n_unresolved += cc[C_UNRES];
            report->n_exact_searches += cc[C_SEARCH];
            report->n_search_capped += cc[C_NUMERIC];
            for (int ph = 0; ph < 4; ++ph) report->ms_phase[4 + ph] += cc[C_T_BOUNDS + ph] / wall_khz;
        }
        report->pairs_evaluated = pairs;
        // the finer split goes to the named work counters (while timing is on)
        static const char *names[C_NCOUNT - C_T_COVER] = {
            "greedy_cover_ticks", "greedy_vnew_ticks", "greedy_threat_ticks", "greedy_reval_ticks",
            "greedy_threatened", "rmin_scan_ticks", "rmin_ray_ticks", "rmin_list_ticks", "rmin_search_ticks",
            "rmin_calls", "rmin_passes", "rmin_list_len", "rmin_local_len", "rmin_searches", "ln_early", "ln_first",
            "ln_loop", "ln_rounds", "ln_fallback", "ln_first_ticks", "ln_loop_ticks", "ln_fallback_ticks",
            "ln_fallback_caps", "ln_stalled", "ln_early_ticks", "rmin_wide_passes", "rmin_open_passes",
            "rmin_pre_held", "rmin_pull_ticks"};
        for (int k = C_T_COVER; k < C_NCOUNT; ++k) {
            unsigned long long tot = 0;
            for (int i = 0; i < ninst; ++i) tot += cnt[C_NCOUNT * i + k];
            add_count(names[k - C_T_COVER], (int64_t)tot);
        }
        add_count("wall_clock_khz", (int64_t)wall_khz);
        {
            // the longest instance's device time (bounds + candidates + r_min + record)
            unsigned long long mx = 0;
            for (int i = 0; i < ninst; ++i) {
                unsigned long long t = 0;
                for (int ph = 0; ph < 4; ++ph) t += cnt[C_NCOUNT * i + C_T_BOUNDS + ph];
                mx = std::max(mx, t);
            }
            add_count("greedy_instance_max_ticks", (int64_t)mx);
        }
        {
            unsigned long long tot = 0;
            for (int i = 0; i < ninst; ++i) tot += cnt[C_NCOUNT * i + C_WALKS];
            add_count("exist_walks", (int64_t)tot);
        }
        report->ms_phase[0] = t2 - t1;
        report->ms_phase[1] = t1 - t0;
        report->ms_phase[2] = t3 - t2;
    }
    // 4. optional certificate of each instance's final set
    if (o.flags & SDFI_OPT_CERTIFY) {
        int64_t pv_tot = 0, wv_tot = 0;
        for (int i = 0; i < ninst; ++i) {
            int64_t ni = soff[i + 1] - soff[i], mi = qoff[i + 1] - qoff[i];
            Carver cc2(c.base + c.used + 256, ws_bytes > c.used + 256 ? ws_bytes - c.used - 256 : 0);
            double *pvb = cc2.take<double>(4 * (ni + mi));
            double *wb = cc2.take<double>(3 * (ni + mi));
            if (!cc2.ok()) {
                set_error("workspace too small for the certificate");
                return SDFI_ERR_WORKSPACE;
            }
            const double *sw = sample_witness ? sample_witness + 3 * soff[i] : b.win + 3 * soff[i];
            pack_set_kernel<<<(unsigned)((ni + mi + 255) / 256), 256, 0, st>>>(
                samples + 4 * soff[i], ni, queries + 3 * qoff[i], values + qoff[i], mi, sw, witness + 3 * qoff[i],
                pvb, wb);
            int64_t pv = 0, wv = 0;
            sdfi_status s = run_certify(pvb, wb, ni + mi, &pv, &wv, cc2, o, st);
            if (s != SDFI_OK) return s;
            pv_tot += pv;
            wv_tot += wv;
        }
        if (report) {
            report->n_violations_pairwise = pv_tot;
            report->n_violations_witness = wv_tot;
            report->ms_phase[3] = now_ms() - t3;
        }
    }
    return SDFI_OK;
}

extern "C" sdfi_status sdfi_greedy_interpolate(const double *samples, int64_t n, const double *queries, int64_t m,
                                               const int64_t *order_in, double *values, int64_t *order_out,
                                               int64_t *active, uint8_t *kind, double *witness,
                                               double *sample_witness, sdfi_report *report, void *ws,
                                               size_t ws_bytes, const sdfi_options *opt, sdfi_stream stream) {
    sdfi_options o;
    sdfi_status s = read_options(opt, &o);
    if (s != SDFI_OK) return s;
    SDFI_CHECK_ARG(n >= 1 && m >= 0 && n + m < (int64_t(1) << 31), "sizes out of range");
    if (m == 0) return SDFI_OK;
    SDFI_CHECK_ARG(samples && queries && values && order_out && active && kind && witness, "null array argument");
    SDFI_CHECK_ARG(order_in || o.grid > 0, "order_in is NULL and opt->grid is 0");
    if (o.grid > 0 && !order_in)
        SDFI_CHECK_ARG((int64_t)o.grid * o.grid * o.grid == n && m == 8 * n,
                       "grid %d needs n = grid^3 samples and m = 8 n refinement queries", o.grid);
    if (ws_bytes < greedy_ws(n, m, o) || !ws) {
        set_error("workspace of %zu bytes is below the %zu required", ws_bytes, greedy_ws(n, m, o));
        return SDFI_ERR_WORKSPACE;
    }
    int64_t soff[2] = {0, n}, qoff[2] = {0, m};
    int32_t g = o.grid;
    return greedy_common(1, soff, qoff, &g, samples, queries, order_in, values, order_out, active, kind, witness,
                         sample_witness, report, ws, ws_bytes, o, to_hip(stream));
}

extern "C" sdfi_status sdfi_greedy_interpolate_batched(int32_t num_instances, const int64_t *sample_offsets,
                                                       const int64_t *query_offsets, const int32_t *grids,
                                                       const double *samples, const double *queries, double *values,
                                                       int64_t *order_out, int64_t *active, uint8_t *kind,
                                                       double *witness, sdfi_report *report, void *ws,
                                                       size_t ws_bytes, const sdfi_options *opt, sdfi_stream stream) {
    sdfi_options o;
    sdfi_status s = read_options(opt, &o);
    if (s != SDFI_OK) return s;
    SDFI_CHECK_ARG(num_instances >= 1 && num_instances <= 65535, "num_instances out of range");
    SDFI_CHECK_ARG(sample_offsets && query_offsets && grids, "null host offset/grid array");
    SDFI_CHECK_ARG(sample_offsets[0] == 0 && query_offsets[0] == 0, "offsets must start at 0");
    for (int i = 0; i < num_instances; ++i) {
        int64_t ni = sample_offsets[i + 1] - sample_offsets[i], mi = query_offsets[i + 1] - query_offsets[i];
        SDFI_CHECK_ARG(grids[i] > 0 && (int64_t)grids[i] * grids[i] * grids[i] == ni && mi == 8 * ni,
                       "instance %d: grid %d needs grid^3 samples and 8x as many queries", i, grids[i]);
    }
    const int64_t n = sample_offsets[num_instances], m = query_offsets[num_instances];
    SDFI_CHECK_ARG(n + m < (int64_t(1) << 31), "total size out of range");
    SDFI_CHECK_ARG(samples && queries && values && order_out && active && kind && witness, "null array argument");
    size_t need = greedy_ws(n + num_instances, m, o) + (size_t)num_instances * greedy_instance_ws(o);
    if (ws_bytes < need || !ws) {
        set_error("workspace of %zu bytes is below the %zu required", ws_bytes, need);
        return SDFI_ERR_WORKSPACE;
    }
    return greedy_common(num_instances, sample_offsets, query_offsets, grids, samples, queries, nullptr, values,
                         order_out, active, kind, witness, nullptr, report, ws, ws_bytes, o, to_hip(stream));
}
