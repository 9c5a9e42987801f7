// Device geometry of the exact validity tests (Prop. 1 (ii)) and of the
// minimum valid radius (proof of Prop. 2), in float64, one wavefront each.
//
// A ball (p, s) covers point x of sphere (o, r) when |x - p| < |s| - tol.
// In unit directions v = (x - o)/r that is the open cap v.u > c with
//   u = (p - o)/D, c = (r^2 + D^2 - R^2)/(2 r D), D = |p - o|, R = |s| - tol.
// The rim of cap e is v(t) = c_e u_e + rho_e (cos t e1 + sin t e2); cap f
// covers the open arc A cos t + B sin t > K of that rim with
//   A = rho_e e1.u_f, B = rho_e e2.u_f, K = c_f - c_e u_e.u_f.
// Rim points are kept as unit vectors P = (cos t, sin t): an arc is its
// centre direction C = (A, B)/|(A, B)| and its half-width beta, cos beta =
// K/|(A, B)|, so its ends are C rotated by -beta and +beta and no angle is
// ever formed; advances along the rim are ordered by a monotone stand-in for
// the angle (no trigonometric function is evaluated anywhere).
//
// Rim walk.  Starting at a point, if some arcs cover it, jump to the
// farthest end among them; stop at the first point no arc covers or when the
// start is passed (rim covered).  Each arc is jumped over at most once per turn.
//
// Lazy search.  A sphere with caps K has an uncovered point iff it has one
// w.r.t. every subset; the search keeps a working subset K' (<= KMAX caps in
// LDS), finds uncovered points w.r.t. K' by rim walks, and verifies them
// against all caps.  A verified point is a true witness; a candidate covered
// by cap f adds f to K'.  If K' covers the sphere, so does K.  The nearest
// uncovered point to q is found the same way: the K'-nearest point is never
// farther than the true one, so a verified K'-nearest point is the answer.
// When K' is full the search falls back to walking every rim of K.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

namespace sdfi {
namespace geom {

constexpr int KMAX = 128;            // working cap subset per wavefront
constexpr double NUDGE = 1e-7;       // witnesses move this far (rad) off the rim they sit on
constexpr double COVER_EPS = 1e-13;  // cover margins v.u - c up to this count as uncovered (rounding)
constexpr int FALLBACK_LDS = 512;     // cap list of the exhaustive search held in LDS
constexpr int FALLBACK_GLOBAL = 8192;  // cap list held in global scratch (a wavefront's share of the workspace)

enum { ST_NONE = 0, ST_FOUND = 1, ST_NUMERIC = 2 };

struct Cap {
    double u[3];
    double c;
};

// The balls of a search: rows [0, N) of p4 (x, y, z, s), plus an optional
// extra ball, minus ball `skip`.  Balls are shrunk by `tol`.  With `lb < inf`
// only balls with |lq - p| < |s| + lb take part (a local set: balls that can
// cover a point within lb of lq).
struct Balls {
    const double *p4 = nullptr;
    int64_t N = 0;
    double extra[4] = {0.0, 0.0, 0.0, 0.0};
    int has_extra = 0;
    double tol = 0.0;
    int64_t skip = -1;
    double lq[3] = {0.0, 0.0, 0.0};
    double lb = INFINITY;
    const int64_t *idx = nullptr;    // optional: the balls are rows idx[0..N) of p4 instead of [0, N)
    const int32_t *idx32 = nullptr;  // the same with 32-bit row indices (a search's own compacted list)
    // optional region of interest on the searched sphere, the cap {v : v.ru >= rc}
    // (rs = sqrt(1 - rc^2)); caps that cannot meet it are ignored.  Exact for
    // every question asked about points of the region.
    int use_region = 0;
    double ru[3] = {0.0, 0.0, 0.0}, rc = -1.0, rs = 0.0;
    // searches over these balls skip the subset rounds and go straight to
    // the exhaustive rim walk (testing that path)
    int walk_only = 0;
};

__device__ inline double dot3(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

__device__ inline double dist3(const double *a, const double *b) {
#pragma clang fp contract(off)
    double dx = a[0] - b[0], dy = a[1] - b[1], dz = a[2] - b[2];
    return sqrt(dx * dx + dy * dy + dz * dz);
}

__device__ inline int64_t ball_row(const Balls &B, int64_t f) {
    return B.idx32 ? (int64_t)B.idx32[f] : (B.idx ? B.idx[f] : f);
}
__device__ inline const double *ball_ptr(const Balls &B, int64_t f) {
    if (f >= B.N) return B.extra;
    return B.p4 + 4 * ball_row(B, f);
}
__device__ inline int64_t ball_count(const Balls &B) { return B.N + (B.has_extra ? 1 : 0); }

// cap of ball f on sphere (o, r): 0 = no cap, 1 = cap written, 2 = the ball holds the whole sphere
__device__ inline int cap_of(const Balls &B, int64_t f, const double *o, double r, Cap &cap) {
#pragma clang fp contract(off)
    if (f == B.skip) return 0;
    const double *p = ball_ptr(B, f);
    if (B.lb < INFINITY && !(dist3(B.lq, p) < fabs(p[3]) + B.lb)) return 0;
    double R = fabs(p[3]) - B.tol;
    if (!(R > 0.0)) return 0;
    double v[3] = {p[0] - o[0], p[1] - o[1], p[2] - o[2]};
    double D = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
    if (D + r < R) return 2;
    if (!(D > 0.0) || !(fabs(D - r) < R)) return 0;
    cap.u[0] = v[0] / D;
    cap.u[1] = v[1] / D;
    cap.u[2] = v[2] / D;
    cap.c = (r * r + D * D - R * R) / (2.0 * r * D);
    if (B.use_region) {
        // two caps of angular radii a_f, a_q meet iff the angle between their axes
        // is below a_f + a_q: always when a_f + a_q >= pi (c_f <= -rc), otherwise
        // iff u_f.ru > cos(a_f + a_q) = c_f rc - s_f rs
        double cf = fmin(1.0, fmax(-1.0, cap.c));
        if (cf > -B.rc + 1e-12) {
            double sf = sqrt(fmax(0.0, 1.0 - cf * cf));
            if (!(dot3(cap.u, B.ru) > cf * B.rc - sf * B.rs - 1e-12)) return 0;
        }
    }
    return 1;
}

__device__ inline void basis(const double *u, double *e1, double *e2) {
    // e1 = u x a (a the x axis unless u is close to it), e2 = u x e1
    double a[3] = {1.0, 0.0, 0.0};
    if (fabs(u[0]) >= 0.9) {
        a[0] = 0.0;
        a[1] = 1.0;
    }
    e1[0] = u[1] * a[2] - u[2] * a[1];
    e1[1] = u[2] * a[0] - u[0] * a[2];
    e1[2] = u[0] * a[1] - u[1] * a[0];
    double n = sqrt(dot3(e1, e1));
    e1[0] /= n;
    e1[1] /= n;
    e1[2] /= n;
    e2[0] = u[1] * e1[2] - u[2] * e1[1];
    e2[1] = u[2] * e1[0] - u[0] * e1[2];
    e2[2] = u[0] * e1[1] - u[1] * e1[0];
}

struct Rim {
    double u[3], c, rho, e1[3], e2[3];
};

__device__ inline void make_rim(const Cap &cp, Rim &R) {
    R.u[0] = cp.u[0];
    R.u[1] = cp.u[1];
    R.u[2] = cp.u[2];
    R.c = cp.c;
    R.rho = sqrt(fmax(0.0, 1.0 - cp.c * cp.c));
    basis(cp.u, R.e1, R.e2);
}

// point of the rim at P = (cos t, sin t)
__device__ inline void rim_dir(const Rim &R, double px, double py, double *v) {
    for (int j = 0; j < 3; ++j) v[j] = R.c * R.u[j] + R.rho * (px * R.e1[j] + py * R.e2[j]);
}

struct Arc {
    double cx, cy;  // centre direction
    double k, s;    // cos and sin of the half-width
    double amp;     // |(A, B)|: the cover margin v.u_f - c_f at P is amp (C.P - k)
};

// arc of cap f on rim R: returns 0 none, 1 arc, 2 whole rim
__device__ inline int arc_of(const Rim &R, const Cap &f, Arc &a) {
    const double A = R.rho * dot3(R.e1, f.u), Bc = R.rho * dot3(R.e2, f.u);
    const double K = f.c - R.c * dot3(R.u, f.u);
    const double amp = sqrt(A * A + Bc * Bc);
    if (K < -amp) return 2;
    if (!(amp > K)) return 0;
    a.cx = A / amp;
    a.cy = Bc / amp;
    a.k = fmin(1.0, fmax(-1.0, K / amp));
    a.s = sqrt(fmax(0.0, 1.0 - a.k * a.k));
    a.amp = amp;
    return 1;
}

// the same test as the cover scans (margin v.u_f - c_f > COVER_EPS), so that a
// point the walk leaves uncovered is not found covered by a cap of the walk
__device__ inline bool arc_covers(const Arc &a, double px, double py) {
    return a.amp * (a.cx * px + a.cy * py - a.k) > COVER_EPS;
}

// dir > 0: the end met walking forward (C rotated by +beta); dir < 0: the start
__device__ inline void arc_end(const Arc &a, int dir, double &ex, double &ey) {
    const double s = dir > 0 ? a.s : -a.s;
    ex = a.cx * a.k - a.cy * s;
    ey = a.cy * a.k + a.cx * s;
}

// increasing function of the forward angle in [0, 2 pi) from P to E
__device__ inline double pseudo_angle(double px, double py, double ex, double ey) {
    const double d = px * ex + py * ey, cr = px * ey - py * ex;
    return cr >= 0.0 ? 1.0 - d : 3.0 + d;
}

// Caps of a rim walk: the wave's working subset, or every cap of the sphere.
struct SubsetCaps {
    const Cap *kp;
    int k;
    __device__ int64_t count() const { return k; }
    __device__ bool get(int64_t f, Cap &c) const {
        c = kp[f];
        return true;
    }
};
struct ListCaps {
    const Balls *B;
    const double *o;
    double r;
    const int32_t *cl;  // ball indices of B with a cap on the sphere
    int cnt;
    __device__ int64_t count() const { return cnt; }
    __device__ bool get(int64_t f, Cap &c) const { return cap_of(*B, cl ? (int64_t)cl[f] : f, o, r, c) == 1; }
};

// Walk rim R over the caps of `src` (skipping index `self`) from P0 in
// direction dir (+1 forward to arc ends, -1 backward to arc starts).
// Returns 1 with the first uncovered point and whether the walk moved, 0 if
// the rim is covered, 2 if the step cap was hit.
template <class Src>
__device__ inline int rim_walk(const Rim &R, const Src &src, int64_t self, double p0x, double p0y, int dir,
                               int64_t max_it, double *px_out, double *py_out, int *moved) {
    double px = p0x, py = p0y;
    int mv = 0;
    const int64_t k = src.count();
    for (int64_t it = 0; it <= max_it; ++it) {
        bool cov = false;
        double best = -1.0, bx = px, by = py;
        for (int64_t f = 0; f < k; ++f) {
            if (f == self) continue;
            Cap cf;
            if (!src.get(f, cf)) continue;
            Arc a;
            const int st = arc_of(R, cf, a);
            if (st == 2) return 0;
            if (st == 0 || !arc_covers(a, px, py)) continue;
            cov = true;
            double ex, ey;
            arc_end(a, dir, ex, ey);
            const double pa = dir > 0 ? pseudo_angle(px, py, ex, ey) : pseudo_angle(ex, ey, px, py);
            if (pa > best) {
                best = pa;
                bx = ex;
                by = ey;
            }
        }
        if (!cov) {
            *px_out = px;
            *py_out = py;
            *moved = mv;
            return 1;
        }
        // a full turn: the start lies in the stretch (P, E] about to be jumped
        if (mv) {
            const double ps = dir > 0 ? pseudo_angle(px, py, p0x, p0y) : pseudo_angle(p0x, p0y, px, py);
            if (ps <= best) return 0;
        }
        const double nn = sqrt(bx * bx + by * by);
        px = bx / nn;
        py = by / nn;
        mv = 1;
    }
    return 2;
}

// Midpoint of the uncovered stretch that starts at P (forward) among caps
// kp[0..k) other than `self`.
__device__ inline void gap_mid(const Rim &R, const Cap *kp, int k, int self, double px, double py, double *mx,
                               double *my) {
    double best = 5.0, sx = 0.0, sy = 0.0;
    for (int f = 0; f < k; ++f) {
        if (f == self) continue;
        Arc a;
        if (arc_of(R, kp[f], a) != 1) continue;
        double ex, ey;
        arc_end(a, -1, ex, ey);
        const double pa = pseudo_angle(px, py, ex, ey);
        if (pa < best) {
            best = pa;
            sx = ex;
            sy = ey;
        }
    }
    if (best > 4.0) {  // no arc: the whole rim is free, take the antipode
        *mx = -px;
        *my = -py;
        return;
    }
    const double hx = px + sx, hy = py + sy, hn = sqrt(hx * hx + hy * hy);
    if (hn < 1e-8) {  // half a turn: a quarter turn forward
        *mx = -py;
        *my = px;
        return;
    }
    const double sg = best <= 2.0 ? 1.0 : -1.0;
    *mx = sg * hx / hn;
    *my = sg * hy / hn;
}

// ---- wave-level helpers (all 64 lanes call them together) ----

__device__ inline double wmax(double v) {
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ inline double wmin(double v) {
    for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ inline int64_t wmin_i64(int64_t v) {
    for (int o = 32; o > 0; o >>= 1) {
        int64_t w = __shfl_xor(v, o, 64);
        v = w < v ? w : v;
    }
    return v;
}
__device__ inline void wave_sync_lds() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

__device__ inline int wor(int v) {
    for (int o = 32; o > 0; o >>= 1) v |= __shfl_xor(v, o, 64);
    return v;
}

// Largest cover margin v.u_f - c_f over all caps of the sphere (ball `excl`
// left out) and the smallest ball index attaining it; also reports a ball
// holding the whole sphere.  margin > 0 means v is covered.
//
// The cap margin equals (R^2 - |x - p|^2) / (2 r D) for x = o + r v, so balls
// with R^2 - |x - p|^2 <= -PRE_EPS neither cover x nor hold the sphere and are
// skipped before the cap is formed (PRE_EPS is far above the rounding of
// either expression, so no ball that the cap form would count is skipped).
// Balls are read U rows per lane at a time so that their loads overlap.
constexpr double PRE_EPS = 1e-12;

// Does ball f hold every point of the region of interest of sphere (o, r)?
// The region cap (axis ru, angular radius a) lies inside the open cap of f
// (axis u, angular radius b > a) iff angle(ru, u) < b - a, i.e.
// ru.u > cos(b - a) = c rc + sin(b) rs; decided with a margin.
__device__ inline bool region_held(const Balls &B, const Cap &cp) {
    if (!(cp.c < B.rc - 1e-12)) return false;
    const double sb = sqrt(fmax(0.0, 1.0 - cp.c * cp.c));
    return dot3(B.ru, cp.u) > cp.c * B.rc + sb * B.rs + 1e-12;
}

__device__ inline void wave_cover(const Balls &B, const double *o, double r, const double *v, int64_t excl,
                                  double *mx, int64_t *arg, int *whole, int *holds_region = nullptr,
                                  int64_t *holder = nullptr) {
    constexpr int U = 4;
    const int lane = threadIdx.x & 63;
    const double x[3] = {o[0] + r * v[0], o[1] + r * v[1], o[2] + r * v[2]};
    double best = -INFINITY;
    int64_t bi = INT64_MAX, hi = INT64_MAX;
    int wh = 0, hr = 0;
    const bool region = holds_region && B.use_region;
    const int64_t n = ball_count(B);
    for (int64_t f0 = 0; f0 < n; f0 += 64 * U) {
        double px[U], py[U], pz[U], ps[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t f = f0 + 64 * u + lane;
            const double *p = ball_ptr(B, f < n ? f : n - 1);
            px[u] = p[0];
            py[u] = p[1];
            pz[u] = p[2];
            ps[u] = p[3];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t f = f0 + 64 * u + lane;
            const double R = fabs(ps[u]) - B.tol;
            const double dx = x[0] - px[u], dy = x[1] - py[u], dz = x[2] - pz[u];
            const double pre = R * R - (dx * dx + dy * dy + dz * dz);
            if (f >= n || f == excl || !(R > 0.0) || !(pre > -PRE_EPS)) continue;
            Cap cp;
            int s = cap_of(B, f, o, r, cp);
            if (s == 2) {
                wh = 1;
                continue;
            }
            if (s == 0) continue;
            double m = dot3(v, cp.u) - cp.c;
            if (m > best) {
                best = m;
                bi = f;
            }
            if (region && region_held(B, cp)) {
                hr = 1;
                hi = hi < f ? hi : f;
            }
        }
        // a holder settles the caller's question; the margins are not needed then
        if (holder && wor(hr)) break;
    }
    double g = wmax(best);
    int64_t cand = (best == g) ? bi : INT64_MAX;
    *mx = g;
    *arg = wmin_i64(cand);
    *whole = wor(wh);
    if (holds_region) *holds_region = wor(hr);
    if (holder) *holder = wmin_i64(hi);
}

// The indices of the balls with a cap on sphere (o, r), in index order, into
// cl (this wave's list of ccap entries, LDS or global); returns their number,
// which may exceed ccap (then the list holds the first ccap only).
__device__ inline int wave_list_caps(const Balls &B, const double *o, double r, int32_t *cl, int ccap) {
    const int lane = threadIdx.x & 63;
    int cnt = 0;
    const int64_t n = ball_count(B);
    for (int64_t f0 = 0; f0 < n; f0 += 64) {
        const int64_t f = f0 + lane;
        Cap cp;
        const int take = f < n && cap_of(B, f, o, r, cp) == 1;
        const unsigned long long m = __ballot(take);
        const int pos = cnt + (int)__popcll(m & ((1ull << lane) - 1ull));
        if (take && pos < ccap) cl[pos] = (int32_t)f;
        cnt += (int)__popcll(m);
    }
    __threadfence_block();
    wave_sync_lds();
    return cnt;
}

// wave_cover at v together with the list of the balls that have a cap on the
// sphere: their rows of B.p4 in index order into cl (ccap entries; the extra
// ball is reported apart).  *cnt: listed rows (may exceed ccap); *ecap: the
// extra ball has a cap; *argpos: the position of *arg in the list (*cnt for
// the extra ball).  A ball meets the sphere iff |r - R| < D < r + R; the
// squared test only skips balls clearly apart, cap_of decides the rest.
__device__ inline void wave_cover_list(const Balls &B, const double *o, double r, const double *v, double *mx,
                                       int64_t *arg, int *whole, int32_t *cl, int ccap, int *cnt_out, int *ecap,
                                       int64_t *argpos, int64_t fb = 0, int64_t fe = -1) {
    const int lane = threadIdx.x & 63;
    double best = -INFINITY;
    int64_t bi = INT64_MAX, bp = INT64_MAX;
    int wh = 0, ec = 0, cnt = 0;
    const int64_t n = fe < 0 ? ball_count(B) : fe;  // balls [fb, n) of B
    for (int64_t f0 = fb; f0 < n; f0 += 64) {
        const int64_t f = f0 + lane;
        int take = 0;
        double m = -INFINITY;
        if (f < n && f != B.skip) {
            const double *p = ball_ptr(B, f);
            const double R = fabs(p[3]) - B.tol;
            const double dx = p[0] - o[0], dy = p[1] - o[1], dz = p[2] - o[2];
            const double D2 = dx * dx + dy * dy + dz * dz;
            const bool apart = !(R > 0.0) || D2 > (r + R) * (r + R) * (1.0 + 1e-12) + 1e-300 ||
                               (R < r && D2 < (r - R) * (r - R) * (1.0 - 1e-12));
            if (!apart) {
                Cap cp;
                const int st = cap_of(B, f, o, r, cp);
                if (st == 2) wh = 1;
                if (st == 1) {
                    m = dot3(v, cp.u) - cp.c;
                    if (f < B.N) take = 1;
                    else ec = 1;
                }
            }
        }
        const unsigned long long bal = __ballot(take);
        const int pos = cnt + (int)__popcll(bal & ((1ull << lane) - 1ull));
        if (take && pos < ccap) cl[pos] = (int32_t)ball_row(B, f);
        if (m > best) {
            best = m;
            bi = f;
            bp = f < B.N ? pos : -1;  // -1: the extra ball, placed after the rows
        }
        cnt += (int)__popcll(bal);
    }
    __threadfence_block();
    wave_sync_lds();
    const double g = wmax(best);
    const int64_t cand = (best == g) ? bi : INT64_MAX;
    *mx = g;
    *arg = wmin_i64(cand);
    const int64_t pc = (best == g && bi == *arg) ? bp : INT64_MAX;
    const int64_t ap = wmin_i64(pc == -1 ? (int64_t)cnt : pc);
    *argpos = ap;
    *whole = wor(wh);
    *ecap = wor(ec);
    *cnt_out = cnt;
}

__device__ inline int lazy_exist_rest(const Balls &B0, const double *o, double r, const double *vh, Cap *kp,
                                      int64_t *kid, int32_t *cl, int ccap, double *x, unsigned long long *walks,
                                      double mx, int64_t arg, int whole, int ncl, int ecap, int64_t argpos);

// Exact: does sphere (o, r) have a point no ball covers?  Writes one (nudged
// off the rim it was found on) to x.  kp: this wave's LDS scratch (KMAX caps),
// kid: their ball indices.  hint orders the search only.
__device__ inline int lazy_exist(const Balls &B0, const double *o, double r, const double *hint, Cap *kp,
                                 int64_t *kid, int32_t *cl, int ccap, double *x,
                                 unsigned long long *walks = nullptr) {
    const int lane = threadIdx.x & 63;
    Balls B = B0;
    if (!(r > 0.0)) {
        // a sphere of radius 0 is its centre: covered iff |o - p| < |s| - tol for some ball
        double best = -INFINITY;
        const int64_t n = ball_count(B);
        for (int64_t f = lane; f < n; f += 64) {
            if (f == B.skip) continue;
            const double *p = ball_ptr(B, f);
            if (B.lb < INFINITY && !(dist3(B.lq, p) < fabs(p[3]) + B.lb)) continue;
            best = fmax(best, fabs(p[3]) - B.tol - dist3(o, p));
        }
        if (wmax(best) > 0.0) return ST_NONE;
        x[0] = o[0];
        x[1] = o[1];
        x[2] = o[2];
        return ST_FOUND;
    }
    double vh[3] = {1.0, 0.0, 0.0};
    if (hint) {
        double g[3] = {hint[0] - o[0], hint[1] - o[1], hint[2] - o[2]};
        double gn = sqrt(dot3(g, g));
        if (gn > 0.0) {
            vh[0] = g[0] / gn;
            vh[1] = g[1] / gn;
            vh[2] = g[2] / gn;
        }
    }
    double mx;
    int64_t arg;
    int whole;
    // the first test also lists the balls that meet the sphere; when they fit
    // in cl the rest of the search runs over that list only
    int ncl = 0, ecap = 0;
    int64_t argpos = 0;
    wave_cover_list(B, o, r, vh, &mx, &arg, &whole, cl, ccap, &ncl, &ecap, &argpos);
    return lazy_exist_rest(B, o, r, vh, kp, kid, cl, ccap, x, walks, mx, arg, whole, ncl, ecap, argpos);
}

// Step 1 of a round of the lazy search: each lane walks rims lane and
// lane + 64 of the working subset kp[0..k) and keeps the first gap it finds:
// found, the rim's index frim, the rim R and the gap's midpoint (mxp, myp)
// in its frame; numeric when a walk hit its step cap.
__device__ inline void subset_gap(const Cap *kp, int k, int &found, int &numeric, int &frim, Rim &R, double &mxp,
                                  double &myp) {
    const int lane = threadIdx.x & 63;
    const SubsetCaps sub{kp, k};
    found = 0;
    numeric = 0;
    frim = -1;
    mxp = 0.0;
    myp = 0.0;
    for (int e = lane; e < k && !found; e += 64) {
        make_rim(kp[e], R);
        double px, py;
        int mv;
        const int st = rim_walk(R, sub, e, 1.0, 0.0, 1, k + 4, &px, &py, &mv);
        if (st == 1) {
            found = 1;
            frim = e;
            gap_mid(R, kp, k, e, px, py, &mxp, &myp);
        } else if (st == 2) {
            numeric = 1;
        }
    }
}

// A verified uncovered direction v on the rim of cap `rim`: moved off that rim
// (into the gap) by NUDGE when the moved point is still uncovered (one wave).
__device__ inline void nudge_off_rim(const Balls &B, const double *o, double r, const Cap &rim, double *v) {
    const double uv = dot3(rim.u, v);
    const double tg[3] = {rim.u[0] - uv * v[0], rim.u[1] - uv * v[1], rim.u[2] - uv * v[2]};
    const double tn = sqrt(dot3(tg, tg));
    if (tn > 0.0) {
        double w[3] = {v[0] - NUDGE * tg[0] / tn, v[1] - NUDGE * tg[1] / tn, v[2] - NUDGE * tg[2] / tn};
        const double wn = sqrt(dot3(w, w));
        w[0] /= wn;
        w[1] /= wn;
        w[2] /= wn;
        double m2;
        int64_t a2;
        int wh2;
        wave_cover(B, o, r, w, -1, &m2, &a2, &wh2);
        if (!(m2 > COVER_EPS)) {
            v[0] = w[0];
            v[1] = w[1];
            v[2] = w[2];
        }
    }
}

// The balls of the search after the first cover test: the listed balls that
// meet the sphere when they all fit in cl (positions into cl, the extra ball
// after them), else B itself.
__device__ inline Balls search_balls(const Balls &B, int32_t *cl, int ncl, int ccap, int ecap) {
    if (ncl > ccap) return B;
    Balls C = B;
    C.N = ncl;
    C.idx = nullptr;
    C.idx32 = cl;
    C.skip = -1;
    C.lb = INFINITY;
    C.has_extra = B.has_extra && ecap;
    return C;
}

__device__ inline int exist_fallback(const Balls &B, const double *o, double r, int32_t *cl, int ccap, bool compact,
                                     double *x, unsigned long long *walks);

// lazy_exist after its first cover test at direction vh: margin mx at ball
// arg (position argpos in the list), whole-sphere holder found, the ncl balls
// meeting the sphere listed in cl (when ncl <= ccap), the extra ball meets it
// (ecap).
__device__ inline int lazy_exist_rest(const Balls &B0, const double *o, double r, const double *vh, Cap *kp,
                                      int64_t *kid, int32_t *cl, int ccap, double *x, unsigned long long *walks,
                                      double mx, int64_t arg, int whole, int ncl, int ecap, int64_t argpos) {
    const int lane = threadIdx.x & 63;
    if (whole) return ST_NONE;
    if (!(mx > COVER_EPS)) {
        for (int j = 0; j < 3; ++j) x[j] = o[j] + r * vh[j];
        return ST_FOUND;
    }
    const bool compact = ncl <= ccap;
    const Balls B = search_balls(B0, cl, ncl, ccap, ecap);
    if (compact) arg = argpos;
    int k = 0;
    if (lane == 0) {
        kid[0] = arg;
        cap_of(B, arg, o, r, kp[0]);
    }
    k = 1;
    wave_sync_lds();
    for (int round = 0; round < (B.walk_only ? 0 : 4 * KMAX); ++round) {
        // 1. uncovered gap midpoints w.r.t. the working subset
        int found, numeric, frim;
        double mxp, myp;
        Rim R;
        subset_gap(kp, k, found, numeric, frim, R, mxp, myp);
        if (!wor(found)) {
            if (wor(numeric)) break;  // no proof of coverage: fall back
            return ST_NONE;           // the subset covers the sphere
        }
        // 2. verify candidates in lane order; collect the cap covering each
        int added = 0;
        for (int cl = 0; cl < 64; ++cl) {
            const int f_cl = __shfl(found, cl, 64);
            if (!f_cl) continue;
            const int rim_cl = __shfl(frim, cl, 64);
            double v[3] = {0.0, 0.0, 0.0};
            if (lane == cl) rim_dir(R, mxp, myp, v);
            v[0] = __shfl(v[0], cl, 64);
            v[1] = __shfl(v[1], cl, 64);
            v[2] = __shfl(v[2], cl, 64);
            const int64_t self = kid[rim_cl];
            wave_cover(B, o, r, v, self, &mx, &arg, &whole);
            if (!(mx > COVER_EPS)) {
                // verified; try to move it off the rim of `self`
                nudge_off_rim(B, o, r, kp[rim_cl], v);
                for (int j = 0; j < 3; ++j) x[j] = o[j] + r * v[j];
                return ST_FOUND;
            }
            // add the covering cap unless already present
            bool have = false;
            for (int e = 0; e < k; ++e) have |= (kid[e] == arg);
            if (!have && k < KMAX) {
                if (lane == 0) {
                    kid[k] = arg;
                    cap_of(B, arg, o, r, kp[k]);
                }
                wave_sync_lds();
                ++k;
                ++added;
            }
        }
        wave_sync_lds();
        if (added == 0) break;  // subset full or no progress: fall back
    }
    return exist_fallback(B, o, r, cl, ccap, compact, x, walks);
}

// The last resort of the existence search (one wave).
__device__ inline int exist_fallback(const Balls &B, const double *o, double r, int32_t *cl, int ccap, bool compact,
                                     double *x, unsigned long long *walks) {
    const int lane = threadIdx.x & 63;
    // Fallback: walk every rim of every cap (lanes over rims) against the
    // listed caps.  Its cost grows with the cube of the cap count, so it is
    // bounded by the list's size ccap: beyond it the search reports a numeric
    // failure.
    // (after compaction every ball of B has a cap and B's own list stands in)
    if (walks && lane == 0) atomicAdd(walks, 1ull);  // searches that reach the exhaustive walk
    const int ncap = compact ? (int)ball_count(B) : wave_list_caps(B, o, r, cl, ccap);
    if (!compact && ncap > ccap) return ST_NUMERIC;  // the list holds only the first ccap
    const int32_t *lst = compact ? nullptr : cl;
    const ListCaps all{&B, o, r, lst, ncap};
    for (int e0 = 0; e0 < ncap; e0 += 64) {
        const int e = e0 + lane;
        int64_t first = INT64_MAX;
        double fx[3] = {0.0, 0.0, 0.0};
        Cap ce;
        if (e < ncap && cap_of(B, lst ? (int64_t)lst[e] : (int64_t)e, o, r, ce) == 1) {
            Rim R;
            make_rim(ce, R);
            double px, py;
            int mv;
            if (rim_walk(R, all, e, 1.0, 0.0, 1, ncap + 8, &px, &py, &mv) == 1) {
                first = e;
                double v[3];
                rim_dir(R, px, py, v);
                for (int j = 0; j < 3; ++j) fx[j] = o[j] + r * v[j];
            }
        }
        const int64_t g = wmin_i64(first);
        if (g != INT64_MAX) {
            const int src = (int)(g - e0);
            for (int j = 0; j < 3; ++j) x[j] = __shfl(fx[j], src, 64);
            return ST_FOUND;
        }
    }
    return ST_NONE;
}

// lazy_exist kept out of line, for callers whose own code it would bloat (the
// greedy's candidate check; a nearest search whose q is the sphere's centre)
__device__ __noinline__ int lazy_exist_call(const Balls &B, const double *o, double r, const double *hint, Cap *kp,
                                            int64_t *kid, int32_t *cl, int ccap, double *x,
                                            unsigned long long *walks = nullptr) {
    return lazy_exist(B, o, r, hint, kp, kid, cl, ccap, x, walks);
}

// The region of interest of a nearest search: the points of sphere (o, r)
// within `bound` of q, the cap {v : v.g/|g| >= rc} with g = q - o.  Returns
// 0 when no point of the sphere is that close; else 1, with B's region set
// (use_region 0 when the region is the whole sphere).
__device__ inline int set_region(Balls &B, const double *o, double r, const double *q, double bound) {
    const double g[3] = {q[0] - o[0], q[1] - o[1], q[2] - o[2]};
    const double gn = sqrt(dot3(g, g));
    B.use_region = 0;
    if (bound < INFINITY && gn > 0.0) {
        const double rc = (r * r + gn * gn - bound * bound) / (2.0 * r * gn);
        if (rc > 1.0) return 0;
        if (rc > -1.0) {
            B.use_region = 1;
            B.ru[0] = g[0] / gn;
            B.ru[1] = g[1] / gn;
            B.ru[2] = g[2] / gn;
            B.rc = rc;
            B.rs = sqrt(fmax(0.0, 1.0 - rc * rc));
        }
    }
    if (gn > 0.0 && fabs(gn - r) > bound) return 0;  // the nearest point of the sphere is farther
    return 1;
}

// Does one of the balls ring[0..nh) (indices of B, -1 empty, read as they
// stand) hold every point of B's region?  Exact for each ball read.
__device__ inline bool held_by(const Balls &B, const double *o, double r, const int64_t *ring, int nh) {
    if (!B.use_region) return false;
    for (int j = 0; j < nh; ++j) {
        const int64_t f = __hip_atomic_load(&ring[j], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (f < 0 || f >= ball_count(B)) continue;
        Cap ch;
        const int st = cap_of(B, f, o, r, ch);
        if (st == 2 || (st == 1 && region_held(B, ch))) return true;
    }
    return false;
}

// Recently seen balls that held a whole search region (ball indices, -1
// empty): a ring of NHOLD entries shared by the wavefronts of a work-group
// (LDS) or of a team of groups (global memory).  Entries may be replaced while another wave reads them; any
// ball index read is a valid ball, and the holding test is exact for it.
constexpr int NHOLD = 32;
struct Holders {
    int64_t *h;  // NHOLD entries
    int *next;   // ring position (LDS)
    // optional search profile: early, first, loop, rounds, fallback, first
    // ticks, loop ticks, fallback ticks, fallback caps, stalled rounds, early
    // ticks
    unsigned long long *prof = nullptr;
    __device__ void note(int k, unsigned long long v) {
        if (prof && (threadIdx.x & 63) == 0) atomicAdd(&prof[k], v);
    }
    __device__ void push(int64_t f) {
        if ((threadIdx.x & 63) == 0) {
            const int slot = atomicAdd(next, 1) & (NHOLD - 1);
            __hip_atomic_store(&h[slot], f, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
};

// Nearest point to q of the uncovered part of sphere (o, r) if nearer than
// bound (strictly less or equal kept: ties are broken by the caller).
// Returns 0 none, 1 radial foot point (T), 2 rim nearest point (D), 3 rim arc
// end (U), -1 numeric failure; writes distance and point.
__device__ __noinline__ int lazy_nearest(const Balls &B0, const double *o, double r, const double *q, double bound, Cap *kp,
                                   int64_t *kid, int32_t *cl, int ccap, double *dist_out, double *x,
                                   Holders *hold = nullptr) {
    const int lane = threadIdx.x & 63;
    const unsigned long long t_enter = (hold && hold->prof) ? wall_clock64() : 0ull;
    double g[3] = {q[0] - o[0], q[1] - o[1], q[2] - o[2]};
    double gn = sqrt(dot3(g, g));
    // only points of the sphere within `bound` of q matter: the cap v.g/|g| >= rc
    Balls B = B0;
    if (!set_region(B, o, r, q, bound) && gn > 0.0) {
        if (hold) hold->note(0, 1);
        if (hold) hold->note(10, wall_clock64() - t_enter);
        return 0;  // no point of the sphere is that close
    }
    double mx;
    int64_t arg;
    int whole;
    if (!(gn > 0.0)) {
        if (r > bound) return 0;
        int s = lazy_exist_call(B, o, r, nullptr, kp, kid, cl, ccap, x);
        if (s == ST_NUMERIC) {
            *dist_out = r;
            return -1;
        }
        if (s != ST_FOUND) return 0;
        *dist_out = r;
        return 1;
    }
    double v0[3] = {g[0] / gn, g[1] / gn, g[2] / gn};
    double d0 = fabs(gn - r);
    // a single ball holding every point of the sphere within the bound ends
    // the search; the balls that did so recently (ball indices of B0) are
    // tried on their own first
    int held = 0;
    if (hold && B.use_region) {
        // one recent holder per lane
        if (wor(lane < NHOLD && held_by(B, o, r, hold->h + lane, 1))) {
            hold->note(0, 1);
            hold->note(10, wall_clock64() - t_enter);
            return 0;
        }
    }
    int64_t hnew = INT64_MAX;
    const unsigned long long t_first = (hold && hold->prof) ? wall_clock64() : 0ull;
    wave_cover(B, o, r, v0, -1, &mx, &arg, &whole, &held, hold ? &hnew : nullptr);
    if (hold) hold->note(5, wall_clock64() - t_first);
    if (held && hold) hold->push(hnew);
    if (whole || held || !(mx > COVER_EPS)) {
        if (hold) hold->note(1, 1);
    } else if (hold) {
        hold->note(2, 1);
    }
    if (whole || held) return 0;
    if (!(mx > COVER_EPS)) {
        for (int j = 0; j < 3; ++j) x[j] = o[j] + r * v0[j];
        *dist_out = d0;
        return 1;
    }
    const unsigned long long t_loop = (hold && hold->prof) ? wall_clock64() : 0ull;
    struct LoopTicks {
        Holders *h;
        unsigned long long t;
        __device__ ~LoopTicks() {
            if (h) h->note(6, wall_clock64() - t);
        }
    } loop_ticks{hold, t_loop};
    int k = 1;
    if (lane == 0) {
        kid[0] = arg;
        cap_of(B, arg, o, r, kp[0]);
    }
    wave_sync_lds();
    double lowest = d0;  // every uncovered point is at least this far from q
    for (int round = 0; round < (B.walk_only ? 0 : 8 * KMAX); ++round) {
        if (hold) hold->note(3, 1);
        const SubsetCaps sub{kp, k};
        double cd = INFINITY, cpx = 0.0, cpy = 0.0;
        int ckind = 0, crim = -1;
        Rim R, Rb;
        for (int e = lane; e < k; e += 64) {
            make_rim(kp[e], R);
            // lower bound: distance from q to the rim circle
            const double ug = dot3(R.u, g);
            const double perp = sqrt(fmax(gn * gn - ug * ug, 0.0));
            const double vg = R.c * ug + R.rho * perp;
            const double lbd = sqrt(fmax(r * r + gn * gn - 2.0 * r * vg, 0.0));
            if (!(lbd <= bound)) continue;
            // the rim point nearest q, then the nearest uncovered one on either side
            double sx = dot3(R.e1, g), sy = dot3(R.e2, g);
            const double sn = sqrt(sx * sx + sy * sy);
            if (sn > 0.0) {
                sx /= sn;
                sy /= sn;
            } else {
                sx = 1.0;
                sy = 0.0;
            }
            double fx, fy, bx, by;
            int fm, bm, kind_e = 0;
            double tx = 0.0, ty = 0.0;
            const int sp = rim_walk(R, sub, e, sx, sy, 1, k + 4, &fx, &fy, &fm);
            if (sp == 1 && !fm) {
                tx = sx;
                ty = sy;
                kind_e = 2;
            } else if (sp == 1) {
                const int sm = rim_walk(R, sub, e, sx, sy, -1, k + 4, &bx, &by, &bm);
                const bool back = sm == 1 && pseudo_angle(bx, by, sx, sy) < pseudo_angle(sx, sy, fx, fy);
                tx = back ? bx : fx;
                ty = back ? by : fy;
                kind_e = 3;
            }
            if (kind_e) {
                double v[3];
                rim_dir(R, tx, ty, v);
                const double y[3] = {o[0] + r * v[0], o[1] + r * v[1], o[2] + r * v[2]};
                const double de = dist3(y, q);
                if (de <= bound && de < cd) {
                    cd = de;
                    cpx = tx;
                    cpy = ty;
                    ckind = kind_e;
                    crim = e;
                    Rb = R;
                }
            }
        }
        const double best = wmin(cd);
        if (best == INFINITY) return 0;
        lowest = fmax(lowest, best);  // the subset-nearest distance never exceeds the true one
        // the lowest rim index with the best distance
        const int64_t cand = (cd == best && ckind) ? ((int64_t)crim << 8) + lane : INT64_MAX;
        const int64_t pick = wmin_i64(cand);
        if (pick == INT64_MAX) {  // no lane holds the best distance (NaN geometry): no answer
            *dist_out = lowest;
            return -1;
        }
        const int src = (int)(pick & 255);
        const int srim = (int)(pick >> 8);
        double v[3] = {0.0, 0.0, 0.0};
        if (lane == src) rim_dir(Rb, cpx, cpy, v);
        v[0] = __shfl(v[0], src, 64);
        v[1] = __shfl(v[1], src, 64);
        v[2] = __shfl(v[2], src, 64);
        const int kind = __shfl(ckind, src, 64);
        wave_cover(B, o, r, v, kid[srim], &mx, &arg, &whole, &held);
        if (held) return 0;
        if (!(mx > COVER_EPS)) {
            for (int j = 0; j < 3; ++j) x[j] = o[j] + r * v[j];
            *dist_out = best;
            return kind;
        }
        bool have = false;
        for (int e = 0; e < k; ++e) have |= (kid[e] == arg);
        if (have && hold) hold->note(9, 1);
        if (have || k >= KMAX) break;
        if (lane == 0) {
            kid[k] = arg;
            cap_of(B, arg, o, r, kp[k]);
        }
        wave_sync_lds();
        ++k;
    }
    // Fallback: every rim against every listed cap (bounded as in
    // lazy_exist).  When capped, return -1 with the last subset-nearest
    // distance, a lower bound.
    if (hold) hold->note(4, 1);
    struct FallbackTicks {
        Holders *h;
        unsigned long long t;
        __device__ ~FallbackTicks() {
            if (h) h->note(7, wall_clock64() - t);
        }
    } fallback_ticks{hold, (hold && hold->prof) ? wall_clock64() : 0ull};
    const int ncap = wave_list_caps(B, o, r, cl, ccap);
    if (hold) hold->note(8, (unsigned long long)ncap);
    if (ncap > ccap) {
        *dist_out = lowest;
        return -1;
    }
    const ListCaps all{&B, o, r, cl, ncap};
    double bd = INFINITY, bx[3] = {0.0, 0.0, 0.0};
    int bkind = 0;
    double wbest = bound;  // wave-wide best so far: rims farther than it are skipped
    for (int e0 = 0; e0 < ncap; e0 += 64) {
        const int e = e0 + lane;
        Cap ce;
        Rim R;
        bool live = e < ncap && cap_of(B, cl[e], o, r, ce) == 1;
        if (live) {
            make_rim(ce, R);
            const double ug = dot3(R.u, g);
            const double perp = sqrt(fmax(gn * gn - ug * ug, 0.0));
            const double lbd = sqrt(fmax(r * r + gn * gn - 2.0 * r * (R.c * ug + R.rho * perp), 0.0));
            live = lbd <= wbest * (1.0 + 1e-12) + 1e-15;  // a rim farther than the best cannot win
        }
        if (live) {
            double sx = dot3(R.e1, g), sy = dot3(R.e2, g);
            const double sn = sqrt(sx * sx + sy * sy);
            if (sn > 0.0) {
                sx /= sn;
                sy /= sn;
            } else {
                sx = 1.0;
                sy = 0.0;
            }
            for (int dir = 1; dir >= -1; dir -= 2) {
                double px, py;
                int mv;
                if (rim_walk(R, all, e, sx, sy, dir, ncap + 8, &px, &py, &mv) != 1) continue;
                double v[3];
                rim_dir(R, px, py, v);
                const double y[3] = {o[0] + r * v[0], o[1] + r * v[1], o[2] + r * v[2]};
                const double d = dist3(y, q);
                if (d < bd) {
                    bd = d;
                    bkind = mv ? 3 : 2;
                    bx[0] = y[0];
                    bx[1] = y[1];
                    bx[2] = y[2];
                }
            }
        }
        wbest = fmin(wbest, wmin(bd));
    }
    const double best = wmin(bd);
    if (!(best <= bound)) return 0;
    const int64_t cand = (bd == best) ? lane : INT64_MAX;
    const int src = (int)wmin_i64(cand);
    for (int j = 0; j < 3; ++j) x[j] = __shfl(bx[j], src, 64);
    *dist_out = best;
    return __shfl(bkind, src, 64);
}

}  // namespace geom
}  // namespace sdfi
