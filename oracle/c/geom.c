/* Plain C float64 helpers of the CPU oracle (test infrastructure only).
 *
 * Same definitions as oracle/spheres.py, written out as loops so the oracle
 * can run the greedy on test-sized inputs in seconds.  A point x is covered
 * by sample (p, s) when |x - p| < |s| - tol (touching is uncovered, Prop. 1).
 * On a sphere (o, r) every ball cuts an open cap {v : v.u > c}; the sphere
 * has an uncovered point iff no ball meets it or some cap rim keeps an
 * angle no other cap covers (the rim intersection points are the triple
 * points U of Def. 1, the rim points nearest a query are the points D).
 * Single-threaded, no vector intrinsics, no FMA contraction (-ffp-contract=off).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#define TWO_PI 6.283185307179586476925286766559

typedef struct { double u[3]; double c; } cap_t;
typedef struct { double a, b; } piece_t;

static double dist3(const double *a, const double *b)
{
    double dx = a[0] - b[0], dy = a[1] - b[1], dz = a[2] - b[2];
    return sqrt(dx * dx + dy * dy + dz * dz);
}

static double dot3(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

int og_point_covered(const double *x, const double *P, const double *S, long N, double tol)
{
    for (long i = 0; i < N; ++i)
        if (dist3(x, P + 3 * i) < fabs(S[i]) - tol) return 1;
    return 0;
}

/* lo = max(s - d), hi = min(s + d); argmax/argmin = smallest index within tie of the extreme */
void og_bounds_one(const double *q, const double *P, const double *S, long N, double tie,
                   double *lo, double *hi, long *a, long *b)
{
    double l = -INFINITY, h = INFINITY;
    for (long i = 0; i < N; ++i) {
        double d = dist3(q, P + 3 * i);
        if (S[i] - d > l) l = S[i] - d;
        if (S[i] + d < h) h = S[i] + d;
    }
    long ia = -1, ib = -1;
    for (long i = 0; i < N && (ia < 0 || ib < 0); ++i) {
        double d = dist3(q, P + 3 * i);
        if (ia < 0 && S[i] - d >= l - tie) ia = i;
        if (ib < 0 && S[i] + d <= h + tie) ib = i;
    }
    *lo = l; *hi = h; *a = ia; *b = ib;
}

/* caps of sphere (o, r); returns -1 if one ball holds the whole sphere */
static long gather_caps(const double *o, double r, const double *P, const double *S, long N, double tol,
                        cap_t *caps)
{
    long k = 0;
    for (long i = 0; i < N; ++i) {
        double R = fabs(S[i]) - tol;
        if (!(R > 0.0)) continue;
        double v[3] = {P[3 * i] - o[0], P[3 * i + 1] - o[1], P[3 * i + 2] - o[2]};
        double D = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
        if (D + r < R) return -1;
        if (D > 0.0 && fabs(D - r) < R) {
            caps[k].u[0] = v[0] / D; caps[k].u[1] = v[1] / D; caps[k].u[2] = v[2] / D;
            caps[k].c = (r * r + D * D - R * R) / (2.0 * r * D);
            ++k;
        }
    }
    return k;
}

static void basis(const double *u, double *e1, double *e2)
{
    double a[3] = {1.0, 0.0, 0.0};
    if (fabs(u[0]) >= 0.9) { a[0] = 0.0; a[1] = 1.0; }
    /* e1 = u x a, normalised; e2 = u x e1 */
    e1[0] = u[1] * a[2] - u[2] * a[1];
    e1[1] = u[2] * a[0] - u[0] * a[2];
    e1[2] = u[0] * a[1] - u[1] * a[0];
    double n = sqrt(dot3(e1, e1));
    e1[0] /= n; e1[1] /= n; e1[2] /= n;
    e2[0] = u[1] * e1[2] - u[2] * e1[1];
    e2[1] = u[2] * e1[0] - u[0] * e1[2];
    e2[2] = u[0] * e1[1] - u[1] * e1[0];
}

static int cmp_piece(const void *x, const void *y)
{
    double a = ((const piece_t *)x)->a, b = ((const piece_t *)y)->a;
    return (a > b) - (a < b);
}

/* uncovered closed angle intervals on the rim of cap e; returns count
 * (0 = rim fully covered).  gaps holds 2*count angles. */
static long rim_gaps(const cap_t *caps, long k, long e, piece_t *pieces, double *gaps)
{
    const cap_t *ce = caps + e;
    double rho = sqrt(fmax(0.0, 1.0 - ce->c * ce->c));
    double e1[3], e2[3];
    basis(ce->u, e1, e2);
    long np = 0;
    for (long f = 0; f < k; ++f) {
        if (f == e) continue;
        const cap_t *cf = caps + f;
        double A = rho * dot3(e1, cf->u);
        double B = rho * dot3(e2, cf->u);
        double K = cf->c - ce->c * dot3(ce->u, cf->u);
        double amp = hypot(A, B);
        if (K < -amp) return 0;
        if (!(amp > K)) continue;
        double phi = atan2(B, A);
        double t = K / amp;
        if (t > 1.0) t = 1.0;
        if (t < -1.0) t = -1.0;
        double beta = acos(t);
        double s = phi - beta, en = phi + beta;
        double shift = floor(s / TWO_PI) * TWO_PI;
        s -= shift; en -= shift;
        if (en > TWO_PI) {
            pieces[np].a = s; pieces[np].b = INFINITY; ++np;
            pieces[np].a = -INFINITY; pieces[np].b = en - TWO_PI; ++np;
        } else {
            pieces[np].a = s; pieces[np].b = en; ++np;
        }
    }
    if (np == 0) { gaps[0] = 0.0; gaps[1] = TWO_PI; return 1; }
    qsort(pieces, (size_t)np, sizeof(piece_t), cmp_piece);
    long ng = 0;
    double x = 0.0;
    for (long i = 0; i < np; ++i) {
        if (x >= TWO_PI) break;
        if (pieces[i].a < x) {
            if (pieces[i].b > x) x = pieces[i].b;
        } else {
            gaps[2 * ng] = x;
            gaps[2 * ng + 1] = pieces[i].a < TWO_PI ? pieces[i].a : TWO_PI;
            ++ng;
            x = pieces[i].b;
        }
    }
    if (x < TWO_PI) { gaps[2 * ng] = x; gaps[2 * ng + 1] = TWO_PI; ++ng; }
    return ng;
}

static void rim_point(const double *o, double r, const cap_t *c, double t, double *x)
{
    double rho = sqrt(fmax(0.0, 1.0 - c->c * c->c));
    double e1[3], e2[3];
    basis(c->u, e1, e2);
    double ct = cos(t), st = sin(t);
    for (int j = 0; j < 3; ++j) x[j] = o[j] + r * (c->c * c->u[j] + rho * (ct * e1[j] + st * e2[j]));
}

static int dir_uncovered(const cap_t *caps, long k, const double *v);

/* Move a rim point a tiny angle (1e-7) away from cap e so the witness keeps a
 * margin against rounding; keep the original if that would enter a cap. */
static void off_rim(const double *o, double r, double *x, const cap_t *caps, long k, long e)
{
    double v[3] = {(x[0] - o[0]) / r, (x[1] - o[1]) / r, (x[2] - o[2]) / r};
    double uv = dot3(caps[e].u, v);
    double t[3] = {caps[e].u[0] - uv * v[0], caps[e].u[1] - uv * v[1], caps[e].u[2] - uv * v[2]};
    double tn = sqrt(dot3(t, t));
    if (tn == 0.0) return;
    double w[3] = {v[0] - 1e-7 * t[0] / tn, v[1] - 1e-7 * t[1] / tn, v[2] - 1e-7 * t[2] / tn};
    double wn = sqrt(dot3(w, w));
    w[0] /= wn; w[1] /= wn; w[2] /= wn;
    if (dir_uncovered(caps, k, w))
        for (int j = 0; j < 3; ++j) x[j] = o[j] + r * w[j];
}

typedef struct { double key; long idx; } keyed_t;
static int cmp_keyed(const void *x, const void *y)
{
    const keyed_t *a = x, *b = y;
    if (a->key < b->key) return -1;
    if (a->key > b->key) return 1;
    return (a->idx > b->idx) - (a->idx < b->idx);
}

static int dir_uncovered(const cap_t *caps, long k, const double *v)
{
    for (long f = 0; f < k; ++f)
        if (dot3(v, caps[f].u) > caps[f].c) return 0;
    return 1;
}

/* Some uncovered point of sphere (o, r) into x; returns 1 if found, 0 if the
 * sphere is fully covered.  hint (may be NULL) only orders the rims. */
int og_uncovered_point(const double *o, double r, const double *P, const double *S, long N, double tol,
                       const double *hint, double *x)
{
    if (r <= 0.0) {
        if (og_point_covered(o, P, S, N, tol)) return 0;
        x[0] = o[0]; x[1] = o[1]; x[2] = o[2];
        return 1;
    }
    cap_t *caps = malloc(sizeof(cap_t) * (size_t)(N > 0 ? N : 1));
    long k = gather_caps(o, r, P, S, N, tol, caps);
    if (k < 0) { free(caps); return 0; }
    double vh[3] = {1.0, 0.0, 0.0};
    if (hint) {
        double g[3] = {hint[0] - o[0], hint[1] - o[1], hint[2] - o[2]};
        double n = sqrt(dot3(g, g));
        if (n > 0.0) { vh[0] = g[0] / n; vh[1] = g[1] / n; vh[2] = g[2] / n; }
    }
    if (k == 0 || dir_uncovered(caps, k, vh)) {
        for (int j = 0; j < 3; ++j) x[j] = o[j] + r * vh[j];
        free(caps);
        return 1;
    }
    keyed_t *ord = malloc(sizeof(keyed_t) * (size_t)k);
    for (long e = 0; e < k; ++e) {
        double cu = dot3(caps[e].u, vh);
        cu = cu > 1.0 ? 1.0 : (cu < -1.0 ? -1.0 : cu);
        double cc = caps[e].c > 1.0 ? 1.0 : (caps[e].c < -1.0 ? -1.0 : caps[e].c);
        ord[e].key = fabs(acos(cu) - acos(cc));
        ord[e].idx = e;
    }
    qsort(ord, (size_t)k, sizeof(keyed_t), cmp_keyed);
    piece_t *pieces = malloc(sizeof(piece_t) * (size_t)(2 * k + 2));
    double *gaps = malloc(sizeof(double) * (size_t)(4 * k + 4));
    int found = 0;
    for (long i = 0; i < k && !found; ++i) {
        long e = ord[i].idx;
        long ng = rim_gaps(caps, k, e, pieces, gaps);
        if (ng > 0) {
            long bi = 0;
            for (long g = 1; g < ng; ++g)
                if (gaps[2 * g + 1] - gaps[2 * g] > gaps[2 * bi + 1] - gaps[2 * bi]) bi = g;
            rim_point(o, r, caps + e, 0.5 * (gaps[2 * bi] + gaps[2 * bi + 1]), x);
            off_rim(o, r, x, caps, k, e);
            found = 1;
        }
    }
    free(gaps); free(pieces); free(ord); free(caps);
    return found;
}

/* Nearest point to q of the uncovered part of sphere (o, r), if nearer than
 * bound.  Returns 0 (none), 1 (radial foot point, T), 2 (rim nearest point,
 * D) or 3 (rim arc end point, U); writes the distance and the point. */
int og_nearest_uncovered(const double *o, double r, const double *P, const double *S, long N,
                         const double *q, double bound, double tol, double *dist_out, double *x)
{
    double g[3] = {q[0] - o[0], q[1] - o[1], q[2] - o[2]};
    double gn = sqrt(dot3(g, g));
    if (r <= 0.0) {
        if (og_point_covered(o, P, S, N, tol) || !(gn < bound)) return 0;
        *dist_out = gn; x[0] = o[0]; x[1] = o[1]; x[2] = o[2];
        return 1;
    }
    cap_t *caps = malloc(sizeof(cap_t) * (size_t)(N > 0 ? N : 1));
    long k = gather_caps(o, r, P, S, N, tol, caps);
    if (k < 0) { free(caps); return 0; }
    if (gn > 0.0) {
        double v0[3] = {g[0] / gn, g[1] / gn, g[2] / gn};
        double d0 = fabs(gn - r);
        if (!(d0 < bound)) { free(caps); return 0; }
        if (k == 0 || dir_uncovered(caps, k, v0)) {
            for (int j = 0; j < 3; ++j) x[j] = o[j] + r * v0[j];
            *dist_out = d0;
            free(caps);
            return 1;
        }
    } else {
        free(caps);
        if (!(r < bound)) return 0;
        if (!og_uncovered_point(o, r, P, S, N, tol, NULL, x)) return 0;
        *dist_out = r;
        return 1;
    }
    keyed_t *ord = malloc(sizeof(keyed_t) * (size_t)k);
    for (long e = 0; e < k; ++e) {
        double ug = dot3(caps[e].u, g);
        double perp = sqrt(fmax(gn * gn - ug * ug, 0.0));
        double rho = sqrt(fmax(1.0 - caps[e].c * caps[e].c, 0.0));
        double vg = caps[e].c * ug + rho * perp;
        ord[e].key = sqrt(fmax(r * r + gn * gn - 2.0 * r * vg, 0.0));
        ord[e].idx = e;
    }
    qsort(ord, (size_t)k, sizeof(keyed_t), cmp_keyed);
    piece_t *pieces = malloc(sizeof(piece_t) * (size_t)(2 * k + 2));
    double *gaps = malloc(sizeof(double) * (size_t)(4 * k + 4));
    double best = bound;
    int kind = 0;
    for (long i = 0; i < k; ++i) {
        if (ord[i].key >= best) break;
        long e = ord[i].idx;
        long ng = rim_gaps(caps, k, e, pieces, gaps);
        if (ng == 0) continue;
        double e1[3], e2[3];
        basis(caps[e].u, e1, e2);
        double ts = atan2(dot3(e2, g), dot3(e1, g));
        ts = ts - floor(ts / TWO_PI) * TWO_PI;
        for (long gi = 0; gi < ng; ++gi) {
            double t0 = gaps[2 * gi], t1 = gaps[2 * gi + 1], t;
            int inside = 0;
            if (t0 <= ts && ts <= t1) { t = ts; inside = 1; }
            else {
                double d0 = fabs(ts - t0), d1 = fabs(ts - t1);
                d0 = fmin(d0, TWO_PI - d0);
                d1 = fmin(d1, TWO_PI - d1);
                t = d0 <= d1 ? t0 : t1;
            }
            double y[3];
            rim_point(o, r, caps + e, t, y);
            double d = dist3(y, q);
            if (d < best) {
                best = d; kind = inside ? 2 : 3;
                x[0] = y[0]; x[1] = y[1]; x[2] = y[2];
            }
        }
    }
    free(gaps); free(pieces); free(ord); free(caps);
    if (kind) *dist_out = best;
    return kind;
}

typedef struct { double lb; long idx; } lbidx_t;
static int cmp_lb(const void *x, const void *y)
{
    const lbidx_t *a = x, *b = y;
    if (a->lb < b->lb) return -1;
    if (a->lb > b->lb) return 1;
    return (a->idx > b->idx) - (a->idx < b->idx);
}

/* Minimum valid radius of a query q of sign sigma: the distance from q to
 * the contour of the union of sigma-balls (proof of Prop. 2).  The contour is
 * that of the balls shrunk by the uniqueness tolerance `tie` only (not by
 * tol), so the contact point lies outside every tol-shrunk ball with margin
 * tol - tie and the new sphere keeps an uncovered neighbourhood there, while
 * exactly tangent spheres still leave non-degenerate gaps.  q counts as
 * inside a ball when d < |s| - tol.  Returns the
 * kind of the nearest contour point (0: q in no sigma-ball, radius 0;
 * 1 T, 2 D, 3 U; -1 nothing found).  W (nullable, NaN rows allowed) holds
 * known uncovered points; the nearest one on a sigma-sphere bounds the
 * search from above. */
/* Distance from q to the points of sphere (p, r) outside the open ball
 * (c, R) (INFINITY if none), taken a hair short.  A point of the sphere is
 * v = p + r u with |u| = 1; the ball holds the cap u.a > cos_t with a the unit
 * direction from p to c and cos_t = (r^2 + D^2 - R^2)/(2 r D).  If the
 * direction g from p to q lies outside that cap, the nearest point is the
 * radial one (distance |d - r|); otherwise it lies on the cap's rim, where
 * u.g is largest at cos_t (g.a) + sin_t sqrt(1 - (g.a)^2). */
static double dist_outside(const double *q, const double *p, double r, const double *c, double R)
{
    double d = dist3(q, p), D = dist3(c, p);
    double foot = fabs(d - r);
    if (!(R > 0.0) || !(r > 0.0) || !(D > 0.0) || !(d > 0.0)) return foot;
    if (D + r < R * (1.0 - 1e-12) - 1e-15) return INFINITY;
    if (!(D < r + R) || !(D + R > r)) return foot;
    double cos_t = (r * r + D * D - R * R) / (2.0 * r * D);
    if (!(cos_t > -1.0 && cos_t < 1.0)) return foot;
    double ga = ((q[0] - p[0]) * (c[0] - p[0]) + (q[1] - p[1]) * (c[1] - p[1]) + (q[2] - p[2]) * (c[2] - p[2])) / (d * D);
    if (!(ga > cos_t)) return foot;
    double ug = cos_t * ga + sqrt(fmax(0.0, 1.0 - cos_t * cos_t)) * sqrt(fmax(0.0, 1.0 - ga * ga));
    double rim = sqrt(fmax(0.0, r * r + d * d - 2.0 * r * d * ug));
    return fmax(foot, rim * (1.0 - 1e-12) - 1e-15);
}

int og_min_valid_radius(const double *q, int sigma, const double *P, const double *S, long N, double tol,
                        double tie, const double *W, double *r_out, double *x, long *sphere)
{
    long cnt = 0, deepest = -1;
    double depth = -INFINITY;
    lbidx_t *ord = malloc(sizeof(lbidx_t) * (size_t)(N > 0 ? N : 1));
    int inside = 0;
    double best = INFINITY;
    for (long i = 0; i < N; ++i) {
        int sg = S[i] > tie ? 1 : (S[i] < -tie ? -1 : 0);
        if (sg != sigma) continue;
        double R = fabs(S[i]);
        double d = dist3(q, P + 3 * i);
        if (d < R - tol) inside = 1;
        if (R - d > depth) { depth = R - d; deepest = i; }
        ord[cnt].lb = fabs(d - R);
        ord[cnt].idx = i;
        ++cnt;
        if (W && !isnan(W[3 * i])) {
            double dw = dist3(W + 3 * i, q);
            if (dw < best) best = dw;
        }
    }
    if (!inside) {
        free(ord);
        *r_out = 0.0; x[0] = q[0]; x[1] = q[1]; x[2] = q[2]; *sphere = -1;
        return 0;
    }
    double bound = isinf(best) ? INFINITY : best * (1.0 + 1e-12) + 1e-15;
    /* Only balls reaching within `bound` of q can cover a point nearer than
     * bound: |x - q| < bound and |x - p| < |s| give |q - p| < |s| + bound.
     * Restricting coverage tests to them leaves every answer below bound exact. */
    const double *LPc = P, *LSc = S;
    double *LP = NULL, *LS = NULL;
    long LN = N;
    long *lmap = NULL;
    if (!isinf(bound)) {
        LP = malloc(sizeof(double) * 3 * (size_t)(N > 0 ? N : 1));
        LS = malloc(sizeof(double) * (size_t)(N > 0 ? N : 1));
        lmap = malloc(sizeof(long) * (size_t)(N > 0 ? N : 1));
        LN = 0;
        for (long i = 0; i < N; ++i) {
            if (dist3(q, P + 3 * i) < fabs(S[i]) + bound) {
                LP[3 * LN] = P[3 * i]; LP[3 * LN + 1] = P[3 * i + 1]; LP[3 * LN + 2] = P[3 * i + 2];
                LS[LN] = S[i];
                lmap[LN] = i;
                ++LN;
            }
        }
        LPc = LP; LSc = LS;
    }
    int kind = 0;
    double y[3], d;
    int kk = og_nearest_uncovered(P + 3 * deepest, fabs(S[deepest]), LPc, LSc, LN, q, bound, tie, &d, y);
    if (kk) {
        bound = d; kind = kk; *sphere = deepest;
        x[0] = y[0]; x[1] = y[1]; x[2] = y[2];
        if (kk == 1) {
            free(ord);
            if (lmap) { free(LP); free(LS); free(lmap); }
            *r_out = d;
            return 1;
        }
    }
    qsort(ord, (size_t)cnt, sizeof(lbidx_t), cmp_lb);
    /* an uncovered point of sphere i lies outside every other ball, the
     * deepest one (contour balls shrunk by tie) included */
    const double Rd = fabs(S[deepest]) - tie;
    for (long k = 0; k < cnt; ++k) {
        if (ord[k].lb >= bound) break;
        long i = ord[k].idx;
        if (i == deepest) continue;
        if (dist_outside(q, P + 3 * i, fabs(S[i]), P + 3 * deepest, Rd) >= bound) continue;
        kk = og_nearest_uncovered(P + 3 * i, fabs(S[i]), LPc, LSc, LN, q, bound, tie, &d, y);
        if (kk && d < bound) {
            bound = d; kind = kk; *sphere = i;
            x[0] = y[0]; x[1] = y[1]; x[2] = y[2];
        }
    }
    free(ord);
    if (lmap) { free(LP); free(LS); free(lmap); }
    if (!kind) {
        if (W) return og_min_valid_radius(q, sigma, P, S, N, tol, tie, NULL, r_out, x, sphere);
        return -1;
    }
    *r_out = bound;
    return kind;
}
