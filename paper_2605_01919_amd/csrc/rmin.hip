// Minimum valid radius of many points (Corollary 1: all are computed
// independently and are jointly valid) and the pseudo-SDF repair built on it
// (Sec. 6): fully covered samples are found with the exact witness search,
// removed together, and re-assigned their minimum valid radius.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cstring>
#include <vector>

#include "block_dev.h"
#include "common.h"

namespace sdfi {



namespace {

constexpr int RW = 4;  // wavefronts per point
constexpr int RBS = RW * 64;
constexpr int RGRID = 512;   // persistent work-groups

struct RShared {
    blk::Shared<RW> S;
    geom::Cap kp[RW][geom::KMAX];
    int64_t kid[RW][geom::KMAX];
};

// Points pts[k] (k x 3); force[k] = +1/-1 imposes the sign (removed samples
// keep theirs), 0 lets containment choose it.  Writes value, kind, contact
// point.  A point with an imposed sign that lies in no ball of that sign is
// UNRESOLVED and keeps `keep[k]` (if non-null).
__global__ __launch_bounds__(RBS) void rmin_kernel(const double *pts, const int8_t *force, const double *keep,
                                                   int64_t K, const double *p4, const double *W, int64_t nb,
                                                   double tol, double tie, double *val, uint8_t *kind, double *wout,
                                                   int64_t *lists, int32_t *flists, int fcap) {
    __shared__ RShared SH;
    int64_t *list = lists + (int64_t)blockIdx.x * 3 * (nb + 1);  // candidates, local set, near rows
    int32_t *flist = flists + (int64_t)blockIdx.x * RW * fcap;
    for (int64_t k = blockIdx.x; k < K; k += gridDim.x) {
        const double q[3] = {pts[3 * k], pts[3 * k + 1], pts[3 * k + 2]};
        int sigma = force ? force[k] : 0;
        if (sigma == 0) {
            // sign forced by containment: the deepest containing ball (Sec. 4.3)
            double depth = -INFINITY;
            for (int64_t c = threadIdx.x; c < nb; c += RBS) {
                const double *p = p4 + 4 * c;
                double d = geom::dist3(q, p);
                if (d < fabs(p[3]) - tol) depth = fmax(depth, fabs(p[3]) - d);
            }
            depth = blk::bmax(depth, SH.S);
            int64_t who = INT64_MAX;
            if (depth > -INFINITY)
                for (int64_t c = threadIdx.x; c < nb; c += RBS) {
                    const double *p = p4 + 4 * c;
                    double d = geom::dist3(q, p);
                    if (d < fabs(p[3]) - tol && fabs(p[3]) - d == depth) who = who < c ? who : c;
                }
            who = blk::bmin_i64(who, SH.S);
            sigma = who == INT64_MAX ? 0 : blk::sign_class(p4[4 * who + 3], tie);
        }
        double r = 0.0, x[3] = {q[0], q[1], q[2]};
        int64_t sph = -1;
        int kk = sigma == 0 ? 0
                            : blk::rmin_block<RW>(q, sigma, p4, W, nb, tol, tie, list, SH.kp, SH.kid, flist, fcap, SH.S, &r, x,
                                                  &sph, nullptr, 0, nullptr, list + 2 * (nb + 1));
        if (threadIdx.x == 0) {
            bool forced = force && force[k] != 0;
            if (kk > 0) {
                val[k] = sigma * r;
                kind[k] = kk == 1 ? SDFI_KIND_RMIN_T : (kk == 2 ? SDFI_KIND_RMIN_D : SDFI_KIND_RMIN_U);
            } else if (kk == 0 && !forced) {
                val[k] = 0.0;
                kind[k] = SDFI_KIND_ZERO;
            } else {
                val[k] = keep ? keep[k] : NAN;
                kind[k] = SDFI_KIND_UNRESOLVED;
            }
            wout[3 * k] = x[0];
            wout[3 * k + 1] = x[1];
            wout[3 * k + 2] = x[2];
        }
        __syncthreads();
    }
}

__global__ void gather_kernel(const double *p4, const double *W, const int64_t *idx, int64_t k, double *o4,
                              double *ow) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < k) {
        int64_t s = idx[i];
        for (int j = 0; j < 4; ++j) o4[4 * i + j] = p4[4 * s + j];
        for (int j = 0; j < 3; ++j) ow[3 * i + j] = W[3 * s + j];
    }
}

__global__ void removed_points_kernel(const double *p4, const int64_t *idx, int64_t k, double tie, double *pts,
                                      int8_t *force, double *keep) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < k) {
        int64_t s = idx[i];
        for (int j = 0; j < 3; ++j) pts[3 * i + j] = p4[4 * s + j];
        force[i] = (int8_t)blk::sign_class(p4[4 * s + 3], tie);
        keep[i] = p4[4 * s + 3];
    }
}

__global__ void init_repair_kernel(const double *p4, int64_t n, const uint8_t *wstat, double *repaired,
                                   uint8_t *removed, uint8_t *kind) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) {
        repaired[i] = p4[4 * i + 3];
        removed[i] = wstat[i] ? 0 : 1;
        kind[i] = SDFI_KIND_KEPT;
    }
}

__global__ void scatter_repair_kernel(const int64_t *ridx, int64_t nr, const double *rval, const uint8_t *rkind,
                                      double *repaired, uint8_t *kind) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < nr) {
        int64_t s = ridx[i];
        repaired[s] = rval[i];
        kind[s] = rkind[i];
    }
}

int flist_cap(int64_t nb) { return (int)std::min<int64_t>(geom::FALLBACK_GLOBAL, nb + 1); }

double now_ms() {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

sdfi_status launch_rmin(const double *pts, const int8_t *force, const double *keep, int64_t K, const double *p4,
                        const double *W, int64_t nb, const sdfi_options &o, double *val, uint8_t *kind, double *wout,
                        int64_t *lists, int32_t *flists, hipStream_t st) {
    if (K == 0) return SDFI_OK;
    int grid = (int)std::min<int64_t>(K, RGRID);
    // each wave's cap list for exhaustive searches: every ball of a small set, FALLBACK_GLOBAL otherwise
    const int fcap = flist_cap(nb);
    KernelTimer tm("rmin", st);
    rmin_kernel<<<grid, RBS, 0, st>>>(pts, force, keep, K, p4, W, nb, o.tol, o.tie_tol, val, kind, wout, lists,
                                      flists, fcap);
    tm.stop();
    SDFI_HIP(hipGetLastError());
    return SDFI_OK;
}

}  // namespace

size_t rmin_ws(int64_t n, int64_t m, const sdfi_options &) {
    Carver c(nullptr, 0, true);
    c.take<char>(check_ws(0));                    // input checks
    c.take<double>(3 * (n + 1));                  // witnesses
    c.take<uint8_t>(n + 1);                       // status
    c.take<int64_t>((size_t)RGRID * 3 * (n + 1)); // per work-group lists
    c.take<int32_t>((size_t)RGRID * RW * flist_cap(n)); // per wave cap lists
    return c.used + 1024;
}

size_t repair_ws(int64_t n, int64_t m, const sdfi_options &) {
    Carver c(nullptr, 0, true);
    c.take<char>(check_ws(0));                    // input checks
    c.take<double>(3 * (n + 1));                  // witnesses of all samples
    c.take<uint8_t>(n + 1);                       // status
    c.take<int64_t>(n + 1);                       // kept indices
    c.take<int64_t>(n + 1);                       // removed indices
    c.take<double>(4 * (n + 1));                  // base samples
    c.take<double>(3 * (n + 1));                  // base witnesses
    c.take<double>(3 * (n + 1));                  // removed points
    c.take<int8_t>(n + 1);                        // their signs
    c.take<double>(n + 1);                        // their original values
    c.take<double>(n + 1);                        // their radii
    c.take<uint8_t>(n + 1);                       // their kinds
    c.take<double>(3 * (n + m + 1));              // contact points
    c.take<int64_t>((size_t)RGRID * 3 * (n + 1)); // per work-group lists
    c.take<int32_t>((size_t)RGRID * RW * flist_cap(n)); // per wave cap lists
    return c.used + 4096;
}

}  // namespace sdfi

using namespace sdfi;

extern "C" sdfi_status sdfi_min_valid_radius(const double *samples, int64_t n, const double *queries, int64_t m,
                                             double *values, uint8_t *kind, double *witness, void *ws,
                                             size_t ws_bytes, const sdfi_options *opt, sdfi_stream stream) {
    sdfi_options o;
    sdfi_status s = read_options(opt, &o);
    if (s != SDFI_OK) return s;
    SDFI_CHECK_ARG(n >= 1 && n < (int64_t(1) << 31) && m >= 0 && m < (int64_t(1) << 31), "sizes out of range");
    if (m == 0) return SDFI_OK;
    SDFI_CHECK_ARG(samples && queries && values && kind && witness, "null array argument");
    if (ws_bytes < rmin_ws(n, m, o) || !ws) {
        set_error("workspace of %zu bytes is below the %zu required", ws_bytes, rmin_ws(n, m, o));
        return SDFI_ERR_WORKSPACE;
    }
    hipStream_t st = to_hip(stream);
    Carver c(ws, ws_bytes);
    char *chk = c.take<char>(check_ws(0));
    double *W = c.take<double>(3 * (n + 1));
    uint8_t *wst = c.take<uint8_t>(n + 1);
    int64_t *lists = c.take<int64_t>((size_t)RGRID * 3 * (n + 1));
    int32_t *flists = c.take<int32_t>((size_t)RGRID * RW * flist_cap(n));
    s = validate_inputs(samples, n, queries, m, nullptr, 0, 0, true, chk, check_ws(0), o, st);
    if (s != SDFI_OK) return s;
    s = run_witnesses(samples, n, W, wst, o, st);
    if (s != SDFI_OK) return s;
    return launch_rmin(queries, nullptr, nullptr, m, samples, W, n, o, values, kind, witness, lists, flists, st);
}

extern "C" sdfi_status sdfi_repair(const double *samples, int64_t n, const double *queries, int64_t m,
                                   double *repaired, uint8_t *removed, double *query_values, uint8_t *kind,
                                   sdfi_report *report, void *ws, size_t ws_bytes, const sdfi_options *opt,
                                   sdfi_stream stream) {
    sdfi_options o;
    sdfi_status s = read_options(opt, &o);
    if (s != SDFI_OK) return s;
    SDFI_CHECK_ARG(n >= 1 && n < (int64_t(1) << 31) && m >= 0 && m < (int64_t(1) << 31), "sizes out of range");
    SDFI_CHECK_ARG(samples && repaired && removed && kind && (m == 0 || (queries && query_values)),
                   "null array argument");
    if (ws_bytes < repair_ws(n, m, o) || !ws) {
        set_error("workspace of %zu bytes is below the %zu required", ws_bytes, repair_ws(n, m, o));
        return SDFI_ERR_WORKSPACE;
    }
    hipStream_t st = to_hip(stream);
    Carver c(ws, ws_bytes);
    char *chk = c.take<char>(check_ws(0));
    double *W = c.take<double>(3 * (n + 1));
    uint8_t *wst = c.take<uint8_t>(n + 1);
    int64_t *kidx = c.take<int64_t>(n + 1);
    int64_t *ridx = c.take<int64_t>(n + 1);
    double *bp = c.take<double>(4 * (n + 1));
    double *bw = c.take<double>(3 * (n + 1));
    double *rpts = c.take<double>(3 * (n + 1));
    int8_t *rforce = c.take<int8_t>(n + 1);
    double *rkeep = c.take<double>(n + 1);
    double *rval = c.take<double>(n + 1);
    uint8_t *rkind = c.take<uint8_t>(n + 1);
    double *contact = c.take<double>(3 * (n + m + 1));
    int64_t *lists = c.take<int64_t>((size_t)RGRID * 3 * (n + 1));
    int32_t *flists = c.take<int32_t>((size_t)RGRID * RW * flist_cap(n));
    s = validate_inputs(samples, n, queries, m, nullptr, 0, 0, true, chk, check_ws(0), o, st);
    if (s != SDFI_OK) return s;
    double t0 = now_ms();
    // 1. fully covered samples (Prop. 1 (ii) fails): no witness against all inputs
    s = run_witnesses(samples, n, W, wst, o, st);
    if (s != SDFI_OK) return s;
    std::vector<uint8_t> h(n);
    SDFI_HIP(hipMemcpyAsync(h.data(), wst, n, hipMemcpyDeviceToHost, st));
    SDFI_HIP(hipStreamSynchronize(st));
    double t1 = now_ms();
    // 2. remove them all at once
    std::vector<int64_t> keep_i, rem_i;
    for (int64_t i = 0; i < n; ++i) (h[i] ? keep_i : rem_i).push_back(i);
    const int64_t nk = (int64_t)keep_i.size(), nr = (int64_t)rem_i.size();
    if (nk == 0) {
        set_error("every sample sphere is fully covered");
        return SDFI_ERR_INVALID_INPUT;
    }
    SDFI_HIP(hipMemcpyAsync(kidx, keep_i.data(), sizeof(int64_t) * nk, hipMemcpyHostToDevice, st));
    if (nr) SDFI_HIP(hipMemcpyAsync(ridx, rem_i.data(), sizeof(int64_t) * nr, hipMemcpyHostToDevice, st));
    gather_kernel<<<(unsigned)((nk + 255) / 256), 256, 0, st>>>(samples, W, kidx, nk, bp, bw);
    if (nr)
        removed_points_kernel<<<(unsigned)((nr + 255) / 256), 256, 0, st>>>(samples, ridx, nr, o.tie_tol, rpts,
                                                                            rforce, rkeep);
    SDFI_HIP(hipGetLastError());
    double t2 = now_ms();
    // 3. minimum valid radii of the removed points (their sign) and of the queries
    s = launch_rmin(rpts, rforce, rkeep, nr, bp, bw, nk, o, rval, rkind, contact, lists, flists, st);
    if (s != SDFI_OK) return s;
    s = launch_rmin(queries, nullptr, nullptr, m, bp, bw, nk, o, query_values, kind + n, contact + 3 * nr, lists,
                    flists, st);
    if (s != SDFI_OK) return s;
    init_repair_kernel<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(samples, n, wst, repaired, removed, kind);
    if (nr)
        scatter_repair_kernel<<<(unsigned)((nr + 255) / 256), 256, 0, st>>>(ridx, nr, rval, rkind, repaired, kind);
    SDFI_HIP(hipGetLastError());
    SDFI_HIP(hipStreamSynchronize(st));
    if (report) {
        std::memset(report, 0, sizeof(*report));
        report->n_removed = nr;
        report->ms_phase[0] = t1 - t0;
        report->ms_phase[1] = t2 - t1;
        report->ms_phase[2] = now_ms() - t2;
    }
    return SDFI_OK;
}
