/* sdfi: consistent signed-distance interpolation on AMD Instinct MI355X (gfx950).
 *
 * C ABI of the hot path of "Greed for the Spheres: A Signed Distance
 * Interpolation Method" (Chen, Mupparaju, Batty, Sellan, Stein).
 *
 * Terms.  A sample (p, s) is the sphere centred at p with radius |s| and the
 * sign of s (Sec. 3.1).  A set of samples is valid (Prop. 1) when no two
 * spheres of different sign intersect (touching is allowed) and every sphere
 * has a point that lies in no other open ball (an uncovered point).  A point
 * x counts as covered by sample (p, s) when |x - p| < |s| - tol; values with
 * |s| <= tie_tol have no sign.  Appendix B fixes tol = 1e-6 and the
 * uniqueness tolerance tie_tol = 1e-9 and restricts everything to [-1,1]^3.
 *
 * Conventions shared by every entry point:
 *  - Arrays are device pointers unless a parameter says "host".  Samples are
 *    n x 4 float64 rows (x, y, z, s); query points are m x 3 float64 rows.
 *  - The caller owns every buffer and the stream.  Scratch memory comes from
 *    the caller's workspace `ws` of `ws_bytes` bytes (device memory, 256-byte
 *    aligned); sdfi_workspace_size() gives the size.  Outputs may not alias
 *    inputs.
 *  - Work is ordered on `stream` (a hipStream_t; NULL is the null stream).
 *    Entry points that take a host `report` or that need host decisions
 *    (noted per function) synchronise the stream before returning.
 *  - Errors: a status is returned and sdfi_last_error() gives a message
 *    (thread-local).  Argument errors are found on the host before any launch
 *    and leave outputs untouched.  Per-query outcomes go into `kind` codes.
 *  - Calls on different streams may run concurrently from different threads.
 */
#ifndef SDFI_H
#define SDFI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ihipStream_t *sdfi_stream;

typedef enum {
    SDFI_OK = 0,
    SDFI_ERR_INVALID_ARGUMENT = 1, /* null pointer, negative size, bad option */
    SDFI_ERR_DEVICE = 2,           /* a HIP call failed */
    SDFI_ERR_WORKSPACE = 3,        /* ws_bytes below sdfi_workspace_size() */
    SDFI_ERR_INVALID_INPUT = 4,    /* input samples violate Prop. 1 (when checked) */
    SDFI_ERR_DOMAIN = 5,           /* a point outside the domain box, or off the stated grid */
    SDFI_ERR_UNSUPPORTED = 6,      /* size beyond a documented limit */
    SDFI_ERR_NUMERIC = 7           /* an internal search hit its iteration cap */
} sdfi_status;

/* precision of the dense pairwise sweeps */
enum {
    SDFI_PREC_FP64 = 0,              /* everything in float64 */
    SDFI_PREC_FP32_FP64_RECHECK = 1  /* float32 sweep, float64 decides near-ties */
};

/* per-query outcome codes */
enum {
    SDFI_KIND_KEPT = 0,        /* repair: input sample kept unchanged */
    SDFI_KIND_HI = 1,          /* value = hi, tangent to the argmin constraint */
    SDFI_KIND_LO = 2,          /* value = lo, tangent to the argmax constraint */
    SDFI_KIND_ZERO = 3,        /* value 0: the point lies in no ball */
    SDFI_KIND_RMIN_T = 4,      /* minimum valid radius at a radial foot point */
    SDFI_KIND_RMIN_D = 5,      /* ... at the nearest point of an intersection circle */
    SDFI_KIND_RMIN_U = 6,      /* ... at a triple intersection point */
    SDFI_KIND_COINCIDENT = 7,  /* the query coincides with an existing sample */
    SDFI_KIND_INFEASIBLE = 254,/* lo > hi + tol: the constraints contradict */
    SDFI_KIND_UNRESOLVED = 255 /* no valid value found */
};

/* bound flags (sdfi_bounds) */
enum {
    SDFI_FLAG_INFEASIBLE = 1,    /* lo > hi + tol */
    SDFI_FLAG_INSIDE_POS = 2,    /* lo > tol: strictly inside a positive ball (sign forced +) */
    SDFI_FLAG_INSIDE_NEG = 4,    /* hi < -tol: strictly inside a negative ball (sign forced -) */
    SDFI_FLAG_TIE_LO = 8,        /* two or more constraints within tie_tol of lo */
    SDFI_FLAG_TIE_HI = 16,       /* two or more constraints within tie_tol of hi */
    SDFI_FLAG_HI_OPPOSITE = 32,  /* hi bound by an opposite-sign (non-intersection) constraint */
    SDFI_FLAG_LO_OPPOSITE = 64   /* lo bound by an opposite-sign constraint */
};

/* option flags */
enum {
    SDFI_OPT_CERTIFY = 1,      /* greedy/repair: run the Prop. 1 certificate on the result */
    SDFI_OPT_INPUT_CHECK = 2,  /* greedy: fail with SDFI_ERR_INVALID_INPUT if the samples violate Prop. 1 */
    SDFI_OPT_EXHAUSTIVE = 4    /* greedy: every exact sphere search that is not settled by its first
                                  cover scan walks every rim against every cap (the search's
                                  last resort) instead of growing a working cap subset; the
                                  answers are the same, only slower.  For testing that path. */
};

typedef struct {
    uint32_t struct_size;  /* sizeof(sdfi_options) */
    int32_t precision;     /* SDFI_PREC_* */
    double tol;            /* containment tolerance, default 1e-6 */
    double tie_tol;        /* uniqueness tolerance, default 1e-9 */
    double domain_lo[3];   /* default -1 */
    double domain_hi[3];   /* default +1 */
    int32_t grid;          /* input grid resolution N (samples at the cell centres of an
                              N^3 grid on [0,1]^3, x fastest), 0 = scattered samples */
    int32_t block_size;    /* threads per work-group of the greedy kernels: 256 or 512
                              (4 or 8 wavefronts per instance), 0 = 512, or 256 when a
                              batched launch has more instances than resident
                              512-thread work-groups */
    uint32_t flags;        /* SDFI_OPT_* */
    int32_t groups;        /* work-groups that share one greedy instance (a team: its
                              minimum-radius and re-validation searches are spread over
                              them; a cooperative launch), at most this many per
                              instance; 0 = 16; 1 = one group per instance.  A single
                              instance gets them all (capped at the groups the device
                              keeps resident); a batch shares the resident groups out
                              in proportion to each instance's pair count when there
                              are at least two per instance, else runs one group per
                              instance.  Teams need every group resident at once: other
                              kernels running on the device meanwhile can delay them
                              (a team that waits past its bound fails with
                              SDFI_ERR_DEVICE). */
} sdfi_options;

typedef struct {
    int64_t pairs_evaluated;       /* query x constraint pairs reduced by the bound sweeps */
    int64_t n_hi, n_lo, n_zero, n_rmin, n_coincident, n_infeasible, n_unresolved;
    int64_t n_fp64_rechecks;       /* queries resolved by a full float64 rescan */
    int64_t n_exact_searches;      /* exact uncovered-point searches run */
    int64_t n_violations_pairwise; /* certificate: pairs breaking the cone */
    int64_t n_violations_witness;  /* certificate: witnesses off their sphere or covered */
    int64_t n_removed;             /* repair: fully covered samples removed */
    int64_t n_search_capped;       /* exact searches that hit their work cap (candidate rejected or
                                      query UNRESOLVED; never an unproven acceptance) */
    double ms_phase[8];            /* wall time per phase, see each entry point */
} sdfi_report;

typedef enum {
    SDFI_OP_BOUNDS = 0,
    SDFI_OP_CERTIFY = 1,
    SDFI_OP_ORDER = 2,
    SDFI_OP_WITNESS = 3,
    SDFI_OP_GREEDY = 4,
    SDFI_OP_RMIN = 5,
    SDFI_OP_REPAIR = 6,
    SDFI_OP_BACKWARD = 7,
    SDFI_OP_GREEDY_INSTANCE = 8  /* bytes each instance of a batched launch adds (n, m ignored) */
} sdfi_op;

/* Fill `opt` with the defaults above. */
void sdfi_default_options(sdfi_options *opt);

/* Message of the last non-OK status returned on this thread. */
const char *sdfi_last_error(void);

/* Library version string. */
const char *sdfi_version(void);

/* Kernel timing for measurements.  While enabled, entry points record HIP
 * events on the caller's stream around their main kernels, under these names:
 * "sweep" and "resolve" (sdfi_bounds), "certify", "greedy", "witness",
 * "rmin".  Enabling does not change results. */
void sdfi_timing_enable(int on);

/* Total milliseconds and number of launches recorded under `name` since the
 * last reset (waits for the recorded events).  Unknown names give 0. */
sdfi_status sdfi_timing_query(const char *name, double *ms, int64_t *launches);

/* Work counters recorded while timing is enabled, summed since the last
 * reset (waits for the recorded work).  "sweep_pairs_skipped": query x sample
 * pairs that the float32 bound sweep of sdfi_bounds ruled out a whole tile at
 * a time, from the tile's box and value range, without evaluating them (their
 * values can neither be a bound nor lie within its tie band, so the results
 * equal those of the full sweep).  "bounds_list_overflows": query sides whose
 * candidate tile list overflowed, resolved by a scan of every tile that can
 * reach the band.  Unknown
 * names give 0. */
sdfi_status sdfi_counter_query(const char *name, int64_t *value);

/* Forget all recorded timings and counters. */
void sdfi_timing_reset(void);

/* Workspace bytes that entry point `op` needs for n samples and m queries
 * (for SDFI_OP_CERTIFY n is the set size and m is ignored).  A batched greedy
 * launch of B instances needs SDFI_OP_GREEDY with n = total samples + B and
 * m = total queries, plus B times SDFI_OP_GREEDY_INSTANCE. */
sdfi_status sdfi_workspace_size(sdfi_op op, int64_t n, int64_t m, const sdfi_options *opt, size_t *bytes);

/* Pairwise consistency bounds of every query (Sec. 4.3, "Further performance
 * improvements": a value must not intersect an opposite-sign sphere and
 * must not contain, or be contained by, a same-sign sphere; in signed form
 * both are the cone |s - s_i| <= |q - p_i|).
 *   lo[j] = max_i (s_i - |q_j - p_i|),  hi[j] = min_i (s_i + |q_j - p_i|)
 *   argmax[j] / argmin[j] = smallest i within tie_tol of lo / hi
 *   flags[j] = SDFI_FLAG_* bits.
 * samples n x 4, queries m x 3; outputs have m entries (argmax/argmin int32).
 * n >= 1; m >= 0 (m = 0 is a no-op).  n < 2^31.  Asynchronous: the inputs
 * are not checked on the host, so a sample with a NaN coordinate or value
 * takes part in no extreme, and a query with a NaN coordinate gets
 * lo = -inf, hi = +inf and argmax = argmin = -1. */
sdfi_status sdfi_bounds(const double *samples, int64_t n, const double *queries, int64_t m,
                        double *lo, double *hi, int32_t *argmax, int32_t *argmin, uint32_t *flags,
                        void *ws, size_t ws_bytes, const sdfi_options *opt, sdfi_stream stream);

/* sdfi_bounds for callers that cannot allocate (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the same
 * kernels and results, with the workspace taken from a scratch array of
 * 64 MiB that the library holds in device memory (one per GPU, kept until the
 * process ends) instead of a caller workspace.  Nothing is allocated: no
 * hipMalloc, no events, no pinned memory (kernel timers and work counters
 * record nothing during this call).  The caller still provides inputs and
 * outputs as for sdfi_bounds.
 * Limit: sizes whose sdfi_workspace_size(SDFI_OP_BOUNDS, n, m, opt) exceeds
 * 64 MiB are rejected with SDFI_ERR_UNSUPPORTED before any device work (e.g.
 * n = 110592, m = 262144 fits in either precision).
 * Every call on one GPU uses that GPU's one array: calls that overlap on the
 * same GPU (different streams or threads without ordering) race and give
 * wrong results; calls ordered on one stream are safe.  The first call on a
 * device looks the array's address up (hipGetSymbolAddress) with that device
 * current.  Asynchronous. */
sdfi_status sdfi_bounds_noalloc(const double *samples, int64_t n, const double *queries, int64_t m, double *lo,
                                double *hi, int32_t *argmax, int32_t *argmin, uint32_t *flags,
                                const sdfi_options *opt, sdfi_stream stream);

/* Certificate of Prop. 1 for a final set of N samples (pts_values N x 4)
 * with one claimed uncovered point per sphere (witness N x 3):
 *   (i)  |s_x - s_y| <= |p_x - p_y| + tol for every pair;
 *   (ii) every witness lies on its sphere (within tol) and in no other
 *        open ball (|w - p_y| >= |s_y| - tol, with 1e-9 rounding slack).
 * Rows whose value is NaN (queries left without a value) are not part of
 * the set.  The float32 screen's band is derived on the device from the
 * largest coordinate and value magnitudes, so the counts equal a float64
 * evaluation at any scale.  Counts go to report->n_violations_pairwise / _witness and
 * report->pairs_evaluated.  `report` is host memory and required;
 * synchronises the stream. */
sdfi_status sdfi_certify(const double *pts_values, const double *witness, int64_t N, sdfi_report *report,
                         void *ws, size_t ws_bytes, const sdfi_options *opt, sdfi_stream stream);

/* Refinement order (Sec. 4.2): covered-area ratio of every grid cell from
 * its 8^3 regular sub-points, best-first flood fill from the least covered
 * cell (ties: smaller linear index), each popped cell emitting its 8 child
 * cells in ascending child ratio (ties: child index bx + 2by + 4bz).
 * Needs opt->grid = N > 0 (samples on the N^3 cell centres).
 * If `queries` is NULL the m = (2N)^3 queries are the child cell centres and
 * order_out[k] is the linear index in the (2N)^3 grid of the k-th query.
 * Otherwise the m scattered queries are bucketed by the input cell holding
 * them (cells in flood-fill order, queries of one cell by index).
 * order_out: m int64 (device).  Synchronises the stream (the flood fill
 * runs on the host).  SDFI_ERR_DOMAIN if sample i does not lie in cell i of
 * that grid (x fastest); SDFI_ERR_INVALID_ARGUMENT for NaN or infinite
 * inputs. */
sdfi_status sdfi_refinement_order(const double *samples, int64_t n, const double *queries, int64_t m,
                                  int64_t *order_out, void *ws, size_t ws_bytes, const sdfi_options *opt,
                                  sdfi_stream stream);

/* One uncovered point per sample sphere (Prop. 1 (ii)); status_out[i] = 1 if
 * found (witness_out[i] set), 0 if the sphere is fully covered by the other
 * balls.  witness_out n x 3, status_out n uint8.  Asynchronous. */
sdfi_status sdfi_sample_witnesses(const double *samples, int64_t n, double *witness_out, uint8_t *status_out,
                                  void *ws, size_t ws_bytes, const sdfi_options *opt, sdfi_stream stream);

/* Greedy sequential interpolation (Sec. 3.3 interpolate_sdf_to applied in
 * the refinement order of Sec. 4): each query gets, in order, the best-
 * scoring value among hi and lo that keeps the augmented set valid (Prop. 1
 * checked exactly: the new sphere keeps an uncovered point and so does every
 * existing sphere), else the paper's fallback, the minimum valid radius
 * (0 outside every ball).
 *   order_in: m int64 (device) or NULL for the refinement order of
 *             sdfi_refinement_order (needs opt->grid).
 *   values: m float64; order_out: m int64 (acceptance order);
 *   active: m int64 (tangent constraint: id < n is a sample, n + j is query j;
 *           -1 for ZERO; for RMIN_* the sphere carrying the contact point);
 *   kind: m uint8 (SDFI_KIND_*); witness: m x 3 (an uncovered point of each
 *   query sphere, as last updated); sample_witness: n x 3 or NULL.
 * m < 2^31 and n + m < 2^31.  Synchronises the stream.
 * Errors (found before the greedy starts): SDFI_ERR_INVALID_ARGUMENT for NaN
 * or infinite inputs or an order_in that is not a permutation of [0, m);
 * SDFI_ERR_DOMAIN for a sample or query point outside the domain box,
 * or (order_in NULL) sample i or query j outside cell i (j) of the N^3
 * ((2N)^3) grid; with SDFI_OPT_INPUT_CHECK, SDFI_ERR_INVALID_INPUT
 * when the samples violate Prop. 1 (a sphere without an uncovered point, or
 * a pair breaking the cone: opposite-sign spheres that intersect, or a
 * sphere inside another's ball).  Without INPUT_CHECK such inputs are
 * interpolated as given: a query whose bounds contradict (lo > hi + tol)
 * gets kind SDFI_KIND_INFEASIBLE and value NaN.
 * report (host, may be NULL): counts; ms_phase[0] order, [1] witnesses,
 * [2] greedy, [3] certificate; [4..7] device time of the greedy steps spent
 * in the bound scans, the candidate checks, the minimum valid radius and the
 * bookkeeping (summed over instances, device wall clock). */
sdfi_status sdfi_greedy_interpolate(const double *samples, int64_t n, const double *queries, int64_t m,
                                    const int64_t *order_in, double *values, int64_t *order_out,
                                    int64_t *active, uint8_t *kind, double *witness, double *sample_witness,
                                    sdfi_report *report, void *ws, size_t ws_bytes, const sdfi_options *opt,
                                    sdfi_stream stream);

/* Many independent greedy interpolations in one persistent launch.
 * Instance b owns samples rows [sample_offsets[b], sample_offsets[b+1]) and
 * query rows [query_offsets[b], query_offsets[b+1]) of the concatenated
 * arrays; grids[b] is its input grid resolution (> 0; queries are its
 * (2 grids[b])^3 child cell centres and order_in is not taken).  Outputs are
 * concatenated like the queries; `active` ids are local to the instance.
 * Results equal num_instances calls of sdfi_greedy_interpolate.  Each
 * instance runs on one work-group or on a team of them (opt->groups), the
 * largest instances first.  ws_bytes: at least
 * sdfi_workspace_size(SDFI_OP_GREEDY, total samples + num_instances, total
 * queries) + num_instances * sdfi_workspace_size(SDFI_OP_GREEDY_INSTANCE).
 * Errors as for sdfi_greedy_interpolate, naming the instance; the report
 * sums over instances.
 * sample_offsets, query_offsets, grids: host arrays.  Synchronises. */
sdfi_status sdfi_greedy_interpolate_batched(int32_t num_instances, const int64_t *sample_offsets,
                                            const int64_t *query_offsets, const int32_t *grids,
                                            const double *samples, const double *queries, double *values,
                                            int64_t *order_out, int64_t *active, uint8_t *kind, double *witness,
                                            sdfi_report *report, void *ws, size_t ws_bytes,
                                            const sdfi_options *opt, sdfi_stream stream);

/* Minimum valid radius (proof of Prop. 2; Corollary 1; Sec. 6): for each
 * point, sign * distance to the contour of the union of same-sign balls,
 * with the sign forced by containment (0 and SDFI_KIND_ZERO outside every
 * ball).  By Corollary 1 all outputs are jointly valid with the samples.
 * values m float64, kind m uint8, witness m x 3 (the contact point).
 * Synchronises the stream (input check): SDFI_ERR_INVALID_ARGUMENT for NaN
 * or infinite inputs, SDFI_ERR_DOMAIN for a sample or query point outside
 * the domain box. */
sdfi_status sdfi_min_valid_radius(const double *samples, int64_t n, const double *queries, int64_t m,
                                  double *values, uint8_t *kind, double *witness, void *ws, size_t ws_bytes,
                                  const sdfi_options *opt, sdfi_stream stream);

/* Pseudo-SDF repair (Sec. 6): find every fully covered sample sphere,
 * remove all of them, give each removed point the minimum valid radius
 * against the rest with its original sign, and give each extension query
 * the minimum valid radius (sign forced by containment).
 *   repaired: n (kept samples unchanged); removed: n uint8;
 *   query_values: m; kind: n + m uint8 (KEPT, RMIN_*, ZERO, UNRESOLVED).
 * Synchronises the stream.  report (may be NULL): n_removed, ms_phase[0]
 * detection, [1] removal, [2] radii.  SDFI_ERR_INVALID_ARGUMENT for NaN or
 * infinite inputs, SDFI_ERR_DOMAIN for a sample or query point outside the
 * domain box. */
sdfi_status sdfi_repair(const double *samples, int64_t n, const double *queries, int64_t m, double *repaired,
                        uint8_t *removed, double *query_values, uint8_t *kind, sdfi_report *report, void *ws,
                        size_t ws_bytes, const sdfi_options *opt, sdfi_stream stream);

/* Gradient of sum_j grad_values[j] * values[j] with respect to the sample
 * values and positions, through the active-parent forest of a greedy run
 * (HI: v = s_t + |q - p_t|; LO: v = s_t - |q - p_t|; COINCIDENT: v = s_t;
 * RMIN_T: v = sign * ||q - p_t| - |s_t||; ZERO, RMIN_D and RMIN_U add
 * nothing).  Inputs are the outputs of sdfi_greedy_interpolate.
 * grad_s: n, grad_p: n x 3 (overwritten).  Asynchronous. */
sdfi_status sdfi_greedy_backward(const double *grad_values, const double *samples, int64_t n,
                                 const double *queries, int64_t m, const double *values, const int64_t *active,
                                 const uint8_t *kind, double *grad_s, double *grad_p, void *ws, size_t ws_bytes,
                                 sdfi_stream stream);

#ifdef __cplusplus
}
#endif

#endif /* SDFI_H */
