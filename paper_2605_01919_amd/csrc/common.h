// Host-side helpers shared by the sdfi entry points: status/error handling,
// option validation and workspace carving.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <string>

#include "../../include/sdfi.h"

namespace sdfi {

void set_error(const char *fmt, ...);

#define SDFI_CHECK_ARG(cond, ...)                 \
    do {                                          \
        if (!(cond)) {                            \
            ::sdfi::set_error(__VA_ARGS__);       \
            return SDFI_ERR_INVALID_ARGUMENT;     \
        }                                         \
    } while (0)

#define SDFI_HIP(call)                                                          \
    do {                                                                        \
        hipError_t e_ = (call);                                                 \
        if (e_ != hipSuccess) {                                                 \
            ::sdfi::set_error("%s failed: %s (%s:%d)", #call, hipGetErrorString(e_), __FILE__, __LINE__); \
            return SDFI_ERR_DEVICE;                                             \
        }                                                                       \
    } while (0)

// While an entry point that must not allocate runs on this thread, timers and
// work counters record nothing (they create events and pinned host words).
extern thread_local bool g_no_alloc;
struct NoAllocScope {
    bool prev;
    NoAllocScope() : prev(g_no_alloc) { g_no_alloc = true; }
    ~NoAllocScope() { g_no_alloc = prev; }
};

// Records a pair of HIP events around a kernel when timing is enabled.
struct KernelTimer {
    hipEvent_t a = nullptr, b = nullptr;
    const char *name;
    hipStream_t st;
    KernelTimer(const char *name, hipStream_t st);
    void stop();
};

// While timing is enabled: add the device int64 at `dev` (read once the work
// queued on `st` so far has finished) to the counter `name`.
void note_count(const char *name, const int64_t *dev, hipStream_t st);

// Whether kernel timing is enabled (and this thread may record).
bool timing_enabled();

// While timing is enabled: add a host value to the counter `name`.
void add_count(const char *name, int64_t value);

// Validated copy of the caller's options (defaults when opt == NULL).
sdfi_status read_options(const sdfi_options *opt, sdfi_options *out);

// Bump allocator over the caller's workspace; every carve is 256-byte aligned.
struct Carver {
    char *base;
    size_t cap;
    size_t used = 0;
    bool dry;  // sizing pass: base may be null
    Carver(void *b, size_t c, bool d = false) : base(static_cast<char *>(b)), cap(c), dry(d) {}
    template <typename T>
    T *take(size_t count) {
        size_t off = (used + 255) & ~size_t(255);
        used = off + count * sizeof(T);
        if (dry) return nullptr;
        return reinterpret_cast<T *>(base + off);
    }
    bool ok() const { return dry || used <= cap; }
};

inline hipStream_t to_hip(sdfi_stream s) { return reinterpret_cast<hipStream_t>(s); }

// workspace sizes per operation (defined next to each operation)
size_t bounds_ws(int64_t n, int64_t m, const sdfi_options &o);
size_t certify_ws(int64_t N, const sdfi_options &o);
size_t order_ws(int64_t n, int64_t m, const sdfi_options &o);
size_t witness_ws(int64_t n, const sdfi_options &o);
size_t greedy_instance_ws(const sdfi_options &o);
size_t greedy_ws(int64_t n, int64_t m, const sdfi_options &o);
size_t rmin_ws(int64_t n, int64_t m, const sdfi_options &o);
size_t repair_ws(int64_t n, int64_t m, const sdfi_options &o);
size_t backward_ws(int64_t n, int64_t m);

// Device-side input checks, one read-back: non-finite inputs or an order_in
// that is not a permutation (SDFI_ERR_INVALID_ARGUMENT); with grid > 0
// (qgrid > 0) samples (queries) outside their own cell of that grid on
// [0,1]^3, and with `domain` sample or query points outside the options'
// domain box (SDFI_ERR_DOMAIN).  `order` may be null.  Synchronises.
size_t check_ws(int64_t m, int64_t njobs = 1);
sdfi_status validate_inputs(const double *samples, int64_t n, const double *queries, int64_t m,
                            const int64_t *order, int grid, int qgrid, bool domain, void *scratch,
                            size_t scratch_bytes, const sdfi_options &o, hipStream_t st);
// The same checks for many input sets (one flag word each, one read-back);
// errors name the failing job when there are several.  `order` of a job may
// be null; check_ws(total m of the jobs with an order, njobs) bytes.
struct CheckJob {
    const double *samples;
    int64_t n;
    const double *queries;
    int64_t m;
    const int64_t *order;
    int grid, qgrid;
};
sdfi_status validate_jobs(const CheckJob *jobs, int njobs, bool domain, void *scratch, size_t scratch_bytes,
                          const sdfi_options &o, hipStream_t st);

// One uncovered point per sample (witness kernel).  With seg (device, nseg + 1
// offsets) the rows form independent sets, each tested against itself only.
sdfi_status run_witnesses(const double *samples, int64_t n, double *w, uint8_t *st, const sdfi_options &o,
                          hipStream_t s, const int64_t *seg = nullptr, int nseg = 1);

// dense bound sweep used by sdfi_bounds and internally (samples n x 4)
sdfi_status run_bounds(const double *samples, int64_t n, const double *queries, int64_t m, double *lo,
                       double *hi, int32_t *argmax, int32_t *argmin, uint32_t *flags, Carver &ws,
                       const sdfi_options &o, hipStream_t st, int64_t *overflow_count);

sdfi_status run_certify(const double *pv, const double *wit, int64_t N, int64_t *pair_viol, int64_t *wit_viol,
                        Carver &ws, const sdfi_options &o, hipStream_t st);

}  // namespace sdfi
