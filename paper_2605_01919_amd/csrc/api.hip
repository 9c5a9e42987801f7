// Library-wide entry points: options, errors, version, workspace sizes.
#include "common.h"

#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

namespace sdfi {

static thread_local char g_err[512] = "";
thread_local bool g_no_alloc = false;

void set_error(const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
}

namespace {
struct Pending {
    std::string name;
    hipEvent_t a, b;
};
std::mutex g_tm;
bool g_timing = false;
std::vector<Pending> g_pending;
std::map<std::string, std::pair<double, int64_t>> g_acc;
struct PendingCount {
    std::string name;
    int64_t *host;  // pinned
    hipEvent_t done;
};
std::vector<PendingCount> g_pcount;
std::map<std::string, int64_t> g_count;

void drain_locked() {
    for (auto &p : g_pending) {
        float ms = 0.0f;
        if (hipEventSynchronize(p.b) == hipSuccess && hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
            auto &e = g_acc[p.name];
            e.first += ms;
            e.second += 1;
        }
        (void)hipEventDestroy(p.a);
        (void)hipEventDestroy(p.b);
    }
    g_pending.clear();
    for (auto &p : g_pcount) {
        if (hipEventSynchronize(p.done) == hipSuccess) g_count[p.name] += *p.host;
        (void)hipEventDestroy(p.done);
        (void)hipHostFree(p.host);
    }
    g_pcount.clear();
}
}  // namespace

KernelTimer::KernelTimer(const char *n, hipStream_t s) : name(n), st(s) {
    if (g_no_alloc) return;
    std::lock_guard<std::mutex> lk(g_tm);
    if (!g_timing) return;
    if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) {
        a = b = nullptr;
        return;
    }
    (void)hipEventRecord(a, st);
}

void KernelTimer::stop() {
    if (!a) return;
    (void)hipEventRecord(b, st);
    std::lock_guard<std::mutex> lk(g_tm);
    g_pending.push_back({name, a, b});
    a = b = nullptr;
}

void note_count(const char *n, const int64_t *dev, hipStream_t st) {
    if (g_no_alloc) return;
    std::lock_guard<std::mutex> lk(g_tm);
    if (!g_timing) return;
    PendingCount p{n, nullptr, nullptr};
    if (hipHostMalloc((void **)&p.host, sizeof(int64_t), hipHostMallocDefault) != hipSuccess) return;
    if (hipEventCreate(&p.done) != hipSuccess) {
        (void)hipHostFree(p.host);
        return;
    }
    if (hipMemcpyAsync(p.host, dev, sizeof(int64_t), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipEventRecord(p.done, st) != hipSuccess) {
        (void)hipEventDestroy(p.done);
        (void)hipHostFree(p.host);
        return;
    }
    g_pcount.push_back(p);
}

bool timing_enabled() {
    if (g_no_alloc) return false;
    std::lock_guard<std::mutex> lk(g_tm);
    return g_timing;
}

void add_count(const char *n, int64_t v) {
    if (g_no_alloc) return;
    std::lock_guard<std::mutex> lk(g_tm);
    if (g_timing) g_count[n] += v;
}

sdfi_status read_options(const sdfi_options *opt, sdfi_options *out) {
    sdfi_default_options(out);
    if (!opt) return SDFI_OK;
    if (opt->struct_size != sizeof(sdfi_options)) {
        set_error("sdfi_options.struct_size is %u, expected %zu", opt->struct_size, sizeof(sdfi_options));
        return SDFI_ERR_INVALID_ARGUMENT;
    }
    *out = *opt;
    if (out->precision != SDFI_PREC_FP64 && out->precision != SDFI_PREC_FP32_FP64_RECHECK) {
        set_error("unknown precision %d", out->precision);
        return SDFI_ERR_INVALID_ARGUMENT;
    }
    if (!(out->tol >= 0.0) || !(out->tie_tol >= 0.0)) {
        set_error("tolerances must be non-negative");
        return SDFI_ERR_INVALID_ARGUMENT;
    }
    if (out->grid < 0 || out->grid > 1024) {
        set_error("grid must be in [0, 1024], got %d", out->grid);
        return SDFI_ERR_INVALID_ARGUMENT;
    }
    if (out->block_size != 0 && out->block_size != 256 && out->block_size != 512) {
        set_error("block_size must be 0, 256 or 512, got %d", out->block_size);
        return SDFI_ERR_INVALID_ARGUMENT;
    }
    if (out->groups < 0 || out->groups > 1024) {
        set_error("groups must be in [0, 1024], got %d", out->groups);
        return SDFI_ERR_INVALID_ARGUMENT;
    }
    if (out->flags & ~(uint32_t)(SDFI_OPT_CERTIFY | SDFI_OPT_INPUT_CHECK | SDFI_OPT_EXHAUSTIVE)) {
        set_error("unknown option flags 0x%x", out->flags);
        return SDFI_ERR_INVALID_ARGUMENT;
    }
    for (int k = 0; k < 3; ++k) {
        if (!(out->domain_lo[k] < out->domain_hi[k])) {
            set_error("empty domain box on axis %d", k);
            return SDFI_ERR_INVALID_ARGUMENT;
        }
    }
    return SDFI_OK;
}

}  // namespace sdfi

extern "C" {

void sdfi_default_options(sdfi_options *o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->struct_size = sizeof(sdfi_options);
    o->precision = SDFI_PREC_FP32_FP64_RECHECK;
    o->tol = 1e-6;
    o->tie_tol = 1e-9;
    for (int k = 0; k < 3; ++k) {
        o->domain_lo[k] = -1.0;
        o->domain_hi[k] = 1.0;
    }
    o->grid = 0;
    o->block_size = 0;
    o->flags = 0;
}

const char *sdfi_last_error(void) { return sdfi::g_err; }

void sdfi_timing_enable(int on) {
    std::lock_guard<std::mutex> lk(sdfi::g_tm);
    sdfi::g_timing = on != 0;
}

sdfi_status sdfi_timing_query(const char *name, double *ms, int64_t *launches) {
    SDFI_CHECK_ARG(name && ms && launches, "null argument");
    std::lock_guard<std::mutex> lk(sdfi::g_tm);
    sdfi::drain_locked();
    auto it = sdfi::g_acc.find(name);
    *ms = it == sdfi::g_acc.end() ? 0.0 : it->second.first;
    *launches = it == sdfi::g_acc.end() ? 0 : it->second.second;
    return SDFI_OK;
}

sdfi_status sdfi_counter_query(const char *name, int64_t *value) {
    SDFI_CHECK_ARG(name && value, "null argument");
    std::lock_guard<std::mutex> lk(sdfi::g_tm);
    sdfi::drain_locked();
    auto it = sdfi::g_count.find(name);
    *value = it == sdfi::g_count.end() ? 0 : it->second;
    return SDFI_OK;
}

void sdfi_timing_reset(void) {
    std::lock_guard<std::mutex> lk(sdfi::g_tm);
    sdfi::drain_locked();
    sdfi::g_acc.clear();
    sdfi::g_count.clear();
}

const char *sdfi_version(void) { return "sdfi 0.1 gfx950"; }

sdfi_status sdfi_workspace_size(sdfi_op op, int64_t n, int64_t m, const sdfi_options *opt, size_t *bytes) {
    using namespace sdfi;
    sdfi_options o;
    sdfi_status s = read_options(opt, &o);
    if (s != SDFI_OK) return s;
    SDFI_CHECK_ARG(bytes != nullptr, "bytes is null");
    SDFI_CHECK_ARG(n >= 0 && m >= 0, "negative size");
    switch (op) {
    case SDFI_OP_BOUNDS: *bytes = bounds_ws(n > 0 ? n : 1, m, o); break;
    case SDFI_OP_CERTIFY: *bytes = certify_ws(n, o); break;
    case SDFI_OP_ORDER: *bytes = order_ws(n, m, o); break;
    case SDFI_OP_WITNESS: *bytes = witness_ws(n, o); break;
    case SDFI_OP_GREEDY: *bytes = greedy_ws(n, m, o); break;
    case SDFI_OP_RMIN: *bytes = rmin_ws(n, m, o); break;
    case SDFI_OP_REPAIR: *bytes = repair_ws(n, m, o); break;
    case SDFI_OP_BACKWARD: *bytes = backward_ws(n, m); break;
    case SDFI_OP_GREEDY_INSTANCE: *bytes = greedy_instance_ws(o); break;
    default: set_error("unknown op %d", (int)op); return SDFI_ERR_INVALID_ARGUMENT;
    }
    return SDFI_OK;
}

}  // extern "C"
