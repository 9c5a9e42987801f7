// Entry points not built yet: report SDFI_ERR_UNSUPPORTED.
#include "common.h"

namespace sdfi {
size_t order_ws(int64_t, int64_t, const sdfi_options &) { return 256; }
size_t witness_ws(int64_t, const sdfi_options &) { return 256; }
size_t greedy_ws(int64_t, int64_t, const sdfi_options &) { return 256; }
size_t rmin_ws(int64_t, int64_t, const sdfi_options &) { return 256; }
size_t repair_ws(int64_t, int64_t, const sdfi_options &) { return 256; }
size_t backward_ws(int64_t, int64_t) { return 256; }
}  // namespace sdfi

extern "C" {
static sdfi_status pending(const char *name) {
    sdfi::set_error("%s is not available in this build", name);
    return SDFI_ERR_UNSUPPORTED;
}
sdfi_status sdfi_refinement_order(const double *, int64_t, const double *, int64_t, int64_t *, void *, size_t,
                                  const sdfi_options *, sdfi_stream) { return pending("sdfi_refinement_order"); }
sdfi_status sdfi_sample_witnesses(const double *, int64_t, double *, uint8_t *, void *, size_t,
                                  const sdfi_options *, sdfi_stream) { return pending("sdfi_sample_witnesses"); }
sdfi_status sdfi_greedy_interpolate(const double *, int64_t, const double *, int64_t, const int64_t *, double *,
                                    int64_t *, int64_t *, uint8_t *, double *, double *, sdfi_report *, void *,
                                    size_t, const sdfi_options *, sdfi_stream) { return pending("sdfi_greedy_interpolate"); }
sdfi_status sdfi_greedy_interpolate_batched(int32_t, const int64_t *, const int64_t *, const int32_t *,
                                            const double *, const double *, double *, int64_t *, int64_t *,
                                            uint8_t *, double *, sdfi_report *, void *, size_t,
                                            const sdfi_options *, sdfi_stream) { return pending("sdfi_greedy_interpolate_batched"); }
sdfi_status sdfi_min_valid_radius(const double *, int64_t, const double *, int64_t, double *, uint8_t *, double *,
                                  void *, size_t, const sdfi_options *, sdfi_stream) { return pending("sdfi_min_valid_radius"); }
sdfi_status sdfi_repair(const double *, int64_t, const double *, int64_t, double *, uint8_t *, double *, uint8_t *,
                        sdfi_report *, void *, size_t, const sdfi_options *, sdfi_stream) { return pending("sdfi_repair"); }
sdfi_status sdfi_greedy_backward(const double *, const double *, int64_t, const double *, int64_t, const double *,
                                 const int64_t *, const uint8_t *, double *, double *, void *, size_t,
                                 sdfi_stream) { return pending("sdfi_greedy_backward"); }
}
