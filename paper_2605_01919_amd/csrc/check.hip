// Input validation shared by the synchronous entry points: non-finite
// coordinates or values, sample or query points outside the domain box
// (Appendix B considers only points of [-1,1]^d; spheres may reach beyond
// it), samples that are not the cell centres
// of the grid the refinement order assumes (Sec. 4.1), and caller orders that
// are not permutations.  Each check runs on the device and leaves a few flag
// words that the host reads back once.
#include <vector>

#include "common.h"

namespace sdfi {

namespace {

enum : unsigned {
    BAD_NONFINITE = 1,    // a coordinate or value is NaN or infinite
    BAD_SAMPLE_DOMAIN = 2,// a sample point lies outside the domain box
    BAD_POINT_DOMAIN = 4, // a query point lies outside the domain box
    BAD_GRID = 8,         // a sample (query) is not the expected grid cell centre
    BAD_PERM_RANGE = 16,  // an order entry outside [0, m)
    BAD_PERM_REPEAT = 32  // an order entry repeated (so another is missing)
};

struct Box {
    double lo[3], hi[3];
};

__global__ void scan_kernel(const double *__restrict__ samples, int64_t n, const double *__restrict__ queries,
                            int64_t m, Box box, double tol, int grid, int qgrid, unsigned *flag) {
    unsigned f = 0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n + m; i += stride) {
        if (i < n) {
            const double *p = samples + 4 * i;
            if (!isfinite(p[0]) || !isfinite(p[1]) || !isfinite(p[2]) || !isfinite(p[3])) {
                f |= BAD_NONFINITE;
                continue;
            }
            for (int k = 0; k < 3; ++k)
                if (p[k] < box.lo[k] - tol || p[k] > box.hi[k] + tol) f |= BAD_SAMPLE_DOMAIN;
            if (grid > 0) {
                // sample i must lie in cell (i % N, i / N % N, i / N^2) (its centre,
                // up to perturbations such as finite differences)
                const int64_t c[3] = {i % grid, (i / grid) % grid, i / ((int64_t)grid * grid)};
                for (int k = 0; k < 3; ++k)
                    if (!(fabs(p[k] - (c[k] + 0.5) / grid) < 0.5 / grid)) f |= BAD_GRID;
            }
        } else {
            const double *q = queries + 3 * (i - n);
            if (!isfinite(q[0]) || !isfinite(q[1]) || !isfinite(q[2])) {
                f |= BAD_NONFINITE;
                continue;
            }
            for (int k = 0; k < 3; ++k)
                if (q[k] < box.lo[k] - tol || q[k] > box.hi[k] + tol) f |= BAD_POINT_DOMAIN;
            if (qgrid > 0) {
                const int64_t j = i - n;
                const int64_t c[3] = {j % qgrid, (j / qgrid) % qgrid, j / ((int64_t)qgrid * qgrid)};
                for (int k = 0; k < 3; ++k)
                    if (!(fabs(q[k] - (c[k] + 0.5) / qgrid) < 0.5 / qgrid)) f |= BAD_GRID;
            }
        }
    }
    if (f) atomicOr(flag, f);
}

__global__ void zero_u32_kernel(unsigned *p, int64_t k) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < k) p[i] = 0u;
}

__global__ void perm_count_kernel(const int64_t *__restrict__ order, int64_t m, unsigned *seen, unsigned *flag) {
    const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (k >= m) return;
    const int64_t j = order[k];
    if (j < 0 || j >= m) {
        atomicOr(flag, (unsigned)BAD_PERM_RANGE);
        return;
    }
    if (atomicAdd(&seen[j], 1u) != 0u) atomicOr(flag, (unsigned)BAD_PERM_REPEAT);
}

}  // namespace

size_t check_ws(int64_t m, int64_t njobs) {
    return sizeof(unsigned) * (size_t)(m + 64 * ((njobs + 63) / 64)) + 512;
}

sdfi_status validate_jobs(const CheckJob *jobs, int njobs, bool domain, void *scratch, size_t scratch_bytes,
                          const sdfi_options &o, hipStream_t st) {
    int64_t mtot = 0;
    for (int j = 0; j < njobs; ++j)
        if (jobs[j].order) mtot += jobs[j].m;
    if (njobs <= 0) return SDFI_OK;
    if (scratch_bytes < check_ws(mtot, njobs)) {
        set_error("workspace too small for the input checks");
        return SDFI_ERR_WORKSPACE;
    }
    // one flag word per job, then the permutation counts of the jobs with an order
    unsigned *flag = static_cast<unsigned *>(scratch);
    unsigned *seen = flag + 64 * ((njobs + 63) / 64);
    zero_u32_kernel<<<(njobs + 255) / 256, 256, 0, st>>>(flag, njobs);
    if (mtot > 0) zero_u32_kernel<<<(unsigned)((mtot + 255) / 256), 256, 0, st>>>(seen, mtot);
    Box box;
    for (int k = 0; k < 3; ++k) {
        // without the domain check the box is unbounded and only the other tests run
        box.lo[k] = domain ? o.domain_lo[k] : -INFINITY;
        box.hi[k] = domain ? o.domain_hi[k] : INFINITY;
    }
    int64_t spos = 0;
    for (int j = 0; j < njobs; ++j) {
        const CheckJob &J = jobs[j];
        const int64_t tot = J.n + J.m;
        if (tot > 0) {
            const unsigned blocks = (unsigned)std::min<int64_t>((tot + 255) / 256, 2048);
            scan_kernel<<<blocks, 256, 0, st>>>(J.samples, J.n, J.queries, J.m, box, o.tol, J.grid, J.qgrid,
                                                flag + j);
        }
        if (J.order && J.m > 0) {
            perm_count_kernel<<<(unsigned)((J.m + 255) / 256), 256, 0, st>>>(J.order, J.m, seen + spos, flag + j);
            spos += J.m;
        }
    }
    SDFI_HIP(hipGetLastError());
    std::vector<unsigned> h(njobs);
    SDFI_HIP(hipMemcpyAsync(h.data(), flag, sizeof(unsigned) * njobs, hipMemcpyDeviceToHost, st));
    SDFI_HIP(hipStreamSynchronize(st));
    for (int j = 0; j < njobs; ++j) {
        char where[48] = "";
        if (njobs > 1) snprintf(where, sizeof where, "instance %d: ", j);
        if (h[j] & BAD_NONFINITE) {
            set_error("%san input coordinate or value is NaN or infinite", where);
            return SDFI_ERR_INVALID_ARGUMENT;
        }
        if (h[j] & (BAD_PERM_RANGE | BAD_PERM_REPEAT)) {
            set_error("%sorder_in is not a permutation of [0, m): %s", where,
                      (h[j] & BAD_PERM_RANGE) ? "an entry lies outside [0, m)" : "an entry is repeated");
            return SDFI_ERR_INVALID_ARGUMENT;
        }
        if (h[j] & BAD_GRID) {
            set_error("%sthe samples (queries) do not lie in the cells of the %d^3 (%d^3) grid on [0,1]^3, x fastest",
                      where, jobs[j].grid, jobs[j].qgrid);
            return SDFI_ERR_DOMAIN;
        }
        if (h[j] & BAD_SAMPLE_DOMAIN) {
            set_error("%sa sample point lies outside the domain box (Appendix B considers only its points)", where);
            return SDFI_ERR_DOMAIN;
        }
        if (h[j] & BAD_POINT_DOMAIN) {
            set_error("%sa query point lies outside the domain box", where);
            return SDFI_ERR_DOMAIN;
        }
    }
    return SDFI_OK;
}

sdfi_status validate_inputs(const double *samples, int64_t n, const double *queries, int64_t m,
                            const int64_t *order, int grid, int qgrid, bool domain, void *scratch,
                            size_t scratch_bytes, const sdfi_options &o, hipStream_t st) {
    CheckJob J{samples, n, queries, m, order, grid, qgrid};
    return validate_jobs(&J, 1, domain, scratch, scratch_bytes, o, st);
}

}  // namespace sdfi
