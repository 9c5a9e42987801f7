// Refinement order (Sec. 4.2): covered-area ratios of grid cells from 8^3
// regular sub-points each (GPU), then a best-first flood fill (host).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <queue>
#include <vector>

#include "common.h"

namespace sdfi {

namespace {

constexpr int SUB = 8;

// Covered sub-points of one cell of a res^3 grid on [0,1]^3, for a work-group
// of 512 threads: thread t tests sub-point ((t%8 + 0.5)/8, ...) against the
// balls, starting with the sample of the input-grid cell (resolution N) that
// holds it.  Returns the count in thread 0.
__device__ int count_cell(const double *__restrict__ p4, int64_t n, int N, int res, int64_t cell, double tol,
                          int *red) {
    const int t = threadIdx.x;
    const int64_t cx = cell % res, cy = (cell / res) % res, cz = cell / ((int64_t)res * res);
    const double size = 1.0 / res;
    // corner + size * (k + 0.5)/8 per axis, the same rounding as the definition
    double x[3];
    {
#pragma clang fp contract(off)
        x[0] = (double)cx * size + size * (((t % SUB) + 0.5) / SUB);
        x[1] = (double)cy * size + size * ((((t / SUB) % SUB) + 0.5) / SUB);
        x[2] = (double)cz * size + size * (((t / (SUB * SUB)) + 0.5) / SUB);
    }
    int ix = min(N - 1, (int)(x[0] * N)), iy = min(N - 1, (int)(x[1] * N)), iz = min(N - 1, (int)(x[2] * N));
    int64_t own = ix + (int64_t)N * (iy + (int64_t)N * iz);
    auto covers = [&](int64_t i) {
#pragma clang fp contract(off)
        const double *p = p4 + 4 * i;
        double dx = x[0] - p[0], dy = x[1] - p[1], dz = x[2] - p[2];
        return sqrt(dx * dx + dy * dy + dz * dz) < fabs(p[3]) - tol;
    };
    int cov = own < n ? covers(own) : 0;
    for (int64_t i = 0; i < n && !cov; ++i) cov = covers(i);
    unsigned long long m = __ballot(cov);
    if ((t & 63) == 0) red[t >> 6] = __popcll(m);
    __syncthreads();
    int sum = 0;
    if (t == 0)
        for (int w = 0; w < 8; ++w) sum += red[w];
    return sum;
}

// One work-group per cell of one grid.
__global__ __launch_bounds__(512) void covered_kernel(const double *__restrict__ p4, int64_t n, int N, int res,
                                                      int64_t cell0, double tol, int *__restrict__ counts) {
    __shared__ int red[8];
    const int64_t cell = cell0 + blockIdx.x;
    const int sum = count_cell(p4, n, N, res, cell, tol, red);
    if (threadIdx.x == 0) counts[cell] = sum;
}

// Covered counts of many grids in one launch: job k owns global blocks
// [start[k], start[k+1]) and counts the res_k^3 cells of the samples
// p4 + 4 sample_off[k] (n_k samples on an N_k^3 grid) into out + out_off[k].
struct CellJob {
    int64_t sample_off, n, out_off;
    int N, res;
};

__global__ __launch_bounds__(512) void covered_jobs_kernel(const double *__restrict__ p4_all, const CellJob *jobs,
                                                           const int64_t *start, int njobs, int64_t block0,
                                                           double tol, int *__restrict__ out) {
    __shared__ int red[8];
    const int64_t gb = block0 + blockIdx.x;
    int lo = 0, hi = njobs - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (start[mid] <= gb) lo = mid;
        else hi = mid - 1;
    }
    const CellJob J = jobs[lo];
    const int64_t cell = gb - start[lo];
    const int sum = count_cell(p4_all + 4 * J.sample_off, J.n, J.N, J.res, cell, tol, red);
    if (threadIdx.x == 0) out[J.out_off + cell] = sum;
}

sdfi_status counts_of(const double *p4, int64_t n, int N, int res, int *dev_counts, std::vector<int> &host,
                      const sdfi_options &o, hipStream_t st) {
    const int64_t cells = (int64_t)res * res * res;
    for (int64_t c0 = 0; c0 < cells; c0 += (1 << 20)) {
        int64_t cnt = std::min<int64_t>(1 << 20, cells - c0);
        covered_kernel<<<(unsigned)cnt, 512, 0, st>>>(p4, n, N, res, c0, o.tol, dev_counts);
        SDFI_HIP(hipGetLastError());
    }
    host.resize(cells);
    SDFI_HIP(hipMemcpyAsync(host.data(), dev_counts, sizeof(int) * cells, hipMemcpyDeviceToHost, st));
    SDFI_HIP(hipStreamSynchronize(st));
    return SDFI_OK;
}

std::vector<int64_t> flood(const std::vector<int> &cnt, int res) {
    const int64_t cells = (int64_t)res * res * res;
    typedef std::pair<int, int64_t> key;  // (count, linear index)
    std::priority_queue<key, std::vector<key>, std::greater<key>> pq;
    int64_t start = 0;
    for (int64_t c = 1; c < cells; ++c)
        if (cnt[c] < cnt[start]) start = c;
    std::vector<char> seen(cells, 0), queued(cells, 0);
    pq.push({cnt[start], start});
    queued[start] = 1;
    std::vector<int64_t> out;
    out.reserve(cells);
    const int dx[6] = {-1, 1, 0, 0, 0, 0}, dy[6] = {0, 0, -1, 1, 0, 0}, dz[6] = {0, 0, 0, 0, -1, 1};
    while (!pq.empty()) {
        key k = pq.top();
        pq.pop();
        int64_t c = k.second;
        if (seen[c]) continue;
        seen[c] = 1;
        out.push_back(c);
        int64_t x = c % res, y = (c / res) % res, z = c / ((int64_t)res * res);
        for (int e = 0; e < 6; ++e) {
            int64_t X = x + dx[e], Y = y + dy[e], Z = z + dz[e];
            if (X < 0 || Y < 0 || Z < 0 || X >= res || Y >= res || Z >= res) continue;
            int64_t nb = X + res * (Y + (int64_t)res * Z);
            if (!queued[nb]) {
                queued[nb] = 1;
                pq.push({cnt[nb], nb});
            }
        }
    }
    return out;
}

// the children of the cells in flood order, each cell's 8 by ascending child
// count (ties: child index bx + 2 by + 4 bz), as linear (2N)^3 indices
void emit_children(const std::vector<int64_t> &cells, const int *child, int N, int64_t *out) {
    const int64_t F = 2 * (int64_t)N;
    int64_t k = 0;
    for (int64_t c : cells) {
        int64_t x = c % N, y = (c / N) % N, z = c / ((int64_t)N * N);
        std::pair<int, int> kids[8];
        int64_t qi[8];
        for (int b = 0; b < 8; ++b) {
            int64_t q = (2 * x + (b & 1)) + F * ((2 * y + ((b >> 1) & 1)) + F * (2 * z + ((b >> 2) & 1)));
            kids[b] = {child[q], b};
            qi[b] = q;
        }
        std::sort(kids, kids + 8);
        for (int b = 0; b < 8; ++b) out[k++] = qi[kids[b].second];
    }
}

}  // namespace

size_t order_ws(int64_t n, int64_t m, const sdfi_options &o) {
    // (2N)^3 cell counts; without a grid (batched instances) the parent and
    // child counts of every instance: 9 n
    int64_t fine = (int64_t)2 * o.grid;
    int64_t cells = o.grid > 0 ? fine * fine * fine : 9 * n;
    return sizeof(int) * (size_t)std::max<int64_t>(cells, 1) + 4096 + check_ws(0) +
           (o.grid > 0 ? 0 : (sizeof(CellJob) + sizeof(int64_t)) * (size_t)(2 * n + 4) + 1024);
}

// Refinement orders of many grid instances (instance b: samples rows
// [soff[b], soff[b+1]) on a grids[b]^3 grid, queries its (2 grids[b])^3 child
// cells): every covered count in one launch, one read-back, the flood fills
// on the host, one upload.
sdfi_status run_order_batched(int ninst, const int64_t *soff, const int32_t *grids, const double *samples,
                              int64_t *order_out, Carver &ws, const sdfi_options &o, hipStream_t st) {
    std::vector<CellJob> jobs;
    std::vector<int64_t> start(1, 0);
    int64_t outpos = 0;
    for (int b = 0; b < ninst; ++b) {
        const int N = grids[b];
        for (int res : {N, 2 * N}) {
            CellJob J;
            J.sample_off = soff[b];
            J.n = soff[b + 1] - soff[b];
            J.out_off = outpos;
            J.N = N;
            J.res = res;
            const int64_t cells = (int64_t)res * res * res;
            jobs.push_back(J);
            start.push_back(start.back() + cells);
            outpos += cells;
        }
    }
    const int njobs = (int)jobs.size();
    int *dc = ws.take<int>(outpos > 0 ? outpos : 1);
    CellJob *dj = ws.take<CellJob>(njobs);
    int64_t *ds = ws.take<int64_t>(njobs + 1);
    if (!ws.ok()) {
        set_error("workspace too small for the refinement orders");
        return SDFI_ERR_WORKSPACE;
    }
    SDFI_HIP(hipMemcpyAsync(dj, jobs.data(), sizeof(CellJob) * njobs, hipMemcpyHostToDevice, st));
    SDFI_HIP(hipMemcpyAsync(ds, start.data(), sizeof(int64_t) * (njobs + 1), hipMemcpyHostToDevice, st));
    for (int64_t b0 = 0; b0 < outpos; b0 += (int64_t(1) << 24)) {
        const int64_t cnt = std::min<int64_t>(int64_t(1) << 24, outpos - b0);
        covered_jobs_kernel<<<(unsigned)cnt, 512, 0, st>>>(samples, dj, ds, njobs, b0, o.tol, dc);
        SDFI_HIP(hipGetLastError());
    }
    std::vector<int> host(outpos);
    SDFI_HIP(hipMemcpyAsync(host.data(), dc, sizeof(int) * outpos, hipMemcpyDeviceToHost, st));
    SDFI_HIP(hipStreamSynchronize(st));
    std::vector<int64_t> order;
    int64_t total = 0;
    for (int b = 0; b < ninst; ++b) total += (int64_t)8 * grids[b] * grids[b] * grids[b];
    order.resize(total);
    int64_t qpos = 0;
    for (int b = 0; b < ninst; ++b) {
        const int N = grids[b];
        std::vector<int> parent(host.begin() + jobs[2 * b].out_off,
                                host.begin() + jobs[2 * b].out_off + (int64_t)N * N * N);
        std::vector<int64_t> cells = flood(parent, N);
        emit_children(cells, host.data() + jobs[2 * b + 1].out_off, N, order.data() + qpos);
        qpos += (int64_t)8 * N * N * N;
    }
    SDFI_HIP(hipMemcpyAsync(order_out, order.data(), sizeof(int64_t) * total, hipMemcpyHostToDevice, st));
    SDFI_HIP(hipStreamSynchronize(st));
    return SDFI_OK;
}

sdfi_status run_order(const double *samples, int64_t n, const double *queries, int64_t m, int64_t *order_out,
                      Carver &ws, const sdfi_options &o, hipStream_t st) {
    const int N = o.grid;
    int *dc = ws.take<int>((size_t)8 * N * N * N);
    if (!ws.ok()) {
        set_error("workspace too small for the refinement order");
        return SDFI_ERR_WORKSPACE;
    }
    std::vector<int> parent, child;
    sdfi_status s = counts_of(samples, n, N, N, dc, parent, o, st);
    if (s != SDFI_OK) return s;
    std::vector<int64_t> cells = flood(parent, N);
    std::vector<int64_t> order;
    order.reserve(m);
    if (!queries) {
        s = counts_of(samples, n, N, 2 * N, dc, child, o, st);
        if (s != SDFI_OK) return s;
        order.resize(cells.size() * 8);
        emit_children(cells, child.data(), N, order.data());
    } else {
        std::vector<double> hq(3 * m);
        SDFI_HIP(hipMemcpyAsync(hq.data(), queries, sizeof(double) * 3 * m, hipMemcpyDeviceToHost, st));
        SDFI_HIP(hipStreamSynchronize(st));
        std::vector<int64_t> rank((size_t)N * N * N);
        for (size_t k = 0; k < cells.size(); ++k) rank[cells[k]] = (int64_t)k;
        std::vector<std::pair<int64_t, int64_t>> key(m);
        for (int64_t j = 0; j < m; ++j) {
            int64_t c[3];
            for (int a = 0; a < 3; ++a) c[a] = std::min<int64_t>(N - 1, std::max<int64_t>(0, (int64_t)std::floor(hq[3 * j + a] * N)));
            key[j] = {rank[c[0] + N * (c[1] + (int64_t)N * c[2])], j};
        }
        std::sort(key.begin(), key.end());
        for (auto &k : key) order.push_back(k.second);
    }
    if ((int64_t)order.size() != m) {
        set_error("refinement order produced %zu entries for %lld queries", order.size(), (long long)m);
        return SDFI_ERR_INVALID_ARGUMENT;
    }
    SDFI_HIP(hipMemcpyAsync(order_out, order.data(), sizeof(int64_t) * m, hipMemcpyHostToDevice, st));
    SDFI_HIP(hipStreamSynchronize(st));
    return SDFI_OK;
}

}  // namespace sdfi

extern "C" sdfi_status sdfi_refinement_order(const double *samples, int64_t n, const double *queries, int64_t m,
                                             int64_t *order_out, void *ws, size_t ws_bytes, const sdfi_options *opt,
                                             sdfi_stream stream) {
    using namespace sdfi;
    sdfi_options o;
    sdfi_status s = read_options(opt, &o);
    if (s != SDFI_OK) return s;
    SDFI_CHECK_ARG(o.grid > 0, "sdfi_refinement_order needs opt->grid > 0");
    SDFI_CHECK_ARG((int64_t)o.grid * o.grid * o.grid == n, "n must equal grid^3");
    SDFI_CHECK_ARG(samples && order_out, "null array argument");
    if (!queries) SDFI_CHECK_ARG(m == 8 * n, "refinement queries: m must be 8 n");
    SDFI_CHECK_ARG(m >= 0, "negative m");
    if (m == 0) return SDFI_OK;
    if (ws_bytes < order_ws(n, m, o) || !ws) {
        set_error("workspace of %zu bytes is below the %zu required", ws_bytes, order_ws(n, m, o));
        return SDFI_ERR_WORKSPACE;
    }
    Carver c(ws, ws_bytes);
    char *chk = c.take<char>(check_ws(0));
    s = validate_inputs(samples, n, queries, queries ? m : 0, nullptr, o.grid, 0, false, chk, check_ws(0), o,
                        to_hip(stream));
    if (s != SDFI_OK) return s;
    return run_order(samples, n, queries, m, order_out, c, o, to_hip(stream));
}
