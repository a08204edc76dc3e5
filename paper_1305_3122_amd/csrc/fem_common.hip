// fem_common.hip -- error state, fill kernels, device-wide exclusive scan, HIP
// graph capture helpers.
#include "fem_internal.h"

#include <cstring>

namespace fem {

namespace {
thread_local char g_msg[512] = "";
}

int set_error(int code, const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_msg, sizeof(g_msg), fmt, ap);
    va_end(ap);
    return code;
}

void clear_error() { g_msg[0] = '\0'; }

const char *last_error() { return g_msg; }

// ---------------------------------------------------------------- fills

__global__ void k_fill_i32(int32_t *p, int64_t n, int32_t v) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void k_fill_f64(double *p, int64_t n, double v) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

static unsigned fill_grid(int64_t n) {
    int64_t g = (n + 255) / 256;
    if (g > 65536) g = 65536;
    return static_cast<unsigned>(g < 1 ? 1 : g);
}

int fill_i32(int32_t *p, int64_t n, int32_t v, hipStream_t s) {
    if (n <= 0) return FEM_OK;
    hipLaunchKernelGGL(k_fill_i32, dim3(fill_grid(n)), dim3(256), 0, s, p, n, v);
    FEM_LAUNCH_CHECK();
    return FEM_OK;
}

int fill_f64(double *p, int64_t n, double v, hipStream_t s) {
    if (n <= 0) return FEM_OK;
    hipLaunchKernelGGL(k_fill_f64, dim3(fill_grid(n)), dim3(256), 0, s, p, n, v);
    FEM_LAUNCH_CHECK();
    return FEM_OK;
}

// ---------------------------------------------------------------- scan
//
// Reduce-then-scan over chunks of SCAN_CHUNK counts: (1) one workgroup per
// chunk sums it, (2) one workgroup scans the chunk sums, (3) one workgroup per
// chunk scans its chunk and adds the chunk offset.  Sums are int64.

constexpr int SCAN_THREADS = 256;
constexpr int SCAN_ITEMS = 4;
constexpr int SCAN_CHUNK = SCAN_THREADS * SCAN_ITEMS;

int64_t scan_partials(int64_t n) { return (n + SCAN_CHUNK - 1) / SCAN_CHUNK + 1; }

// Exclusive scan of one value per thread across a workgroup of SCAN_THREADS;
// returns the exclusive prefix and writes the workgroup total to *total.
__device__ inline long long block_exclusive_scan(long long v, long long *total) {
    __shared__ long long wsum[SCAN_THREADS / WAVE];
    const int lane = threadIdx.x & (WAVE - 1);
    const int wid = threadIdx.x / WAVE;
    long long inc = wave_inclusive_scan(v);
    if (lane == WAVE - 1) wsum[wid] = inc;
    __syncthreads();
    long long off = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < SCAN_THREADS / WAVE; ++w) {
        if (w < wid) off += wsum[w];
        tot += wsum[w];
    }
    __syncthreads();
    *total = tot;
    return off + inc - v;
}

__global__ __launch_bounds__(SCAN_THREADS) void k_scan_reduce(const int32_t *in, int64_t n,
                                                              long long *part) {
    const int64_t base = (int64_t)blockIdx.x * SCAN_CHUNK;
    long long s = 0;
#pragma unroll
    for (int t = 0; t < SCAN_ITEMS; ++t) {
        int64_t i = base + (int64_t)t * SCAN_THREADS + threadIdx.x;
        if (i < n) s += in[i];
    }
    long long tot;
    block_exclusive_scan(s, &tot);
    if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

__global__ __launch_bounds__(SCAN_THREADS) void k_scan_partials(long long *part, int64_t nparts,
                                                                int32_t *out, int64_t n,
                                                                long long *total_dev,
                                                                int *err_dev) {
    // each thread owns a contiguous run of partial sums
    const int64_t per = (nparts + SCAN_THREADS - 1) / SCAN_THREADS;
    const int64_t b0 = threadIdx.x * per;
    const int64_t b1 = (b0 + per < nparts) ? b0 + per : nparts;
    long long s = 0;
    for (int64_t b = b0; b < b1; ++b) s += part[b];
    long long tot;
    long long off = block_exclusive_scan(s, &tot);
    for (int64_t b = b0; b < b1; ++b) {
        long long v = part[b];
        part[b] = off;
        off += v;
    }
    if (threadIdx.x == 0) {
        *total_dev = tot;
        if (tot > INT32_MAX) atomicOr(err_dev, ERR_OVERFLOW);
        out[n] = static_cast<int32_t>(tot);
    }
}

__global__ __launch_bounds__(SCAN_THREADS) void k_scan_down(const int32_t *in, int64_t n,
                                                            const long long *part, int32_t *out) {
    const int64_t base = (int64_t)blockIdx.x * SCAN_CHUNK + (int64_t)threadIdx.x * SCAN_ITEMS;
    int32_t v[SCAN_ITEMS];
    long long s = 0;
#pragma unroll
    for (int t = 0; t < SCAN_ITEMS; ++t) {
        v[t] = (base + t < n) ? in[base + t] : 0;
        s += v[t];
    }
    long long tot;
    long long off = block_exclusive_scan(s, &tot) + part[blockIdx.x];
#pragma unroll
    for (int t = 0; t < SCAN_ITEMS; ++t) {
        if (base + t < n) out[base + t] = static_cast<int32_t>(off);
        off += v[t];
    }
}

int exclusive_scan_i32(const int32_t *in, int32_t *out, int64_t n, long long *part,
                       long long *total_dev, int *err_dev, hipStream_t s) {
    const int64_t nparts = (n + SCAN_CHUNK - 1) / SCAN_CHUNK;
    if (nparts > 0) {
        hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)nparts), dim3(SCAN_THREADS), 0, s, in, n,
                           part);
        FEM_LAUNCH_CHECK();
    }
    hipLaunchKernelGGL(k_scan_partials, dim3(1), dim3(SCAN_THREADS), 0, s, part, nparts, out, n,
                       total_dev, err_dev);
    FEM_LAUNCH_CHECK();
    if (nparts > 0) {
        hipLaunchKernelGGL(k_scan_down, dim3((unsigned)nparts), dim3(SCAN_THREADS), 0, s, in, n,
                           part, out);
        FEM_LAUNCH_CHECK();
    }
    return FEM_OK;
}

}  // namespace fem

// ---------------------------------------------------------------- C ABI

extern "C" const char *fem_last_error(void) { return fem::last_error(); }

extern "C" int fem_version(void) { return 200; }

extern "C" int fem_graph_begin(void *stream) {
    fem::clear_error();
    FEM_REQUIRE(stream != nullptr, FEM_EINVAL, "fem_graph_begin: the NULL stream cannot be captured");
    FEM_HIP_CHECK(hipStreamBeginCapture(fem::as_stream(stream), hipStreamCaptureModeThreadLocal));
    return FEM_OK;
}

extern "C" int fem_graph_end(void *stream, void **graph_out) {
    fem::clear_error();
    FEM_REQUIRE(stream != nullptr && graph_out != nullptr, FEM_EINVAL,
                "fem_graph_end: NULL stream or graph_out");
    hipGraph_t g = nullptr;
    FEM_HIP_CHECK(hipStreamEndCapture(fem::as_stream(stream), &g));
    hipGraphExec_t ex = nullptr;
    hipError_t e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess)
        return fem::set_error(FEM_EHIP, "hipGraphInstantiate: %s", hipGetErrorString(e));
    *graph_out = reinterpret_cast<void *>(ex);
    return FEM_OK;
}

extern "C" int fem_graph_launch(void *graph, void *stream) {
    fem::clear_error();
    FEM_REQUIRE(graph != nullptr, FEM_EINVAL, "fem_graph_launch: NULL graph");
    FEM_HIP_CHECK(hipGraphLaunch(reinterpret_cast<hipGraphExec_t>(graph), fem::as_stream(stream)));
    return FEM_OK;
}

extern "C" int fem_graph_destroy(void *graph) {
    fem::clear_error();
    if (graph == nullptr) return FEM_OK;
    FEM_HIP_CHECK(hipGraphExecDestroy(reinterpret_cast<hipGraphExec_t>(graph)));
    return FEM_OK;
}
