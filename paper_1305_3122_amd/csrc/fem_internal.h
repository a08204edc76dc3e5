// fem_internal.h -- shared host/device helpers of the gfx950 assembly library.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdint>
#include <cstdio>

#include "../../include/fem_p1.h"

namespace fem {

// ---------------------------------------------------------------- errors

int set_error(int code, const char *fmt, ...);
void clear_error();

#define FEM_HIP_CHECK(expr)                                                              \
    do {                                                                                 \
        hipError_t e_ = (expr);                                                          \
        if (e_ != hipSuccess)                                                            \
            return ::fem::set_error(FEM_EHIP, "%s: %s (%s:%d)", #expr,                   \
                                    hipGetErrorString(e_), __FILE__, __LINE__);          \
    } while (0)

#define FEM_LAUNCH_CHECK() FEM_HIP_CHECK(hipGetLastError())

#define FEM_REQUIRE(cond, code, ...)                                                     \
    do {                                                                                 \
        if (!(cond))                                                                     \
            return ::fem::set_error((code), __VA_ARGS__);                                \
    } while (0)

inline hipStream_t as_stream(void *s) { return reinterpret_cast<hipStream_t>(s); }

inline unsigned grid_for(int64_t n, int block) {
    int64_t g = (n + block - 1) / block;
    return static_cast<unsigned>(g < 1 ? 1 : g);
}

// ---------------------------------------------------------------- constants

constexpr int WAVE = 64;

// Device-side error bits of the symbolic phase.
enum : int {
    ERR_RANGE = 1,        // vertex index outside [0, nq)
    ERR_DEGEN = 2,        // repeated vertex in a triangle
    ERR_OVERFLOW = 4,     // a prefix sum exceeded int32
    ERR_ROWLEN = 8,       // a row longer than 65535 entries
};

// Layout of the small counter block at the head of the pattern workspace.
struct PatternCounters {
    int err;              // OR of ERR_* bits
    int wide_count;       // vertices routed to the workgroup-per-row path
    int max_row_len;      // longest CSR row
    int max_inc;          // most triangles around one vertex
    int mid_count;        // vertices routed to the per-lane LDS path
    int pad_;
    long long total[4];   // totals written by the scans
};

// ---------------------------------------------------------------- fan codes
//
// Fan code of a CSR row i (fem_fan_plan, one uint64 per row): the neighbour
// slots of vertex i in the order its triangles are met turning around i,
// such that step j of the walk is the triangle (i, s_j, s_{j+1}) in that
// triangle's own vertex order (indices mod n for a closed fan).
//   bits 0..3       n, the number of neighbour slots; 0: the row has no
//                   single consistently oriented fan (or is too long), and
//                   is summed in ascending triangle order instead
//   bit  4          closed (vertex inside the mesh: n triangles; else n - 1)
//   bits 5..8       the row slot of the diagonal entry
//   bits 9 + 4j ..  slot s_j, j < n <= FAN_NMAX
constexpr int FAN_NMAX = 13;

__host__ __device__ inline int fan_n(uint64_t c) { return (int)(c & 15u); }
__host__ __device__ inline bool fan_closed(uint64_t c) { return ((c >> 4) & 1u) != 0; }
__host__ __device__ inline int fan_pd(uint64_t c) { return (int)((c >> 5) & 15u); }
__host__ __device__ inline int fan_slot(uint64_t c, int j) { return (int)((c >> (9 + 4 * j)) & 15u); }

// ---------------------------------------------------------------- device helpers

// Inclusive prefix sum over the 64 lanes of a wave.
template <typename T>
__device__ inline T wave_inclusive_scan(T v) {
    const int lane = threadIdx.x & (WAVE - 1);
#pragma unroll
    for (int d = 1; d < WAVE; d <<= 1) {
        T u = __shfl_up(v, d, WAVE);
        if (lane >= d) v += u;
    }
    return v;
}

template <typename T>
__device__ inline T wave_sum(T v) {
#pragma unroll
    for (int d = WAVE / 2; d > 0; d >>= 1) v += __shfl_xor(v, d, WAVE);
    return v;
}

// Zero / fill kernels (used instead of hipMemsetAsync so that captured
// graphs replay correctly).
__global__ void k_fill_i32(int32_t *p, int64_t n, int32_t v);
// Bucket partitions: in place over counts[blk][b] (nblk rows of nbkt), each
// entry becomes the count of bucket b in the rows before blk; bsum[b] gets
// the column total.  COLSCAN_WAVES * 64 threads per workgroup, 64 buckets per
// workgroup.
constexpr int COLSCAN_WAVES = 16;
__global__ void k_bkt_colscan(int32_t nbkt, int32_t nblk, int32_t *counts, int32_t *bsum);
__global__ void k_fill_f64(double *p, int64_t n, double v);

int fill_i32(int32_t *p, int64_t n, int32_t v, hipStream_t s);
int fill_f64(double *p, int64_t n, double v, hipStream_t s);

// Exclusive scan of n int32 counts into out[0..n] (out[n] = total).  `part`
// needs scan_partials(n) int64 slots.  The total is also stored to
// *total_dev; ERR_OVERFLOW is OR-ed into *err_dev if it exceeds INT32_MAX.
int64_t scan_partials(int64_t n);
int exclusive_scan_i32(const int32_t *in, int32_t *out, int64_t n, long long *part,
                       long long *total_dev, int *err_dev, hipStream_t s);

}  // namespace fem
