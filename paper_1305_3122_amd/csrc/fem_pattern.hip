// fem_pattern.hip -- symbolic phase: CSR pattern, triangle lists per vertex,
// row-relative positions and the optional slot map.
//
// Replaces the global index arrays Ig, Jg of the vectorised assembly
// (Section 5, Remark on Ig/Jg) and the sort/compress that sparse(Ig,Jg,Kg)
// performs.  Instead of sorting 9 nme triplets, every vertex gathers the
// triangles around it and sorts/uniques its own neighbour list in LDS: a P1
// row holds the vertex itself and its mesh neighbours, so rows are short.
//
//   1 count      one lane per triangle: mesh checks, triangles per vertex
//   2 scan       -> inc_ptr
//   3 fill       one lane per triangle: inc[] (unordered inside a vertex)
//   4 rows       one lane per vertex: sort its triangles by id, gather the
//                two other vertices of each, sort+unique in LDS -> row length,
//                row-relative positions (inc_pos), sorted columns (staged)
//   4w rows_wide one workgroup per vertex with more than LANE_MAX triangles
//   5 scan       -> row_ptr, nnz            (host waits here once)
//   6 copy       staged columns -> col_idx
//   7 slot       one lane per triangle: binary search of its 9 entries
#include "fem_internal.h"

namespace fem {

// Triangles per vertex handled by the one-lane-per-vertex path.
constexpr int LANE_MAX = 16;
constexpr int CAND_MAX = 2 * LANE_MAX + 1;

__global__ __launch_bounds__(256) void k_count(int32_t nme, const int32_t *__restrict__ me,
                                               int32_t nq, int32_t *__restrict__ deg,
                                               PatternCounters *cnt) {
    const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (k >= nme) return;
    const int32_t a = me[3 * k], b = me[3 * k + 1], c = me[3 * k + 2];
    if ((uint32_t)a >= (uint32_t)nq || (uint32_t)b >= (uint32_t)nq || (uint32_t)c >= (uint32_t)nq) {
        atomicOr(&cnt->err, ERR_RANGE);
        return;
    }
    if (a == b || b == c || a == c) {
        atomicOr(&cnt->err, ERR_DEGEN);
        return;
    }
    atomicAdd(&deg[a], 1);
    atomicAdd(&deg[b], 1);
    atomicAdd(&deg[c], 1);
}

__global__ __launch_bounds__(256) void k_fill(int32_t nme, const int32_t *__restrict__ me,
                                              int32_t nq, const int32_t *__restrict__ inc_ptr,
                                              int32_t *__restrict__ cursor,
                                              int32_t *__restrict__ inc) {
    const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (k >= nme) return;
    int32_t v[3] = {me[3 * k], me[3 * k + 1], me[3 * k + 2]};
    if ((uint32_t)v[0] >= (uint32_t)nq || (uint32_t)v[1] >= (uint32_t)nq ||
        (uint32_t)v[2] >= (uint32_t)nq || v[0] == v[1] || v[1] == v[2] || v[0] == v[2])
        return;  // skipped consistently with k_count
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const int32_t pos = atomicSub(&cursor[v[a]], 1) - 1;
        inc[(int64_t)inc_ptr[v[a]] + pos] = static_cast<int32_t>(3 * k + a);
    }
}

__device__ inline int32_t lower_bound(const int32_t *a, int32_t n, int32_t x) {
    int32_t lo = 0, hi = n;
    while (lo < hi) {
        int32_t mid = (lo + hi) >> 1;
        if (a[mid] < x) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// Per-lane LDS arrays are stored [slot][lane] so that the 64 lanes of a wave
// touch 64 consecutive words (no bank conflicts).
#define LANE_AT(arr, t) arr[(t) * WAVE + lane]

__global__ __launch_bounds__(WAVE) void k_rows(int32_t nq, const int32_t *__restrict__ inc_ptr,
                                               int32_t *__restrict__ inc,
                                               const int32_t *__restrict__ me,
                                               int32_t *__restrict__ rowlen,
                                               int32_t *__restrict__ stage,
                                               uint32_t *__restrict__ inc_pos,
                                               int32_t *__restrict__ wide_list,
                                               PatternCounters *cnt) {
    __shared__ int32_t s_inc[LANE_MAX * WAVE];
    __shared__ int32_t s_nb[2 * LANE_MAX * WAVE];
    __shared__ int32_t s_col[CAND_MAX * WAVE];
    const int lane = threadIdx.x;
    const int64_t v = blockIdx.x * (int64_t)WAVE + lane;
    const bool in = v < nq;
    const int32_t is = in ? inc_ptr[v] : 0;
    const int32_t d0 = in ? inc_ptr[v + 1] - is : 0;
    const bool wide = d0 > LANE_MAX;
    const int32_t d = wide ? 0 : d0;
    if (wide) {
        wide_list[atomicAdd(&cnt->wide_count, 1)] = static_cast<int32_t>(v);
        rowlen[v] = 0;
    }
    // triangles of v in ascending id (insertion sort)
    for (int t = 0; t < d; ++t) {
        const int32_t x = inc[is + t];
        int j = t;
        while (j > 0 && LANE_AT(s_inc, j - 1) > x) {
            LANE_AT(s_inc, j) = LANE_AT(s_inc, j - 1);
            --j;
        }
        LANE_AT(s_inc, j) = x;
    }
    // the other two vertices of each triangle, in cyclic order after v
    for (int t = 0; t < d; ++t) {
        const int32_t x = LANE_AT(s_inc, t);
        inc[is + t] = x;
        const int64_t k = x / 3;
        const int a = x - 3 * static_cast<int32_t>(k);
        const int a1 = a == 2 ? 0 : a + 1;
        const int a2 = a == 0 ? 2 : a - 1;
        LANE_AT(s_nb, 2 * t) = me[3 * k + a1];
        LANE_AT(s_nb, 2 * t + 1) = me[3 * k + a2];
    }
    // sorted unique columns: v itself and every neighbour (none if v is unused)
    int n = 0;
    for (int t = -1; t < 2 * d; ++t) {
        const int32_t x = t < 0 ? static_cast<int32_t>(v) : LANE_AT(s_nb, t);
        int j = n;
        while (j > 0 && LANE_AT(s_col, j - 1) > x) --j;
        if (j > 0 && LANE_AT(s_col, j - 1) == x) continue;
        for (int m = n; m > j; --m) LANE_AT(s_col, m) = LANE_AT(s_col, m - 1);
        LANE_AT(s_col, j) = x;
        ++n;
    }
    if (d == 0) n = 0;
    // row-relative positions of the two neighbours of each triangle
    for (int t = 0; t < d; ++t) {
        int32_t lo1 = 0, hi1 = n, lo2 = 0, hi2 = n;
        const int32_t x1 = LANE_AT(s_nb, 2 * t), x2 = LANE_AT(s_nb, 2 * t + 1);
        while (lo1 < hi1) {
            int32_t mid = (lo1 + hi1) >> 1;
            if (LANE_AT(s_col, mid) < x1) lo1 = mid + 1;
            else hi1 = mid;
        }
        while (lo2 < hi2) {
            int32_t mid = (lo2 + hi2) >> 1;
            if (LANE_AT(s_col, mid) < x2) lo2 = mid + 1;
            else hi2 = mid;
        }
        inc_pos[is + t] = static_cast<uint32_t>(lo1) | (static_cast<uint32_t>(lo2) << 16);
    }
    if (in && !wide) {
        rowlen[v] = n;
        const int64_t base = 2 * (int64_t)is + v;
        for (int u = 0; u < n; ++u) stage[base + u] = LANE_AT(s_col, u);
    }
    // one atomic per wave for the maxima
    int mr = n, mi = d0;
#pragma unroll
    for (int o = WAVE / 2; o > 0; o >>= 1) {
        mr = max(mr, __shfl_xor(mr, o, WAVE));
        mi = max(mi, __shfl_xor(mi, o, WAVE));
    }
    if (lane == 0) {
        atomicMax(&cnt->max_row_len, mr);
        atomicMax(&cnt->max_inc, mi);
    }
}
#undef LANE_AT

// One workgroup per vertex with more than LANE_MAX triangles.  Straight
// O(d^2) rank sorts in global memory: such vertices are rare.  `scratch` has
// the same layout as `stage` (2 d + 1 slots at 2 inc_ptr[v] + v).
__global__ __launch_bounds__(256) void k_rows_wide(const int32_t *__restrict__ inc_ptr,
                                                   int32_t *__restrict__ inc,
                                                   const int32_t *__restrict__ me,
                                                   int32_t *__restrict__ rowlen,
                                                   int32_t *__restrict__ stage,
                                                   int32_t *__restrict__ scratch,
                                                   uint32_t *__restrict__ inc_pos,
                                                   const int32_t *__restrict__ wide_list,
                                                   PatternCounters *cnt) {
    __shared__ int32_t s_len;
    const int nwide = cnt->wide_count;
    for (int wv = blockIdx.x; wv < nwide; wv += gridDim.x) {
        const int32_t v = wide_list[wv];
        const int32_t is = inc_ptr[v];
        const int32_t d = inc_ptr[v + 1] - is;
        const int64_t base = 2 * (int64_t)is + v;
        int32_t *cand = scratch + base;   // 2d + 1 slots
        int32_t *cols = stage + base;     // 2d + 1 slots
        // 1. sort the triangle ids (distinct): rank sort through `cols`
        for (int t = threadIdx.x; t < d; t += blockDim.x) {
            const int32_t x = inc[is + t];
            int32_t r = 0;
            for (int s = 0; s < d; ++s) r += inc[is + s] < x;
            cols[r] = x;
        }
        __syncthreads();
        for (int t = threadIdx.x; t < d; t += blockDim.x) inc[is + t] = cols[t];
        __syncthreads();
        // 2. candidates: v, then the two other vertices of each triangle
        for (int t = threadIdx.x; t < d; t += blockDim.x) {
            const int32_t x = inc[is + t];
            const int64_t k = x / 3;
            const int a = x - 3 * static_cast<int32_t>(k);
            cand[1 + 2 * t] = me[3 * k + (a == 2 ? 0 : a + 1)];
            cand[2 + 2 * t] = me[3 * k + (a == 0 ? 2 : a - 1)];
        }
        if (threadIdx.x == 0) cand[0] = v;
        __syncthreads();
        // 3. stable rank sort of the 2d+1 candidates into `cols`
        const int n = 2 * d + 1;
        for (int t = threadIdx.x; t < n; t += blockDim.x) {
            const int32_t x = cand[t];
            int32_t r = 0;
            for (int s = 0; s < n; ++s) r += (cand[s] < x) || (cand[s] == x && s < t);
            cols[r] = x;
        }
        __syncthreads();
        // 4. unique (serial: rare rows)
        if (threadIdx.x == 0) {
            int32_t m = 0;
            for (int t = 0; t < n; ++t)
                if (m == 0 || cols[t] != cols[m - 1]) cols[m++] = cols[t];
            s_len = m;
            rowlen[v] = m;
            atomicMax(&cnt->max_row_len, m);
            if (m > 65535) atomicOr(&cnt->err, ERR_ROWLEN);
        }
        __syncthreads();
        const int32_t m = s_len;
        // 5. row-relative positions
        for (int t = threadIdx.x; t < d; t += blockDim.x) {
            const int32_t p1 = lower_bound(cols, m, cand[1 + 2 * t]);
            const int32_t p2 = lower_bound(cols, m, cand[2 + 2 * t]);
            inc_pos[is + t] = static_cast<uint32_t>(p1 & 0xffff) | (static_cast<uint32_t>(p2) << 16);
        }
        __syncthreads();
    }
}

__global__ __launch_bounds__(256) void k_copy_cols(int32_t nq, const int32_t *__restrict__ row_ptr,
                                                   const int32_t *__restrict__ inc_ptr,
                                                   const int32_t *__restrict__ stage,
                                                   int32_t *__restrict__ col_idx) {
    const int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (v >= nq) return;
    const int32_t rs = row_ptr[v], L = row_ptr[v + 1] - rs;
    const int64_t base = 2 * (int64_t)inc_ptr[v] + v;
    for (int u = 0; u < L; ++u) col_idx[(int64_t)rs + u] = stage[base + u];
}

__global__ __launch_bounds__(256) void k_slot(int32_t nme, const int32_t *__restrict__ me,
                                              const int32_t *__restrict__ row_ptr,
                                              const int32_t *__restrict__ col_idx,
                                              int32_t *__restrict__ slot) {
    const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (k >= nme) return;
    const int32_t v[3] = {me[3 * k], me[3 * k + 1], me[3 * k + 2]};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const int32_t rs = row_ptr[v[a]], L = row_ptr[v[a] + 1] - rs;
#pragma unroll
        for (int b = 0; b < 3; ++b)
            slot[(int64_t)(3 * b + a) * nme + k] = rs + lower_bound(col_idx + rs, L, v[b]);
    }
}

__global__ __launch_bounds__(256) void k_transpose(int32_t nq, const int32_t *__restrict__ row_ptr,
                                                   const int32_t *__restrict__ col_idx,
                                                   int32_t *__restrict__ tpos) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= nq) return;
    for (int32_t p = row_ptr[i]; p < row_ptr[i + 1]; ++p) {
        const int32_t j = col_idx[p];
        const int32_t rs = row_ptr[j], L = row_ptr[j + 1] - rs;
        const int32_t t = lower_bound(col_idx + rs, L, static_cast<int32_t>(i));
        tpos[p] = (t < L && col_idx[rs + t] == i) ? rs + t : -1;
    }
}

__global__ __launch_bounds__(256) void k_elas_pattern(int32_t nq, const int32_t *__restrict__ row_ptr,
                                                      const int32_t *__restrict__ col_idx,
                                                      int32_t *__restrict__ row_ptr_e,
                                                      int32_t *__restrict__ col_idx_e) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i > nq) return;
    const int32_t rs = row_ptr[i];
    if (i == nq) {
        row_ptr_e[2 * i] = 4 * rs;
        return;
    }
    const int32_t L = row_ptr[i + 1] - rs;
    row_ptr_e[2 * i] = 4 * rs;
    row_ptr_e[2 * i + 1] = 4 * rs + 2 * L;
    for (int32_t p = 0; p < L; ++p) {
        const int32_t j = col_idx[rs + p];
        const int64_t e = 4 * (int64_t)rs + 2 * p;
        col_idx_e[e] = 2 * j;
        col_idx_e[e + 1] = 2 * j + 1;
        col_idx_e[e + 2 * L] = 2 * j;
        col_idx_e[e + 2 * L + 1] = 2 * j + 1;
    }
}

// ---------------------------------------------------------------- workspace layout

namespace {
struct PatternWork {
    PatternCounters *cnt;
    int32_t *deg, *rowlen, *wide;
    long long *part;
    int32_t *stage, *scratch;
    size_t bytes;
};

inline size_t align_up(size_t x) { return (x + 255) & ~size_t(255); }

PatternWork carve(int32_t nq, int32_t nme, char *base) {
    PatternWork w{};
    size_t off = 0;
    auto take = [&](size_t bytes) {
        char *p = base ? base + off : nullptr;
        off += align_up(bytes);
        return p;
    };
    const size_t stage_n = 6 * (size_t)nme + (size_t)nq + 1;
    w.cnt = reinterpret_cast<PatternCounters *>(take(sizeof(PatternCounters)));
    w.deg = reinterpret_cast<int32_t *>(take(sizeof(int32_t) * (size_t)nq));
    w.rowlen = reinterpret_cast<int32_t *>(take(sizeof(int32_t) * (size_t)nq));
    w.wide = reinterpret_cast<int32_t *>(take(sizeof(int32_t) * (size_t)nq));
    w.part = reinterpret_cast<long long *>(take(sizeof(long long) * (size_t)scan_partials(nq)));
    w.stage = reinterpret_cast<int32_t *>(take(sizeof(int32_t) * stage_n));
    w.scratch = reinterpret_cast<int32_t *>(take(sizeof(int32_t) * stage_n));
    w.bytes = off;
    return w;
}
}  // namespace

}  // namespace fem

using namespace fem;

extern "C" int64_t fem_nnz_bound(int32_t nq, int32_t nme) {
    return (int64_t)(nq > 0 ? nq : 0) + 6 * (int64_t)(nme > 0 ? nme : 0);
}

extern "C" int fem_pattern_workspace(int32_t nq, int32_t nme, size_t *bytes) {
    clear_error();
    FEM_REQUIRE(bytes != nullptr, FEM_EINVAL, "fem_pattern_workspace: bytes is NULL");
    FEM_REQUIRE(nq >= 1 && nme >= 0, FEM_EINVAL, "fem_pattern_workspace: need nq >= 1, nme >= 0");
    *bytes = carve(nq, nme, nullptr).bytes;
    return FEM_OK;
}

extern "C" int fem_pattern(int32_t nq, int32_t nme, const int32_t *me, int32_t *row_ptr,
                           int32_t *col_idx, int64_t col_cap, int32_t *inc_ptr, int32_t *inc,
                           uint32_t *inc_pos, int32_t *slot, void *work, size_t work_bytes,
                           int64_t *nnz_out, void *stream) {
    clear_error();
    FEM_REQUIRE(nq >= 1, FEM_EINVAL, "fem_pattern: nq must be >= 1 (got %d)", nq);
    FEM_REQUIRE(nme >= 0, FEM_EINVAL, "fem_pattern: nme must be >= 0 (got %d)", nme);
    FEM_REQUIRE(3 * (int64_t)nme <= INT32_MAX && fem_nnz_bound(nq, nme) <= INT32_MAX,
                FEM_EOVERFLOW, "fem_pattern: nq + 6 nme = %lld exceeds int32",
                (long long)fem_nnz_bound(nq, nme));
    FEM_REQUIRE(row_ptr && inc_ptr && nnz_out && work, FEM_EINVAL,
                "fem_pattern: NULL row_ptr, inc_ptr, work or nnz_out");
    FEM_REQUIRE(nme == 0 || (me && inc && inc_pos), FEM_EINVAL,
                "fem_pattern: NULL me, inc or inc_pos");
    FEM_REQUIRE(col_cap >= 0 && (col_cap == 0 || col_idx), FEM_EINVAL,
                "fem_pattern: NULL col_idx or negative col_cap");
    const PatternWork W = carve(nq, nme, static_cast<char *>(work));
    FEM_REQUIRE(work_bytes >= W.bytes, FEM_ENOSPC,
                "fem_pattern: workspace of %zu bytes, need %zu", work_bytes, W.bytes);
    hipStream_t s = as_stream(stream);

    int st;
    if ((st = fill_i32(reinterpret_cast<int32_t *>(W.cnt), sizeof(PatternCounters) / 4, 0, s))) return st;
    if ((st = fill_i32(W.deg, nq, 0, s))) return st;
    if (nme > 0) {
        hipLaunchKernelGGL(k_count, dim3(grid_for(nme, 256)), dim3(256), 0, s, nme, me, nq, W.deg,
                           W.cnt);
        FEM_LAUNCH_CHECK();
    }
    if ((st = exclusive_scan_i32(W.deg, inc_ptr, nq, W.part, &W.cnt->total[0], &W.cnt->err, s)))
        return st;
    if (nme > 0) {
        hipLaunchKernelGGL(k_fill, dim3(grid_for(nme, 256)), dim3(256), 0, s, nme, me, nq, inc_ptr,
                           W.deg, inc);
        FEM_LAUNCH_CHECK();
    }
    hipLaunchKernelGGL(k_rows, dim3(grid_for(nq, WAVE)), dim3(WAVE), 0, s, nq, inc_ptr, inc, me,
                       W.rowlen, W.stage, inc_pos, W.wide, W.cnt);
    FEM_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_rows_wide, dim3(256), dim3(256), 0, s, inc_ptr, inc, me, W.rowlen, W.stage,
                       W.scratch, inc_pos, W.wide, W.cnt);
    FEM_LAUNCH_CHECK();
    if ((st = exclusive_scan_i32(W.rowlen, row_ptr, nq, W.part, &W.cnt->total[1], &W.cnt->err, s)))
        return st;

    PatternCounters h{};
    FEM_HIP_CHECK(hipMemcpyAsync(&h, W.cnt, sizeof(h), hipMemcpyDeviceToHost, s));
    FEM_HIP_CHECK(hipStreamSynchronize(s));
    FEM_REQUIRE(!(h.err & ERR_RANGE), FEM_ERANGE, "fem_pattern: a vertex index of me is outside [0, %d)", nq);
    FEM_REQUIRE(!(h.err & ERR_DEGEN), FEM_EDEGEN, "fem_pattern: a triangle repeats a vertex");
    FEM_REQUIRE(!(h.err & ERR_OVERFLOW), FEM_EOVERFLOW, "fem_pattern: count overflow");
    FEM_REQUIRE(!(h.err & ERR_ROWLEN) && h.max_row_len <= 65535, FEM_EUNSUPPORTED,
                "fem_pattern: a row has %d entries (limit 65535)", h.max_row_len);
    const int64_t nnz = h.total[1];
    FEM_REQUIRE(nnz <= col_cap, FEM_ENOSPC, "fem_pattern: nnz = %lld exceeds col_cap = %lld",
                (long long)nnz, (long long)col_cap);
    hipLaunchKernelGGL(k_copy_cols, dim3(grid_for(nq, 256)), dim3(256), 0, s, nq, row_ptr, inc_ptr,
                       W.stage, col_idx);
    FEM_LAUNCH_CHECK();
    if (slot && nme > 0) {
        hipLaunchKernelGGL(k_slot, dim3(grid_for(nme, 256)), dim3(256), 0, s, nme, me, row_ptr,
                           col_idx, slot);
        FEM_LAUNCH_CHECK();
    }
    *nnz_out = nnz;
    return FEM_OK;
}

extern "C" int fem_transpose_map(int32_t nq, int64_t nnz, const int32_t *row_ptr,
                                 const int32_t *col_idx, int32_t *tpos, void *stream) {
    clear_error();
    FEM_REQUIRE(nq >= 1 && nnz >= 0 && nnz <= INT32_MAX, FEM_EINVAL, "fem_transpose_map: bad sizes");
    FEM_REQUIRE(row_ptr && (nnz == 0 || (col_idx && tpos)), FEM_EINVAL, "fem_transpose_map: NULL array");
    hipLaunchKernelGGL(k_transpose, dim3(grid_for(nq, 256)), dim3(256), 0, as_stream(stream), nq,
                       row_ptr, col_idx, tpos);
    FEM_LAUNCH_CHECK();
    return FEM_OK;
}

extern "C" int fem_elas_pattern(int32_t nq, int64_t nnz, const int32_t *row_ptr,
                                const int32_t *col_idx, int32_t *row_ptr_e, int32_t *col_idx_e,
                                void *stream) {
    clear_error();
    FEM_REQUIRE(nq >= 1 && nnz >= 0, FEM_EINVAL, "fem_elas_pattern: bad sizes");
    FEM_REQUIRE(2 * (int64_t)nq <= INT32_MAX && 4 * nnz <= INT32_MAX, FEM_EOVERFLOW,
                "fem_elas_pattern: 4 nnz = %lld exceeds int32", (long long)(4 * nnz));
    FEM_REQUIRE(row_ptr && row_ptr_e && (nnz == 0 || (col_idx && col_idx_e)), FEM_EINVAL,
                "fem_elas_pattern: NULL array");
    hipLaunchKernelGGL(k_elas_pattern, dim3(grid_for((int64_t)nq + 1, 256)), dim3(256), 0,
                       as_stream(stream), nq, row_ptr, col_idx, row_ptr_e, col_idx_e);
    FEM_LAUNCH_CHECK();
    return FEM_OK;
}
