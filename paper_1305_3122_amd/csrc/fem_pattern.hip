// fem_pattern.hip -- symbolic phase: CSR pattern, triangle lists per vertex,
// row-relative positions and the optional slot map.
//
// Replaces the global index arrays Ig, Jg of the vectorised assembly
// (Section 6, the remark that Ig and Jg need no loop) and the sort/compress
// that sparse(Ig, Jg, Kg) performs.  Instead of sorting 9 nme triplets, the
// 3 nme (vertex, triangle) incidences are grouped by vertex, and every vertex
// sorts/uniques its own short neighbour list (a P1 row holds the vertex and
// its neighbours).
//
// Grouping by vertex (the transpose of me) without global atomics: a
// two-level counting sort over buckets of consecutive vertex ids.
//   1 bucket count    about 256 workgroups of 512 threads, each over a
//                     contiguous range of triangles: mesh checks and an LDS
//                     histogram of the buckets
//   2 scan            bucket-major offsets of every (bucket, workgroup) run
//   3 bucket scatter  the same workgroups write each incidence (3k + a and
//                     the other two vertices) into its (bucket, workgroup) run
// Fine path (default while nq <= 512 * HIST_MAX, about 18.9M vertices):
// buckets of 512 vertices.
//   4 bucket rows     one workgroup per bucket, everything in LDS: counting
//                     sort by vertex -> inc_ptr; per vertex the triangles by
//                     id and the distinct neighbours (sorting networks in
//                     registers up to 8 triangles, LDS up to 64) -> inc,
//                     inc_pos; the bucket's rows staged in its own region
//   5 scan            of the bucket totals
//   6 bucket copy     staged rows -> col_idx, and row_ptr
// Coarse path (a bucket above 4096 incidences or a vertex above 64
// triangles, or nq above 18.9M): buckets of 4096 vertices sorted by
// k_bkt_sort, then one lane per vertex (k_rows), a lane with its list in LDS
// (k_rows_mid) or a workgroup per vertex (k_rows_wide), a scan of the row
// lengths and k_copy_cols.  Beyond 4096 * HIST_MAX (about 151M) vertices the
// grouping is a global-atomic count and fill (k_count, k_fill) instead.
//   slot    one lane per triangle: binary search of its 9 entries
#include <type_traits>

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
                                              int32_t *__restrict__ inc, int2 *__restrict__ nbr) {
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
        nbr[(int64_t)inc_ptr[v[a]] + pos] = make_int2(v[(a + 1) % 3], v[(a + 2) % 3]);
    }
}

// Maximum into a counter shared by every wave: read first, so that the
// atomic (serialised on one address) is issued only while the value grows.
__device__ inline void max_into(int *dst, int v) {
    if (v > __hip_atomic_load(dst, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) atomicMax(dst, v);
}

// ---------------------------------------------------------------- bucket sort
//
// Buckets are ranges of 2^bs consecutive vertex ids.  A first pass
// partitions the incidences by bucket (k_bkt_count, k_bkt_colscan and a scan
// of the bucket totals, k_bkt_scatter: each workgroup of triangles writes one
// contiguous run per bucket).  Then
// either
//   fine buckets (512 vertices): k_bkt_rows does everything for a bucket in
//     LDS -- counting sort by vertex, per-vertex rows -- and stages the
//     bucket's rows; a scan of the bucket totals then gives each bucket's
//     offset in col_idx, and k_bkt_copy writes row_ptr and col_idx;
//   coarse buckets (4096 vertices, very large meshes or a bucket too large for
//     LDS): k_bkt_sort writes the triangle lists, then the per-vertex kernels.

constexpr int BKT_THREADS = 512;
constexpr int FINE_SHIFT = 9;                 // 512 vertices per fine bucket
constexpr int FINE_V = 1 << FINE_SHIFT;
constexpr int FINE_CAP = 4096;                // incidences a fine bucket may hold in LDS
constexpr int COARSE_SHIFT = 12;              // 4096 vertices per coarse bucket
constexpr int COARSE_V = 1 << COARSE_SHIFT;
constexpr int FINE_DMAX = 64;                // triangles per vertex on the fine path
constexpr int HIST_MAX = 36864;               // buckets an LDS histogram holds (144 KiB)
constexpr int NBLK_TARGET = 256;              // triangle workgroups of the partition pass

// device-side error bits of the fine path
enum : int { ERR_BUCKET = 16, ERR_NOSPC = 32 };

// Bucket records.  Wide (16 B): (v, 3k + a, next, previous).  Packed (12 B,
// fine buckets of meshes with nq <= 2^23 vertices): (3k + a, next | (v mod
// FINE_V) << 23, previous).  rec_* give the vertex relative to its bucket,
// the key and the two neighbours, whichever the layout; a vertex of -1 marks
// an empty slot.
constexpr int PACK_SHIFT = 23;
constexpr int32_t PACK_MASK = (1 << PACK_SHIFT) - 1;

struct Rec {
    int32_t lv, key, n1, n2;
};

template <bool PK>
__device__ __forceinline__ Rec load_rec(const int32_t *__restrict__ ent, int64_t e, int32_t v0) {
    if constexpr (PK) {
        const int32_t *p = ent + 3 * e;
        const int32_t k = p[0], a = p[1], c = p[2];
        return Rec{static_cast<int32_t>(static_cast<uint32_t>(a) >> PACK_SHIFT), k, a & PACK_MASK, c};
    } else {
        const int4 r = reinterpret_cast<const int4 *>(ent)[e];
        return Rec{r.x - v0, r.y, r.z, r.w};
    }
}

template <bool PK>
__device__ __forceinline__ void store_rec(int32_t *__restrict__ ent, int64_t e, int32_t v, int32_t key,
                                          int32_t n1, int32_t n2) {
    if constexpr (PK) {
        int32_t *p = ent + 3 * e;
        p[0] = key;
        p[1] = n1 | ((v & (FINE_V - 1)) << PACK_SHIFT);
        p[2] = n2;
    } else {
        reinterpret_cast<int4 *>(ent)[e] = make_int4(v, key, n1, n2);
    }
}

__device__ inline bool tri_ok(int32_t a, int32_t b, int32_t c, int32_t nq) {
    return (uint32_t)a < (uint32_t)nq && (uint32_t)b < (uint32_t)nq && (uint32_t)c < (uint32_t)nq &&
           a != b && b != c && a != c;
}

// counts[blk * nbkt + b] = incidences of workgroup blk (tpb triangles)
// falling in bucket b (each workgroup writes one contiguous row); mesh checks.
__global__ __launch_bounds__(BKT_THREADS) void k_bkt_count(int32_t nme, const int32_t *__restrict__ me,
                                                          int32_t nq, int bs, int32_t nbkt, int32_t tpb,
                                                          int32_t *__restrict__ counts,
                                                          PatternCounters *cnt) {
    extern __shared__ int32_t s_hist[];
    for (int b = threadIdx.x; b < nbkt; b += BKT_THREADS) s_hist[b] = 0;
    __syncthreads();
    int bad = 0;
    const int64_t k0 = (int64_t)blockIdx.x * tpb;
    const int64_t k1 = (k0 + tpb < nme) ? k0 + tpb : nme;
    constexpr int H = 16;   // triangles with independent loads in flight per thread
    for (int64_t kb = k0 + threadIdx.x; kb < k1; kb += H * BKT_THREADS) {
        int32_t v[H][3];
#pragma unroll
        for (int j = 0; j < H; ++j) {
            const int64_t k = kb + j * BKT_THREADS;
            v[j][0] = v[j][1] = v[j][2] = 0;
            if (k < k1) {
                v[j][0] = me[3 * k];
                v[j][1] = me[3 * k + 1];
                v[j][2] = me[3 * k + 2];
            }
        }
#pragma unroll
        for (int j = 0; j < H; ++j) {
            if (kb + j * BKT_THREADS >= k1) continue;
            const int32_t a = v[j][0], b = v[j][1], c = v[j][2];
            if ((uint32_t)a >= (uint32_t)nq || (uint32_t)b >= (uint32_t)nq ||
                (uint32_t)c >= (uint32_t)nq) {
                bad |= ERR_RANGE;
                continue;
            }
            if (a == b || b == c || a == c) {
                bad |= ERR_DEGEN;
                continue;
            }
            atomicAdd(&s_hist[a >> bs], 1);
            atomicAdd(&s_hist[b >> bs], 1);
            atomicAdd(&s_hist[c >> bs], 1);
        }
    }
    if (bad) atomicOr(&cnt->err, bad);
    __syncthreads();
    for (int b = threadIdx.x; b < nbkt; b += BKT_THREADS)
        counts[(int64_t)blockIdx.x * nbkt + b] = s_hist[b];
}

// In place over counts[blk][b]: each entry becomes the number of bucket b's
// incidences in workgroups before blk, and bsum[b] the bucket's total.  One
// lane per bucket, the COLSCAN_WAVES waves of a workgroup over equal parts of
// the workgroup range (their partial sums meet in LDS); every read and write
// covers 64 consecutive buckets.
__global__ __launch_bounds__(COLSCAN_WAVES * WAVE) void k_bkt_colscan(int32_t nbkt, int32_t nblk,
                                                                     int32_t *__restrict__ counts,
                                                                     int32_t *__restrict__ bsum) {
    constexpr int NW = COLSCAN_WAVES;
    __shared__ int32_t s_part[NW][WAVE];
    const int lane = threadIdx.x & (WAVE - 1), w = threadIdx.x / WAVE;
    const int32_t b = blockIdx.x * WAVE + lane;
    const bool ok = b < nbkt;
    const int32_t Q = (nblk + NW - 1) / NW;
    const int32_t k0 = w * Q, k1 = (k0 + Q < nblk) ? k0 + Q : nblk;
    constexpr int H = 8;   // loads in flight per lane
    int32_t sum = 0;
    for (int32_t k = k0; k < k1; k += H) {
        int32_t c[H];
#pragma unroll
        for (int j = 0; j < H; ++j) c[j] = (ok && k + j < k1) ? counts[(int64_t)(k + j) * nbkt + b] : 0;
#pragma unroll
        for (int j = 0; j < H; ++j) sum += c[j];
    }
    s_part[w][lane] = sum;
    __syncthreads();
    int32_t run = 0;
    for (int u = 0; u < w; ++u) run += s_part[u][lane];
    for (int32_t k = k0; k < k1; k += H) {
        int32_t c[H];
#pragma unroll
        for (int j = 0; j < H; ++j) c[j] = (ok && k + j < k1) ? counts[(int64_t)(k + j) * nbkt + b] : 0;
#pragma unroll
        for (int j = 0; j < H; ++j) {
            if (ok && k + j < k1) counts[(int64_t)(k + j) * nbkt + b] = run;
            run += c[j];
        }
    }
    if (ok && w == NW - 1) bsum[b] = run;
}

// Same triangles per workgroup as k_bkt_count: each incidence goes to the run
// of its (bucket, workgroup) pair as one record.
template <bool PK>
__global__ __launch_bounds__(BKT_THREADS) void k_bkt_scatter(int32_t nme, const int32_t *__restrict__ me,
                                                            int32_t nq, int bs, int32_t nbkt,
                                                            int32_t tpb,
                                                            const int32_t *__restrict__ offs,
                                                            const int32_t *__restrict__ bstart,
                                                            int32_t *__restrict__ ent) {
    extern __shared__ int32_t s_cur[];
    // the run of (b, this workgroup) starts at the bucket's start plus the
    // incidences of the workgroups before it (one contiguous row of offs)
    const int32_t *row = offs + (int64_t)blockIdx.x * nbkt;
    for (int b = threadIdx.x; b < nbkt; b += BKT_THREADS) s_cur[b] = bstart[b] + row[b];
    __syncthreads();
    const int64_t k0 = (int64_t)blockIdx.x * tpb;
    const int64_t k1 = (k0 + tpb < nme) ? k0 + tpb : nme;
    constexpr int H = 16;   // triangles with independent loads in flight per thread
    for (int64_t kb = k0 + threadIdx.x; kb < k1; kb += H * BKT_THREADS) {
        int32_t v[H][3];
#pragma unroll
        for (int j = 0; j < H; ++j) {
            const int64_t k = kb + j * BKT_THREADS;
            v[j][0] = v[j][1] = v[j][2] = -1;
            if (k < k1) {
                v[j][0] = me[3 * k];
                v[j][1] = me[3 * k + 1];
                v[j][2] = me[3 * k + 2];
            }
        }
#pragma unroll
        for (int j = 0; j < H; ++j) {
            const int64_t k = kb + j * BKT_THREADS;
            if (k >= k1 || !tri_ok(v[j][0], v[j][1], v[j][2], nq)) continue;
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const int32_t pos = atomicAdd(&s_cur[v[j][a] >> bs], 1);
                store_rec<PK>(ent, pos, v[j][a], static_cast<int32_t>(3 * k + a), v[j][(a + 1) % 3],
                              v[j][(a + 2) % 3]);
            }
        }
    }
}

// Coarse path: one workgroup per bucket of COARSE_V vertices: counting sort of
// its incidences by vertex in LDS.  Writes inc_ptr for the bucket's vertices
// and the (unordered within a vertex) triangle lists and neighbour pairs.
__global__ __launch_bounds__(BKT_THREADS) void k_bkt_sort(int32_t nq, const int32_t *__restrict__ bstart,
                                                         const int32_t *__restrict__ ent_w,
                                                         int32_t *__restrict__ inc_ptr,
                                                         int32_t *__restrict__ inc,
                                                         int2 *__restrict__ nbr) {
    __shared__ int32_t s_cnt[COARSE_V];
    __shared__ int32_t s_wsum[BKT_THREADS / WAVE];
    const int4 *ent = reinterpret_cast<const int4 *>(ent_w);
    const int32_t b = blockIdx.x;
    const int64_t e0 = bstart[b], e1 = bstart[b + 1];
    const int32_t v0 = b << COARSE_SHIFT;
    for (int i = threadIdx.x; i < COARSE_V; i += BKT_THREADS) s_cnt[i] = 0;
    __syncthreads();
    constexpr int B8 = 8;   // batches of independent loads per thread
    for (int64_t e = e0 + threadIdx.x; e < e1; e += B8 * BKT_THREADS) {
        int32_t lv[B8];
#pragma unroll
        for (int u = 0; u < B8; ++u) {
            const int64_t x = e + u * BKT_THREADS;
            lv[u] = x < e1 ? ent[x].x - v0 : -1;
        }
#pragma unroll
        for (int u = 0; u < B8; ++u)
            if (lv[u] >= 0) atomicAdd(&s_cnt[lv[u]], 1);
    }
    __syncthreads();
    constexpr int PER = COARSE_V / BKT_THREADS;
    int32_t loc[PER];
    int32_t sum = 0;
#pragma unroll
    for (int t = 0; t < PER; ++t) {
        loc[t] = s_cnt[threadIdx.x * PER + t];
        sum += loc[t];
    }
    const int lane = threadIdx.x & (WAVE - 1), wid = threadIdx.x / WAVE;
    int32_t incl = wave_inclusive_scan(sum);
    if (lane == WAVE - 1) s_wsum[wid] = incl;
    __syncthreads();
    int32_t run = incl - sum;
    for (int w = 0; w < wid; ++w) run += s_wsum[w];
#pragma unroll
    for (int t = 0; t < PER; ++t) {
        const int32_t lv = threadIdx.x * PER + t;
        s_cnt[lv] = run;   // becomes the cursor
        if (v0 + lv < nq) inc_ptr[v0 + lv] = static_cast<int32_t>(e0) + run;
        run += loc[t];
    }
    if (b == (int32_t)gridDim.x - 1 && threadIdx.x == 0) inc_ptr[nq] = static_cast<int32_t>(e1);
    __syncthreads();
    for (int64_t e = e0 + threadIdx.x; e < e1; e += B8 * BKT_THREADS) {
        int4 x[B8];
#pragma unroll
        for (int u = 0; u < B8; ++u) {
            const int64_t y = e + u * BKT_THREADS;
            x[u] = y < e1 ? ent[y] : make_int4(-1, 0, 0, 0);
        }
#pragma unroll
        for (int u = 0; u < B8; ++u) {
            if (x[u].x < 0) continue;
            const int64_t pos = e0 + atomicAdd(&s_cnt[x[u].x - v0], 1);
            inc[pos] = x[u].y;
            nbr[pos] = make_int2(x[u].z, x[u].w);
        }
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

// Fan code of a row (layout in fem_internal.h) from its d triangles in
// ascending order and the row length: pos(t) gives triangle t's packed
// positions p1 | p2 << 16 (next and previous vertex in the triangle's own
// order), so triangle t links slot p1 -> p2 and the fan is the chain of these
// links.  The code is nonzero only if every slot is left by at most one
// triangle and entered by at most one, the links form one closed cycle or
// one open path through all d triangles, and every off-diagonal slot is on
// it; otherwise (inconsistent orientation, several fans meeting at the
// vertex, a non-manifold edge, more than FAN_NMAX neighbours) it is 0.  A
// closed fan starts at the first triangle's p1, an open one at its only slot
// that no triangle enters.
template <typename Pos>
__device__ inline uint64_t fan_code(int d, int32_t len, Pos pos) {
    if (!(d >= 1 && d <= FAN_NMAX && len >= 3 && len <= FAN_NMAX + 1)) return 0;
    uint64_t succ = 0, p2t = 0;   // nibble tables: slot -> triangle, triangle -> p2
    uint32_t outm = 0, inm = 0;
    bool ok = true;
    for (int t = 0; t < d && ok; ++t) {
        const uint32_t pp = pos(t);
        const uint32_t p1 = pp & 0xffffu, p2 = pp >> 16;
        ok = p1 < 16 && p2 < 16 && !((outm >> p1) & 1u) && !((inm >> p2) & 1u);
        if (ok) {
            outm |= 1u << p1;
            inm |= 1u << p2;
            succ |= (uint64_t)t << (4 * p1);
            p2t |= (uint64_t)p2 << (4 * t);
        }
    }
    const uint32_t used = outm | inm, starts = outm & ~inm;
    const bool closed = starts == 0;
    ok = ok && __builtin_popcount(used) + 1 == len &&
         (closed ? outm == inm
                 : (__builtin_popcount(starts) == 1 && __builtin_popcount(inm & ~outm) == 1));
    if (!ok) return 0;
    const int s0 = closed ? (int)(pos(0) & 0xffffu) : __builtin_ctz(starts);
    int s = s0, n = 0;
    uint64_t slots = 0;
    for (int j = 0; j < d && ok; ++j) {
        // every step leaves its slot; a closed walk meets s0 again only at the end
        ok = ((outm >> s) & 1u) && !(j > 0 && s == s0);
        if (ok) {
            slots |= (uint64_t)s << (4 * n++);
            s = (int)((p2t >> (4 * ((succ >> (4 * s)) & 15u))) & 15u);
        }
    }
    if (!ok) return 0;
    if (closed) ok = s == s0;
    else slots |= (uint64_t)s << (4 * n++);
    if (!(ok && n + 1 == len && n <= FAN_NMAX)) return 0;
    const int pd = __builtin_ctz(~used);
    return (uint64_t)n | ((uint64_t)(closed ? 1 : 0) << 4) | ((uint64_t)pd << 5) | (slots << 9);
}

// Fan code of every row from the triangle lists (patterns of the coarse
// and atomic paths, or built elsewhere).
__global__ __launch_bounds__(256) void k_fan_plan(int32_t nq, const int32_t *__restrict__ row_ptr,
                                                  const int32_t *__restrict__ inc_ptr,
                                                  const uint32_t *__restrict__ inc_pos,
                                                  uint64_t *__restrict__ fan) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= nq) return;
    const int32_t is = inc_ptr[i], d = inc_ptr[i + 1] - is;
    const int32_t len = row_ptr[i + 1] - row_ptr[i];
    fan[i] = fan_code(d, len, [&](int t) { return inc_pos[is + t]; });
}

// Bitonic sorting networks on register arrays (all indices static after
// unrolling, so the arrays stay in VGPRs).  sort_kv: key + two payloads.
template <int N>
__device__ __forceinline__ void bitonic_sort_kv(int32_t (&k)[N], int32_t (&p)[N], int32_t (&r)[N]) {
#pragma unroll
    for (int size = 2; size <= N; size <<= 1)
#pragma unroll
        for (int stride = size >> 1; stride > 0; stride >>= 1)
#pragma unroll
            for (int i = 0; i < N; ++i) {
                const int l = i ^ stride;
                if (l > i) {
                    const bool up = (i & size) == 0;
                    const bool sw = (k[i] > k[l]) == up;
                    const int32_t k0 = k[i], p0 = p[i], r0 = r[i];
                    k[i] = sw ? k[l] : k0;
                    p[i] = sw ? p[l] : p0;
                    r[i] = sw ? r[l] : r0;
                    k[l] = sw ? k0 : k[l];
                    p[l] = sw ? p0 : p[l];
                    r[l] = sw ? r0 : r[l];
                }
            }
}

template <int N>
__device__ __forceinline__ void bitonic_sort(int32_t (&k)[N]) {
#pragma unroll
    for (int size = 2; size <= N; size <<= 1)
#pragma unroll
        for (int stride = size >> 1; stride > 0; stride >>= 1)
#pragma unroll
            for (int i = 0; i < N; ++i) {
                const int l = i ^ stride;
                if (l > i) {
                    const bool up = (i & size) == 0;
                    const int32_t a = k[i], b = k[l];
                    k[i] = up ? min(a, b) : max(a, b);
                    k[l] = up ? max(a, b) : min(a, b);
                }
            }
}

// Sorting network over unsigned words (ascending).
template <int N, typename T>
__device__ __forceinline__ void bitonic_sort_u(T (&k)[N]) {
#pragma unroll
    for (int size = 2; size <= N; size <<= 1)
#pragma unroll
        for (int stride = size >> 1; stride > 0; stride >>= 1)
#pragma unroll
            for (int i = 0; i < N; ++i) {
                const int l = i ^ stride;
                if (l > i) {
                    const bool up = (i & size) == 0;
                    const T a = k[i], b = k[l];
                    k[i] = up ? (a < b ? a : b) : (a < b ? b : a);
                    k[l] = up ? (a < b ? b : a) : (a < b ? a : b);
                }
            }
}

// Triangles per vertex handled entirely in registers by k_rows.
constexpr int REG_MAX = 8;

// Exclusive scan of one int per thread over a workgroup of BKT_THREADS.
__device__ __noinline__ int32_t block_exclusive_scan_i32(int32_t v, int32_t *s_wsum, int32_t *total) {
    const int lane = threadIdx.x & (WAVE - 1), wid = threadIdx.x / WAVE;
    const int32_t incl = wave_inclusive_scan(v);
    if (lane == WAVE - 1) s_wsum[wid] = incl;
    __syncthreads();
    int32_t off = incl - v, tot = 0;
#pragma unroll
    for (int w = 0; w < BKT_THREADS / WAVE; ++w) {
        if (w < wid) off += s_wsum[w];
        tot += s_wsum[w];
    }
    __syncthreads();
    *total = tot;
    return off;
}

// Fine path: one workgroup (one thread per vertex) per bucket of FINE_V
// vertices, everything in LDS:
//   1 count the bucket's incidences per vertex, scan -> inc_ptr
//   2 counting sort of (3k + a, next, previous) by vertex into LDS
//   3 per vertex: triangles by id, distinct neighbours, row length
//   4 offsets of the rows inside the bucket (rowoff) and the bucket's total
//   5 inc (triangles by id) and inc_pos (their neighbours' places in the row)
//   6 the bucket's rows, one after the other, into its own part of `stage`
//     (at 2 e0 + v0: at most 2 n + FINE_V entries for n incidences)
// k_bkt_copy then moves each bucket's rows to col_idx once the bucket totals
// are scanned.  A bucket with more than FINE_CAP incidences, or a vertex with
// more than FINE_DMAX triangles, sets ERR_BUCKET: the host then rebuilds with
// the coarse path.
template <bool PK>
__global__ __launch_bounds__(BKT_THREADS) void k_bkt_rows(
    int32_t nq, int32_t nbkt, const int32_t *__restrict__ bstart,
    const int32_t *__restrict__ ent, int32_t *__restrict__ inc_ptr,
    int32_t *__restrict__ inc, uint32_t *__restrict__ inc_pos, uint64_t *__restrict__ fan,
    int32_t *__restrict__ rowoff, int32_t *__restrict__ btot, int32_t *__restrict__ stage,
    PatternCounters *cnt) {
    __shared__ int32_t s_cur[FINE_V];
    __shared__ int32_t s_key[FINE_CAP], s_n1[FINE_CAP], s_n2[FINE_CAP];
    __shared__ int32_t s_wsum[BKT_THREADS / WAVE];
    const int tid = threadIdx.x;
    const int32_t b = blockIdx.x;
    const int64_t e0 = bstart[b], e1 = bstart[b + 1];
    const bool fits = e1 - e0 <= FINE_CAP;
    const int32_t v0 = b << FINE_SHIFT;
    const int64_t v = (int64_t)v0 + tid;
    int32_t d = 0, is = 0;
    // ---- 1 count, scan (the bucket's records stay in registers)
    constexpr int EPT = FINE_CAP / BKT_THREADS;
    Rec x[EPT];
#pragma unroll
    for (int u = 0; u < EPT; ++u) {
        const int64_t y = e0 + tid + u * BKT_THREADS;
        x[u] = (fits && y < e1) ? load_rec<PK>(ent, y, v0) : Rec{-1, 0, 0, 0};
    }
    s_cur[tid] = 0;
    __syncthreads();
#pragma unroll
    for (int u = 0; u < EPT; ++u)
        if (x[u].lv >= 0) atomicAdd(&s_cur[x[u].lv], 1);
    __syncthreads();
    d = s_cur[tid];
    int32_t unused;
    is = block_exclusive_scan_i32(d, s_wsum, &unused);
    s_cur[tid] = is;
    if (v < nq) inc_ptr[v] = static_cast<int32_t>(e0) + is;
    if (b == nbkt - 1 && tid == 0) inc_ptr[nq] = static_cast<int32_t>(e1);
    __syncthreads();
    // ---- 2 counting sort into LDS
#pragma unroll
    for (int u = 0; u < EPT; ++u) {
        if (x[u].lv < 0) continue;
        const int32_t p = atomicAdd(&s_cur[x[u].lv], 1);
        s_key[p] = x[u].key;
        s_n1[p] = x[u].n1;
        s_n2[p] = x[u].n2;
    }
    __syncthreads();
    // ---- 3 per vertex: triangles by id, distinct neighbours, row length
    bool bad = !fits;
    int32_t L = 0;
    // register path (d <= REG_MAX): candidate words (neighbour << 4 |
    // origin), origin 2 t or 2 t + 1 for the first or second neighbour of
    // slice entry t; sorted, equal neighbours are adjacent and fm flags the
    // first of each
    using CW = typename std::conditional<PK, uint32_t, uint64_t>::type;
    constexpr CW CW_NONE = ~CW(0);
    CW c[2 * REG_MAX];
    uint32_t fm = 0;
    // LDS path (REG_MAX < d <= FINE_DMAX): candidate u is entry u % 2 of the
    // neighbour pair of triangle u / 2; m0, m1 flag the first occurrences
    uint64_t m0 = 0, m1 = 0;
    auto cand = [&](int u) { return (u & 1) ? s_n2[is + (u >> 1)] : s_n1[is + (u >> 1)]; };
    auto first = [&](int u) { return ((u < 64 ? m0 >> u : m1 >> (u - 64)) & 1) != 0; };
    auto lds_rank = [&](int32_t y) {
        int32_t r = (int32_t)v < y ? 1 : 0;
        for (int u = 0; u < 2 * d; ++u) r += (first(u) && cand(u) < y) ? 1 : 0;
        return r;
    };
    if (!fits || v >= nq) {
        d = 0;
    }
    const bool in_regs = d <= REG_MAX;
    if (in_regs) {
#pragma unroll
        for (int t = 0; t < REG_MAX; ++t) {
            c[2 * t] = c[2 * t + 1] = CW_NONE;
            if (t < d) {
                c[2 * t] = ((CW)s_n1[is + t] << 4) | (CW)(2 * t);
                c[2 * t + 1] = ((CW)s_n2[is + t] << 4) | (CW)(2 * t + 1);
            }
        }
        bitonic_sort_u<2 * REG_MAX>(c);
        // a candidate's distinct index is the running count of first
        // occurrences; its row position adds 1 past v; each origin's
        // position goes back to the slice (first neighbour to s_n1, second
        // to s_n2: both have been read)
        int32_t nd = 0;
#pragma unroll
        for (int k = 0; k < 2 * REG_MAX; ++k) {
            if (c[k] != CW_NONE) {
                const int32_t y = (int32_t)(c[k] >> 4);
                const bool f = k == 0 || y != (int32_t)(c[k - 1] >> 4);
                fm |= f ? 1u << k : 0u;
                nd += f ? 1 : 0;
                const int o = (int)(c[k] & 15u);
                const int32_t pos = nd - 1 + (y > (int32_t)v ? 1 : 0);
                if (o & 1) s_n2[is + (o >> 1)] = pos;
                else s_n1[is + (o >> 1)] = pos;
            }
        }
        L = d > 0 ? nd + 1 : 0;
        // the triangles by id (words key << 3 | slice entry), and their
        // position pairs, back into the vertex's own LDS slice in that order
        // (copied out in step 5)
        uint64_t kt[REG_MAX];
#pragma unroll
        for (int t = 0; t < REG_MAX; ++t)
            kt[t] = t < d ? ((uint64_t)(uint32_t)s_key[is + t] << 3) | (uint64_t)t : ~uint64_t(0);
        bitonic_sort_u<REG_MAX>(kt);
        uint32_t pk[REG_MAX];
#pragma unroll
        for (int j = 0; j < REG_MAX; ++j) {
            pk[j] = 0;
            if (j < d) {
                const int t = (int)(kt[j] & 7u);
                pk[j] = (uint32_t)s_n1[is + t] | ((uint32_t)s_n2[is + t] << 16);
            }
        }
#pragma unroll
        for (int j = 0; j < REG_MAX; ++j)
            if (j < d) {
                s_key[is + j] = (int32_t)(kt[j] >> 3);
                s_n1[is + j] = (int32_t)pk[j];
            }
    } else if (d <= FINE_DMAX) {
        // insertion sort of the vertex's LDS slice by triangle
        for (int t = 1; t < d; ++t) {
            const int32_t y = s_key[is + t], a1 = s_n1[is + t], a2 = s_n2[is + t];
            int j = t;
            while (j > 0 && s_key[is + j - 1] > y) {
                s_key[is + j] = s_key[is + j - 1];
                s_n1[is + j] = s_n1[is + j - 1];
                s_n2[is + j] = s_n2[is + j - 1];
                --j;
            }
            s_key[is + j] = y;
            s_n1[is + j] = a1;
            s_n2[is + j] = a2;
        }
        int32_t nd = 0;
        for (int u = 0; u < 2 * d; ++u) {
            const int32_t y = cand(u);
            bool fu = true;
            for (int w = 0; w < u && fu; ++w) fu = cand(w) != y;
            if (fu) {
                if (u < 64) m0 |= 1ull << u;
                else m1 |= 1ull << (u - 64);
                ++nd;
            }
        }
        L = nd + 1;
    } else {
        bad = true;
    }
    if (bad) atomicOr(&cnt->err, ERR_BUCKET);
    // ---- 4 row offsets inside the bucket
    int32_t Tb;
    const int32_t lro = block_exclusive_scan_i32(L, s_wsum, &Tb);
    if (v < nq) rowoff[v] = lro;
    if (tid == 0) btot[b] = Tb;
    // ---- 5 inc / inc_pos.  The register path has put its sorted triangles
    // and positions into its own LDS slices (s_key, s_n1) in step 3; the LDS
    // path (whose s_n1 / s_n2 are still read in step 6) writes its positions
    // directly and marks its slice afterwards; the whole bucket is then
    // copied out coalesced.
    constexpr uint32_t POS_DIRECT = 0xffffffffu;   // never a position pair here
    const int64_t ib = e0 + is;
    if (!bad && d > 0 && !in_regs) {
        for (int t = 0; t < d; ++t)
            inc_pos[ib + t] = static_cast<uint32_t>(lds_rank(s_n1[is + t])) |
                              (static_cast<uint32_t>(lds_rank(s_n2[is + t])) << 16);
    }
    // ---- 6 the rows, into the bucket's part of stage
    if (L > 0 && !bad) {
        int32_t *out = stage + 2 * e0 + v0 + lro;
        if (in_regs) {
            int32_t below = 0;
            bool vdone = false;
#pragma unroll
            for (int k = 0; k < 2 * REG_MAX; ++k) {
                if ((fm >> k) & 1u) {
                    const int32_t y = (int32_t)(c[k] >> 4);
                    if (!vdone && y > (int32_t)v) {
                        out[below] = (int32_t)v;
                        vdone = true;
                    }
                    out[below + (vdone ? 1 : 0)] = y;
                    ++below;
                }
            }
            if (!vdone) out[below] = (int32_t)v;
        } else {
            for (int u = 0; u < 2 * d; ++u)
                if (first(u)) out[lds_rank(cand(u))] = cand(u);
            out[lds_rank((int32_t)v)] = (int32_t)v;
            for (int t = 0; t < d; ++t) s_n1[is + t] = static_cast<int32_t>(POS_DIRECT);
        }
    }
    __syncthreads();
    if (fits) {
        const int32_t n = static_cast<int32_t>(e1 - e0);
        // streaming stores: the row kernels read inc and inc_pos only for
        // rows without a fan code
        for (int32_t p = tid; p < n; p += BKT_THREADS) {
            __builtin_nontemporal_store(s_key[p], inc + e0 + p);
            const uint32_t pp = static_cast<uint32_t>(s_n1[p]);
            if (pp != POS_DIRECT) __builtin_nontemporal_store(pp, inc_pos + e0 + p);
        }
    }
    // ---- maxima
    int mr = L, mi = d;
#pragma unroll
    for (int o = WAVE / 2; o > 0; o >>= 1) {
        mr = max(mr, __shfl_xor(mr, o, WAVE));
        mi = max(mi, __shfl_xor(mi, o, WAVE));
    }
    if ((tid & (WAVE - 1)) == 0) {
        max_into(&cnt->max_row_len, mr);
        max_into(&cnt->max_inc, mi);
    }
    // ---- the fan code, last, when the sort's registers are free: from the
    // positions in the vertex's LDS slice (register path; the copy-out above
    // only read it) or in inc_pos (LDS path)
    if (fan && v < nq) {
        uint64_t code = 0;
        if (!bad && d > 0) {
            if (in_regs) code = fan_code(d, L, [&](int t) { return static_cast<uint32_t>(s_n1[is + t]); });
            else code = fan_code(d, L, [&](int t) { return inc_pos[ib + t]; });
        }
        fan[v] = code;
    }
}

// Bucket b's rows, staged by k_bkt_rows, to col_idx at bptr[b] (the scan of
// the bucket totals), and row_ptr of its vertices.
__global__ __launch_bounds__(256) void k_bkt_copy(int32_t nq, int32_t nbkt,
                                                 const int32_t *__restrict__ bstart,
                                                 const int32_t *__restrict__ bptr,
                                                 const int32_t *__restrict__ rowoff,
                                                 const int32_t *__restrict__ stage,
                                                 int32_t *__restrict__ row_ptr,
                                                 int32_t *__restrict__ col_idx, int64_t col_cap,
                                                 PatternCounters *cnt) {
    const int32_t b = blockIdx.x;
    const int64_t e0 = bstart[b];
    const int32_t v0 = b << FINE_SHIFT;
    const int32_t P = bptr[b], T = bptr[b + 1] - P;
    for (int t = threadIdx.x; t < FINE_V; t += 256)
        if (v0 + t < nq) row_ptr[v0 + t] = P + rowoff[v0 + t];
    if (b == nbkt - 1 && threadIdx.x == 0) row_ptr[nq] = bptr[nbkt];
    if (P + (int64_t)T > col_cap) {
        if (threadIdx.x == 0) atomicOr(&cnt->err, ERR_NOSPC);
        return;
    }
    const int32_t *src = stage + 2 * e0 + v0;
    constexpr int H = 8;   // loads in flight per thread
    for (int i0 = threadIdx.x; i0 < T; i0 += H * 256) {
        int32_t x[H];
#pragma unroll
        for (int j = 0; j < H; ++j) {
            const int i = i0 + j * 256;
            x[j] = i < T ? src[i] : 0;
        }
#pragma unroll
        for (int j = 0; j < H; ++j) {
            const int i = i0 + j * 256;
            if (i < T) col_idx[P + i] = x[j];
        }
    }
}

// Per-lane LDS arrays are stored [slot][lane] so that the 64 lanes of a wave
// touch 64 consecutive words (no bank conflicts).
#define LANE_AT(arr, t) arr[(t) * WAVE + lane]

__global__ __launch_bounds__(WAVE) void k_rows(int32_t nq, const int32_t *__restrict__ inc_ptr,
                                               int32_t *__restrict__ inc,
                                               const int2 *__restrict__ nbr,
                                               int32_t *__restrict__ rowlen,
                                               int32_t *__restrict__ stage,
                                               uint32_t *__restrict__ inc_pos,
                                               int32_t *__restrict__ mid_list,
                                               int32_t *__restrict__ wide_list,
                                               PatternCounters *cnt) {
    const int lane = threadIdx.x;
    const int64_t v = blockIdx.x * (int64_t)WAVE + lane;
    const bool in = v < nq;
    const int32_t is = in ? inc_ptr[v] : 0;
    const int32_t d0 = in ? inc_ptr[v + 1] - is : 0;
    // more than REG_MAX triangles: the LDS path (<= LANE_MAX) or the
    // workgroup-per-vertex path
    if (d0 > LANE_MAX) wide_list[atomicAdd(&cnt->wide_count, 1)] = static_cast<int32_t>(v);
    else if (d0 > REG_MAX) mid_list[atomicAdd(&cnt->mid_count, 1)] = static_cast<int32_t>(v);
    const int32_t d = d0 > REG_MAX ? 0 : d0;
    int n = 0;
    if (d <= REG_MAX) {
        // ---- common case, all in registers: sort the (at most 8) triangles
        // by id with their neighbour pairs, sort the 2d neighbours, and rank
        // columns by counting distinct smaller values
        int32_t key[REG_MAX], n1[REG_MAX], n2[REG_MAX];
#pragma unroll
        for (int t = 0; t < REG_MAX; ++t) {
            key[t] = n1[t] = n2[t] = INT32_MAX;
            if (t < d) {
                key[t] = inc[is + t];
                const int2 nb = nbr[is + t];
                n1[t] = nb.x;
                n2[t] = nb.y;
            }
        }
        bitonic_sort_kv<REG_MAX>(key, n1, n2);
        int32_t c[2 * REG_MAX];
#pragma unroll
        for (int t = 0; t < REG_MAX; ++t) {
            if (t < d) inc[is + t] = key[t];
            c[2 * t] = n1[t];
            c[2 * t + 1] = n2[t];
        }
        bitonic_sort<2 * REG_MAX>(c);
        // first occurrence flags; v itself is never its own neighbour
        bool f[2 * REG_MAX];
#pragma unroll
        for (int k = 0; k < 2 * REG_MAX; ++k)
            f[k] = c[k] != INT32_MAX && (k == 0 || c[k] != c[k - 1]);
        auto rank = [&](int32_t x) {
            int32_t r = (int32_t)v < x ? 1 : 0;
#pragma unroll
            for (int k = 0; k < 2 * REG_MAX; ++k) r += (f[k] && c[k] < x) ? 1 : 0;
            return r;
        };
#pragma unroll
        for (int t = 0; t < REG_MAX; ++t)
            if (t < d)
                inc_pos[is + t] = static_cast<uint32_t>(rank(n1[t])) |
                                  (static_cast<uint32_t>(rank(n2[t])) << 16);
        if (d > 0) {
            const int64_t base = 2 * (int64_t)is + v;
            int32_t below = 0;   // distinct neighbours written so far
            bool vdone = false;
#pragma unroll
            for (int k = 0; k < 2 * REG_MAX; ++k) {
                if (f[k]) {
                    if (!vdone && c[k] > (int32_t)v) {
                        stage[base + below] = (int32_t)v;
                        vdone = true;
                    }
                    stage[base + below + (vdone ? 1 : 0)] = c[k];
                    ++below;
                }
            }
            if (!vdone) stage[base + below] = (int32_t)v;
            n = below + 1;
        }
    }
    if (in && d0 <= REG_MAX) rowlen[v] = n;
    // one atomic per wave for the maxima
    int mr = n, mi = d0;
#pragma unroll
    for (int o = WAVE / 2; o > 0; o >>= 1) {
        mr = max(mr, __shfl_xor(mr, o, WAVE));
        mi = max(mi, __shfl_xor(mi, o, WAVE));
    }
    if (lane == 0) {
        max_into(&cnt->max_row_len, mr);
        max_into(&cnt->max_inc, mi);
    }
}

// Vertices with REG_MAX < d <= LANE_MAX triangles: one lane per vertex with
// per-lane LDS lists (insertion sorts), looping over the list built by k_rows.
__global__ __launch_bounds__(WAVE) void k_rows_mid(const int32_t *__restrict__ inc_ptr,
                                                   int32_t *__restrict__ inc,
                                                   const int2 *__restrict__ nbr,
                                                   int32_t *__restrict__ rowlen,
                                                   int32_t *__restrict__ stage,
                                                   uint32_t *__restrict__ inc_pos,
                                                   const int32_t *__restrict__ mid_list,
                                                   PatternCounters *cnt) {
    __shared__ int32_t s_inc[LANE_MAX * WAVE];
    __shared__ int32_t s_nb[2 * LANE_MAX * WAVE];
    __shared__ int32_t s_col[CAND_MAX * WAVE];
    const int lane = threadIdx.x;
    const int nmid = cnt->mid_count;
    for (int64_t idx = blockIdx.x * (int64_t)WAVE + lane; idx - lane < nmid; idx += (int64_t)gridDim.x * WAVE) {
    const bool in = idx < nmid;
    const int64_t v = in ? mid_list[idx] : 0;
    const int32_t is = in ? inc_ptr[v] : 0;
    const int32_t d = in ? inc_ptr[v + 1] - is : 0;
    int n = 0;
    // load the triangle ids and neighbour pairs (independent loads), then
    // sort them by triangle id (insertion sort in LDS)
    for (int t = 0; t < d; ++t) {
        LANE_AT(s_inc, t) = inc[is + t];
        const int2 nb = nbr[is + t];
        LANE_AT(s_nb, 2 * t) = nb.x;
        LANE_AT(s_nb, 2 * t + 1) = nb.y;
    }
    for (int t = 1; t < d; ++t) {
        const int32_t x = LANE_AT(s_inc, t);
        const int32_t n1 = LANE_AT(s_nb, 2 * t), n2 = LANE_AT(s_nb, 2 * t + 1);
        int j = t;
        while (j > 0 && LANE_AT(s_inc, j - 1) > x) {
            LANE_AT(s_inc, j) = LANE_AT(s_inc, j - 1);
            LANE_AT(s_nb, 2 * j) = LANE_AT(s_nb, 2 * j - 2);
            LANE_AT(s_nb, 2 * j + 1) = LANE_AT(s_nb, 2 * j - 1);
            --j;
        }
        LANE_AT(s_inc, j) = x;
        LANE_AT(s_nb, 2 * j) = n1;
        LANE_AT(s_nb, 2 * j + 1) = n2;
    }
    for (int t = 0; t < d; ++t) inc[is + t] = LANE_AT(s_inc, t);
    // sorted unique columns: v itself and every neighbour
    for (int t = -1; t < 2 * d; ++t) {
        const int32_t x = t < 0 ? static_cast<int32_t>(v) : LANE_AT(s_nb, t);
        int j = n;
        while (j > 0 && LANE_AT(s_col, j - 1) > x) --j;
        if (j > 0 && LANE_AT(s_col, j - 1) == x) continue;
        for (int m = n; m > j; --m) LANE_AT(s_col, m) = LANE_AT(s_col, m - 1);
        LANE_AT(s_col, j) = x;
        ++n;
    }
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
    {
        const int64_t base = 2 * (int64_t)is + v;
        for (int u = 0; u < n; ++u) stage[base + u] = LANE_AT(s_col, u);
    }
    if (in) rowlen[v] = n;
    int mr = n;
#pragma unroll
    for (int o = WAVE / 2; o > 0; o >>= 1) mr = max(mr, __shfl_xor(mr, o, WAVE));
    if (lane == 0) max_into(&cnt->max_row_len, mr);
    }
}
#undef LANE_AT

// One workgroup per vertex with more than LANE_MAX triangles.  Straight
// O(d^2) rank sorts in global memory: such vertices are rare.  `scratch` has
// the same layout as `stage` (2 d + 1 slots at 2 inc_ptr[v] + v).
__global__ __launch_bounds__(256) void k_rows_wide(const int32_t *__restrict__ inc_ptr,
                                                   int32_t *__restrict__ inc,
                                                   const int2 *__restrict__ nbr,
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
        // 1. sort the triangle ids (distinct) with their neighbour pairs: rank
        // sort, ids through `cols`, pairs through `cand`
        for (int t = threadIdx.x; t < d; t += blockDim.x) {
            const int32_t x = inc[is + t];
            int32_t r = 0;
            for (int s = 0; s < d; ++s) r += inc[is + s] < x;
            cols[r] = x;
            const int2 nb = nbr[is + t];
            cand[1 + 2 * r] = nb.x;
            cand[2 + 2 * r] = nb.y;
        }
        __syncthreads();
        for (int t = threadIdx.x; t < d; t += blockDim.x) inc[is + t] = cols[t];
        // 2. candidates: v, then the two other vertices of each triangle
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
            max_into(&cnt->max_row_len, m);
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

// Tile of 64 rows: the staged columns of each row (2 inc_ptr[v] + v) are
// copied into the contiguous col_idx slice of the tile, one output entry per
// lane (coalesced writes).
__global__ __launch_bounds__(WAVE) void k_copy_cols(int32_t nq, const int32_t *__restrict__ row_ptr,
                                                    const int32_t *__restrict__ inc_ptr,
                                                    const int32_t *__restrict__ stage,
                                                    int32_t *__restrict__ col_idx) {
    __shared__ int32_t s_rs[WAVE + 1];
    __shared__ int64_t s_base[WAVE];
    const int lane = threadIdx.x;
    const int64_t r0 = blockIdx.x * (int64_t)WAVE;
    const int64_t i = r0 + lane;
    const int nr = (int)((r0 + WAVE < nq ? r0 + WAVE : nq) - r0);
    if (lane < nr) {
        s_rs[lane] = row_ptr[i];
        s_base[lane] = 2 * (int64_t)inc_ptr[i] + i;
    }
    if (lane == 0) s_rs[nr] = row_ptr[r0 + nr];
    __syncthreads();
    const int32_t E0 = s_rs[0], Ew = s_rs[nr] - E0;
    for (int e = lane; e < Ew; e += WAVE) {
        const int32_t g = E0 + e;
        int lo = 0, hi = nr - 1;   // last row with s_rs[row] <= g
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (s_rs[mid] <= g) lo = mid;
            else hi = mid - 1;
        }
        col_idx[g] = stage[s_base[lo] + (g - s_rs[lo])];
    }
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

constexpr int ELAS_STAGE = 8 * WAVE;   // scalar entries of a tile staged in LDS (2 + 8 KiB)

// Tile of 64 scalar rows = a contiguous slice of Ew scalar entries and of
// 4 Ew elasticity entries.  One lane per scalar entry (coalesced read of
// col_idx): its row is found by a search over the tile's 64 row offsets in
// LDS, and it writes the pair (2c, 2c+1) into both elasticity rows 2i and
// 2i+1 (8-byte aligned: 4 rs + 2k and 4 rs + 2L + 2k are even).
__global__ __launch_bounds__(WAVE) void k_elas_pattern(int32_t nq, const int32_t *__restrict__ row_ptr,
                                                       const int32_t *__restrict__ col_idx,
                                                       int32_t *__restrict__ row_ptr_e,
                                                       int32_t *__restrict__ col_idx_e,
                                                       int aligned16) {
    constexpr int U = ELAS_STAGE / WAVE;
    __shared__ int32_t s_rs[WAVE + 1];
    __shared__ int32_t s_col[ELAS_STAGE];
    __shared__ __align__(16) int32_t s_out[4 * ELAS_STAGE];
    const int lane = threadIdx.x;
    const int64_t r0 = blockIdx.x * (int64_t)WAVE;
    const int64_t i = r0 + lane;
    const int nr = (int)((r0 + WAVE < nq ? r0 + WAVE : nq) - r0);
    if (lane < nr) s_rs[lane] = row_ptr[i];
    if (lane == 0) s_rs[nr] = row_ptr[r0 + nr];
    __syncthreads();
    if (lane < nr) {
        const int32_t rs = s_rs[lane], L = s_rs[lane + 1] - rs;
        __builtin_nontemporal_store(4 * rs, row_ptr_e + 2 * i);
        __builtin_nontemporal_store(4 * rs + 2 * L, row_ptr_e + 2 * i + 1);
    }
    if (r0 + nr == nq && lane == 0) row_ptr_e[2 * (int64_t)nq] = 4 * s_rs[nr];
    const int32_t E0 = s_rs[0], Ew = s_rs[nr] - E0;
    // tiles of at most ELAS_STAGE entries: the tile's columns are loaded with
    // all loads in flight, each lane expands its own row in LDS, and the
    // tile's output (from 4 E0 ints: 16-byte aligned when col_idx_e is) is
    // written as int4
    if (aligned16 && Ew <= ELAS_STAGE) {
        int32_t cv[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int e = lane + u * WAVE;
            cv[u] = e < Ew ? __builtin_nontemporal_load(col_idx + E0 + e) : 0;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int e = lane + u * WAVE;
            if (e < Ew) s_col[e] = cv[u];
        }
        __syncthreads();
        if (lane < nr) {
            // row 2i: [4 off + 2k + beta], row 2i+1: [4 off + 2 L + 2k + beta]
            const int32_t off = s_rs[lane] - E0, L = s_rs[lane + 1] - s_rs[lane];
            int2 *o0 = reinterpret_cast<int2 *>(s_out + 4 * off);
            int2 *o1 = reinterpret_cast<int2 *>(s_out + 4 * off + 2 * L);
            for (int32_t k = 0; k < L; ++k) {
                const int32_t c = s_col[off + k];
                const int2 v = make_int2(2 * c, 2 * c + 1);
                o0[k] = v;
                o1[k] = v;
            }
        }
        __syncthreads();
        typedef int v4i __attribute__((ext_vector_type(4)));
        v4i *dst = reinterpret_cast<v4i *>(col_idx_e + 4 * (int64_t)E0);
        const v4i *src = reinterpret_cast<const v4i *>(s_out);
        for (int32_t t = lane; t < Ew; t += WAVE) __builtin_nontemporal_store(src[t], dst + t);
        return;
    }
    // otherwise one lane per scalar entry, int2 stores straight to col_idx_e
    for (int32_t e = lane; e < Ew; e += WAVE) {
        const int32_t g = E0 + e;
        const int32_t c = col_idx[g];
        // the row holding g: the last row start <= g (empty rows share a start)
        int lo = 0, hi = nr - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (s_rs[mid] <= g) lo = mid;
            else hi = mid - 1;
        }
        const int32_t rs = s_rs[lo], L = s_rs[lo + 1] - rs, k = g - rs;
        const int2 v = make_int2(2 * c, 2 * c + 1);
        int32_t *base = col_idx_e + 4 * (int64_t)rs + 2 * k;
        *reinterpret_cast<int2 *>(base) = v;
        *reinterpret_cast<int2 *>(base + 2 * L) = v;
    }
}

// ---------------------------------------------------------------- workspace layout

namespace {
// One level of the bucket partition: `nbkt` buckets of 2^shift vertices,
// `nblk` triangle workgroups of `tpb` triangles each.
struct BucketPlan {
    int32_t shift, nbkt, nblk, tpb;
    int64_t ncounts() const { return (int64_t)nbkt * nblk; }
};

BucketPlan plan_buckets(int32_t nq, int32_t nme, int shift) {
    BucketPlan p{shift, 0, 0, 0};
    const int64_t nbkt = ((int64_t)nq + (1ll << shift) - 1) >> shift;
    if (nme <= 0 || nbkt > HIST_MAX) return p;
    int64_t tpb = ((int64_t)nme + NBLK_TARGET - 1) / NBLK_TARGET;
    tpb = (tpb + BKT_THREADS - 1) / BKT_THREADS * BKT_THREADS;
    p.nbkt = (int32_t)nbkt;
    p.tpb = (int32_t)tpb;
    p.nblk = (int32_t)(((int64_t)nme + tpb - 1) / tpb);
    return p;
}

struct PatternWork {
    PatternCounters *cnt;
    int32_t *btot, *bptr;                  // fine path: bucket totals and their scan
    int32_t *deg, *rowlen, *wide, *mid, *counts;
    int32_t *bstart;                       // start of each bucket's incidences (+ the total)
    long long *part;
    int2 *nbr;
    int32_t *ent;                          // bucket records (12 or 16 B); the region
                                           //   is reused for `stage` and `scratch`
    int32_t *stage, *scratch;
    BucketPlan fine, coarse;               // nbkt == 0: level not usable
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
    w.fine = plan_buckets(nq, nme, FINE_SHIFT);
    w.coarse = plan_buckets(nq, nme, COARSE_SHIFT);
    const bool bucket = w.coarse.nbkt > 0;
    const size_t stage_n = 6 * (size_t)nme + (size_t)nq + 1;
    int64_t ncounts = w.fine.ncounts() > w.coarse.ncounts() ? w.fine.ncounts() : w.coarse.ncounts();
    const int64_t nscan = ncounts > nq ? ncounts : nq;
    w.cnt = reinterpret_cast<PatternCounters *>(take(sizeof(PatternCounters)));
    w.btot = reinterpret_cast<int32_t *>(take(sizeof(int32_t) * (size_t)(w.fine.nbkt + 1)));
    w.bptr = reinterpret_cast<int32_t *>(take(sizeof(int32_t) * (size_t)(w.fine.nbkt + 1)));
    w.deg = reinterpret_cast<int32_t *>(take(sizeof(int32_t) * (size_t)nq));
    w.rowlen = reinterpret_cast<int32_t *>(take(sizeof(int32_t) * (size_t)nq));
    w.wide = reinterpret_cast<int32_t *>(take(sizeof(int32_t) * (size_t)nq));
    w.mid = reinterpret_cast<int32_t *>(take(sizeof(int32_t) * (size_t)nq));
    w.counts = reinterpret_cast<int32_t *>(take(sizeof(int32_t) * (size_t)(ncounts + 1)));
    const int32_t nbkt_max = w.fine.nbkt > w.coarse.nbkt ? w.fine.nbkt : w.coarse.nbkt;
    w.bstart = reinterpret_cast<int32_t *>(take(sizeof(int32_t) * (size_t)(nbkt_max + 1)));
    w.part = reinterpret_cast<long long *>(take(sizeof(long long) * (size_t)scan_partials(nscan)));
    // nbr (coarse and atomic paths) doubles as the fine path's row staging
    // area, which must not alias the bucket records it is built from
    const size_t nbr_bytes = sizeof(int2) * (3 * (size_t)nme + 1);
    const size_t fstage_bytes = sizeof(int32_t) * (6 * (size_t)nme + (size_t)nq + FINE_V);
    w.nbr = reinterpret_cast<int2 *>(take(nbr_bytes > fstage_bytes ? nbr_bytes : fstage_bytes));
    const size_t ent_bytes = bucket ? sizeof(int4) * 3 * (size_t)nme : 0;
    const size_t stage_bytes = align_up(sizeof(int32_t) * stage_n);
    char *big = take(ent_bytes > 2 * stage_bytes ? ent_bytes : 2 * stage_bytes);
    w.ent = reinterpret_cast<int32_t *>(big);
    w.stage = reinterpret_cast<int32_t *>(big);
    w.scratch = reinterpret_cast<int32_t *>(big ? big + stage_bytes : nullptr);
    w.bytes = off;
    return w;
}

// Partition the incidences into the buckets of plan P: counts per
// (workgroup, bucket), per bucket their prefix over the workgroups and the
// bucket totals, the scan of those into bstart (the total number of
// incidences at bstart[P.nbkt]), and the scatter into ent_*.
int partition(const PatternWork &W, const BucketPlan &P, bool packed, int32_t nq, int32_t nme,
              const int32_t *me, hipStream_t s) {
    const size_t hist_lds = sizeof(int32_t) * (size_t)P.nbkt;
    hipLaunchKernelGGL(k_bkt_count, dim3(P.nblk), dim3(BKT_THREADS), hist_lds, s, nme, me, nq,
                       P.shift, P.nbkt, P.tpb, W.counts, W.cnt);
    FEM_LAUNCH_CHECK();
    int st;
    hipLaunchKernelGGL(k_bkt_colscan, dim3(grid_for(P.nbkt, WAVE)), dim3(COLSCAN_WAVES * WAVE), 0, s,
                       P.nbkt, P.nblk, W.counts, W.bstart);
    FEM_LAUNCH_CHECK();
    if ((st = exclusive_scan_i32(W.bstart, W.bstart, P.nbkt, W.part, &W.cnt->total[2], &W.cnt->err, s)))
        return st;
    if (packed)
        hipLaunchKernelGGL(k_bkt_scatter<true>, dim3(P.nblk), dim3(BKT_THREADS), hist_lds, s, nme, me,
                           nq, P.shift, P.nbkt, P.tpb, W.counts, W.bstart, W.ent);
    else
        hipLaunchKernelGGL(k_bkt_scatter<false>, dim3(P.nblk), dim3(BKT_THREADS), hist_lds, s, nme, me,
                           nq, P.shift, P.nbkt, P.tpb, W.counts, W.bstart, W.ent);
    FEM_LAUNCH_CHECK();
    return FEM_OK;
}

int check_mesh_errors(const PatternCounters &h, int32_t nq) {
    FEM_REQUIRE(!(h.err & ERR_RANGE), FEM_ERANGE, "fem_pattern: a vertex index of me is outside [0, %d)", nq);
    FEM_REQUIRE(!(h.err & ERR_DEGEN), FEM_EDEGEN, "fem_pattern: a triangle repeats a vertex");
    FEM_REQUIRE(!(h.err & ERR_OVERFLOW), FEM_EOVERFLOW, "fem_pattern: count overflow");
    return FEM_OK;
}
}  // namespace

}  // namespace fem

using namespace fem;

namespace {
int g_pattern_path = FEM_PATTERN_AUTO;
}

extern "C" int fem_pattern_set_path(int path) {
    clear_error();
    FEM_REQUIRE(path == FEM_PATTERN_AUTO || path == FEM_PATTERN_COARSE || path == FEM_PATTERN_ATOMIC,
                FEM_EINVAL, "fem_pattern_set_path: unknown path %d", path);
    g_pattern_path = path;
    return FEM_OK;
}

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
                           uint32_t *inc_pos, uint64_t *fan, int32_t *slot, void *work,
                           size_t work_bytes, int64_t *nnz_out, void *stream) {
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
    PatternCounters h{};
    auto read_counters = [&]() -> int {
        FEM_HIP_CHECK(hipMemcpyAsync(&h, W.cnt, sizeof(h), hipMemcpyDeviceToHost, s));
        FEM_HIP_CHECK(hipStreamSynchronize(s));
        return FEM_OK;
    };
    const int32_t n_cnt_words = sizeof(PatternCounters) / 4;
    if ((st = fill_i32(reinterpret_cast<int32_t *>(W.cnt), n_cnt_words, 0, s))) return st;
    const int path = g_pattern_path;
    FEM_REQUIRE(path != FEM_PATTERN_COARSE || W.coarse.nbkt > 0 || nme == 0, FEM_EUNSUPPORTED,
                "fem_pattern: the coarse path cannot hold nq = %d", nq);
    bool done = false;
    if (W.fine.nbkt > 0 && path == FEM_PATTERN_AUTO) {
        // fine path: partition into 512-vertex buckets; one kernel sorts each
        // bucket and writes inc_ptr, inc, inc_pos and the staged rows; the
        // scan of the bucket totals places the rows in col_idx
        // 12-byte records when a vertex index leaves 9 spare bits
        const bool packed = nq <= (1 << PACK_SHIFT);
        if ((st = partition(W, W.fine, packed, nq, nme, me, s))) return st;
        int32_t *fstage = reinterpret_cast<int32_t *>(W.nbr);
        if (packed)
            hipLaunchKernelGGL(k_bkt_rows<true>, dim3(W.fine.nbkt), dim3(BKT_THREADS), 0, s, nq,
                               W.fine.nbkt, W.bstart, W.ent,
                               inc_ptr, inc, inc_pos, fan, W.rowlen, W.btot, fstage, W.cnt);
        else
            hipLaunchKernelGGL(k_bkt_rows<false>, dim3(W.fine.nbkt), dim3(BKT_THREADS), 0, s, nq,
                               W.fine.nbkt, W.bstart, W.ent,
                               inc_ptr, inc, inc_pos, fan, W.rowlen, W.btot, fstage, W.cnt);
        FEM_LAUNCH_CHECK();
        if ((st = exclusive_scan_i32(W.btot, W.bptr, W.fine.nbkt, W.part, &W.cnt->total[1],
                                     &W.cnt->err, s)))
            return st;
        hipLaunchKernelGGL(k_bkt_copy, dim3(W.fine.nbkt), dim3(256), 0, s, nq, W.fine.nbkt,
                           W.bstart, W.bptr, W.rowlen, fstage, row_ptr, col_idx, col_cap,
                           W.cnt);
        FEM_LAUNCH_CHECK();
        if ((st = read_counters())) return st;
        if ((st = check_mesh_errors(h, nq))) return st;
        // a bucket too large for LDS (or a vertex with very many triangles):
        // start again on the coarse path
        done = !(h.err & ERR_BUCKET);
        if (!done && (st = fill_i32(reinterpret_cast<int32_t *>(W.cnt), n_cnt_words, 0, s))) return st;
    }
    if (!done) {
        if (W.coarse.nbkt > 0 && path != FEM_PATTERN_ATOMIC) {
            // group the incidences by vertex: two-level counting sort, no global atomics
            if ((st = partition(W, W.coarse, false, nq, nme, me, s))) return st;
            hipLaunchKernelGGL(k_bkt_sort, dim3(W.coarse.nbkt), dim3(BKT_THREADS), 0, s, nq, W.bstart,
                               W.ent, inc_ptr, inc, W.nbr);
            FEM_LAUNCH_CHECK();
        } else {
            if ((st = fill_i32(W.deg, nq, 0, s))) return st;
            if (nme > 0) {
                hipLaunchKernelGGL(k_count, dim3(grid_for(nme, 256)), dim3(256), 0, s, nme, me, nq,
                                   W.deg, W.cnt);
                FEM_LAUNCH_CHECK();
            }
            if ((st = exclusive_scan_i32(W.deg, inc_ptr, nq, W.part, &W.cnt->total[0], &W.cnt->err, s)))
                return st;
            if (nme > 0) {
                hipLaunchKernelGGL(k_fill, dim3(grid_for(nme, 256)), dim3(256), 0, s, nme, me, nq,
                                   inc_ptr, W.deg, inc, W.nbr);
                FEM_LAUNCH_CHECK();
            }
        }
        hipLaunchKernelGGL(k_rows, dim3(grid_for(nq, WAVE)), dim3(WAVE), 0, s, nq, inc_ptr, inc,
                           W.nbr, W.rowlen, W.stage, inc_pos, W.mid, W.wide, W.cnt);
        FEM_LAUNCH_CHECK();
        hipLaunchKernelGGL(k_rows_mid, dim3(1024), dim3(WAVE), 0, s, inc_ptr, inc, W.nbr, W.rowlen,
                           W.stage, inc_pos, W.mid, W.cnt);
        FEM_LAUNCH_CHECK();
        hipLaunchKernelGGL(k_rows_wide, dim3(256), dim3(256), 0, s, inc_ptr, inc, W.nbr, W.rowlen,
                           W.stage, W.scratch, inc_pos, W.wide, W.cnt);
        FEM_LAUNCH_CHECK();
        if ((st = exclusive_scan_i32(W.rowlen, row_ptr, nq, W.part, &W.cnt->total[1], &W.cnt->err, s)))
            return st;
        if ((st = read_counters())) return st;
        if ((st = check_mesh_errors(h, nq))) return st;
        FEM_REQUIRE(!(h.err & ERR_ROWLEN) && h.max_row_len <= 65535, FEM_EUNSUPPORTED,
                    "fem_pattern: a row has %d entries (limit 65535)", h.max_row_len);
        FEM_REQUIRE(h.total[1] <= col_cap, FEM_ENOSPC, "fem_pattern: nnz = %lld exceeds col_cap = %lld",
                    (long long)h.total[1], (long long)col_cap);
        hipLaunchKernelGGL(k_copy_cols, dim3(grid_for(nq, WAVE)), dim3(WAVE), 0, s, nq, row_ptr,
                           inc_ptr, W.stage, col_idx);
        FEM_LAUNCH_CHECK();
        if (fan) {
            hipLaunchKernelGGL(k_fan_plan, dim3(grid_for(nq, 256)), dim3(256), 0, s, nq, row_ptr,
                               inc_ptr, inc_pos, fan);
            FEM_LAUNCH_CHECK();
        }
    }
    const int64_t nnz = h.total[1];
    FEM_REQUIRE(!(h.err & ERR_NOSPC) && nnz <= col_cap, FEM_ENOSPC,
                "fem_pattern: nnz = %lld exceeds col_cap = %lld", (long long)nnz, (long long)col_cap);
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

extern "C" int fem_fan_plan(int32_t nq, int32_t nme, const int32_t *row_ptr, const int32_t *inc_ptr,
                            const uint32_t *inc_pos, uint64_t *fan, void *stream) {
    clear_error();
    FEM_REQUIRE(nq >= 1 && nme >= 0, FEM_EINVAL, "fem_fan_plan: bad sizes");
    FEM_REQUIRE(row_ptr && inc_ptr && fan && (nme == 0 || inc_pos), FEM_EINVAL,
                "fem_fan_plan: NULL array");
    hipLaunchKernelGGL(k_fan_plan, dim3(grid_for(nq, 256)), dim3(256), 0, as_stream(stream), nq,
                       row_ptr, inc_ptr, inc_pos, fan);
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
    FEM_REQUIRE((reinterpret_cast<uintptr_t>(col_idx_e) & 7) == 0, FEM_EINVAL,
                "fem_elas_pattern: col_idx_e must be 8-byte aligned");
    hipLaunchKernelGGL(k_elas_pattern, dim3(grid_for(nq, WAVE)), dim3(WAVE), 0,
                       as_stream(stream), nq, row_ptr, col_idx, row_ptr_e, col_idx_e,
                       (reinterpret_cast<uintptr_t>(col_idx_e) & 15) == 0 ? 1 : 0);
    FEM_LAUNCH_CHECK();
    return FEM_OK;
}
