// fem_tet.hip -- P1 tetrahedra in 3D (the extension the Conclusion names):
// mass and stiffness matrices, row by row.
//
// Pattern (fem_tet_pattern).  The row of vertex v holds v and every vertex
// that shares a tetrahedron with it.  The 4 nme (vertex, tetrahedron)
// incidences are grouped by vertex with a two-level counting sort over
// buckets of 128 consecutive vertex ids (no global atomics):
//   1 bucket count    about 256 workgroups over contiguous ranges of
//                     tetrahedra: mesh checks and an LDS histogram
//   2 offsets         per bucket, the prefix of its counts over the
//                     workgroups (k_bkt_colscan), and the scan of the bucket
//                     totals: the start of every (bucket, workgroup) run
//   3 bucket scatter  one 16-byte record per incidence: (4 k + a, the other
//                     three vertices in the order a+1, a+2, a+3 mod 4, and
//                     the vertex relative to its bucket)
//   4 bucket rows     one workgroup per bucket, one lane per vertex, all in
//                     LDS: counting sort by vertex -> inc_ptr; per vertex the
//                     distinct neighbours in a small hash set, sorted by a
//                     network in registers -> the row; the tetrahedra sorted
//                     by id -> inc, and the row slots of each tetrahedron's
//                     other three vertices -> inc_pos
//   5 scan            of the bucket totals
//   6 bucket copy     staged rows -> col_idx, and row_ptr
// General path (more than 128 * 36864 vertices, a bucket above TB_CAP
// incidences, a vertex in more than 32 tetrahedra or with more than 27
// neighbours, or chosen with fem_tet_pattern_set_path): the index arrays of
// all 16 local entries (triplet t = r nme + k for entry r = 4 b + a of
// element k: row me[k][a], column me[k][b]) compressed by fem_sparse; the
// contributors of a row's diagonal entry are its incidences, merged by
// tetrahedron id -> inc; the slots by binary search in the row -> inc_pos.
// Both paths give the same arrays, bit for bit.
//
// Values (fem_tet_assemble).  One lane per row: the coordinates of the row's
// vertices (relative to the row's own vertex) are staged in LDS, then the
// lane walks its tetrahedra in ascending id, computes the element row of its
// vertex and adds it to per-slot accumulators in LDS; the wave's rows leave
// as one contiguous, coalesced range.  Every entry is summed in ascending
// tetrahedron order, so the values are bitwise reproducible.
//
// Element matrices, for K = (x0, x1, x2, x3) with x0 the row's vertex,
// e_i = x_i - x0, D = det[e1 e2 e3]: the rows of [e1 e2 e3]^{-1} are c1 / D,
// c2 / D, c3 / D with c1 = e2 x e3, c2 = e3 x e1, c3 = e1 x e2, so
// grad lambda_i = c_i / D with c0 = -(c1 + c2 + c3), and with |K| = |D| / 6
//   stiffness  S_0b = |K| grad lambda_0 . grad lambda_b = c0 . c_b / (6 |D|)
//   mass       M_0b = |K| (1 + delta_0b) / 20 = |D| (1 + delta_0b) / 120
// Both are invariant under a relabelling of x1..x3, so only the row slots of
// the other three vertices are needed, not their local order.

#include "fem_internal.h"

extern "C" int fem_sparse_workspace(int32_t m, int32_t n, int64_t nt, size_t *bytes);
extern "C" int fem_sparse(int32_t m, int32_t n, int64_t nt, const int32_t *I, const int32_t *J,
                          const double *V, int32_t *row_ptr, int32_t *col_idx, double *vals,
                          int64_t col_cap, int32_t *contrib_ptr, int32_t *contrib, void *work,
                          size_t work_bytes, int64_t *nnz_out, void *stream);

namespace fem {
namespace {

constexpr int TET_M = 1, TET_S = 4;   // FEM_OP_MASS, FEM_OP_STIFF

// device-side error bits (beside ERR_RANGE, ERR_DEGEN, ERR_OVERFLOW, ERR_ROWLEN)
enum : int { TERR_BUCKET = 16, TERR_NOSPC = 32 };

constexpr int TB_SHIFT = 7;                  // 128 vertices per bucket
constexpr int TB_V = 1 << TB_SHIFT;
constexpr int TB_CAP = 3584;                 // incidences a bucket may hold in LDS
constexpr int TB_EPT = TB_CAP / TB_V;        // records per thread of k_tbkt_rows
constexpr int TB_DMAX = 32;                  // tetrahedra per vertex (sorting network)
constexpr int TB_HS = 32;                    // hash slots per vertex
constexpr int TB_NMAX = 27;                  // distinct neighbours per vertex
constexpr int TB_HIST_MAX = 36864;           // buckets an LDS histogram holds (144 KiB)
constexpr int TB_BLK_TARGET = 256;           // workgroups of the partition pass
constexpr int TB_PART_THREADS = 512;
constexpr int POS_BITS = 10;                 // inc_pos: three 10-bit row slots
constexpr int ROW_MAX = 1 << POS_BITS;       // longest row inc_pos can address
constexpr uint32_t HASH_EMPTY = 0xffffffffu;
constexpr int32_t VID_MASK = (1 << 24) - 1;  // bucket records: vertex ids below 2^24

inline size_t align_up(size_t x) { return (x + 255) & ~size_t(255); }

__device__ inline bool tet_ok(const int (&v)[4], int32_t nq) {
    return (uint32_t)v[0] < (uint32_t)nq && (uint32_t)v[1] < (uint32_t)nq &&
           (uint32_t)v[2] < (uint32_t)nq && (uint32_t)v[3] < (uint32_t)nq && v[0] != v[1] &&
           v[0] != v[2] && v[0] != v[3] && v[1] != v[2] && v[1] != v[3] && v[2] != v[3];
}

__device__ inline int tet_err(const int (&v)[4], int32_t nq) {
    for (int a = 0; a < 4; ++a)
        if ((uint32_t)v[a] >= (uint32_t)nq) return ERR_RANGE;
    return tet_ok(v, nq) ? 0 : ERR_DEGEN;
}

// ------------------------------------------------------------------ partition

// counts[blk * nbkt + b] = incidences of workgroup blk (tpb tetrahedra)
// whose vertex falls in bucket b (each workgroup writes one contiguous row);
// mesh checks.
__global__ __launch_bounds__(TB_PART_THREADS) void k_tbkt_count(int32_t nme, const int4 *__restrict__ me,
                                                               int32_t nq, int32_t nbkt, int32_t tpb,
                                                               int32_t *__restrict__ counts,
                                                               PatternCounters *cnt) {
    extern __shared__ int32_t s_hist[];
    for (int b = threadIdx.x; b < nbkt; b += TB_PART_THREADS) s_hist[b] = 0;
    __syncthreads();
    int bad = 0;
    const int64_t k0 = (int64_t)blockIdx.x * tpb;
    const int64_t k1 = (k0 + tpb < nme) ? k0 + tpb : nme;
    constexpr int H = 8;   // tetrahedra with loads in flight per thread
    for (int64_t kb = k0 + threadIdx.x; kb < k1; kb += H * TB_PART_THREADS) {
        int4 t[H];
#pragma unroll
        for (int j = 0; j < H; ++j) {
            const int64_t k = kb + j * TB_PART_THREADS;
            t[j] = k < k1 ? me[k] : make_int4(0, 0, 0, 0);
        }
#pragma unroll
        for (int j = 0; j < H; ++j) {
            if (kb + j * TB_PART_THREADS >= k1) continue;
            const int v[4] = {t[j].x, t[j].y, t[j].z, t[j].w};
            const int e = tet_err(v, nq);
            if (e) {
                bad |= e;
                continue;
            }
#pragma unroll
            for (int a = 0; a < 4; ++a) atomicAdd(&s_hist[v[a] >> TB_SHIFT], 1);
        }
    }
    if (bad) atomicOr(&cnt->err, bad);
    __syncthreads();
    for (int b = threadIdx.x; b < nbkt; b += TB_PART_THREADS)
        counts[(int64_t)blockIdx.x * nbkt + b] = s_hist[b];
}

// Same tetrahedra per workgroup as k_tbkt_count: each incidence (k, a) goes
// to the run of its (bucket, workgroup) pair as the record
// (4 k + a, me[k][a+1] | (v mod TB_V) << 24, me[k][a+2], me[k][a+3]).
__global__ __launch_bounds__(TB_PART_THREADS) void k_tbkt_scatter(int32_t nme, const int4 *__restrict__ me,
                                                                 int32_t nq, int32_t nbkt, int32_t tpb,
                                                                 const int32_t *__restrict__ offs,
                                                                 const int32_t *__restrict__ bstart,
                                                                 int4 *__restrict__ ent) {
    extern __shared__ int32_t s_cur[];
    // the run of (b, this workgroup): the bucket's start plus the incidences
    // of the workgroups before it (one contiguous row of offs)
    const int32_t *row = offs + (int64_t)blockIdx.x * nbkt;
    for (int b = threadIdx.x; b < nbkt; b += TB_PART_THREADS) s_cur[b] = bstart[b] + row[b];
    __syncthreads();
    const int64_t k0 = (int64_t)blockIdx.x * tpb;
    const int64_t k1 = (k0 + tpb < nme) ? k0 + tpb : nme;
    constexpr int H = 8;
    for (int64_t kb = k0 + threadIdx.x; kb < k1; kb += H * TB_PART_THREADS) {
        int4 t[H];
#pragma unroll
        for (int j = 0; j < H; ++j) {
            const int64_t k = kb + j * TB_PART_THREADS;
            t[j] = k < k1 ? me[k] : make_int4(-1, -1, -1, -1);
        }
#pragma unroll
        for (int j = 0; j < H; ++j) {
            const int64_t k = kb + j * TB_PART_THREADS;
            const int v[4] = {t[j].x, t[j].y, t[j].z, t[j].w};
            if (k >= k1 || !tet_ok(v, nq)) continue;
#pragma unroll
            for (int a = 0; a < 4; ++a) {
                const int32_t pos = atomicAdd(&s_cur[v[a] >> TB_SHIFT], 1);
                ent[pos] = make_int4(static_cast<int32_t>(4 * k + a),
                                     v[(a + 1) & 3] | ((v[a] & (TB_V - 1)) << 24), v[(a + 2) & 3],
                                     v[(a + 3) & 3]);
            }
        }
    }
}

// ------------------------------------------------------------------ bucket rows

template <int N>
__device__ __forceinline__ void bitonic_sort_u32(uint32_t (&k)[N]) {
#pragma unroll
    for (int size = 2; size <= N; size <<= 1)
#pragma unroll
        for (int stride = size >> 1; stride > 0; stride >>= 1)
#pragma unroll
            for (int i = 0; i < N; ++i) {
                const int l = i ^ stride;
                if (l > i) {
                    const bool up = (i & size) == 0;
                    const uint32_t a = k[i], b = k[l];
                    k[i] = up ? min(a, b) : max(a, b);
                    k[l] = up ? max(a, b) : min(a, b);
                }
            }
}

// Exclusive scan of one int per thread over a workgroup of TB_V threads.
__device__ __noinline__ int32_t tb_block_scan(int32_t v, int32_t *s_wsum, int32_t *total) {
    const int lane = threadIdx.x & (WAVE - 1), wid = threadIdx.x / WAVE;
    const int32_t incl = wave_inclusive_scan(v);
    if (lane == WAVE - 1) s_wsum[wid] = incl;
    __syncthreads();
    int32_t off = incl - v, tot = 0;
#pragma unroll
    for (int w = 0; w < TB_V / WAVE; ++w) {
        if (w < wid) off += s_wsum[w];
        tot += s_wsum[w];
    }
    __syncthreads();
    *total = tot;
    return off;
}

__device__ __forceinline__ uint32_t tb_hash(int32_t u) {
    return ((uint32_t)u * 2654435761u) >> (32 - 5);   // top 5 bits: TB_HS = 32 slots
}

// One workgroup (one thread per vertex) per bucket of TB_V vertices, all in
// LDS (steps 4 of the header).  The bucket's rows go to its own region of
// `stage` (at 3 e0 + v0: a vertex in d tetrahedra has at most 3 d + 1
// entries); k_tbkt_copy moves them once the bucket totals are scanned.  A
// bucket or vertex beyond the limits sets TERR_BUCKET and the host runs the
// general path instead.
__global__ __launch_bounds__(TB_V) void k_tbkt_rows(int32_t nq, int32_t nbkt,
                                                   const int32_t *__restrict__ bstart,
                                                   const int4 *__restrict__ ent,
                                                   int32_t *__restrict__ inc_ptr,
                                                   int32_t *__restrict__ inc,
                                                   uint32_t *__restrict__ inc_pos,
                                                   int32_t *__restrict__ rowoff,
                                                   int32_t *__restrict__ btot,
                                                   int32_t *__restrict__ stage, PatternCounters *cnt) {
    __shared__ int32_t s_cur[TB_V];
    // the vertices' slices of the records, each slice start moved on by the
    // vertex's index (one word of padding per vertex): slices of about 24
    // words would otherwise start on a few banks only
    __shared__ int32_t s_key[TB_CAP + TB_V], s_n1[TB_CAP + TB_V], s_n2[TB_CAP + TB_V],
        s_n3[TB_CAP + TB_V];
    __shared__ uint32_t s_hash[TB_HS * TB_V];   // [slot][vertex]
    __shared__ int32_t s_wsum[TB_V / WAVE];
    const int tid = threadIdx.x;
    const int32_t b = blockIdx.x;
    const int64_t e0 = bstart[b], e1 = bstart[b + 1];
    const bool fits = e1 - e0 <= TB_CAP;
    const int32_t v0 = b << TB_SHIFT;
    const int32_t v = v0 + tid;
    // ---- count and scan (the bucket's records stay in registers)
    int4 x[TB_EPT];
#pragma unroll
    for (int u = 0; u < TB_EPT; ++u) {
        const int64_t y = e0 + tid + u * TB_V;
        x[u] = (fits && y < e1) ? ent[y] : make_int4(0, -1, 0, 0);
    }
    s_cur[tid] = 0;
    __syncthreads();
#pragma unroll
    for (int u = 0; u < TB_EPT; ++u)
        if (x[u].y >= 0) atomicAdd(&s_cur[(uint32_t)x[u].y >> 24], 1);
    __syncthreads();
    int32_t d = s_cur[tid];
    int32_t unused;
    const int32_t is = tb_block_scan(d, s_wsum, &unused);
    const int32_t js = is + tid;   // the slice in LDS (padded)
    s_cur[tid] = js;
    if (v < nq) inc_ptr[v] = static_cast<int32_t>(e0) + is;
    if (b == nbkt - 1 && tid == 0) inc_ptr[nq] = static_cast<int32_t>(e1);
    __syncthreads();
    // ---- counting sort into LDS
#pragma unroll
    for (int u = 0; u < TB_EPT; ++u) {
        if (x[u].y < 0) continue;
        const int32_t p = atomicAdd(&s_cur[(uint32_t)x[u].y >> 24], 1);
        s_key[p] = x[u].x;
        s_n1[p] = x[u].y & VID_MASK;
        s_n2[p] = x[u].z;
        s_n3[p] = x[u].w;
    }
    __syncthreads();
    // ---- distinct neighbours: a hash set per vertex
    uint32_t *hs = s_hash + tid;   // slot s at hs[s * TB_V]
#pragma unroll
    for (int s = 0; s < TB_HS; ++s) hs[s * TB_V] = HASH_EMPTY;
    if (v >= nq) d = 0;
    bool bad = !fits || d > TB_DMAX;
    int32_t nd = 0;
    // linear probing; the set never fills (at most TB_NMAX of TB_HS slots),
    // so a probe ends at y or at an empty slot
    auto insert = [&](int32_t y) {
        uint32_t h = tb_hash(y), e = hs[h * TB_V];
#pragma unroll 1
        for (int it = 1; it < TB_HS && e != (uint32_t)y && e != HASH_EMPTY; ++it) {
            h = (h + 1) & (TB_HS - 1);
            e = hs[h * TB_V];
        }
        if (e == HASH_EMPTY) {
            if (nd == TB_NMAX) bad = true;
            else {
                hs[h * TB_V] = (uint32_t)y;
                ++nd;
            }
        }
    };
    if (!bad) {
        for (int t = 0; t < d && !bad; ++t) {
            insert(s_n1[js + t]);
            insert(s_n2[js + t]);
            insert(s_n3[js + t]);
        }
    }
    if (bad) atomicOr(&cnt->err, TERR_BUCKET);
    const int32_t L = (!bad && d > 0) ? nd + 1 : 0;
    // ---- row offsets inside the bucket
    int32_t Tb;
    const int32_t lro = tb_block_scan(L, s_wsum, &Tb);
    if (v < nq) rowoff[v] = lro;
    if (tid == 0) btot[b] = Tb;
    if (L > 0) {
        // the row: the hash set sorted by a network (entry u << 5 | slot),
        // v in its place; each slot learns its position (u | pos << 24)
        int32_t *out = stage + 3 * e0 + v0 + lro;
        uint32_t dist[TB_HS];
#pragma unroll
        for (int s = 0; s < TB_HS; ++s) {
            const uint32_t e = hs[s * TB_V];
            dist[s] = e == HASH_EMPTY ? HASH_EMPTY : (e << 5) | (uint32_t)s;
        }
        bitonic_sort_u32<TB_HS>(dist);
        int32_t below = 0;   // neighbours below v
#pragma unroll
        for (int r = 0; r < TB_HS; ++r) {
            if (r < nd) {
                const int32_t u = (int32_t)(dist[r] >> 5);
                const int pos = r + (u > v ? 1 : 0);
                hs[(dist[r] & 31u) * TB_V] = (uint32_t)u | ((uint32_t)pos << 24);
                out[pos] = u;
                below += u < v ? 1 : 0;
            }
        }
        out[below] = v;
        // every neighbour is in the set: the probe ends at its slot
        auto slot_of = [&](int32_t y) -> uint32_t {
            uint32_t h = tb_hash(y), e = hs[h * TB_V];
#pragma unroll 1
            for (int it = 1; it < TB_HS && (e & (uint32_t)VID_MASK) != (uint32_t)y; ++it) {
                h = (h + 1) & (TB_HS - 1);
                e = hs[h * TB_V];
            }
            return e >> 24;
        };
        // each tetrahedron's slots, packed into its record's first neighbour
        for (int t = 0; t < d; ++t) {
            const int j = js + t;
            s_n1[j] = (int32_t)(slot_of(s_n1[j]) | (slot_of(s_n2[j]) << POS_BITS) |
                                (slot_of(s_n3[j]) << (2 * POS_BITS)));
        }
        // the tetrahedra by id (entry k << 5 | index in the vertex's slice)
        uint32_t sk[TB_DMAX];
#pragma unroll
        for (int t = 0; t < TB_DMAX; ++t)
            sk[t] = t < d ? ((uint32_t)(s_key[js + t] >> 2) << 5) | (uint32_t)t : HASH_EMPTY;
        bitonic_sort_u32<TB_DMAX>(sk);
        // the sorted order goes to the vertex's hash slots, no longer needed
#pragma unroll
        for (int t = 0; t < TB_DMAX; ++t) hs[t * TB_V] = sk[t];
        const int64_t ib = e0 + is;
        for (int t = 0; t < d; ++t) {
            const int j = js + (int)(hs[t * TB_V] & 31u);
            inc[ib + t] = s_key[j];
            inc_pos[ib + t] = (uint32_t)s_n1[j];
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
        if (mr > __hip_atomic_load(&cnt->max_row_len, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
            atomicMax(&cnt->max_row_len, mr);
        if (mi > __hip_atomic_load(&cnt->max_inc, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
            atomicMax(&cnt->max_inc, mi);
    }
}

// Bucket b's staged rows to col_idx at bptr[b], and row_ptr of its vertices.
__global__ __launch_bounds__(256) void k_tbkt_copy(int32_t nq, int32_t nbkt,
                                                  const int32_t *__restrict__ bstart,
                                                  const int32_t *__restrict__ bptr,
                                                  const int32_t *__restrict__ rowoff,
                                                  const int32_t *__restrict__ stage,
                                                  int32_t *__restrict__ row_ptr,
                                                  int32_t *__restrict__ col_idx, int64_t col_cap,
                                                  PatternCounters *cnt) {
    const int32_t b = blockIdx.x;
    const int64_t e0 = bstart[b];
    const int32_t v0 = b << TB_SHIFT;
    const int32_t P = bptr[b], T = bptr[b + 1] - P;
    for (int t = threadIdx.x; t < TB_V; t += 256)
        if (v0 + t < nq) row_ptr[v0 + t] = P + rowoff[v0 + t];
    if (b == nbkt - 1 && threadIdx.x == 0) row_ptr[nq] = bptr[nbkt];
    if (P + (int64_t)T > col_cap) {
        if (threadIdx.x == 0) atomicOr(&cnt->err, TERR_NOSPC);
        return;
    }
    const int32_t *src = stage + 3 * e0 + v0;
    for (int i = threadIdx.x; i < T; i += 256) col_idx[P + i] = src[i];
}

// ------------------------------------------------------------------ general path

// Ig / Jg of element k (one lane per element; the writes for a fixed entry r
// are coalesced across lanes).  Invalid elements are reported and contribute
// vertex 0, so that the compression still runs in bounds.
__global__ __launch_bounds__(256) void k_tet_triplets(int32_t nme, const int4 *__restrict__ me,
                                                      int32_t nq, int32_t *__restrict__ I,
                                                      int32_t *__restrict__ J, PatternCounters *cnt) {
    const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (k >= nme) return;
    const int4 t = me[k];
    int v[4] = {t.x, t.y, t.z, t.w};
    const int e = tet_err(v, nq);
    if (e) {
        atomicOr(&cnt->err, e);
#pragma unroll
        for (int a = 0; a < 4; ++a) v[a] = 0;
    }
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
        for (int a = 0; a < 4; ++a) {
            const int64_t s = (int64_t)(4 * b + a) * nme + k;
            I[s] = v[a];
            J[s] = v[b];
        }
}

__device__ inline int32_t find_in_row(const int32_t *__restrict__ row, int32_t L, int32_t y) {
    int32_t lo = 0, hi = L;
    while (lo < hi) {
        const int32_t mid = (lo + hi) >> 1;
        if (row[mid] < y) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// Per vertex: its incidences are the contributors of its diagonal entry
// (triplets r = 5 a); deg[v] = their number.  Rows beyond ROW_MAX entries
// cannot be addressed by inc_pos.
__global__ __launch_bounds__(256) void k_tet_deg(int32_t nq, const int32_t *__restrict__ row_ptr,
                                                 const int32_t *__restrict__ col_idx,
                                                 const int32_t *__restrict__ cptr,
                                                 int32_t *__restrict__ deg, PatternCounters *cnt) {
    const int32_t v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= nq) return;
    const int32_t rs = row_ptr[v], L = row_ptr[v + 1] - rs;
    int32_t d = 0;
    if (L > 0) {
        const int32_t pd = find_in_row(col_idx + rs, L, v);
        d = cptr[rs + pd + 1] - cptr[rs + pd];
    }
    deg[v] = d;
    if (L > ROW_MAX) atomicOr(&cnt->err, ERR_ROWLEN);
    if (L > __hip_atomic_load(&cnt->max_row_len, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
        atomicMax(&cnt->max_row_len, L);
    if (d > __hip_atomic_load(&cnt->max_inc, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
        atomicMax(&cnt->max_inc, d);
}

// Per vertex: the diagonal contributors t = 5 a nme + k are four runs (a =
// 0..3) ascending in k; merged by k they give inc (4 k + a), and the other
// three vertices of each tetrahedron are found in the row.
__global__ __launch_bounds__(256) void k_tet_derive(int32_t nq, int32_t nme, const int4 *__restrict__ me,
                                                    const int32_t *__restrict__ row_ptr,
                                                    const int32_t *__restrict__ col_idx,
                                                    const int32_t *__restrict__ cptr,
                                                    const int32_t *__restrict__ contrib,
                                                    const int32_t *__restrict__ inc_ptr,
                                                    int32_t *__restrict__ inc,
                                                    uint32_t *__restrict__ inc_pos) {
    const int32_t v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= nq) return;
    const int32_t rs = row_ptr[v], L = row_ptr[v + 1] - rs;
    const int32_t is = inc_ptr[v], d = inc_ptr[v + 1] - is;
    if (L == 0 || d == 0 || L > ROW_MAX) return;
    const int32_t *row = col_idx + rs;
    const int32_t pd = find_in_row(row, L, v);
    const int32_t *c = contrib + cptr[rs + pd];
    // run a covers [lo[a], lo[a + 1]): the first t >= 5 a nme
    int32_t lo[5];
    lo[0] = 0;
    lo[4] = d;
    for (int a = 1; a < 4; ++a) {
        const int64_t thr = 5ll * a * nme;
        int32_t l = lo[a - 1], h = d;
        while (l < h) {
            const int32_t m = (l + h) >> 1;
            if ((int64_t)c[m] < thr) l = m + 1;
            else h = m;
        }
        lo[a] = l;
    }
    int32_t cur[4] = {lo[0], lo[1], lo[2], lo[3]};
    for (int32_t j = 0; j < d; ++j) {
        int best = -1;
        int32_t bk = 0;
        for (int a = 0; a < 4; ++a) {
            if (cur[a] < lo[a + 1]) {
                const int32_t k = c[cur[a]] - 5 * a * nme;
                if (best < 0 || k < bk) {
                    best = a;
                    bk = k;
                }
            }
        }
        ++cur[best];
        const int4 t = me[bk];
        const int32_t w[4] = {t.x, t.y, t.z, t.w};
        inc[is + j] = 4 * bk + best;
        inc_pos[is + j] = (uint32_t)find_in_row(row, L, w[(best + 1) & 3]) |
                          ((uint32_t)find_in_row(row, L, w[(best + 2) & 3]) << POS_BITS) |
                          ((uint32_t)find_in_row(row, L, w[(best + 3) & 3]) << (2 * POS_BITS));
    }
}

// ------------------------------------------------------------------ values

// Row of the element matrices of x0's vertex in the tetrahedron (x0, x1, x2,
// x3), from e_i = x_i - x0: diagonal and the three off-diagonal entries.
struct TetRow {
    double md, mo;            // mass: diagonal, off-diagonal
    double sd, s1, s2, s3;    // stiffness: diagonal, towards x1, x2, x3
};

// Cross and dot products with explicit fused multiply-adds (the library is
// built without contraction, so every kernel that calls tet_row rounds the
// same way).
__device__ __forceinline__ void cross_fma(const double (&a)[3], const double (&b)[3], double (&o)[3]) {
    o[0] = fma(a[1], b[2], -(a[2] * b[1]));
    o[1] = fma(a[2], b[0], -(a[0] * b[2]));
    o[2] = fma(a[0], b[1], -(a[1] * b[0]));
}

__device__ __forceinline__ double dot_fma(const double (&a)[3], const double (&b)[3]) {
    return fma(a[0], b[0], fma(a[1], b[1], a[2] * b[2]));
}

template <int MASK>
__device__ __forceinline__ TetRow tet_row(const double (&e1)[3], const double (&e2)[3],
                                          const double (&e3)[3]) {
    double c1[3];
    cross_fma(e2, e3, c1);
    const double aD = fabs(dot_fma(e1, c1));
    TetRow r{};
    if constexpr ((MASK & TET_M) != 0) {
        r.mo = aD * (1.0 / 120.0);
        r.md = r.mo + r.mo;
    }
    if constexpr ((MASK & TET_S) != 0) {
        double c2[3], c3[3], c0[3];
        cross_fma(e3, e1, c2);
        cross_fma(e1, e2, c3);
#pragma unroll
        for (int i = 0; i < 3; ++i) c0[i] = -(c1[i] + c2[i] + c3[i]);
        // 1 / (6 |D|): the hardware reciprocal and two Newton-Raphson steps
        // (e = 1 - x r, r += r e), to within an ulp or two of the quotient
        const double x6 = 6.0 * aD;
        double s6 = __builtin_amdgcn_rcp(x6);
        s6 = fma(s6, fma(-x6, s6, 1.0), s6);
        s6 = fma(s6, fma(-x6, s6, 1.0), s6);
        r.sd = dot_fma(c0, c0) * s6;
        r.s1 = dot_fma(c0, c1) * s6;
        r.s2 = dot_fma(c0, c2) * s6;
        r.s3 = dot_fma(c0, c3) * s6;
    }
    return r;
}

constexpr int TROW_LM = 16;   // row slots a lane keeps in LDS
constexpr int TROW_IP = 32;   // tetrahedra per row whose slots are loaded up front

// What a lane holds of its row in one group of WAVE consecutive rows.
struct TetRowLoad {
    int32_t v, rs, L, is, d;
    double x0[3];
    int32_t u[TROW_LM];       // the row's vertex ids (unused slots: vertex 0)
    uint32_t pp[TROW_IP];     // its first tetrahedra's slots
    double y[TROW_LM][3];     // the coordinates of its vertices
};

// One lane per row, one wave (a group of WAVE consecutive rows) per
// workgroup.  LDS: X [LM][3][WAVE] the row's vertices relative to the row's
// own, A [NA][LM][WAVE] the per-slot sums (through which the group's rows
// leave, coalesced).  The loads come in three dependent stages, each issued
// whole: the row and tetrahedron ranges; the row's vertex ids and its first
// TROW_IP tetrahedra's slots; the coordinates.  The sums read registers and
// LDS only.  A row longer than LM is summed by its lane one slot at a time
// from global memory (same terms, same order, so the same values bit for
// bit).
template <int MASK>
__global__ __launch_bounds__(WAVE) void k_tet_rows(int32_t nq, const double *__restrict__ q,
                                                   const int32_t *__restrict__ row_ptr,
                                                   const int32_t *__restrict__ col_idx,
                                                   const int32_t *__restrict__ inc_ptr,
                                                   const uint32_t *__restrict__ inc_pos,
                                                   double *__restrict__ vm, double *__restrict__ vs,
                                                   int accumulate) {
    constexpr bool HM = (MASK & TET_M) != 0, HS = (MASK & TET_S) != 0;
    constexpr int LM = TROW_LM, IP = TROW_IP;
    __shared__ double X[LM * 3 * WAVE];
    __shared__ double A[(HM ? 1 : 0) + (HS ? 1 : 0)][LM * WAVE];
    const int lane = threadIdx.x;
    constexpr int MI = HM ? 0 : -1, SI = (HM && HS) ? 1 : 0;
    auto XA = [&](int p, int c) -> double & { return X[(p * 3 + c) * WAVE + lane]; };
    auto AM = [&](int p) -> double & { return A[MI < 0 ? 0 : MI][p * WAVE + lane]; };
    auto AS = [&](int p) -> double & { return A[SI][p * WAVE + lane]; };
    const int32_t nnz_all = row_ptr[nq], ninc_all = inc_ptr[nq];

    // load stage 1: ranges and the row's own vertex
    auto load_head = [&](int32_t r0, TetRowLoad &g) {
        g.v = r0 + lane;
        g.rs = g.L = g.is = g.d = 0;
        g.x0[0] = g.x0[1] = g.x0[2] = 0.0;
        if (g.v < nq) {
            g.rs = row_ptr[g.v];
            g.L = row_ptr[g.v + 1] - g.rs;
            g.is = inc_ptr[g.v];
            g.d = inc_ptr[g.v + 1] - g.is;
            g.x0[0] = q[3 * (int64_t)g.v];
            g.x0[1] = q[3 * (int64_t)g.v + 1];
            g.x0[2] = q[3 * (int64_t)g.v + 2];
        }
    };
    // load stage 2: vertex ids and slots, 16 bytes per load (4-byte aligned,
    // which global loads accept) where the arrays reach that far
    auto load_ids = [&](TetRowLoad &g) {
        const bool on = g.L <= LM && g.L > 0;
        if (on && g.rs + LM <= nnz_all) {
#pragma unroll
            for (int j = 0; j < LM; j += 4) {
                int4 w;
                __builtin_memcpy(&w, col_idx + g.rs + j, sizeof(int4));
                g.u[j] = w.x;
                g.u[j + 1] = w.y;
                g.u[j + 2] = w.z;
                g.u[j + 3] = w.w;
            }
        } else {
#pragma unroll
            for (int p = 0; p < LM; ++p) g.u[p] = (on && p < g.L) ? col_idx[g.rs + p] : 0;
        }
        if (on && g.is + IP <= ninc_all) {
#pragma unroll
            for (int j = 0; j < IP; j += 4) {
                uint4 w;
                __builtin_memcpy(&w, inc_pos + g.is + j, sizeof(uint4));
                g.pp[j] = w.x;
                g.pp[j + 1] = w.y;
                g.pp[j + 2] = w.z;
                g.pp[j + 3] = w.w;
            }
        } else {
#pragma unroll
            for (int t = 0; t < IP; ++t) g.pp[t] = (on && t < g.d) ? inc_pos[g.is + t] : 0u;
        }
#pragma unroll
        for (int p = 0; p < LM; ++p) g.u[p] = (on && p < g.L) ? g.u[p] : 0;
#pragma unroll
        for (int t = 0; t < IP; ++t) g.pp[t] = (on && t < g.d) ? g.pp[t] : 0u;
    };
    // load stage 3: a vertex's three coordinates in two loads (16 + 8 bytes; the
    // 16-byte one is 8-byte aligned), no branch (unused slots read vertex 0)
    auto load_coords = [&](TetRowLoad &g) {
#pragma unroll
        for (int p = 0; p < LM; ++p) {
            const double *qu = q + 3 * (int64_t)g.u[p];
            double2 xy;
            __builtin_memcpy(&xy, qu, sizeof(double2));
            g.y[p][0] = xy.x;
            g.y[p][1] = xy.y;
            g.y[p][2] = qu[2];
        }
    };

    // the sums of one group, then its rows out
    auto run_group = [&](int32_t r0, const TetRowLoad &g) {
        const bool valid = g.v < nq;
        const bool fast = g.L <= LM;
        const uint64_t longmask = __ballot(!fast);
        const int32_t rsv = valid ? g.rs : nnz_all;   // rows past nq start at the end
        const int32_t R1 = r0 + WAVE < nq ? row_ptr[r0 + WAVE] : nnz_all;
        // the most tetrahedra of a row summed in LDS, over the wave (all
        // lanes take part; the others count 0)
        int32_t dmax = (fast && g.L > 0) ? g.d : 0;
#pragma unroll
        for (int o = WAVE / 2; o > 0; o >>= 1) dmax = max(dmax, __shfl_xor(dmax, o, WAVE));
        int32_t pd = 0;
        if (fast && g.L > 0) {
#pragma unroll
            for (int p = 0; p < LM; ++p) {
                if (p < g.L) {
#pragma unroll
                    for (int c = 0; c < 3; ++c) XA(p, c) = g.y[p][c] - g.x0[c];
                    if (g.u[p] == g.v) pd = p;
                    if constexpr (HM) AM(p) = 0.0;
                    if constexpr (HS) AS(p) = 0.0;
                }
            }
            // one step per tetrahedron: its three slots are distinct, so
            // the six accumulators are read together with the coordinates
            // and written back together (one LDS round trip).  A lane past
            // its last tetrahedron steps on the diagonal slot, whose sum is
            // overwritten at the end (only the diagonal sums keep their
            // values), so that the steps need no branch and pairs of them
            // can overlap
            const uint32_t wpd = (uint32_t)pd | ((uint32_t)pd << POS_BITS) | ((uint32_t)pd << (2 * POS_BITS));
            double dM = 0.0, dS = 0.0;
            auto step = [&](uint32_t w, bool on) {
                w = on ? w : wpd;
                const int p1 = w & (ROW_MAX - 1), p2 = (w >> POS_BITS) & (ROW_MAX - 1),
                          p3 = (w >> (2 * POS_BITS)) & (ROW_MAX - 1);
                double e1[3], e2[3], e3[3];
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    e1[c] = XA(p1, c);
                    e2[c] = XA(p2, c);
                    e3[c] = XA(p3, c);
                }
                double m1 = 0.0, m2 = 0.0, m3 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
                if constexpr (HM) {
                    m1 = AM(p1);
                    m2 = AM(p2);
                    m3 = AM(p3);
                }
                if constexpr (HS) {
                    s1 = AS(p1);
                    s2 = AS(p2);
                    s3 = AS(p3);
                }
                const TetRow r = tet_row<MASK>(e1, e2, e3);
                if constexpr (HM) {
                    dM = on ? dM + r.md : dM;
                    AM(p1) = m1 + r.mo;
                    AM(p2) = m2 + r.mo;
                    AM(p3) = m3 + r.mo;
                }
                if constexpr (HS) {
                    dS = on ? dS + r.sd : dS;
                    AS(p1) = s1 + r.s1;
                    AS(p2) = s2 + r.s2;
                    AS(p3) = s3 + r.s3;
                }
            };
#pragma unroll
            for (int t = 0; t < IP; t += 2) {
                if (t < dmax) {
                    step(g.pp[t], t < g.d);
                    step(g.pp[t + 1], t + 1 < g.d);
                }
            }
            for (int32_t t = IP; t < dmax; ++t) step(t < g.d ? inc_pos[g.is + t] : 0u, t < g.d);
            if constexpr (HM) AM(pd) = dM;
            if constexpr (HS) AS(pd) = dS;
        } else if (!fast) {
            // long row: slot by slot, the terms of that slot in ascending order
            const int32_t *row = col_idx + g.rs;
            pd = find_in_row(row, g.L, g.v);
            for (int32_t p = 0; p < g.L; ++p) {
                double sm = 0.0, ss = 0.0;
                for (int32_t t = 0; t < g.d; ++t) {
                    const uint32_t w = inc_pos[g.is + t];
                    const int p1 = w & (ROW_MAX - 1), p2 = (w >> POS_BITS) & (ROW_MAX - 1),
                              p3 = (w >> (2 * POS_BITS)) & (ROW_MAX - 1);
                    if (!(p == pd || p == p1 || p == p2 || p == p3)) continue;
                    double e[3][3];
                    const int ps[3] = {p1, p2, p3};
#pragma unroll
                    for (int i = 0; i < 3; ++i) {
                        const int64_t uu = row[ps[i]];
#pragma unroll
                        for (int c = 0; c < 3; ++c) e[i][c] = q[3 * uu + c] - g.x0[c];
                    }
                    const TetRow r = tet_row<MASK>(e[0], e[1], e[2]);
                    if (p == pd) {
                        sm += r.md;
                        ss += r.sd;
                    } else {
                        sm += r.mo;
                        ss += p == p1 ? r.s1 : (p == p2 ? r.s2 : r.s3);
                    }
                }
                if constexpr (HM) vm[g.rs + p] = accumulate ? vm[g.rs + p] + sm : sm;
                if constexpr (HS) vs[g.rs + p] = accumulate ? vs[g.rs + p] + ss : ss;
            }
        }
        // the workgroup is one wave, whose LDS accesses complete in program
        // order: a scheduling barrier orders the sums before the write-out.
        // The group's rows leave as one contiguous range.
        __builtin_amdgcn_wave_barrier();
        const int32_t R0 = __shfl(rsv, 0, WAVE);
        auto put = [&](int32_t e, int o, int p) {
            if constexpr (HM) {
                const double a = A[MI < 0 ? 0 : MI][p * WAVE + o];
                vm[e] = accumulate ? vm[e] + a : a;
            }
            if constexpr (HS) {
                const double a = A[SI][p * WAVE + o];
                vs[e] = accumulate ? vs[e] + a : a;
            }
        };
        if (longmask == 0) {
            // every row of the group has at most LM entries (the range at
            // most LM * WAVE): each lane copies its sums in CSR order into
            // the coordinate LDS (no longer needed), and the range is then
            // written in order; both sides touch consecutive words
            constexpr int NA = (HM ? 1 : 0) + (HS ? 1 : 0);
            double *T = X;   // [NA][LM * WAVE]
            for (int p = 0; p < g.L; ++p) {
                if constexpr (HM) T[g.rs - R0 + p] = AM(p);
                if constexpr (HS) T[(NA - 1) * LM * WAVE + g.rs - R0 + p] = AS(p);
            }
            __builtin_amdgcn_wave_barrier();
            // overwrites are streaming stores (separate loops: merged with the
            // accumulate path's store, the hint would be dropped)
            const double *TS = T + (NA - 1) * LM * WAVE;
            if (!accumulate) {
                for (int32_t e = R0 + lane; e < R1; e += WAVE) {
                    if constexpr (HM) __builtin_nontemporal_store(T[e - R0], vm + e);
                    if constexpr (HS) __builtin_nontemporal_store(TS[e - R0], vs + e);
                }
            } else {
                for (int32_t e = R0 + lane; e < R1; e += WAVE) {
                    if constexpr (HM) vm[e] += T[e - R0];
                    if constexpr (HS) vs[e] += TS[e - R0];
                }
            }
        } else {
            // entry e belongs to the last row whose start is <= e (empty
            // rows share the next start); the search reads the starts from
            // the other lanes, all lanes taking part
            for (int32_t base = R0; base < R1; base += WAVE) {
                const int32_t e = base + lane;
                int lo = 0;
#pragma unroll
                for (int stp = WAVE / 2; stp > 0; stp >>= 1) {
                    const int cand = lo + stp;
                    const int32_t sc = __shfl(rsv, cand < WAVE ? cand : WAVE - 1, WAVE);
                    if (cand < WAVE && sc <= e) lo = cand;
                }
                // every lane reads its row's start before any lane leaves the pass
                const int32_t rlo = __shfl(rsv, lo, WAVE);
                const int p = e - rlo;
                if (e >= R1 || ((longmask >> lo) & 1u) || p >= LM) continue;
                put(e, lo, p);
            }
        }
        __builtin_amdgcn_wave_barrier();   // the rows have left LDS
    };

    const int32_t r0 = blockIdx.x * WAVE;
    TetRowLoad g;
    load_head(r0, g);
    load_ids(g);
    load_coords(g);
    run_group(r0, g);
}

// ------------------------------------------------------------------ workspace

struct TetBucketPlan {
    int32_t nbkt, nblk, tpb;   // nbkt == 0: the bucket path cannot hold the mesh
    int64_t ncounts() const { return (int64_t)nbkt * nblk; }
};

TetBucketPlan plan_tet_buckets(int32_t nq, int32_t nme) {
    TetBucketPlan p{0, 0, 0};
    const int64_t nbkt = ((int64_t)nq + TB_V - 1) >> TB_SHIFT;
    if (nme <= 0 || nbkt > TB_HIST_MAX || nq > VID_MASK) return p;
    int64_t tpb = ((int64_t)nme + TB_BLK_TARGET - 1) / TB_BLK_TARGET;
    tpb = (tpb + TB_PART_THREADS - 1) / TB_PART_THREADS * TB_PART_THREADS;
    p.nbkt = (int32_t)nbkt;
    p.tpb = (int32_t)tpb;
    p.nblk = (int32_t)(((int64_t)nme + tpb - 1) / tpb);
    return p;
}

// Counters, then two alternatives sharing one region: the bucket path
// (counts, scan partials, totals, row offsets, records, staged rows) or the
// general path (triplets, contributor lists, fem_sparse's workspace, degrees).
struct TetPatternWork {
    PatternCounters *cnt;
    TetBucketPlan plan;
    int32_t *counts, *bstart, *btot, *bptr, *rowoff, *stage;
    long long *part;
    int4 *ent;
    int32_t *I, *J, *cptr, *contrib, *deg;
    long long *gpart;
    char *sparse;
    size_t sparse_bytes, bytes;
};

TetPatternWork carve_tet(int32_t nq, int32_t nme, char *base, int *st) {
    TetPatternWork w{};
    const int64_t nt = 16 * (int64_t)nme;
    size_t sb = 0;
    *st = fem_sparse_workspace(nq, nq, nt, &sb);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        char *p = base ? base + off : nullptr;
        off += align_up(bytes);
        return p;
    };
    w.cnt = reinterpret_cast<PatternCounters *>(take(sizeof(PatternCounters)));
    const size_t shared0 = off;
    // general path
    const size_t ntn = (size_t)(nt > 0 ? nt : 1);
    w.I = reinterpret_cast<int32_t *>(take(sizeof(int32_t) * ntn));
    w.J = reinterpret_cast<int32_t *>(take(sizeof(int32_t) * ntn));
    w.cptr = reinterpret_cast<int32_t *>(take(sizeof(int32_t) * (ntn + 1)));
    w.contrib = reinterpret_cast<int32_t *>(take(sizeof(int32_t) * ntn));
    w.deg = reinterpret_cast<int32_t *>(take(sizeof(int32_t) * (size_t)nq));
    w.gpart = reinterpret_cast<long long *>(take(sizeof(long long) * (size_t)scan_partials(nq)));
    w.sparse = take(sb);
    w.sparse_bytes = sb;
    const size_t general_end = off;
    // bucket path, over the same bytes
    off = shared0;
    w.plan = plan_tet_buckets(nq, nme);
    if (w.plan.nbkt > 0) {
        const int64_t nc = w.plan.ncounts();
        w.counts = reinterpret_cast<int32_t *>(take(sizeof(int32_t) * (size_t)(nc + 1)));
        w.bstart = reinterpret_cast<int32_t *>(take(sizeof(int32_t) * (size_t)(w.plan.nbkt + 1)));
        w.part = reinterpret_cast<long long *>(take(sizeof(long long) * (size_t)scan_partials(nc)));
        w.btot = reinterpret_cast<int32_t *>(take(sizeof(int32_t) * (size_t)(w.plan.nbkt + 1)));
        w.bptr = reinterpret_cast<int32_t *>(take(sizeof(int32_t) * (size_t)(w.plan.nbkt + 1)));
        w.rowoff = reinterpret_cast<int32_t *>(take(sizeof(int32_t) * (size_t)nq));
        w.ent = reinterpret_cast<int4 *>(take(sizeof(int4) * 4 * (size_t)nme));
        w.stage = reinterpret_cast<int32_t *>(take(sizeof(int32_t) * (12 * (size_t)nme + (size_t)nq + TB_V)));
    }
    w.bytes = off > general_end ? off : general_end;
    return w;
}

int tet_check_errors(const PatternCounters &h, int32_t nq) {
    FEM_REQUIRE(!(h.err & ERR_RANGE), FEM_ERANGE, "fem_tet_pattern: a vertex index of me is outside [0, %d)", nq);
    FEM_REQUIRE(!(h.err & ERR_DEGEN), FEM_EDEGEN, "fem_tet_pattern: an element repeats a vertex");
    FEM_REQUIRE(!(h.err & ERR_OVERFLOW), FEM_EOVERFLOW, "fem_tet_pattern: count overflow");
    return FEM_OK;
}

int g_tet_path = FEM_PATTERN_AUTO;

}  // namespace
}  // namespace fem

using namespace fem;

extern "C" int fem_tet_pattern_set_path(int path) {
    clear_error();
    FEM_REQUIRE(path == FEM_PATTERN_AUTO || path == FEM_PATTERN_COARSE, FEM_EINVAL,
                "fem_tet_pattern_set_path: path must be FEM_PATTERN_AUTO or FEM_PATTERN_COARSE (got %d)",
                path);
    g_tet_path = path;
    return FEM_OK;
}

extern "C" int64_t fem_tet_nnz_bound(int32_t nq, int32_t nme) {
    return (int64_t)(nq > 0 ? nq : 0) + 12 * (int64_t)(nme > 0 ? nme : 0);
}

extern "C" int fem_tet_pattern_workspace(int32_t nq, int32_t nme, size_t *bytes) {
    clear_error();
    FEM_REQUIRE(bytes != nullptr, FEM_EINVAL, "fem_tet_pattern_workspace: bytes is NULL");
    FEM_REQUIRE(nq >= 1 && nme >= 0, FEM_EINVAL, "fem_tet_pattern_workspace: need nq >= 1, nme >= 0");
    FEM_REQUIRE(16 * (int64_t)nme <= INT32_MAX, FEM_EOVERFLOW,
                "fem_tet_pattern_workspace: 16 nme exceeds int32");
    int st = FEM_OK;
    const TetPatternWork W = carve_tet(nq, nme, nullptr, &st);
    if (st) return st;
    *bytes = W.bytes;
    return FEM_OK;
}

extern "C" int fem_tet_pattern(int32_t nq, int32_t nme, const int32_t *me, int32_t *row_ptr,
                               int32_t *col_idx, int64_t col_cap, int32_t *inc_ptr, int32_t *inc,
                               uint32_t *inc_pos, void *work, size_t work_bytes, int64_t *nnz_out,
                               void *stream) {
    clear_error();
    FEM_REQUIRE(nq >= 1 && nme >= 0, FEM_EINVAL, "fem_tet_pattern: need nq >= 1, nme >= 0");
    FEM_REQUIRE(16 * (int64_t)nme <= INT32_MAX, FEM_EOVERFLOW, "fem_tet_pattern: 16 nme exceeds int32");
    FEM_REQUIRE(row_ptr && inc_ptr && work && nnz_out, FEM_EINVAL,
                "fem_tet_pattern: NULL row_ptr, inc_ptr, work or nnz_out");
    FEM_REQUIRE(nme == 0 || (me && inc && inc_pos), FEM_EINVAL, "fem_tet_pattern: NULL me, inc or inc_pos");
    FEM_REQUIRE(col_cap >= 0 && (col_cap == 0 || col_idx), FEM_EINVAL,
                "fem_tet_pattern: NULL col_idx or negative col_cap");
    FEM_REQUIRE((reinterpret_cast<uintptr_t>(me) & 15) == 0, FEM_EINVAL,
                "fem_tet_pattern: me must be 16-byte aligned");
    int st = FEM_OK;
    const TetPatternWork W = carve_tet(nq, nme, static_cast<char *>(work), &st);
    if (st) return st;
    FEM_REQUIRE(work_bytes >= W.bytes, FEM_ENOSPC, "fem_tet_pattern: workspace of %zu bytes, need %zu",
                work_bytes, W.bytes);
    hipStream_t s = as_stream(stream);
    const int4 *me4 = reinterpret_cast<const int4 *>(me);
    PatternCounters h{};
    auto read_counters = [&]() -> int {
        FEM_HIP_CHECK(hipMemcpyAsync(&h, W.cnt, sizeof(h), hipMemcpyDeviceToHost, s));
        FEM_HIP_CHECK(hipStreamSynchronize(s));
        return FEM_OK;
    };
    const int32_t n_cnt_words = sizeof(PatternCounters) / 4;
    if ((st = fill_i32(reinterpret_cast<int32_t *>(W.cnt), n_cnt_words, 0, s))) return st;
    if (nme == 0) {
        // no incidences: every row is empty
        if ((st = fill_i32(row_ptr, (int64_t)nq + 1, 0, s))) return st;
        if ((st = fill_i32(inc_ptr, (int64_t)nq + 1, 0, s))) return st;
        FEM_HIP_CHECK(hipStreamSynchronize(s));
        *nnz_out = 0;
        return FEM_OK;
    }
    bool done = false;
    int64_t nnz = 0;
    if (W.plan.nbkt > 0 && g_tet_path == FEM_PATTERN_AUTO) {
        const TetBucketPlan &P = W.plan;
        const size_t hist_lds = sizeof(int32_t) * (size_t)P.nbkt;
        hipLaunchKernelGGL(k_tbkt_count, dim3(P.nblk), dim3(TB_PART_THREADS), hist_lds, s, nme, me4, nq,
                           P.nbkt, P.tpb, W.counts, W.cnt);
        FEM_LAUNCH_CHECK();
        hipLaunchKernelGGL(k_bkt_colscan, dim3(grid_for(P.nbkt, WAVE)), dim3(COLSCAN_WAVES * WAVE), 0, s,
                           P.nbkt, P.nblk, W.counts, W.bstart);
        FEM_LAUNCH_CHECK();
        if ((st = exclusive_scan_i32(W.bstart, W.bstart, P.nbkt, W.part, &W.cnt->total[2], &W.cnt->err,
                                     s)))
            return st;
        hipLaunchKernelGGL(k_tbkt_scatter, dim3(P.nblk), dim3(TB_PART_THREADS), hist_lds, s, nme, me4,
                           nq, P.nbkt, P.tpb, W.counts, W.bstart, W.ent);
        FEM_LAUNCH_CHECK();
        hipLaunchKernelGGL(k_tbkt_rows, dim3(P.nbkt), dim3(TB_V), 0, s, nq, P.nbkt, W.bstart, W.ent,
                           inc_ptr, inc, inc_pos, W.rowoff, W.btot, W.stage, W.cnt);
        FEM_LAUNCH_CHECK();
        if ((st = exclusive_scan_i32(W.btot, W.bptr, P.nbkt, W.part, &W.cnt->total[1], &W.cnt->err, s)))
            return st;
        hipLaunchKernelGGL(k_tbkt_copy, dim3(P.nbkt), dim3(256), 0, s, nq, P.nbkt, W.bstart, W.bptr,
                           W.rowoff, W.stage, row_ptr, col_idx, col_cap, W.cnt);
        FEM_LAUNCH_CHECK();
        if ((st = read_counters())) return st;
        if ((st = tet_check_errors(h, nq))) return st;
        done = !(h.err & TERR_BUCKET);
        nnz = h.total[1];
        if (done) {
            FEM_REQUIRE(!(h.err & TERR_NOSPC) && nnz <= col_cap, FEM_ENOSPC,
                        "fem_tet_pattern: nnz = %lld exceeds col_cap = %lld", (long long)nnz,
                        (long long)col_cap);
        } else if ((st = fill_i32(reinterpret_cast<int32_t *>(W.cnt), n_cnt_words, 0, s))) {
            return st;
        }
    }
    if (!done) {
        hipLaunchKernelGGL(k_tet_triplets, dim3(grid_for(nme, 256)), dim3(256), 0, s, nme, me4, nq, W.I,
                           W.J, W.cnt);
        FEM_LAUNCH_CHECK();
        if ((st = read_counters())) return st;
        if ((st = tet_check_errors(h, nq))) return st;
        const int64_t nt = 16 * (int64_t)nme;
        st = fem_sparse(nq, nq, nt, W.I, W.J, nullptr, row_ptr, col_idx, nullptr, col_cap, W.cptr,
                        W.contrib, W.sparse, W.sparse_bytes, &nnz, stream);
        if (st) return st;
        hipLaunchKernelGGL(k_tet_deg, dim3(grid_for(nq, 256)), dim3(256), 0, s, nq, row_ptr, col_idx,
                           W.cptr, W.deg, W.cnt);
        FEM_LAUNCH_CHECK();
        if ((st = exclusive_scan_i32(W.deg, inc_ptr, nq, W.gpart, &W.cnt->total[0], &W.cnt->err, s)))
            return st;
        hipLaunchKernelGGL(k_tet_derive, dim3(grid_for(nq, 256)), dim3(256), 0, s, nq, nme, me4, row_ptr,
                           col_idx, W.cptr, W.contrib, inc_ptr, inc, inc_pos);
        FEM_LAUNCH_CHECK();
        if ((st = read_counters())) return st;
        FEM_REQUIRE(!(h.err & ERR_ROWLEN), FEM_EUNSUPPORTED,
                    "fem_tet_pattern: a row has %d entries (inc_pos addresses at most %d)",
                    h.max_row_len, ROW_MAX);
    }
    *nnz_out = nnz;
    return FEM_OK;
}

extern "C" int fem_tet_assemble(int ops, int32_t nq, int32_t nme, int64_t nnz, const double *q,
                                const int32_t *row_ptr, const int32_t *col_idx,
                                const int32_t *inc_ptr, const uint32_t *inc_pos, double *vals_M,
                                double *vals_S, int flags, void *stream) {
    clear_error();
    FEM_REQUIRE(ops == TET_M || ops == TET_S || ops == (TET_M | TET_S), FEM_EINVAL,
                "fem_tet_assemble: ops must be FEM_OP_MASS and/or FEM_OP_STIFF");
    FEM_REQUIRE(nq >= 1 && nme >= 0 && nnz >= 0 && nnz <= INT32_MAX, FEM_EINVAL,
                "fem_tet_assemble: bad sizes");
    FEM_REQUIRE((flags & ~FEM_ACCUMULATE) == 0, FEM_EINVAL,
                "fem_tet_assemble: only FEM_ACCUMULATE is supported (the sums are deterministic)");
    FEM_REQUIRE(q && row_ptr && inc_ptr, FEM_EINVAL, "fem_tet_assemble: NULL q, row_ptr or inc_ptr");
    FEM_REQUIRE(nnz == 0 || (col_idx && inc_pos), FEM_EINVAL, "fem_tet_assemble: NULL col_idx or inc_pos");
    FEM_REQUIRE(!(ops & TET_M) || nnz == 0 || vals_M, FEM_EINVAL, "fem_tet_assemble: NULL vals_M");
    FEM_REQUIRE(!(ops & TET_S) || nnz == 0 || vals_S, FEM_EINVAL, "fem_tet_assemble: NULL vals_S");
    if (nnz == 0) return FEM_OK;
    hipStream_t s = as_stream(stream);
    const int acc = (flags & FEM_ACCUMULATE) ? 1 : 0;
    const unsigned g = grid_for(nq, WAVE);
    if (ops == (TET_M | TET_S))
        hipLaunchKernelGGL(k_tet_rows<TET_M | TET_S>, dim3(g), dim3(WAVE), 0, s, nq, q, row_ptr, col_idx,
                           inc_ptr, inc_pos, vals_M, vals_S, acc);
    else if (ops == TET_M)
        hipLaunchKernelGGL(k_tet_rows<TET_M>, dim3(g), dim3(WAVE), 0, s, nq, q, row_ptr, col_idx, inc_ptr,
                           inc_pos, vals_M, nullptr, acc);
    else
        hipLaunchKernelGGL(k_tet_rows<TET_S>, dim3(g), dim3(WAVE), 0, s, nq, q, row_ptr, col_idx, inc_ptr,
                           inc_pos, nullptr, vals_S, acc);
    FEM_LAUNCH_CHECK();
    return FEM_OK;
}
