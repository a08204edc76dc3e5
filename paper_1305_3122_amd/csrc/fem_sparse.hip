// fem_sparse.hip -- general sparse(I, J, V, m, n): triplets with duplicates
// summed into CSR (rows ascending, columns ascending, structural zeros kept),
// the compression every OptV2 assembly ends in (Section 4 for the storage,
// Section 6 for the triplet arrays Ig, Jg, Kg).
//
// Bucketed by row in two levels, no global atomics:
//   k_sp_count / scan / k_sp_scatter   triplets -> runs of (coarse bucket,
//                                      workgroup): row mod Rc, (column, t),
//                                      value; 256 to 512 coarse buckets, so the
//                                      runs are long and the count matrix small
//   k_sp_split                         one workgroup per coarse bucket splits
//                                      it into fine buckets of 2^rf rows, rf
//                                      chosen per coarse bucket from its own
//                                      row density (the largest whose fullest
//                                      bucket fits in LDS) -> fine_off, cshift
//   k_sp_rows (LDS) / k_sp_rows_big    a workgroup per fine bucket at a time:
//                                      counting sort by row, then each row
//                                      sorted by (column, t) as 64-bit keys,
//                                      duplicates summed in ascending t; rows
//                                      staged per bucket at slots from a block
//                                      scan of run starts, sorted triplet
//                                      order written as the contributor list
//                                      (every step parallel over the triplets)
//   scan of bucket totals / k_sp_copy  rows -> col_idx / values, row_ptr
// Every value is the sum of its triplets' values in ascending t, so the result
// is bitwise reproducible and equal to a sequential left-to-right sum.

#include "fem_internal.h"

namespace fem {

namespace {

constexpr int SP_THREADS = 256;       // fine-bucket kernels
constexpr int SPP_THREADS = 1024;     // partition and split kernels
constexpr int SP_CAP = 2688;          // triplets of a bucket held in LDS (3 workgroups / CU)
constexpr int SP_RMAX_SHIFT = 9;      // at most 512 rows per fine bucket
constexpr int SP_COARSE_TARGET = 512; // coarse buckets: long runs in the first scatter, and
                                      // one split workgroup per CU or more
constexpr int SP_COARSE_MAX = 4096;   // coarse buckets the partition's LDS holds
constexpr int SP_SPLIT_MAX_SHIFT = 12;  // at most 4096 fine buckets per coarse one
constexpr int SP_NBLK_TARGET = 256;   // triplet workgroups of the partition pass (one per CU,
                                      // so that the runs they fill fit the L2 of their XCD)
constexpr int SP_COPY_GRID = 4096;    // workgroups looping over the fine bucket slots
constexpr int SP_ADAPT_SHIFT = 2;     // fine buckets down to 1/4 of the planned rows where the
                                      // rows are denser than average

enum : int { SP_ERR_RANGE = 1, SP_ERR_OVERFLOW = 4, SP_ERR_NOSPC = 32 };

struct SparseCounters {
    int err;
    int big_count;        // buckets too large for LDS, listed for k_sp_rows_big
    int max_row;          // most triplets in one row
    int pad_;
    long long total[4];   // scan totals: [1] nnz, [2] triplets
};

__device__ inline void max_into_sp(int *dst, int v) {
    if (v > __hip_atomic_load(dst, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) atomicMax(dst, v);
}

// counts[b * nblk + blk]: triplets of workgroup blk (tpb triplets) in coarse
// bucket b; range checks.
__global__ __launch_bounds__(SPP_THREADS) void k_sp_count(int64_t nt, const int32_t *__restrict__ I,
                                                         const int32_t *__restrict__ J, int32_t m,
                                                         int32_t n, int rs, int32_t nbkt, int64_t tpb,
                                                         int32_t *__restrict__ counts,
                                                         SparseCounters *cnt) {
    extern __shared__ int32_t s_hist[];
    const int32_t nblk = gridDim.x;
    for (int b = threadIdx.x; b < nbkt; b += SPP_THREADS) s_hist[b] = 0;
    __syncthreads();
    const int64_t t0 = (int64_t)blockIdx.x * tpb;
    const int64_t t1 = (t0 + tpb < nt) ? t0 + tpb : nt;
    int bad = 0;
    constexpr int H = 4;
    for (int64_t tb = t0 + threadIdx.x; tb < t1; tb += H * SPP_THREADS) {
        int32_t i[H], j[H];
#pragma unroll
        for (int u = 0; u < H; ++u) {
            const int64_t t = tb + u * SPP_THREADS;
            i[u] = t < t1 ? I[t] : 0;
            j[u] = t < t1 ? J[t] : 0;
        }
#pragma unroll
        for (int u = 0; u < H; ++u) {
            if (tb + u * SPP_THREADS >= t1) continue;
            if ((uint32_t)i[u] >= (uint32_t)m || (uint32_t)j[u] >= (uint32_t)n) {
                bad = 1;
                continue;
            }
            atomicAdd(&s_hist[i[u] >> rs], 1);
        }
    }
    if (bad) atomicOr(&cnt->err, SP_ERR_RANGE);
    __syncthreads();
    for (int b = threadIdx.x; b < nbkt; b += SPP_THREADS)
        counts[(int64_t)b * nblk + blockIdx.x] = s_hist[b];
}

// Tile multisplit: a workgroup's TILE elements (IPT per thread: bucket key
// in [0, nk), or -1 for none, and the payload rl / ct / val) are sorted by
// bucket in LDS, then each bucket's elements of the tile are written as one
// contiguous segment at the workgroup's cursor for that bucket, g_cur[key]
// (advanced by the segment).  Consecutive tiles extend the same runs, so the
// runs' lines fill while they are still in L2.  LDS (dynamic): cnt [nk+1] |
// gcur [nk] | key [TILE] | rl [TILE] | ct [TILE] | val [TILE].
constexpr int TILE = 4096;        // the first-level scatter (one workgroup per CU)
constexpr int TILE_SPLIT = 4096;  // the split (one workgroup per coarse bucket): the per-tile
                                  // work on the fine counters is amortised over more triplets;
constexpr int TILE_SPLIT_NV = 8192;  // twice that without values (no value array in LDS)

struct TileLds {
    int32_t *cnt, *gcur, *rl;
    uint16_t *key;
    int2 *ct;
    double *val;
};

template <int T, bool HV = true>
__device__ inline TileLds tile_lds(int32_t nk) {
    extern __shared__ __align__(16) unsigned char s_dyn[];
    TileLds L;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        unsigned char *p = s_dyn + off;
        off += (bytes + 15) & ~size_t(15);
        return p;
    };
    L.cnt = reinterpret_cast<int32_t *>(take(sizeof(int32_t) * (nk + 1)));
    L.gcur = reinterpret_cast<int32_t *>(take(sizeof(int32_t) * nk));
    L.key = reinterpret_cast<uint16_t *>(take(sizeof(uint16_t) * T));
    L.rl = reinterpret_cast<int32_t *>(take(sizeof(int32_t) * T));
    L.ct = reinterpret_cast<int2 *>(take(sizeof(int2) * T));
    L.val = HV ? reinterpret_cast<double *>(take(sizeof(double) * T)) : nullptr;
    return L;
}

template <int T, bool HV = true>
inline size_t tile_lds_bytes(int32_t nk) {
    auto up = [](size_t b) { return (b + 15) & ~size_t(15); };
    return up(4 * (size_t)(nk + 1)) + up(4 * (size_t)nk) + up(2 * (size_t)T) + up(4 * (size_t)T) +
           up(8 * (size_t)T) + (HV ? up(8 * (size_t)T) : 0);
}

// Exclusive scan of cnt[0, nk) in place over the workgroup; cnt[nk] = total.
__device__ inline void block_scan_counts(int32_t *cnt, int32_t nk, int32_t *s_wsum) {
    const int tid = threadIdx.x;
    const int per = (nk + SPP_THREADS - 1) / SPP_THREADS;
    int32_t mine = 0;
    for (int k = 0; k < per; ++k) {
        const int32_t j = tid * per + k;
        if (j < nk) mine += cnt[j];
    }
    const int lane = tid & (WAVE - 1), wid = tid / WAVE;
    const int32_t incl = wave_inclusive_scan(mine);
    if (lane == WAVE - 1) s_wsum[wid] = incl;
    __syncthreads();
    int32_t run = incl - mine, tot = 0;
    for (int w = 0; w < SPP_THREADS / WAVE; ++w) {
        if (w < wid) run += s_wsum[w];
        tot += s_wsum[w];
    }
    for (int k = 0; k < per; ++k) {
        const int32_t j = tid * per + k;
        if (j < nk) {
            const int32_t c = cnt[j];
            cnt[j] = run;
            run += c;
        }
    }
    if (tid == 0) cnt[nk] = tot;
    __syncthreads();
}

template <int IPT>
__device__ inline void tile_multisplit(const TileLds &L, int32_t nk, const int32_t (&key)[IPT],
                                       const int32_t (&prl)[IPT], const int2 (&pct)[IPT],
                                       const double (&pval)[IPT], bool has_val, int32_t *s_wsum,
                                       int32_t *__restrict__ out_rl, int2 *__restrict__ out_ct,
                                       double *__restrict__ out_val) {
    const int tid = threadIdx.x;
    for (int32_t k = tid; k < nk; k += SPP_THREADS) L.cnt[k] = 0;
    __syncthreads();
    int32_t rank[IPT];
#pragma unroll
    for (int u = 0; u < IPT; ++u) rank[u] = key[u] >= 0 ? atomicAdd(&L.cnt[key[u]], 1) : 0;
    __syncthreads();
    block_scan_counts(L.cnt, nk, s_wsum);
#pragma unroll
    for (int u = 0; u < IPT; ++u) {
        if (key[u] < 0) continue;
        const int32_t p = L.cnt[key[u]] + rank[u];
        L.key[p] = static_cast<uint16_t>(key[u]);
        L.rl[p] = prl[u];
        L.ct[p] = pct[u];
        if (has_val) L.val[p] = pval[u];
    }
    __syncthreads();
    const int32_t ntile = L.cnt[nk];
    for (int32_t p = tid; p < ntile; p += SPP_THREADS) {
        const int32_t k = L.key[p];
        const int64_t g = (int64_t)L.gcur[k] + (p - L.cnt[k]);
        out_rl[g] = L.rl[p];
        out_ct[g] = L.ct[p];
        if (has_val) out_val[g] = L.val[p];
    }
    __syncthreads();
    for (int32_t k = tid; k < nk; k += SPP_THREADS) L.gcur[k] += L.cnt[k + 1] - L.cnt[k];
    __syncthreads();
}

// Same triplets per workgroup as k_sp_count: each goes to the run of its
// (coarse bucket, workgroup) pair, as rl = row mod Rc, ct = (column, t) and
// rval = V[t] (three arrays, so that the split's count reads rl alone).
__global__ __launch_bounds__(SPP_THREADS) void k_sp_scatter(int64_t nt, const int32_t *__restrict__ I,
                                                           const int32_t *__restrict__ J,
                                                           const double *__restrict__ V, int32_t m,
                                                           int32_t n, int rs, int32_t nbkt, int64_t tpb,
                                                           const int32_t *__restrict__ offs,
                                                           int32_t *__restrict__ rl, int2 *__restrict__ ct,
                                                           double *__restrict__ rval) {
    __shared__ int32_t s_wsum[SPP_THREADS / WAVE];
    constexpr int IPT = TILE / SPP_THREADS;
    const TileLds L = tile_lds<TILE>(nbkt);
    const int32_t nblk = gridDim.x;
    for (int b = threadIdx.x; b < nbkt; b += SPP_THREADS)
        L.gcur[b] = offs[(int64_t)b * nblk + blockIdx.x];
    __syncthreads();
    const int64_t t0 = (int64_t)blockIdx.x * tpb;
    const int64_t t1 = (t0 + tpb < nt) ? t0 + tpb : nt;
    const int32_t rmask = (1 << rs) - 1;
    // the next tile's loads are issued before this tile's multisplit, so
    // they are in flight while it runs
    int32_t ni[IPT], nj[IPT];
    double nv[IPT];
    auto load = [&](int64_t tb) {
#pragma unroll
        for (int u = 0; u < IPT; ++u) {
            const int64_t t = tb + threadIdx.x + u * SPP_THREADS;
            ni[u] = t < t1 ? I[t] : -1;
            nj[u] = t < t1 ? J[t] : -1;
            nv[u] = (V && t < t1) ? V[t] : 0.0;
        }
    };
    if (t0 < t1) load(t0);
    for (int64_t tb = t0; tb < t1; tb += TILE) {
        int32_t key[IPT], prl[IPT];
        int2 pct[IPT];
        double pval[IPT];
#pragma unroll
        for (int u = 0; u < IPT; ++u) {
            const int64_t t = tb + threadIdx.x + u * SPP_THREADS;
            const int32_t i = ni[u], j = nj[u];
            pval[u] = nv[u];
            const bool ok = (uint32_t)i < (uint32_t)m && (uint32_t)j < (uint32_t)n;
            key[u] = ok ? (i >> rs) : -1;
            prl[u] = i & rmask;
            pct[u] = make_int2(j, static_cast<int32_t>(t));
        }
        if (tb + TILE < t1) load(tb + TILE);
        tile_multisplit(L, nbkt, key, prl, pct, pval, V != nullptr, s_wsum, rl, ct, rval);
    }
}

// One workgroup per coarse bucket: its triplets, sorted into nf = Rc / Rf
// fine buckets (counting sort, tiles multisplit in order), and the fine
// buckets' starts fine_off[cb * nf + j].
// Row range of fine bucket b: coarse bucket cb = b >> fshift uses the first
// 2^(rc - cshift[cb]) of its 2^fshift slots, 2^cshift[cb] rows each; the
// other slots are empty (R = 0).  Without a split (cshift NULL) the fine
// buckets are the coarse ones.
__device__ __forceinline__ void fine_rows(int32_t b, int rc, int fshift, const int32_t *cshift,
                                          int32_t *v0, int32_t *R) {
    const int32_t cb = b >> fshift, j = b & ((1 << fshift) - 1);
    const int rfc = cshift ? cshift[cb] : rc;
    if (j >= (1 << (rc - rfc))) {
        *v0 = cb << rc;
        *R = 0;
        return;
    }
    *v0 = (cb << rc) + (j << rfc);
    *R = 1 << rfc;
}

// One workgroup per coarse bucket: triplets counted per sub-bucket of
// 2^rmin rows, then the bucket's fine size 2^rfc (rmin <= rfc <= rmax) is the
// largest whose fullest fine bucket holds at most SP_CAP triplets (rmin if
// none does); its triplets are split into those fine buckets.
template <int TS, bool HV>
__global__ __launch_bounds__(SPP_THREADS) void k_sp_split(
    int32_t nbkt_c, int32_t nblk, int rc, int rmin, int rmax,
    const int32_t *__restrict__ offs, const int32_t *__restrict__ total_ptr,
    const int32_t *__restrict__ rl, const int2 *__restrict__ ct, const double *__restrict__ rval,
    int32_t *__restrict__ rl2, int2 *__restrict__ ct2, double *__restrict__ rval2,
    int32_t *__restrict__ fine_off, int32_t *__restrict__ cshift) {
    __shared__ int32_t s_wsum[SPP_THREADS / WAVE];
    __shared__ int32_t s_lmax[SP_SPLIT_MAX_SHIFT + 1];
    const int tid = threadIdx.x;
    const int32_t cb = blockIdx.x;
    const int fshift = rc - rmin;
    const int32_t nsub = 1 << fshift;
    constexpr int IPT = TS / SPP_THREADS;
    const TileLds L = tile_lds<TS, HV>(nsub);
    const int64_t total = *total_ptr;
    const int64_t e0 = offs[(int64_t)cb * nblk];
    const int64_t e1 = (cb + 1 < nbkt_c) ? offs[(int64_t)(cb + 1) * nblk] : total;
    for (int j = tid; j < nsub; j += SPP_THREADS) L.cnt[j] = 0;
    if (tid <= SP_SPLIT_MAX_SHIFT) s_lmax[tid] = 0;
    __syncthreads();
    for (int64_t xb = e0 + tid; xb < e1; xb += 8 * SPP_THREADS) {
        int32_t r0[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int64_t x = xb + u * SPP_THREADS;
            r0[u] = x < e1 ? rl[x] : -1;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u)
            if (r0[u] >= 0) atomicAdd(&L.cnt[r0[u] >> rmin], 1);
    }
    __syncthreads();
    block_scan_counts(L.cnt, nsub, s_wsum);   // L.cnt[j]: triplets before sub-bucket j
    const int lmax = rmax - rmin;
    for (int l = 0; l <= lmax; ++l) {
        int32_t mx = 0;
        for (int32_t g = tid; g < (nsub >> l); g += SPP_THREADS)
            mx = max(mx, L.cnt[(g + 1) << l] - L.cnt[g << l]);
#pragma unroll
        for (int o = WAVE / 2; o > 0; o >>= 1) mx = max(mx, __shfl_xor(mx, o, WAVE));
        if ((tid & (WAVE - 1)) == 0 && mx > 0) atomicMax(&s_lmax[l], mx);
    }
    __syncthreads();
    int lb = 0;
    for (int l = lmax; l > 0; --l)
        if (s_lmax[l] <= SP_CAP) {
            lb = l;
            break;
        }
    const int rfc = rmin + lb;
    const int32_t nk = nsub >> lb;
    for (int32_t j = tid; j < nsub; j += SPP_THREADS) {
        const int64_t fb = ((int64_t)cb << fshift) + j;
        if (j < nk) {
            const int32_t st = static_cast<int32_t>(e0 + L.cnt[j << lb]);
            fine_off[fb] = st;
            L.gcur[j] = st;
        } else {
            fine_off[fb] = static_cast<int32_t>(e1);
        }
    }
    if (tid == 0) cshift[cb] = rfc;
    if (cb == nbkt_c - 1 && tid == 0) fine_off[(int64_t)nbkt_c << fshift] = static_cast<int32_t>(total);
    __syncthreads();
    const int32_t fmask = (1 << rfc) - 1;
    // the next tile's loads are issued before this tile's multisplit, so
    // they are in flight while it runs
    int32_t nr[IPT];
    int2 nc[IPT];
    double nv[HV ? IPT : 1];
    auto load = [&](int64_t xb) {
#pragma unroll
        for (int u = 0; u < IPT; ++u) {
            const int64_t x = xb + tid + u * SPP_THREADS;
            nr[u] = x < e1 ? rl[x] : -1;
            nc[u] = x < e1 ? ct[x] : make_int2(0, 0);
            if constexpr (HV) nv[u] = x < e1 ? rval[x] : 0.0;
        }
    };
    if (e0 < e1) load(e0);
    for (int64_t xb = e0; xb < e1; xb += TS) {
        int32_t key[IPT], prl[IPT];
        int2 pct[IPT];
        double pval[IPT];
#pragma unroll
        for (int u = 0; u < IPT; ++u) {
            const int32_t r0 = nr[u];
            key[u] = r0 >= 0 ? (r0 >> rfc) : -1;
            prl[u] = r0 & fmask;
            pct[u] = nc[u];
            if constexpr (HV) pval[u] = nv[u];
            else pval[u] = 0.0;
        }
        if (xb + TS < e1) load(xb + TS);
        tile_multisplit(L, nk, key, prl, pct, pval, HV, s_wsum, rl2, ct2, rval2);
    }
}

__global__ void k_sp_fine_off(int32_t nbkt, int32_t nblk, const int32_t *__restrict__ offs,
                              const int32_t *__restrict__ total_ptr, int32_t *__restrict__ fine_off) {
    const int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (b < nbkt) fine_off[b] = offs[b * nblk];
    if (b == nbkt) fine_off[b] = *total_ptr;
}

__device__ inline int32_t block_scan_sp(int32_t v, int32_t *s_wsum, int32_t *total) {
    const int lane = threadIdx.x & (WAVE - 1), wid = threadIdx.x / WAVE;
    const int32_t incl = wave_inclusive_scan(v);
    if (lane == WAVE - 1) s_wsum[wid] = incl;
    __syncthreads();
    int32_t off = incl - v, tot = 0;
#pragma unroll
    for (int w = 0; w < SP_THREADS / WAVE; ++w) {
        if (w < wid) off += s_wsum[w];
        tot += s_wsum[w];
    }
    __syncthreads();
    *total = tot;
    return off;
}

// The row (inside the bucket) holding bucket position x: the last row start
// <= x (empty rows share their start with the next row).
__device__ __forceinline__ int32_t row_of(const int32_t *s_rs, int32_t R, int32_t x) {
    int32_t lo = 0, hi = R - 1;
    while (lo < hi) {
        const int32_t mid = (lo + hi + 1) >> 1;
        if (s_rs[mid] <= x) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// (column, t) of a triplet as one key whose unsigned order is the (column, t)
// order (t breaks ties, so the order is the stable one).
__device__ __forceinline__ uint64_t sp_key(int32_t c, int32_t t) {
    return ((uint64_t)(uint32_t)c << 32) | (uint32_t)t;
}
__device__ __forceinline__ int32_t key_col(uint64_t k) { return (int32_t)(k >> 32); }
__device__ __forceinline__ int32_t key_t(uint64_t k) { return (int32_t)(uint32_t)k; }

// The rows of one bucket, with the bucket's triplets (grouped by row, row r at
// [s_rs[r], s_rs[r+1])) as keys and values in `key`, `val` (LDS or global
// scratch) at [0, nb), every step parallel over the triplets:
//   1 each triplet's place in its row is the number of smaller keys in the
//     row: perm[s + rank] = its index
//   2 every sorted position writes its triplet's t as the contributor list;
//     a position starts a run (an entry of the CSR row) if it is the first
//     of its row or its column differs from the previous position's; with a
//     contiguous range of positions per thread, a block scan of the threads'
//     run counts gives each run its slot among the bucket's entries, staged
//     at e0 + slot with the sum of the run (ascending t) and the run's first
//     place; rows record their first slot (rowoff), the bucket its entry
//     count (btot)
template <typename KeyT, typename ValT, typename PermT>
__device__ void sp_bucket_rows(int32_t R, int32_t nb, int32_t v0, int32_t m, int64_t e0,
                               const int32_t *s_rs, const KeyT *key, const ValT *val, PermT *perm,
                               bool has_val, int32_t *s_wsum,
                               int32_t *__restrict__ stage_col, double *__restrict__ stage_val,
                               int32_t *__restrict__ stage_cptr, int32_t *__restrict__ contrib,
                               int32_t *__restrict__ rowoff, int32_t *__restrict__ btot,
                               int32_t b) {
    const int tid = threadIdx.x;
    for (int32_t x = tid; x < nb; x += SP_THREADS) {
        const int32_t r = row_of(s_rs, R, x);
        const int32_t s = s_rs[r], e = s_rs[r + 1];
        const uint64_t kx = key[x];
        int32_t rank = 0, j = s;
        for (; j + 4 <= e; j += 4) {
            const uint64_t k0 = key[j], k1 = key[j + 1], k2 = key[j + 2], k3 = key[j + 3];
            rank += (k0 < kx ? 1 : 0) + (k1 < kx ? 1 : 0) + (k2 < kx ? 1 : 0) + (k3 < kx ? 1 : 0);
        }
        for (; j < e; ++j) rank += key[j] < kx ? 1 : 0;
        perm[s + rank] = static_cast<PermT>(x);
    }
    __syncthreads();
    // the contributor list, in sorted order (coalesced)
    if (contrib)
        for (int32_t y = tid; y < nb; y += SP_THREADS) contrib[e0 + y] = key_t(key[perm[y]]);
    // each thread a contiguous range of sorted positions: count its run
    // starts, scan, then stage them
    const int32_t per = (nb + SP_THREADS - 1) / SP_THREADS;
    const int32_t y0 = min(nb, tid * per), y1 = min(nb, y0 + per);
    int32_t nrun = 0;
    if (y0 < y1) {
        int32_t r = row_of(s_rs, R, y0);
        int32_t pc = y0 > s_rs[r] ? key_col(key[perm[y0 - 1]]) : 0;
        for (int32_t y = y0; y < y1; ++y) {
            while (s_rs[r + 1] <= y) ++r;
            const int32_t c = key_col(key[perm[y]]);
            nrun += (y == s_rs[r] || c != pc) ? 1 : 0;
            pc = c;
        }
    }
    int32_t T;
    int32_t slot = block_scan_sp(nrun, s_wsum, &T);
    if (y0 < y1) {
        int32_t r = row_of(s_rs, R, y0);
        int32_t pc = y0 > s_rs[r] ? key_col(key[perm[y0 - 1]]) : 0;
        for (int32_t y = y0; y < y1; ++y) {
            while (s_rs[r + 1] <= y) ++r;
            const int32_t c = key_col(key[perm[y]]);
            const bool rs = y == s_rs[r];
            if (rs) {
                // this row and the empty rows just before it start at slot
                if (v0 + r < m) rowoff[v0 + r] = slot;
                for (int32_t q = r - 1; q >= 0 && s_rs[q] == y; --q)
                    if (v0 + q < m) rowoff[v0 + q] = slot;
            }
            if (rs || c != pc) {
                const int64_t o = e0 + slot;
                stage_col[o] = c;
                if (stage_cptr) stage_cptr[o] = static_cast<int32_t>(e0 + y);
                if (has_val) {
                    const int32_t e = s_rs[r + 1];
                    double acc = static_cast<double>(val[perm[y]]);
                    for (int32_t z = y + 1; z < e && key_col(key[perm[z]]) == c; ++z)
                        acc += static_cast<double>(val[perm[z]]);
                    stage_val[o] = acc;
                }
                ++slot;
            }
            pc = c;
        }
    }
    // rows after the bucket's last triplet (and all rows of an empty bucket)
    for (int32_t r = tid; r < R; r += SP_THREADS)
        if (s_rs[r] == nb && v0 + r < m) rowoff[v0 + r] = T;
    if (tid == 0) btot[b] = T;
}

// One workgroup per fine bucket slot (unused slots return at once); a bucket
// whose triplets fit in LDS is done here, larger ones are listed for
// k_sp_rows_big.
template <bool HV>
__global__ __launch_bounds__(SP_THREADS) void k_sp_rows(
    int32_t m, int32_t nbkt, int rc, int fshift, const int32_t *__restrict__ cshift,
    const int32_t *__restrict__ fine_off, const int32_t *__restrict__ rl,
    const int2 *__restrict__ ct, const double *__restrict__ rval,
    int32_t *__restrict__ stage_col,
    double *__restrict__ stage_val, int32_t *__restrict__ stage_cptr, int32_t *__restrict__ contrib,
    int32_t *__restrict__ rowoff, int32_t *__restrict__ btot, int32_t *__restrict__ big,
    SparseCounters *cnt) {
    __shared__ uint64_t s_key[SP_CAP];
    __shared__ double s_val[HV ? SP_CAP : 1];
    __shared__ uint16_t s_perm[SP_CAP];
    __shared__ int32_t s_rs[(1 << SP_RMAX_SHIFT) + 1];
    __shared__ int32_t s_len[1 << SP_RMAX_SHIFT];
    __shared__ int32_t s_wsum[SP_THREADS / WAVE];
    const int tid = threadIdx.x;
    const int32_t b = blockIdx.x;
    int32_t mxrow = 0;
    {
        int32_t v0, R;
        fine_rows(b, rc, fshift, cshift, &v0, &R);
        if (R == 0) {   // an unused slot of its coarse bucket
            if (tid == 0) btot[b] = 0;
            return;
        }
        const int64_t e0 = fine_off[b], e1 = fine_off[b + 1];
        const int32_t nb = static_cast<int32_t>(e1 - e0);
        if (e1 - e0 > SP_CAP) {
            if (tid == 0) big[atomicAdd(&cnt->big_count, 1)] = b;
            return;
        }
        // 1 the bucket's triplets into registers (all loads in flight),
        // triplets per row, scan -> row starts
        constexpr int EPT = (SP_CAP + SP_THREADS - 1) / SP_THREADS;
        int32_t xr[EPT];
        int2 xc[EPT];
        double xv[HV ? EPT : 1];
#pragma unroll
        for (int u = 0; u < EPT; ++u) {
            const int32_t x = tid + u * SP_THREADS;
            xr[u] = x < nb ? rl[e0 + x] : -1;
            xc[u] = x < nb ? ct[e0 + x] : make_int2(0, 0);
            if constexpr (HV) xv[u] = x < nb ? rval[e0 + x] : 0.0;
        }
        for (int32_t r = tid; r < R; r += SP_THREADS) s_len[r] = 0;
        __syncthreads();
#pragma unroll
        for (int u = 0; u < EPT; ++u)
            if (xr[u] >= 0) atomicAdd(&s_len[xr[u]], 1);
        __syncthreads();
        const int per = (R + SP_THREADS - 1) / SP_THREADS;
        int32_t mine = 0;
        for (int k = 0; k < per; ++k) {
            const int32_t r = tid * per + k;
            if (r < R) {
                mine += s_len[r];
                mxrow = max(mxrow, s_len[r]);
            }
        }
        int32_t T;
        int32_t run = block_scan_sp(mine, s_wsum, &T);
        for (int k = 0; k < per; ++k) {
            const int32_t r = tid * per + k;
            if (r < R) {
                const int32_t c = s_len[r];
                s_rs[r] = run;
                s_len[r] = run;   // cursor
                run += c;
            }
        }
        if (tid == 0) s_rs[R] = nb;
        __syncthreads();
        // 2 counting sort by row into LDS
#pragma unroll
        for (int u = 0; u < EPT; ++u) {
            if (xr[u] < 0) continue;
            const int32_t p = atomicAdd(&s_len[xr[u]], 1);
            s_key[p] = sp_key(xc[u].x, xc[u].y);
            if constexpr (HV) s_val[p] = xv[u];
        }
        __syncthreads();
        sp_bucket_rows(R, nb, v0, m, e0, s_rs, s_key, s_val, s_perm, HV, s_wsum, stage_col, stage_val,
                       stage_cptr, contrib, rowoff, btot, b);
    }
#pragma unroll
    for (int o = WAVE / 2; o > 0; o >>= 1) mxrow = max(mxrow, __shfl_xor(mxrow, o, WAVE));
    if ((tid & (WAVE - 1)) == 0 && mxrow > 0) max_into_sp(&cnt->max_row, mxrow);
}

// Buckets listed by k_sp_rows (more than SP_CAP triplets): the same steps
// with the triplets in global scratch (gkey, gval, gperm at the bucket's own
// range [e0, e1)).  Slower, for skewed inputs only.
__global__ __launch_bounds__(SP_THREADS) void k_sp_rows_big(
    int32_t m, int rc, int fshift, const int32_t *__restrict__ cshift,
    const int32_t *__restrict__ fine_off, const int32_t *__restrict__ rl,
    const int2 *__restrict__ ct, const double *__restrict__ rval, int has_val,
    uint64_t *__restrict__ gkey, double *__restrict__ gval, int32_t *__restrict__ gperm,
    int32_t *__restrict__ stage_col,
    double *__restrict__ stage_val, int32_t *__restrict__ stage_cptr, int32_t *__restrict__ contrib,
    int32_t *__restrict__ rowoff, int32_t *__restrict__ btot, const int32_t *__restrict__ big,
    SparseCounters *cnt) {
    __shared__ int32_t s_rs[(1 << SP_RMAX_SHIFT) + 1];
    __shared__ int32_t s_len[1 << SP_RMAX_SHIFT];
    __shared__ int32_t s_wsum[SP_THREADS / WAVE];
    const int tid = threadIdx.x;
    const int32_t nbig = cnt->big_count;
    for (int32_t q = blockIdx.x; q < nbig; q += gridDim.x) {
        const int32_t b = big[q];
        const int64_t e0 = fine_off[b], e1 = fine_off[b + 1];
        const int32_t nb = static_cast<int32_t>(e1 - e0);
        int32_t v0, R;
        fine_rows(b, rc, fshift, cshift, &v0, &R);
        for (int32_t r = tid; r < R; r += SP_THREADS) s_len[r] = 0;
        __syncthreads();
        for (int32_t x = tid; x < nb; x += SP_THREADS) atomicAdd(&s_len[rl[e0 + x]], 1);
        __syncthreads();
        const int per = (R + SP_THREADS - 1) / SP_THREADS;
        int32_t mine = 0, mx = 0;
        for (int k = 0; k < per; ++k) {
            const int32_t r = tid * per + k;
            if (r < R) {
                mine += s_len[r];
                mx = max(mx, s_len[r]);
            }
        }
        int32_t T;
        int32_t run = block_scan_sp(mine, s_wsum, &T);
        for (int k = 0; k < per; ++k) {
            const int32_t r = tid * per + k;
            if (r < R) {
                const int32_t c = s_len[r];
                s_rs[r] = run;
                s_len[r] = run;
                run += c;
            }
        }
        if (tid == 0) s_rs[R] = nb;
#pragma unroll
        for (int o = WAVE / 2; o > 0; o >>= 1) mx = max(mx, __shfl_xor(mx, o, WAVE));
        if ((tid & (WAVE - 1)) == 0) max_into_sp(&cnt->max_row, mx);
        __syncthreads();
        uint64_t *bk = gkey + e0;
        double *bv = gval + e0;
        for (int32_t x = tid; x < nb; x += SP_THREADS) {
            const int2 c = ct[e0 + x];
            const int32_t p = atomicAdd(&s_len[rl[e0 + x]], 1);
            bk[p] = sp_key(c.x, c.y);
            if (has_val) bv[p] = rval[e0 + x];
        }
        __syncthreads();
        sp_bucket_rows(R, nb, v0, m, e0, s_rs, bk, bv, gperm + e0, has_val != 0, s_wsum, stage_col,
                       stage_val, stage_cptr, contrib, rowoff, btot, b);
        __syncthreads();
    }
}

// Bucket b's staged rows to col_idx / values / contrib_ptr at bptr[b], and
// row_ptr of its rows (workgroups loop over the slots).
__global__ __launch_bounds__(SP_THREADS) void k_sp_copy(
    int32_t m, int32_t nbkt, int rc, int fshift, const int32_t *__restrict__ cshift,
    const int32_t *__restrict__ fine_off,
    const int32_t *__restrict__ bptr, const int32_t *__restrict__ rowoff,
    const int32_t *__restrict__ stage_col, const double *__restrict__ stage_val,
    const int32_t *__restrict__ stage_cptr, int32_t *__restrict__ row_ptr,
    int32_t *__restrict__ col_idx, double *__restrict__ vals, int32_t *__restrict__ contrib_ptr,
    int64_t col_cap, int64_t nt, SparseCounters *cnt) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        row_ptr[m] = bptr[nbkt];
        if (contrib_ptr && bptr[nbkt] <= col_cap) contrib_ptr[bptr[nbkt]] = static_cast<int32_t>(nt);
    }
    for (int32_t b = blockIdx.x; b < nbkt; b += gridDim.x) {
        int32_t v0, R;
        fine_rows(b, rc, fshift, cshift, &v0, &R);
        if (R == 0) continue;
        const int64_t e0 = fine_off[b];
        const int32_t P = bptr[b], T = bptr[b + 1] - P;
        for (int32_t r = threadIdx.x; r < R; r += SP_THREADS)
            if (v0 + r < m) row_ptr[v0 + r] = P + rowoff[v0 + r];
        if (P + (int64_t)T > col_cap) {
            if (threadIdx.x == 0) atomicOr(&cnt->err, SP_ERR_NOSPC);
            continue;
        }
        constexpr int H = 4;   // entries with their loads in flight per thread
        for (int32_t x0 = threadIdx.x; x0 < T; x0 += H * SP_THREADS) {
            int32_t c[H], cp[H];
            double v[H];
#pragma unroll
            for (int j = 0; j < H; ++j) {
                const int32_t x = x0 + j * SP_THREADS;
                const bool in = x < T;
                c[j] = in ? stage_col[e0 + x] : 0;
                v[j] = (in && vals) ? stage_val[e0 + x] : 0.0;
                cp[j] = (in && contrib_ptr) ? stage_cptr[e0 + x] : 0;
            }
            // streaming stores: the outputs are not read again by this call
#pragma unroll
            for (int j = 0; j < H; ++j) {
                const int32_t x = x0 + j * SP_THREADS;
                if (x >= T) continue;
                __builtin_nontemporal_store(c[j], col_idx + P + x);
                if (vals) __builtin_nontemporal_store(v[j], vals + P + x);
                if (contrib_ptr) __builtin_nontemporal_store(cp[j], contrib_ptr + P + x);
            }
        }
    }
}

// vals[p] = sum of V[contrib[k]] for k in [contrib_ptr[p], contrib_ptr[p+1]),
// in that order (ascending t): one lane per entry.
__global__ __launch_bounds__(256) void k_sp_values(int64_t nnz, const int32_t *__restrict__ cptr,
                                                   const int32_t *__restrict__ contrib,
                                                   const double *__restrict__ V,
                                                   double *__restrict__ vals, int accumulate) {
    const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (p >= nnz) return;
    double acc = 0.0;
    // H contributors at a time, all loads in flight, added in ascending order
    constexpr int H = 4;
    const int32_t k0 = cptr[p], k1 = cptr[p + 1];
    for (int32_t k = k0; k < k1; k += H) {
        int32_t c[H];
#pragma unroll
        for (int j = 0; j < H; ++j) c[j] = k + j < k1 ? contrib[k + j] : -1;
        double x[H];
#pragma unroll
        for (int j = 0; j < H; ++j) x[j] = c[j] >= 0 ? V[c[j]] : 0.0;
#pragma unroll
        for (int j = 0; j < H; ++j)
            if (c[j] >= 0) acc += x[j];
    }
    // a streaming store: nothing reads vals again in this call
    __builtin_nontemporal_store(accumulate ? vals[p] + acc : acc, vals + p);
}

struct SparsePlan {
    int rf, rc;            // log2 rows per fine bucket at the average density / per coarse bucket
    int rmin, rmax;        // log2 rows per fine bucket: the range the split chooses from
    int32_t nbkt_f, nbkt_c, nblk;   // nbkt_f: fine bucket slots, 2^(rc - rmin) per coarse bucket
    int64_t tpb;
    int fshift() const { return rc - rmin; }
    int64_t ncounts() const { return (int64_t)nbkt_c * nblk; }
};

// Fine buckets: a power of two of rows with about SP_CAP / 2 triplets on
// average; coarse buckets: the fewest powers of two of fine buckets that keep
// at most SP_COARSE_MAX of them.
bool plan_sparse(int32_t m, int64_t nt, SparsePlan *p) {
    const double avg = m > 0 ? (double)nt / (double)m : 0.0;
    int rf = 0;
    while (rf < SP_RMAX_SHIFT && avg * (double)(1 << (rf + 1)) <= 0.875 * SP_CAP) ++rf;
    int rc = rf;
    while (rc < 31 && (((int64_t)m + (1ll << rc) - 1) >> rc) > SP_COARSE_TARGET) ++rc;
    // no more than 2^SP_SPLIT_MAX_SHIFT fine buckets per coarse one: fewer,
    // larger coarse buckets beat larger fine ones while the histogram fits
    while (rc - rf > SP_SPLIT_MAX_SHIFT && (((int64_t)m + (1ll << (rc - 1)) - 1) >> (rc - 1)) <= SP_COARSE_MAX)
        --rc;
    if (rc - rf > SP_SPLIT_MAX_SHIFT) rf = rc - SP_SPLIT_MAX_SHIFT;
    if (rf > SP_RMAX_SHIFT) return false;
    int rmin = rf > SP_ADAPT_SHIFT ? rf - SP_ADAPT_SHIFT : 0;
    if (rc - rmin > SP_SPLIT_MAX_SHIFT) rmin = rc - SP_SPLIT_MAX_SHIFT;
    p->rf = rf;
    p->rc = rc;
    p->rmin = rmin;
    p->rmax = rc < SP_RMAX_SHIFT ? rc : SP_RMAX_SHIFT;
    p->nbkt_c = (int32_t)(((int64_t)m + (1ll << rc) - 1) >> rc);
    p->nbkt_f = p->nbkt_c << (rc - rmin);
    int64_t tpb = (nt + SP_NBLK_TARGET - 1) / SP_NBLK_TARGET;
    tpb = (tpb + SPP_THREADS - 1) / SPP_THREADS * SPP_THREADS;
    if (tpb < SPP_THREADS) tpb = SPP_THREADS;
    p->tpb = tpb;
    p->nblk = (int32_t)((nt + tpb - 1) / tpb);
    if (p->nblk < 1) p->nblk = 1;
    return true;
}

struct SparseWork {
    SparseCounters *cnt;
    int32_t *counts, *rl, *rl2, *gperm, *stage_col, *stage_cptr, *rowoff, *btot, *bptr,
        *big, *fine_off, *cshift;
    uint64_t *gkey;
    int2 *ct, *ct2;
    double *rval, *rval2, *gval, *stage_val;
    long long *part;
    size_t bytes;
};

inline size_t align_up(size_t x) { return (x + 255) & ~size_t(255); }

SparseWork carve_sparse(int32_t m, int64_t nt, const SparsePlan &P, char *base) {
    SparseWork w{};
    size_t off = 0;
    auto take = [&](size_t bytes) {
        char *p = base ? base + off : nullptr;
        off += align_up(bytes);
        return p;
    };
    const size_t ntc = (size_t)(nt > 0 ? nt : 1);
    const int64_t nscan = P.ncounts() > P.nbkt_f ? P.ncounts() : P.nbkt_f;
    w.cnt = reinterpret_cast<SparseCounters *>(take(sizeof(SparseCounters)));
    w.counts = reinterpret_cast<int32_t *>(take(sizeof(int32_t) * (size_t)(P.ncounts() + 1)));
    w.part = reinterpret_cast<long long *>(take(sizeof(long long) * (size_t)scan_partials(nscan)));
    w.fine_off = reinterpret_cast<int32_t *>(take(sizeof(int32_t) * (size_t)(P.nbkt_f + 1)));
    w.btot = reinterpret_cast<int32_t *>(take(sizeof(int32_t) * (size_t)(P.nbkt_f + 1)));
    w.bptr = reinterpret_cast<int32_t *>(take(sizeof(int32_t) * (size_t)(P.nbkt_f + 1)));
    w.big = reinterpret_cast<int32_t *>(take(sizeof(int32_t) * (size_t)P.nbkt_f));
    w.cshift = reinterpret_cast<int32_t *>(take(sizeof(int32_t) * (size_t)P.nbkt_c));
    w.rowoff = reinterpret_cast<int32_t *>(take(sizeof(int32_t) * (size_t)(m > 0 ? m : 1)));
    w.rl = reinterpret_cast<int32_t *>(take(sizeof(int32_t) * ntc));
    w.ct = reinterpret_cast<int2 *>(take(sizeof(int2) * ntc));
    w.rval = reinterpret_cast<double *>(take(sizeof(double) * ntc));
    const bool split = P.fshift() > 0;
    w.rl2 = split ? reinterpret_cast<int32_t *>(take(sizeof(int32_t) * ntc)) : w.rl;
    w.ct2 = split ? reinterpret_cast<int2 *>(take(sizeof(int2) * ntc)) : w.ct;
    w.rval2 = split ? reinterpret_cast<double *>(take(sizeof(double) * ntc)) : w.rval;
    w.gkey = reinterpret_cast<uint64_t *>(take(sizeof(uint64_t) * ntc));
    w.gperm = reinterpret_cast<int32_t *>(take(sizeof(int32_t) * ntc));
    w.gval = reinterpret_cast<double *>(take(sizeof(double) * ntc));
    w.stage_col = reinterpret_cast<int32_t *>(take(sizeof(int32_t) * ntc));
    w.stage_cptr = reinterpret_cast<int32_t *>(take(sizeof(int32_t) * ntc));
    w.stage_val = reinterpret_cast<double *>(take(sizeof(double) * ntc));
    w.bytes = off;
    return w;
}

}  // namespace
}  // namespace fem

using namespace fem;

extern "C" int fem_sparse_workspace(int32_t m, int32_t n, int64_t nt, size_t *bytes) {
    clear_error();
    FEM_REQUIRE(bytes != nullptr, FEM_EINVAL, "fem_sparse_workspace: bytes is NULL");
    FEM_REQUIRE(m >= 1 && n >= 1 && nt >= 0, FEM_EINVAL, "fem_sparse_workspace: need m, n >= 1, nt >= 0");
    FEM_REQUIRE(nt <= INT32_MAX, FEM_EOVERFLOW, "fem_sparse_workspace: nt exceeds int32");
    SparsePlan P;
    FEM_REQUIRE(plan_sparse(m, nt, &P), FEM_EUNSUPPORTED, "fem_sparse_workspace: m = %d too large", m);
    *bytes = carve_sparse(m, nt, P, nullptr).bytes;
    return FEM_OK;
}

extern "C" int fem_sparse(int32_t m, int32_t n, int64_t nt, const int32_t *I, const int32_t *J,
                          const double *V, int32_t *row_ptr, int32_t *col_idx, double *vals,
                          int64_t col_cap, int32_t *contrib_ptr, int32_t *contrib, void *work,
                          size_t work_bytes, int64_t *nnz_out, void *stream) {
    clear_error();
    FEM_REQUIRE(m >= 1 && n >= 1 && nt >= 0, FEM_EINVAL, "fem_sparse: need m, n >= 1, nt >= 0");
    FEM_REQUIRE(nt <= INT32_MAX, FEM_EOVERFLOW, "fem_sparse: nt = %lld exceeds int32", (long long)nt);
    FEM_REQUIRE(row_ptr && work && nnz_out, FEM_EINVAL, "fem_sparse: NULL row_ptr, work or nnz_out");
    FEM_REQUIRE(nt == 0 || (I && J), FEM_EINVAL, "fem_sparse: NULL I or J");
    FEM_REQUIRE(!vals || nt == 0 || V, FEM_EINVAL, "fem_sparse: values requested without V");
    FEM_REQUIRE(col_cap >= 0 && (col_cap == 0 || col_idx), FEM_EINVAL,
                "fem_sparse: NULL col_idx or negative col_cap");
    FEM_REQUIRE(!contrib_ptr == !contrib, FEM_EINVAL,
                "fem_sparse: contrib_ptr and contrib go together");
    SparsePlan P;
    FEM_REQUIRE(plan_sparse(m, nt, &P), FEM_EUNSUPPORTED, "fem_sparse: m = %d too large", m);
    const SparseWork W = carve_sparse(m, nt, P, static_cast<char *>(work));
    FEM_REQUIRE(work_bytes >= W.bytes, FEM_ENOSPC, "fem_sparse: workspace of %zu bytes, need %zu",
                work_bytes, W.bytes);
    hipStream_t s = as_stream(stream);
    int st;
    if ((st = fill_i32(reinterpret_cast<int32_t *>(W.cnt), sizeof(SparseCounters) / 4, 0, s))) return st;
    const bool has_val = vals != nullptr;
    const size_t hist_lds = sizeof(int32_t) * (size_t)P.nbkt_c;
    if (nt > 0) {
        hipLaunchKernelGGL(k_sp_count, dim3(P.nblk), dim3(SPP_THREADS), hist_lds, s, nt, I, J, m, n,
                           P.rc, P.nbkt_c, P.tpb, W.counts, W.cnt);
        FEM_LAUNCH_CHECK();
    } else {
        if ((st = fill_i32(W.counts, P.ncounts(), 0, s))) return st;
    }
    if ((st = exclusive_scan_i32(W.counts, W.counts, P.ncounts(), W.part, &W.cnt->total[2],
                                 &W.cnt->err, s)))
        return st;
    if (nt > 0) {
        hipLaunchKernelGGL(k_sp_scatter, dim3(P.nblk), dim3(SPP_THREADS), tile_lds_bytes<TILE>(P.nbkt_c), s,
                           nt, I, J,
                           has_val ? V : nullptr, m, n, P.rc, P.nbkt_c, P.tpb, W.counts, W.rl, W.ct,
                           W.rval);
        FEM_LAUNCH_CHECK();
    }
    const int32_t *total_ptr = W.counts + P.ncounts();
    const int32_t *cshift = P.fshift() > 0 ? W.cshift : nullptr;
    if (P.fshift() > 0) {
        const size_t lds_v = tile_lds_bytes<TILE_SPLIT, true>(1 << P.fshift());
        const size_t lds_nv = tile_lds_bytes<TILE_SPLIT_NV, false>(1 << P.fshift());
        if (has_val)
            hipLaunchKernelGGL((k_sp_split<TILE_SPLIT, true>), dim3(P.nbkt_c), dim3(SPP_THREADS),
                               lds_v, s, P.nbkt_c, P.nblk,
                               P.rc, P.rmin, P.rmax, W.counts, total_ptr, W.rl, W.ct, W.rval, W.rl2,
                               W.ct2, W.rval2, W.fine_off, W.cshift);
        else
            hipLaunchKernelGGL((k_sp_split<TILE_SPLIT_NV, false>), dim3(P.nbkt_c), dim3(SPP_THREADS),
                               lds_nv, s, P.nbkt_c,
                               P.nblk, P.rc, P.rmin, P.rmax, W.counts, total_ptr, W.rl, W.ct, W.rval,
                               W.rl2, W.ct2, W.rval2, W.fine_off, W.cshift);
    } else {
        hipLaunchKernelGGL(k_sp_fine_off, dim3(grid_for((int64_t)P.nbkt_f + 1, 256)), dim3(256), 0, s,
                           P.nbkt_f, P.nblk, W.counts, total_ptr, W.fine_off);
    }
    FEM_LAUNCH_CHECK();
    const unsigned grows = (unsigned)P.nbkt_f;
    if (has_val)
        hipLaunchKernelGGL(k_sp_rows<true>, dim3(grows), dim3(SP_THREADS), 0, s, m, P.nbkt_f, P.rc,
                           P.fshift(), cshift, W.fine_off, W.rl2, W.ct2, W.rval2, W.stage_col,
                           W.stage_val, contrib_ptr ? W.stage_cptr : nullptr, contrib, W.rowoff, W.btot,
                           W.big, W.cnt);
    else
        hipLaunchKernelGGL(k_sp_rows<false>, dim3(grows), dim3(SP_THREADS), 0, s, m, P.nbkt_f, P.rc,
                           P.fshift(), cshift, W.fine_off, W.rl2, W.ct2, W.rval2, W.stage_col,
                           W.stage_val, contrib_ptr ? W.stage_cptr : nullptr, contrib, W.rowoff, W.btot,
                           W.big, W.cnt);
    FEM_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_sp_rows_big, dim3(256), dim3(SP_THREADS), 0, s, m, P.rc, P.fshift(), cshift,
                       W.fine_off, W.rl2,
                       W.ct2, W.rval2, has_val ? 1 : 0, W.gkey, W.gval, W.gperm, W.stage_col, W.stage_val,
                       contrib_ptr ? W.stage_cptr : nullptr, contrib, W.rowoff, W.btot, W.big, W.cnt);
    FEM_LAUNCH_CHECK();
    if ((st = exclusive_scan_i32(W.btot, W.bptr, P.nbkt_f, W.part, &W.cnt->total[1], &W.cnt->err, s)))
        return st;
    const unsigned gcopy = (unsigned)(P.nbkt_f < SP_COPY_GRID ? P.nbkt_f : SP_COPY_GRID);
    hipLaunchKernelGGL(k_sp_copy, dim3(gcopy), dim3(SP_THREADS), 0, s, m, P.nbkt_f, P.rc,
                       P.fshift(), cshift,
                       W.fine_off, W.bptr, W.rowoff, W.stage_col, has_val ? W.stage_val : nullptr,
                       W.stage_cptr, row_ptr, col_idx, vals, contrib_ptr, col_cap, nt, W.cnt);
    FEM_LAUNCH_CHECK();
    SparseCounters h{};
    FEM_HIP_CHECK(hipMemcpyAsync(&h, W.cnt, sizeof(h), hipMemcpyDeviceToHost, s));
    FEM_HIP_CHECK(hipStreamSynchronize(s));
    FEM_REQUIRE(!(h.err & SP_ERR_RANGE), FEM_ERANGE,
                "fem_sparse: an index of I is outside [0, %d) or of J outside [0, %d)", m, n);
    FEM_REQUIRE(!(h.err & SP_ERR_OVERFLOW), FEM_EOVERFLOW, "fem_sparse: count overflow");
    const int64_t nnz = h.total[1];
    FEM_REQUIRE(!(h.err & SP_ERR_NOSPC) && nnz <= col_cap, FEM_ENOSPC,
                "fem_sparse: nnz = %lld exceeds col_cap = %lld", (long long)nnz, (long long)col_cap);
    *nnz_out = nnz;
    return FEM_OK;
}

extern "C" int fem_sparse_values(int64_t nnz, const int32_t *contrib_ptr, const int32_t *contrib,
                                 const double *V, double *vals, int flags, void *stream) {
    clear_error();
    FEM_REQUIRE(nnz >= 0 && nnz <= INT32_MAX, FEM_EINVAL, "fem_sparse_values: bad nnz");
    FEM_REQUIRE((flags & ~FEM_ACCUMULATE) == 0, FEM_EINVAL,
                "fem_sparse_values: only FEM_ACCUMULATE is supported");
    FEM_REQUIRE(contrib_ptr && (nnz == 0 || (contrib && V && vals)), FEM_EINVAL,
                "fem_sparse_values: NULL array");
    if (nnz == 0) return FEM_OK;
    hipLaunchKernelGGL(k_sp_values, dim3(grid_for(nnz, 256)), dim3(256), 0, as_stream(stream), nnz,
                       contrib_ptr, contrib, V, vals, (flags & FEM_ACCUMULATE) ? 1 : 0);
    FEM_LAUNCH_CHECK();
    return FEM_OK;
}
