// fem_sparse.hip -- general sparse(I, J, V, m, n): triplets with duplicates
// summed into CSR (rows ascending, columns ascending, structural zeros kept),
// the compression every OptV2 assembly ends in (Section 4 for the storage,
// Section 6 for the triplet arrays Ig, Jg, Kg).
//
// Bucketed by row, no global atomics:
//   k_sp_count / scan / k_sp_scatter   triplets -> runs of (bucket, workgroup):
//                                      (row mod R, column, t) + value
//   k_sp_rows (LDS) / k_sp_rows_big    one workgroup per bucket of R rows:
//                                      counting sort by row, then each row
//                                      sorted by (column, t), duplicates
//                                      summed in ascending t; rows staged per
//                                      bucket, sorted triplet order written as
//                                      the contributor list
//   scan of bucket totals / k_sp_copy  rows -> col_idx / values, row_ptr
// Every value is the sum of its triplets' values in ascending t, so the result
// is bitwise reproducible and equal to a sequential left-to-right sum.

#include "fem_internal.h"

namespace fem {

namespace {

constexpr int SP_THREADS = 256;
constexpr int SP_CAP = 3072;          // triplets of a bucket held in LDS (3 workgroups / CU)
constexpr int SP_RMAX_SHIFT = 9;      // at most 512 rows per bucket
constexpr int SP_HIST_MAX = 36864;    // buckets an LDS histogram holds
constexpr int SP_NBLK_TARGET = 256;   // triplet workgroups of the partition pass

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

// counts[b * nblk + blk]: triplets of workgroup blk (tpb triplets) in bucket b
__global__ __launch_bounds__(SP_THREADS) void k_sp_count(int64_t nt, const int32_t *__restrict__ I,
                                                        const int32_t *__restrict__ J, int32_t m,
                                                        int32_t n, int rs, int32_t nbkt, int64_t tpb,
                                                        int32_t *__restrict__ counts,
                                                        SparseCounters *cnt) {
    extern __shared__ int32_t s_hist[];
    const int32_t nblk = gridDim.x;
    for (int b = threadIdx.x; b < nbkt; b += SP_THREADS) s_hist[b] = 0;
    __syncthreads();
    const int64_t t0 = (int64_t)blockIdx.x * tpb;
    const int64_t t1 = (t0 + tpb < nt) ? t0 + tpb : nt;
    int bad = 0;
    for (int64_t t = t0 + threadIdx.x; t < t1; t += SP_THREADS) {
        const int32_t i = I[t], j = J[t];
        if ((uint32_t)i >= (uint32_t)m || (uint32_t)j >= (uint32_t)n) {
            bad = 1;
            continue;
        }
        atomicAdd(&s_hist[i >> rs], 1);
    }
    if (bad) atomicOr(&cnt->err, SP_ERR_RANGE);
    __syncthreads();
    for (int b = threadIdx.x; b < nbkt; b += SP_THREADS)
        counts[(int64_t)b * nblk + blockIdx.x] = s_hist[b];
}

// Same triplets per workgroup as k_sp_count: each goes to the run of its
// (bucket, workgroup) pair: rec = (row mod R, column, t), val = V[t].
__global__ __launch_bounds__(SP_THREADS) void k_sp_scatter(int64_t nt, const int32_t *__restrict__ I,
                                                          const int32_t *__restrict__ J,
                                                          const double *__restrict__ V, int32_t m,
                                                          int32_t n, int rs, int32_t nbkt, int64_t tpb,
                                                          const int32_t *__restrict__ offs,
                                                          int32_t *__restrict__ rec,
                                                          double *__restrict__ rval) {
    extern __shared__ int32_t s_cur[];
    const int32_t nblk = gridDim.x;
    for (int b = threadIdx.x; b < nbkt; b += SP_THREADS)
        s_cur[b] = offs[(int64_t)b * nblk + blockIdx.x];
    __syncthreads();
    const int64_t t0 = (int64_t)blockIdx.x * tpb;
    const int64_t t1 = (t0 + tpb < nt) ? t0 + tpb : nt;
    const int32_t rmask = (1 << rs) - 1;
    for (int64_t t = t0 + threadIdx.x; t < t1; t += SP_THREADS) {
        const int32_t i = I[t], j = J[t];
        if ((uint32_t)i >= (uint32_t)m || (uint32_t)j >= (uint32_t)n) continue;
        const int32_t pos = atomicAdd(&s_cur[i >> rs], 1);
        int32_t *r = rec + 3 * (int64_t)pos;
        r[0] = i & rmask;
        r[1] = j;
        r[2] = static_cast<int32_t>(t);
        if (V) rval[pos] = V[t];
    }
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

// The rows of one bucket, with the bucket's triplets (sorted by row) in
// arrays `col`, `tt`, `val` (LDS or global scratch) at [0, nb):
//   1 each row sorted by (column, t) (insertion sort; t breaks ties, so the
//     order is the stable one)
//   2 unique columns -> row lengths; scan -> offsets inside the bucket
//   3 each row's unique columns, the sums of their runs (ascending t) and the
//     start of each run in the sorted triplet order, staged at e0 + offset
// Rows are taken by the threads in turn (thread r: rows r, r + 256, ...).
template <typename ColT, typename ValT>
__device__ void sp_bucket_rows(int32_t R, int32_t v0, int32_t m, int64_t e0, const int32_t *s_rs,
                               ColT *col, ColT *tt, ValT *val, bool has_val, int32_t *s_len,
                               int32_t *s_wsum, int32_t *__restrict__ stage_col,
                               double *__restrict__ stage_val, int32_t *__restrict__ stage_cptr,
                               int32_t *__restrict__ rowoff, int32_t *__restrict__ btot, int32_t b) {
    const int tid = threadIdx.x;
    for (int32_t r = tid; r < R; r += SP_THREADS) {
        const int32_t s = s_rs[r], e = s_rs[r + 1];
        for (int32_t x = s + 1; x < e; ++x) {
            const int32_t c = col[x], t = tt[x];
            double vx = has_val ? static_cast<double>(val[x]) : 0.0;
            int32_t y = x;
            while (y > s && (col[y - 1] > c || (col[y - 1] == c && tt[y - 1] > t))) {
                col[y] = col[y - 1];
                tt[y] = tt[y - 1];
                if (has_val) val[y] = val[y - 1];
                --y;
            }
            col[y] = c;
            tt[y] = t;
            if (has_val) val[y] = vx;
        }
        int32_t L = 0;
        for (int32_t x = s; x < e; ++x) L += (x == s || col[x] != col[x - 1]) ? 1 : 0;
        s_len[r] = L;
    }
    __syncthreads();
    // offsets of the rows inside the bucket (R / 256 rows per thread, in order)
    const int per = (R + SP_THREADS - 1) / SP_THREADS;
    int32_t mine = 0;
    for (int k = 0; k < per; ++k) {
        const int32_t r = tid * per + k;
        if (r < R) mine += s_len[r];
    }
    int32_t T;
    int32_t run = block_scan_sp(mine, s_wsum, &T);
    for (int k = 0; k < per; ++k) {
        const int32_t r = tid * per + k;
        if (r < R) {
            const int32_t L = s_len[r];
            s_len[r] = run;   // now the row's offset inside the bucket
            if (v0 + r < m) rowoff[v0 + r] = run;
            run += L;
        }
    }
    if (tid == 0) btot[b] = T;
    __syncthreads();
    for (int32_t r = tid; r < R; r += SP_THREADS) {
        const int32_t s = s_rs[r], e = s_rs[r + 1];
        int64_t o = e0 + s_len[r];
        for (int32_t x = s; x < e;) {
            const int32_t c = col[x];
            double acc = 0.0;
            int32_t y = x;
            for (; y < e && col[y] == c; ++y)
                if (has_val) acc += static_cast<double>(val[y]);
            stage_col[o] = c;
            if (has_val) stage_val[o] = acc;
            if (stage_cptr) stage_cptr[o] = static_cast<int32_t>(e0 + x);
            ++o;
            x = y;
        }
    }
}

// One workgroup per bucket whose triplets fit in LDS; larger buckets are
// listed for k_sp_rows_big.
__global__ __launch_bounds__(SP_THREADS) void k_sp_rows(
    int32_t m, int32_t nbkt, int32_t nblk, int rs, const int32_t *__restrict__ offs,
    const int32_t *__restrict__ total_ptr, const int32_t *__restrict__ rec,
    const double *__restrict__ rval, int has_val, int32_t *__restrict__ stage_col,
    double *__restrict__ stage_val, int32_t *__restrict__ stage_cptr, int32_t *__restrict__ contrib,
    int32_t *__restrict__ rowoff, int32_t *__restrict__ btot, int32_t *__restrict__ big,
    SparseCounters *cnt) {
    __shared__ int32_t s_col[SP_CAP], s_t[SP_CAP];
    __shared__ double s_val[SP_CAP];
    __shared__ int32_t s_rs[(1 << SP_RMAX_SHIFT) + 1];
    __shared__ int32_t s_len[1 << SP_RMAX_SHIFT];
    __shared__ int32_t s_wsum[SP_THREADS / WAVE];
    const int tid = threadIdx.x;
    const int32_t b = blockIdx.x;
    const int32_t R = 1 << rs;
    const int64_t total = *total_ptr;
    const int64_t e0 = offs[(int64_t)b * nblk];
    const int64_t e1 = (b + 1 < nbkt) ? offs[(int64_t)(b + 1) * nblk] : total;
    const int32_t nb = static_cast<int32_t>(e1 - e0);
    if (e1 - e0 > SP_CAP) {
        if (tid == 0) big[atomicAdd(&cnt->big_count, 1)] = b;
        return;
    }
    const int32_t v0 = b << rs;
    // 1 triplets per row, scan -> row starts
    for (int32_t r = tid; r < R; r += SP_THREADS) s_len[r] = 0;
    __syncthreads();
    for (int32_t x = tid; x < nb; x += SP_THREADS) atomicAdd(&s_len[rec[3 * (e0 + x)]], 1);
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
            s_len[r] = run;   // cursor
            run += c;
        }
    }
    if (tid == 0) s_rs[R] = nb;
#pragma unroll
    for (int o = WAVE / 2; o > 0; o >>= 1) mx = max(mx, __shfl_xor(mx, o, WAVE));
    if ((tid & (WAVE - 1)) == 0) max_into_sp(&cnt->max_row, mx);
    __syncthreads();
    // 2 counting sort by row into LDS
    for (int32_t x = tid; x < nb; x += SP_THREADS) {
        const int32_t *rr = rec + 3 * (e0 + x);
        const int32_t p = atomicAdd(&s_len[rr[0]], 1);
        s_col[p] = rr[1];
        s_t[p] = rr[2];
        if (has_val) s_val[p] = rval[e0 + x];
    }
    __syncthreads();
    sp_bucket_rows(R, v0, m, e0, s_rs, s_col, s_t, s_val, has_val != 0, s_len, s_wsum, stage_col,
                   stage_val, stage_cptr, rowoff, btot, b);
    // the sorted triplet order of the bucket = its part of the contributor list
    if (contrib) {
        __syncthreads();
        for (int32_t x = tid; x < nb; x += SP_THREADS) contrib[e0 + x] = s_t[x];
    }
}

// Buckets listed by k_sp_rows (more than SP_CAP triplets): the same steps
// with the triplets in global scratch (gcol, gt, gval at the bucket's own
// range [e0, e1)).  Slower, for skewed inputs only.
__global__ __launch_bounds__(SP_THREADS) void k_sp_rows_big(
    int32_t m, int32_t nbkt, int32_t nblk, int rs, const int32_t *__restrict__ offs,
    const int32_t *__restrict__ total_ptr, const int32_t *__restrict__ rec,
    const double *__restrict__ rval, int has_val, int32_t *__restrict__ gcol,
    int32_t *__restrict__ gt, double *__restrict__ gval, int32_t *__restrict__ stage_col,
    double *__restrict__ stage_val, int32_t *__restrict__ stage_cptr, int32_t *__restrict__ contrib,
    int32_t *__restrict__ rowoff, int32_t *__restrict__ btot, const int32_t *__restrict__ big,
    SparseCounters *cnt) {
    __shared__ int32_t s_rs[(1 << SP_RMAX_SHIFT) + 1];
    __shared__ int32_t s_len[1 << SP_RMAX_SHIFT];
    __shared__ int32_t s_wsum[SP_THREADS / WAVE];
    const int tid = threadIdx.x;
    const int32_t nbig = cnt->big_count;
    const int32_t R = 1 << rs;
    const int64_t total = *total_ptr;
    for (int32_t q = blockIdx.x; q < nbig; q += gridDim.x) {
        const int32_t b = big[q];
        const int64_t e0 = offs[(int64_t)b * nblk];
        const int64_t e1 = (b + 1 < nbkt) ? offs[(int64_t)(b + 1) * nblk] : total;
        const int32_t nb = static_cast<int32_t>(e1 - e0);
        const int32_t v0 = b << rs;
        for (int32_t r = tid; r < R; r += SP_THREADS) s_len[r] = 0;
        __syncthreads();
        for (int32_t x = tid; x < nb; x += SP_THREADS) atomicAdd(&s_len[rec[3 * (e0 + x)]], 1);
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
        int32_t *bc = gcol + e0;
        int32_t *bt = gt + e0;
        double *bv = gval + e0;
        for (int32_t x = tid; x < nb; x += SP_THREADS) {
            const int32_t *rr = rec + 3 * (e0 + x);
            const int32_t p = atomicAdd(&s_len[rr[0]], 1);
            bc[p] = rr[1];
            bt[p] = rr[2];
            if (has_val) bv[p] = rval[e0 + x];
        }
        __syncthreads();
        sp_bucket_rows(R, v0, m, e0, s_rs, bc, bt, bv, has_val != 0, s_len, s_wsum, stage_col,
                       stage_val, stage_cptr, rowoff, btot, b);
        __syncthreads();
        if (contrib)
            for (int32_t x = tid; x < nb; x += SP_THREADS) contrib[e0 + x] = bt[x];
        __syncthreads();
    }
}

// Bucket b's staged rows to col_idx / values / contrib_ptr at bptr[b], and
// row_ptr of its rows.
__global__ __launch_bounds__(SP_THREADS) void k_sp_copy(
    int32_t m, int32_t nbkt, int32_t nblk, int rs, const int32_t *__restrict__ offs,
    const int32_t *__restrict__ bptr, const int32_t *__restrict__ rowoff,
    const int32_t *__restrict__ stage_col, const double *__restrict__ stage_val,
    const int32_t *__restrict__ stage_cptr, int32_t *__restrict__ row_ptr,
    int32_t *__restrict__ col_idx, double *__restrict__ vals, int32_t *__restrict__ contrib_ptr,
    int64_t col_cap, int64_t nt, SparseCounters *cnt) {
    const int32_t b = blockIdx.x;
    const int64_t e0 = offs[(int64_t)b * nblk];
    const int32_t v0 = b << rs, R = 1 << rs;
    const int32_t P = bptr[b], T = bptr[b + 1] - P;
    for (int32_t r = threadIdx.x; r < R; r += SP_THREADS)
        if (v0 + r < m) row_ptr[v0 + r] = P + rowoff[v0 + r];
    if (b == nbkt - 1 && threadIdx.x == 0) {
        row_ptr[m] = bptr[nbkt];
        if (contrib_ptr && bptr[nbkt] <= col_cap) contrib_ptr[bptr[nbkt]] = static_cast<int32_t>(nt);
    }
    if (P + (int64_t)T > col_cap) {
        if (threadIdx.x == 0) atomicOr(&cnt->err, SP_ERR_NOSPC);
        return;
    }
    for (int32_t x = threadIdx.x; x < T; x += SP_THREADS) {
        col_idx[P + x] = stage_col[e0 + x];
        if (vals) vals[P + x] = stage_val[e0 + x];
        if (contrib_ptr) contrib_ptr[P + x] = stage_cptr[e0 + x];
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
    for (int32_t k = cptr[p]; k < cptr[p + 1]; ++k) acc += V[contrib[k]];
    if (accumulate) vals[p] += acc;
    else vals[p] = acc;
}

struct SparsePlan {
    int rs;                // log2 rows per bucket
    int32_t nbkt, nblk;
    int64_t tpb;
    int64_t ncounts() const { return (int64_t)nbkt * nblk; }
};

// Rows per bucket: a power of two with about SP_CAP / 2 triplets per bucket
// on average, at least enough that the buckets fit an LDS histogram.
bool plan_sparse(int32_t m, int64_t nt, SparsePlan *p) {
    int rs = 0;
    while (rs < SP_RMAX_SHIFT && ((int64_t)m + (1ll << rs) - 1) >> rs > SP_HIST_MAX) ++rs;
    if (((int64_t)m + (1ll << rs) - 1) >> rs > SP_HIST_MAX) return false;
    const double avg = m > 0 ? (double)nt / (double)m : 0.0;
    int rs_fit = 0;
    while (rs_fit < SP_RMAX_SHIFT && avg * (double)(1 << (rs_fit + 1)) <= SP_CAP / 2) ++rs_fit;
    if (rs_fit > SP_RMAX_SHIFT) rs_fit = SP_RMAX_SHIFT;
    p->rs = rs > rs_fit ? rs : rs_fit;
    p->nbkt = (int32_t)(((int64_t)m + (1ll << p->rs) - 1) >> p->rs);
    int64_t tpb = (nt + SP_NBLK_TARGET - 1) / SP_NBLK_TARGET;
    tpb = (tpb + SP_THREADS - 1) / SP_THREADS * SP_THREADS;
    if (tpb < SP_THREADS) tpb = SP_THREADS;
    p->tpb = tpb;
    p->nblk = (int32_t)((nt + tpb - 1) / tpb);
    if (p->nblk < 1) p->nblk = 1;
    return true;
}

struct SparseWork {
    SparseCounters *cnt;
    int32_t *counts, *rec, *gcol, *gt, *stage_col, *stage_cptr, *rowoff, *btot, *bptr, *big;
    double *rval, *gval, *stage_val;
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
    const int64_t nscan = P.ncounts() > P.nbkt ? P.ncounts() : P.nbkt;
    w.cnt = reinterpret_cast<SparseCounters *>(take(sizeof(SparseCounters)));
    w.counts = reinterpret_cast<int32_t *>(take(sizeof(int32_t) * (size_t)(P.ncounts() + 1)));
    w.part = reinterpret_cast<long long *>(take(sizeof(long long) * (size_t)scan_partials(nscan)));
    w.btot = reinterpret_cast<int32_t *>(take(sizeof(int32_t) * (size_t)(P.nbkt + 1)));
    w.bptr = reinterpret_cast<int32_t *>(take(sizeof(int32_t) * (size_t)(P.nbkt + 1)));
    w.big = reinterpret_cast<int32_t *>(take(sizeof(int32_t) * (size_t)P.nbkt));
    w.rowoff = reinterpret_cast<int32_t *>(take(sizeof(int32_t) * (size_t)(m > 0 ? m : 1)));
    w.rec = reinterpret_cast<int32_t *>(take(3 * sizeof(int32_t) * ntc));
    w.rval = reinterpret_cast<double *>(take(sizeof(double) * ntc));
    w.gcol = reinterpret_cast<int32_t *>(take(sizeof(int32_t) * ntc));
    w.gt = reinterpret_cast<int32_t *>(take(sizeof(int32_t) * ntc));
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
    const size_t hist_lds = sizeof(int32_t) * (size_t)P.nbkt;
    if (nt > 0) {
        hipLaunchKernelGGL(k_sp_count, dim3(P.nblk), dim3(SP_THREADS), hist_lds, s, nt, I, J, m, n,
                           P.rs, P.nbkt, P.tpb, W.counts, W.cnt);
        FEM_LAUNCH_CHECK();
    } else {
        if ((st = fill_i32(W.counts, P.ncounts(), 0, s))) return st;
    }
    if ((st = exclusive_scan_i32(W.counts, W.counts, P.ncounts(), W.part, &W.cnt->total[2],
                                 &W.cnt->err, s)))
        return st;
    if (nt > 0) {
        hipLaunchKernelGGL(k_sp_scatter, dim3(P.nblk), dim3(SP_THREADS), hist_lds, s, nt, I, J,
                           has_val ? V : nullptr, m, n, P.rs, P.nbkt, P.tpb, W.counts, W.rec, W.rval);
        FEM_LAUNCH_CHECK();
    }
    const int32_t *total_ptr = W.counts + P.ncounts();
    hipLaunchKernelGGL(k_sp_rows, dim3(P.nbkt), dim3(SP_THREADS), 0, s, m, P.nbkt, P.nblk, P.rs,
                       W.counts, total_ptr, W.rec, W.rval, has_val ? 1 : 0, W.stage_col, W.stage_val,
                       contrib_ptr ? W.stage_cptr : nullptr, contrib, W.rowoff, W.btot, W.big, W.cnt);
    FEM_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_sp_rows_big, dim3(256), dim3(SP_THREADS), 0, s, m, P.nbkt, P.nblk, P.rs,
                       W.counts, total_ptr, W.rec, W.rval, has_val ? 1 : 0, W.gcol, W.gt, W.gval,
                       W.stage_col, W.stage_val, contrib_ptr ? W.stage_cptr : nullptr, contrib,
                       W.rowoff, W.btot, W.big, W.cnt);
    FEM_LAUNCH_CHECK();
    if ((st = exclusive_scan_i32(W.btot, W.bptr, P.nbkt, W.part, &W.cnt->total[1], &W.cnt->err, s)))
        return st;
    hipLaunchKernelGGL(k_sp_copy, dim3(P.nbkt), dim3(SP_THREADS), 0, s, m, P.nbkt, P.nblk, P.rs,
                       W.counts, W.bptr, W.rowoff, W.stage_col, has_val ? W.stage_val : nullptr,
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
