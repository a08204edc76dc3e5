// fem_tet.hip -- P1 tetrahedra in 3D (the extension the Conclusion names):
// mass and stiffness matrices, assembled the OptV2 way on the GPU.
//
//   fem_tet_pattern    the index arrays Ig, Jg of all 16 local entries (triplet
//                      t = r nme + k for entry r = 4 b + a of element k: row
//                      me[k][a], column me[k][b]) compressed by fem_sparse into
//                      the CSR pattern and the contributor lists (the triplets
//                      of each entry, ascending)
//   fem_tet_assemble   k_tet_elem: one lane per tetrahedron writes what its
//                      element matrices hold (the paper's Kg, reduced to the
//                      mass factor and the 10 distinct stiffness entries);
//                      k_tet_sum: one lane per CSR entry adds its contributors
//                      in ascending t (bitwise reproducible)
//
// Element matrices, for K = (x0, x1, x2, x3), e_i = x_i - x0, D = det[e1 e2 e3]:
// the rows of J^{-1} = [e1 e2 e3]^{-1} are c1 / D, c2 / D, c3 / D with
// c1 = e2 x e3, c2 = e3 x e1, c3 = e1 x e2, so grad lambda_a = c_a / D with
// c0 = -(c1 + c2 + c3), and with |K| = |D| / 6
//   stiffness  S_ab = |K| grad lambda_a . grad lambda_b = c_a . c_b / (6 |D|)
//   mass       M_ab = |K| (1 + delta_ab) / 20 = |D| (1 + delta_ab) / 120

#include "fem_internal.h"

extern "C" int fem_sparse_workspace(int32_t m, int32_t n, int64_t nt, size_t *bytes);
extern "C" int fem_sparse(int32_t m, int32_t n, int64_t nt, const int32_t *I, const int32_t *J,
                          const double *V, int32_t *row_ptr, int32_t *col_idx, double *vals,
                          int64_t col_cap, int32_t *contrib_ptr, int32_t *contrib, void *work,
                          size_t work_bytes, int64_t *nnz_out, void *stream);

namespace fem {
namespace {

enum : int { TET_ERR_RANGE = 1, TET_ERR_DEGEN = 2 };
constexpr int TET_M = 1, TET_S = 4;   // FEM_OP_MASS, FEM_OP_STIFF

inline size_t align_up(size_t x) { return (x + 255) & ~size_t(255); }

// Ig / Jg of element k (one lane per element; writes for a fixed entry r are
// coalesced across lanes).  Invalid elements are reported and contribute
// vertex 0 so that the compression still runs in bounds.
__global__ __launch_bounds__(256) void k_tet_triplets(int32_t nme, const int32_t *__restrict__ me,
                                                      int32_t nq, int32_t *__restrict__ I,
                                                      int32_t *__restrict__ J, int *err) {
    const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (k >= nme) return;
    const int4 t = reinterpret_cast<const int4 *>(me)[k];
    int v[4] = {t.x, t.y, t.z, t.w};
    int bad = 0;
#pragma unroll
    for (int a = 0; a < 4; ++a)
        if ((uint32_t)v[a] >= (uint32_t)nq) bad |= TET_ERR_RANGE;
    if (!bad && (v[0] == v[1] || v[0] == v[2] || v[0] == v[3] || v[1] == v[2] || v[1] == v[3] ||
                 v[2] == v[3]))
        bad |= TET_ERR_DEGEN;
    if (bad) {
        atomicOr(err, bad);
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

__device__ __forceinline__ void cross3(const double *u, const double *w, double *o) {
    o[0] = u[1] * w[2] - u[2] * w[1];
    o[1] = u[2] * w[0] - u[0] * w[2];
    o[2] = u[0] * w[1] - u[1] * w[0];
}

// Record of element k: |K| / 20 = |D| / 120 (the mass is that times 1 + delta_ab)
// and / or the 10 distinct entries of the symmetric stiffness, a <= b, at
// 1 + sym(a, b) (or sym(a, b) without the mass).  c_a . c_b is summed over the
// components in the same order for (a, b) and (b, a), so the two are equal
// bit for bit and one of them stands for both.
template <int MASK>
struct TetRec {
    static constexpr int M = (MASK & TET_M) ? 1 : 0;
    static constexpr int N = M + ((MASK & TET_S) ? 10 : 0);   // doubles per element
};

__host__ __device__ constexpr int tet_sym(int i, int j) { return i * (7 - i) / 2 + j; }   // i <= j

template <int MASK>
__global__ __launch_bounds__(256) void k_tet_elem(int32_t nme, const double *__restrict__ q,
                                                  const int32_t *__restrict__ me,
                                                  double *__restrict__ kg) {
    using R = TetRec<MASK>;
    const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (k >= nme) return;
    const int4 t = reinterpret_cast<const int4 *>(me)[k];
    const int v[4] = {t.x, t.y, t.z, t.w};
    double x[4][3];
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        x[a][0] = q[3 * (int64_t)v[a]];
        x[a][1] = q[3 * (int64_t)v[a] + 1];
        x[a][2] = q[3 * (int64_t)v[a] + 2];
    }
    double e[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int c = 0; c < 3; ++c) e[i][c] = x[i + 1][c] - x[0][c];
    double cv[4][3];
    cross3(e[1], e[2], cv[1]);
    cross3(e[2], e[0], cv[2]);
    cross3(e[0], e[1], cv[3]);
#pragma unroll
    for (int c = 0; c < 3; ++c) cv[0][c] = -(cv[1][c] + cv[2][c] + cv[3][c]);
    const double D = e[0][0] * cv[1][0] + e[0][1] * cv[1][1] + e[0][2] * cv[1][2];
    const double aD = fabs(D);
    double *rec = kg + R::N * k;
    if constexpr (R::M) rec[0] = aD / 120.0;
    if constexpr ((MASK & TET_S) != 0) {
        const double s6 = 1.0 / (6.0 * aD);
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = a; b < 4; ++b)
                rec[R::M + tet_sym(a, b)] =
                    (cv[a][0] * cv[b][0] + cv[a][1] * cv[b][1] + cv[a][2] * cv[b][2]) * s6;
    }
}

// One lane per CSR entry: the sum of its contributors in ascending t; the
// contributor t = r nme + k (r = 4 b + a) is element k's entry (a, b).
template <int MASK>
__global__ __launch_bounds__(256) void k_tet_sum(int64_t nnz, const int32_t *__restrict__ cptr,
                                                 const int32_t *__restrict__ contrib, int32_t nme,
                                                 double inv_nme, const double *__restrict__ kg,
                                                 double *__restrict__ vm, double *__restrict__ vs,
                                                 int accumulate) {
    using R = TetRec<MASK>;
    const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (p >= nnz) return;
    const uint32_t ntr = 16u * (uint32_t)nme;
    double am = 0.0, as = 0.0;
    const int32_t k0 = cptr[p], k1 = cptr[p + 1];
    // H contributors at a time: their triplet ids, then the record values
    // they read, all loads in flight; the terms are then added in ascending
    // order, as one at a time would
    constexpr int H = 8;
    for (int32_t k = k0; k < k1; k += H) {
        int32_t tc[H];
#pragma unroll
        for (int j = 0; j < H; ++j) tc[j] = k + j < k1 ? contrib[k + j] : -1;
        bool ok[H], diag[H];
        double xm[H], xs[H];
#pragma unroll
        for (int j = 0; j < H; ++j) {
            // past the list, or not a triplet of these nme elements
            ok[j] = (uint32_t)tc[j] < ntr;
            diag[j] = false;
            xm[j] = xs[j] = 0.0;
            if (!ok[j]) continue;
            // r = tc / nme: the double quotient is off by at most one
            int32_t rq = (int32_t)((double)tc[j] * inv_nme);
            int32_t e = tc[j] - rq * nme;
            if (e < 0) {
                --rq;
                e += nme;
            } else if (e >= nme) {
                ++rq;
                e -= nme;
            }
            const int a = rq & 3, b = rq >> 2;
            const double *rec = kg + R::N * (int64_t)e;
            diag[j] = a == b;
            if constexpr (R::M) xm[j] = rec[0];
            if constexpr ((MASK & TET_S) != 0) xs[j] = rec[R::M + tet_sym(min(a, b), max(a, b))];
        }
#pragma unroll
        for (int j = 0; j < H; ++j) {
            if (!ok[j]) continue;
            if constexpr (R::M) am += diag[j] ? 2.0 * xm[j] : xm[j];
            if constexpr ((MASK & TET_S) != 0) as += xs[j];
        }
    }
    if (MASK & TET_M) {
        if (accumulate) vm[p] += am;
        else vm[p] = am;
    }
    if (MASK & TET_S) {
        if (accumulate) vs[p] += as;
        else vs[p] = as;
    }
}

struct TetPatternWork {
    int *err;
    int32_t *I, *J;
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
    w.err = reinterpret_cast<int *>(take(sizeof(int) * 64));
    w.I = reinterpret_cast<int32_t *>(take(sizeof(int32_t) * (size_t)(nt > 0 ? nt : 1)));
    w.J = reinterpret_cast<int32_t *>(take(sizeof(int32_t) * (size_t)(nt > 0 ? nt : 1)));
    w.sparse = take(sb);
    w.sparse_bytes = sb;
    w.bytes = off;
    return w;
}

}  // namespace
}  // namespace fem

using namespace fem;

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
                               int32_t *col_idx, int64_t col_cap, int32_t *contrib_ptr,
                               int32_t *contrib, void *work, size_t work_bytes, int64_t *nnz_out,
                               void *stream) {
    clear_error();
    FEM_REQUIRE(nq >= 1 && nme >= 0, FEM_EINVAL, "fem_tet_pattern: need nq >= 1, nme >= 0");
    FEM_REQUIRE(16 * (int64_t)nme <= INT32_MAX, FEM_EOVERFLOW, "fem_tet_pattern: 16 nme exceeds int32");
    FEM_REQUIRE(row_ptr && work && nnz_out && contrib_ptr, FEM_EINVAL,
                "fem_tet_pattern: NULL row_ptr, contrib_ptr, work or nnz_out");
    FEM_REQUIRE(nme == 0 || (me && contrib), FEM_EINVAL, "fem_tet_pattern: NULL me or contrib");
    FEM_REQUIRE((reinterpret_cast<uintptr_t>(me) & 15) == 0, FEM_EINVAL,
                "fem_tet_pattern: me must be 16-byte aligned");
    int st = FEM_OK;
    const TetPatternWork W = carve_tet(nq, nme, static_cast<char *>(work), &st);
    if (st) return st;
    FEM_REQUIRE(work_bytes >= W.bytes, FEM_ENOSPC, "fem_tet_pattern: workspace of %zu bytes, need %zu",
                work_bytes, W.bytes);
    hipStream_t s = as_stream(stream);
    if ((st = fill_i32(W.err, 1, 0, s))) return st;
    if (nme > 0) {
        hipLaunchKernelGGL(k_tet_triplets, dim3(grid_for(nme, 256)), dim3(256), 0, s, nme, me, nq,
                           W.I, W.J, W.err);
        FEM_LAUNCH_CHECK();
    }
    int64_t nnz = 0;
    st = fem_sparse(nq, nq, 16 * (int64_t)nme, W.I, W.J, nullptr, row_ptr, col_idx, nullptr,
                    col_cap, contrib_ptr, contrib, W.sparse, W.sparse_bytes, &nnz, stream);
    int herr = 0;
    FEM_HIP_CHECK(hipMemcpyAsync(&herr, W.err, sizeof(int), hipMemcpyDeviceToHost, s));
    FEM_HIP_CHECK(hipStreamSynchronize(s));
    FEM_REQUIRE(!(herr & TET_ERR_RANGE), FEM_ERANGE, "fem_tet_pattern: a vertex index of me is outside [0, %d)", nq);
    FEM_REQUIRE(!(herr & TET_ERR_DEGEN), FEM_EDEGEN, "fem_tet_pattern: an element repeats a vertex");
    if (st) return st;
    *nnz_out = nnz;
    return FEM_OK;
}

extern "C" int fem_tet_assemble_workspace(int32_t nme, int ops, size_t *bytes) {
    clear_error();
    FEM_REQUIRE(bytes != nullptr && nme >= 0, FEM_EINVAL, "fem_tet_assemble_workspace: bad arguments");
    FEM_REQUIRE(ops == TET_M || ops == TET_S || ops == (TET_M | TET_S), FEM_EINVAL,
                "fem_tet_assemble_workspace: ops must be FEM_OP_MASS and/or FEM_OP_STIFF");
    const int per = (ops & TET_M ? 1 : 0) + (ops & TET_S ? 10 : 0);   // doubles per element
    *bytes = align_up(sizeof(double) * per * (size_t)(nme > 0 ? nme : 1));
    return FEM_OK;
}

extern "C" int fem_tet_assemble(int ops, int32_t nq, int32_t nme, int64_t nnz, const double *q,
                                const int32_t *me, const int32_t *contrib_ptr,
                                const int32_t *contrib, double *vals_M, double *vals_S, void *work,
                                size_t work_bytes, int flags, void *stream) {
    clear_error();
    FEM_REQUIRE(ops == TET_M || ops == TET_S || ops == (TET_M | TET_S), FEM_EINVAL,
                "fem_tet_assemble: ops must be FEM_OP_MASS and/or FEM_OP_STIFF");
    FEM_REQUIRE(nq >= 1 && nme >= 0 && nnz >= 0 && nnz <= INT32_MAX, FEM_EINVAL,
                "fem_tet_assemble: bad sizes");
    FEM_REQUIRE((flags & ~FEM_ACCUMULATE) == 0, FEM_EINVAL,
                "fem_tet_assemble: only FEM_ACCUMULATE is supported (the sums are deterministic)");
    FEM_REQUIRE(nme == 0 || (q && me && work), FEM_EINVAL, "fem_tet_assemble: NULL q, me or work");
    FEM_REQUIRE(contrib_ptr && (nnz == 0 || contrib), FEM_EINVAL, "fem_tet_assemble: NULL contributor list");
    FEM_REQUIRE(!(ops & TET_M) || nnz == 0 || vals_M, FEM_EINVAL, "fem_tet_assemble: NULL vals_M");
    FEM_REQUIRE(!(ops & TET_S) || nnz == 0 || vals_S, FEM_EINVAL, "fem_tet_assemble: NULL vals_S");
    FEM_REQUIRE((reinterpret_cast<uintptr_t>(me) & 15) == 0 && (reinterpret_cast<uintptr_t>(work) & 15) == 0,
                FEM_EINVAL, "fem_tet_assemble: me and work must be 16-byte aligned");
    size_t need = 0;
    fem_tet_assemble_workspace(nme, ops, &need);
    FEM_REQUIRE(work_bytes >= need, FEM_ENOSPC, "fem_tet_assemble: workspace %zu < %zu", work_bytes, need);
    hipStream_t s = as_stream(stream);
    double *kg = static_cast<double *>(work);
    const int acc = (flags & FEM_ACCUMULATE) ? 1 : 0;
    const unsigned ge = grid_for(nme, 256), gs = grid_for(nnz, 256);
    const double inv = nme > 0 ? 1.0 / (double)nme : 0.0;
    if (ops == (TET_M | TET_S)) {
        if (nme > 0) hipLaunchKernelGGL(k_tet_elem<TET_M | TET_S>, dim3(ge), dim3(256), 0, s, nme, q, me, kg);
        if (nnz > 0)
            hipLaunchKernelGGL(k_tet_sum<TET_M | TET_S>, dim3(gs), dim3(256), 0, s, nnz, contrib_ptr,
                               contrib, nme, inv, kg, vals_M, vals_S, acc);
    } else if (ops == TET_M) {
        if (nme > 0) hipLaunchKernelGGL(k_tet_elem<TET_M>, dim3(ge), dim3(256), 0, s, nme, q, me, kg);
        if (nnz > 0)
            hipLaunchKernelGGL(k_tet_sum<TET_M>, dim3(gs), dim3(256), 0, s, nnz, contrib_ptr, contrib,
                               nme, inv, kg, vals_M, nullptr, acc);
    } else {
        if (nme > 0) hipLaunchKernelGGL(k_tet_elem<TET_S>, dim3(ge), dim3(256), 0, s, nme, q, me, kg);
        if (nnz > 0)
            hipLaunchKernelGGL(k_tet_sum<TET_S>, dim3(gs), dim3(256), 0, s, nnz, contrib_ptr, contrib,
                               nme, inv, kg, nullptr, vals_S, acc);
    }
    FEM_LAUNCH_CHECK();
    return FEM_OK;
}
