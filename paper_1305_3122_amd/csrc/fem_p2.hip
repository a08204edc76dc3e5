// fem_p2.hip -- P2 (quadratic Lagrange) triangles, the P_k extension the
// Conclusion names: mass and stiffness matrices on the degrees of freedom
// {vertices} + {edges}, assembled the OptV2 way on the GPU.
//
//   fem_p2_dofs      edge numbering: the three sides (lower, higher vertex) of
//                    every triangle go through fem_sparse as triplets; the CSR
//                    position of a side is its edge number (so edges are
//                    ranked in lexicographic order of their vertex pairs) and
//                    the contributor lists say which local side of which
//                    triangle it is.  Output: dofs [nme][6] = (v0, v1, v2,
//                    nq + e0, nq + e1, nq + e2), e_a the edge opposite v_a,
//                    and optionally edges [ne][2].
//   fem_p2_pattern   Ig, Jg of all 36 local entries (triplet t = r nme + k for
//                    entry r = 6 b + a: row dofs[k][a], column dofs[k][b])
//                    compressed by fem_sparse into the CSR pattern and the
//                    contributor lists.
//   fem_p2_assemble  k_p2_elem: one lane per triangle writes four numbers;
//                    k_p2_sum: one lane per CSR entry adds its contributors in
//                    ascending t (bitwise reproducible), each contributor's
//                    value being a small-integer combination of those numbers.
//
// Why four numbers suffice.  With r_a = x_b - x_c the side opposite vertex a
// ((a, b, c) cyclic), |T| = |r_1 x r_2| / 2 and grad lambda_a . grad lambda_b =
// <r_a, r_b> / (4 |T|^2).  Put s_c = <r_a, r_b> / (4 |T|) for the pair {a, b}
// opposite c (the off-diagonal P1 stiffness entry, minus half the cotangent of
// the angle at c) and S = s_0 + s_1 + s_2.  Integrating the products of
// grad(lambda_a (2 lambda_a - 1)) = (4 lambda_a - 1) grad lambda_a and
// grad(4 lambda_b lambda_c) = 4 (lambda_c grad lambda_b + lambda_b grad lambda_c)
// exactly (int lambda_a = |T| / 3, int lambda_a^2 = |T| / 6,
// int lambda_a lambda_b = |T| / 12), and using sum_b grad lambda_b = 0:
//   vertex a, vertex a           s_a - S          (= -(s_b + s_c))
//   vertex a, vertex b != a      -s_c / 3
//   vertex a, edge opposite a    0
//   vertex a, edge opposite z    4 s_z / 3        (z != a)
//   edge e, edge e               -8 S / 3
//   edge p, edge r != p          8 s_x / 3        (x the third index)
// and the mass entries are |T| / 180 times
//   6 (vertex, same), -1 (vertex, other vertex), -4 (vertex, opposite edge),
//   0 (vertex, adjacent edge), 32 (edge, same), 16 (edge, other edge).
// So k_p2_elem stores (|T| / 180, s_0 / 3, s_1 / 3, s_2 / 3) and every
// contributor is an integer combination of those.

#include "fem_internal.h"

extern "C" int fem_sparse_workspace(int32_t m, int32_t n, int64_t nt, size_t *bytes);
extern "C" int fem_sparse(int32_t m, int32_t n, int64_t nt, const int32_t *I, const int32_t *J,
                          const double *V, int32_t *row_ptr, int32_t *col_idx, double *vals,
                          int64_t col_cap, int32_t *contrib_ptr, int32_t *contrib, void *work,
                          size_t work_bytes, int64_t *nnz_out, void *stream);

namespace fem {
namespace {

enum : int { P2_ERR_RANGE = 1, P2_ERR_DEGEN = 2 };
constexpr int P2_M = 1, P2_S = 4;   // FEM_OP_MASS, FEM_OP_STIFF

inline size_t align_up(size_t x) { return (x + 255) & ~size_t(255); }

// ---------------------------------------------------------------- coefficients

// Packed signed bytes (mass, stiffness on s_0 / 3, s_1 / 3, s_2 / 3) of local
// entry r = 6 b + a, from the table in the header comment.
struct P2Coef {
    int m, s[3];
};

constexpr P2Coef p2_coef(int a, int b) {
    P2Coef c{0, {0, 0, 0}};
    if (a < 3 && b < 3) {
        if (a == b) {
            c.m = 6;
            c.s[(a + 1) % 3] = -3;
            c.s[(a + 2) % 3] = -3;
        } else {
            c.m = -1;
            c.s[3 - a - b] = -1;
        }
    } else if (a >= 3 && b >= 3) {
        if (a == b) {
            c.m = 32;
            c.s[0] = c.s[1] = c.s[2] = -8;
        } else {
            c.m = 16;
            c.s[3 - (a - 3) - (b - 3)] = 8;
        }
    } else {
        const int v = a < 3 ? a : b, z = (a < 3 ? b : a) - 3;
        if (v == z) {
            c.m = -4;
        } else {
            c.s[z] = 4;
        }
    }
    return c;
}

constexpr uint32_t pack_coef(P2Coef c) {
    return (uint32_t)(uint8_t)(int8_t)c.m | (uint32_t)(uint8_t)(int8_t)c.s[0] << 8 |
           (uint32_t)(uint8_t)(int8_t)c.s[1] << 16 | (uint32_t)(uint8_t)(int8_t)c.s[2] << 24;
}

struct P2Table {
    uint32_t w[36];
};

constexpr P2Table make_table() {
    P2Table t{};
    for (int b = 0; b < 6; ++b)
        for (int a = 0; a < 6; ++a) t.w[6 * b + a] = pack_coef(p2_coef(a, b));
    return t;
}

__constant__ P2Table P2_TABLE = make_table();
static_assert(p2_coef(0, 0).m == 6 && p2_coef(0, 0).s[1] == -3 && p2_coef(0, 0).s[0] == 0, "vertex diagonal");
static_assert(p2_coef(1, 5).s[2] == 4 && p2_coef(1, 5).m == 0 && p2_coef(1, 4).m == -4 && p2_coef(1, 4).s[1] == 0, "vertex-edge");
static_assert(p2_coef(4, 1).m == -4 && p2_coef(3, 5).s[1] == 8 && p2_coef(4, 4).m == 32, "edge rows");

__device__ __forceinline__ int sbyte(uint32_t w, int i) { return (int)(int8_t)(uint8_t)(w >> (8 * i)); }

// ---------------------------------------------------------------- dofs

// The three sides of triangle k as triplets (lower, higher vertex) at
// t = a nme + k for the side opposite local vertex a; the vertex part of dofs.
// Invalid triangles are reported and contribute the pair (0, 0) so that the
// compression still runs in bounds.
__global__ __launch_bounds__(256) void k_p2_sides(int32_t nme, const int32_t *__restrict__ me,
                                                  int32_t nq, int32_t *__restrict__ I,
                                                  int32_t *__restrict__ J,
                                                  int32_t *__restrict__ dofs, int *err) {
    const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (k >= nme) return;
    int v[3] = {me[3 * k], me[3 * k + 1], me[3 * k + 2]};
    int bad = 0;
#pragma unroll
    for (int a = 0; a < 3; ++a)
        if ((uint32_t)v[a] >= (uint32_t)nq) bad |= P2_ERR_RANGE;
    if (!bad && (v[0] == v[1] || v[1] == v[2] || v[0] == v[2])) bad |= P2_ERR_DEGEN;
    if (bad) {
        atomicOr(err, bad);
        v[0] = v[1] = v[2] = 0;
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const int u = v[(a + 1) % 3], w = v[(a + 2) % 3];
        I[(int64_t)a * nme + k] = min(u, w);
        J[(int64_t)a * nme + k] = max(u, w);
        dofs[6 * k + a] = v[a];
    }
}

// One lane per edge: its number goes to the edge slot of each triangle side
// that produced it.
__global__ __launch_bounds__(256) void k_p2_edge_dofs(int32_t ne, const int32_t *__restrict__ cptr,
                                                      const int32_t *__restrict__ contrib,
                                                      int32_t nme, int32_t nq,
                                                      int32_t *__restrict__ dofs) {
    const int32_t e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= ne) return;
    for (int32_t i = cptr[e]; i < cptr[e + 1]; ++i) {
        const int32_t t = contrib[i];
        const int32_t a = t >= 2 * nme ? 2 : (t >= nme ? 1 : 0);
        dofs[6 * (int64_t)(t - a * nme) + 3 + a] = nq + e;
    }
}

// One lane per vertex: the (lower, higher) pairs of the edges in its row.
__global__ __launch_bounds__(256) void k_p2_edge_list(int32_t nq, const int32_t *__restrict__ rp,
                                                      const int32_t *__restrict__ col,
                                                      int32_t *__restrict__ edges) {
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nq) return;
    for (int32_t e = rp[i]; e < rp[i + 1]; ++e)
        reinterpret_cast<int2 *>(edges)[e] = make_int2(i, col[e]);
}

// ---------------------------------------------------------------- pattern

// Ig / Jg of element k (one lane per element; writes for a fixed entry r are
// coalesced across lanes).
__global__ __launch_bounds__(256) void k_p2_triplets(int32_t nme, const int32_t *__restrict__ dofs,
                                                     int32_t *__restrict__ I,
                                                     int32_t *__restrict__ J) {
    const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (k >= nme) return;
    const int2 *d2 = reinterpret_cast<const int2 *>(dofs + 6 * k);
    const int2 p0 = d2[0], p1 = d2[1], p2 = d2[2];
    const int d[6] = {p0.x, p0.y, p1.x, p1.y, p2.x, p2.y};
#pragma unroll
    for (int b = 0; b < 6; ++b)
#pragma unroll
        for (int a = 0; a < 6; ++a) {
            const int64_t s = (int64_t)(6 * b + a) * nme + k;
            I[s] = d[a];
            J[s] = d[b];
        }
}

// ---------------------------------------------------------------- values

// (|T| / 180, s_0 / 3, s_1 / 3, s_2 / 3) of triangle k.
__global__ __launch_bounds__(256) void k_p2_elem(int32_t nme, const double *__restrict__ q,
                                                 const int32_t *__restrict__ me,
                                                 double4 *__restrict__ ed) {
    const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (k >= nme) return;
    const double2 *q2 = reinterpret_cast<const double2 *>(q);
    const double2 x0 = q2[me[3 * k]], x1 = q2[me[3 * k + 1]], x2 = q2[me[3 * k + 2]];
    const double r0x = x1.x - x2.x, r0y = x1.y - x2.y;
    const double r1x = x2.x - x0.x, r1y = x2.y - x0.y;
    const double r2x = x0.x - x1.x, r2y = x0.y - x1.y;
    const double ad = fabs(r0x * r1y - r0y * r1x);     // 2 |T|
    const double inv = 1.0 / (6.0 * ad);                // 1 / (3 * 4 |T|)
    ed[k] = make_double4(ad / 360.0, (r1x * r2x + r1y * r2y) * inv, (r2x * r0x + r2y * r0y) * inv,
                         (r0x * r1x + r0y * r1y) * inv);
}

// One lane per CSR entry: the sum of its contributors in ascending t, the
// contributor t = r nme + k being the combination of table word r with the
// numbers of triangle k.
template <int MASK>
__global__ __launch_bounds__(256) void k_p2_sum(int64_t nnz, const int32_t *__restrict__ cptr,
                                                const int32_t *__restrict__ contrib, int32_t nme,
                                                double inv_nme, const double4 *__restrict__ ed,
                                                double *__restrict__ vm, double *__restrict__ vs,
                                                int accumulate) {
    __shared__ uint32_t tab[36];
    if (threadIdx.x < 36) tab[threadIdx.x] = P2_TABLE.w[threadIdx.x];
    __syncthreads();
    const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (p >= nnz) return;
    const uint32_t nt = 36u * (uint32_t)nme;
    double am = 0.0, as = 0.0;
    const int32_t i0 = cptr[p], i1 = cptr[p + 1];
    // H contributors at a time: their triplet ids, then their element
    // records, all loads in flight; the terms are then added in ascending
    // order, as one at a time would
    constexpr int H = 4;
    const double *edx = reinterpret_cast<const double *>(ed);
    for (int32_t i = i0; i < i1; i += H) {
        int32_t tt[H];
#pragma unroll
        for (int j = 0; j < H; ++j) tt[j] = i + j < i1 ? contrib[i + j] : -1;
        bool ok[H];
        uint32_t w[H];
        double4 e[H];
#pragma unroll
        for (int j = 0; j < H; ++j) {
            const int32_t t = tt[j];
            // past the list, or not a triplet of these nme triangles
            ok[j] = (uint32_t)t < nt;
            w[j] = 0;
            e[j] = make_double4(0.0, 0.0, 0.0, 0.0);
            if (!ok[j]) continue;
            // r = t / nme: the double quotient is off by at most one
            int32_t r = (int32_t)((double)t * inv_nme);
            int32_t k = t - r * nme;
            if (k < 0) {
                --r;
                k += nme;
            } else if (k >= nme) {
                ++r;
                k -= nme;
            }
            w[j] = tab[r];
            if constexpr (MASK & P2_S) e[j] = ed[k];
            else e[j].x = edx[4 * (int64_t)k];
        }
#pragma unroll
        for (int j = 0; j < H; ++j) {
            if (!ok[j]) continue;
            if (MASK & P2_M) am += sbyte(w[j], 0) * e[j].x;
            if (MASK & P2_S) as += sbyte(w[j], 1) * e[j].y + sbyte(w[j], 2) * e[j].z + sbyte(w[j], 3) * e[j].w;
        }
    }
    if (MASK & P2_M) {
        if (accumulate) vm[p] += am;
        else vm[p] = am;
    }
    if (MASK & P2_S) {
        if (accumulate) vs[p] += as;
        else vs[p] = as;
    }
}

// ---------------------------------------------------------------- workspaces

struct Carver {
    char *base;
    size_t off = 0;
    char *take(size_t bytes) {
        char *p = base ? base + off : nullptr;
        off += align_up(bytes);
        return p;
    }
};

struct DofsWork {
    int *err;
    int32_t *I, *J, *rp, *col, *cptr, *contrib;
    char *sparse;
    size_t sparse_bytes, bytes;
};

DofsWork carve_dofs(int32_t nq, int32_t nme, char *base, int *st) {
    DofsWork w{};
    const int64_t nt = 3 * (int64_t)nme;
    const size_t n = (size_t)(nt > 0 ? nt : 1);
    size_t sb = 0;
    *st = fem_sparse_workspace(nq, nq, nt, &sb);
    Carver c{base};
    w.err = reinterpret_cast<int *>(c.take(sizeof(int) * 64));
    w.I = reinterpret_cast<int32_t *>(c.take(sizeof(int32_t) * n));
    w.J = reinterpret_cast<int32_t *>(c.take(sizeof(int32_t) * n));
    w.rp = reinterpret_cast<int32_t *>(c.take(sizeof(int32_t) * ((size_t)nq + 1)));
    w.col = reinterpret_cast<int32_t *>(c.take(sizeof(int32_t) * n));
    w.cptr = reinterpret_cast<int32_t *>(c.take(sizeof(int32_t) * (n + 1)));
    w.contrib = reinterpret_cast<int32_t *>(c.take(sizeof(int32_t) * n));
    w.sparse = c.take(sb);
    w.sparse_bytes = sb;
    w.bytes = c.off;
    return w;
}

struct PatternWork {
    int32_t *I, *J;
    char *sparse;
    size_t sparse_bytes, bytes;
};

PatternWork carve_p2_pattern(int32_t ndof, int32_t nme, char *base, int *st) {
    PatternWork w{};
    const int64_t nt = 36 * (int64_t)nme;
    const size_t n = (size_t)(nt > 0 ? nt : 1);
    size_t sb = 0;
    *st = fem_sparse_workspace(ndof, ndof, nt, &sb);
    Carver c{base};
    w.I = reinterpret_cast<int32_t *>(c.take(sizeof(int32_t) * n));
    w.J = reinterpret_cast<int32_t *>(c.take(sizeof(int32_t) * n));
    w.sparse = c.take(sb);
    w.sparse_bytes = sb;
    w.bytes = c.off;
    return w;
}

}  // namespace
}  // namespace fem

using namespace fem;

extern "C" int fem_p2_dofs_workspace(int32_t nq, int32_t nme, size_t *bytes) {
    clear_error();
    FEM_REQUIRE(bytes != nullptr, FEM_EINVAL, "fem_p2_dofs_workspace: bytes is NULL");
    FEM_REQUIRE(nq >= 1 && nme >= 0, FEM_EINVAL, "fem_p2_dofs_workspace: need nq >= 1, nme >= 0");
    FEM_REQUIRE(36 * (int64_t)nme <= INT32_MAX, FEM_EOVERFLOW, "fem_p2_dofs_workspace: 36 nme exceeds int32");
    int st = FEM_OK;
    const DofsWork W = carve_dofs(nq, nme, nullptr, &st);
    if (st) return st;
    *bytes = W.bytes;
    return FEM_OK;
}

extern "C" int fem_p2_dofs(int32_t nq, int32_t nme, const int32_t *me, int32_t *dofs,
                           int32_t *edges, int64_t edge_cap, void *work, size_t work_bytes,
                           int64_t *ne_out, void *stream) {
    clear_error();
    FEM_REQUIRE(nq >= 1 && nme >= 0, FEM_EINVAL, "fem_p2_dofs: need nq >= 1, nme >= 0");
    FEM_REQUIRE(36 * (int64_t)nme <= INT32_MAX, FEM_EOVERFLOW, "fem_p2_dofs: 36 nme exceeds int32");
    FEM_REQUIRE(work && ne_out, FEM_EINVAL, "fem_p2_dofs: NULL work or ne_out");
    FEM_REQUIRE(nme == 0 || (me && dofs), FEM_EINVAL, "fem_p2_dofs: NULL me or dofs");
    FEM_REQUIRE((reinterpret_cast<uintptr_t>(dofs) & 7) == 0, FEM_EINVAL,
                "fem_p2_dofs: dofs must be 8-byte aligned");
    FEM_REQUIRE(!edges || ((reinterpret_cast<uintptr_t>(edges) & 7) == 0 && edge_cap >= 0), FEM_EINVAL,
                "fem_p2_dofs: edges must be 8-byte aligned, edge_cap >= 0");
    int st = FEM_OK;
    const DofsWork W = carve_dofs(nq, nme, static_cast<char *>(work), &st);
    if (st) return st;
    FEM_REQUIRE(work_bytes >= W.bytes, FEM_ENOSPC, "fem_p2_dofs: workspace of %zu bytes, need %zu",
                work_bytes, W.bytes);
    hipStream_t s = as_stream(stream);
    if ((st = fill_i32(W.err, 1, 0, s))) return st;
    if (nme > 0) {
        hipLaunchKernelGGL(k_p2_sides, dim3(grid_for(nme, 256)), dim3(256), 0, s, nme, me, nq, W.I, W.J,
                           dofs, W.err);
        FEM_LAUNCH_CHECK();
    }
    const int64_t nt = 3 * (int64_t)nme;
    int64_t ne = 0;
    st = fem_sparse(nq, nq, nt, W.I, W.J, nullptr, W.rp, W.col, nullptr, nt, W.cptr, W.contrib,
                    W.sparse, W.sparse_bytes, &ne, stream);
    int herr = 0;
    FEM_HIP_CHECK(hipMemcpyAsync(&herr, W.err, sizeof(int), hipMemcpyDeviceToHost, s));
    FEM_HIP_CHECK(hipStreamSynchronize(s));
    FEM_REQUIRE(!(herr & P2_ERR_RANGE), FEM_ERANGE, "fem_p2_dofs: a vertex index of me is outside [0, %d)", nq);
    FEM_REQUIRE(!(herr & P2_ERR_DEGEN), FEM_EDEGEN, "fem_p2_dofs: a triangle repeats a vertex");
    if (st) return st;
    FEM_REQUIRE((int64_t)nq + ne <= INT32_MAX, FEM_EOVERFLOW, "fem_p2_dofs: nq + ne exceeds int32");
    FEM_REQUIRE(!edges || ne <= edge_cap, FEM_ENOSPC, "fem_p2_dofs: ne = %lld exceeds edge_cap = %lld",
                (long long)ne, (long long)edge_cap);
    if (ne > 0) {
        hipLaunchKernelGGL(k_p2_edge_dofs, dim3(grid_for(ne, 256)), dim3(256), 0, s, (int32_t)ne, W.cptr,
                           W.contrib, nme, nq, dofs);
        FEM_LAUNCH_CHECK();
        if (edges) {
            hipLaunchKernelGGL(k_p2_edge_list, dim3(grid_for(nq, 256)), dim3(256), 0, s, nq, W.rp, W.col,
                               edges);
            FEM_LAUNCH_CHECK();
        }
    }
    *ne_out = ne;
    return FEM_OK;
}

extern "C" int fem_p2_pattern_workspace(int32_t ndof, int32_t nme, size_t *bytes) {
    clear_error();
    FEM_REQUIRE(bytes != nullptr, FEM_EINVAL, "fem_p2_pattern_workspace: bytes is NULL");
    FEM_REQUIRE(ndof >= 1 && nme >= 0, FEM_EINVAL, "fem_p2_pattern_workspace: need ndof >= 1, nme >= 0");
    FEM_REQUIRE(36 * (int64_t)nme <= INT32_MAX, FEM_EOVERFLOW,
                "fem_p2_pattern_workspace: 36 nme exceeds int32");
    int st = FEM_OK;
    const PatternWork W = carve_p2_pattern(ndof, nme, nullptr, &st);
    if (st) return st;
    *bytes = W.bytes;
    return FEM_OK;
}

extern "C" int fem_p2_pattern(int32_t ndof, int32_t nme, const int32_t *dofs, int32_t *row_ptr,
                              int32_t *col_idx, int64_t col_cap, int32_t *contrib_ptr,
                              int32_t *contrib, void *work, size_t work_bytes, int64_t *nnz_out,
                              void *stream) {
    clear_error();
    FEM_REQUIRE(ndof >= 1 && nme >= 0, FEM_EINVAL, "fem_p2_pattern: need ndof >= 1, nme >= 0");
    FEM_REQUIRE(36 * (int64_t)nme <= INT32_MAX, FEM_EOVERFLOW, "fem_p2_pattern: 36 nme exceeds int32");
    FEM_REQUIRE(row_ptr && work && nnz_out && contrib_ptr, FEM_EINVAL,
                "fem_p2_pattern: NULL row_ptr, contrib_ptr, work or nnz_out");
    FEM_REQUIRE(nme == 0 || (dofs && contrib), FEM_EINVAL, "fem_p2_pattern: NULL dofs or contrib");
    FEM_REQUIRE((reinterpret_cast<uintptr_t>(dofs) & 7) == 0, FEM_EINVAL,
                "fem_p2_pattern: dofs must be 8-byte aligned");
    int st = FEM_OK;
    const PatternWork W = carve_p2_pattern(ndof, nme, static_cast<char *>(work), &st);
    if (st) return st;
    FEM_REQUIRE(work_bytes >= W.bytes, FEM_ENOSPC, "fem_p2_pattern: workspace of %zu bytes, need %zu",
                work_bytes, W.bytes);
    hipStream_t s = as_stream(stream);
    if (nme > 0) {
        hipLaunchKernelGGL(k_p2_triplets, dim3(grid_for(nme, 256)), dim3(256), 0, s, nme, dofs, W.I, W.J);
        FEM_LAUNCH_CHECK();
    }
    return fem_sparse(ndof, ndof, 36 * (int64_t)nme, W.I, W.J, nullptr, row_ptr, col_idx, nullptr,
                      col_cap, contrib_ptr, contrib, W.sparse, W.sparse_bytes, nnz_out, stream);
}

extern "C" int fem_p2_assemble_workspace(int32_t nme, size_t *bytes) {
    clear_error();
    FEM_REQUIRE(bytes != nullptr && nme >= 0, FEM_EINVAL, "fem_p2_assemble_workspace: bad arguments");
    *bytes = align_up(sizeof(double4) * (size_t)(nme > 0 ? nme : 1));
    return FEM_OK;
}

extern "C" int fem_p2_assemble(int ops, int32_t nq, int32_t nme, int64_t nnz, const double *q,
                               const int32_t *me, const int32_t *contrib_ptr, const int32_t *contrib,
                               double *vals_M, double *vals_S, void *work, size_t work_bytes, int flags,
                               void *stream) {
    clear_error();
    FEM_REQUIRE(ops == P2_M || ops == P2_S || ops == (P2_M | P2_S), FEM_EINVAL,
                "fem_p2_assemble: ops must be FEM_OP_MASS and/or FEM_OP_STIFF");
    FEM_REQUIRE(nq >= 1 && nme >= 0 && nnz >= 0 && nnz <= INT32_MAX, FEM_EINVAL,
                "fem_p2_assemble: bad sizes");
    FEM_REQUIRE(36 * (int64_t)nme <= INT32_MAX, FEM_EOVERFLOW, "fem_p2_assemble: 36 nme exceeds int32");
    FEM_REQUIRE((flags & ~FEM_ACCUMULATE) == 0, FEM_EINVAL,
                "fem_p2_assemble: only FEM_ACCUMULATE is supported (the sums are deterministic)");
    FEM_REQUIRE(nme == 0 || (q && me && work), FEM_EINVAL, "fem_p2_assemble: NULL q, me or work");
    FEM_REQUIRE(contrib_ptr && (nnz == 0 || contrib), FEM_EINVAL, "fem_p2_assemble: NULL contributor list");
    FEM_REQUIRE(!(ops & P2_M) || nnz == 0 || vals_M, FEM_EINVAL, "fem_p2_assemble: NULL vals_M");
    FEM_REQUIRE(!(ops & P2_S) || nnz == 0 || vals_S, FEM_EINVAL, "fem_p2_assemble: NULL vals_S");
    FEM_REQUIRE((reinterpret_cast<uintptr_t>(q) & 15) == 0 && (reinterpret_cast<uintptr_t>(work) & 31) == 0,
                FEM_EINVAL, "fem_p2_assemble: q must be 16-byte and work 32-byte aligned");
    FEM_REQUIRE(nnz == 0 || nme > 0, FEM_EINVAL, "fem_p2_assemble: entries without triangles");
    size_t need = 0;
    fem_p2_assemble_workspace(nme, &need);
    FEM_REQUIRE(work_bytes >= need, FEM_ENOSPC, "fem_p2_assemble: workspace %zu < %zu", work_bytes, need);
    hipStream_t s = as_stream(stream);
    double4 *ed = static_cast<double4 *>(work);
    const int acc = (flags & FEM_ACCUMULATE) ? 1 : 0;
    if (nme > 0) {
        hipLaunchKernelGGL(k_p2_elem, dim3(grid_for(nme, 256)), dim3(256), 0, s, nme, q, me, ed);
        FEM_LAUNCH_CHECK();
    }
    if (nnz == 0) return FEM_OK;
    const unsigned gs = grid_for(nnz, 256);
    const double inv = 1.0 / (double)nme;
    if (ops == (P2_M | P2_S))
        hipLaunchKernelGGL(k_p2_sum<P2_M | P2_S>, dim3(gs), dim3(256), 0, s, nnz, contrib_ptr, contrib, nme,
                           inv, ed, vals_M, vals_S, acc);
    else if (ops == P2_M)
        hipLaunchKernelGGL(k_p2_sum<P2_M>, dim3(gs), dim3(256), 0, s, nnz, contrib_ptr, contrib, nme, inv,
                           ed, vals_M, nullptr, acc);
    else
        hipLaunchKernelGGL(k_p2_sum<P2_S>, dim3(gs), dim3(256), 0, s, nnz, contrib_ptr, contrib, nme, inv,
                           ed, nullptr, vals_S, acc);
    FEM_LAUNCH_CHECK();
    return FEM_OK;
}
