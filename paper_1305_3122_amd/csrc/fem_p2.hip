// fem_p2.hip -- P2 (quadratic Lagrange) triangles, the P_k extension the
// Conclusion names: mass and stiffness matrices on the degrees of freedom
// {vertices} + {edges}.
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
//                    compressed by fem_sparse into the CSR pattern; the
//                    contributors of a row's diagonal entry (r = 7 a) are the
//                    row's triangles, merged by id -> inc (6 k + a), and the
//                    row slots of each triangle's six DOFs -> inc_pos.  The
//                    contributor lists stay in the workspace.
//   fem_p2_assemble  k_p2_elem: one lane per triangle writes four numbers;
//                    k_p2_rows: one lane per DOF row walks its triangles in
//                    ascending id and adds each one's six entries of the row
//                    (small-integer combinations of those numbers) to
//                    per-slot sums in LDS; the rows leave coalesced (bitwise
//                    reproducible).
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
// element entry is an integer combination of those.

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

// ---------------------------------------------------------------- rows

constexpr int P2_POS_BITS = 10;                  // inc_pos: six 10-bit row slots
constexpr int P2_ROW_MAX = 1 << P2_POS_BITS;     // longest row inc_pos can address
enum : int { P2_ERR_ROWLEN = 4 };

__device__ inline int32_t p2_find(const int32_t *__restrict__ row, int32_t L, int32_t y) {
    int32_t lo = 0, hi = L;
    while (lo < hi) {
        const int32_t mid = (lo + hi) >> 1;
        if (row[mid] < y) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// Per DOF row: its triangles are the contributors of its diagonal entry
// (r = 7 a); deg[i] = their number.
__global__ __launch_bounds__(256) void k_p2_deg(int32_t ndof, const int32_t *__restrict__ row_ptr,
                                                const int32_t *__restrict__ col_idx,
                                                const int32_t *__restrict__ cptr,
                                                int32_t *__restrict__ deg, int *err) {
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ndof) return;
    const int32_t rs = row_ptr[i], L = row_ptr[i + 1] - rs;
    int32_t d = 0;
    if (L > 0) {
        const int32_t pd = p2_find(col_idx + rs, L, i);
        d = cptr[rs + pd + 1] - cptr[rs + pd];
    }
    deg[i] = d;
    if (L > P2_ROW_MAX) atomicOr(err, P2_ERR_ROWLEN);
}

// Per DOF row: the diagonal contributors t = 7 a nme + k are the row's
// triangles (k, a); sorted by k they give inc (6 k + a), and each triangle's
// six DOFs are found in the row: inc_pos holds their slots in local order
// (bits 10 b .. 10 b + 9 for local DOF b) and a in bits 60-62.  One lane per
// row, one wave per workgroup: a row of at most P2_DL entries is searched in
// LDS ([slot][lane]) and up to P2_DD triangles are sorted by a network in
// registers (words k << 3 | a); longer rows are searched in global memory
// and their triangles merged from the six runs of their contributor list.
constexpr int P2_DL = 32, P2_DD = 16;

template <int N>
__device__ __forceinline__ void p2_sort_u32(uint32_t (&k)[N]) {
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

__global__ __launch_bounds__(WAVE) void k_p2_derive(int32_t ndof, int32_t nme,
                                                   const int32_t *__restrict__ dofs,
                                                   const int32_t *__restrict__ row_ptr,
                                                   const int32_t *__restrict__ col_idx,
                                                   const int32_t *__restrict__ cptr,
                                                   const int32_t *__restrict__ contrib,
                                                   const int32_t *__restrict__ inc_ptr,
                                                   int32_t *__restrict__ inc,
                                                   uint64_t *__restrict__ inc_pos) {
    __shared__ int32_t s_row[P2_DL * WAVE];   // [slot][lane]
    const int lane = threadIdx.x;
    const int32_t i = blockIdx.x * WAVE + lane;
    if (i >= ndof) return;
    const int32_t rs = row_ptr[i], L = row_ptr[i + 1] - rs;
    const int32_t is = inc_ptr[i], d = inc_ptr[i + 1] - is;
    if (L == 0 || d == 0 || L > P2_ROW_MAX) return;
    const int32_t *row = col_idx + rs;
    const int32_t *c = contrib + cptr[rs + p2_find(row, L, i)];
    if (L <= P2_DL && d <= P2_DD) {
        // the row into LDS, its loads all in flight
        int32_t rv[P2_DL];
#pragma unroll
        for (int p = 0; p < P2_DL; ++p) rv[p] = p < L ? row[p] : 0;
#pragma unroll
        for (int p = 0; p < P2_DL; ++p)
            if (p < L) s_row[p * WAVE + lane] = rv[p];
        auto find = [&](int32_t y) {
            int32_t lo = 0, hi = L;
            while (lo < hi) {
                const int32_t mid = (lo + hi) >> 1;
                if (s_row[mid * WAVE + lane] < y) lo = mid + 1;
                else hi = mid;
            }
            return lo;
        };
        // contributor t = 7 a nme + k: a from the run the value falls in
        uint32_t w[P2_DD];
#pragma unroll
        for (int j = 0; j < P2_DD; ++j) {
            w[j] = 0xffffffffu;
            if (j < d) {
                const int32_t t = c[j];
                int a = 0;
#pragma unroll
                for (int b = 1; b < 6; ++b) a += (int64_t)t >= 7ll * b * nme ? 1 : 0;
                w[j] = ((uint32_t)(t - 7 * a * nme) << 3) | (uint32_t)a;
            }
        }
        if (d <= 4) {
            // edge rows (one or two triangles) and other short rows
            uint32_t w4[4] = {w[0], w[1], w[2], w[3]};
            p2_sort_u32<4>(w4);
#pragma unroll
            for (int j = 0; j < 4; ++j) w[j] = w4[j];
        } else {
            p2_sort_u32<P2_DD>(w);
        }
        // the triangles' DOFs, all loads in flight, then their slots
        int2 dk[P2_DD][3];
#pragma unroll
        for (int j = 0; j < P2_DD; ++j) {
            const int2 *src = reinterpret_cast<const int2 *>(dofs + 6 * (int64_t)(j < d ? (int32_t)(w[j] >> 3) : 0));
#pragma unroll
            for (int h = 0; h < 3; ++h) dk[j][h] = j < d ? src[h] : make_int2(0, 0);
        }
#pragma unroll
        for (int j = 0; j < P2_DD; ++j) {
            if (j < d) {
                const int32_t k = (int32_t)(w[j] >> 3);
                const int a = (int)(w[j] & 7u);
                const int32_t dd[6] = {dk[j][0].x, dk[j][0].y, dk[j][1].x, dk[j][1].y, dk[j][2].x, dk[j][2].y};
                uint64_t pw = (uint64_t)a << 60;
#pragma unroll
                for (int b = 0; b < 6; ++b) pw |= (uint64_t)find(dd[b]) << (P2_POS_BITS * b);
                inc[is + j] = 6 * k + a;
                inc_pos[is + j] = pw;
            }
        }
        return;
    }
    int32_t lo[7];   // run a covers [lo[a], lo[a + 1]): the first t >= 7 a nme
    lo[0] = 0;
    lo[6] = d;
    for (int a = 1; a < 6; ++a) {
        const int64_t thr = 7ll * a * nme;
        int32_t l = lo[a - 1], h = d;
        while (l < h) {
            const int32_t m = (l + h) >> 1;
            if ((int64_t)c[m] < thr) l = m + 1;
            else h = m;
        }
        lo[a] = l;
    }
    int32_t cur[6] = {lo[0], lo[1], lo[2], lo[3], lo[4], lo[5]};
    for (int32_t j = 0; j < d; ++j) {
        int best = -1;
        int32_t bk = 0;
        for (int a = 0; a < 6; ++a) {
            if (cur[a] < lo[a + 1]) {
                const int32_t k = c[cur[a]] - 7 * a * nme;
                if (best < 0 || k < bk) {
                    best = a;
                    bk = k;
                }
            }
        }
        ++cur[best];
        uint64_t w = (uint64_t)best << 60;
        for (int b = 0; b < 6; ++b)
            w |= (uint64_t)p2_find(row, L, dofs[6 * (int64_t)bk + b]) << (P2_POS_BITS * b);
        inc[is + j] = 6 * bk + best;
        inc_pos[is + j] = w;
    }
}

constexpr int P2_LM_V = 24;   // row slots a lane keeps in LDS: vertex rows (3 v + 1 for valence v)
constexpr int P2_LM_E = 10;   // edge rows (9 on an interior edge)
constexpr int P2_IP_V = 8;    // triangles per row whose records are loaded up front: vertex rows
constexpr int P2_IP_E = 2;    // edge rows

// The contribution of triangle record e to entry (a, b) of its element
// matrices: table word 6 b + a applied to (|T| / 180, s_0 / 3, s_1 / 3, s_2 / 3).
template <int MASK>
__device__ __forceinline__ void p2_term(uint32_t cw, const double4 &e, double &m, double &s) {
    if constexpr ((MASK & P2_M) != 0) m = sbyte(cw, 0) * e.x;
    if constexpr ((MASK & P2_S) != 0) s = sbyte(cw, 1) * e.y + sbyte(cw, 2) * e.z + sbyte(cw, 3) * e.w;
}

// One lane per DOF row over rows [r_begin, r_end), one wave per workgroup;
// vertex rows and edge rows go to separate launches with their own LM and
// IP, so that the short edge rows need less LDS and fewer registers.  The
// row's first IP triangles' ids, slots and records are loaded up front;
// then one pass over them per operator: the per-slot sums in LDS (A
// [LM][WAVE]; per triangle, its six slots are distinct, so the six sums are
// read together and written back together), then the wave's rows leave as
// one contiguous, coalesced range, each entry finding its lane and slot in
// an owner table (LM WAVE ints; written row by row from the lanes the rows
// took 1.4-1.6x as long).  One operator at a time halves the LDS, and the
// owner table is half a transposition buffer of doubles, so a CU holds more
// workgroups.  A row longer than LM is summed by its lane slot by slot from global
// memory (same terms, same order, so the same values bit for bit).
template <int MASK, int LM, int IP>
__global__ __launch_bounds__(WAVE) void k_p2_rows(int32_t r_begin, int32_t r_end,
                                                  const int32_t *__restrict__ row_ptr,
                                                  const int32_t *__restrict__ inc_ptr,
                                                  const int32_t *__restrict__ inc,
                                                  const uint64_t *__restrict__ inc_pos,
                                                  const double4 *__restrict__ ed,
                                                  double *__restrict__ vm, double *__restrict__ vs,
                                                  int accumulate) {
    constexpr bool HM = (MASK & P2_M) != 0, HS = (MASK & P2_S) != 0;
    constexpr int NA = (HM ? 1 : 0) + (HS ? 1 : 0);
    __shared__ double A[LM * WAVE];
    __shared__ int32_t own[LM * WAVE];   // (lane << 8 | slot) of each entry of the range
    __shared__ uint32_t tab[36];
    const int lane = threadIdx.x;
    if (lane < 36) tab[lane] = P2_TABLE.w[lane];
    const int32_t r0 = r_begin + blockIdx.x * WAVE;
    const int32_t i = r0 + lane;
    const bool valid = i < r_end;
    int32_t rs = 0, L = 0, is = 0, d = 0;
    if (valid) {
        rs = row_ptr[i];
        L = row_ptr[i + 1] - rs;
        is = inc_ptr[i];
        d = inc_ptr[i + 1] - is;
    }
    const int32_t end_all = row_ptr[r_end];
    const int32_t rsv = valid ? rs : end_all;   // rows past the range start at its end
    const int32_t R1 = r0 + WAVE < r_end ? row_ptr[r0 + WAVE] : end_all;
    const bool fast = L <= LM;
    const uint64_t longmask = __ballot(!fast);
    auto AX = [&](int p) -> double & { return A[p * WAVE + lane]; };
    __syncthreads();   // the table
    // the first IP triangles: ids and slots, then their records
    int32_t kk[IP];
    uint64_t ww[IP];
    double4 ee[IP];
    if (fast && L > 0) {
#pragma unroll
        for (int t = 0; t < IP; ++t) {
            kk[t] = t < d ? inc[is + t] / 6 : 0;
            ww[t] = t < d ? inc_pos[is + t] : 0ull;
        }
#pragma unroll
        for (int t = 0; t < IP; ++t) ee[t] = ed[kk[t]];
    } else if (!fast) {
        // long row: slot by slot, the terms of that slot in ascending order
        for (int32_t p = 0; p < L; ++p) {
            double sm = 0.0, ss = 0.0;
            for (int32_t t = 0; t < d; ++t) {
                const uint64_t w = inc_pos[is + t];
                const int a = (int)(w >> 60);
                for (int b = 0; b < 6; ++b) {
                    if ((int)((w >> (P2_POS_BITS * b)) & (P2_ROW_MAX - 1)) != p) continue;
                    double m = 0.0, s = 0.0;
                    p2_term<MASK>(tab[6 * b + a], ed[inc[is + t] / 6], m, s);
                    sm += m;
                    ss += s;
                }
            }
            if constexpr (HM) vm[rs + p] = accumulate ? vm[rs + p] + sm : sm;
            if constexpr (HS) vs[rs + p] = accumulate ? vs[rs + p] + ss : ss;
        }
    }
    const int32_t R0 = __shfl(rsv, 0, WAVE);
#pragma unroll
    for (int op = 0; op < NA; ++op) {
        // the operator of this pass: mass first when both are asked for
        const bool is_m = HM && op == 0;
        double *out = is_m ? vm : vs;
        if (fast && L > 0) {
            for (int p = 0; p < L; ++p) AX(p) = 0.0;
            auto step = [&](uint64_t w, const double4 &e) {
                const int a = (int)(w >> 60);
                int sl[6];
                double o[6];
#pragma unroll
                for (int b = 0; b < 6; ++b) {
                    sl[b] = (int)((w >> (P2_POS_BITS * b)) & (P2_ROW_MAX - 1));
                    o[b] = AX(sl[b]);
                }
#pragma unroll
                for (int b = 0; b < 6; ++b) {
                    double m = 0.0, s = 0.0;
                    if (is_m) p2_term<P2_M>(tab[6 * b + a], e, m, s);
                    else p2_term<P2_S>(tab[6 * b + a], e, m, s);
                    AX(sl[b]) = o[b] + (is_m ? m : s);
                }
            };
#pragma unroll
            for (int t = 0; t < IP; ++t)
                if (t < d) step(ww[t], ee[t]);
            for (int32_t t = IP; t < d; ++t) step(inc_pos[is + t], ed[inc[is + t] / 6]);
        }
        // the workgroup is one wave, whose LDS accesses complete in program
        // order: scheduling barriers order the sums, the transposition and
        // the write-out
        __builtin_amdgcn_wave_barrier();
        if (longmask == 0) {
            // every row has at most LM entries (the range at most LM WAVE):
            // the owner table (written once, on the first pass) names each
            // entry's lane and slot, and the range is written in order
            if (op == 0) {
                for (int p = 0; p < L; ++p) own[rs - R0 + p] = (lane << 8) | p;
                __builtin_amdgcn_wave_barrier();
            }
            // overwrites are streaming stores (separate loops: merged with the
            // accumulate path's store, the hint would be dropped)
            auto owned = [&](int32_t e) {
                const int32_t o = own[e - R0];
                return A[(o & 255) * WAVE + (o >> 8)];
            };
            if (!accumulate) {
                for (int32_t e = R0 + lane; e < R1; e += WAVE) __builtin_nontemporal_store(owned(e), out + e);
            } else {
                for (int32_t e = R0 + lane; e < R1; e += WAVE) out[e] += owned(e);
            }
        } else {
            // entry e belongs to the last row whose start is <= e (empty
            // rows share the next start); all lanes take part in the search
            for (int32_t base = R0; base < R1; base += WAVE) {
                const int32_t e = base + lane;
                int lo = 0;
#pragma unroll
                for (int stp = WAVE / 2; stp > 0; stp >>= 1) {
                    const int cand = lo + stp;
                    const int32_t sc = __shfl(rsv, cand < WAVE ? cand : WAVE - 1, WAVE);
                    if (cand < WAVE && sc <= e) lo = cand;
                }
                const int32_t rlo = __shfl(rsv, lo, WAVE);
                const int p = e - rlo;
                if (e >= R1 || ((longmask >> lo) & 1u) || p >= LM) continue;
                const double v = A[p * WAVE + lo];
                out[e] = accumulate ? out[e] + v : v;
            }
        }
        __builtin_amdgcn_wave_barrier();
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
    int *err;
    int32_t *I, *J, *cptr, *contrib, *deg;
    long long *part;
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
    w.err = reinterpret_cast<int *>(c.take(sizeof(int) * 64));
    w.I = reinterpret_cast<int32_t *>(c.take(sizeof(int32_t) * n));
    w.J = reinterpret_cast<int32_t *>(c.take(sizeof(int32_t) * n));
    w.cptr = reinterpret_cast<int32_t *>(c.take(sizeof(int32_t) * (n + 1)));
    w.contrib = reinterpret_cast<int32_t *>(c.take(sizeof(int32_t) * n));
    w.deg = reinterpret_cast<int32_t *>(c.take(sizeof(int32_t) * (size_t)ndof));
    w.part = reinterpret_cast<long long *>(c.take(sizeof(long long) * (size_t)(scan_partials(ndof) + 8)));
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
                              int32_t *col_idx, int64_t col_cap, int32_t *inc_ptr, int32_t *inc,
                              uint64_t *inc_pos, void *work, size_t work_bytes, int64_t *nnz_out,
                              void *stream) {
    clear_error();
    FEM_REQUIRE(ndof >= 1 && nme >= 0, FEM_EINVAL, "fem_p2_pattern: need ndof >= 1, nme >= 0");
    FEM_REQUIRE(36 * (int64_t)nme <= INT32_MAX, FEM_EOVERFLOW, "fem_p2_pattern: 36 nme exceeds int32");
    FEM_REQUIRE(row_ptr && inc_ptr && work && nnz_out, FEM_EINVAL,
                "fem_p2_pattern: NULL row_ptr, inc_ptr, work or nnz_out");
    FEM_REQUIRE(nme == 0 || (dofs && inc && inc_pos), FEM_EINVAL, "fem_p2_pattern: NULL dofs, inc or inc_pos");
    FEM_REQUIRE(col_cap >= 0 && (col_cap == 0 || col_idx), FEM_EINVAL,
                "fem_p2_pattern: NULL col_idx or negative col_cap");
    FEM_REQUIRE((reinterpret_cast<uintptr_t>(dofs) & 7) == 0 && (reinterpret_cast<uintptr_t>(inc_pos) & 7) == 0,
                FEM_EINVAL, "fem_p2_pattern: dofs and inc_pos must be 8-byte aligned");
    int st = FEM_OK;
    const PatternWork W = carve_p2_pattern(ndof, nme, static_cast<char *>(work), &st);
    if (st) return st;
    FEM_REQUIRE(work_bytes >= W.bytes, FEM_ENOSPC, "fem_p2_pattern: workspace of %zu bytes, need %zu",
                work_bytes, W.bytes);
    hipStream_t s = as_stream(stream);
    if ((st = fill_i32(W.err, 2, 0, s))) return st;
    if (nme > 0) {
        hipLaunchKernelGGL(k_p2_triplets, dim3(grid_for(nme, 256)), dim3(256), 0, s, nme, dofs, W.I, W.J);
        FEM_LAUNCH_CHECK();
    }
    int64_t nnz = 0;
    if ((st = fem_sparse(ndof, ndof, 36 * (int64_t)nme, W.I, W.J, nullptr, row_ptr, col_idx, nullptr,
                         col_cap, W.cptr, W.contrib, W.sparse, W.sparse_bytes, &nnz, stream)))
        return st;
    hipLaunchKernelGGL(k_p2_deg, dim3(grid_for(ndof, 256)), dim3(256), 0, s, ndof, row_ptr, col_idx, W.cptr,
                       W.deg, W.err);
    FEM_LAUNCH_CHECK();
    long long *tot = W.part + scan_partials(ndof);
    if ((st = exclusive_scan_i32(W.deg, inc_ptr, ndof, W.part, tot, W.err + 1, s))) return st;
    hipLaunchKernelGGL(k_p2_derive, dim3(grid_for(ndof, WAVE)), dim3(WAVE), 0, s, ndof, nme, dofs, row_ptr,
                       col_idx, W.cptr, W.contrib, inc_ptr, inc, inc_pos);
    FEM_LAUNCH_CHECK();
    int herr[2] = {0, 0};
    FEM_HIP_CHECK(hipMemcpyAsync(herr, W.err, sizeof(herr), hipMemcpyDeviceToHost, s));
    FEM_HIP_CHECK(hipStreamSynchronize(s));
    FEM_REQUIRE(!(herr[0] & P2_ERR_ROWLEN), FEM_EUNSUPPORTED,
                "fem_p2_pattern: a row has more than %d entries", P2_ROW_MAX);
    *nnz_out = nnz;
    return FEM_OK;
}

extern "C" int fem_p2_assemble_workspace(int32_t nme, size_t *bytes) {
    clear_error();
    FEM_REQUIRE(bytes != nullptr && nme >= 0, FEM_EINVAL, "fem_p2_assemble_workspace: bad arguments");
    *bytes = align_up(sizeof(double4) * (size_t)(nme > 0 ? nme : 1));
    return FEM_OK;
}

extern "C" int fem_p2_assemble(int ops, int32_t nq, int32_t nme, int32_t ndof, int64_t nnz,
                               const double *q, const int32_t *me, const int32_t *row_ptr,
                               const int32_t *inc_ptr, const int32_t *inc, const uint64_t *inc_pos,
                               double *vals_M, double *vals_S, void *work, size_t work_bytes, int flags,
                               void *stream) {
    clear_error();
    FEM_REQUIRE(ops == P2_M || ops == P2_S || ops == (P2_M | P2_S), FEM_EINVAL,
                "fem_p2_assemble: ops must be FEM_OP_MASS and/or FEM_OP_STIFF");
    FEM_REQUIRE(nq >= 1 && nme >= 0 && ndof >= nq && nnz >= 0 && nnz <= INT32_MAX, FEM_EINVAL,
                "fem_p2_assemble: bad sizes");
    FEM_REQUIRE(36 * (int64_t)nme <= INT32_MAX, FEM_EOVERFLOW, "fem_p2_assemble: 36 nme exceeds int32");
    FEM_REQUIRE((flags & ~FEM_ACCUMULATE) == 0, FEM_EINVAL,
                "fem_p2_assemble: only FEM_ACCUMULATE is supported (the sums are deterministic)");
    FEM_REQUIRE(nme == 0 || (q && me && work), FEM_EINVAL, "fem_p2_assemble: NULL q, me or work");
    FEM_REQUIRE(row_ptr && inc_ptr && (nnz == 0 || (inc && inc_pos)), FEM_EINVAL,
                "fem_p2_assemble: NULL row_ptr, inc_ptr, inc or inc_pos");
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
    // vertex rows [0, nq), then edge rows [nq, ndof)
    const int32_t nv = nq < ndof ? nq : ndof;
    const unsigned gv = grid_for(nv, WAVE), ge = grid_for(ndof - nv, WAVE);
    if (ops == (P2_M | P2_S)) {
        hipLaunchKernelGGL((k_p2_rows<P2_M | P2_S, P2_LM_V, P2_IP_V>), dim3(gv), dim3(WAVE), 0, s, 0, nv, row_ptr,
                           inc_ptr, inc, inc_pos, ed, vals_M, vals_S, acc);
        if (ndof > nv)
            hipLaunchKernelGGL((k_p2_rows<P2_M | P2_S, P2_LM_E, P2_IP_E>), dim3(ge), dim3(WAVE), 0, s, nv, ndof, row_ptr,
                               inc_ptr, inc, inc_pos, ed, vals_M, vals_S, acc);
    } else if (ops == P2_M) {
        hipLaunchKernelGGL((k_p2_rows<P2_M, P2_LM_V, P2_IP_V>), dim3(gv), dim3(WAVE), 0, s, 0, nv, row_ptr, inc_ptr, inc,
                           inc_pos, ed, vals_M, nullptr, acc);
        if (ndof > nv)
            hipLaunchKernelGGL((k_p2_rows<P2_M, P2_LM_E, P2_IP_E>), dim3(ge), dim3(WAVE), 0, s, nv, ndof, row_ptr, inc_ptr,
                               inc, inc_pos, ed, vals_M, nullptr, acc);
    } else {
        hipLaunchKernelGGL((k_p2_rows<P2_S, P2_LM_V, P2_IP_V>), dim3(gv), dim3(WAVE), 0, s, 0, nv, row_ptr, inc_ptr, inc,
                           inc_pos, ed, nullptr, vals_S, acc);
        if (ndof > nv)
            hipLaunchKernelGGL((k_p2_rows<P2_S, P2_LM_E, P2_IP_E>), dim3(ge), dim3(WAVE), 0, s, nv, ndof, row_ptr, inc_ptr,
                               inc, inc_pos, ed, nullptr, vals_S, acc);
    }
    FEM_LAUNCH_CHECK();
    return FEM_OK;
}
