// fem_numeric.hip -- numeric phase: element matrices and their summation
// into the CSR values.
//
// Element formulas (FP64, no MFMA: the work is a gather/scatter bound by
// memory, not a dense contraction):
//   |T| = |det| / 2, det = (q2-q1) x (q3-q1)
//   mass (eq. MassElem)            |T|/12 [2 1 1; 1 2 1; 1 1 2]
//   weighted mass (eq. MassWElem)  |T|/30 (3w_a + w_b + w_c) on the diagonal,
//                                  |T|/30 (w_a + w_b + w_c/2) off it (c third)
//   stiffness (eq. StiffMatElem)   <r_a, r_b> / (4|T|), r = (q2-q3, q3-q1, q1-q2)
//   elasticity                     |T| B^T C B, gradients perp(r_a) / det
// Any subset of the four operators is assembled in one pass (`ops` mask), so
// that the gathers of q and w -- the dominant cost on a relabelled mesh,
// where every gather is a random access -- are shared.
//
// Two summation schemes:
//
// FEM_DETERMINISTIC -- row owner.  One lane owns one CSR row (one vertex i)
//   and walks the triangles around i (inc_ptr / inc_pos), computing the row of
//   each element matrix that belongs to i and adding it into the row's
//   entries.  A wave owns 64 consecutive rows, whose entries are contiguous in
//   col_idx/values: it stages that slice in LDS (gathered vertex coordinates,
//   accumulators), so every read of the pattern and every write of values is
//   coalesced and written exactly once; the only random accesses are the
//   gathers of q (and w) by column.  Each element is evaluated once per
//   vertex (three times), which costs flops, not bytes.  Every value is summed
//   by one lane in ascending triangle order: bitwise reproducible.
// FEM_ATOMIC -- one lane per triangle computes the full element matrices and
//   adds them through the slot map with FP64 atomics (global_atomic_add_f64).
#include "fem_internal.h"

#include <mutex>

namespace fem {

// operator bits (same values as FEM_OP_* of the C ABI)
enum : int { M_BIT = 1, W_BIT = 2, S_BIT = 4, K_BIT = 8 };

template <int MASK> struct Ops {
    static constexpr bool M = (MASK & M_BIT) != 0, W = (MASK & W_BIT) != 0;
    static constexpr bool S = (MASK & S_BIT) != 0, K = (MASK & K_BIT) != 0;
    static constexpr int NS = (M ? 1 : 0) + (W ? 1 : 0) + (S ? 1 : 0);   // scalar accumulators
    static constexpr int IM = 0, IW = M ? 1 : 0, IS = (M ? 1 : 0) + (W ? 1 : 0);
    static constexpr int NV = NS + (K ? 4 : 0);                           // accumulators per entry
};

struct Lame {
    double lam, mu;
};

// Row of the element matrices that belongs to vertex 0 of the triangle
// (x0, x1, x2), a cyclic rotation of the triangle's own vertex order (so the
// orientation and the edge vectors r are those of the paper's formulas).
// c[m][0] diagonal term of scalar operator m, c[m][1] / c[m][2] the terms of
// columns x1 / x2; ce[b] the 2x2 elasticity block (row-major) of column b.
template <int MASK>
__device__ __forceinline__ void elem_row(double x0, double y0, double x1, double y1, double x2,
                                         double y2, double w0, double w1, double w2, Lame L,
                                         double (&c)[Ops<MASK>::NS > 0 ? Ops<MASK>::NS : 1][3],
                                         double (&ce)[3][4]) {
    using O = Ops<MASK>;
    const double e1x = x1 - x0, e1y = y1 - y0;
    const double e2x = x2 - x0, e2y = y2 - y0;
    const double det = e1x * e2y - e2x * e1y;
    const double ad = fabs(det);
    const double area = 0.5 * ad;
    if constexpr (O::S) {
        // r0 = x1 - x2, r1 = x2 - x0, r2 = x0 - x1;  S_0b = <r0, rb> / (2 |det|)
        const double r0x = x1 - x2, r0y = y1 - y2;
        const double inv = 1.0 / (2.0 * ad);
        c[O::IS][0] = (r0x * r0x + r0y * r0y) * inv;
        c[O::IS][1] = (r0x * e2x + r0y * e2y) * inv;
        c[O::IS][2] = -(r0x * e1x + r0y * e1y) * inv;
    }
    if constexpr (O::M) {
        c[O::IM][0] = area / 6.0;
        c[O::IM][1] = area / 12.0;
        c[O::IM][2] = area / 12.0;
    }
    if constexpr (O::W) {
        const double a30 = area / 30.0;
        c[O::IW][0] = a30 * (3.0 * w0 + w1 + w2);
        c[O::IW][1] = a30 * (w0 + w1 + 0.5 * w2);
        c[O::IW][2] = a30 * (w0 + 0.5 * w1 + w2);
    }
    if constexpr (O::K) {
        const double id = 1.0 / det;
        const double g0x = (y1 - y2) * id, g0y = -(x1 - x2) * id;
        const double gx[3] = {g0x, e2y * id, -e1y * id};
        const double gy[3] = {g0y, -e2x * id, e1x * id};
        const double l2m = L.lam + 2.0 * L.mu;
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            ce[b][0] = area * (l2m * g0x * gx[b] + L.mu * g0y * gy[b]);   // (x, x)
            ce[b][1] = area * (L.lam * g0x * gy[b] + L.mu * g0y * gx[b]); // (x, y)
            ce[b][2] = area * (L.lam * g0y * gx[b] + L.mu * g0x * gy[b]); // (y, x)
            ce[b][3] = area * (l2m * g0y * gy[b] + L.mu * g0x * gx[b]);   // (y, y)
        }
    }
}

struct Outs {
    double *o[4];   // M, Mw, S, K (K in the 2x2 block layout of fem_elas_pattern)
};

// Stores the n values of an LDS tile to o, coalesced: lane l takes entries
// l, l + 64, ...  Overwrites are streaming stores (nothing reads the values
// back in this pass); the accumulate path adds in place.  The two paths are
// separate loops: merged into one store, the streaming hint would be dropped.
__device__ __forceinline__ void tile_store(double *__restrict__ o, const double *src, int n, int lane,
                                           int accumulate) {
    if (!accumulate) {
        for (int e = lane; e < n; e += WAVE) __builtin_nontemporal_store(src[e], o + e);
    } else {
        for (int e = lane; e < n; e += WAVE) o[e] += src[e];
    }
}

// (x, y, w, 0) records, so that a vertex costs one random access.
__global__ __launch_bounds__(256) void k_pack_qw(int32_t nq, const double2 *__restrict__ q,
                                                 const double *__restrict__ w,
                                                 double4 *__restrict__ qw) {
    const int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (v >= nq) return;
    const double2 a = q[v];
    qw[v] = make_double4(a.x, a.y, w ? w[v] : 0.0, 0.0);
}

// FEM_CHECK_AREA: flag triangles of zero area (det of the edge vectors
// u = q2 - q3, v = q3 - q1), where the element formulas divide by zero.
__global__ __launch_bounds__(256) void k_check_area(int32_t nme, const double2 *__restrict__ q,
                                                    const int32_t *__restrict__ me, int *flag) {
    const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (k >= nme) return;
    const double2 x1 = q[me[3 * k]], x2 = q[me[3 * k + 1]], x3 = q[me[3 * k + 2]];
    const double ux = x2.x - x3.x, uy = x2.y - x3.y, vx = x3.x - x1.x, vy = x3.y - x1.y;
    if (ux * vy - uy * vx == 0.0) atomicOr(flag, 1);
}

// ------------------------------------------------------------------ row owner
//
// Tile = 64 consecutive rows (one per lane) = a contiguous slice of col_idx /
// values and of inc_pos.  Staged in three rounds of independent loads, each
// issued in full before anything waits on it:
//   A  row_ptr / inc_ptr bounds of the lane's row and of the tile
//   B  the tile's columns (registers) and triangle positions (LDS), streaming
//   C  the gathers of q (and w) by column
// then every lane sums its row from LDS and the tile is written back
// coalesced.  U = LDS entries per tile / 64.  The diagonal position of a row
// is the one position no triangle refers to (p1, p2 are always neighbours).

template <int MASK, int U>
__global__ __launch_bounds__(WAVE) void k_rows_numeric(
    int32_t nq, const double *__restrict__ q, const double *__restrict__ w,
    const double4 *__restrict__ qw, const int32_t *__restrict__ row_ptr,
    const int32_t *__restrict__ col_idx, const int32_t *__restrict__ inc_ptr,
    const uint32_t *__restrict__ inc_pos, Outs out, Lame L, int accumulate, int64_t ntiles) {
    using O = Ops<MASK>;
    constexpr int NS = O::NS;
    constexpr int NSA = NS > 0 ? NS : 1;
    constexpr int EB = U * WAVE;
    // LDS tile: scalar acc [NS EB] | K acc [4 EB] | q [EB] (double2) | w [EB] | ipos [EB]
    extern __shared__ double smem[];
    double *s_acc = smem;
    double *s_k = s_acc + (size_t)NS * EB;
    double2 *s_q = reinterpret_cast<double2 *>(s_k + (O::K ? 4 * EB : 0));
    double *s_w = reinterpret_cast<double *>(s_q + EB);
    uint32_t *s_ip = reinterpret_cast<uint32_t *>(s_w + (O::W ? EB : 0));
    const int lane = threadIdx.x;
    const double2 *q2 = reinterpret_cast<const double2 *>(q);

    for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        // ---- round A
        const int64_t r0 = tile * WAVE;
        const int64_t r1 = (r0 + WAVE < nq) ? r0 + WAVE : nq;
        const int64_t i = r0 + lane;
        const bool active = i < nq;
        const int32_t E0 = row_ptr[r0], E1 = row_ptr[r1];
        const int32_t I0 = inc_ptr[r0], I1 = inc_ptr[r1];
        const int32_t rs = active ? row_ptr[i] : 0;
        const int32_t re = active ? row_ptr[i + 1] : 0;
        const int32_t is = active ? inc_ptr[i] : 0;
        const int32_t ie = active ? inc_ptr[i + 1] : 0;
        const int32_t Ew = E1 - E0, Iw = I1 - I0, len = re - rs;

        if (Ew <= EB && Iw <= EB) {
            // ---- round B
            int32_t cidx[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int e = lane + u * WAVE;
                cidx[u] = e < Ew ? __builtin_nontemporal_load(col_idx + E0 + e) : 0;
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int t = lane + u * WAVE;
                if (t < Iw) s_ip[t] = __builtin_nontemporal_load(inc_pos + I0 + t);
            }
            // ---- round C: one random access per column (packed records if given)
            double2 qv[U];
            double wv[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int e = lane + u * WAVE;
                wv[u] = 0.0;
                if (e < Ew) {
                    if (O::W && qw) {
                        const double4 r = qw[cidx[u]];
                        qv[u] = make_double2(r.x, r.y);
                        wv[u] = r.z;
                    } else {
                        qv[u] = q2[cidx[u]];
                        if constexpr (O::W) wv[u] = w[cidx[u]];
                    }
                } else {
                    qv[u] = make_double2(0.0, 0.0);
                }
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int e = lane + u * WAVE;
                if (e < Ew) {
                    s_q[e] = qv[u];
                    if constexpr (O::W) s_w[e] = wv[u];
#pragma unroll
                    for (int m = 0; m < NS; ++m) s_acc[m * EB + e] = 0.0;
                }
            }
            if constexpr (O::K) {
#pragma unroll
                for (int u = 0; u < 4 * U; ++u) {
                    const int e = lane + u * WAVE;
                    if (e < 4 * Ew) s_k[e] = 0.0;
                }
            }
            __syncthreads();
            // ---- each lane: the triangles around its vertex, ascending id
            if (active && len > 0) {
                const int32_t off = rs - E0;
                int32_t pd;
                if (len <= 64) {
                    uint64_t seen = 0;
                    for (int32_t t = is - I0; t < ie - I0; ++t) {
                        const uint32_t pp = s_ip[t];
                        seen |= (1ull << (pp & 0xffffu)) | (1ull << (pp >> 16));
                    }
                    pd = __builtin_ctzll(~seen);
                } else {
                    int32_t lo = 0, hi = len;
                    while (lo < hi) {
                        const int32_t mid = (lo + hi) >> 1;
                        if (col_idx[rs + mid] < (int32_t)i) lo = mid + 1;
                        else hi = mid;
                    }
                    pd = lo;
                }
                const double2 x0 = s_q[off + pd];
                const double w0 = O::W ? s_w[off + pd] : 0.0;
                double dg[NSA], dk[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
                for (int m = 0; m < NSA; ++m) dg[m] = 0.0;
                for (int32_t t = is - I0; t < ie - I0; ++t) {
                    const uint32_t pp = s_ip[t];
                    const int32_t p1 = (int32_t)(pp & 0xffffu), p2 = (int32_t)(pp >> 16);
                    const double2 x1 = s_q[off + p1], x2 = s_q[off + p2];
                    double c[NSA][3];
                    double ce[3][4];
                    elem_row<MASK>(x0.x, x0.y, x1.x, x1.y, x2.x, x2.y, w0,
                                   O::W ? s_w[off + p1] : 0.0, O::W ? s_w[off + p2] : 0.0, L, c, ce);
#pragma unroll
                    for (int m = 0; m < NS; ++m) {
                        dg[m] += c[m][0];
                        s_acc[m * EB + off + p1] += c[m][1];
                        s_acc[m * EB + off + p2] += c[m][2];
                    }
                    if constexpr (O::K) {
                        // row 2i: [4 off + 2p + beta], row 2i+1: [+ 2 len]
                        const int32_t b0 = 4 * off;
#pragma unroll
                        for (int z = 0; z < 4; ++z) dk[z] += ce[0][z];
                        s_k[b0 + 2 * p1] += ce[1][0];
                        s_k[b0 + 2 * p1 + 1] += ce[1][1];
                        s_k[b0 + 2 * len + 2 * p1] += ce[1][2];
                        s_k[b0 + 2 * len + 2 * p1 + 1] += ce[1][3];
                        s_k[b0 + 2 * p2] += ce[2][0];
                        s_k[b0 + 2 * p2 + 1] += ce[2][1];
                        s_k[b0 + 2 * len + 2 * p2] += ce[2][2];
                        s_k[b0 + 2 * len + 2 * p2 + 1] += ce[2][3];
                    }
                }
#pragma unroll
                for (int m = 0; m < NS; ++m) s_acc[m * EB + off + pd] += dg[m];
                if constexpr (O::K) {
                    const int32_t b0 = 4 * off;
                    s_k[b0 + 2 * pd] += dk[0];
                    s_k[b0 + 2 * pd + 1] += dk[1];
                    s_k[b0 + 2 * len + 2 * pd] += dk[2];
                    s_k[b0 + 2 * len + 2 * pd + 1] += dk[3];
                }
            }
            __syncthreads();
            // ---- write the tile back, coalesced (no read unless accumulating)
            if (!accumulate) {
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int e = lane + u * WAVE;
                    if (e < Ew) {
#pragma unroll
                        for (int m = 0; m < NS; ++m)
                            __builtin_nontemporal_store(s_acc[m * EB + e], out.o[m] + E0 + e);
                    }
                }
                if constexpr (O::K) {
                    double *ok = out.o[3] + 4 * (int64_t)E0;
#pragma unroll
                    for (int u = 0; u < 4 * U; ++u) {
                        const int e = lane + u * WAVE;
                        if (e < 4 * Ew) __builtin_nontemporal_store(s_k[e], ok + e);
                    }
                }
            } else {
                for (int e = lane; e < Ew; e += WAVE) {
#pragma unroll
                    for (int m = 0; m < NS; ++m) out.o[m][E0 + e] += s_acc[m * EB + e];
                }
                if constexpr (O::K) {
                    double *ok = out.o[3] + 4 * (int64_t)E0;
                    for (int e = lane; e < 4 * Ew; e += WAVE) ok[e] += s_k[e];
                }
            }
            __syncthreads();
        } else if (active && len > 0) {
            // ---- tile too large for LDS: the lane works on its own row in
            // global memory (same order of additions, so same results)
            double *os[NSA];
#pragma unroll
            for (int m = 0; m < NSA; ++m) os[m] = m < NS ? out.o[m] + rs : nullptr;
            double *ok = O::K ? out.o[3] + 4 * (int64_t)rs : nullptr;
            if (!accumulate) {
                for (int e = 0; e < len; ++e) {
#pragma unroll
                    for (int m = 0; m < NS; ++m) os[m][e] = 0.0;
                }
                if constexpr (O::K)
                    for (int e = 0; e < 4 * len; ++e) ok[e] = 0.0;
            }
            const int32_t *cr = col_idx + rs;
            int32_t pd = 0;
            while (pd < len - 1 && cr[pd] != (int32_t)i) ++pd;
            const double x0 = q[2 * i], y0 = q[2 * i + 1];
            const double w0 = O::W ? w[i] : 0.0;
            double dg[NSA], dk[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int m = 0; m < NSA; ++m) dg[m] = 0.0;
            for (int32_t t = is; t < ie; ++t) {
                const uint32_t pp = inc_pos[t];
                const int32_t p1 = (int32_t)(pp & 0xffffu), p2 = (int32_t)(pp >> 16);
                const int64_t j1 = cr[p1], j2 = cr[p2];
                double c[NSA][3];
                double ce[3][4];
                elem_row<MASK>(x0, y0, q[2 * j1], q[2 * j1 + 1], q[2 * j2], q[2 * j2 + 1], w0,
                               O::W ? w[j1] : 0.0, O::W ? w[j2] : 0.0, L, c, ce);
#pragma unroll
                for (int m = 0; m < NS; ++m) {
                    dg[m] += c[m][0];
                    os[m][p1] += c[m][1];
                    os[m][p2] += c[m][2];
                }
                if constexpr (O::K) {
#pragma unroll
                    for (int z = 0; z < 4; ++z) dk[z] += ce[0][z];
                    ok[2 * p1] += ce[1][0];
                    ok[2 * p1 + 1] += ce[1][1];
                    ok[2 * len + 2 * p1] += ce[1][2];
                    ok[2 * len + 2 * p1 + 1] += ce[1][3];
                    ok[2 * p2] += ce[2][0];
                    ok[2 * p2 + 1] += ce[2][1];
                    ok[2 * len + 2 * p2] += ce[2][2];
                    ok[2 * len + 2 * p2 + 1] += ce[2][3];
                }
            }
#pragma unroll
            for (int m = 0; m < NS; ++m) os[m][pd] += dg[m];
            if constexpr (O::K) {
                ok[2 * pd] += dk[0];
                ok[2 * pd + 1] += dk[1];
                ok[2 * len + 2 * pd] += dk[2];
                ok[2 * len + 2 * pd + 1] += dk[3];
            }
        }
    }
}

// ------------------------------------------------------------------ row owner, registers
//
// Same tiling and load rounds as above, but each lane keeps the accumulators
// of its row in registers (rows of at most LMAX entries: a static slot loop
// adds each triangle's terms into slots p1 / p2), so LDS only stages the
// gathered coordinates and the triangle positions, and is then reused to
// transpose the accumulators for coalesced stores.  Far more waves fit per CU
// than with LDS accumulators.
//
// The scalar operators and the elasticity blocks are summed in two phases
// over the same staged tile: the gathers are paid once, and the registers
// held at any time are those of one phase (3 x LMAX or 4 x LMAX
// accumulators, not 7 x LMAX).  Lanes whose row is longer than LMAX, or whose
// tile does not fit the stage, sum LMAX entries at a time from global memory;
// the order of additions is the same everywhere.

// Adds the row terms of one triangle (owner x0, the other two vertices at row
// slots p1 / p2) to the slot registers and to the diagonal sums.
template <int PM, int LMAX>
__device__ __forceinline__ void add_tri(double x0, double y0, double x1, double y1, double x2,
                                        double y2, double w0, double w1, double w2, Lame L,
                                        int32_t p1, int32_t p2, double (&acc)[Ops<PM>::NV][LMAX],
                                        double (&dg)[Ops<PM>::NV]) {
    using O = Ops<PM>;
    double c[O::NS > 0 ? O::NS : 1][3];
    double ce[3][4];
    elem_row<PM>(x0, y0, x1, y1, x2, y2, w0, w1, w2, L, c, ce);
#pragma unroll
    for (int m = 0; m < O::NS; ++m) dg[m] += c[m][0];
    if constexpr (O::K) {
#pragma unroll
        for (int z = 0; z < 4; ++z) dg[O::NS + z] += ce[0][z];
    }
#pragma unroll
    for (int k = 0; k < LMAX; ++k) {
        const bool h1 = k == p1, h2 = k == p2;
#pragma unroll
        for (int m = 0; m < O::NS; ++m) acc[m][k] += h1 ? c[m][1] : (h2 ? c[m][2] : 0.0);
        if constexpr (O::K) {
#pragma unroll
            for (int z = 0; z < 4; ++z) acc[O::NS + z][k] += h1 ? ce[1][z] : (h2 ? ce[2][z] : 0.0);
        }
    }
}

// Row sums of the operators in PM from the staged tile (zero when the lane's
// row is not summed here); the diagonal slot pd gets its sums last.
template <int PM, int LMAX>
__device__ __forceinline__ void tile_sum(bool in_regs, const double2 *s_q, const double *s_w,
                                         const uint32_t *s_ip, int32_t off, int32_t t0, int32_t t1,
                                         int32_t pd, double2 x0, double w0, Lame L,
                                         double (&acc)[Ops<PM>::NV][LMAX]) {
    using O = Ops<PM>;
#pragma unroll
    for (int v = 0; v < O::NV; ++v)
#pragma unroll
        for (int k = 0; k < LMAX; ++k) acc[v][k] = 0.0;
    if (!in_regs) return;
    double dg[O::NV];
#pragma unroll
    for (int v = 0; v < O::NV; ++v) dg[v] = 0.0;
    for (int32_t t = t0; t < t1; ++t) {
        const uint32_t pp = s_ip[t];
        const int32_t p1 = (int32_t)(pp & 0xffffu), p2 = (int32_t)(pp >> 16);
        const double2 x1 = s_q[off + p1], x2 = s_q[off + p2];
        add_tri<PM, LMAX>(x0.x, x0.y, x1.x, x1.y, x2.x, x2.y, w0, O::W ? s_w[off + p1] : 0.0,
                          O::W ? s_w[off + p2] : 0.0, L, p1, p2, acc, dg);
    }
#pragma unroll
    for (int k = 0; k < LMAX; ++k)
        if (k == pd) {
#pragma unroll
            for (int v = 0; v < O::NV; ++v) acc[v][k] += dg[v];
        }
}

// Row entries [c0, c0 + LMAX) of the operators in PM, summed from global
// memory over the lane's triangles in the same order as tile_sum.
template <int PM, int LMAX>
__device__ __forceinline__ void chunk_sum(const double *q, const double *w, const int32_t *cr,
                                          const uint32_t *inc_pos, int32_t is, int32_t ie,
                                          int32_t c0, int32_t pd, double x0, double y0, double w0,
                                          Lame L, double (&ch)[Ops<PM>::NV][LMAX]) {
    using O = Ops<PM>;
#pragma unroll
    for (int v = 0; v < O::NV; ++v)
#pragma unroll
        for (int k = 0; k < LMAX; ++k) ch[v][k] = 0.0;
    double dg[O::NV];
#pragma unroll
    for (int v = 0; v < O::NV; ++v) dg[v] = 0.0;
    for (int32_t t = is; t < ie; ++t) {
        const uint32_t pp = inc_pos[t];
        const int32_t p1 = (int32_t)(pp & 0xffffu), p2 = (int32_t)(pp >> 16);
        const int64_t j1 = cr[p1], j2 = cr[p2];
        add_tri<PM, LMAX>(x0, y0, q[2 * j1], q[2 * j1 + 1], q[2 * j2], q[2 * j2 + 1], w0,
                          O::W ? w[j1] : 0.0, O::W ? w[j2] : 0.0, L, p1 - c0, p2 - c0, ch, dg);
    }
#pragma unroll
    for (int k = 0; k < LMAX; ++k)
        if (c0 + k == pd) {
#pragma unroll
            for (int v = 0; v < O::NV; ++v) ch[v][k] += dg[v];
        }
}

template <int MASK, int U, int LMAX>
__global__ __launch_bounds__(WAVE) void k_rows_reg(
    int32_t nq, const double *__restrict__ q, const double *__restrict__ w,
    const double4 *__restrict__ qw, const int32_t *__restrict__ row_ptr,
    const int32_t *__restrict__ col_idx, const int32_t *__restrict__ inc_ptr,
    const uint32_t *__restrict__ inc_pos, Outs out, Lame L, int accumulate, int64_t ntiles) {
    using O = Ops<MASK>;
    constexpr int MS = MASK & (M_BIT | W_BIT | S_BIT);   // scalar operators (phase 1)
    constexpr int NS = O::NS;
    constexpr int EB = U * WAVE;
    // LDS: stage [SD EB doubles] | ipos [EB words].  The stage holds q
    // (doubles [0, 2 EB)) and w ([2 EB, 3 EB)).  With K it has 4 EB doubles:
    // [3 EB, 4 EB) is the scalar transposition buffer (the staged coordinates
    // must outlive phase 1), and the whole stage takes the K transposition (4
    // doubles per entry) once phase 2 has summed.  Without K the scalar
    // transposition reuses the stage.
    constexpr int SD = O::K ? 4 : (O::W ? 3 : 2); // doubles per entry in the stage
    extern __shared__ double smem[];
    double *s_stage = smem;
    double2 *s_q = reinterpret_cast<double2 *>(smem);
    double *s_w = smem + 2 * EB;
    double *s_t = O::K ? smem + 3 * EB : smem;
    uint32_t *s_ip = reinterpret_cast<uint32_t *>(smem + SD * EB);
    const int lane = threadIdx.x;
    const double2 *q2 = reinterpret_cast<const double2 *>(q);

    for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const int64_t r0 = tile * WAVE;
        const int64_t r1 = (r0 + WAVE < nq) ? r0 + WAVE : nq;
        const int64_t i = r0 + lane;
        const bool active = i < nq;
        const int32_t E0 = row_ptr[r0], E1 = row_ptr[r1];
        const int32_t I0 = inc_ptr[r0], I1 = inc_ptr[r1];
        const int32_t rs = active ? row_ptr[i] : 0;
        const int32_t re = active ? row_ptr[i + 1] : 0;
        const int32_t is = active ? inc_ptr[i] : 0;
        const int32_t ie = active ? inc_ptr[i + 1] : 0;
        const int32_t Ew = E1 - E0, Iw = I1 - I0, len = re - rs;
        const bool tile_fits = Ew <= EB && Iw <= EB;

        if (tile_fits) {
            int32_t cidx[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int e = lane + u * WAVE;
                cidx[u] = e < Ew ? __builtin_nontemporal_load(col_idx + E0 + e) : 0;
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int t = lane + u * WAVE;
                if (t < Iw) s_ip[t] = __builtin_nontemporal_load(inc_pos + I0 + t);
            }
            double2 qv[U];
            double wv[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int e = lane + u * WAVE;
                wv[u] = 0.0;
                if (e < Ew) {
                    if (O::W && qw) {
                        const double4 r = qw[cidx[u]];
                        qv[u] = make_double2(r.x, r.y);
                        wv[u] = r.z;
                    } else {
                        qv[u] = q2[cidx[u]];
                        if constexpr (O::W) wv[u] = w[cidx[u]];
                    }
                } else {
                    qv[u] = make_double2(0.0, 0.0);
                }
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int e = lane + u * WAVE;
                if (e < Ew) {
                    s_q[e] = qv[u];
                    if constexpr (O::W) s_w[e] = wv[u];
                }
            }
            __syncthreads();
        }
        const bool in_regs = tile_fits && active && len > 0 && len <= LMAX;
        // rows not summed in registers stage zeros in the tile stores (their
        // lane writes them after the tile, below)
        const bool zero_row = !in_regs && active && len > 0;
        const int32_t off = rs - E0;
        int32_t pd = 0;
        double2 x0 = make_double2(0.0, 0.0);
        double w0 = 0.0;
        if (in_regs) {
            uint64_t seen = 0;
            for (int32_t t = is - I0; t < ie - I0; ++t) {
                const uint32_t pp = s_ip[t];
                seen |= (1ull << (pp & 0xffffu)) | (1ull << (pp >> 16));
            }
            pd = __builtin_ctzll(~seen);
            x0 = s_q[off + pd];
            if constexpr (O::W) w0 = s_w[off + pd];
        }
        if constexpr (MS != 0) {
            // ---- phase 1: scalar operators, one transposition per operator
            double acc[NS][LMAX];
            tile_sum<MS, LMAX>(in_regs, s_q, s_w, s_ip, off, is - I0, ie - I0, pd, x0, w0, L, acc);
            if (tile_fits) {
                if constexpr (!O::K) __syncthreads();   // s_t is the stage: all reads done
#pragma unroll
                for (int m = 0; m < NS; ++m) {
                    if (in_regs) {
#pragma unroll
                        for (int k = 0; k < LMAX; ++k)
                            if (k < len) s_t[off + k] = acc[m][k];
                    } else if (zero_row) {
                        for (int k = 0; k < len; ++k) s_t[off + k] = 0.0;
                    }
                    __syncthreads();
                    tile_store(out.o[m] + E0, s_t, Ew, lane, accumulate);
                    __syncthreads();
                }
            }
        }
        if constexpr (O::K) {
            // ---- phase 2: elasticity 2x2 blocks from the same staged tile
            double acc[4][LMAX];
            tile_sum<K_BIT, LMAX>(in_regs, s_q, s_w, s_ip, off, is - I0, ie - I0, pd, x0, w0, L, acc);
            if (tile_fits) {
                __syncthreads();   // everyone is done reading the staged coordinates
                if (in_regs) {
                    // row 2i: [4 off + 2k + beta], row 2i+1: [4 off + 2 len + 2k + beta]
#pragma unroll
                    for (int k = 0; k < LMAX; ++k)
                        if (k < len) {
                            s_stage[4 * off + 2 * k] = acc[0][k];
                            s_stage[4 * off + 2 * k + 1] = acc[1][k];
                            s_stage[4 * off + 2 * len + 2 * k] = acc[2][k];
                            s_stage[4 * off + 2 * len + 2 * k + 1] = acc[3][k];
                        }
                } else if (zero_row) {
                    for (int k = 0; k < 4 * len; ++k) s_stage[4 * off + k] = 0.0;
                }
                __syncthreads();
                tile_store(out.o[3] + 4 * (int64_t)E0, s_stage, 4 * Ew, lane, accumulate);
                __syncthreads();
            }
        }
        if (zero_row) {
            // ---- long row or tile too large: the lane's own row, LMAX
            // entries at a time, each chunk summed from zero over the
            // triangles in the register path's order and then stored (or
            // added), so a row's values do not depend on the path it takes.
            // The tile stores above wrote 0 (or added 0) at this row, and the
            // workgroup barrier after them made those stores complete first.
            const int32_t *cr = col_idx + rs;
            int32_t pdg = 0;
            while (pdg < len - 1 && cr[pdg] != (int32_t)i) ++pdg;
            const double xg = q[2 * i], yg = q[2 * i + 1];
            const double wg = O::W ? w[i] : 0.0;
            for (int32_t c0 = 0; c0 < len; c0 += LMAX) {
                if constexpr (MS != 0) {
                    double ch[NS][LMAX];
                    chunk_sum<MS, LMAX>(q, w, cr, inc_pos, is, ie, c0, pdg, xg, yg, wg, L, ch);
#pragma unroll
                    for (int k = 0; k < LMAX; ++k) {
                        const int32_t e = c0 + k;
                        if (e >= len) break;
#pragma unroll
                        for (int m = 0; m < NS; ++m) {
                            double *o = out.o[m] + rs + e;
                            if (accumulate) *o += ch[m][k];
                            else *o = ch[m][k];
                        }
                    }
                }
                if constexpr (O::K) {
                    double ch[4][LMAX];
                    chunk_sum<K_BIT, LMAX>(q, w, cr, inc_pos, is, ie, c0, pdg, xg, yg, wg, L, ch);
                    // row 2i: [4 rs + 2e + beta], row 2i+1: [4 rs + 2 len + 2e + beta]
                    double *ok = out.o[3] + 4 * (int64_t)rs;
#pragma unroll
                    for (int k = 0; k < LMAX; ++k) {
                        const int32_t e = c0 + k;
                        if (e >= len) break;
                        const int64_t at[4] = {2 * e, 2 * e + 1, 2 * len + 2 * e, 2 * len + 2 * e + 1};
#pragma unroll
                        for (int z = 0; z < 4; ++z) {
                            if (accumulate) ok[at[z]] += ch[z][k];
                            else ok[at[z]] = ch[z][k];
                        }
                    }
                }
            }
        }
    }
}

// ------------------------------------------------------------------ row owner, fan order
//
// With the fan codes of fem_fan_plan, a lane walks the triangles of its row
// in the order they are met turning around the vertex: step j is the
// triangle (i, s_j, s_{j+1}), so slot s_j receives the c2 term of step j-1
// and the c1 term of step j -- two terms, whose floating-point sum does not
// depend on their order, hence the same bits as the ascending-triangle sum
// -- and no per-triangle search over the row's slots is needed.  The
// diagonal sums its terms in walk order.  Each neighbour is gathered once,
// into a register of its walk position (the row's own coordinates are read
// coalesced), so the gathered records need no LDS; LDS only transposes the
// finished values for coalesced stores.  Rows without a fan code are summed
// per lane in ascending triangle order (the chunk path of k_rows_reg).

// One walk over the fan of the lane's row, each value written into the LDS
// transposition buffer as soon as it is complete: slot s_j (j >= 1) after
// step j (c2 of step j-1 plus c1 of step j), s_0 at the end (closed fans:
// c1 of step 0 plus c2 of the last step) or after step 0 (open fans, where
// the last slot gets the last c2 alone), the diagonal at the end.  Scalar
// operator m of PM goes to buf[m EB + off + slot]; the elasticity block of
// a slot to buf[4 off + 2 slot + beta] (row 2i) and buf[4 off + 2 len +
// 2 slot + beta] (row 2i+1).
template <int PM, int N, int EB>
__device__ __forceinline__ void fan_walk_lds(uint64_t code, int n, bool closed, double2 xi, double wi,
                                             const double2 (&x)[N], const double (&wn)[N], Lame L,
                                             double *buf, int32_t off, int32_t len) {
    using O = Ops<PM>;
    constexpr int NV = O::NV;
    auto put_lds = [&](int sl, const double (&val)[NV]) {
#pragma unroll
        for (int m = 0; m < O::NS; ++m) buf[m * EB + off + sl] = val[m];
        if constexpr (O::K) {
            *reinterpret_cast<double2 *>(buf + 4 * off + 2 * sl) = make_double2(val[O::NS], val[O::NS + 1]);
            *reinterpret_cast<double2 *>(buf + 4 * off + 2 * len + 2 * sl) =
                make_double2(val[O::NS + 2], val[O::NS + 3]);
        }
    };
    double dg[NV], carry[NV], first[NV];
#pragma unroll
    for (int m = 0; m < NV; ++m) dg[m] = carry[m] = first[m] = 0.0;
    const int d = closed ? n : n - 1;
#pragma unroll
    for (int j = 0; j < N; ++j) {
        if (j < d) {
            const bool wrap = j + 1 >= n;   // last step of a closed fan: back to s_0
            const int jn = j + 1 < N ? j + 1 : 0;
            const double2 x2 = wrap ? x[0] : x[jn];
            const double w2 = wrap ? wn[0] : wn[jn];
            double c[O::NS > 0 ? O::NS : 1][3];
            double ce[3][4];
            elem_row<PM>(xi.x, xi.y, x[j].x, x[j].y, x2.x, x2.y, wi, wn[j], w2, L, c, ce);
            double c1[NV], c2[NV];
#pragma unroll
            for (int m = 0; m < O::NS; ++m) {
                dg[m] += c[m][0];
                c1[m] = c[m][1];
                c2[m] = c[m][2];
            }
            if constexpr (O::K) {
#pragma unroll
                for (int z = 0; z < 4; ++z) {
                    dg[O::NS + z] += ce[0][z];
                    c1[O::NS + z] = ce[1][z];
                    c2[O::NS + z] = ce[2][z];
                }
            }
            if (j == 0) {
#pragma unroll
                for (int m = 0; m < NV; ++m) first[m] = c1[m];
                if (!closed) put_lds(fan_slot(code, 0), first);
            } else {
                double val[NV];
#pragma unroll
                for (int m = 0; m < NV; ++m) val[m] = carry[m] + c1[m];
                put_lds(fan_slot(code, j), val);
            }
#pragma unroll
            for (int m = 0; m < NV; ++m) carry[m] = c2[m];
        }
    }
    if (closed) {
        double val[NV];
#pragma unroll
        for (int m = 0; m < NV; ++m) val[m] = first[m] + carry[m];
        put_lds(fan_slot(code, 0), val);
    } else {
        put_lds(fan_slot(code, n - 1), carry);
    }
    put_lds(fan_pd(code), dg);
}

// Stores one value of the lane's own row (fallback paths).
__device__ __forceinline__ void put(double *o, int64_t e, double v, int accumulate) {
    if (accumulate) o[e] += v;
    else o[e] = v;
}

// The fan walk of one row from global memory, every value stored directly
// (fan rows longer than the register walk, or in a tile too large for LDS).
// Same steps and order of additions as fan_walk_lds.
template <int MASK>
__device__ void fan_row_global(int64_t i, int32_t rs, int32_t len, uint64_t code,
                               const double2 *__restrict__ q2, const double *__restrict__ w,
                               const int32_t *__restrict__ col_idx, Outs out, Lame L,
                               int accumulate) {
    using O = Ops<MASK>;
    constexpr int NS = O::NS, NV = O::NV;
    const int n = fan_n(code);
    const bool closed = fan_closed(code);
    const int d = closed ? n : n - 1;
    const int32_t *cr = col_idx + rs;
    const double2 xi = q2[i];
    const double wi = O::W ? w[i] : 0.0;
    const int64_t j0 = cr[fan_slot(code, 0)];
    const double2 x0 = q2[j0];
    const double w0 = O::W ? w[j0] : 0.0;
    double2 xa = x0;
    double wa = w0;
    double dg[NV], carry[NV], first[NV];
#pragma unroll
    for (int m = 0; m < NV; ++m) dg[m] = carry[m] = first[m] = 0.0;
    // slot s of operator m (K: z-th value of the 2 x 2 block) of this row
    auto store = [&](int m, int sl, double val) {
        if (m < NS) {
            put(out.o[m] + rs, sl, val, accumulate);
        } else {
            const int z = m - NS;
            const int64_t at = 4 * (int64_t)rs + (z >= 2 ? 2 * len : 0) + 2 * sl + (z & 1);
            put(out.o[3], at, val, accumulate);
        }
    };
    for (int j = 0; j < d; ++j) {
        const bool wrap = j + 1 >= n;
        double2 xb = x0;
        double wb = w0;
        if (!wrap) {
            const int64_t jb = cr[fan_slot(code, j + 1)];
            xb = q2[jb];
            wb = O::W ? w[jb] : 0.0;
        }
        double c[NS > 0 ? NS : 1][3];
        double ce[3][4];
        elem_row<MASK>(xi.x, xi.y, xa.x, xa.y, xb.x, xb.y, wi, wa, wb, L, c, ce);
        double c0[NV], c1[NV], c2[NV];
#pragma unroll
        for (int m = 0; m < NS; ++m) {
            c0[m] = c[m][0];
            c1[m] = c[m][1];
            c2[m] = c[m][2];
        }
        if constexpr (O::K) {
#pragma unroll
            for (int z = 0; z < 4; ++z) {
                c0[NS + z] = ce[0][z];
                c1[NS + z] = ce[1][z];
                c2[NS + z] = ce[2][z];
            }
        }
#pragma unroll
        for (int m = 0; m < NV; ++m) {
            dg[m] += c0[m];
            if (j == 0) first[m] = c1[m];
            else store(m, fan_slot(code, j), carry[m] + c1[m]);
            carry[m] = c2[m];
        }
        xa = xb;
        wa = wb;
    }
#pragma unroll
    for (int m = 0; m < NV; ++m) {
        if (closed) {
            store(m, fan_slot(code, 0), first[m] + carry[m]);
        } else {
            store(m, fan_slot(code, 0), first[m]);
            store(m, fan_slot(code, n - 1), carry[m]);
        }
        store(m, fan_pd(code), dg[m]);
    }
}

template <int MASK, int U, int N>
__global__ __launch_bounds__(WAVE) void k_rows_fan(
    int32_t nq, const double *__restrict__ q, const double *__restrict__ w,
    const double4 *__restrict__ qw, const int32_t *__restrict__ row_ptr,
    const int32_t *__restrict__ col_idx, const int32_t *__restrict__ inc_ptr,
    const uint32_t *__restrict__ inc_pos, const uint64_t *__restrict__ fan, Outs out, Lame L,
    int accumulate, int64_t ntiles) {
    using O = Ops<MASK>;
    constexpr int MS = MASK & (M_BIT | W_BIT | S_BIT);   // scalar operators (phase 1)
    constexpr int NS = O::NS;
    constexpr int EB = U * WAVE;
    // LDS: the transposition buffer, NS EB doubles for the scalar operators
    // (all at once) and 4 EB for the 2 x 2 blocks of K.
    extern __shared__ double smem[];
    const int lane = threadIdx.x;
    const double2 *q2 = reinterpret_cast<const double2 *>(q);

    for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const int64_t r0 = tile * WAVE;
        const int64_t r1 = (r0 + WAVE < nq) ? r0 + WAVE : nq;
        const int64_t i = r0 + lane;
        const bool active = i < nq;
        const int32_t E0 = row_ptr[r0], E1 = row_ptr[r1];
        const int32_t rs = active ? row_ptr[i] : 0;
        const int32_t re = active ? row_ptr[i + 1] : 0;
        const uint64_t code = active ? fan[i] : 0;
        const int32_t Ew = E1 - E0, len = re - rs;
        const int n = fan_n(code);
        const bool closed = fan_closed(code);
        const bool tile_fits = Ew <= EB;
        const bool fan_row = active && n >= 2 && len == n + 1;
        const bool in_regs = tile_fits && fan_row && n <= N;
        const int32_t off = rs - E0;

        // ---- gathers: the neighbours in walk order, the row's own vertex
        int32_t cj[N];
#pragma unroll
        for (int j = 0; j < N; ++j) cj[j] = (in_regs && j < n) ? col_idx[rs + fan_slot(code, j)] : -1;
        double2 x[N];
        double wn[N];
        double2 xi = make_double2(0.0, 0.0);
        double wi = 0.0;
        if (O::W && qw) {
            double4 r[N];
#pragma unroll
            for (int j = 0; j < N; ++j) r[j] = cj[j] >= 0 ? qw[cj[j]] : make_double4(0.0, 0.0, 0.0, 0.0);
            const double4 ri = in_regs ? qw[i] : make_double4(0.0, 0.0, 0.0, 0.0);
#pragma unroll
            for (int j = 0; j < N; ++j) {
                x[j] = make_double2(r[j].x, r[j].y);
                wn[j] = r[j].z;
            }
            xi = make_double2(ri.x, ri.y);
            wi = ri.z;
        } else {
#pragma unroll
            for (int j = 0; j < N; ++j) {
                x[j] = cj[j] >= 0 ? q2[cj[j]] : make_double2(0.0, 0.0);
                wn[j] = (O::W && cj[j] >= 0) ? w[cj[j]] : 0.0;
            }
            if (in_regs) {
                xi = q2[i];
                if constexpr (O::W) wi = w[i];
            }
        }
        const bool zero_row = !in_regs && active && len > 0;

        if constexpr (MS != 0) {
            // ---- phase 1: the scalar operators, all transposed at once
            if (tile_fits) {
                if (in_regs) {
                    fan_walk_lds<MS, N, EB>(code, n, closed, xi, wi, x, wn, L, smem, off, len);
                } else if (zero_row) {
#pragma unroll
                    for (int m = 0; m < NS; ++m)
                        for (int k = 0; k < len; ++k) smem[m * EB + off + k] = 0.0;
                }
                __syncthreads();
#pragma unroll
                for (int m = 0; m < NS; ++m) tile_store(out.o[m] + E0, smem + m * EB, Ew, lane, accumulate);
                __syncthreads();
            }
        }
        if constexpr (O::K) {
            // ---- phase 2: elasticity 2 x 2 blocks.  Row 2i: [4 off + 2 s + beta],
            // row 2i+1: [4 off + 2 len + 2 s + beta]
            if (tile_fits) {
                if (in_regs) {
                    fan_walk_lds<K_BIT, N, EB>(code, n, closed, xi, wi, x, wn, L, smem, off, len);
                } else if (zero_row) {
                    for (int k = 0; k < 4 * len; ++k) smem[4 * off + k] = 0.0;
                }
                __syncthreads();
                tile_store(out.o[3] + 4 * (int64_t)E0, smem, 4 * Ew, lane, accumulate);
                __syncthreads();
            }
        }
        if (zero_row) {
            // ---- fan rows the registers or the tile cannot hold: the same walk
            // from global memory; rows without a fan: ascending triangle order,
            // LMAX_REG entries at a time (as k_rows_reg).  The tile stores above
            // wrote 0 (or added 0) here, and their barrier ordered them first.
            if (fan_row) {
                fan_row_global<MASK>(i, rs, len, code, q2, w, col_idx, out, L, accumulate);
            } else {
                constexpr int LM = 8;
                const int32_t *cr = col_idx + rs;
                const int32_t is = inc_ptr[i], ie = inc_ptr[i + 1];
                int32_t pdg = 0;
                while (pdg < len - 1 && cr[pdg] != (int32_t)i) ++pdg;
                const double xg = q[2 * i], yg = q[2 * i + 1];
                const double wg = O::W ? w[i] : 0.0;
                for (int32_t c0 = 0; c0 < len; c0 += LM) {
                    if constexpr (MS != 0) {
                        double ch[NS][LM];
                        chunk_sum<MS, LM>(q, w, cr, inc_pos, is, ie, c0, pdg, xg, yg, wg, L, ch);
#pragma unroll
                        for (int k = 0; k < LM; ++k) {
                            const int32_t e = c0 + k;
                            if (e >= len) break;
#pragma unroll
                            for (int m = 0; m < NS; ++m) put(out.o[m] + rs, e, ch[m][k], accumulate);
                        }
                    }
                    if constexpr (O::K) {
                        double ch[4][LM];
                        chunk_sum<K_BIT, LM>(q, w, cr, inc_pos, is, ie, c0, pdg, xg, yg, wg, L, ch);
                        double *ok = out.o[3] + 4 * (int64_t)rs;
#pragma unroll
                        for (int k = 0; k < LM; ++k) {
                            const int32_t e = c0 + k;
                            if (e >= len) break;
                            put(ok, 2 * e, ch[0][k], accumulate);
                            put(ok, 2 * e + 1, ch[1][k], accumulate);
                            put(ok, 2 * len + 2 * e, ch[2][k], accumulate);
                            put(ok, 2 * len + 2 * e + 1, ch[3][k], accumulate);
                        }
                    }
                }
            }
        }
    }
}

// ------------------------------------------------------------------ triangle + atomics

template <int MASK>
__global__ __launch_bounds__(256) void k_elem_atomic(int32_t nme, const double *__restrict__ q,
                                                     const double *__restrict__ w,
                                                     const int32_t *__restrict__ me,
                                                     const int32_t *__restrict__ slot,
                                                     const int32_t *__restrict__ row_ptr, Outs out,
                                                     Lame L) {
    using O = Ops<MASK>;
    constexpr int NS = O::NS;
    constexpr int NSA = NS > 0 ? NS : 1;
    const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (k >= nme) return;
    const int32_t v[3] = {me[3 * k], me[3 * k + 1], me[3 * k + 2]};
    double x[3], y[3], wl[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const double2 qc = reinterpret_cast<const double2 *>(q)[v[a]];
        x[a] = qc.x;
        y[a] = qc.y;
        wl[a] = O::W ? w[v[a]] : 0.0;
    }
    int32_t sl[9];
#pragma unroll
    for (int r = 0; r < 9; ++r) sl[r] = slot[(int64_t)r * nme + k];
    // rows a = 0, 1, 2 of the element matrices via the cyclic rotations
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const int a1 = (a + 1) % 3, a2 = (a + 2) % 3;
        double c[NSA][3];
        double ce[3][4];
        elem_row<MASK>(x[a], y[a], x[a1], y[a1], x[a2], y[a2], wl[a], wl[a1], wl[a2], L, c, ce);
        const int bcol[3] = {a, a1, a2};
#pragma unroll
        for (int bb = 0; bb < 3; ++bb) {
            const int32_t p = sl[3 * bcol[bb] + a];
#pragma unroll
            for (int m = 0; m < NS; ++m) unsafeAtomicAdd(out.o[m] + p, c[m][bb]);
        }
        if constexpr (O::K) {
            const int32_t rs = row_ptr[v[a]];
            const int32_t len = row_ptr[v[a] + 1] - rs;
#pragma unroll
            for (int bb = 0; bb < 3; ++bb) {
                const int32_t p = sl[3 * bcol[bb] + a] - rs;
                const int64_t base = 4 * (int64_t)rs + 2 * p;
                unsafeAtomicAdd(out.o[3] + base, ce[bb][0]);
                unsafeAtomicAdd(out.o[3] + base + 1, ce[bb][1]);
                unsafeAtomicAdd(out.o[3] + base + 2 * len, ce[bb][2]);
                unsafeAtomicAdd(out.o[3] + base + 2 * len + 1, ce[bb][3]);
            }
        }
    }
}

// ------------------------------------------------------------------ host side

namespace {

constexpr int DEFAULT_EB = 512;

struct Args {
    int ops;
    int32_t nq, nme;
    int64_t nnz;
    const double *q, *w;
    const int32_t *me, *row_ptr, *col_idx, *inc_ptr, *slot;
    const uint32_t *inc_pos;
    const uint64_t *fan;   // fan codes of fem_fan_plan, or NULL
    double *vals[4];   // M, Mw, S, K
    Lame L;
    void *work;
    size_t work_bytes;
    int flags;
    hipStream_t s;
};

template <int MASK>
size_t lds_bytes(int eb) {
    using O = Ops<MASK>;
    return (size_t)eb * (8 * O::NS + (O::K ? 32 : 0) + 16 + (O::W ? 8 : 0) + 4);
}

// scalar outputs are compacted in M, Mw, S order; K stays in slot 3
Outs outs_for(const Args &a) {
    Outs o{{nullptr, nullptr, nullptr, a.vals[3]}};
    int m = 0;
    for (int b = 0; b < 3; ++b)
        if (a.ops & (1 << b)) o.o[m++] = a.vals[b];
    return o;
}

constexpr int LMAX_REG = 8;   // row entries kept in registers by k_rows_reg

template <int MASK>
size_t lds_bytes_reg(int eb) {
    using O = Ops<MASK>;
    const int sd = O::K ? 4 : (O::W ? 3 : 2);
    return (size_t)eb * (8 * sd + 4);
}

template <int MASK, int U>
int launch_reg_u(const Args &a, const double4 *qw, int grid_blocks) {
    const int64_t ntiles = (a.nq + WAVE - 1) / WAVE;
    const int64_t grid = grid_blocks > 0 ? (grid_blocks < ntiles ? grid_blocks : ntiles) : ntiles;
    FEM_REQUIRE(grid <= INT32_MAX, FEM_EOVERFLOW, "too many tiles");
    const size_t lds = lds_bytes_reg<MASK>(U * WAVE);
    hipLaunchKernelGGL((k_rows_reg<MASK, U, LMAX_REG>), dim3((unsigned)grid), dim3(WAVE), lds, a.s,
                       a.nq, a.q, a.w, qw, a.row_ptr, a.col_idx, a.inc_ptr, a.inc_pos, outs_for(a),
                       a.L, (a.flags & FEM_ACCUMULATE) ? 1 : 0, ntiles);
    FEM_LAUNCH_CHECK();
    return FEM_OK;
}

template <int MASK>
int launch_reg(const Args &a, const double4 *qw, int eb, int grid_blocks) {
    if (eb <= 0) eb = DEFAULT_EB;
    const int u = (eb + WAVE - 1) / WAVE;
    if (u <= 4) return launch_reg_u<MASK, 4>(a, qw, grid_blocks);
    if (u <= 7) return launch_reg_u<MASK, 7>(a, qw, grid_blocks);
    if (u <= 8) return launch_reg_u<MASK, 8>(a, qw, grid_blocks);
    if (u <= 10) return launch_reg_u<MASK, 10>(a, qw, grid_blocks);
    if (u <= 12) return launch_reg_u<MASK, 12>(a, qw, grid_blocks);
    return launch_reg_u<MASK, 16>(a, qw, grid_blocks);
}

constexpr int FAN_REG = 8;   // neighbour slots walked in registers by k_rows_fan

template <int MASK, int U>
int launch_fan_u(const Args &a, const double4 *qw, int grid_blocks) {
    const int64_t ntiles = (a.nq + WAVE - 1) / WAVE;
    const int64_t grid = grid_blocks > 0 ? (grid_blocks < ntiles ? grid_blocks : ntiles) : ntiles;
    FEM_REQUIRE(grid <= INT32_MAX, FEM_EOVERFLOW, "too many tiles");
    constexpr int NS = Ops<MASK>::NS;
    const size_t lds = (size_t)U * WAVE * 8 * (Ops<MASK>::K ? (NS > 4 ? NS : 4) : NS);
    hipLaunchKernelGGL((k_rows_fan<MASK, U, FAN_REG>), dim3((unsigned)grid), dim3(WAVE), lds, a.s,
                       a.nq, a.q, a.w, qw, a.row_ptr, a.col_idx, a.inc_ptr, a.inc_pos, a.fan,
                       outs_for(a), a.L, (a.flags & FEM_ACCUMULATE) ? 1 : 0, ntiles);
    FEM_LAUNCH_CHECK();
    return FEM_OK;
}

template <int MASK>
int launch_fan(const Args &a, const double4 *qw, int eb, int grid_blocks) {
    if (eb <= 0) eb = DEFAULT_EB;
    const int u = (eb + WAVE - 1) / WAVE;
    if (u <= 4) return launch_fan_u<MASK, 4>(a, qw, grid_blocks);
    if (u <= 7) return launch_fan_u<MASK, 7>(a, qw, grid_blocks);
    if (u <= 8) return launch_fan_u<MASK, 8>(a, qw, grid_blocks);
    if (u <= 10) return launch_fan_u<MASK, 10>(a, qw, grid_blocks);
    if (u <= 12) return launch_fan_u<MASK, 12>(a, qw, grid_blocks);
    return launch_fan_u<MASK, 16>(a, qw, grid_blocks);
}

template <int MASK, int U>
int launch_rows_u(const Args &a, const double4 *qw, int grid_blocks) {
    const int64_t ntiles = (a.nq + WAVE - 1) / WAVE;
    const int64_t grid = grid_blocks > 0 ? (grid_blocks < ntiles ? grid_blocks : ntiles) : ntiles;
    FEM_REQUIRE(grid <= INT32_MAX, FEM_EOVERFLOW, "too many tiles");
    const size_t lds = lds_bytes<MASK>(U * WAVE);
    FEM_REQUIRE(lds <= 64 * 1024, FEM_EINVAL, "lds_entries %d needs %zu bytes of LDS (limit 65536)",
                U * WAVE, lds);
    hipLaunchKernelGGL((k_rows_numeric<MASK, U>), dim3((unsigned)grid), dim3(WAVE), lds, a.s, a.nq,
                       a.q, a.w, qw, a.row_ptr, a.col_idx, a.inc_ptr, a.inc_pos, outs_for(a), a.L,
                       (a.flags & FEM_ACCUMULATE) ? 1 : 0, ntiles);
    FEM_LAUNCH_CHECK();
    return FEM_OK;
}

template <int MASK>
int launch_rows(const Args &a, const double4 *qw, int eb, int grid_blocks) {
    if (eb <= 0) eb = DEFAULT_EB;
    int u = (eb + WAVE - 1) / WAVE;
    // keep the LDS tile within 64 KiB for the wide operator sets
    while (u > 4 && lds_bytes<MASK>(u * WAVE) > 64 * 1024) --u;
    if (u <= 4) return launch_rows_u<MASK, 4>(a, qw, grid_blocks);
    if (u <= 7) return launch_rows_u<MASK, 7>(a, qw, grid_blocks);
    if (u <= 8) return launch_rows_u<MASK, 8>(a, qw, grid_blocks);
    if (u <= 10) return launch_rows_u<MASK, 10>(a, qw, grid_blocks);
    if (u <= 12) return launch_rows_u<MASK, 12>(a, qw, grid_blocks);
    return launch_rows_u<MASK, 16>(a, qw, grid_blocks);
}

template <int MASK>
int launch_atomic(const Args &a) {
    using O = Ops<MASK>;
    if (!(a.flags & FEM_ACCUMULATE)) {
        int st;
        for (int b = 0; b < 3; ++b)
            if ((MASK & (1 << b)) && (st = fill_f64(a.vals[b], a.nnz, 0.0, a.s))) return st;
        if (O::K && (st = fill_f64(a.vals[3], 4 * a.nnz, 0.0, a.s))) return st;
    }
    if (a.nme == 0) return FEM_OK;
    hipLaunchKernelGGL(k_elem_atomic<MASK>, dim3(grid_for(a.nme, 256)), dim3(256), 0, a.s, a.nme,
                       a.q, a.w, a.me, a.slot, a.row_ptr, outs_for(a), a.L);
    FEM_LAUNCH_CHECK();
    return FEM_OK;
}

template <int MASK>
int run_mask(const Args &a, const double4 *qw, const fem_tune *tune) {
    if (a.flags & FEM_ATOMIC) return launch_atomic<MASK>(a);
    const int eb = tune ? tune->lds_entries : 0, grid = tune ? tune->grid_blocks : 0;
    if (tune && tune->variant == 1) return launch_rows<MASK>(a, qw, eb, grid);
    if (a.fan) return launch_fan<MASK>(a, qw, eb, grid);
    return launch_reg<MASK>(a, qw, eb, grid);
}

inline size_t qw_bytes(int32_t nq) { return (sizeof(double4) * (size_t)nq + 255) & ~size_t(255); }

int run_ops(const Args &a, const fem_tune *tune);

int run(const char *fn, const Args &a, const fem_tune *tune) {
    FEM_REQUIRE(a.ops >= 1 && a.ops <= 15, FEM_EINVAL, "%s: ops must be a nonzero subset of FEM_OP_*", fn);
    FEM_REQUIRE(a.nq >= 1 && a.nme >= 0 && a.nnz >= 0, FEM_EINVAL, "%s: bad sizes nq=%d nme=%d nnz=%lld",
                fn, a.nq, a.nme, (long long)a.nnz);
    FEM_REQUIRE(a.nnz <= INT32_MAX && (!(a.ops & K_BIT) || 4 * a.nnz <= INT32_MAX), FEM_EOVERFLOW,
                "%s: nnz exceeds int32 indexing", fn);
    FEM_REQUIRE((a.flags & ~(FEM_ATOMIC | FEM_ACCUMULATE | FEM_CHECK_AREA | FEM_PACKED_QW)) == 0,
                FEM_EINVAL, "%s: unknown flags 0x%x", fn, a.flags);
    if (a.flags & FEM_PACKED_QW) {
        FEM_REQUIRE((a.ops & W_BIT) && !(a.flags & FEM_ATOMIC), FEM_EINVAL,
                    "%s: FEM_PACKED_QW needs FEM_OP_WMASS and the row-owner scheme", fn);
        FEM_REQUIRE(a.work && a.work_bytes >= sizeof(double4) * (size_t)a.nq, FEM_ENOSPC,
                    "%s: FEM_PACKED_QW needs the workspace that holds the packed records", fn);
    }
    FEM_REQUIRE(a.q && a.row_ptr, FEM_EINVAL, "%s: NULL q or row_ptr", fn);
    for (int b = 0; b < 4; ++b)
        FEM_REQUIRE(!(a.ops & (1 << b)) || a.nnz == 0 || a.vals[b], FEM_EINVAL, "%s: NULL output", fn);
    FEM_REQUIRE(!(a.ops & W_BIT) || a.w, FEM_EINVAL, "%s: NULL w", fn);
    FEM_REQUIRE(!(a.ops & K_BIT) || a.L.lam + a.L.mu > 0.0, FEM_EINVAL,
                "%s: need lambda + mu > 0 (got %g)", fn, a.L.lam + a.L.mu);
    if (a.flags & FEM_ATOMIC) {
        FEM_REQUIRE(a.nme == 0 || (a.me && a.slot), FEM_EINVAL, "%s: FEM_ATOMIC needs me and slot", fn);
    } else {
        FEM_REQUIRE(a.nnz == 0 || (a.col_idx && a.inc_ptr && a.inc_pos), FEM_EINVAL,
                    "%s: NULL col_idx, inc_ptr or inc_pos", fn);
    }
    // zero-area check: its flag lives after the packed records
    int *area_flag = nullptr;
    if (a.flags & FEM_CHECK_AREA) {
        const size_t off = (a.ops & W_BIT) ? qw_bytes(a.nq) : 0;
        FEM_REQUIRE(a.work && a.work_bytes >= off + sizeof(int), FEM_ENOSPC,
                    "%s: FEM_CHECK_AREA needs the workspace of fem_assemble_workspace", fn);
        FEM_REQUIRE(a.nme == 0 || a.me, FEM_EINVAL, "%s: FEM_CHECK_AREA needs me", fn);
        area_flag = reinterpret_cast<int *>(static_cast<char *>(a.work) + off);
        int st;
        if ((st = fill_i32(area_flag, 1, 0, a.s))) return st;
        if (a.nme > 0) {
            hipLaunchKernelGGL(k_check_area, dim3(grid_for(a.nme, 256)), dim3(256), 0, a.s, a.nme,
                               reinterpret_cast<const double2 *>(a.q), a.me, area_flag);
            FEM_LAUNCH_CHECK();
        }
    }
    const int st = run_ops(a, tune);
    if (st || !area_flag) return st;
    int hflag = 0;
    FEM_HIP_CHECK(hipMemcpyAsync(&hflag, area_flag, sizeof(int), hipMemcpyDeviceToHost, a.s));
    FEM_HIP_CHECK(hipStreamSynchronize(a.s));
    FEM_REQUIRE(!hflag, FEM_EDEGEN, "%s: a triangle has zero area", fn);
    return FEM_OK;
}

int run_ops(const Args &a, const fem_tune *tune) {
    // packed (x, y, w) records when the weighted mass is requested and a
    // workspace is given: one random access per column instead of two.
    // FEM_PACKED_QW: the workspace holds them already (same q and w)
    const double4 *qw = nullptr;
    if ((a.ops & W_BIT) && !(a.flags & FEM_ATOMIC) && a.work &&
        a.work_bytes >= sizeof(double4) * (size_t)a.nq) {
        double4 *p = static_cast<double4 *>(a.work);
        if (!(a.flags & FEM_PACKED_QW)) {
            hipLaunchKernelGGL(k_pack_qw, dim3(grid_for(a.nq, 256)), dim3(256), 0, a.s, a.nq,
                               reinterpret_cast<const double2 *>(a.q), a.w, p);
            FEM_LAUNCH_CHECK();
        }
        qw = p;
    }
    switch (a.ops) {
    case 1: return run_mask<1>(a, qw, tune);
    case 2: return run_mask<2>(a, qw, tune);
    case 3: return run_mask<3>(a, qw, tune);
    case 4: return run_mask<4>(a, qw, tune);
    case 5: return run_mask<5>(a, qw, tune);
    case 6: return run_mask<6>(a, qw, tune);
    case 7: return run_mask<7>(a, qw, tune);
    case 8: return run_mask<8>(a, qw, tune);
    case 9: return run_mask<9>(a, qw, tune);
    case 10: return run_mask<10>(a, qw, tune);
    case 11: return run_mask<11>(a, qw, tune);
    case 12: return run_mask<12>(a, qw, tune);
    case 13: return run_mask<13>(a, qw, tune);
    case 14: return run_mask<14>(a, qw, tune);
    default: return run_mask<15>(a, qw, tune);
    }
}

Args make_args(int ops, int32_t nq, int32_t nme, int64_t nnz, const double *q, const double *w,
               const int32_t *me, const int32_t *row_ptr, const int32_t *col_idx,
               const int32_t *inc_ptr, const uint32_t *inc_pos, const uint64_t *fan,
               const int32_t *slot, double lam, double mu, double *vM, double *vW, double *vS,
               double *vK, void *work, size_t work_bytes, int flags, void *stream) {
    Args a{};
    a.ops = ops;
    a.nq = nq;
    a.nme = nme;
    a.nnz = nnz;
    a.q = q;
    a.w = w;
    a.me = me;
    a.row_ptr = row_ptr;
    a.col_idx = col_idx;
    a.inc_ptr = inc_ptr;
    a.inc_pos = inc_pos;
    a.fan = fan;
    a.slot = slot;
    a.L = {lam, mu};
    a.vals[0] = vM;
    a.vals[1] = vW;
    a.vals[2] = vS;
    a.vals[3] = vK;
    a.work = work;
    a.work_bytes = work_bytes;
    a.flags = flags;
    a.s = as_stream(stream);
    return a;
}

}  // namespace
}  // namespace fem

using namespace fem;

extern "C" int fem_assemble_workspace(int32_t nq, int ops, size_t *bytes) {
    clear_error();
    FEM_REQUIRE(bytes && nq >= 1, FEM_EINVAL, "fem_assemble_workspace: bad arguments");
    *bytes = ((ops & FEM_OP_WMASS) ? qw_bytes(nq) : 0) + 256;
    return FEM_OK;
}

extern "C" int fem_assemble(int ops, int32_t nq, int32_t nme, int64_t nnz, const double *q,
                            const double *w, const int32_t *me, const int32_t *row_ptr,
                            const int32_t *col_idx, const int32_t *inc_ptr, const uint32_t *inc_pos,
                            const uint64_t *fan, const int32_t *slot, double lambda, double mu,
                            double *vals_M,
                            double *vals_Mw, double *vals_S, double *vals_K, void *work,
                            size_t work_bytes, const fem_tune *tune, int flags, void *stream) {
    clear_error();
    Args a = make_args(ops, nq, nme, nnz, q, w, me, row_ptr, col_idx, inc_ptr, inc_pos, fan, slot,
                       lambda, mu, vals_M, vals_Mw, vals_S, vals_K, work, work_bytes, flags, stream);
    return run("fem_assemble", a, tune);
}

// ------------------------------------------------------------ gather probe
//
// Measurement aid: the random accesses of the row-owner kernels without
// their arithmetic.  Every entry e of the column stream reads col_idx[e] and
// the 16-byte record q[col_idx[e]] (mode 0), or the record q[e mod nq] in
// stream order instead (mode 1: the same loads with perfect locality); the
// sums go to one double per thread so that no load is dropped.
namespace fem {
__global__ __launch_bounds__(256) void k_gather_probe(int64_t nnz, int32_t nq,
                                                      const int32_t *__restrict__ col_idx,
                                                      const double2 *__restrict__ q, int mode,
                                                      double *__restrict__ sink) {
    constexpr int H = 8;   // loads in flight per thread
    const int64_t tid = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int64_t nth = (int64_t)gridDim.x * blockDim.x;
    double acc = 0.0;
    for (int64_t e0 = tid; e0 < nnz; e0 += H * nth) {
        int32_t c[H];
#pragma unroll
        for (int h = 0; h < H; ++h) {
            const int64_t e = e0 + h * nth;
            c[h] = e < nnz ? (mode == 0 ? col_idx[e] : (int32_t)(e % nq)) : -1;
        }
        double2 x[H];
#pragma unroll
        for (int h = 0; h < H; ++h) x[h] = c[h] >= 0 ? q[c[h]] : make_double2(0.0, 0.0);
#pragma unroll
        for (int h = 0; h < H; ++h) acc += x[h].x + x[h].y;
    }
    sink[tid] = acc;
}
}  // namespace fem

extern "C" int fem_gather_probe_threads(void) { return 2048 * 256; }

extern "C" int fem_gather_probe(int64_t nnz, int32_t nq, const int32_t *col_idx, const double *q,
                                int mode, double *sink, void *stream) {
    clear_error();
    FEM_REQUIRE(nnz >= 0 && nq >= 1 && (mode == 0 || mode == 1), FEM_EINVAL,
                "fem_gather_probe: bad arguments");
    FEM_REQUIRE(q && sink && (nnz == 0 || col_idx), FEM_EINVAL, "fem_gather_probe: NULL array");
    hipLaunchKernelGGL(k_gather_probe, dim3(2048), dim3(256), 0, as_stream(stream), nnz, nq, col_idx,
                       reinterpret_cast<const double2 *>(q), mode, sink);
    FEM_LAUNCH_CHECK();
    return FEM_OK;
}

// ------------------------------------------------------------ allocation-free variant
//
// fem_assemble without a workspace argument: the packed (x, y, w) records of
// the weighted mass and the FEM_CHECK_AREA flag live in one file-scope device
// array instead.  Every GPU the library runs on holds its own copy for the
// life of the process; host code addresses it only through the pointer
// hipGetSymbolAddress returns on that device (the array's own name is a
// host-side stand-in there, not a device address).
namespace fem {
constexpr size_t NOALLOC_BYTES = size_t(FEM_NOALLOC_MAX_NQ) * 32 + 256;
static __device__ __align__(256) unsigned char scratch[NOALLOC_BYTES];

namespace {
constexpr int NOALLOC_MAX_DEVICES = 64;
std::once_flag g_scratch_once[NOALLOC_MAX_DEVICES];
void *g_scratch_ptr[NOALLOC_MAX_DEVICES];
hipError_t g_scratch_err[NOALLOC_MAX_DEVICES];

// The device address of `scratch` on the current device, looked up once per
// device (with that device current) and kept.
int scratch_for_current_device(void **out) {
    int dev = -1;
    FEM_HIP_CHECK(hipGetDevice(&dev));
    FEM_REQUIRE(dev >= 0 && dev < NOALLOC_MAX_DEVICES, FEM_EUNSUPPORTED,
                "fem_assemble_noalloc: device %d beyond the %d supported", dev, NOALLOC_MAX_DEVICES);
    std::call_once(g_scratch_once[dev], [dev]() {
        void *p = nullptr;
        g_scratch_err[dev] = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        g_scratch_ptr[dev] = g_scratch_err[dev] == hipSuccess ? p : nullptr;
    });
    FEM_REQUIRE(g_scratch_err[dev] == hipSuccess && g_scratch_ptr[dev], FEM_EHIP,
                "fem_assemble_noalloc: hipGetSymbolAddress: %s", hipGetErrorString(g_scratch_err[dev]));
    *out = g_scratch_ptr[dev];
    return FEM_OK;
}
}  // namespace
}  // namespace fem

extern "C" int fem_assemble_noalloc(int ops, int32_t nq, int32_t nme, int64_t nnz, const double *q,
                                    const double *w, const int32_t *me, const int32_t *row_ptr,
                                    const int32_t *col_idx, const int32_t *inc_ptr,
                                    const uint32_t *inc_pos, const uint64_t *fan,
                                    const int32_t *slot, double lambda, double mu, double *vals_M,
                                    double *vals_Mw, double *vals_S, double *vals_K,
                                    const fem_tune *tune, int flags, void *stream) {
    clear_error();
    FEM_REQUIRE(!(flags & FEM_PACKED_QW), FEM_EINVAL,
                "fem_assemble_noalloc: FEM_PACKED_QW is not accepted (the scratch is shared by every "
                "call on the device)");
    const bool packs = (ops & FEM_OP_WMASS) && !(flags & FEM_ATOMIC);
    const bool needs = packs || (flags & FEM_CHECK_AREA);
    FEM_REQUIRE(!needs || (nq >= 0 && nq <= FEM_NOALLOC_MAX_NQ), FEM_ENOSPC,
                "fem_assemble_noalloc: nq = %d exceeds the %d vertices its scratch holds for the "
                "weighted mass or FEM_CHECK_AREA",
                nq, FEM_NOALLOC_MAX_NQ);
    void *scr = nullptr;
    if (needs) {
        int st;
        if ((st = scratch_for_current_device(&scr))) return st;
    }
    Args a = make_args(ops, nq, nme, nnz, q, w, me, row_ptr, col_idx, inc_ptr, inc_pos, fan, slot,
                       lambda, mu, vals_M, vals_Mw, vals_S, vals_K, scr, scr ? NOALLOC_BYTES : 0,
                       flags, stream);
    return run("fem_assemble_noalloc", a, tune);
}

extern "C" int fem_assemble_mass(int32_t nq, int32_t nme, int64_t nnz, const double *q,
                                 const int32_t *me, const int32_t *row_ptr, const int32_t *col_idx,
                                 const int32_t *inc_ptr, const uint32_t *inc_pos,
                                 const uint64_t *fan, const int32_t *slot, double *values, int flags,
                                 void *stream) {
    clear_error();
    Args a = make_args(M_BIT, nq, nme, nnz, q, nullptr, me, row_ptr, col_idx, inc_ptr, inc_pos, fan,
                       slot, 0, 0, values, nullptr, nullptr, nullptr, nullptr, 0, flags, stream);
    return run("fem_assemble_mass", a, nullptr);
}

extern "C" int fem_assemble_wmass(int32_t nq, int32_t nme, int64_t nnz, const double *q,
                                  const int32_t *me, const int32_t *row_ptr, const int32_t *col_idx,
                                  const int32_t *inc_ptr, const uint32_t *inc_pos,
                                  const uint64_t *fan, const int32_t *slot, const double *w,
                                  double *values, int flags,
                                  void *stream) {
    clear_error();
    Args a = make_args(W_BIT, nq, nme, nnz, q, w, me, row_ptr, col_idx, inc_ptr, inc_pos, fan, slot,
                       0, 0, nullptr, values, nullptr, nullptr, nullptr, 0, flags, stream);
    return run("fem_assemble_wmass", a, nullptr);
}

extern "C" int fem_assemble_stiff(int32_t nq, int32_t nme, int64_t nnz, const double *q,
                                  const int32_t *me, const int32_t *row_ptr, const int32_t *col_idx,
                                  const int32_t *inc_ptr, const uint32_t *inc_pos,
                                  const uint64_t *fan, const int32_t *slot, double *values,
                                  int flags, void *stream) {
    clear_error();
    Args a = make_args(S_BIT, nq, nme, nnz, q, nullptr, me, row_ptr, col_idx, inc_ptr, inc_pos, fan,
                       slot, 0, 0, nullptr, nullptr, values, nullptr, nullptr, 0, flags, stream);
    return run("fem_assemble_stiff", a, nullptr);
}

extern "C" int fem_assemble_stiff_mass(int32_t nq, int32_t nme, int64_t nnz, const double *q,
                                       const int32_t *me, const int32_t *row_ptr,
                                       const int32_t *col_idx, const int32_t *inc_ptr,
                                       const uint32_t *inc_pos, const uint64_t *fan,
                                       const int32_t *slot, double *vals_S, double *vals_M,
                                       int flags, void *stream) {
    clear_error();
    Args a = make_args(S_BIT | M_BIT, nq, nme, nnz, q, nullptr, me, row_ptr, col_idx, inc_ptr,
                       inc_pos, fan, slot, 0, 0, vals_M, nullptr, vals_S, nullptr, nullptr, 0, flags,
                       stream);
    return run("fem_assemble_stiff_mass", a, nullptr);
}

extern "C" int fem_assemble_stiff_wmass(int32_t nq, int32_t nme, int64_t nnz, const double *q,
                                        const int32_t *me, const int32_t *row_ptr,
                                        const int32_t *col_idx, const int32_t *inc_ptr,
                                        const uint32_t *inc_pos, const uint64_t *fan,
                                        const int32_t *slot, const double *w, double *vals_S,
                                        double *vals_Mw, int flags,
                                        void *stream) {
    clear_error();
    Args a = make_args(S_BIT | W_BIT, nq, nme, nnz, q, w, me, row_ptr, col_idx, inc_ptr, inc_pos,
                       fan, slot, 0, 0, nullptr, vals_Mw, vals_S, nullptr, nullptr, 0, flags, stream);
    return run("fem_assemble_stiff_wmass", a, nullptr);
}

extern "C" int fem_assemble_elas(int32_t nq, int32_t nme, int64_t nnz, const double *q,
                                 const int32_t *me, const int32_t *row_ptr, const int32_t *col_idx,
                                 const int32_t *inc_ptr, const uint32_t *inc_pos,
                                 const uint64_t *fan, const int32_t *slot, double lambda, double mu,
                                 double *values_e,
                                 int flags, void *stream) {
    clear_error();
    Args a = make_args(K_BIT, nq, nme, nnz, q, nullptr, me, row_ptr, col_idx, inc_ptr, inc_pos, fan,
                       slot, lambda, mu, nullptr, nullptr, nullptr, values_e, nullptr, 0, flags, stream);
    return run("fem_assemble_elas", a, nullptr);
}

extern "C" int fem_assemble_stiff_mass_batched(int32_t nb, int32_t nq, int64_t nnz, const double *q,
                                               const int32_t *row_ptr, const int32_t *col_idx,
                                               const int32_t *inc_ptr, const uint32_t *inc_pos,
                                               const uint64_t *fan, double *vals_S, double *vals_M,
                                               const fem_tune *tune, int flags, void *stream) {
    clear_error();
    FEM_REQUIRE(nb >= 1, FEM_EINVAL, "fem_assemble_stiff_mass_batched: nb must be >= 1");
    FEM_REQUIRE((flags & FEM_ATOMIC) == 0, FEM_EINVAL,
                "fem_assemble_stiff_mass_batched: only the row-owner scheme is batched");
    Args a = make_args(S_BIT | M_BIT, nq, 0, nnz, q, nullptr, nullptr, row_ptr, col_idx, inc_ptr,
                       inc_pos, fan, nullptr, 0, 0, vals_M, nullptr, vals_S, nullptr, nullptr, 0,
                       flags, stream);
    return run("fem_assemble_stiff_mass_batched", a, tune);
}

// -------------------------------------------------------------------- batch helper

namespace fem {
// One lane per connectivity entry; the mesh of triangle k is found by binary
// search of elem_off (nb + 1 sorted offsets, cached).
__global__ __launch_bounds__(256) void k_globalize(int32_t nb, const int64_t *__restrict__ vtx_off,
                                                   const int64_t *__restrict__ elem_off,
                                                   int64_t n3, const int32_t *__restrict__ src,
                                                   int32_t *__restrict__ dst) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n3) return;
    const int64_t k = i / 3;
    int32_t lo = 0, hi = nb;   // largest b with elem_off[b] <= k
    while (hi - lo > 1) {
        const int32_t mid = (lo + hi) >> 1;
        if (elem_off[mid] <= k) lo = mid;
        else hi = mid;
    }
    dst[i] = src[i] + static_cast<int32_t>(vtx_off[lo]);
}
}  // namespace fem

extern "C" int fem_batch_globalize(int32_t nb, int32_t nme, const int64_t *vtx_off,
                                   const int64_t *elem_off, const int32_t *me_local,
                                   int32_t *me_global, void *stream) {
    clear_error();
    FEM_REQUIRE(nb >= 1 && nme >= 0 && vtx_off && elem_off, FEM_EINVAL,
                "fem_batch_globalize: bad arguments");
    FEM_REQUIRE(3 * (int64_t)nme <= INT32_MAX, FEM_EOVERFLOW, "fem_batch_globalize: 3 nme exceeds int32");
    if (nme == 0) return FEM_OK;
    FEM_REQUIRE(me_local && me_global, FEM_EINVAL, "fem_batch_globalize: NULL connectivity");
    const int64_t n3 = 3 * (int64_t)nme;
    hipLaunchKernelGGL(k_globalize, dim3(grid_for(n3, 256)), dim3(256), 0, as_stream(stream), nb,
                       vtx_off, elem_off, n3, me_local, me_global);
    FEM_LAUNCH_CHECK();
    return FEM_OK;
}
