// fem_numeric.hip -- numeric phase: element matrices and their summation
// into the CSR values.
//
// Element formulas (FP64, no MFMA: the work is a gather/scatter bound by HBM,
// not a dense contraction):
//   |T| = |det| / 2, det = (q2-q1) x (q3-q1)
//   mass (eq. MassElem)            |T|/12 [2 1 1; 1 2 1; 1 1 2]
//   weighted mass (eq. MassWElem)  |T|/30 (3w_a + w_b + w_c) on the diagonal,
//                                  |T|/30 (w_a + w_b + w_c/2) off it (c third)
//   stiffness (eq. StiffMatElem)   <r_a, r_b> / (4|T|), r = (q2-q3, q3-q1, q1-q2)
//   elasticity                     |T| B^T C B, gradients r_a^perp / det
//
// Two summation schemes:
//
// FEM_DETERMINISTIC -- row owner.  One lane owns one CSR row (one vertex i)
//   and walks the triangles around i (inc_ptr / inc_pos), computing the row of
//   each element matrix that belongs to i and adding it into the row's
//   entries.  A wave owns 64 consecutive rows, whose entries are contiguous in
//   col_idx/values: it stages that slice in LDS (columns, gathered vertex
//   coordinates, accumulators), so every read of the pattern and every write
//   of values is coalesced and written exactly once; the only random
//   accesses are the gathers of q (and w) by column.  Each element is
//   evaluated once per vertex (three times), which costs flops, not bytes.
//   Every value is summed by one lane in ascending triangle order, so results
//   are bitwise reproducible.
// FEM_ATOMIC -- one lane per triangle computes the full element matrix and
//   adds it through the slot map with FP64 atomics (global_atomic_add_f64).
#include "fem_internal.h"

namespace fem {

enum Op : int { OP_MASS = 0, OP_WMASS, OP_STIFF, OP_STIFF_MASS, OP_STIFF_WMASS, OP_ELAS };

template <int OP> struct OpInfo;
template <> struct OpInfo<OP_MASS> { static constexpr int NACC = 1, NOUT = 1; static constexpr bool W = false; };
template <> struct OpInfo<OP_WMASS> { static constexpr int NACC = 1, NOUT = 1; static constexpr bool W = true; };
template <> struct OpInfo<OP_STIFF> { static constexpr int NACC = 1, NOUT = 1; static constexpr bool W = false; };
template <> struct OpInfo<OP_STIFF_MASS> { static constexpr int NACC = 2, NOUT = 2; static constexpr bool W = false; };
template <> struct OpInfo<OP_STIFF_WMASS> { static constexpr int NACC = 2, NOUT = 2; static constexpr bool W = true; };
template <> struct OpInfo<OP_ELAS> { static constexpr int NACC = 4, NOUT = 1; static constexpr bool W = false; };

struct Lame {
    double lam, mu;
};

// Row of the element matrices that belongs to vertex 0 of the triangle
// (x0, x1, x2), where (0, 1, 2) is a cyclic rotation of the triangle's own
// vertex order (so orientation and the edge vectors r are those of the
// paper's formulas).  c[0] is the diagonal term, c[1] / c[2] the terms of
// columns x1 / x2.  For elasticity c holds the three 2x2 blocks, row-major.
template <int OP>
__device__ __forceinline__ void elem_row(double x0, double y0, double x1, double y1, double x2,
                                         double y2, double w0, double w1, double w2, Lame L,
                                         double (&c)[OpInfo<OP>::NACC][3],
                                         double (&ce)[3][4]) {
    const double e1x = x1 - x0, e1y = y1 - y0;
    const double e2x = x2 - x0, e2y = y2 - y0;
    const double det = e1x * e2y - e2x * e1y;
    const double ad = fabs(det);
    const double area = 0.5 * ad;
    if constexpr (OP == OP_STIFF || OP == OP_STIFF_MASS || OP == OP_STIFF_WMASS) {
        // r0 = x1 - x2, r1 = x2 - x0, r2 = x0 - x1;  S_0b = <r0, rb> / (2 |det|)
        const double r0x = x1 - x2, r0y = y1 - y2;
        const double inv = 1.0 / (2.0 * ad);
        c[0][0] = (r0x * r0x + r0y * r0y) * inv;
        c[0][1] = (r0x * e2x + r0y * e2y) * inv;
        c[0][2] = -(r0x * e1x + r0y * e1y) * inv;
    }
    if constexpr (OP == OP_MASS || OP == OP_STIFF_MASS) {
        constexpr int m = (OP == OP_MASS) ? 0 : 1;
        c[m][0] = area / 6.0;
        c[m][1] = area / 12.0;
        c[m][2] = area / 12.0;
    }
    if constexpr (OP == OP_WMASS || OP == OP_STIFF_WMASS) {
        constexpr int m = (OP == OP_WMASS) ? 0 : 1;
        const double a30 = area / 30.0;
        c[m][0] = a30 * (3.0 * w0 + w1 + w2);
        c[m][1] = a30 * (w0 + w1 + 0.5 * w2);
        c[m][2] = a30 * (w0 + 0.5 * w1 + w2);
    }
    if constexpr (OP == OP_ELAS) {
        // gradients of the barycentric functions: perp(r_a) / det
        const double id = 1.0 / det;
        const double g0x = (y1 - y2) * id, g0y = -(x1 - x2) * id;
        const double g1x = e2y * id, g1y = -e2x * id;
        const double g2x = -e1y * id, g2y = e1x * id;
        const double gx[3] = {g0x, g1x, g2x}, gy[3] = {g0y, g1y, g2y};
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

// ------------------------------------------------------------------ row owner

template <int OP>
__global__ __launch_bounds__(WAVE) void k_rows_numeric(
    int32_t nq, const double *__restrict__ q, const double *__restrict__ w,
    const int32_t *__restrict__ row_ptr, const int32_t *__restrict__ col_idx,
    const int32_t *__restrict__ inc_ptr, const uint32_t *__restrict__ inc_pos,
    double *__restrict__ out0, double *__restrict__ out1, Lame L, int eb, int accumulate,
    int64_t ntiles) {
    using I = OpInfo<OP>;
    constexpr int NACC = I::NACC;
    extern __shared__ double smem[];
    // LDS tile: acc[NACC * eb] | qx[eb] | qy[eb] | (w[eb]) | col[eb] (int32)
    double *s_acc = smem;
    double *s_qx = s_acc + (size_t)NACC * eb;
    double *s_qy = s_qx + eb;
    double *s_w = s_qy + eb;
    int32_t *s_col = reinterpret_cast<int32_t *>(s_w + (I::W ? eb : 0));
    const int lane = threadIdx.x;

    for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const int64_t r0 = tile * WAVE;
        const int64_t r1 = (r0 + WAVE < nq) ? r0 + WAVE : nq;
        const int64_t i = r0 + lane;
        const bool active = i < nq;
        const int32_t E0 = row_ptr[r0];
        const int32_t E1 = row_ptr[r1];
        const int32_t Ew = E1 - E0;
        const int32_t rs = active ? row_ptr[i] : 0;
        const int32_t re = active ? row_ptr[i + 1] : 0;
        const int32_t len = re - rs;

        if (Ew <= eb) {
            // ---- stage the tile: columns, gathered coordinates, zeroed accumulators
            for (int e = lane; e < Ew; e += WAVE) {
                const int32_t cidx = col_idx[E0 + e];
                s_col[e] = cidx;
                const double2 qc = reinterpret_cast<const double2 *>(q)[cidx];
                s_qx[e] = qc.x;
                s_qy[e] = qc.y;
                if constexpr (I::W) s_w[e] = w[cidx];
            }
            if constexpr (OP == OP_ELAS) {
                for (int e = lane; e < 4 * Ew; e += WAVE) s_acc[e] = 0.0;
            } else {
#pragma unroll
                for (int m = 0; m < NACC; ++m)
                    for (int e = lane; e < Ew; e += WAVE) s_acc[m * eb + e] = 0.0;
            }
            __syncthreads();
            // ---- each lane: the triangles around its vertex, ascending id
            if (active && len > 0) {
                const int32_t off = rs - E0;
                int32_t pd = 0;
                while (pd < len - 1 && s_col[off + pd] != (int32_t)i) ++pd;
                const double x0 = s_qx[off + pd], y0 = s_qy[off + pd];
                const double w0 = I::W ? s_w[off + pd] : 0.0;
                double dg[NACC];
#pragma unroll
                for (int m = 0; m < NACC; ++m) dg[m] = 0.0;
                const int32_t t1 = inc_ptr[i + 1];
                for (int32_t t = inc_ptr[i]; t < t1; ++t) {
                    const uint32_t pp = inc_pos[t];
                    const int32_t p1 = off + (int32_t)(pp & 0xffffu);
                    const int32_t p2 = off + (int32_t)(pp >> 16);
                    double c[NACC][3];
                    double ce[3][4];
                    elem_row<OP>(x0, y0, s_qx[p1], s_qy[p1], s_qx[p2], s_qy[p2], w0,
                                 I::W ? s_w[p1] : 0.0, I::W ? s_w[p2] : 0.0, L, c, ce);
                    if constexpr (OP == OP_ELAS) {
                        // row 2i: [off*4 + 2p + beta], row 2i+1: [+ 2 len]
                        const int32_t b0 = 4 * off;
                        const int32_t q1 = p1 - off, q2 = p2 - off;
                        dg[0] += ce[0][0];
                        dg[1] += ce[0][1];
                        dg[2] += ce[0][2];
                        dg[3] += ce[0][3];
                        s_acc[b0 + 2 * q1] += ce[1][0];
                        s_acc[b0 + 2 * q1 + 1] += ce[1][1];
                        s_acc[b0 + 2 * len + 2 * q1] += ce[1][2];
                        s_acc[b0 + 2 * len + 2 * q1 + 1] += ce[1][3];
                        s_acc[b0 + 2 * q2] += ce[2][0];
                        s_acc[b0 + 2 * q2 + 1] += ce[2][1];
                        s_acc[b0 + 2 * len + 2 * q2] += ce[2][2];
                        s_acc[b0 + 2 * len + 2 * q2 + 1] += ce[2][3];
                    } else {
#pragma unroll
                        for (int m = 0; m < NACC; ++m) {
                            dg[m] += c[m][0];
                            s_acc[m * eb + p1] += c[m][1];
                            s_acc[m * eb + p2] += c[m][2];
                        }
                    }
                }
                if constexpr (OP == OP_ELAS) {
                    const int32_t b0 = 4 * off;
                    s_acc[b0 + 2 * pd] += dg[0];
                    s_acc[b0 + 2 * pd + 1] += dg[1];
                    s_acc[b0 + 2 * len + 2 * pd] += dg[2];
                    s_acc[b0 + 2 * len + 2 * pd + 1] += dg[3];
                } else {
#pragma unroll
                    for (int m = 0; m < NACC; ++m) s_acc[m * eb + off + pd] += dg[m];
                }
            }
            __syncthreads();
            // ---- write the tile back, coalesced
            if constexpr (OP == OP_ELAS) {
                for (int e = lane; e < 4 * Ew; e += WAVE) {
                    const int64_t g = 4 * (int64_t)E0 + e;
                    out0[g] = accumulate ? out0[g] + s_acc[e] : s_acc[e];
                }
            } else {
                for (int e = lane; e < Ew; e += WAVE) {
                    out0[E0 + e] = accumulate ? out0[E0 + e] + s_acc[e] : s_acc[e];
                    if constexpr (I::NOUT == 2)
                        out1[E0 + e] = accumulate ? out1[E0 + e] + s_acc[eb + e] : s_acc[eb + e];
                }
            }
            __syncthreads();
        } else if (active && len > 0) {
            // ---- tile too large for LDS: the lane works on its own row in
            // global memory (same order of additions, so same results)
            const int32_t nrow = (OP == OP_ELAS) ? 4 * len : len;
            double *o0 = out0 + ((OP == OP_ELAS) ? 4 * (int64_t)rs : (int64_t)rs);
            double *o1 = (I::NOUT == 2) ? out1 + rs : nullptr;
            if (!accumulate) {
                for (int e = 0; e < nrow; ++e) o0[e] = 0.0;
                if constexpr (I::NOUT == 2)
                    for (int e = 0; e < len; ++e) o1[e] = 0.0;
            }
            const int32_t *cr = col_idx + rs;
            int32_t pd = 0;
            while (pd < len - 1 && cr[pd] != (int32_t)i) ++pd;
            const double x0 = q[2 * i], y0 = q[2 * i + 1];
            const double w0 = I::W ? w[i] : 0.0;
            double dg[NACC];
#pragma unroll
            for (int m = 0; m < NACC; ++m) dg[m] = 0.0;
            const int32_t t1 = inc_ptr[i + 1];
            for (int32_t t = inc_ptr[i]; t < t1; ++t) {
                const uint32_t pp = inc_pos[t];
                const int32_t p1 = (int32_t)(pp & 0xffffu), p2 = (int32_t)(pp >> 16);
                const int32_t j1 = cr[p1], j2 = cr[p2];
                double c[NACC][3];
                double ce[3][4];
                elem_row<OP>(x0, y0, q[2 * (int64_t)j1], q[2 * (int64_t)j1 + 1], q[2 * (int64_t)j2],
                             q[2 * (int64_t)j2 + 1], w0, I::W ? w[j1] : 0.0, I::W ? w[j2] : 0.0, L,
                             c, ce);
                if constexpr (OP == OP_ELAS) {
                    dg[0] += ce[0][0];
                    dg[1] += ce[0][1];
                    dg[2] += ce[0][2];
                    dg[3] += ce[0][3];
                    o0[2 * p1] += ce[1][0];
                    o0[2 * p1 + 1] += ce[1][1];
                    o0[2 * len + 2 * p1] += ce[1][2];
                    o0[2 * len + 2 * p1 + 1] += ce[1][3];
                    o0[2 * p2] += ce[2][0];
                    o0[2 * p2 + 1] += ce[2][1];
                    o0[2 * len + 2 * p2] += ce[2][2];
                    o0[2 * len + 2 * p2 + 1] += ce[2][3];
                } else {
                    o0[p1] += c[0][1];
                    o0[p2] += c[0][2];
                    dg[0] += c[0][0];
                    if constexpr (I::NOUT == 2) {
                        o1[p1] += c[1][1];
                        o1[p2] += c[1][2];
                        dg[1] += c[1][0];
                    }
                }
            }
            if constexpr (OP == OP_ELAS) {
                o0[2 * pd] += dg[0];
                o0[2 * pd + 1] += dg[1];
                o0[2 * len + 2 * pd] += dg[2];
                o0[2 * len + 2 * pd + 1] += dg[3];
            } else {
                o0[pd] += dg[0];
                if constexpr (I::NOUT == 2) o1[pd] += dg[1];
            }
        }
    }
}

// ------------------------------------------------------------------ triangle + atomics

template <int OP>
__global__ __launch_bounds__(256) void k_elem_atomic(int32_t nme, const double *__restrict__ q,
                                                     const double *__restrict__ w,
                                                     const int32_t *__restrict__ me,
                                                     const int32_t *__restrict__ slot,
                                                     const int32_t *__restrict__ row_ptr,
                                                     double *__restrict__ out0,
                                                     double *__restrict__ out1, Lame L) {
    using I = OpInfo<OP>;
    const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (k >= nme) return;
    const int32_t v[3] = {me[3 * k], me[3 * k + 1], me[3 * k + 2]};
    double x[3], y[3], wl[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const double2 qc = reinterpret_cast<const double2 *>(q)[v[a]];
        x[a] = qc.x;
        y[a] = qc.y;
        wl[a] = I::W ? w[v[a]] : 0.0;
    }
    int32_t sl[9];
#pragma unroll
    for (int r = 0; r < 9; ++r) sl[r] = slot[(int64_t)r * nme + k];
    // rows a = 0, 1, 2 of the element matrices via the cyclic rotations
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const int a1 = (a + 1) % 3, a2 = (a + 2) % 3;
        double c[I::NACC][3];
        double ce[3][4];
        elem_row<OP>(x[a], y[a], x[a1], y[a1], x[a2], y[a2], wl[a], wl[a1], wl[a2], L, c, ce);
        const int bcol[3] = {a, a1, a2};
        if constexpr (OP == OP_ELAS) {
            const int32_t rs = row_ptr[v[a]];
            const int32_t len = row_ptr[v[a] + 1] - rs;
#pragma unroll
            for (int bb = 0; bb < 3; ++bb) {
                const int32_t p = sl[3 * bcol[bb] + a] - rs;
                const int64_t base = 4 * (int64_t)rs + 2 * p;
                unsafeAtomicAdd(out0 + base, ce[bb][0]);
                unsafeAtomicAdd(out0 + base + 1, ce[bb][1]);
                unsafeAtomicAdd(out0 + base + 2 * len, ce[bb][2]);
                unsafeAtomicAdd(out0 + base + 2 * len + 1, ce[bb][3]);
            }
        } else {
#pragma unroll
            for (int bb = 0; bb < 3; ++bb) {
                const int32_t p = sl[3 * bcol[bb] + a];
                unsafeAtomicAdd(out0 + p, c[0][bb]);
                if constexpr (I::NOUT == 2) unsafeAtomicAdd(out1 + p, c[1][bb]);
            }
        }
    }
}

// ------------------------------------------------------------------ host side

namespace {

constexpr int DEFAULT_EB = 512;

template <int OP> size_t lds_bytes(int eb) {
    using I = OpInfo<OP>;
    return (size_t)eb * (8 * I::NACC + 16 + (I::W ? 8 : 0) + 4);
}

struct Args {
    int32_t nq, nme;
    int64_t nnz;
    const double *q, *w;
    const int32_t *me, *row_ptr, *col_idx, *inc_ptr, *slot;
    const uint32_t *inc_pos;
    double *out0, *out1;
    Lame L;
    int flags;
    hipStream_t s;
};

int check_common(const char *fn, const Args &a, bool need_w, int nout) {
    FEM_REQUIRE(a.nq >= 1 && a.nme >= 0 && a.nnz >= 0, FEM_EINVAL, "%s: bad sizes nq=%d nme=%d nnz=%lld",
                fn, a.nq, a.nme, (long long)a.nnz);
    FEM_REQUIRE(a.nnz <= INT32_MAX, FEM_EOVERFLOW, "%s: nnz exceeds int32", fn);
    FEM_REQUIRE((a.flags & ~(FEM_ATOMIC | FEM_ACCUMULATE)) == 0, FEM_EINVAL, "%s: unknown flags 0x%x", fn,
                a.flags);
    FEM_REQUIRE(a.q && a.row_ptr, FEM_EINVAL, "%s: NULL q or row_ptr", fn);
    FEM_REQUIRE(a.nnz == 0 || (a.out0 && (nout < 2 || a.out1)), FEM_EINVAL, "%s: NULL output", fn);
    FEM_REQUIRE(!need_w || a.w, FEM_EINVAL, "%s: NULL w", fn);
    if (a.flags & FEM_ATOMIC) {
        FEM_REQUIRE(a.nme == 0 || (a.me && a.slot), FEM_EINVAL, "%s: FEM_ATOMIC needs me and slot", fn);
    } else {
        FEM_REQUIRE(a.nnz == 0 || (a.col_idx && a.inc_ptr && a.inc_pos), FEM_EINVAL,
                    "%s: NULL col_idx, inc_ptr or inc_pos", fn);
    }
    return FEM_OK;
}

template <int OP>
int launch_rows(const Args &a, int eb, int grid_blocks) {
    using I = OpInfo<OP>;
    if (a.nq == 0) return FEM_OK;
    if (eb <= 0) eb = DEFAULT_EB;
    eb = (eb + WAVE - 1) / WAVE * WAVE;
    const int64_t ntiles = (a.nq + WAVE - 1) / WAVE;
    const int64_t grid = grid_blocks > 0 ? (grid_blocks < ntiles ? grid_blocks : ntiles) : ntiles;
    FEM_REQUIRE(grid <= INT32_MAX, FEM_EOVERFLOW, "too many tiles");
    const size_t lds = lds_bytes<OP>(eb);
    FEM_REQUIRE(lds <= 64 * 1024, FEM_EINVAL, "lds_entries %d needs %zu bytes of LDS (limit 65536)", eb, lds);
    hipLaunchKernelGGL(k_rows_numeric<OP>, dim3((unsigned)grid), dim3(WAVE), lds, a.s, a.nq, a.q, a.w,
                       a.row_ptr, a.col_idx, a.inc_ptr, a.inc_pos, a.out0, a.out1, a.L, eb,
                       (a.flags & FEM_ACCUMULATE) ? 1 : 0, ntiles);
    FEM_LAUNCH_CHECK();
    (void)I::NOUT;
    return FEM_OK;
}

template <int OP>
int launch_atomic(const Args &a) {
    using I = OpInfo<OP>;
    const int64_t nvals = (OP == OP_ELAS) ? 4 * a.nnz : a.nnz;
    if (!(a.flags & FEM_ACCUMULATE)) {
        int st = fill_f64(a.out0, nvals, 0.0, a.s);
        if (st) return st;
        if (I::NOUT == 2 && (st = fill_f64(a.out1, a.nnz, 0.0, a.s))) return st;
    }
    if (a.nme == 0) return FEM_OK;
    hipLaunchKernelGGL(k_elem_atomic<OP>, dim3(grid_for(a.nme, 256)), dim3(256), 0, a.s, a.nme, a.q,
                       a.w, a.me, a.slot, a.row_ptr, a.out0, a.out1, a.L);
    FEM_LAUNCH_CHECK();
    return FEM_OK;
}

template <int OP>
int run(const char *fn, const Args &a, const fem_tune *tune = nullptr) {
    using I = OpInfo<OP>;
    int st = check_common(fn, a, I::W, I::NOUT);
    if (st) return st;
    if (a.flags & FEM_ATOMIC) return launch_atomic<OP>(a);
    return launch_rows<OP>(a, tune ? tune->lds_entries : 0, tune ? tune->grid_blocks : 0);
}

}  // namespace
}  // namespace fem

using namespace fem;

extern "C" int fem_assemble_mass(int32_t nq, int32_t nme, int64_t nnz, const double *q,
                                 const int32_t *me, const int32_t *row_ptr, const int32_t *col_idx,
                                 const int32_t *inc_ptr, const uint32_t *inc_pos,
                                 const int32_t *slot, double *values, int flags, void *stream) {
    clear_error();
    Args a{nq, nme, nnz, q, nullptr, me, row_ptr, col_idx, inc_ptr, slot, inc_pos, values, nullptr,
           {0, 0}, flags, as_stream(stream)};
    return run<OP_MASS>("fem_assemble_mass", a);
}

extern "C" int fem_assemble_wmass(int32_t nq, int32_t nme, int64_t nnz, const double *q,
                                  const int32_t *me, const int32_t *row_ptr, const int32_t *col_idx,
                                  const int32_t *inc_ptr, const uint32_t *inc_pos,
                                  const int32_t *slot, const double *w, double *values, int flags,
                                  void *stream) {
    clear_error();
    Args a{nq, nme, nnz, q, w, me, row_ptr, col_idx, inc_ptr, slot, inc_pos, values, nullptr,
           {0, 0}, flags, as_stream(stream)};
    return run<OP_WMASS>("fem_assemble_wmass", a);
}

extern "C" int fem_assemble_stiff(int32_t nq, int32_t nme, int64_t nnz, const double *q,
                                  const int32_t *me, const int32_t *row_ptr, const int32_t *col_idx,
                                  const int32_t *inc_ptr, const uint32_t *inc_pos,
                                  const int32_t *slot, double *values, int flags, void *stream) {
    clear_error();
    Args a{nq, nme, nnz, q, nullptr, me, row_ptr, col_idx, inc_ptr, slot, inc_pos, values, nullptr,
           {0, 0}, flags, as_stream(stream)};
    return run<OP_STIFF>("fem_assemble_stiff", a);
}

extern "C" int fem_assemble_stiff_mass(int32_t nq, int32_t nme, int64_t nnz, const double *q,
                                       const int32_t *me, const int32_t *row_ptr,
                                       const int32_t *col_idx, const int32_t *inc_ptr,
                                       const uint32_t *inc_pos, const int32_t *slot,
                                       double *vals_S, double *vals_M, int flags, void *stream) {
    clear_error();
    Args a{nq, nme, nnz, q, nullptr, me, row_ptr, col_idx, inc_ptr, slot, inc_pos, vals_S, vals_M,
           {0, 0}, flags, as_stream(stream)};
    return run<OP_STIFF_MASS>("fem_assemble_stiff_mass", a);
}

extern "C" int fem_assemble_stiff_wmass(int32_t nq, int32_t nme, int64_t nnz, const double *q,
                                        const int32_t *me, const int32_t *row_ptr,
                                        const int32_t *col_idx, const int32_t *inc_ptr,
                                        const uint32_t *inc_pos, const int32_t *slot,
                                        const double *w, double *vals_S, double *vals_Mw, int flags,
                                        void *stream) {
    clear_error();
    Args a{nq, nme, nnz, q, w, me, row_ptr, col_idx, inc_ptr, slot, inc_pos, vals_S, vals_Mw,
           {0, 0}, flags, as_stream(stream)};
    return run<OP_STIFF_WMASS>("fem_assemble_stiff_wmass", a);
}

extern "C" int fem_assemble_elas(int32_t nq, int32_t nme, int64_t nnz, const double *q,
                                 const int32_t *me, const int32_t *row_ptr, const int32_t *col_idx,
                                 const int32_t *inc_ptr, const uint32_t *inc_pos,
                                 const int32_t *slot, double lambda, double mu, double *values_e,
                                 int flags, void *stream) {
    clear_error();
    FEM_REQUIRE(lambda + mu > 0.0, FEM_EINVAL, "fem_assemble_elas: need lambda + mu > 0 (got %g)",
                lambda + mu);
    FEM_REQUIRE(4 * nnz <= INT32_MAX, FEM_EOVERFLOW, "fem_assemble_elas: 4 nnz exceeds int32");
    Args a{nq, nme, nnz, q, nullptr, me, row_ptr, col_idx, inc_ptr, slot, inc_pos, values_e, nullptr,
           {lambda, mu}, flags, as_stream(stream)};
    return run<OP_ELAS>("fem_assemble_elas", a);
}

extern "C" int fem_assemble_stiff_mass_batched(int32_t nb, int32_t nq, int64_t nnz, const double *q,
                                               const int32_t *row_ptr, const int32_t *col_idx,
                                               const int32_t *inc_ptr, const uint32_t *inc_pos,
                                               double *vals_S, double *vals_M,
                                               const fem_tune *tune, int flags, void *stream) {
    clear_error();
    FEM_REQUIRE(nb >= 1, FEM_EINVAL, "fem_assemble_stiff_mass_batched: nb must be >= 1");
    FEM_REQUIRE((flags & FEM_ATOMIC) == 0, FEM_EINVAL,
                "fem_assemble_stiff_mass_batched: only the row-owner scheme is batched");
    Args a{nq, 0, nnz, q, nullptr, nullptr, row_ptr, col_idx, inc_ptr, nullptr, inc_pos, vals_S,
           vals_M, {0, 0}, flags, as_stream(stream)};
    return run<OP_STIFF_MASS>("fem_assemble_stiff_mass_batched", a, tune);
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
