// fem_adjoint.hip -- hand-written adjoint of the stiffness + weighted mass
// assembly: gradient of L = <GS, S(q)> + <GM, Mw(q, w)> with respect to the
// vertex coordinates q and the vertex weights w.
//
// Row-owner decomposition.  L = sum_i sum_{T around i} tau(i, T) where
// tau(i, T) = sum_b GS[i, b] S^T_{ib} + GM[i, b] Mw^T_{ib} uses only row i of
// GS and GM.  Pass 1 (one lane per row, the same tiling as the forward) walks
// the triangles around i, differentiates tau(i, T) with respect to the three
// vertices of T and the three weights, keeps the part for i in registers and
// adds the parts for the two neighbours j into H[i, j] (LDS), then writes H:
// H[i, j] = d(sum_T tau(i, T)) / d(q_j, w_j).  Pass 2 (one lane per vertex u)
// sums column u of H: dL/d(q_u, w_u) = sum_v H[v, u].  With the transpose map
// tpos, pass 1 stores H[i, j] at the place of entry (j, i), so pass 2 reads
// row u in place; without it, pass 1 stores H in row order and pass 2 finds
// each transposed entry by search.  Either way the same values are added in
// the same order.  With the fan codes of fem_fan_plan, pass 1 walks a row's
// triangles in the order met around i, as the forward kernels do: each
// H[i, j] is then the sum of the two steps that share the edge (i, j), the
// diagonal part sums in walk order, and no slot of the row is searched per
// triangle.  No atomics; every sum has a fixed order, so the result is
// bitwise reproducible.
//
// Derivatives for the triangle (x0, x1, x2) (cyclic rotation starting at i),
// r0 = x1 - x2, r1 = x2 - x0, r2 = x0 - x1, D = (x1 - x0) x (x2 - x0),
// d|D|/dx_c = sign(D) perp(r_c), perp(r) = (r_y, -r_x):
//   stiffness  tau_S = N / (2|D|), N = <r0, R>, R = g0 r0 + g1 r1 + g2 r2
//              dN/dx0 = (g2 - g1) r0, dN/dx1 = R + (g0 - g2) r0,
//              dN/dx2 = -R + (g1 - g0) r0,
//              dtau_S/dx_c = dN/dx_c / (2|D|) - N / (2|D|^2) d|D|/dx_c
//   w-mass     tau_M = |D| P / 60, P = h0 (3w0+w1+w2) + h1 (w0+w1+w2/2)
//                                      + h2 (w0+w1/2+w2)          (eq. MassWElem)
//              dtau_M/dx_c = P / 60 d|D|/dx_c,
//              dtau_M/dw = |D|/60 (3h0+h1+h2, h0+h1+h2/2, h0+h1/2+h2)
// with g_b = GS[i, b], h_b = GM[i, b] for the columns b = (x0, x1, x2).
#include "fem_internal.h"

namespace fem {

struct AdjGrad {
    double gx[3], gy[3], gw[3];
};

template <bool HS, bool HM>
__device__ __forceinline__ void adj_tau(double x0, double y0, double x1, double y1, double x2,
                                        double y2, double w0, double w1, double w2, double g0,
                                        double g1, double g2, double h0, double h1, double h2,
                                        AdjGrad &o) {
    const double r0x = x1 - x2, r0y = y1 - y2;
    const double r1x = x2 - x0, r1y = y2 - y0;
    const double r2x = x0 - x1, r2y = y0 - y1;
    const double D = (x1 - x0) * (y2 - y0) - (x2 - x0) * (y1 - y0);
    const double ad = fabs(D);
    const double sg = D > 0.0 ? 1.0 : (D < 0.0 ? -1.0 : 0.0);
    // d|D|/dx_c
    const double dDx[3] = {sg * r0y, sg * r1y, sg * r2y};
    const double dDy[3] = {-sg * r0x, -sg * r1x, -sg * r2x};
#pragma unroll
    for (int c = 0; c < 3; ++c) o.gx[c] = o.gy[c] = o.gw[c] = 0.0;
    if constexpr (HS) {
        const double Rx = g0 * r0x + g1 * r1x + g2 * r2x;
        const double Ry = g0 * r0y + g1 * r1y + g2 * r2y;
        const double N = r0x * Rx + r0y * Ry;
        const double inv = 1.0 / (2.0 * ad);
        const double k = N * inv / ad;
        const double dNx[3] = {(g2 - g1) * r0x, Rx + (g0 - g2) * r0x, -Rx + (g1 - g0) * r0x};
        const double dNy[3] = {(g2 - g1) * r0y, Ry + (g0 - g2) * r0y, -Ry + (g1 - g0) * r0y};
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            o.gx[c] += dNx[c] * inv - k * dDx[c];
            o.gy[c] += dNy[c] * inv - k * dDy[c];
        }
    }
    if constexpr (HM) {
        const double P = h0 * (3.0 * w0 + w1 + w2) + h1 * (w0 + w1 + 0.5 * w2) +
                         h2 * (w0 + 0.5 * w1 + w2);
        const double p60 = P / 60.0;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            o.gx[c] += p60 * dDx[c];
            o.gy[c] += p60 * dDy[c];
        }
        const double a60 = ad / 60.0;
        o.gw[0] = a60 * (3.0 * h0 + h1 + h2);
        o.gw[1] = a60 * (h0 + h1 + 0.5 * h2);
        o.gw[2] = a60 * (h0 + 0.5 * h1 + h2);
    }
}

// (x, y, w, 0) records: one random access per column in pass 1.
__global__ __launch_bounds__(256) void k_adj_pack(int32_t nq, const double2 *__restrict__ q,
                                                  const double *__restrict__ w,
                                                  double4 *__restrict__ qw) {
    const int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (v >= nq) return;
    const double2 a = q[v];
    qw[v] = make_double4(a.x, a.y, w ? w[v] : 0.0, 0.0);
}

// Pass 1: tile of 64 rows (one per lane), staged like the forward kernel.
// LDS: q (x, y) | w | GS | GM | ipos per entry; each lane keeps the H
// accumulators (x, y, w) of its row in registers (rows of at most LMAX
// entries), then LDS is reused to transpose them, and H is written coalesced
// as (hx, hy, hw, 0) records so that pass 2 reads one record per entry.  Rows
// longer than LMAX (or tiles too large for LDS) take the per-lane
// global-memory path; the order of additions is the same everywhere.
template <bool HS, bool HM, int U, int LMAX>
__global__ __launch_bounds__(WAVE) void k_adj_rows(int32_t nq, const double4 *__restrict__ qw,
                                                   const int32_t *__restrict__ row_ptr,
                                                   const int32_t *__restrict__ col_idx,
                                                   const int32_t *__restrict__ inc_ptr,
                                                   const uint32_t *__restrict__ inc_pos,
                                                   const int32_t *__restrict__ tpos,
                                                   const double *__restrict__ GS,
                                                   const double *__restrict__ GM,
                                                   double4 *__restrict__ H, int64_t ntiles) {
    constexpr int EB = U * WAVE;
    extern __shared__ double smem[];
    double2 *s_q = reinterpret_cast<double2 *>(smem);
    double *s_w = smem + 2 * EB;
    double *s_gs = smem + 3 * EB;
    double *s_gm = smem + 4 * EB;
    uint32_t *s_ip = reinterpret_cast<uint32_t *>(smem + 5 * EB);
    double *s_stage = smem;   // 3 doubles per entry, after the sums
    const int lane = threadIdx.x;
    for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const int64_t r0 = tile * WAVE;
        const int64_t r1 = (r0 + WAVE < nq) ? r0 + WAVE : nq;
        const int64_t i = r0 + lane;
        const bool active = i < nq;
        const int32_t E0 = row_ptr[r0], E1 = row_ptr[r1], Ew = E1 - E0;
        const int32_t I0 = inc_ptr[r0], I1 = inc_ptr[r1], Iw = I1 - I0;
        const int32_t rs = active ? row_ptr[i] : 0;
        const int32_t len = active ? row_ptr[i + 1] - rs : 0;
        const int32_t is = active ? inc_ptr[i] : 0;
        const int32_t ie = active ? inc_ptr[i + 1] : 0;
        const bool tile_fits = Ew <= EB && Iw <= EB;
        if (tile_fits) {
            int32_t cidx[U];
            double gsv[U], gmv[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int e = lane + u * WAVE;
                cidx[u] = e < Ew ? __builtin_nontemporal_load(col_idx + E0 + e) : 0;
                gsv[u] = (HS && e < Ew) ? __builtin_nontemporal_load(GS + E0 + e) : 0.0;
                gmv[u] = (HM && e < Ew) ? __builtin_nontemporal_load(GM + E0 + e) : 0.0;
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int t = lane + u * WAVE;
                if (t < Iw) s_ip[t] = __builtin_nontemporal_load(inc_pos + I0 + t);
            }
            double4 qv[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int e = lane + u * WAVE;
                qv[u] = e < Ew ? qw[cidx[u]] : make_double4(0.0, 0.0, 0.0, 0.0);
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int e = lane + u * WAVE;
                if (e < Ew) {
                    s_q[e] = make_double2(qv[u].x, qv[u].y);
                    s_w[e] = qv[u].z;
                    if constexpr (HS) s_gs[e] = gsv[u];
                    if constexpr (HM) s_gm[e] = gmv[u];
                }
            }
            __syncthreads();
        }
        const bool in_regs = tile_fits && active && len > 0 && len <= LMAX;
        double hx[LMAX], hy[LMAX], hw[LMAX];
#pragma unroll
        for (int k = 0; k < LMAX; ++k) hx[k] = hy[k] = hw[k] = 0.0;
        if (in_regs) {
            const int32_t off = rs - E0;
            uint64_t seen = 0;
            for (int32_t t = is - I0; t < ie - I0; ++t) {
                const uint32_t pp = s_ip[t];
                seen |= (1ull << (pp & 0xffffu)) | (1ull << (pp >> 16));
            }
            const int32_t pd = __builtin_ctzll(~seen);
            const double2 x0 = s_q[off + pd];
            const double w0 = s_w[off + pd];
            const double g0 = HS ? s_gs[off + pd] : 0.0, h0 = HM ? s_gm[off + pd] : 0.0;
            double ox = 0.0, oy = 0.0, ow = 0.0;
            for (int32_t t = is - I0; t < ie - I0; ++t) {
                const uint32_t pp = s_ip[t];
                const int32_t p1 = (int32_t)(pp & 0xffffu), p2 = (int32_t)(pp >> 16);
                const double2 x1 = s_q[off + p1], x2 = s_q[off + p2];
                AdjGrad o;
                adj_tau<HS, HM>(x0.x, x0.y, x1.x, x1.y, x2.x, x2.y, w0, s_w[off + p1],
                                s_w[off + p2], g0, HS ? s_gs[off + p1] : 0.0,
                                HS ? s_gs[off + p2] : 0.0, h0, HM ? s_gm[off + p1] : 0.0,
                                HM ? s_gm[off + p2] : 0.0, o);
                ox += o.gx[0];
                oy += o.gy[0];
                ow += o.gw[0];
#pragma unroll
                for (int k = 0; k < LMAX; ++k) {
                    const bool a1 = k == p1, a2 = k == p2;
                    hx[k] += a1 ? o.gx[1] : (a2 ? o.gx[2] : 0.0);
                    hy[k] += a1 ? o.gy[1] : (a2 ? o.gy[2] : 0.0);
                    if constexpr (HM) hw[k] += a1 ? o.gw[1] : (a2 ? o.gw[2] : 0.0);
                }
            }
#pragma unroll
            for (int k = 0; k < LMAX; ++k)
                if (k == pd) {
                    hx[k] += ox;
                    hy[k] += oy;
                    hw[k] += ow;
                }
        }
        if (tile_fits) {
            __syncthreads();   // everyone is done reading the staged inputs
            const int32_t off = rs - E0;
            if (in_regs) {
#pragma unroll
                for (int k = 0; k < LMAX; ++k)
                    if (k < len) {
                        s_stage[3 * (off + k)] = hx[k];
                        s_stage[3 * (off + k) + 1] = hy[k];
                        s_stage[3 * (off + k) + 2] = hw[k];
                    }
            } else if (active && len > 0) {
                for (int k = 0; k < 3 * len; ++k) s_stage[3 * off + k] = 0.0;
            }
            __syncthreads();
            // with tpos, each value goes to the place of its transposed entry
            int32_t dst[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int e = lane + u * WAVE;
                dst[u] = e < Ew ? (tpos ? tpos[E0 + e] : E0 + e) : 0;
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int e = lane + u * WAVE;
                if (e < Ew && dst[u] >= 0)   // tpos -1: no transposed entry, no place
                    H[dst[u]] = make_double4(s_stage[3 * e], s_stage[3 * e + 1], s_stage[3 * e + 2], 0.0);
            }
            __syncthreads();
        }
        if (!in_regs && active && len > 0) {
            // long row or tile too large: own row in global memory, same order
            // (each entry at its own place, transposed with tpos)
            // (an entry without a transposed partner, tpos -1, has no place:
            // nothing would read it, and it is skipped)
            auto hat = [&](int32_t e) -> int32_t { return tpos ? tpos[rs + e] : rs + e; };
            auto hadd = [&](int32_t e, double gx, double gy, double gw) {
                const int32_t d = hat(e);
                if (d < 0) return;
                double4 h = H[d];
                h.x += gx;
                h.y += gy;
                h.z += gw;
                H[d] = h;
            };
            for (int e = 0; e < len; ++e) {
                const int32_t d = hat(e);
                if (d >= 0) H[d] = make_double4(0.0, 0.0, 0.0, 0.0);
            }
            const int32_t *cr = col_idx + rs;
            int32_t pd = 0;
            while (pd < len - 1 && cr[pd] != (int32_t)i) ++pd;
            const double4 xi = qw[i];
            const double g0 = HS ? GS[rs + pd] : 0.0, h0 = HM ? GM[rs + pd] : 0.0;
            double ox = 0.0, oy = 0.0, ow = 0.0;
            for (int32_t t = is; t < ie; ++t) {
                const uint32_t pp = inc_pos[t];
                const int32_t p1 = (int32_t)(pp & 0xffffu), p2 = (int32_t)(pp >> 16);
                const double4 x1 = qw[cr[p1]], x2 = qw[cr[p2]];
                AdjGrad o;
                adj_tau<HS, HM>(xi.x, xi.y, x1.x, x1.y, x2.x, x2.y, xi.z, x1.z, x2.z, g0,
                                HS ? GS[rs + p1] : 0.0, HS ? GS[rs + p2] : 0.0, h0,
                                HM ? GM[rs + p1] : 0.0, HM ? GM[rs + p2] : 0.0, o);
                ox += o.gx[0];
                oy += o.gy[0];
                ow += o.gw[0];
                hadd(p1, o.gx[1], o.gy[1], o.gw[1]);
                hadd(p2, o.gx[2], o.gy[2], o.gw[2]);
            }
            hadd(pd, ox, oy, ow);
        }
    }
}

// Pass 1 over fan codes: tile of 64 rows, one per lane.  LDS: the tile's GS
// and GM values (read coalesced) and the H records (x, y, w) of the tile;
// each lane gathers its neighbours' (x, y, w) records in walk order into
// registers, walks the fan, and writes every H value into LDS as soon as it
// is complete (slot s_j after step j, s_0 and the last slot at the end);
// then H is stored as in k_adj_rows.  Rows without a fan code, with more
// than N neighbours or in a tile too large for LDS take the per-lane
// global-memory path of k_adj_rows (ascending triangles).
template <bool HS, bool HM, int U, int N>
__global__ __launch_bounds__(WAVE) void k_adj_rows_fan(int32_t nq, const double4 *__restrict__ qw,
                                                       const int32_t *__restrict__ row_ptr,
                                                       const int32_t *__restrict__ col_idx,
                                                       const int32_t *__restrict__ inc_ptr,
                                                       const uint32_t *__restrict__ inc_pos,
                                                       const uint64_t *__restrict__ fan,
                                                       const int32_t *__restrict__ tpos,
                                                       const double *__restrict__ GS,
                                                       const double *__restrict__ GM,
                                                       double4 *__restrict__ H, int64_t ntiles) {
    constexpr int EB = U * WAVE;
    extern __shared__ double smem[];
    double *s_gs = smem;            // [EB]
    double *s_gm = smem + EB;       // [EB]
    double *s_h = smem + 2 * EB;    // [3 EB]: (x, y, w) per entry
    const int lane = threadIdx.x;
    for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const int64_t r0 = tile * WAVE;
        const int64_t r1 = (r0 + WAVE < nq) ? r0 + WAVE : nq;
        const int64_t i = r0 + lane;
        const bool active = i < nq;
        const int32_t E0 = row_ptr[r0], E1 = row_ptr[r1], Ew = E1 - E0;
        const int32_t rs = active ? row_ptr[i] : 0;
        const int32_t len = active ? row_ptr[i + 1] - rs : 0;
        const uint64_t code = active ? fan[i] : 0;
        const int n = fan_n(code);
        const bool closed = fan_closed(code);
        const bool tile_fits = Ew <= EB;
        const bool in_regs = tile_fits && active && n >= 2 && n <= N && len == n + 1;
        const bool zero_row = !in_regs && active && len > 0;
        const int32_t off = rs - E0;
        if (tile_fits) {
            double gsv[U], gmv[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int e = lane + u * WAVE;
                gsv[u] = (HS && e < Ew) ? __builtin_nontemporal_load(GS + E0 + e) : 0.0;
                gmv[u] = (HM && e < Ew) ? __builtin_nontemporal_load(GM + E0 + e) : 0.0;
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int e = lane + u * WAVE;
                if (e < Ew) {
                    if constexpr (HS) s_gs[e] = gsv[u];
                    if constexpr (HM) s_gm[e] = gmv[u];
                }
            }
        }
        // the neighbours' records in walk order, the row's own one
        int32_t cj[N];
#pragma unroll
        for (int j = 0; j < N; ++j) cj[j] = (in_regs && j < n) ? col_idx[rs + fan_slot(code, j)] : -1;
        double4 x[N];
#pragma unroll
        for (int j = 0; j < N; ++j) x[j] = cj[j] >= 0 ? qw[cj[j]] : make_double4(0.0, 0.0, 0.0, 0.0);
        const double4 xi = in_regs ? qw[i] : make_double4(0.0, 0.0, 0.0, 0.0);
        if (tile_fits) __syncthreads();   // G staged
        if (in_regs) {
            const int32_t pd = fan_pd(code);
            const double g0 = HS ? s_gs[off + pd] : 0.0, h0 = HM ? s_gm[off + pd] : 0.0;
            auto put = [&](int sl, double hx, double hy, double hw) {
                double *p = s_h + 3 * (off + sl);
                p[0] = hx;
                p[1] = hy;
                p[2] = hw;
            };
            double ox = 0.0, oy = 0.0, ow = 0.0;
            double cx = 0.0, cy = 0.0, cw = 0.0, fx = 0.0, fy = 0.0, fw = 0.0;
            const int d = closed ? n : n - 1;
#pragma unroll
            for (int j = 0; j < N; ++j) {
                if (j < d) {
                    const bool wrap = j + 1 >= n;
                    const int jn = j + 1 < N ? j + 1 : 0;
                    const int32_t a = off + fan_slot(code, j);
                    const int32_t b = off + (wrap ? fan_slot(code, 0) : fan_slot(code, jn));
                    const double4 x2 = wrap ? x[0] : x[jn];
                    AdjGrad o;
                    adj_tau<HS, HM>(xi.x, xi.y, x[j].x, x[j].y, x2.x, x2.y, xi.z, x[j].z, x2.z, g0,
                                    HS ? s_gs[a] : 0.0, HS ? s_gs[b] : 0.0, h0,
                                    HM ? s_gm[a] : 0.0, HM ? s_gm[b] : 0.0, o);
                    ox += o.gx[0];
                    oy += o.gy[0];
                    ow += o.gw[0];
                    if (j == 0) {
                        fx = o.gx[1];
                        fy = o.gy[1];
                        fw = o.gw[1];
                        if (!closed) put(fan_slot(code, 0), fx, fy, fw);
                    } else {
                        put(fan_slot(code, j), cx + o.gx[1], cy + o.gy[1], cw + o.gw[1]);
                    }
                    cx = o.gx[2];
                    cy = o.gy[2];
                    cw = o.gw[2];
                }
            }
            if (closed) put(fan_slot(code, 0), fx + cx, fy + cy, fw + cw);
            else put(fan_slot(code, n - 1), cx, cy, cw);
            put(pd, ox, oy, ow);
        } else if (tile_fits && zero_row) {
            for (int k = 0; k < 3 * len; ++k) s_h[3 * off + k] = 0.0;
        }
        if (tile_fits) {
            __syncthreads();
            // with tpos, each value goes to the place of its transposed entry
            int32_t dst[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int e = lane + u * WAVE;
                dst[u] = e < Ew ? (tpos ? tpos[E0 + e] : E0 + e) : 0;
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int e = lane + u * WAVE;
                if (e < Ew && dst[u] >= 0)   // tpos -1: no transposed entry, no place
                    H[dst[u]] = make_double4(s_h[3 * e], s_h[3 * e + 1], s_h[3 * e + 2], 0.0);
            }
            __syncthreads();
        }
        if (zero_row) {
            // ascending triangles from global memory, as in k_adj_rows (each
            // entry at its own place, transposed with tpos; tpos -1 skipped)
            auto hat = [&](int32_t e) -> int32_t { return tpos ? tpos[rs + e] : rs + e; };
            auto hadd = [&](int32_t e, double gx, double gy, double gw) {
                const int32_t dd = hat(e);
                if (dd < 0) return;
                double4 h = H[dd];
                h.x += gx;
                h.y += gy;
                h.z += gw;
                H[dd] = h;
            };
            if (!tile_fits) {
                for (int e = 0; e < len; ++e) {
                    const int32_t dd = hat(e);
                    if (dd >= 0) H[dd] = make_double4(0.0, 0.0, 0.0, 0.0);
                }
            }
            const int32_t is = inc_ptr[i], ie = inc_ptr[i + 1];
            const int32_t *cr = col_idx + rs;
            int32_t pd = 0;
            while (pd < len - 1 && cr[pd] != (int32_t)i) ++pd;
            const double4 x0 = qw[i];
            const double g0 = HS ? GS[rs + pd] : 0.0, h0 = HM ? GM[rs + pd] : 0.0;
            double ox = 0.0, oy = 0.0, ow = 0.0;
            for (int32_t t = is; t < ie; ++t) {
                const uint32_t pp = inc_pos[t];
                const int32_t p1 = (int32_t)(pp & 0xffffu), p2 = (int32_t)(pp >> 16);
                const double4 x1 = qw[cr[p1]], x2 = qw[cr[p2]];
                AdjGrad o;
                adj_tau<HS, HM>(x0.x, x0.y, x1.x, x1.y, x2.x, x2.y, x0.z, x1.z, x2.z, g0,
                                HS ? GS[rs + p1] : 0.0, HS ? GS[rs + p2] : 0.0, h0,
                                HM ? GM[rs + p1] : 0.0, HM ? GM[rs + p2] : 0.0, o);
                ox += o.gx[0];
                oy += o.gy[0];
                ow += o.gw[0];
                hadd(p1, o.gx[1], o.gy[1], o.gw[1]);
                hadd(p2, o.gx[2], o.gy[2], o.gw[2]);
            }
            hadd(pd, ox, oy, ow);
        }
    }
}

__device__ inline int32_t find_in_row(const int32_t *__restrict__ col_idx, int32_t rs, int32_t re,
                                      int32_t x) {
    int32_t lo = rs, hi = re;
    while (lo < hi) {
        const int32_t mid = (lo + hi) >> 1;
        if (col_idx[mid] < x) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// Pass 2: column sums of H, one lane per vertex u, ascending position in row u.
__global__ __launch_bounds__(256) void k_adj_cols(int32_t nq, const int32_t *__restrict__ row_ptr,
                                                  const int32_t *__restrict__ col_idx,
                                                  const int32_t *__restrict__ tpos,
                                                  const double4 *__restrict__ H,
                                                  double *__restrict__ dq, double *__restrict__ dw,
                                                  int accumulate) {
    const int64_t u = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (u >= nq) return;
    double gx = 0.0, gy = 0.0, gw = 0.0;
    const int32_t rs = row_ptr[u], re = row_ptr[u + 1];
    for (int32_t p = rs; p < re; ++p) {
        int32_t t;
        if (tpos) {
            t = tpos[p];
        } else {
            const int32_t v = col_idx[p];
            const int32_t re_v = row_ptr[v + 1];
            t = find_in_row(col_idx, row_ptr[v], re_v, static_cast<int32_t>(u));
            if (t >= re_v || col_idx[t] != (int32_t)u) t = -1;
        }
        if (t < 0) continue;   // no transposed entry (never for a P1 pattern)
        const double4 h = H[t];
        gx += h.x;
        gy += h.y;
        gw += h.z;
    }
    if (accumulate) {
        dq[2 * u] += gx;
        dq[2 * u + 1] += gy;
        if (dw) dw[u] += gw;
    } else {
        dq[2 * u] = gx;
        dq[2 * u + 1] = gy;
        if (dw) dw[u] = gw;
    }
}

// Pass 2 with the transpose map: tile of 64 vertices u (one per lane).  Pass
// 1 has stored H transposed, so the tile's values are contiguous and read
// coalesced; each lane then sums its row from LDS in ascending position (the
// same order as k_adj_cols).
template <int U>
__global__ __launch_bounds__(WAVE) void k_adj_cols_tpos(int32_t nq, const int32_t *__restrict__ row_ptr,
                                                        const int32_t *__restrict__ tpos,
                                                        const double4 *__restrict__ H,
                                                        double *__restrict__ dq, double *__restrict__ dw,
                                                        int accumulate, int64_t ntiles) {
    constexpr int EB = U * WAVE;
    __shared__ double s_h[3 * EB];
    const int lane = threadIdx.x;
    for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const int64_t r0 = tile * WAVE;
        const int64_t r1 = (r0 + WAVE < nq) ? r0 + WAVE : nq;
        const int64_t u = r0 + lane;
        const bool active = u < nq;
        const int32_t E0 = row_ptr[r0], E1 = row_ptr[r1], Ew = E1 - E0;
        const int32_t rs = active ? row_ptr[u] : 0;
        const int32_t re = active ? row_ptr[u + 1] : 0;
        double gx = 0.0, gy = 0.0, gw = 0.0;
        if (Ew <= EB) {
            double4 h[U];
#pragma unroll
            for (int k = 0; k < U; ++k) {
                const int e = lane + k * WAVE;
                h[k] = e < Ew ? H[E0 + e] : make_double4(0.0, 0.0, 0.0, 0.0);
            }
#pragma unroll
            for (int k = 0; k < U; ++k) {
                const int e = lane + k * WAVE;
                if (e < Ew) {
                    s_h[3 * e] = h[k].x;
                    s_h[3 * e + 1] = h[k].y;
                    s_h[3 * e + 2] = h[k].z;
                }
            }
            __syncthreads();
            for (int32_t e = rs - E0; e < re - E0; ++e) {
                gx += s_h[3 * e];
                gy += s_h[3 * e + 1];
                gw += s_h[3 * e + 2];
            }
            __syncthreads();
        } else {
            for (int32_t p = rs; p < re; ++p) {
                const double4 hv = H[p];   // already transposed by pass 1
                gx += hv.x;
                gy += hv.y;
                gw += hv.z;
            }
        }
        if (!active) continue;
        if (accumulate) {
            dq[2 * u] += gx;
            dq[2 * u + 1] += gy;
            if (dw) dw[u] += gw;
        } else {
            dq[2 * u] = gx;
            dq[2 * u + 1] = gy;
            if (dw) dw[u] = gw;
        }
    }
}

// ------------------------------------------------------------------ elasticity
//
// L = <G, K(q; lambda, mu)> on the interleaved elasticity pattern (G[e] for
// the entry (2i + alpha, 2j + beta) of the scalar entry j = k-th column of
// row i at 4 row_ptr[i] + 2 alpha len_i + 2 k + beta).  Row-owner split as
// above: L = sum_i sum_{T around i} tau(i, T), with, for the triangle
// (x0, x1, x2) rotated to start at i, r0 = x1 - x2, r1 = x2 - x0,
// r2 = x0 - x1, rho_c = perp(r_c) = (r_c,y, -r_c,x), D = (x1-x0) x (x2-x0):
//   K^e block (0, b) = P(rho_0, rho_b) / (2|D|), P the bilinear form of
//   B^T C B, so tau = N / (2|D|) with N = rho_0 . R, R = sum_b W_b rho_b and
//     W_b = [[(l+2m) gxx + m gyy, l gxy + m gyx],
//            [m gxy + l gyx,      m gxx + (l+2m) gyy]]   (g = G block (i, b))
//   dN: gamma_0 = R + W_0^T rho_0, gamma_b = W_b^T rho_0 (b = 1, 2),
//       h_b = (-gamma_b,y, gamma_b,x) (d rho = perp d r),
//       dN/dx0 = h2 - h1, dN/dx1 = h0 - h2, dN/dx2 = h1 - h0
//   dtau/dx_c = dN/dx_c / (2|D|) - N / (2|D|^2) sign(D) rho_c
//   lambda, mu: W is linear in them, W = l W_l + m W_m, and
//     dtau/dl = rho_0 . sum_b W_l,b rho_b / (2|D|) (same for m).
struct ElasTau {
    double n, nl, nm;          // N, N_lambda, N_mu
    double d[3][2];            // dN / dx_c
};

__device__ __forceinline__ void elas_tau(const double (&x)[3][2], const double (&g)[3][4], double lam,
                                         double mu, ElasTau &o) {
    double rho[3][2];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const int c1 = (c + 1) % 3, c2 = (c + 2) % 3;
        const double rx = x[c1][0] - x[c2][0], ry = x[c1][1] - x[c2][1];
        rho[c][0] = ry;
        rho[c][1] = -rx;
    }
    const double l2m = lam + 2.0 * mu;
    double R[2] = {0.0, 0.0}, Rl[2] = {0.0, 0.0}, Rm[2] = {0.0, 0.0};
    double W[3][4];   // xx, xy, yx, yy
#pragma unroll
    for (int b = 0; b < 3; ++b) {
        const double gxx = g[b][0], gxy = g[b][1], gyx = g[b][2], gyy = g[b][3];
        W[b][0] = l2m * gxx + mu * gyy;
        W[b][1] = lam * gxy + mu * gyx;
        W[b][2] = mu * gxy + lam * gyx;
        W[b][3] = mu * gxx + l2m * gyy;
        R[0] += W[b][0] * rho[b][0] + W[b][1] * rho[b][1];
        R[1] += W[b][2] * rho[b][0] + W[b][3] * rho[b][1];
        Rl[0] += gxx * rho[b][0] + gxy * rho[b][1];
        Rl[1] += gyx * rho[b][0] + gyy * rho[b][1];
        Rm[0] += (2.0 * gxx + gyy) * rho[b][0] + gyx * rho[b][1];
        Rm[1] += gxy * rho[b][0] + (gxx + 2.0 * gyy) * rho[b][1];
    }
    o.n = rho[0][0] * R[0] + rho[0][1] * R[1];
    o.nl = rho[0][0] * Rl[0] + rho[0][1] * Rl[1];
    o.nm = rho[0][0] * Rm[0] + rho[0][1] * Rm[1];
    double h[3][2];
#pragma unroll
    for (int b = 0; b < 3; ++b) {
        double gx = W[b][0] * rho[0][0] + W[b][2] * rho[0][1];
        double gy = W[b][1] * rho[0][0] + W[b][3] * rho[0][1];
        if (b == 0) {
            gx += R[0];
            gy += R[1];
        }
        h[b][0] = -gy;
        h[b][1] = gx;
    }
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        o.d[0][c] = h[2][c] - h[1][c];
        o.d[1][c] = h[0][c] - h[2][c];
        o.d[2][c] = h[1][c] - h[0][c];
    }
    // finish: dtau/dx_c, with |D| and its derivative
    const double D = (x[1][0] - x[0][0]) * (x[2][1] - x[0][1]) - (x[2][0] - x[0][0]) * (x[1][1] - x[0][1]);
    const double aD = fabs(D);
    const double sg = D > 0.0 ? 1.0 : (D < 0.0 ? -1.0 : 0.0);
    const double inv = 1.0 / (2.0 * aD);
    const double k = o.n * inv / aD;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        o.d[c][0] = o.d[c][0] * inv - k * sg * rho[c][0];
        o.d[c][1] = o.d[c][1] * inv - k * sg * rho[c][1];
    }
    o.nl *= inv;
    o.nm *= inv;
}

// Pass 1 of the elasticity adjoint: tile of 64 rows (one per lane).  LDS:
// q (x, y) | the tile's 4 Ew values of G | ipos; H accumulators (x, y) of the
// lane's row in registers, then transposed through LDS and written as
// (hx, hy) records; the tile's dtau/dlambda, dtau/dmu sums go to lm[tile].
template <int U, int LMAX>
__global__ __launch_bounds__(WAVE) void k_adj_elas_rows(
    int32_t nq, const double *__restrict__ q, const int32_t *__restrict__ row_ptr,
    const int32_t *__restrict__ col_idx, const int32_t *__restrict__ inc_ptr,
    const uint32_t *__restrict__ inc_pos, const int32_t *__restrict__ tpos,
    const double *__restrict__ G, double lam, double mu, double2 *__restrict__ H,
    double2 *__restrict__ lm, int64_t ntiles) {
    constexpr int EB = U * WAVE;
    extern __shared__ double smem[];
    double2 *s_q = reinterpret_cast<double2 *>(smem);
    double *s_g = smem + 2 * EB;
    uint32_t *s_ip = reinterpret_cast<uint32_t *>(smem + 6 * EB);
    double *s_stage = smem;   // 2 doubles per entry, after the sums
    const int lane = threadIdx.x;
    const double2 *q2 = reinterpret_cast<const double2 *>(q);
    for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const int64_t r0 = tile * WAVE;
        const int64_t r1 = (r0 + WAVE < nq) ? r0 + WAVE : nq;
        const int64_t i = r0 + lane;
        const bool active = i < nq;
        const int32_t E0 = row_ptr[r0], E1 = row_ptr[r1], Ew = E1 - E0;
        const int32_t I0 = inc_ptr[r0], I1 = inc_ptr[r1], Iw = I1 - I0;
        const int32_t rs = active ? row_ptr[i] : 0;
        const int32_t len = active ? row_ptr[i + 1] - rs : 0;
        const int32_t is = active ? inc_ptr[i] : 0;
        const int32_t ie = active ? inc_ptr[i + 1] : 0;
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
            // the tile's 4 Ew values of G, eight loads in flight per lane
            const double *gt = G + 4 * (int64_t)E0;
            for (int e0 = 0; e0 < 4 * Ew; e0 += 8 * WAVE) {
                double gv[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const int e = e0 + lane + u * WAVE;
                    gv[u] = e < 4 * Ew ? __builtin_nontemporal_load(gt + e) : 0.0;
                }
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const int e = e0 + lane + u * WAVE;
                    if (e < 4 * Ew) s_g[e] = gv[u];
                }
            }
            double2 qv[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int e = lane + u * WAVE;
                qv[u] = e < Ew ? q2[cidx[u]] : make_double2(0.0, 0.0);
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int e = lane + u * WAVE;
                if (e < Ew) s_q[e] = qv[u];
            }
            __syncthreads();
        }
        const bool in_regs = tile_fits && active && len > 0 && len <= LMAX;
        double hx[LMAX], hy[LMAX];
#pragma unroll
        for (int k = 0; k < LMAX; ++k) hx[k] = hy[k] = 0.0;
        double sl = 0.0, sm = 0.0;
        if (in_regs) {
            const int32_t off = rs - E0;
            uint64_t seen = 0;
            for (int32_t t = is - I0; t < ie - I0; ++t) {
                const uint32_t pp = s_ip[t];
                seen |= (1ull << (pp & 0xffffu)) | (1ull << (pp >> 16));
            }
            const int32_t pd = __builtin_ctzll(~seen);
            const double *gr = s_g + 4 * off;   // row 2i at gr[2k + beta], row 2i+1 at gr[2len + 2k + beta]
            double x[3][2], g[3][4];
            x[0][0] = s_q[off + pd].x;
            x[0][1] = s_q[off + pd].y;
            g[0][0] = gr[2 * pd];
            g[0][1] = gr[2 * pd + 1];
            g[0][2] = gr[2 * len + 2 * pd];
            g[0][3] = gr[2 * len + 2 * pd + 1];
            double ox = 0.0, oy = 0.0;
            for (int32_t t = is - I0; t < ie - I0; ++t) {
                const uint32_t pp = s_ip[t];
                const int32_t p1 = (int32_t)(pp & 0xffffu), p2 = (int32_t)(pp >> 16);
                x[1][0] = s_q[off + p1].x;
                x[1][1] = s_q[off + p1].y;
                x[2][0] = s_q[off + p2].x;
                x[2][1] = s_q[off + p2].y;
                g[1][0] = gr[2 * p1];
                g[1][1] = gr[2 * p1 + 1];
                g[1][2] = gr[2 * len + 2 * p1];
                g[1][3] = gr[2 * len + 2 * p1 + 1];
                g[2][0] = gr[2 * p2];
                g[2][1] = gr[2 * p2 + 1];
                g[2][2] = gr[2 * len + 2 * p2];
                g[2][3] = gr[2 * len + 2 * p2 + 1];
                ElasTau o;
                elas_tau(x, g, lam, mu, o);
                ox += o.d[0][0];
                oy += o.d[0][1];
                sl += o.nl;
                sm += o.nm;
#pragma unroll
                for (int k = 0; k < LMAX; ++k) {
                    const bool a1 = k == p1, a2 = k == p2;
                    hx[k] += a1 ? o.d[1][0] : (a2 ? o.d[2][0] : 0.0);
                    hy[k] += a1 ? o.d[1][1] : (a2 ? o.d[2][1] : 0.0);
                }
            }
#pragma unroll
            for (int k = 0; k < LMAX; ++k)
                if (k == pd) {
                    hx[k] += ox;
                    hy[k] += oy;
                }
        }
        if (tile_fits) {
            __syncthreads();   // everyone is done reading the staged inputs
            const int32_t off = rs - E0;
            if (in_regs) {
#pragma unroll
                for (int k = 0; k < LMAX; ++k)
                    if (k < len) {
                        s_stage[2 * (off + k)] = hx[k];
                        s_stage[2 * (off + k) + 1] = hy[k];
                    }
            } else if (active && len > 0) {
                for (int k = 0; k < 2 * len; ++k) s_stage[2 * off + k] = 0.0;
            }
            __syncthreads();
            // with tpos, each value goes to the place of its transposed entry
            int32_t dst[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int e = lane + u * WAVE;
                dst[u] = e < Ew ? (tpos ? tpos[E0 + e] : E0 + e) : 0;
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int e = lane + u * WAVE;
                if (e < Ew && dst[u] >= 0)   // tpos -1: no transposed entry, no place
                    H[dst[u]] = make_double2(s_stage[2 * e], s_stage[2 * e + 1]);
            }
            __syncthreads();
        }
        if (!in_regs && active && len > 0) {
            // long row or tile too large: own row in global memory, same order
            // (each entry at its own place, transposed with tpos)
            // (an entry without a transposed partner, tpos -1, is skipped)
            auto hat = [&](int32_t e) -> int32_t { return tpos ? tpos[rs + e] : rs + e; };
            auto hadd = [&](int32_t e, double gx, double gy) {
                const int32_t d = hat(e);
                if (d < 0) return;
                double2 h = H[d];
                h.x += gx;
                h.y += gy;
                H[d] = h;
            };
            for (int e = 0; e < len; ++e) {
                const int32_t d = hat(e);
                if (d >= 0) H[d] = make_double2(0.0, 0.0);
            }
            const int32_t *cr = col_idx + rs;
            int32_t pd = 0;
            while (pd < len - 1 && cr[pd] != (int32_t)i) ++pd;
            const double *gr = G + 4 * (int64_t)rs;
            double x[3][2], g[3][4];
            x[0][0] = q[2 * i];
            x[0][1] = q[2 * i + 1];
            g[0][0] = gr[2 * pd];
            g[0][1] = gr[2 * pd + 1];
            g[0][2] = gr[2 * len + 2 * pd];
            g[0][3] = gr[2 * len + 2 * pd + 1];
            double ox = 0.0, oy = 0.0;
            for (int32_t t = is; t < ie; ++t) {
                const uint32_t pp = inc_pos[t];
                const int32_t p1 = (int32_t)(pp & 0xffffu), p2 = (int32_t)(pp >> 16);
                const int64_t j1 = cr[p1], j2 = cr[p2];
                x[1][0] = q[2 * j1];
                x[1][1] = q[2 * j1 + 1];
                x[2][0] = q[2 * j2];
                x[2][1] = q[2 * j2 + 1];
                g[1][0] = gr[2 * p1];
                g[1][1] = gr[2 * p1 + 1];
                g[1][2] = gr[2 * len + 2 * p1];
                g[1][3] = gr[2 * len + 2 * p1 + 1];
                g[2][0] = gr[2 * p2];
                g[2][1] = gr[2 * p2 + 1];
                g[2][2] = gr[2 * len + 2 * p2];
                g[2][3] = gr[2 * len + 2 * p2 + 1];
                ElasTau o;
                elas_tau(x, g, lam, mu, o);
                ox += o.d[0][0];
                oy += o.d[0][1];
                sl += o.nl;
                sm += o.nm;
                hadd(p1, o.d[1][0], o.d[1][1]);
                hadd(p2, o.d[2][0], o.d[2][1]);
            }
            hadd(pd, ox, oy);
        }
        // the tile's dtau/dlambda, dtau/dmu sums (a fixed shuffle tree)
        const double tl = wave_sum(sl), tm = wave_sum(sm);
        if (lane == 0) lm[tile] = make_double2(tl, tm);
    }
}

// Pass 1 of the elasticity adjoint over fan codes (as k_adj_rows_fan): LDS
// holds the tile's 4 Ew values of G and its H records (x, y); each lane
// gathers its neighbours' coordinates in walk order and writes every H value
// into LDS once complete.  The tile's dtau/dlambda, dtau/dmu sums go to
// lm[tile] (walk order inside a row).  Other rows: the per-lane global-memory
// path of k_adj_elas_rows.
template <int U, int N>
__global__ __launch_bounds__(WAVE) void k_adj_elas_rows_fan(
    int32_t nq, const double *__restrict__ q, const int32_t *__restrict__ row_ptr,
    const int32_t *__restrict__ col_idx, const int32_t *__restrict__ inc_ptr,
    const uint32_t *__restrict__ inc_pos, const uint64_t *__restrict__ fan,
    const int32_t *__restrict__ tpos, const double *__restrict__ G, double lam, double mu,
    double2 *__restrict__ H, double2 *__restrict__ lm, int64_t ntiles) {
    constexpr int EB = U * WAVE;
    extern __shared__ double smem[];
    double *s_g = smem;             // [4 EB]: the tile's G in the elasticity layout
    double *s_h = smem + 4 * EB;    // [2 EB]: (x, y) per entry
    const int lane = threadIdx.x;
    const double2 *q2 = reinterpret_cast<const double2 *>(q);
    for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const int64_t r0 = tile * WAVE;
        const int64_t r1 = (r0 + WAVE < nq) ? r0 + WAVE : nq;
        const int64_t i = r0 + lane;
        const bool active = i < nq;
        const int32_t E0 = row_ptr[r0], E1 = row_ptr[r1], Ew = E1 - E0;
        const int32_t rs = active ? row_ptr[i] : 0;
        const int32_t len = active ? row_ptr[i + 1] - rs : 0;
        const uint64_t code = active ? fan[i] : 0;
        const int n = fan_n(code);
        const bool closed = fan_closed(code);
        const bool tile_fits = Ew <= EB;
        const bool in_regs = tile_fits && active && n >= 2 && n <= N && len == n + 1;
        const bool zero_row = !in_regs && active && len > 0;
        const int32_t off = rs - E0;
        if (tile_fits) {
            // the tile's 4 Ew values of G, eight loads in flight per lane
            const double *gt = G + 4 * (int64_t)E0;
            for (int e0 = 0; e0 < 4 * Ew; e0 += 8 * WAVE) {
                double gv[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const int e = e0 + lane + u * WAVE;
                    gv[u] = e < 4 * Ew ? __builtin_nontemporal_load(gt + e) : 0.0;
                }
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const int e = e0 + lane + u * WAVE;
                    if (e < 4 * Ew) s_g[e] = gv[u];
                }
            }
        }
        int32_t cj[N];
#pragma unroll
        for (int j = 0; j < N; ++j) cj[j] = (in_regs && j < n) ? col_idx[rs + fan_slot(code, j)] : -1;
        double2 xn[N];
#pragma unroll
        for (int j = 0; j < N; ++j) xn[j] = cj[j] >= 0 ? q2[cj[j]] : make_double2(0.0, 0.0);
        const double2 xi = in_regs ? q2[i] : make_double2(0.0, 0.0);
        if (tile_fits) __syncthreads();   // G staged
        double sl = 0.0, sm = 0.0;
        if (in_regs) {
            const int32_t pd = fan_pd(code);
            const double *gr = s_g + 4 * off;   // row 2i at gr[2k + beta], row 2i+1 at gr[2len + 2k + beta]
            auto gblock = [&](int sl_, double (&g)[4]) {
                g[0] = gr[2 * sl_];
                g[1] = gr[2 * sl_ + 1];
                g[2] = gr[2 * len + 2 * sl_];
                g[3] = gr[2 * len + 2 * sl_ + 1];
            };
            auto put = [&](int sl_, double hx, double hy) {
                s_h[2 * (off + sl_)] = hx;
                s_h[2 * (off + sl_) + 1] = hy;
            };
            double x[3][2], g[3][4];
            x[0][0] = xi.x;
            x[0][1] = xi.y;
            gblock(pd, g[0]);
            double ox = 0.0, oy = 0.0, cx = 0.0, cy = 0.0, fx = 0.0, fy = 0.0;
            const int d = closed ? n : n - 1;
#pragma unroll
            for (int j = 0; j < N; ++j) {
                if (j < d) {
                    const bool wrap = j + 1 >= n;
                    const int jn = j + 1 < N ? j + 1 : 0;
                    const double2 x2 = wrap ? xn[0] : xn[jn];
                    x[1][0] = xn[j].x;
                    x[1][1] = xn[j].y;
                    x[2][0] = x2.x;
                    x[2][1] = x2.y;
                    gblock(fan_slot(code, j), g[1]);
                    gblock(wrap ? fan_slot(code, 0) : fan_slot(code, jn), g[2]);
                    ElasTau o;
                    elas_tau(x, g, lam, mu, o);
                    ox += o.d[0][0];
                    oy += o.d[0][1];
                    sl += o.nl;
                    sm += o.nm;
                    if (j == 0) {
                        fx = o.d[1][0];
                        fy = o.d[1][1];
                        if (!closed) put(fan_slot(code, 0), fx, fy);
                    } else {
                        put(fan_slot(code, j), cx + o.d[1][0], cy + o.d[1][1]);
                    }
                    cx = o.d[2][0];
                    cy = o.d[2][1];
                }
            }
            if (closed) put(fan_slot(code, 0), fx + cx, fy + cy);
            else put(fan_slot(code, n - 1), cx, cy);
            put(pd, ox, oy);
        } else if (tile_fits && zero_row) {
            for (int k = 0; k < 2 * len; ++k) s_h[2 * off + k] = 0.0;
        }
        if (tile_fits) {
            __syncthreads();
            // with tpos, each value goes to the place of its transposed entry
            int32_t dst[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int e = lane + u * WAVE;
                dst[u] = e < Ew ? (tpos ? tpos[E0 + e] : E0 + e) : 0;
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int e = lane + u * WAVE;
                if (e < Ew && dst[u] >= 0)   // tpos -1: no transposed entry, no place
                    H[dst[u]] = make_double2(s_h[2 * e], s_h[2 * e + 1]);
            }
            __syncthreads();
        }
        if (zero_row) {
            // ascending triangles from global memory, as in k_adj_elas_rows
            auto hat = [&](int32_t e) -> int32_t { return tpos ? tpos[rs + e] : rs + e; };
            auto hadd = [&](int32_t e, double gx, double gy) {
                const int32_t dd = hat(e);
                if (dd < 0) return;
                double2 h = H[dd];
                h.x += gx;
                h.y += gy;
                H[dd] = h;
            };
            if (!tile_fits) {
                for (int e = 0; e < len; ++e) {
                    const int32_t dd = hat(e);
                    if (dd >= 0) H[dd] = make_double2(0.0, 0.0);
                }
            }
            const int32_t is = inc_ptr[i], ie = inc_ptr[i + 1];
            const int32_t *cr = col_idx + rs;
            int32_t pd = 0;
            while (pd < len - 1 && cr[pd] != (int32_t)i) ++pd;
            const double *gr = G + 4 * (int64_t)rs;
            double x[3][2], g[3][4];
            x[0][0] = q[2 * i];
            x[0][1] = q[2 * i + 1];
            g[0][0] = gr[2 * pd];
            g[0][1] = gr[2 * pd + 1];
            g[0][2] = gr[2 * len + 2 * pd];
            g[0][3] = gr[2 * len + 2 * pd + 1];
            double ox = 0.0, oy = 0.0;
            for (int32_t t = is; t < ie; ++t) {
                const uint32_t pp = inc_pos[t];
                const int32_t p1 = (int32_t)(pp & 0xffffu), p2 = (int32_t)(pp >> 16);
                const int64_t j1 = cr[p1], j2 = cr[p2];
                x[1][0] = q[2 * j1];
                x[1][1] = q[2 * j1 + 1];
                x[2][0] = q[2 * j2];
                x[2][1] = q[2 * j2 + 1];
                g[1][0] = gr[2 * p1];
                g[1][1] = gr[2 * p1 + 1];
                g[1][2] = gr[2 * len + 2 * p1];
                g[1][3] = gr[2 * len + 2 * p1 + 1];
                g[2][0] = gr[2 * p2];
                g[2][1] = gr[2 * p2 + 1];
                g[2][2] = gr[2 * len + 2 * p2];
                g[2][3] = gr[2 * len + 2 * p2 + 1];
                ElasTau o;
                elas_tau(x, g, lam, mu, o);
                ox += o.d[0][0];
                oy += o.d[0][1];
                sl += o.nl;
                sm += o.nm;
                hadd(p1, o.d[1][0], o.d[1][1]);
                hadd(p2, o.d[2][0], o.d[2][1]);
            }
            hadd(pd, ox, oy);
        }
        // the tile's dtau/dlambda, dtau/dmu sums (a fixed shuffle tree)
        const double tl = wave_sum(sl), tm = wave_sum(sm);
        if (lane == 0) lm[tile] = make_double2(tl, tm);
    }
}

// Pass 2 of the elasticity adjoint: dq[u] = sum over row u of H at the
// transposed positions, ascending position.  With tpos, pass 1 has already
// stored every value at the place of its transposed entry, so row u is read
// in place; without it, each transposed entry is found by search.
template <int U>
__global__ __launch_bounds__(WAVE) void k_adj_elas_cols(int32_t nq, const int32_t *__restrict__ row_ptr,
                                                        const int32_t *__restrict__ col_idx,
                                                        const int32_t *__restrict__ tpos,
                                                        const double2 *__restrict__ H,
                                                        double *__restrict__ dq, int accumulate,
                                                        int64_t ntiles, const double2 *__restrict__ lm,
                                                        double *__restrict__ dlm) {
    constexpr int EB = U * WAVE;
    __shared__ double s_h[2 * EB];
    const int lane = threadIdx.x;
    // dL/dlambda, dL/dmu: workgroup 0 (dispatched first, beside the column
    // sums) adds pass 1's per-tile sums in a fixed order -- lane t takes
    // entries t, t + 64, ... in turn, then a fixed butterfly over the wave --
    // so the result is bitwise reproducible.
    const int lead = dlm ? 1 : 0;
    if (dlm && blockIdx.x == 0) {
        double l = 0.0, m = 0.0;
        for (int64_t i0 = lane; i0 < ntiles; i0 += 4 * WAVE) {
            double2 v[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const int64_t i = i0 + k * WAVE;
                v[k] = i < ntiles ? lm[i] : make_double2(0.0, 0.0);
            }
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                l += v[k].x;
                m += v[k].y;
            }
        }
        l = wave_sum(l);
        m = wave_sum(m);
        if (lane == 0) {
            if (accumulate) {
                dlm[0] += l;
                dlm[1] += m;
            } else {
                dlm[0] = l;
                dlm[1] = m;
            }
        }
        return;
    }
    for (int64_t tile = blockIdx.x - lead; tile < ntiles; tile += gridDim.x - lead) {
        const int64_t r0 = tile * WAVE;
        const int64_t r1 = (r0 + WAVE < nq) ? r0 + WAVE : nq;
        const int64_t u = r0 + lane;
        const bool active = u < nq;
        const int32_t E0 = row_ptr[r0], E1 = row_ptr[r1], Ew = E1 - E0;
        const int32_t rs = active ? row_ptr[u] : 0;
        const int32_t re = active ? row_ptr[u + 1] : 0;
        double gx = 0.0, gy = 0.0;
        if (tpos && Ew <= EB) {
            double2 h[U];
#pragma unroll
            for (int k = 0; k < U; ++k) {
                const int e = lane + k * WAVE;
                h[k] = e < Ew ? H[E0 + e] : make_double2(0.0, 0.0);
            }
#pragma unroll
            for (int k = 0; k < U; ++k) {
                const int e = lane + k * WAVE;
                if (e < Ew) {
                    s_h[2 * e] = h[k].x;
                    s_h[2 * e + 1] = h[k].y;
                }
            }
            __syncthreads();
            for (int32_t e = rs - E0; e < re - E0; ++e) {
                gx += s_h[2 * e];
                gy += s_h[2 * e + 1];
            }
            __syncthreads();
        } else {
            for (int32_t p = rs; p < re; ++p) {
                int32_t tp;
                if (tpos) {
                    tp = p;   // already transposed by pass 1
                } else {
                    const int32_t v = col_idx[p];
                    int32_t lo = row_ptr[v], hi = row_ptr[v + 1];
                    while (lo < hi) {
                        const int32_t mid = (lo + hi) >> 1;
                        if (col_idx[mid] < (int32_t)u) lo = mid + 1;
                        else hi = mid;
                    }
                    tp = lo;
                }
                const double2 hv = H[tp];
                gx += hv.x;
                gy += hv.y;
            }
        }
        if (!active) continue;
        if (accumulate) {
            dq[2 * u] += gx;
            dq[2 * u + 1] += gy;
        } else {
            dq[2 * u] = gx;
            dq[2 * u + 1] = gy;
        }
    }
}

namespace {
constexpr int ADJ_U = 8;

constexpr int ADJ_LMAX = 8;

constexpr int ADJ_FAN = 8;   // neighbour slots walked in registers by k_adj_rows_fan

template <bool HS, bool HM>
int launch_adj(int32_t nq, const double4 *qw, const int32_t *row_ptr, const int32_t *col_idx,
               const int32_t *inc_ptr, const uint32_t *inc_pos, const uint64_t *fan,
               const int32_t *tpos, const double *GS, const double *GM, double4 *H, hipStream_t s) {
    const int64_t ntiles = (nq + WAVE - 1) / WAVE;
    if (fan) {
        const size_t lds = (size_t)ADJ_U * WAVE * 5 * 8;
        hipLaunchKernelGGL((k_adj_rows_fan<HS, HM, ADJ_U, ADJ_FAN>), dim3((unsigned)ntiles), dim3(WAVE),
                           lds, s, nq, qw, row_ptr, col_idx, inc_ptr, inc_pos, fan, tpos, GS, GM, H,
                           ntiles);
        FEM_LAUNCH_CHECK();
        return FEM_OK;
    }
    const size_t lds = (size_t)ADJ_U * WAVE * (5 * 8 + 4);
    hipLaunchKernelGGL((k_adj_rows<HS, HM, ADJ_U, ADJ_LMAX>), dim3((unsigned)ntiles), dim3(WAVE), lds,
                       s, nq, qw, row_ptr, col_idx, inc_ptr, inc_pos, tpos, GS, GM, H, ntiles);
    FEM_LAUNCH_CHECK();
    return FEM_OK;
}

inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }
}  // namespace

}  // namespace fem

using namespace fem;

extern "C" int fem_adjoint_workspace(int32_t nq, int64_t nnz, size_t *bytes) {
    clear_error();
    FEM_REQUIRE(bytes && nq >= 1 && nnz >= 0, FEM_EINVAL, "fem_adjoint_workspace: bad arguments");
    *bytes = align256(sizeof(double4) * (size_t)nq) + sizeof(double4) * (size_t)(nnz > 0 ? nnz : 1);
    return FEM_OK;
}

extern "C" int fem_adjoint_stiff_wmass(int32_t nq, int32_t nme, int64_t nnz, const double *q,
                                       const double *w, const int32_t *row_ptr,
                                       const int32_t *col_idx, const int32_t *inc_ptr,
                                       const uint32_t *inc_pos, const uint64_t *fan,
                                       const int32_t *tpos, const double *GS, const double *GM,
                                       double *dq, double *dw,
                                       void *work, size_t work_bytes, int flags, void *stream) {
    clear_error();
    FEM_REQUIRE(nq >= 1 && nme >= 0 && nnz >= 0 && nnz <= INT32_MAX, FEM_EINVAL,
                "fem_adjoint_stiff_wmass: bad sizes");
    FEM_REQUIRE((flags & ~(FEM_ACCUMULATE | FEM_PACKED_QW)) == 0, FEM_EINVAL,
                "fem_adjoint_stiff_wmass: only FEM_ACCUMULATE and FEM_PACKED_QW are supported");
    FEM_REQUIRE(q && row_ptr && dq && work, FEM_EINVAL, "fem_adjoint_stiff_wmass: NULL q, row_ptr, dq or work");
    FEM_REQUIRE(nnz == 0 || (col_idx && inc_ptr && inc_pos), FEM_EINVAL,
                "fem_adjoint_stiff_wmass: NULL pattern array");
    FEM_REQUIRE(!GM || (w && dw), FEM_EINVAL, "fem_adjoint_stiff_wmass: the GM term needs w and dw");
    size_t need = 0;
    fem_adjoint_workspace(nq, nnz, &need);
    FEM_REQUIRE(work_bytes >= need, FEM_ENOSPC, "fem_adjoint_stiff_wmass: workspace %zu < %zu",
                work_bytes, need);
    hipStream_t s = as_stream(stream);
    double4 *qw = static_cast<double4 *>(work);
    double4 *H = reinterpret_cast<double4 *>(static_cast<char *>(work) + align256(sizeof(double4) * (size_t)nq));
    if (!(flags & FEM_PACKED_QW)) {
        hipLaunchKernelGGL(k_adj_pack, dim3(grid_for(nq, 256)), dim3(256), 0, s, nq,
                           reinterpret_cast<const double2 *>(q), GM ? w : nullptr, qw);
        FEM_LAUNCH_CHECK();
    }
    int st;
    if (GS && GM)
        st = launch_adj<true, true>(nq, qw, row_ptr, col_idx, inc_ptr, inc_pos, fan, tpos, GS, GM, H, s);
    else if (GS)
        st = launch_adj<true, false>(nq, qw, row_ptr, col_idx, inc_ptr, inc_pos, fan, tpos, GS, GM, H, s);
    else if (GM)
        st = launch_adj<false, true>(nq, qw, row_ptr, col_idx, inc_ptr, inc_pos, fan, tpos, GS, GM, H, s);
    else st = fill_f64(reinterpret_cast<double *>(H), 4 * nnz, 0.0, s);
    if (st) return st;
    const int acc = (flags & FEM_ACCUMULATE) ? 1 : 0;
    if (tpos) {
        const int64_t ntiles = (nq + WAVE - 1) / WAVE;
        hipLaunchKernelGGL(k_adj_cols_tpos<ADJ_U>, dim3((unsigned)ntiles), dim3(WAVE), 0, s, nq,
                           row_ptr, tpos, H, dq, dw, acc, ntiles);
    } else {
        hipLaunchKernelGGL(k_adj_cols, dim3(grid_for(nq, 256)), dim3(256), 0, s, nq, row_ptr,
                           col_idx, tpos, H, dq, dw, acc);
    }
    FEM_LAUNCH_CHECK();
    return FEM_OK;
}

extern "C" int fem_adjoint_elas_workspace(int32_t nq, int64_t nnz, size_t *bytes) {
    clear_error();
    FEM_REQUIRE(bytes && nq >= 1 && nnz >= 0, FEM_EINVAL, "fem_adjoint_elas_workspace: bad arguments");
    *bytes = align256(sizeof(double2) * (size_t)nq) + sizeof(double2) * (size_t)(nnz > 0 ? nnz : 1);
    return FEM_OK;
}

extern "C" int fem_adjoint_elas(int32_t nq, int32_t nme, int64_t nnz, const double *q,
                                const int32_t *row_ptr, const int32_t *col_idx,
                                const int32_t *inc_ptr, const uint32_t *inc_pos, const uint64_t *fan,
                                const int32_t *tpos, double lambda, double mu, const double *G,
                                double *dq, double *dlm, void *work, size_t work_bytes, int flags,
                                void *stream) {
    clear_error();
    FEM_REQUIRE(nq >= 1 && nme >= 0 && nnz >= 0 && 4 * nnz <= INT32_MAX, FEM_EINVAL,
                "fem_adjoint_elas: bad sizes");
    FEM_REQUIRE((flags & ~FEM_ACCUMULATE) == 0, FEM_EINVAL,
                "fem_adjoint_elas: only FEM_ACCUMULATE is supported");
    FEM_REQUIRE(q && row_ptr && dq && work, FEM_EINVAL, "fem_adjoint_elas: NULL q, row_ptr, dq or work");
    FEM_REQUIRE(nnz == 0 || (col_idx && inc_ptr && inc_pos && G), FEM_EINVAL,
                "fem_adjoint_elas: NULL pattern array or G");
    size_t need = 0;
    fem_adjoint_elas_workspace(nq, nnz, &need);
    FEM_REQUIRE(work_bytes >= need, FEM_ENOSPC, "fem_adjoint_elas: workspace %zu < %zu", work_bytes, need);
    hipStream_t s = as_stream(stream);
    double2 *lm = static_cast<double2 *>(work);
    double2 *H = reinterpret_cast<double2 *>(static_cast<char *>(work) + align256(sizeof(double2) * (size_t)nq));
    const int64_t ntiles = (nq + WAVE - 1) / WAVE;
    if (fan) {
        const size_t lds = (size_t)ADJ_U * WAVE * 6 * 8;
        hipLaunchKernelGGL((k_adj_elas_rows_fan<ADJ_U, ADJ_FAN>), dim3((unsigned)ntiles), dim3(WAVE), lds,
                           s, nq, q, row_ptr, col_idx, inc_ptr, inc_pos, fan, tpos, G, lambda, mu, H,
                           lm, ntiles);
    } else {
        const size_t lds = (size_t)ADJ_U * WAVE * (6 * 8 + 4);
        hipLaunchKernelGGL((k_adj_elas_rows<ADJ_U, ADJ_LMAX>), dim3((unsigned)ntiles), dim3(WAVE), lds, s,
                           nq, q, row_ptr, col_idx, inc_ptr, inc_pos, tpos, G, lambda, mu, H, lm, ntiles);
    }
    FEM_LAUNCH_CHECK();
    const int acc = (flags & FEM_ACCUMULATE) ? 1 : 0;
    hipLaunchKernelGGL(k_adj_elas_cols<ADJ_U>, dim3((unsigned)(ntiles + (dlm ? 1 : 0))), dim3(WAVE), 0, s,
                       nq, row_ptr, col_idx, tpos, H, dq, acc, ntiles, lm, dlm);
    FEM_LAUNCH_CHECK();
    return FEM_OK;
}
