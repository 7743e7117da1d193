// march2.h -- band-limited ray march with deferred crossing solves.
//
// Same quantity as march.h (exact below-lengths of every surface, paper
// Sec. 2.1.1 opacity of the layered density), organised for CDNA wavefronts:
//
//  * Bands.  Surface l can only be crossed while z(t) lies in its band
//    [min_l - margin, max_l + margin] over the chain's node values; before
//    the band the ray is certainly below it, after the band certainly above.
//    Each ray therefore tests surface l only on the cell pieces inside its
//    band, starts the 2-D cell walk at the lowest band and jumps over height
//    gaps where no band is active (every surface is certain there).
//  * Deferred solves.  A piece whose z-range overlaps the patch's corner range
//    is ambiguous; instead of solving it at once (which makes the whole wave
//    wait on the few lanes that need it) the lane appends it to its own queue
//    in LDS.  Queues are drained when some lane's queue is full and at the
//    end of the ray, so most solves run with most lanes active.  Each lane
//    only ever adds its own entries, in its own order: the result does not
//    depend on the other lanes, and repeat runs are bitwise identical.
//
// The crossing decision of a queued piece uses the same boundary formulas as
// march.h, so two cells that meet at an edge still see identical end values.
#pragma once

#include "march.h"

namespace mc {

template <typename T, int S, bool TOP_LDS>
__device__ __forceinline__ const T *surface_ptr(const T *sh, const T *top_g, int N, int l) {
    if (TOP_LDS) return sh + l * N;
    return l < S - 1 ? sh + l * N : top_g;
}

// Below-length of one queued piece [ta, tb] of cell (a, b) and surface l.
template <typename T, int S, bool TOP_LDS>
__device__ __forceinline__ T solve_piece(const MarchParams<T> &P, const T *sh, const T *top_g, T qx, T qy, T qz,
                                         T dx, T dy, T dz, bool xpos, bool ypos, T ta, T tb, uint32_t pk,
                                         int &l) {
    const int a = pk & 0xFF, b = (pk >> 8) & 0xFF;
    l = (pk >> 16) & 0xF;
    const int ek = (pk >> 20) & 0xF, xk = (pk >> 24) & 0xF;
    const int C = P.C;
    const T *Hl = surface_ptr<T, S, TOP_LDS>(sh, top_g, P.R * C, l);
    const int base = a * C + b;
    const T h00 = Hl[base], h01 = Hl[base + 1], h10 = Hl[base + C], h11 = Hl[base + C + 1];
    const T z0 = dfma(ta, dz, qz), z1 = dfma(tb, dz, qz);
    const T se = dfma(dfma(ta, dx, qx), P.ihx, -T(a)), we = dfma(dfma(ta, dy, qy), P.ihy, -T(b));
    const T sx = dfma(dfma(tb, dx, qx), P.ihx, -T(a)), wx = dfma(dfma(tb, dy, qy), P.ihy, -T(b));
    const T fe = boundary_value(ek, true, xpos, ypos, z0, se, we, h00, h10, h01, h11);
    const T fx = boundary_value(xk, false, xpos, ypos, z1, sx, wx, h00, h10, h01, h11);
    const T c2 = -(h11 - h10 - h01 + h00) * (dx * P.ihx) * (dy * P.ihy);
    return cell_below_length(fe, fx, c2, tb - ta);
}

template <typename T>
__device__ __forceinline__ void cswap(T &a0, T &a1, T &b0, T &b1) {
    // order the pairs (a0, a1), (b0, b1) by their first element
    const bool sw = b0 < a0;
    const T x0 = sw ? b0 : a0, x1 = sw ? b1 : a1;
    const T y0 = sw ? a0 : b0, y1 = sw ? a1 : b1;
    a0 = x0;
    a1 = x1;
    b0 = y0;
    b1 = y1;
}

// March one ray.  qt/qp: this lane's queue (slot stride BLOCK).
template <typename T, int S, bool TOP_LDS, int BLOCK, int Q>
__device__ __forceinline__ T march_ray2(const MarchParams<T> &P, const T *sh, const T *top_g, const T *lo,
                                        const T *hi, T qx, T qy, T qz, T dx, T dy, T dz, T *qt, uint32_t *qp,
                                        T (&L)[S]) {
    const T INF = dev_inf<T>();
    const int R = P.R, C = P.C;
    const T idx = dx != T(0) ? T(1) / dx : T(0);
    const T idy = dy != T(0) ? T(1) / dy : T(0);
    const T idz = T(1) / dz;
    const bool xpos = dx > T(0), ypos = dy > T(0);
    T Texit = (P.ztop - qz) * idz;
    if (dx > T(0)) Texit = dmin(Texit, (P.xmax - qx) * idx);
    if (dx < T(0)) Texit = dmin(Texit, (T(0) - qx) * idx);
    if (dy > T(0)) Texit = dmin(Texit, (P.ymax - qy) * idy);
    if (dy < T(0)) Texit = dmin(Texit, (T(0) - qy) * idy);
    Texit = dmax(Texit, T(0));
    // per-surface band in t; below before it, above after it
    T tlo[S], thi[S];
#pragma unroll
    for (int l = 0; l < S; ++l) {
        tlo[l] = dmin(dmax((lo[l] - qz) * idz, T(0)), Texit);
        thi[l] = dmin(dmax((hi[l] - qz) * idz, T(0)), Texit);
        L[l] = tlo[l];
    }
    // bands sorted by start; gaps between their union
    T slo[S], shi[S];
#pragma unroll
    for (int l = 0; l < S; ++l) {
        slo[l] = tlo[l];
        shi[l] = thi[l];
    }
#pragma unroll
    for (int i = 0; i < S; ++i)
#pragma unroll
        for (int j = 0; j + 1 < S - i; ++j) cswap(slo[j], shi[j], slo[j + 1], shi[j + 1]);
    constexpr int NG = S > 1 ? S - 1 : 1;
    T glo[NG], ghi[NG];
    T reach = shi[0];
#pragma unroll
    for (int k = 1; k < S; ++k) {
        const bool g = slo[k] > reach;
        glo[k - 1] = g ? reach : INF;
        ghi[k - 1] = g ? slo[k] : INF;
        reach = dmax(reach, shi[k]);
    }
    if (S == 1) glo[0] = ghi[0] = INF;
#pragma unroll
    for (int i = 0; i < NG; ++i)
#pragma unroll
        for (int j = 0; j + 1 < NG - i; ++j) cswap(glo[j], ghi[j], glo[j + 1], ghi[j + 1]);
    const T t_start = slo[0], t_stop = reach;
    int qn = 0;

    auto flush = [&]() {
        for (int k = 0; k < qn; ++k) {
            const T ta = qt[(2 * k) * BLOCK], tb = qt[(2 * k + 1) * BLOCK];
            const uint32_t pk = qp[k * BLOCK];
            int l;
            const T len = solve_piece<T, S, TOP_LDS>(P, sh, top_g, qx, qy, qz, dx, dy, dz, xpos, ypos, ta, tb, pk, l);
#pragma unroll
            for (int s = 0; s < S; ++s)
                if (s == l) L[s] += len;
        }
        qn = 0;
    };

    if (t_start < t_stop) {
        const int sxs = xpos ? 1 : -1, sys = ypos ? 1 : -1;
        int a, b;
        auto locate = [&](T t) {
            const T x = dfma(t, dx, qx), y = dfma(t, dy, qy);
            a = (int)floor(x * P.ihx);
            b = (int)floor(y * P.ihy);
            a = a < 0 ? 0 : (a > R - 2 ? R - 2 : a);
            b = b < 0 ? 0 : (b > C - 2 ? C - 2 : b);
        };
        locate(t_start);
        T t0 = t_start;
        int ekind = kPoint;
        const int max_it = S * (R + C) + 2 * S;
        for (int it = 0; it < max_it; ++it) {
            const T tnx = xpos ? (T(a + 1) * P.hx - qx) * idx : (dx < T(0) ? (T(a) * P.hx - qx) * idx : INF);
            const T tny = ypos ? (T(b + 1) * P.hy - qy) * idy : (dy < T(0) ? (T(b) * P.hy - qy) * idy : INF);
            const bool stepx = tnx <= tny;
            const T tn = stepx ? tnx : tny;
            const int na = a + (stepx ? sxs : 0), nb = b + (stepx ? 0 : sys);
            const bool in_range = na >= 0 && na <= R - 2 && nb >= 0 && nb <= C - 2;
            const T tcap = dmin(t_stop, glo[0]);
            const bool edge = (tn < tcap) && in_range;
            const T t1 = dmax(dmin(tn, tcap), t0);
            const int xkind = edge ? (stepx ? kXEdge : kYEdge) : kPoint;
            const int base = a * C + b;
            const uint32_t cell_bits = (uint32_t)a | ((uint32_t)b << 8);
#pragma unroll
            for (int l = 0; l < S; ++l) {
                const T ta = dmax(t0, tlo[l]), tb = dmin(t1, thi[l]);
                if (ta < tb) {
                    const T *Hl = surface_ptr<T, S, TOP_LDS>(sh, top_g, R * C, l);
                    const T h00 = Hl[base], h01 = Hl[base + 1], h10 = Hl[base + C], h11 = Hl[base + C + 1];
                    const T hmin = dmin(dmin(h00, h10), dmin(h01, h11));
                    const T hmax = dmax(dmax(h00, h10), dmax(h01, h11));
                    const T za = dfma(ta, dz, qz), zb = dfma(tb, dz, qz);
                    if (zb < hmin - P.margin) {
                        L[l] += tb - ta;
                    } else if (!(za > hmax + P.margin)) {
                        const int ek = (ta == t0) ? ekind : kPoint;
                        const int xk = (tb == t1) ? xkind : kPoint;
                        qt[(2 * qn) * BLOCK] = ta;
                        qt[(2 * qn + 1) * BLOCK] = tb;
                        qp[qn * BLOCK] = cell_bits | ((uint32_t)l << 16) | ((uint32_t)ek << 20) | ((uint32_t)xk << 24);
                        ++qn;
                    }
                }
                if (__any(qn == Q)) flush();
            }
            if (edge) {
                a = na;
                b = nb;
                t0 = t1;
                ekind = stepx ? kXEdge : kYEdge;
            } else if (!(tn >= tcap) || !(t1 < t_stop)) {
                break;   // left the box sideways, or past the last band
            } else {
                // jump over a height gap where every surface is certain
                t0 = ghi[0];
#pragma unroll
                for (int k = 0; k + 1 < NG; ++k) {
                    glo[k] = glo[k + 1];
                    ghi[k] = ghi[k + 1];
                }
                glo[NG - 1] = ghi[NG - 1] = INF;
                locate(t0);
                ekind = kPoint;
            }
        }
    }
    flush();
    T O = T(0);
#pragma unroll
    for (int l = 0; l < S; ++l) O += P.rho_diff[l] * L[l];
    return O;
}

// One block = one chain x one tile of rays (as k_march_lik), with the
// band-limited march and the per-lane crossing queues in LDS after the
// surfaces.
template <typename T, int S, bool TOP_LDS, int BLOCK, int Q>
__global__ __launch_bounds__(BLOCK) void k_march_lik2(MarchParams<T> P) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *sh = reinterpret_cast<T *>(smem_raw);
    __shared__ double red[16];
    __shared__ T band[2 * kMaxSurfaces];
    const int chain = blockIdx.y, tile = blockIdx.x, tid = threadIdx.x;
    if (P.only_nan && !(P.only_nan[chain] != P.only_nan[chain])) return;
    const int N = P.R * P.C;
    const size_t surf_elems = (size_t)N * (TOP_LDS ? S : S - 1);
    const size_t surf_bytes = (surf_elems * sizeof(T) + 15) & ~(size_t)15;
    T *qt = reinterpret_cast<T *>(smem_raw + surf_bytes) + tid;
    uint32_t *qp = reinterpret_cast<uint32_t *>(smem_raw + surf_bytes + sizeof(T) * 2 * Q * BLOCK) + tid;
    const T *Hc = P.heights + (size_t)chain * (S - 1) * N;
    T mn[S], mx[S];
#pragma unroll
    for (int l = 0; l < S - 1; ++l) {
        T a = dev_inf<T>(), b = -dev_inf<T>();
        for (int i = tid; i < N; i += BLOCK) {
            T v = Hc[l * N + i];
            sh[l * N + i] = v;
            a = dmin(a, v);
            b = dmax(b, v);
        }
        mn[l] = a;
        mx[l] = b;
    }
    if (TOP_LDS) {
        for (int i = tid; i < N; i += BLOCK) sh[(S - 1) * N + i] = P.top[i];
    }
    {
        __shared__ T wred[2 * kMaxSurfaces][BLOCK / kWave];
        const int lane = tid % kWave, wid = tid / kWave;
#pragma unroll
        for (int l = 0; l < S - 1; ++l) {
            T a = wave_min(mn[l]), b = wave_max(mx[l]);
            if (lane == 0) {
                wred[2 * l][wid] = a;
                wred[2 * l + 1][wid] = b;
            }
        }
        __syncthreads();
        if (tid == 0) {
#pragma unroll
            for (int l = 0; l < S - 1; ++l) {
                T a = wred[2 * l][0], b = wred[2 * l + 1][0];
                for (int w = 1; w < BLOCK / kWave; ++w) {
                    a = dmin(a, wred[2 * l][w]);
                    b = dmax(b, wred[2 * l + 1][w]);
                }
                band[l] = a - P.margin;
                band[kMaxSurfaces + l] = b + P.margin;
            }
            band[S - 1] = P.top_min - P.margin;
            band[kMaxSurfaces + S - 1] = P.top_max + P.margin;
        }
        __syncthreads();
    }
    T lo[S], hi[S];
#pragma unroll
    for (int l = 0; l < S; ++l) {
        lo[l] = band[l];
        hi[l] = band[kMaxSurfaces + l];
    }
    double acc = 0.0;
    const int r0 = tile * P.rays_per_block;
    const int r1 = min(r0 + P.rays_per_block, P.n_ray);
    for (int ray = r0 + tid; ray < r1; ray += BLOCK) {
        const int s = ray / P.n_pix;
        T L[S];
        const T O = march_ray2<T, S, TOP_LDS, BLOCK, Q>(P, sh, P.top, lo, hi, P.sensor[3 * s], P.sensor[3 * s + 1],
                                                        P.sensor[3 * s + 2], P.dx[ray], P.dy[ray], P.dz[ray], qt,
                                                        qp, L);
        if (P.opacity) P.opacity[(size_t)chain * P.n_ray + ray] = O;
        const double Od = (double)O;
        acc += -P.c_over_L[ray] * Od - P.expo[ray] * exp(-Od * P.inv_L);
    }
    const double tot = block_sum<BLOCK>(acc, red);
    if (tid == 0) P.partials[(size_t)chain * P.n_tiles + tile] = tot;
}

}  // namespace mc
