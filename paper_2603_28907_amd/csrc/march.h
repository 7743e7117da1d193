// march.h -- exact ray march through bilinear layer height fields, fused with
// the per-pixel Poisson term and a deterministic per-block reduction.
//
// Opacity (paper Sec. 2.1.1) of the layered density (eq. def_LM_density_grid,
// continuum form): O = sum_l (rho_l - rho_{l+1}) L_l, with L_l the length of
// ray inside the box lying below surface l.  Inside a grid cell the surface
// restricted to the ray is a quadratic in t, so L_l is a sum of exact
// per-cell pieces.
//
// Robust per-cell evaluation.  Each cell interval [t0, t1] of the 2-D cell
// walk is either certain (the ray's z-range lies entirely below the patch
// minimum or above its maximum, with a rounding margin) or ambiguous.  In an
// ambiguous cell the signs of f = z - h at the two ends decide the number of
// crossings; each end value is computed by one formula that depends only on
// the boundary point (the lerp along the shared cell edge), so the two cells
// that meet at a boundary see the same bits and a crossing is never dropped
// or counted twice.  The in-cell quadratic is rebuilt from the two end values
// and the patch curvature c2 = -D ds dw.
#pragma once

#include "device_common.h"

namespace mc {

enum BoundaryKind : int { kPoint = 0, kXEdge = 1, kYEdge = 2 };

template <typename T>
struct MarchParams {
    int R, C, n_ray, n_pix, n_tiles, rays_per_block;
    int n_chains;                      // chains in the launch
    T hx, hy, ihx, ihy, xmax, ymax;   // cell sizes, their inverses, (R-1) hx, (C-1) hy
    T ztop;                            // max of the top surface
    T margin;                          // rounding margin for the certain tests
    T top_min, top_max;                // range of the top surface
    T rho_diff[kMaxSurfaces];          // rho_l - rho_{l+1}
    const T *sensor;                   // [n_s][3]
    const T *dx, *dy, *dz;             // [n_ray] ray directions
    const double *c_over_L;            // [n_ray] C_p / Lambda
    const double *expo;                // [n_ray] E_p
    double inv_L;                      // 1 / Lambda
    const T *top;                      // [R*C] fixed top surface
    const T *heights;                  // [n_chains][S-1][R*C]
    T *opacity;                        // [n_chains][n_ray] or null
    double *partials;                  // [n_chains][n_tiles]
    const double *only_nan;            // if set, chains whose entry is not NaN are skipped
};

// Below-length of one cell piece given the end values fe, fx of f = z - h and
// the curvature c2 of f along the ray (tau in [0, tau1]).
template <typename T>
__device__ __forceinline__ T cell_below_length(T fe, T fx, T c2, T tau1) {
    const bool be = fe < T(0), bx = fx < T(0);
    // quadratic through (0, fe) and (tau1, fx) with curvature c2
    const T c1 = (fx - fe) / tau1 - c2 * tau1;
    if (be != bx) {
        // exactly one crossing in the cell
        T disc = dmax(c1 * c1 - T(4) * c2 * fe, T(0));
        T sq = dsqrt(disc);
        T q = T(-0.5) * (c1 + (c1 >= T(0) ? sq : -sq));
        T r1 = q / c2, r2 = fe / q;
        T d1 = dmax(dmax(-r1, r1 - tau1), T(0));
        T d2 = dmax(dmax(-r2, r2 - tau1), T(0));
        bool use1 = (d1 < d2) || (d2 != d2);
        T r = use1 ? r1 : r2;
        if (r != r) r = tau1 * fe / (fe - fx);   // secant fallback
        r = dmin(dmax(r, T(0)), tau1);
        return be ? r : tau1 - r;
    }
    if (c2 != T(0)) {
        const T tv = -c1 / (T(2) * c2);
        if (tv > T(0) && tv < tau1) {
            const T fv = fe + tv * (c1 + c2 * tv);
            if ((fv < T(0)) != be) {
                // two crossings around the vertex
                T disc = dmax(c1 * c1 - T(4) * c2 * fe, T(0));
                T half = dsqrt(disc) / (T(2) * dabs(c2));
                T ta = dmax(tv - half, T(0)), tb = dmin(tv + half, tau1);
                T inner = dmax(tb - ta, T(0));
                return be ? tau1 - inner : inner;
            }
        }
    }
    return be ? tau1 : T(0);
}

// Geometry of one cell piece shared by all surfaces.
template <typename T>
struct CellPiece {
    T t0, t1, z0, z1;
    T se, we, sx, wx;   // local coordinates at entry and exit
    int ekind, xkind;
};

// f = z - h at a boundary point of the piece.  kind/entry pick the formula:
// an x-edge (node row) lerps along y, a y-edge (node column) lerps along x,
// a point inside the box uses the full bilinear patch.
template <typename T>
__device__ __forceinline__ T boundary_value(int kind, bool entry, bool xpos, bool ypos, T z, T s, T w,
                                            T h00, T h10, T h01, T h11) {
    if (kind == kXEdge) {
        // entry: row a if moving +x else a+1; exit: the opposite row
        bool lower = (entry == xpos);
        T hA = lower ? h00 : h10, hB = lower ? h01 : h11;
        return z - dfma(w, hB - hA, hA);
    }
    if (kind == kYEdge) {
        bool lower = (entry == ypos);
        T hA = lower ? h00 : h01, hB = lower ? h10 : h11;
        return z - dfma(s, hB - hA, hA);
    }
    T hl = dfma(s, h10 - h00, h00), hh = dfma(s, h11 - h01, h01);
    return z - dfma(w, hh - hl, hl);
}

// March one ray.  surf_free points to the chain's free surfaces in LDS
// ([S-1][R*C]); surf_top to the top surface (LDS or global).  lo/hi are the
// per-surface bands (min - margin, max + margin) of this chain.
template <typename T, int S>
__device__ __forceinline__ T march_ray(const MarchParams<T> &P, const T *surf_free, const T *surf_top,
                                       const T *lo, const T *hi, T qx, T qy, T qz, T dx, T dy, T dz,
                                       T (&L)[S]) {
    const T INF = dev_inf<T>();
    const int R = P.R, C = P.C;
    const T idx = dx != T(0) ? T(1) / dx : T(0);
    const T idy = dy != T(0) ? T(1) / dy : T(0);
    const T idz = T(1) / dz;
    const bool xpos = dx > T(0), ypos = dy > T(0);
    // box exit
    T Texit = (P.ztop - qz) * idz;
    if (dx > T(0)) Texit = dmin(Texit, (P.xmax - qx) * idx);
    if (dx < T(0)) Texit = dmin(Texit, (T(0) - qx) * idx);
    if (dy > T(0)) Texit = dmin(Texit, (P.ymax - qy) * idy);
    if (dy < T(0)) Texit = dmin(Texit, (T(0) - qy) * idy);
    Texit = dmax(Texit, T(0));
    // the window of z where some surface may be crossed
    T zlo = lo[0], zhi = hi[0];
#pragma unroll
    for (int l = 1; l < S; ++l) {
        zlo = dmin(zlo, lo[l]);
        zhi = dmax(zhi, hi[l]);
    }
    const T t_start = dmax((zlo - qz) * idz, T(0));
    const T t_stop = dmin((zhi - qz) * idz, Texit);
#pragma unroll
    for (int l = 0; l < S; ++l) L[l] = dmin(t_start, Texit);
    if (t_start < t_stop) {
        const T x0 = dfma(t_start, dx, qx), y0 = dfma(t_start, dy, qy);
        int a = (int)floor(x0 * P.ihx), b = (int)floor(y0 * P.ihy);
        a = a < 0 ? 0 : (a > R - 2 ? R - 2 : a);
        b = b < 0 ? 0 : (b > C - 2 ? C - 2 : b);
        const int sxs = xpos ? 1 : -1, sys = ypos ? 1 : -1;
        T t0 = t_start;
        int ekind = kPoint;
        for (int it = 0; it < R + C; ++it) {
            T tnx = xpos ? (T(a + 1) * P.hx - qx) * idx : (dx < T(0) ? (T(a) * P.hx - qx) * idx : INF);
            T tny = ypos ? (T(b + 1) * P.hy - qy) * idy : (dy < T(0) ? (T(b) * P.hy - qy) * idy : INF);
            const bool stepx = tnx <= tny;
            const T tn = stepx ? tnx : tny;
            const int na = a + (stepx ? sxs : 0), nb = b + (stepx ? 0 : sys);
            const bool last = !(tn < t_stop) || na < 0 || na > R - 2 || nb < 0 || nb > C - 2;
            const T t1 = dmax(dmin(tn, t_stop), t0);
            const int xkind = last ? kPoint : (stepx ? kXEdge : kYEdge);
            const T tau1 = t1 - t0;
            if (tau1 > T(0)) {
                const T z0 = dfma(t0, dz, qz), z1 = dfma(t1, dz, qz);
                const T se = dfma(dfma(t0, dx, qx), P.ihx, -T(a)), we = dfma(dfma(t0, dy, qy), P.ihy, -T(b));
                const T sx = dfma(dfma(t1, dx, qx), P.ihx, -T(a)), wx = dfma(dfma(t1, dy, qy), P.ihy, -T(b));
                const T ds = dx * P.ihx, dw = dy * P.ihy;
                const int base = a * C + b;
#pragma unroll
                for (int l = 0; l < S; ++l) {
                    const T *Hl = (l < S - 1) ? surf_free + l * (R * C) : surf_top;
                    const T h00 = Hl[base], h01 = Hl[base + 1], h10 = Hl[base + C], h11 = Hl[base + C + 1];
                    const T hmin = dmin(dmin(h00, h10), dmin(h01, h11));
                    const T hmax = dmax(dmax(h00, h10), dmax(h01, h11));
                    T len;
                    if (z1 < hmin - P.margin) {
                        len = tau1;
                    } else if (z0 > hmax + P.margin) {
                        len = T(0);
                    } else {
                        const T fe = boundary_value(ekind, true, xpos, ypos, z0, se, we, h00, h10, h01, h11);
                        const T fx = boundary_value(xkind, false, xpos, ypos, z1, sx, wx, h00, h10, h01, h11);
                        const T c2 = -(h11 - h10 - h01 + h00) * ds * dw;
                        len = cell_below_length(fe, fx, c2, tau1);
                    }
                    L[l] += len;
                }
            }
            if (last) break;
            a = na;
            b = nb;
            t0 = t1;
            ekind = stepx ? kXEdge : kYEdge;
        }
    }
    T O = T(0);
#pragma unroll
    for (int l = 0; l < S; ++l) O += P.rho_diff[l] * L[l];
    return O;
}

// One block = one chain x one tile of rays.  Stages the chain's surfaces in
// LDS, marches its rays, adds the float64 Poisson terms
//   -C_p O_p / Lambda - E_p exp(-O_p / Lambda)
// (the ray-independent part C_p log E_p - log C_p! is added on the host side)
// and writes one fixed-order partial sum per block.
template <typename T, int S, bool TOP_LDS, int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_march_lik(MarchParams<T> P) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *sh = reinterpret_cast<T *>(smem_raw);
    __shared__ double red[16];
    __shared__ T band[2 * kMaxSurfaces];
    const int chain = blockIdx.y, tile = blockIdx.x, tid = threadIdx.x;
    if (P.only_nan && !(P.only_nan[chain] != P.only_nan[chain])) return;
    const int N = P.R * P.C;
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
    mn[S - 1] = P.top_min;
    mx[S - 1] = P.top_max;
    // block-reduce the free-surface ranges
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
    const T *top_ptr = TOP_LDS ? sh + (S - 1) * N : P.top;
    double acc = 0.0;
    const int r0 = tile * P.rays_per_block;
    const int r1 = min(r0 + P.rays_per_block, P.n_ray);
    for (int ray = r0 + tid; ray < r1; ray += BLOCK) {
        const int s = ray / P.n_pix;
        T L[S];
        T O = march_ray<T, S>(P, sh, top_ptr, lo, hi, P.sensor[3 * s], P.sensor[3 * s + 1], P.sensor[3 * s + 2],
                              P.dx[ray], P.dy[ray], P.dz[ray], L);
        if (P.opacity) P.opacity[(size_t)chain * P.n_ray + ray] = O;
        const double Od = (double)O;
        acc += -P.c_over_L[ray] * Od - P.expo[ray] * exp(-Od * P.inv_L);
    }
    double tot = block_sum<BLOCK>(acc, red);
    if (tid == 0) P.partials[(size_t)chain * P.n_tiles + tile] = tot;
}

}  // namespace mc
