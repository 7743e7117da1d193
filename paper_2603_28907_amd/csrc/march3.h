// march3.h -- surface-major band walks (any precision; the float64 march).
//
// Exact below-lengths L_l of every surface (paper Sec. 2.1.1 opacity of the
// layered density).  Each thread marches its ray through one surface at a
// time:
//
//   for each surface l:
//     [t_lo, t_hi] = the t-range where z(t) lies in the band of surface l
//                    (chain-wide node min/max widened by a rounding margin);
//     L_l = t_lo (the ray is certainly below surface l before its band);
//     walk the cells of [t_lo, t_hi] and add each cell's exact below-length.
//
// The band window in t depends only on the sensor height and the ray's
// vertical direction, and a wavefront holds 64 pixels of one zenith ring of
// one sensor, so the 64 lanes walk the same t-window in near lockstep: the
// loop body is short, trip counts are close, and the occasional crossing
// solve runs inline.  Per-ray constants (reciprocal directions, box exit,
// the DDA offsets) are precomputed on the host, chain independent.
//
// Crossing decisions use the boundary formulas of march_common.h: the end
// values of a cell piece come from the lerp along the shared cell edge, so
// adjacent cells see identical bits and a crossing is never dropped or double
// counted.
#pragma once

#include "march_common.h"

namespace mc {

// Per-ray constants (host precomputed, chain independent), SoA [n_ray].
template <typename T>
struct RayConsts {
    const T *idx, *idy, *idz;   // 1/d (0 where d = 0)
    const T *ox, *oy;           // -q_x/d_x, -q_y/d_y (+inf where d = 0)
    const T *texit;             // box exit parameter
};

__device__ __forceinline__ float fast_rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double fast_rcp(double x) { return 1.0 / x; }

// Below-length of one cell piece [0, tau1] given the end values fe, fx of
// f = z - h and the curvature c2 of f along the ray: one crossing when the
// end signs differ (stable quadratic root), two around an interior vertex of
// the opposite sign, else none.  Reciprocal-based arithmetic (float: the
// hardware reciprocal, 1 ulp; double: exact division).
template <typename T>
__device__ __forceinline__ T cell_below_length_fast(T fe, T fx, T c2, T tau1) {
    const bool be = fe < T(0), bx = fx < T(0);
    const T c1 = (fx - fe) * fast_rcp(tau1) - c2 * tau1;
    if (be != bx) {
        T disc = dmax(c1 * c1 - T(4) * c2 * fe, T(0));
        T sq = dsqrt(disc);
        T q = T(-0.5) * (c1 + (c1 >= T(0) ? sq : -sq));
        T r1 = q * fast_rcp(c2), r2 = fe * fast_rcp(q);
        T d1 = dmax(dmax(-r1, r1 - tau1), T(0));
        T d2 = dmax(dmax(-r2, r2 - tau1), T(0));
        bool use1 = (d1 < d2) || (d2 != d2);
        T r = use1 ? r1 : r2;
        if (r != r) r = tau1 * fe * fast_rcp(fe - fx);
        r = dmin(dmax(r, T(0)), tau1);
        return be ? r : tau1 - r;
    }
    if (c2 != T(0)) {
        const T ic2 = fast_rcp(c2);
        const T tv = T(-0.5) * c1 * ic2;
        if (tv > T(0) && tv < tau1) {
            const T fv = fe + tv * (c1 + c2 * tv);
            if ((fv < T(0)) != be) {
                T disc = dmax(c1 * c1 - T(4) * c2 * fe, T(0));
                T half = T(0.5) * dsqrt(disc) * dabs(ic2);
                T ta = dmax(tv - half, T(0)), tb = dmin(tv + half, tau1);
                T inner = dmax(tb - ta, T(0));
                return be ? tau1 - inner : inner;
            }
        }
    }
    return be ? tau1 : T(0);
}

// Below-length of surface Hl along one ray inside [tl, th] (a band window:
// certainly below at tl, certainly above at th unless th is the box exit).
template <typename T>
__device__ __forceinline__ T walk_surface(const MarchParams<T> &P, const T *Hl, T qx, T qy, T qz, T dx, T dy,
                                          T dz, T idx, T idy, T ox, T oy, T tl, T th) {
    const int R = P.R, C = P.C;
    const bool xpos = dx > T(0), ypos = dy > T(0);
    T len = T(0);
    // cell of the window start
    const T x0 = dfma(tl, dx, qx), y0 = dfma(tl, dy, qy);
    int a = (int)floor(x0 * P.ihx), b = (int)floor(y0 * P.ihy);
    a = a < 0 ? 0 : (a > R - 2 ? R - 2 : a);
    b = b < 0 ? 0 : (b > C - 2 ? C - 2 : b);
    const int sxs = xpos ? 1 : -1, sys = ypos ? 1 : -1;
    // coordinate of the next x (y) node line the ray meets
    T xn = T(xpos ? a + 1 : a) * P.hx, yn = T(ypos ? b + 1 : b) * P.hy;
    const T dxn = xpos ? P.hx : -P.hx, dyn = ypos ? P.hy : -P.hy;
    const T ds = dx * P.ihx, dw = dy * P.ihy;
    T t0 = tl, z0 = dfma(tl, dz, qz);
    int ekind = kPoint;
    for (int it = 0; it < R + C; ++it) {
        const T tnx = dfma(xn, idx, ox), tny = dfma(yn, idy, oy);
        const bool stepx = tnx <= tny;
        const T tn = stepx ? tnx : tny;
        const int na = stepx ? a + sxs : a, nb = stepx ? b : b + sys;
        const bool in_range = (unsigned)na <= (unsigned)(R - 2) && (unsigned)nb <= (unsigned)(C - 2);
        const bool edge = (tn < th) && in_range;
        const T t1 = dmax(dmin(tn, th), t0);
        const T z1 = dfma(t1, dz, qz);
        const int base = a * C + b;
        const T h00 = Hl[base], h01 = Hl[base + 1], h10 = Hl[base + C], h11 = Hl[base + C + 1];
        const T hmin = dmin(dmin(h00, h01), dmin(h10, h11));
        const T hmax = dmax(dmax(h00, h01), dmax(h10, h11));
        if (z1 < hmin - P.margin) {
            len += t1 - t0;
        } else if (!(z0 > hmax + P.margin) && t1 > t0) {
            const int xkind = edge ? (stepx ? kXEdge : kYEdge) : kPoint;
            const T se = dfma(dfma(t0, dx, qx), P.ihx, -T(a)), we = dfma(dfma(t0, dy, qy), P.ihy, -T(b));
            const T sx = dfma(dfma(t1, dx, qx), P.ihx, -T(a)), wx = dfma(dfma(t1, dy, qy), P.ihy, -T(b));
            const T fe = boundary_value(ekind, true, xpos, ypos, z0, se, we, h00, h10, h01, h11);
            const T fx = boundary_value(xkind, false, xpos, ypos, z1, sx, wx, h00, h10, h01, h11);
            const T c2 = -(h11 - h10 - h01 + h00) * ds * dw;
            len += cell_below_length_fast(fe, fx, c2, t1 - t0);
        }
        if (!edge) break;
        if (stepx) {
            a = na;
            xn += dxn;
            ekind = kXEdge;
        } else {
            b = nb;
            yn += dyn;
            ekind = kYEdge;
        }
        t0 = t1;
        z0 = z1;
    }
    return len;
}

// Body of one block: chain `chain`, ray tile `tile`; sh = the block's LDS.
template <typename T, int S, bool TOP_LDS, int BLOCK>
__device__ __forceinline__ void march_block3(const MarchParams<T> &P, const RayConsts<T> &K, int chain, int tile,
                                             T *sh) {
    __shared__ double red[16];
    __shared__ T band[2 * kMaxSurfaces];
    const int tid = threadIdx.x;
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
    double acc = 0.0;
    const int r0 = tile * P.rays_per_block;
    const int r1 = min(r0 + P.rays_per_block, P.n_ray);
    for (int ray = r0 + tid; ray < r1; ray += BLOCK) {
        const int s = ray / P.n_pix;
        const T qx = P.sensor[3 * s], qy = P.sensor[3 * s + 1], qz = P.sensor[3 * s + 2];
        const T dx = P.dx[ray], dy = P.dy[ray], dz = P.dz[ray];
        const T idx = K.idx[ray], idy = K.idy[ray], idz = K.idz[ray];
        const T ox = K.ox[ray], oy = K.oy[ray], Texit = K.texit[ray];
        T O = T(0);
#pragma unroll
        for (int l = 0; l < S; ++l) {
            const T *Hl = (l < S - 1 || TOP_LDS) ? sh + l * N : P.top;
            const T tl = dmin(dmax((band[l] - qz) * idz, T(0)), Texit);
            const T th = dmin(dmax((band[kMaxSurfaces + l] - qz) * idz, T(0)), Texit);
            T L = tl;
            if (tl < th) L += walk_surface<T>(P, Hl, qx, qy, qz, dx, dy, dz, idx, idy, ox, oy, tl, th);
            O += P.rho_diff[l] * L;
        }
        if (P.opacity) P.opacity[(size_t)chain * P.n_ray + ray] = O;
        const double Od = (double)O;
        acc += -P.c_over_L[ray] * Od - P.expo[ray] * exp(-Od * P.inv_L);
    }
    const double tot = block_sum<BLOCK>(acc, red);
    if (tid == 0) P.partials[(size_t)chain * P.n_tiles + tile] = tot;
}

template <typename T, int S, bool TOP_LDS, int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_march_lik3(MarchParams<T> P, RayConsts<T> K) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    int chain, tile;
    if (!xcd_chain_tile(P.n_tiles, P.n_chains, chain, tile)) return;
    march_block3<T, S, TOP_LDS, BLOCK>(P, K, chain, tile, reinterpret_cast<T *>(smem_raw));
}

}  // namespace mc
