// adjoint.h -- gradient of the log posterior with respect to every surface
// height, and the MALA step that consumes it.
//
// Likelihood part.  L_l (the below-length of surface l along a ray) moves
// with each crossing t_c of surface l: with f = z - h, a node n of the
// crossing's patch changes the crossing by dt_c/dH_n = w_n(t_c) / f'(t_c),
// so dL_l/dH_n = sum over crossings of w_n / |f'(t_c)| (an entry into the
// region below adds, an exit adds too: both widen it).  With
// dO/dL_l = rho_l - rho_{l+1} and dLL/dO_p = (lambda_p - C_p)/Lambda, every
// crossing scatters (rho_l - rho_{l+1}) g_p w_n / |f'| into four nodes.
//
// The adjoint kernel re-walks each ray exactly as the forward walk does
// (same band windows, same boundary values, same crossing decisions), finds
// the crossing positions of the in-cell quadratic and adds their weighted
// contributions into a per-chain 64-bit fixed-point accumulator (2^-32 per
// unit) with global integer atomics, so gradients are bitwise reproducible.
//
// Prior part (paper Sec. 2.2.1, written in H-space): with
//   G_i = d log p / d w_i = -s^2 (4(1-r) w_i + r (4 w_i - sum_{j~i} w_j)) + w_i,
// dw/du = 1/phi(w), u = (H - a)/d, v = (b - H)/d, d = b - a:
//   d/dH_l = G/(phi d),  d/da = -G v/(phi d) + 1/d,  d/db = -G u/(phi d) - 1/d.
#pragma once

#include "march3.h"
#include "march5.h"
#include "prior.h"

namespace mc {

constexpr double kGradFix = 4294967296.0;   // 2^32 fixed-point units per gradient unit
constexpr double kGradFixInv = 1.0 / 4294967296.0;

// Crossings of the piece quadratic p(tau) = fe + c1 tau + c2 tau^2 with
// p(tau1) = fx (the same case analysis as cell_below_length).  Returns the
// number of crossings (0..2), their positions and |p'| there.
template <typename T>
__device__ __forceinline__ int cell_crossings(T fe, T fx, T c2, T tau1, T *tc, T *fp) {
    const bool be = fe < T(0), bx = fx < T(0);
    const T c1 = (fx - fe) / tau1 - c2 * tau1;
    if (be != bx) {
        T disc = dmax(c1 * c1 - T(4) * c2 * fe, T(0));
        T sq = dsqrt(disc);
        T q = T(-0.5) * (c1 + (c1 >= T(0) ? sq : -sq));
        T r1 = q / c2, r2 = fe / q;
        T d1 = dmax(dmax(-r1, r1 - tau1), T(0));
        T d2 = dmax(dmax(-r2, r2 - tau1), T(0));
        bool use1 = (d1 < d2) || (d2 != d2);
        T r = use1 ? r1 : r2;
        if (r != r) r = tau1 * fe / (fe - fx);
        r = dmin(dmax(r, T(0)), tau1);
        tc[0] = r;
        fp[0] = dabs(c1 + T(2) * c2 * r);
        return 1;
    }
    if (c2 != T(0)) {
        const T tv = -c1 / (T(2) * c2);
        if (tv > T(0) && tv < tau1) {
            const T fv = fe + tv * (c1 + c2 * tv);
            if ((fv < T(0)) != be) {
                T disc = dmax(c1 * c1 - T(4) * c2 * fe, T(0));
                T half = dsqrt(disc) / (T(2) * dabs(c2));
                T ta = dmax(tv - half, T(0)), tb = dmin(tv + half, tau1);
                tc[0] = ta;
                tc[1] = tb;
                fp[0] = dabs(c1 + T(2) * c2 * ta);
                fp[1] = dabs(c1 + T(2) * c2 * tb);
                return 2;
            }
        }
    }
    return 0;
}

__device__ __forceinline__ void add_fixed(unsigned long long *p, double v) {
    const double sv = v * kGradFix;
    // saturate far outside any physical gradient instead of wrapping
    const double cl = fmin(fmax(sv, -9.0e18), 9.0e18);
    atomicAdd(p, (unsigned long long)(long long)__builtin_rint(cl));
}

// Re-walk one surface of one ray and scatter scale * w_n / |f'| per crossing.
template <typename T>
__device__ __forceinline__ void walk_surface_adjoint(const MarchParams<T> &P, const T *Hl, T qx, T qy, T qz, T dx,
                                                     T dy, T dz, T idx, T idy, T ox, T oy, T tl, T th, double scale,
                                                     unsigned long long *G) {
    const int R = P.R, C = P.C;
    const bool xpos = dx > T(0), ypos = dy > T(0);
    const T x0 = dfma(tl, dx, qx), y0 = dfma(tl, dy, qy);
    int a = (int)floor(x0 * P.ihx), b = (int)floor(y0 * P.ihy);
    a = a < 0 ? 0 : (a > R - 2 ? R - 2 : a);
    b = b < 0 ? 0 : (b > C - 2 ? C - 2 : b);
    const int sxs = xpos ? 1 : -1, sys = ypos ? 1 : -1;
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
        if (!(z1 < hmin - P.margin) && !(z0 > hmax + P.margin) && t1 > t0) {
            const int xkind = edge ? (stepx ? kXEdge : kYEdge) : kPoint;
            const T se = dfma(dfma(t0, dx, qx), P.ihx, -T(a)), we = dfma(dfma(t0, dy, qy), P.ihy, -T(b));
            const T sx = dfma(dfma(t1, dx, qx), P.ihx, -T(a)), wx = dfma(dfma(t1, dy, qy), P.ihy, -T(b));
            const T fe = boundary_value(ekind, true, xpos, ypos, z0, se, we, h00, h10, h01, h11);
            const T fx = boundary_value(xkind, false, xpos, ypos, z1, sx, wx, h00, h10, h01, h11);
            const T c2 = -(h11 - h10 - h01 + h00) * ds * dw;
            T tc[2], fp[2];
            const int nc = cell_crossings(fe, fx, c2, t1 - t0, tc, fp);
            for (int k = 0; k < nc; ++k) {
                if (!(fp[k] > T(0))) continue;   // tangency: a kink of lp, no derivative
                const T t = t0 + tc[k];
                // a crossing on the box lid z = max H_S is the kink of that max
                // (the ray leaves the box there); it carries no derivative
                if (dfma(t, dz, qz) >= P.lid) continue;
                const T s = dmin(dmax(dfma(dfma(t, dx, qx), P.ihx, -T(a)), T(0)), T(1));
                const T w = dmin(dmax(dfma(dfma(t, dy, qy), P.ihy, -T(b)), T(0)), T(1));
                const double g = scale / (double)fp[k];
                const double ws = (double)s, ww = (double)w;
                add_fixed(G + base, g * (1.0 - ws) * (1.0 - ww));
                add_fixed(G + base + C, g * ws * (1.0 - ww));
                add_fixed(G + base + 1, g * (1.0 - ws) * ww);
                add_fixed(G + base + C + 1, g * ws * ww);
            }
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
}

// One block = one chain x one tile of rays (XCD-aware 1-D grid, as the
// forward march); g_p from the forward opacities, or given (gpbuf).
// gfix: [n_chains][S][R*C] fixed-point accumulators (zeroed beforehand).
template <typename T, int S, bool TOP_LDS, int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_adjoint(MarchParams<T> P, RayConsts<T> K, const T *opacity,
                                                   unsigned long long *gfix, const T *gpbuf) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *sh = reinterpret_cast<T *>(smem_raw);
    __shared__ T band[2 * kMaxSurfaces];
    const int tid = threadIdx.x;
    int chain, tile;
    if (!xcd_chain_tile(P.n_tiles, P.n_chains, chain, tile)) return;
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
    unsigned long long *Gc = gfix + (size_t)chain * S * N;
    const int r0 = tile * P.rays_per_block;
    const int r1 = min(r0 + P.rays_per_block, P.n_ray);
    for (int ray = r0 + tid; ray < r1; ray += BLOCK) {
        const int s = ray / P.n_pix;
        double gp;
        if (gpbuf) {   // dLL/dO given (solid-angle pixels)
            gp = (double)gpbuf[(size_t)chain * P.n_ray + ray];
        } else {
            const double Od = (double)opacity[(size_t)chain * P.n_ray + ray];
            gp = P.expo[ray] * exp(-Od * P.inv_L) * P.inv_L - P.c_over_L[ray];   // dLL/dO = (lambda - C)/Lambda
        }
        const T qx = P.sensor[3 * s], qy = P.sensor[3 * s + 1], qz = P.sensor[3 * s + 2];
        const T dx = P.dx[ray], dy = P.dy[ray], dz = P.dz[ray];
        const T idx = K.idx[ray], idy = K.idy[ray], idz = K.idz[ray];
        const T ox = K.ox[ray], oy = K.oy[ray], Texit = K.texit[ray];
#pragma unroll
        for (int l = 0; l < S; ++l) {
            const T *Hl = (l < S - 1 || TOP_LDS) ? sh + l * N : P.top;
            const T tl = dmin(dmax((band[l] - qz) * idz, T(0)), Texit);
            const T th = dmin(dmax((band[kMaxSurfaces + l] - qz) * idz, T(0)), Texit);
            const double scale = gp * (double)P.rho_diff[l];
            if (tl < th && scale != 0.0)
                walk_surface_adjoint<T>(P, Hl, qx, qy, qz, dx, dy, dz, idx, idy, ox, oy, tl, th, scale, Gc + l * N);
        }
    }
}

// ---------------------------------------------------------------------------
// float32 adjoint on the lean walk of k_march_lik4
// ---------------------------------------------------------------------------

// float32 adjoint by re-walking the rays (the chains whose crossing records
// overflowed), per-node sums formed in LDS.  One block = one (chain, surface
// l, window of node rows): it stages surface l, zeroes 64-bit fixed-point
// accumulators for the window's nodes, walks every ray of the chain through
// surface l (the walk and classification of k_march_lik4, started at the
// band window or, with several windows, at the first cell whose node rows can
// meet the window: the walk's cell indices are integers, so either start
// reproduces the forward walk's bits), adds each crossing's four node
// contributions that fall in the window with LDS integer atomics, and stores
// the window into the chain's gradient (the block owns those nodes; the
// record adjoint wrote zeros there for this chain).  Integer sums are
// order-independent, so the result is bitwise reproducible and equals the
// record adjoint's.  Blocks of chains whose records are complete
// (ovf[chain] == 0) exit at once: the grid has no per-tile blocks, so the
// launch costs little when no chain overflowed.
struct AdjointLdsShape {
    int n_windows, window_rows;
};

template <int S, int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_adjoint_lds(MarchParams<float> P, RayConsts<float> K, const float *gpbuf,
                                                       const int *ovf, unsigned long long *gfix, AdjointLdsShape W_) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ float band[2];
    __shared__ float wred[2][BLOCK / kWave];
    const int tid = threadIdx.x;
    int chain, sub;
    if (!xcd_chain_tile(S * W_.n_windows, P.n_chains, chain, sub)) return;
    if (!ovf[chain]) return;
    const int l = sub / W_.n_windows, win = sub - l * W_.n_windows;
    const int N = P.R * P.C, C = P.C;
    const int row0 = win * W_.window_rows;
    const int rows = min(W_.window_rows, P.R - row0);
    float *Hl = reinterpret_cast<float *>(smem_raw);
    unsigned long long *acc =
        reinterpret_cast<unsigned long long *>(smem_raw + (((size_t)N * sizeof(float) + 15) & ~(size_t)15));
    // stage surface l and its band
    const float *src = l < S - 1 ? P.heights + ((size_t)chain * (S - 1) + l) * N : P.top;
    float mn = __builtin_huge_valf(), mx = -__builtin_huge_valf();
    for (int i = tid; i < N; i += BLOCK) {
        const float v = src[i];
        Hl[i] = v;
        mn = fminf(mn, v);
        mx = fmaxf(mx, v);
    }
    for (int i = tid; i < rows * C; i += BLOCK) acc[i] = 0ull;
    {
        const float a = wave_min(mn), b = wave_max(mx);
        if (tid % kWave == 0) {
            wred[0][tid / kWave] = a;
            wred[1][tid / kWave] = b;
        }
        __syncthreads();
        if (tid == 0) {
            float a2 = wred[0][0], b2 = wred[1][0];
            for (int w = 1; w < BLOCK / kWave; ++w) {
                a2 = fminf(a2, wred[0][w]);
                b2 = fmaxf(b2, wred[1][w]);
            }
            band[0] = (l < S - 1 ? a2 : P.top_min) - P.margin;
            band[1] = (l < S - 1 ? b2 : P.top_max) + P.margin;
        }
        __syncthreads();
    }
    const float rho = P.rho_diff[l];
    const int lo = row0 * C, hi = (row0 + rows) * C;   // node offsets of the window
    for (int ray = tid; ray < P.n_ray; ray += BLOCK) {
        const int sidx = ray / P.n_pix;
        const float scale = gpbuf[(size_t)chain * P.n_ray + ray] * rho;   // (lambda - C)/Lambda (rho_l - rho_l+1)
        const float qx = P.sensor[3 * sidx], qz = P.sensor[3 * sidx + 2];
        const float dx = P.dx[ray], dz = P.dz[ray];
        // the ray in cell units, as in the march
        const float qxi = qx * P.ihx, qyi = P.sensor[3 * sidx + 1] * P.ihy;
        const float dxi = dx * P.ihx, dyi = P.dy[ray] * P.ihy;
        const float idx = K.idx[ray], idy = K.idy[ray], idz = K.idz[ray];
        const float ox = K.ox[ray], oy = K.oy[ray], Texit = K.texit[ray];
        const float kxy = -dxi * dyi;   // the march's curvature factor
        float tl = fminf(fmaxf((band[0] - qz) * idz, 0.f), Texit);
        float th = fminf(fmaxf((band[1] - qz) * idz, 0.f), Texit);
        if (W_.n_windows > 1) {
            // only cells whose node rows meet the window can add to it: cell
            // rows row0-1 .. row0+rows-1, i.e. x in [(row0-1) hx, (row0+rows) hx];
            // one more cell on each side absorbs rounding of the clip
            const float xa = (float)(row0 - 2) * P.hx, xb = (float)(row0 + rows + 1) * P.hx;
            if (dx != 0.f) {
                const float ta = __builtin_fmaf(xa, idx, ox), tb = __builtin_fmaf(xb, idx, ox);
                tl = fmaxf(tl, fminf(ta, tb));
                th = fminf(th, fmaxf(ta, tb));
            } else if (qx < xa || qx > xb) {
                continue;
            }
        }
        if (!(tl < th) || scale == 0.f) continue;
        Walk W = walk_init(P, qxi, qyi, qz, dxi, dyi, dz, idx, idy, ox, oy, tl, th);
        for (;;) {   // at most R + C - 4 steps, as in the march
            const Step st = walk_step(W, qz, dz);
            const int off = (int)(W.off >> 2);
            const float h00 = Hl[off], h01 = Hl[off + 1], h10 = Hl[off + C], h11 = Hl[off + C + 1];
            const float hmin = fminf(fminf(h00, h01), fminf(h10, h11));
            const float hmax = fmaxf(fmaxf(h00, h01), fmaxf(h10, h11));
            // the cell's node rows a, a+1 must meet the window
            if (off + C + 1 >= lo && off < hi && !(st.z1 < hmin - P.margin) && !(W.z0 > hmax + P.margin) &&
                st.t1 > W.t0) {
                const float t0 = W.t0, tau1 = st.t1 - W.t0;
                const float qxa = qxi - walk_af(W), qyb = qyi - walk_bf(W);
                PieceCross pc;
                (void)solve_cell_piece<true>(h00, h01, h10, h11, qxa, qyb, dxi, dyi, kxy, W.t0, st.t1, W.z0, st.z1,
                                             W.enx, W.eny, st.edge && st.stepx, st.edge && !st.stepx, &pc);
                const float *fp = pc.fp;
#pragma unroll
                for (int k = 0; k < 2; ++k) {   // at most two crossings; unrolled to keep them in registers
                    if (k >= pc.n) break;
                    if (!(fp[k] > 0.f)) continue;   // tangency: a kink of lp, no derivative
                    const float t = __builtin_fmaf(pc.s[k], tau1, t0);
                    if (__builtin_fmaf(t, dz, qz) >= P.lid) continue;   // the box lid: a kink
                    const float s = fminf(fmaxf(__builtin_fmaf(t, dxi, qxa), 0.f), 1.f);
                    const float w = fminf(fmaxf(__builtin_fmaf(t, dyi, qyb), 0.f), 1.f);
                    const float g = scale * __builtin_amdgcn_rcpf(fp[k]);
                    const float cv[4] = {g * (1.f - s) * (1.f - w), g * (1.f - s) * w, g * s * (1.f - w), g * s * w};
                    const int no[4] = {off, off + 1, off + C, off + C + 1};
#pragma unroll
                    for (int m = 0; m < 4; ++m) {
                        if (no[m] >= lo && no[m] < hi) {
                            const float sv = fminf(fmaxf(cv[m] * 4294967296.0f, -9.0e18f), 9.0e18f);
                            atomicAdd(acc + (no[m] - lo), (unsigned long long)(long long)__builtin_rintf(sv));
                        }
                    }
                }
            }
            if (!st.edge) break;
            walk_advance(W, st);
        }
    }
    __syncthreads();
    unsigned long long *G = gfix + ((size_t)chain * S + l) * N + lo;
    for (int i = tid; i < rows * C; i += BLOCK) G[i] = acc[i];
}

// float32 adjoint from the crossing records of the gradient march (no walk).
// One block = one (chain, surface l, window of node rows; one window while
// the surface's 64-bit accumulators fit the LDS): it zeroes the window's
// fixed-point accumulators in LDS, reads every record of (chain, l) over all
// ray tiles, adds the contributions (rho_l - rho_{l+1}) g_p w_n / |f'| of
// the nodes in the window with LDS integer atomics, and stores the window's
// sums into the chain's gradient: the block owns those nodes, so no global
// atomics and no zeroing beforehand.  A chain whose records overflowed gets
// zeros here and its gradient from k_adjoint_lds.  fwd_block: the block
// size of the gradient march (the width of a record row).
constexpr int kRecBatch = 8;   // records per thread in flight in the record adjoint

template <int S, int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_adjoint_rec(MarchParams<float> P, CrossRecs X, int fwd_block,
                                                       AdjointLdsShape W_, unsigned long long *gfix) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    unsigned long long *acc = reinterpret_cast<unsigned long long *>(smem_raw);
    int chain, sub;
    if (!xcd_chain_tile(S * W_.n_windows, P.n_chains, chain, sub)) return;
    const int l = sub / W_.n_windows, win = sub - l * W_.n_windows;
    const int N = P.R * P.C, C = P.C, tid = threadIdx.x;
    const int row0 = win * W_.window_rows;
    const int rows = min(W_.window_rows, P.R - row0);
    const int lo = row0 * C, hi = (row0 + rows) * C;   // node offsets of the window
    for (int i = tid; i < rows * C; i += BLOCK) acc[i] = 0ull;
    __syncthreads();
    if (!X.ovf[chain]) {
        const float rho = P.rho_diff[l];
        const float *gpc = X.gp + (size_t)chain * P.n_ray;
        for (int tile = 0; tile < P.n_tiles; ++tile) {
            const size_t cb = (size_t)(chain * P.n_tiles + tile) * S + l;
            const uint32_t *cnt = X.cnt + cb * fwd_block;
            const uint4 *rec = X.rec + cb * (size_t)X.slots * fwd_block;
            const int ray0 = tile * P.rays_per_block;
            for (int j = tid; j < fwd_block; j += BLOCK) {
                const int n = (int)cnt[j];
                // kRecBatch records at a time: their loads, then the dLL/dO
                // gathers they name, are all in flight before the first is used
                for (int k0 = 0; k0 < n; k0 += kRecBatch) {
                    uint4 r[kRecBatch];
                    float gv[kRecBatch];
#pragma unroll
                    for (int u = 0; u < kRecBatch; ++u)
                        if (k0 + u < n) r[u] = rec[(size_t)(k0 + u) * fwd_block + j];
#pragma unroll
                    for (int u = 0; u < kRecBatch; ++u)
                        if (k0 + u < n) gv[u] = gpc[ray0 + j + (int)((r[u].x >> 18) & 0x3Fu) * fwd_block];
#pragma unroll
                    for (int u = 0; u < kRecBatch; ++u) {
                        if (k0 + u >= n) break;
                        const int off = (int)(r[u].x & 0xFFFFu);
                        if (off + C + 1 < lo || off >= hi) continue;   // the cell's node rows miss the window
                        const float g = (gv[u] * rho) * __uint_as_float(r[u].w);
                        const float s = __uint_as_float(r[u].y), w = __uint_as_float(r[u].z);
                        const float cv[4] = {g * (1.f - s) * (1.f - w), g * (1.f - s) * w, g * s * (1.f - w),
                                             g * s * w};
                        const int no[4] = {off, off + 1, off + C, off + C + 1};
#pragma unroll
                        for (int m = 0; m < 4; ++m) {
                            if (no[m] >= lo && no[m] < hi) {
                                const float sv = fminf(fmaxf(cv[m] * 4294967296.0f, -9.0e18f), 9.0e18f);
                                atomicAdd(acc + (no[m] - lo), (unsigned long long)(long long)__builtin_rintf(sv));
                            }
                        }
                    }
                }
            }
        }
    }
    __syncthreads();
    unsigned long long *G = gfix + ((size_t)chain * S + l) * N + lo;
    for (int i = tid; i < rows * C; i += BLOCK) G[i] = acc[i];
}

__global__ void k_fill_i32(int *p, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

__global__ void k_fill_u64(unsigned long long *p, size_t n) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0ull;
}

// Log posterior and its gradient per chain (one block per chain): the log
// prior with its gradient, the fixed-order sum of the likelihood partials,
// and the likelihood gradient gfix ([n][S][N] in 2^-32 fixed point, or null
// without sensors) added in.  grad: [n][S][N], every entry written; rows of
// chains whose log posterior is -inf are zero.
//
// Node n of layer l gets its own prior term's derivative, then (one layer
// later) the derivative of layer l+1's term through that layer's lower
// bound; the top node gets every layer's term.  Each thread owns the same
// nodes in every layer and accumulates in grad itself, in a fixed order.
template <typename T, int S, int BLOCK>
__global__ __launch_bounds__(BLOCK, 4) void k_prior_grad(PriorParams<T> P, const unsigned long long *gfix,
                                                         T *grad) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    double *w = reinterpret_cast<double *>(smem_raw);   // [N]
    __shared__ double red[16];
    __shared__ int ired[16];
    __shared__ int zero_rows;
    const int c = blockIdx.x, tid = threadIdx.x;
    const int R = P.R, C = P.C, N = R * C;
    const T *H = P.heights + (size_t)c * (S - 1) * N;
    T *g = grad + (size_t)c * S * N;
    const unsigned long long *gf = gfix ? gfix + (size_t)c * S * N : nullptr;
    auto lik = [&](int k) -> double { return gf ? (double)(long long)gf[k] * kGradFixInv : 0.0; };
    double lp = 0.0;
    int ok = 1;
    // node (i, j) of n = tid + k BLOCK, stepped without a division per node
    const int bi = BLOCK / C, bj = BLOCK - bi * C;
    const int i0 = tid / C, j0 = tid - i0 * C;
    // loops kept rolled: the Phi^-1 call is out of line, and an unrolled body
    // keeps more values live across it (spilled around every call)
#pragma unroll 1
    for (int l = 0; l < S - 1; ++l) {
        double sw2 = 0.0, sld = 0.0;
#pragma unroll 1
        for (int n = tid; n < N; n += BLOCK) {
            const double h = (double)H[l * N + n];
            const double a = l ? (double)H[(l - 1) * N + n] : 0.0;
            const double b = P.top64[n];
            const double d = b - a, id = 1.0 / d;
            const double u = (h - a) * id, v = (b - h) * id;
            const bool good = (d > 0.0) && (u > 0.0) && (v > 0.0);
            ok &= good ? 1 : 0;
            const double wi = good ? probit_uv(u, v) : 0.0;
            w[n] = wi;
            sw2 += wi * wi;
            // log(b - a) of the first surface is log(top): summed once on the host
            if (l) sld += good ? log(d) : 0.0;
        }
        if (l == 0) sld = tid == 0 ? P.sum_log_top : 0.0;
        __syncthreads();
        double se = 0.0;
        const double r = P.r[l], s11 = P.s11[l];
        int i = i0, j = j0;
#pragma unroll 1
        for (int n = tid; n < N; n += BLOCK, i += bi, j += bj) {
            if (j >= C) {
                j -= C;
                ++i;
            }
            const double wi = w[n];
            const double wr = w[i * C + (j + 1 == C ? 0 : j + 1)], wl = w[i * C + (j == 0 ? C - 1 : j - 1)];
            const double wd = w[(i + 1 == R ? 0 : i + 1) * C + j], wu = w[(i == 0 ? R - 1 : i - 1) * C + j];
            se += (wi - wr) * (wi - wr) + (wi - wd) * (wi - wd);
            const double h = (double)H[l * N + n];
            const double a = l ? (double)H[(l - 1) * N + n] : 0.0;
            const double b = P.top64[n];
            const double d = b - a, id = 1.0 / d;
            const double u = (h - a) * id, v = (b - h) * id;
            double own = 0.0, below = 0.0, top = 0.0;
            if ((d > 0.0) && (u > 0.0) && (v > 0.0)) {
                const double G = -s11 * (4.0 * (1.0 - r) * wi + r * (4.0 * wi - (wr + wl + wd + wu))) + wi;
                // 1 / phi(w) = sqrt(2 pi) exp(w^2 / 2): a product instead of a
                // division; single precision suffices for a float32 gradient
                double iphi;
                if constexpr (sizeof(T) == 4)
                    iphi = (double)expf((float)(0.5 * wi * wi));
                else
                    iphi = exp(0.5 * wi * wi);
                own = G * iphi * 2.5066282746310002416 * id;   // dlp/du / d
                below = id - own * v;
                top = -own * u - id;
            }
            g[l * N + n] = (T)(lik(l * N + n) + own);
            if (l) g[(l - 1) * N + n] = (T)((double)g[(l - 1) * N + n] + below);
            const int kt = (S - 1) * N + n;
            g[kt] = (T)((l ? (double)g[kt] : lik(kt)) + top);
        }
        const double SW2 = block_sum<BLOCK>(sw2, red);
        const double SLD = block_sum<BLOCK>(sld, red);
        const double SE = block_sum<BLOCK>(se, red);
        lp += 0.5 * P.logdet[l] - 0.5 * s11 * (4.0 * (1.0 - r) * SW2 + r * SE) + 0.5 * N * log(s11) + 0.5 * SW2 - SLD;
    }
    ok = block_and<BLOCK>(ok, ired);
    if (tid == 0) {
        double ll = 0.0;
        if (P.has_lik) {
            const double *pp = P.partials + (size_t)c * P.n_tiles;
            for (int t = 0; t < P.n_tiles; ++t) ll += pp[t];
            ll += P.kconst;
        }
        const double v = ok ? lp + ll : -__builtin_huge_val();
        P.lp_out[c] = v;
        zero_rows = v == -__builtin_huge_val();
    }
    __syncthreads();
    if (zero_rows)
        for (int k = tid; k < S * N; k += BLOCK) g[k] = T(0);
}

// MALA proposal: prop = H + (eps^2/2) m g + eps sqrt(m) z, z from tag 2.
// g: [n][S][N] (free layers used), inv_mass: [S-1][N] float64 or null.
template <typename T>
__global__ void k_propose_mala(const T *H, const T *g, T *prop, const double *inv_mass, int M, int SN, double eps,
                               uint64_t seed, const uint64_t *step_base, int step_k) {
    const int c = blockIdx.y;
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (2 * j >= M) return;
    const uint64_t step = *step_base + (uint64_t)step_k;
    double z[2];
    rng_normal2(seed, (uint32_t)c, step, kTagMala, (uint32_t)j, z[0], z[1]);
#pragma unroll
    for (int e = 0; e < 2; ++e) {
        const int n = 2 * j + e;
        if (n >= M) break;
        const double m = inv_mass ? inv_mass[n] : 1.0;
        const size_t k = (size_t)c * M + n;
        const double mean = (double)H[k] + 0.5 * eps * eps * m * (double)g[(size_t)c * SN + n];
        prop[k] = (T)(mean + eps * sqrt(m) * z[e]);
    }
}

// MALA decision per chain (one block per chain):
//   log alpha = lp' - lp + log q(H | H') - log q(H' | H),
//   log q(y | x) = -sum (y - x - (eps^2/2) m g(x))^2 / (2 eps^2 m),
// on acceptance copy the proposal, its gradient and lp.
template <typename T, int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_mala_finalize(T *H, const T *prop, T *g_cur, const T *g_prop,
                                                         double *lp_cur, const double *lp_prop, int64_t *n_acc,
                                                         const double *inv_mass, int M, int SN, double eps,
                                                         uint64_t seed, const uint64_t *step_base, int step_k) {
    __shared__ double red[16];
    __shared__ int s_acc;
    const int c = blockIdx.x, tid = threadIdx.x;
    const T *Hc = H + (size_t)c * M;
    const T *Pc = prop + (size_t)c * M;
    const T *gc = g_cur + (size_t)c * SN;
    const T *gq = g_prop + (size_t)c * SN;
    double fwd = 0.0, bwd = 0.0;
    const double e2 = eps * eps, k1 = 0.5 / e2;
    for (int n = tid; n < M; n += BLOCK) {
        const double m = inv_mass ? inv_mass[n] : 1.0;
        const double k = inv_mass ? k1 / m : k1;   // 1 / (2 eps^2 m)
        const double h = (double)Hc[n], q = (double)Pc[n];
        const double df = q - h - 0.5 * e2 * m * (double)gc[n];
        const double db = h - q - 0.5 * e2 * m * (double)gq[n];
        fwd -= df * df * k;
        bwd -= db * db * k;
    }
    const double F = block_sum<BLOCK>(fwd, red);
    const double B = block_sum<BLOCK>(bwd, red);
    if (tid == 0) {
        const double lpp = lp_prop[c];
        double la = -__builtin_huge_val();
        if (lpp > -__builtin_huge_val()) la = lpp - lp_cur[c] + B - F;
        const uint64_t step = *step_base + (uint64_t)step_k;
        const double u = rng_uniform(seed, (uint32_t)c, step, kTagAccept, 0);
        const int acc = log(u) < la;
        if (acc) {
            lp_cur[c] = lpp;
            n_acc[c] += 1;
        }
        s_acc = acc;
    }
    __syncthreads();
    if (s_acc) {
        T *Hw = H + (size_t)c * M;
        T *gw = g_cur + (size_t)c * SN;
        for (int n = tid; n < M; n += BLOCK) Hw[n] = Pc[n];
        for (int n = tid; n < SN; n += BLOCK) gw[n] = gq[n];
    }
}

}  // namespace mc
