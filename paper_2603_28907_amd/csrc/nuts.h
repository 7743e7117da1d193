// The paper's sampler (Sec. 3.1): NUTS (Hoffman & Gelman 2014) in its
// multinomial form with the generalised no-U-turn criterion (Betancourt
// 2017), dual-averaging step size and windowed diagonal mass adaptation,
// and nested R-hat over super-chains (Sec. 3.2).
//
// Chains run in lock step: at doubling d every chain still active grows a
// subtree of 2^d leaves on its own side, one leapfrog step (one batched
// log-posterior gradient) per leaf, and the host stops once no chain is
// active.  The bookkeeping of a leaf (energy, divergence, multinomial
// proposal, U-turn checks of the blocks it completes, merge into the tree) is
// one block per chain.  Random numbers: momentum normals (tag 5, pair i/2),
// the side of doubling d (tag 6, j = d), the leaf proposal draw (tag 7,
// j = leaf index in the trajectory), the subtree merge draw (tag 8, j = d).
#pragma once
#include <hip/hip_runtime.h>

#include "device_common.h"

namespace mc {

constexpr int kNutsBlock = 1024;   // one block per chain: 16 wavefronts keep the CU busy with few chains
constexpr int kNutsMaxDepth = 10;
enum NutsTag : uint32_t { kTagNutsMomentum = 5, kTagNutsDirection = 6, kTagNutsLeaf = 7, kTagNutsMerge = 8 };

struct NutsChain {
    int side, active, depth, n_leap, diverged, turned;
    uint32_t leaf;
    double H0, logW, logWs, sum_acc, lpS, lpP, eps;
    // dual averaging of log(step size)
    double log_eps, log_eps_bar, h_bar, mu;
    double da_t;
};

template <typename T>
struct NutsParams {
    int M, SN, n, L;                 // free values per chain, gradient stride, chains, levels (max_depth + 1)
    double max_dh, target;
    uint64_t seed, step;
    const double *inv_mass;          // [n][M] or null (identity)
    NutsChain *ch;                   // [n]
    T *x;                            // chain states [n][M]
    double *lp;                      // [n]
    T *gcur;                         // [n][SN] gradient of the states (free part first)
    T *xe[2];                        // ends [n][M]
    double *pe[2];
    T *ge[2];
    T *xw;                           // leapfrog positions, the gradient's input [n][M]
    const double *lpw;               // [n] log posterior at xw
    const T *gw;                     // [n][SN] gradient at xw
    T *xs, *gs, *xp, *gp;            // subtree and tree proposals [n][M]
    double *rho, *pnear;             // [n][M]
    double *R, *F, *sR, *sF, *sL;    // [L][n][M] block sums, first momenta, saved first halves
};

__device__ __forceinline__ double nuts_logaddexp(double a, double b) {
    if (a == -__builtin_huge_val()) return b;
    if (b == -__builtin_huge_val()) return a;
    const double m = a > b ? a : b;
    return m + log(exp(a - m) + exp(b - m));
}

template <typename T>
__device__ __forceinline__ double im_at(const NutsParams<T> &P, size_t c, int k) {
    return P.inv_mass ? P.inv_mass[c * P.M + k] : 1.0;
}

// Turning test of the merge of A (grown first: sum rA, far end aF, near end
// aN) and B (sum rB, near end bN, far end bF); all threads of the block call
// it and get the same answer.
template <typename T>
__device__ bool nuts_turning(const NutsParams<T> &P, size_t c, const double *rA, const double *aF, const double *aN,
                             const double *rB, const double *bN, const double *bF, double *red,
                             double *rAB = nullptr, double *fAB = nullptr, double *lAB = nullptr) {
    double d[6] = {0, 0, 0, 0, 0, 0};
    for (int k = threadIdx.x; k < P.M; k += kNutsBlock) {
        const size_t o = c * P.M + k;
        const double im = im_at(P, c, k);
        const double r1 = rA[o] + rB[o], r2 = rA[o] + bN[o], r3 = aN[o] + rB[o];
        if (rAB) {   // the merged block's momentum sum and first momentum (and last)
            rAB[o] = r1;
            fAB[o] = aF[o];
            if (lAB) lAB[o] = bF[o];
        }
        d[0] += aF[o] * im * r1;
        d[1] += bF[o] * im * r1;
        d[2] += aF[o] * im * r2;
        d[3] += bN[o] * im * r2;
        d[4] += aN[o] * im * r3;
        d[5] += bF[o] * im * r3;
    }
    bool ok = true;
#pragma unroll
    for (int q = 0; q < 6; ++q) ok = ok && block_sum<kNutsBlock>(d[q], red) > 0.0;
    return !ok;
}

// Start of a transition: momentum, energy, the tree as the current point,
// the side of the first doubling.  Chains outside the support do not move.
template <typename T>
__global__ __launch_bounds__(kNutsBlock) void k_nuts_begin(NutsParams<T> P) {
    __shared__ double red[16];
    const size_t c = blockIdx.x;
    NutsChain &h = P.ch[c];
    const size_t o = c * P.M;
    double kin = 0.0;
    for (int j = threadIdx.x; 2 * j < P.M; j += kNutsBlock) {
        double z0, z1;
        rng_normal2(P.seed, (uint32_t)c, P.step, kTagNutsMomentum, (uint32_t)j, z0, z1);
        const int k0 = 2 * j;
        const double m0 = im_at(P, c, k0), p0 = z0 / sqrt(m0);
        P.pe[0][o + k0] = p0;
        kin += m0 * p0 * p0;
        if (k0 + 1 < P.M) {
            const double m1 = im_at(P, c, k0 + 1), p1 = z1 / sqrt(m1);
            P.pe[0][o + k0 + 1] = p1;
            kin += m1 * p1 * p1;
        }
    }
    kin = block_sum<kNutsBlock>(kin, red);
    for (int k = threadIdx.x; k < P.M; k += kNutsBlock) {
        const T x = P.x[o + k], g = P.gcur[c * P.SN + k];
        const double p = P.pe[0][o + k];
        P.pe[1][o + k] = p;
        P.xe[0][o + k] = x;
        P.xe[1][o + k] = x;
        P.ge[0][o + k] = g;
        P.ge[1][o + k] = g;
        P.xp[o + k] = x;
        P.gp[o + k] = g;
        P.xw[o + k] = x;
        P.rho[o + k] = p;
    }
    const double ud = rng_uniform(P.seed, (uint32_t)c, P.step, kTagNutsDirection, 0);
    const int side = ud < 0.5 ? 0 : 1;
    for (int k = threadIdx.x; k < P.M; k += kNutsBlock) P.pnear[o + k] = P.pe[side][o + k];
    if (threadIdx.x == 0) {
        const double lp = P.lp[c];
        h.side = side;
        h.active = lp > -__builtin_huge_val() ? 1 : 0;
        h.depth = 0;
        h.n_leap = 0;
        h.diverged = 0;
        h.turned = 0;
        h.leaf = 0;
        h.H0 = -lp + 0.5 * kin;
        h.logW = 0.0;
        h.logWs = -__builtin_huge_val();
        h.sum_acc = 0.0;
        h.lpP = lp;
        h.lpS = lp;
    }
}

// First half of a leapfrog step of every active chain: momentum half step and
// position step on the chain's growing side; the new position also goes to
// xw, the batched gradient's input.  Grid: (ceil(M / 256), n).
template <typename T>
__global__ __launch_bounds__(256) void k_nuts_leap_pos(NutsParams<T> P) {
    const size_t c = blockIdx.y;
    const int k = blockIdx.x * 256 + threadIdx.x;
    const NutsChain &h = P.ch[c];
    if (!h.active || k >= P.M) return;
    const int s = h.side;
    const double v = s ? 1.0 : -1.0, e = h.eps;
    const size_t o = c * P.M + k;
    const double ph = P.pe[s][o] + 0.5 * v * e * (double)P.ge[s][o];
    P.pe[s][o] = ph;
    const T x = (T)((double)P.xe[s][o] + v * e * im_at(P, c, k) * ph);
    P.xe[s][o] = x;
    P.xw[o] = x;
}

// Second half of leaf i (0-based in the subtree) at doubling d: momentum half
// step, energy, divergence, multinomial proposal, block sums and U-turn
// checks, and at the last leaf the merge into the tree and the next side.
template <typename T>
__global__ __launch_bounds__(kNutsBlock) void k_nuts_leap_fin(NutsParams<T> P, int i, int d) {
    __shared__ double red[16];
    __shared__ int s_flag;
    const size_t c = blockIdx.x;
    NutsChain &h = P.ch[c];
    if (!h.active) return;   // uniform over the block
    const int s = h.side;
    const double v = s ? 1.0 : -1.0, e = h.eps;
    const size_t o = c * P.M;
    double kin = 0.0;
    for (int k = threadIdx.x; k < P.M; k += kNutsBlock) {
        const T g = P.gw[c * P.SN + k];
        const double p = P.pe[s][o + k] + 0.5 * v * e * (double)g;
        P.pe[s][o + k] = p;
        P.ge[s][o + k] = g;
        kin += im_at(P, c, k) * p * p;
    }
    kin = block_sum<kNutsBlock>(kin, red);
    if (threadIdx.x == 0) {
        const double lpl = P.lpw[c];
        const double dH = (-lpl + 0.5 * kin) - h.H0;
        h.n_leap += 1;
        int flag;   // 0: stop, 1: keep going without taking the leaf, 2: take the leaf
        if (!(dH <= P.max_dh)) {
            h.diverged = 1;
            if (dH == dH) h.sum_acc += fmin(1.0, exp(-dH));
            flag = 0;
        } else {
            const double lw = -dH;
            h.sum_acc += fmin(1.0, exp(lw));
            const double lws = nuts_logaddexp(h.logWs, lw);
            const double ul = rng_uniform(P.seed, (uint32_t)c, P.step, kTagNutsLeaf, h.leaf);
            h.leaf += 1;
            const bool take = i == 0 || log(ul) < lw - lws;
            h.logWs = lws;
            if (take) h.lpS = lpl;
            flag = take ? 2 : 1;
        }
        s_flag = flag;
    }
    __syncthreads();
    const int flag = s_flag;
    if (flag == 0) {
        if (threadIdx.x == 0) h.active = 0;
        return;
    }
    const T *xl = P.xe[s] + o;
    const double *pl = P.pe[s] + o;
    const bool save0 = d > 0 && ((i + 1) & 1);
    for (int k = threadIdx.x; k < P.M; k += kNutsBlock) {
        if (flag == 2) {
            P.xs[o + k] = xl[k];
            P.gs[o + k] = P.ge[s][o + k];
        }
        // the level-0 block is the leaf itself; as the first half of its
        // parent it goes straight to the saved halves
        if (save0) {
            P.sR[o + k] = pl[k];
            P.sF[o + k] = pl[k];
            P.sL[o + k] = pl[k];
        } else {
            P.R[o + k] = pl[k];
            P.F[o + k] = pl[k];
        }
    }
    __syncthreads();
    // blocks completed by this leaf, from level 1 up: the halves of each must
    // not turn, and the block's momentum sum is the sum of its halves' sums
    // (as in the recursive tree) and its first momentum its first half's.  A
    // block that is the first half of its parent is written to the saved
    // halves (sum, first and last momentum), a second half or the whole
    // subtree to R, F.
    bool turning = false;
    for (int j = 1; j <= d && !turning; ++j) {
        if (((i + 1) & ((1 << j) - 1)) != 0) break;
        const size_t a = (size_t)(j - 1) * P.n * P.M, b = (size_t)j * P.n * P.M;
        const bool save = j < d && (((i + 1) >> j) & 1);
        turning = nuts_turning(P, c, P.sR + a, P.sF + a, P.sL + a, P.R + a, P.F + a, P.pe[s], red,
                               (save ? P.sR : P.R) + b, (save ? P.sF : P.F) + b, save ? P.sL + b : nullptr);
    }
    if (turning) {
        if (threadIdx.x == 0) h.active = 0;
        return;
    }
    if (i != (1 << d) - 1) return;
    // the subtree is complete and valid: merge it into the tree
    __syncthreads();
    if (threadIdx.x == 0) {
        const double um = rng_uniform(P.seed, (uint32_t)c, P.step, kTagNutsMerge, (uint32_t)d);
        s_flag = log(um) < h.logWs - h.logW ? 1 : 0;
        if (s_flag) h.lpP = h.lpS;
        h.logW = nuts_logaddexp(h.logW, h.logWs);
    }
    __syncthreads();
    const size_t ad = (size_t)d * P.n * P.M;
    if (s_flag) {
        for (int k = threadIdx.x; k < P.M; k += kNutsBlock) {
            P.xp[o + k] = P.xs[o + k];
            P.gp[o + k] = P.gs[o + k];
        }
    }
    const bool turned = nuts_turning(P, c, P.rho, P.pe[1 - s], P.pnear, P.R + ad, P.F + ad, P.pe[s], red);
    for (int k = threadIdx.x; k < P.M; k += kNutsBlock) P.rho[o + k] += P.R[ad + o + k];
    const int depth = d + 1;
    const bool more = !turned && depth < P.L - 1;
    int ns = 0;
    if (more) {
        const double ud = rng_uniform(P.seed, (uint32_t)c, P.step, kTagNutsDirection, (uint32_t)depth);
        ns = ud < 0.5 ? 0 : 1;
        for (int k = threadIdx.x; k < P.M; k += kNutsBlock) P.pnear[o + k] = P.pe[ns][o + k];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        h.depth = depth;
        h.turned = turned ? 1 : 0;
        h.active = more ? 1 : 0;
        h.side = ns;
        h.logWs = -__builtin_huge_val();
    }
}

// End of a transition: the tree's proposal becomes the chain state, and the
// per-transition statistics are written.
template <typename T>
__global__ __launch_bounds__(kNutsBlock) void k_nuts_end(NutsParams<T> P, int32_t *depth_out, int32_t *nleap_out,
                                                          int32_t *div_out, double *acc_out, int64_t col,
                                                          int64_t stride) {
    const size_t c = blockIdx.x;
    const NutsChain &h = P.ch[c];
    const size_t o = c * P.M;
    for (int k = threadIdx.x; k < P.M; k += kNutsBlock) {
        P.x[o + k] = P.xp[o + k];
        P.gcur[c * P.SN + k] = P.gp[o + k];
    }
    if (threadIdx.x == 0) {
        P.lp[c] = h.lpP;
        const size_t q = c * (size_t)stride + (size_t)col;
        if (depth_out) depth_out[q] = h.depth;
        if (nleap_out) nleap_out[q] = h.n_leap;
        if (div_out) div_out[q] = h.diverged;
        if (acc_out) acc_out[q] = h.n_leap ? h.sum_acc / h.n_leap : 0.0;
    }
}

// Number of chains still building (one block).
__global__ void k_nuts_count_active(const NutsChain *ch, int n, int *out) {
    __shared__ int cnt;
    if (threadIdx.x == 0) cnt = 0;
    __syncthreads();
    int mine = 0;
    for (int c = threadIdx.x; c < n; c += blockDim.x) mine += ch[c].active;
    atomicAdd(&cnt, mine);
    __syncthreads();
    if (threadIdx.x == 0) *out = cnt;
}

// Step-size state of every chain at the start of a run: eps from the caller,
// dual averaging restarted there; while warming up the step used is always
// exp(log_eps).
__global__ void k_nuts_da_init(NutsChain *ch, const double *eps, int n, int warm) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n) return;
    NutsChain &h = ch[c];
    h.mu = log(10.0 * eps[c]);
    h.log_eps = log(eps[c]);
    h.log_eps_bar = 0.0;
    h.h_bar = 0.0;
    h.da_t = 0.0;
    h.eps = warm ? exp(h.log_eps) : eps[c];
}

// Warm-up bookkeeping after transition k: dual averaging of log(eps) toward
// the acceptance target (gamma 0.05, t0 10, kappa 0.75); in slow windows a
// Welford update of the per-coordinate mean and sum of squares (wn = draws
// so far in the window, this one included); at a window end the inverse mass
// (n/(n+5)) var + 1e-3 * 5/(n+5) and a restart of dual averaging; at the
// last warm-up transition eps = exp(log_eps_bar).  One block per chain.
template <typename T>
__global__ __launch_bounds__(kNutsBlock) void k_nuts_adapt(NutsParams<T> P, double *inv_mass, double *wm,
                                                            double *w2, int64_t wn, int in_slow, int window_end,
                                                            int last) {
    const size_t c = blockIdx.x;
    NutsChain &h = P.ch[c];
    const size_t o = c * P.M;
    if (in_slow) {
        for (int k = threadIdx.x; k < P.M; k += kNutsBlock) {
            const double x = (double)P.x[o + k];
            if (wn == 1) {
                wm[o + k] = x;
                w2[o + k] = 0.0;
            } else {
                const double dlt = x - wm[o + k];
                wm[o + k] += dlt / (double)wn;
                w2[o + k] += dlt * (x - wm[o + k]);
            }
            if (window_end) {
                const double nn = (double)wn;
                const double var = wn > 1 ? w2[o + k] / (nn - 1.0) : 0.0;
                inv_mass[o + k] = (nn / (nn + 5.0)) * var + 1e-3 * (5.0 / (nn + 5.0));
            }
        }
    }
    if (threadIdx.x == 0) {
        const double acc = h.n_leap ? h.sum_acc / h.n_leap : 0.0;
        h.da_t += 1.0;
        const double t = h.da_t, t0 = 10.0;
        h.h_bar = (1.0 - 1.0 / (t + t0)) * h.h_bar + (P.target - acc) / (t + t0);
        h.log_eps = h.mu - sqrt(t) / 0.05 * h.h_bar;
        const double eta = pow(t, -0.75);
        h.log_eps_bar = eta * h.log_eps + (1.0 - eta) * h.log_eps_bar;
        if (in_slow && window_end) {
            const double e = exp(h.log_eps);
            h.mu = log(10.0 * e);
            h.log_eps = log(e);
            h.log_eps_bar = 0.0;
            h.h_bar = 0.0;
            h.da_t = 0.0;
        }
        h.eps = exp(h.log_eps);
        if (last) h.eps = exp(h.log_eps_bar);
    }
}

__global__ void k_nuts_eps_out(const NutsChain *ch, double *eps, int n) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c < n) eps[c] = ch[c].eps;
}

// Nested R-hat per coordinate from one draw per chain (chains c = k*n_within
// + m form n_super super-chains): B = between-super-chain variance of the
// super-chain means, W = mean over super-chains of the variance of their
// chains about the super-chain mean; out = sqrt(1 + B / W).  One thread per
// coordinate; sums in a fixed order.
template <typename T>
__global__ void k_nested_rhat(const T *x, int M, int n_super, int n_within, double *out) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= M) return;
    double xbar = 0.0;
    for (int s = 0; s < n_super; ++s) {
        double m = 0.0;
        for (int w = 0; w < n_within; ++w) m += (double)x[(size_t)(s * n_within + w) * M + k];
        xbar += m / n_within;
    }
    xbar /= n_super;
    double B = 0.0, W = 0.0;
    for (int s = 0; s < n_super; ++s) {
        double m = 0.0;
        for (int w = 0; w < n_within; ++w) m += (double)x[(size_t)(s * n_within + w) * M + k];
        m /= n_within;
        B += (m - xbar) * (m - xbar);
        double v = 0.0;
        for (int w = 0; w < n_within; ++w) {
            const double dd = (double)x[(size_t)(s * n_within + w) * M + k] - m;
            v += dd * dd;
        }
        W += v / (n_within - 1);
    }
    B /= (n_super - 1);
    W /= n_super;
    out[k] = sqrt(1.0 + B / W);
}

}  // namespace mc
