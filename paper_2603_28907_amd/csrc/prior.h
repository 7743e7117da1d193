// prior.h -- per-chain log prior (Gaussian copula over a periodic proper CAR
// field, paper Sec. 2.2.1), the fixed-order sum of the likelihood partials,
// and the fused Metropolis decision.
//
// For free surface l with a = H_{l-1} (0 for l = 1), b = H_top, N = R C:
//   u = (H_l - a)/(b - a),  w = Phi^-1(u),  x = s w,  s^2 = Sigma_11(r_l)
//   log p(H_l | H_{l-1}) = 1/2 log det Q - 1/2 x^T Q x + N log s
//                          + 1/2 sum w^2 - sum log(b - a)
//   x^T Q x = s^2 [ 4(1-r) sum w^2 + r sum_{right/down edges} (w_i - w_j)^2 ]
// (Q = diag(A1) - rA on the periodic 4-neighbour grid; the 2 pi terms cancel.)
// log det Q and Sigma_11 come from the host (closed form on the torus).
#pragma once

#include "device_common.h"

namespace mc {

template <typename T>
struct PriorParams {
    int R, C, n_tiles, has_lik;
    const T *heights;                  // [n][S-1][N] states whose lp is computed
    const double *top64;               // [N]
    double logdet[kMaxSurfaces - 1];   // per free surface
    double s11[kMaxSurfaces - 1];
    double r[kMaxSurfaces - 1];
    double sum_log_top;                // sum_n log(top_n)
    const double *partials;            // [n][n_tiles]
    double kconst;                     // sum_p C_p log E_p - log C_p!
    double *lp_out;                    // [n] (plain mode)
    const double *only_nan;            // if set, chains whose entry is not NaN are skipped
    // Metropolis mode: heights are proposals; compare with lp_cur, on
    // acceptance copy the proposal into `state` and count it.
    int mh;
    double *lp_cur;
    int64_t *n_acc;
    T *state;
    uint64_t seed;
    const uint64_t *step_base;
    int step_k;
    // Hierarchical r (Sec. 2.2.1, r_l ~ Uniform(0, 1)): with r_chain set the
    // CAR constants come per chain from the torus eigenvalue table, and in
    // Metropolis mode with sample_r each r_l takes a logit-scale Metropolis
    // step after the H decision.
    double *r_chain;                   // [n][S-1] or null (problem r)
    const double *eig_g, *eig_w;       // distinct cos(2 pi k/R) + cos(2 pi m/C), multiplicities
    int n_eig;
    double *stat_sw2, *stat_se;        // [n][S-1] sum w^2 and edge sum of the current states
    int sample_r;
    double r_step;
    int64_t *n_acc_r;                  // [n][S-1] or null
};

// log det Q(r) and Sigma_11(r) on the R x C torus from its eigenvalues
// mu = 4 - 2 r g (g over the distinct values with their multiplicities),
// summed by the whole block in a fixed order.
template <typename T, int BLOCK>
__device__ __forceinline__ void car_consts_block(const PriorParams<T> &P, double r, int N, double *red,
                                                 double &logdet, double &s11) {
    double sl = 0.0, si = 0.0;
    for (int k = threadIdx.x; k < P.n_eig; k += BLOCK) {
        const double mu = 4.0 - 2.0 * r * P.eig_g[k];
        sl += P.eig_w[k] * log(mu);
        si += P.eig_w[k] / mu;
    }
    logdet = block_sum<BLOCK>(sl, red);
    s11 = block_sum<BLOCK>(si, red) / (double)N;
}

// The r-dependent part of log p(H_l | H_{l-1}, r) given sum w^2 and the edge sum.
__device__ __forceinline__ double car_r_terms(double r, double logdet, double s11, double sw2, double se, int N) {
    return 0.5 * logdet - 0.5 * s11 * (4.0 * (1.0 - r) * sw2 + r * se) + 0.5 * N * log(s11);
}

// Threads per prior block: grids of 8192 nodes and more use 1024 so that a
// block whose workspace fills much of the LDS still keeps 16 wavefronts.
constexpr int kPriorBlockLarge = 1024;
constexpr int kPriorLargeNodes = 8192;

// w = Phi^-1(u) with u = (h-a)/d and v = 1-u = (b-h)/d; the tail nearer to u
// is evaluated directly.  Kept out of line: inlined into a node loop, the
// compiler hoists the polynomial coefficients of Phi^-1 out of the loop into
// some 200 vector registers (one wavefront per SIMD).
__device__ __attribute__((noinline)) double probit_uv(double u, double v) {
    const bool lower = u <= 0.5;
    const double w = normcdfinv(lower ? u : v);   // one call: the tails share the code
    return lower ? w : -w;
}

// Body of one block for chain c; w = LDS workspace of R*C values in the
// state precision T (the Phi^-1 values are formed and summed in float64; the
// copy kept for the neighbour differences is rounded to T, which in float32
// mode is far below the float32 march's own rounding and halves the LDS a
// block holds).  HIER: every chain carries its own r (P.r_chain), and in MH
// mode r is updated after the H decision; the fixed-r instance keeps none of
// that code (and none of its registers).
template <typename T, int S, int BLOCK, bool HIER = false>
__device__ __forceinline__ void prior_block(const PriorParams<T> &P, int c, T *w, int step_k) {
    __shared__ double red[16];
    __shared__ int ired[16];
    __shared__ int s_acc, s_fin;
    __shared__ double s_sw2[kMaxSurfaces], s_se[kMaxSurfaces], s_ld[kMaxSurfaces], s_s11[kMaxSurfaces],
        s_r[kMaxSurfaces];
    const int tid = threadIdx.x;
    if (P.only_nan && !(P.only_nan[c] != P.only_nan[c])) return;
    const int R = P.R, C = P.C, N = R * C;
    const T *H = P.heights + (size_t)c * (S - 1) * N;
    double lp = 0.0;
    int ok = 1;
#pragma unroll 1
    for (int l = 0; l < S - 1; ++l) {
        double sw2 = 0.0, sld = 0.0;
#pragma unroll 1
        for (int n = tid; n < N; n += BLOCK) {
            const double h = (double)H[l * N + n];
            const double a = l ? (double)H[(l - 1) * N + n] : 0.0;
            const double b = P.top64[n];
            const double d = b - a;
            const double id = 1.0 / d;
            const double u = (h - a) * id, v = (b - h) * id;
            const bool good = (d > 0.0) && (u > 0.0) && (v > 0.0);
            ok &= good ? 1 : 0;
            const double wi = good ? probit_uv(u, v) : 0.0;
            w[n] = (T)wi;
            sw2 += wi * wi;
            // log(b - a) of the first surface is log(top): summed once on the host
            if (l) sld += good ? log(d) : 0.0;
        }
        if (l == 0) sld = tid == 0 ? P.sum_log_top : 0.0;
        __syncthreads();
        double se = 0.0;
#pragma unroll 1
        for (int n = tid; n < N; n += BLOCK) {
            const int i = n / C, j = n - i * C;
            const double wi = (double)w[n];
            const double wr = (double)w[i * C + (j + 1 == C ? 0 : j + 1)];
            const double wd = (double)w[(i + 1 == R ? 0 : i + 1) * C + j];
            se += (wi - wr) * (wi - wr) + (wi - wd) * (wi - wd);
        }
        const double SW2 = block_sum<BLOCK>(sw2, red);
        const double SLD = block_sum<BLOCK>(sld, red);
        const double SE = block_sum<BLOCK>(se, red);
        double r = P.r[l], ld = P.logdet[l], s11 = P.s11[l];
        if (HIER) {
            r = P.r_chain[(size_t)c * (S - 1) + l];
            car_consts_block<T, BLOCK>(P, r, N, red, ld, s11);
        }
        lp += car_r_terms(r, ld, s11, SW2, SE, N) + 0.5 * SW2 - SLD;
        if (tid == 0) {
            s_sw2[l] = SW2;
            s_se[l] = SE;
            s_ld[l] = ld;
            s_s11[l] = s11;
            s_r[l] = r;
        }
    }
    ok = block_and<BLOCK>(ok, ired);
    // sum of the likelihood partials of the chain's tiles: strided per thread,
    // then a block sum (fixed order for a given BLOCK)
    double llp = 0.0;
    if (P.has_lik) {
        const double *pp = P.partials + (size_t)c * P.n_tiles;
        for (int t = tid; t < P.n_tiles; t += BLOCK) llp += pp[t];
    }
    const double ll_sum = block_sum<BLOCK>(llp, red);
    if (HIER && !P.mh && P.stat_sw2 && tid == 0) {
        for (int l = 0; l < S - 1; ++l) {
            P.stat_sw2[(size_t)c * (S - 1) + l] = s_sw2[l];
            P.stat_se[(size_t)c * (S - 1) + l] = s_se[l];
        }
    }
    if (tid == 0) {
        const double ll = P.has_lik ? ll_sum + P.kconst : 0.0;
        const double total = ok ? lp + ll : -__builtin_huge_val();
        if (!P.mh) {
            P.lp_out[c] = total;
        } else {
            const uint64_t step = *P.step_base + (uint64_t)step_k;
            const double u = rng_uniform(P.seed, (uint32_t)c, step, kTagAccept, 0);
            const double la = total - P.lp_cur[c];
            const int acc = log(u) < la;
            if (acc) {
                P.lp_cur[c] = total;
                P.n_acc[c] += 1;
            }
            s_acc = acc;
            s_fin = P.lp_cur[c] > -__builtin_huge_val();
        }
    }
    if (P.mh) {
        __syncthreads();
        if (s_acc) {
            const int M = (S - 1) * N;
            T *dst = P.state + (size_t)c * M;
            for (int n = tid; n < M; n += BLOCK) dst[n] = H[n];
        }
        if (HIER && P.sample_r) {
            // r_l given the current H, one surface at a time
            const uint64_t step = *P.step_base + (uint64_t)step_k;
#pragma unroll 1
            for (int l = 0; l < S - 1; ++l) {
                const size_t at = (size_t)c * (S - 1) + l;
                const double sw2 = s_acc ? s_sw2[l] : P.stat_sw2[at];
                const double se = s_acc ? s_se[l] : P.stat_se[at];
                const double r = s_r[l];
                double z0, z1;
                rng_normal2(P.seed, (uint32_t)c, step, kTagRProposal, (uint32_t)(l / 2), z0, z1);
                const double rn = 1.0 / (1.0 + exp(-(log(r / (1.0 - r)) + P.r_step * ((l & 1) ? z1 : z0))));
                double la = -__builtin_huge_val(), dlp = 0.0;
                if (rn > 0.0 && rn < 1.0) {   // uniform across the block
                    double ldn, s11n;
                    car_consts_block<T, BLOCK>(P, rn, N, red, ldn, s11n);
                    if (s_fin)
                        dlp = car_r_terms(rn, ldn, s11n, sw2, se, N) - car_r_terms(r, s_ld[l], s_s11[l], sw2, se, N);
                    la = dlp + log(rn * (1.0 - rn)) - log(r * (1.0 - r));
                }
                if (tid == 0) {
                    const double u = rng_uniform(P.seed, (uint32_t)c, step, kTagRAccept, (uint32_t)l);
                    if (log(u) < la) {
                        P.r_chain[at] = rn;
                        if (s_fin) P.lp_cur[c] += dlp;
                        if (P.n_acc_r) P.n_acc_r[at] += 1;
                    }
                }
            }
            if (tid == 0 && s_acc) {
                for (int l = 0; l < S - 1; ++l) {
                    P.stat_sw2[(size_t)c * (S - 1) + l] = s_sw2[l];
                    P.stat_se[(size_t)c * (S - 1) + l] = s_se[l];
                }
            }
        }
    }
}

template <typename T, int S, int BLOCK, bool HIER>
__global__ __launch_bounds__(BLOCK, 4) void k_prior_finalize(PriorParams<T> P) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    prior_block<T, S, BLOCK, HIER>(P, blockIdx.x, reinterpret_cast<T *>(smem_raw), P.step_k);
}

// Random-walk proposal: prop = H + sigma z, z_i the (i%2)-th normal of pair
// j = i/2 of (chain, step, tag 0); computed in float64, stored in T.
template <typename T>
__global__ void k_propose_rw(const T *H, T *prop, int M, double sigma, uint64_t seed,
                             const uint64_t *step_base, int step_k) {
    const int c = blockIdx.y;
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (2 * j >= M) return;
    const uint64_t step = *step_base + (uint64_t)step_k;
    double z0, z1;
    rng_normal2(seed, (uint32_t)c, step, kTagProposal, (uint32_t)j, z0, z1);
    const size_t base = (size_t)c * M + 2 * (size_t)j;
    prop[base] = (T)((double)H[base] + sigma * z0);
    if (2 * j + 1 < M) prop[base + 1] = (T)((double)H[base + 1] + sigma * z1);
}

// lp[c] = tmp[c] where lp[c] is NaN (initial log posterior of a run).
__global__ void k_fill_nan(double *lp, const double *tmp, int n) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c < n && lp[c] != lp[c]) lp[c] = tmp[c];
}

__global__ void k_set_u64(uint64_t *p, uint64_t v) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *p = v;
}

__global__ void k_add_u64(uint64_t *p, uint64_t v) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *p += v;
}

__global__ void k_debug_philox(uint64_t seed, uint32_t chain, uint64_t step, uint32_t tag, uint32_t j0, int n,
                               uint32_t *out_u32, double *out_normal) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint32_t w[4];
    rng_words(seed, chain, step, tag, j0 + (uint32_t)i, w);
    if (out_u32) {
        out_u32[4 * i] = w[0];
        out_u32[4 * i + 1] = w[1];
        out_u32[4 * i + 2] = w[2];
        out_u32[4 * i + 3] = w[3];
    }
    if (out_normal) {
        double z0, z1;
        rng_normal2(seed, chain, step, tag, j0 + (uint32_t)i, z0, z1);
        out_normal[2 * i] = z0;
        out_normal[2 * i + 1] = z1;
    }
}

}  // namespace mc
