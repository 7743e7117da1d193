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
};

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
// block holds).
template <typename T, int S, int BLOCK>
__device__ __forceinline__ void prior_block(const PriorParams<T> &P, int c, T *w, int step_k) {
    __shared__ double red[16];
    __shared__ int ired[16];
    __shared__ int s_acc;
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
        const double r = P.r[l], s11 = P.s11[l];
        lp += 0.5 * P.logdet[l] - 0.5 * s11 * (4.0 * (1.0 - r) * SW2 + r * SE) + 0.5 * N * log(s11) +
              0.5 * SW2 - SLD;
    }
    ok = block_and<BLOCK>(ok, ired);
    if (tid == 0) {
        double ll = 0.0;
        if (P.has_lik) {
            const double *pp = P.partials + (size_t)c * P.n_tiles;
            for (int t = 0; t < P.n_tiles; ++t) ll += pp[t];
            ll += P.kconst;
        }
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
        }
    }
    if (P.mh) {
        __syncthreads();
        if (s_acc) {
            const int M = (S - 1) * N;
            T *dst = P.state + (size_t)c * M;
            for (int n = tid; n < M; n += BLOCK) dst[n] = H[n];
        }
    }
}

template <typename T, int S, int BLOCK>
__global__ __launch_bounds__(BLOCK, 4) void k_prior_finalize(PriorParams<T> P) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    prior_block<T, S, BLOCK>(P, blockIdx.x, reinterpret_cast<T *>(smem_raw), P.step_k);
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
