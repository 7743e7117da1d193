// The latent parametrisation the paper's sampler runs on (Sec. 2.2.1,
// 3.1): the CAR fields x_l ~ N(0, Q_l^-1) of the free surfaces, mapped to
// heights by the copula map w = x / sqrt(Sigma11_l), u = Phi(w),
// H_l = (1 - u) H_{l-1} + u H_top (H_0 = 0).  The log density of x is
//   log L(H(x)) + sum_l [ log det(Q_l)/2 - x_l' Q_l x_l / 2 - (N/2) log 2 pi ],
// with no boundaries, and its gradient is the likelihood gradient in H (the
// adjoint march) carried through the map node by node, top layer first:
// D_l = dlogL/dH_l + (1 - u_{l+1}) D_{l+1}, dlogL/dx_l = D_l (H_top - H_{l-1})
// phi(w_l) / sqrt(Sigma11_l), plus -Q_l x_l from the prior.
#pragma once
#include <hip/hip_runtime.h>

#include "adjoint.h"
#include "device_common.h"
#include "prior.h"

namespace mc {

template <typename T>
struct LatentParams {
    int R, C, N, S1, SN, n, n_tiles, has_lik;
    int xs;                        // values per chain in x: S1 N, or S1 N + S1 with logit r appended
    double s[kMaxSurfaces];        // sqrt(Sigma11_l)
    double r[kMaxSurfaces];        // CAR dependence
    double logdet[kMaxSurfaces];   // log det Q_l
    double kconst;                 // likelihood constant
    const double *top64;           // [N]
    const T *x;                    // [n][xs] latent states (S1 fields of N, then logit r when sampled)
    T *H;                          // [n][S1][N] heights (the march's input)
    const unsigned long long *gfix;   // [n][SN] likelihood gradient in H, 2^-32 fixed point
    const double *partials;        // [n][n_tiles] likelihood partial sums
    double *lp;                    // [n]
    T *gx;                         // [n][SN] gradient in x (free part first, then the logit-r part or zeros)
    // r sampled per chain (rc set): constants of each chain's r, [n][S1][kRc]
    double *rc;
    const double *eig_g, *eig_w;   // distinct torus eigenvalue terms and their multiplicities
    int n_eig;
};

// Per-chain constants of r (rc[c][l][.]): r, sqrt(Sigma11(r)), log det Q(r),
// d log det Q / dr, d Sigma11 / dr.
enum { kRcR = 0, kRcS, kRcLogdet, kRcDlogdet, kRcDs11, kRc };

// One block per chain: r = logistic(eta) for every free surface and the
// torus sums over the distinct eigenvalues mu = 4 - 2 r g (multiplicity w):
// log det Q = sum w log mu, Sigma11 = sum w / mu / N, and their r-derivatives
// sum -2 w g / mu and sum 2 w g / mu^2 / N.
template <typename T, int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_latent_r_consts(LatentParams<T> P) {
    __shared__ double red[16];
    const size_t c = blockIdx.x;
    for (int l = 0; l < P.S1; ++l) {
        const double eta = (double)P.x[c * P.xs + (size_t)P.S1 * P.N + l];
        const double r = 1.0 / (1.0 + exp(-eta));
        double a = 0.0, b = 0.0, da = 0.0, db = 0.0;
        for (int k = threadIdx.x; k < P.n_eig; k += BLOCK) {
            const double g = P.eig_g[k], w = P.eig_w[k], mu = 4.0 - 2.0 * r * g;
            a += w * log(mu);
            b += w / mu;
            da += -2.0 * w * g / mu;
            db += 2.0 * w * g / (mu * mu);
        }
        a = block_sum<BLOCK>(a, red);
        b = block_sum<BLOCK>(b, red);
        da = block_sum<BLOCK>(da, red);
        db = block_sum<BLOCK>(db, red);
        if (threadIdx.x == 0) {
            double *o = P.rc + (c * P.S1 + l) * kRc;
            o[kRcR] = r;
            o[kRcS] = sqrt(b / (double)P.N);
            o[kRcLogdet] = a;
            o[kRcDlogdet] = da;
            o[kRcDs11] = db / (double)P.N;
        }
    }
}

__device__ __forceinline__ double std_cdf(double w) { return 0.5 * erfc(-w * 0.70710678118654752440); }

// H_l of one node from the latent values, in float64: the lower tail when
// w <= 0 and the upper tail otherwise.
__device__ __forceinline__ double latent_h(double a, double b, double w) {
    return w <= 0.0 ? a + std_cdf(w) * (b - a) : b - std_cdf(-w) * (b - a);
}

template <typename T>
__global__ void k_latent_to_heights(LatentParams<T> P) {
    const size_t c = blockIdx.y;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= P.N) return;
    const double b = P.top64[i];
    double a = 0.0;
    for (int l = 0; l < P.S1; ++l) {
        const double s = P.rc ? P.rc[(c * P.S1 + l) * kRc + kRcS] : P.s[l];
        const double h = latent_h(a, b, (double)P.x[c * P.xs + (size_t)l * P.N + i] / s);
        P.H[(c * P.S1 + l) * P.N + i] = (T)h;
        a = h;
    }
}

// The inverse map: x_l = sqrt(Sigma11_l) Phi^-1(u), u and 1 - u from the
// heights directly (the same tail rule as the prior).
template <typename T>
__global__ void k_heights_to_latent(const T *H, T *x, const double *top64, int N, int S1, double s0, double s1,
                                    double s2) {
    const size_t c = blockIdx.y;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const double b = top64[i], sl[3] = {s0, s1, s2};
    double a = 0.0;
    for (int l = 0; l < S1; ++l) {
        const size_t o = (c * S1 + l) * N + i;
        const double h = (double)H[o], d = b - a;
        x[o] = (T)(sl[l] * probit_uv((h - a) / d, (b - h) / d));
        a = h;
    }
}

// Log density and gradient in x (and in logit r when sampled), one block per
// chain (512 threads: few chains still keep the compute units busy, without
// spilling the per-node layer values).  With r sampled the density gains
// log(r (1 - r)) per surface (the flat prior's Jacobian in eta = logit r) and
//   dlogp/deta_l = r (1 - r) (dlogL/dr_l + (d log det Q/dr)/2 + x_l' A x_l / 2) + 1 - 2 r,
//   dlogL/dr_l = sum_i D_l,i (H_top - H_{l-1}) phi(w) (-w (dSigma11/dr) / (2 Sigma11)).
template <typename T, int S, int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_latent_finish(LatentParams<T> P) {
    __shared__ double red[16];
    const size_t c = blockIdx.x;
    const int tid = threadIdx.x;
    constexpr int S1 = S - 1, NA = S1 > 0 ? S1 : 1;   // free surfaces; array extent
    double llp = 0.0;
    if (P.has_lik)
        for (int t = tid; t < P.n_tiles; t += BLOCK) llp += P.partials[c * P.n_tiles + t];
    double sl[NA], rl[NA], kr[NA];
#pragma unroll
    for (int l = 0; l < S1; ++l) {
        const double *rc = P.rc ? P.rc + (c * S1 + l) * kRc : nullptr;
        sl[l] = rc ? rc[kRcS] : P.s[l];
        rl[l] = rc ? rc[kRcR] : P.r[l];
        kr[l] = rc ? -rc[kRcDs11] / (2.0 * sl[l] * sl[l]) : 0.0;   // (dw/dr) / w
    }
    double quadl[NA] = {}, xaxl[NA] = {}, drl[NA] = {};   // x_l' Q_l x_l, x_l' A x_l, dlogL/dr_l of this thread's nodes
    const T *xc = P.x + c * (size_t)P.xs;
    for (int n = tid; n < P.N; n += BLOCK) {
        const int i = n / P.C, j = n - i * P.C;
        const int jr = j + 1 == P.C ? 0 : j + 1, jl = j == 0 ? P.C - 1 : j - 1;
        const int id = i + 1 == P.R ? 0 : i + 1, iu = i == 0 ? P.R - 1 : i - 1;
        const double b = P.top64[n];
        double xv[NA], qx[NA], av[NA], wv[NA];
        double a = 0.0;
#pragma unroll
        for (int l = 0; l < S1; ++l) {
            const T *xl = xc + (size_t)l * P.N;
            xv[l] = (double)xl[n];
            const double nb = (double)xl[i * P.C + jr] + (double)xl[i * P.C + jl] + (double)xl[id * P.C + j] +
                              (double)xl[iu * P.C + j];
            qx[l] = 4.0 * xv[l] - rl[l] * nb;
            quadl[l] += xv[l] * qx[l];
            xaxl[l] += xv[l] * nb;
            wv[l] = xv[l] / sl[l];
            av[l] = a;
            a = latent_h(a, b, wv[l]);
        }
        // chain rule, top layer first
        double D = 0.0;
#pragma unroll
        for (int l = S1 - 1; l >= 0; --l) {
            const size_t o = c * P.SN + (size_t)l * P.N + n;
            const double gh = P.has_lik ? (double)(long long)P.gfix[o] * kGradFixInv : 0.0;
            D = gh + (l < S1 - 1 ? std_cdf(-wv[l + 1]) * D : 0.0);
            const double phi = 0.39894228040143267794 * exp(-0.5 * wv[l] * wv[l]);
            const double dh = D * (b - av[l]) * phi;   // dlogL/dw_l
            P.gx[o] = (T)(dh / sl[l] - qx[l]);
            drl[l] += dh * wv[l] * kr[l];
        }
        P.gx[c * P.SN + (size_t)S1 * P.N + n] = T(0);
    }
    const double ll = block_sum<BLOCK>(llp, red);
    double prior = 0.0;
#pragma unroll
    for (int l = 0; l < S1; ++l) {
        const double ql = block_sum<BLOCK>(quadl[l], red);
        const double *rc = P.rc ? P.rc + (c * S1 + l) * kRc : nullptr;
        prior += 0.5 * (rc ? rc[kRcLogdet] : P.logdet[l]) - 0.5 * ql - 0.5 * P.N * 1.83787706640934548356;   // log(2 pi)
        if (rc) {
            const double xax = block_sum<BLOCK>(xaxl[l], red);
            const double dr = block_sum<BLOCK>(drl[l], red);
            const double r = rc[kRcR];
            prior += log(r * (1.0 - r));
            if (tid == 0)
                P.gx[c * P.SN + (size_t)S1 * P.N + l] =
                    (T)(r * (1.0 - r) * (dr + 0.5 * rc[kRcDlogdet] + 0.5 * xax) + (1.0 - 2.0 * r));
        }
    }
    if (tid == 0) P.lp[c] = prior + (P.has_lik ? ll + P.kconst : 0.0);
}

}  // namespace mc
