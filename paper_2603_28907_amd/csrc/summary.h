// summary.h -- chain initialisation and posterior summaries for the serving
// loop.
//
// Paper Sec. 3.2 keeps only the last state of every chain; a job's summary
// is computed from those states on the device: per-node mean and standard
// deviation over chains, the chain with the highest log posterior (a MAP
// estimate among the samples, paper Sec. 4) and the acceptance count.  All
// sums run in float64 in a fixed order, so a summary is deterministic.
#pragma once

#include "device_common.h"

namespace mc {

// Every chain starts from the same state init[M] (float64 on the device).
template <typename T>
__global__ void k_broadcast_init(const double *__restrict__ init, T *__restrict__ H, int n, int M) {
    const size_t tot = (size_t)n * M;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < tot; i += (size_t)gridDim.x * blockDim.x)
        H[i] = (T)init[i % M];
}

// Per node m: mean and population standard deviation over the n chains
// (two passes, chains in index order).
template <typename T>
__global__ void k_node_summary(const T *__restrict__ H, int n, int M, double *__restrict__ mean,
                               double *__restrict__ sd) {
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= M) return;
    double s = 0.0;
    for (int c = 0; c < n; ++c) s += (double)H[(size_t)c * M + m];
    const double mu = s / n;
    double v = 0.0;
    for (int c = 0; c < n; ++c) {
        const double d = (double)H[(size_t)c * M + m] - mu;
        v = dfma(d, d, v);
    }
    mean[m] = mu;
    sd[m] = dsqrt(v / n);
}

// One block: the highest log posterior (lowest chain index on ties; -inf
// chains count, NaN never wins) and the total acceptance count.
// out[0] = best log posterior, out[1] = its chain (as double), out[2] = accepted.
template <int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_chain_summary(const double *__restrict__ lp,
                                                         const int64_t *__restrict__ acc, int n,
                                                         double *__restrict__ out) {
    __shared__ double sv[BLOCK];
    __shared__ int si[BLOCK];
    __shared__ long long sa[BLOCK];
    const int t = threadIdx.x;
    double bv = -dev_inf<double>();
    int bi = n;   // sentinel: no chain yet
    long long a = 0;
    for (int c = t; c < n; c += BLOCK) {
        const double v = lp[c];
        if (v > bv || (bi == n && !(v != v))) {
            bv = v;
            bi = c;
        }
        a += acc[c];
    }
    sv[t] = bv;
    si[t] = bi;
    sa[t] = a;
    __syncthreads();
    for (int w = BLOCK / 2; w > 0; w /= 2) {
        if (t < w) {
            const double ov = sv[t + w];
            const int oi = si[t + w];
            if (oi < n && (si[t] == n || ov > sv[t] || (ov == sv[t] && oi < si[t]))) {
                sv[t] = ov;
                si[t] = oi;
            }
            sa[t] += sa[t + w];
        }
        __syncthreads();
    }
    if (t == 0) {
        out[0] = sv[0];
        out[1] = (double)(si[0] < n ? si[0] : 0);
        out[2] = (double)sa[0];
    }
}

// The state of the chain chosen by k_chain_summary, widened to float64.
template <typename T>
__global__ void k_copy_chain(const T *__restrict__ H, int M, const double *__restrict__ chain_idx,
                             double *__restrict__ out) {
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= M) return;
    const size_t c = (size_t)chain_idx[0];
    out[m] = (double)H[c * M + m];
}

}  // namespace mc
