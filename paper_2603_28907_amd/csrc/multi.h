// multi.h -- many heterogeneous problems per launch.
//
// Paper Sec. 3.2 runs many independent chains vectorised on one device; here
// many independent *problems* (different grids, sensors, pixel counts and
// chain counts) share each launch of an MCMC step.  Work items live in device
// tables: (problem, chain, ray tile) for the march, (problem, chain) for the
// proposal and the prior/Metropolis step.  Each block reads its item and the
// problem's descriptor with uniform (scalar) loads and runs exactly the
// device function the single-problem kernels use, so a chain's results do not
// depend on what else shares the launch.
#pragma once

#include "march3.h"
#include "march5.h"
#include "prior.h"

namespace mc {

// Random-walk proposal descriptor of one problem.
template <typename T>
struct ProposeDesc {
    const T *H;
    T *prop;
    int M;
    double sigma;
    uint64_t seed;
    const uint64_t *step_base;
};

// Items with problem index -1 are padding and are skipped.
//
// Persistent march over a static work table: block b takes items b, b + grid,
// b + 2 grid, ... (the table is sorted by decreasing cost on the host).  A
// static schedule keeps every item on a fixed block, so results do not depend
// on timing.  Each item's block body ends in a block-wide reduction, after
// which the staged surfaces may be overwritten by the next item.
//
// PERSIST = false is the one-item-per-block form (grid = number of items):
// without the loop the descriptor stays in scalar registers.
template <int S, bool TOP_LDS, int BLOCK, bool PERSIST>
__global__ __launch_bounds__(BLOCK, PERSIST ? 1 : march_waves_per_simd<BLOCK>()) void k_march_multi4(const MarchParams<float> *Ps, const RayConsts<float> *Ks,
                                                        const int4 *items, int n_items) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    if (!PERSIST) {
        const int4 it = items[blockIdx.x];
        if (it.x < 0) return;
        march_block4<S, TOP_LDS, BLOCK>(Ps[it.x], Ks[it.x], it.y, it.z, reinterpret_cast<float *>(smem_raw));
        return;
    }
    for (int i = blockIdx.x; i < n_items; i += gridDim.x) {
        const int4 it = items[i];
        if (it.x < 0) continue;
        const MarchParams<float> P = Ps[it.x];
        const RayConsts<float> K = Ks[it.x];
        march_block4<S, TOP_LDS, BLOCK>(P, K, it.y, it.z, reinterpret_cast<float *>(smem_raw));
        __syncthreads();
    }
}

template <typename T, int S, bool TOP_LDS, int BLOCK, bool PERSIST>
__global__ __launch_bounds__(BLOCK) void k_march_multi3(const MarchParams<T> *Ps, const RayConsts<T> *Ks,
                                                        const int4 *items, int n_items) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    if (!PERSIST) {
        const int4 it = items[blockIdx.x];
        if (it.x < 0) return;
        march_block3<T, S, TOP_LDS, BLOCK>(Ps[it.x], Ks[it.x], it.y, it.z, reinterpret_cast<T *>(smem_raw));
        return;
    }
    for (int i = blockIdx.x; i < n_items; i += gridDim.x) {
        const int4 it = items[i];
        if (it.x < 0) continue;
        const MarchParams<T> P = Ps[it.x];
        const RayConsts<T> K = Ks[it.x];
        march_block3<T, S, TOP_LDS, BLOCK>(P, K, it.y, it.z, reinterpret_cast<T *>(smem_raw));
        __syncthreads();
    }
}

template <typename T, int S, int BLOCK, bool HIER>
__global__ __launch_bounds__(BLOCK, 4) void k_prior_multi(const PriorParams<T> *Ps, const int2 *items, int step_k) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int2 it = items[blockIdx.x];
    prior_block<T, S, BLOCK, HIER>(Ps[it.x], it.y, reinterpret_cast<T *>(smem_raw), step_k);
}

// One block per (problem, chain): the pairs of normals of that chain.
template <typename T>
__global__ void k_propose_multi(const ProposeDesc<T> *Ds, const int2 *items, int step_k) {
    const int2 it = items[blockIdx.x];
    const ProposeDesc<T> D = Ds[it.x];
    const int c = it.y;
    const uint64_t step = *D.step_base + (uint64_t)step_k;
    const int pairs = (D.M + 1) / 2;
    for (int j = threadIdx.x; j < pairs; j += blockDim.x) {
        double z0, z1;
        rng_normal2(D.seed, (uint32_t)c, step, kTagProposal, (uint32_t)j, z0, z1);
        const size_t base = (size_t)c * D.M + 2 * (size_t)j;
        D.prop[base] = (T)((double)D.H[base] + D.sigma * z0);
        if (2 * j + 1 < D.M) D.prop[base + 1] = (T)((double)D.H[base + 1] + D.sigma * z1);
    }
}

__global__ void k_set_u64_multi(uint64_t *const *ptrs, const uint64_t *vals, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) *ptrs[i] = vals[i];
}

__global__ void k_add_u64_multi(uint64_t *const *ptrs, int n, uint64_t v) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) *ptrs[i] += v;
}

}  // namespace mc
