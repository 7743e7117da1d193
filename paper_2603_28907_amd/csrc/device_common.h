// device_common.h -- shared device helpers for the gfx950 kernels: counter-
// based random numbers, deterministic wave/block reductions, small math.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mc {

constexpr int kWave = 64;          // CDNA wavefront width
constexpr int kMaxSurfaces = 4;    // S (including the fixed top) supported by the kernels

// MI355X has 8 XCDs, each with its own L2; consecutive workgroups of a
// launch are dispatched to the XCDs round-robin.
constexpr int kXcds = 8;

// XCD-aware block -> (chain, tile) map of a 1-D grid of
// n_tiles * round_up(n_chains, kXcds) blocks: block b runs on XCD b % kXcds
// and every tile of a chain goes to the same XCD, in consecutive slots, so
// the chain's surfaces are read from HBM once and then hit that XCD's L2.
// Returns false for the padding blocks of a ragged last group.
__device__ __forceinline__ bool xcd_chain_tile(int n_tiles, int n_chains, int &chain, int &tile) {
    const int b = blockIdx.x, x = b % kXcds, k = b / kXcds;
    chain = (k / n_tiles) * kXcds + x;
    tile = k % n_tiles;
    return chain < n_chains;
}

enum RngTag : uint32_t { kTagProposal = 0, kTagAccept = 1, kTagMala = 2, kTagRProposal = 3, kTagRAccept = 4 };

// Philox4x32-10 (Salmon, Moraes, Dror & Shaw, SC'11): ten rounds of two
// 32x32->64-bit multiplications whose high halves are mixed with the other
// two counter words and the key; the key advances by the Weyl increments
// between rounds.
__device__ __forceinline__ void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        const uint32_t m0 = 0xD2511F53u, m1 = 0xCD9E8D57u;
        uint32_t lo0 = m0 * c[0], hi0 = __umulhi(m0, c[0]);
        uint32_t lo1 = m1 * c[2], hi1 = __umulhi(m1, c[2]);
        uint32_t x0 = hi1 ^ c[1] ^ k0;
        uint32_t x2 = hi0 ^ c[3] ^ k1;
        c[0] = x0;
        c[1] = lo1;
        c[2] = x2;
        c[3] = lo0;
    }
}

// Counter (j, step lo32, step hi16 | tag << 16, chain), key = seed.
__device__ __forceinline__ void rng_words(uint64_t seed, uint32_t chain, uint64_t step, uint32_t tag,
                                          uint32_t j, uint32_t w[4]) {
    w[0] = j;
    w[1] = (uint32_t)step;
    w[2] = ((uint32_t)(step >> 32) & 0xFFFFu) | (tag << 16);
    w[3] = chain;
    philox4x32_10(w, (uint32_t)seed, (uint32_t)(seed >> 32));
}

// 53-bit uniform in [0,1) from two words.
__device__ __forceinline__ double uniform53(uint32_t a, uint32_t b) {
    return ((double)(a >> 5) * 67108864.0 + (double)(b >> 6)) * (1.0 / 9007199254740992.0);
}

__device__ __forceinline__ double rng_uniform(uint64_t seed, uint32_t chain, uint64_t step, uint32_t tag,
                                              uint32_t j) {
    uint32_t w[4];
    rng_words(seed, chain, step, tag, j, w);
    return uniform53(w[0], w[1]);
}

// Two standard normals by Box-Muller in float64.
__device__ __forceinline__ void rng_normal2(uint64_t seed, uint32_t chain, uint64_t step, uint32_t tag,
                                            uint32_t j, double &z0, double &z1) {
    uint32_t w[4];
    rng_words(seed, chain, step, tag, j, w);
    double ua = uniform53(w[0], w[1]), ub = uniform53(w[2], w[3]);
    double rad = sqrt(-2.0 * log(1.0 - ua));
    double th = 6.283185307179586476925286766559 * ub;
    z0 = rad * cos(th);
    z1 = rad * sin(th);
}

// Wave-level sum with a fixed butterfly order (bitwise reproducible).
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}
__device__ __forceinline__ float wave_min(float v) {
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) v = fminf(v, __shfl_xor(v, off, kWave));
    return v;
}
__device__ __forceinline__ float wave_max(float v) {
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) v = fmaxf(v, __shfl_xor(v, off, kWave));
    return v;
}
__device__ __forceinline__ double wave_min(double v) {
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) v = fmin(v, __shfl_xor(v, off, kWave));
    return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, kWave));
    return v;
}
__device__ __forceinline__ int wave_and(int v) {
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) v &= __shfl_xor(v, off, kWave);
    return v;
}

// Block-wide sum in a fixed order: waves reduce by butterfly, then wave 0
// adds the per-wave partials in wave order.  `scratch` holds >= 16 doubles.
// All threads get the result.
template <int BLOCK>
__device__ __forceinline__ double block_sum(double v, double *scratch) {
    constexpr int NW = BLOCK / kWave;
    v = wave_sum(v);
    const int lane = threadIdx.x % kWave, wid = threadIdx.x / kWave;
    __syncthreads();
    if (lane == 0) scratch[wid] = v;
    __syncthreads();
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < NW; ++w) t += scratch[w];
    __syncthreads();
    return t;
}

template <int BLOCK>
__device__ __forceinline__ int block_and(int v, int *scratch) {
    constexpr int NW = BLOCK / kWave;
    v = wave_and(v);
    const int lane = threadIdx.x % kWave, wid = threadIdx.x / kWave;
    __syncthreads();
    if (lane == 0) scratch[wid] = v;
    __syncthreads();
    int t = 1;
#pragma unroll
    for (int w = 0; w < NW; ++w) t &= scratch[w];
    __syncthreads();
    return t;
}

template <typename T> __device__ __forceinline__ T dev_inf();
template <> __device__ __forceinline__ float dev_inf<float>() { return __builtin_huge_valf(); }
template <> __device__ __forceinline__ double dev_inf<double>() { return __builtin_huge_val(); }

__device__ __forceinline__ float dfma(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double dfma(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float dmin(float a, float b) { return fminf(a, b); }
__device__ __forceinline__ double dmin(double a, double b) { return fmin(a, b); }
__device__ __forceinline__ float dmax(float a, float b) { return fmaxf(a, b); }
__device__ __forceinline__ double dmax(double a, double b) { return fmax(a, b); }
__device__ __forceinline__ float dsqrt(float a) { return __builtin_sqrtf(a); }
__device__ __forceinline__ double dsqrt(double a) { return __builtin_sqrt(a); }
__device__ __forceinline__ float dabs(float a) { return fabsf(a); }
__device__ __forceinline__ double dabs(double a) { return fabs(a); }

}  // namespace mc
