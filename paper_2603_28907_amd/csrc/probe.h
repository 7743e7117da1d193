// probe.h -- VALU issue-rate microbenchmark (roofline denominator).
//
// Each thread runs 8 independent dependency chains of one fused multiply-add
// (float32 or float64, one non-packed VALU instruction each) for `iters`
// rounds; enough waves are launched to fill every SIMD.
// lane-ops/s = threads * iters * 8 / time.
#pragma once

#include "device_common.h"

namespace mc {

enum ProbeKind { kProbeF32Fma = 0, kProbeF64Fma = 1 };

template <typename T>
__global__ __launch_bounds__(256) void k_valu_probe(T *out, int iters, T m, T c) {
    const T s = (T)(threadIdx.x + 1);
    T a0 = s, a1 = s + (T)1, a2 = s + (T)2, a3 = s + (T)3, a4 = s + (T)4, a5 = s + (T)5, a6 = s + (T)6,
      a7 = s + (T)7;
    for (int i = 0; i < iters; ++i) {
        a0 = dfma(a0, m, c); a1 = dfma(a1, m, c); a2 = dfma(a2, m, c); a3 = dfma(a3, m, c);
        a4 = dfma(a4, m, c); a5 = dfma(a5, m, c); a6 = dfma(a6, m, c); a7 = dfma(a7, m, c);
    }
    const T r = ((a0 + a1) + (a2 + a3)) + ((a4 + a5) + (a6 + a7));
    if (r == (T)-12345) out[blockIdx.x * blockDim.x + threadIdx.x] = r;   // keeps the chains live
}

}  // namespace mc
