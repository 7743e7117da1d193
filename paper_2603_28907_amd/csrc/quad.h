// Solid-angle pixels (eq. expected_counts): the expected count of a pixel
// as a quadrature over sub-rays of its solid angle with a tabulated muon
// intensity of the opacity.
#pragma once
#include <hip/hip_runtime.h>

#include "device_common.h"

namespace mc {

// Solid-angle pixels (eq. expected_counts): lambda_p = sum_q w_q I(O_q) over
// the pixel's n_sub consecutive sub-rays, log I interpolated linearly on
// uniform opacity nodes (the last segment continued beyond the table), and
// the float64 Poisson term C log(lambda) - lambda per (chain, pixel).  Grid
// (tiles of 256 pixels, chains); one partial sum per block.  gp (optional,
// [n][n_ray]): dLL/dO of every sub-ray for the gradient,
// (C_p / lambda_p - 1) w_q I(O_q) dlogI/dO on O_q's table segment.
template <typename T>
__global__ __launch_bounds__(256) void k_quad_lik(const T *opacity, int n_ray, int n_px, int n_sub,
                                                  const double *w, const double *log_i, int n_tab, double inv_do,
                                                  const double *cnt, double *partials, int n_tiles,
                                                  const double *only_nan, T *gp = nullptr) {
    __shared__ double red[16];
    const size_t c = blockIdx.y;
    if (only_nan && !(only_nan[c] != only_nan[c])) return;   // uniform over the block
    const int px = blockIdx.x * 256 + threadIdx.x;
    double term = 0.0;
    if (px < n_px) {
        double lam = 0.0;
        for (int q = 0; q < n_sub; ++q) {
            const int r = px * n_sub + q;
            const double t = (double)opacity[c * n_ray + r] * inv_do;
            int j = (int)floor(t);
            j = j < 0 ? 0 : (j > n_tab - 2 ? n_tab - 2 : j);
            const double f = t - j;
            lam += w[r] * exp(log_i[j] + f * (log_i[j + 1] - log_i[j]));
        }
        term = cnt[px] * log(lam) - lam;
        if (gp) {
            const double a = cnt[px] / lam - 1.0;
            for (int k = 0; k < n_sub; ++k) {
                const int r = px * n_sub + k;
                const double t = (double)opacity[c * n_ray + r] * inv_do;
                int j = (int)floor(t);
                j = j < 0 ? 0 : (j > n_tab - 2 ? n_tab - 2 : j);
                const double f = t - j, dl = log_i[j + 1] - log_i[j];
                gp[c * n_ray + r] = (T)(a * w[r] * exp(log_i[j] + f * dl) * dl * inv_do);
            }
        }
    }
    const double s = block_sum<256>(term, red);
    if (threadIdx.x == 0) partials[c * n_tiles + blockIdx.x] = s;
}

}  // namespace mc
