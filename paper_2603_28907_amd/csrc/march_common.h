// march_common.h -- launch parameters and the shared-edge boundary rule of
// the ray-march kernels.
//
// Opacity (paper Sec. 2.1.1) of the layered density (eq. def_LM_density_grid,
// continuum form): O = sum_l (rho_l - rho_{l+1}) L_l, with L_l the length of
// the ray inside the box lying below surface l.  Inside a grid cell a
// bilinear surface restricted to the ray is a quadratic in t, so L_l is a sum
// of exact per-cell pieces.
//
// Robust per-cell evaluation.  Each cell interval [t0, t1] of the 2-D cell
// walk is either certain (the ray's z-range lies entirely below the patch
// minimum or above its maximum, with a rounding margin) or ambiguous.  In an
// ambiguous cell the signs of f = z - h at the two ends decide the number of
// crossings; each end value is computed by one formula that depends only on
// the boundary point (the lerp along the shared cell edge), so the two cells
// that meet at a boundary see the same bits and a crossing is never dropped
// or counted twice.  The in-cell quadratic is rebuilt from the two end values
// and the patch curvature c2 = -D ds dw.
#pragma once

#include "device_common.h"

namespace mc {

enum BoundaryKind : int { kPoint = 0, kXEdge = 1, kYEdge = 2 };

template <typename T>
struct MarchParams {
    int R, C, n_ray, n_pix, n_tiles, rays_per_block;
    int n_chains;                      // chains in the launch
    T hx, hy, ihx, ihy, xmax, ymax;   // cell sizes, their inverses, (R-1) hx, (C-1) hy
    T ztop;                            // max of the top surface
    T margin;                          // rounding margin for the certain tests
    T lid;                             // crossings at or above this height meet the box lid (a kink of lp)
    T top_min, top_max;                // range of the top surface
    T rho_diff[kMaxSurfaces];          // rho_l - rho_{l+1}
    const T *sensor;                   // [n_s][3]
    const T *dx, *dy, *dz;             // [n_ray] ray directions
    const double *c_over_L;            // [n_ray] C_p / Lambda
    const double *expo;                // [n_ray] E_p
    double inv_L;                      // 1 / Lambda
    const T *top;                      // [R*C] fixed top surface
    const T *heights;                  // [n_chains][S-1][R*C]
    T *opacity;                        // [n_chains][n_ray] or null
    double *partials;                  // [n_chains][n_tiles]
    const double *only_nan;            // if set, chains whose entry is not NaN are skipped
};

// f = z - h at a boundary point of the piece.  kind/entry pick the formula:
// an x-edge (node row) lerps along y, a y-edge (node column) lerps along x,
// a point inside the box uses the full bilinear patch.
template <typename T>
__device__ __forceinline__ T boundary_value(int kind, bool entry, bool xpos, bool ypos, T z, T s, T w,
                                            T h00, T h10, T h01, T h11) {
    if (kind == kXEdge) {
        // entry: row a if moving +x else a+1; exit: the opposite row
        bool lower = (entry == xpos);
        T hA = lower ? h00 : h10, hB = lower ? h01 : h11;
        return z - dfma(w, hB - hA, hA);
    }
    if (kind == kYEdge) {
        bool lower = (entry == ypos);
        T hA = lower ? h00 : h01, hB = lower ? h10 : h11;
        return z - dfma(s, hB - hA, hA);
    }
    T hl = dfma(s, h10 - h00, h00), hh = dfma(s, h11 - h01, h01);
    return z - dfma(w, hh - hl, hl);
}

}  // namespace mc
