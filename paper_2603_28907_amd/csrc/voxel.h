// The paper's own forward model as an alternate likelihood backend: the
// sigmoid-smoothed voxel density R-hat(H) (eqs. smooth_layer_indicators and
// def_LM_density_grid_smooth) and the linearised expected counts
// lambda-hat = lambda(R0) + G (R-hat - R0) (eq. expected_counts_linearized_approx),
// with G_pv = -lambda_p(R0) L_pv / Lambda and L_pv the length of ray p in
// voxel v.  Since G's row p is a multiple of the ray's voxel lengths,
// lambda-hat_p = lambda_p(R0) (1 - (O_p(R-hat) - O_p(R0)) / Lambda), where
// O_p(R) = sum_v L_pv R_v: one gather-and-sum along the ray's voxel list.
//
// Layout: the smoothed densities are kept in groups of 64 chains, each group
// contiguous and chain-fastest inside: rhat[((c/64) * V + v) * 64 + c%64]
// for V = R*C*n_z voxels.  A wavefront walking one ray for the 64 chains of
// a group reads 64 consecutive values per voxel (256 bytes in float32) while
// the ray's voxel list is the same for every lane.
#pragma once
#include <hip/hip_runtime.h>

#include "device_common.h"

namespace mc {

constexpr int kVoxLanes = 64;          // chains per wavefront
constexpr int kVoxWaves = 4;           // wavefronts per block
constexpr int kVoxRaysPerWave = 4;     // rays one wavefront walks in turn
constexpr int kVoxRaysPerTile = kVoxWaves * kVoxRaysPerWave;
// ray-voxel pieces whose density rows one wavefront has in flight at once;
// the voxel and length lists carry kVoxPad padding entries past their end
// (voxel 0, length 0), so a batch, and the prefetch of the next batch's
// voxel indices, may read past the ray's last piece
constexpr int kVoxBatch = 16;
constexpr int kVoxPad = 2 * kVoxBatch;
// most transposed-list entries one gradient work item (one wavefront) sums:
// a column's list is cut into items of this length, so the columns above the
// sensors, whose lists run to tens of thousands of entries, do not leave one
// wavefront working long after the rest
constexpr int kVoxItemEntries = 1024;
// float32 sigmoids whose argument exceeds this in magnitude are taken as
// exactly 0 or 1: the neglected part, below exp(-30) = 9.4e-14, is far
// under the float32 rounding of the density.
constexpr float kVoxSatF32 = 30.0f;

template <typename T>
struct VoxParams {
    int R, C, N, n_z, M;       // grid, nodes, levels, heights per chain ((S-1)*N)
    int n_chains, n_pad;       // chains, chains rounded up to a multiple of 64
    const T *heights;          // [n][S-1][R][C]
    const T *top;              // [N]
    T *rhat;                   // [n_pad/64][N*n_z][64]
    double dz, inv_gamma;
    double drho[kMaxSurfaces];   // rho_l - rho_{l+1} for units l = 1..S (rho_{S+1} = 0, the air)
    double rho1;
    const double *floor_sig;     // [n_z] sigma(-z_k / gamma): the floor's smooth indicator
    const double *inv_norm;      // [n_z] 1 / (1 - sigma(-z_k / gamma)): 1 / sum_l D_l
    // linearised likelihood
    int n_ray, n_tiles;
    const int *ray_off;          // [n_ray + 1] CSR offsets of the rays' voxel lists
    const int *vox;              // [nnz] voxel index (i*C + j)*n_z + k
    const T *len;                // [nnz] length of the ray inside that voxel (m)
    const double *lam0, *o0;     // [n_ray] lambda_p(R0), O_p(R0)
    const double *cnt;           // [n_ray] observed counts
    double inv_atten;
    double *partials;            // [n][n_tiles] per-chain, per-tile sums of C log(lambda) - lambda
    T *opacity;                  // optional [n][n_ray]: O_p(R-hat)
    const double *only_nan;      // optional [n]: chains whose value is not NaN are skipped
    // gradient (optional)
    T *alpha;                    // [n_pad/64][n_ray][64]: dLL/dO_p = (C_p / lambda-hat_p - 1)(-lambda_p(R0) / Lambda)
    const int *t_off;            // [N*n_z + 1] CSR offsets of the voxels' ray lists (the transpose of G's pattern)
    const int *t_ray;            // [nnz] ray index
    const T *t_len;              // [nnz] length of that ray inside the voxel
    const int *items;            // [n_items][4] gradient work items: column, first level, entry range [eb, ee)
    int n_items;
    unsigned long long *gfix;    // [n][S][N] fixed-point gradient of the likelihood (zeroed, then added into)
};

// A wavefront-uniform read of a list that no kernel of the launch writes,
// through the scalar unit (constant address space).
template <typename T>
__device__ __forceinline__ T vox_uniform(const T *a, int i) {
    return ((const __attribute__((address_space(4))) T *)a)[i];
}

// sigma = 1 / (1 + exp(x)), x = (z - H) / gamma
__device__ __forceinline__ double vox_sigma(double x) { return 1.0 / (1.0 + exp(x)); }
__device__ __forceinline__ float vox_sigma(float x) {
    if (x >= kVoxSatF32) return 0.0f;
    if (x <= -kVoxSatF32) return 1.0f;
    return __builtin_amdgcn_rcpf(1.0f + __expf(x));
}

// R-hat for every voxel of one column and one chain per thread.  Block:
// 256 threads = 4 wavefronts of 64 consecutive chains of one column; grid:
// (column, group of 256 chains).  Writes are 64 consecutive chains per level.
//   R-hat = (sum_{l=1..S} (rho_l - rho_{l+1}) sigma_l - rho_1 sigma_0) / (1 - sigma_0)
// is the normalised mixture sum_l W_l rho_l with the floor (sigma_0) and the
// air (indicator 1) as the outer interfaces, telescoped.
template <typename T, int S>
__global__ __launch_bounds__(256) void k_vox_density(VoxParams<T> P) {
    const int col = blockIdx.x;
    const int c = blockIdx.y * 256 + threadIdx.x;
    if (c >= P.n_pad) return;
    const bool live = c < P.n_chains && !(P.only_nan && !(P.only_nan[c] != P.only_nan[c]));
    T h[S];
#pragma unroll
    for (int l = 0; l < S - 1; ++l) h[l] = live ? P.heights[(size_t)c * P.M + (size_t)l * P.N + col] : T(0);
    h[S - 1] = P.top[col];
    T drho[S];
#pragma unroll
    for (int l = 0; l < S; ++l) drho[l] = (T)P.drho[l];
    const T rho1 = (T)P.rho1, ig = (T)P.inv_gamma, dz = (T)P.dz;
    const size_t V = (size_t)P.N * P.n_z;
    T *out = P.rhat + ((size_t)(c / kVoxLanes) * V + (size_t)col * P.n_z) * kVoxLanes + c % kVoxLanes;
    // float32: the levels [klo, khi] outside which sigma_l saturates (to 1
    // below, 0 above) on every live lane of the wavefront, with a margin of
    // one level; there sigma_l is the constant vox_sigma would return, and
    // the sum is the same bit for bit.  float64 evaluates every sigmoid.
    int klo[S], khi[S];
#pragma unroll
    for (int l = 0; l < S; ++l) {
        klo[l] = INT_MIN;
        khi[l] = INT_MAX;
        if constexpr (std::is_same<T, float>::value) {
            const float lim = (float)P.n_z + 2.0f, w = kVoxSatF32 / ig;   // 30 gamma
            float lo = -lim, hi = lim;   // lanes that are not live widen nothing
            if (live) {
                if (__builtin_isfinite(h[l])) {
                    lo = floorf(fminf(fmaxf((h[l] - w) / dz - 0.5f, -2.0f), lim)) - 1.0f;
                    hi = ceilf(fminf(fmaxf((h[l] + w) / dz - 0.5f, -2.0f), lim)) + 1.0f;
                } else {   // evaluated everywhere, as vox_sigma would
                    lo = -lim - 1.0f;
                    hi = 2.0f * lim;
                }
            }
            klo[l] = __builtin_amdgcn_readfirstlane((int)wave_min(lo));
            khi[l] = __builtin_amdgcn_readfirstlane((int)wave_max(hi));
        }
    }
#pragma unroll 2
    for (int k = 0; k < P.n_z; ++k) {
        const T z = ((T)k + T(0.5)) * dz;
        T acc = -rho1 * (T)P.floor_sig[k];
#pragma unroll
        for (int l = 0; l < S; ++l) {
            const T sg = k < klo[l] ? T(1) : (k > khi[l] ? T(0) : vox_sigma((z - h[l]) * ig));
            acc += drho[l] * sg;
        }
        out[(size_t)k * kVoxLanes] = live ? acc * (T)P.inv_norm[k] : T(0);
    }
}

// Linearised likelihood.  One wavefront walks kVoxRaysPerWave consecutive
// rays for 64 chains (lane = chain); the voxel list of the current ray is
// wavefront-uniform (scalar loads) and each voxel is one 64-chain row of
// rhat.  Block order: chain groups one after another, and within a group
// XCD x takes the contiguous tile range [x*tpx, (x+1)*tpx) (one sensor's
// neighbouring rays per L2), so the blocks in flight read about one group's
// densities, which then stay in the memory-side cache.  Each block writes
// one partial sum per chain, summed over its rays in a fixed order.
template <typename T>
__global__ __launch_bounds__(kVoxWaves * kVoxLanes) void k_vox_lik(VoxParams<T> P) {
    __shared__ double red[kVoxWaves][kVoxLanes];
    const int n_groups = P.n_pad / kVoxLanes;
    const int b = blockIdx.x, x = b % kXcds, k = b / kXcds;
    const int tpx = (P.n_tiles + kXcds - 1) / kXcds;
    const int group = k / tpx, tile = x * tpx + k % tpx;
    if (group >= n_groups || tile >= P.n_tiles) return;
    const int lane = threadIdx.x & (kVoxLanes - 1);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kVoxLanes);
    const int c = group * kVoxLanes + lane;
    const bool live = c < P.n_chains && !(P.only_nan && !(P.only_nan[c] != P.only_nan[c]));
    // the group's rows; a row's 64 values sit at a uniform address plus lane * sizeof(T)
    const T *grp = P.rhat + (size_t)group * P.N * P.n_z * kVoxLanes;
    const unsigned ul = (unsigned)lane;
    auto row_at = [&](int v) -> T { return (grp + (size_t)(unsigned)v * kVoxLanes)[ul]; };
    double tsum = 0.0;
    const int p0 = tile * kVoxRaysPerTile + wave * kVoxRaysPerWave;
    const int p1 = min(p0 + kVoxRaysPerWave, P.n_ray);
    for (int p = p0; p < p1; ++p) {
        const int beg = vox_uniform(P.ray_off, p), end = vox_uniform(P.ray_off, p + 1);
        double o = 0.0;
        // kVoxBatch rows in flight; the last batch of a ray reads padding or
        // the next ray's voxels for its missing pieces and adds nothing of
        // them.  The next batch's voxel indices are loaded while the rows are
        // in flight.
        int vx[kVoxBatch];
#pragma unroll
        for (int u = 0; u < kVoxBatch; ++u) vx[u] = vox_uniform(P.vox, beg + u);
        for (int e = beg; e < end; e += kVoxBatch) {
            T v[kVoxBatch], w[kVoxBatch];
#pragma unroll
            for (int u = 0; u < kVoxBatch; ++u) v[u] = row_at(vx[u]);
#pragma unroll
            for (int u = 0; u < kVoxBatch; ++u) w[u] = vox_uniform(P.len, e + u);
#pragma unroll
            for (int u = 0; u < kVoxBatch; ++u) {
                vx[u] = vox_uniform(P.vox, e + kVoxBatch + u);
                // keeps the load here, ahead of the sums, instead of sunk to the loop's end
                asm volatile("" ::"s"(vx[u]));
            }
            if (e + kVoxBatch <= end) {
#pragma unroll
                for (int u = 0; u < kVoxBatch; ++u) o += (double)(w[u] * v[u]);
            } else {
#pragma unroll
                for (int u = 0; u < kVoxBatch; ++u)
                    if (e + u < end) o += (double)(w[u] * v[u]);
            }
        }
        if (P.opacity && live) P.opacity[(size_t)c * P.n_ray + p] = (T)o;
        const double l0 = vox_uniform(P.lam0, p), cp = vox_uniform(P.cnt, p);
        const double lam = l0 - (o - vox_uniform(P.o0, p)) * (l0 * P.inv_atten);
        tsum += lam > 0.0 ? cp * log(lam) - lam : -__builtin_huge_val();
        if (P.alpha)
            P.alpha[((size_t)group * P.n_ray + p) * kVoxLanes + lane] =
                lam > 0.0 ? (T)((cp / lam - 1.0) * (-l0 * P.inv_atten)) : T(0);
    }
    red[wave][lane] = tsum;
    __syncthreads();
    if (wave == 0 && live) {
        double s = red[0][lane];
#pragma unroll
        for (int w = 1; w < kVoxWaves; ++w) s += red[w][lane];
        P.partials[(size_t)c * P.n_tiles + tile] = s;
    }
}

// Gradient of the linearised likelihood with respect to every height.
// dLL/dRhat_v = sum_p alpha_p L_pv (a gather over voxel v's ray list, the
// transpose of G's pattern), and Rhat of voxel (n, k) depends on column n
// alone: dRhat/dH_l,n = (rho_l - rho_{l+1}) sigma_l (1 - sigma_l) /
// (gamma (1 - sigma_0)).  A column's list entries are contiguous, level
// after level; the list is cut into work items of at most kVoxItemEntries
// entries.  One wavefront per (item, 64-chain group), lane = chain: it sums
// the item's entries level by level (one 64-chain row of alpha per entry,
// kVoxBatch rows in flight, the next batch's ray indices loaded while they
// are in flight; products in T, sums in float64, as in the likelihood) and
// adds each level's sum, times the level's sigmoid
// derivatives, into the S height derivatives.  The gradient is linear in the
// level sums, so a level split between two items contributes its two parts.
// Each item adds its derivatives in the 2^-32 fixed point of the march's
// adjoint to gfix (zeroed beforehand) with integer atomics: exact, so the
// result does not depend on the order of the items.
// Blocks of 4 items, in units of kVoxGradUnit blocks; XCD x takes the units
// u with u % 8 == x of each group in turn: neighbouring columns, which share
// rays, go through one L2, and the heavy columns near the sensors are spread
// over all XCDs.
constexpr int kVoxGradUnit = 16;
template <typename T, int S>
__global__ __launch_bounds__(256) void k_vox_grad(VoxParams<T> P) {
    const int n_ib = (P.n_items + 3) / 4;
    const int upx = (n_ib + kVoxGradUnit * kXcds - 1) / (kVoxGradUnit * kXcds);   // units per XCD
    const int b = blockIdx.x, x = b % kXcds, q = b / kXcds;
    const int group = q / (upx * kVoxGradUnit), j = q % (upx * kVoxGradUnit);
    const int ib = ((j / kVoxGradUnit) * kXcds + x) * kVoxGradUnit + j % kVoxGradUnit;
    if (group >= P.n_pad / kVoxLanes || ib >= n_ib) return;
    const int it = ib * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x / kVoxLanes);
    if (it >= P.n_items) return;
    const int col = vox_uniform(P.items, 4 * it), k0 = vox_uniform(P.items, 4 * it + 1);
    const int eb = vox_uniform(P.items, 4 * it + 2), ee = vox_uniform(P.items, 4 * it + 3);
    const int lane = threadIdx.x & (kVoxLanes - 1);
    const int c = group * kVoxLanes + lane;
    const bool live = c < P.n_chains;
    T h[S];
#pragma unroll
    for (int l = 0; l < S - 1; ++l) h[l] = live ? P.heights[(size_t)c * P.M + (size_t)l * P.N + col] : T(0);
    h[S - 1] = P.top[col];
    double g[S];
#pragma unroll
    for (int l = 0; l < S; ++l) g[l] = 0.0;
    const T ig = (T)P.inv_gamma, dz = (T)P.dz;
    // the group's alpha rows; a row's 64 values sit at a uniform address plus lane * sizeof(T)
    const T *agrp = P.alpha + (size_t)group * P.n_ray * kVoxLanes;
    const unsigned ul = (unsigned)lane;
    auto arow = [&](int r) -> T { return (agrp + (size_t)(unsigned)r * kVoxLanes)[ul]; };
    const int vb = col * P.n_z;
    int k = k0, kend = vox_uniform(P.t_off, vb + k0 + 1);   // level k's entries end at kend
    int ix[kVoxBatch];
#pragma unroll
    for (int u = 0; u < kVoxBatch; ++u) ix[u] = vox_uniform(P.t_ray, eb + u);
    double B = 0.0;
    for (int e = eb; e < ee;) {
        // this batch: entries [e, en) of level k; a partial batch reads padding
        // or the following entries for its missing ones and adds nothing of them
        const int en = min(min(e + kVoxBatch, kend), ee);
        T a[kVoxBatch], w[kVoxBatch];
#pragma unroll
        for (int u = 0; u < kVoxBatch; ++u) a[u] = arow(ix[u]);
#pragma unroll
        for (int u = 0; u < kVoxBatch; ++u) w[u] = vox_uniform(P.t_len, e + u);
#pragma unroll
        for (int u = 0; u < kVoxBatch; ++u) {
            ix[u] = vox_uniform(P.t_ray, en + u);   // the next batch starts at en
            // keeps the load here, ahead of the sums, instead of sunk to the loop's end
            asm volatile("" ::"s"(ix[u]));
        }
        if (en - e == kVoxBatch) {
#pragma unroll
            for (int u = 0; u < kVoxBatch; ++u) B += (double)(a[u] * w[u]);
        } else {
#pragma unroll
            for (int u = 0; u < kVoxBatch; ++u)
                if (u < en - e) B += (double)(a[u] * w[u]);
        }
        if (en == kend || en == ee) {   // level k is complete, or the item ends inside it
            const T z = ((T)k + T(0.5)) * dz;
            const double bn = B * P.inv_gamma * vox_uniform(P.inv_norm, k);
#pragma unroll
            for (int l = 0; l < S; ++l) {
                const double sg = (double)vox_sigma((z - h[l]) * ig);
                g[l] += bn * P.drho[l] * (sg * (1.0 - sg));
            }
            B = 0.0;
            if (en < ee)   // the next level with entries (one exists: the item goes on)
                while (k + 1 < P.n_z) {
                    kend = vox_uniform(P.t_off, vb + (++k) + 1);
                    if (kend > en) break;
                }
        }
        e = en;
    }
    if (!live) return;
#pragma unroll
    for (int l = 0; l < S; ++l) {
        const double sv = fmin(fmax(g[l] * 4294967296.0, -9.0e18), 9.0e18);
        atomicAdd(P.gfix + ((size_t)c * S + l) * P.N + col, (unsigned long long)(long long)__builtin_rint(sv));
    }
}

}  // namespace mc
