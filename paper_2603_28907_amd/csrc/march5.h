// march5.h -- lean surface-major band walks (float32).
//
// Same quantity and the same boundary-value rule as march.h / march3.h (exact
// below-lengths of every surface, paper Sec. 2.1.1), with the per-cell work
// cut down for CDNA wavefronts:
//
//  * cell bookkeeping is incremental (node-line coordinates, LDS byte offset,
//    remaining cells to the grid edge): no integer multiplies in the loop;
//  * a piece's two end values share the row and column lerps of its patch and
//    are formed with selects, without branches; they are bit-identical to the
//    shared-edge formulas of march.h, so adjacent cells agree on every sign;
//  * the in-cell quadratic is solved without branches (hardware reciprocal and
//    square root, 1 ulp each).
//
// Two ways of running the ambiguous pieces:
//  k_march_lik4 -- solve in the lane that met the piece (v3's structure);
//  k_march_lik5 -- append the piece to a per-wave compacted ring in LDS and
//                  solve 64 pieces at a time, one per lane, so the solver runs
//                  with every lane busy.  A solved length is added to its
//                  owner's 32-bit fixed-point accumulator (2^-20 m per unit)
//                  with an LDS integer atomic: integer addition is
//                  associative, so the result does not depend on which lane
//                  solved what, and repeat runs are bitwise identical.
#pragma once

#include "march3.h"

namespace mc {

__device__ __forceinline__ float raw_sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }

// Branch-free below-length of a piece of length tau1 with end values fe, fx
// and curvature c2 of f = z - h (the cases of cell_below_length).  Solved in
// the normalised variable s = tau / tau1 on [0, 1]:
//   f(s) = fe + B s + A s^2,  A = c2 tau1^2,  B = fx - fe - A,
// which needs two hardware reciprocals and one square root.  The stable root
// fe / q also covers A = 0 (q = -B there: the straight-line crossing).
__device__ __forceinline__ float piece_length(float fe, float fx, float c2, float tau1) {
    const bool be = fe < 0.f, bx = fx < 0.f;
    const float A = c2 * tau1 * tau1;
    const float B = (fx - fe) - A;
    const float iA = __builtin_amdgcn_rcpf(A);
    const float disc = fmaxf(B * B - 4.f * A * fe, 0.f);
    const float sq = raw_sqrt(disc);
    // one crossing: the stable pair of roots, keep the one nearest [0, 1]
    const float q = -0.5f * (B + (B >= 0.f ? sq : -sq));
    const float s1 = q * iA, s2 = fe * __builtin_amdgcn_rcpf(q);
    const float d1 = fmaxf(fmaxf(-s1, s1 - 1.f), 0.f);
    const float d2 = fmaxf(fmaxf(-s2, s2 - 1.f), 0.f);
    const float sr = fminf(fmaxf(((d1 < d2) || (d2 != d2)) ? s1 : s2, 0.f), 1.f);
    const float r = sr * tau1;
    const float one = be ? r : tau1 - r;
    // same signs: two crossings around an interior vertex of the opposite sign
    const float sv = -0.5f * B * iA;
    const float fv = fe + sv * (B + A * sv);
    const bool two = (A != 0.f) && (sv > 0.f) && (sv < 1.f) && ((fv < 0.f) != be);
    const float half = 0.5f * sq * fabsf(iA);
    const float inner = fmaxf(fminf(sv + half, 1.f) - fmaxf(sv - half, 0.f), 0.f) * tau1;
    const float none = be ? tau1 : 0.f;
    const float twol = be ? tau1 - inner : inner;
    return (be != bx) ? one : (two ? twol : none);
}

// f = z - h at a piece end.  kind: 0 point, 1 x-edge, 2 y-edge; `xrow1`
// (`ycol1`) selects the node row a+1 (column b+1) for an x-edge (y-edge).
// Row lerps r0 (row a) and r1 (row a+1) run along w; column lerps c0, c1
// along s; a point uses the bilinear value lerp(r0, r1, s).
struct Patch {
    float h00, h01, h10, h11, dr0, dr1, dc0, dc1;
};

__device__ __forceinline__ Patch make_patch(float h00, float h01, float h10, float h11) {
    Patch p;
    p.h00 = h00;
    p.h01 = h01;
    p.h10 = h10;
    p.h11 = h11;
    p.dr0 = h01 - h00;
    p.dr1 = h11 - h10;
    p.dc0 = h10 - h00;
    p.dc1 = h11 - h01;
    return p;
}

__device__ __forceinline__ float end_value(const Patch &p, int kind, bool xrow1, bool ycol1, float z, float s,
                                           float w) {
    const float r0 = __builtin_fmaf(w, p.dr0, p.h00), r1 = __builtin_fmaf(w, p.dr1, p.h10);
    const float c0 = __builtin_fmaf(s, p.dc0, p.h00), c1 = __builtin_fmaf(s, p.dc1, p.h01);
    const float hx = xrow1 ? r1 : r0;
    const float hy = ycol1 ? c1 : c0;
    const float hp = __builtin_fmaf(s, r1 - r0, r0);
    const float h = kind == kXEdge ? hx : (kind == kYEdge ? hy : hp);
    return z - h;
}

// Below-length of one piece [t0, t1] of cell (af, bf) (cell origin indices
// as floats) of a surface patch.
__device__ __forceinline__ float solve_cell_piece(const Patch &p, float af, float bf, float ihx, float ihy, float qx,
                                                  float qy, float qz, float dx, float dy, float dz, float t0,
                                                  float t1, int ekind, int xkind) {
    const bool xpos = dx > 0.f, ypos = dy > 0.f;
    const float z0 = __builtin_fmaf(t0, dz, qz), z1 = __builtin_fmaf(t1, dz, qz);
    const float se = __builtin_fmaf(__builtin_fmaf(t0, dx, qx), ihx, -af);
    const float we = __builtin_fmaf(__builtin_fmaf(t0, dy, qy), ihy, -bf);
    const float sx = __builtin_fmaf(__builtin_fmaf(t1, dx, qx), ihx, -af);
    const float wx = __builtin_fmaf(__builtin_fmaf(t1, dy, qy), ihy, -bf);
    // entry edge: row a+1 when moving -x, column b+1 when moving -y; exit: the opposite
    const float fe = end_value(p, ekind, !xpos, !ypos, z0, se, we);
    const float fx = end_value(p, xkind, xpos, ypos, z1, sx, wx);
    const float c2 = -(p.dr1 - p.dr0) * (dx * ihx) * (dy * ihy);
    return piece_length(fe, fx, c2, t1 - t0);
}

// Cell walk state shared by the two kernels.
struct Walk {
    float xn, yn, dxn, dyn;   // next node-line coordinates and their steps
    float af, bf;             // cell origin indices as floats
    int off, offx, offy;      // element offset of node (a, b) in the surface and its steps
    int remx, remy;           // cells left before the grid edge along x / y
    float t0, z0;
    int ekind;
};

__device__ __forceinline__ Walk walk_init(const MarchParams<float> &P, float qx, float qy, float qz, float dx,
                                          float dy, float dz, float tl) {
    const int R = P.R, C = P.C;
    const bool xpos = dx > 0.f, ypos = dy > 0.f;
    const float x0 = __builtin_fmaf(tl, dx, qx), y0 = __builtin_fmaf(tl, dy, qy);
    int a = (int)floorf(x0 * P.ihx), b = (int)floorf(y0 * P.ihy);
    a = a < 0 ? 0 : (a > R - 2 ? R - 2 : a);
    b = b < 0 ? 0 : (b > C - 2 ? C - 2 : b);
    Walk W;
    W.xn = (float)(xpos ? a + 1 : a) * P.hx;
    W.yn = (float)(ypos ? b + 1 : b) * P.hy;
    W.dxn = xpos ? P.hx : -P.hx;
    W.dyn = ypos ? P.hy : -P.hy;
    W.af = (float)a;
    W.bf = (float)b;
    W.off = a * C + b;
    W.offx = xpos ? C : -C;
    W.offy = ypos ? 1 : -1;
    W.remx = xpos ? R - 2 - a : a;
    W.remy = ypos ? C - 2 - b : b;
    W.t0 = tl;
    W.z0 = __builtin_fmaf(tl, dz, qz);
    W.ekind = kPoint;
    return W;
}

// One step of a walk: the piece [t0, t1] of the current cell.  Returns
// whether the walk continues; fills the piece and its classification.
struct Step {
    float t1, z1;
    int xkind;
    bool edge, stepx;
};

__device__ __forceinline__ Step walk_step(const Walk &W, float qz, float dz, float idx, float idy, float ox,
                                          float oy, float th) {
    Step s;
    const float tnx = __builtin_fmaf(W.xn, idx, ox), tny = __builtin_fmaf(W.yn, idy, oy);
    s.stepx = tnx <= tny;
    const float tn = s.stepx ? tnx : tny;
    const bool room = s.stepx ? (W.remx > 0) : (W.remy > 0);
    s.edge = (tn < th) && room;
    s.t1 = fmaxf(fminf(tn, th), W.t0);
    s.z1 = __builtin_fmaf(s.t1, dz, qz);
    s.xkind = s.edge ? (s.stepx ? kXEdge : kYEdge) : kPoint;
    return s;
}

__device__ __forceinline__ void walk_advance(Walk &W, const Step &s) {
    // value selects (a branch here makes the compiler select between field
    // addresses and keep the walk state in scratch memory)
    const bool sx = s.stepx;
    W.xn = sx ? W.xn + W.dxn : W.xn;
    W.yn = sx ? W.yn : W.yn + W.dyn;
    W.af = sx ? W.af + (W.dxn > 0.f ? 1.f : -1.f) : W.af;
    W.bf = sx ? W.bf : W.bf + (W.dyn > 0.f ? 1.f : -1.f);
    W.off += sx ? W.offx : W.offy;
    W.remx = sx ? W.remx - 1 : W.remx;
    W.remy = sx ? W.remy : W.remy - 1;
    W.ekind = sx ? kXEdge : kYEdge;
    W.t0 = s.t1;
    W.z0 = s.z1;
}

// Stage the chain's free surfaces (and the top if TOP_LDS) and reduce the
// per-surface bands; common prologue of the lean kernels.
template <int S, bool TOP_LDS, int BLOCK>
__device__ __forceinline__ void stage_surfaces(const MarchParams<float> &P, float *sh, float *band, int chain) {
    const int tid = threadIdx.x, N = P.R * P.C;
    const float *Hc = P.heights + (size_t)chain * (S - 1) * N;
    float mn[S], mx[S];
#pragma unroll
    for (int l = 0; l < S - 1; ++l) {
        float a = __builtin_huge_valf(), b = -__builtin_huge_valf();
        for (int i = tid; i < N; i += BLOCK) {
            float v = Hc[l * N + i];
            sh[l * N + i] = v;
            a = fminf(a, v);
            b = fmaxf(b, v);
        }
        mn[l] = a;
        mx[l] = b;
    }
    if (TOP_LDS) {
        for (int i = tid; i < N; i += BLOCK) sh[(S - 1) * N + i] = P.top[i];
    }
    __shared__ float wred[2 * kMaxSurfaces][BLOCK / kWave];
    const int lane = tid % kWave, wid = tid / kWave;
#pragma unroll
    for (int l = 0; l < S - 1; ++l) {
        float a = wave_min(mn[l]), b = wave_max(mx[l]);
        if (lane == 0) {
            wred[2 * l][wid] = a;
            wred[2 * l + 1][wid] = b;
        }
    }
    __syncthreads();
    if (tid == 0) {
#pragma unroll
        for (int l = 0; l < S - 1; ++l) {
            float a = wred[2 * l][0], b = wred[2 * l + 1][0];
            for (int w = 1; w < BLOCK / kWave; ++w) {
                a = fminf(a, wred[2 * l][w]);
                b = fmaxf(b, wred[2 * l + 1][w]);
            }
            band[l] = a - P.margin;
            band[kMaxSurfaces + l] = b + P.margin;
        }
        band[S - 1] = P.top_min - P.margin;
        band[kMaxSurfaces + S - 1] = P.top_max + P.margin;
    }
    __syncthreads();
}

// ---------------------------------------------------------------------------
// v4: inline solves
// ---------------------------------------------------------------------------
template <int S, bool TOP_LDS, int BLOCK>
__device__ __forceinline__ void march_block4(const MarchParams<float> &P, const RayConsts<float> &K, int chain,
                                             int tile, float *sh) {
    __shared__ double red[16];
    __shared__ float band[2 * kMaxSurfaces];
    const int tid = threadIdx.x;
    if (P.only_nan && !(P.only_nan[chain] != P.only_nan[chain])) return;
    stage_surfaces<S, TOP_LDS, BLOCK>(P, sh, band, chain);
    const int N = P.R * P.C, C = P.C;
    double acc = 0.0;
    const int r0 = tile * P.rays_per_block;
    const int r1 = min(r0 + P.rays_per_block, P.n_ray);
    for (int ray = r0 + tid; ray < r1; ray += BLOCK) {
        const int s = ray / P.n_pix;
        const float qx = P.sensor[3 * s], qy = P.sensor[3 * s + 1], qz = P.sensor[3 * s + 2];
        const float dx = P.dx[ray], dy = P.dy[ray], dz = P.dz[ray];
        const float idx = K.idx[ray], idy = K.idy[ray], idz = K.idz[ray];
        const float ox = K.ox[ray], oy = K.oy[ray], Texit = K.texit[ray];
        float O = 0.f;
#pragma unroll
        for (int l = 0; l < S; ++l) {
            const float *Hl = (l < S - 1 || TOP_LDS) ? sh + l * N : P.top;
            const float tl = fminf(fmaxf((band[l] - qz) * idz, 0.f), Texit);
            const float th = fminf(fmaxf((band[kMaxSurfaces + l] - qz) * idz, 0.f), Texit);
            float L = tl;
            if (tl < th) {
                Walk W = walk_init(P, qx, qy, qz, dx, dy, dz, tl);
                for (int it = 0; it < P.R + P.C; ++it) {
                    const Step st = walk_step(W, qz, dz, idx, idy, ox, oy, th);
                    const float h00 = Hl[W.off], h01 = Hl[W.off + 1], h10 = Hl[W.off + C], h11 = Hl[W.off + C + 1];
                    const float hmin = fminf(fminf(h00, h01), fminf(h10, h11));
                    const float hmax = fmaxf(fmaxf(h00, h01), fmaxf(h10, h11));
                    if (st.z1 < hmin - P.margin) {
                        L += st.t1 - W.t0;
                    } else if (!(W.z0 > hmax + P.margin) && st.t1 > W.t0) {
                        const Patch pt = make_patch(h00, h01, h10, h11);
                        L += solve_cell_piece(pt, W.af, W.bf, P.ihx, P.ihy, qx, qy, qz, dx, dy, dz, W.t0, st.t1,
                                              W.ekind, st.xkind);
                    }
                    if (!st.edge) break;
                    walk_advance(W, st);
                }
            }
            O += P.rho_diff[l] * L;
        }
        if (P.opacity) P.opacity[(size_t)chain * P.n_ray + ray] = O;
        const double Od = (double)O;
        acc += -P.c_over_L[ray] * Od - P.expo[ray] * exp(-Od * P.inv_L);
    }
    const double tot = block_sum<BLOCK>(acc, red);
    if (tid == 0) P.partials[(size_t)chain * P.n_tiles + tile] = tot;
}

// At least 6 wavefronts per SIMD: the walk is latency-bound, and 6 resident
// waves beat 5 even with a few registers spilled (512-thread blocks keep the
// LDS from capping residency below 6 on 64x64 grids).
constexpr int kMarchWavesPerSimd = 6;

template <int S, bool TOP_LDS, int BLOCK>
__global__ __launch_bounds__(BLOCK, kMarchWavesPerSimd) void k_march_lik4(MarchParams<float> P, RayConsts<float> K) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    int chain, tile;
    if (!xcd_chain_tile(P.n_tiles, P.n_chains, chain, tile)) return;
    march_block4<S, TOP_LDS, BLOCK>(P, K, chain, tile, reinterpret_cast<float *>(smem_raw));
}

// ---------------------------------------------------------------------------
// v5: compacted per-wave solve ring
// ---------------------------------------------------------------------------
constexpr int kRing = 128;                 // ring slots per wave (>= 2 x 64)
constexpr float kFixScale = 1048576.f;     // 2^20 fixed-point units per metre
constexpr float kFixInv = 1.f / 1048576.f;

// LDS layout per wave: ring of (t0, t1, packed) and S x 64 accumulators.
struct WaveRing {
    float *t0, *t1;
    uint32_t *pk;
    uint32_t *acc;   // [S][64]
};

// packed: a (8) | b << 8 | ekind << 16 | xkind << 18 | l << 20 | owner lane << 24
template <int S, bool TOP_LDS>
__device__ __forceinline__ void ring_solve(const MarchParams<float> &P, const float *sh, const WaveRing &rg,
                                           int head, int n, float qx, float qy, float qz, float dx, float dy,
                                           float dz) {
    const int lane = threadIdx.x % kWave;
    const int slot = (head + lane) & (kRing - 1);
    const float t0 = rg.t0[slot], t1 = rg.t1[slot];
    const uint32_t pk = rg.pk[slot];
    const int owner = (int)(pk >> 24);
    // the owner's ray (every lane takes part in the shuffles)
    const float oqx = __shfl(qx, owner, kWave), oqy = __shfl(qy, owner, kWave), oqz = __shfl(qz, owner, kWave);
    const float odx = __shfl(dx, owner, kWave), ody = __shfl(dy, owner, kWave), odz = __shfl(dz, owner, kWave);
    if (lane < n) {
        const int a = pk & 0xFF, b = (pk >> 8) & 0xFF, ek = (pk >> 16) & 3, xk = (pk >> 18) & 3;
        const int l = (pk >> 20) & 0xF;
        const int C = P.C, N = P.R * C;
        const float *Hl = (TOP_LDS || l < S - 1) ? sh + l * N : P.top;
        const int off = a * C + b;
        const Patch pt = make_patch(Hl[off], Hl[off + 1], Hl[off + C], Hl[off + C + 1]);
        const float len = solve_cell_piece(pt, (float)a, (float)b, P.ihx, P.ihy, oqx, oqy, oqz, odx, ody, odz, t0, t1,
                                           ek, xk);
        const uint32_t fix = (uint32_t)(fminf(len, 4000.f) * kFixScale + 0.5f);
        atomicAdd(&rg.acc[l * kWave + owner], fix);
    }
}

template <int S, bool TOP_LDS, int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_march_lik5(MarchParams<float> P, RayConsts<float> K) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    float *sh = reinterpret_cast<float *>(smem_raw);
    __shared__ double red[16];
    __shared__ float band[2 * kMaxSurfaces];
    constexpr int NW = BLOCK / kWave;
    __shared__ float ring_t0[NW][kRing], ring_t1[NW][kRing];
    __shared__ uint32_t ring_pk[NW][kRing];
    __shared__ uint32_t ring_acc[NW][S * kWave];
    const int tid = threadIdx.x;
    int chain, tile;
    if (!xcd_chain_tile(P.n_tiles, P.n_chains, chain, tile)) return;
    if (P.only_nan && !(P.only_nan[chain] != P.only_nan[chain])) return;
    stage_surfaces<S, TOP_LDS, BLOCK>(P, sh, band, chain);
    const int wid = tid / kWave, lane = tid % kWave;
    WaveRing rg{ring_t0[wid], ring_t1[wid], ring_pk[wid], ring_acc[wid]};
#pragma unroll
    for (int l = 0; l < S; ++l) rg.acc[l * kWave + lane] = 0u;
    const int N = P.R * P.C, C = P.C;
    double acc = 0.0;
    const int r0 = tile * P.rays_per_block;
    const int r1 = min(r0 + P.rays_per_block, P.n_ray);
    // every lane of the wave loops over the same number of ray slots
    const int n_slots = (P.rays_per_block + BLOCK - 1) / BLOCK;
    int head = 0, count = 0;   // wave-uniform ring state
    for (int k = 0; k < n_slots; ++k) {
        const int ray = r0 + k * BLOCK + tid;
        const bool live = ray < r1;
        const int rr = live ? ray : r0;
        const int s = rr / P.n_pix;
        const float qx = P.sensor[3 * s], qy = P.sensor[3 * s + 1], qz = P.sensor[3 * s + 2];
        const float dx = P.dx[rr], dy = P.dy[rr], dz = P.dz[rr];
        const float idx = K.idx[rr], idy = K.idy[rr], idz = K.idz[rr];
        const float ox = K.ox[rr], oy = K.oy[rr], Texit = K.texit[rr];
        float L[S];
#pragma unroll
        for (int l = 0; l < S; ++l) {
            const float *Hl = (l < S - 1 || TOP_LDS) ? sh + l * N : P.top;
            const float tl = fminf(fmaxf((band[l] - qz) * idz, 0.f), Texit);
            const float th = fminf(fmaxf((band[kMaxSurfaces + l] - qz) * idz, 0.f), Texit);
            float Ll = tl;
            bool done = !(tl < th) || !live;
            Walk W = walk_init(P, qx, qy, qz, dx, dy, dz, tl);
            for (int it = 0; it < P.R + P.C && __any(!done); ++it) {
                bool amb = false;
                Step st;
                if (!done) {
                    st = walk_step(W, qz, dz, idx, idy, ox, oy, th);
                    const float h00 = Hl[W.off], h01 = Hl[W.off + 1], h10 = Hl[W.off + C], h11 = Hl[W.off + C + 1];
                    const float hmin = fminf(fminf(h00, h01), fminf(h10, h11));
                    const float hmax = fmaxf(fmaxf(h00, h01), fmaxf(h10, h11));
                    if (st.z1 < hmin - P.margin) Ll += st.t1 - W.t0;
                    else amb = !(W.z0 > hmax + P.margin) && st.t1 > W.t0;
                }
                // append the ambiguous pieces of this step to the wave's ring
                const uint64_t mask = __ballot(amb);
                if (amb) {
                    const int pos = (head + count + (int)__builtin_amdgcn_mbcnt_hi(
                                                           (uint32_t)(mask >> 32),
                                                           __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u))) &
                                    (kRing - 1);
                    rg.t0[pos] = W.t0;
                    rg.t1[pos] = st.t1;
                    rg.pk[pos] = (uint32_t)(int)W.af | ((uint32_t)(int)W.bf << 8) | ((uint32_t)W.ekind << 16) |
                                 ((uint32_t)st.xkind << 18) | ((uint32_t)l << 20) | ((uint32_t)lane << 24);
                }
                count += __popcll(mask);
                if (count >= kWave) {
                    ring_solve<S, TOP_LDS>(P, sh, rg, head, kWave, qx, qy, qz, dx, dy, dz);
                    head = (head + kWave) & (kRing - 1);
                    count -= kWave;
                }
                if (!done) {
                    if (!st.edge) done = true;
                    else walk_advance(W, st);
                }
            }
            L[l] = Ll;
        }
        // drain what is left for this ray, then fold the accumulators in
        if (count > 0) {
            ring_solve<S, TOP_LDS>(P, sh, rg, head, count, qx, qy, qz, dx, dy, dz);
            head = (head + count) & (kRing - 1);
            count = 0;
        }
        // the other lanes' LDS atomics on this lane's accumulators are done
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
        float O = 0.f;
#pragma unroll
        for (int l = 0; l < S; ++l) {
            const uint32_t fx = rg.acc[l * kWave + lane];
            rg.acc[l * kWave + lane] = 0u;
            O += P.rho_diff[l] * (L[l] + (float)fx * kFixInv);
        }
        if (live) {
            if (P.opacity) P.opacity[(size_t)chain * P.n_ray + ray] = O;
            const double Od = (double)O;
            acc += -P.c_over_L[ray] * Od - P.expo[ray] * exp(-Od * P.inv_L);
        }
    }
    const double tot = block_sum<BLOCK>(acc, red);
    if (tid == 0) P.partials[(size_t)chain * P.n_tiles + tile] = tot;
}

}  // namespace mc
