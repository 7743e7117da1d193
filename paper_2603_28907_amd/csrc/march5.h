// march5.h -- lean surface-major band walks (float32).
//
// Same quantity and the same boundary-value rule as march3.h (exact
// below-lengths of every surface, paper Sec. 2.1.1), with the per-cell work
// cut down for CDNA wavefronts:
//
//  * cell bookkeeping is incremental (cell indices as floats, byte offsets of
//    the nodes): no integer multiplies in the loop, no step counter;
//  * a piece's end values are bilinear values from lerps with exact end
//    points, with the coordinate across a node line set to exactly 0 or 1, so
//    two cells that share an edge compute the same bits there and agree on
//    every sign;
//  * the in-cell quadratic is solved without branches (hardware reciprocal and
//    square root, 1 ulp each).
//
// Each lane solves the ambiguous pieces of its own ray inline (k_march_lik4).
#pragma once

#include "march3.h"

namespace mc {

__device__ __forceinline__ float raw_sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }

// e^x in float64 for the per-pixel Poisson term (x = -O / Lambda), written
// out: x = k ln2 + r with k = rint(x / ln2) and r = x - k ln2 by Cody and
// Waite's two-part ln 2 (the high part has trailing zero bits, so k times it
// is exact for |k| < 2^21), |r| <= ln2 / 2; e^r by its Taylor series to
// degree 13 (truncation below 1e-17 relative); 2^k by ldexp.  The series
// coefficients 1/n! come from constant memory with scalar loads, so they sit
// in scalar registers (as constants of the ray loop the compiler would keep
// them, and a copy of each per use, in vector registers).
__constant__ double kExpTaylor[12] = {
    1.6059043836821614599e-10, 2.0876756987868098979e-09, 2.5052108385441718775e-08, 2.7557319223985890653e-07,
    2.7557319223985890653e-06, 2.4801587301587301587e-05, 1.9841269841269841270e-04, 1.3888888888888888889e-03,
    8.3333333333333333333e-03, 4.1666666666666666667e-02, 1.6666666666666666667e-01, 0.5};   // 1/n!, n = 13..2

__device__ __forceinline__ double exp_f64(double x) {
    const double k = fmin(fmax(rint(x * 1.4426950408889634074), -1100.0), 1100.0);
    double r = __builtin_fma(-k, 6.93147180369123816490e-01, x);
    r = __builtin_fma(-k, 1.90821492927058770002e-10, r);
    double p = kExpTaylor[0];
#pragma unroll
    for (int i = 1; i < 12; ++i) p = __builtin_fma(p, r, kExpTaylor[i]);
    p = __builtin_fma(p, r, 1.0);
    p = __builtin_fma(p, r, 1.0);
    return ldexp(p, (int)k);
}

// Crossings of one piece in the normalised variable s = tau / tau1, with
// |f'(tau)| at each (for the crossing records of the gradient march).
struct PieceCross {
    int n;
    float s[2], fp[2];
};

// Branch-free below-length of a piece of length tau1 with end values fe, fx
// and curvature c2 of f = z - h (the cases of cell_below_length_fast).
// Solved in the normalised variable s = tau / tau1 on [0, 1]:
//   f(s) = fe + B s + A s^2,  A = c2 tau1^2,  B = fx - fe - A,
// which needs two hardware reciprocals and one square root.  With
// hB = -B / 2 the roots are (hB -+ sqrt(hB^2 - A fe)) / A and the vertex is
// sv = hB / A with f(sv) = fe - hB sv.  The stable root fe / q also covers
// A = 0 (q = -B there: the straight-line crossing).  With REC the crossings
// are reported too: the one root when the end signs differ, else the two
// roots around an interior vertex of the opposite sign; |f'| = |B + 2 A s| / tau1.
template <bool REC = false>
__device__ __forceinline__ float piece_length(float fe, float fx, float c2, float tau1, PieceCross *pc = nullptr) {
    const bool be = fe < 0.f, bx = fx < 0.f;
    const float A = c2 * tau1 * tau1;
    const float B = (fx - fe) - A;
    const float hB = -0.5f * B;
    const float iA = __builtin_amdgcn_rcpf(A);
    // half the square root of the discriminant B^2 - 4 A fe
    const float sq = raw_sqrt(fmaxf(__builtin_fmaf(hB, hB, -(A * fe)), 0.f));
    // one crossing: the stable pair of roots, keep the one nearest [0, 1]
    const float q = hB + (hB <= 0.f ? -sq : sq);
    const float s1 = q * iA, s2 = fe * __builtin_amdgcn_rcpf(q);
    const float d1 = fmaxf(fmaxf(-s1, s1 - 1.f), 0.f);
    const float d2 = fmaxf(fmaxf(-s2, s2 - 1.f), 0.f);
    const float sr = fminf(fmaxf(((d1 < d2) || (d2 != d2)) ? s1 : s2, 0.f), 1.f);
    const float r = sr * tau1;
    const float one = be ? r : tau1 - r;
    // same signs: two crossings around an interior vertex of the opposite sign
    const float sv = hB * iA;
    const float fv = __builtin_fmaf(-sv, hB, fe);
    const bool two = (A != 0.f) && (sv > 0.f) && (sv < 1.f) && ((fv < 0.f) != be);
    const float aiA = fabsf(iA);
    const float sa = fmaxf(__builtin_fmaf(-aiA, sq, sv), 0.f), sb = fminf(__builtin_fmaf(aiA, sq, sv), 1.f);
    const float inner = fmaxf(sb - sa, 0.f) * tau1;
    const float none = be ? tau1 : 0.f;
    const float twol = be ? tau1 - inner : inner;
    if constexpr (REC) {
        const float it1 = __builtin_amdgcn_rcpf(tau1);
        pc->n = (be != bx) ? 1 : (two ? 2 : 0);
        pc->s[0] = (be != bx) ? sr : sa;
        pc->s[1] = sb;
        pc->fp[0] = fabsf(B + 2.f * A * pc->s[0]) * it1;
        pc->fp[1] = fabsf(B + 2.f * A * sb) * it1;
    }
    return (be != bx) ? one : (two ? twol : none);
}

// Bilinear height of a cell at local coordinates (s, w) in [0, 1]^2 from
// lerps with exact end points: lerp(u, v, t) = t v + (u - t u) gives u at
// t = 0 and v at t = 1 exactly.  A piece end on a node line takes that
// coordinate exactly (0 or 1), so there the value is the plain lerp along the
// shared edge, and the two cells that share the edge compute the same bits
// (adjacent cells agree on every sign).
__device__ __forceinline__ float lerp_exact(float u, float v, float t) {
    return __builtin_fmaf(t, v, __builtin_fmaf(-t, u, u));
}

__device__ __forceinline__ float cell_height(float h00, float h01, float h10, float h11, float s, float w) {
    return lerp_exact(lerp_exact(h00, h01, w), lerp_exact(h10, h11, w), s);
}

// Below-length of one piece [t0, t1] of a cell with corner heights h00 (node
// (a, b)), h01 (a, b+1), h10 (a+1, b), h11 (a+1, b+1).  The ray in cell
// units: x / h_x = t dxi + qxi, so the local coordinate is s = t dxi + qxa
// with qxa = qxi - a (w likewise with qyb = qyi - b).  z0, z1: the ray's
// heights at t0, t1 (the walk's own values); enx (eny): the piece starts on
// an x (y) node line, xedge (yedge): it ends on one; kxy = -dxi dyi, the
// ray's factor of the patch curvature.
template <bool REC = false>
__device__ __forceinline__ float solve_cell_piece(float h00, float h01, float h10, float h11, float qxa, float qyb,
                                                  float dxi, float dyi, float kxy, float t0, float t1, float z0,
                                                  float z1, bool enx, bool eny, bool xedge, bool yedge,
                                                  PieceCross *pc = nullptr) {
    const bool xpos = dxi > 0.f, ypos = dyi > 0.f;
    // a walk along +x enters a cell on its row a (s = 0) and leaves on row
    // a + 1 (s = 1); along -x the other way round (w, y likewise)
    const float se = enx ? (xpos ? 0.f : 1.f) : __builtin_fmaf(t0, dxi, qxa);
    const float we = eny ? (ypos ? 0.f : 1.f) : __builtin_fmaf(t0, dyi, qyb);
    const float sx = xedge ? (xpos ? 1.f : 0.f) : __builtin_fmaf(t1, dxi, qxa);
    const float wx = yedge ? (ypos ? 1.f : 0.f) : __builtin_fmaf(t1, dyi, qyb);
    const float fe = z0 - cell_height(h00, h01, h10, h11, se, we);
    const float fx = z1 - cell_height(h00, h01, h10, h11, sx, wx);
    const float c2 = ((h11 - h10) - (h01 - h00)) * kxy;
    return piece_length<REC>(fe, fx, c2, t1 - t0, pc);
}

// Cell walk state (also used by the adjoint).  The cell indices are kept
// as integer-valued floats, so the parameter where the ray leaves a cell
// across an x (y) node line, t = a t_x + o_x, depends only on the cell: a
// walk started at any cell of a ray reproduces the bits of the walk that
// reached that cell.
struct Walk {
    float af, bf;             // cell origin indices (a, b) as floats (exact small integers)
    float tx, ty;             // h_x / d_x, h_y / d_y: parameter step per cell
    float ox, oy;             // parameter of the exit line of cell index 0 in the walk's direction
    float th;                 // end of the walk: the band end, or the grid edge if that comes first
    float gx, gy;             // the index step along x and y (+1 or -1)
    unsigned off, offx, offy; // byte offset of node (a, b) in the surface and its steps (mod 2^32)
    float t0, z0;
    bool enx, eny;            // the current piece starts on an x (y) node line
};

__device__ __forceinline__ float walk_af(const Walk &W) { return W.af; }
__device__ __forceinline__ float walk_bf(const Walk &W) { return W.bf; }

// The ray in cell units: x / h_x = t dxi + qxi, y / h_y = t dyi + qyi.
// ox, oy: the ray's parameter at the node lines x = 0 and y = 0 (+inf for a
// ray parallel to that axis, whose step tx or ty is then 0).
__device__ __forceinline__ Walk walk_init(const MarchParams<float> &P, float qxi, float qyi, float qz, float dxi,
                                          float dyi, float dz, float idx, float idy, float ox, float oy, float tl,
                                          float th) {
    const int R = P.R, C = P.C;
    const bool xpos = dxi > 0.f, ypos = dyi > 0.f;
    int a = (int)floorf(__builtin_fmaf(tl, dxi, qxi)), b = (int)floorf(__builtin_fmaf(tl, dyi, qyi));
    a = a < 0 ? 0 : (a > R - 2 ? R - 2 : a);
    b = b < 0 ? 0 : (b > C - 2 ? C - 2 : b);
    Walk W;
    W.af = (float)a;
    W.bf = (float)b;
    W.tx = P.hx * idx;
    W.ty = P.hy * idy;
    // the exit line of cell a is a + 1 along +x and a along -x
    W.ox = xpos ? ox + W.tx : ox;
    W.oy = ypos ? oy + W.ty : oy;
    // the last cells in the walk's directions are xe = R - 2 or 0 (ye = C - 2
    // or 0), whose exit lines are the grid edge: th is clipped to their
    // parameters.  A step along x needs t(af) < th <= t(xe), so af != xe (equal
    // indices give equal bits): a and b move one by one toward xe and ye and
    // never past them, every cell of the walk is inside the grid, and the walk
    // takes at most R + C - 4 steps
    const float xe = xpos ? (float)(R - 2) : 0.f, ye = ypos ? (float)(C - 2) : 0.f;
    W.th = fminf(th, fminf(__builtin_fmaf(xe, W.tx, W.ox), __builtin_fmaf(ye, W.ty, W.oy)));
    W.gx = xpos ? 1.f : -1.f;
    W.gy = ypos ? 1.f : -1.f;
    W.off = (unsigned)(a * C + b) * 4u;
    W.offx = xpos ? 4u * (unsigned)C : 0u - 4u * (unsigned)C;
    W.offy = ypos ? 4u : 0u - 4u;
    W.t0 = tl;
    W.z0 = __builtin_fmaf(tl, dz, qz);
    W.enx = W.eny = false;
    return W;
}

// One step of a walk: the piece [t0, t1] of the current cell and its
// classification; `edge` says whether the walk continues.
struct Step {
    float t1, z1;
    bool edge, stepx;
};

// Minimum (maximum) of four corner heights in two instructions.  Written in
// assembly because the compiler canonicalizes the loaded operands of a
// two-operand min or max first (two more instructions per cell); the heights
// are finite, for which canonicalizing changes nothing.
__device__ __forceinline__ float min4(float a, float b, float c, float d) {
    float m, r;
    asm("v_min_f32 %0, %1, %2" : "=v"(m) : "v"(c), "v"(d));
    asm("v_min3_f32 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(m));
    return r;
}

__device__ __forceinline__ float max4(float a, float b, float c, float d) {
    float m, r;
    asm("v_max_f32 %0, %1, %2" : "=v"(m) : "v"(c), "v"(d));
    asm("v_max3_f32 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(m));
    return r;
}

// Height of the node `boff` bytes past H (the walk keeps byte offsets: the
// address of a node is one add, with no scaling or base constant per cell).
__device__ __forceinline__ float node_at(const float *H, unsigned boff) {
    return *reinterpret_cast<const float *>(reinterpret_cast<const char *>(H) + boff);
}

__device__ __forceinline__ Step walk_step(const Walk &W, float qz, float dz) {
    Step s;
    const float tnx = __builtin_fmaf(W.af, W.tx, W.ox), tny = __builtin_fmaf(W.bf, W.ty, W.oy);
    s.stepx = tnx <= tny;
    const float tn = s.stepx ? tnx : tny;
    s.edge = tn < W.th;
    // max(min(tn, th), t0) as one median: t0 <= th along the walk, and tn is
    // finite or +inf (an axis-parallel ray has step 0 and offset +inf)
    s.t1 = __builtin_amdgcn_fmed3f(tn, W.th, W.t0);
    s.z1 = __builtin_fmaf(s.t1, dz, qz);
    return s;
}

__device__ __forceinline__ void walk_advance(Walk &W, const Step &s) {
    // value selects (a branch here makes the compiler select between field
    // addresses and keep the walk state in scratch memory)
    const bool sx = s.stepx;
    W.af = sx ? W.af + W.gx : W.af;
    W.bf = sx ? W.bf : W.bf + W.gy;
    W.off += sx ? W.offx : W.offy;
    W.enx = sx;
    W.eny = !sx;
    W.t0 = s.t1;
    W.z0 = s.z1;
}

// Stage the chain's free surfaces (and the top if TOP_LDS) and reduce the
// per-surface bands; prologue of the lean march and its adjoint.
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
// Crossing records (the gradient march)
// ---------------------------------------------------------------------------
// The march that precedes the adjoint records every crossing it solves: per
// (chain, ray tile, surface l) a list per thread, laid out [slot][thread] so
// that a wavefront's lanes write and later read neighbouring records.  One
// record (16 bytes) holds the cell offset a C + b (16 bits), l (2 bits) and
// the slot k of the ray among the thread's rays (ray = tile start + thread +
// k BLOCK; 6 bits), the local coordinates (s, w) of the crossing in the cell
// and 1/|f'| there.  The adjoint then needs no walk: every node
// contribution of the crossing form is (rho_l - rho_{l+1}) g_p w_n / |f'|,
// with g_p = dLL/dO_p, which the march also writes per ray.  A thread whose
// slots of a surface run out sets the chain's overflow flag; the adjoint
// re-walks such chains.
struct CrossRecs {
    uint4 *rec;        // [n_chains][n_tiles][S][slots][BLOCK]
    uint32_t *cnt;     // [n_chains][n_tiles][S][BLOCK] records kept per thread
    int *ovf;          // [n_chains] 1 when some thread's slots ran out (else untouched)
    float *gp;         // [n_chains][n_ray] dLL/dO_p = (lambda_p - C_p) / Lambda
    int slots;         // records per thread and surface
};

// ---------------------------------------------------------------------------
// v4: inline solves
// ---------------------------------------------------------------------------
template <int S, bool TOP_LDS, int BLOCK, bool REC = false>
__device__ __forceinline__ void march_block4(const MarchParams<float> &P, const RayConsts<float> &K, int chain,
                                             int tile, float *sh, const CrossRecs &X = CrossRecs{}) {
    __shared__ double red[16];
    __shared__ float band[2 * kMaxSurfaces];
    const int tid = threadIdx.x;
    if (P.only_nan && !(P.only_nan[chain] != P.only_nan[chain])) return;
    stage_surfaces<S, TOP_LDS, BLOCK>(P, sh, band, chain);
    const int N = P.R * P.C;
    const unsigned C4 = 4u * (unsigned)P.C;
    double acc = 0.0;
    const int r0 = tile * P.rays_per_block;
    const int r1 = min(r0 + P.rays_per_block, P.n_ray);
    // the index of this thread's next record of each surface, in LDS rather
    // than registers (the gradient march is tight on registers at 6 waves per
    // SIMD): record k of surface l goes to (l slots + k) BLOCK + thread
    __shared__ unsigned rec_next[REC ? S : 1][REC ? BLOCK : 1];
    if constexpr (REC) {
#pragma unroll
        for (int l = 0; l < S; ++l) rec_next[l][tid] = (unsigned)(l * X.slots * BLOCK + tid);
    }
    // this block's record lists (a block-uniform base) and this thread's
    // offset inside them: a 32-bit index, no per-lane 64-bit pointer to keep
    uint4 *const recb = X.rec + (size_t)(chain * P.n_tiles + tile) * S * (size_t)X.slots * BLOCK;
    // sensor s and pixel p of the thread's ray, stepped with the ray (no
    // division per ray)
    int s = 0, pix = 0;
    if (r0 + tid < r1) {
        s = (r0 + tid) / P.n_pix;
        pix = r0 + tid - s * P.n_pix;
    }
    for (int ray = r0 + tid; ray < r1; ray += BLOCK) {
        // per-ray tables through 32-bit byte offsets (one address add each)
        const unsigned b4 = 4u * (unsigned)ray;
        const float qz = P.sensor[3 * s + 2], dz = node_at(P.dz, b4);
        // the ray in cell units
        const float qxi = P.sensor[3 * s] * P.ihx, qyi = P.sensor[3 * s + 1] * P.ihy;
        const float dxi = node_at(P.dx, b4) * P.ihx, dyi = node_at(P.dy, b4) * P.ihy;
        const float idx = node_at(K.idx, b4), idy = node_at(K.idy, b4), idz = node_at(K.idz, b4);
        const float ox = node_at(K.ox, b4), oy = node_at(K.oy, b4), Texit = node_at(K.texit, b4);
        const float kxy = -dxi * dyi;
        float O = 0.f;
#pragma unroll
        for (int l = 0; l < S; ++l) {
            const float *Hl = (l < S - 1 || TOP_LDS) ? sh + l * N : P.top;
            const float tl = fminf(fmaxf((band[l] - qz) * idz, 0.f), Texit);
            const float th = fminf(fmaxf((band[kMaxSurfaces + l] - qz) * idz, 0.f), Texit);
            float L = tl;
            if (tl < th) {
                Walk W = walk_init(P, qxi, qyi, qz, dxi, dyi, dz, idx, idy, ox, oy, tl, th);
                // no step counter: the walk ends within R + C - 4 steps (walk_init)
                for (;;) {
                    const Step st = walk_step(W, qz, dz);
                    const float h00 = node_at(Hl, W.off), h01 = node_at(Hl, W.off + 4u);
                    const float h10 = node_at(Hl, W.off + C4), h11 = node_at(Hl, W.off + C4 + 4u);
                    const float hmin = min4(h00, h01, h10, h11), hmax = max4(h00, h01, h10, h11);
                    if (st.z1 < hmin - P.margin) {
                        L += st.t1 - W.t0;
                    } else if (!(W.z0 > hmax + P.margin) && st.t1 > W.t0) {
                        const float qxa = qxi - walk_af(W), qyb = qyi - walk_bf(W);
                        const bool xedge = st.edge && st.stepx, yedge = st.edge && !st.stepx;
                        if constexpr (REC) {
                            PieceCross pc;
                            L += solve_cell_piece<true>(h00, h01, h10, h11, qxa, qyb, dxi, dyi, kxy, W.t0, st.t1, W.z0,
                                                        st.z1, W.enx, W.eny, xedge, yedge, &pc);
                            const float tau1 = st.t1 - W.t0;
                            // at most two crossings: unrolled, so the crossing
                            // data stay in registers (an indexed array would
                            // live in scratch memory)
#pragma unroll
                            for (int k = 0; k < 2; ++k) {
                                if (k >= pc.n) break;
                                const float fp = pc.fp[k];
                                if (!(fp > 0.f)) continue;   // tangency: a kink of lp, no derivative
                                const float t = __builtin_fmaf(pc.s[k], tau1, W.t0);
                                if (__builtin_fmaf(t, dz, qz) >= P.lid) continue;   // the box lid: a kink
                                const float sc = fminf(fmaxf(__builtin_fmaf(t, dxi, qxa), 0.f), 1.f);
                                const float wc = fminf(fmaxf(__builtin_fmaf(t, dyi, qyb), 0.f), 1.f);
                                // the thread and its ray slot follow from the ray index
                                // (ray = r0 + tid + kslot BLOCK): nothing more to keep live
                                const unsigned rr = (unsigned)(ray - r0);
                                const unsigned lane_t = rr % BLOCK, kslot = rr / BLOCK;
                                const unsigned ri = rec_next[l][lane_t];
                                if (ri < (unsigned)((l + 1) * X.slots * BLOCK))
                                    recb[ri] =
                                        make_uint4((W.off >> 2) | ((uint32_t)l << 16) | (kslot << 18),
                                                   __float_as_uint(sc), __float_as_uint(wc),
                                                   __float_as_uint(__builtin_amdgcn_rcpf(fp)));
                                rec_next[l][lane_t] = ri + BLOCK;
                            }
                        } else {
                            L += solve_cell_piece(h00, h01, h10, h11, qxa, qyb, dxi, dyi, kxy, W.t0, st.t1, W.z0,
                                                  st.z1, W.enx, W.eny, xedge, yedge);
                        }
                    }
                    if (!st.edge) break;
                    walk_advance(W, st);
                }
            }
            O += P.rho_diff[l] * L;
        }
        if (P.opacity) P.opacity[(size_t)chain * P.n_ray + ray] = O;
        const double Od = (double)O;
        const double lam = P.expo[ray] * exp_f64(-Od * P.inv_L);
        acc += -P.c_over_L[ray] * Od - lam;
        if constexpr (REC) X.gp[(size_t)chain * P.n_ray + ray] = (float)(lam * P.inv_L - P.c_over_L[ray]);
        pix += BLOCK;
        while (pix >= P.n_pix) {
            pix -= P.n_pix;
            ++s;
        }
    }
    if constexpr (REC) {
        bool over = false;
#pragma unroll
        for (int l = 0; l < S; ++l) {
            const int nr = (int)((rec_next[l][tid] - (unsigned)(l * X.slots * BLOCK + tid)) / BLOCK);
            X.cnt[((size_t)(chain * P.n_tiles + tile) * S + l) * BLOCK + tid] = (uint32_t)min(nr, X.slots);
            over |= nr > X.slots;
        }
        if (over) X.ovf[chain] = 1;
    }
    const double tot = block_sum<BLOCK>(acc, red);
    if (tid == 0) P.partials[(size_t)chain * P.n_tiles + tile] = tot;
}

// Register budget of the march: 8 wavefronts per SIMD (64 VGPRs, which the
// forward march fits without scratch; 512-thread blocks keep the LDS from
// capping residency below that on 64x64 grids).  The gradient march keeps 6
// (80 VGPRs): its record code spills at 64.  1024-thread blocks serve grids
// whose surfaces take most of the LDS (one block, 4 wavefronts per SIMD):
// there the register budget of 4 wavefronts costs no residency.
template <int BLOCK>
constexpr int march_waves_per_simd() { return BLOCK >= 1024 ? 4 : 8; }
template <int BLOCK>
constexpr int march_rec_waves_per_simd() { return BLOCK >= 1024 ? 4 : 6; }

template <int S, bool TOP_LDS, int BLOCK>
__global__ __launch_bounds__(BLOCK, march_waves_per_simd<BLOCK>()) void k_march_lik4(MarchParams<float> P,
                                                                                    RayConsts<float> K) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    int chain, tile;
    if (!xcd_chain_tile(P.n_tiles, P.n_chains, chain, tile)) return;
    march_block4<S, TOP_LDS, BLOCK>(P, K, chain, tile, reinterpret_cast<float *>(smem_raw));
}

// The gradient march: the same walk, plus the crossing records and dLL/dO
// of every ray.
template <int S, bool TOP_LDS, int BLOCK>
__global__ __launch_bounds__(BLOCK, march_rec_waves_per_simd<BLOCK>()) void k_march_rec4(MarchParams<float> P,
                                                                                    RayConsts<float> K, CrossRecs X) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    int chain, tile;
    if (!xcd_chain_tile(P.n_tiles, P.n_chains, chain, tile)) return;
    march_block4<S, TOP_LDS, BLOCK, true>(P, K, chain, tile, reinterpret_cast<float *>(smem_raw), X);
}

}  // namespace mc
