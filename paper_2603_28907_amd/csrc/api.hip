// api.hip -- host side of the muoncave C ABI (include/muoncave.h): handle,
// validation, float64 precompute, device uploads, kernel launches and the
// graph-captured MCMC loop.  One translation unit; device code lives in the
// headers it includes.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <type_traits>
#include <vector>

#include "muoncave.h"
#include "march3.h"
#include "march5.h"
#include "adjoint.h"
#include "multi.h"
#include "prior.h"
#include "probe.h"
#include "voxel.h"
#include "quad.h"
#include "nuts.h"
#include "latent.h"

using namespace mc;

// Workspace of logpost_batch_noalloc: the per-(chain, ray tile) partial sums
// of the likelihood, [n_chains][n_tiles] float64.  Every device the library
// runs on holds its own copy until the process ends.  Host code never uses
// this name as an address: mc_create resolves the device address once per
// device with hipGetSymbolAddress and keeps it in g_scratch_ptr.
constexpr size_t kScratchDoubles = 131072;   // 1 MiB
static __device__ __align__(256) double scratch[kScratchDoubles];

namespace {

std::mutex g_scratch_mu;
std::map<int, double *> g_scratch_ptr;   // device -> address of its `scratch`

constexpr int kPriorBlock = 256;
constexpr int kMaxNodes = 16384;   // n_rows * n_cols limit (prior workspace lives in LDS)

std::string g_create_error;

struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
};

struct GraphKey {
    int n = -1, kernel = -1, G = 0;
    const void *heights = nullptr, *lp = nullptr, *acc = nullptr, *inv_mass = nullptr;
    const void *r_state = nullptr, *acc_r = nullptr;
    double step_size = 0, r_step = 0;
    uint64_t seed = 0;
    bool operator==(const GraphKey &o) const {
        return n == o.n && kernel == o.kernel && G == o.G && heights == o.heights && lp == o.lp &&
               acc == o.acc && inv_mass == o.inv_mass && step_size == o.step_size && seed == o.seed &&
               r_state == o.r_state && acc_r == o.acc_r && r_step == o.r_step;
    }
};

}  // namespace

// Default launch shape by precision and grid size (measured on MI355X):
// float32 uses the lean band walks; from 48x48 nodes 512-thread blocks let
// 6 wavefronts per SIMD stay resident under the LDS the surfaces take; grids
// of 128x128 nodes and more hold the free surfaces in 128 KB of LDS, one block
// per compute unit, so they take 1024-thread blocks.
static mc_tuning default_tuning(int prec, size_t n_nodes) {
    if (prec == MC_F64) return mc_tuning{3, 256, 4, 1, 0, 0, 0};
    if (n_nodes >= 128 * 128) return mc_tuning{4, 1024, 16, 0, 0, 0, 0};
    if (n_nodes >= 48 * 48) return mc_tuning{4, 512, 16, 0, 0, 0, 0};
    return mc_tuning{4, 256, 8, 0, 0, 0, 0};
}

struct mc_problem {
    int device = 0;
    int prec = MC_F32;
    std::string err;
    size_t max_lds = 65536;
    bool have_geom = false, have_sensors = false, have_counts = false;
    // geometry
    int S = 0, R = 0, C = 0;
    double X = 0, Y = 0, ztop = 0, top_min = 0, top_max = 0;
    double sum_log_top = 0;   // sum of log(top) over the nodes, in node order
    std::vector<double> density, top, car_r, logdet, s11;
    void *d_top = nullptr;      // [N] in prec
    double *d_eig_g = nullptr, *d_eig_w = nullptr;   // distinct torus eigenvalue terms, multiplicities
    int n_eig = 0;
    double *d_top64 = nullptr;  // [N] f64
    // sensors
    int n_s = 0, n_pix = 0, n_ray = 0;
    double atten = 1.0;
    std::vector<double> pos, dirs, expo;
    void *d_sensor = nullptr, *d_dx = nullptr, *d_dy = nullptr, *d_dz = nullptr;
    double *d_expo = nullptr, *d_coL = nullptr;
    void *d_rc[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};   // per-ray constants
    double kconst = 0.0;
    double *d_cnt64 = nullptr;   // [n_ray] counts as f64
    double kconst_vox = 0.0;     // -sum lgamma(C + 1)
    // the paper's smoothed voxel model (vox_nz = 0: exact march)
    int vox_nz = 0;
    double vox_gamma = 1.0, vox_dz = 0.0;
    std::vector<double> vox_drho;   // [S] rho_l - rho_{l+1}
    int *d_vox_off = nullptr, *d_vox_idx = nullptr;
    void *d_vox_len = nullptr;   // [nnz] in prec
    int *d_vox_toff = nullptr, *d_vox_tray = nullptr;   // the transpose: rays of each voxel
    int *d_vox_items = nullptr;  // [vox_n_items][4] gradient work items over the transposed lists
    int vox_n_items = 0;
    void *d_vox_tlen = nullptr;  // [nnz] in prec
    DevBuf valpha;               // [n_pad/64][n_ray][64] dLL/dO of the voxel model (gradient)
    double *d_vox_lam0 = nullptr, *d_vox_o0 = nullptr, *d_vox_fsig = nullptr, *d_vox_inorm = nullptr;
    size_t vox_nnz = 0;
    DevBuf rhat;   // [R*C*n_z][n_pad] smoothed densities of the chains
    // solid-angle pixels (quad_nsub = 0: one ray per pixel)
    int quad_nsub = 0, quad_npx = 0, quad_ntab = 0;
    double quad_omax = 0.0, kconst_quad = 0.0;
    double *d_quad_w = nullptr, *d_quad_tab = nullptr, *d_quad_cnt = nullptr;
    DevBuf nutsbuf;   // NUTS trees, proposals and warm-up accumulators
    // workspaces (grow only)
    DevBuf partials, prop, lptmp;
    DevBuf rstat;   // [2][n][S-1] sum w^2 and edge sums of the current states (r sampling)
    DevBuf obuf, gfix, gcur, gprop, lpprop;   // gradient and MALA workspaces
    DevBuf xrec, xcnt, xovf, xgp;   // crossing records of the float32 gradient march
    uint64_t *d_step = nullptr;
    mc_tuning tune = {3, 256, 4, 1, 0, 0, 0};
    bool tune_user = false;   // launch shape set through mc_set_tuning (else chosen per grid)
    uint64_t gen = 1;   // bumped whenever device pointers or baked constants change
    // graph cache
    hipStream_t cap_stream = nullptr;
    hipGraphExec_t gexec = nullptr;
    GraphKey gkey;
};

namespace {

struct DeviceGuard {
    int old = -1;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&old) != hipSuccess) old = -1;
        if (old != dev) (void)hipSetDevice(dev);
    }
    ~DeviceGuard() {
        int cur = -1;
        if (old >= 0 && hipGetDevice(&cur) == hipSuccess && cur != old) (void)hipSetDevice(old);
    }
};

mc_status fail(mc_problem *p, mc_status s, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    if (p) p->err = buf;
    else g_create_error = buf;
    return s;
}

#define HIP_TRY(p, expr)                                                                         \
    do {                                                                                         \
        hipError_t e_ = (expr);                                                                  \
        if (e_ != hipSuccess)                                                                    \
            return fail((p), e_ == hipErrorOutOfMemory ? MC_ERR_NOMEM : MC_ERR_DEVICE, "%s: %s", \
                        #expr, hipGetErrorString(e_));                                           \
    } while (0)

void free_ptr(void *&ptr) {
    if (ptr) (void)hipFree(ptr);
    ptr = nullptr;
}
void free_ptr(double *&ptr) {
    if (ptr) (void)hipFree(ptr);
    ptr = nullptr;
}

void drop_graph(mc_problem *p) {
    if (p->gexec) (void)hipGraphExecDestroy(p->gexec);
    p->gexec = nullptr;
    p->gkey = GraphKey();
    p->gen += 1;
}

void clear_quadrature(mc_problem *p) {
    if (p->quad_nsub > 0) drop_graph(p);
    p->quad_nsub = p->quad_npx = p->quad_ntab = 0;
    for (double **q : {&p->d_quad_w, &p->d_quad_tab, &p->d_quad_cnt}) free_ptr(*q);
}

void clear_voxel_model(mc_problem *p) {
    if (p->vox_nz > 0) drop_graph(p);
    p->vox_nz = 0;
    p->vox_nnz = 0;
    free_ptr(p->d_vox_len);
    free_ptr(p->d_vox_tlen);
    for (double **q : {&p->d_vox_lam0, &p->d_vox_o0, &p->d_vox_fsig, &p->d_vox_inorm}) free_ptr(*q);
    p->vox_n_items = 0;
    for (int **q : {&p->d_vox_off, &p->d_vox_idx, &p->d_vox_toff, &p->d_vox_tray, &p->d_vox_items}) {
        if (*q) (void)hipFree(*q);
        *q = nullptr;
    }
}

// Grow-only workspace.  A reallocation invalidates the cached graph, whose
// kernel nodes hold the old pointers.
mc_status ensure(mc_problem *p, DevBuf &b, size_t bytes) {
    if (b.bytes >= bytes) return MC_OK;
    drop_graph(p);
    if (b.p) (void)hipFree(b.p);
    b.p = nullptr;
    b.bytes = 0;
    HIP_TRY(p, hipMalloc(&b.p, bytes));
    b.bytes = bytes;
    return MC_OK;
}

template <typename T>
mc_status upload(mc_problem *p, void *&dst, const std::vector<double> &src) {
    free_ptr(dst);
    if (src.empty()) return MC_OK;
    std::vector<T> tmp(src.begin(), src.end());
    HIP_TRY(p, hipMalloc(&dst, sizeof(T) * tmp.size()));
    HIP_TRY(p, hipMemcpy(dst, tmp.data(), sizeof(T) * tmp.size(), hipMemcpyHostToDevice));
    return MC_OK;
}

mc_status upload_prec(mc_problem *p, void *&dst, const std::vector<double> &src) {
    return p->prec == MC_F64 ? upload<double>(p, dst, src) : upload<float>(p, dst, src);
}

size_t elem_size(const mc_problem *p) { return p->prec == MC_F64 ? 8 : 4; }

// Eigenvalues of Q = diag(A1) - rA on the periodic R x C grid are
// mu_km = 4 - 2r(cos(2 pi k/R) + cos(2 pi m/C)); log det Q is their log-sum
// and Sigma_11 their mean inverse (the diagonal of Q^-1 is constant).
void torus_car_constants(int R, int C, double r, double &logdet, double &s11) {
    const double two_pi = 6.283185307179586476925286766559;
    std::vector<double> cr(R), cc(C);
    for (int k = 0; k < R; ++k) cr[k] = std::cos(two_pi * k / R);
    for (int m = 0; m < C; ++m) cc[m] = std::cos(two_pi * m / C);
    long double sl = 0, si = 0;
    for (int k = 0; k < R; ++k)
        for (int m = 0; m < C; ++m) {
            double mu = 4.0 - 2.0 * r * (cr[k] + cc[m]);
            sl += std::log(mu);
            si += 1.0 / mu;
        }
    logdet = (double)sl;
    s11 = (double)(si / ((long double)R * C));
}

// ---------------------------------------------------------------------------
// Launch helpers
// ---------------------------------------------------------------------------

struct Tiling {
    int rays_per_block, n_tiles;
};

Tiling tiling(const mc_problem *p) {
    Tiling t;
    if (p->vox_nz > 0) {
        t.rays_per_block = kVoxRaysPerTile;
        t.n_tiles = p->n_ray > 0 ? (p->n_ray + kVoxRaysPerTile - 1) / kVoxRaysPerTile : 0;
        return t;
    }
    t.rays_per_block = p->tune.block * p->tune.rays_per_thread;
    t.n_tiles = p->n_ray > 0 ? (p->n_ray + t.rays_per_block - 1) / t.rays_per_block : 0;
    return t;
}

// Partial sums per chain of the likelihood stage the prior kernel adds up:
// the march's tiles, or the voxel or solid-angle pixel kernels'.
int lik_tiles(const mc_problem *p) {
    if (p->quad_nsub > 0) return (p->quad_npx + 255) / 256;
    return tiling(p).n_tiles;
}

// Slots the partials buffer needs per chain (the march writes its own tiles
// before the pixel kernel writes its).
int partial_slots(const mc_problem *p) { return std::max(tiling(p).n_tiles, lik_tiles(p)); }

bool top_in_lds(const mc_problem *p) {
    size_t N = (size_t)p->R * p->C;
    if (!p->tune.top_in_lds) return false;
    return ((N * p->S * elem_size(p) + 15) & ~(size_t)15) + 4096 <= p->max_lds;
}

template <typename T>
RayConsts<T> ray_consts(const mc_problem *p) {
    RayConsts<T> K;
    K.idx = (const T *)p->d_rc[0];
    K.idy = (const T *)p->d_rc[1];
    K.idz = (const T *)p->d_rc[2];
    K.ox = (const T *)p->d_rc[3];
    K.oy = (const T *)p->d_rc[4];
    K.texit = (const T *)p->d_rc[5];
    return K;
}

template <typename T, int S, bool TL, int B>
hipError_t launch_v3_shape(dim3 grid, size_t lds, hipStream_t st, const MarchParams<T> &P, const RayConsts<T> &K) {
    auto k = k_march_lik3<T, S, TL, B>;
    if (lds > 65536) (void)hipFuncSetAttribute((const void *)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL(k, grid, dim3(B), lds, st, P, K);
    return hipGetLastError();
}

template <typename T, int S, bool TL>
hipError_t launch_v3(int block, dim3 grid, size_t lds, hipStream_t st, const MarchParams<T> &P, const RayConsts<T> &K) {
    if constexpr (std::is_same<T, double>::value) {
        return launch_v3_shape<T, S, TL, 256>(grid, lds, st, P, K);
    } else {
        if (block == 256) return launch_v3_shape<T, S, TL, 256>(grid, lds, st, P, K);
        if (block == 512) return launch_v3_shape<T, S, TL, 512>(grid, lds, st, P, K);
        return launch_v3_shape<T, S, TL, 1024>(grid, lds, st, P, K);
    }
}

template <int S, bool TL, int B>
hipError_t launch_v4_shape(dim3 grid, size_t lds, hipStream_t st, const MarchParams<float> &P,
                           const RayConsts<float> &K) {
    auto k = k_march_lik4<S, TL, B>;
    if (lds > 65536) (void)hipFuncSetAttribute((const void *)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL(k, grid, dim3(B), lds, st, P, K);
    return hipGetLastError();
}

template <int S, bool TL>
hipError_t launch_v4(int block, dim3 grid, size_t lds, hipStream_t st, const MarchParams<float> &P,
                     const RayConsts<float> &K) {
    if (block == 256) return launch_v4_shape<S, TL, 256>(grid, lds, st, P, K);
    if (block == 512) return launch_v4_shape<S, TL, 512>(grid, lds, st, P, K);
    return launch_v4_shape<S, TL, 1024>(grid, lds, st, P, K);
}

template <typename T>
MarchParams<T> march_params(const mc_problem *p, const T *heights, T *opacity, double *partials) {
    MarchParams<T> P;
    Tiling t = tiling(p);
    P.R = p->R;
    P.C = p->C;
    P.n_ray = p->n_ray;
    P.n_pix = p->n_pix;
    P.n_tiles = t.n_tiles;
    P.rays_per_block = t.rays_per_block;
    P.hx = (T)(p->X / (p->R - 1));
    P.hy = (T)(p->Y / (p->C - 1));
    P.ihx = (T)((p->R - 1) / p->X);
    P.ihy = (T)((p->C - 1) / p->Y);
    P.xmax = (T)(p->R - 1) * P.hx;
    P.ymax = (T)(p->C - 1) * P.hy;
    P.ztop = (T)p->ztop;
    // rounding margin for the certain-below / certain-above tests
    double eps = sizeof(T) == 4 ? 1.1920929e-07 : 2.220446049250313e-16;
    double zscale = std::fabs(p->ztop) + std::fabs(p->top_min) + 1.0;
    P.margin = (T)(256.0 * eps * zscale);
    // the lid band of the gradient: 16 float32 ulps below the lid (a crossing
    // there is within the float32 rounding of the lid's kink); float64: the margin
    P.lid = sizeof(T) == 4 ? (T)((float)p->ztop - 16.0f * (std::nextafter((float)p->ztop, 1e30f) - (float)p->ztop))
                           : (T)(p->ztop - 256.0 * eps * zscale);
    P.top_min = (T)p->top_min;
    P.top_max = (T)p->top_max;
    for (int l = 0; l < kMaxSurfaces; ++l) {
        double here = l < p->S ? p->density[l] : 0.0;
        double above = l + 1 < p->S ? p->density[l + 1] : 0.0;
        P.rho_diff[l] = (T)(here - above);
    }
    P.sensor = (const T *)p->d_sensor;
    P.dx = (const T *)p->d_dx;
    P.dy = (const T *)p->d_dy;
    P.dz = (const T *)p->d_dz;
    P.c_over_L = p->d_coL;
    P.expo = p->d_expo;
    P.inv_L = 1.0 / p->atten;
    P.top = (const T *)p->d_top;
    P.heights = heights;
    P.opacity = opacity;
    P.partials = partials;
    P.only_nan = nullptr;
    P.n_chains = 0;
    return P;
}

template <typename T, int S>
mc_status launch_march(mc_problem *p, int n, const T *heights, T *opacity, double *partials, hipStream_t st,
                       const double *only_nan = nullptr) {
    MarchParams<T> P = march_params<T>(p, heights, opacity, partials);
    P.only_nan = only_nan;
    P.n_chains = n;
    // XCD-aware 1-D grid (see xcd_chain_tile)
    const dim3 grid((unsigned)P.n_tiles * (unsigned)((n + kXcds - 1) / kXcds * kXcds));
    size_t N = (size_t)p->R * p->C;
    bool tl = top_in_lds(p);
    int variant = p->tune.march_variant;
    if (variant == 4 && sizeof(T) != 4) variant = 3;   // the lean walk is float32 only
    if (variant == 4) {
        size_t lds = N * (tl ? S : S - 1) * sizeof(T);
        if (lds + 16384 > p->max_lds) {
            tl = false;
            lds = N * (S - 1) * sizeof(T);
        }
        if (lds + 16384 > p->max_lds) return fail(p, MC_ERR_UNSUPPORTED, "grid %dx%d too large for LDS", p->R, p->C);
        if constexpr (std::is_same<T, float>::value) {
            RayConsts<float> K = ray_consts<float>(p);
            hipError_t e = tl ? launch_v4<S, true>(p->tune.block, grid, lds, st, P, K)
                              : launch_v4<S, false>(p->tune.block, grid, lds, st, P, K);
            HIP_TRY(p, e);
        }
        return MC_OK;
    }
    size_t lds = N * (tl ? S : S - 1) * sizeof(T);
    if (lds + 2048 > p->max_lds) return fail(p, MC_ERR_UNSUPPORTED, "grid %dx%d too large for LDS", p->R, p->C);
    RayConsts<T> K = ray_consts<T>(p);
    hipError_t e = tl ? launch_v3<T, S, true>(p->tune.block, grid, lds, st, P, K)
                      : launch_v3<T, S, false>(p->tune.block, grid, lds, st, P, K);
    HIP_TRY(p, e);
    return MC_OK;
}

template <typename T>
PriorParams<T> prior_params(const mc_problem *p, const T *heights, const double *partials) {
    PriorParams<T> P;
    memset(&P, 0, sizeof(P));
    P.R = p->R;
    P.C = p->C;
    P.n_tiles = lik_tiles(p);
    P.has_lik = p->n_ray > 0 ? 1 : 0;
    P.heights = heights;
    P.top64 = p->d_top64;
    for (int l = 0; l < p->S - 1; ++l) {
        P.logdet[l] = p->logdet[l];
        P.s11[l] = p->s11[l];
        P.r[l] = p->car_r[l];
    }
    P.sum_log_top = p->sum_log_top;
    P.eig_g = p->d_eig_g;
    P.eig_w = p->d_eig_w;
    P.n_eig = p->n_eig;
    P.partials = partials;
    P.kconst = p->vox_nz > 0 ? p->kconst_vox : (p->quad_nsub > 0 ? p->kconst_quad : p->kconst);
    return P;
}

template <typename T, int S, int B>
void launch_prior_shape(int n, size_t lds, const PriorParams<T> &P, hipStream_t st) {
    auto k = P.r_chain ? k_prior_finalize<T, S, B, true> : k_prior_finalize<T, S, B, false>;
    if (lds > 65536) (void)hipFuncSetAttribute((const void *)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL(k, dim3(n), dim3(B), lds, st, P);
}

template <typename T, int S>
mc_status launch_prior(mc_problem *p, int n, const PriorParams<T> &P, hipStream_t st) {
    const size_t N = (size_t)p->R * p->C, lds = sizeof(T) * N;
    if (N >= (size_t)kPriorLargeNodes) launch_prior_shape<T, S, kPriorBlockLarge>(n, lds, P, st);
    else launch_prior_shape<T, S, kPriorBlock>(n, lds, P, st);
    HIP_TRY(p, hipGetLastError());
    return MC_OK;
}

// ---------------------------------------------------------------------------
// The smoothed voxel model
// ---------------------------------------------------------------------------

int vox_n_pad(int n) { return (n + kVoxLanes - 1) / kVoxLanes * kVoxLanes; }

template <typename T>
VoxParams<T> vox_params(const mc_problem *p, int n, const T *heights, T *opacity, double *partials,
                        const double *only_nan) {
    VoxParams<T> V;
    memset(&V, 0, sizeof(V));
    V.R = p->R;
    V.C = p->C;
    V.N = p->R * p->C;
    V.n_z = p->vox_nz;
    V.M = (p->S - 1) * V.N;
    V.n_chains = n;
    V.n_pad = vox_n_pad(n);
    V.heights = heights;
    V.top = (const T *)p->d_top;
    V.rhat = (T *)p->rhat.p;
    V.dz = p->vox_dz;
    V.inv_gamma = 1.0 / p->vox_gamma;
    for (int l = 0; l < p->S; ++l) V.drho[l] = p->vox_drho[l];
    V.rho1 = p->density[0];
    V.floor_sig = p->d_vox_fsig;
    V.inv_norm = p->d_vox_inorm;
    V.n_ray = p->n_ray;
    V.n_tiles = tiling(p).n_tiles;
    V.ray_off = p->d_vox_off;
    V.vox = p->d_vox_idx;
    V.len = (const T *)p->d_vox_len;
    V.lam0 = p->d_vox_lam0;
    V.o0 = p->d_vox_o0;
    V.cnt = p->d_cnt64;
    V.inv_atten = 1.0 / p->atten;
    V.partials = partials;
    V.opacity = opacity;
    V.only_nan = only_nan;
    return V;
}

size_t rhat_bytes(const mc_problem *p, int n) {
    return (size_t)p->R * p->C * p->vox_nz * vox_n_pad(n) * elem_size(p);
}

template <typename T, int S>
void launch_vox_density(const VoxParams<T> &V, hipStream_t st) {
    hipLaunchKernelGGL((k_vox_density<T, S>), dim3(V.N, (V.n_pad + 255) / 256), dim3(256), 0, st, V);
}

template <typename T>
void launch_vox_lik(const VoxParams<T> &V, hipStream_t st) {
    const int groups = V.n_pad / kVoxLanes;
    const int tpx = (V.n_tiles + kXcds - 1) / kXcds;   // tiles per XCD and group
    const dim3 grid((unsigned)groups * (unsigned)tpx * kXcds);
    hipLaunchKernelGGL((k_vox_lik<T>), grid, dim3(kVoxWaves * kVoxLanes), 0, st, V);
}

// rhat must already hold rhat_bytes(p, n).
template <typename T, int S>
mc_status launch_voxel(mc_problem *p, int n, const T *heights, T *opacity, double *partials, hipStream_t st,
                       const double *only_nan) {
    VoxParams<T> V = vox_params<T>(p, n, heights, opacity, partials, only_nan);
    launch_vox_density<T, S>(V, st);
    launch_vox_lik<T>(V, st);
    HIP_TRY(p, hipGetLastError());
    return MC_OK;
}

// Solid-angle pixels: the march over every sub-ray with its opacities to
// obuf (its own per-ray terms, computed with zero counts, are overwritten),
// then the per-pixel likelihood.  opacity (optional) receives a copy of the
// sub-ray opacities.
template <typename T, int S>
mc_status launch_quad(mc_problem *p, int n, const T *heights, T *opacity, hipStream_t st, const double *only_nan) {
    T *ob = (T *)p->obuf.p;
    mc_status s;
    if ((s = launch_march<T, S>(p, n, heights, ob, (double *)p->partials.p, st, only_nan)) != MC_OK) return s;
    const int tiles = lik_tiles(p);
    hipLaunchKernelGGL(k_quad_lik<T>, dim3(tiles, n), dim3(256), 0, st, (const T *)ob, p->n_ray, p->quad_npx,
                       p->quad_nsub, (const double *)p->d_quad_w, (const double *)p->d_quad_tab, p->quad_ntab,
                       (p->quad_ntab - 1) / p->quad_omax, (const double *)p->d_quad_cnt, (double *)p->partials.p,
                       tiles, only_nan);
    HIP_TRY(p, hipGetLastError());
    if (opacity) HIP_TRY(p, hipMemcpyAsync(opacity, ob, sizeof(T) * (size_t)n * p->n_ray, hipMemcpyDeviceToDevice, st));
    return MC_OK;
}

mc_status check_ready(mc_problem *p) {
    if (!p) return MC_ERR_ARG;
    if (!p->have_geom) return fail(p, MC_ERR_STATE, "load_geometry_grid has not been called");
    if (!p->have_sensors) return fail(p, MC_ERR_STATE, "set_sensors has not been called");
    if (p->n_ray > 0 && !p->have_counts) return fail(p, MC_ERR_STATE, "set_counts has not been called");
    return MC_OK;
}

// r_chain ([n][S-1], optional): per-chain dependence parameters; stat
// (optional, [2][n][S-1]): receives sum w^2 and the edge sums.
template <typename T, int S>
mc_status logpost_impl(mc_problem *p, int n, const T *heights, double *lp, T *opacity, hipStream_t st,
                       const double *only_nan = nullptr, double *r_chain = nullptr, double *stat = nullptr) {
    Tiling t = tiling(p);
    mc_status s;
    if (p->n_ray > 0) {
        if ((s = ensure(p, p->partials, sizeof(double) * (size_t)n * partial_slots(p))) != MC_OK) return s;
        (void)t;
        if (p->quad_nsub > 0) {
            if ((s = ensure(p, p->obuf, sizeof(T) * (size_t)n * p->n_ray)) != MC_OK) return s;
            if ((s = launch_quad<T, S>(p, n, heights, opacity, st, only_nan)) != MC_OK) return s;
        } else if (p->vox_nz > 0) {
            if ((s = ensure(p, p->rhat, rhat_bytes(p, n))) != MC_OK) return s;
            if ((s = launch_voxel<T, S>(p, n, heights, opacity, (double *)p->partials.p, st, only_nan)) != MC_OK)
                return s;
        } else if ((s = launch_march<T, S>(p, n, heights, opacity, (double *)p->partials.p, st, only_nan)) !=
                   MC_OK) {
            return s;
        }
    }
    PriorParams<T> P = prior_params<T>(p, heights, (const double *)p->partials.p);
    P.lp_out = lp;
    P.only_nan = only_nan;
    P.r_chain = r_chain;
    if (stat) {
        P.stat_sw2 = stat;
        P.stat_se = stat + (size_t)n * (S - 1);
    }
    return launch_prior<T, S>(p, n, P, st);
}

template <typename T>
mc_status logpost_dispatch(mc_problem *p, int n, const void *heights, double *lp, void *opacity, hipStream_t st) {
    switch (p->S) {
        case 2: return logpost_impl<T, 2>(p, n, (const T *)heights, lp, (T *)opacity, st);
        case 3: return logpost_impl<T, 3>(p, n, (const T *)heights, lp, (T *)opacity, st);
        case 4: return logpost_impl<T, 4>(p, n, (const T *)heights, lp, (T *)opacity, st);
    }
    return fail(p, MC_ERR_UNSUPPORTED, "n_surfaces %d", p->S);
}

// logpost_batch on the exact march with the likelihood partials in the
// device's `scratch` array (ws): the same kernels, no workspace allocation.
template <typename T, int S>
mc_status logpost_noalloc_impl(mc_problem *p, int n, const T *heights, double *lp, T *opacity, hipStream_t st,
                               double *ws) {
    mc_status s;
    if (p->n_ray > 0 && (s = launch_march<T, S>(p, n, heights, opacity, ws, st)) != MC_OK) return s;
    PriorParams<T> P = prior_params<T>(p, heights, ws);
    P.lp_out = lp;
    return launch_prior<T, S>(p, n, P, st);
}

template <typename T>
mc_status logpost_noalloc_dispatch(mc_problem *p, int n, const void *heights, double *lp, void *opacity,
                                   hipStream_t st, double *ws) {
    switch (p->S) {
        case 2: return logpost_noalloc_impl<T, 2>(p, n, (const T *)heights, lp, (T *)opacity, st, ws);
        case 3: return logpost_noalloc_impl<T, 3>(p, n, (const T *)heights, lp, (T *)opacity, st, ws);
        case 4: return logpost_noalloc_impl<T, 4>(p, n, (const T *)heights, lp, (T *)opacity, st, ws);
    }
    return fail(p, MC_ERR_UNSUPPORTED, "n_surfaces %d", p->S);
}

template <typename T, int S, int B>
void launch_prior_grad(int n, size_t lds, const PriorParams<T> &P, const unsigned long long *gfix, T *grad,
                       hipStream_t st) {
    auto k = k_prior_grad<T, S, B>;
    if (lds > 65536) (void)hipFuncSetAttribute((const void *)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL(k, dim3(n), dim3(B), lds, st, P, gfix, grad);
}

template <typename T, int S, bool TL, int B>
void launch_adjoint_shape(dim3 grid, size_t lds, const MarchParams<T> &M, const RayConsts<T> &K, const T *obuf,
                          unsigned long long *gfix, const T *gpbuf, hipStream_t st) {
    auto k = k_adjoint<T, S, TL, B>;
    if (lds > 65536) (void)hipFuncSetAttribute((const void *)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL(k, grid, dim3(B), lds, st, M, K, obuf, gfix, gpbuf);
}

template <int S, int B>
void launch_adjoint_lds_shape(dim3 grid, size_t lds, const MarchParams<float> &M, const RayConsts<float> &K,
                              const float *gp, const int *ovf, unsigned long long *gfix, AdjointLdsShape w,
                              hipStream_t st) {
    auto k = k_adjoint_lds<S, B>;
    if (lds > 65536) (void)hipFuncSetAttribute((const void *)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL(k, grid, dim3(B), lds, st, M, K, gp, ovf, gfix, w);
}

template <int S, int B>
void launch_adjoint_rec_shape(dim3 grid, size_t lds, const MarchParams<float> &M, const CrossRecs &X, int fwd_block,
                              AdjointLdsShape w, unsigned long long *gfix, hipStream_t st) {
    auto k = k_adjoint_rec<S, B>;
    if (lds > 65536) (void)hipFuncSetAttribute((const void *)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL(k, grid, dim3(B), lds, st, M, X, fwd_block, w, gfix);
}

// Crossing-record slots per thread and surface of the gradient march:
// twice the rays a thread marches plus 16 (the crossings of one surface per
// ray are 1 on average at the benchmark shapes, and a thread's count varies
// by a few times its square root; with 2 x rays only, one thread list in a
// few hundred overflowed at 8 rays per thread, sending its chain to the
// re-walk nearly every call), or the tuning's grad_slots (-1: none, so every
// chain takes the re-walk).  Slots cost memory, not traffic: only written
// records are read.
int cross_slots(const mc_problem *p) {
    if (p->tune.grad_slots < 0) return 0;
    if (p->tune.grad_slots > 0) return p->tune.grad_slots;
    return 2 * p->tune.rays_per_thread + 16;
}

CrossRecs cross_recs(const mc_problem *p) {
    CrossRecs X;
    X.rec = (uint4 *)p->xrec.p;
    X.cnt = (uint32_t *)p->xcnt.p;
    X.ovf = (int *)p->xovf.p;
    X.gp = (float *)p->xgp.p;
    X.slots = cross_slots(p);
    return X;
}

template <int S, bool TL, int B>
void launch_march_rec_shape(dim3 grid, size_t lds, hipStream_t st, const MarchParams<float> &P,
                            const RayConsts<float> &K, const CrossRecs &X) {
    auto k = k_march_rec4<S, TL, B>;
    if (lds > 65536) (void)hipFuncSetAttribute((const void *)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL(k, grid, dim3(B), lds, st, P, K, X);
}

// The float32 gradient march: the forward march of n states with the
// crossing records and dLL/dO of every ray (the partials feed the prior
// kernel as usual).  Clears the overflow flags first.
template <int S>
mc_status launch_march_rec(mc_problem *p, int n, const float *heights, hipStream_t st, float *opacity = nullptr) {
    MarchParams<float> P = march_params<float>(p, heights, opacity, (double *)p->partials.p);
    P.n_chains = n;
    const CrossRecs X = cross_recs(p);
    hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, X.ovf, n);
    const dim3 grid((unsigned)P.n_tiles * (unsigned)((n + kXcds - 1) / kXcds * kXcds));
    const size_t N = (size_t)p->R * p->C;
    const int b = p->tune.block;
    // static LDS: the march's reductions (< 16 KiB) and the record indices (S x block)
    const size_t fixed = 16384 + (size_t)S * b * sizeof(unsigned);
    bool tl = top_in_lds(p);
    size_t lds = N * (tl ? S : S - 1) * sizeof(float);
    if (lds + fixed > p->max_lds) {
        tl = false;
        lds = N * (S - 1) * sizeof(float);
    }
    if (lds + fixed > p->max_lds) return fail(p, MC_ERR_UNSUPPORTED, "grid %dx%d too large for LDS", p->R, p->C);
    const RayConsts<float> K = ray_consts<float>(p);
    if (tl) {
        if (b == 256) launch_march_rec_shape<S, true, 256>(grid, lds, st, P, K, X);
        else if (b == 512) launch_march_rec_shape<S, true, 512>(grid, lds, st, P, K, X);
        else launch_march_rec_shape<S, true, 1024>(grid, lds, st, P, K, X);
    } else {
        if (b == 256) launch_march_rec_shape<S, false, 256>(grid, lds, st, P, K, X);
        else if (b == 512) launch_march_rec_shape<S, false, 512>(grid, lds, st, P, K, X);
        else launch_march_rec_shape<S, false, 1024>(grid, lds, st, P, K, X);
    }
    HIP_TRY(p, hipGetLastError());
    return MC_OK;
}


// The adjoint march of n states (forward opacities in p->obuf).  float32:
// k_adjoint_lds with node-row windows sized so that one surface and the
// window's 64-bit accumulators fit the LDS; float64: the direct scatter.
// Forward tiling and XCD-aware grids; 1024-thread blocks when a block takes
// more than 64 KB of LDS (one block per compute unit).
template <typename T, int S>
mc_status launch_adjoint(mc_problem *p, int n, const T *heights, unsigned long long *gfix, hipStream_t st) {
    const size_t N = (size_t)p->R * p->C;
    MarchParams<T> M = march_params<T>(p, heights, nullptr, (double *)p->partials.p);
    M.n_chains = n;
    RayConsts<T> K = ray_consts<T>(p);
    if constexpr (std::is_same<T, float>::value) {   // float32: the record adjoint, re-walks on overflow
        const size_t row_bytes = (size_t)p->C * sizeof(unsigned long long);
        const CrossRecs X = cross_recs(p);
        // the record adjoint: windows of node rows whose accumulators fit the LDS
        {
            const size_t budget = p->max_lds - 1024;
            AdjointLdsShape w;
            w.window_rows = (int)std::min<size_t>((size_t)p->R, budget / row_bytes);
            if (p->tune.adjoint_rows > 0) w.window_rows = std::min(w.window_rows, p->tune.adjoint_rows);
            w.n_windows = (p->R + w.window_rows - 1) / w.window_rows;
            const size_t lds = (size_t)w.window_rows * row_bytes;
            const dim3 grid((unsigned)(S * w.n_windows) * (unsigned)((n + kXcds - 1) / kXcds * kXcds));
            const int fb = p->tune.block;
            if (lds > 65536) launch_adjoint_rec_shape<S, 1024>(grid, lds, M, X, fb, w, gfix, st);
            else if (lds > 16384) launch_adjoint_rec_shape<S, 512>(grid, lds, M, X, fb, w, gfix, st);
            else launch_adjoint_rec_shape<S, 256>(grid, lds, M, X, fb, w, gfix, st);
            HIP_TRY(p, hipGetLastError());
        }
        // the re-walk of chains whose records overflowed (other chains' blocks exit at once)
        const size_t surf = (N * sizeof(float) + 15) & ~(size_t)15;
        if (surf + 4096 + row_bytes > p->max_lds)
            return fail(p, MC_ERR_UNSUPPORTED, "grid %dx%d too large for LDS", p->R, p->C);
        const size_t budget = p->max_lds - surf - 4096;
        AdjointLdsShape w;
        w.n_windows = (int)(((size_t)p->R * row_bytes + budget - 1) / budget);
        w.window_rows = (p->R + w.n_windows - 1) / w.n_windows;
        if (p->tune.adjoint_rows > 0) w.window_rows = std::min(w.window_rows, p->tune.adjoint_rows);
        w.n_windows = (p->R + w.window_rows - 1) / w.window_rows;
        const size_t lds = surf + (size_t)w.window_rows * row_bytes;
        const dim3 grid((unsigned)(S * w.n_windows) * (unsigned)((n + kXcds - 1) / kXcds * kXcds));
        // up to 64 KB of LDS: 512-thread blocks, so the LDS that limits blocks
        // per CU still leaves 6 wavefronts per SIMD (256 threads left 3)
        if (lds > 65536) launch_adjoint_lds_shape<S, 1024>(grid, lds, M, K, X.gp, X.ovf, gfix, w, st);
        else launch_adjoint_lds_shape<S, 512>(grid, lds, M, K, X.gp, X.ovf, gfix, w, st);
        HIP_TRY(p, hipGetLastError());
        return MC_OK;
    } else {   // float64: the direct scatter
        const bool tl = N * S * sizeof(T) + 4096 <= p->max_lds;
        const size_t lds = N * (tl ? S : S - 1) * sizeof(T);
        if (lds + 2048 > p->max_lds) return fail(p, MC_ERR_UNSUPPORTED, "grid %dx%d too large for LDS", p->R, p->C);
        const dim3 grid((unsigned)M.n_tiles * (unsigned)((n + kXcds - 1) / kXcds * kXcds));
        const T *ob = (const T *)p->obuf.p;
        const T *gpb = p->quad_nsub > 0 ? (const T *)p->xgp.p : nullptr;   // dLL/dO of the sub-rays
        const bool big = lds > 65536;
        if (tl) {
            if (big) launch_adjoint_shape<T, S, true, 1024>(grid, lds, M, K, ob, gfix, gpb, st);
            else launch_adjoint_shape<T, S, true, 256>(grid, lds, M, K, ob, gfix, gpb, st);
        } else {
            if (big) launch_adjoint_shape<T, S, false, 1024>(grid, lds, M, K, ob, gfix, gpb, st);
            else launch_adjoint_shape<T, S, false, 256>(grid, lds, M, K, ob, gfix, gpb, st);
        }
        HIP_TRY(p, hipGetLastError());
        return MC_OK;
    }
}

// Log posterior and gradient of n states into lp and grad ([n][S][N] in T):
// forward march with opacities, prior and its gradient, adjoint march,
// combine.  Workspaces must be ensured by the caller (ensure_grad_ws).
// The likelihood part of the gradient of n states into the fixed-point
// accumulators gfix [n][S][R*C] (every entry written), and the partial sums
// of the likelihood.  float32: the gradient march with crossing records and
// the record adjoint; float64: the march with opacities, then the re-walking
// scatter into zeroed accumulators.
template <typename T, int S>
mc_status lik_grad(mc_problem *p, int n, const T *heights, unsigned long long *gfix, hipStream_t st) {
    mc_status s;
    if (p->vox_nz > 0) {   // the smoothed voxel model: density, likelihood with dLL/dO, back-projection
        VoxParams<T> V = vox_params<T>(p, n, heights, nullptr, (double *)p->partials.p, nullptr);
        V.alpha = (T *)p->valpha.p;
        V.t_off = p->d_vox_toff;
        V.t_ray = p->d_vox_tray;
        V.t_len = (const T *)p->d_vox_tlen;
        V.items = p->d_vox_items;
        V.n_items = p->vox_n_items;
        V.gfix = gfix;
        launch_vox_density<T, S>(V, st);
        launch_vox_lik<T>(V, st);
        const size_t tot = (size_t)S * V.N * n;   // the items add into zeroed accumulators
        hipLaunchKernelGGL(k_fill_u64, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, gfix, tot);
        HIP_TRY(p, hipGetLastError());
        if (V.n_items > 0) {
            const int n_ib = (V.n_items + 3) / 4;
            const int upx = (n_ib + kVoxGradUnit * kXcds - 1) / (kVoxGradUnit * kXcds);
            hipLaunchKernelGGL((k_vox_grad<T, S>),
                               dim3((unsigned)(kXcds * upx * kVoxGradUnit * (V.n_pad / kVoxLanes))), dim3(256), 0, st,
                               V);
            HIP_TRY(p, hipGetLastError());
        }
        return MC_OK;
    }
    const bool quad = p->quad_nsub > 0;
    if constexpr (std::is_same<T, float>::value) {
        if ((s = launch_march_rec<S>(p, n, heights, st, quad ? (float *)p->obuf.p : nullptr)) != MC_OK) return s;
    } else {
        const size_t tot = (size_t)S * p->R * p->C * n;
        hipLaunchKernelGGL(k_fill_u64, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, gfix, tot);
        HIP_TRY(p, hipGetLastError());
        if ((s = launch_march<T, S>(p, n, heights, (T *)p->obuf.p, (double *)p->partials.p, st)) != MC_OK) return s;
    }
    if (quad) {
        // solid-angle pixels: the pixel likelihood from the sub-ray opacities, and
        // each sub-ray's dLL/dO in place of the march's one-ray value
        const int tiles = lik_tiles(p);
        hipLaunchKernelGGL(k_quad_lik<T>, dim3(tiles, n), dim3(256), 0, st, (const T *)p->obuf.p, p->n_ray,
                           p->quad_npx, p->quad_nsub, (const double *)p->d_quad_w, (const double *)p->d_quad_tab,
                           p->quad_ntab, (p->quad_ntab - 1) / p->quad_omax, (const double *)p->d_quad_cnt,
                           (double *)p->partials.p, tiles, (const double *)nullptr, (T *)p->xgp.p);
        HIP_TRY(p, hipGetLastError());
    }
    return launch_adjoint<T, S>(p, n, heights, gfix, st);
}

template <typename T, int S>
mc_status grad_eval(mc_problem *p, int n, const T *heights, double *lp, T *grad, hipStream_t st) {
    const size_t N = (size_t)p->R * p->C;
    unsigned long long *gfix = (unsigned long long *)p->gfix.p;
    mc_status s;
    if (p->n_ray > 0 && (s = lik_grad<T, S>(p, n, heights, gfix, st)) != MC_OK) return s;
    PriorParams<T> P = prior_params<T>(p, heights, (const double *)p->partials.p);
    P.lp_out = lp;
    const unsigned long long *gl = p->n_ray > 0 ? gfix : nullptr;
    const size_t lds = sizeof(double) * N;
    if (N >= (size_t)kPriorLargeNodes) launch_prior_grad<T, S, kPriorBlockLarge>(n, lds, P, gl, grad, st);
    else launch_prior_grad<T, S, kPriorBlock>(n, lds, P, gl, grad, st);
    HIP_TRY(p, hipGetLastError());
    return MC_OK;
}

template <typename T, int S>
mc_status ensure_grad_ws(mc_problem *p, int n) {
    const size_t N = (size_t)p->R * p->C, SN = (size_t)S * N;
    mc_status s;
    Tiling t = tiling(p);
    if (p->n_ray > 0) {
        if ((s = ensure(p, p->partials, sizeof(double) * (size_t)n * partial_slots(p))) != MC_OK) return s;
        if (p->quad_nsub > 0) {   // sub-ray opacities and dLL/dO (also in float64)
            if ((s = ensure(p, p->obuf, sizeof(T) * (size_t)n * p->n_ray)) != MC_OK) return s;
            if ((s = ensure(p, p->xgp, sizeof(T) * (size_t)n * p->n_ray)) != MC_OK) return s;
        }
        if (p->vox_nz > 0) {
            if ((s = ensure(p, p->rhat, rhat_bytes(p, n))) != MC_OK) return s;
            if ((s = ensure(p, p->valpha, sizeof(T) * (size_t)vox_n_pad(n) * p->n_ray)) != MC_OK) return s;
        } else if constexpr (std::is_same<T, float>::value) {
            const size_t rows = (size_t)n * t.n_tiles * S;   // (chain, tile, surface) record lists
            if ((s = ensure(p, p->xrec, 16 * rows * (size_t)cross_slots(p) * p->tune.block)) != MC_OK) return s;
            if ((s = ensure(p, p->xcnt, 4 * rows * p->tune.block)) != MC_OK) return s;
            if ((s = ensure(p, p->xovf, sizeof(int) * (size_t)n)) != MC_OK) return s;
            if ((s = ensure(p, p->xgp, sizeof(float) * (size_t)n * p->n_ray)) != MC_OK) return s;
        } else {
            if ((s = ensure(p, p->obuf, sizeof(T) * (size_t)n * p->n_ray)) != MC_OK) return s;
        }
    }
    if (p->n_ray > 0 && (s = ensure(p, p->gfix, sizeof(unsigned long long) * SN * n)) != MC_OK) return s;
    return MC_OK;
}

template <typename T, int S>
mc_status logpost_grad_impl(mc_problem *p, int n, const T *heights, double *lp, T *grad, hipStream_t st) {
    mc_status s;
    if ((s = ensure_grad_ws<T, S>(p, n)) != MC_OK) return s;
    return grad_eval<T, S>(p, n, heights, lp, grad, st);
}

template <typename T>
mc_status logpost_grad_dispatch(mc_problem *p, int n, const void *heights, double *lp, void *grad, hipStream_t st) {
    switch (p->S) {
        case 2: return logpost_grad_impl<T, 2>(p, n, (const T *)heights, lp, (T *)grad, st);
        case 3: return logpost_grad_impl<T, 3>(p, n, (const T *)heights, lp, (T *)grad, st);
        case 4: return logpost_grad_impl<T, 4>(p, n, (const T *)heights, lp, (T *)grad, st);
    }
    return fail(p, MC_ERR_UNSUPPORTED, "n_surfaces %d", p->S);
}

// One MALA step: propose from the cached gradient, evaluate lp and gradient
// at the proposal, decide, copy.
template <typename T, int S>
mc_status mala_step(mc_problem *p, int n, T *heights, double *lp, int64_t *acc, const mc_run_config *cfg, int k,
                    hipStream_t st) {
    const int M = (S - 1) * p->R * p->C;
    const int SN = S * p->R * p->C;
    T *prop = (T *)p->prop.p;
    T *gcur = (T *)p->gcur.p, *gprop = (T *)p->gprop.p;
    double *lpp = (double *)p->lpprop.p;
    dim3 pg((M / 2 + 1 + 255) / 256, n);
    hipLaunchKernelGGL(k_propose_mala<T>, pg, dim3(256), 0, st, (const T *)heights, (const T *)gcur, prop,
                       cfg->inv_mass, M, SN, cfg->step_size, cfg->seed, (const uint64_t *)p->d_step, k);
    HIP_TRY(p, hipGetLastError());
    mc_status s;
    if ((s = grad_eval<T, S>(p, n, prop, lpp, gprop, st)) != MC_OK) return s;
    // one block per chain; large grids take 1024 threads (more loads in flight per chain)
    const bool big = (size_t)M >= (size_t)kPriorLargeNodes;
    auto kfin = big ? k_mala_finalize<T, kPriorBlockLarge> : k_mala_finalize<T, kPriorBlock>;
    hipLaunchKernelGGL(kfin, dim3(n), dim3(big ? kPriorBlockLarge : kPriorBlock), 0, st, heights,
                       (const T *)prop, gcur, (const T *)gprop, lp, (const double *)lpp, acc, cfg->inv_mass, M, SN,
                       cfg->step_size, cfg->seed, (const uint64_t *)p->d_step, k);
    HIP_TRY(p, hipGetLastError());
    return MC_OK;
}

// One random-walk Metropolis step (propose, march the proposals, prior +
// decision + copy) with the step number read from p->d_step plus k.
template <typename T, int S>
mc_status rw_step(mc_problem *p, int n, T *heights, double *lp, int64_t *acc, const mc_run_config *cfg, int k,
                  hipStream_t st) {
    const int M = (S - 1) * p->R * p->C;
    T *prop = (T *)p->prop.p;
    dim3 pg((M / 2 + 1 + 255) / 256, n);
    hipLaunchKernelGGL(k_propose_rw<T>, pg, dim3(256), 0, st, (const T *)heights, prop, M, cfg->step_size,
                       cfg->seed, (const uint64_t *)p->d_step, k);
    HIP_TRY(p, hipGetLastError());
    mc_status s;
    if (p->n_ray > 0) {
        if (p->quad_nsub > 0)
            s = launch_quad<T, S>(p, n, prop, nullptr, st, nullptr);
        else if (p->vox_nz > 0)
            s = launch_voxel<T, S>(p, n, prop, nullptr, (double *)p->partials.p, st, nullptr);
        else
            s = launch_march<T, S>(p, n, prop, nullptr, (double *)p->partials.p, st);
        if (s != MC_OK) return s;
    }
    PriorParams<T> P = prior_params<T>(p, prop, (const double *)p->partials.p);
    P.mh = 1;
    P.lp_cur = lp;
    P.n_acc = acc;
    P.state = heights;
    P.seed = cfg->seed;
    P.step_base = p->d_step;
    P.step_k = k;
    if (cfg->r_state) {
        P.r_chain = cfg->r_state;
        P.sample_r = 1;
        P.r_step = cfg->r_step;
        P.n_acc_r = cfg->n_accept_r;
        P.stat_sw2 = (double *)p->rstat.p;
        P.stat_se = (double *)p->rstat.p + (size_t)n * (S - 1);
    }
    return launch_prior<T, S>(p, n, P, st);
}

template <typename T, int S>
mc_status mcmc_impl(mc_problem *p, const mc_run_config *cfg, int n, T *heights, double *lp, int64_t *acc,
                    hipStream_t st) {
    const int M = (S - 1) * p->R * p->C;
    const size_t SN = (size_t)S * p->R * p->C;
    Tiling t = tiling(p);
    mc_status s;
    const bool mala = cfg->kernel == 1;
    if ((s = ensure(p, p->prop, sizeof(T) * (size_t)n * M)) != MC_OK) return s;
    if ((s = ensure(p, p->lptmp, sizeof(double) * (size_t)n)) != MC_OK) return s;
    if (p->n_ray > 0 && (s = ensure(p, p->partials, sizeof(double) * (size_t)n * partial_slots(p))) != MC_OK) return s;
    if (p->n_ray > 0 && p->vox_nz > 0 && (s = ensure(p, p->rhat, rhat_bytes(p, n))) != MC_OK) return s;
    if (p->n_ray > 0 && p->quad_nsub > 0 && (s = ensure(p, p->obuf, sizeof(T) * (size_t)n * p->n_ray)) != MC_OK)
        return s;
    (void)t;
    if (mala) {
        if ((s = ensure_grad_ws<T, S>(p, n)) != MC_OK) return s;
        if ((s = ensure(p, p->gcur, sizeof(T) * SN * n)) != MC_OK) return s;
        if ((s = ensure(p, p->gprop, sizeof(T) * SN * n)) != MC_OK) return s;
        if ((s = ensure(p, p->lpprop, sizeof(double) * (size_t)n)) != MC_OK) return s;
        // MALA needs the gradient of the current states: lp and gradient are recomputed
        if ((s = grad_eval<T, S>(p, n, heights, lp, (T *)p->gcur.p, st)) != MC_OK) return s;
    } else if (cfg->r_state) {
        // with r sampled: log posterior and the w-statistics of every chain at its own r
        if ((s = ensure(p, p->rstat, 2 * sizeof(double) * (size_t)n * (S - 1))) != MC_OK) return s;
        if ((s = logpost_impl<T, S>(p, n, heights, lp, nullptr, st, nullptr, cfg->r_state, (double *)p->rstat.p)) !=
            MC_OK)
            return s;
    } else {
        // initial log posterior where the caller passed NaN (other chains exit at once)
        if ((s = logpost_impl<T, S>(p, n, heights, (double *)p->lptmp.p, nullptr, st, lp)) != MC_OK) return s;
        hipLaunchKernelGGL(k_fill_nan, dim3((n + 255) / 256), dim3(256), 0, st, lp, (const double *)p->lptmp.p, n);
    }
    hipLaunchKernelGGL(k_set_u64, dim3(1), dim3(1), 0, st, p->d_step, cfg->step_offset);
    HIP_TRY(p, hipGetLastError());
    auto step_fn = [&](int k, hipStream_t ss) {
        return mala ? mala_step<T, S>(p, n, heights, lp, acc, cfg, k, ss) : rw_step<T, S>(p, n, heights, lp, acc, cfg, k, ss);
    };
    const int G = cfg->graph_steps < 1 ? 1 : cfg->graph_steps;
    int64_t done = 0;
    if (G > 1 && cfg->n_steps >= G) {
        GraphKey key;
        key.n = n;
        key.kernel = cfg->kernel;
        key.G = G;
        key.heights = heights;
        key.lp = lp;
        key.acc = acc;
        key.inv_mass = cfg->inv_mass;
        key.step_size = cfg->step_size;
        key.seed = cfg->seed;
        key.r_state = cfg->r_state;
        key.acc_r = cfg->n_accept_r;
        key.r_step = cfg->r_step;
        if (!(p->gexec && p->gkey == key)) {
            if (p->gexec) {
                (void)hipGraphExecDestroy(p->gexec);
                p->gexec = nullptr;
            }
            if (!p->cap_stream) HIP_TRY(p, hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking));
            HIP_TRY(p, hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeThreadLocal));
            mc_status cs = MC_OK;
            for (int k = 0; k < G && cs == MC_OK; ++k) cs = step_fn(k, p->cap_stream);
            if (cs == MC_OK) hipLaunchKernelGGL(k_add_u64, dim3(1), dim3(1), 0, p->cap_stream, p->d_step, (uint64_t)G);
            hipGraph_t graph = nullptr;
            hipError_t e = hipStreamEndCapture(p->cap_stream, &graph);
            if (cs != MC_OK) {
                if (graph) (void)hipGraphDestroy(graph);
                return cs;
            }
            if (e != hipSuccess) return fail(p, MC_ERR_DEVICE, "graph capture: %s", hipGetErrorString(e));
            e = hipGraphInstantiate(&p->gexec, graph, nullptr, nullptr, 0);
            (void)hipGraphDestroy(graph);
            if (e != hipSuccess) {
                p->gexec = nullptr;
                return fail(p, MC_ERR_DEVICE, "graph instantiate: %s", hipGetErrorString(e));
            }
            p->gkey = key;
        }
        for (; done + G <= cfg->n_steps; done += G) HIP_TRY(p, hipGraphLaunch(p->gexec, st));
    }
    // remaining steps as eager launches
    const int64_t rest = cfg->n_steps - done;
    for (int64_t k = 0; k < rest; ++k)
        if ((s = step_fn((int)k, st)) != MC_OK) return s;
    if (rest > 0) hipLaunchKernelGGL(k_add_u64, dim3(1), dim3(1), 0, st, p->d_step, (uint64_t)rest);
    HIP_TRY(p, hipGetLastError());
    return MC_OK;
}

template <typename T, int S>
mc_status time_march_impl(mc_problem *p, int n, const T *heights, int iters, hipStream_t st, float *ms) {
    Tiling t = tiling(p);
    mc_status s;
    if ((s = ensure(p, p->partials, sizeof(double) * (size_t)n * t.n_tiles)) != MC_OK) return s;
    hipEvent_t e0, e1;
    HIP_TRY(p, hipEventCreate(&e0));
    HIP_TRY(p, hipEventCreate(&e1));
    HIP_TRY(p, hipEventRecord(e0, st));
    for (int i = 0; i < iters && s == MC_OK; ++i) s = launch_march<T, S>(p, n, heights, nullptr, (double *)p->partials.p, st);
    HIP_TRY(p, hipEventRecord(e1, st));
    HIP_TRY(p, hipEventSynchronize(e1));
    float total = 0.f;
    HIP_TRY(p, hipEventElapsedTime(&total, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    *ms = total / (float)iters;
    return s;
}

// Mean time of the adjoint kernel alone: one full gradient evaluation sets
// up the forward opacities, then `iters` adjoint launches are timed (their
// accumulations are discarded).
template <typename T, int S>
mc_status time_adjoint_impl(mc_problem *p, int n, const T *heights, int iters, hipStream_t st, float *ms) {
    const size_t SN = (size_t)S * p->R * p->C;
    mc_status s;
    if ((s = ensure_grad_ws<T, S>(p, n)) != MC_OK) return s;
    if ((s = ensure(p, p->lptmp, sizeof(double) * (size_t)n)) != MC_OK) return s;
    if ((s = ensure(p, p->gcur, sizeof(T) * SN * n)) != MC_OK) return s;
    if ((s = grad_eval<T, S>(p, n, heights, (double *)p->lptmp.p, (T *)p->gcur.p, st)) != MC_OK) return s;
    hipEvent_t e0, e1;
    HIP_TRY(p, hipEventCreate(&e0));
    HIP_TRY(p, hipEventCreate(&e1));
    HIP_TRY(p, hipEventRecord(e0, st));
    for (int i = 0; i < iters && s == MC_OK; ++i)
        s = launch_adjoint<T, S>(p, n, heights, (unsigned long long *)p->gfix.p, st);
    HIP_TRY(p, hipEventRecord(e1, st));
    HIP_TRY(p, hipEventSynchronize(e1));
    float total = 0.f;
    HIP_TRY(p, hipEventElapsedTime(&total, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    *ms = total / (float)iters;
    return s;
}

template <typename T>
mc_status time_adjoint_dispatch(mc_problem *p, int n, const void *heights, int iters, hipStream_t st, float *ms) {
    switch (p->S) {
        case 2: return time_adjoint_impl<T, 2>(p, n, (const T *)heights, iters, st, ms);
        case 3: return time_adjoint_impl<T, 3>(p, n, (const T *)heights, iters, st, ms);
        case 4: return time_adjoint_impl<T, 4>(p, n, (const T *)heights, iters, st, ms);
    }
    return fail(p, MC_ERR_UNSUPPORTED, "n_surfaces %d", p->S);
}

template <typename T>
mc_status time_march_dispatch(mc_problem *p, int n, const void *heights, int iters, hipStream_t st, float *ms) {
    switch (p->S) {
        case 2: return time_march_impl<T, 2>(p, n, (const T *)heights, iters, st, ms);
        case 3: return time_march_impl<T, 3>(p, n, (const T *)heights, iters, st, ms);
        case 4: return time_march_impl<T, 4>(p, n, (const T *)heights, iters, st, ms);
    }
    return fail(p, MC_ERR_UNSUPPORTED, "n_surfaces %d", p->S);
}

template <typename T>
mc_status mcmc_dispatch(mc_problem *p, const mc_run_config *cfg, int n, void *heights, double *lp, int64_t *acc,
                        hipStream_t st) {
    switch (p->S) {
        case 2: return mcmc_impl<T, 2>(p, cfg, n, (T *)heights, lp, acc, st);
        case 3: return mcmc_impl<T, 3>(p, cfg, n, (T *)heights, lp, acc, st);
        case 4: return mcmc_impl<T, 4>(p, cfg, n, (T *)heights, lp, acc, st);
    }
    return fail(p, MC_ERR_UNSUPPORTED, "n_surfaces %d", p->S);
}

// ---------------------------------------------------------------------------
// Many problems per launch
// ---------------------------------------------------------------------------

constexpr int kMultiBlock = 256;

struct MultiClass {
    void *items = nullptr;   // int4 [n_items]
    int n_items = 0;
    size_t lds = 0;
    bool top_lds = false;
    int block = kMultiBlock;
    hipStream_t side = nullptr;   // classes after the first run on their own stream
    hipEvent_t done = nullptr;
};

struct MultiPlan {
    // key
    std::vector<mc_problem *> ps;
    std::vector<int> n;
    std::vector<const void *> H, lp, acc;
    std::vector<uint64_t> gens, seeds;
    std::vector<double> sigma;
    std::vector<const void *> r, acc_r;   // sampled r: per-chain r and r acceptances (else null)
    std::vector<double> r_step;
    bool hier = false;
    int G = 0, device = 0;
    // device tables
    void *d_mp = nullptr, *d_rc = nullptr, *d_pp = nullptr, *d_pd = nullptr, *d_chain_items = nullptr;
    void *d_step_ptrs = nullptr, *d_step_vals = nullptr;
    int n_chain_items = 0, n_chain_items_large = 0;   // items [0, large) have grids of kPriorLargeNodes+
    size_t prior_lds = 0, prior_lds_large = 0;
    std::vector<MultiClass> classes;
    hipGraphExec_t gexec = nullptr;
    hipStream_t cap = nullptr;
    hipEvent_t fork = nullptr;
    int persistent_blocks = 0;
    ~MultiPlan() {
        if (gexec) (void)hipGraphExecDestroy(gexec);
        if (cap) (void)hipStreamDestroy(cap);
        if (fork) (void)hipEventDestroy(fork);
        for (void *q : {d_mp, d_rc, d_pp, d_pd, d_chain_items, d_step_ptrs, d_step_vals})
            if (q) (void)hipFree(q);
        for (auto &c : classes) {
            if (c.items) (void)hipFree(c.items);
            if (c.side) (void)hipStreamDestroy(c.side);
            if (c.done) (void)hipEventDestroy(c.done);
        }
    }
};

std::vector<MultiPlan *> g_multi_plans;   // small cache of built plans (most recent last)
std::mutex g_multi_mu;                     // guards g_multi_plans

template <typename X>
mc_status upload_vec(mc_problem *err, void *&dst, const std::vector<X> &v) {
    if (dst) (void)hipFree(dst);
    dst = nullptr;
    if (v.empty()) return MC_OK;
    HIP_TRY(err, hipMalloc(&dst, sizeof(X) * v.size()));
    HIP_TRY(err, hipMemcpy(dst, v.data(), sizeof(X) * v.size(), hipMemcpyHostToDevice));
    return MC_OK;
}

template <typename T, int S>
mc_status build_multi_plan(MultiPlan *pl, const mc_run_config *cfgs) {
    const int np = (int)pl->ps.size();
    mc_problem *e = pl->ps[0];
    std::vector<MarchParams<T>> mp(np);
    std::vector<RayConsts<T>> rc(np);
    std::vector<PriorParams<T>> pp(np);
    std::vector<ProposeDesc<T>> pd(np);
    std::vector<uint64_t *> steps(np);
    for (int i = 0; i < np; ++i) {
        mc_problem *p = pl->ps[i];
        const T *prop = (const T *)p->prop.p;
        mp[i] = march_params<T>(p, prop, nullptr, (double *)p->partials.p);
        mp[i].n_chains = pl->n[i];
        rc[i] = ray_consts<T>(p);
        pp[i] = prior_params<T>(p, prop, (const double *)p->partials.p);
        pp[i].mh = 1;
        pp[i].lp_cur = (double *)pl->lp[i];
        pp[i].n_acc = (int64_t *)pl->acc[i];
        pp[i].state = (T *)pl->H[i];
        pp[i].seed = cfgs[i].seed;
        pp[i].step_base = p->d_step;
        if (cfgs[i].r_state) {
            pp[i].r_chain = cfgs[i].r_state;
            pp[i].sample_r = 1;
            pp[i].r_step = cfgs[i].r_step;
            pp[i].n_acc_r = cfgs[i].n_accept_r;
            pp[i].stat_sw2 = (double *)p->rstat.p;
            pp[i].stat_se = (double *)p->rstat.p + (size_t)pl->n[i] * (S - 1);
        }
        pd[i].H = (const T *)pl->H[i];
        pd[i].prop = (T *)p->prop.p;
        pd[i].M = (S - 1) * p->R * p->C;
        pd[i].sigma = cfgs[i].step_size;
        pd[i].seed = cfgs[i].seed;
        pd[i].step_base = p->d_step;
        steps[i] = p->d_step;
    }
    mc_status s;
    if ((s = upload_vec(e, pl->d_mp, mp)) != MC_OK) return s;
    if ((s = upload_vec(e, pl->d_rc, rc)) != MC_OK) return s;
    if ((s = upload_vec(e, pl->d_pp, pp)) != MC_OK) return s;
    if ((s = upload_vec(e, pl->d_pd, pd)) != MC_OK) return s;
    if ((s = upload_vec(e, pl->d_step_ptrs, steps)) != MC_OK) return s;
    std::vector<uint64_t> zero(np, 0);
    if ((s = upload_vec(e, pl->d_step_vals, zero)) != MC_OK) return s;
    // chains, largest grids first
    std::vector<int> order(np);
    for (int i = 0; i < np; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
        return (size_t)pl->ps[a]->R * pl->ps[a]->C > (size_t)pl->ps[b]->R * pl->ps[b]->C;
    });
    // chain items, large grids (1024-thread prior blocks) first
    std::vector<int2> chains;
    size_t lds_large = 0, lds_small = 0;
    int n_large = 0;
    for (int i : order) {
        const size_t N = (size_t)pl->ps[i]->R * pl->ps[i]->C;
        const bool large = N >= (size_t)kPriorLargeNodes;
        for (int c = 0; c < pl->n[i]; ++c) chains.push_back(make_int2(i, c));
        if (large) n_large += pl->n[i];
        (large ? lds_large : lds_small) = std::max(large ? lds_large : lds_small, sizeof(T) * N);
    }
    pl->n_chain_items = (int)chains.size();
    pl->n_chain_items_large = n_large;
    pl->prior_lds = lds_small;
    pl->prior_lds_large = lds_large;
    if ((s = upload_vec(e, pl->d_chain_items, chains)) != MC_OK) return s;
    // march classes: one per (grid size, top placement, block size), heaviest
    // first; items within a class sorted by decreasing ray count
    std::map<std::tuple<size_t, int, int>, std::vector<int>> cls;
    std::map<std::tuple<size_t, int, int>, double> work;
    for (int i = 0; i < np; ++i) {
        mc_problem *p = pl->ps[i];
        if (p->n_ray == 0) continue;
        size_t N = (size_t)p->R * p->C;
        bool tl = N * S * sizeof(T) + 16384 <= p->max_lds;
        int block = std::is_same<T, float>::value ? p->tune.block : kMultiBlock;
        auto key = std::make_tuple(N, tl ? 1 : 0, block);
        cls[key].push_back(i);
        work[key] += (double)pl->n[i] * p->n_ray * std::sqrt((double)N);
    }
    std::vector<std::tuple<size_t, int, int>> keys;
    for (auto &kv : cls) keys.push_back(kv.first);
    std::stable_sort(keys.begin(), keys.end(), [&](const auto &a, const auto &b) { return work[a] > work[b]; });
    for (auto &key : keys) {
        MultiClass mc_;
        mc_.top_lds = std::get<1>(key) != 0;
        mc_.block = std::get<2>(key);
        mc_.lds = std::get<0>(key) * (mc_.top_lds ? S : S - 1) * sizeof(T);
        if (mc_.lds + 2048 > e->max_lds) return fail(e, MC_ERR_UNSUPPORTED, "grid too large for LDS");
        std::vector<int> members = cls[key];
        std::stable_sort(members.begin(), members.end(), [&](int a, int b) {
            return tiling(pl->ps[a]).rays_per_block > tiling(pl->ps[b]).rays_per_block;
        });
        // XCD-aware order: item j runs on XCD j % kXcds; each chain's tiles
        // go to one XCD (the least loaded so far), in consecutive slots, so
        // its surfaces are read from HBM once.  Short lanes are padded with
        // items the kernel skips (problem -1).
        std::vector<int4> lane[kXcds];
        for (int i : members) {
            Tiling t = tiling(pl->ps[i]);
            for (int c = 0; c < pl->n[i]; ++c) {
                int x = 0;
                for (int q = 1; q < kXcds; ++q)
                    if (lane[q].size() < lane[x].size()) x = q;
                for (int tt = 0; tt < t.n_tiles; ++tt) lane[x].push_back(make_int4(i, c, tt, 0));
            }
        }
        size_t L = 0;
        for (auto &v : lane) L = std::max(L, v.size());
        std::vector<int4> items(L * kXcds, make_int4(-1, 0, 0, 0));
        for (int x = 0; x < kXcds; ++x)
            for (size_t k = 0; k < lane[x].size(); ++k) items[k * kXcds + x] = lane[x][k];
        mc_.n_items = (int)items.size();
        if ((s = upload_vec(e, mc_.items, items)) != MC_OK) return s;
        if (!pl->classes.empty()) {
            HIP_TRY(e, hipStreamCreateWithFlags(&mc_.side, hipStreamNonBlocking));
            HIP_TRY(e, hipEventCreateWithFlags(&mc_.done, hipEventDisableTiming));
        }
        pl->classes.push_back(mc_);
    }
    if (pl->classes.size() > 1) HIP_TRY(e, hipEventCreateWithFlags(&pl->fork, hipEventDisableTiming));
    int ncu = 256;
    (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, pl->device);
    pl->persistent_blocks = e->tune.multi_blocks_per_cu > 0 ? e->tune.multi_blocks_per_cu * ncu : INT32_MAX;
    return MC_OK;
}

template <int S, bool TL, int B, bool PERSIST>
void launch_multi4_shape(const MultiPlan *pl, const MultiClass &c, int grid, hipStream_t st) {
    auto kk = k_march_multi4<S, TL, B, PERSIST>;
    if (c.lds > 65536) (void)hipFuncSetAttribute((const void *)kk, hipFuncAttributeMaxDynamicSharedMemorySize, (int)c.lds);
    hipLaunchKernelGGL(kk, dim3(grid), dim3(B), c.lds, st, (const MarchParams<float> *)pl->d_mp,
                       (const RayConsts<float> *)pl->d_rc, (const int4 *)c.items, c.n_items);
}

template <int S, bool TL, int B>
void launch_multi4(const MultiPlan *pl, const MultiClass &c, int grid, hipStream_t st) {
    if (grid < c.n_items) launch_multi4_shape<S, TL, B, true>(pl, c, grid, st);
    else launch_multi4_shape<S, TL, B, false>(pl, c, grid, st);
}

template <typename T, int S, bool TL, bool PERSIST>
void launch_multi3_shape(const MultiPlan *pl, const MultiClass &c, int grid, hipStream_t st) {
    auto kk = k_march_multi3<T, S, TL, kMultiBlock, PERSIST>;
    if (c.lds > 65536) (void)hipFuncSetAttribute((const void *)kk, hipFuncAttributeMaxDynamicSharedMemorySize, (int)c.lds);
    hipLaunchKernelGGL(kk, dim3(grid), dim3(kMultiBlock), c.lds, st, (const MarchParams<T> *)pl->d_mp,
                       (const RayConsts<T> *)pl->d_rc, (const int4 *)c.items, c.n_items);
}

template <typename T, int S, bool TL>
void launch_multi3(const MultiPlan *pl, const MultiClass &c, int grid, hipStream_t st) {
    if (grid < c.n_items) launch_multi3_shape<T, S, TL, true>(pl, c, grid, st);
    else launch_multi3_shape<T, S, TL, false>(pl, c, grid, st);
}

template <typename T, int S>
void launch_multi_class(const MultiPlan *pl, const MultiClass &c, hipStream_t st) {
    const int grid = std::min(c.n_items, pl->persistent_blocks);
    if (grid <= 0) return;
    if constexpr (std::is_same<T, float>::value) {
        if (c.top_lds) {
            if (c.block == 256) launch_multi4<S, true, 256>(pl, c, grid, st);
            else if (c.block == 512) launch_multi4<S, true, 512>(pl, c, grid, st);
            else launch_multi4<S, true, 1024>(pl, c, grid, st);
        } else {
            if (c.block == 256) launch_multi4<S, false, 256>(pl, c, grid, st);
            else if (c.block == 512) launch_multi4<S, false, 512>(pl, c, grid, st);
            else launch_multi4<S, false, 1024>(pl, c, grid, st);
        }
    } else {
        if (c.top_lds) launch_multi3<T, S, true>(pl, c, grid, st);
        else launch_multi3<T, S, false>(pl, c, grid, st);
    }
}

// One MCMC step of every chain of every problem: proposal, the march classes
// (concurrently, on forked streams), then the prior and Metropolis step.
template <typename T, int S>
mc_status multi_step(MultiPlan *pl, int k, hipStream_t st) {
    mc_problem *e = pl->ps[0];
    hipLaunchKernelGGL(k_propose_multi<T>, dim3(pl->n_chain_items), dim3(256), 0, st,
                       (const ProposeDesc<T> *)pl->d_pd, (const int2 *)pl->d_chain_items, k);
    HIP_TRY(e, hipGetLastError());
    const size_t nc = pl->classes.size();
    if (nc > 1) {
        HIP_TRY(e, hipEventRecord(pl->fork, st));
        for (size_t c = 1; c < nc; ++c) HIP_TRY(e, hipStreamWaitEvent(pl->classes[c].side, pl->fork, 0));
    }
    for (size_t c = 0; c < nc; ++c) {
        const MultiClass &mc_ = pl->classes[c];
        hipStream_t cs = c == 0 ? st : mc_.side;
        launch_multi_class<T, S>(pl, mc_, cs);
        HIP_TRY(e, hipGetLastError());
        if (c > 0) HIP_TRY(e, hipEventRecord(mc_.done, cs));
    }
    for (size_t c = 1; c < nc; ++c) HIP_TRY(e, hipStreamWaitEvent(st, pl->classes[c].done, 0));
    const int2 *items = (const int2 *)pl->d_chain_items;
    const int nl = pl->n_chain_items_large, ns = pl->n_chain_items - nl;
    if (nl > 0) {
        auto kp = pl->hier ? k_prior_multi<T, S, kPriorBlockLarge, true> : k_prior_multi<T, S, kPriorBlockLarge, false>;
        if (pl->prior_lds_large > 65536)
            (void)hipFuncSetAttribute((const void *)kp, hipFuncAttributeMaxDynamicSharedMemorySize, (int)pl->prior_lds_large);
        hipLaunchKernelGGL(kp, dim3(nl), dim3(kPriorBlockLarge), pl->prior_lds_large, st,
                           (const PriorParams<T> *)pl->d_pp, items, k);
    }
    if (ns > 0) {
        auto kp = pl->hier ? k_prior_multi<T, S, kPriorBlock, true> : k_prior_multi<T, S, kPriorBlock, false>;
        if (pl->prior_lds > 65536)
            (void)hipFuncSetAttribute((const void *)kp, hipFuncAttributeMaxDynamicSharedMemorySize, (int)pl->prior_lds);
        hipLaunchKernelGGL(kp, dim3(ns), dim3(kPriorBlock), pl->prior_lds, st, (const PriorParams<T> *)pl->d_pp,
                           items + nl, k);
    }
    HIP_TRY(e, hipGetLastError());
    return MC_OK;
}

// init_lp: compute the log posterior of chains whose entry is NaN first (the
// public entry point); the serving loop computes it once at admission.
template <typename T, int S>
mc_status mcmc_multi_impl(int np, mc_problem *const *ps, const mc_run_config *cfgs, const int *n_chains,
                          void *const *heights, double *const *lps, int64_t *const *accs, hipStream_t st,
                          bool init_lp = true) {
    mc_problem *e = ps[0];
    mc_status s;
    // workspaces and initial log posteriors, per problem
    for (int i = 0; i < np; ++i) {
        mc_problem *p = ps[i];
        const int n = n_chains[i];
        const int M = (S - 1) * p->R * p->C;
        Tiling t = tiling(p);
        if ((s = ensure(p, p->prop, sizeof(T) * (size_t)n * M)) != MC_OK) return s;
        if ((s = ensure(p, p->lptmp, sizeof(double) * (size_t)n)) != MC_OK) return s;
        if (p->n_ray > 0 && (s = ensure(p, p->partials, sizeof(double) * (size_t)n * t.n_tiles)) != MC_OK) return s;
        if (cfgs[i].r_state) {
            // with r sampled: log posterior and w-statistics of every chain at its own r
            // (always: the statistics feed the r updates)
            if ((s = ensure(p, p->rstat, 2 * sizeof(double) * (size_t)n * (S - 1))) != MC_OK) return s;
            if ((s = logpost_impl<T, S>(p, n, (const T *)heights[i], lps[i], nullptr, st, nullptr, cfgs[i].r_state,
                                        (double *)p->rstat.p)) != MC_OK)
                return s;
            continue;
        }
        if (!init_lp) continue;
        if ((s = logpost_impl<T, S>(p, n, (const T *)heights[i], (double *)p->lptmp.p, nullptr, st, lps[i])) != MC_OK)
            return s;
        hipLaunchKernelGGL(k_fill_nan, dim3((n + 255) / 256), dim3(256), 0, st, lps[i], (const double *)p->lptmp.p, n);
        HIP_TRY(p, hipGetLastError());
    }
    // find or build the plan
    MultiPlan *pl = nullptr;
    const int G = cfgs[0].graph_steps < 1 ? 1 : cfgs[0].graph_steps;
    for (MultiPlan *q : g_multi_plans) {
        bool same = (int)q->ps.size() == np && q->G == G;
        for (int i = 0; same && i < np; ++i)
            same = q->ps[i] == ps[i] && q->n[i] == n_chains[i] && q->H[i] == heights[i] && q->lp[i] == lps[i] &&
                   q->acc[i] == accs[i] && q->gens[i] == ps[i]->gen && q->seeds[i] == cfgs[i].seed &&
                   q->sigma[i] == cfgs[i].step_size && q->r[i] == cfgs[i].r_state &&
                   q->acc_r[i] == cfgs[i].n_accept_r && q->r_step[i] == cfgs[i].r_step;
        if (same) {
            pl = q;
            break;
        }
    }
    if (!pl) {
        pl = new MultiPlan();
        pl->G = G;
        pl->device = e->device;
        for (int i = 0; i < np; ++i) {
            pl->ps.push_back(ps[i]);
            pl->n.push_back(n_chains[i]);
            pl->H.push_back(heights[i]);
            pl->lp.push_back(lps[i]);
            pl->acc.push_back(accs[i]);
            pl->gens.push_back(ps[i]->gen);
            pl->seeds.push_back(cfgs[i].seed);
            pl->sigma.push_back(cfgs[i].step_size);
            pl->r.push_back(cfgs[i].r_state);
            pl->acc_r.push_back(cfgs[i].n_accept_r);
            pl->r_step.push_back(cfgs[i].r_state ? cfgs[i].r_step : 0.0);
        }
        pl->hier = cfgs[0].r_state != nullptr;
        if ((s = build_multi_plan<T, S>(pl, cfgs)) != MC_OK) {
            delete pl;
            return s;
        }
        g_multi_plans.push_back(pl);
        if (g_multi_plans.size() > 4) {
            delete g_multi_plans.front();
            g_multi_plans.erase(g_multi_plans.begin());
        }
    }
    // step counters of every problem
    std::vector<uint64_t> offs(np);
    for (int i = 0; i < np; ++i) offs[i] = cfgs[i].step_offset;
    HIP_TRY(e, hipMemcpyAsync(pl->d_step_vals, offs.data(), sizeof(uint64_t) * np, hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL(k_set_u64_multi, dim3((np + 255) / 256), dim3(256), 0, st, (uint64_t *const *)pl->d_step_ptrs,
                       (const uint64_t *)pl->d_step_vals, np);
    HIP_TRY(e, hipGetLastError());
    HIP_TRY(e, hipStreamSynchronize(st));   // the host step-offset array goes out of scope
    const int64_t n_steps = cfgs[0].n_steps;
    int64_t done = 0;
    if (G > 1 && n_steps >= G) {
        if (!pl->gexec) {
            if (!pl->cap) HIP_TRY(e, hipStreamCreateWithFlags(&pl->cap, hipStreamNonBlocking));
            HIP_TRY(e, hipStreamBeginCapture(pl->cap, hipStreamCaptureModeThreadLocal));
            mc_status cs = MC_OK;
            for (int k = 0; k < G && cs == MC_OK; ++k) cs = multi_step<T, S>(pl, k, pl->cap);
            if (cs == MC_OK)
                hipLaunchKernelGGL(k_add_u64_multi, dim3((np + 255) / 256), dim3(256), 0, pl->cap,
                                   (uint64_t *const *)pl->d_step_ptrs, np, (uint64_t)G);
            hipGraph_t graph = nullptr;
            hipError_t er = hipStreamEndCapture(pl->cap, &graph);
            if (cs != MC_OK) {
                if (graph) (void)hipGraphDestroy(graph);
                return cs;
            }
            if (er != hipSuccess) return fail(e, MC_ERR_DEVICE, "graph capture: %s", hipGetErrorString(er));
            er = hipGraphInstantiate(&pl->gexec, graph, nullptr, nullptr, 0);
            (void)hipGraphDestroy(graph);
            if (er != hipSuccess) {
                pl->gexec = nullptr;
                return fail(e, MC_ERR_DEVICE, "graph instantiate: %s", hipGetErrorString(er));
            }
        }
        for (; done + G <= n_steps; done += G) HIP_TRY(e, hipGraphLaunch(pl->gexec, st));
    }
    const int64_t rest = n_steps - done;
    for (int64_t k = 0; k < rest; ++k)
        if ((s = multi_step<T, S>(pl, (int)k, st)) != MC_OK) return s;
    if (rest > 0)
        hipLaunchKernelGGL(k_add_u64_multi, dim3((np + 255) / 256), dim3(256), 0, st, (uint64_t *const *)pl->d_step_ptrs,
                           np, (uint64_t)rest);
    HIP_TRY(e, hipGetLastError());
    return MC_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------

extern "C" {

const char *mc_version(void) { return "muoncave 0.1 (gfx950)"; }

mc_status mc_create(int hip_device, int precision, mc_problem **out) {
    if (!out) return fail(nullptr, MC_ERR_ARG, "out is NULL");
    *out = nullptr;
    if (precision != MC_F32 && precision != MC_F64) return fail(nullptr, MC_ERR_ARG, "precision %d", precision);
    int count = 0;
    hipError_t e = hipGetDeviceCount(&count);
    if (e != hipSuccess || count <= 0) return fail(nullptr, MC_ERR_DEVICE, "no HIP device");
    if (hip_device < 0 || hip_device >= count) return fail(nullptr, MC_ERR_ARG, "device %d of %d", hip_device, count);
    mc_problem *p = new mc_problem();
    p->device = hip_device;
    p->prec = precision;
    p->tune = default_tuning(precision, 64 * 64);
    DeviceGuard g(hip_device);
    {
        // once per device, with that device current
        std::lock_guard<std::mutex> lk(g_scratch_mu);
        if (!g_scratch_ptr.count(hip_device)) {
            double *ptr = nullptr;
            hipError_t se = hipGetSymbolAddress((void **)&ptr, HIP_SYMBOL(scratch));
            if (se != hipSuccess || !ptr) {
                delete p;
                return fail(nullptr, MC_ERR_DEVICE, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(se));
            }
            g_scratch_ptr[hip_device] = ptr;
        }
    }
    int lds = 0;
    if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, hip_device) == hipSuccess && lds > 0)
        p->max_lds = (size_t)lds;
    if (hipMalloc((void **)&p->d_step, sizeof(uint64_t)) != hipSuccess) {
        delete p;
        return fail(nullptr, MC_ERR_NOMEM, "hipMalloc failed");
    }
    *out = p;
    return MC_OK;
}

void mc_destroy(mc_problem *p) {
    if (!p) return;
    DeviceGuard g(p->device);
    (void)hipDeviceSynchronize();
    std::lock_guard<std::mutex> lock(g_multi_mu);
    for (size_t i = 0; i < g_multi_plans.size();) {
        MultiPlan *q = g_multi_plans[i];
        if (std::find(q->ps.begin(), q->ps.end(), p) != q->ps.end()) {
            delete q;
            g_multi_plans.erase(g_multi_plans.begin() + i);
        } else {
            ++i;
        }
    }
    drop_graph(p);   // destroys and clears the graph, so nothing below destroys it again
    if (p->cap_stream) (void)hipStreamDestroy(p->cap_stream);
    free_ptr(p->d_top);
    free_ptr(p->d_top64);
    free_ptr(p->d_eig_g);
    free_ptr(p->d_eig_w);
    free_ptr(p->d_sensor);
    free_ptr(p->d_dx);
    free_ptr(p->d_dy);
    free_ptr(p->d_dz);
    free_ptr(p->d_expo);
    free_ptr(p->d_coL);
    free_ptr(p->d_cnt64);
    clear_voxel_model(p);
    for (double **q : {&p->d_quad_w, &p->d_quad_tab, &p->d_quad_cnt}) free_ptr(*q);
    for (int k = 0; k < 6; ++k) free_ptr(p->d_rc[k]);
    for (DevBuf *b : {&p->partials, &p->prop, &p->lptmp, &p->obuf, &p->gfix, &p->gcur, &p->gprop,
                      &p->lpprop, &p->rstat, &p->rhat, &p->nutsbuf, &p->xrec, &p->xcnt, &p->xovf, &p->xgp,
                      &p->valpha})
        if (b->p) (void)hipFree(b->p);
    if (p->d_step) (void)hipFree(p->d_step);
    delete p;
}

const char *mc_last_error(const mc_problem *p) { return p ? p->err.c_str() : g_create_error.c_str(); }

mc_status load_geometry_grid(mc_problem *p, int n_surfaces, int n_rows, int n_cols, double extent_x_m,
                             double extent_y_m, const double *density, const double *top, const double *car_r) {
    if (!p) return MC_ERR_ARG;
    if (n_surfaces < 2 || n_surfaces > kMaxSurfaces) return fail(p, MC_ERR_ARG, "n_surfaces %d not in [2,4]", n_surfaces);
    if (n_rows < 3 || n_cols < 3 || n_rows > 256 || n_cols > 256 || n_rows * n_cols > kMaxNodes)
        return fail(p, MC_ERR_ARG, "grid %dx%d: need 3 <= side <= 256 and rows*cols <= %d", n_rows, n_cols, kMaxNodes);
    if (!(extent_x_m > 0) || !(extent_y_m > 0) || !std::isfinite(extent_x_m) || !std::isfinite(extent_y_m))
        return fail(p, MC_ERR_ARG, "extents must be positive");
    if (!density || !top || !car_r) return fail(p, MC_ERR_ARG, "NULL array");
    for (int l = 0; l < n_surfaces; ++l)
        if (!(density[l] >= 0) || !std::isfinite(density[l])) return fail(p, MC_ERR_ARG, "density[%d] invalid", l);
    for (int l = 0; l < n_surfaces - 1; ++l)
        if (!(car_r[l] >= 0.0 && car_r[l] < 1.0)) return fail(p, MC_ERR_ARG, "car_r[%d] not in [0,1)", l);
    const int N = n_rows * n_cols;
    double tmin = INFINITY, tmax = -INFINITY;
    for (int i = 0; i < N; ++i) {
        if (!(top[i] > 0) || !std::isfinite(top[i])) return fail(p, MC_ERR_ARG, "top[%d] must be > 0", i);
        tmin = std::min(tmin, top[i]);
        tmax = std::max(tmax, top[i]);
    }
    DeviceGuard g(p->device);
    p->have_geom = p->have_sensors = p->have_counts = false;
    clear_voxel_model(p);
    clear_quadrature(p);
    p->S = n_surfaces;
    p->R = n_rows;
    p->C = n_cols;
    p->X = extent_x_m;
    p->Y = extent_y_m;
    p->density.assign(density, density + n_surfaces);
    p->top.assign(top, top + N);
    p->car_r.assign(car_r, car_r + n_surfaces - 1);
    p->ztop = tmax;
    p->sum_log_top = 0.0;
    for (int i = 0; i < N; ++i) p->sum_log_top += std::log(top[i]);
    p->top_min = tmin;
    p->top_max = tmax;
    p->logdet.resize(n_surfaces - 1);
    p->s11.resize(n_surfaces - 1);
    for (int l = 0; l < n_surfaces - 1; ++l) torus_car_constants(n_rows, n_cols, car_r[l], p->logdet[l], p->s11[l]);
    mc_status s;
    {
        // distinct g = cos(2 pi k/R) + cos(2 pi m/C) over k <= R/2, m <= C/2 with
        // multiplicities (k and R-k give the same cosine), for per-chain r
        std::vector<double> eg, ew;
        for (int k = 0; k <= n_rows / 2; ++k) {
            const double wk = (k == 0 || 2 * k == n_rows) ? 1.0 : 2.0;
            for (int m = 0; m <= n_cols / 2; ++m) {
                const double wm = (m == 0 || 2 * m == n_cols) ? 1.0 : 2.0;
                eg.push_back(std::cos(2.0 * M_PI * k / n_rows) + std::cos(2.0 * M_PI * m / n_cols));
                ew.push_back(wk * wm);
            }
        }
        void *q = p->d_eig_g;
        if ((s = upload<double>(p, q, eg)) != MC_OK) return s;
        p->d_eig_g = (double *)q;
        q = p->d_eig_w;
        if ((s = upload<double>(p, q, ew)) != MC_OK) return s;
        p->d_eig_w = (double *)q;
        p->n_eig = (int)eg.size();
    }
    if ((s = upload_prec(p, p->d_top, p->top)) != MC_OK) return s;
    void *t64 = p->d_top64;
    if ((s = upload<double>(p, t64, p->top)) != MC_OK) return s;
    p->d_top64 = (double *)t64;
    if (!p->tune_user) p->tune = default_tuning(p->prec, (size_t)N);
    drop_graph(p);
    p->have_geom = true;
    return MC_OK;
}

mc_status set_sensors(mc_problem *p, int n_sensors, const double *pos, int n_pix, const double *dirs,
                      const double *exposure, double atten_len) {
    if (!p) return MC_ERR_ARG;
    if (!p->have_geom) return fail(p, MC_ERR_STATE, "load_geometry_grid has not been called");
    if (n_sensors < 0 || n_pix < 0) return fail(p, MC_ERR_ARG, "negative sizes");
    if (n_sensors > 0 && n_pix == 0) return fail(p, MC_ERR_ARG, "n_pix must be > 0 when there are sensors");
    if ((long long)n_sensors * n_pix > (1LL << 30)) return fail(p, MC_ERR_ARG, "too many rays");
    if (!(atten_len > 0) || !std::isfinite(atten_len)) return fail(p, MC_ERR_ARG, "atten_len must be > 0");
    const int n_ray = n_sensors * n_pix;
    if (n_ray > 0 && (!pos || !dirs || !exposure)) return fail(p, MC_ERR_ARG, "NULL array");
    for (int s = 0; s < n_sensors; ++s) {
        double x = pos[3 * s], y = pos[3 * s + 1], z = pos[3 * s + 2];
        if (!(x >= 0 && x <= p->X && y >= 0 && y <= p->Y && z >= 0 && z < p->ztop))
            return fail(p, MC_ERR_ARG, "sensor %d outside the box", s);
    }
    for (int r = 0; r < n_ray; ++r) {
        double dx = dirs[3 * r], dy = dirs[3 * r + 1], dz = dirs[3 * r + 2];
        double nrm = std::sqrt(dx * dx + dy * dy + dz * dz);
        if (!(dz > 0) || !(std::fabs(nrm - 1.0) < 1e-6)) return fail(p, MC_ERR_ARG, "dirs[%d] must be a unit vector with d_z > 0", r);
        if (!(exposure[r] > 0) || !std::isfinite(exposure[r])) return fail(p, MC_ERR_ARG, "exposure[%d] must be > 0", r);
    }
    DeviceGuard g(p->device);
    p->have_sensors = p->have_counts = false;
    clear_voxel_model(p);
    clear_quadrature(p);
    p->n_s = n_sensors;
    p->n_pix = n_pix;
    p->n_ray = n_ray;
    p->atten = atten_len;
    p->pos.assign(pos, pos + 3 * (size_t)n_sensors);
    std::vector<double> dx(n_ray), dy(n_ray), dz(n_ray);
    for (int r = 0; r < n_ray; ++r) {
        dx[r] = dirs[3 * r];
        dy[r] = dirs[3 * r + 1];
        dz[r] = dirs[3 * r + 2];
    }
    p->expo.assign(exposure, exposure + n_ray);
    p->dirs.assign(dirs, dirs + 3 * (size_t)n_ray);
    // chain-independent per-ray constants of the cell walk, in float64 then
    // rounded once: reciprocal directions, DDA offsets -q/d, box exit
    std::vector<double> rc[6];
    for (auto &v : rc) v.resize(n_ray);
    const double xmax = (double)(p->R - 1) * (p->X / (p->R - 1)), ymax = (double)(p->C - 1) * (p->Y / (p->C - 1));
    for (int r = 0; r < n_ray; ++r) {
        const int sidx = r / n_pix;
        const double qx = pos[3 * sidx], qy = pos[3 * sidx + 1], qz = pos[3 * sidx + 2];
        const double ix = dx[r] != 0 ? 1.0 / dx[r] : 0.0, iy = dy[r] != 0 ? 1.0 / dy[r] : 0.0;
        rc[0][r] = ix;
        rc[1][r] = iy;
        rc[2][r] = 1.0 / dz[r];
        rc[3][r] = dx[r] != 0 ? -qx * ix : INFINITY;
        rc[4][r] = dy[r] != 0 ? -qy * iy : INFINITY;
        double T = (p->ztop - qz) / dz[r];
        if (dx[r] > 0) T = std::min(T, (xmax - qx) / dx[r]);
        if (dx[r] < 0) T = std::min(T, -qx / dx[r]);
        if (dy[r] > 0) T = std::min(T, (ymax - qy) / dy[r]);
        if (dy[r] < 0) T = std::min(T, -qy / dy[r]);
        rc[5][r] = std::max(T, 0.0);
    }
    mc_status s;
    for (int k = 0; k < 6; ++k)
        if ((s = upload_prec(p, p->d_rc[k], rc[k])) != MC_OK) return s;
    if ((s = upload_prec(p, p->d_sensor, p->pos)) != MC_OK) return s;
    if ((s = upload_prec(p, p->d_dx, dx)) != MC_OK) return s;
    if ((s = upload_prec(p, p->d_dy, dy)) != MC_OK) return s;
    if ((s = upload_prec(p, p->d_dz, dz)) != MC_OK) return s;
    void *e = p->d_expo;
    if ((s = upload<double>(p, e, p->expo)) != MC_OK) return s;
    p->d_expo = (double *)e;
    drop_graph(p);
    p->have_sensors = true;
    return MC_OK;
}

mc_status set_counts(mc_problem *p, const int32_t *counts) {
    if (!p) return MC_ERR_ARG;
    if (!p->have_sensors) return fail(p, MC_ERR_STATE, "set_sensors has not been called");
    if (p->n_ray > 0 && !counts) return fail(p, MC_ERR_ARG, "counts is NULL");
    if (p->quad_nsub > 0) {
        // one count per pixel; the march's own per-ray terms see zero counts
        std::vector<double> cq(p->quad_npx), zero(p->n_ray, 0.0);
        long double KQ = 0;
        for (int i = 0; i < p->quad_npx; ++i) {
            if (counts[i] < 0) return fail(p, MC_ERR_ARG, "counts[%d] < 0", i);
            cq[i] = counts[i];
            KQ -= std::lgamma(cq[i] + 1.0);
        }
        DeviceGuard g(p->device);
        drop_graph(p);
        mc_status s;
        void *d = p->d_quad_cnt;
        if ((s = upload<double>(p, d, cq)) != MC_OK) return s;
        p->d_quad_cnt = (double *)d;
        d = p->d_coL;
        if ((s = upload<double>(p, d, zero)) != MC_OK) return s;
        p->d_coL = (double *)d;
        d = p->d_cnt64;
        if ((s = upload<double>(p, d, zero)) != MC_OK) return s;
        p->d_cnt64 = (double *)d;
        p->kconst = 0.0;
        p->kconst_quad = (double)KQ;
        p->have_counts = true;
        return MC_OK;
    }
    std::vector<double> coL(p->n_ray), c64(p->n_ray);
    long double K = 0, KV = 0;
    for (int r = 0; r < p->n_ray; ++r) {
        if (counts[r] < 0) return fail(p, MC_ERR_ARG, "counts[%d] < 0", r);
        double c = counts[r];
        coL[r] = c / p->atten;
        c64[r] = c;
        K += c * std::log(p->expo[r]) - std::lgamma(c + 1.0);
        KV -= std::lgamma(c + 1.0);
    }
    DeviceGuard g(p->device);
    drop_graph(p);   // the graph holds the old count pointer and constant
    void *d = p->d_coL;
    mc_status s;
    if ((s = upload<double>(p, d, coL)) != MC_OK) return s;
    p->d_coL = (double *)d;
    d = p->d_cnt64;
    if ((s = upload<double>(p, d, c64)) != MC_OK) return s;
    p->d_cnt64 = (double *)d;
    p->kconst = (double)K;
    p->kconst_vox = (double)KV;
    p->have_counts = true;
    return MC_OK;
}

mc_status logpost_batch_noalloc(mc_problem *p, int n_chains, const void *heights, double *logpost, void *opacity,
                                void *stream) {
    mc_status s = check_ready(p);
    if (s != MC_OK) return s;
    if (n_chains < 0) return fail(p, MC_ERR_ARG, "n_chains < 0");
    if (n_chains == 0) return MC_OK;
    if (!heights || !logpost) return fail(p, MC_ERR_ARG, "NULL device pointer");
    if (n_chains > 65535) return fail(p, MC_ERR_ARG, "n_chains > 65535");
    if (p->vox_nz > 0 || p->quad_nsub > 0)
        return fail(p, MC_ERR_UNSUPPORTED, "logpost_batch_noalloc runs the exact march with one ray per pixel only");
    const size_t need = p->n_ray > 0 ? (size_t)n_chains * (size_t)tiling(p).n_tiles : 0;
    if (need > kScratchDoubles)
        return fail(p, MC_ERR_ARG,
                    "logpost_batch_noalloc: %d chains x %d ray tiles = %zu partial sums exceed its fixed workspace "
                    "of %zu (fewer chains per call, or more rays per thread)",
                    n_chains, tiling(p).n_tiles, need, kScratchDoubles);
    double *ws = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_scratch_mu);
        auto it = g_scratch_ptr.find(p->device);
        if (it != g_scratch_ptr.end()) ws = it->second;
    }
    if (!ws) return fail(p, MC_ERR_STATE, "no workspace address for device %d", p->device);
    DeviceGuard g(p->device);
    hipStream_t st = (hipStream_t)stream;
    return p->prec == MC_F64 ? logpost_noalloc_dispatch<double>(p, n_chains, heights, logpost, opacity, st, ws)
                             : logpost_noalloc_dispatch<float>(p, n_chains, heights, logpost, opacity, st, ws);
}

mc_status logpost_batch(mc_problem *p, int n_chains, const void *heights, double *logpost, void *opacity,
                        void *stream) {
    mc_status s = check_ready(p);
    if (s != MC_OK) return s;
    if (n_chains < 0) return fail(p, MC_ERR_ARG, "n_chains < 0");
    if (n_chains == 0) return MC_OK;
    if (!heights || !logpost) return fail(p, MC_ERR_ARG, "NULL device pointer");
    if (n_chains > 65535) return fail(p, MC_ERR_ARG, "n_chains > 65535");
    DeviceGuard g(p->device);
    hipStream_t st = (hipStream_t)stream;
    return p->prec == MC_F64 ? logpost_dispatch<double>(p, n_chains, heights, logpost, opacity, st)
                             : logpost_dispatch<float>(p, n_chains, heights, logpost, opacity, st);
}

mc_status logpost_grad_batch(mc_problem *p, int n_chains, const void *heights, double *logpost, void *grad,
                             void *stream) {
    mc_status s = check_ready(p);
    if (s != MC_OK) return s;
    if (n_chains < 0) return fail(p, MC_ERR_ARG, "n_chains < 0");
    if (n_chains == 0) return MC_OK;
    if (!heights || !logpost || !grad) return fail(p, MC_ERR_ARG, "NULL device pointer");
    if (n_chains > 65535) return fail(p, MC_ERR_ARG, "n_chains > 65535");
    DeviceGuard g(p->device);
    hipStream_t st = (hipStream_t)stream;
    return p->prec == MC_F64 ? logpost_grad_dispatch<double>(p, n_chains, heights, logpost, grad, st)
                             : logpost_grad_dispatch<float>(p, n_chains, heights, logpost, grad, st);
}

mc_status mcmc_run(mc_problem *p, const mc_run_config *cfg, int n_chains, void *heights, double *logpost,
                   int64_t *n_accept, void *stream) {
    mc_status s = check_ready(p);
    if (s != MC_OK) return s;
    if (!cfg) return fail(p, MC_ERR_ARG, "cfg is NULL");
    if (n_chains < 0 || cfg->n_steps < 0) return fail(p, MC_ERR_ARG, "negative sizes");
    if (n_chains == 0) return MC_OK;
    if (n_chains > 65535) return fail(p, MC_ERR_ARG, "n_chains > 65535");
    if (!heights || !logpost || !n_accept) return fail(p, MC_ERR_ARG, "NULL device pointer");
    if (!(cfg->step_size >= 0) || !std::isfinite(cfg->step_size)) return fail(p, MC_ERR_ARG, "step_size invalid");
    if (cfg->kernel != 0 && cfg->kernel != 1) return fail(p, MC_ERR_ARG, "kernel %d", cfg->kernel);
    if (cfg->r_state && cfg->kernel != 0) return fail(p, MC_ERR_UNSUPPORTED, "r sampling runs with random-walk Metropolis");
    if (cfg->r_state && (!(cfg->r_step >= 0) || !std::isfinite(cfg->r_step))) return fail(p, MC_ERR_ARG, "r_step invalid");
    if (cfg->n_accept_r && !cfg->r_state) return fail(p, MC_ERR_ARG, "n_accept_r without r_state");
    if (cfg->step_offset + (uint64_t)cfg->n_steps >= (1ULL << 48)) return fail(p, MC_ERR_ARG, "step counter exceeds 48 bits");
    DeviceGuard g(p->device);
    hipStream_t st = (hipStream_t)stream;
    return p->prec == MC_F64 ? mcmc_dispatch<double>(p, cfg, n_chains, heights, logpost, n_accept, st)
                             : mcmc_dispatch<float>(p, cfg, n_chains, heights, logpost, n_accept, st);
}

}  // extern "C"

// ---------------------------------------------------------------------------
// The latent parametrisation
// ---------------------------------------------------------------------------

template <typename T>
LatentParams<T> latent_params(const mc_problem *p, int n, const T *x, T *H, double *lp, T *gx) {
    LatentParams<T> L;
    memset(&L, 0, sizeof(L));
    L.R = p->R;
    L.C = p->C;
    L.N = p->R * p->C;
    L.S1 = p->S - 1;
    L.SN = p->S * L.N;
    L.n = n;
    L.n_tiles = tiling(p).n_tiles;
    L.has_lik = p->n_ray > 0 ? 1 : 0;
    for (int l = 0; l < p->S - 1; ++l) {
        L.s[l] = std::sqrt(p->s11[l]);
        L.r[l] = p->car_r[l];
        L.logdet[l] = p->logdet[l];
    }
    L.kconst = p->kconst;
    L.xs = L.S1 * L.N;
    L.top64 = p->d_top64;
    L.x = x;
    L.H = H;
    L.gfix = (const unsigned long long *)p->gfix.p;
    L.partials = (const double *)p->partials.p;
    L.lp = lp;
    L.gx = gx;
    return L;
}

// Log density and gradient of the latent states x [n][S-1][R][C]; the
// heights go to p->prop (which must hold n states), the gradient to gx
// [n][S][R][C] (the top row zero).
template <typename T, int S>
mc_status grad_eval_latent(mc_problem *p, int n, const T *x, double *lp, T *gx, hipStream_t st) {
    const size_t N = (size_t)p->R * p->C;
    LatentParams<T> L = latent_params<T>(p, n, x, (T *)p->prop.p, lp, gx);
    hipLaunchKernelGGL(k_latent_to_heights<T>, dim3((unsigned)((N + 255) / 256), n), dim3(256), 0, st, L);
    HIP_TRY(p, hipGetLastError());
    mc_status s;
    if (p->n_ray > 0 && (s = lik_grad<T, S>(p, n, L.H, (unsigned long long *)p->gfix.p, st)) != MC_OK) return s;
    hipLaunchKernelGGL((k_latent_finish<T, S, 512>), dim3(n), dim3(512), 0, st, L);
    HIP_TRY(p, hipGetLastError());
    return MC_OK;
}

// The same with every chain's dependence parameters sampled: z [n][S1 N + S1]
// holds the fields, then logit r (the paper's latent vector of all
// unknowns); gz takes the logit-r gradient in the first S1 entries of the
// top row.  rc: [n][S1][kRc] scratch for the per-chain constants of r.
template <typename T, int S>
mc_status grad_eval_latent_r(mc_problem *p, int n, const T *z, double *lp, T *gz, double *rc, hipStream_t st) {
    const size_t N = (size_t)p->R * p->C;
    LatentParams<T> L = latent_params<T>(p, n, z, (T *)p->prop.p, lp, gz);
    L.xs = (S - 1) * (int)N + (S - 1);
    L.rc = rc;
    L.eig_g = p->d_eig_g;
    L.eig_w = p->d_eig_w;
    L.n_eig = p->n_eig;
    hipLaunchKernelGGL((k_latent_r_consts<T, 256>), dim3(n), dim3(256), 0, st, L);
    hipLaunchKernelGGL(k_latent_to_heights<T>, dim3((unsigned)((N + 255) / 256), n), dim3(256), 0, st, L);
    HIP_TRY(p, hipGetLastError());
    mc_status s;
    if (p->n_ray > 0 && (s = lik_grad<T, S>(p, n, L.H, (unsigned long long *)p->gfix.p, st)) != MC_OK) return s;
    hipLaunchKernelGGL((k_latent_finish<T, S, 512>), dim3(n), dim3(512), 0, st, L);
    HIP_TRY(p, hipGetLastError());
    return MC_OK;
}

// Packing of the sampler's state with r: z[c] = (x[c], logit r[c]) and back.
template <typename T>
__global__ void k_pack_latent_r(const T *x, const double *r, T *z, int M, int S1, int n) {
    const size_t c = blockIdx.y;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < M) z[c * (M + S1) + i] = x[c * M + i];
    else if (i < M + S1) {
        const double rv = r[c * S1 + (i - M)];
        z[c * (M + S1) + i] = (T)log(rv / (1.0 - rv));
    }
}

template <typename T>
__global__ void k_unpack_latent_r(const T *z, T *x, double *r, int M, int S1, int n) {
    const size_t c = blockIdx.y;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < M) x[c * M + i] = z[c * (M + S1) + i];
    else if (i < M + S1) r[c * S1 + (i - M)] = 1.0 / (1.0 + exp(-(double)z[c * (M + S1) + i]));
}

// ---------------------------------------------------------------------------
// NUTS
// ---------------------------------------------------------------------------

namespace {

// Warm-up windows (Stan's layout): an initial buffer of 75, slow windows from
// 25 doubling, the last absorbing what would leave less than twice its
// length, and a terminal buffer of 50; below 150 warm-up transitions
// 15 % / 75 % / 10 %, below 20 step size only.
void nuts_warmup_layout(int64_t n_warmup, int64_t &init_buf, int64_t &base_win, int64_t &term_buf) {
    init_buf = 75;
    base_win = 25;
    term_buf = 50;
    if (n_warmup < 20) {
        init_buf = n_warmup;
        base_win = 0;
        term_buf = 0;
        return;
    }
    if (init_buf + base_win + term_buf > n_warmup) {
        init_buf = (int64_t)(0.15 * (double)n_warmup);
        term_buf = (int64_t)(0.1 * (double)n_warmup);
        base_win = n_warmup - init_buf - term_buf;
    }
}

bool nuts_in_slow(int64_t n_warmup, int64_t k) {
    int64_t ib, bw, tb;
    nuts_warmup_layout(n_warmup, ib, bw, tb);
    return bw > 0 && k >= ib && k < n_warmup - tb;
}

bool nuts_window_end(int64_t n_warmup, int64_t k) {
    int64_t ib, bw, tb;
    nuts_warmup_layout(n_warmup, ib, bw, tb);
    if (bw == 0) return false;
    const int64_t slow_end = n_warmup - tb;
    for (int64_t start = ib, len = bw; start < slow_end; len *= 2) {
        int64_t end = start + len;
        if (end + 2 * len > slow_end) end = slow_end;
        if (k == end - 1) return true;
        start = end;
    }
    return false;
}

struct NutsLayout {
    size_t ch, xe[2], ge[2], xw, xs, gs, xp, gp, gw, pe[2], rho, pnear, wm, w2, R, F, sR, sF, sL, lpw, cnt, total;
};

NutsLayout nuts_layout(size_t n, size_t M, size_t SN, size_t L, size_t esz) {
    NutsLayout l;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t at = off;
        off += (bytes + 255) & ~(size_t)255;
        return at;
    };
    l.ch = take(n * sizeof(NutsChain));
    for (int e = 0; e < 2; ++e) l.xe[e] = take(n * M * esz);
    for (int e = 0; e < 2; ++e) l.ge[e] = take(n * M * esz);
    l.xw = take(n * M * esz);
    l.xs = take(n * M * esz);
    l.gs = take(n * M * esz);
    l.xp = take(n * M * esz);
    l.gp = take(n * M * esz);
    l.gw = take(n * SN * esz);
    for (int e = 0; e < 2; ++e) l.pe[e] = take(n * M * 8);
    l.rho = take(n * M * 8);
    l.pnear = take(n * M * 8);
    l.wm = take(n * M * 8);
    l.w2 = take(n * M * 8);
    l.R = take(L * n * M * 8);
    l.F = take(L * n * M * 8);
    l.sR = take(L * n * M * 8);
    l.sF = take(L * n * M * 8);
    l.sL = take(L * n * M * 8);
    l.lpw = take(n * 8);
    l.cnt = take(sizeof(int));
    l.total = off;
    return l;
}

}  // namespace

template <typename T, int S>
mc_status nuts_impl(mc_problem *p, const mc_nuts_config *cfg, int n, T *heights, double *lp, double *eps,
                    double *inv_mass, int32_t *depth_out, int32_t *nleap_out, int32_t *div_out, double *acc_out,
                    hipStream_t st) {
    const size_t N = (size_t)p->R * p->C, MH = (size_t)(S - 1) * N, SN = (size_t)S * N;
    // with r sampled the state is z = (x, logit r): S - 1 more values per chain
    const bool with_r = cfg->r_state != nullptr;
    const size_t M = MH + (with_r ? S - 1 : 0);
    const int L = cfg->max_depth + 1;
    mc_status s;
    if ((s = ensure_grad_ws<T, S>(p, n)) != MC_OK) return s;
    if ((s = ensure(p, p->gcur, sizeof(T) * SN * n)) != MC_OK) return s;
    if (cfg->latent && (s = ensure(p, p->prop, sizeof(T) * MH * n)) != MC_OK) return s;
    double *rc = nullptr;
    if (with_r) {
        if ((s = ensure(p, p->rstat, sizeof(double) * (size_t)n * (S - 1) * kRc)) != MC_OK) return s;
        rc = (double *)p->rstat.p;
    }
    auto target = [&](const T *xs, double *lps, T *gs) {
        if (with_r) return grad_eval_latent_r<T, S>(p, n, xs, lps, gs, rc, st);
        return cfg->latent ? grad_eval_latent<T, S>(p, n, xs, lps, gs, st) : grad_eval<T, S>(p, n, xs, lps, gs, st);
    };
    const NutsLayout lay = nuts_layout(n, M, SN, L, sizeof(T));
    const size_t zoff = lay.total, ztotal = lay.total + (with_r ? ((n * M * sizeof(T) + 255) & ~(size_t)255) : 0);
    if ((s = ensure(p, p->nutsbuf, ztotal)) != MC_OK) return s;
    char *base = (char *)p->nutsbuf.p;
    T *const user_x = heights;
    if (with_r) {
        heights = (T *)(base + zoff);
        const dim3 g((unsigned)((M + 255) / 256), (unsigned)n);
        hipLaunchKernelGGL(k_pack_latent_r<T>, g, dim3(256), 0, st, (const T *)user_x, (const double *)cfg->r_state,
                           heights, (int)MH, S - 1, n);
        HIP_TRY(p, hipGetLastError());
    }
    NutsParams<T> P;
    memset(&P, 0, sizeof(P));
    P.M = (int)M;
    P.SN = (int)SN;
    P.n = n;
    P.L = L;
    P.max_dh = cfg->max_delta_h;
    P.target = cfg->target_accept;
    P.seed = cfg->seed;
    P.inv_mass = inv_mass;
    P.ch = (NutsChain *)(base + lay.ch);
    P.x = heights;
    P.lp = lp;
    P.gcur = (T *)p->gcur.p;
    for (int e = 0; e < 2; ++e) {
        P.xe[e] = (T *)(base + lay.xe[e]);
        P.ge[e] = (T *)(base + lay.ge[e]);
        P.pe[e] = (double *)(base + lay.pe[e]);
    }
    P.xw = (T *)(base + lay.xw);
    P.lpw = (const double *)(base + lay.lpw);
    P.gw = (const T *)(base + lay.gw);
    P.xs = (T *)(base + lay.xs);
    P.gs = (T *)(base + lay.gs);
    P.xp = (T *)(base + lay.xp);
    P.gp = (T *)(base + lay.gp);
    P.rho = (double *)(base + lay.rho);
    P.pnear = (double *)(base + lay.pnear);
    P.R = (double *)(base + lay.R);
    P.F = (double *)(base + lay.F);
    P.sR = (double *)(base + lay.sR);
    P.sF = (double *)(base + lay.sF);
    P.sL = (double *)(base + lay.sL);
    double *wm = (double *)(base + lay.wm), *w2 = (double *)(base + lay.w2);
    int *d_cnt = (int *)(base + lay.cnt);
    // log posterior and gradient of the starting states
    if ((s = target(heights, lp, P.gcur)) != MC_OK) return s;
    hipLaunchKernelGGL(k_nuts_da_init, dim3((n + 255) / 256), dim3(256), 0, st, P.ch, (const double *)eps, n,
                       cfg->n_warmup > 0 ? 1 : 0);
    HIP_TRY(p, hipGetLastError());
    const int64_t total = cfg->n_warmup + cfg->n_steps;
    const dim3 pos_grid((unsigned)((M + 255) / 256), (unsigned)n);
    int64_t wn = 0;
    for (int64_t k = 0; k < total; ++k) {
        P.step = cfg->step_offset + (uint64_t)k;
        hipLaunchKernelGGL(k_nuts_begin<T>, dim3(n), dim3(kNutsBlock), 0, st, P);
        HIP_TRY(p, hipGetLastError());
        for (int d = 0; d < cfg->max_depth; ++d) {
            for (int i = 0; i < (1 << d); ++i) {
                hipLaunchKernelGGL(k_nuts_leap_pos<T>, pos_grid, dim3(256), 0, st, P);
                if ((s = target(P.xw, (double *)P.lpw, (T *)P.gw)) != MC_OK) return s;
                hipLaunchKernelGGL(k_nuts_leap_fin<T>, dim3(n), dim3(kNutsBlock), 0, st, P, i, d);
                HIP_TRY(p, hipGetLastError());
            }
            if (d + 1 < cfg->max_depth) {
                // stop doubling once every chain's tree is finished
                hipLaunchKernelGGL(k_nuts_count_active, dim3(1), dim3(256), 0, st, (const NutsChain *)P.ch, n, d_cnt);
                int active = 0;
                HIP_TRY(p, hipMemcpyAsync(&active, d_cnt, sizeof(int), hipMemcpyDeviceToHost, st));
                HIP_TRY(p, hipStreamSynchronize(st));
                if (active == 0) break;
            }
        }
        hipLaunchKernelGGL(k_nuts_end<T>, dim3(n), dim3(kNutsBlock), 0, st, P, depth_out, nleap_out, div_out,
                           acc_out, k, total);
        HIP_TRY(p, hipGetLastError());
        if (k < cfg->n_warmup) {
            const bool slow = cfg->adapt_mass && nuts_in_slow(cfg->n_warmup, k);
            if (slow) ++wn;
            const bool wend = slow && nuts_window_end(cfg->n_warmup, k);
            hipLaunchKernelGGL(k_nuts_adapt<T>, dim3(n), dim3(kNutsBlock), 0, st, P, inv_mass, wm, w2, wn,
                               slow ? 1 : 0, wend ? 1 : 0, k == cfg->n_warmup - 1 ? 1 : 0);
            HIP_TRY(p, hipGetLastError());
            if (wend) wn = 0;
        }
    }
    hipLaunchKernelGGL(k_nuts_eps_out, dim3((n + 255) / 256), dim3(256), 0, st, (const NutsChain *)P.ch, eps, n);
    HIP_TRY(p, hipGetLastError());
    if (with_r) {
        const dim3 g((unsigned)((M + 255) / 256), (unsigned)n);
        hipLaunchKernelGGL(k_unpack_latent_r<T>, g, dim3(256), 0, st, (const T *)heights, user_x, cfg->r_state,
                           (int)MH, S - 1, n);
        HIP_TRY(p, hipGetLastError());
    }
    return MC_OK;
}

template <typename T>
mc_status nuts_dispatch(mc_problem *p, const mc_nuts_config *cfg, int n, void *heights, double *lp, double *eps,
                        double *inv_mass, int32_t *depth, int32_t *nleap, int32_t *div, double *acc, hipStream_t st) {
    switch (p->S) {
        case 2: return nuts_impl<T, 2>(p, cfg, n, (T *)heights, lp, eps, inv_mass, depth, nleap, div, acc, st);
        case 3: return nuts_impl<T, 3>(p, cfg, n, (T *)heights, lp, eps, inv_mass, depth, nleap, div, acc, st);
        case 4: return nuts_impl<T, 4>(p, cfg, n, (T *)heights, lp, eps, inv_mass, depth, nleap, div, acc, st);
    }
    return fail(p, MC_ERR_UNSUPPORTED, "n_surfaces %d", p->S);
}

extern "C" {

mc_status nuts_run(mc_problem *p, const mc_nuts_config *cfg, int n_chains, void *heights, double *logpost,
                   double *step_size, double *inv_mass, int32_t *tree_depth, int32_t *n_leapfrog, int32_t *diverged,
                   double *accept_stat, void *stream) {
    mc_status s = check_ready(p);
    if (s != MC_OK) return s;
    if (!cfg) return fail(p, MC_ERR_ARG, "cfg is NULL");
    if (n_chains < 0 || cfg->n_warmup < 0 || cfg->n_steps < 0) return fail(p, MC_ERR_ARG, "negative sizes");
    if (n_chains == 0) return MC_OK;
    if (n_chains > 65535) return fail(p, MC_ERR_ARG, "n_chains > 65535");
    if (!heights || !logpost || !step_size) return fail(p, MC_ERR_ARG, "NULL device pointer");
    if (cfg->max_depth < 1 || cfg->max_depth > kNutsMaxDepth)
        return fail(p, MC_ERR_ARG, "max_depth %d not in [1, %d]", cfg->max_depth, kNutsMaxDepth);
    if (!(cfg->max_delta_h > 0) || !std::isfinite(cfg->max_delta_h)) return fail(p, MC_ERR_ARG, "max_delta_h invalid");
    if (!(cfg->target_accept > 0 && cfg->target_accept < 1)) return fail(p, MC_ERR_ARG, "target_accept not in (0, 1)");
    if (cfg->adapt_mass && !inv_mass) return fail(p, MC_ERR_ARG, "adapt_mass needs inv_mass");
    if (cfg->r_state && !cfg->latent)
        return fail(p, MC_ERR_ARG, "r_state is sampled on the latent parametrisation (latent = 1)");
    if (cfg->step_offset + (uint64_t)(cfg->n_warmup + cfg->n_steps) >= (1ULL << 48))
        return fail(p, MC_ERR_ARG, "step counter exceeds 48 bits");
    DeviceGuard g(p->device);
    hipStream_t st = (hipStream_t)stream;
    return p->prec == MC_F64
               ? nuts_dispatch<double>(p, cfg, n_chains, heights, logpost, step_size, inv_mass, tree_depth,
                                       n_leapfrog, diverged, accept_stat, st)
               : nuts_dispatch<float>(p, cfg, n_chains, heights, logpost, step_size, inv_mass, tree_depth,
                                      n_leapfrog, diverged, accept_stat, st);
}

mc_status nested_rhat(mc_problem *p, int n_super, int n_within, const void *heights, double *rhat, void *stream) {
    if (!p) return MC_ERR_ARG;
    if (!p->have_geom) return fail(p, MC_ERR_STATE, "load_geometry_grid has not been called");
    if (n_super < 2 || n_within < 2) return fail(p, MC_ERR_ARG, "need at least 2 super-chains of 2 chains");
    if ((long long)n_super * n_within > 65535) return fail(p, MC_ERR_ARG, "more than 65535 chains");
    if (!heights || !rhat) return fail(p, MC_ERR_ARG, "NULL device pointer");
    DeviceGuard g(p->device);
    hipStream_t st = (hipStream_t)stream;
    const int M = (p->S - 1) * p->R * p->C;
    const dim3 grid((M + 255) / 256);
    if (p->prec == MC_F64)
        hipLaunchKernelGGL(k_nested_rhat<double>, grid, dim3(256), 0, st, (const double *)heights, M, n_super,
                           n_within, rhat);
    else
        hipLaunchKernelGGL(k_nested_rhat<float>, grid, dim3(256), 0, st, (const float *)heights, M, n_super,
                           n_within, rhat);
    HIP_TRY(p, hipGetLastError());
    return MC_OK;
}

mc_status latent_to_heights(mc_problem *p, int n_chains, const void *x, void *heights, void *stream) {
    if (!p) return MC_ERR_ARG;
    if (!p->have_geom) return fail(p, MC_ERR_STATE, "load_geometry_grid has not been called");
    if (n_chains < 0 || n_chains > 65535) return fail(p, MC_ERR_ARG, "n_chains %d", n_chains);
    if (n_chains == 0) return MC_OK;
    if (!x || !heights) return fail(p, MC_ERR_ARG, "NULL device pointer");
    DeviceGuard g(p->device);
    hipStream_t st = (hipStream_t)stream;
    const int N = p->R * p->C;
    const dim3 grid((N + 255) / 256, n_chains);
    if (p->prec == MC_F64) {
        LatentParams<double> L = latent_params<double>(p, n_chains, (const double *)x, (double *)heights, nullptr, nullptr);
        hipLaunchKernelGGL(k_latent_to_heights<double>, grid, dim3(256), 0, st, L);
    } else {
        LatentParams<float> L = latent_params<float>(p, n_chains, (const float *)x, (float *)heights, nullptr, nullptr);
        hipLaunchKernelGGL(k_latent_to_heights<float>, grid, dim3(256), 0, st, L);
    }
    HIP_TRY(p, hipGetLastError());
    return MC_OK;
}

mc_status heights_to_latent(mc_problem *p, int n_chains, const void *heights, void *x, void *stream) {
    if (!p) return MC_ERR_ARG;
    if (!p->have_geom) return fail(p, MC_ERR_STATE, "load_geometry_grid has not been called");
    if (n_chains < 0 || n_chains > 65535) return fail(p, MC_ERR_ARG, "n_chains %d", n_chains);
    if (n_chains == 0) return MC_OK;
    if (!x || !heights) return fail(p, MC_ERR_ARG, "NULL device pointer");
    DeviceGuard g(p->device);
    hipStream_t st = (hipStream_t)stream;
    const int N = p->R * p->C, S1 = p->S - 1;
    double sl[3] = {0, 0, 0};
    for (int l = 0; l < S1; ++l) sl[l] = std::sqrt(p->s11[l]);
    const dim3 grid((N + 255) / 256, n_chains);
    if (p->prec == MC_F64)
        hipLaunchKernelGGL(k_heights_to_latent<double>, grid, dim3(256), 0, st, (const double *)heights, (double *)x,
                           (const double *)p->d_top64, N, S1, sl[0], sl[1], sl[2]);
    else
        hipLaunchKernelGGL(k_heights_to_latent<float>, grid, dim3(256), 0, st, (const float *)heights, (float *)x,
                           (const double *)p->d_top64, N, S1, sl[0], sl[1], sl[2]);
    HIP_TRY(p, hipGetLastError());
    return MC_OK;
}

mc_status mcmc_run_multi(int n_problems, mc_problem *const *problems, const mc_run_config *cfgs,
                         const int *n_chains, void *const *heights, double *const *logposts,
                         int64_t *const *n_accept, void *stream) {
    if (n_problems <= 0 || !problems || !cfgs || !n_chains || !heights || !logposts || !n_accept)
        return fail(nullptr, MC_ERR_ARG, "invalid arguments");
    mc_problem *e = problems[0];
    if (!e) return MC_ERR_ARG;
    for (int i = 0; i < n_problems; ++i) {
        mc_problem *p = problems[i];
        if (!p) return fail(e, MC_ERR_ARG, "problem %d is NULL", i);
        mc_status s = check_ready(p);
        if (s != MC_OK) return fail(e, s, "problem %d: %s", i, p->err.c_str());
        if (p->device != e->device || p->prec != e->prec || p->S != e->S)
            return fail(e, MC_ERR_ARG, "problem %d: device, precision and n_surfaces must match problem 0", i);
        for (int j = 0; j < i; ++j)
            if (problems[j] == p) return fail(e, MC_ERR_ARG, "problem %d repeats problem %d", i, j);
        if (cfgs[i].kernel != 0) return fail(e, MC_ERR_UNSUPPORTED, "mcmc_run_multi runs random-walk Metropolis");
        if ((cfgs[i].r_state != nullptr) != (cfgs[0].r_state != nullptr))
            return fail(e, MC_ERR_ARG, "r_state must be given for every problem or for none");
        if (cfgs[i].r_state && (!(cfgs[i].r_step >= 0) || !std::isfinite(cfgs[i].r_step)))
            return fail(e, MC_ERR_ARG, "r_step invalid");
        if (cfgs[i].n_accept_r && !cfgs[i].r_state) return fail(e, MC_ERR_ARG, "n_accept_r without r_state");
        if (p->vox_nz > 0 || p->quad_nsub > 0)
            return fail(e, MC_ERR_UNSUPPORTED, "problem %d: mcmc_run_multi runs the exact march with one ray per pixel", i);
        if (cfgs[i].n_steps != cfgs[0].n_steps || cfgs[i].graph_steps != cfgs[0].graph_steps)
            return fail(e, MC_ERR_ARG, "n_steps and graph_steps must be equal across problems");
        if (!(cfgs[i].step_size >= 0) || !std::isfinite(cfgs[i].step_size)) return fail(e, MC_ERR_ARG, "step_size");
        if (cfgs[i].step_offset + (uint64_t)cfgs[i].n_steps >= (1ULL << 48)) return fail(e, MC_ERR_ARG, "step counter");
        if (n_chains[i] <= 0 || n_chains[i] > 65535) return fail(e, MC_ERR_ARG, "n_chains[%d]", i);
        if (!heights[i] || !logposts[i] || !n_accept[i]) return fail(e, MC_ERR_ARG, "NULL device pointer");
    }
    if (cfgs[0].n_steps < 0) return fail(e, MC_ERR_ARG, "n_steps < 0");
    DeviceGuard g(e->device);
    std::lock_guard<std::mutex> lock(g_multi_mu);
    hipStream_t st = (hipStream_t)stream;
    if (e->prec == MC_F64) {
        switch (e->S) {
            case 2: return mcmc_multi_impl<double, 2>(n_problems, problems, cfgs, n_chains, heights, logposts, n_accept, st);
            case 3: return mcmc_multi_impl<double, 3>(n_problems, problems, cfgs, n_chains, heights, logposts, n_accept, st);
            case 4: return mcmc_multi_impl<double, 4>(n_problems, problems, cfgs, n_chains, heights, logposts, n_accept, st);
        }
    } else {
        switch (e->S) {
            case 2: return mcmc_multi_impl<float, 2>(n_problems, problems, cfgs, n_chains, heights, logposts, n_accept, st);
            case 3: return mcmc_multi_impl<float, 3>(n_problems, problems, cfgs, n_chains, heights, logposts, n_accept, st);
            case 4: return mcmc_multi_impl<float, 4>(n_problems, problems, cfgs, n_chains, heights, logposts, n_accept, st);
        }
    }
    return fail(e, MC_ERR_UNSUPPORTED, "n_surfaces %d", e->S);
}

namespace {

// Voxel walk of one ray inside the box [0,X]x[0,Y]x[0,Z_top]: a 3-D DDA
// over the column boundaries x = (i+1/2) dx, y = (j+1/2) dy (voxel columns
// are centred on the nodes) and the level boundaries z = k dz.  Appends
// (voxel index, length) for every piece of positive length.
void voxel_walk(const mc_problem *p, int n_z, double dz, const double q[3], const double u[3],
                std::vector<int> &vi, std::vector<double> &vl) {
    const int R = p->R, C = p->C;
    const double dx = p->X / (R - 1), dy = p->Y / (C - 1);
    double T = (p->ztop - q[2]) / u[2];
    if (u[0] > 0) T = std::min(T, (p->X - q[0]) / u[0]);
    if (u[0] < 0) T = std::min(T, -q[0] / u[0]);
    if (u[1] > 0) T = std::min(T, (p->Y - q[1]) / u[1]);
    if (u[1] < 0) T = std::min(T, -q[1] / u[1]);
    if (!(T > 0)) return;
    int i = std::min(std::max((int)std::floor(q[0] / dx + 0.5), 0), R - 1);
    int j = std::min(std::max((int)std::floor(q[1] / dy + 0.5), 0), C - 1);
    int k = std::min(std::max((int)std::floor(q[2] / dz), 0), n_z - 1);
    auto next_x = [&](int a) {
        if (u[0] > 0 && a < R - 1) return ((a + 0.5) * dx - q[0]) / u[0];
        if (u[0] < 0 && a > 0) return ((a - 0.5) * dx - q[0]) / u[0];
        return (double)INFINITY;
    };
    auto next_y = [&](int b) {
        if (u[1] > 0 && b < C - 1) return ((b + 0.5) * dy - q[1]) / u[1];
        if (u[1] < 0 && b > 0) return ((b - 0.5) * dy - q[1]) / u[1];
        return (double)INFINITY;
    };
    auto next_z = [&](int c) { return c < n_z - 1 ? ((c + 1) * dz - q[2]) / u[2] : (double)INFINITY; };
    double tx = next_x(i), ty = next_y(j), tz = next_z(k), t = 0.0;
    for (int guard = 0; guard < R + C + n_z + 4 && t < T; ++guard) {
        const double tn = std::min(std::min(tx, ty), std::min(tz, T));
        if (tn > t) {
            vi.push_back((i * C + j) * n_z + k);
            vl.push_back(tn - t);
        }
        if (tn >= T) break;
        if (tx == tn) tx = next_x(i += u[0] > 0 ? 1 : -1);
        if (ty == tn) ty = next_y(j += u[1] > 0 ? 1 : -1);
        if (tz == tn) tz = next_z(++k);
        t = tn;
    }
}

}  // namespace

mc_status set_voxel_model(mc_problem *p, int n_z, double gamma, const double *ref_heights) {
    if (!p) return MC_ERR_ARG;
    if (!p->have_geom) return fail(p, MC_ERR_STATE, "load_geometry_grid has not been called");
    if (!p->have_sensors) return fail(p, MC_ERR_STATE, "set_sensors has not been called");
    if (n_z < 0 || n_z > 4096) return fail(p, MC_ERR_ARG, "n_z %d not in [0, 4096]", n_z);
    DeviceGuard g(p->device);
    if (n_z == 0) {
        clear_voxel_model(p);
        return MC_OK;
    }
    if (!(gamma > 0) || !std::isfinite(gamma)) return fail(p, MC_ERR_ARG, "gamma must be > 0");
    if (!ref_heights) return fail(p, MC_ERR_ARG, "ref_heights is NULL");
    const int S = p->S, N = p->R * p->C;
    for (size_t i = 0; i < (size_t)(S - 1) * N; ++i)
        if (!std::isfinite(ref_heights[i])) return fail(p, MC_ERR_ARG, "ref_heights[%zu] not finite", i);
    clear_voxel_model(p);
    if (p->quad_nsub > 0) return fail(p, MC_ERR_STATE, "pixel quadrature is set: switch it off first");
    const double dz = p->ztop / n_z;
    std::vector<double> drho(S);
    for (int l = 0; l < S; ++l) drho[l] = p->density[l] - (l + 1 < S ? p->density[l + 1] : 0.0);
    // the floor's smooth indicator and the normaliser per level
    std::vector<double> fsig(n_z), inorm(n_z);
    for (int k = 0; k < n_z; ++k) {
        const double z = (k + 0.5) * dz;
        fsig[k] = 1.0 / (1.0 + std::exp(z / gamma));
        inorm[k] = 1.0 + std::exp(-z / gamma);
    }
    // R0 = R-hat(H_ref), float64
    const size_t V = (size_t)N * n_z;
    std::vector<double> r0(V);
    for (int n = 0; n < N; ++n) {
        double h[kMaxSurfaces];
        for (int l = 0; l < S - 1; ++l) h[l] = ref_heights[(size_t)l * N + n];
        h[S - 1] = p->top[n];
        for (int k = 0; k < n_z; ++k) {
            const double z = (k + 0.5) * dz;
            double acc = -p->density[0] * fsig[k];
            for (int l = 0; l < S; ++l) acc += drho[l] / (1.0 + std::exp((z - h[l]) / gamma));
            r0[(size_t)n * n_z + k] = acc * inorm[k];
        }
    }
    // voxel walks of every ray, lambda(R0) and O(R0)
    std::vector<int> off(p->n_ray + 1), vi;
    std::vector<double> vl, lam0(p->n_ray), o0(p->n_ray);
    vi.reserve((size_t)p->n_ray * (p->R + p->C + n_z) / 2);
    vl.reserve(vi.capacity());
    for (int r = 0; r < p->n_ray; ++r) {
        off[r] = (int)vi.size();
        const size_t b0 = vi.size();
        voxel_walk(p, n_z, dz, p->pos.data() + 3 * (r / p->n_pix), p->dirs.data() + 3 * (size_t)r, vi, vl);
        if (vi.size() > (size_t)INT32_MAX) return fail(p, MC_ERR_UNSUPPORTED, "more than 2^31 ray-voxel pieces");
        double o = 0.0;
        for (size_t e = b0; e < vi.size(); ++e) o += vl[e] * r0[vi[e]];
        o0[r] = o;
        lam0[r] = p->expo[r] * std::exp(-o / p->atten);
    }
    off[p->n_ray] = (int)vi.size();
    mc_status s;
    void *q = nullptr;
    HIP_TRY(p, hipMalloc(&q, sizeof(int) * off.size()));
    p->d_vox_off = (int *)q;
    HIP_TRY(p, hipMemcpy(q, off.data(), sizeof(int) * off.size(), hipMemcpyHostToDevice));
    if (!vi.empty()) {
        // kVoxPad padding entries (voxel 0, length 0) past the end: the
        // likelihood kernel reads its lists in whole batches, one ahead
        const size_t nnz = vi.size();
        vi.resize(nnz + kVoxPad, 0);
        vl.resize(nnz + kVoxPad, 0.0);
        q = nullptr;
        HIP_TRY(p, hipMalloc(&q, sizeof(int) * vi.size()));
        p->d_vox_idx = (int *)q;
        HIP_TRY(p, hipMemcpy(q, vi.data(), sizeof(int) * vi.size(), hipMemcpyHostToDevice));
        if ((s = upload_prec(p, p->d_vox_len, vl)) != MC_OK) return s;
        vi.resize(nnz);
        vl.resize(nnz);
    }
    {
        // the transpose (voxel -> rays crossing it, in ray order) for the gradient's gather
        const size_t V = (size_t)p->R * p->C * n_z;
        std::vector<int> toff(V + 1, 0), tray(vi.size());
        std::vector<double> tlen(vi.size());
        for (int v : vi) ++toff[(size_t)v + 1];
        for (size_t v = 0; v < V; ++v) toff[v + 1] += toff[v];
        std::vector<int> fill(toff.begin(), toff.end() - 1);
        for (int r = 0; r < p->n_ray; ++r)
            for (int e = off[r]; e < off[r + 1]; ++e) {
                const int at = fill[vi[e]]++;
                tray[at] = r;
                tlen[at] = vl[e];
            }
        HIP_TRY(p, hipMalloc(&q, sizeof(int) * toff.size()));
        p->d_vox_toff = (int *)q;
        HIP_TRY(p, hipMemcpy(q, toff.data(), sizeof(int) * toff.size(), hipMemcpyHostToDevice));
        // the gradient's work items: each column's entries cut into pieces of
        // at most kVoxItemEntries, with the level of each piece's first entry
        std::vector<int> items;
        for (int c = 0; c < p->R * p->C; ++c) {
            const size_t vb = (size_t)c * n_z;
            const int e0 = toff[vb], e1 = toff[vb + n_z];
            int k = 0;
            for (int e = e0; e < e1; e += kVoxItemEntries) {
                while (toff[vb + k + 1] <= e) ++k;
                items.insert(items.end(), {c, k, e, std::min(e + kVoxItemEntries, e1)});
            }
        }
        if (!items.empty()) {
            q = nullptr;
            HIP_TRY(p, hipMalloc(&q, sizeof(int) * items.size()));
            p->d_vox_items = (int *)q;
            HIP_TRY(p, hipMemcpy(q, items.data(), sizeof(int) * items.size(), hipMemcpyHostToDevice));
            p->vox_n_items = (int)(items.size() / 4);
        }
        if (!vi.empty()) {
            // kVoxPad padding entries (ray 0, length 0): the gradient reads whole batches
            tray.resize(tray.size() + kVoxPad, 0);
            tlen.resize(tlen.size() + kVoxPad, 0.0);
            q = nullptr;
            HIP_TRY(p, hipMalloc(&q, sizeof(int) * tray.size()));
            p->d_vox_tray = (int *)q;
            HIP_TRY(p, hipMemcpy(q, tray.data(), sizeof(int) * tray.size(), hipMemcpyHostToDevice));
            if ((s = upload_prec(p, p->d_vox_tlen, tlen)) != MC_OK) return s;
        }
    }
    for (auto pr : {std::make_pair(&p->d_vox_lam0, &lam0), std::make_pair(&p->d_vox_o0, &o0),
                    std::make_pair(&p->d_vox_fsig, &fsig), std::make_pair(&p->d_vox_inorm, &inorm)}) {
        void *d = nullptr;
        if ((s = upload<double>(p, d, *pr.second)) != MC_OK) return s;
        *pr.first = (double *)d;
    }
    p->vox_nnz = vi.size();
    p->vox_drho = drho;
    p->vox_gamma = gamma;
    p->vox_dz = dz;
    p->vox_nz = n_z;
    drop_graph(p);
    return MC_OK;
}

mc_status set_pixel_quadrature(mc_problem *p, int n_sub, const double *weights, int n_table, double o_max,
                               const double *log_intensity) {
    if (!p) return MC_ERR_ARG;
    if (!p->have_sensors) return fail(p, MC_ERR_STATE, "set_sensors has not been called");
    DeviceGuard g(p->device);
    if (n_sub == 0) {
        clear_quadrature(p);
        p->have_counts = false;
        return MC_OK;
    }
    if (n_sub < 0 || p->n_pix % n_sub != 0) return fail(p, MC_ERR_ARG, "n_sub %d does not divide n_pix %d", n_sub, p->n_pix);
    if (n_table < 2 || !(o_max > 0) || !std::isfinite(o_max)) return fail(p, MC_ERR_ARG, "table: n_table >= 2, o_max > 0");
    if (!weights || !log_intensity) return fail(p, MC_ERR_ARG, "NULL array");
    for (int r = 0; r < p->n_ray; ++r)
        if (!(weights[r] > 0) || !std::isfinite(weights[r])) return fail(p, MC_ERR_ARG, "weights[%d] must be > 0", r);
    for (int j = 0; j < n_table; ++j)
        if (!std::isfinite(log_intensity[j])) return fail(p, MC_ERR_ARG, "log_intensity[%d] not finite", j);
    clear_voxel_model(p);
    clear_quadrature(p);
    mc_status s;
    void *d = nullptr;
    if ((s = upload<double>(p, d, std::vector<double>(weights, weights + p->n_ray))) != MC_OK) return s;
    p->d_quad_w = (double *)d;
    d = nullptr;
    if ((s = upload<double>(p, d, std::vector<double>(log_intensity, log_intensity + n_table))) != MC_OK) return s;
    p->d_quad_tab = (double *)d;
    p->quad_nsub = n_sub;
    p->quad_npx = p->n_ray / n_sub;
    p->quad_ntab = n_table;
    p->quad_omax = o_max;
    p->have_counts = false;   // counts are per pixel from now on
    drop_graph(p);
    return MC_OK;
}

mc_status mc_voxel_info(const mc_problem *p, int *n_z, int64_t *n_pieces) {
    if (!p || !n_z || !n_pieces) return MC_ERR_ARG;
    *n_z = p->vox_nz;
    *n_pieces = (int64_t)p->vox_nnz;
    return MC_OK;
}

mc_status mc_time_voxel(mc_problem *p, int n_chains, const void *heights, int iters, void *stream,
                        float *ms_density, float *ms_likelihood) {
    mc_status s = check_ready(p);
    if (s != MC_OK) return s;
    if (n_chains <= 0 || n_chains > 65535 || iters <= 0 || !heights || !ms_density || !ms_likelihood)
        return fail(p, MC_ERR_ARG, "invalid arguments");
    if (p->vox_nz == 0 || p->n_ray == 0) return fail(p, MC_ERR_STATE, "no voxel model or no rays");
    DeviceGuard g(p->device);
    hipStream_t st = (hipStream_t)stream;
    if ((s = ensure(p, p->rhat, rhat_bytes(p, n_chains))) != MC_OK) return s;
    if ((s = ensure(p, p->partials, sizeof(double) * (size_t)n_chains * tiling(p).n_tiles)) != MC_OK) return s;
    hipEvent_t ev[3] = {nullptr, nullptr, nullptr};
    for (auto &e : ev) HIP_TRY(p, hipEventCreate(&e));
    float ms[2] = {0, 0};
    hipError_t err = hipSuccess;
    auto run = [&](auto tag) {
        using T = decltype(tag);
        VoxParams<T> V = vox_params<T>(p, n_chains, (const T *)heights, nullptr, (double *)p->partials.p, nullptr);
        auto dens = [&]() {
            switch (p->S) {
                case 2: launch_vox_density<T, 2>(V, st); break;
                case 3: launch_vox_density<T, 3>(V, st); break;
                default: launch_vox_density<T, 4>(V, st); break;
            }
        };
        dens();
        launch_vox_lik<T>(V, st);   // warm
        (void)hipEventRecord(ev[0], st);
        for (int i = 0; i < iters; ++i) dens();
        (void)hipEventRecord(ev[1], st);
        for (int i = 0; i < iters; ++i) launch_vox_lik<T>(V, st);
        (void)hipEventRecord(ev[2], st);
        err = hipEventSynchronize(ev[2]);
    };
    if (p->prec == MC_F64) run(double(0));
    else run(float(0));
    if (err == hipSuccess) err = hipEventElapsedTime(&ms[0], ev[0], ev[1]);
    if (err == hipSuccess) err = hipEventElapsedTime(&ms[1], ev[1], ev[2]);
    for (auto &e : ev) (void)hipEventDestroy(e);
    HIP_TRY(p, err);
    *ms_density = ms[0] / iters;
    *ms_likelihood = ms[1] / iters;
    return MC_OK;
}

mc_status mc_set_tuning(mc_problem *p, const mc_tuning *t) {
    if (!p || !t) return MC_ERR_ARG;
    if (t->march_variant != 3 && t->march_variant != 4)
        return fail(p, MC_ERR_UNSUPPORTED, "march_variant %d is not built (3 and 4 are)", t->march_variant);
    if (!(t->block == 256 || (p->prec == MC_F32 && (t->block == 512 || t->block == 1024))))
        return fail(p, MC_ERR_UNSUPPORTED, "block %d not built for this precision", t->block);
    if (t->rays_per_thread < 1 || t->rays_per_thread > 64) return fail(p, MC_ERR_ARG, "rays_per_thread %d", t->rays_per_thread);
    if (t->multi_blocks_per_cu < 0 || t->multi_blocks_per_cu > 16)
        return fail(p, MC_ERR_ARG, "multi_blocks_per_cu %d", t->multi_blocks_per_cu);
    if (t->grad_slots < -1 || t->grad_slots > 1024) return fail(p, MC_ERR_ARG, "grad_slots %d", t->grad_slots);
    if (t->adjoint_rows < 0) return fail(p, MC_ERR_ARG, "adjoint_rows %d", t->adjoint_rows);
    DeviceGuard g(p->device);
    drop_graph(p);
    p->tune = *t;
    p->tune_user = true;
    return MC_OK;
}

mc_status mc_get_tuning(const mc_problem *p, mc_tuning *t) {
    if (!p || !t) return MC_ERR_ARG;
    *t = p->tune;
    return MC_OK;
}

mc_status mc_time_march(mc_problem *p, int n_chains, const void *heights, int iters, void *stream,
                        float *ms_per_launch) {
    mc_status s = check_ready(p);
    if (s != MC_OK) return s;
    if (n_chains <= 0 || n_chains > 65535 || iters <= 0 || !heights || !ms_per_launch)
        return fail(p, MC_ERR_ARG, "invalid arguments");
    if (p->n_ray == 0) return fail(p, MC_ERR_STATE, "no rays");
    if (p->vox_nz > 0) return fail(p, MC_ERR_STATE, "the voxel model is set: use mc_time_voxel");
    DeviceGuard g(p->device);
    hipStream_t st = (hipStream_t)stream;
    return p->prec == MC_F64 ? time_march_dispatch<double>(p, n_chains, heights, iters, st, ms_per_launch)
                             : time_march_dispatch<float>(p, n_chains, heights, iters, st, ms_per_launch);
}

mc_status mc_time_adjoint(mc_problem *p, int n_chains, const void *heights, int iters, void *stream,
                          float *ms_per_launch) {
    mc_status s = check_ready(p);
    if (s != MC_OK) return s;
    if (n_chains <= 0 || n_chains > 65535 || iters <= 0 || !heights || !ms_per_launch)
        return fail(p, MC_ERR_ARG, "invalid arguments");
    if (p->n_ray == 0) return fail(p, MC_ERR_STATE, "no rays");
    if (p->vox_nz > 0 || p->quad_nsub > 0)
        return fail(p, MC_ERR_UNSUPPORTED, "gradients follow the exact march with one ray per pixel");
    DeviceGuard g(p->device);
    hipStream_t st = (hipStream_t)stream;
    return p->prec == MC_F64 ? time_adjoint_dispatch<double>(p, n_chains, heights, iters, st, ms_per_launch)
                             : time_adjoint_dispatch<float>(p, n_chains, heights, iters, st, ms_per_launch);
}

mc_status mc_measure_valu_rate(int hip_device, int kind, double *lane_ops_per_s) {
    if (!lane_ops_per_s || (kind != kProbeF32Fma && kind != kProbeF64Fma)) return MC_ERR_ARG;
    DeviceGuard g(hip_device);
    int ncu = 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, hip_device) != hipSuccess || ncu <= 0)
        return MC_ERR_DEVICE;
    const int blocks = ncu * 32;   // 256-thread blocks: 32 waves per SIMD over the launch
    const int iters = 1 << 16;
    void *out = nullptr;
    if (hipMalloc(&out, (size_t)blocks * 256 * 8) != hipSuccess) return MC_ERR_NOMEM;
    hipStream_t st = nullptr;
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
        (void)hipFree(out);
        return MC_ERR_DEVICE;
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    float best = 0.f;
    for (int rep = 0; rep < 4; ++rep) {
        (void)hipEventRecord(e0, st);
        if (kind == kProbeF32Fma)
            hipLaunchKernelGGL(k_valu_probe<float>, dim3(blocks), dim3(256), 0, st, (float *)out, iters,
                               0.999999f, 1e-7f);
        else
            hipLaunchKernelGGL(k_valu_probe<double>, dim3(blocks), dim3(256), 0, st, (double *)out, iters,
                               0.999999, 1e-7);
        (void)hipEventRecord(e1, st);
        (void)hipEventSynchronize(e1);
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        if (rep > 0 && (best == 0.f || ms < best)) best = ms;
    }
    const hipError_t e = hipGetLastError();
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipStreamDestroy(st);
    (void)hipFree(out);
    if (e != hipSuccess || best <= 0.f) return MC_ERR_DEVICE;
    *lane_ops_per_s = (double)blocks * 256.0 * iters * 8.0 / (best * 1e-3);
    return MC_OK;
}

mc_status mc_debug_philox(int hip_device, uint64_t seed, uint32_t chain, uint64_t step, uint32_t tag, uint32_t j0,
                          int n, uint32_t *out_u32, double *out_normal) {
    if (n < 0) return MC_ERR_ARG;
    if (n == 0) return MC_OK;
    DeviceGuard g(hip_device);
    hipLaunchKernelGGL(k_debug_philox, dim3((n + 255) / 256), dim3(256), 0, (hipStream_t)0, seed, chain, step, tag, j0,
                       n, out_u32, out_normal);
    if (hipGetLastError() != hipSuccess) return MC_ERR_DEVICE;
    if (hipDeviceSynchronize() != hipSuccess) return MC_ERR_DEVICE;
    return MC_OK;
}

}  // extern "C"

// serving loop (mc_server_*)
#include "server.h"
