/*
 * muoncave.h -- C ABI of the MI355X (gfx950) library for batched posterior
 * evaluation and MCMC over surface-based block-cave geometries from muon
 * counts (Biron-Lattes et al., arXiv 2603.28907).
 *
 * Model (paper Sec. 2):
 *   - Layer model (Sec. 2.1.3): S height fields H_1 < ... < H_S on an
 *     n_rows x n_cols node grid over the footprint [0,X] x [0,Y]; H_S (the
 *     terrain) is known, H_1..H_{S-1} are inferred.  Nodes are vertex-centred,
 *     x_i = i X/(n_rows-1), y_j = j Y/(n_cols-1); row index i runs along x,
 *     H[l][i][j] is stored in C order (the array-indexing figure).  Surfaces
 *     are bilinear inside each grid cell.
 *   - Density (eq. def_LM_density_grid, continuum form): unit l, between
 *     surface l-1 and l (surface 0 = the floor z = 0), has density rho_l;
 *     density is 0 above H_S and outside the box [0,X]x[0,Y]x[0,max H_S].
 *   - Opacity (Sec. 2.1.1): O = integral of density along the ray from the
 *     sensor, evaluated exactly through the height fields.
 *   - Expected counts (eq. expected_counts, one ray per pixel, exponential
 *     attenuation): lambda_p = E_p exp(-O_p / Lambda).
 *   - Likelihood (eq. def_likelihood): C_p ~ Poisson(lambda_p), normalised.
 *   - Prior (Sec. 2.2.1): per free surface, a Gaussian copula over a periodic
 *     proper CAR field with dependence r_l, H_l = (1-u) H_{l-1} + u H_S,
 *     written as a density in H-space (normalised).
 *   - logpost = log-likelihood + log prior; states outside the support
 *     0 < H_1 < ... < H_{S-1} < H_S give -inf.
 *
 * Units: metres for lengths and heights, g/cm^3 for densities, opacity in
 * (g/cm^3 x m), Lambda in the same unit.
 *
 * Ownership: host arrays passed to the set-up calls are copied before the
 * call returns.  Device arrays passed to the *_batch and run calls belong to
 * the caller; the library never frees them.  Library-internal device memory
 * belongs to the handle and is released by mc_destroy.
 *
 * Synchrony: the set-up calls are synchronous.  logpost_batch,
 * logpost_grad_batch and mcmc_run enqueue work on `stream` (a hipStream_t
 * passed as void*; NULL = the default stream) and return without waiting.
 *
 * Errors: every call returns an mc_status; mc_last_error() gives a message
 * for the last non-OK status of that handle.  MC_ERR_STATE reports a call
 * made out of order (e.g. logpost_batch before set_counts).
 *
 * Threads: one handle is used by one host thread at a time; different
 * handles may be used concurrently.
 */
#ifndef MUONCAVE_H
#define MUONCAVE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mc_problem mc_problem;

typedef enum {
    MC_OK = 0,
    MC_ERR_ARG = -1,          /* invalid argument (shape, range, NULL) */
    MC_ERR_STATE = -2,        /* call out of order */
    MC_ERR_NOMEM = -3,        /* device allocation failed */
    MC_ERR_DEVICE = -4,       /* HIP runtime error */
    MC_ERR_UNSUPPORTED = -5   /* valid request this build does not handle (e.g. grid too large) */
} mc_status;

typedef enum {
    MC_F32 = 0,   /* heights, opacities and the ray march in float32; sums in float64 */
    MC_F64 = 1    /* everything in float64 */
} mc_precision;

/* Create a handle bound to HIP device `hip_device` computing in `precision`. */
mc_status mc_create(int hip_device, int precision, mc_problem **out);

/* Release the handle and its device memory (waits for its pending work). */
void mc_destroy(mc_problem *p);

/* Message for the last non-OK status of `p` (or of the last failed
   mc_create when p is NULL).  Valid until the next call on the handle. */
const char *mc_last_error(const mc_problem *p);

/*
 * Geometry (Sec. 2.1.3 layer model, Sec. 2.2.1 prior parameters).
 *   n_surfaces S in [2, 4]: S-1 free surfaces plus the known top.
 *   n_rows, n_cols >= 3 (the periodic 4-neighbour graph needs 3 nodes per
 *   direction) and <= 256.
 *   extent_x_m, extent_y_m > 0: footprint size.
 *   density[S]: density of unit l = 1..S (>= 0).
 *   top[n_rows*n_cols]: the known top surface H_S (> 0), C order.
 *   car_r[S-1]: CAR dependence r_l in [0, 1) of each free surface.
 * Resets sensors and counts.
 */
mc_status load_geometry_grid(mc_problem *p, int n_surfaces, int n_rows, int n_cols,
                             double extent_x_m, double extent_y_m, const double *density,
                             const double *top, const double *car_r);

/*
 * Sensors and pixels (Sec. 2.1.1 radiographs; one ray per pixel).
 *   pos[n_sensors*3]: sensor positions (x,y inside the footprint, 0 <= z < max top).
 *   dirs[n_sensors*n_pix*3]: unit pixel directions with d_z > 0; ray
 *   r = s*n_pix + k belongs to sensor s.
 *   exposure[n_sensors*n_pix] > 0: E_p (exposure time x acceptance x flux scale).
 *   atten_len > 0: Lambda.
 * n_sensors = 0 (no data: the posterior is the prior) is allowed.  Resets counts.
 */
mc_status set_sensors(mc_problem *p, int n_sensors, const double *pos, int n_pix,
                      const double *dirs, const double *exposure, double atten_len);

/* Observed counts C_p >= 0, [n_sensors*n_pix] (eq. def_likelihood). */
mc_status set_counts(mc_problem *p, const int32_t *counts);

/*
 * Likelihood backend: the paper's own forward model (Sec. 2.1.2 and 2.1.4) in
 * place of the exact ray march.  The density is the sigmoid-smoothed voxel
 * grid R-hat(H) (eqs. def_sigmoid, smooth_layer_indicators,
 * def_LM_density_grid_smooth) and the expected counts are linearised around
 * R0 = R-hat(H_ref) with the sensitivity matrix G = d lambda / dR at R0
 * (eq. expected_counts_linearized_approx):
 *   lambda-hat_p = lambda_p(R0) (1 - (O_p(R-hat) - O_p(R0)) / Lambda),
 *   O_p(R) = sum_v L_pv R_v, L_pv the length of ray p inside voxel v.
 * Voxel columns are centred on the grid nodes (x(i) = i), n_z levels of
 * dz = max(top)/n_z fill [0, max(top)], and the indicator heights are the
 * level centres (k + 1/2) dz.  The air above the top surface is a unit of
 * density 0.  A state with lambda-hat_p <= 0 at some pixel has log
 * posterior -inf.  The prior is unchanged.
 *   n_z in [1, 4096]: voxel levels; 0 switches back to the exact march.
 *   gamma > 0: sigmoid scale in metres (the paper uses 1).
 *   ref_heights[(S-1)*R*C]: host array, the free surfaces of H_ref (the top
 *   is the problem's); copied.
 * Needs geometry and sensors; load_geometry_grid and set_sensors switch the
 * model off again.  While it is on, logpost_batch, logpost_grad_batch,
 * mcmc_run (random walk with or without sampled r, and MALA) and nuts_run
 * use it; mcmc_run_multi, mc_time_march and mc_time_adjoint return
 * MC_ERR_UNSUPPORTED or MC_ERR_STATE.  The opacity output of logpost_batch
 * then holds O_p(R-hat).  Its gradient (the paper's reason for the sigmoid,
 * Sec. 2.1.4): dLL/dH_l,n = sum_k B_(n,k) (rho_l - rho_{l+1}) s (1 - s) /
 * (gamma (1 - s_0)), s = sigmoid((H_l,n - z_k) / gamma), s_0 the floor's, with
 * B_v = sum_p (C_p / lambda-hat_p - 1) G_pv gathered over the rays that
 * cross voxel v.  Device memory: the ray-voxel lists and their transpose
 * (8 or 12 bytes per piece each) and, per call, R*C*n_z*round_up(n_chains,
 * 64) smoothed densities in the state precision (plus n_rays of dLL/dO per
 * chain for gradients).
 */
mc_status set_voxel_model(mc_problem *p, int n_z, double gamma, const double *ref_heights);

/*
 * Solid-angle pixels (eq. expected_counts): the expected count of a pixel
 * is the integral of the muon intensity I(O) times exposure and detector
 * efficiency over its solid angle, here a quadrature over sub-rays.  The
 * rays given to set_sensors become sub-rays: each group of n_sub consecutive
 * rays of a sensor (n_sub divides n_pix) is one pixel, with
 *   lambda_p = sum_q weights[q] I(O_q),
 * weights [n_rays] > 0 (Delta t x sub-cell solid angle x efficiency), and
 * log I tabulated at n_table uniform opacity nodes over [0, o_max] (linear
 * interpolation in log I; beyond o_max the last segment continues).  After
 * this call set_counts takes one count per pixel (n_rays / n_sub values) and
 * must be called again; logpost_batch, logpost_grad_batch, mcmc_run (random
 * walk and MALA) and nuts_run use the quadrature, and the opacity output
 * holds the sub-rays' opacities.  The gradient gives each sub-ray
 *   dLL/dO_q = (C_p / lambda_p - 1) weights[q] I(O_q) dlog I/dO(O_q)
 * (the slope of O_q's table segment) and sums its crossings as for one ray
 * per pixel.  mcmc_run_multi, the server and the voxel model are refused
 * while it is set.  n_sub = 0 switches back to one ray per pixel (counts
 * must be set again); set_sensors and load_geometry_grid switch it off.
 */
mc_status set_pixel_quadrature(mc_problem *p, int n_sub, const double *weights, int n_table, double o_max,
                               const double *log_intensity);

/* The voxel model's levels (0 when it is off) and the number of ray-voxel
   pieces over all rays (the non-zeros of the sensitivity matrix G). */
mc_status mc_voxel_info(const mc_problem *p, int *n_z, int64_t *n_pieces);

/*
 * Log posterior of n_chains states.
 *   heights: device, [n_chains][S-1][n_rows][n_cols] in the handle's precision.
 *   logpost: device, [n_chains] float64 (written).
 *   opacity: device, [n_chains][n_sensors*n_pix] in the handle's precision, or
 *            NULL; if given, every ray's opacity is written (also for chains
 *            outside the support).
 * n_chains = 0 is a no-op.
 */
mc_status logpost_batch(mc_problem *p, int n_chains, const void *heights, double *logpost,
                        void *opacity, void *stream);

/*
 * logpost_batch for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same arguments, kernels and results as logpost_batch, with no
 * hipMalloc, hipFree or other allocating call.  Its workspace (the float64
 * partial sums of the likelihood per chain and ray tile) is a fixed 1 MiB
 * array per device, resolved by mc_create: n_chains x n_tiles must be at
 * most 131072, with n_tiles = ceil(n_sensors*n_pix / (block x
 * rays_per_thread)) of the handle's launch shape (mc_get_tuning); larger
 * requests return MC_ERR_ARG.  Exact march with one ray per pixel only:
 * while set_voxel_model or set_pixel_quadrature is on it returns
 * MC_ERR_UNSUPPORTED.  Every call on one device shares that array and
 * nothing in it needs to start at zero; calls that overlap in time on one
 * device (other streams, other handles, other host threads) race on it and
 * must be serialised by the caller.
 */
mc_status logpost_batch_noalloc(mc_problem *p, int n_chains, const void *heights, double *logpost,
                                void *opacity, void *stream);

/*
 * Log posterior and its gradient with respect to every surface height,
 * including the fixed top surface.
 *   grad: device, [n_chains][S][n_rows][n_cols] in the handle's precision;
 *         rows of chains outside the support are zero.
 * The likelihood part uses the crossing form dO/dH_n = (rho_l - rho_{l+1})
 * sum over crossings of w_n / |d(z-h)/dt|; lp is piecewise smooth in H.
 * float32: the march that precedes the adjoint records each crossing (cell,
 * local coordinates, 1/|f'|) and dLL/dO of every ray, and the adjoint sums
 * the node contributions from those records; chains whose record slots
 * overflow (see mc_tuning.grad_slots) are re-walked instead, with the same
 * result bit for bit.  Under set_voxel_model the gradient is the voxel
 * model's, under set_pixel_quadrature the solid-angle pixels' (see there).
 */
mc_status logpost_grad_batch(mc_problem *p, int n_chains, const void *heights, double *logpost,
                             void *grad, void *stream);

typedef struct {
    int kernel;             /* 0 = random-walk Metropolis, 1 = MALA */
    int64_t n_steps;        /* MCMC steps per chain in this call (>= 0) */
    int graph_steps;        /* steps per captured HIP graph (>= 1; 1 = eager launches) */
    double step_size;       /* RW: proposal sd sigma (m); MALA: eps */
    const double *inv_mass; /* device [S-1][n_rows][n_cols] diagonal M^-1 (MALA), or NULL = 1 */
    uint64_t seed;          /* Philox4x32-10 key */
    uint64_t step_offset;   /* steps already taken: a resumed run uses the same seed
                               and offset = steps done, and is bitwise identical */
    double *r_state;        /* device [n_chains][S-1] float64 in (0, 1), in/out, or NULL:
                               sample each chain's CAR dependence parameters too */
    double r_step;          /* sd of the r proposal on the logit scale (r_state set) */
    int64_t *n_accept_r;    /* device [n_chains][S-1] int64 in/out (r accepts), or NULL */
} mc_run_config;

/*
 * Run n_steps MCMC steps of every chain (paper Sec. 3.1: only posterior
 * ratios are needed; many independent chains run on one device and only the
 * last state is kept).
 *   heights:  device, [n_chains][S-1][n_rows][n_cols], in/out.
 *   logpost:  device, [n_chains] float64, in/out; NaN entries are computed first.
 *   n_accept: device, [n_chains] int64, in/out (incremented per acceptance).
 * Random numbers: Philox4x32-10 keyed by `seed`, counter (j, step lo32,
 * step hi16 | tag << 16, chain) with tag 0 = RW proposal normals,
 * 1 = accept uniform, 2 = MALA normals, 3 = r proposal normals, 4 = r
 * accept uniforms; chain = index in this call.
 *
 * Hierarchical dependence (paper Sec. 2.2.1: r_l iid Uniform(0, 1) a
 * priori): with cfg->r_state set (random-walk only), every step is followed
 * by one Metropolis update of each r_l of each chain on the logit scale,
 * eta' = logit(r_l) + r_step * z (z: component l % 2 of normal pair l / 2 of
 * tag 3), accepted with probability
 *   min(1, p(H | r') r'(1 - r') / (p(H | r) r(1 - r)))
 * (first uniform of pair l of tag 4; a state outside the support moves r
 * under its prior alone).  logpost then holds log p(C | H) + log p(H | r)
 * with each chain's own r, and is recomputed for every chain on entry.
 */
mc_status mcmc_run(mc_problem *p, const mc_run_config *cfg, int n_chains, void *heights,
                   double *logpost, int64_t *n_accept, void *stream);

/*
 * Launch shape of the ray-march kernel (performance only; results agree to
 * rounding).  march_variant: 3 = surface-major band walks (any precision;
 * float64 handles always run it), 4 = lean band walks with branch-free
 * inline crossing solves (float32).  Other values return
 * MC_ERR_UNSUPPORTED.  block: threads per block (256, 512 or 1024; float64
 * handles use 256), rays_per_thread: rays each thread marches per launch
 * (1..64), top_in_lds: stage the fixed top surface in LDS when it fits (else
 * it is read from global memory).  Until mc_set_tuning is called the shape
 * follows the grid loaded last: float32 {4, 256, 8, 0} below 48x48 nodes,
 * {4, 512, 16, 0} up to 128x128, {4, 1024, 16, 0} from 128x128 on; float64
 * {3, 256, 4, 1}.  multi_blocks_per_cu (0..16, read from problems[0] by
 * mcmc_run_multi): 0 launches one block per (problem, chain, ray tile) work
 * item, k > 0 a persistent grid of k blocks per compute unit that strides
 * over the work table.  Gradients (float32): the march that precedes the
 * adjoint records every crossing, grad_slots records per thread and surface
 * (0 = 2 x rays_per_thread + 16; -1 = none, every chain's gradient then comes
 * from re-walking its rays, as it does for a chain whose records overflow);
 * adjoint_rows > 0 caps the node rows an adjoint block accumulates at once
 * (0 = as many as fit the LDS).  Both change performance only.
 */
typedef struct {
    int march_variant;
    int block;
    int rays_per_thread;
    int top_in_lds;
    int multi_blocks_per_cu;
    int grad_slots;
    int adjoint_rows;
} mc_tuning;

mc_status mc_set_tuning(mc_problem *p, const mc_tuning *t);
mc_status mc_get_tuning(const mc_problem *p, mc_tuning *t);

/*
 * The paper's sampler (Sec. 3.1, 3.2): NUTS (Hoffman & Gelman 2014) in its
 * multinomial form with the generalised no-U-turn criterion, dual-averaging
 * step size adaptation toward target_accept and windowed diagonal
 * inverse-mass estimation during warm-up, on the exact march's gradient.
 * Chains run in lock step: one batched log-posterior gradient per leapfrog
 * step for all chains, doublings stop once every tree is finished.
 * Definition (shared with the reference implementation in the tests):
 *   momentum p_i = z_i / sqrt(inv_mass_i), z_i the (i%2)-th normal of pair
 *   i/2 of Philox (chain, step, tag 5); doubling d grows the side v = -1 iff
 *   the first uniform of (tag 6, j = d) is < 1/2; inside a subtree leaf k
 *   becomes the proposal with probability w_k / sum_{j<=k} w_j (tag 7, j =
 *   leaf index in the trajectory), w = exp(H0 - H); a valid subtree's
 *   proposal replaces the tree's with probability min(1, W_sub / W_tree)
 *   (tag 8, j = d); H - H0 > max_delta_h (or NaN) is a divergence, which
 *   drops the subtree and ends the transition; each completed block of two
 *   halves, and each merge, passes the three generalised criteria or ends
 *   the transition (a turning subtree is dropped).  A state of zero density
 *   does not move.  Warm-up: transition k uses exp(log eps_k) of dual
 *   averaging (gamma 0.05, t0 10, kappa 0.75); slow windows (initial buffer
 *   75, windows from 25 doubling, terminal buffer 50; 15/75/10 % below 150
 *   transitions) end with inv_mass = (n/(n+5)) var + 1e-3 * 5/(n+5) of their
 *   draws and a restart of dual averaging from the current step; after the
 *   warm-up eps = exp(log eps_bar).  Step k of the call uses Philox step
 *   step_offset + k.
 */
typedef struct {
    int64_t n_warmup;       /* adapting transitions first (>= 0) */
    int64_t n_steps;        /* transitions after the warm-up (>= 0) */
    int max_depth;          /* tree depth cap in [1, 10]; the paper's 256-step cap is 8 */
    int adapt_mass;         /* 1: estimate inv_mass during the warm-up (needs inv_mass) */
    double max_delta_h;     /* divergence threshold on H - H0 (> 0; 1000 is usual) */
    double target_accept;   /* dual-averaging target in (0, 1); the paper uses 0.8 */
    uint64_t seed;          /* Philox4x32-10 key */
    uint64_t step_offset;   /* Philox step of the first transition */
    int latent;             /* 1: the states are the latent CAR fields x (the paper's sampler
                               parametrisation, see latent_to_heights); 0: the heights */
    double *r_state;        /* device [n][S-1] float64 in (0, 1), in/out, or NULL: sample every
                               chain's CAR dependence r_l too (latent = 1 only; see nuts_run) */
} mc_nuts_config;

/*
 * NUTS on n_chains chains (stream-ordered, device arrays):
 *   heights [n][S-1][R][C] in/out, logpost [n] out (recomputed on entry),
 *   step_size [n] f64 in/out (in: the start of dual averaging, or the step
 *   used when n_warmup = 0; out: the adapted step), inv_mass [n][S-1][R][C]
 *   f64 in/out or NULL (identity), and optional per-transition outputs
 *   [n][n_warmup + n_steps]: tree_depth, n_leapfrog, diverged (int32) and
 *   accept_stat (f64, mean of min(1, w) over the leaves computed).
 * Device memory: about (6 + 5 (max_depth + 1)) * 8 + 9 * sizeof(state)
 * bytes per chain and free node, plus the gradient workspaces.  Errors:
 * MC_ERR_ARG for invalid sizes or pointers.  Under set_voxel_model or
 * set_pixel_quadrature NUTS runs on that model's gradient.
 * Hierarchical r (Sec. 2.2.1, r_l ~ Uniform(0, 1); Sec. 3.1, the sampler's
 * vector holds all unknowns): with cfg->r_state and latent = 1 each chain's
 * state is z = (x, eta), eta_l = logit r_l, of log density
 *   log L(H(x, r)) + sum_l [log det(Q(r_l))/2 - x_l' Q(r_l) x_l / 2
 *                           - (N/2) log 2 pi + log(r_l (1 - r_l))],
 * H(x, r) the copula map with Sigma11(r_l) (closed-form torus sums per
 * chain).  inv_mass is then [n][(S-1) R C + S-1] (the fields, then eta),
 * logpost holds that density, and r_state is updated.  Momentum normals are
 * drawn over the S-1 extra coordinates as over the others (pair i/2).
 */
mc_status nuts_run(mc_problem *p, const mc_nuts_config *cfg, int n_chains, void *heights, double *logpost,
                   double *step_size, double *inv_mass, int32_t *tree_depth, int32_t *n_leapfrog,
                   int32_t *diverged, double *accept_stat, void *stream);

/*
 * The latent parametrisation (Sec. 2.2.1, 3.1): the CAR fields x_l ~
 * N(0, Q_l^-1) of the free surfaces, [n][S-1][R][C] in the state precision,
 * and the heights H_l = (1 - u) H_{l-1} + u H_top, u = Phi(x_l /
 * sqrt(Sigma11_l)), H_0 = 0, at the problem's r.  With cfg->latent = 1,
 * nuts_run samples x with log density log L(H(x)) + sum_l [log det(Q_l)/2 -
 * x_l' Q_l x_l / 2 - (N/2) log 2 pi], which has no boundaries; logpost then
 * holds that density.  Both maps are stream-ordered on device arrays; the
 * inverse takes strictly ordered heights under the top (others give
 * non-finite x).
 */
mc_status latent_to_heights(mc_problem *p, int n_chains, const void *x, void *heights, void *stream);
mc_status heights_to_latent(mc_problem *p, int n_chains, const void *heights, void *x, void *stream);

/*
 * Nested R-hat (Sec. 3.2) of every free node from one draw per chain:
 * chains c = k*n_within + m of heights [n_super*n_within][S-1][R][C] form
 * n_super super-chains.  rhat[(S-1)*R*C] (device f64) = sqrt(1 + B / W), B
 * the variance of the super-chain means (divisor n_super - 1), W the mean
 * over super-chains of the variance of their chains about the super-chain
 * mean (divisor n_within - 1).  n_super, n_within >= 2.
 */
mc_status nested_rhat(mc_problem *p, int n_super, int n_within, const void *heights, double *rhat,
                      void *stream);

/*
 * Random-walk Metropolis on many independent problems at once (paper
 * Sec. 3.2: independent chains vectorised on one device, here across
 * problems as well).  Problem i runs cfgs[i] on its n_chains[i] chains with
 * device arrays heights[i], logposts[i], n_accept[i] laid out as in
 * mcmc_run.  Every step is one proposal launch and one prior/accept launch
 * for all chains of all problems, plus one persistent march launch per grid
 * size class over a static work table of (problem, chain, ray tile) items;
 * cfgs[0].graph_steps steps are captured in one HIP graph.  A chain's
 * results equal those of mcmc_run on its problem alone with the same
 * launch shape (the same device code runs for it).
 * Sampled r (Sec. 2.2.1): cfgs[i].r_state (with r_step, n_accept_r) as in
 * mcmc_run, given for every problem or for none; log posteriors are then
 * recomputed on entry at each chain's r.
 * Requirements: the same device, precision and n_surfaces for every problem,
 * kernel = 0, equal n_steps and graph_steps, distinct handles.  Errors are
 * reported on problems[0] (mc_last_error(problems[0])).
 */
mc_status mcmc_run_multi(int n_problems, mc_problem *const *problems, const mc_run_config *cfgs,
                         const int *n_chains, void *const *heights, double *const *logposts,
                         int64_t *const *n_accept, void *stream);

/* ------------------------------------------------------------------------ */
/* Serving: posterior-inference jobs batched as they arrive                  */
/* ------------------------------------------------------------------------ */
/*
 * A server owns one GPU and a scheduler thread.  Jobs (one inference problem
 * each: geometry, sensors, counts, chains, steps) are submitted at any time
 * and wait in a FIFO queue; the scheduler admits the queue head whenever
 * fewer than max_jobs jobs are resident and the job's device footprint fits
 * in the memory budget beside the resident ones.  Resident jobs keep their
 * chain state in device memory and advance together in rounds of
 * steps_per_round random-walk Metropolis steps (one mcmc_run_multi-style
 * graph launch per round over every resident job); jobs join and leave at
 * round boundaries, and admission work (uploads, the initial log posterior)
 * overlaps the running round.  When a job has taken n_steps steps the
 * scheduler computes its posterior summary on the device from the last state
 * of every chain (paper Sec. 3.2 keeps only each chain's last state): the
 * per-node mean and standard deviation over chains, the chain with the
 * highest log posterior and its state, and the acceptance rate; copies it to
 * host memory and frees the job's device memory.
 *
 * A job's results depend only on its own description: it draws its random
 * numbers from its own seed with the step counter it has reached, and its
 * launch shape is a function of its grid, so it gives the same bits alone
 * and in any mix.
 */
typedef struct mc_server mc_server;

typedef struct {
    int device;
    int precision;          /* MC_F32 or MC_F64 */
    size_t memory_budget;   /* bytes of device memory resident jobs may use; 0 = free memory - reserve */
    size_t reserve;         /* bytes kept free when memory_budget = 0 */
    int max_jobs;           /* jobs resident at once (>= 1) */
    int steps_per_round;    /* steps per round (>= 1), captured as one HIP graph */
} mc_server_config;

/* Host arrays are copied by mc_server_submit and may be freed on return.
 * Shapes and units as in load_geometry_grid / set_sensors / set_counts;
 * init[S-1][R][C] is the common starting state of every chain (the paper's
 * shared initialisation); block / rays_per_thread = 0 take the default
 * launch shape for the grid. */
typedef struct {
    int n_surfaces, n_rows, n_cols;
    double extent_x, extent_y;
    const double *density, *top, *car_r;
    int n_sensors, n_pix;
    const double *sensor_pos, *dirs, *exposure;
    double atten_len;
    const int32_t *counts;
    int n_chains;
    const double *init;
    int64_t n_steps;
    double step_size;
    uint64_t seed;
    int block, rays_per_thread;
    double r_step;          /* > 0: every chain also samples its r_l (start: car_r), by the logit-scale
                               random walk of this step as in mcmc_run; 0: r fixed at car_r */
} mc_job_desc;

enum { MC_JOB_QUEUED = 0, MC_JOB_RUNNING = 1, MC_JOB_DONE = 2, MC_JOB_FAILED = 3 };

typedef struct {
    int status;                         /* MC_JOB_* */
    int map_chain;                      /* chain with the highest final log posterior */
    int64_t steps_done;
    double t_submit, t_admit, t_done;   /* seconds on the server's steady clock (0 = not yet) */
    double accept_rate;                 /* accepted / (n_chains * n_steps) */
    double map_logpost;
    size_t footprint;                   /* device bytes charged against the budget */
    double r_mean[3];                   /* sampled r: mean over chains of each free surface's last r */
    double r_accept_rate;               /* sampled r: accepted / (n_chains * (S-1) * n_steps) */
} mc_job_info;

typedef struct {
    int64_t submitted, admitted, done, failed, rounds;
    int resident, queued, max_resident;
    size_t bytes_in_use, peak_bytes, budget;
    double busy_seconds;                /* wall time with at least one resident job */
    double now;                         /* the server clock */
} mc_server_stats;

mc_status mc_server_create(const mc_server_config *cfg, mc_server **out);
/* Stops accepting jobs, lets resident and queued jobs finish when drain != 0
 * (else abandons them), joins the scheduler and frees everything. */
void mc_server_destroy(mc_server *s, int drain);
const char *mc_server_last_error(const mc_server *s);
/* Validates and copies the job; fails with MC_ERR_NOMEM when its footprint
 * exceeds the whole budget. */
mc_status mc_server_submit(mc_server *s, const mc_job_desc *job, int64_t *job_id);
/* State of a job; once MC_JOB_DONE the summary is copied into the non-NULL
 * host arrays mean, std, map_state (each [S-1][R][C] float64). */
mc_status mc_server_poll(mc_server *s, int64_t job_id, mc_job_info *info, double *mean, double *std,
                         double *map_state);
/* Forget a finished job's summary (host memory). */
mc_status mc_server_release(mc_server *s, int64_t job_id);
/* Blocks until every submitted job is done or failed, or timeout_s passes
 * (MC_ERR_STATE on time-out). */
mc_status mc_server_wait_idle(mc_server *s, double timeout_s);
mc_status mc_server_get_stats(mc_server *s, mc_server_stats *st);

/* ------------------------------------------------------------------------ */
/* Test support                                                              */
/* ------------------------------------------------------------------------ */

/* Writes the Philox4x32-10 draws the samplers use, for n consecutive j
   starting at j0: out_u32[n*4] raw words and out_normal[n*2] Box-Muller
   normals (device pointers; either may be NULL).  Synchronous. */
mc_status mc_debug_philox(int hip_device, uint64_t seed, uint32_t chain, uint64_t step, uint32_t tag,
                          uint32_t j0, int n, uint32_t *out_u32, double *out_normal);

/*
 * Measurement support: the sustained issue rate of non-packed vector FMAs
 * (kind 0 = float32 v_fma_f32, 1 = float64 v_fma_f64) on `hip_device`, in
 * lane-operations per second, from a kernel of independent FMA chains that
 * fills every SIMD (best of 3 timed launches).  Synchronous.  MC_ERR_ARG for
 * a NULL output or unknown kind.
 */
mc_status mc_measure_valu_rate(int hip_device, int kind, double *lane_ops_per_s);

/* Times the ray-march kernel alone: `iters` back-to-back launches of the
   march over n_chains states (device `heights`, as in logpost_batch) between
   two HIP events recorded on `stream`; waits for them and writes the mean
   milliseconds per launch.  For benchmarks and roofline reports. */
mc_status mc_time_march(mc_problem *p, int n_chains, const void *heights, int iters, void *stream,
                        float *ms_per_launch);

/*
 * Timing of the voxel model's two kernels alone (HIP events on `stream`,
 * `iters` back-to-back launches each): the smoothed-density kernel and the
 * linearised-likelihood kernel, mean milliseconds per launch.  Needs
 * set_voxel_model; heights as for logpost_batch.
 */
mc_status mc_time_voxel(mc_problem *p, int n_chains, const void *heights, int iters, void *stream,
                        float *ms_density, float *ms_likelihood);

/* Mean milliseconds per launch of the adjoint march kernel alone on
 * `stream` (HIP events over `iters` launches), after one full gradient
 * evaluation of the n_chains states has produced its forward opacities.
 * Synchronous; the handle's gradient workspaces are used and overwritten. */
mc_status mc_time_adjoint(mc_problem *p, int n_chains, const void *heights, int iters, void *stream,
                          float *ms_per_launch);

/* Library version string. */
const char *mc_version(void);

#ifdef __cplusplus
}
#endif

#endif /* MUONCAVE_H */
