/*
 * muon_oracle.c -- plain FP64 CPU oracle for the block-cave muon-tomography
 * posterior (arXiv 2603.28907).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is compiled and called by the test
 * suite, the smoke check and the benchmark's CPU-baseline leg.  The product
 * (HIP) path never links, loads or calls it, and it shares no code with it.
 *
 * Everything here is written for clarity over speed: one ray at a time, one
 * cell at a time, FP64 throughout.  Each function names the passage of the
 * paper it follows.
 *
 * Readings of the paper taken here, where it is silent or schematic:
 *  - Geometry: vertex-centred nodes x_i = i*X/(R-1), y_j = j*Y/(C-1); row i
 *    runs along x, column j along y, H[l][i][j] in C order (Sec. 2.1.1, the
 *    array-indexing figure).  Surfaces are bilinear inside each cell.
 *  - Density: unit l lies between surface l-1 and l (surface 0 = floor z=0)
 *    with density rho[l-1]; zero above the top surface and outside the box
 *    [0,X]x[0,Y]x[0,Z_top], Z_top = max of the top surface (the continuum
 *    form of the layer density eq. def_LM_density_grid with the Heaviside
 *    indicator).
 *  - Opacity: O = int rho du along the ray (Sec. 2.1.1) evaluated exactly:
 *    O = sum_l (rho_l - rho_{l+1}) * L_l, where L_l is the length of ray
 *    inside the box lying below surface l.
 *  - Expected counts: lambda_p = E_p * exp(-O_p / Lambda), one ray per pixel
 *    (eq. expected_counts with the intensity replaced by an exponential
 *    attenuation and the solid-angle integral by its midpoint value).
 *  - Likelihood: independent Poisson counts (eq. def_likelihood), normalised
 *    (the -lgamma(C+1) term is kept).
 *  - Prior: Gaussian copula over a periodic proper CAR field per free
 *    surface (Sec. 2.2.1): H_l = (1-u) H_{l-1} + u H_top, u = Phi(x/sqrt(S11)),
 *    x ~ N(0, Q^-1), Q = diag(A1) - r A on the periodic 4-neighbour grid.
 *    Its density in H-space is written out by change of variables.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

typedef struct {
    int S, R, C;              /* surfaces incl. the fixed top; node grid rows x cols */
    double X, Y;              /* footprint extents (m) */
    const double *density;    /* [S]   density of unit l = 1..S (g/cm^3) */
    const double *top;        /* [R*C] fixed top surface (m) */
    const double *car_r;      /* [S-1] CAR dependence per free surface */
    int n_s, n_pix;           /* sensors, pixels per sensor */
    const double *pos;        /* [n_s*3] */
    const double *dirs;       /* [n_s*n_pix*3] unit vectors, d_z > 0 */
    const double *exposure;   /* [n_s*n_pix] */
    double atten;             /* Lambda, in the opacity unit (g/cm^3 * m) */
    const int32_t *counts;    /* [n_s*n_pix] observed counts (may be NULL) */
    /* Smoothed voxel forward model (Sec. 2.1.2, 2.1.4); n_z = 0 selects the
       exact march.  vox_ref = Rhat(H_ref) [R][C][n_z], the linearisation point. */
    int n_z;
    double gamma;
    const double *vox_ref;
    /* Solid-angle pixels (eq. expected_counts): with n_sub > 0 the rays are
       sub-rays, n_sub consecutive ones per pixel, lambda_p = sum_q sub_w[q]
       I(O_q) with log I tabulated at n_tab uniform nodes over [0, tab_omax];
       counts then hold one value per pixel. */
    int n_sub;
    const double *sub_w;
    int n_tab;
    double tab_omax;
    const double *tab_logI;
} orc_problem;

typedef struct {
    double cells;       /* cells visited with positive length */
    double tests;       /* (cell, surface) pairs examined */
    double roots;       /* quadratic roots found strictly inside a cell interval */
    double crossings;   /* sign changes of z - h along the ray */
    double min_fprime;  /* smallest |d(z-h)/dt| at a crossing (conditioning) */
    /* optional conditioning report of the crossing-form gradient (for the
       tolerances of tests): per node, a bound on how far an evaluation that
       rounds z - h by eps_z and each contribution by eps_rel can move the
       gradient of this ray's term */
    double *gcond;      /* [S][R][C] accumulator, or NULL */
    double cond_g;      /* |dLL/dO| of the ray */
    double cond_gerr;   /* bound on the error of dLL/dO of the ray */
    double eps_z, eps_rel;
    double eps_w;       /* absolute rounding of a bilinear weight (local coordinates) */
    double lid_band;    /* crossings this close below the box lid may be dropped as its kink */
} orc_stats;

/* ------------------------------------------------------------------------- */
/* Geometry helpers                                                            */
/* ------------------------------------------------------------------------- */

static double top_max(const orc_problem *p) {
    double m = -INFINITY;
    for (int i = 0; i < p->R * p->C; ++i) if (p->top[i] > m) m = p->top[i];
    return m;
}

/* Bilinear surface value at local cell coordinates (s, w) in [0,1]^2. */
static double bilinear(const double *Hl, int C, int a, int b, double s, double w) {
    double h00 = Hl[a * C + b], h10 = Hl[(a + 1) * C + b];
    double h01 = Hl[a * C + b + 1], h11 = Hl[(a + 1) * C + b + 1];
    return h00 * (1 - s) * (1 - w) + h10 * s * (1 - w) + h01 * (1 - s) * w + h11 * s * w;
}

/* Ray parameter at which the ray leaves the box (Sec. 2.1.1: the domain is a box). */
static double exit_param(const orc_problem *p, const double q[3], const double d[3], double ztop) {
    double T = (ztop - q[2]) / d[2];
    if (d[0] > 0) T = fmin(T, (p->X - q[0]) / d[0]);
    if (d[0] < 0) T = fmin(T, -q[0] / d[0]);
    if (d[1] > 0) T = fmin(T, (p->Y - q[1]) / d[1]);
    if (d[1] < 0) T = fmin(T, -q[1] / d[1]);
    return T > 0 ? T : 0.0;
}

/* Real roots of c2 t^2 + c1 t + c0 strictly inside (0, tmax), sorted. */
static int roots_in(double c2, double c1, double c0, double tmax, double out[2]) {
    double r[2];
    int n = 0;
    if (c2 == 0.0) {
        if (c1 != 0.0) r[n++] = -c0 / c1;
    } else {
        double disc = c1 * c1 - 4.0 * c2 * c0;
        if (disc >= 0.0) {
            double sq = sqrt(disc);
            double q = -0.5 * (c1 + (c1 >= 0 ? sq : -sq));
            if (q != 0.0) { r[n++] = q / c2; r[n++] = c0 / q; }
            else r[n++] = 0.0; /* c1 = c0 = 0: double root at 0 */
        }
    }
    int k = 0;
    for (int i = 0; i < n; ++i) if (r[i] > 0.0 && r[i] < tmax) out[k++] = r[i];
    if (k == 2 && out[0] > out[1]) { double t = out[0]; out[0] = out[1]; out[1] = t; }
    if (k == 2 && out[0] == out[1]) k = 1;
    return k;
}

/*
 * March one ray through all S surfaces.
 *
 * surf: [S][R][C] all surfaces (free ones then the top).
 * L:    [S] output, L[l] = length of ray (inside the box) below surface l+1.
 * gO:   optional [S][R][C] accumulator; if non-NULL, gscale * dO/dH is added
 *       (the crossing form of the derivative: each crossing t_c of surface l
 *       moves with dt_c/dH_n = w_n / f'(t_c), where f = z - h and w_n is the
 *       bilinear weight of node n at the crossing point).
 * Returns the opacity O = sum_l (rho_l - rho_{l+1}) L_l.
 *
 * Method: walk the cells crossed by the ray's xy-projection in order
 * (Amanatides & Woo 2-D traversal).  In a cell the surface restricted to the
 * ray is a quadratic in t, so f(t) = z(t) - h(t) is a quadratic; its roots
 * split the cell interval into pieces, and each piece is classified by the
 * sign of f evaluated directly (not through the quadratic) at its midpoint.
 */
static double march_ray(const orc_problem *p, const double *surf, const double q[3],
                        const double d[3], double ztop, double *L, double *gO, double gscale,
                        orc_stats *st) {
    const int S = p->S, R = p->R, C = p->C;
    const double hx = p->X / (R - 1), hy = p->Y / (C - 1);
    const double T = exit_param(p, q, d, ztop);
    int prev_below[16];
    for (int l = 0; l < S; ++l) { L[l] = 0.0; prev_below[l] = -1; }

    int a = (int)floor(q[0] / hx), b = (int)floor(q[1] / hy);
    if (a > R - 2) a = R - 2;
    if (a < 0) a = 0;
    if (b > C - 2) b = C - 2;
    if (b < 0) b = 0;
    double t0 = 0.0;
    while (t0 < T) {
        double tnx = INFINITY, tny = INFINITY;
        if (d[0] > 0) tnx = ((a + 1) * hx - q[0]) / d[0];
        if (d[0] < 0) tnx = (a * hx - q[0]) / d[0];
        if (d[1] > 0) tny = ((b + 1) * hy - q[1]) / d[1];
        if (d[1] < 0) tny = (b * hy - q[1]) / d[1];
        double t1 = fmin(fmin(tnx, tny), T);
        if (t1 > t0) {
            if (st) st->cells += 1;
            /* local coordinates at the cell entry and their rates along the ray */
            double s0 = (q[0] + t0 * d[0]) / hx - a, w0 = (q[1] + t0 * d[1]) / hy - b;
            double z0 = q[2] + t0 * d[2];
            double ds = d[0] / hx, dw = d[1] / hy, tau1 = t1 - t0;
            for (int l = 0; l < S; ++l) {
                const double *Hl = surf + (size_t)l * R * C;
                double h00 = Hl[a * C + b], h10 = Hl[(a + 1) * C + b];
                double h01 = Hl[a * C + b + 1], h11 = Hl[(a + 1) * C + b + 1];
                double A = h10 - h00, B = h01 - h00, D = h11 - h10 - h01 + h00;
                /* f(tau) = c0 + c1 tau + c2 tau^2, tau = t - t0 */
                double c0 = z0 - (h00 + A * s0 + B * w0 + D * s0 * w0);
                double c1 = d[2] - (A * ds + B * dw + D * (s0 * dw + w0 * ds));
                double c2 = -D * ds * dw;
                double r[2];
                int nr = roots_in(c2, c1, c0, tau1, r);
                if (st) { st->tests += 1; st->roots += nr; }
                if (st && st->gcond && nr == 0 && c2 != 0.0) {
                    /* a near miss: an extremum of f within eps_z of zero may be a
                       pair of crossings at rounding depth, |f'| = 2 sqrt(|c2| eps_z) */
                    double tv = -c1 / (2.0 * c2);
                    if (tv > 0.0 && tv < tau1 && fabs(c0 + tv * (c1 + c2 * tv)) <= st->eps_z) {
                        double sv = s0 + tv * ds, wv = w0 + tv * dw;
                        double drho = fabs(p->density[l] - (l + 1 < S ? p->density[l + 1] : 0.0));
                        double fpair = 2.0 * sqrt(fabs(c2) * st->eps_z);
                        double wt[4] = {(1 - sv) * (1 - wv), sv * (1 - wv), (1 - sv) * wv, sv * wv};
                        size_t nd[4] = {(size_t)a * C + b, (size_t)(a + 1) * C + b, (size_t)a * C + b + 1,
                                        (size_t)(a + 1) * C + b + 1};
                        double *G = st->gcond + (size_t)l * R * C;
                        for (int m = 0; m < 4; ++m) G[nd[m]] += drho * st->cond_g * fabs(wt[m]) * 2.0 / fpair;
                    }
                }
                double cuts[4];
                int nc = 0;
                cuts[nc++] = 0.0;
                for (int k = 0; k < nr; ++k) cuts[nc++] = r[k];
                cuts[nc++] = tau1;
                for (int k = 0; k + 1 < nc; ++k) {
                    double len = cuts[k + 1] - cuts[k];
                    /* pieces at the rounding scale of t carry no sign information
                       (e.g. a root within rounding of a cell edge or of the exit
                       point); skipping them changes L by at most 1e-12 (1 + T) */
                    if (!(len > 1e-12 * (1.0 + T))) continue;
                    double tm = 0.5 * (cuts[k] + cuts[k + 1]);
                    double sm = s0 + tm * ds, wm = w0 + tm * dw;
                    double fm = (z0 + tm * d[2]) - bilinear(Hl, C, a, b, sm, wm);
                    int below = fm < 0.0;
                    if (below) L[l] += len;
                    if (prev_below[l] >= 0 && prev_below[l] != below) {
                        /* a crossing at the start of this piece */
                        double tc = cuts[k];
                        double fp = c1 + 2.0 * c2 * tc;
                        if (st) {
                            st->crossings += 1;
                            if (fabs(fp) < st->min_fprime) st->min_fprime = fabs(fp);
                        }
                        if (st && st->gcond && fp != 0.0) {
                            /* the crossing moves by eps_z/|f'|: its bilinear weights by
                               (|ds|+|dw|) eps_z/|f'| and 1/|f'| by |f''| eps_z/|f'|^3; a
                               crossing within eps_z of tangency may vanish with its partner */
                            double sc = s0 + tc * ds, wc = w0 + tc * dw;
                            double f1 = fabs(fp), f2 = 2.0 * fabs(c2), kw = fabs(ds) + fabs(dw);
                            double drho = fabs(p->density[l] - (l + 1 < S ? p->density[l + 1] : 0.0));
                            double pair = f1 * f1 <= 4.0 * fabs(c2) * st->eps_z ? 2.0 / f1 : 0.0;
                            double wt[4] = {(1 - sc) * (1 - wc), sc * (1 - wc), (1 - sc) * wc, sc * wc};
                            size_t nd[4] = {(size_t)a * C + b, (size_t)(a + 1) * C + b, (size_t)a * C + b + 1,
                                            (size_t)(a + 1) * C + b + 1};
                            /* near a cell edge the float32 walk may place the crossing in the
                               neighbouring cell, whose patch has another slope: |f'| jumps
                               there (the bilinear surface is only continuous), so the
                               contribution can take the neighbour's 1/|f'|.  The band: node
                               lines rounded by 2^-22 (X + |q| + T) in space, the crossing
                               by 2 eps_z |d| / |f'|. */
                            double jump = 0.0;
                            for (int e = 0; e < 4; ++e) {
                                int ax = e < 2;                       /* x-edge (s = 0, 1) or y-edge (w = 0, 1) */
                                int hi = e & 1;
                                double dist = ax ? (hi ? 1.0 - sc : sc) * hx : (hi ? 1.0 - wc : wc) * hy;
                                double band = ldexp((ax ? p->X + fabs(q[0]) : p->Y + fabs(q[1])) + T, -22) +
                                              2.0 * st->eps_z * fabs(ax ? d[0] : d[1]) / f1;
                                if (!(dist <= band)) continue;
                                int na = a + (ax ? (hi ? 1 : -1) : 0), nb = b + (ax ? 0 : (hi ? 1 : -1));
                                if (na < 0 || na > R - 2 || nb < 0 || nb > C - 2) continue;
                                double sn = sc - (na - a), wn = wc - (nb - b);   /* local coordinates in the neighbour */
                                double n00 = Hl[na * C + nb], n10 = Hl[(na + 1) * C + nb];
                                double n01 = Hl[na * C + nb + 1], n11 = Hl[(na + 1) * C + nb + 1];
                                double Dn = n11 - n10 - n01 + n00;
                                double slope = ((n10 - n00) + Dn * wn) * ds + ((n01 - n00) + Dn * sn) * dw;
                                double fn = fabs(d[2] - slope);
                                double j = fn > 0.0 ? fabs(1.0 / f1 - 1.0 / fn) : INFINITY;
                                if (j > jump) jump = j;
                            }
                            /* a crossing just below the box lid may be taken for the lid's kink
                               and dropped: its whole contribution */
                            double zc = z0 + tc * d[2];
                            double lid = ztop - zc <= st->lid_band + 2.0 * st->eps_z * fabs(d[2]) / f1 ? 1.0 / f1 : 0.0;
                            double *G = st->gcond + (size_t)l * R * C;
                            for (int m = 0; m < 4; ++m) {
                                double w = fabs(wt[m]);
                                /* |f'| comes from the end values of the cell's piece of length
                                   tau1: their rounding moves it by 2 eps_z / tau1 */
                                G[nd[m]] += drho * (st->cond_g * (w * (st->eps_rel / f1 + f2 * st->eps_z / (f1 * f1 * f1) +
                                                                       2.0 * st->eps_z / (tau1 * f1 * f1) + pair + jump + lid) +
                                                                  (kw * st->eps_z / f1 + 2.0 * st->eps_w) / f1) +
                                                    st->cond_gerr * w / f1);
                            }
                        }
                        if (gO && fp != 0.0) {
                            double sc = s0 + tc * ds, wc = w0 + tc * dw;
                            double g = gscale * (p->density[l] - (l + 1 < S ? p->density[l + 1] : 0.0)) / fabs(fp);
                            double *G = gO + (size_t)l * R * C;
                            G[a * C + b] += g * (1 - sc) * (1 - wc);
                            G[(a + 1) * C + b] += g * sc * (1 - wc);
                            G[a * C + b + 1] += g * (1 - sc) * wc;
                            G[(a + 1) * C + b + 1] += g * sc * wc;
                        }
                    }
                    prev_below[l] = below;
                }
            }
        }
        if (t1 >= T) break;
        if (tnx <= tny) a += d[0] > 0 ? 1 : -1;
        else b += d[1] > 0 ? 1 : -1;
        if (a < 0 || a > R - 2 || b < 0 || b > C - 2) break;
        t0 = t1;
    }
    double O = 0.0;
    for (int l = 0; l < S; ++l) {
        double rho_above = (l + 1 < S) ? p->density[l + 1] : 0.0;
        O += (p->density[l] - rho_above) * L[l];
    }
    return O;
}

/* Build [S][R][C] from the free surfaces [S-1][R][C] and the fixed top. */
static double *stack_surfaces(const orc_problem *p, const double *free_h) {
    size_t N = (size_t)p->R * p->C;
    double *s = (double *)malloc(sizeof(double) * N * p->S);
    memcpy(s, free_h, sizeof(double) * N * (p->S - 1));
    memcpy(s + N * (p->S - 1), p->top, sizeof(double) * N);
    return s;
}

/* ------------------------------------------------------------------------- */
/* Forward model: opacity, expected counts, likelihood                        */
/* ------------------------------------------------------------------------- */

/* Opacity of every ray for one state of the free surfaces.
   O: [n_s*n_pix]; Lout: optional [n_s*n_pix][S]; st: optional totals. */
void orc_opacity(const orc_problem *p, const double *free_h, double *O, double *Lout, orc_stats *st) {
    double *surf = stack_surfaces(p, free_h);
    double ztop = top_max(p);
    double L[16];
    if (st) { memset(st, 0, sizeof(*st)); st->min_fprime = INFINITY; }
    for (int s = 0; s < p->n_s; ++s)
        for (int k = 0; k < p->n_pix; ++k) {
            int ray = s * p->n_pix + k;
            O[ray] = march_ray(p, surf, p->pos + 3 * s, p->dirs + 3 * (size_t)ray, ztop, L, NULL, 0.0, st);
            if (Lout) for (int l = 0; l < p->S; ++l) Lout[(size_t)ray * p->S + l] = L[l];
        }
    free(surf);
}

/* Poisson log-likelihood of the counts given opacities (eq. def_likelihood):
   sum_p C_p log(lambda_p) - lambda_p - log(C_p!),  lambda_p = E_p exp(-O_p/Lambda). */
double orc_loglik(const orc_problem *p, const double *O) {
    double ll = 0.0;
    int n = p->n_s * p->n_pix;
    for (int i = 0; i < n; ++i) {
        double lam = p->exposure[i] * exp(-O[i] / p->atten);
        double c = (double)p->counts[i];
        ll += c * (log(p->exposure[i]) - O[i] / p->atten) - lam - lgamma(c + 1.0);
    }
    return ll;
}

/* ------------------------------------------------------------------------- */
/* Prior: Gaussian copula over a periodic proper CAR field (Sec. 2.2.1)       */
/* ------------------------------------------------------------------------- */

/* Standard normal c.d.f. through the complementary error function. */
static double Phi(double w) { return 0.5 * erfc(-w / sqrt(2.0)); }

/* Inverse standard normal c.d.f. for u in (0, 0.5]: safeguarded Newton
   iteration on log Phi(w) = log u (concave in w, so the tails converge as
   fast as the centre) inside the bracket [-40, 0]. */
double orc_ndtri_lower(double u) {
    if (!(u > 0.0)) return -INFINITY;
    if (u >= 0.5) return 0.0;
    double lu = log(u);
    double lo = -40.0, hi = 0.0, w = -1.0;
    for (int it = 0; it < 400; ++it) {
        double P = Phi(w);
        double g = log(P) - lu; /* increasing in w */
        if (g > 0) hi = w; else lo = w;
        double pdf = exp(-0.5 * w * w) / sqrt(2.0 * M_PI);
        double wn = (P > 0 && pdf > 0) ? w - g * P / pdf : 0.5 * (lo + hi);
        if (!(wn > lo && wn < hi)) wn = 0.5 * (lo + hi);
        if (fabs(wn - w) <= 4e-16 * fabs(w)) { w = wn; break; }
        w = wn;
    }
    return w;
}

/* Phi^-1(u) where u = (H-a)/(b-a) and v = 1-u = (b-H)/(b-a) are both given:
   the tail nearer to u is evaluated directly, the other through symmetry. */
static double ndtri_uv(double u, double v) {
    return (u <= 0.5) ? orc_ndtri_lower(u) : -orc_ndtri_lower(v);
}

/* log det Q and Sigma_11 = (Q^-1)_11 for Q = diag(A1) - rA on the periodic
   R x C grid.  Q is block-circulant, so its eigenvalues are
   mu_km = 4 - 2r(cos(2 pi k/R) + cos(2 pi m/C)), and by translation
   invariance the diagonal of Q^-1 is its trace over N. */
void orc_car_consts(int R, int C, double r, double *logdet, double *sigma11) {
    double sl = 0.0, si = 0.0;
    for (int k = 0; k < R; ++k)
        for (int m = 0; m < C; ++m) {
            double mu = 4.0 - 2.0 * r * (cos(2.0 * M_PI * k / R) + cos(2.0 * M_PI * m / C));
            sl += log(mu);
            si += 1.0 / mu;
        }
    *logdet = sl;
    *sigma11 = si / ((double)R * C);
}

/*
 * log prior density of the free surfaces, in H-space.
 * For free surface l with a = H_{l-1} (0 for l = 1) and b = H_top:
 *   u = (H_l - a)/(b - a),  w = Phi^-1(u),  x = s w,  s = sqrt(Sigma_11),
 *   log p(H_l | H_{l-1}) = log N(x; 0, Q^-1) + sum log|dx/du| + sum log|du/dH|
 *     = 1/2 log det Q - 1/2 x^T Q x + N log s + 1/2 sum w^2 - sum log(b - a)
 * (the (N/2) log 2 pi terms of the normal density and of phi(w) cancel), with
 *   x^T Q x = 4(1-r) sum x_i^2 + r sum_{edges} (x_i - x_j)^2
 * over the 2N right/down edges of the periodic grid.  States outside the
 * support 0 < H_1 < ... < H_{S-1} < H_top give -inf.
 * If grad is non-NULL ([S][R][C]), the gradient is added to it.
 */
static double log_prior_grad_r(const orc_problem *p, const double *free_h, const double *r_vals, double *grad);

double orc_log_prior_grad(const orc_problem *p, const double *free_h, double *grad) {
    return log_prior_grad_r(p, free_h, p->car_r, grad);
}

/* The same density with the dependence parameters r_vals[S-1] given
   explicitly (the hierarchical model treats them as unknowns). */
double orc_log_prior_r(const orc_problem *p, const double *free_h, const double *r_vals) {
    return log_prior_grad_r(p, free_h, r_vals, NULL);
}

static double log_prior_grad_r(const orc_problem *p, const double *free_h, const double *r_vals, double *grad) {
    const int R = p->R, C = p->C, N = R * C;
    double total = 0.0;
    double *w = (double *)malloc(sizeof(double) * N);
    double *u = (double *)malloc(sizeof(double) * N);
    double *dd = (double *)malloc(sizeof(double) * N);
    for (int l = 0; l < p->S - 1; ++l) {
        const double *H = free_h + (size_t)l * N;
        const double *A = (l == 0) ? NULL : free_h + (size_t)(l - 1) * N;
        double logdet, s11;
        double r = r_vals[l];
        orc_car_consts(R, C, r, &logdet, &s11);
        double s = sqrt(s11);
        double sum_w2 = 0.0, sum_logd = 0.0;
        for (int i = 0; i < N; ++i) {
            double a = A ? A[i] : 0.0, b = p->top[i];
            double d = b - a;
            double ui = (H[i] - a) / d, vi = (b - H[i]) / d;
            if (!(d > 0.0) || !(ui > 0.0) || !(vi > 0.0)) {
                free(w); free(u); free(dd);
                return -INFINITY;
            }
            w[i] = ndtri_uv(ui, vi);
            u[i] = ui;
            dd[i] = d;
            sum_w2 += w[i] * w[i];
            sum_logd += log(d);
        }
        double sx2 = 0.0, sedge = 0.0;
        for (int i = 0; i < R; ++i)
            for (int j = 0; j < C; ++j) {
                double xi = s * w[i * C + j];
                double xr = s * w[i * C + (j + 1) % C];
                double xd = s * w[((i + 1) % R) * C + j];
                sx2 += xi * xi;
                sedge += (xi - xr) * (xi - xr) + (xi - xd) * (xi - xd);
            }
        double quad = 4.0 * (1.0 - r) * sx2 + r * sedge;
        total += 0.5 * logdet - 0.5 * quad + N * log(s) + 0.5 * sum_w2 - sum_logd;

        if (grad) {
            double *gH = grad + (size_t)l * N;
            double *gA = (l == 0) ? NULL : grad + (size_t)(l - 1) * N;
            double *gB = grad + (size_t)(p->S - 1) * N;
            for (int i = 0; i < R; ++i)
                for (int j = 0; j < C; ++j) {
                    int n = i * C + j;
                    double wi = w[n];
                    double nb = w[i * C + (j + 1) % C] + w[i * C + (j + C - 1) % C] +
                                w[((i + 1) % R) * C + j] + w[((i + R - 1) % R) * C + j];
                    /* d/dw_n of the log density in w-space */
                    double G = -s11 * (4.0 * (1.0 - r) * wi + r * (4.0 * wi - nb)) + wi;
                    double phi = exp(-0.5 * wi * wi) / sqrt(2.0 * M_PI);
                    double gu = G / phi; /* d/du_n */
                    double d = dd[n];
                    gH[n] += gu / d;
                    if (gA) gA[n] += gu * (u[n] - 1.0) / d + 1.0 / d;
                    gB[n] += -gu * u[n] / d - 1.0 / d;
                }
        }
    }
    free(w); free(u); free(dd);
    return total;
}

double orc_log_prior(const orc_problem *p, const double *free_h) {
    return orc_log_prior_grad(p, free_h, NULL);
}

/* ------------------------------------------------------------------------- */
/* Posterior                                                                   */
/* ------------------------------------------------------------------------- */

double orc_voxel_logpost_lik(const orc_problem *p, const double *free_h, double *O);
double orc_quad_loglik(const orc_problem *p, const double *O, double *lam);

/* log posterior (likelihood + prior, normalised) of one state. */
double orc_logpost(const orc_problem *p, const double *free_h) {
    double lpr = orc_log_prior(p, free_h);
    if (lpr == -INFINITY) return -INFINITY;
    int n = p->n_s * p->n_pix;
    if (n == 0) return lpr;
    if (p->n_z > 0) return lpr + orc_voxel_logpost_lik(p, free_h, NULL);
    if (p->n_sub > 0) {
        double *O = (double *)malloc(sizeof(double) * n);
        orc_opacity(p, free_h, O, NULL, NULL);
        double ll = orc_quad_loglik(p, O, NULL);
        free(O);
        return lpr + ll;
    }
    double *O = (double *)malloc(sizeof(double) * n);
    orc_opacity(p, free_h, O, NULL, NULL);
    double ll = orc_loglik(p, O);
    free(O);
    return ll + lpr;
}

/* log posterior of n_chains states [n_chains][S-1][R][C], parallel over chains. */
void orc_logpost_batch(const orc_problem *p, int n_chains, const double *free_all, double *lp) {
    size_t M = (size_t)(p->S - 1) * p->R * p->C;
#pragma omp parallel for schedule(dynamic, 1)
    for (int c = 0; c < n_chains; ++c) lp[c] = orc_logpost(p, free_all + M * c);
}

/*
 * Gradient of the log posterior with respect to every surface height,
 * grad: [S][R][C] (the fixed top surface included).  Returns the log
 * posterior.  Out-of-support states return -inf and a zero gradient.
 * Likelihood part: dLL/dO_p = (lambda_p - C_p)/Lambda times dO_p/dH from the
 * crossing form in march_ray; prior part from orc_log_prior_grad.
 */
double orc_loglik_grad_add(const orc_problem *p, const double *free_h, double *grad);

static double voxel_loglik_grad_add(const orc_problem *p, const double *surf, double *grad);
static double quad_loglik_grad_add(const orc_problem *p, const double *free_h, double *grad);

/* Log-likelihood and its gradient (added to grad [S][R][C]) under the
   problem's forward model: the exact march (one ray per pixel, or the
   solid-angle quadrature over sub-rays), or the smoothed voxel model. */
static double loglik_grad_add_any(const orc_problem *p, const double *free_h, double *grad) {
    if (p->n_z == 0 && p->n_sub > 0) return quad_loglik_grad_add(p, free_h, grad);
    if (p->n_z == 0) return orc_loglik_grad_add(p, free_h, grad);
    if (p->n_s * p->n_pix == 0) return 0.0;
    double *surf = stack_surfaces(p, free_h);
    double ll = voxel_loglik_grad_add(p, surf, grad);
    free(surf);
    return ll;
}

double orc_grad(const orc_problem *p, const double *free_h, double *grad) {
    size_t NS = (size_t)p->S * p->R * p->C;
    memset(grad, 0, sizeof(double) * NS);
    double lpr = orc_log_prior_grad(p, free_h, grad);
    if (lpr == -INFINITY) { memset(grad, 0, sizeof(double) * NS); return -INFINITY; }
    double ll = loglik_grad_add_any(p, free_h, grad);
    if (ll == -INFINITY) { memset(grad, 0, sizeof(double) * NS); return -INFINITY; }
    return lpr + ll;
}

/* Log-likelihood (eq. def_likelihood) of a state and its gradient in every
   surface height, added into grad [S][R][C]. */
double orc_loglik_grad_add(const orc_problem *p, const double *free_h, double *grad) {
    int n = p->n_s * p->n_pix;
    if (n == 0) return 0.0;
    double *surf = stack_surfaces(p, free_h);
    double ztop = top_max(p);
    double L[16], ll = 0.0;
    for (int s = 0; s < p->n_s; ++s)
        for (int k = 0; k < p->n_pix; ++k) {
            int ray = s * p->n_pix + k;
            const double *q = p->pos + 3 * s, *d = p->dirs + 3 * (size_t)ray;
            double O = march_ray(p, surf, q, d, ztop, L, NULL, 0.0, NULL);
            double lam = p->exposure[ray] * exp(-O / p->atten);
            double c = (double)p->counts[ray];
            ll += c * (log(p->exposure[ray]) - O / p->atten) - lam - lgamma(c + 1.0);
            double g = (lam - c) / p->atten;
            march_ray(p, surf, q, d, ztop, L, grad, g, NULL);
        }
    free(surf);
    return ll;
}

/* OpenMP threads a batch call uses (for reporting host timings). */
int orc_max_threads(void) { return omp_get_max_threads(); }

void orc_grad_batch(const orc_problem *p, int n_chains, const double *free_all, double *lp, double *grad_all) {
    size_t M = (size_t)(p->S - 1) * p->R * p->C, NS = (size_t)p->S * p->R * p->C;
#pragma omp parallel for schedule(dynamic, 1)
    for (int c = 0; c < n_chains; ++c) lp[c] = orc_grad(p, free_all + M * c, grad_all + NS * c);
}

/* ------------------------------------------------------------------------- */
/* Counter-based RNG: Philox4x32-10 (Salmon, Moraes, Dror & Shaw, SC'11)      */
/* ------------------------------------------------------------------------- */

/* One Philox4x32 round: two 32x32->64 multiplications of counter words 0 and
   2 by the round multipliers, hi/lo halves mixed with words 1, 3 and the key. */
static void philox_round(uint32_t ctr[4], const uint32_t key[2]) {
    uint64_t p0 = (uint64_t)0xD2511F53u * ctr[0];
    uint64_t p1 = (uint64_t)0xCD9E8D57u * ctr[2];
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t n0 = hi1 ^ ctr[1] ^ key[0];
    uint32_t n2 = hi0 ^ ctr[3] ^ key[1];
    ctr[0] = n0; ctr[1] = lo1; ctr[2] = n2; ctr[3] = lo0;
}

/* Ten rounds; the key is advanced by the Weyl constants between rounds. */
void orc_philox4x32_10(const uint32_t in[4], const uint32_t key_in[2], uint32_t out[4]) {
    uint32_t ctr[4] = {in[0], in[1], in[2], in[3]};
    uint32_t key[2] = {key_in[0], key_in[1]};
    for (int r = 0; r < 10; ++r) {
        if (r > 0) { key[0] += 0x9E3779B9u; key[1] += 0xBB67AE85u; }
        philox_round(ctr, key);
    }
    memcpy(out, ctr, sizeof(ctr));
}

/* Counter layout: (j, step lo32, step hi16 | tag << 16, chain); key = seed. */
static void philox_draw(uint64_t seed, uint32_t chain, uint64_t step, uint32_t tag, uint32_t j, uint32_t out[4]) {
    uint32_t ctr[4] = {j, (uint32_t)step, (uint32_t)((step >> 32) & 0xFFFFu) | (tag << 16), chain};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    orc_philox4x32_10(ctr, key, out);
}

/* 53-bit uniform in [0,1) from two 32-bit words. */
static double u53(uint32_t a, uint32_t b) {
    return ((double)(a >> 5) * 67108864.0 + (double)(b >> 6)) * (1.0 / 9007199254740992.0);
}

void orc_uniform_pair(uint64_t seed, uint32_t chain, uint64_t step, uint32_t tag, uint32_t j, double u[2]) {
    uint32_t o[4];
    philox_draw(seed, chain, step, tag, j, o);
    u[0] = u53(o[0], o[1]);
    u[1] = u53(o[2], o[3]);
}

/* Two standard normals by the Box-Muller transform of one uniform pair. */
void orc_normal_pair(uint64_t seed, uint32_t chain, uint64_t step, uint32_t tag, uint32_t j, double z[2]) {
    double u[2];
    orc_uniform_pair(seed, chain, step, tag, j, u);
    double rad = sqrt(-2.0 * log(1.0 - u[0]));
    double th = 2.0 * M_PI * u[1];
    z[0] = rad * cos(th);
    z[1] = rad * sin(th);
}

void orc_raw_philox(uint64_t seed, uint32_t chain, uint64_t step, uint32_t tag, uint32_t j, uint32_t out[4]) {
    philox_draw(seed, chain, step, tag, j, out);
}

/* ------------------------------------------------------------------------- */
/* MCMC: random-walk Metropolis and MALA                                       */
/* ------------------------------------------------------------------------- */

enum { TAG_PROPOSAL = 0, TAG_ACCEPT = 1, TAG_MOMENTUM = 2, TAG_R_PROPOSAL = 3, TAG_R_ACCEPT = 4,
       TAG_NUTS_MOMENTUM = 5, TAG_NUTS_DIRECTION = 6, TAG_NUTS_LEAF = 7, TAG_NUTS_MERGE = 8 };

static double round_state(double x, int state_f32) { return state_f32 ? (double)(float)x : x; }

/*
 * Random-walk Metropolis on the free surfaces (Sec. 3.1: MCMC needs the
 * posterior only up to a constant, so log alpha = lp' - lp).
 * Proposal H' = H + sigma z with z_i the (i%2)-th normal of pair j = i/2 of
 * (chain, step, tag 0); accept iff log U < log alpha with U the first uniform
 * of (chain, step, tag 1, j = 0).  free_all/lp/n_acc are updated in place;
 * lp entries that are NaN on entry are computed first.  If margins is non-NULL,
 * margins[c*n_steps + k] = |log U - log alpha| of step k (decision margin).
 * state_f32 != 0 rounds every proposed state to float32 (states stored in
 * single precision).
 */
void orc_mcmc_rw(const orc_problem *p, int n_chains, double *free_all, double *lp, int64_t *n_acc,
                 int64_t n_steps, uint64_t step_offset, double sigma, uint64_t seed, int state_f32,
                 double *margins) {
    size_t M = (size_t)(p->S - 1) * p->R * p->C;
#pragma omp parallel for schedule(dynamic, 1)
    for (int c = 0; c < n_chains; ++c) {
        double *H = free_all + M * c;
        double *prop = (double *)malloc(sizeof(double) * M);
        if (isnan(lp[c])) lp[c] = orc_logpost(p, H);
        for (int64_t k = 0; k < n_steps; ++k) {
            uint64_t step = step_offset + (uint64_t)k;
            for (size_t i = 0; i < M; i += 2) {
                double z[2];
                orc_normal_pair(seed, (uint32_t)c, step, TAG_PROPOSAL, (uint32_t)(i / 2), z);
                prop[i] = round_state(H[i] + sigma * z[0], state_f32);
                if (i + 1 < M) prop[i + 1] = round_state(H[i + 1] + sigma * z[1], state_f32);
            }
            double lpp = orc_logpost(p, prop);
            double u[2];
            orc_uniform_pair(seed, (uint32_t)c, step, TAG_ACCEPT, 0, u);
            double la = lpp - lp[c];
            double lu = log(u[0]);
            if (margins) margins[(size_t)c * n_steps + k] = fabs(lu - la);
            if (lu < la) {
                memcpy(H, prop, sizeof(double) * M);
                lp[c] = lpp;
                n_acc[c] += 1;
            }
        }
        free(prop);
    }
}

/*
 * Metropolis-adjusted Langevin (HMC with one leapfrog step, Sec. 3.1):
 *   H' = H + (eps^2/2) M^-1 g(H) + eps M^-1/2 z,   z from tag 2,
 *   log alpha = lp' - lp + log q(H | H') - log q(H' | H),
 *   log q(y | x) = -sum_i (y_i - x_i - (eps^2/2) Minv_i g_i(x))^2 / (2 eps^2 Minv_i).
 * inv_mass: [S-1][R][C] or NULL (= 1).  Only the free surfaces move.
 */
void orc_mcmc_mala(const orc_problem *p, int n_chains, double *free_all, double *lp, int64_t *n_acc,
                   int64_t n_steps, uint64_t step_offset, double eps, const double *inv_mass,
                   uint64_t seed, int state_f32, double *margins) {
    size_t M = (size_t)(p->S - 1) * p->R * p->C, NS = (size_t)p->S * p->R * p->C;
#pragma omp parallel for schedule(dynamic, 1)
    for (int c = 0; c < n_chains; ++c) {
        double *H = free_all + M * c;
        double *prop = (double *)malloc(sizeof(double) * M);
        double *g = (double *)malloc(sizeof(double) * NS);
        double *gp = (double *)malloc(sizeof(double) * NS);
        lp[c] = orc_grad(p, H, g);
        for (int64_t k = 0; k < n_steps; ++k) {
            uint64_t step = step_offset + (uint64_t)k;
            double lq_fwd = 0.0;
            for (size_t i = 0; i < M; i += 2) {
                double z[2];
                orc_normal_pair(seed, (uint32_t)c, step, TAG_MOMENTUM, (uint32_t)(i / 2), z);
                for (int e = 0; e < 2 && i + e < M; ++e) {
                    size_t n = i + e;
                    double mi = inv_mass ? inv_mass[n] : 1.0;
                    double mean = H[n] + 0.5 * eps * eps * mi * g[n];
                    prop[n] = round_state(mean + eps * sqrt(mi) * z[e], state_f32);
                    double dv = prop[n] - mean;
                    lq_fwd -= dv * dv / (2.0 * eps * eps * mi);
                }
            }
            double lpp = orc_grad(p, prop, gp);
            double la = -INFINITY;
            if (lpp > -INFINITY) {
                double lq_bwd = 0.0;
                for (size_t n = 0; n < M; ++n) {
                    double mi = inv_mass ? inv_mass[n] : 1.0;
                    double mean = prop[n] + 0.5 * eps * eps * mi * gp[n];
                    double dv = H[n] - mean;
                    lq_bwd -= dv * dv / (2.0 * eps * eps * mi);
                }
                la = lpp - lp[c] + lq_bwd - lq_fwd;
            }
            double u[2];
            orc_uniform_pair(seed, (uint32_t)c, step, TAG_ACCEPT, 0, u);
            double lu = log(u[0]);
            if (margins) margins[(size_t)c * n_steps + k] = fabs(lu - la);
            if (lu < la) {
                memcpy(H, prop, sizeof(double) * M);
                memcpy(g, gp, sizeof(double) * NS);
                lp[c] = lpp;
                n_acc[c] += 1;
            }
        }
        free(prop); free(g); free(gp);
    }
}

/* Single-ray march exposed for tests: returns O, fills L[S] and stats. */
/*
 * Random-walk Metropolis on the free surfaces and, within each step, on the
 * hierarchical dependence parameters r_l of the CAR layers (Sec. 2.2.1:
 * r_l iid Uniform(0, 1) a priori).  Step k of chain c:
 *   1. H-update: as orc_mcmc_rw, with the chain's own r in the prior;
 *   2. for each free surface l in order: eta = logit(r_l), eta' = eta + tau z
 *      (z: component l % 2 of normal pair l / 2 of tag 3), r' = 1/(1+e^-eta');
 *      the target density of eta is p(C | H) p(H | r) r (1 - r) (the uniform
 *      prior carried to eta), so
 *        log alpha = log p(H | r') - log p(H | r) + log(r'(1-r')) - log(r(1-r))
 *      (the likelihood does not depend on r); accept iff log U < log alpha with
 *      U the first uniform of pair l of tag 4; a proposal that rounds to 0 or
 *      1 is rejected.
 * r_all: [n_chains][S-1] in/out; n_acc_r: [n_chains][S-1] in/out (may be NULL);
 * lp: the log posterior log p(C|H) + log p(H|r), NaN entries computed first.
 * margins (optional, [n_chains][n_steps][S]): |log U - log alpha| of the
 * H decision and of each r decision.
 */
void orc_mcmc_rw_r(const orc_problem *p, int n_chains, double *free_all, double *r_all, double *lp,
                   int64_t *n_acc, int64_t *n_acc_r, int64_t n_steps, uint64_t step_offset, double sigma,
                   double tau, uint64_t seed, int state_f32, double *margins) {
    const int S1 = p->S - 1;
    size_t M = (size_t)S1 * p->R * p->C;
    const int n_ray = p->n_s * p->n_pix;
#pragma omp parallel for schedule(dynamic, 1)
    for (int c = 0; c < n_chains; ++c) {
        double *H = free_all + M * c;
        double *r = r_all + (size_t)S1 * c;
        double *prop = (double *)malloc(sizeof(double) * M);
        double *O = n_ray ? (double *)malloc(sizeof(double) * n_ray) : NULL;
        if (isnan(lp[c])) {
            double pr = orc_log_prior_r(p, H, r);
            double ll = 0.0;
            if (pr > -INFINITY && n_ray) {
                orc_opacity(p, H, O, NULL, NULL);
                ll = orc_loglik(p, O);
            }
            lp[c] = pr + ll;
        }
        for (int64_t k = 0; k < n_steps; ++k) {
            uint64_t step = step_offset + (uint64_t)k;
            double *mg = margins ? margins + ((size_t)c * n_steps + k) * (S1 + 1) : NULL;
            /* 1. H */
            for (size_t i = 0; i < M; i += 2) {
                double z[2];
                orc_normal_pair(seed, (uint32_t)c, step, TAG_PROPOSAL, (uint32_t)(i / 2), z);
                prop[i] = round_state(H[i] + sigma * z[0], state_f32);
                if (i + 1 < M) prop[i + 1] = round_state(H[i + 1] + sigma * z[1], state_f32);
            }
            double lpp = orc_log_prior_r(p, prop, r);
            if (lpp > -INFINITY && n_ray) {
                orc_opacity(p, prop, O, NULL, NULL);
                lpp += orc_loglik(p, O);
            }
            double u[2];
            orc_uniform_pair(seed, (uint32_t)c, step, TAG_ACCEPT, 0, u);
            double la = lpp - lp[c], lu = log(u[0]);
            if (mg) mg[0] = fabs(lu - la);
            if (lu < la) {
                memcpy(H, prop, sizeof(double) * M);
                lp[c] = lpp;
                n_acc[c] += 1;
            }
            /* 2. r_l, one surface at a time */
            for (int l = 0; l < S1; ++l) {
                double z[2];
                orc_normal_pair(seed, (uint32_t)c, step, TAG_R_PROPOSAL, (uint32_t)(l / 2), z);
                double rl = r[l];
                double eta = log(rl / (1.0 - rl)) + tau * z[l % 2];
                double rn = 1.0 / (1.0 + exp(-eta));
                double la_r = -INFINITY, d_prior = 0.0;
                if (rn > 0.0 && rn < 1.0) {
                    const double jac = log(rn * (1.0 - rn)) - log(rl * (1.0 - rl));
                    if (lp[c] > -INFINITY) {
                        double p0 = orc_log_prior_r(p, H, r);
                        r[l] = rn;
                        double p1 = orc_log_prior_r(p, H, r);
                        r[l] = rl;
                        d_prior = p1 - p0;
                    }
                    /* a state outside the support has p(H | r) = 0 for every r:
                       there r moves under its prior alone and lp stays -inf */
                    la_r = d_prior + jac;
                }
                double ur[2];
                orc_uniform_pair(seed, (uint32_t)c, step, TAG_R_ACCEPT, (uint32_t)l, ur);
                double lur = log(ur[0]);
                if (mg) mg[1 + l] = fabs(lur - la_r);
                if (lur < la_r) {
                    r[l] = rn;
                    lp[c] += d_prior;
                    if (n_acc_r) n_acc_r[(size_t)S1 * c + l] += 1;
                }
            }
        }
        free(prop);
        free(O);
    }
}

double orc_march_one(const orc_problem *p, const double *free_h, const double q[3], const double d[3],
                     double *L, orc_stats *st) {
    double *surf = stack_surfaces(p, free_h);
    if (st) { memset(st, 0, sizeof(*st)); st->min_fprime = INFINITY; }
    double O = march_ray(p, surf, q, d, top_max(p), L, NULL, 0.0, st);
    free(surf);
    return O;
}

/* Conditioning report of the likelihood gradient (test tolerances only):
   out [S][R][C] = per node, the sum over the rays' crossings of the bound
   described at orc_stats.gcond (weights rounded by eps_w, crossings within
   lid_band of the box lid dropped), with dL/dO of each ray from its opacity and
   its error lambda |dO| / Lambda^2 from the opacity error dO of the ray:
   dO_ray[ray] when given, else o_rel |O| + rho_max n_cross eps_z / min|f'|
   + 1e-6.  With g_ray (and g_err) given, |g_ray[ray]| and g_err[ray] take the
   place of that one-ray dL/dO and its error (the solid-angle pixel model,
   whose dL/dO of a sub-ray also depends on the pixel's other sub-rays). */
void orc_grad_conditioning(const orc_problem *p, const double *free_h, double eps_z, double eps_rel, double eps_w,
                           double lid_band, const double *dO_ray, double o_rel, const double *g_ray,
                           const double *g_err, double *out) {
    double *surf = stack_surfaces(p, free_h);
    double ztop = top_max(p), L[16], rho_max = 0.0;
    for (int l = 0; l < p->S; ++l) rho_max = fmax(rho_max, fabs(p->density[l]));
    memset(out, 0, sizeof(double) * (size_t)p->S * p->R * p->C);
    for (int s = 0; s < p->n_s; ++s)
        for (int k = 0; k < p->n_pix; ++k) {
            int ray = s * p->n_pix + k;
            const double *q = p->pos + 3 * s, *d = p->dirs + 3 * (size_t)ray;
            orc_stats st;
            memset(&st, 0, sizeof(st));
            st.min_fprime = INFINITY;
            double O = march_ray(p, surf, q, d, ztop, L, NULL, 0.0, &st);
            double lam = p->exposure[ray] * exp(-O / p->atten);
            double dO = o_rel * fabs(O) + 1e-6;
            if (st.crossings > 0) dO += rho_max * st.crossings * eps_z / fmax(st.min_fprime, 1e-12);
            if (dO_ray) dO = fabs(dO_ray[ray]);
            orc_stats st2;
            memset(&st2, 0, sizeof(st2));
            st2.min_fprime = INFINITY;
            st2.gcond = out;
            st2.cond_g = g_ray ? fabs(g_ray[ray]) : fabs(lam - (double)p->counts[ray]) / p->atten;
            st2.cond_gerr = g_ray ? g_err[ray] : lam * dO / (p->atten * p->atten);
            st2.eps_z = eps_z;
            st2.eps_rel = eps_rel;
            st2.eps_w = eps_w;
            st2.lid_band = lid_band;
            march_ray(p, surf, q, d, ztop, L, NULL, 0.0, &st2);
        }
    free(surf);
}

/* Per-ray diagnostics for every ray: crossings and the smallest |f'| at a
   crossing (used to widen tolerances for ill-conditioned rays). */
void orc_ray_stats(const orc_problem *p, const double *free_h, double *crossings, double *min_fprime,
                   double *cells) {
    double *surf = stack_surfaces(p, free_h);
    double ztop = top_max(p), L[16];
    for (int s = 0; s < p->n_s; ++s)
        for (int k = 0; k < p->n_pix; ++k) {
            int ray = s * p->n_pix + k;
            orc_stats st;
            memset(&st, 0, sizeof(st));
            st.min_fprime = INFINITY;
            march_ray(p, surf, p->pos + 3 * s, p->dirs + 3 * (size_t)ray, ztop, L, NULL, 0.0, &st);
            if (crossings) crossings[ray] = st.crossings;
            if (min_fprime) min_fprime[ray] = st.min_fprime;
            if (cells) cells[ray] = st.cells;
        }
    free(surf);
}

/* ------------------------------------------------------------------------- */
/* The paper's smoothed voxel forward model, linearised (Sec. 2.1.2, 2.1.4)   */
/* ------------------------------------------------------------------------- */
/*
 * Readings taken here:
 *  - The density grid shares the layer grid's lateral indices (the map
 *    (i,j) -> (x(i), y(j)) is the identity): voxel column (i,j) is the box
 *    [x_i - dx/2, x_i + dx/2] x [y_j - dy/2, y_j + dy/2] clipped to the
 *    footprint, dx = X/(R-1), dy = Y/(C-1).  Vertically n_z voxels of
 *    dz = Z_top/n_z fill [0, Z_top]; the height the paper writes k*dz is taken
 *    at the voxel's centre, z_k = (k + 1/2) dz.  Linear voxel index
 *    (i*C + j)*n_z + k (right-most index fastest).
 *  - Units: the S units of the layer model plus the air above the top surface
 *    (density 0; its upper interface is at +infinity, so its smooth indicator
 *    is 1 - sigma(H_S - z)).  With it the normalised weights form a partition
 *    of unity that leaves the air empty, as the hard-interface density does.
 *  - R0 = Rhat(H_ref) for a reference geometry given by the caller.
 *  - G_pv = d lambda_p / d R_v at R0 = -lambda_p(R0) L_pv / Lambda, with L_pv
 *    the length of ray p inside voxel v, lambda_p(R) = E_p exp(-O_p(R)/Lambda)
 *    and O_p(R) = sum_v L_pv R_v (the opacity of a piecewise-constant field).
 *  - A state whose linearised count lambda-hat_p is <= 0 at some pixel has
 *    zero likelihood (log posterior -inf).
 */

/* Scaled sigmoid (eq. def_sigmoid). */
double orc_sigmoid(double u, double gamma) { return 1.0 / (1.0 + exp(-u / gamma)); }

/* Normalised weights W[(i*C + j)*n_z + k][l], l = 0..S (units 1..S, then the
   air), from the smooth indicators D (eq. smooth_layer_indicators) divided by
   their sum (eq. def_LM_density_grid_smooth).  surf: [S][R][C], all surfaces. */
void orc_voxel_weights(const orc_problem *p, const double *surf, int n_z, double gamma, double *W) {
    const int S = p->S;
    const size_t N = (size_t)p->R * p->C;
    const double dz = top_max(p) / n_z;
    double D[17];
    for (size_t n = 0; n < N; ++n)
        for (int k = 0; k < n_z; ++k) {
            const double z = (k + 0.5) * dz;
            double below_prev = orc_sigmoid(0.0 - z, gamma);   /* H_0 = 0, the floor */
            double sum = 0.0;
            for (int l = 1; l <= S + 1; ++l) {
                const double below = l <= S ? orc_sigmoid(surf[(size_t)(l - 1) * N + n] - z, gamma) : 1.0;
                D[l - 1] = below - below_prev;
                sum += D[l - 1];
                below_prev = below;
            }
            double *w = W + ((size_t)n * n_z + k) * (S + 1);
            for (int l = 0; l <= S; ++l) w[l] = D[l] / sum;
        }
}

/* Smoothed density Rhat [R][C][n_z] = sum_l W_l R^(l) (eq. def_LM_density_grid_smooth). */
void orc_voxel_density(const orc_problem *p, const double *surf, int n_z, double gamma, double *Rhat) {
    const int S = p->S;
    const size_t V = (size_t)p->R * p->C * n_z;
    double *W = (double *)malloc(sizeof(double) * V * (S + 1));
    orc_voxel_weights(p, surf, n_z, gamma, W);
    for (size_t v = 0; v < V; ++v) {
        double r = 0.0;
        for (int l = 0; l < S; ++l) r += W[v * (S + 1) + l] * p->density[l];
        Rhat[v] = r;   /* the air (l = S) has density 0 */
    }
    free(W);
}

static int cmp_double(const void *a, const void *b) {
    double x = *(const double *)a, y = *(const double *)b;
    return (x > y) - (x < y);
}

/* Pieces of ray (q, d) inside the box, split at every voxel boundary plane
   (x = (i+1/2) dx, y = (j+1/2) dy, z = k dz) crossed inside (0, T): the
   crossing parameters are sorted and each interval's midpoint names its
   voxel.  vox/len hold at least R + C + n_z + 1 entries; returns the count. */
static int voxel_pieces(const orc_problem *p, const double q[3], const double d[3], int n_z, int *vox,
                        double *len) {
    const double ztop = top_max(p), T = exit_param(p, q, d, ztop);
    const double dx = p->X / (p->R - 1), dy = p->Y / (p->C - 1), dz = ztop / n_z;
    double *t = (double *)malloc(sizeof(double) * (p->R + p->C + n_z + 2));
    int m = 0;
    t[m++] = 0.0;
    t[m++] = T;
    for (int i = 0; i + 1 < p->R; ++i)
        if (d[0] != 0.0) {
            double tc = ((i + 0.5) * dx - q[0]) / d[0];
            if (tc > 0.0 && tc < T) t[m++] = tc;
        }
    for (int j = 0; j + 1 < p->C; ++j)
        if (d[1] != 0.0) {
            double tc = ((j + 0.5) * dy - q[1]) / d[1];
            if (tc > 0.0 && tc < T) t[m++] = tc;
        }
    for (int k = 1; k < n_z; ++k) {
        double tc = (k * dz - q[2]) / d[2];
        if (tc > 0.0 && tc < T) t[m++] = tc;
    }
    qsort(t, m, sizeof(double), cmp_double);
    int n = 0;
    for (int a = 0; a + 1 < m; ++a) {
        const double l = t[a + 1] - t[a];
        if (!(l > 0.0)) continue;
        const double tm = 0.5 * (t[a] + t[a + 1]);
        const double x = q[0] + tm * d[0], y = q[1] + tm * d[1], z = q[2] + tm * d[2];
        int i = (int)floor(x / dx + 0.5), j = (int)floor(y / dy + 0.5), k = (int)floor(z / dz);
        i = i < 0 ? 0 : (i > p->R - 1 ? p->R - 1 : i);
        j = j < 0 ? 0 : (j > p->C - 1 ? p->C - 1 : j);
        k = k < 0 ? 0 : (k > n_z - 1 ? n_z - 1 : k);
        vox[n] = (i * p->C + j) * n_z + k;
        len[n] = l;
        ++n;
    }
    free(t);
    return n;
}

/* Pieces of ray `ray` for the problem's n_z (tests). */
int orc_voxel_pieces(const orc_problem *p, int ray, int n_z, int *vox, double *len) {
    const int s = ray / p->n_pix;
    return voxel_pieces(p, p->pos + 3 * s, p->dirs + 3 * (size_t)ray, n_z, vox, len);
}

/* Linearised Poisson log-likelihood (eq. expected_counts_linearized_approx in
   eq. def_likelihood) of the smoothed density Rhat [R][C][n_z]:
   lambda-hat = lambda(R0) + G (Rhat - R0).  O (optional) receives the
   voxel opacity O_p(Rhat) of every ray. */
double orc_voxel_loglik(const orc_problem *p, const double *Rhat, double *O) {
    const int n_z = p->n_z, nr = p->n_s * p->n_pix;
    const double *R0 = p->vox_ref;
    int *vox = (int *)malloc(sizeof(int) * (p->R + p->C + n_z + 1));
    double *len = (double *)malloc(sizeof(double) * (p->R + p->C + n_z + 1));
    double ll = 0.0;
    for (int ray = 0; ray < nr; ++ray) {
        const int m = orc_voxel_pieces(p, ray, n_z, vox, len);
        double o = 0.0, o0 = 0.0;
        for (int a = 0; a < m; ++a) {
            o += len[a] * Rhat[vox[a]];
            o0 += len[a] * R0[vox[a]];
        }
        if (O) O[ray] = o;
        const double lam0 = p->exposure[ray] * exp(-o0 / p->atten);
        double lam = lam0;
        for (int a = 0; a < m; ++a) {
            const double g = -lam0 * len[a] / p->atten;   /* G_pv */
            lam += g * (Rhat[vox[a]] - R0[vox[a]]);
        }
        const double c = (double)p->counts[ray];
        if (!(lam > 0.0)) ll = -INFINITY;
        else ll += c * log(lam) - lam - lgamma(c + 1.0);
    }
    free(vox);
    free(len);
    return ll;
}

/* Gradient of the linearised voxel likelihood with respect to every surface
   height (the paper smooths the layer indicators so that gradient-based
   samplers can run on this model, Sec. 2.1.4).  By the chain rule through
   eq. expected_counts_linearized_approx and eq. def_LM_density_grid_smooth:
     dLL/dlambda-hat_p = C_p / lambda-hat_p - 1,
     dlambda-hat_p/dRhat_v = G_pv = -lambda_p(R0) L_pv / Lambda,
     B_v = dLL/dRhat_v = sum_p (C_p / lambda-hat_p - 1) G_pv,
   and Rhat of voxel (n, k) depends on the heights of column n only:
     Rhat = (sum_{l=1..S} (rho_l - rho_{l+1}) sigma_l - rho_1 sigma_0) / (1 - sigma_0),
     sigma_l = sigmoid((H_l,n - z_k) / gamma), rho_{S+1} = 0 (the air),
     dRhat/dH_l,n = (rho_l - rho_{l+1}) sigma_l (1 - sigma_l) / (gamma (1 - sigma_0)).
   So dLL/dH_l,n = sum_k B_(n,k) dRhat_(n,k)/dH_l,n.  grad [S][R][C] (the
   top surface included) is added to; returns LL (-inf, adding nothing, when
   some lambda-hat_p <= 0). */
static double voxel_loglik_grad_add(const orc_problem *p, const double *surf, double *grad) {
    const int S = p->S, n_z = p->n_z, nr = p->n_s * p->n_pix;
    const size_t N = (size_t)p->R * p->C, V = N * n_z;
    const double *R0 = p->vox_ref, gamma = p->gamma, dz = top_max(p) / n_z;
    double *Rhat = (double *)malloc(sizeof(double) * V), *B = (double *)calloc(V, sizeof(double));
    int *vox = (int *)malloc(sizeof(int) * (p->R + p->C + n_z + 1));
    double *len = (double *)malloc(sizeof(double) * (p->R + p->C + n_z + 1));
    orc_voxel_density(p, surf, n_z, gamma, Rhat);
    double ll = 0.0;
    for (int ray = 0; ray < nr; ++ray) {
        const int m = orc_voxel_pieces(p, ray, n_z, vox, len);
        double o0 = 0.0;
        for (int a = 0; a < m; ++a) o0 += len[a] * R0[vox[a]];
        const double lam0 = p->exposure[ray] * exp(-o0 / p->atten);
        double lam = lam0;
        for (int a = 0; a < m; ++a) lam += (-lam0 * len[a] / p->atten) * (Rhat[vox[a]] - R0[vox[a]]);
        const double c = (double)p->counts[ray];
        if (!(lam > 0.0)) { ll = -INFINITY; break; }
        ll += c * log(lam) - lam - lgamma(c + 1.0);
        const double dl = c / lam - 1.0;
        for (int a = 0; a < m; ++a) B[vox[a]] += dl * (-lam0 * len[a] / p->atten);
    }
    if (ll > -INFINITY) {
        for (size_t n = 0; n < N; ++n)
            for (int k = 0; k < n_z; ++k) {
                const double z = (k + 0.5) * dz;
                const double norm = 1.0 - orc_sigmoid(0.0 - z, gamma);
                for (int l = 0; l < S; ++l) {
                    const double sg = orc_sigmoid(surf[(size_t)l * N + n] - z, gamma);
                    const double drho = p->density[l] - (l + 1 < S ? p->density[l + 1] : 0.0);
                    grad[(size_t)l * N + n] += B[n * n_z + k] * drho * sg * (1.0 - sg) / (gamma * norm);
                }
            }
    }
    free(Rhat);
    free(B);
    free(vox);
    free(len);
    return ll;
}

/* Likelihood part of the log posterior under the voxel model; O as above. */
double orc_voxel_logpost_lik(const orc_problem *p, const double *free_h, double *O) {
    double *surf = stack_surfaces(p, free_h);
    const size_t V = (size_t)p->R * p->C * p->n_z;
    double *Rhat = (double *)malloc(sizeof(double) * V);
    orc_voxel_density(p, surf, p->n_z, p->gamma, Rhat);
    const double ll = orc_voxel_loglik(p, Rhat, O);
    free(Rhat);
    free(surf);
    return ll;
}

/* ------------------------------------------------------------------------- */
/* The paper's sampler: NUTS with step-size and diagonal-mass adaptation,     */
/* and nested R-hat (Sec. 3.1, 3.2)                                            */
/* ------------------------------------------------------------------------- */
/*
 * One NUTS transition (Hoffman & Gelman 2014) in its multinomial form with
 * the generalised no-U-turn criterion (Betancourt 2017), as the paper's
 * sampler library runs it.  The paper fixes the sampler, the 256-step
 * trajectory cap (tree depth 8), the 0.8 acceptance target and diagonal
 * preconditioning; the remaining details are read as follows.
 *  - Momentum p ~ N(0, M), M = diag(1/inv_mass): p_i = z_i / sqrt(inv_mass_i),
 *    z_i the (i%2)-th normal of pair i/2 of (chain, step, tag 5).
 *    H = -lp + p.(inv_mass p)/2.  Leapfrog of step v*eps (v = +-1):
 *    p += v eps/2 g;  x += v eps inv_mass p;  g = grad lp(x);  p += v eps/2 g.
 *  - The tree doubles up to max_depth times.  Doubling d extends the end on
 *    side v by a subtree of 2^d leaves, v = -1 iff the first uniform of
 *    (tag 6, j = d) is below 1/2.
 *  - A leaf with H - H0 > max_dH (or NaN) is a divergence: the subtree is
 *    dropped and the transition ends.
 *  - Inside a subtree the proposal is drawn leaf by leaf: leaf k replaces
 *    it with probability w_k / (w_1 + ... + w_k), w = exp(H0 - H), using the
 *    first uniform of (tag 7, j = index of the leaf in the trajectory); a
 *    valid subtree's proposal replaces the tree's with probability
 *    min(1, W_subtree / W_tree) (tag 8, j = d), and W_tree += W_subtree.
 *  - U-turns: whenever two adjacent halves A (grown first) and B of a block
 *    are complete (inside the subtree, and the old tree with the subtree),
 *    the block is turning unless crit(a_far, b_far, rho_A + rho_B),
 *    crit(a_far, b_near, rho_A + p_b_near) and crit(a_near, b_far,
 *    p_a_near + rho_B) all hold; crit(x, y, rho) = (x.M^-1 rho > 0 and
 *    y.M^-1 rho > 0), rho = sum of the momenta in the span, a_far/b_far the
 *    outer ends, a_near/b_near the adjacent ones.  A turning subtree is
 *    dropped; a turning tree ends the transition after its merge.
 *  - Acceptance statistic: mean over all leaves computed of min(1, w).
 *  - A state of zero density (outside the support) does not move.
 * Random numbers come from the same Philox4x32-10 streams as the other
 * samplers (key = seed, counter (j, step, tag, chain)).
 */
#define ORC_NUTS_MAX_DEPTH 12

/* Planted mistakes, for tests that show a pin can see them (0 = none):
 * bit 0 skips the U-turn checks of the blocks inside a subtree (only the
 * merges of whole subtrees are checked); bit 1 merges the proposal of a
 * subtree that turned inside instead of dropping it; bit 2 drops the
 * Jacobian of r = logistic(eta) from the latent density with r. */
static int g_nuts_fault = 0;
void orc_nuts_set_fault(int flags) { g_nuts_fault = flags; }

typedef double (*orc_target_fn)(const void *ctx, const double *x, double *grad);

typedef struct {
    int depth, n_leap, diverged, turned;
    double accept_stat, margin;
} orc_nuts_stats;

static double crit_dot(const double *x, const double *im, const double *rho, size_t M) {
    double s = 0.0;
    for (size_t i = 0; i < M; ++i) s += x[i] * (im ? im[i] : 1.0) * rho[i];
    return s;
}

static double nrm2(const double *x, size_t M) {
    double s = 0.0;
    for (size_t i = 0; i < M; ++i) s += x[i] * x[i];
    return sqrt(s);
}

/* One criterion: both ends' sharp momenta have a positive projection on rho.
   The margin records how close each dot product came to zero, relative. */
static int crit_ok(const double *x, const double *y, const double *rho, const double *im, size_t M,
                   double *margin) {
    double dx = crit_dot(x, im, rho, M), dy = crit_dot(y, im, rho, M);
    double sc = nrm2(rho, M) + 1e-300;
    double mx = fabs(dx) / (sc * (nrm2(x, M) + 1e-300)), my = fabs(dy) / (sc * (nrm2(y, M) + 1e-300));
    if (mx < *margin) *margin = mx;
    if (my < *margin) *margin = my;
    return dx > 0.0 && dy > 0.0;
}

/* turning of the merge of A (grown first) and B; tmp: M scratch */
static int turning3(const double *rho_a, const double *a_far, const double *a_near, const double *rho_b,
                    const double *b_near, const double *b_far, const double *im, size_t M, double *tmp,
                    double *margin) {
    int ok = 1;
    for (size_t i = 0; i < M; ++i) tmp[i] = rho_a[i] + rho_b[i];
    ok &= crit_ok(a_far, b_far, tmp, im, M, margin);
    for (size_t i = 0; i < M; ++i) tmp[i] = rho_a[i] + b_near[i];
    ok &= crit_ok(a_far, b_near, tmp, im, M, margin);
    for (size_t i = 0; i < M; ++i) tmp[i] = a_near[i] + rho_b[i];
    ok &= crit_ok(a_near, b_far, tmp, im, M, margin);
    return !ok;
}

static double logaddexp(double a, double b) {
    if (a == -INFINITY) return b;
    if (b == -INFINITY) return a;
    double m = a > b ? a : b;
    return m + log(exp(a - m) + exp(b - m));
}

static double first_uniform(uint64_t seed, uint32_t chain, uint64_t step, uint32_t tag, uint32_t j) {
    double u[2];
    orc_uniform_pair(seed, chain, step, tag, j, u);
    return u[0];
}

/* x, lp, g: the chain's state (updated in place); im: inverse mass or NULL */
static void nuts_transition(orc_target_fn target, const void *ctx, size_t M, double *x, double *lp, double *g,
                            double eps, const double *im, int max_depth, double max_dh, uint64_t seed,
                            uint32_t chain, uint64_t step, int state_f32, orc_nuts_stats *st) {
    const int L = max_depth + 1;
    if (!(*lp > -INFINITY)) {   /* a state of zero density does not move */
        st->depth = st->n_leap = st->diverged = st->turned = 0;
        st->accept_stat = 0.0;
        st->margin = INFINITY;
        return;
    }
    /* ends of the tree: [0] = backward (v = -1) side, [1] = forward side */
    double *xe[2], *pe[2], *ge[2];
    double *xs = malloc(sizeof(double) * M), *gs = malloc(sizeof(double) * M);     /* subtree proposal */
    double *xp = malloc(sizeof(double) * M), *gp = malloc(sizeof(double) * M);     /* tree proposal */
    double *rho = malloc(sizeof(double) * M), *p_near = malloc(sizeof(double) * M), *tmp = malloc(sizeof(double) * M);
    double *R = malloc(sizeof(double) * M * L), *F = malloc(sizeof(double) * M * L);
    double *sR = malloc(sizeof(double) * M * L), *sF = malloc(sizeof(double) * M * L), *sL = malloc(sizeof(double) * M * L);
    for (int e = 0; e < 2; ++e) {
        xe[e] = malloc(sizeof(double) * M);
        pe[e] = malloc(sizeof(double) * M);
        ge[e] = malloc(sizeof(double) * M);
    }
    /* momentum and the initial energy */
    double kin = 0.0;
    for (size_t i = 0; i < M; i += 2) {
        double z[2];
        orc_normal_pair(seed, chain, step, TAG_NUTS_MOMENTUM, (uint32_t)(i / 2), z);
        for (int e = 0; e < 2 && i + e < M; ++e) {
            double mi = im ? im[i + e] : 1.0;
            pe[0][i + e] = z[e] / sqrt(mi);
            kin += mi * pe[0][i + e] * pe[0][i + e];
        }
    }
    const double H0 = -*lp + 0.5 * kin;
    memcpy(pe[1], pe[0], sizeof(double) * M);
    for (int e = 0; e < 2; ++e) {
        memcpy(xe[e], x, sizeof(double) * M);
        memcpy(ge[e], g, sizeof(double) * M);
    }
    memcpy(xp, x, sizeof(double) * M);
    memcpy(gp, g, sizeof(double) * M);
    double lpp = *lp, logW = 0.0, sum_acc = 0.0, margin = INFINITY;
    memcpy(rho, pe[0], sizeof(double) * M);
    int depth = 0, n_leap = 0, diverged = 0, turned = 0;
    uint32_t leaf = 0;
    while (depth < max_depth) {
        const double ud = first_uniform(seed, chain, step, TAG_NUTS_DIRECTION, (uint32_t)depth);
        if (fabs(ud - 0.5) < margin) margin = fabs(ud - 0.5);
        const int side = ud < 0.5 ? 0 : 1;
        const double v = side ? 1.0 : -1.0;
        memcpy(p_near, pe[side], sizeof(double) * M);
        double logWs = -INFINITY, lps = 0.0;
        int valid = 1, turned_inside = 0;
        const int n_sub = 1 << depth;
        for (int i = 0; i < n_sub && valid; ++i) {
            /* leapfrog from this side's end */
            double *xx = xe[side], *pp = pe[side], *gg = ge[side];
            for (size_t k = 0; k < M; ++k) {
                pp[k] += 0.5 * v * eps * gg[k];
                xx[k] = round_state(xx[k] + v * eps * (im ? im[k] : 1.0) * pp[k], state_f32);
            }
            double lpl = target(ctx, xx, gg);
            double kl = 0.0;
            for (size_t k = 0; k < M; ++k) {
                pp[k] += 0.5 * v * eps * gg[k];
                kl += (im ? im[k] : 1.0) * pp[k] * pp[k];
            }
            ++n_leap;
            const double dH = (-lpl + 0.5 * kl) - H0;
            if (isfinite(dH) && fabs(dH - max_dh) < margin) margin = fabs(dH - max_dh);
            if (!(dH <= max_dh)) {          /* divergence (NaN included) */
                diverged = 1;
                valid = 0;
                if (dH == dH) sum_acc += fmin(1.0, exp(-dH));
                break;
            }
            const double lw = -dH;
            sum_acc += fmin(1.0, exp(lw));
            const double logWs_new = logaddexp(logWs, lw);
            const double ul = first_uniform(seed, chain, step, TAG_NUTS_LEAF, leaf);
            ++leaf;
            if (i > 0 && fabs(log(ul) - (lw - logWs_new)) < margin) margin = fabs(log(ul) - (lw - logWs_new));
            if (i == 0 || log(ul) < lw - logWs_new) {
                memcpy(xs, xx, sizeof(double) * M);
                memcpy(gs, gg, sizeof(double) * M);
                lps = lpl;
            }
            logWs = logWs_new;
            /* block bookkeeping: a level-j block holds 2^j consecutive leaves;
               its momentum sum is the sum of its two halves' sums, as in the
               recursive tree (the level-0 block is the leaf itself) */
            memcpy(R, pp, sizeof(double) * M);
            memcpy(F, pp, sizeof(double) * M);
            for (int j = 1; j <= depth; ++j) {
                if (((i + 1) & ((1 << j) - 1)) != 0) break;   /* blocks complete from level 1 up */
                /* a level-j block completed: halves A = saved sibling, B = the level j-1 block */
                const size_t a = (size_t)(j - 1) * M;
                if (!(g_nuts_fault & 1) && turning3(sR + a, sF + a, sL + a, R + a, F + a, pp, im, M, tmp, &margin)) {
                    valid = 0;
                    turned_inside = 1;
                    break;
                }
                double *Rj = R + (size_t)j * M;
                for (size_t k = 0; k < M; ++k) Rj[k] = sR[a + k] + R[a + k];
                memcpy(F + (size_t)j * M, sF + a, sizeof(double) * M);
            }
            if (!valid) break;
            for (int j = 0; j < depth; ++j) {
                if (((i + 1) & ((1 << j) - 1)) != 0 || !(((i + 1) >> j) & 1)) continue;
                /* a level-j block completed as the first half of its parent */
                const size_t a = (size_t)j * M;
                memcpy(sR + a, R + a, sizeof(double) * M);
                memcpy(sF + a, F + a, sizeof(double) * M);
                memcpy(sL + a, pp, sizeof(double) * M);
            }
        }
        if (!valid && !(turned_inside && (g_nuts_fault & 2))) break;
        /* merge the subtree into the tree */
        const double um = first_uniform(seed, chain, step, TAG_NUTS_MERGE, (uint32_t)depth);
        if (fabs(log(um) - (logWs - logW)) < margin) margin = fabs(log(um) - (logWs - logW));
        if (log(um) < logWs - logW) {
            memcpy(xp, xs, sizeof(double) * M);
            memcpy(gp, gs, sizeof(double) * M);
            lpp = lps;
        }
        logW = logaddexp(logW, logWs);
        const double *rho_b = R + (size_t)depth * M, *b_near = F + (size_t)depth * M;
        turned = turning3(rho, pe[1 - side], p_near, rho_b, b_near, pe[side], im, M, tmp, &margin);
        for (size_t k = 0; k < M; ++k) rho[k] += rho_b[k];
        ++depth;
        if (turned || !valid) break;
    }
    memcpy(x, xp, sizeof(double) * M);
    memcpy(g, gp, sizeof(double) * M);
    *lp = lpp;
    st->depth = depth;
    st->n_leap = n_leap;
    st->diverged = diverged;
    st->turned = turned;
    st->accept_stat = n_leap ? sum_acc / n_leap : 0.0;
    st->margin = margin;
    for (int e = 0; e < 2; ++e) { free(xe[e]); free(pe[e]); free(ge[e]); }
    free(xs); free(gs); free(xp); free(gp); free(rho); free(p_near); free(tmp);
    free(R); free(F); free(sR); free(sF); free(sL);
}

/* The cave posterior as a target: log posterior and its gradient in the free surfaces. */
typedef struct { const orc_problem *p; double *gfull; } cave_ctx;

static double cave_target(const void *vctx, const double *x, double *grad) {
    const cave_ctx *c = (const cave_ctx *)vctx;
    const size_t M = (size_t)(c->p->S - 1) * c->p->R * c->p->C;
    double lp = orc_grad(c->p, x, c->gfull);
    memcpy(grad, c->gfull, sizeof(double) * M);
    return lp;
}

double orc_latent_logpost_grad(const orc_problem *p, const double *x, double *gx);

/* The cave posterior in the latent parametrisation. */
static double latent_target(const void *vctx, const double *x, double *grad) {
    const cave_ctx *c = (const cave_ctx *)vctx;
    return orc_latent_logpost_grad(c->p, x, grad);
}

double orc_latent_r_logpost_grad(const orc_problem *p, const double *z, double *gz);

static double latent_r_target(const void *vctx, const double *z, double *grad) {
    const cave_ctx *c = (const cave_ctx *)vctx;
    return orc_latent_r_logpost_grad(c->p, z, grad);
}

/* A Gaussian test target N(0, diag(sd^2)) in M dimensions (for pins). */
typedef struct { size_t M; const double *sd; } gauss_ctx;

static double gauss_target(const void *vctx, const double *x, double *grad) {
    const gauss_ctx *c = (const gauss_ctx *)vctx;
    double lp = 0.0;
    for (size_t i = 0; i < c->M; ++i) {
        double s2 = c->sd[i] * c->sd[i];
        lp -= 0.5 * x[i] * x[i] / s2;
        grad[i] = -x[i] / s2;
    }
    return lp;
}

/* A Gaussian test target N(0, P^-1) with a dense precision matrix P
   (M x M, row-major): lp = -x.P x / 2, grad = -P x (for pins). */
typedef struct { size_t M; const double *prec; } gauss_dense_ctx;

static double gauss_dense_target(const void *vctx, const double *x, double *grad) {
    const gauss_dense_ctx *c = (const gauss_dense_ctx *)vctx;
    double lp = 0.0;
    for (size_t i = 0; i < c->M; ++i) {
        double px = 0.0;
        for (size_t j = 0; j < c->M; ++j) px += c->prec[i * c->M + j] * x[j];
        grad[i] = -px;
        lp -= 0.5 * x[i] * px;
    }
    return lp;
}

/* n_steps NUTS transitions at a fixed step size eps on the dense Gaussian
   target, for every chain c (Philox chain index c); inv_mass [M] shared by
   the chains or NULL.  Per-transition outputs [n_chains][n_steps]. */
void orc_nuts_dense(size_t M, const double *prec, int n_chains, double *x_all, double eps, const double *inv_mass,
                    int max_depth, double max_dh, int64_t n_steps, uint64_t seed, uint64_t step_offset,
                    int32_t *depth_out, int32_t *n_leap_out, int32_t *div_out, int32_t *turned_out,
                    double *acc_out, double *margin_out) {
    if (max_depth > ORC_NUTS_MAX_DEPTH) max_depth = ORC_NUTS_MAX_DEPTH;
    gauss_dense_ctx gc = {M, prec};
#pragma omp parallel for schedule(dynamic, 64)
    for (int c = 0; c < n_chains; ++c) {
        double *x = x_all + M * c;
        double *g = malloc(sizeof(double) * M);
        double lp = gauss_dense_target(&gc, x, g);
        double margin = INFINITY;
        for (int64_t k = 0; k < n_steps; ++k) {
            orc_nuts_stats st;
            nuts_transition(gauss_dense_target, &gc, M, x, &lp, g, eps, inv_mass, max_depth, max_dh, seed,
                            (uint32_t)c, step_offset + (uint64_t)k, 0, &st);
            const size_t o = (size_t)c * n_steps + k;
            if (depth_out) depth_out[o] = st.depth;
            if (n_leap_out) n_leap_out[o] = st.n_leap;
            if (div_out) div_out[o] = st.diverged;
            if (turned_out) turned_out[o] = st.turned;
            if (acc_out) acc_out[o] = st.accept_stat;
            if (st.margin < margin) margin = st.margin;
        }
        if (margin_out) margin_out[c] = margin;
        free(g);
    }
}

/* Dual averaging of log(step size) (Hoffman & Gelman 2014, Sec. 3.2), per chain. */
typedef struct { double log_eps, log_eps_bar, h_bar, mu; int64_t t; } orc_dual_avg;

static void da_restart(orc_dual_avg *d, double eps) {
    d->mu = log(10.0 * eps);
    d->log_eps = log(eps);
    d->log_eps_bar = 0.0;
    d->h_bar = 0.0;
    d->t = 0;
}

static void da_update(orc_dual_avg *d, double accept_stat, double target) {
    const double gamma = 0.05, t0 = 10.0, kappa = 0.75;
    d->t += 1;
    const double t = (double)d->t;
    d->h_bar = (1.0 - 1.0 / (t + t0)) * d->h_bar + (target - accept_stat) / (t + t0);
    d->log_eps = d->mu - sqrt(t) / gamma * d->h_bar;
    const double eta = pow(t, -kappa);
    d->log_eps_bar = eta * d->log_eps + (1.0 - eta) * d->log_eps_bar;
}

/* Warm-up windows: an initial buffer (step size only), slow windows that
   double in length and each end with a mass-matrix update, and a terminal
   buffer (step size only).  Defaults 75 / 25 / 50; when they do not fit,
   15 % / 75 % / 10 % of the warm-up.  Returns 1 if the window containing
   iteration k (0-based) ends at k and is a slow window. */
static void warmup_layout(int64_t n_warmup, int64_t *init_buf, int64_t *base_win, int64_t *term_buf) {
    *init_buf = 75; *base_win = 25; *term_buf = 50;
    if (n_warmup < 20) { *init_buf = n_warmup; *base_win = 0; *term_buf = 0; return; }
    if (*init_buf + *base_win + *term_buf > n_warmup) {
        *init_buf = (int64_t)(0.15 * n_warmup);
        *term_buf = (int64_t)(0.1 * n_warmup);
        *base_win = n_warmup - *init_buf - *term_buf;
    }
}

int orc_warmup_window_end(int64_t n_warmup, int64_t k) {
    int64_t ib, bw, tb;
    warmup_layout(n_warmup, &ib, &bw, &tb);
    if (bw == 0) return 0;
    const int64_t slow_end = n_warmup - tb;
    int64_t start = ib, len = bw;
    while (start < slow_end) {
        int64_t end = start + len;
        /* a window that would leave less than twice its length before the terminal buffer absorbs it */
        if (end + 2 * len > slow_end) end = slow_end;
        if (k == end - 1) return 1;
        start = end;
        len *= 2;
    }
    return 0;
}

int orc_warmup_in_slow(int64_t n_warmup, int64_t k) {
    int64_t ib, bw, tb;
    warmup_layout(n_warmup, &ib, &bw, &tb);
    return bw > 0 && k >= ib && k < n_warmup - tb;
}

/*
 * NUTS on the cave posterior (or, with gauss_sd non-NULL, on N(0, diag(sd^2))
 * in M = n_dim dimensions), chains in parallel; with latent != 0 the states
 * are the latent CAR fields x and the target is their log density.  Chain c: state x[c] (M),
 * lp[c] (NaN: computed first), step size eps[c] (in/out), inverse mass
 * inv_mass[c] ([n][M], in/out; NULL = identity, not adapted).
 * n_warmup > 0 runs that many adapting transitions first (dual averaging to
 * target_accept; with inv_mass, windowed variance estimates: each slow window
 * ends with inv_mass = (n/(n+5)) var + 1e-3 * 5/(n+5) of its draws, and every
 * window end restarts dual averaging from the current step size); then
 * n_steps transitions at the adapted eps = exp(log_eps_bar).  Step k of the
 * whole run uses Philox step step_offset + k.  Outputs (optional):
 * depth/n_leap/diverged [n][n_warmup + n_steps], accept_stat likewise,
 * margin [n] = smallest decision margin seen.
 */
void orc_nuts(const orc_problem *p, size_t n_dim, const double *gauss_sd, int latent, int n_chains, double *x_all,
              double *lp, double *eps, double *inv_mass, int max_depth, double max_dh, int64_t n_warmup,
              int64_t n_steps, double target_accept, uint64_t seed, uint64_t step_offset, int state_f32,
              int32_t *depth_out, int32_t *n_leap_out, int32_t *div_out, double *acc_out, double *margin_out) {
    /* latent: 0 = heights, 1 = the CAR fields x, 2 = x and logit r (one r per free surface) */
    const size_t M = gauss_sd ? n_dim : (size_t)(p->S - 1) * p->R * p->C + (latent == 2 ? p->S - 1 : 0);
    const size_t NS = gauss_sd ? n_dim : (size_t)p->S * p->R * p->C;
    if (max_depth > ORC_NUTS_MAX_DEPTH) max_depth = ORC_NUTS_MAX_DEPTH;
    const int64_t total = n_warmup + n_steps;
#pragma omp parallel for schedule(dynamic, 1)
    for (int c = 0; c < n_chains; ++c) {
        double *x = x_all + M * c;
        double *im = inv_mass ? inv_mass + M * c : NULL;
        double *g = malloc(sizeof(double) * M);
        double *gfull = malloc(sizeof(double) * NS);
        double *wm = malloc(sizeof(double) * M), *w2 = malloc(sizeof(double) * M);   /* Welford */
        int64_t wn = 0;
        cave_ctx cc = {p, gfull};
        gauss_ctx gc = {M, gauss_sd};
        orc_target_fn tf = gauss_sd ? gauss_target
                                    : (latent == 2 ? latent_r_target : (latent ? latent_target : cave_target));
        const void *ctx = gauss_sd ? (const void *)&gc : (const void *)&cc;
        double l = tf(ctx, x, g);
        if (isnan(lp[c])) lp[c] = l;
        orc_dual_avg da;
        da_restart(&da, eps[c]);
        double margin = INFINITY;
        for (int64_t k = 0; k < total; ++k) {
            const int warm = k < n_warmup;
            const double e = warm ? exp(da.log_eps) : eps[c];
            orc_nuts_stats st;
            nuts_transition(tf, ctx, M, x, &lp[c], g, e, im, max_depth, max_dh, seed, (uint32_t)c,
                            step_offset + (uint64_t)k, state_f32, &st);
            if (st.margin < margin) margin = st.margin;
            const size_t o = (size_t)c * total + k;
            if (depth_out) depth_out[o] = st.depth;
            if (n_leap_out) n_leap_out[o] = st.n_leap;
            if (div_out) div_out[o] = st.diverged;
            if (acc_out) acc_out[o] = st.accept_stat;
            if (!warm) continue;
            da_update(&da, st.accept_stat, target_accept);
            if (im && orc_warmup_in_slow(n_warmup, k)) {
                ++wn;
                for (size_t i = 0; i < M; ++i) {
                    if (wn == 1) { wm[i] = x[i]; w2[i] = 0.0; continue; }
                    const double d = x[i] - wm[i];
                    wm[i] += d / wn;
                    w2[i] += d * (x[i] - wm[i]);
                }
                if (orc_warmup_window_end(n_warmup, k)) {
                    const double n = (double)wn;
                    for (size_t i = 0; i < M; ++i) {
                        const double var = wn > 1 ? w2[i] / (n - 1.0) : 0.0;
                        im[i] = (n / (n + 5.0)) * var + 1e-3 * (5.0 / (n + 5.0));
                    }
                    wn = 0;
                    da_restart(&da, exp(da.log_eps));
                }
            }
            if (k == n_warmup - 1) eps[c] = exp(da.log_eps_bar);
        }
        if (margin_out) margin_out[c] = margin;
        free(g); free(gfull); free(wm); free(w2);
    }
}

/*
 * Nested R-hat (the paper's convergence diagnostic, Sec. 3.2) from one draw
 * per chain: chains c = k*n_within + m form n_super super-chains of n_within.
 * Per coordinate i: super-chain means xk, overall mean x, between-super-chain
 * variance B = sum_k (xk - x)^2 / (K - 1), within W = mean_k of the variance
 * of the chains of super-chain k about xk (divisor n_within - 1; the
 * within-chain variance of a single draw is zero); nR = sqrt(1 + B / W).
 * x_all: [n_super*n_within][n_dim]; out: [n_dim].
 */
void orc_nested_rhat(int n_super, int n_within, size_t n_dim, const double *x_all, double *out) {
    for (size_t i = 0; i < n_dim; ++i) {
        double xbar = 0.0, B = 0.0, W = 0.0;
        double *xk = malloc(sizeof(double) * n_super);
        for (int k = 0; k < n_super; ++k) {
            double s = 0.0;
            for (int m = 0; m < n_within; ++m) s += x_all[(size_t)(k * n_within + m) * n_dim + i];
            xk[k] = s / n_within;
            xbar += xk[k];
        }
        xbar /= n_super;
        for (int k = 0; k < n_super; ++k) {
            B += (xk[k] - xbar) * (xk[k] - xbar);
            double v = 0.0;
            for (int m = 0; m < n_within; ++m) {
                double d = x_all[(size_t)(k * n_within + m) * n_dim + i] - xk[k];
                v += d * d;
            }
            W += v / (n_within - 1);
        }
        B /= (n_super - 1);
        W /= n_super;
        out[i] = sqrt(1.0 + B / W);
        free(xk);
    }
}

/* ------------------------------------------------------------------------- */
/* The latent parametrisation the paper's sampler runs on (Sec. 2.2.1, 3.1)   */
/* ------------------------------------------------------------------------- */
/*
 * The unknowns of the model are the CAR fields x_l ~ N(0, Q_l^-1) of the free
 * surfaces; the heights are their image under the copula map,
 *   w = x / sqrt(Sigma11_l),  u = Phi(w),  H_l = (1 - u) H_{l-1} + u H_top
 * (H_0 = 0).  The sampler's latent vector is x.  Its log density is
 *   log L(H(x)) + sum_l [ log det(Q_l)/2 - x_l' Q_l x_l / 2 - (N/2) log 2 pi ],
 * the same normalisation as the density in H (which is this one divided by
 * |det dH/dx|).  For accuracy H is formed from the lower tail u when w <= 0
 * and from the upper tail 1 - u = Phi(-w) otherwise.
 */
void orc_latent_to_heights(const orc_problem *p, const double *x, double *H) {
    const int N = p->R * p->C;
    for (int l = 0; l < p->S - 1; ++l) {
        double logdet, s11;
        orc_car_consts(p->R, p->C, p->car_r[l], &logdet, &s11);
        const double s = sqrt(s11);
        for (int i = 0; i < N; ++i) {
            const double a = l ? H[(size_t)(l - 1) * N + i] : 0.0, b = p->top[i];
            const double w = x[(size_t)l * N + i] / s;
            H[(size_t)l * N + i] = w <= 0.0 ? a + Phi(w) * (b - a) : b - Phi(-w) * (b - a);
        }
    }
}

void orc_heights_to_latent(const orc_problem *p, const double *H, double *x) {
    const int N = p->R * p->C;
    for (int l = 0; l < p->S - 1; ++l) {
        double logdet, s11;
        orc_car_consts(p->R, p->C, p->car_r[l], &logdet, &s11);
        const double s = sqrt(s11);
        for (int i = 0; i < N; ++i) {
            const double a = l ? H[(size_t)(l - 1) * N + i] : 0.0, b = p->top[i];
            const double h = H[(size_t)l * N + i];
            x[(size_t)l * N + i] = s * ndtri_uv((h - a) / (b - a), (b - h) / (b - a));
        }
    }
}

/* Log density of the latent vector and (optional) its gradient [S-1][R][C].
   Chain rule at each node, top layer first: with a_l = H_{l-1},
   dH_l/dx_l = (H_top - a_l) phi(w_l) / sqrt(Sigma11_l) and dH_l/da_l = 1 - u_l,
   D_l = dlogL/dH_l + (1 - u_{l+1}) D_{l+1} and dlogL/dx_l = D_l dH_l/dx_l. */
/* d/dr of log det Q(r) and of Sigma11(r) on the R x C torus, from the
   eigenvalues mu_km = 4 - 2 r c_km, c_km = cos(2 pi k / R) + cos(2 pi m / C):
   d log det Q / dr = sum -2 c_km / mu_km, d Sigma11 / dr = sum 2 c_km / mu_km^2 / N. */
static void car_consts_dr(int R, int C, double r, double *dlogdet, double *ds11) {
    double a = 0.0, b = 0.0;
    for (int k = 0; k < R; ++k)
        for (int m = 0; m < C; ++m) {
            const double c = cos(2.0 * M_PI * k / R) + cos(2.0 * M_PI * m / C);
            const double mu = 4.0 - 2.0 * r * c;
            a += -2.0 * c / mu;
            b += 2.0 * c / (mu * mu);
        }
    *dlogdet = a;
    *ds11 = b / ((double)R * C);
}

/*
 * The sampler's latent vector with the hierarchical dependence (Sec. 2.2.1:
 * r_l ~ Uniform(0, 1) a priori; Sec. 3.1: the sampler runs on a vector of
 * all unknowns): z = (x_1 .. x_{S-1}, eta_1 .. eta_{S-1}), eta = logit r, so
 * z has no boundaries.  Its log density is
 *   log L(H(x, r)) + sum_l [ log det Q(r_l)/2 - x_l' Q(r_l) x_l / 2
 *                            - (N/2) log 2 pi + log(r_l (1 - r_l)) ],
 * the last term the Jacobian dr/deta of the flat prior; H(x, r) is the copula
 * map with s_l = sqrt(Sigma11(r_l)).  Gradient in eta_l: r (1 - r) times
 *   dlogL/dr_l + (d log det Q / dr)/2 + x_l' A x_l / 2   (Q = 4 I - r A),
 * plus 1 - 2 r; dlogL/dr_l = sum_i D_l,i (b_i - a_l,i) phi(w) dw/dr with
 * w = x / s, dw/dr = -w (dSigma11/dr) / (2 s^2) and D the total derivative
 * of log L in H_l (through the layers above).  gz (optional) has the layout
 * of z.
 */
double orc_latent_r_logpost_grad(const orc_problem *p, const double *z, double *gz) {
    const int S1 = p->S - 1, R = p->R, C = p->C, N = R * C;
    const double *x = z, *eta = z + (size_t)S1 * N;
    const size_t NS = (size_t)p->S * N;
    double r[16], sl[16], ld[16], dld[16], ds11[16];
    for (int l = 0; l < S1; ++l) {
        r[l] = 1.0 / (1.0 + exp(-eta[l]));
        double s11;
        orc_car_consts(R, C, r[l], &ld[l], &s11);
        sl[l] = sqrt(s11);
        car_consts_dr(R, C, r[l], &dld[l], &ds11[l]);
    }
    double *H = calloc((size_t)S1 * N, sizeof(double)), *gH = calloc(NS, sizeof(double));
    for (int l = 0; l < S1; ++l)
        for (int i = 0; i < N; ++i) {
            const double a = l ? H[(size_t)(l - 1) * N + i] : 0.0, b = p->top[i];
            const double w = x[(size_t)l * N + i] / sl[l];
            H[(size_t)l * N + i] = w <= 0.0 ? a + Phi(w) * (b - a) : b - Phi(-w) * (b - a);
        }
    double lp = loglik_grad_add_any(p, H, gH);
    double dr[16];
    for (int l = 0; l < S1; ++l) dr[l] = 0.0;
    for (int i = 0; i < N; ++i) {
        double D = 0.0;
        for (int l = S1 - 1; l >= 0; --l) {
            const double a = l ? H[(size_t)(l - 1) * N + i] : 0.0, b = p->top[i];
            const double w = x[(size_t)l * N + i] / sl[l];
            D = gH[(size_t)l * N + i] + (l < S1 - 1 ? Phi(-x[(size_t)(l + 1) * N + i] / sl[l + 1]) * D : 0.0);
            const double phi = exp(-0.5 * w * w) / sqrt(2.0 * M_PI);
            if (gz) gz[(size_t)l * N + i] = D * (b - a) * phi / sl[l];
            dr[l] += D * (b - a) * phi * (-w * ds11[l] / (2.0 * sl[l] * sl[l]));
        }
    }
    for (int l = 0; l < S1; ++l) {
        const double *xl = x + (size_t)l * N;
        double quad = 0.0, xax = 0.0;
        for (int i = 0; i < R; ++i)
            for (int j = 0; j < C; ++j) {
                const int n = i * C + j;
                const double nb = xl[i * C + (j + 1) % C] + xl[i * C + (j + C - 1) % C] +
                                  xl[((i + 1) % R) * C + j] + xl[((i + R - 1) % R) * C + j];
                const double qx = 4.0 * xl[n] - r[l] * nb;
                quad += xl[n] * qx;
                xax += xl[n] * nb;
                if (gz) gz[(size_t)l * N + n] -= qx;
            }
        const int jac = !(g_nuts_fault & 4);   /* planted mistake (tests): drop the Jacobian */
        lp += 0.5 * ld[l] - 0.5 * quad - 0.5 * N * log(2.0 * M_PI) + (jac ? log(r[l] * (1.0 - r[l])) : 0.0);
        if (gz)
            gz[(size_t)S1 * N + l] =
                r[l] * (1.0 - r[l]) * (dr[l] + 0.5 * dld[l] + 0.5 * xax) + (jac ? 1.0 - 2.0 * r[l] : 0.0);
    }
    free(H); free(gH);
    return lp;
}

double orc_latent_logpost_grad(const orc_problem *p, const double *x, double *gx) {
    const int S1 = p->S - 1, N = p->R * p->C, R = p->R, C = p->C;
    const size_t M = (size_t)S1 * N, NS = (size_t)p->S * N;
    double *H = malloc(sizeof(double) * M), *gH = calloc(NS, sizeof(double));
    double sl[16], ld[16];
    for (int l = 0; l < S1; ++l) {
        double s11;
        orc_car_consts(R, C, p->car_r[l], &ld[l], &s11);
        sl[l] = sqrt(s11);
    }
    orc_latent_to_heights(p, x, H);
    double lp = loglik_grad_add_any(p, H, gH);
    if (gx) {
        for (int i = 0; i < N; ++i) {
            double D = 0.0;
            for (int l = S1 - 1; l >= 0; --l) {
                const double a = l ? H[(size_t)(l - 1) * N + i] : 0.0, b = p->top[i];
                const double w = x[(size_t)l * N + i] / sl[l];
                D = gH[(size_t)l * N + i] + (l < S1 - 1 ? Phi(-x[(size_t)(l + 1) * N + i] / sl[l + 1]) * D : 0.0);
                const double phi = exp(-0.5 * w * w) / sqrt(2.0 * M_PI);
                gx[(size_t)l * N + i] = D * (b - a) * phi / sl[l];
            }
        }
    }
    /* the prior: x_l ~ N(0, Q_l^-1), Q = 4 I - r A on the periodic grid */
    for (int l = 0; l < S1; ++l) {
        const double r = p->car_r[l];
        const double *xl = x + (size_t)l * N;
        double quad = 0.0;
        for (int i = 0; i < R; ++i)
            for (int j = 0; j < C; ++j) {
                const int n = i * C + j;
                const double nb = xl[i * C + (j + 1) % C] + xl[i * C + (j + C - 1) % C] +
                                  xl[((i + 1) % R) * C + j] + xl[((i + R - 1) % R) * C + j];
                const double qx = 4.0 * xl[n] - r * nb;
                quad += xl[n] * qx;
                if (gx) gx[(size_t)l * N + n] -= qx;
            }
        lp += 0.5 * ld[l] - 0.5 * quad - 0.5 * N * log(2.0 * M_PI);
    }
    free(H); free(gH);
    return lp;
}

/* ------------------------------------------------------------------------- */
/* Solid-angle pixels (eq. expected_counts)                                   */
/* ------------------------------------------------------------------------- */
/*
 * The expected count of pixel p is the exposure-weighted integral of the
 * muon intensity over the pixel's solid angle.  Here the integral is a
 * quadrature over n_sub sub-rays whose weights hold Delta t, the solid angle
 * of each sub-cell and the detector efficiency in its direction, and the
 * intensity is a function of the opacity given as a table of log I at
 * uniform nodes O_j = j * tab_omax / (n_tab - 1), interpolated linearly in
 * log I (beyond the last node, the last segment continued).
 */
double orc_log_intensity(const orc_problem *p, double O) {
    const double dO = p->tab_omax / (p->n_tab - 1);
    double t = O / dO;
    int j = (int)floor(t);
    if (j < 0) j = 0;
    if (j > p->n_tab - 2) j = p->n_tab - 2;
    const double f = t - j;
    return p->tab_logI[j] + f * (p->tab_logI[j + 1] - p->tab_logI[j]);
}

/* Poisson log-likelihood of the per-pixel counts; lam (optional) receives
   lambda_p of every pixel.  O: opacities of the sub-rays. */
/* d log I / dO on the segment of the table that orc_log_intensity uses. */
static double log_intensity_slope(const orc_problem *p, double O) {
    const double dO = p->tab_omax / (p->n_tab - 1);
    int j = (int)floor(O / dO);
    if (j < 0) j = 0;
    if (j > p->n_tab - 2) j = p->n_tab - 2;
    return (p->tab_logI[j + 1] - p->tab_logI[j]) / dO;
}

/* Gradient of the solid-angle pixel likelihood (eq. expected_counts as a
   quadrature): lambda_p = sum_q w_q I(O_q), so sub-ray q of pixel p carries
   dLL/dO_q = (C_p / lambda_p - 1) w_q I(O_q) dlogI/dO(O_q), and its crossings
   scatter that through the crossing form as a single ray does.  grad
   [S][R][C] is added to; returns LL. */
static double quad_loglik_grad_add(const orc_problem *p, const double *free_h, double *grad) {
    const int nr = p->n_s * p->n_pix, npx = nr / p->n_sub;
    if (nr == 0) return 0.0;
    double *surf = stack_surfaces(p, free_h);
    double *O = (double *)malloc(sizeof(double) * nr), *lam = (double *)malloc(sizeof(double) * npx);
    const double ztop = top_max(p);
    double L[16];
    for (int ray = 0; ray < nr; ++ray) {
        const int s = ray / p->n_pix;
        O[ray] = march_ray(p, surf, p->pos + 3 * s, p->dirs + 3 * (size_t)ray, ztop, L, NULL, 0.0, NULL);
    }
    const double ll = orc_quad_loglik(p, O, lam);
    for (int ray = 0; ray < nr; ++ray) {
        const int s = ray / p->n_pix, px = ray / p->n_sub;
        const double c = (double)p->counts[px];
        const double g = (c / lam[px] - 1.0) * p->sub_w[ray] * exp(orc_log_intensity(p, O[ray])) *
                         log_intensity_slope(p, O[ray]);
        march_ray(p, surf, p->pos + 3 * s, p->dirs + 3 * (size_t)ray, ztop, L, grad, g, NULL);
    }
    free(surf);
    free(O);
    free(lam);
    return ll;
}

double orc_quad_loglik(const orc_problem *p, const double *O, double *lam) {
    const int nr = p->n_s * p->n_pix, npx = nr / p->n_sub;
    double ll = 0.0;
    for (int px = 0; px < npx; ++px) {
        double l = 0.0;
        for (int q = 0; q < p->n_sub; ++q) {
            const int r = px * p->n_sub + q;
            l += p->sub_w[r] * exp(orc_log_intensity(p, O[r]));
        }
        if (lam) lam[px] = l;
        const double c = (double)p->counts[px];
        ll += c * log(l) - l - lgamma(c + 1.0);
    }
    return ll;
}
