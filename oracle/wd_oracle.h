/*
 * wd_oracle.h -- plain FP64 CPU oracle for PDE-based wall distance
 * (Kakumani, Vadlamani & Tucker, "On the use of high order central
 * difference schemes for differential equation based wall distance
 * computations", arXiv 2111.09859).
 *
 * TEST INFRASTRUCTURE.  This library exists only to check the GPU path.
 * Only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark may load it.  It shares no code, header, table or constant
 * generator with the GPU library, and it never includes anything from it.
 *
 * Conventions (all arrays are dense, x index fastest):
 *   point (i0,i1,i2) -> q = i0 + n0*(i1 + n1*i2); n2 = 1 in 2D.
 *   metrics: ndim*ndim SoA components, component (l*ndim+m) holds
 *            d xi_l / d x_m  (Sec. 3.1, transformed equations).
 *   coords:  ndim SoA components x_m.
 */
#ifndef WD_ORACLE_H
#define WD_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

enum { WDO_WALL = 0, WDO_NEUMANN = 1, WDO_OUTFLOW = 2, WDO_PERIODIC = 3 };
enum { WDO_EIKONAL = 0, WDO_HJ = 1, WDO_POISSON = 2 };
enum { WDO_GAMMA_LINEAR = 0, WDO_GAMMA_LAD = 1 };
enum { WDO_E2 = 0, WDO_E4 = 1, WDO_E6 = 2, WDO_C4 = 3, WDO_C6 = 4, WDO_UW = 5 };
enum { WDO_RK3 = 0, WDO_RK4 = 1 };

typedef struct {
    int ndim;
    int n[3];
    int bc[3][2];              /* per direction, low / high face        */
    int uniform;               /* 1: Cartesian spacing h[]; 0: coords    */
    double h[3];
    const double *coords;      /* ndim SoA components (uniform == 0)     */
    double period[3][3];       /* x_m(i_l + n_l) = x_m(i_l) + period[l][m] */
    const unsigned char *mask; /* optional, 1 = solid point              */
    int metric_form;           /* 0: inverse of the coordinate Jacobian;
                                  1: conservative form (3D; see
                                  wdo_metrics)                          */
} wdo_grid;

typedef struct {
    int equation;              /* WDO_EIKONAL / WDO_HJ / WDO_POISSON      */
    int gamma;                 /* WDO_GAMMA_LINEAR / WDO_GAMMA_LAD        */
    int curvature;             /* 1: Nakanishi-type curvature correction  */
    double eps;                /* Gamma = eps*phi                         */
    double C;                  /* LAD constant                            */
    double nu0;                /* curvature stabiliser coefficient        */
    double eps0;               /* regulariser of the unit normal          */
    int scheme;                /* WDO_E2 .. WDO_C6, or WDO_UW: the paper's
                                  first-order upwind baseline (Sec. 3.2.1,
                                  Eqs. UW1-UW5) with 2nd-order central
                                  Laplacian and metrics                   */
    int filter;                /* 1: implicit filter after each step      */
    double alpha_f;
    int rk;                    /* WDO_RK3 (SSP) / WDO_RK4                 */
    double sigma;              /* local time step safety factor           */
    double tol;                /* stop when max |phi - phi_o| <= tol      */
    int max_iter;
    int fixed_iters;           /* > 0: run exactly this many iterations   */
    int lad_raw;               /* LAD reading: 0 (default) = sensor C|S|
                                  from phi^n once per iteration, smoothed by
                                  the truncated Gaussian filter along each
                                  direction; 1 = unsmoothed, recomputed from
                                  each stage value (kept to document its
                                  instability)                           */
    int uw_printed;            /* UW switch weights: 0 (default) = n_{i-1}
                                  weighs the backward difference B and
                                  n_{i+1} the forward one F; 1 = the
                                  pairing as printed (n_{i-1} with F)      */
} wdo_method;

/* 1-D operators in index space (unit spacing).  jump: f(i+n) = f(i)+jump
 * for periodic lines (coordinate seams).  Return 0 on success. */
int wdo_deriv_line(int n, int periodic, int scheme, double jump,
                   const double *f, double *df);
int wdo_filter_line(int n, int periodic, double alpha_f,
                    const double *f, double *out);

/* Metric terms by the solve's own scheme (d xi_l / d x_m). */
int wdo_metrics(const wdo_grid *g, int scheme, double *met);

/* One evaluation of the pseudo-time right-hand side at phi.  Any output
 * pointer may be NULL.  dt is the local pseudo time step at phi. */
int wdo_eval(const wdo_grid *g, const wdo_method *m, const double *met,
             const double *phi, const double *lad_in, double *R, double *gmag,
             double *gam, double *lap, double *kap, double *dt);

/* LAD diffusivity field of Eq. (Gamma_form2)'s second argument at phi
 * (smoothed unless m->lad_raw). */
int wdo_lad_field(const wdo_grid *g, const wdo_method *m, const double *met,
                  const double *phi, double *out);

/* The nine-point smoothing of the LAD diffusivity applied to one line
 * (ends clamped unless periodic); n >= 9. */
int wdo_gauss_line(int n, int periodic, const double *f, double *out);

/* Threads shared among the grid-wide loops (n <= 0: keep the current
 * count); returns the count now in force.  Results do not depend on it. */
int wdo_set_threads(int n);

/* Boundary conditions and solid mask, in place. */
void wdo_apply_bc(const wdo_grid *g, double *phi);

/* Pseudo-time march.  warm: 0 -> phi starts at zero.  hist receives
 * (Linf, L2) of the pseudo-step change per iteration.  Returns 0 when
 * converged (or fixed_iters done), 1 when max_iter was exhausted, -3 on a
 * non-finite residual, -1 on bad arguments. */
int wdo_solve(const wdo_grid *g, const wdo_method *m, double *phi, int warm,
              double *hist, int hist_cap, int *iters);

/* Poisson auxiliary variable -> distance. */
int wdo_poisson_distance(const wdo_grid *g, int scheme, const double *met,
                         const double *phip, double *d);

/* Brute-force nearest distance from npts points to nwall wall samples. */
/* Level-set burnback (Sec. 5.5, Eq. levelset with its right-hand side
 * read as 0): phi_s is the signed distance, positive on the solid
 * (propellant) side, negative in the gas; uniform grids only.
 *   wdo_signed_distance: phi_s = d_solid where solid[q], else -d_gas.
 *   wdo_levelset_advance: nsteps classical RK4 steps of
 *     d phi_s / dt = -F |grad phi_s| (upwind switch of Eqs. UW3-UW5),
 *     zero-gradient faces after every stage.
 *   wdo_level_length: 2D length of the iso-line phi_s = level (linear
 *     interpolation on cell edges, saddles split by the cell mean).    */
void wdo_signed_distance(long n, const unsigned char *solid, const double *d_solid,
                         const double *d_gas, double *phi_s);
int wdo_levelset_advance(const wdo_grid *g, double speed, double dt, int nsteps,
                         double *phi);
double wdo_level_length(const wdo_grid *g, const double *phi, double level);

void wdo_brute_force(int ndim, int npts, const double *pts, int nwall,
                     const double *wall, double *d);

#ifdef __cplusplus
}
#endif
#endif
