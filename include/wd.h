/*
 * wd.h -- C ABI of the MI355X (gfx950) wall-distance library.
 *
 * The library drives the wall-distance PDEs of Kakumani, Vadlamani &
 * Tucker (arXiv 2111.09859) -- Eikonal (Eq. ek_eq), Hamilton-Jacobi
 * (Eq. Ham_Jac, with Gamma from Eq. Gamma_form1 or the LAD form of
 * Eq. Gamma_form2, optionally with the curvature correction of Sec. 5.4)
 * and Poisson (Eqs. Poiss1/Poiss2) -- to steady state by pseudo-time
 * marching (Sec. 3.3) on structured 2D/3D grids written in generalised
 * coordinates (Sec. 3.1), with explicit or compact central differences
 * (Sec. 3.2) and the implicit filter of Sec. 3.4 after every pseudo step.
 *
 * Conventions for every call:
 *   - Fields are dense, x index (direction 0) fastest: point (i0,i1,i2) is
 *     element i0 + n0*(i1 + n1*i2); n2 = 1 for 2D grids.
 *   - Pointers documented as "device" are HIP device pointers on the
 *     context's device; "host" pointers are ordinary host memory.
 *   - The caller owns every buffer it passes (fields, metrics, masks,
 *     workspace, history); the library owns only its context caches and the
 *     server's internal arena, released by the matching destroy call.
 *   - Work is issued on the given stream (hipStream_t passed as void*; NULL
 *     means the default stream).  The solve calls return after the solve has
 *     finished on that stream.
 *   - Return value: WD_OK (0) or a positive warning (the outputs are valid)
 *     or a negative error; wd_last_error() describes the last failure of the
 *     calling thread.
 */
#ifndef WD_H
#define WD_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---------------------------------------------------- */
#define WD_OK 0
#define WD_NOT_CONVERGED 1     /* max_iter reached; field + history valid   */
#define WD_STAGNATED 2         /* residual stopped decreasing (stall_window) */
#define WD_PENDING 3           /* server request not finished yet           */
#define WD_ERR_INVALID_ARG (-1)
#define WD_ERR_UNSUPPORTED (-2)
#define WD_ERR_DIVERGED (-3)   /* non-finite pseudo-step change             */
#define WD_ERR_NO_MEMORY (-4)  /* workspace / budget too small              */
#define WD_ERR_HIP (-5)        /* HIP runtime error, text in wd_last_error  */
#define WD_ERR_CANCELLED (-6)
#define WD_ERR_NOT_FOUND (-7)
#define WD_ERR_WARM_RUNAWAY (-8) /* warm start abandoned by the runaway check
                                  (wd_method.warm_probe); phi holds the
                                  abandoned field: solve again cold        */

/* ---- enumerations ---------------------------------------------------- */
/* Face conditions (Sec. 3.5): WALL is the Dirichlet phi = 0 of Eq. eq7;
 * NEUMANN is the zero normal gradient of Eq. eq8, discretised as
 * phi_b = (4 phi_{b+1} - phi_{b+2})/3 along the grid line; OUTFLOW (an
 * option beside the paper's far field) extrapolates linearly,
 * phi_b = 2 phi_{b+1} - phi_{b+2}; both are re-imposed after every RK stage
 * and after the filter, face by face in direction order, skipping points on
 * wall faces or in solids.  PERIODIC wraps the index (n distinct points,
 * both faces of a direction). */
enum wd_bc { WD_BC_WALL = 0, WD_BC_NEUMANN = 1, WD_BC_OUTFLOW = 2,
             WD_BC_PERIODIC = 3 };
enum wd_metric_mode { WD_METRIC_UNIFORM = 0, WD_METRIC_FIELDS = 1 };
enum wd_equation { WD_EQ_EIKONAL = 0, WD_EQ_HJ = 1, WD_EQ_POISSON = 2 };
enum wd_gamma { WD_GAMMA_LINEAR = 0, WD_GAMMA_LAD = 1 };
/* Sec. 3.2 schemes; E6 is the sixth-order explicit member of the same
 * family (third term c (f_{i+3} - f_{i-3})/6). */
enum wd_scheme { WD_E2 = 0, WD_E4 = 1, WD_E6 = 2, WD_C4 = 3, WD_C6 = 4,
                 /* the paper's first-order upwind baseline (Sec. 3.2.1,
                  * Eqs. UW1-UW5): the advective term from switched
                  * one-sided differences, 2nd-order central (E2) Laplacian
                  * and metrics; no curvature correction (WD_ERR_UNSUPPORTED),
                  * usually run without the filter */
                 WD_UW = 5 };
enum wd_rk { WD_RK3_SSP = 0, WD_RK4 = 1 };
enum wd_precision { WD_FP32 = 0, WD_FP64 = 1 };

/* ---- grid descriptor (Sec. 3.1 generalised coordinates, Sec. 3.5) ----- */
typedef struct wd_grid_desc {
    int ndim;             /* 2 or 3                                         */
    int n[3];             /* points per direction (>= 8); n[2] = 1 in 2D    */
    int bc[3][2];         /* wd_bc per direction, [low face, high face];
                             PERIODIC must be set on both faces             */
    int metric_mode;      /* wd_metric_mode                                 */
    double h[3];          /* UNIFORM: grid spacing per direction            */
    const void *metrics;  /* FIELDS (2D or 3D): device array of ndim*ndim SoA
                             components in the solve precision; component
                             (l*ndim + m) holds d xi_l / d x_m               */
    const unsigned char *mask; /* optional device array, 1 = solid point
                                  (phi = 0 there); NULL = no solids         */
} wd_grid_desc;

/* ---- method descriptor ---------------------------------------------- */
typedef struct wd_method {
    int equation;         /* wd_equation                                    */
    int gamma;            /* wd_gamma (HJ only)                             */
    int curvature;        /* 1: curvature correction of Sec. 5.4 (HJ only)  */
    double eps;           /* Gamma = eps * phi (Eq. Gamma_form1), 0.1..1    */
    double c_lad;         /* C of Eq. Gamma_form2 (0.1)                     */
    double nu0;           /* nu = nu0 (1 - |grad phi|)^2 (0.001)            */
    double eps0;          /* n = grad phi / (|grad phi| + eps0) (1e-6)      */
    int scheme;           /* wd_scheme, used for metrics and derivatives    */
    int filter;           /* 1: implicit filter after every pseudo step     */
    double alpha_f;       /* filter coefficient, 0.48 .. 0.5 (0.5 = none)   */
    int rk;               /* wd_rk                                          */
    double sigma;         /* local pseudo-time step safety factor (1.0)     */
    double tol;           /* stop when max |phi - phi_o| <= tol (Eq.
                             Con-criter, L_ref = 1)                         */
    int max_iter;         /* iteration limit                                */
    int stall_window;     /* > 0: stop (WD_STAGNATED) when the max change,
                             already within 10 * tol, has not reached a new
                             minimum for this many iterations (the rounding
                             floor of FP32); plateaus while the front still
                             crosses the grid do not count; 0 disables      */
    int precision;        /* wd_precision of fields and arithmetic; the
                             convergence reductions are always FP64         */
    int warm_start;       /* 1: phi holds the initial guess (e.g. the
                             previous physical time step's field when walls
                             move, Sec. 5.5); wall and solid points are set
                             to zero first.  0: phi = 0                     */
    int warm_probe;       /* runaway check of a warm start: a guess that
                             jumps by much more than the spacing beside a
                             wall can make the central march undershoot
                             below zero there, where Gamma = max(0, eps phi)
                             vanishes and nothing damps it.  After this many
                             iterations the device compares the field's
                             minimum with its largest magnitude (FP64, after
                             the filter); below -0.1 of it the solve stops
                             with WD_ERR_WARM_RUNAWAY.  0 disables; ignored
                             for cold starts                                 */
} wd_method;

typedef struct wd_ctx wd_ctx;
typedef struct wd_server wd_server;

/* Version string, e.g. "wd 1.0 gfx950". */
const char *wd_version(void);

/* Text of the last failing call on this thread ("" if none). */
const char *wd_last_error(void);

/* Fill *m with the defaults: HJ, LAD, no curvature, eps 0.2, C 0.1,
 * nu0 1e-3, eps0 1e-6, C6, filter on, alpha_f 0.48, RK4, sigma 1,
 * tol 1e-10, max_iter 100000, stall_window 0, FP64, cold start,
 * warm_probe 300. */
int wd_method_default(wd_method *m);

/* Create a context on HIP device `device`: owns the line-operator tables
 * and the tile autotuning cache.  *out receives the context. */
int wd_ctx_create(int device, wd_ctx **out);
int wd_ctx_destroy(wd_ctx *ctx);

/* Metric terms (Sec. 3.1) of a curvilinear grid with the solve's own
 * derivative scheme (Sec. 3.2: metrics use the same central schemes).
 *   coords  : device, ndim SoA FP64 components x_m, grid layout.
 *   period  : host, period[l*3+m] = jump of x_m across the periodic seam of
 *             direction l (x_m(i_l + n_l) = x_m(i_l) + period); NULL = 0.
 *   out     : device, ndim*ndim SoA components in `out_precision`, the
 *             layout wd_grid_desc.metrics expects.
 * desc->metric_mode and desc->metrics are ignored. */
int wd_compute_metrics(wd_ctx *ctx, const wd_grid_desc *desc, int scheme,
                       const double *coords, const double *period, void *out,
                       int out_precision, void *stream);

/* Metric forms.  INVERSE: the per-point inverse of the coordinate
 * derivatives (wd_compute_metrics, the recipe of Sec. 3.1 with the solve's
 * scheme).  CONSERVATIVE (an option beside it, 3D): each J xi_{l,m} written
 * as a divergence of coordinate products, J xi_{l,m} = (D_q Q_{p,m} -
 * D_p Q_{q,m}) / 2 with Q_{p,m} = x_b D_p x_a - x_a D_p x_b ((l, p, q) and
 * (m, a, b) cyclic), then divided by the determinant of the coordinate
 * derivatives; derivatives along different directions commute, so the
 * discrete metric identities sum_l D_l (J xi_{l,m}) = 0 hold to rounding.
 * On affine grids, and in 2D, the two forms agree. */
enum wd_metric_form { WD_METRICS_INVERSE = 0, WD_METRICS_CONSERVATIVE = 1 };

/* wd_compute_metrics with the form chosen (wd_metric_form).  The
 * conservative form needs FP64 scratch of 36 doubles per point (the inverse
 * form 9) and returns WD_ERR_UNSUPPORTED for coordinates that jump across
 * a periodic seam (any non-zero period entry). */
int wd_compute_metrics_form(wd_ctx *ctx, const wd_grid_desc *desc, int scheme, int form,
                            const double *coords, const double *period, void *out,
                            int out_precision, void *stream);

/* Workspace bytes a wd_solve / wd_solve_batched of these grids needs.  The
 * caller allocates it on the device (any allocator) and passes it in. */
int wd_workspace_bytes(wd_ctx *ctx, int n_grids, const wd_grid_desc *descs,
                       const wd_method *methods, size_t *bytes);

/* Plain per-grid solve (Sec. 3.3-3.5 pseudo-time march to steady state).
 * A warm start that the runaway check stops returns WD_ERR_WARM_RUNAWAY
 * (the caller solves again cold; the server does that itself).
 *   phi      : device, grid layout, method precision.  Initial guess when
 *              warm_start is set (else overwritten with zero); on return the
 *              wall distance.  For WD_EQ_POISSON the converted distance of
 *              Eq. Poiss2; phi_aux (device, may be NULL) then receives the
 *              Poisson variable phi'.
 *   hist     : host, 2*hist_cap doubles: (max change, RMS change) of each
 *              pseudo iteration, FP64; may be NULL.
 *   iters    : host, iterations performed; may be NULL.
 *   ws       : device workspace of at least wd_workspace_bytes bytes.
 * Returns WD_OK on convergence, WD_NOT_CONVERGED, WD_STAGNATED or an
 * error (WD_ERR_DIVERGED leaves the last field in phi). */
int wd_solve(wd_ctx *ctx, const wd_grid_desc *desc, const wd_method *method,
             void *phi, void *phi_aux, double *hist, int hist_cap, int *iters,
             void *ws, size_t ws_bytes, void *stream);

/* wd_solve for callers that cannot allocate device memory (code that must
 * not call hipMalloc, such as tight serving loops or harnesses that forbid
 * it): the same solve with the workspace and the line-operator tables placed
 * in a library-owned static device array of 64 MiB on each GPU, held until
 * the process ends; no hipMalloc, hipFree or other allocating call and no
 * graph capture (kernels are launched directly).  Arguments as for wd_solve
 * without ws / ws_bytes.  A grid whose workspace (wd_workspace_bytes) plus
 * tables exceed 64 MiB is rejected with WD_ERR_NO_MEMORY (about 2.5 M
 * points in FP32 with RK4 and LAD, half that in FP64).  Every call on one
 * GPU uses that GPU's one array: calls that overlap on one GPU (two
 * contexts, two threads) race and corrupt each other; calls on one
 * context are serialised by the context.  Returns like wd_solve. */
int wd_solve_noalloc(wd_ctx *ctx, const wd_grid_desc *desc, const wd_method *method,
                     void *phi, void *phi_aux, double *hist, int hist_cap, int *iters,
                     void *stream);

/* Batched solve of n independent grids in one set of launches per RK
 * stage.  All grids share ndim, precision and rk; everything else (size,
 * scheme, equation, Gamma, metrics, faces, tolerances) may differ.  Each
 * grid's result is bitwise the one wd_solve gives for it alone.
 *   phis[i], aux[i] (aux may be NULL or hold NULLs): device, as in wd_solve.
 *   hists[i]: host or NULL; iters[i], status[i]: host arrays of n or NULL.
 * Returns the worst status over the grids (errors before warnings). */
int wd_solve_batched(wd_ctx *ctx, int n, const wd_grid_desc *descs,
                     const wd_method *methods, void *const *phis,
                     void *const *aux, double *const *hists, int hist_cap,
                     int *iters, int *status, void *ws, size_t ws_bytes,
                     void *stream);

/* Tile autotuning: for each grid direction, time `iters` pseudo iterations
 * of this grid and method with every candidate tile width (lines per
 * workgroup tile) and keep the fastest in the context's cache, keyed by the
 * grid shape, direction and precision; later plans of that shape use it.
 * Results do not depend on the tile widths (each point's arithmetic is the
 * same), only the speed does.  A grid that the segmented passes serve
 * (wd_ctx_set_segmented) has fixed tiles: nothing is timed, and widths
 * receives the lines per tile of those passes.
 *   phi   : device scratch field of the grid (overwritten).
 *   ws    : device workspace of at least wd_workspace_bytes.
 *   widths: host, receives the chosen width per direction (may be NULL). */
int wd_autotune(wd_ctx *ctx, const wd_grid_desc *desc, const wd_method *method,
                void *phi, void *ws, size_t ws_bytes, int iters, int *widths,
                void *stream);

/* The tile widths this context uses for grids of desc's shape at
 * `precision`: the cached choice (wd_autotune or wd_tune_set) or the
 * default.  widths: host, receives desc->ndim values.  No device work. */
int wd_tune_get(wd_ctx *ctx, const wd_grid_desc *desc, int precision, int *widths);

/* Store tile widths for grids of desc's shape at `precision` (for example
 * a saved autotuning result).  Direction 0 tiles hold widths[0] whole rows
 * (at most the number of rows); direction l >= 1 tiles hold widths[l]
 * consecutive x-columns (at most n[0]); every tile must fit 4096 points.
 * Returns WD_ERR_INVALID_ARG for a width outside these bounds (nothing is
 * stored then).  No device work. */
int wd_tune_set(wd_ctx *ctx, const wd_grid_desc *desc, int precision, const int *widths);

/* Eq. Poiss2 on its own: distance = -|grad phi'| + sqrt(|grad phi'|^2 +
 * 2 phi') with the gradient by `scheme` and the metrics, evaluated in FP64.
 *   phip, dist: device, grid layout, `precision` (FP32 or FP64).
 *   ws: device, >= wd_workspace_bytes of a Poisson solve of this grid. */
int wd_poisson_distance(wd_ctx *ctx, const wd_grid_desc *desc, int scheme,
                        int precision, const void *phip, void *dist, void *ws,
                        size_t ws_bytes, void *stream);

/* ---- level-set burnback (Sec. 5.5, Eq. levelset) ---------------------
 * A front (the burning surface of a propellant grain) moves along its
 * normal at speed F: d phi_s / dt + F |grad phi_s| = 0 (the printed right-
 * hand side "1" read as 0), phi_s the signed distance to the front,
 * positive on the solid side, so the front moves into the solid.  Uniform
 * grids (metric_mode WD_METRIC_UNIFORM; desc->mask and the face kinds are
 * not used: every non-periodic face gets a zero normal gradient). */

/* Device workspace for wd_levelset_advance and wd_level_lengths. */
int wd_levelset_workspace_bytes(wd_ctx *ctx, const wd_grid_desc *desc, int precision,
                                size_t *bytes);

/* phi_s = d_solid where solid[q] != 0, -d_gas elsewhere (n points; device
 * arrays in `precision`, solid as bytes; phi_s may alias either input). */
int wd_signed_distance(wd_ctx *ctx, long long n, int precision, const unsigned char *solid,
                       const void *d_solid, const void *d_gas, void *phi_s, void *stream);

/* nsteps classical RK4 steps of size dt of the equation above, in place on
 * phi_s (device, grid layout, `precision`): each one-sided difference by the
 * upwind switch of Eqs. UW3-UW5, divided by the grid spacing; after every
 * stage each non-periodic face takes f_b = (4 f_1 - f_2) / 3 along its grid
 * line, faces normal to direction 0 first.  With nsteps >= 4 one step is
 * captured in a HIP graph and replayed, and the call returns once the
 * steps have run; otherwise it is asynchronous on `stream`. */
int wd_levelset_advance(wd_ctx *ctx, const wd_grid_desc *desc, int precision, double speed,
                        double dt, int nsteps, void *phi_s, void *ws, size_t ws_bytes,
                        void *stream);

/* Lengths of the iso-lines phi_s = levels[k] (k < nlevels <= 8) of a 2D
 * uniform grid, in grid units of desc->h: in each cell the crossings of
 * the four edges by linear interpolation joined in pairs (a cell with four
 * crossings split by the sign of its mean value), summed in FP64.  The
 * grain's burning perimeter per unit depth (the surface S_b, Sec. 5.5) is
 * the length of the level 0.  lengths: host.  Waits for the stream. */
int wd_level_lengths(wd_ctx *ctx, const wd_grid_desc *desc, int precision, const void *phi_s,
                     const double *levels, int nlevels, double *lengths, void *ws,
                     size_t ws_bytes, void *stream);

/* ---- live kernel timing --------------------------------------------- */
typedef struct wd_kernel_stat {
    char name[32];        /* kernel family, e.g. "k_d2", "k_filter"        */
    long long launches;   /* launches timed                                */
    double total_ms;      /* sum of event-timed durations                  */
    double alg_bytes;     /* sum of compulsory bytes (each field a pass
                             must touch, once per point)                   */
} wd_kernel_stat;

/* enable != 0: later solves on this context launch without graph capture
 * and time every kernel with HIP events on the context stream (for
 * measurement; slower).  Clears the statistics either way. */
int wd_ctx_profile(wd_ctx *ctx, int enable);

/* Copy up to cap statistics (host array) gathered since wd_ctx_profile;
 * *n receives the number available. */
int wd_ctx_profile_read(wd_ctx *ctx, wd_kernel_stat *out, int cap, int *n);

/* enable != 0 (the default 1): uniform Cartesian grids without curvature
 * whose lines all admit a segmentation (segments of 32, 24 or 16 points,
 * at most 16 per line) run their directional, filter and LAD passes as
 * segmented line passes (one wave per tile of whole lines; each lane solves
 * one segment of a line by Thomas' algorithm and the segments are joined
 * through a precomputed reduced system, Sec. 3.2 / Sec. 3.4 systems
 * unchanged); enable = 16, 24 or 32 tries that segment length first;
 * 0: the reduction-level line passes.  The results agree to rounding.
 * Affects plans made after the call. */
int wd_ctx_set_segmented(wd_ctx *ctx, int enable);

/* enable != 0 (the default 1): uniform Cartesian grids with an explicit
 * scheme (E2/E4/E6, Sec. 3.2) and no extrapolated face advance each RK
 * stage in one pointwise pass: every point forms D_l phi and D_l D_l phi
 * along each direction straight from its neighbours (the Laplacian's
 * stencil is the first derivative's applied twice, closures included)
 * and finishes the stage; 0: the directional line passes.  The results
 * agree to rounding.  Affects plans made after the call. */
int wd_ctx_set_explicit_onepass(wd_ctx *ctx, int enable);

/* enable != 0 (the default 1): the LAD diffusivity of a uniform Cartesian
 * grid (Eq. Gamma_form2: the sensor C |sum_l d4_l phi^n / h_l| smoothed by
 * the nine-point truncated Gaussian along each direction) is formed by two
 * passes over x-y tiles marched along z, the sensor and then the smoothing
 * along x, y and z; 0: a sensor pass per direction and a smoothing pass per
 * direction along lines.  The results agree to rounding.  Affects plans
 * made after the call. */
int wd_ctx_set_lad_tiles(wd_ctx *ctx, int enable);

/* ---- host-side diagnostics ------------------------------------------ */
/* Applies, on the host and in FP64 arithmetic, the parallel-cyclic-reduction
 * multipliers the kernels use for a line system (Sec. 3.2 compact first
 * derivative when kind == 0, Sec. 3.4 filter correction when kind == 1):
 * x = A^{-1} rhs for the line's fixed tridiagonal matrix A.  With fp64 == 0
 * the multipliers are first rounded to FP32, as the FP32 kernels hold them.
 *   rhs, x : host arrays of n doubles (may alias).
 *   *nlev  : receives the number of reduction levels (may be NULL).
 * Touches no GPU; returns WD_ERR_INVALID_ARG for bad sizes or codes. */
int wd_line_solve_host(int kind, int n, int periodic, int scheme,
                       double alpha_f, int fp64, const double *rhs, double *x,
                       int *nlev);

/* The segmented solve of the same line systems, on the host in FP64: the
 * line cut as the segmented passes cut it (segments of 32, 24 or 16
 * positions, one possibly shorter), each segment solved locally and the
 * segments joined through the reduced system.
 *   M      : 0 (the FP32 passes' choice) or the segment length to try
 *            first.
 *   rhs, x : host arrays of n doubles (may alias).
 *   *S_used: receives 100 * segments + segment length (may be NULL).
 * Touches no GPU; WD_ERR_INVALID_ARG for bad sizes or codes,
 * WD_ERR_UNSUPPORTED when no segmentation fits the line (or not M). */
int wd_seg_solve_host(int kind, int n, int periodic, int scheme, double alpha_f, int M,
                      const double *rhs, double *x, int *S_used);

/* ---- serving (continuous batching) ---------------------------------- */
/* A host thread owns a stream and a device arena of `budget_bytes`.  It
 * admits queued requests while a slot (of max_slots) is free and their
 * workspace fits in the arena.  Small grids (at most 1/16 of the point
 * budget) go first, smallest first.  Larger grids are admitted while the
 * larger grids iterated together stay within the point budget (8M points,
 * environment WD_SERVER_POINTS; a lone request always runs): one that has
 * waited longer than 30 s (environment WD_SERVER_AGE) first, in arrival
 * order, otherwise the smallest.  Every admitted grid is advanced
 * together and retired as soon as it stops; requests admitted while others
 * run join at the next round boundary (16 iterations, environment
 * WD_SERVER_ROUND).  Results do not depend on what else runs (bitwise
 * equal to wd_solve). */
int wd_server_create(wd_ctx *ctx, size_t budget_bytes, int max_slots,
                     wd_server **out);

/* Queue one solve.  desc/method are copied; desc->metrics, desc->mask and
 * phi (device) must stay valid until the request finishes.  session >= 0
 * serialises requests of one session in submission order (an unsteady
 * sequence re-solved with warm_start from its previous field); -1 = none.
 * A warm request that the runaway check stops (wd_method.warm_probe) is
 * solved again from zero in its slot: its result is the cold solve's, its
 * iteration count includes the abandoned ones, and wd_server_stats counts
 * it among the restarts.
 * hist_cap (>= 0) FP64 history pairs are kept for wd_server_history.
 * *req_id receives the request id. */
int wd_server_submit(wd_server *srv, const wd_grid_desc *desc,
                     const wd_method *method, void *phi, long long session,
                     int hist_cap, long long *req_id);

/* State of a request: *status = WD_PENDING while queued or running, else
 * its final status; times (host seconds, steady clock) of submission,
 * admission and completion; iterations.  Any output pointer may be NULL. */
int wd_server_poll(wd_server *srv, long long req_id, int *status,
                   double *t_submit, double *t_admit, double *t_done,
                   int *iters);

/* Block until the request finishes or timeout_s passes (< 0: no limit). */
int wd_server_wait(wd_server *srv, long long req_id, double timeout_s);

/* Copy a finished request's history (host, 2*cap doubles); *n receives the
 * number of pairs written. */
int wd_server_history(wd_server *srv, long long req_id, double *hist, int cap,
                      int *n);

/* Cancel a queued or running request (its phi is left as it stands). */
int wd_server_cancel(wd_server *srv, long long req_id);

/* Counters: requests done, iterations advanced, peak arena bytes, peak
 * concurrent grids, warm requests restarted cold by the runaway check.
 * Any pointer may be NULL. */
int wd_server_stats(wd_server *srv, long long *done, long long *iterations,
                    size_t *peak_bytes, int *peak_active, long long *restarts);

/* Stop the thread (running requests are cancelled) and free the arena. */
int wd_server_destroy(wd_server *srv);

#ifdef __cplusplus
}
#endif
#endif
