/*
 * wd_oracle.c -- plain FP64 CPU oracle for PDE-based wall distance
 * (Kakumani, Vadlamani & Tucker, arXiv 2111.09859).
 *
 * TEST INFRASTRUCTURE.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this library.  It is written
 * from the paper's equations in their order, with plain loops, a Thomas
 * solver and a Sherman-Morrison cyclic solver, and shares nothing with the
 * GPU library.
 *
 * What each part follows:
 *   - transformed equations, contravariant velocity, chain-rule Laplacian:
 *     Sec. 3.1, Eqs. (Ek_eq_trans), (Ham_Jac_trans), (Poiss_trans);
 *   - first derivatives (explicit E2/E4 and compact C4/C6 central schemes,
 *     interior formula of Sec. 3.2 "Enhanced solver"); E6 adds the
 *     standard third term c (f_{i+3}-f_{i-3})/6;
 *   - pseudo-time forms: Eqs. (USeq1), (USeq3), (USeq4); 4-stage RK with
 *     local time stepping (Sec. 3.3);
 *   - convergence: Eq. (Con-criter);
 *   - implicit filter: Sec. 3.4 (order 10 inside, reduced near boundaries);
 *   - boundary conditions and initialisation: Sec. 3.5, Eqs. (eq7), (eq8);
 *   - Gamma: Eqs. (Gamma_form1), (Gamma_form2);
 *   - curvature correction: Sec. 5.4 (modified Nakanishi form);
 *   - Poisson distance: Eq. (Poiss2).
 * Readings where the paper is silent (boundary closures, near-boundary
 * filter, local time step, LAD discretisation, Neumann discretisation,
 * Poisson sign) are listed with each function below.
 *
 * Parity unpinned (against the paper) by construction: the exact discrete
 * local time step and the LAD discretisation (the grid spacing as
 * 1/|grad xi_l|, the fourth difference moved inward near a boundary, the
 * nine-point Gaussian smoothing) are readings of what the paper leaves
 * open.  The tests pin their constants and closed forms (the step on a
 * constant field, the smoothing weights from their moments, the field on
 * known profiles), not that these are the readings the authors used.
 */
#include "wd_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Threads of the grid-wide loops.  Only loops whose iterations are
 * independent (whole grid lines, single points) are shared out, and each
 * result is computed by the same operations in the same order whatever the
 * thread count; the reductions over the grid stay sequential. */
int wdo_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0)
        omp_set_num_threads(n);
    return omp_get_max_threads();
#else
    (void)n;
    return 1;
#endif
}

/* ------------------------------------------------------------------ */
/* Scheme coefficients.  Interior relation (index space):
 *   al f'_{i-1} + f'_i + al f'_{i+1}
 *      = a (f_{i+1}-f_{i-1})/2 + b (f_{i+2}-f_{i-2})/4 + c (f_{i+3}-f_{i-3})/6
 * E2: a=1.  E4: a=4/3, b=-1/3.  E6: a=3/2, b=-3/5, c=1/10.
 * C4: al=1/4, a=3/2.  C6: al=1/3, a=14/9, b=1/9.                         */
typedef struct {
    double al, a, b, c;
    int radius;   /* half width of the explicit right-hand side */
    int compact;
} scheme_t;

static scheme_t scheme_of(int s)
{
    scheme_t r;
    memset(&r, 0, sizeof r);
    switch (s) {
    case WDO_E2:
    case WDO_UW: r.a = 1.0; r.radius = 1; break;   /* UW: central parts are E2 */
    case WDO_E4: r.a = 4.0 / 3.0; r.b = -1.0 / 3.0; r.radius = 2; break;
    case WDO_E6: r.a = 1.5; r.b = -0.6; r.c = 0.1; r.radius = 3; break;
    case WDO_C4: r.al = 0.25; r.a = 1.5; r.radius = 1; r.compact = 1; break;
    default:     r.al = 1.0 / 3.0; r.a = 14.0 / 9.0; r.b = 1.0 / 9.0;
                 r.radius = 2; r.compact = 1; break;
    }
    return r;
}

/* Largest modified wavenumber of each scheme, three decimals (used only in
 * the local time step below). */
static double kprime_of(int s)
{
    switch (s) {
    case WDO_E2: return 1.0;
    case WDO_UW: return 1.0;    /* diffusive part (E2); the upwind term uses 2 */
    case WDO_E4: return 1.372;
    case WDO_E6: return 1.586;
    case WDO_C4: return 1.732;
    default:     return 1.989;
    }
}

/* value of a line at integer position i, with periodic wrap and seam jump */
static double lval(const double *f, int n, int periodic, double jump, int i)
{
    if (!periodic)
        return f[i];
    int w = (i >= 0) ? i / n : -((-i + n - 1) / n);
    int k = i - w * n;
    return f[k] + (double)w * jump;
}

/* ------------------------------------------------------------------ */
/* Tridiagonal solvers.  Row i: a[i] x[i-1] + b[i] x[i] + c[i] x[i+1] = d[i]. */
static void thomas(int n, const double *a, const double *b, const double *c,
                   double *d, double *w)
{
    double beta = b[0];
    d[0] /= beta;
    for (int i = 1; i < n; ++i) {
        w[i] = c[i - 1] / beta;
        beta = b[i] - a[i] * w[i];
        d[i] = (d[i] - a[i] * d[i - 1]) / beta;
    }
    for (int i = n - 2; i >= 0; --i)
        d[i] -= w[i + 1] * d[i + 1];
}

/* Cyclic system: a[0] multiplies x[n-1], c[n-1] multiplies x[0].
 * Sherman-Morrison on top of two Thomas solves. */
static void cyclic(int n, const double *a, const double *b, const double *c,
                   double *d)
{
    double *bb = malloc(sizeof(double) * n);
    double *u = calloc(n, sizeof(double));
    double *w = malloc(sizeof(double) * n);
    double gam = -b[0];
    for (int i = 0; i < n; ++i) bb[i] = b[i];
    bb[0] = b[0] - gam;
    bb[n - 1] = b[n - 1] - c[n - 1] * a[0] / gam;
    thomas(n, a, bb, c, d, w);          /* d <- y */
    u[0] = gam;
    u[n - 1] = c[n - 1];
    thomas(n, a, bb, c, u, w);          /* u <- z */
    double fact = (d[0] + a[0] * d[n - 1] / gam) /
                  (1.0 + u[0] + a[0] * u[n - 1] / gam);
    for (int i = 0; i < n; ++i) d[i] -= fact * u[i];
    free(bb); free(u); free(w);
}

/* ------------------------------------------------------------------ */
/* Explicit one-sided / biased closures at distance k from a boundary,
 * applied to g_j (g_0 on the boundary, j increasing inward).  Reading of
 * the closures the paper defers to its reference [visbal]:
 *   E2, node 0 : (-3, 4, -1)/2                         (exact to degree 2)
 *   E4/E6, node 0: (-25, 48, -36, 16, -3)/12           (degree 4)
 *   E4/E6, node 1: (-3, -10, 18, -6, 1)/12             (degree 4)
 *   E6, node 2   : fourth-order central (1, -8, 0, 8, -1)/12 */
static double explicit_closure(int scheme, int k, const double *g)
{
    if (scheme == WDO_E2)
        return (-3.0 * g[0] + 4.0 * g[1] - g[2]) / 2.0;
    if (k == 0)
        return (-25.0 * g[0] + 48.0 * g[1] - 36.0 * g[2] + 16.0 * g[3]
                - 3.0 * g[4]) / 12.0;
    if (k == 1)
        return (-3.0 * g[0] - 10.0 * g[1] + 18.0 * g[2] - 6.0 * g[3]
                + g[4]) / 12.0;
    return (g[0] - 8.0 * g[1] + 8.0 * g[3] - g[4]) / 12.0;
}

static double central_rhs(const scheme_t *s, const double *f, int n,
                          int periodic, double jump, int i)
{
    double r = s->a * (lval(f, n, periodic, jump, i + 1)
                       - lval(f, n, periodic, jump, i - 1)) / 2.0;
    if (s->radius >= 2 && s->b != 0.0)
        r += s->b * (lval(f, n, periodic, jump, i + 2)
                     - lval(f, n, periodic, jump, i - 2)) / 4.0;
    if (s->radius >= 3)
        r += s->c * (lval(f, n, periodic, jump, i + 3)
                     - lval(f, n, periodic, jump, i - 3)) / 6.0;
    return r;
}

/* First derivative along a line (Sec. 3.2).  Compact boundary reading:
 *   node 0   : f'_0 + 3 f'_1 = -17/6 f_0 + 3/2 f_1 + 3/2 f_2 - 1/6 f_3
 *   node 1   : (C6 only) the C4 row 1/4 f'_0 + f'_1 + 1/4 f'_2 = 3/4 (f_2 - f_0)
 * mirrored (with the sign of the right-hand side flipped) at the far end. */
int wdo_deriv_line(int n, int periodic, int scheme, double jump,
                   const double *f, double *df)
{
    if (scheme == WDO_UW)
        scheme = WDO_E2;   /* the upwind baseline's central derivatives */
    scheme_t s = scheme_of(scheme);
    if (n < 8 || scheme < WDO_E2 || scheme > WDO_C6)
        return -1;
    if (!s.compact) {
        for (int i = 0; i < n; ++i) {
            if (periodic || (i >= s.radius && i <= n - 1 - s.radius)) {
                df[i] = central_rhs(&s, f, n, periodic, jump, i);
            } else if (i < s.radius) {
                df[i] = explicit_closure(scheme, i, f);
            } else {
                int k = n - 1 - i;
                double g[5];
                for (int j = 0; j < 5; ++j) g[j] = f[n - 1 - j];
                df[i] = -explicit_closure(scheme, k, g);
            }
        }
        return 0;
    }
    double *a = malloc(sizeof(double) * n);
    double *b = malloc(sizeof(double) * n);
    double *c = malloc(sizeof(double) * n);
    double *w = malloc(sizeof(double) * n);
    for (int i = 0; i < n; ++i) {
        a[i] = s.al; b[i] = 1.0; c[i] = s.al;
        if (periodic) {
            df[i] = central_rhs(&s, f, n, 1, jump, i);
            continue;
        }
        if (i == 0) {
            a[i] = 0.0; c[i] = 3.0;
            df[i] = -17.0 / 6.0 * f[0] + 1.5 * f[1] + 1.5 * f[2] - f[3] / 6.0;
        } else if (i == n - 1) {
            a[i] = 3.0; c[i] = 0.0;
            df[i] = -(-17.0 / 6.0 * f[n - 1] + 1.5 * f[n - 2] + 1.5 * f[n - 3]
                      - f[n - 4] / 6.0);
        } else if (scheme == WDO_C6 && (i == 1 || i == n - 2)) {
            a[i] = 0.25; c[i] = 0.25;
            df[i] = 0.75 * (f[i + 1] - f[i - 1]);
        } else {
            df[i] = central_rhs(&s, f, n, 0, 0.0, i);
        }
    }
    if (periodic)
        cyclic(n, a, b, c, df);
    else
        thomas(n, a, b, c, df, w);
    free(a); free(b); free(c); free(w);
    return 0;
}

/* ------------------------------------------------------------------ */
/* Implicit filter (Sec. 3.4):
 *   af fh_{i-1} + fh_i + af fh_{i+1} = sum_{n=0}^{N} a_n/2 (f_{i+n} + f_{i-n})
 * with the published coefficients of the order-2N family (Gaitonde &
 * Visbal), written as functions of af.  Reading of the boundary treatment:
 * boundary points are not filtered; a point at distance k = 1..4 from a
 * non-periodic boundary uses the centred order-2k member; N = 5 elsewhere. */
static void filter_coeffs(int N, double af, double *an)
{
    for (int k = 0; k < 6; ++k) an[k] = 0.0;
    switch (N) {
    case 1:
        an[0] = 0.5 + af;
        an[1] = 0.5 + af;
        break;
    case 2:
        an[0] = 5.0 / 8.0 + 3.0 * af / 4.0;
        an[1] = 0.5 + af;
        an[2] = -1.0 / 8.0 + af / 4.0;
        break;
    case 3:
        an[0] = 11.0 / 16.0 + 5.0 * af / 8.0;
        an[1] = 15.0 / 32.0 + 17.0 * af / 16.0;
        an[2] = -3.0 / 16.0 + 3.0 * af / 8.0;
        an[3] = 1.0 / 32.0 - af / 16.0;
        break;
    case 4:
        an[0] = 93.0 / 128.0 + 70.0 * af / 128.0;
        an[1] = 7.0 / 16.0 + 18.0 * af / 16.0;
        an[2] = -7.0 / 32.0 + 14.0 * af / 32.0;
        an[3] = 1.0 / 16.0 - af / 8.0;
        an[4] = -1.0 / 128.0 + af / 64.0;
        break;
    default:
        an[0] = (193.0 + 126.0 * af) / 256.0;
        an[1] = (105.0 + 302.0 * af) / 256.0;
        an[2] = 15.0 * (-1.0 + 2.0 * af) / 64.0;
        an[3] = 45.0 * (1.0 - 2.0 * af) / 512.0;
        an[4] = 5.0 * (-1.0 + 2.0 * af) / 256.0;
        an[5] = (1.0 - 2.0 * af) / 512.0;
        break;
    }
}

int wdo_filter_line(int n, int periodic, double alpha_f, const double *f,
                    double *out)
{
    if (n < 8)
        return -1;
    double an[6];
    if (periodic) {
        double *a = malloc(sizeof(double) * n);
        double *b = malloc(sizeof(double) * n);
        double *c = malloc(sizeof(double) * n);
        filter_coeffs(5, alpha_f, an);
        for (int i = 0; i < n; ++i) {
            a[i] = alpha_f; b[i] = 1.0; c[i] = alpha_f;
            double r = 0.0;
            for (int k = 0; k <= 5; ++k)
                r += an[k] / 2.0 * (lval(f, n, 1, 0.0, i + k)
                                    + lval(f, n, 1, 0.0, i - k));
            out[i] = r;
        }
        cyclic(n, a, b, c, out);
        free(a); free(b); free(c);
        return 0;
    }
    /* unknowns are points 1..n-2; the boundary values stay as they are */
    int m = n - 2;
    double *a = malloc(sizeof(double) * m);
    double *b = malloc(sizeof(double) * m);
    double *c = malloc(sizeof(double) * m);
    double *d = malloc(sizeof(double) * m);
    double *w = malloc(sizeof(double) * m);
    for (int i = 1; i <= n - 2; ++i) {
        int dist = i < n - 1 - i ? i : n - 1 - i;
        int N = dist < 5 ? dist : 5;
        filter_coeffs(N, alpha_f, an);
        double r = 0.0;
        for (int k = 0; k <= N; ++k)
            r += an[k] / 2.0 * (f[i + k] + f[i - k]);
        int j = i - 1;
        a[j] = alpha_f; b[j] = 1.0; c[j] = alpha_f;
        if (i == 1) r -= alpha_f * f[0];
        if (i == n - 2) r -= alpha_f * f[n - 1];
        d[j] = r;
    }
    thomas(m, a, b, c, d, w);
    out[0] = f[0];
    out[n - 1] = f[n - 1];
    for (int j = 0; j < m; ++j) out[j + 1] = d[j];
    free(a); free(b); free(c); free(d); free(w);
    return 0;
}

/* ------------------------------------------------------------------ */
/* Grid helpers */
static long npoints(const wdo_grid *g)
{
    long N = 1;
    for (int l = 0; l < g->ndim; ++l) N *= g->n[l];
    return N;
}

static long stride_of(const wdo_grid *g, int l)
{
    long s = 1;
    for (int k = 0; k < l; ++k) s *= g->n[k];
    return s;
}

/* base offset of line k of direction l */
static long line_base(const wdo_grid *g, int l, long k)
{
    int n0 = g->n[0], n1 = g->ndim > 1 ? g->n[1] : 1;
    if (l == 0)
        return k * n0;
    if (l == 1) {
        long i0 = k % n0, i2 = k / n0;
        return i0 + i2 * (long)n0 * n1;
    }
    {
        long i0 = k % n0, i1 = k / n0;
        return i0 + i1 * n0;
    }
}

static void index_of(const wdo_grid *g, long q, int *idx)
{
    idx[0] = (int)(q % g->n[0]);
    long r = q / g->n[0];
    idx[1] = g->ndim > 1 ? (int)(r % g->n[1]) : 0;
    idx[2] = g->ndim > 2 ? (int)(r / g->n[1]) : 0;
}

/* apply D_l to field f (grid-shaped), jump for coordinate seams */
static int deriv_dir(const wdo_grid *g, int l, int scheme, double jump,
                     const double *f, double *out)
{
    int n = g->n[l];
    long s = stride_of(g, l);
    long nl = npoints(g) / n;
    int periodic = g->bc[l][0] == WDO_PERIODIC;
    int rc = 0;
#pragma omp parallel
    {
        double *line = malloc(sizeof(double) * n);
        double *dl = malloc(sizeof(double) * n);
#pragma omp for schedule(static)
        for (long k = 0; k < nl; ++k) {
            long base = line_base(g, l, k);
            for (int i = 0; i < n; ++i) line[i] = f[base + i * s];
            if (wdo_deriv_line(n, periodic, scheme, jump, line, dl)) {
#pragma omp atomic write
                rc = -1;
                continue;
            }
            for (int i = 0; i < n; ++i) out[base + i * s] = dl[i];
        }
        free(line); free(dl);
    }
    return rc;
}

static int filter_dir(const wdo_grid *g, int l, double af, double *f)
{
    int n = g->n[l];
    long s = stride_of(g, l);
    long nl = npoints(g) / n;
    int periodic = g->bc[l][0] == WDO_PERIODIC;
    int rc = 0;
#pragma omp parallel
    {
        double *line = malloc(sizeof(double) * n);
        double *fl = malloc(sizeof(double) * n);
#pragma omp for schedule(static)
        for (long k = 0; k < nl; ++k) {
            long base = line_base(g, l, k);
            for (int i = 0; i < n; ++i) line[i] = f[base + i * s];
            if (wdo_filter_line(n, periodic, af, line, fl)) {
#pragma omp atomic write
                rc = -1;
                continue;
            }
            for (int i = 0; i < n; ++i) f[base + i * s] = fl[i];
        }
        free(line); free(fl);
    }
    return rc;
}

/* ------------------------------------------------------------------ */
/* Metrics (Sec. 3.1 with the solve's own scheme, Sec. 3.2): the Jacobian
 * J[m][l] = d x_m / d xi_l from the derivative operator, then its inverse
 * M[l][m] = d xi_l / d x_m at every point.
 *
 * metric_form 1 (3D, an option beside the paper's recipe): the
 * conservative form of the metric terms.  The cofactor of d x_m / d xi_l
 * is written as a divergence, J xi_{l,m} = sum over the Levi-Civita
 * symbols of D_q (x_b D_p x_a) / 2, which for (m, a, b) and (l, p, q)
 * cyclic is
 *   Q_{p,m} = x_b J[a][p] - x_a J[b][p],
 *   J xi_{l,m} = (D_q Q_{p,m} - D_p Q_{q,m}) / 2,
 * and xi_{l,m} = (J xi_{l,m}) / det J.  Because derivatives along
 * different directions commute, sum_l D_l (J xi_{l,m}) = 0 holds to
 * rounding (the discrete metric identity); on an affine grid the two forms
 * agree.  Coordinates that jump across a periodic seam are not supported
 * in this form (the products would jump by a varying amount). */
static int metrics_conservative(const wdo_grid *g, int scheme, const double *J, double *met)
{
    long N = npoints(g);
    for (int l = 0; l < 3; ++l)
        for (int m = 0; m < 3; ++m)
            if (g->period[l][m] != 0.0) return -2;
    double *Q = malloc(sizeof(double) * N * 9);
    double *Dq = malloc(sizeof(double) * N);
    double *Dp = malloc(sizeof(double) * N);
    double *T = malloc(sizeof(double) * N * 9);
    int rc = 0;
    /* Q[p][m] */
    for (int p = 0; p < 3; ++p)
        for (int m = 0; m < 3; ++m) {
            int a = (m + 1) % 3, b = (m + 2) % 3;
            const double *xa = g->coords + a * N, *xb = g->coords + b * N;
            const double *Jap = J + (a * 3 + p) * N, *Jbp = J + (b * 3 + p) * N;
            double *q = Q + (p * 3 + m) * N;
            for (long k = 0; k < N; ++k) q[k] = xb[k] * Jap[k] - xa[k] * Jbp[k];
        }
    /* J xi_{l,m} */
    for (int l = 0; l < 3 && !rc; ++l) {
        int p = (l + 1) % 3, q = (l + 2) % 3;
        for (int m = 0; m < 3 && !rc; ++m) {
            rc = deriv_dir(g, q, scheme, 0.0, Q + (p * 3 + m) * N, Dq);
            if (!rc) rc = deriv_dir(g, p, scheme, 0.0, Q + (q * 3 + m) * N, Dp);
            double *t = T + (l * 3 + m) * N;
            for (long k = 0; k < N; ++k) t[k] = 0.5 * (Dq[k] - Dp[k]);
        }
    }
    if (!rc)
        for (long k = 0; k < N; ++k) {
            double A[3][3];
            for (int m = 0; m < 3; ++m)
                for (int l = 0; l < 3; ++l)
                    A[m][l] = J[(m * 3 + l) * N + k];
            double det = A[0][0] * (A[1][1] * A[2][2] - A[1][2] * A[2][1])
                       - A[0][1] * (A[1][0] * A[2][2] - A[1][2] * A[2][0])
                       + A[0][2] * (A[1][0] * A[2][1] - A[1][1] * A[2][0]);
            for (int l = 0; l < 3; ++l)
                for (int m = 0; m < 3; ++m)
                    met[(l * 3 + m) * N + k] = T[(l * 3 + m) * N + k] / det;
        }
    free(Q); free(Dq); free(Dp); free(T);
    return rc;
}

int wdo_metrics(const wdo_grid *g, int scheme, double *met)
{
    int d = g->ndim;
    long N = npoints(g);
    if (g->uniform) {
        for (int l = 0; l < d; ++l)
            for (int m = 0; m < d; ++m)
                for (long q = 0; q < N; ++q)
                    met[(l * d + m) * N + q] = (l == m) ? 1.0 / g->h[l] : 0.0;
        return 0;
    }
    double *J = malloc(sizeof(double) * N * d * d);
    for (int m = 0; m < d; ++m)
        for (int l = 0; l < d; ++l) {
            int rc = deriv_dir(g, l, scheme, g->period[l][m],
                               g->coords + m * N, J + (m * d + l) * N);
            if (rc) { free(J); return rc; }
        }
    if (d == 3 && g->metric_form == 1) {
        int rc = metrics_conservative(g, scheme, J, met);
        free(J);
        return rc;
    }
#pragma omp parallel for schedule(static)
    for (long q = 0; q < N; ++q) {
        double A[3][3], Inv[3][3];
        for (int m = 0; m < d; ++m)
            for (int l = 0; l < d; ++l)
                A[m][l] = J[(m * d + l) * N + q];
        if (d == 2) {
            double det = A[0][0] * A[1][1] - A[0][1] * A[1][0];
            Inv[0][0] = A[1][1] / det;
            Inv[0][1] = -A[0][1] / det;
            Inv[1][0] = -A[1][0] / det;
            Inv[1][1] = A[0][0] / det;
        } else {
            double det = A[0][0] * (A[1][1] * A[2][2] - A[1][2] * A[2][1])
                       - A[0][1] * (A[1][0] * A[2][2] - A[1][2] * A[2][0])
                       + A[0][2] * (A[1][0] * A[2][1] - A[1][1] * A[2][0]);
            Inv[0][0] = (A[1][1] * A[2][2] - A[1][2] * A[2][1]) / det;
            Inv[0][1] = (A[0][2] * A[2][1] - A[0][1] * A[2][2]) / det;
            Inv[0][2] = (A[0][1] * A[1][2] - A[0][2] * A[1][1]) / det;
            Inv[1][0] = (A[1][2] * A[2][0] - A[1][0] * A[2][2]) / det;
            Inv[1][1] = (A[0][0] * A[2][2] - A[0][2] * A[2][0]) / det;
            Inv[1][2] = (A[0][2] * A[1][0] - A[0][0] * A[1][2]) / det;
            Inv[2][0] = (A[1][0] * A[2][1] - A[1][1] * A[2][0]) / det;
            Inv[2][1] = (A[0][1] * A[2][0] - A[0][0] * A[2][1]) / det;
            Inv[2][2] = (A[0][0] * A[1][1] - A[0][1] * A[1][0]) / det;
        }
        /* Inv[l][m] is d xi_l / d x_m */
        for (int l = 0; l < d; ++l)
            for (int m = 0; m < d; ++m)
                met[(l * d + m) * N + q] = Inv[l][m];
    }
    free(J);
    return 0;
}

/* ------------------------------------------------------------------ */
/* Boundary conditions (Sec. 3.5).  Wall faces and solid points are set to
 * zero (Eq. eq7).  Reading of the far-field Neumann condition (Eq. eq8):
 * second-order one-sided zero gradient along the grid line normal to the
 * face, phi_b = (4 phi_{b+1} - phi_{b+2}) / 3.  Outflow faces (an option
 * beside the paper's far field) extrapolate linearly along the grid line,
 * phi_b = 2 phi_{b+1} - phi_{b+2}.  Both are applied face by face in the
 * order (dir 0 low, dir 0 high, dir 1 low, ...) after the zeroing, and
 * skip points that lie on a wall face or inside a solid. */
static int on_wall(const wdo_grid *g, const int *idx)
{
    for (int l = 0; l < g->ndim; ++l) {
        if (idx[l] == 0 && g->bc[l][0] == WDO_WALL) return 1;
        if (idx[l] == g->n[l] - 1 && g->bc[l][1] == WDO_WALL) return 1;
    }
    return 0;
}

void wdo_apply_bc(const wdo_grid *g, double *phi)
{
    long N = npoints(g);
#pragma omp parallel for schedule(static)
    for (long q = 0; q < N; ++q) {
        int idx[3];
        index_of(g, q, idx);
        if (on_wall(g, idx) || (g->mask && g->mask[q]))
            phi[q] = 0.0;
    }
    for (int l = 0; l < g->ndim; ++l)
        for (int side = 0; side < 2; ++side) {
            int code = g->bc[l][side];
            if (code != WDO_NEUMANN && code != WDO_OUTFLOW) continue;
            long s = stride_of(g, l);
            int target = side == 0 ? 0 : g->n[l] - 1;
            long inward = side == 0 ? s : -s;
#pragma omp parallel for schedule(static)
            for (long q = 0; q < N; ++q) {
                int idx[3];
                index_of(g, q, idx);
                if (idx[l] != target) continue;
                if (on_wall(g, idx) || (g->mask && g->mask[q])) continue;
                if (code == WDO_NEUMANN)
                    phi[q] = (4.0 * phi[q + inward] - phi[q + 2 * inward]) / 3.0;
                else
                    phi[q] = 2.0 * phi[q + inward] - phi[q + 2 * inward];
            }
        }
}

/* ------------------------------------------------------------------ */
/* Five-point fourth difference along direction l at every point.  Reading
 * of Eq. (Gamma_form2)'s fourth derivative: index-space difference
 * f_{i-2} - 4 f_{i-1} + 6 f_i - 4 f_{i+1} + f_{i+2}; the two points nearest
 * a non-periodic boundary take the value of the nearest point where the
 * stencil fits. */
static void fourth_diff_dir(const wdo_grid *g, int l, const double *f,
                            double *out)
{
    int n = g->n[l];
    long s = stride_of(g, l);
    long nl = npoints(g) / n;
    int periodic = g->bc[l][0] == WDO_PERIODIC;
#pragma omp parallel for schedule(static)
    for (long k = 0; k < nl; ++k) {
        long base = line_base(g, l, k);
        for (int i = 0; i < n; ++i) {
            int c = i;
            if (!periodic) {
                if (c < 2) c = 2;
                if (c > n - 3) c = n - 3;
            }
            double v[5];
            for (int j = -2; j <= 2; ++j) {
                int p = c + j;
                if (periodic) p = ((p % n) + n) % n;
                v[j + 2] = f[base + p * s];
            }
            out[base + i * s] = v[0] - 4.0 * v[1] + 6.0 * v[2] - 4.0 * v[3] + v[4];
        }
    }
}

/* Truncated Gaussian smoothing along direction l (nine points, Kawai & Lele
 * style), in place; non-periodic lines use the nearest in-range value
 * beyond the ends. */
static void gauss_dir(const wdo_grid *g, int l, double *f, double *tmp)
{
    static const double b[5] = {3565.0 / 10368.0, 3091.0 / 12960.0,
                                1997.0 / 25920.0, 149.0 / 12960.0,
                                107.0 / 103680.0};
    int n = g->n[l];
    long s = stride_of(g, l);
    long nl = npoints(g) / n;
    int periodic = g->bc[l][0] == WDO_PERIODIC;
#pragma omp parallel for schedule(static)
    for (long k = 0; k < nl; ++k) {
        long base = line_base(g, l, k);
        for (int i = 0; i < n; ++i) {
            double acc = 0.0;
            for (int o = -4; o <= 4; ++o) {
                int p = i + o;
                if (periodic) p = ((p % n) + n) % n;
                else p = p < 0 ? 0 : (p > n - 1 ? n - 1 : p);
                acc += b[o < 0 ? -o : o] * f[base + p * s];
            }
            tmp[base + i * s] = acc;
        }
        for (int i = 0; i < n; ++i) f[base + i * s] = tmp[base + i * s];
    }
}

/* The smoothing of one line on its own (a test accessor of gauss_dir). */
int wdo_gauss_line(int n, int periodic, const double *f, double *out)
{
    if (n < 9)
        return -1;
    wdo_grid g;
    memset(&g, 0, sizeof g);
    g.ndim = 2;
    g.n[0] = n;
    g.n[1] = 1;
    g.n[2] = 1;
    g.bc[0][0] = g.bc[0][1] = periodic ? WDO_PERIODIC : WDO_WALL;
    g.uniform = 1;
    double *tmp = malloc(sizeof(double) * n);
    for (int i = 0; i < n; ++i) out[i] = f[i];
    gauss_dir(&g, 0, out, tmp);
    free(tmp);
    return 0;
}

/* LAD diffusivity (second argument of Eq. Gamma_form2):
 *   C | sum_l (sum_m xi_{l,m}^2)^2 d4_l phi dx_l^3 |,  dx_l = 1/|grad xi_l|
 * (reading: dx_l from the metrics, d4 the five-point index difference).
 * Reading of the LAD scheme the paper follows (Kawai & Lele): the
 * diffusivity is smoothed with their truncated Gaussian filter along each
 * direction in turn. */
int wdo_lad_field(const wdo_grid *g, const wdo_method *m, const double *met,
                  const double *phi, double *out)
{
    int d = g->ndim;
    long N = npoints(g);
    double *tmp = malloc(sizeof(double) * N);
    for (long q = 0; q < N; ++q) out[q] = 0.0;
    for (int l = 0; l < d; ++l) {
        fourth_diff_dir(g, l, phi, tmp);
#pragma omp parallel for schedule(static)
        for (long q = 0; q < N; ++q) {
            double s2 = 0.0;
            for (int mm = 0; mm < d; ++mm) {
                double e = met[(l * d + mm) * N + q];
                s2 += e * e;
            }
            double dx = 1.0 / sqrt(s2);
            out[q] += s2 * s2 * tmp[q] * dx * dx * dx;
        }
    }
#pragma omp parallel for schedule(static)
    for (long q = 0; q < N; ++q) out[q] = m->C * fabs(out[q]);
    if (!m->lad_raw)
        for (int l = 0; l < d; ++l) gauss_dir(g, l, out, tmp);
    free(tmp);
    return 0;
}

/* Advective term of the upwind baseline (Sec. 3.2.1).  Along each grid
 * direction l, with unit index spacing, B = phi_i - phi_{i-1} and
 * F = phi_{i+1} - phi_i (periodic lines wrap; at the two ends of a
 * non-periodic line the missing one equals the other).  The derivative that
 * enters the contravariant velocity (Eq. UW3) takes the switch weights of
 * Eqs. UW4-UW5, SIGN(1, x) = +1 for x >= 0 and -1 otherwise:
 *   n_{i-1} = (1 + SIGN(1, F+B)) (1 + SIGN(1, B)) / 4,
 *   n_{i+1} = (1 - SIGN(1, F+B)) (1 - SIGN(1, F)) / 4,
 *   phi_l ~ n_{i-1} B + n_{i+1} F   (reading: n_{i-1} weighs the i-1 side;
 *   uw_printed = 1 pairs them as printed, n_{i-1} F + n_{i+1} B),
 * so a rising line uses B, a falling one F, a minimum 0 and a ridge the
 * steeper side.  U_m = sum_l xi_{l,m} phi_l, Uh_l = sum_m xi_{l,m} U_m and
 * (Eq. UW1) U.grad(phi) = sum_l [(Uh_l + |Uh_l|) B + (Uh_l - |Uh_l|) F] / 2.
 * adv receives U.grad(phi), g2 receives |U|^2. */
static void uw_advection(const wdo_grid *g, const wdo_method *m, const double *met,
                         const double *phi, double *adv, double *g2)
{
    int d = g->ndim;
    long N = npoints(g);
#pragma omp parallel for schedule(static)
    for (long q = 0; q < N; ++q) {
        int idx[3];
        index_of(g, q, idx);
        double B[3], F[3], D[3];
        for (int l = 0; l < d; ++l) {
            int n = g->n[l], i = idx[l];
            long s = stride_of(g, l);
            int periodic = g->bc[l][0] == WDO_PERIODIC;
            int has_m = i > 0 || periodic, has_p = i < n - 1 || periodic;
            long qm = i > 0 ? q - s : q + (long)(n - 1) * s;
            long qp = i < n - 1 ? q + s : q - (long)(n - 1) * s;
            double b = has_m ? phi[q] - phi[qm] : 0.0;
            double f = has_p ? phi[qp] - phi[q] : 0.0;
            if (!has_m) b = f;
            if (!has_p) f = b;
            double sfb = (f + b) >= 0.0 ? 1.0 : -1.0;
            double sb = b >= 0.0 ? 1.0 : -1.0, sf = f >= 0.0 ? 1.0 : -1.0;
            double nm = 0.25 * (1.0 + sfb) * (1.0 + sb);
            double np = 0.25 * (1.0 - sfb) * (1.0 - sf);
            B[l] = b;
            F[l] = f;
            D[l] = m->uw_printed ? nm * f + np * b : nm * b + np * f;
        }
        double Um[3] = {0.0, 0.0, 0.0}, s2 = 0.0;
        for (int mm = 0; mm < d; ++mm) {
            for (int l = 0; l < d; ++l) Um[mm] += met[(l * d + mm) * N + q] * D[l];
            s2 += Um[mm] * Um[mm];
        }
        double a = 0.0;
        for (int l = 0; l < d; ++l) {
            double uh = 0.0;
            for (int mm = 0; mm < d; ++mm) uh += met[(l * d + mm) * N + q] * Um[mm];
            a += 0.5 * (uh + fabs(uh)) * B[l] + 0.5 * (uh - fabs(uh)) * F[l];
        }
        adv[q] = a;
        g2[q] = s2;
    }
}

/* Right-hand side of the pseudo-time equation at phi (Sec. 3.3):
 *   Eikonal (USeq1):  R = 1 - U.grad(phi) = 1 - |grad phi|^2
 *   HJ      (USeq3):  R = 1 + Gamma lap(phi) - |grad phi|^2
 *   HJ + curvature:   R = 1 + (Gamma + nu) (lap(phi) - max(0, |grad phi| kappa))
 *                         - |grad phi|^2      (Sec. 5.4; Gamma is either form)
 *   Poisson (USeq4):  R = 1 + lap(phi)
 * with U_m = sum_l xi_{l,m} D_l phi and lap = sum_m sum_l xi_{l,m} D_l U_m
 * (Eq. Ham_Jac_trans).  Reading of the local time step (the paper only
 * names local time stepping):
 *   dt = sigma / ( 2 k' S1 max(|grad phi|, 1) + k'^2 (Gamma + nu) S2 ),
 *   S1 = sum_l |grad xi_l|, S2 = sum_l |grad xi_l|^2, k' the scheme's
 *   largest modified wavenumber; Eikonal drops the second term, Poisson
 *   uses dt = sigma / (k'^2 S2). */
int wdo_eval(const wdo_grid *g, const wdo_method *m, const double *met,
             const double *phi, const double *lad_in, double *R, double *gmag,
             double *gam, double *lap, double *kap, double *dt)
{
    int d = g->ndim;
    long N = npoints(g);
    int rc = 0;
    double *F = malloc(sizeof(double) * N * d);
    double *U = malloc(sizeof(double) * N * d);
    double *tmp = malloc(sizeof(double) * N);
    double *L = calloc(N, sizeof(double));
    double *K = calloc(N, sizeof(double));
    double *G = malloc(sizeof(double) * N);
    for (int l = 0; l < d && !rc; ++l)
        rc = deriv_dir(g, l, m->scheme, 0.0, phi, F + l * N);
    for (int mm = 0; mm < d; ++mm)
#pragma omp parallel for schedule(static)
        for (long q = 0; q < N; ++q) {
            double u = 0.0;
            for (int l = 0; l < d; ++l)
                u += met[(l * d + mm) * N + q] * F[l * N + q];
            U[mm * N + q] = u;
        }
#pragma omp parallel for schedule(static)
    for (long q = 0; q < N; ++q) {
        double s = 0.0;
        for (int mm = 0; mm < d; ++mm) s += U[mm * N + q] * U[mm * N + q];
        G[q] = sqrt(s);
    }
    int uw = m->scheme == WDO_UW && m->equation != WDO_POISSON;
    double *Adv = NULL, *G2 = NULL;
    if (uw) {
        if (m->equation == WDO_HJ && m->curvature) {
            free(F); free(U); free(tmp); free(L); free(K); free(G);
            return -1;   /* the baseline has no curvature correction */
        }
        Adv = malloc(sizeof(double) * N);
        G2 = malloc(sizeof(double) * N);
        uw_advection(g, m, met, phi, Adv, G2);
        for (long q = 0; q < N; ++q) G[q] = sqrt(G2[q]);
    }
    int need_lap = m->equation != WDO_EIKONAL;
    int curv = m->equation == WDO_HJ && m->curvature;
    if (need_lap)
        for (int mm = 0; mm < d && !rc; ++mm)
            for (int l = 0; l < d && !rc; ++l) {
                rc = deriv_dir(g, l, m->scheme, 0.0, U + mm * N, tmp);
#pragma omp parallel for schedule(static)
                for (long q = 0; q < N; ++q)
                    L[q] += met[(l * d + mm) * N + q] * tmp[q];
            }
    if (curv) {
        double *nv = malloc(sizeof(double) * N);
        for (int mm = 0; mm < d && !rc; ++mm) {
#pragma omp parallel for schedule(static)
            for (long q = 0; q < N; ++q)
                nv[q] = U[mm * N + q] / (G[q] + m->eps0);
            for (int l = 0; l < d && !rc; ++l) {
                rc = deriv_dir(g, l, m->scheme, 0.0, nv, tmp);
#pragma omp parallel for schedule(static)
                for (long q = 0; q < N; ++q)
                    K[q] += met[(l * d + mm) * N + q] * tmp[q];
            }
        }
        free(nv);
    }
    /* Gamma: standard eps*phi (Gamma_form1) or min(eps*phi, LAD field)
     * (Gamma_form2); clipped at zero. */
    double *Gam = calloc(N, sizeof(double));
    if (m->equation == WDO_HJ) {
        double *S = NULL;
        const double *lad = lad_in;
        if (m->gamma == WDO_GAMMA_LAD && !lad) {
            S = malloc(sizeof(double) * N);
            wdo_lad_field(g, m, met, phi, S);
            lad = S;
        }
#pragma omp parallel for schedule(static)
        for (long q = 0; q < N; ++q) {
            double gq = m->eps * phi[q];
            if (m->gamma == WDO_GAMMA_LAD && lad[q] < gq) gq = lad[q];
            Gam[q] = gq > 0.0 ? gq : 0.0;
        }
        free(S);
    }
    double kp = kprime_of(m->scheme);
    /* the upwind term's largest modified wavenumber: |1 - e^{-i w}| <= 2 */
    double kadv = m->scheme == WDO_UW ? 2.0 : kp;
#pragma omp parallel for schedule(static)
    for (long q = 0; q < N; ++q) {
        double g2 = 0.0;
        for (int mm = 0; mm < d; ++mm) g2 += U[mm * N + q] * U[mm * N + q];
        if (uw) g2 = Adv[q];    /* U.grad(phi) by Eqs. UW1-UW5 */
        double nu = curv ? m->nu0 * (1.0 - G[q]) * (1.0 - G[q]) : 0.0;
        double r;
        if (m->equation == WDO_EIKONAL)
            r = 1.0 - g2;
        else if (m->equation == WDO_POISSON)
            r = 1.0 + L[q];
        else if (curv) {
            double gk = G[q] * K[q];
            r = 1.0 + (Gam[q] + nu) * (L[q] - (gk > 0.0 ? gk : 0.0)) - g2;
        } else
            r = 1.0 + Gam[q] * L[q] - g2;
        if (R) R[q] = r;
        if (gmag) gmag[q] = G[q];
        if (gam) gam[q] = Gam[q];
        if (lap) lap[q] = L[q];
        if (kap) kap[q] = K[q];
        if (dt) {
            double S1 = 0.0, S2 = 0.0;
            for (int l = 0; l < d; ++l) {
                double s2 = 0.0;
                for (int mm = 0; mm < d; ++mm) {
                    double e = met[(l * d + mm) * N + q];
                    s2 += e * e;
                }
                S1 += sqrt(s2);
                S2 += s2;
            }
            double gm = G[q] > 1.0 ? G[q] : 1.0;
            double den;
            if (m->equation == WDO_EIKONAL)
                den = 2.0 * kadv * S1 * gm;
            else if (m->equation == WDO_POISSON)
                den = kp * kp * S2;
            else
                den = 2.0 * kadv * S1 * gm + kp * kp * (Gam[q] + nu) * S2;
            dt[q] = m->sigma / den;
        }
    }
    free(F); free(U); free(tmp); free(L); free(K); free(G); free(Gam);
    free(Adv); free(G2);
    return rc;
}

/* ------------------------------------------------------------------ */
/* Pseudo-time march (Sec. 3.3-3.5, Fig. flow chart (b)):
 *   phi = 0, BCs; per iteration: local dt from phi^n; RK stages, each
 *   followed by the BCs; filter along xi, eta, zeta in turn; BCs;
 *   r_n = max |phi^{n+1} - phi^n| (Eq. Con-criter); stop when r_n <= tol.
 * RK4 is the classical four-stage scheme; RK3 is the Shu-Osher SSP
 * scheme (reading: a three-stage option beside the paper's RK4). */
int wdo_solve(const wdo_grid *g, const wdo_method *m, double *phi, int warm,
              double *hist, int hist_cap, int *iters)
{
    if (!g || !m || !phi || g->ndim < 2 || g->ndim > 3)
        return -1;
    long N = npoints(g);
    int d = g->ndim;
    double *met = malloc(sizeof(double) * N * d * d);
    if (wdo_metrics(g, m->scheme, met)) { free(met); return -1; }
    double *pn = malloc(sizeof(double) * N);
    double *p = malloc(sizeof(double) * N);
    double *k1 = malloc(sizeof(double) * N);
    double *k2 = malloc(sizeof(double) * N);
    double *k3 = malloc(sizeof(double) * N);
    double *k4 = malloc(sizeof(double) * N);
    double *dt = malloc(sizeof(double) * N);
    double *lad = NULL;
    if (m->equation == WDO_HJ && m->gamma == WDO_GAMMA_LAD && !m->lad_raw)
        lad = malloc(sizeof(double) * N);
    if (!warm)
        for (long q = 0; q < N; ++q) phi[q] = 0.0;
    wdo_apply_bc(g, phi);
    int status = 1, it = 0;
    int limit = m->fixed_iters > 0 ? m->fixed_iters : m->max_iter;
    for (it = 0; it < limit; ++it) {
        memcpy(pn, phi, sizeof(double) * N);
        if (lad)
            wdo_lad_field(g, m, met, pn, lad);
        if (m->rk == WDO_RK4) {
            wdo_eval(g, m, met, pn, lad, k1, NULL, NULL, NULL, NULL, dt);
#pragma omp parallel for schedule(static)
            for (long q = 0; q < N; ++q) p[q] = pn[q] + dt[q] / 2.0 * k1[q];
            wdo_apply_bc(g, p);
            wdo_eval(g, m, met, p, lad, k2, NULL, NULL, NULL, NULL, NULL);
#pragma omp parallel for schedule(static)
            for (long q = 0; q < N; ++q) p[q] = pn[q] + dt[q] / 2.0 * k2[q];
            wdo_apply_bc(g, p);
            wdo_eval(g, m, met, p, lad, k3, NULL, NULL, NULL, NULL, NULL);
#pragma omp parallel for schedule(static)
            for (long q = 0; q < N; ++q) p[q] = pn[q] + dt[q] * k3[q];
            wdo_apply_bc(g, p);
            wdo_eval(g, m, met, p, lad, k4, NULL, NULL, NULL, NULL, NULL);
#pragma omp parallel for schedule(static)
            for (long q = 0; q < N; ++q)
                phi[q] = pn[q] + dt[q] / 6.0 * (k1[q] + 2.0 * k2[q]
                                                + 2.0 * k3[q] + k4[q]);
            wdo_apply_bc(g, phi);
        } else {
            wdo_eval(g, m, met, pn, lad, k1, NULL, NULL, NULL, NULL, dt);
#pragma omp parallel for schedule(static)
            for (long q = 0; q < N; ++q) p[q] = pn[q] + dt[q] * k1[q];
            wdo_apply_bc(g, p);
            wdo_eval(g, m, met, p, lad, k2, NULL, NULL, NULL, NULL, NULL);
#pragma omp parallel for schedule(static)
            for (long q = 0; q < N; ++q)
                k3[q] = 0.75 * pn[q] + 0.25 * (p[q] + dt[q] * k2[q]);
            wdo_apply_bc(g, k3);
            wdo_eval(g, m, met, k3, lad, k2, NULL, NULL, NULL, NULL, NULL);
#pragma omp parallel for schedule(static)
            for (long q = 0; q < N; ++q)
                phi[q] = pn[q] / 3.0 + 2.0 / 3.0 * (k3[q] + dt[q] * k2[q]);
            wdo_apply_bc(g, phi);
        }
        if (m->filter) {
            for (int l = 0; l < d; ++l)
                filter_dir(g, l, m->alpha_f, phi);
            wdo_apply_bc(g, phi);
        }
        double rmax = 0.0, s2 = 0.0;
        for (long q = 0; q < N; ++q) {
            double e = fabs(phi[q] - pn[q]);
            if (e > rmax || e != e) rmax = e;
            s2 += e * e;
        }
        double l2 = sqrt(s2 / (double)N);
        if (hist && it < hist_cap) {
            hist[2 * it] = rmax;
            hist[2 * it + 1] = l2;
        }
        if (!isfinite(rmax) || !isfinite(l2)) {
            status = -3;
            ++it;
            break;
        }
        if (m->fixed_iters <= 0 && rmax <= m->tol) {
            status = 0;
            ++it;
            break;
        }
    }
    if (m->fixed_iters > 0 && status == 1)
        status = 0;
    if (iters) *iters = it;
    free(met); free(pn); free(p); free(k1); free(k2); free(k3); free(k4);
    free(dt); free(lad);
    return status;
}

/* ------------------------------------------------------------------ */
/* Eq. (Poiss2) with the minus sign (reading: the root that vanishes at the
 * wall and gives min(y, 1-y) in a channel), gradient by the solve's scheme
 * and metrics. */
int wdo_poisson_distance(const wdo_grid *g, int scheme, const double *met,
                         const double *phip, double *dist)
{
    int d = g->ndim;
    long N = npoints(g);
    double *F = malloc(sizeof(double) * N * d);
    int rc = 0;
    for (int l = 0; l < d && !rc; ++l)
        rc = deriv_dir(g, l, scheme, 0.0, phip, F + l * N);
    for (long q = 0; q < N && !rc; ++q) {
        double s = 0.0;
        for (int mm = 0; mm < d; ++mm) {
            double u = 0.0;
            for (int l = 0; l < d; ++l)
                u += met[(l * d + mm) * N + q] * F[l * N + q];
            s += u * u;
        }
        double inner = s + 2.0 * phip[q];
        if (inner < 0.0) inner = 0.0;
        dist[q] = -sqrt(s) + sqrt(inner);
    }
    free(F);
    return rc;
}

/* Nearest-wall search by brute force (the search approach of Sec. 1),
 * used only to check tiny cases. */
void wdo_brute_force(int ndim, int npts, const double *pts, int nwall,
                     const double *wall, double *dist)
{
    for (int i = 0; i < npts; ++i) {
        double best = INFINITY;
        for (int k = 0; k < nwall; ++k) {
            double s = 0.0;
            for (int m = 0; m < ndim; ++m) {
                double e = pts[i * ndim + m] - wall[k * ndim + m];
                s += e * e;
            }
            if (s < best) best = s;
        }
        dist[i] = sqrt(best);
    }
}


/* ------------------------------------------------------------------ */
/* Level-set burnback (Sec. 5.5).                                      */

void wdo_signed_distance(long n, const unsigned char *solid, const double *d_solid,
                         const double *d_gas, double *phi_s)
{
    for (long q = 0; q < n; ++q) phi_s[q] = solid[q] ? d_solid[q] : -d_gas[q];
}

/* |grad phi| at every point: along each direction the upwind switch of
 * Eqs. UW3-UW5 (the reading documented at uw_advection) picks B, F or 0,
 * divided by the uniform spacing. */
static void levelset_grad(const wdo_grid *g, const double *phi, double *gm)
{
    long N = npoints(g);
    for (long q = 0; q < N; ++q) {
        int idx[3];
        index_of(g, q, idx);
        double s2 = 0.0;
        for (int l = 0; l < g->ndim; ++l) {
            int n = g->n[l], i = idx[l];
            long s = stride_of(g, l);
            int periodic = g->bc[l][0] == WDO_PERIODIC;
            int has_m = i > 0 || periodic, has_p = i < n - 1 || periodic;
            long qm = i > 0 ? q - s : q + (long)(n - 1) * s;
            long qp = i < n - 1 ? q + s : q - (long)(n - 1) * s;
            double b = has_m ? phi[q] - phi[qm] : 0.0;
            double f = has_p ? phi[qp] - phi[q] : 0.0;
            if (!has_m) b = f;
            if (!has_p) f = b;
            double d;
            if (f + b >= 0.0) d = b >= 0.0 ? b : 0.0;
            else d = f < 0.0 ? f : 0.0;
            d /= g->h[l];
            s2 += d * d;
        }
        gm[q] = sqrt(s2);
    }
}

/* zero normal gradient on every non-periodic face: (4 f_1 - f_2) / 3 */
static void levelset_faces(const wdo_grid *g, double *phi)
{
    long N = npoints(g);
    for (int l = 0; l < g->ndim; ++l) {
        if (g->bc[l][0] == WDO_PERIODIC) continue;
        long s = stride_of(g, l);
        for (long q = 0; q < N; ++q) {
            int idx[3];
            index_of(g, q, idx);
            if (idx[l] == 0) phi[q] = (4.0 * phi[q + s] - phi[q + 2 * s]) / 3.0;
            else if (idx[l] == g->n[l] - 1) phi[q] = (4.0 * phi[q - s] - phi[q - 2 * s]) / 3.0;
        }
    }
}

int wdo_levelset_advance(const wdo_grid *g, double speed, double dt, int nsteps, double *phi)
{
    if (!g->uniform || nsteps < 0) return -1;
    long N = npoints(g);
    double *k = malloc(sizeof(double) * N * 5);
    if (!k) return -2;
    double *k1 = k, *k2 = k + N, *k3 = k + 2 * N, *k4 = k + 3 * N, *st = k + 4 * N;
    for (int it = 0; it < nsteps; ++it) {
        /* classical RK4: k_j = -F |grad phi| at the stage values */
        levelset_grad(g, phi, k1);
        for (long q = 0; q < N; ++q) st[q] = phi[q] - 0.5 * dt * speed * k1[q];
        levelset_faces(g, st);
        levelset_grad(g, st, k2);
        for (long q = 0; q < N; ++q) st[q] = phi[q] - 0.5 * dt * speed * k2[q];
        levelset_faces(g, st);
        levelset_grad(g, st, k3);
        for (long q = 0; q < N; ++q) st[q] = phi[q] - dt * speed * k3[q];
        levelset_faces(g, st);
        levelset_grad(g, st, k4);
        for (long q = 0; q < N; ++q)
            phi[q] -= dt * speed * (k1[q] + 2.0 * k2[q] + 2.0 * k3[q] + k4[q]) / 6.0;
        levelset_faces(g, phi);
    }
    free(k);
    return 0;
}

/* crossing of the iso-value 0 on the edge from a (value va) to b (vb) */
static void edge_point(double xa, double ya, double va, double xb, double yb, double vb,
                       double *x, double *y)
{
    double t = va / (va - vb);
    *x = xa + t * (xb - xa);
    *y = ya + t * (yb - ya);
}

double wdo_level_length(const wdo_grid *g, const double *phi, double level)
{
    if (g->ndim != 2 || !g->uniform) return -1.0;
    int nx = g->n[0], ny = g->n[1];
    double hx = g->h[0], hy = g->h[1], total = 0.0;
    for (int j = 0; j + 1 < ny; ++j)
        for (int i = 0; i + 1 < nx; ++i) {
            /* corners counter-clockwise: (i,j) (i+1,j) (i+1,j+1) (i,j+1) */
            double v[4] = {phi[(long)j * nx + i] - level, phi[(long)j * nx + i + 1] - level,
                           phi[(long)(j + 1) * nx + i + 1] - level,
                           phi[(long)(j + 1) * nx + i] - level};
            double cx[4] = {0.0, hx, hx, 0.0}, cy[4] = {0.0, 0.0, hy, hy};
            double px[4], py[4];
            int np = 0, edge[4];
            for (int e = 0; e < 4; ++e) {
                int a = e, b = (e + 1) & 3;
                if ((v[a] >= 0.0) != (v[b] >= 0.0)) {
                    edge_point(cx[a], cy[a], v[a], cx[b], cy[b], v[b], &px[np], &py[np]);
                    edge[np++] = e;
                }
            }
            if (np == 2) {
                total += hypot(px[1] - px[0], py[1] - py[0]);
            } else if (np == 4) {
                /* saddle: the cell mean decides which corners connect */
                double mean = 0.25 * (v[0] + v[1] + v[2] + v[3]);
                int same = (mean >= 0.0) == (v[0] >= 0.0);
                /* crossings lie on edges 0,1,2,3 in order; corner 0 is cut
                   off with edges 3,0 when the centre differs from it */
                if (same) {
                    total += hypot(px[1] - px[0], py[1] - py[0]);   /* edges 0-1 */
                    total += hypot(px[3] - px[2], py[3] - py[2]);   /* edges 2-3 */
                } else {
                    total += hypot(px[3] - px[0], py[3] - py[0]);   /* edges 3-0 */
                    total += hypot(px[2] - px[1], py[2] - py[1]);   /* edges 1-2 */
                }
                (void)edge;
            }
        }
    return total;
}
