/*
 * fdlb_oracle.c -- plain FP64 CPU implementation of the fully discrete
 * finite-difference lattice Boltzmann scheme (Ghiroldi & Gibelli,
 * "A finite-difference lattice Boltzmann approach for gas microflows").
 *
 * TEST INFRASTRUCTURE ONLY.  Called by the test suite, the package's smoke
 * check and the benchmark's CPU-baseline leg; never by the GPU library, and
 * it includes nothing from it.
 *
 * What it computes, in the paper's order and notation:
 *   - populations f_alpha are the weighted values of Eq. (2), stored raw (not
 *     as deviations), layout f[alpha][y][x];
 *   - density and momentum are the sums of Eqs. (6)-(7);
 *   - the equilibrium is the linearised isothermal Maxwellian of Eq. (5) in
 *     weighted form, f_alpha^eq = w_alpha rho (1 + xi_alpha . u) (Eq. 3);
 *   - one time step is a first-order splitting of Eq. (1): an explicit-Euler
 *     relaxation  g = f - (dt/Kn)(f - f^eq)  followed by first-order upwind
 *     transport of xi_alpha . grad f_alpha (the paragraph that introduces the
 *     fully discrete scheme, just before the Couette problem is set up);
 *   - walls re-emit the populations that leave the wall (xi . n > 0, n the
 *     inward normal) as w_alpha rho_w (1 + xi_t u_w) (Eq. 8, weighted form),
 *     with rho_w from the impermeability sum of Eq. (9) over the populations
 *     that arrive at the wall (xi . n < 0), divided by the flux the emission
 *     carries per unit wall density.  For a half-range rule that flux is
 *     (2 pi)^(-1/2) and this is Eq. (9) as printed; for a full-range rule (the
 *     paper's standard lattice with walls) it keeps the wall impermeable.
 *
 * Readings where the paper is silent:
 *   grid: cell-centred cells, walls on the outer cell faces, the wall value
 *     acting as the upwind neighbour of the wall cell; rho_w taken from the
 *     wall cell's post-relaxation populations; relax then transport (the
 *     reverse order is available for the test that shows steady rho and u do
 *     not depend on it); unsplit two-dimensional donor cell.
 *
 * Build: gcc -O2 -fopenmp -ffp-contract=off (no FMA contraction).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

enum { WALL_BOTTOM = 0, WALL_TOP = 1, WALL_LEFT = 2, WALL_RIGHT = 3 };

typedef struct {
    int32_t nx, ny;             /* cells along x and y */
    int32_t periodic_x;         /* 1: x wraps; 0: walls at x = 0 and x = 1 */
    int32_t periodic_y;
    int32_t q;                  /* number of discrete velocities */
    int32_t order;              /* 0: relax then transport; 1: transport then relax */
    double wall_u[4];           /* tangential wall speed: bottom, top (along +x); left, right (along +y) */
    double dt, dx, dy;
    double omega;               /* dt / Kn (0 for free-molecular flow) */
    const double *xi_x, *xi_y, *w;
} oracle_problem;

#define IDX(P, a, x, y) (((size_t)(a) * (size_t)(P)->ny + (size_t)(y)) * (size_t)(P)->nx + (size_t)(x))

/* Eqs. (6)-(7): rho = sum f, rho u = sum xi f.  Output arrays of nx*ny, [y][x]. */
void oracle_moments(const oracle_problem *P, const double *f, double *rho, double *ux, double *uy)
{
    int y;
#pragma omp parallel for schedule(static)
    for (y = 0; y < P->ny; ++y) {
        for (int x = 0; x < P->nx; ++x) {
            double r = 0.0, jx = 0.0, jy = 0.0;
            for (int a = 0; a < P->q; ++a) {
                double fa = f[IDX(P, a, x, y)];
                r += fa;
                jx += P->xi_x[a] * fa;
                jy += P->xi_y[a] * fa;
            }
            size_t c = (size_t)y * P->nx + x;
            rho[c] = r;
            ux[c] = jx / r;
            uy[c] = jy / r;
        }
    }
}

/* Explicit-Euler relaxation of Eq. (1): g = f - omega (f - f^eq), with
 * f^eq_alpha = w_alpha rho (1 + xi_alpha . u) (Eqs. 3 and 5). */
static void relax(const oracle_problem *P, const double *f, double *g)
{
    int y;
#pragma omp parallel for schedule(static)
    for (y = 0; y < P->ny; ++y) {
        for (int x = 0; x < P->nx; ++x) {
            double r = 0.0, jx = 0.0, jy = 0.0;
            for (int a = 0; a < P->q; ++a) {
                double fa = f[IDX(P, a, x, y)];
                r += fa;
                jx += P->xi_x[a] * fa;
                jy += P->xi_y[a] * fa;
            }
            double ux = jx / r, uy = jy / r;
            for (int a = 0; a < P->q; ++a) {
                size_t i = IDX(P, a, x, y);
                double feq = P->w[a] * r * (1.0 + P->xi_x[a] * ux + P->xi_y[a] * uy);
                g[i] = f[i] - P->omega * (f[i] - feq);
            }
        }
    }
}

/* Component of xi_alpha along the inward normal of a wall, and along its tangent. */
static double xi_normal(const oracle_problem *P, int wall, int a)
{
    switch (wall) {
    case WALL_BOTTOM: return P->xi_y[a];
    case WALL_TOP: return -P->xi_y[a];
    case WALL_LEFT: return P->xi_x[a];
    default: return -P->xi_x[a];
    }
}

static double xi_tangent(const oracle_problem *P, int wall, int a)
{
    return (wall == WALL_BOTTOM || wall == WALL_TOP) ? P->xi_x[a] : P->xi_y[a];
}

/* The cell adjacent to face `pos` of a wall. */
static void wall_cell(const oracle_problem *P, int wall, int pos, int *x, int *y)
{
    switch (wall) {
    case WALL_BOTTOM: *x = pos; *y = 0; break;
    case WALL_TOP: *x = pos; *y = P->ny - 1; break;
    case WALL_LEFT: *x = 0; *y = pos; break;
    default: *x = P->nx - 1; *y = pos; break;
    }
}

static int wall_len(const oracle_problem *P, int wall)
{
    return (wall == WALL_BOTTOM || wall == WALL_TOP) ? P->nx : P->ny;
}

static int wall_active(const oracle_problem *P, int wall)
{
    return (wall == WALL_BOTTOM || wall == WALL_TOP) ? !P->periodic_y : !P->periodic_x;
}

/* Flux leaving a wall per unit wall density under Eq. (8): sum over xi.n > 0 of (xi.n) w_alpha.
 * (The factor 1 + xi_t u_w adds nothing: the tangential rule is symmetric.)  A half-range rule
 * integrates xi over the half-line exactly, so there it is (2 pi)^(-1/2). */
static double emitted_flux(const oracle_problem *P, int wall)
{
    double s = 0.0;
    for (int a = 0; a < P->q; ++a) {
        double xn = xi_normal(P, wall, a);
        if (xn > 0.0) s += xn * P->w[a];
    }
    return s;
}

/* Eq. (9) for a general wall, read as the impermeability condition: the wall density whose
 * emission carries away exactly the flux that arrives,
 *   rho_w = -sum_{xi.n<0} (xi.n) g_alpha / sum_{xi.n>0} (xi.n) w_alpha,
 * which is -(2 pi)^(1/2) sum_{xi.n<0} (xi.n) g_alpha for a half-range rule. */
static double wall_density(const oracle_problem *P, const double *g, int wall, int pos)
{
    int x, y;
    wall_cell(P, wall, pos, &x, &y);
    double s = 0.0;
    for (int a = 0; a < P->q; ++a) {
        double xn = xi_normal(P, wall, a);
        if (xn < 0.0) s += xn * g[IDX(P, a, x, y)];
    }
    return -s / emitted_flux(P, wall);
}

/* Eq. (8), weighted form: populations leaving the wall are w_alpha rho_w (1 + xi_t u_w). */
static double wall_emission(const oracle_problem *P, int wall, double rho_w, int a)
{
    return P->w[a] * rho_w * (1.0 + xi_tangent(P, wall, a) * P->wall_u[wall]);
}

/* Wall densities of all four walls, rhow[wall * L + pos] with L = max(nx, ny). */
static void all_wall_densities(const oracle_problem *P, const double *g, double *rhow)
{
    int L = P->nx > P->ny ? P->nx : P->ny;
    for (int wall = 0; wall < 4; ++wall) {
        if (!wall_active(P, wall)) continue;
        for (int pos = 0; pos < wall_len(P, wall); ++pos)
            rhow[wall * L + pos] = wall_density(P, g, wall, pos);
    }
}

/* Value of population a at the upwind neighbour of cell (x, y) along one axis:
 * the neighbour cell, its periodic image, or the wall emission on the face. */
static double upwind_x(const oracle_problem *P, const double *g, const double *rhow, int a, int x, int y)
{
    int L = P->nx > P->ny ? P->nx : P->ny;
    double cx = P->xi_x[a];
    if (cx > 0.0) {
        if (x > 0) return g[IDX(P, a, x - 1, y)];
        if (P->periodic_x) return g[IDX(P, a, P->nx - 1, y)];
        return wall_emission(P, WALL_LEFT, rhow[WALL_LEFT * L + y], a);
    }
    if (cx < 0.0) {
        if (x < P->nx - 1) return g[IDX(P, a, x + 1, y)];
        if (P->periodic_x) return g[IDX(P, a, 0, y)];
        return wall_emission(P, WALL_RIGHT, rhow[WALL_RIGHT * L + y], a);
    }
    return g[IDX(P, a, x, y)];
}

static double upwind_y(const oracle_problem *P, const double *g, const double *rhow, int a, int x, int y)
{
    int L = P->nx > P->ny ? P->nx : P->ny;
    double cy = P->xi_y[a];
    if (cy > 0.0) {
        if (y > 0) return g[IDX(P, a, x, y - 1)];
        if (P->periodic_y) return g[IDX(P, a, x, P->ny - 1)];
        return wall_emission(P, WALL_BOTTOM, rhow[WALL_BOTTOM * L + x], a);
    }
    if (cy < 0.0) {
        if (y < P->ny - 1) return g[IDX(P, a, x, y + 1)];
        if (P->periodic_y) return g[IDX(P, a, x, 0)];
        return wall_emission(P, WALL_TOP, rhow[WALL_TOP * L + x], a);
    }
    return g[IDX(P, a, x, y)];
}

/* First-order upwind (donor-cell) transport over one time step:
 * f_new = g - nu_x (g - g_upwind_x) - nu_y (g - g_upwind_y), nu = dt |xi| / dx. */
static void transport(const oracle_problem *P, const double *g, double *fnew, double *rhow)
{
    all_wall_densities(P, g, rhow);
    int y;
#pragma omp parallel for schedule(static)
    for (y = 0; y < P->ny; ++y) {
        for (int a = 0; a < P->q; ++a) {
            double nux = P->dt * fabs(P->xi_x[a]) / P->dx;
            double nuy = P->dt * fabs(P->xi_y[a]) / P->dy;
            for (int x = 0; x < P->nx; ++x) {
                size_t i = IDX(P, a, x, y);
                double gc = g[i];
                double gx = upwind_x(P, g, rhow, a, x, y);
                double gy = upwind_y(P, g, rhow, a, x, y);
                fnew[i] = gc - nux * (gc - gx) - nuy * (gc - gy);
            }
        }
    }
}

size_t oracle_work_doubles(const oracle_problem *P)
{
    size_t n = (size_t)P->q * P->nx * P->ny;
    size_t L = P->nx > P->ny ? P->nx : P->ny;
    return n + 4 * L;
}

/* One time step f -> fnew.  work must hold oracle_work_doubles() doubles. */
void oracle_step(const oracle_problem *P, const double *f, double *fnew, double *work)
{
    size_t n = (size_t)P->q * P->nx * P->ny;
    double *g = work, *rhow = work + n;
    if (P->order == 0) {
        relax(P, f, g);
        transport(P, g, fnew, rhow);
    } else {
        transport(P, f, g, rhow);
        relax(P, g, fnew);
    }
}

/* Per-step change of the velocity field: R = ||u_new - u_old||_2 / ||u_new||_2 over all cells. */
static double residual(int ncell, const double *ux0, const double *uy0, const double *ux1, const double *uy1)
{
    double num = 0.0, den = 0.0;
    for (int c = 0; c < ncell; ++c) {
        double dx = ux1[c] - ux0[c], dy = uy1[c] - uy0[c];
        num += dx * dx + dy * dy;
        den += ux1[c] * ux1[c] + uy1[c] * uy1[c];
    }
    if (den > 0.0) return sqrt(num / den);
    return num > 0.0 ? INFINITY : 0.0;
}

/*
 * March f (in place) for at most max_steps steps.  If tol > 0, stop after the
 * first step whose residual is below tol.  res_hist (may be NULL) receives the
 * residual of every step taken.  Returns the number of steps taken, or -1 on
 * allocation failure.
 */
int64_t oracle_solve(const oracle_problem *P, double *f, int64_t max_steps, double tol, double *res_hist)
{
    size_t n = (size_t)P->q * P->nx * P->ny;
    int ncell = P->nx * P->ny;
    double *fn = malloc(n * sizeof(double));
    double *work = malloc(oracle_work_doubles(P) * sizeof(double));
    double *m = malloc((size_t)6 * ncell * sizeof(double));
    if (!fn || !work || !m) {
        free(fn); free(work); free(m);
        return -1;
    }
    double *rho = m, *ux0 = m + ncell, *uy0 = m + 2 * ncell, *ux1 = m + 3 * ncell, *uy1 = m + 4 * ncell;
    oracle_moments(P, f, rho, ux0, uy0);
    int64_t s = 0;
    double *cur = f, *nxt = fn;
    while (s < max_steps) {
        oracle_step(P, cur, nxt, work);
        ++s;
        oracle_moments(P, nxt, rho, ux1, uy1);
        double R = residual(ncell, ux0, uy0, ux1, uy1);
        if (res_hist) res_hist[s - 1] = R;
        double *t = cur; cur = nxt; nxt = t;
        memcpy(ux0, ux1, ncell * sizeof(double));
        memcpy(uy0, uy1, ncell * sizeof(double));
        if (tol > 0.0 && R < tol) break;
    }
    if (cur != f) memcpy(f, cur, n * sizeof(double));
    free(fn); free(work); free(m);
    return s;
}

/* xy stress of the post-relaxation state per cell: p_xy = sum xi_x xi_y g. */
void oracle_pxy(const oracle_problem *P, const double *f, double *pxy)
{
    size_t n = (size_t)P->q * P->nx * P->ny;
    double *g = malloc(n * sizeof(double));
    if (!g) return;
    relax(P, f, g);
    for (int y = 0; y < P->ny; ++y)
        for (int x = 0; x < P->nx; ++x) {
            double s = 0.0;
            for (int a = 0; a < P->q; ++a) s += P->xi_x[a] * P->xi_y[a] * g[IDX(P, a, x, y)];
            pxy[(size_t)y * P->nx + x] = s;
        }
    free(g);
}

/*
 * State on the faces of one wall after relaxation: populations arriving at
 * the wall (xi . n < 0) and those moving along it (xi . n = 0) carry the wall
 * cell's value, those leaving it carry the emission of Eq. (8).  Per face:
 * density, tangential velocity and xy stress.  Returns 0, or -1 if the wall
 * is not present (periodic axis) or on allocation failure.
 */
int oracle_wall_profile(const oracle_problem *P, const double *f, int wall, double *rho_face,
                        double *u_t, double *pxy_face)
{
    if (wall < 0 || wall > 3 || !wall_active(P, wall)) return -1;
    size_t n = (size_t)P->q * P->nx * P->ny;
    double *g = malloc(n * sizeof(double));
    if (!g) return -1;
    relax(P, f, g);
    for (int pos = 0; pos < wall_len(P, wall); ++pos) {
        int x, y;
        wall_cell(P, wall, pos, &x, &y);
        double rw = wall_density(P, g, wall, pos);
        double r = 0.0, jt = 0.0, pxy = 0.0;
        for (int a = 0; a < P->q; ++a) {
            double gf = xi_normal(P, wall, a) > 0.0 ? wall_emission(P, wall, rw, a) : g[IDX(P, a, x, y)];
            r += gf;
            jt += xi_tangent(P, wall, a) * gf;
            pxy += P->xi_x[a] * P->xi_y[a] * gf;
        }
        rho_face[pos] = r;
        u_t[pos] = jt / r;
        pxy_face[pos] = pxy;
    }
    free(g);
    return 0;
}

/* Equilibrium state f_alpha = w_alpha rho (1 + xi_alpha . u) (Eqs. 3 and 5) from cell fields. */
void oracle_equilibrium(const oracle_problem *P, const double *rho, const double *ux, const double *uy,
                        double *f)
{
    for (int a = 0; a < P->q; ++a)
        for (int y = 0; y < P->ny; ++y)
            for (int x = 0; x < P->nx; ++x) {
                size_t c = (size_t)y * P->nx + x;
                f[IDX(P, a, x, y)] = P->w[a] * rho[c] * (1.0 + P->xi_x[a] * ux[c] + P->xi_y[a] * uy[c]);
            }
}

int oracle_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Threads of the parallel loops from now on (at least 1); returns the number in effect. */
int oracle_set_threads(int n)
{
#ifdef _OPENMP
    omp_set_num_threads(n > 0 ? n : 1);
    return omp_get_max_threads();
#else
    (void)n;
    return 1;
#endif
}
