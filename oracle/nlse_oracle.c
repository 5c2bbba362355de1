/*
 * FP64 CPU oracle for the NLSEmagic integrator (Caplan, arXiv:1203.1263).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow reference that the
 * GPU library is checked against.  Only the test suite, the smoke check and
 * the CPU-baseline leg of the benchmark may load it; the product path never
 * does.  It shares no code, header or constant with the GPU library.
 *
 * What it computes (all in double precision, no FMA contraction; the build
 * passes -ffp-contract=off):
 *   - the right-hand side F(Psi) = i [ a Lap(Psi) + (s|Psi|^2 - V) Psi ]
 *     (Sec. "Fourth-order Runge-Kutta", definition of F under Eq. RK4);
 *   - the Laplacian by CD2 (step 1 of Eqs. 2shoc1d / 2d2shocs1 / 3d2shocs) or
 *     by the two-step compact scheme 2SHOC (Eqs. 2shoc1d2 / 2d2shocs2 /
 *     3d2shocs2), where step 1 stores D and step 2 combines D and Psi;
 *   - boundary conditions (Sec. "Boundary conditions"): Dirichlet, time form
 *     Eq. BCDdt and Laplacian form Eq. BCDlap; modulus-squared Dirichlet (MSD),
 *     time form Eq. msd and Laplacian form Eq. BCMSDlap; Laplacian-zero (L0),
 *     time form Eq. BCL0dt and Laplacian form Eq. BCL0lap;
 *   - classic RK4 (Eq. RK4) with its four slopes k_1..k_4 and weights
 *     1/6, 1/3, 1/3, 1/6;
 *   - the linear stability bounds, Eqs. stblincd and stblin2shoc;
 *   - discrete mass and energy (the paper defines neither; the standard NLSE
 *     invariants are used, see orc_mass_energy).
 *
 * Readings where the paper is silent:
 *   - grid points include both end points and every point with an index equal
 *     to 0 or N_d-1 on an active axis is a boundary point;
 *   - the MSD "interior neighbour" b-1 of a boundary point b is the point one
 *     step inward along every axis on which b lies on the boundary (a corner
 *     takes the diagonal interior point);
 *   - in the MSD formulas a ratio over a neighbour with |Psi_q|^2 == 0 is
 *     taken as 0;
 *   - the Dirichlet time form freezes whatever (complex) boundary value is
 *     given; B is not enforced separately.
 *
 * Layout: complex values are interleaved (re, im) doubles; the linear index is
 * x + Nx*(y + Ny*z); unused dimensions have extent 1.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#define ORC_BC_DIRICHLET 0
#define ORC_BC_MSD 1
#define ORC_BC_L0 2

#define ORC_OK 0
#define ORC_EINVAL -1
#define ORC_ENOMEM -2

typedef struct {
    int ndim;
    long n[3];
    long stride[3];
    long npts;
    double h, a, s;
    const double *V; /* real, may be NULL (V == 0) */
} grid_t;

static int grid_init(grid_t *g, int ndim, const long *n, double h, double a,
                     double s, const double *V)
{
    if (ndim < 1 || ndim > 3 || !(h > 0) || !(a > 0)) return ORC_EINVAL;
    g->ndim = ndim;
    for (int d = 0; d < 3; ++d) g->n[d] = 1;
    for (int d = 0; d < ndim; ++d) {
        if (n[d] < 3) return ORC_EINVAL;
        g->n[d] = n[d];
    }
    g->stride[0] = 1;
    g->stride[1] = g->n[0];
    g->stride[2] = g->n[0] * g->n[1];
    g->npts = g->n[0] * g->n[1] * g->n[2];
    g->h = h;
    g->a = a;
    g->s = s;
    g->V = V;
    return ORC_OK;
}

static void coords(const grid_t *g, long p, long c[3])
{
    c[0] = p % g->n[0];
    c[1] = (p / g->n[0]) % g->n[1];
    c[2] = p / (g->n[0] * g->n[1]);
}

/* A point is on the boundary if any active coordinate is 0 or N_d-1. */
static int is_boundary(const grid_t *g, const long c[3])
{
    for (int d = 0; d < g->ndim; ++d)
        if (c[d] == 0 || c[d] == g->n[d] - 1) return 1;
    return 0;
}

/* MSD interior neighbour: one step inward on every boundary axis. */
static long inward(const grid_t *g, const long c[3])
{
    long q[3] = {c[0], c[1], c[2]};
    for (int d = 0; d < g->ndim; ++d) {
        if (c[d] == 0) q[d] = 1;
        else if (c[d] == g->n[d] - 1) q[d] = g->n[d] - 2;
    }
    return q[0] + g->n[0] * (q[1] + g->n[1] * q[2]);
}

static double vpot(const grid_t *g, long p) { return g->V ? g->V[p] : 0.0; }

/* N = s|Psi|^2 - V, the nonlinear-plus-potential factor of Eqs. BCMSDlap / nbnb1. */
static double nl(const grid_t *g, const double *psi, long p)
{
    double re = psi[2 * p], im = psi[2 * p + 1];
    return g->s * (re * re + im * im) - vpot(g, p);
}

/* Re(z / w) with the zero-denominator reading. */
static double re_ratio(double zr, double zi, double wr, double wi)
{
    double m = wr * wr + wi * wi;
    if (m == 0.0) return 0.0;
    return (zr * wr + zi * wi) / m;
}

/* Im(z / w) with the zero-denominator reading. */
static double im_ratio(double zr, double zi, double wr, double wi)
{
    double m = wr * wr + wi * wi;
    if (m == 0.0) return 0.0;
    return (zi * wr - zr * wi) / m;
}

/* CD2 Laplacian at an interior point: sum over axes of
 * (Psi_{+e} - 2 Psi + Psi_{-e}) / h^2 (step 1 of the 2SHOC equations, which
 * the paper also names as the standard central difference). */
static void cd2_at(const grid_t *g, const double *u, long p, double out[2])
{
    double h2 = g->h * g->h;
    for (int k = 0; k < 2; ++k) {
        double acc = 0.0;
        for (int d = 0; d < g->ndim; ++d) {
            long st = g->stride[d];
            acc += u[2 * (p + st) + k] - 2.0 * u[2 * p + k] + u[2 * (p - st) + k];
        }
        out[k] = acc / h2;
    }
}

/* 2SHOC step 1 over the whole grid: D = CD2 at interior points, and at
 * boundary points the Laplacian form of the boundary condition:
 *   Dirichlet (Eq. BCDlap): D_b = -(1/a) N_b Psi_b
 *   MSD (Eq. BCMSDlap):     D_b = [ Re(D_q / Psi_q) + (N_q - N_b)/a ] Psi_b,
 *   L0 (Eq. BCL0lap):       D_b = 0,
 * where Im(i z) = Re(z) and D_q is the interior CD2 value at q. */
static void compute_D(const grid_t *g, int bc, const double *u, double *D)
{
    long np = g->npts;
#pragma omp parallel for schedule(static)
    for (long p = 0; p < np; ++p) {
        long c[3];
        coords(g, p, c);
        if (!is_boundary(g, c)) cd2_at(g, u, p, &D[2 * p]);
    }
#pragma omp parallel for schedule(static)
    for (long p = 0; p < np; ++p) {
        long c[3];
        coords(g, p, c);
        if (!is_boundary(g, c)) continue;
        double ur = u[2 * p], ui = u[2 * p + 1];
        double Nb = nl(g, u, p);
        if (bc == ORC_BC_DIRICHLET) {
            D[2 * p] = -(1.0 / g->a) * Nb * ur;
            D[2 * p + 1] = -(1.0 / g->a) * Nb * ui;
        } else if (bc == ORC_BC_L0) {
            D[2 * p] = 0.0;
            D[2 * p + 1] = 0.0;
        } else {
            long q = inward(g, c);
            double Dq[2];
            cd2_at(g, u, q, Dq);
            double fac = re_ratio(Dq[0], Dq[1], u[2 * q], u[2 * q + 1]) +
                         (nl(g, u, q) - Nb) / g->a;
            D[2 * p] = fac * ur;
            D[2 * p + 1] = fac * ui;
        }
    }
}

/* 2SHOC step 2 at an interior point.
 *  1D (Eq. 2shoc1d2): L = (7/6) D_i - (D_{i+1} + D_{i-1}) / 12
 *  2D (Eq. 2d2shocs2): L = -(1/12)[ sum of the 4 face D - 12 D ]
 *                          + (1/(6h^2)) [ sum of the 4 corner Psi - 4 Psi ]
 *  3D (Eq. 3d2shocs2): L = -(1/12)[ sum of the 6 face D - 10 D ]
 *                          + (1/(6h^2)) [ sum of the 12 edge Psi - 12 Psi ]
 * The 3D edge points are the in-plane corners of each of the three
 * coordinate planes through the point. */
static void shoc_at(const grid_t *g, const double *u, const double *D, long p,
                    double out[2])
{
    double h2 = g->h * g->h;
    for (int k = 0; k < 2; ++k) {
        if (g->ndim == 1) {
            out[k] = (7.0 / 6.0) * D[2 * p + k] -
                     (D[2 * (p + 1) + k] + D[2 * (p - 1) + k]) / 12.0;
            continue;
        }
        double faces = 0.0;
        for (int d = 0; d < g->ndim; ++d) {
            long st = g->stride[d];
            faces += D[2 * (p + st) + k] + D[2 * (p - st) + k];
        }
        double edges = 0.0;
        for (int d1 = 0; d1 < g->ndim; ++d1)
            for (int d2 = d1 + 1; d2 < g->ndim; ++d2) {
                long s1 = g->stride[d1], s2 = g->stride[d2];
                edges += u[2 * (p + s1 + s2) + k] + u[2 * (p + s1 - s2) + k] +
                         u[2 * (p - s1 + s2) + k] + u[2 * (p - s1 - s2) + k];
            }
        double cD = (g->ndim == 2) ? 12.0 : 10.0;
        double cU = (g->ndim == 2) ? 4.0 : 12.0;
        out[k] = -(1.0 / 12.0) * (faces - cD * D[2 * p + k]) +
                 (1.0 / (6.0 * h2)) * (edges - cU * u[2 * p + k]);
    }
}

/* Laplacian at every interior point (boundary entries are left as zero; they
 * are never used because F at boundary points comes from the boundary
 * condition, and 2SHOC at the first interior layer reads the boundary D). */
static void compute_L(const grid_t *g, int order, int bc, const double *u,
                      double *L, double *D)
{
    long np = g->npts;
    if (order == 4) compute_D(g, bc, u, D);
#pragma omp parallel for schedule(static)
    for (long p = 0; p < np; ++p) {
        long c[3];
        coords(g, p, c);
        if (is_boundary(g, c)) {
            L[2 * p] = 0.0;
            L[2 * p + 1] = 0.0;
        } else if (order == 2) {
            cd2_at(g, u, p, &L[2 * p]);
        } else {
            shoc_at(g, u, D, p, &L[2 * p]);
        }
    }
}

/* F(Psi) = i [ a L + N Psi ] at interior points (definition under Eq. RK4;
 * split form Eq. fsplit).  Boundary points:
 *   Dirichlet (Eq. BCDdt): F_b = 0
 *   MSD (Eq. msd):         F_b = i Im(F_q / Psi_q) Psi_b
 *   L0 (Eq. BCL0dt):       F_b = i N_b Psi_b. */
static void compute_F(const grid_t *g, int order, int bc, const double *u,
                      double *F, double *L, double *D)
{
    long np = g->npts;
    compute_L(g, order, bc, u, L, D);
#pragma omp parallel for schedule(static)
    for (long p = 0; p < np; ++p) {
        long c[3];
        coords(g, p, c);
        if (is_boundary(g, c)) continue;
        double ur = u[2 * p], ui = u[2 * p + 1];
        double N = nl(g, u, p);
        double wr = g->a * L[2 * p] + N * ur; /* w = a L + N Psi */
        double wi = g->a * L[2 * p + 1] + N * ui;
        F[2 * p] = -wi; /* i * w */
        F[2 * p + 1] = wr;
    }
#pragma omp parallel for schedule(static)
    for (long p = 0; p < np; ++p) {
        long c[3];
        coords(g, p, c);
        if (!is_boundary(g, c)) continue;
        if (bc == ORC_BC_DIRICHLET) {
            F[2 * p] = 0.0;
            F[2 * p + 1] = 0.0;
        } else if (bc == ORC_BC_L0) {
            double Nb = nl(g, u, p);
            F[2 * p] = -Nb * u[2 * p + 1]; /* i * N_b * Psi_b */
            F[2 * p + 1] = Nb * u[2 * p];
        } else {
            long q = inward(g, c);
            double w = im_ratio(F[2 * q], F[2 * q + 1], u[2 * q], u[2 * q + 1]);
            /* i * w * Psi_b */
            F[2 * p] = -w * u[2 * p + 1];
            F[2 * p + 1] = w * u[2 * p];
        }
    }
}

static int check_scheme(int order, int bc)
{
    if (order != 2 && order != 4) return ORC_EINVAL;
    if (bc != ORC_BC_DIRICHLET && bc != ORC_BC_MSD && bc != ORC_BC_L0) return ORC_EINVAL;
    return ORC_OK;
}

/* ---------------------------------------------------------------- exports */

/* Linear stability bound of RK4+CD (Eq. stblincd) and RK4+2SHOC
 * (Eq. stblin2shoc): k < h^2 / (d sqrt(2) a), times 3/4 for 2SHOC. */
double orc_dt_max(int ndim, int order, double h, double a)
{
    double k = h * h / ((double)ndim * sqrt(2.0) * a);
    if (order == 4) k *= 0.75;
    return k;
}

/* Right-hand side F(psi) on the whole grid. */
int orc_rhs(int ndim, const long *n, double h, double a, double s,
            const double *V, int order, int bc, const double *psi, double *F)
{
    grid_t g;
    int rc = grid_init(&g, ndim, n, h, a, s, V);
    if (rc) return rc;
    if ((rc = check_scheme(order, bc))) return rc;
    double *L = calloc(2 * g.npts, sizeof(double));
    double *D = calloc(2 * g.npts, sizeof(double));
    if (!L || !D) {
        free(L);
        free(D);
        return ORC_ENOMEM;
    }
    compute_F(&g, order, bc, psi, F, L, D);
    free(L);
    free(D);
    return ORC_OK;
}

/* Scheme Laplacian at interior points (boundary entries 0). */
int orc_laplacian(int ndim, const long *n, double h, double a, double s,
                  const double *V, int order, int bc, const double *psi,
                  double *L)
{
    grid_t g;
    int rc = grid_init(&g, ndim, n, h, a, s, V);
    if (rc) return rc;
    if ((rc = check_scheme(order, bc))) return rc;
    double *D = calloc(2 * g.npts, sizeof(double));
    if (!D) return ORC_ENOMEM;
    compute_L(&g, order, bc, psi, L, D);
    free(D);
    return ORC_OK;
}

/* nsteps of the classic fourth-order Runge-Kutta method (Sec. "Fourth-order
 * Runge-Kutta", Eq. RK4), in place, written with its four slopes:
 *   k_1 = F(Psi),  k_2 = F(Psi + (dt/2) k_1),  k_3 = F(Psi + (dt/2) k_2),
 *   k_4 = F(Psi + dt k_3),  Psi <- Psi + (dt/6)(k_1 + 2 k_2 + 2 k_3 + k_4).
 * Each slope is a full-grid evaluation of F with its boundary forms; the
 * argument of the next slope is formed from the unchanged Psi. */
int orc_rk4(int ndim, const long *n, double h, double a, double s,
            const double *V, int order, int bc, double dt, long nsteps,
            double *psi)
{
    grid_t g;
    int rc = grid_init(&g, ndim, n, h, a, s, V);
    if (rc) return rc;
    if ((rc = check_scheme(order, bc))) return rc;
    if (!(dt > 0) || nsteps < 0) return ORC_EINVAL;
    long m = 2 * g.npts;
    /* stage offsets c_2..c_4 of the Butcher tableau, as fractions of dt */
    const double c[4] = {0.0, 0.5, 0.5, 1.0};
    double *k[4] = {NULL, NULL, NULL, NULL};
    double *arg = calloc(m, sizeof(double));
    double *L = calloc(m, sizeof(double));
    double *D = calloc(m, sizeof(double));
    int ok = arg && L && D;
    for (int j = 0; j < 4; ++j) {
        k[j] = calloc(m, sizeof(double));
        ok = ok && k[j];
    }
    if (!ok) {
        for (int j = 0; j < 4; ++j) free(k[j]);
        free(arg); free(L); free(D);
        return ORC_ENOMEM;
    }
    for (long it = 0; it < nsteps; ++it) {
        compute_F(&g, order, bc, psi, k[0], L, D);
        for (int j = 1; j < 4; ++j) {
            const double *prev = k[j - 1];
            const double step = c[j] * dt;
#pragma omp parallel for schedule(static)
            for (long i = 0; i < m; ++i) arg[i] = psi[i] + step * prev[i];
            compute_F(&g, order, bc, arg, k[j], L, D);
        }
#pragma omp parallel for schedule(static)
        for (long i = 0; i < m; ++i) {
            double slope = k[0][i] + 2.0 * k[1][i] + 2.0 * k[2][i] + k[3][i];
            psi[i] = psi[i] + (dt / 6.0) * slope;
        }
    }
    for (int j = 0; j < 4; ++j) free(k[j]);
    free(arg); free(L); free(D);
    return ORC_OK;
}

/* Discrete mass and energy (not defined in the paper; standard NLSE
 * invariants).  For i Psi_t = -a Lap Psi + V Psi - s|Psi|^2 Psi the
 * Hamiltonian is H = int a|grad Psi|^2 + V|Psi|^2 - (s/2)|Psi|^4, and after
 * summation by parts the kinetic term is -a Re(conj(Psi) Lap Psi):
 *   M = h^d sum_all |Psi|^2
 *   E = h^d [ sum_interior -a Re(conj(Psi) L_h Psi)
 *             + sum_all ( V|Psi|^2 - (s/2)|Psi|^4 ) ]
 * with L_h the scheme Laplacian of the given order (2SHOC reading the
 * boundary D of the given boundary condition).  Sums run serially in index
 * order. */
int orc_mass_energy(int ndim, const long *n, double h, double a, double s,
                    const double *V, int order, int bc, const double *psi,
                    double *out)
{
    grid_t g;
    int rc = grid_init(&g, ndim, n, h, a, s, V);
    if (rc) return rc;
    if ((rc = check_scheme(order, bc))) return rc;
    double *L = calloc(2 * g.npts, sizeof(double));
    double *D = calloc(2 * g.npts, sizeof(double));
    if (!L || !D) {
        free(L);
        free(D);
        return ORC_ENOMEM;
    }
    compute_L(&g, order, bc, psi, L, D);
    double hd = pow(g.h, (double)g.ndim);
    double mass = 0.0, kin = 0.0, pot = 0.0;
    for (long p = 0; p < g.npts; ++p) {
        long c[3];
        coords(&g, p, c);
        double re = psi[2 * p], im = psi[2 * p + 1];
        double rho = re * re + im * im;
        mass += rho;
        pot += vpot(&g, p) * rho - 0.5 * g.s * rho * rho;
        if (!is_boundary(&g, c)) kin += -g.a * (re * L[2 * p] + im * L[2 * p + 1]);
    }
    out[0] = hd * mass;
    out[1] = hd * (kin + pot);
    free(L);
    free(D);
    return ORC_OK;
}
