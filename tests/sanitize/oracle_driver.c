/* Driver for the sanitizer build of the FP64 oracle (test infrastructure,
 * CPU only).  oracle/nlse_oracle.c is compiled with AddressSanitizer and
 * UndefinedBehaviorSanitizer (serially, without OpenMP) and every entry point
 * runs on the smallest and on ragged grids of 1, 2 and 3 dimensions, both
 * schemes, all three boundary conditions, with and without a potential,
 * plus the argument checks.  A sanitizer report aborts the program. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

double orc_dt_max(int ndim, int order, double h, double a);
int orc_rhs(int ndim, const long *n, double h, double a, double s, const double *V, int order, int bc,
            const double *psi, double *F);
int orc_laplacian(int ndim, const long *n, double h, double a, double s, const double *V, int order, int bc,
                  const double *psi, double *L);
int orc_rk4(int ndim, const long *n, double h, double a, double s, const double *V, int order, int bc, double dt,
            long nsteps, double *psi);
int orc_mass_energy(int ndim, const long *n, double h, double a, double s, const double *V, int order, int bc,
                    const double *psi, double *out);

static int failures = 0;
#define EXPECT(c)                                          \
    do {                                                   \
        if (!(c)) {                                        \
            fprintf(stderr, "line %d: %s\n", __LINE__, #c); \
            ++failures;                                    \
        }                                                  \
    } while (0)

int main(void)
{
    const long shapes[][3] = {{3, 1, 1},  {5, 1, 1},  {37, 1, 1}, {3, 3, 1},
                              {9, 5, 1},  {17, 4, 1}, {3, 3, 3},  {6, 5, 4}};
    const int dims[] = {1, 1, 1, 2, 2, 2, 3, 3};
    for (int k = 0; k < 8; ++k) {
        const long *n = shapes[k];
        const long npts = n[0] * n[1] * n[2];
        double *psi = malloc(2 * npts * sizeof(double));
        double *out = malloc(2 * npts * sizeof(double));
        double *V = malloc(npts * sizeof(double));
        for (long p = 0; p < npts; ++p) {
            psi[2 * p] = 1.0 + 0.1 * sin(0.7 * p);
            psi[2 * p + 1] = 0.2 * cos(1.3 * p);
            V[p] = 0.05 * p / (double)npts;
        }
        for (int order = 2; order <= 4; order += 2)
            for (int bc = 0; bc < 3; ++bc)
                for (int withv = 0; withv < 2; ++withv) {
                    const double *v = withv ? V : NULL;
                    double me[3];
                    EXPECT(orc_rhs(dims[k], n, 0.3, 0.7, -0.9, v, order, bc, psi, out) == 0);
                    EXPECT(orc_laplacian(dims[k], n, 0.3, 0.7, -0.9, v, order, bc, psi, out) == 0);
                    EXPECT(orc_mass_energy(dims[k], n, 0.3, 0.7, -0.9, v, order, bc, psi, me) == 0);
                    for (long p = 0; p < 2 * npts; ++p) out[p] = psi[p];
                    const double dt = 0.5 * orc_dt_max(dims[k], order, 0.3, 0.7);
                    EXPECT(orc_rk4(dims[k], n, 0.3, 0.7, -0.9, v, order, bc, dt, 3, out) == 0);
                    for (long p = 0; p < 2 * npts; ++p) EXPECT(isfinite(out[p]));
                }
        /* argument checks */
        EXPECT(orc_rhs(dims[k], n, 0.3, 0.7, -0.9, NULL, 3, 0, psi, out) != 0);
        EXPECT(orc_rhs(dims[k], n, 0.3, 0.7, -0.9, NULL, 2, 5, psi, out) != 0);
        free(psi);
        free(out);
        free(V);
    }
    const long bad[3] = {2, 1, 1};
    double x[8] = {0}, y[8] = {0};
    EXPECT(orc_rhs(1, bad, 0.3, 0.7, -0.9, NULL, 2, 0, x, y) != 0);
    EXPECT(orc_rhs(0, bad, 0.3, 0.7, -0.9, NULL, 2, 0, x, y) != 0);
    if (failures) {
        fprintf(stderr, "%d failed checks\n", failures);
        return 1;
    }
    printf("sanitized oracle checks passed\n");
    return 0;
}
