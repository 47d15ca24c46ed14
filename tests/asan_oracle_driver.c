/*
 * The C oracle under AddressSanitizer and UndefinedBehaviorSanitizer (TEST
 * INFRASTRUCTURE: built with gcc by tests/test_host_sanitizers.py together with
 * oracle/lbm_oracle.c).  Full steps (spread -> collide -> interpolate ->
 * propagate -> advance) on small non-cubic periodic grids, with points near and
 * beyond the periodic seams and negative coordinates, then the moments and an
 * equilibrium; checks the exact mass conservation of the method on the way.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

void orc_spread(int nx, int ny, int nz, int64_t n, const double* pos, const double* frc, int zero_net, double* g);
void orc_collide(int nx, int ny, int nz, double rho0, double tau, const double* df, const double* g, double* out,
                 double* rho, double* u);
void orc_stream(int nx, int ny, int nz, const double* dfstar, double* df);
void orc_moments(int nx, int ny, int nz, double rho0, const double* df, const double* g, double* rho, double* u);
void orc_interp(int nx, int ny, int nz, const double* u, int64_t n, const double* pos, double* U);
void orc_advect(int nx, int ny, int nz, double rho0, double tau, int64_t n, double* pos, const double* frc,
                const double* U, const double* inv_a, const double* inv_aL);
void orc_equilibrium(int nx, int ny, int nz, double rho0, const double* rho, const double* u, double* df);

static double frand(unsigned* s)
{
    *s = *s * 1664525u + 1013904223u;
    return (*s >> 8) / 16777216.0;
}

static int run(int nx, int ny, int nz, int npts, int steps, unsigned seed)
{
    const int64_t N = (int64_t)nx * ny * nz;
    double* df = calloc(19 * N, sizeof(double));
    double* dfs = calloc(19 * N, sizeof(double));
    double* g = calloc(3 * N, sizeof(double));
    double* rho = calloc(N, sizeof(double));
    double* u = calloc(3 * N, sizeof(double));
    double* pos = malloc(3 * sizeof(double) * npts);
    double* frc = malloc(3 * sizeof(double) * npts);
    double* U = malloc(3 * sizeof(double) * npts);
    double* ia = malloc(sizeof(double) * npts);
    double* ial = malloc(sizeof(double) * npts);
    const double L[3] = {nx, ny, nz};
    for (int i = 0; i < npts; ++i) {
        for (int a = 0; a < 3; ++a) {
            pos[3 * i + a] = (frand(&seed) * 3.0 - 1.0) * L[a];   /* also outside [0, L) */
            frc[3 * i + a] = (frand(&seed) - 0.5) * 1e-3;
        }
        ia[i] = 1.0 / 0.2;
        ial[i] = 0.77;
    }
    if (npts > 0) {
        pos[0] = L[0] - 1e-12;   /* on the seams */
        pos[1] = 0.0;
    }
    int bad = 0;
    for (int t = 0; t < steps; ++t) {
        orc_spread(nx, ny, nz, npts, pos, frc, t & 1, g);
        orc_collide(nx, ny, nz, 1.0, 0.7, df, g, dfs, rho, u);
        orc_interp(nx, ny, nz, u, npts, pos, U);
        orc_stream(nx, ny, nz, dfs, df);
        orc_advect(nx, ny, nz, 1.0, 0.7, npts, pos, frc, U, ia, ial);
        double m = 0.0;
        for (int64_t k = 0; k < 19 * N; ++k) m += df[k];
        if (!(fabs(m) < 1e-12)) ++bad;
    }
    orc_moments(nx, ny, nz, 1.0, df, g, rho, u);
    orc_equilibrium(nx, ny, nz, 1.0, rho, u, dfs);
    for (int64_t k = 0; k < 19 * N; ++k)
        if (!isfinite(dfs[k])) ++bad;
    free(df); free(dfs); free(g); free(rho); free(u); free(pos); free(frc); free(U); free(ia); free(ial);
    return bad;
}

int main(void)
{
    int bad = run(4, 5, 6, 7, 12, 1u) + run(9, 4, 7, 13, 8, 2u) + run(6, 6, 4, 1, 5, 3u) + run(5, 7, 5, 0, 3, 4u);
    if (bad) {
        fprintf(stderr, "%d failed checks\n", bad);
        return 1;
    }
    printf("oracle checks passed\n");
    return 0;
}
