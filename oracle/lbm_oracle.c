/*
 * Plain FP64 CPU oracle for the forced lattice Boltzmann step with
 * off-lattice point forces (Nash, Adhikari & Cates, "Singular forces and
 * point-like colloids in lattice Boltzmann hydrodynamics").
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path may link, load or
 * call this file; only the tests, the smoke check and the benchmark's CPU
 * baseline do.  It shares no code, table or constant with the HIP library.
 *
 * Everything is written as the paper states it, in the order the paper
 * states it, with no blocking or fusion:
 *   - D3Q19 velocity set and weights, c_s^2 = 1/3 (Sec. II, the DdQn
 *     quadrature behind Eq. eqf; D3Q19 is the standard Qian set).
 *   - State: auxiliary populations fbar_i (Eq. transformf), held as the
 *     deviation df_i = fbar_i - w_i rho0 (same arithmetic, better rounding).
 *   - Collision: the projected-ghost MRT post-collision state of Eq. fiexp
 *     with the momentum A and stress B that follow it, the sign of the
 *     (S - rho v v) term taken from the general scheme Eq. mrtlbe.
 *   - Propagation along c_i (the relax-then-propagate split after
 *     Eq. halftransform).
 *   - Spreading F(r) = sum_a f_a deltaP(r - R_a) with Peskin's 4-point
 *     kernel, Eq. deltadef (Sec. III).
 *   - Interpolation with the same kernel and the colloid update
 *     R' = v(R) + F/(6 pi eta) (1/a - 1/a_L) (Sec. IV).
 *
 * Readings where the paper is silent: the grid field is the force density
 * g = rho F; u = (sum fbar c + g/2)/rho; all six stress modes relax with
 * omega = 1/(tau + 1/2); ghosts are zero after collision; nodes sit at
 * integer coordinates on a periodic box; a step is spread -> moments ->
 * interpolate -> collide -> propagate -> advance colloids (explicit Euler).
 *
 * Built with  gcc -O2 -ffp-contract=off -fopenmp -shared -fPIC.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

#define NQ 19

/* D3Q19: rest, 6 faces, 12 edges. */
static const int CX[NQ] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
static const int CY[NQ] = {0, 0, 0, 1, -1, 0, 0, 1, 1, -1, -1, 0, 0, 0, 0, 1, -1, 1, -1};
static const int CZ[NQ] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, 1, -1, -1, 1, 1, -1, -1};

static double weight(int i)
{
    int c2 = CX[i] * CX[i] + CY[i] * CY[i] + CZ[i] * CZ[i];
    if (c2 == 0) return 1.0 / 3.0;
    if (c2 == 1) return 1.0 / 18.0;
    return 1.0 / 36.0;
}

static const double CS2 = 1.0 / 3.0;

/* c_i and Q_i = c_i c_i - cs^2 I as doubles, filled once by tables(). */
static double CD[NQ][3];
static double QD[NQ][3][3];
static double WD[NQ];

static void tables(void)
{
    for (int i = 0; i < NQ; ++i) {
        const int c[3] = {CX[i], CY[i], CZ[i]};
        for (int a = 0; a < 3; ++a) {
            CD[i][a] = (double)c[a];
            for (int b = 0; b < 3; ++b) QD[i][a][b] = (double)(c[a] * c[b]) - (a == b ? CS2 : 0.0);
        }
        WD[i] = weight(i);
    }
}

static int wrap(int64_t k, int n)
{
    int64_t r = k % n;
    return (int)(r < 0 ? r + n : r);
}

/* Periodic neighbour of coordinate x (0 <= x < n) shifted by d in {-1, 0, 1}. */
static int shift1(int x, int d, int n)
{
    int r = x + d;
    if (r < 0) r += n;
    if (r >= n) r -= n;
    return r;
}

/* Peskin's regularised one-dimensional kernel, Eq. deltadef. */
double orc_phi(double r)
{
    double a = fabs(r);
    if (a <= 1.0) return (3.0 - 2.0 * a + sqrt(1.0 + 4.0 * a - 4.0 * a * a)) / 8.0;
    if (a <= 2.0) return (5.0 - 2.0 * a - sqrt(-7.0 + 12.0 * a - 4.0 * a * a)) / 8.0;
    return 0.0;
}

int orc_nq(void) { return NQ; }

void orc_velocities(int* c_out /* [19][3] */, double* w_out /* [19] */)
{
    for (int i = 0; i < NQ; ++i) {
        c_out[3 * i + 0] = CX[i];
        c_out[3 * i + 1] = CY[i];
        c_out[3 * i + 2] = CZ[i];
        w_out[i] = weight(i);
    }
}

/*
 * Regularised spreading, Sec. III:  g(x) = sum_a F_a deltaP(x - R_a), with
 * deltaP the product of three one-dimensional kernels (h = 1).  Each node is
 * taken at the periodic image of R_a nearest to it; for L >= 4 at most one
 * image lies within the kernel's support of +-2.  Particles are added in
 * index order.  zero_net != 0 adds the uniform density -sum_a F_a / N.
 * g is [3][nz][ny][nx].
 */
void orc_spread(int nx, int ny, int nz, int64_t n, const double* pos, const double* frc,
                int zero_net, double* g)
{
    const int64_t N = (int64_t)nx * ny * nz;
    memset(g, 0, sizeof(double) * 3 * N);
    double total[3] = {0.0, 0.0, 0.0};
    for (int64_t a = 0; a < n; ++a) {
        const double* R = pos + 3 * a;
        const double* F = frc + 3 * a;
        const int64_t fx = (int64_t)floor(R[0]), fy = (int64_t)floor(R[1]), fz = (int64_t)floor(R[2]);
        for (int64_t kz = fz - 2; kz <= fz + 2; ++kz) {
            const double pz = orc_phi((double)kz - R[2]);
            if (pz == 0.0) continue;
            for (int64_t ky = fy - 2; ky <= fy + 2; ++ky) {
                const double py = orc_phi((double)ky - R[1]);
                if (py == 0.0) continue;
                for (int64_t kx = fx - 2; kx <= fx + 2; ++kx) {
                    const double px = orc_phi((double)kx - R[0]);
                    if (px == 0.0) continue;
                    const double d = px * py * pz;
                    const int64_t idx = ((int64_t)wrap(kz, nz) * ny + wrap(ky, ny)) * nx + wrap(kx, nx);
                    g[0 * N + idx] += F[0] * d;
                    g[1 * N + idx] += F[1] * d;
                    g[2 * N + idx] += F[2] * d;
                }
            }
        }
        total[0] += F[0];
        total[1] += F[1];
        total[2] += F[2];
    }
    if (zero_net) {
        for (int c = 0; c < 3; ++c) {
            const double share = total[c] / (double)N;
            for (int64_t idx = 0; idx < N; ++idx) g[c * N + idx] -= share;
        }
    }
}

/*
 * Hydrodynamic moments of the auxiliary populations at one node
 * (Eq. macrovariables2, first two lines):
 *   rho = rho0 + sum df_i,  rho u = sum df_i c_i + g/2.
 */
static void node_moments(const double* df, int64_t N, int64_t idx, double rho0, const double* g,
                         double* drho, double j[3], double Sbar[3][3], double* rho, double u[3])
{
    double s = 0.0, jx = 0.0, jy = 0.0, jz = 0.0;
    double P[3][3] = {{0}};
    for (int i = 0; i < NQ; ++i) {
        const double f = df[i * N + idx];
        s += f;
        jx += f * CD[i][0];
        jy += f * CD[i][1];
        jz += f * CD[i][2];
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) P[a][b] += f * QD[i][a][b];
    }
    *drho = s;
    j[0] = jx;
    j[1] = jy;
    j[2] = jz;
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) Sbar[a][b] = P[a][b];
    *rho = rho0 + s;
    for (int a = 0; a < 3; ++a) u[a] = (j[a] + 0.5 * g[a]) / *rho;
}

/*
 * Collision of every node (Eq. fiexp with its A and B):
 *   A = sum fbar c + g
 *   B = Sbar - omega (Sbar - rho u u - tau (u g + g u)),  omega = 1/(tau + 1/2)
 *   df*_i = w_i [ drho + A.c_i / cs^2 + B:Q_i / (2 cs^4) ],  Q_i = c_i c_i - cs^2 I
 * g may be NULL (no force).  rho_out and u_out ([3][N]) receive the physical
 * moments at this time if not NULL.
 */
void orc_collide(int nx, int ny, int nz, double rho0, double tau, const double* df, const double* g,
                 double* dfstar, double* rho_out, double* u_out)
{
    const int64_t N = (int64_t)nx * ny * nz;
    const double omega = 1.0 / (tau + 0.5);
    tables();
#pragma omp parallel for schedule(static)
    for (int64_t idx = 0; idx < N; ++idx) {
        double gl[3] = {0.0, 0.0, 0.0};
        if (g) {
            gl[0] = g[0 * N + idx];
            gl[1] = g[1 * N + idx];
            gl[2] = g[2 * N + idx];
        }
        double drho, j[3], Sb[3][3], rho, u[3];
        node_moments(df, N, idx, rho0, gl, &drho, j, Sb, &rho, u);
        double A[3], B[3][3];
        for (int a = 0; a < 3; ++a) A[a] = j[a] + gl[a];
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b)
                B[a][b] = Sb[a][b] - omega * (Sb[a][b] - rho * u[a] * u[b] - tau * (u[a] * gl[b] + gl[a] * u[b]));
        for (int i = 0; i < NQ; ++i) {
            double Ac = 0.0, BQ = 0.0;
            for (int a = 0; a < 3; ++a) {
                Ac += A[a] * CD[i][a];
                for (int b = 0; b < 3; ++b) BQ += B[a][b] * QD[i][a][b];
            }
            dfstar[i * N + idx] = WD[i] * (drho + Ac / CS2 + BQ / (2.0 * CS2 * CS2));
        }
        if (rho_out) rho_out[idx] = rho;
        if (u_out) {
            u_out[0 * N + idx] = u[0];
            u_out[1 * N + idx] = u[1];
            u_out[2 * N + idx] = u[2];
        }
    }
}

/* Propagation: df_i(x + c_i) = df*_i(x) on the periodic box. */
void orc_stream(int nx, int ny, int nz, const double* dfstar, double* df)
{
    const int64_t N = (int64_t)nx * ny * nz;
#pragma omp parallel for schedule(static)
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                const int64_t src = ((int64_t)z * ny + y) * nx + x;
                for (int i = 0; i < NQ; ++i) {
                    const int64_t dst =
                        ((int64_t)shift1(z, CZ[i], nz) * ny + shift1(y, CY[i], ny)) * nx + shift1(x, CX[i], nx);
                    df[i * N + dst] = dfstar[i * N + src];
                }
            }
}

/* Physical moments (Eq. macrovariables2) without colliding. */
void orc_moments(int nx, int ny, int nz, double rho0, const double* df, const double* g, double* rho_out,
                 double* u_out)
{
    const int64_t N = (int64_t)nx * ny * nz;
    tables();
#pragma omp parallel for schedule(static)
    for (int64_t idx = 0; idx < N; ++idx) {
        double gl[3] = {0.0, 0.0, 0.0};
        if (g) {
            gl[0] = g[0 * N + idx];
            gl[1] = g[1 * N + idx];
            gl[2] = g[2 * N + idx];
        }
        double drho, j[3], Sb[3][3], rho, u[3];
        node_moments(df, N, idx, rho0, gl, &drho, j, Sb, &rho, u);
        if (rho_out) rho_out[idx] = rho;
        for (int a = 0; a < 3; ++a) u_out[a * N + idx] = u[a];
    }
}

/*
 * Interpolation with the spreading kernel (Sec. IV):
 *   U(R) = sum_x u(x) deltaP(x - R), nearest periodic image as in spreading.
 */
void orc_interp(int nx, int ny, int nz, const double* u, int64_t n, const double* pos, double* U)
{
    const int64_t N = (int64_t)nx * ny * nz;
#pragma omp parallel for schedule(static)
    for (int64_t a = 0; a < n; ++a) {
        const double* R = pos + 3 * a;
        const int64_t fx = (int64_t)floor(R[0]), fy = (int64_t)floor(R[1]), fz = (int64_t)floor(R[2]);
        double s[3] = {0.0, 0.0, 0.0};
        for (int64_t kz = fz - 2; kz <= fz + 2; ++kz) {
            const double pz = orc_phi((double)kz - R[2]);
            if (pz == 0.0) continue;
            for (int64_t ky = fy - 2; ky <= fy + 2; ++ky) {
                const double py = orc_phi((double)ky - R[1]);
                if (py == 0.0) continue;
                for (int64_t kx = fx - 2; kx <= fx + 2; ++kx) {
                    const double px = orc_phi((double)kx - R[0]);
                    if (px == 0.0) continue;
                    const double d = px * py * pz;
                    const int64_t idx = ((int64_t)wrap(kz, nz) * ny + wrap(ky, ny)) * nx + wrap(kx, nx);
                    s[0] += u[0 * N + idx] * d;
                    s[1] += u[1 * N + idx] * d;
                    s[2] += u[2 * N + idx] * d;
                }
            }
        }
        U[3 * a + 0] = s[0];
        U[3 * a + 1] = s[1];
        U[3 * a + 2] = s[2];
    }
}

/*
 * Colloid update (Sec. IV, explicit Euler with dt = 1):
 *   R <- R + U + F/(6 pi eta) (1/a - 1/a_L),  eta = rho0 tau / 3,
 * then R is wrapped into [0, L).  inv_aL holds 1/a_L per particle.
 */
void orc_advect(int nx, int ny, int nz, double rho0, double tau, int64_t n, double* pos, const double* frc,
                const double* U, const double* inv_a, const double* inv_aL)
{
    const double eta = rho0 * tau * CS2;
    const double L[3] = {(double)nx, (double)ny, (double)nz};
    for (int64_t a = 0; a < n; ++a) {
        const double mob = (inv_a[a] - inv_aL[a]) / (6.0 * M_PI * eta);
        for (int c = 0; c < 3; ++c) {
            double r = pos[3 * a + c] + U[3 * a + c] + frc[3 * a + c] * mob;
            r -= L[c] * floor(r / L[c]);
            if (r >= L[c]) r -= L[c];
            pos[3 * a + c] = r;
        }
    }
}

/*
 * Equilibrium deviation from a (rho, u) field, Eq. eqf:
 *   df_i = w_i [ rho + rho u.c_i / cs^2 + rho u u : Q_i / (2 cs^4) ] - w_i rho0.
 */
void orc_equilibrium(int nx, int ny, int nz, double rho0, const double* rho, const double* u, double* df)
{
    const int64_t N = (int64_t)nx * ny * nz;
#pragma omp parallel for schedule(static)
    for (int64_t idx = 0; idx < N; ++idx) {
        const double r = rho[idx];
        const double v[3] = {u[idx], u[N + idx], u[2 * N + idx]};
        for (int i = 0; i < NQ; ++i) {
            const int c[3] = {CX[i], CY[i], CZ[i]};
            double vc = 0.0, vvQ = 0.0;
            for (int a = 0; a < 3; ++a) {
                vc += v[a] * c[a];
                for (int b = 0; b < 3; ++b) vvQ += v[a] * v[b] * (c[a] * c[b] - (a == b ? CS2 : 0.0));
            }
            df[i * N + idx] = weight(i) * (r + r * vc / CS2 + r * vvQ / (2.0 * CS2 * CS2)) - weight(i) * rho0;
        }
    }
}

/* Threads the parallel loops use, and a way to set them (for timing the oracle). */
int orc_threads(void) { return omp_get_max_threads(); }
void orc_set_threads(int n) { omp_set_num_threads(n); }
