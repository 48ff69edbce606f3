/*
 * lll_oracle.c -- plain, slow, FP64 reference for the pulse-noise
 * Landau-Lifshitz-Langevin method (D. A. Garanin, "Pulse-noise approach for
 * classical spin systems", arXiv:1610.04914).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file.  Only the test suite, the smoke check and the benchmark's
 * CPU-baseline leg may use it.  It shares no source with the GPU path.
 *
 * Build: gcc -O2 -fno-fast-math -ffp-contract=off -fPIC -shared
 *
 * Units: gamma = mu_0 = k_B = 1 (Sec. II, last paragraph; Eq. (2) sets k_B = 1).
 * Lattice: simple cubic Lx x Ly x Lz, site index i = x + Lx*(y + Ly*z).
 * State: one array of length 3N, component-major: s[0..N) = s_x,
 * s[N..2N) = s_y, s[2N..3N) = s_z (the paper's Appendix stores the spin
 * component as the first of four array indices).
 *
 * Every function is a direct transcription of the definition it cites, with
 * no blocking, fusion or reordering.  Readings of passages where the paper is
 * silent are marked READING.
 *
 * The site-by-site loops of the effective field, the right-hand side and the
 * RK4 update carry an OpenMP pragma.  It only takes effect in a second build
 * made with -fopenmp, which times the oracle on all host cores; every
 * iteration writes its own sites and no sum is split, so both builds give
 * identical results.  The test suite uses the build without -fopenmp.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Threads a parallel loop uses: the OpenMP team size, or 1 when compiled without OpenMP. */
int orc_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

#define ORC_OK 0
#define ORC_EINVAL (-1)
#define ORC_ENOMEM (-2)

typedef struct {
    int32_t Lx, Ly, Lz;
    int32_t bc; /* 0 = periodic, 1 = free (a missing neighbour contributes nothing) */
} orc_geom;

typedef struct {
    double J;               /* exchange: E = -J sum over bonds s_i . s_j (each bond once) */
    double H[3];            /* external field: E = -H . s_i */
    double D;               /* uniform uniaxial anisotropy: E = -D (s_i . e)^2 */
    double e[3];            /* uniform easy axis (normalised here) */
    const double* D_site;   /* optional per-site D_i [N]; overrides D when non-NULL */
    const double* e_site;   /* optional per-site easy axes, component-major [3N] */
    double lambda;          /* dimensionless damping */
    double T;               /* temperature */
    double dt;              /* RK step delta t */
    double Dt;              /* pulse spacing Delta t = n * delta t */
    int32_t precession;     /* 1: full Eq. (1); 0: slow equation (precession dropped) */
    int32_t pad_;
} orc_params;

typedef struct {
    double E_total, E_exch, E_zeeman, E_anis;
    double m[3];
    double max_norm_dev;
} orc_obs;

static int64_t nsites(const orc_geom* g) { return (int64_t)g->Lx * g->Ly * g->Lz; }

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 counter-based generator, from its published definition     */
/* (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy as 1, 2,  */
/* 3", SC'11): ten rounds of two 32x32->64 multiplies with the multipliers  */
/* 0xD2511F53 and 0xCD9E8D57, the key bumped by the Weyl constants          */
/* 0x9E3779B9 and 0xBB67AE85 between rounds.                                */
/* ------------------------------------------------------------------------ */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* READING (counter layout): counter = (site i, pulse k mod 2^32, replica r,
 * tag), key = (seed mod 2^32, seed >> 32).  Tags: 0 = noise kick,
 * 1 = random-sphere initial state.  One block of four words per site and
 * pulse, so the stream does not depend on how the lattice is tiled. */
static void philox_site(uint64_t seed, uint32_t i, uint32_t k, uint32_t r, uint32_t tag,
                        uint32_t w[4])
{
    uint32_t ctr[4] = {i, k, r, tag};
    uint32_t key[2] = {(uint32_t)(seed & 0xFFFFFFFFu), (uint32_t)(seed >> 32)};
    orc_philox4x32_10(ctr, key, w);
}

/* Words for counters (i0 + j, c1, c2, c3), j = 0..n-1, written as out[4j..4j+3]. */
void orc_philox_stream(uint64_t seed, uint32_t i0, int64_t n, uint32_t c1, uint32_t c2,
                       uint32_t c3, uint32_t* out)
{
    for (int64_t j = 0; j < n; ++j)
        philox_site(seed, (uint32_t)(i0 + (uint32_t)j), c1, c2, c3, out + 4 * j);
}

/* Uniform in the open interval (0,1): u = (w + 1/2) 2^-32, exact in FP64. */
double orc_u01(uint32_t w) { return ((double)w + 0.5) * (1.0 / 4294967296.0); }

static const double ORC_TWO_PI = 6.283185307179586;

/* Box-Muller (the paper's Appendix names it as its normal generator): three
 * unit normals from the four words of one block; the fourth normal of the
 * second pair is not used. */
void orc_gauss3(uint64_t seed, uint32_t i, uint32_t k, uint32_t r, uint32_t tag, double G[3])
{
    uint32_t w[4];
    philox_site(seed, i, k, r, tag, w);
    double u0 = orc_u01(w[0]), u1 = orc_u01(w[1]);
    double u2 = orc_u01(w[2]), u3 = orc_u01(w[3]);
    double r0 = sqrt(-2.0 * log(u0));
    double r1 = sqrt(-2.0 * log(u2));
    G[0] = r0 * cos(ORC_TWO_PI * u1);
    G[1] = r0 * sin(ORC_TWO_PI * u1);
    G[2] = r1 * cos(ORC_TWO_PI * u3);
}

/* ------------------------------------------------------------------------ */
/* Initial states                                                           */
/* ------------------------------------------------------------------------ */

/* Uniform on the unit sphere from one Philox block (tag 1, pulse 0):
 * z = 2 u0 - 1, azimuth = 2 pi u1 (Archimedes' hat-box theorem). */
void orc_init_random_sphere(const orc_geom* g, uint64_t seed, uint32_t r, double* s)
{
    int64_t N = nsites(g);
    for (int64_t i = 0; i < N; ++i) {
        uint32_t w[4];
        philox_site(seed, (uint32_t)i, 0u, r, 1u, w);
        double z = 2.0 * orc_u01(w[0]) - 1.0;
        double ph = ORC_TWO_PI * orc_u01(w[1]);
        double rho = sqrt(1.0 - z * z);
        s[i] = rho * cos(ph);
        s[N + i] = rho * sin(ph);
        s[2 * N + i] = z;
    }
}

/* Completely ordered state along dir (Sec. III and IV start from ordered states). */
void orc_init_direction(const orc_geom* g, const double dir[3], double* s)
{
    int64_t N = nsites(g);
    double n = sqrt(dir[0] * dir[0] + dir[1] * dir[1] + dir[2] * dir[2]);
    for (int64_t i = 0; i < N; ++i) {
        s[i] = dir[0] / n;
        s[N + i] = dir[1] / n;
        s[2 * N + i] = dir[2] / n;
    }
}

/* ------------------------------------------------------------------------ */
/* Effective field and energy                                               */
/* ------------------------------------------------------------------------ */

/* Neighbour of site (x,y,z) one step along axis a (0,1,2) in direction
 * d (+1/-1); returns -1 when it is missing (free boundaries).  Periodic
 * boundaries use (coordinate +- 1) mod L, so L = 1 and L = 2 give self and
 * repeated bonds, counted as written. */
static int64_t neighbour(const orc_geom* g, int x, int y, int z, int a, int d)
{
    int c[3] = {x, y, z};
    int L[3] = {g->Lx, g->Ly, g->Lz};
    int v = c[a] + d;
    if (v < 0 || v >= L[a]) {
        if (g->bc == 1) return -1;
        v = ((v % L[a]) + L[a]) % L[a];
    }
    c[a] = v;
    return (int64_t)c[0] + (int64_t)g->Lx * ((int64_t)c[1] + (int64_t)g->Ly * c[2]);
}

static void easy_axis(const orc_params* p, int64_t N, int64_t i, double e[3], double* D)
{
    if (p->e_site) {
        e[0] = p->e_site[i]; e[1] = p->e_site[N + i]; e[2] = p->e_site[2 * N + i];
    } else {
        double n = sqrt(p->e[0] * p->e[0] + p->e[1] * p->e[1] + p->e[2] * p->e[2]);
        if (n > 0) { e[0] = p->e[0] / n; e[1] = p->e[1] / n; e[2] = p->e[2] / n; }
        else { e[0] = 0; e[1] = 0; e[2] = 1; }
    }
    *D = p->D_site ? p->D_site[i] : p->D;
}

/* Effective field h_i = -dE/ds_i for E = -J sum_<ij> s_i.s_j - sum_i H.s_i
 * - sum_i D_i (s_i.e_i)^2 (Eq. (1)'s H_eff; the anisotropy sign and factor
 * follow Eq. (12), H = -D s_z^2 - H s_x):
 *   h_i = J sum_{j in nn(i)} s_j + H + 2 D_i (s_i.e_i) e_i. */
void orc_heff(const orc_geom* g, const orc_params* p, const double* s, double* h)
{
    int64_t N = nsites(g);
#pragma omp parallel for
    for (int z = 0; z < g->Lz; ++z)
        for (int y = 0; y < g->Ly; ++y)
            for (int x = 0; x < g->Lx; ++x) {
                int64_t i = x + (int64_t)g->Lx * (y + (int64_t)g->Ly * z);
                double sum[3] = {0, 0, 0};
                for (int a = 0; a < 3; ++a)
                    for (int d = -1; d <= 1; d += 2) {
                        int64_t j = neighbour(g, x, y, z, a, d);
                        if (j < 0) continue;
                        sum[0] += s[j]; sum[1] += s[N + j]; sum[2] += s[2 * N + j];
                    }
                double e[3], D;
                easy_axis(p, N, i, e, &D);
                double se = s[i] * e[0] + s[N + i] * e[1] + s[2 * N + i] * e[2];
                for (int c = 0; c < 3; ++c)
                    h[c * N + i] = p->J * sum[c] + p->H[c] + 2.0 * D * se * e[c];
            }
}

/* Energy parts: out[0] = exchange (each bond once, via the +x, +y, +z bond
 * of every site), out[1] = Zeeman, out[2] = anisotropy. */
void orc_energy_parts(const orc_geom* g, const orc_params* p, const double* s, double out[3])
{
    int64_t N = nsites(g);
    double ex = 0, ze = 0, an = 0;
    for (int z = 0; z < g->Lz; ++z)
        for (int y = 0; y < g->Ly; ++y)
            for (int x = 0; x < g->Lx; ++x) {
                int64_t i = x + (int64_t)g->Lx * (y + (int64_t)g->Ly * z);
                for (int a = 0; a < 3; ++a) {
                    int64_t j = neighbour(g, x, y, z, a, +1);
                    if (j < 0) continue;
                    ex += -p->J * (s[i] * s[j] + s[N + i] * s[N + j] + s[2 * N + i] * s[2 * N + j]);
                }
                ze += -(p->H[0] * s[i] + p->H[1] * s[N + i] + p->H[2] * s[2 * N + i]);
                double e[3], D;
                easy_axis(p, N, i, e, &D);
                double se = s[i] * e[0] + s[N + i] * e[1] + s[2 * N + i] * e[2];
                an += -D * se * se;
            }
    out[0] = ex; out[1] = ze; out[2] = an;
}

/* ------------------------------------------------------------------------ */
/* Noise-free right-hand side, Eq. (1) with zeta = 0 and gamma = 1.         */
/* ------------------------------------------------------------------------ */
static void cross(const double a[3], const double b[3], double c[3])
{
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}

/* f_i = s_i x h_i - lambda s_i x (s_i x h_i)   (precessional case), or
 * f_i =           - lambda s_i x (s_i x h_i)   (slow equation, Sec. II: the
 * precession term is dropped).  The double cross product is evaluated as
 * written, without using |s| = 1. */
void orc_rhs(const orc_geom* g, const orc_params* p, const double* s, double* f)
{
    int64_t N = nsites(g);
    double* h = (double*)malloc(sizeof(double) * 3 * N);
    orc_heff(g, p, s, h);
#pragma omp parallel for
    for (int64_t i = 0; i < N; ++i) {
        double si[3] = {s[i], s[N + i], s[2 * N + i]};
        double hi[3] = {h[i], h[N + i], h[2 * N + i]};
        double sh[3], ssh[3];
        cross(si, hi, sh);
        cross(si, sh, ssh);
        for (int c = 0; c < 3; ++c)
            f[c * N + i] = (p->precession ? sh[c] : 0.0) - p->lambda * ssh[c];
    }
    free(h);
}

/* ------------------------------------------------------------------------ */
/* Integrators for x' = f(x) on the whole lattice vector, step h = dt.       */
/* Classical RK4 is the method of the hot path; Heun, RK2-midpoint and      */
/* Butcher's RK5 are the tableaux listed in the paper's Appendix and serve  */
/* as cross-checks.  No renormalisation of spins inside a segment.          */
/* ------------------------------------------------------------------------ */
static void axpy_into(int64_t M, double* out, const double* x, double a, const double* k)
{
#pragma omp parallel for
    for (int64_t j = 0; j < M; ++j) out[j] = x[j] + a * k[j];
}

static void scale_by(int64_t M, double* k, double a)
{
#pragma omp parallel for
    for (int64_t j = 0; j < M; ++j) k[j] *= a;
}

/* Classical fourth-order Runge-Kutta:
 * k1 = h f(x), k2 = h f(x + k1/2), k3 = h f(x + k2/2), k4 = h f(x + k3),
 * x' = x + (k1 + 2 k2 + 2 k3 + k4) / 6. */
void orc_step_rk4(const orc_geom* g, const orc_params* p, double* s, int64_t n_steps)
{
    int64_t M = 3 * nsites(g);
    double* k1 = (double*)malloc(sizeof(double) * M);
    double* k2 = (double*)malloc(sizeof(double) * M);
    double* k3 = (double*)malloc(sizeof(double) * M);
    double* k4 = (double*)malloc(sizeof(double) * M);
    double* y = (double*)malloc(sizeof(double) * M);
    double hh = p->dt;
    for (int64_t n = 0; n < n_steps; ++n) {
        orc_rhs(g, p, s, k1);
        scale_by(M, k1, hh);
        axpy_into(M, y, s, 0.5, k1);
        orc_rhs(g, p, y, k2);
        scale_by(M, k2, hh);
        axpy_into(M, y, s, 0.5, k2);
        orc_rhs(g, p, y, k3);
        scale_by(M, k3, hh);
        axpy_into(M, y, s, 1.0, k3);
        orc_rhs(g, p, y, k4);
        scale_by(M, k4, hh);
#pragma omp parallel for
        for (int64_t j = 0; j < M; ++j)
            s[j] = s[j] + (k1[j] + 2.0 * k2[j] + 2.0 * k3[j] + k4[j]) / 6.0;
    }
    free(k1); free(k2); free(k3); free(k4); free(y);
}

/* Heun (Appendix): K1 = h f(x), K2 = h f(x + K1), x' = x + (K1 + K2)/2. */
void orc_step_heun(const orc_geom* g, const orc_params* p, double* s, int64_t n_steps)
{
    int64_t M = 3 * nsites(g);
    double* k1 = (double*)malloc(sizeof(double) * M);
    double* k2 = (double*)malloc(sizeof(double) * M);
    double* y = (double*)malloc(sizeof(double) * M);
    for (int64_t n = 0; n < n_steps; ++n) {
        orc_rhs(g, p, s, k1);
        for (int64_t j = 0; j < M; ++j) k1[j] *= p->dt;
        axpy_into(M, y, s, 1.0, k1);
        orc_rhs(g, p, y, k2);
        for (int64_t j = 0; j < M; ++j) k2[j] *= p->dt;
        for (int64_t j = 0; j < M; ++j) s[j] = s[j] + 0.5 * (k1[j] + k2[j]);
    }
    free(k1); free(k2); free(y);
}

/* RK2 midpoint (Appendix): K1 = h f(x), K2 = h f(x + K1/2), x' = x + K2. */
void orc_step_rk2mid(const orc_geom* g, const orc_params* p, double* s, int64_t n_steps)
{
    int64_t M = 3 * nsites(g);
    double* k1 = (double*)malloc(sizeof(double) * M);
    double* k2 = (double*)malloc(sizeof(double) * M);
    double* y = (double*)malloc(sizeof(double) * M);
    for (int64_t n = 0; n < n_steps; ++n) {
        orc_rhs(g, p, s, k1);
        for (int64_t j = 0; j < M; ++j) k1[j] *= p->dt;
        axpy_into(M, y, s, 0.5, k1);
        orc_rhs(g, p, y, k2);
        for (int64_t j = 0; j < M; ++j) k2[j] *= p->dt;
        for (int64_t j = 0; j < M; ++j) s[j] = s[j] + k2[j];
    }
    free(k1); free(k2); free(y);
}

/* Butcher's six-stage fifth-order Runge-Kutta (Appendix):
 * K1 = h f(x)
 * K2 = h f(x + K1/4)
 * K3 = h f(x + (K1 + K2)/8)
 * K4 = h f(x - K2/2 + K3)
 * K5 = h f(x + 3 (K1 + 3 K4)/16)
 * K6 = h f(x + (-3 K1 + 2 K2 + 12 (K3 - K4) + 8 K5)/7)
 * x' = x + (7 K1 + 32 K3 + 12 K4 + 32 K5 + 7 K6)/90 */
void orc_step_rk5b(const orc_geom* g, const orc_params* p, double* s, int64_t n_steps)
{
    int64_t M = 3 * nsites(g);
    double* K[6];
    for (int q = 0; q < 6; ++q) K[q] = (double*)malloc(sizeof(double) * M);
    double* y = (double*)malloc(sizeof(double) * M);
    double hh = p->dt;
    for (int64_t n = 0; n < n_steps; ++n) {
        orc_rhs(g, p, s, K[0]);
        for (int64_t j = 0; j < M; ++j) K[0][j] *= hh;
        for (int64_t j = 0; j < M; ++j) y[j] = s[j] + K[0][j] / 4.0;
        orc_rhs(g, p, y, K[1]);
        for (int64_t j = 0; j < M; ++j) K[1][j] *= hh;
        for (int64_t j = 0; j < M; ++j) y[j] = s[j] + (K[0][j] + K[1][j]) / 8.0;
        orc_rhs(g, p, y, K[2]);
        for (int64_t j = 0; j < M; ++j) K[2][j] *= hh;
        for (int64_t j = 0; j < M; ++j) y[j] = s[j] - K[1][j] / 2.0 + K[2][j];
        orc_rhs(g, p, y, K[3]);
        for (int64_t j = 0; j < M; ++j) K[3][j] *= hh;
        for (int64_t j = 0; j < M; ++j) y[j] = s[j] + 3.0 * (K[0][j] + 3.0 * K[3][j]) / 16.0;
        orc_rhs(g, p, y, K[4]);
        for (int64_t j = 0; j < M; ++j) K[4][j] *= hh;
        for (int64_t j = 0; j < M; ++j)
            y[j] = s[j] + (-3.0 * K[0][j] + 2.0 * K[1][j] + 12.0 * (K[2][j] - K[3][j]) +
                           8.0 * K[4][j]) / 7.0;
        orc_rhs(g, p, y, K[5]);
        for (int64_t j = 0; j < M; ++j) K[5][j] *= hh;
        for (int64_t j = 0; j < M; ++j)
            s[j] = s[j] + (7.0 * K[0][j] + 32.0 * K[2][j] + 12.0 * K[3][j] + 32.0 * K[4][j] +
                           7.0 * K[5][j]) / 90.0;
    }
    for (int q = 0; q < 6; ++q) free(K[q]);
    free(y);
}

/* ------------------------------------------------------------------------ */
/* Pulse-noise kick, Eqs. (5)-(6)                                           */
/* ------------------------------------------------------------------------ */

/* Rotation of s by the vector angle phi = phi n, |n| = 1 (Eq. (6)):
 * s' = s cos(phi) + (n x s) sin(phi) + n (s.n) (1 - cos(phi)).
 * READING: phi = 0 is the identity (no small-angle expansion). */
void orc_rotate(const double s[3], const double phv[3], double out[3])
{
    double ph = sqrt(phv[0] * phv[0] + phv[1] * phv[1] + phv[2] * phv[2]);
    if (ph == 0.0) { out[0] = s[0]; out[1] = s[1]; out[2] = s[2]; return; }
    double n[3] = {phv[0] / ph, phv[1] / ph, phv[2] / ph};
    double c = cos(ph), sn = sin(ph);
    double nxs[3];
    cross(n, s, nxs);
    double sdn = s[0] * n[0] + s[1] * n[1] + s[2] * n[2];
    for (int q = 0; q < 3; ++q) out[q] = s[q] * c + nxs[q] * sn + n[q] * sdn * (1.0 - c);
}

/* Kick number k at temperature T (Eq. (5)): phi = sqrt(Lambda_N Delta t) G
 * with Lambda_N = 2 gamma lambda T / mu_0 = 2 lambda T; READING: the square
 * root scales each Cartesian component of G.  Each spin is rotated by
 * Eq. (6), then READING: renormalised to unit length (the paper requires
 * conserved spin length; renormalisation happens after kicks only).
 * Returns max_i | |s_i'| - 1 | measured before the renormalisation.
 * site_id (optional) gives the counter of every site when the array holds a
 * cut-out of a larger lattice; NULL means site i uses counter i. */
double orc_kick_indexed(const orc_geom* g, const orc_params* p, double T, uint64_t seed,
                        uint32_t r, uint64_t k, const uint32_t* site_id, double* s)
{
    int64_t N = nsites(g);
    double sigma = sqrt(2.0 * p->lambda * T * p->Dt);
    double maxdev = 0.0;
    for (int64_t i = 0; i < N; ++i) {
        double G[3];
        uint32_t id = site_id ? site_id[i] : (uint32_t)i;
        orc_gauss3(seed, id, (uint32_t)k, r, 0u, G);
        double phv[3] = {sigma * G[0], sigma * G[1], sigma * G[2]};
        double si[3] = {s[i], s[N + i], s[2 * N + i]}, so[3];
        orc_rotate(si, phv, so);
        double nrm = sqrt(so[0] * so[0] + so[1] * so[1] + so[2] * so[2]);
        double dev = fabs(nrm - 1.0);
        if (dev > maxdev) maxdev = dev;
        s[i] = so[0] / nrm;
        s[N + i] = so[1] / nrm;
        s[2 * N + i] = so[2] / nrm;
    }
    return maxdev;
}

/* The kick of the whole lattice: site i draws its normals from counter i. */
double orc_kick(const orc_geom* g, const orc_params* p, double T, uint64_t seed, uint32_t r,
                uint64_t k, double* s)
{
    return orc_kick_indexed(g, p, T, seed, r, k, NULL, s);
}

/* ------------------------------------------------------------------------ */
/* Observables (measured at the end of every interval, Sec. III.A).          */
/* ------------------------------------------------------------------------ */
void orc_observables(const orc_geom* g, const orc_params* p, const double* s, orc_obs* o)
{
    int64_t N = nsites(g);
    double parts[3];
    orc_energy_parts(g, p, s, parts);
    o->E_exch = parts[0];
    o->E_zeeman = parts[1];
    o->E_anis = parts[2];
    o->E_total = parts[0] + parts[1] + parts[2];
    double m[3] = {0, 0, 0}, md = 0;
    for (int64_t i = 0; i < N; ++i) {
        m[0] += s[i]; m[1] += s[N + i]; m[2] += s[2 * N + i];
        double nrm = sqrt(s[i] * s[i] + s[N + i] * s[N + i] + s[2 * N + i] * s[2 * N + i]);
        double dev = fabs(nrm - 1.0);
        if (dev > md) md = dev;
    }
    o->m[0] = m[0] / N; o->m[1] = m[1] / N; o->m[2] = m[2] / N;
    o->max_norm_dev = md;
}

/* ------------------------------------------------------------------------ */
/* Schedule (Eq. (7), Suzuki-Trotter splitting with the kick in the middle  */
/* of every interval).  n = Delta t / delta t must be an integer.           */
/* READING: an interval is n1 = floor(n/2) RK4 steps, kick, n2 = n - n1      */
/* steps, then measurement; for odd n the kick sits one step early.          */
/* ------------------------------------------------------------------------ */
int64_t orc_steps_per_interval(const orc_params* p)
{
    if (!(p->dt > 0) || !(p->Dt > 0)) return -1;
    double q = p->Dt / p->dt;
    double n = floor(q + 0.5);
    if (n < 1 || fabs(q - n) > 1e-9 * n) return -1;
    return (int64_t)n;
}

/* Runs n_pulses intervals with pulse indices first_pulse .. first_pulse +
 * n_pulses - 1.  T_per_pulse (optional) gives the temperature of each kick.
 * Every obs_every-th interval (obs_every > 0) appends one orc_obs to trace.
 * Returns the largest pre-renormalisation norm deviation seen in any kick, or
 * a negative value on invalid input. */
double orc_run(const orc_geom* g, const orc_params* p, uint64_t seed, uint32_t r,
               uint64_t first_pulse, int64_t n_pulses, const double* T_per_pulse,
               int32_t obs_every, double* s, orc_obs* trace)
{
    int64_t n = orc_steps_per_interval(p);
    if (n < 1) return -1.0;
    int64_t n1 = n / 2, n2 = n - n1;
    double maxdev = 0.0;
    int64_t m = 0;
    for (int64_t q = 0; q < n_pulses; ++q) {
        uint64_t k = first_pulse + (uint64_t)q;
        double T = T_per_pulse ? T_per_pulse[q] : p->T;
        orc_step_rk4(g, p, s, n1);
        double d = orc_kick(g, p, T, seed, r, k, s);
        if (d > maxdev) maxdev = d;
        orc_step_rk4(g, p, s, n2);
        if (obs_every > 0 && ((q + 1) % obs_every) == 0 && trace) {
            orc_observables(g, p, s, &trace[m]);
            ++m;
        }
    }
    return maxdev;
}

/* ------------------------------------------------------------------------ */
/* Discrete adjoint (reverse mode) of orc_run for                            */
/*   L = <c, s_T> + wE * E(s_T) + wm . m(s_T),   m = sum_i s_i / N,          */
/* where c is an optional cotangent of the final state (the gradient, with   */
/* respect to s_T, of whatever loss the caller computes from s_T itself),    */
/* with respect to the initial state s_0 and the parameters H (3), J and D   */
/* (per-site D_i when D_site is given, else the uniform D).  The kicks are    */
/* fixed by the seed and do not depend on the parameters.                    */
/*                                                                           */
/* Plainly: all intermediate states are stored (no checkpointing), and each  */
/* RK4 step is reversed stage by stage:                                      */
/*   y1 = x, y2 = x + k1/2, y3 = x + k2/2, y4 = x + k3, k_j = dt f(y_j),      */
/*   xbar' given:  xbar = xbar', kbar1 = kbar4 = xbar'/6, kbar2 = kbar3 = xbar'/3 */
/*   ybar4 = dt Jf(y4)^T kbar4; xbar += ybar4; kbar3 += ybar4                 */
/*   ybar3 = dt Jf(y3)^T kbar3; xbar += ybar3; kbar2 += ybar3 / 2             */
/*   ybar2 = dt Jf(y2)^T kbar2; xbar += ybar2; kbar1 += ybar2 / 2             */
/*   ybar1 = dt Jf(y1)^T kbar1; xbar += ybar1                                 */
/* where, for f = s x h - lam s x (s x h) and a cotangent u of f:              */
/*   (df/dh)^T u = u x s - lam [ s (s.u) - u (s.s) ]                           */
/*   (df/ds)^T u (h fixed) = h x u - lam [ u (s.h) + h (s.u) - 2 s (h.u) ]     */
/* (slow equation: drop the first term of each), and h depends on s through  */
/* the symmetric stencil, so ybar_i = (df/ds)^T_i u_i + J sum_nn q_j          */
/* + 2 D_i e_i (e_i . q_i) with q_i = (df/dh)^T_i u_i.  Parameter cotangents: */
/* Hbar += sum_i q_i, Jbar += sum_i q_i . sum_nn s_j, Dbar_i += q_i . 2 (s_i.e_i) e_i. */
/* Kick reverse: s'' = s'/|s'|, s' = R s  =>  sbar = R^T (I - s'' s''^T) sbar'' / |s'|. */
/* ------------------------------------------------------------------------ */

/* Transposed stage Jacobian product: given the stage input y and the
 * cotangent u of f(y) (already multiplied by dt), adds the cotangent of y to
 * ybar and the parameter cotangents. */
static void rhs_vjp(const orc_geom* g, const orc_params* p, const double* y, const double* u,
                    double* ybar, double gH[3], double* gJ, double* gD)
{
    int64_t N = nsites(g);
    double lam = p->lambda;
    double* h = (double*)malloc(sizeof(double) * 3 * N);
    double* q = (double*)malloc(sizeof(double) * 3 * N);
    orc_heff(g, p, y, h);
    for (int64_t i = 0; i < N; ++i) {
        double s[3] = {y[i], y[N + i], y[2 * N + i]};
        double hh[3] = {h[i], h[N + i], h[2 * N + i]};
        double uu[3] = {u[i], u[N + i], u[2 * N + i]};
        double su = s[0] * uu[0] + s[1] * uu[1] + s[2] * uu[2];
        double ss = s[0] * s[0] + s[1] * s[1] + s[2] * s[2];
        double sh = s[0] * hh[0] + s[1] * hh[1] + s[2] * hh[2];
        double hu = hh[0] * uu[0] + hh[1] * uu[1] + hh[2] * uu[2];
        double uxs[3], hxu[3];
        cross(uu, s, uxs);
        cross(hh, uu, hxu);
        for (int c = 0; c < 3; ++c) {
            double qc = -lam * (s[c] * su - uu[c] * ss);
            double lc = -lam * (uu[c] * sh + hh[c] * su - 2.0 * s[c] * hu);
            if (p->precession) { qc += uxs[c]; lc += hxu[c]; }
            q[c * N + i] = qc;
            ybar[c * N + i] += lc;
        }
    }
    for (int z = 0; z < g->Lz; ++z)
        for (int yy = 0; yy < g->Ly; ++yy)
            for (int x = 0; x < g->Lx; ++x) {
                int64_t i = x + (int64_t)g->Lx * (yy + (int64_t)g->Ly * z);
                double qs[3] = {0, 0, 0}, ys[3] = {0, 0, 0};
                for (int a = 0; a < 3; ++a)
                    for (int d = -1; d <= 1; d += 2) {
                        int64_t j = neighbour(g, x, yy, z, a, d);
                        if (j < 0) continue;
                        for (int c = 0; c < 3; ++c) {
                            qs[c] += q[c * N + j];
                            ys[c] += y[c * N + j];
                        }
                    }
                double e[3], D;
                easy_axis(p, N, i, e, &D);
                double qi[3] = {q[i], q[N + i], q[2 * N + i]};
                double si[3] = {y[i], y[N + i], y[2 * N + i]};
                double eq = e[0] * qi[0] + e[1] * qi[1] + e[2] * qi[2];
                double se = e[0] * si[0] + e[1] * si[1] + e[2] * si[2];
                for (int c = 0; c < 3; ++c) {
                    ybar[c * N + i] += p->J * qs[c] + 2.0 * D * e[c] * eq;
                    gH[c] += qi[c];
                }
                *gJ += qi[0] * ys[0] + qi[1] * ys[1] + qi[2] * ys[2];
                double dD = 2.0 * se * eq;
                if (p->D_site) gD[i] += dD; else gD[0] += dD;
            }
    free(h);
    free(q);
}

/* Loss and its gradients.  cot: [3N] cotangent c of s_T, or NULL for c = 0.
 * g_s0 [3N] (may be NULL), g_H[3], g_J[1], g_D [N] when D_site is given else
 * [1].  Returns ORC_OK or an error. */
int orc_adjoint(const orc_geom* g, const orc_params* p, uint64_t seed, uint32_t r,
                uint64_t first_pulse, int64_t n_pulses, const double* T_per_pulse,
                const double* s0, double wE, const double wm[3], const double* cot,
                double* loss, double* g_s0, double g_H[3], double* g_J, double* g_D)
{
    int64_t n = orc_steps_per_interval(p);
    if (n < 1) return ORC_EINVAL;
    int64_t n1 = n / 2, n2 = n - n1;
    int64_t N = nsites(g), M = 3 * N;
    int64_t n_ops = n_pulses * (n + 1);
    /* op j: 0 = RK4 step, 1 = kick; states[j] = state before op j. */
    int8_t* op = (int8_t*)malloc((size_t)n_ops);
    uint64_t* opk = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)n_ops);
    double* opT = (double*)malloc(sizeof(double) * (size_t)n_ops);
    double* states = (double*)malloc(sizeof(double) * (size_t)(M * (n_ops + 1)));
    if (!op || !opk || !opT || !states) { free(op); free(opk); free(opT); free(states); return ORC_ENOMEM; }
    int64_t j = 0;
    for (int64_t qp = 0; qp < n_pulses; ++qp) {
        uint64_t k = first_pulse + (uint64_t)qp;
        double T = T_per_pulse ? T_per_pulse[qp] : p->T;
        for (int64_t a = 0; a < n1; ++a) { op[j] = 0; opk[j] = k; opT[j] = T; ++j; }
        op[j] = 1; opk[j] = k; opT[j] = T; ++j;
        for (int64_t a = 0; a < n2; ++a) { op[j] = 0; opk[j] = k; opT[j] = T; ++j; }
    }
    memcpy(states, s0, sizeof(double) * M);
    for (j = 0; j < n_ops; ++j) {
        double* cur = states + M * (j + 1);
        memcpy(cur, states + M * j, sizeof(double) * M);
        if (op[j] == 0) orc_step_rk4(g, p, cur, 1);
        else orc_kick(g, p, opT[j], seed, r, opk[j], cur);
    }
    const double* sT = states + M * n_ops;

    /* Loss and its direct gradient. */
    orc_obs o;
    orc_observables(g, p, sT, &o);
    *loss = wE * o.E_total + wm[0] * o.m[0] + wm[1] * o.m[1] + wm[2] * o.m[2];
    if (cot)
        for (int64_t a = 0; a < M; ++a) *loss += cot[a] * sT[a];
    double* sbar = (double*)calloc((size_t)M, sizeof(double));
    double* h = (double*)malloc(sizeof(double) * M);
    orc_heff(g, p, sT, h);
    for (int c = 0; c < 3; ++c)
        for (int64_t i = 0; i < N; ++i) sbar[c * N + i] = -wE * h[c * N + i] + wm[c] / (double)N;
    if (cot)
        for (int64_t a = 0; a < M; ++a) sbar[a] += cot[a];
    g_H[0] = g_H[1] = g_H[2] = 0.0;
    *g_J = 0.0;
    int64_t nD = p->D_site ? N : 1;
    for (int64_t i = 0; i < nD; ++i) g_D[i] = 0.0;
    for (int64_t i = 0; i < N; ++i) {
        g_H[0] += -wE * sT[i]; g_H[1] += -wE * sT[N + i]; g_H[2] += -wE * sT[2 * N + i];
    }
    {
        double parts[3];
        orc_params pj = *p;
        pj.J = 1.0;
        orc_energy_parts(g, &pj, sT, parts); /* exchange energy per unit J */
        *g_J += wE * parts[0];
        for (int64_t i = 0; i < N; ++i) {
            double e[3], D;
            easy_axis(p, N, i, e, &D);
            double se = sT[i] * e[0] + sT[N + i] * e[1] + sT[2 * N + i] * e[2];
            if (p->D_site) g_D[i] += -wE * se * se; else g_D[0] += -wE * se * se;
        }
    }

    double* xbar = (double*)malloc(sizeof(double) * M);
    double* kb[4];
    for (int q = 0; q < 4; ++q) kb[q] = (double*)malloc(sizeof(double) * M);
    double* y = (double*)malloc(sizeof(double) * M);
    double* yb = (double*)malloc(sizeof(double) * M);
    double* f = (double*)malloc(sizeof(double) * M);
    double* ystage[4];
    for (int q = 0; q < 4; ++q) ystage[q] = (double*)malloc(sizeof(double) * M);
    double* u = (double*)malloc(sizeof(double) * M);

    for (j = n_ops - 1; j >= 0; --j) {
        const double* x = states + M * j;
        if (op[j] == 1) {
            /* kick reverse */
            double sigma = sqrt(2.0 * p->lambda * opT[j] * p->Dt);
            for (int64_t i = 0; i < N; ++i) {
                double G[3];
                orc_gauss3(seed, (uint32_t)i, (uint32_t)opk[j], r, 0u, G);
                double phv[3] = {sigma * G[0], sigma * G[1], sigma * G[2]};
                double si[3] = {x[i], x[N + i], x[2 * N + i]}, sp[3];
                orc_rotate(si, phv, sp);
                double nrm = sqrt(sp[0] * sp[0] + sp[1] * sp[1] + sp[2] * sp[2]);
                double sh[3] = {sp[0] / nrm, sp[1] / nrm, sp[2] / nrm};
                double b[3] = {sbar[i], sbar[N + i], sbar[2 * N + i]};
                double sb = sh[0] * b[0] + sh[1] * b[1] + sh[2] * b[2];
                double bp[3] = {(b[0] - sh[0] * sb) / nrm, (b[1] - sh[1] * sb) / nrm,
                                (b[2] - sh[2] * sb) / nrm};
                double mphv[3] = {-phv[0], -phv[1], -phv[2]}, bo[3];
                orc_rotate(bp, mphv, bo); /* R^T = rotation by -phi */
                sbar[i] = bo[0]; sbar[N + i] = bo[1]; sbar[2 * N + i] = bo[2];
            }
            continue;
        }
        /* forward stages of this step */
        double hh = p->dt;
        memcpy(ystage[0], x, sizeof(double) * M);
        orc_rhs(g, p, ystage[0], f);
        for (int64_t a = 0; a < M; ++a) ystage[1][a] = x[a] + 0.5 * (hh * f[a]);
        orc_rhs(g, p, ystage[1], f);
        for (int64_t a = 0; a < M; ++a) ystage[2][a] = x[a] + 0.5 * (hh * f[a]);
        orc_rhs(g, p, ystage[2], f);
        for (int64_t a = 0; a < M; ++a) ystage[3][a] = x[a] + (hh * f[a]);
        /* reverse */
        for (int64_t a = 0; a < M; ++a) {
            xbar[a] = sbar[a];
            kb[0][a] = sbar[a] / 6.0;
            kb[1][a] = sbar[a] / 3.0;
            kb[2][a] = sbar[a] / 3.0;
            kb[3][a] = sbar[a] / 6.0;
        }
        for (int st = 3; st >= 0; --st) {
            for (int64_t a = 0; a < M; ++a) { u[a] = hh * kb[st][a]; yb[a] = 0.0; }
            rhs_vjp(g, p, ystage[st], u, yb, g_H, g_J, g_D);
            for (int64_t a = 0; a < M; ++a) {
                xbar[a] += yb[a];
                if (st == 3) kb[2][a] += yb[a];
                else if (st == 2) kb[1][a] += 0.5 * yb[a];
                else if (st == 1) kb[0][a] += 0.5 * yb[a];
            }
        }
        memcpy(sbar, xbar, sizeof(double) * M);
    }
    if (g_s0) memcpy(g_s0, sbar, sizeof(double) * M);

    free(op); free(opk); free(opT); free(states); free(sbar); free(h); free(xbar);
    for (int q = 0; q < 4; ++q) { free(kb[q]); free(ystage[q]); }
    free(y); free(yb); free(f); free(u);
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Thermally activated escape of a uniaxial spin in a transverse field      */
/* (Sec. III.B): E = -D s_z^2 - H s_x, h = H/(2D) < 1, minima at            */
/* sin(theta) = h, saddle at s = (1, 0, 0).                                  */
/* ------------------------------------------------------------------------ */
/* First-passage time of run `run`.  The spin starts at the bottom of the
 * well with phi = 0, sin(theta) = h, i.e. s = (h, 0, sqrt(1 - h^2)), and
 * follows the pulse-noise schedule of orc_run (n1 steps, kick, n2 steps per
 * interval; pulses 0, 1, ...); the normals of pulse k come from counter
 * (run, k, r, tag 0).  READING: the run stops at the first step end or kick
 * after which s_z < 0 (the paper stops after the line s_z = 0 is crossed); the
 * time is the number of completed steps times dt (a kick takes no time).
 * method: 0 RK4, 1 RK2 midpoint, 2 Butcher RK5.  Returns -1 when no crossing
 * happens within max_pulses intervals, -2 on invalid input. */
double orc_escape_time(double D, double H, double lambda, double T, double dt, double Dt,
                       int32_t precession, int32_t method, uint64_t seed, uint32_t r,
                       uint32_t run, int64_t max_pulses)
{
    orc_geom g = {1, 1, 1, 1}; /* one site, free boundaries: no exchange */
    orc_params p;
    memset(&p, 0, sizeof p);
    p.J = 0.0;
    p.H[0] = H;
    p.D = D;
    p.e[2] = 1.0;
    p.lambda = lambda;
    p.T = T;
    p.dt = dt;
    p.Dt = Dt;
    p.precession = precession;
    int64_t n = orc_steps_per_interval(&p);
    if (n < 1 || !(D > 0) || method < 0 || method > 2) return -2.0;
    double hh = H / (2.0 * D);
    if (!(hh >= 0.0 && hh < 1.0)) return -2.0;
    double s[3] = {hh, 0.0, sqrt(1.0 - hh * hh)};
    int64_t n1 = n / 2;
    for (int64_t k = 0; k < max_pulses; ++k) {
        for (int64_t q = 0; q < n; ++q) {
            if (q == n1) {
                orc_kick_indexed(&g, &p, T, seed, r, (uint64_t)k, &run, s);
                if (s[2] < 0.0) return (double)(k * n + q) * dt;
            }
            if (method == 0) orc_step_rk4(&g, &p, s, 1);
            else if (method == 1) orc_step_rk2mid(&g, &p, s, 1);
            else orc_step_rk5b(&g, &p, s, 1);
            if (s[2] < 0.0) return (double)(k * n + q + 1) * dt;
        }
    }
    return -1.0;
}
