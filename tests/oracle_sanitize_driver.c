/*
 * Exercises every entry point of the FP64 oracle on tiny and odd lattices
 * (sizes 1, 2, 3, 5, 17; periodic and free boundaries; uniform and per-site
 * anisotropy) so that a build with AddressSanitizer and UndefinedBehavior-
 * Sanitizer can report out-of-bounds accesses, leaks or undefined behaviour.
 * Built and run by tests/test_oracle_sanitizers.py; exits 0 when every call
 * returns normally and every result is finite.
 */
#include "../oracle/lll_oracle.c"

#include <stdio.h>

static int finite_all(const double* v, int64_t n)
{
    for (int64_t i = 0; i < n; ++i)
        if (!isfinite(v[i])) return 0;
    return 1;
}

int main(void)
{
    const int32_t shapes[][3] = {{1, 1, 1}, {2, 2, 2}, {3, 2, 5}, {5, 1, 2}, {17, 3, 2}, {1, 5, 3}};
    int bad = 0;
    uint32_t words[4 * 8];
    orc_philox_stream(42, 0xFFFFFFF0u, 8, 1, 2, 3, words);
    for (size_t q = 0; q < sizeof shapes / sizeof shapes[0]; ++q) {
        for (int32_t bc = 0; bc < 2; ++bc) {
            orc_geom g = {shapes[q][0], shapes[q][1], shapes[q][2], bc};
            const int64_t N = nsites(&g);
            double* s = malloc(sizeof(double) * 3 * N);
            double* t = malloc(sizeof(double) * 3 * N);
            double* h = malloc(sizeof(double) * 3 * N);
            double* Ds = malloc(sizeof(double) * N);
            double* es = malloc(sizeof(double) * 3 * N);
            double* gs = malloc(sizeof(double) * 3 * N);
            double* gD = malloc(sizeof(double) * N);
            uint32_t* ids = malloc(sizeof(uint32_t) * N);
            for (int64_t i = 0; i < N; ++i) {
                Ds[i] = 0.1 + 0.01 * (double)(i % 7);
                es[i] = 0.6; es[N + i] = 0.0; es[2 * N + i] = 0.8;
                ids[i] = (uint32_t)(3 * i + 1);
            }
            for (int site = 0; site < 2; ++site) {
                orc_params p;
                memset(&p, 0, sizeof p);
                p.J = 1.0; p.H[0] = 0.1; p.H[2] = 0.2; p.D = 0.05;
                p.e[0] = 0.0; p.e[1] = 0.0; p.e[2] = 1.0;
                p.D_site = site ? Ds : NULL;
                p.e_site = site ? es : NULL;
                p.lambda = 0.05; p.T = 0.5; p.dt = 0.1; p.Dt = 0.3; p.precession = 1;
                orc_init_random_sphere(&g, 7, 1, s);
                double dir[3] = {1.0, 2.0, 2.0};
                orc_init_direction(&g, dir, t);
                orc_heff(&g, &p, s, h);
                double e3[3];
                orc_energy_parts(&g, &p, s, e3);
                orc_rhs(&g, &p, s, h);
                memcpy(t, s, sizeof(double) * 3 * N);
                orc_step_rk4(&g, &p, t, 2);
                orc_step_rk2mid(&g, &p, t, 2);
                orc_step_rk5b(&g, &p, t, 2);
                orc_step_heun(&g, &p, t, 2);
                (void)orc_kick(&g, &p, p.T, 5, 0, 3, t);
                (void)orc_kick_indexed(&g, &p, p.T, 5, 0, 4, ids, t);
                orc_obs o[4];
                double Tp[4] = {0.5, 0.4, 0.3, 0.0};
                p.precession = site;  /* both equations */
                (void)orc_run(&g, &p, 5, 2, 0, 4, Tp, 1, t, o);
                double wm[3] = {0.0, 0.0, 1.0}, loss, gH[3], gJ, gDu;
                /* with and without a final-state cotangent (h serves as one) */
                int st = orc_adjoint(&g, &p, 5, 2, 0, 2, NULL, s, 1.0, wm, site ? h : NULL, &loss,
                                     gs, gH, &gJ, site ? gD : &gDu);
                bad |= st != ORC_OK;
                bad |= !finite_all(t, 3 * N) || !finite_all(gs, 3 * N) || !finite_all(gH, 3);
                bad |= !finite_all(e3, 3) || !isfinite(loss) || !isfinite(gJ);
            }
            free(s); free(t); free(h); free(Ds); free(es); free(gs); free(gD); free(ids);
        }
    }
    for (int32_t m = 0; m < 3; ++m) {
        double tt = orc_escape_time(1.0, 1.0, 0.1, 0.2, 1.0 / 6.0, 1.0, 1, m, 3, 0, 7, 50);
        bad |= !(tt >= -1.0);
    }
    bad |= orc_escape_time(1.0, 1.0, 0.1, 0.2, 0.1, 0.25, 1, 0, 3, 0, 7, 50) != -2.0;
    if (bad) {
        printf("non-finite result or error status\n");
        return 1;
    }
    printf("oracle sanitizer run ok\n");
    return 0;
}
