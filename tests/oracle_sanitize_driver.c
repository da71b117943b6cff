/* Runs the FP64 oracle (oracle/swe_oracle.c, compiled into this program)
 * over small cases covering every boundary kind, friction law, land mask,
 * wet-dry front, uniform and gridded wind, gridded stress, nested boundary
 * snapshots and the time-step update policy, through each of its entry
 * points.  Built with AddressSanitizer and UndefinedBehaviorSanitizer by
 * tests/test_host_sanitized.py: any out-of-bounds access, use of
 * uninitialised heap memory through a sanitizer report, or undefined
 * arithmetic stops the run.  Exit 0 when every result is finite. */
#include "swe_oracle.h"

#include <math.h>
#include <stdio.h>
#include <stdlib.h>

static unsigned long long g_state = 88172645463325252ULL;
static double urand(void)
{
    g_state ^= g_state << 13;
    g_state ^= g_state >> 7;
    g_state ^= g_state << 17;
    return (double)(g_state >> 11) / 9007199254740992.0;
}

static int all_finite(const double *a, size_t n)
{
    for (size_t k = 0; k < n; ++k)
        if (!isfinite(a[k])) return 0;
    return 1;
}

static int run_case(int nx, int ny, const int bc[4], int friction, int land_on, int wet_dry, int w10_kind,
                    double dt_interval)
{
    const size_t nc = (size_t)nx * ny, nk = (size_t)(nx + 1) * (ny + 1), P = 2 * (size_t)nx + 2 * (size_t)ny;
    double *Hc = malloc(nk * sizeof(double)), *f = malloc(nc * sizeof(double)), *north = malloc(nc * sizeof(double));
    double *eta = malloc(nc * sizeof(double)), *hu = malloc(nc * sizeof(double)), *hv = malloc(nc * sizeof(double));
    unsigned char *land = land_on ? malloc(nc) : NULL;
    for (int j = 0; j <= ny; ++j)
        for (int i = 0; i <= nx; ++i) {
            double H = 30.0 + 20.0 * sin(0.3 * i) * cos(0.2 * j) + 5.0 * urand();
            if (wet_dry && i > nx / 2) H = 2.0 - 0.8 * (i - nx / 2);  /* a beach rising above the datum */
            Hc[(size_t)j * (nx + 1) + i] = H;
        }
    if (bc[0] == OR_BC_PERIODIC)
        for (int j = 0; j <= ny; ++j) Hc[(size_t)j * (nx + 1) + nx] = Hc[(size_t)j * (nx + 1)];
    if (bc[2] == OR_BC_PERIODIC)
        for (int i = 0; i <= nx; ++i) Hc[(size_t)ny * (nx + 1) + i] = Hc[i];
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            const size_t o = (size_t)j * nx + i;
            const double Hb = 0.25 * (Hc[(size_t)j * (nx + 1) + i] + Hc[(size_t)j * (nx + 1) + i + 1] +
                                      Hc[(size_t)(j + 1) * (nx + 1) + i] + Hc[(size_t)(j + 1) * (nx + 1) + i + 1]);
            f[o] = 1.1e-4 + 2e-6 * j;
            north[o] = 0.3 * urand();
            eta[o] = 0.2 * sin(0.5 * i + 0.3 * j);
            if (eta[o] + Hb < 0.0) eta[o] = -Hb;
            hu[o] = Hb > 0.5 ? 0.5 * urand() : 0.0;
            hv[o] = Hb > 0.5 ? -0.3 * urand() : 0.0;
            if (land) land[o] = (urand() < 0.15) ? 1 : 0;
        }
    /* the wet-dry cases run unforced: stress on a dry beach accelerates the
     * desingularised velocity there (no configuration forces a front) */
    double wind_t[2] = {0.0, 100.0}, wind_tau[4] = {0.1, -0.05, 0.02, 0.08};
    if (wet_dry)
        for (int k = 0; k < 4; ++k) wind_tau[k] = 0.0;
    double bnd_t[3] = {0.0, 50.0, 200.0};
    double *bnd = malloc(3 * 3 * P * sizeof(double));
    for (size_t k = 0; k < 3 * 3 * P; ++k) bnd[k] = (k % 3 == 0) ? 0.1 * urand() : 0.01 * urand();
    const int nxw = 4, nyw = 3;
    double w10_t[2] = {0.0, 300.0};
    double *w10 = malloc(2 * (size_t)nyw * nxw * 2 * sizeof(double));
    for (size_t k = 0; k < 2 * (size_t)nyw * nxw * 2; ++k) w10[k] = w10_kind ? 0.1 * urand() : 15.0 * urand() - 5.0;

    or_params p = {0};
    p.nx = nx; p.ny = ny; p.dx = 500.0; p.dy = 700.0; p.g = 9.81; p.courant = 0.45; p.theta = 1.3; p.kappa = 1e-3;
    for (int k = 0; k < 4; ++k) p.bc[k] = bc[k];
    p.friction = friction;
    p.friction_coeff = friction == OR_FRIC_MANNING ? 0.03 : 3e-3;
    p.rho_w = 1025.0; p.frs_width = 10; p.frs_d0 = 2.0;
    p.wind_n = 2; p.wind_t = wind_t; p.wind_tau = wind_tau;
    const int nested = bc[0] == OR_BC_NESTED || bc[1] == OR_BC_NESTED || bc[2] == OR_BC_NESTED || bc[3] == OR_BC_NESTED;
    p.bnd_n = nested ? 3 : 0; p.bnd_t = bnd_t; p.bnd = bnd;
    if (w10_kind >= 0) { p.w10_n = 2; p.w10_nx = nxw; p.w10_ny = nyw; p.w10_t = w10_t; p.w10 = w10; p.w10_kind = w10_kind; }
    p.rho_a = 1.225;
    p.dt_interval = dt_interval;
    or_static s = {Hc, land, f, north};

    double *M = malloc(3 * nc * sizeof(double)), *faces = malloc(12 * nc * sizeof(double)), *S = malloc(nc * sizeof(double));
    double dts[40];
    int ok = 1;
    ok &= or_rhs(&p, &s, eta, hu, hv, 3.0, M, M + nc, M + 2 * nc, faces) == 0 && all_finite(M, 3 * nc) &&
          all_finite(faces, 12 * nc);
    ok &= or_friction(&p, &s, eta, hu, hv, S) == 0 && all_finite(S, nc);
    const double dt = or_cfl_dt(&p, &s, eta, hu, hv);
    ok &= dt > 0.0;
    double t = 0.0;
    ok &= or_step(&p, &s, eta, hu, hv, &t, isfinite(dt) ? dt : 1.0) == 0;
    ok &= or_run(&p, &s, eta, hu, hv, &t, 30, 0.0, 0.0, NULL, dts) == 30;
    const int64_t k_end = or_run(&p, &s, eta, hu, hv, &t, 400, t + 40.0, 0.0, NULL, NULL);
    ok &= k_end >= 1 && k_end <= 400;
    ok &= or_run(&p, &s, eta, hu, hv, &t, 5, 0.0, 0.0, dts, NULL) == 5;
    double mass, energy;
    or_diagnostics(&p, &s, eta, hu, hv, &mass, &energy);
    ok &= isfinite(mass) && isfinite(energy) && all_finite(eta, nc) && all_finite(hu, nc) && all_finite(hv, nc);
    free(Hc); free(f); free(north); free(eta); free(hu); free(hv); free(land); free(bnd); free(w10);
    free(M); free(faces); free(S);
    if (!ok) printf("FAIL case %dx%d bc %d %d %d %d friction %d land %d wet-dry %d w10 %d\n", nx, ny, bc[0], bc[1], bc[2],
                    bc[3], friction, land_on, wet_dry, w10_kind);
    return ok;
}

int main(void)
{
    const int bcs[][4] = {{0, 0, 0, 0}, {1, 1, 1, 1}, {2, 2, 2, 2}, {2, 0, 1, 1}, {1, 1, 2, 0}, {0, 2, 0, 2}};
    const int shapes[][2] = {{2, 2}, {3, 5}, {13, 9}, {24, 17}};
    int bad = 0, n = 0;
    for (size_t b = 0; b < sizeof bcs / sizeof bcs[0]; ++b)
        for (size_t sh = 0; sh < sizeof shapes / sizeof shapes[0]; ++sh)
            for (int fr = 0; fr < 4; ++fr) {
                const int land_on = (int)((b + sh + fr) % 2), wet_dry = fr == OR_FRIC_MANNING;
                const int w10 = wet_dry ? -1 : (int)((b + fr) % 3) - 1;  /* none, wind at 10 m, stress */
                const double dti = (sh == 2 && fr == 1) ? 7.0 : 0.0;
                /* nested data is not made consistent with a beach above the
                 * datum: the wet-dry cases take walls where a side is nested */
                int bc[4];
                for (int k = 0; k < 4; ++k) bc[k] = (wet_dry && bcs[b][k] == OR_BC_NESTED) ? OR_BC_WALL : bcs[b][k];
                bad += !run_case(shapes[sh][0], shapes[sh][1], bc, fr, land_on, wet_dry, w10, dti);
                ++n;
            }
    printf("oracle cases %d bad %d\n", n, bad);
    return bad != 0;
}
