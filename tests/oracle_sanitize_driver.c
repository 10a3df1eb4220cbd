/*
 * Drives every entry point of the FP64 oracle on two small scenes, for a build
 * with the address and undefined-behaviour sanitizers (tests/test_oracle_sanitize.py).
 * Exit status 0 when every call returned sensible values; the sanitizers abort on
 * any invalid access or undefined operation.
 *
 * Scene A (2D): a walled tank with an oil drop and a one-column piston of MOVING
 * particles, seeded velocities.  Scene B (3D): a periodic two-phase lattice box.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "sphx_oracle.h"

static uint64_t lcg = 88172645463325252ull;
static double urand(void) /* uniform in [-1, 1) */
{
    lcg = lcg * 6364136223846793005ull + 1442695040888963407ull;
    return (double)(lcg >> 11) / 4503599627370496.0 - 1.0;
}

static so_params base_params(int dim, double h)
{
    so_params p;
    memset(&p, 0, sizeof p);
    p.dim = dim;
    p.renorm_every = 1;
    p.h = h;
    p.gamma = 7.0;
    p.delta_coef = 0.1;
    p.alpha_s = 0.02;
    p.c_cfl = 0.25;
    p.c_force = 0.25;
    p.c_visc = 0.125;
    p.c_st = 0.25;
    return p;
}

static int finite_all(const double* v, int64_t n)
{
    for (int64_t i = 0; i < n; ++i)
        if (!isfinite(v[i])) return 0;
    return 1;
}

/* Every call of the oracle on one scene; returns 0 when all is well. */
static int exercise(const so_params* p, const so_phase* ph, int64_t n, const double* x, const double* u,
                    const double* rho, const double* m, const uint8_t* phase, const uint8_t* kind, int moving)
{
    so_ctx* c = so_create(p, ph, 2, n, x, u, rho, m, phase, kind);
    if (!c) return 1;
    int64_t* off = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
    int64_t tot[2] = {0, 0};
    for (int method = 1; method <= 2; ++method) {
        so_set_neighbor_method(c, method);
        tot[method - 1] = so_neighbors(c, off, NULL, 0);
        int32_t* idx = (int32_t*)calloc((size_t)tot[method - 1] + 1, sizeof(int32_t));
        if (so_neighbors(c, off, idx, tot[method - 1]) != tot[method - 1]) return 2;
        if (off[n] != tot[method - 1]) return 3;
        free(idx);
    }
    if (tot[0] != tot[1] || tot[0] == 0) return 4;
    so_renormalize(c);
    if (so_rates(c) <= 0) return 5;
    if (!(so_dt(c) > 0.0)) return 6;
    double* f = (double*)calloc((size_t)n * 9, sizeof(double));
    const int fields[] = {SO_X, SO_U, SO_RHO, SO_A, SO_DRHO, SO_AP, SO_AV, SO_AS, SO_SDRHO,
                          SO_SAP, SO_SAV, SO_SAS, SO_P, SO_GRADC, SO_TENSOR};
    for (size_t k = 0; k < sizeof fields / sizeof fields[0]; ++k) {
        if (so_get(c, fields[k], f) != 0) return 7;
        const int64_t w = fields[k] == SO_TENSOR ? 9 : (fields[k] == SO_RHO || fields[k] == SO_DRHO ||
                                                        fields[k] == SO_P || fields[k] == SO_SDRHO) ? 1 : 3;
        if (!finite_all(f, n * w)) return 8;
    }
    double terms[10];
    if (so_pair_terms(c, 0, 0, terms) != -1) return 9;   /* i is not its own neighbour */
    if (so_step(c, 3) <= 0) return 10;
    if (moving) {
        const double disp[3] = {0.0005, 0.0, 0.0}, vel[3] = {0.05, 0.0, 0.0};
        so_set_moving(c, disp, vel);
    }
    so_set_threads(1);
    if (so_step(c, 2) <= 0) return 11;
    if (so_stepcount(c) != 5 || !(so_time(c) > 0.0)) return 12;
    if (so_get(c, SO_X, f) != 0 || !finite_all(f, n * 3)) return 13;
    if (so_set(c, SO_U, f) != 0) return 14;   /* any finite array is a valid state */
    free(f);
    free(off);
    so_destroy(c);
    return 0;
}

int main(void)
{
    const double dx = 1e-3, h = 1.3e-3;
    const so_phase ph[2] = {{1000.0, 1e-6, 10.0}, {900.0, 5e-6, 10.0}};
    double w[3], vv[3];
    (void)so_kernel_w(2, h, 0.5 * h);
    (void)so_kernel_f(3, h, 0.5 * h);
    (void)so_eos(1001.0, 1000.0, 10.0, 7.0);

    /* scene A: 2D tank 20 x 16 fluid, three wall layers, piston column at x < 0 */
    {
        const int nx = 20, ny = 16, L = 3;
        const int64_t cap = (int64_t)(nx + 2 * L) * (ny + L + 4);
        double *x = calloc((size_t)cap * 3, sizeof(double)), *u = calloc((size_t)cap * 3, sizeof(double));
        double *rho = calloc((size_t)cap, sizeof(double)), *m = calloc((size_t)cap, sizeof(double));
        uint8_t *phase = calloc((size_t)cap, 1), *kind = calloc((size_t)cap, 1);
        int64_t n = 0;
        for (int j = -L; j < ny + 4; ++j)
            for (int i = -L; i < nx + L; ++i) {
                const int inside = i >= 0 && i < nx && j >= 0;
                if (inside && j >= ny) continue;                 /* free surface */
                x[3 * n] = (i + 0.5) * dx;
                x[3 * n + 1] = (j + 0.5) * dx;
                kind[n] = inside ? SO_FLUID : (i == -1 && j >= 0 ? SO_MOVING : SO_WALL);
                const double cx = (i + 0.5) - 10.0, cy = (j + 0.5) - 6.0;
                phase[n] = inside && cx * cx + cy * cy < 16.0 ? 1 : 0;
                rho[n] = ph[phase[n]].rho0 * (1.0 + 0.003 * urand());
                m[n] = ph[phase[n]].rho0 * dx * dx;
                if (inside) {
                    u[3 * n] = 0.05 * urand();
                    u[3 * n + 1] = 0.05 * urand();
                }
                ++n;
            }
        so_params p = base_params(2, h);
        p.gravity[1] = -9.81;
        p.lo[0] = -L * dx; p.hi[0] = (nx + L) * dx;
        p.lo[1] = -L * dx; p.hi[1] = 2.0 * (ny + 4) * dx;
        p.n_piston = 1;
        p.piston_a[0] = -0.002;
        p.piston_w[0] = 10.0;
        p.piston_t_end = 1.0;
        so_piston(&p, 0.01, &w[0], &vv[0]);
        const int rc = exercise(&p, ph, n, x, u, rho, m, phase, kind, 1);
        if (rc) { fprintf(stderr, "scene A failed at check %d\n", rc); return rc; }
        free(x); free(u); free(rho); free(m); free(phase); free(kind);
    }
    /* scene B: 3D periodic 8^3 lattice with an oil ball, Eq. (11) and Eq. (5) forms */
    {
        const int k = 8;
        const int64_t n = (int64_t)k * k * k;
        double *x = calloc((size_t)n * 3, sizeof(double)), *u = calloc((size_t)n * 3, sizeof(double));
        double *rho = calloc((size_t)n, sizeof(double)), *m = calloc((size_t)n, sizeof(double));
        uint8_t *phase = calloc((size_t)n, 1), *kind = calloc((size_t)n, 1);
        int64_t q = 0;
        for (int a = 0; a < k; ++a)
            for (int b = 0; b < k; ++b)
                for (int c = 0; c < k; ++c, ++q) {
                    x[3 * q] = (a + 0.5 + 0.05 * urand()) * dx;
                    x[3 * q + 1] = (b + 0.5 + 0.05 * urand()) * dx;
                    x[3 * q + 2] = (c + 0.5 + 0.05 * urand()) * dx;
                    const double r2 = (a - 3.5) * (a - 3.5) + (b - 3.5) * (b - 3.5) + (c - 3.5) * (c - 3.5);
                    phase[q] = r2 < 6.0 ? 1 : 0;
                    rho[q] = ph[phase[q]].rho0 * (1.0 + 0.003 * urand());
                    m[q] = ph[phase[q]].rho0 * dx * dx * dx;
                    for (int d = 0; d < 3; ++d) u[3 * q + d] = 0.05 * urand();
                }
        so_params p = base_params(3, h);
        p.visc_form = 1;
        p.cont_form = 1;
        for (int d = 0; d < 3; ++d) {
            p.lo[d] = 0.0;
            p.hi[d] = k * dx;
            p.periodic[d] = 1;
        }
        const int rc = exercise(&p, ph, n, x, u, rho, m, phase, kind, 0);
        if (rc) { fprintf(stderr, "scene B failed at check %d\n", rc); return 100 + rc; }
        free(x); free(u); free(rho); free(m); free(phase); free(kind);
    }
    printf("oracle driver ok\n");
    return 0;
}
