/*
 * FP64 CPU oracle of the two-phase WCSPH step (arXiv 1702.07760, Sec. II).
 * TEST INFRASTRUCTURE ONLY -- see sphx_oracle.h.
 *
 * Everything is evaluated the obvious way: one particle i at a time, its
 * neighbours j in ascending index order, full FP64, no blocking, no fusion.
 * Build with -ffp-contract=off so that every expression rounds as written.
 *
 * Readings where the paper is silent (kernel, self terms, time step,
 * integrator, wall properties) are the ones listed in the design notes:
 *   kernel      Wendland C2, support 2h;  grad_i W_ij = F(r) (x_i - x_j)
 *   neighbours  N(i) = { j != i : |x_i - x_j|^2 < 4 h^2 }, minimal image in
 *               periodic dimensions, |r|^2 = fma(rz,rz,fma(ry,ry,rx*rx))
 *   Eq. (7)     sums over i itself and its same-phase neighbours
 *   Eq. (15)    1/|grad C|, and T = 0 where grad C = 0
 *   walls       phase 0 (water); fixed position and velocity; density evolves
 *   time step   min of the CFL, force, viscous and capillary limits
 *   integrator  explicit midpoint predictor-corrector, neighbours rebuilt at
 *               the predicted positions
 */
#include "sphx_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

struct so_ctx {
    so_params p;
    so_phase ph[2];
    int32_t nphase;
    int64_t n;
    double *x, *u, *rho, *m, *x0;
    uint8_t *phase, *kind;
    double t;
    int64_t step;
    /* motion of the MOVING particles set from outside (so_set_moving): displacement
     * mv_disp + mv_vel (t - mv_t0) and velocity mv_vel, in place of the piston */
    int mv_host;
    double mv_disp[3], mv_vel[3], mv_t0;
    int32_t nb_method;
    int nb_valid;                 /* neighbour list matches the current positions */
    int64_t *nb_off;
    int32_t *nb_idx;
    int64_t nb_cap;
    double *P, *g, *T;            /* pressure, colour gradient (n x 3), tensor (n x 9) */
    double *drho, *a, *aP, *aV, *aS;
    double *s_drho, *s_aP, *s_aV, *s_aS;
    int have_rates;
};

/* ------------------------------------------------------------------ kernel */

static double kernel_alpha(int32_t dim, double h)
{
    return dim == 2 ? 7.0 / (4.0 * M_PI * h * h) : 21.0 / (16.0 * M_PI * h * h * h);
}

double so_kernel_w(int32_t dim, double h, double r)
{
    double q = r / h;
    if (q >= 2.0) return 0.0;
    double t = 1.0 - 0.5 * q;
    return kernel_alpha(dim, h) * t * t * t * t * (2.0 * q + 1.0);
}

/* dW/dr = -5 alpha q/h (1 - q/2)^3, so grad_i W_ij = dW/dr r_ij / r = F r_ij with
 * F = -5 alpha / h^2 (1 - q/2)^3 (no 1/r: r = 0 is harmless). */
double so_kernel_f(int32_t dim, double h, double r)
{
    double q = r / h;
    if (q >= 2.0) return 0.0;
    double t = 1.0 - 0.5 * q;
    return -5.0 * kernel_alpha(dim, h) / (h * h) * t * t * t;
}

/* --------------------------------------------------------- state equation */

double so_eos(double rho, double rho0, double c0, double gamma)
{
    double beta = rho0 * c0 * c0 / gamma;          /* Eq. (4) */
    return beta * (pow(rho / rho0, gamma) - 1.0);  /* Eq. (3) */
}

/* -------------------------------------------------------------- wavemaker */

void so_piston(const so_params* p, double t, double* d, double* v)
{
    double te = t < p->piston_t_end ? t : p->piston_t_end;
    double dd = 0.0, vv = 0.0;
    for (int k = 0; k < p->n_piston; ++k) {
        dd += p->piston_a[k] * (cos(p->piston_w[k] * te + p->piston_phi[k]) - cos(p->piston_phi[k]));
        if (t < p->piston_t_end)
            vv -= p->piston_a[k] * p->piston_w[k] * sin(p->piston_w[k] * t + p->piston_phi[k]);
    }
    *d = dd;
    *v = vv;
}

/* ------------------------------------------------------------- bookkeeping */

void so_set_threads(int32_t nthreads)
{
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
}

int32_t so_get_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

static void* xalloc(size_t bytes)
{
    void* q = calloc(bytes ? bytes : 1, 1);
    if (!q) abort();
    return q;
}

so_ctx* so_create(const so_params* p, const so_phase* phases, int32_t nphase, int64_t n,
                  const double* x, const double* u, const double* rho, const double* m,
                  const uint8_t* phase, const uint8_t* kind)
{
    if (!p || !phases || nphase < 1 || nphase > 2 || n < 0) return NULL;
    if (p->dim != 2 && p->dim != 3) return NULL;
    so_ctx* c = (so_ctx*)xalloc(sizeof(so_ctx));
    c->p = *p;
    c->nphase = nphase;
    for (int k = 0; k < nphase; ++k) c->ph[k] = phases[k];
    if (nphase == 1) c->ph[1] = phases[0];
    c->n = n;
    size_t n3 = (size_t)n * 3 * sizeof(double), n1 = (size_t)n * sizeof(double);
    c->x = xalloc(n3); c->u = xalloc(n3); c->x0 = xalloc(n3);
    c->rho = xalloc(n1); c->m = xalloc(n1);
    c->phase = xalloc((size_t)n); c->kind = xalloc((size_t)n);
    memcpy(c->x, x, n3); memcpy(c->x0, x, n3); memcpy(c->u, u, n3);
    memcpy(c->rho, rho, n1); memcpy(c->m, m, n1);
    memcpy(c->phase, phase, (size_t)n); memcpy(c->kind, kind, (size_t)n);
    c->P = xalloc(n1); c->g = xalloc(n3); c->T = xalloc(n3 * 3);
    c->drho = xalloc(n1); c->a = xalloc(n3); c->aP = xalloc(n3); c->aV = xalloc(n3); c->aS = xalloc(n3);
    c->s_drho = xalloc(n1); c->s_aP = xalloc(n1); c->s_aV = xalloc(n1); c->s_aS = xalloc(n1);
    c->nb_off = xalloc((size_t)(n + 1) * sizeof(int64_t));
    c->nb_cap = 0;
    c->nb_idx = NULL;
    return c;
}

void so_destroy(so_ctx* c)
{
    if (!c) return;
    void* all[] = {c->x, c->u, c->x0, c->rho, c->m, c->phase, c->kind, c->P, c->g, c->T,
                   c->drho, c->a, c->aP, c->aV, c->aS, c->s_drho, c->s_aP, c->s_aV, c->s_aS,
                   c->nb_off, c->nb_idx};
    for (size_t k = 0; k < sizeof(all) / sizeof(all[0]); ++k) free(all[k]);
    free(c);
}

void so_set_neighbor_method(so_ctx* c, int32_t method)
{
    c->nb_method = method;
    c->nb_valid = 0;
}

double so_time(const so_ctx* c) { return c->t; }
int64_t so_stepcount(const so_ctx* c) { return c->step; }

/* ------------------------------------------------------------- neighbours */

/* r_ij = x_i - x_j with the minimal image in periodic dimensions; returns |r|^2 */
static double pair_vector(const so_ctx* c, int64_t i, int64_t j, double r[3])
{
    for (int d = 0; d < 3; ++d) {
        if (d >= c->p.dim) { r[d] = 0.0; continue; }
        double v = c->x[3 * i + d] - c->x[3 * j + d];
        if (c->p.periodic[d]) {
            double L = c->p.hi[d] - c->p.lo[d];
            if (v > 0.5 * L) v -= L;
            else if (v < -0.5 * L) v += L;
        }
        r[d] = v;
    }
    return fma(r[2], r[2], fma(r[1], r[1], r[0] * r[0]));
}

static void ensure_nb_cap(so_ctx* c, int64_t total)
{
    if (total > c->nb_cap) {
        free(c->nb_idx);
        c->nb_cap = total + total / 8 + 16;
        c->nb_idx = (int32_t*)xalloc((size_t)c->nb_cap * sizeof(int32_t));
    }
}

static void nb_brute(so_ctx* c)
{
    const int64_t n = c->n;
    const double cut2 = 4.0 * c->p.h * c->p.h;
    int64_t* off = c->nb_off;
    off[0] = 0;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < n; ++i) {
        int64_t cnt = 0;
        double r[3];
        for (int64_t j = 0; j < n; ++j)
            if (j != i && pair_vector(c, i, j, r) < cut2) ++cnt;
        off[i + 1] = cnt;
    }
    for (int64_t i = 0; i < n; ++i) off[i + 1] += off[i];
    ensure_nb_cap(c, off[n]);
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < n; ++i) {
        int64_t k = off[i];
        double r[3];
        for (int64_t j = 0; j < n; ++j)
            if (j != i && pair_vector(c, i, j, r) < cut2) c->nb_idx[k++] = (int32_t)j;
    }
}

static void sort_ascending(int32_t* v, int64_t len)
{
    for (int64_t a = 1; a < len; ++a) {
        int32_t key = v[a];
        int64_t b = a - 1;
        while (b >= 0 && v[b] > key) { v[b + 1] = v[b]; --b; }
        v[b + 1] = key;
    }
}

/* Uniform cells of side >= 2h; the 3^dim surrounding cells hold every candidate.
 * Returns -1 when a periodic dimension has fewer than 3 cells. */
static int nb_cells(so_ctx* c)
{
    const int64_t n = c->n;
    const int dim = c->p.dim;
    const double h = c->p.h, cut2 = 4.0 * h * h;
    int64_t nc[3] = {1, 1, 1};
    double cs[3] = {1.0, 1.0, 1.0};
    for (int d = 0; d < dim; ++d) {
        double L = c->p.hi[d] - c->p.lo[d];
        int64_t k = (int64_t)floor(L / (2.0 * h));
        if (k < 1) k = 1;
        if (c->p.periodic[d] && k < 3) return -1;
        nc[d] = k;
        cs[d] = L / (double)k;
    }
    const int64_t ncell = nc[0] * nc[1] * nc[2];
    int64_t* kc = (int64_t*)xalloc((size_t)n * 3 * sizeof(int64_t));
    int64_t* cell = (int64_t*)xalloc((size_t)n * sizeof(int64_t));
    for (int64_t i = 0; i < n; ++i) {
        for (int d = 0; d < 3; ++d) {
            int64_t k = 0;
            if (d < dim) {
                k = (int64_t)floor((c->x[3 * i + d] - c->p.lo[d]) / cs[d]);
                if (k < 0) k = 0;
                if (k > nc[d] - 1) k = nc[d] - 1;
            }
            kc[3 * i + d] = k;
        }
        cell[i] = kc[3 * i] + nc[0] * (kc[3 * i + 1] + nc[1] * kc[3 * i + 2]);
    }
    int64_t* start = (int64_t*)xalloc((size_t)(ncell + 1) * sizeof(int64_t));
    int64_t* order = (int64_t*)xalloc((size_t)(n ? n : 1) * sizeof(int64_t));
    for (int64_t i = 0; i < n; ++i) start[cell[i] + 1]++;
    for (int64_t k = 0; k < ncell; ++k) start[k + 1] += start[k];
    int64_t* fill = (int64_t*)xalloc((size_t)(ncell + 1) * sizeof(int64_t));
    memcpy(fill, start, (size_t)(ncell + 1) * sizeof(int64_t));
    for (int64_t i = 0; i < n; ++i) order[fill[cell[i]]++] = i;
    free(fill);

    int64_t* off = c->nb_off;
    off[0] = 0;
    for (int pass = 0; pass < 2; ++pass) {
        if (pass == 1) {
            for (int64_t i = 0; i < n; ++i) off[i + 1] += off[i];
            ensure_nb_cap(c, off[n]);
        }
#pragma omp parallel for schedule(dynamic, 64)
        for (int64_t i = 0; i < n; ++i) {
            int64_t cnt = 0, base = pass ? off[i] : 0;
            double r[3];
            int64_t lo3[3], hi3[3];
            for (int d = 0; d < 3; ++d) {
                lo3[d] = d < dim ? -1 : 0;
                hi3[d] = d < dim ? 1 : 0;
            }
            for (int64_t d2 = lo3[2]; d2 <= hi3[2]; ++d2)
                for (int64_t d1 = lo3[1]; d1 <= hi3[1]; ++d1)
                    for (int64_t d0 = lo3[0]; d0 <= hi3[0]; ++d0) {
                        int64_t kk[3] = {kc[3 * i] + d0, kc[3 * i + 1] + d1, kc[3 * i + 2] + d2};
                        int skip = 0;
                        for (int d = 0; d < dim; ++d) {
                            if (c->p.periodic[d]) kk[d] = (kk[d] + nc[d]) % nc[d];
                            else if (kk[d] < 0 || kk[d] >= nc[d]) skip = 1;
                        }
                        if (skip) continue;
                        int64_t cc = kk[0] + nc[0] * (kk[1] + nc[1] * kk[2]);
                        for (int64_t s = start[cc]; s < start[cc + 1]; ++s) {
                            int64_t j = order[s];
                            if (j == i || pair_vector(c, i, j, r) >= cut2) continue;
                            if (pass) c->nb_idx[base + cnt] = (int32_t)j;
                            ++cnt;
                        }
                    }
            if (pass) sort_ascending(c->nb_idx + base, cnt);
            else off[i + 1] = cnt;
        }
    }
    free(kc); free(cell); free(start); free(order);
    return 0;
}

static void build_neighbors(so_ctx* c)
{
    if (c->nb_valid) return;
    int method = c->nb_method;
    if (method == 0) method = c->n <= 5000 ? 1 : 2;
    if (method == 2 && nb_cells(c) == 0) {
        c->nb_valid = 1;
        return;
    }
    nb_brute(c);
    c->nb_valid = 1;
}

int64_t so_neighbors(so_ctx* c, int64_t* off, int32_t* idx, int64_t cap)
{
    build_neighbors(c);
    int64_t total = c->nb_off[c->n];
    if (off) memcpy(off, c->nb_off, (size_t)(c->n + 1) * sizeof(int64_t));
    if (idx && cap >= total) memcpy(idx, c->nb_idx, (size_t)total * sizeof(int32_t));
    return total;
}

/* ------------------------------------------------- Eq. (7) renormalisation */

void so_renormalize(so_ctx* c)
{
    build_neighbors(c);
    const int64_t n = c->n;
    const int dim = c->p.dim;
    const double h = c->p.h;
    const double w0 = so_kernel_w(dim, h, 0.0);
    double* rn = (double*)xalloc((size_t)n * sizeof(double));
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t i = 0; i < n; ++i) {
        double num = c->m[i] * w0;                 /* j = i */
        double den = c->m[i] / c->rho[i] * w0;
        double r[3];
        for (int64_t k = c->nb_off[i]; k < c->nb_off[i + 1]; ++k) {
            int64_t j = c->nb_idx[k];
            if (c->phase[j] != c->phase[i]) continue;   /* only the n' same-phase particles */
            double w = so_kernel_w(dim, h, sqrt(pair_vector(c, i, j, r)));
            num += c->m[j] * w;
            den += c->m[j] / c->rho[j] * w;
        }
        rn[i] = num / den;
    }
    memcpy(c->rho, rn, (size_t)n * sizeof(double));
    free(rn);
    c->have_rates = 0;
}

/* ------------------------------------------------------------------ rates */

typedef struct {
    double cont;     /* continuity: V_j u_ij . gradW (Eq. 6) or m_j u_ij . gradW (Eq. 5) */
    double mp[3];    /* m_i times the pressure contribution, Eq. (8) */
    double v[3];     /* Eq. (10): the contribution itself; Eq. (11): m_i times it */
    double ms[3];    /* m_i times the surface-tension contribution, Eq. (17) */
} pair_t;

static void pair_terms_at(const so_ctx* c, int64_t i, int64_t j, const double r[3], double r2,
                          pair_t* o)
{
    const int dim = c->p.dim;
    const double h = c->p.h;
    const double F = so_kernel_f(dim, h, sqrt(r2));
    double gw[3], uij[3];
    for (int d = 0; d < 3; ++d) {
        gw[d] = F * r[d];                            /* grad_i W_ij */
        uij[d] = c->u[3 * i + d] - c->u[3 * j + d];  /* u_ij = u_i - u_j */
    }
    const double Vi = c->m[i] / c->rho[i], Vj = c->m[j] / c->rho[j];
    const double udg = uij[0] * gw[0] + uij[1] * gw[1] + uij[2] * gw[2];
    o->cont = (c->p.cont_form == 1 ? c->m[j] : Vj) * udg;

    /* Eq. (8): -(m_i m_j)(P_i/rho_i^2 + P_j/rho_j^2) grad_i W_ij */
    const double Ai = c->P[i] / (c->rho[i] * c->rho[i]);
    const double Aj = c->P[j] / (c->rho[j] * c->rho[j]);
    const double cp = (c->m[i] * c->m[j]) * (Ai + Aj);
    for (int d = 0; d < 3; ++d) o->mp[d] = -(cp * gw[d]);

    /* Eqs. (10)-(13): r_ij . grad_i W_ij / (|r_ij|^2 + delta^2) */
    const double delta = c->p.delta_coef * h;
    const double rgw = r[0] * gw[0] + r[1] * gw[1] + r[2] * gw[2];
    const double lap = rgw / (r2 + delta * delta);
    const so_phase* pi = &c->ph[c->phase[i]];
    const so_phase* pj = &c->ph[c->phase[j]];
    double cv;
    if (c->p.visc_form == 1) {
        double mui = pi->nu * pi->rho0, muj = pj->nu * pj->rho0;
        double muij = (mui + muj) > 0.0 ? 2.0 * mui * muj / (mui + muj) : 0.0;  /* Eq. (13) */
        cv = (Vi * Vj) * (2.0 * muij) * lap;
    } else {
        double nuij = (pi->nu + pj->nu) > 0.0 ? 2.0 * pi->nu * pj->nu / (pi->nu + pj->nu) : 0.0; /* Eq. (12) */
        cv = Vj * (2.0 * nuij) * lap;
    }
    for (int d = 0; d < 3; ++d) o->v[d] = cv * uij[d];

    /* Eq. (17) times m_i: (T_i / sigma_i^2 + T_j / sigma_j^2) . grad_i W_ij, 1/sigma = V */
    const double* Ti = c->T + 9 * i;
    const double* Tj = c->T + 9 * j;
    for (int a = 0; a < 3; ++a) {
        double s = 0.0;
        for (int b = 0; b < 3; ++b) s += (Ti[3 * a + b] * (Vi * Vi) + Tj[3 * a + b] * (Vj * Vj)) * gw[b];
        o->ms[a] = s;
    }
}

static double norm3(const double v[3]) { return sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]); }

static void compute_rates(so_ctx* c)
{
    build_neighbors(c);
    const int64_t n = c->n;
    const int dim = c->p.dim;
    const double h = c->p.h;

    /* Eqs. (3)-(4) */
    for (int64_t i = 0; i < n; ++i) {
        const so_phase* ph = &c->ph[c->phase[i]];
        c->P[i] = so_eos(c->rho[i], ph->rho0, ph->c0, c->p.gamma);
    }

    /* Eq. (16) with C_i^y = 0, sigma = rho / m; then Eq. (15) */
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t i = 0; i < n; ++i) {
        double s[3] = {0.0, 0.0, 0.0}, r[3];
        for (int64_t k = c->nb_off[i]; k < c->nb_off[i + 1]; ++k) {
            int64_t j = c->nb_idx[k];
            if (c->phase[j] == c->phase[i]) continue;     /* C_j^y = 1 only for the other phase */
            double r2 = pair_vector(c, i, j, r);
            double F = so_kernel_f(dim, h, sqrt(r2));
            double sj = c->rho[j] / c->m[j];
            for (int d = 0; d < 3; ++d) s[d] += (F * r[d]) / (sj * sj);
        }
        double si = c->rho[i] / c->m[i];
        double* gi = c->g + 3 * i;
        for (int d = 0; d < 3; ++d) gi[d] = si * s[d];
        double gn = norm3(gi);
        double* Ti = c->T + 9 * i;
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) {
                double v = 0.0;
                if (gn > 0.0) {
                    double iso = (a == b && a < dim) ? gn * gn / (double)dim : 0.0;
                    v = c->p.alpha_s * (iso - gi[a] * gi[b]) / gn;
                }
                Ti[3 * a + b] = v;
            }
    }

    /* Eqs. (6), (8), (10)/(11), (17) and gravity */
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t i = 0; i < n; ++i) {
        double cs = 0.0, scs = 0.0;
        double sp[3] = {0, 0, 0}, sv[3] = {0, 0, 0}, ss[3] = {0, 0, 0};
        double ssp = 0.0, ssv = 0.0, sss = 0.0;
        double r[3];
        const double rho_fac = c->p.cont_form == 1 ? 1.0 : c->rho[i];
        for (int64_t k = c->nb_off[i]; k < c->nb_off[i + 1]; ++k) {
            int64_t j = c->nb_idx[k];
            double r2 = pair_vector(c, i, j, r);
            pair_t t;
            pair_terms_at(c, i, j, r, r2, &t);
            cs += t.cont;
            scs += fabs(rho_fac * t.cont);
            for (int d = 0; d < 3; ++d) { sp[d] += t.mp[d]; sv[d] += t.v[d]; ss[d] += t.ms[d]; }
            ssp += norm3(t.mp);
            ssv += norm3(t.v);
            sss += norm3(t.ms);
        }
        c->drho[i] = rho_fac * cs;
        c->s_drho[i] = scs;
        const double mi = c->m[i];
        const double vfac = c->p.visc_form == 1 ? 1.0 / mi : 1.0;
        const int fluid = c->kind[i] == SO_FLUID;
        for (int d = 0; d < 3; ++d) {
            double ap = fluid ? sp[d] / mi : 0.0;
            double av = fluid ? sv[d] * vfac : 0.0;
            double as = fluid ? ss[d] / mi : 0.0;
            c->aP[3 * i + d] = ap;
            c->aV[3 * i + d] = av;
            c->aS[3 * i + d] = as;
            c->a[3 * i + d] = fluid ? ap + av + as + (d < dim ? c->p.gravity[d] : 0.0) : 0.0;
        }
        c->s_aP[i] = fluid ? ssp / mi : 0.0;
        c->s_aV[i] = fluid ? ssv * vfac : 0.0;
        c->s_aS[i] = fluid ? sss / mi : 0.0;
    }
    c->have_rates = 1;
}

int64_t so_rates(so_ctx* c)
{
    compute_rates(c);
    return c->nb_off[c->n];
}

int32_t so_pair_terms(const so_ctx* c, int64_t i, int64_t j, double* out)
{
    if (!c->have_rates || i < 0 || j < 0 || i >= c->n || j >= c->n) return -1;
    int found = 0;
    for (int64_t k = c->nb_off[i]; k < c->nb_off[i + 1]; ++k)
        if (c->nb_idx[k] == j) found = 1;
    if (!found) return -1;
    double r[3];
    double r2 = pair_vector(c, i, j, r);
    pair_t t;
    pair_terms_at(c, i, j, r, r2, &t);
    for (int d = 0; d < 3; ++d) {
        out[d] = t.mp[d];
        out[3 + d] = t.v[d];
        out[6 + d] = t.ms[d];
    }
    out[9] = t.cont;
    return 0;
}

/* -------------------------------------------------------------- time step */

double so_dt(so_ctx* c)
{
    if (c->p.dt_fixed > 0.0) return c->p.dt_fixed;
    if (!c->have_rates) compute_rates(c);
    const double h = c->p.h;
    double umax = 0.0, amax = 0.0;
    for (int64_t i = 0; i < c->n; ++i) {
        if (c->kind[i] == SO_WALL) continue;
        double un = norm3(c->u + 3 * i);
        if (un > umax) umax = un;
        if (c->kind[i] == SO_FLUID) {
            double an = norm3(c->a + 3 * i);
            if (an > amax) amax = an;
        }
    }
    double cmax = 0.0, numax = 0.0, rho0min = INFINITY;
    for (int k = 0; k < c->nphase; ++k) {
        if (c->ph[k].c0 > cmax) cmax = c->ph[k].c0;
        if (c->ph[k].nu > numax) numax = c->ph[k].nu;
        if (c->ph[k].rho0 < rho0min) rho0min = c->ph[k].rho0;
    }
    double dt = c->p.c_cfl * h / (cmax + umax);
    if (amax > 0.0) dt = fmin(dt, c->p.c_force * sqrt(h / amax));
    if (numax > 0.0) dt = fmin(dt, c->p.c_visc * h * h / numax);
    if (c->p.alpha_s > 0.0 && c->nphase == 2)
        dt = fmin(dt, c->p.c_st * sqrt(rho0min * h * h * h / (2.0 * M_PI * c->p.alpha_s)));
    return dt;
}

/* ------------------------------------------------------------- integrator */

static void wrap_periodic(so_ctx* c, int64_t i)
{
    for (int d = 0; d < c->p.dim; ++d) {
        if (!c->p.periodic[d]) continue;
        double L = c->p.hi[d] - c->p.lo[d];
        double* v = c->x + 3 * i + d;
        if (*v >= c->p.hi[d]) *v -= L;
        else if (*v < c->p.lo[d]) *v += L;
    }
}

/* x = xn + f dt v, u = un + f dt a, rho = rhon + f dt drho, with the rates of the
 * current state c->a, c->drho and the velocity v of the current state. */
static void advance(so_ctx* c, const double* xn, const double* un, const double* rhon,
                    double fdt, double t_new)
{
    /* displacement and velocity of the MOVING particles at t_new */
    double dmv[3] = {0.0, 0.0, 0.0}, vmv[3] = {0.0, 0.0, 0.0};
    if (c->mv_host) {
        for (int d = 0; d < 3; ++d) {
            dmv[d] = c->mv_disp[d] + c->mv_vel[d] * (t_new - c->mv_t0);
            vmv[d] = c->mv_vel[d];
        }
    } else {
        so_piston(&c->p, t_new, &dmv[0], &vmv[0]);
    }
    const int64_t n = c->n;
    for (int64_t i = 0; i < n; ++i) {
        double xi[3], ui[3];
        if (c->kind[i] == SO_FLUID) {
            for (int d = 0; d < 3; ++d) {
                xi[d] = xn[3 * i + d] + fdt * c->u[3 * i + d];
                ui[d] = un[3 * i + d] + fdt * c->a[3 * i + d];
            }
        } else if (c->kind[i] == SO_MOVING) {
            for (int d = 0; d < 3; ++d) {
                xi[d] = c->x0[3 * i + d] + dmv[d];
                ui[d] = vmv[d];
            }
        } else {
            for (int d = 0; d < 3; ++d) {
                xi[d] = xn[3 * i + d];
                ui[d] = un[3 * i + d];
            }
        }
        for (int d = 0; d < 3; ++d) {
            c->x[3 * i + d] = xi[d];
            c->u[3 * i + d] = ui[d];
        }
        c->rho[i] = rhon[i] + fdt * c->drho[i];
        wrap_periodic(c, i);
    }
    c->nb_valid = 0;
    c->have_rates = 0;
}

void so_set_moving(so_ctx* c, const double disp[3], const double vel[3])
{
    c->mv_host = 1;
    for (int d = 0; d < 3; ++d) {
        c->mv_disp[d] = d < c->p.dim ? disp[d] : 0.0;
        c->mv_vel[d] = d < c->p.dim ? vel[d] : 0.0;
    }
    c->mv_t0 = c->t;
    /* the MOVING particles take the new motion at once: reference position + disp,
     * velocity vel */
    for (int64_t i = 0; i < c->n; ++i) {
        if (c->kind[i] != SO_MOVING) continue;
        for (int d = 0; d < 3; ++d) {
            c->x[3 * i + d] = c->x0[3 * i + d] + c->mv_disp[d];
            c->u[3 * i + d] = c->mv_vel[d];
        }
    }
    c->nb_valid = 0;
    c->have_rates = 0;
}

int64_t so_step(so_ctx* c, int32_t nsteps)
{
    const int64_t n = c->n;
    double* xn = (double*)xalloc((size_t)n * 3 * sizeof(double));
    double* un = (double*)xalloc((size_t)n * 3 * sizeof(double));
    double* rn = (double*)xalloc((size_t)n * sizeof(double));
    int64_t inter = 0;
    for (int32_t s = 0; s < nsteps; ++s) {
        if (c->p.renorm_every > 0 && c->step % c->p.renorm_every == 0) so_renormalize(c);
        inter += so_rates(c);                                  /* R(S^n) */
        const double dt = so_dt(c);
        memcpy(xn, c->x, (size_t)n * 3 * sizeof(double));
        memcpy(un, c->u, (size_t)n * 3 * sizeof(double));
        memcpy(rn, c->rho, (size_t)n * sizeof(double));
        advance(c, xn, un, rn, 0.5 * dt, c->t + 0.5 * dt);     /* S* */
        inter += so_rates(c);                                  /* R(S*) at N(x*) */
        advance(c, xn, un, rn, dt, c->t + dt);                 /* S^{n+1} */
        c->t += dt;
        c->step += 1;
    }
    free(xn); free(un); free(rn);
    return inter;
}

/* ---------------------------------------------------------------- get/set */

int32_t so_get(const so_ctx* c, int32_t field, double* out)
{
    const size_t n1 = (size_t)c->n * sizeof(double), n3 = 3 * n1;
    switch (field) {
    case SO_X: memcpy(out, c->x, n3); return 0;
    case SO_U: memcpy(out, c->u, n3); return 0;
    case SO_RHO: memcpy(out, c->rho, n1); return 0;
    case SO_A: memcpy(out, c->a, n3); return 0;
    case SO_DRHO: memcpy(out, c->drho, n1); return 0;
    case SO_AP: memcpy(out, c->aP, n3); return 0;
    case SO_AV: memcpy(out, c->aV, n3); return 0;
    case SO_AS: memcpy(out, c->aS, n3); return 0;
    case SO_SDRHO: memcpy(out, c->s_drho, n1); return 0;
    case SO_SAP: memcpy(out, c->s_aP, n1); return 0;
    case SO_SAV: memcpy(out, c->s_aV, n1); return 0;
    case SO_SAS: memcpy(out, c->s_aS, n1); return 0;
    case SO_P: memcpy(out, c->P, n1); return 0;
    case SO_GRADC: memcpy(out, c->g, n3); return 0;
    case SO_TENSOR: memcpy(out, c->T, 3 * n3); return 0;
    default: return -1;
    }
}

int32_t so_set(so_ctx* c, int32_t field, const double* in)
{
    const size_t n1 = (size_t)c->n * sizeof(double), n3 = 3 * n1;
    switch (field) {
    case SO_X: memcpy(c->x, in, n3); c->nb_valid = 0; break;
    case SO_U: memcpy(c->u, in, n3); break;
    case SO_RHO: memcpy(c->rho, in, n1); break;
    default: return -1;
    }
    c->have_rates = 0;
    return 0;
}
