/*
 * FP64 CPU oracle of the two-phase weakly compressible SPH step of
 * Wei et al., "Behavior of Oil under Breaking Waves by a Two-phase SPH Model"
 * (arXiv 1702.07760), Sec. II, Eqs. (1)-(17), plus the readings documented in
 * the repository design notes where the paper is silent (kernel, time step,
 * integrator).
 *
 * TEST INFRASTRUCTURE ONLY.  This library is plain, slow and written to be
 * checked against the paper by eye.  It shares no code, header, table or
 * helper with the GPU library; only the tests, the smoke check and the CPU
 * baseline leg of the benchmark may load it.
 */
#ifndef SPHX_ORACLE_H
#define SPHX_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SO_MAX_PISTON 16

typedef struct {
    int32_t dim;          /* 2 or 3 */
    int32_t visc_form;    /* 0: Eq. (10) kinematic harmonic mean; 1: Eq. (11) dynamic */
    int32_t cont_form;    /* 0: Eq. (6) volume form; 1: Eq. (5) single-phase mass form */
    int32_t renorm_every; /* Eq. (7) applied at steps with step % renorm_every == 0; 0 never */
    double h;             /* smoothing length; kernel support 2h */
    double gamma;         /* Tait exponent, Eq. (3) */
    double delta_coef;    /* delta = delta_coef * h, Eq. (9) */
    double alpha_s;       /* interfacial tension coefficient, Eq. (15) */
    double gravity[3];
    double lo[3], hi[3];  /* domain; periodic dims have period hi - lo */
    int32_t periodic[3];
    double c_cfl, c_force, c_visc, c_st;
    double dt_fixed;      /* > 0: use this step instead of the adaptive one */
    int32_t n_piston;     /* MOVING particles: x = x0 + d(t) e_x */
    double piston_t_end;  /* d(t) = sum_k a_k (cos(w_k t' + phi_k) - cos(phi_k)), t' = min(t, t_end) */
    double piston_a[SO_MAX_PISTON], piston_w[SO_MAX_PISTON], piston_phi[SO_MAX_PISTON];
} so_params;

typedef struct { double rho0, nu, c0; } so_phase;

enum { SO_FLUID = 0, SO_WALL = 1, SO_MOVING = 2 };

/* field ids for so_get / so_set */
enum {
    SO_X = 0, SO_U = 1, SO_RHO = 2, SO_A = 3, SO_DRHO = 4,
    SO_AP = 5, SO_AV = 6, SO_AS = 7,             /* acceleration terms, n x 3 */
    SO_SDRHO = 8, SO_SAP = 9, SO_SAV = 10, SO_SAS = 11, /* per-particle sum of |pair term| */
    SO_P = 12, SO_GRADC = 13,                    /* pressure (n), colour gradient (n x 3) */
    SO_TENSOR = 14                               /* surface stress tensor, n x 9 */
};

typedef struct so_ctx so_ctx;

/* Wendland C2 kernel with support 2h (reading of the unstated kernel). */
double so_kernel_w(int32_t dim, double h, double r);
/* grad_i W_ij = so_kernel_f(r) * (x_i - x_j) */
double so_kernel_f(int32_t dim, double h, double r);
/* Tait pressure, Eqs. (3)-(4) */
double so_eos(double rho, double rho0, double c0, double gamma);
/* piston displacement and velocity */
void so_piston(const so_params* p, double t, double* d, double* v);

so_ctx* so_create(const so_params* p, const so_phase* phases, int32_t nphase, int64_t n,
                  const double* x, const double* u, const double* rho, const double* m,
                  const uint8_t* phase, const uint8_t* kind);
void so_destroy(so_ctx* c);
/* From now on the MOVING particles sit at their initial position + disp + vel (t - t_now)
 * with velocity vel, in place of the piston (components beyond dim are ignored); they
 * are placed there at once.  Not from the paper: the library's motion set from outside. */
void so_set_moving(so_ctx* c, const double disp[3], const double vel[3]);
void so_set_threads(int32_t nthreads);
int32_t so_get_threads(void);
/* method: 0 auto (brute force up to 5000 particles), 1 brute force, 2 cell list */
void so_set_neighbor_method(so_ctx* c, int32_t method);

/* neighbours at the current positions; CSR with ids ascending.  Returns the total
 * count; writes only when cap >= total. */
int64_t so_neighbors(so_ctx* c, int64_t* off, int32_t* idx, int64_t cap);
/* Eq. (7) at the current positions (Jacobi: every read is the old density) */
void so_renormalize(so_ctx* c);
/* rates Eqs. (3)-(17) at the current state; returns the interaction count */
int64_t so_rates(so_ctx* c);
/* adaptive step from the last rates (or dt_fixed) */
double so_dt(so_ctx* c);
/* nsteps full steps; returns the interactions summed over all rate evaluations */
int64_t so_step(so_ctx* c, int32_t nsteps);
double so_time(const so_ctx* c);
int64_t so_stepcount(const so_ctx* c);
int32_t so_get(const so_ctx* c, int32_t field, double* out);
int32_t so_set(so_ctx* c, int32_t field, const double* in);
/* pair contributions of j to i at the current state, after so_rates:
 * out[0..2] m_i * (pressure acceleration), out[3..5] m_i * (viscous, Eq. (11) form
 * when visc_form == 1 else the Eq. (10) term), out[6..8] m_i * (surface tension),
 * out[9] continuity sum term.  Returns 0, or -1 if j is not a neighbour of i. */
int32_t so_pair_terms(const so_ctx* c, int64_t i, int64_t j, double* out);

#ifdef __cplusplus
}
#endif
#endif
