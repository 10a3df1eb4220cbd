/*
 * sphx -- MI355X (gfx950) library for the per-step particle loop of the
 * two-phase weakly compressible SPH method of Wei et al., "Behavior of Oil
 * under Breaking Waves by a Two-phase SPH Model" (arXiv 1702.07760), Sec. II.
 *
 * C ABI.  Plain pointers and sizes only.  Every call returns an sphx_status;
 * nothing throws across the boundary.  A context is not thread-safe; distinct
 * contexts are independent.  All device work is queued on the stream given to
 * sphx_create (a HIP stream handle, never the legacy null stream if the step
 * is to be graph-captured).
 *
 * Ownership.  Host input arrays are copied during the call that takes them.
 * Device memory for the particle state is one caller-owned workspace of
 * sphx_workspace_size() bytes, bound with sphx_bind_workspace(); it must
 * outlive the context.  The step path (build, renormalise, rates, integrate,
 * step) never allocates.  The read-back calls (sphx_get_field,
 * sphx_get_neighbors, sphx_get_state) synchronise the stream and may allocate
 * temporary host or device memory.
 *
 * Errors.  Argument errors return SPHX_E_ARG (or SPHX_E_STATE for calls in the
 * wrong order) and leave the context unchanged.  Faults found on the device
 * (non-finite state, particles leaving a non-periodic domain, a time step
 * violating the neighbour-skin bound) are sticky bits of a device status word,
 * reported by the next sphx_sync or read-back call and cleared by it.
 * sphx_last_error() gives a readable message for the last failing call.
 */
#ifndef SPHX_H
#define SPHX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sphx_ctx sphx_ctx;

typedef enum {
    SPHX_OK = 0,
    SPHX_E_ARG = 1,        /* invalid argument; nothing changed */
    SPHX_E_NODEV = 2,      /* no usable gfx950 device */
    SPHX_E_HIP = 3,        /* a HIP runtime call failed */
    SPHX_E_WORKSPACE = 4,  /* workspace missing, too small or misaligned (256 B) */
    SPHX_E_STATE = 5,      /* call out of order (e.g. step before init_particles) */
    SPHX_E_NONFINITE = 6,  /* device: a rate or state value became NaN/Inf */
    SPHX_E_DOMAIN = 7,     /* device: a particle left a non-periodic domain */
    SPHX_E_DT = 8,         /* device: a step would take a particle more than half the
                              neighbour skin from its position at the last build (a
                              fixed or explicit dt too long for the particles' speed) */
    SPHX_E_STALL = 9       /* device: a grid barrier of the one-launch neighbour build timed
                              out; the work queued from that build on was not done and the
                              state is kept as the build found it (see
                              SPHX_OPT_ONE_LAUNCH_BUILD) */
} sphx_status;

typedef enum { SPHX_FP64 = 0, SPHX_FP32_CELLREL = 1 } sphx_precision;
typedef enum { SPHX_FLUID = 0, SPHX_WALL = 1, SPHX_MOVING = 2 } sphx_kind;

#define SPHX_MAX_PISTON 16

/* One phase: reference density rho0 (Eq. (3)), kinematic viscosity nu = mu/rho0
 * (Eqs. (10), (12)), sound speed c0 giving beta = rho0 c0^2 / gamma (Eq. (4)). */
typedef struct {
    double rho0, nu, c0;
} sphx_phase;

/* Parameters of one simulation instance (one independent tank). */
typedef struct {
    int32_t dim;          /* 2 or 3; the same for every instance of a context */
    int32_t visc_form;    /* 0: Eq. (10) kinematic harmonic mean; 1: Eq. (11) dynamic */
    int32_t cont_form;    /* 0: Eq. (6) volume form; 1: Eq. (5) mass form */
    int32_t renorm_every; /* Eq. (7) at steps with step % renorm_every == 0; 0 = never */
    double h;             /* smoothing length; Wendland C2 kernel of support 2h */
    double gamma;         /* Tait exponent; must be 7 (Eq. (3)) */
    double delta_coef;    /* delta = delta_coef * h (Eq. (9)) */
    double alpha_s;       /* interfacial tension coefficient (Eq. (15)) */
    double gravity[3];
    double lo[3], hi[3];  /* domain box; cells tile it; periodic period = hi - lo */
    int32_t periodic[3];
    double skin_coef;     /* cells are >= (2 + skin_coef) h, the list radius (2 + skin_coef) h; a
                             step that would take a particle more than skin_coef h / 2 from
                             its position at the last build is refused (SPHX_E_DT); it does
                             not enter the adaptive step */
    double c_cfl, c_force, c_visc, c_st; /* time-step coefficients */
    double dt_fixed;      /* > 0: fixed step instead of the adaptive one */
    int32_t n_piston;     /* MOVING particles follow x = x0 + d(t) e_x with */
    double piston_t_end;  /* d(t) = sum_k a_k (cos(w_k t' + phi_k) - cos phi_k), t' = min(t, t_end) */
    double piston_a[SPHX_MAX_PISTON], piston_w[SPHX_MAX_PISTON], piston_phi[SPHX_MAX_PISTON];
} sphx_params;

/* Field ids for sphx_get_field.  Vector fields are n x 3 (row-major, unused
 * components zero), scalars n; always FP64 and in original particle order. */
enum {
    SPHX_F_X = 0, SPHX_F_U = 1, SPHX_F_RHO = 2,
    SPHX_F_A = 3,            /* total acceleration of the last rate evaluation (0 for non-fluid) */
    SPHX_F_DRHO = 4,         /* density rate of the last rate evaluation */
    SPHX_F_AP = 5, SPHX_F_AV = 6, SPHX_F_AS = 7, /* terms of Eqs. (8), (10)/(11), (17); need SPHX_OPT_DEBUG_TERMS */
    SPHX_F_P = 12,           /* Tait pressure of the current density as the device derived it
                                (from its stored m P / rho^2; FP32 form: to FP32 rounding) */
    SPHX_F_GRADC = 13        /* colour gradient of the last rate evaluation (Eq. (16)) */
};

/* Options for sphx_set_option. */
enum {
    SPHX_OPT_DEBUG_TERMS = 1, /* 1: compute_forces also stores the three acceleration terms */
    SPHX_OPT_BLOCK = 2,       /* threads per block of the neighbour passes: 64, 128, 192 or 256
                                 (default: 3D 128, or 256 from 2^19 particles; 2D 64, or 128
                                 from 2^16 particles except FP64 from 2^20) */
    SPHX_OPT_XCD_REMAP = 3,   /* tile order of the neighbour passes: 0 dispatch order; 1 consecutive
                                 tiles on one XCD; K = 2, 4, ..., 64 also gives the K workgroups
                                 a CU holds at once K consecutive tiles, assuming round-robin
                                 dispatch over an XCD's 32 CUs; -C (C = 2, 4, ..., 64) deals
                                 chunks of C consecutive tiles round-robin to the XCDs
                                 (default: 3D 0; 2D 4 in FP32, 1 in FP64, 16 where the 2D
                                 block is 128) */
    SPHX_OPT_GRAPH = 4,       /* 1: sphx_step replays a captured hipGraph per step (default 1) */
    SPHX_OPT_LANES = 5,       /* lanes that share one particle's neighbour loop in the renormalisation
                                 pass: 1, 2 or 4 (default 4; 1 for 2D contexts of 2^20
                                 particles or more); each lane takes every lanes-th
                                 neighbour and the partial sums are combined in-wave (the colour
                                 pass always runs 8 lanes per particle) */
    SPHX_OPT_FORCE_LANES = 7, /* the same for the force pass (default 2 in 3D, 1 in 2D) */
    SPHX_OPT_PROFILE = 6,     /* 1: no graphs; every kernel group is bracketed by HIP events on the
                                 context stream and its time is reported in sphx_stats */
    SPHX_OPT_ONE_LAUNCH_BUILD = 8, /* 1 (default): the neighbour build (cell sort and list) is one
                                 launch, sized to the blocks the device holds at once, whose phases
                                 meet at grid barriers; without a rebuild it ends after the
                                 decision.  0: seven launches.  A barrier that waits too long (its
                                 blocks were not all resident, e.g. other work shared the device)
                                 stops that build part-way, and every pass queued after it returns
                                 without work until the next sphx_sync (or read-back call).  That
                                 call rebuilds the neighbour structure from the state the build
                                 found, which no pass changed (the steps from that build on are
                                 not taken: sphx_stats tells how many were), and returns
                                 SPHX_E_STALL; the context builds with seven launches from then
                                 on */
    SPHX_OPT_FORCE_STALL = 9, /* for tests of that recovery: 1..5 makes grid barrier 1..5 of the next
                                 one-launch build time out at once (0: none, the default) */
    SPHX_OPT_COLOUR_IN_PREDICT = 10 /* 1: the colour pass at the predicted state runs in the
                                 predictor's launch, its blocks computing the predicted state
                                 of each particle of the colour list and of its other-phase
                                 neighbours themselves (one launch less per step); 0: in a
                                 launch of its own after the predictor.  Identical results.
                                 sphx_init_particles sets 1 when at most 1,024 particles have a
                                 phase other than 0 (a short colour list), else 0 */
};

/* Kernel groups timed under SPHX_OPT_PROFILE. */
enum {
    SPHX_PH_BUILD = 0,        /* hash, scan, sort, gather, cell flags */
    SPHX_PH_RENORM = 1,       /* Eq. (7) pass (with the state derivation after it, outside sphx_step) */
    SPHX_PH_COLOUR = 2,       /* Eq. (16) passes (in sphx_step, the one at S^n shares a launch with
                                 the state derivation after Eq. (7)) */
    SPHX_PH_FORCE = 3,        /* Eqs. (6), (8), (10)/(11), (17) pass at S^n (compute_forces, first
                                 rate evaluation of a step) */
    SPHX_PH_INTEGRATE = 4,    /* time step, predictor, and the launch that holds the rates at S*
                                 and the corrector */
    SPHX_NPH = 5
};

/* Run statistics, from the device after sphx_sync. */
typedef struct {
    int64_t steps;            /* steps completed (instance 0) */
    double t;                 /* simulated time of instance 0 */
    double dt;                /* last time step of instance 0 */
    int64_t interactions;     /* ordered pairs (i, j != i, r_ij < 2h) summed over every
                                 force evaluation since the last reset */
    int64_t ncells;           /* cells over all instances */
    int64_t builds;           /* neighbour builds (sort + list) so far, instance 0 */
    double phase_ms[5];       /* SPHX_OPT_PROFILE: summed event time per kernel group */
    int64_t phase_launches[5];/* SPHX_OPT_PROFILE: timed launches per kernel group */
    int64_t colour_particles; /* particles with another phase in their neighbour list at the
                                 last build: the work list of the colour pass (Eq. (16)) */
    int64_t two_level_builds; /* one-launch rebuilds whose later grid barriers took the
                                 two-level form (one L2 write-back and invalidation per XCD) */
} sphx_stats;

/* Bytes of device workspace for ninst instances holding counts[b] particles. */
size_t sphx_workspace_size(int32_t precision, const sphx_params* per_inst, int32_t ninst,
                           const int64_t* counts);

/* Create a context.  per_inst[ninst]; phases[ninst * nphase] (row b holds the phases of
 * instance b; nphase 1 or 2, phase 0 is water and boundary particles must be phase 0);
 * counts[ninst] particles per instance; stream is a hipStream_t (may be NULL: the legacy
 * stream, no graph capture). */
sphx_status sphx_create(int32_t precision, const sphx_params* per_inst, const sphx_phase* phases,
                        int32_t nphase, int32_t ninst, const int64_t* counts, void* stream,
                        sphx_ctx** out);
void sphx_destroy(sphx_ctx* ctx);
/* Message of the last failing call on ctx; with ctx NULL, why the calling thread's last
 * sphx_create failed. */
const char* sphx_last_error(const sphx_ctx* ctx);

/* Bind caller-owned device memory (>= sphx_workspace_size bytes, 256-byte aligned). */
sphx_status sphx_bind_workspace(sphx_ctx* ctx, void* dev_ptr, size_t bytes);

/* Size of the static workspace below: 64 MiB per device. */
#define SPHX_STATIC_WORKSPACE_BYTES (64ull << 20)

/* For callers that cannot allocate device memory (code under graph capture, serving
 * loops, harnesses that forbid hipMalloc): the variant of sphx_bind_workspace that
 * binds the library's own static workspace of the context's device instead of caller
 * memory.  It allocates nothing, device or host.  Each device holds one static
 * workspace of SPHX_STATIC_WORKSPACE_BYTES from the loading of the library until the
 * process ends; a context that needs more (sphx_workspace_size) gets SPHX_E_WORKSPACE
 * and stays as it was.  Every context bound to it on one device shares it, and it keeps
 * what the last context left there (init_particles sets up everything a run reads):
 * binding a second context takes the workspace away from the first, whose later calls
 * return SPHX_E_WORKSPACE until it is bound again and init_particles runs again.  Calls
 * of two contexts bound to the same device's static workspace that overlap in time
 * race.  As with sphx_bind_workspace, call init_particles next. */
sphx_status sphx_bind_static_workspace(sphx_ctx* ctx);

/* Copy the particle state from host arrays in original order (n = sum of counts):
 * x, u: n x 3 FP64 row-major; rho, m: n FP64; phase, kind: n uint8.  Validates every
 * value (finite, inside the box, positive density and mass, phase < nphase, boundary
 * particles in phase 0), then builds the neighbour structure and waits for it.  May be
 * called again to start over with the same layout.  Returns SPHX_E_STALL if that first
 * build stalled (the particles are then in place, built with seven launches). */
sphx_status sphx_init_particles(sphx_ctx* ctx, const double* x, const double* u, const double* rho,
                                const double* m, const uint8_t* phase, const uint8_t* kind);

/* Neighbour search at the current positions: cell hash, stable sort by cell (ties by
 * original index), reorder of the state, cell start table, neighbour list.  The sums of
 * Sec. II (Eqs. (5)-(17)) run over the neighbours j of particle i, the particles within
 * the kernel's support 2h; the paper leaves the search to the code it builds on, so the
 * cells of (2 + skin) h and the list radius with its skin are this library's (skin_coef
 * in sphx_params).  The other calls rebuild by themselves whenever a particle's
 * displacement since the last build, plus the half step the next predictor can give
 * it (half the fixed step, or of the CFL step at zero speed, times its speed), could
 * exceed 99 % of half the skin; this call forces a rebuild.
 * No arguments besides the context; errors as for sphx_step. */
sphx_status sphx_build_neighbors(sphx_ctx* ctx);

/* Eq. (7): rho_i = sum m_j W_ij / sum (m_j/rho_j) W_ij over i and its same-phase
 * neighbours, every particle at once from the old densities. */
sphx_status sphx_renormalize_density(sphx_ctx* ctx);

/* Rates at the current state, no state change: Tait pressure (Eqs. (3)-(4)), colour
 * gradient and surface stress (Eqs. (14)-(16)), density rate (Eq. (6) or (5)) and
 * acceleration (Eqs. (8), (10) or (11), (17), gravity). */
sphx_status sphx_compute_forces(sphx_ctx* ctx);

/* One midpoint predictor-corrector step from the rates of the last compute_forces:
 * time step (dt > 0 fixes it, dt <= 0 takes the adaptive one on the device),
 * predictor, rates at the predicted state, corrector.  The paper gives the rates
 * (Eqs. (3)-(17)) and no time integrator; the integrator and the adaptive step (CFL
 * with the reduced sound speed of Sec. II.A, force, viscous and capillary limits) are
 * the usual WCSPH ones.  Moving (piston) particles follow Eq. (18) or sphx_set_moving;
 * boundary particles keep their positions.  SPHX_E_STATE without fresh rates,
 * SPHX_E_ARG for a non-finite dt; a step longer than the neighbour skin allows is
 * refused on the device (SPHX_E_DT at the next sync). */
sphx_status sphx_integrate_step(sphx_ctx* ctx, double dt);

/* nsteps full steps: neighbour rebuild when due, Eq. (7) when due, rates, integrate.
 * Each step is one replay of a captured hipGraph when SPHX_OPT_GRAPH is on and the
 * stream allows it (both decisions are taken on the device). */
sphx_status sphx_step(sphx_ctx* ctx, int32_t nsteps);

/* Prescribe the motion of instance inst's MOVING particles from now on (the wavemaker
 * of Sec. IV driven from outside, in place of the piston series of sphx_params): each
 * sits at its reference position + disp + vel (t - t_call) with velocity vel, t_call
 * being the instance's time at the call (read from the device: the call synchronises the
 * stream).  The call places them there at once, and the next step rebuilds the
 * neighbour structure.  disp, vel: 3 doubles, m and m/s; components beyond the dimension are
 * ignored.  The steps take the motion at t, t + dt/2 and t + dt like the series.
 * SPHX_E_ARG for a bad instance, non-finite values or motion along a periodic axis;
 * SPHX_E_STATE if the scene has no MOVING particles.  sphx_init_particles returns the
 * particles to the series; sphx_set_state keeps the motion last set. */
sphx_status sphx_set_moving(sphx_ctx* ctx, int32_t inst, const double* disp, const double* vel);

sphx_status sphx_set_option(sphx_ctx* ctx, int32_t option, int64_t value);
/* Current value of an option (the defaults chosen at sphx_create included). */
sphx_status sphx_get_option(sphx_ctx* ctx, int32_t option, int64_t* value);

/* Wait for the stream; map the device status word to a status and clear it. */
sphx_status sphx_sync(sphx_ctx* ctx);
sphx_status sphx_get_stats(sphx_ctx* ctx, sphx_stats* out);
sphx_status sphx_reset_interactions(sphx_ctx* ctx);

/* Copy one field to host_out in original particle order, FP64 (see the field ids). */
sphx_status sphx_get_field(sphx_ctx* ctx, int32_t field, double* host_out);

/* Neighbour lists at the current positions in CSR form, original ids, ascending:
 * off[n+1], ids[need].  *need receives the total; ids is written when cap >= need. */
sphx_status sphx_get_neighbors(sphx_ctx* ctx, int64_t* off, int32_t* ids, int64_t cap,
                               int64_t* need);

/* Opaque snapshot of the full state (including compensation terms, time, step count
 * and the time step); a restored context continues bit-identically.  sphx_set_state
 * takes a blob from a context of the same layout, checks that every index in it is in
 * range (SPHX_E_ARG and no change otherwise); errors still pending from the replaced
 * state are dropped. */
sphx_status sphx_get_state(sphx_ctx* ctx, void* host_blob, size_t cap, size_t* need);
sphx_status sphx_set_state(sphx_ctx* ctx, const void* host_blob, size_t bytes);

#ifdef __cplusplus
}
#endif
#endif
