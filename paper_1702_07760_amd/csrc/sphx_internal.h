// Internal interface between the C-ABI runtime (sphx_api.hip) and the gfx950
// kernels (sphx_kernels.hip).  Not installed, not part of the ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sphx {

constexpr int kMaxPiston = 16;

// Status word bits (sticky, set by kernels with atomicOr).
enum : uint32_t { ST_NONFINITE = 1u, ST_DOMAIN = 2u, ST_DT = 4u, ST_STALL = 8u };

// Particle info word: phase in bit 0, kind in bits 1-2, instance in bits 8-31; bit 7
// marks, from one list build to the next, a particle of the colour-pass list.
constexpr uint32_t kInfoColour = 0x80u;
__host__ __device__ inline uint32_t info_phase(uint32_t w) { return w & 1u; }
__host__ __device__ inline uint32_t info_kind(uint32_t w) { return (w >> 1) & 3u; }
__host__ __device__ inline uint32_t info_inst(uint32_t w) { return w >> 8; }
__host__ __device__ inline uint32_t make_info(uint32_t phase, uint32_t kind, uint32_t inst)
{
    return (phase & 1u) | ((kind & 3u) << 1) | (inst << 8);
}
enum : uint32_t { K_FLUID = 0, K_WALL = 1, K_MOVING = 2 };

// Per-instance constants, built on the host from sphx_params + sphx_phase.
// Neighbour-list capacity per particle (lattice: 20 / 80 neighbours within 2h in 2D /
// 3D).  The list walk reads whole batches of (entries per batch) x (lanes per particle)
// entries, which must divide the capacity for those reads to stay inside the list (the
// walk checks this at compile time).
constexpr uint32_t kListCap2 = 48u, kListCap3 = 128u;
static_assert(kListCap2 % 16u == 0 && kListCap3 % 16u == 0, "capacities are multiples of the padding");

// Interaction count: kInterSlots 64-bit counters, kInterStride words (128 bytes) apart.
// Wave w of a force launch adds into counter w mod kInterSlots, so the adds of
// concurrent waves land on different cache lines; the host sums the counters.
constexpr uint32_t kInterSlots = 256u, kInterStride = 16u;

// Neighbour-list entry: particle index j in the low 25 bits; in FP32 the cell offset
// delta = c_i - c_j (components in {-1, 0, 1}) as two bits per axis, delta_x + 1 in bits
// 25-26, delta_y + 1 in bits 27-28, delta_z + 1 in bits 29-30; the phase of j in bit 31
// (phases never change, so the list carries them).  A list is padded with the entry
// kSentinel-index n up to a multiple of kListPad entries, so that the walks read whole
// batches without checking each entry against the count: index n is a record placed
// far outside every domain, so it is never within the cutoff.
constexpr uint32_t kIdxBits = 25, kIdxMask = (1u << kIdxBits) - 1u, kPhaseShift = 31;
constexpr uint32_t kListPad = 16u;

// Words of the one-launch build's barrier area: 1024 words of epoch, release, group and
// go words (each on a cache line of its own), then 4096 arrival slots and 4096 XCD ids,
// one of each per block.
constexpr uint32_t kBarWords = 1024u + 2u * 4096u;

struct InstDev {
    double lo[3], hi[3], span[3], cs[3];
    int32_t nc[3];
    int32_t periodic[3];
    uint32_t cell_base, ncell;
    int32_t dim, visc_form, cont_form, renorm_every;
    double h, inv_h, cut2, cutl2, wcoef, fcoef, delta2, alpha_s, skin;
    // rebuild once some particle's reach, its displacement since the build plus the
    // longest half step it can take next (dt_bound / 2 times its speed), exceeds
    // rebuild_e (99 % of half the skin); dt_bound: the fixed step, else the CFL step at
    // zero speed, c_cfl h / max c0, which no adaptive step exceeds
    double rebuild_e, dt_bound;
    double g[3];
    double rho0[2], beta[2], nu[2];
    double vpair[2][2];   // 2 nu_ij (Eq. (10)) or 2 mu_ij (Eq. (11)) by phase pair
    double dt_fixed, c_cfl, c_force, cmax, dt_const; // dt_const: min of viscous and capillary limits
    int32_t n_piston;
    double piston_t_end;
    double pa[kMaxPiston], pw[kMaxPiston], pphi[kMaxPiston];
    // host-set motion of the MOVING particles (sphx_set_moving), replacing the piston
    // series when mv_host = 1: displacement mv_disp + mv_vel (t - mv_t0), velocity mv_vel
    int32_t mv_host;
    double mv_disp[3], mv_vel[3], mv_t0;
    // particle mass by phase, valid when umass = 1: every particle of the instance with
    // that phase has this mass (the force pass then reads no mass per neighbour)
    int32_t umass;
    double mass[2];
    // FP32 copies for the cell-relative kernels; f_cs_lo = cs - f_cs (the part of the
    // cell size FP32 drops, carried into the compensation term when offsets re-cell)
    float f_cs[3], f_cs_lo[3], f_inv_h, f_cut2, f_cutl2, f_fcoef, f_wcoef, f_delta2, f_alpha_s, f_g[3];
    float f_vpair[2][2], f_rho0[2], f_mass[2];
};

// The first particle found outside a non-periodic domain: the first hash that sees one
// claims the record.  Original index, instance, absolute position and the cell index
// that position maps to (before clamping into the grid).
struct FaultRec {
    uint32_t claimed, id, inst, pad;
    int32_t cell[4];
    double x[4];
};

// Per-instance run variables on the device.
struct InstRun {
    unsigned long long umax2;  // bit pattern of max |u|^2 (FP64, non-negative)
    unsigned long long amax2;  // bit pattern of max |a|^2
    unsigned long long reach2; // bit pattern of the largest (|x - x_build| + dt_bound |u| / 2)^2
                               // over the last corrector's state (0 after a build)
    double dt, t, t_next;
    long long step;
    long long builds;          // neighbour builds so far
};

// One copy of the cell-sorted particle state.
struct StateSet {
    void* pos;   // R4: FP64 (x, y, z, w); FP32 (ox, oy, oz, w); w = m P / rho^2 during rate
                 //     evaluations, q = (rho - rho0) / rho from a state update to Eq. (7)
    void* vel;   // R4: (ux, uy, uz, +-V), V = m / rho; the sign of w is the interface flag
    void* aux;   // R4: (m, m P / rho^2, V, rho); w is rho in FP64 and rho - rho0 in FP32
    float4* plo; // FP32 only: compensation of (ox, oy, oz, rho - rho0)
    float4* vlo; // FP32 only: compensation of (ux, uy, uz)
};

struct Sorted {          // arrays shared by the state sets of one sort order
    uint32_t* key;       // global cell key (instance cell base + local linear cell)
    uint32_t* id;        // original particle index
    uint32_t* info;
    double4* ref;        // x0 of MOVING particles (absolute)
};

struct Dev {
    int precision;       // 0 FP64, 1 FP32 cell-relative
    int dim;
    int ninst;
    int64_t n;
    uint32_t ncell;      // total over instances
    const InstDev* inst; // device
    InstRun* run;        // device
    uint32_t* status;
    FaultRec* fault;     // details of the first ST_DOMAIN
    unsigned long long* inter;
    int* curp;           // which state set (0/1) holds the current sorted state
    int* prevp;          // during a rebuild: the set being sorted from (the old curp)
    unsigned* bar;       // the one-launch build's grid barriers: epoch base, release, group and
                         // go words, then an arrival slot and an XCD id per block (kBarWords)
    uint32_t* flags;     // [0] rebuild in this step, [1] rebuild requested by the host,
                         // [2] pos.w holds q = (rho - rho0) / rho rather than m P / rho^2,
                         // [3] one-launch rebuilds that took the two-level barrier
    // build scratch
    uint32_t* cnt;       // ncell
    uint32_t* cstart;    // ncell + 1
    uint32_t* scan_tmp;  // block sums
    uint32_t* newkey;    // n (old order)
    uint32_t* slot;      // n
    uint32_t* tsrc;      // n
    uint32_t* tid;       // n
    // neighbour list of the current sort order, column-major: entry q of i at
    // q * lstride + i, the row stride n rounded up to whole 128-byte lines
    uint32_t* nbl;       // lstride * cap entries (index | cell-offset code << 25 | phase << 31)
    uint32_t* nbc;       // n counts (> cap: overflowed, the passes walk the stencil)
    uint32_t* ilist;     // colour-pass particles (another phase in the list), in build order
    uint32_t* icount;    // their number
    uint32_t cap;
    uint32_t lstride;
    void* xb;            // R4: positions at the last build (FP32: cell offsets)
    // state
    StateSet S[2];       // double-buffered current state
    Sorted O[2];
    StateSet star;       // predicted state
    void* rho_tmp;       // renormalised density (R)
    void* acc;           // R4: (ax, ay, az, drho)
    void* gc;            // R4: (gx, gy, gz, |g|)
    void* terms;         // 3 x R4 per particle (debug)
};

struct Launch {
    int block = 64;      // threads per block of the neighbour passes (per-form defaults at create)
    int xcd_remap = 1;   // 0 dispatch order, 1 XCD-contiguous tiles, K >= 2 also K tiles per CU
    int lanes = 4;       // lanes per particle in the renormalisation pass (1, 2, 4)
    int force_lanes = 1; // lanes per particle in the force pass (1, 2, 4)
    bool one_launch_build = true;   // the build as one launch with grid barriers (else seven)
    bool colour_in_predict = true;  // the colour pass at S* inside the predictor's launch
    int stall_at = 0;    // test hook: barrier of the one-launch build forced to time out (0: none)
    bool debug_terms = false;
};

// --- launchers (sphx_kernels.hip); all asynchronous on the given stream.  The current
// state set and the rebuild decision live on the device, so one captured graph serves
// every step.
void launch_build(const Dev& d, const Launch& L, hipStream_t s);     // decide, then sort + list if due
void launch_nlist(const Dev& d, const Launch& L, hipStream_t s);     // list of the current order
void launch_renorm(const Dev& d, bool force, const Launch& L, hipStream_t s);
void launch_colour(const Dev& d, bool star, const Launch& L, hipStream_t s);
void launch_force(const Dev& d, bool star, bool reduce_max, bool correct, const Launch& L, hipStream_t s);
void launch_derive(const Dev& d, const Launch& L, hipStream_t s);
void launch_restore(const Dev& d, hipStream_t s);
// Eq. (7) (parts bit 0), then the derive pass and the colour pass at S^n (bit 1)
void launch_renorm_colour(const Dev& d, const Launch& L, hipStream_t s, int parts = 3);
void launch_predict(const Dev& d, double dt_override, const Launch& L, hipStream_t s);   // a9 and S*
void launch_place_moving(const Dev& d, uint32_t inst, hipStream_t s);   // sphx_set_moving
// neighbour export: counts (pass 0) or ids (pass 1) in sorted order
void launch_export(const Dev& d, int pass, const uint32_t* off, uint32_t* out,
                   const Launch& L, hipStream_t s);

} // namespace sphx
