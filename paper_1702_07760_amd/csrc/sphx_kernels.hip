// gfx950 kernels of the two-phase WCSPH step (arXiv 1702.07760, Sec. II).
//
// Layout: particles live in cell-sorted order, structure-of-arrays of 16/32-byte
// records so that a wave reads them coalesced.  In the neighbour passes one lane, or a
// group of 2 or 4 consecutive lanes, owns particle i and gathers over its neighbours j
// from a column-major neighbour list; a group splits the list and adds its partial sums
// with in-wave shuffles.  There are no atomics on floating-point data: the only atomics
// are integer counters and the order-independent max-reductions of the time step, so
// every result is deterministic.  Per-instance constants of a neighbour loop are held
// in scalar registers, one pass per distinct instance in a wave.
//
// Two precision forms share every kernel through the template parameter R:
//   double : absolute FP64 positions, FP64 everything;
//   float  : positions as (cell, FP32 offset inside the cell), density as
//            rho - rho0 in FP32, FP64 only for the Tait pressure, the time-step
//            reduction and the cell origins; compensated (Kahan) updates.
#include "sphx_internal.h"

#include <math.h>
#include <type_traits>
#include <algorithm>

namespace sphx {

template <class R> struct V4;
template <> struct V4<double> { using T = double4; };
template <> struct V4<float> { using T = float4; };
template <class R> using R4 = typename V4<R>::T;

// ------------------------------------------------------------------ helpers

__device__ __forceinline__ uint32_t tile_index(int remap)
{
    const uint32_t b = blockIdx.x, G = gridDim.x;
    if (!remap) return b;
    if (remap < 0) {
        // chunks of C = -remap consecutive tiles dealt round-robin to the 8 XCDs: each
        // XCD's L2 sees runs of neighbouring tiles, and every region's work is spread
        // over all XCDs (a bijection on the full rounds of 8 C workgroups)
        constexpr uint32_t X = 8;
        const uint32_t C = (uint32_t)(-remap), full = (G / (X * C)) * (X * C);
        if (b >= full) return b;
        const uint32_t xcd = b % X, j = b / X;
        return ((j / C) * X + xcd) * C + j % C;
    }
    // Workgroups are dealt round-robin to the 8 XCDs; give each XCD a contiguous run of
    // tiles so that neighbouring particles share one L2.
    const uint32_t X = 8, full = (G / X) * X;
    if (b >= full) return b;
    const uint32_t per = G / X, xcd = b % X;
    uint32_t j = b / X;
    if (remap >= 2) {
        // and within an XCD, assuming its 32 CUs are dealt round-robin as well, give the
        // K = remap workgroups a CU holds at once K consecutive tiles (shared neighbours
        // in its L1); a bijection on each full chunk of 32 K workgroups
        constexpr uint32_t S = 32;
        const uint32_t K = (uint32_t)remap, C = S * K;
        if (j / C < per / C) {
            const uint32_t r = j % C;
            j = (j / C) * C + (r % S) * K + r / S;
        }
    }
    return xcd * per + j;
}

__device__ __forceinline__ int wrapi(int c, int n) { return c < 0 ? c + n : (c >= n ? c - n : c); }

template <class IC>
__device__ __forceinline__ void cell_of_key(const IC& I, uint32_t key, int c[3])
{
    uint32_t l = key - I.cell_base;
    c[0] = (int)(l % (uint32_t)I.nc[0]);
    l /= (uint32_t)I.nc[0];
    c[1] = (int)(l % (uint32_t)I.nc[1]);
    c[2] = (int)(l / (uint32_t)I.nc[1]);
}

__device__ __forceinline__ double wave_max(double v)
{
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    return v;
}

// Running maximum of a non-negative double kept as its bit pattern.  The plain read
// first skips the atomic when it cannot raise the value (values only grow, so a stale
// read can only cost an extra atomic, never lose an update).
__device__ __forceinline__ void max_update(unsigned long long* slot, double v)
{
    const unsigned long long bits = (unsigned long long)__double_as_longlong(v);
    if (bits > *(volatile unsigned long long*)slot) atomicMax(slot, bits);
}

__device__ __forceinline__ unsigned long long wave_sum(unsigned long long v)
{
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Tait pressure, Eqs. (3)-(4), gamma = 7, evaluated in FP64 from rho / rho0.
__device__ __forceinline__ double tait(double y, double beta)
{
    const double y2 = y * y, y4 = y2 * y2;
    return beta * (y4 * y2 * y - 1.0);
}

// Displacement d(t) and velocity v(t) of the MOVING particles: the piston series along
// x (Eq. (18) and its sums), or the host-set linear motion.
__device__ inline void moving_motion(const InstDev& I, double t, double d[3], double v[3])
{
    if (I.mv_host) {
        for (int q = 0; q < 3; ++q) {
            d[q] = I.mv_disp[q] + I.mv_vel[q] * (t - I.mv_t0);
            v[q] = I.mv_vel[q];
        }
        return;
    }
    const double te = t < I.piston_t_end ? t : I.piston_t_end;
    d[0] = d[1] = d[2] = 0.0;
    v[0] = v[1] = v[2] = 0.0;
    for (int k = 0; k < I.n_piston; ++k) {
        d[0] += I.pa[k] * (cos(I.pw[k] * te + I.pphi[k]) - cos(I.pphi[k]));
        if (t < I.piston_t_end) v[0] -= I.pa[k] * I.pw[k] * sin(I.pw[k] * t + I.pphi[k]);
    }
}

// ------------------------------------------- per-instance constants in SGPRs

__device__ __forceinline__ uint32_t ufirst(uint32_t v) { return (uint32_t)__builtin_amdgcn_readfirstlane((int)v); }
__device__ __forceinline__ int32_t ufirst(int32_t v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ float ufirst(float v) { return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v))); }
__device__ __forceinline__ double ufirst(double v)
{
    const long long b = __double_as_longlong(v);
    const uint32_t lo = ufirst((uint32_t)b), hi = ufirst((uint32_t)(b >> 32));
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// The per-instance constants that the neighbour loops read, held in scalar registers
// (loaded once per wave instead of once per neighbour).  Built only where every
// active lane of the wave belongs to one instance; unused fields cost nothing.
struct InstU {
    uint32_t cell_base;
    int32_t nc[3], periodic[3], cont_form, visc_form;
    int32_t umass;
    double span[3], cut2, cutl2, inv_h, wcoef, fcoef, delta2, alpha_s, g[3], rho0[2], vpair[2][2], mass[2];
    float f_cs[3], f_inv_h, f_cut2, f_cutl2, f_fcoef, f_wcoef, f_delta2, f_alpha_s, f_g[3], f_vpair[2][2],
        f_mass[2];
};

__device__ __forceinline__ InstU uniform_inst(const InstDev& I)
{
    InstU u;
    u.cell_base = ufirst(I.cell_base);
    for (int q = 0; q < 3; ++q) {
        u.nc[q] = ufirst(I.nc[q]);
        u.periodic[q] = ufirst(I.periodic[q]);
        u.span[q] = ufirst(I.span[q]);
        u.g[q] = ufirst(I.g[q]);
        u.f_cs[q] = ufirst(I.f_cs[q]);
        u.f_g[q] = ufirst(I.f_g[q]);
    }
    u.cont_form = ufirst(I.cont_form);
    u.visc_form = ufirst(I.visc_form);
    u.umass = ufirst(I.umass);
    u.cut2 = ufirst(I.cut2);
    u.cutl2 = ufirst(I.cutl2);
    u.inv_h = ufirst(I.inv_h);
    u.wcoef = ufirst(I.wcoef);
    u.fcoef = ufirst(I.fcoef);
    u.delta2 = ufirst(I.delta2);
    u.alpha_s = ufirst(I.alpha_s);
    u.f_inv_h = ufirst(I.f_inv_h);
    u.f_cut2 = ufirst(I.f_cut2);
    u.f_cutl2 = ufirst(I.f_cutl2);
    u.f_fcoef = ufirst(I.f_fcoef);
    u.f_wcoef = ufirst(I.f_wcoef);
    u.f_delta2 = ufirst(I.f_delta2);
    u.f_alpha_s = ufirst(I.f_alpha_s);
    for (int a = 0; a < 2; ++a) {
        u.rho0[a] = ufirst(I.rho0[a]);
        u.mass[a] = ufirst(I.mass[a]);
        u.f_mass[a] = ufirst(I.f_mass[a]);
        for (int b = 0; b < 2; ++b) {
            u.vpair[a][b] = ufirst(I.vpair[a][b]);
            u.f_vpair[a][b] = ufirst(I.f_vpair[a][b]);
        }
    }
    return u;
}

// Runs f(instance constants) for the active lanes, one distinct instance at a time
// (a single pass when the wave lies inside one instance, the usual case).  The loop is
// driven by the ballot mask of lanes still to do, a value that changes every pass: a
// loop keyed on readfirstlane alone looks invariant to the optimiser, which may then
// assume its first pass covers every lane.
template <class F>
__device__ __forceinline__ void per_instance(const Dev& d, uint32_t inst, F&& f)
{
    unsigned long long todo = __ballot(1);
    while (todo) {
        const int leader = __ffsll((long long)todo) - 1;
        const uint32_t u = ufirst((uint32_t)__shfl((int)inst, leader, 64));
        const bool mine = inst == u;
        todo &= ~__ballot(mine);
        if (mine) {
            const InstU I = uniform_inst(d.inst[u]);
            f(I);
        }
    }
}

// --------------------------------------------------------- lane geometry

// What lane i needs to turn a candidate record into r_ij = x_i - x_j.
template <class R> struct Lane;

template <> struct Lane<double> {
    double x[3];
    int c[3];
    template <class IC> __device__ void load(const IC& I, const double4& p, uint32_t key)
    {
        x[0] = p.x; x[1] = p.y; x[2] = p.z;
        cell_of_key(I, key, c);
    }
};

template <> struct Lane<float> {
    float om[3];   // offset minus one cell size: r = (c_i - c_j + 1) s + om - o_j
    int c[3];
    template <class IC> __device__ void load(const IC& I, const float4& p, uint32_t key)
    {
        om[0] = p.x - I.f_cs[0]; om[1] = p.y - I.f_cs[1]; om[2] = p.z - I.f_cs[2];
        cell_of_key(I, key, c);
    }
};

// Per-row constants: the y/z cell offsets of a stencil row are fixed.
template <class R> struct Row {
    uint32_t base;   // key of the row's first cell
    uint32_t code;   // (delta_y + 1) << 2 | (delta_z + 1) << 4, delta = c_i - c_j
    float dy1, dz1;  // delta_y + 1, delta_z + 1 as floats
};

// Neighbour-list entries (layout with the list constants): the phase of j is bit 31.
__device__ __forceinline__ uint32_t entry_phase(uint32_t e) { return e >> kPhaseShift; }

template <int DIM>
__device__ __forceinline__ double dist2(double rx, double ry, double rz)
{
    // the same rounding as the oracle: fma(rz, rz, fma(ry, ry, rx*rx))
    return DIM == 3 ? fma(rz, rz, fma(ry, ry, rx * rx)) : fma(ry, ry, rx * rx);
}

template <int DIM>
__device__ __forceinline__ float dist2(float rx, float ry, float rz)
{
    return DIM == 3 ? fmaf(rz, rz, fmaf(ry, ry, rx * rx)) : fmaf(ry, ry, rx * rx);
}

template <class IC>
__device__ __forceinline__ double min_image(double v, const IC& I, int d)
{
    if (I.periodic[d]) {
        const double L = I.span[d];
        if (v > 0.5 * L) v -= L;
        else if (v < -0.5 * L) v += L;
    }
    return v;
}

// r_ij for a stencil candidate (FP64: absolute positions, minimal image).  Returns the
// list-entry offset code (unused in FP64).
template <int DIM, class IC>
__device__ __forceinline__ uint32_t pair_r(const IC& I, const Lane<double>& L, const Row<double>&,
                                           const double4& pj, int, double r[3])
{
    r[0] = min_image(L.x[0] - pj.x, I, 0);
    r[1] = min_image(L.x[1] - pj.y, I, 1);
    r[2] = DIM == 3 ? min_image(L.x[2] - pj.z, I, 2) : 0.0;
    return 0u;
}

// r_ij for a stencil candidate (FP32: cell offsets; dcx = c_i - c_j along x).
template <int DIM, class IC>
__device__ __forceinline__ uint32_t pair_r(const IC& I, const Lane<float>& L, const Row<float>& row,
                                           const float4& pj, int dcx, float r[3])
{
    r[0] = fmaf((float)(dcx + 1), I.f_cs[0], L.om[0] - pj.x);
    r[1] = fmaf(row.dy1, I.f_cs[1], L.om[1] - pj.y);
    r[2] = DIM == 3 ? fmaf(row.dz1, I.f_cs[2], L.om[2] - pj.z) : 0.0f;
    return (uint32_t)(dcx + 1) | row.code;
}

// r_ij for a list entry e (same arithmetic as the stencil form above).
template <int DIM, class IC>
__device__ __forceinline__ void list_pair_r(const IC& I, const Lane<double>& L, const double4& pj,
                                            uint32_t, double r[3])
{
    r[0] = min_image(L.x[0] - pj.x, I, 0);
    r[1] = min_image(L.x[1] - pj.y, I, 1);
    r[2] = DIM == 3 ? min_image(L.x[2] - pj.z, I, 2) : 0.0;
}

template <int DIM, class IC>
__device__ __forceinline__ void list_pair_r(const IC& I, const Lane<float>& L, const float4& pj,
                                            uint32_t e, float r[3])
{
    const uint32_t cx = (e >> kIdxBits) & 3u, cy = (e >> (kIdxBits + 2)) & 3u, cz = (e >> (kIdxBits + 4)) & 3u;
    r[0] = fmaf((float)cx, I.f_cs[0], L.om[0] - pj.x);
    r[1] = fmaf((float)cy, I.f_cs[1], L.om[1] - pj.y);
    r[2] = DIM == 3 ? fmaf((float)cz, I.f_cs[2], L.om[2] - pj.z) : 0.0f;
}

template <class R, class IC> __device__ __forceinline__ R cut2_of(const IC& I)
{
    if constexpr (sizeof(R) == 8) return I.cut2;
    else return I.f_cut2;
}
template <class R, class IC> __device__ __forceinline__ R cutl2_of(const IC& I)
{
    if constexpr (sizeof(R) == 8) return I.cutl2;
    else return I.f_cutl2;
}

// Candidates loaded per batch in the stencil walk (independent loads in flight).
template <class R> struct StencilBatch { static constexpr int U = 8; };
template <> struct StencilBatch<double> { static constexpr int U = 4; };

// Visit every j != i with |r_ij|^2 < cut2 among the 3^d cells around i's cell:
// body(j, r_ij, |r_ij|^2, record of j, phase of j, list code).  A row of the stencil is
// one or two runs of consecutive sorted particles; a candidate's x cell offset follows
// from its index against the starts of i's cell and the next (FP32), its phase from
// the sorted info array.  When P lanes share particle i,
// lane `sub` takes every P-th candidate of each cell run.  U candidates are loaded per
// batch.  With ALL, the lanes of a group step through each run together and the body
// is called for every candidate slot with a flag `in` (a candidate j != i within the
// cutoff), so that the group can rank its accepted candidates with a ballot.
template <class R, int DIM, int P = 1, int U = StencilBatch<R>::U, bool ALL = false, class IC, class PS, class Body>
__device__ __forceinline__ void for_neighbors(const IC& I, const uint32_t* __restrict__ cstart,
                                              const Sorted& O, const PS& pos, uint32_t i,
                                              const Lane<R>& L, R cut2, uint32_t sub, Body&& body)
{
    const uint32_t* __restrict__ infos = O.info;
    const int nx = I.nc[0];
    const int zlo = DIM == 3 ? -1 : 0, zhi = DIM == 3 ? 1 : 0;
    for (int dz = zlo; dz <= zhi; ++dz) {
        int cz = L.c[2] + dz;
        if (DIM == 3) {
            if (I.periodic[2]) cz = wrapi(cz, I.nc[2]);
            else if (cz < 0 || cz >= I.nc[2]) continue;
        }
        for (int dy = -1; dy <= 1; ++dy) {
            int cy = L.c[1] + dy;
            if (I.periodic[1]) cy = wrapi(cy, I.nc[1]);
            else if (cy < 0 || cy >= I.nc[1]) continue;
            Row<R> row;
            row.base = I.cell_base + (uint32_t)nx * ((uint32_t)cy + (uint32_t)I.nc[1] * (uint32_t)cz);
            row.code = ((uint32_t)(1 - dy) << 2) | ((uint32_t)(1 - dz) << 4);
            row.dy1 = (float)(1 - dy);
            row.dz1 = (float)(1 - dz);
            // runs [a, b) and, per run, dcx = db - (k >= m0) - (k >= m1): m0 and m1 are
            // the starts of i's cell and the next where the run reaches them
            uint32_t a0, b0, a1 = 0, b1 = 0, m00, m01 = ~0u, m10 = ~0u, m11 = ~0u;
            int db0 = 1, db1 = 0;
            const int x0 = L.c[0] - 1, x1 = L.c[0] + 1;
            if (!I.periodic[0]) {
                a0 = cstart[row.base + (uint32_t)max(x0, 0)];
                b0 = cstart[row.base + (uint32_t)min(x1, nx - 1) + 1];
                m00 = cstart[row.base + (uint32_t)L.c[0]];
                m01 = cstart[row.base + (uint32_t)L.c[0] + 1];
            } else if (x0 < 0) {
                // cell nx - 1 (dcx = 1), then cells 0 and 1 (dcx = 0, -1)
                a0 = cstart[row.base + (uint32_t)(nx - 1)];
                b0 = cstart[row.base + (uint32_t)nx];
                m00 = ~0u;
                a1 = cstart[row.base];
                b1 = cstart[row.base + (uint32_t)x1 + 1];
                m10 = cstart[row.base + 1];
            } else if (x1 >= nx) {
                // cells nx - 2 and nx - 1 (dcx = 1, 0), then cell 0 (dcx = -1)
                a0 = cstart[row.base + (uint32_t)x0];
                b0 = cstart[row.base + (uint32_t)nx];
                m00 = cstart[row.base + (uint32_t)(nx - 1)];
                a1 = cstart[row.base];
                b1 = cstart[row.base + 1];
                db1 = -1;
            } else {
                a0 = cstart[row.base + (uint32_t)x0];
                b0 = cstart[row.base + (uint32_t)x1 + 1];
                m00 = cstart[row.base + (uint32_t)L.c[0]];
                m01 = cstart[row.base + (uint32_t)L.c[0] + 1];
            }
            for (int seg = 0; seg < 2; ++seg) {
                const uint32_t a = seg ? a1 : a0, b = seg ? b1 : b0;
                const uint32_t m0 = seg ? m10 : m00, m1 = seg ? m11 : m01;
                const int db = seg ? db1 : db0;
                if constexpr (ALL) {
                    // group-uniform trip count: every lane of the group sees every slot
                    for (uint32_t kb = a; kb < b; kb += U * P) {
                        const uint32_t k0 = kb + sub;
                        R4<R> pj[U];
                        uint32_t fj[U];
#pragma unroll
                        for (int u = 0; u < U; ++u) {
                            const uint32_t kk = min(k0 + (uint32_t)(u * P), b - 1);
                            pj[u] = pos[kk];
                            fj[u] = infos[kk];
                        }
#pragma unroll
                        for (int u = 0; u < U; ++u) {
                            const uint32_t k = k0 + (uint32_t)(u * P);
                            R r[3];
                            const int dcx = db - (int)(k >= m0) - (int)(k >= m1);
                            const uint32_t code = pair_r<DIM>(I, L, row, pj[u], dcx, r);
                            const R r2 = dist2<DIM>(r[0], r[1], r[2]);
                            body(k, r, r2, pj[u], info_phase(fj[u]), code, k < b && k != i && r2 < cut2);
                        }
                    }
                } else {
                    for (uint32_t k0 = a + sub; k0 < b; k0 += U * P) {
                        R4<R> pj[U];
                        uint32_t fj[U];
#pragma unroll
                        for (int u = 0; u < U; ++u) {
                            const uint32_t kk = min(k0 + (uint32_t)(u * P), b - 1);
                            pj[u] = pos[kk];
                            fj[u] = infos[kk];
                        }
#pragma unroll
                        for (int u = 0; u < U; ++u) {
                            const uint32_t k = k0 + (uint32_t)(u * P);
                            if (k < b && k != i) {
                                R r[3];
                                const int dcx = db - (int)(k >= m0) - (int)(k >= m1);
                                const uint32_t code = pair_r<DIM>(I, L, row, pj[u], dcx, r);
                                const R r2 = dist2<DIM>(r[0], r[1], r[2]);
                                if (r2 < cut2) body(k, r, r2, pj[u], info_phase(fj[u]), code);
                            }
                        }
                    }
                }
            }
        }
    }
}

struct NoExtra {};

// Largest block of the neighbour passes.  Larger blocks (tried up to 1024 threads) were
// slower on the 3D drop: fewer, larger workgroups leave a longer tail, and the register
// cap of a 1024-thread block (128) makes the force pass spill.
template <class R> struct MaxBlock { static constexpr int value = 256; };

// Visit the entries of i's neighbour list with |r_ij|^2 < 4h^2 at the positions `pos`
// (an array of records, or anything that gives particle k's record as pos[k]):
// body(j, r_ij, |r_ij|^2, record of j, phase of j, load(j)).  Entries are stored column-major
// (entry q of particle i at q * lstride + i), so a wave reads them coalesced; U entries are
// fetched per batch so that their loads are in flight together.  With P lanes per
// particle, lane `sub` takes the entries q = t P + sub: the row offset t P lstride is
// the same for all lanes (it is taken into scalar registers, so a list load needs no
// per-lane address arithmetic) and the lane part sub lstride + i is fixed.  The row
// stride is n rounded up to 32 entries, so that every row starts on a 128-byte line.  A batch may read
// entries past cnt: the list is padded with the sentinel entry (index n, a record far
// outside the domain) up to a multiple of kListPad, which every batch end stays below,
// so no entry is checked against the count.
// With SKIP, entries of phase skip_phase (known from the entry) are passed over before
// anything of them is read.
template <class R, int DIM, int U, int P, bool SKIP = false, class IC, class PS, class Load, class Body>
__device__ __forceinline__ void for_list(const Dev& d, const IC& I, const PS& pos,
                                         uint32_t i, const Lane<R>& L, uint32_t cnt, uint32_t sub,
                                         Load&& load, Body&& body, uint32_t skip_phase = 0)
{
    static_assert(kListPad % (U * P) == 0, "a batch of U entries on P lanes must divide the list padding");
    using X = decltype(load(0u));
    const uint32_t ls = d.lstride;
    const uint32_t lane_off = (sub * ls + i) * 4u;   // < 2^30: lstride <= 2^25, sub < 8
    const R cut2 = cut2_of<R>(I);
    // t is the same in every active lane (all lanes run the same batches; lanes only
    // leave the loop early), so the row address is wave-uniform: a list load is a buffer
    // load whose resource (the row's base) is built in scalar registers, with the lane's
    // fixed 32-bit offset
    auto entry = [&](uint32_t t) {
        const uint32_t* row = d.nbl + (size_t)ufirst(t) * ((size_t)P * ls);
        const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc((void*)row, (short)0, 0x7fffffff, 0x00020000);
        return (uint32_t)__builtin_amdgcn_raw_buffer_load_b32(rs, (int)lane_off, 0, 0);
    };
    // the entries of the next batch are in flight while a batch is computed; they are
    // requested after the current gathers: vector loads retire in order, so a wait for
    // the gathers does not wait for the list entries too
    uint32_t nxt[U];
    if (sub < cnt) {
#pragma unroll
        for (int u = 0; u < U; ++u) nxt[u] = entry((uint32_t)u);
    }
    for (uint32_t t0 = 0; t0 * P + sub < cnt; t0 += U) {
        uint32_t e[U];
        R4<R> pj[U];
        X x[U];
#pragma unroll
        for (int u = 0; u < U; ++u) e[u] = nxt[u];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint32_t k = e[u] & kIdxMask;
            if (!SKIP || entry_phase(e[u]) != skip_phase) {
                pj[u] = pos[k];
                x[u] = load(k);
            }
        }
        if ((t0 + U) * P + sub < cnt) {
#pragma unroll
            for (int u = 0; u < U; ++u) nxt[u] = entry(t0 + U + (uint32_t)u);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (!SKIP || entry_phase(e[u]) != skip_phase) {
                R r[3];
                list_pair_r<DIM>(I, L, pj[u], e[u], r);
                const R r2 = dist2<DIM>(r[0], r[1], r[2]);
                if (r2 < cut2) body(e[u] & kIdxMask, r, r2, pj[u], entry_phase(e[u]), x[u]);
            }
        }
    }
}

// The list walk of a pass with many lanes per particle (U P entries per round, more
// than the padding): an entry past the count reads as the sentinel, and the entry loads
// take plain 64-bit addresses.  Entries of phase skip_phase are passed over before their
// records are read.  For the short walks of the colour pass, whose time is the latency
// of one walk: with 64 lanes, one round covers a whole list.
template <class R, int DIM, int U, int P, class IC, class PS, class Load, class Body>
__device__ __forceinline__ void for_list_wide(const Dev& d, const IC& I, const PS& pos, uint32_t i,
                                              const Lane<R>& L, uint32_t cnt, uint32_t sub, Load&& load,
                                              Body&& body, uint32_t skip_phase)
{
    using X = decltype(load(0u));
    const size_t n = (size_t)d.n;
    const R cut2 = cut2_of<R>(I);
    for (uint32_t q0 = sub; q0 < cnt; q0 += (uint32_t)(U * P)) {
        uint32_t e[U];
        R4<R> pj[U];
        X x[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint32_t q = q0 + (uint32_t)(u * P);
            e[u] = q < cnt ? d.nbl[(size_t)q * d.lstride + i] : (uint32_t)n;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (entry_phase(e[u]) != skip_phase) {
                const uint32_t k = e[u] & kIdxMask;
                pj[u] = pos[k];
                x[u] = load(k);
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (entry_phase(e[u]) != skip_phase) {
                R r[3];
                list_pair_r<DIM>(I, L, pj[u], e[u], r);
                const R r2 = dist2<DIM>(r[0], r[1], r[2]);
                if (r2 < cut2) body(e[u] & kIdxMask, r, r2, pj[u], entry_phase(e[u]), x[u]);
            }
        }
    }
}

// Either the list (normal case) or, for a particle whose list overflowed, the stencil.
// The stencil fallback is rare and walks one candidate at a time: batching it would
// raise the register count, and so lower the occupancy, of the common list path.
// WIDE: the list walk of for_list_wide (SKIP implied).
template <class R, int DIM, int U, int P, bool SKIP = false, bool WIDE = false, class IC, class PS, class Load,
          class Body>
__device__ __forceinline__ void for_each_neighbor(const Dev& d, const IC& I, const Sorted& O,
                                                  const PS& pos, uint32_t i, const Lane<R>& L,
                                                  uint32_t sub, Load&& load, Body&& body, uint32_t skip_phase = 0)
{
    const uint32_t cnt = d.nbc[i];
    if (cnt <= d.cap) {
        if constexpr (WIDE) for_list_wide<R, DIM, U, P>(d, I, pos, i, L, cnt, sub, load, body, skip_phase);
        else for_list<R, DIM, U, P, SKIP>(d, I, pos, i, L, cnt, sub, load, body, skip_phase);
    } else {
        for_neighbors<R, DIM, P, 1>(I, d.cstart, O, pos, i, L, cut2_of<R>(I), sub,
                                 [&](uint32_t k, const R* r, R r2, const R4<R>& pj, uint32_t phj, uint32_t) {
                                     body(k, r, r2, pj, phj, load(k));
                                 });
    }
}

// Sum over the P consecutive lanes that share one particle (P a power of two up to 64;
// the lanes of a group are all active or all inactive).
template <int P, class T>
__device__ __forceinline__ T group_sum(T v)
{
    static_assert(P >= 1 && P <= 64 && (P & (P - 1)) == 0, "lanes per particle");
    if (P >= 2) v += __shfl_xor(v, 1, 64);
    if (P >= 4) v += __shfl_xor(v, 2, 64);
    if (P >= 8) v += __shfl_xor(v, 4, 64);
    if (P >= 16) v += __shfl_xor(v, 8, 64);
    if (P >= 32) v += __shfl_xor(v, 16, 64);
    if (P >= 64) v += __shfl_xor(v, 32, 64);
    return v;
}

// Particle and sub-lane of this thread in a neighbour pass with P lanes per particle.
template <int P>
__device__ __forceinline__ void lane_split(int remap, uint32_t& i, uint32_t& sub)
{
    const uint32_t t = tile_index(remap) * blockDim.x + threadIdx.x;
    i = t / P;
    sub = t % P;
}

// ---------------------------------------------------------- neighbour build

// a1: cell hash.  FP64 takes floor((x - lo)/s); FP32 finds the cell that an offset
// which left its cell moved into (the gather then moves the offset, folding the
// rounding of the shift into the compensation term).  Each particle bumps its cell
// counter (the returned value is its provisional slot).

// FP32 form: the cell of a particle whose offset o (compensation e) left its cell c.  The
// offset moves by whole cells, o - sh cs = (o - sh s) - sh (cs - s) with s the FP32 cell
// size: o - sh s is taken with its rounding error (TwoSum; sh s is exact for |sh| <= 2),
// and that error and -sh (cs - s) go into the compensation term.  Returns true when the
// particle left a non-periodic domain (its cell is then clamped); raw receives the cells
// before clamping.  The hash takes the new cell from it and the gather the moved offset,
// both from the unchanged old state set, so a build stopped before its end leaves that
// set as it was.
template <int DIM>
__device__ __forceinline__ bool recell(const InstDev& I, uint32_t* status, int c[3], float o[3], float e[3],
                                       int raw[3])
{
    bool out = false;
    for (int dd = 0; dd < DIM; ++dd) {
        if (!isfinite(o[dd])) {
            atomicOr(status, ST_NONFINITE);
            o[dd] = 0.0f;
        }
        const float s = I.f_cs[dd];
        const float sh = fminf(fmaxf(floorf(o[dd] / s), -1.0e6f), 1.0e6f);
        raw[dd] = c[dd] + (int)sh;
        if (sh != 0.0f) {
            const float b = -sh * s;
            const float sum = o[dd] + b;
            const float bv = sum - o[dd];
            const float err = (o[dd] - (sum - bv)) + (b - bv);
            o[dd] = sum;
            e[dd] += err - sh * I.f_cs_lo[dd];
            int ci = c[dd] + (int)sh;
            if (I.periodic[dd]) {
                ci = ((ci % I.nc[dd]) + I.nc[dd]) % I.nc[dd];
            } else if (ci < 0 || ci >= I.nc[dd]) {
                out = true;
                ci = ci < 0 ? 0 : I.nc[dd] - 1;
            }
            c[dd] = ci;
        }
    }
    return out;
}

// a1 for one particle: its new cell key.
template <class R, int DIM>
__device__ __forceinline__ uint32_t hash_one(const Dev& d, int cur, uint32_t k)
{
    const Sorted& O = d.O[cur];
    const uint32_t info = O.info[k];
    const InstDev& I = d.inst[info_inst(info)];
    int c[3] = {0, 0, 0};
    int raw[3] = {0, 0, 0};     // cells before clamping (for the fault record)
    double xa[3] = {0.0, 0.0, 0.0};
    bool out = false;
    if constexpr (sizeof(R) == 8) {
        const double4 p = ((const double4*)d.S[cur].pos)[k];
        const double x[3] = {p.x, p.y, p.z};
        for (int dd = 0; dd < DIM; ++dd) {
            if (!isfinite(x[dd])) atomicOr(d.status, ST_NONFINITE);
            double v = floor((x[dd] - I.lo[dd]) / I.cs[dd]);
            int ci = isfinite(v) ? (int)fmax(fmin(v, 1e9), -1e9) : 0;
            raw[dd] = ci;
            xa[dd] = x[dd];
            if (ci < 0 || ci >= I.nc[dd]) {
                if (!I.periodic[dd]) out = true;
                ci = ci < 0 ? 0 : I.nc[dd] - 1;
            }
            c[dd] = ci;
        }
    } else {
        const float4 p = ((const float4*)d.S[cur].pos)[k];
        const float4 lo = d.S[cur].plo[k];
        cell_of_key(I, O.key[k], c);
        float o[3] = {p.x, p.y, p.z};
        float e[3] = {lo.x, lo.y, lo.z};
        for (int dd = 0; dd < DIM; ++dd)
            xa[dd] = I.lo[dd] + (double)c[dd] * I.cs[dd] + (double)o[dd] + (double)e[dd];
        out = recell<DIM>(I, d.status, c, o, e, raw);
    }
    if (out) {
        atomicOr(d.status, ST_DOMAIN);
        if (atomicCAS(&d.fault->claimed, 0u, 1u) == 0u) {
            d.fault->id = O.id[k];
            d.fault->inst = info_inst(info);
            for (int dd = 0; dd < 3; ++dd) {
                d.fault->cell[dd] = raw[dd];
                d.fault->x[dd] = xa[dd];
            }
        }
    }
    return I.cell_base + (uint32_t)c[0] + (uint32_t)I.nc[0] * ((uint32_t)c[1] + (uint32_t)I.nc[1] * (uint32_t)c[2]);
}


// A grid barrier of a one-launch build timed out: every later build and every pass that
// changes the state or its rates returns at once, so the state stays as that build found
// it until the host rebuilds.
__device__ __forceinline__ bool stalled(const Dev& d)
{
    return (*d.status & ST_STALL) != 0u;
}

// Start of a step (or of a rate evaluation): rebuild the sort and the list when the host
// asked for it, or when some particle's reach (its displacement since the last build
// plus the longest half step the coming predictor can give it) is within 1 % of half
// the skin.  Every block takes the decision from the same inputs (nothing changes them
// before the scan's middle pass, which resets them); block 0 publishes it in flag 0.
// No rebuild either after a grid barrier of the one-launch build stalled.
__device__ __forceinline__ bool build_decision(const Dev& d)
{
    __shared__ int any;
    if (threadIdx.x == 0) any = d.flags[1] ? 1 : 0;
    __syncthreads();
    for (int b = threadIdx.x; b < d.ninst; b += blockDim.x)
        if (sqrt(__longlong_as_double((long long)d.run[b].reach2)) > d.inst[b].rebuild_e) atomicOr(&any, 1);
    __syncthreads();
    const bool rebuild = any != 0 && !stalled(d);
    if (blockIdx.x == 0 && threadIdx.x == 0) d.flags[0] = rebuild ? 1u : 0u;
    return rebuild;
}

// a1 for slot k of a wave (k >= n: an idle lane; the whole wave takes part).
template <class R, int DIM>
__device__ __forceinline__ void hash_phase(const Dev& d, int cur, uint32_t k)
{
    const bool valid = k < d.n;
    uint32_t key = 0;
    if (valid) key = hash_one<R, DIM>(d, cur, k);
    // lanes of one wave mostly share a cell: one counter update per distinct key
    const int lane = threadIdx.x & 63;
    unsigned long long todo = __ballot(valid);
    uint32_t slot = 0;
    while (todo) {
        const int leader = __ffsll((long long)todo) - 1;
        const uint32_t kl = __shfl(key, leader, 64);
        const unsigned long long same = __ballot(valid && key == kl) & todo;
        uint32_t base = 0;
        if (lane == leader) base = atomicAdd(&d.cnt[kl], (uint32_t)__popcll(same));
        base = __shfl(base, leader, 64);
        if ((same >> lane) & 1ull) slot = base + (uint32_t)__popcll(same & ((1ull << lane) - 1ull));
        todo &= ~same;
    }
    if (valid) {
        d.newkey[k] = key;
        d.slot[k] = slot;
    }
}

template <class R, int DIM>
__global__ void k_hash(Dev d)
{
    if (!build_decision(d)) return;
    hash_phase<R, DIM>(d, *d.curp, blockIdx.x * blockDim.x + threadIdx.x);
}

// a4 (cell start table): exclusive scan of the per-cell counts in three passes.
constexpr int SCAN_THREADS = 256, SCAN_ITEMS = 8, SCAN_TILE = SCAN_THREADS * SCAN_ITEMS;

__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t v, uint32_t& total)
{
    __shared__ uint32_t wsum[SCAN_THREADS / 64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    uint32_t incl = v;
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t t = __shfl_up(incl, off, 64);
        if (lane >= off) incl += t;
    }
    if (lane == 63) wsum[w] = incl;
    __syncthreads();
    uint32_t base = 0;
    total = 0;
    for (int k = 0; k < SCAN_THREADS / 64; ++k) {
        if (k < w) base += wsum[k];
        total += wsum[k];
    }
    __syncthreads();
    return base + incl - v;
}

// Pass 1 for one tile (the whole block takes part): its sum into sums[tile].
__device__ __forceinline__ void scan_reduce_tile(const uint32_t* __restrict__ in, uint32_t n,
                                                 uint32_t* __restrict__ sums, uint32_t tile)
{
    const uint32_t base = tile * SCAN_TILE + threadIdx.x * SCAN_ITEMS;
    uint32_t s = 0;
    for (int j = 0; j < SCAN_ITEMS; ++j)
        if (base + j < n) s += in[base + j];
    uint32_t total;
    block_exclusive_scan(s, total);
    if (threadIdx.x == 0) sums[tile] = total;
}

__global__ void k_scan_reduce(const uint32_t* __restrict__ gate, const uint32_t* __restrict__ in, uint32_t n,
                              uint32_t* __restrict__ sums)
{
    if (!*gate) return;
    scan_reduce_tile(in, n, sums, blockIdx.x);
}

// After every hash block has taken the decision (one block): the decision's inputs are
// reset, and so is the count of colour-pass particles the list build appends.
__device__ __forceinline__ void reset_decision(const Dev& d)
{
    if (threadIdx.x == 0) {
        d.flags[1] = 0u;
        *d.icount = 0u;
    }
    for (int b = threadIdx.x; b < d.ninst; b += blockDim.x) d.run[b].reach2 = 0ull;
}

// The gathered copy becomes the current state set (one block); prevp keeps the old one.
__device__ __forceinline__ void flip_sets(const Dev& d)
{
    if (threadIdx.x == 0) {
        *d.prevp = *d.curp;
        *d.curp = 1 - *d.curp;
    }
    for (int b = threadIdx.x; b < d.ninst; b += blockDim.x) d.run[b].builds += 1;
}

// Sum of the tile sums before tile t (the whole block takes part).
__device__ __forceinline__ uint32_t tile_prefix(const uint32_t* __restrict__ sums, uint32_t t)
{
    uint32_t v = 0;
    for (uint32_t u = threadIdx.x; u < t; u += blockDim.x) v += sums[u];
    uint32_t total;
    block_exclusive_scan(v, total);
    return total;
}

// Pass 2 (one block): exclusive scan of the tile sums, in place.
__device__ __forceinline__ void scan_top_block(const Dev& d, uint32_t* __restrict__ sums, uint32_t ntiles)
{
    // the seven-launch build flips here: its later launches read the old set through prevp
    reset_decision(d);
    flip_sets(d);
    // one block; each thread owns a run of ceil(ntiles / 256) tile sums
    const uint32_t per = (ntiles + SCAN_THREADS - 1) / SCAN_THREADS;
    const uint32_t a = threadIdx.x * per;
    uint32_t s = 0;
    for (uint32_t j = 0; j < per; ++j)
        if (a + j < ntiles) s += sums[a + j];
    uint32_t total;
    uint32_t run = block_exclusive_scan(s, total);
    for (uint32_t j = 0; j < per; ++j)
        if (a + j < ntiles) {
            const uint32_t v = sums[a + j];
            sums[a + j] = run;
            run += v;
        }
}

__global__ void k_scan_top(Dev d, uint32_t* __restrict__ sums, uint32_t ntiles)
{
    if (!d.flags[0]) return;
    scan_top_block(d, sums, ntiles);
}

// Pass 3 for one tile, whose cells start at `prefix`: writes cstart[0..n] and clears
// the counters for the next build.
__device__ __forceinline__ void scan_down_tile(uint32_t* __restrict__ cnt, uint32_t n, uint32_t prefix,
                                               uint32_t* __restrict__ out, uint32_t tile)
{
    const uint32_t base = tile * SCAN_TILE + threadIdx.x * SCAN_ITEMS;
    uint32_t v[SCAN_ITEMS];
    uint32_t s = 0;
    for (int j = 0; j < SCAN_ITEMS; ++j) {
        v[j] = base + j < n ? cnt[base + j] : 0u;
        s += v[j];
    }
    uint32_t total;
    uint32_t run = block_exclusive_scan(s, total) + prefix;
    for (int j = 0; j < SCAN_ITEMS; ++j) {
        const uint32_t idx = base + j;
        if (idx < n) {
            out[idx] = run;
            cnt[idx] = 0u;
            if (idx == n - 1) out[n] = run + v[j];
        }
        run += v[j];
    }
}

__global__ void k_scan_down(const uint32_t* __restrict__ gate, uint32_t* __restrict__ cnt, uint32_t n,
                            const uint32_t* __restrict__ sums, uint32_t* __restrict__ out)
{
    if (!*gate) return;
    scan_down_tile(cnt, n, sums[blockIdx.x], out, blockIdx.x);
}

// Provisional scatter into the cell's segment (a slot outside [0, n) can only follow a
// stalled barrier, whose build is abandoned: it is skipped).
__device__ __forceinline__ void scatter_one(const Dev& d, int old, uint32_t k)
{
    if (k >= d.n) return;
    const uint32_t p = d.cstart[d.newkey[k]] + d.slot[k];
    if (p >= d.n) return;
    d.tsrc[p] = k;
    d.tid[p] = d.O[old].id[k];
}

__global__ void k_scatter(Dev d)
{
    if (!d.flags[0]) return;
    scatter_one(d, *d.prevp, blockIdx.x * blockDim.x + threadIdx.x);
}

// a2 made unique, a3: within a cell, order by original id (rank = number of smaller
// ids), and copy the particle's state from the old set (`old`) into its slot of the new
// one (FP32: with its offset moved into the new cell).
template <class R, int DIM>
__device__ __forceinline__ void rank_one(const Dev& d, int old, uint32_t s, int with_ref)
{
    if (s >= d.n) return;
    const uint32_t src = d.tsrc[s];
    if (src >= d.n) return;
    const uint32_t key = d.newkey[src];
    const uint32_t a = d.cstart[key], b = min(d.cstart[key + 1], (uint32_t)d.n);
    const uint32_t me = d.tid[s];
    uint32_t r = 0;
    for (uint32_t t = a; t < b; ++t) r += d.tid[t] < me ? 1u : 0u;
    const uint32_t k = a + r;
    if (k >= d.n) return;
    const Sorted& A = d.O[old];
    const Sorted& B = d.O[1 - old];
    B.key[k] = key;
    B.id[k] = me;
    B.info[k] = A.info[src];
    if (with_ref) B.ref[k] = A.ref[src];
    const StateSet& SA = d.S[old];
    const StateSet& SB = d.S[1 - old];
    ((R4<R>*)SB.vel)[k] = ((const R4<R>*)SA.vel)[src];
    ((R4<R>*)SB.aux)[k] = ((const R4<R>*)SA.aux)[src];
    if constexpr (sizeof(R) == 4) {
        const InstDev& I = d.inst[info_inst(A.info[src])];
        const float4 p = ((const float4*)SA.pos)[src];
        const float4 lo = SA.plo[src];
        int c[3] = {0, 0, 0}, raw[3];
        cell_of_key(I, A.key[src], c);
        float o[3] = {p.x, p.y, p.z};
        float e[3] = {lo.x, lo.y, lo.z};
        recell<DIM>(I, d.status, c, o, e, raw);
        ((float4*)SB.pos)[k] = make_float4(o[0], o[1], o[2], p.w);
        SB.plo[k] = make_float4(e[0], e[1], e[2], lo.w);
        SB.vlo[k] = SA.vlo[src];
    } else {
        ((R4<R>*)SB.pos)[k] = ((const R4<R>*)SA.pos)[src];
    }
}

template <class R, int DIM>
__global__ void k_rank(Dev d, int with_ref)
{
    if (!d.flags[0]) return;
    rank_one<R, DIM>(d, *d.prevp, blockIdx.x * blockDim.x + threadIdx.x, with_ref);
}

// Neighbour list at the current positions: every j within the cell size (2 + skin) h
// (with a rounding margin).  Together with the rebuild rule this holds every pair within
// 2h at any state evaluated before the next rebuild.  NlistLanes lanes share a particle
// and take every NlistLanes-th candidate; a ballot ranks each slot's accepted
// candidates, so the list keeps the candidate order (the same as one lane would write).
// Particles with an other-phase particle in their list (the only ones whose colour
// gradient can be non-zero) are appended to the colour-pass index list; every other
// particle gets a zero gradient and a cleared interface flag here, once per build.
// Two lanes in FP32 (128 particles per 256-thread block), four in FP64, whose records
// are twice as large: its staged runs for 128 particles would exceed the LDS buffer.
template <class R> struct NlistLanes { static constexpr int value = sizeof(R) == 4 ? 2 : 4; };
template <class R> struct NlistTile { static constexpr uint32_t value = 256u / NlistLanes<R>::value; };

// LDS staging of the list build.  The consecutive particles of a block (128 in FP32, 64
// in FP64) usually lie in a few cells of one cell row; the candidates of all of them are
// then the runs of nine rows (three in 2D) over that x range plus one cell on each side.
// The block copies those runs (position record, phase in w) into LDS once with coalesced
// loads, and every lane walks its particle's stencil there instead of gathering each
// candidate from memory (about 540 per particle).  A block whose particles span two rows
// or two instances, whose x range wraps a periodic x axis, or whose runs exceed the
// buffer walks memory as before.  The staged walk visits the same candidates in the same
// order, so the list is the same.
constexpr uint32_t kStageBytes = 39936u;   // four blocks of the build fit one CU's 160 KB of LDS
template <class R> struct Stage {
    static constexpr uint32_t cap = kStageBytes / sizeof(R4<R>);
    static constexpr uint32_t slack = 16;   // a batch (U P candidates) may read this far past a run
    uint32_t g0[9], l0[10];   // per stencil row present: first staged index, its LDS offset
    uint32_t rbase[9];        // key of the row's cell xlo
    int xlo, ok;
};

template <class R> __device__ __forceinline__ R phase_as(uint32_t ph)
{
    if constexpr (sizeof(R) == 8) return (double)ph;
    else return __uint_as_float(ph);
}
template <class R> __device__ __forceinline__ uint32_t phase_of(R w)
{
    if constexpr (sizeof(R) == 8) return (uint32_t)w;
    else return __float_as_uint(w);
}

// Stages the runs for the block's particles i0 .. i0 + NlistTile - 1 (those below n).
// Called by every thread of the block; returns the same answer in all of them.
template <class R, int DIM>
__device__ bool stage_rows(const Dev& d, int cur, uint32_t i0, R4<R>* rec, Stage<R>& h)
{
    const Sorted& O = d.O[cur];
    const uint32_t n = (uint32_t)d.n;
    if (threadIdx.x == 0) {
        h.ok = 0;
        const uint32_t ie = min(i0 + NlistTile<R>::value, n) - 1u;
        const uint32_t inst = info_inst(O.info[i0]);
        if (inst == info_inst(O.info[ie])) {
            const InstDev& I = d.inst[inst];
            int ca[3], cb[3];
            cell_of_key(I, O.key[i0], ca);
            cell_of_key(I, O.key[ie], cb);
            const int nx = I.nc[0];
            int xlo = ca[0] - 1, xhi = cb[0] + 1;
            bool ok = ca[1] == cb[1] && ca[2] == cb[2];
            if (I.periodic[0]) ok = ok && xlo >= 0 && xhi < nx;
            xlo = max(xlo, 0);
            xhi = min(xhi, nx - 1);
            ok = ok && xhi - xlo < 256;   // a record's cell index from xlo takes 8 bits
            uint32_t r = 0, tot = 0;
            const int zlo = DIM == 3 ? -1 : 0, zhi = DIM == 3 ? 1 : 0;
            for (int dz = zlo; dz <= zhi && ok; ++dz) {
                int cz = ca[2] + dz;
                if (DIM == 3) {
                    if (I.periodic[2]) cz = wrapi(cz, I.nc[2]);
                    else if (cz < 0 || cz >= I.nc[2]) continue;
                }
                for (int dy = -1; dy <= 1; ++dy) {
                    int cy = ca[1] + dy;
                    if (I.periodic[1]) cy = wrapi(cy, I.nc[1]);
                    else if (cy < 0 || cy >= I.nc[1]) continue;
                    const uint32_t base = I.cell_base + (uint32_t)nx * ((uint32_t)cy + (uint32_t)I.nc[1] * (uint32_t)cz);
                    const uint32_t g0 = d.cstart[base + (uint32_t)xlo], g1 = d.cstart[base + (uint32_t)xhi + 1];
                    h.g0[r] = g0;
                    h.l0[r] = tot;
                    h.rbase[r] = base + (uint32_t)xlo;
                    tot += g1 - g0;
                    ++r;
                }
            }
            h.l0[r] = tot;
            h.xlo = xlo;
            h.ok = ok && tot + Stage<R>::slack <= Stage<R>::cap ? (int)r + 1 : 0;
        }
    }
    __syncthreads();
    const int nr = h.ok - 1;
    if (nr < 0) return false;
    const uint32_t tot = h.l0[nr];
    const R4<R>* pos = (const R4<R>*)d.S[cur].pos;
    for (uint32_t q = threadIdx.x; q < tot; q += blockDim.x) {
        int r = 0;
        while (q >= h.l0[r + 1]) ++r;
        const uint32_t k = h.g0[r] + (q - h.l0[r]);
        R4<R> v = pos[k];
        // w: the phase in bit 0, the cell's x index from xlo in bits 8-15 (at most 34 cells)
        v.w = phase_as<R>(info_phase(O.info[k]) | ((O.key[k] - h.rbase[r]) << 8));
        rec[q] = v;
    }
    __syncthreads();
    return true;
}

// The stencil walk of for_neighbors (ALL form, x axis not wrapping) over the staged runs.
template <class R, int DIM, int P, int U, class IC, class Body>
__device__ __forceinline__ void for_staged(const IC& I, const uint32_t* __restrict__ cstart, const R4<R>* rec,
                                           const Stage<R>& h, uint32_t i, const Lane<R>& L, R cut2,
                                           uint32_t sub, Body&& body)
{
    const int nx = I.nc[0];
    const int zlo = DIM == 3 ? -1 : 0, zhi = DIM == 3 ? 1 : 0;
    const float cx1 = (float)(L.c[0] - h.xlo + 1);   // c_i + 1 along x, from xlo
    int rr = 0;
    for (int dz = zlo; dz <= zhi; ++dz) {
        int cz = L.c[2] + dz;
        if (DIM == 3) {
            if (I.periodic[2]) cz = wrapi(cz, I.nc[2]);
            else if (cz < 0 || cz >= I.nc[2]) continue;
        }
        for (int dy = -1; dy <= 1; ++dy) {
            int cy = L.c[1] + dy;
            if (I.periodic[1]) cy = wrapi(cy, I.nc[1]);
            else if (cy < 0 || cy >= I.nc[1]) continue;
            Row<R> row;
            row.base = I.cell_base + (uint32_t)nx * ((uint32_t)cy + (uint32_t)I.nc[1] * (uint32_t)cz);
            row.code = ((uint32_t)(1 - dy) << 2) | ((uint32_t)(1 - dz) << 4);
            row.dy1 = (float)(1 - dy);
            row.dz1 = (float)(1 - dz);
            const uint32_t a = cstart[row.base + (uint32_t)max(L.c[0] - 1, 0)];
            const uint32_t b = cstart[row.base + (uint32_t)min(L.c[0] + 1, nx - 1) + 1];
            const R4<R>* rw = rec + h.l0[rr] - h.g0[rr];   // staged record of candidate k: rw[k]
            ++rr;
            // a batch reads up to U P - 1 records past b, inside the buffer's slack; those
            // slots are not taken
            for (uint32_t kb = a; kb < b; kb += U * P) {
                const uint32_t k0 = kb + sub;
                const R4<R>* rk = rw + k0;
                R4<R> pj[U];
#pragma unroll
                for (int u = 0; u < U; ++u) pj[u] = rk[u * P];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const uint32_t k = k0 + (uint32_t)(u * P);
                    const uint32_t wb = phase_of<R>(pj[u].w);
                    R r[3];
                    uint32_t code;
                    if constexpr (sizeof(R) == 4) {
                        // c_i - c_j + 1 along x, from the record's cell index
                        const float fx = cx1 - (float)((wb >> 8) & 0xFFu);
                        r[0] = fmaf(fx, I.f_cs[0], L.om[0] - pj[u].x);
                        r[1] = fmaf(row.dy1, I.f_cs[1], L.om[1] - pj[u].y);
                        r[2] = DIM == 3 ? fmaf(row.dz1, I.f_cs[2], L.om[2] - pj[u].z) : 0.0f;
                        code = (uint32_t)fx | row.code;
                    } else {
                        code = pair_r<DIM>(I, L, row, pj[u], 0, r);
                    }
                    const R r2 = dist2<DIM>(r[0], r[1], r[2]);
                    body(k, r, r2, pj[u], wb & 1u, code, k < b && k != i && r2 < cut2);
                }
            }
        }
    }
}

template <class R, int DIM>
__device__ __forceinline__ void nlist_one(const Dev& d, int cur, uint32_t i, uint32_t sub,
                                          const R4<R>* rec = nullptr, const Stage<R>* stage = nullptr)
{
    constexpr int P = NlistLanes<R>::value;
    const Sorted& O = d.O[cur];
    const R4<R>* pos = (const R4<R>*)d.S[cur].pos;
    const R4<R> pi = pos[i];
    if (sub == 0) ((R4<R>*)d.xb)[i] = pi;
    const uint32_t lane = threadIdx.x & 63, gbase = lane & ~(uint32_t)(P - 1);
    const uint32_t gmask = (1u << P) - 1u, below = (1u << sub) - 1u;
    per_instance(d, info_inst(O.info[i]), [&](const InstU& I) {
        Lane<R> L;
        L.load(I, pi, O.key[i]);
        const uint32_t ph = info_phase(O.info[i]);
        uint32_t* nb = d.nbl + i;
        const size_t n = (size_t)d.n, ls = d.lstride;
        const uint32_t cap = d.cap;
        uint32_t cnt = 0;
        uint32_t other = 0;
        auto take = [&](uint32_t k, const R*, R, const R4<R>&, uint32_t phj, uint32_t code, bool in) {
            uint32_t rank, accepted;
            if constexpr (P == 2) {
                // the pair's other lane by a lane swap (DPP quad_perm [1, 0, 3, 2]): lane 1's
                // candidate follows lane 0's
                const uint32_t mine = in ? 1u : 0u;
                const uint32_t theirs = (uint32_t)__builtin_amdgcn_mov_dpp((int)mine, 0xB1, 0xF, 0xF, false);
                rank = sub & theirs;
                accepted = mine + theirs;
            } else {
                const uint32_t grp = (uint32_t)(__ballot(in) >> gbase) & gmask;
                rank = (uint32_t)__popc(grp & below);
                accepted = (uint32_t)__popc(grp);
            }
            if (in) {
                const uint32_t q = cnt + rank;
                if (q < cap) nb[(size_t)q * ls] = k | (code << kIdxBits) | (phj << kPhaseShift);
                other |= phj ^ ph;
            }
            cnt += accepted;
        };
        if (stage)
            for_staged<R, DIM, P, StencilBatch<R>::U>(I, d.cstart, rec, *stage, i, L, cutl2_of<R>(I), sub, take);
        else
            for_neighbors<R, DIM, P, StencilBatch<R>::U, true>(I, d.cstart, O, pos, i, L, cutl2_of<R>(I), sub, take);
        // pad with the sentinel entry (index n, code 0, phase 0) to a multiple of kListPad
        if (cnt <= cap) {
            const uint32_t end = (cnt + kListPad - 1u) & ~(kListPad - 1u);
            for (uint32_t q = cnt + sub; q < end; q += P) nb[(size_t)q * ls] = (uint32_t)n;
        }
        const bool gother = ((uint32_t)(__ballot(other != 0u) >> gbase) & gmask) != 0u;
        if (sub == 0) {
            d.nbc[i] = cnt;
            const uint32_t f = O.info[i];
            O.info[i] = gother ? (f | kInfoColour) : (f & ~kInfoColour);
        }
        const bool append = sub == 0 && gother;
        const unsigned long long m = __ballot(append);
        const int leader = __ffsll((long long)m) - 1;
        uint32_t base = 0;
        if ((int)lane == leader) base = atomicAdd(d.icount, (uint32_t)__popcll(m));
        base = __shfl(base, leader < 0 ? 0 : leader, 64);
        if (append) {
            d.ilist[base + (uint32_t)__popcll(m & ((1ull << lane) - 1ull))] = i;
        } else if (sub == 0 && !gother) {
            R4<R> z;
            z.x = z.y = z.z = z.w = (R)0;
            ((R4<R>*)d.gc)[i] = z;
            R* vw = (R*)d.S[cur].vel + 4 * (size_t)i + 3;
            *vw = fabs(*vw);
        }
    });
}

// The list of the block's particles i0 .. i0 + NlistTile - 1: staged when the runs allow it.
// Every thread of the (256-thread) block calls it.
template <class R, int DIM>
__device__ __forceinline__ void nlist_tile(const Dev& d, int cur, uint32_t i0)
{
    __shared__ R4<R> rec[Stage<R>::cap];
    __shared__ Stage<R> stage;
    const bool staged = stage_rows<R, DIM>(d, cur, i0, rec, stage);
    const uint32_t i = i0 + threadIdx.x / NlistLanes<R>::value, sub = threadIdx.x % NlistLanes<R>::value;
    if (i < d.n) nlist_one<R, DIM>(d, cur, i, sub, rec, staged ? &stage : nullptr);
    __syncthreads();   // the buffer is refilled by the block's next tile
}

template <class R, int DIM>
__global__ void __launch_bounds__(256) k_nlist(Dev d, int remap)
{
    if (!d.flags[0]) return;
    const uint32_t i0 = tile_index(remap) * NlistTile<R>::value;
    if (i0 >= d.n) return;
    nlist_tile<R, DIM>(d, *d.curp, i0);
}

// Grid-wide barrier of the one-launch build, whose grid is sized so that all its blocks
// are resident together.  Nothing is contended: each block stores the barrier's epoch
// into its own arrival slot, block 0's threads wait for all slots together, then block
// 0 stores the epoch into eight release words on separate cache lines, each polled by
// one eighth of the blocks.  Epochs grow across launches (word 0 holds the next base),
// so no slot needs clearing.  Every wait is bounded: a block that waits too long
// records ST_STALL and returns false, as do the blocks that wait on it after; later
// builds and every pass of the step are then skipped, and the host rebuilds from the
// current state set, which the stopped build has not touched.  `forced` makes every
// wait of this barrier time out at once, so that tests can take the stall path without
// waiting.
constexpr uint32_t kBarrierSpins = 1u << 20;
constexpr uint32_t kBarRelease = 32;     // release word r at bar[kBarRelease * (1 + r)], r < 8
constexpr uint32_t kBarGroup = 512;      // two-level barrier: group word of group g at bar[kBarGroup + 32 g]
constexpr uint32_t kBarGo = 768;         // and its go word at bar[kBarGo + 32 g]
constexpr uint32_t kBarSlots = 1024;     // arrival slot of block b at bar[kBarSlots + b]
constexpr uint32_t kBarMaxBlocks = 4096; // the one-launch build uses at most this many blocks
constexpr uint32_t kBarXcc = kBarSlots + kBarMaxBlocks;   // XCD id of block b at bar[kBarXcc + b]
static_assert(kBarXcc + kBarMaxBlocks == kBarWords, "barrier area layout");

// Polls with relaxed loads (coherent, without the cache invalidation an acquire load
// carries on every iteration); the caller fences once after the wait.
__device__ __forceinline__ bool bar_wait(unsigned* w, unsigned epoch)
{
    uint32_t spins = 0;
    while ((int)(__hip_atomic_load(w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) - epoch) < 0) {
        __builtin_amdgcn_s_sleep(4);
        if (++spins >= kBarrierSpins) return false;
    }
    return true;
}

__device__ __forceinline__ bool grid_sync(const Dev& d, unsigned epoch, bool forced)
{
    __shared__ int ok;
    unsigned* bar = d.bar;
    __syncthreads();
    if (threadIdx.x == 0) {
        ok = 1;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");   // the block's writes, then its arrival
        __hip_atomic_store(&bar[kBarSlots + blockIdx.x], epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    if (blockIdx.x == 0) {
        __syncthreads();
        bool good = true;
        for (uint32_t b = threadIdx.x; b < gridDim.x && good; b += blockDim.x)
            good = !forced && bar_wait(&bar[kBarSlots + b], epoch);
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");   // what the arrivals this lane saw released
        if (!good) ok = 0;
        __syncthreads();
        if (threadIdx.x == 0 && ok) {
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            for (uint32_t r = 0; r < 8; ++r)
                __hip_atomic_store(&bar[kBarRelease * (1 + r)], epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    } else if (threadIdx.x == 0) {
        if (forced || !bar_wait(&bar[kBarRelease * (1 + (blockIdx.x & 7))], epoch)) ok = 0;
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");   // everything released before the epoch
    }
    __syncthreads();
    if (!ok && threadIdx.x == 0) atomicOr(d.status, ST_STALL);
    return ok != 0;
}

// The XCD (accelerator complex die) this wave runs on.
__device__ __forceinline__ uint32_t xcd_id() { return __builtin_amdgcn_s_getreg((3 << 11) | 20) & 15u; }

// Two-level form of grid_sync for a grid whose blocks b = g (mod 8) all run on one XCD
// (the caller checks this).  An agent-scope release writes back the whole L2 of the
// issuing wave's XCD and an acquire invalidates it; when every block does both, each of
// the eight L2s is written back and invalidated once per block (128 times on the 3D
// drop's grid of 1,024) while the other blocks of that XCD are already loading the next
// phase's data into it, and the phases after such a barrier ran 3 to 7 times slower than
// the same work as launches of their own.  Here block g < 8 leads group g: it waits for
// its members' arrivals, writes its XCD's L2 back once and posts the group word; block 0
// releases when every group has posted; each leader then invalidates its XCD's L2 once
// and posts the group's go word, on which the members invalidate only their own CU's L1.
// A member's stores are in its XCD's L2 once the block's barrier has waited for them,
// and that L2 is written back after the member arrived; a load after the go word misses
// an L2 invalidated after the release.  Waits are bounded as in grid_sync.
__device__ __forceinline__ bool grid_sync_two_level(const Dev& d, unsigned epoch, bool forced)
{
    __shared__ int ok;
    unsigned* bar = d.bar;
    const uint32_t nb = gridDim.x, G = min(nb, 8u), b = blockIdx.x;
    __syncthreads();   // every wave's stores have completed in this XCD's L2
    if (threadIdx.x == 0) {
        ok = 1;
        __hip_atomic_store(&bar[kBarSlots + b], epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    if (b < G) {
        bool good = true;
        for (uint32_t m = b + 8u * threadIdx.x; m < nb && good; m += 8u * blockDim.x)
            good = !forced && bar_wait(&bar[kBarSlots + m], epoch);
        const int arrived = __syncthreads_and(good ? 1 : 0);
        if (threadIdx.x == 0) {
            if (arrived) {
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");   // the group's writes, then its word
                __hip_atomic_store(&bar[kBarGroup + 32u * b], epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            } else {
                ok = 0;
            }
        }
        if (b == 0) {
            __syncthreads();
            bool posted = ok != 0;
            if (threadIdx.x < G && posted)
                posted = !forced && bar_wait(&bar[kBarGroup + 32u * threadIdx.x], epoch);
            const int all = __syncthreads_and(posted ? 1 : 0);
            if (threadIdx.x == 0) {
                if (all) {
                    for (uint32_t r = 0; r < G; ++r)
                        __hip_atomic_store(&bar[kBarRelease * (1 + r)], epoch, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT);
                } else {
                    ok = 0;
                }
            }
        }
        if (threadIdx.x == 0) {
            if (!ok || forced || !bar_wait(&bar[kBarRelease * (1 + b)], epoch)) ok = 0;
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");   // this XCD's L2 and this CU's L1
            if (ok) __hip_atomic_store(&bar[kBarGo + 32u * b], epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    } else if (threadIdx.x == 0) {
        if (forced || !bar_wait(&bar[kBarGo + 32u * (b & 7u)], epoch)) ok = 0;
        asm volatile("s_waitcnt vmcnt(0)\n\tbuffer_inv sc0" ::: "memory");   // this CU's L1
    }
    __syncthreads();
    if (!ok && threadIdx.x == 0) atomicOr(d.status, ST_STALL);
    return ok != 0;
}

// The whole build in one launch.  Every block takes the rebuild decision; on the steps
// without a rebuild (most of them) the launch ends there, where the seven-launch form
// pays for seven launches.  On a rebuild the phases above run grid-stride, separated by
// grid barriers.  stall_at = b in 1..5 forces barrier b to time out (0: none).
template <class R, int DIM>
__global__ void __launch_bounds__(256) k_build(Dev d, uint32_t ntiles, int with_ref, int stall_at)
{
    if (!build_decision(d)) return;
    const uint32_t n = d.n, T = gridDim.x * blockDim.x;
    // the phases read the old set and write the other one; the current-set word flips
    // only after the last barrier, so a build that stops at a barrier leaves the old set
    // current and whole
    const int old = *d.curp;
    // this launch's barrier epochs are base + 1 .. base + 5; block 0 advances the base
    // after the last barrier, when every block has read it
    const unsigned base = __hip_atomic_load(&d.bar[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (threadIdx.x == 0)
        __hip_atomic_store(&d.bar[kBarXcc + blockIdx.x], xcd_id(), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    for (uint32_t b0 = blockIdx.x * blockDim.x; b0 < n; b0 += T) hash_phase<R, DIM>(d, old, b0 + threadIdx.x);
    if (!grid_sync(d, base + 1, stall_at == 1)) return;
    // barriers 2-5 take the two-level form when the blocks of each residue mod 8 share an
    // XCD (the dispatcher deals blocks round-robin over the eight XCDs); every block reads
    // the same ids after barrier 1, so all take the same form
    bool same = true;
    for (uint32_t m = threadIdx.x; m < gridDim.x; m += blockDim.x)
        same = same && __hip_atomic_load(&d.bar[kBarXcc + m], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) ==
                           __hip_atomic_load(&d.bar[kBarXcc + (m & 7u)], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const bool two = __syncthreads_and(same ? 1 : 0) != 0;
    if (two && blockIdx.x == 0 && threadIdx.x == 0) d.flags[3] += 1u;   // counted for sphx_get_stats
    auto sync = [&](unsigned e, bool forced) {
        return two ? grid_sync_two_level(d, e, forced) : grid_sync(d, e, forced);
    };
    for (uint32_t t = blockIdx.x; t < ntiles; t += gridDim.x) scan_reduce_tile(d.cnt, d.ncell, d.scan_tmp, t);
    if (!sync(base + 2, stall_at == 2)) return;
    // each tile sums the tile sums before it (few), so the scan needs no middle pass
    if (blockIdx.x == 0) reset_decision(d);
    for (uint32_t t = blockIdx.x; t < ntiles; t += gridDim.x)
        scan_down_tile(d.cnt, d.ncell, tile_prefix(d.scan_tmp, t), d.cstart, t);
    if (!sync(base + 3, stall_at == 3)) return;
    for (uint32_t k = blockIdx.x * blockDim.x + threadIdx.x; k < n; k += T) scatter_one(d, old, k);
    if (!sync(base + 4, stall_at == 4)) return;
    for (uint32_t k = blockIdx.x * blockDim.x + threadIdx.x; k < n; k += T) rank_one<R, DIM>(d, old, k, with_ref);
    if (!sync(base + 5, stall_at == 5)) return;
    if (blockIdx.x == 0) {
        flip_sets(d);   // read by the launches after this one; the list below takes 1 - old
        if (threadIdx.x == 0) __hip_atomic_store(&d.bar[0], base + 5, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    for (uint32_t i0 = blockIdx.x * NlistTile<R>::value; i0 < n; i0 += gridDim.x * NlistTile<R>::value)
        nlist_tile<R, DIM>(d, 1 - old, i0);
}

// ------------------------------------------------------ per-particle state

// Density of particle k as FP64 (FP32 form stores rho - rho0).
template <class R, class IC>
__device__ __forceinline__ double rho_of(const IC& I, uint32_t phase, R stored)
{
    if constexpr (sizeof(R) == 8) return stored;
    else return (phase ? I.rho0[1] : I.rho0[0]) + (double)stored;   // no dynamic index: I may live in SGPRs
}

// Derived quantities of one particle from its stored density: V = m / rho into vel.w
// (positive: interface flag cleared) and aux.z (the copy read by the renormalisation),
// m P / rho^2 into aux.y, the density itself into aux.w.  The w slot of the position
// record holds m P / rho^2 while rates are evaluated (the force pass reads it per
// neighbour); from a state update to the next Eq. (7) it holds q = (rho - rho0) / rho
// instead, the one number per neighbour that Eq. (7) needs when masses are uniform
// per phase (device flag 2 says which).
template <class R>
__device__ __forceinline__ void derive_values(const InstDev& I, uint32_t phase, R stored, R m_, R& V, R& mA)
{
    const double rho = rho_of<R>(I, phase, stored);
    const double y = sizeof(R) == 8 ? rho / I.rho0[phase] : 1.0 + (double)stored / I.rho0[phase];
    const double P = tait(y, I.beta[phase]);
    const double m = (double)m_;
    V = (R)(m / rho);
    mA = (R)(m * (P / (rho * rho)));
}

template <class R>
__device__ __forceinline__ R q_of(const InstDev& I, uint32_t phase, R stored)
{
    const double rho = rho_of<R>(I, phase, stored);
    const double dr = sizeof(R) == 8 ? rho - I.rho0[phase] : (double)stored;
    return (R)(dr / rho);
}

template <class R>
__device__ __forceinline__ void derive_one(const InstDev& I, uint32_t phase, R stored, R4<R>& pos, R4<R>& vel,
                                           R4<R>& aux, bool qfield)
{
    R V, mA;
    derive_values<R>(I, phase, stored, aux.x, V, mA);
    pos.w = qfield ? q_of<R>(I, phase, stored) : mA;
    vel.w = V;
    aux.y = mA;
    aux.z = V;
    aux.w = stored;
}

// After Eq. (7): move the renormalised density into the state and re-derive.
// Eq. (7) runs at steps with step % renorm_every == 0 (or when the host asks for it).
__device__ __forceinline__ bool renorm_due(const Dev& d)
{
    const int e = d.inst[0].renorm_every;
    return e > 0 && d.run[0].step % e == 0;
}

// mode 0 (set-up): derive from the stored density, q into pos.w.
// mode 1 (after Eq. (7)): derive from the renormalised density when Eq. (7) ran, else
//   only put m P / rho^2 back into pos.w.
// mode 2: only put m P / rho^2 back into pos.w (before rates outside a full step).
// Modes 1 and 2 clear flag 2 (pos.w holds q); the host sets it after mode 0.
template <class R>
__global__ void k_derive(Dev d, int mode, int force)
{
    if (stalled(d)) return;
    const int cur = *d.curp;
    const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k == 0 && mode != 0) d.flags[2] = 0u;
    if (k >= d.n) return;
    const StateSet& S = d.S[cur];
    const bool fresh = mode == 1 && (force || renorm_due(d));
    if (mode != 0 && !fresh) {
        ((R*)S.pos)[4 * (size_t)k + 3] = ((const R*)S.aux)[4 * (size_t)k + 1];
        return;
    }
    const uint32_t info = d.O[cur].info[k];
    const InstDev& I = d.inst[info_inst(info)];
    R4<R> aux = ((R4<R>*)S.aux)[k];
    const R r = fresh ? ((const R*)d.rho_tmp)[k] : aux.w;
    R V, mA;
    derive_values<R>(I, info_phase(info), r, aux.x, V, mA);
    // only pos.w, V (vel.w) and the aux record change: loads and stores of the whole
    // position and velocity records would triple this kernel's traffic
    ((R*)S.pos)[4 * (size_t)k + 3] = mode == 0 ? q_of<R>(I, info_phase(info), r) : mA;
    ((R*)S.vel)[4 * (size_t)k + 3] = V;
    aux.y = mA;
    aux.z = V;
    aux.w = r;
    ((R4<R>*)S.aux)[k] = aux;
    if constexpr (sizeof(R) == 4)
        if (fresh) S.plo[k].w = 0.0f;   // a fresh value: no carried error
}

// -------------------------------------------------------- Eq. (7) renormalise

// Square root and reciprocal: IEEE in FP64; the single-instruction hardware forms
// (about 1 ulp) in the FP32 path, whose error budget is set by the cell-relative
// position encoding.
__device__ __forceinline__ double fsqrt(double x) { return sqrt(x); }
__device__ __forceinline__ float fsqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ double frcp(double x) { return 1.0 / x; }
__device__ __forceinline__ float frcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double fdiv(double a, double b) { return a / b; }
__device__ __forceinline__ float fdiv(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }

// Wendland C2: W = alpha (1 - q/2)^4 (2q + 1); grad_i W_ij = F r_ij with
// F = -5 alpha / h^2 (1 - q/2)^3, q = |r| / h.
template <class R, class IC> __device__ __forceinline__ R kernel_w(const IC& I, R r2)
{
    // 1 - q/2 and 2q + 1 as fused multiply-adds of |r| (wave-uniform factors)
    if constexpr (sizeof(R) == 8) {
        const double s = sqrt(r2), t = fma(s, -0.5 * I.inv_h, 1.0), t2 = t * t;
        return I.wcoef * (t2 * t2) * fma(s, 2.0 * I.inv_h, 1.0);
    } else {
        const float s = fsqrt(r2), t = fmaf(s, -0.5f * I.f_inv_h, 1.0f), t2 = t * t;
        return I.f_wcoef * (t2 * t2) * fmaf(s, 2.0f * I.f_inv_h, 1.0f);
    }
}

// W / alpha_d: Eq. (7) is a ratio of two kernel sums, so the constant factor cancels.
template <class R, class IC> __device__ __forceinline__ R kernel_w_shape(const IC& I, R r2)
{
    if constexpr (sizeof(R) == 8) {
        const double s = sqrt(r2), t = fma(s, -0.5 * I.inv_h, 1.0), t2 = t * t;
        return (t2 * t2) * fma(s, 2.0 * I.inv_h, 1.0);
    } else {
        const float s = fsqrt(r2), t = fmaf(s, -0.5f * I.f_inv_h, 1.0f), t2 = t * t;
        return (t2 * t2) * fmaf(s, 2.0f * I.f_inv_h, 1.0f);
    }
}

// (1 - q/2)^3 = F / (-5 alpha_d / h^2): the force pass sums with it and applies the
// constant factor once per particle.
template <class R, class IC> __device__ __forceinline__ R kernel_t3(const IC& I, R r2)
{
    if constexpr (sizeof(R) == 8) {
        const double t = fma(sqrt(r2), -0.5 * I.inv_h, 1.0);
        return t * t * t;
    } else {
        const float t = fmaf(fsqrt(r2), -0.5f * I.f_inv_h, 1.0f);
        return t * t * t;
    }
}

template <class R, class IC> __device__ __forceinline__ R kernel_f(const IC& I, R r2)
{
    // t = 1 - q/2 as one fused multiply-add of |r| (the factor -1/(2h) is wave-uniform)
    if constexpr (sizeof(R) == 8) {
        const double t = fma(sqrt(r2), -0.5 * I.inv_h, 1.0);
        return I.fcoef * (t * t * t);
    } else {
        const float t = fmaf(fsqrt(r2), -0.5f * I.f_inv_h, 1.0f);
        return I.f_fcoef * (t * t * t);
    }
}

template <class R, int DIM, int P>
__global__ void __launch_bounds__(MaxBlock<R>::value) k_renorm(Dev d, int remap, int force)
{
    if (stalled(d) || (!force && !renorm_due(d))) return;
    uint32_t i, sub;
    lane_split<P>(remap, i, sub);
    if (i >= d.n) return;
    const int cur = *d.curp;
    const Sorted& O = d.O[cur];
    const StateSet& S = d.S[cur];
    const R4<R>* pos = (const R4<R>*)S.pos;
    const R4<R>* vel = (const R4<R>*)S.vel;
    const R4<R>* aux = (const R4<R>*)S.aux;
    const R4<R> pi = pos[i];
    const uint32_t info = O.info[i];
    const uint32_t ph = info_phase(info);
    const bool qpos = d.flags[2] != 0u;   // pos.w holds q = (rho - rho0) / rho
    per_instance(d, info_inst(info), [&](const InstU& I) {
        Lane<R> L;
        L.load(I, pi, O.key[i]);
        // the self term once per particle, on its first lane; every sum below carries W
        // without its constant factor alpha_d, which cancels in the quotient of Eq. (7)
        const R w0 = sub == 0 ? (R)1 : (R)0;
        const double rho0 = ph ? I.rho0[1] : I.rho0[0];
        if (qpos && I.umass) {
            // every j in the sums has i's phase and so i's mass m: Eq. (7) becomes
            // sum W / sum (W / rho_j) = rho0 S / (S - Q) with S = sum W_ij and
            // Q = sum W_ij q_j, since 1 / rho_j = (1 - q_j) / rho0; one record per neighbour
            R sw = w0, sq = w0 * pi.w;
            for_each_neighbor<R, DIM, sizeof(R) == 8 ? 2 : 4, P>(d, I, O, pos, i, L, sub,
                [](uint32_t) { return NoExtra{}; },
                [&](uint32_t, const R*, R r2, const R4<R>& pj, uint32_t phj, NoExtra) {
                    if (phj != ph) return;
                    const R w = kernel_w_shape<R>(I, r2);
                    sw += w;
                    sq += w * pj.w;
                });
            sw = group_sum<P>(sw);
            sq = group_sum<P>(sq);
            if (sub == 0) {
                const double S = sw, Q = sq;
                // FP32 stores rho - rho0 = rho0 Q / (S - Q)
                ((R*)d.rho_tmp)[i] = sizeof(R) == 8 ? (R)(rho0 * S / (S - Q)) : (R)(rho0 * Q / (S - Q));
            }
            return;
        }
        struct Pair { R a, b; };
        R num, den;
        if constexpr (sizeof(R) == 8) {
            // Eq. (7) as written: sum m_j W_ij / sum (m_j / rho_j) W_ij, self included
            num = aux[i].x * w0;
            den = aux[i].z * w0;
            // m_j and V_j (the copy in aux.z) from one record
            for_each_neighbor<R, DIM, 2, P>(d, I, O, pos, i, L, sub,
                [&](uint32_t k) { return Pair{aux[k].x, aux[k].z}; },
                [&](uint32_t, const R*, R r2, const R4<R>&, uint32_t phj, const Pair& x) {
                    if (phj != ph) return;
                    const R w = kernel_w_shape<R>(I, r2);
                    num += x.a * w;
                    den += x.b * w;
                });
        } else {
            // the same quotient minus rho0, as a V_j W_ij-weighted mean of (rho_j - rho0):
            // m_j - rho0 V_j = V_j (rho_j - rho0), so nothing cancels in FP32
            num = aux[i].z * w0 * aux[i].w;
            den = aux[i].z * w0;
            // (V_j, rho_j - rho0) as one 8-byte load of aux.zw
            for_each_neighbor<R, DIM, 4, P>(d, I, O, pos, i, L, sub,
                [&](uint32_t k) {
                    const float2 zw = *(const float2*)&aux[k].z;
                    return Pair{zw.x, zw.y};
                },
                [&](uint32_t, const R*, R r2, const R4<R>&, uint32_t phj, const Pair& x) {
                    if (phj != ph) return;
                    const R vw = x.a * kernel_w_shape<R>(I, r2);
                    num += vw * x.b;
                    den += vw;
                });
        }
        num = group_sum<P>(num);
        den = group_sum<P>(den);
        if (sub == 0) ((R*)d.rho_tmp)[i] = num / den;
    });
}

// ----------------------------------------------- Eq. (16) colour gradient (pass A)

// Lanes per particle of the colour pass.  It runs over the compact list of particles
// with another phase in their neighbour list.  When that list is short (about 1 % of
// the particles in a drop), the pass takes the time of one particle's walk, and a whole
// wave per particle (kColourWide lanes, two entries each) takes a list of up to 128
// entries in one round.  When the list holds more particles than the grid has waves
// (many drops, long slicks) the pass is bound by throughput instead: kColourLanes lanes
// per particle then walk it grid-stride, kColourBatch entries per batch (their product
// divides the list padding).
constexpr int kColourLanes = 8, kColourWide = 64, kColourBatch = 2;

template <class R, class IC>
__device__ __forceinline__ R v_of(const IC& I, uint32_t phase, R m, R stored)
{
    return (R)((double)m / rho_of<R>(I, phase, stored));
}

template <class R> struct MV { R a, b; };

// Where the colour pass takes its state.  A source gives the positions (src.pos[k]),
// what V_k needs, requested with the position (src.load(k)), V_k from that and the
// position record for a neighbour of phase ph (src.vk), and V_i (src.vi).
//
// At a state whose derive pass has run: V from the velocity record (|w|).
template <class R> struct ColourFromVel {
    const R4<R>* pos;
    const R4<R>* vel;
    __device__ MV<R> load(uint32_t k) const { return MV<R>{fabs(vel[k].w), (R)0}; }
    template <class IC> __device__ R vk(const IC&, uint32_t, const MV<R>& x, const R4<R>&) const { return x.a; }
    template <class IC> __device__ R vi(const IC&, uint32_t i, uint32_t) const { return fabs(vel[i].w); }
};

// In the derive pass's own launch: V = m / rho from the density that pass derives from
// (the renormalised one in rho_tmp, or the stored one in aux.w), with its arithmetic.
template <class R> struct ColourFromRho {
    const R4<R>* pos;
    const R* aux;      // records of 4
    const R* dens;     // density of k at dens[k * stride]
    uint32_t stride;
    bool umass;
    __device__ MV<R> load(uint32_t k) const
    {
        return MV<R>{umass ? (R)0 : aux[4 * (size_t)k], dens[(size_t)k * stride]};
    }
    template <class IC> __device__ R vk(const IC& I, uint32_t ph, const MV<R>& x, const R4<R>&) const
    {
        R m;
        if constexpr (sizeof(R) == 8) m = umass ? (ph ? I.mass[1] : I.mass[0]) : x.a;
        else m = umass ? (ph ? I.f_mass[1] : I.f_mass[0]) : x.a;
        return v_of<R>(I, ph, m, x.b);
    }
    template <class IC> __device__ R vi(const IC& I, uint32_t i, uint32_t ph) const
    {
        return v_of<R>(I, ph, aux[4 * (size_t)i], dens[(size_t)i * stride]);
    }
};

// Eq. (16) for colour-list entry g on the P lanes of its group; writes the gradient and
// the interface flag (the sign of V in the velocity record `vel_out`).  make_src(I)
// gives the source for i's instance.
template <class R, int DIM, int P, bool WIDE, class MakeSrc>
__device__ __forceinline__ void colour_one(const Dev& d, int cur, uint32_t g, uint32_t sub, R4<R>* vel_out,
                                           MakeSrc&& make_src)
{
    const Sorted& O = d.O[cur];
    R4<R>* gc = (R4<R>*)d.gc;
    const uint32_t i = d.ilist[g];
    const uint32_t info = O.info[i];
    const uint32_t ph = info_phase(info);
    R s[3] = {0, 0, 0};
    R vi = 0;
    per_instance(d, info_inst(info), [&](const InstU& I) {
        const auto src = make_src(I, info);
        Lane<R> L;
        L.load(I, src.pos[i], O.key[i]);
        vi = src.vi(I, i, ph);
        // C_j^y = 1 only for the other phase: the list walk skips i's own phase
        for_each_neighbor<R, DIM, kColourBatch, P, true, WIDE>(d, I, O, src.pos, i, L, sub,
            [&](uint32_t k) { return src.load(k); },
            [&](uint32_t, const R* r, R r2, const R4<R>& pj, uint32_t phj, const MV<R>& x) {
                if (phj == ph) return;                           // (the stencil fallback)
                const R vk = src.vk(I, phj, x, pj);              // V_k = 1 / sigma_k
                const R f = kernel_f<R>(I, r2) * (vk * vk);
                s[0] += f * r[0];
                s[1] += f * r[1];
                s[2] += f * r[2];
            }, ph);
    });
    R g3[3];                                                     // sigma_i = 1 / V_i
    g3[0] = group_sum<P>(s[0]) / vi;
    g3[1] = group_sum<P>(s[1]) / vi;
    g3[2] = group_sum<P>(s[2]) / vi;
    const R gn = sqrt(g3[0] * g3[0] + g3[1] * g3[1] + g3[2] * g3[2]);
    if (sub == 0) {
        R4<R> out;
        out.x = g3[0]; out.y = g3[1]; out.z = g3[2]; out.w = gn;
        gc[i] = out;
        R* vw = (R*)vel_out + 4 * (size_t)i + 3;
        *vw = gn > 0 ? -vi : vi;          // interface flag: the sign of V in the velocity record
    }
}

// The colour list on nthr threads (this one is thread t): a whole wave per particle
// when the list fits the threads that way, else kColourLanes lanes per particle,
// grid-stride.
template <class R, int DIM, class MakeSrc>
__device__ __forceinline__ void colour_walk(const Dev& d, int cur, uint32_t t, uint32_t nthr, R4<R>* vel_out,
                                            MakeSrc&& make_src)
{
    const uint32_t count = *d.icount;
    if ((uint64_t)count * kColourWide <= nthr) {
        const uint32_t g = t / kColourWide;
        if (g < count) colour_one<R, DIM, kColourWide, true>(d, cur, g, t % kColourWide, vel_out, make_src);
    } else {
        constexpr int P = kColourLanes;
        for (uint32_t g = t / P; g < count; g += nthr / P)
            colour_one<R, DIM, P, false>(d, cur, g, t % P, vel_out, make_src);
    }
}

template <class R, int DIM>
__global__ void __launch_bounds__(MaxBlock<R>::value) k_colour(Dev d, int star)
{
    if (stalled(d)) return;
    const int cur = *d.curp;
    const StateSet& S = star ? d.star : d.S[cur];
    colour_walk<R, DIM>(d, cur, blockIdx.x * blockDim.x + threadIdx.x, gridDim.x * blockDim.x, (R4<R>*)S.vel,
                        [&](const InstU&, uint32_t) {
                            return ColourFromVel<R>{(const R4<R>*)S.pos, (const R4<R>*)S.vel};
                        });
}

// The derive pass after Eq. (7) and the colour pass at S^n in one launch: the first
// cblocks blocks walk the colour list (their V values come from the density the derive
// pass reads, so they need none of its writes), the rest derive.  Only the colour
// blocks write V, with its sign, for the particles of the colour list.
template <class R, int DIM>
__global__ void __launch_bounds__(256) k_derive_colour(Dev d, int force, uint32_t cblocks)
{
    if (stalled(d)) return;
    const int cur = *d.curp;
    const bool fresh = force || renorm_due(d);
    if (blockIdx.x < cblocks) {
        const StateSet& S = d.S[cur];
        const R* aux = (const R*)S.aux;
        // the density derived from: renormalised (rho_tmp) or stored (aux.w)
        const R* dens = fresh ? (const R*)d.rho_tmp : aux + 3;
        const uint32_t dstride = fresh ? 1u : 4u;
        colour_walk<R, DIM>(d, cur, blockIdx.x * blockDim.x + threadIdx.x, cblocks * blockDim.x, (R4<R>*)S.vel,
                            [&](const InstU& I, uint32_t) {
                                return ColourFromRho<R>{(const R4<R>*)S.pos, aux, dens, dstride, I.umass != 0};
                            });
        return;
    }
    const uint32_t k = (blockIdx.x - cblocks) * blockDim.x + threadIdx.x;
    if (k == 0) d.flags[2] = 0u;
    if (k >= d.n) return;
    const StateSet& S = d.S[cur];
    if (!fresh) {
        ((R*)S.pos)[4 * (size_t)k + 3] = ((const R*)S.aux)[4 * (size_t)k + 1];
        return;
    }
    const uint32_t info = d.O[cur].info[k];
    const InstDev& I = d.inst[info_inst(info)];
    R4<R> aux = ((R4<R>*)S.aux)[k];
    const R r = ((const R*)d.rho_tmp)[k];
    R V, mA;
    derive_values<R>(I, info_phase(info), r, aux.x, V, mA);
    ((R*)S.pos)[4 * (size_t)k + 3] = mA;
    if (!(info & kInfoColour)) ((R*)S.vel)[4 * (size_t)k + 3] = V;
    aux.y = mA;
    aux.z = V;
    aux.w = r;
    ((R4<R>*)S.aux)[k] = aux;
    if constexpr (sizeof(R) == 4) S.plo[k].w = 0.0f;
}

// ------------------------------------------ Eqs. (6), (8), (10)/(11), (17) (pass B)

// (T V^2) . w for T = alpha (|g|^2 I / d - g g^T) / |g|, with c = alpha V^2 / |g|.
template <class R, int DIM>
__device__ __forceinline__ void tension_dot(R c, const R g[3], R gn2, const R w[3], R out[3])
{
    const R gw = g[0] * w[0] + g[1] * w[1] + g[2] * w[2];
    const R iso = gn2 * (R)(1.0 / DIM);
    for (int a = 0; a < 3; ++a) out[a] = c * (iso * w[a] - g[a] * gw);
}

// List entries per batch in the force pass: more loads in flight per wave against
// more registers (fewer waves per SIMD).  U * lanes must divide the list capacity.
#ifndef SPHX_FORCE_BATCH
#define SPHX_FORCE_BATCH 4
#endif
#ifndef SPHX_FORCE_BATCH64
#define SPHX_FORCE_BATCH64 4
#endif
template <class R, int P> struct ForceBatch {
    static constexpr int B = sizeof(R) == 8 ? SPHX_FORCE_BATCH64 : SPHX_FORCE_BATCH;
    static constexpr int U = B * P <= 16 ? B : 16 / P;
};

// Per-lane state of the force pass for particle i: its own quantities, the sums of
// Eqs. (6), (8), (10)/(11), (17) over its neighbours, and the epilogue that turns them
// into the rates.
// SPLIT keeps the three acceleration terms apart (for the debug output of each); without
// it they go into one sum, acc, each term pre-scaled so that fc * acc is the acceleration
// (three registers per lane instead of nine).
template <class R, int DIM, bool SPLIT = true> struct ForceLane {
    uint32_t info, ph;
    bool fluid, fli, massform;
    R4<R> vi;
    R mi, Ai, alpha, ci, gi2, vp0, vp1, delta2;
    R mA0, mA1;   // m_j A_i for a neighbour of phase 0 / 1 (masses uniform per phase)
    R sfac;       // !SPLIT: 1 / (m_i fc), the scale of the surface-tension terms in acc
    R gi[3];
    R cont, ap[3], av[3], as[3], acc[3];
    uint32_t cnt;

    template <class IC>
    __device__ __forceinline__ void init(const IC& I, uint32_t info_, const R4<R>& vi_, const R4<R>& xi,
                                         const R4<R>* __restrict__ gc, uint32_t i)
    {
        // vi_ = (u_i, +-V_i), the sign of V being the interface flag; xi = (m_i, m_i A_i)
        info = info_;
        ph = info_phase(info);
        fluid = info_kind(info) == K_FLUID;
        vi = vi_;
        mi = xi.x;
        Ai = xi.y / mi;                          // P_i / rho_i^2
        fli = vi_.w < (R)0;                      // interface flag
        alpha = sizeof(R) == 8 ? (R)I.alpha_s : (R)I.f_alpha_s;
        gi[0] = gi[1] = gi[2] = 0;
        ci = 0;
        gi2 = 0;
        if (fli) {
            const R4<R> g4 = gc[i];
            gi[0] = g4.x; gi[1] = g4.y; gi[2] = g4.z;
            gi2 = g4.w * g4.w;
            ci = alpha * (vi.w * vi.w) / g4.w;
        }
        // selects, not a dynamic index, keep the table in scalar registers
        if constexpr (sizeof(R) == 8) {
            vp0 = ph ? I.vpair[1][0] : I.vpair[0][0];
            vp1 = ph ? I.vpair[1][1] : I.vpair[0][1];
            delta2 = I.delta2;
        } else {
            vp0 = ph ? I.f_vpair[1][0] : I.f_vpair[0][0];
            vp1 = ph ? I.f_vpair[1][1] : I.f_vpair[0][1];
            delta2 = I.f_delta2;
        }
        massform = I.cont_form == 1;
        if constexpr (sizeof(R) == 8) { mA0 = I.mass[0] * Ai; mA1 = I.mass[1] * Ai; }
        else { mA0 = I.f_mass[0] * Ai; mA1 = I.f_mass[1] * Ai; }
        if constexpr (!SPLIT) {
            // Eq. (11) carries 1 / rho_i (the vfac of finish); the tension terms carry
            // 1 / m_i and, against the fc applied to acc, 1 / fc
            const R fc = sizeof(R) == 8 ? (R)I.fcoef : (R)I.f_fcoef;
            if (I.visc_form == 1) {
                const R vfac = (R)(1.0 / rho_of<R>(I, ph, xi.w));
                vp0 *= vfac;
                vp1 *= vfac;
            }
            sfac = (R)1 / (mi * fc);
        }
        cont = 0;
        for (int q = 0; q < 3; ++q) ap[q] = av[q] = as[q] = acc[q] = 0;
        cnt = 0;
    }

    // One neighbour j = k with r_ij, |r_ij|^2 < 4h^2, position record pj = (x_j, m_j A_j),
    // phase phj, velocity record vk = (u_j, +-V_j), the sign of V_j being j's interface
    // flag, mass mj, and m_j A_i.  MF: the mass form of the continuity equation (Eq. (5)).
    // grad_i W_ij = F r_ij enters through F times scalars of r_ij (u_ij . r_ij, the
    // pressure factor), so the gradient vector itself is formed only for surface tension.
    // cont, ap and av are summed without the kernel's constant factor -5 alpha_d / h^2,
    // which finish() applies once.
    template <bool MF, class IC>
    __device__ __forceinline__ void pair(const IC& I, const R4<R>* __restrict__ gc, uint32_t k, const R* r,
                                         R r2, const R4<R>& pj, uint32_t phj, const R4<R>& vk, R mj, R mjAi)
    {
        ++cnt;
        const R T = kernel_t3<R>(I, r2);                          // F / (-5 alpha_d / h^2)
        const R u[3] = {vi.x - vk.x, vi.y - vk.y, vi.z - vk.z}; // u_ij
        const R ur = u[0] * r[0] + u[1] * r[1] + u[2] * r[2];
        const R Vj = fabs(vk.w);
        cont += (MF ? mj : Vj) * (T * ur);                         // Eq. (6) / (5)
        if (!fluid) return;
        const R pcT = (mjAi + pj.w) * T;                          // m_j (A_i + A_j) T
        const R lap = (T * r2) * frcp(r2 + delta2);               // r.gradW / (r^2 + delta^2), unscaled
        const R cv = Vj * (phj ? vp1 : vp0) * lap;
        if constexpr (SPLIT) {
            ap[0] -= pcT * r[0]; ap[1] -= pcT * r[1]; ap[2] -= pcT * r[2];
            av[0] += cv * u[0]; av[1] += cv * u[1]; av[2] += cv * u[2];
        } else {
            for (int q = 0; q < 3; ++q) acc[q] += cv * u[q] - pcT * r[q];
        }
        const bool flk = vk.w < (R)0;
        if (fli || flk) {
            const R F = (sizeof(R) == 8 ? (R)I.fcoef : (R)I.f_fcoef) * T;
            const R w[3] = {F * r[0], F * r[1], F * r[2]};       // grad_i W_ij
            R t[3];
            if (fli) {
                tension_dot<R, DIM>(ci, gi, gi2, w, t);
                if constexpr (SPLIT) { as[0] += t[0]; as[1] += t[1]; as[2] += t[2]; }
                else { acc[0] += sfac * t[0]; acc[1] += sfac * t[1]; acc[2] += sfac * t[2]; }
            }
            if (flk) {
                const R4<R> g4 = gc[k];
                const R gk[3] = {g4.x, g4.y, g4.z};
                const R ck = fdiv(alpha * (vk.w * vk.w), g4.w);
                tension_dot<R, DIM>(ck, gk, g4.w * g4.w, w, t);
                if constexpr (SPLIT) { as[0] += t[0]; as[1] += t[1]; as[2] += t[2]; }
                else { acc[0] += sfac * t[0]; acc[1] += sfac * t[1]; acc[2] += sfac * t[2]; }
            }
        }
    }

    // Combine the P lanes of the particle, then (on its first lane) store the rates
    // (and the three terms when asked) and return |u_i|^2, |a_i|^2 for the time step.
    template <int P, bool REDUCE, bool TERMS, class IC>
    __device__ __forceinline__ void finish(const Dev& d, const IC& I, uint32_t i, uint32_t sub, R rho_stored,
                                           double& umag2, double& amag2)
    {
        const R fc = sizeof(R) == 8 ? (R)I.fcoef : (R)I.f_fcoef;
        cont = fc * group_sum<P>(cont);
        for (int q = 0; q < 3; ++q) {
            if constexpr (SPLIT) {
                ap[q] = fc * group_sum<P>(ap[q]);
                av[q] = fc * group_sum<P>(av[q]);
                as[q] = group_sum<P>(as[q]);
            } else {
                acc[q] = fc * group_sum<P>(acc[q]);
            }
        }
        const double rho_i = rho_of<R>(I, ph, rho_stored);
        R4<R> out;
        out.w = massform ? cont : (R)rho_i * cont;
        R a[3] = {0, 0, 0};
        if (fluid) {
            const R vfac = I.visc_form == 1 ? (R)(1.0 / rho_i) : (R)1;
            for (int q = 0; q < 3; ++q) {
                const R gq = sizeof(R) == 8 ? (R)I.g[q] : (R)I.f_g[q];
                if constexpr (SPLIT) {
                    av[q] *= vfac;
                    as[q] /= mi;
                    a[q] = ap[q] + av[q] + as[q] + gq;
                } else {
                    a[q] = acc[q] + gq;
                }
            }
        }
        out.x = a[0]; out.y = a[1]; out.z = a[2];
        if (sub == 0) ((R4<R>*)d.acc)[i] = out;
        if (TERMS && sub == 0) {
            R4<R>* T = (R4<R>*)d.terms;
            R4<R> t;
            t.w = 0;
            t.x = fluid ? ap[0] : 0; t.y = fluid ? ap[1] : 0; t.z = fluid ? ap[2] : 0;
            T[3 * (size_t)i + 0] = t;
            t.x = av[0]; t.y = av[1]; t.z = av[2];
            T[3 * (size_t)i + 1] = t;
            t.x = as[0]; t.y = as[1]; t.z = as[2];
            T[3 * (size_t)i + 2] = t;
        }
        if (!isfinite((double)out.x) || !isfinite((double)out.y) || !isfinite((double)out.z) ||
            !isfinite((double)out.w))
            atomicOr(d.status, ST_NONFINITE);
        if (REDUCE && sub == 0) {
            if (info_kind(info) != K_WALL) {
                const double ux = vi.x, uy = vi.y, uz = vi.z;
                umag2 = ux * ux + uy * uy + uz * uz;
            }
            if (fluid) amag2 = (double)a[0] * a[0] + (double)a[1] * a[1] + (double)a[2] * a[2];
        }
    }
};

// Per-instance running maxima (bit patterns of non-negative doubles) from one block:
// each wave's maximum, then, when every wave that contributes lies in the same instance,
// one update per block. Each update is a device-coherent read and at most one atomic,
// so fewer of them shorten the end of every wave (force pass at S^n on the 3D drop:
// 85 -> 78 us). Every thread of the block calls this once per launch.
template <int K>
__device__ __forceinline__ void block_max(const Dev& d, bool mine, uint32_t b, const double (&v)[K],
                                          unsigned long long InstRun::*const (&field)[K])
{
    __shared__ double s_m[K][4];
    __shared__ uint32_t s_b[4];
    __shared__ int s_f[4];
    const uint32_t wv = threadIdx.x >> 6, nw = blockDim.x >> 6, lane = threadIdx.x & 63;
    const uint32_t b0 = __shfl(b, 0, 64);
    const bool uniform = __all(!mine || b == b0);
    const bool any = __any(mine);
    double wm[K];
#pragma unroll
    for (int k = 0; k < K; ++k) wm[k] = wave_max(v[k]);
    if (lane == 0) {
#pragma unroll
        for (int k = 0; k < K; ++k) s_m[k][wv] = wm[k];
        s_b[wv] = b0;
        s_f[wv] = (uniform ? 1 : 0) | (any ? 2 : 0);
    }
    __syncthreads();
    bool one = true, have = false;
    uint32_t bb = 0;
    for (uint32_t q = 0; q < nw; ++q) {
        if (!(s_f[q] & 1)) one = false;
        if (s_f[q] & 2) {
            if (have && s_b[q] != bb) one = false;
            bb = s_b[q];
            have = true;
        }
    }
    if (one) {
        if (threadIdx.x == 0 && have) {
#pragma unroll
            for (int k = 0; k < K; ++k) {
                double m = 0.0;
                for (uint32_t q = 0; q < nw; ++q)
                    if (s_f[q] & 2) m = fmax(m, s_m[k][q]);
                max_update(&(d.run[bb].*field[k]), m);
            }
        }
    } else if (uniform) {
        if (lane == 0 && any) {
#pragma unroll
            for (int k = 0; k < K; ++k) max_update(&(d.run[b0].*field[k]), wm[k]);
        }
    } else if (mine) {
#pragma unroll
        for (int k = 0; k < K; ++k) max_update(&(d.run[b].*field[k]), v[k]);
    }
}

// Reductions at the end of a force pass: the interaction count (per wave) always, the
// |u|^2 and |a|^2 maxima for the time step (per block) when REDUCE.
template <bool REDUCE>
__device__ __forceinline__ void force_reduce(const Dev& d, bool valid, uint32_t inst, unsigned long long nint,
                                             double umag2, double amag2)
{
    const unsigned long long wsum = wave_sum(nint);
    // one add per wave, spread over the counters: a single counter serialised every wave
    // of the launch on one address (the 256 batched tanks ran 40 % slower for it)
    const uint32_t w = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if ((threadIdx.x & 63) == 0 && wsum) atomicAdd(d.inter + (size_t)(w % kInterSlots) * kInterStride, wsum);
    if (REDUCE) {
        const double v[2] = {umag2, amag2};
        static constexpr unsigned long long InstRun::*f[2] = {&InstRun::umax2, &InstRun::amax2};
        block_max<2>(d, valid, inst, v, f);
    }
}

template <class R, int DIM>
__device__ double correct_one(const Dev& d, int cur, uint32_t k, uint32_t& inst);
__device__ void finish_steps(const Dev& d);

// Per instance: the largest reach of the new state (for the next rebuild decision).
__device__ __forceinline__ void reach_reduce(const Dev& d, bool mine, uint32_t b, double reach2)
{
    const double v[1] = {reach2};
    static constexpr unsigned long long InstRun::*f[1] = {&InstRun::reach2};
    block_max<1>(d, mine, b, v, f);
}

// With CORRECT (the pass at S*), each particle's corrector follows its rates in the same
// launch: it reads and writes only that particle's records of S^n and reads its own
// S* velocity and rates, while the force pass at S* reads S* records only.
template <class R, int DIM, int P, bool REDUCE, bool TERMS, bool CORRECT>
__global__ void __launch_bounds__(MaxBlock<R>::value) k_force(Dev d, int star, int remap)
{
    if (stalled(d)) return;
    const int cur = *d.curp;
    uint32_t i, sub;
    lane_split<P>(remap, i, sub);
    const bool valid = i < d.n;
    const Sorted& O = d.O[cur];
    const StateSet& S = star ? d.star : d.S[cur];
    const R4<R>* pos = (const R4<R>*)S.pos;
    const R4<R>* vel = (const R4<R>*)S.vel;
    const R4<R>* aux = (const R4<R>*)S.aux;
    const R4<R>* gc = (const R4<R>*)d.gc;
    double umag2 = 0.0, amag2 = 0.0;
    unsigned long long nint = 0;
    uint32_t inst = 0;
    if (valid) {
        const uint32_t info = O.info[i];
        inst = info_inst(info);
        per_instance(d, inst, [&](const InstU& I) {
            const R4<R> pi = pos[i];
            Lane<R> L;
            L.load(I, pi, O.key[i]);
            ForceLane<R, DIM, TERMS> F;
            F.init(I, info, vel[i], aux[i], gc, i);
            // per neighbour: the position record (x_j, m_j A_j) and the velocity record
            // (u_j, +-V_j); m_j from the per-phase table when the instance's masses are
            // uniform per phase, else from the aux record
            R m0, m1;
            if constexpr (sizeof(R) == 8) { m0 = I.mass[0]; m1 = I.mass[1]; }
            else { m0 = I.f_mass[0]; m1 = I.f_mass[1]; }
            struct VM { R4<R> v; R m; };
            // one loop per case (masses uniform per phase or not; Eq. (6) or Eq. (5)), so
            // that the walk carries no per-neighbour branch on them
            auto walk = [&](auto uniform, auto massform) {
                constexpr bool UM = decltype(uniform)::value, MF = decltype(massform)::value;
                for_each_neighbor<R, DIM, ForceBatch<R, P>::U, P>(d, I, O, pos, i, L, sub,
                    [&](uint32_t k) {
                        VM x;
                        x.v = vel[k];
                        if constexpr (UM) x.m = (R)0;
                        else x.m = aux[k].x;
                        return x;
                    },
                    [&](uint32_t k, const R* r, R r2, const R4<R>& pj, uint32_t phj, const VM& x) {
                        if constexpr (UM)
                            F.template pair<MF>(I, gc, k, r, r2, pj, phj, x.v, MF ? (phj ? m1 : m0) : (R)0,
                                                phj ? F.mA1 : F.mA0);
                        else
                            F.template pair<MF>(I, gc, k, r, r2, pj, phj, x.v, x.m, x.m * F.Ai);
                    });
            };
            if (I.umass) {
                if (I.cont_form == 1) walk(std::true_type{}, std::true_type{});
                else walk(std::true_type{}, std::false_type{});
            } else {
                if (I.cont_form == 1) walk(std::false_type{}, std::true_type{});
                else walk(std::false_type{}, std::false_type{});
            }
            nint = F.cnt;
            F.template finish<P, REDUCE, TERMS>(d, I, i, sub, aux[i].w, umag2, amag2);
        });
    }
    force_reduce<REDUCE>(d, valid, inst, nint, umag2, amag2);
    if constexpr (CORRECT) {
        finish_steps(d);
        const bool mine = valid && sub == 0;
        double reach2 = 0.0;
        uint32_t b = 0;
        if (mine) reach2 = correct_one<R, DIM>(d, cur, i, b);
        reach_reduce(d, mine, b, reach2);
    }
}

// ----------------------------------------------------------- time step (a9)

// The time step of instance b from the maxima of the last rate evaluation at S^n (or
// the override / fixed value).  Every thread that asks gets the same value: the same
// arithmetic on the same inputs.
__device__ __forceinline__ double step_dt(const Dev& d, uint32_t b, double dt_override, double& umax)
{
    const InstDev& I = d.inst[b];
    const InstRun& R = d.run[b];
    umax = sqrt(__longlong_as_double((long long)R.umax2));
    const double amax = sqrt(__longlong_as_double((long long)R.amax2));
    double dt;
    if (dt_override > 0.0) dt = dt_override;
    else if (I.dt_fixed > 0.0) dt = I.dt_fixed;
    else {
        dt = I.c_cfl * I.h / (I.cmax + umax);
        if (amax > 0.0) dt = fmin(dt, I.c_force * sqrt(I.h / amax));
        dt = fmin(dt, I.dt_const);
    }
    return dt;
}

// Store each instance's step (run by the predictor's threads t0 of nthr, stride over
// instances).
__device__ __forceinline__ void store_steps(const Dev& d, double dt_override, uint32_t t0, uint32_t nthr)
{
    for (uint32_t b = t0; b < (uint32_t)d.ninst; b += nthr) {
        double umax;
        const double dt = step_dt(d, b, dt_override, umax);
        // the corrector reuses the list of S^n: every pair within 2h at the predicted
        // positions must still be in it, which holds while no particle gets more than
        // half the skin from its build position.  A particle's displacement plus
        // dt_bound / 2 times its speed is at most the largest reach e (none since a
        // build), and every speed is at most umax, so the half step keeps each particle
        // within max(e + (dt - dt_bound) umax / 2, dt umax / 2) of its build position;
        // a step beyond skin / 2 is refused: an override longer than dt_bound, or, right
        // after a build, dt umax / 2 beyond skin / 2 (the adaptive step allows that only
        // above max|u| = c0 skin / (c_cfl - skin), 2 c0 / 3 at the defaults, far outside
        // the weakly compressible regime).
        const InstDev& I = d.inst[b];
        const double e = sqrt(__longlong_as_double((long long)d.run[b].reach2));
        const double far = fmax(e + 0.5 * fmax(dt - I.dt_bound, 0.0) * umax, 0.5 * dt * umax);
        if (far > 0.5 * I.skin * (1.0 + 1e-12) || !(dt > 0.0)) atomicOr(d.status, ST_DT);
        d.run[b].dt = dt;
        d.run[b].t_next = d.run[b].t + dt;
    }
}

// End of a step (grid-stride over instances; run by the corrector, whose particle
// updates read dt and t_next only).
__device__ void finish_steps(const Dev& d)
{
    const uint32_t t0 = blockIdx.x * blockDim.x + threadIdx.x, stride = gridDim.x * blockDim.x;
    if (t0 == 0) d.flags[2] = 1u;   // the corrector leaves q in pos.w
    for (uint32_t b = t0; b < (uint32_t)d.ninst; b += stride) {
        d.run[b].t = d.run[b].t_next;
        d.run[b].step += 1;
        d.run[b].umax2 = 0ull;   // the predictor has taken this step's dt from them
        d.run[b].amax2 = 0ull;
    }
}

// -------------------------------------------------------- integrator (a10)

// Moving particle position at time t, written into a record of the set (FP64 absolute;
// FP32 as the offset inside the particle's current cell).
template <class R>
__device__ __forceinline__ void moving_state(const InstDev& I, const double4& x0, uint32_t key, double t,
                                             R4<R>& p, R4<R>& v)
{
    double dd[3], vv[3];
    moving_motion(I, t, dd, vv);
    const double x[3] = {x0.x + dd[0], x0.y + dd[1], x0.z + dd[2]};
    if constexpr (sizeof(R) == 8) {
        p.x = x[0]; p.y = x[1]; p.z = x[2];
    } else {
        int c[3];
        cell_of_key(I, key, c);
        p.x = (float)((x[0] - I.lo[0]) - (double)c[0] * I.cs[0]);
        p.y = (float)((x[1] - I.lo[1]) - (double)c[1] * I.cs[1]);
        p.z = (float)((x[2] - I.lo[2]) - (double)c[2] * I.cs[2]);
    }
    v.x = (R)vv[0]; v.y = (R)vv[1]; v.z = (R)vv[2];
}

__device__ __forceinline__ double wrap_coord(double x, const InstDev& I, int d)
{
    if (I.periodic[d]) {
        if (x >= I.hi[d]) x -= I.span[d];
        else if (x < I.lo[d]) x += I.span[d];
    }
    return x;
}

// Kahan-compensated s += y with the running compensation e.
__device__ __forceinline__ void kahan_add(float& s, float& e, float y)
{
    const float yy = y + e;
    const float t = s + yy;
    e = yy - (t - s);
    s = t;
}

// The predictor's position update of particle k (kind from its info word): fluid
// particles move by hdt u, moving ones follow the piston, walls stay.
template <class R, int DIM>
__device__ __forceinline__ void advance_pos(const Dev& d, int cur, uint32_t k, uint32_t kind, const InstDev& I,
                                            uint32_t b, double hdt, R4<R>& p, R4<R>& v)
{
    if (kind == K_FLUID) {
        if constexpr (sizeof(R) == 8) {
            p.x = wrap_coord(fma(hdt, v.x, p.x), I, 0);
            p.y = wrap_coord(fma(hdt, v.y, p.y), I, 1);
            p.z = DIM == 3 ? wrap_coord(fma(hdt, v.z, p.z), I, 2) : p.z;
        } else {
            const R h = (R)hdt;
            p.x = fmaf(h, v.x, p.x); p.y = fmaf(h, v.y, p.y); p.z = fmaf(h, v.z, p.z);
        }
    } else if (kind == K_MOVING) {
        moving_state<R>(I, d.O[cur].ref[k], d.O[cur].key[k], d.run[b].t + hdt, p, v);
    }
}

// Density (stored form) at S*: rho^n + (dt/2) D rho^n.
template <class R>
__device__ __forceinline__ R pred_rho(R stored, double hdt, R rate)
{
    return fma((R)hdt, rate, stored);
}

// S* for particle k (no writes).
template <class R, int DIM>
__device__ __forceinline__ void predict_state(const Dev& d, int cur, uint32_t k, uint32_t info, const InstDev& I,
                                              double hdt, R4<R>& p, R4<R>& v, R4<R>& x)
{
    const StateSet& S = d.S[cur];
    const uint32_t b = info_inst(info);
    p = ((const R4<R>*)S.pos)[k];
    v = ((const R4<R>*)S.vel)[k];
    x = ((const R4<R>*)S.aux)[k];
    const R4<R> a = ((const R4<R>*)d.acc)[k];
    const uint32_t kind = info_kind(info);
    advance_pos<R, DIM>(d, cur, k, kind, I, b, hdt, p, v);
    if (kind == K_FLUID) {
        const R h = (R)hdt;
        v.x += h * a.x; v.y += h * a.y; v.z += h * a.z;
    }
    derive_one<R>(I, info_phase(info), pred_rho<R>(x.w, hdt, a.w), p, v, x, false);
}

// The predicted state S* of any particle, computed from S^n and its rates with the
// predictor's own arithmetic: pos[k] is its position record with V* in w (the sentinel
// index n gives the far-away record of S^n).  Neighbours share i's instance, so they
// share its half step hdt.
template <class R, int DIM> struct PredictedPos {
    const Dev* d;
    int cur;
    double hdt;
    __device__ R4<R> operator[](uint32_t k) const
    {
        if (k >= d->n) return ((const R4<R>*)d->S[cur].pos)[k];
        const uint32_t info = d->O[cur].info[k];
        R4<R> p, v, x;
        predict_state<R, DIM>(*d, cur, k, info, d->inst[info_inst(info)], hdt, p, v, x);
        p.w = v.w;
        return p;
    }
};

// Colour source at S* computed in the predictor's launch (V* from the predicted record).
template <class R, int DIM> struct ColourPredicted {
    PredictedPos<R, DIM> pos;
    __device__ MV<R> load(uint32_t) const { return MV<R>{(R)0, (R)0}; }
    template <class IC> __device__ R vk(const IC&, uint32_t, const MV<R>&, const R4<R>& pj) const { return pj.w; }
    template <class IC> __device__ R vi(const IC&, uint32_t i, uint32_t) const { return pos[i].w; }
};

// S* = S^n + dt/2 R(S^n), and in the same launch Eq. (16) at S*: the first cblocks
// blocks walk the colour list, computing the predicted state of i and of its
// other-phase neighbours themselves, so they need none of the predictor's writes.  The
// colour blocks write V* with its sign for the particles of the colour list; the
// predictor blocks write the rest of their velocity records and everything of the
// other particles.  Without colour blocks (cblocks = 0) the predictor writes every
// record whole, and the colour pass at S* follows in a launch of its own.
template <class R, int DIM>
__global__ void __launch_bounds__(256) k_predict(Dev d, double dt_override, uint32_t cblocks)
{
    if (stalled(d)) return;
    const int cur = *d.curp;
    if (blockIdx.x < cblocks) {
        colour_walk<R, DIM>(d, cur, blockIdx.x * blockDim.x + threadIdx.x, cblocks * blockDim.x, (R4<R>*)d.star.vel,
                            [&](const InstU&, uint32_t info) {
                                double umax;
                                const double hdt = 0.5 * step_dt(d, info_inst(info), dt_override, umax);
                                return ColourPredicted<R, DIM>{PredictedPos<R, DIM>{&d, cur, hdt}};
                            });
        return;
    }
    const uint32_t k = (blockIdx.x - cblocks) * blockDim.x + threadIdx.x;
    store_steps(d, dt_override, k, (gridDim.x - cblocks) * blockDim.x);
    if (k >= d.n) return;
    const uint32_t info = d.O[cur].info[k];
    const uint32_t b = info_inst(info);
    double umax;
    const double hdt = 0.5 * step_dt(d, b, dt_override, umax);
    R4<R> p, v, x;
    predict_state<R, DIM>(d, cur, k, info, d.inst[b], hdt, p, v, x);
    ((R4<R>*)d.star.pos)[k] = p;
    if (cblocks > 0 && (info & kInfoColour)) {
        R* vr = (R*)d.star.vel + 4 * (size_t)k;
        vr[0] = v.x;
        vr[1] = v.y;
        vr[2] = v.z;
    } else {
        ((R4<R>*)d.star.vel)[k] = v;
    }
    ((R4<R>*)d.star.aux)[k] = x;
}

// S^{n+1} = S^n + dt R(S*), in place
// Corrector for one particle; returns |x - x_build|^2 and its instance.
template <class R, int DIM>
__device__ double correct_one(const Dev& d, int cur, uint32_t k, uint32_t& inst)
{
    const Sorted& O = d.O[cur];
    const StateSet& S = d.S[cur];
    const uint32_t info = O.info[k];
    const uint32_t b = info_inst(info);
    inst = b;
    const InstDev& I = d.inst[b];
    const double dt = d.run[b].dt;
    const uint32_t kind = info_kind(info);
    R4<R> p = ((const R4<R>*)S.pos)[k];
    R4<R> v = ((const R4<R>*)S.vel)[k];
    R4<R> x = ((const R4<R>*)S.aux)[k];
    const R4<R> us = ((const R4<R>*)d.star.vel)[k];
    const R4<R> a = ((const R4<R>*)d.acc)[k];
    R r = x.w;
    bool bad = false;
    if constexpr (sizeof(R) == 8) {
        if (kind == K_FLUID) {
            p.x = wrap_coord(p.x + dt * us.x, I, 0);
            p.y = wrap_coord(p.y + dt * us.y, I, 1);
            p.z = DIM == 3 ? wrap_coord(p.z + dt * us.z, I, 2) : p.z;
            v.x += dt * a.x; v.y += dt * a.y; v.z += dt * a.z;
        } else if (kind == K_MOVING) {
            moving_state<R>(I, O.ref[k], O.key[k], d.run[b].t_next, p, v);
        }
        r += dt * a.w;
    } else {
        const float fdt = (float)dt;
        float4 pl = S.plo[k], vl = S.vlo[k];
        if (kind == K_FLUID) {
            kahan_add(p.x, pl.x, fdt * us.x);
            kahan_add(p.y, pl.y, fdt * us.y);
            if (DIM == 3) kahan_add(p.z, pl.z, fdt * us.z);
            kahan_add(v.x, vl.x, fdt * a.x);
            kahan_add(v.y, vl.y, fdt * a.y);
            if (DIM == 3) kahan_add(v.z, vl.z, fdt * a.z);
        } else if (kind == K_MOVING) {
            moving_state<R>(I, O.ref[k], O.key[k], d.run[b].t_next, p, v);
            pl.x = pl.y = pl.z = 0.0f;
        }
        kahan_add(r, pl.w, fdt * a.w);
        S.plo[k] = pl;
        S.vlo[k] = vl;
    }
    bad = !isfinite((double)p.x) || !isfinite((double)p.y) || !isfinite((double)p.z) ||
          !isfinite((double)v.x) || !isfinite((double)v.y) || !isfinite((double)v.z) || !isfinite((double)r);
    if (bad) atomicOr(d.status, ST_NONFINITE);
    derive_one<R>(I, info_phase(info), r, p, v, x, true);
    ((R4<R>*)S.pos)[k] = p;
    ((R4<R>*)S.vel)[k] = v;
    ((R4<R>*)S.aux)[k] = x;
    // the reach: displacement since the build plus the longest half step the next
    // predictor can give this particle
    const double speed2 = kind == K_WALL ? 0.0 : (double)v.x * v.x + (double)v.y * v.y + (DIM == 3 ? (double)v.z * v.z : 0.0);
    const R4<R> xb = ((const R4<R>*)d.xb)[k];
    const double ex = (double)p.x - (double)xb.x, ey = (double)p.y - (double)xb.y;
    const double ez = DIM == 3 ? (double)p.z - (double)xb.z : 0.0;
    const double e = sqrt(ex * ex + ey * ey + ez * ez) + 0.5 * I.dt_bound * sqrt(speed2);
    return e * e;
}


// A motion set from outside (sphx_set_moving): the MOVING particles of instance `inst`
// take its state at the instance's current time at once (FP32: as offsets in their
// current cells with the compensation cleared, as the corrector places them).
template <class R>
__global__ void k_place_moving(Dev d, uint32_t inst)
{
    const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < d.n) {
        const int cur = *d.curp;
        const Sorted& O = d.O[cur];
        const uint32_t info = O.info[k];
        if (info_inst(info) == inst && info_kind(info) == K_MOVING) {
            const InstDev& I = d.inst[inst];
            const StateSet& S = d.S[cur];
            R4<R> p = ((const R4<R>*)S.pos)[k];
            R4<R> v = ((const R4<R>*)S.vel)[k];
            moving_state<R>(I, O.ref[k], O.key[k], d.run[inst].t, p, v);
            ((R4<R>*)S.pos)[k] = p;
            ((R4<R>*)S.vel)[k] = v;
            if constexpr (sizeof(R) == 4) {
                float4 pl = S.plo[k];
                pl.x = pl.y = pl.z = 0.0f;
                S.plo[k] = pl;
            }
        }
    }
}

// ------------------------------------------------------- neighbour export

template <class R, int DIM>
__global__ void k_export(Dev d, int pass, const uint32_t* __restrict__ off, uint32_t* __restrict__ out)
{
    const int cur = *d.curp;
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= d.n) return;
    const Sorted& O = d.O[cur];
    const R4<R>* pos = (const R4<R>*)d.S[cur].pos;
    const R4<R> pi = pos[i];
    const InstDev& I = d.inst[info_inst(O.info[i])];
    Lane<R> L;
    L.load(I, pi, O.key[i]);
    uint32_t c = 0;
    const uint32_t base = pass ? off[i] : 0;
    // the same neighbour walk as the physics passes
    for_each_neighbor<R, DIM, 4, 1>(d, I, O, pos, i, L, 0u, [](uint32_t) { return NoExtra{}; },
        [&](uint32_t k, const R*, R, const R4<R>&, uint32_t, NoExtra) {
            if (pass) out[base + c] = O.id[k];
            ++c;
        });
    if (!pass) out[i] = c;
}

// ================================================================ launchers

static inline unsigned blocks_for(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

// Blocks of the one-launch build: as many as the device holds at once (all must be
// resident for the grid barriers), no more than the largest phase can use.
template <class R, int DIM>
static unsigned build_grid(const Dev& d, uint32_t ntiles)
{
    static int per_cu = -1;   // depends on the kernel and the architecture only
    if (per_cu < 0) {
        int v = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&v, k_build<R, DIM>, 256, 0) != hipSuccess) v = 0;
        per_cu = v;
    }
    int dev = 0, ncu = 0;
    if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) !=
                                                 hipSuccess)
        ncu = 0;
    const uint64_t resident = std::min<uint64_t>((uint64_t)per_cu * (uint64_t)ncu, kBarMaxBlocks);
    uint64_t need = std::max<uint64_t>(blocks_for(d.n * NlistLanes<R>::value, 256), ntiles);
    if (need < 1) need = 1;
    return (unsigned)std::min<uint64_t>(resident, need);
}

template <class R, int DIM>
static void build_impl(const Dev& d, const Launch& L, hipStream_t s)
{
    const int B = 256;
    const uint32_t ntiles = (d.ncell + SCAN_TILE - 1) / SCAN_TILE;
    if (L.one_launch_build) {
        const unsigned g = build_grid<R, DIM>(d, ntiles);
        if (g > 0) {
            hipLaunchKernelGGL((k_build<R, DIM>), dim3(g), dim3(256), 0, s, d, ntiles, d.O[0].ref ? 1 : 0,
                               L.stall_at);
            return;
        }
    }
    // seven launches, each returning at once on the (usual) steps without a rebuild
    const uint32_t* gate = d.flags;
    hipLaunchKernelGGL((k_hash<R, DIM>), dim3(blocks_for(d.n, B)), dim3(B), 0, s, d);
    hipLaunchKernelGGL(k_scan_reduce, dim3(ntiles), dim3(SCAN_THREADS), 0, s, gate, d.cnt, d.ncell, d.scan_tmp);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(SCAN_THREADS), 0, s, d, d.scan_tmp, ntiles);
    hipLaunchKernelGGL(k_scan_down, dim3(ntiles), dim3(SCAN_THREADS), 0, s, gate, d.cnt, d.ncell, d.scan_tmp, d.cstart);
    hipLaunchKernelGGL(k_scatter, dim3(blocks_for(d.n, B)), dim3(B), 0, s, d);
    hipLaunchKernelGGL((k_rank<R, DIM>), dim3(blocks_for(d.n, B)), dim3(B), 0, s, d, d.O[0].ref ? 1 : 0);
    // 256-thread blocks: most steps skip the build, and a skipped launch costs in
    // proportion to its workgroup count
    hipLaunchKernelGGL((k_nlist<R, DIM>), dim3(blocks_for(d.n * NlistLanes<R>::value, 256)), dim3(256), 0, s, d,
                       L.xcd_remap);
}

#define SPHX_DISPATCH(PREC, DIM, CALL)                                  \
    do {                                                                \
        if ((PREC) == 0) {                                              \
            if ((DIM) == 2) { using R = double; constexpr int D = 2; CALL; } \
            else { using R = double; constexpr int D = 3; CALL; }       \
        } else {                                                        \
            if ((DIM) == 2) { using R = float; constexpr int D = 2; CALL; } \
            else { using R = float; constexpr int D = 3; CALL; }        \
        }                                                               \
    } while (0)

void launch_build(const Dev& d, const Launch& L, hipStream_t s)
{
    SPHX_DISPATCH(d.precision, d.dim, (build_impl<R, D>(d, L, s)));
}

void launch_nlist(const Dev& d, const Launch& L, hipStream_t s)
{
    SPHX_DISPATCH(d.precision, d.dim, ({
        hipLaunchKernelGGL((k_nlist<R, D>), dim3(blocks_for(d.n * NlistLanes<R>::value, 256)), dim3(256), 0, s, d,
                           L.xcd_remap);
    }));
}

// Lanes per particle of the neighbour passes: 1, 2 or 4 (checked by the runtime).
#define SPHX_LANES(LANES, CALL)                                         \
    do {                                                                \
        if ((LANES) == 4) { constexpr int P = 4; CALL; }                \
        else if ((LANES) == 2) { constexpr int P = 2; CALL; }           \
        else { constexpr int P = 1; CALL; }                             \
    } while (0)

void launch_renorm(const Dev& d, bool force, const Launch& L, hipStream_t s)
{
    const int f = force ? 1 : 0;
    const dim3 grid(blocks_for(d.n * L.lanes, L.block)), block(L.block);
    SPHX_DISPATCH(d.precision, d.dim, ({
        SPHX_LANES(L.lanes, ({ hipLaunchKernelGGL((k_renorm<R, D, P>), grid, block, 0, s, d, L.xcd_remap, f); }));
        hipLaunchKernelGGL((k_derive<R>), dim3(blocks_for(d.n, 256)), dim3(256), 0, s, d, 1, f);
    }));
}

void launch_derive(const Dev& d, const Launch&, hipStream_t s)
{
    SPHX_DISPATCH(d.precision, d.dim, ({
        hipLaunchKernelGGL((k_derive<R>), dim3(blocks_for(d.n, 256)), dim3(256), 0, s, d, 0, 0);
    }));
}

void launch_restore(const Dev& d, hipStream_t s)
{
    SPHX_DISPATCH(d.precision, d.dim, ({
        hipLaunchKernelGGL((k_derive<R>), dim3(blocks_for(d.n, 256)), dim3(256), 0, s, d, 2, 0);
    }));
}

void launch_renorm_colour(const Dev& d, const Launch& L, hipStream_t s, int parts)
{
    const dim3 grid(blocks_for(d.n * L.lanes, L.block)), block(L.block);
    // colour blocks: the list length is known only on the device (grid-stride)
    const unsigned cb = std::min<unsigned>(blocks_for(d.n * kColourLanes, 256), 1024u);
    const unsigned db = blocks_for(d.n, 256);
    SPHX_DISPATCH(d.precision, d.dim, ({
        if (parts & 1)
            SPHX_LANES(L.lanes, ({ hipLaunchKernelGGL((k_renorm<R, D, P>), grid, block, 0, s, d, L.xcd_remap, 0); }));
        if (parts & 2) hipLaunchKernelGGL((k_derive_colour<R, D>), dim3(cb + db), dim3(256), 0, s, d, 0, cb);
    }));
}

void launch_colour(const Dev& d, bool star, const Launch& L, hipStream_t s)
{
    // grid-stride over the colour list, whose length is known only on the device
    const unsigned nb = blocks_for(d.n * kColourLanes, L.block);
    const dim3 grid(nb < 4096u ? nb : 4096u), block(L.block);
    SPHX_DISPATCH(d.precision, d.dim, ({
        hipLaunchKernelGGL((k_colour<R, D>), grid, block, 0, s, d, star ? 1 : 0);
    }));
}

// The rates at S^n (with the time-step maxima) or, with `correct`, at S* followed by
// the corrector.
void launch_force(const Dev& d, bool star, bool reduce_max, bool correct, const Launch& L, hipStream_t s)
{
    const int st = star ? 1 : 0;
    const dim3 grid(blocks_for(d.n * L.force_lanes, L.block)), block(L.block);
    SPHX_DISPATCH(d.precision, d.dim, SPHX_LANES(L.force_lanes, ({
        if (correct) {
            if (L.debug_terms) hipLaunchKernelGGL((k_force<R, D, P, false, true, true>), grid, block, 0, s, d, st, L.xcd_remap);
            else hipLaunchKernelGGL((k_force<R, D, P, false, false, true>), grid, block, 0, s, d, st, L.xcd_remap);
        } else if (L.debug_terms) {
            if (reduce_max) hipLaunchKernelGGL((k_force<R, D, P, true, true, false>), grid, block, 0, s, d, st, L.xcd_remap);
            else hipLaunchKernelGGL((k_force<R, D, P, false, true, false>), grid, block, 0, s, d, st, L.xcd_remap);
        } else {
            if (reduce_max) hipLaunchKernelGGL((k_force<R, D, P, true, false, false>), grid, block, 0, s, d, st, L.xcd_remap);
            else hipLaunchKernelGGL((k_force<R, D, P, false, false, false>), grid, block, 0, s, d, st, L.xcd_remap);
        }
    })));
}

void launch_predict(const Dev& d, double dt_override, const Launch& L, hipStream_t s)
{
    // colour blocks first: the list length is known only on the device
    const unsigned cb = L.colour_in_predict ? std::min<unsigned>(blocks_for(d.n * kColourLanes, 256), 1024u) : 0u;
    SPHX_DISPATCH(d.precision, d.dim, ({
        hipLaunchKernelGGL((k_predict<R, D>), dim3(cb + blocks_for(d.n, 256)), dim3(256), 0, s, d, dt_override, cb);
    }));
}

void launch_place_moving(const Dev& d, uint32_t inst, hipStream_t s)
{
    SPHX_DISPATCH(d.precision, d.dim, ({
        hipLaunchKernelGGL((k_place_moving<R>), dim3(blocks_for(d.n, 256)), dim3(256), 0, s, d, inst);
    }));
}



void launch_export(const Dev& d, int pass, const uint32_t* off, uint32_t* out, const Launch&, hipStream_t s)
{
    SPHX_DISPATCH(d.precision, d.dim, ({
        hipLaunchKernelGGL((k_export<R, D>), dim3(blocks_for(d.n, 256)), dim3(256), 0, s, d, pass, off, out);
    }));
}

} // namespace sphx
