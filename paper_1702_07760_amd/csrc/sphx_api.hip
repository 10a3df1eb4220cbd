// C-ABI runtime of the sphx library: validation, workspace carving, step
// sequencing, hipGraph capture and read-back in original particle order.
#include "sphx.h"
#include "sphx_internal.h"

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <limits>
#include <mutex>
#include <string>
#include <vector>

using namespace sphx;

// The static workspace of sphx_bind_static_workspace: device memory for callers that
// cannot allocate.  Each device holds its own copy from the loading of this library
// until the process ends.  Host code never passes `scratch` itself to the device (on
// the host the name stands for a host-side shadow, not a device address): it takes
// each device's address once with hipGetSymbolAddress and uses that.
static __device__ __align__(256) unsigned char scratch[SPHX_STATIC_WORKSPACE_BYTES];

struct sphx_ctx {
    int precision = 0, dim = 0, ninst = 0, nphase = 0;
    int device = 0;               // the device current at sphx_create
    bool static_ws = false;       // bound to the device's static workspace ...
    uint64_t static_gen = 0;      // ... as its static_gen-th binding
    int64_t n = 0;
    std::vector<sphx_params> params;
    std::vector<sphx_phase> phases;     // ninst * 2 (nphase == 1 duplicates phase 0)
    std::vector<int64_t> counts, offsets;
    std::vector<InstDev> inst;
    uint32_t ncell = 0;
    hipStream_t stream = nullptr;
    int num_cu = 256;
    void* ws = nullptr;
    size_t ws_bytes = 0;
    Dev dev{};
    Launch launch{};
    bool bound = false, inited = false, rates_valid = false;
    bool has_moving = false;
    bool use_graph = true;
    hipGraphExec_t graph = nullptr;    // one step; the state parity lives on the device
    hipGraphExec_t graph_k = nullptr;  // kGraphSteps steps: one replay, fewer launch gaps
    bool profile = false;
    std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> events;   // (group, start/stop)
    double phase_ms[SPHX_NPH] = {0, 0, 0, 0, 0};
    int64_t phase_launches[SPHX_NPH] = {0, 0, 0, 0, 0};
    std::string err;
};

namespace {

sphx_status fail(sphx_ctx* c, sphx_status s, const char* fmt, ...)
{
    if (c) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof buf, fmt, ap);
        va_end(ap);
        c->err = buf;
    }
    return s;
}

#define HIP_OK(c, call)                                                                     \
    do {                                                                                    \
        hipError_t e_ = (call);                                                             \
        if (e_ != hipSuccess) return fail((c), SPHX_E_HIP, "%s: %s", #call, hipGetErrorString(e_)); \
    } while (0)

// ---------------------------------------------------------------- geometry

struct Grid {
    int32_t nc[3];
    double cs[3];
};

bool grid_of(const sphx_params& p, Grid& g, std::string& why)
{
    const double reach = (2.0 + p.skin_coef) * p.h;
    for (int d = 0; d < 3; ++d) {
        if (d >= p.dim) { g.nc[d] = 1; g.cs[d] = 1.0; continue; }
        const double L = p.hi[d] - p.lo[d];
        double k = std::floor(L / reach);
        if (!(k >= 1.0)) k = 1.0;
        if (k > 1e7) { why = "domain too large for the cell grid"; return false; }
        g.nc[d] = (int32_t)k;
        g.cs[d] = L / k;
        if (p.periodic[d] && g.nc[d] < 3) { why = "a periodic dimension needs at least 3 cells (period >= 3 (2 + skin) h)"; return false; }
    }
    return true;
}

bool check_params(const sphx_params& p, int dim, std::string& why)
{
    auto fin = [](double v) { return std::isfinite(v); };
    if (p.dim != 2 && p.dim != 3) { why = "dim must be 2 or 3"; return false; }
    if (p.dim != dim) { why = "every instance must have the same dim"; return false; }
    if (!(fin(p.h) && p.h > 0)) { why = "h must be positive"; return false; }
    if (p.gamma != 7.0) { why = "gamma must be 7"; return false; }
    if (!(fin(p.delta_coef) && p.delta_coef >= 0)) { why = "delta_coef must be >= 0"; return false; }
    if (!(fin(p.alpha_s) && p.alpha_s >= 0)) { why = "alpha_s must be >= 0"; return false; }
    if (p.visc_form != 0 && p.visc_form != 1) { why = "visc_form must be 0 or 1"; return false; }
    if (p.cont_form != 0 && p.cont_form != 1) { why = "cont_form must be 0 or 1"; return false; }
    if (p.renorm_every < 0) { why = "renorm_every must be >= 0"; return false; }
    if (!(fin(p.skin_coef) && p.skin_coef > 0 && p.skin_coef <= 2)) { why = "skin_coef must be in (0, 2]"; return false; }
    if (!(p.c_cfl > 0 && p.c_force > 0 && p.c_visc > 0 && p.c_st > 0)) { why = "time-step coefficients must be positive"; return false; }
    if (!(fin(p.dt_fixed) && p.dt_fixed >= 0)) { why = "dt_fixed must be >= 0"; return false; }
    if (p.n_piston < 0 || p.n_piston > SPHX_MAX_PISTON) { why = "n_piston out of range"; return false; }
    for (int d = 0; d < 3; ++d) {
        if (!fin(p.gravity[d])) { why = "gravity must be finite"; return false; }
        if (d >= p.dim) continue;
        if (!(fin(p.lo[d]) && fin(p.hi[d]) && p.hi[d] > p.lo[d])) { why = "lo < hi required"; return false; }
        if (p.periodic[d] != 0 && p.periodic[d] != 1) { why = "periodic must be 0 or 1"; return false; }
    }
    Grid g;
    return grid_of(p, g, why);
}

InstDev make_inst(const sphx_params& p, const sphx_phase* ph2, int nphase, uint32_t cell_base)
{
    InstDev I;
    std::memset(&I, 0, sizeof I);
    Grid g;
    std::string why;
    grid_of(p, g, why);
    I.ncell = 1;
    for (int d = 0; d < 3; ++d) {
        const bool act = d < p.dim;
        I.lo[d] = act ? p.lo[d] : 0.0;
        I.hi[d] = act ? p.hi[d] : 1.0;
        I.span[d] = I.hi[d] - I.lo[d];
        I.cs[d] = g.cs[d];
        I.nc[d] = g.nc[d];
        I.periodic[d] = act ? p.periodic[d] : 0;
        I.g[d] = act ? p.gravity[d] : 0.0;
        I.ncell *= (uint32_t)g.nc[d];
        I.f_cs[d] = (float)g.cs[d];
        I.f_cs_lo[d] = (float)(g.cs[d] - (double)I.f_cs[d]);
        I.f_g[d] = (float)I.g[d];
    }
    I.cell_base = cell_base;
    I.dim = p.dim;
    I.visc_form = p.visc_form;
    I.cont_form = p.cont_form;
    I.renorm_every = p.renorm_every;
    const double h = p.h;
    const double alpha = p.dim == 2 ? 7.0 / (4.0 * M_PI * h * h) : 21.0 / (16.0 * M_PI * h * h * h);
    I.h = h;
    I.inv_h = 1.0 / h;
    I.cut2 = 4.0 * h * h;
    // neighbour-list radius: the cell size (2 + skin) h, with a margin far above FP32 rounding
    const double rl = (2.0 + p.skin_coef) * h;
    I.cutl2 = rl * rl * (1.0 + 2e-5);
    // the list (and the cells) stay valid while no particle is more than skin/2 from its
    // position at the build, at S^n and at the predicted state S*: a pair within 2h there
    // was then within (2 + skin) h at the build.  The rebuild rule keeps the displacement
    // at S^n plus the half step dt/2 max|u| below 99 % of skin/2 (dt_bound bounds dt);
    // the predictor refuses a step that would break it (SPHX_E_DT)
    I.rebuild_e = 0.495 * p.skin_coef * h;
    I.wcoef = alpha;
    I.fcoef = -5.0 * alpha / (h * h);
    const double delta = p.delta_coef * h;
    I.delta2 = delta * delta;
    I.alpha_s = p.alpha_s;
    I.skin = p.skin_coef * h;
    double cmax = 0, numax = 0, rho0min = std::numeric_limits<double>::infinity();
    for (int q = 0; q < 2; ++q) {
        const sphx_phase& f = ph2[q];
        I.rho0[q] = f.rho0;
        I.beta[q] = f.rho0 * f.c0 * f.c0 / p.gamma;
        I.nu[q] = f.nu;
        if (q < nphase) {
            cmax = std::max(cmax, f.c0);
            numax = std::max(numax, f.nu);
            rho0min = std::min(rho0min, f.rho0);
        }
    }
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) {
            double v;
            if (p.visc_form == 1) {
                const double ma = ph2[a].nu * ph2[a].rho0, mb = ph2[b].nu * ph2[b].rho0;
                v = (ma + mb) > 0 ? 2.0 * ma * mb / (ma + mb) : 0.0;   // Eq. (13)
            } else {
                const double na = ph2[a].nu, nb = ph2[b].nu;
                v = (na + nb) > 0 ? 2.0 * na * nb / (na + nb) : 0.0;   // Eq. (12)
            }
            I.vpair[a][b] = 2.0 * v;
            I.f_vpair[a][b] = (float)(2.0 * v);
        }
    I.dt_fixed = p.dt_fixed;
    I.c_cfl = p.c_cfl;
    I.c_force = p.c_force;
    I.cmax = cmax;
    I.dt_bound = p.dt_fixed > 0 ? p.dt_fixed : (cmax > 0 ? p.c_cfl * h / cmax : 0.0);
    double lim = std::numeric_limits<double>::infinity();
    if (numax > 0) lim = std::min(lim, p.c_visc * h * h / numax);
    if (p.alpha_s > 0 && nphase == 2) lim = std::min(lim, p.c_st * std::sqrt(rho0min * h * h * h / (2.0 * M_PI * p.alpha_s)));
    I.dt_const = lim;
    I.n_piston = p.n_piston;
    I.piston_t_end = p.piston_t_end;
    for (int k = 0; k < p.n_piston; ++k) {
        I.pa[k] = p.piston_a[k];
        I.pw[k] = p.piston_w[k];
        I.pphi[k] = p.piston_phi[k];
    }
    I.f_inv_h = (float)I.inv_h;
    I.f_cut2 = (float)I.cut2;
    I.f_cutl2 = (float)I.cutl2;
    I.f_fcoef = (float)I.fcoef;
    I.f_wcoef = (float)I.wcoef;
    I.f_delta2 = (float)I.delta2;
    I.f_alpha_s = (float)I.alpha_s;
    I.f_rho0[0] = (float)I.rho0[0];
    I.f_rho0[1] = (float)I.rho0[1];
    return I;
}

// ---------------------------------------------------------------- workspace

struct Carver {
    char* base;
    size_t off = 0;
    explicit Carver(void* b) : base((char*)b) {}
    template <class T> T* take(size_t count)
    {
        off = (off + 255) & ~size_t(255);
        T* p = base ? (T*)(base + off) : nullptr;
        off += count * sizeof(T);
        return p;
    }
};

// Lays every device array out in the workspace (or only measures when base is null).
uint32_t list_cap(int dim) { return dim == 3 ? kListCap3 : kListCap2; }

size_t carve(Dev& d, void* base, int precision, int dim, int64_t n, uint32_t ncell, int ninst)
{
    Carver c(base);
    const size_t R = precision == 0 ? 8 : 4;
    const size_t un = (size_t)n;
    d.inst = c.take<InstDev>(ninst);
    d.run = c.take<InstRun>(ninst);
    d.status = c.take<uint32_t>(1);
    d.fault = c.take<FaultRec>(1);
    d.inter = c.take<unsigned long long>((size_t)kInterSlots * kInterStride);
    d.curp = c.take<int>(1);
    d.prevp = c.take<int>(1);
    d.bar = c.take<unsigned>(kBarWords);   // the one-launch build's barrier words and slots
    d.flags = c.take<uint32_t>(4);
    d.cnt = c.take<uint32_t>(ncell);
    d.cstart = c.take<uint32_t>((size_t)ncell + 1);
    d.scan_tmp = c.take<uint32_t>((ncell + 2047) / 2048 + 1);
    d.cap = list_cap(dim);
    d.lstride = (uint32_t)((un + 31) & ~(size_t)31);
    d.nbl = c.take<uint32_t>((size_t)d.lstride * d.cap);
    d.nbc = c.take<uint32_t>(un);
    d.ilist = c.take<uint32_t>(un);
    d.icount = c.take<uint32_t>(1);
    d.xb = c.take<char>(un * 4 * R);
    d.newkey = c.take<uint32_t>(un);
    d.slot = c.take<uint32_t>(un);
    d.tsrc = c.take<uint32_t>(un);
    d.tid = c.take<uint32_t>(un);
    // the gathered records have one more slot: index n, the sentinel of padded lists
    for (int s = 0; s < 2; ++s) {
        d.S[s].pos = c.take<char>((un + 1) * 4 * R);
        d.S[s].vel = c.take<char>((un + 1) * 4 * R);
        d.S[s].aux = c.take<char>((un + 1) * 4 * R);
        d.S[s].plo = precision ? c.take<float4>(un) : nullptr;
        d.S[s].vlo = precision ? c.take<float4>(un) : nullptr;
        d.O[s].key = c.take<uint32_t>(un);
        d.O[s].id = c.take<uint32_t>(un);
        d.O[s].info = c.take<uint32_t>(un);
        d.O[s].ref = c.take<double4>(un);
    }
    d.star.pos = c.take<char>((un + 1) * 4 * R);
    d.star.vel = c.take<char>((un + 1) * 4 * R);
    d.star.aux = c.take<char>((un + 1) * 4 * R);
    d.star.plo = nullptr;
    d.star.vlo = nullptr;
    d.rho_tmp = c.take<char>((un + 1) * R);
    d.acc = c.take<char>(un * 4 * R);
    d.gc = c.take<char>((un + 1) * 4 * R);
    d.terms = c.take<char>(un * 12 * R);
    return (c.off + 255) & ~size_t(255);
}

bool setup_cells(const sphx_params* per, int ninst, std::vector<uint32_t>& base, uint32_t& total, std::string& why)
{
    uint64_t acc = 0;
    base.resize(ninst);
    for (int b = 0; b < ninst; ++b) {
        Grid g;
        if (!grid_of(per[b], g, why)) return false;
        base[b] = (uint32_t)acc;
        acc += (uint64_t)g.nc[0] * g.nc[1] * g.nc[2];
        if (acc >= (1ull << 31)) { why = "too many cells"; return false; }
    }
    total = (uint32_t)acc;
    return true;
}

// ---------------------------------------------------------------- stepping

void drop_graphs(sphx_ctx* c);
sphx_status request_rebuild(sphx_ctx* c);
void enqueue_build(sphx_ctx* c);

sphx_status status_of(sphx_ctx* c)
{
    uint32_t st = 0;
    HIP_OK(c, hipStreamSynchronize(c->stream));
    HIP_OK(c, hipMemcpy(&st, c->dev.status, sizeof st, hipMemcpyDeviceToHost));
    if (st) {
        const uint32_t zero = 0;
        HIP_OK(c, hipMemcpy(c->dev.status, &zero, sizeof zero, hipMemcpyHostToDevice));
    }
    if (st & ST_STALL) {
        // the build stopped at a grid barrier and every pass after it returned at once.
        // The current state set is whole (the build writes only the other set before its
        // last barrier and makes it current after that barrier); the cell table and the
        // list are not.  Clear what the next build expects cleared (barrier words that
        // may hold this launch's epochs, the cell counters) and rebuild from the current
        // set with seven launches, as every later build will be.
        HIP_OK(c, hipMemset(c->dev.bar, 0, kBarWords * sizeof(unsigned)));
        HIP_OK(c, hipMemset(c->dev.cnt, 0, (size_t)c->ncell * sizeof(uint32_t)));
        c->launch.one_launch_build = false;
        c->launch.stall_at = 0;
        c->rates_valid = false;
        drop_graphs(c);
        if (const sphx_status e = request_rebuild(c)) return e;
        enqueue_build(c);
        HIP_OK(c, hipStreamSynchronize(c->stream));
        return fail(c, SPHX_E_STALL, "a grid barrier of the one-launch neighbour build timed out (its blocks were "
                                     "not all resident): the work queued from that build on was not done, the "
                                     "state is as the build found it, and builds use seven launches from now on");
    }
    if (st & ST_NONFINITE) return fail(c, SPHX_E_NONFINITE, "a rate or state value became non-finite");
    if (st & ST_DOMAIN) {
        FaultRec f;
        HIP_OK(c, hipMemcpy(&f, c->dev.fault, sizeof f, hipMemcpyDeviceToHost));
        HIP_OK(c, hipMemset(c->dev.fault, 0, sizeof f));
        if (!f.claimed) return fail(c, SPHX_E_DOMAIN, "a particle left a non-periodic domain");
        const InstDev& I = c->inst[f.inst < (uint32_t)c->ninst ? f.inst : 0];
        return fail(c, SPHX_E_DOMAIN,
                    "a particle left a non-periodic domain: particle %u (instance %u) at (%.9g, %.9g, %.9g) m, "
                    "cell (%d, %d, %d) of a %d x %d x %d grid",
                    f.id, f.inst, f.x[0], f.x[1], f.x[2], f.cell[0], f.cell[1], f.cell[2], I.nc[0], I.nc[1], I.nc[2]);
    }
    if (st & ST_DT) return fail(c, SPHX_E_DT, "a step would take a particle more than half the neighbour skin "
                                               "from its position at the last neighbour build");
    return SPHX_OK;
}

// Per device: the address of its static workspace (0 until the first binding there)
// and the number of bindings so far; a context bound to it owns it while no later
// binding has taken it.
constexpr int kMaxDevices = 64;
std::mutex g_static_mu;
void* g_static_ptr[kMaxDevices];
std::atomic<uint64_t> g_static_gen[kMaxDevices];

sphx_status owns_workspace(sphx_ctx* c)
{
    if (c->static_ws && g_static_gen[c->device].load(std::memory_order_acquire) != c->static_gen)
        return fail(c, SPHX_E_WORKSPACE, "another context has since bound the static workspace of this device; "
                                         "bind a workspace and call init_particles again");
    return SPHX_OK;
}

// Why the last sphx_create of this thread failed (sphx_last_error(NULL) returns it).
thread_local std::string g_create_err;

sphx_status create_fail(sphx_status s, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_create_err = buf;
    return s;
}

// The calls that step or read the particle state need one that is whole.
sphx_status have_state(sphx_ctx* c)
{
    if (!c) return SPHX_E_ARG;
    if (const sphx_status st = owns_workspace(c)) return st;
    if (!c->inited) return fail(c, SPHX_E_STATE, "init_particles first");
    return SPHX_OK;
}

// Brackets the launches of one kernel group with events when profiling.
struct Timed {
    sphx_ctx* c;
    int group;
    hipEvent_t a = nullptr, b = nullptr;
    Timed(sphx_ctx* ctx, int g) : c(ctx), group(g)
    {
        if (c->profile && hipEventCreate(&a) == hipSuccess && hipEventCreate(&b) == hipSuccess)
            (void)hipEventRecord(a, c->stream);
    }
    ~Timed()
    {
        if (a && b) {
            (void)hipEventRecord(b, c->stream);
            c->events.push_back({group, {a, b}});
        }
    }
};

void collect_events(sphx_ctx* c)
{
    for (auto& e : c->events) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, e.second.first, e.second.second) == hipSuccess) {
            c->phase_ms[e.first] += ms;
            c->phase_launches[e.first] += 1;
        }
        (void)hipEventDestroy(e.second.first);
        (void)hipEventDestroy(e.second.second);
    }
    c->events.clear();
}

void enqueue_build(sphx_ctx* c)
{
    Timed t(c, SPHX_PH_BUILD);
    launch_build(c->dev, c->launch, c->stream);
}

// The rates at S^n (colour unless done already, force with the time-step maxima) or at
// S* (colour, force and, in the same launch, the corrector that ends the step).
void enqueue_rates(sphx_ctx* c, bool star, bool reduce, bool colour = true)
{
    if (colour) {
        Timed t(c, SPHX_PH_COLOUR);
        launch_colour(c->dev, star, c->launch, c->stream);
    }
    // the launch at S* also holds the corrector: it is timed with the integrator, so the
    // force group holds the pure force pass at S^n
    Timed t(c, star ? SPHX_PH_INTEGRATE : SPHX_PH_FORCE);
    launch_force(c->dev, star, reduce, star, c->launch, c->stream);
}

void enqueue_integrate(sphx_ctx* c, double dt_override)
{
    {
        Timed t(c, SPHX_PH_INTEGRATE);
        launch_predict(c->dev, dt_override, c->launch, c->stream);   // a9 (and the colour pass at S*)
    }
    // the corrector runs in the force launch at S*
    enqueue_rates(c, true, false, !c->launch.colour_in_predict);
}

void enqueue_renorm(sphx_ctx* c, bool force)
{
    Timed t(c, SPHX_PH_RENORM);
    launch_renorm(c->dev, force, c->launch, c->stream);
}

// One full step: neighbour structure (rebuilt only when due), Eq. (7) when due, rates
// at S^n, time step, predictor, rates at S*, corrector.
void enqueue_step(sphx_ctx* c)
{
    enqueue_build(c);
    // Eq. (7) when due, then the derive pass with the colour pass at S^n in one launch
    // (timed as two groups when profiling)
    if (c->profile) {
        {
            Timed t(c, SPHX_PH_RENORM);
            launch_renorm_colour(c->dev, c->launch, c->stream, 1);
        }
        Timed t(c, SPHX_PH_COLOUR);
        launch_renorm_colour(c->dev, c->launch, c->stream, 2);
    } else {
        launch_renorm_colour(c->dev, c->launch, c->stream, 3);
    }
    enqueue_rates(c, false, true, false);
    enqueue_integrate(c, 0.0);
}

sphx_status request_rebuild(sphx_ctx* c)
{
    const uint32_t one = 1;
    HIP_OK(c, hipMemcpyAsync(c->dev.flags + 1, &one, sizeof one, hipMemcpyHostToDevice, c->stream));
    return SPHX_OK;
}

// Current state set (synchronises the stream).
int device_cur(sphx_ctx* c)
{
    int cur = 0;
    if (hipStreamSynchronize(c->stream) != hipSuccess) return 0;
    if (hipMemcpy(&cur, c->dev.curp, sizeof cur, hipMemcpyDeviceToHost) != hipSuccess) return 0;
    return cur & 1;
}

void drop_graphs(sphx_ctx* c)
{
    if (c->graph_k) {
        (void)hipGraphExecDestroy(c->graph_k);
        c->graph_k = nullptr;
    }
    if (c->graph) {
        (void)hipGraphExecDestroy(c->graph);
        c->graph = nullptr;
    }
}

} // namespace

// ----------------------------------------------------------- checkpoints

namespace {
struct BlobHeader {
    uint64_t magic;
    int32_t precision, dim, ninst, cur;
    int64_t n;
    uint32_t ncell, rates_valid, cap, qpos;   // qpos: device flag 2 (pos.w holds q)
};
constexpr uint64_t kMagic = 0x5350485853543035ull;   // "SPHXST05"

struct Span { void* p; size_t bytes; };

// Everything a continuation depends on, in the sorted order of state set `s`: the state,
// the cell table, the neighbour list and its build positions, the per-instance run
// variables and the last rates.
// The per-instance mass table: umass stays 1 for an instance while all its particles
// of one phase share one mass.  particle(i, inst, phase, mass) describes particle i.
template <class F>
void mass_table(sphx_ctx* c, int64_t n, F&& particle)
{
    std::vector<char> seen((size_t)c->ninst * 2, 0);
    for (InstDev& I : c->inst) {
        I.umass = 1;
        I.mass[0] = I.mass[1] = 0.0;
    }
    for (int64_t i = 0; i < n; ++i) {
        uint32_t b = 0, q = 0;
        double m = 0.0;
        particle(i, b, q, m);
        InstDev& I = c->inst[b];
        char& s = seen[(size_t)b * 2 + q];
        if (!s) {
            I.mass[q] = m;
            s = 1;
        } else if (m != I.mass[q]) {
            I.umass = 0;
        }
    }
    for (InstDev& I : c->inst) {
        I.f_mass[0] = (float)I.mass[0];
        I.f_mass[1] = (float)I.mass[1];
    }
}

std::vector<Span> state_spans(sphx_ctx* c, int s)
{
    const size_t n = (size_t)c->n, R = c->precision ? 4 : 8;
    Dev& d = c->dev;
    std::vector<Span> v = {
        {d.S[s].pos, n * 4 * R}, {d.S[s].vel, n * 4 * R}, {d.S[s].aux, n * 4 * R},
        {d.O[s].key, n * 4}, {d.O[s].id, n * 4}, {d.O[s].info, n * 4}, {d.cstart, ((size_t)c->ncell + 1) * 4},
        {d.run, sizeof(InstRun) * c->ninst}, {d.acc, n * 4 * R}, {d.gc, n * 4 * R},
        {d.nbl, (size_t)d.lstride * d.cap * 4}, {d.nbc, n * 4}, {d.ilist, n * 4}, {d.icount, 4}, {d.xb, n * 4 * R}};
    if (c->precision) {
        v.push_back({d.S[s].plo, n * 16});
        v.push_back({d.S[s].vlo, n * 16});
    }
    if (d.O[s].ref) v.push_back({d.O[s].ref, n * 32});
    return v;
}

// Full steps per replay of the long step graph: each replay of a graph leaves a launch
// gap of several microseconds before its first kernel.
constexpr int32_t kGraphSteps = 8;

// Captures `steps` full steps into an executable graph; on failure turns graphs off
// for this context and returns null (the steps then run eagerly).
hipGraphExec_t capture_steps(sphx_ctx* c, int32_t steps)
{
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    bool ok = hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal) == hipSuccess;
    if (ok) {
        for (int32_t k = 0; k < steps; ++k) enqueue_step(c);
        ok = hipStreamEndCapture(c->stream, &graph) == hipSuccess && graph &&
             hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) == hipSuccess;
        if (graph) (void)hipGraphDestroy(graph);
    }
    if (!ok) {
        exec = nullptr;
        c->use_graph = false;
        (void)hipGetLastError();
    }
    return exec;
}
} // namespace

namespace {
// Lays the context's arrays out in dev_ptr (the body of both workspace bindings).
sphx_status bind_memory(sphx_ctx* c, void* dev_ptr, size_t bytes)
{
    if (!dev_ptr || ((uintptr_t)dev_ptr & 255)) return fail(c, SPHX_E_WORKSPACE, "workspace must be non-null and 256-byte aligned");
    Dev d{};
    const size_t need = carve(d, nullptr, c->precision, c->dim, c->n, c->ncell, c->ninst);
    if (bytes < need) return fail(c, SPHX_E_WORKSPACE, "workspace too small: %zu < %zu bytes", bytes, need);
    if (c->stream || c->bound) HIP_OK(c, hipStreamSynchronize(c->stream));
    drop_graphs(c);
    c->dev = Dev{};
    carve(c->dev, dev_ptr, c->precision, c->dim, c->n, c->ncell, c->ninst);
    c->dev.precision = c->precision;
    c->dev.dim = c->dim;
    c->dev.ninst = c->ninst;
    c->dev.n = c->n;
    c->dev.ncell = c->ncell;
    c->ws = dev_ptr;
    c->ws_bytes = bytes;
    c->bound = true;
    c->inited = false;
    c->static_ws = false;
    return SPHX_OK;
}
} // namespace

// ===================================================================== C ABI

extern "C" {

size_t sphx_workspace_size(int32_t precision, const sphx_params* per_inst, int32_t ninst, const int64_t* counts)
{
    if (!per_inst || !counts || ninst < 1 || (precision != 0 && precision != 1)) return 0;
    int64_t n = 0;
    for (int b = 0; b < ninst; ++b) {
        if (counts[b] < 1) return 0;
        n += counts[b];
    }
    std::vector<uint32_t> base;
    uint32_t total;
    std::string why;
    if (!setup_cells(per_inst, ninst, base, total, why)) return 0;
    Dev d{};
    return carve(d, nullptr, precision, per_inst[0].dim, n, total, ninst);
}

sphx_status sphx_create(int32_t precision, const sphx_params* per_inst, const sphx_phase* phases, int32_t nphase,
                        int32_t ninst, const int64_t* counts, void* stream, sphx_ctx** out)
{
    g_create_err.clear();
    if (!out) return create_fail(SPHX_E_ARG, "null output pointer");
    *out = nullptr;
    if (!per_inst || !phases || !counts) return create_fail(SPHX_E_ARG, "null argument");
    if (precision != SPHX_FP64 && precision != SPHX_FP32_CELLREL) return create_fail(SPHX_E_ARG, "unknown precision %d", (int)precision);
    if (ninst < 1 || ninst > (1 << 20) || nphase < 1 || nphase > 2)
        return create_fail(SPHX_E_ARG, "ninst must be in [1, 2^20] and nphase 1 or 2");
    int64_t n = 0;
    for (int b = 0; b < ninst; ++b) {
        if (counts[b] < 1) return create_fail(SPHX_E_ARG, "instance %d has no particles", b);
        n += counts[b];
    }
    if (n >= (1ll << 25)) return create_fail(SPHX_E_ARG, "%lld particles: at most 2^25 - 1 (25-bit list indices)", (long long)n);
    std::string why;
    for (int b = 0; b < ninst; ++b) {
        if (!check_params(per_inst[b], per_inst[0].dim, why)) return create_fail(SPHX_E_ARG, "instance %d: %s", b, why.c_str());
        if (per_inst[b].renorm_every != per_inst[0].renorm_every)
            return create_fail(SPHX_E_ARG, "every instance needs the same renorm_every");
        for (int q = 0; q < nphase; ++q) {
            const sphx_phase& f = phases[(size_t)b * nphase + q];
            if (!(std::isfinite(f.rho0) && f.rho0 > 0 && std::isfinite(f.nu) && f.nu >= 0 && std::isfinite(f.c0) && f.c0 > 0))
                return create_fail(SPHX_E_ARG, "instance %d phase %d: rho0, c0 > 0 and nu >= 0 required", b, q);
        }
    }
    std::vector<uint32_t> base;
    uint32_t total;
    if (!setup_cells(per_inst, ninst, base, total, why)) return create_fail(SPHX_E_ARG, "%s", why.c_str());

    int devid = 0;
    hipError_t he = hipGetDevice(&devid);
    if (he != hipSuccess) return create_fail(SPHX_E_NODEV, "hipGetDevice: %s", hipGetErrorString(he));
    hipDeviceProp_t prop;
    he = hipGetDeviceProperties(&prop, devid);
    if (he != hipSuccess) return create_fail(SPHX_E_NODEV, "hipGetDeviceProperties: %s", hipGetErrorString(he));
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return create_fail(SPHX_E_NODEV, "device %d is %s, not gfx950", devid, prop.gcnArchName);
    if (devid < 0 || devid >= kMaxDevices) return create_fail(SPHX_E_NODEV, "device index %d beyond %d", devid, kMaxDevices);
    sphx_ctx* c = new sphx_ctx();
    c->precision = precision;
    c->device = devid;
    // launch shape, measured (alternating runs, ms per step): 3D runs two force lanes per
    // particle and tiles in plain dispatch order, in 128-thread blocks (3D drop, FP32:
    // 0.247 against 0.258 for 64 threads with four tiles per CU) or 256 from 2^19
    // particles (3D flume 2.39 against 2.44); 2D keeps one lane and 64-thread blocks,
    // consecutive tiles per XCD in FP64 and four per CU in FP32
    const bool d3 = per_inst[0].dim == 3;
    c->launch.force_lanes = d3 ? 2 : 1;
    c->launch.xcd_remap = d3 ? 0 : (precision == 0 ? 1 : 4);
    c->launch.block = d3 ? (n >= (1 << 19) ? 256 : 128) : 64;
    // 2D from 2^16 particles (except FP64 from 2^20): 128-thread blocks, 16 tiles per CU
    // (2D flume FP32 0.105 against 0.113 ms per step, FP64 0.132 against 0.138; 256 FP32
    // tanks 1.73 against 1.81; the 2k-particle drop and the FP64 tanks keep the above)
    if (!d3 && n >= (1 << 16) && (precision == 1 || n < (1 << 20))) {
        c->launch.block = 128;
        c->launch.xcd_remap = 16;
    }
    // 2D lists hold about 20 entries: once a million particles fill the device, one lane
    // per particle in Eq. (7) beats four (256 FP32 tanks, 6 M particles: 2.98 against
    // 3.18 ms per step); smaller scenes need the parallelism of four
    if (per_inst[0].dim == 2 && n >= (1 << 20)) c->launch.lanes = 1;   // FP64: 3.43 against 3.49 ms
    c->dim = per_inst[0].dim;
    c->ninst = ninst;
    c->nphase = nphase;
    c->n = n;
    c->params.assign(per_inst, per_inst + ninst);
    c->phases.resize((size_t)ninst * 2);
    for (int b = 0; b < ninst; ++b)
        for (int q = 0; q < 2; ++q) c->phases[(size_t)b * 2 + q] = phases[(size_t)b * nphase + (q < nphase ? q : 0)];
    c->counts.assign(counts, counts + ninst);
    c->offsets.resize(ninst + 1);
    c->offsets[0] = 0;
    for (int b = 0; b < ninst; ++b) c->offsets[b + 1] = c->offsets[b] + counts[b];
    c->ncell = total;
    c->inst.resize(ninst);
    for (int b = 0; b < ninst; ++b) c->inst[b] = make_inst(per_inst[b], &c->phases[(size_t)b * 2], nphase, base[b]);
    c->stream = (hipStream_t)stream;
    c->num_cu = prop.multiProcessorCount;
    c->use_graph = stream != nullptr;
    *out = c;
    return SPHX_OK;
}

void sphx_destroy(sphx_ctx* c)
{
    if (!c) return;
    drop_graphs(c);
    if (c->stream || c->bound) (void)hipStreamSynchronize(c->stream);
    collect_events(c);
    delete c;
}

const char* sphx_last_error(const sphx_ctx* c)
{
    if (c) return c->err.c_str();
    return g_create_err.empty() ? "null context" : g_create_err.c_str();
}


sphx_status sphx_bind_workspace(sphx_ctx* c, void* dev_ptr, size_t bytes)
{
    if (!c) return SPHX_E_ARG;
    return bind_memory(c, dev_ptr, bytes);
}

sphx_status sphx_bind_static_workspace(sphx_ctx* c)
{
    if (!c) return SPHX_E_ARG;
    Dev d{};
    const size_t need = carve(d, nullptr, c->precision, c->dim, c->n, c->ncell, c->ninst);
    if (need > (size_t)SPHX_STATIC_WORKSPACE_BYTES)
        return fail(c, SPHX_E_WORKSPACE, "the context needs %zu bytes of workspace; the static workspace holds %zu "
                                         "(bind caller memory with sphx_bind_workspace instead)",
                    need, (size_t)SPHX_STATIC_WORKSPACE_BYTES);
    std::lock_guard<std::mutex> lock(g_static_mu);
    void*& ptr = g_static_ptr[c->device];
    if (!ptr) {
        // once per device, with that device current
        int prev = 0;
        HIP_OK(c, hipGetDevice(&prev));
        HIP_OK(c, hipSetDevice(c->device));
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        const hipError_t e2 = hipSetDevice(prev);
        if (e != hipSuccess || !p)
            return fail(c, SPHX_E_HIP, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
        if (e2 != hipSuccess) return fail(c, SPHX_E_HIP, "hipSetDevice: %s", hipGetErrorString(e2));
        ptr = p;
    }
    if (const sphx_status st = bind_memory(c, ptr, (size_t)SPHX_STATIC_WORKSPACE_BYTES)) return st;
    c->static_ws = true;
    c->static_gen = g_static_gen[c->device].fetch_add(1, std::memory_order_acq_rel) + 1;
    return SPHX_OK;
}

sphx_status sphx_init_particles(sphx_ctx* c, const double* x, const double* u, const double* rho, const double* m,
                                const uint8_t* phase, const uint8_t* kind)
{
    if (!c) return SPHX_E_ARG;
    if (!c->bound) return fail(c, SPHX_E_STATE, "bind a workspace first");
    if (const sphx_status st = owns_workspace(c)) return st;
    if (!x || !u || !rho || !m || !phase || !kind) return fail(c, SPHX_E_ARG, "null array");
    const int64_t n = c->n;
    const bool f32 = c->precision == 1;
    const size_t R = f32 ? 4 : 8;
    // validate everything before touching the device
    bool moving = false;
    for (int b = 0; b < c->ninst; ++b) {
        const sphx_params& p = c->params[b];
        for (int64_t i = c->offsets[b]; i < c->offsets[b + 1]; ++i) {
            for (int d = 0; d < 3; ++d) {
                if (!std::isfinite(u[3 * i + d])) return fail(c, SPHX_E_ARG, "particle %lld: non-finite velocity", (long long)i);
                if (d >= c->dim) continue;
                const double v = x[3 * i + d];
                if (!std::isfinite(v)) return fail(c, SPHX_E_ARG, "particle %lld: non-finite position", (long long)i);
                const bool inside = p.periodic[d] ? (v >= p.lo[d] && v < p.hi[d]) : (v >= p.lo[d] && v <= p.hi[d]);
                if (!inside) return fail(c, SPHX_E_ARG, "particle %lld outside the domain", (long long)i);
            }
            if (!(std::isfinite(rho[i]) && rho[i] > 0)) return fail(c, SPHX_E_ARG, "particle %lld: density must be positive", (long long)i);
            if (!(std::isfinite(m[i]) && m[i] > 0)) return fail(c, SPHX_E_ARG, "particle %lld: mass must be positive", (long long)i);
            if (phase[i] >= c->nphase) return fail(c, SPHX_E_ARG, "particle %lld: phase out of range", (long long)i);
            if (kind[i] > SPHX_MOVING) return fail(c, SPHX_E_ARG, "particle %lld: bad kind", (long long)i);
            if (kind[i] != SPHX_FLUID && phase[i] != 0) return fail(c, SPHX_E_ARG, "particle %lld: boundary particles carry phase 0", (long long)i);
            moving |= kind[i] == SPHX_MOVING;
        }
    }
    c->has_moving = moving;
    // a short colour list (a few drops) is walked beside the predictor: its wave per
    // particle covers the list in one round there
    int64_t other = 0;
    for (int64_t i = 0; i < n; ++i) other += phase[i] != 0;
    c->launch.colour_in_predict = other <= 1024;
    drop_graphs(c);
    for (auto& I : c->inst) I.mv_host = 0;   // MOVING particles follow the piston series again

    std::vector<char> pos(n * 4 * R), vel(n * 4 * R), aux(n * 4 * R);
    std::vector<float4> plo(f32 ? n : 0), vlo(f32 ? n : 0);
    std::vector<uint32_t> key(n), id(n), info(n);
    std::vector<double4> ref(n);
    for (int b = 0; b < c->ninst; ++b) {
        const InstDev& I = c->inst[b];
        for (int64_t i = c->offsets[b]; i < c->offsets[b + 1]; ++i) {
            const double xi[3] = {x[3 * i], c->dim > 1 ? x[3 * i + 1] : 0.0, c->dim > 2 ? x[3 * i + 2] : 0.0};
            id[i] = (uint32_t)i;
            info[i] = make_info(phase[i], kind[i], (uint32_t)b);
            ref[i] = make_double4(xi[0], xi[1], xi[2], 0.0);
            int cc[3];
            for (int d = 0; d < 3; ++d) {
                double k = d < c->dim ? std::floor((xi[d] - I.lo[d]) / I.cs[d]) : 0.0;
                k = std::min(std::max(k, 0.0), (double)(I.nc[d] - 1));
                cc[d] = (int)k;
            }
            key[i] = I.cell_base + (uint32_t)cc[0] + (uint32_t)I.nc[0] * ((uint32_t)cc[1] + (uint32_t)I.nc[1] * (uint32_t)cc[2]);
            const double r0 = I.rho0[phase[i]];
            if (!f32) {
                ((double4*)pos.data())[i] = make_double4(xi[0], xi[1], xi[2], 0.0);   // w = m P / rho^2: derived
                ((double4*)vel.data())[i] = make_double4(u[3 * i], c->dim > 1 ? u[3 * i + 1] : 0.0, c->dim > 2 ? u[3 * i + 2] : 0.0, 0.0);
                ((double4*)aux.data())[i] = make_double4(m[i], 0.0, 0.0, rho[i]);   // V, m P / rho^2: derived
            } else {
                float o[3], e[3], uu[3], ue[3];
                for (int d = 0; d < 3; ++d) {
                    const double off = d < c->dim ? (xi[d] - I.lo[d]) - (double)cc[d] * I.cs[d] : 0.0;
                    o[d] = (float)off;
                    e[d] = (float)(off - (double)o[d]);
                    const double ud = d < c->dim ? u[3 * i + d] : 0.0;
                    uu[d] = (float)ud;
                    ue[d] = (float)(ud - (double)uu[d]);
                }
                const double dr = rho[i] - r0;
                const float drf = (float)dr;
                ((float4*)pos.data())[i] = make_float4(o[0], o[1], o[2], 0.0f);   // w: derived
                plo[i] = make_float4(e[0], e[1], e[2], (float)(dr - (double)drf));
                ((float4*)vel.data())[i] = make_float4(uu[0], uu[1], uu[2], 0.0f);
                vlo[i] = make_float4(ue[0], ue[1], ue[2], 0.0f);
                ((float4*)aux.data())[i] = make_float4((float)m[i], 0.0f, 0.0f, drf);
            }
        }
    }
    mass_table(c, n, [&](int64_t i, uint32_t& b, uint32_t& q, double& mi) {
        b = info_inst(info[i]);
        q = phase[i];
        mi = f32 ? (double)(float)m[i] : m[i];
    });
    Dev& d = c->dev;
    const hipStream_t s = c->stream;
    HIP_OK(c, hipMemcpyAsync((void*)d.inst, c->inst.data(), sizeof(InstDev) * c->ninst, hipMemcpyHostToDevice, s));
    std::vector<InstRun> run(c->ninst);
    std::memset(run.data(), 0, sizeof(InstRun) * c->ninst);
    HIP_OK(c, hipMemcpyAsync(d.run, run.data(), sizeof(InstRun) * c->ninst, hipMemcpyHostToDevice, s));
    HIP_OK(c, hipMemsetAsync(d.status, 0, sizeof(uint32_t), s));
    HIP_OK(c, hipMemsetAsync(d.fault, 0, sizeof(FaultRec), s));
    HIP_OK(c, hipMemsetAsync(d.inter, 0, sizeof(unsigned long long) * kInterSlots * kInterStride, s));
    HIP_OK(c, hipMemsetAsync(d.icount, 0, sizeof(uint32_t), s));
    HIP_OK(c, hipMemsetAsync(d.bar, 0, kBarWords * sizeof(unsigned), s));
    HIP_OK(c, hipMemsetAsync(d.cnt, 0, sizeof(uint32_t) * c->ncell, s));
    HIP_OK(c, hipMemsetAsync(d.acc, 0, n * 4 * R, s));
    HIP_OK(c, hipMemsetAsync(d.gc, 0, (n + 1) * 4 * R, s));
    HIP_OK(c, hipMemsetAsync(d.terms, 0, n * 12 * R, s));
    HIP_OK(c, hipMemcpyAsync(d.S[0].pos, pos.data(), pos.size(), hipMemcpyHostToDevice, s));
    HIP_OK(c, hipMemcpyAsync(d.S[0].vel, vel.data(), vel.size(), hipMemcpyHostToDevice, s));
    HIP_OK(c, hipMemcpyAsync(d.S[0].aux, aux.data(), aux.size(), hipMemcpyHostToDevice, s));
    if (f32) {
        HIP_OK(c, hipMemcpyAsync(d.S[0].plo, plo.data(), n * sizeof(float4), hipMemcpyHostToDevice, s));
        HIP_OK(c, hipMemcpyAsync(d.S[0].vlo, vlo.data(), n * sizeof(float4), hipMemcpyHostToDevice, s));
    }
    // the sentinel record at index n of every gathered array (no kernel writes it): a
    // position far outside every domain, zero velocity, volume and mass
    std::vector<char> spos(4 * R), szero(4 * R, 0);
    if (f32) ((float4*)spos.data())[0] = make_float4(1e30f, 1e30f, 1e30f, 0.0f);
    else ((double4*)spos.data())[0] = make_double4(1e150, 1e150, 1e150, 0.0);
    for (StateSet* set : {&d.S[0], &d.S[1], &d.star}) {
        HIP_OK(c, hipMemcpyAsync((char*)set->pos + n * 4 * R, spos.data(), 4 * R, hipMemcpyHostToDevice, s));
        HIP_OK(c, hipMemcpyAsync((char*)set->vel + n * 4 * R, szero.data(), 4 * R, hipMemcpyHostToDevice, s));
        HIP_OK(c, hipMemcpyAsync((char*)set->aux + n * 4 * R, szero.data(), 4 * R, hipMemcpyHostToDevice, s));
    }
    HIP_OK(c, hipMemcpyAsync(d.O[0].key, key.data(), n * 4, hipMemcpyHostToDevice, s));
    HIP_OK(c, hipMemcpyAsync(d.O[0].id, id.data(), n * 4, hipMemcpyHostToDevice, s));
    HIP_OK(c, hipMemcpyAsync(d.O[0].info, info.data(), n * 4, hipMemcpyHostToDevice, s));
    // the reference-position buffers as the workspace lays them out (an earlier init may
    // have switched them off)
    Dev lay{};
    carve(lay, c->ws, c->precision, c->dim, c->n, c->ncell, c->ninst);
    HIP_OK(c, hipMemcpyAsync(lay.O[0].ref, ref.data(), n * sizeof(double4), hipMemcpyHostToDevice, s));
    // valid (if stale) contents everywhere a build stopped part-way could leave a kernel
    // reading: the other sorted set and the list counts
    HIP_OK(c, hipMemsetAsync(d.O[1].key, 0, n * 4, s));
    HIP_OK(c, hipMemsetAsync(d.O[1].id, 0, n * 4, s));
    HIP_OK(c, hipMemsetAsync(d.O[1].info, 0, n * 4, s));
    HIP_OK(c, hipMemsetAsync(d.nbc, 0, n * 4, s));
    // the gather moves `ref` only when some particle is MOVING
    d.O[0].ref = moving ? lay.O[0].ref : nullptr;
    d.O[1].ref = moving ? lay.O[1].ref : nullptr;
    const int zero = 0;
    // the first build is requested; the set-up derive leaves q in pos.w; no build has
    // taken the two-level barrier yet
    const uint32_t flags[4] = {0u, 1u, 1u, 0u};
    HIP_OK(c, hipMemcpyAsync(d.curp, &zero, sizeof zero, hipMemcpyHostToDevice, s));
    HIP_OK(c, hipMemcpyAsync(d.flags, flags, sizeof flags, hipMemcpyHostToDevice, s));
    launch_derive(d, c->launch, s);
    enqueue_build(c);
    c->inited = true;
    c->rates_valid = false;
    HIP_OK(c, hipGetLastError());
    return status_of(c);   // synchronises; reports a first build that stalled
}

sphx_status sphx_build_neighbors(sphx_ctx* c)
{
    if (!c) return SPHX_E_ARG;
    if (const sphx_status st = have_state(c)) return st;
    sphx_status st = request_rebuild(c);
    if (st) return st;
    enqueue_build(c);
    c->rates_valid = false;
    HIP_OK(c, hipGetLastError());
    return SPHX_OK;
}

sphx_status sphx_renormalize_density(sphx_ctx* c)
{
    if (!c) return SPHX_E_ARG;
    if (const sphx_status st = have_state(c)) return st;
    enqueue_build(c);
    enqueue_renorm(c, true);
    c->rates_valid = false;
    HIP_OK(c, hipGetLastError());
    return SPHX_OK;
}

sphx_status sphx_compute_forces(sphx_ctx* c)
{
    if (!c) return SPHX_E_ARG;
    if (const sphx_status st = have_state(c)) return st;
    enqueue_build(c);
    launch_restore(c->dev, c->stream);   // m P / rho^2 into pos.w, wherever q was left there
    enqueue_rates(c, false, true);
    c->rates_valid = true;
    HIP_OK(c, hipGetLastError());
    return SPHX_OK;
}

sphx_status sphx_integrate_step(sphx_ctx* c, double dt)
{
    if (!c) return SPHX_E_ARG;
    if (const sphx_status st = have_state(c)) return st;
    if (!c->rates_valid) return fail(c, SPHX_E_STATE, "compute_forces first");
    if (!std::isfinite(dt)) return fail(c, SPHX_E_ARG, "dt must be finite");
    enqueue_integrate(c, dt > 0 ? dt : 0.0);
    c->rates_valid = false;
    HIP_OK(c, hipGetLastError());
    return SPHX_OK;
}

sphx_status sphx_step(sphx_ctx* c, int32_t nsteps)
{
    if (!c) return SPHX_E_ARG;
    if (const sphx_status st = have_state(c)) return st;
    if (nsteps < 0) return fail(c, SPHX_E_ARG, "nsteps must be >= 0");
    int32_t k = 0;
    while (k < nsteps) {
        const bool graphs = c->use_graph && !c->profile;
        if (graphs && nsteps - k >= kGraphSteps) {
            if (!c->graph_k) c->graph_k = capture_steps(c, kGraphSteps);
            if (c->graph_k) {
                HIP_OK(c, hipGraphLaunch(c->graph_k, c->stream));
                k += kGraphSteps;
                continue;
            }
        }
        if (c->use_graph && !c->profile && !c->graph) c->graph = capture_steps(c, 1);
        if (c->use_graph && !c->profile && c->graph) HIP_OK(c, hipGraphLaunch(c->graph, c->stream));
        else enqueue_step(c);
        ++k;
    }
    c->rates_valid = false;
    HIP_OK(c, hipGetLastError());
    return SPHX_OK;
}

sphx_status sphx_set_moving(sphx_ctx* c, int32_t inst, const double* disp, const double* vel)
{
    if (const sphx_status st = have_state(c)) return st;
    if (inst < 0 || inst >= c->ninst) return fail(c, SPHX_E_ARG, "instance %d out of range", (int)inst);
    if (!disp || !vel) return fail(c, SPHX_E_ARG, "null array");
    if (!c->has_moving) return fail(c, SPHX_E_STATE, "the scene has no MOVING particles");
    const sphx_params& p = c->params[inst];
    double dv[3] = {0, 0, 0}, vv[3] = {0, 0, 0};
    for (int q = 0; q < c->dim; ++q) {
        if (!std::isfinite(disp[q]) || !std::isfinite(vel[q])) return fail(c, SPHX_E_ARG, "non-finite motion");
        if (p.periodic[q] && (disp[q] != 0.0 || vel[q] != 0.0))
            return fail(c, SPHX_E_ARG, "no motion along the periodic axis %d", q);
        dv[q] = disp[q];
        vv[q] = vel[q];
    }
    // the motion starts from the instance's current time, read from the device
    InstRun r;
    HIP_OK(c, hipStreamSynchronize(c->stream));
    HIP_OK(c, hipMemcpy(&r, c->dev.run + inst, sizeof r, hipMemcpyDeviceToHost));
    InstDev& I = c->inst[inst];
    I.mv_host = 1;
    for (int q = 0; q < 3; ++q) {
        I.mv_disp[q] = dv[q];
        I.mv_vel[q] = vv[q];
    }
    I.mv_t0 = r.t;
    HIP_OK(c, hipMemcpy((void*)(c->dev.inst + inst), &I, sizeof I, hipMemcpyHostToDevice));
    // the particles take the new motion at once, and the next build sorts them where
    // they now are
    launch_place_moving(c->dev, (uint32_t)inst, c->stream);
    if (const sphx_status e = request_rebuild(c)) return e;
    c->rates_valid = false;
    HIP_OK(c, hipGetLastError());
    return SPHX_OK;
}

sphx_status sphx_set_option(sphx_ctx* c, int32_t option, int64_t value)
{
    if (!c) return SPHX_E_ARG;
    switch (option) {
    case SPHX_OPT_DEBUG_TERMS: c->launch.debug_terms = value != 0; break;
    case SPHX_OPT_BLOCK:
        if (value < 64 || value > 256 || value % 64) return fail(c, SPHX_E_ARG, "block must be 64, 128, 192 or 256");
        c->launch.block = (int)value;
        break;
    case SPHX_OPT_XCD_REMAP: {
        const int64_t mag = value < 0 ? -value : value;
        if (mag > 64 || (mag > 1 && (mag & (mag - 1))) || value == -1)
            return fail(c, SPHX_E_ARG, "xcd_remap must be 0, 1, or plus or minus a power of two from 2 to 64");
        c->launch.xcd_remap = (int)value;
        break;
    }
    case SPHX_OPT_LANES:
    case SPHX_OPT_FORCE_LANES:
        if (value != 1 && value != 2 && value != 4) return fail(c, SPHX_E_ARG, "lanes must be 1, 2 or 4");
        (option == SPHX_OPT_LANES ? c->launch.lanes : c->launch.force_lanes) = (int)value;
        break;
    case SPHX_OPT_GRAPH: c->use_graph = value != 0 && c->stream != nullptr; break;
    case SPHX_OPT_ONE_LAUNCH_BUILD: c->launch.one_launch_build = value != 0; break;
    case SPHX_OPT_COLOUR_IN_PREDICT: c->launch.colour_in_predict = value != 0; break;
    case SPHX_OPT_FORCE_STALL:
        if (value < 0 || value > 5) return fail(c, SPHX_E_ARG, "force_stall must be 0..5");
        c->launch.stall_at = (int)value;
        break;
    case SPHX_OPT_PROFILE:
        c->profile = value != 0;
        for (int q = 0; q < SPHX_NPH; ++q) {
            c->phase_ms[q] = 0;
            c->phase_launches[q] = 0;
        }
        break;
    default: return fail(c, SPHX_E_ARG, "unknown option %d", (int)option);
    }
    drop_graphs(c);
    return SPHX_OK;
}

sphx_status sphx_get_option(sphx_ctx* c, int32_t option, int64_t* value)
{
    if (!c || !value) return SPHX_E_ARG;
    switch (option) {
    case SPHX_OPT_DEBUG_TERMS: *value = c->launch.debug_terms; break;
    case SPHX_OPT_BLOCK: *value = c->launch.block; break;
    case SPHX_OPT_XCD_REMAP: *value = c->launch.xcd_remap; break;
    case SPHX_OPT_LANES: *value = c->launch.lanes; break;
    case SPHX_OPT_FORCE_LANES: *value = c->launch.force_lanes; break;
    case SPHX_OPT_GRAPH: *value = c->use_graph; break;
    case SPHX_OPT_ONE_LAUNCH_BUILD: *value = c->launch.one_launch_build; break;
    case SPHX_OPT_COLOUR_IN_PREDICT: *value = c->launch.colour_in_predict; break;
    case SPHX_OPT_FORCE_STALL: *value = c->launch.stall_at; break;
    case SPHX_OPT_PROFILE: *value = c->profile; break;
    default: return fail(c, SPHX_E_ARG, "unknown option %d", (int)option);
    }
    return SPHX_OK;
}

sphx_status sphx_sync(sphx_ctx* c)
{
    if (!c) return SPHX_E_ARG;
    if (!c->bound) return fail(c, SPHX_E_STATE, "no workspace");
    if (const sphx_status st = owns_workspace(c)) return st;
    return status_of(c);
}

sphx_status sphx_get_stats(sphx_ctx* c, sphx_stats* out)
{
    if (!c || !out) return SPHX_E_ARG;
    if (const sphx_status st = owns_workspace(c)) return st;
    if (!c->inited) return fail(c, SPHX_E_STATE, "init_particles first");
    const sphx_status st = status_of(c);
    InstRun r;
    unsigned long long inter = 0;
    HIP_OK(c, hipMemcpy(&r, c->dev.run, sizeof r, hipMemcpyDeviceToHost));
    std::vector<unsigned long long> slots((size_t)kInterSlots * kInterStride);
    HIP_OK(c, hipMemcpy(slots.data(), c->dev.inter, slots.size() * sizeof(unsigned long long), hipMemcpyDeviceToHost));
    for (uint32_t q = 0; q < kInterSlots; ++q) inter += slots[(size_t)q * kInterStride];
    out->steps = r.step;
    out->t = r.t;
    out->dt = r.dt;
    out->interactions = (int64_t)inter;
    out->ncells = c->ncell;
    out->builds = r.builds;
    uint32_t icount = 0;
    HIP_OK(c, hipMemcpy(&icount, c->dev.icount, sizeof icount, hipMemcpyDeviceToHost));
    out->colour_particles = icount;
    uint32_t two = 0;
    HIP_OK(c, hipMemcpy(&two, c->dev.flags + 3, sizeof two, hipMemcpyDeviceToHost));
    out->two_level_builds = two;
    collect_events(c);
    for (int q = 0; q < SPHX_NPH; ++q) {
        out->phase_ms[q] = c->phase_ms[q];
        out->phase_launches[q] = c->phase_launches[q];
    }
    return st;
}

sphx_status sphx_reset_interactions(sphx_ctx* c)
{
    if (!c) return SPHX_E_ARG;
    if (!c->bound) return fail(c, SPHX_E_STATE, "no workspace");
    if (const sphx_status st = owns_workspace(c)) return st;
    HIP_OK(c, hipMemsetAsync(c->dev.inter, 0, sizeof(unsigned long long) * kInterSlots * kInterStride, c->stream));
    return SPHX_OK;
}

sphx_status sphx_get_field(sphx_ctx* c, int32_t field, double* out)
{
    if (!c || !out) return SPHX_E_ARG;
    if (const sphx_status st = have_state(c)) return st;
    const sphx_status st = status_of(c);
    const int64_t n = c->n;
    const bool f32 = c->precision == 1;
    const size_t R = f32 ? 4 : 8;
    const Dev& d = c->dev;
    const int cur = device_cur(c);
    const StateSet& S = d.S[cur];
    const Sorted& O = d.O[cur];
    std::vector<uint32_t> id(n), info(n), key(n);
    HIP_OK(c, hipMemcpy(id.data(), O.id, n * 4, hipMemcpyDeviceToHost));
    HIP_OK(c, hipMemcpy(info.data(), O.info, n * 4, hipMemcpyDeviceToHost));
    HIP_OK(c, hipMemcpy(key.data(), O.key, n * 4, hipMemcpyDeviceToHost));
    auto fetch4 = [&](const void* src, std::vector<double>& v) -> sphx_status {
        std::vector<char> raw(n * 4 * R);
        HIP_OK(c, hipMemcpy(raw.data(), src, raw.size(), hipMemcpyDeviceToHost));
        v.resize(n * 4);
        for (int64_t k = 0; k < 4 * n; ++k) v[k] = f32 ? (double)((float*)raw.data())[k] : ((double*)raw.data())[k];
        return SPHX_OK;
    };
    std::vector<float4> lo;
    auto rho_of = [&](const std::vector<double>& r, int64_t k) {
        if (!f32) return r[4 * k + 3];   // density in aux.w
        const InstDev& I = c->inst[info_inst(info[k])];
        return I.rho0[info_phase(info[k])] + r[4 * k + 3] + (double)lo[k].w;
    };
    std::vector<double> a, b;
    sphx_status e = SPHX_OK;
    switch (field) {
    case SPHX_F_X: {
        if ((e = fetch4(S.pos, a))) return e;
        if (f32) {
            lo.resize(n);
            HIP_OK(c, hipMemcpy(lo.data(), S.plo, n * sizeof(float4), hipMemcpyDeviceToHost));
        }
        for (int64_t k = 0; k < n; ++k) {
            double* o = out + 3 * (size_t)id[k];
            if (!f32) {
                for (int q = 0; q < 3; ++q) o[q] = q < c->dim ? a[4 * k + q] : 0.0;
            } else {
                const InstDev& I = c->inst[info_inst(info[k])];
                uint32_t l = key[k] - I.cell_base;
                int cc[3];
                cc[0] = (int)(l % (uint32_t)I.nc[0]);
                l /= (uint32_t)I.nc[0];
                cc[1] = (int)(l % (uint32_t)I.nc[1]);
                cc[2] = (int)(l / (uint32_t)I.nc[1]);
                const float e3[3] = {lo[k].x, lo[k].y, lo[k].z};
                for (int q = 0; q < 3; ++q)
                    o[q] = q < c->dim ? I.lo[q] + (double)cc[q] * I.cs[q] + a[4 * k + q] + (double)e3[q] : 0.0;
            }
        }
        break;
    }
    case SPHX_F_U: {
        if ((e = fetch4(S.vel, a))) return e;
        std::vector<float4> vl;
        if (f32) {
            vl.resize(n);
            HIP_OK(c, hipMemcpy(vl.data(), S.vlo, n * sizeof(float4), hipMemcpyDeviceToHost));
        }
        for (int64_t k = 0; k < n; ++k) {
            double* o = out + 3 * (size_t)id[k];
            const float e3[3] = {f32 ? vl[k].x : 0.f, f32 ? vl[k].y : 0.f, f32 ? vl[k].z : 0.f};
            for (int q = 0; q < 3; ++q) o[q] = q < c->dim ? a[4 * k + q] + (double)e3[q] : 0.0;
        }
        break;
    }
    case SPHX_F_RHO:
    case SPHX_F_P: {
        if ((e = fetch4(S.aux, a))) return e;
        if (f32) {
            lo.resize(n);
            HIP_OK(c, hipMemcpy(lo.data(), S.plo, n * sizeof(float4), hipMemcpyDeviceToHost));
        }
        for (int64_t k = 0; k < n; ++k) {
            if (field == SPHX_F_RHO) {
                out[id[k]] = rho_of(a, k);
                continue;
            }
            // the pressure the device derived: aux holds (m, m P / rho^2, V, rho or rho - rho0),
            // with rho taken as the device takes it (the FP32 form without its compensation term)
            const InstDev& I = c->inst[info_inst(info[k])];
            const double r = f32 ? I.rho0[info_phase(info[k])] + a[4 * k + 3] : a[4 * k + 3];
            out[id[k]] = a[4 * k + 1] * (r * r) / a[4 * k];
        }
        break;
    }
    case SPHX_F_A:
    case SPHX_F_DRHO:
    case SPHX_F_GRADC: {
        if ((e = fetch4(field == SPHX_F_GRADC ? d.gc : d.acc, a))) return e;
        for (int64_t k = 0; k < n; ++k) {
            if (field == SPHX_F_DRHO) out[id[k]] = a[4 * k + 3];
            else
                for (int q = 0; q < 3; ++q) out[3 * (size_t)id[k] + q] = q < c->dim ? a[4 * k + q] : 0.0;
        }
        break;
    }
    case SPHX_F_AP:
    case SPHX_F_AV:
    case SPHX_F_AS: {
        if (!c->launch.debug_terms) return fail(c, SPHX_E_STATE, "enable SPHX_OPT_DEBUG_TERMS before compute_forces");
        std::vector<char> raw(n * 12 * R);
        HIP_OK(c, hipMemcpy(raw.data(), d.terms, raw.size(), hipMemcpyDeviceToHost));
        const int t = field - SPHX_F_AP;
        for (int64_t k = 0; k < n; ++k)
            for (int q = 0; q < 3; ++q) {
                const size_t at = (size_t)(3 * k + t) * 4 + q;
                out[3 * (size_t)id[k] + q] = q < c->dim ? (f32 ? (double)((float*)raw.data())[at] : ((double*)raw.data())[at]) : 0.0;
            }
        break;
    }
    default: return fail(c, SPHX_E_ARG, "unknown field %d", (int)field);
    }
    (void)b;
    return st;
}

sphx_status sphx_get_neighbors(sphx_ctx* c, int64_t* off, int32_t* ids, int64_t cap, int64_t* need)
{
    if (!c || !off || !need) return SPHX_E_ARG;
    if (const sphx_status st = have_state(c)) return st;
    enqueue_build(c);
    const int cur = device_cur(c);
    const int64_t n = c->n;
    uint32_t *dcnt = nullptr, *doff = nullptr, *dids = nullptr;
    HIP_OK(c, hipMalloc(&dcnt, n * 4));
    launch_export(c->dev, 0, nullptr, dcnt, c->launch, c->stream);
    std::vector<uint32_t> cnt(n), id(n);
    hipError_t e = hipMemcpyAsync(cnt.data(), dcnt, n * 4, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(id.data(), c->dev.O[cur].id, n * 4, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) {
        (void)hipFree(dcnt);
        return fail(c, SPHX_E_HIP, "neighbour count: %s", hipGetErrorString(e));
    }
    std::vector<uint32_t> soff(n + 1, 0);
    for (int64_t k = 0; k < n; ++k) soff[k + 1] = soff[k] + cnt[k];
    const int64_t total = soff[n];
    // per original id
    std::vector<int64_t> ocnt(n);
    for (int64_t k = 0; k < n; ++k) ocnt[id[k]] = cnt[k];
    off[0] = 0;
    for (int64_t i = 0; i < n; ++i) off[i + 1] = off[i] + ocnt[i];
    *need = total;
    if (!ids || cap < total) {
        (void)hipFree(dcnt);
        return SPHX_OK;
    }
    std::vector<uint32_t> sids(total > 0 ? total : 1);
    e = hipMalloc(&doff, (n + 1) * 4);
    if (e == hipSuccess) e = hipMalloc(&dids, (total > 0 ? total : 1) * 4);
    if (e == hipSuccess) e = hipMemcpyAsync(doff, soff.data(), (n + 1) * 4, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) {
        launch_export(c->dev, 1, doff, dids, c->launch, c->stream);
        e = hipMemcpyAsync(sids.data(), dids, total * 4, hipMemcpyDeviceToHost, c->stream);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    (void)hipFree(dcnt);
    if (doff) (void)hipFree(doff);
    if (dids) (void)hipFree(dids);
    if (e != hipSuccess) return fail(c, SPHX_E_HIP, "neighbour export: %s", hipGetErrorString(e));
    for (int64_t k = 0; k < n; ++k) {
        int32_t* dst = ids + off[id[k]];
        for (uint32_t q = 0; q < cnt[k]; ++q) dst[q] = (int32_t)sids[soff[k] + q];
        std::sort(dst, dst + cnt[k]);
    }
    return status_of(c);
}


sphx_status sphx_get_state(sphx_ctx* c, void* blob, size_t cap, size_t* need)
{
    if (!c || !need) return SPHX_E_ARG;
    if (const sphx_status st = have_state(c)) return st;
    const int cur = device_cur(c);
    auto spans = state_spans(c, cur);
    size_t total = sizeof(BlobHeader);
    for (auto& s : spans) total += s.bytes;
    *need = total;
    if (!blob || cap < total) return SPHX_OK;
    const sphx_status st = status_of(c);
    uint32_t qpos = 0;
    HIP_OK(c, hipMemcpy(&qpos, c->dev.flags + 2, sizeof qpos, hipMemcpyDeviceToHost));
    BlobHeader h{kMagic, c->precision, c->dim, c->ninst, cur, c->n, c->ncell, (uint32_t)c->rates_valid,
                 c->dev.cap, qpos};
    char* p = (char*)blob;
    std::memcpy(p, &h, sizeof h);
    p += sizeof h;
    for (auto& s : spans) {
        HIP_OK(c, hipMemcpy(p, s.p, s.bytes, hipMemcpyDeviceToHost));
        p += s.bytes;
    }
    return st;
}

sphx_status sphx_set_state(sphx_ctx* c, const void* blob, size_t bytes)
{
    if (!c || !blob) return SPHX_E_ARG;
    if (const sphx_status st = owns_workspace(c)) return st;
    if (!c->inited) return fail(c, SPHX_E_STATE, "init_particles first (same scene layout)");
    BlobHeader h;
    if (bytes < sizeof h) return fail(c, SPHX_E_ARG, "blob too small");
    std::memcpy(&h, blob, sizeof h);
    if (h.magic != kMagic || h.precision != c->precision || h.dim != c->dim || h.ninst != c->ninst || h.n != c->n ||
        h.ncell != c->ncell || h.cap != c->dev.cap || (h.cur != 0 && h.cur != 1))
        return fail(c, SPHX_E_ARG, "blob does not match this context");
    auto spans = state_spans(c, h.cur);
    size_t total = sizeof h;
    for (auto& s : spans) total += s.bytes;
    if (bytes != total) return fail(c, SPHX_E_ARG, "blob size mismatch");
    HIP_OK(c, hipStreamSynchronize(c->stream));
    const char* p = (const char*)blob + sizeof h;
    // the mass table of the blob's particles: aux (third span) holds m in x, info (sixth)
    // the instance and phase
    {
        const bool f32 = c->precision == 1;
        const char* aux = p + spans[0].bytes + spans[1].bytes;
        const char* inf = aux + spans[2].bytes + spans[3].bytes + spans[4].bytes;
        auto info_at = [&](int64_t i) {
            uint32_t f;
            std::memcpy(&f, inf + 4 * (size_t)i, 4);
            return f;
        };
        for (int64_t i = 0; i < c->n; ++i) {
            const uint32_t f = info_at(i);
            if (info_inst(f) >= (uint32_t)c->ninst || info_phase(f) >= (uint32_t)c->nphase)
                return fail(c, SPHX_E_ARG, "blob: particle %lld has a bad instance or phase", (long long)i);
        }
        // every index the kernels follow must stay in range
        std::vector<const char*> at(spans.size());
        const char* q = p;
        for (size_t k = 0; k < spans.size(); ++k) {
            at[k] = q;
            q += spans[k].bytes;
        }
        auto u32 = [](const char* base, size_t i) {
            uint32_t v;
            std::memcpy(&v, base + 4 * i, 4);
            return v;
        };
        const uint32_t n = (uint32_t)c->n, nc = c->ncell, cap = c->dev.cap;
        const char *key = at[3], *id = at[4], *cst = at[6], *nbl = at[10], *nbc = at[11], *il = at[12];
        for (uint32_t i = 0; i < n; ++i) {
            const InstDev& I = c->inst[info_inst(info_at(i))];
            const uint32_t k = u32(key, i);
            if (k < I.cell_base || k >= I.cell_base + I.ncell || u32(id, i) >= n)
                return fail(c, SPHX_E_ARG, "blob: particle %u has a bad cell key or id", i);
        }
        if (u32(cst, 0) != 0 || u32(cst, nc) != n)
            return fail(c, SPHX_E_ARG, "blob: cell table does not span the particles");
        for (uint32_t k = 0; k < nc; ++k)
            if (u32(cst, k + 1) < u32(cst, k)) return fail(c, SPHX_E_ARG, "blob: cell table not ascending");
        for (uint32_t i = 0; i < n; ++i) {
            // entries below the count name particles; the padding after them, which the
            // walks also read, names at most the sentinel record n
            const uint32_t cnt = u32(nbc, i);
            const uint32_t m = std::min(cnt, cap);
            const uint32_t padded = cnt <= cap ? std::min((cnt + kListPad - 1u) & ~(kListPad - 1u), cap) : cap;
            for (uint32_t e = 0; e < padded; ++e)
                if ((u32(nbl, (size_t)e * c->dev.lstride + i) & kIdxMask) >= (e < m ? n : n + 1))
                    return fail(c, SPHX_E_ARG, "blob: neighbour list of particle %u out of range", i);
        }
        const uint32_t ni = u32(at[13], 0);
        if (ni > n) return fail(c, SPHX_E_ARG, "blob: colour-pass count out of range");
        for (uint32_t e = 0; e < ni; ++e)
            if (u32(il, e) >= n) return fail(c, SPHX_E_ARG, "blob: colour-pass index out of range");
        mass_table(c, c->n, [&](int64_t i, uint32_t& b, uint32_t& q, double& mi) {
            const uint32_t f = info_at(i);
            b = info_inst(f);
            q = info_phase(f);
            if (f32) {
                float v;
                std::memcpy(&v, aux + 16 * (size_t)i, 4);
                mi = v;
            } else {
                std::memcpy(&mi, aux + 32 * (size_t)i, 8);
            }
        });
    }
    for (auto& s : spans) {
        HIP_OK(c, hipMemcpy(s.p, p, s.bytes, hipMemcpyHostToDevice));
        p += s.bytes;
    }
    HIP_OK(c, hipMemcpy((void*)c->dev.inst, c->inst.data(), sizeof(InstDev) * c->ninst, hipMemcpyHostToDevice));
    const int cur = h.cur;
    const uint32_t flags[3] = {0u, 0u, h.qpos ? 1u : 0u};
    HIP_OK(c, hipMemcpy(c->dev.curp, &cur, sizeof cur, hipMemcpyHostToDevice));
    HIP_OK(c, hipMemcpy(c->dev.flags, flags, sizeof flags, hipMemcpyHostToDevice));
    HIP_OK(c, hipMemset(c->dev.cnt, 0, (size_t)c->ncell * 4));
    // errors still pending belong to the state this call replaced
    HIP_OK(c, hipMemset(c->dev.status, 0, sizeof(uint32_t)));
    HIP_OK(c, hipMemset(c->dev.fault, 0, sizeof(FaultRec)));
    const Sorted& other = c->dev.O[1 - cur];   // valid (if stale) for a build that stops part-way
    HIP_OK(c, hipMemset(other.key, 0, (size_t)c->n * 4));
    HIP_OK(c, hipMemset(other.id, 0, (size_t)c->n * 4));
    HIP_OK(c, hipMemset(other.info, 0, (size_t)c->n * 4));
    c->rates_valid = h.rates_valid != 0;
    return SPHX_OK;
}

} // extern "C"
