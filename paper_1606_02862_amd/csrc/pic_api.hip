// Host side of the C ABI declared in include/pic.h: argument validation,
// device memory, kernel orchestration on the handle's stream, diagnostics and
// state transfer.  No exception crosses the ABI.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <limits>
#include <string>
#include <type_traits>
#include <vector>

#include "ionize_internal.hpp"

using namespace pic;

struct pic_ctx {
    pic_grid_t grid{};
    int order = 1;
    int nsp = 0;
    Species sp[PIC_MAX_SPECIES];
    GridView g{};          // geometry always; FP32 field pointers in FP32 mode
    GridView64 g64{};      // FP64 mode: geometry and field pointers
    bool fp64 = false;
    DiagBuffers diag{};
    hipStream_t stream = nullptr;
    pic_alloc_t alloc{};
    bool use_cb = false;
    std::vector<void*> owned;
    int32_t* flags_host = nullptr;  // pinned
    int device = 0;                 // current device at pic_init
    int64_t step = 0;
    bool rho_prev_valid = false;    // diag.rho_prev holds rho before the last cycle (PIC_OPT_CONTINUITY)
    std::string err;
    // timing
    bool timing = false;
    pic_timing_t tacc{};
    std::vector<hipEvent_t> ev;
    int ev_used = 0;
    int64_t pending_particles = 0;
    int pending_launches = 0;
    // ionisation
    double* gl = nullptr;                    // 64 nodes then 64 weights
    double* ne = nullptr;                    // per-cell n_e (cm^-3)
    double* kT = nullptr;                    // per-cell kT_e (eV)
    double* mom4 = nullptr;                  // per-cell sum w and mean u (energy loss)
    double* de = nullptr;                    // per-cell ionisation energy to pay (energy loss)
    int32_t* old_count = nullptr;            // per-supercell electron count before the appends
    double* nu[PIC_MAX_SPECIES] = {};        // per ion slot rate (1/s)
    double* rtab[PIC_MAX_SPECIES] = {};      // tabulated subshell sums (PIC_RATE_TABLE), built at first use
    bool rtab_ready[PIC_MAX_SPECIES] = {};
    unsigned long long* fbl[PIC_MAX_SPECIES] = {};  // per ion slot: surrogate fallback list
    unsigned long long* counters = nullptr;  // CNT_WORDS ionisation counters (fallback list, striped active / ionised)
    hipEvent_t iev[4] = {};
    // surrogate per ion species
    struct Mlp {
        float* params = nullptr;
        float* m = nullptr;
        float* v = nullptr;
        float* grad = nullptr;   // a summed gradient (pic_mlp_loss_grad)
        float* part = nullptr;   // a training step's per-workgroup gradient rows
        double* lpart = nullptr; // and squared-error sums
        double mu = 0.0, s = 1.0;
        double t_min = 1.0, t_max = 1e4, n_min = 1e19, n_max = 1e23;
        int act = PIC_MLP_SILU;
        bool ready = false;
    } mlp[PIC_MAX_SPECIES];
};

static thread_local std::string g_init_error;

namespace {

int fail(pic_ctx* c, int code, const char* fmt, ...) __attribute__((format(printf, 3, 4)));
int fail(pic_ctx* c, int code, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (c) c->err = buf;
    else g_init_error = buf;
    return code;
}

#define HIPCHK(ctx, expr)                                                                              \
    do {                                                                                               \
        hipError_t e_ = (expr);                                                                        \
        if (e_ != hipSuccess) return fail((ctx), PIC_ERR_HIP, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

void* dev_alloc(pic_ctx* c, size_t bytes)
{
    if (bytes == 0) bytes = 256;
    bytes = (bytes + 255) & ~(size_t)255;
    void* p = nullptr;
    if (c->use_cb) {
        p = c->alloc.alloc(bytes, c->alloc.user);
        if (p && ((uintptr_t)p & 255)) {  // the kernels' vector accesses rely on the alignment
            c->alloc.free(p, c->alloc.user);
            p = nullptr;
        }
    } else if (hipMalloc(&p, bytes) != hipSuccess) {
        p = nullptr;
    }
    if (p) c->owned.push_back(p);
    return p;
}

void dev_free(pic_ctx* c, void* p)
{
    if (!p) return;
    for (size_t i = 0; i < c->owned.size(); ++i)
        if (c->owned[i] == p) {
            c->owned[i] = c->owned.back();
            c->owned.pop_back();
            break;
        }
    if (c->use_cb) c->alloc.free(p, c->alloc.user);
    else (void)hipFree(p);
}

void release_all(pic_ctx* c)
{
    for (void* p : c->owned) {
        if (c->use_cb) c->alloc.free(p, c->alloc.user);
        else (void)hipFree(p);
    }
    c->owned.clear();
    for (hipEvent_t e : c->ev) (void)hipEventDestroy(e);
    c->ev.clear();
    for (hipEvent_t& e : c->iev)
        if (e) { (void)hipEventDestroy(e); e = nullptr; }
    if (c->flags_host) (void)hipHostFree(c->flags_host);
    c->flags_host = nullptr;
}

bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

int validate(const pic_grid_t* g, const pic_species_t* sp, int n, pic_shape_t shape)
{
    if (!g || !sp) return fail(nullptr, PIC_ERR_ARG, "grid and species must not be NULL");
    if (g->nx <= 0 || g->ny <= 0 || g->nz <= 0 || g->nx % SX || g->ny % SY || g->nz % SZ)
        return fail(nullptr, PIC_ERR_ARG, "grid %dx%dx%d is not a positive multiple of the %dx%dx%d supercell", g->nx,
                    g->ny, g->nz, SX, SY, SZ);
    const double ncell = (double)g->nx * g->ny * g->nz;
    if (3.0 * ncell >= 2147483647.0) return fail(nullptr, PIC_ERR_ARG, "grid too large (3 N must fit in int32)");
    if (!finite_pos(g->dx) || !finite_pos(g->dy) || !finite_pos(g->dz) || !finite_pos(g->dt))
        return fail(nullptr, PIC_ERR_ARG, "dx, dy, dz, dt must be positive and finite");
    const double courant = g->dt * std::sqrt(1.0 / (g->dx * g->dx) + 1.0 / (g->dy * g->dy) + 1.0 / (g->dz * g->dz));
    if (!(courant < 1.0)) return fail(nullptr, PIC_ERR_ARG, "time step violates the Courant limit (%.4f >= 1)", courant);
    for (int d = 0; d < 3; ++d)
        if (!std::isfinite(g->b0[d])) return fail(nullptr, PIC_ERR_ARG, "b0 must be finite");
    if (!std::isfinite(g->rho_bg)) return fail(nullptr, PIC_ERR_ARG, "rho_bg must be finite");
    if (shape != PIC_SHAPE_CIC && shape != PIC_SHAPE_TSC && shape != PIC_SHAPE_PCS)
        return fail(nullptr, PIC_ERR_ARG, "unknown shape %d", (int)shape);
    if (g->precision != PIC_PRECISION_FP32 && g->precision != PIC_PRECISION_FP64)
        return fail(nullptr, PIC_ERR_ARG, "unknown precision %d", (int)g->precision);
    if (g->gather != PIC_GATHER_STANDARD && g->gather != PIC_GATHER_GALERKIN)
        return fail(nullptr, PIC_ERR_ARG, "unknown gather %d", (int)g->gather);
    if (g->options & ~(PIC_OPT_DETERMINISTIC_J | PIC_OPT_CONTINUITY))
        return fail(nullptr, PIC_ERR_ARG, "unknown options 0x%x", (unsigned)g->options);
    if ((g->options & PIC_OPT_DETERMINISTIC_J) && g->precision != PIC_PRECISION_FP32)
        return fail(nullptr, PIC_ERR_ARG, "PIC_OPT_DETERMINISTIC_J needs FP32 (the FP64 tile sums are floating point)");
    if (n < 1 || n > PIC_MAX_SPECIES) return fail(nullptr, PIC_ERR_ARG, "n_species must be in 1..%d", PIC_MAX_SPECIES);
    double ids = 0.0;
    for (int s = 0; s < n; ++s) {
        const pic_species_t& p = sp[s];
        if (!finite_pos(p.mass)) return fail(nullptr, PIC_ERR_ARG, "species %d: mass must be positive", s);
        if (!std::isfinite(p.charge)) return fail(nullptr, PIC_ERR_ARG, "species %d: charge must be finite", s);
        if (p.ppc < 0 || p.ppc > 4096) return fail(nullptr, PIC_ERR_ARG, "species %d: ppc out of range", s);
        if (!(p.density >= 0.0) || !std::isfinite(p.density)) return fail(nullptr, PIC_ERR_ARG, "species %d: density", s);
        if (!(p.u_th >= 0.0) || !std::isfinite(p.u_th)) return fail(nullptr, PIC_ERR_ARG, "species %d: u_th", s);
        const double b2 = p.drift_beta[0] * p.drift_beta[0] + p.drift_beta[1] * p.drift_beta[1] +
                          p.drift_beta[2] * p.drift_beta[2];
        if (!(b2 < 1.0)) return fail(nullptr, PIC_ERR_ARG, "species %d: |drift_beta| must be < 1", s);
        if (p.layout < PIC_LAYOUT_UNIFORM || p.layout > PIC_LAYOUT_BEAMS)
            return fail(nullptr, PIC_ERR_ARG, "species %d: unknown layout", s);
        if (p.coincident_with >= 0) {
            const int t = p.coincident_with;
            if (t >= n || t == s) return fail(nullptr, PIC_ERR_ARG, "species %d: bad coincident_with", s);
            if (sp[t].coincident_with >= 0) return fail(nullptr, PIC_ERR_ARG, "species %d: coincident target must place itself", s);
            if (sp[t].ppc < p.ppc) return fail(nullptr, PIC_ERR_ARG, "species %d: coincident target has fewer ppc", s);
        } else if (p.coincident_with != -1) {
            return fail(nullptr, PIC_ERR_ARG, "species %d: coincident_with must be -1 or a species index", s);
        }
        if (p.z_max < 0 || p.z_max > PIC_MAX_ZSTATES - 1) return fail(nullptr, PIC_ERR_ARG, "species %d: z_max", s);
        if (p.z_max > 0) {
            if (p.z_init < 0 || p.z_init > p.z_max) return fail(nullptr, PIC_ERR_ARG, "species %d: z_init", s);
            for (int z = 0; z < p.z_max; ++z) {
                if (!finite_pos(p.ionization_ev[z]))
                    return fail(nullptr, PIC_ERR_ARG, "species %d: ionisation data of state %d", s, z);
                const pic_lotz_shell_t* L = p.lotz[z];
                if (L[0].q <= 0 || L[0].p_ev != p.ionization_ev[z])
                    return fail(nullptr, PIC_ERR_ARG,
                                "species %d: lotz subshell 0 of state %d must have q > 0 and p_ev = ionization_ev", s, z);
                bool end = false;
                for (int j = 0; j < PIC_LOTZ_SHELLS; ++j) {
                    if (L[j].q < 0) return fail(nullptr, PIC_ERR_ARG, "species %d: lotz q < 0 (state %d)", s, z);
                    if (L[j].q == 0) { end = true; continue; }
                    if (end) return fail(nullptr, PIC_ERR_ARG, "species %d: lotz subshell after an unused slot (state %d)", s, z);
                    if (!(L[j].p_ev >= p.ionization_ev[z]) || !std::isfinite(L[j].p_ev) || !finite_pos(L[j].a) ||
                        !(L[j].b >= 0.0 && L[j].b <= 1.0) || !(L[j].c >= 0.0 && std::isfinite(L[j].c)))
                        return fail(nullptr, PIC_ERR_ARG, "species %d: lotz subshell %d of state %d (p_ev, a, b, c)", s, j, z);
                }
            }
            if (p.max_events < 0 || p.max_events > PIC_MAX_ZSTATES)
                return fail(nullptr, PIC_ERR_ARG, "species %d: max_events", s);
            if (p.energy_loss != 0 && p.energy_loss != 1) return fail(nullptr, PIC_ERR_ARG, "species %d: energy_loss", s);
        }
        if (p.ionize_into != -1) {
            if (p.ionize_into < 0 || p.ionize_into >= n || p.ionize_into == s || p.z_max == 0)
                return fail(nullptr, PIC_ERR_ARG, "species %d: bad ionize_into", s);
            if (g->precision == PIC_PRECISION_FP64)
                return fail(nullptr, PIC_ERR_ARG, "species %d: ionisation runs in FP32 only", s);
            if (sp[p.ionize_into].z_max != 0) return fail(nullptr, PIC_ERR_ARG, "species %d: ionize_into target has charge states", s);
        }
        if (p.cap_ppc < 0 || p.cap_ppc > 8192) return fail(nullptr, PIC_ERR_ARG, "species %d: cap_ppc", s);
        if (p.cap_ppc > 0 && p.cap_ppc < p.ppc) return fail(nullptr, PIC_ERR_ARG, "species %d: cap_ppc < ppc", s);
        ids += ncell * p.ppc;
        if (p.z_max > 0 && p.ionize_into >= 0) ids += ncell * p.ppc * p.z_max;
    }
    if (ids >= 4294967295.0) return fail(nullptr, PIC_ERR_ARG, "particle ids would not fit in 32 bits");
    return PIC_OK;
}

// Frames and arrival lists of the real arrays of one species, in R.
template <class R>
int alloc_real_arrays(pic_ctx* c, int s, SpeciesViewT<R>& v, size_t n, size_t ni)
{
    R** fl[] = {&v.x, &v.y, &v.z, &v.ux, &v.uy, &v.uz, &v.w};
    for (R** f : fl)
        if (!(*f = (R*)dev_alloc(c, n * sizeof(R)))) return fail(c, PIC_ERR_OOM, "species %d: frames", s);
    R** fi[] = {&v.ix, &v.iy, &v.iz, &v.iux, &v.iuy, &v.iuz, &v.iw};
    for (R** f : fi)
        if (!(*f = (R*)dev_alloc(c, ni * sizeof(R)))) return fail(c, PIC_ERR_OOM, "species %d: arrivals", s);
    return PIC_OK;
}

template <class R> GridViewT<R>& gview(pic_ctx* c);
template <> GridView& gview<float>(pic_ctx* c) { return c->g; }
template <> GridView64& gview<double>(pic_ctx* c) { return c->g64; }
template <class R> SpeciesViewT<R>& sview(pic_ctx* c, int s);
template <> SpeciesView& sview<float>(pic_ctx* c, int s) { return c->sp[s].v; }
template <> SpeciesView64& sview<double>(pic_ctx* c, int s) { return c->sp[s].v64; }

int alloc_species(pic_ctx* c, int s)
{
    Species& S = c->sp[s];
    SpeciesView& v = S.v;
    const pic_species_t& d = S.desc;
    const int nsc = c->g.nsc;
    int cap_ppc = d.cap_ppc > 0 ? d.cap_ppc : (d.ppc * 3 + 1) / 2;
    if (cap_ppc < 1) cap_ppc = 1;
    if (c->order >= 2) cap_ppc += cap_ppc & 1;  // whole 512-particle frames per supercell
    v.cap = cap_ppc * SC_CELLS;
    int cap_in = v.cap / 4;
    cap_in = std::max(cap_in, 256);
    cap_in = std::min(cap_in, c->order == 1 ? 2048 : MAX_MIGRATE);  // what the particle kernel's LDS can absorb
    v.cap_in = cap_in;
    const size_t n = (size_t)nsc * v.cap, ni = (size_t)2 * nsc * cap_in;  // two step parities
    const int rc = c->fp64 ? alloc_real_arrays(c, s, S.v64, n, ni) : alloc_real_arrays(c, s, v, n, ni);
    if (rc) return rc;
    if (!(v.id = (uint32_t*)dev_alloc(c, n * 4))) return fail(c, PIC_ERR_OOM, "species %d: ids", s);
    v.zs = nullptr;
    v.izs = nullptr;
    if (d.z_max > 0) {
        if (!(v.zs = (uint8_t*)dev_alloc(c, n))) return fail(c, PIC_ERR_OOM, "species %d: charge states", s);
        if (!(v.izs = (uint8_t*)dev_alloc(c, ni))) return fail(c, PIC_ERR_OOM, "species %d: arrivals", s);
    }
    if (!(v.iid = (uint32_t*)dev_alloc(c, ni * 4))) return fail(c, PIC_ERR_OOM, "species %d: arrivals", s);
    if (!(v.holes = (int32_t*)dev_alloc(c, ni * 4))) return fail(c, PIC_ERR_OOM, "species %d: holes", s);
    if (!(v.count = (int32_t*)dev_alloc(c, (size_t)nsc * 4))) return fail(c, PIC_ERR_OOM, "species %d: counts", s);
    if (!(v.in_count = (int32_t*)dev_alloc(c, (size_t)2 * nsc * 4))) return fail(c, PIC_ERR_OOM, "species %d: counts", s);
    if (!(v.hole_count = (int32_t*)dev_alloc(c, (size_t)nsc * 4))) return fail(c, PIC_ERR_OOM, "species %d: counts", s);
    v.charge = (float)d.charge;
    v.mass = (float)d.mass;
    // the FP64 view shares every integer array and size
    SpeciesView64& w = S.v64;
    w.id = v.id; w.zs = v.zs; w.count = v.count; w.cap = v.cap;
    w.iid = v.iid; w.izs = v.izs; w.in_count = v.in_count; w.holes = v.holes; w.hole_count = v.hole_count;
    w.cap_in = v.cap_in;
    w.charge = d.charge;
    w.mass = d.mass;
    HIPCHK(c, launch_zero_i32(v.count, nsc, c->stream));
    HIPCHK(c, launch_zero_i32(v.in_count, 2 * nsc, c->stream));
    HIPCHK(c, launch_zero_i32(v.hole_count, nsc, c->stream));
    return PIC_OK;
}

bool ionising(const pic_ctx* c, int s)
{
    return c->sp[s].desc.z_max > 0 && c->sp[s].desc.ionize_into >= 0;
}

int alloc_ionisation(pic_ctx* c)
{
    bool any = false;
    for (int s = 0; s < c->nsp; ++s) any = any || (c->sp[s].desc.z_max > 0);
    if (!any) return PIC_OK;
    const int64_t N = (int64_t)c->grid.nx * c->grid.ny * c->grid.nz;
    if (!(c->gl = (double*)dev_alloc(c, 2 * GL_NODES * 8)) || !(c->ne = (double*)dev_alloc(c, N * 8)) ||
        !(c->kT = (double*)dev_alloc(c, N * 8)) || !(c->counters = (unsigned long long*)dev_alloc(c, CNT_WORDS * 8)))
        return fail(c, PIC_ERR_OOM, "device allocation of ionisation buffers failed");
    for (int s = 0; s < c->nsp; ++s) {
        if (c->sp[s].desc.z_max == 0) continue;
        if (!(c->nu[s] = (double*)dev_alloc(c, (size_t)c->g.nsc * c->sp[s].v.cap * 8)) ||
            !(c->rtab[s] = (double*)dev_alloc(c, (size_t)PIC_MAX_ZSTATES * RATE_TABLE_N * 8)) ||
            !(c->fbl[s] = (unsigned long long*)dev_alloc(c, (size_t)c->g.nsc * c->sp[s].v.cap * 8)))
            return fail(c, PIC_ERR_OOM, "device allocation of ionisation rates failed");
        pic_ctx::Mlp& m = c->mlp[s];
        if (!(m.params = (float*)dev_alloc(c, PIC_MLP_NPARAM * 4)) || !(m.m = (float*)dev_alloc(c, PIC_MLP_NPARAM * 4)) ||
            !(m.v = (float*)dev_alloc(c, PIC_MLP_NPARAM * 4)) || !(m.grad = (float*)dev_alloc(c, PIC_MLP_NPARAM * 4)) ||
            !(m.part = (float*)dev_alloc(c, (size_t)MLP_PART_ROWS * MLP_PART_STRIDE * 4)) ||
            !(m.lpart = (double*)dev_alloc(c, (size_t)MLP_PART_ROWS * 8)))
            return fail(c, PIC_ERR_OOM, "device allocation of the surrogate failed");
        HIPCHK(c, launch_zero_f32(m.grad, PIC_MLP_NPARAM, c->stream));
        if (c->sp[s].desc.energy_loss && !c->de) {
            if (!(c->mom4 = (double*)dev_alloc(c, N * 4 * 8)) || !(c->de = (double*)dev_alloc(c, N * 8)) ||
                !(c->old_count = (int32_t*)dev_alloc(c, (size_t)c->g.nsc * 4)))
                return fail(c, PIC_ERR_OOM, "device allocation of energy-loss buffers failed");
        }
    }
    const double* w;
    const double* x = gauss_laguerre_nodes(&w);
    double rule[2 * GL_NODES];
    for (int k = 0; k < GL_NODES; ++k) { rule[k] = x[k]; rule[GL_NODES + k] = w[k]; }
    HIPCHK(c, hipMemcpyAsync(c->gl, rule, sizeof rule, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    for (hipEvent_t& e : c->iev) HIPCHK(c, hipEventCreate(&e));
    return PIC_OK;
}

IonTables ion_tables(const pic_ctx* c, int s)
{
    IonTables t{};
    const pic_species_t& d = c->sp[s].desc;
    for (int z = 0; z < PIC_MAX_ZSTATES; ++z) {
        t.P[z] = z < d.z_max ? d.ionization_ev[z] : 1.0;
        for (int j = 0; j < PIC_LOTZ_SHELLS; ++j) {
            const pic_lotz_shell_t& L = d.lotz[z][j];
            const bool used = z < d.z_max && L.q > 0;
            t.sp[z][j] = used ? L.p_ev : 1.0;
            t.aq[z][j] = used ? L.a * L.q : 0.0;
            t.sb[z][j] = used ? L.b : 0.0;
            t.sc[z][j] = used ? L.c : 0.0;
            if (used) t.ns[z] = j + 1;
        }
    }
    t.z_max = d.z_max;
    return t;
}

// Build the species' rate table on the handle's stream at its first use.
int ensure_rate_table(pic_ctx* c, int s)
{
    if (c->rtab_ready[s]) return PIC_OK;
    HIPCHK(c, launch_rate_table_build(ion_tables(c, s), c->gl, c->rtab[s], c->stream));
    c->rtab_ready[s] = true;
    return PIC_OK;
}

MlpLaunch mlp_launch(const pic_ctx* c, int s)
{
    const pic_ctx::Mlp& m = c->mlp[s];
    return MlpLaunch{m.params, m.mu, m.s, m.t_min, m.t_max, m.n_min, m.n_max, m.act};
}

// Plasma frequency (1/s) of the reference density, SI.
double omega_p(double n_ref_cm3)
{
    const double e = 1.602176634e-19, eps0 = 8.8541878128e-12, me = 9.1093837015e-31;
    return std::sqrt(n_ref_cm3 * 1e6 * e * e / (eps0 * me));
}

int read_flags(pic_ctx* c)
{
    HIPCHK(c, hipMemcpyAsync(c->flags_host, c->g.flags, NFLAGS * sizeof(int32_t), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    int32_t f[NFLAGS];
    std::memcpy(f, c->flags_host, sizeof f);
    if (f[FLAG_CAPACITY] || f[FLAG_MIGRATE] || f[FLAG_CFL] || f[FLAG_NONFINITE]) {
        HIPCHK(c, launch_zero_i32(c->g.flags, NFLAGS, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        if (f[FLAG_CAPACITY]) return fail(c, PIC_ERR_CAPACITY, "a supercell's frames overflowed");
        if (f[FLAG_MIGRATE]) return fail(c, PIC_ERR_CAPACITY, "a supercell's migration buffer overflowed");
        if (f[FLAG_CFL]) return fail(c, PIC_ERR_CFL, "a particle moved one cell or more in one step (or went non-finite)");
        return fail(c, PIC_ERR_NONFINITE, "non-finite value");
    }
    return PIC_OK;
}

template <class R>
int mark_reference_t(pic_ctx* c)
{
    const int64_t N = (int64_t)c->grid.nx * c->grid.ny * c->grid.nz;
    HIPCHK(c, launch_zero_f64(c->diag.rho, N, c->stream));
    for (int s = 0; s < c->nsp; ++s)
        HIPCHK(c, launch_rho_deposit<R>(gview<R>(c), sview<R>(c, s), c->order, c->diag.rho, c->stream));
    HIPCHK(c, launch_gauss<R>(gview<R>(c), c->diag, c->grid.rho_bg, 0, false, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return PIC_OK;
}

int mark_reference(pic_ctx* c) { return c->fp64 ? mark_reference_t<double>(c) : mark_reference_t<float>(c); }

hipEvent_t next_event(pic_ctx* c)
{
    if (c->ev_used == (int)c->ev.size()) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        c->ev.push_back(e);
    }
    return c->ev[c->ev_used++];
}

int collect_timing(pic_ctx* c)
{
    if (c->ev_used == 0) return PIC_OK;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    for (int i = 0; i + 3 < c->ev_used; i += 4) {
        float a = 0, b = 0, d = 0;
        HIPCHK(c, hipEventElapsedTime(&a, c->ev[i], c->ev[i + 1]));
        HIPCHK(c, hipEventElapsedTime(&b, c->ev[i + 1], c->ev[i + 2]));
        HIPCHK(c, hipEventElapsedTime(&d, c->ev[i + 2], c->ev[i + 3]));
        c->tacc.push_ms += a;
        c->tacc.migrate_ms += b;
        c->tacc.field_ms += d;
    }
    c->tacc.push_launches += c->pending_launches;
    c->tacc.push_particles += c->pending_particles;
    c->pending_launches = 0;
    c->pending_particles = 0;
    c->ev_used = 0;
    return PIC_OK;
}

// Bound of one particle's current contribution, |q w| max(dx, dy, dz) / (dV dt).
double push_vmax(const pic_ctx* c, int s)
{
    const Species& S = c->sp[s];
    const pic_grid_t& g = c->grid;
    const double qmax = std::fabs(S.desc.charge) * (S.desc.z_max > 0 ? S.desc.z_max : 1);
    const double dmax = std::max(g.dx, std::max(g.dy, g.dz));
    return qmax * S.wmax * dmax / (g.dx * g.dy * g.dz * g.dt);
}

int64_t host_count(pic_ctx* c, int s, std::vector<int32_t>& counts)
{
    counts.resize(c->g.nsc);
    if (hipMemcpyAsync(counts.data(), c->sp[s].v.count, counts.size() * 4, hipMemcpyDeviceToHost, c->stream) != hipSuccess)
        return -1;
    if (hipStreamSynchronize(c->stream) != hipSuccess) return -1;
    int64_t t = 0;
    for (int32_t v : counts) t += v;
    return t;
}

// Particle and field transfers, templated on the device real type R and the
// host view (FP32 or FP64 momenta and weights).
template <class R, class V>
int get_particles_t(pic_ctx* c, int s, V* v)
{
    using U = typename std::remove_pointer<decltype(v->ux)>::type;
    const SpeciesViewT<R>& sv = sview<R>(c, s);
    std::vector<int32_t> cnt;
    const int64_t total = host_count(c, s, cnt);
    if (total < 0) return fail(c, PIC_ERR_HIP, "count readback failed");
    v->count = total;
    if (!v->x || !v->y || !v->z || !v->ux || !v->uy || !v->uz || !v->w || !v->id)
        return fail(c, PIC_ERR_ARG, "view arrays must not be NULL");
    if (v->capacity < total) return fail(c, PIC_ERR_ARG, "view capacity %lld < %lld particles", (long long)v->capacity, (long long)total);
    const size_t n = (size_t)c->g.nsc * sv.cap;
    std::vector<R> a[7];
    const R* src[7] = {sv.x, sv.y, sv.z, sv.ux, sv.uy, sv.uz, sv.w};
    for (int k = 0; k < 7; ++k) {
        a[k].resize(n);
        HIPCHK(c, hipMemcpyAsync(a[k].data(), src[k], n * sizeof(R), hipMemcpyDeviceToHost, c->stream));
    }
    std::vector<uint32_t> ids(n);
    std::vector<uint8_t> zs;
    HIPCHK(c, hipMemcpyAsync(ids.data(), sv.id, n * 4, hipMemcpyDeviceToHost, c->stream));
    if (sv.zs) {
        zs.resize(n);
        HIPCHK(c, hipMemcpyAsync(zs.data(), sv.zs, n, hipMemcpyDeviceToHost, c->stream));
    }
    HIPCHK(c, hipStreamSynchronize(c->stream));
    std::vector<size_t> order;
    order.reserve(total);
    for (int sc = 0; sc < c->g.nsc; ++sc)
        for (int t = 0; t < cnt[sc]; ++t) order.push_back((size_t)sc * sv.cap + t);
    std::sort(order.begin(), order.end(), [&](size_t p, size_t q) { return ids[p] < ids[q]; });
    for (int64_t k = 0; k < total; ++k) {
        const size_t p = order[k];
        const int sc = (int)(p / sv.cap);
        const int scx = sc % c->g.ncx, scy = (sc / c->g.ncx) % c->g.ncy, scz = sc / (c->g.ncx * c->g.ncy);
        v->x[k] = (double)(scx * SX) + (double)a[0][p];
        v->y[k] = (double)(scy * SY) + (double)a[1][p];
        v->z[k] = (double)(scz * SZ) + (double)a[2][p];
        v->ux[k] = (U)a[3][p];
        v->uy[k] = (U)a[4][p];
        v->uz[k] = (U)a[5][p];
        v->w[k] = (U)a[6][p];
        v->id[k] = ids[p];
        if (v->zstate) v->zstate[k] = sv.zs ? zs[p] : 0;
    }
    return PIC_OK;
}

template <class R, class V>
int set_particles_t(pic_ctx* c, int s, const V* v)
{
    if (v->count < 0) return fail(c, PIC_ERR_ARG, "negative count");
    if (v->count > 0 && (!v->x || !v->y || !v->z || !v->ux || !v->uy || !v->uz || !v->w || !v->id))
        return fail(c, PIC_ERR_ARG, "view arrays must not be NULL");
    const SpeciesViewT<R>& sv = sview<R>(c, s);
    const GridView& g = c->g;
    const size_t n = (size_t)g.nsc * sv.cap;
    std::vector<int32_t> cnt(g.nsc, 0);
    std::vector<R> a[7];
    for (auto& x : a) x.assign(n, R(0));
    std::vector<uint32_t> ids(n, 0);
    std::vector<uint8_t> zs(sv.zs ? n : 0, 0);
    const R lim[3] = {face_below<R>((R)SX), face_below<R>((R)SY), face_below<R>((R)SZ)};
    const double rmax = (double)std::numeric_limits<R>::max();
    double wmax = 0.0;
    for (int64_t k = 0; k < v->count; ++k) {
        const double p[3] = {v->x[k], v->y[k], v->z[k]};
        const int dims[3] = {g.nx, g.ny, g.nz}, sdim[3] = {SX, SY, SZ};
        int sci[3];
        R rel[3];
        for (int d = 0; d < 3; ++d) {
            if (!(p[d] >= 0.0 && p[d] < (double)dims[d]))
                return fail(c, PIC_ERR_ARG, "particle %lld: position %g outside [0,%d)", (long long)k, p[d], dims[d]);
            sci[d] = (int)std::floor(p[d] / sdim[d]);
            if (sci[d] >= dims[d] / sdim[d]) sci[d] = dims[d] / sdim[d] - 1;
            rel[d] = std::min((R)(p[d] - (double)(sci[d] * sdim[d])), lim[d]);
            if (rel[d] < R(0)) rel[d] = R(0);
        }
        const double u[4] = {(double)v->ux[k], (double)v->uy[k], (double)v->uz[k], (double)v->w[k]};
        for (double x : u)
            if (!std::isfinite(x) || std::fabs(x) > rmax)
                return fail(c, PIC_ERR_ARG, "particle %lld: non-finite momentum or weight", (long long)k);
        if (v->id[k] < 0 || v->id[k] > 0xFFFFFFFFLL) return fail(c, PIC_ERR_ARG, "particle %lld: id out of range", (long long)k);
        const int sc = sci[0] + g.ncx * (sci[1] + g.ncy * sci[2]);
        if (cnt[sc] >= sv.cap) return fail(c, PIC_ERR_CAPACITY, "supercell %d holds more than %d particles", sc, sv.cap);
        wmax = std::max(wmax, std::fabs(u[3]));
        const size_t q = (size_t)sc * sv.cap + cnt[sc]++;
        a[0][q] = rel[0]; a[1][q] = rel[1]; a[2][q] = rel[2];
        a[3][q] = (R)u[0]; a[4][q] = (R)u[1]; a[5][q] = (R)u[2]; a[6][q] = (R)u[3];
        ids[q] = (uint32_t)v->id[k];
        if (sv.zs) {
            const int z = v->zstate ? v->zstate[k] : c->sp[s].desc.z_init;
            if (z < 0 || z > c->sp[s].desc.z_max) return fail(c, PIC_ERR_ARG, "particle %lld: charge state out of range", (long long)k);
            zs[q] = (uint8_t)z;
        }
    }
    R* dst[7] = {sv.x, sv.y, sv.z, sv.ux, sv.uy, sv.uz, sv.w};
    for (int k = 0; k < 7; ++k)
        HIPCHK(c, hipMemcpyAsync(dst[k], a[k].data(), n * sizeof(R), hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(sv.id, ids.data(), n * 4, hipMemcpyHostToDevice, c->stream));
    if (sv.zs) HIPCHK(c, hipMemcpyAsync(sv.zs, zs.data(), n, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(sv.count, cnt.data(), (size_t)g.nsc * 4, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    c->sp[s].wmax = wmax;
    c->sp[s].wheld = wmax;
    c->rho_prev_valid = false;
    return PIC_OK;
}

template <class R, class T>
int get_fields_t(pic_ctx* c, T* E, T* B, T* J)
{
    const size_t n3 = (size_t)3 * c->grid.nx * c->grid.ny * c->grid.nz;
    const GridViewT<R>& g = gview<R>(c);
    const R* src[3] = {g.E, g.B, g.J};
    T* dst[3] = {E, B, J};
    std::vector<R> tmp;
    for (int f = 0; f < 3; ++f) {
        if (!dst[f]) continue;
        if constexpr (std::is_same<R, T>::value) {
            HIPCHK(c, hipMemcpyAsync(dst[f], src[f], n3 * sizeof(R), hipMemcpyDeviceToHost, c->stream));
            HIPCHK(c, hipStreamSynchronize(c->stream));
        } else {
            tmp.resize(n3);
            HIPCHK(c, hipMemcpyAsync(tmp.data(), src[f], n3 * sizeof(R), hipMemcpyDeviceToHost, c->stream));
            HIPCHK(c, hipStreamSynchronize(c->stream));
            for (size_t i = 0; i < n3; ++i) dst[f][i] = (T)tmp[i];
        }
    }
    return PIC_OK;
}

template <class R, class T>
int set_fields_t(pic_ctx* c, const T* E, const T* B, const T* J)
{
    const size_t n3 = (size_t)3 * c->grid.nx * c->grid.ny * c->grid.nz;
    const double rmax = (double)std::numeric_limits<R>::max();
    const T* src[3] = {E, B, J};
    for (const T* f : src)
        if (f)
            for (size_t i = 0; i < n3; ++i)
                if (!std::isfinite((double)f[i]) || std::fabs((double)f[i]) > rmax)
                    return fail(c, PIC_ERR_ARG, "non-finite field value at %zu", i);
    const GridViewT<R>& g = gview<R>(c);
    R* dst[3] = {g.E, g.B, g.J};
    std::vector<R> tmp;
    for (int f = 0; f < 3; ++f) {
        if (!src[f]) continue;
        if constexpr (std::is_same<R, T>::value) {
            HIPCHK(c, hipMemcpyAsync(dst[f], src[f], n3 * sizeof(R), hipMemcpyHostToDevice, c->stream));
            HIPCHK(c, hipStreamSynchronize(c->stream));
        } else {
            tmp.resize(n3);
            for (size_t i = 0; i < n3; ++i) tmp[i] = (R)src[f][i];
            HIPCHK(c, hipMemcpyAsync(dst[f], tmp.data(), n3 * sizeof(R), hipMemcpyHostToDevice, c->stream));
            HIPCHK(c, hipStreamSynchronize(c->stream));
        }
    }
    c->rho_prev_valid = false;
    return PIC_OK;
}

// The cycles of pic_step in real type R.
template <class R>
int step_t(pic_ctx* c, int n)
{
    GridViewT<R>& g = gview<R>(c);
    const int64_t N = (int64_t)c->grid.nx * c->grid.ny * c->grid.nz;
    const double dt = c->grid.dt;
    for (int it = 0; it < n; ++it) {
        hipEvent_t e0 = nullptr, e1 = nullptr, e2 = nullptr, e3 = nullptr;
        if (c->timing) {
            e0 = next_event(c); e1 = next_event(c); e2 = next_event(c); e3 = next_event(c);
            if (!e0 || !e1 || !e2 || !e3) return fail(c, PIC_ERR_HIP, "event creation failed");
            HIPCHK(c, hipEventRecord(e0, c->stream));
        }
        // the cycle's common fixed-point scale of the deterministic J: that of the largest bound
        float jscale_g = 0.0f;
        if (g.J64) {
            double vg = 0.0;
            for (int s = 0; s < c->nsp; ++s)
                if (c->sp[s].desc.mobile) vg = std::max(vg, push_vmax(c, s));
            jscale_g = fixed_scale(vg);
            g.jinv64 = 1.0 / (double)jscale_g;
            HIPCHK(c, launch_zero_f64(reinterpret_cast<double*>(g.J64), 3 * N, c->stream));  // all-zero bits
        } else {
            HIPCHK(c, launch_zero_r(g.J, 3 * N, c->stream));
        }
        // step `it` writes its leavers to parity it & 1 and absorbs the previous step's
        const int wpar = it & 1, apar = it > 0 ? ((it - 1) & 1) : -1;
        for (int s = 0; s < c->nsp; ++s) {
            if (!c->sp[s].desc.mobile) continue;
            HIPCHK(c, launch_push<R>(g, sview<R>(c, s), c->order, c->grid.gather == PIC_GATHER_GALERKIN,
                                     push_vmax(c, s), jscale_g, apar, wpar, c->stream));
            c->pending_launches += c->timing ? 1 : 0;
        }
        if (c->timing) HIPCHK(c, hipEventRecord(e1, c->stream));
        if (it == n - 1)  // last step of the call: leave the frames dense
            for (int s = 0; s < c->nsp; ++s) {
                if (!c->sp[s].desc.mobile) continue;
                HIPCHK(c, launch_migrate<R>(g, sview<R>(c, s), wpar, c->stream));
            }
        if (c->timing) HIPCHK(c, hipEventRecord(e2, c->stream));
        HIPCHK(c, launch_yee_b<R>(g, 0.5 * dt, c->stream));
        HIPCHK(c, launch_yee_e<R>(g, dt, c->stream));
        HIPCHK(c, launch_yee_b<R>(g, 0.5 * dt, c->stream));
        if (c->timing) HIPCHK(c, hipEventRecord(e3, c->stream));
        ++c->step;
    }
    return PIC_OK;
}

// FP64 diagnostics of the state in real type R (results in diag.result).
template <class R>
int moments_t(pic_ctx* c)
{
    const int64_t N = (int64_t)c->grid.nx * c->grid.ny * c->grid.nz;
    GridViewT<R>& g = gview<R>(c);
    HIPCHK(c, launch_zero_f64(c->diag.result, D_NSLOTS, c->stream));
    HIPCHK(c, launch_field_energy<R>(g, c->diag, c->stream));
    for (int s = 0; s < c->nsp; ++s) HIPCHK(c, launch_kinetic<R>(g, sview<R>(c, s), c->diag, s, c->stream));
    HIPCHK(c, launch_zero_f64(c->diag.rho, N, c->stream));
    for (int s = 0; s < c->nsp; ++s)
        HIPCHK(c, launch_rho_deposit<R>(g, sview<R>(c, s), c->order, c->diag.rho, c->stream));
    HIPCHK(c, launch_gauss<R>(g, c->diag, c->grid.rho_bg, 1, c->rho_prev_valid, c->stream));
    return PIC_OK;
}

// rho before the next cycle, for the continuity residual of that cycle
template <class R>
int keep_rho_t(pic_ctx* c)
{
    const int64_t N = (int64_t)c->grid.nx * c->grid.ny * c->grid.nz;
    HIPCHK(c, launch_zero_f64(c->diag.rho_prev, N, c->stream));
    for (int s = 0; s < c->nsp; ++s)
        HIPCHK(c, launch_rho_deposit<R>(gview<R>(c), sview<R>(c, s), c->order, c->diag.rho_prev, c->stream));
    return PIC_OK;
}

}  // namespace

extern "C" {

int pic_abi_version(void) { return PIC_ABI_VERSION; }

const char* pic_last_error(const pic_ctx* ctx) { return ctx ? ctx->err.c_str() : g_init_error.c_str(); }

int pic_init(pic_ctx** out, const pic_grid_t* grid, const pic_species_t* species, int n_species, pic_shape_t shape,
             const pic_alloc_t* alloc, void* hip_stream)
{
    if (!out) return fail(nullptr, PIC_ERR_ARG, "out must not be NULL");
    *out = nullptr;
    int rc = validate(grid, species, n_species, shape);
    if (rc) return rc;
    if (alloc && (!alloc->alloc || !alloc->free)) return fail(nullptr, PIC_ERR_ARG, "allocator needs alloc and free");
    pic_ctx* c = new (std::nothrow) pic_ctx();
    if (!c) return fail(nullptr, PIC_ERR_OOM, "host allocation failed");
    c->grid = *grid;
    c->order = (int)shape;
    c->nsp = n_species;
    c->stream = (hipStream_t)hip_stream;
    if (alloc) {
        c->alloc = *alloc;
        c->use_cb = true;
    }
    GridView& g = c->g;
    g.nx = grid->nx; g.ny = grid->ny; g.nz = grid->nz;
    g.ncx = grid->nx / SX; g.ncy = grid->ny / SY; g.ncz = grid->nz / SZ;
    g.nsc = g.ncx * g.ncy * g.ncz;
    {   // z-fastest slabs when each XCD's share is whole z-layers, plain slabs otherwise
        const int per = g.nsc / 8, nxy = g.ncx * g.ncy;
        g.xcd_remap = (g.nsc % 8 != 0) ? 0 : (per % nxy == 0) ? per / nxy : 1;
    }
    g.dx = (float)grid->dx; g.dy = (float)grid->dy; g.dz = (float)grid->dz; g.dt = (float)grid->dt;
    g.b0x = (float)grid->b0[0]; g.b0y = (float)grid->b0[1]; g.b0z = (float)grid->b0[2];
    c->fp64 = grid->precision == PIC_PRECISION_FP64;
    GridView64& g64 = c->g64;
    g64.nx = g.nx; g64.ny = g.ny; g64.nz = g.nz;
    g64.ncx = g.ncx; g64.ncy = g.ncy; g64.ncz = g.ncz;
    g64.nsc = g.nsc;
    g64.xcd_remap = g.xcd_remap;
    g64.dx = grid->dx; g64.dy = grid->dy; g64.dz = grid->dz; g64.dt = grid->dt;
    g64.b0x = grid->b0[0]; g64.b0y = grid->b0[1]; g64.b0z = grid->b0[2];
    const int64_t N = (int64_t)grid->nx * grid->ny * grid->nz;

    auto bail = [&](int code) {
        std::string msg = c->err;
        release_all(c);
        delete c;
        if (!msg.empty()) g_init_error = msg;
        return code;
    };
    if (hipGetDevice(&c->device) != hipSuccess || noalloc_scratch_setup(c->device) != hipSuccess) {
        c->err = "device query or static staging buffer address failed";
        return bail(PIC_ERR_HIP);
    }
    if (hipHostMalloc((void**)&c->flags_host, NFLAGS * sizeof(int32_t)) != hipSuccess) {
        c->flags_host = nullptr;
        c->err = "pinned host allocation failed";
        return bail(PIC_ERR_HIP);
    }
    bool fields_ok = (g.flags = (int32_t*)dev_alloc(c, 64)) != nullptr;
    if (c->fp64)
        fields_ok = fields_ok && (g64.E = (double*)dev_alloc(c, 3 * N * 8)) && (g64.B = (double*)dev_alloc(c, 3 * N * 8)) &&
                    (g64.J = (double*)dev_alloc(c, 3 * N * 8));
    else
        fields_ok = fields_ok && (g.E = (float*)dev_alloc(c, 3 * N * 4)) && (g.B = (float*)dev_alloc(c, 3 * N * 4)) &&
                    (g.J = (float*)dev_alloc(c, 3 * N * 4));
    g64.flags = g.flags;
    if (!fields_ok) {
        c->err = "device allocation of fields failed";
        return bail(PIC_ERR_OOM);
    }
    c->diag.npartial = std::max(8 * 1024, g.nsc);
    if (!(c->diag.rho = (double*)dev_alloc(c, N * 8)) || !(c->diag.g0 = (double*)dev_alloc(c, N * 8)) ||
        !(c->diag.partial = (double*)dev_alloc(c, (size_t)c->diag.npartial * 8)) ||
        !(c->diag.result = (double*)dev_alloc(c, D_NSLOTS * 8)) ||
        ((grid->options & PIC_OPT_CONTINUITY) && !(c->diag.rho_prev = (double*)dev_alloc(c, N * 8)))) {
        c->err = "device allocation of diagnostics failed";
        return bail(PIC_ERR_OOM);
    }
    if ((grid->options & PIC_OPT_DETERMINISTIC_J) &&
        !(g.J64 = (unsigned long long*)dev_alloc(c, 3 * N * 8))) {
        c->err = "device allocation of the fixed-point current failed";
        return bail(PIC_ERR_OOM);
    }
    const bool zero_failed =
        c->fp64 ? (launch_zero_f64(g64.E, 3 * N, c->stream) || launch_zero_f64(g64.B, 3 * N, c->stream) ||
                   launch_zero_f64(g64.J, 3 * N, c->stream))
                : (launch_zero_f32(g.E, 3 * N, c->stream) || launch_zero_f32(g.B, 3 * N, c->stream) ||
                   launch_zero_f32(g.J, 3 * N, c->stream));
    if (zero_failed || launch_zero_i32(g.flags, 16, c->stream) || launch_zero_f64(c->diag.result, D_NSLOTS, c->stream) ||
        (g.J64 && launch_zero_f64(reinterpret_cast<double*>(g.J64), 3 * N, c->stream))) {
        c->err = "field initialisation launch failed";
        return bail(PIC_ERR_HIP);
    }
    // species: ids are assigned in species order, cell-major within a species
    int64_t off = 0;
    const double dV = grid->dx * grid->dy * grid->dz;
    for (int s = 0; s < n_species; ++s) {
        Species& S = c->sp[s];
        S.desc = species[s];
        S.id_offset = off;
        S.n_init = N * species[s].ppc;
        S.weight = species[s].ppc > 0 ? species[s].density * dV / species[s].ppc : 0.0;
        S.wmax = S.weight;
        S.wheld = S.weight;
        off += S.n_init;
    }
    for (int s = 0; s < n_species; ++s) {
        if ((rc = alloc_species(c, s))) return bail(rc);
    }
    // one deposit queue shared by the species (their particle kernels run one after another)
    g.qcap = 0;
    for (int s = 0; s < n_species; ++s) g.qcap = std::max(g.qcap, c->sp[s].v.cap);
    g.qcap = (g.qcap + 511) / 512 * 512;  // whole 512-lane workgroups' worth of slots
    g64.qcap = g.qcap;
    const bool q_ok = c->fp64 ? (g64.qbuf = (double4*)dev_alloc(c, (size_t)2 * g.nsc * g.qcap * sizeof(double4))) != nullptr
                              : (g.qbuf = (float4*)dev_alloc(c, (size_t)2 * g.nsc * g.qcap * sizeof(float4))) != nullptr;
    if (!q_ok) {
        c->err = "device allocation of the deposit queue failed";
        return bail(PIC_ERR_OOM);
    }
    if ((rc = alloc_ionisation(c))) return bail(rc);
    for (int s = 0; s < n_species; ++s) {
        Species& S = c->sp[s];
        const pic_species_t& d = S.desc;
        if (d.ppc == 0) continue;
        const double b2 = d.drift_beta[0] * d.drift_beta[0] + d.drift_beta[1] * d.drift_beta[1] +
                          d.drift_beta[2] * d.drift_beta[2];
        const double gam = 1.0 / std::sqrt(1.0 - b2);
        const double drift_u[3] = {gam * d.drift_beta[0], gam * d.drift_beta[1], gam * d.drift_beta[2]};
        int pos_index = s, pos_ppc = d.ppc;
        int64_t pos_off = S.id_offset;
        if (d.coincident_with >= 0) {
            pos_index = d.coincident_with;
            pos_ppc = c->sp[pos_index].desc.ppc;
            pos_off = c->sp[pos_index].id_offset;
        }
        const hipError_t e =
            c->fp64 ? launch_init_species<double>(g64, S.v64, grid->seed, s, d.ppc, S.id_offset, pos_index, pos_ppc,
                                                  pos_off, d.u_th, drift_u, d.layout, S.weight, d.z_init, c->stream)
                    : launch_init_species<float>(g, S.v, grid->seed, s, d.ppc, S.id_offset, pos_index, pos_ppc, pos_off,
                                                 d.u_th, drift_u, d.layout, S.weight, d.z_init, c->stream);
        if (e != hipSuccess) {
            c->err = "init launch failed";
            return bail(PIC_ERR_HIP);
        }
    }
    if ((rc = mark_reference(c))) return bail(rc);
    *out = c;
    return PIC_OK;
}

int pic_destroy(pic_ctx* ctx)
{
    if (!ctx) return PIC_OK;
    (void)hipStreamSynchronize(ctx->stream);
    release_all(ctx);
    delete ctx;
    return PIC_OK;
}

int pic_step(pic_ctx* c, int n)
{
    if (!c) return fail(nullptr, PIC_ERR_ARG, "ctx is NULL");
    if (n < 0) return fail(c, PIC_ERR_ARG, "n must be >= 0");
    int rc0 = PIC_OK;
    if ((c->grid.options & PIC_OPT_CONTINUITY) && n > 0) {
        // the cycles but the last (frames dense again after them), rho, the last cycle
        if (n > 1) rc0 = c->fp64 ? step_t<double>(c, n - 1) : step_t<float>(c, n - 1);
        if (!rc0) rc0 = c->fp64 ? keep_rho_t<double>(c) : keep_rho_t<float>(c);
        if (!rc0) rc0 = c->fp64 ? step_t<double>(c, 1) : step_t<float>(c, 1);
        c->rho_prev_valid = rc0 == PIC_OK;
    } else {
        rc0 = c->fp64 ? step_t<double>(c, n) : step_t<float>(c, n);
    }
    if (rc0) return rc0;
    if (c->timing) {
        // particles processed: counts before the step are what each push launch read
        for (int s = 0; s < c->nsp; ++s)
            if (c->sp[s].desc.mobile) {
                std::vector<int32_t> cnt;
                const int64_t t = host_count(c, s, cnt);
                if (t < 0) return fail(c, PIC_ERR_HIP, "count readback failed");
                c->pending_particles += t * n;
            }
        int rc = collect_timing(c);
        if (rc) return rc;
    }
    return read_flags(c);
}

int pic_timing(pic_ctx* c, int enable, pic_timing_t* out)
{
    if (!c) return fail(nullptr, PIC_ERR_ARG, "ctx is NULL");
    int rc = collect_timing(c);
    if (rc) return rc;
    if (out) *out = c->tacc;
    if (enable == 1) {
        c->tacc = pic_timing_t{};
        c->timing = true;
    } else if (enable == 0) {
        c->timing = false;
    }
    return PIC_OK;
}

int pic_mark_reference(pic_ctx* c)
{
    if (!c) return fail(nullptr, PIC_ERR_ARG, "ctx is NULL");
    return mark_reference(c);
}

int pic_moments(pic_ctx* c, pic_moments_t* out)
{
    if (!c || !out) return fail(c, PIC_ERR_ARG, "ctx and out must not be NULL");
    const int rc = c->fp64 ? moments_t<double>(c) : moments_t<float>(c);
    if (rc) return rc;
    double r[D_NSLOTS];
    HIPCHK(c, hipMemcpyAsync(r, c->diag.result, sizeof r, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    std::memset(out, 0, sizeof *out);
    out->w_e = r[D_WE];
    out->w_b = r[D_WB];
    out->kinetic_total = 0.0;
    for (int s = 0; s < c->nsp; ++s) {
        out->kinetic[s] = r[D_KIN0 + s];
        out->kinetic_total += r[D_KIN0 + s];
        std::vector<int32_t> cnt;
        out->count[s] = host_count(c, s, cnt);
    }
    out->charge_total = r[D_CHARGE];
    out->rho_max = r[D_RHOMAX];
    out->gauss_max = r[D_GAUSS];
    out->divb_max = r[D_DIVB];
    out->step = c->step;
    out->nonfinite = (int32_t)r[D_NONFINITE];
    out->continuity_max = c->rho_prev_valid ? r[D_CONT] : -1.0;
    out->j_max = r[D_JMAX];
    if (out->nonfinite) return fail(c, PIC_ERR_NONFINITE, "%d non-finite field entries", out->nonfinite);
    return PIC_OK;
}

int pic_get_run_state(pic_ctx* c, pic_run_state_t* out)
{
    if (!c || !out) return fail(c, PIC_ERR_ARG, "ctx and out must not be NULL");
    std::memset(out, 0, sizeof *out);
    out->step = c->step;
    out->seed = c->grid.seed;
    for (int s = 0; s < c->nsp; ++s) out->weight_bound[s] = c->sp[s].wmax;
    return PIC_OK;
}

int pic_set_run_state(pic_ctx* c, const pic_run_state_t* in)
{
    if (!c || !in) return fail(c, PIC_ERR_ARG, "ctx and in must not be NULL");
    if (in->step < 0) return fail(c, PIC_ERR_ARG, "step must be >= 0");
    for (int s = 0; s < c->nsp; ++s) {
        const double b = in->weight_bound[s];
        if (!std::isfinite(b) || b < c->sp[s].wheld)
            return fail(c, PIC_ERR_ARG, "species %d: weight bound %g below the largest held |w| %g", s, b,
                        c->sp[s].wheld);
    }
    c->step = in->step;
    c->grid.seed = in->seed;
    for (int s = 0; s < c->nsp; ++s) c->sp[s].wmax = in->weight_bound[s];
    return PIC_OK;
}

int pic_particle_count(pic_ctx* c, int s, int64_t* count)
{
    if (!c || !count) return fail(c, PIC_ERR_ARG, "ctx and count must not be NULL");
    if (s < 0 || s >= c->nsp) return fail(c, PIC_ERR_ARG, "species %d out of range", s);
    std::vector<int32_t> cnt;
    const int64_t t = host_count(c, s, cnt);
    if (t < 0) return fail(c, PIC_ERR_HIP, "count readback failed");
    *count = t;
    return PIC_OK;
}

int pic_get_particles(pic_ctx* c, int s, pic_particles_view_t* v)
{
    if (!c || !v) return fail(c, PIC_ERR_ARG, "ctx and view must not be NULL");
    if (s < 0 || s >= c->nsp) return fail(c, PIC_ERR_ARG, "species %d out of range", s);
    return c->fp64 ? get_particles_t<double>(c, s, v) : get_particles_t<float>(c, s, v);
}

int pic_get_particles64(pic_ctx* c, int s, pic_particles64_view_t* v)
{
    if (!c || !v) return fail(c, PIC_ERR_ARG, "ctx and view must not be NULL");
    if (s < 0 || s >= c->nsp) return fail(c, PIC_ERR_ARG, "species %d out of range", s);
    return c->fp64 ? get_particles_t<double>(c, s, v) : get_particles_t<float>(c, s, v);
}

int pic_set_particles(pic_ctx* c, int s, const pic_particles_view_t* v)
{
    if (!c || !v) return fail(c, PIC_ERR_ARG, "ctx and view must not be NULL");
    if (s < 0 || s >= c->nsp) return fail(c, PIC_ERR_ARG, "species %d out of range", s);
    return c->fp64 ? set_particles_t<double>(c, s, v) : set_particles_t<float>(c, s, v);
}

int pic_set_particles64(pic_ctx* c, int s, const pic_particles64_view_t* v)
{
    if (!c || !v) return fail(c, PIC_ERR_ARG, "ctx and view must not be NULL");
    if (s < 0 || s >= c->nsp) return fail(c, PIC_ERR_ARG, "species %d out of range", s);
    return c->fp64 ? set_particles_t<double>(c, s, v) : set_particles_t<float>(c, s, v);
}

int pic_get_fields(pic_ctx* c, float* E, float* B, float* J)
{
    if (!c) return fail(nullptr, PIC_ERR_ARG, "ctx is NULL");
    return c->fp64 ? get_fields_t<double>(c, E, B, J) : get_fields_t<float>(c, E, B, J);
}

int pic_get_fields64(pic_ctx* c, double* E, double* B, double* J)
{
    if (!c) return fail(nullptr, PIC_ERR_ARG, "ctx is NULL");
    return c->fp64 ? get_fields_t<double>(c, E, B, J) : get_fields_t<float>(c, E, B, J);
}

int pic_set_fields(pic_ctx* c, const float* E, const float* B, const float* J)
{
    if (!c) return fail(nullptr, PIC_ERR_ARG, "ctx is NULL");
    return c->fp64 ? set_fields_t<double>(c, E, B, J) : set_fields_t<float>(c, E, B, J);
}

int pic_set_fields64(pic_ctx* c, const double* E, const double* B, const double* J)
{
    if (!c) return fail(nullptr, PIC_ERR_ARG, "ctx is NULL");
    return c->fp64 ? set_fields_t<double>(c, E, B, J) : set_fields_t<float>(c, E, B, J);
}

}  // extern "C"

namespace {

// One ionisation step.  Staged: the cell moments, the rate of every ion and
// the draw and append as three launches over the grid (the rate stage timed
// on its own).  Fused (the exact rate): one launch that does all three per
// supercell, so that the moments' streams of some workgroups overlap the
// FP64 quadrature of others.  The surrogate and the table always run staged:
// fused into the surrogate's persistent kernel (three waves per SIMD for its
// registers) the moments and the draw measured slower than on their own.
int ionize_impl(pic_ctx* c, pic_rate_mode_t mode, bool staged, pic_ionize_stats_t* out)
{
    if (!c) return fail(nullptr, PIC_ERR_ARG, "ctx is NULL");
    if (mode != PIC_RATE_EXACT && mode != PIC_RATE_MLP && mode != PIC_RATE_TABLE)
        return fail(c, PIC_ERR_ARG, "unknown rate mode %d", (int)mode);
    int nion = 0;
    for (int s = 0; s < c->nsp; ++s)
        if (ionising(c, s)) {
            ++nion;
            if (mode == PIC_RATE_MLP && !c->mlp[s].ready)
                return fail(c, PIC_ERR_STATE, "species %d: no trained or loaded surrogate", s);
            if (mode == PIC_RATE_TABLE) {
                const int rc = ensure_rate_table(c, s);
                if (rc != PIC_OK) return rc;
            }
        }
    if (!nion) return fail(c, PIC_ERR_STATE, "no ionising species (z_max > 0 with ionize_into >= 0)");
    c->rho_prev_valid = false;
    pic_ionize_stats_t st{};
    int64_t n0 = 0;
    for (int s = 0; s < c->nsp; ++s) n0 += c->sp[s].n_init;
    const double dV = c->grid.dx * c->grid.dy * c->grid.dz;
    const double dt_phys = c->grid.dt / omega_p(c->grid.n_ref_cm3);
    float rate_ms = 0.0f, total_ms = 0.0f;
    for (int s = 0; s < c->nsp; ++s) {
        if (!ionising(c, s)) continue;
        const int e = c->sp[s].desc.ionize_into;
        const IonTables tab = ion_tables(c, s);
        HIPCHK(c, launch_zero_i32((int32_t*)c->counters, 2 * CNT_WORDS, c->stream));
        HIPCHK(c, hipEventRecord(c->iev[0], c->stream));
        const pic_species_t& d = c->sp[s].desc;
        const bool eloss = d.energy_loss != 0;
        const bool fused = !staged && mode == PIC_RATE_EXACT;
        DrawArgs a{};
        a.seed = c->grid.seed;
        a.step = c->step;
        a.species_index = s;
        a.ion_id_offset = c->sp[s].id_offset;
        a.id_base_new = n0;
        a.dt_phys = dt_phys;
        a.max_events = d.max_events;
        a.energy_loss = eloss ? 1 : 0;
        const DrawBuffers db{c->ne, c->kT, c->gl, eloss ? c->mom4 : nullptr, eloss ? c->de : nullptr,
                             eloss ? c->old_count : nullptr};
        const double nrdv = c->grid.n_ref_cm3 / dV;
        if (eloss) HIPCHK(c, launch_zero_f64(c->de, (int64_t)c->grid.nx * c->grid.ny * c->grid.nz, c->stream));
        if (fused) {
            HIPCHK(c, launch_ionize_exact(c->g, c->sp[s].v, c->sp[e].v, tab, a, db, nrdv, c->ne, c->kT,
                                          eloss ? c->mom4 : nullptr, c->counters, c->stream));
        } else {
            HIPCHK(c, launch_moments(c->g, c->sp[e].v, nrdv, c->ne, c->kT, eloss ? c->mom4 : nullptr, c->stream));
            HIPCHK(c, hipEventRecord(c->iev[1], c->stream));
            if (mode == PIC_RATE_EXACT)
                HIPCHK(c, launch_rate_exact(c->g, c->sp[s].v, tab, c->ne, c->kT, c->nu[s], c->gl, c->stream));
            else if (mode == PIC_RATE_TABLE)
                HIPCHK(c, launch_rate_table(c->g, c->sp[s].v, tab, c->ne, c->kT, c->nu[s], c->rtab[s], c->gl,
                                            c->counters, c->fbl[s], c->stream));
            else
                HIPCHK(c, launch_rate_mlp(c->g, c->sp[s].v, tab, mlp_launch(c, s), c->ne, c->kT, c->nu[s], c->gl,
                                          c->counters, c->fbl[s], c->stream));
            HIPCHK(c, hipEventRecord(c->iev[2], c->stream));
            HIPCHK(c, launch_draw_append(c->g, c->sp[s].v, c->sp[e].v, tab, a, c->nu[s], db, c->counters, c->stream));
        }
        if (eloss) HIPCHK(c, launch_energy_loss(c->g, c->sp[e].v, db, c->stream));
        HIPCHK(c, hipEventRecord(c->iev[3], c->stream));
        unsigned long long cnt[CNT_WORDS];
        HIPCHK(c, hipMemcpyAsync(cnt, c->counters, sizeof cnt, hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        float r = -1.f, t = 0.f;
        if (!fused) HIPCHK(c, hipEventElapsedTime(&r, c->iev[1], c->iev[2]));
        HIPCHK(c, hipEventElapsedTime(&t, c->iev[0], c->iev[3]));
        rate_ms += r;
        total_ms += t;
        for (int k = 0; k < CNT_STRIPES; ++k) {
            st.ions_active += (int64_t)cnt[CNT_ACTIVE + k];
            st.ionized += (int64_t)cnt[CNT_FIRED + k];
        }
        st.fallback += (int64_t)cnt[CNT_FALLBACK];
        std::vector<int32_t> cc;
        st.electrons = host_count(c, e, cc);
        c->sp[e].wmax = std::max(c->sp[e].wmax, c->sp[s].wmax);  // born electrons carry ion weights
        c->sp[e].wheld = std::max(c->sp[e].wheld, c->sp[s].wheld);
    }
    st.rate_ms = rate_ms < 0.0f ? -1.0 : rate_ms;
    st.total_ms = total_ms;
    if (out) *out = st;
    return read_flags(c);
}

}  // namespace

extern "C" {

int pic_ionize(pic_ctx* c, pic_rate_mode_t mode, pic_ionize_stats_t* out) { return ionize_impl(c, mode, false, out); }

int pic_ionize_staged(pic_ctx* c, pic_rate_mode_t mode, pic_ionize_stats_t* out)
{
    return ionize_impl(c, mode, true, out);
}

int pic_cell_moments(pic_ctx* c, int s, double* ne_out, double* kT_out)
{
    if (!c) return fail(nullptr, PIC_ERR_ARG, "ctx is NULL");
    if (s < 0 || s >= c->nsp || !ionising(c, s)) return fail(c, PIC_ERR_ARG, "species %d does not ionise", s);
    const int e = c->sp[s].desc.ionize_into;
    const int64_t N = (int64_t)c->grid.nx * c->grid.ny * c->grid.nz;
    const double dV = c->grid.dx * c->grid.dy * c->grid.dz;
    HIPCHK(c, launch_moments(c->g, c->sp[e].v, c->grid.n_ref_cm3 / dV, c->ne, c->kT, nullptr, c->stream));
    if (ne_out) HIPCHK(c, hipMemcpyAsync(ne_out, c->ne, N * 8, hipMemcpyDeviceToHost, c->stream));
    if (kT_out) HIPCHK(c, hipMemcpyAsync(kT_out, c->kT, N * 8, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return PIC_OK;
}

int pic_cell_moments_device(pic_ctx* c, int s, const double** ne_dev, const double** kT_dev)
{
    if (!c) return fail(nullptr, PIC_ERR_ARG, "ctx is NULL");
    if (s < 0 || s >= c->nsp || !ionising(c, s)) return fail(c, PIC_ERR_ARG, "species %d does not ionise", s);
    const int e = c->sp[s].desc.ionize_into;
    const double dV = c->grid.dx * c->grid.dy * c->grid.dz;
    HIPCHK(c, launch_moments(c->g, c->sp[e].v, c->grid.n_ref_cm3 / dV, c->ne, c->kT, nullptr, c->stream));
    if (ne_dev) *ne_dev = c->ne;
    if (kT_dev) *kT_dev = c->kT;
    return PIC_OK;
}

}  // extern "C"

namespace {

// Arguments of pic_rate_eval(_noalloc); builds the rate table at its first use.
int rate_eval_check(pic_ctx* c, pic_rate_mode_t mode, int s, int64_t n, const double* kT, const double* ne,
                    const int32_t* Z, double* ln_rate)
{
    if (!c) return fail(nullptr, PIC_ERR_ARG, "ctx is NULL");
    if (mode != PIC_RATE_EXACT && mode != PIC_RATE_MLP && mode != PIC_RATE_TABLE)
        return fail(c, PIC_ERR_ARG, "unknown rate mode %d", (int)mode);
    if (s < 0 || s >= c->nsp || c->sp[s].desc.z_max == 0) return fail(c, PIC_ERR_ARG, "species %d has no charge states", s);
    if (n < 0 || (n > 0 && (!kT || !ne || !Z || !ln_rate))) return fail(c, PIC_ERR_ARG, "bad sample arrays");
    if (mode == PIC_RATE_MLP && !c->mlp[s].ready) return fail(c, PIC_ERR_STATE, "species %d: no surrogate", s);
    if (mode == PIC_RATE_TABLE) return ensure_rate_table(c, s);
    return PIC_OK;
}

// ln nu of n host samples through device staging st (inputs copied in, the
// rate kernel of the mode, the result copied out), synchronous.
int rate_eval_staged(pic_ctx* c, pic_rate_mode_t mode, int s, int64_t n, const double* kT, const double* ne,
                     const int32_t* Z, double* ln_rate, const NoallocStaging& st)
{
    hipError_t e = hipMemcpyAsync(st.kT, kT, n * 8, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(st.ne, ne, n * 8, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(st.Z, Z, n * 4, hipMemcpyHostToDevice, c->stream);
    const IonTables tab = ion_tables(c, s);
    if (e == hipSuccess)
        e = mode == PIC_RATE_EXACT ? launch_ln_rate_exact(n, st.kT, st.ne, st.Z, tab, c->gl, st.out, c->stream)
            : mode == PIC_RATE_TABLE
                ? launch_ln_rate_table(n, st.kT, st.ne, st.Z, tab, c->rtab[s], c->gl, st.out, c->stream)
                : launch_ln_rate_mlp(n, st.kT, st.ne, st.Z, tab, mlp_launch(c, s), c->gl, st.out, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(ln_rate, st.out, n * 8, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return fail(c, PIC_ERR_HIP, "rate evaluation: %s", hipGetErrorString(e));
    return PIC_OK;
}

}  // namespace

extern "C" {

int pic_rate_eval(pic_ctx* c, pic_rate_mode_t mode, int s, int64_t n, const double* kT, const double* ne,
                  const int32_t* Z, double* ln_rate)
{
    const int rc0 = rate_eval_check(c, mode, s, n, kT, ne, Z, ln_rate);
    if (rc0 != PIC_OK) return rc0;
    if (n == 0) return PIC_OK;
    double* d = (double*)dev_alloc(c, (size_t)n * 3 * 8);
    int32_t* dz = (int32_t*)dev_alloc(c, (size_t)n * 4);
    if (!d || !dz) {
        dev_free(c, d);
        dev_free(c, dz);
        return fail(c, PIC_ERR_OOM, "rate evaluation buffers");
    }
    const int rc = rate_eval_staged(c, mode, s, n, kT, ne, Z, ln_rate, NoallocStaging{d, d + n, d + 2 * n, dz});
    dev_free(c, d);
    dev_free(c, dz);
    return rc;
}

int pic_rate_eval_noalloc(pic_ctx* c, pic_rate_mode_t mode, int s, int64_t n, const double* kT, const double* ne,
                          const int32_t* Z, double* ln_rate)
{
    const int rc = rate_eval_check(c, mode, s, n, kT, ne, Z, ln_rate);
    if (rc != PIC_OK) return rc;
    if (n > PIC_RATE_EVAL_NOALLOC_MAX)
        return fail(c, PIC_ERR_ARG, "n = %lld exceeds PIC_RATE_EVAL_NOALLOC_MAX (%d)", (long long)n,
                    PIC_RATE_EVAL_NOALLOC_MAX);
    if (n == 0) return PIC_OK;
    unsigned char* base = noalloc_scratch(c->device);
    if (!base) return fail(c, PIC_ERR_STATE, "no static staging buffer on device %d", c->device);
    return rate_eval_staged(c, mode, s, n, kT, ne, Z, ln_rate, noalloc_staging(base));
}

int pic_mlp_train(pic_ctx* c, int s, const pic_mlp_train_cfg_t* cfg, pic_mlp_report_t* out)
{
    if (!c || !cfg) return fail(c, PIC_ERR_ARG, "ctx and cfg must not be NULL");
    if (s < 0 || s >= c->nsp || c->sp[s].desc.z_max == 0) return fail(c, PIC_ERR_ARG, "species %d has no charge states", s);
    if (c->sp[s].desc.z_max > 6) return fail(c, PIC_ERR_ARG, "the surrogate has 6 charge-state inputs");
    if (cfg->batch < 64 || cfg->batch % 64 || cfg->n_train < cfg->batch || cfg->steps < 1)
        return fail(c, PIC_ERR_ARG, "batch must be a positive multiple of 64 and n_train >= batch, steps >= 1");
    if (!(cfg->t_min_ev > 0 && cfg->t_max_ev > cfg->t_min_ev && cfg->n_min_cm3 > 0 && cfg->n_max_cm3 > cfg->n_min_cm3))
        return fail(c, PIC_ERR_ARG, "sampling ranges must be positive and increasing");
    if (!(cfg->lr > 0 && cfg->lr_final >= 0)) return fail(c, PIC_ERR_ARG, "learning rates");
    if (cfg->activation != PIC_MLP_SILU && cfg->activation != PIC_MLP_RELU)
        return fail(c, PIC_ERR_ARG, "activation must be PIC_MLP_SILU or PIC_MLP_RELU");
    pic_ctx::Mlp& m = c->mlp[s];
    const int64_t n = cfg->n_train;
    float* X = (float*)dev_alloc(c, (size_t)n * 8 * 4);
    double* r = (double*)dev_alloc(c, (size_t)n * 8);
    float* t = (float*)dev_alloc(c, (size_t)n * 4);
    double* scratch = (double*)dev_alloc(c, (size_t)(1024 + 2) * 8);
    double* losses = (double*)dev_alloc(c, (size_t)cfg->steps * 8);
    auto cleanup = [&]() {
        dev_free(c, X); dev_free(c, r); dev_free(c, t); dev_free(c, scratch); dev_free(c, losses);
    };
    if (!X || !r || !t || !scratch || !losses) {
        cleanup();
        return fail(c, PIC_ERR_OOM, "training buffers");
    }
    const IonTables tab = ion_tables(c, s);
    MlpGen ga{std::log10(cfg->t_min_ev), std::log10(cfg->t_max_ev), std::log10(cfg->n_min_cm3), std::log10(cfg->n_max_cm3)};
    double* mu_s = scratch + 1024;
    hipError_t e = hipEventRecord(c->iev[0], c->stream);
    if (e == hipSuccess) e = launch_mlp_gen(n, cfg->seed, ga, tab, c->gl, X, r, c->stream);
    if (e == hipSuccess) e = launch_mlp_standardize(n, r, scratch, mu_s, t, c->stream);
    if (e == hipSuccess) e = launch_mlp_init(cfg->seed, m.params, m.m, m.v, c->stream);
    if (e == hipSuccess) e = launch_zero_f64(losses, cfg->steps, c->stream);
    const uint64_t draw_seed = (cfg->seed ^ 0x5DEECE66DULL) | 1ULL;
    double b1t = 1.0, b2t = 1.0;
    for (int it = 0; it < cfg->steps && e == hipSuccess; ++it) {
        MlpStep ms{X, t, n, cfg->batch, draw_seed, it, cfg->activation};
        int rows = 0;
        e = launch_mlp_step(m.params, ms, m.part, m.lpart, &rows, c->stream);
        b1t *= 0.9;
        b2t *= 0.999;
        const double lr = cfg->lr_final + 0.5 * (cfg->lr - cfg->lr_final) *
                                              (1.0 + std::cos(3.14159265358979323846 * it / cfg->steps));
        if (e == hipSuccess)
            e = launch_mlp_adam(m.params, m.part, rows, m.lpart, losses + it, m.m, m.v, (float)lr, (float)(1.0 - b1t),
                                (float)(1.0 - b2t), c->stream);
    }
    if (e == hipSuccess) e = hipEventRecord(c->iev[1], c->stream);
    std::vector<double> lh(cfg->steps);
    double msv[2] = {0.0, 1.0};
    if (e == hipSuccess) e = hipMemcpyAsync(lh.data(), losses, (size_t)cfg->steps * 8, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(msv, mu_s, 16, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    float ms_total = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms_total, c->iev[0], c->iev[1]);
    cleanup();
    if (e != hipSuccess) return fail(c, PIC_ERR_HIP, "training: %s", hipGetErrorString(e));
    m.mu = msv[0];
    m.s = msv[1];
    m.act = cfg->activation;
    m.t_min = cfg->t_min_ev; m.t_max = cfg->t_max_ev; m.n_min = cfg->n_min_cm3; m.n_max = cfg->n_max_cm3;
    m.ready = true;
    if (out) {
        out->loss_first = lh[0] / cfg->batch;
        const int k0 = std::max(0, cfg->steps - 100);
        double acc = 0.0;
        for (int i = k0; i < cfg->steps; ++i) acc += lh[i];
        out->loss_last = acc / (cfg->steps - k0) / cfg->batch;
        out->mu = m.mu;
        out->s = m.s;
        out->train_ms = ms_total;
        out->steps = cfg->steps;
    }
    return PIC_OK;
}

int pic_mlp_get_params(pic_ctx* c, int s, float* params, double* mu_s, double* range, int32_t* activation)
{
    if (!c) return fail(nullptr, PIC_ERR_ARG, "ctx is NULL");
    if (s < 0 || s >= c->nsp || c->sp[s].desc.z_max == 0) return fail(c, PIC_ERR_ARG, "species %d has no charge states", s);
    const pic_ctx::Mlp& m = c->mlp[s];
    if (params) {
        HIPCHK(c, hipMemcpyAsync(params, m.params, PIC_MLP_NPARAM * 4, hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
    }
    if (mu_s) { mu_s[0] = m.mu; mu_s[1] = m.s; }
    if (range) { range[0] = m.t_min; range[1] = m.t_max; range[2] = m.n_min; range[3] = m.n_max; }
    if (activation) *activation = m.act;
    return PIC_OK;
}

int pic_mlp_set_params(pic_ctx* c, int s, const float* params, const double* mu_s, const double* range,
                       int32_t activation)
{
    if (!c) return fail(nullptr, PIC_ERR_ARG, "ctx is NULL");
    if (s < 0 || s >= c->nsp || c->sp[s].desc.z_max == 0) return fail(c, PIC_ERR_ARG, "species %d has no charge states", s);
    if (!params || !mu_s) return fail(c, PIC_ERR_ARG, "params and mu_s must not be NULL");
    for (int i = 0; i < PIC_MLP_NPARAM; ++i)
        if (!std::isfinite(params[i])) return fail(c, PIC_ERR_ARG, "non-finite parameter %d", i);
    if (!(mu_s[1] > 0) || !std::isfinite(mu_s[0])) return fail(c, PIC_ERR_ARG, "bad standardisation");
    if (activation != PIC_MLP_SILU && activation != PIC_MLP_RELU)
        return fail(c, PIC_ERR_ARG, "activation must be PIC_MLP_SILU or PIC_MLP_RELU");
    pic_ctx::Mlp& m = c->mlp[s];
    if (range) {
        if (!(range[0] > 0 && range[1] > range[0] && range[2] > 0 && range[3] > range[2]))
            return fail(c, PIC_ERR_ARG, "bad trained range");
        m.t_min = range[0]; m.t_max = range[1]; m.n_min = range[2]; m.n_max = range[3];
    }
    HIPCHK(c, hipMemcpyAsync(m.params, params, PIC_MLP_NPARAM * 4, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    m.mu = mu_s[0];
    m.s = mu_s[1];
    m.act = activation;
    m.ready = true;
    return PIC_OK;
}

int pic_mlp_loss_grad(pic_ctx* c, int s, int64_t n, const float* X, const float* t, double* loss, float* grad)
{
    if (!c) return fail(nullptr, PIC_ERR_ARG, "ctx is NULL");
    if (s < 0 || s >= c->nsp || c->sp[s].desc.z_max == 0) return fail(c, PIC_ERR_ARG, "species %d has no charge states", s);
    if (n < 64 || n % 64 || n > (1 << 24) || !X || !t || !loss || !grad)
        return fail(c, PIC_ERR_ARG, "n must be a positive multiple of 64 with X, t, loss, grad given");
    pic_ctx::Mlp& m = c->mlp[s];
    float* dX = (float*)dev_alloc(c, (size_t)n * 9 * 4);
    double* dl = (double*)dev_alloc(c, 8);
    if (!dX || !dl) {
        dev_free(c, dX);
        dev_free(c, dl);
        return fail(c, PIC_ERR_OOM, "gradient buffers");
    }
    hipError_t e = hipMemcpyAsync(dX, X, n * 8 * 4, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(dX + n * 8, t, n * 4, hipMemcpyHostToDevice, c->stream);
    MlpStep ms{dX, dX + n * 8, n, (int)n, 0, 0, m.act};
    int rows = 0;
    if (e == hipSuccess) e = launch_mlp_step(m.params, ms, m.part, m.lpart, &rows, c->stream);
    if (e == hipSuccess) e = launch_mlp_grad(m.part, rows, m.lpart, m.grad, dl, c->stream);
    double lsum = 0.0;
    if (e == hipSuccess) e = hipMemcpyAsync(grad, m.grad, PIC_MLP_NPARAM * 4, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(&lsum, dl, 8, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    dev_free(c, dX);
    dev_free(c, dl);
    if (e != hipSuccess) return fail(c, PIC_ERR_HIP, "gradient: %s", hipGetErrorString(e));
    *loss = lsum / (double)n;
    return PIC_OK;
}

}  // extern "C"
