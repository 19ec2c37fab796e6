// Host side of the C ABI declared in include/pic.h: argument validation,
// device memory, kernel orchestration on the handle's stream, diagnostics and
// state transfer.  No exception crosses the ABI.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "pic_internal.hpp"

using namespace pic;

struct pic_ctx {
    pic_grid_t grid{};
    int order = 1;
    int nsp = 0;
    Species sp[PIC_MAX_SPECIES];
    GridView g{};
    DiagBuffers diag{};
    hipStream_t stream = nullptr;
    pic_alloc_t alloc{};
    bool use_cb = false;
    std::vector<void*> owned;
    int32_t* flags_host = nullptr;  // pinned
    int64_t step = 0;
    std::string err;
    // timing
    bool timing = false;
    pic_timing_t tacc{};
    std::vector<hipEvent_t> ev;
    int ev_used = 0;
    int64_t pending_particles = 0;
    int pending_launches = 0;
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
    } else if (hipMalloc(&p, bytes) != hipSuccess) {
        p = nullptr;
    }
    if (p) c->owned.push_back(p);
    return p;
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
    if (shape != PIC_SHAPE_CIC && shape != PIC_SHAPE_TSC) return fail(nullptr, PIC_ERR_ARG, "unknown shape %d", (int)shape);
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
            for (int z = 0; z < p.z_max; ++z)
                if (!finite_pos(p.ionization_ev[z]) || p.lotz_q[z] < 0)
                    return fail(nullptr, PIC_ERR_ARG, "species %d: ionisation data of state %d", s, z);
        }
        if (p.ionize_into != -1) {
            if (p.ionize_into < 0 || p.ionize_into >= n || p.ionize_into == s || p.z_max == 0)
                return fail(nullptr, PIC_ERR_ARG, "species %d: bad ionize_into", s);
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

int alloc_species(pic_ctx* c, int s)
{
    Species& S = c->sp[s];
    SpeciesView& v = S.v;
    const pic_species_t& d = S.desc;
    const int nsc = c->g.nsc;
    int cap_ppc = d.cap_ppc > 0 ? d.cap_ppc : (d.ppc * 3 + 1) / 2;
    if (cap_ppc < 1) cap_ppc = 1;
    v.cap = cap_ppc * SC_CELLS;
    int cap_in = v.cap / 4;
    cap_in = std::max(cap_in, 256);
    cap_in = std::min(cap_in, MAX_MIGRATE);
    v.cap_in = cap_in;
    const size_t n = (size_t)nsc * v.cap, ni = (size_t)nsc * cap_in;
    float** fl[] = {&v.x, &v.y, &v.z, &v.ux, &v.uy, &v.uz, &v.w};
    for (float** f : fl)
        if (!(*f = (float*)dev_alloc(c, n * 4))) return fail(c, PIC_ERR_OOM, "species %d: frames", s);
    if (!(v.id = (uint32_t*)dev_alloc(c, n * 4))) return fail(c, PIC_ERR_OOM, "species %d: ids", s);
    v.zs = nullptr;
    v.izs = nullptr;
    if (d.z_max > 0) {
        if (!(v.zs = (uint8_t*)dev_alloc(c, n))) return fail(c, PIC_ERR_OOM, "species %d: charge states", s);
        if (!(v.izs = (uint8_t*)dev_alloc(c, ni))) return fail(c, PIC_ERR_OOM, "species %d: arrivals", s);
    }
    float** fi[] = {&v.ix, &v.iy, &v.iz, &v.iux, &v.iuy, &v.iuz, &v.iw};
    for (float** f : fi)
        if (!(*f = (float*)dev_alloc(c, ni * 4))) return fail(c, PIC_ERR_OOM, "species %d: arrivals", s);
    if (!(v.iid = (uint32_t*)dev_alloc(c, ni * 4))) return fail(c, PIC_ERR_OOM, "species %d: arrivals", s);
    if (!(v.holes = (int32_t*)dev_alloc(c, ni * 4))) return fail(c, PIC_ERR_OOM, "species %d: holes", s);
    if (!(v.count = (int32_t*)dev_alloc(c, (size_t)nsc * 4))) return fail(c, PIC_ERR_OOM, "species %d: counts", s);
    if (!(v.in_count = (int32_t*)dev_alloc(c, (size_t)nsc * 4))) return fail(c, PIC_ERR_OOM, "species %d: counts", s);
    if (!(v.hole_count = (int32_t*)dev_alloc(c, (size_t)nsc * 4))) return fail(c, PIC_ERR_OOM, "species %d: counts", s);
    v.charge = (float)d.charge;
    v.mass = (float)d.mass;
    HIPCHK(c, launch_zero_i32(v.count, nsc, c->stream));
    HIPCHK(c, launch_zero_i32(v.in_count, nsc, c->stream));
    HIPCHK(c, launch_zero_i32(v.hole_count, nsc, c->stream));
    return PIC_OK;
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

int mark_reference(pic_ctx* c)
{
    const int64_t N = (int64_t)c->grid.nx * c->grid.ny * c->grid.nz;
    HIPCHK(c, launch_zero_f64(c->diag.rho, N, c->stream));
    for (int s = 0; s < c->nsp; ++s) HIPCHK(c, launch_rho_deposit(c->g, c->sp[s].v, c->order, c->diag.rho, c->stream));
    HIPCHK(c, launch_gauss(c->g, c->diag, c->grid.rho_bg, 0, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return PIC_OK;
}

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
    g.xcd_remap = (g.nsc % 8 == 0) ? 1 : 0;
    g.dx = (float)grid->dx; g.dy = (float)grid->dy; g.dz = (float)grid->dz; g.dt = (float)grid->dt;
    g.b0x = (float)grid->b0[0]; g.b0y = (float)grid->b0[1]; g.b0z = (float)grid->b0[2];
    const int64_t N = (int64_t)grid->nx * grid->ny * grid->nz;

    auto bail = [&](int code) {
        std::string msg = c->err;
        release_all(c);
        delete c;
        if (!msg.empty()) g_init_error = msg;
        return code;
    };
    if (hipHostMalloc((void**)&c->flags_host, NFLAGS * sizeof(int32_t)) != hipSuccess) {
        c->flags_host = nullptr;
        c->err = "pinned host allocation failed";
        return bail(PIC_ERR_HIP);
    }
    if (!(g.E = (float*)dev_alloc(c, 3 * N * 4)) || !(g.B = (float*)dev_alloc(c, 3 * N * 4)) ||
        !(g.J = (float*)dev_alloc(c, 3 * N * 4)) || !(g.flags = (int32_t*)dev_alloc(c, 64))) {
        c->err = "device allocation of fields failed";
        return bail(PIC_ERR_OOM);
    }
    c->diag.npartial = std::max(4 * 1024, g.nsc);
    if (!(c->diag.rho = (double*)dev_alloc(c, N * 8)) || !(c->diag.g0 = (double*)dev_alloc(c, N * 8)) ||
        !(c->diag.partial = (double*)dev_alloc(c, (size_t)c->diag.npartial * 8)) ||
        !(c->diag.result = (double*)dev_alloc(c, D_NSLOTS * 8))) {
        c->err = "device allocation of diagnostics failed";
        return bail(PIC_ERR_OOM);
    }
    if (launch_zero_f32(g.E, 3 * N, c->stream) || launch_zero_f32(g.B, 3 * N, c->stream) ||
        launch_zero_f32(g.J, 3 * N, c->stream) || launch_zero_i32(g.flags, 16, c->stream) ||
        launch_zero_f64(c->diag.result, D_NSLOTS, c->stream)) {
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
        off += S.n_init;
    }
    for (int s = 0; s < n_species; ++s) {
        if ((rc = alloc_species(c, s))) return bail(rc);
    }
    // one deposit queue shared by the species (their particle kernels run one after another)
    g.qcap = 0;
    for (int s = 0; s < n_species; ++s) g.qcap = std::max(g.qcap, c->sp[s].v.cap);
    if (!(g.qbuf = (float*)dev_alloc(c, (size_t)7 * g.nsc * g.qcap * 4))) {
        c->err = "device allocation of the deposit queue failed";
        return bail(PIC_ERR_OOM);
    }
    for (int s = 0; s < n_species; ++s) {
        Species& S = c->sp[s];
        const pic_species_t& d = S.desc;
        if (d.ppc == 0) continue;
        const double b2 = d.drift_beta[0] * d.drift_beta[0] + d.drift_beta[1] * d.drift_beta[1] +
                          d.drift_beta[2] * d.drift_beta[2];
        const double gam = 1.0 / std::sqrt(1.0 - b2);
        const float drift_u[3] = {(float)(gam * d.drift_beta[0]), (float)(gam * d.drift_beta[1]),
                                  (float)(gam * d.drift_beta[2])};
        int pos_index = s, pos_ppc = d.ppc;
        int64_t pos_off = S.id_offset;
        if (d.coincident_with >= 0) {
            pos_index = d.coincident_with;
            pos_ppc = c->sp[pos_index].desc.ppc;
            pos_off = c->sp[pos_index].id_offset;
        }
        if (launch_init_species(g, S.v, grid->seed, s, d.ppc, S.id_offset, pos_index, pos_ppc, pos_off, (float)d.u_th,
                                drift_u, d.layout, (float)S.weight, d.z_init, c->stream) != hipSuccess) {
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
    const int64_t N = (int64_t)c->grid.nx * c->grid.ny * c->grid.nz;
    const float dt = (float)c->grid.dt;
    for (int it = 0; it < n; ++it) {
        hipEvent_t e0 = nullptr, e1 = nullptr, e2 = nullptr, e3 = nullptr;
        if (c->timing) {
            e0 = next_event(c); e1 = next_event(c); e2 = next_event(c); e3 = next_event(c);
            if (!e0 || !e1 || !e2 || !e3) return fail(c, PIC_ERR_HIP, "event creation failed");
            HIPCHK(c, hipEventRecord(e0, c->stream));
        }
        HIPCHK(c, launch_zero_f32(c->g.J, 3 * N, c->stream));
        for (int s = 0; s < c->nsp; ++s) {
            if (!c->sp[s].desc.mobile) continue;
            HIPCHK(c, launch_push(c->g, c->sp[s].v, c->order, (float)push_vmax(c, s), c->stream));
            c->pending_launches += c->timing ? 1 : 0;
        }
        if (c->timing) HIPCHK(c, hipEventRecord(e1, c->stream));
        for (int s = 0; s < c->nsp; ++s) {
            if (!c->sp[s].desc.mobile) continue;
            HIPCHK(c, launch_migrate(c->g, c->sp[s].v, c->stream));
        }
        if (c->timing) HIPCHK(c, hipEventRecord(e2, c->stream));
        HIPCHK(c, launch_yee_b(c->g, 0.5f * dt, c->stream));
        HIPCHK(c, launch_yee_e(c->g, dt, c->stream));
        HIPCHK(c, launch_yee_b(c->g, 0.5f * dt, c->stream));
        if (c->timing) HIPCHK(c, hipEventRecord(e3, c->stream));
        ++c->step;
    }
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
    const int64_t N = (int64_t)c->grid.nx * c->grid.ny * c->grid.nz;
    HIPCHK(c, launch_zero_f64(c->diag.result, D_NSLOTS, c->stream));
    HIPCHK(c, launch_field_energy(c->g, c->diag, c->stream));
    for (int s = 0; s < c->nsp; ++s) HIPCHK(c, launch_kinetic(c->g, c->sp[s].v, c->diag, s, c->stream));
    HIPCHK(c, launch_zero_f64(c->diag.rho, N, c->stream));
    for (int s = 0; s < c->nsp; ++s) HIPCHK(c, launch_rho_deposit(c->g, c->sp[s].v, c->order, c->diag.rho, c->stream));
    HIPCHK(c, launch_gauss(c->g, c->diag, c->grid.rho_bg, 1, c->stream));
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
    if (out->nonfinite) return fail(c, PIC_ERR_NONFINITE, "%d non-finite field entries", out->nonfinite);
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
    const SpeciesView& sv = c->sp[s].v;
    std::vector<int32_t> cnt;
    const int64_t total = host_count(c, s, cnt);
    if (total < 0) return fail(c, PIC_ERR_HIP, "count readback failed");
    v->count = total;
    if (!v->x || !v->y || !v->z || !v->ux || !v->uy || !v->uz || !v->w || !v->id)
        return fail(c, PIC_ERR_ARG, "view arrays must not be NULL");
    if (v->capacity < total) return fail(c, PIC_ERR_ARG, "view capacity %lld < %lld particles", (long long)v->capacity, (long long)total);
    const size_t n = (size_t)c->g.nsc * sv.cap;
    std::vector<float> a[7];
    const float* src[7] = {sv.x, sv.y, sv.z, sv.ux, sv.uy, sv.uz, sv.w};
    for (int k = 0; k < 7; ++k) {
        a[k].resize(n);
        HIPCHK(c, hipMemcpyAsync(a[k].data(), src[k], n * 4, hipMemcpyDeviceToHost, c->stream));
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
        v->ux[k] = a[3][p];
        v->uy[k] = a[4][p];
        v->uz[k] = a[5][p];
        v->w[k] = a[6][p];
        v->id[k] = ids[p];
        if (v->zstate) v->zstate[k] = sv.zs ? zs[p] : 0;
    }
    return PIC_OK;
}

int pic_set_particles(pic_ctx* c, int s, const pic_particles_view_t* v)
{
    if (!c || !v) return fail(c, PIC_ERR_ARG, "ctx and view must not be NULL");
    if (s < 0 || s >= c->nsp) return fail(c, PIC_ERR_ARG, "species %d out of range", s);
    if (v->count < 0) return fail(c, PIC_ERR_ARG, "negative count");
    if (v->count > 0 && (!v->x || !v->y || !v->z || !v->ux || !v->uy || !v->uz || !v->w || !v->id))
        return fail(c, PIC_ERR_ARG, "view arrays must not be NULL");
    const SpeciesView& sv = c->sp[s].v;
    const GridView& g = c->g;
    const size_t n = (size_t)g.nsc * sv.cap;
    std::vector<int32_t> cnt(g.nsc, 0);
    std::vector<float> a[7];
    for (auto& x : a) x.assign(n, 0.0f);
    std::vector<uint32_t> ids(n, 0);
    std::vector<uint8_t> zs(sv.zs ? n : 0, 0);
    const float lim[3] = {XMAX, YMAX, ZMAX};
    double wmax = 0.0;
    for (int64_t k = 0; k < v->count; ++k) {
        const double p[3] = {v->x[k], v->y[k], v->z[k]};
        const int dims[3] = {g.nx, g.ny, g.nz}, sdim[3] = {SX, SY, SZ};
        int sci[3];
        float rel[3];
        for (int d = 0; d < 3; ++d) {
            if (!(p[d] >= 0.0 && p[d] < (double)dims[d]))
                return fail(c, PIC_ERR_ARG, "particle %lld: position %g outside [0,%d)", (long long)k, p[d], dims[d]);
            sci[d] = (int)std::floor(p[d] / sdim[d]);
            if (sci[d] >= dims[d] / sdim[d]) sci[d] = dims[d] / sdim[d] - 1;
            rel[d] = std::min((float)(p[d] - (double)(sci[d] * sdim[d])), lim[d]);
            if (rel[d] < 0.0f) rel[d] = 0.0f;
        }
        if (!std::isfinite(v->ux[k]) || !std::isfinite(v->uy[k]) || !std::isfinite(v->uz[k]) || !std::isfinite(v->w[k]))
            return fail(c, PIC_ERR_ARG, "particle %lld: non-finite momentum or weight", (long long)k);
        if (v->id[k] < 0 || v->id[k] > 0xFFFFFFFFLL) return fail(c, PIC_ERR_ARG, "particle %lld: id out of range", (long long)k);
        const int sc = sci[0] + g.ncx * (sci[1] + g.ncy * sci[2]);
        if (cnt[sc] >= sv.cap) return fail(c, PIC_ERR_CAPACITY, "supercell %d holds more than %d particles", sc, sv.cap);
        wmax = std::max(wmax, (double)std::fabs(v->w[k]));
        const size_t q = (size_t)sc * sv.cap + cnt[sc]++;
        a[0][q] = rel[0]; a[1][q] = rel[1]; a[2][q] = rel[2];
        a[3][q] = v->ux[k]; a[4][q] = v->uy[k]; a[5][q] = v->uz[k]; a[6][q] = v->w[k];
        ids[q] = (uint32_t)v->id[k];
        if (sv.zs) {
            const int z = v->zstate ? v->zstate[k] : c->sp[s].desc.z_init;
            if (z < 0 || z > c->sp[s].desc.z_max) return fail(c, PIC_ERR_ARG, "particle %lld: charge state out of range", (long long)k);
            zs[q] = (uint8_t)z;
        }
    }
    float* dst[7] = {sv.x, sv.y, sv.z, sv.ux, sv.uy, sv.uz, sv.w};
    for (int k = 0; k < 7; ++k) HIPCHK(c, hipMemcpyAsync(dst[k], a[k].data(), n * 4, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(sv.id, ids.data(), n * 4, hipMemcpyHostToDevice, c->stream));
    if (sv.zs) HIPCHK(c, hipMemcpyAsync(sv.zs, zs.data(), n, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(sv.count, cnt.data(), (size_t)g.nsc * 4, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    c->sp[s].wmax = wmax;
    return PIC_OK;
}

int pic_get_fields(pic_ctx* c, float* E, float* B, float* J)
{
    if (!c) return fail(nullptr, PIC_ERR_ARG, "ctx is NULL");
    const size_t bytes = (size_t)3 * c->grid.nx * c->grid.ny * c->grid.nz * 4;
    if (E) HIPCHK(c, hipMemcpyAsync(E, c->g.E, bytes, hipMemcpyDeviceToHost, c->stream));
    if (B) HIPCHK(c, hipMemcpyAsync(B, c->g.B, bytes, hipMemcpyDeviceToHost, c->stream));
    if (J) HIPCHK(c, hipMemcpyAsync(J, c->g.J, bytes, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return PIC_OK;
}

int pic_set_fields(pic_ctx* c, const float* E, const float* B, const float* J)
{
    if (!c) return fail(nullptr, PIC_ERR_ARG, "ctx is NULL");
    const size_t n3 = (size_t)3 * c->grid.nx * c->grid.ny * c->grid.nz;
    for (const float* f : {E, B, J})
        if (f)
            for (size_t i = 0; i < n3; ++i)
                if (!std::isfinite(f[i])) return fail(c, PIC_ERR_ARG, "non-finite field value at %zu", i);
    if (E) HIPCHK(c, hipMemcpyAsync(c->g.E, E, n3 * 4, hipMemcpyHostToDevice, c->stream));
    if (B) HIPCHK(c, hipMemcpyAsync(c->g.B, B, n3 * 4, hipMemcpyHostToDevice, c->stream));
    if (J) HIPCHK(c, hipMemcpyAsync(c->g.J, J, n3 * 4, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return PIC_OK;
}

}  // extern "C"
