// Monte Carlo electron-impact ionisation: per-cell electron moments, the
// exact Maxwellian-averaged Lotz rate by 64-point Gauss-Laguerre quadrature
// in FP64, the Philox draw per ion and the append of the new electrons to
// the ion's own supercell.
#include "ionize_internal.hpp"

namespace pic {

// ---------------------------------------------------------------- moments
// Nearest-grid-point moments of one species per cell (sum w, sum w u,
// sum w |u|^2) accumulated in FP64 in LDS, one workgroup per supercell, then
// n_e = (sum w / dV) n_ref and kT = m_e c^2 (sum w u^2 / N - |ubar|^2) / 3;
// with mom4, also N = sum w and ubar per cell.
__global__ __launch_bounds__(BLOCK) void k_moments(GridView g, SpeciesView e, double n_ref_over_dv, double* ne,
                                                   double* kT, double* mom4)
{
    __shared__ double acc[5][SC_CELLS];
    const int sc = blockIdx.x;
    const int tid = threadIdx.x;
#pragma unroll
    for (int k = 0; k < 5; ++k) acc[k][tid] = 0.0;
    __syncthreads();
    const int n = e.count[sc];
    const int64_t base = (int64_t)sc * e.cap;
#pragma unroll 4
    for (int t = tid; t < n; t += BLOCK) {
        const int64_t p = base + t;
        const int cell = (int)e.x[p] + SX * ((int)e.y[p] + SY * (int)e.z[p]);
        const double w = e.w[p], ux = e.ux[p], uy = e.uy[p], uz = e.uz[p];
        atomicAdd(&acc[0][cell], w);
        atomicAdd(&acc[1][cell], w * ux);
        atomicAdd(&acc[2][cell], w * uy);
        atomicAdd(&acc[3][cell], w * uz);
        atomicAdd(&acc[4][cell], w * (ux * ux + uy * uy + uz * uz));
    }
    __syncthreads();
    const int scx = sc % g.ncx, scy = (sc / g.ncx) % g.ncy, scz = sc / (g.ncx * g.ncy);
    const int lx = tid & 7, ly = (tid >> 3) & 7, lz = tid >> 6;
    const int64_t gi = (int64_t)(scx * SX + lx) + (int64_t)g.nx * ((scy * SY + ly) + (int64_t)g.ny * (scz * SZ + lz));
    const double N = acc[0][tid];
    double t_ev = 0.0, n_cm3 = 0.0, bx = 0.0, by = 0.0, bz = 0.0;
    if (N > 0.0) {
        bx = acc[1][tid] / N, by = acc[2][tid] / N, bz = acc[3][tid] / N;
        t_ev = ME_C2_EV * (acc[4][tid] / N - (bx * bx + by * by + bz * bz)) / 3.0;
        t_ev = t_ev > 0.0 ? t_ev : 0.0;
        n_cm3 = N * n_ref_over_dv;
    }
    ne[gi] = n_cm3;
    kT[gi] = t_ev;
    if (mom4) {
        mom4[4 * gi] = N;
        mom4[4 * gi + 1] = bx;
        mom4[4 * gi + 2] = by;
        mom4[4 * gi + 3] = bz;
    }
}

hipError_t launch_moments(const GridView& g, const SpeciesView& e, double n_ref_over_dv, double* ne, double* kT,
                          double* mom4, hipStream_t st)
{
    hipLaunchKernelGGL(k_moments, dim3(g.nsc), dim3(BLOCK), 0, st, g, e, n_ref_over_dv, ne, kT, mom4);
    return hipGetLastError();
}

// ---------------------------------------------------------------- exact rate
__global__ __launch_bounds__(BLOCK) void k_rate_exact(GridView g, SpeciesView ion, IonTables tab, const double* ne,
                                                      const double* kT, double* nu, const double* gl)
{
    __shared__ double glx[GL_NODES], glw[GL_NODES];
    const int sc = blockIdx.x;
    const int tid = threadIdx.x;
    if (tid < GL_NODES) { glx[tid] = gl[tid]; glw[tid] = gl[GL_NODES + tid]; }
    __syncthreads();
    const int n = ion.count[sc];
    const int64_t base = (int64_t)sc * ion.cap;
    const int scx = sc % g.ncx, scy = (sc / g.ncx) % g.ncy, scz = sc / (g.ncx * g.ncy);
    for (int t = tid; t < n; t += BLOCK) {
        const int64_t p = base + t;
        const int Z = ion.zs[p];
        double v = 0.0;
        if (Z < tab.z_max) {
            const int64_t gi = (int64_t)(scx * SX + (int)ion.x[p]) +
                               (int64_t)g.nx * ((scy * SY + (int)ion.y[p]) + (int64_t)g.ny * (scz * SZ + (int)ion.z[p]));
            v = rate_exact(kT[gi], ne[gi], tab, Z, glx, glw);
        }
        nu[p] = v;
    }
}

hipError_t launch_rate_exact(const GridView& g, const SpeciesView& ion, const IonTables& tab, const double* ne,
                             const double* kT, double* nu, const double* gl, hipStream_t st)
{
    hipLaunchKernelGGL(k_rate_exact, dim3(g.nsc), dim3(BLOCK), 0, st, g, ion, tab, ne, kT, nu, gl);
    return hipGetLastError();
}

// Exact ln nu for independent samples (rate evaluation entry point).
__global__ __launch_bounds__(BLOCK) void k_ln_rate_exact(int64_t n, const double* kT, const double* ne,
                                                         const int32_t* Z, IonTables tab, const double* gl,
                                                         double* out)
{
    __shared__ double glx[GL_NODES], glw[GL_NODES];
    if (threadIdx.x < GL_NODES) { glx[threadIdx.x] = gl[threadIdx.x]; glw[threadIdx.x] = gl[GL_NODES + threadIdx.x]; }
    __syncthreads();
    const int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (i >= n) return;
    const int z = Z[i];
    out[i] = (z >= 0 && z < tab.z_max) ? ln_rate_exact(kT[i], ne[i], tab, z, glx, glw) : -INFINITY;
}

hipError_t launch_ln_rate_exact(int64_t n, const double* kT, const double* ne, const int32_t* Z, const IonTables& tab,
                                const double* gl, double* out, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_ln_rate_exact, dim3((unsigned)((n + BLOCK - 1) / BLOCK)), dim3(BLOCK), 0, st, n, kT, ne, Z,
                       tab, gl, out);
    return hipGetLastError();
}

// ---------------------------------------------------------------- draw + append
__device__ inline uint64_t word(const Philox4& r, int e)
{
    return e == 0 ? r.v[0] : e == 1 ? r.v[1] : e == 2 ? r.v[2] : r.v[3];
}

// Events of one ion.  One event: the Philox uniform u_0 of (id, species, 2,
// step) below p = 1 - exp(-nu dt_phys).  Several: the waiting-time chain,
// event e adding -ln(1 - u_e) / nu_{Z+e} while the running time stays below
// dt_phys; u_e is word e % 4 of the block of (id, species, 2, step) for e < 4
// and of (id, species, 6, step) after; later events take the exact rate.
template <bool CHAIN>
__device__ inline int ion_events(const IonTables& tab, const DrawArgs& a, uint32_t id, int Z0, double nu0, double kT,
                                 double ne, const double* glx, const double* glw)
{
    const Philox4 r = philox4x64_10((uint64_t)id, (uint64_t)a.species_index, PURPOSE_IONIZE, (uint64_t)a.step, a.seed, 0);
    if constexpr (!CHAIN) return u01(r.v[0]) < -expm1(-nu0 * a.dt_phys) ? 1 : 0;
    Philox4 r2{};
    double t = 0.0;
    int nev = 0;
    for (int e = 0; e < a.max_events && Z0 + e < tab.z_max; ++e) {
        const double rate = e == 0 ? nu0 : rate_exact(kT, ne, tab, Z0 + e, glx, glw);
        if (!(rate > 0.0)) break;
        if (e == 4)
            r2 = philox4x64_10((uint64_t)id, (uint64_t)a.species_index, PURPOSE_IONIZE_MORE, (uint64_t)a.step, a.seed, 0);
        const double u = u01(e < 4 ? word(r, e) : word(r2, e - 4));
        t += -log1p(-u) / rate;
        if (!(t < a.dt_phys)) break;
        ++nev;
    }
    return nev;
}

// Per ion with Z < z_max (counted, striped, at CNT_ACTIVE): its events, then
// one electron per event at the end of the same supercell's electron frames
// (one LDS atomic per ion with events), with the position, momentum and
// weight of the ion; the charge state rises by the events that found a slot.
// With energy loss, w * P_Z of those events goes to the cell's de and the
// supercell's electron count before the appends to old_count.
// CHAIN: max_events > 1 (the instantiation for one event carries no quadrature).
template <bool CHAIN>
__global__ __launch_bounds__(BLOCK) void k_draw_append(GridView g, SpeciesView ion, SpeciesView el, IonTables tab,
                                                       DrawArgs a, const double* nu, DrawBuffers db,
                                                       unsigned long long* counters)
{
    __shared__ double glx[GL_NODES], glw[GL_NODES];
    __shared__ int s_add, s_fired, s_active;
    const int sc = blockIdx.x;
    const int tid = threadIdx.x;
    if (CHAIN && tid < GL_NODES) { glx[tid] = db.gl[tid]; glw[tid] = db.gl[GL_NODES + tid]; }
    if (tid == 0) { s_add = 0; s_fired = 0; s_active = 0; }
    __syncthreads();
    const int n = ion.count[sc];
    const int ebase = el.count[sc];
    const int room = el.cap - ebase;
    const int64_t base = (int64_t)sc * ion.cap;
    const int64_t ebase64 = (int64_t)sc * el.cap;
    const int scx = sc % g.ncx, scy = (sc / g.ncx) % g.ncy, scz = sc / (g.ncx * g.ncy);
    bool full = false;
    int fired = 0, active = 0;
    // chunks of DRAW_PER slots per lane: every load of a chunk is issued
    // before the first decision, so the lanes wait on memory once per chunk
    constexpr int DRAW_PER = 4;
    for (int c0 = 0; c0 < n; c0 += BLOCK * DRAW_PER) {
        int zs[DRAW_PER];
        uint32_t ids[DRAW_PER];
        double nus[DRAW_PER];
#pragma unroll
        for (int k = 0; k < DRAW_PER; ++k) {
            const int t = c0 + k * BLOCK + tid;
            zs[k] = tab.z_max;  // inactive
            ids[k] = 0;
            nus[k] = 0.0;
            if (t < n) {
                const int64_t p = base + t;
                zs[k] = ion.zs[p];
                ids[k] = ion.id[p];
                nus[k] = nu[p];
            }
        }
#pragma unroll
        for (int k = 0; k < DRAW_PER; ++k) {
            const int Z0 = zs[k];
            if (Z0 >= tab.z_max) continue;
            ++active;
            const int64_t p = base + c0 + k * BLOCK + tid;
            // the ion's cell, for later events' rates and the energy account only
            const bool need_cell = CHAIN || a.energy_loss;
            const int64_t gi = need_cell ? (int64_t)(scx * SX + (int)ion.x[p]) +
                                               (int64_t)g.nx * ((scy * SY + (int)ion.y[p]) +
                                                                (int64_t)g.ny * (scz * SZ + (int)ion.z[p]))
                                         : 0;
            const uint32_t id = ids[k];
            const int nev = ion_events<CHAIN>(tab, a, id, Z0, nus[k], CHAIN ? db.kT[gi] : 0.0,
                                              CHAIN ? db.ne[gi] : 0.0, glx, glw);
            if (nev == 0) continue;
            const int b = atomicAdd(&s_add, nev);
            int done = 0;
            double dE = 0.0;
            for (int e = 0; e < nev; ++e) {
                const int kk = b + e;
                if (kk >= room) { full = true; break; }
                const int64_t q = ebase64 + ebase + kk;
                const int znew = Z0 + e + 1;
                el.x[q] = ion.x[p]; el.y[q] = ion.y[p]; el.z[q] = ion.z[p];
                el.ux[q] = ion.ux[p]; el.uy[q] = ion.uy[p]; el.uz[q] = ion.uz[p];
                el.w[q] = ion.w[p];
                el.id[q] = (uint32_t)(a.id_base_new + (int64_t)(id - (uint32_t)a.ion_id_offset) * tab.z_max +
                                      (znew - 1));
                dE += tab.P[Z0 + e];
                ++done;
            }
            if (done) {
                ion.zs[p] = (uint8_t)(Z0 + done);
                fired += done;
                if (a.energy_loss) atomicAdd(&db.de[gi], (double)ion.w[p] * dE);
            }
        }
    }
    if (full) g.flags[FLAG_CAPACITY] = 1;
    if (fired) atomicAdd(&s_fired, fired);
    if (active) atomicAdd(&s_active, active);
    __syncthreads();
    if (tid == 0) {
        if (s_active) atomicAdd(&counters[CNT_ACTIVE + sc % CNT_STRIPES], (unsigned long long)s_active);
        const int added = s_add < room ? s_add : room;
        el.count[sc] = ebase + added;
        if (a.energy_loss) db.old_count[sc] = ebase;
        if (s_fired) atomicAdd(&counters[CNT_FIRED + sc % CNT_STRIPES], (unsigned long long)s_fired);
    }
}

hipError_t launch_draw_append(const GridView& g, const SpeciesView& ion, const SpeciesView& el, const IonTables& tab,
                              const DrawArgs& a, const double* nu, const DrawBuffers& b, unsigned long long* counters,
                              hipStream_t st)
{
    if (a.energy_loss && (!b.de || !b.old_count || !b.mom4)) return hipErrorInvalidValue;
    if (a.max_events > 1)
        hipLaunchKernelGGL(k_draw_append<true>, dim3(g.nsc), dim3(BLOCK), 0, st, g, ion, el, tab, a, nu, b, counters);
    else
        hipLaunchKernelGGL(k_draw_append<false>, dim3(g.nsc), dim3(BLOCK), 0, st, g, ion, el, tab, a, nu, b, counters);
    return hipGetLastError();
}

// ---------------------------------------------------------------- energy loss
// The electrons present before the appends (slots below old_count) of a cell
// with de > 0 and 3/2 N kT > 0: u <- ubar + f (u - ubar),
// f = sqrt(max(0, 1 - de / (3/2 N kT))), in FP64.
__global__ __launch_bounds__(BLOCK) void k_energy_loss(GridView g, SpeciesView el, DrawBuffers db)
{
    const int sc = blockIdx.x;
    const int n = db.old_count[sc];
    const int64_t base = (int64_t)sc * el.cap;
    const int scx = sc % g.ncx, scy = (sc / g.ncx) % g.ncy, scz = sc / (g.ncx * g.ncy);
    for (int t = threadIdx.x; t < n; t += BLOCK) {
        const int64_t p = base + t;
        const int64_t gi = (int64_t)(scx * SX + (int)el.x[p]) +
                           (int64_t)g.nx * ((scy * SY + (int)el.y[p]) + (int64_t)g.ny * (scz * SZ + (int)el.z[p]));
        const double d = db.de[gi];
        if (!(d > 0.0)) continue;
        const double heat = 1.5 * db.mom4[4 * gi] * db.kT[gi];
        if (!(heat > 0.0)) continue;
        const double f2 = 1.0 - d / heat;
        const double f = f2 > 0.0 ? sqrt(f2) : 0.0;
        const double bx = db.mom4[4 * gi + 1], by = db.mom4[4 * gi + 2], bz = db.mom4[4 * gi + 3];
        el.ux[p] = (float)(bx + f * ((double)el.ux[p] - bx));
        el.uy[p] = (float)(by + f * ((double)el.uy[p] - by));
        el.uz[p] = (float)(bz + f * ((double)el.uz[p] - bz));
    }
}

hipError_t launch_energy_loss(const GridView& g, const SpeciesView& el, const DrawBuffers& b, hipStream_t st)
{
    if (!b.de || !b.old_count || !b.mom4) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_energy_loss, dim3(g.nsc), dim3(BLOCK), 0, st, g, el, b);
    return hipGetLastError();
}

}  // namespace pic
