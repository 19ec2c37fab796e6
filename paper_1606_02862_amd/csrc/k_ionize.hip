// Monte Carlo electron-impact ionisation: per-cell electron moments, the
// exact Maxwellian-averaged Lotz rate by 64-point Gauss-Laguerre quadrature
// in FP64, the Philox draw per ion and the append of the new electrons to
// the ion's own supercell.
#include "ionize_step.hpp"

namespace pic {

// ---------------------------------------------------------------- moments
// Nearest-grid-point moments of one species per cell (sum w, sum w u,
// sum w |u|^2) accumulated in FP64 in LDS, one workgroup per supercell, then
// n_e = (sum w / dV) n_ref and kT = m_e c^2 (sum w u^2 / N - |ubar|^2) / 3;
// with mom4, also N = sum w and ubar per cell.
__global__ __launch_bounds__(BLOCK) void k_moments(GridView g, SpeciesView e, double n_ref_over_dv, double* ne,
                                                   double* kT, double* mom4)
{
    __shared__ MomLds m;
    const int sc = blockIdx.x;
    moments_accumulate(e, sc, m);
    const int cell = threadIdx.x;
    moments_store(moments_cell(m, cell, n_ref_over_dv), cell_index(g, sc, cell), ne, kT, mom4);
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
    __shared__ DrawLds s_d;
    const int sc = blockIdx.x;
    const int tid = threadIdx.x;
    if (CHAIN && tid < GL_NODES) { glx[tid] = db.gl[tid]; glw[tid] = db.gl[GL_NODES + tid]; }
    if (tid == 0) s_d = DrawLds{0, 0, 0};
    __syncthreads();
    const int n = ion.count[sc];
    const int ebase = el.count[sc];
    const int room = el.cap - ebase;
    const int64_t base = (int64_t)sc * ion.cap;
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
            const int64_t p = base + c0 + k * BLOCK + tid;
            int nev = 0;
            int64_t gi = 0;
            if (Z0 < tab.z_max) {
                ++active;
                // the ion's cell, for later events' rates and the energy account only
                if (CHAIN || a.energy_loss)
                    gi = (int64_t)(scx * SX + (int)ion.x[p]) +
                         (int64_t)g.nx * ((scy * SY + (int)ion.y[p]) + (int64_t)g.ny * (scz * SZ + (int)ion.z[p]));
                nev = ion_events<CHAIN>(tab, a, ids[k], Z0, nus[k], CHAIN ? db.kT[gi] : 0.0, CHAIN ? db.ne[gi] : 0.0,
                                        glx, glw);
            }
            const int b = wave_reserve<CHAIN>(nev, &s_d.add);  // every lane of the wave
            if (nev) fired += append_events(ion, el, tab, a, db.de, sc, p, gi, ids[k], Z0, nev, b, ebase, room, full);
        }
    }
    if (full) g.flags[FLAG_CAPACITY] = 1;
    if (fired) atomicAdd(&s_d.fired, fired);
    if (active) atomicAdd(&s_d.active, active);
    __syncthreads();
    if (tid == 0) draw_finish(el, a, db, sc, ebase, room, s_d, counters);
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

// One ionisation step of one ion species with the exact rate, fused per
// supercell (one workgroup each): the electron moments of its cells in LDS
// (written to the grid as well), then for each of its ions the exact rate
// from its cell's moments and the draw and append of its events.
template <bool CHAIN>
__global__ __launch_bounds__(BLOCK) void k_ionize_exact(GridView g, SpeciesView ion, SpeciesView el, IonTables tab,
                                                        DrawArgs a, DrawBuffers db, double n_ref_over_dv, double* ne,
                                                        double* kT, double* mom4, unsigned long long* counters)
{
    __shared__ MomLds mom;
    __shared__ double glx[GL_NODES], glw[GL_NODES];
    __shared__ DrawLds s_d;
    const int sc = blockIdx.x;
    const int tid = threadIdx.x;
    if (tid < GL_NODES) { glx[tid] = db.gl[tid]; glw[tid] = db.gl[GL_NODES + tid]; }
    if (tid == 0) s_d = DrawLds{0, 0, 0};
    moments_accumulate(el, sc, mom);  // its barriers also publish the rule and the reset above
    {
        // each thread reads and rewrites only its own cell's column
        const CellMoments cm = moments_cell(mom, tid, n_ref_over_dv);
        moments_store(cm, cell_index(g, sc, tid), ne, kT, mom4);
        mom.acc[0][tid] = cm.ne;
        mom.acc[1][tid] = cm.kT;
    }
    __syncthreads();
    const int n = ion.count[sc];
    const int ebase = el.count[sc];
    const int room = el.cap - ebase;
    const int64_t base = (int64_t)sc * ion.cap;
    bool full = false;
    int fired = 0, active = 0;
    for (int t0 = 0; t0 < n; t0 += BLOCK) {  // every lane runs every pass (the appends are per wave)
        const int t = t0 + tid;
        const int64_t p = base + t;
        const int Z = t < n ? (int)ion.zs[p] : tab.z_max;
        int nev = 0, cell = 0;
        uint32_t id = 0;
        if (Z < tab.z_max) {
            ++active;
            cell = (int)ion.x[p] + SX * ((int)ion.y[p] + SY * (int)ion.z[p]);
            const double cne = mom.acc[0][cell], ckT = mom.acc[1][cell];
            const double nu0 = rate_exact(ckT, cne, tab, Z, glx, glw);
            id = ion.id[p];
            nev = ion_events<CHAIN>(tab, a, id, Z, nu0, ckT, cne, glx, glw);
        }
        const int b = wave_reserve<CHAIN>(nev, &s_d.add);
        if (nev) {
            const int64_t gi = a.energy_loss ? cell_index(g, sc, cell) : 0;
            fired += append_events(ion, el, tab, a, db.de, sc, p, gi, id, Z, nev, b, ebase, room, full);
        }
    }
    if (full) g.flags[FLAG_CAPACITY] = 1;
    if (fired) atomicAdd(&s_d.fired, fired);
    if (active) atomicAdd(&s_d.active, active);
    __syncthreads();
    if (tid == 0) draw_finish(el, a, db, sc, ebase, room, s_d, counters);
}

hipError_t launch_ionize_exact(const GridView& g, const SpeciesView& ion, const SpeciesView& el, const IonTables& tab,
                               const DrawArgs& a, const DrawBuffers& db, double n_ref_over_dv, double* ne, double* kT,
                               double* mom4, unsigned long long* counters, hipStream_t st)
{
    if (a.energy_loss && (!db.de || !db.old_count || !mom4)) return hipErrorInvalidValue;
    if (a.max_events > 1)
        hipLaunchKernelGGL(k_ionize_exact<true>, dim3(g.nsc), dim3(BLOCK), 0, st, g, ion, el, tab, a, db, n_ref_over_dv,
                           ne, kT, mom4, counters);
    else
        hipLaunchKernelGGL(k_ionize_exact<false>, dim3(g.nsc), dim3(BLOCK), 0, st, g, ion, el, tab, a, db,
                           n_ref_over_dv, ne, kT, mom4, counters);
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
