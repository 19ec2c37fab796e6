// Device code of one ionisation step shared by the staged kernels (cell
// moments, rate and draw as three launches over the whole grid) and the fused
// ones (all three for one supercell in one workgroup): the supercell's
// electron moments in LDS, the events of one ion and the append of their
// electrons.
#pragma once

#include "ionize_internal.hpp"

namespace pic {

static_assert(BLOCK == SC_CELLS, "one thread per cell of a supercell in the moments");

// ---------------------------------------------------------------- moments
// Per cell of one supercell: sum w, sum w ux, sum w uy, sum w uz, sum w |u|^2.
struct MomLds {
    double acc[5][SC_CELLS];
};

// Nearest-grid-point sums of the supercell's electrons, accumulated in FP64
// by LDS atomics.  Every thread of the workgroup calls it; it starts and
// ends with a barrier.  The electrons are read once per step: non-temporal
// loads keep them from displacing what the caches hold for the other stages.
__device__ inline void moments_accumulate(const SpeciesView& e, int sc, MomLds& m)
{
    auto ld = [](const auto& a) { return __builtin_nontemporal_load(&a); };
    const int tid = threadIdx.x;
#pragma unroll
    for (int k = 0; k < 5; ++k) m.acc[k][tid] = 0.0;
    __syncthreads();
    const int n = e.count[sc];
    const int64_t base = (int64_t)sc * e.cap;
#pragma unroll 4
    for (int t = tid; t < n; t += BLOCK) {
        const int64_t p = base + t;
        const int cell = (int)ld(e.x[p]) + SX * ((int)ld(e.y[p]) + SY * (int)ld(e.z[p]));
        const double w = ld(e.w[p]), ux = ld(e.ux[p]), uy = ld(e.uy[p]), uz = ld(e.uz[p]);
        atomicAdd(&m.acc[0][cell], w);
        atomicAdd(&m.acc[1][cell], w * ux);
        atomicAdd(&m.acc[2][cell], w * uy);
        atomicAdd(&m.acc[3][cell], w * uz);
        atomicAdd(&m.acc[4][cell], w * (ux * ux + uy * uy + uz * uz));
    }
    __syncthreads();
}

// The cell's n_e = (sum w / dV) n_ref and kT = m_e c^2 (sum w u^2 / N -
// |ubar|^2) / 3 (0 for an empty cell), and N = sum w and ubar.
struct CellMoments {
    double ne, kT, N, bx, by, bz;
};

__device__ inline CellMoments moments_cell(const MomLds& m, int cell, double n_ref_over_dv)
{
    CellMoments r{0.0, 0.0, m.acc[0][cell], 0.0, 0.0, 0.0};
    if (r.N > 0.0) {
        r.bx = m.acc[1][cell] / r.N, r.by = m.acc[2][cell] / r.N, r.bz = m.acc[3][cell] / r.N;
        const double t_ev = ME_C2_EV * (m.acc[4][cell] / r.N - (r.bx * r.bx + r.by * r.by + r.bz * r.bz)) / 3.0;
        r.kT = t_ev > 0.0 ? t_ev : 0.0;
        r.ne = r.N * n_ref_over_dv;
    }
    return r;
}

// Grid index of cell `cell` (x fastest) of supercell sc.
__device__ inline int64_t cell_index(const GridView& g, int sc, int cell)
{
    const int scx = sc % g.ncx, scy = (sc / g.ncx) % g.ncy, scz = sc / (g.ncx * g.ncy);
    const int lx = cell & 7, ly = (cell >> 3) & 7, lz = cell >> 6;
    return (int64_t)(scx * SX + lx) + (int64_t)g.nx * ((scy * SY + ly) + (int64_t)g.ny * (scz * SZ + lz));
}

// Writes the cell's n_e and kT (and, with mom4, N and ubar) to the grid.
__device__ inline void moments_store(const CellMoments& c, int64_t gi, double* ne, double* kT, double* mom4)
{
    ne[gi] = c.ne;
    kT[gi] = c.kT;
    if (mom4) {
        mom4[4 * gi] = c.N;
        mom4[4 * gi + 1] = c.bx;
        mom4[4 * gi + 2] = c.by;
        mom4[4 * gi + 3] = c.bz;
    }
}

// ---------------------------------------------------------------- events
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

// Stream compaction of the appends: every lane of the wave calls it with its
// ion's event count (0 without events or without an ion).  The lanes' slots
// follow from an exclusive prefix sum over the wave (a ballot and a bit count
// when CHAIN is false and every count is 0 or 1), and the wave's block of
// slots from one LDS atomic on *s_add (the supercell's appends so far).
// Returns the lane's first slot index (relative to the supercell's electrons
// before the step).
template <bool CHAIN>
__device__ inline int wave_reserve(int nev, int* s_add)
{
    const int lane = threadIdx.x & 63;
    int incl, total;
    if constexpr (CHAIN) {
        incl = nev;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int v = __shfl_up(incl, o, 64);
            if (lane >= o) incl += v;
        }
        total = __shfl(incl, 63, 64);
    } else {
        const unsigned long long m = __ballot(nev != 0);
        incl = __popcll(m & (~0ull >> (63 - lane)));
        total = __popcll(m);
    }
    int b = 0;
    if (total) {  // wave-uniform
        if (lane == 0) b = atomicAdd(s_add, total);
        b = __shfl(b, 0, 64);
    }
    return b + incl - nev;
}

// The electrons of an ion's nev events, appended after the supercell's
// electron frames from slot index b (wave_reserve), at most `room` in all
// (the rest set `full`).  Each carries the ion's position, momentum and
// weight and the id id_base_new + (ion id - ion_id_offset) z_max + Z - 1 of
// the charge state Z it creates.  The ion's charge state rises by the events
// that found a slot; with energy loss, w times their ionisation energies goes
// to the cell's de.  Returns that count.
__device__ inline int append_events(const SpeciesView& ion, const SpeciesView& el, const IonTables& tab,
                                    const DrawArgs& a, double* de, int sc, int64_t p, int64_t gi, uint32_t id, int Z0,
                                    int nev, int b, int ebase, int room, bool& full)
{
    int done = 0;
    double dE = 0.0;
    for (int e = 0; e < nev; ++e) {
        const int kk = b + e;
        if (kk >= room) {
            full = true;
            break;
        }
        const int64_t q = (int64_t)sc * el.cap + ebase + kk;
        const int znew = Z0 + e + 1;
        el.x[q] = ion.x[p]; el.y[q] = ion.y[p]; el.z[q] = ion.z[p];
        el.ux[q] = ion.ux[p]; el.uy[q] = ion.uy[p]; el.uz[q] = ion.uz[p];
        el.w[q] = ion.w[p];
        el.id[q] = (uint32_t)(a.id_base_new + (int64_t)(id - (uint32_t)a.ion_id_offset) * tab.z_max + (znew - 1));
        dE += tab.P[Z0 + e];
        ++done;
    }
    if (done) {
        ion.zs[p] = (uint8_t)(Z0 + done);
        if (a.energy_loss) atomicAdd(&de[gi], (double)ion.w[p] * dE);
    }
    return done;
}

// Per-supercell bookkeeping of the draw, in LDS.
struct DrawLds {
    int add, fired, active;
};

// After the supercell's last append (behind a barrier): its electron count,
// the energy-loss count before the appends, and the striped counters.
__device__ inline void draw_finish(const SpeciesView& el, const DrawArgs& a, const DrawBuffers& db, int sc, int ebase,
                                   int room, const DrawLds& d, unsigned long long* counters)
{
    if (d.active) atomicAdd(&counters[CNT_ACTIVE + sc % CNT_STRIPES], (unsigned long long)d.active);
    const int added = d.add < room ? d.add : room;
    el.count[sc] = ebase + added;
    if (a.energy_loss) db.old_count[sc] = ebase;
    if (d.fired) atomicAdd(&counters[CNT_FIRED + sc % CNT_STRIPES], (unsigned long long)d.fired);
}

}  // namespace pic
