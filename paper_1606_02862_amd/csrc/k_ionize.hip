// Monte Carlo electron-impact ionisation: per-cell electron moments, the
// exact Maxwellian-averaged Lotz rate by 64-point Gauss-Laguerre quadrature
// in FP64, the Philox draw per ion and the append of the new electrons to
// the ion's own supercell.
#include "pic_device.hpp"

namespace pic {

// ---------------------------------------------------------------- moments
// Nearest-grid-point moments of one species per cell (sum w, sum w u,
// sum w |u|^2) accumulated in FP64 in LDS, one workgroup per supercell, then
// n_e = (sum w / dV) n_ref and kT = m_e c^2 (sum w u^2 / N - |ubar|^2) / 3.
__global__ __launch_bounds__(BLOCK) void k_moments(GridView g, SpeciesView e, double n_ref_over_dv, double* ne,
                                                   double* kT)
{
    __shared__ double acc[5][SC_CELLS];
    const int sc = blockIdx.x;
    const int tid = threadIdx.x;
#pragma unroll
    for (int k = 0; k < 5; ++k) acc[k][tid] = 0.0;
    __syncthreads();
    const int n = e.count[sc];
    const int64_t base = (int64_t)sc * e.cap;
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
    double t_ev = 0.0, n_cm3 = 0.0;
    if (N > 0.0) {
        const double bx = acc[1][tid] / N, by = acc[2][tid] / N, bz = acc[3][tid] / N;
        t_ev = ME_C2_EV * (acc[4][tid] / N - (bx * bx + by * by + bz * bz)) / 3.0;
        t_ev = t_ev > 0.0 ? t_ev : 0.0;
        n_cm3 = N * n_ref_over_dv;
    }
    ne[gi] = n_cm3;
    kT[gi] = t_ev;
}

hipError_t launch_moments(const GridView& g, const SpeciesView& e, double n_ref_over_dv, double* ne, double* kT,
                          hipStream_t st)
{
    hipLaunchKernelGGL(k_moments, dim3(g.nsc), dim3(BLOCK), 0, st, g, e, n_ref_over_dv, ne, kT);
    return hipGetLastError();
}

// ---------------------------------------------------------------- exact rate
__global__ __launch_bounds__(BLOCK) void k_rate_exact(GridView g, SpeciesView ion, IonTables tab, const double* ne,
                                                      const double* kT, double* nu, const double* gl,
                                                      unsigned long long* counters)
{
    __shared__ double glx[GL_NODES], glw[GL_NODES];
    __shared__ int s_active;
    const int sc = blockIdx.x;
    const int tid = threadIdx.x;
    if (tid < GL_NODES) { glx[tid] = gl[tid]; glw[tid] = gl[GL_NODES + tid]; }
    if (tid == 0) s_active = 0;
    __syncthreads();
    const int n = ion.count[sc];
    const int64_t base = (int64_t)sc * ion.cap;
    const int scx = sc % g.ncx, scy = (sc / g.ncx) % g.ncy, scz = sc / (g.ncx * g.ncy);
    int active = 0;
    for (int t = tid; t < n; t += BLOCK) {
        const int64_t p = base + t;
        const int Z = ion.zs[p];
        double v = 0.0;
        if (Z < tab.z_max) {
            ++active;
            const int64_t gi = (int64_t)(scx * SX + (int)ion.x[p]) +
                               (int64_t)g.nx * ((scy * SY + (int)ion.y[p]) + (int64_t)g.ny * (scz * SZ + (int)ion.z[p]));
            v = rate_exact(kT[gi], ne[gi], tab.P[Z], tab.q[Z], glx, glw);
        }
        nu[p] = v;
    }
    atomicAdd(&s_active, active);
    __syncthreads();
    if (tid == 0 && s_active) atomicAdd(&counters[0], (unsigned long long)s_active);
}

hipError_t launch_rate_exact(const GridView& g, const SpeciesView& ion, const IonTables& tab, const double* ne,
                             const double* kT, double* nu, const double* gl, unsigned long long* counters,
                             hipStream_t st)
{
    hipLaunchKernelGGL(k_rate_exact, dim3(g.nsc), dim3(BLOCK), 0, st, g, ion, tab, ne, kT, nu, gl, counters);
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
    out[i] = (z >= 0 && z < tab.z_max) ? ln_rate_exact(kT[i], ne[i], tab.P[z], tab.q[z], glx, glw) : -INFINITY;
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
// p = 1 - exp(-nu dt_phys); the ion ionises when its Philox uniform
// (id, species, 2, step) is below p.  The new electron takes a slot at the end
// of the same supercell's electron frames (wave ballot + one LDS atomic per
// wave), position / momentum / weight of the ion.
__global__ __launch_bounds__(BLOCK) void k_draw_append(GridView g, SpeciesView ion, SpeciesView el, IonTables tab,
                                                       DrawArgs a, const double* nu, unsigned long long* counters)
{
    __shared__ int s_add, s_fired;
    const int sc = blockIdx.x;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    if (tid == 0) { s_add = 0; s_fired = 0; }
    __syncthreads();
    const int n = ion.count[sc];
    const int ebase = el.count[sc];
    const int room = el.cap - ebase;
    const int64_t base = (int64_t)sc * ion.cap;
    const int64_t ebase64 = (int64_t)sc * el.cap;
    bool full = false;
    for (int f = 0; f < n; f += BLOCK) {
        const int t = f + tid;
        bool fire = false;
        int64_t p = 0;
        if (t < n) {
            p = base + t;
            const int Z = ion.zs[p];
            if (Z < tab.z_max) {
                const double prob = -expm1(-nu[p] * a.dt_phys);
                const Philox4 r = philox4x64_10((uint64_t)ion.id[p], (uint64_t)a.species_index, PURPOSE_IONIZE,
                                                (uint64_t)a.step, a.seed, 0);
                fire = u01(r.v[0]) < prob;
            }
        }
        const unsigned long long m = __ballot(fire);
        if (m) {
            const int leader = __ffsll((long long)m) - 1;
            int b = 0;
            if (lane == leader) b = atomicAdd(&s_add, __popcll(m));
            b = __shfl(b, leader, 64);
            if (fire) {
                const int k = b + __popcll(m & ((1ull << lane) - 1ull));
                if (k < room) {
                    const int64_t q = ebase64 + ebase + k;
                    const int znew = ion.zs[p] + 1;
                    el.x[q] = ion.x[p]; el.y[q] = ion.y[p]; el.z[q] = ion.z[p];
                    el.ux[q] = ion.ux[p]; el.uy[q] = ion.uy[p]; el.uz[q] = ion.uz[p];
                    el.w[q] = ion.w[p];
                    el.id[q] = (uint32_t)(a.id_base_new + (int64_t)(ion.id[p] - (uint32_t)a.ion_id_offset) * tab.z_max +
                                          (znew - 1));
                    ion.zs[p] = (uint8_t)znew;
                    atomicAdd(&s_fired, 1);
                } else {
                    full = true;
                }
            }
        }
    }
    if (full) g.flags[FLAG_CAPACITY] = 1;
    __syncthreads();
    if (tid == 0) {
        const int added = s_add < room ? s_add : room;
        el.count[sc] = ebase + added;
        if (s_fired) atomicAdd(&counters[1], (unsigned long long)s_fired);
    }
}

hipError_t launch_draw_append(const GridView& g, const SpeciesView& ion, const SpeciesView& el, const IonTables& tab,
                              const DrawArgs& a, const double* nu, unsigned long long* counters, hipStream_t st)
{
    hipLaunchKernelGGL(k_draw_append, dim3(g.nsc), dim3(BLOCK), 0, st, g, ion, el, tab, a, nu, counters);
    return hipGetLastError();
}

}  // namespace pic
