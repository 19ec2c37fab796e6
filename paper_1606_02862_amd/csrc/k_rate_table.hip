// Tabulated ionisation rate: per charge state Z, the subshell sum
//   h_Z(s) = ln sum_j (a_j q_j / p_j) e^{-(p_j - P_Z)/kT} S_j(kT / p_j),  s = ln kT,
// built once on the GPU by the exact 64-point Gauss-Laguerre quadrature at
// RATE_TABLE_N points uniform in s, then read by Catmull-Rom cubic
// interpolation:  nu = n_e vbar(kT) / kT e^{h_Z(ln kT) - P_Z/kT}.  The steep
// factor e^{-P_Z/kT} and the vbar / kT prefactor stay analytic, so the table
// holds a slowly varying function; outside [RATE_TABLE_TMIN, RATE_TABLE_TMAX]
// the exact quadrature is used.
#include "ionize_internal.hpp"

namespace pic {

// Node i at s = s0 + i ds, s0 one spacing below ln TMIN and ln TMAX at node
// N - 2, so that every kT in range has the four nodes i-1 .. i+2 of its
// interval.
__host__ __device__ inline double rate_table_ds()
{
    return (log(RATE_TABLE_TMAX) - log(RATE_TABLE_TMIN)) / (RATE_TABLE_N - 3);
}
__host__ __device__ inline double rate_table_s0() { return log(RATE_TABLE_TMIN) - rate_table_ds(); }

__global__ __launch_bounds__(BLOCK) void k_rate_table_build(IonTables tab, const double* gl, double* out)
{
    __shared__ double glx[GL_NODES], glw[GL_NODES];
    if (threadIdx.x < GL_NODES) { glx[threadIdx.x] = gl[threadIdx.x]; glw[threadIdx.x] = gl[GL_NODES + threadIdx.x]; }
    __syncthreads();
    const int i = blockIdx.x * BLOCK + threadIdx.x;
    if (i >= tab.z_max * RATE_TABLE_N) return;
    const int z = i / RATE_TABLE_N, k = i % RATE_TABLE_N;
    const double kT = exp(rate_table_s0() + k * rate_table_ds());
    out[i] = log(lotz_shells(kT, tab, z, glx, glw));
}

hipError_t launch_rate_table_build(const IonTables& tab, const double* gl, double* table, hipStream_t st)
{
    const int n = tab.z_max * RATE_TABLE_N;
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_rate_table_build, dim3((n + BLOCK - 1) / BLOCK), dim3(BLOCK), 0, st, tab, gl, table);
    return hipGetLastError();
}

// h_Z(ln kT) for kT in [TMIN, TMAX]: Catmull-Rom, the cubic through the
// interval's end nodes p1, p2 with end slopes (p2 - p0)/2 and (p3 - p1)/2.
__device__ inline double table_h(double kT, int Z, const double* table)
{
    const double t = (log(kT) - rate_table_s0()) * (1.0 / rate_table_ds());
    int i = (int)t;
    i = i < 1 ? 1 : (i > RATE_TABLE_N - 3 ? RATE_TABLE_N - 3 : i);
    const double f = t - i;
    const double* h = table + Z * RATE_TABLE_N + i;
    const double p0 = h[-1], p1 = h[0], p2 = h[1], p3 = h[2];
    return p1 + 0.5 * f * ((p2 - p0) + f * ((2.0 * p0 - 5.0 * p1 + 4.0 * p2 - p3) + f * (3.0 * (p1 - p2) + p3 - p0)));
}

__device__ inline bool in_table(double kT, double ne)
{
    return kT >= RATE_TABLE_TMIN && kT <= RATE_TABLE_TMAX && ne > 0.0;
}

// nu from the table for kT in range (returns false outside, or where n_e is
// not positive: then the caller takes the exact path).
__device__ inline bool rate_from_table(double kT, double ne, const IonTables& tab, int Z, const double* table,
                                       double& nu)
{
    if (!in_table(kT, ne)) return false;
    nu = ne * vbar_cm_s(kT) / kT * exp(table_h(kT, Z, table) - tab.P[Z] / kT);
    return true;
}

// One thread per ion slot: blockIdx.x the supercell, blockIdx.y the chunk of
// BLOCK slots (many short blocks keep enough loads in flight).  Ions whose
// cell lies outside the table's kT range are appended to fb_list (their
// count in counters[CNT_FALLBACK]) and take the exact quadrature in the fallback kernel.
__global__ __launch_bounds__(BLOCK) void k_rate_table(GridView g, SpeciesView ion, IonTables tab, const double* ne,
                                                      const double* kT, double* nu, const double* table,
                                                      unsigned long long* counters, unsigned long long* fb_list)
{
    const int sc = blockIdx.x;
    const int tid = threadIdx.x, lane = tid & 63;
    const int n = ion.count[sc];
    const int t0 = blockIdx.y * BLOCK;
    if (t0 >= n) return;  // block-uniform
    const int64_t base = (int64_t)sc * ion.cap;
    const int scx = sc % g.ncx, scy = (sc / g.ncx) % g.ncy, scz = sc / (g.ncx * g.ncy);
    {
        const int t = t0 + tid;
        const int64_t p = base + t;
        bool fb = false;
        if (t < n) {
            const int Z = ion.zs[p];
            double v = 0.0;
            if (Z < tab.z_max) {
                const int64_t gi = (int64_t)(scx * SX + (int)ion.x[p]) +
                                   (int64_t)g.nx * ((scy * SY + (int)ion.y[p]) + (int64_t)g.ny * (scz * SZ + (int)ion.z[p]));
                const double t_ev = kT[gi], n_cm3 = ne[gi];
                fb = !rate_from_table(t_ev, n_cm3, tab, Z, table, v) && t_ev > 0.0 && n_cm3 > 0.0;
            }
            nu[p] = v;
        }
        const unsigned long long fmask = __ballot(fb);
        if (fmask) {  // rare
            const int leader = __ffsll((long long)fmask) - 1;
            unsigned long long fbase = 0;
            if (lane == leader) fbase = atomicAdd(&counters[CNT_FALLBACK], (unsigned long long)__popcll(fmask));
            fbase = __shfl(fbase, leader, 64);
            if (fb)
                fb_list[fbase + (unsigned)__builtin_amdgcn_mbcnt_hi((unsigned)(fmask >> 32),
                                                                   __builtin_amdgcn_mbcnt_lo((unsigned)fmask, 0u))] =
                    (unsigned long long)p;
        }
    }
}

hipError_t launch_rate_table(const GridView& g, const SpeciesView& ion, const IonTables& tab, const double* ne,
                             const double* kT, double* nu, const double* table, const double* gl,
                             unsigned long long* counters, unsigned long long* fb_list, hipStream_t st)
{
    const dim3 grid(g.nsc, (ion.cap + BLOCK - 1) / BLOCK);
    hipLaunchKernelGGL(k_rate_table, grid, dim3(BLOCK), 0, st, g, ion, tab, ne, kT, nu, table, counters, fb_list);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_rate_fallback(g, ion, tab, ne, kT, nu, gl, fb_list, counters, st);
}

// ln nu of independent samples from the table (exact outside its range).
__global__ __launch_bounds__(BLOCK) void k_ln_rate_table(int64_t n, const double* kT, const double* ne,
                                                         const int32_t* Z, IonTables tab, const double* table,
                                                         const double* gl, double* out)
{
    __shared__ double glx[GL_NODES], glw[GL_NODES];
    if (threadIdx.x < GL_NODES) { glx[threadIdx.x] = gl[threadIdx.x]; glw[threadIdx.x] = gl[GL_NODES + threadIdx.x]; }
    __syncthreads();
    const int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (i >= n) return;
    const int z = Z[i];
    if (!(z >= 0 && z < tab.z_max)) {
        out[i] = -INFINITY;
        return;
    }
    const double t_ev = kT[i], n_cm3 = ne[i];
    if (in_table(t_ev, n_cm3)) {
        out[i] = log(n_cm3 * vbar_cm_s(t_ev) / t_ev) + table_h(t_ev, z, table) - tab.P[z] / t_ev;
    } else {
        out[i] = ln_rate_exact(t_ev, n_cm3, tab, z, glx, glw);
    }
}

hipError_t launch_ln_rate_table(int64_t n, const double* kT, const double* ne, const int32_t* Z, const IonTables& tab,
                                const double* table, const double* gl, double* out, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_ln_rate_table, dim3((unsigned)((n + BLOCK - 1) / BLOCK)), dim3(BLOCK), 0, st, n, kT, ne, Z,
                       tab, table, gl, out);
    return hipGetLastError();
}

}  // namespace pic
