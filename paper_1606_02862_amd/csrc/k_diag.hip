// FP64 diagnostics: field and kinetic energies, node charge density, the
// Gauss residual G = div E - rho against its reference, div B, and a count of
// non-finite field entries.  Two-pass reductions: each workgroup writes its
// partial sum / maximum, then one workgroup combines the partials in a fixed
// order, so the results do not depend on scheduling.
#include "pic_device.hpp"

namespace pic {

constexpr int RED_BLOCKS = 1024;

__device__ inline double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ inline double wave_max(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}

// Sum (is_max = false) or maximum over the 256 lanes; result valid in lane 0.
__device__ inline double block_reduce(double v, bool is_max, double* scratch)
{
    v = is_max ? wave_max(v) : wave_sum(v);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) scratch[wave] = v;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == 0) {
        r = scratch[0];
        for (int w = 1; w < BLOCK / 64; ++w) r = is_max ? fmax(r, scratch[w]) : r + scratch[w];
    }
    return r;
}

template <class R>
__global__ __launch_bounds__(BLOCK) void k_field_energy(GridViewT<R> g, double* partial)
{
    __shared__ double scratch[BLOCK / 64];
    const int64_t N3 = 3LL * g.nx * g.ny * g.nz;
    double se = 0.0, sb = 0.0, bad = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x; i < N3; i += (int64_t)gridDim.x * BLOCK) {
        const double e = g.E[i], b = g.B[i];
        if (!isfinite(e) || !isfinite(b)) bad += 1.0;
        else { se += e * e; sb += b * b; }
    }
    se = block_reduce(se, false, scratch);
    sb = block_reduce(sb, false, scratch);
    bad = block_reduce(bad, false, scratch);
    if (threadIdx.x == 0) {
        partial[3 * blockIdx.x + 0] = se;
        partial[3 * blockIdx.x + 1] = sb;
        partial[3 * blockIdx.x + 2] = bad;
    }
}

// Combine nb partials of `stride` values each; value v goes to result[dst[v]]
// scaled by scale[v], as a sum or (op bit v set) a maximum.
struct Finalize {
    int nb, stride, nvals;
    int dst[8];
    double scale[8];
    unsigned max_mask;
};

__global__ __launch_bounds__(BLOCK) void k_finalize(const double* partial, Finalize f, double* result)
{
    __shared__ double scratch[BLOCK / 64];
    for (int v = 0; v < f.nvals; ++v) {
        const bool mx = (f.max_mask >> v) & 1u;
        double a = 0.0;
        for (int b = threadIdx.x; b < f.nb; b += BLOCK) {
            const double x = partial[(int64_t)b * f.stride + v];
            a = mx ? fmax(a, x) : a + x;
        }
        a = block_reduce(a, mx, scratch);
        if (threadIdx.x == 0) result[f.dst[v]] = a * f.scale[v];
    }
}

template <class R>
hipError_t launch_field_energy(const GridViewT<R>& g, const DiagBuffers& d, hipStream_t st)
{
    hipLaunchKernelGGL(k_field_energy<R>, dim3(RED_BLOCKS), dim3(BLOCK), 0, st, g, d.partial);
    Finalize f{};
    f.nb = RED_BLOCKS;
    f.stride = 3;
    f.nvals = 3;
    const double dV = (double)g.dx * g.dy * g.dz;
    f.dst[0] = D_WE; f.scale[0] = 0.5 * dV;
    f.dst[1] = D_WB; f.scale[1] = 0.5 * dV;
    f.dst[2] = D_NONFINITE; f.scale[2] = 1.0;
    f.max_mask = 0;
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(BLOCK), 0, st, d.partial, f, d.result);
    return hipGetLastError();
}

// ---------------------------------------------------------------- kinetic
template <class R>
__global__ __launch_bounds__(BLOCK) void k_kinetic(GridViewT<R> g, SpeciesViewT<R> s, double* partial)
{
    __shared__ double scratch[BLOCK / 64];
    const int sc = blockIdx.x;
    const int n = s.count[sc];
    const int64_t base = (int64_t)sc * s.cap;
    double acc = 0.0;
    for (int t = threadIdx.x; t < n; t += BLOCK) {
        const double ux = s.ux[base + t], uy = s.uy[base + t], uz = s.uz[base + t];
        const double u2 = ux * ux + uy * uy + uz * uz;
        acc += (double)s.w[base + t] * (u2 / (1.0 + sqrt(1.0 + u2)));  // gamma - 1
    }
    acc = block_reduce(acc, false, scratch);
    if (threadIdx.x == 0) partial[sc] = acc * (double)s.mass;
}

template <class R>
hipError_t launch_kinetic(const GridViewT<R>& g, const SpeciesViewT<R>& s, const DiagBuffers& d, int slot,
                          hipStream_t st)
{
    hipLaunchKernelGGL(k_kinetic<R>, dim3(g.nsc), dim3(BLOCK), 0, st, g, s, d.partial);
    Finalize f{};
    f.nb = g.nsc;
    f.stride = 1;
    f.nvals = 1;
    f.dst[0] = D_KIN0 + slot;
    f.scale[0] = 1.0;
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(BLOCK), 0, st, d.partial, f, d.result);
    return hipGetLastError();
}

// ---------------------------------------------------------------- rho
template <int ORDER>
__device__ inline void rho_weights(double x, int* first, double* w)
{
    if constexpr (ORDER == 1) {
        const double f = floor(x), d = x - f;
        *first = (int)f;
        w[0] = 1.0 - d;
        w[1] = d;
    } else if constexpr (ORDER == 2) {
        const double r = floor(x + 0.5), d = x - r;
        *first = (int)r - 1;
        w[0] = 0.5 * (0.5 - d) * (0.5 - d);
        w[1] = 0.75 - d * d;
        w[2] = 0.5 * (0.5 + d) * (0.5 + d);
    } else {
        const double f = floor(x), d = x - f, e = 1.0 - d;
        *first = (int)f - 1;
        w[0] = e * e * e / 6.0;
        w[1] = 2.0 / 3.0 - d * d * (1.0 - 0.5 * d);
        w[2] = 2.0 / 3.0 - e * e * (1.0 - 0.5 * e);
        w[3] = d * d * d / 6.0;
    }
}

// Charge density in FP64: each workgroup deposits its supercell's particles
// into an LDS tile of nodes [-1, S+1] per axis (every shape's support from a
// particle inside the supercell lies there) with native FP64 LDS atomics,
// then adds the tile to rho with one global FP64 atomic per node.
constexpr int RHO_TX = SX + 3, RHO_TY = SY + 3, RHO_TZ = SZ + 3, RHO_TN = RHO_TX * RHO_TY * RHO_TZ;

template <int ORDER, class R>
__global__ __launch_bounds__(BLOCK) void k_rho(GridViewT<R> g, SpeciesViewT<R> s, double* rho)
{
    __shared__ double tile[RHO_TN];
    const int sc = blockIdx.x;
    const int tid = threadIdx.x;
    for (int t = tid; t < RHO_TN; t += BLOCK) tile[t] = 0.0;
    __syncthreads();
    const int n = s.count[sc];
    const int scx = sc % g.ncx, scy = (sc / g.ncx) % g.ncy, scz = sc / (g.ncx * g.ncy);
    const int64_t base = (int64_t)sc * s.cap;
    const double inv_dv = 1.0 / ((double)g.dx * g.dy * g.dz);
    for (int t = tid; t < n; t += BLOCK) {
        const int64_t p = base + t;
        double q = s.charge;
        if (s.zs) q *= (double)s.zs[p];
        const double qw = q * (double)s.w[p] * inv_dv;
        int fx, fy, fz;
        double wx[4], wy[4], wz[4];
        rho_weights<ORDER>((double)s.x[p], &fx, wx);
        rho_weights<ORDER>((double)s.y[p], &fy, wy);
        rho_weights<ORDER>((double)s.z[p], &fz, wz);
        // a particle inside its supercell always passes; anything else is skipped
        if (fx < -1 || fx > SX + 1 - ORDER || fy < -1 || fy > SY + 1 - ORDER || fz < -1 || fz > SZ + 1 - ORDER) continue;
#pragma unroll
        for (int c = 0; c <= ORDER; ++c)
#pragma unroll
            for (int b = 0; b <= ORDER; ++b) {
                const int row = ((fz + c + 1) * RHO_TY + (fy + b + 1)) * RHO_TX + (fx + 1);
                const double wyz = qw * wy[b] * wz[c];
#pragma unroll
                for (int a = 0; a <= ORDER; ++a) atomicAdd(&tile[row + a], wyz * wx[a]);
            }
    }
    __syncthreads();
    for (int t = tid; t < RHO_TN; t += BLOCK) {
        const double v = tile[t];
        if (v == 0.0) continue;
        const int tx = t % RHO_TX, ty = (t / RHO_TX) % RHO_TY, tz = t / (RHO_TX * RHO_TY);
        int gx = scx * SX + tx - 1, gy = scy * SY + ty - 1, gz = scz * SZ + tz - 1;
        gx += (gx < 0) ? g.nx : 0; gx -= (gx >= g.nx) ? g.nx : 0;
        gy += (gy < 0) ? g.ny : 0; gy -= (gy >= g.ny) ? g.ny : 0;
        gz += (gz < 0) ? g.nz : 0; gz -= (gz >= g.nz) ? g.nz : 0;
        unsafeAtomicAdd(&rho[gx + (int64_t)g.nx * (gy + (int64_t)g.ny * gz)], v);
    }
}

template <class R>
hipError_t launch_rho_deposit(const GridViewT<R>& g, const SpeciesViewT<R>& s, int order, double* rho,
                              hipStream_t st)
{
    if (order == 1) hipLaunchKernelGGL((k_rho<1, R>), dim3(g.nsc), dim3(BLOCK), 0, st, g, s, rho);
    else if (order == 2) hipLaunchKernelGGL((k_rho<2, R>), dim3(g.nsc), dim3(BLOCK), 0, st, g, s, rho);
    else hipLaunchKernelGGL((k_rho<3, R>), dim3(g.nsc), dim3(BLOCK), 0, st, g, s, rho);
    return hipGetLastError();
}

// ---------------------------------------------------------------- Gauss
// mode 0: store G = div E - rho as the reference; mode 1: reduce
// max |G - G0|, max |rho|, sum rho dV, max |div B| (at cell centres), max |J|
// and, with rho_prev, the continuity residual max |div J + (rho - rho_prev)/dt|
// (div J with the backward differences of div E, at the nodes).
constexpr int GAUSS_VALS = 6;

template <class R>
__global__ __launch_bounds__(BLOCK) void k_gauss(GridViewT<R> g, const double* rho, double* g0, double rho_bg, int mode,
                                                 const double* rho_prev, double* partial)
{
    __shared__ double scratch[BLOCK / 64];
    const int N = g.nx * g.ny * g.nz;
    const double idx = 1.0 / (double)g.dx, idy = 1.0 / (double)g.dy, idz = 1.0 / (double)g.dz;
    const double idt = 1.0 / (double)g.dt;
    double gmax = 0.0, rmax = 0.0, rsum = 0.0, bmax = 0.0, cmax = 0.0, jmax = 0.0;
    for (int c = blockIdx.x * BLOCK + threadIdx.x; c < N; c += gridDim.x * BLOCK) {
        const int i = c % g.nx, j = (c / g.nx) % g.ny, k = c / (g.nx * g.ny);
        const int im = (i == 0) ? c + g.nx - 1 : c - 1;
        const int jm = (j == 0) ? c + (g.ny - 1) * g.nx : c - g.nx;
        const int km = (k == 0) ? c + (g.nz - 1) * g.nx * g.ny : c - g.nx * g.ny;
        const int ip = (i + 1 == g.nx) ? c - i : c + 1;
        const int jp = (j + 1 == g.ny) ? c - j * g.nx : c + g.nx;
        const int kp = (k + 1 == g.nz) ? c - k * g.nx * g.ny : c + g.nx * g.ny;
        const double divE = ((double)g.E[c] - (double)g.E[im]) * idx +
                            ((double)g.E[N + c] - (double)g.E[N + jm]) * idy +
                            ((double)g.E[2 * N + c] - (double)g.E[2 * N + km]) * idz;
        const double r = rho[c] + rho_bg;
        const double G = divE - r;
        if (mode == 0) {
            g0[c] = G;
        } else {
            const double divB = ((double)g.B[ip] - (double)g.B[c]) * idx +
                                ((double)g.B[N + jp] - (double)g.B[N + c]) * idy +
                                ((double)g.B[2 * N + kp] - (double)g.B[2 * N + c]) * idz;
            gmax = fmax(gmax, fabs(G - g0[c]));
            rmax = fmax(rmax, fabs(r));
            rsum += r;
            bmax = fmax(bmax, fabs(divB));
            jmax = fmax(jmax, fmax(fabs((double)g.J[c]), fmax(fabs((double)g.J[N + c]), fabs((double)g.J[2 * N + c]))));
            if (rho_prev) {
                const double divJ = ((double)g.J[c] - (double)g.J[im]) * idx +
                                    ((double)g.J[N + c] - (double)g.J[N + jm]) * idy +
                                    ((double)g.J[2 * N + c] - (double)g.J[2 * N + km]) * idz;
                cmax = fmax(cmax, fabs(divJ + (rho[c] - rho_prev[c]) * idt));
            }
        }
    }
    if (mode == 0) return;
    gmax = block_reduce(gmax, true, scratch);
    rmax = block_reduce(rmax, true, scratch);
    rsum = block_reduce(rsum, false, scratch);
    bmax = block_reduce(bmax, true, scratch);
    cmax = block_reduce(cmax, true, scratch);
    jmax = block_reduce(jmax, true, scratch);
    if (threadIdx.x == 0) {
        double* p = partial + GAUSS_VALS * blockIdx.x;
        p[0] = gmax;
        p[1] = rmax;
        p[2] = rsum;
        p[3] = bmax;
        p[4] = cmax;  // 0 without rho_prev
        p[5] = jmax;
    }
}

template <class R>
hipError_t launch_gauss(const GridViewT<R>& g, const DiagBuffers& d, double rho_bg, int mode, bool cont, hipStream_t st)
{
    if (mode != 0 && d.npartial < GAUSS_VALS * RED_BLOCKS) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_gauss<R>, dim3(RED_BLOCKS), dim3(BLOCK), 0, st, g, d.rho, d.g0, rho_bg, mode,
                       cont ? (const double*)d.rho_prev : nullptr, d.partial);
    if (mode == 0) return hipGetLastError();
    Finalize f{};
    f.nb = RED_BLOCKS;
    f.stride = GAUSS_VALS;
    f.nvals = GAUSS_VALS;
    f.dst[0] = D_GAUSS; f.scale[0] = 1.0;
    f.dst[1] = D_RHOMAX; f.scale[1] = 1.0;
    f.dst[2] = D_CHARGE; f.scale[2] = (double)g.dx * g.dy * g.dz;
    f.dst[3] = D_DIVB; f.scale[3] = 1.0;
    f.dst[4] = D_CONT; f.scale[4] = 1.0;
    f.dst[5] = D_JMAX; f.scale[5] = 1.0;
    f.max_mask = 0b111011;
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(BLOCK), 0, st, d.partial, f, d.result);
    return hipGetLastError();
}

#define PIC_DIAG_INSTANCES(R)                                                                                   \
    template hipError_t launch_field_energy<R>(const GridViewT<R>&, const DiagBuffers&, hipStream_t);         \
    template hipError_t launch_kinetic<R>(const GridViewT<R>&, const SpeciesViewT<R>&, const DiagBuffers&, int, \
                                          hipStream_t);                                                       \
    template hipError_t launch_rho_deposit<R>(const GridViewT<R>&, const SpeciesViewT<R>&, int, double*,       \
                                              hipStream_t);                                                   \
    template hipError_t launch_gauss<R>(const GridViewT<R>&, const DiagBuffers&, double, int, bool, hipStream_t);
PIC_DIAG_INSTANCES(float)
PIC_DIAG_INSTANCES(double)
#undef PIC_DIAG_INSTANCES

}  // namespace pic
