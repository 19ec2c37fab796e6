// Initial particle state, one workgroup per supercell and one lane per cell:
// ppc particles per cell written frame by frame (slot s of every cell lands in
// frame s), so each frame holds exactly one particle per cell.
#include "pic_device.hpp"

namespace pic {

struct InitArgs {
    uint64_t seed;
    int species_index, ppc, pos_index, pos_ppc;
    int64_t id_offset, pos_id_offset;
    double u_th, drift[3], weight;  // rounded to R before use
    int layout, z_init;
};

template <class R>
__global__ __launch_bounds__(BLOCK) void k_init_species(GridViewT<R> g, SpeciesViewT<R> s, InitArgs a)
{
    const int sc = blockIdx.x;
    const int c = threadIdx.x;
    const int lx = c & 7, ly = (c >> 3) & 7, lz = c >> 6;
    const int scx = sc % g.ncx, scy = (sc / g.ncx) % g.ncy, scz = sc / (g.ncx * g.ncy);
    const int i = scx * SX + lx, j = scy * SY + ly, k = scz * SZ + lz;
    const int64_t cell = (int64_t)i + (int64_t)g.nx * ((int64_t)j + (int64_t)g.ny * k);
    const double two_pi = 6.283185307179586476925286766559;
    const int64_t base = (int64_t)sc * s.cap;
    const double uth = (double)(R)a.u_th;
    const double drift[3] = {(double)(R)a.drift[0], (double)(R)a.drift[1], (double)(R)a.drift[2]};
    // rounding to R must not push a particle onto the supercell's far face
    const R xm = face_below<R>((R)SX), ym = face_below<R>((R)SY), zm = face_below<R>((R)SZ);
    for (int slot = 0; slot < a.ppc; ++slot) {
        const int64_t myid = cell * a.ppc + slot + a.id_offset;
        const int64_t pid = cell * a.pos_ppc + slot + a.pos_id_offset;
        const Philox4 pr = philox4x64_10((uint64_t)pid, (uint64_t)a.pos_index, PURPOSE_POSITION, 0, a.seed, 0);
        const Philox4 mr = philox4x64_10((uint64_t)myid, (uint64_t)a.species_index, PURPOSE_MOMENTUM, 0, a.seed, 0);
        R x = (R)((double)lx + u01(pr.v[0]));
        R y = (R)((double)ly + u01(pr.v[1]));
        R z = (R)((double)lz + u01(pr.v[2]));
        x = x < xm ? x : xm;
        y = y < ym ? y : ym;
        z = z < zm ? z : zm;
        const double b0 = u01(mr.v[0]), b1 = u01(mr.v[1]), b2 = u01(mr.v[2]), b3 = u01(mr.v[3]);
        const double r0 = sqrt(-2.0 * log(b0)), r1 = sqrt(-2.0 * log(b2));
        const double n0 = r0 * cos(two_pi * b1), n1 = r0 * sin(two_pi * b1), n2 = r1 * cos(two_pi * b3);
        double sign = 1.0;
        if (a.layout == PIC_LAYOUT_SHEAR) sign = (4 * j >= g.ny && 4 * j < 3 * g.ny) ? 1.0 : -1.0;
        if (a.layout == PIC_LAYOUT_BEAMS) sign = (slot % 2 == 0) ? 1.0 : -1.0;
        const int64_t p = base + (int64_t)slot * BLOCK + c;
        s.x[p] = x;
        s.y[p] = y;
        s.z[p] = z;
        s.ux[p] = (R)(sign * drift[0] + uth * n0);
        s.uy[p] = (R)(sign * drift[1] + uth * n1);
        s.uz[p] = (R)(sign * drift[2] + uth * n2);
        s.w[p] = (R)a.weight;
        s.id[p] = (uint32_t)myid;
        if (s.zs) s.zs[p] = (uint8_t)a.z_init;
    }
    if (c == 0) s.count[sc] = a.ppc * BLOCK;
}

template <class R>
hipError_t launch_init_species(const GridViewT<R>& g, const SpeciesViewT<R>& s, uint64_t seed, int species_index,
                               int ppc, int64_t id_offset, int pos_index, int pos_ppc, int64_t pos_id_offset,
                               double u_th, const double drift_u[3], int layout, double weight, int z_init,
                               hipStream_t st)
{
    InitArgs a;
    a.seed = seed;
    a.species_index = species_index;
    a.ppc = ppc;
    a.pos_index = pos_index;
    a.pos_ppc = pos_ppc;
    a.id_offset = id_offset;
    a.pos_id_offset = pos_id_offset;
    a.u_th = u_th;
    a.drift[0] = drift_u[0];
    a.drift[1] = drift_u[1];
    a.drift[2] = drift_u[2];
    a.weight = weight;
    a.layout = layout;
    a.z_init = z_init;
    hipLaunchKernelGGL(k_init_species<R>, dim3(g.nsc), dim3(BLOCK), 0, st, g, s, a);
    return hipGetLastError();
}

template hipError_t launch_init_species<float>(const GridView&, const SpeciesView&, uint64_t, int, int, int64_t, int,
                                               int, int64_t, double, const double*, int, double, int, hipStream_t);
template hipError_t launch_init_species<double>(const GridView64&, const SpeciesView64&, uint64_t, int, int, int64_t,
                                                int, int, int64_t, double, const double*, int, double, int,
                                                hipStream_t);

// ---------------------------------------------------------------- fills
// Plain fill kernels (used instead of hipMemsetAsync so that a captured
// graph replays them correctly).
template <typename T>
__global__ void k_zero(T* p, int64_t n)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = T(0);
}

template <typename T>
static hipError_t zero_n(T* p, int64_t n, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    int64_t blocks = (n + BLOCK - 1) / BLOCK;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(k_zero<T>, dim3((unsigned)blocks), dim3(BLOCK), 0, st, p, n);
    return hipGetLastError();
}

hipError_t launch_zero_f32(float* p, int64_t n, hipStream_t st) { return zero_n(p, n, st); }
hipError_t launch_zero_f64(double* p, int64_t n, hipStream_t st) { return zero_n(p, n, st); }
hipError_t launch_zero_i32(int32_t* p, int64_t n, hipStream_t st) { return zero_n(p, n, st); }

}  // namespace pic
