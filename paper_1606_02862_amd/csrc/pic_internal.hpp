// Internal structures of the gfx950 particle-in-cell library: device views
// passed to kernels by value, and the launchers each kernel file provides.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/pic.h"

namespace pic {

// Supercell: 8 x 8 x 4 = 256 cells, one 256-lane workgroup (4 wave64) each,
// as in the paper's block-per-supercell mapping.  A frame is 256 slots.
constexpr int SX = PIC_SUPERCELL_X, SY = PIC_SUPERCELL_Y, SZ = PIC_SUPERCELL_Z;
constexpr int SC_CELLS = SX * SY * SZ;
constexpr int BLOCK = 256;
constexpr int MAX_MIGRATE = 4096;  // per supercell, per species, per step

// Largest float below a power of two s (the far face of a supercell).
__host__ __device__ constexpr float below(float s) { return s - s * 0x1p-24f; }
constexpr float XMAX = below((float)SX), YMAX = below((float)SY), ZMAX = below((float)SZ);

// Device error flags (int32 each).
enum Flag { FLAG_CAPACITY = 0, FLAG_MIGRATE = 1, FLAG_CFL = 2, FLAG_NONFINITE = 3, NFLAGS = 4 };

// Views are templated on the real type R of particles, fields and currents:
// float (the default path) or double (the FP64 variant of the PIC cycle).
template <class R> struct Vec4;
template <> struct Vec4<float> { using type = float4; };
template <> struct Vec4<double> { using type = double4; };

template <class R>
struct GridViewT {
    int nx, ny, nz;        // cells
    int ncx, ncy, ncz;     // supercells per axis
    int nsc;               // number of supercells
    int xcd_remap;         // block -> supercell order (sc_of_block): 0 identity, L >= 1 XCD slabs of L z-layers
    R dx, dy, dz, dt;
    R b0x, b0y, b0z;
    R* E;                  // 3 * N, component-major, x fastest
    R* B;
    R* J;
    int32_t* flags;
    typename Vec4<R>::type* qbuf;  // deposit queue: nsc * qcap records of 2 (x0,y0,z0,qw | x1,y1,z1,-)
    int qcap;              // queue slots per supercell (>= every species' frame capacity; a multiple of 512)
    // PIC_OPT_DETERMINISTIC_J (FP32): 3 * N int64 fixed-point current at the
    // cycle's common scale, which the E update converts (times jinv64) into J;
    // nullptr otherwise
    unsigned long long* J64;
    double jinv64;
};

template <class R>
struct SpeciesViewT {
    R *x, *y, *z;           // supercell-relative positions in cells: [0,8)x[0,8)x[0,4)
    R *ux, *uy, *uz;        // u = gamma v
    R* w;                   // macro weight
    uint32_t* id;
    uint8_t* zs;            // charge state, or nullptr
    int32_t* count;         // particles per supercell
    int cap;                // slots per supercell (multiple of 256)
    // arrival lists: per step parity and destination supercell, cap_in slots
    R *ix, *iy, *iz, *iux, *iuy, *iuz, *iw;
    uint32_t* iid;
    uint8_t* izs;
    int32_t* in_count;      // arrivals per parity and supercell (2 * nsc)
    int32_t* holes;         // per source supercell: vacated slots
    int32_t* hole_count;
    int cap_in;
    R charge;               // in e (per unit Z when zs != nullptr)
    R mass;
};

using GridView = GridViewT<float>;
using SpeciesView = SpeciesViewT<float>;
using GridView64 = GridViewT<double>;
using SpeciesView64 = SpeciesViewT<double>;

// Largest value below the far face of a supercell of extent s in type R.
template <class R> __host__ __device__ constexpr R face_below(R s);
template <> __host__ __device__ constexpr float face_below<float>(float s) { return s - s * 0x1p-24f; }
template <> __host__ __device__ constexpr double face_below<double>(double s) { return s - s * 0x1p-53; }

struct Species {
    SpeciesView v;         // FP32 frames (the default path)
    SpeciesView64 v64;     // FP64 frames (the FP64 variant)
    pic_species_t desc;
    int64_t n_init;        // particles at t = 0
    int64_t id_offset;     // first id at t = 0
    double weight;
    double wmax;           // bound of |w| that sets the fixed-point current scale (>= wheld)
    double wheld;          // largest |w| known to be held (init, set, ionisation electrons)
};

// Map a workgroup index to a supercell so that the 8 XCDs (which receive
// workgroups round-robin) each work on one contiguous slab of nsc/8
// supercells and share its guard cells in their own L2.  remap = 0: the
// identity; remap = L >= 1: the slab is L whole z-layers of nxy = ncx*ncy
// supercells (L = 1 also stands for a slab that is not), and within it the
// blocks walk z fastest, so that the neighbours of a supercell along every
// axis, not only x and y, run at about the same time.
__host__ __device__ inline int sc_of_block(int b, int nsc, int nxy, int remap)
{
    if (!remap) return b;
    const int per = nsc >> 3, i = b >> 3;
    return (b & 7) * per + (i % remap) * nxy + i / remap;
}

// ---------------------------------------------------------------- launchers
// The PIC-cycle launchers exist for R = float and R = double.
template <class R>
hipError_t launch_init_species(const GridViewT<R>& g, const SpeciesViewT<R>& s, uint64_t seed, int species_index,
                               int ppc, int64_t id_offset, int pos_index, int pos_ppc, int64_t pos_id_offset,
                               double u_th, const double drift_u[3], int layout, double weight, int z_init,
                               hipStream_t st);
hipError_t launch_zero_f32(float* p, int64_t n, hipStream_t st);
hipError_t launch_zero_f64(double* p, int64_t n, hipStream_t st);
hipError_t launch_zero_i32(int32_t* p, int64_t n, hipStream_t st);
inline hipError_t launch_zero_r(float* p, int64_t n, hipStream_t st) { return launch_zero_f32(p, n, st); }
inline hipError_t launch_zero_r(double* p, int64_t n, hipStream_t st) { return launch_zero_f64(p, n, st); }
// vmax: upper bound of |q w| max(dx,dy,dz) / (dV dt) over the species' particles
// apar: parity of the arrivals to absorb first (-1: none); wpar: parity the
// leavers of this step are written to
// galerkin: the reduced-order gather along staggered axes (PIC_GATHER_GALERKIN)
// jscale_g: with g.J64, the cycle's common fixed-point scale (2^30 over the
// largest vmax of the cycle's species); each tile is rescaled to it at the flush
template <class R>
hipError_t launch_push(const GridViewT<R>& g, const SpeciesViewT<R>& s, int order, bool galerkin, double vmax,
                       float jscale_g, int apar, int wpar, hipStream_t st);
// Fixed-point scale of a current tile: 2^30 over the bound vmax of one contribution.
inline float fixed_scale(double vmax)
{
    const float vf = (float)vmax;
    return vf > 0.0f ? 1073741824.0f / vf : 1.0f;
}
template <class R>
hipError_t launch_migrate(const GridViewT<R>& g, const SpeciesViewT<R>& s, int par, hipStream_t st);
template <class R>
hipError_t launch_yee_b(const GridViewT<R>& g, double coef, hipStream_t st);
template <class R>
hipError_t launch_yee_e(const GridViewT<R>& g, double coef, hipStream_t st);

// FP64 diagnostics.  partial buffers hold one entry per workgroup.
struct DiagBuffers {
    double* rho;       // N
    double* g0;        // N, Gauss reference
    double* partial;   // scratch for block partial sums / maxima
    int npartial;
    double* rho_prev;  // N, rho before the last cycle (PIC_OPT_CONTINUITY), or nullptr
    double* result;    // small device result vector
};
template <class R>
hipError_t launch_field_energy(const GridViewT<R>& g, const DiagBuffers& d, hipStream_t st);
template <class R>
hipError_t launch_kinetic(const GridViewT<R>& g, const SpeciesViewT<R>& s, const DiagBuffers& d, int slot,
                          hipStream_t st);
template <class R>
hipError_t launch_rho_deposit(const GridViewT<R>& g, const SpeciesViewT<R>& s, int order, double* rho,
                              hipStream_t st);
// mode 0: record G0; mode 1: the reductions, plus the continuity residual
// against d.rho_prev when cont is set
template <class R>
hipError_t launch_gauss(const GridViewT<R>& g, const DiagBuffers& d, double rho_bg, int mode, bool cont, hipStream_t st);

// Result vector layout of the diagnostics.
enum DiagSlot {
    D_WE = 0, D_WB = 1, D_NONFINITE = 2, D_CHARGE = 3, D_RHOMAX = 4, D_GAUSS = 5, D_DIVB = 6,
    D_KIN0 = 8,  // + species index
    D_CONT = 12, D_JMAX = 13,
    D_NSLOTS = 16
};

}  // namespace pic
