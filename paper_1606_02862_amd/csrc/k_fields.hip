// Yee FDTD updates on the periodic staggered grid (Yee 1966), four
// x-consecutive cells per lane (nx is a multiple of the supercell width, so a
// group never straddles a row), x fastest so every component row is read and
// written in coalesced 4-element vectors:
//   B -= coef * curl E   (forward differences of E, at the B locations)
//   E += coef * (curl B - J)   (backward differences of B, at the E locations;
//                               J converted from its fixed-point sums first when kept so)
// The x differences take one scalar from the neighbouring group (wrapped).
// The PIC cycle applies B(dt/2), E(dt), B(dt/2).
#include "pic_device.hpp"

namespace pic {

static_assert(SX % 4 == 0, "rows of whole 4-cell groups");

// Four consecutive values, loaded and stored as one 16-byte (FP32) or
// 32-byte (FP64) vector; the offsets used are multiples of 4 elements.
template <class R>
struct Quad {
    R v[4];
};
template <class R> struct VecOf;
template <> struct VecOf<float> { using T = float4; };
template <> struct VecOf<double> { using T = double4; };

template <class R>
__device__ inline Quad<R> ld4(const R* p)
{
    const typename VecOf<R>::T a = *reinterpret_cast<const typename VecOf<R>::T*>(p);
    return Quad<R>{{a.x, a.y, a.z, a.w}};
}
template <class R>
__device__ inline void st4(R* p, const Quad<R>& q)
{
    typename VecOf<R>::T a;
    a.x = q.v[0]; a.y = q.v[1]; a.z = q.v[2]; a.w = q.v[3];
    *reinterpret_cast<typename VecOf<R>::T*>(p) = a;
}

template <class R>
__global__ __launch_bounds__(BLOCK) void k_yee_b(GridViewT<R> g, R cx, R cy, R cz)
{
    const int N = g.nx * g.ny * g.nz;
    const int c = 4 * (blockIdx.x * BLOCK + threadIdx.x);  // first cell of the group
    if (c >= N) return;
    const int i = c % g.nx, j = (c / g.nx) % g.ny, k = c / (g.nx * g.ny);
    const int ip = (i + 4 == g.nx) ? c - i : c + 4;  // first cell of the next group along x
    const int jp = (j + 1 == g.ny) ? c - j * g.nx : c + g.nx;
    const int kp = (k + 1 == g.nz) ? c - k * g.nx * g.ny : c + g.nx * g.ny;
    const R* Ex = g.E;
    const R* Ey = g.E + N;
    const R* Ez = g.E + 2 * N;
    const Quad<R> ex = ld4(Ex + c), ey = ld4(Ey + c), ez = ld4(Ez + c);
    const Quad<R> ex_j = ld4(Ex + jp), ex_k = ld4(Ex + kp), ey_k = ld4(Ey + kp), ez_j = ld4(Ez + jp);
    const R ey_i[4] = {ey.v[1], ey.v[2], ey.v[3], Ey[ip]};  // E_y, E_z one cell up along x
    const R ez_i[4] = {ez.v[1], ez.v[2], ez.v[3], Ez[ip]};
    Quad<R> bx = ld4(g.B + c), by = ld4(g.B + N + c), bz = ld4(g.B + 2 * N + c);
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const R curl_x = cy * (ez_j.v[e] - ez.v[e]) - cz * (ey_k.v[e] - ey.v[e]);
        const R curl_y = cz * (ex_k.v[e] - ex.v[e]) - cx * (ez_i[e] - ez.v[e]);
        const R curl_z = cx * (ey_i[e] - ey.v[e]) - cy * (ex_j.v[e] - ex.v[e]);
        bx.v[e] -= curl_x;
        by.v[e] -= curl_y;
        bz.v[e] -= curl_z;
    }
    st4(g.B + c, bx);
    st4(g.B + N + c, by);
    st4(g.B + 2 * N + c, bz);
}

template <class R>
__global__ __launch_bounds__(BLOCK) void k_yee_e(GridViewT<R> g, R cx, R cy, R cz, R coef)
{
    const int N = g.nx * g.ny * g.nz;
    const int c = 4 * (blockIdx.x * BLOCK + threadIdx.x);
    if (c >= N) return;
    const int i = c % g.nx, j = (c / g.nx) % g.ny, k = c / (g.nx * g.ny);
    const int im = (i == 0) ? c + g.nx - 1 : c - 1;  // the cell before the group along x
    const int jm = (j == 0) ? c + (g.ny - 1) * g.nx : c - g.nx;
    const int km = (k == 0) ? c + (g.nz - 1) * g.nx * g.ny : c - g.nx * g.ny;
    const R* Bx = g.B;
    const R* By = g.B + N;
    const R* Bz = g.B + 2 * N;
    const Quad<R> bx = ld4(Bx + c), by = ld4(By + c), bz = ld4(Bz + c);
    const Quad<R> bx_j = ld4(Bx + jm), bx_k = ld4(Bx + km), by_k = ld4(By + km), bz_j = ld4(Bz + jm);
    const R by_i[4] = {By[im], by.v[0], by.v[1], by.v[2]};  // B_y, B_z one cell down along x
    const R bz_i[4] = {Bz[im], bz.v[0], bz.v[1], bz.v[2]};
    Quad<R> jx, jy, jz;
    if (g.J64) {  // PIC_OPT_DETERMINISTIC_J: J from its fixed-point sums (kept in g.J too)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            jx.v[e] = (R)((double)(long long)g.J64[c + e] * g.jinv64);
            jy.v[e] = (R)((double)(long long)g.J64[N + c + e] * g.jinv64);
            jz.v[e] = (R)((double)(long long)g.J64[2 * N + c + e] * g.jinv64);
        }
        st4(g.J + c, jx);
        st4(g.J + N + c, jy);
        st4(g.J + 2 * N + c, jz);
    } else {
        jx = ld4(g.J + c);
        jy = ld4(g.J + N + c);
        jz = ld4(g.J + 2 * N + c);
    }
    Quad<R> ex = ld4(g.E + c), ey = ld4(g.E + N + c), ez = ld4(g.E + 2 * N + c);
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const R curl_x = cy * (bz.v[e] - bz_j.v[e]) - cz * (by.v[e] - by_k.v[e]);
        const R curl_y = cz * (bx.v[e] - bx_k.v[e]) - cx * (bz.v[e] - bz_i[e]);
        const R curl_z = cx * (by.v[e] - by_i[e]) - cy * (bx.v[e] - bx_j.v[e]);
        ex.v[e] += curl_x - coef * jx.v[e];
        ey.v[e] += curl_y - coef * jy.v[e];
        ez.v[e] += curl_z - coef * jz.v[e];
    }
    st4(g.E + c, ex);
    st4(g.E + N + c, ey);
    st4(g.E + 2 * N + c, ez);
}

// coef / dx etc. are rounded to R once on the host side of the launch
template <class R>
hipError_t launch_yee_b(const GridViewT<R>& g, double coef, hipStream_t st)
{
    const int N = g.nx * g.ny * g.nz;
    if (g.nx % 4) return hipErrorInvalidValue;
    const R cf = (R)coef;
    hipLaunchKernelGGL(k_yee_b<R>, dim3((N / 4 + BLOCK - 1) / BLOCK), dim3(BLOCK), 0, st, g, cf / g.dx, cf / g.dy,
                       cf / g.dz);
    return hipGetLastError();
}

template <class R>
hipError_t launch_yee_e(const GridViewT<R>& g, double coef, hipStream_t st)
{
    const int N = g.nx * g.ny * g.nz;
    if (g.nx % 4) return hipErrorInvalidValue;
    const R cf = (R)coef;
    hipLaunchKernelGGL(k_yee_e<R>, dim3((N / 4 + BLOCK - 1) / BLOCK), dim3(BLOCK), 0, st, g, cf / g.dx, cf / g.dy,
                       cf / g.dz, cf);
    return hipGetLastError();
}

template hipError_t launch_yee_b<float>(const GridView&, double, hipStream_t);
template hipError_t launch_yee_b<double>(const GridView64&, double, hipStream_t);
template hipError_t launch_yee_e<float>(const GridView&, double, hipStream_t);
template hipError_t launch_yee_e<double>(const GridView64&, double, hipStream_t);

}  // namespace pic
