// Yee FDTD updates on the periodic staggered grid (Yee 1966), one lane per
// cell, x fastest so every component row is read and written coalesced:
//   B -= coef * curl E   (forward differences of E, at the B locations)
//   E += coef * (curl B - J)   (backward differences of B, at the E locations;
//                               J converted from its fixed-point sums first when kept so)
// The PIC cycle applies B(dt/2), E(dt), B(dt/2).
#include "pic_device.hpp"

namespace pic {

template <class R>
__global__ __launch_bounds__(BLOCK) void k_yee_b(GridViewT<R> g, R cx, R cy, R cz)
{
    const int N = g.nx * g.ny * g.nz;
    const int c = blockIdx.x * BLOCK + threadIdx.x;
    if (c >= N) return;
    const int i = c % g.nx, j = (c / g.nx) % g.ny, k = c / (g.nx * g.ny);
    const int ip = (i + 1 == g.nx) ? c - i : c + 1;
    const int jp = (j + 1 == g.ny) ? c - j * g.nx : c + g.nx;
    const int kp = (k + 1 == g.nz) ? c - k * g.nx * g.ny : c + g.nx * g.ny;
    const R* Ex = g.E;
    const R* Ey = g.E + N;
    const R* Ez = g.E + 2 * N;
    const R ex = Ex[c], ey = Ey[c], ez = Ez[c];
    const R curl_x = cy * (Ez[jp] - ez) - cz * (Ey[kp] - ey);
    const R curl_y = cz * (Ex[kp] - ex) - cx * (Ez[ip] - ez);
    const R curl_z = cx * (Ey[ip] - ey) - cy * (Ex[jp] - ex);
    g.B[c] -= curl_x;
    g.B[N + c] -= curl_y;
    g.B[2 * N + c] -= curl_z;
}

template <class R>
__global__ __launch_bounds__(BLOCK) void k_yee_e(GridViewT<R> g, R cx, R cy, R cz, R coef)
{
    const int N = g.nx * g.ny * g.nz;
    const int c = blockIdx.x * BLOCK + threadIdx.x;
    if (c >= N) return;
    const int i = c % g.nx, j = (c / g.nx) % g.ny, k = c / (g.nx * g.ny);
    const int im = (i == 0) ? c + g.nx - 1 : c - 1;
    const int jm = (j == 0) ? c + (g.ny - 1) * g.nx : c - g.nx;
    const int km = (k == 0) ? c + (g.nz - 1) * g.nx * g.ny : c - g.nx * g.ny;
    const R* Bx = g.B;
    const R* By = g.B + N;
    const R* Bz = g.B + 2 * N;
    const R bx = Bx[c], by = By[c], bz = Bz[c];
    const R curl_x = cy * (bz - Bz[jm]) - cz * (by - By[km]);
    const R curl_y = cz * (bx - Bx[km]) - cx * (bz - Bz[im]);
    const R curl_z = cx * (by - By[im]) - cy * (bx - Bx[jm]);
    R jx, jy, jz;
    if (g.J64) {  // PIC_OPT_DETERMINISTIC_J: J from its fixed-point sums (kept in g.J too)
        jx = (R)((double)(long long)g.J64[c] * g.jinv64);
        jy = (R)((double)(long long)g.J64[N + c] * g.jinv64);
        jz = (R)((double)(long long)g.J64[2 * N + c] * g.jinv64);
        g.J[c] = jx;
        g.J[N + c] = jy;
        g.J[2 * N + c] = jz;
    } else {
        jx = g.J[c];
        jy = g.J[N + c];
        jz = g.J[2 * N + c];
    }
    g.E[c] += curl_x - coef * jx;
    g.E[N + c] += curl_y - coef * jy;
    g.E[2 * N + c] += curl_z - coef * jz;
}

// coef / dx etc. are rounded to R once on the host side of the launch
template <class R>
hipError_t launch_yee_b(const GridViewT<R>& g, double coef, hipStream_t st)
{
    const int N = g.nx * g.ny * g.nz;
    const R cf = (R)coef;
    hipLaunchKernelGGL(k_yee_b<R>, dim3((N + BLOCK - 1) / BLOCK), dim3(BLOCK), 0, st, g, cf / g.dx, cf / g.dy,
                       cf / g.dz);
    return hipGetLastError();
}

template <class R>
hipError_t launch_yee_e(const GridViewT<R>& g, double coef, hipStream_t st)
{
    const int N = g.nx * g.ny * g.nz;
    const R cf = (R)coef;
    hipLaunchKernelGGL(k_yee_e<R>, dim3((N + BLOCK - 1) / BLOCK), dim3(BLOCK), 0, st, g, cf / g.dx, cf / g.dy,
                       cf / g.dz, cf);
    return hipGetLastError();
}

template hipError_t launch_yee_b<float>(const GridView&, double, hipStream_t);
template hipError_t launch_yee_b<double>(const GridView64&, double, hipStream_t);
template hipError_t launch_yee_e<float>(const GridView&, double, hipStream_t);
template hipError_t launch_yee_e<double>(const GridView64&, double, hipStream_t);

}  // namespace pic
