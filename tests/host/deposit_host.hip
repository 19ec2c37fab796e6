// Host-side driver of the particle kernel's deposit arithmetic (test
// infrastructure).  It runs the same esirkepov_axis / deposit /
// deposit_cross1 code that the particle kernel inlines, on the CPU, for one
// or more particles of one supercell, and returns the current tile in a
// uniform layout so that a test can compare it with a plain deposit on the
// whole periodic grid.
//
// Paths (as the particle kernel chooses them):
//   0  in line: the first shape node is unchanged on every axis, window of
//      ORDER + 1 nodes per axis;
//   1  general: window of ORDER + 2 nodes per axis (queued particles);
//   2  single axis: the first node changed along exactly one axis (queued
//      FP32 CIC particles); CIC and TSC only.
// Accumulation: plain (sum in double) when jscale is 0, else the fixed-point
// rule of the FP32 tile: the coefficients are multiplied by jscale (in the
// kernel's precision), each contribution is truncated to int32 and summed as
// int64; the largest |contribution| before the conversion is reported, so
// that a test can check the bound that keeps it inside int32.
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>

#include "../../paper_1606_02862_amd/csrc/pic_deposit.hpp"

namespace {

using namespace pic;

// Output layout: per component, nodes [-HL, S + HL] per axis.
constexpr int HL = 3;
constexpr int OX = SX + 2 * HL + 1, OY = SY + 2 * HL + 1, OZ = SZ + 2 * HL + 1, ON = OX * OY * OZ;

struct PlainAdd {
    template <class R> void operator()(double* p, R v) const { *p += (double)v; }
};
struct FixedAdd {
    double* vmax;
    template <class R> void operator()(int64_t* p, R v) const
    {
        *vmax = std::fmax(*vmax, std::fabs((double)v));
        *p += (int64_t)(int32_t)v;  // the kernel's conversion: truncation toward zero
    }
};

template <int ORDER>
struct Layout {  // current-tile geometry of the particle kernel for this order
    static constexpr bool PCS = ORDER == 3;
    static constexpr int JL = PCS ? PcsTile::JL : Tile<ORDER>::JL;
    static constexpr int JX = PCS ? PcsTile::JX : Tile<ORDER>::JX;
    static constexpr int JY = PCS ? PcsTile::JY : Tile<ORDER>::JY;
    static constexpr int JN = PCS ? PcsTile::JNT : 3 * Tile<ORDER>::JN;
    static int off(int c) { return PCS ? PcsTile::joff(c) : c * Tile<ORDER>::JN; }
    static int nz(int c) { return PCS ? PcsTile::jz(c) : Tile<ORDER>::JZ; }
};

template <int ORDER, class R, class A, class Add>
int one_particle(Add add, A* tJ, int path, const double* p0, const double* p1, const R* coef)
{
    using T = Tile<ORDER>;
    constexpr int JL = Layout<ORDER>::JL;
    const R x0 = (R)p0[0], y0 = (R)p0[1], z0 = (R)p0[2];
    const R x1 = (R)p1[0], y1 = (R)p1[1], z1 = (R)p1[2];
    if (path == 0) {
        R wnx[T::NP], wny[T::NP], wnz[T::NP], w1x[T::NP], w1y[T::NP], w1z[T::NP];
        const int inx = shape_weights<ORDER>(x0, wnx), iny = shape_weights<ORDER>(y0, wny),
                  inz = shape_weights<ORDER>(z0, wnz);
        const int fx1 = shape_weights<ORDER>(x1, w1x), fy1 = shape_weights<ORDER>(y1, w1y),
                  fz1 = shape_weights<ORDER>(z1, w1z);
        if (fx1 != inx || fy1 != iny || fz1 != inz) return -2;
        R DSx[T::NP], DSy[T::NP], DSz[T::NP];
        for (int k = 0; k < T::NP; ++k) {
            DSx[k] = w1x[k] - wnx[k];
            DSy[k] = w1y[k] - wny[k];
            DSz[k] = w1z[k] - wnz[k];
        }
        deposit<ORDER, T::NP>(add, tJ, inx + JL, iny + JL, inz + JL, wnx, DSx, wny, DSy, wnz, DSz, coef[0], coef[1],
                              coef[2]);
        return 0;
    }
    R S0x[T::W], DSx[T::W], S0y[T::W], DSy[T::W], S0z[T::W], DSz[T::W];
    const int mx = esirkepov_axis<ORDER>(x0, x1, S0x, DSx) + JL;
    const int my = esirkepov_axis<ORDER>(y0, y1, S0y, DSy) + JL;
    const int mz = esirkepov_axis<ORDER>(z0, z1, S0z, DSz) + JL;
    if (path == 1) {
        deposit<ORDER, T::W>(add, tJ, mx, my, mz, S0x, DSx, S0y, DSy, S0z, DSz, coef[0], coef[1], coef[2]);
        return 0;
    }
    if constexpr (ORDER != 3) {
        R w[T::NP];
        const int cx = shape_weights<ORDER>(x0, w) != shape_weights<ORDER>(x1, w);
        const int cy = shape_weights<ORDER>(y0, w) != shape_weights<ORDER>(y1, w);
        const int cz = shape_weights<ORDER>(z0, w) != shape_weights<ORDER>(z1, w);
        if (cx + cy + cz != 1) return -2;
        const int ax = cx ? 0 : cy ? 1 : 2;
        deposit_cross1<ORDER>(add, tJ, ax, mx, my, mz, S0x, DSx, S0y, DSy, S0z, DSz, coef[0], coef[1], coef[2]);
        return 0;
    }
    return -1;
}

template <int ORDER, class R>
int run(int path, int64_t n, const double* x0, const double* x1, const double* coef, double jscale, double* out,
        double* maxsum)
{
    using L = Layout<ORDER>;
    R c[3] = {(R)coef[0], (R)coef[1], (R)coef[2]};
    std::memset(out, 0, sizeof(double) * 3 * ON);
    *maxsum = 0.0;
    if (jscale > 0.0) {
        // the kernel folds the scale into the coefficients (in R) before the products
        for (int d = 0; d < 3; ++d) c[d] = (R)coef[d] * (R)jscale;
        int64_t* tJ = (int64_t*)std::calloc(L::JN, sizeof(int64_t));
        for (int64_t p = 0; p < n; ++p) {
            const int r = one_particle<ORDER, R>(FixedAdd{maxsum}, tJ, path, x0 + 3 * p, x1 + 3 * p, c);
            if (r) { std::free(tJ); return r; }
        }
        for (int comp = 0; comp < 3; ++comp)
            for (int z = 0; z < L::nz(comp); ++z)
                for (int y = 0; y < L::JY; ++y)
                    for (int x = 0; x < L::JX; ++x) {
                        const int64_t v = tJ[L::off(comp) + (z * L::JY + y) * L::JX + x];
                        out[comp * ON + ((z - L::JL + HL) * OY + (y - L::JL + HL)) * OX + (x - L::JL + HL)] =
                            (double)v / jscale;
                    }
        std::free(tJ);
        return 0;
    }
    double* tJ = (double*)std::calloc(L::JN, sizeof(double));
    for (int64_t p = 0; p < n; ++p) {
        const int r = one_particle<ORDER, R>(PlainAdd(), tJ, path, x0 + 3 * p, x1 + 3 * p, c);
        if (r) { std::free(tJ); return r; }
    }
    for (int comp = 0; comp < 3; ++comp)
        for (int z = 0; z < L::nz(comp); ++z)
            for (int y = 0; y < L::JY; ++y)
                for (int x = 0; x < L::JX; ++x)
                    out[comp * ON + ((z - L::JL + HL) * OY + (y - L::JL + HL)) * OX + (x - L::JL + HL)] =
                        tJ[L::off(comp) + (z * L::JY + y) * L::JX + x];
    std::free(tJ);
    return 0;
}

}  // namespace

extern "C" {

// Output dimensions and the node offset of element 0 (supercell-relative).
void pdh_layout(int* dims, int* lo)
{
    dims[0] = OX; dims[1] = OY; dims[2] = OZ;
    *lo = -HL;
}

// precision 0: FP32 arithmetic, 1: FP64.  x0, x1: n x 3 supercell-relative
// positions.  coef: the three current coefficients -(q w dx_d) / (dV dt).
// out: 3 x OZ x OY x OX doubles.  Returns 0, -1 for an unsupported
// combination, -2 when a particle does not qualify for the path.
int pdh_deposit(int precision, int order, int path, int64_t n, const double* x0, const double* x1, const double* coef,
                double jscale, double* out, double* maxsum)
{
    if (precision == 0) {
        if (order == 1) return run<1, float>(path, n, x0, x1, coef, jscale, out, maxsum);
        if (order == 2) return run<2, float>(path, n, x0, x1, coef, jscale, out, maxsum);
        if (order == 3) return run<3, float>(path, n, x0, x1, coef, jscale, out, maxsum);
    } else {
        if (order == 1) return run<1, double>(path, n, x0, x1, coef, jscale, out, maxsum);
        if (order == 2) return run<2, double>(path, n, x0, x1, coef, jscale, out, maxsum);
        if (order == 3) return run<3, double>(path, n, x0, x1, coef, jscale, out, maxsum);
    }
    return -1;
}

}  // extern "C"
