// Esirkepov charge-conserving current deposition of one particle into a
// supercell's current tile, and the tile geometry of the particle kernel.
//
// These functions hold the deposit arithmetic of the particle kernel and are
// callable on the host as well, so that the same code can be checked on the
// CPU against a plain deposit on the whole grid.  The accumulation into the
// tile is a functor (add(pointer, value)): the kernel passes its fixed-point
// (FP32) or FP64 LDS atomic, a host caller any plain add.
#pragma once

#include "pic_device.hpp"

namespace pic {

template <int ORDER, class R = float>
struct Tile {
    // gather tile: nodes [-GL, S + ORDER - GL] per axis (the staggered first
    // node reaches -1 for CIC and TSC and -2 for PCS)
    static constexpr int GL = (ORDER + 1) / 2;
    static constexpr int GX = SX + 1 + ORDER, GY = SY + 1 + ORDER, GZ = SZ + 1 + ORDER;
    static constexpr int GN = GX * GY * GZ;
    // current tile: nodes [-ORDER, S + ORDER] per axis
    static constexpr int JL = ORDER;
    static constexpr int JX = SX + 2 * ORDER + 1, JY = SY + 2 * ORDER + 1, JZ = SZ + 2 * ORDER + 1;
    static constexpr int JN = JX * JY * JZ;
    static constexpr int NP = ORDER + 1;  // shape points per axis
    static constexpr int W = ORDER + 2;   // Esirkepov window per axis (general case)
    // LDS of the particle kernel: field tiles, then the current tile (one
    // 8-byte accumulator per node and component: int64 fixed point in FP32,
    // double in FP64) at a 16-byte aligned offset
    static constexpr int FBYTES = (6 * GN * (int)sizeof(R) + 15) / 16 * 16;
    static constexpr int SMEM = FBYTES + 3 * JN * 8;
};

// PCS keeps only what its stencils reach, which halves its LDS and lets two
// workgroups share a CU (for CIC and TSC the same trimming measured 1-2 %
// slower than the full boxes above, which they keep).  Field components share
// the row and plane pitch of the full box; along z a component on the nodes
// needs planes [-1, SZ + 1] and one staggered by half a cell (E_z, B_x, B_y)
// [-2, SZ + 1].  Element (x, y, z) of component c is at
// fbase(c) + ((z + GL) GY + y + GL) GX + x + GL.  The current tile takes nodes
// [-2, S + 2] per axis (the deposit window's first node never lies below -2)
// and J_z one plane less along z.
template <int D = 0>  // a template so that its constants may use its own functions
struct PcsTileT {
    using T = Tile<3>;
    static constexpr int GL = T::GL, GX = T::GX, GY = T::GY;
    static constexpr bool zstag(int c) { return c == 2 || c == 3 || c == 4; }
    static constexpr int zlo(int c) { return zstag(c) ? -2 : -1; }
    static constexpr int zn(int c) { return zstag(c) ? SZ + 4 : SZ + 3; }
    static constexpr int foff(int c) { return c == 0 ? 0 : foff(c - 1) + zn(c - 1) * GX * GY; }
    static constexpr int fbase(int c) { return foff(c) - (zlo(c) + GL) * GX * GY; }
    static constexpr int FN = foff(6);
    static constexpr int JL = 2;
    static constexpr int JX = SX + 2 * JL + 1, JY = SY + 2 * JL + 1, JZ = SZ + 2 * JL + 1;
    static constexpr int JN = JX * JY * JZ;  // a full component box (J_x, J_y)
    static constexpr int jz(int c) { return c == 2 ? JZ - 1 : JZ; }
    static constexpr int joff(int c) { return c == 0 ? 0 : joff(c - 1) + jz(c - 1) * JX * JY; }
    static constexpr int JNT = joff(3);
    // the current tile at a 16-byte aligned offset (at least the natural
    // alignment of its atomics, loads and stores)
    template <class R> static constexpr int fbytes() { return (FN * (int)sizeof(R) + 15) / 16 * 16; }
    template <class R> static constexpr int smem() { return fbytes<R>() + JNT * 8; }
};
using PcsTile = PcsTileT<>;

// Old shape and shape change on the general window [m, m + W) of one axis.
template <int ORDER, class R>
__host__ __device__ inline int esirkepov_axis(R x0, R x1, R* S0, R* DS)
{
    using T = Tile<ORDER>;
    R w0[T::NP], w1[T::NP];
    const int f0 = shape_weights<ORDER>(x0, w0);
    const int f1 = shape_weights<ORDER>(x1, w1);
    const int m = f0 < f1 ? f0 : f1;
    const int o0 = f0 - m, o1 = f1 - m;  // 0 or 1
#pragma unroll
    for (int k = 0; k < T::W; ++k) {
        const R a = (k < T::NP) ? w0[k] : R(0);
        const R b = (k >= 1) ? w0[k - 1] : R(0);
        const R c = (k < T::NP) ? w1[k] : R(0);
        const R d = (k >= 1) ? w1[k - 1] : R(0);
        const R s0 = o0 ? b : a;
        const R s1 = o1 ? d : c;
        S0[k] = s0;
        DS[k] = s1 - s0;
    }
    return m;
}

// Esirkepov deposit of one particle on a window of W nodes per axis starting
// at tile nodes (mx, my, mz):
//   W_x(a,b,c) = DSx_a [S0y_b S0z_c + (DSy_b S0z_c + S0y_b DSz_c)/2 + DSy_b DSz_c/3]
//   J_x(a+1/2, b, c) = -(q w dx / (dV dt)) sum_{a' <= a} W_x(a',b,c)
// (cyclically for y and z), with the transverse factor written as
// (S0y + DSy/2) S0z + (S0y/2 + DSy/3) DSz.
template <int ORDER, int W, class R, class A, class Add>
__host__ __device__ inline void deposit(Add add, A* tJ, int mx, int my, int mz, const R* S0x, const R* DSx, const R* S0y, const R* DSy,
                               const R* S0z, const R* DSz, R cx, R cy, R cz)
{
    using T = Tile<ORDER>;
    const R third = R(1) / R(3);
    const R half = R(0.5);
    R Px[W], Qx[W], Py[W], Qy[W], Pz[W], Qz[W];
#pragma unroll
    for (int k = 0; k < W; ++k) {
        Px[k] = rfma(half, DSx[k], S0x[k]); Qx[k] = rfma(third, DSx[k], half * S0x[k]);
        Py[k] = rfma(half, DSy[k], S0y[k]); Qy[k] = rfma(third, DSy[k], half * S0y[k]);
        Pz[k] = rfma(half, DSz[k], S0z[k]); Qz[k] = rfma(third, DSz[k], half * S0z[k]);
    }
    R Rx[W - 1], Ry[W - 1], Rz[W - 1];  // running sums of DS (the last one is zero)
    Rx[0] = DSx[0]; Ry[0] = DSy[0]; Rz[0] = DSz[0];
#pragma unroll
    for (int k = 1; k < W - 1; ++k) {
        Rx[k] = Rx[k - 1] + DSx[k]; Ry[k] = Ry[k - 1] + DSy[k]; Rz[k] = Rz[k - 1] + DSz[k];
    }
    // PCS: the trimmed current tile (PcsTile), same origin in every component
    constexpr bool PCS = ORDER == 3;
    constexpr int TJX = PCS ? PcsTile::JX : T::JX, TJY = PCS ? PcsTile::JY : T::JY;
    A* Jx = tJ;
    A* Jy = tJ + (PCS ? PcsTile::joff(1) : T::JN);
    A* Jz = tJ + (PCS ? PcsTile::joff(2) : 2 * T::JN);
#pragma unroll
    for (int c = 0; c < W; ++c)
#pragma unroll
        for (int b = 0; b < W; ++b) {
            const int row = ((mz + c) * TJY + (my + b)) * TJX + mx;
            const R ax = cx * rfma(Py[b], S0z[c], Qy[b] * DSz[c]);
#pragma unroll
            for (int a = 0; a < W - 1; ++a) add(&Jx[row + a], ax * Rx[a]);
        }
#pragma unroll
    for (int c = 0; c < W; ++c)
#pragma unroll
        for (int a = 0; a < W; ++a) {
            const R ay = cy * rfma(Pz[c], S0x[a], Qz[c] * DSx[a]);
#pragma unroll
            for (int b = 0; b < W - 1; ++b) add(&Jy[((mz + c) * TJY + (my + b)) * TJX + (mx + a)], ay * Ry[b]);
        }
#pragma unroll
    for (int b = 0; b < W; ++b)
#pragma unroll
        for (int a = 0; a < W; ++a) {
            const R az = cz * rfma(Px[a], S0y[b], Qx[a] * DSy[b]);
#pragma unroll
            for (int c = 0; c < W - 1; ++c) add(&Jz[((mz + c) * TJY + (my + b)) * TJX + (mx + a)], az * Rz[c]);
        }
}

// Esirkepov deposit of a particle whose first shape node changed along one
// axis only (ax = 0, 1, 2 for x, y, z).  Along the two other axes the
// general window's last node has zero weight, so they take ORDER + 1 nodes:
// for CIC 8 + 6 + 6 atomics instead of 3 x 18.  The axes are relabelled per
// lane, a = ax, b = ax + 1, c = ax + 2 (mod 3), with the tile strides and
// current components following, so lanes that crossed along different axes
// share every instruction.  The terms are those of deposit(); the transverse
// factor of J_b is written as P_a S0_c + Q_a DS_c, the same sum.
template <int ORDER, class R, class A, class Add>
__host__ __device__ inline void deposit_cross1(Add add, A* tJ, int ax, int mx, int my, int mz, const R* S0x, const R* DSx,
                                      const R* S0y, const R* DSy, const R* S0z, const R* DSz, R cx, R cy, R cz)
{
    // the strides and component offsets below are those of the full tile
    // boxes (Tile); PCS keeps trimmed boxes (PcsTile) and never comes here
    static_assert(ORDER != 3, "deposit_cross1 addresses the Tile layout");
    using T = Tile<ORDER>;
    constexpr int W = T::W, NP = T::NP;
    const bool ix = ax == 0, iy = ax == 1;
    R S0a[W], DSa[W], S0b[NP], DSb[NP], S0c[NP], DSc[NP];
#pragma unroll
    for (int k = 0; k < W; ++k) {
        S0a[k] = ix ? S0x[k] : iy ? S0y[k] : S0z[k];
        DSa[k] = ix ? DSx[k] : iy ? DSy[k] : DSz[k];
    }
#pragma unroll
    for (int k = 0; k < NP; ++k) {
        S0b[k] = ix ? S0y[k] : iy ? S0z[k] : S0x[k];
        DSb[k] = ix ? DSy[k] : iy ? DSz[k] : DSx[k];
        S0c[k] = ix ? S0z[k] : iy ? S0x[k] : S0y[k];
        DSc[k] = ix ? DSz[k] : iy ? DSx[k] : DSy[k];
    }
    const R ca = ix ? cx : iy ? cy : cz, cb = ix ? cy : iy ? cz : cx, cc = ix ? cz : iy ? cx : cy;
    constexpr int PX = 1, PY = T::JX, PZ = T::JX * T::JY;  // tile strides
    const int sa = ix ? PX : iy ? PY : PZ, sb = ix ? PY : iy ? PZ : PX, sc = ix ? PZ : iy ? PX : PY;
    A* const Ja = tJ + (ix ? 0 : iy ? 1 : 2) * T::JN;
    A* const Jb = tJ + (ix ? 1 : iy ? 2 : 0) * T::JN;
    A* const Jc = tJ + (ix ? 2 : iy ? 0 : 1) * T::JN;
    const int o = mx * PX + my * PY + mz * PZ;
    const R third = R(1) / R(3);
    const R half = R(0.5);
    R Pa[W], Qa[W], Pb[NP], Qb[NP];
#pragma unroll
    for (int k = 0; k < W; ++k) { Pa[k] = rfma(half, DSa[k], S0a[k]); Qa[k] = rfma(third, DSa[k], half * S0a[k]); }
#pragma unroll
    for (int k = 0; k < NP; ++k) { Pb[k] = rfma(half, DSb[k], S0b[k]); Qb[k] = rfma(third, DSb[k], half * S0b[k]); }
    R Ra[W - 1], Rb[NP - 1], Rc[NP - 1];  // running sums of DS
    Ra[0] = DSa[0]; Rb[0] = DSb[0]; Rc[0] = DSc[0];
#pragma unroll
    for (int k = 1; k < W - 1; ++k) Ra[k] = Ra[k - 1] + DSa[k];
#pragma unroll
    for (int k = 1; k < NP - 1; ++k) { Rb[k] = Rb[k - 1] + DSb[k]; Rc[k] = Rc[k - 1] + DSc[k]; }
#pragma unroll
    for (int c = 0; c < NP; ++c)
#pragma unroll
        for (int b = 0; b < NP; ++b) {
            const R v = ca * rfma(Pb[b], S0c[c], Qb[b] * DSc[c]);
#pragma unroll
            for (int a = 0; a < W - 1; ++a) add(&Ja[o + c * sc + b * sb + a * sa], v * Ra[a]);
        }
#pragma unroll
    for (int c = 0; c < NP; ++c)
#pragma unroll
        for (int a = 0; a < W; ++a) {
            const R v = cb * rfma(Pa[a], S0c[c], Qa[a] * DSc[c]);
#pragma unroll
            for (int b = 0; b < NP - 1; ++b) add(&Jb[o + c * sc + b * sb + a * sa], v * Rb[b]);
        }
#pragma unroll
    for (int b = 0; b < NP; ++b)
#pragma unroll
        for (int a = 0; a < W; ++a) {
            const R v = cc * rfma(Pa[a], S0b[b], Qa[a] * DSb[b]);
#pragma unroll
            for (int c = 0; c < NP - 1; ++c) add(&Jc[o + c * sc + b * sb + a * sa], v * Rc[c]);
        }
}

}  // namespace pic
