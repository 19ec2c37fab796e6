// The particle kernel: per supercell, field gather (CIC/TSC on the Yee grid),
// relativistic Boris push, move, and Esirkepov charge-conserving current
// deposition, fused in one pass over the supercell's frames.
//
// One 256-lane workgroup (4 wave64) per supercell, the paper's
// block-per-supercell mapping.  E and B for the supercell plus guard nodes are
// staged once into LDS; lane l handles slot l of every 256-slot frame, so each
// frame is read and written with fully coalesced fp32 loads and stores.  The
// current of all the supercell's particles accumulates in an LDS tile (plus
// guards) and is flushed to global J once, with global float atomics because
// neighbouring tiles overlap.  Particles that leave the supercell are appended
// to the destination supercell's arrival list and their slot is recorded as a
// hole for the migration kernel.
//
// The LDS current tile is 64-bit fixed point.  On gfx950 an LDS float atomic
// add is serialised lane by lane (about 3 CU cycles per active lane, ~190
// cycles per wave64 instruction) while 64-bit integer LDS atomics issue in
// ~8-14 cycles per wave instruction.  Each contribution is scaled by
// 2^30 / vmax (vmax bounds any single contribution: |q w| dx_d / (dV dt)),
// rounded to int32 and added as int64, so the tile sums are exact and
// independent of the order of the atomics; the flush converts once to fp32.
#include "pic_device.hpp"

namespace pic {

template <int ORDER>
struct Tile {
    // gather tile: nodes [-1, S + ORDER] per axis
    static constexpr int GX = SX + 1 + ORDER, GY = SY + 1 + ORDER, GZ = SZ + 1 + ORDER;
    static constexpr int GN = GX * GY * GZ;
    // current tile: nodes [-ORDER, S + ORDER] per axis
    static constexpr int JL = ORDER;
    static constexpr int JX = SX + 2 * ORDER + 1, JY = SY + 2 * ORDER + 1, JZ = SZ + 2 * ORDER + 1;
    static constexpr int JN = JX * JY * JZ;
    static constexpr int NP = ORDER + 1;  // shape points per axis
    static constexpr int W = ORDER + 2;   // Esirkepov window per axis
};

// Separable interpolation of one staged component: sum_c wz sum_b wy sum_a wx f.
template <int ORDER>
__device__ inline float interp(const float* f, int ix, int iy, int iz, const float* wx, const float* wy,
                               const float* wz)
{
    using T = Tile<ORDER>;
    float acc = 0.0f;
#pragma unroll
    for (int c = 0; c < T::NP; ++c) {
        float accy = 0.0f;
#pragma unroll
        for (int b = 0; b < T::NP; ++b) {
            const float* row = f + ((iz + c + 1) * T::GY + (iy + b + 1)) * T::GX + (ix + 1);
            float accx = 0.0f;
#pragma unroll
            for (int a = 0; a < T::NP; ++a) accx = fmaf(wx[a], row[a], accx);
            accy = fmaf(wy[b], accx, accy);
        }
        acc = fmaf(wz[c], accy, acc);
    }
    return acc;
}

// Old and new shape on the Esirkepov window [m, m + W) of one axis.
template <int ORDER>
__device__ inline int esirkepov_axis(float x0, float x1, float* S0, float* DS)
{
    using T = Tile<ORDER>;
    float w0[T::NP], w1[T::NP];
    const int f0 = shape_weights<ORDER>(x0, w0);
    const int f1 = shape_weights<ORDER>(x1, w1);
    const int m = min(f0, f1);
    const int o0 = f0 - m, o1 = f1 - m;  // 0 or 1
#pragma unroll
    for (int k = 0; k < T::W; ++k) {
        const float a = (k < T::NP) ? w0[k] : 0.0f;
        const float b = (k >= 1) ? w0[k - 1] : 0.0f;
        const float c = (k < T::NP) ? w1[k] : 0.0f;
        const float d = (k >= 1) ? w1[k - 1] : 0.0f;
        const float s0 = o0 ? b : a;
        const float s1 = o1 ? d : c;
        S0[k] = s0;
        DS[k] = s1 - s0;
    }
    return m;
}

// Fixed-point contribution: round(v * scale) as a sign-extended 64-bit integer.
__device__ inline void jadd(unsigned long long* p, float v, float scale)
{
    const int iv = __float2int_rn(v * scale);
    atomicAdd(p, (unsigned long long)(long long)iv);
}

template <int ORDER, bool HAS_Z, int NT>
__global__ __launch_bounds__(NT) void k_push(GridView g, SpeciesView s, float jscale, float jinv)
{
    using T = Tile<ORDER>;
    __shared__ float fE[3][T::GN];
    __shared__ float fB[3][T::GN];
    __shared__ unsigned long long tJ[3][T::JN];
    __shared__ int s_holes;

    const int sc = sc_of_block(blockIdx.x, g.nsc, g.xcd_remap);
    const int tid = threadIdx.x;
    const int scx = sc % g.ncx, scy = (sc / g.ncx) % g.ncy, scz = sc / (g.ncx * g.ncy);
    const int ox = scx * SX, oy = scy * SY, oz = scz * SZ;
    const int N = g.nx * g.ny * g.nz;

    // ---- stage E, B with guards; zero the current tile
    for (int t = tid; t < T::GN; t += NT) {
        const int tx = t % T::GX, ty = (t / T::GX) % T::GY, tz = t / (T::GX * T::GY);
        int gx = ox + tx - 1, gy = oy + ty - 1, gz = oz + tz - 1;
        gx += (gx < 0) ? g.nx : 0; gx -= (gx >= g.nx) ? g.nx : 0;
        gy += (gy < 0) ? g.ny : 0; gy -= (gy >= g.ny) ? g.ny : 0;
        gz += (gz < 0) ? g.nz : 0; gz -= (gz >= g.nz) ? g.nz : 0;
        const int gi = gx + g.nx * (gy + g.ny * gz);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            fE[c][t] = g.E[c * N + gi];
            fB[c][t] = g.B[c * N + gi];
        }
    }
    for (int t = tid; t < 3 * T::JN; t += NT) (&tJ[0][0])[t] = 0ull;
    if (tid == 0) s_holes = 0;
    __syncthreads();

    const int n = s.count[sc];
    const int64_t base = (int64_t)sc * s.cap;
    const float dt = g.dt;
    const float cdx = dt / g.dx, cdy = dt / g.dy, cdz = dt / g.dz;
    const float inv_dvdt = 1.0f / (g.dx * g.dy * g.dz * dt);
    const float jcx = -g.dx * inv_dvdt, jcy = -g.dy * inv_dvdt, jcz = -g.dz * inv_dvdt;
    const float third = 1.0f / 3.0f;
    bool bad = false;

    for (int f = 0; f < n; f += NT) {
        const int slot = f + tid;
        if (slot >= n) break;
        const int64_t p = base + slot;
        const float x0 = s.x[p], y0 = s.y[p], z0 = s.z[p];
        float ux = s.ux[p], uy = s.uy[p], uz = s.uz[p];
        const float wgt = s.w[p];
        float q = s.charge;
        if constexpr (HAS_Z) q *= (float)s.zs[p];

        // ---- gather at node-centred and half-shifted positions per axis
        float wnx[T::NP], wny[T::NP], wnz[T::NP], wsx[T::NP], wsy[T::NP], wsz[T::NP];
        const int inx = shape_weights<ORDER>(x0, wnx), isx = shape_weights<ORDER>(x0 - 0.5f, wsx);
        const int iny = shape_weights<ORDER>(y0, wny), isy = shape_weights<ORDER>(y0 - 0.5f, wsy);
        const int inz = shape_weights<ORDER>(z0, wnz), isz = shape_weights<ORDER>(z0 - 0.5f, wsz);
        const float Ex = interp<ORDER>(fE[0], isx, iny, inz, wsx, wny, wnz);
        const float Ey = interp<ORDER>(fE[1], inx, isy, inz, wnx, wsy, wnz);
        const float Ez = interp<ORDER>(fE[2], inx, iny, isz, wnx, wny, wsz);
        const float Bx = interp<ORDER>(fB[0], inx, isy, isz, wnx, wsy, wsz) + g.b0x;
        const float By = interp<ORDER>(fB[1], isx, iny, isz, wsx, wny, wsz) + g.b0y;
        const float Bz = interp<ORDER>(fB[2], isx, isy, inz, wsx, wsy, wnz) + g.b0z;

        // ---- relativistic Boris: half kick, rotation, half kick
        const float h = 0.5f * q / s.mass * dt;
        const float umx = fmaf(h, Ex, ux), umy = fmaf(h, Ey, uy), umz = fmaf(h, Ez, uz);
        const float gm = sqrtf(1.0f + umx * umx + umy * umy + umz * umz);
        const float hg = h / gm;
        const float tx = hg * Bx, ty = hg * By, tz = hg * Bz;
        const float sf = 2.0f / (1.0f + tx * tx + ty * ty + tz * tz);
        const float upx = umx + (umy * tz - umz * ty);
        const float upy = umy + (umz * tx - umx * tz);
        const float upz = umz + (umx * ty - umy * tx);
        ux = fmaf(h, Ex, umx + sf * (upy * tz - upz * ty));
        uy = fmaf(h, Ey, umy + sf * (upz * tx - upx * tz));
        uz = fmaf(h, Ez, umz + sf * (upx * ty - upy * tx));

        // ---- move
        const float ig = 1.0f / sqrtf(1.0f + ux * ux + uy * uy + uz * uz);
        const float ddx = cdx * ux * ig, ddy = cdy * uy * ig, ddz = cdz * uz * ig;
        if (!(fabsf(ddx) < 1.0f && fabsf(ddy) < 1.0f && fabsf(ddz) < 1.0f)) {
            bad = true;  // a displacement of a cell or more (or NaN): keep the particle where it was
            continue;
        }
        const float x1 = x0 + ddx, y1 = y0 + ddy, z1 = z0 + ddz;

        // ---- Esirkepov current into the LDS tile
        {
            float S0x[T::W], DSx[T::W], S0y[T::W], DSy[T::W], S0z[T::W], DSz[T::W];
            const int mx = esirkepov_axis<ORDER>(x0, x1, S0x, DSx) + T::JL;
            const int my = esirkepov_axis<ORDER>(y0, y1, S0y, DSy) + T::JL;
            const int mz = esirkepov_axis<ORDER>(z0, z1, S0z, DSz) + T::JL;
            const float qw = q * wgt;
            // Esirkepov weights, factored: for the x current
            //   A(b,c) = S0y S0z + (DSy S0z + S0y DSz)/2 + DSy DSz/3
            //          = (S0y + DSy/2) S0z + (S0y/2 + DSy/3) DSz,
            // and cyclically for y and z.
            float Px[T::W], Qx[T::W], Py[T::W], Qy[T::W], Pz[T::W], Qz[T::W];
#pragma unroll
            for (int k = 0; k < T::W; ++k) {
                Px[k] = fmaf(0.5f, DSx[k], S0x[k]); Qx[k] = fmaf(third, DSx[k], 0.5f * S0x[k]);
                Py[k] = fmaf(0.5f, DSy[k], S0y[k]); Qy[k] = fmaf(third, DSy[k], 0.5f * S0y[k]);
                Pz[k] = fmaf(0.5f, DSz[k], S0z[k]); Qz[k] = fmaf(third, DSz[k], 0.5f * S0z[k]);
            }
            // running sums of DS along each axis (the last one is zero)
            float Rx[T::W - 1], Ry[T::W - 1], Rz[T::W - 1];
            Rx[0] = DSx[0]; Ry[0] = DSy[0]; Rz[0] = DSz[0];
#pragma unroll
            for (int k = 1; k < T::W - 1; ++k) {
                Rx[k] = Rx[k - 1] + DSx[k]; Ry[k] = Ry[k - 1] + DSy[k]; Rz[k] = Rz[k - 1] + DSz[k];
            }
            const float cx = jcx * qw, cy = jcy * qw, cz = jcz * qw;
            unsigned long long* Jx = &tJ[0][0];
            unsigned long long* Jy = &tJ[1][0];
            unsigned long long* Jz = &tJ[2][0];
#pragma unroll
            for (int c = 0; c < T::W; ++c)
#pragma unroll
                for (int b = 0; b < T::W; ++b) {
                    const int row = ((mz + c) * T::JY + (my + b)) * T::JX + mx;
                    const float ax = cx * fmaf(Py[b], S0z[c], Qy[b] * DSz[c]);
#pragma unroll
                    for (int a = 0; a < T::W - 1; ++a) jadd(&Jx[row + a], ax * Rx[a], jscale);
                }
#pragma unroll
            for (int c = 0; c < T::W; ++c)
#pragma unroll
                for (int a = 0; a < T::W; ++a) {
                    const float ay = cy * fmaf(Pz[c], S0x[a], Qz[c] * DSx[a]);
#pragma unroll
                    for (int b = 0; b < T::W - 1; ++b)
                        jadd(&Jy[((mz + c) * T::JY + (my + b)) * T::JX + (mx + a)], ay * Ry[b], jscale);
                }
#pragma unroll
            for (int b = 0; b < T::W; ++b)
#pragma unroll
                for (int a = 0; a < T::W; ++a) {
                    const float az = cz * fmaf(Px[a], S0y[b], Qx[a] * DSy[b]);
#pragma unroll
                    for (int c = 0; c < T::W - 1; ++c)
                        jadd(&Jz[((mz + c) * T::JY + (my + b)) * T::JX + (mx + a)], az * Rz[c], jscale);
                }
        }

        // ---- store, or hand the particle to its new supercell
        const int mvx = (x1 < 0.0f) ? -1 : (x1 >= (float)SX ? 1 : 0);
        const int mvy = (y1 < 0.0f) ? -1 : (y1 >= (float)SY ? 1 : 0);
        const int mvz = (z1 < 0.0f) ? -1 : (z1 >= (float)SZ ? 1 : 0);
        if ((mvx | mvy | mvz) == 0) {
            s.x[p] = x1; s.y[p] = y1; s.z[p] = z1;
            s.ux[p] = ux; s.uy[p] = uy; s.uz[p] = uz;
        } else {
            int dx_ = scx + mvx, dy_ = scy + mvy, dz_ = scz + mvz;
            dx_ += (dx_ < 0) ? g.ncx : 0; dx_ -= (dx_ >= g.ncx) ? g.ncx : 0;
            dy_ += (dy_ < 0) ? g.ncy : 0; dy_ -= (dy_ >= g.ncy) ? g.ncy : 0;
            dz_ += (dz_ < 0) ? g.ncz : 0; dz_ -= (dz_ >= g.ncz) ? g.ncz : 0;
            const int dest = dx_ + g.ncx * (dy_ + g.ncy * dz_);
            // shift into the destination's frame; x - (-8) can round up onto the far face
            const float nx1 = fminf(x1 - (float)(mvx * SX), XMAX);
            const float ny1 = fminf(y1 - (float)(mvy * SY), YMAX);
            const float nz1 = fminf(z1 - (float)(mvz * SZ), ZMAX);
            const int k = atomicAdd(&s.in_count[dest], 1);
            if (k < s.cap_in) {
                const int64_t q_ = (int64_t)dest * s.cap_in + k;
                s.ix[q_] = nx1; s.iy[q_] = ny1; s.iz[q_] = nz1;
                s.iux[q_] = ux; s.iuy[q_] = uy; s.iuz[q_] = uz;
                s.iw[q_] = wgt;
                s.iid[q_] = s.id[p];
                if constexpr (HAS_Z) s.izs[q_] = s.zs[p];
            } else {
                g.flags[FLAG_MIGRATE] = 1;
            }
            const int hidx = atomicAdd(&s_holes, 1);
            if (hidx < s.cap_in) s.holes[(int64_t)sc * s.cap_in + hidx] = slot;
        }
    }
    if (bad) g.flags[FLAG_CFL] = 1;
    __syncthreads();

    // ---- flush the current tile (guards overlap neighbouring supercells)
    for (int t = tid; t < T::JN; t += NT) {
        const int tx = t % T::JX, ty = (t / T::JX) % T::JY, tz = t / (T::JX * T::JY);
        int gx = ox + tx - T::JL, gy = oy + ty - T::JL, gz = oz + tz - T::JL;
        gx += (gx < 0) ? g.nx : 0; gx -= (gx >= g.nx) ? g.nx : 0;
        gy += (gy < 0) ? g.ny : 0; gy -= (gy >= g.ny) ? g.ny : 0;
        gz += (gz < 0) ? g.nz : 0; gz -= (gz >= g.nz) ? g.nz : 0;
        const int gi = gx + g.nx * (gy + g.ny * gz);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const long long iv = (long long)tJ[c][t];
            if (iv != 0) unsafeAtomicAdd(&g.J[c * N + gi], (float)((double)iv * (double)jinv));
        }
    }
    if (tid == 0) {
        const int h = s_holes;
        s.hole_count[sc] = h < s.cap_in ? h : s.cap_in;
        if (h > s.cap_in) g.flags[FLAG_MIGRATE] = 1;
    }
}

hipError_t launch_push(const GridView& g, const SpeciesView& s, int order, float vmax, hipStream_t st)
{
    const dim3 grid(g.nsc);
    const bool hz = s.zs != nullptr;
    // fixed-point scale: one contribution is at most vmax in magnitude -> |int| <= 2^30
    const float jscale = vmax > 0.0f ? 1073741824.0f / vmax : 1.0f;
    const float jinv = 1.0f / jscale;
    if (order == 1) {
        if (hz) hipLaunchKernelGGL((k_push<1, true, 256>), grid, dim3(256), 0, st, g, s, jscale, jinv);
        else hipLaunchKernelGGL((k_push<1, false, 256>), grid, dim3(256), 0, st, g, s, jscale, jinv);
    } else {
        if (hz) hipLaunchKernelGGL((k_push<2, true, 512>), grid, dim3(512), 0, st, g, s, jscale, jinv);
        else hipLaunchKernelGGL((k_push<2, false, 512>), grid, dim3(512), 0, st, g, s, jscale, jinv);
    }
    return hipGetLastError();
}

}  // namespace pic
