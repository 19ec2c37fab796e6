// The particle kernel: per supercell, field gather (CIC, TSC or PCS on the Yee
// grid, standard or Galerkin),
// relativistic Boris push, move, and Esirkepov charge-conserving current
// deposition, fused in one pass over the supercell's frames.
//
// One workgroup per supercell, the paper's block-per-supercell mapping.  E
// and B for the supercell plus guard nodes are staged once into LDS; lane l
// handles slot l of every frame, so frames are read and written with fully
// coalesced fp32 loads and stores.  The current of all the supercell's
// particles accumulates in an LDS tile (plus guards) and is flushed to global
// J once, with global float atomics because neighbouring tiles overlap.
// Particles that leave the supercell are appended to the destination
// supercell's arrival list and their slot is recorded as a hole for the
// migration kernel.
//
// Current tile in 64-bit fixed point: on gfx950 an LDS float atomic add is
// serialised lane by lane (about 3 CU cycles per active lane, ~190 cycles per
// wave64 instruction) while 64-bit integer LDS atomics issue in ~8-14 cycles
// per wave instruction whatever the number of active lanes.  Each
// contribution is scaled by 2^30 / vmax (vmax bounds any single contribution:
// |q w| dx_d / (dV dt) times Esirkepov factors that lie in [-1, 1]), truncated
// to int32 and added as int64, so tile sums are exact and
// independent of the order of the atomics; the flush converts once.  (A 32-bit
// tile would need a scale that keeps every node sum of a supercell below 2^31,
// 2^31 / (n vmax) for n particles: measured, its rounding misses the 1e-4
// current bound on a thermal TSC plasma, whose node currents are small sums
// of large, mostly cancelling contributions.)
//
// The FP64 variant (R = double) accumulates the tile with native FP64 LDS
// atomics and flushes with FP64 global atomics instead.
//
// Two deposit paths (same Esirkepov arithmetic): a particle whose first shape
// node is unchanged on all three axes (it stays in its cell for CIC, keeps its
// nearest node for TSC) needs only an (ORDER+1)-node window per axis, which
// is done in line (CIC: 12 atomics instead of 54).  The others are queued in
// a per-supercell scratch list (wave ballot + popcount for the slots; for CIC
// each wave owns a region of it, so no LDS counter is needed) and
// deposited after the frame loop with the full (ORDER+2)-node window, so that
// no wave runs the wide window for a few of its lanes.  For CIC and TSC
// the queue keeps the particles whose first node changed along one axis only
// apart from the others: they deposit on a window that is wide along that
// axis alone (CIC 20 instead of 54 atomics, TSC 75 instead of 144).
#include <type_traits>

#include "pic_deposit.hpp"
#include "pic_migrate.hpp"

namespace pic {

// Largest arrival list the particle kernel can absorb in its LDS scratch.
__host__ __device__ constexpr int max_cap_in(int order)
{
    return order == 1 ? 2048 : 4096;
}
// LDS scratch of fill_supercell: three lists of cap_in ints and a bit mask.
constexpr int fill_scratch_bytes(int order)
{
    return (3 * max_cap_in(order) + (max_cap_in(order) + 31) / 32) * 4;
}
constexpr int cmax(int a, int b) { return a > b ? a : b; }
// Byte offset of the current tile in the particle kernel's LDS.
template <int ORDER, class R> constexpr int jtile_offset()
{
    return ORDER == 3 ? PcsTile::fbytes<R>() : Tile<ORDER, R>::FBYTES;
}
// LDS of the particle kernel: the tiles, or the arrival scratch that uses the
// same bytes before the tiles are staged, whichever is larger.
template <int ORDER, class R> constexpr int smem_bytes()
{
    return cmax(ORDER == 3 ? PcsTile::smem<R>() : Tile<ORDER, R>::SMEM, fill_scratch_bytes(ORDER));
}
// The current tile's 64-bit atomics, loads and stores need their natural
// alignment (a misaligned 64-bit LDS atomic faults); every instantiation keeps
// the tile on a 16-byte boundary and inside the kernel's LDS.
static_assert(jtile_offset<1, float>() % 16 == 0 && jtile_offset<1, double>() % 16 == 0, "CIC current tile alignment");
static_assert(jtile_offset<2, float>() % 16 == 0 && jtile_offset<2, double>() % 16 == 0, "TSC current tile alignment");
static_assert(jtile_offset<3, float>() % 16 == 0 && jtile_offset<3, double>() % 16 == 0, "PCS current tile alignment");
static_assert(jtile_offset<1, float>() + 3 * Tile<1>::JN * 8 <= smem_bytes<1, float>() &&
              jtile_offset<2, float>() + 3 * Tile<2>::JN * 8 <= smem_bytes<2, float>() &&
              jtile_offset<3, float>() + PcsTile::JNT * 8 <= smem_bytes<3, float>() &&
              jtile_offset<1, double>() + 3 * Tile<1>::JN * 8 <= smem_bytes<1, double>() &&
              jtile_offset<2, double>() + 3 * Tile<2>::JN * 8 <= smem_bytes<2, double>() &&
              jtile_offset<3, double>() + PcsTile::JNT * 8 <= smem_bytes<3, double>(),
              "current tile inside the LDS allocation");

// Current-tile accumulator: 64-bit fixed point for FP32, FP64 for FP64.
template <class R>
using JAcc = typename std::conditional<std::is_same<R, float>::value, unsigned long long, double>::type;
static_assert(sizeof(JAcc<float>) == 8 && sizeof(JAcc<double>) == 8, "8-byte current accumulators");

// Separable interpolation of one staged component: sum_c wz sum_b wy sum_a wx f
// over PX x PY x PZ nodes, f0 pointing at the component's first node (x
// fastest in the tile of a shape of order ORDER).
template <int ORDER, int PX, int PY, int PZ, class R>
__device__ inline R interp_n(const R* f0, const R* wx, const R* wy, const R* wz)
{
    using T = Tile<ORDER>;
    R acc = R(0);
#pragma unroll
    for (int c = 0; c < PZ; ++c) {
        R accy = R(0);
#pragma unroll
        for (int b = 0; b < PY; ++b) {
            const R* row = f0 + (c * T::GY + b) * T::GX;
            R accx = R(0);
#pragma unroll
            for (int a = 0; a < PX; ++a) accx = rfma(wx[a], row[a], accx);
            accy = rfma(wy[b], accx, accy);
        }
        acc = rfma(wz[c], accy, acc);
    }
    return acc;
}
template <int ORDER, class R>
__device__ inline R interp(const R* f0, const R* wx, const R* wy, const R* wz)
{
    constexpr int P = ORDER + 1;
    return interp_n<ORDER, P, P, P>(f0, wx, wy, wz);
}

// Fixed-point contribution (v already scaled, |v| <= 2^30), truncated to
// int32 and added as a sign-extended int64.  Truncation moves each
// contribution by less than 2^-30 vmax.
__device__ inline void jadd(unsigned long long* p, float v)
{
    const int iv = (int)v;
    atomicAdd(p, (unsigned long long)(long long)iv);
}
// FP64: a native LDS atomic add.
__device__ inline void jadd(double* p, double v) { atomicAdd(p, v); }
// The tile accumulation handed to the deposit functions.
struct LdsAdd {
    __device__ void operator()(unsigned long long* p, float v) const { jadd(p, v); }
    __device__ void operator()(double* p, double v) const { jadd(p, v); }
};

// Element at a 32-bit byte offset from a block-uniform base: lets the compiler
// use the scalar-base + 32-bit-offset global addressing form.
template <typename E>
__device__ inline E& at(E* base, unsigned byte_off)
{
    return *reinterpret_cast<E*>(reinterpret_cast<char*>(base) + byte_off);
}
template <typename E>
__device__ inline const E& at(const E* base, unsigned byte_off)
{
    return *reinterpret_cast<const E*>(reinterpret_cast<const char*>(base) + byte_off);
}

// Particle streams of the frame loop (read once, written once per step):
// with STREAM the loads and stores carry the non-temporal hint.  Measured
// about 1 % faster for CIC and slightly slower for TSC, so only CIC sets it.
template <bool STREAM, typename E>
__device__ inline E ld_part(const E* base, unsigned byte_off)
{
    if constexpr (STREAM) return __builtin_nontemporal_load(&at(base, byte_off));
    else return at(base, byte_off);
}
template <bool STREAM, typename E>
__device__ inline void st_part(E* base, unsigned byte_off, E v)
{
    if constexpr (STREAM) __builtin_nontemporal_store(v, &at(base, byte_off));
    else at(base, byte_off) = v;
}

// Add one node of a supercell's fixed-point current tile to global J: as an
// FP32 atomic, or (PIC_OPT_DETERMINISTIC_J) rescaled to the cycle's common
// scale (jratio <= 1, rounded to nearest) and added to the 64-bit fixed-point
// J, whose integer sums do not depend on the order of the tiles.
__device__ inline void flush_node(const GridView& g, int i, long long iv, float jinv, double jratio)
{
    if (iv == 0) return;
    if (g.J64) {
        const long long v = jratio == 1.0 ? iv : __double2ll_rn((double)iv * jratio);
        if (v != 0) atomicAdd(&g.J64[i], (unsigned long long)v);
    } else {
        unsafeAtomicAdd(&g.J[i], (float)((double)iv * (double)jinv));
    }
}

// Waves per SIMD the register budget is fitted to: 4 in FP32, 2 in FP64.
template <class R> constexpr int push_waves() { return std::is_same<R, float>::value ? 4 : 2; }

template <int ORDER, bool HAS_Z, bool GAL, int NT, class R>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(push_waves<R>())))
void k_push(GridViewT<R> g, SpeciesViewT<R> s, R jscale, R jinv, double jratio, int apar, int wpar)
{
    using T = Tile<ORDER, R>;
    using A = JAcc<R>;
    using R4 = typename Vec4<R>::type;
    constexpr unsigned RB = sizeof(R);
    constexpr bool PCS = ORDER == 3;  // PCS uses the trimmed tiles of PcsTile
    constexpr bool STREAM = ORDER == 1 && std::is_same<R, float>::value;
    constexpr int JL = PCS ? PcsTile::JL : T::JL;
    __shared__ __align__(16) unsigned char smem[smem_bytes<ORDER, R>()];
    R(*fE)[T::GN] = reinterpret_cast<R(*)[T::GN]>(smem);
    R(*fB)[T::GN] = reinterpret_cast<R(*)[T::GN]>(smem + 3 * T::GN * RB);
    R* const F = reinterpret_cast<R*>(smem);  // PCS: the six boxes at PcsTile::fbase
    A* tJ = reinterpret_cast<A*>(smem + jtile_offset<ORDER, R>());
    __shared__ int s_holes, s_queue, s_queue_m, s_cnt[3];
    // FP32 CIC: each wave appends its queued particles to a region of its own
    // (no LDS atomic, and no wait on one, inside the frame loop); measured 1 %
    // faster for CIC and 2-3 % slower for TSC, which keeps the shared queue
    constexpr bool WAVEQ = std::is_same<R, float>::value && ORDER == 1;
    // the other CIC and TSC kernels: one queue per supercell, its single-axis
    // crossers filled from the front and the others from the back (two LDS counters)
    constexpr bool QCLASS = !WAVEQ && ORDER <= 2;
    constexpr int NW = NT / 64;
    __shared__ int s_qn[NW], s_qo[NW];

    const int sc = sc_of_block(blockIdx.x, g.nsc, g.ncx * g.ncy, g.xcd_remap);
    // arrivals of the previous step first (frames dense again before pushing)
    if (apar >= 0) fill_supercell<NT>(g, s, sc, apar, reinterpret_cast<int*>(smem), s_cnt);
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int scx = sc % g.ncx, scy = (sc / g.ncx) % g.ncy, scz = sc / (g.ncx * g.ncy);
    const int ox = scx * SX, oy = scy * SY, oz = scz * SZ;
    const int N = g.nx * g.ny * g.nz;

    // ---- stage E, B with guards; zero the current tile
    for (int t = tid; t < T::GN; t += NT) {
        const int tx = t % T::GX, ty = (t / T::GX) % T::GY, tz = t / (T::GX * T::GY);
        int gx = ox + tx - T::GL, gy = oy + ty - T::GL, gz = oz + tz - T::GL;
        gx += (gx < 0) ? g.nx : 0; gx -= (gx >= g.nx) ? g.nx : 0;
        gy += (gy < 0) ? g.ny : 0; gy -= (gy >= g.ny) ? g.ny : 0;
        gz += (gz < 0) ? g.nz : 0; gz -= (gz >= g.nz) ? g.nz : 0;
        const int gi = gx + g.nx * (gy + g.ny * gz);
        if constexpr (PCS) {  // each component keeps the planes its stencil reaches
            const int z = tz - T::GL;
#pragma unroll
            for (int c = 0; c < 6; ++c)
                if (z >= PcsTile::zlo(c) && z < PcsTile::zlo(c) + PcsTile::zn(c))
                    F[PcsTile::fbase(c) + t] = c < 3 ? g.E[c * N + gi] : g.B[(c - 3) * N + gi];
        } else {
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                fE[c][t] = g.E[c * N + gi];
                fB[c][t] = g.B[c * N + gi];
            }
        }
    }
    for (int t = tid; t < (PCS ? PcsTile::JNT : 3 * T::JN); t += NT) tJ[t] = A(0);
    if (tid == 0) { s_holes = 0; s_queue = 0; s_queue_m = 0; }
    __syncthreads();
    const int wave = tid >> 6;
    const int rw = g.qcap / NW;  // queue region of one wave: >= its slots of every frame
    int qn = 0;                  // records this wave has queued (the same in all its active lanes):
    int qo = 0;                  // qn single-axis crossers from the front of its region, qo others from the back

    const int n = s.count[sc];
    const int64_t base = (int64_t)sc * s.cap;
    const int64_t qbase = (int64_t)sc * g.qcap;
    const R dt = g.dt;
    const R cdx = dt / g.dx, cdy = dt / g.dy, cdz = dt / g.dz;
    const R inv_dvdt = R(1) / (g.dx * g.dy * g.dz * dt);
    // current coefficients with the fixed-point scale folded in (1 in FP64)
    const R jcx = -g.dx * inv_dvdt * jscale, jcy = -g.dy * inv_dvdt * jscale, jcz = -g.dz * inv_dvdt * jscale;
    const R qm = R(0.5) * dt / s.mass;
    const R xm = face_below<R>((R)SX), ym = face_below<R>((R)SY), zm = face_below<R>((R)SZ);
    bool bad = false;

    // this supercell's frames: block-uniform base pointers, 32-bit slot offsets
    R* const px = s.x + base;
    R* const py = s.y + base;
    R* const pz = s.z + base;
    R* const pux = s.ux + base;
    R* const puy = s.uy + base;
    R* const puz = s.uz + base;
    const R* const pw = s.w + base;
    const uint8_t* const pzs = HAS_Z ? s.zs + base : nullptr;

    // ---- the frame loop: lane tid takes slot tid of every frame.  The
    // particle streams are software-pipelined: the loads of a later frame are
    // in flight while this one is computed.  With DEPTH2 (FP32 CIC and TSC)
    // two register sets alternate and the loop is unrolled by two, so the loads of
    // frame f + 2 are in flight during frame f and no register is copied
    // before its load has returned; otherwise one set holds frame f + 1.
    constexpr bool DEPTH2 = std::is_same<R, float>::value && ORDER <= 2;
    struct Part {
        R x, y, z, ux, uy, uz, w;
        int zs;
    };
    // unconditional (the last particle again past the end) so that no branch
    // obscures the order of these loads relative to the stores before them
    auto load_part = [&](int sl) {
        const unsigned un = RB * (unsigned)sl;
        Part p;
        p.x = ld_part<STREAM>(px, un); p.y = ld_part<STREAM>(py, un); p.z = ld_part<STREAM>(pz, un);
        p.ux = ld_part<STREAM>(pux, un); p.uy = ld_part<STREAM>(puy, un); p.uz = ld_part<STREAM>(puz, un);
        p.w = ld_part<STREAM>(pw, un);
        p.zs = 0;
        if constexpr (HAS_Z) p.zs = pzs[sl];
        return p;
    };
    // a copy of a prefetched set into new registers: an opaque move, so the
    // register allocator cannot merge the copy with the set and the next loads
    // of the set can target the set's own registers (no copy of an in-flight load)
    auto fresh = [](const Part& a) {
        Part c;
        asm("v_mov_b32 %0, %1" : "=v"(c.x) : "v"(a.x));
        asm("v_mov_b32 %0, %1" : "=v"(c.y) : "v"(a.y));
        asm("v_mov_b32 %0, %1" : "=v"(c.z) : "v"(a.z));
        asm("v_mov_b32 %0, %1" : "=v"(c.ux) : "v"(a.ux));
        asm("v_mov_b32 %0, %1" : "=v"(c.uy) : "v"(a.uy));
        asm("v_mov_b32 %0, %1" : "=v"(c.uz) : "v"(a.uz));
        asm("v_mov_b32 %0, %1" : "=v"(c.w) : "v"(a.w));
        asm("v_mov_b32 %0, %1" : "=v"(c.zs) : "v"(a.zs));
        return c;
    };
    // valid = false: a lane past the end of the last frame of a pair runs the
    // body on a copy of the last particle; it deposits and queues nothing, is
    // never a leaver and only stores into its own free slot (slot < cap)
    auto push_one = [&](const int slot, const Part& pp, const bool valid) {
        const unsigned u = RB * (unsigned)slot;  // byte offset of the slot
        const R x0 = pp.x, y0 = pp.y, z0 = pp.z;
        const R ux0 = pp.ux, uy0 = pp.uy, uz0 = pp.uz;
        const R wgt = pp.w;
        R q = s.charge;
        if constexpr (HAS_Z) q *= (R)pp.zs;

        // ---- gather at node-centred and half-shifted positions per axis;
        // the Galerkin gather takes the shape one order lower (ORDER nodes)
        // along each axis on which a component is staggered
        constexpr int SO = GAL ? ORDER - 1 : ORDER;
        constexpr int P = T::NP, Q = SO + 1;
        R wnx[P], wny[P], wnz[P], wsx[P], wsy[P], wsz[P];
        const int inx = shape_weights<ORDER>(x0, wnx), isx = shape_weights<SO>(x0 - R(0.5), wsx);
        const int iny = shape_weights<ORDER>(y0, wny), isy = shape_weights<SO>(y0 - R(0.5), wsy);
        const int inz = shape_weights<ORDER>(z0, wnz), isz = shape_weights<SO>(z0 - R(0.5), wsz);
        // tile index of the node-centred first node; the staggered first nodes
        // differ from it by one node at most per axis and lie in the tile
        const int bn = ((inz + T::GL) * T::GY + (iny + T::GL)) * T::GX + (inx + T::GL);
        const int ox_ = isx - inx, oy_ = (isy - iny) * T::GX, oz_ = (isz - inz) * (T::GX * T::GY);
        R Ex, Ey, Ez, Bx, By, Bz;
        if constexpr (PCS) {
            Ex = interp_n<ORDER, Q, P, P>(&F[PcsTile::fbase(0) + bn + ox_], wsx, wny, wnz);
            Ey = interp_n<ORDER, P, Q, P>(&F[PcsTile::fbase(1) + bn + oy_], wnx, wsy, wnz);
            Ez = interp_n<ORDER, P, P, Q>(&F[PcsTile::fbase(2) + bn + oz_], wnx, wny, wsz);
            Bx = interp_n<ORDER, P, Q, Q>(&F[PcsTile::fbase(3) + bn + oy_ + oz_], wnx, wsy, wsz) + g.b0x;
            By = interp_n<ORDER, Q, P, Q>(&F[PcsTile::fbase(4) + bn + ox_ + oz_], wsx, wny, wsz) + g.b0y;
            Bz = interp_n<ORDER, Q, Q, P>(&F[PcsTile::fbase(5) + bn + ox_ + oy_], wsx, wsy, wnz) + g.b0z;
        } else {
            Ex = interp_n<ORDER, Q, P, P>(&fE[0][bn + ox_], wsx, wny, wnz);
            Ey = interp_n<ORDER, P, Q, P>(&fE[1][bn + oy_], wnx, wsy, wnz);
            Ez = interp_n<ORDER, P, P, Q>(&fE[2][bn + oz_], wnx, wny, wsz);
            Bx = interp_n<ORDER, P, Q, Q>(&fB[0][bn + oy_ + oz_], wnx, wsy, wsz) + g.b0x;
            By = interp_n<ORDER, Q, P, Q>(&fB[1][bn + ox_ + oz_], wsx, wny, wsz) + g.b0y;
            Bz = interp_n<ORDER, Q, Q, P>(&fB[2][bn + ox_ + oy_], wsx, wsy, wnz) + g.b0z;
        }

        // ---- relativistic Boris: half kick, rotation, half kick
        const R h = q * qm;
        const R umx = rfma(h, Ex, ux0), umy = rfma(h, Ey, uy0), umz = rfma(h, Ez, uz0);
        const R hg = h * rrsq(R(1) + umx * umx + umy * umy + umz * umz);
        const R tx = hg * Bx, ty = hg * By, tz = hg * Bz;
        const R sf = R(2) * rrcp(R(1) + tx * tx + ty * ty + tz * tz);
        const R upx = umx + (umy * tz - umz * ty);
        const R upy = umy + (umz * tx - umx * tz);
        const R upz = umz + (umx * ty - umy * tx);
        R ux = rfma(h, Ex, umx + sf * (upy * tz - upz * ty));
        R uy = rfma(h, Ey, umy + sf * (upz * tx - upx * tz));
        R uz = rfma(h, Ez, umz + sf * (upx * ty - upy * tx));

        // ---- move
        const R ig = rrsq(R(1) + ux * ux + uy * uy + uz * uz);
        const R ddx = cdx * ux * ig, ddy = cdy * uy * ig, ddz = cdz * uz * ig;
        // a displacement of a cell or more (or NaN) keeps the particle where it
        // was, momentum included, and is reported.  In FP32 no branch leaves
        // the iteration here, so every lane reaches the stores below: a path
        // without them makes the compiler wait for all of this frame's stores
        // before the next frame's prefetched values can be used.  The FP64
        // instantiations keep the early exit (with the branch-free form the
        // FP64 PCS kernel, which spills, deposited wrong currents although its
        // IR differs only by the selects).
        const bool ok = rabs(ddx) < R(1) && rabs(ddy) < R(1) && rabs(ddz) < R(1);
        if constexpr (std::is_same<R, double>::value) {
            if (!ok) {
                bad = true;
                return;
            }
        }
        bad |= valid && !ok;
        if (!ok) { ux = ux0; uy = uy0; uz = uz0; }
        const R x1 = ok ? x0 + ddx : x0, y1 = ok ? y0 + ddy : y0, z1 = ok ? z0 + ddz : z0;

        // ---- current: in line when the first shape node is unchanged on every axis
        const R qw = q * wgt;
        R w1x[T::NP], w1y[T::NP], w1z[T::NP];
        const int fx1 = shape_weights<ORDER>(x1, w1x);
        const int fy1 = shape_weights<ORDER>(y1, w1y);
        const int fz1 = shape_weights<ORDER>(z1, w1z);
        const bool same = (fx1 == inx) && (fy1 == iny) && (fz1 == inz);
        if (same && valid) {
            R DSx[T::NP], DSy[T::NP], DSz[T::NP];
#pragma unroll
            for (int k = 0; k < T::NP; ++k) {
                DSx[k] = w1x[k] - wnx[k];
                DSy[k] = w1y[k] - wny[k];
                DSz[k] = w1z[k] - wnz[k];
            }
            deposit<ORDER, T::NP>(LdsAdd(), tJ, inx + JL, iny + JL, inz + JL, wnx, DSx, wny, DSy, wnz, DSz,
                                  jcx * qw, jcy * qw, jcz * qw);
        }
        // queue the others; one 32-byte record per particle: x0 y0 z0 qw | x1 y1 z1 s,
        // s the axis of a single-axis crossing where the queues keep that class
        // apart (per-wave regions for FP32 CIC, front and back of the supercell's
        // queue for the other CIC and TSC kernels), -1 for the others there
        const unsigned long long qmask = __ballot(!same && valid);
        if (qmask) {
            if constexpr (WAVEQ) {  // the wave's own region, crossers of one axis first
                const unsigned long long below = (1ull << lane) - 1ull;
                const int nax = (fx1 != inx) + (fy1 != iny) + (fz1 != inz);
                const unsigned long long smask = __ballot(valid && nax == 1);
                const unsigned long long mmask = qmask & ~smask;
                if (!same && valid) {
                    const bool one = nax == 1;
                    const int slot = one ? wave * rw + qn + __popcll(smask & below)
                                         : wave * rw + rw - 1 - (qo + __popcll(mmask & below));
                    const R ax = one ? R(fx1 != inx ? 0 : fy1 != iny ? 1 : 2) : R(-1);
                    R4* e = g.qbuf + 2 * (qbase + slot);
                    e[0] = make4(x0, y0, z0, qw);
                    e[1] = make4(x1, y1, z1, ax);
                }
                qn += __popcll(smask);
                qo += __popcll(mmask);
            } else if constexpr (QCLASS) {
                const unsigned long long below = (1ull << lane) - 1ull;
                const int nax = (fx1 != inx) + (fy1 != iny) + (fz1 != inz);
                const unsigned long long smask = __ballot(valid && !same && nax == 1);
                const unsigned long long mmask = qmask & ~smask;
                const int leader = __ffsll((long long)qmask) - 1;
                int sb = 0, mb = 0;
                if (lane == leader) {
                    if (smask) sb = atomicAdd(&s_queue, __popcll(smask));
                    if (mmask) mb = atomicAdd(&s_queue_m, __popcll(mmask));
                }
                sb = __shfl(sb, leader, 64);
                mb = __shfl(mb, leader, 64);
                if (!same && valid) {
                    const bool one = nax == 1;
                    const int slot = one ? sb + __popcll(smask & below) : g.qcap - 1 - (mb + __popcll(mmask & below));
                    const R ax = one ? R(fx1 != inx ? 0 : fy1 != iny ? 1 : 2) : R(-1);
                    R4* e = g.qbuf + 2 * (qbase + slot);
                    e[0] = make4(x0, y0, z0, qw);
                    e[1] = make4(x1, y1, z1, ax);
                }
            } else {  // contiguous slots per wave from one LDS atomic
                const int leader = __ffsll((long long)qmask) - 1;
                int qb = 0;
                if (lane == leader) qb = atomicAdd(&s_queue, __popcll(qmask));
                qb = __shfl(qb, leader, 64);
                if (!same && valid) {
                    R4* e = g.qbuf + 2 * (qbase + qb + __popcll(qmask & ((1ull << lane) - 1ull)));
                    e[0] = make4(x0, y0, z0, qw);
                    e[1] = make4(x1, y1, z1, R(0));
                }
            }
        }

        // ---- store in place; a particle that left the supercell keeps its
        // unshifted position here and its slot goes on the hole list, handed
        // over after the frame loop so no wave waits on a global atomic here
        st_part<STREAM>(px, u, x1); st_part<STREAM>(py, u, y1); st_part<STREAM>(pz, u, z1);
        st_part<STREAM>(pux, u, ux); st_part<STREAM>(puy, u, uy); st_part<STREAM>(puz, u, uz);
        const bool left = valid && ((x1 < R(0)) || (x1 >= (R)SX) || (y1 < R(0)) || (y1 >= (R)SY) ||
                                    (z1 < R(0)) || (z1 >= (R)SZ));
        const unsigned long long lmask = __ballot(left);
        if (lmask) {
            const int leader = __ffsll((long long)lmask) - 1;
            int hb = 0;
            if (lane == leader) hb = atomicAdd(&s_holes, __popcll(lmask));
            if constexpr (WAVEQ) hb = __builtin_amdgcn_readlane(hb, leader);
            else hb = __shfl(hb, leader, 64);
            const int hidx = hb + __popcll(lmask & ((1ull << lane) - 1ull));
            if (left) {
                if (hidx < s.cap_in) {
                    s.holes[(int64_t)sc * s.cap_in + hidx] = slot;
                } else {
                    // hole list full (reported through FLAG_MIGRATE below): keep the
                    // particle inside its supercell so every later access stays in bounds
                    at(px, u) = rmin(rmax(x1, R(0)), xm);
                    at(py, u) = rmin(rmax(y1, R(0)), ym);
                    at(pz, u) = rmin(rmax(z1, R(0)), zm);
                }
            }
        }
    };
    Part pa{}, pb{};
    if (n > 0) {  // block-uniform; lanes past the end load the last particle again
        pa = load_part(tid < n ? tid : n - 1);
        if constexpr (DEPTH2) {
            pb = load_part(NT + tid < n ? NT + tid : n - 1);
            // set A has arrived, set B stays in flight: the loop's waits then
            // count the steady state's loads and stores, not this prologue's
            constexpr int LOADS = HAS_Z ? 8 : 7;
            __builtin_amdgcn_s_waitcnt(0x0F70 | LOADS);  // vmcnt(LOADS)
        }
    }
    if constexpr (DEPTH2) {
        // pairs of frames whose second frame holds particles (so the first is
        // full): every lane runs both halves, none leaves the loop early, and
        // no memory access of the body lies on a path the compiler must treat
        // as skippable, so the waits it places count the steady state.  The
        // last frame of a pair ends at or below the slab's capacity (a
        // multiple of the frame size above the count).
        int f = 0;
        for (; f + NT < n; f += 2 * NT) {
            {
                const int slot = f + tid;
                const Part cur = fresh(pa);
                pa = load_part(slot + 2 * NT < n ? slot + 2 * NT : n - 1);
                push_one(slot, cur, true);
            }
            {
                const int slot = f + NT + tid;
                const Part cur = fresh(pb);
                pb = load_part(slot + 2 * NT < n ? slot + 2 * NT : n - 1);
                push_one(slot, cur, slot < n);
            }
        }
        if (f < n) {  // a last, single frame (set A)
            const int slot = f + tid;
            if (slot < n) push_one(slot, fresh(pa), true);
        }
    } else {
        (void)pb;
        for (int f = 0; f < n; f += NT) {
            const int slot = f + tid;
            if (slot >= n) break;
            const Part cur = pa;
            pa = load_part(slot + NT < n ? slot + NT : n - 1);
            push_one(slot, cur, true);
        }
    }
    if (bad) g.flags[FLAG_CFL] = 1;
    // lane 0 of a wave takes part in every frame its wave does, so it holds the count
    if (WAVEQ && lane == 0) { s_qn[wave] = qn; s_qo[wave] = qo; }
    __syncthreads();

    // ---- queued particles, all lanes busy
    auto queued = [&](int rec, bool one) {
        const R4* e = g.qbuf + 2 * (qbase + rec);
        const R4 a = e[0], b = e[1];
        const R x0 = a.x, y0 = a.y, z0 = a.z, qw = a.w;
        const R x1 = b.x, y1 = b.y, z1 = b.z;
        R S0x[T::W], DSx[T::W], S0y[T::W], DSy[T::W], S0z[T::W], DSz[T::W];
        const int mx = esirkepov_axis<ORDER>(x0, x1, S0x, DSx) + JL;
        const int my = esirkepov_axis<ORDER>(y0, y1, S0y, DSy) + JL;
        const int mz = esirkepov_axis<ORDER>(z0, z1, S0z, DSz) + JL;
        if constexpr (WAVEQ || QCLASS) {  // the queues that hold single-axis records
            if (one) {
                const int ax = min(max((int)b.w, 0), 2);
                deposit_cross1<ORDER>(LdsAdd(), tJ, ax, mx, my, mz, S0x, DSx, S0y, DSy, S0z, DSz, jcx * qw, jcy * qw, jcz * qw);
                return;
            }
        }
        deposit<ORDER, T::W>(LdsAdd(), tJ, mx, my, mz, S0x, DSx, S0y, DSy, S0z, DSz, jcx * qw, jcy * qw, jcz * qw);
    };
    if constexpr (WAVEQ) {
        // single-axis crossers (front of each wave's region), then the others (back)
        int qpre[NW], mpre[NW];
        int nq = 0, nm = 0;
#pragma unroll
        for (int w = 0; w < NW; ++w) { qpre[w] = nq; nq += s_qn[w]; mpre[w] = nm; nm += s_qo[w]; }
        for (int t = tid; t < nq; t += NT) {
            int rec = t;  // the last wave whose first index is <= t (waves may queue none)
#pragma unroll
            for (int k = 1; k < NW; ++k)
                if (t >= qpre[k]) rec = k * rw + (t - qpre[k]);
            queued(rec, true);
        }
        for (int t = tid; t < nm; t += NT) {
            int rec = rw - 1 - t;
#pragma unroll
            for (int k = 1; k < NW; ++k)
                if (t >= mpre[k]) rec = k * rw + rw - 1 - (t - mpre[k]);
            queued(rec, false);
        }
    } else if constexpr (QCLASS) {  // single-axis crossers (front), then the others (back)
        const int n1 = s_queue, nm = s_queue_m;
        for (int t = tid; t < n1; t += NT) queued(t, true);
        for (int t = tid; t < nm; t += NT) queued(g.qcap - 1 - t, false);
    } else {
        const int nq = s_queue;
        for (int t = tid; t < nq; t += NT) queued(t, false);
    }

    // ---- hand the leavers to their destination supercells' arrival lists
    const int nh = min(s_holes, s.cap_in);
    for (int t = tid; t < nh; t += NT) {
        const int slot = s.holes[(int64_t)sc * s.cap_in + t];
        const int64_t p = base + slot;
        const R x1 = s.x[p], y1 = s.y[p], z1 = s.z[p];
        const R lux = s.ux[p], luy = s.uy[p], luz = s.uz[p], lw = s.w[p];
        const uint32_t lid = s.id[p];
        const uint8_t lzs = HAS_Z ? s.zs[p] : (uint8_t)0;
        const int mvx = (x1 < R(0)) ? -1 : (x1 >= (R)SX ? 1 : 0);
        const int mvy = (y1 < R(0)) ? -1 : (y1 >= (R)SY ? 1 : 0);
        const int mvz = (z1 < R(0)) ? -1 : (z1 >= (R)SZ ? 1 : 0);
        int dx_ = scx + mvx, dy_ = scy + mvy, dz_ = scz + mvz;
        dx_ += (dx_ < 0) ? g.ncx : 0; dx_ -= (dx_ >= g.ncx) ? g.ncx : 0;
        dy_ += (dy_ < 0) ? g.ncy : 0; dy_ -= (dy_ >= g.ncy) ? g.ncy : 0;
        dz_ += (dz_ < 0) ? g.ncz : 0; dz_ -= (dz_ >= g.ncz) ? g.ncz : 0;
        const int dest = dx_ + g.ncx * (dy_ + g.ncy * dz_);
        // the slot in the destination's arrival list: one reservation per
        // destination and wave.  The active lanes are grouped by destination
        // (ballots only); each group's first lane then reserves the group's
        // slots, all groups in one atomic instruction.  Device-scope atomics
        // are resolved beyond the XCD's L2, where those on one address queue
        // behind each other: one per leaver cost 8 % of the CIC launch.
        unsigned long long todo = __ballot(true);
        int leader_of = lane, rank = 0, group = 0;
        while (todo) {
            const int first = __ffsll((long long)todo) - 1;
            const int d = __builtin_amdgcn_readlane(dest, first);
            const unsigned long long m = __ballot(dest == d) & todo;
            if ((m >> lane) & 1ull) {
                leader_of = first;
                rank = __popcll(m & ((1ull << lane) - 1ull));
            }
            if (lane == first) group = __popcll(m);
            todo &= ~m;
        }
        int kb = 0;
        if (group) kb = atomicAdd(&s.in_count[wpar * g.nsc + dest], group);
        const int k = __shfl(kb, leader_of, 64) + rank;
        if (k < s.cap_in) {
            const int64_t q_ = inbox_index(s, g.nsc, wpar, dest, k);
            // shift into the destination's frame; x - (-8) can round up onto the far face
            s.ix[q_] = rmin(x1 - (R)(mvx * SX), xm);
            s.iy[q_] = rmin(y1 - (R)(mvy * SY), ym);
            s.iz[q_] = rmin(z1 - (R)(mvz * SZ), zm);
            s.iux[q_] = lux; s.iuy[q_] = luy; s.iuz[q_] = luz;
            s.iw[q_] = lw;
            s.iid[q_] = lid;
            if constexpr (HAS_Z) s.izs[q_] = lzs;
        } else {
            g.flags[FLAG_MIGRATE] = 1;
        }
    }
    __syncthreads();

    // ---- flush the current tile (guards overlap neighbouring supercells)
    if constexpr (PCS) {
        for (int t = tid; t < PcsTile::JN; t += NT) {  // the J_x / J_y box; J_z has one plane less
            const int tx = t % PcsTile::JX, ty = (t / PcsTile::JX) % PcsTile::JY, tz = t / (PcsTile::JX * PcsTile::JY);
            int gx = ox + tx - JL, gy = oy + ty - JL, gz = oz + tz - JL;
            gx += (gx < 0) ? g.nx : 0; gx -= (gx >= g.nx) ? g.nx : 0;
            gy += (gy < 0) ? g.ny : 0; gy -= (gy >= g.ny) ? g.ny : 0;
            gz += (gz < 0) ? g.nz : 0; gz -= (gz >= g.nz) ? g.nz : 0;
            const int gi = gx + g.nx * (gy + g.ny * gz);
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                if (tz >= PcsTile::jz(c)) continue;
                if constexpr (std::is_same<R, float>::value) {
                    const long long iv = (long long)tJ[PcsTile::joff(c) + t];
                    flush_node(g, c * N + gi, iv, jinv, jratio);
                } else {
                    const double v = tJ[PcsTile::joff(c) + t];
                    if (v != 0.0) unsafeAtomicAdd(&g.J[c * N + gi], v);
                }
            }
        }
    } else {
        for (int t = tid; t < T::JN; t += NT) {
            const int tx = t % T::JX, ty = (t / T::JX) % T::JY, tz = t / (T::JX * T::JY);
            int gx = ox + tx - T::JL, gy = oy + ty - T::JL, gz = oz + tz - T::JL;
            gx += (gx < 0) ? g.nx : 0; gx -= (gx >= g.nx) ? g.nx : 0;
            gy += (gy < 0) ? g.ny : 0; gy -= (gy >= g.ny) ? g.ny : 0;
            gz += (gz < 0) ? g.nz : 0; gz -= (gz >= g.nz) ? g.nz : 0;
            const int gi = gx + g.nx * (gy + g.ny * gz);
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                if constexpr (std::is_same<R, float>::value) {
                    const long long iv = (long long)tJ[c * T::JN + t];
                    flush_node(g, c * N + gi, iv, jinv, jratio);
                } else {
                    const double v = tJ[c * T::JN + t];
                    if (v != 0.0) unsafeAtomicAdd(&g.J[c * N + gi], v);
                }
            }
        }
    }
    if (tid == 0) {
        const int h = s_holes;
        s.hole_count[sc] = h < s.cap_in ? h : s.cap_in;
        if (h > s.cap_in) g.flags[FLAG_MIGRATE] = 1;
    }
}

template <int ORDER, int NT, class R>
static void launch_push_order(const GridViewT<R>& g, const SpeciesViewT<R>& s, bool gal, R jscale, R jinv,
                              double jratio, int apar, int wpar, hipStream_t st)
{
    const dim3 grid(g.nsc), block(NT);
    const bool hz = s.zs != nullptr;
    if (gal) {
        if (hz) hipLaunchKernelGGL((k_push<ORDER, true, true, NT, R>), grid, block, 0, st, g, s, jscale, jinv, jratio, apar, wpar);
        else hipLaunchKernelGGL((k_push<ORDER, false, true, NT, R>), grid, block, 0, st, g, s, jscale, jinv, jratio, apar, wpar);
    } else {
        if (hz) hipLaunchKernelGGL((k_push<ORDER, true, false, NT, R>), grid, block, 0, st, g, s, jscale, jinv, jratio, apar, wpar);
        else hipLaunchKernelGGL((k_push<ORDER, false, false, NT, R>), grid, block, 0, st, g, s, jscale, jinv, jratio, apar, wpar);
    }
}

template <class R>
hipError_t launch_push(const GridViewT<R>& g, const SpeciesViewT<R>& s, int order, bool galerkin, double vmax,
                       float jscale_g, int apar, int wpar, hipStream_t st)
{
    // the deposit queue holds a full supercell, split evenly over the waves of a workgroup
    const int nt = order == 1 ? 256 : 512;
    // whole frames per slab: the paired frame loop runs every lane of a pair's
    // second frame, and a lane past the count stores into its own free slot
    if (s.cap % nt != 0 || s.cap > g.qcap || g.qcap % (nt / 64) != 0) return hipErrorInvalidValue;
    if (s.cap_in > max_cap_in(order)) return hipErrorInvalidValue;
    R jscale = R(1), jinv = R(1);
    double jratio = 1.0;
    if constexpr (std::is_same<R, float>::value) {
        // fixed-point scale: one contribution is at most vmax in magnitude -> |int| <= 2^30
        jscale = fixed_scale(vmax);
        jinv = 1.0f / jscale;
        // the common scale of the deterministic J is never finer than the species' own
        if (g.J64) {
            if (!(jscale_g > 0.0f) || jscale_g > jscale) return hipErrorInvalidValue;
            jratio = (double)jscale_g / (double)jscale;
        }
    }
    if (order == 1) launch_push_order<1, 256>(g, s, galerkin, jscale, jinv, jratio, apar, wpar, st);
    else if (order == 2) launch_push_order<2, 512>(g, s, galerkin, jscale, jinv, jratio, apar, wpar, st);
    else launch_push_order<3, 512>(g, s, galerkin, jscale, jinv, jratio, apar, wpar, st);
    return hipGetLastError();
}

template hipError_t launch_push<float>(const GridView&, const SpeciesView&, int, bool, double, float, int, int,
                                       hipStream_t);
template hipError_t launch_push<double>(const GridView64&, const SpeciesView64&, int, bool, double, float, int, int,
                                        hipStream_t);

}  // namespace pic
