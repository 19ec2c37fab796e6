// Learned ionisation-rate surrogate: 8 -> 64 -> 64 -> 1 network with SiLU or
// ReLU hidden activations (a template parameter of every kernel), BF16
// weights and activations on the matrix cores, FP32 accumulation.
//
// Wave tiling: a wave evaluates 16 samples at a time.  Lane l works on sample
// l % 16 for layer 1 and on hidden units 8*(l/16) + j (+32) so that its
// activations are directly the A operand of v_mfma_f32_16x16x32_bf16
// (A[i][k]: lane i + 16*(k/8) holds k % 8); layer 2 is 2 K-steps x 4 N-tiles
// = 8 MFMAs with W2 held in registers as the B operand; the result tile
// (D[i][n]: lane n%16 + 16*(i/4) holds i % 4) gets b2 + the activation and the dot
// with W3 as per-lane partial sums reduced over the 16 lanes of a row group.
// Layer 1 (2 continuous inputs + one-hot charge state) is a VALU column
// gather; the prior and the exact fallback are an FP32 / FP64 epilogue.
//
// Training uses the same forward plus a backward pass per 16-sample tile:
// dW2 = dZ2^T H1 and dH1 = dZ2 W2 on MFMA (16x16x16 over the samples and
// 16x16x32 over the hidden units), the small layers on VALU; gradients are
// summed per wave in registers / LDS and added to a global accumulator once
// per wave; Adam updates FP32 master weights.
#include "ionize_internal.hpp"

namespace pic {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr int NH = 64, NIN = 8;
constexpr int OFF_W1 = 0, OFF_B1 = NH * NIN, OFF_W2 = OFF_B1 + NH, OFF_B2 = OFF_W2 + NH * NH, OFF_W3 = OFF_B2 + NH,
              OFF_B3 = OFF_W3 + NH, NPARAM = OFF_B3 + 1;
static_assert(NPARAM == PIC_MLP_NPARAM, "parameter count");

__device__ inline float bf16r(float x) { return (float)(__bf16)x; }
__device__ inline float sigm(float z) { return __builtin_amdgcn_rcpf(1.0f + __expf(-z)); }
__device__ inline float silu(float z) { return z * sigm(z); }
__device__ inline float dsilu(float z)
{
    const float s = sigm(z);
    return s * (1.0f + z * (1.0f - s));
}
// The hidden activation and its derivative (ReLU': 1 for z > 0, else 0).
template <int ACT> __device__ inline float act_f(float z)
{
    if constexpr (ACT == PIC_MLP_RELU) return fmaxf(z, 0.0f);
    else return silu(z);
}
template <int ACT> __device__ inline float dact_f(float z)
{
    if constexpr (ACT == PIC_MLP_RELU) return z > 0.0f ? 1.0f : 0.0f;
    else return dsilu(z);
}

// Per charge state z: P_z, and the constant of the analytic prior (the
// outermost subshell's plain Lotz rate with e^{P/kT} E1(P/kT) replaced by
// ln(1 + kT/P))
// ln nu_prior = ln(n_e vbar a q / (P kT)) - P/kT + ln ln(1 + kT/P), with
// vbar = c sqrt(8 kT / (pi m_e c^2)):  c_z = ln(c sqrt(8 / (pi m_e c^2)) a_z q_z / P_z).
struct PriorTab {
    float P[PIC_MAX_ZSTATES], invP[PIC_MAX_ZSTATES], c[PIC_MAX_ZSTATES];
};

__device__ inline void fill_prior(const IonTables& tab, PriorTab& T)
{
    const int z = threadIdx.x;
    if (z < PIC_MAX_ZSTATES) {
        const double P = z < tab.z_max ? tab.P[z] : 1.0, aq = z < tab.z_max ? tab.aq[z][0] : LOTZ_A;
        T.P[z] = (float)P;
        T.invP[z] = (float)(1.0 / P);
        T.c[z] = (float)log(C_CM_S * sqrt(8.0 / (M_PI * ME_C2_EV)) * aq / P);
    }
}

// Network inputs x0 = (log10 kT - 2) / 2, x1 = (log10 n_e - 21) / 2 and the
// prior, in FP32 from the hardware base-2 logarithm; ln(1 + u) by the
// identity ln(1 + u) = u ln(w) / (w - 1), w = fl(1 + u), which keeps full
// relative accuracy for small u.
__device__ inline void inputs_prior(float kT, float ne, const PriorTab& T, int z, float& x0, float& x1, float& prior)
{
    constexpr float LN2 = 0.693147180559945309f, HALF_LOG10_2 = 0.150514997831990598f;
    const float l2t = __log2f(kT), l2n = __log2f(ne);
    x0 = fmaf(l2t, HALF_LOG10_2, -1.0f);
    x1 = fmaf(l2n, HALF_LOG10_2, -10.5f);
    const float u = kT * T.invP[z];
    const float w = 1.0f + u;
    const float l1p = w == 1.0f ? u : u * (LN2 * __log2f(w)) / (w - 1.0f);
    prior = LN2 * (l2n - 0.5f * l2t + __log2f(l1p)) + T.c[z] - T.P[z] / kT;
}

// Inference layout: the network runs transposed, hidden units as MFMA rows
// and 16 samples as columns, so that each layer's result tile (D[h][n]: lane
// n + 16*(h/4) of 16-row tile t holds hidden 16t + 4*(h/4) + e, e = 0..3) is
// already the next layer's B operand once its K index is relabelled.  A lane
// of group g = lane/16 holds, for K step s, the hidden units
//   kperm(s, g, j) = 32s + 16*(j/4) + 4g + j%4,   j = 0..7,
// and the weights of the next layer are loaded with the same relabelling (a
// contraction does not depend on the order of its K index).
__device__ inline int kperm(int s, int g, int j) { return 32 * s + 16 * (j >> 2) + 4 * g + (j & 3); }

// Layer 1 runs on a 16x16x16 MFMA with an augmented K of 16.  The inputs x0
// and x1 enter as two BF16 parts each (hi + mid carry 16 significant bits,
// well below the BF16 resolution of the activations), in the order x0_hi,
// x1_hi, x0_mid, x1_mid; then the six one-hot charge-state columns; then b1
// as three BF16 parts against a constant input of 1; then three zero columns.
// Every part is multiplied exactly by its BF16 weight, so layer 1 is the
// product of BF16 weights with the FP32 inputs plus the FP32 bias, up to the
// order of the FP32 sums.
// Inference runs the hidden layers in base 2: layer l computes z' = L z
// (L = log2 e) and the activation s(z') = z' / (1 + 2^{-z'}) = L silu(z), so
// that the activation needs no multiply before its exp2.  This folds L into
// W1, b1 and b2 and 1/L into W3 (W2 is unchanged: L silu(z1) feeds z2' =
// W2 (L silu(z1)) + L b2 = L z2).  The BF16 weights are rounded after the
// scaling.  ReLU commutes with the positive factor (max(L z, 0) = L max(z, 0)),
// so the same scaled weights serve both activations.
constexpr float LOG2E = 1.44269504088896341f;

__device__ inline float w1_aug(const float* P, int h, int k)
{
    if (k < 4) return bf16r(LOG2E * P[OFF_W1 + h * NIN + (k & 1)]);
    if (k < 10) return bf16r(LOG2E * P[OFF_W1 + h * NIN + 2 + (k - 4)]);
    if (k > 12) return 0.0f;
    const float b = LOG2E * P[OFF_B1 + h];
    const float hi = bf16r(b), mid = bf16r(b - hi), lo = bf16r(b - hi - mid);
    return k == 10 ? hi : (k == 11 ? mid : lo);
}

// The network slices one lane holds in registers (lane = c + 16g).
struct Net {
    bf16x4 a1[4];      // layer 1 A operand: row 16t + c, K columns 4g..4g+3 of the augmented W1
    bf16x8 a2[4][2];   // layer 2 A operand: W2[16t + c][kperm(s, g, j)]
    bf16x8 a3[2];      // head A operand: W3[kperm(s, g, j)] in rows c = 0, 4, 8, 12, zero elsewhere
    floatx4 b2[4];     // layer 2 bias in the result layout: b2[16t + 4g + e]
    float b3;
    // input column of group g (K rows 4g..4g+3) for charge state z:
    // (0x3F80 << 16 (z - zbase) if 0 <= z - zbase < 4) | cbits, BF16 1.0 = 0x3F80
    int zbase;
    uint64_t cbits;
};

__device__ inline void load_net(const float* P, int lane, Net& n)
{
    const int g = lane >> 4, c = lane & 15;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
#pragma unroll
        for (int e = 0; e < 4; ++e) n.a1[t][e] = (__bf16)w1_aug(P, 16 * t + c, 4 * g + e);
#pragma unroll
        for (int s = 0; s < 2; ++s)
#pragma unroll
            for (int j = 0; j < 8; ++j) n.a2[t][s][j] = (__bf16)P[OFF_W2 + (16 * t + c) * NH + kperm(s, g, j)];
#pragma unroll
        for (int e = 0; e < 4; ++e) n.b2[t][e] = LOG2E * P[OFF_B2 + 16 * t + 4 * g + e];
    }
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
        for (int j = 0; j < 8; ++j)
            n.a3[s][j] = (__bf16)((c & 3) == 0 ? P[OFF_W3 + kperm(s, g, j)] * (1.0f / LOG2E) : 0.0f);
    n.b3 = P[OFF_B3];
    n.zbase = g == 1 ? 0 : (g == 2 ? 4 : 64);                  // one-hot columns 0..3 and 4..5
    n.cbits = g == 2 ? 0x3F803F8000000000ull : (g == 3 ? 0x3F80ull : 0ull);  // b1 hi, mid | b1 lo
}

// Base-2 SiLU s(z) = z / (1 + 2^{-z}) (hardware exp2 and reciprocal).
__device__ inline float silu2(float z) { return z * __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(-z)); }

// The activation (base-2 SiLU, or ReLU) of a result tile pair, packed as the
// next layer's B operand for K step s.
template <int ACT> __device__ inline float act2(float z)
{
    if constexpr (ACT == PIC_MLP_RELU) return fmaxf(z, 0.0f);
    else return silu2(z);
}
template <int ACT> __device__ inline bf16x8 act_pack(const floatx4& lo, const floatx4& hi)
{
    bf16x8 r;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        r[e] = (__bf16)act2<ACT>(lo[e]);
        r[4 + e] = (__bf16)act2<ACT>(hi[e]);
    }
    return r;
}

// Forward of 16 samples: lane c + 16g supplies sample c's inputs (the packed
// BF16 pairs (x0_hi, x1_hi) and (x0_mid, x1_mid), and the charge state z;
// every group the same sample).  Returns y of sample c in every lane of
// column c.
template <int ACT> __device__ inline float forward16(const Net& n, int g, uint32_t xhi, uint32_t xmid, int z)
{
    const unsigned d = (unsigned)(z - n.zbase);
    const uint64_t onehot = d < 4u ? (0x3F80ull << (16u * d)) : 0ull;
    const uint64_t col = g == 0 ? ((uint64_t)xmid << 32 | xhi) : (onehot | n.cbits);
    bf16x4 xb;
    __builtin_memcpy(&xb, &col, 8);
    const floatx4 zero = {0.f, 0.f, 0.f, 0.f};
    floatx4 d1[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) d1[t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(n.a1[t], xb, zero, 0, 0, 0);
    const bf16x8 h1a = act_pack<ACT>(d1[0], d1[1]), h1b = act_pack<ACT>(d1[2], d1[3]);
    floatx4 d2[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        d2[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(n.a2[t][0], h1a, n.b2[t], 0, 0, 0);
        d2[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(n.a2[t][1], h1b, d2[t], 0, 0, 0);
    }
    const bf16x8 h2a = act_pack<ACT>(d2[0], d2[1]), h2b = act_pack<ACT>(d2[2], d2[3]);
    floatx4 d3 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(n.a3[0], h2a, zero, 0, 0, 0);
    d3 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(n.a3[1], h2b, d3, 0, 0, 0);
    return d3[0] + n.b3;  // row 4g of the head tile: y of sample c
}

// BF16 hi and mid parts of (x0, x1), packed as (x0, x1) pairs.
__device__ inline void split_inputs(float x0, float x1, uint32_t& hi, uint32_t& mid)
{
    const __bf16 h0 = (__bf16)x0, h1 = (__bf16)x1;
    const __bf16 m0 = (__bf16)(x0 - (float)h0), m1 = (__bf16)(x1 - (float)h1);
    uint16_t a, b, c, e;
    __builtin_memcpy(&a, &h0, 2); __builtin_memcpy(&b, &h1, 2);
    __builtin_memcpy(&c, &m0, 2); __builtin_memcpy(&e, &m1, 2);
    hi = (uint32_t)a | (uint32_t)b << 16;
    mid = (uint32_t)c | (uint32_t)e << 16;
}

// Forward of the 64 samples a wave holds, one per lane (z < 0: no sample).
// Sub-tile q takes the samples of lanes 16q..16q+15; its result for sample
// 16q + c lands in lane c + 16g for every g, so lane 16q + c reads its own.
template <int ACT> __device__ inline float forward64(const Net& n, int lane, float x0, float x1, int z)
{
    const int g = lane >> 4;
    uint32_t xhi, xmid;
    split_inputs(x0, x1, xhi, xmid);
    float y = 0.0f;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int src = 16 * q + (lane & 15);
        const int zq = __shfl(z, src, 64);
        if (__ballot(zq >= 0) == 0) continue;  // wave-uniform: the 16 samples are the same in every group
        const uint32_t hq = (uint32_t)__shfl((int)xhi, src, 64), mq = (uint32_t)__shfl((int)xmid, src, 64);
        const float yq = forward16<ACT>(n, g, hq, mq, zq);
        if (g == q) y = yq;
    }
    return y;
}

// ---------------------------------------------------------------- inference
// Exact FP64 rate for the (rare) samples outside the trained range, kept out
// of line so that its register footprint does not lower the occupancy of the
// surrogate path.
__device__ __noinline__ double fallback_rate(double kT, double ne, const IonTables& tab, int Z, const double* glx,
                                            const double* glw)
{
    return rate_exact(kT, ne, tab, Z, glx, glw);
}

struct MlpArgs {
    const float* params;
    float mu, s;
    float t_min, t_max, n_min, n_max;  // trained range (eV, cm^-3)
};


// Per supercell of ions: nu[p] for every ion (0 for Z >= z_max).  Ions whose
// inputs lie outside the trained range are appended to `fb_list` (their
// count in counters[CNT_FALLBACK]) and take the exact FP64 quadrature in a second,
// small kernel, so that the quadrature's registers do not lower this
// kernel's occupancy.  Persistent workgroups
// (weights loaded once); a wave takes 64 ions of a supercell at a time, one
// per lane.
template <int ACT>
__global__ __launch_bounds__(BLOCK) void k_rate_mlp(GridView g, SpeciesView ion, IonTables tab, MlpArgs m,
                                                    const double* ne, const double* kT, double* nu,
                                                    unsigned long long* counters, unsigned long long* fb_list)
{
    __shared__ PriorTab PT;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    fill_prior(tab, PT);
    Net net;
    load_net(m.params, lane, net);
    __syncthreads();
    for (int sc = blockIdx.x; sc < g.nsc; sc += gridDim.x) {
        const int n = ion.count[sc];
        const int64_t base = (int64_t)sc * ion.cap;
        const int scx = sc % g.ncx, scy = (sc / g.ncx) % g.ncy, scz = sc / (g.ncx * g.ncy);
        for (int t = 64 * wave + lane; t - lane < n; t += BLOCK) {
            float x0 = 0.f, x1 = 0.f, prior = 0.f;
            int Z = 0, zin = -1;
            bool act = false, inr = false;
            const int64_t p = base + t;
            if (t < n) {
                Z = ion.zs[p];
                act = Z < tab.z_max;
                const int64_t gi = (int64_t)(scx * SX + (int)ion.x[p]) +
                                   (int64_t)g.nx * ((scy * SY + (int)ion.y[p]) + (int64_t)g.ny * (scz * SZ + (int)ion.z[p]));
                const float fkT = (float)kT[gi], fne = (float)ne[gi];
                inr = act && Z < 6 && fkT >= m.t_min && fkT <= m.t_max && fne >= m.n_min && fne <= m.n_max;
                if (inr) {
                    inputs_prior(fkT, fne, PT, Z, x0, x1, prior);
                    zin = Z;
                }
            }
            const float y = forward64<ACT>(net, lane, x0, x1, zin);
            const bool fb = act && !inr;
            const unsigned long long fmask = __ballot(fb);
            if (fmask) {  // wave-uniform; rare
                const int leader = __ffsll((long long)fmask) - 1;
                unsigned long long fbase = 0;
                if (lane == leader) fbase = atomicAdd(&counters[CNT_FALLBACK], (unsigned long long)__popcll(fmask));
                fbase = __shfl(fbase, leader, 64);
                if (fb)
                    fb_list[fbase + (unsigned)__builtin_amdgcn_mbcnt_hi((unsigned)(fmask >> 32),
                                                                       __builtin_amdgcn_mbcnt_lo((unsigned)fmask, 0u))] =
                        (unsigned long long)p;
            }
            if (t < n) {
                // ln nu <= ~40 on the trained range; fallback ions are written by the second kernel
                nu[p] = inr ? (double)__expf(prior + m.mu + m.s * y) : 0.0;
            }
        }
    }
}

// The exact FP64 rate for the ions listed by k_rate_mlp.
__global__ __launch_bounds__(BLOCK) void k_rate_fallback(GridView g, SpeciesView ion, IonTables tab, const double* ne,
                                                         const double* kT, double* nu, const double* gl,
                                                         const unsigned long long* fb_list,
                                                         const unsigned long long* counters)
{
    __shared__ double glx[GL_NODES], glw[GL_NODES];
    if (threadIdx.x < GL_NODES) { glx[threadIdx.x] = gl[threadIdx.x]; glw[threadIdx.x] = gl[GL_NODES + threadIdx.x]; }
    __syncthreads();
    const unsigned long long cnt = counters[CNT_FALLBACK];
    for (unsigned long long i = (unsigned long long)blockIdx.x * BLOCK + threadIdx.x; i < cnt;
         i += (unsigned long long)gridDim.x * BLOCK) {
        const int64_t p = (int64_t)fb_list[i];
        const int sc = (int)(p / ion.cap);
        const int scx = sc % g.ncx, scy = (sc / g.ncx) % g.ncy, scz = sc / (g.ncx * g.ncy);
        const int64_t gi = (int64_t)(scx * SX + (int)ion.x[p]) +
                           (int64_t)g.nx * ((scy * SY + (int)ion.y[p]) + (int64_t)g.ny * (scz * SZ + (int)ion.z[p]));
        const int Z = ion.zs[p];
        nu[p] = rate_exact(kT[gi], ne[gi], tab, Z, glx, glw);
    }
}

hipError_t launch_rate_mlp(const GridView& g, const SpeciesView& ion, const IonTables& tab, const MlpLaunch& ml,
                           const double* ne, const double* kT, double* nu, const double* gl,
                           unsigned long long* counters, unsigned long long* fb_list, hipStream_t st)
{
    MlpArgs m{ml.params, (float)ml.mu, (float)ml.s, (float)ml.t_min, (float)ml.t_max, (float)ml.n_min, (float)ml.n_max};
    const int blocks = g.nsc < 1024 ? g.nsc : 1024;
    if (ml.act == PIC_MLP_RELU)
        hipLaunchKernelGGL(k_rate_mlp<PIC_MLP_RELU>, dim3(blocks), dim3(BLOCK), 0, st, g, ion, tab, m, ne, kT, nu,
                           counters, fb_list);
    else
        hipLaunchKernelGGL(k_rate_mlp<PIC_MLP_SILU>, dim3(blocks), dim3(BLOCK), 0, st, g, ion, tab, m, ne, kT, nu,
                           counters, fb_list);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_rate_fallback(g, ion, tab, ne, kT, nu, gl, fb_list, counters, st);
}

hipError_t launch_rate_fallback(const GridView& g, const SpeciesView& ion, const IonTables& tab, const double* ne,
                                const double* kT, double* nu, const double* gl, const unsigned long long* fb_list,
                                const unsigned long long* counters, hipStream_t st)
{
    hipLaunchKernelGGL(k_rate_fallback, dim3(256), dim3(BLOCK), 0, st, g, ion, tab, ne, kT, nu, gl, fb_list, counters);
    return hipGetLastError();
}

// ln nu of independent samples by the surrogate (exact fallback outside range).
template <int ACT>
__global__ __launch_bounds__(BLOCK) void k_ln_rate_mlp(int64_t n, const double* kT, const double* ne, const int32_t* Zs,
                                                       IonTables tab, MlpArgs m, const double* gl, double* out)
{
    __shared__ double glx[GL_NODES], glw[GL_NODES];
    __shared__ PriorTab PT;
    __shared__ IonTables s_tab;  // the out-of-line fallback reads the tables from LDS
    const int tid = threadIdx.x, lane = tid & 63;
    if (tid < GL_NODES) { glx[tid] = gl[tid]; glw[tid] = gl[GL_NODES + tid]; }
    if (tid == 0) s_tab = tab;
    fill_prior(tab, PT);
    Net net;
    load_net(m.params, lane, net);
    __syncthreads();
    const int64_t stride = (int64_t)gridDim.x * BLOCK;
    for (int64_t i = (int64_t)blockIdx.x * BLOCK + tid; i - lane < n; i += stride) {
        float x0 = 0.f, x1 = 0.f, prior = 0.f;
        int Z = -1, zin = -1;
        bool inr = false;
        if (i < n) {
            Z = Zs[i];
            const float fkT = (float)kT[i], fne = (float)ne[i];
            inr = Z >= 0 && Z < tab.z_max && Z < 6 && fkT >= m.t_min && fkT <= m.t_max && fne >= m.n_min &&
                  fne <= m.n_max;
            if (inr) {
                inputs_prior(fkT, fne, PT, Z, x0, x1, prior);
                zin = Z;
            }
        }
        const float y = forward64<ACT>(net, lane, x0, x1, zin);
        if (i < n) {
            if (inr) {
                out[i] = (double)(prior + m.mu + m.s * y);
            } else if (Z >= 0 && Z < tab.z_max) {
                const double v = fallback_rate(kT[i], ne[i], s_tab, Z, glx, glw);
                out[i] = v > 0.0 ? log(v) : -INFINITY;
            } else {
                out[i] = -INFINITY;
            }
        }
    }
}

hipError_t launch_ln_rate_mlp(int64_t n, const double* kT, const double* ne, const int32_t* Z, const IonTables& tab,
                              const MlpLaunch& ml, const double* gl, double* out, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    MlpArgs m{ml.params, (float)ml.mu, (float)ml.s, (float)ml.t_min, (float)ml.t_max, (float)ml.n_min, (float)ml.n_max};
    int64_t blocks = (n + BLOCK - 1) / BLOCK;
    if (blocks > 1024) blocks = 1024;
    if (ml.act == PIC_MLP_RELU)
        hipLaunchKernelGGL(k_ln_rate_mlp<PIC_MLP_RELU>, dim3((unsigned)blocks), dim3(BLOCK), 0, st, n, kT, ne, Z, tab,
                           m, gl, out);
    else
        hipLaunchKernelGGL(k_ln_rate_mlp<PIC_MLP_SILU>, dim3((unsigned)blocks), dim3(BLOCK), 0, st, n, kT, ne, Z, tab,
                           m, gl, out);
    return hipGetLastError();
}

// ---------------------------------------------------------------- training data
// Sample i: Philox (i, 0, 3, 0) -> log-uniform kT and n_e, Z uniform in 0..5;
// features (x0, x1, one-hot Z) and the exact residual target
// r = ln nu_exact - ln nu_prior (FP64; the prior here in FP64 too).
__global__ __launch_bounds__(BLOCK) void k_mlp_gen(int64_t n, uint64_t seed, MlpGen a, IonTables tab, const double* gl,
                                                   float* X, double* r)
{
    __shared__ double glx[GL_NODES], glw[GL_NODES];
    if (threadIdx.x < GL_NODES) { glx[threadIdx.x] = gl[threadIdx.x]; glw[threadIdx.x] = gl[GL_NODES + threadIdx.x]; }
    __syncthreads();
    const int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (i >= n) return;
    const Philox4 u = philox4x64_10((uint64_t)i, 0, PURPOSE_MLP_DATA, 0, seed, 0);
    const double lt = a.lt_min + (a.lt_max - a.lt_min) * u01(u.v[0]);
    const double ln10n = a.ln_min + (a.ln_max - a.ln_min) * u01(u.v[1]);
    int Z = (int)(u01(u.v[2]) * 6.0);
    Z = Z > 5 ? 5 : Z;
    const double kT = pow(10.0, lt), ne = pow(10.0, ln10n);
    float* x = X + i * NIN;
    x[0] = (float)((lt - 2.0) * 0.5);
    x[1] = (float)((ln10n - 21.0) * 0.5);
    for (int k = 0; k < 6; ++k) x[2 + k] = (k == Z) ? 1.0f : 0.0f;
    const double P = tab.P[Z], aq = tab.aq[Z][0];
    const double z = P / kT;
    const double prior = log(ne * vbar_cm_s(kT) * aq / (P * kT)) - z + log(log1p(1.0 / z));
    r[i] = ln_rate_exact(kT, ne, tab, Z, glx, glw) - prior;
}

hipError_t launch_mlp_gen(int64_t n, uint64_t seed, const MlpGen& a, const IonTables& tab, const double* gl, float* X,
                          double* r, hipStream_t st)
{
    hipLaunchKernelGGL(k_mlp_gen, dim3((unsigned)((n + BLOCK - 1) / BLOCK)), dim3(BLOCK), 0, st, n, seed, a, tab, gl, X,
                       r);
    return hipGetLastError();
}

// Mean and standard deviation of r (two passes, FP64): partial sums per block,
// then one block finishes; target t = (r - mu) / s written as FP32.
__global__ __launch_bounds__(BLOCK) void k_mlp_moments(int64_t n, const double* r, double* partial)
{
    __shared__ double sa[BLOCK / 64], sb[BLOCK / 64];
    double a = 0.0, b = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x; i < n; i += (int64_t)gridDim.x * BLOCK) {
        a += r[i];
        b += r[i] * r[i];
    }
    for (int o = 32; o > 0; o >>= 1) { a += __shfl_xor(a, o, 64); b += __shfl_xor(b, o, 64); }
    if ((threadIdx.x & 63) == 0) { sa[threadIdx.x >> 6] = a; sb[threadIdx.x >> 6] = b; }
    __syncthreads();
    if (threadIdx.x == 0) {
        double ta = 0.0, tb = 0.0;
        for (int w = 0; w < BLOCK / 64; ++w) { ta += sa[w]; tb += sb[w]; }
        partial[2 * blockIdx.x] = ta;
        partial[2 * blockIdx.x + 1] = tb;
    }
}

__global__ void k_mlp_moments_final(int64_t n, int nb, const double* partial, double* mu_s)
{
    if (threadIdx.x != 0) return;
    double a = 0.0, b = 0.0;
    for (int i = 0; i < nb; ++i) { a += partial[2 * i]; b += partial[2 * i + 1]; }
    const double mu = a / (double)n;
    double var = b / (double)n - mu * mu;
    var = var > 1e-300 ? var : 1e-300;
    mu_s[0] = mu;
    mu_s[1] = sqrt(var);
}

__global__ __launch_bounds__(BLOCK) void k_mlp_targets(int64_t n, const double* r, const double* mu_s, float* t)
{
    const int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (i < n) t[i] = (float)((r[i] - mu_s[0]) / mu_s[1]);
}

hipError_t launch_mlp_standardize(int64_t n, const double* r, double* partial, double* mu_s, float* t, hipStream_t st)
{
    const int nb = 512;
    hipLaunchKernelGGL(k_mlp_moments, dim3(nb), dim3(BLOCK), 0, st, n, r, partial);
    hipLaunchKernelGGL(k_mlp_moments_final, dim3(1), dim3(64), 0, st, n, nb, partial, mu_s);
    hipLaunchKernelGGL(k_mlp_targets, dim3((unsigned)((n + BLOCK - 1) / BLOCK)), dim3(BLOCK), 0, st, n, r, mu_s, t);
    return hipGetLastError();
}

// Initial weights: uniform(-1,1) * sqrt(3 / fan_in) from Philox (p, 0, 5, 0); biases 0.
__global__ void k_mlp_init(uint64_t seed, float* P, float* adam_m, float* adam_v)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= NPARAM) return;
    const Philox4 u = philox4x64_10((uint64_t)i, 0, PURPOSE_MLP_INIT, 0, seed, 0);
    const double v = 2.0 * u01(u.v[0]) - 1.0;
    float w = 0.0f;
    if (i < OFF_B1) w = (float)(v * sqrt(3.0 / NIN));
    else if (i >= OFF_W2 && i < OFF_B2) w = (float)(v * sqrt(3.0 / NH));
    else if (i >= OFF_W3 && i < OFF_B3) w = (float)(v * sqrt(3.0 / NH));
    P[i] = w;
    adam_m[i] = 0.0f;
    adam_v[i] = 0.0f;
}

hipError_t launch_mlp_init(uint64_t seed, float* P, float* m, float* v, hipStream_t st)
{
    hipLaunchKernelGGL(k_mlp_init, dim3((NPARAM + 255) / 256), dim3(256), 0, st, seed, P, m, v);
    return hipGetLastError();
}

// ---------------------------------------------------------------- training step
// Forward + backward of a minibatch.  Sample slot b of the batch is training
// sample b (draw_seed == 0) or Philox (b, step, 4, 0) mod n_data.  Every wave
// takes 16-sample tiles.  The block's gradient and squared-error sum (its
// waves' partials added in wave order in LDS) go to row blockIdx.x of part
// and lpart: no atomics, so the sums have a fixed order and training is
// reproducible bit for bit.  (With one device-scope atomic add per wave and
// parameter, those on one address queued behind each other beyond the L2 and
// took a third of the step.)
struct StepArgs {
    const float* X;      // [n_data][8]
    const float* t;      // [n_data]
    int64_t n_data;
    int batch;
    uint64_t draw_seed;
    int64_t step;
};

template <int ACT>
__global__ __launch_bounds__(BLOCK) void k_mlp_step(const float* P, StepArgs a, float* part, double* lpart)
{
    __shared__ float sW2[NH][NH + 1];                 // W2 (bf16-rounded), [out][in]
    __shared__ float sW1[NH][NIN], sB1[NH], sW3[NH];
    // per-wave H1 tiles [sample][k] and dZ2 tiles [sample][n]; after the
    // rounds, the block's gradient
    __shared__ float tiles[2][BLOCK / 64][16][NH + 1];
    auto& h1t = tiles[0];
    auto& dz2t = tiles[1];
    static_assert(sizeof(tiles) >= NPARAM * sizeof(float), "the block gradient fits the tiles");
    __shared__ float gW1[BLOCK / 64][NH][NIN + 1];     // per-wave dW1 | db1
    __shared__ double sL[BLOCK / 64];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int g = lane >> 4, c = lane & 15;
    for (int i = tid; i < NH * NH; i += BLOCK) sW2[i / NH][i % NH] = bf16r(P[OFF_W2 + i]);
    for (int i = tid; i < NH * NIN; i += BLOCK) sW1[i / NIN][i % NIN] = bf16r(P[OFF_W1 + i]);
    for (int i = tid; i < NH; i += BLOCK) { sB1[i] = P[OFF_B1 + i]; sW3[i] = bf16r(P[OFF_W3 + i]); }
    for (int i = lane; i < NH * (NIN + 1); i += 64) gW1[wave][i / (NIN + 1)][i % (NIN + 1)] = 0.0f;
    __syncthreads();
    const float b3 = P[OFF_B3];
    float b2v[4];
    for (int t = 0; t < 4; ++t) b2v[t] = P[OFF_B2 + 16 * t + c];

    floatx4 accW2[4][4];  // dW2 tiles [n-tile][k-tile]
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) accW2[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};
    float gW3[4] = {0.f, 0.f, 0.f, 0.f}, gB2[4] = {0.f, 0.f, 0.f, 0.f}, gB3 = 0.f;
    double lsum = 0.0;
    const float inv_b = 1.0f / (float)a.batch;

    auto sample = [&](int b) -> int64_t {
        if (a.draw_seed == 0) return b;
        const Philox4 u = philox4x64_10((uint64_t)b, (uint64_t)a.step, PURPOSE_MLP_BATCH, 0, a.draw_seed, 0);
        return (int64_t)(u.v[0] % (uint64_t)a.n_data);
    };
    const int ntile = a.batch / 16;
    const int nwave = gridDim.x * (BLOCK / 64);
    // every wave of the block runs the same number of rounds (barriers inside)
    for (int round = blockIdx.x * (BLOCK / 64); round < ntile; round += nwave) {
        const int tile = round + wave;
        const bool valid = tile < ntile;
        bf16x8 h1[2];
        float z2[4][4], dy[4];
        if (valid) {
            const int64_t si = sample(16 * tile + c);
            float x[NIN];
            for (int k = 0; k < NIN; ++k) x[k] = a.X[si * NIN + k];
            // layer 1 for hidden units 32s + 8g + j of sample c
            for (int s = 0; s < 2; ++s)
                for (int j = 0; j < 8; ++j) {
                    const int k = 32 * s + 8 * g + j;
                    float z = sB1[k];
                    for (int q = 0; q < NIN; ++q) z = fmaf(sW1[k][q], x[q], z);
                    const float h = bf16r(act_f<ACT>(z));
                    h1[s][j] = (__bf16)h;
                    h1t[wave][c][k] = h;
                }
            // layer 2 + head: rows i = 4g + r, columns n = 16t + c
            float y[4] = {0.f, 0.f, 0.f, 0.f};
            for (int t = 0; t < 4; ++t) {
                bf16x8 w[2];
                for (int s = 0; s < 2; ++s)
                    for (int j = 0; j < 8; ++j) w[s][j] = (__bf16)sW2[16 * t + c][32 * s + 8 * g + j];
                floatx4 d = {0.f, 0.f, 0.f, 0.f};
                d = __builtin_amdgcn_mfma_f32_16x16x32_bf16(h1[0], w[0], d, 0, 0, 0);
                d = __builtin_amdgcn_mfma_f32_16x16x32_bf16(h1[1], w[1], d, 0, 0, 0);
                for (int r = 0; r < 4; ++r) {
                    z2[t][r] = d[r] + b2v[t];
                    y[r] = fmaf(sW3[16 * t + c], bf16r(act_f<ACT>(z2[t][r])), y[r]);
                }
            }
            for (int r = 0; r < 4; ++r) {
                float v = y[r];
                v += __shfl_xor(v, 1, 64);
                v += __shfl_xor(v, 2, 64);
                v += __shfl_xor(v, 4, 64);
                v += __shfl_xor(v, 8, 64);
                const int64_t so = sample(16 * tile + 4 * g + r);
                const float res = v + b3 - a.t[so];
                dy[r] = 2.0f * res * inv_b;
                if (c == 0) lsum += (double)res * res;
            }
            // head and layer-2 backward: dZ2[i][n] = dy_i W3[n] act'(z2)
            for (int t = 0; t < 4; ++t)
                for (int r = 0; r < 4; ++r) {
                    const float h2 = bf16r(act_f<ACT>(z2[t][r]));
                    gW3[t] = fmaf(dy[r], h2, gW3[t]);
                    const float dz = dy[r] * sW3[16 * t + c] * dact_f<ACT>(z2[t][r]);
                    gB2[t] += dz;
                    dz2t[wave][4 * g + r][16 * t + c] = dz;
                }
            for (int r = 0; r < 4; ++r) gB3 += (c == 0) ? dy[r] : 0.0f;
        }
        __syncthreads();  // h1t / dz2t of this round complete
        if (valid) {
            // dW2[n][k] += sum_i dZ2[i][n] H1[i][k]: 16x16x16 MFMA, K = the 16 samples
            for (int tn = 0; tn < 4; ++tn) {
                bf16x4 A;
                for (int j = 0; j < 4; ++j) A[j] = (__bf16)dz2t[wave][4 * g + j][16 * tn + c];
                for (int tk = 0; tk < 4; ++tk) {
                    bf16x4 Bv;
                    for (int j = 0; j < 4; ++j) Bv[j] = (__bf16)h1t[wave][4 * g + j][16 * tk + c];
                    accW2[tn][tk] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(A, Bv, accW2[tn][tk], 0, 0, 0);
                }
            }
            // dH1[i][k] = sum_n dZ2[i][n] W2[n][k]: 16x16x32 MFMA over n; rows 4g + r, column 16tk + c
            bf16x8 dA[2];
            for (int s = 0; s < 2; ++s)
                for (int j = 0; j < 8; ++j) dA[s][j] = (__bf16)dz2t[wave][c][32 * s + 8 * g + j];
            for (int tk = 0; tk < 4; ++tk) {
                bf16x8 Bv[2];
                for (int s = 0; s < 2; ++s)
                    for (int j = 0; j < 8; ++j) Bv[s][j] = (__bf16)sW2[32 * s + 8 * g + j][16 * tk + c];
                floatx4 d = {0.f, 0.f, 0.f, 0.f};
                d = __builtin_amdgcn_mfma_f32_16x16x32_bf16(dA[0], Bv[0], d, 0, 0, 0);
                d = __builtin_amdgcn_mfma_f32_16x16x32_bf16(dA[1], Bv[1], d, 0, 0, 0);
                // dZ1 = dH1 act'(z1) for samples 4g + r at unit k; dW1 / db1 partials
                const int k = 16 * tk + c;
                float part[NIN + 1];
                for (int q = 0; q <= NIN; ++q) part[q] = 0.0f;
                for (int r = 0; r < 4; ++r) {
                    const int64_t so = sample(16 * tile + 4 * g + r);
                    float xs[NIN];
                    for (int q = 0; q < NIN; ++q) xs[q] = a.X[so * NIN + q];
                    float z1 = sB1[k];
                    for (int q = 0; q < NIN; ++q) z1 = fmaf(sW1[k][q], xs[q], z1);
                    const float dz1 = d[r] * dact_f<ACT>(z1);
                    for (int q = 0; q < NIN; ++q) part[q] = fmaf(dz1, xs[q], part[q]);
                    part[NIN] += dz1;
                }
                // sum over the four row groups (lanes c, c+16, c+32, c+48); lane c owns the entry
                for (int q = 0; q <= NIN; ++q) {
                    float v = part[q];
                    v += __shfl_xor(v, 16, 64);
                    v += __shfl_xor(v, 32, 64);
                    if (g == 0) gW1[wave][k][q] += v;
                }
            }
        }
        __syncthreads();  // the next round overwrites h1t / dz2t
    }
    // ---- the block's gradient: every wave's partial of every parameter, added
    // in wave order (the tiles are free after the last round's barrier)
    float* sG = &tiles[0][0][0][0];
    float w3[4], b2[4];
    for (int t = 0; t < 4; ++t) {
        float v = gW3[t], w = gB2[t];
        v += __shfl_xor(v, 16, 64); v += __shfl_xor(v, 32, 64);
        w += __shfl_xor(w, 16, 64); w += __shfl_xor(w, 32, 64);
        w3[t] = v;
        b2[t] = w;
    }
    float b3s = gB3;
    double l = lsum;
    for (int o = 32; o > 0; o >>= 1) {
        b3s += __shfl_xor(b3s, o, 64);
        l += __shfl_xor(l, o, 64);
    }
    // what this lane owns: 64 entries of W2, 9 of W1 | b1, with g == 0 the
    // lane's 4 + 4 of W3 and b2, and lane 0 b3
    constexpr int N1 = NH * (NIN + 1) / 64;
    static_assert(NH * (NIN + 1) % 64 == 0, "W1 | b1 split evenly over the lanes");
    int pos[64 + N1 + 8];
    float val[64 + N1 + 8];
#pragma unroll
    for (int tn = 0; tn < 4; ++tn)
#pragma unroll
        for (int tk = 0; tk < 4; ++tk)
#pragma unroll
            for (int r = 0; r < 4; ++r) {  // D[m = n][nn = k]: row 16tn + 4g + r, column 16tk + c
                pos[16 * tn + 4 * tk + r] = OFF_W2 + (16 * tn + 4 * g + r) * NH + 16 * tk + c;
                val[16 * tn + 4 * tk + r] = accW2[tn][tk][r];
            }
#pragma unroll
    for (int e = 0; e < N1; ++e) {
        const int i = lane + 64 * e, k = i / (NIN + 1), q = i % (NIN + 1);
        pos[64 + e] = q < NIN ? OFF_W1 + k * NIN + q : OFF_B1 + k;
        val[64 + e] = gW1[wave][k][q];
    }
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        pos[64 + N1 + t] = OFF_W3 + 16 * t + c;
        val[64 + N1 + t] = w3[t];
        pos[64 + N1 + 4 + t] = OFF_B2 + 16 * t + c;
        val[64 + N1 + 4 + t] = b2[t];
    }
    constexpr int NA = 64 + N1, NB = NA + 8;  // entries of every lane; of the g == 0 lanes
    for (int w = 0; w < BLOCK / 64; ++w) {
        if (wave == w) {
            if (w > 0) {  // every load before the first store: one wait
                float old[NB], old3 = 0.0f;
#pragma unroll
                for (int e = 0; e < NA; ++e) old[e] = sG[pos[e]];
                if (g == 0)
#pragma unroll
                    for (int e = NA; e < NB; ++e) old[e] = sG[pos[e]];
                if (lane == 0) old3 = sG[OFF_B3];
#pragma unroll
                for (int e = 0; e < NA; ++e) val[e] += old[e];
                if (g == 0)
#pragma unroll
                    for (int e = NA; e < NB; ++e) val[e] += old[e];
                b3s += old3;
            }
#pragma unroll
            for (int e = 0; e < NA; ++e) sG[pos[e]] = val[e];
            if (g == 0)
#pragma unroll
                for (int e = NA; e < NB; ++e) sG[pos[e]] = val[e];
            if (lane == 0) {
                sG[OFF_B3] = b3s;
                sL[w] = l;
            }
        }
        __syncthreads();
    }
    float* row = part + (size_t)blockIdx.x * MLP_PART_STRIDE;
    for (int i = tid; i < NPARAM; i += BLOCK) row[i] = sG[i];
    if (tid == 0) {
        double ls = 0.0;
        for (int w = 0; w < BLOCK / 64; ++w) ls += sL[w];
        lpart[blockIdx.x] = ls;
    }
}

hipError_t launch_mlp_step(const float* P, const MlpStep& s, float* part, double* lpart, int* rows, hipStream_t st)
{
    StepArgs a{s.X, s.t, s.n_data, s.batch, s.draw_seed, s.step};
    int blocks = s.batch / 16 / (BLOCK / 64);
    if (blocks > MLP_PART_ROWS) blocks = MLP_PART_ROWS;
    if (blocks < 1) blocks = 1;
    *rows = blocks;
    if (s.act == PIC_MLP_RELU) hipLaunchKernelGGL(k_mlp_step<PIC_MLP_RELU>, dim3(blocks), dim3(BLOCK), 0, st, P, a, part, lpart);
    else hipLaunchKernelGGL(k_mlp_step<PIC_MLP_SILU>, dim3(blocks), dim3(BLOCK), 0, st, P, a, part, lpart);
    return hipGetLastError();
}

// The summed gradient of parameter i: four lanes per parameter each add every
// fourth row in row order, then two shuffle steps add the four sums.  With
// ADAM, Adam on the FP32 master weights (beta1 0.9, beta2 0.999, eps 1e-8);
// otherwise the sum goes to grad.  Thread 0 also sums the rows' squared errors.
template <bool ADAM>
__global__ __launch_bounds__(BLOCK) void k_mlp_reduce(float* P, const float* part, int rows, const double* lpart,
                                                      double* loss, float* grad, float* m, float* v, float lr, float bc1,
                                                      float bc2)
{
    const int gid = blockIdx.x * BLOCK + threadIdx.x;
    const int i = gid >> 2, j = gid & 3;
    float sum = 0.0f;
    if (i < NPARAM) {
#pragma unroll 4
        for (int r = j; r < rows; r += 4) sum += part[(size_t)r * MLP_PART_STRIDE + i];
    }
    sum += __shfl_xor(sum, 1, 64);
    sum += __shfl_xor(sum, 2, 64);
    if (gid == 0) {
        double ls = 0.0;
        for (int r = 0; r < rows; ++r) ls += lpart[r];
        *loss = ls;
    }
    if (i >= NPARAM || j != 0) return;
    if constexpr (ADAM) {
        const float mi = 0.9f * m[i] + 0.1f * sum;
        const float vi = 0.999f * v[i] + 0.001f * sum * sum;
        m[i] = mi;
        v[i] = vi;
        P[i] -= lr * (mi / bc1) / (sqrtf(vi / bc2) + 1e-8f);
    } else {
        grad[i] = sum;
    }
}

hipError_t launch_mlp_adam(float* P, const float* part, int rows, const double* lpart, double* loss, float* m, float* v,
                           float lr, float bc1, float bc2, hipStream_t st)
{
    if (rows < 1 || rows > MLP_PART_ROWS) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_mlp_reduce<true>, dim3((4 * NPARAM + BLOCK - 1) / BLOCK), dim3(BLOCK), 0, st, P, part, rows,
                       lpart, loss, nullptr, m, v, lr, bc1, bc2);
    return hipGetLastError();
}

hipError_t launch_mlp_grad(const float* part, int rows, const double* lpart, float* grad, double* loss, hipStream_t st)
{
    if (rows < 1 || rows > MLP_PART_ROWS) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_mlp_reduce<false>, dim3((4 * NPARAM + BLOCK - 1) / BLOCK), dim3(BLOCK), 0, st, nullptr, part,
                       rows, lpart, loss, grad, nullptr, nullptr, 0.0f, 1.0f, 1.0f);
    return hipGetLastError();
}

}  // namespace pic
