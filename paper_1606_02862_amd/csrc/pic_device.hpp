// Device-side helpers shared by the kernels: the Philox4x64-10 generator and
// its counter layout, the real-type helpers, and the B-spline assignment
// weights from NGP (order 0) to PCS (order 3).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pic_internal.hpp"

namespace pic {

// Philox4x64-10 (Salmon, Moraes, Dror, Shaw; "Parallel random numbers: as
// easy as 1, 2, 3", SC'11): ten rounds, each two 64x64 -> 128-bit products of
// counter words with fixed multipliers, xor-mixed with a key that advances by
// the Weyl constants between rounds.
struct Philox4 {
    uint64_t v[4];
};

__device__ inline Philox4 philox4x64_10(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3, uint64_t k0, uint64_t k1)
{
    constexpr uint64_t M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
    constexpr uint64_t W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t lo0 = M0 * c0, hi0 = __umul64hi(M0, c0);
        const uint64_t lo1 = M1 * c2, hi1 = __umul64hi(M1, c2);
        const uint64_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
        c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
        k0 += W0; k1 += W1;
    }
    return Philox4{{c0, c1, c2, c3}};
}

// Uniform double in (0,1) from the top 53 bits of a word.
__device__ inline double u01(uint64_t w)
{
    return ((double)(w >> 11) + 0.5) * 0x1.0p-53;
}

// Counter layout: (particle id, species, purpose, step), key (seed, 0).
enum Purpose {
    PURPOSE_POSITION = 0,
    PURPOSE_MOMENTUM = 1,
    PURPOSE_IONIZE = 2,
    PURPOSE_MLP_DATA = 3,   // surrogate training samples
    PURPOSE_MLP_BATCH = 4,  // minibatch draws
    PURPOSE_MLP_INIT = 5,   // initial weights
    PURPOSE_IONIZE_MORE = 6 // ionisation events 4..7 of one step
};

// ---------------------------------------------------------------- real type
// Overloads for the templated PIC kernels (R = float or double).  1/sqrt and
// 1/x are the hardware approximations in FP32 (the push stays within its
// parity bound by a wide margin) and IEEE sqrt and division in FP64.
__host__ __device__ inline float rfloor(float x) { return floorf(x); }
__host__ __device__ inline double rfloor(double x) { return floor(x); }
__host__ __device__ inline float rfma(float a, float b, float c) { return fmaf(a, b, c); }
__host__ __device__ inline double rfma(double a, double b, double c) { return fma(a, b, c); }
__host__ __device__ inline float rabs(float x) { return fabsf(x); }
__host__ __device__ inline double rabs(double x) { return fabs(x); }
__host__ __device__ inline float rmin(float a, float b) { return fminf(a, b); }
__host__ __device__ inline double rmin(double a, double b) { return fmin(a, b); }
__host__ __device__ inline float rmax(float a, float b) { return fmaxf(a, b); }
__host__ __device__ inline double rmax(double a, double b) { return fmax(a, b); }
__device__ inline float rrsq(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ inline double rrsq(double x) { return 1.0 / sqrt(x); }
__device__ inline float rrcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ inline double rrcp(double x) { return 1.0 / x; }
__device__ inline float4 make4(float a, float b, float c, float d) { return make_float4(a, b, c, d); }
__device__ inline double4 make4(double a, double b, double c, double d) { return make_double4(a, b, c, d); }

// ---------------------------------------------------------------- shapes
// NGP (order 0, used by the Galerkin gather): node floor(x + 1/2), weight 1.
// CIC: nodes f, f+1 with f = floor(x); weights 1-d, d (d = x - f).
// TSC: nodes r-1, r, r+1 with r = floor(x + 1/2); d = x - r in [-1/2, 1/2):
//      1/2 (1/2 - d)^2, 3/4 - d^2, 1/2 (1/2 + d)^2.
// PCS (cubic B-spline): nodes f-1 .. f+2 with f = floor(x), d = x - f, e = 1 - d:
//      e^3/6, 2/3 - d^2 (1 - d/2), 2/3 - e^2 (1 - e/2), d^3/6.
template <int ORDER, class R>
__host__ __device__ inline int shape_weights(R x, R* w)
{
    static_assert(ORDER >= 0 && ORDER <= 3, "NGP, CIC, TSC or PCS");
    if constexpr (ORDER == 0) {
        const R f = rfloor(x + R(0.5));  // nearest node, the upper one on a tie
        w[0] = R(1);
        return (int)f;
    } else if constexpr (ORDER == 1) {
        const R f = rfloor(x);
        const R d = x - f;
        w[0] = R(1) - d;
        w[1] = d;
        return (int)f;
    } else if constexpr (ORDER == 2) {
        const R r = rfloor(x + R(0.5));
        const R d = x - r;
        const R a = R(0.5) - d, b = R(0.5) + d;
        w[0] = R(0.5) * a * a;
        w[1] = R(0.75) - d * d;
        w[2] = R(0.5) * b * b;
        return (int)r - 1;
    } else {
        const R f = rfloor(x);
        const R d = x - f, e = R(1) - d;
        const R sixth = R(1) / R(6), two3 = R(2) / R(3);
        w[0] = sixth * e * e * e;
        w[1] = two3 - d * d * (R(1) - R(0.5) * d);
        w[2] = two3 - e * e * (R(1) - R(0.5) * e);
        w[3] = sixth * d * d * d;
        return (int)f - 1;
    }
}

}  // namespace pic
