// Measurement probes for the benchmark's rooflines (not part of the PIC
// library's ABI): the LDS bandwidth of the device, measured with
// conflict-free wave64 LDS reads and 64-bit LDS atomics, and a copy kernel
// with one dword per lane per access, whose bytes are known exactly, to
// calibrate the HBM traffic counters for the particle kernel's dword streams.
#include <hip/hip_runtime.h>

#include <stddef.h>
#include <stdint.h>

namespace {

constexpr int NT = 256;
constexpr int WORDS = 8192;  // 32 KB of LDS per workgroup
constexpr int NA = 16;       // LDS accesses per lane per iteration

// OP 0: ds_read_b64, OP 1: ds_add_u64; lane l of wave w touches
// consecutive 8-byte words, so every wave instruction is conflict-free.
template <int OP>
__global__ __launch_bounds__(NT) void k_lds(int iters, unsigned* sink)
{
    __shared__ __align__(16) unsigned long long buf[WORDS / 2];
    for (int i = threadIdx.x; i < WORDS / 2; i += NT) buf[i] = i;
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    unsigned a[NA];
#pragma unroll
    for (int k = 0; k < NA; ++k) a[k] = (unsigned)(((wave * NA + k) * 64) % (WORDS / 2 - 64) + lane);
    unsigned long long acc = 0;
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int k = 0; k < NA; ++k) {
            if constexpr (OP == 0) acc += buf[a[k]];
            else atomicAdd(&buf[a[k]], 1ull);
        }
        __builtin_amdgcn_s_waitcnt(0xc07f);  // lgkmcnt(0): the iteration's LDS accesses are done
    }
    __syncthreads();
    if (acc == 0x5eedull || buf[threadIdx.x] == 0x5eedull) sink[0] = (unsigned)acc;
}

__global__ __launch_bounds__(NT) void k_copy_dword(const float* __restrict__ src, float* __restrict__ dst, size_t n)
{
    for (size_t i = (size_t)blockIdx.x * NT + threadIdx.x; i < n; i += (size_t)gridDim.x * NT) dst[i] = src[i];
}

}  // namespace

extern "C" {

// LDS bytes per second of the whole device for op 0 (ds_read_b64) or 1
// (ds_add_u64), conflict-free, 4 workgroups per CU; 0 on error.
double probe_lds_bandwidth(int op, int iters)
{
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return 0.0;
    unsigned* sink = nullptr;
    if (hipMalloc(&sink, 256) != hipSuccess) return 0.0;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) { (void)hipFree(sink); return 0.0; }
    const dim3 grid(4 * cus), block(NT);
    double best = 0.0;
    for (int rep = 0; rep < 3; ++rep) {
        (void)hipEventRecord(e0, 0);
        if (op == 0) hipLaunchKernelGGL(k_lds<0>, grid, block, 0, 0, iters, sink);
        else hipLaunchKernelGGL(k_lds<1>, grid, block, 0, 0, iters, sink);
        (void)hipEventRecord(e1, 0);
        float ms = 0.0f;
        if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess || ms <= 0.0f) break;
        const double bytes = (double)grid.x * NT * iters * NA * 8.0;
        if (rep > 0 && bytes / (ms * 1e-3) > best) best = bytes / (ms * 1e-3);  // rep 0 warms up
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipFree(sink);
    return best;
}

// dst[i] = src[i] for n floats (device pointers), one dword per lane per
// access, `reps` times on the null stream; returns 0 on success.
int probe_copy_dword(const float* src, float* dst, size_t n, int reps)
{
    for (int r = 0; r < reps; ++r) hipLaunchKernelGGL(k_copy_dword, dim3(4096), dim3(NT), 0, 0, src, dst, n);
    return hipDeviceSynchronize() == hipSuccess ? 0 : 1;
}

}  // extern "C"
