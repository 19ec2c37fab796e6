// Rate evaluation that allocates nothing: the staging buffers of
// pic_rate_eval live in one file-scope device array per GPU instead of
// memory from the handle's allocator.
//
// The array's name is a host-side stand-in in host code; the device address
// of each GPU's copy comes from hipGetSymbolAddress, taken once per device
// (at pic_init, with that device current) and kept per device.
// Only that address is ever handed to kernels or copies.  Nothing in the
// array needs to start at zero: a call copies its inputs in before the rate
// kernel reads them, and the kernel writes every output that is copied back.
// Every call on a GPU shares that GPU's array, so calls that overlap on one
// GPU race.
#include <hip/hip_runtime.h>

#include <mutex>

#include "ionize_internal.hpp"

namespace pic {

// Staging of one pic_rate_eval_noalloc call: kT, n_e and ln nu (doubles) and
// Z (int32) for up to PIC_RATE_EVAL_NOALLOC_MAX samples, at fixed offsets.
constexpr size_t NOALLOC_BYTES = (size_t)PIC_RATE_EVAL_NOALLOC_MAX * (3 * sizeof(double) + sizeof(int32_t));
static __device__ __align__(256) unsigned char scratch[NOALLOC_BYTES];

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch[MAX_DEVICES] = {};
}  // namespace

hipError_t noalloc_scratch_setup(int device)
{
    if (device < 0 || device >= MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch[device]) return hipSuccess;
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch[device] = p;
    return hipSuccess;
}

unsigned char* noalloc_scratch(int device)
{
    if (device < 0 || device >= MAX_DEVICES) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    return static_cast<unsigned char*>(g_scratch[device]);
}

NoallocStaging noalloc_staging(unsigned char* base)
{
    constexpr size_t M = PIC_RATE_EVAL_NOALLOC_MAX;
    NoallocStaging s{};
    s.kT = reinterpret_cast<double*>(base);
    s.ne = reinterpret_cast<double*>(base + M * sizeof(double));
    s.out = reinterpret_cast<double*>(base + 2 * M * sizeof(double));
    s.Z = reinterpret_cast<int32_t*>(base + 3 * M * sizeof(double));
    return s;
}

}  // namespace pic
