// dk_noalloc.hip -- the allocation-free variant of dk_mlmc_level_pair.
//
// Its device workspace (level tables, the centring run, per-sample values of one chunk, chunk
// moments) is a file-scope device array of fixed size that every GPU the library runs on holds
// for the life of the process.  In host code the array's name is only a stand-in for the symbol:
// its device address is obtained once per device with hipGetSymbolAddress, with that device
// current, and that address alone is handed to the kernels.
#include <hip/hip_runtime.h>

#include <mutex>

#include "dk_internal.h"

namespace {

constexpr size_t kScratchBytes = size_t(32) << 20;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device (looked up on the first call per device).
int scratch_address(void** out)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return dk::set_error(DK_EDEVICE, hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices) return dk::set_error(DK_EUNSUPPORTED, "device index beyond 63");
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) return dk::set_error(DK_EDEVICE, "hipGetSymbolAddress(scratch) failed");
        g_ptr[dev] = p;
    }
    *out = g_ptr[dev];
    return DK_OK;
}

}  // namespace

extern "C" int dk_mlmc_level_pair_noalloc(const dk_problem* problem, int32_t level, uint64_t first_sample,
                                          uint64_t n_samples, uint32_t stream_tag, dk_moments* sums_out,
                                          double* per_sample_out, void* stream)
{
    void* arena = nullptr;
    const int rc = scratch_address(&arena);
    if (rc) return rc;
    return dk::level_pair_arena(problem, level, first_sample, n_samples, stream_tag, sums_out, per_sample_out, arena,
                                kScratchBytes, (hipStream_t)stream);
}
