// kmc_score_replay_noalloc (declared in include/kmc.h): the score replay with
// its own buffers in a static device array instead of the context's
// workspace, for callers that cannot allocate device memory at the point of
// the call.
//
// `scratch` is a file-scope device array of kNoAllocScratchBytes.  In host
// code its name is only a host-side handle, never a device address: the
// array's address on a device is looked up once per device, with that device
// current, by hipGetSymbolAddress, and only that address is handed to the
// kernels.  Every call on one GPU uses the same array, which keeps the last
// call's contents; the replay clears what must start at zero (its hop
// counters) with a kernel.  Calls that overlap on one GPU (other streams,
// other threads) race on the array.
#include "../../include/kmc.h"

#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "kmc_internal.h"

struct kmc_ctx;

namespace kmc {
kmc_status record_error(kmc_status s, const std::string &msg);
size_t replay_region_bytes(const kmc_ctx *c);
kmc_status score_replay_in_region(kmc_ctx *c, const int8_t *occ0_dev, int64_t step0, int64_t n_steps,
                                  const double *weight_dev, double *grad_dev, unsigned char *region,
                                  size_t region_bytes);
}  // namespace kmc

namespace {

constexpr size_t kNoAllocScratchBytes = (size_t)64 << 20;  // 64 MiB per GPU
constexpr int kMaxGpus = 64;

static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

std::mutex g_lock;
unsigned char *g_scratch_ptr[kMaxGpus] = {};

// The device address of `scratch` on the current device (looked up on the
// first call on that device).
kmc_status scratch_on_current_device(unsigned char **out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return kmc::record_error(KMC_EHIP, std::string("hipGetDevice: ") + hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxGpus) return kmc::record_error(KMC_EUNSUPPORTED, "device index beyond 63");
    std::lock_guard<std::mutex> guard(g_lock);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return kmc::record_error(KMC_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch_ptr[dev] = static_cast<unsigned char *>(p);
    }
    *out = g_scratch_ptr[dev];
    return KMC_OK;
}

}  // namespace

extern "C" kmc_status kmc_score_replay_noalloc(kmc_ctx *ctx, const int8_t *occ0_dev, int64_t step0, int64_t n_steps,
                                               const double *weight_dev, double *grad_dev) {
    if (!ctx) return kmc::record_error(KMC_EINVAL, "context is NULL");
    unsigned char *region = nullptr;
    kmc_status s = scratch_on_current_device(&region);
    if (s != KMC_OK) return s;
    return kmc::score_replay_in_region(ctx, occ0_dev, step0, n_steps, weight_dev, grad_dev, region,
                                       kNoAllocScratchBytes);
}
