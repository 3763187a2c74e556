// Training-pixel selection with no allocation: nvc_select_pixels with its
// workspace in a static device buffer of the library, for callers that
// cannot allocate device memory.
//
// `scratch` is a device symbol: in host code its name is not a device
// address.  Its address on the current device is looked up once per device
// with hipGetSymbolAddress (every GPU holds its own copy of the array at its
// own address) and only that pointer is handed to the kernels.  Every call
// on a GPU shares that GPU's array; the pixel counts that must start at zero
// are cleared by a fill kernel at the start of every call (no memset), and
// the other parts are fully written before they are read.  Calls that
// overlap on one GPU (on two streams) race on the array.
#include <mutex>

#include <hip/hip_runtime.h>

#include "nvc_internal.hpp"

namespace nvc {

// Largest image: 2^23 pixels (3840 x 2160 fits).  Workspace of the pixel
// counting sort: counts and offsets (4 B each per pixel), one sum per 4096
// pixels, and 512 bytes of slack: 64 MiB + 8.5 KiB.
constexpr int64_t kNoallocMaxPix = (int64_t)1 << 23;
constexpr int64_t kNoallocScratchBytes = (2 * kNoallocMaxPix + kNoallocMaxPix / 4096) * 4 + 512;

static __device__ __align__(256) unsigned char scratch[kNoallocScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// The current device's address of `scratch`, looked up on the first call on that device.
hipError_t scratch_address(void** out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}
}  // namespace

int64_t select_pixels_noalloc_max_pixels() { return kNoallocMaxPix; }

hipError_t launch_select_pixels_noalloc(uint64_t seed, uint32_t frame, const uint32_t* frame_dev, int64_t n_pix,
                                        int64_t batch, int32_t* pix, hipStream_t st) {
    if (n_pix > kNoallocMaxPix || select_pixels_workspace_bytes(n_pix) > kNoallocScratchBytes)
        return hipErrorInvalidValue;                      // rejected on the host before this point
    void* ptr = nullptr;
    const hipError_t e = scratch_address(&ptr);
    if (e != hipSuccess) return e;
    return launch_select_pixels(seed, frame, frame_dev, n_pix, batch, pix, ptr, st);
}

}  // namespace nvc
