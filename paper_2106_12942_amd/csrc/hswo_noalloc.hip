// hswo_noalloc.hip -- rhseg_segment_noalloc: RHSEG whose scratch is the
// library's own static device array instead of a caller workspace, for
// callers that cannot allocate device memory (code under stream capture,
// serving loops that must not allocate).
//
// The array is `scratch` below: HSWO_NOALLOC_SCRATCH_BYTES, 256-byte aligned,
// one copy per GPU, held from the library's load on that GPU until the
// process ends. Host code never passes the array's name to a kernel or a
// copy: on the host that name is only a stand-in, so the device address of
// each GPU's copy is looked up once per device (hipGetSymbolAddress, with that
// device current, at the first call on it) and kept in g_scratch.
//
// Every call on one GPU reuses that GPU's array and leaves its last contents
// there. The kernels clear everything they read before writing it (counters
// and seam hash tables by fill kernels, region state by the initialisation
// kernels), so no call depends on what an earlier one left. Two calls that
// overlap on one GPU (two host threads, or two streams) race on the array.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <mutex>

#include "hswo.h"
#include "hswo_internal.h"

static __device__ __align__(256) unsigned char scratch[HSWO_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int MAX_DEVICES = 64;
std::mutex g_mu;
void* g_scratch[MAX_DEVICES] = {};  // device address of each GPU's copy (null: not looked up yet)

// The current device's copy of the array, looked up on the first call on
// that device.
int scratch_on_current_device(void** out) {
    char msg[256];
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) {
        snprintf(msg, sizeof(msg), "hipGetDevice: %s", hipGetErrorString(e));
        return hswo::set_error(HSWO_E_DEVICE, msg);
    }
    if (dev < 0 || dev >= MAX_DEVICES) {
        snprintf(msg, sizeof(msg), "device %d: rhseg_segment_noalloc serves devices 0..%d", dev, MAX_DEVICES - 1);
        return hswo::set_error(HSWO_E_UNSUPPORTED, msg);
    }
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_scratch[dev]) {
        void* ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || ptr == nullptr) {
            snprintf(msg, sizeof(msg), "hipGetSymbolAddress(scratch) on device %d: %s", dev,
                     e != hipSuccess ? hipGetErrorString(e) : "null address");
            return hswo::set_error(HSWO_E_DEVICE, msg);
        }
        if (reinterpret_cast<uintptr_t>(ptr) % 256) {
            snprintf(msg, sizeof(msg), "scratch on device %d is not 256-byte aligned", dev);
            return hswo::set_error(HSWO_E_DEVICE, msg);
        }
        g_scratch[dev] = ptr;
    }
    *out = g_scratch[dev];
    return HSWO_OK;
}

}  // namespace

extern "C" int rhseg_segment_noalloc(const void* cube, int32_t H, int32_t W, int32_t B, int32_t dtype,
                                     const hswo_params* p, int32_t rnb_levels, int32_t* labels,
                                     hswo_merge_rec* merge_log, hswo_stats* stats, void* hip_stream) {
    hswo::clear_error();
    if (rnb_levels < 1 || rnb_levels > 16) return hswo::set_error(HSWO_E_INVAL, "rnb_levels must be in [1,16]");
    return hswo::rhseg_in_scratch(cube, H, W, B, dtype, p, rnb_levels, labels, merge_log, stats,
                                  scratch_on_current_device, (size_t)HSWO_NOALLOC_SCRATCH_BYTES,
                                  reinterpret_cast<hipStream_t>(hip_stream));
}
