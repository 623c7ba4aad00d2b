// The fixed device scratch of hough_hier_detect_noalloc: one array per
// device, part of the library's code object, so a call that must not
// allocate device memory (code under HIP graph capture, tight serving loops,
// harnesses that forbid allocation) carves everything it needs from it.
// Every call on a device shares that device's array and leaves its contents
// behind; calls that overlap on one device race.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "hh_engine.hpp"

static __device__ __align__(256) char scratch[256ll << 20];

namespace hh {

const int64_t kNoAllocScratchBytes = 256ll << 20;

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_addr[kMaxDevices] = {};
}  // namespace

// The name `scratch` in host code is a host-side stand-in; kernels must be
// given the device address hipGetSymbolAddress reports for the current
// device, which this keeps per device.
void* noalloc_scratch(int device)
{
    if (device < 0 || device >= kMaxDevices) throw Error{HH_EDEVICE, "device ordinal out of range"};
    std::lock_guard<std::mutex> g(g_mu);
    if (!g_addr[device]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            throw Error{HH_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e)};
        }
        g_addr[device] = p;
    }
    return g_addr[device];
}

}  // namespace hh
