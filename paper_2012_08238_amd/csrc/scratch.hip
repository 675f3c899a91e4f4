// Execution without any allocation: the workspace of sfft_execute_noalloc lives in
// one file-scope device array per GPU instead of the plan's own workspace.
//
// The array's name is a host-side stand-in in host code; its device address is taken
// once per device with hipGetSymbolAddress (scratch_address, called by plan creation
// with that device current) and only that address is used afterwards: in the scratch
// descriptors that plan creation uploads, through which the kernels reach it exactly as
// they reach a plan's workspace. Every call on one GPU shares the array and leaves its
// contents behind; the kernels clear what must start at zero (the candidate counter,
// at the start of the bucketization) and write everything else before reading it.
// Calls that overlap on one GPU race on the array.
#include <mutex>

#include "common.hpp"
#include "internal.hpp"

namespace {
constexpr size_t kScratchBytes = size_t(64) << 20;   // 64 MiB per GPU, held until the process ends
constexpr int kMaxDevices = 64;
}  // namespace

static __device__ __align__(256) char scratch[kScratchBytes];

namespace {

std::mutex g_scratch_mu;
char* g_scratch_ptr[kMaxDevices] = {};
hipError_t g_scratch_err[kMaxDevices] = {};
bool g_scratch_done[kMaxDevices] = {};

}  // namespace

namespace sfft {

size_t scratch_bytes() { return kScratchBytes; }

hipError_t scratch_address(int device, char** out) {
    *out = nullptr;
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_done[device]) {
        int cur = -1;
        hipError_t e = hipGetDevice(&cur);
        if (e == hipSuccess && cur != device) e = hipErrorInvalidDevice;   // the caller makes `device` current
        void* p = nullptr;
        if (e == hipSuccess) e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        g_scratch_err[device] = e;
        g_scratch_ptr[device] = e == hipSuccess ? static_cast<char*>(p) : nullptr;
        g_scratch_done[device] = true;
    }
    *out = g_scratch_ptr[device];
    return g_scratch_err[device];
}

}  // namespace sfft

extern "C" sfft_status sfft_execute_noalloc(sfft_plan_t p, const void* x_dev, int64_t* out_idx, void* out_val,
                                            double* out_resid, sfft_stream_t stream) {
    return sfft::plan_execute(p, x_dev, out_idx, out_val, out_resid, stream, /*scratch=*/true);
}
