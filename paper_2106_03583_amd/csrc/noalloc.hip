// Entry points that allocate nothing, for callers that cannot allocate
// device memory (code under HIP graph capture, tight serving loops,
// harnesses that forbid allocation).  Their scratch is a file-scope device
// array: every GPU the library runs on holds its own copy until the process
// ends.  Host code never passes the array's name to a kernel (on the host it
// is only a stand-in for the symbol); it passes the device address that
// hipGetSymbolAddress returns, looked up once per device.
#include <mutex>

#include "internal.h"

namespace {

constexpr size_t kScratchDoubles = size_t(1) << 20;  // 8 MiB per device

__device__ __align__(256) double scratch[kScratchDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
double* g_ptr[kMaxDevices] = {};

// Device address of this device's scratch array (looked up on first use).
int scratch_address(int dev, double** out) {
    if (dev < 0 || dev >= kMaxDevices) return MBP_ERR_INVALID;
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_ptr[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
            (void)hipGetLastError();
            return MBP_ERR_HIP;
        }
        g_ptr[dev] = static_cast<double*>(p);
    }
    *out = g_ptr[dev];
    return MBP_OK;
}

}  // namespace

extern "C" {

size_t mbp_noalloc_scratch_bytes(void) { return kScratchDoubles * sizeof(double); }

int mbp_residual_norm_noalloc(const mbp_plan* plan, const double* rhs_dev, const double* p_dev, double rhs_shift,
                              double* out_dev, void* stream) {
    if (!plan || !rhs_dev || !p_dev || !out_dev) return MBP_ERR_INVALID;
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return MBP_ERR_HIP;
    if (dev != plan->device) return MBP_ERR_INVALID;
    if (mbp::resnorm_scratch_doubles(plan) > kScratchDoubles) return MBP_ERR_TOO_LARGE;
    double* part = nullptr;
    const int st = scratch_address(dev, &part);
    if (st != MBP_OK) return st;
    mbp::launch_resnorm3d(plan, rhs_dev, p_dev, rhs_shift, part, out_dev, static_cast<hipStream_t>(stream));
    return hipGetLastError() == hipSuccess ? MBP_OK : MBP_ERR_HIP;
}

}  // extern "C"
