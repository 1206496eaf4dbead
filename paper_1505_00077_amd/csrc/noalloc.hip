// bf_gp_forward_noalloc: the GP forward with its workspace in a static device
// array instead of a caller-provided buffer, for callers that cannot allocate
// device memory (code under stream capture, tight serving loops, harnesses
// that forbid hipMalloc).
//
// The array `scratch` below is a device-side object: in host code its name is
// only a stand-in and must never be passed to a kernel or a copy.  Its device
// address is looked up once per device with hipGetSymbolAddress (with that
// device current) and kept in g_scratch_ptr; only that address is handed to
// the kernels.  Each device holds its own copy of the array until the process
// ends.  Calls on one device share it, so two calls that overlap on one device
// (different streams, no ordering) race on it.
#include <stdio.h>

#include <mutex>

#include "../../include/bfgp.h"
#include "launch.hpp"

namespace bfgp {
int gp_forward_check(const float *img, const float *out, int H, int W, int pitch, double sigma_s, double sigma_r,
                     int N, unsigned flags, const void *saved, size_t *ws_need);
int set_error(int code, const char *msg);
}  // namespace bfgp

namespace {

constexpr size_t kScratchBytes = (size_t)BF_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;

std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices];  // device address of `scratch` per device, once looked up

}  // namespace

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

// Device address of this device's copy of `scratch` (the current device).
int scratch_for_current_device(void **ptr) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return bfgp::set_error(BF_EHIP, hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices) return bfgp::set_error(BF_EUNSUPPORTED, "device ordinal beyond 63");
    std::lock_guard<std::mutex> g(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) return bfgp::set_error(BF_EHIP, "hipGetSymbolAddress(scratch) failed");
        g_scratch_ptr[dev] = p;
    }
    *ptr = g_scratch_ptr[dev];
    return BF_OK;
}

}  // namespace

extern "C" {

int bf_gp_forward_noalloc(const float *img, float *out, int H, int W, int pitch, double sigma_s, double sigma_r,
                          int N, unsigned flags, void *saved, void *stream) {
    // every argument is checked on the host before any HIP call
    size_t need = 0;
    int rc = bfgp::gp_forward_check(img, out, H, W, pitch, sigma_s, sigma_r, N, flags, saved, &need);
    if (rc) return rc;
    if (need > kScratchBytes) {
        char msg[160];
        snprintf(msg, sizeof msg, "needs %zu bytes of workspace; the static scratch holds %zu", need, kScratchBytes);
        return bfgp::set_error(BF_ENOMEM, msg);
    }
    void *ptr = nullptr;
    if ((rc = scratch_for_current_device(&ptr))) return rc;
    // the same kernels as bf_gp_forward, on the device copy of the array; the
    // forward writes every word of its workspace before reading it (the
    // statistics partials, the status word and the stack pad included), so
    // nothing left by an earlier call needs clearing
    return bf_gp_forward(img, out, H, W, pitch, sigma_s, sigma_r, N, flags, saved, ptr, kScratchBytes, stream);
}

}  // extern "C"
