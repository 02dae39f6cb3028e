// noalloc.hip -- step 3 of Alg. 1 on a static device work array, for callers
// that cannot allocate device memory (code under HIP graph capture, tight
// serving loops, harnesses that forbid hipMalloc).
//
// hamls_grid_to_coeffs keeps its step-3 work memory (ring spectra, axis-pass
// buffers, folded FP32 spectra) in the plan and grows it with the largest F it
// has seen, which allocates.  hamls_grid_to_coeffs_noalloc runs the same
// kernels with that work memory carved from `scratch`, a file-scope device
// array of kScratchBytes that every GPU the library runs on holds until the
// process ends.  Its device address is looked up once per device with
// hipGetSymbolAddress (the array's name is only a host-side stand-in) and
// kept; kernels receive that address.  Every call on one GPU shares the
// array, so calls that overlap on one GPU (two streams, two threads) race.
// The kernels write every work element they read, so nothing is cleared.
#include <mutex>

#include "common.h"

namespace hamls {
namespace {

constexpr size_t kScratchBytes = (size_t)128 << 20;  // 128 MiB
constexpr int kMaxDevices = 64;

__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
unsigned char* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device (looked up once).
hamls_status scratch_address(int device, unsigned char** out) {
    if (device < 0 || device >= kMaxDevices) {
        set_error("device %d outside [0, %d)", device, kMaxDevices);
        return HAMLS_ERR_UNSUPPORTED;
    }
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void* p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_status(e, "hipGetSymbolAddress(scratch)");
        if (!p) {
            set_error("hipGetSymbolAddress(scratch) returned a null address");
            return HAMLS_ERR_DEVICE;
        }
        g_scratch_ptr[device] = (unsigned char*)p;
    }
    *out = g_scratch_ptr[device];
    return HAMLS_OK;
}

size_t round256(size_t b) { return (b + 255) & ~(size_t)255; }

}  // namespace
}  // namespace hamls

using namespace hamls;

extern "C" {

size_t hamls_noalloc_scratch_bytes(void) { return kScratchBytes; }

hamls_status hamls_grid_to_coeffs_noalloc(hamls_plan_t plan, const double* grid_values, int32_t F,
                                          double* coeffs, void* stream) {
    Plan* P = (Plan*)plan;
    if (!P || !grid_values || !coeffs) {
        set_error("null argument");
        return HAMLS_ERR_INVALID_ARG;
    }
    if (F < 1 || F > 4096) {
        set_error("F outside [1, 4096]");
        return HAMLS_ERR_INVALID_ARG;
    }
    const CoeffWorkSize z = coeff_work_size(*P, F);
    const size_t b0 = round256(sizeof(double) * (size_t)z.d0);
    const size_t b1 = round256(sizeof(double) * (size_t)z.d1);
    const size_t b2 = round256(sizeof(float) * (size_t)z.f0);
    if (b0 + b1 + b2 > kScratchBytes) {
        set_error("step-3 work of %d fields needs %zu bytes, above the %zu-byte static work array "
                  "(call with fewer fields)",
                  F, b0 + b1 + b2, kScratchBytes);
        return HAMLS_ERR_INVALID_ARG;
    }
    int dev = -1;
    HAMLS_HIP(hipGetDevice(&dev));
    if (dev != P->device) {
        set_error("the current device %d is not the plan's device %d", dev, P->device);
        return HAMLS_ERR_INVALID_ARG;
    }
    unsigned char* base = nullptr;
    const hamls_status st = scratch_address(dev, &base);
    if (st != HAMLS_OK) return st;
    CoeffWork W;
    W.d0 = z.d0 > 0 ? (double*)base : nullptr;
    W.d0_len = z.d0;
    W.d1 = z.d1 > 0 ? (double*)(base + b0) : nullptr;
    W.f0 = z.f0 > 0 ? (float*)(base + b0 + b1) : nullptr;
    W.f0_len = z.f0;
    return run_grid_to_coeffs(P, grid_values, F, coeffs, W, (hipStream_t)stream, false);
}

}  // extern "C"
