// purify_phi_noalloc: y = Phi x with its intermediates in a file-scope device array.
//
// purify_phi keeps the row-transformed image (n x K) and the oversampled grid (K x K)
// between its three launches in the plan's workspace.  This variant keeps them in `scratch`,
// a fixed array in the library's own device memory, so the call allocates nothing and
// touches no workspace buffer.  The array is one per device, loaded with the library's code
// object and held until the process ends; every call on a device shares it, so calls that
// overlap on one device race with each other (and the array keeps the last call's
// contents: each call overwrites both regions before reading them).
#include <mutex>

#include "common.h"

namespace purify {
namespace {

constexpr size_t SCRATCH_BYTES = (size_t)48 << 20;   // 48 MiB: n <= 1024 in FP32, n <= 512 in FP64
constexpr int SCRATCH_MAX_DEVICES = 64;

static __device__ __align__(256) unsigned char scratch[SCRATCH_BYTES];

std::mutex g_scratch_mu;
void* g_scratch_ptr[SCRATCH_MAX_DEVICES] = {};   // device address of `scratch`, per device

size_t round256(size_t b) { return (b + 255) / 256 * 256; }

// Device address of the current device's copy of `scratch` (looked up once per device, with
// that device current).
purify_status scratch_address(void** out) {
    int dev = -1;
    PURIFY_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= SCRATCH_MAX_DEVICES) {
        set_error("purify_phi_noalloc: device index beyond the library's table");
        return PURIFY_E_DEVICE;
    }
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        PURIFY_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) {
            set_error("purify_phi_noalloc: no device address for the scratch array");
            return PURIFY_E_DEVICE;
        }
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return PURIFY_OK;
}

template <typename T>
void phi_into(const Plan& P, const cpx<T>* x, cpx<T>* y, char* base, hipStream_t s) {
    cpx<T>* tmp = (cpx<T>*)base;
    cpx<T>* grid = (cpx<T>*)(base + round256((size_t)P.n * P.K * sizeof(cpx<T>)));
    launch_fft_rows_fwd<T>(P, x, tmp, s);
    launch_fft_cols_fwd<T>(P, (const cpx<T>*)tmp, grid, s);
    launch_degrid<T>(P, (const cpx<T>*)grid, y, P.perm, 1.0, s);
}

}  // namespace
}  // namespace purify

using namespace purify;

extern "C" purify_status purify_phi_noalloc(const purify_plan* plan, const void* x, void* y, void* stream) {
    if (!plan || !x || !y) {
        set_error("purify_phi_noalloc: null plan or vector");
        return PURIFY_E_INVALID;
    }
    const Plan& P = plan->P;
    const size_t need = round256((size_t)P.n * P.K * P.elem) + (size_t)P.K * P.K * P.elem;
    if (need > SCRATCH_BYTES) {
        set_error("purify_phi_noalloc: the plan needs " + std::to_string(need) + " bytes of scratch, more than the " +
                  std::to_string(SCRATCH_BYTES) + " the library holds (n <= 1024 in FP32, n <= 512 in FP64)");
        return PURIFY_E_INVALID;
    }
    void* base = nullptr;
    const purify_status st = scratch_address(&base);
    if (st != PURIFY_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    if (P.precision == PURIFY_FP64)
        phi_into<double>(P, (const cpx<double>*)x, (cpx<double>*)y, (char*)base, s);
    else
        phi_into<float>(P, (const cpx<float>*)x, (cpx<float>*)y, (char*)base, s);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        set_error(std::string("purify_phi_noalloc: kernel launch: ") + hipGetErrorString(e));
        return PURIFY_E_DEVICE;
    }
    return PURIFY_OK;
}
