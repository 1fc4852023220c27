// Allocation-free product: arrow_spmm with its workspace in a fixed device
// array of this library instead of caller memory (for callers that cannot
// allocate: graph capture, serving loops, harnesses that forbid it).
//
// The array lives once per GPU for the life of the process.  Host code never
// passes its name to a kernel (in host code the name is a host-side stand-in,
// not a device address): the device address is looked up once per device with
// hipGetSymbolAddress, with that device current, and only that pointer is used.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "arrow.h"
#include "internal.h"

namespace arrow {
namespace {

static __device__ __align__(256) unsigned char scratch[ARROW_STATIC_WORKSPACE_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_ptr[kMaxDevices] = {};

// Device address of `scratch` on `device` (looked up once per device).
arrow_status_t scratch_ptr(int device, void **out) {
    *out = nullptr;
    if (device < 0 || device >= kMaxDevices) {
        set_error("device index out of range for the static workspace");
        return ARROW_ERR_INVALID_ARG;
    }
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_ptr[device]) {
        int prev = -1;
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        hipError_t e = hipSetDevice(device);
        void *ptr = nullptr;
        if (e == hipSuccess) e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (prev >= 0 && prev != device) hipSetDevice(prev);
        if (e != hipSuccess || !ptr) {
            set_error(std::string("hipGetSymbolAddress of the static workspace: ") +
                      hipGetErrorString(e));
            return ARROW_ERR_HIP;
        }
        g_ptr[device] = ptr;
    }
    *out = g_ptr[device];
    return ARROW_OK;
}

}  // namespace
}  // namespace arrow

extern "C" arrow_status_t arrow_spmm_static(arrow_plan_t p, const arrow_operand_t *ops,
                                            int32_t num_ops, void *stream) {
    if (!p || (num_ops > 0 && !ops) || num_ops < 0) {
        arrow::set_error("NULL plan or operands");
        return ARROW_ERR_INVALID_ARG;
    }
    size_t need = 0;
    for (int32_t i = 0; i < num_ops; ++i) {
        size_t b = 0;
        if (arrow_status_t st = arrow_workspace_size(p, ops[i].k, ops[i].dtype, &b)) return st;
        need += b;
    }
    if (need > (size_t)ARROW_STATIC_WORKSPACE_BYTES) {
        arrow::set_error("the products need " + std::to_string(need) +
                         " workspace bytes, more than the static workspace holds (" +
                         std::to_string((size_t)ARROW_STATIC_WORKSPACE_BYTES) +
                         "); use arrow_spmm with a caller workspace");
        return ARROW_ERR_UNSUPPORTED;
    }
    void *ws = nullptr;
    if (arrow_status_t st = arrow::scratch_ptr(arrow::plan_device(p), &ws)) return st;
    return arrow_spmm(p, ops, num_ops, ws, (size_t)ARROW_STATIC_WORKSPACE_BYTES, stream);
}
