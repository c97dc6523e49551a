// Allocation-free variant of the resistance-gradient contraction, for callers
// that cannot allocate (code under HIP graph capture, tight serving loops):
// its scratch -- the two per-outlet dot products -- lives in a file-scope
// device array instead of the context's workspace, and its output goes to a
// caller-owned device buffer, so a call enqueues three kernels and nothing
// else (no allocation, no copy, no synchronisation).
#include <hip/hip_runtime.h>

#include <mutex>

#include "kernels.h"

namespace {

constexpr int kMaxDevices = 64;

// scratch[0 .. n_out): a^k . lambda_v; scratch[kNoAllocMaxOutlets .. + n_out): a^k . x_v
__device__ __align__(256) double scratch[2 * ns::kNoAllocMaxOutlets];

std::mutex g_mu;
double* g_scratch[kMaxDevices] = {};  // device address of `scratch` on each device

}  // namespace

namespace ns {

// Device address of this file's scratch array on `device` (the current
// device); looked up once per device with that device current.
hipError_t noalloc_scratch(int device, double** out) {
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_scratch[device]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch[device] = static_cast<double*>(p);
    }
    *out = g_scratch[device];
    return hipSuccess;
}

}  // namespace ns

extern "C" ns_status ns_resistance_gradient_noalloc(ns_ctx* c, const double* d_lambda, const double* d_x,
                                                    double* d_grad, hipStream_t st) {
    if (!c) return NS_ERR_ARG;
    if (!c->bound) {
        c->err = "context not bound";
        return NS_ERR_STATE;
    }
    if (!c->assembled || !c->resistance_mode) {
        c->err = "the last assembly did not take resistance outlets";
        return NS_ERR_STATE;
    }
    const int NO = c->sym.n_out;
    if (NO == 0) return NS_OK;
    if (NO > ns::kNoAllocMaxOutlets) {
        c->err = "ns_resistance_gradient_noalloc supports at most " + std::to_string(ns::kNoAllocMaxOutlets) +
                 " outlets";
        return NS_ERR_ARG;
    }
    if (!d_lambda || !d_x || !d_grad) {
        c->err = "null argument";
        return NS_ERR_ARG;
    }
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev != c->device) {
        c->err = "the context's device is not the current device";
        return NS_ERR_STATE;
    }
    double* s = c->noalloc_scratch;  // looked up at bind, with the context's device current
    if (!s) {
        c->err = "scratch address not set up";
        return NS_ERR_STATE;
    }
    ns::outlet_dot<double>(NO, c->d_optr, c->d_onode, c->d_a_msk, nullptr, d_lambda, s, st);
    ns::outlet_dot<double>(NO, c->d_optr, c->d_onode, c->d_a_msk, nullptr, d_x, s + ns::kNoAllocMaxOutlets, st);
    ns::resistance_grad(NO, s, s + ns::kNoAllocMaxOutlets, c->d_Q, c->a_f, c->c_f, d_grad, st);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        c->err = std::string("kernel launch failed: ") + hipGetErrorString(e);
        return NS_ERR_HIP;
    }
    return NS_OK;
}
