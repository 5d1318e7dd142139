// chom_mlp_loss_grad_noalloc: the surrogate's loss and gradient evaluation
// with its working memory in a file-scope device array instead of allocations.
//
// Each GPU the library runs on holds its own copy of `scratch` until the
// process ends.  In host code the array's name is only a stand-in for the
// symbol: its device address is looked up once per device
// (hipGetSymbolAddress, with that device current) and only that address is
// handed to kernels.  Every call on a device shares that device's array, so
// calls that overlap on one device race; each call clears what must start at
// zero (the flag, the gradient) with kernels, never with memset nodes.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>
#include <string>

#include "internal.h"
#include "mlp.h"

namespace {

constexpr long long kMaxRows = 4096;   // records per call
constexpr long long kBytes = chom::mlp::ws_bytes(kMaxRows);
constexpr int kMaxDevices = 64;

std::mutex g_mu;
unsigned char *g_addr[kMaxDevices] = {};

}  // namespace

static __device__ __align__(256) unsigned char scratch[kBytes];

namespace {

// Device address of this device's copy of `scratch` (looked up on first use).
int scratch_address(unsigned char **out) {
    int dev = -1;
    const hipError_t ge = hipGetDevice(&dev);
    if (ge != hipSuccess || dev < 0 || dev >= kMaxDevices) {
        chom::set_error("chom_mlp_loss_grad_noalloc: no usable current device");
        return CHOM_EDEVICE;
    }
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_addr[dev] == nullptr) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || p == nullptr) {
            chom::set_error(std::string("chom_mlp_loss_grad_noalloc: hipGetSymbolAddress failed: ") +
                            hipGetErrorString(e));
            return CHOM_EDEVICE;
        }
        g_addr[dev] = static_cast<unsigned char *>(p);
    }
    *out = g_addr[dev];
    return CHOM_OK;
}

}  // namespace

extern "C" int chom_mlp_loss_grad_noalloc(chom_mlp *mlp, int32_t member, const chom_params *params, const double *C,
                                          const double *K, const double *D, int64_t n, double *loss, float *grad) {
    if (!mlp || !params || !C || !K || !D || !loss || !grad) {
        chom::set_error("chom_mlp_loss_grad_noalloc: null argument");
        return CHOM_EINVAL;
    }
    if (n < 1 || n > kMaxRows) {
        chom::set_error("chom_mlp_loss_grad_noalloc: n must be in [1, " + std::to_string(kMaxRows) +
                        "] (the size of the library's static workspace)");
        return CHOM_EINVAL;
    }
    if (!chom::mlp_ready(mlp, member)) {
        chom::set_error("chom_mlp_loss_grad_noalloc: bad member or no standardisation record");
        return CHOM_EINVAL;
    }
    unsigned char *ws = nullptr;
    const int st = scratch_address(&ws);
    if (st != CHOM_OK) return st;
    const int r = chom::mlp_loss_grad_ws(mlp, member, reinterpret_cast<const double *>(params), C, K, D, n, loss, grad,
                                         ws, kMaxRows);
    if (r != CHOM_OK) chom::set_error(std::string("chom_mlp_loss_grad_noalloc: ") + chom_last_error());
    return r;
}
