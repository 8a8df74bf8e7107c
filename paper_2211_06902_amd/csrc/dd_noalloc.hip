// dd_apply_D_block without device allocations: the four half fields the
// operator packs into (x_e, x_o, y_e, y_o) live in a preallocated scratch
// array of fixed size, one per device, instead of the context's workspaces.
//
// In host code `scratch` names a host-side stand-in, not device memory: the
// device address of each device's copy is taken once per device with
// hipGetSymbolAddress (that device current) and only that address is handed
// to kernels.  Every call on a device shares its copy, so calls that overlap
// on one device race; nothing in it needs to start at zero (the pack writes
// every x_e, x_o element and the hops every y_e, y_o element before they are
// read).
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "dd_host.h"
#include "dd_internal.h"

namespace {

constexpr size_t kScratchBytes = size_t(128) << 20;  // 128 MiB per device
constexpr int kMaxDevices = 64;

}  // namespace

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

std::mutex g_mu;
void *g_scratch[kMaxDevices] = {};

// Device address of this device's scratch copy; the caller has made `device`
// current.
hipError_t scratch_address(int device, void **out)
{
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_scratch[device]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch[device] = p;
    }
    *out = g_scratch[device];
    return hipSuccess;
}

}  // namespace

using namespace dd;

extern "C" dd_status dd_apply_D_block_noalloc(dd_ctx *ctx, const dd_blocks *B, const dd_gauge *G, double kappa,
                                              dd_prec prec, const void *x_dev, void *y_dev, int32_t n_rhs)
{
    const void *links = nullptr, *clover = nullptr;
    dd_status st = apply_D_check(ctx, B, G, prec, kappa, x_dev, y_dev, n_rhs, &links, &clover);
    if (st != DD_OK) return st;
    const size_t slot = (apply_D_half_bytes(B, n_rhs, prec) + 255) & ~size_t(255);
    if (4 * slot > kScratchBytes)
        return fail(ctx, DD_EINVAL,
                    "dd_apply_D_block_noalloc: " + std::to_string(4 * slot) + " bytes of scratch needed, the limit is " +
                        std::to_string(kScratchBytes) + " (total_sites * n_rhs * 48 * bytes per real)");
    HIPCHECK(ctx, enter(ctx));  // makes the context's device current
    void *base = nullptr;
    HIPCHECK(ctx, scratch_address(ctx->device, &base));
    char *c = static_cast<char *>(base);
    void *const hf[4] = {c, c + slot, c + 2 * slot, c + 3 * slot};
    // no kernel timers here: their events are created on first use
    const bool timing = ctx->timing;
    ctx->timing = false;
    st = apply_D_with(ctx, B, links, clover, kappa, prec, x_dev, y_dev, n_rhs, hf);
    ctx->timing = timing;
    return st;
}
