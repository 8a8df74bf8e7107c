// Host-side helpers shared by the C ABI translation units of libdd.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <string>
#include <vector>

#include "dd_internal.h"

namespace dd {

dd_status fail(dd_ctx *ctx, dd_status st, const std::string &msg);
void *workspace(dd_ctx *ctx, const std::string &name, size_t bytes, hipError_t *err);
size_t prec_bytes(dd_prec p);
hipError_t enter(dd_ctx *ctx);
TileTable tiles_for(const dd_blocks *B, int nr, int g);
int rhs_group(const dd_ctx *ctx, int nr, dd_prec sp, dd_prec lk);
int hop_group(const dd_ctx *ctx, int nr, dd_prec sp, dd_prec lk);
BlkArgs blk_args(const dd_blocks *B, const TileTable &tt, int nr, int g);
const void *links_for(const dd_gauge *G, dd_prec prec);
double hop_bytes(const dd_blocks *B, int nr, dd_prec prec, double extra_vectors);
hipError_t run_hop(dd_ctx *ctx, const dd_blocks *B, const BlkArgs &ba, const HopArgs &ha, dd_prec prec);
// Segments per block of the x0-walk that run_hop takes for these blocks, rhs
// group and precision; 0 when it takes the chunked kernel.
int hop_walk_segments(dd_ctx *ctx, const dd_blocks *B, const BlkArgs &ba, dd_prec prec);
// Dhat = 1 - kappa^2 H_eo H_oe as one x0-walk kernel (launch_dhat_walk): when
// it applies to these blocks, rhs and spinor/link precision, and its launch.
bool dhat_walk_applies(const dd_ctx *ctx, const dd_blocks *B, const BlkArgs &ba, dd_prec prec);
hipError_t run_dhat(dd_ctx *ctx, const dd_blocks *B, const BlkArgs &ba, const HopArgs &ha, dd_prec prec);
bool dlam_walk_applies(const dd_ctx *ctx, const dd_blocks *B, dd_prec prec);
double dlam_bytes(const dd_blocks *B, int nr, dd_prec prec);
// rhs per workgroup of the one-kernel Dhat (1 or 3)
int dhat_rhs_per_wg(const dd_ctx *ctx, const dd_blocks *B, int n_rhs);
HopArgs hop_args(void *out, const void *in, const void *links, int parity, double c_hop);
// releases the context's dense-LU library handle
void logdet_release(dd_ctx *ctx);

// y = D_Lambda x (dd_apply_D_block): argument checks (links of the precision,
// kappa of the clover term), the bytes of each of its four half fields, and
// the operator with the half fields x_e, x_o, y_e, y_o given (pack, one hop
// launch per parity, unpack; synchronizes).  clover: the clover term A in the
// arithmetic precision (null for the Wilson operator), applied in place to
// y before the hops.
dd_status apply_D_check(dd_ctx *ctx, const dd_blocks *B, const dd_gauge *G, dd_prec prec, double kappa,
                        const void *x_dev, void *y_dev, int32_t n_rhs, const void **links, const void **clover);
size_t apply_D_half_bytes(const dd_blocks *B, int n_rhs, dd_prec prec);
dd_status apply_D_with(dd_ctx *ctx, const dd_blocks *B, const void *links, const void *clover, double kappa,
                       dd_prec prec, const void *x_dev, void *y_dev, int32_t n_rhs, void *const hf[4]);
// The gauge's clover matrices (A, or A^-1 with inverse) for spinors of the
// precision that arithmetic precision prec computes in; null without a
// clover term.  clover_check: the clover term was built for this kappa.
const void *clover_for(const dd_gauge *G, dd_prec prec, bool inverse);
// The kernels address a block's half fields of n_rhs rhs with 32-bit byte
// offsets: true when the largest block's FP64 half fields fit.
bool rhs_fit(const dd_blocks *B, int n_rhs);
dd_status clover_check(dd_ctx *ctx, const dd_gauge *G, double kappa);

// Timing of one kernel launch of a class (events only while timing is on).
struct TimedLaunch {
    dd_ctx *ctx;
    int kclass;
    hipEvent_t stop = nullptr;
    TimedLaunch(dd_ctx *c, int k, double bytes) : ctx(c), kclass(k)
    {
        if (!ctx->timing) return;
        Timer &t = ctx->timers[kclass];
        if (t.used == t.ev.size()) {
            hipEvent_t a, b;
            hipEventCreate(&a);
            hipEventCreate(&b);
            t.ev.push_back({a, b});
        }
        hipEventRecord(t.ev[t.used].first, ctx->stream);
        stop = t.ev[t.used].second;
        t.used++;
        t.bytes += bytes;
    }
    ~TimedLaunch()
    {
        if (stop) hipEventRecord(stop, ctx->stream);
    }
};

template <typename T>
hipError_t upload(T **dst, const std::vector<T> &src)
{
    const size_t bytes = std::max<size_t>(src.size() * sizeof(T), sizeof(T));
    hipError_t e = hipMalloc((void **)dst, bytes);
    if (e != hipSuccess) return e;
    if (!src.empty()) e = hipMemcpy(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice);
    return e;
}

}  // namespace dd

#define HIPCHECK(ctx, expr)                                                                      \
    do {                                                                                         \
        hipError_t e_ = (expr);                                                                  \
        if (e_ != hipSuccess)                                                                    \
            return ::dd::fail((ctx), e_ == hipErrorOutOfMemory ? DD_ENOMEM : DD_EDEVICE,          \
                              std::string(#expr) + ": " + hipGetErrorString(e_));                \
    } while (0)
