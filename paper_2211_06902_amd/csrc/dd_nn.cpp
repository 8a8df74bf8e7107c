// Host side of the learned block preconditioner: network handle, batched
// application, loss and gradients, and the Adam training loop over (source,
// solution) pairs produced by the block solver.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <random>
#include <string>
#include <vector>

#include "dd_host.h"
#include "dd_internal.h"
#include "dd_nn.h"

using namespace dd;

namespace {

constexpr int kCh[4] = {24, 32, 32, 24};
constexpr int kChunksDw = 64;  // row chunks of the weight-gradient reduction

int64_t layer_size(int l) { return 81LL * kCh[l] * kCh[l + 1]; }

// Device buffers of one batch: input, pre-activations, output, target and
// the backward temporaries, for up to `rows` rows.
struct Batch {
    float *X, *Z1, *Z2, *O, *T, *G3, *H2, *D2, *H1, *D1;
};

bool same_shape(const dd_nn *nn, const dd_blocks *B)
{
    for (int b = 0; b < B->nb; b++)
        for (int m = 0; m < 4; m++)
            if (B->box[16 * b + 4 + m] != nn->e.e[m]) return false;
    return true;
}

}  // namespace

namespace dd {

hipError_t nn_forward(dd_ctx *ctx, const dd_nn *nn, const float *X, float *Z1, float *Z2, float *O, int64_t nrows)
{
    hipStream_t st = ctx->stream;
    const int a = nn->act;
    hipError_t e;
    if ((e = launch_conv(X, nn->d_w + nn->off[0], Z1, nrows, nn->e, 24, 32, 0, st)) != hipSuccess) return e;
    if ((e = launch_conv(Z1, nn->d_w + nn->off[1], Z2, nrows, nn->e, 32, 32, a, st)) != hipSuccess) return e;
    return launch_conv(Z2, nn->d_w + nn->off[2], O, nrows, nn->e, 32, 24, a, st);
}

bool nn_fits(const dd_nn *nn, const dd_blocks *B) { return same_shape(nn, B); }

hipError_t nn_forward_bf16(dd_ctx *ctx, dd_nn *nn, const uint16_t *Xb, uint16_t *Zb1, uint16_t *Zb2, float *O,
                           int64_t nrows, const int32_t *active, int pair0, const int32_t *origin, int nb,
                           const NnHalfIn *hin)
{
    hipStream_t st = ctx->stream;
    hipError_t e = hipSuccess;
    if (nn->bf16_step != nn->step) {
        for (int l = 0; l < 3 && e == hipSuccess; l++)
            e = launch_weights_bf16(nn->d_w + nn->off[l], nn->d_wbf + l * 81 * 1024, kCh[l], kCh[l + 1], st);
        if (e != hipSuccess) return e;
        nn->bf16_step = nn->step;
    }
    const int v = ctx->nn_kernel;
    // with block origins (an even half field in, its even sites out): layer 1
    // skips the zero odd input sites (reading the half field itself when hin
    // is given), layer 3 computes the even sites only
    if ((e = launch_conv_mfma(Xb, nn->d_wbf, Zb1, nrows, nn->e, nn->act, false, v, active, pair0, origin, nb,
                              hin ? 3 : 1, st, hin)) != hipSuccess)
        return e;
    if ((e = launch_conv_mfma(Zb1, nn->d_wbf + 81 * 1024, Zb2, nrows, nn->e, nn->act, false, v, active, pair0, origin,
                              nb, 0, st)) != hipSuccess)
        return e;
    return launch_conv_mfma(Zb2, nn->d_wbf + 2 * 81 * 1024, O, nrows, nn->e, 0, true, v, active, pair0, origin, nb,
                            hin && hin->out ? 4 : 2, st, hin);
}

// the LDS kernel handles the block shape (x0-slices of at most 512 sites, even extents)
static bool nn_slice_fits(const dd_nn *nn)
{
    return nn->e.e[1] * nn->e.e[2] * nn->e.e[3] <= 512 && (nn->e.e[3] & 1) == 0;
}

hipError_t nn_apply_half(dd_ctx *ctx, dd_nn *nn, const dd_blocks *B, const void *v, void *z, int n_rhs, dd_prec sp,
                         const int32_t *active, int32_t *flags)
{
    const int S = nn->e.S;
    const int np = n_rhs * B->nb;
    const int chunk = (int)std::max<int64_t>(1, std::min<int64_t>(np, (int64_t(1) << 30) / ((int64_t)S * 32 * 4)));
    hipError_t e = hipSuccess;
    const size_t rows = (size_t)chunk * S;
    const bool bf = nn->infer_prec == DD_BF16;
    const size_t hb = bf ? 2 : 4;  // bytes per hidden value
    void *X = workspace(ctx, "nn_hX", rows * (bf ? 32 * 2 : 24 * 4), &e);
    void *Z1 = X ? workspace(ctx, "nn_hZ1", rows * 32 * hb, &e) : nullptr;
    void *Z2 = Z1 ? workspace(ctx, "nn_hZ2", rows * 32 * hb, &e) : nullptr;
    float *O = Z2 ? (float *)workspace(ctx, "nn_hO", rows * 24 * 4, &e) : nullptr;
    if (!O) return e;
    HalfRows hr{B->d_perm, B->d_perm_off, B->d_soff, B->d_h, B->nb, n_rhs, 0, 0, S};
    for (int p0 = 0; p0 < np && e == hipSuccess; p0 += chunk) {
        hr.pair0 = p0;
        hr.npairs = std::min(chunk, np - p0);
        const int64_t nrows = (int64_t)hr.npairs * S;
        if (bf) {
            // FP32 half fields feed the first layer directly (LDS kernel); else via BF16 rows
            const bool fused = sp == DD_F32 && ctx->nn_kernel == 1 && nn_slice_fits(nn);
            const NnHalfIn hin{(const float *)v, (float *)z, B->d_perm, B->d_perm_off, B->d_soff, B->d_h, n_rhs};
            if (!fused) e = launch_half_rows_bf16(v, (uint16_t *)X, sp, hr, ctx->stream);
            TimedLaunch tl(ctx, DD_KCLASS_NN_BF16, 2.0 * 81 * (24 * 32 + 32 * 32 + 32 * 24) * (double)nrows);
            if (e == hipSuccess)
                e = nn_forward_bf16(ctx, nn, (uint16_t *)X, (uint16_t *)Z1, (uint16_t *)Z2, O, nrows, active, p0,
                                    B->d_origin, B->nb, fused ? &hin : nullptr);
        } else {
            e = launch_half_rows(v, (float *)X, nullptr, sp, hr, 0, ctx->stream);
            if (e == hipSuccess) e = nn_forward(ctx, nn, (float *)X, (float *)Z1, (float *)Z2, O, nrows);
        }
        // (the fused path wrote z itself)
        if (e == hipSuccess && !(bf && sp == DD_F32 && ctx->nn_kernel == 1 && nn_slice_fits(nn)))
            e = launch_half_rows(nullptr, O, z, sp, hr, 1, ctx->stream);
    }
    // a pair whose network output is not finite falls back to the identity
    if (e == hipSuccess) e = launch_nn_guard(B, v, z, sp, n_rhs, active, flags, ctx->stream);
    return e;
}

}  // namespace dd

namespace {

// gradients of all weights into nn->d_g for dL/dOut in b.G3 (forward values in b)
hipError_t nn_backward(dd_ctx *ctx, dd_nn *nn, Batch &b, int64_t nrows)
{
    hipStream_t st = ctx->stream;
    const int a = nn->act;
    const int64_t n32 = nrows * 32;
    hipError_t e;
    // layer 3
    if ((e = launch_conv_dw(b.Z2, b.G3, nn->d_part, nn->d_g + nn->off[2], nrows, kChunksDw, nn->e, 32, 24, a, st)) != hipSuccess) return e;
    if ((e = launch_flip_weights(nn->d_w + nn->off[2], nn->d_wf, 32, 24, st)) != hipSuccess) return e;
    if ((e = launch_conv(b.G3, nn->d_wf, b.H2, nrows, nn->e, 24, 32, 0, st)) != hipSuccess) return e;
    float *dZ2 = b.H2;
    if (a) {
        if ((e = launch_relu_grad(b.H2, b.Z2, b.D2, n32, st)) != hipSuccess) return e;
        dZ2 = b.D2;
    }
    // layer 2
    if ((e = launch_conv_dw(b.Z1, dZ2, nn->d_part, nn->d_g + nn->off[1], nrows, kChunksDw, nn->e, 32, 32, a, st)) != hipSuccess) return e;
    if ((e = launch_flip_weights(nn->d_w + nn->off[1], nn->d_wf, 32, 32, st)) != hipSuccess) return e;
    if ((e = launch_conv(dZ2, nn->d_wf, b.H1, nrows, nn->e, 32, 32, 0, st)) != hipSuccess) return e;
    float *dZ1 = b.H1;
    if (a) {
        if ((e = launch_relu_grad(b.H1, b.Z1, b.D1, n32, st)) != hipSuccess) return e;
        dZ1 = b.D1;
    }
    // layer 1
    return launch_conv_dw(b.X, dZ1, nn->d_part, nn->d_g + nn->off[0], nrows, kChunksDw, nn->e, 24, 32, 0, st);
}

// A set of (source, solution) pairs in the solver's layout [n_rhs][total_sites][24]
// (FP64): row base (in sites) and origin parity of every pair = rhs * n_blocks + block.
struct PairSet {
    int64_t *d_base = nullptr;
    int32_t *d_opar = nullptr;
    int n = 0;
    void release()
    {
        if (d_base) hipFree(d_base);
        if (d_opar) hipFree(d_opar);
        d_base = nullptr;
        d_opar = nullptr;
    }
};

hipError_t make_pairs(const dd_blocks *B, int n_rhs, PairSet *ps)
{
    std::vector<int64_t> base((size_t)n_rhs * B->nb);
    std::vector<int32_t> opar((size_t)n_rhs * B->nb);
    const int64_t tot = B->soff[B->nb];
    for (int r = 0; r < n_rhs; r++)
        for (int b = 0; b < B->nb; b++) {
            base[(size_t)r * B->nb + b] = r * tot + B->soff[b];
            const int32_t *o = &B->box[16 * b];
            opar[(size_t)r * B->nb + b] = (o[0] + o[1] + o[2] + o[3]) & 1;
        }
    ps->n = (int)base.size();
    hipError_t e = upload(&ps->d_base, base);
    if (e == hipSuccess) e = upload(&ps->d_opar, opar);
    return e;
}

struct Work {
    Batch b;
    int32_t *d_idx;
    double *d_lpart, *d_den, *d_loss;
};

dd_status get_work(dd_ctx *ctx, int batch, int S, Work *w)
{
    hipError_t e = hipSuccess;
    const size_t r = (size_t)batch * S;
    auto get = [&](const char *name, size_t bytes) -> void * {
        if (e != hipSuccess) return nullptr;
        return workspace(ctx, name, bytes, &e);
    };
    w->b.X = (float *)get("nn_X", r * 24 * 4);
    w->b.Z1 = (float *)get("nn_Z1", r * 32 * 4);
    w->b.Z2 = (float *)get("nn_Z2", r * 32 * 4);
    w->b.O = (float *)get("nn_O", r * 24 * 4);
    w->b.T = (float *)get("nn_T", r * 24 * 4);
    w->b.G3 = (float *)get("nn_G3", r * 24 * 4);
    w->b.H2 = (float *)get("nn_H2", r * 32 * 4);
    w->b.D2 = (float *)get("nn_D2", r * 32 * 4);
    w->b.H1 = (float *)get("nn_H1", r * 32 * 4);
    w->b.D1 = (float *)get("nn_D1", r * 32 * 4);
    w->d_idx = (int32_t *)get("nn_idx", (size_t)std::max(batch, 1) * 4);
    w->d_lpart = (double *)get("nn_lpart", (size_t)batch * 16 * 2 * 8);
    w->d_den = (double *)get("nn_den", (size_t)batch * 8);
    w->d_loss = (double *)get("nn_loss", 2 * 8);
    if (e != hipSuccess) return fail(ctx, DD_ENOMEM, std::string("network workspace: ") + hipGetErrorString(e));
    return DD_OK;
}

}  // namespace

extern "C" {

int64_t dd_nn_num_weights(void) { return layer_size(0) + layer_size(1) + layer_size(2); }

dd_status dd_nn_create(dd_ctx *ctx, const int32_t extent[4], int32_t act, const float *weights_host, dd_nn **out)
{
    if (!ctx || !extent || !weights_host || !out) return fail(ctx, DD_EINVAL, "null argument");
    *out = nullptr;
    if (act != DD_NN_LINEAR && act != DD_NN_RELU) return fail(ctx, DD_EINVAL, "act must be DD_NN_LINEAR or DD_NN_RELU");
    for (int m = 0; m < 4; m++)
        if (extent[m] < 1 || extent[m] > 64) return fail(ctx, DD_EINVAL, "network block extents must be in 1..64");
    HIPCHECK(ctx, enter(ctx));
    dd_nn *nn = new dd_nn;
    nn->ctx = ctx;
    nn->device = ctx->device;
    nn->act = act;
    nn->e.S = 1;
    for (int m = 0; m < 4; m++) {
        nn->e.e[m] = extent[m];
        nn->e.S *= extent[m];
    }
    nn->off[0] = 0;
    for (int l = 0; l < 3; l++) nn->off[l + 1] = nn->off[l] + layer_size(l);
    nn->nw = nn->off[3];
    const size_t wb = (size_t)nn->nw * sizeof(float);
    hipError_t e = hipSuccess;
    float **bufs[] = {&nn->d_w, &nn->d_g, &nn->d_m, &nn->d_v};
    for (float **p : bufs)
        if (e == hipSuccess) e = hipMalloc((void **)p, wb);
    if (e == hipSuccess) e = hipMalloc((void **)&nn->d_wf, 81 * 32 * 32 * sizeof(float));
    if (e == hipSuccess) e = hipMalloc((void **)&nn->d_wbf, 3 * 81 * 32 * 32 * sizeof(uint16_t));
    if (e == hipSuccess) e = hipMalloc((void **)&nn->d_part, (size_t)kChunksDw * 81 * 32 * 32 * sizeof(float));
    if (e == hipSuccess) e = hipMemcpy(nn->d_w, weights_host, wb, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemset(nn->d_m, 0, wb);
    if (e == hipSuccess) e = hipMemset(nn->d_v, 0, wb);
    if (e != hipSuccess) {
        dd_nn_free(nn);
        return fail(ctx, e == hipErrorOutOfMemory ? DD_ENOMEM : DD_EDEVICE, std::string("network: ") + hipGetErrorString(e));
    }
    *out = nn;
    return DD_OK;
}

dd_status dd_nn_free(dd_nn *nn)
{
    if (!nn) return DD_EINVAL;
    hipSetDevice(nn->device);
    void *ptrs[] = {nn->d_w, nn->d_g, nn->d_m, nn->d_v, nn->d_wf, nn->d_part, nn->d_wbf};
    for (void *p : ptrs)
        if (p) hipFree(p);
    delete nn;
    return DD_OK;
}

dd_status dd_nn_get_weights(dd_ctx *ctx, const dd_nn *nn, float *weights_host)
{
    if (!ctx || !nn || !weights_host) return fail(ctx, DD_EINVAL, "null argument");
    HIPCHECK(ctx, enter(ctx));
    HIPCHECK(ctx, hipMemcpyAsync(weights_host, nn->d_w, nn->nw * sizeof(float), hipMemcpyDeviceToHost, ctx->stream));
    HIPCHECK(ctx, hipStreamSynchronize(ctx->stream));
    return DD_OK;
}

dd_status dd_nn_apply(dd_ctx *ctx, dd_nn *nn, dd_prec prec, const float *x_dev, float *y_dev, int64_t n)
{
    if (!ctx || !nn || (n > 0 && (!x_dev || !y_dev))) return fail(ctx, DD_EINVAL, "null argument");
    if (n < 0) return fail(ctx, DD_EINVAL, "n must be >= 0");
    if (prec != DD_F32 && prec != DD_BF16) return fail(ctx, DD_EINVAL, "network precision must be DD_F32 or DD_BF16");
    HIPCHECK(ctx, enter(ctx));
    const int64_t chunk = std::max<int64_t>(1, (int64_t(1) << 28) / ((int64_t)nn->e.S * 32 * 4));  // ~256 MiB per buffer
    hipError_t e = hipSuccess;
    const size_t rows = (size_t)std::max<int64_t>(std::min(n, chunk) * nn->e.S, 1);
    void *Z1 = workspace(ctx, "nn_aZ1", rows * 32 * 4, &e);
    void *Z2 = Z1 ? workspace(ctx, "nn_aZ2", rows * 32 * 4, &e) : nullptr;
    void *Xb = Z2 ? workspace(ctx, "nn_aXb", rows * 32 * 2, &e) : nullptr;
    if (!Xb) return fail(ctx, DD_ENOMEM, std::string("network workspace: ") + hipGetErrorString(e));
    for (int64_t i0 = 0; i0 < n; i0 += chunk) {
        const int64_t m = std::min(chunk, n - i0);
        const int64_t off = i0 * nn->e.S * 24, nrows = m * nn->e.S;
        if (prec == DD_F32) {
            HIPCHECK(ctx, nn_forward(ctx, nn, x_dev + off, (float *)Z1, (float *)Z2, y_dev + off, nrows));
        } else {
            HIPCHECK(ctx, launch_rows_f32_to_bf16(x_dev + off, (uint16_t *)Xb, nrows, ctx->stream));
            HIPCHECK(ctx, nn_forward_bf16(ctx, nn, (uint16_t *)Xb, (uint16_t *)Z1, (uint16_t *)Z2, y_dev + off, nrows,
                                          nullptr, 0));
        }
    }
    HIPCHECK(ctx, hipStreamSynchronize(ctx->stream));
    return DD_OK;
}

dd_status dd_nn_apply_blocks(dd_ctx *ctx, dd_nn *nn, const dd_blocks *B, const void *x_dev, void *y_dev,
                             int32_t n_rhs)
{
    if (!ctx || !nn || !B || !x_dev || !y_dev) return fail(ctx, DD_EINVAL, "null argument");
    if (n_rhs < 1 || n_rhs > kMaxRhs) return fail(ctx, DD_EINVAL, "n_rhs must be in 1..64");
    if (B->ctx != ctx) return fail(ctx, DD_EINVAL, "blocks belong to another context (or have no device tables)");
    if (!nn_fits(nn, B)) return fail(ctx, DD_EINVAL, "every block must have the network's extent");
    HIPCHECK(ctx, enter(ctx));
    hipError_t e = hipSuccess;
    const size_t half = (size_t)(B->soff[B->nb] / 2) * 24 * n_rhs * sizeof(float);
    void *xe = workspace(ctx, "nb_xe", half, &e);
    void *xo = xe ? workspace(ctx, "nb_xo", half, &e) : nullptr;
    void *ze = xo ? workspace(ctx, "nb_ze", half, &e) : nullptr;
    if (!ze) return fail(ctx, DD_ENOMEM, std::string("workspace: ") + hipGetErrorString(e));
    // FP32 half fields as inside a solve; the odd half is unused on input and zero on output
    HIPCHECK(ctx, launch_pack_spinor(B, (const double *)x_dev, xe, xo, DD_F32, n_rhs, ctx->stream));
    HIPCHECK(ctx, nn_apply_half(ctx, nn, B, xe, ze, n_rhs, DD_F32));
    HIPCHECK(ctx, hipMemsetAsync(xo, 0, half, ctx->stream));
    HIPCHECK(ctx, launch_unpack_spinor(B, ze, xo, (double *)y_dev, DD_F32, n_rhs, ctx->stream));
    HIPCHECK(ctx, hipStreamSynchronize(ctx->stream));
    return DD_OK;
}

dd_status dd_nn_set_inference(dd_ctx *ctx, dd_nn *nn, dd_prec prec)
{
    if (!ctx || !nn) return fail(ctx, DD_EINVAL, "null argument");
    if (prec != DD_F32 && prec != DD_BF16) return fail(ctx, DD_EINVAL, "network precision must be DD_F32 or DD_BF16");
    nn->infer_prec = prec;
    return DD_OK;
}

dd_status dd_nn_loss_grad(dd_ctx *ctx, dd_nn *nn, const dd_blocks *B, const void *src_dev, const void *sol_dev,
                          int32_t n_rhs, const int32_t *pairs_host, int32_t n_pairs, int32_t mask_even, double *loss,
                          float *grad_host)
{
    if (!ctx || !nn || !B || !src_dev || !sol_dev || !pairs_host || !loss) return fail(ctx, DD_EINVAL, "null argument");
    if (n_pairs < 1 || n_rhs < 1) return fail(ctx, DD_EINVAL, "need at least one pair");
    if (!same_shape(nn, B)) return fail(ctx, DD_EINVAL, "every block must have the network's extent");
    for (int i = 0; i < n_pairs; i++)
        if (pairs_host[i] < 0 || pairs_host[i] >= n_rhs * B->nb) return fail(ctx, DD_EINVAL, "pair index out of range");
    HIPCHECK(ctx, enter(ctx));
    Work w;
    dd_status s = get_work(ctx, n_pairs, nn->e.S, &w);
    if (s != DD_OK) return s;
    PairSet ps;
    hipError_t e = make_pairs(B, n_rhs, &ps);
    hipStream_t st = ctx->stream;
    const int64_t nrows = (int64_t)n_pairs * nn->e.S;
    if (e == hipSuccess) e = hipMemcpyAsync(w.d_idx, pairs_host, n_pairs * 4, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemsetAsync(w.d_loss, 0, 16, st);
    if (e == hipSuccess)
        e = launch_gather_rows((const double *)src_dev, (const double *)sol_dev, ps.d_base, w.d_idx, w.b.X, w.b.T,
                               n_pairs, nn->e.S, st);
    if (e == hipSuccess) e = nn_forward(ctx, nn, w.b.X, w.b.Z1, w.b.Z2, w.b.O, nrows);
    if (e == hipSuccess)
        e = launch_loss(w.b.O, w.b.T, ps.d_opar, w.d_idx, w.d_lpart, w.d_den, w.d_loss, w.b.G3, n_pairs, mask_even,
                        nn->e, st);
    if (e == hipSuccess) e = nn_backward(ctx, nn, w.b, nrows);
    double lh[2] = {0, 0};
    if (e == hipSuccess) e = hipMemcpyAsync(lh, w.d_loss, 16, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess && grad_host)
        e = hipMemcpyAsync(grad_host, nn->d_g, nn->nw * sizeof(float), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    ps.release();
    HIPCHECK(ctx, e);
    *loss = lh[0];
    return DD_OK;
}

void dd_nn_train_params_default(dd_nn_train_params *p)
{
    if (!p) return;
    std::memset(p, 0, sizeof(*p));
    p->epochs = 4;
    p->batch = 32;
    p->lr = 1e-3;
    p->beta1 = 0.9;
    p->beta2 = 0.999;
    p->eps = 1e-8;
    p->seed = 4100;
    p->mask_even = 1;
}

dd_status dd_nn_train(dd_ctx *ctx, dd_nn *nn, const dd_blocks *B, const void *src_dev, const void *sol_dev,
                      int32_t n_rhs, const void *val_src_dev, const void *val_sol_dev, int32_t val_n_rhs,
                      const dd_nn_train_params *params, double *train_loss, double *val_loss)
{
    if (!ctx || !nn || !B || !src_dev || !sol_dev) return fail(ctx, DD_EINVAL, "null argument");
    if (n_rhs < 1) return fail(ctx, DD_EINVAL, "n_rhs must be >= 1");
    if (!same_shape(nn, B)) return fail(ctx, DD_EINVAL, "every block must have the network's extent");
    dd_nn_train_params p;
    if (params) p = *params;
    else dd_nn_train_params_default(&p);
    if (p.epochs < 1 || p.batch < 1 || !(p.lr > 0)) return fail(ctx, DD_EINVAL, "bad training parameters");
    const bool has_val = val_src_dev && val_sol_dev && val_n_rhs > 0;
    HIPCHECK(ctx, enter(ctx));
    Work w;
    dd_status s = get_work(ctx, p.batch, nn->e.S, &w);
    if (s != DD_OK) return s;
    PairSet tr, va;
    hipError_t e = make_pairs(B, n_rhs, &tr);
    if (e == hipSuccess && has_val) e = make_pairs(B, val_n_rhs, &va);
    int32_t *d_perm = e == hipSuccess ? (int32_t *)workspace(ctx, "nn_perm", (size_t)tr.n * 4, &e) : nullptr;
    hipStream_t st = ctx->stream;
    std::vector<int32_t> perm(tr.n);
    std::vector<int32_t> vidx(has_val ? va.n : 0);
    std::iota(vidx.begin(), vidx.end(), 0);
    int32_t *d_vidx = (e == hipSuccess && has_val) ? (int32_t *)workspace(ctx, "nn_vidx", (size_t)va.n * 4, &e) : nullptr;
    if (e == hipSuccess && has_val) e = hipMemcpyAsync(d_vidx, vidx.data(), va.n * 4, hipMemcpyHostToDevice, st);
    for (int ep = 0; ep < p.epochs && e == hipSuccess; ep++) {
        std::iota(perm.begin(), perm.end(), 0);
        std::mt19937_64 rng(p.seed + (uint64_t)ep);
        std::shuffle(perm.begin(), perm.end(), rng);
        e = hipMemcpyAsync(d_perm, perm.data(), tr.n * 4, hipMemcpyHostToDevice, st);
        if (e == hipSuccess) e = hipMemsetAsync(w.d_loss, 0, 16, st);
        for (int i0 = 0; i0 < tr.n && e == hipSuccess; i0 += p.batch) {
            const int nb = std::min(p.batch, tr.n - i0);
            const int64_t nrows = (int64_t)nb * nn->e.S;
            e = launch_gather_rows((const double *)src_dev, (const double *)sol_dev, tr.d_base, d_perm + i0, w.b.X,
                                   w.b.T, nb, nn->e.S, st);
            if (e == hipSuccess) e = nn_forward(ctx, nn, w.b.X, w.b.Z1, w.b.Z2, w.b.O, nrows);
            if (e == hipSuccess)
                e = launch_loss(w.b.O, w.b.T, tr.d_opar, d_perm + i0, w.d_lpart, w.d_den, w.d_loss, w.b.G3, nb,
                                p.mask_even, nn->e, st);
            if (e == hipSuccess) e = nn_backward(ctx, nn, w.b, nrows);
            if (e == hipSuccess)
                e = launch_adam(nn->d_w, nn->d_g, nn->d_m, nn->d_v, nn->nw, (float)p.lr, (float)p.beta1,
                                (float)p.beta2, (float)p.eps, ++nn->step, st);
        }
        double lh[2] = {0, 0};
        if (e == hipSuccess) e = hipMemcpyAsync(lh, w.d_loss, 16, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (train_loss) train_loss[ep] = lh[1] > 0 ? lh[0] / lh[1] : 0.0;
        if (has_val && e == hipSuccess) {
            e = hipMemsetAsync(w.d_loss, 0, 16, st);
            double sum = 0;
            int cnt = 0;
            for (int i0 = 0; i0 < va.n && e == hipSuccess; i0 += p.batch) {
                const int nb = std::min(p.batch, va.n - i0);
                e = launch_gather_rows((const double *)val_src_dev, (const double *)val_sol_dev, va.d_base,
                                       d_vidx + i0, w.b.X, w.b.T, nb, nn->e.S, st);
                if (e == hipSuccess) e = nn_forward(ctx, nn, w.b.X, w.b.Z1, w.b.Z2, w.b.O, (int64_t)nb * nn->e.S);
                if (e == hipSuccess)
                    e = launch_loss(w.b.O, w.b.T, va.d_opar, d_vidx + i0, w.d_lpart, w.d_den, w.d_loss, nullptr, nb,
                                    p.mask_even, nn->e, st);
                // the batch loss is a mean over its pairs: weight it by the pair count
                if (e == hipSuccess) e = hipMemcpyAsync(lh, w.d_loss, 16, hipMemcpyDeviceToHost, st);
                if (e == hipSuccess) e = hipStreamSynchronize(st);
                if (e == hipSuccess) {
                    sum += lh[0] * nb;
                    cnt += nb;
                    e = hipMemsetAsync(w.d_loss, 0, 16, st);
                }
            }
            if (val_loss) val_loss[ep] = cnt ? sum / cnt : 0.0;
        }
    }
    tr.release();
    va.release();
    HIPCHECK(ctx, e);
    HIPCHECK(ctx, hipStreamSynchronize(st));
    return DD_OK;
}

}  // extern "C"
