// The learned block preconditioner's handle (host side).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "dd_internal.h"

struct dd_nn {
    dd_ctx *ctx = nullptr;  // creating context (identity only)
    int device = 0;
    int act = 0;            // DD_NN_LINEAR or DD_NN_RELU
    dd::NnExt e{};          // block extent the network works on
    int64_t off[4] = {0, 0, 0, 0};  // layer offsets in the weight arrays
    int64_t nw = 0;                 // number of weights
    float *d_w = nullptr;   // FP32 weights, layers back to back, each [81][c_in][c_out]
    float *d_g = nullptr;   // gradients
    float *d_m = nullptr;   // Adam first moments
    float *d_v = nullptr;   // Adam second moments
    float *d_wf = nullptr;  // one layer's flipped weights (backward pass)
    float *d_part = nullptr;  // weight-gradient partials per row chunk
    int step = 0;             // Adam steps taken
    uint16_t *d_wbf = nullptr;  // BF16 inference weights, per layer [81][32 out][32 in]
    int bf16_step = -1;         // Adam step the BF16 weights were made at
    int infer_prec = DD_BF16;   // precision of the network inside solves (DD_BF16 or DD_F32)
};

namespace dd {

// the network on nrows rows: X [rows][24] -> O [rows][24], keeping the
// pre-activations Z1, Z2 [rows][32]
hipError_t nn_forward(dd_ctx *ctx, const dd_nn *nn, const float *X, float *Z1, float *Z2, float *O, int64_t nrows);

// z = N(v) for every (block, rhs) pair of an even half field in the library
// layout (inner precision sp); v and z may not alias.  Blocks must all have
// the network's extent (checked by the caller).
// With active (per pair, may be null) the BF16 network skips pairs whose flag is 0
// and leaves their z unchanged.  A pair whose output is not finite gets z = v
// (the identity) and, with flags given, flags[pair] |= 16.
hipError_t nn_apply_half(dd_ctx *ctx, dd_nn *nn, const dd_blocks *B, const void *v, void *z, int n_rhs, dd_prec sp,
                         const int32_t *active = nullptr, int32_t *flags = nullptr);
bool nn_fits(const dd_nn *nn, const dd_blocks *B);

// the network in BF16 on the matrix cores: Xb [rows][32] BF16 -> O [rows][24] FP32.
// With block origins (origin [nb][4], pair p on block p % nb) the input must
// be zero on odd sites and only the even sites of O are written.
// With hin as well, the input is that even half field (FP32) and Xb is unused;
// with hin->out, the even output sites go into that half field and O is unused.
hipError_t nn_forward_bf16(dd_ctx *ctx, dd_nn *nn, const uint16_t *Xb, uint16_t *Zb1, uint16_t *Zb2, float *O,
                           int64_t nrows, const int32_t *active, int pair0, const int32_t *origin = nullptr,
                           int nb = 0, const NnHalfIn *hin = nullptr);

}  // namespace dd
