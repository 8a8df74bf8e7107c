// The global rest of the multi-boson action, eq. (globalMB) of Section 4:
//
//   S^r_k = || u_k chi_k + W_{dPi1,dL0} chi_k ||^2 summed over dPi_1,
//
// field k taken at z = u_k (as the block-local term is), with
// W_{dPi1,dL0} chi = Dhat_{dPi1}^{-1} Dhat_{dPi1,dL0} chi.  Eliminating
// Lambda1bar from D_{Lambda_1} (Lambda_1 = Lambda1bar u dPi_1) shows that this
// is [D_{Lambda_1}^{-1} D_{Lambda_1,dL0} chi] restricted to dPi_1: one solve on
// the inactive region Lambda_1 (Dirichlet at the active boxes) per field.  The
// library does exactly that on a dd_make_inactive domain: the source is the
// domain's exterior hops (from the active boxes, dd_mb_exterior_source), the
// solve is dd_block_solve, and a fixed-order reduction over the dPi_1 list
// gives each field's value.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "dd_host.h"
#include "dd_internal.h"

using namespace dd;

namespace {

constexpr int kGlobChunk = 4096;  // dPi_1 sites per workgroup

// partial[k][c] = sum over the dPi_1 sites of chunk c of |u_k chi_k + v_k|^2
// (12 complex components per site); chi [n_fields][V][24] and v [nf][V][24]
// (FP64, canonical site order); fixed-order sums.
__global__ void __launch_bounds__(256) k_mb_global(const int64_t *dpi1, int64_t n, const double *u, const double *chi,
                                                   const double *v, int64_t V, int nchunk, double *partial)
{
    __shared__ double red[256];
    const int c = blockIdx.x, k = blockIdx.y;
    const double ur = u[2 * k], ui = u[2 * k + 1];
    const double *ck = chi + (int64_t)k * V * 24, *vk = v + (int64_t)k * V * 24;
    double acc = 0;
    const int64_t i0 = (int64_t)c * kGlobChunk, i1 = min(i0 + kGlobChunk, n);
    for (int64_t i = i0 + threadIdx.x; i < i1; i += 256) {
        const int64_t s = dpi1[i] * 24;
#pragma unroll
        for (int q = 0; q < 12; q++) {
            const double xr = ck[s + 2 * q], xi = ck[s + 2 * q + 1];
            const double wr = ur * xr - ui * xi + vk[s + 2 * q];
            const double wi = ur * xi + ui * xr + vk[s + 2 * q + 1];
            acc += wr * wr + wi * wi;
        }
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[(int64_t)k * nchunk + c] = red[0];
}

}  // namespace

extern "C" dd_status dd_mb_global_action(dd_ctx *ctx, const dd_blocks *D, const dd_gauge *G, double kappa,
                                         int32_t n_fields, const double *u_host, const void *chi_global_dev,
                                         const dd_solve_params *params, double *S_field_host, double *S_total_host,
                                         dd_solve_stats *stats)
{
    if (!ctx || !D || !G || !u_host || !chi_global_dev) return fail(ctx, DD_EINVAL, "null argument");
    if (!D->inactive) return fail(ctx, DD_EINVAL, "the blocks are not an inactive-region domain (dd_make_inactive)");
    if (G->blocks != D) return fail(ctx, DD_EINVAL, "gauge was loaded for other blocks");
    if (n_fields < 1 || n_fields > kMaxRhs) return fail(ctx, DD_EINVAL, "n_fields must be in 1..64");
    HIPCHECK(ctx, enter(ctx));
    dd_solve_params prm;
    if (params) prm = *params;
    else dd_solve_params_default(&prm);
    const int64_t V = D->soff[1];
    const int64_t n = (int64_t)D->dpi1.size();
    const int nchunk = (int)std::max<int64_t>(1, (n + kGlobChunk - 1) / kGlobChunk);
    // fields per solve: the source and the solution (FP64) and the solver's
    // workspace grow with the fields of a call; the context's own workspaces
    // count as free (as for the block-local action)
    int fc = ctx->mb_fields;
    if (fc <= 0) {
        size_t fr = 0, tot = 0;
        HIPCHECK(ctx, hipMemGetInfo(&fr, &tot));
        for (const auto &kv : ctx->ws) fr += kv.second.bytes;
        const double per_field =
            (double)V * (2 * 192.0 + 576.0 + 132.0 * prec_bytes(prm.inner_prec == DD_F64 ? DD_F64 : DD_F32));
        fc = (int)std::max(1.0, std::floor(0.6 * (double)fr / per_field));
    }
    fc = std::min<int>(fc, n_fields);
    while (fc > 1 && !rhs_fit(D, fc)) fc--;  // 32-bit offsets of the domain's half fields
    hipError_t e = hipSuccess;
    const size_t fbytes = (size_t)V * 24 * fc * sizeof(double);
    double *f = (double *)workspace(ctx, "mg_f", fbytes, &e);
    double *v = f ? (double *)workspace(ctx, "mg_v", fbytes, &e) : nullptr;
    double *ud = v ? (double *)workspace(ctx, "mg_u", (size_t)n_fields * 2 * sizeof(double), &e) : nullptr;
    double *part = ud ? (double *)workspace(ctx, "mg_part", (size_t)nchunk * fc * sizeof(double), &e) : nullptr;
    if (!part) return fail(ctx, DD_ENOMEM, std::string("workspace: ") + hipGetErrorString(e));
    HIPCHECK(ctx, hipMemcpyAsync(ud, u_host, (size_t)n_fields * 2 * sizeof(double), hipMemcpyHostToDevice,
                                 ctx->stream));
    std::vector<double> S(n_fields, 0.0), hp((size_t)nchunk * fc);
    dd_status st_all = DD_OK;
    double seconds = 0;
    int32_t cycles = 0, resolved = 0;
    int64_t inner = 0;
    for (int f0 = 0; f0 < n_fields; f0 += fc) {
        const int nf = std::min(fc, n_fields - f0);
        const double *chi = (const double *)chi_global_dev + (size_t)f0 * V * 24;
        // source D_{Lambda_1, dLambda_0} chi: the hops from the active boxes
        HIPCHECK(ctx, hipMemsetAsync(f, 0, (size_t)V * 24 * nf * sizeof(double), ctx->stream));
        dd_status st = dd_mb_exterior_source(ctx, D, G, kappa, nf, chi, f, 2);
        if (st != DD_OK) return st;
        dd_solve_stats cs;
        std::memset(&cs, 0, sizeof(cs));
        if (stats) {
            cs.iters = stats->iters ? stats->iters + f0 : nullptr;
            cs.true_relres = stats->true_relres ? stats->true_relres + f0 : nullptr;
            cs.flags = stats->flags ? stats->flags + f0 : nullptr;
        }
        st = dd_block_solve(ctx, D, G, kappa, f, v, nf, &prm, &cs);
        if (st != DD_OK && st != DD_ENOCONV) return st;
        if (st == DD_ENOCONV) st_all = DD_ENOCONV;
        seconds += cs.seconds;
        cycles = std::max(cycles, cs.outer_cycles);
        inner += cs.inner_iterations;
        resolved += cs.resolved_pairs;
        if (n > 0) {
            hipLaunchKernelGGL(k_mb_global, dim3(nchunk, nf), dim3(256), 0, ctx->stream, D->d_dpi1, n, ud + 2 * f0, chi,
                               v, V, nchunk, part);
            HIPCHECK(ctx, hipGetLastError());
            HIPCHECK(ctx, hipMemcpyAsync(hp.data(), part, (size_t)nchunk * nf * sizeof(double), hipMemcpyDeviceToHost,
                                         ctx->stream));
            HIPCHECK(ctx, hipStreamSynchronize(ctx->stream));
            for (int k = 0; k < nf; k++)
                for (int c = 0; c < nchunk; c++) S[f0 + k] += hp[(size_t)k * nchunk + c];
        }
    }
    double tot = 0;
    for (int k = 0; k < n_fields; k++) tot += S[k];
    if (S_field_host) std::memcpy(S_field_host, S.data(), (size_t)n_fields * sizeof(double));
    if (S_total_host) *S_total_host = tot;
    if (stats) {
        stats->seconds = seconds;
        stats->outer_cycles = cycles;
        stats->inner_iterations = inner;
        stats->rhs_per_solve = fc;
        stats->resolved_pairs = resolved;
    }
    if (st_all == DD_ENOCONV) ctx->err = "some fields' solves on the inactive region missed the tolerance";
    return st_all;
}
