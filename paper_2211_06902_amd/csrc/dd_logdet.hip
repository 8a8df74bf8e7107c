// Per-block log-determinants ln det D_Lambda in FP64 (the block factors of
// eq. detD, Section 3: ln det D_{Omega_0^a} on framed blocks and
// ln det D_{Phi_1^a} on frames).
//
// det D_Lambda = det Dhat with Dhat = 1 - kappa^2 H_eo H_oe on the even sites
// (the odd-odd and even-even blocks of D_Lambda are the identity).  With the
// clover term, det D_Lambda = det A_ee det A_oo det Dhat' with
// Dhat' = 1 - kappa^2 A_ee^-1 H_eo A_oo^-1 H_oe (A^-1 applied in the hops) and
// ln det A(x) per site by LU of its two 6x6 chirality blocks.  Dhat is
// assembled as a dense n x n complex matrix per block (n = 12 h, h the sites
// of one parity), column batches of 64 unit vectors at a time through the
// FP64 hop kernels; the matrices are LU-factorised with partial pivoting by
// rocSOLVER's batched complex getrf (a plain library factorisation), and
// ln det = sum_i ln U_ii + i pi (number of row interchanges).
#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "dd_host.h"
#include "dd_internal.h"

using namespace dd;

namespace {

constexpr int kCols = 64;          // unit vectors per batch (rhs of the hop launches)
constexpr int kMaxLogdetDim = 6144;  // largest n = 12 h handled

// The even half field of kCols rhs holding the unit vectors j0 .. j0 + kCols - 1
// of blocks b0, b0 + 1, ... (one per grid row): column j = 12 h + a has the
// real part of complex component a (spin-colour) at even site h equal to one.
__global__ void __launch_bounds__(256) k_unit_batch(double *e, const int64_t *soff, int hb, int j0, int64_t per_block,
                                                    int b0)
{
    const int b = b0 + blockIdx.y;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= per_block) return;
    // t = (r * 24 + c) * hb + h within the block
    const int h = (int)(t % hb), rc = (int)(t / hb), c = rc % 24, r = rc / 24;
    const double v = (c % 2 == 0 && 12 * h + c / 2 == j0 + r) ? 1.0 : 0.0;
    e[(soff[b] >> 1) * 24 * kCols + t] = v;
}

// A[b][j][i] (column-major n x n, complex) = (Dhat e_j)_i for the batch's columns j < n.
__global__ void __launch_bounds__(256) k_gather_cols(const double *out, const int64_t *soff, int hb, int j0, int n,
                                                      double2 *A, int b0)
{
    const int bl = blockIdx.y, b = b0 + bl;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)kCols * n) return;
    const int r = (int)(t / n), i = (int)(t % n), j = j0 + r;
    if (j >= n) return;
    const int h = i / 12, a = i % 12;
    const double *o = out + (soff[b] >> 1) * 24 * kCols + ((int64_t)r * 24 + 2 * a) * hb + h;
    A[(size_t)bl * n * n + (size_t)j * n + i] = make_double2(o[0], o[hb]);
}

// ln det of each factorised matrix: sum of ln U_ii (complex) and i pi per row
// interchange, summed in a fixed order; the phase is wrapped into (-pi, pi].
__global__ void __launch_bounds__(256) k_logdet(const double2 *A, const int32_t *ipiv, int n, int b0, double *out)
{
    __shared__ double sre[256], sim[256];
    const int bl = blockIdx.x;
    const double2 *M = A + (size_t)bl * n * n;
    const int32_t *pv = ipiv + (size_t)bl * n;
    double re = 0, im = 0;
    for (int i = threadIdx.x; i < n; i += 256) {
        const double2 d = M[(size_t)i * n + i];
        re += 0.5 * log(d.x * d.x + d.y * d.y);
        im += atan2(d.y, d.x) + (pv[i] != i + 1 ? M_PI : 0.0);
    }
    sre[threadIdx.x] = re;
    sim[threadIdx.x] = im;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
            sre[threadIdx.x] += sre[threadIdx.x + w];
            sim[threadIdx.x] += sim[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        double ph = fmod(sim[0], 2 * M_PI);
        if (ph > M_PI) ph -= 2 * M_PI;
        if (ph <= -M_PI) ph += 2 * M_PI;
        out[2 * (b0 + bl)] = sre[0];
        out[2 * (b0 + bl) + 1] = ph;
    }
}

}  // namespace

extern "C" dd_status dd_block_logdet(dd_ctx *ctx, const dd_blocks *B, const dd_gauge *G, double kappa,
                                     double *logdet_dev, double *total_host)
{
    if (!ctx || !B || !G || (!logdet_dev && !total_host)) return fail(ctx, DD_EINVAL, "null argument");
    if (G->blocks != B) return fail(ctx, DD_EINVAL, "gauge was loaded for other blocks");
    const bool cl = G->d_cla64 != nullptr;
    if (cl) {
        const dd_status cs = clover_check(ctx, G, kappa);
        if (cs != DD_OK) return cs;
    }
    if (B->nb == 0 || B->nb > 65535) return fail(ctx, DD_EINVAL, "need 1..65535 blocks");
    const int hb = B->shapes[B->shape_of[0]].h;
    for (int k = 1; k < B->nb; k++)
        if (B->shapes[B->shape_of[k]].h != hb)
            return fail(ctx, DD_EUNSUPPORTED, "dd_block_logdet needs blocks of one size (sites per parity)");
    const int n = 12 * hb;
    if (n > kMaxLogdetDim) return fail(ctx, DD_EUNSUPPORTED, "block too large for a dense determinant (12 h > 6144)");
    HIPCHECK(ctx, enter(ctx));
    hipStream_t st = ctx->stream;
    hipError_t e = hipSuccess;
    const size_t half = (size_t)(B->soff[B->nb] / 2) * 24 * kCols * sizeof(double);
    double *fe = (double *)workspace(ctx, "ld_e", half, &e);
    double *fo = fe ? (double *)workspace(ctx, "ld_o", half, &e) : nullptr;
    double *fy = fo ? (double *)workspace(ctx, "ld_y", half, &e) : nullptr;
    double *ld = fy ? (double *)workspace(ctx, "ld_out", (size_t)B->nb * 2 * sizeof(double), &e) : nullptr;
    // matrices of as many blocks at a time as fit in 8 GiB
    const size_t mat = (size_t)n * n * sizeof(double2);
    const int chunk = (int)std::max<size_t>(1, std::min<size_t>((size_t)B->nb, (size_t(8) << 30) / mat));
    double2 *A = ld ? (double2 *)workspace(ctx, "ld_A", mat * chunk, &e) : nullptr;
    int32_t *ipiv = A ? (int32_t *)workspace(ctx, "ld_piv", (size_t)chunk * n * sizeof(int32_t), &e) : nullptr;
    int32_t *info = ipiv ? (int32_t *)workspace(ctx, "ld_info", (size_t)chunk * sizeof(int32_t), &e) : nullptr;
    if (!info) return fail(ctx, DD_ENOMEM, std::string("logdet workspace: ") + hipGetErrorString(e));
    if (!ctx->blas) {
        if (rocblas_create_handle(reinterpret_cast<rocblas_handle *>(&ctx->blas)) != rocblas_status_success)
            return fail(ctx, DD_EDEVICE, "rocblas_create_handle failed");
    }
    rocblas_handle hdl = reinterpret_cast<rocblas_handle>(ctx->blas);
    if (rocblas_set_stream(hdl, st) != rocblas_status_success) return fail(ctx, DD_EDEVICE, "rocblas_set_stream failed");
    const int g = 1;
    const BlkArgs ba = blk_args(B, tiles_for(B, kCols, g), kCols, g);
    const double k2 = kappa * kappa;
    const bool timing = ctx->timing;
    ctx->timing = false;
    for (int b0 = 0; b0 < B->nb && e == hipSuccess; b0 += chunk) {
        const int nc = std::min(chunk, B->nb - b0);
        // the hop walks launch this group's blocks only (the chunked hop does
        // every block; the others' results are not read)
        for (int j0 = 0; j0 < n; j0 += kCols) {
            const int64_t per = (int64_t)kCols * 24 * hb;
            hipLaunchKernelGGL(k_unit_batch, dim3((unsigned)((per + 255) / 256), nc), dim3(256), 0, st, fe,
                               B->d_soff, hb, j0, per, b0);
            if ((e = hipGetLastError()) != hipSuccess) break;
            // fo = H_oe e, then fy = e - kappa^2 H_eo fo; with the clover term
            // each hop result is multiplied by A^-1 of its output site
            HopArgs h1 = hop_args(fo, fe, G->d_u64, 1, 1.0);
            h1.clover = cl ? G->d_cli64 : nullptr;
            h1.b_lo = b0;
            h1.b_hi = b0 + nc;
            if ((e = run_hop(ctx, B, ba, h1, DD_F64)) != hipSuccess) break;
            HopArgs h2 = hop_args(fy, fo, G->d_u64, 0, -k2);
            h2.self = fe;
            h2.c_self = 1.0;
            h2.clover = cl ? G->d_cli64 : nullptr;
            h2.b_lo = b0;
            h2.b_hi = b0 + nc;
            if ((e = run_hop(ctx, B, ba, h2, DD_F64)) != hipSuccess) break;
            const int64_t cols = (int64_t)kCols * n;
            hipLaunchKernelGGL(k_gather_cols, dim3((unsigned)((cols + 255) / 256), nc), dim3(256), 0, st, fy,
                               B->d_soff, hb, j0, n, A, b0);
            if ((e = hipGetLastError()) != hipSuccess) break;
        }
        if (e != hipSuccess) break;
        if (rocsolver_zgetrf_strided_batched(hdl, n, n, reinterpret_cast<rocblas_double_complex *>(A), n,
                                             (rocblas_stride)n * n, ipiv, (rocblas_stride)n, info, nc) !=
            rocblas_status_success) {
            ctx->timing = timing;
            return fail(ctx, DD_EDEVICE, "rocsolver_zgetrf_strided_batched failed");
        }
        hipLaunchKernelGGL(k_logdet, dim3(nc), dim3(256), 0, st, A, ipiv, n, b0, ld);
        e = hipGetLastError();
    }
    ctx->timing = timing;
    HIPCHECK(ctx, e);
    if (cl) {
        // det D_Lambda = det A_ee det A_oo det(1 - kappa^2 A_ee^-1 H_eo A_oo^-1 H_oe)
        double *site = (double *)workspace(ctx, "ld_clsite", (size_t)B->soff[B->nb] * 2 * sizeof(double), &e);
        if (!site) return fail(ctx, DD_ENOMEM, std::string("logdet workspace: ") + hipGetErrorString(e));
        HIPCHECK(ctx, launch_clover_logdet_add(B, G->d_cla64, site, ld, st));
    }
    if (logdet_dev)
        HIPCHECK(ctx, hipMemcpyAsync(logdet_dev, ld, (size_t)B->nb * 2 * sizeof(double), hipMemcpyDeviceToDevice, st));
    if (total_host) {
        std::vector<double> h((size_t)B->nb * 2);
        HIPCHECK(ctx, hipMemcpyAsync(h.data(), ld, h.size() * sizeof(double), hipMemcpyDeviceToHost, st));
        HIPCHECK(ctx, hipStreamSynchronize(st));
        double re = 0, im = 0;
        for (int k = 0; k < B->nb; k++) {
            re += h[2 * k];
            im += h[2 * k + 1];
        }
        im = std::fmod(im, 2 * M_PI);
        if (im > M_PI) im -= 2 * M_PI;
        if (im <= -M_PI) im += 2 * M_PI;
        total_host[0] = re;
        total_host[1] = im;
    }
    HIPCHECK(ctx, hipStreamSynchronize(st));
    return DD_OK;
}

namespace dd {

void logdet_release(dd_ctx *ctx)
{
    if (ctx->blas) rocblas_destroy_handle(reinterpret_cast<rocblas_handle>(ctx->blas));
    ctx->blas = nullptr;
}

}  // namespace dd
