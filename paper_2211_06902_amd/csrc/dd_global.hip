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
#include <chrono>
#include <cmath>
#include <complex>
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
    prm.x0 = 0;  // the solutions are internal workspaces
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

// ------------------------------------------------------------------------
// W_z chi as a vector on dPi, the multi-boson field generation and the
// reweighting factor (Section 4: eqs. MBaction, localMB, globalMB and rw; the
// field generation is the method's one global inversion, on a vector of dPi,
// Conclusions).
//
// The rows of W_z chi on dLambda_0^a are the vector whose norm is S_MB^a,
// z chi + D_{Omega_0^a}^{-1} xi^a with xi^a the hops of chi from dPi into the
// block (dd_mb_exterior_source, parts 3); the rows on dPi_1 are those whose
// norm is S^r_MB, z chi + [D_{Lambda_1}^{-1} D_{Lambda_1,dLambda_0} chi]
// (dd_mb_global_action).  Vectors are FP64 fields of the whole lattice in
// canonical order, zero off dPi.

namespace {

constexpr int kDotChunk = 16384;  // complex entries per workgroup of the per-field dot products

// out[k][g_i] = z_k in[k][g_i] + (y ? y[k * ystride + yi_i] : 0) for the n
// sites g_i of a list; out is [nf][V][24], y [nf][ystride].  One thread per
// complex entry (12 per site row), so that a wavefront reads and writes about
// five whole 192-byte rows instead of touching 64 rows per instruction.
// Sites are distinct, so every entry is written by one thread.
__global__ void __launch_bounds__(256) k_rows(const int64_t *gidx, const int64_t *yidx, int64_t n, int nf,
                                              const double *z, const double *in, const double *y, int64_t ystride,
                                              int64_t V, double *out)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n * nf * 12) return;
    const int j = (int)(t % 12);
    const int64_t r = t / 12;
    const int k = (int)(r / n);
    const int64_t i = r - (int64_t)k * n;
    const int64_t g = gidx[i];
    const double zr = z[2 * k], zi = z[2 * k + 1];
    const double2 c = *reinterpret_cast<const double2 *>(in + ((int64_t)k * V + g) * 24 + 2 * j);
    double vr = zr * c.x - zi * c.y, vi = zr * c.y + zi * c.x;
    if (y) {
        const double2 a = *reinterpret_cast<const double2 *>(y + (int64_t)k * ystride + yidx[i] * 24 + 2 * j);
        vr += a.x;
        vi += a.y;
    }
    *reinterpret_cast<double2 *>(out + ((int64_t)k * V + g) * 24 + 2 * j) = make_double2(vr, vi);
}

hipError_t launch_rows(const int64_t *gidx, const int64_t *yidx, int64_t n, int nf, const double *z, const double *in,
                       const double *y, int64_t ystride, int64_t V, double *out, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_rows, dim3((unsigned)((n * nf * 12 + 255) / 256)), dim3(256), 0, s, gidx, yidx, n, nf, z, in,
                       y, ystride, V, out);
    return hipGetLastError();
}

// Up to three complex dot products <a_d, b_d> = sum conj(a_d) b_d per field
// over n complex entries each; partial[((k * nchunk + c) * 3 + d) * 2 + {re, im}]
// holds chunk c's fixed-order sum.
struct DotArgs {
    const double *a[3];
    const double *b[3];
    int nd;
};

__global__ void __launch_bounds__(256) k_field_dots(DotArgs da, int64_t n, int nchunk, double *partial)
{
    __shared__ double red[6][256];
    const int c = blockIdx.x, k = blockIdx.y;
    const int64_t i0 = (int64_t)c * kDotChunk, i1 = min(i0 + (int64_t)kDotChunk, n);
    double acc[6] = {0, 0, 0, 0, 0, 0};
    for (int64_t i = i0 + threadIdx.x; i < i1; i += 256) {
        const int64_t o = ((int64_t)k * n + i) * 2;
        for (int d = 0; d < da.nd; d++) {
            const double ar = da.a[d][o], ai = da.a[d][o + 1], br = da.b[d][o], bi = da.b[d][o + 1];
            acc[2 * d] += ar * br + ai * bi;
            acc[2 * d + 1] += ar * bi - ai * br;
        }
    }
    for (int j = 0; j < 2 * da.nd; j++) red[j][threadIdx.x] = acc[j];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            for (int j = 0; j < 2 * da.nd; j++) red[j][threadIdx.x] += red[j][threadIdx.x + w];
        __syncthreads();
    }
    if ((int)threadIdx.x < 2 * da.nd)
        partial[((int64_t)k * nchunk + c) * 6 + threadIdx.x] = red[threadIdx.x][0];
}

// out[k] = sum_j coef[k][j] x_j[k] over n complex entries per field (x_j may be
// null; out may be one of the x_j: each entry is read before it is written).
__global__ void __launch_bounds__(256) k_lincomb(int64_t n, int nf, const double *coef, const double *x0,
                                                 const double *x1, const double *x2, double *out)
{
    const int64_t total = n * nf;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int k = (int)(t / n);
        const double *cf = coef + 6 * k;
        double vr = 0, vi = 0;
        const double *xs[3] = {x0, x1, x2};
#pragma unroll
        for (int j = 0; j < 3; j++) {
            if (!xs[j]) continue;
            const double xr = xs[j][2 * t], xi = xs[j][2 * t + 1];
            vr += cf[2 * j] * xr - cf[2 * j + 1] * xi;
            vi += cf[2 * j] * xi + cf[2 * j + 1] * xr;
        }
        out[2 * t] = vr;
        out[2 * t + 1] = vi;
    }
}

using cplx = std::complex<double>;

// The operator W_z on groups of up to fc fields, with its workspaces.
struct WOp {
    dd_ctx *ctx = nullptr;
    const dd_blocks *B = nullptr, *D = nullptr;
    const dd_gauge *G = nullptr, *GD = nullptr;
    double kappa = 0;
    dd_solve_params prm{};
    int fc = 1;
    int64_t V = 0, totalB = 0, nbnd = 0, n1 = 0;
    int64_t *gidx = nullptr, *yidx = nullptr;  // dLambda_0 sites: global index, block-layout index
    double *xi = nullptr, *y = nullptr, *f = nullptr, *v = nullptr;
    double *partial = nullptr, *coef = nullptr;
    int nchunk = 1;
    std::vector<double> hpart;
    // accumulated over the applications
    double seconds = 0;
    int64_t inner = 0;
    int32_t cycles = 0;
    int64_t applies = 0;
    bool missed = false;  // some inner solve missed its tolerance
    double worst = 0;     // largest inner true relative residual
};

dd_status wop_check(dd_ctx *ctx, const dd_blocks *B, const dd_gauge *G, const dd_blocks *D, const dd_gauge *GD)
{
    if (!D->inactive || D->parent != B->serial)
        return fail(ctx, DD_EINVAL, "domain must be dd_make_inactive of these blocks");
    if (G->blocks != B || GD->blocks != D) return fail(ctx, DD_EINVAL, "a gauge was loaded for other blocks");
    // the clover term: both solves must see the same operator
    if ((G->d_cla64 != nullptr) != (GD->d_cla64 != nullptr) ||
        (G->d_cla64 && (G->cl_csw != GD->cl_csw || G->cl_kappa != GD->cl_kappa)))
        return fail(ctx, DD_EINVAL, "the two gauges must carry the same clover term (or none)");
    if (B->x_code.empty() || B->bnd.empty())
        return fail(ctx, DD_EINVAL, "the blocks have no inner boxes (dLambda_0 is empty)");
    return DD_OK;
}

// Fields per group: the operator's four FP64 fields (block layout and lattice)
// plus the solver's workspace, and `extra` lattice fields of the caller.
int wop_fields(dd_ctx *ctx, const dd_blocks *B, const dd_blocks *D, const dd_solve_params &prm, int extra,
               int n_fields, hipError_t *err)
{
    int fc = ctx->mb_fields;
    if (fc <= 0) {
        size_t fr = 0, tot = 0;
        *err = hipMemGetInfo(&fr, &tot);
        if (*err != hipSuccess) return 0;
        for (const auto &kv : ctx->ws) fr += kv.second.bytes;
        const double V = (double)D->soff[1], T = (double)B->soff[B->nb];
        const double per_field = 2 * 192.0 * T + (2.0 + extra) * 192.0 * V +
                                 std::max(T, V) * (576.0 + 132.0 * prec_bytes(prm.inner_prec == DD_F64 ? DD_F64 : DD_F32));
        fc = (int)std::max(1.0, std::floor(0.5 * (double)fr / per_field));
    }
    fc = std::min(fc, std::min(n_fields, kMaxRhs));
    while (fc > 1 && (!rhs_fit(B, fc) || !rhs_fit(D, fc))) fc--;
    return fc;
}

dd_status wop_init(WOp &w, dd_ctx *ctx, const dd_blocks *B, const dd_gauge *G, const dd_blocks *D,
                   const dd_gauge *GD, double kappa, const dd_solve_params *params, int fc)
{
    w.ctx = ctx;
    w.B = B;
    w.G = G;
    w.D = D;
    w.GD = GD;
    w.kappa = kappa;
    if (params) w.prm = *params;
    else dd_solve_params_default(&w.prm);
    w.prm.x0 = 0;  // the solutions are internal workspaces
    w.fc = fc;
    w.V = D->soff[1];
    w.totalB = B->soff[B->nb];
    w.nbnd = (int64_t)B->bnd.size();
    w.n1 = (int64_t)D->dpi1.size();
    // dLambda_0 sites: global canonical index and index in the block layout
    std::vector<int64_t> hg(w.nbnd), hy(w.nbnd);
    for (int b = 0; b < B->nb; b++) {
        const int32_t *bx = &B->box[16 * b];
        for (int64_t q = B->boff[b]; q < B->boff[b + 1]; q++) {
            int l = B->bnd[q], c[4];
            for (int m = 3; m >= 0; m--) {
                c[m] = l % bx[4 + m];
                l /= bx[4 + m];
            }
            int64_t g = 0;
            for (int m = 0; m < 4; m++) g = g * B->L[m] + (bx[m] + c[m]) % B->L[m];
            hg[q] = g;
            hy[q] = B->soff[b] + B->bnd[q];
        }
    }
    w.nchunk = (int)std::max<int64_t>(1, (w.V * 12 + kDotChunk - 1) / kDotChunk);
    w.hpart.assign((size_t)w.nchunk * fc * 6, 0.0);
    hipError_t e = hipSuccess;
    const size_t fb = (size_t)fc * w.totalB * 24 * sizeof(double), fl = (size_t)fc * w.V * 24 * sizeof(double);
    w.gidx = (int64_t *)workspace(ctx, "wop_gidx", (size_t)w.nbnd * 8, &e);
    if (w.gidx) w.yidx = (int64_t *)workspace(ctx, "wop_yidx", (size_t)w.nbnd * 8, &e);
    if (w.yidx) w.xi = (double *)workspace(ctx, "wop_xi", fb, &e);
    if (w.xi) w.y = (double *)workspace(ctx, "wop_y", fb, &e);
    if (w.y) w.f = (double *)workspace(ctx, "wop_f", fl, &e);
    if (w.f) w.v = (double *)workspace(ctx, "wop_v", fl, &e);
    if (w.v) w.partial = (double *)workspace(ctx, "wop_part", w.hpart.size() * sizeof(double), &e);
    if (w.partial) w.coef = (double *)workspace(ctx, "wop_coef", (size_t)8 * kMaxRhs * 6 * sizeof(double), &e);
    if (!w.coef) return fail(ctx, DD_ENOMEM, std::string("workspace: ") + hipGetErrorString(e));
    HIPCHECK(ctx, hipMemcpyAsync(w.gidx, hg.data(), (size_t)w.nbnd * 8, hipMemcpyHostToDevice, ctx->stream));
    HIPCHECK(ctx, hipMemcpyAsync(w.yidx, hy.data(), (size_t)w.nbnd * 8, hipMemcpyHostToDevice, ctx->stream));
    HIPCHECK(ctx, hipStreamSynchronize(ctx->stream));
    return DD_OK;
}

dd_status wop_solve(WOp &w, const dd_blocks *X, const dd_gauge *GX, const double *src, double *sol, int nf)
{
    const int np = nf * X->nb;
    std::vector<int32_t> it(np), fl(np);
    std::vector<double> rr(np);
    dd_solve_stats cs;
    std::memset(&cs, 0, sizeof(cs));
    cs.iters = it.data();
    cs.true_relres = rr.data();
    cs.flags = fl.data();
    const dd_status st = dd_block_solve(w.ctx, X, GX, w.kappa, src, sol, nf, &w.prm, &cs);
    if (st != DD_OK && st != DD_ENOCONV) return st;
    if (st == DD_ENOCONV) w.missed = true;
    w.seconds += cs.seconds;
    w.inner += cs.inner_iterations;
    w.cycles = std::max(w.cycles, cs.outer_cycles);
    for (double r : rr) w.worst = std::max(w.worst, r);
    return DD_OK;
}

// out = W_z chi for nf <= fc fields; z_dev [nf][2] on the device; out must not
// be chi.
dd_status wop_apply(WOp &w, int nf, const double *z_dev, const double *chi, double *out)
{
    dd_ctx *ctx = w.ctx;
    const hipStream_t s = ctx->stream;
    HIPCHECK(ctx, hipMemsetAsync(w.xi, 0, (size_t)nf * w.totalB * 24 * sizeof(double), s));
    HIPCHECK(ctx, hipMemsetAsync(w.f, 0, (size_t)nf * w.V * 24 * sizeof(double), s));
    HIPCHECK(ctx, hipMemsetAsync(out, 0, (size_t)nf * w.V * 24 * sizeof(double), s));
    dd_status st = dd_mb_exterior_source(ctx, w.B, w.G, w.kappa, nf, chi, w.xi, 3);
    if (st != DD_OK) return st;
    if ((st = wop_solve(w, w.B, w.G, w.xi, w.y, nf)) != DD_OK) return st;
    HIPCHECK(ctx, launch_rows(w.gidx, w.yidx, w.nbnd, nf, z_dev, chi, w.y, w.totalB * 24, w.V, out, s));
    if (w.n1 > 0) {
        if ((st = dd_mb_exterior_source(ctx, w.D, w.GD, w.kappa, nf, chi, w.f, 2)) != DD_OK) return st;
        if ((st = wop_solve(w, w.D, w.GD, w.f, w.v, nf)) != DD_OK) return st;
        HIPCHECK(ctx, launch_rows(w.D->d_dpi1, w.D->d_dpi1, w.n1, nf, z_dev, chi, w.v, w.V * 24, w.V, out, s));
    }
    w.applies++;
    return DD_OK;
}

// out = in on dPi, zero elsewhere (one_dev: [nf][2] of 1 + 0i)
dd_status wop_restrict(WOp &w, int nf, const double *one_dev, const double *in, double *out)
{
    dd_ctx *ctx = w.ctx;
    HIPCHECK(ctx, hipMemsetAsync(out, 0, (size_t)nf * w.V * 24 * sizeof(double), ctx->stream));
    HIPCHECK(ctx, launch_rows(w.gidx, w.yidx, w.nbnd, nf, one_dev, in, nullptr, 0, w.V, out, ctx->stream));
    if (w.n1 > 0)
        HIPCHECK(ctx, launch_rows(w.D->d_dpi1, w.D->d_dpi1, w.n1, nf, one_dev, in, nullptr, 0, w.V, out, ctx->stream));
    return DD_OK;
}

// per-field <a_d, b_d> for d < nd (host result [nf][nd])
dd_status wop_dots(WOp &w, int nf, int nd, const double *const *a, const double *const *b, std::vector<cplx> &res)
{
    dd_ctx *ctx = w.ctx;
    DotArgs da{};
    da.nd = nd;
    for (int d = 0; d < nd; d++) {
        da.a[d] = a[d];
        da.b[d] = b[d];
    }
    hipLaunchKernelGGL(k_field_dots, dim3(w.nchunk, nf), dim3(256), 0, ctx->stream, da, w.V * 12, w.nchunk,
                       w.partial);
    HIPCHECK(ctx, hipGetLastError());
    HIPCHECK(ctx, hipMemcpyAsync(w.hpart.data(), w.partial, (size_t)nf * w.nchunk * 6 * sizeof(double),
                                 hipMemcpyDeviceToHost, ctx->stream));
    HIPCHECK(ctx, hipStreamSynchronize(ctx->stream));
    res.assign((size_t)nf * nd, cplx(0, 0));
    for (int k = 0; k < nf; k++)
        for (int c = 0; c < w.nchunk; c++)
            for (int d = 0; d < nd; d++) {
                const double *p = &w.hpart[((size_t)k * w.nchunk + c) * 6 + 2 * d];
                res[(size_t)k * nd + d] += cplx(p[0], p[1]);
            }
    return DD_OK;
}

// out = sum_j coef[k][j] x_j for each field; slot picks a coefficient buffer
// (the host copy must stay alive until the stream has read it: every caller
// synchronises before it reuses a slot)
dd_status wop_lincomb(WOp &w, int slot, int nf, const std::vector<cplx> &coef, const double *x0, const double *x1,
                      const double *x2, double *out)
{
    dd_ctx *ctx = w.ctx;
    double *cd = w.coef + (size_t)slot * kMaxRhs * 6;
    HIPCHECK(ctx, hipMemcpyAsync(cd, coef.data(), (size_t)nf * 3 * sizeof(cplx), hipMemcpyHostToDevice, ctx->stream));
    const int64_t n = w.V * 12;
    const int64_t blocks = std::min<int64_t>((n * nf + 255) / 256, 65536);
    hipLaunchKernelGGL(k_lincomb, dim3((unsigned)blocks), dim3(256), 0, ctx->stream, n, nf, cd, x0, x1, x2, out);
    HIPCHECK(ctx, hipGetLastError());
    return DD_OK;
}

void wop_stats(const WOp &w, dd_solve_stats *stats)
{
    if (!stats) return;
    stats->seconds = w.seconds;
    stats->outer_cycles = w.cycles;
    stats->inner_iterations = w.inner;
    stats->rhs_per_solve = w.fc;
}

}  // namespace

extern "C" dd_status dd_mb_apply_W(dd_ctx *ctx, const dd_blocks *B, const dd_gauge *G, const dd_blocks *D,
                                   const dd_gauge *GD, double kappa, int32_t n_fields, const double *z_host,
                                   const void *chi_global_dev, void *out_global_dev, const dd_solve_params *params,
                                   dd_solve_stats *stats)
{
    if (!ctx || !B || !G || !D || !GD || !z_host || !chi_global_dev || !out_global_dev)
        return fail(ctx, DD_EINVAL, "null argument");
    if (chi_global_dev == out_global_dev) return fail(ctx, DD_EINVAL, "out must not be chi");
    if (n_fields < 1 || n_fields > kMaxRhs) return fail(ctx, DD_EINVAL, "n_fields must be in 1..64");
    dd_status st = wop_check(ctx, B, G, D, GD);
    if (st != DD_OK) return st;
    HIPCHECK(ctx, enter(ctx));
    dd_solve_params prm;
    if (params) prm = *params;
    else dd_solve_params_default(&prm);
    hipError_t e = hipSuccess;
    const int fc = wop_fields(ctx, B, D, prm, 0, n_fields, &e);
    if (fc < 1) return fail(ctx, DD_EDEVICE, hipGetErrorString(e));
    WOp w;
    if ((st = wop_init(w, ctx, B, G, D, GD, kappa, &prm, fc)) != DD_OK) return st;
    double *zd = (double *)workspace(ctx, "wop_z", (size_t)n_fields * 2 * sizeof(double), &e);
    if (!zd) return fail(ctx, DD_ENOMEM, std::string("workspace: ") + hipGetErrorString(e));
    HIPCHECK(ctx, hipMemcpyAsync(zd, z_host, (size_t)n_fields * 2 * sizeof(double), hipMemcpyHostToDevice, ctx->stream));
    for (int f0 = 0; f0 < n_fields; f0 += fc) {
        const int nf = std::min(fc, n_fields - f0);
        const size_t o = (size_t)f0 * w.V * 24;
        if ((st = wop_apply(w, nf, zd + 2 * f0, (const double *)chi_global_dev + o, (double *)out_global_dev + o)) !=
            DD_OK)
            return st;
    }
    HIPCHECK(ctx, hipStreamSynchronize(ctx->stream));
    wop_stats(w, stats);
    if (w.missed) {
        ctx->err = "some inner solves missed the tolerance";
        return DD_ENOCONV;
    }
    return DD_OK;
}

extern "C" dd_status dd_mb_generate(dd_ctx *ctx, const dd_blocks *B, const dd_gauge *G, const dd_blocks *D,
                                    const dd_gauge *GD, double kappa, int32_t n_fields, const double *u_host,
                                    const void *eta_global_dev, void *chi_global_dev, double tol, int32_t maxit,
                                    const dd_solve_params *params, int32_t *iters_host, double *relres_host,
                                    dd_solve_stats *stats)
{
    if (!ctx || !B || !G || !D || !GD || !u_host || !eta_global_dev || !chi_global_dev)
        return fail(ctx, DD_EINVAL, "null argument");
    if (eta_global_dev == chi_global_dev) return fail(ctx, DD_EINVAL, "chi must not be eta");
    if (n_fields < 1 || n_fields > kMaxRhs) return fail(ctx, DD_EINVAL, "n_fields must be in 1..64");
    if (!(tol > 0) || maxit < 1) return fail(ctx, DD_EINVAL, "tol must be > 0 and maxit >= 1");
    dd_status st = wop_check(ctx, B, G, D, GD);
    if (st != DD_OK) return st;
    HIPCHECK(ctx, enter(ctx));
    const auto t0 = std::chrono::steady_clock::now();
    dd_solve_params prm;
    if (params) prm = *params;
    else dd_solve_params_default(&prm);
    hipError_t e = hipSuccess;
    const int fc = wop_fields(ctx, B, D, prm, 6, n_fields, &e);
    if (fc < 1) return fail(ctx, DD_EDEVICE, hipGetErrorString(e));
    WOp w;
    if ((st = wop_init(w, ctx, B, G, D, GD, kappa, &prm, fc)) != DD_OK) return st;
    const size_t fl = (size_t)fc * w.V * 24 * sizeof(double);
    double *vec[6] = {};
    const char *names[6] = {"gen_r", "gen_rh", "gen_p", "gen_v", "gen_s", "gen_t"};
    for (int i = 0; i < 6; i++)
        if (!(vec[i] = (double *)workspace(ctx, names[i], fl, &e)))
            return fail(ctx, DD_ENOMEM, std::string("workspace: ") + hipGetErrorString(e));
    double *r = vec[0], *rh = vec[1], *p = vec[2], *v = vec[3], *s = vec[4], *t = vec[5];
    double *ud = (double *)workspace(ctx, "gen_u", (size_t)n_fields * 2 * sizeof(double), &e);
    double *one = ud ? (double *)workspace(ctx, "gen_one", (size_t)kMaxRhs * 2 * sizeof(double), &e) : nullptr;
    if (!one) return fail(ctx, DD_ENOMEM, std::string("workspace: ") + hipGetErrorString(e));
    std::vector<double> hone(2 * kMaxRhs, 0.0);
    for (int k = 0; k < kMaxRhs; k++) hone[2 * k] = 1.0;
    HIPCHECK(ctx, hipMemcpyAsync(ud, u_host, (size_t)n_fields * 2 * sizeof(double), hipMemcpyHostToDevice, ctx->stream));
    HIPCHECK(ctx, hipMemcpyAsync(one, hone.data(), hone.size() * sizeof(double), hipMemcpyHostToDevice, ctx->stream));
    // Inner tolerance of the W applications inside the iteration: the error a
    // Krylov method tolerates in its operator grows as its residual falls, so
    // with relative residual rho the inner solves need only reach
    // 0.1 tol / rho (at most 1e-6, never below the requested inner tolerance).  The
    // true residual is taken with the requested one, and a field left above
    // tol restarts from its current solution (at most twice).
    const double tol_req = w.prm.tol;
    auto relaxed = [&](double rho) { return std::max(tol_req, std::min(1e-6, 0.1 * tol / std::max(rho, 1e-300))); };
    bool all_ok = true;
    for (int f0 = 0; f0 < n_fields; f0 += fc) {
        const int nf = std::min(fc, n_fields - f0);
        const size_t o = (size_t)f0 * w.V * 24;
        const double *eta = (const double *)eta_global_dev + o;
        double *x = (double *)chi_global_dev + o;
        const double *zu = ud + 2 * f0;
        const size_t bytes = (size_t)nf * w.V * 24 * sizeof(double);
        // r = b = eta on dPi; x = 0
        if ((st = wop_restrict(w, nf, one, eta, r)) != DD_OK) return st;
        HIPCHECK(ctx, hipMemsetAsync(x, 0, bytes, ctx->stream));
        std::vector<cplx> d;
        {
            const double *a[1] = {r}, *b[1] = {r};
            if ((st = wop_dots(w, nf, 1, a, b, d)) != DD_OK) return st;
        }
        std::vector<double> bn(nf), rr(nf, 1.0), rel(nf, 0.0);
        std::vector<int> live(nf), its(nf, 0), broke(nf, 0);
        for (int k = 0; k < nf; k++) {
            bn[k] = std::sqrt(d[k].real());
            live[k] = bn[k] > 0;
        }
        std::vector<cplx> cp(3 * nf), cs(3 * nf), cx(3 * nf), cr(3 * nf);
        int it = 0;
        for (int pass = 0; pass < 3; pass++) {
            // rh = r; p = v = 0
            HIPCHECK(ctx, hipMemcpyAsync(rh, r, bytes, hipMemcpyDeviceToDevice, ctx->stream));
            HIPCHECK(ctx, hipMemsetAsync(p, 0, bytes, ctx->stream));
            HIPCHECK(ctx, hipMemsetAsync(v, 0, bytes, ctx->stream));
            std::vector<cplx> rho(nf, 1.0), alpha(nf, 1.0), omega(nf, 1.0);
            while (it < maxit) {
                int nlive = 0;
                double rmax = 0;
                for (int k = 0; k < nf; k++)
                    if (live[k]) {
                        nlive++;
                        rmax = std::max(rmax, rr[k]);
                    }
                if (!nlive) break;
                it++;
                w.prm.tol = relaxed(rmax);
                {
                    const double *a[1] = {rh}, *b[1] = {r};
                    if ((st = wop_dots(w, nf, 1, a, b, d)) != DD_OK) return st;
                }
                for (int k = 0; k < nf; k++) {
                    cplx beta = 0;
                    if (live[k]) {
                        if (d[k] == 0.0) {
                            live[k] = 0;
                            broke[k] = 1;
                        } else {
                            beta = (d[k] / rho[k]) * (alpha[k] / omega[k]);
                            rho[k] = d[k];
                        }
                    }
                    // p = r + beta (p - omega v); a stopped field gets p = 0
                    cp[3 * k] = live[k] ? 1.0 : 0.0;
                    cp[3 * k + 1] = live[k] ? beta : 0.0;
                    cp[3 * k + 2] = live[k] ? -beta * omega[k] : 0.0;
                }
                if ((st = wop_lincomb(w, 0, nf, cp, r, p, v, p)) != DD_OK) return st;
                if ((st = wop_apply(w, nf, zu, p, v)) != DD_OK) return st;
                {
                    const double *a[1] = {rh}, *b[1] = {v};
                    if ((st = wop_dots(w, nf, 1, a, b, d)) != DD_OK) return st;
                }
                for (int k = 0; k < nf; k++) {
                    if (live[k]) {
                        if (d[k] == 0.0) {
                            live[k] = 0;
                            broke[k] = 1;
                        } else {
                            alpha[k] = rho[k] / d[k];
                        }
                    }
                    // s = r - alpha v (0 for a stopped field)
                    cs[3 * k] = live[k] ? 1.0 : 0.0;
                    cs[3 * k + 1] = live[k] ? -alpha[k] : 0.0;
                    cs[3 * k + 2] = 0.0;
                }
                if ((st = wop_lincomb(w, 1, nf, cs, r, v, nullptr, s)) != DD_OK) return st;
                if ((st = wop_apply(w, nf, zu, s, t)) != DD_OK) return st;
                {
                    const double *a[2] = {t, t}, *b[2] = {s, t};
                    if ((st = wop_dots(w, nf, 2, a, b, d)) != DD_OK) return st;
                }
                for (int k = 0; k < nf; k++) {
                    const cplx ts = d[2 * k], tt = d[2 * k + 1];
                    cplx om = 0;
                    if (live[k] && tt.real() > 0) om = ts / tt;
                    // x += alpha p + omega s;  r = s - omega t  (stopped fields keep both)
                    cx[3 * k] = 1.0;
                    cx[3 * k + 1] = live[k] ? alpha[k] : 0.0;
                    cx[3 * k + 2] = live[k] ? om : 0.0;
                    cr[3 * k] = live[k] ? 1.0 : 0.0;
                    cr[3 * k + 1] = live[k] ? -om : 0.0;
                    cr[3 * k + 2] = live[k] ? 0.0 : 1.0;
                    if (live[k]) {
                        if (om == 0.0 && tt.real() > 0) broke[k] = 1;
                        omega[k] = om;
                    }
                }
                if ((st = wop_lincomb(w, 2, nf, cx, x, p, s, x)) != DD_OK) return st;
                if ((st = wop_lincomb(w, 3, nf, cr, s, t, r, r)) != DD_OK) return st;
                {
                    const double *a[1] = {r}, *b[1] = {r};
                    if ((st = wop_dots(w, nf, 1, a, b, d)) != DD_OK) return st;
                }
                for (int k = 0; k < nf; k++) {
                    if (!live[k]) continue;
                    its[k] = it;
                    rr[k] = std::sqrt(std::max(d[k].real(), 0.0)) / bn[k];
                    if (rr[k] <= tol || omega[k] == 0.0) live[k] = 0;
                }
            }
            // true residual eta - W x on dPi, with the requested inner tolerance
            w.prm.tol = tol_req;
            if ((st = wop_restrict(w, nf, one, eta, s)) != DD_OK) return st;
            if ((st = wop_apply(w, nf, zu, x, t)) != DD_OK) return st;
            std::vector<cplx> c1(3 * nf);
            for (int k = 0; k < nf; k++) {
                c1[3 * k] = 1.0;
                c1[3 * k + 1] = -1.0;
                c1[3 * k + 2] = 0.0;
            }
            if ((st = wop_lincomb(w, 4, nf, c1, s, t, nullptr, s)) != DD_OK) return st;
            {
                const double *a[1] = {s}, *b[1] = {s};
                if ((st = wop_dots(w, nf, 1, a, b, d)) != DD_OK) return st;
            }
            bool again = false;
            for (int k = 0; k < nf; k++) {
                rel[k] = bn[k] > 0 ? std::sqrt(std::max(d[k].real(), 0.0)) / bn[k] : 0.0;
                live[k] = bn[k] > 0 && !broke[k] && rel[k] > tol;
                rr[k] = rel[k];
                again = again || live[k];
            }
            if (!again || it >= maxit) break;
            // restart the fields above tol from the true residual
            HIPCHECK(ctx, hipMemcpyAsync(r, s, bytes, hipMemcpyDeviceToDevice, ctx->stream));
        }
        for (int k = 0; k < nf; k++) {
            if (iters_host) iters_host[f0 + k] = its[k];
            if (relres_host) relres_host[f0 + k] = rel[k];
            if (!(rel[k] <= 10 * tol) || broke[k]) all_ok = false;
        }
    }
    HIPCHECK(ctx, hipStreamSynchronize(ctx->stream));
    wop_stats(w, stats);
    if (stats) stats->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (!all_ok || w.missed) {
        ctx->err = w.missed ? "some inner solves missed the tolerance"
                            : "some fields missed the tolerance (true residual above 10 tol or a breakdown)";
        return DD_ENOCONV;
    }
    return DD_OK;
}

extern "C" dd_status dd_mb_log_reweight(dd_ctx *ctx, const dd_blocks *B, const dd_gauge *G, const dd_blocks *D,
                                        const dd_gauge *GD, double kappa, int32_t N, double c, int32_t order,
                                        int32_t n_vec, const void *eta_global_dev, const dd_solve_params *params,
                                        double *terms_host, double *estimate_host, dd_solve_stats *stats)
{
    if (!ctx || !B || !G || !D || !GD || !eta_global_dev) return fail(ctx, DD_EINVAL, "null argument");
    if (N < 2 || (N & 1) || !(c > 0.0 && c < 1.0)) return fail(ctx, DD_EINVAL, "N must be even and 0 < c < 1");
    if (order < 1 || order > 64) return fail(ctx, DD_EINVAL, "order must be in 1..64");
    if (n_vec < 1 || n_vec > kMaxRhs) return fail(ctx, DD_EINVAL, "n_vec must be in 1..64");
    dd_status st = wop_check(ctx, B, G, D, GD);
    if (st != DD_OK) return st;
    HIPCHECK(ctx, enter(ctx));
    const auto tstart = std::chrono::steady_clock::now();
    dd_solve_params prm;
    if (params) prm = *params;
    else dd_solve_params_default(&prm);
    hipError_t e = hipSuccess;
    const int fc = wop_fields(ctx, B, D, prm, 5, n_vec, &e);
    if (fc < 1) return fail(ctx, DD_EDEVICE, hipGetErrorString(e));
    WOp w;
    if ((st = wop_init(w, ctx, B, G, D, GD, kappa, &prm, fc)) != DD_OK) return st;
    const size_t fl = (size_t)fc * w.V * 24 * sizeof(double);
    double *vec[5] = {};
    const char *names[5] = {"rw_e0", "rw_w", "rw_ta", "rw_tb", "rw_out"};
    for (int i = 0; i < 5; i++)
        if (!(vec[i] = (double *)workspace(ctx, names[i], fl, &e)))
            return fail(ctx, DD_ENOMEM, std::string("workspace: ") + hipGetErrorString(e));
    double *e0 = vec[0], *wv = vec[1], *ta = vec[2], *tb = vec[3], *wo = vec[4];
    double *zc = (double *)workspace(ctx, "rw_z", (size_t)kMaxRhs * 4 * sizeof(double), &e);
    if (!zc) return fail(ctx, DD_ENOMEM, std::string("workspace: ") + hipGetErrorString(e));
    double *zero = zc, *one = zc + 2 * kMaxRhs;
    {
        std::vector<double> h(4 * kMaxRhs, 0.0);
        for (int k = 0; k < kMaxRhs; k++) h[2 * kMaxRhs + 2 * k] = 1.0;
        HIPCHECK(ctx, hipMemcpyAsync(zc, h.data(), h.size() * sizeof(double), hipMemcpyHostToDevice, ctx->stream));
    }
    // T_{N+1}(1/c) by the three-term recurrence
    double tp = 1.0, tc = 1.0 / c;
    for (int j = 0; j < N; j++) {
        const double tn = 2.0 / c * tc - tp;
        tp = tc;
        tc = tn;
    }
    const double tnorm = tc;
    std::vector<cplx> terms(n_vec, 0.0);
    for (int f0 = 0; f0 < n_vec; f0 += fc) {
        const int nf = std::min(fc, n_vec - f0);
        const size_t bytes = (size_t)nf * w.V * 24 * sizeof(double);
        const double *eta = (const double *)eta_global_dev + (size_t)f0 * w.V * 24;
        if ((st = wop_restrict(w, nf, one, eta, e0)) != DD_OK) return st;
        HIPCHECK(ctx, hipMemcpyAsync(wv, e0, bytes, hipMemcpyDeviceToDevice, ctx->stream));
        std::vector<cplx> c1(3 * nf), c2(3 * nf), c3(3 * nf), d;
        for (int k = 0; k < nf; k++) {
            c1[3 * k] = -1.0 / c;  // t_1 = X t_0 = -W_0 t_0 / c
            c1[3 * k + 1] = c1[3 * k + 2] = 0.0;
            c2[3 * k] = -2.0 / c;  // t_{j+1} = 2 X t_j - t_{j-1}
            c2[3 * k + 1] = -1.0;
            c2[3 * k + 2] = 0.0;
            c3[3 * k] = 1.0 / tnorm;  // R y = T_{N+1}(X) y / T_{N+1}(1/c)
            c3[3 * k + 1] = c3[3 * k + 2] = 0.0;
        }
        for (int m = 1; m <= order; m++) {
            // ta = t_0 = w; tb = t_1
            HIPCHECK(ctx, hipMemcpyAsync(ta, wv, bytes, hipMemcpyDeviceToDevice, ctx->stream));
            if ((st = wop_apply(w, nf, zero, ta, wo)) != DD_OK) return st;
            if ((st = wop_lincomb(w, 0, nf, c1, wo, nullptr, nullptr, tb)) != DD_OK) return st;
            double *lo = ta, *hi = tb;
            for (int j = 1; j <= N; j++) {
                if ((st = wop_apply(w, nf, zero, hi, wo)) != DD_OK) return st;
                if ((st = wop_lincomb(w, 1 + (j & 1), nf, c2, wo, lo, nullptr, lo)) != DD_OK) return st;
                std::swap(lo, hi);
            }
            if ((st = wop_lincomb(w, 3, nf, c3, hi, nullptr, nullptr, wv)) != DD_OK) return st;
            const double *a[1] = {e0}, *b[1] = {wv};
            if ((st = wop_dots(w, nf, 1, a, b, d)) != DD_OK) return st;
            for (int k = 0; k < nf; k++) terms[f0 + k] -= d[k] / (double)m;
        }
    }
    cplx mean = 0;
    for (int j = 0; j < n_vec; j++) mean += terms[j];
    mean /= (double)n_vec;
    if (terms_host)
        for (int j = 0; j < n_vec; j++) {
            terms_host[2 * j] = terms[j].real();
            terms_host[2 * j + 1] = terms[j].imag();
        }
    if (estimate_host) {
        estimate_host[0] = mean.real();
        estimate_host[1] = mean.imag();
    }
    wop_stats(w, stats);
    if (stats) stats->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - tstart).count();
    if (w.missed) {
        ctx->err = "some inner solves missed the tolerance";
        return DD_ENOCONV;
    }
    return DD_OK;
}
