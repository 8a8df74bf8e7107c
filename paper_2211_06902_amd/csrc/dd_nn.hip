// Kernels of the learned block preconditioner: a 4D convolutional network
// (three 3^4 correlations, 24 -> 32 -> 32 -> 24 channels, zero padding at the
// block faces, no bias, identity or ReLU between layers) with its training
// (backward pass, relative squared error, Adam) in FP32.
//
// Activations are row-major [row][channel] with one row per (sample, block
// site), sites in box-local canonical order (x3 fastest): a tap of the
// correlation reads the neighbour's whole channel vector with vector loads.
// Weights are [tap][c_in][c_out] with tap = 27 (t0+1) + 9 (t1+1) + 3 (t2+1) +
// (t3+1); every thread of a kernel reads the same weight at the same time, so
// those loads are wave-uniform.
#include <hip/hip_runtime.h>

#include "dd_internal.h"

namespace dd {

namespace {

__device__ __forceinline__ void site_coords(int y, const NnExt &e, int c[4])
{
    c[3] = y % e.e[3];
    y /= e.e[3];
    c[2] = y % e.e[2];
    y /= e.e[2];
    c[1] = y % e.e[1];
    c[0] = y / e.e[1];
}

// Input transform applied on load: 0 as stored, 1 max(x, 0) (the activation
// of the previous layer), 2 x where the mask array is positive (else 0).
template <int MODE>
__device__ __forceinline__ float in_tf(float x, float m)
{
    if constexpr (MODE == 1) return fmaxf(x, 0.0f);
    else if constexpr (MODE == 2) return m > 0.0f ? x : 0.0f;
    else return x;
}

}  // namespace

// Y[row, o] = sum_t sum_c W[t, c, o] tf(X[row + t, c]); one thread per row.
template <int CIN, int COUT, int MODE>
__global__ void __launch_bounds__(256) k_conv(const float *__restrict__ X, const float *__restrict__ Msk,
                                              const float *__restrict__ W, float *__restrict__ Y, int64_t nrows,
                                              NnExt e)
{
    const int64_t row = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (row >= nrows) return;
    const int64_t n = row / e.S;
    const int y = (int)(row - n * e.S);
    int c[4];
    site_coords(y, e, c);
    float acc[COUT];
#pragma unroll
    for (int o = 0; o < COUT; o++) acc[o] = 0.0f;
    const int st[4] = {e.e[1] * e.e[2] * e.e[3], e.e[2] * e.e[3], e.e[3], 1};
    for (int t0 = -1; t0 <= 1; t0++) {
        if ((unsigned)(c[0] + t0) >= (unsigned)e.e[0]) continue;
        for (int t1 = -1; t1 <= 1; t1++) {
            if ((unsigned)(c[1] + t1) >= (unsigned)e.e[1]) continue;
            for (int t2 = -1; t2 <= 1; t2++) {
                if ((unsigned)(c[2] + t2) >= (unsigned)e.e[2]) continue;
#pragma unroll
                for (int t3 = -1; t3 <= 1; t3++) {
                    if ((unsigned)(c[3] + t3) >= (unsigned)e.e[3]) continue;
                    const int tap = ((t0 + 1) * 3 + (t1 + 1)) * 9 + (t2 + 1) * 3 + (t3 + 1);
                    const int64_t nb = n * e.S + y + t0 * st[0] + t1 * st[1] + t2 * st[2] + t3 * st[3];
                    const float4 *xr = reinterpret_cast<const float4 *>(X + nb * CIN);
                    const float4 *mr = reinterpret_cast<const float4 *>(Msk + (MODE == 2 ? nb * CIN : 0));
                    const float *wr = W + tap * CIN * COUT;
#pragma unroll
                    for (int q = 0; q < CIN / 4; q++) {
                        const float4 xv = xr[q];
                        float4 mv = make_float4(0, 0, 0, 0);
                        if constexpr (MODE == 2) mv = mr[q];
                        const float xs[4] = {in_tf<MODE>(xv.x, mv.x), in_tf<MODE>(xv.y, mv.y), in_tf<MODE>(xv.z, mv.z),
                                             in_tf<MODE>(xv.w, mv.w)};
#pragma unroll
                        for (int j = 0; j < 4; j++)
#pragma unroll
                            for (int o = 0; o < COUT; o++) acc[o] = __builtin_fmaf(xs[j], wr[(4 * q + j) * COUT + o], acc[o]);
                    }
                }
            }
        }
    }
    float4 *yr = reinterpret_cast<float4 *>(Y + row * COUT);
#pragma unroll
    for (int q = 0; q < COUT / 4; q++) yr[q] = make_float4(acc[4 * q], acc[4 * q + 1], acc[4 * q + 2], acc[4 * q + 3]);
}

// Partial weight gradients of one tap over one chunk of rows:
// part[chunk][tap][c][o] = sum_{rows r of the chunk} tf(X[r + tap, c]) dY[r, o].
template <int CIN, int COUT, int MODE>
__global__ void __launch_bounds__(256) k_conv_dw(const float *__restrict__ X, const float *__restrict__ Msk,
                                                 const float *__restrict__ dY, float *__restrict__ part,
                                                 int64_t nrows, int64_t rows_per_chunk, NnExt e)
{
    constexpr int R = 64;                       // rows staged at a time
    constexpr int KPT = (CIN * COUT + 255) / 256;  // accumulators per thread
    __shared__ float xs[R][CIN];
    __shared__ float ds[R][COUT];
    const int tap = blockIdx.x, chunk = blockIdx.y;
    const int t[4] = {tap / 27 - 1, (tap / 9) % 3 - 1, (tap / 3) % 3 - 1, tap % 3 - 1};
    const int st[4] = {e.e[1] * e.e[2] * e.e[3], e.e[2] * e.e[3], e.e[3], 1};
    const int64_t r0 = (int64_t)chunk * rows_per_chunk;
    const int64_t r1 = min(nrows, r0 + rows_per_chunk);
    float acc[KPT];
#pragma unroll
    for (int k = 0; k < KPT; k++) acc[k] = 0.0f;
    for (int64_t rb = r0; rb < r1; rb += R) {
        // stage R rows of dY and the matching neighbour rows of X (zero outside the block)
        for (int i = threadIdx.x; i < R * CIN; i += 256) {
            const int rr = i / CIN, cc = i - rr * CIN;
            const int64_t row = rb + rr;
            float v = 0.0f;
            if (row < r1) {
                const int64_t n = row / e.S;
                const int y = (int)(row - n * e.S);
                int c[4];
                site_coords(y, e, c);
                bool in = true;
#pragma unroll
                for (int m = 0; m < 4; m++) in = in && (unsigned)(c[m] + t[m]) < (unsigned)e.e[m];
                if (in) {
                    const int64_t nb = n * e.S + y + t[0] * st[0] + t[1] * st[1] + t[2] * st[2] + t[3] * st[3];
                    v = in_tf<MODE>(X[nb * CIN + cc], MODE == 2 ? Msk[nb * CIN + cc] : 0.0f);
                }
            }
            xs[rr][cc] = v;
        }
        for (int i = threadIdx.x; i < R * COUT; i += 256) {
            const int rr = i / COUT, oo = i - rr * COUT;
            const int64_t row = rb + rr;
            ds[rr][oo] = row < r1 ? dY[row * COUT + oo] : 0.0f;
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < KPT; k++) {
            const int idx = threadIdx.x + 256 * k;
            if (idx < CIN * COUT) {
                const int cc = idx / COUT, oo = idx - cc * COUT;
                float a = acc[k];
#pragma unroll 8
                for (int rr = 0; rr < R; rr++) a = __builtin_fmaf(xs[rr][cc], ds[rr][oo], a);
                acc[k] = a;
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int k = 0; k < KPT; k++) {
        const int idx = threadIdx.x + 256 * k;
        if (idx < CIN * COUT) part[((int64_t)chunk * 81 + tap) * CIN * COUT + idx] = acc[k];
    }
}

// out[k] = sum_j part[j][k] over nchunk chunks, in chunk order
__global__ void k_sum_chunks(const float *__restrict__ part, float *__restrict__ out, int64_t n, int nchunk)
{
    const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (k >= n) return;
    float s = 0.0f;
    for (int j = 0; j < nchunk; j++) s += part[(int64_t)j * n + k];
    out[k] = s;
}

// dZ = dH where the pre-activation Z is positive, else 0 (ReLU backward)
__global__ void k_relu_grad(const float *__restrict__ dH, const float *__restrict__ Z, float *__restrict__ dZ, int64_t n)
{
    const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (k < n) dZ[k] = Z[k] > 0.0f ? dH[k] : 0.0f;
}

// W'[t][o][c] = W[80 - t][c][o]: the weights of the transposed correlation
__global__ void k_flip_weights(const float *__restrict__ W, float *__restrict__ Wf, int cin, int cout)
{
    const int k = blockIdx.x * 256 + threadIdx.x;
    if (k >= 81 * cin * cout) return;
    const int t = k / (cin * cout), r = k - t * cin * cout, c = r / cout, o = r - c * cout;
    Wf[((int64_t)t * cout + o) * cin + c] = W[((int64_t)(80 - t) * cin + c) * cout + o];
}

// Training batch: X[i][s][:] = src rows of sample idx[i] (FP64 -> FP32), T likewise from sol.
__global__ void k_gather_rows(const double *__restrict__ src, const double *__restrict__ sol,
                              const int64_t *__restrict__ base, const int32_t *__restrict__ idx, float *__restrict__ X,
                              float *__restrict__ T, int n, int S)
{
    const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t per = (int64_t)S * 24;
    if (k >= (int64_t)n * per) return;
    const int i = (int)(k / per);
    const int64_t off = base[idx[i]] * 24 + (k - i * per);
    X[k] = (float)src[off];
    T[k] = (float)sol[off];
}

// Per-sample sums over the masked sites (global parity even, or all):
// part[i][chunk] = (sum |out - T|^2, sum |T|^2); one workgroup per (sample, chunk).
__global__ void __launch_bounds__(256) k_loss_parts(const float *__restrict__ out, const float *__restrict__ T,
                                                    const int32_t *__restrict__ opar, const int32_t *__restrict__ idx,
                                                    double *__restrict__ part, int mask_even, int nchunk, NnExt e)
{
    __shared__ double r0[4], r1[4];
    const int i = blockIdx.y, chunk = blockIdx.x;
    const int per = (e.S + nchunk - 1) / nchunk;
    const int s0 = chunk * per, s1 = min(e.S, s0 + per);
    const int op = opar[idx[i]];
    double a = 0, b = 0;
    for (int s = s0 + threadIdx.x; s < s1; s += 256) {
        int c[4];
        site_coords(s, e, c);
        if (mask_even && ((c[0] + c[1] + c[2] + c[3] + op) & 1)) continue;
        const int64_t o = ((int64_t)i * e.S + s) * 24;
        for (int ch = 0; ch < 24; ch++) {
            const double d = (double)out[o + ch] - (double)T[o + ch], tv = (double)T[o + ch];
            a += d * d;
            b += tv * tv;
        }
    }
    for (int off = 32; off >= 1; off >>= 1) {
        a += __shfl_xor(a, off, 64);
        b += __shfl_xor(b, off, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        r0[threadIdx.x >> 6] = a;
        r1[threadIdx.x >> 6] = b;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        part[((int64_t)i * nchunk + chunk) * 2] = ((r0[0] + r0[1]) + r0[2]) + r0[3];
        part[((int64_t)i * nchunk + chunk) * 2 + 1] = ((r1[0] + r1[1]) + r1[2]) + r1[3];
    }
}

// per-sample ratios num/den and the batch loss sum (one thread; n is a batch)
__global__ void k_loss_fin(const double *__restrict__ part, double *__restrict__ den, double *__restrict__ loss_acc,
                           int n, int nchunk)
{
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    double tot = 0;
    for (int i = 0; i < n; i++) {
        double a = 0, b = 0;
        for (int j = 0; j < nchunk; j++) {
            a += part[((int64_t)i * nchunk + j) * 2];
            b += part[((int64_t)i * nchunk + j) * 2 + 1];
        }
        den[i] = b;
        tot += b > 0 ? a / b : 0.0;
    }
    loss_acc[0] += tot / n;
    loss_acc[1] += 1.0;
}

// dOut = 2 mask (out - T) / (den_i n)
__global__ void k_loss_grad(const float *__restrict__ out, const float *__restrict__ T,
                            const int32_t *__restrict__ opar, const int32_t *__restrict__ idx,
                            const double *__restrict__ den, float *__restrict__ g, int n, int mask_even, NnExt e)
{
    const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t per = (int64_t)e.S * 24;
    if (k >= (int64_t)n * per) return;
    const int i = (int)(k / per);
    const int s = (int)((k - i * per) / 24);
    int c[4];
    site_coords(s, e, c);
    const bool on = !mask_even || !((c[0] + c[1] + c[2] + c[3] + opar[idx[i]]) & 1);
    g[k] = on && den[i] > 0 ? (float)(2.0 * ((double)out[k] - (double)T[k]) / (den[i] * n)) : 0.0f;
}

// Adam step t on n parameters
__global__ void k_adam(float *__restrict__ w, const float *__restrict__ g, float *__restrict__ m, float *__restrict__ v,
                       int64_t n, float lr, float b1, float b2, float eps, float c1, float c2)
{
    const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (k >= n) return;
    const float gk = g[k];
    const float mk = b1 * m[k] + (1.0f - b1) * gk;
    const float vk = b2 * v[k] + (1.0f - b2) * gk * gk;
    m[k] = mk;
    v[k] = vk;
    w[k] -= lr * (mk / c1) / (sqrtf(vk / c2) + eps);
}

// Network rows of pairs pair0 .. pair0 + npairs - 1 from an even half field in
// the library layout: the block's even sites carry the field, odd sites zero.
template <typename SP>
__global__ void k_half_to_rows(const SP *__restrict__ half, float *__restrict__ rows, HalfRows hr)
{
    const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (k >= (int64_t)hr.npairs * hr.S) return;
    const int pl = (int)(k / hr.S), q = (int)(k - (int64_t)pl * hr.S);
    const int pair = hr.pair0 + pl, b = pair % hr.nb, r = pair / hr.nb;
    const int hb = hr.h[b];
    const int s = hr.perm[hr.perm_off[b] + q];
    float v[24];
    if (q < hb) {
        const SP *src = half + (hr.soff[b] >> 1) * 24 * hr.n_rhs + (int64_t)r * 24 * hb + q;
#pragma unroll
        for (int c = 0; c < 24; c++) v[c] = (float)src[(int64_t)c * hb];
    } else {
#pragma unroll
        for (int c = 0; c < 24; c++) v[c] = 0.0f;
    }
    // a row is 96 contiguous bytes: six 16-byte stores
    float4 *row = reinterpret_cast<float4 *>(rows + ((int64_t)pl * hr.S + s) * 24);
#pragma unroll
    for (int i = 0; i < 6; i++) row[i] = make_float4(v[4 * i], v[4 * i + 1], v[4 * i + 2], v[4 * i + 3]);
}

// even sites of network rows back into an even half field
template <typename SP>
__global__ void k_rows_to_half(const float *__restrict__ rows, SP *__restrict__ half, HalfRows hr)
{
    const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (k >= (int64_t)hr.npairs * hr.S) return;
    const int pl = (int)(k / hr.S), q = (int)(k - (int64_t)pl * hr.S);
    const int pair = hr.pair0 + pl, b = pair % hr.nb, r = pair / hr.nb;
    const int hb = hr.h[b];
    if (q >= hb) return;
    const int s = hr.perm[hr.perm_off[b] + q];
    const float4 *row = reinterpret_cast<const float4 *>(rows + ((int64_t)pl * hr.S + s) * 24);
    float v[24];
#pragma unroll
    for (int i = 0; i < 6; i++) {
        const float4 t = row[i];
        v[4 * i] = t.x;
        v[4 * i + 1] = t.y;
        v[4 * i + 2] = t.z;
        v[4 * i + 3] = t.w;
    }
    SP *dst = half + (hr.soff[b] >> 1) * 24 * hr.n_rhs + (int64_t)r * 24 * hb + q;
#pragma unroll
    for (int c = 0; c < 24; c++) dst[(int64_t)c * hb] = (SP)v[c];
}

// ------------------------------------------------- BF16 matrix-core inference
//
// Implicit GEMM per tap: for the 81 offsets t, Y[rows, :] += X[rows + t, :] W[t]
// with K = 32 input channels per tap (zero padded), N = 32 output channels and
// the rows of a wavefront in tiles of 16; v_mfma_f32_16x16x32_bf16 multiplies a
// 16 x 32 tile of neighbour rows by the tap's 32 x 16 weight block with FP32
// accumulation.  Lane l supplies row (l mod 16) of A and column (l mod 16) of B,
// each with the 8 consecutive channels 8 (l / 16) .. 8 (l / 16) + 7 (16 bytes);
// it receives rows 4 (l / 16) .. 4 (l / 16) + 3 of column (l mod 16) of the
// 16 x 16 product.

typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(4))) float f32x4;

__device__ __forceinline__ uint16_t f2bf(float f)
{
    const uint32_t u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)(((u >> 16) & 0x8000u) | 0x7fc0u);
    return (uint16_t)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}

// Y = act(conv(X, W)): X [rows][32] BF16, Wt [81][32 out][32 in] BF16;
// OUT_F32: Y [rows][24] FP32 (last layer), else [rows][32] BF16 after ACT.
// A wavefront computes 64 rows x 32 channels; a workgroup 256 rows.
template <int ACT, bool OUT_F32>
__global__ void __launch_bounds__(256) k_conv_mfma(const uint16_t *__restrict__ X, const uint16_t *__restrict__ Wt,
                                                   void *__restrict__ Y, int64_t nrows, NnExt e)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t row0 = ((int64_t)blockIdx.x * 4 + wave) * 64;
    if (row0 >= nrows) return;
    const int kg = lane >> 4, li = lane & 15;
    const int st[4] = {e.e[1] * e.e[2] * e.e[3], e.e[2] * e.e[3], e.e[3], 1};
    int64_t arow[4];
    int ac[4][4];
    bool alive[4];
#pragma unroll
    for (int rt = 0; rt < 4; rt++) {
        arow[rt] = row0 + rt * 16 + li;
        alive[rt] = arow[rt] < nrows;
        const int64_t n = arow[rt] / e.S;
        site_coords((int)(arow[rt] - n * e.S), e, ac[rt]);
    }
    f32x4 acc[4][2];
#pragma unroll
    for (int rt = 0; rt < 4; rt++)
#pragma unroll
        for (int ct = 0; ct < 2; ct++) acc[rt][ct] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    const bf16x8 zero = {};
    for (int tap = 0; tap < 81; tap++) {
        const int t0 = tap / 27 - 1, t1 = (tap / 9) % 3 - 1, t2 = (tap / 3) % 3 - 1, t3 = tap % 3 - 1;
        const int off = t0 * st[0] + t1 * st[1] + t2 * st[2] + t3 * st[3];
        bf16x8 bv[2];
#pragma unroll
        for (int ct = 0; ct < 2; ct++)
            bv[ct] = *reinterpret_cast<const bf16x8 *>(Wt + ((int64_t)(tap * 32 + ct * 16 + li) * 32 + kg * 8));
        bf16x8 av[4];
#pragma unroll
        for (int rt = 0; rt < 4; rt++) {
            const bool in = alive[rt] && (unsigned)(ac[rt][0] + t0) < (unsigned)e.e[0] &&
                            (unsigned)(ac[rt][1] + t1) < (unsigned)e.e[1] &&
                            (unsigned)(ac[rt][2] + t2) < (unsigned)e.e[2] && (unsigned)(ac[rt][3] + t3) < (unsigned)e.e[3];
            av[rt] = in ? *reinterpret_cast<const bf16x8 *>(X + (arow[rt] + off) * 32 + kg * 8) : zero;
        }
#pragma unroll
        for (int rt = 0; rt < 4; rt++)
#pragma unroll
            for (int ct = 0; ct < 2; ct++)
                acc[rt][ct] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[rt], bv[ct], acc[rt][ct], 0, 0, 0);
    }
#pragma unroll
    for (int rt = 0; rt < 4; rt++)
#pragma unroll
        for (int ct = 0; ct < 2; ct++)
#pragma unroll
            for (int i = 0; i < 4; i++) {
                const int64_t r = row0 + rt * 16 + 4 * kg + i;
                const int col = ct * 16 + li;
                if (r >= nrows) continue;
                float v = acc[rt][ct][i];
                if constexpr (OUT_F32) {
                    if (col < 24) reinterpret_cast<float *>(Y)[r * 24 + col] = v;
                } else {
                    if (ACT) v = fmaxf(v, 0.0f);
                    reinterpret_cast<uint16_t *>(Y)[r * 32 + col] = f2bf(v);
                }
            }
}

// The same layer with the input staged in LDS: one workgroup per block walks its
// x0-slices, keeping the three input slices x0 - 1, x0, x0 + 1 in a ring of LDS
// buffers (rows padded to 80 bytes against bank conflicts; slices outside the
// block are zero), so every input row is read from HBM once per layer and the
// 81 taps read their neighbour rows from LDS.  Needs e1 e2 e3 <= 512.
//
// PAR = 0: wave w computes output rows 64 w .. 64 w + 63 of the slice.
// PAR = 1, 2 (the solver's even half fields, blocks of even extents): rows
// are taken by parity class (y1 + y2 + y3 even or odd), waves 0..3 the even
// class and 4..7 the odd one, so that the global parity of a wave's rows is
// one value per slice.  PAR = 1: the input is zero on odd sites, so only the
// taps reaching even sites are multiplied (41 or 40 of 81).  PAR = 2: only
// the even output sites are needed, so the waves whose class is odd in a
// slice skip it (spreading the even rows over all waves, two tiles each, was
// measured slower: each weight fragment then feeds half as many products).
// The skipped products are exact zeros or unused rows: the results of the
// rows kept are the same.  PAR = 3 (first layer) reads its input from the
// FP32 even half field, PAR = 4 (last layer) writes its even output sites
// into the FP32 even half field hin.out, both instead of network rows.
// origin: the block origins [nb][4] (global parity of a site = parity of
// origin + local coordinates).
constexpr int kSliceMax = 512;
constexpr int kRowPad = 40;     // bf16 per LDS row (32 + 8 padding)
constexpr int kTrStride = 257;  // floats per channel of the PAR = 4 transpose (odd: no bank conflicts)
static_assert(24 * kTrStride * 4 <= kSliceMax * kRowPad * 2, "transpose fits a ring buffer");

template <int ACT, bool OUT_F32, int PAR>
__global__ void __launch_bounds__(512) k_conv_mfma_lds(const uint16_t *__restrict__ X, const uint16_t *__restrict__ Wt,
                                                       void *__restrict__ Y, NnExt e, const int32_t *__restrict__ active,
                                                       int pair0, const int32_t *__restrict__ origin, int nb, NnHalfIn hin)
{
    __shared__ uint16_t ring[3][kSliceMax][kRowPad];
    // blocks whose (block, rhs) pair is no longer iterated are skipped
    if (active && !active[pair0 + (int)blockIdx.x]) return;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int kg = lane >> 4, li = lane & 15;
    const int R = e.e[1] * e.e[2] * e.e[3];
    const int64_t base = (int64_t)blockIdx.x * e.S;  // first row of this block
    constexpr int RT = 4;  // 16-row tiles per wavefront
    // parity class of the wave's rows and the parity of the block origin
    const int cls = PAR ? wave >> 2 : 0;
    int opar = 0;
    if constexpr (PAR != 0) {
        const int32_t *o = origin + 4 * ((pair0 + (int)blockIdx.x) % nb);
        opar = (o[0] + o[1] + o[2] + o[3]) & 1;
    }
    // output coordinates (x1, x2, x3) and slice row of this lane's row in each
    // 16-row tile; for PAR != 0 the row is the j-th of its parity class (line
    // (y1, y2), y3 = 2 m + ((class + y1 + y2) & 1)), and x3 is set per slice
    int oc[RT][3], orw[RT], om[RT];
    bool orow[RT];
#pragma unroll
    for (int rt = 0; rt < RT; rt++) {
        if constexpr (PAR == 0) {
            int r = wave * 64 + rt * 16 + li;
            orow[rt] = r < R;
            r = min(r, R - 1);
            orw[rt] = r;
            oc[rt][2] = r % e.e[3];
            r /= e.e[3];
            oc[rt][1] = r % e.e[2];
            oc[rt][0] = r / e.e[2];
            om[rt] = 0;
        } else {
            const int h3 = e.e[3] >> 1;
            int j = (wave & 3) * 64 + rt * 16 + li;
            orow[rt] = j < (R >> 1);
            j = min(j, (R >> 1) - 1);
            om[rt] = j % h3;
            const int line = j / h3;
            oc[rt][1] = line % e.e[2];
            oc[rt][0] = line / e.e[2];
            oc[rt][2] = 0;
            orw[rt] = 0;
        }
    }
    // x3 and the slice row of the class-cl rows (PAR != 0)
    auto set_class = [&](int cl) {
#pragma unroll
        for (int rt = 0; rt < RT; rt++) {
            oc[rt][2] = 2 * om[rt] + ((cl + oc[rt][0] + oc[rt][1]) & 1);
            orw[rt] = (oc[rt][0] * e.e[2] + oc[rt][1]) * e.e[3] + oc[rt][2];
        }
    };
    if constexpr (PAR != 0) set_class(cls);
    // slice s into registers (zero outside the block) and from there into its
    // ring buffer.  PAR = 3: from the even half field (FP32, component-major):
    // thread t takes even site t % 256 of the slice and components
    // 12 (t / 256) .. + 11, converts them to BF16 into the site's row and
    // zeroes the same channels of the odd row next to it (rows 2m, 2m + 1 of
    // the block hold one even site each).  Else: 4 pieces of 16 bytes of the
    // BF16 rows per thread.
    const float *hbase = nullptr;
    const int32_t *pm = nullptr;
    int hbk = 0, pb = 0, prhs = 0;
    if constexpr (PAR >= 3) {
        const int pair = pair0 + (int)blockIdx.x;
        pb = pair % nb;
        prhs = pair / nb;
        hbk = hin.h[pb];
        hbase = hin.half + (hin.soff[pb] >> 1) * 24 * hin.n_rhs + (int64_t)prhs * 24 * hbk;
        pm = hin.perm + hin.perm_off[pb];
    }
    struct Pre {
        uint4 u[4];
        float f[12];
        int row;
    };
    auto fetch_slice = [&](int s, Pre &pre) {
        const bool in = s >= 0 && s < e.e[0];
        if constexpr (PAR == 3) {
            const int ql = threadIdx.x & 255, g = threadIdx.x >> 8, hs = R >> 1;
            pre.row = -1;
#pragma unroll
            for (int i = 0; i < 12; i++) pre.f[i] = 0.0f;
            if (in && ql < hs) {
                const int q = s * hs + ql;
                pre.row = pm[q] - s * R;
#pragma unroll
                for (int i = 0; i < 12; i++) pre.f[i] = hbase[(int64_t)(g * 12 + i) * hbk + q];
            }
        } else {
#pragma unroll
            for (int i = 0; i < 4; i++) {
                const int k = threadIdx.x + 512 * i;
                pre.u[i] = make_uint4(0, 0, 0, 0);
                if (in && k < R * 4)
                    pre.u[i] = *reinterpret_cast<const uint4 *>(X + (base + (int64_t)s * R + (k >> 2)) * 32 + (k & 3) * 8);
            }
        }
    };
    auto put_slice = [&](int s, const Pre &pre) {
        uint16_t(*dst)[kRowPad] = ring[(s + 3) % 3];
        if constexpr (PAR == 3) {
            const bool in = s >= 0 && s < e.e[0];
            if (!in) {
                for (int k = threadIdx.x; k < R * 4; k += 512)
                    *reinterpret_cast<uint4 *>(&dst[k >> 2][(k & 3) * 8]) = make_uint4(0, 0, 0, 0);
            } else if (pre.row >= 0) {
                const int g = threadIdx.x >> 8;
                uint2 *ev = reinterpret_cast<uint2 *>(&dst[pre.row][g * 12]);
                uint2 *od = reinterpret_cast<uint2 *>(&dst[pre.row ^ 1][g * 12]);
#pragma unroll
                for (int i = 0; i < 3; i++) {
                    ev[i] = make_uint2((uint32_t)f2bf(pre.f[4 * i]) | ((uint32_t)f2bf(pre.f[4 * i + 1]) << 16),
                                       (uint32_t)f2bf(pre.f[4 * i + 2]) | ((uint32_t)f2bf(pre.f[4 * i + 3]) << 16));
                    od[i] = make_uint2(0, 0);
                }
                if (g == 1) {  // padding channels 24..31 of both rows
                    *reinterpret_cast<uint4 *>(&dst[pre.row][24]) = make_uint4(0, 0, 0, 0);
                    *reinterpret_cast<uint4 *>(&dst[pre.row ^ 1][24]) = make_uint4(0, 0, 0, 0);
                }
            }
        } else {
#pragma unroll
            for (int i = 0; i < 4; i++) {
                const int k = threadIdx.x + 512 * i;
                if (k < R * 4) *reinterpret_cast<uint4 *>(&dst[k >> 2][(k & 3) * 8]) = pre.u[i];
            }
        }
    };
    {
        Pre pre;
        fetch_slice(-1, pre);
        put_slice(-1, pre);
        fetch_slice(0, pre);
        put_slice(0, pre);
        fetch_slice(1, pre);
        put_slice(1, pre);
    }
    __syncthreads();
    const bf16x8 zero = {};
    for (int a = 0; a < e.e[0]; a++) {
        // slice a + 2 is fetched during the products of slice a
        Pre pre;
        fetch_slice(a + 2, pre);
        // global parity of this wave's output rows in slice a
        const int gpar = (opar + a + cls) & 1;
        const bool work = (PAR != 2 && PAR != 4) || gpar == 0;
        f32x4 acc[RT][2];
#pragma unroll
        for (int rt = 0; rt < RT; rt++)
#pragma unroll
            for (int ct = 0; ct < 2; ct++) acc[rt][ct] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
        if (work)
        for (int t0 = -1; t0 <= 1; t0++) {
            const uint16_t(*src)[kRowPad] = ring[(a + t0 + 3) % 3];
            for (int t1 = -1; t1 <= 1; t1++)
                for (int t2 = -1; t2 <= 1; t2++) {
#pragma unroll
                    for (int t3 = -1; t3 <= 1; t3++) {
                        // PAR = 1: the tap reaches an odd (zero) input site
                        if ((PAR == 1 || PAR == 3) && ((gpar + t0 + t1 + t2 + t3) & 1)) continue;
                        const int tap = ((t0 + 1) * 3 + (t1 + 1)) * 9 + (t2 + 1) * 3 + (t3 + 1);
                        bf16x8 bv[2];
#pragma unroll
                        for (int ct = 0; ct < 2; ct++)
                            bv[ct] = *reinterpret_cast<const bf16x8 *>(Wt + ((int64_t)(tap * 32 + ct * 16 + li) * 32 + kg * 8));
                        bf16x8 av[RT];
#pragma unroll
                        for (int rt = 0; rt < RT; rt++) {
                            const int y1 = oc[rt][0] + t1, y2 = oc[rt][1] + t2, y3 = oc[rt][2] + t3;
                            const bool in = orow[rt] && (unsigned)y1 < (unsigned)e.e[1] &&
                                            (unsigned)y2 < (unsigned)e.e[2] && (unsigned)y3 < (unsigned)e.e[3];
                            const int r = in ? (y1 * e.e[2] + y2) * e.e[3] + y3 : 0;
                            av[rt] = in ? *reinterpret_cast<const bf16x8 *>(&src[r][kg * 8]) : zero;
                        }
#pragma unroll
                        for (int rt = 0; rt < RT; rt++)
#pragma unroll
                            for (int ct = 0; ct < 2; ct++)
                                acc[rt][ct] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[rt], bv[ct], acc[rt][ct], 0, 0, 0);
                    }
                }
        }
        if constexpr (PAR == 4) {
            // even output sites straight into the FP32 half field: the tile goes
            // through LDS (the ring buffer slice a + 2 will fill, free now) so
            // that the global stores run along the sites.  Even row j of the
            // slice is its even site j.
            __syncthreads();  // every wave is done with slice a - 1
            float *tr = reinterpret_cast<float *>(&ring[(a + 2) % 3][0][0]);
            if (work)
#pragma unroll
                for (int rt = 0; rt < RT; rt++)
#pragma unroll
                    for (int ct = 0; ct < 2; ct++) {
                        const int c = ct * 16 + li;
#pragma unroll
                        for (int i = 0; i < 4; i++) {
                            const int j = (wave & 3) * 64 + rt * 16 + 4 * kg + i;
                            if (c < 24 && j < (R >> 1)) tr[c * kTrStride + j] = acc[rt][ct][i];
                        }
                    }
            __syncthreads();
            float *zb = hin.out + (hin.soff[pb] >> 1) * 24 * hin.n_rhs + (int64_t)prhs * 24 * hbk + a * (R >> 1);
            for (int k = threadIdx.x; k < 24 * (R >> 1); k += 512) {
                const int c = k / (R >> 1), j = k - c * (R >> 1);
                zb[(int64_t)c * hbk + j] = tr[c * kTrStride + j];
            }
        }
        // store this slice's output rows
        if (PAR != 4 && work)
#pragma unroll
        for (int rt = 0; rt < RT; rt++)
#pragma unroll
            for (int ct = 0; ct < 2; ct++)
#pragma unroll
                for (int i = 0; i < 4; i++) {
                    // accumulator element i of lane (kg, li) is row 4 kg + i, column li of the tile
                    const int src_lane = 4 * kg + i;
                    const int r = __shfl(orw[rt], src_lane, 64);
                    const bool live = __shfl((int)orow[rt], src_lane, 64) != 0;
                    const int col = ct * 16 + li;
                    if (!live) continue;
                    const int64_t row = base + (int64_t)a * R + r;
                    float v = acc[rt][ct][i];
                    if constexpr (OUT_F32) {
                        if (col < 24) reinterpret_cast<float *>(Y)[row * 24 + col] = v;
                    } else {
                        if (ACT) v = fmaxf(v, 0.0f);
                        reinterpret_cast<uint16_t *>(Y)[row * 32 + col] = f2bf(v);
                    }
                }
        __syncthreads();  // every wave is done with slice a - 1 (PAR = 4: and the transpose)
        if (a + 2 <= e.e[0]) put_slice(a + 2, pre);
        __syncthreads();
    }
}

// Wt[t][o][c] = bf16(W[t][c][o]) for o < cout, c < cin; 0 elsewhere (32 x 32 per tap)
__global__ void k_weights_bf16(const float *__restrict__ W, uint16_t *__restrict__ Wt, int cin, int cout)
{
    const int k = blockIdx.x * 256 + threadIdx.x;
    if (k >= 81 * 32 * 32) return;
    const int t = k / 1024, o = (k / 32) % 32, c = k % 32;
    Wt[k] = (o < cout && c < cin) ? f2bf(W[((int64_t)t * cin + c) * cout + o]) : (uint16_t)0;
}

// network rows in BF16 (32 channels, 24..31 zero) from an even half field
template <typename SP>
__global__ void k_half_to_rows_bf16(const SP *__restrict__ half, uint16_t *__restrict__ rows, HalfRows hr)
{
    // thread k: canonical rows 2 m and 2 m + 1 of one pair's block; with even
    // extents exactly one of them is even, and it is the m-th even site
    const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int hS = hr.S >> 1;
    if (k >= (int64_t)hr.npairs * hS) return;
    const int pl = (int)(k / hS), m = (int)(k - (int64_t)pl * hS);
    const int pair = hr.pair0 + pl, b = pair % hr.nb, r = pair / hr.nb;
    const int hb = hr.h[b];
    const int s = hr.perm[hr.perm_off[b] + m];  // 2 m or 2 m + 1
    uint32_t pk[16];  // channel pairs (2c, 2c+1), low half first
#pragma unroll
    for (int i = 0; i < 16; i++) pk[i] = 0;
    const SP *src = half + (hr.soff[b] >> 1) * 24 * hr.n_rhs + (int64_t)r * 24 * hb + m;
#pragma unroll
    for (int c = 0; c < 12; c++)
        pk[c] = (uint32_t)f2bf((float)src[(int64_t)(2 * c) * hb]) | ((uint32_t)f2bf((float)src[(int64_t)(2 * c + 1) * hb]) << 16);
    // the two rows are 128 contiguous bytes: eight 16-byte stores
    uint4 *row = reinterpret_cast<uint4 *>(rows + ((int64_t)pl * hr.S + 2 * m) * 32);
    const bool first = s == 2 * m;
    const uint4 z = make_uint4(0, 0, 0, 0);
#pragma unroll
    for (int i = 0; i < 4; i++) {
        const uint4 v = make_uint4(pk[4 * i], pk[4 * i + 1], pk[4 * i + 2], pk[4 * i + 3]);
        row[i] = first ? v : z;
        row[4 + i] = first ? z : v;
    }
}

// FP32 rows [rows][24] -> BF16 rows [rows][32]
__global__ void k_rows_f32_to_bf16(const float *__restrict__ X, uint16_t *__restrict__ Xb, int64_t nrows)
{
    const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (k >= nrows * 32) return;
    const int64_t r = k / 32;
    const int c = (int)(k - r * 32);
    Xb[k] = c < 24 ? f2bf(X[r * 24 + c]) : (uint16_t)0;
}

// ------------------------------------------------------------ launchers



static inline dim3 g256(int64_t n) { return dim3((unsigned)((n + 255) / 256)); }

hipError_t launch_conv(const float *X, const float *W, float *Y, int64_t nrows, const NnExt &e, int cin, int cout,
                       int mode, hipStream_t st)
{
    if (nrows <= 0) return hipSuccess;
#define CV(CI, CO, M)                                                                                              \
    if (cin == CI && cout == CO && mode == M) {                                                                  \
        hipLaunchKernelGGL((k_conv<CI, CO, M>), g256(nrows), dim3(256), 0, st, X, nullptr, W, Y, nrows, e);     \
        return hipGetLastError();                                                                                \
    }
    CV(24, 32, 0) CV(32, 32, 0) CV(32, 32, 1) CV(32, 24, 0) CV(32, 24, 1)
#undef CV
    return hipErrorInvalidValue;
}

hipError_t launch_conv_dw(const float *X, const float *dY, float *part, float *dW, int64_t nrows, int nchunk,
                          const NnExt &e, int cin, int cout, int mode, hipStream_t st)
{
    const int64_t per = (nrows + nchunk - 1) / nchunk;
    dim3 g(81, nchunk);
    bool ok = false;
#define DW(CI, CO, M)                                                                                            \
    if (!ok && cin == CI && cout == CO && mode == M) {                                                         \
        hipLaunchKernelGGL((k_conv_dw<CI, CO, M>), g, dim3(256), 0, st, X, nullptr, dY, part, nrows, per, e); \
        ok = true;                                                                                             \
    }
    DW(24, 32, 0) DW(32, 32, 0) DW(32, 32, 1) DW(32, 24, 0) DW(32, 24, 1)
#undef DW
    if (!ok) return hipErrorInvalidValue;
    const int64_t n = 81LL * cin * cout;
    hipLaunchKernelGGL(k_sum_chunks, g256(n), dim3(256), 0, st, part, dW, n, nchunk);
    return hipGetLastError();
}

hipError_t launch_relu_grad(const float *dH, const float *Z, float *dZ, int64_t n, hipStream_t st)
{
    hipLaunchKernelGGL(k_relu_grad, g256(n), dim3(256), 0, st, dH, Z, dZ, n);
    return hipGetLastError();
}

hipError_t launch_flip_weights(const float *W, float *Wf, int cin, int cout, hipStream_t st)
{
    hipLaunchKernelGGL(k_flip_weights, g256(81LL * cin * cout), dim3(256), 0, st, W, Wf, cin, cout);
    return hipGetLastError();
}

hipError_t launch_gather_rows(const double *src, const double *sol, const int64_t *base, const int32_t *idx, float *X,
                              float *T, int n, int S, hipStream_t st)
{
    hipLaunchKernelGGL(k_gather_rows, g256((int64_t)n * S * 24), dim3(256), 0, st, src, sol, base, idx, X, T, n, S);
    return hipGetLastError();
}

hipError_t launch_loss(const float *out, const float *T, const int32_t *opar, const int32_t *idx, double *part,
                       double *den, double *loss_acc, float *grad, int n, int mask_even, const NnExt &e,
                       hipStream_t st)
{
    constexpr int nchunk = 16;
    hipLaunchKernelGGL(k_loss_parts, dim3(nchunk, n), dim3(256), 0, st, out, T, opar, idx, part, mask_even, nchunk, e);
    hipLaunchKernelGGL(k_loss_fin, dim3(1), dim3(64), 0, st, part, den, loss_acc, n, nchunk);
    if (grad)
        hipLaunchKernelGGL(k_loss_grad, g256((int64_t)n * e.S * 24), dim3(256), 0, st, out, T, opar, idx, den, grad, n,
                           mask_even, e);
    return hipGetLastError();
}

hipError_t launch_half_rows(const void *half, float *rows, void *half_out, dd_prec sp, const HalfRows &hr, int dir,
                            hipStream_t st)
{
    const dim3 g = g256((int64_t)hr.npairs * hr.S);
    if (dir == 0) {
        if (sp == DD_F64) hipLaunchKernelGGL(k_half_to_rows<double>, g, dim3(256), 0, st, (const double *)half, rows, hr);
        else hipLaunchKernelGGL(k_half_to_rows<float>, g, dim3(256), 0, st, (const float *)half, rows, hr);
    } else {
        if (sp == DD_F64) hipLaunchKernelGGL(k_rows_to_half<double>, g, dim3(256), 0, st, rows, (double *)half_out, hr);
        else hipLaunchKernelGGL(k_rows_to_half<float>, g, dim3(256), 0, st, rows, (float *)half_out, hr);
    }
    return hipGetLastError();
}

hipError_t launch_conv_mfma(const uint16_t *X, const uint16_t *Wt, void *Y, int64_t nrows, const NnExt &e, int act,
                            bool out_f32, int variant, const int32_t *active, int pair0, const int32_t *origin, int nb,
                            int parity_mode, hipStream_t st, const NnHalfIn *hin)
{
    if (nrows <= 0) return hipSuccess;
    const int R = e.e[1] * e.e[2] * e.e[3];
    // the parity modes need even e3 (rows of one class per line) and the block origins
    const int par = origin && (e.e[3] & 1) == 0 ? parity_mode : 0;
    if (par == 3 && (!hin || variant != 1 || out_f32 || R > kSliceMax || nrows % e.S != 0)) return hipErrorInvalidValue;
    if (par == 4 && (!hin || !hin->out || variant != 1 || !out_f32 || R > kSliceMax || nrows % e.S != 0))
        return hipErrorInvalidValue;
    if (R <= kSliceMax && nrows % e.S == 0 && variant == 1) {
        const dim3 g((unsigned)(nrows / e.S)), t(512);
        const NnHalfIn h0 = hin ? *hin : NnHalfIn{};
#define CM(A, F, P) hipLaunchKernelGGL((k_conv_mfma_lds<A, F, P>), g, t, 0, st, X, Wt, Y, e, active, pair0, origin, nb, h0)
        if (out_f32) {
            if (par == 4) CM(0, true, 4); else if (par == 2) CM(0, true, 2); else CM(0, true, 0);
        } else if (act) {
            if (par == 3) CM(1, false, 3); else if (par == 1) CM(1, false, 1); else CM(1, false, 0);
        } else {
            if (par == 3) CM(0, false, 3); else if (par == 1) CM(0, false, 1); else CM(0, false, 0);
        }
#undef CM
        return hipGetLastError();
    }
    const dim3 g((unsigned)((nrows + 255) / 256));
    if (out_f32) hipLaunchKernelGGL((k_conv_mfma<0, true>), g, dim3(256), 0, st, X, Wt, Y, nrows, e);
    else if (act) hipLaunchKernelGGL((k_conv_mfma<1, false>), g, dim3(256), 0, st, X, Wt, Y, nrows, e);
    else hipLaunchKernelGGL((k_conv_mfma<0, false>), g, dim3(256), 0, st, X, Wt, Y, nrows, e);
    return hipGetLastError();
}

hipError_t launch_weights_bf16(const float *W, uint16_t *Wt, int cin, int cout, hipStream_t st)
{
    hipLaunchKernelGGL(k_weights_bf16, g256(81 * 32 * 32), dim3(256), 0, st, W, Wt, cin, cout);
    return hipGetLastError();
}

hipError_t launch_half_rows_bf16(const void *half, uint16_t *rows, dd_prec sp, const HalfRows &hr, hipStream_t st)
{
    if (hr.S & 1) return hipErrorInvalidValue;
    const dim3 g = g256((int64_t)hr.npairs * (hr.S >> 1));
    if (sp == DD_F64) hipLaunchKernelGGL(k_half_to_rows_bf16<double>, g, dim3(256), 0, st, (const double *)half, rows, hr);
    else hipLaunchKernelGGL(k_half_to_rows_bf16<float>, g, dim3(256), 0, st, (const float *)half, rows, hr);
    return hipGetLastError();
}

hipError_t launch_rows_f32_to_bf16(const float *X, uint16_t *Xb, int64_t nrows, hipStream_t st)
{
    hipLaunchKernelGGL(k_rows_f32_to_bf16, g256(nrows * 32), dim3(256), 0, st, X, Xb, nrows);
    return hipGetLastError();
}

hipError_t launch_adam(float *w, const float *g, float *m, float *v, int64_t n, float lr, float b1, float b2, float eps,
                       int t, hipStream_t st)
{
    const float c1 = 1.0f - powf(b1, (float)t), c2 = 1.0f - powf(b2, (float)t);
    hipLaunchKernelGGL(k_adam, g256(n), dim3(256), 0, st, w, g, m, v, n, lr, b1, b2, eps, c1, c2);
    return hipGetLastError();
}

}  // namespace dd
