// HIP kernels of libdd for gfx950.
//
// Data layout (device, library-owned):
//   half field  (one parity of a spinor field, all blocks, all rhs):
//       element (block b, component c in 0..23, eo site h, rhs r) at
//       (soff[b]/2)*24*n_rhs + c*(h_b*n_rhs) + h*n_rhs + r
//     i.e. per block a component-major structure of arrays whose innermost
//     index is the right-hand side.  A wavefront reading one component of
//     consecutive (site, rhs) items touches consecutive addresses, and all
//     right-hand sides of a site sit next to each other, so one link load
//     serves every rhs of the site in the same instruction.
//     Component c = 2*(3*spin + colour) + {0: re, 1: im}.
//   links: [block site slot (eo order, even sites first)][mu][3][3][re,im],
//     the forward link U_mu(x) of every block site; links that leave the
//     block are stored as zero and never read.
//   neighbour table per block shape: [parity][h][8] int32, entries
//     2*mu = x+mu, 2*mu+1 = x-mu as the eo index inside the other parity,
//     -1 if the hop is dropped (Dirichlet), bit 30 set if the hop crosses
//     the antiperiodic time edge.
//
// Work decomposition of every site kernel: one workgroup of kTile threads
// handles kTile consecutive (site, rhs) items of one block ("tile").  Tiles
// are numbered block after block; the launch index is remapped so that
// consecutive tiles go to the same XCD (the hardware deals workgroups to the
// 8 XCDs round-robin), keeping a block's neighbour reads in one L2.
#include <hip/hip_runtime.h>

#include "dd_internal.h"

namespace dd {

// ------------------------------------------------------------- helpers

__device__ __forceinline__ int xcd_tile(int bid, int n)
{
    const int q = n >> 3, rem = n & 7, k = bid & 7, j = bid >> 3;
    return k * q + min(k, rem) + j;
}

__device__ __forceinline__ uint16_t f32_to_bf16_rne(float f)
{
    const uint32_t u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)(((u >> 16) & 0x8000u) | 0x7fc0u);
    const uint32_t lsb = (u >> 16) & 1u;
    return (uint16_t)((u + 0x7fffu + lsb) >> 16);
}

__device__ __forceinline__ float bf16_to_f32(uint32_t b) { return __uint_as_float(b << 16); }

// load the 18 reals of one link into registers of type AC
template <typename AC>
__device__ __forceinline__ void load_link(const double *p, AC u[18])
{
    const double2 *q = reinterpret_cast<const double2 *>(p);
#pragma unroll
    for (int k = 0; k < 9; k++) {
        const double2 v = q[k];
        u[2 * k] = (AC)v.x;
        u[2 * k + 1] = (AC)v.y;
    }
}
template <typename AC>
__device__ __forceinline__ void load_link(const float *p, AC u[18])
{
    const float2 *q = reinterpret_cast<const float2 *>(p);
#pragma unroll
    for (int k = 0; k < 9; k++) {
        const float2 v = q[k];
        u[2 * k] = (AC)v.x;
        u[2 * k + 1] = (AC)v.y;
    }
}
template <typename AC>
__device__ __forceinline__ void load_link(const uint16_t *p, AC u[18])
{
    const uint32_t *q = reinterpret_cast<const uint32_t *>(p);
#pragma unroll
    for (int k = 0; k < 9; k++) {
        const uint32_t w = q[k];
        u[2 * k] = (AC)bf16_to_f32(w & 0xffffu);
        u[2 * k + 1] = (AC)bf16_to_f32(w >> 16);
    }
}

// c * (re, im) for the coefficient codes 0:+1 1:-1 2:+i 3:-i
template <int CODE, typename AC>
__device__ __forceinline__ void cmul_code(AC re, AC im, AC &ore, AC &oim)
{
    if constexpr (CODE == 0) { ore = re; oim = im; }
    else if constexpr (CODE == 1) { ore = -re; oim = -im; }
    else if constexpr (CODE == 2) { ore = -im; oim = re; }
    else { ore = im; oim = -re; }
}

// Spin structure of the projected hop (1 -/+ gamma_mu) in the chiral basis.
// Half spinor: h_s = psi_s + a_s * psi_{pi_s} (s = 0, 1); after the colour
// multiply W = U h (or U^+ h) the full spinor is (W_0, W_1, b_0 W_{sig_0}, b_1 W_{sig_1}).
template <int MU, bool FWD> struct Proj;
template <> struct Proj<0, true>  { static constexpr int pi0 = 2, pi1 = 3, a0 = 0, a1 = 0, s0 = 0, s1 = 1, b0 = 0, b1 = 0; };
template <> struct Proj<0, false> { static constexpr int pi0 = 2, pi1 = 3, a0 = 1, a1 = 1, s0 = 0, s1 = 1, b0 = 1, b1 = 1; };
template <> struct Proj<1, true>  { static constexpr int pi0 = 3, pi1 = 2, a0 = 2, a1 = 2, s0 = 1, s1 = 0, b0 = 3, b1 = 3; };
template <> struct Proj<1, false> { static constexpr int pi0 = 3, pi1 = 2, a0 = 3, a1 = 3, s0 = 1, s1 = 0, b0 = 2, b1 = 2; };
template <> struct Proj<2, true>  { static constexpr int pi0 = 3, pi1 = 2, a0 = 0, a1 = 1, s0 = 1, s1 = 0, b0 = 1, b1 = 0; };
template <> struct Proj<2, false> { static constexpr int pi0 = 3, pi1 = 2, a0 = 1, a1 = 0, s0 = 1, s1 = 0, b0 = 0, b1 = 1; };
template <> struct Proj<3, true>  { static constexpr int pi0 = 2, pi1 = 3, a0 = 2, a1 = 3, s0 = 0, s1 = 1, b0 = 3, b1 = 2; };
template <> struct Proj<3, false> { static constexpr int pi0 = 2, pi1 = 3, a0 = 3, a1 = 2, s0 = 0, s1 = 1, b0 = 2, b1 = 3; };

// acc += sg * (1 -/+ gamma_mu) W psi, psi given as 24 reals
template <int MU, bool FWD, typename AC>
__device__ __forceinline__ void hop_term(AC acc[24], const AC psi[24], const AC u[18], AC sg)
{
    using P = Proj<MU, FWD>;
    AC h[2][3][2];
#pragma unroll
    for (int c = 0; c < 3; c++) {
        AC re, im;
        cmul_code<P::a0>(psi[2 * (3 * P::pi0 + c)], psi[2 * (3 * P::pi0 + c) + 1], re, im);
        h[0][c][0] = sg * (psi[2 * c] + re);
        h[0][c][1] = sg * (psi[2 * c + 1] + im);
        cmul_code<P::a1>(psi[2 * (3 * P::pi1 + c)], psi[2 * (3 * P::pi1 + c) + 1], re, im);
        h[1][c][0] = sg * (psi[2 * (3 + c)] + re);
        h[1][c][1] = sg * (psi[2 * (3 + c) + 1] + im);
    }
    AC w[2][3][2];
#pragma unroll
    for (int s = 0; s < 2; s++)
#pragma unroll
        for (int a = 0; a < 3; a++) {
            AC re = 0, im = 0;
#pragma unroll
            for (int b = 0; b < 3; b++) {
                AC ur, ui;
                if constexpr (FWD) {  // U[a][b]
                    ur = u[2 * (3 * a + b)];
                    ui = u[2 * (3 * a + b) + 1];
                } else {              // conj(U[b][a])
                    ur = u[2 * (3 * b + a)];
                    ui = -u[2 * (3 * b + a) + 1];
                }
                re += ur * h[s][b][0] - ui * h[s][b][1];
                im += ur * h[s][b][1] + ui * h[s][b][0];
            }
            w[s][a][0] = re;
            w[s][a][1] = im;
        }
#pragma unroll
    for (int a = 0; a < 3; a++) {
        acc[2 * a] += w[0][a][0];
        acc[2 * a + 1] += w[0][a][1];
        acc[2 * (3 + a)] += w[1][a][0];
        acc[2 * (3 + a) + 1] += w[1][a][1];
        AC re, im;
        cmul_code<P::b0>(w[P::s0][a][0], w[P::s0][a][1], re, im);
        acc[2 * (6 + a)] += re;
        acc[2 * (6 + a) + 1] += im;
        cmul_code<P::b1>(w[P::s1][a][0], w[P::s1][a][1], re, im);
        acc[2 * (9 + a)] += re;
        acc[2 * (9 + a) + 1] += im;
    }
}

template <typename SP, typename AC>
__device__ __forceinline__ void load_spinor(const SP *p, int64_t cs, AC psi[24])
{
#pragma unroll
    for (int c = 0; c < 24; c++) psi[c] = (AC)p[c * cs];
}

template <int MU, typename SP, typename LK, typename AC>
__device__ __forceinline__ void hop_dir(AC acc[24], const int32_t *nb, const SP *in, int64_t cs, int nr,
                                        const LK *lk, int slot_self, int other0)
{
    const int32_t ef = nb[2 * MU];
    if (ef >= 0) {
        const int idx = ef & kNbrMask;
        const AC sg = (ef & kNbrSign) ? (AC)-1 : (AC)1;
        AC psi[24], u[18];
        load_spinor(in + (int64_t)idx * nr, cs, psi);
        load_link(lk + ((int64_t)slot_self * 4 + MU) * 18, u);
        hop_term<MU, true>(acc, psi, u, sg);
    }
    const int32_t eb = nb[2 * MU + 1];
    if (eb >= 0) {
        const int idx = eb & kNbrMask;
        const AC sg = (eb & kNbrSign) ? (AC)-1 : (AC)1;
        AC psi[24], u[18];
        load_spinor(in + (int64_t)idx * nr, cs, psi);
        load_link(lk + ((int64_t)(other0 + idx) * 4 + MU) * 18, u);
        hop_term<MU, false>(acc, psi, u, sg);
    }
}

// per-(tile, rhs) reduction of up to kNRed values; every thread must call it
__device__ __forceinline__ void tile_reduce(double (*red)[kTile], const double v[kNRed], int nred,
                                            double *partial, int tile, int64_t item0, int nr)
{
    for (int k = 0; k < nred; k++) red[k][threadIdx.x] = v[k];
    __syncthreads();
    const int j = threadIdx.x;
    if (j < nr) {
        const int rj = (int)((item0 + j) % nr);
        for (int k = 0; k < nred; k++) {
            double s = 0;
            for (int m = j; m < kTile; m += nr) s += red[k][m];
            partial[((int64_t)tile * nr + rj) * kNRed + k] = s;
        }
    }
}

// --------------------------------------------------------------- hop

template <typename SP, typename LK, typename AC>
__global__ void __launch_bounds__(kTile) k_hop(BlkArgs ba, HopArgs ha)
{
    __shared__ double red[kNRed][kTile];
    const int tile = xcd_tile(blockIdx.x, ba.ntiles);
    const int b = ba.tile_block[tile];
    const int nr = ba.n_rhs;
    const int hb = ba.h[b];
    const int64_t items = (int64_t)hb * nr;
    const int64_t item0 = (int64_t)(tile - ba.blk_tile0[b]) * kTile;
    const int64_t item = item0 + threadIdx.x;
    const bool live = item < items;
    const int64_t base = (ba.soff[b] >> 1) * 24 * nr;
    const int p = ha.parity;
    double dv[kNRed] = {0, 0, 0, 0};
    if (live) {
        const int site = (int)(item / nr);
        const int r = (int)(item - (int64_t)site * nr);
        const int32_t *nb = ba.nbr + ba.nbr_off[b] + (int64_t)(p * hb + site) * 8;
        const LK *lk = reinterpret_cast<const LK *>(ha.links) + ba.soff[b] * 72;
        const SP *in = reinterpret_cast<const SP *>(ha.in) + base + r;
        int32_t nbl[8];
        {
            const int4 *q = reinterpret_cast<const int4 *>(nb);
            const int4 a0 = q[0], a1 = q[1];
            nbl[0] = a0.x; nbl[1] = a0.y; nbl[2] = a0.z; nbl[3] = a0.w;
            nbl[4] = a1.x; nbl[5] = a1.y; nbl[6] = a1.z; nbl[7] = a1.w;
        }
        AC acc[24];
#pragma unroll
        for (int c = 0; c < 24; c++) acc[c] = 0;
        const int slot = p * hb + site;
        const int other0 = (1 - p) * hb;
        hop_dir<0>(acc, nbl, in, items, nr, lk, slot, other0);
        hop_dir<1>(acc, nbl, in, items, nr, lk, slot, other0);
        hop_dir<2>(acc, nbl, in, items, nr, lk, slot, other0);
        hop_dir<3>(acc, nbl, in, items, nr, lk, slot, other0);

        const int64_t off = base + item;
        SP *out = reinterpret_cast<SP *>(ha.out) + off;
        const SP *self = ha.self ? reinterpret_cast<const SP *>(ha.self) + off : nullptr;
        const SP *add = ha.add ? reinterpret_cast<const SP *>(ha.add) + off : nullptr;
        const SP *aux = ha.aux ? reinterpret_cast<const SP *>(ha.aux) + off : nullptr;
        const AC ch = (AC)ha.c_hop, cself = (AC)ha.c_self, cadd = (AC)ha.c_add;
#pragma unroll
        for (int k = 0; k < 12; k++) {
            SP o[2];
            double sv[2] = {0, 0};
#pragma unroll
            for (int ri = 0; ri < 2; ri++) {
                const int c = 2 * k + ri;
                AC v = ch * acc[c];
                if (self) {
                    const SP s = self[c * items];
                    sv[ri] = (double)s;
                    v += cself * (AC)s;
                }
                if (add) v += cadd * (AC)add[c * items];
                o[ri] = (SP)v;
                out[c * items] = o[ri];
            }
            const double ore = (double)o[0], oim = (double)o[1];
            if (ha.dot_mode == kDotAuxOut) {
                const double are = (double)aux[(2 * k) * items], aim = (double)aux[(2 * k + 1) * items];
                dv[0] += are * ore + aim * oim;
                dv[1] += are * oim - aim * ore;
            } else if (ha.dot_mode == kDotOutSelfOutOut) {
                dv[0] += ore * sv[0] + oim * sv[1];
                dv[1] += ore * sv[1] - oim * sv[0];
                dv[2] += ore * ore + oim * oim;
            } else if (ha.dot_mode == kDotOutOut) {
                dv[0] += ore * ore + oim * oim;
            }
        }
    }
    if (ha.dot_mode != kDotNone) {
        const int nred = ha.dot_mode == kDotAuxOut ? 2 : (ha.dot_mode == kDotOutSelfOutOut ? 3 : 1);
        tile_reduce(red, dv, nred, ha.partial, tile, item0, nr);
    }
}

hipError_t launch_hop(const BlkArgs &ba, const HopArgs &ha, dd_prec prec, hipStream_t s)
{
    if (ba.ntiles <= 0) return hipSuccess;
    dim3 g(ba.ntiles), t(kTile);
    switch (prec) {
    case DD_F64: hipLaunchKernelGGL((k_hop<double, double, double>), g, t, 0, s, ba, ha); break;
    case DD_F32: hipLaunchKernelGGL((k_hop<float, float, float>), g, t, 0, s, ba, ha); break;
    case DD_BF16: hipLaunchKernelGGL((k_hop<float, uint16_t, float>), g, t, 0, s, ba, ha); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------- packing

struct PackGeom {
    int L[4];
    int nb;
    const int64_t *soff;
    const int32_t *h;
    const int64_t *nbr_off;
    const int32_t *nbr;
    const int64_t *perm_off;
    const int32_t *perm;
    const int32_t *origin;
    const int32_t *ext;
};

__device__ __forceinline__ int find_block(const int64_t *soff, int nb, int64_t q)
{
    int lo = 0, hi = nb;  // soff[lo] <= q < soff[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (soff[mid] <= q) lo = mid; else hi = mid;
    }
    return lo;
}

__device__ __forceinline__ void local_coords(int y, const int32_t *e, int c[4])
{
    c[3] = y % e[3]; y /= e[3];
    c[2] = y % e[2]; y /= e[2];
    c[1] = y % e[1]; y /= e[1];
    c[0] = y;
}

template <typename LT>
__device__ __forceinline__ LT cvt_link(double v);
template <> __device__ __forceinline__ double cvt_link<double>(double v) { return v; }
template <> __device__ __forceinline__ float cvt_link<float>(double v) { return (float)v; }
template <> __device__ __forceinline__ uint16_t cvt_link<uint16_t>(double v) { return f32_to_bf16_rne((float)v); }

template <typename LT>
__global__ void __launch_bounds__(256) k_pack_gauge(PackGeom g, const double *U, LT *dst, int64_t total)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= total) return;
    const int b = find_block(g.soff, g.nb, q);
    const int s = (int)(q - g.soff[b]);
    const int hb = g.h[b];
    const int y = g.perm[g.perm_off[b] + s];
    int c[4];
    local_coords(y, g.ext + 4 * b, c);
    int x[4];
    for (int m = 0; m < 4; m++) x[m] = (g.origin[4 * b + m] + c[m]) % g.L[m];
    const int64_t n = (((int64_t)x[0] * g.L[1] + x[1]) * g.L[2] + x[2]) * g.L[3] + x[3];
    const int32_t *nb = g.nbr + g.nbr_off[b] + (int64_t)s * 8;  // slot s = p*h + site
    (void)hb;
    for (int mu = 0; mu < 4; mu++) {
        LT *o = dst + (q * 4 + mu) * 18;
        if (nb[2 * mu] >= 0) {
            const double *u = U + (n * 4 + mu) * 18;
            for (int k = 0; k < 18; k++) o[k] = cvt_link<LT>(u[k]);
        } else {
            for (int k = 0; k < 18; k++) o[k] = (LT)0;
        }
    }
}

static PackGeom pack_geom(const dd_blocks *B)
{
    PackGeom g;
    for (int m = 0; m < 4; m++) g.L[m] = B->L[m];
    g.nb = B->nb;
    g.soff = B->d_soff;
    g.h = B->d_h;
    g.nbr_off = B->d_nbr_off;
    g.nbr = B->d_nbr;
    g.perm_off = B->d_perm_off;
    g.perm = B->d_perm;
    g.origin = B->d_origin;
    g.ext = B->d_ext;
    return g;
}

hipError_t launch_pack_gauge(const dd_blocks *B, const double *U, dd_prec prec, void *dst, hipStream_t s)
{
    const int64_t total = B->soff[B->nb];
    if (total == 0) return hipSuccess;
    const PackGeom g = pack_geom(B);
    dim3 grid((unsigned)((total + 255) / 256)), t(256);
    switch (prec) {
    case DD_F64: hipLaunchKernelGGL(k_pack_gauge<double>, grid, t, 0, s, g, U, (double *)dst, total); break;
    case DD_F32: hipLaunchKernelGGL(k_pack_gauge<float>, grid, t, 0, s, g, U, (float *)dst, total); break;
    case DD_BF16: hipLaunchKernelGGL(k_pack_gauge<uint16_t>, grid, t, 0, s, g, U, (uint16_t *)dst, total); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// boundary layout [r][q][24] (q = block site, box-local canonical) <-> half fields
template <typename SP, bool PACK>
__global__ void __launch_bounds__(256) k_spinor_xfer(PackGeom g, double *ext_f, SP *even, SP *odd,
                                                    int nr, int64_t total)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= total * nr) return;
    const int r = (int)(t / total);
    const int64_t q = t - (int64_t)r * total;  // block site in eo order
    const int b = find_block(g.soff, g.nb, q);
    const int s = (int)(q - g.soff[b]);
    const int hb = g.h[b];
    const int p = s >= hb;
    const int site = s - p * hb;
    const int y = g.perm[g.perm_off[b] + s];
    double *e = ext_f + ((int64_t)r * total + g.soff[b] + y) * 24;
    SP *hf = (p ? odd : even) + (g.soff[b] >> 1) * 24 * nr + (int64_t)site * nr + r;
    const int64_t cs = (int64_t)hb * nr;
    for (int c = 0; c < 24; c++) {
        if constexpr (PACK) hf[c * cs] = (SP)e[c];
        else e[c] = (double)hf[c * cs];
    }
}

hipError_t launch_pack_spinor(const dd_blocks *B, const double *src, void *even, void *odd, dd_prec prec,
                              int n_rhs, hipStream_t s)
{
    const int64_t total = B->soff[B->nb];
    if (total == 0 || n_rhs == 0) return hipSuccess;
    const PackGeom g = pack_geom(B);
    dim3 grid((unsigned)((total * n_rhs + 255) / 256)), t(256);
    if (prec == DD_F64)
        hipLaunchKernelGGL((k_spinor_xfer<double, true>), grid, t, 0, s, g, (double *)src, (double *)even,
                           (double *)odd, n_rhs, total);
    else
        hipLaunchKernelGGL((k_spinor_xfer<float, true>), grid, t, 0, s, g, (double *)src, (float *)even,
                           (float *)odd, n_rhs, total);
    return hipGetLastError();
}

hipError_t launch_unpack_spinor(const dd_blocks *B, const void *even, const void *odd, double *dst,
                                dd_prec prec, int n_rhs, hipStream_t s)
{
    const int64_t total = B->soff[B->nb];
    if (total == 0 || n_rhs == 0) return hipSuccess;
    const PackGeom g = pack_geom(B);
    dim3 grid((unsigned)((total * n_rhs + 255) / 256)), t(256);
    if (prec == DD_F64)
        hipLaunchKernelGGL((k_spinor_xfer<double, false>), grid, t, 0, s, g, dst, (double *)even,
                           (double *)odd, n_rhs, total);
    else
        hipLaunchKernelGGL((k_spinor_xfer<float, false>), grid, t, 0, s, g, dst, (float *)even,
                           (float *)odd, n_rhs, total);
    return hipGetLastError();
}

// ------------------------------------------------------------ elementwise

template <typename S, typename D>
__global__ void __launch_bounds__(256) k_convert(const S *src, D *dst, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = (D)src[i];
}

hipError_t launch_convert(const void *src, dd_prec sp, void *dst, dd_prec dp, int64_t n, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    dim3 grid((unsigned)((n + 255) / 256)), t(256);
    if (sp == DD_F64 && dp == DD_F32)
        hipLaunchKernelGGL((k_convert<double, float>), grid, t, 0, s, (const double *)src, (float *)dst, n);
    else if (sp == DD_F32 && dp == DD_F64)
        hipLaunchKernelGGL((k_convert<float, double>), grid, t, 0, s, (const float *)src, (double *)dst, n);
    else if (sp == DD_F64 && dp == DD_F64)
        return hipMemcpyAsync(dst, src, n * sizeof(double), hipMemcpyDeviceToDevice, s);
    else if (sp == DD_F32 && dp == DD_F32)
        return hipMemcpyAsync(dst, src, n * sizeof(float), hipMemcpyDeviceToDevice, s);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}


// ------------------------------------------------------ Krylov site kernels

// common prologue of the per-item kernels: tile -> (block, site, rhs, pair)
struct Item {
    int b, r, pair, tile;
    int64_t off, cs, item0;
    bool live;
};

__device__ __forceinline__ Item item_of(const BlkArgs &ba)
{
    Item it;
    it.tile = xcd_tile(blockIdx.x, ba.ntiles);
    it.b = ba.tile_block[it.tile];
    const int nr = ba.n_rhs;
    const int64_t items = (int64_t)ba.h[it.b] * nr;
    it.item0 = (int64_t)(it.tile - ba.blk_tile0[it.b]) * kTile;
    const int64_t item = it.item0 + threadIdx.x;
    it.live = item < items;
    const int site = it.live ? (int)(item / nr) : 0;
    it.r = it.live ? (int)(item - (int64_t)site * nr) : 0;
    it.pair = it.r * ba.nb + it.b;
    it.off = (ba.soff[it.b] >> 1) * 24 * nr + item;
    it.cs = items;
    return it;
}

// x_p += e_p for the pairs still above tolerance (FP64 accumulator)
template <typename SE>
__global__ void __launch_bounds__(kTile) k_accum(BlkArgs ba, double *x, const SE *e, const int32_t *active)
{
    const Item it = item_of(ba);
    if (!it.live || !active[it.pair]) return;
#pragma unroll 4
    for (int c = 0; c < 24; c++) x[it.off + c * it.cs] += (double)e[it.off + c * it.cs];
}

hipError_t launch_accum(const BlkArgs &ba, double *x, const void *e, dd_prec ep, const int32_t *active,
                        hipStream_t s)
{
    if (ba.ntiles <= 0) return hipSuccess;
    dim3 g(ba.ntiles), t(kTile);
    if (ep == DD_F64)
        hipLaunchKernelGGL(k_accum<double>, g, t, 0, s, ba, x, (const double *)e, active);
    else
        hipLaunchKernelGGL(k_accum<float>, g, t, 0, s, ba, x, (const float *)e, active);
    return hipGetLastError();
}

// BiCGStab start: r = rh = p = rhs, x = 0; |rhs|^2 per (tile, rhs)
template <typename SP>
__global__ void __launch_bounds__(kTile) k_bicg_init(BlkArgs ba, const SP *rhs, SP *r, SP *rh, SP *p, SP *x,
                                                     double *partial, const int32_t *outer_active)
{
    __shared__ double red[kNRed][kTile];
    const Item it = item_of(ba);
    double dv[kNRed] = {0, 0, 0, 0};
    if (it.live && outer_active[it.pair]) {
        for (int c = 0; c < 24; c++) {
            const int64_t i = it.off + c * it.cs;
            const SP v = rhs[i];
            r[i] = v;
            rh[i] = v;
            p[i] = v;
            x[i] = (SP)0;
            dv[0] += (double)v * (double)v;
        }
    }
    tile_reduce(red, dv, 1, partial, it.tile, it.item0, ba.n_rhs);
}

// s = r - alpha v
template <typename SP>
__global__ void __launch_bounds__(kTile) k_bicg_s(BlkArgs ba, const SP *r, const SP *v, SP *s, PairState ps)
{
    const Item it = item_of(ba);
    if (!it.live || !ps.active[it.pair]) return;
    const double ar = ps.alpha[2 * it.pair], ai = ps.alpha[2 * it.pair + 1];
    using AC = SP;
    const AC a_r = (AC)ar, a_i = (AC)ai;
#pragma unroll 4
    for (int k = 0; k < 12; k++) {
        const int64_t i0 = it.off + (2 * k) * it.cs, i1 = i0 + it.cs;
        const AC vr = (AC)v[i0], vi = (AC)v[i1];
        s[i0] = (SP)((AC)r[i0] - (a_r * vr - a_i * vi));
        s[i1] = (SP)((AC)r[i1] - (a_r * vi + a_i * vr));
    }
}

// x += alpha p + omega s;  r = s - omega t;  <rh, r> and |r|^2 per (tile, rhs)
template <typename SP>
__global__ void __launch_bounds__(kTile) k_bicg_xr(BlkArgs ba, SP *x, const SP *p, const SP *s, const SP *t,
                                                   SP *r, const SP *rh, double *partial, PairState ps)
{
    __shared__ double red[kNRed][kTile];
    const Item it = item_of(ba);
    double dv[kNRed] = {0, 0, 0, 0};
    if (it.live && ps.active[it.pair]) {
        using AC = SP;
        const AC a_r = (AC)ps.alpha[2 * it.pair], a_i = (AC)ps.alpha[2 * it.pair + 1];
        const AC w_r = (AC)ps.omega[2 * it.pair], w_i = (AC)ps.omega[2 * it.pair + 1];
#pragma unroll 2
        for (int k = 0; k < 12; k++) {
            const int64_t i0 = it.off + (2 * k) * it.cs, i1 = i0 + it.cs;
            const AC pr = (AC)p[i0], pi = (AC)p[i1];
            const AC sr = (AC)s[i0], si = (AC)s[i1];
            const AC tr = (AC)t[i0], ti = (AC)t[i1];
            x[i0] = (SP)((AC)x[i0] + (a_r * pr - a_i * pi) + (w_r * sr - w_i * si));
            x[i1] = (SP)((AC)x[i1] + (a_r * pi + a_i * pr) + (w_r * si + w_i * sr));
            const SP nr_ = (SP)(sr - (w_r * tr - w_i * ti));
            const SP ni_ = (SP)(si - (w_r * ti + w_i * tr));
            r[i0] = nr_;
            r[i1] = ni_;
            const double hr = (double)rh[i0], hi = (double)rh[i1];
            const double rr_ = (double)nr_, ri_ = (double)ni_;
            dv[0] += hr * rr_ + hi * ri_;
            dv[1] += hr * ri_ - hi * rr_;
            dv[2] += rr_ * rr_ + ri_ * ri_;
        }
    }
    tile_reduce(red, dv, 3, partial, it.tile, it.item0, ba.n_rhs);
}

// p = r + beta (p - omega v)
template <typename SP>
__global__ void __launch_bounds__(kTile) k_bicg_p(BlkArgs ba, const SP *r, const SP *v, SP *p, PairState ps)
{
    const Item it = item_of(ba);
    if (!it.live || !ps.active[it.pair]) return;
    using AC = SP;
    const AC b_r = (AC)ps.beta[2 * it.pair], b_i = (AC)ps.beta[2 * it.pair + 1];
    const AC w_r = (AC)ps.omega[2 * it.pair], w_i = (AC)ps.omega[2 * it.pair + 1];
#pragma unroll 4
    for (int k = 0; k < 12; k++) {
        const int64_t i0 = it.off + (2 * k) * it.cs, i1 = i0 + it.cs;
        const AC vr = (AC)v[i0], vi = (AC)v[i1];
        const AC qr = (AC)p[i0] - (w_r * vr - w_i * vi);
        const AC qi = (AC)p[i1] - (w_r * vi + w_i * vr);
        p[i0] = (SP)((AC)r[i0] + (b_r * qr - b_i * qi));
        p[i1] = (SP)((AC)r[i1] + (b_r * qi + b_i * qr));
    }
}

hipError_t launch_bicg_init(const BlkArgs &ba, dd_prec sp, const void *rhs, void *r, void *rh, void *p,
                            void *x, double *partial, const int32_t *outer_active, hipStream_t st)
{
    if (ba.ntiles <= 0) return hipSuccess;
    dim3 g(ba.ntiles), t(kTile);
    if (sp == DD_F64)
        hipLaunchKernelGGL(k_bicg_init<double>, g, t, 0, st, ba, (const double *)rhs, (double *)r, (double *)rh,
                           (double *)p, (double *)x, partial, outer_active);
    else
        hipLaunchKernelGGL(k_bicg_init<float>, g, t, 0, st, ba, (const float *)rhs, (float *)r, (float *)rh,
                           (float *)p, (float *)x, partial, outer_active);
    return hipGetLastError();
}

hipError_t launch_bicg_s(const BlkArgs &ba, dd_prec sp, const void *r, const void *v, void *s,
                         const PairState &ps, hipStream_t st)
{
    if (ba.ntiles <= 0) return hipSuccess;
    dim3 g(ba.ntiles), t(kTile);
    if (sp == DD_F64)
        hipLaunchKernelGGL(k_bicg_s<double>, g, t, 0, st, ba, (const double *)r, (const double *)v, (double *)s, ps);
    else
        hipLaunchKernelGGL(k_bicg_s<float>, g, t, 0, st, ba, (const float *)r, (const float *)v, (float *)s, ps);
    return hipGetLastError();
}

hipError_t launch_bicg_xr(const BlkArgs &ba, dd_prec sp, void *x, const void *p, const void *s, const void *tv,
                          void *r, const void *rh, double *partial, const PairState &ps, hipStream_t st)
{
    if (ba.ntiles <= 0) return hipSuccess;
    dim3 g(ba.ntiles), t(kTile);
    if (sp == DD_F64)
        hipLaunchKernelGGL(k_bicg_xr<double>, g, t, 0, st, ba, (double *)x, (const double *)p, (const double *)s,
                           (const double *)tv, (double *)r, (const double *)rh, partial, ps);
    else
        hipLaunchKernelGGL(k_bicg_xr<float>, g, t, 0, st, ba, (float *)x, (const float *)p, (const float *)s,
                           (const float *)tv, (float *)r, (const float *)rh, partial, ps);
    return hipGetLastError();
}

hipError_t launch_bicg_p(const BlkArgs &ba, dd_prec sp, const void *r, const void *v, void *p,
                         const PairState &ps, hipStream_t st)
{
    if (ba.ntiles <= 0) return hipSuccess;
    dim3 g(ba.ntiles), t(kTile);
    if (sp == DD_F64)
        hipLaunchKernelGGL(k_bicg_p<double>, g, t, 0, st, ba, (const double *)r, (const double *)v, (double *)p, ps);
    else
        hipLaunchKernelGGL(k_bicg_p<float>, g, t, 0, st, ba, (const float *)r, (const float *)v, (float *)p, ps);
    return hipGetLastError();
}

// ------------------------------------------------------ per-pair scalars

// sum over the tiles of the pair's block of partial[.][r][k]
__device__ __forceinline__ double pair_sum(const BlkArgs &ba, const double *partial, int b, int r, int k)
{
    double s = 0;
    const int t1 = ba.blk_tile0[b + 1];
    for (int t = ba.blk_tile0[b]; t < t1; t++) s += partial[((int64_t)t * ba.n_rhs + r) * kNRed + k];
    return s;
}

__device__ __forceinline__ bool finite(double v) { return isfinite(v); }

__global__ void k_sc_init(BlkArgs ba, const double *partial, PairState ps, const int32_t *outer_active)
{
    const int pair = blockIdx.x * blockDim.x + threadIdx.x;
    if (pair >= ps.np) return;
    const int b = pair % ba.nb, r = pair / ba.nb;
    if (!outer_active[pair]) {
        ps.active[pair] = 0;
        return;
    }
    const double bb = pair_sum(ba, partial, b, r, 0);
    ps.bb[pair] = bb;
    ps.rr[pair] = bb;
    ps.rho[2 * pair] = bb;
    ps.rho[2 * pair + 1] = 0;
    ps.omega[2 * pair] = 1;
    ps.omega[2 * pair + 1] = 0;
    const bool ok = finite(bb) && bb > 0;
    ps.active[pair] = ok ? 1 : 0;
    if (!finite(bb)) ps.flags[pair] |= 4;
}

__global__ void k_sc_alpha(BlkArgs ba, const double *partial, PairState ps)
{
    const int pair = blockIdx.x * blockDim.x + threadIdx.x;
    if (pair >= ps.np || !ps.active[pair]) return;
    const int b = pair % ba.nb, r = pair / ba.nb;
    const double vr = pair_sum(ba, partial, b, r, 0), vi = pair_sum(ba, partial, b, r, 1);
    const double rr = ps.rho[2 * pair], ri = ps.rho[2 * pair + 1];
    const double den = vr * vr + vi * vi;
    const double ar = (rr * vr + ri * vi) / den, ai = (ri * vr - rr * vi) / den;
    if (!(den > 0) || !finite(ar) || !finite(ai)) {
        ps.active[pair] = 0;
        ps.flags[pair] |= 2;
        return;
    }
    ps.alpha[2 * pair] = ar;
    ps.alpha[2 * pair + 1] = ai;
}

__global__ void k_sc_omega(BlkArgs ba, const double *partial, PairState ps)
{
    const int pair = blockIdx.x * blockDim.x + threadIdx.x;
    if (pair >= ps.np || !ps.active[pair]) return;
    const int b = pair % ba.nb, r = pair / ba.nb;
    const double tsr = pair_sum(ba, partial, b, r, 0), tsi = pair_sum(ba, partial, b, r, 1);
    const double tt = pair_sum(ba, partial, b, r, 2);
    const double wr = tsr / tt, wi = tsi / tt;
    if (!(tt > 0) || !finite(wr) || !finite(wi)) {
        ps.active[pair] = 0;
        ps.flags[pair] |= 2;
        return;
    }
    ps.omega[2 * pair] = wr;
    ps.omega[2 * pair + 1] = wi;
}

__global__ void k_sc_beta(BlkArgs ba, const double *partial, PairState ps, double tol2)
{
    const int pair = blockIdx.x * blockDim.x + threadIdx.x;
    if (pair >= ps.np || !ps.active[pair]) return;
    const int b = pair % ba.nb, r = pair / ba.nb;
    const double nr_ = pair_sum(ba, partial, b, r, 0), ni_ = pair_sum(ba, partial, b, r, 1);
    const double rr = pair_sum(ba, partial, b, r, 2);
    ps.iters[pair] += 1;
    ps.rr[pair] = rr;
    if (!finite(rr)) {
        ps.active[pair] = 0;
        ps.flags[pair] |= 4;
        return;
    }
    if (rr <= tol2 * ps.bb[pair]) {
        ps.active[pair] = 0;
        return;
    }
    // beta = (rho_new / rho) * (alpha / omega)
    const double pr = ps.rho[2 * pair], pi = ps.rho[2 * pair + 1];
    const double ar = ps.alpha[2 * pair], ai = ps.alpha[2 * pair + 1];
    const double wr = ps.omega[2 * pair], wi = ps.omega[2 * pair + 1];
    const double d1 = pr * pr + pi * pi;
    const double q1r = (nr_ * pr + ni_ * pi) / d1, q1i = (ni_ * pr - nr_ * pi) / d1;
    const double d2 = wr * wr + wi * wi;
    const double q2r = (ar * wr + ai * wi) / d2, q2i = (ai * wr - ar * wi) / d2;
    const double br = q1r * q2r - q1i * q2i, bi = q1r * q2i + q1i * q2r;
    if (!finite(br) || !finite(bi)) {
        ps.active[pair] = 0;
        ps.flags[pair] |= 2;
        return;
    }
    ps.beta[2 * pair] = br;
    ps.beta[2 * pair + 1] = bi;
    ps.rho[2 * pair] = nr_;
    ps.rho[2 * pair + 1] = ni_;
}

// true residual |b - D x|^2 = even + odd partials; first call also sets |b|^2
__global__ void k_sc_outer(BlkArgs ba, const double *pe, const double *po, int first, double tol2, OuterState os,
                           int np)
{
    const int pair = blockIdx.x * blockDim.x + threadIdx.x;
    if (pair >= np) return;
    const int b = pair % ba.nb, r = pair / ba.nb;
    const double rr = pair_sum(ba, pe, b, r, 0) + pair_sum(ba, po, b, r, 0);
    if (first) {
        os.bb[pair] = rr;
        os.flags[pair] = 0;
    }
    os.rr[pair] = rr;
    if (!finite(rr)) {
        os.flags[pair] |= 4;
        os.active[pair] = 0;
        return;
    }
    const bool conv = rr <= tol2 * os.bb[pair];
    os.active[pair] = conv ? 0 : 1;
    if (conv) os.flags[pair] |= 1;
    else os.flags[pair] &= ~1;
}

static inline dim3 pair_grid(int np) { return dim3((unsigned)((np + 255) / 256)); }

hipError_t launch_sc_init(const BlkArgs &ba, const double *partial, const PairState &ps, const int32_t *outer_active,
                          hipStream_t s)
{
    hipLaunchKernelGGL(k_sc_init, pair_grid(ps.np), dim3(256), 0, s, ba, partial, ps, outer_active);
    return hipGetLastError();
}
hipError_t launch_sc_alpha(const BlkArgs &ba, const double *partial, const PairState &ps, hipStream_t s)
{
    hipLaunchKernelGGL(k_sc_alpha, pair_grid(ps.np), dim3(256), 0, s, ba, partial, ps);
    return hipGetLastError();
}
hipError_t launch_sc_omega(const BlkArgs &ba, const double *partial, const PairState &ps, hipStream_t s)
{
    hipLaunchKernelGGL(k_sc_omega, pair_grid(ps.np), dim3(256), 0, s, ba, partial, ps);
    return hipGetLastError();
}
hipError_t launch_sc_beta(const BlkArgs &ba, const double *partial, const PairState &ps, double tol,
                          hipStream_t s)
{
    hipLaunchKernelGGL(k_sc_beta, pair_grid(ps.np), dim3(256), 0, s, ba, partial, ps, tol * tol);
    return hipGetLastError();
}
hipError_t launch_sc_outer(const BlkArgs &ba, const double *pe, const double *po, int first, double tol,
                           const OuterState &os, hipStream_t s)
{
    const int np = ba.n_rhs * ba.nb;
    hipLaunchKernelGGL(k_sc_outer, pair_grid(np), dim3(256), 0, s, ba, pe, po, first, tol * tol, os, np);
    return hipGetLastError();
}

// ------------------------------------------------- multi-boson boundary norm

// S[b] = sum_k sum_{i in dLambda_0^b} | u_k chi_k(i) + y_k(i) |^2, FP64.
// y: solutions in the boundary layout [k][q][24]; chi: [k][q_bnd][24].
__global__ void __launch_bounds__(256) k_mb_norm(int nb, int nf, const double *u, const double *chi,
                                                 const double *y, const int64_t *soff, const int64_t *boff,
                                                 const int32_t *bnd, int64_t total, int64_t total_bnd, double *S)
{
    __shared__ double red[256];
    const int b = blockIdx.x;
    const int64_t b0 = boff[b], nbd = boff[b + 1] - b0;
    double acc = 0;
    for (int64_t t = threadIdx.x; t < nbd * nf; t += blockDim.x) {
        const int k = (int)(t / nbd);
        const int64_t i = t - (int64_t)k * nbd;
        const double ur = u[2 * k], ui = u[2 * k + 1];
        const double *c = chi + ((int64_t)k * total_bnd + b0 + i) * 24;
        const double *yy = y + ((int64_t)k * total + soff[b] + bnd[b0 + i]) * 24;
        for (int j = 0; j < 12; j++) {
            const double cr = c[2 * j], ci = c[2 * j + 1];
            const double vr = ur * cr - ui * ci + yy[2 * j];
            const double vi = ur * ci + ui * cr + yy[2 * j + 1];
            acc += vr * vr + vi * vi;
        }
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) S[b] = red[0];
}

hipError_t launch_mb_norm(const dd_blocks *B, int n_fields, const double *u, const double *chi, const double *y,
                          double *S, hipStream_t s)
{
    if (B->nb == 0) return hipSuccess;
    hipLaunchKernelGGL(k_mb_norm, dim3(B->nb), dim3(256), 0, s, B->nb, n_fields, u, chi, y, B->d_soff, B->d_boff,
                       B->d_bnd, (int64_t)B->soff[B->nb], (int64_t)B->boff[B->nb], S);
    return hipGetLastError();
}

}  // namespace dd
