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

// ------------------------------------------------- G right-hand sides per thread
//
// A thread owns one site and G consecutive right-hand sides (G | n_rhs), so
// each link it loads serves G spinors and every component is one vector load
// of G contiguous values (16 bytes for 4 floats or 2 doubles).

template <typename T, int G>
__device__ __forceinline__ void ldv(const T *p, T (&v)[G])
{
    constexpr int B = (int)sizeof(T) * G;
    if constexpr (B % 16 == 0) {
#pragma unroll
        for (int k = 0; k < B / 16; k++) {
            const uint4 q = reinterpret_cast<const uint4 *>(p)[k];
            __builtin_memcpy(reinterpret_cast<char *>(v) + 16 * k, &q, 16);
        }
    } else if constexpr (B == 8) {
        const uint2 q = *reinterpret_cast<const uint2 *>(p);
        __builtin_memcpy(v, &q, 8);
    } else {
#pragma unroll
        for (int j = 0; j < G; j++) v[j] = p[j];
    }
}

template <typename T, int G>
__device__ __forceinline__ void stv(T *p, const T (&v)[G])
{
    constexpr int B = (int)sizeof(T) * G;
    if constexpr (B % 16 == 0) {
#pragma unroll
        for (int k = 0; k < B / 16; k++) {
            uint4 q;
            __builtin_memcpy(&q, reinterpret_cast<const char *>(v) + 16 * k, 16);
            reinterpret_cast<uint4 *>(p)[k] = q;
        }
    } else if constexpr (B == 8) {
        uint2 q;
        __builtin_memcpy(&q, v, 8);
        *reinterpret_cast<uint2 *>(p) = q;
    } else {
#pragma unroll
        for (int j = 0; j < G; j++) p[j] = v[j];
    }
}

// (tile, thread) -> block, site, rhs group
struct Item {
    int b, site, rg, tile, titem0, ng;
    int64_t off, cs;
    bool live;
};

__device__ __forceinline__ Item item_of(const BlkArgs &ba)
{
    Item it;
    it.tile = xcd_tile(blockIdx.x, ba.ntiles);
    it.b = ba.tile_block[it.tile];
    const int nr = ba.n_rhs;
    it.ng = nr / ba.g;
    const int hb = ba.h[it.b];
    const int titems = hb * it.ng;
    it.titem0 = (it.tile - ba.blk_tile0[it.b]) * kTile;
    const int titem = it.titem0 + (int)threadIdx.x;
    it.live = titem < titems;
    it.site = it.live ? titem / it.ng : 0;
    it.rg = it.live ? titem - it.site * it.ng : 0;
    it.off = (ba.soff[it.b] >> 1) * 24 * nr + (int64_t)it.site * nr + (int64_t)it.rg * ba.g;
    it.cs = (int64_t)hb * nr;
    return it;
}

// Per-(tile, rhs) sums of up to kNRed values; every thread of the tile calls it.
template <int G>
__device__ __forceinline__ void tile_reduce(double (*red)[kTile], const double (&dv)[G][kNRed], int nred,
                                            double *partial, const Item &it, int nr)
{
    for (int k = 0; k < nred; k++) {
#pragma unroll
        for (int j = 0; j < G; j++) red[j][threadIdx.x] = dv[j][k];
        __syncthreads();
        const int t = threadIdx.x;
        if (t < nr) {
            const int q = t / G, jj = t - (t / G) * G;
            const int start = ((q - it.titem0 % it.ng) % it.ng + it.ng) % it.ng;
            double s = 0;
            for (int m = start; m < kTile; m += it.ng) s += red[jj][m];
            partial[((int64_t)it.tile * nr + t) * kNRed + k] = s;
        }
        __syncthreads();
    }
}

// acc[j] += sg * (1 -/+ gamma_mu) W psi_j(idx) for the G rhs, accumulating the
// colour contributions of the projected half spinor straight into acc.
template <int MU, bool FWD, typename SP, typename AC, int G>
__device__ __forceinline__ void hop_term_g(AC (&acc)[G][24], const SP *in, int64_t cs, int64_t site_off,
                                           const AC (&u)[18], AC sg)
{
    using P = Proj<MU, FWD>;
#pragma unroll
    for (int c = 0; c < 3; c++) {
        SP v[4][2][G];
#pragma unroll
        for (int sp = 0; sp < 4; sp++)
#pragma unroll
            for (int ri = 0; ri < 2; ri++) ldv<SP, G>(in + (2 * (3 * sp + c) + ri) * cs + site_off, v[sp][ri]);
#pragma unroll
        for (int j = 0; j < G; j++) {
            AC h[2][2];
            AC re, im;
            cmul_code<P::a0>((AC)v[P::pi0][0][j], (AC)v[P::pi0][1][j], re, im);
            h[0][0] = sg * ((AC)v[0][0][j] + re);
            h[0][1] = sg * ((AC)v[0][1][j] + im);
            cmul_code<P::a1>((AC)v[P::pi1][0][j], (AC)v[P::pi1][1][j], re, im);
            h[1][0] = sg * ((AC)v[1][0][j] + re);
            h[1][1] = sg * ((AC)v[1][1][j] + im);
#pragma unroll
            for (int a = 0; a < 3; a++) {
                AC ur, ui;
                if constexpr (FWD) {  // U[a][c]
                    ur = u[2 * (3 * a + c)];
                    ui = u[2 * (3 * a + c) + 1];
                } else {              // conj(U[c][a])
                    ur = u[2 * (3 * c + a)];
                    ui = -u[2 * (3 * c + a) + 1];
                }
                AC d[2][2];
#pragma unroll
                for (int s = 0; s < 2; s++) {
                    d[s][0] = ur * h[s][0] - ui * h[s][1];
                    d[s][1] = ur * h[s][1] + ui * h[s][0];
                }
                acc[j][2 * a] += d[0][0];
                acc[j][2 * a + 1] += d[0][1];
                acc[j][2 * (3 + a)] += d[1][0];
                acc[j][2 * (3 + a) + 1] += d[1][1];
                cmul_code<P::b0>(d[P::s0][0], d[P::s0][1], re, im);
                acc[j][2 * (6 + a)] += re;
                acc[j][2 * (6 + a) + 1] += im;
                cmul_code<P::b1>(d[P::s1][0], d[P::s1][1], re, im);
                acc[j][2 * (9 + a)] += re;
                acc[j][2 * (9 + a) + 1] += im;
            }
        }
    }
}

template <int MU, typename SP, typename LK, typename AC, int G>
__device__ __forceinline__ void hop_dir(AC (&acc)[G][24], const int32_t (&nb)[8], const SP *in, int64_t cs, int nr,
                                        const LK *lk, int slot_self, int other0)
{
    const int32_t ef = nb[2 * MU];
    if (ef >= 0) {
        const int idx = ef & kNbrMask;
        const AC sg = (ef & kNbrSign) ? (AC)-1 : (AC)1;
        AC u[18];
        load_link(lk + ((int64_t)slot_self * 4 + MU) * 18, u);
        hop_term_g<MU, true, SP, AC, G>(acc, in, cs, (int64_t)idx * nr, u, sg);
    }
    const int32_t eb = nb[2 * MU + 1];
    if (eb >= 0) {
        const int idx = eb & kNbrMask;
        const AC sg = (eb & kNbrSign) ? (AC)-1 : (AC)1;
        AC u[18];
        load_link(lk + ((int64_t)(other0 + idx) * 4 + MU) * 18, u);
        hop_term_g<MU, false, SP, AC, G>(acc, in, cs, (int64_t)idx * nr, u, sg);
    }
}

// --------------------------------------------------------------- hop

template <typename SP, typename LK, typename AC, int G>
__global__ void __launch_bounds__(kTile) k_hop(BlkArgs ba, HopArgs ha)
{
    __shared__ double red[G][kTile];
    const Item it = item_of(ba);
    const int nr = ba.n_rhs;
    const int p = ha.parity;
    double dv[G][kNRed];
#pragma unroll
    for (int j = 0; j < G; j++)
#pragma unroll
        for (int k = 0; k < kNRed; k++) dv[j][k] = 0;
    if (it.live) {
        const int hb = ba.h[it.b];
        const int32_t *nbp = ba.nbr + ba.nbr_off[it.b] + (int64_t)(p * hb + it.site) * 8;
        int32_t nb[8];
        {
            const int4 *q = reinterpret_cast<const int4 *>(nbp);
            const int4 a0 = q[0], a1 = q[1];
            nb[0] = a0.x; nb[1] = a0.y; nb[2] = a0.z; nb[3] = a0.w;
            nb[4] = a1.x; nb[5] = a1.y; nb[6] = a1.z; nb[7] = a1.w;
        }
        const LK *lk = reinterpret_cast<const LK *>(ha.links) + ba.soff[it.b] * 72;
        // input pointer at this block and rhs group; neighbour sites add idx * nr
        const SP *in = reinterpret_cast<const SP *>(ha.in) + (ba.soff[it.b] >> 1) * 24 * nr + (int64_t)it.rg * G;
        AC acc[G][24];
#pragma unroll
        for (int j = 0; j < G; j++)
#pragma unroll
            for (int c = 0; c < 24; c++) acc[j][c] = 0;
        const int slot = p * hb + it.site;
        const int other0 = (1 - p) * hb;
        hop_dir<0, SP, LK, AC, G>(acc, nb, in, it.cs, nr, lk, slot, other0);
        hop_dir<1, SP, LK, AC, G>(acc, nb, in, it.cs, nr, lk, slot, other0);
        hop_dir<2, SP, LK, AC, G>(acc, nb, in, it.cs, nr, lk, slot, other0);
        hop_dir<3, SP, LK, AC, G>(acc, nb, in, it.cs, nr, lk, slot, other0);

        SP *out = reinterpret_cast<SP *>(ha.out) + it.off;
        const SP *self = ha.self ? reinterpret_cast<const SP *>(ha.self) + it.off : nullptr;
        const SP *add = ha.add ? reinterpret_cast<const SP *>(ha.add) + it.off : nullptr;
        const SP *aux = ha.aux ? reinterpret_cast<const SP *>(ha.aux) + it.off : nullptr;
        const AC ch = (AC)ha.c_hop, cself = (AC)ha.c_self, cadd = (AC)ha.c_add;
#pragma unroll
        for (int k = 0; k < 12; k++) {
            SP o[2][G], sv[2][G], av[2][G];
#pragma unroll
            for (int ri = 0; ri < 2; ri++) {
                const int c = 2 * k + ri;
                AC v[G];
#pragma unroll
                for (int j = 0; j < G; j++) v[j] = ch * acc[j][c];
                if (self) {
                    ldv<SP, G>(self + c * it.cs, sv[ri]);
#pragma unroll
                    for (int j = 0; j < G; j++) v[j] += cself * (AC)sv[ri][j];
                }
                if (add) {
                    SP w[G];
                    ldv<SP, G>(add + c * it.cs, w);
#pragma unroll
                    for (int j = 0; j < G; j++) v[j] += cadd * (AC)w[j];
                }
#pragma unroll
                for (int j = 0; j < G; j++) o[ri][j] = (SP)v[j];
                stv<SP, G>(out + c * it.cs, o[ri]);
                if (ha.dot_mode == kDotAuxOut) ldv<SP, G>(aux + c * it.cs, av[ri]);
            }
#pragma unroll
            for (int j = 0; j < G; j++) {
                const double ore = (double)o[0][j], oim = (double)o[1][j];
                if (ha.dot_mode == kDotAuxOut) {
                    const double are = (double)av[0][j], aim = (double)av[1][j];
                    dv[j][0] += are * ore + aim * oim;
                    dv[j][1] += are * oim - aim * ore;
                } else if (ha.dot_mode == kDotOutSelfOutOut) {
                    const double sre = (double)sv[0][j], sim = (double)sv[1][j];
                    dv[j][0] += ore * sre + oim * sim;
                    dv[j][1] += ore * sim - oim * sre;
                    dv[j][2] += ore * ore + oim * oim;
                } else if (ha.dot_mode == kDotOutOut) {
                    dv[j][0] += ore * ore + oim * oim;
                }
            }
        }
    }
    if (ha.dot_mode != kDotNone) {
        const int nred = ha.dot_mode == kDotAuxOut ? 2 : (ha.dot_mode == kDotOutSelfOutOut ? 3 : 1);
        tile_reduce<G>(red, dv, nred, ha.partial, it, nr);
    }
}

template <int G>
static hipError_t launch_hop_g(const BlkArgs &ba, const HopArgs &ha, dd_prec prec, hipStream_t s)
{
    dim3 g(ba.ntiles), t(kTile);
    switch (prec) {
    case DD_F64: hipLaunchKernelGGL((k_hop<double, double, double, G>), g, t, 0, s, ba, ha); break;
    case DD_F32: hipLaunchKernelGGL((k_hop<float, float, float, G>), g, t, 0, s, ba, ha); break;
    case DD_BF16: hipLaunchKernelGGL((k_hop<float, uint16_t, float, G>), g, t, 0, s, ba, ha); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_hop(const BlkArgs &ba, const HopArgs &ha, dd_prec prec, hipStream_t s)
{
    if (ba.ntiles <= 0) return hipSuccess;
    switch (ba.g) {
    case 1: return launch_hop_g<1>(ba, ha, prec, s);
    case 2: return launch_hop_g<2>(ba, ha, prec, s);
    case 4: return launch_hop_g<4>(ba, ha, prec, s);
    default: return hipErrorInvalidValue;
    }
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

// boundary layout [r][q][24] (q = block site, box-local canonical) <-> half fields.
// Thread t -> (eo block site q = t / n_rhs, rhs r = t % n_rhs): consecutive
// threads write consecutive half-field addresses; each thread moves one
// 192-byte spinor record of the boundary layout with 16-byte accesses.
template <typename SP, bool PACK>
__global__ void __launch_bounds__(256) k_spinor_xfer(PackGeom g, double *ext_f, SP *even, SP *odd,
                                                    int nr, int64_t total)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= total * nr) return;
    const int64_t q = t / nr;  // block site in eo order
    const int r = (int)(t - q * nr);
    const int b = find_block(g.soff, g.nb, q);
    const int s = (int)(q - g.soff[b]);
    const int hb = g.h[b];
    const int p = s >= hb;
    const int site = s - p * hb;
    const int y = g.perm[g.perm_off[b] + s];
    double2 *e = reinterpret_cast<double2 *>(ext_f + ((int64_t)r * total + g.soff[b] + y) * 24);
    SP *hf = (p ? odd : even) + (g.soff[b] >> 1) * 24 * nr + (int64_t)site * nr + r;
    const int64_t cs = (int64_t)hb * nr;
#pragma unroll
    for (int k = 0; k < 12; k++) {
        if constexpr (PACK) {
            const double2 v = e[k];
            hf[(2 * k) * cs] = (SP)v.x;
            hf[(2 * k + 1) * cs] = (SP)v.y;
        } else {
            e[k] = make_double2((double)hf[(2 * k) * cs], (double)hf[(2 * k + 1) * cs]);
        }
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
//
// Same (site, G rhs) decomposition as the hop.  Pairs that are no longer
// active keep their x (the update is selected away), everything else is
// computed unconditionally: pairs never mix, so values of frozen pairs do
// not reach active ones.

template <int G>
__device__ __forceinline__ void pair_flags(const BlkArgs &ba, const Item &it, const int32_t *active, bool (&act)[G],
                                           bool &any)
{
    any = false;
#pragma unroll
    for (int j = 0; j < G; j++) {
        act[j] = it.live && active[(it.rg * G + j) * ba.nb + it.b] != 0;
        any = any || act[j];
    }
}

// x_p += e_p for the pairs still above tolerance (FP64 accumulator)
template <typename SE, int G>
__global__ void __launch_bounds__(kTile) k_accum(BlkArgs ba, double *x, const SE *e, const int32_t *active)
{
    const Item it = item_of(ba);
    bool act[G], any;
    pair_flags<G>(ba, it, active, act, any);
    if (!any) return;
    for (int c = 0; c < 24; c++) {
        double xv[G];
        SE ev[G];
        ldv<double, G>(x + it.off + c * it.cs, xv);
        ldv<SE, G>(e + it.off + c * it.cs, ev);
#pragma unroll
        for (int j = 0; j < G; j++)
            if (act[j]) xv[j] += (double)ev[j];
        stv<double, G>(x + it.off + c * it.cs, xv);
    }
}

// BiCGStab start: r = rh = p = rhs, x = 0; |rhs|^2 per (tile, rhs)
template <typename SP, int G>
__global__ void __launch_bounds__(kTile) k_bicg_init(BlkArgs ba, const SP *rhs, SP *r, SP *rh, SP *p, SP *x,
                                                     double *partial, const int32_t *outer_active)
{
    __shared__ double red[G][kTile];
    const Item it = item_of(ba);
    double dv[G][kNRed] = {};
    bool act[G], any;
    pair_flags<G>(ba, it, outer_active, act, any);
    if (any) {
        for (int c = 0; c < 24; c++) {
            const int64_t i = it.off + c * it.cs;
            SP v[G], z[G];
            ldv<SP, G>(rhs + i, v);
#pragma unroll
            for (int j = 0; j < G; j++) {
                z[j] = (SP)0;
                dv[j][0] += act[j] ? (double)v[j] * (double)v[j] : 0.0;
            }
            stv<SP, G>(r + i, v);
            stv<SP, G>(rh + i, v);
            stv<SP, G>(p + i, v);
            stv<SP, G>(x + i, z);
        }
    }
    tile_reduce<G>(red, dv, 1, partial, it, ba.n_rhs);
}

template <int G>
__device__ __forceinline__ void load_coef(const double *arr, const BlkArgs &ba, const Item &it, double (&re)[G],
                                          double (&im)[G])
{
#pragma unroll
    for (int j = 0; j < G; j++) {
        const int pr = (it.rg * G + j) * ba.nb + it.b;
        re[j] = arr[2 * pr];
        im[j] = arr[2 * pr + 1];
    }
}

// s = r - alpha v
template <typename SP, int G>
__global__ void __launch_bounds__(kTile) k_bicg_s(BlkArgs ba, const SP *r, const SP *v, SP *s, PairState ps)
{
    const Item it = item_of(ba);
    bool act[G], any;
    pair_flags<G>(ba, it, ps.active, act, any);
    if (!any) return;
    double ar[G], ai[G];
    load_coef<G>(ps.alpha, ba, it, ar, ai);
#pragma unroll 2
    for (int k = 0; k < 12; k++) {
        const int64_t i0 = it.off + (2 * k) * it.cs, i1 = i0 + it.cs;
        SP vr[G], vi[G], rr[G], ri[G], sr[G], si[G];
        ldv<SP, G>(v + i0, vr);
        ldv<SP, G>(v + i1, vi);
        ldv<SP, G>(r + i0, rr);
        ldv<SP, G>(r + i1, ri);
#pragma unroll
        for (int j = 0; j < G; j++) {
            const SP a_r = (SP)ar[j], a_i = (SP)ai[j];
            sr[j] = rr[j] - (a_r * vr[j] - a_i * vi[j]);
            si[j] = ri[j] - (a_r * vi[j] + a_i * vr[j]);
        }
        stv<SP, G>(s + i0, sr);
        stv<SP, G>(s + i1, si);
    }
}

// x += alpha p + omega s (active pairs);  r = s - omega t;  <rh, r>, |r|^2 per (tile, rhs)
template <typename SP, int G>
__global__ void __launch_bounds__(kTile) k_bicg_xr(BlkArgs ba, SP *x, const SP *p, const SP *s, const SP *t, SP *r,
                                                   const SP *rh, double *partial, PairState ps)
{
    __shared__ double red[G][kTile];
    const Item it = item_of(ba);
    double dv[G][kNRed] = {};
    bool act[G], any;
    pair_flags<G>(ba, it, ps.active, act, any);
    if (any) {
        double ar[G], ai[G], wr[G], wi[G];
        load_coef<G>(ps.alpha, ba, it, ar, ai);
        load_coef<G>(ps.omega, ba, it, wr, wi);
        for (int k = 0; k < 12; k++) {
            const int64_t i0 = it.off + (2 * k) * it.cs, i1 = i0 + it.cs;
            SP pr[G], pi[G], sr[G], si[G], tr[G], ti[G], xr[G], xi[G], nr_[G], ni_[G], hr[G], hi[G];
            ldv<SP, G>(p + i0, pr);
            ldv<SP, G>(p + i1, pi);
            ldv<SP, G>(s + i0, sr);
            ldv<SP, G>(s + i1, si);
            ldv<SP, G>(t + i0, tr);
            ldv<SP, G>(t + i1, ti);
            ldv<SP, G>(x + i0, xr);
            ldv<SP, G>(x + i1, xi);
            ldv<SP, G>(rh + i0, hr);
            ldv<SP, G>(rh + i1, hi);
#pragma unroll
            for (int j = 0; j < G; j++) {
                const SP a_r = (SP)ar[j], a_i = (SP)ai[j], w_r = (SP)wr[j], w_i = (SP)wi[j];
                const SP nxr = xr[j] + (a_r * pr[j] - a_i * pi[j]) + (w_r * sr[j] - w_i * si[j]);
                const SP nxi = xi[j] + (a_r * pi[j] + a_i * pr[j]) + (w_r * si[j] + w_i * sr[j]);
                xr[j] = act[j] ? nxr : xr[j];
                xi[j] = act[j] ? nxi : xi[j];
                nr_[j] = sr[j] - (w_r * tr[j] - w_i * ti[j]);
                ni_[j] = si[j] - (w_r * ti[j] + w_i * tr[j]);
                const double a = (double)hr[j], b = (double)hi[j], c = (double)nr_[j], d = (double)ni_[j];
                dv[j][0] += a * c + b * d;
                dv[j][1] += a * d - b * c;
                dv[j][2] += c * c + d * d;
            }
            stv<SP, G>(x + i0, xr);
            stv<SP, G>(x + i1, xi);
            stv<SP, G>(r + i0, nr_);
            stv<SP, G>(r + i1, ni_);
        }
    }
    tile_reduce<G>(red, dv, 3, partial, it, ba.n_rhs);
}

// p = r + beta (p - omega v)
template <typename SP, int G>
__global__ void __launch_bounds__(kTile) k_bicg_p(BlkArgs ba, const SP *r, const SP *v, SP *p, PairState ps)
{
    const Item it = item_of(ba);
    bool act[G], any;
    pair_flags<G>(ba, it, ps.active, act, any);
    if (!any) return;
    double br[G], bi[G], wr[G], wi[G];
    load_coef<G>(ps.beta, ba, it, br, bi);
    load_coef<G>(ps.omega, ba, it, wr, wi);
#pragma unroll 2
    for (int k = 0; k < 12; k++) {
        const int64_t i0 = it.off + (2 * k) * it.cs, i1 = i0 + it.cs;
        SP vr[G], vi[G], pr[G], pi[G], rr[G], ri[G];
        ldv<SP, G>(v + i0, vr);
        ldv<SP, G>(v + i1, vi);
        ldv<SP, G>(p + i0, pr);
        ldv<SP, G>(p + i1, pi);
        ldv<SP, G>(r + i0, rr);
        ldv<SP, G>(r + i1, ri);
#pragma unroll
        for (int j = 0; j < G; j++) {
            const SP b_r = (SP)br[j], b_i = (SP)bi[j], w_r = (SP)wr[j], w_i = (SP)wi[j];
            const SP qr = pr[j] - (w_r * vr[j] - w_i * vi[j]);
            const SP qi = pi[j] - (w_r * vi[j] + w_i * vr[j]);
            pr[j] = rr[j] + (b_r * qr - b_i * qi);
            pi[j] = ri[j] + (b_r * qi + b_i * qr);
        }
        stv<SP, G>(p + i0, pr);
        stv<SP, G>(p + i1, pi);
    }
}

hipError_t launch_accum(const BlkArgs &ba, double *x, const void *e, dd_prec ep, const int32_t *active,
                        hipStream_t st)
{
    if (ba.ntiles <= 0) return hipSuccess;
    dim3 g(ba.ntiles), t(kTile);
    const bool d = ep == DD_F64;
    switch (ba.g) {
    case 1:
        if (d) hipLaunchKernelGGL((k_accum<double, 1>), g, t, 0, st, ba, x, (const double *)e, active);
        else hipLaunchKernelGGL((k_accum<float, 1>), g, t, 0, st, ba, x, (const float *)e, active);
        break;
    case 2:
        if (d) hipLaunchKernelGGL((k_accum<double, 2>), g, t, 0, st, ba, x, (const double *)e, active);
        else hipLaunchKernelGGL((k_accum<float, 2>), g, t, 0, st, ba, x, (const float *)e, active);
        break;
    case 4:
        if (d) hipLaunchKernelGGL((k_accum<double, 4>), g, t, 0, st, ba, x, (const double *)e, active);
        else hipLaunchKernelGGL((k_accum<float, 4>), g, t, 0, st, ba, x, (const float *)e, active);
        break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename SP, int G>
static void launch_init_t(const BlkArgs &ba, const void *rhs, void *r, void *rh, void *p, void *x, double *partial,
                          const int32_t *oa, hipStream_t st)
{
    hipLaunchKernelGGL((k_bicg_init<SP, G>), dim3(ba.ntiles), dim3(kTile), 0, st, ba, (const SP *)rhs, (SP *)r,
                       (SP *)rh, (SP *)p, (SP *)x, partial, oa);
}
template <typename SP, int G>
static void launch_s_t(const BlkArgs &ba, const void *r, const void *v, void *s, const PairState &ps, hipStream_t st)
{
    hipLaunchKernelGGL((k_bicg_s<SP, G>), dim3(ba.ntiles), dim3(kTile), 0, st, ba, (const SP *)r, (const SP *)v,
                       (SP *)s, ps);
}
template <typename SP, int G>
static void launch_xr_t(const BlkArgs &ba, void *x, const void *p, const void *s, const void *t, void *r,
                        const void *rh, double *partial, const PairState &ps, hipStream_t st)
{
    hipLaunchKernelGGL((k_bicg_xr<SP, G>), dim3(ba.ntiles), dim3(kTile), 0, st, ba, (SP *)x, (const SP *)p,
                       (const SP *)s, (const SP *)t, (SP *)r, (const SP *)rh, partial, ps);
}
template <typename SP, int G>
static void launch_p_t(const BlkArgs &ba, const void *r, const void *v, void *p, const PairState &ps, hipStream_t st)
{
    hipLaunchKernelGGL((k_bicg_p<SP, G>), dim3(ba.ntiles), dim3(kTile), 0, st, ba, (const SP *)r, (const SP *)v,
                       (SP *)p, ps);
}

#define DD_DISPATCH(FN, SPREC, ...)                                                   \
    do {                                                                              \
        if (ba.ntiles <= 0) return hipSuccess;                                        \
        const bool d_ = (SPREC) == DD_F64;                                            \
        switch (ba.g) {                                                               \
        case 1: if (d_) FN<double, 1>(__VA_ARGS__); else FN<float, 1>(__VA_ARGS__); break; \
        case 2: if (d_) FN<double, 2>(__VA_ARGS__); else FN<float, 2>(__VA_ARGS__); break; \
        case 4: if (d_) FN<double, 4>(__VA_ARGS__); else FN<float, 4>(__VA_ARGS__); break; \
        default: return hipErrorInvalidValue;                                         \
        }                                                                             \
        return hipGetLastError();                                                     \
    } while (0)

hipError_t launch_bicg_init(const BlkArgs &ba, dd_prec sp, const void *rhs, void *r, void *rh, void *p, void *x,
                            double *partial, const int32_t *outer_active, hipStream_t st)
{
    DD_DISPATCH(launch_init_t, sp, ba, rhs, r, rh, p, x, partial, outer_active, st);
}

hipError_t launch_bicg_s(const BlkArgs &ba, dd_prec sp, const void *r, const void *v, void *s, const PairState &ps,
                         hipStream_t st)
{
    DD_DISPATCH(launch_s_t, sp, ba, r, v, s, ps, st);
}

hipError_t launch_bicg_xr(const BlkArgs &ba, dd_prec sp, void *x, const void *p, const void *s, const void *tv,
                          void *r, const void *rh, double *partial, const PairState &ps, hipStream_t st)
{
    DD_DISPATCH(launch_xr_t, sp, ba, x, p, s, tv, r, rh, partial, ps, st);
}

hipError_t launch_bicg_p(const BlkArgs &ba, dd_prec sp, const void *r, const void *v, void *p, const PairState &ps,
                         hipStream_t st)
{
    DD_DISPATCH(launch_p_t, sp, ba, r, v, p, ps, st);
}

// ------------------------------------------------------ per-pair scalars
//
// One wavefront per (block, rhs) pair: the lanes stride over the block's
// tiles, a fixed butterfly sums them (the same order on every run), and lane
// 0 updates the pair's recurrence scalars in FP64.

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

template <int NK>
__device__ __forceinline__ void pair_sums(const BlkArgs &ba, const double *partial, int b, int r, int lane,
                                          double (&s)[NK])
{
#pragma unroll
    for (int k = 0; k < NK; k++) s[k] = 0;
    const int t1 = ba.blk_tile0[b + 1];
    for (int t = ba.blk_tile0[b] + lane; t < t1; t += 64)
#pragma unroll
        for (int k = 0; k < NK; k++) s[k] += partial[((int64_t)t * ba.n_rhs + r) * kNRed + k];
#pragma unroll
    for (int k = 0; k < NK; k++) s[k] = wave_sum(s[k]);
}

__device__ __forceinline__ bool finite(double v) { return isfinite(v); }

#define DD_PAIR_PROLOGUE(NP)                                                   \
    const int lane = threadIdx.x & 63;                                         \
    const int pair = (int)((blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6); \
    if (pair >= (NP)) return;                                                  \
    const int b = pair % ba.nb, r = pair / ba.nb;

__global__ void __launch_bounds__(256) k_sc_init(BlkArgs ba, const double *partial, PairState ps,
                                                 const int32_t *outer_active)
{
    DD_PAIR_PROLOGUE(ps.np)
    double s[1];
    pair_sums<1>(ba, partial, b, r, lane, s);
    if (lane != 0) return;
    if (!outer_active[pair]) {
        ps.active[pair] = 0;
        return;
    }
    const double bb = s[0];
    ps.bb[pair] = bb;
    ps.rr[pair] = bb;
    ps.rho[2 * pair] = bb;
    ps.rho[2 * pair + 1] = 0;
    ps.omega[2 * pair] = 1;
    ps.omega[2 * pair + 1] = 0;
    ps.active[pair] = (finite(bb) && bb > 0) ? 1 : 0;
    if (!finite(bb)) ps.flags[pair] |= 4;
}

__global__ void __launch_bounds__(256) k_sc_alpha(BlkArgs ba, const double *partial, PairState ps)
{
    DD_PAIR_PROLOGUE(ps.np)
    if (!ps.active[pair]) return;
    double s[2];
    pair_sums<2>(ba, partial, b, r, lane, s);
    if (lane != 0) return;
    const double vr = s[0], vi = s[1];
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

__global__ void __launch_bounds__(256) k_sc_omega(BlkArgs ba, const double *partial, PairState ps)
{
    DD_PAIR_PROLOGUE(ps.np)
    if (!ps.active[pair]) return;
    double s[3];
    pair_sums<3>(ba, partial, b, r, lane, s);
    if (lane != 0) return;
    const double tt = s[2];
    const double wr = s[0] / tt, wi = s[1] / tt;
    if (!(tt > 0) || !finite(wr) || !finite(wi)) {
        ps.active[pair] = 0;
        ps.flags[pair] |= 2;
        return;
    }
    ps.omega[2 * pair] = wr;
    ps.omega[2 * pair + 1] = wi;
}

__global__ void __launch_bounds__(256) k_sc_beta(BlkArgs ba, const double *partial, PairState ps, double tol2)
{
    DD_PAIR_PROLOGUE(ps.np)
    if (!ps.active[pair]) return;
    double s[3];
    pair_sums<3>(ba, partial, b, r, lane, s);
    if (lane != 0) return;
    const double nr_ = s[0], ni_ = s[1], rr = s[2];
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
__global__ void __launch_bounds__(256) k_sc_outer(BlkArgs ba, const double *pe, const double *po, int first,
                                                  double tol2, OuterState os, int np)
{
    DD_PAIR_PROLOGUE(np)
    double se[1], so[1];
    pair_sums<1>(ba, pe, b, r, lane, se);
    pair_sums<1>(ba, po, b, r, lane, so);
    if (lane != 0) return;
    const double rr = se[0] + so[0];
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

static inline dim3 pair_grid(int np) { return dim3((unsigned)((np + 3) / 4)); }

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
hipError_t launch_sc_beta(const BlkArgs &ba, const double *partial, const PairState &ps, double tol, hipStream_t s)
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
