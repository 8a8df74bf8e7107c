// Device-side building blocks of the Wilson hopping stencil shared by the
// kernels of libdd: buffer addressing, link loads, the spin projectors of
// the chiral basis and the projected hop term of one direction.
#pragma once

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

// Buffer addressing: a descriptor holds a wave-uniform base and size; a load
// takes a per-lane byte offset (VGPR) plus a wave-uniform byte offset (SGPR),
// so the 24 components of a spinor (uniform stride) share one VGPR offset and
// cost no address arithmetic.  Accesses beyond the size read 0 / are dropped.
struct Buf {
    __amdgpu_buffer_rsrc_t r;
};
__device__ __forceinline__ Buf make_buf(const void *p, uint32_t bytes)
{
    return Buf{__builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, (int)bytes, 0x00020000)};
}
// Cache policy of a buffer access (the instruction's cache-policy bits on
// gfx950; bit 1 = non-temporal).  kStream marks single-use spinor streams,
// so that they do not push out of L2 and the MALL the links that every rhs
// group of a launch reads again; kKeep (no hint) is for data that a launch
// re-reads, such as a Krylov basis.
enum : int { kKeep = 0, kStream = 2 };

template <typename T, int CP = kStream>
__device__ __forceinline__ T bload(const Buf &b, uint32_t voff, uint32_t soff)
{
    if constexpr (sizeof(T) == 8) {
        return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(b.r, (int)voff, (int)soff, CP));
    } else if constexpr (sizeof(T) == 4) {
        return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(b.r, (int)voff, (int)soff, CP));
    } else {
        static_assert(sizeof(T) == 2, "2, 4 or 8 byte elements");
        return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b16(b.r, (int)voff, (int)soff, CP));
    }
}
template <typename T, int CP = kStream>
__device__ __forceinline__ void bstore(const Buf &b, T v, uint32_t voff, uint32_t soff)
{
    if constexpr (sizeof(T) == 8) {
        using u2 = __attribute__((ext_vector_type(2))) uint32_t;
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u2, v), b.r, (int)voff, (int)soff, CP);
    } else {
        static_assert(sizeof(T) == 4, "4 or 8 byte elements");
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), b.r, (int)voff, (int)soff, CP);
    }
}

// Link layout per block: element (site slot s, mu, complex entry k = 3*row + col
// of rows 0 and 1, re/im) at soff[b]*48 + ((mu*6 + k)*S_b + s)*2 + ri.
// Consecutive slots are adjacent, so a wavefront reading entry k of one
// direction for consecutive sites touches one line.  load_link: voff = byte
// offset of the slot's pair, soff = byte offset of entry 0 of direction mu,
// kstride = bytes between entries; neg = the hop crosses the antiperiodic
// time edge (rows 0 and 1 are stored with that sign already).

// u[12..17] = s * conj(row0 x row1): row 2 of an SU(3) matrix, with the sign s
// of the stored rows
template <typename AC>
__device__ __forceinline__ void rebuild_row2(AC (&u)[18], bool neg)
{
    const AC sg = neg ? (AC)-1 : (AC)1;
#pragma unroll
    for (int c = 0; c < 3; c++) {
        const int c1 = (c + 1) % 3, c2 = (c + 2) % 3;
        // a_{c1} b_{c2} - a_{c2} b_{c1}, a = row 0, b = row 1
        const AC ar1 = u[2 * c1], ai1 = u[2 * c1 + 1], ar2 = u[2 * c2], ai2 = u[2 * c2 + 1];
        const AC br1 = u[6 + 2 * c1], bi1 = u[6 + 2 * c1 + 1], br2 = u[6 + 2 * c2], bi2 = u[6 + 2 * c2 + 1];
        const AC re = (ar1 * br2 - ai1 * bi2) - (ar2 * br1 - ai2 * bi1);
        const AC im = (ar1 * bi2 + ai1 * br2) - (ar2 * bi1 + ai2 * br1);
        u[12 + 2 * c] = sg * re;
        u[12 + 2 * c + 1] = -sg * im;
    }
}

template <typename AC>
__device__ __forceinline__ void load_link(const Buf &b, const double *, uint32_t voff, uint32_t soff,
                                          uint32_t kstride, AC (&u)[18], bool neg)
{
#pragma unroll
    for (int k = 0; k < kLinkK; k++) {
        const auto q = __builtin_amdgcn_raw_buffer_load_b128(b.r, (int)voff, (int)(soff + k * kstride), 0);
        u[2 * k] = (AC)__builtin_bit_cast(double, __builtin_shufflevector(q, q, 0, 1));
        u[2 * k + 1] = (AC)__builtin_bit_cast(double, __builtin_shufflevector(q, q, 2, 3));
    }
    if constexpr (kLinkK == 6) rebuild_row2(u, neg);
}
template <typename AC>
__device__ __forceinline__ void load_link(const Buf &b, const float *, uint32_t voff, uint32_t soff, uint32_t kstride,
                                          AC (&u)[18], bool neg)
{
#pragma unroll
    for (int k = 0; k < kLinkK; k++) {
        // take the 8 bytes as one integer: indexing the returned vector lets
        // the compiler shrink the load to its first dword
        const uint64_t q =
            __builtin_bit_cast(uint64_t, __builtin_amdgcn_raw_buffer_load_b64(b.r, (int)voff, (int)(soff + k * kstride), 0));
        u[2 * k] = (AC)__uint_as_float((uint32_t)q);
        u[2 * k + 1] = (AC)__uint_as_float((uint32_t)(q >> 32));
    }
    if constexpr (kLinkK == 6) rebuild_row2(u, neg);
}
template <typename AC>
__device__ __forceinline__ void load_link(const Buf &b, const uint16_t *, uint32_t voff, uint32_t soff,
                                          uint32_t kstride, AC (&u)[18], bool neg)
{
#pragma unroll
    for (int k = 0; k < kLinkK; k++) {
        const uint32_t w = __builtin_amdgcn_raw_buffer_load_b32(b.r, (int)voff, (int)(soff + k * kstride), 0);
        u[2 * k] = (AC)bf16_to_f32(w & 0xffffu);
        u[2 * k + 1] = (AC)bf16_to_f32(w >> 16);
    }
    if constexpr (kLinkK == 6) rebuild_row2(u, neg);
}

// a * b + c in one rounding
__device__ __forceinline__ float fmad(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmad(double a, double b, double c) { return __builtin_fma(a, b, c); }

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

// ------------------------------------------------------------- vectors

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


// a value every lane of the wavefront holds: keep it in a scalar register
__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ int64_t uni64(int64_t v)
{
    const uint64_t u = (uint64_t)v;
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)u), hi = __builtin_amdgcn_readfirstlane((uint32_t)(u >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

// ------------------------------------------------------------- hop term

// Sources of a neighbour's spinor for the G rhs of a thread: global memory or
// the LDS copy of the tile's chunk.  load(comp, v) fills v with component comp.
// Offsets are 32-bit and relative to wave-uniform block bases.
template <typename SP, int G>
struct SrcGlobal {
    Buf b;          // the block's half field
    uint32_t voff;  // bytes to (rhs group, component 0, neighbour site)
    uint32_t cstr;  // bytes between components (h_b elements)
    __device__ __forceinline__ void load(int comp, SP (&v)[G]) const
    {
#pragma unroll
        for (int j = 0; j < G; j++) v[j] = bload<SP>(b, voff, (uint32_t)(j * 24 + comp) * cstr);
    }
};
template <typename SP, int G>
struct SrcLds {
    const SP *p;  // stage + lidx * G
    __device__ __forceinline__ void load(int comp, SP (&v)[G]) const { ldv<SP, G>(p + comp * kTile * G, v); }
};

// The upper half of the projected hop (1 -/+ gamma_mu) W psi_j for the G rhs:
// project the neighbour's spinor to the half spinor h (2 spins x 3 colours)
// and multiply by W = U (forward) or U^+ (backward); w[j][2*(3*s + a) + ri].
// The antiperiodic time sign is part of the link.
template <int MU, bool FWD, typename SP, typename AC, int G, typename SRC>
__device__ __forceinline__ void hop_half(AC (&w)[G][12], const SRC &src, const AC (&u)[18])
{
    using P = Proj<MU, FWD>;
    AC h[G][2][3][2];
#pragma unroll
    for (int c = 0; c < 3; c++) {
        SP v[4][2][G];
#pragma unroll
        for (int sp = 0; sp < 4; sp++)
#pragma unroll
            for (int ri = 0; ri < 2; ri++) src.load(2 * (3 * sp + c) + ri, v[sp][ri]);
#pragma unroll
        for (int j = 0; j < G; j++) {
            AC re, im;
            cmul_code<P::a0>((AC)v[P::pi0][0][j], (AC)v[P::pi0][1][j], re, im);
            h[j][0][c][0] = (AC)v[0][0][j] + re;
            h[j][0][c][1] = (AC)v[0][1][j] + im;
            cmul_code<P::a1>((AC)v[P::pi1][0][j], (AC)v[P::pi1][1][j], re, im);
            h[j][1][c][0] = (AC)v[1][0][j] + re;
            h[j][1][c][1] = (AC)v[1][1][j] + im;
        }
    }
#pragma unroll
    for (int j = 0; j < G; j++) {
        // explicit fused multiply-add chains: one multiply and five FMAs per
        // real component
#pragma unroll
        for (int s = 0; s < 2; s++)
#pragma unroll
            for (int a = 0; a < 3; a++) {
                AC re, im;
#pragma unroll
                for (int c = 0; c < 3; c++) {
                    AC ur, ui;
                    if constexpr (FWD) {  // U[a][c]
                        ur = u[2 * (3 * a + c)];
                        ui = u[2 * (3 * a + c) + 1];
                    } else {              // conj(U[c][a])
                        ur = u[2 * (3 * c + a)];
                        ui = -u[2 * (3 * c + a) + 1];
                    }
                    const AC hr = h[j][s][c][0], hi = h[j][s][c][1];
                    if (c == 0) {
                        re = ur * hr;
                        im = ur * hi;
                    } else {
                        re = fmad(ur, hr, re);
                        im = fmad(ur, hi, im);
                    }
                    re = fmad(-ui, hi, re);
                    im = fmad(ui, hr, im);
                }
                w[j][2 * (3 * s + a)] = re;
                w[j][2 * (3 * s + a) + 1] = im;
            }
    }
}

// acc += the full spinor of a hop from its upper half w: (W_0, W_1, b_0
// W_{sig_0}, b_1 W_{sig_1}).
template <int MU, bool FWD, typename AC>
__device__ __forceinline__ void hop_expand(AC (&acc)[24], const AC (&w)[12])
{
    using P = Proj<MU, FWD>;
#pragma unroll
    for (int a = 0; a < 3; a++) {
        acc[2 * a] += w[2 * a];
        acc[2 * a + 1] += w[2 * a + 1];
        acc[2 * (3 + a)] += w[2 * (3 + a)];
        acc[2 * (3 + a) + 1] += w[2 * (3 + a) + 1];
        AC re, im;
        cmul_code<P::b0>(w[2 * (3 * P::s0 + a)], w[2 * (3 * P::s0 + a) + 1], re, im);
        acc[2 * (6 + a)] += re;
        acc[2 * (6 + a) + 1] += im;
        cmul_code<P::b1>(w[2 * (3 * P::s1 + a)], w[2 * (3 * P::s1 + a) + 1], re, im);
        acc[2 * (9 + a)] += re;
        acc[2 * (9 + a) + 1] += im;
    }
}

// acc[j] += (1 -/+ gamma_mu) W psi_j for the G rhs.
template <int MU, bool FWD, typename SP, typename AC, int G, typename SRC>
__device__ __forceinline__ void hop_term(AC (&acc)[G][24], const SRC &src, const AC (&u)[18])
{
    AC w[G][12];
    hop_half<MU, FWD, SP, AC, G>(w, src, u);
#pragma unroll
    for (int j = 0; j < G; j++) hop_expand<MU, FWD, AC>(acc[j], w[j]);
}

struct HopCtx {
    int h0, tv;          // staged other-parity sites [h0, h0 + tv)
    int grp_off;         // element offset of the thread's rhs group in the block's half field
    int slot_self, other0;
    uint32_t cstr;       // bytes between spinor components (h_b elements)
    uint32_t kstr;       // bytes between link entries (S_b pairs)
    Buf in_b, lk_b;      // the block's input half field and links
};

// Adds the hop along direction MU (forward or backward) to acc when the
// neighbour entry e is not dropped.  With LDS, neighbours inside the staged
// chunk are read from `stage`; all others from global memory.
template <int MU, bool FWD, typename SP, typename LK, typename AC, int G, bool LDS = true>
__device__ __forceinline__ void hop_one(AC (&acc)[G][24], int32_t e, const SP *stage, const HopCtx &hc)
{
    if (e < 0) return;
    const int idx = e & kNbrMask;
    AC u[18];
    const int slot = FWD ? hc.slot_self : hc.other0 + idx;
    load_link(hc.lk_b, (const LK *)nullptr, (uint32_t)slot * 2 * (uint32_t)sizeof(LK), MU * kLinkK * hc.kstr, hc.kstr, u,
              (e & kNbrSign) != 0);
    const int lidx = idx - hc.h0;
    if (LDS && (unsigned)lidx < (unsigned)hc.tv) {
        const SrcLds<SP, G> src{stage + lidx * G};
        hop_term<MU, FWD, SP, AC, G>(acc, src, u);
    } else {
        const SrcGlobal<SP, G> src{hc.in_b, (uint32_t)(hc.grp_off + idx) * (uint32_t)sizeof(SP), hc.cstr};
        hop_term<MU, FWD, SP, AC, G>(acc, src, u);
    }
}

// Adds the hop along MU (forward or backward) with the neighbour's spinor at
// LDS position lidx of `stage` and the link at `slot` (the site's own slot
// forward, the neighbour's backward), when the entry e is not dropped.
template <int MU, bool FWD, typename SP, typename LK, typename AC, int G>
__device__ __forceinline__ void hop_at(AC (&acc)[G][24], int32_t e, const SP *stage, int lidx, int slot,
                                       const HopCtx &hc)
{
    if (e < 0) return;
    AC u[18];
    load_link(hc.lk_b, (const LK *)nullptr, (uint32_t)slot * 2 * (uint32_t)sizeof(LK), MU * kLinkK * hc.kstr, hc.kstr, u,
              (e & kNbrSign) != 0);
    const SrcLds<SP, G> src{stage + lidx * G};
    hop_term<MU, FWD, SP, AC, G>(acc, src, u);
}

// The upper half (hop_half) of the hop along MU with the neighbour's spinor
// at LDS position lidx and the link at `slot`; zero when e is dropped.
template <int MU, bool FWD, typename SP, typename LK, typename AC, int G>
__device__ __forceinline__ void hop_half_at(AC (&w)[G][12], int32_t e, const SP *stage, int lidx, int slot,
                                            const HopCtx &hc)
{
    if (e < 0) {
#pragma unroll
        for (int j = 0; j < G; j++)
#pragma unroll
            for (int i = 0; i < 12; i++) w[j][i] = 0;
        return;
    }
    AC u[18];
    load_link(hc.lk_b, (const LK *)nullptr, (uint32_t)slot * 2 * (uint32_t)sizeof(LK), MU * kLinkK * hc.kstr, hc.kstr, u,
              (e & kNbrSign) != 0);
    const SrcLds<SP, G> src{stage + lidx * G};
    hop_half<MU, FWD, SP, AC, G>(w, src, u);
}

// ------------------------------------------------------------- x0-walk

// x0-walk of the hop over one block and one rhs: a workgroup walks the
// block's x0-slices; thread k owns eo site k of every slice (hs sites per
// parity and slice).  The eo order makes the x0-neighbour of a site the same
// position k of the adjacent slice of the other parity, so each input slice
// is read from global memory once: staged in LDS, it feeds the hops along
// 1..3 of its own output slice (neighbours inside the slice) and the x0 hops
// of the two adjacent output slices at position k.  One accumulator rides
// along: it holds output slice q-1 until its x0+ hop arrives with input
// slice q, and the x0- hop of output slice q+1, computed from input slice q,
// waits as its 12-real upper half.

struct WalkPos {
    int p, hb, hs, k, s0, s1;  // output parity, sites per parity, per slice; thread; output slices [s0, s1)
    const int32_t *nbt;        // neighbour table of the output parity
};

// Loads input slice q of the thread's G rhs at its site (component c of rhs
// j in v[c][j]).
template <typename SP, int G>
__device__ __forceinline__ void walk_load(SP (&v)[24][G], const HopCtx &hc, int q, int hs, int k)
{
    const uint32_t vo = (uint32_t)(hc.grp_off + q * hs + k) * (uint32_t)sizeof(SP);
#pragma unroll
    for (int j = 0; j < G; j++)
#pragma unroll
        for (int c = 0; c < 24; c++) v[c][j] = bload<SP>(hc.in_b, vo, (uint32_t)(j * 24 + c) * hc.cstr);
}

// Copies the thread's spinors v of one input slice into the stage
// (component-major, kTile sites per component, the G rhs of a site adjacent).
template <typename SP, int G>
__device__ __forceinline__ void walk_stage(SP *stage, const SP (&v)[24][G], int k)
{
#pragma unroll
    for (int c = 0; c < 24; c++) stv<SP, G>(stage + (c * kTile + k) * G, v[c]);
}

// Input slice q is in the stage.  acc holds output slice q-1: its x0+ hop is
// added and epi(acc, h) finishes it (site h) when it belongs to [s0, s1);
// acc then restarts as output slice q (carry: the upper half of its x0- hop)
// with the hops along 1..3, and carry becomes the x0- half of output slice
// q+1.  G rhs per thread share the link loads and the rebuilt rows.
template <typename SP, typename LK, typename AC, int G, typename EPI>
__device__ __forceinline__ void walk_step(AC (&acc)[G][24], AC (&carry)[G][12], int q, const WalkPos &w,
                                          const SP *stage, const HopCtx &hc, EPI &&epi)
{
    if (q - 1 >= w.s0) {
        const int h = (q - 1) * w.hs + w.k;
        hop_at<0, true, SP, LK, AC, G>(acc, w.nbt[h * 8], stage, w.k, w.p * w.hb + h, hc);
        epi(acc, h);
    }
    if (q >= w.s0 && q < w.s1) {
#pragma unroll
        for (int j = 0; j < G; j++) {
#pragma unroll
            for (int c = 0; c < 24; c++) acc[j][c] = 0;
            hop_expand<0, false, AC>(acc[j], carry[j]);
        }
        const int h = q * w.hs + w.k, base = q * w.hs, oth = (1 - w.p) * w.hb, own = w.p * w.hb + h;
        const int4 *t4 = reinterpret_cast<const int4 *>(w.nbt + h * 8);
        const int4 a0 = t4[0], a1 = t4[1];
        const int32_t nb[6] = {a0.z, a0.w, a1.x, a1.y, a1.z, a1.w};
        int li[6];
#pragma unroll
        for (int i = 0; i < 6; i++) li[i] = (nb[i] & kNbrMask) - base;
        hop_at<1, true, SP, LK, AC, G>(acc, nb[0], stage, li[0], own, hc);
        hop_at<1, false, SP, LK, AC, G>(acc, nb[1], stage, li[1], oth + base + li[1], hc);
        hop_at<2, true, SP, LK, AC, G>(acc, nb[2], stage, li[2], own, hc);
        hop_at<2, false, SP, LK, AC, G>(acc, nb[3], stage, li[3], oth + base + li[3], hc);
        hop_at<3, true, SP, LK, AC, G>(acc, nb[4], stage, li[4], own, hc);
        hop_at<3, false, SP, LK, AC, G>(acc, nb[5], stage, li[5], oth + base + li[5], hc);
    }
    if (q + 1 < w.s1) {
        const int h = (q + 1) * w.hs + w.k;
        hop_half_at<0, false, SP, LK, AC, G>(carry, w.nbt[h * 8 + 1], stage, w.k, (1 - w.p) * w.hb + q * w.hs + w.k,
                                             hc);
    }
}

// The whole walk over output slices [w.s0, w.s1) (input slices one beyond
// each end when they exist).  Every thread of the workgroup calls it (it has
// barriers); threads k >= hs only take part in those.  ld(q, v) produces the
// thread's spinors of input slice q (every slice in [max(s0-1, 0),
// min(s1+1, ns)) once, in order); epi(acc, h) writes output site h of the
// thread's G rhs.
template <typename SP, typename LK, typename AC, int G, typename EPI, typename LD>
__device__ __forceinline__ void walk_run(const WalkPos &w, int ns, SP *stage, const HopCtx &hc, EPI &&epi, LD &&ld)
{
    const int qa = max(w.s0 - 1, 0), qb = min(w.s1 + 1, ns);
    const bool live = w.k < w.hs;
    AC acc[G][24], carry[G][12];
#pragma unroll
    for (int j = 0; j < G; j++) {
#pragma unroll
        for (int c = 0; c < 24; c++) acc[j][c] = 0;
#pragma unroll
        for (int c = 0; c < 12; c++) carry[j][c] = 0;
    }
    for (int q = qa; q < qb; q++) {
        if (live) {
            SP v[24][G];
            ld(q, v);
            walk_stage<SP, G>(stage, v, w.k);
        }
        __syncthreads();
        if (live) walk_step<SP, LK, AC, G>(acc, carry, q, w, stage, hc, epi);
        __syncthreads();
    }
    // the block's last slice has no x0+ neighbour: when the walk ends there,
    // its output is finished here
    if (live && qb == w.s1) epi(acc, (w.s1 - 1) * w.hs + w.k);
}

// The walk with the input slices read from hc.in_b.
template <typename SP, typename LK, typename AC, int G, typename EPI>
__device__ __forceinline__ void walk_run(const WalkPos &w, int ns, SP *stage, const HopCtx &hc, EPI &&epi)
{
    walk_run<SP, LK, AC, G>(w, ns, stage, hc, epi,
                            [&](int q, SP (&v)[24][G]) { walk_load<SP, G>(v, hc, q, w.hs, w.k); });
}

// Dhat-type product in one pass over a block's x0-slices, one rhs per
// thread: out = epilogue of H_eo (H_oe in) on the even sites.  Two walks of
// the same workgroup (wodd over the odd output sites, weven over the even
// ones, both over all ns slices): step q stages input slice q (ld(q, v)) in
// sa, which finishes slice q-1 of the odd intermediate; that slice goes to
// sb (rounded to SP, as a stored field would be) and the second walk takes
// it, finishing output slice q-2 with epi(acc, h).  The intermediate never
// leaves LDS.  Two barriers per step: the second walk's reads of sb come
// before the next writes of sb by the first barrier of the next step, and
// the first walk's reads of sa before the next staging by the second.
// With alive false the thread only takes part in the barriers (a workgroup
// walking several rhs, one of which has nothing to do).
// xf(a, h) transforms each finished intermediate site h (odd parity) before it
// is stored (the clover term's A_oo^-1); the overload without it stores as is.
template <typename SP, typename LK, typename AC, typename LD, typename EPI, typename XF>
__device__ __forceinline__ void dhat_run(const WalkPos &wodd, const WalkPos &weven, int ns, SP *sa, SP *sb,
                                         const HopCtx &hc, LD &&ld, EPI &&epi, bool alive, XF &&xf)
{
    const int k = wodd.k, hs = wodd.hs;
    const bool live = alive && k < hs;
    AC acc1[1][24], car1[1][12], acc2[1][24], car2[1][12];
#pragma unroll
    for (int c = 0; c < 24; c++) acc1[0][c] = acc2[0][c] = 0;
#pragma unroll
    for (int c = 0; c < 12; c++) car1[0][c] = car2[0][c] = 0;
    auto to_sb = [&](const AC (&acc)[1][24], int h) {
        AC a[24];
#pragma unroll
        for (int c = 0; c < 24; c++) a[c] = acc[0][c];
        xf(a, h);
#pragma unroll
        for (int c = 0; c < 24; c++) sb[c * kTile + k] = (SP)a[c];
    };
    for (int q = 0; q <= ns; q++) {
        if (live && q < ns) {
            SP v[24][1];
            ld(q, v);
            walk_stage<SP, 1>(sa, v, k);
        }
        __syncthreads();
        if (live) {
            if (q < ns)
                walk_step<SP, LK, AC, 1>(acc1, car1, q, wodd, sa, hc, to_sb);
            else
                to_sb(acc1, (ns - 1) * hs + k);  // the last slice has no x0+ neighbour
        }
        __syncthreads();
        if (live && q >= 1) walk_step<SP, LK, AC, 1>(acc2, car2, q - 1, weven, sb, hc, epi);
    }
    if (live) epi(acc2, (ns - 1) * hs + k);
}

template <typename SP, typename LK, typename AC, typename LD, typename EPI>
__device__ __forceinline__ void dhat_run(const WalkPos &wodd, const WalkPos &weven, int ns, SP *sa, SP *sb,
                                         const HopCtx &hc, LD &&ld, EPI &&epi, bool alive = true)
{
    dhat_run<SP, LK, AC>(wodd, weven, ns, sa, sb, hc, ld, epi, alive, [](AC (&)[24], int) {});
}

// ------------------------------------------------------------ clover term

// v <- C v for one site's spinor v[24] (component 2 (3 s + c) + re/im): C is
// block diagonal in the chirality (spins 0, 1 and spins 2, 3 of the chiral
// basis), each block a hermitian 6x6 over (spin within the block, colour)
// stored as its 6 real diagonal entries, then the 15 complex entries above
// the diagonal row by row ((0,1), (0,2), .., (0,5), (1,2), .., (4,5)); the
// entries below are their conjugates.  Real k of the site's kCloverReals is
// at byte voff + k * kstr of cb (one site per voff, structure of arrays).
template <typename CT, typename AC>
__device__ __forceinline__ void clover_mul(AC (&v)[24], const Buf &cb, uint32_t voff, uint32_t kstr)
{
#pragma unroll
    for (int c = 0; c < 2; c++) {
        AC xr[6], xi[6], yr[6], yi[6];
#pragma unroll
        for (int i = 0; i < 6; i++) {
            xr[i] = v[2 * (6 * c + i)];
            xi[i] = v[2 * (6 * c + i) + 1];
            const AC d = (AC)bload<CT, kKeep>(cb, voff, (uint32_t)(c * kCloverHalf + i) * kstr);
            yr[i] = d * xr[i];
            yi[i] = d * xi[i];
        }
        int t = 0;
#pragma unroll
        for (int i = 0; i < 6; i++)
#pragma unroll
            for (int j = i + 1; j < 6; j++, t++) {
                const uint32_t k = (uint32_t)(c * kCloverHalf + 6 + 2 * t);
                const AC hr = (AC)bload<CT, kKeep>(cb, voff, k * kstr);
                const AC hi = (AC)bload<CT, kKeep>(cb, voff, (k + 1) * kstr);
                // y_i += h_ij x_j, y_j += conj(h_ij) x_i
                yr[i] = fmad(hr, xr[j], fmad(-hi, xi[j], yr[i]));
                yi[i] = fmad(hr, xi[j], fmad(hi, xr[j], yi[i]));
                yr[j] = fmad(hr, xr[i], fmad(hi, xi[i], yr[j]));
                yi[j] = fmad(hr, xi[i], fmad(-hi, xr[i], yi[j]));
            }
#pragma unroll
        for (int i = 0; i < 6; i++) {
            v[2 * (6 * c + i)] = yr[i];
            v[2 * (6 * c + i) + 1] = yi[i];
        }
    }
}

// ------------------------------------------------------ site geometry

// What the packing kernels need to map a block slot to its global site.
struct PackGeom {
    int L[4];
    int nb;
    const int64_t *soff;
    const int32_t *h;
    const int64_t *nbr_off;
    const int32_t *nbr;
    const int64_t *perm_off;
    const int32_t *perm;
    const int32_t *iperm;
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

inline PackGeom pack_geom(const dd_blocks *B)
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
    g.iperm = B->d_iperm;
    g.origin = B->d_origin;
    g.ext = B->d_ext;
    return g;
}

}  // namespace dd
