// HIP kernels of libdd for gfx950.
//
// Data layout (device, library-owned):
//   half field (one parity of a spinor field, all blocks, all rhs): for block
//     b with h_b sites per parity, element (rhs r, component c in 0..23, eo
//     site h) at (soff[b]/2)*24*n_rhs + (r*24 + c)*h_b + h, i.e. per block and
//     rhs a component-major structure of arrays with the site innermost.
//     Component c = 2*(3*spin + colour) + {0: re, 1: im}.
//   links: per block [mu][k = 3*row + col, rows 0 and 1][eo site][re, im], the
//     first two rows of the forward link U_mu(x) of every block site (row 2 is
//     rebuilt in the kernels); links that leave the block are zero.
//   neighbour table per block shape: [parity][h][8] int32, entries
//     2*mu = x+mu, 2*mu+1 = x-mu as the eo index inside the other parity,
//     -1 if the hop is dropped (Dirichlet), bit 30 set if the hop crosses
//     the antiperiodic time edge.
//
// Work decomposition of every site kernel: a workgroup ("tile") of kTile
// threads handles one rhs group (G consecutive right-hand sides) on a chunk
// of consecutive eo sites of one block; thread tid owns site h0 + tid and its
// G rhs.  A chunk is a whole number of x0-slices when a slice has at most
// kTile sites per parity, so the hops along directions 1..3 of a chunk stay
// inside the same eo index range of the other parity.  Tiles are numbered
// block, chunk, group (group fastest) and the launch index is remapped so
// that consecutive tiles go to the same XCD (workgroups are dealt to the 8
// XCDs round-robin), keeping a block's shared reads in one L2.
// Every load or store of one component by a wavefront covers 64 consecutive
// sites of one rhs: 256 contiguous bytes in FP32.
#include <hip/hip_runtime.h>

#include "dd_internal.h"
#include "dd_stencil.h"

namespace dd {

// ------------------------------------------------------------- tiles

struct Tile {
    int tile, b, grp, h0, tv, hb, site, tid;
    bool live;
    int64_t base;  // element of (rhs grp*G, component 0, site) in the half fields
};

__device__ __forceinline__ Tile tile_of(const BlkArgs &ba)
{
    Tile t;
    t.tile = uni(xcd_tile(blockIdx.x, ba.ntiles));
    const int ng = ba.n_rhs / ba.g;
    const int cidx = t.tile / ng;
    t.grp = t.tile - cidx * ng;
    t.b = uni(ba.chunk_block[cidx]);
    const int chunk = cidx - uni(ba.blk_chunk0[t.b]);
    t.hb = uni(ba.h[t.b]);
    const int T = uni(ba.chunk[t.b]);
    t.h0 = chunk * T;
    t.tv = min(T, t.hb - t.h0);
    t.tid = threadIdx.x;
    t.live = t.tid < t.tv;
    t.site = t.h0 + t.tid;
    t.base = (ba.soff[t.b] >> 1) * 24 * ba.n_rhs + (int64_t)t.grp * ba.g * 24 * t.hb + t.site;
    return t;
}

// element offset of component c of the thread's j-th rhs, relative to Tile::base
__device__ __forceinline__ int64_t eoff(const Tile &t, int j, int c) { return ((int64_t)j * 24 + c) * t.hb; }

// Per-(tile, rhs) sums: a fixed tree over the tile's threads for each of the
// G rhs and each of the nred values; partial[(tile * G + j) * kNRed + k].
template <int G>
__device__ __forceinline__ void tile_sum(double (*red)[kTile], const double (&dv)[G][kNRed], int nred,
                                         double *partial, int tile)
{
    const int tid = threadIdx.x;
    for (int k = 0; k < nred; k++) {
#pragma unroll
        for (int j = 0; j < G; j++) red[j][tid] = dv[j][k];
        __syncthreads();
        for (int w = kTile / 2; w > 0; w >>= 1) {
            if (tid < w)
#pragma unroll
                for (int j = 0; j < G; j++) red[j][tid] += red[j][tid + w];
            __syncthreads();
        }
        if (tid < G) partial[((int64_t)tile * G + tid) * kNRed + k] = red[tid][0];
        __syncthreads();
    }
}

// ------------------------------------------------------------- hop


// The BiCGStab shadow residual rh: any fixed vector with <rh, r_0> != 0
// serves, so with FP32 spinors the solver keeps r_0 rounded to BF16 (half the
// bytes of the two dot products per iteration that read it), with FP64 r_0.
template <typename SP>
struct ShadowT {
    using T = SP;
};
template <>
struct ShadowT<float> {
    using T = uint16_t;
};
__device__ __forceinline__ double shadow_val(double v) { return v; }
__device__ __forceinline__ float shadow_val(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }
__device__ __forceinline__ double to_shadow(double v, double *) { return v; }
__device__ __forceinline__ uint16_t to_shadow(float v, uint16_t *) { return f32_to_bf16_rne(v); }

// Output operands of the hop epilogue, as block-relative buffer descriptors;
// an absent operand gets a zero-size descriptor (its loads return 0).  In
// mode kDotAuxOut the aux operand is the shadow residual (ShadowT).
struct EpiBufs {
    Buf out_b, self_b, add_b, aux_b;
    bool has_self, has_add;
};

template <typename SP>
__device__ __forceinline__ EpiBufs epi_bufs(const HopArgs &ha, int64_t hbase, uint32_t fbytes)
{
    using SH = typename ShadowT<SP>::T;
    EpiBufs eb;
    eb.out_b = make_buf(reinterpret_cast<const SP *>(ha.out) + hbase, fbytes);
    eb.self_b = make_buf(ha.self ? reinterpret_cast<const SP *>(ha.self) + hbase : nullptr, ha.self ? fbytes : 0);
    eb.add_b = make_buf(ha.add ? reinterpret_cast<const SP *>(ha.add) + hbase : nullptr, ha.add ? fbytes : 0);
    if (ha.dot_mode == kDotAuxOut)
        eb.aux_b = make_buf(reinterpret_cast<const SH *>(ha.aux) + hbase, fbytes / sizeof(SP) * sizeof(SH));
    else if (ha.dot_mode == kDotOutAuxOutOut)
        eb.aux_b = make_buf(reinterpret_cast<const SP *>(ha.aux) + hbase, fbytes);
    else
        eb.aux_b = make_buf(nullptr, 0);
    eb.has_self = ha.self != nullptr;
    eb.has_add = ha.add != nullptr;
    return eb;
}

// out = c_hop*acc + c_self*self + c_add*add at one site and rhs (my: byte
// offset of its component 0, cstr: bytes between components), and the fused
// dot products of the mode added to dv.  Two halves of 12 reals: all operand
// loads of a half are issued before its stores (a store to `out` could alias
// them, which would otherwise serialise every load behind the previous
// store).  Fully unrolled: acc is indexed by the component, and a runtime
// index would put it in scratch.
// DM: the dot mode, or -1 to take it from ha at run time; PARTS: the
// batches of loads (more batches, fewer registers).
template <typename SP, typename AC, int DM, int PARTS = 2>
__device__ __forceinline__ void hop_epilogue(const AC (&acc)[24], double (&dv)[kNRed], const HopArgs &ha,
                                             const EpiBufs &eb, uint32_t my, uint32_t cstr)
{
    const int mode = DM >= 0 ? DM : ha.dot_mode;
    const AC ch = (AC)ha.c_hop, cself = (AC)ha.c_self, cadd = (AC)ha.c_add;
    constexpr int NQ = 24 / PARTS;
#pragma unroll
    for (int half = 0; half < PARTS; half++) {
        SP sx[NQ], dx[NQ], ax[NQ];
#pragma unroll
        for (int q = 0; q < NQ; q++) {
            const uint32_t so = (uint32_t)(NQ * half + q) * cstr;
            sx[q] = bload<SP>(eb.self_b, my, so);
            dx[q] = bload<SP>(eb.add_b, my, so);
            if (mode == kDotAuxOut) {
                using SH = typename ShadowT<SP>::T;
                constexpr uint32_t sh = sizeof(SP) / sizeof(SH);  // byte offsets scale with the element size
                ax[q] = (SP)shadow_val(bload<SH>(eb.aux_b, my / sh, so / sh));
            } else {
                ax[q] = bload<SP>(eb.aux_b, my, so);
            }
        }
#pragma unroll
        for (int k = 0; k < NQ / 2; k++) {
            double o[2], sv[2], av[2];
#pragma unroll
            for (int ri = 0; ri < 2; ri++) {
                const int q = 2 * k + ri;
                const uint32_t so = (uint32_t)(NQ * half + q) * cstr;
                AC v = ch * acc[NQ * half + q];
                if (eb.has_self) v = fmad(cself, (AC)sx[q], v);
                if (eb.has_add) v = fmad(cadd, (AC)dx[q], v);
                const SP ov = (SP)v;
                bstore<SP>(eb.out_b, ov, my, so);
                o[ri] = (double)ov;
                sv[ri] = (double)sx[q];
                av[ri] = (double)ax[q];
            }
            if (mode == kDotAuxOut) {
                dv[0] += av[0] * o[0] + av[1] * o[1];
                dv[1] += av[0] * o[1] - av[1] * o[0];
            } else if (mode == kDotOutSelfOutOut) {
                dv[0] += o[0] * sv[0] + o[1] * sv[1];
                dv[1] += o[0] * sv[1] - o[1] * sv[0];
                dv[2] += o[0] * o[0] + o[1] * o[1];
            } else if (mode == kDotOutAuxOutOut) {
                dv[0] += o[0] * av[0] + o[1] * av[1];
                dv[1] += o[0] * av[1] - o[1] * av[0];
                dv[2] += o[0] * o[0] + o[1] * o[1];
            } else if (mode == kDotOutOut) {
                dv[0] += o[0] * o[0] + o[1] * o[1];
            }
        }
    }
}

__host__ __device__ constexpr int dot_nred(int mode)
{
    return mode == kDotAuxOut ? 2 : (mode == kDotOutSelfOutOut || mode == kDotOutAuxOutOut ? 3 : (mode == kDotOutOut ? 1 : 0));
}

// out = c_add*add + c_self*self + c_hop * (H in) on the sites of one parity,
// `in` on the other parity.  The tile first copies its chunk of `in` (its rhs
// group) into LDS; hops that land inside the chunk read LDS, the others
// (direction 0 across the chunk edge) read global memory.  CL: the hop result
// at each output site is multiplied by that site's clover matrix (ha.clover)
// before the epilogue, as in the walk hop (one rhs per thread).
template <typename SP, typename LK, typename AC, int G, bool CL = false>
__global__ void __launch_bounds__(kTile) k_hop(BlkArgs ba, HopArgs ha)
{
    static_assert(!CL || G == 1, "clover hops take one rhs per thread");
    __shared__ SP stage[24 * kTile * G];
    __shared__ double red[G][kTile];
    const Tile t = tile_of(ba);
    const int p = ha.parity;
    // wave-uniform block bases and buffer descriptors; per-thread offsets are 32-bit
    const int64_t soff = uni64(ba.soff[t.b]);
    const int64_t hbase = (soff >> 1) * 24 * ba.n_rhs;
    const uint32_t fbytes = (uint32_t)(ba.n_rhs * 24 * t.hb) * (uint32_t)sizeof(SP);  // block's half field
    HopCtx hc;
    hc.h0 = t.h0;
    hc.tv = ha.use_lds ? t.tv : 0;
    hc.cstr = (uint32_t)t.hb * (uint32_t)sizeof(SP);
    hc.kstr = (uint32_t)(4 * t.hb) * (uint32_t)sizeof(LK);  // S_b = 2 h_b slots, (re, im) per slot
    hc.grp_off = t.grp * G * 24 * t.hb;
    hc.in_b = make_buf(reinterpret_cast<const SP *>(ha.in) + hbase, fbytes);
    hc.lk_b = make_buf(reinterpret_cast<const LK *>(ha.links) + soff * kLinkReals,
                       (uint32_t)(2 * t.hb * kLinkReals) * (uint32_t)sizeof(LK));
    const uint32_t my = (uint32_t)(hc.grp_off + t.site) * (uint32_t)sizeof(SP);  // bytes to (group, comp 0, own site)
    if (t.live && ha.use_lds) {
#pragma unroll 4
        for (int c = 0; c < 24; c++) {
            SP v[G];
#pragma unroll
            for (int j = 0; j < G; j++) v[j] = bload<SP>(hc.in_b, my, (uint32_t)(j * 24 + c) * hc.cstr);
            stv<SP, G>(stage + (c * kTile + t.tid) * G, v);
        }
    }
    __syncthreads();
    double dv[G][kNRed];
#pragma unroll
    for (int j = 0; j < G; j++)
#pragma unroll
        for (int k = 0; k < kNRed; k++) dv[j][k] = 0;
    if (t.live) {
        const int32_t *nbp = ba.nbr + uni64(ba.nbr_off[t.b]) + (unsigned)((p * t.hb + t.site) * 8);
        int32_t nb[8];
        {
            const int4 *q = reinterpret_cast<const int4 *>(nbp);
            const int4 a0 = q[0], a1 = q[1];
            nb[0] = a0.x; nb[1] = a0.y; nb[2] = a0.z; nb[3] = a0.w;
            nb[4] = a1.x; nb[5] = a1.y; nb[6] = a1.z; nb[7] = a1.w;
        }
        hc.slot_self = p * t.hb + t.site;
        hc.other0 = (1 - p) * t.hb;
        AC acc[G][24];
#pragma unroll
        for (int j = 0; j < G; j++)
#pragma unroll
            for (int c = 0; c < 24; c++) acc[j][c] = 0;
        hop_one<0, true, SP, LK, AC, G>(acc, nb[0], stage, hc);
        hop_one<0, false, SP, LK, AC, G>(acc, nb[1], stage, hc);
        hop_one<1, true, SP, LK, AC, G>(acc, nb[2], stage, hc);
        hop_one<1, false, SP, LK, AC, G>(acc, nb[3], stage, hc);
        hop_one<2, true, SP, LK, AC, G>(acc, nb[4], stage, hc);
        hop_one<2, false, SP, LK, AC, G>(acc, nb[5], stage, hc);
        hop_one<3, true, SP, LK, AC, G>(acc, nb[6], stage, hc);
        hop_one<3, false, SP, LK, AC, G>(acc, nb[7], stage, hc);

        const EpiBufs eb = epi_bufs<SP>(ha, hbase, fbytes);
        if constexpr (CL) {
            const Buf clb = make_buf(reinterpret_cast<const SP *>(ha.clover) + soff * kCloverReals,
                                     (uint32_t)(kCloverReals * 2 * t.hb) * (uint32_t)sizeof(SP));
            clover_mul<SP, AC>(acc[0], clb, (uint32_t)hc.slot_self * (uint32_t)sizeof(SP),
                               (uint32_t)(2 * t.hb) * (uint32_t)sizeof(SP));
        }
#pragma unroll
        for (int j = 0; j < G; j++) hop_epilogue<SP, AC, -1>(acc[j], dv[j], ha, eb, my + (uint32_t)(j * 24) * hc.cstr, hc.cstr);
    }
    if (ha.dot_mode != kDotNone) {
        tile_sum<G>(red, dv, dot_nred(ha.dot_mode), ha.partial, t.tile);
    }
}

hipError_t launch_hop(const BlkArgs &ba, const HopArgs &ha, dd_prec prec, hipStream_t s)
{
    if (ha.pre != kPreNone) return hipErrorInvalidValue;  // staging updates are x0-walk only
    if (ba.ntiles <= 0) return hipSuccess;
    dim3 g(ba.ntiles), t(kTile);
    if (ha.clover) {  // clover hops: one rhs per thread
        if (ba.g != 1) return hipErrorInvalidValue;
        if (prec == DD_F64)
            hipLaunchKernelGGL((k_hop<double, double, double, 1, true>), g, t, 0, s, ba, ha);
        else if (prec == DD_F32)
            hipLaunchKernelGGL((k_hop<float, float, float, 1, true>), g, t, 0, s, ba, ha);
        else if (prec == DD_BF16)
            hipLaunchKernelGGL((k_hop<float, uint16_t, float, 1, true>), g, t, 0, s, ba, ha);
        else
            return hipErrorInvalidValue;
        return hipGetLastError();
    }
    if (prec == DD_F64 && ba.g == 1)
        hipLaunchKernelGGL((k_hop<double, double, double, 1>), g, t, 0, s, ba, ha);
    else if (prec == DD_F32 && ba.g == 1)
        hipLaunchKernelGGL((k_hop<float, float, float, 1>), g, t, 0, s, ba, ha);
    else if (prec == DD_F32 && ba.g == 2)
        hipLaunchKernelGGL((k_hop<float, float, float, 2>), g, t, 0, s, ba, ha);
    else if (prec == DD_BF16 && ba.g == 1)
        hipLaunchKernelGGL((k_hop<float, uint16_t, float, 1>), g, t, 0, s, ba, ha);
    else if (prec == DD_BF16 && ba.g == 2)
        hipLaunchKernelGGL((k_hop<float, uint16_t, float, 2>), g, t, 0, s, ba, ha);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

// Staging load of the walk with a BiCGStab update of the input (PRE: kPreP
// or kPreS) for the G rhs of the thread: the updated spinors go to the stage
// and, on the slices the tile owns, back to `in`.  Pairs that stopped keep
// their input.  Coefficients are rounded to SP as in k_bicg_p and k_bicg_s.
template <typename SP, int G, int PRE>
struct PreLoad {
    Buf in_b, r_b, v_b;
    uint32_t cstr;
    bool act[G], zero[G];  // zero: beta = 0, the direction restarts as r
    SP c0r[G], c0i[G], c1r[G], c1i[G];

    __device__ __forceinline__ void operator()(SP (&v)[24][G], uint32_t vo, bool own) const
    {
#pragma unroll
        for (int j = 0; j < G; j++) {
            const uint32_t jo = (uint32_t)(j * 24) * cstr;
            if (!act[j]) {
#pragma unroll
                for (int c = 0; c < 24; c++) v[c][j] = bload<SP>(in_b, vo, jo + (uint32_t)c * cstr);
                continue;
            }
#pragma unroll
            for (int a = 0; a < 12; a++) {
                const uint32_t o0 = jo + (uint32_t)(2 * a) * cstr, o1 = o0 + cstr;
                const SP rr = bload<SP>(r_b, vo, o0), ri = bload<SP>(r_b, vo, o1);
                SP nr, ni;
                if (PRE == kPreS) {
                    const SP vr = bload<SP>(v_b, vo, o0), vi = bload<SP>(v_b, vo, o1);
                    nr = rr - (c0r[j] * vr - c0i[j] * vi);
                    ni = ri - (c0r[j] * vi + c0i[j] * vr);
                } else if (zero[j]) {
                    nr = rr;
                    ni = ri;
                } else {
                    const SP vr = bload<SP>(v_b, vo, o0), vi = bload<SP>(v_b, vo, o1);
                    const SP pr = bload<SP>(in_b, vo, o0), pi = bload<SP>(in_b, vo, o1);
                    const SP qr = pr - (c1r[j] * vr - c1i[j] * vi);
                    const SP qi = pi - (c1r[j] * vi + c1i[j] * vr);
                    nr = rr + (c0r[j] * qr - c0i[j] * qi);
                    ni = ri + (c0r[j] * qi + c0i[j] * qr);
                }
                v[2 * a][j] = nr;
                v[2 * a + 1][j] = ni;
            }
            if (own) {
#pragma unroll
                for (int c = 0; c < 24; c++) bstore<SP>(in_b, v[c][j], vo, jo + (uint32_t)c * cstr);
            }
        }
    }
};

// x0-walk of the hop (the walk itself is in dd_stencil.h): a tile walks one
// of nseg segments of a block's x0-slices for one group of G rhs.  PRE: the
// BiCGStab update of the input done while staging it (kPre*).
// CL: the hop result at each output site is multiplied by that site's clover
// matrix (ha.clover) before the epilogue (one rhs per thread).
template <typename SP, typename LK, typename AC, int G, int DM, int PRE = kPreNone, bool CL = false>
__global__ void __launch_bounds__(kTile) __attribute__((amdgpu_waves_per_eu(sizeof(SP) == 8 && G == 1 && !CL && (DM == kDotNone || DM == kDotOutOut) ? 3 : 1)))
k_hop_walk(BlkArgs ba, WalkArgs wa, HopArgs ha)
{
    static_assert(!CL || G == 1, "clover hops take one rhs per thread");
    __shared__ SP stage[24 * kTile * G];
    __shared__ double red[G][kTile];
    const int tile = uni(wa.tile0 + xcd_tile(blockIdx.x, wa.ntiles));
    const int b = tile / wa.per;
    const int nr = ba.n_rhs, ng = nr / G;
    const int rel = tile - b * wa.per;
    const int grp = rel % ng, seg = rel / ng;
    WalkPos w;
    w.p = ha.parity;
    w.hb = uni(ba.h[b]);
    const int ns = uni(wa.ext[4 * b]);  // x0-slices of the block
    w.hs = w.hb / ns;
    w.k = threadIdx.x;
    w.s0 = seg * ns / wa.nseg;
    w.s1 = (seg + 1) * ns / wa.nseg;
    if (ha.skip_act) {
        // every pair of the tile's rhs group stopped iterating: the workgroup leaves
        bool any = false;
#pragma unroll
        for (int j = 0; j < G; j++) any = any || ha.skip_act[(grp * G + j) * ba.nb + b] != 0;
        if (!any) return;
    }
    if (ha.bytes_acc && threadIdx.x == 0) atomicAdd(ha.bytes_acc, ha.bytes_site * (w.s1 - w.s0) * w.hs * G);
    const int64_t soff = uni64(ba.soff[b]);
    const int64_t hbase = (soff >> 1) * 24 * nr;
    const uint32_t fbytes = (uint32_t)(nr * 24 * w.hb) * (uint32_t)sizeof(SP);
    HopCtx hc;
    hc.h0 = 0;
    hc.tv = 0;
    hc.slot_self = 0;
    hc.other0 = 0;
    hc.cstr = (uint32_t)w.hb * (uint32_t)sizeof(SP);
    hc.kstr = (uint32_t)(4 * w.hb) * (uint32_t)sizeof(LK);
    hc.grp_off = grp * G * 24 * w.hb;
    hc.in_b = make_buf(reinterpret_cast<const SP *>(ha.in) + hbase, fbytes);
    hc.lk_b = make_buf(reinterpret_cast<const LK *>(ha.links) + soff * kLinkReals,
                       (uint32_t)(2 * w.hb * kLinkReals) * (uint32_t)sizeof(LK));
    const EpiBufs eb = epi_bufs<SP>(ha, hbase, fbytes);
    w.nbt = ba.nbr + uni64(ba.nbr_off[b]) + (int64_t)w.p * w.hb * 8;
    double dv[G][kNRed];
#pragma unroll
    for (int j = 0; j < G; j++)
#pragma unroll
        for (int i = 0; i < kNRed; i++) dv[j][i] = 0;
    const Buf clb = make_buf(CL ? reinterpret_cast<const SP *>(ha.clover) + soff * kCloverReals : nullptr,
                             CL ? (uint32_t)(kCloverReals * 2 * w.hb) * (uint32_t)sizeof(SP) : 0u);
    auto epi = [&](const AC (&acc)[G][24], int h) {
#pragma unroll
        for (int j = 0; j < G; j++) {
            const uint32_t my = (uint32_t)(hc.grp_off + j * 24 * w.hb + h) * (uint32_t)sizeof(SP);
            if constexpr (CL) {
                AC a[24];
#pragma unroll
                for (int c = 0; c < 24; c++) a[c] = acc[j][c];
                clover_mul<SP, AC>(a, clb, (uint32_t)(w.p * w.hb + h) * (uint32_t)sizeof(SP),
                                   (uint32_t)(2 * w.hb) * (uint32_t)sizeof(SP));
                hop_epilogue<SP, AC, DM>(a, dv[j], ha, eb, my, hc.cstr);
            } else {
                hop_epilogue<SP, AC, DM>(acc[j], dv[j], ha, eb, my, hc.cstr);
            }
        }
    };
    if constexpr (PRE == kPreNone) {
        walk_run<SP, LK, AC, G>(w, ns, stage, hc, epi);
    } else {
        PreLoad<SP, G, PRE> pl;
        pl.in_b = hc.in_b;
        pl.r_b = make_buf(reinterpret_cast<const SP *>(ha.pre_r) + hbase, fbytes);
        pl.v_b = make_buf(reinterpret_cast<const SP *>(ha.pre_v) + hbase, fbytes);
        pl.cstr = hc.cstr;
#pragma unroll
        for (int j = 0; j < G; j++) {
            const int pr = (grp * G + j) * ba.nb + b;
            pl.act[j] = ha.pre_act[pr] != 0;
            const double c0r = ha.pre_c0[2 * pr], c0i = ha.pre_c0[2 * pr + 1];
            pl.c0r[j] = (SP)c0r;
            pl.c0i[j] = (SP)c0i;
            pl.zero[j] = c0r == 0.0 && c0i == 0.0;
            pl.c1r[j] = PRE == kPreP ? (SP)ha.pre_c1[2 * pr] : (SP)0;
            pl.c1i[j] = PRE == kPreP ? (SP)ha.pre_c1[2 * pr + 1] : (SP)0;
        }
        walk_run<SP, LK, AC, G>(w, ns, stage, hc, epi, [&](int q, SP (&v)[24][G]) {
            pl(v, (uint32_t)(hc.grp_off + q * w.hs + w.k) * (uint32_t)sizeof(SP), q >= w.s0 && q < w.s1);
        });
    }
    if (DM != kDotNone) {
        // partial sums in the chunk tiles' slots: segment seg in chunk slot seg,
        // the block's remaining chunk slots zero
        constexpr int nred = dot_nred(DM);
        const int c0 = uni(ba.blk_chunk0[b]), nch = uni(ba.blk_chunk0[b + 1]) - c0, t0 = c0 * ng;
        tile_sum<G>(red, dv, nred, ha.partial, t0 + seg * ng + grp);
        if (seg == 0)
            for (int i = threadIdx.x; i < (nch - wa.nseg) * G * nred; i += kTile) {
                const int ch = wa.nseg + i / (G * nred), j = (i / nred) % G, k = i % nred;
                ha.partial[((int64_t)(t0 + ch * ng + grp) * G + j) * kNRed + k] = 0;
            }
    }
}

template <typename SP, typename LK, typename AC, int G, bool CL>
static void launch_walk_cl(const BlkArgs &ba, const WalkArgs &wa, const HopArgs &ha, hipStream_t s)
{
    dim3 g(wa.ntiles), t(kTile);
    if (ha.pre == kPreP) {
        hipLaunchKernelGGL((k_hop_walk<SP, LK, AC, G, kDotNone, kPreP, CL>), g, t, 0, s, ba, wa, ha);
        return;
    }
    if (ha.pre == kPreS) {
        hipLaunchKernelGGL((k_hop_walk<SP, LK, AC, G, kDotNone, kPreS, CL>), g, t, 0, s, ba, wa, ha);
        return;
    }
    switch (ha.dot_mode) {
    case kDotNone: hipLaunchKernelGGL((k_hop_walk<SP, LK, AC, G, kDotNone, kPreNone, CL>), g, t, 0, s, ba, wa, ha); break;
    case kDotAuxOut: hipLaunchKernelGGL((k_hop_walk<SP, LK, AC, G, kDotAuxOut, kPreNone, CL>), g, t, 0, s, ba, wa, ha); break;
    case kDotOutSelfOutOut: hipLaunchKernelGGL((k_hop_walk<SP, LK, AC, G, kDotOutSelfOutOut, kPreNone, CL>), g, t, 0, s, ba, wa, ha); break;
    case kDotOutOut: hipLaunchKernelGGL((k_hop_walk<SP, LK, AC, G, kDotOutOut, kPreNone, CL>), g, t, 0, s, ba, wa, ha); break;
    default: hipLaunchKernelGGL((k_hop_walk<SP, LK, AC, G, kDotOutAuxOutOut, kPreNone, CL>), g, t, 0, s, ba, wa, ha); break;
    }
}

template <typename SP, typename LK, typename AC, int G>
static void launch_walk_t(const BlkArgs &ba, const WalkArgs &wa, const HopArgs &ha, hipStream_t s)
{
    if constexpr (G == 1) {
        if (ha.clover) {
            launch_walk_cl<SP, LK, AC, G, true>(ba, wa, ha, s);
            return;
        }
    }
    launch_walk_cl<SP, LK, AC, G, false>(ba, wa, ha, s);
}

hipError_t launch_hop_walk(const BlkArgs &ba, const WalkArgs &wa, const HopArgs &ha, dd_prec prec, hipStream_t s)
{
    if (wa.ntiles <= 0) return hipSuccess;
    if (wa.nseg < 1 || ha.dot_mode < kDotNone || ha.dot_mode > kDotOutAuxOutOut) return hipErrorInvalidValue;
    // the launch covers whole blocks of the tile grid: [tile0, tile0 + ntiles) within nb * per
    if (wa.per != wa.nseg * (ba.n_rhs / ba.g) || wa.tile0 < 0 || wa.tile0 % wa.per || wa.ntiles % wa.per ||
        (int64_t)wa.tile0 + wa.ntiles > (int64_t)ba.nb * wa.per)
        return hipErrorInvalidValue;
    if (ha.pre < kPreNone || ha.pre > kPreS) return hipErrorInvalidValue;
    if (ha.clover && ba.g != 1) return hipErrorInvalidValue;  // clover hops: one rhs per thread
    // the staging updates: no fused dots; kPreP rewrites its input in place,
    // which only one tile per site may read
    if (ha.pre != kPreNone && (ha.dot_mode != kDotNone || !ha.pre_r || !ha.pre_v || !ha.pre_c0 || !ha.pre_act ||
                               (ha.pre == kPreP && (wa.nseg != 1 || !ha.pre_c1))))
        return hipErrorInvalidValue;
    if (prec == DD_F64 && ba.g == 1)
        launch_walk_t<double, double, double, 1>(ba, wa, ha, s);
    else if (prec == DD_F32 && ba.g == 1)
        launch_walk_t<float, float, float, 1>(ba, wa, ha, s);
    else if (prec == DD_F32 && ba.g == 2)
        launch_walk_t<float, float, float, 2>(ba, wa, ha, s);
    else if (prec == DD_BF16 && ba.g == 1)
        launch_walk_t<float, uint16_t, float, 1>(ba, wa, ha, s);
    else if (prec == DD_BF16 && ba.g == 2)
        launch_walk_t<float, uint16_t, float, 2>(ba, wa, ha, s);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

// Dhat on the even sites in one x0-walk per (block, rhs):
//   out = c_self self + c_hop H_eo (H_oe in)   (+ the fused dots of DM),
// the odd intermediate H_oe in living in LDS one x0-slice at a time and never
// in global memory.  Step q stages input slice q (with the BiCGStab update
// PRE), which finishes intermediate slice q-1 in the second LDS slice; the
// second hop then takes that slice and finishes output slice q-2.  Both hops
// are x0-walks of the same block (dd_stencil.h), the first over the odd
// output sites, the second over the even ones.  One segment per block, one
// rhs per thread (the two LDS slices of 24 x 256 reals per rhs).
// A workgroup walks NR rhs of one block (NR groups of kTile threads, each with
// its own slices, in lockstep through the shared barriers): the groups load
// the same links within one barrier interval, so a block's links come from
// HBM about once per NR rhs instead of once per rhs.  NR = 3 keeps the same
// three groups of kTile threads per compute unit as NR = 1 (144 KB of LDS).
// Dot partials go to the chunk slots of the site kernels' tile table (rhs
// group ba.g): slot 0 of the block holds the sum, its other slots are zero.
// CL: the clover term's asymmetric form 1 - kappa^2 A_ee^-1 H_eo A_oo^-1 H_oe,
// A_oo^-1 (ha.clover) applied to each intermediate site before it goes to
// LDS and A_ee^-1 to each output site before the epilogue (one rhs per
// workgroup).
template <typename SP, typename LK, typename AC, int DM, int PRE, int NR, bool CL = false>
__global__ void __launch_bounds__(kTile * NR) k_dhat_walk(BlkArgs ba, WalkArgs wa, HopArgs ha)
{
    static_assert(!CL || NR == 1, "the clover Dhat walk takes one rhs per workgroup");
    __shared__ SP sa[NR][24 * kTile];  // input slice q
    __shared__ SP sb[NR][24 * kTile];  // intermediate slice q-1
    __shared__ double red[NR][kTile];
    const int tile = uni(xcd_tile(blockIdx.x, wa.ntiles));
    const int b = tile / wa.per;
    const int nr = ba.n_rhs;
    const int gi = NR == 1 ? 0 : uni((int)(threadIdx.x / kTile));  // rhs group of the wavefront
    const int r = (tile - b * wa.per) * NR + gi;
    const int hb = uni(ba.h[b]);
    // a group whose rhs is past n_rhs or whose pair stopped iterating only
    // takes part in the barriers; a workgroup with no such group leaves
    bool alive = r < nr && (!ha.skip_act || ha.skip_act[r * ba.nb + b]);
    if (NR > 1) {
        bool any = false;
#pragma unroll
        for (int j = 0; j < NR; j++) {
            const int rj = (tile - b * wa.per) * NR + j;
            any = any || (rj < nr && (!ha.skip_act || ha.skip_act[rj * ba.nb + b]));
        }
        if (!any) return;
    } else if (!alive) {
        return;
    }
    const int k = (int)(threadIdx.x % kTile);
    if (ha.bytes_acc && alive && k == 0) atomicAdd(ha.bytes_acc, ha.bytes_site * hb);
    const int rr = alive ? r : 0;  // addresses of a group that does nothing stay in range
    const int ns = uni(wa.ext[4 * b]);
    const int hs = hb / ns;
    const int32_t *nbt = ba.nbr + uni64(ba.nbr_off[b]);
    const WalkPos wodd{1, hb, hs, k, 0, ns, nbt + (int64_t)hb * 8};
    const WalkPos weven{0, hb, hs, k, 0, ns, nbt};
    const int64_t soff = uni64(ba.soff[b]);
    const int64_t hbase = (soff >> 1) * 24 * nr;
    const uint32_t fbytes = (uint32_t)(nr * 24 * hb) * (uint32_t)sizeof(SP);
    HopCtx hc;
    hc.h0 = 0;
    hc.tv = 0;
    hc.slot_self = 0;
    hc.other0 = 0;
    hc.cstr = (uint32_t)hb * (uint32_t)sizeof(SP);
    hc.kstr = (uint32_t)(4 * hb) * (uint32_t)sizeof(LK);
    hc.grp_off = rr * 24 * hb;
    hc.in_b = make_buf(reinterpret_cast<const SP *>(ha.in) + hbase, fbytes);
    hc.lk_b = make_buf(reinterpret_cast<const LK *>(ha.links) + soff * kLinkReals,
                       (uint32_t)(2 * hb * kLinkReals) * (uint32_t)sizeof(LK));
    const EpiBufs eb = epi_bufs<SP>(ha, hbase, fbytes);
    PreLoad<SP, 1, PRE> pl;
    if constexpr (PRE != kPreNone) {
        pl.in_b = hc.in_b;
        pl.r_b = make_buf(reinterpret_cast<const SP *>(ha.pre_r) + hbase, fbytes);
        pl.v_b = make_buf(reinterpret_cast<const SP *>(ha.pre_v) + hbase, fbytes);
        pl.cstr = hc.cstr;
        const int pr = rr * ba.nb + b;
        pl.act[0] = ha.pre_act[pr] != 0;
        const double c0r = ha.pre_c0[2 * pr], c0i = ha.pre_c0[2 * pr + 1];
        pl.c0r[0] = (SP)c0r;
        pl.c0i[0] = (SP)c0i;
        pl.zero[0] = c0r == 0.0 && c0i == 0.0;
        pl.c1r[0] = PRE == kPreP ? (SP)ha.pre_c1[2 * pr] : (SP)0;
        pl.c1i[0] = PRE == kPreP ? (SP)ha.pre_c1[2 * pr + 1] : (SP)0;
    }
    double dv[1][kNRed];
#pragma unroll
    for (int i = 0; i < kNRed; i++) dv[0][i] = 0;
    const Buf clb = make_buf(CL ? reinterpret_cast<const SP *>(ha.clover) + soff * kCloverReals : nullptr,
                             CL ? (uint32_t)(kCloverReals * 2 * hb) * (uint32_t)sizeof(SP) : 0u);
    const uint32_t clk = (uint32_t)(2 * hb) * (uint32_t)sizeof(SP);
    auto to_out = [&](const AC (&acc)[1][24], int h) {
        if constexpr (CL) {
            AC a[24];
#pragma unroll
            for (int c = 0; c < 24; c++) a[c] = acc[0][c];
            clover_mul<SP, AC>(a, clb, (uint32_t)h * (uint32_t)sizeof(SP), clk);  // A_ee^-1, even slot h
            hop_epilogue<SP, AC, DM>(a, dv[0], ha, eb, (uint32_t)(hc.grp_off + h) * (uint32_t)sizeof(SP), hc.cstr);
        } else {
            hop_epilogue<SP, AC, DM>(acc[0], dv[0], ha, eb, (uint32_t)(hc.grp_off + h) * (uint32_t)sizeof(SP),
                                     hc.cstr);
        }
    };
    auto to_sb = [&](AC (&a)[24], int h) {
        if constexpr (CL) clover_mul<SP, AC>(a, clb, (uint32_t)(hb + h) * (uint32_t)sizeof(SP), clk);  // A_oo^-1
    };
    auto ld = [&](int q, SP (&v)[24][1]) {
        const uint32_t vo = (uint32_t)(hc.grp_off + q * hs + k) * (uint32_t)sizeof(SP);
        if constexpr (PRE == kPreNone) {
#pragma unroll
            for (int c = 0; c < 24; c++) v[c][0] = bload<SP>(hc.in_b, vo, (uint32_t)c * hc.cstr);
        } else {
            pl(v, vo, true);
        }
    };
    dhat_run<SP, LK, AC>(wodd, weven, ns, sa[gi], sb[gi], hc, ld, to_out, alive, to_sb);
    if (DM != kDotNone) {
        // per-group fixed-order sums over the group's kTile threads
        constexpr int nred = dot_nred(DM);
        const int gb = ba.g, ngb = nr / gb;
        const int c0 = uni(ba.blk_chunk0[b]), nch = uni(ba.blk_chunk0[b + 1]) - c0, t0 = c0 * ngb;
        for (int q = 0; q < nred; q++) {
            red[gi][k] = dv[0][q];
            __syncthreads();
            for (int w = kTile / 2; w > 0; w >>= 1) {
                if (k < w) red[gi][k] += red[gi][k + w];
                __syncthreads();
            }
            if (alive && k == 0) ha.partial[((int64_t)(t0 + rr / gb) * gb + rr % gb) * kNRed + q] = red[gi][0];
            __syncthreads();
        }
        if (alive)
            for (int i = k; i < (nch - 1) * nred; i += kTile) {
                const int ch = 1 + i / nred, kk = i % nred;
                ha.partial[((int64_t)(t0 + ch * ngb + rr / gb) * gb + rr % gb) * kNRed + kk] = 0;
            }
    }
}

template <typename SP, typename LK, typename AC, int NR, bool CL = false>
static hipError_t launch_dhat_t(const BlkArgs &ba, const WalkArgs &wa, const HopArgs &ha, hipStream_t s)
{
    dim3 g(wa.ntiles), t(kTile * NR);
#define DD_DHAT(DMV, PREV) hipLaunchKernelGGL((k_dhat_walk<SP, LK, AC, DMV, PREV, NR, CL>), g, t, 0, s, ba, wa, ha)
    if (ha.pre == kPreP && ha.dot_mode == kDotAuxOut) DD_DHAT(kDotAuxOut, kPreP);
    else if (ha.pre == kPreS && ha.dot_mode == kDotOutSelfOutOut) DD_DHAT(kDotOutSelfOutOut, kPreS);
    else if (ha.pre == kPreNone && ha.dot_mode == kDotAuxOut) DD_DHAT(kDotAuxOut, kPreNone);
    else if (ha.pre == kPreNone && ha.dot_mode == kDotOutSelfOutOut) DD_DHAT(kDotOutSelfOutOut, kPreNone);
    else if (ha.pre == kPreNone && ha.dot_mode == kDotOutAuxOutOut) DD_DHAT(kDotOutAuxOutOut, kPreNone);
    else if (ha.pre == kPreNone && ha.dot_mode == kDotNone) DD_DHAT(kDotNone, kPreNone);
    else return hipErrorInvalidValue;
#undef DD_DHAT
    return hipGetLastError();
}

hipError_t launch_dhat_walk(const BlkArgs &ba, const WalkArgs &wa, const HopArgs &ha, dd_prec prec, hipStream_t s)
{
    if (ha.clover && wa.nseg != 1) return hipErrorInvalidValue;  // clover: one rhs per workgroup
    if (wa.ntiles <= 0) return hipSuccess;
    // one walk of a whole block per rhs (wa.nseg rhs per workgroup: 1 or 3);
    // the output is the even parity
    const int nrw = wa.nseg;
    if ((nrw != 1 && nrw != 3) || ha.parity != 0 || ba.n_rhs % ba.g != 0 || wa.per != (ba.n_rhs + nrw - 1) / nrw ||
        wa.ntiles != ba.nb * wa.per)
        return hipErrorInvalidValue;
    if (ha.pre != kPreNone && (!ha.pre_r || !ha.pre_v || !ha.pre_c0 || !ha.pre_act || (ha.pre == kPreP && !ha.pre_c1)))
        return hipErrorInvalidValue;
    if (ha.clover) {
        if (prec == DD_F32) return launch_dhat_t<float, float, float, 1, true>(ba, wa, ha, s);
        if (prec == DD_BF16) return launch_dhat_t<float, uint16_t, float, 1, true>(ba, wa, ha, s);
        return hipErrorInvalidValue;
    }
    if (prec == DD_F32) return nrw == 3 ? launch_dhat_t<float, float, float, 3>(ba, wa, ha, s)
                                         : launch_dhat_t<float, float, float, 1>(ba, wa, ha, s);
    if (prec == DD_BF16) return nrw == 3 ? launch_dhat_t<float, uint16_t, float, 3>(ba, wa, ha, s)
                                          : launch_dhat_t<float, uint16_t, float, 1>(ba, wa, ha, s);
    return hipErrorInvalidValue;
}

// D_Lambda in one x0-walk per (block, rhs): both parities of input slice q
// are staged in LDS (2 x 24 x kTile reals); the even-output walk takes its
// hops from the staged odd sites and the odd-output walk from the staged even
// ones (walk_step of dd_stencil.h, as in the hop kernels), so x is read from
// memory once; the epilogue's self term x_p comes back from the cache.
template <typename SP, typename LK, typename AC>
__global__ void __launch_bounds__(kTile) k_dlam_walk(BlkArgs ba, DlamArgs da)
{
    __shared__ SP stage[2][24 * kTile];
    const int tile = uni(xcd_tile(blockIdx.x, da.ntiles));
    const int nr = ba.n_rhs;
    const int b = tile / nr, r = tile - b * nr;
    const int hb = uni(ba.h[b]);
    const int ns = uni(da.ext[4 * b]);
    const int hs = hb / ns;
    const int k = threadIdx.x;
    const bool live = k < hs;
    if (da.bytes_acc && k == 0) atomicAdd(da.bytes_acc, da.bytes_walk);
    const int32_t *nbt = ba.nbr + uni64(ba.nbr_off[b]);
    const WalkPos weven{0, hb, hs, k, 0, ns, nbt};
    const WalkPos wodd{1, hb, hs, k, 0, ns, nbt + (int64_t)hb * 8};
    const int64_t soff = uni64(ba.soff[b]);
    const int64_t hbase = (soff >> 1) * 24 * nr;
    const uint32_t fbytes = (uint32_t)(nr * 24 * hb) * (uint32_t)sizeof(SP);
    HopCtx hc;
    hc.h0 = 0;
    hc.tv = 0;
    hc.slot_self = 0;
    hc.other0 = 0;
    hc.cstr = (uint32_t)hb * (uint32_t)sizeof(SP);
    hc.kstr = (uint32_t)(4 * hb) * (uint32_t)sizeof(LK);
    hc.grp_off = r * 24 * hb;
    hc.lk_b = make_buf(reinterpret_cast<const LK *>(da.links) + soff * kLinkReals,
                       (uint32_t)(2 * hb * kLinkReals) * (uint32_t)sizeof(LK));
    const Buf xe = make_buf(reinterpret_cast<const SP *>(da.xe) + hbase, fbytes);
    const Buf xo = make_buf(reinterpret_cast<const SP *>(da.xo) + hbase, fbytes);
    const Buf ye = make_buf(reinterpret_cast<const SP *>(da.ye) + hbase, fbytes);
    const Buf yo = make_buf(reinterpret_cast<const SP *>(da.yo) + hbase, fbytes);
    const AC ch = (AC)da.c_hop;
    auto epi = [&](const Buf &xb, const Buf &yb, const AC (&acc)[1][24], int h) {
        const uint32_t my = (uint32_t)(hc.grp_off + h) * (uint32_t)sizeof(SP);
#pragma unroll
        for (int half = 0; half < 2; half++) {
            SP sx[12];
#pragma unroll
            for (int q = 0; q < 12; q++) sx[q] = bload<SP>(xb, my, (uint32_t)(12 * half + q) * hc.cstr);
#pragma unroll
            for (int q = 0; q < 12; q++)
                bstore<SP>(yb, (SP)fmad(ch, acc[0][12 * half + q], (AC)sx[q]), my,
                           (uint32_t)(12 * half + q) * hc.cstr);
        }
    };
    auto epi_e = [&](const AC (&acc)[1][24], int h) { epi(xe, ye, acc, h); };
    auto epi_o = [&](const AC (&acc)[1][24], int h) { epi(xo, yo, acc, h); };
    AC acc0[1][24], car0[1][12], acc1[1][24], car1[1][12];
#pragma unroll
    for (int c = 0; c < 24; c++) acc0[0][c] = acc1[0][c] = 0;
#pragma unroll
    for (int c = 0; c < 12; c++) car0[0][c] = car1[0][c] = 0;
    for (int q = 0; q < ns; q++) {
        if (live) {
            const uint32_t vo = (uint32_t)(hc.grp_off + q * hs + k) * (uint32_t)sizeof(SP);
            SP v[24][1];
#pragma unroll
            for (int c = 0; c < 24; c++) v[c][0] = bload<SP>(xe, vo, (uint32_t)c * hc.cstr);
            walk_stage<SP, 1>(stage[0], v, k);
#pragma unroll
            for (int c = 0; c < 24; c++) v[c][0] = bload<SP>(xo, vo, (uint32_t)c * hc.cstr);
            walk_stage<SP, 1>(stage[1], v, k);
        }
        __syncthreads();
        if (live) {
            walk_step<SP, LK, AC, 1>(acc0, car0, q, weven, stage[1], hc, epi_e);
            walk_step<SP, LK, AC, 1>(acc1, car1, q, wodd, stage[0], hc, epi_o);
        }
        __syncthreads();
    }
    if (live) {  // the last slice has no x0+ neighbour
        epi_e(acc0, (ns - 1) * hs + k);
        epi_o(acc1, (ns - 1) * hs + k);
    }
}

hipError_t launch_dlam_walk(const BlkArgs &ba, const DlamArgs &da, dd_prec prec, hipStream_t s)
{
    if (da.ntiles <= 0) return hipSuccess;
    if (da.ntiles != ba.nb * ba.n_rhs || !da.ext) return hipErrorInvalidValue;
    dim3 g(da.ntiles), t(kTile);
    if (prec == DD_F32)
        hipLaunchKernelGGL((k_dlam_walk<float, float, float>), g, t, 0, s, ba, da);
    else if (prec == DD_BF16)
        hipLaunchKernelGGL((k_dlam_walk<float, uint16_t, float>), g, t, 0, s, ba, da);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

// ---------------------------------------------------------------- packing

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
    const int64_t S = 2 * (int64_t)g.h[b];
    const int y = g.perm[g.perm_off[b] + s];
    int c[4];
    local_coords(y, g.ext + 4 * b, c);
    int x[4];
    for (int m = 0; m < 4; m++) x[m] = (g.origin[4 * b + m] + c[m]) % g.L[m];
    const int64_t n = (((int64_t)x[0] * g.L[1] + x[1]) * g.L[2] + x[2]) * g.L[3] + x[3];
    const int32_t *nb = g.nbr + g.nbr_off[b] + (int64_t)s * 8;  // slot s = p*h + site
    LT *blk = dst + g.soff[b] * kLinkReals;
    for (int mu = 0; mu < 4; mu++) {
        const int32_t e = nb[2 * mu];
        const bool in = e >= 0;
        // a link across the antiperiodic time edge is stored with the -1 of the
        // fermion boundary condition (rows 0 and 1; the rebuilt row 2 takes it
        // from the neighbour entry's sign bit), so both hops through it pick it up
        const double sg = (in && (e & kNbrSign)) ? -1.0 : 1.0;
        const double *u = U + (n * 4 + mu) * 18;
        for (int k = 0; k < kLinkK; k++) {
            LT *o = blk + (((int64_t)mu * kLinkK + k) * S + s) * 2;
            o[0] = in ? cvt_link<LT>(sg * u[2 * k]) : (LT)0;
            o[1] = in ? cvt_link<LT>(sg * u[2 * k + 1]) : (LT)0;
        }
    }
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
// Thread t -> (rhs r = t / total, block site q = t % total in the boundary
// layout's box-local canonical order).  The boundary layout holds thread t's
// 192-byte spinor record at record t, so a workgroup's records are one
// contiguous range: it is read or written with lane-contiguous 16-byte
// accesses and transposed through LDS (records padded to 13 slots).  On the
// half-field side consecutive threads alternate between the two parities,
// each writing consecutive sites.
template <typename SP, bool PACK>
__global__ void __launch_bounds__(256) k_spinor_xfer(PackGeom g, double *ext_f, SP *even, SP *odd,
                                                    int nr, int64_t total)
{
    constexpr int kRec = 13;  // LDS slots (double2) per record: 12 used
    __shared__ double2 tr[256 * kRec];
    const int64_t n = total * nr;
    const int64_t t0 = (int64_t)blockIdx.x * 256;
    const int64_t t = t0 + threadIdx.x;
    double2 *ext2 = reinterpret_cast<double2 *>(ext_f) + t0 * 12;  // this workgroup's records
    const int64_t nel = (n - t0 < 256 ? n - t0 : 256) * 12;     // their 16-byte elements
    if constexpr (PACK) {
#pragma unroll
        for (int k = 0; k < 12; k++) {
            const int e = k * 256 + threadIdx.x;
            if (e < nel) tr[(e / 12) * kRec + e % 12] = ext2[e];
        }
        __syncthreads();
    }
    if (t < n) {
        const int r = (int)(t / total);
        const int64_t q = t - (int64_t)r * total;  // block site in canonical order
        const int b = find_block(g.soff, g.nb, q);
        const int y = (int)(q - g.soff[b]);
        const int hb = g.h[b];
        const int s = g.iperm[g.perm_off[b] + y];  // its eo position
        const int p = s >= hb;
        const int site = s - p * hb;
        SP *hf = (p ? odd : even) + (g.soff[b] >> 1) * 24 * nr + (int64_t)r * 24 * hb + site;
        double2 *rec = tr + threadIdx.x * kRec;
#pragma unroll
        for (int k = 0; k < 12; k++) {
            if constexpr (PACK) {
                const double2 v = rec[k];
                hf[(int64_t)(2 * k) * hb] = (SP)v.x;
                hf[(int64_t)(2 * k + 1) * hb] = (SP)v.y;
            } else {
                rec[k] = make_double2((double)hf[(int64_t)(2 * k) * hb], (double)hf[(int64_t)(2 * k + 1) * hb]);
            }
        }
    }
    if constexpr (!PACK) {
        __syncthreads();
#pragma unroll
        for (int k = 0; k < 12; k++) {
            const int e = k * 256 + threadIdx.x;
            if (e < nel) ext2[e] = tr[(e / 12) * kRec + e % 12];
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
// Same tiles as the hop.  Pairs that are no longer active keep their x (the
// update is selected away); everything else is computed unconditionally:
// pairs never mix, so values of frozen pairs do not reach active ones.

template <int G>
__device__ __forceinline__ bool pair_flags(const BlkArgs &ba, const Tile &t, const int32_t *active, bool (&act)[G])
{
    bool any = false;
#pragma unroll
    for (int j = 0; j < G; j++) {
        act[j] = t.live && active[(t.grp * G + j) * ba.nb + t.b] != 0;
        any = any || act[j];
    }
    return any;
}

template <int G>
__device__ __forceinline__ void load_coef(const double *arr, const BlkArgs &ba, const Tile &t, double (&re)[G],
                                          double (&im)[G])
{
#pragma unroll
    for (int j = 0; j < G; j++) {
        const int pr = (t.grp * G + j) * ba.nb + t.b;
        re[j] = arr[2 * pr];
        im[j] = arr[2 * pr + 1];
    }
}

// x_p += e_p for the pairs still above tolerance (FP64 accumulator)
template <typename SE, int G>
__global__ void __launch_bounds__(kTile) k_accum(BlkArgs ba, double *x, const SE *e, const int32_t *active)
{
    const Tile t = tile_of(ba);
    bool act[G];
    if (!pair_flags<G>(ba, t, active, act)) return;
    x += t.base;
    e += t.base;
#pragma unroll
    for (int j = 0; j < G; j++) {
        if (!act[j]) continue;
        // all loads of a half spinor before its stores (x could alias e as far
        // as the compiler knows)
#pragma unroll
        for (int half = 0; half < 2; half++) {
            double xv[12];
            SE ev[12];
#pragma unroll
            for (int q = 0; q < 12; q++) {
                xv[q] = x[eoff(t, j, 12 * half + q)];
                ev[q] = e[eoff(t, j, 12 * half + q)];
            }
#pragma unroll
            for (int q = 0; q < 12; q++) x[eoff(t, j, 12 * half + q)] = xv[q] + (double)ev[q];
        }
    }
}

// |a|^2 per (tile, rhs) of a half field (the partials of the hop's dot mode
// kDotOutOut)
template <typename SP, int G>
__global__ void __launch_bounds__(kTile) k_norm2(BlkArgs ba, const SP *a, double *partial)
{
    __shared__ double red[G][kTile];
    const Tile t = tile_of(ba);
    double dv[G][kNRed] = {};
    if (t.live) {
#pragma unroll
        for (int j = 0; j < G; j++) {
            SP v[24];
#pragma unroll
            for (int c = 0; c < 24; c++) v[c] = a[t.base + eoff(t, j, c)];
#pragma unroll
            for (int c = 0; c < 24; c++) dv[j][0] += (double)v[c] * (double)v[c];
        }
    }
    tile_sum<G>(red, dv, 1, partial, t.tile);
}

// BiCGStab start: r = p = rhs, rh = rhs in the shadow type (ShadowT), x = 0;
// |rhs|^2 and <rh, rhs> per (tile, rhs).  p may be null (the first direction
// update of the iteration writes p = r).
template <typename SP, int G>
__global__ void __launch_bounds__(kTile) k_bicg_init(BlkArgs ba, const SP *rhs, SP *r, typename ShadowT<SP>::T *rh,
                                                     SP *p, SP *x, double *partial, const int32_t *outer_active)
{
    __shared__ double red[G][kTile];
    const Tile t = tile_of(ba);
    double dv[G][kNRed] = {};
    bool act[G];
    if (pair_flags<G>(ba, t, outer_active, act)) {
#pragma unroll
        for (int j = 0; j < G; j++) {
            if (!act[j]) continue;
#pragma unroll
            for (int half = 0; half < 2; half++) {
                SP v[12];
#pragma unroll
                for (int q = 0; q < 12; q++) v[q] = rhs[t.base + eoff(t, j, 12 * half + q)];
#pragma unroll
                for (int q = 0; q < 12; q++) {
                    const int64_t i = t.base + eoff(t, j, 12 * half + q);
                    r[i] = v[q];
                    rh[i] = to_shadow(v[q], rh);
                    if (p) p[i] = v[q];
                    x[i] = (SP)0;
                    dv[j][0] += (double)v[q] * (double)v[q];
                }
#pragma unroll
                for (int k = 0; k < 6; k++) {
                    // conj(rh) rhs for one complex component
                    const double ar = (double)shadow_val(to_shadow(v[2 * k], rh));
                    const double ai = (double)shadow_val(to_shadow(v[2 * k + 1], rh));
                    const double br = (double)v[2 * k], bi = (double)v[2 * k + 1];
                    dv[j][1] += ar * br + ai * bi;
                    dv[j][2] += ar * bi - ai * br;
                }
            }
        }
    }
    tile_sum<G>(red, dv, 3, partial, t.tile);
}

// s = r - alpha v
template <typename SP, int G>
__global__ void __launch_bounds__(kTile) k_bicg_s(BlkArgs ba, const SP *r, const SP *v, SP *s, PairState ps)
{
    const Tile t = tile_of(ba);
    bool act[G];
    if (!pair_flags<G>(ba, t, ps.active, act)) return;
    double ar[G], ai[G];
    load_coef<G>(ps.alpha, ba, t, ar, ai);
#pragma unroll
    for (int j = 0; j < G; j++) {
        if (!act[j]) continue;
        const SP a_r = (SP)ar[j], a_i = (SP)ai[j];
        // all loads of a half spinor before its stores (s could alias r, v
        // as far as the compiler knows)
#pragma unroll
        for (int half = 0; half < 2; half++) {
            SP rv[12], vv[12];
#pragma unroll
            for (int q = 0; q < 12; q++) {
                const int64_t i = t.base + eoff(t, j, 12 * half + q);
                rv[q] = r[i];
                vv[q] = v[i];
            }
#pragma unroll
            for (int k = 0; k < 6; k++) {
                const int q0 = 2 * k, q1 = q0 + 1;
                const int64_t i0 = t.base + eoff(t, j, 12 * half + q0), i1 = i0 + t.hb;
                s[i0] = rv[q0] - (a_r * vv[q0] - a_i * vv[q1]);
                s[i1] = rv[q1] - (a_r * vv[q1] + a_i * vv[q0]);
            }
        }
    }
}

// x += alpha p + omega s;  r = s - omega t;  <rh, r>, |r|^2 per (tile, rhs)
template <typename SP, int G>
__global__ void __launch_bounds__(kTile) k_bicg_xr(BlkArgs ba, SP *x, const SP *p, const SP *sx, const SP *s,
                                                   const SP *tv, SP *r, const typename ShadowT<SP>::T *rh,
                                                   double *partial, PairState ps)
{
    // x += alpha p + omega sx (sx = s, or M s with a right preconditioner M); r = s - omega t
    const bool own_sx = sx != s;
    __shared__ double red[G][kTile];
    const Tile t = tile_of(ba);
    double dv[G][kNRed] = {};
    bool act[G];
    if (pair_flags<G>(ba, t, ps.active, act)) {
        double ar[G], ai[G], wr[G], wi[G];
        load_coef<G>(ps.alpha, ba, t, ar, ai);
        load_coef<G>(ps.omega, ba, t, wr, wi);
#pragma unroll
        for (int j = 0; j < G; j++) {
            if (!act[j]) continue;
            const SP a_r = (SP)ar[j], a_i = (SP)ai[j], w_r = (SP)wr[j], w_i = (SP)wi[j];
            // two halves of 12 reals: every operand load of a half is issued
            // before its stores (x and r could alias the operands as far as
            // the compiler knows, which would otherwise order each load after
            // the previous store)
#pragma unroll
            for (int half = 0; half < 2; half++) {
                SP pv[12], sv[12], tq[12], xv[12], xo[12];
                double hv[12];
#pragma unroll
                for (int q = 0; q < 12; q++) {
                    const int64_t i = t.base + eoff(t, j, 12 * half + q);
                    pv[q] = p[i];
                    sv[q] = s[i];
                    tq[q] = tv[i];
                    xv[q] = own_sx ? sx[i] : sv[q];
                    xo[q] = x[i];
                    hv[q] = (double)shadow_val(rh[i]);
                }
#pragma unroll
                for (int k = 0; k < 6; k++) {
                    const int q0 = 2 * k, q1 = q0 + 1;
                    const int64_t i0 = t.base + eoff(t, j, 12 * half + q0), i1 = i0 + t.hb;
                    x[i0] = xo[q0] + (a_r * pv[q0] - a_i * pv[q1]) + (w_r * xv[q0] - w_i * xv[q1]);
                    x[i1] = xo[q1] + (a_r * pv[q1] + a_i * pv[q0]) + (w_r * xv[q1] + w_i * xv[q0]);
                    const SP nr_ = sv[q0] - (w_r * tq[q0] - w_i * tq[q1]);
                    const SP ni_ = sv[q1] - (w_r * tq[q1] + w_i * tq[q0]);
                    r[i0] = nr_;
                    r[i1] = ni_;
                    const double a = hv[q0], bq = hv[q1], c = (double)nr_, d = (double)ni_;
                    dv[j][0] += a * c + bq * d;
                    dv[j][1] += a * d - bq * c;
                    dv[j][2] += c * c + d * d;
                }
            }
        }
    }
    tile_sum<G>(red, dv, 3, partial, t.tile);
}

// p = r + beta (p - omega v)
template <typename SP, int G>
__global__ void __launch_bounds__(kTile) k_bicg_p(BlkArgs ba, const SP *r, const SP *v, SP *p, PairState ps)
{
    const Tile t = tile_of(ba);
    bool act[G];
    if (!pair_flags<G>(ba, t, ps.active, act)) return;
    double br[G], bi[G], wr[G], wi[G];
    load_coef<G>(ps.beta, ba, t, br, bi);
    load_coef<G>(ps.omega, ba, t, wr, wi);
#pragma unroll
    for (int j = 0; j < G; j++) {
        if (!act[j]) continue;
        const SP b_r = (SP)br[j], b_i = (SP)bi[j], w_r = (SP)wr[j], w_i = (SP)wi[j];
        // all loads of a half spinor before its stores (as in k_bicg_s)
#pragma unroll
        for (int half = 0; half < 2; half++) {
            SP rv[12], vv[12], pv[12];
#pragma unroll
            for (int q = 0; q < 12; q++) {
                const int64_t i = t.base + eoff(t, j, 12 * half + q);
                rv[q] = r[i];
                vv[q] = v[i];
                pv[q] = p[i];
            }
#pragma unroll
            for (int k = 0; k < 6; k++) {
                const int q0 = 2 * k, q1 = q0 + 1;
                const int64_t i0 = t.base + eoff(t, j, 12 * half + q0), i1 = i0 + t.hb;
                const SP qr = pv[q0] - (w_r * vv[q0] - w_i * vv[q1]);
                const SP qi = pv[q1] - (w_r * vv[q1] + w_i * vv[q0]);
                p[i0] = rv[q0] + (b_r * qr - b_i * qi);
                p[i1] = rv[q1] + (b_r * qi + b_i * qr);
            }
        }
    }
}

template <typename SE, int G>
static void launch_accum_t(const BlkArgs &ba, double *x, const void *e, const int32_t *active, hipStream_t st)
{
    hipLaunchKernelGGL((k_accum<SE, G>), dim3(ba.ntiles), dim3(kTile), 0, st, ba, x, (const SE *)e, active);
}
template <typename SP, int G>
static void launch_norm2_t(const BlkArgs &ba, const void *a, double *partial, hipStream_t st)
{
    hipLaunchKernelGGL((k_norm2<SP, G>), dim3(ba.ntiles), dim3(kTile), 0, st, ba, (const SP *)a, partial);
}
template <typename SP, int G>
static void launch_init_t(const BlkArgs &ba, const void *rhs, void *r, void *rh, void *p, void *x, double *partial,
                          const int32_t *oa, hipStream_t st)
{
    hipLaunchKernelGGL((k_bicg_init<SP, G>), dim3(ba.ntiles), dim3(kTile), 0, st, ba, (const SP *)rhs, (SP *)r,
                       (typename ShadowT<SP>::T *)rh, (SP *)p, (SP *)x, partial, oa);
}
template <typename SP, int G>
static void launch_s_t(const BlkArgs &ba, const void *r, const void *v, void *s, const PairState &ps, hipStream_t st)
{
    hipLaunchKernelGGL((k_bicg_s<SP, G>), dim3(ba.ntiles), dim3(kTile), 0, st, ba, (const SP *)r, (const SP *)v,
                       (SP *)s, ps);
}
template <typename SP, int G>
static void launch_xr_t(const BlkArgs &ba, void *x, const void *p, const void *sx, const void *s, const void *t,
                        void *r, const void *rh, double *partial, const PairState &ps, hipStream_t st)
{
    hipLaunchKernelGGL((k_bicg_xr<SP, G>), dim3(ba.ntiles), dim3(kTile), 0, st, ba, (SP *)x, (const SP *)p,
                       (const SP *)sx, (const SP *)s, (const SP *)t, (SP *)r,
                       (const typename ShadowT<SP>::T *)rh, partial, ps);
}
template <typename SP, int G>
static void launch_p_t(const BlkArgs &ba, const void *r, const void *v, void *p, const PairState &ps, hipStream_t st)
{
    hipLaunchKernelGGL((k_bicg_p<SP, G>), dim3(ba.ntiles), dim3(kTile), 0, st, ba, (const SP *)r, (const SP *)v,
                       (SP *)p, ps);
}

// dispatch on the spinor precision and the rhs group (1, 2 or 4)
#define DD_DISPATCH(FN, SPREC, ...)                                                              \
    do {                                                                                         \
        if (ba.ntiles <= 0) return hipSuccess;                                                   \
        const bool d_ = (SPREC) == DD_F64;                                                       \
        switch (ba.g) {                                                                          \
        case 1: if (d_) FN<double, 1>(__VA_ARGS__); else FN<float, 1>(__VA_ARGS__); break;       \
        case 2: if (d_) FN<double, 2>(__VA_ARGS__); else FN<float, 2>(__VA_ARGS__); break;       \
        case 4: if (d_) FN<double, 4>(__VA_ARGS__); else FN<float, 4>(__VA_ARGS__); break;       \
        default: return hipErrorInvalidValue;                                                    \
        }                                                                                        \
        return hipGetLastError();                                                                \
    } while (0)

hipError_t launch_accum(const BlkArgs &ba, double *x, const void *e, dd_prec ep, const int32_t *active,
                        hipStream_t st)
{
    DD_DISPATCH(launch_accum_t, ep, ba, x, e, active, st);
}

hipError_t launch_norm2(const BlkArgs &ba, dd_prec sp, const void *a, double *partial, hipStream_t st)
{
    DD_DISPATCH(launch_norm2_t, sp, ba, a, partial, st);
}

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

hipError_t launch_bicg_xr(const BlkArgs &ba, dd_prec sp, void *x, const void *p, const void *sx, const void *s,
                          const void *tv, void *r, const void *rh, double *partial, const PairState &ps, hipStream_t st)
{
    DD_DISPATCH(launch_xr_t, sp, ba, x, p, sx, s, tv, r, rh, partial, ps, st);
}

hipError_t launch_bicg_p(const BlkArgs &ba, dd_prec sp, const void *r, const void *v, void *p, const PairState &ps,
                         hipStream_t st)
{
    DD_DISPATCH(launch_p_t, sp, ba, r, v, p, ps, st);
}

// ------------------------------------------------------ per-pair scalars
//
// One wavefront per (block, rhs) pair: the lanes stride over the block's
// tiles of the pair's rhs group, a fixed butterfly sums them (the same order
// on every run), and lane 0 updates the pair's recurrence scalars in FP64.

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
    const int ng = ba.n_rhs / ba.g, grp = r / ba.g, j = r - grp * ba.g;
    const int c0 = ba.blk_chunk0[b], nchunk = ba.blk_chunk0[b + 1] - c0, t0 = c0 * ng;
    for (int ch = lane; ch < nchunk; ch += 64) {
        const int t = t0 + ch * ng + grp;
#pragma unroll
        for (int k = 0; k < NK; k++) s[k] += partial[((int64_t)t * ba.g + j) * kNRed + k];
    }
#pragma unroll
    for (int k = 0; k < NK; k++) s[k] = wave_sum(s[k]);
}

__device__ __forceinline__ bool finite(double v) { return isfinite(v); }

#define DD_PAIR_PROLOGUE(NP)                                                   \
    const int lane = threadIdx.x & 63;                                         \
    const int pair = (int)((blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6); \
    if (pair >= (NP)) return;                                                  \
    const int b = pair % ba.nb, r = pair / ba.nb;

__global__ void __launch_bounds__(256) k_sc_init(BlkArgs ba, const double *partial, PairState ps, OuterState os,
                                                 double tol_in, double tol_out, int adapt)
{
    DD_PAIR_PROLOGUE(ps.np)
    double s[3];
    pair_sums<3>(ba, partial, b, r, lane, s);
    if (lane != 0) return;
    if (!os.active[pair]) {
        ps.active[pair] = 0;
        return;
    }
    double t = tol_in;
    if (adapt && os.rr[pair] > 0) t = fmax(t, fmin(0.3 * tol_out * sqrt(os.bb[pair] / os.rr[pair]), 0.1));
    ps.tol2[pair] = t * t;
    const double bb = s[0];
    ps.bb[pair] = bb;
    ps.rr[pair] = bb;
    ps.rho[2 * pair] = s[1];  // <rh, r_0>
    ps.rho[2 * pair + 1] = s[2];
    ps.omega[2 * pair] = 1;
    ps.omega[2 * pair + 1] = 0;
    ps.beta[2 * pair] = 0;  // a direction update before the first iteration gives p = r
    ps.beta[2 * pair + 1] = 0;
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

__global__ void __launch_bounds__(256) k_sc_beta(BlkArgs ba, const double *partial, PairState ps)
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
    if (rr <= ps.tol2[pair] * ps.bb[pair]) {
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
    if (os.only && !os.only[pair]) {  // not part of this solve
        os.active[pair] = 0;
        return;
    }
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

hipError_t launch_sc_init(const BlkArgs &ba, const double *partial, const PairState &ps, const OuterState &os,
                          double tol_in, double tol_out, int adapt, hipStream_t s)
{
    hipLaunchKernelGGL(k_sc_init, pair_grid(ps.np), dim3(256), 0, s, ba, partial, ps, os, tol_in, tol_out, adapt);
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
hipError_t launch_sc_beta(const BlkArgs &ba, const double *partial, const PairState &ps, hipStream_t s)
{
    hipLaunchKernelGGL(k_sc_beta, pair_grid(ps.np), dim3(256), 0, s, ba, partial, ps);
    return hipGetLastError();
}
hipError_t launch_sc_outer(const BlkArgs &ba, const double *pe, const double *po, int first, double tol,
                           const OuterState &os, hipStream_t s)
{
    const int np = ba.n_rhs * ba.nb;
    hipLaunchKernelGGL(k_sc_outer, pair_grid(np), dim3(256), 0, s, ba, pe, po, first, tol * tol, os, np);
    return hipGetLastError();
}

// ------------------------------------------------- pair merge, network guard

__global__ void __launch_bounds__(256) k_merge_pairs(const double *src, double *dst, const int32_t *mask,
                                                      const int64_t *soff, int nb, int64_t total, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t site = i / 24, r = site / total, q = site - r * total;
    const int b = find_block(soff, nb, q);
    if (mask[r * nb + b]) dst[i] = src[i];
}

hipError_t launch_merge_pairs(const dd_blocks *B, const double *src, double *dst, const int32_t *mask, int n_rhs,
                              hipStream_t s)
{
    const int64_t total = B->soff[B->nb], n = (int64_t)n_rhs * total * 24;
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_merge_pairs, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, src, dst, mask, B->d_soff,
                       B->nb, total, n);
    return hipGetLastError();
}

// One workgroup per pair: a non-finite value anywhere in the pair's z makes
// z = v for the whole pair.  Nothing is cleared beforehand (the flag lives in
// LDS), so the kernel can be replayed from a captured graph.
template <typename SP>
__global__ void __launch_bounds__(256) k_nn_guard(const SP *v, SP *z, const int64_t *soff, const int32_t *h, int nb,
                                                   int n_rhs, const int32_t *active, int32_t *flags)
{
    __shared__ int bad;
    const int pair = blockIdx.x, r = pair / nb, b = pair - r * nb;
    if (active && !active[pair]) return;
    const int hb = h[b];
    const int64_t base = (soff[b] >> 1) * 24 * n_rhs + (int64_t)r * 24 * hb;
    const int n = 24 * hb;
    if (threadIdx.x == 0) bad = 0;
    __syncthreads();
    int mine = 0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) mine |= !isfinite(z[base + i]);
    if (mine) bad = 1;
    __syncthreads();
    if (!bad) return;
    for (int i = threadIdx.x; i < n; i += blockDim.x) z[base + i] = v[base + i];
    if (threadIdx.x == 0 && flags) flags[pair] |= 16;
}

hipError_t launch_nn_guard(const dd_blocks *B, const void *v, void *z, dd_prec sp, int n_rhs, const int32_t *active,
                           int32_t *flags, hipStream_t s)
{
    const int np = n_rhs * B->nb;
    if (np == 0) return hipSuccess;
    if (sp == DD_F64)
        hipLaunchKernelGGL(k_nn_guard<double>, dim3(np), dim3(256), 0, s, (const double *)v, (double *)z, B->d_soff,
                           B->d_h, B->nb, n_rhs, active, flags);
    else
        hipLaunchKernelGGL(k_nn_guard<float>, dim3(np), dim3(256), 0, s, (const float *)v, (float *)z, B->d_soff,
                           B->d_h, B->nb, n_rhs, active, flags);
    return hipGetLastError();
}

// ------------------------------------------------- multi-boson boundary norm

// S[b] = sum_k sum_{i in dLambda_0^b} | u_k chi_k(i) + y_k(i) |^2, FP64.
// y: solutions in the boundary layout [k][q][24]; chi: [k][q_bnd][24].
__global__ void __launch_bounds__(256) k_mb_norm(int nb, int nf, const double *u, const double *chi,
                                                 const double *y, const int64_t *soff, const int64_t *boff,
                                                 const int32_t *bnd, int64_t total, int64_t total_bnd, double *S,
                                                 int accumulate)
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
    if (threadIdx.x == 0) S[b] = (accumulate ? S[b] : 0.0) + red[0];
}

hipError_t launch_mb_norm(const dd_blocks *B, int n_fields, const double *u, const double *chi, const double *y,
                          double *S, int accumulate, hipStream_t s)
{
    if (B->nb == 0) return hipSuccess;
    hipLaunchKernelGGL(k_mb_norm, dim3(B->nb), dim3(256), 0, s, B->nb, n_fields, u, chi, y, B->d_soff, B->d_boff,
                       B->d_bnd, (int64_t)B->soff[B->nb], (int64_t)B->boff[B->nb], S, accumulate);
    return hipGetLastError();
}

// ------------------------------------------------- multi-boson exterior source

__global__ void __launch_bounds__(256) k_gather_ext_links(const double *U, const int64_t *xlink, double *uext,
                                                           int64_t n)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n * 18) return;
    const int64_t e = t / 18, k = t - e * 18;
    uext[t] = U[xlink[e] * 18 + k];
}

hipError_t launch_gather_ext_links(const dd_blocks *B, const double *U, double *uext, hipStream_t s)
{
    const int64_t n = (int64_t)B->x_code.size();
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_gather_ext_links, dim3((unsigned)((n * 18 + 255) / 256)), dim3(256), 0, s, U, B->d_x_link,
                       uext, n);
    return hipGetLastError();
}

// a field of the global lattice, read at one site: component c of the spinor
struct SrcSite {
    const double *p;
    __device__ __forceinline__ void load(int comp, double (&v)[1]) const { v[0] = p[comp]; }
};

// One thread per (receiving site group, field): the hops of chi from the
// group's exterior sites, -kappa (1 -/+ gamma_mu) W chi with W the link (or
// its adjoint) of the hop, summed in FP64 and added to xi at the site.
__global__ void __launch_bounds__(256) k_mb_exterior(const int32_t *gb, const int32_t *gs, const int32_t *gfirst,
                                                      const int32_t *code, const int64_t *nbr, const double *uext,
                                                      const int64_t *soff, const double *chi, double *xi, int ng, int nf,
                                                      int64_t V, int64_t total, double kappa, int parts)
{
    // one thread per (receiving site, field), the fields of a site in adjacent
    // lanes: their link loads are one address, served once per wavefront
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)ng * nf) return;
    const int g = (int)(t / nf), f = (int)(t % nf);
    double acc[1][24];
#pragma unroll
    for (int c = 0; c < 24; c++) acc[0][c] = 0;
    for (int e = gfirst[g]; e < gfirst[g + 1]; e++) {
        const int cd = code[e];
        if (!((cd >> 4) & parts)) continue;
        double u[18];
        const double sg = (cd & 8) ? -1.0 : 1.0;
#pragma unroll
        for (int k = 0; k < 18; k++) u[k] = sg * uext[(int64_t)e * 18 + k];
        const SrcSite src{chi + ((int64_t)f * V + nbr[e]) * 24};
        switch (cd & 7) {
        case 0: hop_term<0, true, double, double, 1>(acc, src, u); break;
        case 1: hop_term<0, false, double, double, 1>(acc, src, u); break;
        case 2: hop_term<1, true, double, double, 1>(acc, src, u); break;
        case 3: hop_term<1, false, double, double, 1>(acc, src, u); break;
        case 4: hop_term<2, true, double, double, 1>(acc, src, u); break;
        case 5: hop_term<2, false, double, double, 1>(acc, src, u); break;
        case 6: hop_term<3, true, double, double, 1>(acc, src, u); break;
        default: hop_term<3, false, double, double, 1>(acc, src, u); break;
        }
    }
    double *out = xi + ((int64_t)f * total + soff[gb[g]] + gs[g]) * 24;
#pragma unroll
    for (int c = 0; c < 24; c++) out[c] = fmad(-kappa, acc[0][c], out[c]);
}

hipError_t launch_mb_exterior(const dd_blocks *B, const double *uext, double kappa, int n_fields, const double *chi,
                              double *xi, int parts, hipStream_t s)
{
    const int ng = (int)B->xg_block.size();
    if (ng == 0 || n_fields == 0) return hipSuccess;
    if (!uext) return hipErrorInvalidValue;
    const int64_t V = (int64_t)B->L[0] * B->L[1] * B->L[2] * B->L[3];
    const int64_t n = (int64_t)ng * n_fields;
    hipLaunchKernelGGL(k_mb_exterior, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, B->d_xg_block, B->d_xg_site,
                       B->d_xg_first, B->d_x_code, B->d_x_nbr, uext, B->d_soff, chi, xi, ng, n_fields, V,
                       B->soff[B->nb], kappa, parts);
    return hipGetLastError();
}

}  // namespace dd
