// Persistent batched GMRES(m) for the even-odd reduced block systems
// Dhat e = f, Dhat = 1 - kappa^2 H_eo H_oe, one system per (block, rhs) pair.
//
// One workgroup solves one pair at a time, entirely on chip: Dhat (with FP32
// spinors its two eo hops in one pass over the x0-slices, the intermediate in
// LDS), classical Gram-Schmidt with FP64 dot products and FP64 vector updates
// and a second pass when cancellation calls for it, the Hessenberg matrix,
// complex Givens rotations, the residual estimate and the back substitution
// all stay inside the workgroup, so a pair needs no kernel launch per Krylov
// step and no host round trip.  A fixed grid of workgroups (as many as fit on the chip)
// pulls pairs from work queues with a global atomic counter until the queues
// are empty; blocks of uneven size are balanced by the queue order (largest
// first), and with one queue per XCD a block's right-hand sides are solved by
// workgroups of one XCD, so that they share the block's links in one L2.
//
// Vectors of a pair are component-major with the site innermost (stride h,
// the block's sites per parity), in the library's half-field layout for the
// caller's f and e and in per-workgroup basis slots of the workspace.
#include <hip/hip_runtime.h>

#include "dd_internal.h"
#include "dd_stencil.h"


namespace dd {

namespace {

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Sum of v over the workgroup, returned to every thread: a butterfly inside
// each wavefront, then the wavefronts in order (a fixed order).
template <int NT>
__device__ __forceinline__ double wg_sum1(double v, double *red)
{
    constexpr int NW = NT / 64;
    const double s = wave_sum(v);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    double t = 0;
#pragma unroll
    for (int w = 0; w < NW; w++) t += red[w];
    __syncthreads();
    return t;
}

// The workgroup's basis slot: M + 2 vectors behind one buffer descriptor,
// vector i at byte offset i * vbytes (an SGPR offset of the buffer loads).
struct Slot {
    Buf b;
    uint32_t vbytes;
};

struct PairGeo {
    int h;               // sites per parity
    const int32_t *nbr;  // the block shape's neighbour table [parity][h][8]
    Buf lk_b;            // the block's links
    uint32_t kstr;       // bytes between link entries
    Buf cl_b;            // the block's A^-1 of the clover term (walk hops with CL)
    uint32_t cl_kstr;    // bytes between its reals
};

// out = c_hop (H in) + c_self self + c_add add on the sites of parity p of
// one pair (`in` on the other parity); self and add may be null.  Returns the
// thread's share of |out|^2.  The caller separates it from readers of `out`
// at other sites with a barrier.
template <typename SP, typename LK, int NT>
__device__ __forceinline__ double wg_hop(const PairGeo &g, int p, const SP *in, SP *out, const SP *self, double c_self,
                                         double c_hop, const SP *add, double c_add)
{
    using AC = SP;
    HopCtx hc;
    hc.h0 = 0;
    hc.tv = 0;
    hc.grp_off = 0;
    hc.cstr = (uint32_t)g.h * (uint32_t)sizeof(SP);
    hc.kstr = g.kstr;
    hc.in_b = make_buf(in, (uint32_t)(24 * g.h) * (uint32_t)sizeof(SP));
    hc.lk_b = g.lk_b;
    hc.other0 = (1 - p) * g.h;
    const AC ch = (AC)c_hop, cs = (AC)c_self, ca = (AC)c_add;
    double nn = 0;
    for (int s = threadIdx.x; s < g.h; s += NT) {
        const int4 *q = reinterpret_cast<const int4 *>(g.nbr + (size_t)(p * g.h + s) * 8);
        const int4 a0 = q[0], a1 = q[1];
        hc.slot_self = p * g.h + s;
        AC acc[1][24];
#pragma unroll
        for (int c = 0; c < 24; c++) acc[0][c] = 0;
        hop_one<0, true, SP, LK, AC, 1, false>(acc, a0.x, nullptr, hc);
        hop_one<0, false, SP, LK, AC, 1, false>(acc, a0.y, nullptr, hc);
        hop_one<1, true, SP, LK, AC, 1, false>(acc, a0.z, nullptr, hc);
        hop_one<1, false, SP, LK, AC, 1, false>(acc, a0.w, nullptr, hc);
        hop_one<2, true, SP, LK, AC, 1, false>(acc, a1.x, nullptr, hc);
        hop_one<2, false, SP, LK, AC, 1, false>(acc, a1.y, nullptr, hc);
        hop_one<3, true, SP, LK, AC, 1, false>(acc, a1.z, nullptr, hc);
        hop_one<3, false, SP, LK, AC, 1, false>(acc, a1.w, nullptr, hc);
#pragma unroll
        for (int c = 0; c < 24; c++) {
            const size_t o = (size_t)c * g.h + s;
            AC v = ch * acc[0][c];
            if (self) v = fmad(cs, self[o], v);
            if (add) v = fmad(ca, add[o], v);
            const SP ov = (SP)v;
            out[o] = ov;
            nn += (double)ov * (double)ov;
        }
    }
    return nn;
}

// wg_hop by the x0-walk (dd_stencil.h): the input slices staged in LDS one
// after the other, each read once.  For blocks whose x0-slices hold at most
// kTile sites per parity; all threads call it.  CL: the hop result at each
// output site is multiplied by its A^-1 (g.cl_b) before the combination.
template <typename SP, typename LK, int NT, bool CL = false>
__device__ __forceinline__ double wg_hop_walk(const PairGeo &g, int p, int ns, SP *stage, const SP *in, SP *out,
                                              const SP *self, double c_self, double c_hop, const SP *add, double c_add)
{
    using AC = SP;
    WalkPos w;
    w.p = p;
    w.hb = g.h;
    w.hs = g.h / ns;
    w.k = threadIdx.x;
    w.s0 = 0;
    w.s1 = ns;
    w.nbt = g.nbr + (size_t)p * g.h * 8;
    HopCtx hc;
    hc.h0 = 0;
    hc.tv = 0;
    hc.slot_self = 0;
    hc.other0 = 0;
    hc.grp_off = 0;
    hc.cstr = (uint32_t)g.h * (uint32_t)sizeof(SP);
    hc.kstr = g.kstr;
    hc.in_b = make_buf(in, (uint32_t)(24 * g.h) * (uint32_t)sizeof(SP));
    hc.lk_b = g.lk_b;
    const AC ch = (AC)c_hop, cs = (AC)c_self, ca = (AC)c_add;
    const uint32_t vbytes = (uint32_t)(24 * g.h) * (uint32_t)sizeof(SP);
    const Buf ob = make_buf(out, vbytes), sb = make_buf(self, self ? vbytes : 0), ab = make_buf(add, add ? vbytes : 0);
    const bool has_self = self != nullptr, has_add = add != nullptr;
    double nn = 0;
    walk_run<SP, LK, AC, 1>(w, ns, stage, hc, [&](const AC (&acc1)[1][24], int h) {
        AC acc[24];
#pragma unroll
        for (int c = 0; c < 24; c++) acc[c] = acc1[0][c];
        if constexpr (CL) clover_mul<SP, AC>(acc, g.cl_b, (uint32_t)(p * g.h + h) * (uint32_t)sizeof(SP), g.cl_kstr);
        const uint32_t vo = (uint32_t)h * (uint32_t)sizeof(SP);
#pragma unroll
        for (int half = 0; half < 2; half++) {
            SP sv[12], av[12];
#pragma unroll
            for (int q = 0; q < 12; q++) {
                sv[q] = bload<SP, kKeep>(sb, vo, (uint32_t)(12 * half + q) * hc.cstr);
                av[q] = bload<SP, kKeep>(ab, vo, (uint32_t)(12 * half + q) * hc.cstr);
            }
#pragma unroll
            for (int q = 0; q < 12; q++) {
                AC v = ch * acc[12 * half + q];
                if (has_self) v = fmad(cs, (AC)sv[q], v);
                if (has_add) v = fmad(ca, (AC)av[q], v);
                const SP ov = (SP)v;
                bstore<SP, kKeep>(ob, ov, vo, (uint32_t)(12 * half + q) * hc.cstr);
                nn += (double)ov * (double)ov;
            }
        }
    });
    return nn;
}

// out = c_hop H_eo (H_oe in) + c_self self + c_add add on the even sites of
// one pair in one pass over the x0-slices (dhat_run in dd_stencil.h): the odd
// intermediate stays in LDS (sa: input slice, sb: intermediate slice).  One
// rhs per thread, FP32 spinors; self and add may be null.  Returns the
// thread's share of |out|^2.  All threads call it.  CL: the clover term's
// A_oo^-1 on each intermediate site before it goes to LDS and A_ee^-1 on the
// hop result at each output site (out = c_hop A_ee^-1 H_eo A_oo^-1 H_oe in + ..).
template <typename SP, typename LK, int NT, bool CL = false>
__device__ __forceinline__ double wg_dhat_walk(const PairGeo &g, int ns, SP *sa, SP *sb, const SP *in, SP *out,
                                               const SP *self, double c_self, double c_hop, const SP *add,
                                               double c_add)
{
    using AC = SP;
    const int hs = g.h / ns, k = threadIdx.x;
    const WalkPos wodd{1, g.h, hs, k, 0, ns, g.nbr + (size_t)g.h * 8};
    const WalkPos weven{0, g.h, hs, k, 0, ns, g.nbr};
    HopCtx hc;
    hc.h0 = 0;
    hc.tv = 0;
    hc.slot_self = 0;
    hc.other0 = 0;
    hc.grp_off = 0;
    hc.cstr = (uint32_t)g.h * (uint32_t)sizeof(SP);
    hc.kstr = g.kstr;
    hc.in_b = make_buf(in, (uint32_t)(24 * g.h) * (uint32_t)sizeof(SP));
    hc.lk_b = g.lk_b;
    const AC ch = (AC)c_hop, cs = (AC)c_self, ca = (AC)c_add;
    const uint32_t vbytes = (uint32_t)(24 * g.h) * (uint32_t)sizeof(SP);
    const Buf ob = make_buf(out, vbytes), fb = make_buf(self, self ? vbytes : 0), ab = make_buf(add, add ? vbytes : 0);
    const bool has_self = self != nullptr, has_add = add != nullptr;
    double nn = 0;
    auto epi = [&](const AC (&acc1)[1][24], int h) {
        AC acc[24];
#pragma unroll
        for (int c = 0; c < 24; c++) acc[c] = acc1[0][c];
        if constexpr (CL) clover_mul<SP, AC>(acc, g.cl_b, (uint32_t)h * (uint32_t)sizeof(SP), g.cl_kstr);  // A_ee^-1
        const uint32_t vo = (uint32_t)h * (uint32_t)sizeof(SP);
#pragma unroll
        for (int half = 0; half < 2; half++) {
            SP sv[12], av[12];
#pragma unroll
            for (int q = 0; q < 12; q++) {
                sv[q] = bload<SP, kKeep>(fb, vo, (uint32_t)(12 * half + q) * hc.cstr);
                av[q] = bload<SP, kKeep>(ab, vo, (uint32_t)(12 * half + q) * hc.cstr);
            }
#pragma unroll
            for (int q = 0; q < 12; q++) {
                AC v = ch * acc[12 * half + q];
                if (has_self) v = fmad(cs, (AC)sv[q], v);
                if (has_add) v = fmad(ca, (AC)av[q], v);
                const SP ov = (SP)v;
                bstore<SP, kKeep>(ob, ov, vo, (uint32_t)(12 * half + q) * hc.cstr);
                nn += (double)ov * (double)ov;
            }
        }
    };
    dhat_run<SP, LK, AC>(
        wodd, weven, ns, sa, sb, hc, [&](int q, SP (&v)[24][1]) { walk_load<SP, 1>(v, hc, q, hs, k); }, epi, true,
        [&](AC (&a)[24], int h) {
            if constexpr (CL) clover_mul<SP, AC>(a, g.cl_b, (uint32_t)(g.h + h) * (uint32_t)sizeof(SP), g.cl_kstr);
        });
    return nn;
}

// out[2i] + i out[2i+1] = <V_i, V_iw> = sum conj(V_i) V_iw for i <= j, FP64
// products and sums.  Every thread runs over its own elements and keeps the
// sums of a group of up to 8 basis vectors (all loads of an element issued
// together; V_iw read once per group, each V_i once); then a butterfly inside
// each wavefront and the wavefronts in order through LDS (red: NT / 64 * NV
// doubles).  With norm, out[NV - 1] = |V_iw|^2.  Ends with a barrier.
template <typename SP, int M, int NT, int NV>
__device__ __forceinline__ void gs_dots(const Slot &sl, int iw, int h, int j, bool norm, double *out, double *red)
{
    constexpr int NW = NT / 64, GS = 8;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const uint32_t hb = (uint32_t)h * (uint32_t)sizeof(SP), wo = (uint32_t)iw * sl.vbytes;
#pragma unroll 1
    for (int i0 = 0; i0 <= j; i0 += GS) {
        const bool do_norm = norm && i0 == 0;
        double d[2 * GS], nn = 0;
#pragma unroll
        for (int k = 0; k < 2 * GS; k++) d[k] = 0;
#pragma unroll 1
        for (int cc = 0; cc < 12; cc++)
#pragma unroll 1
            for (int s = threadIdx.x; s < h; s += NT) {
                const uint32_t vo = (uint32_t)(2 * cc * h + s) * (uint32_t)sizeof(SP);
                const double wr = (double)bload<SP, kKeep>(sl.b, vo, wo), wi = (double)bload<SP, kKeep>(sl.b, vo, wo + hb);
                // the basis offsets are recomputed here (scalar arithmetic) rather
                // than hoisted out of the loops into scalar registers
                uint32_t vbytes = sl.vbytes;
                __asm__ volatile("" : "+s"(vbytes));
#pragma unroll
                for (int k = 0; k < GS; k++)
                    if (i0 + k <= j) {
                        const uint32_t io = (uint32_t)(i0 + k) * vbytes;
                        const double vr = (double)bload<SP, kKeep>(sl.b, vo, io), vi = (double)bload<SP, kKeep>(sl.b, vo, io + hb);
                        d[2 * k] = fma(vr, wr, fma(vi, wi, d[2 * k]));
                        d[2 * k + 1] = fma(vr, wi, fma(-vi, wr, d[2 * k + 1]));
                    }
                if (do_norm) nn = fma(wr, wr, fma(wi, wi, nn));
            }
#pragma unroll
        for (int k = 0; k < GS; k++)
            if (i0 + k <= j) {
                const double re = wave_sum(d[2 * k]), im = wave_sum(d[2 * k + 1]);
                if (lane == 0) {
                    red[wave * NV + 2 * (i0 + k)] = re;
                    red[wave * NV + 2 * (i0 + k) + 1] = im;
                }
            }
        if (do_norm) {
            const double sn = wave_sum(nn);
            if (lane == 0) red[wave * NV + NV - 1] = sn;
        }
    }
    __syncthreads();
    const int k = threadIdx.x;
    if (k < 2 * (j + 1) || (norm && k == NV - 1)) {
        double t = 0;
#pragma unroll
        for (int w = 0; w < NW; w++) t += red[w * NV + k];
        out[k] = t;
    }
    __syncthreads();
}

// dst = (dst + sgn * sum_{i0<=i<n} c_i V_i) * scale with complex c_i from LDS (read
// as used, so that they take no registers), FP64 arithmetic, stored in SP; dst is
// a buffer and the byte offset of the vector in it.  Each thread updates its
// own elements: no barrier inside.
template <typename SP, int M, int NT>
__device__ __forceinline__ void combine(const Slot &sl, const Buf &db, uint32_t dso, int h, int n, const double *c,
                                        double sgn, double scale, int i0 = 0)
{
    const uint32_t hb = (uint32_t)h * (uint32_t)sizeof(SP);
#pragma unroll 1
    for (int cc = 0; cc < 12; cc++)
#pragma unroll 1
        for (int s = threadIdx.x; s < h; s += NT) {
            // compiler-only fence: the coefficients are re-read from LDS in every
            // iteration instead of being held in registers across the loop
            __asm__ volatile("" ::: "memory");
            const uint32_t vo = (uint32_t)(2 * cc * h + s) * (uint32_t)sizeof(SP);
            double wr = (double)bload<SP, kKeep>(db, vo, dso), wi = (double)bload<SP, kKeep>(db, vo, dso + hb);
            // the basis offsets are recomputed here (scalar arithmetic) rather
            // than hoisted out of the loops into scalar registers
            uint32_t vbytes = sl.vbytes;
            __asm__ volatile("" : "+s"(vbytes));
#pragma unroll
            for (int i = 0; i <= M; i++)
                if (i >= i0 && i < n) {
                    const uint32_t io = (uint32_t)i * vbytes;
                    const double vr = (double)bload<SP, kKeep>(sl.b, vo, io), vi = (double)bload<SP, kKeep>(sl.b, vo, io + hb);
                    const double cr = sgn * c[2 * i], ci = sgn * c[2 * i + 1];
                    wr = fma(cr, vr, fma(-ci, vi, wr));
                    wi = fma(cr, vi, fma(ci, vr, wi));
                }
            bstore<SP, kKeep>(db, (SP)(wr * scale), vo, dso);
            bstore<SP, kKeep>(db, (SP)(wi * scale), vo, dso + hb);
        }
}

// Stop codes of a Krylov step
enum { kGoOn = 0, kRestart = 1, kConverged = 2, kMaxIter = 3, kNonFinite = 4, kPaused = 5 };

}  // namespace

// One launch solves every pair listed in the queues whose `active` flag is set
// and leaves e = Dhat^{-1} f (to the relative tolerance, or the last iterate)
// in x; every workgroup leaves the loop once all queues are drained.
// WALK: the hops walk the x0-slices, else wg_hop; with FP32 spinors both
// hops of Dhat are one pass over the slices (wg_dhat_walk), with FP64 two
// (wg_hop_walk).  FP32 spinors: at most 168 registers, so that three
// wavefronts share a SIMD.
template <typename SP, typename LK, int M, int NT, bool WALK, bool CL = false>
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(sizeof(SP) == 4 && !CL ? 3 : 1))) k_gmres(GmArgs a)
{
    static_assert(!CL || WALK, "the clover term takes the walking hops");
    constexpr bool FUSED = WALK && sizeof(SP) == 4;
    constexpr int NW = NT / 64;
    constexpr int NV = 2 * (M + 1) + 1;
    static_assert(NV <= NT, "one thread per reduced value");
    __shared__ double red[NW];
    __shared__ SP stage[WALK ? 24 * kTile : 1];  // input slice of the walking hops
    // the Gram-Schmidt sums (sum, red2) and the back substitution's y share
    // one buffer with the intermediate slice of wg_dhat_walk: they are dead
    // while it runs (barriers on both sides), and three workgroups of 256
    // threads keep fitting on a compute unit
    constexpr int NSUM = NW * NV + NV + 2 * (M + 1);
    constexpr int NSL = FUSED ? 24 * kTile * (int)sizeof(SP) / (int)sizeof(double) : 0;
    __shared__ double xbuf[NSL > NSUM ? NSL : NSUM];
    double *const red2 = xbuf, *const sum = xbuf + NW * NV, *const yv = sum + NV;
    SP *const stage2 = reinterpret_cast<SP *>(xbuf);
    // the Hessenberg matrix's entries i <= j (the subdiagonal is folded into the
    // rotations at once and never stored), packed by columns: H_ij at
    // hm(i, j)[0] + i hm(i, j)[1]
    __shared__ double Hm[M * (M + 1)];
    auto hm = [&](int i, int j) { return Hm + (j * (j + 1) + 2 * i); };
    __shared__ double cs[M], sn[2 * M], gv[2 * (M + 1)];
    __shared__ int s_pair, s_stop;
    __shared__ double s_est;

    SP *V = reinterpret_cast<SP *>(a.ws) + (int64_t)blockIdx.x * (M + 2) * a.vstr;
    SP *tmp = V + (int64_t)(M + 1) * a.vstr;
    Slot sl;
    sl.vbytes = (uint32_t)a.vstr * (uint32_t)sizeof(SP);
    sl.b = make_buf(V, (uint32_t)(M + 2) * sl.vbytes);
    const int m = a.m;
    const double k2 = a.k2;
    int tried = 0;  // thread 0: queues found empty so far
    const int q0 = (int)(blockIdx.x % (unsigned)a.nq);
    for (;;) {
        if (threadIdx.x == 0) {
            int pr = -1;
            while (tried < a.nq) {
                const int qq = (q0 + tried) % a.nq;
                const int k = atomicAdd(a.qctr + qq, 1);
                if (k < a.qoff[qq + 1] - a.qoff[qq]) {
                    pr = a.queue[a.qoff[qq] + k];
                    break;
                }
                tried++;
            }
            s_pair = pr;
        }
        __syncthreads();
        const int pair = uni(s_pair);
        __syncthreads();
        if (pair < 0) break;
        if (!a.active[pair]) continue;

        const int b = pair % a.nb, r = pair / a.nb;
        const int h = uni(a.h[b]);
        const int ns = uni(a.ext[4 * b]);  // x0-slices of the block
        const int64_t so = uni64(a.soff[b]);
        PairGeo g;
        g.h = h;
        g.nbr = a.nbr + uni64(a.nbr_off[b]);
        g.kstr = (uint32_t)(4 * h) * (uint32_t)sizeof(LK);
        g.lk_b = make_buf(reinterpret_cast<const LK *>(a.links) + so * kLinkReals,
                          (uint32_t)(2 * h * kLinkReals) * (uint32_t)sizeof(LK));
        g.cl_b = make_buf(CL ? reinterpret_cast<const SP *>(a.clover) + so * kCloverReals : nullptr,
                          CL ? (uint32_t)(kCloverReals * 2 * h) * (uint32_t)sizeof(SP) : 0u);
        g.cl_kstr = (uint32_t)(2 * h) * (uint32_t)sizeof(SP);
        const int64_t pb = (so >> 1) * 24 * a.n_rhs + (int64_t)r * 24 * h;
        const SP *f = reinterpret_cast<const SP *>(a.rhs) + pb;
        SP *x = reinterpret_cast<SP *>(a.x) + pb;
        SP *rg = a.r ? reinterpret_cast<SP *>(a.r) + pb : nullptr;  // paused residual
        const SP *z0 = a.z0 ? reinterpret_cast<const SP *>(a.z0) + pb : nullptr;
        const int n = 24 * h;
        // algorithmic bytes (kept by thread 0): a vector of the pair, and one eo
        // hop's links shared by the block's n_rhs pairs
        const double vb = (double)n * sizeof(SP);
        const double lb = (double)a.nlinks[b] * kLinkAlgReals * sizeof(LK) / a.n_rhs;
        double moved;

        // fresh start: beta0 = |f|, x = 0, V_0 = f / beta0; resumed: V_0 = r / |r|
        const SP *start = a.resume ? rg : f;
        double nn = 0;
        for (int e = threadIdx.x; e < n; e += NT) {
            const double v = (double)start[e];
            nn = fma(v, v, nn);
        }
        double beta = sqrt(wg_sum1<NT>(nn, red));
        const double beta0 = a.resume ? a.beta0[pair] : beta;
        double tolp = a.tol;
        if (a.adapt && a.orr[pair] > 0)
            tolp = fmax(tolp, fmin(0.3 * a.tol_out * sqrt(a.obb[pair] / a.orr[pair]), 0.1));
        const bool ok0 = isfinite(beta) && beta > 0;
        const double inv0 = ok0 ? 1.0 / beta : 0.0;
        for (int e = threadIdx.x; e < n; e += NT) {
            V[e] = (SP)((double)start[e] * inv0);
            if (!a.resume) x[e] = (SP)0;
        }
        moved = a.resume ? 3.0 * vb : 4.0 * vb;
        if (threadIdx.x == 0 && !a.resume && a.beta0) a.beta0[pair] = beta0;
        __syncthreads();
        int it = 0, stop = ok0 ? kGoOn : (beta == 0 ? kConverged : kNonFinite);
        if (ok0 && beta <= tolp * beta0) stop = kConverged;
        double est = ok0 ? beta : 0.0;
        int cycles = 0;
        while (stop == kGoOn || stop == kRestart) {
            if (threadIdx.x == 0) {
                for (int i = 0; i <= M; i++) gv[2 * i] = gv[2 * i + 1] = 0;
                gv[0] = beta;
            }
            int k = 0;
            stop = kGoOn;
            const bool use_z = z0 && cycles == 0;
            for (int j = 0; j < m && stop == kGoOn; j++) {
                SP *vj = V + (int64_t)j * a.vstr, *w = V + (int64_t)(j + 1) * a.vstr;
                // w = Dhat v_j, or with the flexible first direction z_0 = N(v_0) =
                // N(r) / beta: w = Dhat z_0
                const bool zf = j == 0 && use_z;
                const SP *src = zf ? z0 : vj;
                const double cs1 = zf ? 1.0 / beta : 1.0, ch1 = zf ? -k2 / beta : -k2;
                if constexpr (FUSED) {
                    wg_dhat_walk<SP, LK, NT, CL>(g, ns, stage, stage2, src, w, src, cs1, ch1, nullptr, 0.0);
                } else if constexpr (WALK) {
                    wg_hop_walk<SP, LK, NT, CL>(g, 1, ns, stage, src, tmp, nullptr, 0.0, 1.0, nullptr, 0.0);
                    __syncthreads();
                    wg_hop_walk<SP, LK, NT, CL>(g, 0, ns, stage, tmp, w, src, cs1, ch1, nullptr, 0.0);
                } else {
                    wg_hop<SP, LK, NT>(g, 1, src, tmp, nullptr, 0.0, 1.0, nullptr, 0.0);
                    __syncthreads();
                    wg_hop<SP, LK, NT>(g, 0, tmp, w, src, cs1, ch1, nullptr, 0.0);
                }
                __syncthreads();
                // Classical Gram-Schmidt with FP64 sums and updates: h = V^H w and
                // |w|^2 in one pass; then |w - V h|^2 = |w|^2 - |h|^2 (V
                // orthonormal).  When that keeps less than a fraction eta of |w|
                // (cancellation), a second pass reorthogonalizes (CGS2): w -= V h,
                // then the corrections c = V^H w and |w|^2.  The last pass writes
                // v_{j+1} = (w - V s) / hn with s = h, or s = c after a second pass.
                gs_dots<SP, M, NT, NV>(sl, j + 1, h, j, true, sum, red2);
                if (threadIdx.x == 0)
                    for (int i = 0; i <= j; i++) {
                        hm(i, j)[0] = sum[2 * i];
                        hm(i, j)[1] = sum[2 * i + 1];
                    }
                double s2 = 0;
                for (int i = 0; i <= j; i++) s2 += sum[2 * i] * sum[2 * i] + sum[2 * i + 1] * sum[2 * i + 1];
                double hh = sum[NV - 1] - s2;
                const uint32_t wso = (uint32_t)(j + 1) * sl.vbytes;
                const bool second = !(hh > a.reorth2 * sum[NV - 1]);
                if (second) {
                    combine<SP, M, NT>(sl, sl.b, wso, h, j + 1, sum, -1.0, 1.0);
                    __syncthreads();
                    gs_dots<SP, M, NT, NV>(sl, j + 1, h, j, true, sum, red2);
                    s2 = 0;
                    for (int i = 0; i <= j; i++) s2 += sum[2 * i] * sum[2 * i] + sum[2 * i + 1] * sum[2 * i + 1];
                    hh = sum[NV - 1] - s2;
                    if (threadIdx.x == 0)
                        for (int i = 0; i <= j; i++) {
                            hm(i, j)[0] += sum[2 * i];
                            hm(i, j)[1] += sum[2 * i + 1];
                        }
                    moved += (2.0 * (j + 1) + 4.0) * vb;
                }
                const double hn = sqrt(fmax(hh, 0.0));
                if (threadIdx.x == 0) {
                    // previous rotations on column j: (a, b) <- (c a + s b, -conj(s) a + c b)
                    for (int i = 0; i < j; i++) {
                        double *pa = hm(i, j), *pb2 = hm(i + 1, j);
                        const double ar = pa[0], ai = pa[1], br = pb2[0], bi = pb2[1];
                        const double sr = sn[2 * i], si = sn[2 * i + 1], cc = cs[i];
                        pa[0] = cc * ar + (sr * br - si * bi);
                        pa[1] = cc * ai + (sr * bi + si * br);
                        pb2[0] = cc * br - (sr * ar + si * ai);
                        pb2[1] = cc * bi - (sr * ai - si * ar);
                    }
                    // new rotation zeroing the real subdiagonal hn below a = Hm[j][j]
                    double *pd = hm(j, j);
                    const double ar = pd[0], ai = pd[1];
                    const double aa = sqrt(ar * ar + ai * ai);
                    double cc, sr, si;
                    if (aa == 0.0) {
                        cc = 0.0;
                        sr = 1.0;
                        si = 0.0;
                        pd[0] = hn;
                        pd[1] = 0.0;
                    } else {
                        const double t = sqrt(aa * aa + hn * hn);
                        cc = aa / t;
                        sr = ar / aa * (hn / t);
                        si = ai / aa * (hn / t);
                        pd[0] = ar / aa * t;
                        pd[1] = ai / aa * t;
                    }
                    cs[j] = cc;
                    sn[2 * j] = sr;
                    sn[2 * j + 1] = si;
                    const double gr = gv[2 * j], gi = gv[2 * j + 1];
                    gv[2 * j] = cc * gr;
                    gv[2 * j + 1] = cc * gi;
                    gv[2 * j + 2] = -(sr * gr + si * gi);
                    gv[2 * j + 3] = -(sr * gi - si * gr);
                    const double e2 = sqrt(gv[2 * j + 2] * gv[2 * j + 2] + gv[2 * j + 3] * gv[2 * j + 3]);
                    int st = kGoOn;
                    if (!isfinite(e2) || !isfinite(hn) || !isfinite(pd[0]) || !isfinite(pd[1])) st = kNonFinite;
                    else if (e2 <= tolp * beta0 || !(hn > 0.0)) st = kConverged;
                    else if (it + 1 >= a.max_iter) st = kMaxIter;
                    else if (j + 1 == m) st = kRestart;
                    s_stop = st;
                    s_est = e2;
                }
                // third pass: v_{j+1} = (w - V c) / hn (skipped on breakdown)
                const double inv = hn > 0.0 && isfinite(hn) ? 1.0 / hn : 0.0;
                if (inv > 0.0) combine<SP, M, NT>(sl, sl.b, wso, h, j + 1, sum, -1.0, inv);
                __syncthreads();
                stop = s_stop;
                if (stop != kNonFinite) {
                    est = s_est;
                    k = j + 1;
                }
                it++;
                // the product: input and w, the links (with two hops: the
                // intermediate twice, the self term, the input, once more and
                // the links twice); two Gram-Schmidt passes: V_0..V_j and w,
                // then again and w written (a reorthogonalizing pair counted above)
                moved += FUSED ? (2.0 * (j + 1) + 5.0) * vb + lb : (2.0 * (j + 1) + 8.0) * vb + 2.0 * lb;
                __syncthreads();
            }
            // x += V y with R y = g (back substitution on the rotated Hessenberg matrix)
            if (k > 0) {
                if (threadIdx.x == 0) {
                    for (int i = k - 1; i >= 0; i--) {
                        double sr = gv[2 * i], si = gv[2 * i + 1];
                        for (int l = i + 1; l < k; l++) {
                            const double hr = hm(i, l)[0], hi = hm(i, l)[1];
                            sr -= hr * yv[2 * l] - hi * yv[2 * l + 1];
                            si -= hr * yv[2 * l + 1] + hi * yv[2 * l];
                        }
                        const double dr = hm(i, i)[0], di = hm(i, i)[1];
                        const double den = dr * dr + di * di;
                        yv[2 * i] = (sr * dr + si * di) / den;
                        yv[2 * i + 1] = (si * dr - sr * di) / den;
                    }
                }
                __syncthreads();
                combine<SP, M, NT>(sl, make_buf(x, (uint32_t)n * (uint32_t)sizeof(SP)), 0u, h, k, yv, 1.0, 1.0,
                                   use_z ? 1 : 0);
                if (use_z) {
                    // x += (y_0 / beta) z0 on the same elements this thread updated
                    const double zr = yv[0] / beta, zi = yv[1] / beta;
                    for (int cc = 0; cc < 12; cc++)
                        for (int s = threadIdx.x; s < h; s += NT) {
                            const int o = 2 * cc * h + s;
                            const double ar = (double)z0[o], ai = (double)z0[o + h];
                            x[o] = (SP)((double)x[o] + (zr * ar - zi * ai));
                            x[o + h] = (SP)((double)x[o + h] + (zr * ai + zi * ar));
                        }
                    moved += 3.0 * vb;
                }
                moved += (k + 2.0) * vb;
                __syncthreads();
            }
            if (stop != kRestart) break;
            // restart from the explicit residual V_0 = f - Dhat x
            double rn;
            if constexpr (FUSED) {
                rn = wg_dhat_walk<SP, LK, NT, CL>(g, ns, stage, stage2, x, V, x, -1.0, k2, f, 1.0);
            } else if constexpr (WALK) {
                wg_hop_walk<SP, LK, NT, CL>(g, 1, ns, stage, x, tmp, nullptr, 0.0, 1.0, nullptr, 0.0);
                __syncthreads();
                rn = wg_hop_walk<SP, LK, NT, CL>(g, 0, ns, stage, tmp, V, x, -1.0, k2, f, 1.0);
            } else {
                wg_hop<SP, LK, NT>(g, 1, x, tmp, nullptr, 0.0, 1.0, nullptr, 0.0);
                __syncthreads();
                rn = wg_hop<SP, LK, NT>(g, 0, tmp, V, x, -1.0, k2, f, 1.0);
            }
            beta = sqrt(wg_sum1<NT>(rn, red));
            est = beta;
            moved += FUSED ? 3.0 * vb + lb : 6.0 * vb + 2.0 * lb;
            if (!isfinite(beta)) {
                stop = kNonFinite;
                break;
            }
            if (beta <= tolp * beta0) {
                stop = kConverged;
                break;
            }
            cycles++;
            if (a.max_cycles > 0 && cycles >= a.max_cycles && rg) {
                // hand the residual back (for a new first direction) and resume later
                for (int e = threadIdx.x; e < n; e += NT) rg[e] = V[e];
                moved += 2.0 * vb;
                stop = kPaused;
                break;
            }
            const double ib = 1.0 / beta;
            for (int e = threadIdx.x; e < n; e += NT) V[e] = (SP)((double)V[e] * ib);
            moved += 2.0 * vb;
            __syncthreads();
            stop = kRestart;
        }
        if (threadIdx.x == 0) {
            a.iters[pair] += it;
            if (a.bytes) a.bytes[pair] += moved;
            if (stop == kNonFinite) a.flags[pair] |= 4;
            if (a.relres) a.relres[pair] = beta0 > 0 ? est / beta0 : 0.0;
            if (a.more) a.more[pair] = stop == kPaused ? 1 : 0;
        }
        __syncthreads();
    }
}

__global__ void k_fill_i32(int32_t *p, int n, int32_t v)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

namespace {

template <typename SP, typename LK, bool WALK, bool CL>
struct GmKernels {
    static const void *get(int M, int nt)
    {
        if (M == 8 && nt == 256) return (const void *)k_gmres<SP, LK, 8, 256, WALK, CL>;
        if (M == 8 && nt == 512) return (const void *)k_gmres<SP, LK, 8, 512, WALK, CL>;
        if (M == 16 && nt == 256) return (const void *)k_gmres<SP, LK, 16, 256, WALK, CL>;
        if (M == 16 && nt == 512) return (const void *)k_gmres<SP, LK, 16, 512, WALK, CL>;
        return nullptr;
    }
};

template <bool WALK, bool CL>
const void *gmres_kernel_w(dd_prec prec, int M, int nt)
{
    if (prec == DD_F64) return GmKernels<double, double, WALK, CL>::get(M, nt);
    if (prec == DD_F32) return GmKernels<float, float, WALK, CL>::get(M, nt);
    if (prec == DD_BF16) return GmKernels<float, uint16_t, WALK, CL>::get(M, nt);
    return nullptr;
}

// the clover term takes the walking hops only (null otherwise)
const void *gmres_kernel(dd_prec prec, int M, int nt, bool walk, bool cl)
{
    if (cl) return walk ? gmres_kernel_w<true, true>(prec, M, nt) : nullptr;
    return walk ? gmres_kernel_w<true, false>(prec, M, nt) : gmres_kernel_w<false, false>(prec, M, nt);
}

}  // namespace

int gmres_basis_m(int restart) { return restart <= 8 ? 8 : 16; }

hipError_t gmres_occupancy(dd_prec prec, int restart, int nt, bool walk, bool cl, int *wgs_per_cu)
{
    const void *k = gmres_kernel(prec, gmres_basis_m(restart), nt, walk, cl);
    if (!k) return hipErrorInvalidValue;
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(wgs_per_cu, k, nt, 0);
}

hipError_t launch_gmres(const GmArgs &a, dd_prec prec, int nt, int grid, hipStream_t st)
{
    if (a.m < 1 || a.m > 16 || grid < 1 || a.nq < 1) return hipErrorInvalidValue;
    const void *k = gmres_kernel(prec, gmres_basis_m(a.m), nt, a.walk != 0, a.clover != nullptr);
    if (!k) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_fill_i32, dim3((a.nq + 255) / 256), dim3(256), 0, st, a.qctr, a.nq, 0);
    const int np = a.nb * a.n_rhs;
    if (a.more) hipLaunchKernelGGL(k_fill_i32, dim3((np + 255) / 256), dim3(256), 0, st, a.more, np, 0);
    void *args[] = {const_cast<GmArgs *>(&a)};
    return hipLaunchKernel(k, dim3(grid), dim3(nt), args, 0, st);
}

}  // namespace dd
