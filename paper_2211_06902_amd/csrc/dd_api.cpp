// C ABI of libdd: contexts, geometry, gauge packing, D_Lambda application,
// batched block solves and the block-local multi-boson action.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "dd_geometry.h"
#include "dd_host.h"
#include "dd_internal.h"

using namespace dd;

namespace {
const char *kVersion = "libdd 0.1 (gfx950)";
thread_local std::string g_err;  // message of calls made without a context
}  // namespace

namespace dd {

uint64_t next_blocks_serial()
{
    static std::atomic<uint64_t> n{0};
    return ++n;
}

dd_status fail(dd_ctx *ctx, dd_status st, const std::string &msg)
{
    if (ctx) ctx->err = msg;
    else g_err = msg;
    return st;
}

// Grow-only named workspace.  Contents are not preserved on growth.
void *workspace(dd_ctx *ctx, const std::string &name, size_t bytes, hipError_t *err)
{
    DevBuf &b = ctx->ws[name];
    if (b.bytes >= bytes && b.p) return b.p;
    if (b.p) {
        hipStreamSynchronize(ctx->stream);
        hipFree(b.p);
        b.p = nullptr;
        b.bytes = 0;
    }
    void *p = nullptr;
    *err = hipMalloc(&p, std::max<size_t>(bytes, 256));
    if (*err != hipSuccess) return nullptr;
    b.p = p;
    b.bytes = std::max<size_t>(bytes, 256);
    return p;
}

size_t prec_bytes(dd_prec p) { return p == DD_F64 ? 8 : (p == DD_F32 ? 4 : 2); }

// The site kernels' tiles for n_rhs rhs in groups of g: every chunk of every
// block once per rhs group.
TileTable tiles_for(const dd_blocks *B, int nr, int g)
{
    TileTable tt;
    tt.ntiles = B->blk_chunk0[B->nb] * (nr / g);
    return tt;
}

// Tiles of the hop's x0-walk: (nr / g) * nseg per block, ordered block,
// segment, rhs group.  nseg is clamped to the smallest number of chunks of a
// block, so that every segment owns a chunk slot of the dot-product partials.
TileTable walk_for(const dd_blocks *B, int nr, int g, int nseg, int *nseg_used)
{
    int cap = 1 << 20;
    for (int b = 0; b < B->nb; b++) cap = std::min(cap, B->blk_chunk0[b + 1] - B->blk_chunk0[b]);
    nseg = std::max(1, std::min(nseg, cap));
    *nseg_used = nseg;
    TileTable tt;
    tt.ntiles = B->nb * (nr / g) * nseg;
    return tt;
}

// Segments per block of the hop's x0-walk: one, unless the (block, rhs group)
// walks alone would leave the device short of workgroups.
int walk_segments(const dd_ctx *ctx, const dd_blocks *B, int nr)
{
    if (ctx->hop_walk > 0) return ctx->hop_walk;
    const int64_t walks = (int64_t)B->nb * nr;
    const int64_t want = 1024;  // measured: 1536 walks of 8^4 blocks are faster whole than halved
    return (int)std::min<int64_t>(8, std::max<int64_t>(1, (want + walks - 1) / walks));
}

// Right-hand sides per thread for a spinor precision and link precision lk.
// A context override (dd_tune_set) takes precedence when it divides n_rhs.
// Default: two for FP32 spinors with FP32 links (the x0-walk hop then shares
// each link load and rebuilt row between them: measured faster), else one
// (BF16 links and FP64: measured fastest; more rhs per thread cost occupancy).
int rhs_group(const dd_ctx *ctx, int nr, dd_prec sp, dd_prec lk)
{
    const int forced = ctx ? ctx->rhs_group[sp == DD_F64 ? 0 : 1] : 0;
    if (forced > 0 && nr % forced == 0) return forced;
    const int want = sp == DD_F32 && lk == DD_F32 ? 2 : 1;
    for (int g = want; g > 1; g >>= 1)
        if (nr % g == 0) return g;
    return 1;
}

// rhs per thread of the hop kernel: its LDS stage holds 256 sites x G spinors,
// so G is at most 2 for FP32 spinors and 1 for FP64.
int hop_group(const dd_ctx *ctx, int nr, dd_prec sp, dd_prec lk)
{
    const int g = rhs_group(ctx, nr, sp, lk);
    const int cap = sp == DD_F64 ? 1 : 2;
    return g > cap ? cap : g;
}

BlkArgs blk_args(const dd_blocks *B, const TileTable &tt, int nr, int g)
{
    BlkArgs a;
    a.chunk = B->d_chunk;
    a.chunk_block = B->d_chunk_block;
    a.blk_chunk0 = B->d_blk_chunk0;
    a.h = B->d_h;
    a.soff = B->d_soff;
    a.nbr_off = B->d_nbr_off;
    a.nbr = B->d_nbr;
    a.ntiles = tt.ntiles;
    a.n_rhs = nr;
    a.nb = B->nb;
    a.g = g;
    return a;
}

const void *links_for(const dd_gauge *G, dd_prec prec)
{
    if (prec == DD_F64) return G->d_u64;
    if (prec == DD_F32) return G->low == DD_F32 ? (const void *)G->d_u32 : nullptr;
    if (prec == DD_BF16) return G->low == DD_BF16 ? (const void *)G->d_ubf : nullptr;
    return nullptr;
}

// Algorithmic bytes of one hop launch: the half field it reads and the one it
// writes (24 reals per site and rhs each), each extra half-field operand (in
// units of such a field), and every link inside the blocks once (a full SU(3)
// matrix, 18 reals, although only two rows are stored).
double hop_bytes(const dd_blocks *B, int nr, dd_prec prec, double extra_vectors)
{
    const double sf = prec == DD_F64 ? 8.0 : 4.0;
    const double sl = (double)prec_bytes(prec);
    const double half_sites = (double)B->soff[B->nb] / 2.0;
    return nr * half_sites * 24.0 * sf * (2 + extra_vectors) + (double)B->inner_links * kLinkAlgReals * sl;
}

// The aux operand of the fused dots in spinor-field units: the BiCGStab
// shadow residual (mode kDotAuxOut) is BF16 with FP32 spinors, half a field.
static double aux_vectors(const HopArgs &ha, dd_prec prec)
{
    if (!ha.aux) return 0.0;
    if (ha.dot_mode == kDotAuxOut) return prec == DD_F64 ? 1.0 : 0.5;
    return ha.dot_mode == kDotOutAuxOutOut ? 1.0 : 0.0;
}

static bool walk_applies(const dd_ctx *ctx, const dd_blocks *B, const BlkArgs &ba, dd_prec prec)
{
    return ctx->hop_lds && (ba.g == 1 || (ba.g == 2 && prec != DD_F64)) && B->walk && ctx->hop_walk >= 0;
}

int hop_walk_segments(dd_ctx *ctx, const dd_blocks *B, const BlkArgs &ba, dd_prec prec)
{
    if (!walk_applies(ctx, B, ba, prec)) return 0;
    int nseg = 1;
    walk_for(B, ba.n_rhs, ba.g, walk_segments(ctx, B, ba.n_rhs / ba.g), &nseg);
    return nseg;
}

hipError_t run_hop(dd_ctx *ctx, const dd_blocks *B, const BlkArgs &ba, const HopArgs &ha_in, dd_prec prec)
{
    HopArgs ha = ha_in;
    ha.use_lds = ctx->hop_lds ? 1 : 0;
    // operands the kernel reads besides `in` (aux only in the dot modes that use
    // it); the staging updates read r, v (and p) and write the updated input
    const double extra = (ha.self != nullptr) + (ha.add != nullptr) + aux_vectors(ha, prec) +
                         (ha.pre == kPreP ? 3 : (ha.pre == kPreS ? 2 : 0));
    const double bytes = hop_bytes(B, ba.n_rhs, prec, extra);
    const bool walk = walk_applies(ctx, B, ba, prec);
    // the x0-walk skips rhs groups whose pairs all stopped (skip_act); with
    // timing on it then counts the bytes of the tiles it does, as run_dhat
    if (!walk) ha.skip_act = nullptr;
    const bool dev_count = walk && ha.skip_act && ctx->timing && ctx->d_timer_bytes;
    if (dev_count) {
        ha.bytes_acc = ctx->d_timer_bytes + DD_KCLASS_HOP_F64 + (int)prec;
        ha.bytes_site = bytes / ((double)ba.n_rhs * (double)(B->soff[B->nb] / 2));
    }
    TimedLaunch tl(ctx, DD_KCLASS_HOP_F64 + (int)prec, dev_count ? 0.0 : bytes);
    if (walk) {
        int nseg = 1;
        const TileTable wt = walk_for(B, ba.n_rhs, ba.g, walk_segments(ctx, B, ba.n_rhs / ba.g), &nseg);
        WalkArgs wa;
        wa.ext = B->d_ext;
        wa.ntiles = wt.ntiles;
        wa.nseg = nseg;
        wa.per = nseg * (ba.n_rhs / ba.g);
        if (ha.b_hi > ha.b_lo) {  // tiles are block-major: the range's tiles are contiguous
            if (ha.b_lo < 0 || ha.b_hi > B->nb) return hipErrorInvalidValue;
            wa.tile0 = ha.b_lo * wa.per;
            wa.ntiles = (ha.b_hi - ha.b_lo) * wa.per;
        }
        return launch_hop_walk(ba, wa, ha, prec, ctx->stream);
    }
    return launch_hop(ba, ha, prec, ctx->stream);
}

// D_Lambda as one walk over both parities (FP32 spinors; every block admits
// the x0-walk; DD_TUNE_HOP_WALK automatic): otherwise two hop launches
bool dlam_walk_applies(const dd_ctx *ctx, const dd_blocks *B, dd_prec prec)
{
    return (prec == DD_F32 || prec == DD_BF16) && B->walk && ctx->hop_lds && ctx->hop_walk == 0;
}

// Algorithmic bytes of D_Lambda on all blocks: the input and the output (24
// reals per site and rhs each) and every link once (18 reals).
double dlam_bytes(const dd_blocks *B, int nr, dd_prec prec)
{
    const double sf = prec == DD_F64 ? 8.0 : 4.0;
    return nr * (double)B->soff[B->nb] * 48.0 * sf + (double)B->inner_links * kLinkAlgReals * (double)prec_bytes(prec);
}

int dhat_rhs_per_wg(const dd_ctx *ctx, const dd_blocks *B, int n_rhs)
{
    // three rhs per workgroup cut the link re-reads but hide memory latency
    // worse (three walks behind shared barriers); one is the faster default
    (void)B;
    (void)n_rhs;
    return ctx->dhat_rhs == 3 ? 3 : 1;
}

bool dhat_walk_applies(const dd_ctx *ctx, const dd_blocks *B, const BlkArgs &ba, dd_prec prec)
{
    if (!ctx->hop_lds || !B->walk || ctx->hop_walk < 0 || ctx->dhat_walk < 0) return false;
    if (prec != DD_F32 && prec != DD_BF16) return false;
    return walk_segments(ctx, B, ba.n_rhs) == 1;
}

hipError_t run_dhat(dd_ctx *ctx, const dd_blocks *B, const BlkArgs &ba, const HopArgs &ha_in, dd_prec prec)
{
    HopArgs ha = ha_in;
    ha.use_lds = 1;
    // algorithmic operands besides `in` and `out`: the self term when it is
    // not `in` itself, aux in the dot modes that use it, and the staging
    // update's r, v (and p) reads and its write of the updated input
    const double extra = (ha.self != nullptr && ha.self != ha.in) + (ha.add != nullptr) + aux_vectors(ha, prec) +
                         (ha.pre == kPreP ? 3 : (ha.pre == kPreS ? 2 : 0));
    const int kc = prec == DD_F32 ? DD_KCLASS_DHAT_F32 : DD_KCLASS_DHAT_BF16;
    const double bytes = hop_bytes(B, ba.n_rhs, prec, extra);
    // with timing on the kernel counts the bytes of the walks it does (pairs
    // that stopped are skipped): the launch's bytes per eo site and rhs
    const bool dev_count = ctx->timing && ctx->d_timer_bytes;
    if (dev_count) {
        ha.bytes_acc = ctx->d_timer_bytes + kc;
        ha.bytes_site = bytes / ((double)ba.n_rhs * (double)(B->soff[B->nb] / 2));
    }
    TimedLaunch tl(ctx, kc, dev_count ? 0.0 : bytes);
    // rhs per workgroup: three (walked in lockstep, sharing the block's link
    // loads) when n_rhs is a multiple of three and that still gives a few
    // workgroups per compute unit, else one
    const int nrw = ha.clover ? 1 : dhat_rhs_per_wg(ctx, B, ba.n_rhs);
    WalkArgs wa;
    wa.ext = B->d_ext;
    wa.nseg = nrw;  // the Dhat walk is never segmented: nseg holds the rhs per workgroup
    wa.per = (ba.n_rhs + nrw - 1) / nrw;
    wa.ntiles = B->nb * wa.per;
    return launch_dhat_walk(ba, wa, ha, prec, ctx->stream);
}

bool rhs_fit(const dd_blocks *B, int n_rhs)
{
    return (int64_t)n_rhs * B->max_h * 24 * 8 < ((int64_t)1 << 32);
}

const void *clover_for(const dd_gauge *G, dd_prec prec, bool inverse)
{
    if (G->cl_csw == 0.0) return nullptr;
    if (prec == DD_F64) return inverse ? (const void *)G->d_cli64 : (const void *)G->d_cla64;
    return inverse ? (const void *)G->d_cli32 : (const void *)G->d_cla32;
}

dd_status clover_check(dd_ctx *ctx, const dd_gauge *G, double kappa)
{
    if (G->cl_csw != 0.0 && !(std::fabs(kappa - G->cl_kappa) <= 1e-12 * std::fabs(G->cl_kappa)))
        return fail(ctx, DD_EINVAL, "the gauge's clover term was built for another kappa");
    return DD_OK;
}

dd_status apply_D_check(dd_ctx *ctx, const dd_blocks *B, const dd_gauge *G, dd_prec prec, double kappa,
                        const void *x_dev, void *y_dev, int32_t n_rhs, const void **links, const void **clover)
{
    if (!ctx || !B || !G || !x_dev || !y_dev) return fail(ctx, DD_EINVAL, "null argument");
    if (n_rhs < 1 || n_rhs > kMaxRhs) return fail(ctx, DD_EINVAL, "n_rhs must be in 1..64");
    if (G->blocks != B) return fail(ctx, DD_EINVAL, "gauge was loaded for other blocks");
    if (!rhs_fit(B, n_rhs))
        return fail(ctx, DD_EUNSUPPORTED, "too many rhs for the block size (32-bit offsets of the half fields)");
    *links = links_for(G, prec);
    if (!*links) return fail(ctx, DD_EINVAL, "gauge holds no links of the requested precision");
    const dd_status st = clover_check(ctx, G, kappa);
    if (st != DD_OK) return st;
    *clover = clover_for(G, prec, false);
    return DD_OK;
}

size_t apply_D_half_bytes(const dd_blocks *B, int n_rhs, dd_prec prec)
{
    const dd_prec sp = prec == DD_F64 ? DD_F64 : DD_F32;
    return (size_t)(B->soff[B->nb] / 2) * 24 * n_rhs * prec_bytes(sp);
}

dd_status apply_D_with(dd_ctx *ctx, const dd_blocks *Bc, const void *links, const void *clover, double kappa,
                       dd_prec prec, const void *x_dev, void *y_dev, int32_t n_rhs, void *const hf[4])
{
    const dd_prec sp = prec == DD_F64 ? DD_F64 : DD_F32;
    const int g = hop_group(ctx, n_rhs, sp, prec);
    const BlkArgs ba = blk_args(Bc, tiles_for(Bc, n_rhs, g), n_rhs, g);
    void *xe = hf[0], *xo = hf[1], *ye = hf[2], *yo = hf[3];
    HIPCHECK(ctx, launch_pack_spinor(Bc, (const double *)x_dev, xe, xo, sp, n_rhs, ctx->stream));
    if (clover) {
        // y_p = A_pp x_p, then y_p += -kappa H x_{1-p} in place (the hop reads
        // a site's self term before it writes the site)
        for (int p = 0; p < 2; p++)
            HIPCHECK(ctx, launch_clover_apply(Bc, clover, p ? xo : xe, p ? yo : ye, p, n_rhs, sp, nullptr, ctx->stream));
        for (int p = 0; p < 2; p++) {
            HopArgs ha = hop_args(p ? yo : ye, p ? xe : xo, links, p, -kappa);
            ha.self = p ? yo : ye;
            ha.c_self = 1.0;
            HIPCHECK(ctx, run_hop(ctx, Bc, ba, ha, prec));
        }
    } else if (dlam_walk_applies(ctx, Bc, prec)) {
        // one x0-walk per (block, rhs) over both parities; algorithmic bytes
        // as for D_Lambda: x once, y once, the links once
        DlamArgs da;
        da.ext = Bc->d_ext;
        da.ntiles = Bc->nb * n_rhs;
        da.xe = xe;
        da.xo = xo;
        da.ye = ye;
        da.yo = yo;
        da.links = links;
        da.c_hop = -kappa;
        const double bytes = dlam_bytes(Bc, n_rhs, prec);
        const bool dev = ctx->timing && ctx->d_timer_bytes;
        da.bytes_acc = dev ? ctx->d_timer_bytes + DD_KCLASS_HOP_F64 + (int)prec : nullptr;
        da.bytes_walk = bytes / da.ntiles;
        TimedLaunch tl(ctx, DD_KCLASS_HOP_F64 + (int)prec, dev ? 0.0 : bytes);
        HIPCHECK(ctx, launch_dlam_walk(blk_args(Bc, tiles_for(Bc, n_rhs, 1), n_rhs, 1), da, prec, ctx->stream));
    } else {
        for (int p = 0; p < 2; p++) {
            HopArgs ha = hop_args(p ? yo : ye, p ? xe : xo, links, p, -kappa);
            ha.self = p ? xo : xe;
            ha.c_self = 1.0;
            HIPCHECK(ctx, run_hop(ctx, Bc, ba, ha, prec));
        }
    }
    HIPCHECK(ctx, launch_unpack_spinor(Bc, ye, yo, (double *)y_dev, sp, n_rhs, ctx->stream));
    HIPCHECK(ctx, hipStreamSynchronize(ctx->stream));
    return DD_OK;
}

HopArgs hop_args(void *out, const void *in, const void *links, int parity, double c_hop)
{
    HopArgs h;
    std::memset(&h, 0, sizeof(h));
    h.out = out;
    h.in = in;
    h.links = links;
    h.parity = parity;
    h.c_hop = c_hop;
    h.dot_mode = kDotNone;
    return h;
}

}  // namespace dd

// ======================================================================== ABI

extern "C" {

const char *dd_version(void) { return kVersion; }

dd_status dd_create(int device, void *hip_stream, dd_ctx **out)
{
    if (!out) return DD_EINVAL;
    *out = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) return DD_EDEVICE;
    if (hipSetDevice(device) != hipSuccess) return DD_EDEVICE;
    dd_ctx *ctx = new (std::nothrow) dd_ctx();
    if (!ctx) return DD_ENOMEM;
    ctx->device = device;
    // All library work runs on a stream of its own (capturable into graphs);
    // each call first waits for the caller's stream and synchronises before it returns.
    if (hipStreamCreateWithFlags(&ctx->stream, hipStreamNonBlocking) != hipSuccess) {
        delete ctx;
        return DD_EDEVICE;
    }
    ctx->user_stream = (hipStream_t)hip_stream;
    // the event each call records on the caller's stream
    if (hipEventCreateWithFlags(&ctx->enter_ev, hipEventDisableTiming) != hipSuccess) {
        if (ctx->enter_ev) hipEventDestroy(ctx->enter_ev);
        hipStreamDestroy(ctx->stream);
        delete ctx;
        return DD_EDEVICE;
    }
    *out = ctx;
    return DD_OK;
}

dd_status dd_destroy(dd_ctx *ctx)
{
    if (!ctx) return DD_EINVAL;
    hipSetDevice(ctx->device);
    hipStreamSynchronize(ctx->stream);
    for (auto &kv : ctx->ws)
        if (kv.second.p) hipFree(kv.second.p);
    for (auto &t : ctx->timers)
        for (auto &e : t.ev) {
            hipEventDestroy(e.first);
            hipEventDestroy(e.second);
        }
    logdet_release(ctx);
    if (ctx->enter_ev) hipEventDestroy(ctx->enter_ev);
    hipStreamDestroy(ctx->stream);
    delete ctx;
    return DD_OK;
}

const char *dd_last_error(const dd_ctx *ctx) { return ctx ? ctx->err.c_str() : g_err.c_str(); }

}  // extern "C"

namespace dd {

// make the library stream wait for work the caller queued on its own stream
hipError_t enter(dd_ctx *ctx)
{
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) return e;
    (void)hipGetLastError();  // drop a stale error left by unrelated runtime calls
    if ((e = hipEventRecord(ctx->enter_ev, ctx->user_stream)) != hipSuccess) return e;
    return hipStreamWaitEvent(ctx->stream, ctx->enter_ev, 0);
}

dd_status finish_blocks(dd_ctx *ctx, dd_blocks *B, dd_blocks **out)
{
    hipError_t e = hipSuccess;
    std::vector<int32_t> h(B->nb), nl(B->nb), org((size_t)B->nb * 4), ext((size_t)B->nb * 4);
    std::vector<int64_t> nbo(B->nb), pmo(B->nb);
    for (int b = 0; b < B->nb; b++) {
        const Shape &sh = B->shapes[B->shape_of[b]];
        h[b] = sh.h;
        nl[b] = (int32_t)sh.links;
        nbo[b] = sh.nbr_off;
        pmo[b] = sh.perm_off;
        for (int m = 0; m < 4; m++) {
            org[4 * b + m] = B->box[16 * b + m];
            ext[4 * b + m] = B->box[16 * b + 4 + m];
        }
    }
    // chunks of the site kernels: whole x0-slices up to kTile sites per parity
    std::vector<int32_t> chunk(B->nb), chunk_block;
    B->blk_chunk0.assign(B->nb + 1, 0);
    for (int b = 0; b < B->nb; b++) {
        const Shape &sh = B->shapes[B->shape_of[b]];
        const int hs = sh.e[1] * sh.e[2] * sh.e[3] / 2;  // sites per parity of an x0-slice
        int T = hs <= kTile ? hs * (kTile / hs) : kTile;
        T = std::min(T, sh.h);
        chunk[b] = T;
        const int nc = (sh.h + T - 1) / T;
        B->blk_chunk0[b + 1] = B->blk_chunk0[b] + nc;
        for (int c = 0; c < nc; c++) chunk_block.push_back(b);
    }
    B->iperm.assign(B->perm.size(), 0);
    for (const Shape &sh : B->shapes)
        for (int k = 0; k < sh.S; k++) B->iperm[sh.perm_off + B->perm[sh.perm_off + k]] = k;
    if ((e = upload(&B->d_nbr, B->nbr)) != hipSuccess || (e = upload(&B->d_perm, B->perm)) != hipSuccess ||
        (e = upload(&B->d_iperm, B->iperm)) != hipSuccess ||
        (e = upload(&B->d_soff, B->soff)) != hipSuccess || (e = upload(&B->d_h, h)) != hipSuccess ||
        (e = upload(&B->d_nlinks, nl)) != hipSuccess ||
        (e = upload(&B->d_nbr_off, nbo)) != hipSuccess || (e = upload(&B->d_perm_off, pmo)) != hipSuccess ||
        (e = upload(&B->d_origin, org)) != hipSuccess || (e = upload(&B->d_ext, ext)) != hipSuccess ||
        (e = upload(&B->d_bnd, B->bnd)) != hipSuccess || (e = upload(&B->d_boff, B->boff)) != hipSuccess ||
        (e = upload(&B->d_chunk, chunk)) != hipSuccess || (e = upload(&B->d_chunk_block, chunk_block)) != hipSuccess ||
        (e = upload(&B->d_blk_chunk0, B->blk_chunk0)) != hipSuccess ||
        (!B->x_code.empty() &&
         ((e = upload(&B->d_xg_block, B->xg_block)) != hipSuccess || (e = upload(&B->d_xg_site, B->xg_site)) != hipSuccess ||
          (e = upload(&B->d_xg_first, B->xg_first)) != hipSuccess || (e = upload(&B->d_x_code, B->x_code)) != hipSuccess ||
          (e = upload(&B->d_x_nbr, B->x_nbr)) != hipSuccess || (e = upload(&B->d_x_link, B->x_link)) != hipSuccess)) ||
        (!B->dpi1.empty() && (e = upload(&B->d_dpi1, B->dpi1)) != hipSuccess)) {
        dd_free_blocks(B);
        return fail(ctx, DD_EDEVICE, std::string("geometry upload: ") + hipGetErrorString(e));
    }
    *out = B;
    return DD_OK;
}

dd_status make_from_boxes(dd_ctx *ctx, const int32_t L[4], int32_t time_bc, int n, const int32_t *boxes,
                          const int32_t *inner, dd_blocks **out, bool frames = false)
{
    if (!L || !out || (n > 0 && !boxes)) return fail(ctx, DD_EINVAL, "null argument");
    *out = nullptr;
    if (ctx && enter(ctx) != hipSuccess) return fail(ctx, DD_EDEVICE, "hipSetDevice failed");
    dd_blocks *B = new (std::nothrow) dd_blocks();
    if (!B) return fail(ctx, DD_ENOMEM, "out of host memory");
    B->ctx = ctx;
    B->device = ctx ? ctx->device : -1;
    int Li[4] = {L[0], L[1], L[2], L[3]};
    const std::string msg = build_geometry(B, Li, time_bc, n, boxes, inner, frames);
    if (!msg.empty()) {
        delete B;
        return fail(ctx, DD_EINVAL, msg);
    }
    if (!ctx) {  // host tables only: usable for queries, not for device work
        *out = B;
        return DD_OK;
    }
    return finish_blocks(ctx, B, out);
}

}  // namespace dd

extern "C" {

dd_status dd_make_blocks(dd_ctx *ctx, const int32_t L[4], int32_t time_bc, const int32_t *seg, const int32_t nseg[4],
                         const int32_t shift[4], int32_t inner_d, dd_blocks **out)
{
    if (!L || !seg || !nseg || !out) return fail(ctx, DD_EINVAL, "null argument");
    std::vector<std::vector<int32_t>> starts(4), exts(4);
    size_t pos = 0;
    for (int m = 0; m < 4; m++) {
        if (nseg[m] < 1) return fail(ctx, DD_EINVAL, "each direction needs at least one tile");
        int64_t sum = 0;
        for (int k = 0; k < nseg[m]; k++) {
            const int32_t v = seg[pos++];
            if (v < 1) return fail(ctx, DD_EINVAL, "tile extents must be positive");
            const int32_t sh = shift ? shift[m] : 0;
            starts[m].push_back((int32_t)((((sum + sh) % L[m]) + L[m]) % L[m]));
            exts[m].push_back(v);
            sum += v;
        }
        if (sum != L[m]) return fail(ctx, DD_EINVAL, "tile extents must sum to the lattice extent");
    }
    if (inner_d < 0) return fail(ctx, DD_EINVAL, "inner_d must be >= 0");
    std::vector<int32_t> boxes, inner;
    for (int a = 0; a < nseg[0]; a++)
        for (int b = 0; b < nseg[1]; b++)
            for (int c = 0; c < nseg[2]; c++)
                for (int d = 0; d < nseg[3]; d++) {
                    const int t[4] = {a, b, c, d};
                    for (int m = 0; m < 4; m++) boxes.push_back(starts[m][t[m]]);
                    for (int m = 0; m < 4; m++) boxes.push_back(exts[m][t[m]]);
                    for (int m = 0; m < 4; m++) inner.push_back(exts[m][t[m]] == L[m] ? 0 : inner_d);
                    for (int m = 0; m < 4; m++) {
                        const int e = exts[m][t[m]];
                        inner.push_back(e == L[m] ? e : e - 2 * inner_d);
                    }
                }
    const int n = (int)(boxes.size() / 8);
    return make_from_boxes(ctx, L, time_bc, n, boxes.data(), inner.data(), out);
}

dd_status dd_make_blocks_paper(dd_ctx *ctx, const int32_t L[4], int32_t time_bc, const int32_t bd[8],
                               dd_blocks **out)
{
    if (!L || !bd || !out) return fail(ctx, DD_EINVAL, "null argument");
    std::vector<std::vector<int32_t>> st(4);
    for (int m = 0; m < 4; m++) {
        const int b = bd[2 * m], d = bd[2 * m + 1];
        if (b == 0) {
            st[m].push_back(0);
            continue;
        }
        if (b < 1 || d < 1 || L[m] % (b + d) != 0) return fail(ctx, DD_EINVAL, "need b >= 1, d >= 1, (b+d) | L");
        for (int s = 0; s < L[m]; s += b + d) st[m].push_back(s);
    }
    std::vector<int32_t> boxes, inner;
    for (int32_t s0 : st[0])
        for (int32_t s1 : st[1])
            for (int32_t s2 : st[2])
                for (int32_t s3 : st[3]) {
                    const int32_t s[4] = {s0, s1, s2, s3};
                    int32_t o[4], e[4], io[4], ie[4];
                    for (int m = 0; m < 4; m++) {
                        const int b = bd[2 * m], d = bd[2 * m + 1];
                        if (b == 0) {
                            o[m] = 0; e[m] = L[m]; io[m] = 0; ie[m] = L[m];
                        } else {
                            o[m] = ((s[m] - d) % L[m] + L[m]) % L[m];
                            e[m] = b + 2 * d;
                            io[m] = d;
                            ie[m] = b;
                        }
                    }
                    boxes.insert(boxes.end(), o, o + 4);
                    boxes.insert(boxes.end(), e, e + 4);
                    inner.insert(inner.end(), io, io + 4);
                    inner.insert(inner.end(), ie, ie + 4);
                }
    return make_from_boxes(ctx, L, time_bc, (int)(boxes.size() / 8), boxes.data(), inner.data(), out);
}

dd_status dd_make_blocks_boxes(dd_ctx *ctx, const int32_t L[4], int32_t time_bc, int32_t n, const int32_t *boxes,
                               const int32_t *inner, dd_blocks **out)
{
    return make_from_boxes(ctx, L, time_bc, n, boxes, inner, out);
}

dd_status dd_make_frames(dd_ctx *ctx, const dd_blocks *blocks, dd_blocks **out)
{
    if (!blocks || !out) return fail(ctx, DD_EINVAL, "null argument");
    std::vector<int32_t> boxes, inner;
    for (int k = 0; k < blocks->nb; k++) {
        const int32_t *r = &blocks->box[16 * k];
        boxes.insert(boxes.end(), r, r + 8);
        inner.insert(inner.end(), r + 8, r + 16);
    }
    return make_from_boxes(ctx, blocks->L, blocks->tbc, blocks->nb, boxes.data(), inner.data(), out, true);
}

dd_status dd_make_inactive(dd_ctx *ctx, const dd_blocks *blocks, dd_blocks **out)
{
    if (!blocks || !out) return fail(ctx, DD_EINVAL, "null argument");
    *out = nullptr;
    if (ctx && enter(ctx) != hipSuccess) return fail(ctx, DD_EDEVICE, "hipSetDevice failed");
    dd_blocks *D = new (std::nothrow) dd_blocks();
    if (!D) return fail(ctx, DD_ENOMEM, "out of host memory");
    D->ctx = ctx;
    D->device = ctx ? ctx->device : -1;
    D->parent = blocks->serial;
    const std::string msg = build_inactive(D, blocks);
    if (!msg.empty()) {
        delete D;
        return fail(ctx, DD_EINVAL, msg);
    }
    if (!ctx) {  // host tables only
        *out = D;
        return DD_OK;
    }
    return finish_blocks(ctx, D, out);
}

dd_status dd_free_blocks(dd_blocks *B)
{
    if (!B) return DD_EINVAL;
    if (B->device >= 0) hipSetDevice(B->device);
    void *ptrs[] = {B->d_nbr,    B->d_perm,   B->d_iperm,  B->d_soff, B->d_h,    B->d_nlinks,
                    B->d_nbr_off, B->d_perm_off, B->d_origin, B->d_ext,  B->d_bnd,  B->d_boff,
                    B->d_chunk,  B->d_chunk_block, B->d_blk_chunk0, B->d_xg_block, B->d_xg_site,
                    B->d_xg_first, B->d_x_code, B->d_x_nbr, B->d_x_link, B->d_dpi1};
    for (void *p : ptrs)
        if (p) hipFree(p);
    for (auto &kv : B->queues) {
        if (kv.second.d_queue) hipFree(kv.second.d_queue);
        if (kv.second.d_qoff) hipFree(kv.second.d_qoff);
        if (kv.second.d_qctr) hipFree(kv.second.d_qctr);
    }
    delete B;
    return DD_OK;
}

dd_status dd_blocks_query(const dd_blocks *B, int64_t *n_blocks, int64_t *total_sites, int64_t *total_bnd_sites,
                          int64_t *inner_links)
{
    if (!B) return DD_EINVAL;
    if (n_blocks) *n_blocks = B->nb;
    if (total_sites) *total_sites = B->soff[B->nb];
    if (total_bnd_sites) *total_bnd_sites = B->boff[B->nb];
    if (inner_links) *inner_links = B->inner_links;
    return DD_OK;
}

dd_status dd_blocks_tables(const dd_blocks *B, int32_t *boxes, int64_t *sites, int32_t *eo, int32_t *bnd)
{
    if (!B) return DD_EINVAL;
    if (boxes) std::memcpy(boxes, B->box.data(), B->box.size() * sizeof(int32_t));
    for (int b = 0; b < B->nb; b++) {
        const Shape &sh = B->shapes[B->shape_of[b]];
        const int32_t *bx = &B->box[16 * b];
        const int64_t s0 = B->soff[b];
        if (sites) {
            for (int s = 0; s < sh.S; s++) {
                int y[4], r = s;
                y[3] = r % sh.e[3]; r /= sh.e[3];
                y[2] = r % sh.e[2]; r /= sh.e[2];
                y[1] = r % sh.e[1]; r /= sh.e[1];
                y[0] = r;
                int64_t n = 0;
                for (int m = 0; m < 4; m++) n = n * B->L[m] + (bx[m] + y[m]) % B->L[m];
                sites[s0 + s] = n;
            }
        }
        if (eo)
            for (int k = 0; k < sh.S; k++) eo[s0 + B->perm[sh.perm_off + k]] = k;
    }
    if (bnd) std::memcpy(bnd, B->bnd.data(), B->bnd.size() * sizeof(int32_t));
    return DD_OK;
}

dd_status dd_blocks_dpi1(const dd_blocks *B, int64_t *n_sites, int64_t *sites)
{
    if (!B || !n_sites) return DD_EINVAL;
    if (!B->inactive) return fail(nullptr, DD_EINVAL, "not an inactive-region domain (dd_make_inactive)");
    *n_sites = (int64_t)B->dpi1.size();
    if (sites) std::memcpy(sites, B->dpi1.data(), B->dpi1.size() * sizeof(int64_t));
    return DD_OK;
}

dd_status dd_blocks_exterior(const dd_blocks *B, int64_t *n_hops, int32_t *block, int32_t *site, int32_t *code,
                             int64_t *nbr)
{
    if (!B) return DD_EINVAL;
    if (n_hops) *n_hops = (int64_t)B->x_code.size();
    for (size_t g = 0; g < B->xg_block.size(); g++)
        for (int32_t e = B->xg_first[g]; e < B->xg_first[g + 1]; e++) {
            if (block) block[e] = B->xg_block[g];
            if (site) site[e] = B->xg_site[g];
        }
    if (code && !B->x_code.empty()) std::memcpy(code, B->x_code.data(), B->x_code.size() * sizeof(int32_t));
    if (nbr && !B->x_nbr.empty()) std::memcpy(nbr, B->x_nbr.data(), B->x_nbr.size() * sizeof(int64_t));
    return DD_OK;
}

// ------------------------------------------------------------------ gauge

dd_status dd_load_gauge(dd_ctx *ctx, const dd_blocks *B, const void *U_dev, dd_prec low_prec, dd_gauge **out)
{
    if (!ctx || !B || !U_dev || !out) return fail(ctx, DD_EINVAL, "null argument");
    if (B->ctx != ctx) return fail(ctx, DD_EINVAL, "blocks belong to another context (or have no device tables)");
    if (low_prec != DD_F64 && low_prec != DD_F32 && low_prec != DD_BF16) return fail(ctx, DD_EINVAL, "bad precision");
    *out = nullptr;
    HIPCHECK(ctx, enter(ctx));
    dd_gauge *G = new (std::nothrow) dd_gauge();
    if (!G) return fail(ctx, DD_ENOMEM, "out of host memory");
    G->ctx = ctx;
    G->device = ctx->device;
    G->blocks = B;
    G->low = low_prec;
    const size_t nl = (size_t)B->soff[B->nb] * kLinkReals;
    hipError_t e = hipMalloc((void **)&G->d_u64, std::max<size_t>(nl * 8, 8));
    if (e == hipSuccess) e = launch_pack_gauge(B, (const double *)U_dev, DD_F64, G->d_u64, ctx->stream);
    if (e == hipSuccess && low_prec == DD_F32) {
        e = hipMalloc((void **)&G->d_u32, std::max<size_t>(nl * 4, 4));
        if (e == hipSuccess) e = launch_pack_gauge(B, (const double *)U_dev, DD_F32, G->d_u32, ctx->stream);
    }
    if (e == hipSuccess && low_prec == DD_BF16) {
        e = hipMalloc((void **)&G->d_ubf, std::max<size_t>(nl * 2, 2));
        if (e == hipSuccess) e = launch_pack_gauge(B, (const double *)U_dev, DD_BF16, G->d_ubf, ctx->stream);
    }
    if (e == hipSuccess && !B->x_code.empty()) {
        e = hipMalloc((void **)&G->d_uext, B->x_code.size() * 18 * sizeof(double));
        if (e == hipSuccess) e = launch_gather_ext_links(B, (const double *)U_dev, G->d_uext, ctx->stream);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) {
        dd_free_gauge(G);
        return fail(ctx, e == hipErrorOutOfMemory ? DD_ENOMEM : DD_EDEVICE,
                    std::string("gauge packing: ") + hipGetErrorString(e));
    }
    *out = G;
    return DD_OK;
}

dd_status dd_free_gauge(dd_gauge *G)
{
    if (!G) return DD_EINVAL;
    hipSetDevice(G->device);
    if (G->d_u64) hipFree(G->d_u64);
    if (G->d_u32) hipFree(G->d_u32);
    if (G->d_ubf) hipFree(G->d_ubf);
    if (G->d_uext) hipFree(G->d_uext);
    clover_release(G);
    delete G;
    return DD_OK;
}

dd_status dd_gauge_export(dd_ctx *ctx, const dd_gauge *G, dd_prec prec, void *dst_dev)
{
    if (!ctx || !G || !dst_dev) return fail(ctx, DD_EINVAL, "null argument");
    const void *src = links_for(G, prec);
    if (!src) return fail(ctx, DD_EINVAL, "gauge holds no links of that precision");
    HIPCHECK(ctx, enter(ctx));
    const size_t bytes = (size_t)G->blocks->soff[G->blocks->nb] * kLinkReals * prec_bytes(prec);
    HIPCHECK(ctx, hipMemcpyAsync(dst_dev, src, bytes, hipMemcpyDeviceToDevice, ctx->stream));
    HIPCHECK(ctx, hipStreamSynchronize(ctx->stream));
    return DD_OK;
}

// --------------------------------------------------------------- operator

dd_status dd_apply_D_block(dd_ctx *ctx, const dd_blocks *Bc, const dd_gauge *G, double kappa, dd_prec prec,
                           const void *x_dev, void *y_dev, int32_t n_rhs)
{
    const void *links = nullptr, *clover = nullptr;
    const dd_status st = apply_D_check(ctx, Bc, G, prec, kappa, x_dev, y_dev, n_rhs, &links, &clover);
    if (st != DD_OK) return st;
    HIPCHECK(ctx, enter(ctx));
    hipError_t e;
    const size_t half = apply_D_half_bytes(Bc, n_rhs, prec);
    void *hf[4];
    const char *names[4] = {"ap_xe", "ap_xo", "ap_ye", "ap_yo"};
    for (int k = 0; k < 4; k++)
        if (!(hf[k] = workspace(ctx, names[k], half, &e)))
            return fail(ctx, DD_ENOMEM, std::string("workspace: ") + hipGetErrorString(e));
    return apply_D_with(ctx, Bc, links, clover, kappa, prec, x_dev, y_dev, n_rhs, hf);
}

// ------------------------------------------------------------------ timing

dd_status dd_tune_set(dd_ctx *ctx, int32_t what, int32_t value)
{
    if (!ctx) return DD_EINVAL;
    if (what == DD_TUNE_HOP_LDS) {
        ctx->hop_lds = value != 0;
        return DD_OK;
    }
    if (what == DD_TUNE_HOP_WALK) {
        if (value < -1 || value > 64) return fail(ctx, DD_EINVAL, "hop walk must be -1 (off), 0 (automatic) or 1..64 segments");
        ctx->hop_walk = value;
        return DD_OK;
    }
    if (what == DD_TUNE_DHAT_WALK) {
        if (value != 0 && value != -1) return fail(ctx, DD_EINVAL, "Dhat walk must be 0 (where possible) or -1 (never)");
        ctx->dhat_walk = value;
        return DD_OK;
    }
    if (what == DD_TUNE_DHAT_RHS) {
        if (value != 0 && value != 1 && value != 3) return fail(ctx, DD_EINVAL, "Dhat rhs per workgroup must be 0, 1 or 3");
        ctx->dhat_rhs = value;
        return DD_OK;
    }
    if (what == DD_TUNE_BICG_FUSE) {
        if (value != 0 && value != -1) return fail(ctx, DD_EINVAL, "BiCGStab fusion must be 0 (where possible) or -1 (never)");
        ctx->bicg_fuse = value;
        return DD_OK;
    }
    if (what == DD_TUNE_GMRES_REORTH) {
        if (value < -1 || value > 100) return fail(ctx, DD_EINVAL, "reorthogonalization threshold must be -1, 0 or 1..100");
        ctx->gm_reorth = value;
        return DD_OK;
    }
    if (what == DD_TUNE_GMRES_THREADS) {
        if (value != 0 && value != 256 && value != 512)
            return fail(ctx, DD_EINVAL, "GMRES threads per workgroup must be 0, 256 or 512");
        ctx->gm_threads = value;
        return DD_OK;
    }
    if (what == DD_TUNE_GMRES_QUEUES) {
        if (value != 0 && value != 1 && value != 8) return fail(ctx, DD_EINVAL, "GMRES queues must be 0, 1 or 8");
        ctx->gm_queues = value;
        return DD_OK;
    }
    if (what == DD_TUNE_NN_KERNEL) {
        if (value != 0 && value != 1) return fail(ctx, DD_EINVAL, "network kernel must be 0 or 1");
        ctx->nn_kernel = value;
        return DD_OK;
    }
    if (what == DD_TUNE_MB_FIELDS) {
        if (value < 0 || value > kMaxRhs) return fail(ctx, DD_EINVAL, "fields per solve must be in 0..64");
        ctx->mb_fields = value;
        return DD_OK;
    }
    if (what == DD_TUNE_GMRES_WG_PER_CU) {
        if (value < 0 || value > 64) return fail(ctx, DD_EINVAL, "GMRES workgroups per CU must be in 0..64");
        ctx->gm_wg_per_cu = value;
        return DD_OK;
    }
    if (what != DD_TUNE_RHS_GROUP_F64 && what != DD_TUNE_RHS_GROUP_F32)
        return fail(ctx, DD_EINVAL, "unknown tuning knob");
    if (value != 0 && value != 1 && value != 2 && value != 4)
        return fail(ctx, DD_EINVAL, "rhs group must be 0 (automatic), 1, 2 or 4");
    ctx->rhs_group[what] = value;
    return DD_OK;
}

dd_status dd_timer_enable(dd_ctx *ctx, int32_t on)
{
    if (!ctx) return DD_EINVAL;
    if (on && !ctx->d_timer_bytes) {
        hipError_t e;
        const size_t nb = DD_KCLASS_COUNT * sizeof(double);
        double *p = (double *)workspace(ctx, "timer_bytes", nb, &e);
        if (!p) return fail(ctx, DD_ENOMEM, std::string("timer counters: ") + hipGetErrorString(e));
        HIPCHECK(ctx, hipMemsetAsync(p, 0, nb, ctx->stream));
        ctx->d_timer_bytes = p;
    }
    ctx->timing = on != 0;
    return DD_OK;
}

dd_status dd_timer_reset(dd_ctx *ctx)
{
    if (!ctx) return DD_EINVAL;
    if (ctx->d_timer_bytes) hipMemsetAsync(ctx->d_timer_bytes, 0, DD_KCLASS_COUNT * sizeof(double), ctx->stream);
    hipStreamSynchronize(ctx->stream);
    for (auto &t : ctx->timers) {
        t.used = 0;
        t.bytes = 0;
    }
    return DD_OK;
}

dd_status dd_timer_read(dd_ctx *ctx, int32_t kclass, double *total_ms, int64_t *launches, double *alg_bytes)
{
    if (!ctx || kclass < 0 || kclass >= DD_KCLASS_COUNT) return fail(ctx, DD_EINVAL, "bad timer class");
    HIPCHECK(ctx, hipStreamSynchronize(ctx->stream));
    Timer &t = ctx->timers[kclass];
    double tot = 0;
    for (size_t i = 0; i < t.used; i++) {
        float ms = 0;
        HIPCHECK(ctx, hipEventElapsedTime(&ms, t.ev[i].first, t.ev[i].second));
        tot += ms;
    }
    if (total_ms) *total_ms = tot;
    double dev = 0;
    if (ctx->d_timer_bytes)
        HIPCHECK(ctx, hipMemcpy(&dev, ctx->d_timer_bytes + kclass, sizeof(double), hipMemcpyDeviceToHost));
    if (launches) *launches = (int64_t)t.used;
    if (alg_bytes) *alg_bytes = t.bytes + dev;
    return DD_OK;
}

}  // extern "C"
