// Batched block solves x = D_Lambda^{-1} b for all (block, rhs) pairs and the
// block-local multi-boson action of libdd.
//
// Method (the paper needs the solves but prescribes no solver):
//   outer: FP64 defect correction on the true residual r = b - D_Lambda x,
//          computed with FP64 links and spinors, until |r| <= tol |b| per pair;
//   inner: even-odd reduced system Dhat e_e = r_e + kappa H_eo r_o with
//          Dhat = 1 - kappa^2 H_eo H_oe, solved in the inner precision (FP64,
//          FP32, or FP32 spinors with BF16 links), then
//          e_o = r_o + kappa H_oe e_e and x += e.
// Inner methods:
//   BiCGStab: every launch covers all blocks and right-hand sides; per-pair
//          scalars live on the device and pairs that converge are frozen (the
//          x0-walk operator kernels and the vector updates skip them).
//   GMRES(m): one persistent launch per defect-correction cycle; each
//          workgroup solves whole pairs taken from work queues.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "dd_host.h"
#include "dd_internal.h"
#include "dd_nn.h"

using namespace dd;

namespace {

struct Ws {
    double *be, *bo, *xe, *xo, *re, *ro;  // FP64 half fields
    void *rie, *rio;                      // residual in the inner precision
    void *rhs, *xi, *r, *rh, *p, *v, *s, *t, *tmp;
    double *pA, *pB, *pC, *pe, *po;       // dot partials
    PairState ps;
    OuterState os;
};

// A captured graph and its executable, destroyed when the holder goes out of
// scope (also on the early returns of the error paths).
struct GraphHolder {
    hipGraph_t g = nullptr;
    hipGraphExec_t gx = nullptr;
    GraphHolder() = default;
    GraphHolder(const GraphHolder &) = delete;
    GraphHolder &operator=(const GraphHolder &) = delete;
    void reset()
    {
        if (gx) hipGraphExecDestroy(gx);
        if (g) hipGraphDestroy(g);
        gx = nullptr;
        g = nullptr;
    }
    ~GraphHolder() { reset(); }
};

struct Inner {
    dd_ctx *ctx;
    const dd_blocks *B;
    BlkArgs ba;
    Ws *w;
    const void *links;
    dd_prec ip, sp;
    double kappa, tol;
    dd_nn *nn;     // right preconditioner M (linear network) or null
    void *ph, *sh;  // M p, M s
    int n_rhs;
    // vector updates done by the first hop of Dhat as it stages its input
    bool fuse_s, fuse_p;
    bool dhat;  // Dhat as one x0-walk kernel (run_dhat)
    const void *clover;  // A^-1 of the clover term (inner precision) or null
};

// one BiCGStab iteration on all pairs: 6 launches with the one-kernel Dhat
// (dhat), 8 with two hop launches per Dhat, 10 with separate update kernels
// as well; with a right preconditioner M, Dhat is applied to M p and M s and
// x is updated with them.  With fuse_p the direction update
// p = r + beta (p - omega v) that ends an iteration is done by the next
// iteration's Dhat p as it stages p (beta = 0 before the first: p = r); with
// fuse_s Dhat s forms s = r - alpha v as it stages s.
hipError_t bicg_iteration(const Inner &in)
{
    Ws &w = *in.w;
    const double k2 = in.kappa * in.kappa;
    hipError_t e;
    hipStream_t st = in.ctx->stream;
    const void *pp = w.p, *ss = w.s;
    if (in.nn) {
        if ((e = nn_apply_half(in.ctx, in.nn, in.B, w.p, in.ph, in.n_rhs, in.sp, w.ps.active, w.ps.flags)) != hipSuccess) return e;
        pp = in.ph;
    }
    // v = Dhat p; alpha = rho / <rh, v>
    HopArgs h1 = hop_args(w.tmp, pp, in.links, 1, 1.0);
    if (in.fuse_p) {
        h1.pre = kPreP;
        h1.pre_r = w.r;
        h1.pre_v = w.v;
        h1.pre_c0 = w.ps.beta;
        h1.pre_c1 = w.ps.omega;
        h1.pre_act = w.ps.active;
    }
    h1.clover = in.clover;  // with the clover term: A_oo^-1 H_oe p, then p - kappa^2 A_ee^-1 H_eo (..)
    HopArgs h2 = hop_args(w.v, w.tmp, in.links, 0, -k2);
    h2.clover = in.clover;
    h2.self = pp;
    h2.c_self = 1.0;
    h2.aux = w.rh;
    h2.dot_mode = kDotAuxOut;
    h2.partial = w.pA;
    if (in.dhat) {
        HopArgs d = h2;
        d.in = pp;
        d.pre = h1.pre;
        d.pre_r = h1.pre_r;
        d.pre_v = h1.pre_v;
        d.pre_c0 = h1.pre_c0;
        d.pre_c1 = h1.pre_c1;
        d.pre_act = h1.pre_act;
        d.skip_act = w.ps.active;
        if ((e = run_dhat(in.ctx, in.B, in.ba, d, in.ip)) != hipSuccess) return e;
    } else {
        h1.skip_act = h2.skip_act = w.ps.active;
        if ((e = run_hop(in.ctx, in.B, in.ba, h1, in.ip)) != hipSuccess) return e;
        if ((e = run_hop(in.ctx, in.B, in.ba, h2, in.ip)) != hipSuccess) return e;
    }
    if ((e = launch_sc_alpha(in.ba, w.pA, w.ps, st)) != hipSuccess) return e;
    if (!in.fuse_s && (e = launch_bicg_s(in.ba, in.sp, w.r, w.v, w.s, w.ps, st)) != hipSuccess) return e;
    if (in.nn) {
        if ((e = nn_apply_half(in.ctx, in.nn, in.B, w.s, in.sh, in.n_rhs, in.sp, w.ps.active, w.ps.flags)) != hipSuccess) return e;
        ss = in.sh;
    }
    // t = Dhat s; omega = <t, s> / <t, t>
    HopArgs h3 = hop_args(w.tmp, ss, in.links, 1, 1.0);
    if (in.fuse_s) {
        h3.pre = kPreS;
        h3.pre_r = w.r;
        h3.pre_v = w.v;
        h3.pre_c0 = w.ps.alpha;
        h3.pre_act = w.ps.active;
    }
    h3.clover = in.clover;
    HopArgs h4 = hop_args(w.t, w.tmp, in.links, 0, -k2);
    h4.clover = in.clover;
    h4.self = ss;
    h4.c_self = 1.0;
    h4.dot_mode = in.nn ? kDotOutAuxOutOut : kDotOutSelfOutOut;
    h4.aux = in.nn ? w.s : nullptr;
    h4.partial = w.pB;
    if (in.dhat) {
        HopArgs d = h4;
        d.in = ss;
        d.pre = h3.pre;
        d.pre_r = h3.pre_r;
        d.pre_v = h3.pre_v;
        d.pre_c0 = h3.pre_c0;
        d.pre_act = h3.pre_act;
        d.skip_act = w.ps.active;
        if ((e = run_dhat(in.ctx, in.B, in.ba, d, in.ip)) != hipSuccess) return e;
    } else {
        h3.skip_act = h4.skip_act = w.ps.active;
        if ((e = run_hop(in.ctx, in.B, in.ba, h3, in.ip)) != hipSuccess) return e;
        if ((e = run_hop(in.ctx, in.B, in.ba, h4, in.ip)) != hipSuccess) return e;
    }
    if ((e = launch_sc_omega(in.ba, w.pB, w.ps, st)) != hipSuccess) return e;
    if ((e = launch_bicg_xr(in.ba, in.sp, w.xi, pp, ss, w.s, w.t, w.r, w.rh, w.pC, w.ps, st)) != hipSuccess) return e;
    if ((e = launch_sc_beta(in.ba, w.pC, w.ps, st)) != hipSuccess) return e;
    return in.fuse_p ? hipSuccess : launch_bicg_p(in.ba, in.sp, w.r, w.v, w.p, w.ps, st);
}

// Inner tolerance by precision.  FP32: every defect-correction cycle cuts
// the true residual by about the inner tolerance, so 0.3 sqrt(tol) reaches
// tol in two cycles with a margin of ten; not below 1e-6, where the FP32
// operator's rounding takes over.  BF16 links: their rounding (2^-9) bounds
// what an inner solve can gain.
double default_inner_tol(dd_prec ip, double tol)
{
    if (ip == DD_F64) return std::max(0.1 * tol, 1e-14);
    if (ip == DD_F32) return std::max(0.3 * std::sqrt(tol), 1e-6);
    return 2e-3;
}

// Work queues for the persistent solver: blocks are dealt to the nq queues
// largest first, each to the queue with the least work so far (sites x
// rhs); a block's right-hand sides stay adjacent in its queue.
const QueueTable *queues_for(dd_blocks *B, int nr, int nq, hipError_t *err)
{
    *err = hipSuccess;
    const int key = nr * 16 + nq;
    auto it = B->queues.find(key);
    if (it != B->queues.end()) return &it->second;
    std::vector<int> order(B->nb);
    for (int b = 0; b < B->nb; b++) order[b] = b;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
        return B->shapes[B->shape_of[a]].h > B->shapes[B->shape_of[b]].h;
    });
    std::vector<std::vector<int32_t>> q(nq);
    std::vector<int64_t> load(nq, 0);
    for (int b : order) {
        const int k = (int)(std::min_element(load.begin(), load.end()) - load.begin());
        for (int r = 0; r < nr; r++) q[k].push_back(r * B->nb + b);
        load[k] += (int64_t)B->shapes[B->shape_of[b]].h * nr;
    }
    std::vector<int32_t> flat, off(1, 0);
    for (auto &v : q) {
        flat.insert(flat.end(), v.begin(), v.end());
        off.push_back((int32_t)flat.size());
    }
    QueueTable qt;
    qt.nq = nq;
    if ((*err = upload(&qt.d_queue, flat)) != hipSuccess) return nullptr;
    if ((*err = upload(&qt.d_qoff, off)) != hipSuccess) return nullptr;
    if ((*err = upload(&qt.d_qctr, std::vector<int32_t>(nq, 0))) != hipSuccess) return nullptr;
    return &(B->queues[key] = qt);
}

}  // namespace

namespace dd {

// Launch shape of the persistent GMRES kernel: threads per workgroup, number
// of work queues and resident workgroups (grid), from the context's settings
// (dd_tune_set, dd_autotune_gmres) or the defaults.
bool gmres_walk(const dd_ctx *ctx, const dd_blocks *B) { return B->walk && ctx->hop_lds && ctx->hop_walk >= 0; }

hipError_t gmres_schedule(dd_ctx *ctx, dd_prec ip, int restart, int np, bool walk, bool cl, int *nt, int *nq,
                          int *grid)
{
    *nt = ctx->gm_threads > 0 ? ctx->gm_threads : 256;
    *nq = ctx->gm_queues > 0 ? ctx->gm_queues : 8;
    int occ = 0;
    hipError_t e = gmres_occupancy(ip, restart, *nt, walk, cl, &occ);
    if (e != hipSuccess) return e;
    if (occ < 1) return hipErrorInvalidConfiguration;
    int ncu = 0;
    if ((e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, ctx->device)) != hipSuccess) return e;
    const int wpc = ctx->gm_wg_per_cu > 0 ? std::min(ctx->gm_wg_per_cu, occ) : occ;
    *grid = std::max(1, std::min(np, wpc * ncu));
    return hipSuccess;
}

}  // namespace dd

extern "C" {

void dd_solve_params_default(dd_solve_params *p)
{
    if (!p) return;
    std::memset(p, 0, sizeof(*p));
    p->tol = 1e-10;
    p->method = DD_BICGSTAB;
    p->restart = 16;
    p->inner_prec = DD_F32;
    p->inner_tol = 0;
    p->max_outer = 30;
    p->max_inner = 2000;
    p->check_every = 2;
    p->use_graph = 1;
    p->recover = 1;
}

}  // extern "C"

namespace {

// Per-pair results of one batched solve (host copies).
struct PairResults {
    std::vector<int32_t> iters, flags;
    std::vector<double> bb, rr;
};

// The batched solve of dd_block_solve.  With only (device, per pair, may be
// null) the pairs whose entry is 0 take no part: they stay inactive with x = 0.
dd_status block_solve_impl(dd_ctx *ctx, const dd_blocks *Bc, const dd_gauge *G, double kappa, const void *b_dev,
                           void *x_dev, int32_t n_rhs, const dd_solve_params *params, dd_solve_stats *stats,
                           const int32_t *only, PairResults *res)
{
    const auto t_start = std::chrono::steady_clock::now();
    if (!ctx || !Bc || !G || !b_dev || !x_dev) return fail(ctx, DD_EINVAL, "null argument");
    if (n_rhs < 1 || n_rhs > kMaxRhs) return fail(ctx, DD_EINVAL, "n_rhs must be in 1..64");
    if (G->blocks != Bc) return fail(ctx, DD_EINVAL, "gauge was loaded for other blocks");
    if (!rhs_fit(Bc, n_rhs))
        return fail(ctx, DD_EUNSUPPORTED, "too many rhs for the block size (32-bit offsets of the half fields)");
    dd_solve_params prm;
    if (params) prm = *params;
    else dd_solve_params_default(&prm);
    if (!(prm.tol > 0)) return fail(ctx, DD_EINVAL, "tol must be positive");
    if (prm.x0 && x_dev == b_dev) return fail(ctx, DD_EINVAL, "a warm start needs x distinct from b");
    if (prm.method != DD_BICGSTAB && prm.method != DD_GMRES) return fail(ctx, DD_EINVAL, "unknown method");
    const bool gmres = prm.method == DD_GMRES;
    if (gmres && (prm.restart < 1 || prm.restart > 16)) return fail(ctx, DD_EINVAL, "restart must be in 1..16");
    // the network keeps a lazily refreshed BF16 copy of its weights
    dd_nn *nn = const_cast<dd_nn *>(prm.precond);
    if (nn && !gmres && nn->act != DD_NN_LINEAR)
        return fail(ctx, DD_EINVAL, "BiCGStab needs a linear network preconditioner (use DD_GMRES for ReLU)");
    if (nn && !nn_fits(nn, Bc)) return fail(ctx, DD_EINVAL, "every block must have the network's extent");
    const dd_prec ip = prm.inner_prec;
    const void *links = links_for(G, ip);
    if (!links) return fail(ctx, DD_EINVAL, "gauge holds no links of the inner precision");
    const dd_prec sp = ip == DD_F64 ? DD_F64 : DD_F32;
    // the clover term: A (FP64, outer residual) and A^-1 (inner precision) of
    // every block site; the inner system is the asymmetric even-odd form
    // 1 - kappa^2 A_ee^-1 H_eo A_oo^-1 H_oe, its two hops with A^-1 applied
    // to their hop results (walk or chunked hops, one rhs per thread)
    {
        const dd_status cs = clover_check(ctx, G, kappa);
        if (cs != DD_OK) return cs;
    }
    const void *cl_a64 = clover_for(G, DD_F64, false), *cl_inv = clover_for(G, ip, true);
    if (cl_a64) {
        if (gmres && !gmres_walk(ctx, Bc))
            return fail(ctx, DD_EUNSUPPORTED, "the clover term in GMRES needs blocks the x0-walk hop takes");
        if (!cl_inv) return fail(ctx, DD_EINVAL, "gauge holds no clover term of the inner precision");
    }
    const double inner_tol = prm.inner_tol > 0 ? prm.inner_tol : default_inner_tol(ip, prm.tol);
    // with the default inner tolerance and a low-precision inner solve, a later
    // cycle's BiCGStab stops once it has gained what is left to reach tol
    const bool adapt_tol = prm.inner_tol <= 0 && ip != DD_F64;
    const int max_outer = prm.max_outer > 0 ? prm.max_outer : 30;
    const int max_inner = prm.max_inner > 0 ? prm.max_inner : 2000;
    const int check = prm.check_every > 0 ? prm.check_every : 2;
    const bool graph = prm.use_graph && !ctx->timing && !(nn && gmres);

    dd_blocks *B = const_cast<dd_blocks *>(Bc);
    HIPCHECK(ctx, enter(ctx));
    hipError_t e;
    // the FP64 residual kernels and the inner-precision kernels may group rhs
    // differently; a scalar kernel reads partials with the tiling of the
    // kernel that wrote them
    const int g64 = hop_group(ctx, n_rhs, DD_F64, DD_F64), gsp = cl_a64 ? 1 : hop_group(ctx, n_rhs, sp, ip);
    const TileTable tt64 = tiles_for(B, n_rhs, g64), ttsp = tiles_for(B, n_rhs, gsp);
    const BlkArgs ba64 = blk_args(B, tt64, n_rhs, g64);
    const BlkArgs ba = blk_args(B, ttsp, n_rhs, gsp);
    const int np = n_rhs * B->nb;
    const int64_t hel = (B->soff[B->nb] / 2) * 24 * (int64_t)n_rhs;  // elements per half field
    const size_t h64 = (size_t)hel * 8, hsp = (size_t)hel * prec_bytes(sp);
    const size_t npart = (size_t)std::max({tt64.ntiles * g64, ttsp.ntiles * gsp, 1}) * kNRed * sizeof(double);

    Ws w;
    std::memset(&w, 0, sizeof(w));
    e = hipSuccess;
    auto get = [&](const char *name, size_t bytes) -> void * {
        if (e != hipSuccess) return nullptr;
        return workspace(ctx, name, bytes, &e);
    };
    w.be = (double *)get("s_be", h64);
    w.bo = (double *)get("s_bo", h64);
    w.xe = (double *)get("s_xe", h64);
    w.xo = (double *)get("s_xo", h64);
    w.re = (double *)get("s_re", h64);
    w.ro = (double *)get("s_ro", h64);
    if (sp == DD_F64) {
        w.rie = w.re;
        w.rio = w.ro;
    } else {
        w.rie = get("s_rie", hsp);
        w.rio = get("s_rio", hsp);
    }
    w.rhs = get("s_rhs", hsp);
    w.xi = get("s_xi", hsp);
    w.tmp = get("s_tmp", hsp);
    int gm_nt = 0, gm_nq = 0, gm_grid = 0;
    void *gm_ws = nullptr;
    double *gm_bytes = nullptr, *gm_beta0 = nullptr;
    void *gm_r = nullptr, *gm_z0 = nullptr;
    int32_t *gm_more[2] = {nullptr, nullptr};
    void *bc_ph = nullptr, *bc_sh = nullptr;
    const QueueTable *qt = nullptr;
    const int64_t vstr = 24 * (int64_t)B->max_h;
    if (gmres) {
        HIPCHECK(ctx, gmres_schedule(ctx, ip, prm.restart, np, gmres_walk(ctx, B), cl_a64 != nullptr, &gm_nt, &gm_nq,
                                     &gm_grid));
        qt = queues_for(B, n_rhs, gm_nq, &e);
        if (!qt) return fail(ctx, DD_EDEVICE, std::string("work queues: ") + hipGetErrorString(e));
        gm_ws = get("g_basis", (size_t)gm_grid * (gmres_basis_m(prm.restart) + 2) * vstr * prec_bytes(sp));
        gm_bytes = (double *)get("g_bytes", (size_t)np * sizeof(double));
        gm_beta0 = (double *)get("g_beta0", (size_t)np * sizeof(double));
        if (nn) {
            gm_r = get("g_r", hsp);
            gm_z0 = get("g_z0", hsp);
            gm_more[0] = (int32_t *)get("g_moreA", (size_t)np * sizeof(int32_t));
            gm_more[1] = (int32_t *)get("g_moreB", (size_t)np * sizeof(int32_t));
        }
        if ((gmres_basis_m(prm.restart) + 2) * (double)vstr * prec_bytes(sp) >= 4294967296.0)
            return fail(ctx, DD_EUNSUPPORTED, "blocks too large for the GMRES basis slots (32-bit offsets)");
    } else {
        w.r = get("s_r", hsp);
        w.rh = get("s_rh", hsp);
        w.p = get("s_p", hsp);
        w.v = get("s_v", hsp);
        w.s = get("s_s", hsp);
        w.t = get("s_t", hsp);
        if (nn) {
            bc_ph = get("s_ph", hsp);
            bc_sh = get("s_sh", hsp);
        }
    }
    w.pA = (double *)get("s_pA", npart);
    w.pB = (double *)get("s_pB", npart);
    w.pC = (double *)get("s_pC", npart);
    w.pe = (double *)get("s_pe", npart);
    w.po = (double *)get("s_po", npart);
    double *pd = (double *)get("s_pair_d", (size_t)np * 13 * sizeof(double));
    int32_t *pi = (int32_t *)get("s_pair_i", (size_t)np * 5 * sizeof(int32_t));
    if (e != hipSuccess) return fail(ctx, DD_ENOMEM, std::string("solver workspace: ") + hipGetErrorString(e));
    w.ps.rho = pd;
    w.ps.alpha = pd + 2 * np;
    w.ps.omega = pd + 4 * np;
    w.ps.beta = pd + 6 * np;
    w.ps.bb = pd + 8 * np;
    w.ps.rr = pd + 9 * np;
    w.os.bb = pd + 10 * np;
    w.os.rr = pd + 11 * np;
    w.ps.tol2 = pd + 12 * np;
    w.ps.active = pi;
    w.ps.flags = pi + np;
    w.ps.iters = pi + 2 * np;
    w.os.active = pi + 3 * np;
    w.os.flags = pi + 4 * np;
    w.ps.np = np;
    w.os.only = only;

    hipStream_t st = ctx->stream;
    HIPCHECK(ctx, hipMemsetAsync(pi, 0, (size_t)np * 5 * sizeof(int32_t), st));
    HIPCHECK(ctx, hipMemsetAsync(pd, 0, (size_t)np * 13 * sizeof(double), st));
    if (gm_bytes) HIPCHECK(ctx, hipMemsetAsync(gm_bytes, 0, (size_t)np * sizeof(double), st));
    // a warm start packs the caller's guess; otherwise every pair starts from x = 0
    const bool warm = prm.x0 != 0;
    if (warm) {
        HIPCHECK(ctx, launch_pack_spinor(B, (const double *)x_dev, w.xe, w.xo, DD_F64, n_rhs, st));
    } else {
        HIPCHECK(ctx, hipMemsetAsync(w.xe, 0, h64, st));
        HIPCHECK(ctx, hipMemsetAsync(w.xo, 0, h64, st));
    }
    HIPCHECK(ctx, launch_pack_spinor(B, (const double *)b_dev, w.be, w.bo, DD_F64, n_rhs, st));

    Inner in{ctx, B, ba, &w, links, ip, sp, kappa, inner_tol, gmres ? nullptr : nn, bc_ph, bc_sh, n_rhs,
             false, false, false, cl_a64 ? cl_inv : nullptr};
    if (!gmres) {
        in.dhat = dhat_walk_applies(ctx, B, ba, ip);
        if (!nn && ctx->bicg_fuse == 0) {
            const int nseg = in.dhat ? 1 : hop_walk_segments(ctx, B, ba, ip);
            in.fuse_s = nseg >= 1;
            in.fuse_p = nseg == 1;
        }
    }
    std::vector<int32_t> h_act(np);
    // the captured inner iterations; destroyed on every return path
    GraphHolder gh;
    hipGraph_t &g = gh.g;
    hipGraphExec_t &gx = gh.gx;
    int cycles = 0;
    int64_t inner_total = 0;
    dd_status status = DD_OK;
    for (int cyc = 0;; cyc++) {
        // FP64 true residual r_p = b_p - x_p + kappa H x_{1-p}, |r|^2 per pair;
        // the first cycle starts from x = 0, where r = b, unless a warm start
        // gave x: then |b|^2 is taken first (the reference of tol) and the
        // residual of the guess after it
        const bool from_zero = cyc == 0 && !warm;
        double *r_e = from_zero ? w.be : w.re, *r_o = from_zero ? w.bo : w.ro;
        if (cyc == 0 && warm) {
            HIPCHECK(ctx, launch_norm2(ba64, DD_F64, w.be, w.pe, st));
            HIPCHECK(ctx, launch_norm2(ba64, DD_F64, w.bo, w.po, st));
            HIPCHECK(ctx, launch_sc_outer(ba64, w.pe, w.po, 1, prm.tol, w.os, st));
        }
        for (int p = 0; p < 2; p++) {
            if (from_zero) {
                HIPCHECK(ctx, launch_norm2(ba64, DD_F64, p ? w.bo : w.be, p ? w.po : w.pe, st));
                continue;
            }
            HopArgs h = hop_args(p ? w.ro : w.re, p ? w.xe : w.xo, G->d_u64, p, kappa);
            h.self = p ? w.xo : w.xe;
            h.c_self = -1.0;
            if (cl_a64) {
                // r_p = b_p - A_pp x_p + kappa H x_{1-p}: A_pp x_p into r_p first
                HIPCHECK(ctx, launch_clover_apply(B, cl_a64, h.self, h.out, p, n_rhs, DD_F64,
                                                  cyc >= 2 ? w.os.active : nullptr, st));
                h.self = h.out;
            }
            h.add = p ? w.bo : w.be;
            h.c_add = 1.0;
            h.dot_mode = kDotOutOut;
            h.partial = p ? w.po : w.pe;
            // from the second residual on, only the pairs corrected in the
            // last cycle: the others keep their residual and its partial
            // sums, and stay converged (or flagged)
            if (cyc >= 2) h.skip_act = w.os.active;
            HIPCHECK(ctx, run_hop(ctx, B, ba64, h, DD_F64));
        }
        HIPCHECK(ctx, launch_sc_outer(ba64, w.pe, w.po, from_zero, prm.tol, w.os, st));
        HIPCHECK(ctx, hipMemcpyAsync(h_act.data(), w.os.active, np * sizeof(int32_t), hipMemcpyDeviceToHost, st));
        HIPCHECK(ctx, hipStreamSynchronize(st));
        int n_act = 0;
        for (int v : h_act) n_act += v != 0;
        if (n_act == 0 || cyc >= max_outer) break;
        cycles++;
        // inner source rhs_e = r_e + kappa H_eo r_o in the inner precision
        void *ri_e = w.rie, *ri_o = w.rio;
        if (sp != DD_F64) {
            HIPCHECK(ctx, launch_convert(r_e, DD_F64, w.rie, sp, hel, st));
            HIPCHECK(ctx, launch_convert(r_o, DD_F64, w.rio, sp, hel, st));
        } else {
            ri_e = r_e;
            ri_o = r_o;
        }
        {
            // with the clover term: rhs = A_ee^-1 (r_e + kappa H_eo A_oo^-1 r_o),
            // the odd part kept as A_oo^-1 r_o for the odd solution below
            if (cl_a64) {
                // into the residual's own workspace: with FP64 inner solves in
                // the first cycle ri_o is the source b_o itself
                void *dst = sp == DD_F64 ? (void *)w.ro : w.rio;
                HIPCHECK(ctx, launch_clover_apply(B, cl_inv, ri_o, dst, 1, n_rhs, sp, w.os.active, st));
                ri_o = dst;
            }
            HopArgs h = hop_args(w.rhs, ri_o, links, 0, kappa);
            h.self = ri_e;
            h.c_self = 1.0;
            if (cyc >= 1) h.skip_act = w.os.active;  // pairs this cycle solves
            HIPCHECK(ctx, run_hop(ctx, B, ba, h, ip));
            if (cl_a64)
                HIPCHECK(ctx, launch_clover_apply(B, cl_inv, w.rhs, w.rhs, 0, n_rhs, sp, w.os.active, st));
        }
        if (gmres) {
            GmArgs ga;
            ga.h = B->d_h;
            ga.soff = B->d_soff;
            ga.nbr_off = B->d_nbr_off;
            ga.nbr = B->d_nbr;
            ga.nb = B->nb;
            ga.n_rhs = n_rhs;
            ga.links = links;
            ga.rhs = w.rhs;
            ga.x = w.xi;
            ga.active = w.os.active;
            ga.queue = qt->d_queue;
            ga.qoff = qt->d_qoff;
            ga.qctr = qt->d_qctr;
            ga.nq = qt->nq;
            ga.ws = gm_ws;
            ga.vstr = vstr;
            ga.k2 = kappa * kappa;
            ga.tol = inner_tol;
            ga.adapt = adapt_tol ? 1 : 0;
            ga.tol_out = prm.tol;
            ga.obb = w.os.bb;
            ga.orr = w.os.rr;
            ga.m = prm.restart;
            ga.max_iter = max_inner;
            ga.nlinks = B->d_nlinks;
            ga.bytes = ctx->timing ? gm_bytes : nullptr;
            ga.iters = w.ps.iters;
            ga.flags = w.ps.flags;
            ga.relres = nullptr;
            ga.ext = B->d_ext;
            ga.walk = gmres_walk(ctx, B) ? 1 : 0;
            ga.clover = cl_a64 ? cl_inv : nullptr;
            {
                const int pc = ctx->gm_reorth == 0 ? kGmReorthPercent : ctx->gm_reorth;
                ga.reorth2 = pc < 0 ? -1.0 : (pc / 100.0) * (pc / 100.0);
            }
            ga.resume = 0;
            ga.r = gm_r;
            ga.z0 = nullptr;
            ga.max_cycles = 0;
            ga.more = nullptr;
            ga.beta0 = gm_beta0;
            if (nn) {
                // flexible GMRES: first direction N(f) of the first cycle, then N(r) of every
                // precond_cycles-th restart, the network applied to all pairs between launches
                HIPCHECK(ctx, nn_apply_half(ctx, nn, B, w.rhs, gm_z0, n_rhs, sp, nullptr, w.ps.flags));
                ga.z0 = gm_z0;
                ga.max_cycles = prm.precond_cycles > 0 ? prm.precond_cycles : 0;
                ga.more = gm_more[0];
                const int rounds = max_inner / std::max(1, prm.restart * std::max(1, ga.max_cycles)) + 1;
                for (int rd = 0; rd < rounds; rd++) {
                    {
                        TimedLaunch tl(ctx, DD_KCLASS_GMRES, 0.0);
                        HIPCHECK(ctx, launch_gmres(ga, ip, gm_nt, gm_grid, st));
                    }
                    if (ga.max_cycles == 0) break;
                    HIPCHECK(ctx, hipMemcpyAsync(h_act.data(), ga.more, np * sizeof(int32_t), hipMemcpyDeviceToHost, st));
                    HIPCHECK(ctx, hipStreamSynchronize(st));
                    int paused = 0;
                    for (int v : h_act) paused += v != 0;
                    if (paused == 0) break;
                    HIPCHECK(ctx, nn_apply_half(ctx, nn, B, gm_r, gm_z0, n_rhs, sp, nullptr, w.ps.flags));
                    ga.resume = 1;
                    ga.active = ga.more;
                    ga.more = ga.more == gm_more[0] ? gm_more[1] : gm_more[0];
                }
            } else if (graph) {
                // one defect-correction cycle's inner solve as a graph: clear the
                // queue counters, then the persistent launch
                if (!gx) {
                    HIPCHECK(ctx, hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
                    const hipError_t ce = launch_gmres(ga, ip, gm_nt, gm_grid, st);
                    const hipError_t ee = hipStreamEndCapture(st, &g);
                    if (ce != hipSuccess) return fail(ctx, DD_EDEVICE, std::string("capture: ") + hipGetErrorString(ce));
                    HIPCHECK(ctx, ee);
                    HIPCHECK(ctx, hipGraphInstantiate(&gx, g, nullptr, nullptr, 0));
                }
                HIPCHECK(ctx, hipGraphLaunch(gx, st));
            } else {
                TimedLaunch tl(ctx, DD_KCLASS_GMRES, 0.0);
                HIPCHECK(ctx, launch_gmres(ga, ip, gm_nt, gm_grid, st));
            }
        } else {
        HIPCHECK(ctx, launch_bicg_init(ba, sp, w.rhs, w.r, w.rh, in.fuse_p ? nullptr : w.p, w.xi, w.pA, w.os.active, st));
        HIPCHECK(ctx, launch_sc_init(ba, w.pA, w.ps, w.os, in.tol, prm.tol, adapt_tol ? 1 : 0, st));
        // the network's workspaces and BF16 weights exist before any capture
        if (in.nn && !gx) HIPCHECK(ctx, nn_apply_half(ctx, in.nn, B, w.p, in.ph, n_rhs, sp, w.ps.active, w.ps.flags));
        if (graph && !gx) {
            HIPCHECK(ctx, hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
            hipError_t ce = hipSuccess;
            for (int k = 0; k < check && ce == hipSuccess; k++) ce = bicg_iteration(in);
            hipError_t ee = hipStreamEndCapture(st, &g);
            if (ce != hipSuccess) return fail(ctx, DD_EDEVICE, std::string("capture: ") + hipGetErrorString(ce));
            HIPCHECK(ctx, ee);
            HIPCHECK(ctx, hipGraphInstantiate(&gx, g, nullptr, nullptr, 0));
        }
        for (int it = 0; it < max_inner; it += check) {
            if (gx) {
                HIPCHECK(ctx, hipGraphLaunch(gx, st));
            } else {
                for (int k = 0; k < check; k++) HIPCHECK(ctx, bicg_iteration(in));
            }
            inner_total += check;
            HIPCHECK(ctx, hipMemcpyAsync(h_act.data(), w.ps.active, np * sizeof(int32_t), hipMemcpyDeviceToHost, st));
            HIPCHECK(ctx, hipStreamSynchronize(st));
            int live = 0;
            for (int v : h_act) live += v != 0;
            if (live == 0) break;
        }
        }
        // e_o = r_o + kappa H_oe e_e, then x += e on the pairs above tolerance
        {
            HopArgs h = hop_args(w.tmp, w.xi, links, 1, kappa);
            h.self = ri_o;
            h.c_self = 1.0;
            h.clover = cl_inv;  // e_o = A_oo^-1 r_o + kappa A_oo^-1 H_oe e_e
            if (cyc >= 1) h.skip_act = w.os.active;  // the accumulation masks the others
            HIPCHECK(ctx, run_hop(ctx, B, ba, h, ip));
        }
        HIPCHECK(ctx, launch_accum(ba, w.xe, w.xi, sp, w.os.active, st));
        HIPCHECK(ctx, launch_accum(ba, w.xo, w.tmp, sp, w.os.active, st));
    }
    gh.reset();
    HIPCHECK(ctx, launch_unpack_spinor(B, w.xe, w.xo, (double *)x_dev, DD_F64, n_rhs, st));
    std::vector<double> h_bb(np), h_rr(np);
    std::vector<int32_t> h_if(np), h_of(np), h_it(np);
    HIPCHECK(ctx, hipMemcpyAsync(h_bb.data(), w.os.bb, np * sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHECK(ctx, hipMemcpyAsync(h_rr.data(), w.os.rr, np * sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHECK(ctx, hipMemcpyAsync(h_if.data(), w.ps.flags, np * sizeof(int32_t), hipMemcpyDeviceToHost, st));
    HIPCHECK(ctx, hipMemcpyAsync(h_of.data(), w.os.flags, np * sizeof(int32_t), hipMemcpyDeviceToHost, st));
    HIPCHECK(ctx, hipMemcpyAsync(h_it.data(), w.ps.iters, np * sizeof(int32_t), hipMemcpyDeviceToHost, st));
    std::vector<double> h_by;
    if (gmres && ctx->timing) {
        h_by.resize(np);
        HIPCHECK(ctx, hipMemcpyAsync(h_by.data(), gm_bytes, np * sizeof(double), hipMemcpyDeviceToHost, st));
    }
    HIPCHECK(ctx, hipStreamSynchronize(st));
    for (double v : h_by) ctx->timers[DD_KCLASS_GMRES].bytes += v;
    for (int k = 0; k < np; k++) {
        const int fl = (h_of[k] & 5) | (h_if[k] & 6);
        if (!(fl & 1)) status = DD_ENOCONV;
        if (stats) {
            if (stats->iters) stats->iters[k] = h_it[k];
            if (stats->true_relres) stats->true_relres[k] = h_bb[k] > 0 ? std::sqrt(h_rr[k] / h_bb[k]) : 0.0;
            if (stats->flags) stats->flags[k] = fl;
        }
    }
    if (gmres) inner_total = np ? *std::max_element(h_it.begin(), h_it.end()) : 0;
    if (stats) {
        stats->outer_cycles = cycles;
        stats->inner_iterations = inner_total;
        stats->rhs_per_solve = n_rhs;
        stats->resolved_pairs = 0;
        stats->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
    }
    if (res) {
        res->iters = h_it;
        res->bb = h_bb;
        res->rr = h_rr;
        res->flags.resize(np);
        for (int k = 0; k < np; k++) res->flags[k] = (h_of[k] & 5) | (h_if[k] & 6) | (h_if[k] & 16);
    }
    if (status == DD_ENOCONV) ctx->err = "some (block, rhs) pairs missed the tolerance";
    return status;
}

}  // namespace

extern "C" {

dd_status dd_block_solve(dd_ctx *ctx, const dd_blocks *B, const dd_gauge *G, double kappa, const void *b_dev,
                         void *x_dev, int32_t n_rhs, const dd_solve_params *params, dd_solve_stats *stats)
{
    const auto t_start = std::chrono::steady_clock::now();
    dd_solve_params prm;
    if (params) prm = *params;
    else dd_solve_params_default(&prm);
    PairResults res;
    dd_solve_stats st1;
    std::memset(&st1, 0, sizeof(st1));
    dd_status st = block_solve_impl(ctx, B, G, kappa, b_dev, x_dev, n_rhs, &prm, &st1, nullptr, &res);
    if (st != DD_OK && st != DD_ENOCONV) return st;
    const int np = n_rhs * B->nb;
    // recovery: the pairs that missed tol with a finite source (breakdown,
    // a non-finite inner value, or a low-precision or preconditioned inner
    // solve that stalled) are solved again with a plain FP64 inner solve
    int n_re = 0;
    std::vector<int32_t> mask(np, 0);
    if (st == DD_ENOCONV && prm.recover && (prm.inner_prec != DD_F64 || prm.precond)) {
        for (int k = 0; k < np; k++)
            if (!(res.flags[k] & 1) && std::isfinite(res.bb[k])) {
                mask[k] = 1;
                n_re++;
            }
    }
    PairResults res2;
    dd_solve_stats st2;
    std::memset(&st2, 0, sizeof(st2));
    if (n_re > 0) {
        hipError_t e = hipSuccess;
        const size_t xbytes = (size_t)n_rhs * B->soff[B->nb] * 24 * sizeof(double);
        void *x2 = workspace(ctx, "rs_x", xbytes, &e);
        int32_t *dm = x2 ? (int32_t *)workspace(ctx, "rs_mask", (size_t)np * sizeof(int32_t), &e) : nullptr;
        if (!dm) return fail(ctx, DD_ENOMEM, std::string("recovery workspace: ") + hipGetErrorString(e));
        HIPCHECK(ctx, hipMemcpyAsync(dm, mask.data(), (size_t)np * sizeof(int32_t), hipMemcpyHostToDevice, ctx->stream));
        // the same tolerance; the library's default FP64 inner solve and iteration limits
        dd_solve_params p64;
        dd_solve_params_default(&p64);
        p64.tol = prm.tol;
        p64.use_graph = prm.use_graph;
        p64.inner_prec = DD_F64;
        p64.recover = 0;
        const dd_status s2 = block_solve_impl(ctx, B, G, kappa, b_dev, x2, n_rhs, &p64, &st2, dm, &res2);
        if (s2 != DD_OK && s2 != DD_ENOCONV) return s2;
        HIPCHECK(ctx, launch_merge_pairs(B, (const double *)x2, (double *)x_dev, dm, n_rhs, ctx->stream));
        HIPCHECK(ctx, hipStreamSynchronize(ctx->stream));
    }
    st = DD_OK;
    for (int k = 0; k < np; k++) {
        const bool re = mask[k] != 0;
        const int fl = re ? (res2.flags[k] | 8) : res.flags[k];
        const double bb = re ? res2.bb[k] : res.bb[k], rr = re ? res2.rr[k] : res.rr[k];
        if (!(fl & 1)) st = DD_ENOCONV;
        if (stats) {
            if (stats->iters) stats->iters[k] = res.iters[k] + (re ? res2.iters[k] : 0);
            if (stats->true_relres) stats->true_relres[k] = bb > 0 ? std::sqrt(rr / bb) : 0.0;
            if (stats->flags) stats->flags[k] = fl;
        }
    }
    if (stats) {
        stats->outer_cycles = st1.outer_cycles + st2.outer_cycles;
        stats->inner_iterations = st1.inner_iterations + st2.inner_iterations;
        stats->rhs_per_solve = n_rhs;
        stats->resolved_pairs = n_re;
        stats->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
    }
    if (st == DD_ENOCONV) ctx->err = "some (block, rhs) pairs missed the tolerance";
    else ctx->err.clear();
    return st;
}

dd_status dd_autotune_gmres(dd_ctx *ctx, const dd_blocks *B, const dd_gauge *G, double kappa, const void *b_dev,
                            void *x_dev, int32_t n_rhs, const dd_solve_params *params, dd_tune_result *results,
                            int32_t max_results, int32_t *n_results)
{
    if (!ctx || !B || !G || !b_dev || !x_dev) return fail(ctx, DD_EINVAL, "null argument");
    dd_solve_params p;
    if (params) p = *params;
    else dd_solve_params_default(&p);
    if (p.restart < 1 || p.restart > 16) return fail(ctx, DD_EINVAL, "restart must be in 1..16");
    // one outer cycle whose inner solve runs exactly `restart` steps per pair
    p.x0 = 0;
    p.method = DD_GMRES;
    p.max_outer = 1;
    p.inner_tol = 1e-300;
    p.max_inner = p.restart;
    p.use_graph = 0;
    p.recover = 0;  // the timed cycles are not meant to converge
    const bool timing0 = ctx->timing;
    const int nt0 = ctx->gm_threads, nq0 = ctx->gm_queues, w0 = ctx->gm_wg_per_cu;
    auto restore = [&]() {
        ctx->timing = timing0;
        ctx->gm_threads = nt0;
        ctx->gm_queues = nq0;
        ctx->gm_wg_per_cu = w0;
    };
    struct Cand {
        int nt, nq, wpc;
        double ms;
    };
    std::vector<Cand> cand;
    for (int nt : {256, 512}) {
        int occ = 0;
        if (gmres_occupancy(p.inner_prec, p.restart, nt, gmres_walk(ctx, B), G->d_cla64 != nullptr, &occ) !=
                hipSuccess ||
            occ < 1)
            continue;
        for (int nq : {8, 1}) {
            cand.push_back({nt, nq, occ, 0.0});
            if (occ > 1) cand.push_back({nt, nq, (occ + 1) / 2, 0.0});
        }
    }
    if (cand.empty()) return fail(ctx, DD_EDEVICE, "no runnable GMRES schedule");
    // warm-up with the first candidate (workspaces, tables, code loading)
    ctx->gm_threads = cand[0].nt;
    ctx->gm_queues = cand[0].nq;
    ctx->gm_wg_per_cu = cand[0].wpc;
    dd_status st = dd_block_solve(ctx, B, G, kappa, b_dev, x_dev, n_rhs, &p, nullptr);
    if (st != DD_OK && st != DD_ENOCONV) {
        restore();
        return st;
    }
    ctx->timing = true;
    for (Cand &c : cand) {
        ctx->gm_threads = c.nt;
        ctx->gm_queues = c.nq;
        ctx->gm_wg_per_cu = c.wpc;
        dd_timer_reset(ctx);
        st = dd_block_solve(ctx, B, G, kappa, b_dev, x_dev, n_rhs, &p, nullptr);
        if (st != DD_OK && st != DD_ENOCONV) {
            restore();
            return st;
        }
        int64_t n = 0;
        double bytes = 0;
        if ((st = dd_timer_read(ctx, DD_KCLASS_GMRES, &c.ms, &n, &bytes)) != DD_OK) {
            restore();
            return st;
        }
    }
    dd_timer_reset(ctx);
    restore();
    const Cand *best = &cand[0];
    for (const Cand &c : cand)
        if (c.ms < best->ms) best = &c;
    ctx->gm_threads = best->nt;
    ctx->gm_queues = best->nq;
    ctx->gm_wg_per_cu = best->wpc;
    const int nr = std::min<int>((int)cand.size(), std::max(max_results, 0));
    for (int i = 0; results && i < nr; i++) results[i] = {cand[i].nt, cand[i].nq, cand[i].wpc, cand[i].ms};
    if (n_results) *n_results = (int32_t)cand.size();
    ctx->err.clear();
    return DD_OK;
}

// ------------------------------------------------- BiCGStab autotuner

namespace {

// Cache key of a tuning problem: device, lattice, block shapes, n_rhs, inner
// precision.  No quotes or backslashes (it is written as a JSON string).
std::string bicg_tune_key(const dd_ctx *ctx, const dd_blocks *B, int n_rhs, dd_prec ip)
{
    hipDeviceProp_t prop;
    std::string dev = "unknown";
    if (hipGetDeviceProperties(&prop, ctx->device) == hipSuccess)
        dev = std::string(prop.gcnArchName) + "/" + std::to_string(prop.multiProcessorCount) + "cu";
    std::string k = dev + "|L=" + std::to_string(B->L[0]) + "x" + std::to_string(B->L[1]) + "x" +
                    std::to_string(B->L[2]) + "x" + std::to_string(B->L[3]) + "|tbc=" + std::to_string(B->tbc) +
                    "|nb=" + std::to_string(B->nb) + "|shapes=";
    std::vector<int> count(B->shapes.size(), 0);
    for (int b = 0; b < B->nb; b++) count[B->shape_of[b]]++;
    for (size_t i = 0; i < B->shapes.size(); i++) {
        const dd::Shape &sh = B->shapes[i];
        k += std::to_string(sh.e[0]) + "x" + std::to_string(sh.e[1]) + "x" + std::to_string(sh.e[2]) + "x" +
             std::to_string(sh.e[3]) + "h" + std::to_string(sh.hole) + "*" + std::to_string(count[i]) + ";";
    }
    k += "|rhs=" + std::to_string(n_rhs) + "|inner=" + (ip == DD_F64 ? "f64" : ip == DD_F32 ? "f32" : "bf16");
    for (char &c : k)
        if (c == '"' || c == '\\' || (unsigned char)c < 32) c = '_';
    return k;
}

// The cache file: a JSON object with one entry per line,
//   "key": {"rhs_group": g, "dhat_walk": w, "dhat_rhs": r, "bicg_fuse": f, "ms": t},
// read and written by the two functions below (lines that do not parse are
// dropped when the file is rewritten).
bool bicg_cache_read(const char *path, std::vector<std::pair<std::string, dd_bicg_tune_result>> &out)
{
    out.clear();
    FILE *f = std::fopen(path, "r");
    if (!f) return false;
    char line[4096];
    while (std::fgets(line, sizeof(line), f)) {
        const char *q0 = std::strchr(line, '"');
        const char *q1 = q0 ? std::strchr(q0 + 1, '"') : nullptr;
        const char *br = q1 ? std::strchr(q1, '{') : nullptr;
        if (!br) continue;
        dd_bicg_tune_result r{};
        if (std::sscanf(br, "{\"rhs_group\": %d, \"dhat_walk\": %d, \"dhat_rhs\": %d, \"bicg_fuse\": %d, \"ms\": %lf",
                        &r.rhs_group, &r.dhat_walk, &r.dhat_rhs, &r.bicg_fuse, &r.ms) == 5)
            out.emplace_back(std::string(q0 + 1, q1), r);
    }
    std::fclose(f);
    return true;
}

bool bicg_cache_write(const char *path, const std::vector<std::pair<std::string, dd_bicg_tune_result>> &ent)
{
    const std::string tmp = std::string(path) + ".tmp";
    FILE *f = std::fopen(tmp.c_str(), "w");
    if (!f) return false;
    std::fprintf(f, "{\n");
    for (size_t i = 0; i < ent.size(); i++) {
        const dd_bicg_tune_result &r = ent[i].second;
        std::fprintf(f, "\"%s\": {\"rhs_group\": %d, \"dhat_walk\": %d, \"dhat_rhs\": %d, \"bicg_fuse\": %d, \"ms\": %.6f}%s\n",
                     ent[i].first.c_str(), r.rhs_group, r.dhat_walk, r.dhat_rhs, r.bicg_fuse, r.ms,
                     i + 1 < ent.size() ? "," : "");
    }
    std::fprintf(f, "}\n");
    const bool ok = std::fclose(f) == 0;
    return ok && std::rename(tmp.c_str(), path) == 0;
}

}  // namespace

dd_status dd_autotune_bicgstab(dd_ctx *ctx, const dd_blocks *B, const dd_gauge *G, double kappa, const void *b_dev,
                               void *x_dev, int32_t n_rhs, const dd_solve_params *params, const char *cache_path,
                               dd_bicg_tune_result *results, int32_t max_results, int32_t *n_results,
                               int32_t *from_cache)
{
    if (!ctx || !B || !G || !b_dev || !x_dev) return fail(ctx, DD_EINVAL, "null argument");
    if (n_rhs < 1 || n_rhs > kMaxRhs) return fail(ctx, DD_EINVAL, "n_rhs must be in 1..64");
    dd_solve_params p;
    if (params) p = *params;
    else dd_solve_params_default(&p);
    if (p.method != DD_BICGSTAB || p.precond) return fail(ctx, DD_EINVAL, "the BiCGStab autotuner takes plain BiCGStab");
    const dd_prec ip = p.inner_prec;
    const bool f64 = ip == DD_F64;
    int *rg = &ctx->rhs_group[f64 ? DD_TUNE_RHS_GROUP_F64 : DD_TUNE_RHS_GROUP_F32];
    const int rg0 = *rg, dw0 = ctx->dhat_walk, dr0 = ctx->dhat_rhs, bf0 = ctx->bicg_fuse;
    auto apply = [&](const dd_bicg_tune_result &c) {
        *rg = c.rhs_group;
        ctx->dhat_walk = c.dhat_walk;
        ctx->dhat_rhs = c.dhat_rhs;
        ctx->bicg_fuse = c.bicg_fuse;
    };
    auto restore = [&]() {
        *rg = rg0;
        ctx->dhat_walk = dw0;
        ctx->dhat_rhs = dr0;
        ctx->bicg_fuse = bf0;
    };
    if (from_cache) *from_cache = 0;
    if (n_results) *n_results = 0;
    const std::string key = bicg_tune_key(ctx, B, n_rhs, ip);
    std::vector<std::pair<std::string, dd_bicg_tune_result>> ent;
    if (cache_path && bicg_cache_read(cache_path, ent))
        for (const auto &e : ent)
            if (e.first == key) {
                apply(e.second);
                if (results && max_results > 0) results[0] = e.second;
                if (n_results) *n_results = 1;
                if (from_cache) *from_cache = 1;
                return DD_OK;
            }
    // candidates: rhs per thread of the site kernels (1, or 2 when it divides
    // n_rhs); with a low-precision inner solve the one-kernel Dhat (one or
    // three rhs per workgroup; one also with separate update kernels) or two
    // walk hops (with or without the fused staging updates); FP64: the two
    // walk hops only
    std::vector<dd_bicg_tune_result> cand;
    std::vector<int> groups = {1};
    if (n_rhs % 2 == 0) groups.push_back(2);
    for (int g : groups) {
        if (!f64) {
            cand.push_back({g, 0, 1, 0, 0.0});
            cand.push_back({g, 0, 3, 0, 0.0});
            cand.push_back({g, 0, 1, -1, 0.0});
        }
        cand.push_back({g, -1, 0, 0, 0.0});
        cand.push_back({g, -1, 0, -1, 0.0});
    }
    p.recover = 0;
    p.x0 = 0;
    apply(cand[0]);
    dd_status st = dd_block_solve(ctx, B, G, kappa, b_dev, x_dev, n_rhs, &p, nullptr);  // warm-up
    if (st != DD_OK && st != DD_ENOCONV) {
        restore();
        return st;
    }
    for (dd_bicg_tune_result &c : cand) {
        apply(c);
        HIPCHECK(ctx, hipStreamSynchronize(ctx->stream));
        const auto t0 = std::chrono::steady_clock::now();
        st = dd_block_solve(ctx, B, G, kappa, b_dev, x_dev, n_rhs, &p, nullptr);
        if (st != DD_OK && st != DD_ENOCONV) {
            restore();
            return st;
        }
        c.ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    }
    const dd_bicg_tune_result *best = &cand[0];
    for (const dd_bicg_tune_result &c : cand)
        if (c.ms < best->ms) best = &c;
    apply(*best);
    const int nr = std::min<int>((int)cand.size(), std::max(max_results, 0));
    for (int i = 0; results && i < nr; i++) results[i] = cand[i];
    if (n_results) *n_results = (int32_t)cand.size();
    if (cache_path) {
        ent.emplace_back(key, *best);
        if (!bicg_cache_write(cache_path, ent)) return fail(ctx, DD_EINVAL, std::string("cannot write ") + cache_path);
    }
    ctx->err.clear();
    return DD_OK;
}

dd_status dd_multiboson_action(dd_ctx *ctx, const dd_blocks *B, const dd_gauge *G, double kappa, int32_t n_fields,
                               const double *u_host, const void *chi_dev, const void *xi_dev,
                               const dd_solve_params *params, double *S_block_dev, double *S_total_host,
                               dd_solve_stats *stats)
{
    if (!ctx || !B || !G || !u_host || !chi_dev || !xi_dev) return fail(ctx, DD_EINVAL, "null argument");
    if (n_fields < 1 || n_fields > kMaxRhs) return fail(ctx, DD_EINVAL, "n_fields must be in 1..64");
    HIPCHECK(ctx, enter(ctx));
    dd_solve_params prm;
    if (params) prm = *params;
    else dd_solve_params_default(&prm);
    prm.x0 = 0;  // the solutions are internal workspaces
    // fields per block solve: the solver's workspace grows with the rhs of a call
    // (FP64 half fields, inner-precision Krylov vectors and the solutions), so
    // large lattices are solved a few fields at a time.  The context's own
    // workspaces count as free: they are reused or regrown, so the choice does
    // not depend on what earlier calls left allocated.
    const int64_t total = B->soff[B->nb];
    int fc = ctx->mb_fields;
    if (fc <= 0) {
        size_t fr = 0, tot = 0;
        HIPCHECK(ctx, hipMemGetInfo(&fr, &tot));
        for (const auto &kv : ctx->ws) fr += kv.second.bytes;
        const double per_field = (double)total * (192.0 + 576.0 + 132.0 * prec_bytes(prm.inner_prec == DD_F64 ? DD_F64 : DD_F32));
        fc = (int)std::max(1.0, std::floor(0.6 * (double)fr / per_field));
    }
    fc = std::min<int>(fc, n_fields);
    hipError_t e = hipSuccess;
    double *y = (double *)workspace(ctx, "mb_y", (size_t)total * 24 * fc * sizeof(double), &e);
    double *ud = y ? (double *)workspace(ctx, "mb_u", (size_t)n_fields * 2 * sizeof(double), &e) : nullptr;
    double *S = S_block_dev;
    if (ud && !S) S = (double *)workspace(ctx, "mb_S", (size_t)std::max(B->nb, 1) * sizeof(double), &e);
    if (!y || !ud || !S) return fail(ctx, DD_ENOMEM, std::string("workspace: ") + hipGetErrorString(e));
    HIPCHECK(ctx, hipMemcpyAsync(ud, u_host, (size_t)n_fields * 2 * sizeof(double), hipMemcpyHostToDevice,
                                 ctx->stream));
    const int64_t tb = B->boff[B->nb];
    dd_status st_all = DD_OK;
    double seconds = 0;
    int32_t cycles = 0, resolved = 0;
    int64_t inner = 0;
    for (int f0 = 0; f0 < n_fields; f0 += fc) {
        const int nf = std::min(fc, n_fields - f0);
        dd_solve_stats cs;
        std::memset(&cs, 0, sizeof(cs));
        if (stats) {
            const size_t o = (size_t)f0 * B->nb;
            cs.iters = stats->iters ? stats->iters + o : nullptr;
            cs.true_relres = stats->true_relres ? stats->true_relres + o : nullptr;
            cs.flags = stats->flags ? stats->flags + o : nullptr;
        }
        const dd_status st = dd_block_solve(ctx, B, G, kappa, (const double *)xi_dev + (size_t)f0 * total * 24, y, nf,
                                            &prm, &cs);
        if (st != DD_OK && st != DD_ENOCONV) return st;
        if (st == DD_ENOCONV) st_all = DD_ENOCONV;
        seconds += cs.seconds;
        cycles = std::max(cycles, cs.outer_cycles);
        inner += cs.inner_iterations;
        resolved += cs.resolved_pairs;
        HIPCHECK(ctx, launch_mb_norm(B, nf, ud + 2 * f0, (const double *)chi_dev + (size_t)f0 * tb * 24, y, S,
                                     f0 > 0, ctx->stream));
    }
    if (stats) {
        stats->seconds = seconds;
        stats->outer_cycles = cycles;
        stats->inner_iterations = inner;
        stats->rhs_per_solve = fc;
        stats->resolved_pairs = resolved;
    }
    if (S_total_host) {
        std::vector<double> hs(B->nb);
        HIPCHECK(ctx, hipMemcpyAsync(hs.data(), S, B->nb * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
        HIPCHECK(ctx, hipStreamSynchronize(ctx->stream));
        double tot = 0;
        for (double v : hs) tot += v;
        *S_total_host = tot;
    }
    HIPCHECK(ctx, hipStreamSynchronize(ctx->stream));
    if (st_all == DD_ENOCONV) ctx->err = "some (block, field) pairs missed the tolerance";
    return st_all;
}

dd_status dd_mb_exterior_source(dd_ctx *ctx, const dd_blocks *B, const dd_gauge *G, double kappa, int32_t n_fields,
                                const void *chi_global_dev, void *xi_dev, int32_t parts)
{
    if (!ctx || !B || !G || !chi_global_dev || !xi_dev) return fail(ctx, DD_EINVAL, "null argument");
    if (G->blocks != B) return fail(ctx, DD_EINVAL, "gauge was loaded for other blocks");
    if (n_fields < 1 || n_fields > kMaxRhs) return fail(ctx, DD_EINVAL, "n_fields must be in 1..64");
    if (parts < 1 || parts > 3) return fail(ctx, DD_EINVAL, "parts must be 1 (dPi_1), 2 (dLambda_0) or 3 (both)");
    HIPCHECK(ctx, enter(ctx));
    if (!B->x_code.empty()) {
        HIPCHECK(ctx, launch_mb_exterior(B, G->d_uext, kappa, n_fields, (const double *)chi_global_dev,
                                         (double *)xi_dev, parts, ctx->stream));
    }
    HIPCHECK(ctx, hipStreamSynchronize(ctx->stream));
    return DD_OK;
}

dd_status dd_mb_roots(int32_t N, double c, double *u_host)
{
    if (!u_host || N < 2 || (N & 1) || !(c > 0.0 && c < 1.0)) return DD_EINVAL;
    // u_k = 1 - z_k, k = 1 .. N/2, for the zeros z_k of the remainder polynomial
    // (one of each complex-conjugate pair): angle 2 pi k / (N + 1) on the ellipse
    // with semi-axes 1 and sqrt(1 - c^2)
    const double s = std::sqrt(1.0 - c * c);
    for (int k = 1; k <= N / 2; k++) {
        const double th = 2.0 * M_PI * k / (N + 1);
        u_host[2 * (k - 1)] = std::cos(th);
        u_host[2 * (k - 1) + 1] = s * std::sin(th);
    }
    return DD_OK;
}

}  // extern "C"
