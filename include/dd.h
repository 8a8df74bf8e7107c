/*
 * dd.h -- C ABI of libdd, the MI355X library for the block-restricted
 * Wilson-Dirac operator D_Lambda, its batched block solves D_Lambda^{-1} b
 * and the block-local multi-boson action.
 *
 * Paper: M. Saccardi, L. Giusti, "Four-dimensional domain decomposition for
 * the factorization of the fermion determinant" (Lattice 2022).
 *   - Section 1: link variables U_mu(x) on the links (x, x+mu), quark fields
 *     on the sites, local lattice Dirac operator D.
 *   - Section 2: active blocks Lambda_0^a, internal boundaries dLambda_0^a,
 *     frames Phi_1^a and framed blocks Omega_0^a.
 *   - Section 3: restrictions D_X with Dirichlet boundary, the factorisation
 *     of det D (eq. detD) and the off-diagonal blocks of W_1 (eq. offdiagW1),
 *     whose active part is P_{dLambda_0^a} D_{Omega_0^a}^{-1} (...).
 *   - Section 4: the block-local multi-boson action (eq. localMB) and the
 *     roots u_k.
 *
 * Conventions used by every entry point
 * -------------------------------------
 * Lattice L = (L0, L1, L2, L3); direction 0 is time.  Canonical site index
 * n = ((x0*L1 + x1)*L2 + x2)*L3 + x3.  All L_mu must be even.
 * Operator: D = 1 - kappa H,
 *   (H psi)(x) = sum_mu [ (1 - gamma_mu) U_mu(x) psi(x+mu) + (1 + gamma_mu) U_mu(x-mu)^+ psi(x-mu) ]
 * (Wilson-Dirac, hopping normalisation, no clover term), chiral gamma basis
 * gamma_0 = [[0,-1],[-1,0]], gamma_k = [[0,-i sigma_k],[i sigma_k,0]];
 * periodic in space; time antiperiodic (time_bc = -1) or periodic (+1).
 * D_Lambda for a block Lambda drops every hop whose source site lies outside
 * the block (Dirichlet), i.e. it is the principal sub-matrix of D.
 *
 * A block is a box: origin o[4], extent e[4] (even, e_mu <= L_mu); local
 * coordinate y maps to global x = (o + y) mod L.  A box may wrap around the
 * lattice; a box with e_mu == L_mu keeps its wrap-around links.
 * Each block also carries an inner (active) box, given by an offset and an
 * extent relative to the block; its boundary sites (those with a lattice
 * neighbour outside the inner box) form dLambda_0^a of the multi-boson action.
 *
 * Field layouts at the boundary (caller-owned device memory, complex128 as
 * interleaved re, im doubles):
 *   gauge  U[V][4][3][3]                         global canonical order
 *   spinor psi[n_rhs][total_sites][4][3]          blocks concatenated in block
 *                                                 order, each block in box-local
 *                                                 canonical order (local x3 fastest)
 *   chi    [n_fields][total_bnd_sites][4][3]      dLambda_0^a sites of each block,
 *                                                 in box-local canonical order
 *
 * Errors: every function returns a dd_status and never throws; a message is
 * kept in the context (dd_last_error).  Calls are ordered on the context's
 * HIP stream; host outputs are valid on return (the call synchronises).
 * A context is not thread-safe: use one per host thread.
 */
#ifndef DD_H
#define DD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    DD_OK = 0,
    DD_EINVAL = 1,        /* bad argument or shape mismatch */
    DD_ENOMEM = 2,        /* device or host allocation failed */
    DD_EDEVICE = 3,       /* a HIP call failed */
    DD_ENOCONV = 4,       /* some (block, rhs) pair missed the tolerance; stats are filled */
    DD_EUNSUPPORTED = 5   /* valid request the library does not implement */
} dd_status;

typedef enum { DD_F64 = 0, DD_F32 = 1, DD_BF16 = 2 } dd_prec;

typedef struct dd_ctx dd_ctx;
typedef struct dd_blocks dd_blocks;
typedef struct dd_gauge dd_gauge;
typedef struct dd_nn dd_nn;

/* ---------------------------------------------------------------- context */

/* Create a context on HIP device `device`, ordering all work on `hip_stream`
 * (a hipStream_t; NULL = the null stream).  The context owns its workspaces. */
dd_status dd_create(int device, void *hip_stream, dd_ctx **out);
dd_status dd_destroy(dd_ctx *ctx);
/* Last error message of the context (never NULL; "" if none).  With ctx ==
 * NULL: the message of the calling thread's last call made without a context. */
const char *dd_last_error(const dd_ctx *ctx);
/* Library version string. */
const char *dd_version(void);

/* --------------------------------------------------------------- geometry */

/* Tile mode (Section 2, step 1, with the blocks as tiles): the lattice is
 * tiled by boxes.  seg holds, direction after direction, the extents of the
 * consecutive tiles along that direction (nseg[mu] values each, summing to
 * L[mu]); tiles start at shift[mu] and wrap.  Blocks are listed with the tile
 * coordinate of direction 3 fastest.  Each block's inner box is the block
 * shrunk by inner_d sites on both sides in every direction where the block
 * does not span the lattice (inner_d = 0: the inner box is the block).
 * Returns DD_EINVAL for odd extents, extents that do not sum to L, or
 * inner boxes that would be empty. */
dd_status dd_make_blocks(dd_ctx *ctx, const int32_t L[4], int32_t time_bc, const int32_t *seg,
                         const int32_t nseg[4], const int32_t shift[4], int32_t inner_d,
                         dd_blocks **out);

/* Framed blocks of Section 2, step 3 ("box reading"): per direction mu either
 * bd[2mu] = 0 (direction not decomposed) or active extent b = bd[2mu] and gap
 * d = bd[2mu+1] >= 1 with (b + d) | L[mu].  Active blocks Lambda_0^a start at
 * multiples of b + d; the framed block Omega_0^a is the box
 * [s - d, s + b - 1 + d] and becomes the solve domain; Lambda_0^a is its inner
 * box.  Omega extents b + 2d must be even. */
dd_status dd_make_blocks_paper(dd_ctx *ctx, const int32_t L[4], int32_t time_bc,
                               const int32_t bd[8], dd_blocks **out);

/* Explicit list of n boxes: boxes[n][8] = origin[4], extent[4]; inner[n][8]
 * = offset[4], extent[4] of the inner box (NULL: inner box = block). */
dd_status dd_make_blocks_boxes(dd_ctx *ctx, const int32_t L[4], int32_t time_bc, int32_t n,
                               const int32_t *boxes, const int32_t *inner, dd_blocks **out);

/* The frames Phi_1^a = Omega_0^a minus Lambda_0^a of Section 2 as solve
 * domains (the D_{Phi_1^a} of Section 3's Dhat_{dLambda_0^a} and of eq. detD):
 * one block per block of `blocks`, with the same box, whose inner box is a
 * hole.  Every hop into or out of the hole is dropped, so on these blocks
 * D_Lambda is D_{Phi_1^a} on the frame sites and the identity on the hole
 * sites (dd_apply_D_block returns x there; dd_block_solve returns b there,
 * so a source that is zero on the hole gives x = D_{Phi_1^a}^{-1} b on the
 * frame and zero on the hole).  Layouts are those of blocks with the same
 * boxes (hole sites included); the frames carry no dLambda_0 sites.
 * DD_EINVAL when some inner box is its whole block.  ctx may be NULL as for
 * the other constructors. */
dd_status dd_make_frames(dd_ctx *ctx, const dd_blocks *blocks, dd_blocks **out);

/* The inactive region Lambda_1 of Section 2 as one solve domain (for the
 * global rest of the multi-boson action, Section 4 eq. globalMB): a single
 * block spanning the whole lattice (origin 0, extent L: its box-local
 * canonical order is the global one; hops wrap, with the antiperiodic time
 * sign) minus the union of the inner boxes of `blocks` (the active region
 * Lambda_0), whose sites are decoupled as in a frame's hole.  Its exterior
 * hops (dd_blocks_exterior, dd_mb_exterior_source with parts 2) are the hops
 * from the active boxes into the domain; dd_blocks_dpi1 lists its dPi_1
 * sites.  The domain is one block of V sites: its solves take the chunked
 * hop kernel (a block spanning the lattice in x0 has no x0-walk) and memory
 * for V sites per field.  DD_EINVAL when the inner boxes cover the lattice
 * (no inactive region) or the lattice exceeds the block size limit of the
 * constructors (11 184 810 sites, e.g. 56^4; 64^4 is refused).  ctx may be
 * NULL (host tables only). */
dd_status dd_make_inactive(dd_ctx *ctx, const dd_blocks *blocks, dd_blocks **out);
/* The dPi_1 sites of an inactive-region domain (sites of Lambda_1 with some
 * coordinate on a face coordinate of an active box, in directions where the
 * box does not span the lattice), ascending global canonical indices:
 * *n_sites their number; sites (may be NULL) at least that many entries.
 * DD_EINVAL for blocks not made by dd_make_inactive. */
dd_status dd_blocks_dpi1(const dd_blocks *blocks, int64_t *n_sites, int64_t *sites);

dd_status dd_free_blocks(dd_blocks *blocks);

/* Sizes: number of blocks, total block sites (sum of box volumes), total
 * dLambda_0 sites, and links inside the blocks (those D_Lambda keeps). */
dd_status dd_blocks_query(const dd_blocks *blocks, int64_t *n_blocks, int64_t *total_sites,
                          int64_t *total_bnd_sites, int64_t *inner_links);
/* Host copies of the index tables (each pointer may be NULL):
 *   boxes   [n_blocks][16]: origin[4], extent[4], inner offset[4], inner extent[4]
 *   sites   [total_sites]: global canonical index of each block site
 *   eo      [total_sites]: even-odd position of each block site inside its
 *           block (even global parity first, each parity in local canonical order)
 *   bnd     [total_bnd_sites]: box-local canonical index of each dLambda_0 site */
dd_status dd_blocks_tables(const dd_blocks *blocks, int32_t *boxes, int64_t *sites, int32_t *eo,
                           int32_t *bnd);

/* Host copies of the exterior hops of the multi-boson source (see
 * dd_mb_exterior_source), one entry per hop, ordered by block and receiving
 * site (each pointer may be NULL; arrays of *n_hops entries):
 *   block, site  the block and the box-local canonical index of the site the hop enters
 *   code         2 mu + f (f = 1: the exterior site is x - mu), bit 3 set when the hop
 *                crosses the antiperiodic time edge, bits 4-5 the part (1 dPi_1, 2 dLambda_0)
 *   nbr          global canonical index of the exterior site
 * Empty unless some block's inner box is not the whole block. */
dd_status dd_blocks_exterior(const dd_blocks *blocks, int64_t *n_hops, int32_t *block, int32_t *site, int32_t *code,
                             int64_t *nbr);

/* Size limit of every constructor: the kernels address a block's buffers
 * with 32-bit byte offsets from its base, so a block holds at most
 * 11 184 810 sites (its FP64 links below 4 GiB; DD_EINVAL beyond), and calls
 * with n_rhs rhs need n_rhs * (sites of the largest block) * 96 < 2^32
 * (DD_EUNSUPPORTED beyond; never reached by blocks of up to 10^4 sites).
 * The constructors above accept ctx == NULL: the blocks then hold host
 * tables only (for dd_blocks_query / dd_blocks_tables) and every call that
 * needs the device rejects them with DD_EINVAL. */

/* ------------------------------------------------------------------ gauge */

/* Copy the links inside every block from the canonical FP64 field U_dev into
 * the library's packed per-block layout: FP64 always, plus a low-precision
 * copy when low_prec is DD_F32 or DD_BF16 (rounding FP64 -> FP32 to nearest
 * even, then FP32 -> BF16 to nearest even).  U_dev is only read during the
 * call.  The links must be SU(3): only their first two rows are stored. */
dd_status dd_load_gauge(dd_ctx *ctx, const dd_blocks *blocks, const void *U_dev, dd_prec low_prec,
                        dd_gauge **out);
dd_status dd_free_gauge(dd_gauge *gauge);
/* Export the packed links of precision prec into dst_dev (device memory of
 * at least total_sites*4*12 elements of the precision: double, float or
 * uint16 BF16 bits).  Layout per block b (S_b sites, starting at element
 * 48 * site_offset(b)): [mu][k = 3*row + col, rows 0 and 1][eo site][re,im]
 * holding the first two rows of the forward link U_mu(x) of each block site x
 * (even sites first), multiplied by -1 when it crosses the antiperiodic time
 * edge; links that leave the block are zero.  Rounding to FP32/BF16 follows
 * the sign change (exact).  The kernels rebuild row 2 as conj(row0 x row1)
 * (with the edge sign), which is exact for SU(3) links. */
dd_status dd_gauge_export(dd_ctx *ctx, const dd_gauge *gauge, dd_prec prec, void *dst_dev);

/* Give the gauge's operator the clover (Sheikholeslami-Wohlert) term
 * (Section 3 takes D to be the Wilson or Sheikholeslami-Wohlert operator):
 * D = 1 - kappa H + (A - 1) with, at every site x,
 *   A(x) = 1 + i kappa c_sw sum_{mu<nu} sigma_{mu nu} Fhat_{mu nu}(x),
 *   sigma_{mu nu} = (i/2) [gamma_mu, gamma_nu] (chiral basis),
 *   Fhat_{mu nu}(x) = (Q_{mu nu}(x) - Q_{mu nu}(x)^+) / 8,
 * Q_{mu nu}(x) the four plaquettes of the (mu, nu) plane at x, each traversed
 * mu-then-nu; the gauge field is periodic in every direction.  U_dev is the
 * canonical FP64 field of the whole lattice (as for dd_load_gauge; only read
 * during the call): D_Lambda keeps A of the whole lattice at every block
 * site, so boundary sites see links outside their block.  The library
 * computes A and A^-1 per block site in FP64 (FP32 copies for a gauge with
 * FP32 or BF16 links; 72 reals per site and copy).  From then on
 * dd_apply_D_block, dd_apply_D_block_noalloc, dd_block_solve and
 * dd_multiboson_action use this operator and reject another kappa
 * (DD_EINVAL); solves run on 1 - kappa^2 A_ee^-1 H_eo A_oo^-1 H_oe: BiCGStab,
 * optionally right-preconditioned by a network (the hops of blocks the
 * x0-walk cannot take, such as an inactive region, run in the chunked hop
 * kernel), or persistent GMRES (DD_EUNSUPPORTED for blocks the x0-walk cannot
 * take); dd_block_logdet takes det A_ee det A_oo det(that operator).  c_sw = 0
 * removes the term (the Wilson operator).
 * Errors: DD_EINVAL (null argument, non-finite kappa or c_sw), DD_ENOMEM. */
dd_status dd_gauge_set_clover(dd_ctx *ctx, dd_gauge *gauge, const void *U_dev, double kappa, double csw);

/* ------------------------------------------------------------- operator */

/* y = D_Lambda x for every block and every right-hand side (Section 3, the
 * restriction D_X).  x_dev, y_dev: [n_rhs][total_sites][4][3] complex128.
 * prec selects the stencil arithmetic: DD_F64 (FP64 links, spinors and
 * accumulation), DD_F32 (FP32), DD_BF16 (BF16 links, FP32 spinors and
 * accumulation; needs a gauge loaded with low_prec = DD_BF16).  Inputs are
 * rounded to the stencil precision on entry, results widened to FP64. */
dd_status dd_apply_D_block(dd_ctx *ctx, const dd_blocks *blocks, const dd_gauge *gauge, double kappa,
                           dd_prec prec, const void *x_dev, void *y_dev, int32_t n_rhs);

/* dd_apply_D_block for callers that cannot allocate device memory (code
 * that must not call hipMalloc: under stream capture, in tight serving loops,
 * in harnesses that forbid it): the same operator and kernels, with the
 * four half fields it packs into (x_e, x_o, y_e, y_o) taken from a
 * preallocated scratch array of 128 MiB that the library holds on each
 * device until the process ends, instead of the context's workspaces.  The
 * call allocates nothing (no hipMalloc, no library allocation, no event
 * creation; the kernel timers are not used).  Requests whose half fields
 * exceed the array (total_sites * n_rhs * 48 * 8 bytes for DD_F64, * 4
 * otherwise, each of the four rounded up to 256 bytes) return DD_EINVAL.
 * Every call on one device shares that device's array: calls that overlap
 * on one device (several host threads or contexts) race and must be
 * serialized by the caller.  Arguments, layouts and results as for
 * dd_apply_D_block. */
dd_status dd_apply_D_block_noalloc(dd_ctx *ctx, const dd_blocks *blocks, const dd_gauge *gauge, double kappa,
                                   dd_prec prec, const void *x_dev, void *y_dev, int32_t n_rhs);

/* --------------------------------------------------------------- solves */

enum { DD_BICGSTAB = 0, DD_GMRES = 1 };

typedef struct {
    double tol;          /* per-pair true relative residual |b - D x| / |b| (FP64), e.g. 1e-10 */
    int32_t method;      /* DD_BICGSTAB (even-odd BiCGStab) or DD_GMRES (even-odd GMRES(restart)) */
    int32_t restart;     /* GMRES restart length, 1..16 (default 16) */
    dd_prec inner_prec;  /* stencil precision of the inner solve */
    double inner_tol;    /* relative tolerance of each inner solve (<= 0: library default:
                            FP64 max(0.1 tol, 1e-14); FP32 max(0.3 sqrt(tol), 1e-6), two
                            defect-correction cycles; BF16 links 2e-3; with FP32 or BF16
                            inner solves, per pair and cycle at least 0.3 tol |b| / |r| (what
                            is left to reach tol from the true residual r), at most 0.1) */
    int32_t max_outer;   /* defect-correction cycles (<= 0: default 30) */
    int32_t max_inner;   /* iterations per inner solve (<= 0: default 2000) */
    int32_t check_every; /* BiCGStab: inner iterations between convergence polls (<= 0: default 2;
                            pairs that converged stop updating at once, the launches
                            stop at the next poll after the last one) */
    int32_t use_graph;   /* replay inner iterations (BiCGStab) or the persistent inner launch
                            (GMRES) from a captured hipGraph */
    const dd_nn *precond; /* network preconditioner (NULL: none); every block must have the
                             network's extent.  DD_GMRES: flexible GMRES whose first direction
                             of a restart cycle is z = N(r) for the cycle's starting residual r.
                             DD_BICGSTAB: right preconditioning, Dhat N u = f with x = N u
                             (needs a DD_NN_LINEAR network) */
    int32_t precond_cycles; /* with precond: restart cycles between network applications
                               (<= 0: the network is applied once per inner solve) */
    int32_t recover;     /* 1 (default): pairs that miss tol with a finite source after the
                            low-precision or preconditioned solve (stalled inner solves,
                            breakdowns, non-finite inner values) are solved again from x = 0
                            with the library's default FP64 inner BiCGStab and iteration
                            limits (same tol); their flags get bit 3.  0: off */
    int32_t x0;          /* 1: x_dev holds an initial guess on entry (read, then overwritten with
                            the solution; it must not be b_dev): the first cycle takes the FP64
                            residual b - D_Lambda x0 (the tolerance stays relative to |b|), and
                            pairs whose guess already meets tol are not iterated.  0 (default):
                            x_dev is output only and every pair starts from x = 0.  Pairs that
                            recover solves again start from 0.  The multi-boson and global
                            entry points ignore it (their solutions are internal). */
} dd_solve_params;

typedef struct {
    int32_t *iters;       /* [n_rhs*n_blocks] inner iterations per pair (host, caller-owned, may be NULL) */
    double *true_relres;  /* [n_rhs*n_blocks] final FP64 true relative residual (may be NULL) */
    int32_t *flags;       /* [n_rhs*n_blocks] bit 0 converged, bit 1 breakdown seen, bit 2 non-finite,
                             bit 3 solved again in FP64 (recover), bit 4 the network's output was not
                             finite and the identity took its place (may be NULL) */
    double seconds;       /* wall time of the call */
    int32_t outer_cycles; /* defect-correction cycles run */
    int64_t inner_iterations; /* BiCGStab: inner iterations launched (summed over cycles);
                                 GMRES: largest per-pair total of Krylov steps */
    int32_t rhs_per_solve;    /* right-hand sides per batched solve (dd_multiboson_action: the
                                 fields it hands to one dd_block_solve; else n_rhs) */
    int32_t resolved_pairs;   /* pairs that missed tol in the low-precision form and were solved
                                 again with an FP64 inner solve (0 when none or not enabled) */
} dd_solve_stats;

/* Fill p with the defaults (tol 1e-10, BiCGStab, restart 16, FP32 inner). */
void dd_solve_params_default(dd_solve_params *p);

/* x = D_Lambda^{-1} b for every (block, rhs) pair, all blocks in one batch
 * (Section 3: the D_{Omega_0^a}^{-1} of eq. offdiagW1 and eq. localMB).
 * b_dev, x_dev: [n_rhs][total_sites][4][3] complex128; x_dev is output only
 * unless params->x0 asks for a warm start.
 * Method: FP64 defect correction on the true residual around an even-odd
 * Krylov solve of Dhat = 1 - kappa^2 H_eo H_oe in inner_prec.  Pair arrays
 * are ordered pair = rhs * n_blocks + block.  Returns DD_ENOCONV (stats
 * filled) if any pair misses tol. */
dd_status dd_block_solve(dd_ctx *ctx, const dd_blocks *blocks, const dd_gauge *gauge, double kappa,
                         const void *b_dev, void *x_dev, int32_t n_rhs, const dd_solve_params *params,
                         dd_solve_stats *stats);

/* ------------------------------------------------- multi-boson action */

/* The field parameters of Section 4: u_k = 1 - z_k for the N/2 zeros z_k of
 * P_N(z) = (1 - R_{N+1}(z))/z taken one per complex-conjugate pair
 * (k = 1 .. N/2), u_k = cos(2 pi k / (N + 1)) + i sqrt(1 - c^2) sin(2 pi k / (N + 1)).
 * u_host: [N/2][2] (re, im).  DD_EINVAL unless N is even and 0 < c < 1.
 * Host only. */
dd_status dd_mb_roots(int32_t N, double c, double *u_host);

/* Block-local multi-boson action of eq. (localMB), Section 4, for
 * field k taken at z = u_k:
 *   S^a = sum_k sum_{x in dLambda_0^a} | u_k chi_k(x) + (D_{Omega_0^a}^{-1} xi_k^a)(x) |^2
 * where xi_k^a (on the whole block Omega_0^a) collects the hop-in sources of
 * eq. (localMB).  u_host: [n_fields][2] (re, im).  chi_dev:
 * [n_fields][total_bnd_sites][4][3] complex128; xi_dev:
 * [n_fields][total_sites][4][3] complex128.  S_block_dev (may be NULL):
 * [n_blocks] FP64 device output; S_total_host (may be NULL): sum over blocks.
 * The solves use params (NULL: defaults); stats may be NULL.  The fields are
 * solved in groups (see DD_TUNE_MB_FIELDS) whose sums are added in order. */
dd_status dd_multiboson_action(dd_ctx *ctx, const dd_blocks *blocks, const dd_gauge *gauge,
                               double kappa, int32_t n_fields, const double *u_host,
                               const void *chi_dev, const void *xi_dev,
                               const dd_solve_params *params, double *S_block_dev,
                               double *S_total_host, dd_solve_stats *stats);

/* The source xi of eq. (localMB) from the multi-boson fields alone
 * (Section 4; eq. offdiagW1 of Section 3 for its dPi_1 part):
 *   xi_k^a += D_{Omega_0^a, E^a} chi_k   for every block a and field k,
 * i.e. the hops -kappa (1 -/+ gamma_mu) U chi_k into the sites of the block's
 * box Omega_0^a from the sites E^a outside it that are selected by parts:
 *   1: E^a = exterior boundary of Omega_0^a in dPi_1 (the term
 *      D_{Phi_1^a, dOmega^{a*}} chi_{dPi_1});
 *   2: E^a = exterior boundary in dLambda_0 (the active boundaries of the
 *      other blocks).  The dLambda_0^a rows of D_{Omega_0^a}^{-1} applied to
 *      this part equal those of [Dhat_{dLambda_0^a}]^{-1} Dhat^h chi with the
 *      exact hopping term Dhat^h_{aa'} = -D_{dLambda_0^a, Phi_1^a}
 *      D_{Phi_1^a}^{-1} P_{Phi_1^a} D_{Phi_1^{a'}, dLambda_0^{a'}} (the reading
 *      of Section 3's garbled bracket that makes its second decomposition
 *      exact), since Lambda_0^a meets the frame only through dLambda_0^a;
 *   3: both, i.e. the whole source: then dd_multiboson_action with xi and
 *      with chi on dLambda_0^a gives S_MB^a from chi alone.
 * dPi is the set of sites with some coordinate on a face coordinate (first
 * or last) of an inner box, in directions where that box does not span the
 * lattice; dLambda_0 its part in the inner boxes (their boundary sites),
 * dPi_1 the rest.  chi_global_dev: [n_fields][V][4][3] complex128 on the
 * whole lattice in canonical order (only dPi sites are read); xi_dev:
 * [n_fields][total_sites][4][3] complex128 in the block layout, updated in
 * place (FP64).  Blocks whose inner box is the block contribute nothing.
 * The links of the exterior hops are copied by dd_load_gauge (FP64). */
dd_status dd_mb_exterior_source(dd_ctx *ctx, const dd_blocks *blocks, const dd_gauge *gauge, double kappa,
                                int32_t n_fields, const void *chi_global_dev, void *xi_dev, int32_t parts);

/* The global rest of the multi-boson action (Section 4, eq. globalMB) for
 * n_fields fields, field k at z = u_k (as for dd_multiboson_action):
 *   S^r_k = sum_{x in dPi_1} | u_k chi_k(x) + (W_{dPi1,dL0} chi_k)(x) |^2,
 * with W_{dPi1,dL0} chi = Dhat_{dPi1}^{-1} Dhat_{dPi1,dL0} chi computed as
 * [D_{Lambda_1}^{-1} D_{Lambda_1,dLambda_0} chi] on dPi_1 (eliminating
 * Lambda1bar from D_{Lambda_1} gives the same vector): per field, the source
 * from the hops out of the active boxes (dd_mb_exterior_source), one
 * dd_block_solve on the inactive region with params (as for dd_block_solve;
 * NULL: defaults), and an FP64 fixed-order sum over dPi_1.  domain: made by
 * dd_make_inactive; gauge: loaded for it (dd_load_gauge copies the links of
 * its exterior hops), optionally with the clover term.  u_host: [n_fields]
 * complex (re, im); chi_global_dev: [n_fields][V][4][3] complex128 on the
 * whole lattice in canonical order (the values on dPi are read).  Fields are
 * solved a few at a time as memory allows (DD_TUNE_MB_FIELDS forces the
 * group size).  Outputs: S_field_host [n_fields] and *S_total_host (each may
 * be NULL); stats per field (pair = field), may be NULL.  Returns DD_ENOCONV
 * when some field's solve missed the tolerance (its value is still written). */
dd_status dd_mb_global_action(dd_ctx *ctx, const dd_blocks *domain, const dd_gauge *gauge, double kappa,
                              int32_t n_fields, const double *u_host, const void *chi_global_dev,
                              const dd_solve_params *params, double *S_field_host, double *S_total_host,
                              dd_solve_stats *stats);

/* W_z chi of eq. (MBaction), Section 4, as a vector on dPi, one z per field:
 * the rows on dLambda_0^a are the vector whose norm is S_MB^a (eq. localMB),
 *   z chi + D_{Omega_0^a}^{-1} xi^a,  xi^a = the hops of chi from dPi into
 *   Omega_0^a (dd_mb_exterior_source with parts 3), one dd_block_solve on blocks;
 * the rows on dPi_1 are those whose norm is S^r_MB (eq. globalMB),
 *   z chi + [D_{Lambda_1}^{-1} D_{Lambda_1,dLambda_0} chi],  one dd_block_solve on
 *   domain.  At z = 0 this is W_1 - 1, the off-diagonal part of W_1.
 * blocks/gauge: blocks with inner boxes and their gauge; domain/domain_gauge:
 * dd_make_inactive of these blocks and its gauge (the same links; DD_EINVAL
 * for a domain made from other blocks).  With the clover term
 * (dd_gauge_set_clover) on both gauges, same kappa and c_sw, the operator is
 * the Sheikholeslami-Wohlert one (the term is site-diagonal: the exterior
 * hops are unchanged, the solves take it); DD_EINVAL when only one gauge
 * carries it or the two differ.  z_host: [n_fields][2] (re, im).  chi_global_dev,
 * out_global_dev: [n_fields][V][4][3] complex128 on the lattice in canonical
 * order, distinct buffers; chi is read on dPi only, out is written everywhere
 * (zero off dPi).  params: the inner solves (NULL: defaults; their tolerance
 * bounds the error of W_z chi).  stats (may be NULL): seconds, outer cycles,
 * inner iterations and fields per group (rhs_per_solve); the per-pair arrays
 * are not written.  Fields are processed in groups as memory allows
 * (DD_TUNE_MB_FIELDS forces the size).  DD_ENOCONV when an inner solve missed
 * its tolerance (out is still written). */
dd_status dd_mb_apply_W(dd_ctx *ctx, const dd_blocks *blocks, const dd_gauge *gauge, const dd_blocks *domain,
                        const dd_gauge *domain_gauge, double kappa, int32_t n_fields, const double *z_host,
                        const void *chi_global_dev, void *out_global_dev, const dd_solve_params *params,
                        dd_solve_stats *stats);

/* Multi-boson field generation (Section 4; the one global inversion of the
 * method, on a vector of dPi, Conclusions): chi_k = W_{u_k}^{-1} eta_k, so that
 * chi_k has the density exp(-|W_{u_k} chi_k|^2) when eta_k has exp(-|eta_k|^2)
 * (each complex component with real and imaginary parts N(0, 1/2)).  The
 * random numbers are the caller's: eta_global_dev [n_fields][V][4][3]
 * complex128 (read on dPi only).  chi_global_dev: same layout, output (zero off
 * dPi).  Arguments as for dd_mb_apply_W; u_host [n_fields][2].  Method: FP64
 * BiCGStab per field over the vectors on dPi, the fields of a group in one
 * batch (each application of W is dd_mb_apply_W's two batched solves), a
 * field stopping when |r| <= tol |eta|; then one more application gives the
 * true residual |eta - W chi| / |eta|.  Inside the iteration the inner solves
 * of W stop at max(params tol, min(1e-6, 0.1 tol / rho)), rho the largest
 * relative residual |r| / |eta| of the fields still iterating (an inexact
 * Krylov method tolerates operator errors that grow as its residual falls);
 * the true residual takes the params tolerance, and fields whose true residual
 * is above tol restart from their current chi (at most twice, within maxit
 * iterations in all).  iters_host, relres_host [n_fields] (may be NULL):
 * iterations and true relative residual per field.
 * params: the inner solves, whose tolerance should be well below tol.
 * DD_ENOCONV when a field's true residual is above 10 tol, it broke down, or
 * an inner solve missed its tolerance (chi is still written). */
dd_status dd_mb_generate(dd_ctx *ctx, const dd_blocks *blocks, const dd_gauge *gauge, const dd_blocks *domain,
                         const dd_gauge *domain_gauge, double kappa, int32_t n_fields, const double *u_host,
                         const void *eta_global_dev, void *chi_global_dev, double tol, int32_t maxit,
                         const dd_solve_params *params, int32_t *iters_host, double *relres_host,
                         dd_solve_stats *stats);

/* Stochastic estimate of ln W_N, W_N = det{1 - R_{N+1}(W_1)} the reweighting
 * factor of eq. (rw), Section 4.  The remainder is R_{N+1}(z) =
 * T_{N+1}((1 - z)/c) / T_{N+1}(1/c) (the Chebyshev form whose zeros of
 * 1 - R_{N+1} are the roots of dd_mb_roots), applied to a vector by the
 * three-term recurrence in X = (1 - W_1)/c = -W_0/c, N + 1 applications of
 * W_0 (dd_mb_apply_W at z = 0); 1 - W_1 P_N(W_1) is never formed.  Then
 *   ln W_N = Tr ln(1 - R) = -sum_{m >= 1} Tr(R^m) / m,
 * truncated after `order` terms, each trace by the caller's noise vectors:
 *   term_j = -sum_{m=1}^{order} eta_j^+ R^m eta_j / m   (eta_j on dPi).
 * Any noise with E[eta eta^+] = 1 on dPi gives an unbiased estimate of the
 * truncated series; the unit vectors of dPi give it exactly.  N even >= 2,
 * 0 < c < 1 (as for dd_mb_roots), 1 <= order <= 64, 1 <= n_vec <= 64.
 * eta_global_dev: [n_vec][V][4][3] complex128 (read on dPi).  terms_host
 * [n_vec][2] and estimate_host [2] (their mean), each may be NULL.  Other
 * arguments as for dd_mb_apply_W.  Cost: order (N + 1) applications of W.
 * DD_ENOCONV when an inner solve missed its tolerance. */
dd_status dd_mb_log_reweight(dd_ctx *ctx, const dd_blocks *blocks, const dd_gauge *gauge, const dd_blocks *domain,
                             const dd_gauge *domain_gauge, double kappa, int32_t N, double c, int32_t order,
                             int32_t n_vec, const void *eta_global_dev, const dd_solve_params *params,
                             double *terms_host, double *estimate_host, dd_solve_stats *stats);

/* Per-block log-determinants (Section 3, eq. detD and the effective action
 * after it: the block factors ln det D_{Omega_0^a} on framed blocks, and
 * ln det D_{Phi_1^a} on the frames of dd_make_frames), in FP64:
 *   logdet_dev[2 a] = ln |det D_Lambda^a|,  logdet_dev[2 a + 1] = its phase in (-pi, pi]
 * (device, [n_blocks][2], may be NULL); total_host (may be NULL) [2]: the sum
 * over blocks (phase wrapped).  det D_Lambda = det(1 - kappa^2 H_eo H_oe) on
 * the even sites, assembled densely per block from the FP64 links and
 * factorised by batched LU with partial pivoting.  With the clover term
 * (dd_gauge_set_clover, same kappa; DD_EINVAL otherwise) det D_Lambda =
 * det A_ee det A_oo det(1 - kappa^2 A_ee^-1 H_eo A_oo^-1 H_oe), the last
 * assembled the same way with A^-1 in the hops, ln det A(x) of every block
 * site by LU of its two 6x6 chirality blocks.  Every block must have the
 * same number h of sites per parity with 12 h <= 6144 (DD_EUNSUPPORTED
 * otherwise); the dense matrices take 16 (12 h)^2 bytes per block (at most
 * 8 GiB at a time). */
dd_status dd_block_logdet(dd_ctx *ctx, const dd_blocks *blocks, const dd_gauge *gauge, double kappa,
                          double *logdet_dev, double *total_host);

/* ------------------------------------------------------------ tuning */

/* Launch-shape overrides (0 = automatic).  DD_TUNE_RHS_GROUP_F64 / _F32: the
 * number of right-hand sides one thread of the site kernels handles for
 * FP64 / FP32 spinors (1, 2 or 4; ignored when it does not divide n_rhs;
 * automatic: 2 for FP32 spinors with FP32 links, else 1).  Results do not
 * depend on it beyond rounding of the fused dot products' summation order,
 * which is fixed for a given setting. */
/* DD_TUNE_HOP_LDS: 1 (default) stages each hop tile's chunk of the input
 * field in LDS, 0 reads every neighbour from global memory.
 * DD_TUNE_HOP_WALK: the x0-walk of the hop (a workgroup streams the x0-slices
 * of a block for one group of rhs, reading each input slice once), used when
 * every block admits it (no block spans the lattice in x0, at most 512 sites
 * per x0-slice): 0 (default) automatic, -1 never, n >= 1 with each block's
 * slices split into n segments (clamped to what the block shapes allow).
 * Results do not depend on it beyond the summation order of the fused dot
 * products.
 * DD_TUNE_BICG_FUSE: BiCGStab without a preconditioner updates its vectors
 * s = r - alpha v and p = r + beta (p - omega v) inside the first hop of
 * Dhat s and Dhat p, as the x0-walk stages them (p only with one walk
 * segment per block): 0 (default) where the x0-walk runs, -1 never (separate
 * kernels).  Results do not depend on it beyond the rounding of contracted
 * multiply-adds.
 * DD_TUNE_DHAT_WALK: BiCGStab applies Dhat = 1 - kappa^2 H_eo H_oe as one
 * x0-walk kernel per product (the odd intermediate H_oe x stays in LDS, one
 * x0-slice at a time), with FP32 spinors when every block admits the walk
 * and one walk per (block, rhs) covers the device: 0 (default) there, -1
 * never (two hop launches and the intermediate in global memory).  Results
 * do not depend on it beyond the summation order of the fused dot products.
 * DD_TUNE_DHAT_RHS: right-hand sides one workgroup of that kernel walks in
 * lockstep (sharing the block's link loads): 0 (default) or 1 for one, 3 for
 * three (fewer link re-reads, but measured slower on 8^4 blocks: the three
 * walks share barriers and hide memory latency worse).  Results do not depend
 * on it. */
/* Schedule of the persistent GMRES solver (0 = default):
 * DD_TUNE_GMRES_THREADS  threads per workgroup, 256 or 512;
 * DD_TUNE_GMRES_QUEUES   work queues, 1 (one global queue) or 8 (one per XCD:
 *                        a block's right-hand sides go to one XCD);
 * DD_TUNE_GMRES_WG_PER_CU resident workgroups per compute unit, at most what
 *                        fits.  Results depend on the threads per workgroup
 *                        only through the fixed summation order of the
 *                        workgroup's dot products. */
/* DD_TUNE_GMRES_REORTH: Gram-Schmidt of the persistent GMRES.  Each step
 * projects w = Dhat v_j once (classical Gram-Schmidt, FP64 sums and
 * updates) and reorthogonalizes with a second pass when |w - V h| keeps at
 * most p percent of |w|: 0 (default) p = 10, 1..100 that p (100: always, the
 * CGS2 scheme), -1 never. */
/* DD_TUNE_MB_FIELDS: fields dd_multiboson_action hands to one block solve
 * (0 = as many as fit in 60 % of the free device memory).
 * DD_TUNE_NN_KERNEL: BF16 network kernel, 1 (default) one workgroup per block
 * with its input slices staged in LDS, 0 neighbour rows read from global
 * memory (also used when a block's x0-slice exceeds 512 sites). */
enum {
    DD_TUNE_RHS_GROUP_F64 = 0,
    DD_TUNE_RHS_GROUP_F32 = 1,
    DD_TUNE_HOP_LDS = 2,
    DD_TUNE_GMRES_THREADS = 3,
    DD_TUNE_GMRES_QUEUES = 4,
    DD_TUNE_GMRES_WG_PER_CU = 5,
    DD_TUNE_MB_FIELDS = 6,
    DD_TUNE_NN_KERNEL = 7,
    DD_TUNE_HOP_WALK = 8,
    DD_TUNE_GMRES_REORTH = 9,
    DD_TUNE_BICG_FUSE = 10,
    DD_TUNE_DHAT_WALK = 11,
    DD_TUNE_DHAT_RHS = 12
};
dd_status dd_tune_set(dd_ctx *ctx, int32_t what, int32_t value);

/* One timed schedule of the persistent GMRES solver. */
typedef struct {
    int32_t threads;    /* threads per workgroup */
    int32_t queues;     /* work queues */
    int32_t wg_per_cu;  /* resident workgroups per compute unit */
    double ms;          /* time of the persistent launch */
} dd_tune_result;

/* Autotuner of the persistent GMRES schedule for these blocks, n_rhs and
 * params->inner_prec / params->restart: times one restart cycle (exactly
 * `restart` Krylov steps for every pair) of the first inner solve of b under
 * each candidate schedule (threads 256 or 512; 8 queues or 1; all resident
 * workgroups that fit, or half of them), then keeps the fastest in the
 * context, as dd_tune_set would.  x_dev (the size of b) is scratch and is
 * overwritten.  results (may be NULL) receives up to max_results timings in
 * candidate order, n_results (may be NULL) their number.  The solve itself is
 * not meant to converge here.  The kernel timers are reset. */
dd_status dd_autotune_gmres(dd_ctx *ctx, const dd_blocks *blocks, const dd_gauge *gauge, double kappa,
                            const void *b_dev, void *x_dev, int32_t n_rhs, const dd_solve_params *params,
                            dd_tune_result *results, int32_t max_results, int32_t *n_results);

/* One timed configuration of the BiCGStab path (the dd_tune_set knobs it sets). */
typedef struct {
    int32_t rhs_group;  /* DD_TUNE_RHS_GROUP_F32 (or _F64 for an FP64 inner solve): 1 or 2 */
    int32_t dhat_walk;  /* DD_TUNE_DHAT_WALK: 0 (the one-kernel Dhat) or -1 (two walk hops) */
    int32_t dhat_rhs;   /* DD_TUNE_DHAT_RHS: 1 or 3 with the one-kernel Dhat, else 0 */
    int32_t bicg_fuse;  /* DD_TUNE_BICG_FUSE: 0 or -1 (with two walk hops) */
    double ms;          /* wall time of one full dd_block_solve of b */
} dd_bicg_tune_result;

/* Autotuner of the BiCGStab path for these blocks, n_rhs and
 * params->inner_prec (plain BiCGStab; DD_EINVAL otherwise): after one
 * warm-up solve, times one full dd_block_solve of b under each candidate (rhs
 * per thread 1, or 2 when it divides n_rhs; with an FP32 or BF16 inner solve
 * the one-kernel Dhat with 1 or 3 rhs per workgroup (1 also with separate
 * update kernels), or two walk hops with and without the fused staging
 * updates; FP64: the two walk hops) and keeps
 * the fastest in the context, as dd_tune_set would.  x_dev (the size of b) is
 * scratch.  cache_path (may be NULL): a JSON file (an object, one entry per
 * line) keyed by device, lattice, block shapes, n_rhs and inner precision;
 * when it holds this key nothing is timed, the stored configuration is
 * applied and *from_cache is 1; otherwise the winner is added to the file
 * (rewritten through a temporary file; DD_EINVAL if it cannot be written).
 * results (may be NULL): up to max_results timings in candidate order (on a
 * cache hit, the stored entry); n_results, from_cache may be NULL. */
dd_status dd_autotune_bicgstab(dd_ctx *ctx, const dd_blocks *blocks, const dd_gauge *gauge, double kappa,
                               const void *b_dev, void *x_dev, int32_t n_rhs, const dd_solve_params *params,
                               const char *cache_path, dd_bicg_tune_result *results, int32_t max_results,
                               int32_t *n_results, int32_t *from_cache);

/* ---------------------------------------------- learned preconditioner */

/* A small 4D convolutional network that approximates the block inverse on
 * blocks of one extent (not part of the paper, which needs only the exact
 * D_{Omega_0^a}^{-1} of Section 3: the network only speeds up the Krylov
 * solves that provide it, whose FP64 true residual still decides).
 *   layers: three 3^4 correlations with zero padding at the block faces and
 *           no bias, channels 24 -> 32 -> 32 -> 24, activation (identity or
 *           ReLU) after the first two;
 *   fields: rows [n][S][24] FP32, one row per block site in box-local
 *           canonical order (x3 fastest), channel 2 * (3 * spin + colour) +
 *           (0: real, 1: imaginary part);
 *   weights: layer after layer, each [81][c_in][c_out] FP32 with tap
 *           27 (t0 + 1) + 9 (t1 + 1) + 3 (t2 + 1) + (t3 + 1) for the offset
 *           t in {-1, 0, 1}^4 of the input site; dd_nn_num_weights() of them. */
enum { DD_NN_LINEAR = 0, DD_NN_RELU = 1 };
int64_t dd_nn_num_weights(void);
/* The weights are copied (host FP32); the handle keeps FP32 master weights
 * and Adam state on the context's device. */
dd_status dd_nn_create(dd_ctx *ctx, const int32_t extent[4], int32_t act, const float *weights_host, dd_nn **out);
dd_status dd_nn_free(dd_nn *nn);
dd_status dd_nn_get_weights(dd_ctx *ctx, const dd_nn *nn, float *weights_host);
/* y = N(x) on n blocks' rows (device FP32, [n][S][24] each); synchronizes.
 * prec DD_F32: FP32 arithmetic; DD_BF16: weights, input and hidden activations
 * rounded to BF16 (nearest even), products on the matrix cores with FP32
 * accumulation, FP32 output. */
dd_status dd_nn_apply(dd_ctx *ctx, dd_nn *nn, dd_prec prec, const float *x_dev, float *y_dev, int64_t n);
/* The network as a solve applies it to an even-odd reduced system: for every
 * (block, rhs) pair of x_dev ([n_rhs][total_sites][4][3] complex128, the
 * dd_block_solve layout; every block must have the network's extent) the
 * sites of even global parity are rounded to FP32, the network (in the
 * inference precision of dd_nn_set_inference; with BF16 the kernels skip the
 * taps that reach odd input sites and compute only even output sites) maps
 * them with the odd sites taken as zero, and y_dev receives the even output
 * sites widened to FP64 with its odd sites zero.  x_dev is only read;
 * synchronizes.  DD_EINVAL on a block of another extent. */
dd_status dd_nn_apply_blocks(dd_ctx *ctx, dd_nn *nn, const dd_blocks *blocks, const void *x_dev, void *y_dev,
                             int32_t n_rhs);
/* Precision of the network when a solve applies it (default DD_BF16). */
dd_status dd_nn_set_inference(dd_ctx *ctx, dd_nn *nn, dd_prec prec);

typedef struct {
    int32_t epochs;     /* passes over the training pairs (default 4) */
    int32_t batch;      /* pairs per Adam step (default 32) */
    double lr;          /* Adam step size (default 1e-3) */
    double beta1, beta2, eps;  /* Adam constants (0.9, 0.999, 1e-8) */
    uint64_t seed;      /* shuffling: epoch e uses a Mersenne-Twister-64 stream seeded seed + e */
    int32_t mask_even;  /* 1: the loss counts only sites even in global parity (default) */
} dd_nn_train_params;
void dd_nn_train_params_default(dd_nn_train_params *p);

/* Training data are (source, solution) pairs in dd_block_solve's layout:
 * src_dev / sol_dev [n_rhs][total_sites][4][3] complex128 over blocks that all
 * have the network's extent, pair p = rhs * n_blocks + block.  Loss of a batch:
 * mean over its pairs of |M (N(src) - sol)|^2 / |M sol|^2, M the mask above.
 * dd_nn_loss_grad: the loss and FP32 weight gradients (host, may be NULL) of
 * the listed pairs without updating anything.  dd_nn_train: Adam over shuffled
 * batches; per-epoch mean training loss and (with a validation set, else
 * NULL) validation loss into the host arrays [epochs] (may be NULL). */
dd_status dd_nn_loss_grad(dd_ctx *ctx, dd_nn *nn, const dd_blocks *blocks, const void *src_dev, const void *sol_dev,
                          int32_t n_rhs, const int32_t *pairs_host, int32_t n_pairs, int32_t mask_even,
                          double *loss, float *grad_host);
dd_status dd_nn_train(dd_ctx *ctx, dd_nn *nn, const dd_blocks *blocks, const void *src_dev, const void *sol_dev,
                      int32_t n_rhs, const void *val_src_dev, const void *val_sol_dev, int32_t val_n_rhs,
                      const dd_nn_train_params *params, double *train_loss, double *val_loss);

/* ------------------------------------------------------------ timing */

/* Kernel timing for roofline reports: when enabled, every launch of the
 * kernel class is bracketed by HIP events on the context's stream, and its
 * algorithmic bytes (the bytes the method must move, counted per block) are
 * accumulated.  The hop classes are the stencil kernel in each precision
 * (FP64; FP32; FP32 spinors with BF16 links).  Graph replay is disabled
 * while timing is on. */
/* DD_KCLASS_GMRES is the persistent GMRES launch (its algorithmic bytes are
 * counted per pair by the kernel).  DD_KCLASS_NN_BF16 is one BF16 application
 * of the network (three matrix-core launches) inside solves; its "bytes" field
 * counts the network's flops instead (414 720 per block site).
 * DD_KCLASS_DHAT_F32 / _BF16 are the one-kernel applications of Dhat in
 * BiCGStab (DD_TUNE_DHAT_WALK), FP32 spinors with FP32 / BF16 links: bytes
 * are the input and output fields, the operands of the fused dots other than
 * those two, the BiCGStab update's operands and the links once. */
enum {
    DD_KCLASS_HOP_F64 = 0,
    DD_KCLASS_HOP_F32 = 1,
    DD_KCLASS_HOP_BF16 = 2,
    DD_KCLASS_GMRES = 3,
    DD_KCLASS_NN_BF16 = 4,
    DD_KCLASS_DHAT_F32 = 5,
    DD_KCLASS_DHAT_BF16 = 6,
    DD_KCLASS_COUNT = 7
};
dd_status dd_timer_enable(dd_ctx *ctx, int32_t on);
dd_status dd_timer_reset(dd_ctx *ctx);
/* total_ms: summed event time; launches: count; alg_bytes: summed bytes. */
dd_status dd_timer_read(dd_ctx *ctx, int32_t kclass, double *total_ms, int64_t *launches,
                        double *alg_bytes);

#ifdef __cplusplus
}
#endif

#endif /* DD_H */
