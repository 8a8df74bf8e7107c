// Internal declarations of libdd (host side and kernel argument blocks).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <string>
#include <vector>

#include "dd.h"

namespace dd {

// Threads per workgroup of the site kernels; each thread handles one site and
// a group of right-hand sides.
constexpr int kTile = 256;
// Largest number of right-hand sides per call (a tile must hold every rhs).
constexpr int kMaxRhs = 64;
// Reals reduced per (tile, rhs) by the fused dot products.
constexpr int kNRed = 4;
// Links are stored as their first two rows (6 complex entries per direction);
// the kernels rebuild the third row of the SU(3) matrix as conj(row0 x row1).
// GMRES: reorthogonalize (a second Gram-Schmidt pass) when |w - V h| keeps
// at most this percentage of |w|
constexpr int kGmReorthPercent = 10;
constexpr int kLinkK = 6;  // complex entries stored per link: rows 0 and 1 (row 2 is rebuilt)
constexpr int kLinkReals = 4 * kLinkK * 2;  // per site: 4 directions
// clover term per site: two hermitian 6x6 blocks (the chiralities), each as
// 6 real diagonal entries and 15 complex entries above the diagonal
constexpr int kCloverHalf = 36;
constexpr int kCloverReals = 2 * kCloverHalf;
// A link in the algorithmic byte counts: the full 3x3 complex matrix (18
// reals), the amount the operator needs whatever the storage keeps of it.
constexpr int kLinkAlgReals = 18;
// Neighbour-table entry flags: bit 30 = hop across the antiperiodic time edge.
constexpr int32_t kNbrSign = 1 << 30;
constexpr int32_t kNbrMask = kNbrSign - 1;

struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
};

struct Timer {
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev;
    size_t used = 0;
    double bytes = 0;
};

}  // namespace dd

struct dd_ctx {
    int device = 0;
    hipStream_t stream = nullptr;       // library stream (non-blocking, default priority)
    hipStream_t user_stream = nullptr;  // caller's stream; each call waits for it on entry
    hipEvent_t enter_ev = nullptr;      // recorded on user_stream by each call
    void *blas = nullptr;               // rocBLAS handle of the dense LU (created on first use)
    std::string err;
    std::map<std::string, dd::DevBuf> ws;  // named, grow-only workspaces
    bool timing = false;
    dd::Timer timers[DD_KCLASS_COUNT];
    double *d_timer_bytes = nullptr;  // [DD_KCLASS_COUNT] bytes counted by kernels (timing on)
    int rhs_group[2] = {0, 0};  // forced rhs per thread for FP64 / FP32 spinors (0 = automatic)
    bool hop_lds = true;        // stage the hop's chunk of the input in LDS
    int hop_walk = 0;           // x0-walk of the hop: 0 automatic, -1 off, n >= 1 segments per block
    int gm_reorth = 0;          // GMRES reorthogonalization threshold: 0 default, -1 never, 1..100 percent of |w|
    int bicg_fuse = 0;          // BiCGStab updates inside the walk hop: 0 where possible, -1 never
    int dhat_walk = 0;          // Dhat as one x0-walk kernel in BiCGStab: 0 where possible, -1 never
    int dhat_rhs = 0;           // rhs per workgroup of that kernel: 0 automatic, 1 or 3
    int gm_threads = 0;         // persistent GMRES: threads per workgroup (0 = default)
    int gm_queues = 0;          // persistent GMRES: work queues, 1 or 8 (0 = default)
    int gm_wg_per_cu = 0;       // persistent GMRES: resident workgroups per CU (0 = all that fit)
    int mb_fields = 0;          // multi-boson action: fields per block solve (0 = as many as fit)
    int nn_kernel = 1;          // BF16 network kernel: 0 global gathers, 1 LDS slices
};

namespace dd {

// A block shape: everything the stencil needs that does not depend on where
// the block sits, except through the origin parity and the time-edge column.
struct Shape {
    int e[4];
    int full[4];
    int opar;   // parity of the origin
    int tw;     // local x0 of the link that crosses the antiperiodic time edge, or -1
    int S, h;   // sites, sites per parity
    int64_t links;     // links with both ends in the block (the hops D_Lambda keeps)
    int64_t nbr_off;   // offset (entries) of this shape's table in the neighbour array
    int64_t perm_off;  // offset of the eo -> local canonical permutation
    // A frame shape: the solve domain is the box minus the hole hio + [0, hie)
    // (local coordinates); hole sites are decoupled (every hop into or out of
    // the hole is dropped, so D acts as the identity there).
    // hole == 2: the excluded sites are those of mask (local canonical index),
    // e.g. every active box of an inactive-region domain
    int hole = 0;
    int hio[4] = {0, 0, 0, 0}, hie[4] = {0, 0, 0, 0};
    std::vector<uint8_t> mask;
    // Sites per parity of an x0-slice when the x0-walk of the hop applies to
    // the shape (the eo index of a site's x0-neighbour is its own index
    // +/- walk_hs in the other parity, hops along 1..3 stay in the slice, and
    // the x0 hops out of the first and last slices are dropped), else 0.
    int walk_hs = 0;
};

// Tile decomposition of the site kernels: a tile is one rhs group (g
// consecutive rhs) on a chunk of chunk[b] consecutive eo sites of block b
// (whole x0-slices when a slice has at most kTile sites per parity); tiles
// are ordered block, chunk, group (group fastest), so tile t is rhs group
// t % ng of the block's chunk number t / ng in the list of all chunks (ng =
// n_rhs / g).  The chunk list is a property of the blocks (built once with
// them); a tile table is only its size.
struct TileTable {
    int ntiles = 0;
};

// Work queues of the persistent solver: the (block, rhs) pairs split into nq
// queues (one per XCD, or a single one), each ordered largest block first
// with a block's right-hand sides adjacent.
struct QueueTable {
    int nq = 0;
    int32_t *d_queue = nullptr;  // pairs, queue after queue
    int32_t *d_qoff = nullptr;   // [nq + 1] queue offsets
    int32_t *d_qctr = nullptr;   // [nq] counters (cleared by every launch)
};

// a process-wide number for every dd_blocks made (never reused)
uint64_t next_blocks_serial();

}  // namespace dd

struct dd_blocks {
    dd_ctx *ctx = nullptr;  // creating context (identity only; may be destroyed first)
    uint64_t serial = dd::next_blocks_serial();
    uint64_t parent = 0;    // inactive-region domain: serial of the blocks it was made from
    int device = -1;        // device holding the tables (-1: host tables only)
    int L[4] = {0, 0, 0, 0};
    int tbc = -1;
    int nb = 0;
    std::vector<int32_t> box;       // [nb][16] origin, extent, inner offset, inner extent
    std::vector<uint8_t> hole;      // [nb] 1: the solve domain is the box minus the inner box (a frame)
    std::vector<int64_t> soff;      // [nb+1] site offsets
    std::vector<int32_t> shape_of;  // [nb]
    std::vector<dd::Shape> shapes;
    std::vector<int32_t> nbr;       // all shapes: [2][h][8]
    std::vector<int32_t> perm;      // all shapes: [S] eo position -> local canonical index
    std::vector<int32_t> iperm;     // all shapes: [S] local canonical index -> eo position
    std::vector<int32_t> bnd;       // dLambda_0 sites, box-local canonical, blocks concatenated
    std::vector<int64_t> boff;      // [nb+1] offsets into bnd
    int64_t inner_links = 0;
    int max_h = 0;
    // device copies
    int32_t *d_nbr = nullptr;
    int32_t *d_perm = nullptr;
    int32_t *d_iperm = nullptr;
    int64_t *d_soff = nullptr;      // [nb+1]
    int32_t *d_h = nullptr;         // [nb] sites per parity
    int32_t *d_nlinks = nullptr;    // [nb] links inside the block
    int64_t *d_nbr_off = nullptr;   // [nb] neighbour-table offset of the block's shape
    int64_t *d_perm_off = nullptr;  // [nb]
    int32_t *d_origin = nullptr;    // [nb][4]
    int32_t *d_ext = nullptr;       // [nb][4]
    int32_t *d_bnd = nullptr;       // [total bnd] box-local canonical index
    int64_t *d_boff = nullptr;      // [nb+1]
    // chunks of the site kernels' tiles (see TileTable), all blocks in order
    std::vector<int32_t> blk_chunk0;     // [nb+1] first chunk of each block
    int32_t *d_chunk = nullptr;          // [nb] sites per chunk of each block
    int32_t *d_chunk_block = nullptr;    // [total chunks] chunk -> block
    int32_t *d_blk_chunk0 = nullptr;     // [nb+1]
    std::map<int, dd::QueueTable> queues;  // keyed by (n_rhs, number of queues)
    bool walk = false;                     // every shape admits the x0-walk of the hop
    // Exterior hops of the multi-boson source (blocks with an inner box that
    // is not the whole block): each hop from a site of dPi outside a block's
    // box into a box site, grouped by (block, receiving box-local site).
    //   x_code: 2 mu + f (f = 1: the exterior site is x - mu), bit 3 the
    //           antiperiodic time sign, bits 4-5 the part: 1 dPi_1, 2 dLambda_0
    //   x_nbr:  global canonical index of the exterior site
    //   x_link: 4 n + mu of the link in the canonical field (n its lower end)
    std::vector<int32_t> xg_block, xg_site, xg_first;  // [ng], [ng], [ng + 1]
    std::vector<int32_t> x_code;
    std::vector<int64_t> x_nbr, x_link;
    int32_t *d_xg_block = nullptr, *d_xg_site = nullptr, *d_xg_first = nullptr, *d_x_code = nullptr;
    int64_t *d_x_nbr = nullptr, *d_x_link = nullptr;
    // An inactive-region domain (dd_make_inactive): one block, the whole
    // lattice minus the active boxes of the blocks it was made from; its
    // exterior hops are those from the active boxes into the domain (part 2),
    // and dpi1 lists the global canonical index of every site of dPi_1.
    bool inactive = false;
    std::vector<int64_t> dpi1;
    int64_t *d_dpi1 = nullptr;
};

struct dd_gauge {
    dd_ctx *ctx = nullptr;  // creating context (identity only; may be destroyed first)
    int device = 0;
    const dd_blocks *blocks = nullptr;
    dd_prec low = DD_F64;
    double *d_u64 = nullptr;     // [total_sites][4][18]
    float *d_u32 = nullptr;      // when low == DD_F32
    uint16_t *d_ubf = nullptr;   // when low == DD_BF16
    double *d_uext = nullptr;    // [exterior hops][3][3][re, im]: the link of each exterior hop (FP64)
    // clover (Sheikholeslami-Wohlert) term A of every block site and its
    // inverse, two packed hermitian 6x6 blocks (kCloverReals per site, layout
    // of clover_mul); FP32 copies when the links are FP32 or BF16; kappa and
    // c_sw they were built for (csw == 0: none)
    double *d_cla64 = nullptr, *d_cli64 = nullptr;
    float *d_cla32 = nullptr, *d_cli32 = nullptr;
    double cl_kappa = 0.0, cl_csw = 0.0;
};

namespace dd {

// ---------------------------------------------------------------- kernels

// Per-block tables the site kernels read.
struct BlkArgs {
    const int32_t *chunk_block;  // chunk -> block (all chunks of all blocks)
    const int32_t *blk_chunk0;   // [nb + 1] first chunk of each block
    const int32_t *h;
    const int64_t *soff;
    const int64_t *nbr_off;
    const int32_t *nbr;
    int ntiles;
    int n_rhs;
    int nb;  // number of blocks (pair = rhs * nb + block)
    int g;                 // right-hand sides per thread (1, 2 or 4; divides n_rhs)
    const int32_t *chunk;  // sites per chunk of each block
};

// Tiles of the x0-walk of the hop: tile (block, segment, rhs group), group
// fastest, walks the x0-slices of one of nseg equal segments of its block for
// one rhs group; every block has per = nseg * (n_rhs / g) tiles.
struct WalkArgs {
    const int32_t *ext;  // [nb][4] block extents
    int ntiles;
    int nseg;
    int per;
    int tile0 = 0;  // first tile of the launch (the hop walk may cover a range of blocks)
};

enum DotMode { kDotNone = 0, kDotAuxOut = 1, kDotOutSelfOutOut = 2, kDotOutOut = 3, kDotOutAuxOutOut = 4 };

// out = c_add*add + c_self*self + c_hop * (H in), on the sites of `parity`.
// in lives on the other parity.  Optional fused dot products per (tile, rhs).
struct HopArgs {
    void *out;
    const void *in;
    const void *self;
    const void *add;
    const void *aux;
    double c_self, c_hop, c_add;
    const void *links;
    double *partial;  // [ntiles][n_rhs][kNRed]
    int parity;
    int dot_mode;
    int use_lds;  // 0: every neighbour is read from global memory
    // update of `in` while the x0-walk stages it (kPre*; x0-walk only)
    int pre;
    const void *pre_r, *pre_v;
    const double *pre_c0, *pre_c1;  // complex per pair: kPreP beta, omega; kPreS alpha
    const int32_t *pre_act;         // per pair: 0 keeps `in` as it is
    // x0-walk kernels only (the hop walk skips a rhs group when all its pairs
    // have stopped): pairs whose flag is 0 are skipped (nothing of theirs is
    // read again before they restart); with timing, each walk done adds
    // bytes_site algorithmic bytes per eo site and rhs it covers to *bytes_acc
    const int32_t *skip_act;
    double *bytes_acc;
    double bytes_site;
    // x0-walk kernels, one rhs per thread: the block sites' clover matrices in
    // the hop's arithmetic precision (kCloverReals per site); the hop result
    // at an output site is multiplied by that site's matrix before the
    // epilogue combines it with self and add
    const void *clover;
    // blocks [b_lo, b_hi) only, when b_hi > b_lo (run_hop's x0-walk launches
    // just their tiles; the chunked hop does every block): others untouched
    int b_lo, b_hi;
};

// Vector updates of BiCGStab done by the first hop of Dhat as it stages its
// input (each input site is staged by one tile):
//   kPreP: in <- r + beta (in - omega v)   (the search direction; needs a
//          walk of one segment per block, so that no tile reads a site that
//          another has already overwritten)
//   kPreS: in <- r - alpha v                (written by the slice's owner)
enum { kPreNone = 0, kPreP = 1, kPreS = 2 };

// Per-pair Krylov state (device, structure of arrays).
struct PairState {
    double *rho;     // [2*np] complex
    double *alpha;   // [2*np]
    double *omega;   // [2*np]
    double *beta;    // [2*np]
    double *bb;      // [np]  |rhs|^2 of the inner system
    double *rr;      // [np]  |r|^2 (recursive)
    int32_t *active; // [np]  inner iteration still running
    int32_t *flags;  // [np]  bit 1 breakdown, bit 2 non-finite
    int32_t *iters;  // [np]  cumulative inner iterations
    double *tol2;    // [np]  squared relative inner tolerance of the current inner solve
    int np;
};

// Outer (defect-correction) state.
struct OuterState {
    double *bb;         // [np] |b|^2
    double *rr;         // [np] |b - D x|^2
    int32_t *active;    // [np] still above tolerance
    int32_t *flags;     // [np]
    const int32_t *only;  // [np] or null: pairs with 0 take no part (inactive, x = 0)
};

// Arguments of the persistent GMRES kernel: every pair listed in the queues
// with active[pair] set solves Dhat e = f in the inner precision, e in x.
struct GmArgs {
    const int32_t *h;         // [nb] sites per parity
    const int64_t *soff;      // [nb + 1] site offsets
    const int64_t *nbr_off;   // [nb] neighbour-table offsets
    const int32_t *nbr;
    int nb, n_rhs;
    const void *links;        // inner-precision links
    const void *rhs;          // f: even half field (SP)
    void *x;                  // e: even half field (SP), overwritten
    const int32_t *active;    // [np]
    const int32_t *queue;
    const int32_t *qoff;
    int32_t *qctr;
    int nq;
    void *ws;                 // basis slots: grid x (basis vectors) x vstr elements
    int64_t vstr;             // elements per basis vector (24 * largest h)
    double k2;                // kappa^2
    double tol;               // relative residual of the inner solve
    int m;                    // restart length
    int max_iter;             // Krylov steps per pair and launch
    int resume;               // 0: start from x = 0; 1: continue from x and the paused residual r
    void *r;                  // paused residuals (even half field, SP; may be null)
    const void *z0;           // first flexible direction N(r) (even half field, SP; may be null)
    int max_cycles;           // restart cycles before a pair pauses (0: never pause)
    int32_t *more;            // [np] 1 if the pair paused (may be null)
    double *beta0;            // [np] |f| of each pair (written on a fresh start, read on resume)
    const int32_t *nlinks;    // [nb] links inside each block
    double *bytes;            // [np] += algorithmic bytes moved (may be null)
    int32_t *iters;           // [np] += steps taken
    int32_t *flags;           // [np] |= 4 on a non-finite value
    double *relres;           // [np] last residual estimate / |f| (may be null)
    const int32_t *ext;       // [nb][4] block extents
    int walk;                 // 1: the hops walk the x0-slices (every block admits it)
    double reorth2;           // second Gram-Schmidt pass when |w - V h|^2 <= reorth2 |w|^2
    // with adapt, a pair's tolerance is at least 0.3 tol_out |b| / |r| from the
    // outer state (|b|^2 in obb, the current |r|^2 in orr; at most 0.1)
    int adapt;
    double tol_out;
    const double *obb, *orr;
    const void *clover;       // A^-1 of the clover term (SP, block layout) or null; walking hops only
};

// basis vectors the kernel for restart length m keeps per workgroup (its
// compile-time bound plus one)
int gmres_basis_m(int restart);
hipError_t gmres_occupancy(dd_prec prec, int restart, int nt, bool walk, bool cl, int *wgs_per_cu);
hipError_t launch_gmres(const GmArgs &a, dd_prec prec, int nt, int grid, hipStream_t st);
hipError_t gmres_schedule(dd_ctx *ctx, dd_prec ip, int restart, int np, bool walk, int *nt, int *nq, int *grid);
// whether the persistent GMRES kernel's hops take the x0-walk for these blocks
bool gmres_walk(const dd_ctx *ctx, const dd_blocks *B);

// Extent of the block the network works on (all its blocks have one shape).
struct NnExt {
    int e[4];
    int S;
};

// Pairs of a half field seen as network rows (all blocks of one extent).
struct HalfRows {
    const int32_t *perm;      // eo position -> box-local canonical site
    const int64_t *perm_off;  // [nb]
    const int64_t *soff;      // [nb + 1]
    const int32_t *h;         // [nb]
    int nb, n_rhs, pair0, npairs, S;
};

// launch wrappers of the network (dd_nn.hip); activations are rows [row][channel]
// dir 0: half -> rows (odd sites zero); dir 1: rows -> half_out (even sites)
hipError_t launch_half_rows(const void *half, float *rows, void *half_out, dd_prec sp, const HalfRows &hr, int dir,
                            hipStream_t st);
hipError_t launch_conv(const float *X, const float *W, float *Y, int64_t nrows, const NnExt &e, int cin, int cout,
                       int mode, hipStream_t st);
hipError_t launch_conv_dw(const float *X, const float *dY, float *part, float *dW, int64_t nrows, int nchunk,
                          const NnExt &e, int cin, int cout, int mode, hipStream_t st);
hipError_t launch_relu_grad(const float *dH, const float *Z, float *dZ, int64_t n, hipStream_t st);
hipError_t launch_flip_weights(const float *W, float *Wf, int cin, int cout, hipStream_t st);
hipError_t launch_gather_rows(const double *src, const double *sol, const int64_t *base, const int32_t *idx, float *X,
                              float *T, int n, int S, hipStream_t st);
hipError_t launch_loss(const float *out, const float *T, const int32_t *opar, const int32_t *idx, double *part,
                       double *den, double *loss_acc, float *grad, int n, int mask_even, const NnExt &e,
                       hipStream_t st);
hipError_t launch_adam(float *w, const float *g, float *m, float *v, int64_t n, float lr, float b1, float b2, float eps,
                       int t, hipStream_t st);
// BF16 matrix-core inference: X [rows][32] BF16, Wt [81][32][32] BF16; Y BF16 [rows][32]
// (act applied) or, with out_f32, FP32 [rows][24]
// variant 0: neighbour rows gathered from global memory; 1: one workgroup per
// block walking its x0-slices with three input slices in LDS (rows per slice <= 512)
// (variant 1 skips blocks whose pair pair0 + block index has active[] == 0, when active is given).
// With origin ([nb][4] block origins; pair p is block p % nb), variant 1 uses
// the site parity: parity_mode 1 multiplies only the taps reaching even sites
// (the input must be zero on odd sites), 2 computes only the even output rows.
// parity_mode 3: as 1, with the input read from an even half field (FP32) instead of X;
// 4: as 2, with the output written into the even half field out instead of Y.
struct NnHalfIn {
    const float *half;        // even half field of all pairs (library layout)
    float *out;               // even half field written by the last layer (mode 4)
    const int32_t *perm;      // eo position -> block-local canonical site
    const int64_t *perm_off;  // [nb]
    const int64_t *soff;      // [nb + 1]
    const int32_t *h;         // [nb]
    int n_rhs;
};
hipError_t launch_conv_mfma(const uint16_t *X, const uint16_t *Wt, void *Y, int64_t nrows, const NnExt &e, int act,
                            bool out_f32, int variant, const int32_t *active, int pair0, const int32_t *origin, int nb,
                            int parity_mode, hipStream_t st, const NnHalfIn *hin = nullptr);
hipError_t launch_weights_bf16(const float *W, uint16_t *Wt, int cin, int cout, hipStream_t st);
hipError_t launch_half_rows_bf16(const void *half, uint16_t *rows, dd_prec sp, const HalfRows &hr, hipStream_t st);
hipError_t launch_rows_f32_to_bf16(const float *X, uint16_t *Xb, int64_t nrows, hipStream_t st);

// launch wrappers (dd_kernels.hip)
hipError_t launch_pack_gauge(const dd_blocks *B, const double *U, dd_prec prec, void *dst,
                             hipStream_t s);
hipError_t launch_pack_spinor(const dd_blocks *B, const double *src, void *even, void *odd,
                              dd_prec prec, int n_rhs, hipStream_t s);
hipError_t launch_unpack_spinor(const dd_blocks *B, const void *even, const void *odd, double *dst,
                                dd_prec prec, int n_rhs, hipStream_t s);
hipError_t launch_hop(const BlkArgs &ba, const HopArgs &ha, dd_prec prec, hipStream_t s);
hipError_t launch_hop_walk(const BlkArgs &ba, const WalkArgs &wa, const HopArgs &ha, dd_prec prec, hipStream_t s);
// Dhat = c_self self + c_hop H_eo H_oe in on the even sites (one segment per
// block, ntiles = nb * n_rhs walk tiles); FP32 spinors with FP32 or BF16 links.
hipError_t launch_dhat_walk(const BlkArgs &ba, const WalkArgs &wa, const HopArgs &ha, dd_prec prec, hipStream_t s);
// D_Lambda on both parities in one x0-walk per (block, rhs), FP32 spinors:
// y_p = x_p + c_hop (H x)_p for p = even, odd; x is read once from memory
// (both parities of a slice staged in LDS), its self term again from cache.
struct DlamArgs {
    const int32_t *ext;  // [nb][4] block extents
    int ntiles;          // n_blocks * n_rhs walks, rhs fastest
    const void *xe, *xo;
    void *ye, *yo;
    const void *links;
    double c_hop;
    double *bytes_acc;  // with timing: += bytes_walk per walk done
    double bytes_walk;
};
hipError_t launch_dlam_walk(const BlkArgs &ba, const DlamArgs &da, dd_prec prec, hipStream_t s);
// clover term (dd_clover.hip): A and A^-1 of every block site from the global
// FP64 gauge field U[V][4][3][3] (FP64 out; FP32 copies when a32 != null);
// sites with hole[slot] != 0 (hole may be null) get the identity
hipError_t launch_clover_build(const dd_blocks *B, const double *U, double kappa, double csw, double *a64,
                               double *i64, float *a32, float *i32, const uint8_t *hole, hipStream_t s);
// y = C x on half field `parity` of n_rhs rhs (C: kCloverReals per block site
// in the precision of x; x and y may be the same); pairs whose mask is 0 are
// left alone (mask may be null)
void clover_release(dd_gauge *G);  // frees the clover term of a gauge (back to Wilson)
// ld[2 b], ld[2 b + 1] += ln |det A| and arg det A summed over block b's sites
// (site: scratch of 2 doubles per block site)
hipError_t launch_clover_logdet_add(const dd_blocks *B, const double *a64, double *site, double *ld, hipStream_t s);
hipError_t launch_clover_apply(const dd_blocks *B, const void *C, const void *x, void *y, int parity, int n_rhs,
                               dd_prec sp, const int32_t *mask, hipStream_t s);
hipError_t launch_convert(const void *src, dd_prec sp, void *dst, dd_prec dp, int64_t n,
                          hipStream_t s);
hipError_t launch_accum(const BlkArgs &ba, double *x, const void *e, dd_prec ep,
                        const int32_t *active, hipStream_t s);
// |a|^2 per (tile, rhs) of a half field into partial (slot 0 of kNRed)
hipError_t launch_norm2(const BlkArgs &ba, dd_prec sp, const void *a, double *partial, hipStream_t s);
hipError_t launch_bicg_init(const BlkArgs &ba, dd_prec sp, const void *rhs, void *r, void *rh,
                            void *p, void *x, double *partial, const int32_t *outer_active,
                            hipStream_t s);
hipError_t launch_bicg_s(const BlkArgs &ba, dd_prec sp, const void *r, const void *v, void *s,
                         const PairState &ps, hipStream_t st);
hipError_t launch_bicg_xr(const BlkArgs &ba, dd_prec sp, void *x, const void *p, const void *sx, const void *s,
                          const void *t, void *r, const void *rh, double *partial,
                          const PairState &ps, hipStream_t st);
hipError_t launch_bicg_p(const BlkArgs &ba, dd_prec sp, const void *r, const void *v, void *p,
                         const PairState &ps, hipStream_t st);
// Inner tolerance per pair: tol_in, or with adapt at least
// 0.3 tol_out |b| / |r| (what is left to reach the outer tolerance from the
// current true residual; at most 0.1).
hipError_t launch_sc_init(const BlkArgs &ba, const double *partial, const PairState &ps,
                          const OuterState &os, double tol_in, double tol_out, int adapt, hipStream_t s);
hipError_t launch_sc_alpha(const BlkArgs &ba, const double *partial, const PairState &ps,
                           hipStream_t s);
hipError_t launch_sc_omega(const BlkArgs &ba, const double *partial, const PairState &ps,
                           hipStream_t s);
hipError_t launch_sc_beta(const BlkArgs &ba, const double *partial, const PairState &ps, hipStream_t s);
hipError_t launch_sc_outer(const BlkArgs &ba, const double *pe, const double *po, int first,
                           double tol, const OuterState &os, hipStream_t s);
// dst = src on the pairs with mask set (both [n_rhs][total_sites][24] FP64).
hipError_t launch_merge_pairs(const dd_blocks *B, const double *src, double *dst, const int32_t *mask, int n_rhs,
                              hipStream_t s);
// Network output guard: for every pair p of a half field (n_rhs rhs) with
// active[p] set (active may be null), if z holds a non-finite value, z = v
// (the identity) for that pair and flags[p] |= 16 (flags may be null).
hipError_t launch_nn_guard(const dd_blocks *B, const void *v, void *z, dd_prec sp, int n_rhs, const int32_t *active,
                           int32_t *flags, hipStream_t s);
hipError_t launch_mb_norm(const dd_blocks *B, int n_fields, const double *u, const double *chi,
                          const double *y, double *S, int accumulate, hipStream_t s);
// The links of the exterior hops of B from the canonical field U into uext.
hipError_t launch_gather_ext_links(const dd_blocks *B, const double *U, double *uext, hipStream_t s);
// xi[f][block site] += -kappa * sum of the exterior hops (parts selected by
// the bit mask) of chi[f][exterior site] into that site, for every field.
hipError_t launch_mb_exterior(const dd_blocks *B, const double *uext, double kappa, int n_fields,
                              const double *chi, double *xi, int parts, hipStream_t s);

}  // namespace dd
