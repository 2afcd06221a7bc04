// Internal declarations of libta: device state, compensated arithmetic and
// the kernel launchers used by the solver drivers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ta.h"

namespace ta {

constexpr int kTMax = 8;       // largest CTA order
constexpr int kBlock = 256;    // threads per block of every kernel
#ifndef TA_CHUNK
#define TA_CHUNK 1024
#endif
constexpr int kChunk = TA_CHUNK;  // nnz staged through LDS per round (stream kernel)
constexpr int kMaxColNnz = 8192;  // longest A^T row the transpose sorts in LDS at once

// Internal stop code: the recurrence residual passed the tolerance and the
// host must confirm it on the true residual.
constexpr int kStopCandidate = 100;

// ---------------------------------------------------------------------------
// Solver state, one per call, in device memory.  Only step kernels (one
// block, thread 0) write it; every kernel of a chain reads it at entry.
// ---------------------------------------------------------------------------
struct State {
    int32_t done;      // nonzero: the iteration chain does nothing more
    int32_t stop;      // TA_STOP_* or kStopCandidate
    int32_t t;         // CTA order
    int32_t pivot;     // TA: this iteration takes a step
    int32_t pass;      // TA: next pivot test is passed (radius tie)
    int32_t have_c;    // TA: c = A^T r is current
    int32_t fixed_rho; // TA: Algorithm 2
    int32_t replace;   // a true-residual replacement is due
    int32_t rejected;  // TA: a candidate stop failed, b' = A x must be recomputed
    int32_t hmode;     // CTA: 1 = H = A (A symmetric positive semidefinite), 0 = H = A A^T
    int32_t enhanced;  // CTA: the enhanced stop (first-order iterates tested too)
    int32_t enh_hit;   // CTA: this iteration's update is x^; stop NORMAL after it
    int32_t jump;      // CTA: a convex-combination step follows this update
    int32_t last_jump; // CTA: the current iterate came from one
    int32_t pm;        // matrix passes per operator product: 1, or 2 for TA on the normal
                       // equation (M v = A^T (A v))
    int64_t k;         // iterations done
    int64_t rejects;   // candidate stops the true residual rejected
    int64_t max_iter;
    int64_t hist_cap;
    int64_t matvecs;
    int64_t replace_every;
    double nb;         // ||b||
    double tol, tol_nb;
    double tol_normal, nab, tol_ne_nab;
    double rr;         // ||r||^2 of the current residual
    double rb;         // TA: r^T b
    double nc;         // TA: ||c||
    double gamma;      // TA: rho / ||c||
    double alpha_ta;   // TA: step length
    double rho, rho_lo;
    double rho_max;    // TA: > 0 = witness stop once the radius would exceed it
    double accel;      // CTA: > 0 = convex-combination step threshold on ||r_{k+1}|| / ||r_k||
    double astar;      // CTA: its weight on r_k
    double phi[2 * kTMax + 2];  // phi[1..2t]
    double alpha[kTMax];
    double scratch[4];          // results of kernel-level reductions
};

// What a step kernel does with the values it reduced (v[0], v[1], ...).
enum Post : int32_t {
    kPostNone = 0,
    kPostStore,       // state.scratch[arg + i] = v[i]
    kPostCtaInit,     // v0 = ||b||^2: nb, hist[0], loop-top tests (arg = 1: warm start follows)
    kPostCtaWarm,     // v0 = ||b - A x0||^2 (warm start): rr, hist[0], loop-top tests
    kPostNab,         // v0 = ||A^T b||^2
    kPostGram,        // v[0..2t) = phi_1..phi_2t: normal-equation test and the step alpha
    kPostCtaEnd,      // v0 = ||r||^2 after the update: k, hist, convex-step decision, loop top
    kPostCtaJump,     // v0 = ||r||^2 after a convex-combination step: hist, loop-top tests
    kPostCtaReplace,  // v0 = ||b - A x||^2 after a scheduled replacement (arg: products)
    kPostCtaCand,     // v0 = ||b - A x||^2 at a candidate stop: accept or replace (arg: products)
    kPostTaInit,      // v0 = ||b||^2
    kPostTaC,         // v0 = ||c||^2 (unless c is current): tests, pivot or radius update
    kPostTaS,         // v0 = r^T d, v1 = ||d||^2: alpha
    kPostTaEnd,       // v0 = ||r||^2, v1 = r^T b after the step
    kPostTaCand,      // v0 = ||b - A x||^2 at a candidate stop
    kPostTaBp,        // v0 = ||r||^2, v1 = r^T b after b' = A x
    kPostTaWarm,      // v0 = ||r||^2, v1 = r^T b after b' = A x0 (warm start): hist[0], loop top
};

// Which kernels of a chain run.
enum Gate : int32_t {
    kGateAlways = 0,  // unless done
    kGatePivot,       // unless done, and only when state.pivot
    kGateNeedC,       // producer: unless done or c is current; step: unless done
    kGateReplace,     // unless done, and only when state.replace
    kGateIgnoreDone,  // always (kernel-level calls)
    kGateCandidate,   // only when the chain stopped at a candidate (true-residual check)
    kGateFinal,       // only when the solve has finished (final x, exit diagnostics)
    kGateRejected,    // unless done, and only after a rejected TA candidate
    kGateJump,        // unless done, and only when a convex-combination step is due
};

// Epilogues of the matrix-product kernels.
enum Epi : int32_t {
    kEpiNorm = 0,  // y = v;                         v0 += y^2
    kEpiResid,     // y = b - A x (compensated);     v0 += y^2
    kEpiTaD,       // d = fma(gamma, v, -b');        v0 += r d, v1 += d^2
    kEpiTaBp,      // b' = v, r = b - b';            v0 += r^2, v1 += r b
    kEpiNormDot,   // y = v (square M);              v0 += r y (r: the input), v1 += y^2
    kEpiNormPos,   // y = max(v, 0);                 v0 += y^2
};

struct EpiArgs {
    const double *b;   // kEpiResid, kEpiTaBp
    const double *bp;  // kEpiTaD
    const double *r;   // kEpiTaD, kEpiNormDot
    double *r_out;     // kEpiTaBp
};

constexpr int kMaxSlots = 2 * kTMax + 2;

// Where a producing kernel writes its per-block partial sums: value q of
// block i goes to partials[(slot + q) * cap + i].  No atomics, no fences:
// the step kernel that reads them runs after the producer has finished.
struct Out {
    const State *st;
    double2 *partials;
    int64_t cap;
    int32_t slot;
    int32_t gate;
};

// One-block step kernel: reduce slots slot0 .. slot0 + nslots - 1 (count[i]
// partials each) in a fixed order, then run `post` on the values.
struct Step {
    State *st;
    double *hist;
    const double2 *partials;
    int64_t cap;
    int32_t slot0, nslots;
    int32_t count[kMaxSlots];
    int32_t post, arg, gate;
};

// Device view of a matrix operand for y = M x (M is A or an explicit A^T).
enum MatKind : int32_t {
    kCsrRows = 0,    // CSR: one thread per row (LDS-staged) or `lanes` lanes per row
    kDenseRows = 1,  // dense row-major, rows of M, 64 lanes per row
    kDenseCols = 2,  // dense row-major A viewed as M = A^T: one thread per column of A
    kCsrSliced = 3,  // CSR with columns sorted, split into nsl column slices (8 in flight, one per XCD)
    kCsrSell = 4,    // CSR copied into 64-row slices (SELL-64), one thread per row
    kCsrTiled = 5,   // CSR regrouped by column tiles of kTileW; each tile of x staged in LDS
    kCsrMerge = 6,   // CSR split along the merge path of row ends and nonzeros (skewed rows)
};

constexpr int kSlices = 8;  // XCDs of the part: slices go 8 at a time, slice 8 g + s on XCD s
constexpr int kTileW = 8192;     // columns per tile: 64 KB of FP64 x in LDS, 16-bit local index
constexpr int kTileBlock = 512;  // threads of a tiled block: 2 blocks (16 waves) per CU
// W lanes per row take U entries each per round (W U = 8 slots per row and
// round, U = 1 from W = 8 on); PR row passes go together, within the 128
// registers that keep two blocks on a CU; a block's batch covers
// PR kTileBlock / W rows
constexpr int tile_u(int W) { return W >= 8 ? 1 : 8 / W; }
constexpr int tile_pr(int W) { return W == 1 ? 2 : 4; }
constexpr int tile_batch_rows(int W) { return tile_pr(W) * (kTileBlock / W); }
// kCsrMerge: path items (row ends + nonzeros) per thread and per block
#ifndef TA_MERGE_IPT
#define TA_MERGE_IPT 8
#endif
constexpr int kMergeIpt = TA_MERGE_IPT;
constexpr int kMergeItems = kBlock * kMergeIpt;

struct MatView {
    int32_t kind;
    int64_t rows, cols;  // of M
    int64_t ld;
    const int32_t *rp;
    const int32_t *ci;
    const double *val;
    int32_t lanes;       // kCsrRows: 1 = one thread per row, else lanes per row
    const int32_t *seg;  // kCsrSliced: rows x (nsl + 1) slice starts inside each row
    double2 *ypart;      // kCsrSliced: nsl x rows compensated partial sums (workspace);
                         // kCsrTiled: nt x rows; kCsrMerge: 3 mb (per-block head and carry)
    // kCsrSell: slice s (rows 64 s .. 64 s + 63) holds slots [so[s], so[s + 1]),
    // position k of row 64 s + i at slot so[s] + 64 k + i; a row's entries keep
    // their CSR order, and the slots past its end hold column -1, value 0
    const int64_t *so;
    const int32_t *sc;
    const double *sv;
    // kCsrTiled: the entries of tile q (columns q kTileW .. q kTileW + kTileW - 1)
    // stored tile after tile, rows in order inside a tile; the run of row r in
    // tile q is [rp[q rows + r], rp[q rows + r + 1]), its columns in lc as
    // offsets from the tile start (ascending), its values in val.  A block
    // takes the rows [c rchunk, c rchunk + rchunk) of one tile.
    const uint16_t *lc;
    int32_t nt;       // tiles
    int32_t nchunk;   // row chunks per tile
    int64_t rchunk;   // rows per chunk
    // kCsrMerge: block b of the product takes path items [b kMergeItems,
    // (b + 1) kMergeItems) of the rows + nnz; mp[b] (mb + 1 entries) is the
    // number of rows completed before its first item
    const int32_t *mp;
    int64_t mb;
    // kCsrSell: load the slots with non-temporal loads (set when the plan's
    // copies of A and A^T together outgrow the Infinity Cache, so that the
    // stream does not evict the gathered x; smaller ones are better kept)
    int32_t nt_stream;
    int32_t nsl;  // kCsrSliced: column slices, a multiple of kSlices
};

// ---- launchers (kernels.hip); each returns the grid size it used in *blocks ----
// SELL-64 construction: the widest row of each 64-row slice, then the slots
hipError_t launch_sell_widths(int64_t rows, const int32_t *rp, int32_t *w, hipStream_t s);
hipError_t launch_sell_fill(int64_t rows, const int32_t *rp, const int32_t *ci, const double *val,
                            const int64_t *so, int32_t *sc, double *sv, hipStream_t s);
hipError_t launch_matvec(const MatView &M, const double *x, double *y, int32_t epi,
                         const EpiArgs &ea, const Out &o, hipStream_t s, int32_t *blocks);
hipError_t launch_cta_init(int64_t m, const double *b, double *r, double *xy, int64_t nxy,
                           int32_t zero_xy, const Out &o, hipStream_t s, int32_t *blocks);
// rb, yb (optional): the residual and the updated iterate (y, or x) before
// the update, for a convex-combination step
hipError_t launch_cta_update(int64_t m, int64_t n, int32_t t, int32_t minnorm, double *r,
                             double *const *u, double *x, double *const *w, double *y,
                             double *rb, double *yb, const Out &o, hipStream_t s,
                             int32_t *blocks);
// r = a rb + (1 - a) r, xy = a xyb + (1 - a) xy with a = state.astar (gate
// kGateJump); v0 = ||r||^2
hipError_t launch_cta_jump(int64_t m, int64_t nxy, double *r, const double *rb, double *xy,
                           const double *xyb, const Out &o, hipStream_t s, int32_t *blocks);
hipError_t launch_ta_init(int64_t m, int64_t n, const double *b, double *r, double *bp,
                          double *x, int32_t keep_x, const Out &o, hipStream_t s,
                          int32_t *blocks);
hipError_t launch_ta_update(int64_t m, int64_t n, const double *b, double *bp, const double *d,
                            double *r, double *x, const double *c, const Out &o, hipStream_t s,
                            int32_t *blocks);
hipError_t launch_step(const Step &sp, hipStream_t s);
// dst (n x m, row stride ldd) = src^T (m x n, row stride lds), FP64
hipError_t launch_dense_transpose(int64_t m, int64_t n, const double *src, int64_t lds,
                                  double *dst, int64_t ldd, hipStream_t s);
// *d = h, from a kernel argument
hipError_t launch_state_set(State *d, const State &h, hipStream_t s);
hipError_t launch_check_csr(int64_t m, int64_t n, int64_t nnz, const int32_t *rp,
                            const int32_t *ci, int32_t *flag, hipStream_t s);
hipError_t launch_slice_segments(int64_t m, const int32_t *rp, const int32_t *ci_sorted,
                                 int64_t cols, int32_t nsl, int32_t *seg, hipStream_t s);
// Tile-major copy of a CSR whose columns are sorted inside each row (the
// kCsrTiled layout): trp (nt rows + 1), lc and tval (nnz each).  work:
// nt rows + cdiv(nt rows, 1024) + 8 int32 entries.
hipError_t launch_tile_build(int64_t rows, int64_t cols, const int32_t *rp, const int32_t *ci_sorted,
                             const double *val_sorted, int32_t *trp, uint16_t *lc, double *tval,
                             int32_t *work, hipStream_t s);
// kCsrMerge partition: mp[b] for b = 0 .. mb
hipError_t launch_merge_part(int64_t rows, const int32_t *rp, int64_t mb, int32_t *mp,
                             hipStream_t s);
// out[0] = max(out[0], longest row of the CSR rp); out must hold a value <= 0 first
hipError_t launch_row_max(int64_t rows, const int32_t *rp, int32_t *out, hipStream_t s);
hipError_t launch_norm2(int64_t n, const double *x, const Out &o, hipStream_t s,
                        int32_t *blocks);
hipError_t launch_csr_outer(int64_t m, const int32_t *rp, const int32_t *ci, const double *u,
                            const double *v, double alpha, double *out, hipStream_t s);
// Canonical CSR of A^T.  flag (one int32) is cleared and stays zero: every
// CSR that passes validation is handled (the callers' check of it remains).
hipError_t launch_transpose(int64_t m, int64_t n, int64_t nnz, const int32_t *rp,
                            const int32_t *ci, const double *val, int32_t *at_rp,
                            int32_t *at_ci, double *at_val, int32_t *work, int32_t *flag,
                            hipStream_t s);

int64_t matvec_blocks(const MatView &M);
int64_t elementwise_blocks(int64_t n);

}  // namespace ta
