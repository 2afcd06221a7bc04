// Host side of libta: argument checks, workspace, the iteration chains of
// CTA (Algorithm 1, H = A A^T) and TA (Algorithms 2 and 3), and the C ABI.
//
// A solve enqueues chunks of iterations; every kernel of a chain reads the
// device State first and does nothing once the solve has stopped, so the
// only device-to-host traffic inside the loop is one small State read per
// chunk.  A candidate stop (recurrence residual below tolerance) is confirmed
// on the true FP64 residual before the solve ends, as in the oracle.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <initializer_list>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "common.hpp"
#include "host.hpp"

namespace ta {

// pinned host copy of the State, one per host thread
static State *host_state() {
    static thread_local State *h = nullptr;
    if (h == nullptr) {
        if (hipHostMalloc(reinterpret_cast<void **>(&h), sizeof(State)) != hipSuccess) h = nullptr;
    }
    return h;
}

// noalloc: into `out` directly (pageable host memory, no pinned buffer)
static int read_state(State *d, State &out, hipStream_t s, bool noalloc = false) {
    if (noalloc) {
        HIP_TRY(hipMemcpyAsync(&out, d, sizeof(State), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        return TA_OK;
    }
    State *h = host_state();
    if (h == nullptr) return hip_fail(hipErrorOutOfMemory, "hipHostMalloc");
    HIP_TRY(hipMemcpyAsync(h, d, sizeof(State), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    out = *h;
    return TA_OK;
}

// ---------------------------------------------------------------------------
// validation
// ---------------------------------------------------------------------------
static int validate_opts(const ta_mat *A, const ta_opts *o, int solver) {
    if (o == nullptr) return TA_EINVAL;
    if (!(o->tol >= 0.0 && o->tol < 1.0)) return TA_EINVAL;
    if (!(o->tol_normal >= 0.0 && o->tol_normal < 1.0)) return TA_EINVAL;
    if (o->max_iter < 0 || o->replace_every < 0 || o->chunk < 0) return TA_EINVAL;
    if (o->launch_mode != 0 && o->launch_mode != 1) return TA_EINVAL;
    if (o->h_mode != 0 && o->h_mode != 1) return TA_EINVAL;
    if (o->h_mode == 1 && (solver != 0 || A->m != A->n)) return TA_EINVAL;
    if (o->t_cycle != 0 && (o->t_cycle != 1 || solver == 2)) return TA_EINVAL;
    if (o->nonneg != 0 && (o->nonneg != 1 || solver != 2)) return TA_EINVAL;
    if (o->enhanced != 0 && (o->enhanced != 1 || solver == 2)) return TA_EINVAL;
    if (o->normal_eq != 0 && (o->normal_eq != 1 || solver != 2)) return TA_EINVAL;
    if (!(o->accel >= 0.0 && o->accel < 1.0) || (o->accel > 0.0 && solver == 2))
        return TA_EINVAL;
    if (!(o->rho_max >= 0.0) || !isfinite(o->rho_max) || (o->rho_max > 0.0 && solver != 2))
        return TA_EINVAL;
    // FP32 / BF16 products: one-shot CTA only (run on the batched engine, which
    // refines in FP64 at fixed chunk ends), without the per-iteration options
    if (o->precision != TA_FP64) {
        if (o->precision != TA_FP32 && o->precision != TA_BF16) return TA_EINVAL;
        if (solver != 0 && solver != 1) return TA_EINVAL;
        if (o->warm_start || o->replace_every || o->h_mode || o->t_cycle || o->enhanced ||
            o->accel != 0.0)
            return TA_EINVAL;
    }
    if (solver == 0 || solver == 1) {
        if (o->t < 1 || o->t > kTMax) return TA_EINVAL;
        if (A->m > 0 && o->t > A->m) return TA_EINVAL;
        if (solver == 1 && o->warm_start) return TA_EINVAL;
    } else if (solver == 2) {
        if (!(o->rho0 >= 0.0) || !isfinite(o->rho0)) return TA_EINVAL;
        if (o->fixed_rho && !(o->rho0 > 0.0)) return TA_EINVAL;
    } else {
        return TA_EINVAL;
    }
    return TA_OK;
}

// ---------------------------------------------------------------------------
// operator: views of A and A^T
// ---------------------------------------------------------------------------
static int pick_lanes(int64_t nnz, int64_t rows) {
    const double avg = rows > 0 ? (double)nnz / (double)rows : 0.0;
    if (avg <= 16.0) return 1;
    if (avg <= 32.0) return 8;
    if (avg <= 64.0) return 16;
    if (avg <= 128.0) return 32;
    return 64;
}

// Matrices whose rows hold more nonzeros than 16 per row, on average, get
// lanes-per-row kernels.  With at least kTileMinCols columns and runs of at
// least kTileMinRun entries per (column tile, row) on average they are
// regrouped by column tiles whose x is staged in LDS; otherwise, with at
// least kSliceMinCols columns, they are split into XCD column slices so the
// gathered x stays in L2.  (The tiles trade one L2 request per nonzero for
// a partial sum per (tile, row): they pay while the runs are long enough.)
constexpr int64_t kSliceMinCols = 1 << 17;
constexpr int64_t kTileMinCols = 2 * kTileW;
constexpr int64_t kTileMinRun = 3;
#ifndef TA_TILE_BLOCKS
#define TA_TILE_BLOCKS 2048
#endif

static int64_t n_tiles(int64_t cols) { return (cols + kTileW - 1) / kTileW; }

// A CSR view whose longest row holds at least kMergeMinRow nonzeros is split
// along the merge path when that row holds at least kMergeSkew times the
// average (skewed rows: before column tiles or slices, whose lanes per row
// are chosen from the average too), or, where neither tiles nor slices take
// it, when the row kernels (one thread or a fixed number of lanes per row)
// would run fewer than kMergeMinBlocks blocks and the path more (a few long
// rows leave most of the chip idle).
#ifndef TA_MERGE_SKEW
#define TA_MERGE_SKEW 32
#endif
constexpr int64_t kMergeSkew = TA_MERGE_SKEW;
constexpr int64_t kMergeMinRow = 512;
constexpr int64_t kMergeMinBlocks = 512;

static int64_t merge_blocks(int64_t rows, int64_t nnz) {
    return std::max<int64_t>(1, (rows + nnz + kMergeItems - 1) / kMergeItems);
}

static bool skewed(int64_t rows, int64_t nnz, int64_t longest) {
    return rows > 0 && longest >= kMergeMinRow && longest * rows >= kMergeSkew * nnz;
}

static bool use_merge(int64_t rows, int64_t nnz, int64_t longest, int lanes) {
    if (rows <= 0 || longest < kMergeMinRow) return false;
    if (skewed(rows, nnz, longest)) return true;
    const int64_t row_blocks = (rows * std::max(lanes, 1) + kBlock - 1) / kBlock;
    return row_blocks < kMergeMinBlocks && merge_blocks(rows, nnz) > row_blocks;
}

static int pick_slice_lanes(int64_t nnz, int64_t rows, int32_t nsl);

// Column slices per operand: 8 g (g a power of two) so that one slice of x
// takes at most TA_SLICE_BYTES.  Measured on the LP shape's A pass (600
// random columns per row): n = 1e7, 8 slices of 10 MB 747 us, 16 of 5 MB
// 626 us, 32 759 us, 64 884 us (more slices add a partial sum and a segment
// bound per row and slice); n = 4e6, 8 slices of 4 MB 206 us, 16 235 us.
#ifndef TA_SLICE_BYTES
#define TA_SLICE_BYTES (8 << 20)
#endif
static int32_t n_slices(int64_t cols) {
    int32_t g = 1;
    while (g < 64 && 8 * cols > (int64_t)kSlices * g * TA_SLICE_BYTES) g *= 2;
    return kSlices * g;
}

static bool use_tiles(int64_t nnz, int64_t rows, int64_t cols) {
    if (rows <= 0 || cols < kTileMinCols) return false;
    const int64_t runs = n_tiles(cols) * rows;
    return runs * kTileMinRun <= nnz && runs < (int64_t(1) << 30);
}

// Lanes per row for the tiled kernel (the fewest, from 2, with 4 W at least
// the average run; W = 2 puts a run of up to 8 entries in one round), and
// the row chunks: about TA_TILE_BLOCKS blocks in all (measured
// on the 10000 x 1e6 LP shape: 2048 blocks of one or two batches beat 1024
// or 4096), each chunk a whole number of the block's batches.
static MatView tiled_view(int64_t rows, int64_t cols, int64_t nnz, const int32_t *trp,
                          const uint16_t *lc, const double *tval) {
    const int64_t nt = n_tiles(cols);
    const double run = (double)nnz / (double)(nt * rows);
#ifdef TA_TILE_LANES
    const int W = TA_TILE_LANES;
#else
    int W = 2;
    while (W < 64 && 4.0 * W < run) W *= 2;
#endif
    const int64_t G = tile_batch_rows(W);
    int64_t nchunk = std::max<int64_t>(1, (TA_TILE_BLOCKS + nt - 1) / nt);
    nchunk = std::min(nchunk, (rows + G - 1) / G);
    int64_t rchunk = (rows + nchunk - 1) / nchunk;
    rchunk = (rchunk + G - 1) / G * G;
    nchunk = (rows + rchunk - 1) / rchunk;
    MatView v{kCsrTiled, rows, cols, 0, trp, nullptr, tval, W, nullptr, nullptr};
    v.lc = lc;
    v.nt = (int32_t)nt;
    v.nchunk = (int32_t)nchunk;
    v.rchunk = rchunk;
    return v;
}

// A regrouped layout with fewer than kRegroupMinBlocks blocks leaves most of
// the chip idle; the merge path then takes the operand when it has more
// (measured: 600 rows of 9000 entries over 20000 columns, 57 tiled blocks,
// 67.7 us tiled against 33.8 us on the merge path; 64 rows of 2e5 entries
// over 1e6 columns, 246 tiled blocks, 42.8 us against 92.6 us).
constexpr int64_t kRegroupMinBlocks = 128;

static int64_t tiled_blocks(int64_t rows, int64_t cols, int64_t nnz) {
    const MatView v = tiled_view(rows, cols, nnz, nullptr, nullptr, nullptr);
    return (int64_t)v.nt * v.nchunk;
}

// ---------------------------------------------------------------------------
// Plan: a prepared operator.  Holds A^T (canonical CSR built on the device)
// and, for long-row matrices, a column-sorted copy of A with its slice
// table.  Immutable after creation, so one plan can serve calls on several
// streams at once; per-call scratch lives in each call's workspace.
// ---------------------------------------------------------------------------
// Lanes per row for the sliced kernel, from the nonzeros per (row, slice).
static int pick_slice_lanes(int64_t nnz, int64_t rows, int32_t nsl) {
#ifdef TA_SLICE_LANES
    return TA_SLICE_LANES;
#endif
    const double avg = rows > 0 ? (double)nnz / (double)rows / nsl : 0.0;
    if (avg <= 32.0) return 4;
    if (avg <= 64.0) return 8;
    if (avg <= 128.0) return 16;
    if (avg <= 256.0) return 32;
    return 64;
}

struct Plan {
    ta_mat desc{};
    MatView A{}, AT{};
    bool has_t = false;
    void *mem = nullptr;
    void *mem_sell = nullptr;   // SELL-64 copies of the views that take them
    void *mem_merge = nullptr;  // merge-path partitions of the views that take them
    hipStream_t s_mem = nullptr;
};

static void plan_free(Plan *P) {
    if (P->mem != nullptr) (void)hipFreeAsync(P->mem, P->s_mem);
    if (P->mem_sell != nullptr) (void)hipFreeAsync(P->mem_sell, P->s_mem);
    if (P->mem_merge != nullptr) (void)hipFreeAsync(P->mem_merge, P->s_mem);
    P->mem = nullptr;
    P->mem_sell = nullptr;
    P->mem_merge = nullptr;
}

// Merge-path partitions for the CSR views that the row kernels would take
// and use_merge selects (A's longest row is known from the validation; A^T's
// is measured on the device and read back).
static int plan_merge(Plan *P, int64_t nnz, int64_t longest_a, hipStream_t s) {
    MatView *vs[2] = {&P->A, P->has_t ? &P->AT : nullptr};
    bool cand[2] = {false, false};
    for (int i = 0; i < 2; ++i)
        cand[i] = vs[i] != nullptr && vs[i]->kind == kCsrRows && vs[i]->rows > 0;
    if ((!cand[0] && !cand[1]) || nnz < kMergeMinRow) return TA_OK;
    int rc = TA_OK;
    int64_t longest[2] = {longest_a, 0};
    if (cand[1]) {
        Workspace wt(s);
        int32_t *dmax = nullptr;
        wt.reserve(&dmax, 1);
        if ((rc = wt.commit()) != TA_OK) return rc;
        HIP_TRY(hipMemsetAsync(dmax, 0, sizeof(int32_t), s));
        HIP_TRY(launch_row_max(vs[1]->rows, vs[1]->rp, dmax, s));
        int32_t h = 0;
        HIP_TRY(hipMemcpyAsync(&h, dmax, sizeof(h), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        longest[1] = h;
    }
    bool use[2] = {false, false};
    int64_t mb[2] = {0, 0};
    for (int i = 0; i < 2; ++i) {
        use[i] = cand[i] && use_merge(vs[i]->rows, nnz, longest[i], vs[i]->lanes);
        if (use[i]) mb[i] = merge_blocks(vs[i]->rows, nnz);
    }
    if (!use[0] && !use[1]) return TA_OK;
    Workspace mw(s);
    int32_t *mp[2] = {nullptr, nullptr};
    for (int i = 0; i < 2; ++i)
        if (use[i]) mw.reserve(&mp[i], mb[i] + 1);
    if ((rc = mw.commit()) != TA_OK) return rc;
    for (int i = 0; i < 2; ++i)
        if (use[i]) {
            HIP_TRY(launch_merge_part(vs[i]->rows, vs[i]->rp, mb[i], mp[i], s));
            vs[i]->kind = kCsrMerge;
            vs[i]->mp = mp[i];
            vs[i]->mb = mb[i];
        }
    P->mem_merge = mw.release();
    return TA_OK;
}

// The MI355X's Infinity Cache (MALL) in front of HBM
constexpr int64_t kInfinityCacheBytes = int64_t(256) << 20;

// SELL-64 copies for the one-thread-per-row CSR views whose 64-row slices
// pad the entries by at most a quarter (rows of even length: stencils,
// banded and degree-bounded sparse matrices).  Widths come back to the host
// for the slice offsets; the slots are filled on the device.  Plans whose A
// and A^T together outgrow the Infinity Cache stream the slots with
// non-temporal loads (measured on the 2896^2 Poisson matrix: 135 -> 123 us;
// on the 1e4 x 1e6 LP shape's A^T, 144 MB with A, they made 27 -> 35 us).

static int plan_sell(Plan *P, int64_t nnz, hipStream_t s) {
    MatView *vs[2] = {&P->A, P->has_t ? &P->AT : nullptr};
    int64_t nsl[2] = {0, 0};
    for (int i = 0; i < 2; ++i)
        if (vs[i] != nullptr && vs[i]->kind == kCsrRows && vs[i]->lanes == 1 && vs[i]->rows > 0)
            nsl[i] = (vs[i]->rows + 63) / 64;
    if (nsl[0] + nsl[1] == 0 || nnz <= 0) return TA_OK;
    Workspace wt(s);
    int32_t *dw = nullptr;
    wt.reserve(&dw, nsl[0] + nsl[1]);
    int rc = wt.commit();
    if (rc != TA_OK) return rc;
    for (int i = 0; i < 2; ++i)
        if (nsl[i] > 0) HIP_TRY(launch_sell_widths(vs[i]->rows, vs[i]->rp, dw + (i ? nsl[0] : 0), s));
    std::vector<int32_t> hw((size_t)(nsl[0] + nsl[1]));
    HIP_TRY(hipMemcpyAsync(hw.data(), dw, sizeof(int32_t) * hw.size(), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    std::vector<int64_t> so[2];
    bool use[2] = {false, false};
    for (int i = 0; i < 2; ++i) {
        if (nsl[i] == 0) continue;
        so[i].assign((size_t)nsl[i] + 1, 0);
        for (int64_t q = 0; q < nsl[i]; ++q)
            so[i][q + 1] = so[i][q] + 64 * (int64_t)hw[(size_t)((i ? nsl[0] : 0) + q)];
        use[i] = so[i][nsl[i]] <= nnz + nnz / 4;
    }
    if (!use[0] && !use[1]) return TA_OK;
    Workspace sw(s);
    int64_t *d_so[2] = {nullptr, nullptr};
    int32_t *d_sc[2] = {nullptr, nullptr};
    double *d_sv[2] = {nullptr, nullptr};
    for (int i = 0; i < 2; ++i)
        if (use[i]) {
            sw.reserve(&d_so[i], nsl[i] + 1);
            sw.reserve(&d_sc[i], so[i][nsl[i]]);
            sw.reserve(&d_sv[i], so[i][nsl[i]]);
        }
    if ((rc = sw.commit()) != TA_OK) return rc;
    for (int i = 0; i < 2; ++i)
        if (use[i]) {
            HIP_TRY(hipMemcpyAsync(d_so[i], so[i].data(), sizeof(int64_t) * so[i].size(),
                                   hipMemcpyHostToDevice, s));
            HIP_TRY(launch_sell_fill(vs[i]->rows, vs[i]->rp, vs[i]->ci, vs[i]->val, d_so[i],
                                     d_sc[i], d_sv[i], s));
            vs[i]->kind = kCsrSell;
            vs[i]->nt_stream = 2 * 12 * nnz > kInfinityCacheBytes;
            vs[i]->so = d_so[i];
            vs[i]->sc = d_sc[i];
            vs[i]->sv = d_sv[i];
        }
    HIP_TRY(hipStreamSynchronize(s));  // the host offsets are read before they go
    P->mem_sell = sw.release();
    return TA_OK;
}

// sell: also build SELL-64 copies (plans and solves; not the one-shot
// products, which would spend more on the copy than they save)
static int plan_build(const ta_mat *M, bool need_t, hipStream_t s, Plan *P, bool sell = false) {
    Range trace("ta:prepare");
    int rc = validate_mat(M);
    if (rc != TA_OK) return rc;
    P->desc = *M;
    const int64_t m = M->m, n = M->n;
    P->has_t = need_t;
    if (M->kind == TA_DENSE_ROWMAJOR) {
        // A^T as a row-major copy, so that both products run 64 lanes per row
        // (the column view of A, one thread per column of A, leaves most of
        // the chip idle on a few hundred columns)
        P->A = MatView{kDenseRows, m, n, M->ld, nullptr, nullptr, M->val, 64, nullptr, nullptr};
        P->AT = MatView{kDenseCols, n, m, M->ld, nullptr, nullptr, M->val, 1, nullptr, nullptr};
        P->has_t = true;
        if (m > 0 && n > 0 && need_t && (m + 31) / 32 <= 65535) {
            Workspace own(s);
            double *at = nullptr;
            own.reserve(&at, n * m);
            if ((rc = own.commit()) != TA_OK) return rc;
            HIP_TRY(launch_dense_transpose(m, n, M->val, M->ld, at, m, s));
            P->AT = MatView{kDenseRows, n, m, m, nullptr, nullptr, at, 64, nullptr, nullptr};
            P->mem = own.release();
            P->s_mem = s;
        }
        return TA_OK;
    }
    const int64_t nnz = M->nnz;
    // validation, and A's longest row (one read back)
    int64_t longest_a = 0;
    {
        Workspace probe(s);
        int32_t *pflag = nullptr;
        probe.reserve(&pflag, 2);
        if ((rc = probe.commit()) != TA_OK) return rc;
        if ((rc = check_csr_longest(M, pflag, &longest_a, s)) != TA_OK) return rc;
    }
    const int la = pick_lanes(nnz, m), lt = pick_lanes(nnz, n);
    // A is regrouped from (A^T)^T, except for skewed rows (the merge path
    // takes them)
    const bool regroup_a = need_t && la > 1 && !skewed(m, nnz, longest_a);
    // blocks of the regrouped layout, and whether the merge path should take
    // the operand instead (for A^T: its average row already holds
    // kMergeMinRow, so its longest does)
    auto starved = [&](int64_t rows, int64_t cols, bool tiled) {
        const int32_t nsl = n_slices(cols);
        const int64_t per = kBlock / pick_slice_lanes(nnz, rows, nsl);  // rows per sliced block
        const int64_t blocks =
            tiled ? tiled_blocks(rows, cols, nnz) : nsl * ((rows + per - 1) / per);
        return blocks < kRegroupMinBlocks && merge_blocks(rows, nnz) > blocks;
    };
    bool tile_a = regroup_a && use_tiles(nnz, m, n);
    bool slice_a = regroup_a && !tile_a && n >= kSliceMinCols;
    if ((tile_a || slice_a) && longest_a >= kMergeMinRow && starved(m, n, tile_a))
        tile_a = slice_a = false;
    bool tile_t = need_t && lt > 1 && use_tiles(nnz, n, m);
    bool slice_t = need_t && lt > 1 && !tile_t && m >= kSliceMinCols;
    if ((tile_t || slice_t) && nnz >= kMergeMinRow * n && starved(n, m, tile_t))
        tile_t = slice_t = false;

    // owned memory
    Workspace own(s);
    int32_t *at_rp = nullptr, *at_ci = nullptr, *ac_ci = nullptr, *a_seg = nullptr,
            *t_seg = nullptr, *a_trp = nullptr, *t_trp = nullptr;
    double *at_val = nullptr, *ac_val = nullptr, *a_tv = nullptr, *t_tv = nullptr;
    uint16_t *a_lc = nullptr, *t_lc = nullptr;
    if (need_t) {
        own.reserve(&at_rp, n + 1);
        own.reserve(&at_ci, nnz);
        own.reserve(&at_val, nnz);
    }
    if (slice_a) {
        own.reserve(&ac_ci, nnz);
        own.reserve(&ac_val, nnz);
        own.reserve(&a_seg, m * (n_slices(n) + 1));
    }
    if (slice_t) own.reserve(&t_seg, n * (n_slices(m) + 1));
    if (tile_a) {
        own.reserve(&a_trp, n_tiles(n) * m + 1);
        own.reserve(&a_lc, nnz);
        own.reserve(&a_tv, nnz);
    }
    if (tile_t) {
        own.reserve(&t_trp, n_tiles(m) * n + 1);
        own.reserve(&t_lc, nnz);
        own.reserve(&t_tv, nnz);
    }
    // temporary memory (a tiled A takes its column-sorted copy from here)
    Workspace tmp(s);
    int32_t *flag = nullptr, *work = nullptr, *ac_rp = nullptr;
    const int64_t mx = std::max(m, n);
    const int64_t ntiles = (std::max<int64_t>(mx, 1) + 1023) / 1024;
    int64_t runs = 0;
    if (tile_a) runs = std::max(runs, n_tiles(n) * m);
    if (tile_t) runs = std::max(runs, n_tiles(m) * n);
    tmp.reserve(&flag, 8);
    if (need_t)
        tmp.reserve(&work, std::max(2 * mx + ntiles + 8 + nnz, runs + (runs + 1023) / 1024 + 8));
    if (slice_a || tile_a) tmp.reserve(&ac_rp, m + 1);
    if (tile_a) {
        tmp.reserve(&ac_ci, nnz);
        tmp.reserve(&ac_val, nnz);
    }
    if ((rc = own.commit()) != TA_OK) return rc;
    if ((rc = tmp.commit()) != TA_OK) return rc;

    P->A = MatView{kCsrRows, m, n, 0, M->row_ptr, M->col_idx, M->val, la, nullptr, nullptr};
    if (need_t) {
        HIP_TRY(launch_transpose(m, n, nnz, M->row_ptr, M->col_idx, M->val, at_rp, at_ci, at_val,
                                 work, flag, s));
        P->AT = MatView{kCsrRows, n, m, 0, at_rp, at_ci, at_val, lt, nullptr, nullptr};
        if (slice_a || tile_a) {
            // (A^T)^T: A with columns sorted inside each row
            HIP_TRY(launch_transpose(n, m, nnz, at_rp, at_ci, at_val, ac_rp, ac_ci, ac_val, work,
                                     flag, s));
        }
        if (slice_a) {
            const int32_t nsl = n_slices(n);
            HIP_TRY(launch_slice_segments(m, M->row_ptr, ac_ci, n, nsl, a_seg, s));
            P->A = MatView{kCsrSliced, m, n, 0, M->row_ptr, ac_ci, ac_val,
                           pick_slice_lanes(nnz, m, nsl), a_seg, nullptr};
            P->A.nsl = nsl;
        }
        if (tile_a) {
            HIP_TRY(launch_tile_build(m, n, ac_rp, ac_ci, ac_val, a_trp, a_lc, a_tv, work, s));
            P->A = tiled_view(m, n, nnz, a_trp, a_lc, a_tv);
        }
        if (slice_t) {
            const int32_t nsl = n_slices(m);
            HIP_TRY(launch_slice_segments(n, at_rp, at_ci, m, nsl, t_seg, s));
            P->AT = MatView{kCsrSliced, n, m, 0, at_rp, at_ci, at_val,
                            pick_slice_lanes(nnz, n, nsl), t_seg, nullptr};
            P->AT.nsl = nsl;
        }
        if (tile_t) {
            HIP_TRY(launch_tile_build(n, m, at_rp, at_ci, at_val, t_trp, t_lc, t_tv, work, s));
            P->AT = tiled_view(n, m, nnz, t_trp, t_lc, t_tv);
        }
        int32_t h = 0;
        HIP_TRY(hipMemcpyAsync(&h, flag, sizeof(int32_t), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        if (h) return TA_ENOTSUP;
    }
    P->mem = own.release();
    P->s_mem = s;
    if ((rc = plan_merge(P, nnz, longest_a, s)) != TA_OK) return rc;
    if (sell) return plan_sell(P, nnz, s);
    return TA_OK;
}

// Per-call launch helper: producers write into slots of `partials`, step
// kernels reduce them.  Views carry this call's slice scratch.
struct Chain {
    State *st = nullptr;
    double *hist = nullptr;
    double2 *partials = nullptr;
    int64_t cap = 0;  // partials per slot
    hipStream_t s = nullptr;
    MatView A{}, AT{};

    // reserve the per-call pieces every chain needs
    void reserve(Workspace &ws, const Plan &P, int32_t nslots) {
        A = P.A;
        AT = P.AT;
        cap = std::max(matvec_blocks(P.A), elementwise_blocks(std::max(P.desc.m, P.desc.n)));
        if (P.has_t) cap = std::max(cap, matvec_blocks(P.AT));
        cap = std::max<int64_t>(cap, 1);
        ws.reserve(&st, 1);
        ws.reserve(&partials, (int64_t)nslots * cap);
        if (A.kind == kCsrSliced) ws.reserve(&A.ypart, (int64_t)A.nsl * std::max<int64_t>(A.rows, 1));
        if (P.has_t && AT.kind == kCsrSliced)
            ws.reserve(&AT.ypart, (int64_t)AT.nsl * std::max<int64_t>(AT.rows, 1));
        if (A.kind == kCsrTiled) ws.reserve(&A.ypart, (int64_t)A.nt * std::max<int64_t>(A.rows, 1));
        if (P.has_t && AT.kind == kCsrTiled)
            ws.reserve(&AT.ypart, (int64_t)AT.nt * std::max<int64_t>(AT.rows, 1));
        if (A.kind == kCsrMerge) ws.reserve(&A.ypart, 3 * A.mb);
        if (P.has_t && AT.kind == kCsrMerge) ws.reserve(&AT.ypart, 3 * AT.mb);
    }
    Out out(int32_t slot, int32_t gate) const {
        Out o;
        o.st = st;
        o.partials = partials;
        o.cap = cap;
        o.slot = slot;
        o.gate = gate;
        return o;
    }
    hipError_t step(int32_t slot0, std::initializer_list<int32_t> counts, int32_t post, int32_t arg,
                    int32_t gate, bool with_hist = true) const {
        Step sp;
        memset(&sp, 0, sizeof sp);
        sp.st = st;
        sp.hist = with_hist ? hist : nullptr;
        sp.partials = partials;
        sp.cap = cap;
        sp.slot0 = slot0;
        sp.nslots = (int32_t)counts.size();
        int i = 0;
        for (int32_t c : counts) sp.count[i++] = c;
        sp.post = post;
        sp.arg = arg;
        sp.gate = gate;
        return launch_step(sp, s);
    }
};

static State initial_state(const ta_opts *o, int64_t hist_cap, double *hist) {
    State h;
    memset(&h, 0, sizeof h);
    h.t = o->t;
    h.max_iter = o->max_iter;
    h.hist_cap = hist != nullptr ? hist_cap : 0;
    h.replace_every = o->replace_every;
    h.tol = o->tol;
    h.tol_normal = o->tol_normal;
    h.rho = o->rho0;
    h.fixed_rho = o->fixed_rho;
    h.hmode = o->h_mode;
    h.rho_max = o->rho_max;
    h.enhanced = o->enhanced;
    h.accel = o->accel;
    h.pm = 1;
    return h;
}

// One State upload from a pinned buffer of its own.  Every solve ends with a
// synchronising State read, so when the next solve of this host thread
// starts, the previous upload from the buffer has completed.
static int upload_state(State *d, const State &h, hipStream_t s, bool noalloc = false) {
    if (noalloc) {  // from a kernel argument: no pinned staging buffer
        HIP_TRY(launch_state_set(d, h, s));
        return TA_OK;
    }
    static thread_local State *up = nullptr;
    if (up == nullptr &&
        hipHostMalloc(reinterpret_cast<void **>(&up), sizeof(State)) != hipSuccess) {
        up = nullptr;
        return hip_fail(hipErrorOutOfMemory, "hipHostMalloc");
    }
    *up = h;
    HIP_TRY(hipMemcpyAsync(d, up, sizeof(State), hipMemcpyHostToDevice, s));
    return TA_OK;
}

// Exit diagnostics, enqueued behind every chunk and run only once the solve
// has finished: ||b - A x||^2, ||A^T (b - A x)||^2 and ||A^T b||^2 of the
// final x into State.scratch[0..2].
// with_nb: also ||b||^2 into State.scratch[3] (TA on the normal equation,
// whose State.nb is ||A^T b||); needs a fourth partials slot.
static hipError_t enqueue_exit_diagnostics(const Chain &c, const double *b, const double *x,
                                           double *tmp_m, double *tmp_n, bool with_nb = false) {
    EpiArgs ea{};
    ea.b = b;
    int32_t g0 = 0, g1 = 0, g2 = 0, g3 = 0;
    hipError_t e;
    if ((e = launch_matvec(c.A, x, tmp_m, kEpiResid, ea, c.out(0, kGateFinal), c.s, &g0)) !=
        hipSuccess)
        return e;
    if ((e = launch_matvec(c.AT, tmp_m, tmp_n, kEpiNorm, EpiArgs{}, c.out(1, kGateFinal), c.s,
                           &g1)) != hipSuccess)
        return e;
    if ((e = launch_matvec(c.AT, b, tmp_n, kEpiNorm, EpiArgs{}, c.out(2, kGateFinal), c.s, &g2)) !=
        hipSuccess)
        return e;
    if (!with_nb) return c.step(0, {g0, g1, g2}, kPostStore, 0, kGateFinal, false);
    if ((e = launch_norm2(c.A.rows, b, c.out(3, kGateFinal), c.s, &g3)) != hipSuccess) return e;
    return c.step(0, {g0, g1, g2, g3}, kPostStore, 0, kGateFinal, false);
}

// nb_scratch: ||b|| is in State.scratch[3] rather than State.nb
static void fill_diagnostics(const State &h, ta_info *info, bool nb_scratch = false) {
    const double nb = nb_scratch ? sqrt(h.scratch[3]) : h.nb;
    info->rel_res = nb > 0.0 ? sqrt(h.scratch[0]) / nb : 0.0;
    const double nab = sqrt(h.scratch[2]);
    info->rel_normal = (nb > 0.0 && nab > 0.0) ? sqrt(h.scratch[1]) / nab : 0.0;
}

static void fill_info(const State &h, ta_info *info) {
    info->iters = h.k;
    info->matvecs = h.matvecs;
    info->stop = h.stop;
    info->rho = h.rho;
    info->rho_lo = h.rho_lo;
}

// Chunk schedule: short chunks first (small solves stop early), then longer.
struct Chunker {
    int64_t next;
    int64_t cap;
    explicit Chunker(int32_t fixed) : next(fixed > 0 ? fixed : 4), cap(fixed > 0 ? fixed : 64) {}
    int64_t take() {
        const int64_t c = next;
        next = std::min(cap, next * 2);
        return c;
    }
};

static int check_solve_args(const ta_mat *M, const double *b, double *x, const ta_opts *o,
                            double *hist, int64_t hist_cap, ta_info *info, int solver) {
    if (info == nullptr) return TA_EINVAL;
    memset(info, 0, sizeof *info);
    int rc = validate_mat(M);
    if (rc == TA_OK) rc = validate_opts(M, o, solver);
    if (rc != TA_OK) return rc;
    if ((M->m > 0 && b == nullptr) || (M->n > 0 && x == nullptr)) return TA_EINVAL;
    if (hist != nullptr && hist_cap < 0) return TA_EINVAL;
    return TA_OK;
}

// Empty system (m = 0, so b = 0): x = 0 at once.
static int solve_empty(const ta_mat *M, double *x, double *hist, int64_t hist_cap, ta_info *info,
                       double rho0, hipStream_t s) {
    if (M->n > 0) HIP_TRY(hipMemsetAsync(x, 0, sizeof(double) * (size_t)M->n, s));
    if (hist != nullptr && hist_cap > 0) HIP_TRY(hipMemsetAsync(hist, 0, sizeof(double), s));
    HIP_TRY(hipStreamSynchronize(s));
    info->stop = TA_STOP_RESIDUAL;
    info->rho = rho0;
    return TA_OK;
}

// Chunks of a chain captured once as HIP graphs and replayed.  Every kernel
// of a chain takes its state from device memory (State, vectors, partials)
// and its launch arguments are fixed for the whole solve, so a replay does
// exactly the work of the launches it was captured from; a chunk's launches
// depend only on its length and on whether candidate checks follow every
// iteration (the key).  Not used with order cycling (the order of each
// iteration depends on its index) or by the no-allocation entry point
// (instantiating a graph allocates).
struct ChunkGraphs {
    hipStream_t cap = nullptr;
    std::vector<std::pair<int64_t, hipGraphExec_t>> ex;
    ChunkGraphs() = default;
    ChunkGraphs(const ChunkGraphs &) = delete;
    ChunkGraphs &operator=(const ChunkGraphs &) = delete;
    ~ChunkGraphs() {
        for (auto &e : ex) (void)hipGraphExecDestroy(e.second);
        if (cap != nullptr) (void)hipStreamDestroy(cap);
    }
};

// Enqueue one chunk on s: body() enqueues on c.s; with g, it runs once on a
// capture stream for each key and the graph is launched on s.
template <class F>
static int enqueue_chunk(ChunkGraphs *g, int64_t key, Chain &c, hipStream_t s, F &&body) {
    c.s = s;
    if (g == nullptr) return body();
    hipGraphExec_t ge = nullptr;
    for (auto &e : g->ex)
        if (e.first == key) ge = e.second;
    if (ge == nullptr) {
        if (g->cap == nullptr) HIP_TRY(hipStreamCreateWithFlags(&g->cap, hipStreamNonBlocking));
        c.s = g->cap;
        HIP_TRY(hipStreamBeginCapture(g->cap, hipStreamCaptureModeThreadLocal));
        const int rc = body();
        hipGraph_t gr = nullptr;
        const hipError_t ce = hipStreamEndCapture(g->cap, &gr);
        c.s = s;
        if (rc != TA_OK || ce != hipSuccess) {
            if (gr != nullptr) (void)hipGraphDestroy(gr);
            return rc != TA_OK ? rc : hip_fail(ce, "hipStreamEndCapture");
        }
        const hipError_t ie = hipGraphInstantiate(&ge, gr, nullptr, nullptr, 0);
        (void)hipGraphDestroy(gr);
        HIP_TRY(ie);
        g->ex.emplace_back(key, ge);
    }
    HIP_TRY(hipGraphLaunch(ge, s));
    return TA_OK;
}

// Host loop guard shared by the chains.  Every chunk either finishes the
// solve or advances the iteration count, except a chunk that ends on a
// candidate check right at its start (the next chunk then runs at least one
// iteration, since a rejected candidate is not re-tested before the next
// step).  Two chunks in a row without progress therefore mean a broken
// chain: the call returns an error instead of polling forever.
struct Progress {
    int64_t k_last = -1;
    int stalls = 0;
    bool stalled(const State &h) {
        stalls = h.k == k_last ? stalls + 1 : 0;
        k_last = h.k;
        return stalls >= 2;
    }
};

// ---------------------------------------------------------------------------
// CTA (x-form and y-form)
// ---------------------------------------------------------------------------
// ext, ext_cap: a caller-held device buffer to carve the workspace from
// (cta_solve_plan_noalloc); nullptr = allocate stream-ordered
static int cta_run(const Plan &P, const double *b, double *x, const ta_opts *o, double *hist,
                   int64_t hist_cap, ta_info *info, hipStream_t s, bool minnorm,
                   void *ext = nullptr, size_t ext_cap = 0) {
    const ta_mat *M = &P.desc;
    int rc = check_solve_args(M, b, x, o, hist, hist_cap, info, minnorm ? 1 : 0);
    if (rc != TA_OK) return rc;
    if (!P.has_t || o->precision != TA_FP64) return TA_EINVAL;  // a plan holds FP64 only
    const int64_t m = M->m, n = M->n;
    const int t = o->t;
    if (m == 0) return solve_empty(M, x, hist, hist_cap, info, 0.0, s);

    const bool noalloc = ext != nullptr;
    Workspace ws = noalloc ? Workspace(s, ext, ext_cap) : Workspace(s);
    Chain c;
    c.s = s;
    c.hist = hist;
    c.reserve(ws, P, 2 * t + 1);
    // H = A (A square, symmetric positive semidefinite): the chain u_{j+1} =
    // A u_j alone, phi_{2j+1} = u_j^T u_{j+1}, phi_{2j+2} = ||u_{j+1}||^2, and
    // x += sum_i alpha_i u_{i-1} (the y-form update applied to x)
    const bool ha = o->h_mode == 1;
    double *r = nullptr, *y = nullptr, *tmp_n = nullptr;
    double *u[kTMax + 1] = {}, *w[kTMax] = {};
    ws.reserve(&r, m);
    for (int j = 1; j <= t; ++j) ws.reserve(&u[j], m);
    const int nw = ha ? 0 : (minnorm ? 1 : t);
    for (int j = 0; j < nw; ++j) ws.reserve(&w[j], n);
    if (minnorm) ws.reserve(&y, m);
    ws.reserve(&tmp_n, n);
    // convex-combination step: the residual and the updated iterate (y, or x)
    // before each update
    const bool acc = o->accel > 0.0;
    const int64_t nupd = minnorm ? m : n;
    double *rb = nullptr, *xyb = nullptr;
    if (acc) {
        ws.reserve(&rb, m);
        ws.reserve(&xyb, nupd);
    }
    if ((rc = ws.commit()) != TA_OK) return rc;

    State h0 = initial_state(o, hist_cap, hist);
    if ((rc = upload_state(c.st, h0, s, noalloc)) != TA_OK) return rc;
    u[0] = r;
    double *const xy = minnorm ? y : x;
    const int64_t nxy = minnorm ? m : n;
    const bool warm = o->warm_start && !minnorm;
    const int32_t R = 2 * t;  // slot of ||r||^2
    const int32_t products = minnorm ? 2 : 1;
    int32_t g = 0, gr = 0;

    // initial state: r = b, x = 0 (or y = 0), ||b||
    HIP_TRY(launch_cta_init(m, b, r, xy, nxy, warm ? 0 : 1, c.out(R, kGateAlways), s, &g));
    HIP_TRY(c.step(R, {g}, kPostCtaInit, warm ? 1 : 0, kGateAlways));
    if (o->tol_normal > 0.0) {
        HIP_TRY(launch_matvec(c.AT, b, tmp_n, kEpiNorm, EpiArgs{}, c.out(0, kGateAlways), s, &g));
        HIP_TRY(c.step(0, {g}, kPostNab, 0, kGateAlways));
    }
    EpiArgs eres{};
    eres.b = b;
    if (warm) {
        HIP_TRY(launch_matvec(c.A, x, r, kEpiResid, eres, c.out(R, kGateAlways), s, &g));
        HIP_TRY(c.step(R, {g}, kPostCtaWarm, 0, kGateAlways));
    }

    int32_t gphi[2 * kTMax] = {};
    // order of the iteration with index k: t, or the cycle 1, 2, ..., t, ..., 2
    auto order_of = [&](int64_t k) -> int {
        if (!o->t_cycle || t <= 1) return t;
        const int64_t p = k % (2 * (int64_t)t - 2);
        return (int)(p < t ? p + 1 : 2 * (int64_t)t - 1 - p);
    };
    auto enqueue_iteration = [&](int tk) -> int {
        for (int j = 0; j < tk; ++j) {
            if (ha) {
                EpiArgs ed{};
                ed.r = u[j];
                HIP_TRY(launch_matvec(c.A, u[j], u[j + 1], kEpiNormDot, ed,
                                      c.out(2 * j, kGateAlways), c.s, &gphi[2 * j]));
                gphi[2 * j + 1] = gphi[2 * j];
                continue;
            }
            double *wj = w[minnorm ? 0 : j];
            HIP_TRY(launch_matvec(c.AT, u[j], wj, kEpiNorm, EpiArgs{}, c.out(2 * j, kGateAlways), c.s,
                                  &gphi[2 * j]));
            HIP_TRY(launch_matvec(c.A, wj, u[j + 1], kEpiNorm, EpiArgs{},
                                  c.out(2 * j + 1, kGateAlways), c.s, &gphi[2 * j + 1]));
        }
        Step sp;
        memset(&sp, 0, sizeof sp);
        sp.st = c.st;
        sp.partials = c.partials;
        sp.cap = c.cap;
        sp.slot0 = 0;
        sp.nslots = 2 * tk;
        for (int i = 0; i < 2 * tk; ++i) sp.count[i] = gphi[i];
        sp.post = kPostGram;
        sp.arg = tk;
        sp.gate = kGateAlways;
        HIP_TRY(launch_step(sp, c.s));
        HIP_TRY(launch_cta_update(m, n, tk, (minnorm || ha) ? 1 : 0, r, u, x, w, ha ? x : y,
                                  rb, xyb, c.out(R, kGateAlways), c.s, &g));
        HIP_TRY(c.step(R, {g}, kPostCtaEnd, 0, kGateAlways));
        if (acc) {
            int32_t gj = 0;
            HIP_TRY(launch_cta_jump(m, nupd, r, rb, minnorm ? y : x, xyb, c.out(R, kGateJump), c.s,
                                    &gj));
            HIP_TRY(c.step(R, {gj}, kPostCtaJump, 0, kGateJump));
        }
        if (o->replace_every > 0) {
            if (minnorm)
                HIP_TRY(launch_matvec(c.AT, y, x, kEpiNorm, EpiArgs{}, c.out(0, kGateReplace), c.s,
                                      nullptr));
            HIP_TRY(launch_matvec(c.A, x, r, kEpiResid, eres, c.out(R, kGateReplace), c.s, &gr));
            HIP_TRY(c.step(R, {gr}, kPostCtaReplace, products, kGateReplace));
        }
        return TA_OK;
    };

    // the candidate check (runs only if the chain stopped at a candidate):
    // x = A^T y in the y-form, then the true residual, accepted or taken as
    // the new recurrence residual
    auto enqueue_check = [&]() -> int {
        if (minnorm)
            HIP_TRY(launch_matvec(c.AT, y, x, kEpiNorm, EpiArgs{}, c.out(0, kGateCandidate), c.s,
                                  nullptr));
        HIP_TRY(launch_matvec(c.A, x, r, kEpiResid, eres, c.out(R, kGateCandidate), c.s, &g));
        HIP_TRY(c.step(R, {g}, kPostCtaCand, products, kGateCandidate));
        return TA_OK;
    };

    // Each chunk: k iterations, then a candidate check, then the final x and
    // the exit diagnostics (run only once the solve has finished).  One State
    // read per chunk.  After the first rejected candidate the recurrence is
    // near the true residual's floor, where candidates can come every
    // iteration: from then on each iteration is followed by the (gated)
    // check, so no chunk stalls on one.
    Chunker ch(o->chunk);
    State h;
    Progress prog;
    ChunkGraphs graphs;
    const bool use_graphs = o->launch_mode == 0 && !noalloc && !o->t_cycle;
    bool inline_checks = false;
    int64_t k_done = 0;  // iterations done when the chunk starts
    for (int64_t chunk_no = 0;; ++chunk_no) {
        const int64_t k = ch.take();
        Range trace("cta:chunk");
        auto body = [&]() -> int {
            for (int64_t i = 0; i < k; ++i) {
                // the order of an iteration is its index's; a chunk that runs
                // into a candidate resumes the schedule from the state's count
                int rb2 = enqueue_iteration(order_of(k_done + i));
                if (rb2 != TA_OK) return rb2;
                if (inline_checks && (rb2 = enqueue_check()) != TA_OK) return rb2;
            }
            int rb3 = TA_OK;
            if (!inline_checks && (rb3 = enqueue_check()) != TA_OK) return rb3;
            if (minnorm)
                HIP_TRY(launch_matvec(c.AT, y, x, kEpiNorm, EpiArgs{}, c.out(0, kGateFinal), c.s,
                                      nullptr));
            HIP_TRY(enqueue_exit_diagnostics(c, b, x, r, tmp_n));
            return TA_OK;
        };
        // the first chunk runs as plain launches (a solve that stops in it
        // pays no capture), later ones from graphs
        if ((rc = enqueue_chunk(use_graphs && chunk_no > 0 ? &graphs : nullptr,
                                2 * k + (inline_checks ? 1 : 0), c, s, body)) != TA_OK)
            return rc;
        if ((rc = read_state(c.st, h, s, noalloc)) != TA_OK) return rc;
        if (h.done && h.stop != kStopCandidate) break;
        k_done = h.k;
        inline_checks = inline_checks || h.rejects > 0;
        if (prog.stalled(h)) {
            hip_msg() = "CTA iteration chain made no progress";
            return TA_EHIP;
        }
    }
    fill_info(h, info);
    if (h.nb == 0.0) {
        HIP_TRY(hipMemsetAsync(x, 0, sizeof(double) * (size_t)n, s));
        HIP_TRY(hipStreamSynchronize(s));
    } else {
        fill_diagnostics(h, info);
    }
    return TA_OK;
}

// ---------------------------------------------------------------------------
// TA (Algorithm 3, or Algorithm 2 with a fixed radius), on A x = b or on the
// normal equation A^T A x = A^T b
// ---------------------------------------------------------------------------
static int ta_run(const Plan &P, const double *b, double *x, const ta_opts *o, double *hist,
                  int64_t hist_cap, ta_info *info, hipStream_t s) {
    const ta_mat *M = &P.desc;
    int rc = check_solve_args(M, b, x, o, hist, hist_cap, info, 2);
    if (rc != TA_OK) return rc;
    if (!P.has_t) return TA_EINVAL;
    const int64_t m = M->m, n = M->n;
    if (m == 0) return solve_empty(M, x, hist, hist_cap, info, o->rho0, s);
    // normal equation: the operator is A^T A (n x n, symmetric), applied as
    // A^T t with t = A v rounded to FP64; the right-hand side is A^T b
    const bool ne = o->normal_eq == 1;
    const int64_t mo = ne ? n : m;  // rows of the operator

    Workspace ws(s);
    Chain c;
    c.s = s;
    c.hist = hist;
    c.reserve(ws, P, 6);  // slot 5: sink for the partial sums of inner passes
    double *r = nullptr, *bp = nullptr, *cv = nullptr, *d = nullptr, *rt = nullptr,
           *tA = nullptr, *bt = nullptr;
    ws.reserve(&r, mo);
    ws.reserve(&bp, mo);
    ws.reserve(&d, mo);
    ws.reserve(&rt, mo);
    ws.reserve(&cv, n);
    ws.reserve(&tA, m);
    if (ne) ws.reserve(&bt, n);
    if ((rc = ws.commit()) != TA_OK) return rc;

    State h0 = initial_state(o, hist_cap, hist);
    h0.pm = ne ? 2 : 1;
    h0.matvecs = ne ? 1 : 0;  // A^T b
    if ((rc = upload_state(c.st, h0, s)) != TA_OK) return rc;
    int32_t g = 0;
    // y = Op v with the epilogue of the outer pass (gate and slot of `out`)
    auto op_apply = [&](const double *v, double *y, int32_t epi, const EpiArgs &ea, const Out &out,
                        int32_t *blocks) -> hipError_t {
        if (!ne) return launch_matvec(c.A, v, y, epi, ea, out, c.s, blocks);
        Out inner = out;
        inner.slot = 5;
        hipError_t e = launch_matvec(c.A, v, tA, kEpiNorm, EpiArgs{}, inner, c.s, nullptr);
        if (e != hipSuccess) return e;
        return launch_matvec(c.AT, tA, y, epi, ea, out, c.s, blocks);
    };
    // y = Op^T v (Op^T = Op on the normal equation)
    auto op_apply_t = [&](const double *v, double *y, int32_t epi, const Out &out,
                          int32_t *blocks) -> hipError_t {
        if (!ne) return launch_matvec(c.AT, v, y, epi, EpiArgs{}, out, c.s, blocks);
        return op_apply(v, y, epi, EpiArgs{}, out, blocks);
    };
    const double *be = b;  // the right-hand side the iteration works on
    if (ne) {
        HIP_TRY(launch_matvec(c.AT, b, bt, kEpiNorm, EpiArgs{}, c.out(5, kGateAlways), c.s, nullptr));
        be = bt;
    }
    // slots: 0 ||c||^2; 1, 2: r^T d, ||d||^2; 3, 4: ||r||^2, r^T b
    const int32_t warm = o->warm_start ? 1 : 0;
    HIP_TRY(launch_ta_init(mo, n, be, r, bp, x, warm, c.out(3, kGateAlways), c.s, &g));
    HIP_TRY(c.step(3, {g}, kPostTaInit, warm, kGateAlways));
    // LP feasibility (x >= 0): c = A^T r is replaced by its positive part
    const int32_t epi_c = o->nonneg ? kEpiNormPos : kEpiNorm;
    if (o->tol_normal > 0.0) {
        HIP_TRY(op_apply_t(be, cv, epi_c, c.out(0, kGateAlways), &g));
        HIP_TRY(c.step(0, {g}, kPostNab, 0, kGateAlways));
    }
    EpiArgs ebp{};
    ebp.b = be;
    ebp.r_out = r;
    if (warm) {  // b' = A x0, r = b - b'
        HIP_TRY(op_apply(x, bp, kEpiTaBp, ebp, c.out(3, kGateAlways), &g));
        HIP_TRY(c.step(3, {g, g}, kPostTaWarm, 0, kGateAlways));
    }

    EpiArgs ed{};
    ed.bp = bp;
    ed.r = r;
    auto enqueue_iteration = [&]() -> int {
        HIP_TRY(op_apply_t(r, cv, epi_c, c.out(0, kGateNeedC), &g));
        HIP_TRY(c.step(0, {g}, kPostTaC, 0, kGateNeedC));
        HIP_TRY(op_apply(cv, d, kEpiTaD, ed, c.out(1, kGatePivot), &g));
        HIP_TRY(c.step(1, {g, g}, kPostTaS, 0, kGatePivot));
        HIP_TRY(launch_ta_update(mo, n, be, bp, d, r, x, cv, c.out(3, kGatePivot), c.s, &g));
        HIP_TRY(c.step(3, {g, g}, kPostTaEnd, 0, kGatePivot));
        return TA_OK;
    };
    EpiArgs eres{};
    eres.b = be;
    // the candidate check (true residual; on the normal equation
    // A^T b - A^T (A x) as one compensated sum per entry) and, after a
    // rejection, b' = Op x and r = b - b'; both run only when due
    auto enqueue_check = [&]() -> int {
        int32_t gc = 0, gb = 0;
        HIP_TRY(op_apply(x, rt, kEpiResid, eres, c.out(3, kGateCandidate), &gc));
        HIP_TRY(c.step(3, {gc}, kPostTaCand, 0, kGateCandidate));
        HIP_TRY(op_apply(x, bp, kEpiTaBp, ebp, c.out(3, kGateRejected), &gb));
        HIP_TRY(c.step(3, {gb, gb}, kPostTaBp, 0, kGateRejected));
        return TA_OK;
    };

    // Once a candidate has been rejected the recurrence runs close to the
    // true residual's floor, where candidates can come every iteration; from
    // then on every iteration is followed by the (gated) check, so a chunk
    // never stalls on one.
    Chunker ch(o->chunk);
    State h;
    Progress prog;
    ChunkGraphs graphs;
    const bool use_graphs = o->launch_mode == 0;
    bool inline_checks = false;
    for (int64_t chunk_no = 0;; ++chunk_no) {
        const int64_t k = ch.take();
        Range trace("ta:chunk");
        auto body = [&]() -> int {
            for (int64_t i = 0; i < k; ++i) {
                int rb2 = enqueue_iteration();
                if (rb2 != TA_OK) return rb2;
                if (inline_checks && (rb2 = enqueue_check()) != TA_OK) return rb2;
            }
            int rb3 = TA_OK;
            if (!inline_checks && (rb3 = enqueue_check()) != TA_OK) return rb3;
            HIP_TRY(enqueue_exit_diagnostics(c, b, x, tA, cv, ne));
            return TA_OK;
        };
        if ((rc = enqueue_chunk(use_graphs && chunk_no > 0 ? &graphs : nullptr,
                                2 * k + (inline_checks ? 1 : 0), c, s, body)) != TA_OK)
            return rc;
        if ((rc = read_state(c.st, h, s)) != TA_OK) return rc;
        if (h.done && h.stop != kStopCandidate) break;
        inline_checks = inline_checks || h.rejects > 0;
        if (prog.stalled(h)) {
            hip_msg() = "TA iteration chain made no progress";
            return TA_EHIP;
        }
    }
    if (warm && h.nb == 0.0) HIP_TRY(hipMemsetAsync(x, 0, sizeof(double) * (size_t)n, s));
    fill_info(h, info);
    if (h.nb > 0.0) fill_diagnostics(h, info, ne);
    return TA_OK;
}

// ---------------------------------------------------------------------------
// Algorithm 4 (section 4.4): approximate minimum-norm solution from an
// approximate solution x_eps, by bisection on the radius of E_{A, rho}
// ---------------------------------------------------------------------------
// ||v|| as one compensated sum (device), read back to the host.
static int device_norm(Chain &c, int64_t n, const double *v, double *out, hipStream_t s) {
    *out = 0.0;
    if (n <= 0) return TA_OK;
    HIP_TRY(hipMemsetAsync(c.st, 0, sizeof(State), s));
    int32_t g = 0;
    HIP_TRY(launch_norm2(n, v, c.out(0, kGateIgnoreDone), s, &g));
    HIP_TRY(c.step(0, {g}, kPostStore, 0, kGateIgnoreDone, false));
    State h;
    int rc = read_state(c.st, h, s);
    if (rc != TA_OK) return rc;
    *out = sqrt(h.scratch[0]);
    return TA_OK;
}

// Upper bound hi = ||x_eps||, lower bound lo = 0; each test runs Algorithm 2
// (fixed radius rho = (hi + lo) / 2) from the last witness's x (0 before the
// first): an approximate solution in the ball lowers hi to rho and is kept,
// a witness raises lo to its Corollary 1 bound.  Stops when hi - lo <= tol
// ||x_eps||, when a test ends on the normal equation (its x is returned), or
// when the iteration budget (summed over the tests) runs out; crossed bounds
// (lo - hi beyond the gap) mean the input was no approximate solution of a
// consistent system: witness stop, x = the last solution found or x_eps.
static int minnorm_run(const Plan &P, const double *b, const double *x_eps, double *x,
                       const ta_opts *o, ta_info *info, int64_t *tests_out, hipStream_t s) {
    const ta_mat *M = &P.desc;
    int rc = check_solve_args(M, b, x, o, nullptr, 0, info, 2);
    if (rc != TA_OK) return rc;
    if (!P.has_t) return TA_EINVAL;
    const int64_t m = M->m, n = M->n;
    if (n > 0 && x_eps == nullptr) return TA_EINVAL;
    if (o->nonneg || o->rho_max > 0.0) return TA_EINVAL;  // Algorithm 4 is stated without the cone
    if (tests_out != nullptr) *tests_out = 0;
    if (m == 0 || n == 0) {
        if (n > 0) HIP_TRY(hipMemsetAsync(x, 0, sizeof(double) * (size_t)n, s));
        HIP_TRY(hipStreamSynchronize(s));
        info->stop = TA_STOP_RESIDUAL;
        return TA_OK;
    }
    Workspace ws(s);
    Chain c;
    c.s = s;
    c.reserve(ws, P, 1);
    double *xt = nullptr, *xw = nullptr;
    ws.reserve(&xt, n);
    ws.reserve(&xw, n);
    if ((rc = ws.commit()) != TA_OK) return rc;
    double nb = 0.0, hi = 0.0, lo = 0.0;
    if ((rc = device_norm(c, m, b, &nb, s)) != TA_OK) return rc;
    if ((rc = device_norm(c, n, x_eps, &hi, s)) != TA_OK) return rc;
    const double gap = o->tol * hi;
    HIP_TRY(hipMemcpyAsync(x, x_eps, sizeof(double) * (size_t)n, hipMemcpyDeviceToDevice, s));
    if (nb == 0.0) {
        HIP_TRY(hipMemsetAsync(x, 0, sizeof(double) * (size_t)n, s));
        hi = 0.0;
    }
    int32_t stop = TA_STOP_RESIDUAL;
    bool have_w = false;
    int64_t tests = 0, iters = 0, matvecs = 0;
    while (nb > 0.0 && hi - lo > gap) {
        if (iters >= o->max_iter) {
            stop = TA_STOP_MAXITER;
            break;
        }
        ta_opts t = *o;
        t.fixed_rho = 1;
        t.rho0 = 0.5 * (hi + lo);
        t.warm_start = have_w ? 1 : 0;
        t.max_iter = o->max_iter - iters;
        if (have_w)
            HIP_TRY(hipMemcpyAsync(xt, xw, sizeof(double) * (size_t)n, hipMemcpyDeviceToDevice, s));
        ta_info ti;
        if ((rc = ta_run(P, b, xt, &t, nullptr, 0, &ti, s)) != TA_OK) return rc;
        ++tests;
        iters += ti.iters;
        matvecs += ti.matvecs;
        if (ti.stop == TA_STOP_RESIDUAL) {
            hi = t.rho0;
            HIP_TRY(hipMemcpyAsync(x, xt, sizeof(double) * (size_t)n, hipMemcpyDeviceToDevice, s));
        } else if (ti.stop == TA_STOP_WITNESS) {
            lo = ti.rho_lo;
            HIP_TRY(hipMemcpyAsync(xw, xt, sizeof(double) * (size_t)n, hipMemcpyDeviceToDevice, s));
            have_w = true;
        } else {
            if (ti.stop == TA_STOP_NORMAL)
                HIP_TRY(hipMemcpyAsync(x, xt, sizeof(double) * (size_t)n, hipMemcpyDeviceToDevice,
                                       s));
            stop = ti.stop;
            break;
        }
    }
    if (stop == TA_STOP_RESIDUAL && lo - hi > gap) stop = TA_STOP_WITNESS;
    // diagnostics of the returned x (not counted): a TA start from x with no iteration
    if (nb > 0.0) {
        ta_opts d = *o;
        d.fixed_rho = 0;
        d.rho0 = 0.0;
        d.warm_start = 1;
        d.max_iter = 0;
        HIP_TRY(hipMemcpyAsync(xt, x, sizeof(double) * (size_t)n, hipMemcpyDeviceToDevice, s));
        ta_info di;
        if ((rc = ta_run(P, b, xt, &d, nullptr, 0, &di, s)) != TA_OK) return rc;
        info->rel_res = di.rel_res;
        info->rel_normal = di.rel_normal;
    }
    HIP_TRY(hipStreamSynchronize(s));
    info->iters = iters;
    info->matvecs = matvecs;
    info->stop = stop;
    info->rho = hi;
    info->rho_lo = lo;
    if (tests_out != nullptr) *tests_out = tests;
    return TA_OK;
}

// ---------------------------------------------------------------------------
// kernel-level entry points
// ---------------------------------------------------------------------------
static int product_run(const Plan &P, int32_t trans, const double *x, double *y, const double *b,
                       double *norm2, hipStream_t s) {
    const ta_mat *M = &P.desc;
    const int64_t rows = trans ? M->n : M->m, cols = trans ? M->m : M->n;
    if ((cols > 0 && x == nullptr) || (rows > 0 && y == nullptr)) return TA_EINVAL;
    if (trans && !P.has_t) return TA_EINVAL;
    if (rows == 0) {
        if (norm2 != nullptr) HIP_TRY(hipMemsetAsync(norm2, 0, sizeof(double), s));
        return TA_OK;
    }
    Workspace ws(s);
    Chain c;
    c.s = s;
    c.reserve(ws, P, 1);
    int rc = ws.commit();
    if (rc != TA_OK) return rc;
    HIP_TRY(hipMemsetAsync(c.st, 0, sizeof(State), s));
    EpiArgs ea{};
    ea.b = b;
    const MatView &V = trans ? c.AT : c.A;
    int32_t g = 0;
    HIP_TRY(launch_matvec(V, x, y, b != nullptr ? kEpiResid : kEpiNorm, ea,
                          c.out(0, kGateIgnoreDone), s, &g));
    HIP_TRY(c.step(0, {g}, kPostStore, 0, kGateIgnoreDone, false));
    if (norm2 != nullptr)
        HIP_TRY(hipMemcpyAsync(norm2, &c.st->scratch[0], sizeof(double), hipMemcpyDeviceToDevice, s));
    return TA_OK;
}

// Average duration of one launch of the product kernel(s) the solvers use
// for y = A x (trans = 0) or y = A^T x (trans = 1), over `reps` back-to-back
// launches bracketed by HIP events on `s`.
static int time_run(const Plan &P, int32_t trans, const double *x, double *y, int32_t reps,
                    double *avg_ms, hipStream_t s) {
    if (reps < 1 || avg_ms == nullptr || x == nullptr || y == nullptr) return TA_EINVAL;
    if (trans && !P.has_t) return TA_EINVAL;
    Workspace ws(s);
    Chain c;
    c.s = s;
    c.reserve(ws, P, 1);
    int rc = ws.commit();
    if (rc != TA_OK) return rc;
    HIP_TRY(hipMemsetAsync(c.st, 0, sizeof(State), s));
    const MatView &V = trans ? c.AT : c.A;
    const Out out = c.out(0, kGateIgnoreDone);
    HIP_TRY(launch_matvec(V, x, y, kEpiNorm, EpiArgs{}, out, s, nullptr));  // warm-up
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    HIP_TRY(hipEventRecord(e0, s));
    for (int32_t i = 0; i < reps; ++i)
        HIP_TRY(launch_matvec(V, x, y, kEpiNorm, EpiArgs{}, out, s, nullptr));
    HIP_TRY(hipEventRecord(e1, s));
    HIP_TRY(hipEventSynchronize(e1));
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    *avg_ms = (double)ms / reps;
    return TA_OK;
}

// One-shot calls: a transient plan on the call's stream.
template <class F>
static int with_plan(const ta_mat *M, bool need_t, hipStream_t s, F &&f, bool sell = false) {
    Plan P;
    int rc = plan_build(M, need_t, s, &P, sell);
    if (rc == TA_OK) rc = f(P);
    plan_free(&P);
    return rc;
}

// ---------------------------------------------------------------------------
// Fixed device buffer of cta_solve_plan_noalloc: one copy on every GPU the
// library is loaded on, held until the process ends.  In host code the name
// `scratch` is a host-side stand-in, never a device address: each device's
// address comes from hipGetSymbolAddress, taken once with that device
// current, and only that address is passed on.
// ---------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[TA_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;

static int scratch_address(void **out) {
    static std::mutex mu;
    static void *addr[kMaxDevices] = {};
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return TA_EINVAL;
    std::lock_guard<std::mutex> lock(mu);
    if (addr[dev] == nullptr) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        if (p == nullptr) return hip_fail(hipErrorInvalidSymbol, "hipGetSymbolAddress(scratch)");
        addr[dev] = p;
    }
    *out = addr[dev];
    return TA_OK;
}

}  // namespace ta

struct ta_plan {
    ta::Plan p;
};

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

#define HIP_TRY_C(call)                                        \
    do {                                                       \
        hipError_t e_ = (call);                                \
        if (e_ != hipSuccess) return ta::hip_fail(e_, #call);  \
    } while (0)

// FP32 / BF16 products for one system: the batched engine on a one-system
// plan with one right-hand side (x stays FP64; no history is written).
static int cta_mixed_one(const ta_mat *A, const double *b, double *x, const ta_opts *opts,
                         ta_info *info, void *stream, int32_t minnorm) {
    if (A->m == 0 || A->n == 0) {  // nothing to iterate: x = 0
        hipStream_t s = (hipStream_t)stream;
        if (A->n > 0) HIP_TRY_C(hipMemsetAsync(x, 0, sizeof(double) * (size_t)A->n, s));
        HIP_TRY_C(hipStreamSynchronize(s));
        info->stop = TA_STOP_RESIDUAL;
        return TA_OK;
    }
    ta_batch_plan *bp = nullptr;
    int rc = ta_batch_plan_create(1, A, opts->precision, &bp, stream);
    if (rc != TA_OK) return rc;
    const int32_t k = 1;
    const double *B[1] = {b};
    double *X[1] = {x};
    rc = cta_solve_batched(bp, &k, B, X, opts, minnorm, info, stream);
    const int rd = ta_batch_plan_destroy(bp);
    return rc != TA_OK ? rc : rd;
}

int cta_solve(const ta_mat *A, const double *b, double *x, const ta_opts *opts, double *hist,
              int64_t hist_cap, ta_info *info, void *stream) {
    hipStream_t s = (hipStream_t)stream;
    if (info == nullptr) return TA_EINVAL;
    int rc = ta::check_solve_args(A, b, x, opts, hist, hist_cap, info, 0);
    if (rc != TA_OK) return rc;
    if (opts->precision != TA_FP64) return cta_mixed_one(A, b, x, opts, info, stream, 0);
    return ta::with_plan(A, true, s, [&](const ta::Plan &P) {
        return ta::cta_run(P, b, x, opts, hist, hist_cap, info, s, false);
    }, true);
}

int cta_minnorm(const ta_mat *A, const double *b, double *x, const ta_opts *opts, double *hist,
                int64_t hist_cap, ta_info *info, void *stream) {
    hipStream_t s = (hipStream_t)stream;
    if (info == nullptr) return TA_EINVAL;
    int rc = ta::check_solve_args(A, b, x, opts, hist, hist_cap, info, 1);
    if (rc != TA_OK) return rc;
    if (opts->precision != TA_FP64) return cta_mixed_one(A, b, x, opts, info, stream, 1);
    return ta::with_plan(A, true, s, [&](const ta::Plan &P) {
        return ta::cta_run(P, b, x, opts, hist, hist_cap, info, s, true);
    }, true);
}

int ta_solve(const ta_mat *A, const double *b, double *x, const ta_opts *opts, double *hist,
             int64_t hist_cap, ta_info *info, void *stream) {
    hipStream_t s = (hipStream_t)stream;
    if (info == nullptr) return TA_EINVAL;
    int rc = ta::check_solve_args(A, b, x, opts, hist, hist_cap, info, 2);
    if (rc != TA_OK) return rc;
    return ta::with_plan(A, true, s, [&](const ta::Plan &P) {
        return ta::ta_run(P, b, x, opts, hist, hist_cap, info, s);
    }, true);
}

int ta_plan_create(const ta_mat *A, ta_plan **plan, void *stream) {
    if (plan == nullptr) return TA_EINVAL;
    *plan = nullptr;
    ta_plan *p = new (std::nothrow) ta_plan;
    if (p == nullptr) return TA_ENOMEM;
    int rc = ta::plan_build(A, true, (hipStream_t)stream, &p->p, true);
    if (rc != TA_OK) {
        ta::plan_free(&p->p);
        delete p;
        return rc;
    }
    *plan = p;
    return TA_OK;
}

int ta_plan_format(const ta_plan *plan, int32_t trans, int32_t *format) {
    if (plan == nullptr || format == nullptr) return TA_EINVAL;
    static_assert(ta::kCsrRows == TA_FMT_CSR_ROWS && ta::kDenseRows == TA_FMT_DENSE_ROWS &&
                      ta::kDenseCols == TA_FMT_DENSE_COLS && ta::kCsrSliced == TA_FMT_CSR_SLICED &&
                      ta::kCsrSell == TA_FMT_SELL64 && ta::kCsrTiled == TA_FMT_CSR_TILED &&
                      ta::kCsrMerge == TA_FMT_CSR_MERGE,
                  "storage kinds");
    *format = trans ? plan->p.AT.kind : plan->p.A.kind;
    return TA_OK;
}

int ta_plan_destroy(ta_plan *plan) {
    if (plan == nullptr) return TA_OK;
    ta::plan_free(&plan->p);
    delete plan;
    return TA_OK;
}

int cta_solve_plan(const ta_plan *plan, const double *b, double *x, const ta_opts *opts,
                   double *hist, int64_t hist_cap, ta_info *info, void *stream) {
    if (plan == nullptr) return TA_EINVAL;
    return ta::cta_run(plan->p, b, x, opts, hist, hist_cap, info, (hipStream_t)stream, false);
}

int cta_solve_plan_noalloc(const ta_plan *plan, const double *b, double *x, const ta_opts *opts,
                           double *hist, int64_t hist_cap, ta_info *info, void *stream) {
    if (plan == nullptr) return TA_EINVAL;
    void *buf = nullptr;
    const int rc = ta::scratch_address(&buf);
    if (rc != TA_OK) return rc;
    return ta::cta_run(plan->p, b, x, opts, hist, hist_cap, info, (hipStream_t)stream, false, buf,
                       TA_NOALLOC_SCRATCH_BYTES);
}

int cta_minnorm_plan(const ta_plan *plan, const double *b, double *x, const ta_opts *opts,
                     double *hist, int64_t hist_cap, ta_info *info, void *stream) {
    if (plan == nullptr) return TA_EINVAL;
    return ta::cta_run(plan->p, b, x, opts, hist, hist_cap, info, (hipStream_t)stream, true);
}

int ta_solve_plan(const ta_plan *plan, const double *b, double *x, const ta_opts *opts,
                  double *hist, int64_t hist_cap, ta_info *info, void *stream) {
    if (plan == nullptr) return TA_EINVAL;
    return ta::ta_run(plan->p, b, x, opts, hist, hist_cap, info, (hipStream_t)stream);
}

int ta_minnorm(const ta_mat *A, const double *b, const double *x_eps, double *x,
               const ta_opts *opts, ta_info *info, int64_t *tests, void *stream) {
    hipStream_t s = (hipStream_t)stream;
    if (info == nullptr) return TA_EINVAL;
    int rc = ta::check_solve_args(A, b, x, opts, nullptr, 0, info, 2);
    if (rc != TA_OK) return rc;
    return ta::with_plan(A, true, s, [&](const ta::Plan &P) {
        return ta::minnorm_run(P, b, x_eps, x, opts, info, tests, s);
    }, true);
}

int ta_minnorm_plan(const ta_plan *plan, const double *b, const double *x_eps, double *x,
                    const ta_opts *opts, ta_info *info, int64_t *tests, void *stream) {
    if (plan == nullptr) return TA_EINVAL;
    return ta::minnorm_run(plan->p, b, x_eps, x, opts, info, tests, (hipStream_t)stream);
}

// The restart of the remark after the theorem on Algorithm 3's properties
// (section 4.3): eps' halved after each run that ends on the normal
// equation, the next run warm-started from that run's x.
int ta_solve_halving(const ta_plan *plan, const double *b, double *x, const ta_opts *opts,
                     int32_t max_halvings, ta_info *info, int32_t *halvings, void *stream) {
    if (plan == nullptr || opts == nullptr || info == nullptr || max_halvings < 0)
        return TA_EINVAL;
    if (opts->normal_eq) return TA_EINVAL;
    ta_opts o = *opts;
    if (!(o.tol_normal > 0.0)) o.tol_normal = o.tol;
    int64_t iters = 0, matvecs = 0;
    int32_t h = 0;
    for (;;) {
        ta_info r;
        memset(&r, 0, sizeof r);
        const int rc = ta::ta_run(plan->p, b, x, &o, nullptr, 0, &r, (hipStream_t)stream);
        if (rc != TA_OK) return rc;
        iters += r.iters;
        matvecs += r.matvecs;
        *info = r;
        if (r.stop != TA_STOP_NORMAL || h >= max_halvings) break;
        o.tol_normal *= 0.5;
        o.warm_start = 1;
        ++h;
    }
    info->iters = iters;
    info->matvecs = matvecs;
    if (halvings != nullptr) *halvings = h;
    return TA_OK;
}

int ta_validate(const ta_mat *A, const ta_opts *opts, int32_t solver) {
    int rc = ta::validate_mat(A);
    if (rc != TA_OK) return rc;
    return ta::validate_opts(A, opts, solver);
}

const char *ta_strerror(int code) {
    switch (code) {
        case TA_OK: return "ok";
        case TA_EINVAL: return "invalid argument";
        case TA_ENOMEM: return "device allocation failed";
        case TA_EHIP: return ta::hip_msg().empty() ? "HIP error" : ta::hip_msg().c_str();
        case TA_ENOTSUP: return "input not supported (outside the sizes the call handles)";
        case TA_ESCRATCH:
            return "the solve needs more device memory than the fixed buffer of "
                   "cta_solve_plan_noalloc holds (64 MiB)";
        default: return "unknown error";
    }
}

int ta_spmv(const ta_mat *A, int32_t trans, const double *x, double *y, double *norm2,
            void *stream) {
    hipStream_t s = (hipStream_t)stream;
    return ta::with_plan(A, trans != 0, s, [&](const ta::Plan &P) {
        return ta::product_run(P, trans, x, y, nullptr, norm2, s);
    });
}

int ta_spmv_plan(const ta_plan *plan, int32_t trans, const double *x, double *y, double *norm2,
                 void *stream) {
    if (plan == nullptr) return TA_EINVAL;
    return ta::product_run(plan->p, trans, x, y, nullptr, norm2, (hipStream_t)stream);
}

int ta_residual(const ta_mat *A, const double *b, const double *x, double *r, double *norm2,
                void *stream) {
    if (b == nullptr && A != nullptr && A->m > 0) return TA_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    return ta::with_plan(A, false, s, [&](const ta::Plan &P) {
        return ta::product_run(P, 0, x, r, b, norm2, s);
    });
}

int ta_time_matvec(const ta_mat *A, int32_t trans, const double *x, double *y, int32_t reps,
                   double *avg_ms, void *stream) {
    hipStream_t s = (hipStream_t)stream;
    return ta::with_plan(A, true, s, [&](const ta::Plan &P) {
        return ta::time_run(P, trans, x, y, reps, avg_ms, s);
    });
}

int ta_time_matvec_plan(const ta_plan *plan, int32_t trans, const double *x, double *y,
                        int32_t reps, double *avg_ms, void *stream) {
    if (plan == nullptr) return TA_EINVAL;
    return ta::time_run(plan->p, trans, x, y, reps, avg_ms, (hipStream_t)stream);
}

int ta_transpose(const ta_mat *A, int32_t *at_row_ptr, int32_t *at_col_idx, double *at_val,
                 void *stream) {
    int rc = ta::validate_mat(A);
    if (rc != TA_OK) return rc;
    if (A->kind != TA_CSR || at_row_ptr == nullptr) return TA_EINVAL;
    if (A->nnz > 0 && (at_col_idx == nullptr || at_val == nullptr)) return TA_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    ta::Workspace ws(s);
    int32_t *work = nullptr, *flag = nullptr;
    const int64_t n = A->n, ntiles = (std::max<int64_t>(n, 1) + 1023) / 1024;
    ws.reserve(&work, 2 * n + ntiles + 8 + A->nnz);
    ws.reserve(&flag, 8);
    if ((rc = ws.commit()) != TA_OK) return rc;
    if ((rc = ta::check_csr_device(A, flag, s)) != TA_OK) return rc;
    hipError_t e = ta::launch_transpose(A->m, n, A->nnz, A->row_ptr, A->col_idx, A->val,
                                        at_row_ptr, at_col_idx, at_val, work, flag, s);
    if (e != hipSuccess) return ta::hip_fail(e, "transpose");
    int32_t h = 0;
    e = hipMemcpyAsync(&h, flag, sizeof(int32_t), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return ta::hip_fail(e, "transpose flag");
    return h ? TA_ENOTSUP : TA_OK;
}

int ta_csr_outer(const ta_mat *A, const double *u, const double *v, double alpha, double *out,
                 void *stream) {
    int rc = ta::validate_mat(A);
    if (rc != TA_OK) return rc;
    if (A->kind != TA_CSR) return TA_EINVAL;
    if (A->nnz > 0 && (u == nullptr || v == nullptr || out == nullptr)) return TA_EINVAL;
    if (A->nnz == 0) return TA_OK;
    hipStream_t s = (hipStream_t)stream;
    ta::Workspace ws(s);
    int32_t *flag = nullptr;
    ws.reserve(&flag, 8);
    if ((rc = ws.commit()) != TA_OK) return rc;
    if ((rc = ta::check_csr_device(A, flag, s)) != TA_OK) return rc;
    hipError_t e = ta::launch_csr_outer(A->m, A->row_ptr, A->col_idx, u, v, alpha, out, s);
    if (e != hipSuccess) return ta::hip_fail(e, "csr outer product");
    return TA_OK;
}

}  // extern "C"
