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
#include <string>
#include <vector>

#include "common.hpp"

namespace ta {

static thread_local std::string g_hip_msg;

static int hip_fail(hipError_t e, const char *what) {
    char buf[256];
    snprintf(buf, sizeof buf, "%s: %s", what, hipGetErrorString(e));
    g_hip_msg = buf;
    return e == hipErrorOutOfMemory ? TA_ENOMEM : TA_EHIP;
}

#define HIP_TRY(call)                                   \
    do {                                                \
        hipError_t e_ = (call);                         \
        if (e_ != hipSuccess) return hip_fail(e_, #call); \
    } while (0)

// ---------------------------------------------------------------------------
// workspace: one stream-ordered allocation carved into aligned pieces
// ---------------------------------------------------------------------------
class Workspace {
   public:
    explicit Workspace(hipStream_t s) : s_(s) {}
    ~Workspace() {
        if (base_ != nullptr) (void)hipFreeAsync(base_, s_);
    }
    template <class T>
    void reserve(T **slot, int64_t count) {
        reqs_.push_back({reinterpret_cast<void **>(slot), (size_t)std::max<int64_t>(count, 1) * sizeof(T)});
    }
    int commit() {
        size_t total = 0;
        for (auto &r : reqs_) total += (r.bytes + 255) & ~size_t(255);
        static thread_local bool pool_set = false;
        if (!pool_set) {
            int dev = 0;
            hipMemPool_t pool;
            if (hipGetDevice(&dev) == hipSuccess && hipDeviceGetDefaultMemPool(&pool, dev) == hipSuccess) {
                uint64_t thr = UINT64_MAX;
                (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &thr);
            }
            pool_set = true;
        }
        HIP_TRY(hipMallocAsync(&base_, total, s_));
        char *p = static_cast<char *>(base_);
        for (auto &r : reqs_) {
            *r.slot = p;
            p += (r.bytes + 255) & ~size_t(255);
        }
        return TA_OK;
    }

   private:
    struct Req {
        void **slot;
        size_t bytes;
    };
    hipStream_t s_;
    void *base_ = nullptr;
    std::vector<Req> reqs_;
};

// pinned host copy of the State, one per host thread
static State *host_state() {
    static thread_local State *h = nullptr;
    if (h == nullptr) {
        if (hipHostMalloc(reinterpret_cast<void **>(&h), sizeof(State)) != hipSuccess) h = nullptr;
    }
    return h;
}

static int read_state(State *d, State &out, hipStream_t s) {
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
static int validate_mat(const ta_mat *A) {
    if (A == nullptr) return TA_EINVAL;
    if (A->m < 0 || A->n < 0 || A->m >= INT32_MAX || A->n >= INT32_MAX) return TA_EINVAL;
    if (A->kind == TA_CSR) {
        if (A->row_ptr == nullptr || A->nnz < 0 || A->nnz >= INT32_MAX) return TA_EINVAL;
        if (A->nnz > 0 && (A->col_idx == nullptr || A->val == nullptr)) return TA_EINVAL;
        return TA_OK;
    }
    if (A->kind == TA_DENSE_ROWMAJOR) {
        if (A->ld < A->n || (A->m > 0 && A->n > 0 && A->val == nullptr)) return TA_EINVAL;
        return TA_OK;
    }
    return TA_EINVAL;
}

static int validate_opts(const ta_mat *A, const ta_opts *o, int solver) {
    if (o == nullptr) return TA_EINVAL;
    if (!(o->tol >= 0.0 && o->tol < 1.0)) return TA_EINVAL;
    if (!(o->tol_normal >= 0.0 && o->tol_normal < 1.0)) return TA_EINVAL;
    if (o->max_iter < 0 || o->replace_every < 0 || o->chunk < 0) return TA_EINVAL;
    if (o->precision != TA_FP64) return TA_EINVAL;  // the solver chains compute in FP64
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

__global__ void k_check_csr(int64_t m, int64_t n, int64_t nnz, const int32_t *rp,
                            const int32_t *ci, int32_t *flag) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i <= m;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t a = rp[i];
        if (i == 0 && a != 0) atomicOr(flag, 1);
        if (i == m && a != nnz) atomicOr(flag, 1);
        if (i < m && rp[i + 1] < a) atomicOr(flag, 1);
    }
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < nnz;
         k += (int64_t)gridDim.x * blockDim.x) {
        const int32_t c = ci[k];
        if (c < 0 || c >= n) atomicOr(flag, 2);
    }
}

// Checks the CSR arrays on the device before any kernel indexes through them.
static int check_csr_device(const ta_mat *A, int32_t *dflag, hipStream_t s) {
    HIP_TRY(hipMemsetAsync(dflag, 0, sizeof(int32_t), s));
    const int64_t work = std::max<int64_t>(A->m + 1, A->nnz);
    const unsigned grid = (unsigned)std::min<int64_t>((work + kBlock - 1) / kBlock, 4096);
    k_check_csr<<<grid, kBlock, 0, s>>>(A->m, A->n, A->nnz, A->row_ptr, A->col_idx, dflag);
    HIP_TRY(hipGetLastError());
    int32_t h = 0;
    HIP_TRY(hipMemcpyAsync(&h, dflag, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    return h ? TA_EINVAL : TA_OK;
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

struct Operator {
    MatView A{}, AT{};
    int32_t *at_rp = nullptr, *at_ci = nullptr;
    double *at_val = nullptr;
    int32_t *tr_work = nullptr;
    int32_t *flag = nullptr;
    int64_t m = 0, n = 0, nnz = 0;
    bool csr = false;

    void reserve(Workspace &ws, const ta_mat *M, bool need_t) {
        m = M->m;
        n = M->n;
        csr = M->kind == TA_CSR;
        nnz = csr ? M->nnz : m * n;
        ws.reserve(&flag, 8);
        if (csr && need_t) {
            const int64_t ntiles = (std::max<int64_t>(n, 1) + 1023) / 1024;
            ws.reserve(&at_rp, n + 1);
            ws.reserve(&at_ci, nnz);
            ws.reserve(&at_val, nnz);
            ws.reserve(&tr_work, 2 * n + ntiles + 8 + nnz);
        }
    }

    // After Workspace::commit.  Validates the CSR and builds A^T if needed.
    int build(const ta_mat *M, bool need_t, hipStream_t s) {
        if (csr) {
            int rc = check_csr_device(M, flag, s);
            if (rc != TA_OK) return rc;
            A = MatView{0, m, n, 0, M->row_ptr, M->col_idx, M->val, pick_lanes(nnz, m)};
            if (need_t) {
                HIP_TRY(launch_transpose(m, n, nnz, M->row_ptr, M->col_idx, M->val, at_rp, at_ci,
                                         at_val, tr_work, flag, s));
                int32_t h = 0;
                HIP_TRY(hipMemcpyAsync(&h, flag, sizeof(int32_t), hipMemcpyDeviceToHost, s));
                HIP_TRY(hipStreamSynchronize(s));
                if (h) return TA_ENOTSUP;
                AT = MatView{0, n, m, 0, at_rp, at_ci, at_val, pick_lanes(nnz, n)};
            }
        } else {
            A = MatView{1, m, n, M->ld, nullptr, nullptr, M->val, 64};
            AT = MatView{2, n, m, M->ld, nullptr, nullptr, M->val, 1};
        }
        return TA_OK;
    }
};

static Tail make_tail(State *st, double *hist, double2 *partials, int32_t post, int32_t arg,
                      int32_t gate) {
    Tail t;
    t.st = st;
    t.hist = hist;
    t.partials = partials;
    t.post = post;
    t.arg = arg;
    t.gate = gate;
    return t;
}

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
    return h;
}

// One State upload; the pinned staging buffer keeps the copy asynchronous.
static int upload_state(State *d, const State &h, hipStream_t s) {
    State *p = host_state();
    if (p == nullptr) return hip_fail(hipErrorOutOfMemory, "hipHostMalloc");
    HIP_TRY(hipStreamSynchronize(s));  // the staging buffer may still be in use
    *p = h;
    HIP_TRY(hipMemcpyAsync(d, p, sizeof(State), hipMemcpyHostToDevice, s));
    HIP_TRY(hipStreamSynchronize(s));
    return TA_OK;
}

// Relative residual and normal-equation residual of the final x (FP64).
static int exit_diagnostics(const Operator &op, const ta_mat *M, const double *b, const double *x,
                            double *tmp_m, double *tmp_n, State *st, double2 *partials,
                            hipStream_t s, double nb, ta_info *info) {
    EpiArgs ea{};
    ea.b = b;
    HIP_TRY(launch_matvec(op.A, x, tmp_m, kEpiResid, ea,
                          make_tail(st, nullptr, partials, kPostStore, 0, kGateIgnoreDone), s));
    HIP_TRY(launch_matvec(op.AT, tmp_m, tmp_n, kEpiNorm, EpiArgs{},
                          make_tail(st, nullptr, partials, kPostStore, 1, kGateIgnoreDone), s));
    HIP_TRY(launch_matvec(op.AT, b, tmp_n, kEpiNorm, EpiArgs{},
                          make_tail(st, nullptr, partials, kPostStore, 2, kGateIgnoreDone), s));
    State h;
    int rc = read_state(st, h, s);
    if (rc != TA_OK) return rc;
    (void)M;
    info->rel_res = nb > 0.0 ? sqrt(h.scratch[0]) / nb : 0.0;
    const double nab = sqrt(h.scratch[2]);
    info->rel_normal = nab > 0.0 ? sqrt(h.scratch[1]) / nab : 0.0;
    return TA_OK;
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

// ---------------------------------------------------------------------------
// CTA (x-form and y-form)
// ---------------------------------------------------------------------------
static int cta_impl(const ta_mat *M, const double *b, double *x, const ta_opts *o, double *hist,
                    int64_t hist_cap, ta_info *info, hipStream_t s, bool minnorm) {
    if (info == nullptr) return TA_EINVAL;
    memset(info, 0, sizeof *info);
    int rc = validate_mat(M);
    if (rc == TA_OK) rc = validate_opts(M, o, minnorm ? 1 : 0);
    if (rc != TA_OK) return rc;
    if ((M->m > 0 && b == nullptr) || (M->n > 0 && x == nullptr)) return TA_EINVAL;
    if (hist != nullptr && hist_cap < 0) return TA_EINVAL;
    const int64_t m = M->m, n = M->n;
    const int t = o->t;
    if (m == 0) {  // empty system: b = 0
        if (n > 0) HIP_TRY(hipMemsetAsync(x, 0, sizeof(double) * (size_t)n, s));
        if (hist != nullptr && hist_cap > 0) HIP_TRY(hipMemsetAsync(hist, 0, sizeof(double), s));
        HIP_TRY(hipStreamSynchronize(s));
        info->stop = TA_STOP_RESIDUAL;
        return TA_OK;
    }

    Workspace ws(s);
    Operator op;
    op.reserve(ws, M, true);
    State *st = nullptr;
    double *r = nullptr, *y = nullptr, *tmp_n = nullptr;
    double *u[kTMax + 1] = {}, *w[kTMax] = {};
    double2 *partials = nullptr;
    ws.reserve(&st, 1);
    ws.reserve(&r, m);
    for (int j = 1; j <= t; ++j) ws.reserve(&u[j], m);
    const int nw = minnorm ? 1 : t;
    for (int j = 0; j < nw; ++j) ws.reserve(&w[j], n);
    if (minnorm) ws.reserve(&y, m);
    ws.reserve(&tmp_n, n);
    // partial capacity: 2 values per block of the widest grid of the chain
    {
        MatView a{}, at{};
        const int64_t nnz = M->kind == TA_CSR ? M->nnz : m * n;
        if (M->kind == TA_CSR) {
            a = MatView{0, m, n, 0, nullptr, nullptr, nullptr, pick_lanes(nnz, m)};
            at = MatView{0, n, m, 0, nullptr, nullptr, nullptr, pick_lanes(nnz, n)};
        } else {
            a = MatView{1, m, n, M->ld, nullptr, nullptr, nullptr, 64};
            at = MatView{2, n, m, M->ld, nullptr, nullptr, nullptr, 1};
        }
        int64_t cap = std::max({matvec_blocks(a), matvec_blocks(at),
                                elementwise_blocks(std::max(m, n)), (int64_t)1});
        ws.reserve(&partials, 2 * cap);
    }
    if ((rc = ws.commit()) != TA_OK) return rc;
    if ((rc = op.build(M, true, s)) != TA_OK) return rc;

    State h0 = initial_state(o, hist_cap, hist);
    if ((rc = upload_state(st, h0, s)) != TA_OK) return rc;
    u[0] = r;
    double *const xy = minnorm ? y : x;
    const int64_t nxy = minnorm ? m : n;
    const bool warm = o->warm_start && !minnorm;

    // initial state: r = b, x = 0 (or y = 0), ||b||
    HIP_TRY(launch_cta_init(m, n, b, r, xy, nxy, warm ? 0 : 1,
                            make_tail(st, hist, partials, kPostCtaInit, warm ? 1 : 0, kGateAlways), s));
    if (o->tol_normal > 0.0)
        HIP_TRY(launch_matvec(op.AT, b, tmp_n, kEpiNorm, EpiArgs{},
                              make_tail(st, nullptr, partials, kPostNab, 0, kGateAlways), s));
    EpiArgs eres{};
    eres.b = b;
    if (warm)
        HIP_TRY(launch_matvec(op.A, x, r, kEpiResid, eres,
                              make_tail(st, hist, partials, kPostCtaWarm, 0, kGateAlways), s));

    auto enqueue_iteration = [&]() -> int {
        for (int j = 0; j < t; ++j) {
            double *wj = w[minnorm ? 0 : j];
            HIP_TRY(launch_matvec(op.AT, u[j], wj, kEpiNorm, EpiArgs{},
                                  make_tail(st, nullptr, partials, kPostPhi, 2 * j + 1, kGateAlways),
                                  s));
            HIP_TRY(launch_matvec(op.A, wj, u[j + 1], kEpiNorm, EpiArgs{},
                                  make_tail(st, nullptr, partials,
                                            j == t - 1 ? kPostPhiGram : kPostPhi, 2 * j + 2,
                                            kGateAlways),
                                  s));
        }
        HIP_TRY(launch_cta_update(m, n, t, minnorm ? 1 : 0, r, u, x, w, y,
                                  make_tail(st, hist, partials, kPostCtaEnd, 0, kGateAlways), s));
        if (o->replace_every > 0) {
            if (minnorm)
                HIP_TRY(launch_matvec(op.AT, y, x, kEpiNorm, EpiArgs{},
                                      make_tail(st, nullptr, partials, kPostCount, 0, kGateReplace),
                                      s));
            HIP_TRY(launch_matvec(op.A, x, r, kEpiResid, eres,
                                  make_tail(st, nullptr, partials, kPostCtaReplace, 0, kGateReplace),
                                  s));
        }
        return TA_OK;
    };

    Chunker ch(o->chunk);
    State h;
    if ((rc = read_state(st, h, s)) != TA_OK) return rc;
    while (!h.done || h.stop == kStopCandidate) {
        if (h.stop == kStopCandidate) {
            if (minnorm)
                HIP_TRY(launch_matvec(op.AT, y, x, kEpiNorm, EpiArgs{},
                                      make_tail(st, nullptr, partials, kPostCount, 0, kGateIgnoreDone),
                                      s));
            HIP_TRY(launch_matvec(op.A, x, r, kEpiResid, eres,
                                  make_tail(st, nullptr, partials, kPostCtaCand, 0, kGateIgnoreDone),
                                  s));
        } else {
            const int64_t k = ch.take();
            for (int64_t i = 0; i < k; ++i)
                if ((rc = enqueue_iteration()) != TA_OK) return rc;
            const int64_t k_before = h.k;
            if ((rc = read_state(st, h, s)) != TA_OK) return rc;
            // every enqueued iteration advances k until the solve stops
            if (!h.done && h.k == k_before) {
                g_hip_msg = "iteration chain made no progress";
                return TA_EHIP;
            }
            continue;
        }
        if ((rc = read_state(st, h, s)) != TA_OK) return rc;
    }
    if (h.nb == 0.0) HIP_TRY(hipMemsetAsync(x, 0, sizeof(double) * (size_t)n, s));
    if (minnorm)
        HIP_TRY(launch_matvec(op.AT, y, x, kEpiNorm, EpiArgs{},
                              make_tail(st, nullptr, partials, kPostNone, 0, kGateIgnoreDone), s));
    fill_info(h, info);
    if (h.nb > 0.0) {
        rc = exit_diagnostics(op, M, b, x, r, tmp_n, st, partials, s, h.nb, info);
        if (rc != TA_OK) return rc;
    } else {
        HIP_TRY(hipStreamSynchronize(s));
    }
    return TA_OK;
}

// ---------------------------------------------------------------------------
// TA (Algorithm 3, or Algorithm 2 with a fixed radius)
// ---------------------------------------------------------------------------
static int ta_impl(const ta_mat *M, const double *b, double *x, const ta_opts *o, double *hist,
                   int64_t hist_cap, ta_info *info, hipStream_t s) {
    if (info == nullptr) return TA_EINVAL;
    memset(info, 0, sizeof *info);
    int rc = validate_mat(M);
    if (rc == TA_OK) rc = validate_opts(M, o, 2);
    if (rc != TA_OK) return rc;
    if ((M->m > 0 && b == nullptr) || (M->n > 0 && x == nullptr)) return TA_EINVAL;
    if (hist != nullptr && hist_cap < 0) return TA_EINVAL;
    const int64_t m = M->m, n = M->n;
    if (m == 0) {
        if (n > 0) HIP_TRY(hipMemsetAsync(x, 0, sizeof(double) * (size_t)n, s));
        if (hist != nullptr && hist_cap > 0) HIP_TRY(hipMemsetAsync(hist, 0, sizeof(double), s));
        HIP_TRY(hipStreamSynchronize(s));
        info->stop = TA_STOP_RESIDUAL;
        info->rho = o->rho0;
        return TA_OK;
    }

    Workspace ws(s);
    Operator op;
    op.reserve(ws, M, true);
    State *st = nullptr;
    double *r = nullptr, *bp = nullptr, *c = nullptr, *d = nullptr, *tmp_m = nullptr;
    double2 *partials = nullptr;
    ws.reserve(&st, 1);
    ws.reserve(&r, m);
    ws.reserve(&bp, m);
    ws.reserve(&d, m);
    ws.reserve(&tmp_m, m);
    ws.reserve(&c, n);
    {
        MatView a{}, at{};
        const int64_t nnz = M->kind == TA_CSR ? M->nnz : m * n;
        if (M->kind == TA_CSR) {
            a = MatView{0, m, n, 0, nullptr, nullptr, nullptr, pick_lanes(nnz, m)};
            at = MatView{0, n, m, 0, nullptr, nullptr, nullptr, pick_lanes(nnz, n)};
        } else {
            a = MatView{1, m, n, M->ld, nullptr, nullptr, nullptr, 64};
            at = MatView{2, n, m, M->ld, nullptr, nullptr, nullptr, 1};
        }
        int64_t cap = std::max({matvec_blocks(a), matvec_blocks(at),
                                elementwise_blocks(std::max(m, n)), (int64_t)1});
        ws.reserve(&partials, 2 * cap);
    }
    if ((rc = ws.commit()) != TA_OK) return rc;
    if ((rc = op.build(M, true, s)) != TA_OK) return rc;

    State h0 = initial_state(o, hist_cap, hist);
    if ((rc = upload_state(st, h0, s)) != TA_OK) return rc;

    HIP_TRY(launch_ta_init(m, n, b, r, bp, x,
                           make_tail(st, hist, partials, kPostTaInit, 0, kGateAlways), s));
    if (o->tol_normal > 0.0)
        HIP_TRY(launch_matvec(op.AT, b, c, kEpiNorm, EpiArgs{},
                              make_tail(st, nullptr, partials, kPostNab, 0, kGateAlways), s));

    EpiArgs ed{};
    ed.bp = bp;
    ed.r = r;
    auto enqueue_iteration = [&]() -> int {
        HIP_TRY(launch_matvec(op.AT, r, c, kEpiNorm, EpiArgs{},
                              make_tail(st, hist, partials, kPostTaC, 0, kGateNeedC), s));
        HIP_TRY(launch_matvec(op.A, c, d, kEpiTaD, ed,
                              make_tail(st, nullptr, partials, kPostTaS, 0, kGatePivot), s));
        HIP_TRY(launch_ta_update(m, n, b, bp, d, r, x, c,
                                 make_tail(st, hist, partials, kPostTaEnd, 0, kGatePivot), s));
        return TA_OK;
    };

    EpiArgs eres{};
    eres.b = b;
    EpiArgs ebp{};
    ebp.b = b;
    ebp.r_out = r;
    Chunker ch(o->chunk);
    State h;
    if ((rc = read_state(st, h, s)) != TA_OK) return rc;
    while (!h.done || h.stop == kStopCandidate) {
        if (h.stop == kStopCandidate) {
            HIP_TRY(launch_matvec(op.A, x, tmp_m, kEpiResid, eres,
                                  make_tail(st, nullptr, partials, kPostTaCand, 0, kGateIgnoreDone),
                                  s));
            HIP_TRY(launch_matvec(op.A, x, bp, kEpiTaBp, ebp,
                                  make_tail(st, nullptr, partials, kPostTaBp, 0, kGateAlways), s));
        } else {
            const int64_t k = ch.take();
            for (int64_t i = 0; i < k; ++i)
                if ((rc = enqueue_iteration()) != TA_OK) return rc;
            const int64_t k_before = h.k;
            if ((rc = read_state(st, h, s)) != TA_OK) return rc;
            // every enqueued iteration advances k until the solve stops
            if (!h.done && h.k == k_before) {
                g_hip_msg = "iteration chain made no progress";
                return TA_EHIP;
            }
            continue;
        }
        if ((rc = read_state(st, h, s)) != TA_OK) return rc;
    }
    fill_info(h, info);
    if (h.nb > 0.0) {
        rc = exit_diagnostics(op, M, b, x, tmp_m, c, st, partials, s, h.nb, info);
        if (rc != TA_OK) return rc;
    } else {
        HIP_TRY(hipStreamSynchronize(s));
    }
    return TA_OK;
}

// ---------------------------------------------------------------------------
// kernel-level entry points
// ---------------------------------------------------------------------------
static int product_impl(const ta_mat *M, int32_t trans, const double *x, double *y,
                        const double *b, double *norm2, hipStream_t s) {
    int rc = validate_mat(M);
    if (rc != TA_OK) return rc;
    const int64_t rows = trans ? M->n : M->m, cols = trans ? M->m : M->n;
    if ((cols > 0 && x == nullptr) || (rows > 0 && y == nullptr)) return TA_EINVAL;
    if (rows == 0) {
        if (norm2 != nullptr) HIP_TRY(hipMemsetAsync(norm2, 0, sizeof(double), s));
        return TA_OK;
    }
    Workspace ws(s);
    Operator op;
    const bool need_t = trans != 0;
    op.reserve(ws, M, need_t);
    State *st = nullptr;
    double2 *partials = nullptr;
    ws.reserve(&st, 1);
    ws.reserve(&partials, 2 * std::max<int64_t>(rows, 1));
    if ((rc = ws.commit()) != TA_OK) return rc;
    if ((rc = op.build(M, need_t, s)) != TA_OK) return rc;
    HIP_TRY(hipMemsetAsync(st, 0, sizeof(State), s));
    EpiArgs ea{};
    ea.b = b;
    const MatView &V = trans ? op.AT : op.A;
    HIP_TRY(launch_matvec(V, x, y, b != nullptr ? kEpiResid : kEpiNorm, ea,
                          make_tail(st, nullptr, partials, kPostStore, 0, kGateIgnoreDone), s));
    if (norm2 != nullptr)
        HIP_TRY(hipMemcpyAsync(norm2, &st->scratch[0], sizeof(double), hipMemcpyDeviceToDevice, s));
    return TA_OK;
}

// Average duration of one launch of the matvec kernel the solvers use for
// y = A x (trans = 0) or y = A^T x (trans = 1), over `reps` back-to-back
// launches bracketed by HIP events on `s`.
static int time_matvec_impl(const ta_mat *M, int32_t trans, const double *x, double *y,
                            int32_t reps, double *avg_ms, hipStream_t s) {
    int rc = validate_mat(M);
    if (rc != TA_OK) return rc;
    if (reps < 1 || avg_ms == nullptr || x == nullptr || y == nullptr) return TA_EINVAL;
    const int64_t rows = trans ? M->n : M->m;
    Workspace ws(s);
    Operator op;
    const bool need_t = trans != 0;
    op.reserve(ws, M, need_t);
    State *st = nullptr;
    double2 *partials = nullptr;
    ws.reserve(&st, 1);
    ws.reserve(&partials, 2 * std::max<int64_t>(rows, 1));
    if ((rc = ws.commit()) != TA_OK) return rc;
    if ((rc = op.build(M, need_t, s)) != TA_OK) return rc;
    HIP_TRY(hipMemsetAsync(st, 0, sizeof(State), s));
    const MatView &V = trans ? op.AT : op.A;
    const Tail tl = make_tail(st, nullptr, partials, kPostStore, 0, kGateIgnoreDone);
    HIP_TRY(launch_matvec(V, x, y, kEpiNorm, EpiArgs{}, tl, s));  // warm-up
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    HIP_TRY(hipEventRecord(e0, s));
    for (int32_t i = 0; i < reps; ++i) HIP_TRY(launch_matvec(V, x, y, kEpiNorm, EpiArgs{}, tl, s));
    HIP_TRY(hipEventRecord(e1, s));
    HIP_TRY(hipEventSynchronize(e1));
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    *avg_ms = (double)ms / reps;
    return TA_OK;
}

}  // namespace ta

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

int cta_solve(const ta_mat *A, const double *b, double *x, const ta_opts *opts, double *hist,
              int64_t hist_cap, ta_info *info, void *stream) {
    return ta::cta_impl(A, b, x, opts, hist, hist_cap, info, (hipStream_t)stream, false);
}

int cta_minnorm(const ta_mat *A, const double *b, double *x, const ta_opts *opts, double *hist,
                int64_t hist_cap, ta_info *info, void *stream) {
    return ta::cta_impl(A, b, x, opts, hist, hist_cap, info, (hipStream_t)stream, true);
}

int ta_solve(const ta_mat *A, const double *b, double *x, const ta_opts *opts, double *hist,
             int64_t hist_cap, ta_info *info, void *stream) {
    return ta::ta_impl(A, b, x, opts, hist, hist_cap, info, (hipStream_t)stream);
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
        case TA_EHIP: return ta::g_hip_msg.empty() ? "HIP error" : ta::g_hip_msg.c_str();
        case TA_ENOTSUP: return "input not supported (a column of A holds more than 8192 entries)";
        default: return "unknown error";
    }
}

int ta_spmv(const ta_mat *A, int32_t trans, const double *x, double *y, double *norm2,
            void *stream) {
    return ta::product_impl(A, trans, x, y, nullptr, norm2, (hipStream_t)stream);
}

int ta_residual(const ta_mat *A, const double *b, const double *x, double *r, double *norm2,
                void *stream) {
    if (b == nullptr && A != nullptr && A->m > 0) return TA_EINVAL;
    return ta::product_impl(A, 0, x, r, b, norm2, (hipStream_t)stream);
}

int ta_time_matvec(const ta_mat *A, int32_t trans, const double *x, double *y, int32_t reps,
                   double *avg_ms, void *stream) {
    return ta::time_matvec_impl(A, trans, x, y, reps, avg_ms, (hipStream_t)stream);
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

}  // extern "C"
