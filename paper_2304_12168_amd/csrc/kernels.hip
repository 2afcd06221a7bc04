// Device kernels of libta (gfx950, wave64).
//
// Every kernel of an iteration chain reads the solver State at entry and
// returns at once when the chain is finished, so the host can enqueue many
// iterations ahead and read one flag per chunk.  Reductions are fused into
// the kernel that produces the vector: each block reduces its part with
// compensated (double-double) arithmetic, writes one partial, and the last
// block to finish (atomic counter) reduces the partials in block order and
// runs the scalar step logic of the method (the "post" action).  There are
// no floating-point atomics, so every result is run-to-run reproducible.
//
// Compensated arithmetic: TwoSum (Knuth) and TwoProduct via fma, combined as
// in Dot2 of Ogita, Rump and Oishi (SIAM J. Sci. Comput. 26, 2005).  Built
// with -ffp-contract=off: every fma below is explicit.
#include <math.h>

#include "common.hpp"

namespace ta {

// ---------------------------------------------------------------------------
// compensated accumulation
// ---------------------------------------------------------------------------
struct Acc {
    double p, s;  // value p + s
};

__device__ __forceinline__ void two_sum(double a, double b, double &x, double &y) {
    x = a + b;
    const double z = x - a;
    y = (a - (x - z)) + (b - z);
}

// acc += h + r where h + r is an exact product split (h = fl(a b), r = error)
__device__ __forceinline__ void acc_add_split(Acc &c, double h, double r) {
    double q;
    two_sum(c.p, h, c.p, q);
    c.s = c.s + (q + r);
}

__device__ __forceinline__ void acc_fma(Acc &c, double a, double b) {
    const double h = a * b;
    const double r = __fma_rn(a, b, -h);
    acc_add_split(c, h, r);
}

__device__ __forceinline__ Acc acc_merge(Acc a, Acc b) {
    Acc o;
    double q;
    two_sum(a.p, b.p, o.p, q);
    o.s = (a.s + b.s) + q;
    return o;
}

__device__ __forceinline__ double acc_val(Acc a) { return a.p + a.s; }

template <int W>
__device__ __forceinline__ Acc group_reduce(Acc v) {
#pragma unroll
    for (int off = W / 2; off > 0; off >>= 1) {
        Acc o;
        o.p = __shfl_xor(v.p, off);
        o.s = __shfl_xor(v.s, off);
        v = acc_merge(v, o);
    }
    return v;
}

// Blocks are handed to the 8 XCDs round-robin; give each XCD a contiguous
// range of logical blocks so neighbouring rows share one L2.
__device__ __forceinline__ int64_t xcd_remap(int64_t b, int64_t G) {
    const int64_t q = G / 8, rem = G % 8;
    const int64_t x = b % 8, i = b / 8;
    return x * q + (x < rem ? x : rem) + i;
}

__device__ __forceinline__ void store_partial(double2 *p, Acc a) {
    uint64_t *q = reinterpret_cast<uint64_t *>(p);
    __hip_atomic_store(q, __double_as_longlong(a.p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(q + 1, __double_as_longlong(a.s), __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ Acc load_partial(const double2 *p) {
    const uint64_t *q = reinterpret_cast<const uint64_t *>(p);
    Acc a;
    a.p = __longlong_as_double(
        __hip_atomic_load(const_cast<uint64_t *>(q), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
    a.s = __longlong_as_double(__hip_atomic_load(const_cast<uint64_t *>(q + 1), __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_AGENT));
    return a;
}

// ---------------------------------------------------------------------------
// The auxiliary equation of CTA (section 3.1, eq. "eqcoeff"), one thread.
// M_ij = phi_{i+j}, g_i = phi_i (i, j = 1..t).  Reading of "minimum-norm
// solution when not unique": ridge solution of an exactly (power-of-two)
// scaled system, continuous in phi.  Steps:
//   order te: t, lowered to i-1 at the first phi_{2i} <= 0;
//   te = 1: alpha_1 = phi_1 / phi_2 (Example 1);
//   else s_i = 2^-floor((e_i - 1)/2) with phi_{2i} = f 2^e_i, f in [0.5, 1);
//        Ms_ij = (phi_{i+j} s_i) s_j, gs_i = phi_i s_i,
//        Ms_ii = fma(Ms_ii, 16 te^2 2^-53, Ms_ii);
//        Cholesky column by column, te lowered to j at a pivot <= 0
//        (te = 1 then uses the closed form);
//        forward / back substitution; alpha_i = s_i alpha~_i.
// ---------------------------------------------------------------------------
constexpr int kGramLds = 2 * kTMax * kTMax + 4 * kTMax;

// lds: kGramLds doubles of workspace (LDS of the calling block)
__device__ int gram_alpha(const double *phi, int t, double *alpha, double *lds) {
    double(*M)[kTMax] = reinterpret_cast<double(*)[kTMax]>(lds);
    double(*L)[kTMax] = reinterpret_cast<double(*)[kTMax]>(lds + kTMax * kTMax);
    double *s = lds + 2 * kTMax * kTMax;
    double *g = s + kTMax;
    double *z = g + kTMax;
    double *at = z + kTMax;
    int te = t;
    for (int i = 0; i < t; ++i) alpha[i] = 0.0;
    for (int i = 1; i <= t; ++i) {
        if (!(phi[2 * i] > 0.0)) {
            te = i - 1;
            break;
        }
    }
    if (te <= 0) return 0;
    if (te >= 2) {
        for (int i = 0; i < te; ++i) {
            int e;
            (void)frexp(phi[2 * (i + 1)], &e);
            const int kk = (int)floor((e - 1) / 2.0);
            s[i] = ldexp(1.0, -kk);
        }
        for (int i = 0; i < te; ++i) {
            for (int j = 0; j < te; ++j) M[i][j] = (phi[i + j + 2] * s[i]) * s[j];
            g[i] = phi[i + 1] * s[i];
        }
        const double ridge = 16.0 * (double)te * (double)te * ldexp(1.0, -53);
        for (int i = 0; i < te; ++i) M[i][i] = __fma_rn(M[i][i], ridge, M[i][i]);
        for (int j = 0; j < te; ++j) {
            double d = M[j][j];
            for (int k = 0; k < j; ++k) d = __fma_rn(-L[j][k], L[j][k], d);
            if (!(d > 0.0)) {
                te = j;
                break;
            }
            L[j][j] = sqrt(d);
            for (int i = j + 1; i < te; ++i) {
                double v = M[i][j];
                for (int k = 0; k < j; ++k) v = __fma_rn(-L[i][k], L[j][k], v);
                L[i][j] = v / L[j][j];
            }
        }
    }
    if (te == 1) {
        alpha[0] = phi[1] / phi[2];
        return 1;
    }
    for (int i = 0; i < te; ++i) {
        double v = g[i];
        for (int k = 0; k < i; ++k) v = __fma_rn(-L[i][k], z[k], v);
        z[i] = v / L[i][i];
    }
    for (int i = te - 1; i >= 0; --i) {
        double v = z[i];
        for (int k = i + 1; k < te; ++k) v = __fma_rn(-L[k][i], at[k], v);
        at[i] = v / L[i][i];
    }
    for (int i = 0; i < te; ++i) alpha[i] = s[i] * at[i];
    return te;
}

// ---------------------------------------------------------------------------
// Scalar step logic run by thread 0 of the last block.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void finish(State *st, int32_t code) {
    st->done = 1;
    st->stop = code;
}

// The tests at the top of the while loop of Algorithms 1 and 3.
__device__ __forceinline__ void loop_top(State *st) {
    if (sqrt(st->rr) <= st->tol_nb)
        finish(st, kStopCandidate);
    else if (st->k >= st->max_iter)
        finish(st, TA_STOP_MAXITER);
}

__device__ __forceinline__ void put_hist(State *st, double *hist) {
    if (hist != nullptr && st->k < st->hist_cap) hist[st->k] = sqrt(st->rr) / st->nb;
}

__device__ void post_action(const Tail &tl, double v0, double v1, bool computed, double *lds) {
    State *st = tl.st;
    switch (tl.post) {
        case kPostNone:
            break;
        case kPostStore:
            st->scratch[tl.arg] = v0;
            break;
        case kPostCount:
            st->matvecs++;
            break;
        case kPostCtaInit:
        case kPostTaInit: {
            const double nb = sqrt(v0);
            st->nb = nb;
            st->tol_nb = st->tol * nb;
            st->rr = v0;
            st->rb = v0;
            st->k = 0;
            if (nb == 0.0) {
                if (tl.hist != nullptr && st->hist_cap > 0) tl.hist[0] = 0.0;
                finish(st, TA_STOP_RESIDUAL);
                break;
            }
            if (tl.arg == 0) {  // arg = 1: a warm start recomputes r next
                put_hist(st, tl.hist);
                loop_top(st);
            }
            break;
        }
        case kPostCtaWarm:
            st->rr = v0;
            st->matvecs++;
            put_hist(st, tl.hist);
            loop_top(st);
            break;
        case kPostNab:
            st->nab = sqrt(v0);
            st->tol_ne_nab = st->tol_normal * st->nab;
            st->matvecs++;
            break;
        case kPostPhi:
            st->phi[tl.arg] = v0;
            st->matvecs++;
            break;
        case kPostPhiGram: {
            st->phi[tl.arg] = v0;
            st->matvecs++;
            const int t = st->t;
            for (int i = 1; i <= 2 * t; ++i)
                if (!isfinite(st->phi[i])) {
                    finish(st, TA_STOP_BREAKDOWN);
                    return;
                }
            if (sqrt(st->phi[1]) <= st->tol_ne_nab || st->phi[2] == 0.0) {
                finish(st, TA_STOP_NORMAL);
                return;
            }
            double *a = lds + kGramLds;
            gram_alpha(st->phi, t, a, lds);
            for (int i = 0; i < t; ++i)
                if (!isfinite(a[i])) {
                    finish(st, TA_STOP_BREAKDOWN);
                    return;
                }
            for (int i = 0; i < t; ++i) st->alpha[i] = a[i];
            break;
        }
        case kPostCtaEnd:
            st->rr = v0;
            st->k++;
            put_hist(st, tl.hist);
            if (st->replace_every > 0 && st->k % st->replace_every == 0)
                st->replace = 1;
            else
                loop_top(st);
            break;
        case kPostCtaReplace:
            st->rr = v0;
            st->replace = 0;
            st->matvecs++;
            loop_top(st);
            break;
        case kPostCtaCand:
            st->matvecs++;
            st->rr = v0;
            if (sqrt(v0) <= st->tol_nb) {
                finish(st, TA_STOP_RESIDUAL);
            } else {
                st->done = 0;
                st->stop = 0;
                if (st->k >= st->max_iter) finish(st, TA_STOP_MAXITER);
            }
            break;
        case kPostTaC: {
            if (computed) {
                st->nc = sqrt(v0);
                st->have_c = 1;
                st->matvecs++;
            }
            const double nc = st->nc, rb = st->rb;
            if (!isfinite(nc) || !isfinite(rb)) {
                finish(st, TA_STOP_BREAKDOWN);
                break;
            }
            if (nc <= st->tol_ne_nab) {
                finish(st, TA_STOP_NORMAL);
                break;
            }
            if (st->pass || st->rho * nc >= rb) {
                st->pivot = 1;
                st->gamma = st->rho / nc;
            } else {
                st->pivot = 0;
                const double q = rb / nc;
                if (st->fixed_rho) {
                    st->rho_lo = q;
                    finish(st, TA_STOP_WITNESS);
                    break;
                }
                if (q > st->rho_lo) st->rho_lo = q;
                st->pass = (q >= 2.0 * st->rho);
                st->rho = (2.0 * st->rho >= q) ? 2.0 * st->rho : q;
                st->k++;
                put_hist(st, tl.hist);
                loop_top(st);
            }
            break;
        }
        case kPostTaS: {
            st->matvecs++;
            const double rd = v0, dd = v1;
            if (!(dd > 0.0) || !isfinite(rd) || !isfinite(dd)) {
                finish(st, TA_STOP_BREAKDOWN);
                break;
            }
            double a = rd / dd;
            if (a < 0.0) a = 0.0;
            if (a > 1.0) a = 1.0;
            st->alpha_ta = a;
            break;
        }
        case kPostTaEnd:
            st->rr = v0;
            st->rb = v1;
            st->pass = 0;
            st->have_c = 0;
            st->pivot = 0;
            st->k++;
            put_hist(st, tl.hist);
            loop_top(st);
            break;
        case kPostTaCand:
            st->matvecs++;
            if (sqrt(v0) <= st->tol_nb) {
                finish(st, TA_STOP_RESIDUAL);
            } else {
                st->done = 0;
                st->stop = 0;
            }
            break;
        case kPostTaBp:
            st->matvecs++;
            st->rr = v0;
            st->rb = v1;
            st->have_c = 0;
            if (st->k >= st->max_iter) finish(st, TA_STOP_MAXITER);
            break;
        default:
            break;
    }
}

// 0: skip, 1: run, 2: only block 0 runs the post action (c is current)
__device__ __forceinline__ int gate_of(const Tail &tl) {
    if (tl.gate == kGateIgnoreDone) return 1;
    const State *st = tl.st;
    if (st->done) return 0;
    if (tl.gate == kGatePivot && !st->pivot) return 0;
    if (tl.gate == kGateReplace && !st->replace) return 0;
    if (tl.gate == kGateNeedC && st->have_c) return 2;
    return 1;
}

// Reduce NV values over the grid; the last block runs the post action.
template <int NV>
__device__ void block_finish(Acc (&v)[NV], const Tail &tl) {
    __shared__ double gram_lds[kGramLds + kTMax];
    __shared__ Acc red[2][kBlock / 64];
    __shared__ int is_last;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < NV; ++q) {
        const Acc w = group_reduce<64>(v[q]);
        if (lane == 0) red[q][wave] = w;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int q = 0; q < NV; ++q) {
            Acc a = red[q][0];
            for (int w = 1; w < kBlock / 64; ++w) a = acc_merge(a, red[q][w]);
            store_partial(&tl.partials[(int64_t)q * gridDim.x + blockIdx.x], a);
        }
        __threadfence();
        const uint32_t prev = atomicAdd(&tl.st->counter, 1u);
        is_last = (prev == gridDim.x - 1);
    }
    __syncthreads();
    if (!is_last) return;
    __threadfence();
#pragma unroll
    for (int q = 0; q < NV; ++q) {
        Acc a = {0.0, 0.0};
        for (int64_t i = threadIdx.x; i < (int64_t)gridDim.x; i += kBlock)
            a = acc_merge(a, load_partial(&tl.partials[(int64_t)q * gridDim.x + i]));
        a = group_reduce<64>(a);
        if (lane == 0) red[q][wave] = a;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double vals[2] = {0.0, 0.0};
#pragma unroll
        for (int q = 0; q < NV; ++q) {
            Acc a = red[q][0];
            for (int w = 1; w < kBlock / 64; ++w) a = acc_merge(a, red[q][w]);
            vals[q] = acc_val(a);
        }
        tl.st->counter = 0;
        post_action(tl, vals[0], vals[1], true, gram_lds);
    }
}

template <int EPI>
struct EpiNV {
    static constexpr int value = (EPI == kEpiTaD || EPI == kEpiTaBp) ? 2 : 1;
};

// Epilogue for one output entry y_row = yv.
template <int EPI>
__device__ __forceinline__ void epilogue(int64_t row, double yv, double *y, const EpiArgs &ea,
                                         const State *st, Acc (&v)[EpiNV<EPI>::value]) {
    if constexpr (EPI == kEpiNorm || EPI == kEpiResid) {
        y[row] = yv;
        acc_fma(v[0], yv, yv);
    } else if constexpr (EPI == kEpiTaD) {
        const double d = __fma_rn(st->gamma, yv, -ea.bp[row]);
        y[row] = d;
        acc_fma(v[0], ea.r[row], d);
        acc_fma(v[1], d, d);
    } else {  // kEpiTaBp
        y[row] = yv;
        const double bv = ea.b[row];
        const double rv = bv - yv;
        ea.r_out[row] = rv;
        acc_fma(v[0], rv, rv);
        acc_fma(v[1], rv, bv);
    }
}

// ---------------------------------------------------------------------------
// CSR, one thread per row, nonzeros staged through LDS.  A block owns 256
// consecutive rows; their nonzeros are read in coalesced chunks, each product
// is split exactly (TwoProduct) by the thread that loads it, and each row is
// then summed by its own thread in storage order.
// ---------------------------------------------------------------------------
template <int EPI>
__global__ __launch_bounds__(kBlock) void k_csr_stream(MatView M, const double *__restrict__ x,
                                                        double *y, EpiArgs ea, Tail tl) {
    const int g = gate_of(tl);
    if (g == 0) return;
    if (g == 2) {
        if (blockIdx.x == 0 && threadIdx.x == 0) post_action(tl, 0.0, 0.0, false, nullptr);
        return;
    }
    __shared__ double sh[kChunk];
    __shared__ double se[kChunk];
    __shared__ int32_t srp[kBlock + 1];
    const int tid = threadIdx.x;
    const int64_t blk = xcd_remap(blockIdx.x, gridDim.x);
    const int64_t r0 = blk * kBlock;
    const int nrows = (int)min((int64_t)kBlock, M.rows - r0);
    if (tid < nrows) srp[tid] = M.rp[r0 + tid];
    if (tid == 0) srp[nrows] = M.rp[r0 + nrows];
    __syncthreads();
    const int32_t k0 = srp[0], k1 = srp[nrows];
    const bool has_row = tid < nrows;
    const int32_t rs = has_row ? srp[tid] : 0;
    const int32_t re = has_row ? srp[tid + 1] : 0;
    Acc acc = {0.0, 0.0};
    if constexpr (EPI == kEpiResid) {
        if (has_row) acc.p = ea.b[r0 + tid];
    }
    for (int32_t base = k0; base < k1; base += kChunk) {
        const int32_t cnt = min((int32_t)kChunk, k1 - base);
        for (int i = tid; i < cnt; i += kBlock) {
            const int32_t k = base + i;
            const double a = M.val[k];
            const double xv = x[M.ci[k]];
            double h = a * xv;
            double e = __fma_rn(a, xv, -h);
            if constexpr (EPI == kEpiResid) {
                h = -h;
                e = -e;
            }
            sh[i] = h;
            se[i] = e;
        }
        __syncthreads();
        const int32_t lo = max(rs, base), hi = min(re, base + cnt);
        for (int32_t k = lo; k < hi; ++k) acc_add_split(acc, sh[k - base], se[k - base]);
        __syncthreads();
    }
    Acc v[EpiNV<EPI>::value] = {};
    if (has_row) epilogue<EPI>(r0 + tid, acc_val(acc), y, ea, tl.st, v);
    block_finish<EpiNV<EPI>::value>(v, tl);
}

// ---------------------------------------------------------------------------
// W lanes per row (CSR with long rows, or the rows of a dense matrix).
// ---------------------------------------------------------------------------
template <int W, int EPI>
__global__ __launch_bounds__(kBlock) void k_rows_vector(MatView M, const double *__restrict__ x,
                                                         double *y, EpiArgs ea, Tail tl) {
    const int g = gate_of(tl);
    if (g == 0) return;
    if (g == 2) {
        if (blockIdx.x == 0 && threadIdx.x == 0) post_action(tl, 0.0, 0.0, false, nullptr);
        return;
    }
    constexpr int G = kBlock / W;
    const int tid = threadIdx.x;
    const int64_t blk = xcd_remap(blockIdx.x, gridDim.x);
    const int64_t row = blk * G + tid / W;
    const int lane = tid % W;
    Acc acc = {0.0, 0.0};
    if (row < M.rows) {
        if constexpr (EPI == kEpiResid) {
            if (lane == 0) acc.p = ea.b[row];
        }
        constexpr double sgn = (EPI == kEpiResid) ? -1.0 : 1.0;
        if (M.dense) {
            const double *a = M.val + row * M.ld;
            for (int64_t j = lane; j < M.cols; j += W) acc_fma(acc, sgn * a[j], x[j]);
        } else {
            const int32_t e = M.rp[row + 1];
            for (int32_t k = M.rp[row] + lane; k < e; k += W)
                acc_fma(acc, sgn * M.val[k], x[M.ci[k]]);
        }
    }
    acc = group_reduce<W>(acc);
    Acc v[EpiNV<EPI>::value] = {};
    if (row < M.rows && lane == 0) epilogue<EPI>(row, acc_val(acc), y, ea, tl.st, v);
    block_finish<EpiNV<EPI>::value>(v, tl);
}

// ---------------------------------------------------------------------------
// Dense A^T u: one thread per column of A, rows in order (coalesced across
// the threads of a wave because A is row-major).
// ---------------------------------------------------------------------------
template <int EPI>
__global__ __launch_bounds__(kBlock) void k_dense_cols(MatView M, const double *__restrict__ x,
                                                        double *y, EpiArgs ea, Tail tl) {
    const int g = gate_of(tl);
    if (g == 0) return;
    if (g == 2) {
        if (blockIdx.x == 0 && threadIdx.x == 0) post_action(tl, 0.0, 0.0, false, nullptr);
        return;
    }
    // M = A^T: M.rows = columns of A, M.cols = rows of A
    const int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    Acc acc = {0.0, 0.0};
    if (j < M.rows) {
        const double *a = M.val + j;
        for (int64_t i = 0; i < M.cols; ++i) acc_fma(acc, a[i * M.ld], x[i]);
    }
    Acc v[EpiNV<EPI>::value] = {};
    if (j < M.rows) epilogue<EPI>(j, acc_val(acc), y, ea, tl.st, v);
    block_finish<EpiNV<EPI>::value>(v, tl);
}

// ---------------------------------------------------------------------------
// element-wise kernels of the chains
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_cta_init(int64_t m, const double *__restrict__ b,
                                                      double *r, double *xy, int64_t nxy,
                                                      int32_t zero_xy, Tail tl) {
    Acc v[1] = {};
    const int64_t N = m > nxy ? m : nxy;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < N;
         i += (int64_t)gridDim.x * kBlock) {
        if (i < m) {
            const double bi = b[i];
            if (r != nullptr) r[i] = bi;
            acc_fma(v[0], bi, bi);
        }
        if (zero_xy && i < nxy) xy[i] = 0.0;
    }
    block_finish<1>(v, tl);
}

struct VecPtrs {
    double *p[kTMax + 1];
};

__global__ __launch_bounds__(kBlock) void k_cta_update(int64_t m, int64_t n, int32_t t,
                                                        int32_t minnorm, double *r, VecPtrs u,
                                                        double *x, VecPtrs w, double *y, Tail tl) {
    if (tl.st->done) return;
    double al[kTMax];
#pragma unroll
    for (int j = 0; j < kTMax; ++j) al[j] = j < t ? tl.st->alpha[j] : 0.0;
    Acc v[1] = {};
    const int64_t N = (minnorm || m > n) ? m : n;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < N;
         i += (int64_t)gridDim.x * kBlock) {
        if (i < m) {
            double ri = r[i];
            if (minnorm) {
                double yi = y[i];
                yi = __fma_rn(al[0], ri, yi);
                for (int j = 1; j < t; ++j) yi = __fma_rn(al[j], u.p[j][i], yi);
                y[i] = yi;
            }
            for (int j = 0; j < t; ++j) ri = __fma_rn(-al[j], u.p[j + 1][i], ri);
            r[i] = ri;
            acc_fma(v[0], ri, ri);
        }
        if (!minnorm && i < n) {
            double xi = x[i];
            for (int j = 0; j < t; ++j) xi = __fma_rn(al[j], w.p[j][i], xi);
            x[i] = xi;
        }
    }
    block_finish<1>(v, tl);
}

__global__ __launch_bounds__(kBlock) void k_ta_init(int64_t m, int64_t n,
                                                     const double *__restrict__ b, double *r,
                                                     double *bp, double *x, Tail tl) {
    Acc v[1] = {};
    const int64_t N = m > n ? m : n;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < N;
         i += (int64_t)gridDim.x * kBlock) {
        if (i < m) {
            const double bi = b[i];
            bp[i] = 0.0;
            r[i] = bi - 0.0;
            acc_fma(v[0], bi, bi);
        }
        if (i < n) x[i] = 0.0;
    }
    block_finish<1>(v, tl);
}

__global__ __launch_bounds__(kBlock) void k_ta_update(int64_t m, int64_t n,
                                                       const double *__restrict__ b, double *bp,
                                                       const double *__restrict__ d, double *r,
                                                       double *x, const double *__restrict__ c,
                                                       Tail tl) {
    const State *st = tl.st;
    if (st->done || !st->pivot) return;
    const double alpha = st->alpha_ta;
    const double beta = alpha * st->gamma;
    const double a1 = 1.0 - alpha;
    Acc v[2] = {};
    const int64_t N = m > n ? m : n;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < N;
         i += (int64_t)gridDim.x * kBlock) {
        if (i < m) {
            const double bpi = __fma_rn(alpha, d[i], bp[i]);
            bp[i] = bpi;
            const double bi = b[i];
            const double ri = bi - bpi;
            r[i] = ri;
            acc_fma(v[0], ri, ri);
            acc_fma(v[1], ri, bi);
        }
        if (i < n) x[i] = __fma_rn(beta, c[i], a1 * x[i]);
    }
    block_finish<2>(v, tl);
}

__global__ __launch_bounds__(kBlock) void k_copy_norm(int64_t n, const double *__restrict__ src,
                                                       double *dst, Tail tl) {
    Acc v[1] = {};
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kBlock) {
        const double s = src[i];
        if (dst != nullptr) dst[i] = s;
        acc_fma(v[0], s, s);
    }
    block_finish<1>(v, tl);
}

// ---------------------------------------------------------------------------
// CSR transpose: count, scan, scatter, per-row sort by source position.
// ---------------------------------------------------------------------------
__global__ void k_tr_count(int64_t nnz, const int32_t *__restrict__ ci, int32_t *cnt) {
    for (int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x; k < nnz;
         k += (int64_t)gridDim.x * kBlock)
        atomicAdd(&cnt[ci[k]], 1);
}

// Exclusive scan of cnt[0..n) into out[0..n] (out[n] = total), in three
// phases over tiles of 1024 entries.
constexpr int kScanTile = 1024;

__device__ int32_t block_scan_excl(int32_t v, int32_t *sh, int32_t &total) {
    // 256 threads; inclusive Hillis-Steele in LDS
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int off = 1; off < kBlock; off <<= 1) {
        const int32_t t = threadIdx.x >= off ? sh[threadIdx.x - off] : 0;
        __syncthreads();
        sh[threadIdx.x] += t;
        __syncthreads();
    }
    total = sh[kBlock - 1];
    const int32_t incl = sh[threadIdx.x];
    __syncthreads();
    return incl - v;
}

__global__ __launch_bounds__(kBlock) void k_scan_tiles(int64_t n, const int32_t *cnt,
                                                        int32_t *out, int32_t *tile_sums) {
    __shared__ int32_t sh[kBlock];
    const int64_t base = (int64_t)blockIdx.x * kScanTile + threadIdx.x * 4;
    int32_t v[4], s = 0;
    for (int q = 0; q < 4; ++q) {
        v[q] = (base + q < n) ? cnt[base + q] : 0;
        s += v[q];
    }
    int32_t total;
    int32_t ex = block_scan_excl(s, sh, total);
    for (int q = 0; q < 4; ++q) {
        if (base + q < n) out[base + q] = ex;
        ex += v[q];
    }
    if (threadIdx.x == 0) tile_sums[blockIdx.x] = total;
}

__global__ __launch_bounds__(kBlock) void k_scan_sums(int64_t ntiles, int32_t *tile_sums,
                                                       int32_t *total_out) {
    __shared__ int32_t sh[kBlock];
    int32_t carry = 0;
    for (int64_t base = 0; base < ntiles; base += kBlock) {
        const int64_t i = base + threadIdx.x;
        const int32_t v = i < ntiles ? tile_sums[i] : 0;
        int32_t total;
        const int32_t ex = block_scan_excl(v, sh, total);
        if (i < ntiles) tile_sums[i] = carry + ex;
        carry += total;
    }
    if (threadIdx.x == 0) *total_out = carry;
}

__global__ void k_scan_add(int64_t n, int32_t *out, const int32_t *tile_sums) {
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kBlock)
        out[i] += tile_sums[i / kScanTile];
}

__device__ __forceinline__ int64_t row_of(const int32_t *rp, int64_t m, int64_t k) {
    // last row r with rp[r] <= k (rows may be empty)
    int64_t lo = 0, hi = m;  // answer in [lo, hi)
    while (hi - lo > 1) {
        const int64_t mid = (lo + hi) >> 1;
        if (rp[mid] <= k)
            lo = mid;
        else
            hi = mid;
    }
    return lo;
}

__global__ void k_tr_scatter(int64_t m, int64_t nnz, const int32_t *__restrict__ rp,
                             const int32_t *__restrict__ ci, const int32_t *__restrict__ at_rp,
                             int32_t *fill, int32_t *src) {
    for (int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x; k < nnz;
         k += (int64_t)gridDim.x * kBlock) {
        const int32_t c = ci[k];
        const int32_t pos = at_rp[c] + atomicAdd(&fill[c], 1);
        src[pos] = (int32_t)k;
    }
}

// Sort each row of the transpose by source position; short rows by one
// thread, longer rows are listed for a block each.
__global__ void k_tr_sort_short(int64_t n, const int32_t *__restrict__ at_rp, int32_t *src,
                                int32_t *long_rows, int32_t *n_long, int32_t *flag) {
    for (int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x; j < n;
         j += (int64_t)gridDim.x * kBlock) {
        const int32_t s = at_rp[j], e = at_rp[j + 1], len = e - s;
        if (len > 32) {
            if (len > kMaxColNnz) atomicOr(flag, 1);
            long_rows[atomicAdd(n_long, 1)] = (int32_t)j;
            continue;
        }
        for (int32_t a = s + 1; a < e; ++a) {
            const int32_t key = src[a];
            int32_t b = a - 1;
            while (b >= s && src[b] > key) {
                src[b + 1] = src[b];
                --b;
            }
            src[b + 1] = key;
        }
    }
}

__global__ __launch_bounds__(kBlock) void k_tr_sort_long(const int32_t *__restrict__ at_rp,
                                                          int32_t *src,
                                                          const int32_t *__restrict__ long_rows,
                                                          const int32_t *__restrict__ n_long) {
    __shared__ int32_t key[kMaxColNnz];
    const int32_t cnt = *n_long;
    for (int32_t li = blockIdx.x; li < cnt; li += gridDim.x) {
        const int32_t j = long_rows[li];
        const int32_t s = at_rp[j], len = at_rp[j + 1] - s;
        if (len > kMaxColNnz) continue;  // reported through the flag
        int P = 1;
        while (P < len) P <<= 1;
        for (int i = threadIdx.x; i < P; i += kBlock) key[i] = i < len ? src[s + i] : INT32_MAX;
        __syncthreads();
        for (int size = 2; size <= P; size <<= 1) {
            for (int stride = size >> 1; stride > 0; stride >>= 1) {
                for (int i = threadIdx.x; i < P; i += kBlock) {
                    const int partner = i ^ stride;
                    if (partner > i) {
                        const bool up = ((i & size) == 0);
                        const int32_t a = key[i], b = key[partner];
                        if ((a > b) == up) {
                            key[i] = b;
                            key[partner] = a;
                        }
                    }
                }
                __syncthreads();
            }
        }
        for (int i = threadIdx.x; i < len; i += kBlock) src[s + i] = key[i];
        __syncthreads();
    }
}

__global__ void k_tr_fill(int64_t m, int64_t nnz, const int32_t *__restrict__ rp,
                          const double *__restrict__ val, const int32_t *__restrict__ src,
                          int32_t *at_ci, double *at_val) {
    for (int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x; p < nnz;
         p += (int64_t)gridDim.x * kBlock) {
        const int32_t k = src[p];
        at_ci[p] = (int32_t)row_of(rp, m, k);
        at_val[p] = val[k];
    }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
static inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

int64_t elementwise_blocks(int64_t n) {
    int64_t b = cdiv(n > 0 ? n : 1, kBlock);
    return b < 4096 ? b : 4096;
}

int64_t matvec_blocks(const MatView &M) {
    const int64_t rows = M.rows > 0 ? M.rows : 1;
    if (M.dense == 2) return cdiv(rows, kBlock);
    if (M.dense == 1 || M.lanes > 1) return cdiv(rows, kBlock / (M.lanes > 1 ? M.lanes : 64));
    return cdiv(rows, kBlock);
}

template <int EPI>
static void launch_vec_lanes(const MatView &M, dim3 grid, const double *x, double *y,
                             const EpiArgs &ea, const Tail &tl, hipStream_t s) {
    switch (M.lanes) {
        case 2: k_rows_vector<2, EPI><<<grid, kBlock, 0, s>>>(M, x, y, ea, tl); break;
        case 4: k_rows_vector<4, EPI><<<grid, kBlock, 0, s>>>(M, x, y, ea, tl); break;
        case 8: k_rows_vector<8, EPI><<<grid, kBlock, 0, s>>>(M, x, y, ea, tl); break;
        case 16: k_rows_vector<16, EPI><<<grid, kBlock, 0, s>>>(M, x, y, ea, tl); break;
        case 32: k_rows_vector<32, EPI><<<grid, kBlock, 0, s>>>(M, x, y, ea, tl); break;
        default: k_rows_vector<64, EPI><<<grid, kBlock, 0, s>>>(M, x, y, ea, tl); break;
    }
}

template <int EPI>
static void launch_matvec_t(const MatView &M, const double *x, double *y, const EpiArgs &ea,
                            const Tail &tl, hipStream_t s) {
    const dim3 grid((unsigned)matvec_blocks(M));
    if (M.dense == 2) {
        k_dense_cols<EPI><<<grid, kBlock, 0, s>>>(M, x, y, ea, tl);
    } else if (M.dense == 1) {
        MatView V = M;
        V.lanes = 64;
        launch_vec_lanes<EPI>(V, grid, x, y, ea, tl, s);
    } else if (M.lanes > 1) {
        launch_vec_lanes<EPI>(M, grid, x, y, ea, tl, s);
    } else {
        k_csr_stream<EPI><<<grid, kBlock, 0, s>>>(M, x, y, ea, tl);
    }
}

hipError_t launch_matvec(const MatView &M, const double *x, double *y, int32_t epi,
                         const EpiArgs &ea, const Tail &tl, hipStream_t s) {
    switch (epi) {
        case kEpiNorm: launch_matvec_t<kEpiNorm>(M, x, y, ea, tl, s); break;
        case kEpiResid: launch_matvec_t<kEpiResid>(M, x, y, ea, tl, s); break;
        case kEpiTaD: launch_matvec_t<kEpiTaD>(M, x, y, ea, tl, s); break;
        case kEpiTaBp: launch_matvec_t<kEpiTaBp>(M, x, y, ea, tl, s); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_cta_init(int64_t m, int64_t n, const double *b, double *r, double *xy,
                           int64_t nxy, int32_t zero_xy, const Tail &tl, hipStream_t s) {
    (void)n;
    const dim3 grid((unsigned)elementwise_blocks(m > nxy ? m : nxy));
    k_cta_init<<<grid, kBlock, 0, s>>>(m, b, r, xy, nxy, zero_xy, tl);
    return hipGetLastError();
}

hipError_t launch_cta_update(int64_t m, int64_t n, int32_t t, int32_t minnorm, double *r,
                             double *const *u, double *x, double *const *w, double *y,
                             const Tail &tl, hipStream_t s) {
    VecPtrs U{}, Wp{};
    for (int j = 0; j <= t && j <= kTMax; ++j) U.p[j] = u[j];
    for (int j = 0; j < t && j < kTMax; ++j) Wp.p[j] = w ? w[j] : nullptr;
    const int64_t N = (minnorm || m > n) ? m : n;
    const dim3 grid((unsigned)elementwise_blocks(N));
    k_cta_update<<<grid, kBlock, 0, s>>>(m, n, t, minnorm, r, U, x, Wp, y, tl);
    return hipGetLastError();
}

hipError_t launch_ta_init(int64_t m, int64_t n, const double *b, double *r, double *bp,
                          double *x, const Tail &tl, hipStream_t s) {
    const dim3 grid((unsigned)elementwise_blocks(m > n ? m : n));
    k_ta_init<<<grid, kBlock, 0, s>>>(m, n, b, r, bp, x, tl);
    return hipGetLastError();
}

hipError_t launch_ta_update(int64_t m, int64_t n, const double *b, double *bp, const double *d,
                            double *r, double *x, const double *c, const Tail &tl,
                            hipStream_t s) {
    const dim3 grid((unsigned)elementwise_blocks(m > n ? m : n));
    k_ta_update<<<grid, kBlock, 0, s>>>(m, n, b, bp, d, r, x, c, tl);
    return hipGetLastError();
}

hipError_t launch_copy_norm(int64_t n, const double *src, double *dst, const Tail &tl,
                            hipStream_t s) {
    const dim3 grid((unsigned)elementwise_blocks(n));
    k_copy_norm<<<grid, kBlock, 0, s>>>(n, src, dst, tl);
    return hipGetLastError();
}

// work: 4 * n + 2 * ntiles + 8 int32 entries (fill, src(nnz) separately)
hipError_t launch_transpose(int64_t m, int64_t n, int64_t nnz, const int32_t *rp,
                            const int32_t *ci, const double *val, int32_t *at_rp,
                            int32_t *at_ci, double *at_val, int32_t *work, int32_t *flag,
                            hipStream_t s) {
    // work layout: cnt/fill [n], long_rows [n], tile sums [ntiles], n_long [1], src [nnz]
    const int64_t ntiles = cdiv(n > 0 ? n : 1, kScanTile);
    int32_t *cnt = work;
    int32_t *long_rows = cnt + n;
    int32_t *tiles = long_rows + n;
    int32_t *n_long = tiles + ntiles;
    int32_t *src = n_long + 8;
    hipError_t e;
    if ((e = hipMemsetAsync(cnt, 0, sizeof(int32_t) * (size_t)n, s)) != hipSuccess) return e;
    if ((e = hipMemsetAsync(n_long, 0, sizeof(int32_t), s)) != hipSuccess) return e;
    if ((e = hipMemsetAsync(flag, 0, sizeof(int32_t), s)) != hipSuccess) return e;
    const dim3 gn((unsigned)elementwise_blocks(nnz));
    if (nnz > 0) k_tr_count<<<gn, kBlock, 0, s>>>(nnz, ci, cnt);
    k_scan_tiles<<<(unsigned)ntiles, kBlock, 0, s>>>(n, cnt, at_rp, tiles);
    k_scan_sums<<<1, kBlock, 0, s>>>(ntiles, tiles, at_rp + n);
    k_scan_add<<<(unsigned)elementwise_blocks(n), kBlock, 0, s>>>(n, at_rp, tiles);
    if ((e = hipMemsetAsync(cnt, 0, sizeof(int32_t) * (size_t)n, s)) != hipSuccess) return e;
    if (nnz > 0) k_tr_scatter<<<gn, kBlock, 0, s>>>(m, nnz, rp, ci, at_rp, cnt, src);
    k_tr_sort_short<<<(unsigned)elementwise_blocks(n), kBlock, 0, s>>>(n, at_rp, src, long_rows,
                                                                        n_long, flag);
    k_tr_sort_long<<<1024, kBlock, 0, s>>>(at_rp, src, long_rows, n_long);
    if (nnz > 0) k_tr_fill<<<gn, kBlock, 0, s>>>(m, nnz, rp, val, src, at_ci, at_val);
    return hipGetLastError();
}

}  // namespace ta
