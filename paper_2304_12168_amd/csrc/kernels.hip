// Device kernels of libta (gfx950, wave64).
//
// Every kernel of an iteration chain reads the solver State at entry and
// returns at once when the chain is finished, so the host can enqueue many
// iterations ahead and read one flag per chunk.  Reductions are fused into
// the kernel that produces the vector: each block reduces its part with
// compensated (double-double) arithmetic and writes one partial per value
// with a plain store.  A one-block step kernel, launched next on the same
// stream, reduces the partials in block order and runs the scalar logic of
// the method (Gram solve, stop tests, TA pivot test).  There are no atomics
// and no cross-block fences on this path (on a multi-XCD part an agent-scope
// fence writes back the whole L2), and no floating-point atomics anywhere,
// so every result is run-to-run reproducible.
//
// Compensated arithmetic: TwoSum (Knuth) and TwoProduct via fma, combined as
// in Dot2 of Ogita, Rump and Oishi (SIAM J. Sci. Comput. 26, 2005).  Built
// with -ffp-contract=off: every fma below is explicit.
#include <math.h>

#include "common.hpp"
#include "device_math.hpp"

namespace ta {

// ---------------------------------------------------------------------------
// Scalar step logic run by thread 0 of a step kernel.
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

__device__ void post_action(const Step &sp, const double *v, bool computed) {
    State *st = sp.st;
    switch (sp.post) {
        case kPostNone:
            break;
        case kPostStore:
            for (int i = 0; i < sp.nslots && sp.arg + i < 4; ++i) st->scratch[sp.arg + i] = v[i];
            break;
        case kPostCtaInit:
        case kPostTaInit: {
            const double nb = sqrt(v[0]);
            st->nb = nb;
            st->tol_nb = st->tol * nb;
            st->rr = v[0];
            st->rb = v[0];
            st->k = 0;
            if (nb == 0.0) {
                if (sp.hist != nullptr && st->hist_cap > 0) sp.hist[0] = 0.0;
                finish(st, TA_STOP_RESIDUAL);
                break;
            }
            if (sp.arg == 0) {  // arg = 1: a warm start recomputes r next
                put_hist(st, sp.hist);
                loop_top(st);
            }
            break;
        }
        case kPostCtaWarm:
            st->rr = v[0];
            st->matvecs++;
            put_hist(st, sp.hist);
            loop_top(st);
            break;
        case kPostNab:
            st->nab = sqrt(v[0]);
            st->tol_ne_nab = st->tol_normal * st->nab;
            st->matvecs += st->pm;
            break;
        case kPostGram: {
            if (sp.arg > 0) st->t = sp.arg;  // order of this iteration (order cycling)
            const int t = st->t;
            for (int i = 0; i < 2 * t; ++i) st->phi[i + 1] = v[i];
            // H = A A^T: 2t products, phi_1 = ||A^T r||^2; H = A: t products, phi_2 = ||A r||^2
            st->matvecs += st->hmode ? t : 2 * t;
            for (int i = 1; i <= 2 * t; ++i)
                if (!isfinite(st->phi[i])) {
                    finish(st, TA_STOP_BREAKDOWN);
                    return;
                }
            const double nr = sqrt(st->hmode ? st->phi[2] : st->phi[1]);
            if (nr <= st->tol_ne_nab || st->phi[2] == 0.0) {
                finish(st, TA_STOP_NORMAL);
                return;
            }
            double phi[2 * kTMax + 2];
            for (int i = 0; i <= 2 * t; ++i) phi[i] = st->phi[i];
            double a[kTMax];
            if (st->enhanced && t >= 2 && st->tol_ne_nab > 0.0) {
                double beta[kTMax];
                if (enhanced_hit(phi, t, st->hmode, st->tol_ne_nab, beta)) {
                    for (int i = 0; i < t; ++i) st->alpha[i] = beta[i];
                    st->enh_hit = 1;
                    return;
                }
            }
            gram_alpha(phi, t, a);
            for (int i = 0; i < t; ++i)
                if (!isfinite(a[i])) {
                    finish(st, TA_STOP_BREAKDOWN);
                    return;
                }
            for (int i = 0; i < t; ++i) st->alpha[i] = a[i];
            break;
        }
        case kPostCtaEnd: {
            const double rr_old = st->rr;
            st->rr = v[0];
            st->k++;
            put_hist(st, sp.hist);
            if (st->enh_hit) {
                finish(st, TA_STOP_NORMAL);  // the update just applied x^ (enhanced stop)
                break;
            }
            // convex-combination step: ||r_{k+1}|| / ||r_k|| = rho >= accel, and
            // the current pair is two steps of F_t (not after such a step)
            int32_t jump = 0;
            if (st->accel > 0.0) {
                const double rho = rr_old > 0.0 ? sqrt(st->rr / rr_old) : 0.0;
                if (!st->last_jump && rho >= st->accel) {
                    jump = 1;
                    st->astar = rho / (rho + 1.0);
                } else {
                    st->last_jump = 0;
                }
            }
            st->jump = jump;
            if (st->replace_every > 0 && st->k % st->replace_every == 0)
                st->replace = 1;
            else if (!jump)
                loop_top(st);
            break;
        }
        case kPostCtaJump:
            st->rr = v[0];
            st->jump = 0;
            st->last_jump = 1;
            put_hist(st, sp.hist);
            if (!st->replace) loop_top(st);
            break;
        case kPostCtaReplace:
            st->rr = v[0];
            st->replace = 0;
            st->matvecs += sp.arg;
            loop_top(st);
            break;
        case kPostCtaCand:
            st->matvecs += sp.arg;
            st->rr = v[0];
            if (sqrt(v[0]) <= st->tol_nb) {
                finish(st, TA_STOP_RESIDUAL);
            } else {
                st->done = 0;
                st->stop = 0;
                st->rejects++;
                if (st->k >= st->max_iter) finish(st, TA_STOP_MAXITER);
            }
            break;
        case kPostTaC: {
            if (computed) {
                st->nc = sqrt(v[0]);
                st->have_c = 1;
                st->matvecs += st->pm;
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
                const double grown = (2.0 * st->rho >= q) ? 2.0 * st->rho : q;
                if (st->rho_max > 0.0 && grown > st->rho_max) {
                    finish(st, TA_STOP_WITNESS);  // no solution within the radius bound
                    break;
                }
                st->pass = (q >= 2.0 * st->rho);
                st->rho = (2.0 * st->rho >= q) ? 2.0 * st->rho : q;
                st->k++;
                put_hist(st, sp.hist);
                loop_top(st);
            }
            break;
        }
        case kPostTaS: {
            st->matvecs += st->pm;
            const double rd = v[0], dd = v[1];
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
            st->rr = v[0];
            st->rb = v[1];
            st->pass = 0;
            st->have_c = 0;
            st->pivot = 0;
            st->k++;
            put_hist(st, sp.hist);
            loop_top(st);
            break;
        case kPostTaCand:
            st->matvecs += st->pm;
            if (sqrt(v[0]) <= st->tol_nb) {
                finish(st, TA_STOP_RESIDUAL);
            } else {
                st->done = 0;
                st->stop = 0;
                st->rejected = 1;
                st->rejects++;
            }
            break;
        case kPostTaWarm:  // warm start: b' = A x, r = b - b'
            st->matvecs += st->pm;
            st->rr = v[0];
            st->rb = v[1];
            st->have_c = 0;
            put_hist(st, sp.hist);
            loop_top(st);
            break;
        case kPostTaBp:
            st->matvecs += st->pm;
            st->rr = v[0];
            st->rb = v[1];
            st->have_c = 0;
            st->rejected = 0;
            if (st->k >= st->max_iter) finish(st, TA_STOP_MAXITER);
            break;
        default:
            break;
    }
}

// Producers: run unless the chain says otherwise.
__device__ __forceinline__ bool gate_open(int32_t gate, const State *st) {
    switch (gate) {
        case kGateIgnoreDone: return true;
        case kGateCandidate: return st->done && st->stop == kStopCandidate;
        case kGateFinal: return st->done && st->stop != kStopCandidate;
        default: break;
    }
    if (st->done) return false;
    if (gate == kGatePivot && !st->pivot) return false;
    if (gate == kGateReplace && !st->replace) return false;
    if (gate == kGateRejected && !st->rejected) return false;
    if (gate == kGateJump && !st->jump) return false;
    return true;
}

__device__ __forceinline__ bool producer_runs(const Out &o) {
    if (!gate_open(o.gate, o.st)) return false;
    if (o.gate == kGateNeedC && o.st->have_c) return false;
    return true;
}

// Block-reduce NV values and write one partial each (thread 0, plain stores).
template <int NV>
__device__ void block_partials(Acc (&v)[NV], const Out &o, int64_t bidx = -1) {
    __shared__ Acc red[2][kBlock / 64];
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
            o.partials[(int64_t)(o.slot + q) * o.cap + (bidx < 0 ? (int64_t)blockIdx.x : bidx)] =
                make_double2(a.p, a.s);
        }
    }
}

// One block: reduce the listed slots in a fixed order, then the step logic.
__global__ __launch_bounds__(kBlock) void k_step(Step sp) {
    const State *st = sp.st;
    if (!gate_open(sp.gate, st)) return;
    const bool computed = !(sp.gate == kGateNeedC && st->have_c);
    __shared__ double vals[kMaxSlots];
    __shared__ Acc red[kBlock / 64];
    // The scalar logic runs on a copy of the state in LDS: one coalesced load
    // of it here, one store after, instead of the one thread's chain of
    // dependent global reads and writes.
    __shared__ State sst;
    constexpr int kStateWords = (int)(sizeof(State) / sizeof(int32_t));
    static_assert(sizeof(State) % sizeof(int32_t) == 0, "State is copied as 32-bit words");
    for (int i = threadIdx.x; i < kStateWords; i += kBlock)
        reinterpret_cast<int32_t *>(&sst)[i] = reinterpret_cast<const int32_t *>(st)[i];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (computed) {
        for (int q = 0; q < sp.nslots; ++q) {
            const double2 *p = sp.partials + (int64_t)(sp.slot0 + q) * sp.cap;
            const int cnt = sp.count[q];
            Acc a = {0.0, 0.0};
            // thread i takes partials i, i + 256, i + 512, ... in that order;
            // eight loads are issued before the merges that consume them
            for (int base = threadIdx.x; base < cnt; base += 8 * kBlock) {
                double2 d[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const int i = base + u * kBlock;
                    d[u] = i < cnt ? p[i] : make_double2(0.0, 0.0);
                }
#pragma unroll
                for (int u = 0; u < 8; ++u)
                    if (base + u * kBlock < cnt) a = acc_merge(a, Acc{d[u].x, d[u].y});
            }
            a = group_reduce<64>(a);
            if (lane == 0) red[wave] = a;
            __syncthreads();
            if (threadIdx.x == 0) {
                Acc b = red[0];
                for (int w = 1; w < kBlock / 64; ++w) b = acc_merge(b, red[w]);
                vals[q] = acc_val(b);
            }
            __syncthreads();
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        Step sl = sp;
        sl.st = &sst;
        post_action(sl, vals, computed);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < kStateWords; i += kBlock)
        reinterpret_cast<int32_t *>(sp.st)[i] = reinterpret_cast<const int32_t *>(&sst)[i];
}

template <int EPI>
struct EpiNV {
    static constexpr int value = (EPI == kEpiTaD || EPI == kEpiTaBp || EPI == kEpiNormDot) ? 2 : 1;
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
    } else if constexpr (EPI == kEpiNormPos) {
        const double yp = yv > 0.0 ? yv : 0.0;
        y[row] = yp;
        acc_fma(v[0], yp, yp);
    } else if constexpr (EPI == kEpiNormDot) {
        y[row] = yv;
        acc_fma(v[0], ea.r[row], yv);
        acc_fma(v[1], yv, yv);
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
                                                        double *y, EpiArgs ea, Out o) {
    if (!producer_runs(o)) return;
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
        for (int i0 = tid; i0 < cnt; i0 += 4 * kBlock) {
            int32_t c[4];
            double a[4], xv[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int i = i0 + u * kBlock;
                c[u] = i < cnt ? __builtin_nontemporal_load(M.ci + base + i) : 0;
                a[u] = i < cnt ? __builtin_nontemporal_load(M.val + base + i) : 0.0;
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) xv[u] = x[c[u]];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int i = i0 + u * kBlock;
                if (i < cnt) {
                    double h = a[u] * xv[u];
                    double e = __fma_rn(a[u], xv[u], -h);
                    if constexpr (EPI == kEpiResid) {
                        h = -h;
                        e = -e;
                    }
                    sh[i] = h;
                    se[i] = e;
                }
            }
        }
        __syncthreads();
        const int32_t lo = max(rs, base), hi = min(re, base + cnt);
        for (int32_t k = lo; k < hi; ++k) acc_add_split(acc, sh[k - base], se[k - base]);
        __syncthreads();
    }
    Acc v[EpiNV<EPI>::value] = {};
    if (has_row) epilogue<EPI>(r0 + tid, acc_val(acc), y, ea, o.st, v);
    block_partials<EpiNV<EPI>::value>(v, o);
}

// ---------------------------------------------------------------------------
// SELL-64: one thread per row, the 64 rows of a slice in one wave.  A slice's
// entries are stored position by position (64 slots each), so every column
// index and value load of the wave is one contiguous access and no row bound
// is loaded.  Terms are added in storage order with the compensated steps of
// k_csr_stream, so both give the same bits.  Up to 6 positions are loaded
// before the first gather (the width is uniform over the wave).  NT: the
// slots are read with non-temporal loads (a separate instantiation: a run-time
// choice between the two loads is merged into one plain load by the compiler).
// ---------------------------------------------------------------------------
template <int EPI, bool NT>
__global__ __launch_bounds__(kBlock) void k_sell(MatView M, const double *__restrict__ x,
                                                  double *y, EpiArgs ea, Out o) {
    if (!producer_runs(o)) return;
    constexpr double sgn = (EPI == kEpiResid) ? -1.0 : 1.0;
    constexpr int UN = 6;
    const int64_t blk = xcd_remap(blockIdx.x, gridDim.x);
    const int64_t row = blk * kBlock + threadIdx.x;
    const int64_t slice = row >> 6;
    const int lane = threadIdx.x & 63;
    Acc acc = {0.0, 0.0};
    if constexpr (EPI == kEpiResid) {
        if (row < M.rows) acc.p = ea.b[row];
    }
    if (slice < ((M.rows + 63) >> 6)) {
        const int64_t off = M.so[slice];
        const int32_t w = (int32_t)((M.so[slice + 1] - off) >> 6);
        const int32_t *__restrict__ c = M.sc + off + lane;
        const double *__restrict__ a = M.sv + off + lane;
        for (int32_t k = 0; k < w; k += UN) {
            int32_t cc[UN];
            double aa[UN], xv[UN];
#pragma unroll
            for (int u = 0; u < UN; ++u) {
                cc[u] = -1;
                aa[u] = 0.0;
                if (k + u < w) {
                    if constexpr (NT) {
                        cc[u] = __builtin_nontemporal_load(c + (int64_t)(k + u) * 64);
                        aa[u] = __builtin_nontemporal_load(a + (int64_t)(k + u) * 64);
                    } else {
                        cc[u] = c[(int64_t)(k + u) * 64];
                        aa[u] = a[(int64_t)(k + u) * 64];
                    }
                }
            }
#pragma unroll
            for (int u = 0; u < UN; ++u) xv[u] = cc[u] >= 0 ? x[cc[u]] : 0.0;
#pragma unroll
            for (int u = 0; u < UN; ++u)
                if (cc[u] >= 0) acc_fma(acc, sgn * aa[u], xv[u]);
        }
    }
    Acc v[EpiNV<EPI>::value] = {};
    if (row < M.rows) epilogue<EPI>(row, acc_val(acc), y, ea, o.st, v);
    block_partials<EpiNV<EPI>::value>(v, o);
}

// widest row of each 64-row slice (one wave per slice)
__global__ __launch_bounds__(kBlock) void k_sell_widths(int64_t rows,
                                                         const int32_t *__restrict__ rp,
                                                         int32_t *w) {
    const int64_t r = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    int32_t len = r < rows ? rp[r + 1] - rp[r] : 0;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) len = max(len, __shfl_xor(len, off));
    if ((threadIdx.x & 63) == 0 && r < rows) w[r >> 6] = len;
}

// every slot of every slice written once: a row's entries, then padding
__global__ __launch_bounds__(kBlock) void k_sell_fill(int64_t rows,
                                                       const int32_t *__restrict__ rp,
                                                       const int32_t *__restrict__ ci,
                                                       const double *__restrict__ val,
                                                       const int64_t *__restrict__ so,
                                                       int32_t *sc, double *sv) {
    const int64_t r = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int64_t s = r >> 6;
    if (s >= ((rows + 63) >> 6)) return;
    const int lane = (int)(r & 63);
    const int64_t off = so[s];
    const int32_t w = (int32_t)((so[s + 1] - off) >> 6);
    int32_t k0 = 0, len = 0;
    if (r < rows) {
        k0 = rp[r];
        len = rp[r + 1] - k0;
    }
    for (int32_t k = 0; k < w; ++k) {
        const int64_t e = off + (int64_t)k * 64 + lane;
        if (k < len) {
            sc[e] = ci[k0 + k];
            sv[e] = val[k0 + k];
        } else {
            sc[e] = -1;
            sv[e] = 0.0;
        }
    }
}

// ---------------------------------------------------------------------------
// W lanes per row (CSR with long rows, or the rows of a dense matrix).
// ---------------------------------------------------------------------------
template <int W, int EPI>
__global__ __launch_bounds__(kBlock) void k_rows_vector(MatView M, const double *__restrict__ x,
                                                         double *y, EpiArgs ea, Out o) {
    if (!producer_runs(o)) return;
    constexpr int G = kBlock / W;
    constexpr double sgn = (EPI == kEpiResid) ? -1.0 : 1.0;
    const int tid = threadIdx.x;
    const int64_t blk = xcd_remap(blockIdx.x, gridDim.x);
    const int64_t row = blk * G + tid / W;
    const int lane = tid % W;
    Acc acc = {0.0, 0.0};
    if (row < M.rows) {
        if constexpr (EPI == kEpiResid) {
            if (lane == 0) acc.p = ea.b[row];
        }
        // rounds of U entries per lane, predicated on the row end, a lane's
        // terms summed in storage order (j, j + W, j + 2W, ...)
        constexpr int U = 8;
        if (M.kind == kDenseRows) {
            const double *a = M.val + row * M.ld;
            for (int64_t j0 = lane; j0 < M.cols; j0 += U * W) {
                double av[U], xv[U];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int64_t j = j0 + u * W;
                    av[u] = j < M.cols ? a[j] : 0.0;
                    xv[u] = j < M.cols ? x[j] : 0.0;
                }
#pragma unroll
                for (int u = 0; u < U; ++u)
                    if (j0 + u * W < M.cols) acc_fma(acc, sgn * av[u], xv[u]);
            }
        } else {
            const int32_t e = M.rp[row + 1];
            for (int32_t k0 = M.rp[row] + lane; k0 < e; k0 += U * W) {
                int32_t c[U];
                double av[U], xv[U];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int32_t k = k0 + u * W;
                    c[u] = -1;
                    av[u] = 0.0;
                    if (k < e) {
                        c[u] = M.ci[k];
                        av[u] = M.val[k];
                    }
                }
#pragma unroll
                for (int u = 0; u < U; ++u) xv[u] = c[u] >= 0 ? x[c[u]] : 0.0;
#pragma unroll
                for (int u = 0; u < U; ++u)
                    if (c[u] >= 0) acc_fma(acc, sgn * av[u], xv[u]);
            }
        }
    }
    acc = group_reduce<W>(acc);
    Acc v[EpiNV<EPI>::value] = {};
    if (row < M.rows && lane == 0) epilogue<EPI>(row, acc_val(acc), y, ea, o.st, v);
    block_partials<EpiNV<EPI>::value>(v, o);
}

// ---------------------------------------------------------------------------
// CSR split into nsl = 8 g column slices, each of a few MB of x.
// Blocks go in g groups of 8 slices: block b takes XCD lane b % 8 (its XCD
// under round-robin dispatch), group (b / 8) / RB and row block (b / 8) % RB,
// so while a group runs each XCD gathers only from its own slice of x, which
// stays in that XCD's L2 (or close to it) and the Infinity Cache.  The matrix stream is read non-temporally so it does
// not evict the slice of x.  Each (row, slice) partial is kept as an
// unrounded compensated pair; the combine kernel merges the slices of a row
// in slice order and runs the epilogue.
// ---------------------------------------------------------------------------
template <int W, int EPI>
__global__ __launch_bounds__(kBlock) void k_rows_sliced(MatView M, const double *__restrict__ x,
                                                         EpiArgs ea, Out o) {
    if (!producer_runs(o)) return;
    constexpr int G = kBlock / W;
    constexpr double sgn = (EPI == kEpiResid) ? -1.0 : 1.0;
    const int tid = threadIdx.x;
    const int64_t RB = (M.rows + G - 1) / G;
    const int64_t t = blockIdx.x / kSlices;
    const int slice = (int)((t / RB) * kSlices + blockIdx.x % kSlices);
    const int64_t row = (t % RB) * G + tid / W;
    const int lane = tid % W;
    if (row >= M.rows) return;  // no block-wide synchronisation below
    Acc acc = {0.0, 0.0};
    if constexpr (EPI == kEpiResid) {
        if (slice == 0 && lane == 0) acc.p = ea.b[row];
    }
    const int32_t *sg = M.seg + row * (M.nsl + 1) + slice;
    const int32_t e = sg[1];
    // Rounds of U entries per lane, each entry predicated on the segment end:
    // a segment of up to U W entries takes one round, i.e. one wait for the
    // index and value loads and one for the gathers.  A lane's terms are still
    // summed in storage order (k, k + W, k + 2W, ...).
    constexpr int U = 8;
    for (int32_t k0 = sg[0] + lane; k0 < e; k0 += U * W) {
        int32_t c[U];
        double a[U], xv[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int32_t k = k0 + u * W;
            c[u] = -1;
            a[u] = 0.0;
            if (k < e) {
                c[u] = __builtin_nontemporal_load(M.ci + k);
                a[u] = __builtin_nontemporal_load(M.val + k);
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) xv[u] = c[u] >= 0 ? x[c[u]] : 0.0;
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (c[u] >= 0) acc_fma(acc, sgn * a[u], xv[u]);
    }
    acc = group_reduce<W>(acc);
    if (lane == 0) M.ypart[(int64_t)slice * M.rows + row] = make_double2(acc.p, acc.s);
}

template <int EPI>
__global__ __launch_bounds__(kBlock) void k_slices_combine(MatView M, double *y, EpiArgs ea,
                                                            Out o) {
    if (!producer_runs(o)) return;
    Acc v[EpiNV<EPI>::value] = {};
    for (int64_t row = (int64_t)blockIdx.x * kBlock + threadIdx.x; row < M.rows;
         row += (int64_t)gridDim.x * kBlock) {
        double2 p = M.ypart[row];
        Acc a = {p.x, p.y};
        for (int sl = 1; sl < M.nsl; ++sl) {
            p = M.ypart[(int64_t)sl * M.rows + row];
            a = acc_merge(a, Acc{p.x, p.y});
        }
        epilogue<EPI>(row, acc_val(a), y, ea, o.st, v);
    }
    block_partials<EpiNV<EPI>::value>(v, o);
}

// ---------------------------------------------------------------------------
// Column tiles staged in LDS (kCsrTiled).  A block copies one tile of x
// (kTileW consecutive entries, coalesced) into LDS and then walks the runs
// of its chunk of rows inside that tile, W lanes per row, gathering from
// LDS: the gathers no longer cost one L2 request per nonzero.  The blocks of
// one tile are consecutive logical blocks, hence on one XCD, so the tile is
// fetched from memory once per XCD and re-read from its L2.  The entries
// and their 16-bit local columns are read non-temporally.  Each
// (tile, row) partial is an unrounded compensated pair; the combine kernel
// merges a row's tiles and runs the epilogue.
// ---------------------------------------------------------------------------
// One batch of a tiled block (tile_pr(W) row passes): the run bounds of
// every pass, then rounds of tile_u(W) entries per lane for all passes at
// once until every run is done (a row of n entries takes ceil(n / (U W))
// rounds), then the group reductions and the partial stores.  `stage` runs
// between the first round's loads and its use of the LDS tile (the first
// batch copies the tile there while its loads are in flight).  A lane's
// terms are summed in storage order (k, k + W, ...); the W lanes of a row
// stay together, so the group reduction sees all of them.
template <int W, int EPI, class Stage>
__device__ __forceinline__ void tiled_batch(const MatView &M, const int32_t *rp, double2 *yp,
                                            const double *xs, int64_t rb, int64_t r1, int lane,
                                            Stage &&stage) {
    constexpr int G = kTileBlock / W, U = tile_u(W), PR = tile_pr(W);
    constexpr double sgn = (EPI == kEpiResid) ? -1.0 : 1.0;
    int32_t sk[PR], ek[PR];
#pragma unroll
    for (int p = 0; p < PR; ++p) {
        const int64_t row = rb + p * G;
        sk[p] = row < r1 ? rp[row] : 0;
        ek[p] = row < r1 ? rp[row + 1] : 0;
    }
    Acc acc[PR];
#pragma unroll
    for (int p = 0; p < PR; ++p) acc[p] = Acc{0.0, 0.0};
    bool first = true;
    for (int32_t off = lane;; off += U * W) {
        int cl[PR][U];
        double a[PR][U];
        bool more = false;
#pragma unroll
        for (int p = 0; p < PR; ++p) {
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int32_t k = sk[p] + off + u * W;
                cl[p][u] = -1;
                a[p][u] = 0.0;
                if (k < ek[p]) {
                    cl[p][u] = (int)__builtin_nontemporal_load(M.lc + k);
                    a[p][u] = __builtin_nontemporal_load(M.val + k);
                }
            }
            more |= sk[p] + (off - lane) + U * W < ek[p];
        }
        if (first) {
            stage();
            first = false;
        }
#pragma unroll
        for (int p = 0; p < PR; ++p)
#pragma unroll
            for (int u = 0; u < U; ++u)
                if (cl[p][u] >= 0) acc_fma(acc[p], sgn * a[p][u], xs[cl[p][u]]);
        if (!more) break;
    }
#pragma unroll
    for (int p = 0; p < PR; ++p) {
        const int64_t row = rb + p * G;
        if (row < r1) {
            const Acc v = group_reduce<W>(acc[p]);
            if (lane == 0) yp[row] = make_double2(v.p, v.s);
        }
    }
}

template <int W, int EPI>
__global__ __launch_bounds__(kTileBlock) void k_rows_tiled(MatView M, const double *__restrict__ x,
                                                            Out o) {
    __shared__ double xs[kTileW];
    if (!producer_runs(o)) return;
    const int64_t L = xcd_remap(blockIdx.x, gridDim.x);
    const int64_t q = L / M.nchunk;
    const int64_t c0 = q * kTileW;
    const int wq = (int)min((int64_t)kTileW, M.cols - c0);
    constexpr int NS = kTileW / kTileBlock;
    double t[NS];
#pragma unroll
    for (int i = 0; i < NS; ++i) {
        const int j = (int)threadIdx.x + i * kTileBlock;
        t[i] = j < wq ? x[c0 + j] : 0.0;
    }
    const int lane = threadIdx.x % W;
    const int64_t r0 = (L % M.nchunk) * M.rchunk;
    const int64_t r1 = min(M.rows, r0 + M.rchunk);
    const int32_t *rp = M.rp + q * M.rows;
    double2 *yp = M.ypart + q * M.rows;
    // the first batch: every thread takes part (rows past r1 predicated off)
    // because the block-wide barrier that publishes the tile sits inside it
    const int64_t rb0 = r0 + threadIdx.x / W;
    tiled_batch<W, EPI>(M, rp, yp, xs, rb0, r1, lane, [&] {
#pragma unroll
        for (int i = 0; i < NS; ++i) xs[threadIdx.x + i * kTileBlock] = t[i];
        __syncthreads();
    });
    for (int64_t rb = rb0 + tile_batch_rows(W); rb < r1; rb += tile_batch_rows(W))
        tiled_batch<W, EPI>(M, rp, yp, xs, rb, r1, lane, [] {});
}

// kCombineLanes lanes per row: lane l merges the partials of tiles l,
// l + kCombineLanes, ... in tile order, the lanes are merged by the group
// reduction, then (for the residual) b is merged in front.
constexpr int kCombineLanes = 8;

template <int EPI>
__global__ __launch_bounds__(kBlock) void k_tiles_combine(MatView M, double *y, EpiArgs ea,
                                                           Out o) {
    if (!producer_runs(o)) return;
    constexpr int CW = kCombineLanes;
    constexpr int U = 8;
    const int lane = threadIdx.x % CW;
    const int64_t row = (int64_t)blockIdx.x * (kBlock / CW) + threadIdx.x / CW;
    Acc a = {0.0, 0.0};
    if (row < M.rows) {
        for (int64_t q0 = lane; q0 < M.nt; q0 += U * CW) {
            double2 p[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int64_t q = q0 + u * CW;
                p[u] = q < M.nt ? M.ypart[q * M.rows + row] : make_double2(0.0, 0.0);
            }
#pragma unroll
            for (int u = 0; u < U; ++u)
                if (q0 + u * CW < M.nt) a = acc_merge(a, Acc{p[u].x, p[u].y});
        }
    }
    a = group_reduce<CW>(a);
    Acc v[EpiNV<EPI>::value] = {};
    if (row < M.rows && lane == 0) {
        if constexpr (EPI == kEpiResid) a = acc_merge(Acc{ea.b[row], 0.0}, a);
        epilogue<EPI>(row, acc_val(a), y, ea, o.st, v);
    }
    block_partials<EpiNV<EPI>::value>(v, o);
}

// ---------------------------------------------------------------------------
// Merge-path CSR product for skewed row lengths (kCsrMerge; the merge-based
// SpMV of Merrill and Garland, SC 2016, restated).  The path merges the row
// ends with the nonzeros: item d of the path is either nonzero k or the end
// of row i, where i + k = d and a row's end follows its last nonzero.  Block
// b takes the kMergeItems items from b kMergeItems on (its first row is
// mp[b], from the plan), and each of its threads kMergeIpt of them, so a long
// row is shared by many threads and a thread crosses many short rows.
//
// A block stages its nonzeros' exact products (TwoProduct) and its row
// pointers in LDS.  A thread sums each row it meets in storage order
// (compensated).  A row that began in an earlier thread and ends here is the
// thread's head; the row it is in when its items run out is its carry.  A
// segmented scan over the block's threads merges each head with the carries
// before it, in thread order; a head whose row began in an earlier block, and
// the block's last carry, go to the block's slots, and k_merge_fixup merges
// those across blocks in block order.  The sums of the rows completed in the
// block are collected in LDS and their epilogues run in row order, so the
// writes of y (and the epilogue's other vectors) are coalesced.  Every row sum
// is a fixed-order merge of compensated pieces, so the result does not
// depend on timing; the residual's b is merged in front of the products.
// ---------------------------------------------------------------------------
// one pad slot per kMergeIpt products, so the lanes' runs start in different banks
constexpr int kMergePad = kMergeItems + kMergeItems / kMergeIpt;

// rows completed among the first d items of the path
__device__ __forceinline__ int64_t merge_split(const int32_t *__restrict__ rp, int64_t rows,
                                               int64_t nnz, int64_t d) {
    int64_t lo = d > nnz ? d - nnz : 0, hi = d < rows ? d : rows;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if ((int64_t)rp[mid + 1] <= d - mid - 1)
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo;
}

__global__ void k_merge_part(int64_t rows, const int32_t *__restrict__ rp, int64_t mb,
                             int32_t *__restrict__ mp) {
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b > mb) return;
    const int64_t nnz = rp[rows], total = rows + nnz;
    const int64_t d = min(b * (int64_t)kMergeItems, total);
    mp[b] = (int32_t)merge_split(rp, rows, nnz, d);
}

// A scan element: the merged carries of a run of threads; f = this element
// starts a run, o = the run starts at thread 0 inside a row begun before the
// block.
struct SegAcc {
    Acc v;
    int32_t f, o;
};

__device__ __forceinline__ SegAcc seg_combine(const SegAcc &a, const SegAcc &b) {
    SegAcc c;
    c.v = b.f ? b.v : acc_merge(a.v, b.v);
    c.f = a.f | b.f;
    c.o = b.f ? b.o : a.o;
    return c;
}

// The block's slots in M.ypart (mb each): head values, carry values, then
// head rows and carry rows as int32.
struct MergeSlots {
    double2 *hv, *cv;
    int32_t *hr, *cr;
};

__device__ __forceinline__ MergeSlots merge_slots(const MatView &M) {
    MergeSlots q;
    q.hv = M.ypart;
    q.cv = M.ypart + M.mb;
    q.hr = reinterpret_cast<int32_t *>(M.ypart + 2 * M.mb);
    q.cr = q.hr + M.mb;
    return q;
}

// A row's value from its compensated sum of the products (negated for the
// residual, whose b is merged in front)
template <int EPI>
__device__ __forceinline__ double merge_row_value(int64_t row, Acc a, const EpiArgs &ea) {
    if constexpr (EPI == kEpiResid) a = acc_merge(Acc{ea.b[row], 0.0}, a);
    return acc_val(a);
}

template <int EPI>
__global__ __launch_bounds__(kBlock) void k_merge_spmv(MatView M, const double *__restrict__ x,
                                                        double *y, EpiArgs ea, Out o) {
    if (!producer_runs(o)) return;
    constexpr double sgn = (EPI == kEpiResid) ? -1.0 : 1.0;
    __shared__ double2 s_hp[kMergePad];
    __shared__ int32_t s_rp[kMergeItems + 2];
    __shared__ double s_wvp[kBlock / 64], s_wvs[kBlock / 64];  // each wave's total, by field
    __shared__ int32_t s_wf[kBlock / 64], s_wo[kBlock / 64];
    __shared__ int32_t s_hr, s_cr;
    __shared__ double2 s_hv, s_cv;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t rows = M.rows;
    const int64_t b = blockIdx.x;
    const int64_t i0 = M.mp[b], i1 = M.mp[b + 1];
    const int64_t nnz = M.rp[rows], total = rows + nnz;
    const int64_t D0 = b * kMergeItems, D1 = min(D0 + (int64_t)kMergeItems, total);
    const int64_t k0 = D0 - i0, k1 = D1 - i1;
    const int nk = (int)(k1 - k0);
    // row pointers rp[i0 .. min(i1, rows - 1) + 1]
    const int nr = i0 < rows ? (int)(min(i1, rows - 1) + 2 - i0) : 0;
    if (nr > 0) {
        int32_t rv[kMergeIpt + 1];
#pragma unroll
        for (int u = 0; u <= kMergeIpt; ++u) rv[u] = M.rp[i0 + min(u * kBlock + tid, nr - 1)];
#pragma unroll
        for (int u = 0; u <= kMergeIpt; ++u)
            if (u * kBlock + tid < nr) s_rp[u * kBlock + tid] = rv[u];
    }
    if (nk > 0) {
        // all loads first (indexes clamped into the block's nonzeros), then
        // the gathers, then the exact products
        int32_t cj[kMergeIpt];
        double av[kMergeIpt], xv[kMergeIpt];
#pragma unroll
        for (int u = 0; u < kMergeIpt; ++u) {
            const int j = min(u * kBlock + tid, nk - 1);
            cj[u] = __builtin_nontemporal_load(M.ci + k0 + j);
            av[u] = __builtin_nontemporal_load(M.val + k0 + j);
        }
#pragma unroll
        for (int u = 0; u < kMergeIpt; ++u) xv[u] = x[cj[u]];
#pragma unroll
        for (int u = 0; u < kMergeIpt; ++u) {
            const int j = u * kBlock + tid;
            if (j < nk) {
                const double a = sgn * av[u];
                const double h = a * xv[u];
                s_hp[j + j / kMergeIpt] = make_double2(h, __fma_rn(a, xv[u], -h));
            }
        }
    }
    if (tid == 0) {
        s_hr = -1;
        s_cr = -1;
    }
    __syncthreads();

    // this thread's start on the path: il rows completed inside the block
    const int64_t dl = min((int64_t)tid * kMergeIpt, D1 - D0);
    const int64_t dle = min(dl + kMergeIpt, D1 - D0);
    int64_t lo = dl > nk ? dl - nk : 0, hi = min(dl, i1 - i0);
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if ((int64_t)s_rp[mid + 1] <= k0 + dl - mid - 1)
            lo = mid + 1;
        else
            hi = mid;
    }
    int64_t i = i0 + lo, k = k0 + dl - lo;
    const bool head0 = i < rows && k > s_rp[i - i0];
    bool head = head0;
    Acc acc = {0.0, 0.0};
    int32_t hr = -1;
    Acc hv = {0.0, 0.0};
    // rows that begin and end in this thread: offset from i0 and sum
    int32_t yr[kMergeIpt];
    Acc yv[kMergeIpt];
    int64_t ks = k;
    int64_t e = i < rows ? s_rp[i - i0 + 1] : 0;
#pragma unroll
    for (int u = 0; u < kMergeIpt; ++u) {
        yr[u] = -1;
        yv[u] = Acc{0.0, 0.0};
        if (dl + u < dle) {
            if (i < rows && k >= e) {  // the end of row i
                if (head) {
                    hr = (int32_t)i;
                    hv = acc;
                    head = false;
                } else {
                    yr[u] = (int32_t)(i - i0);
                    yv[u] = acc;
                }
                ++i;
                acc = Acc{0.0, 0.0};
                ks = k;
                if (i < rows) e = s_rp[i - i0 + 1];
            } else {
                const int64_t j = k - k0;
                const double2 p = s_hp[j + j / kMergeIpt];
                acc_add_split(acc, p.x, p.y);
                ++k;
            }
        }
    }
    const bool carry = i < rows && k > ks;
    const bool cont = head0 && hr < 0;  // inside one row begun before this thread

    // segmented inclusive scan of the carries over the block's threads
    SegAcc c;
    c.v = carry ? acc : Acc{0.0, 0.0};
    c.f = (tid == 0 || !cont) ? 1 : 0;
    c.o = (tid == 0 && cont) ? 1 : 0;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        SegAcc u;
        u.v.p = __shfl_up(c.v.p, off);
        u.v.s = __shfl_up(c.v.s, off);
        u.f = __shfl_up(c.f, off);
        u.o = __shfl_up(c.o, off);
        if (lane >= off) c = seg_combine(u, c);
    }
    if (lane == 63) {
        s_wvp[wave] = c.v.p;
        s_wvs[wave] = c.v.s;
        s_wf[wave] = c.f;
        s_wo[wave] = c.o;
    }
    __syncthreads();  // every walk is done: s_hp now holds the completed rows
    // the inclusive scan up to the thread before this wave (wave 0: unused)
    SegAcc pre;
    pre.v = Acc{s_wvp[0], s_wvs[0]};
    pre.f = s_wf[0];
    pre.o = s_wo[0];
    for (int w = 1; w < wave; ++w) {
        SegAcc q;
        q.v = Acc{s_wvp[w], s_wvs[w]};
        q.f = s_wf[w];
        q.o = s_wo[w];
        pre = seg_combine(pre, q);
    }
    if (wave > 0) c = seg_combine(pre, c);
    // the inclusive scan at the thread before this one
    SegAcc prev;
    prev.v.p = __shfl_up(c.v.p, 1);
    prev.v.s = __shfl_up(c.v.s, 1);
    prev.f = __shfl_up(c.f, 1);
    prev.o = __shfl_up(c.o, 1);
    if (lane == 0) prev = pre;

    // the sums of the rows completed in this block, by row (offset from i0)
    double2 *s_y = s_hp;
#pragma unroll
    for (int u = 0; u < kMergeIpt; ++u)
        if (yr[u] >= 0) s_y[yr[u]] = make_double2(yv[u].p, yv[u].s);
    if (hr >= 0) {
        if (tid == 0) {  // the row began in an earlier block
            s_hr = hr;
            s_hv = make_double2(hv.p, hv.s);
        } else {
            const Acc t = acc_merge(prev.v, hv);
            if (prev.o) {
                s_hr = hr;
                s_hv = make_double2(t.p, t.s);
            } else {
                s_y[hr - i0] = make_double2(t.p, t.s);
            }
        }
    }
    if (tid == kBlock - 1 && carry) {
        s_cr = (int32_t)i;
        s_cv = make_double2(c.v.p, c.v.s);
    }
    __syncthreads();
    if (tid == 0) {
        const MergeSlots q = merge_slots(M);
        q.hr[b] = s_hr;
        q.hv[b] = s_hv;
        q.cr[b] = s_cr;
        q.cv[b] = s_cv;
    }
    // epilogues of the rows completed here, in row order (coalesced); row i0
    // is left to k_merge_fixup when it began in an earlier block
    Acc v[EpiNV<EPI>::value] = {};
    const int64_t r0 = i0 + (i0 < rows && k0 > s_rp[0] ? 1 : 0);
    for (int64_t r = r0 + tid; r < i1; r += kBlock) {
        const double2 a = s_y[r - i0];
        epilogue<EPI>(r, merge_row_value<EPI>(r, Acc{a.x, a.y}, ea), y, ea, o.st, v);
    }
    block_partials<EpiNV<EPI>::value>(v, o);
}

// One wave per block j of k_merge_spmv: a head row r begun in earlier blocks
// is completed from the carries of the run of blocks before j whose carry is
// row r (block j - 1 always is one), then the head.  Lane l takes blocks
// j - 1 - l, j - 65 - l, ... in that order, the lanes then merge in a fixed
// tree.  The first 64 carries are loaded with the head row, before it is
// known.  Partials go after the product kernel's.
template <int EPI>
__global__ __launch_bounds__(kBlock) void k_merge_fixup(MatView M, double *y, EpiArgs ea, Out o) {
    if (!producer_runs(o)) return;
    const int lane = threadIdx.x & 63;
    const int64_t j = (int64_t)blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6);
    const MergeSlots q = merge_slots(M);
    Acc v[EpiNV<EPI>::value] = {};
    const bool valid = j < M.mb;
    const int32_t r = valid ? q.hr[j] : -1;
    int64_t u = j - 1 - lane;
    int32_t cr = valid && u >= 0 ? q.cr[u] : -1;
    double2 cv = valid && u >= 0 ? q.cv[u] : make_double2(0.0, 0.0);
    const double2 h = valid ? q.hv[j] : make_double2(0.0, 0.0);
    if (r >= 0) {
        Acc a = {0.0, 0.0};
        for (;;) {
            const uint64_t out = __ballot(cr != r);
            // the lanes before the first one outside the run belong to it
            const int first_out = out != 0 ? __ffsll((unsigned long long)out) - 1 : 64;
            if (lane < first_out) a = acc_merge(a, Acc{cv.x, cv.y});
            if (out != 0) break;
            u -= 64;
            cr = u >= 0 ? q.cr[u] : -1;
            cv = u >= 0 ? q.cv[u] : make_double2(0.0, 0.0);
        }
        a = group_reduce<64>(a);
        if (lane == 0) {
            a = acc_merge(a, Acc{h.x, h.y});
            epilogue<EPI>(r, merge_row_value<EPI>(r, a, ea), y, ea, o.st, v);
        }
    }
    block_partials<EpiNV<EPI>::value>(v, o, M.mb + blockIdx.x);
}

// First entry of each column slice inside each row of a column-sorted CSR.
__global__ void k_slice_segments(int64_t m, const int32_t *__restrict__ rp,
                                 const int32_t *__restrict__ ci, int64_t slice_w, int32_t nsl,
                                 int32_t *seg) {
    for (int64_t row = (int64_t)blockIdx.x * kBlock + threadIdx.x; row < m;
         row += (int64_t)gridDim.x * kBlock) {
        const int32_t s = rp[row], e = rp[row + 1];
        int32_t *out = seg + row * (nsl + 1);
        out[0] = s;
        for (int sl = 1; sl < nsl; ++sl) {
            const int64_t bound = sl * slice_w;
            int32_t lo = s, hi = e;  // first k with ci[k] >= bound
            while (lo < hi) {
                const int32_t mid = lo + (hi - lo) / 2;
                if (ci[mid] < bound)
                    lo = mid + 1;
                else
                    hi = mid;
            }
            out[sl] = lo;
        }
        out[nsl] = e;
    }
}

// ---------------------------------------------------------------------------
// Dense A^T u: one thread per column of A, rows in order (coalesced across
// the threads of a wave because A is row-major).
// ---------------------------------------------------------------------------
template <int EPI>
__global__ __launch_bounds__(kBlock) void k_dense_cols(MatView M, const double *__restrict__ x,
                                                        double *y, EpiArgs ea, Out o) {
    if (!producer_runs(o)) return;
    // M = A^T: M.rows = columns of A, M.cols = rows of A
    constexpr double sgn = (EPI == kEpiResid) ? -1.0 : 1.0;
    const int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    Acc acc = {0.0, 0.0};
    if (j < M.rows) {
        // the residual form b_j - (M x)_j is one compensated sum starting at b_j
        if constexpr (EPI == kEpiResid) acc.p = ea.b[j];
        const double *a = M.val + j;
        for (int64_t i = 0; i < M.cols; ++i) acc_fma(acc, sgn * a[i * M.ld], x[i]);
    }
    Acc v[EpiNV<EPI>::value] = {};
    if (j < M.rows) epilogue<EPI>(j, acc_val(acc), y, ea, o.st, v);
    block_partials<EpiNV<EPI>::value>(v, o);
}

// ---------------------------------------------------------------------------
// element-wise kernels of the chains
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_cta_init(int64_t m, const double *__restrict__ b,
                                                      double *r, double *xy, int64_t nxy,
                                                      int32_t zero_xy, Out o) {
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
    block_partials<1>(v, o);
}

struct VecPtrs {
    double *p[kTMax + 1];
};

__global__ __launch_bounds__(kBlock) void k_cta_update(int64_t m, int64_t n, int32_t t,
                                                        int32_t minnorm, double *r, VecPtrs u,
                                                        double *x, VecPtrs w, double *y,
                                                        double *rb, double *yb, Out o) {
    if (o.st->done) return;
    double al[kTMax];
#pragma unroll
    for (int j = 0; j < kTMax; ++j) al[j] = j < t ? o.st->alpha[j] : 0.0;
    Acc v[1] = {};
    const int64_t N = (minnorm || m > n) ? m : n;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < N;
         i += (int64_t)gridDim.x * kBlock) {
        if (i < m) {
            double ri = r[i];
            if (rb != nullptr) rb[i] = ri;
            if (minnorm) {
                double yi = y[i];
                if (yb != nullptr) yb[i] = yi;
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
            if (yb != nullptr) yb[i] = xi;
            for (int j = 0; j < t; ++j) xi = __fma_rn(al[j], w.p[j][i], xi);
            x[i] = xi;
        }
    }
    block_partials<1>(v, o);
}

// Convex-combination step (the first-order dynamics theorem of section 3.4):
// r = a r_k + (1 - a) r_{k+1}, and the same for the iterate, a = state.astar.
__global__ __launch_bounds__(kBlock) void k_cta_jump(int64_t m, int64_t nxy, double *r,
                                                      const double *__restrict__ rb, double *xy,
                                                      const double *__restrict__ xyb, Out o) {
    if (!producer_runs(o)) return;
    const double a = o.st->astar, a1 = 1.0 - a;
    Acc v[1] = {};
    const int64_t N = m > nxy ? m : nxy;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < N;
         i += (int64_t)gridDim.x * kBlock) {
        if (i < m) {
            const double ri = __fma_rn(a, rb[i], a1 * r[i]);
            r[i] = ri;
            acc_fma(v[0], ri, ri);
        }
        if (i < nxy) xy[i] = __fma_rn(a, xyb[i], a1 * xy[i]);
    }
    block_partials<1>(v, o);
}

__global__ __launch_bounds__(kBlock) void k_ta_init(int64_t m, int64_t n,
                                                     const double *__restrict__ b, double *r,
                                                     double *bp, double *x, int32_t keep_x,
                                                     Out o) {
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
        if (i < n && !keep_x) x[i] = 0.0;
    }
    block_partials<1>(v, o);
}

// ||x||^2 as one compensated partial per block.
__global__ __launch_bounds__(kBlock) void k_norm2(int64_t n, const double *__restrict__ x, Out o) {
    Acc v[1] = {};
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kBlock)
        acc_fma(v[0], x[i], x[i]);
    block_partials<1>(v, o);
}

__global__ __launch_bounds__(kBlock) void k_ta_update(int64_t m, int64_t n,
                                                       const double *__restrict__ b, double *bp,
                                                       const double *__restrict__ d, double *r,
                                                       double *x, const double *__restrict__ c,
                                                       Out o) {
    const State *st = o.st;
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
    block_partials<2>(v, o);
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
        const int32_t t = (int)threadIdx.x >= off ? sh[threadIdx.x - off] : 0;
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
                                int32_t *long_rows, int32_t *n_long) {
    for (int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x; j < n;
         j += (int64_t)gridDim.x * kBlock) {
        const int32_t s = at_rp[j], e = at_rp[j + 1], len = e - s;
        if (len > 32) {
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

// Ascending bitonic sorting network on keys that are all distinct, in the
// form whose merges all run upwards: the first step of the merge of size K
// pairs i with its mirror i ^ (K - 1), the later steps i with i + J.  Past the
// c real keys the network sees +infinity, which never moves, so the padding to
// a power of two is never stored.
__device__ __forceinline__ void bitonic_pair(int64_t q, int64_t K, int64_t J, int64_t &i,
                                             int64_t &l) {
    if (J == K / 2) {  // the mirror step
        const int64_t h = K / 2, base = (q / h) * K, a = q % h;
        i = base + a;
        l = base + K - 1 - a;
    } else {
        i = (q / J) * 2 * J + q % J;
        l = i + J;
    }
}

// Steps (K, J) for J from jfirst down to 1 of the network on g[0 .. c)
// (c <= kMaxColNnz), in LDS; with jfirst = 0, the whole sort of g.
__device__ void lds_bitonic(int32_t *g, int c, int jfirst, int32_t *key) {
    for (int t = threadIdx.x; t < c; t += kBlock) key[t] = g[t];
    __syncthreads();
    int P = 1;
    while (P < c) P <<= 1;
    for (int K = jfirst > 0 ? 4 * jfirst : 2; K <= (jfirst > 0 ? 4 * jfirst : P); K <<= 1) {
        for (int J = jfirst > 0 ? jfirst : K / 2; J > 0; J >>= 1) {
            for (int q = threadIdx.x; q < P / 2; q += kBlock) {
                int64_t i, l;
                bitonic_pair(q, K, J, i, l);
                if (l < c) {
                    const int32_t x = key[i], y = key[l];
                    if (x > y) {
                        key[i] = y;
                        key[l] = x;
                    }
                }
            }
            __syncthreads();
        }
    }
    for (int t = threadIdx.x; t < c; t += kBlock) g[t] = key[t];
    __syncthreads();
}

// Sorts the source indices of each A^T row with more than 32 entries (one
// block per row).  Up to kMaxColNnz entries the row is sorted in LDS.  A
// longer row runs the same network over the whole row: its chunks of
// kMaxColNnz are sorted in LDS, then each merge of size K > kMaxColNnz makes
// its steps with partners kMaxColNnz or more apart in global memory (one
// block owns the row, so a barrier orders them) and its shorter steps chunk
// by chunk in LDS.
__global__ __launch_bounds__(kBlock) void k_tr_sort_long(const int32_t *__restrict__ at_rp,
                                                          int32_t *src,
                                                          const int32_t *__restrict__ long_rows,
                                                          const int32_t *__restrict__ n_long) {
    __shared__ int32_t key[kMaxColNnz];
    constexpr int C = kMaxColNnz;
    const int32_t cnt = *n_long;
    for (int32_t li = blockIdx.x; li < cnt; li += gridDim.x) {
        const int32_t j = long_rows[li];
        const int32_t s = at_rp[j], len = at_rp[j + 1] - s;
        int32_t *g = src + s;
        if (len <= C) {
            lds_bitonic(g, len, 0, key);
            continue;
        }
        for (int64_t lo = 0; lo < len; lo += C) lds_bitonic(g + lo, (int)min((int64_t)C, len - lo), 0, key);
        int64_t P = 1;
        while (P < len) P <<= 1;
        for (int64_t K = 2 * C; K <= P; K <<= 1) {
            for (int64_t J = K / 2; J >= C; J >>= 1) {
                // 4 pairs per thread and round, loaded before any is compared
                constexpr int R = 4;
                for (int64_t q0 = threadIdx.x; q0 < P / 2; q0 += R * kBlock) {
                    int64_t i[R], l[R];
                    int32_t x[R], y[R];
#pragma unroll
                    for (int u = 0; u < R; ++u) {
                        const int64_t q = q0 + u * kBlock;
                        l[u] = len;  // no pair
                        if (q < P / 2) bitonic_pair(q, K, J, i[u], l[u]);
                        if (l[u] < len) {
                            x[u] = g[i[u]];
                            y[u] = g[l[u]];
                        }
                    }
#pragma unroll
                    for (int u = 0; u < R; ++u)
                        if (l[u] < len && x[u] > y[u]) {
                            g[i[u]] = y[u];
                            g[l[u]] = x[u];
                        }
                }
                __syncthreads();
            }
            for (int64_t lo = 0; lo < len; lo += C)
                lds_bitonic(g + lo, (int)min((int64_t)C, len - lo), C / 2, key);
        }
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
// CSR validation: flag bit 1 for bad row pointers, bit 2 for bad columns
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_check_csr(int64_t m, int64_t n, int64_t nnz, const int32_t *rp,
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
    switch (M.kind) {
        case kDenseCols: return cdiv(rows, kBlock);
        case kDenseRows: return cdiv(rows, kBlock / 64);
        case kCsrSliced: return elementwise_blocks(rows);  // the combine kernel
        case kCsrTiled: return cdiv(rows, kBlock / kCombineLanes);  // the combine kernel
        case kCsrMerge: return M.mb + cdiv(M.mb, kBlock / 64);    // product, then fix-up
        case kCsrSell: return cdiv(rows, kBlock);
        default: return M.lanes > 1 ? cdiv(rows, kBlock / M.lanes) : cdiv(rows, kBlock);
    }
}

template <int EPI>
static void launch_vec_lanes(const MatView &M, dim3 grid, const double *x, double *y,
                             const EpiArgs &ea, const Out &o, hipStream_t s) {
    switch (M.lanes) {
        case 2: k_rows_vector<2, EPI><<<grid, kBlock, 0, s>>>(M, x, y, ea, o); break;
        case 4: k_rows_vector<4, EPI><<<grid, kBlock, 0, s>>>(M, x, y, ea, o); break;
        case 8: k_rows_vector<8, EPI><<<grid, kBlock, 0, s>>>(M, x, y, ea, o); break;
        case 16: k_rows_vector<16, EPI><<<grid, kBlock, 0, s>>>(M, x, y, ea, o); break;
        case 32: k_rows_vector<32, EPI><<<grid, kBlock, 0, s>>>(M, x, y, ea, o); break;
        default: k_rows_vector<64, EPI><<<grid, kBlock, 0, s>>>(M, x, y, ea, o); break;
    }
}

template <int EPI>
static void launch_sliced(const MatView &M, const double *x, const EpiArgs &ea, const Out &o,
                          hipStream_t s) {
    const int W = M.lanes;
    const dim3 grid((unsigned)(M.nsl * cdiv(M.rows > 0 ? M.rows : 1, kBlock / W)));
    switch (W) {
        case 2: k_rows_sliced<2, EPI><<<grid, kBlock, 0, s>>>(M, x, ea, o); break;
        case 4: k_rows_sliced<4, EPI><<<grid, kBlock, 0, s>>>(M, x, ea, o); break;
        case 8: k_rows_sliced<8, EPI><<<grid, kBlock, 0, s>>>(M, x, ea, o); break;
        case 16: k_rows_sliced<16, EPI><<<grid, kBlock, 0, s>>>(M, x, ea, o); break;
        case 32: k_rows_sliced<32, EPI><<<grid, kBlock, 0, s>>>(M, x, ea, o); break;
        default: k_rows_sliced<64, EPI><<<grid, kBlock, 0, s>>>(M, x, ea, o); break;
    }
}

template <int EPI>
static void launch_tiled(const MatView &M, const double *x, const Out &o, hipStream_t s) {
    const dim3 grid((unsigned)((int64_t)M.nt * M.nchunk));
    switch (M.lanes) {
        case 1: k_rows_tiled<1, EPI><<<grid, kTileBlock, 0, s>>>(M, x, o); break;
        case 2: k_rows_tiled<2, EPI><<<grid, kTileBlock, 0, s>>>(M, x, o); break;
        case 4: k_rows_tiled<4, EPI><<<grid, kTileBlock, 0, s>>>(M, x, o); break;
        case 8: k_rows_tiled<8, EPI><<<grid, kTileBlock, 0, s>>>(M, x, o); break;
        case 16: k_rows_tiled<16, EPI><<<grid, kTileBlock, 0, s>>>(M, x, o); break;
        case 32: k_rows_tiled<32, EPI><<<grid, kTileBlock, 0, s>>>(M, x, o); break;
        default: k_rows_tiled<64, EPI><<<grid, kTileBlock, 0, s>>>(M, x, o); break;
    }
}

template <int EPI>
static void launch_matvec_t(const MatView &M, const double *x, double *y, const EpiArgs &ea,
                            const Out &o, hipStream_t s, dim3 grid) {
    switch (M.kind) {
        case kDenseCols: k_dense_cols<EPI><<<grid, kBlock, 0, s>>>(M, x, y, ea, o); break;
        case kDenseRows: {
            MatView V = M;
            V.lanes = 64;
            launch_vec_lanes<EPI>(V, grid, x, y, ea, o, s);
            break;
        }
        case kCsrSliced:
            launch_sliced<EPI>(M, x, ea, o, s);
            k_slices_combine<EPI><<<grid, kBlock, 0, s>>>(M, y, ea, o);
            break;
        case kCsrTiled:
            if (M.rows > 0 && M.nt > 0) launch_tiled<EPI>(M, x, o, s);
            k_tiles_combine<EPI><<<grid, kBlock, 0, s>>>(M, y, ea, o);
            break;
        case kCsrSell:
            if (M.nt_stream)
                k_sell<EPI, true><<<grid, kBlock, 0, s>>>(M, x, y, ea, o);
            else
                k_sell<EPI, false><<<grid, kBlock, 0, s>>>(M, x, y, ea, o);
            break;
        case kCsrMerge:
            k_merge_spmv<EPI><<<dim3((unsigned)M.mb), kBlock, 0, s>>>(M, x, y, ea, o);
            k_merge_fixup<EPI><<<dim3((unsigned)cdiv(M.mb, kBlock / 64)), kBlock, 0, s>>>(M, y, ea, o);
            break;
        default:
            if (M.lanes > 1)
                launch_vec_lanes<EPI>(M, grid, x, y, ea, o, s);
            else
                k_csr_stream<EPI><<<grid, kBlock, 0, s>>>(M, x, y, ea, o);
            break;
    }
}

hipError_t launch_merge_part(int64_t rows, const int32_t *rp, int64_t mb, int32_t *mp,
                             hipStream_t s) {
    k_merge_part<<<dim3((unsigned)cdiv(mb + 1, kBlock)), kBlock, 0, s>>>(rows, rp, mb, mp);
    return hipGetLastError();
}

__global__ __launch_bounds__(kBlock) void k_row_max(int64_t rows, const int32_t *__restrict__ rp,
                                                   int32_t *out) {
    __shared__ int32_t red[kBlock / 64];
    int32_t w = 0;
    for (int64_t r = (int64_t)blockIdx.x * kBlock + threadIdx.x; r < rows;
         r += (int64_t)gridDim.x * kBlock)
        w = max(w, rp[r + 1] - rp[r]);
    for (int off = 32; off > 0; off >>= 1) w = max(w, __shfl_xor(w, off));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = w;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int q = 1; q < kBlock / 64; ++q) w = max(w, red[q]);
        atomicMax(out, w);
    }
}

hipError_t launch_row_max(int64_t rows, const int32_t *rp, int32_t *out, hipStream_t s) {
    if (rows <= 0) return hipSuccess;
    k_row_max<<<dim3((unsigned)elementwise_blocks(rows)), kBlock, 0, s>>>(rows, rp, out);
    return hipGetLastError();
}

hipError_t launch_sell_widths(int64_t rows, const int32_t *rp, int32_t *w, hipStream_t s) {
    if (rows <= 0) return hipSuccess;
    const int64_t g = cdiv(((rows + 63) >> 6) * 64, kBlock);
    k_sell_widths<<<dim3((unsigned)g), kBlock, 0, s>>>(rows, rp, w);
    return hipGetLastError();
}

hipError_t launch_sell_fill(int64_t rows, const int32_t *rp, const int32_t *ci, const double *val,
                            const int64_t *so, int32_t *sc, double *sv, hipStream_t s) {
    if (rows <= 0) return hipSuccess;
    const int64_t g = cdiv(((rows + 63) >> 6) * 64, kBlock);
    k_sell_fill<<<dim3((unsigned)g), kBlock, 0, s>>>(rows, rp, ci, val, so, sc, sv);
    return hipGetLastError();
}

hipError_t launch_matvec(const MatView &M, const double *x, double *y, int32_t epi,
                         const EpiArgs &ea, const Out &o, hipStream_t s, int32_t *blocks) {
    const int64_t g = matvec_blocks(M);
    if (g > o.cap) return hipErrorInvalidValue;
    const dim3 grid((unsigned)g);
    switch (epi) {
        case kEpiNorm: launch_matvec_t<kEpiNorm>(M, x, y, ea, o, s, grid); break;
        case kEpiResid: launch_matvec_t<kEpiResid>(M, x, y, ea, o, s, grid); break;
        case kEpiTaD: launch_matvec_t<kEpiTaD>(M, x, y, ea, o, s, grid); break;
        case kEpiTaBp: launch_matvec_t<kEpiTaBp>(M, x, y, ea, o, s, grid); break;
        case kEpiNormDot: launch_matvec_t<kEpiNormDot>(M, x, y, ea, o, s, grid); break;
        case kEpiNormPos: launch_matvec_t<kEpiNormPos>(M, x, y, ea, o, s, grid); break;
        default: return hipErrorInvalidValue;
    }
    if (blocks != nullptr) *blocks = (int32_t)g;
    return hipGetLastError();
}

hipError_t launch_cta_init(int64_t m, const double *b, double *r, double *xy, int64_t nxy,
                           int32_t zero_xy, const Out &o, hipStream_t s, int32_t *blocks) {
    const int64_t g = elementwise_blocks(m > nxy ? m : nxy);
    if (g > o.cap) return hipErrorInvalidValue;
    k_cta_init<<<dim3((unsigned)g), kBlock, 0, s>>>(m, b, r, xy, nxy, zero_xy, o);
    if (blocks != nullptr) *blocks = (int32_t)g;
    return hipGetLastError();
}

hipError_t launch_cta_update(int64_t m, int64_t n, int32_t t, int32_t minnorm, double *r,
                             double *const *u, double *x, double *const *w, double *y,
                             double *rb, double *yb, const Out &o, hipStream_t s,
                             int32_t *blocks) {
    VecPtrs U{}, Wp{};
    for (int j = 0; j <= t && j <= kTMax; ++j) U.p[j] = u[j];
    for (int j = 0; j < t && j < kTMax; ++j) Wp.p[j] = w ? w[j] : nullptr;
    const int64_t N = (minnorm || m > n) ? m : n;
    const int64_t g = elementwise_blocks(N);
    if (g > o.cap) return hipErrorInvalidValue;
    k_cta_update<<<dim3((unsigned)g), kBlock, 0, s>>>(m, n, t, minnorm, r, U, x, Wp, y, rb, yb,
                                                      o);
    if (blocks != nullptr) *blocks = (int32_t)g;
    return hipGetLastError();
}

hipError_t launch_cta_jump(int64_t m, int64_t nxy, double *r, const double *rb, double *xy,
                           const double *xyb, const Out &o, hipStream_t s, int32_t *blocks) {
    const int64_t g = elementwise_blocks(m > nxy ? m : nxy);
    if (g > o.cap) return hipErrorInvalidValue;
    k_cta_jump<<<dim3((unsigned)g), kBlock, 0, s>>>(m, nxy, r, rb, xy, xyb, o);
    if (blocks != nullptr) *blocks = (int32_t)g;
    return hipGetLastError();
}

hipError_t launch_ta_init(int64_t m, int64_t n, const double *b, double *r, double *bp,
                          double *x, int32_t keep_x, const Out &o, hipStream_t s,
                          int32_t *blocks) {
    const int64_t g = elementwise_blocks(m > n ? m : n);
    if (g > o.cap) return hipErrorInvalidValue;
    k_ta_init<<<dim3((unsigned)g), kBlock, 0, s>>>(m, n, b, r, bp, x, keep_x, o);
    if (blocks != nullptr) *blocks = (int32_t)g;
    return hipGetLastError();
}

hipError_t launch_ta_update(int64_t m, int64_t n, const double *b, double *bp, const double *d,
                            double *r, double *x, const double *c, const Out &o, hipStream_t s,
                            int32_t *blocks) {
    const int64_t g = elementwise_blocks(m > n ? m : n);
    if (g > o.cap) return hipErrorInvalidValue;
    k_ta_update<<<dim3((unsigned)g), kBlock, 0, s>>>(m, n, b, bp, d, r, x, c, o);
    if (blocks != nullptr) *blocks = (int32_t)g;
    return hipGetLastError();
}

hipError_t launch_slice_segments(int64_t m, const int32_t *rp, const int32_t *ci_sorted,
                                 int64_t cols, int32_t nsl, int32_t *seg, hipStream_t s) {
    const int64_t w = cdiv(cols > 0 ? cols : 1, nsl);
    k_slice_segments<<<(unsigned)elementwise_blocks(m), kBlock, 0, s>>>(m, rp, ci_sorted, w, nsl,
                                                                        seg);
    return hipGetLastError();
}

hipError_t launch_check_csr(int64_t m, int64_t n, int64_t nnz, const int32_t *rp,
                            const int32_t *ci, int32_t *flag, hipStream_t s) {
    const int64_t work = (m + 1 > nnz ? m + 1 : nnz);
    const unsigned grid = (unsigned)elementwise_blocks(work);
    k_check_csr<<<grid, kBlock, 0, s>>>(m, n, nnz, rp, ci, flag);
    return hipGetLastError();
}

// Dense transpose through a 32 x 33 LDS tile: dst (n x m, row stride ldd)
// = src^T (m x n, row stride lds).
__global__ __launch_bounds__(kBlock) void k_dense_transpose64(int64_t m, int64_t n,
                                                               const double *__restrict__ src,
                                                               int64_t lds, double *dst,
                                                               int64_t ldd) {
    __shared__ double tile[32][33];
    const int64_t i0 = (int64_t)blockIdx.y * 32, j0 = (int64_t)blockIdx.x * 32;
    const int tx = threadIdx.x % 32, ty = threadIdx.x / 32;  // 32 x 8
    for (int r = ty; r < 32; r += 8)
        if (i0 + r < m && j0 + tx < n) tile[r][tx] = src[(i0 + r) * lds + j0 + tx];
    __syncthreads();
    for (int r = ty; r < 32; r += 8)
        if (j0 + r < n && i0 + tx < m) dst[(j0 + r) * ldd + i0 + tx] = tile[tx][r];
}

hipError_t launch_dense_transpose(int64_t m, int64_t n, const double *src, int64_t lds,
                                  double *dst, int64_t ldd, hipStream_t s) {
    if (m <= 0 || n <= 0) return hipSuccess;
    if ((m + 31) / 32 > 65535) return hipErrorInvalidValue;
    const dim3 grid((unsigned)((n + 31) / 32), (unsigned)((m + 31) / 32));
    k_dense_transpose64<<<grid, kBlock, 0, s>>>(m, n, src, lds, dst, ldd);
    return hipGetLastError();
}

// The whole State from a kernel argument (no host staging buffer).
__global__ void k_state_set(State *d, State h) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *d = h;
}

hipError_t launch_state_set(State *d, const State &h, hipStream_t s) {
    k_state_set<<<1, 64, 0, s>>>(d, h);
    return hipGetLastError();
}

hipError_t launch_step(const Step &sp, hipStream_t s) {
    if (sp.nslots < 0 || sp.nslots > kMaxSlots) return hipErrorInvalidValue;
    for (int i = 0; i < sp.nslots; ++i)
        if (sp.count[i] < 0 || sp.count[i] > sp.cap) return hipErrorInvalidValue;
    k_step<<<1, kBlock, 0, s>>>(sp);
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
                                                                        n_long);
    k_tr_sort_long<<<1024, kBlock, 0, s>>>(at_rp, src, long_rows, n_long);
    if (nnz > 0) k_tr_fill<<<gn, kBlock, 0, s>>>(m, nnz, rp, val, src, at_ci, at_val);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Tile-major copy of a column-sorted CSR (kCsrTiled): the run length of
// every (tile, row), an exclusive scan of the lengths in tile-major order,
// then each row's entries copied to their run with the column made local to
// the tile.  One thread per row; runs are contiguous because the columns
// are sorted, and each (tile, row) slot has one writer.
// ---------------------------------------------------------------------------
__global__ void k_tile_count(int64_t rows, const int32_t *__restrict__ rp,
                             const int32_t *__restrict__ ci, int32_t *cnt) {
    for (int64_t row = (int64_t)blockIdx.x * kBlock + threadIdx.x; row < rows;
         row += (int64_t)gridDim.x * kBlock) {
        const int32_t e = rp[row + 1];
        for (int32_t k = rp[row]; k < e;) {
            const int32_t q = ci[k] / kTileW;
            int32_t k1 = k + 1;
            while (k1 < e && ci[k1] / kTileW == q) ++k1;
            cnt[(int64_t)q * rows + row] = k1 - k;
            k = k1;
        }
    }
}

__global__ void k_tile_fill(int64_t rows, const int32_t *__restrict__ rp,
                            const int32_t *__restrict__ ci, const double *__restrict__ val,
                            const int32_t *__restrict__ trp, uint16_t *lc, double *tval) {
    for (int64_t row = (int64_t)blockIdx.x * kBlock + threadIdx.x; row < rows;
         row += (int64_t)gridDim.x * kBlock) {
        const int32_t e = rp[row + 1];
        for (int32_t k = rp[row]; k < e;) {
            const int32_t q = ci[k] / kTileW;
            int32_t pos = trp[(int64_t)q * rows + row];
            for (; k < e && ci[k] / kTileW == q; ++k, ++pos) {
                lc[pos] = (uint16_t)(ci[k] - q * kTileW);
                tval[pos] = val[k];
            }
        }
    }
}

hipError_t launch_tile_build(int64_t rows, int64_t cols, const int32_t *rp, const int32_t *ci_sorted,
                             const double *val_sorted, int32_t *trp, uint16_t *lc, double *tval,
                             int32_t *work, hipStream_t s) {
    const int64_t N = cdiv(cols > 0 ? cols : 1, kTileW) * rows;
    if (N <= 0) return hipSuccess;
    const int64_t ntiles = cdiv(N, kScanTile);
    int32_t *cnt = work;
    int32_t *tiles = cnt + N;
    hipError_t e;
    if ((e = hipMemsetAsync(cnt, 0, sizeof(int32_t) * (size_t)N, s)) != hipSuccess) return e;
    const dim3 gr((unsigned)elementwise_blocks(rows));
    k_tile_count<<<gr, kBlock, 0, s>>>(rows, rp, ci_sorted, cnt);
    k_scan_tiles<<<(unsigned)ntiles, kBlock, 0, s>>>(N, cnt, trp, tiles);
    k_scan_sums<<<1, kBlock, 0, s>>>(ntiles, tiles, trp + N);
    k_scan_add<<<(unsigned)elementwise_blocks(N), kBlock, 0, s>>>(N, trp, tiles);
    k_tile_fill<<<gr, kBlock, 0, s>>>(rows, rp, ci_sorted, val_sorted, trp, lc, tval);
    return hipGetLastError();
}

// out[k] = (alpha * u[i]) * v[j] for the k-th stored entry (i, j): the
// sparse-pattern outer product of the gradient of the solution map
// (dL/da_ij = -lambda_i x_j).  A block takes 256 consecutive rows, stages
// their row pointers in LDS, and its threads walk the rows' entries in
// storage order (coalesced index loads and stores); each finds its row by
// binary search in LDS (the last row whose start is <= k).
__global__ __launch_bounds__(kBlock) void k_csr_outer(int64_t m, const int32_t *__restrict__ rp,
                                                       const int32_t *__restrict__ ci,
                                                       const double *__restrict__ u,
                                                       const double *__restrict__ v, double alpha,
                                                       double *__restrict__ out) {
    __shared__ int32_t srp[kBlock + 1];
    for (int64_t r0 = (int64_t)blockIdx.x * kBlock; r0 < m; r0 += (int64_t)gridDim.x * kBlock) {
        const int rows = (int)((m - r0) < kBlock ? (m - r0) : kBlock);
        for (int t = threadIdx.x; t <= rows; t += kBlock) srp[t] = rp[r0 + t];
        __syncthreads();
        const int32_t k1 = srp[rows];
        for (int32_t k = srp[0] + threadIdx.x; k < k1; k += kBlock) {
            int lo = 0, hi = rows - 1;
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (srp[mid] <= k)
                    lo = mid;
                else
                    hi = mid - 1;
            }
            out[k] = (alpha * u[r0 + lo]) * v[ci[k]];
        }
        __syncthreads();
    }
}

hipError_t launch_csr_outer(int64_t m, const int32_t *rp, const int32_t *ci, const double *u,
                            const double *v, double alpha, double *out, hipStream_t s) {
    if (m <= 0) return hipSuccess;
    const int64_t nb = (m + kBlock - 1) / kBlock;
    const unsigned g = (unsigned)(nb < 65536 ? nb : 65536);
    k_csr_outer<<<g, kBlock, 0, s>>>(m, rp, ci, u, v, alpha, out);
    return hipGetLastError();
}

hipError_t launch_norm2(int64_t n, const double *x, const Out &o, hipStream_t s,
                        int32_t *blocks) {
    const int64_t g = elementwise_blocks(n);
    if (g > o.cap) return hipErrorInvalidValue;
    k_norm2<<<dim3((unsigned)g), kBlock, 0, s>>>(n, x, o);
    if (blocks != nullptr) *blocks = (int32_t)g;
    return hipGetLastError();
}

}  // namespace ta
