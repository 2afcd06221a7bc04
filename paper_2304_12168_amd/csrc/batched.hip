// Batched CTA: many independent solves -- systems s = 0..S-1, each with k_s
// right-hand sides -- advanced in lockstep by one set of kernels.
//
// Layout.  The systems are concatenated into one block-diagonal CSR (and its
// transpose, built on the device); vectors are row-major blocks of K columns
// (K = the smallest power of two >= max k_s), so the nonzero a_ij of a row
// multiplies the K contiguous entries of row j of the input block: one
// gather per nonzero serves every right-hand side.  A group g = s * K + c is
// one (system, right-hand side) solve with its own CTA state (phi, alpha,
// iteration count, stop code); columns c >= k_s are inactive padding.
//
// Precision.  TA_FP64: products, vectors and reductions in FP64, every row
// sum compensated and taken in storage order, so each group follows the
// single-right-hand-side iteration exactly.  TA_FP32 / TA_BF16: the Krylov
// chain uses FP32 or BF16 matrix values and FP32 vectors with FP32
// accumulation; the Gram entries, the step alpha, the iterate (x or y) and
// every true-residual check stay in FP64.  At the end of each chunk of
// iterations the FP64 true residual b - A x replaces the recurrence
// residual of every running group, so the low-precision products only slow
// convergence; the stop test is always the FP64 true residual.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <condition_variable>
#include <memory>
#include <mutex>
#include <new>
#include <type_traits>
#include <string>
#include <thread>
#include <vector>

#include "common.hpp"
#include "device_math.hpp"
#include "host.hpp"

namespace ta {
namespace bt {

constexpr int kMaxK = 64;  // right-hand sides per system
constexpr int kPhiStride = 2 * kTMax + 2;

enum Status : int32_t { kActive = 0, kCandidate = 1, kFinished = 2, kInactive = 3 };

// rows [r0, r1) of the concatenated matrix, all in system `sys`
// One workgroup's share of a unit: the rows [r0, r1) of system sys are cut
// into chunks of `chunk` rows (chunk = 0: one tile of the kernel, 4 waves'
// rows), and workgroup q of the unit's nq takes chunks q, q + nq, q + 2 nq,
// ...  With one-tile chunks the unit's workgroups sweep its rows side by
// side, so x entries gathered by neighbouring rows (a banded or stencil
// matrix) are reused from L2 while they are still there.  Tables are stored
// in dispatch order (see make_blocks); `part` is the entry's index in system
// order, which addresses its partial sums.  Entries with r0 == r1 are
// padding.
struct BRange {
    int32_t r0, r1, sys, part, q, nq, chunk, pad;
};

// Rows of a workgroup, R rows per wave and 4 waves: the lane's first row
// and the one after `it` (row = -1 when done); c0 is the current chunk.
struct BIter {
    int32_t row, c0;
};
__device__ __forceinline__ int32_t bchunk(const BRange &br, int R) {
    return br.chunk > 0 ? br.chunk : 4 * R;
}
__device__ __forceinline__ BIter brow_scan(const BRange &br, int R, int wave, int rsub,
                                           int32_t c0) {
    const int32_t ch = bchunk(br, R);
    for (; c0 < br.r1; c0 += br.nq * ch) {
        const int32_t row = c0 + wave * R + rsub;
        if (row < c0 + ch && row < br.r1) return BIter{row, c0};
    }
    return BIter{-1, c0};
}
__device__ __forceinline__ BIter brow_first(const BRange &br, int R, int wave, int rsub) {
    return brow_scan(br, R, wave, rsub, br.r0 + br.q * bchunk(br, R));
}
__device__ __forceinline__ BIter brow_next(const BRange &br, int R, int wave, int rsub,
                                           BIter it) {
    const int32_t ch = bchunk(br, R), nxt = it.row + 4 * R;
    if (nxt < it.c0 + ch && nxt < br.r1) return BIter{nxt, it.c0};
    return brow_scan(br, R, wave, rsub, it.c0 + br.nq * ch);
}

// per-group state, structure of arrays over G = nsys * K groups
struct Groups {
    int32_t *status, *stop, *repl;
    int64_t *k, *matvecs;
    double *nb, *tol_nb, *tol_ne_nab, *rr, *phi, *alpha, *diag;
    int32_t *flags;  // [0] every group finished, [1] some group waits for a check
    int32_t *sys_active;   // per system: some group still running
    int32_t *dirty;        // per system: its low-precision accumulator holds updates
    const int32_t *ksys;   // right-hand sides in use per system
    const int32_t *a_blk;  // per system: first block of the A-row table (nsys + 1)
    const int32_t *t_blk;  // per system: first block of the A^T-row table (nsys + 1)
    int32_t nsys, K, t;
    int32_t minnorm, mixed;
    int32_t hmode;  // 1: H = A (square symmetric systems), the chain is A passes only
    int32_t t_cycle;  // 1: the order of a group's iteration k is cycle_order(t, k)
    // convex-combination step (accel = theta > 0): per group, whether the
    // last iteration combined, and this iteration's weight a (0 = none)
    double accel;
    int32_t *jumped;
    double *ajump;
    // the enhanced stop (section 3.2): per group, whether this iteration's
    // update is x^ (the solve then stops NORMAL after it)
    int32_t enhanced;
    int32_t *enh_hit;
    int64_t max_iter;
    double tol, tol_normal;
};

enum BGate : int32_t {
    kBRun = 0,      // unless every group has finished
    kBCheck = 1,    // only when some group waits for a true-residual check
    kBFinal = 2,    // only when every group has finished
    kBAlways = 3,
    kBFinalNew = 4, // finished, and x and b - A x were not just computed by a check
    kBDirty = 5,    // always, for the systems whose low-precision accumulator took updates
};

// flags: [0] every group finished, [1] a check is due, [2] a check ran in
// this chunk's tail (x and b - A x are current for every group)
__device__ __forceinline__ bool bgate(int32_t gate, const Groups &gs) {
    switch (gate) {
        case kBRun: return !gs.flags[0];
        case kBCheck: return gs.flags[1] != 0;
        case kBFinal: return gs.flags[0] != 0;
        case kBFinalNew: return gs.flags[0] != 0 && !gs.flags[2];
        default: return true;
    }
}

__host__ __device__ inline uint16_t f32_to_bf16(float f) {
    uint32_t u;
    memcpy(&u, &f, 4);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40);  // quiet NaN
    u += 0x7fffu + ((u >> 16) & 1u);  // round to nearest even
    return (uint16_t)(u >> 16);
}

__device__ __forceinline__ double ldv(const double *v, int64_t k) { return v[k]; }
__device__ __forceinline__ float ldv(const float *v, int64_t k) { return v[k]; }
__device__ __forceinline__ float ldv(const uint16_t *v, int64_t k) {
    return __uint_as_float((uint32_t)v[k] << 16);
}

// Product epilogues: store and column norms into slot; residual b - M x;
// norms only (no store); store, the dot of each output column with the
// input column at the same rows (square systems, H = A) into slot and the
// norms into slot + 1.
enum BEpi : int32_t { kBNorm = 0, kBResid = 1, kBNormOnly = 2, kBNormDot = 3 };

// Value of lane S of the calling lane's group of KL consecutive lanes (KL a
// power of two, groups aligned).  Groups inside one 16-lane DPP row use a
// DPP broadcast (quad_perm within quads, row_newbcast within rows), which
// needs no LDS round trip; wider groups use a lane shuffle.  Every lane of a
// group is active or inactive together.
template <int KL, int S>
__device__ __forceinline__ int32_t grp_bcast(int32_t v, int lane) {
    if constexpr (KL == 1) {
        return v;
    } else if constexpr (KL == 2) {
        return __builtin_amdgcn_mov_dpp(v, S | S << 2 | (2 + S) << 4 | (2 + S) << 6, 0xF,
                                           0xF, false);
    } else if constexpr (KL == 4) {
        return __builtin_amdgcn_mov_dpp(v, S * 0x55, 0xF, 0xF, false);
    } else if constexpr (KL == 8) {
        const int32_t lo = __builtin_amdgcn_mov_dpp(v, 0x150 + S, 0xF, 0xF, false);
        const int32_t hi = __builtin_amdgcn_mov_dpp(v, 0x158 + S, 0xF, 0xF, false);
        return (lane & 8) ? hi : lo;
    } else if constexpr (KL == 16) {
        return __builtin_amdgcn_mov_dpp(v, 0x150 + S, 0xF, 0xF, false);
    } else {
        return __shfl(v, (lane & ~(KL - 1)) + S);
    }
}
template <int KL, int S>
__device__ __forceinline__ float grp_bcast(float v, int lane) {
    return __int_as_float(grp_bcast<KL, S>(__float_as_int(v), lane));
}
template <int KL, int S>
__device__ __forceinline__ double grp_bcast(double v, int lane) {
    const int64_t w = __double_as_longlong(v);
    const int32_t lo = grp_bcast<KL, S>((int32_t)(uint32_t)w, lane);
    const int32_t hi = grp_bcast<KL, S>((int32_t)(w >> 32), lane);
    return __longlong_as_double((int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo));
}
template <typename F, int... I>
__device__ __forceinline__ void static_for_impl(F &&f, std::integer_sequence<int, I...>) {
    (f(std::integral_constant<int, I>{}), ...);
}
template <int N, typename F>
__device__ __forceinline__ void static_for(F &&f) {
    static_for_impl(f, std::make_integer_sequence<int, N>{});
}

// Column indices and values of one chunk of U nonzeros of a row (positions
// k, k + L, ..., k + (U-1) L below the row end e) for the KL lanes that share
// the row: the lanes load distinct entries and pass them round with group
// broadcasts (KL times less load data than every lane loading every entry);
// gbase is the group's first lane.  Entries past the row end come back as
// j = -1, a = 0.
template <int U, int KL, typename V, typename T>
__device__ __forceinline__ void load_chunk(const int32_t *__restrict__ ci,
                                           const V *__restrict__ val, int32_t k, int32_t e,
                                           int L, int cl, int gbase, T sgn, int32_t (&j)[U],
                                           T (&a)[U]) {
    constexpr int NL = (U + KL - 1) / KL;  // entries loaded per lane
    int32_t jl[NL];
    T al[NL];
#pragma unroll
    for (int q = 0; q < NL; ++q) {
        const int idx = cl + q * KL;
        const int32_t kk = k + idx * L;
        jl[q] = -1;
        al[q] = T(0);
        if (idx < U && kk < e) {
            jl[q] = ci[kk];
            al[q] = sgn * (T)ldv(val, kk);
        }
    }
    const int lane = gbase + cl;
    static_for<U>([&](auto uc) {
        constexpr int u = decltype(uc)::value;
        j[u] = grp_bcast<KL, u % KL>(jl[u / KL], lane);
        a[u] = grp_bcast<KL, u % KL>(al[u / KL], lane);
    });
}

// The two halves of load_chunk, for a loop that issues the loads of one
// row's first chunk before the previous row's gathers are consumed: the raw
// per-lane loads, then (once they have arrived) the group broadcasts.
template <int U, int KL, typename V, typename T>
__device__ __forceinline__ void chunk_raw(const int32_t *__restrict__ ci,
                                          const V *__restrict__ val, int32_t k, int32_t e, int L,
                                          int cl, int32_t (&jl)[(U + KL - 1) / KL],
                                          T (&al)[(U + KL - 1) / KL]) {
    constexpr int NL = (U + KL - 1) / KL;
#pragma unroll
    for (int q = 0; q < NL; ++q) {
        const int idx = cl + q * KL;
        const int32_t kk = k + idx * L;
        jl[q] = -1;
        al[q] = T(0);
        if (idx < U && kk < e) {
            jl[q] = ci[kk];
            al[q] = (T)ldv(val, kk);
        }
    }
}
template <int U, int KL, typename T>
__device__ __forceinline__ void chunk_bcast(const int32_t (&jl)[(U + KL - 1) / KL],
                                            const T (&al)[(U + KL - 1) / KL], int lane,
                                            int32_t (&j)[U], T (&a)[U]) {
    static_for<U>([&](auto uc) {
        constexpr int u = decltype(uc)::value;
        j[u] = grp_bcast<KL, u % KL>(jl[u / KL], lane);
        a[u] = grp_bcast<KL, u % KL>(al[u / KL], lane);
    });
}

// ---------------------------------------------------------------------------
// SpMM: Y = M X (or B - M X) over a block table of M's rows.  A lane covers
// CV consecutive columns with one 16-byte load of the input row (2 doubles or
// 4 floats); KL = K / CV lanes cover the K columns, and L lanes split the
// nonzeros of a row (L = 1: terms in storage order, as the single-vector
// kernels; L > 1: lane-strided terms merged by a fixed butterfly).  Per block
// and column: partial sum of Y^2.
// ---------------------------------------------------------------------------
// Vectors of CV consecutive entries, moved with 16-byte accesses.
template <typename T, int CV>
struct alignas(sizeof(T) * CV) VecT {
    T v[CV];
};
template <typename T, int CV>
__device__ __forceinline__ void vld(const T *p, double (&o)[CV]) {
    const VecT<T, CV> w = *reinterpret_cast<const VecT<T, CV> *>(p);
#pragma unroll
    for (int v = 0; v < CV; ++v) o[v] = (double)w.v[v];
}
template <typename T, int CV>
__device__ __forceinline__ void vst(T *p, const double (&o)[CV]) {
    VecT<T, CV> w;
#pragma unroll
    for (int v = 0; v < CV; ++v) w.v[v] = (T)o[v];
    *reinterpret_cast<VecT<T, CV> *>(p) = w;
}

template <typename X, int CV>
struct VecLoad;
template <>
struct VecLoad<double, 1> {
    __device__ static void ld(const double *p, double *o) { o[0] = p[0]; }
};
template <>
struct VecLoad<double, 2> {
    __device__ static void ld(const double *p, double *o) {
        const double2 v = *reinterpret_cast<const double2 *>(p);
        o[0] = v.x;
        o[1] = v.y;
    }
};
template <>
struct VecLoad<float, 1> {
    __device__ static void ld(const float *p, float *o) { o[0] = p[0]; }
};
template <>
struct VecLoad<float, 2> {
    __device__ static void ld(const float *p, float *o) {
        const float2 v = *reinterpret_cast<const float2 *>(p);
        o[0] = v.x;
        o[1] = v.y;
    }
};
template <>
struct VecLoad<float, 4> {
    __device__ static void ld(const float *p, float *o) {
        const float4 v = *reinterpret_cast<const float4 *>(p);
        o[0] = v.x;
        o[1] = v.y;
        o[2] = v.z;
        o[3] = v.w;
    }
};

// nonzeros per lane in flight in the low-precision SpMM (its U): a row of up
// to this many nonzeros takes one round of gathers
constexpr int64_t kRoundNnz = 6;

// Waves per SIMD asked of the SpMM: the low-precision chain at K = 64 fits
// 64 VGPRs without spilling (8 waves instead of 7); the widths in between
// would spill, and so would the dot epilogue (H = A); the FP64 chain keeps
// what its registers allow.
template <typename X, int K, int EPI>
constexpr int kBspmmWaves = (sizeof(X) != 8 && K == 64 && EPI != kBNormDot) ? 8 : 1;

// Widths whose low-precision SpMM runs the row loop software-pipelined (see
// k_bspmm): measured faster at K = 8, 16, 32; at K = 64 the lookahead's
// registers spill (the kernel is held to 64 VGPRs), at K <= 4 the narrow
// groups load a whole chunk per lane and lose occupancy.
template <typename X, int K>
constexpr bool kSpmmPipe = sizeof(X) != 8 && (K == 8 || K == 16 || K == 32);

template <typename X, int K>
struct Lanes {
    static constexpr int CV0 = sizeof(X) == 8 ? 2 : 4;
    static constexpr int CV = K < CV0 ? K : CV0;  // columns per lane
    static constexpr int KL = K / CV;             // lanes across the columns
};

template <typename V, typename X, int K, int EPI, int U>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(kBspmmWaves<X, K, EPI>)))
void k_bspmm(const int32_t *__restrict__ rp,
                                                   const int32_t *__restrict__ ci,
                                                   const V *__restrict__ val,
                                                   const X *__restrict__ x, X *y,
                                                   const double *__restrict__ b,
                                                   const BRange *__restrict__ blocks, Groups gs,
                                                   double2 *partials, int64_t cap, int32_t slot,
                                                   int32_t gate, int32_t L) {
    if (!bgate(gate, gs)) return;
    constexpr int CV = Lanes<X, K>::CV, KL = Lanes<X, K>::KL;
    constexpr bool kF64 = sizeof(X) == 8;
    const BRange br = blocks[blockIdx.x];
    if (br.r0 >= br.r1) return;
    // the iteration chain skips systems with no running group (their
    // partials are never read); checks and diagnostics cover every system
    if (gate == kBRun && !gs.sys_active[br.sys]) return;
    if (gate == kBDirty && !gs.dirty[br.sys]) return;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int cl = lane % KL, l = (lane / KL) % L, rsub = lane / (KL * L);
    const int RL = 64 / (KL * L);
    const int c0 = cl * CV, gbase = lane - cl;
    Acc part[CV], pdot[CV];  // column norms; dots with the input (kBNormDot)
#pragma unroll
    for (int v = 0; v < CV; ++v) part[v] = pdot[v] = Acc{0.0, 0.0};
    // Rows are visited tile by tile (see BRange).  Nonzeros go in chunks of U
    // per lane, each chunk predicated on the row end: a short row issues all
    // its column-index and x loads in one round.
    if constexpr (kSpmmPipe<X, K>) {
        // Low precision: a lane's rows are software-pipelined one deep.  The
        // column indices and values of the next row's first chunk, and the
        // bounds of the row after it, are loaded right after the current
        // row's gathers are issued, so that for short rows each row waits on
        // one memory latency (the gathers) instead of two (indices, then
        // gathers).  The arithmetic is that of the plain loop.
        constexpr int NL = (U + KL - 1) / KL;
        BIter it = brow_first(br, RL, wave, rsub);
        int32_t s_cur = 0, e_cur = 0, s_nxt = 0, e_nxt = 0;
        if (it.row >= 0) {
            s_cur = rp[it.row];
            e_cur = rp[it.row + 1];
        }
        int32_t jl[NL];
        float al[NL];
        chunk_raw<U, KL>(ci, val, s_cur + l, e_cur, L, cl, jl, al);
        BIter nit = it.row >= 0 ? brow_next(br, RL, wave, rsub, it) : it;
        if (nit.row >= 0) {
            s_nxt = rp[nit.row];
            e_nxt = rp[nit.row + 1];
        }
        while (it.row >= 0) {
            const int64_t row = it.row;
            int32_t j[U];
            float a[U], xv[U][CV];
            chunk_bcast<U, KL>(jl, al, gbase + cl, j, a);
#pragma unroll
            for (int u = 0; u < U; ++u) {
                if (j[u] >= 0) {
                    VecLoad<float, CV>::ld((const float *)x + (int64_t)j[u] * K + c0, xv[u]);
                } else {
#pragma unroll
                    for (int v = 0; v < CV; ++v) xv[u][v] = 0.0f;
                }
            }
            // the next row's first chunk and the bounds of the row after it
            chunk_raw<U, KL>(ci, val, s_nxt + l, e_nxt, L, cl, jl, al);
            const BIter nnit = nit.row >= 0 ? brow_next(br, RL, wave, rsub, nit) : nit;
            int32_t s_nn = 0, e_nn = 0;
            if (nnit.row >= 0) {
                s_nn = rp[nnit.row];
                e_nn = rp[nnit.row + 1];
            }
            float acc[CV];
#pragma unroll
            for (int v = 0; v < CV; ++v) acc[v] = 0.0f;
#pragma unroll
            for (int u = 0; u < U; ++u)
                if (j[u] >= 0) {
#pragma unroll
                    for (int v = 0; v < CV; ++v) acc[v] = fmaf(a[u], xv[u][v], acc[v]);
                }
            // the rest of a row longer than one chunk, as in the plain loop
            for (int32_t k = s_cur + l + U * L; k < e_cur; k += U * L) {
                int32_t j2[U];
                float a2[U], xv2[U][CV];
                load_chunk<U, KL>(ci, val, k, e_cur, L, cl, gbase, 1.0f, j2, a2);
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    if (j2[u] >= 0) {
                        VecLoad<float, CV>::ld((const float *)x + (int64_t)j2[u] * K + c0,
                                               xv2[u]);
                    } else {
#pragma unroll
                        for (int v = 0; v < CV; ++v) xv2[u][v] = 0.0f;
                    }
                }
#pragma unroll
                for (int u = 0; u < U; ++u)
                    if (j2[u] >= 0) {
#pragma unroll
                        for (int v = 0; v < CV; ++v) acc[v] = fmaf(a2[u], xv2[u][v], acc[v]);
                    }
            }
            for (int off = KL; off < KL * L; off <<= 1) {
#pragma unroll
                for (int v = 0; v < CV; ++v) acc[v] += __shfl_xor(acc[v], off);
            }
            if (l == 0) {
                double yv[CV];
#pragma unroll
                for (int v = 0; v < CV; ++v) yv[v] = (double)acc[v];
                if constexpr (EPI != kBNormOnly) vst<X, CV>(y + row * K + c0, yv);
                double xi[CV];
                if constexpr (EPI == kBNormDot) vld<X, CV>(x + row * K + c0, xi);
#pragma unroll
                for (int v = 0; v < CV; ++v) {
                    const double q = (double)(X)yv[v];
                    part[v].p = __fma_rn(q, q, part[v].p);
                    if constexpr (EPI == kBNormDot) pdot[v].p = __fma_rn(q, xi[v], pdot[v].p);
                }
            }
            s_cur = s_nxt;
            e_cur = e_nxt;
            s_nxt = s_nn;
            e_nxt = e_nn;
            it = nit;
            nit = nnit;
        }
    } else {
    // The plain loop: the bounds of a lane's next row are loaded before the
    // current row's nonzeros so that their latency overlaps the gathers.
    BIter it = brow_first(br, RL, wave, rsub);
    int32_t s_cur = 0, e_cur = 0;
    if (it.row >= 0) {
        s_cur = rp[it.row];
        e_cur = rp[it.row + 1];
    }
    while (it.row >= 0) {
        const int64_t row = it.row;
        const BIter nit = brow_next(br, RL, wave, rsub, it);
        int32_t s_nxt = 0, e_nxt = 0;
        if (nit.row >= 0) {
            s_nxt = rp[nit.row];
            e_nxt = rp[nit.row + 1];
        }
        const int32_t e = e_cur;
        double yv[CV];
        if constexpr (kF64) {
            Acc acc[CV];
#pragma unroll
            for (int v = 0; v < CV; ++v) {
                acc[v] = Acc{0.0, 0.0};
                if constexpr (EPI == kBResid) {
                    if (l == 0) acc[v].p = b[row * K + c0 + v];
                }
            }
            constexpr double sgn = (EPI == kBResid) ? -1.0 : 1.0;
            for (int32_t k = s_cur + l; k < e; k += U * L) {
                int32_t j[U];
                double a[U], xv[U][CV];
                load_chunk<U, KL>(ci, val, k, e, L, cl, gbase, sgn, j, a);
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    if (j[u] >= 0) {
                        VecLoad<double, CV>::ld((const double *)x + (int64_t)j[u] * K + c0, xv[u]);
                    } else {
#pragma unroll
                        for (int v = 0; v < CV; ++v) xv[u][v] = 0.0;
                    }
                }
#pragma unroll
                for (int u = 0; u < U; ++u)
                    if (j[u] >= 0) {
#pragma unroll
                        for (int v = 0; v < CV; ++v) acc_fma(acc[v], a[u], xv[u][v]);
                    }
            }
            for (int off = KL; off < KL * L; off <<= 1) {
#pragma unroll
                for (int v = 0; v < CV; ++v) {
                    Acc o;
                    o.p = __shfl_xor(acc[v].p, off);
                    o.s = __shfl_xor(acc[v].s, off);
                    acc[v] = acc_merge(acc[v], o);
                }
            }
#pragma unroll
            for (int v = 0; v < CV; ++v) yv[v] = acc_val(acc[v]);
        } else {
            float acc[CV];
#pragma unroll
            for (int v = 0; v < CV; ++v) acc[v] = 0.0f;
            for (int32_t k = s_cur + l; k < e; k += U * L) {
                int32_t j[U];
                float a[U], xv[U][CV];
                load_chunk<U, KL>(ci, val, k, e, L, cl, gbase, 1.0f, j, a);
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    if (j[u] >= 0) {
                        VecLoad<float, CV>::ld((const float *)x + (int64_t)j[u] * K + c0, xv[u]);
                    } else {
#pragma unroll
                        for (int v = 0; v < CV; ++v) xv[u][v] = 0.0f;
                    }
                }
#pragma unroll
                for (int u = 0; u < U; ++u)
                    if (j[u] >= 0) {
#pragma unroll
                        for (int v = 0; v < CV; ++v) acc[v] = fmaf(a[u], xv[u][v], acc[v]);
                    }
            }
            for (int off = KL; off < KL * L; off <<= 1) {
#pragma unroll
                for (int v = 0; v < CV; ++v) acc[v] += __shfl_xor(acc[v], off);
            }
#pragma unroll
            for (int v = 0; v < CV; ++v) yv[v] = (double)acc[v];
        }
        if (l == 0) {
            if constexpr (EPI != kBNormOnly) vst<X, CV>(y + row * K + c0, yv);
            double xi[CV];
            if constexpr (EPI == kBNormDot) vld<X, CV>(x + row * K + c0, xi);
#pragma unroll
            for (int v = 0; v < CV; ++v) {
                const double q = (double)(X)yv[v];
                // FP64 chains: compensated, as the single-vector kernels; the
                // low-precision chain's FP32 outputs need only an FP64 sum
                if constexpr (kF64) {
                    acc_fma(part[v], q, q);
                    if constexpr (EPI == kBNormDot) acc_fma(pdot[v], q, xi[v]);
                } else {
                    part[v].p = __fma_rn(q, q, part[v].p);
                    if constexpr (EPI == kBNormDot) pdot[v].p = __fma_rn(q, xi[v], pdot[v].p);
                }
            }
        }
        s_cur = s_nxt;
        e_cur = e_nxt;
        it = nit;
    }
    }
    // reduce over the rows of the block for each column: the norms into
    // slot (slot + 1 with the dots, which go to slot)
    __shared__ Acc red[kBlock / 64][K];
    auto write_slot = [&](Acc (&pv)[CV], int32_t sl) {
        for (int off = KL; off < 64; off <<= 1) {
#pragma unroll
            for (int v = 0; v < CV; ++v) {
                Acc o;
                o.p = __shfl_xor(pv[v].p, off);
                o.s = __shfl_xor(pv[v].s, off);
                pv[v] = acc_merge(pv[v], o);
            }
        }
        if (lane < KL) {
#pragma unroll
            for (int v = 0; v < CV; ++v) red[wave][c0 + v] = pv[v];
        }
        __syncthreads();
        if (threadIdx.x < K) {
            Acc a = red[0][threadIdx.x];
            for (int w = 1; w < kBlock / 64; ++w) a = acc_merge(a, red[w][threadIdx.x]);
            partials[((int64_t)sl * K + threadIdx.x) * cap + br.part] = make_double2(a.p, a.s);
        }
    };
    write_slot(part, EPI == kBNormDot ? slot + 1 : slot);
    if constexpr (EPI == kBNormDot) {
        __syncthreads();
        write_slot(pdot, slot);
    }
}

// ---------------------------------------------------------------------------
// Dense systems: Y = M X (or B - M X) with matrix cores.
//
// A dense batch stores every system's matrix (and, separately, its transpose)
// row-major with a row stride padded with zeros to a multiple of 16.  One
// workgroup computes a tile of 64 rows of one system against all K columns:
// wave w takes rows 16 w .. 16 w + 15, as ceil(K / 16) output tiles of 16 x 16
// on the MFMA unit.  The input block is first converted to the instruction's
// input type and transposed, once per product (k_bxprep); per stage of 64
// matrix columns the workgroup copies the K x 64 slice of that transpose into
// LDS, each lane loads 16 consecutive matrix entries of its row (4 steps of
// 4), and the products run as
//   FP64: v_mfma_f64_16x16x4f64, 4 instructions per column tile,
//   FP32: v_mfma_f32_16x16x4f32, 4 instructions per column tile,
//   BF16: v_mfma_f32_16x16x16bf16_1k, 1 instruction per column tile (the FP32
//         vector entries are rounded to BF16 on the way into LDS).
// In sub-step ss of the stage at column kb, lane l supplies row l % 16 and
// matrix columns kb + 16 (l / 16) + 4 ss + e (e = 0..3), and the B operand
// the same columns of the transposed input; the instructions sum over l / 16,
// so every column of the stage is covered once.
// The epilogues are those of the sparse kernel.
struct DSys {
    int64_t off;   // offset of the system's matrix in the packed array
    int32_t ld;    // row stride (elements): a multiple of 16, zero padded
    int32_t cols;  // columns of the matrix = rows of the input block it multiplies
    int32_t x0;    // the system's first row in the input block
    int32_t y0;    // the system's first row in the output block
    int32_t xt0;   // the system's first entry in each row of the transposed input (XT)
};

// Entries per row of the system in XT: its row stride rounded up to a stage.
__host__ __device__ inline int32_t xt_len(int32_t ld) { return (ld + 63) / 64 * 64; }

typedef double dbl4 __attribute__((ext_vector_type(4)));
typedef float flt4 __attribute__((ext_vector_type(4)));
typedef short bf4 __attribute__((ext_vector_type(4)));

template <typename V>
struct MfmaOp;
template <>
struct MfmaOp<double> {
    using In = double;     // LDS / operand element
    using Acc4 = dbl4;
    using AccT = double;
    // D entry v of lane l: row l / 16 + 4 v, column l % 16
    __device__ static int drow(int l, int v) { return l / 16 + 4 * v; }
    __device__ static In conv(double x) { return x; }
    __device__ static void step(const In (&a)[4], const In (&b)[4], Acc4 &acc) {
#pragma unroll
        for (int e = 0; e < 4; ++e) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a[e], b[e], acc, 0, 0, 0);
    }
};
template <>
struct MfmaOp<float> {
    using In = float;
    using Acc4 = flt4;
    using AccT = float;
    // D entry v of lane l: row 4 (l / 16) + v, column l % 16
    __device__ static int drow(int l, int v) { return 4 * (l / 16) + v; }
    __device__ static In conv(float x) { return x; }
    __device__ static void step(const In (&a)[4], const In (&b)[4], Acc4 &acc) {
#pragma unroll
        for (int e = 0; e < 4; ++e) acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a[e], b[e], acc, 0, 0, 0);
    }
};
template <>
struct MfmaOp<uint16_t> {
    using In = uint16_t;
    using Acc4 = flt4;
    using AccT = float;
    __device__ static int drow(int l, int v) { return 4 * (l / 16) + v; }
    __device__ static In conv(float x) { return f32_to_bf16(x); }
    __device__ static void step(const In (&a)[4], const In (&b)[4], Acc4 &acc) {
        bf4 av, bv;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            av[e] = (short)a[e];
            bv[e] = (short)b[e];
        }
        acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, bv, acc, 0, 0, 0);
    }
};

// The input block of a dense product, transposed and converted once per
// product for the matrix cores: XT[c * ldxt + xt0 + k] = X[x0 + k][c] (the
// instruction's input type) for the KP = 16 ceil(K / 16) columns c and the
// xt_len(ld) inputs k of each system, zero past the system's columns and
// past K.  Every workgroup of the product then stages its slices of XT with
// plain 16-byte copies instead of converting and transposing X itself.
template <typename V, typename X, int K>
__global__ __launch_bounds__(kBlock) void k_bxprep(const X *__restrict__ x,
                                                    const DSys *__restrict__ dsys, int64_t ldxt,
                                                    typename MfmaOp<V>::In *xt) {
    // a block moves a tile of 64 inputs k by 16 columns c of one system
    // through LDS: reads along the rows of X, writes along the rows of XT
    using Op = MfmaOp<V>;
    using In = typename Op::In;
    constexpr int NCT = (K + 15) / 16;  // column tiles
    constexpr int TK = 64;
    __shared__ In sh[16][TK + 1];
    const DSys ds = dsys[blockIdx.y];
    const int32_t len = xt_len(ds.ld);
    const int c0 = 16 * (int)(blockIdx.x % NCT);
    for (int32_t k0 = (int32_t)(blockIdx.x / NCT) * TK; k0 < len;
         k0 += (int32_t)(gridDim.x / NCT) * TK) {
        for (int e = threadIdx.x; e < TK * 16; e += kBlock) {
            const int k = e / 16, c = e % 16;
            const bool in = k0 + k < ds.cols && c0 + c < K;
            sh[c][k] = Op::conv(in ? x[((int64_t)ds.x0 + k0 + k) * K + c0 + c] : X(0));
        }
        __syncthreads();
        for (int e = threadIdx.x; e < TK * 16; e += kBlock) {
            const int c = e / TK, k = e % TK;
            xt[(int64_t)(c0 + c) * ldxt + ds.xt0 + k0 + k] = sh[c][k];
        }
        __syncthreads();
    }
}

// Split over the matrix columns: with nseg > 1, workgroup b takes tile
// b / nseg and the seg = b % nseg-th share of the columns (a multiple of 16),
// and writes its raw sums to part_y[seg][row][c] (rows of the whole output
// block); k_bgemm_fin adds the shares in order and applies the epilogue.
template <typename V, typename X, int K, int EPI>
__global__ __launch_bounds__(kBlock) void k_bgemm(const V *__restrict__ mat,
                                                   const DSys *__restrict__ dsys,
                                                   const typename MfmaOp<V>::In *__restrict__ xt,
                                                   int64_t ldxt, X *y,
                                                   const double *__restrict__ b,
                                                   const BRange *__restrict__ blocks, Groups gs,
                                                   double2 *partials, int64_t cap, int32_t slot,
                                                   int32_t gate, int32_t nseg,
                                                   typename MfmaOp<V>::AccT *part_y,
                                                   int64_t rows_all) {
    using Op = MfmaOp<V>;
    using In = typename Op::In;
    constexpr int NT = (K + 15) / 16;  // column tiles
    constexpr int KP = 16 * NT;        // columns held in LDS
    if (!bgate(gate, gs)) return;
    const int seg = blockIdx.x % nseg;
    const BRange br = blocks[blockIdx.x / nseg];
    if (br.r0 >= br.r1) return;
    if (gate == kBRun && !gs.sys_active[br.sys]) return;
    if (gate == kBDirty && !gs.dirty[br.sys]) return;
    const DSys ds = dsys[br.sys];
    const int32_t klen = ((ds.ld / 16 + nseg - 1) / nseg) * 16;
    const int32_t k_lo = min(seg * klen, ds.ld), k_hi = min(k_lo + klen, ds.ld);
    const int32_t k_end = xt_len(ds.ld);  // the system's entries in a row of XT
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int li = lane % 16, g = lane / 16;
    const int64_t arow = (int64_t)br.r0 + wave * 16 + li;  // this lane's A-operand row
    const bool arow_ok = arow < br.r1;
    const V *mrow = mat + ds.off + (arow_ok ? (arow - ds.y0) : 0) * (int64_t)ds.ld;
    // A stage covers KB = 64 matrix columns: lane group g holds columns
    // kb + 16 g + [0, 16) of its row and feeds them as 4 sub-steps of 4; the
    // XT slice of the stage is KP rows of KB entries, copied in 16-byte
    // vectors.  The next stage's A entries and XT vectors are loaded into
    // registers while the current stage's products run.
    constexpr int KB = 64;
    constexpr int EV = 16 / (int)sizeof(In);               // entries per 16-byte vector
    constexpr int VR = KB / EV;                            // vectors per XT row of a stage
    constexpr int NXV = (KP * VR + kBlock - 1) / kBlock;   // vectors per thread
    constexpr int LSB = KB + EV;  // LDS row stride (entries): 16-byte aligned, odd in vectors
    __shared__ __attribute__((aligned(16))) In bt[KP * LSB];  // bt[c * LSB + k]
    typename Op::Acc4 acc[NT];
#pragma unroll
    for (int ct = 0; ct < NT; ++ct)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[ct][v] = 0;
    const In *xsys = xt + ds.xt0;
    auto load_x = [&](int32_t kb, uint4 (&r)[NXV]) {
#pragma unroll
        for (int i = 0; i < NXV; ++i) {
            const int e = threadIdx.x + i * kBlock;
            const int c = e / VR, j = e % VR;
            r[i] = make_uint4(0u, 0u, 0u, 0u);
            if (e < KP * VR && kb + j * EV < k_end)
                r[i] = *reinterpret_cast<const uint4 *>(xsys + (int64_t)c * ldxt + kb + j * EV);
        }
    };
    auto load_a = [&](int32_t kb, In (&a)[16]) {
        if (arow_ok && kb + 16 * g < k_hi) {
            constexpr int NV = 16 * (int)sizeof(In) / 16;
            const uint4 *src = reinterpret_cast<const uint4 *>(mrow + kb + 16 * g);
            uint4 q[NV];
#pragma unroll
            for (int w = 0; w < NV; ++w) q[w] = src[w];
            memcpy(a, q, sizeof a);
        } else {
#pragma unroll
            for (int e = 0; e < 16; ++e) a[e] = In(0);
        }
    };
    uint4 xr[NXV];
    In an[16];
    if (k_lo < k_hi) {
        load_x(k_lo, xr);
        load_a(k_lo, an);
    }
    for (int kb = k_lo; kb < k_hi; kb += KB) {
#pragma unroll
        for (int i = 0; i < NXV; ++i) {
            const int e = threadIdx.x + i * kBlock;
            if (e < KP * VR)
                *reinterpret_cast<uint4 *>(bt + (e / VR) * LSB + (e % VR) * EV) = xr[i];
        }
        In a[16];
#pragma unroll
        for (int e = 0; e < 16; ++e) a[e] = an[e];
        __syncthreads();
        if (kb + KB < k_hi) {
            load_x(kb + KB, xr);
            load_a(kb + KB, an);
        }
#pragma unroll
        for (int ss = 0; ss < 4; ++ss) {
            In as[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) as[e] = a[4 * ss + e];
#pragma unroll
            for (int ct = 0; ct < NT; ++ct) {
                In bv[4];
                const In *src = bt + (ct * 16 + li) * LSB + 16 * g + 4 * ss;
#pragma unroll
                for (int e = 0; e < 4; ++e) bv[e] = src[e];
                Op::step(as, bv, acc[ct]);
            }
        }
        __syncthreads();
    }
    if (nseg > 1) {
#pragma unroll
        for (int ct = 0; ct < NT; ++ct) {
            const int c = ct * 16 + li;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int64_t row = (int64_t)br.r0 + wave * 16 + Op::drow(lane, v);
                if (row < br.r1 && c < K) part_y[((int64_t)seg * rows_all + row) * K + c] = acc[ct][v];
            }
        }
        return;
    }
    // epilogue: store, and per-column sums of squares over the tile's rows
    Acc part[NT];
#pragma unroll
    for (int ct = 0; ct < NT; ++ct) {
        part[ct] = Acc{0.0, 0.0};
        const int c = ct * 16 + li;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int64_t row = (int64_t)br.r0 + wave * 16 + Op::drow(lane, v);
            if (row < br.r1 && c < K) {
                double yv = (double)acc[ct][v];
                if constexpr (EPI == kBResid) yv = b[row * K + c] - yv;
                if constexpr (EPI != kBNormOnly) y[row * K + c] = (X)yv;
                const double q = (double)(X)yv;
                acc_fma(part[ct], q, q);
            }
        }
#pragma unroll
        for (int off = 16; off < 64; off <<= 1) {
            Acc o;
            o.p = __shfl_xor(part[ct].p, off);
            o.s = __shfl_xor(part[ct].s, off);
            part[ct] = acc_merge(part[ct], o);
        }
    }
    __shared__ Acc red[kBlock / 64][KP];
    if (lane < 16) {
#pragma unroll
        for (int ct = 0; ct < NT; ++ct) red[wave][ct * 16 + lane] = part[ct];
    }
    __syncthreads();
    if (threadIdx.x < K) {
        Acc a = red[0][threadIdx.x];
        for (int w = 1; w < kBlock / 64; ++w) a = acc_merge(a, red[w][threadIdx.x]);
        partials[((int64_t)slot * K + threadIdx.x) * cap + br.part] = make_double2(a.p, a.s);
    }
}

constexpr int kMaxShares = 16;  // column shares of a dense product, at most

// Sum of the column shares of k_bgemm (in share order) and the epilogue, per
// 64-row tile: one lane per (row, column), K columns across the lanes, 16
// waves, so that a tile's rows are all in flight at once.
constexpr int kFinBlock = 1024;

template <typename T, typename X, int K, int EPI>
__global__ __launch_bounds__(kFinBlock) void k_bgemm_fin(const T *__restrict__ part_y,
                                                          int32_t nseg, int64_t rows_all, X *y,
                                                          const double *__restrict__ b,
                                                          const BRange *__restrict__ blocks,
                                                          Groups gs, double2 *partials,
                                                          int64_t cap, int32_t slot,
                                                          int32_t gate) {
    constexpr int NW = kFinBlock / 64;
    constexpr int R = K >= 64 ? 1 : 64 / K;      // rows per wave and pass
    constexpr int RU = 1;                         // passes of a lane in flight together
    if (!bgate(gate, gs)) return;
    const BRange br = blocks[blockIdx.x];
    if (br.r0 >= br.r1) return;
    if (gate == kBRun && !gs.sys_active[br.sys]) return;
    if (gate == kBDirty && !gs.dirty[br.sys]) return;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int c = lane % K, rsub = lane / K;
    Acc part = {0.0, 0.0};
    // every share of RU rows is loaded before any is added (at most
    // kMaxShares shares); the adds keep share order
    for (int64_t r0 = br.r0 + wave * R + rsub; r0 < br.r1; r0 += RU * NW * R) {
        T p[RU][kMaxShares];
#pragma unroll
        for (int u = 0; u < RU; ++u) {
            const int64_t row = r0 + u * NW * R;
#pragma unroll
            for (int sg = 0; sg < kMaxShares; ++sg)
                p[u][sg] = (sg < nseg && row < br.r1)
                               ? part_y[((int64_t)sg * rows_all + row) * K + c]
                               : T(0);
        }
#pragma unroll
        for (int u = 0; u < RU; ++u) {
            const int64_t row = r0 + u * NW * R;
            if (row >= br.r1) break;
            double v = 0.0;
#pragma unroll
            for (int sg = 0; sg < kMaxShares; ++sg)
                if (sg < nseg) v += (double)p[u][sg];
            if constexpr (EPI == kBResid) v = b[row * K + c] - v;
            if constexpr (EPI != kBNormOnly) y[row * K + c] = (X)v;
            const double q = (double)(X)v;
            acc_fma(part, q, q);
        }
    }
#pragma unroll
    for (int off = K; off < 64; off <<= 1) {
        Acc o;
        o.p = __shfl_xor(part.p, off);
        o.s = __shfl_xor(part.s, off);
        part = acc_merge(part, o);
    }
    __shared__ Acc red[NW][K];
    if (lane < K) red[wave][lane] = part;
    __syncthreads();
    if (threadIdx.x < K) {
        Acc a = red[0][threadIdx.x];
        for (int w = 1; w < NW; ++w) a = acc_merge(a, red[w][threadIdx.x]);
        partials[((int64_t)slot * K + threadIdx.x) * cap + br.part] = make_double2(a.p, a.s);
    }
}

// Wave-level reduction of one slot over a block range, 8 loads in flight.
__device__ double wave_slot_sum(const double2 *p, int32_t b0, int32_t b1) {
    const int lane = threadIdx.x & 63;
    Acc a = {0.0, 0.0};
    for (int32_t base = b0 + lane; base < b1; base += 8 * 64) {
        double2 d[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int32_t i = base + u * 64;
            d[u] = i < b1 ? p[i] : make_double2(0.0, 0.0);
        }
#pragma unroll
        for (int u = 0; u < 8; ++u)
            if (base + u * 64 < b1) a = acc_merge(a, Acc{d[u].x, d[u].y});
    }
    a = group_reduce<64>(a);
    return acc_val(a);
}

__device__ __forceinline__ void group_loop_top(const Groups &gs, int g) {
    if (sqrt(gs.rr[g]) <= gs.tol_nb[g]) {
        gs.status[g] = kCandidate;
    } else if (gs.k[g] >= gs.max_iter) {
        gs.status[g] = kFinished;
        gs.stop[g] = TA_STOP_MAXITER;
    }
}

// Init: ||b||^2 per group (slot 0 of the A-row table) and, with has_nab,
// ||A^T b||^2 (slot 1 of the A^T-row table).
__global__ __launch_bounds__(kBlock) void k_bstep_init(Groups gs, const double2 *partials,
                                                        int64_t cap, int32_t has_nab) {
    const int g = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (g >= gs.nsys * gs.K) return;
    const int s = g / gs.K, c = g % gs.K;
    const double bb = wave_slot_sum(partials + (int64_t)c * cap, gs.a_blk[s], gs.a_blk[s + 1]);
    const double ab = has_nab ? wave_slot_sum(partials + ((int64_t)gs.K + c) * cap, gs.t_blk[s],
                                              gs.t_blk[s + 1])
                              : 0.0;
    if ((threadIdx.x & 63) != 0) return;
    gs.k[g] = 0;
    gs.matvecs[g] = has_nab ? 1 : 0;
    gs.repl[g] = 0;
    gs.tol_ne_nab[g] = gs.tol_normal * sqrt(ab);
    if (c >= gs.ksys[s]) {
        gs.status[g] = kInactive;
        gs.stop[g] = 0;
        gs.nb[g] = 0.0;
        return;
    }
    const double nb = sqrt(bb);
    gs.nb[g] = nb;
    gs.tol_nb[g] = gs.tol * nb;
    gs.rr[g] = bb;
    if (gs.accel > 0.0) {
        gs.jumped[g] = 0;
        gs.ajump[g] = 0.0;
    }
    if (gs.enhanced) gs.enh_hit[g] = 0;
    gs.status[g] = kActive;
    gs.stop[g] = 0;
    if (nb == 0.0) {
        gs.status[g] = kFinished;
        gs.stop[g] = TA_STOP_RESIDUAL;
        return;
    }
    group_loop_top(gs, g);
}

// Order of iteration k under order cycling: the triangle wave 1, 2, ..., t,
// t - 1, ..., 2, 1, 2, ... (period 2 (t - 1)).
__device__ __forceinline__ int cycle_order(int t, int64_t k) {
    if (t <= 1) return 1;
    const int64_t p = k % (2 * (int64_t)t - 2);
    return (int)(p < t ? p + 1 : 2 * (int64_t)t - 1 - p);
}

// Gram step: one block per group; wave w reduces slots w, w + 4, ...
// (even slots: A^T passes over the A^T-row table, odd: A passes; with
// H = A every slot comes from an A pass).
__global__ __launch_bounds__(kBlock) void k_bstep_gram(Groups gs, const double2 *partials,
                                                        int64_t cap) {
    if (gs.flags[0]) return;
    const int g = blockIdx.x;
    if (gs.status[g] != kActive) return;
    const int s = g / gs.K, c = g % gs.K, t = gs.t;
    const int wave = threadIdx.x >> 6;
    __shared__ double phi[kPhiStride];
    for (int q = wave; q < 2 * t; q += kBlock / 64) {
        const int32_t *tab = (q % 2 == 0 && !gs.hmode) ? gs.t_blk : gs.a_blk;
        const double v = wave_slot_sum(partials + ((int64_t)q * gs.K + c) * cap, tab[s], tab[s + 1]);
        if ((threadIdx.x & 63) == 0) phi[q + 1] = v;
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    // with order cycling the chain still runs t steps for every group; a
    // group of order tk < t uses phi_1 .. phi_2tk and takes alpha_i = 0 past
    // tk, so its update is that of order tk
    const int tk = gs.t_cycle ? cycle_order(t, gs.k[g]) : t;
    double *gp = gs.phi + (int64_t)g * kPhiStride;
    for (int i = 1; i <= 2 * t; ++i) gp[i] = phi[i];
    gs.matvecs[g] += gs.hmode ? tk : 2 * tk;
    for (int i = 1; i <= 2 * tk; ++i)
        if (!isfinite(phi[i])) {
            gs.status[g] = kFinished;
            gs.stop[g] = TA_STOP_BREAKDOWN;
            return;
        }
    // the normal-equation test on ||A^T r||: phi_1, or phi_2 = ||A r||^2 when
    // H = A (A symmetric)
    if (sqrt(gs.hmode ? phi[2] : phi[1]) <= gs.tol_ne_nab[g] || phi[2] == 0.0) {
        gs.status[g] = kFinished;
        gs.stop[g] = TA_STOP_NORMAL;
        return;
    }
    double a[kTMax];
    if (gs.enhanced && tk >= 2 && gs.tol_ne_nab[g] > 0.0 &&
        enhanced_hit(phi, tk, gs.hmode, gs.tol_ne_nab[g], a)) {
        for (int i = 0; i < kTMax; ++i) gs.alpha[(int64_t)g * kTMax + i] = i < tk ? a[i] : 0.0;
        gs.enh_hit[g] = 1;
        return;
    }
    gram_alpha(phi, tk, a);
    for (int i = 0; i < tk; ++i)
        if (!isfinite(a[i])) {
            gs.status[g] = kFinished;
            gs.stop[g] = TA_STOP_BREAKDOWN;
            return;
        }
    for (int i = 0; i < kTMax; ++i) gs.alpha[(int64_t)g * kTMax + i] = i < tk ? a[i] : 0.0;
}

struct BVecs {
    void *p[kTMax + 1];
};

// alpha of the block's system, [j][column], for the update kernels
template <int K>
__device__ __forceinline__ void load_alpha(const Groups &gs, int32_t sys, double (*sal)[K]) {
    for (int i = threadIdx.x; i < kTMax * K; i += kBlock) {
        const int j = i / K, c = i % K;
        sal[j][c] = gs.alpha[((int64_t)sys * K + c) * kTMax + j];
    }
    __syncthreads();
}

// R -= sum alpha_j U_{j+1}; with acc_y, also Y += alpha_1 R_old + sum alpha_j
// U_j (the y-form's y; in the mixed x-form the chunk's Z, x's increment
// being A^T Z).  Over the A-row table; partial ||R||^2 per (block, column) in
// slot 0.  A lane covers CV consecutive columns of a row (16-byte accesses);
// every column runs in FP64 and is rounded once to the vector type.  Y is
// held in YA: FP64, or (mixed precision) the low-precision accumulator of the
// current chunk, folded into the FP64 iterate at the chunk's end.
template <typename X, int K, typename YA>
__global__ __launch_bounds__(kBlock) void k_bupdate_r(BVecs U, X *r, YA *yv,
                                                       const BRange *__restrict__ blocks,
                                                       Groups gs, double2 *partials,
                                                       int64_t cap, int32_t acc_y, X *r_keep,
                                                       YA *y_keep) {
    if (gs.flags[0]) return;
    constexpr int CV = Lanes<X, K>::CV, KL = Lanes<X, K>::KL, R = 64 / KL;
    const BRange br = blocks[blockIdx.x];
    if (br.r0 >= br.r1) return;
    __shared__ double sal[kTMax][K];
    load_alpha<K>(gs, br.sys, sal);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int cl = lane % KL, rsub = lane / KL, c0 = cl * CV;
    const int t = gs.t;
    bool act[CV];
    bool any = false;
#pragma unroll
    for (int v = 0; v < CV; ++v) {
        act[v] = gs.status[br.sys * K + c0 + v] == kActive;
        any |= act[v];
    }
    Acc part[CV];
#pragma unroll
    for (int v = 0; v < CV; ++v) part[v] = Acc{0.0, 0.0};
    if (!std::is_same<YA, double>::value && acc_y && any && rsub == 0)
        gs.dirty[br.sys] = 1;  // benign same-value stores
    if (any) {
        for (BIter it = brow_first(br, R, wave, rsub); it.row >= 0;
             it = brow_next(br, R, wave, rsub, it)) {
            const int64_t e = (int64_t)it.row * K + c0;
            // every load of the row is issued before the first use: R, U_1..U_t
            // (unrolled to the largest order, predicated on t) and Y
            VecT<X, CV> uv[kTMax + 1];
            uv[0] = *reinterpret_cast<const VecT<X, CV> *>(r + e);
#pragma unroll
            for (int j = 1; j <= kTMax; ++j)
                if (j <= t) uv[j] = *reinterpret_cast<const VecT<X, CV> *>((const X *)U.p[j] + e);
            VecT<YA, CV> yw;
            if (acc_y) yw = *reinterpret_cast<const VecT<YA, CV> *>(yv + e);
            // r_k and the iterate before the update, for the convex-combination step
            if (r_keep != nullptr) *reinterpret_cast<VecT<X, CV> *>(r_keep + e) = uv[0];
            if (acc_y && y_keep != nullptr) *reinterpret_cast<VecT<YA, CV> *>(y_keep + e) = yw;
            double ri[CV];
#pragma unroll
            for (int v = 0; v < CV; ++v) ri[v] = (double)uv[0].v[v];
            if (acc_y) {
                double yi[CV];
#pragma unroll
                for (int v = 0; v < CV; ++v)
                    yi[v] = __fma_rn(sal[0][c0 + v], ri[v], (double)yw.v[v]);
#pragma unroll
                for (int j = 1; j < kTMax; ++j)
                    if (j < t) {
#pragma unroll
                        for (int v = 0; v < CV; ++v)
                            if (sal[j][c0 + v] != 0.0)  // past a cycled order (unused u_j)
                                yi[v] = __fma_rn(sal[j][c0 + v], (double)uv[j].v[v], yi[v]);
                    }
#pragma unroll
                for (int v = 0; v < CV; ++v)
                    if (!act[v]) yi[v] = (double)yw.v[v];
                vst<YA, CV>(yv + e, yi);
            }
            double rn[CV];
#pragma unroll
            for (int v = 0; v < CV; ++v) rn[v] = ri[v];
#pragma unroll
            for (int j = 0; j < kTMax; ++j)
                if (j < t) {
#pragma unroll
                    for (int v = 0; v < CV; ++v)
                        if (sal[j][c0 + v] != 0.0)
                            rn[v] = __fma_rn(-sal[j][c0 + v], (double)uv[j + 1].v[v], rn[v]);
                }
#pragma unroll
            for (int v = 0; v < CV; ++v) {
                if (!act[v]) rn[v] = ri[v];
                const double q = (double)(X)rn[v];
                if (act[v]) acc_fma(part[v], q, q);
            }
            vst<X, CV>(r + e, rn);
        }
    }
#pragma unroll
    for (int off = KL; off < 64; off <<= 1) {
#pragma unroll
        for (int v = 0; v < CV; ++v) {
            Acc o;
            o.p = __shfl_xor(part[v].p, off);
            o.s = __shfl_xor(part[v].s, off);
            part[v] = acc_merge(part[v], o);
        }
    }
    __shared__ Acc red[kBlock / 64][K];
    if (rsub == 0) {
#pragma unroll
        for (int v = 0; v < CV; ++v) red[wave][c0 + v] = part[v];
    }
    __syncthreads();
    if (threadIdx.x < K) {
        Acc a = red[0][threadIdx.x];
        for (int w = 1; w < kBlock / 64; ++w) a = acc_merge(a, red[w][threadIdx.x]);
        partials[(int64_t)threadIdx.x * cap + br.part] = make_double2(a.p, a.s);
    }
}

// x-form: X += sum alpha_j W_{j-1}, over the A^T-row table (CV columns per
// lane as in k_bupdate_r).  X is held in XA: FP64, or (mixed precision) the
// low-precision accumulator of the current chunk, folded into the FP64 X by
// k_bfold.
template <typename X, int K, typename XA>
__global__ __launch_bounds__(kBlock) void k_bupdate_x(BVecs W, XA *xv,
                                                       const BRange *__restrict__ blocks,
                                                       Groups gs, XA *x_keep) {
    if (gs.flags[0]) return;
    constexpr int CV = Lanes<X, K>::CV, KL = Lanes<X, K>::KL, R = 64 / KL;
    const BRange br = blocks[blockIdx.x];
    if (br.r0 >= br.r1) return;
    __shared__ double sal[kTMax][K];
    load_alpha<K>(gs, br.sys, sal);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int cl = lane % KL, rsub = lane / KL, c0 = cl * CV;
    bool act[CV];
    bool any = false;
#pragma unroll
    for (int v = 0; v < CV; ++v) {
        act[v] = gs.status[br.sys * K + c0 + v] == kActive;
        any |= act[v];
    }
    if (!any) return;
    if (!std::is_same<XA, double>::value && rsub == 0) gs.dirty[br.sys] = 1;
    const int t = gs.t;
    for (BIter it = brow_first(br, R, wave, rsub); it.row >= 0;
         it = brow_next(br, R, wave, rsub, it)) {
        const int64_t e = (int64_t)it.row * K + c0;
        // all loads of the row first: W_0..W_{t-1} (predicated on t) and X
        VecT<X, CV> wv[kTMax];
#pragma unroll
        for (int j = 0; j < kTMax; ++j)
            if (j < t) wv[j] = *reinterpret_cast<const VecT<X, CV> *>((const X *)W.p[j] + e);
        double xi[CV], x0[CV];
        vld<XA, CV>(xv + e, x0);
        if (x_keep != nullptr) vst<XA, CV>(x_keep + e, x0);  // x_k, for the combination
#pragma unroll
        for (int v = 0; v < CV; ++v) xi[v] = x0[v];
#pragma unroll
        for (int j = 0; j < kTMax; ++j)
            if (j < t) {
#pragma unroll
                for (int v = 0; v < CV; ++v)
                    if (sal[j][c0 + v] != 0.0)
                        xi[v] = __fma_rn(sal[j][c0 + v], (double)wv[j].v[v], xi[v]);
            }
#pragma unroll
        for (int v = 0; v < CV; ++v)
            if (!act[v]) xi[v] = x0[v];
        vst<XA, CV>(xv + e, xi);
    }
}

// F += D, D = 0 over a table's rows, for the systems whose accumulator D
// took updates since the last fold (every column: D is zero where nothing
// was added).  Runs ungated at the end of every chunk, before anything reads
// the FP64 block F.
template <typename X, int K>
__global__ __launch_bounds__(kBlock) void k_bfold(X *d, double *f,
                                                   const BRange *__restrict__ blocks,
                                                   Groups gs, int32_t zero_d) {
    constexpr int CV = Lanes<X, K>::CV, KL = Lanes<X, K>::KL, R = 64 / KL;
    const BRange br = blocks[blockIdx.x];
    if (br.r0 >= br.r1 || !gs.dirty[br.sys]) return;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int cl = lane % KL, rsub = lane / KL, c0 = cl * CV;
    for (BIter it = brow_first(br, R, wave, rsub); it.row >= 0;
         it = brow_next(br, R, wave, rsub, it)) {
        const int64_t e = (int64_t)it.row * K + c0;
        double dv[CV], fv[CV];
        vld<X, CV>(d + e, dv);
        vld<double, CV>(f + e, fv);
#pragma unroll
        for (int v = 0; v < CV; ++v) {
            fv[v] += dv[v];
            dv[v] = 0.0;
        }
        vst<double, CV>(f + e, fv);
        if (zero_d) vst<X, CV>(d + e, dv);
    }
}

// F = D (in FP64), D = 0 over a table's rows, for the systems whose
// accumulator D took updates since the last fold.
template <typename X, int K>
__global__ __launch_bounds__(kBlock) void k_bmove(X *d, double *f,
                                                   const BRange *__restrict__ blocks,
                                                   Groups gs) {
    constexpr int CV = Lanes<X, K>::CV, KL = Lanes<X, K>::KL, R = 64 / KL;
    const BRange br = blocks[blockIdx.x];
    if (br.r0 >= br.r1 || !gs.dirty[br.sys]) return;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int cl = lane % KL, rsub = lane / KL, c0 = cl * CV;
    double z[CV] = {};
    for (BIter it = brow_first(br, R, wave, rsub); it.row >= 0;
         it = brow_next(br, R, wave, rsub, it)) {
        const int64_t e = (int64_t)it.row * K + c0;
        double dv[CV];
        vld<X, CV>(d + e, dv);
        vst<double, CV>(f + e, dv);
        vst<X, CV>(d + e, z);
    }
}

// D = 0 over a table's rows, for the systems whose accumulator took updates.
template <typename X, int K>
__global__ __launch_bounds__(kBlock) void k_bzero(X *d, const BRange *__restrict__ blocks,
                                                   Groups gs) {
    constexpr int CV = Lanes<X, K>::CV, KL = Lanes<X, K>::KL, R = 64 / KL;
    const BRange br = blocks[blockIdx.x];
    if (br.r0 >= br.r1 || !gs.dirty[br.sys]) return;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int cl = lane % KL, rsub = lane / KL, c0 = cl * CV;
    double z[CV] = {};
    for (BIter it = brow_first(br, R, wave, rsub); it.row >= 0;
         it = brow_next(br, R, wave, rsub, it))
        vst<X, CV>(d + (int64_t)it.row * K + c0, z);
}

// after the fold: no accumulator holds updates
__global__ __launch_bounds__(kBlock) void k_bdirty_clear(Groups gs) {
    for (int sy = threadIdx.x; sy < gs.nsys; sy += kBlock) gs.dirty[sy] = 0;
}

// End of an iteration: ||r||^2 per group, k, loop-top tests.
__global__ __launch_bounds__(kBlock) void k_bstep_end(Groups gs, const double2 *partials,
                                                       int64_t cap) {
    if (gs.flags[0]) return;
    const int g = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (g >= gs.nsys * gs.K) return;
    if (gs.status[g] != kActive) return;
    const int s = g / gs.K, c = g % gs.K;
    const double rr = wave_slot_sum(partials + (int64_t)c * cap, gs.a_blk[s], gs.a_blk[s + 1]);
    if ((threadIdx.x & 63) != 0) return;
    const double rr0 = gs.rr[g];
    gs.rr[g] = rr;
    gs.k[g] += 1;
    if (gs.enhanced && gs.enh_hit[g]) {  // the update just applied x^
        gs.status[g] = kFinished;
        gs.stop[g] = TA_STOP_NORMAL;
        return;
    }
    if (gs.accel > 0.0) {
        // the convex-combination step of the theorem on the dynamics of
        // first-order CTA (section 3.4): rho = ||r_{k+1}|| / ||r_k|| >= theta,
        // not twice in a row, weight a = rho / (rho + 1); the loop top then
        // waits for the combined residual (k_bstep_jump)
        const double rho = rr0 > 0.0 ? sqrt(rr / rr0) : 0.0;
        const bool jump = !gs.jumped[g] && rho >= gs.accel;
        gs.jumped[g] = jump ? 1 : 0;
        gs.ajump[g] = jump ? rho / (rho + 1.0) : 0.0;
        if (jump) return;
    }
    group_loop_top(gs, g);
}

// The combination for the groups that take it: r = a r_k + (1 - a) r_{k+1}
// (with r != nullptr; partial ||r||^2 in slot 0) and the same of the iterate
// the table's rows hold (y, x, or the chunk's increment; with xy !=
// nullptr), from the copies the update kernels made of r_k and the iterate
// before the update.
template <typename X, int K, typename XA>
__global__ __launch_bounds__(kBlock) void k_bjump(X *r, const X *__restrict__ rp, XA *xy,
                                                   const XA *__restrict__ xyp,
                                                   const BRange *__restrict__ blocks, Groups gs,
                                                   double2 *partials, int64_t cap) {
    if (gs.flags[0]) return;
    constexpr int CV = Lanes<X, K>::CV, KL = Lanes<X, K>::KL, R = 64 / KL;
    const BRange br = blocks[blockIdx.x];
    if (br.r0 >= br.r1) return;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int cl = lane % KL, rsub = lane / KL, c0 = cl * CV;
    double a[CV];
    bool any = false;
#pragma unroll
    for (int v = 0; v < CV; ++v) {
        const int g = br.sys * K + c0 + v;
        a[v] = gs.status[g] == kActive ? gs.ajump[g] : 0.0;
        any |= a[v] > 0.0;
    }
    Acc part[CV];
#pragma unroll
    for (int v = 0; v < CV; ++v) part[v] = Acc{0.0, 0.0};
    if (any) {
        for (BIter it = brow_first(br, R, wave, rsub); it.row >= 0;
             it = brow_next(br, R, wave, rsub, it)) {
            const int64_t e = (int64_t)it.row * K + c0;
            if (r != nullptr) {
                double rv[CV], pv[CV];
                vld<X, CV>(r + e, rv);
                vld<X, CV>(rp + e, pv);
#pragma unroll
                for (int v = 0; v < CV; ++v)
                    if (a[v] > 0.0) rv[v] = __fma_rn(a[v], pv[v], (1.0 - a[v]) * rv[v]);
                vst<X, CV>(r + e, rv);
#pragma unroll
                for (int v = 0; v < CV; ++v)
                    if (a[v] > 0.0) {
                        const double q = (double)(X)rv[v];
                        acc_fma(part[v], q, q);
                    }
            }
            if (xy != nullptr) {
                double xv[CV], pv[CV];
                vld<XA, CV>(xy + e, xv);
                vld<XA, CV>(xyp + e, pv);
#pragma unroll
                for (int v = 0; v < CV; ++v)
                    if (a[v] > 0.0) xv[v] = __fma_rn(a[v], pv[v], (1.0 - a[v]) * xv[v]);
                vst<XA, CV>(xy + e, xv);
            }
        }
    }
    if (r == nullptr) return;
#pragma unroll
    for (int off = KL; off < 64; off <<= 1) {
#pragma unroll
        for (int v = 0; v < CV; ++v) {
            Acc o;
            o.p = __shfl_xor(part[v].p, off);
            o.s = __shfl_xor(part[v].s, off);
            part[v] = acc_merge(part[v], o);
        }
    }
    __shared__ Acc red[kBlock / 64][K];
    if (rsub == 0) {
#pragma unroll
        for (int v = 0; v < CV; ++v) red[wave][c0 + v] = part[v];
    }
    __syncthreads();
    if (threadIdx.x < K) {
        Acc s2 = red[0][threadIdx.x];
        for (int w = 1; w < kBlock / 64; ++w) s2 = acc_merge(s2, red[w][threadIdx.x]);
        partials[(int64_t)threadIdx.x * cap + br.part] = make_double2(s2.p, s2.s);
    }
}

// After the combination: ||r||^2 of the groups that took it, then their loop top.
__global__ __launch_bounds__(kBlock) void k_bstep_jump(Groups gs, const double2 *partials,
                                                        int64_t cap) {
    if (gs.flags[0]) return;
    const int g = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (g >= gs.nsys * gs.K) return;
    if (gs.status[g] != kActive || !(gs.ajump[g] > 0.0)) return;
    const int s = g / gs.K, c = g % gs.K;
    const double rr = wave_slot_sum(partials + (int64_t)c * cap, gs.a_blk[s], gs.a_blk[s + 1]);
    if ((threadIdx.x & 63) != 0) return;
    gs.rr[g] = rr;
    gs.ajump[g] = 0.0;
    group_loop_top(gs, g);
}

// True-residual check (slot 0 holds ||b - A x||^2 per group): a waiting
// group stops or resumes from the true residual; in mixed precision every
// running group resumes from it.
__global__ __launch_bounds__(kBlock) void k_bstep_check(Groups gs, const double2 *partials,
                                                         int64_t cap, int32_t products) {
    if (!gs.flags[1]) return;
    if (blockIdx.x == 0 && threadIdx.x == 0) gs.flags[2] = 1;
    const int g = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (g >= gs.nsys * gs.K) return;
    const int st = gs.status[g];
    if (st != kCandidate && !(gs.mixed && st == kActive)) return;
    const int s = g / gs.K, c = g % gs.K;
    const double rr = wave_slot_sum(partials + (int64_t)c * cap, gs.a_blk[s], gs.a_blk[s + 1]);
    if ((threadIdx.x & 63) != 0) return;
    gs.matvecs[g] += products;
    if (st == kCandidate && sqrt(rr) <= gs.tol_nb[g]) {
        gs.status[g] = kFinished;
        gs.stop[g] = TA_STOP_RESIDUAL;
        gs.rr[g] = rr;
        return;
    }
    gs.rr[g] = rr;
    gs.repl[g] = 1;
    gs.status[g] = kActive;
    if (sqrt(rr) <= gs.tol_nb[g]) {  // a running (mixed) group already converged
        gs.status[g] = kFinished;
        gs.stop[g] = TA_STOP_RESIDUAL;
        gs.repl[g] = 0;
        return;
    }
    if (gs.k[g] >= gs.max_iter) {
        gs.status[g] = kFinished;
        gs.stop[g] = TA_STOP_MAXITER;
    }
}

// R = true residual for the groups that resume from it.
template <typename X, int K>
__global__ __launch_bounds__(kBlock) void k_breplace(const double *__restrict__ rt, X *r,
                                                      const BRange *__restrict__ blocks,
                                                      Groups gs) {
    if (!gs.flags[1]) return;
    constexpr int R = 64 / K;
    const BRange br = blocks[blockIdx.x];
    if (br.r0 >= br.r1) return;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int c = lane % K, rsub = lane / K;
    const int g = br.sys * K + c;
    if (!gs.repl[g]) return;
    for (BIter it = brow_first(br, R, wave, rsub); it.row >= 0;
         it = brow_next(br, R, wave, rsub, it))
        r[(int64_t)it.row * K + c] = (X)rt[(int64_t)it.row * K + c];
}

// Flags: [0] every group finished, [1] some group waits for a check.
// Clears the replacement marks.
__global__ __launch_bounds__(kBlock) void k_bsummary(Groups gs, int32_t reset_check) {
    __shared__ int any_open, any_wait;
    if (threadIdx.x == 0) {
        any_open = 0;
        any_wait = 0;
    }
    __syncthreads();
    const int G = gs.nsys * gs.K;
    int open = 0, wait = 0;
    for (int g = threadIdx.x; g < G; g += kBlock) {
        const int st = gs.status[g];
        open |= (st == kActive || st == kCandidate);
        wait |= (st == kCandidate);
        gs.repl[g] = 0;
    }
    for (int sy = threadIdx.x; sy < gs.nsys; sy += kBlock) {
        int act = 0;
        for (int c = 0; c < gs.K; ++c) act |= (gs.status[sy * gs.K + c] == kActive);
        gs.sys_active[sy] = act;
    }
    if (open) any_open = 1;  // benign same-value stores
    if (wait) any_wait = 1;
    __syncthreads();
    if (threadIdx.x == 0) {
        // mixed precision: every chunk ends with a true-residual pass
        gs.flags[1] = any_wait || (gs.mixed && any_open);
        gs.flags[0] = !any_open;
        if (reset_check) gs.flags[2] = 0;
    }
}

// Exit diagnostics per group: slots 0, 1, 2 hold ||b - A x||^2 (A-row
// table), ||A^T (b - A x)||^2 and ||A^T b||^2 (A^T-row table).
__global__ __launch_bounds__(kBlock) void k_bstep_diag(Groups gs, const double2 *partials,
                                                        int64_t cap) {
    const int g = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (g >= gs.nsys * gs.K) return;
    const int s = g / gs.K, c = g % gs.K;
    const double r2 = wave_slot_sum(partials + (int64_t)c * cap, gs.a_blk[s], gs.a_blk[s + 1]);
    const double w2 = wave_slot_sum(partials + ((int64_t)gs.K + c) * cap, gs.t_blk[s], gs.t_blk[s + 1]);
    const double v2 =
        wave_slot_sum(partials + ((int64_t)2 * gs.K + c) * cap, gs.t_blk[s], gs.t_blk[s + 1]);
    if ((threadIdx.x & 63) != 0) return;
    const double nb = gs.nb[g];
    gs.diag[(int64_t)g * 3 + 0] = nb > 0.0 ? sqrt(r2) / nb : 0.0;
    const double nab = sqrt(v2);
    gs.diag[(int64_t)g * 3 + 1] = (nb > 0.0 && nab > 0.0) ? sqrt(w2) / nab : 0.0;
}

// System of row i (offsets off[0..nsys]).
__device__ __forceinline__ int sys_of(const int64_t *off, int nsys, int64_t i) {
    int lo = 0, hi = nsys;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (off[mid] <= i)
            lo = mid;
        else
            hi = mid;
    }
    return lo;
}

// pack: Bc[i*K + c] = B_s[(i - ro_s) + c m_s] (column-major user blocks),
// through a 64-row LDS tile so both sides are read and written coalesced.
__global__ __launch_bounds__(kBlock) void k_pack(int64_t M, int32_t K,
                                                  const int64_t *__restrict__ ro, int32_t nsys,
                                                  const int32_t *__restrict__ ksys,
                                                  const double *const *__restrict__ src,
                                                  double *dst) {
    __shared__ double tile[64][kMaxK + 1];
    const int t = threadIdx.x;
    for (int64_t r0 = (int64_t)blockIdx.x * 64; r0 < M; r0 += (int64_t)gridDim.x * 64) {
        const int64_t i = r0 + (t % 64);
        if (i < M) {
            const int sy = sys_of(ro, nsys, i);
            const int64_t ms = ro[sy + 1] - ro[sy];
            for (int c = t / 64; c < K; c += kBlock / 64)
                tile[t % 64][c] = c < ksys[sy] ? src[sy][(i - ro[sy]) + (int64_t)c * ms] : 0.0;
        }
        __syncthreads();
        const int64_t rows = (M - r0) < 64 ? (M - r0) : 64;
        for (int e = t; e < rows * K; e += kBlock) dst[r0 * K + e] = tile[e / K][e % K];
        __syncthreads();
    }
}

__global__ __launch_bounds__(kBlock) void k_unpack(int64_t N, int32_t K,
                                                    const int64_t *__restrict__ co, int32_t nsys,
                                                    const int32_t *__restrict__ ksys,
                                                    const double *__restrict__ src,
                                                    double *const *__restrict__ dst) {
    __shared__ double tile[64][kMaxK + 1];
    const int t = threadIdx.x;
    for (int64_t r0 = (int64_t)blockIdx.x * 64; r0 < N; r0 += (int64_t)gridDim.x * 64) {
        const int64_t rows = (N - r0) < 64 ? (N - r0) : 64;
        for (int e = t; e < rows * K; e += kBlock) tile[e / K][e % K] = src[r0 * K + e];
        __syncthreads();
        const int64_t i = r0 + (t % 64);
        if (i < N) {
            const int sy = sys_of(co, nsys, i);
            const int64_t ns = co[sy + 1] - co[sy];
            for (int c = t / 64; c < K; c += kBlock / 64)
                if (c < ksys[sy]) dst[sy][(i - co[sy]) + (int64_t)c * ns] = tile[t % 64][c];
        }
        __syncthreads();
    }
}

// r = (X) b, ||b||^2 partials (slot 0 over the A-row table)
template <typename X, int K>
__global__ __launch_bounds__(kBlock) void k_binit(const double *__restrict__ b, X *r,
                                                   const BRange *__restrict__ blocks,
                                                   double2 *partials, int64_t cap) {
    constexpr int R = 64 / K;
    const BRange br = blocks[blockIdx.x];
    if (br.r0 >= br.r1) return;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int c = lane % K, rsub = lane / K;
    Acc part = {0.0, 0.0};
    for (BIter it = brow_first(br, R, wave, rsub); it.row >= 0;
         it = brow_next(br, R, wave, rsub, it)) {
        const double v = b[(int64_t)it.row * K + c];
        r[(int64_t)it.row * K + c] = (X)v;
        acc_fma(part, v, v);
    }
#pragma unroll
    for (int off = K; off < 64; off <<= 1) {
        Acc o;
        o.p = __shfl_xor(part.p, off);
        o.s = __shfl_xor(part.s, off);
        part = acc_merge(part, o);
    }
    __shared__ Acc red[kBlock / 64][K];
    if (rsub == 0) red[wave][c] = part;
    __syncthreads();
    if (threadIdx.x < K) {
        Acc a = red[0][threadIdx.x];
        for (int w = 1; w < kBlock / 64; ++w) a = acc_merge(a, red[w][threadIdx.x]);
        partials[(int64_t)threadIdx.x * cap + br.part] = make_double2(a.p, a.s);
    }
}

// low-precision copies of the values
__global__ void k_to_f32(int64_t n, const double *__restrict__ a, float *o) {
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kBlock)
        o[i] = (float)a[i];
}
__global__ void k_to_bf16(int64_t n, const double *__restrict__ a, uint16_t *o) {
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kBlock)
        o[i] = f32_to_bf16((float)a[i]);
}

// concatenation: copy system s's CSR into the block-diagonal matrix
__global__ void k_concat(int64_t m, int64_t nnz, const int32_t *__restrict__ rp,
                         const int32_t *__restrict__ ci, const double *__restrict__ val,
                         int64_t row0, int64_t col0, int64_t k0, int32_t *crp, int32_t *cci,
                         double *cval) {
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < m;
         i += (int64_t)gridDim.x * kBlock)
        crp[row0 + i] = (int32_t)(k0 + rp[i]);
    for (int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x; k < nnz;
         k += (int64_t)gridDim.x * kBlock) {
        cci[k0 + k] = (int32_t)(col0 + ci[k]);
        cval[k0 + k] = val[k];
    }
}

// ===========================================================================
// host side
// ===========================================================================
static inline int64_t cdivh(int64_t a, int64_t b) { return (a + b - 1) / b; }
static inline unsigned grid_for(int64_t n) {
    return (unsigned)std::min<int64_t>(std::max<int64_t>(cdivh(n, kBlock), 1), 4096);
}

struct BatchPlan {
    int32_t nsys = 0, precision = TA_FP64;
    int64_t M = 0, N = 0, nnz = 0;
    std::vector<int64_t> ro, co;  // row / column offsets of the systems (nsys + 1)
    std::vector<int32_t> h_arp, h_trp;  // host copies of the row pointers of A and A^T
    std::vector<uint8_t> square;        // 1 where system s has m_s == n_s
    // dense batches (every system TA_DENSE_ROWMAJOR): packed padded copies of
    // A and A^T (FP64, and the plan precision's copies), per-system layouts
    bool dense = false;
    double *d_val = nullptr, *dt_val = nullptr;
    void *d_low = nullptr, *dt_low = nullptr;
    DSys *d_sysA = nullptr, *d_sysT = nullptr;
    // row length of the transposed, converted input block (XT) of the A and
    // A^T products: the sum of the systems' xt_len
    int64_t xt_a = 0, xt_t = 0;
    int64_t xt_len_a = 0, xt_len_t = 0;  // the longest system row of XT, per orientation
    // row lanes picked by timing for the low-precision products, per
    // (K, value type, orientation); filled on first use
    mutable std::mutex tune_mu;
    mutable std::vector<std::pair<int64_t, int32_t>> tuned;
    int32_t *a_rp = nullptr, *a_ci = nullptr, *t_rp = nullptr, *t_ci = nullptr;
    double *a_val = nullptr, *t_val = nullptr;
    void *a_low = nullptr, *t_low = nullptr;
    void *mem = nullptr;
    hipStream_t s_mem = nullptr;
    // dense batches: the same systems as a CSR plan (every entry stored), on
    // which FP64 solves run with compensated sums, so that each column follows
    // the single-right-hand-side iteration exactly; null if the entries do not
    // fit the CSR limits (FP64 solves then use the FP64 matrix-core sums)
    std::unique_ptr<BatchPlan> csr64;
};

static void bplan_free(BatchPlan *P) {
    if (P->csr64) {
        bplan_free(P->csr64.get());
        P->csr64.reset();
    }
    if (P->mem != nullptr) (void)hipFreeAsync(P->mem, P->s_mem);
    P->mem = nullptr;
}

// One dense system (m x n, row stride ld) as CSR with every entry stored:
// row r holds columns 0 .. n-1 in order.
__global__ __launch_bounds__(kBlock) void k_dense_to_csr(int64_t m, int64_t n,
                                                          const double *__restrict__ val,
                                                          int64_t ld, int32_t *rp, int32_t *ci,
                                                          double *cv) {
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t r = (int64_t)blockIdx.x * kBlock + threadIdx.x; r <= m; r += stride)
        rp[r] = (int32_t)(r * n);
    for (int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x; k < m * n; k += stride) {
        const int64_t r = k / n, c = k - r * n;
        ci[k] = (int32_t)c;
        cv[k] = val[r * ld + c];
    }
}

// Transpose of one dense system: src (m x n, stride lds) -> dst (n x m, stride ldd).
__global__ __launch_bounds__(kBlock) void k_dense_transpose(int64_t m, int64_t n,
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

static int bplan_build_dense(int32_t nsys, const ta_mat *A, int32_t precision, hipStream_t s,
                             BatchPlan *P) {
    P->dense = true;
    if (nsys > 65535) return TA_ENOTSUP;  // the input conversion takes one grid row per system
    std::vector<DSys> ha(nsys), ht(nsys);
    int64_t na = 0, nt = 0;
    for (int32_t i = 0; i < nsys; ++i) {
        const int64_t lda = cdivh(std::max<int64_t>(A[i].n, 1), 16) * 16;
        const int64_t ldt = cdivh(std::max<int64_t>(A[i].m, 1), 16) * 16;
        ha[i] = DSys{na, (int32_t)lda, (int32_t)A[i].n, (int32_t)P->co[i], (int32_t)P->ro[i],
                     (int32_t)P->xt_a};
        ht[i] = DSys{nt, (int32_t)ldt, (int32_t)A[i].m, (int32_t)P->ro[i], (int32_t)P->co[i],
                     (int32_t)P->xt_t};
        na += A[i].m * lda;
        nt += A[i].n * ldt;
        P->xt_a += xt_len((int32_t)lda);
        P->xt_t += xt_len((int32_t)ldt);
        P->xt_len_a = std::max<int64_t>(P->xt_len_a, xt_len((int32_t)lda));
        P->xt_len_t = std::max<int64_t>(P->xt_len_t, xt_len((int32_t)ldt));
    }
    Workspace own(s);
    own.reserve(&P->d_val, std::max<int64_t>(na, 1));
    own.reserve(&P->dt_val, std::max<int64_t>(nt, 1));
    own.reserve(&P->d_sysA, nsys);
    own.reserve(&P->d_sysT, nsys);
    float *al32 = nullptr, *tl32 = nullptr;
    uint16_t *al16 = nullptr, *tl16 = nullptr;
    if (precision == TA_FP32) {
        own.reserve(&al32, std::max<int64_t>(na, 1));
        own.reserve(&tl32, std::max<int64_t>(nt, 1));
    } else if (precision == TA_BF16) {
        own.reserve(&al16, std::max<int64_t>(na, 1));
        own.reserve(&tl16, std::max<int64_t>(nt, 1));
    }
    int rc;
    if ((rc = own.commit()) != TA_OK) return rc;
    HIP_TRY(hipMemsetAsync(P->d_val, 0, sizeof(double) * (size_t)std::max<int64_t>(na, 1), s));
    HIP_TRY(hipMemsetAsync(P->dt_val, 0, sizeof(double) * (size_t)std::max<int64_t>(nt, 1), s));
    for (int32_t i = 0; i < nsys; ++i) {
        if (A[i].m == 0 || A[i].n == 0) continue;
        HIP_TRY(hipMemcpy2DAsync(P->d_val + ha[i].off, sizeof(double) * ha[i].ld, A[i].val,
                                 sizeof(double) * A[i].ld, sizeof(double) * A[i].n, A[i].m,
                                 hipMemcpyDeviceToDevice, s));
        if (cdivh(A[i].m, 32) > 65535) return TA_ENOTSUP;
        const dim3 grid((unsigned)cdivh(A[i].n, 32), (unsigned)cdivh(A[i].m, 32));
        k_dense_transpose<<<grid, kBlock, 0, s>>>(A[i].m, A[i].n, P->d_val + ha[i].off, ha[i].ld,
                                                   P->dt_val + ht[i].off, ht[i].ld);
        HIP_TRY(hipGetLastError());
    }
    if (precision == TA_FP32) {
        k_to_f32<<<grid_for(na), kBlock, 0, s>>>(na, P->d_val, al32);
        k_to_f32<<<grid_for(nt), kBlock, 0, s>>>(nt, P->dt_val, tl32);
        P->d_low = al32;
        P->dt_low = tl32;
    } else if (precision == TA_BF16) {
        k_to_bf16<<<grid_for(na), kBlock, 0, s>>>(na, P->d_val, al16);
        k_to_bf16<<<grid_for(nt), kBlock, 0, s>>>(nt, P->dt_val, tl16);
        P->d_low = al16;
        P->dt_low = tl16;
    }
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemcpyAsync(P->d_sysA, ha.data(), sizeof(DSys) * nsys, hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(P->d_sysT, ht.data(), sizeof(DSys) * nsys, hipMemcpyHostToDevice, s));
    HIP_TRY(hipStreamSynchronize(s));
    P->mem = own.release();
    P->s_mem = s;
    return TA_OK;
}

static int bplan_build(int32_t nsys, const ta_mat *A, int32_t precision, hipStream_t s,
                       BatchPlan *P) {
    if (nsys < 1 || A == nullptr) return TA_EINVAL;
    if (precision != TA_FP64 && precision != TA_FP32 && precision != TA_BF16) return TA_EINVAL;
    const bool dense = A[0].kind == TA_DENSE_ROWMAJOR;
    P->nsys = nsys;
    P->precision = precision;
    P->ro.assign(nsys + 1, 0);
    P->co.assign(nsys + 1, 0);
    P->square.assign(nsys, 0);
    int64_t nnz = 0;
    for (int32_t i = 0; i < nsys; ++i) {
        int rc = validate_mat(&A[i]);
        if (rc != TA_OK) return rc;
        if (A[i].kind != (dense ? TA_DENSE_ROWMAJOR : TA_CSR)) return TA_EINVAL;
        P->ro[i + 1] = P->ro[i] + A[i].m;
        P->co[i + 1] = P->co[i] + A[i].n;
        P->square[i] = A[i].m == A[i].n;
        nnz += dense ? A[i].m * A[i].n : A[i].nnz;
    }
    P->M = P->ro[nsys];
    P->N = P->co[nsys];
    P->nnz = nnz;
    if (dense) {
        if (P->M >= INT32_MAX || P->N >= INT32_MAX) return TA_ENOTSUP;
        int rc = bplan_build_dense(nsys, A, precision, s, P);
        if (rc != TA_OK || nnz >= INT32_MAX) return rc;
        // the CSR copy for FP64 solves
        std::vector<ta_mat> cs((size_t)nsys);
        Workspace tmp(s);
        std::vector<int32_t *> rps((size_t)nsys), cis((size_t)nsys);
        std::vector<double *> cvs((size_t)nsys);
        for (int32_t i = 0; i < nsys; ++i) {
            tmp.reserve(&rps[i], A[i].m + 1);
            tmp.reserve(&cis[i], A[i].m * A[i].n);
            tmp.reserve(&cvs[i], A[i].m * A[i].n);
        }
        if ((rc = tmp.commit()) != TA_OK) return rc;
        for (int32_t i = 0; i < nsys; ++i) {
            k_dense_to_csr<<<grid_for(std::max<int64_t>(A[i].m * A[i].n, A[i].m + 1)), kBlock, 0,
                             s>>>(A[i].m, A[i].n, A[i].val, A[i].ld, rps[i], cis[i], cvs[i]);
            HIP_TRY(hipGetLastError());
            cs[i] = ta_mat{TA_CSR, A[i].m, A[i].n, A[i].m * A[i].n, 0, rps[i], cis[i], cvs[i]};
        }
        std::unique_ptr<BatchPlan> sub(new (std::nothrow) BatchPlan);
        if (!sub) return TA_ENOMEM;
        if ((rc = bplan_build(nsys, cs.data(), TA_FP64, s, sub.get())) != TA_OK) {
            bplan_free(sub.get());
            return rc;
        }
        P->csr64 = std::move(sub);
        return TA_OK;
    }
    if (P->M >= INT32_MAX || P->N >= INT32_MAX || nnz >= INT32_MAX) return TA_ENOTSUP;
    const int64_t M = P->M, N = P->N, mx = std::max(M, N);
    Workspace own(s), tmp(s);
    own.reserve(&P->a_rp, M + 1);
    own.reserve(&P->a_ci, nnz);
    own.reserve(&P->a_val, nnz);
    own.reserve(&P->t_rp, N + 1);
    own.reserve(&P->t_ci, nnz);
    own.reserve(&P->t_val, nnz);
    float *al32 = nullptr, *tl32 = nullptr;
    uint16_t *al16 = nullptr, *tl16 = nullptr;
    if (precision == TA_FP32) {
        own.reserve(&al32, nnz);
        own.reserve(&tl32, nnz);
    } else if (precision == TA_BF16) {
        own.reserve(&al16, nnz);
        own.reserve(&tl16, nnz);
    }
    int32_t *flag = nullptr, *work = nullptr;
    tmp.reserve(&flag, 8);
    tmp.reserve(&work, 2 * mx + cdivh(std::max<int64_t>(mx, 1), 1024) + 8 + nnz);
    int rc;
    if ((rc = own.commit()) != TA_OK) return rc;
    if ((rc = tmp.commit()) != TA_OK) return rc;
    int64_t k0 = 0;
    for (int32_t i = 0; i < nsys; ++i) {
        if ((rc = check_csr_device(&A[i], flag, s)) != TA_OK) return rc;
        const int64_t w = std::max<int64_t>(A[i].m, A[i].nnz);
        if (w > 0)
            k_concat<<<grid_for(w), kBlock, 0, s>>>(A[i].m, A[i].nnz, A[i].row_ptr, A[i].col_idx,
                                                    A[i].val, P->ro[i], P->co[i], k0, P->a_rp,
                                                    P->a_ci, P->a_val);
        HIP_TRY(hipGetLastError());
        k0 += A[i].nnz;
    }
    const int32_t total = (int32_t)nnz;
    HIP_TRY(hipMemcpyAsync(P->a_rp + M, &total, sizeof(int32_t), hipMemcpyHostToDevice, s));
    HIP_TRY(launch_transpose(M, N, nnz, P->a_rp, P->a_ci, P->a_val, P->t_rp, P->t_ci, P->t_val,
                             work, flag, s));
    if (precision == TA_FP32 && nnz > 0) {
        k_to_f32<<<grid_for(nnz), kBlock, 0, s>>>(nnz, P->a_val, al32);
        k_to_f32<<<grid_for(nnz), kBlock, 0, s>>>(nnz, P->t_val, tl32);
        P->a_low = al32;
        P->t_low = tl32;
    } else if (precision == TA_BF16 && nnz > 0) {
        k_to_bf16<<<grid_for(nnz), kBlock, 0, s>>>(nnz, P->a_val, al16);
        k_to_bf16<<<grid_for(nnz), kBlock, 0, s>>>(nnz, P->t_val, tl16);
        P->a_low = al16;
        P->t_low = tl16;
    }
    HIP_TRY(hipGetLastError());
    int32_t h = 0;
    HIP_TRY(hipMemcpyAsync(&h, flag, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    P->h_arp.resize(M + 1);
    P->h_trp.resize(N + 1);
    HIP_TRY(hipMemcpyAsync(P->h_arp.data(), P->a_rp, sizeof(int32_t) * (M + 1),
                           hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(P->h_trp.data(), P->t_rp, sizeof(int32_t) * (N + 1),
                           hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (h) return TA_ENOTSUP;
    P->mem = own.release();
    P->s_mem = s;
    return TA_OK;
}

// Block table of one launch over the rows of the systems that take part
// (nrhs[s] > 0, or all if nrhs is null).  About max(2048, nnz K / 2^16)
// workgroups in all.  Each system is one unit, or for a system heavier than
// 1/16 of the total (weight = nonzeros + rows) several units of contiguous
// rows of about that weight; a unit gets workgroups in proportion to its
// weight (at most one per 8 rows), which interleave over its rows in chunks
// (BRange).  `first[s]` is the index of system s's first workgroup in system
// order.  The count is high enough that the workgroups one XCD holds at a
// time cover about one system: a system whose gathers are scattered over its
// whole input block (random sparsity) then has that block to itself in the
// XCD's L2 while it runs.
//
// Dispatch order: workgroup b of a launch runs on XCD b mod 8, and each XCD
// has its own L2.  The units are dealt to the 8 XCDs heaviest first, each to
// the least loaded one; entry 8 i + x of the table is the i-th workgroup of
// XCD x's list (its units in system order), and shorter lists are padded with
// empty entries.  A system's rows therefore share one L2 (a large system: one
// contiguous share per XCD).
static void make_blocks(const std::vector<int64_t> &off, const std::vector<int32_t> &rp, int K,
                        std::vector<BRange> &tab, std::vector<int32_t> &first,
                        const int32_t *nrhs = nullptr, const uint8_t *sq = nullptr) {
    constexpr int kX = 8;
    const size_t nsys = off.size() - 1;
    auto active = [&](size_t sidx) { return nrhs == nullptr || nrhs[sidx] > 0; };
    auto weight = [&](int64_t r0, int64_t r1) { return (int64_t)(rp[r1] - rp[r0]) + (r1 - r0); };
    int64_t total_nnz = 0, total_w = 0;
    for (size_t sidx = 0; sidx < nsys; ++sidx)
        if (active(sidx)) {
            total_nnz += rp[off[sidx + 1]] - rp[off[sidx]];
            total_w += weight(off[sidx], off[sidx + 1]);
        }
    const int64_t target = std::max<int64_t>(2048, cdivh(total_nnz * K, 1 << 16));
    struct Unit {
        int32_t r0, r1, sys;
        int64_t w, b0, nb;  // first workgroup (system order) and count
    };
    std::vector<Unit> units;
    tab.clear();
    first.assign(off.size(), 0);
    int64_t nlog = 0;
    for (size_t sidx = 0; sidx < nsys; ++sidx) {
        first[sidx] = (int32_t)nlog;
        const int64_t r0 = off[sidx], r1 = off[sidx + 1];
        if (r1 <= r0 || !active(sidx)) continue;
        // a system heavier than 1/16 of the total is cut into a multiple of 8
        // pieces, so that the XCDs can take equal shares of it
        const int64_t ws = weight(r0, r1);
        int64_t pieces = cdivh(ws * 2 * kX, std::max<int64_t>(total_w, 1));
        if (pieces > 1) pieces = kX * cdivh(pieces, kX);
        pieces = std::max<int64_t>(1, std::min<int64_t>(pieces, r1 - r0));
        int64_t start = r0;
        for (int64_t pi = 1; pi <= pieces && start < r1; ++pi) {
            int64_t end = r1;
            if (pi < pieces) {
                // rows up to the pi-th weight quantile of the system
                const int64_t goal = ws * pi / pieces;
                end = start + 1;
                while (end < r1 && weight(r0, end) < goal) ++end;
            }
            Unit u{(int32_t)start, (int32_t)end, (int32_t)sidx, weight(start, end), nlog, 0};
            u.nb = std::max<int64_t>(1, std::min<int64_t>((target * u.w + total_w - 1) / total_w,
                                                          (end - start) / 8));
            nlog += u.nb;
            units.push_back(u);
            start = end;
        }
    }
    first[nsys] = (int32_t)nlog;
    // chunk: one tile (0) for square systems, whose rows are taken to gather
    // near their own index (stencils, banded matrices); else the whole
    // per-workgroup share, contiguous
    auto emit = [&](const Unit &u, std::vector<BRange> &dst) {
        const int64_t rows = u.r1 - u.r0;
        const bool square = sq != nullptr && sq[u.sys];
        const int32_t chunk = square ? 0 : (int32_t)cdivh(rows, u.nb);
        for (int64_t q = 0; q < u.nb; ++q)
            dst.push_back(BRange{u.r0, u.r1, u.sys, (int32_t)(u.b0 + q), (int32_t)q, (int32_t)u.nb,
                                 chunk, 0});
    };
    if (nlog < 2 * kX) {
        for (const Unit &u : units) emit(u, tab);
        return;
    }
    std::vector<size_t> order(units.size());
    for (size_t i = 0; i < units.size(); ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(),
                     [&](size_t a, size_t b) { return units[a].w > units[b].w; });
    std::vector<std::vector<size_t>> mine(kX);
    int64_t load[kX] = {};
    for (size_t i : order) {
        int x = 0;
        for (int y = 1; y < kX; ++y)
            if (load[y] < load[x]) x = y;
        load[x] += units[i].w;
        mine[x].push_back(i);
    }
    std::vector<std::vector<BRange>> lists(kX);
    size_t len = 0;
    for (int x = 0; x < kX; ++x) {
        std::sort(mine[x].begin(), mine[x].end());
        for (size_t i : mine[x]) emit(units[i], lists[x]);
        len = std::max(len, lists[x].size());
    }
    tab.assign(len * kX, BRange{0, 0, 0, -1, 0, 1, 1, 0});
    for (int x = 0; x < kX; ++x)
        for (size_t i = 0; i < lists[x].size(); ++i) tab[i * kX + x] = lists[x][i];
}

// Block table of a dense batch: one entry per 64-row tile of every system
// that takes part, in system order.
static void make_dense_blocks(const std::vector<int64_t> &off, std::vector<BRange> &tab,
                              std::vector<int32_t> &first, const int32_t *nrhs = nullptr) {
    const size_t nsys = off.size() - 1;
    tab.clear();
    first.assign(off.size(), 0);
    for (size_t sidx = 0; sidx < nsys; ++sidx) {
        first[sidx] = (int32_t)tab.size();
        if (nrhs != nullptr && nrhs[sidx] == 0) continue;
        for (int64_t r = off[sidx]; r < off[sidx + 1]; r += 64)
            tab.push_back(BRange{(int32_t)r, (int32_t)std::min<int64_t>(r + 64, off[sidx + 1]),
                                 (int32_t)sidx, (int32_t)tab.size(), 0, 1, 64, 0});
    }
    first[nsys] = (int32_t)tab.size();
}

// Lanes per row: about a quarter of the nonzeros per row, within the lanes
// the columns leave free.
static int pick_row_lanes(int64_t nnz, int64_t rows, int KL) {
    const double avg = rows > 0 ? (double)nnz / (double)rows : 0.0;
    int L = 1;
    while (L * 2 <= 64 / KL && (double)(L * 2) * 4.0 <= avg) L *= 2;
    return L;
}

template <typename V, typename X, int K, int EPI>
static void spmm(const int32_t *rp, const int32_t *ci, const void *val, const void *x, void *y,
                 const double *b, const BRange *tab, int32_t nblk, const Groups &gs,
                 double2 *partials, int64_t cap, int32_t slot, int32_t gate, int32_t L,
                 hipStream_t s) {
    if (nblk <= 0) return;
#ifdef TA_SPMM_UNROLL
    constexpr int kU = TA_SPMM_UNROLL;
#else
    // nonzeros per lane in flight: FP64 vectors hold twice the registers.
    // FP32: 6 keeps a 5-point stencil row to one round at 7 waves per SIMD
    // (8: 6 waves; an 8-nonzero row then takes two rounds)
    constexpr int kU = sizeof(X) == 8 ? 4 : 6;
    static_assert(sizeof(X) == 8 || kU == kRoundNnz, "the group split follows the FP32 round");
#endif
    k_bspmm<V, X, K, EPI, kU><<<nblk, kBlock, 0, s>>>(rp, ci, (const V *)val, (const X *)x, (X *)y,
                                                      b, tab, gs, partials, cap, slot, gate, L);
}

// One product of a batched solve: Y = M X (or B - M X for kBResid) with M = A
// (trans = 0) or A^T (trans = 1) of the plan; V is the matrix element type
// (double = the FP64 values, float / uint16_t = the plan's low-precision copy).
// Dense products split over the matrix columns when there are few row tiles:
// about TA_DENSE_BLOCKS workgroups in all, at most 16 shares (on 4 systems of
// 4096^2 at K = 64, 1024 workgroups beat 512 and 2048: more shares cost their
// merge more than the extra workgroups gain).
#ifndef TA_DENSE_BLOCKS
#define TA_DENSE_BLOCKS 1024
#endif
static int32_t dense_nseg(int32_t nblk) {
    return (int32_t)std::min<int64_t>(
        kMaxShares, std::max<int64_t>(1, cdivh(TA_DENSE_BLOCKS, std::max(nblk, 1))));
}

// Doubles of a dense product's scratch that hold XT (the converted,
// transposed input block; 8 bytes per entry covers every input type),
// ahead of the column shares.
static int64_t dense_xt_doubles(const BatchPlan &P, int K) {
    if (!P.dense) return 0;
    const int64_t kp = 16 * ((K + 15) / 16);
    return (kp * std::max(P.xt_a, P.xt_t) + 31) / 32 * 32;
}

template <typename V, typename X, int K, int EPI>
static void prod(const BatchPlan &P, int trans, const void *x, void *y, const double *b,
                 const BRange *tab, int32_t nblk, const Groups &gs, double2 *partials,
                 int64_t cap, int32_t slot, int32_t gate, int32_t L, hipStream_t s,
                 void *scratch = nullptr) {
    if (nblk <= 0) return;
    const bool low = !std::is_same<V, double>::value;
    if (P.dense) {
        // the dot epilogue (H = A) is not on the matrix cores: dense batches
        // reject H = A in low precision, and FP64 runs on the CSR copy
        if constexpr (EPI == kBNormDot) return;
        // scratch (every dense call site passes one): XT, then the column shares
        using T = typename MfmaOp<V>::AccT;
        using In = typename MfmaOp<V>::In;
        const void *m = low ? (trans ? P.dt_low : P.d_low)
                            : (trans ? (const void *)P.dt_val : (const void *)P.d_val);
        const int64_t rows_all = trans ? P.N : P.M;
        const DSys *dsys = trans ? P.d_sysT : P.d_sysA;
        const int64_t ldxt = trans ? P.xt_t : P.xt_a;
        In *xt = (In *)scratch;
        T *shares = (T *)((double *)scratch + dense_xt_doubles(P, K));
        const int32_t nseg = dense_nseg(nblk);
        const int64_t len_max = trans ? P.xt_len_t : P.xt_len_a;
        const int64_t nct = (K + 15) / 16;
        const dim3 gp((unsigned)(nct * std::max<int64_t>(1, std::min<int64_t>(cdivh(len_max, 64), 256))),
                      (unsigned)P.nsys);
        k_bxprep<V, X, K><<<gp, kBlock, 0, s>>>((const X *)x, dsys, ldxt, xt);
        k_bgemm<V, X, K, EPI><<<(unsigned)(nblk * nseg), kBlock, 0, s>>>(
            (const V *)m, dsys, xt, ldxt, (X *)y, b, tab, gs, partials, cap, slot, gate, nseg,
            shares, rows_all);
        if (nseg > 1)
            k_bgemm_fin<T, X, K, EPI><<<nblk, kFinBlock, 0, s>>>(shares, nseg, rows_all, (X *)y,
                                                                  b, tab, gs, partials, cap, slot,
                                                                  gate);
        return;
    }
    const void *val = low ? (trans ? P.t_low : P.a_low)
                          : (trans ? (const void *)P.t_val : (const void *)P.a_val);
    spmm<V, X, K, EPI>(trans ? P.t_rp : P.a_rp, trans ? P.t_ci : P.a_ci, val, x, y, b, tab, nblk,
                       gs, partials, cap, slot, gate, L, s);
}

// Autotuner of the SpMM's row lanes L (lanes sharing one row; rows per wave
// = 64 / (K / CV * L)).  Every power of two from 1 to 64 / (K / CV) is timed
// on the launch's own block table (one warm-up launch, then 3 timed ones
// between HIP events), and the fastest is kept in the plan for this
// (K, value type, orientation).  Dense plans and single candidates need no
// timing.  x and y are scratch blocks of the launch's input and output shape.
template <typename V, typename X, int K>
static int tuned_lanes(const BatchPlan &P, int trans, const BRange *tab, int32_t nblk,
                       const void *x, void *y, const Groups &gs, double2 *partials, int64_t cap,
                       int32_t fallback, int32_t *L, hipStream_t s, int32_t short_rows) {
    *L = fallback;
    constexpr int KL = Lanes<X, K>::KL;
    if (P.dense || nblk <= 0 || 64 / KL < 2) return TA_OK;
    // per row-length class too: the two parts of a group keep their own lanes
    const int64_t key = (((int64_t)K * 16 + (int64_t)sizeof(V)) * 2 + trans) * 2 + short_rows;
    {
        std::lock_guard<std::mutex> lk(P.tune_mu);
        for (auto &e : P.tuned)
            if (e.first == key) {
                *L = e.second;
                return TA_OK;
            }
    }
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    float best = 0.f;
    int32_t best_l = fallback;
    int rc = TA_OK;
    for (int32_t l = 1; l <= 64 / KL; l <<= 1) {
        prod<V, X, K, kBNorm>(P, trans, x, y, nullptr, tab, nblk, gs, partials, cap, 0, kBAlways,
                              l, s);
        hipError_t err = hipEventRecord(e0, s);
        for (int r = 0; r < 3 && err == hipSuccess; ++r)
            prod<V, X, K, kBNorm>(P, trans, x, y, nullptr, tab, nblk, gs, partials, cap, 0,
                                  kBAlways, l, s);
        if (err == hipSuccess) err = hipEventRecord(e1, s);
        if (err == hipSuccess) err = hipEventSynchronize(e1);
        float ms = 0.f;
        if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
        if (err != hipSuccess) {
            hip_msg() = hipGetErrorString(err);
            rc = TA_EHIP;
            break;
        }
        if (l == 1 || ms < best) {
            best = ms;
            best_l = l;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc != TA_OK) return rc;
    *L = best_l;
    std::lock_guard<std::mutex> lk(P.tune_mu);
    P.tuned.emplace_back(key, best_l);
    return TA_OK;
}

// Groups of one batched solve run side by side, one host thread and stream
// each.  The row-lane autotuner times kernels, so tuning is done one group
// at a time (tune), and no group starts iterating before every group has
// tuned (pending reaches 0): the timings see a quiet GPU.
struct GroupSync {
    std::mutex tune, m;
    std::condition_variable cv;
    int pending = 0;
    void arrive() {
        std::lock_guard<std::mutex> lk(m);
        if (--pending == 0) cv.notify_all();
    }
    void wait() {
        std::unique_lock<std::mutex> lk(m);
        cv.wait(lk, [&] { return pending <= 0; });
    }
};
// Arrives once: explicitly after tuning, or on any early return.
struct Arrival {
    GroupSync *g;
    bool done = false;
    void now() {
        if (g != nullptr && !done) g->arrive();
        done = true;
    }
    ~Arrival() { now(); }
};

// The per-K, per-precision pieces of one solve.
template <typename V, typename X, int K>
struct Engine {
    // info[info_off[s] + c] receives the result of column c of system s.
    static int run(const BatchPlan &P, const int32_t *nrhs, const double *const *B,
                   double *const *Xout, const ta_opts *o, int32_t minnorm, ta_info *info,
                   const int64_t *info_off, hipStream_t s, GroupSync *sync = nullptr) {
        Arrival arrival{sync};
        const int32_t nsys = P.nsys, t = o->t;
        const int64_t M = P.M, N = P.N, G = (int64_t)nsys * K;
        const bool mixed = !std::is_same<V, double>::value;

        std::vector<BRange> ta_tab, tt_tab;
        std::vector<int32_t> a_first, t_first;
        int64_t nnz_run = 0;
        if (P.dense) {
            make_dense_blocks(P.ro, ta_tab, a_first, nrhs);
            make_dense_blocks(P.co, tt_tab, t_first, nrhs);
        } else {
            make_blocks(P.ro, P.h_arp, K, ta_tab, a_first, nrhs, P.square.data());
            make_blocks(P.co, P.h_trp, K, tt_tab, t_first, nrhs, P.square.data());
            for (int32_t i = 0; i < nsys; ++i)
                if (nrhs[i] > 0) nnz_run += P.h_arp[P.ro[i + 1]] - P.h_arp[P.ro[i]];
        }
        const int KLc = Lanes<X, K>::KL, KL64 = Lanes<double, K>::KL;
        int64_t m_run = 0, n_run = 0;
        for (int32_t i = 0; i < nsys; ++i)
            if (nrhs[i] > 0) {
                m_run += P.ro[i + 1] - P.ro[i];
                n_run += P.co[i + 1] - P.co[i];
            }
        int La = pick_row_lanes(nnz_run, m_run, KLc), Lt = pick_row_lanes(nnz_run, n_run, KLc);
        const int La64 = pick_row_lanes(nnz_run, m_run, KL64),
                  Lt64 = pick_row_lanes(nnz_run, n_run, KL64);
        const int32_t na = (int32_t)ta_tab.size(), nt = (int32_t)tt_tab.size();
        const int64_t cap = std::max<int64_t>(std::max(na, nt), 1);
        const int32_t nslots = std::max(2 * t, 3);

        Workspace ws(s);
        double *Bc = nullptr, *Y = nullptr, *Xc = nullptr, *RT = nullptr, *TN = nullptr;
        X *R = nullptr;
        X *U[kTMax + 1] = {}, *W[kTMax] = {};
        // mixed precision: the chunk's increments accumulate in D (rows of A):
        // the y-form's y, or in the x-form Z with x's increment A^T Z; at the
        // chunk's end D is folded into the FP64 iterate
        X *D = nullptr;
        double2 *partials = nullptr;
        BRange *d_ta = nullptr, *d_tt = nullptr;
        int32_t *d_afirst = nullptr, *d_tfirst = nullptr, *d_ksys = nullptr;
        int64_t *d_ro = nullptr, *d_co = nullptr;
        const double **d_B = nullptr;
        double **d_X = nullptr;
        Groups gs{};
        ws.reserve(&Bc, M * K);
        ws.reserve(&R, M * K);
        for (int j = 1; j <= t; ++j) ws.reserve(&U[j], M * K);
        // W_j is kept for the x update only in the FP64 x-form; with H = A
        // (square systems) the chain has no A^T pass, and W_0 only serves the
        // row-lane tuner of the low-precision chain
        const bool ha = o->h_mode == 1;
        const bool one_w = minnorm || mixed;
        for (int j = 0; j < (ha ? (mixed ? 1 : 0) : (one_w ? 1 : t)); ++j) ws.reserve(&W[j], N * K);
        if (minnorm) ws.reserve(&Y, M * K);
        ws.reserve(&Xc, N * K);
        if (mixed) ws.reserve(&D, M * K);
        ws.reserve(&RT, M * K);
        ws.reserve(&TN, N * K);
        // the convex-combination step: r_k and the iterate before each update
        // (y, x with H = A, or the low-precision increment: M rows; the FP64
        // x-form's x: N rows, FP64)
        const bool accel = o->accel > 0.0;
        X *Rk = nullptr, *XYk_lo = nullptr;  // the low-precision increment's copy
        double *XYk_64 = nullptr;            // y's or x's (FP64)
        if (accel) {
            ws.reserve(&Rk, M * K);
            if (mixed)
                ws.reserve(&XYk_lo, M * K);
            else
                ws.reserve(&XYk_64, (minnorm || ha ? M : N) * K);
            ws.reserve(&gs.jumped, G);
            ws.reserve(&gs.ajump, G);
        }
        if (o->enhanced) ws.reserve(&gs.enh_hit, G);
        double *DS = nullptr;  // column shares of the dense products
        if (P.dense)
            ws.reserve(&DS, dense_xt_doubles(P, K) +
                                (int64_t)dense_nseg(std::max(std::min(na, nt), 1)) *
                                    std::max<int64_t>(std::max(M, N), 1) * K);
        ws.reserve(&partials, (int64_t)nslots * K * cap);
        ws.reserve(&d_ta, std::max(na, 1));
        ws.reserve(&d_tt, std::max(nt, 1));
        ws.reserve(&d_afirst, nsys + 1);
        ws.reserve(&d_tfirst, nsys + 1);
        ws.reserve(&d_ksys, nsys);
        ws.reserve(&d_ro, nsys + 1);
        ws.reserve(&d_co, nsys + 1);
        ws.reserve(&d_B, nsys);
        ws.reserve(&d_X, nsys);
        ws.reserve(&gs.status, G);
        ws.reserve(&gs.stop, G);
        ws.reserve(&gs.repl, G);
        ws.reserve(&gs.k, G);
        ws.reserve(&gs.matvecs, G);
        ws.reserve(&gs.nb, G);
        ws.reserve(&gs.tol_nb, G);
        ws.reserve(&gs.tol_ne_nab, G);
        ws.reserve(&gs.rr, G);
        ws.reserve(&gs.phi, G * kPhiStride);
        ws.reserve(&gs.alpha, G * kTMax);
        ws.reserve(&gs.diag, G * 3);
        ws.reserve(&gs.flags, 4);
        ws.reserve(&gs.sys_active, nsys);
        ws.reserve(&gs.dirty, nsys);
        int rc = ws.commit();
        if (rc != TA_OK) return rc;

        // host tables -> device (pageable copies complete before return)
        std::vector<int32_t> ks(nsys);
        for (int32_t i = 0; i < nsys; ++i) ks[i] = nrhs[i];
        HIP_TRY(hipMemcpyAsync(d_ta, ta_tab.data(), sizeof(BRange) * na, hipMemcpyHostToDevice, s));
        HIP_TRY(hipMemcpyAsync(d_tt, tt_tab.data(), sizeof(BRange) * nt, hipMemcpyHostToDevice, s));
        HIP_TRY(hipMemcpyAsync(d_afirst, a_first.data(), sizeof(int32_t) * (nsys + 1),
                               hipMemcpyHostToDevice, s));
        HIP_TRY(hipMemcpyAsync(d_tfirst, t_first.data(), sizeof(int32_t) * (nsys + 1),
                               hipMemcpyHostToDevice, s));
        HIP_TRY(hipMemcpyAsync(d_ksys, ks.data(), sizeof(int32_t) * nsys, hipMemcpyHostToDevice, s));
        HIP_TRY(hipMemcpyAsync(d_ro, P.ro.data(), sizeof(int64_t) * (nsys + 1), hipMemcpyHostToDevice,
                               s));
        HIP_TRY(hipMemcpyAsync(d_co, P.co.data(), sizeof(int64_t) * (nsys + 1), hipMemcpyHostToDevice,
                               s));
        HIP_TRY(hipMemcpyAsync(d_B, B, sizeof(double *) * nsys, hipMemcpyHostToDevice, s));
        HIP_TRY(hipMemcpyAsync(d_X, Xout, sizeof(double *) * nsys, hipMemcpyHostToDevice, s));
        HIP_TRY(hipMemsetAsync(gs.flags, 0, sizeof(int32_t) * 4, s));
        HIP_TRY(hipMemsetAsync(gs.sys_active, 0, sizeof(int32_t) * nsys, s));
        HIP_TRY(hipMemsetAsync(gs.dirty, 0, sizeof(int32_t) * nsys, s));
        HIP_TRY(hipMemsetAsync(Xc, 0, sizeof(double) * (size_t)(N * K), s));
        if (mixed) HIP_TRY(hipMemsetAsync(D, 0, sizeof(X) * (size_t)(M * K), s));
        if (minnorm) HIP_TRY(hipMemsetAsync(Y, 0, sizeof(double) * (size_t)(M * K), s));
        gs.ksys = d_ksys;
        gs.a_blk = d_afirst;
        gs.t_blk = d_tfirst;
        gs.nsys = nsys;
        gs.K = K;
        gs.t = t;
        gs.minnorm = minnorm;
        gs.mixed = mixed;
        gs.hmode = ha ? 1 : 0;
        gs.t_cycle = o->t_cycle;
        gs.accel = o->accel;
        gs.enhanced = o->enhanced;
        gs.max_iter = o->max_iter;
        gs.tol = o->tol;
        gs.tol_normal = o->tol_normal;
        const unsigned gw = (unsigned)cdivh(G, 4);  // one wave per group

        // row lanes of the low-precision chain: timed once per plan and K
        if (mixed && M > 0 && N > 0) {
            std::unique_lock<std::mutex> lk;
            if (sync != nullptr) lk = std::unique_lock<std::mutex>(sync->tune);
            HIP_TRY(hipMemsetAsync(R, 0, sizeof(X) * (size_t)(M * K), s));
            HIP_TRY(hipMemsetAsync(W[0], 0, sizeof(X) * (size_t)(N * K), s));
            const int32_t short_rows = nnz_run <= kRoundNnz * m_run ? 1 : 0;
            if ((rc = tuned_lanes<V, X, K>(P, 1, d_tt, nt, R, W[0], gs, partials, cap, Lt, &Lt,
                                           s, short_rows)) != TA_OK)
                return rc;
            if ((rc = tuned_lanes<V, X, K>(P, 0, d_ta, na, W[0], U[1], gs, partials, cap, La, &La,
                                           s, short_rows)) != TA_OK)
                return rc;
            HIP_TRY(hipStreamSynchronize(s));
        }
        if (sync != nullptr) {
            arrival.now();
            sync->wait();
        }
        // initial state
        if (M > 0)
            k_pack<<<(unsigned)std::min<int64_t>(cdivh(M, 64), 4096), kBlock, 0, s>>>(
                M, K, d_ro, nsys, d_ksys, d_B, Bc);
        if (na > 0) k_binit<X, K><<<na, kBlock, 0, s>>>(Bc, R, d_ta, partials, cap);
        const bool has_nab = o->tol_normal > 0.0;
        if (has_nab)
            prod<double, double, K, kBNormOnly>(P, 1, Bc, TN, nullptr, d_tt, nt,
                                                gs, partials, cap, 1, kBAlways, Lt64, s, DS);
        k_bstep_init<<<gw, kBlock, 0, s>>>(gs, partials, cap, has_nab ? 1 : 0);
        k_bsummary<<<1, kBlock, 0, s>>>(gs, 1);
        HIP_TRY(hipGetLastError());

        // the stream the chunk's kernels go to: s, or the capture stream
        hipStream_t cs = s;
        auto iteration = [&]() {
            for (int j = 0; j < t; ++j) {
                const void *uj = j == 0 ? (const void *)R : (const void *)U[j];
                if (ha) {
                    // u_{j+1} = A u_j; phi_{2j+1} = u_j . u_{j+1}, phi_{2j+2} = ||u_{j+1}||^2
                    prod<V, X, K, kBNormDot>(P, 0, uj, U[j + 1], nullptr, d_ta, na, gs,
                                             partials, cap, 2 * j, kBRun, La, cs, DS);
                    continue;
                }
                X *wj = W[one_w ? 0 : j];
                prod<V, X, K, kBNorm>(P, 1, uj, wj, nullptr, d_tt, nt, gs, partials,
                                      cap, 2 * j, kBRun, Lt, cs, DS);
                prod<V, X, K, kBNorm>(P, 0, wj, U[j + 1], nullptr, d_ta, na, gs,
                                      partials, cap, 2 * j + 1, kBRun, La, cs, DS);
            }
            k_bstep_gram<<<(unsigned)G, kBlock, 0, cs>>>(gs, partials, cap);
            BVecs uv{};
            uv.p[0] = R;
            for (int j = 1; j <= t; ++j) uv.p[j] = U[j];
            // the x-form with H = A takes y-form's update into x itself
            // (x += sum_i alpha_i u_{i-1}); x and the rows of A coincide
            if (na > 0) {
                if (mixed)
                    k_bupdate_r<X, K, X><<<na, kBlock, 0, cs>>>(uv, R, D, d_ta, gs, partials, cap,
                                                                 1, Rk, XYk_lo);
                else
                    k_bupdate_r<X, K, double><<<na, kBlock, 0, cs>>>(
                        uv, R, ha ? Xc : Y, d_ta, gs, partials, cap, (minnorm || ha) ? 1 : 0, Rk,
                        XYk_64);
            }
            if (!minnorm && !mixed && !ha && nt > 0) {
                BVecs wv{};
                for (int j = 0; j < t; ++j) wv.p[j] = W[j];
                k_bupdate_x<X, K, double><<<nt, kBlock, 0, cs>>>(wv, Xc, d_tt, gs, XYk_64);
            }
            k_bstep_end<<<gw, kBlock, 0, cs>>>(gs, partials, cap);
            if (accel) {
                // the combination of r and of the iterate: r and y, x (H = A) or
                // the chunk's increment on the A rows; the FP64 x-form's x on
                // the A^T rows
                if (na > 0) {
                    if (mixed)
                        k_bjump<X, K, X><<<na, kBlock, 0, cs>>>(R, Rk, D, XYk_lo, d_ta, gs,
                                                                 partials, cap);
                    else
                        k_bjump<X, K, double><<<na, kBlock, 0, cs>>>(
                            R, Rk, (minnorm || ha) ? (minnorm ? Y : Xc) : nullptr, XYk_64, d_ta, gs,
                            partials, cap);
                }
                if (!minnorm && !mixed && !ha && nt > 0)
                    k_bjump<X, K, double><<<nt, kBlock, 0, cs>>>(nullptr, nullptr, Xc, XYk_64,
                                                                  d_tt, gs, partials, cap);
                k_bstep_jump<<<gw, kBlock, 0, cs>>>(gs, partials, cap);
            }
            k_bsummary<<<1, kBlock, 0, cs>>>(gs, 1);
        };
        const int32_t products = minnorm ? 2 : 1;
        auto tail = [&]() {
            if (mixed) {
                if (minnorm || ha) {
                    // y += Z (or, with H = A, x += Z: x and the rows coincide)
                    if (na > 0) k_bfold<X, K><<<na, kBlock, 0, cs>>>(D, minnorm ? Y : Xc, d_ta, gs, 1);
                } else {
                    // x += A^T Z (the chunk's increment), Z = 0.  The product
                    // is the FP64 one: with the low-precision A^T the increment
                    // would leave range(A^T) by the values' rounding, and the
                    // x-form would lose its minimum-norm limit (Theorem 1 (4))
                    // on systems with a null space
                    if (na > 0) k_bmove<X, K><<<na, kBlock, 0, cs>>>(D, RT, d_ta, gs);
                    prod<double, double, K, kBNorm>(P, 1, RT, TN, nullptr, d_tt, nt, gs,
                                                    partials, cap, 1, kBDirty, Lt64, cs, DS);
                    if (nt > 0) k_bfold<double, K><<<nt, kBlock, 0, cs>>>(TN, Xc, d_tt, gs, 0);
                }
                k_bdirty_clear<<<1, kBlock, 0, cs>>>(gs);
            }
            // true-residual check for waiting groups (every running group when mixed)
            if (minnorm)
                prod<double, double, K, kBNorm>(P, 1, Y, Xc, nullptr, d_tt, nt, gs,
                                                partials, cap, 1, kBCheck, Lt64, cs, DS);
            prod<double, double, K, kBResid>(P, 0, Xc, RT, Bc, d_ta, na, gs,
                                             partials, cap, 0, kBCheck, La64, cs, DS);
            k_bstep_check<<<gw, kBlock, 0, cs>>>(gs, partials, cap, products);
            if (na > 0) k_breplace<X, K><<<na, kBlock, 0, cs>>>(RT, R, d_ta, gs);
            k_bsummary<<<1, kBlock, 0, cs>>>(gs, 0);
            // exit diagnostics once every group has finished; x (y-form) and
            // b - A x are recomputed only if no check just produced them
            if (minnorm)
                prod<double, double, K, kBNorm>(P, 1, Y, Xc, nullptr, d_tt, nt, gs,
                                                partials, cap, 1, kBFinalNew, Lt64, cs, DS);
            prod<double, double, K, kBResid>(P, 0, Xc, RT, Bc, d_ta, na, gs,
                                             partials, cap, 0, kBFinalNew, La64, cs, DS);
            prod<double, double, K, kBNormOnly>(P, 1, RT, TN, nullptr, d_tt, nt,
                                                gs, partials, cap, 1, kBFinal, Lt64, cs, DS);
            prod<double, double, K, kBNormOnly>(P, 1, Bc, TN, nullptr, d_tt, nt,
                                                gs, partials, cap, 2, kBFinal, Lt64, cs, DS);
        };

        int32_t hflags[4] = {0, 0, 0, 0};
        int64_t chunk = o->chunk > 0 ? o->chunk : 4;
        // mixed precision: a chunk ends with the FP64 true-residual pass, and a
        // group can stop only there; up to 64 iterations between checks with
        // FP32 products, 8 with BF16 (whose recurrence drifts from the true
        // residual within a few dozen iterations)
        const int64_t chunk_cap =
            o->chunk > 0 ? o->chunk : (mixed ? (sizeof(V) == 2 ? 8 : 64) : 64);
        std::vector<int64_t> kh(G), kh_prev(G, -1);
        // Each chunk (iterations + tail) is captured once per length as a HIP
        // graph on a private stream and replayed on s; launch_mode 1 launches
        // the kernels one by one instead.
        struct Graphs {
            std::vector<std::pair<int64_t, hipGraphExec_t>> ex;
            hipStream_t cap = nullptr;
            ~Graphs() {
                for (auto &e : ex) (void)hipGraphExecDestroy(e.second);
                if (cap != nullptr) (void)hipStreamDestroy(cap);
            }
        } graphs;
        const bool use_graph = o->launch_mode == 0;
        auto run_chunk = [&](int64_t n) -> int {
            if (!use_graph) {
                cs = s;
                for (int64_t i = 0; i < n; ++i) iteration();
                tail();
                HIP_TRY(hipGetLastError());
                return TA_OK;
            }
            hipGraphExec_t ge = nullptr;
            for (auto &e : graphs.ex)
                if (e.first == n) ge = e.second;
            if (ge == nullptr) {
                if (graphs.cap == nullptr)
                    HIP_TRY(hipStreamCreateWithFlags(&graphs.cap, hipStreamNonBlocking));
                cs = graphs.cap;
                HIP_TRY(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
                for (int64_t i = 0; i < n; ++i) iteration();
                tail();
                const hipError_t le = hipGetLastError();
                hipGraph_t gr = nullptr;
                const hipError_t ce = hipStreamEndCapture(cs, &gr);
                cs = s;
                HIP_TRY(le);
                HIP_TRY(ce);
                const hipError_t ie = hipGraphInstantiate(&ge, gr, nullptr, nullptr, 0);
                (void)hipGraphDestroy(gr);
                HIP_TRY(ie);
                graphs.ex.emplace_back(n, ge);
            }
            HIP_TRY(hipGraphLaunch(ge, s));
            return TA_OK;
        };
        for (;;) {
            if ((rc = run_chunk(chunk)) != TA_OK) return rc;
            HIP_TRY(hipMemcpyAsync(hflags, gs.flags, sizeof(hflags), hipMemcpyDeviceToHost, s));
            HIP_TRY(hipStreamSynchronize(s));
            if (hflags[0]) break;
            // progress: some group's k or product count moved
            HIP_TRY(hipMemcpyAsync(kh.data(), gs.matvecs, sizeof(int64_t) * G, hipMemcpyDeviceToHost,
                                   s));
            HIP_TRY(hipStreamSynchronize(s));
            if (kh == kh_prev) {
                hip_msg() = "batched iteration made no progress";
                return TA_EHIP;
            }
            kh_prev = kh;
            chunk = std::min(chunk_cap, chunk * 2);
        }
        k_bstep_diag<<<gw, kBlock, 0, s>>>(gs, partials, cap);
        if (N > 0)
            k_unpack<<<(unsigned)std::min<int64_t>(cdivh(N, 64), 4096), kBlock, 0, s>>>(
                N, K, d_co, nsys, d_ksys, Xc, d_X);
        HIP_TRY(hipGetLastError());

        // per-group results to the host
        std::vector<int32_t> hst(G), hstop(G);
        std::vector<int64_t> hk(G), hmv(G);
        std::vector<double> hdiag(G * 3);
        HIP_TRY(hipMemcpyAsync(hst.data(), gs.status, sizeof(int32_t) * G, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipMemcpyAsync(hstop.data(), gs.stop, sizeof(int32_t) * G, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipMemcpyAsync(hk.data(), gs.k, sizeof(int64_t) * G, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipMemcpyAsync(hmv.data(), gs.matvecs, sizeof(int64_t) * G, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipMemcpyAsync(hdiag.data(), gs.diag, sizeof(double) * G * 3, hipMemcpyDeviceToHost,
                               s));
        HIP_TRY(hipStreamSynchronize(s));
        for (int32_t sy = 0; sy < nsys; ++sy)
            for (int32_t c = 0; c < nrhs[sy]; ++c) {
                const int64_t g = (int64_t)sy * K + c;
                ta_info &inf = info[info_off[sy] + c];
                memset(&inf, 0, sizeof inf);
                inf.iters = hk[g];
                inf.matvecs = hmv[g];
                inf.stop = hstop[g];
                inf.rel_res = hdiag[g * 3 + 0];
                inf.rel_normal = hdiag[g * 3 + 1];
            }
        return TA_OK;
    }
};

template <typename V, typename X>
static int run_k(int K, const BatchPlan &P, const int32_t *nrhs, const double *const *B,
                 double *const *Xo, const ta_opts *o, int32_t minnorm, ta_info *info,
                 const int64_t *off, hipStream_t s, GroupSync *g) {
    switch (K) {
        case 1: return Engine<V, X, 1>::run(P, nrhs, B, Xo, o, minnorm, info, off, s, g);
        case 2: return Engine<V, X, 2>::run(P, nrhs, B, Xo, o, minnorm, info, off, s, g);
        case 4: return Engine<V, X, 4>::run(P, nrhs, B, Xo, o, minnorm, info, off, s, g);
        case 8: return Engine<V, X, 8>::run(P, nrhs, B, Xo, o, minnorm, info, off, s, g);
        case 16: return Engine<V, X, 16>::run(P, nrhs, B, Xo, o, minnorm, info, off, s, g);
        case 32: return Engine<V, X, 32>::run(P, nrhs, B, Xo, o, minnorm, info, off, s, g);
        default: return Engine<V, X, 64>::run(P, nrhs, B, Xo, o, minnorm, info, off, s, g);
    }
}

// Cut a system's right-hand sides into two power-of-two pieces (see
// solve_batched); 0 = one piece padded to the next power of two.
#ifndef TA_SPLIT_COLUMNS
#define TA_SPLIT_COLUMNS 1
#endif
constexpr int kSplitColumns = TA_SPLIT_COLUMNS;
// 1 = run the width groups one after another on the caller's stream (a
// measurement build: kernel durations without other groups beside them)
#ifndef TA_SERIAL_GROUPS
#define TA_SERIAL_GROUPS 0
#endif

static int kwidth(int32_t k) {
    int K = 1;
    while (K < k) K <<= 1;
    return K;
}

static int solve_batched(const BatchPlan &P, const int32_t *nrhs, const double *const *B,
                         double *const *Xo, const ta_opts *o, int32_t minnorm, ta_info *info,
                         hipStream_t s) {
    if (nrhs == nullptr || B == nullptr || Xo == nullptr || o == nullptr || info == nullptr)
        return TA_EINVAL;
    if (!(o->tol >= 0.0 && o->tol < 1.0) || !(o->tol_normal >= 0.0 && o->tol_normal < 1.0))
        return TA_EINVAL;
    if (o->t < 1 || o->t > kTMax || o->max_iter < 0 || o->chunk < 0) return TA_EINVAL;
    if (o->launch_mode != 0 && o->launch_mode != 1) return TA_EINVAL;
    if (o->nonneg != 0 || o->rho_max != 0.0 || o->normal_eq != 0) return TA_EINVAL;
    if (o->enhanced != 0 && o->enhanced != 1) return TA_EINVAL;
    if (!(o->accel >= 0.0 && o->accel < 1.0)) return TA_EINVAL;
    if (o->t_cycle != 0 && o->t_cycle != 1) return TA_EINVAL;
    if (o->h_mode != 0 && o->h_mode != 1) return TA_EINVAL;
    if (o->h_mode == 1) {
        // H = A: the x-form on square systems (symmetric positive semidefinite,
        // not checked); dense batches take it in FP64 only (on their CSR copy)
        if (minnorm || (P.dense && o->precision != TA_FP64)) return TA_EINVAL;
        for (int32_t i = 0; i < P.nsys; ++i)
            if (!P.square[i]) return TA_EINVAL;
    }
    if (minnorm && o->warm_start) return TA_EINVAL;
    if (o->precision != TA_FP64 && o->precision != P.precision) return TA_EINVAL;
    if (P.dense && o->precision == TA_FP64 && P.csr64)
        return solve_batched(*P.csr64, nrhs, B, Xo, o, minnorm, info, s);
    int32_t kmax = 0;
    for (int32_t i = 0; i < P.nsys; ++i) {
        if (nrhs[i] < 0 || nrhs[i] > kMaxK) return TA_EINVAL;
        const int64_t m = P.ro[i + 1] - P.ro[i];
        if (m > 0 && o->t > m) return TA_EINVAL;
        if (nrhs[i] > 0 && ((m > 0 && B[i] == nullptr) ||
                            (P.co[i + 1] - P.co[i] > 0 && Xo[i] == nullptr)))
            return TA_EINVAL;
        kmax = std::max(kmax, nrhs[i]);
    }
    if (kmax == 0) return TA_OK;
    // Systems are run in groups of equal vector width K (a power of two), so
    // that a system with few right-hand sides does not stream K - k padding
    // columns.  A system's k columns are cut into at most two pieces: the
    // widest power of two K1 <= k, and the rest k - K1 in the group of the
    // power of two covering it, when that is narrower than K1 (40 = 32 + 8,
    // 44 = 32 + 12 -> 16 wide; 56 stays one piece of 64).  Padding is then
    // below a quarter of the columns instead of up to half; the price is one
    // more pass over the system's matrix per product, cheap beside the vector
    // blocks at these widths.  Columns are
    // contiguous in the column-major B and X, so a piece is a pointer offset.
    // The groups (and their parts, below) run side by side, each on its own
    // host thread and stream, after everything queued on s.
    std::vector<int64_t> off(P.nsys);
    int64_t acc = 0;
    for (int32_t i = 0; i < P.nsys; ++i) {
        off[i] = acc;
        acc += nrhs[i];
    }
    struct Piece {
        int32_t c0 = 0, k = 0;  // first column and width of the system's piece in a group
    };
    // pieces[K][s]
    std::vector<std::vector<Piece>> pieces(8, std::vector<Piece>(P.nsys));
    auto log2i = [](int K) {
        int l = 0;
        while ((1 << l) < K) ++l;
        return l;
    };
    for (int32_t i = 0; i < P.nsys; ++i) {
        const int32_t k = nrhs[i];
        if (k <= 0) continue;
        int32_t K1 = 1;
        while (2 * K1 <= k) K1 <<= 1;
        // a rest wider than K1 / 2 pads to K1 itself: then one piece of 2 K1
        if (K1 == k || !kSplitColumns || kwidth(k - K1) == K1) {
            pieces[log2i(kwidth(k))][i] = Piece{0, k};
        } else {
            pieces[log2i(K1)][i] = Piece{0, K1};
            pieces[log2i(kwidth(k - K1))][i] = Piece{K1, k - K1};
        }
    }
    struct GroupArgs {
        int K;
        std::vector<int32_t> nrhs;
        std::vector<const double *> B;
        std::vector<double *> X;
        std::vector<int64_t> off;
    };
    std::vector<GroupArgs> groups;
    auto add_group = [&](int K, const std::vector<Piece> &pc, const std::vector<uint8_t> &take) {
        GroupArgs ga;
        ga.K = K;
        ga.nrhs.assign(P.nsys, 0);
        ga.B.assign(P.nsys, nullptr);
        ga.X.assign(P.nsys, nullptr);
        ga.off.assign(P.nsys, 0);
        for (int32_t i = 0; i < P.nsys; ++i) {
            if (!take[i] || pc[i].k == 0) continue;
            const int64_t m = P.ro[i + 1] - P.ro[i], n = P.co[i + 1] - P.co[i];
            ga.nrhs[i] = pc[i].k;
            ga.B[i] = B[i] + (int64_t)pc[i].c0 * m;
            ga.X[i] = Xo[i] + (int64_t)pc[i].c0 * n;
            ga.off[i] = off[i] + pc[i].c0;
        }
        groups.push_back(std::move(ga));
    };
    for (int l = 0; (1 << l) <= kwidth(kmax); ++l) {
        const int K = 1 << l;
        const std::vector<Piece> &pc = pieces[l];
        bool any = false;
        for (int32_t i = 0; i < P.nsys; ++i) any = any || pc[i].k > 0;
        if (!any) continue;
        // low-precision chains: each group split once more by row length,
        // systems whose rows fit one round of the SpMM's gathers (at most
        // kRoundNnz nonzeros per row on average) and the rest.  The parts
        // iterate independently, so short-row systems (stencils:
        // latency-bound passes) overlap long-row ones (gather-bound) and
        // neither waits for the other's iteration count.  (The FP64 chain,
        // 4 nonzeros per round, measured slower split this way.)
        if (o->precision == TA_FP64) {
            add_group(K, pc, std::vector<uint8_t>(P.nsys, 1));
            continue;
        }
        std::vector<uint8_t> ta(P.nsys, 0), tb(P.nsys, 0);
        bool ha = false, hb = false;
        for (int32_t i = 0; i < P.nsys; ++i) {
            if (pc[i].k == 0) continue;
            const int64_t rows = P.ro[i + 1] - P.ro[i];
            const int64_t nz = P.dense ? rows * (P.co[i + 1] - P.co[i])
                                       : (int64_t)P.h_arp[P.ro[i + 1]] - P.h_arp[P.ro[i]];
            if (nz <= kRoundNnz * rows) {
                ta[i] = 1;
                ha = true;
            } else {
                tb[i] = 1;
                hb = true;
            }
        }
        if (ha) add_group(K, pc, ta);
        if (hb) add_group(K, pc, tb);
    }
    auto run_group = [&](size_t j, hipStream_t gsm, GroupSync *g) -> int {
        const GroupArgs &ga = groups[j];
        switch (o->precision) {
            case TA_FP32:
                return run_k<float, float>(ga.K, P, ga.nrhs.data(), ga.B.data(), ga.X.data(), o,
                                           minnorm, info, ga.off.data(), gsm, g);
            case TA_BF16:
                return run_k<uint16_t, float>(ga.K, P, ga.nrhs.data(), ga.B.data(), ga.X.data(),
                                              o, minnorm, info, ga.off.data(), gsm, g);
            default:
                return run_k<double, double>(ga.K, P, ga.nrhs.data(), ga.B.data(), ga.X.data(),
                                             o, minnorm, info, ga.off.data(), gsm, g);
        }
    };
    const size_t ng = groups.size();
    if (ng == 1) return run_group(0, s, nullptr);
#if TA_SERIAL_GROUPS
    // measurement build: the groups one after another on s
    for (size_t j = 0; j < ng; ++j) {
        const int rc = run_group(j, s, nullptr);
        if (rc != TA_OK) return rc;
    }
    return TA_OK;
#endif
    struct Streams {
        std::vector<hipStream_t> v;
        hipEvent_t ev = nullptr;
        ~Streams() {
            for (hipStream_t x : v) (void)hipStreamDestroy(x);
            if (ev != nullptr) (void)hipEventDestroy(ev);
        }
    } st;
    HIP_TRY(hipEventCreateWithFlags(&st.ev, hipEventDisableTiming));
    HIP_TRY(hipEventRecord(st.ev, s));
    for (size_t j = 0; j < ng; ++j) {
        hipStream_t x = nullptr;
        HIP_TRY(hipStreamCreateWithFlags(&x, hipStreamNonBlocking));
        st.v.push_back(x);
        HIP_TRY(hipStreamWaitEvent(x, st.ev, 0));
    }
    int dev = 0;  // the caller's device, made current on every group thread
    HIP_TRY(hipGetDevice(&dev));
    GroupSync g;
    g.pending = (int)ng;
    std::vector<int> rcs(ng, TA_OK);
    std::vector<std::string> msgs(ng);
    std::vector<std::thread> th;
    th.reserve(ng);
    size_t started = 0;
    try {
        for (; started < ng; ++started) {
            const size_t j = started;
            th.emplace_back([&, j] {
                const hipError_t e = hipSetDevice(dev);
                rcs[j] = e == hipSuccess ? run_group(j, st.v[j], &g) : hip_fail(e, "hipSetDevice");
                if (e != hipSuccess) g.arrive();
                msgs[j] = hip_msg();
            });
        }
    } catch (...) {
        // groups that never started still count at the barrier
        for (size_t j = started; j < ng; ++j) {
            rcs[j] = TA_ENOMEM;
            msgs[j] = "could not start a host thread";
            g.arrive();
        }
    }
    for (auto &x : th) x.join();
    for (size_t j = 0; j < ng; ++j)
        if (rcs[j] != TA_OK) {
            hip_msg() = msgs[j];
            return rcs[j];
        }
    return TA_OK;
}

// Timing hook: `reps` launches of the SpMM kernel a batched solve with K
// columns uses on A (trans = 0) or A^T (trans = 1), back to back between two
// HIP events on `s`; returns the average milliseconds per launch.
template <typename V, typename X, int K>
static int time_spmm_k(const BatchPlan &P, int32_t trans, int32_t reps, double *avg_ms,
                       hipStream_t s) {
    const bool mixed = !std::is_same<V, double>::value;
    const int64_t rows = trans ? P.N : P.M, cols = trans ? P.M : P.N;
    std::vector<BRange> tab;
    std::vector<int32_t> first;
    if (P.dense)
        make_dense_blocks(trans ? P.co : P.ro, tab, first);
    else
        make_blocks(trans ? P.co : P.ro, trans ? P.h_trp : P.h_arp, K, tab, first, nullptr,
                    P.square.data());
    const int32_t nb = (int32_t)tab.size();
    int L = pick_row_lanes(P.nnz, rows, Lanes<X, K>::KL);
    Workspace ws(s);
    X *xin = nullptr, *yout = nullptr;
    double2 *partials = nullptr;
    BRange *d_tab = nullptr;
    Groups gs{};
    ws.reserve(&xin, std::max<int64_t>(cols, 1) * K);
    ws.reserve(&yout, std::max<int64_t>(rows, 1) * K);
    ws.reserve(&partials, (int64_t)K * std::max(nb, 1));
    ws.reserve(&d_tab, std::max(nb, 1));
    ws.reserve(&gs.flags, 4);
    ws.reserve(&gs.sys_active, P.nsys);
    double *DS = nullptr;
    if (P.dense)
        ws.reserve(&DS, dense_xt_doubles(P, K) +
                            (int64_t)dense_nseg(std::max(nb, 1)) * std::max<int64_t>(rows, 1) * K);
    int rc = ws.commit();
    if (rc != TA_OK) return rc;
    HIP_TRY(hipMemcpyAsync(d_tab, tab.data(), sizeof(BRange) * nb, hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemsetAsync(xin, 0, sizeof(X) * (size_t)(std::max<int64_t>(cols, 1) * K), s));
    HIP_TRY(hipMemsetAsync(gs.flags, 0, sizeof(int32_t) * 4, s));
    gs.nsys = P.nsys;
    gs.K = K;
    if (mixed && (P.dense ? P.d_low : P.a_low) == nullptr) return TA_EINVAL;
    const int64_t cap = std::max(nb, 1);
    const int32_t short_rows = P.nnz <= kRoundNnz * rows ? 1 : 0;
    if (mixed && (rc = tuned_lanes<V, X, K>(P, trans, d_tab, nb, xin, yout, gs, partials, cap, L,
                                            &L, s, short_rows)) != TA_OK)
        return rc;
    prod<V, X, K, kBNorm>(P, trans, xin, yout, nullptr, d_tab, nb, gs, partials, cap, 0, kBAlways,
                          L, s, DS);
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    HIP_TRY(hipEventRecord(e0, s));
    for (int32_t i = 0; i < reps; ++i)
        prod<V, X, K, kBNorm>(P, trans, xin, yout, nullptr, d_tab, nb, gs, partials, cap, 0,
                              kBAlways, L, s, DS);
    HIP_TRY(hipEventRecord(e1, s));
    HIP_TRY(hipEventSynchronize(e1));
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    *avg_ms = (double)ms / reps;
    return TA_OK;
}

template <typename V, typename X>
static int time_spmm(const BatchPlan &P, int32_t K, int32_t trans, int32_t reps, double *avg_ms,
                     hipStream_t s) {
    switch (K) {
        case 1: return time_spmm_k<V, X, 1>(P, trans, reps, avg_ms, s);
        case 2: return time_spmm_k<V, X, 2>(P, trans, reps, avg_ms, s);
        case 4: return time_spmm_k<V, X, 4>(P, trans, reps, avg_ms, s);
        case 8: return time_spmm_k<V, X, 8>(P, trans, reps, avg_ms, s);
        case 16: return time_spmm_k<V, X, 16>(P, trans, reps, avg_ms, s);
        case 32: return time_spmm_k<V, X, 32>(P, trans, reps, avg_ms, s);
        case 64: return time_spmm_k<V, X, 64>(P, trans, reps, avg_ms, s);
        default: return TA_EINVAL;
    }
}

}  // namespace bt
}  // namespace ta

struct ta_batch_plan {
    ta::bt::BatchPlan p;
};

extern "C" {

int ta_batch_plan_create(int32_t nsys, const ta_mat *A, int32_t precision, ta_batch_plan **plan,
                         void *stream) {
    if (plan == nullptr) return TA_EINVAL;
    *plan = nullptr;
    ta_batch_plan *p = new (std::nothrow) ta_batch_plan;
    if (p == nullptr) return TA_ENOMEM;
    const int rc = ta::bt::bplan_build(nsys, A, precision, (hipStream_t)stream, &p->p);
    if (rc != TA_OK) {
        ta::bt::bplan_free(&p->p);
        delete p;
        return rc;
    }
    *plan = p;
    return TA_OK;
}

int ta_batch_plan_destroy(ta_batch_plan *plan) {
    if (plan == nullptr) return TA_OK;
    ta::bt::bplan_free(&plan->p);
    delete plan;
    return TA_OK;
}

int ta_batch_time_spmm(const ta_batch_plan *plan, int32_t K, int32_t trans, int32_t precision,
                       int32_t reps, double *avg_ms, void *stream) {
    if (plan == nullptr || avg_ms == nullptr || reps < 1) return TA_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    const ta::bt::BatchPlan &P0 = plan->p;
    if (precision != TA_FP64 && precision != P0.precision) return TA_EINVAL;
    // FP64 on a dense plan: the kernel its solves run, on the CSR copy
    const ta::bt::BatchPlan &P = (P0.dense && precision == TA_FP64 && P0.csr64) ? *P0.csr64 : P0;
    switch (precision) {
        case TA_FP32: return ta::bt::time_spmm<float, float>(P, K, trans, reps, avg_ms, s);
        case TA_BF16: return ta::bt::time_spmm<uint16_t, float>(P, K, trans, reps, avg_ms, s);
        default: return ta::bt::time_spmm<double, double>(P, K, trans, reps, avg_ms, s);
    }
}

int cta_solve_batched(const ta_batch_plan *plan, const int32_t *nrhs, const double *const *B,
                      double *const *X, const ta_opts *opts, int32_t minnorm, ta_info *info,
                      void *stream) {
    if (plan == nullptr) return TA_EINVAL;
    return ta::bt::solve_batched(plan->p, nrhs, B, X, opts, minnorm ? 1 : 0, info,
                                 (hipStream_t)stream);
}

}  // extern "C"
