// Host-side helpers shared by the drivers of libta: HIP error handling,
// stream-ordered workspace, descriptor checks, trace ranges.
#pragma once

#include <hip/hip_runtime.h>
#include <rocprofiler-sdk-roctx/roctx.h>
#include <stdint.h>
#include <stdio.h>

#include <algorithm>
#include <string>
#include <vector>

#include "common.hpp"

namespace ta {

// Text of the last HIP failure on this host thread (for ta_strerror).
inline std::string &hip_msg() {
    static thread_local std::string msg;
    return msg;
}

inline int hip_fail(hipError_t e, const char *what) {
    char buf[256];
    snprintf(buf, sizeof buf, "%s: %s", what, hipGetErrorString(e));
    hip_msg() = buf;
    return e == hipErrorOutOfMemory ? TA_ENOMEM : TA_EHIP;
}

// A roctx range over a host-side phase (plan preparation, one chunk of
// iterations and its state read-back): rocprofv3 --marker-trace shows them
// beside the kernels.  Without a profiler attached the calls do nothing.
class Range {
   public:
    explicit Range(const char *name) { roctxRangePushA(name); }
    ~Range() { roctxRangePop(); }
    Range(const Range &) = delete;
    Range &operator=(const Range &) = delete;
};

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
    // Carve from a caller-owned device buffer of `cap` bytes instead of
    // allocating: commit() then calls no allocator and fails with
    // TA_ESCRATCH if the pieces do not fit; nothing is freed.
    Workspace(hipStream_t s, void *ext, size_t cap) : s_(s), ext_(ext), ext_cap_(cap) {}
    ~Workspace() {
        if (base_ != nullptr && ext_ == nullptr) (void)hipFreeAsync(base_, s_);
    }
    // pieces are recorded in a fixed table (no host allocation either)
    template <class T>
    void reserve(T **slot, int64_t count) {
        if (nreq_ == kMaxReqs) {
            overflow_ = true;
            return;
        }
        reqs_[nreq_++] = {reinterpret_cast<void **>(slot),
                          (size_t)std::max<int64_t>(count, 1) * sizeof(T)};
    }
    int commit() {
        if (overflow_) return TA_EINVAL;
        size_t total = 0;
        for (int i = 0; i < nreq_; ++i) total += (reqs_[i].bytes + 255) & ~size_t(255);
        if (ext_ != nullptr) {
            if (total > ext_cap_) return TA_ESCRATCH;
            base_ = ext_;
            carve();
            return TA_OK;
        }
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
        carve();
        return TA_OK;
    }
    // hand the allocation to the caller (it is not freed by the destructor)
    void *release() {
        void *b = ext_ == nullptr ? base_ : nullptr;
        base_ = nullptr;
        return b;
    }
    bool external() const { return ext_ != nullptr; }

   private:
    void carve() {
        char *p = static_cast<char *>(base_);
        for (int i = 0; i < nreq_; ++i) {
            *reqs_[i].slot = p;
            p += (reqs_[i].bytes + 255) & ~size_t(255);
        }
    }
    struct Req {
        void **slot;
        size_t bytes;
    };
    static constexpr int kMaxReqs = 64;
    hipStream_t s_;
    void *base_ = nullptr;
    void *ext_ = nullptr;
    size_t ext_cap_ = 0;
    Req reqs_[kMaxReqs];
    int nreq_ = 0;
    bool overflow_ = false;
};

inline int validate_mat(const ta_mat *A) {
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

// Checks the CSR arrays on the device before any kernel indexes through them.
inline int check_csr_device(const ta_mat *A, int32_t *dflag, hipStream_t s) {
    HIP_TRY(hipMemsetAsync(dflag, 0, sizeof(int32_t), s));
    HIP_TRY(launch_check_csr(A->m, A->n, A->nnz, A->row_ptr, A->col_idx, dflag, s));
    int32_t h = 0;
    HIP_TRY(hipMemcpyAsync(&h, dflag, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    return h ? TA_EINVAL : TA_OK;
}

// check_csr_device, also returning the longest row (dflag: 2 entries)
inline int check_csr_longest(const ta_mat *A, int32_t *dflag, int64_t *longest, hipStream_t s) {
    HIP_TRY(hipMemsetAsync(dflag, 0, 2 * sizeof(int32_t), s));
    HIP_TRY(launch_check_csr(A->m, A->n, A->nnz, A->row_ptr, A->col_idx, dflag, s));
    HIP_TRY(launch_row_max(A->m, A->row_ptr, dflag + 1, s));
    int32_t h[2] = {0, 0};
    HIP_TRY(hipMemcpyAsync(h, dflag, sizeof(h), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    *longest = h[1];
    return h[0] ? TA_EINVAL : TA_OK;
}

}  // namespace ta
