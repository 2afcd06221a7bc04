// Host-side helpers shared by the drivers of libta: HIP error handling,
// stream-ordered workspace, descriptor checks.
#pragma once

#include <hip/hip_runtime.h>
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
    // hand the allocation to the caller (it is not freed by the destructor)
    void *release() {
        void *b = base_;
        base_ = nullptr;
        return b;
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

}  // namespace ta
