// lm_host.h -- host-side helpers shared by the C ABI implementation files (lm_api.hip,
// lm_batch.hip): error reporting, stream-ordered workspace, argument checks.  Not part of the
// public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <string>
#include <vector>

#include "lm_internal.h"

namespace lmh {

// Sets the calling thread's last-error text (read by lm_last_error) and returns st.
lm_status fail(lm_status st, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
lm_status fail_hip(hipError_t e, const char* what);
const char* last_error();

#define LM_HIP(expr)                                                  \
    do {                                                              \
        hipError_t e_ = (expr);                                       \
        if (e_ != hipSuccess) return lmh::fail_hip(e_, #expr);        \
    } while (0)

#define LM_TRY(expr)                                                  \
    do {                                                              \
        lm_status s_ = (expr);                                        \
        if (s_ != LM_OK) return s_;                                   \
    } while (0)

// Stream-ordered device allocations released (on the same stream) when the owner dies.
class Workspace {
public:
    explicit Workspace(hipStream_t st) : st_(st) {}
    ~Workspace()
    {
        for (void* p : ptrs_) (void)hipFreeAsync(p, st_);
    }
    Workspace(const Workspace&) = delete;
    Workspace& operator=(const Workspace&) = delete;

    template <class T>
    lm_status get(T** out, int64_t count)
    {
        void* p = nullptr;
        size_t bytes = (size_t)(count > 0 ? count : 1) * sizeof(T);
        hipError_t e = hipMallocAsync(&p, bytes, st_);
        if (e != hipSuccess) return fail_hip(e, "hipMallocAsync");
        ptrs_.push_back(p);
        *out = (T*)p;
        return LM_OK;
    }

private:
    hipStream_t st_;
    std::vector<void*> ptrs_;
};

inline bool is_finite(double x) { return std::isfinite(x); }

// Four HIP events for phase timings, destroyed with the owner.
struct EventTimer {
    hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
    lm_status init()
    {
        for (auto& e : ev) {
            hipError_t err = hipEventCreate(&e);
            if (err != hipSuccess) return fail_hip(err, "hipEventCreate");
        }
        return LM_OK;
    }
    double ms(int a, int b) const
    {
        float t = 0.0f;
        return hipEventElapsedTime(&t, ev[a], ev[b]) == hipSuccess ? (double)t : -1.0;
    }
    ~EventTimer()
    {
        for (auto& e : ev)
            if (e) (void)hipEventDestroy(e);
    }
};

constexpr int64_t kMaxN = (int64_t)1 << 34;

lm_status check_params(const lm_params* prm);
lm_status check_n(int64_t n, const char* name = "n");
// Exponent scale and force constant of the pair bodies.  The pair bodies evaluate the kernel
// as 2^(kq t) (t = r for the conon, r^2 for the Gaussian), so kq carries the factor log2(e).
constexpr double kLog2e = 1.4426950408889634;
void kernel_scales(const lm_params* prm, double* kq, double* wscale);

}  // namespace lmh
