// Shared host/device helpers of the filament library (gfx950).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

#include "fil.h"

namespace fil {

constexpr double kPi = 3.14159265358979323846;

// Thread-local description of the last error; returned by fil_last_error().
void set_error(const std::string& msg);

// Checks a HIP call; on failure records the message and returns FIL_EHIP.
#define FIL_HIP_TRY(expr)                                                                   \
    do {                                                                                    \
        hipError_t _e = (expr);                                                             \
        if (_e != hipSuccess) {                                                             \
            ::fil::set_error(std::string(#expr) + ": " + hipGetErrorString(_e));             \
            return FIL_EHIP;                                                                \
        }                                                                                   \
    } while (0)

#define FIL_CHECK_ARG(cond, msg)                                                            \
    do {                                                                                    \
        if (!(cond)) {                                                                      \
            ::fil::set_error(msg);                                                          \
            return FIL_EINVAL;                                                              \
        }                                                                                   \
    } while (0)

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// 1/sqrt(x) in double: hardware estimate plus one third-order Newton correction,
// y <- y (1 + e/2 + 3 e^2 / 8) with e = 1 - x y^2 (relative error O(e^3)).
__device__ __forceinline__ double rsqrt_f64(double x) {
    double y = __builtin_amdgcn_rsq(x);
    double e = fma(-x * y, y, 1.0);
    return fma(y * e, fma(0.375, e, 0.5), y);
}

}  // namespace fil
