// Host-side helpers shared by the C-ABI entry points: per-thread error text,
// argument checks and launch-error translation.
#pragma once

#include <hip/hip_runtime.h>
#include <stdarg.h>
#include <stdint.h>
#include <stdio.h>

#include "../../include/pvjp.h"

namespace pvjp {

void set_error(const char* fmt, ...);
void clear_error();

#define PVJP_REQUIRE(cond, ...)                \
    do {                                       \
        if (!(cond)) {                         \
            ::pvjp::set_error(__VA_ARGS__);    \
            return PVJP_EINVAL;                \
        }                                      \
    } while (0)

#define PVJP_LAUNCHED(name)                                                          \
    do {                                                                             \
        hipError_t e_ = hipGetLastError();                                           \
        if (e_ != hipSuccess) {                                                      \
            ::pvjp::set_error("%s: launch failed: %s", name, hipGetErrorString(e_)); \
            return PVJP_EDEVICE;                                                     \
        }                                                                            \
    } while (0)

inline hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

inline bool valid_dtype(pvjp_dtype d) { return d == PVJP_F32 || d == PVJP_F64; }
inline bool valid_op(pvjp_op o) { return o >= PVJP_ADD && o <= PVJP_MAX; }
inline size_t dsize(pvjp_dtype d) { return d == PVJP_F64 ? 8 : 4; }

inline bool aligned(const void* p, size_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }

// Grid size for flat elementwise kernels: enough blocks to fill 256 CUs
// several times over, each thread handling a strided range.
inline unsigned flat_grid(int64_t n, int block, int per_thread) {
    int64_t g = ceil_div(n, (int64_t)block * per_thread);
    if (g < 1) g = 1;
    if (g > 65536) g = 65536;
    return (unsigned)g;
}

}  // namespace pvjp
