// Checked mode: device-side counts of the input conditions that the method
// leaves undefined, taken without trapping.
//  - reduce_by_index (Sec. 5.1.2) defines its result only for indices inside
//    [0, m): indices outside are counted (the operators skip them).
//  - scatter (Sec. 5.3) assumes that no target index repeats: its forward
//    sweep saves each overwritten element once and its return sweep zeroes
//    each target once.  Repeats are found with a bitmap of the n targets: the
//    atomic OR that sets a target's bit returns the old word, so every
//    occurrence after the first of a target is counted exactly once.
//  - NaN and infinite values, which the FP rules carry through but which
//    usually mean that the caller's inputs are broken.
// Every count is added to a caller-owned int64 counter block on the device
// (one atomic add per block of the launch), so one block collects the counts
// of many calls until the caller reads and clears it.
#include "common.h"
#include "prims.h"

namespace pvjp {

constexpr int kDiagBlock = 256;

__device__ __forceinline__ int64_t diag_block_sum(int64_t v, int64_t* red) {
    for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o);
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    if (lane == 0) red[w] = v;
    __syncthreads();
    int64_t t = 0;
    if (threadIdx.x == 0)
        for (int i = 0; i < kDiagBlock / kWave; ++i) t += red[i];
    return t;
}

__global__ __launch_bounds__(kDiagBlock) void diag_indices_kernel(const int32_t* __restrict__ inds, int64_t n,
                                                                  int64_t m, unsigned long long* __restrict__ out) {
    __shared__ int64_t red[kDiagBlock / kWave];
    int64_t c = 0;
    for (int64_t i = (int64_t)blockIdx.x * kDiagBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kDiagBlock) {
        const int32_t k = inds[i];
        c += (k < 0 || (int64_t)k >= m) ? 1 : 0;
    }
    const int64_t t = diag_block_sum(c, red);
    if (threadIdx.x == 0 && t) atomicAdd(out, (unsigned long long)t);
}

__global__ __launch_bounds__(kDiagBlock) void diag_zero_kernel(uint32_t* __restrict__ w, int64_t nw) {
    for (int64_t i = (int64_t)blockIdx.x * kDiagBlock + threadIdx.x; i < nw; i += (int64_t)gridDim.x * kDiagBlock)
        w[i] = 0u;
}

// out[0] += out-of-range targets, out[1] += repeated targets.
__global__ __launch_bounds__(kDiagBlock) void diag_scatter_kernel(const int32_t* __restrict__ is, int64_t m, int64_t n,
                                                                  uint32_t* __restrict__ bits,
                                                                  unsigned long long* __restrict__ oob,
                                                                  unsigned long long* __restrict__ dup) {
    __shared__ int64_t red[kDiagBlock / kWave];
    int64_t co = 0, cd = 0;
    for (int64_t j = (int64_t)blockIdx.x * kDiagBlock + threadIdx.x; j < m; j += (int64_t)gridDim.x * kDiagBlock) {
        const int32_t k = is[j];
        if (k < 0 || (int64_t)k >= n) {
            ++co;
            continue;
        }
        const uint32_t bit = 1u << (k & 31);
        const uint32_t old = atomicOr(bits + (k >> 5), bit);
        cd += (old & bit) ? 1 : 0;
    }
    const int64_t to = diag_block_sum(co, red);
    __syncthreads();
    const int64_t td = diag_block_sum(cd, red);
    if (threadIdx.x == 0) {
        if (to) atomicAdd(oob, (unsigned long long)to);
        if (td) atomicAdd(dup, (unsigned long long)td);
    }
}

template <class T>
__global__ __launch_bounds__(kDiagBlock) void diag_nonfinite_kernel(const T* __restrict__ x, int64_t n,
                                                                    unsigned long long* __restrict__ nan,
                                                                    unsigned long long* __restrict__ inf) {
    __shared__ int64_t red[kDiagBlock / kWave];
    int64_t cn = 0, ci = 0;
    for (int64_t i = (int64_t)blockIdx.x * kDiagBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kDiagBlock) {
        const T v = x[i];
        cn += __builtin_isnan(v) ? 1 : 0;
        ci += __builtin_isinf(v) ? 1 : 0;
    }
    const int64_t tn = diag_block_sum(cn, red);
    __syncthreads();
    const int64_t ti = diag_block_sum(ci, red);
    if (threadIdx.x == 0) {
        if (tn) atomicAdd(nan, (unsigned long long)tn);
        if (ti) atomicAdd(inf, (unsigned long long)ti);
    }
}

}  // namespace pvjp

using namespace pvjp;

extern "C" pvjp_status pvjp_diag_indices(const int32_t* inds, int64_t n, int64_t m, int64_t* counters,
                                         void* stream) {
    clear_error();
    PVJP_REQUIRE(n >= 0 && m >= 0, "pvjp_diag_indices: n = %lld, m = %lld out of range", (long long)n, (long long)m);
    PVJP_REQUIRE(counters != nullptr && aligned(counters, 8), "pvjp_diag_indices: counters must be non-NULL, 8-byte aligned");
    if (n == 0) return PVJP_OK;
    PVJP_REQUIRE(inds != nullptr, "pvjp_diag_indices: inds is NULL");
    hipLaunchKernelGGL(diag_indices_kernel, dim3(flat_grid(n, kDiagBlock, 16)), dim3(kDiagBlock), 0,
                       as_stream(stream), inds, n, m, (unsigned long long*)counters + PVJP_DIAG_OOB);
    PVJP_LAUNCHED("pvjp_diag_indices");
    return PVJP_OK;
}

extern "C" size_t pvjp_diag_scatter_ws_bytes(int64_t n) {
    if (n < 0) return 0;
    return align_up((size_t)ceil_div(n > 0 ? n : 1, 32) * 4, 256);
}

extern "C" pvjp_status pvjp_diag_scatter(const int32_t* is, int64_t m, int64_t n, int64_t* counters, void* ws,
                                         size_t ws_bytes, void* stream) {
    clear_error();
    PVJP_REQUIRE(m >= 0 && n >= 0 && n <= INT32_MAX, "pvjp_diag_scatter: m = %lld, n = %lld out of range",
                 (long long)m, (long long)n);
    PVJP_REQUIRE(counters != nullptr && aligned(counters, 8), "pvjp_diag_scatter: counters must be non-NULL, 8-byte aligned");
    if (m == 0) return PVJP_OK;
    PVJP_REQUIRE(is != nullptr, "pvjp_diag_scatter: is is NULL");
    PVJP_REQUIRE(ws != nullptr && aligned(ws, 4), "pvjp_diag_scatter: ws must be non-NULL and 4-byte aligned");
    const size_t need = pvjp_diag_scatter_ws_bytes(n);
    if (ws_bytes < need) {
        set_error("pvjp_diag_scatter: workspace has %zu bytes, needs %zu", ws_bytes, need);
        return PVJP_ENOMEM;
    }
    hipStream_t st = as_stream(stream);
    const int64_t nw = ceil_div(n > 0 ? n : 1, 32);
    hipLaunchKernelGGL(diag_zero_kernel, dim3(flat_grid(nw, kDiagBlock, 4)), dim3(kDiagBlock), 0, st, (uint32_t*)ws,
                       nw);
    unsigned long long* c = (unsigned long long*)counters;
    hipLaunchKernelGGL(diag_scatter_kernel, dim3(flat_grid(m, kDiagBlock, 8)), dim3(kDiagBlock), 0, st, is, m, n,
                       (uint32_t*)ws, c + PVJP_DIAG_OOB, c + PVJP_DIAG_DUP);
    PVJP_LAUNCHED("pvjp_diag_scatter");
    return PVJP_OK;
}

extern "C" pvjp_status pvjp_diag_nonfinite(pvjp_dtype dtype, const void* x, int64_t n, int64_t* counters,
                                           void* stream) {
    clear_error();
    PVJP_REQUIRE(valid_dtype(dtype), "pvjp_diag_nonfinite: unknown dtype %d", (int)dtype);
    PVJP_REQUIRE(n >= 0, "pvjp_diag_nonfinite: n = %lld out of range", (long long)n);
    PVJP_REQUIRE(counters != nullptr && aligned(counters, 8), "pvjp_diag_nonfinite: counters must be non-NULL, 8-byte aligned");
    if (n == 0) return PVJP_OK;
    PVJP_REQUIRE(x != nullptr, "pvjp_diag_nonfinite: x is NULL");
    unsigned long long* c = (unsigned long long*)counters;
    const dim3 g(flat_grid(n, kDiagBlock, 16)), b(kDiagBlock);
    if (dtype == PVJP_F64)
        hipLaunchKernelGGL(diag_nonfinite_kernel<double>, g, b, 0, as_stream(stream), (const double*)x, n,
                           c + PVJP_DIAG_NAN, c + PVJP_DIAG_INF);
    else
        hipLaunchKernelGGL(diag_nonfinite_kernel<float>, g, b, 0, as_stream(stream), (const float*)x, n,
                           c + PVJP_DIAG_NAN, c + PVJP_DIAG_INF);
    PVJP_LAUNCHED("pvjp_diag_nonfinite");
    return PVJP_OK;
}
