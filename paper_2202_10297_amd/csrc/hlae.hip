// reduce_by_index with the log-add-exp operator (Sec. 5.1.2, with the general
// rule of Sec. 5.1.1 inside each bin): hs[b] = log sum over the elements of
// bin b of e^(x_i).  The operator commutes, so ls_i (.) x_i (.) rs_i is the
// bin's total whatever the order of the bin's elements, and the general rule
// gives element i the adjoint hs_bar[b] e^(x_i - hs[b]): one pass, no sort.
// The primal: for FP32 with bins beyond one block's LDS, one pass of the
// bucket partition whose work items take each bin's maximum and then the
// sum of e^(x - maximum) over the same records (FP64), merged per bin by
// rescaling; otherwise this library's reduce_by_index paths in turn: the bin
// maxima (max), the shifted exponentials summed per bin (+, FP64 sums), and
// hs = max + log(sum).  Over the extended reals -inf is the neutral element:
// an empty bin, or one of -inf elements only, gets -inf and a -inf element
// gets adjoint 0.  An element equal to its bin's maximum contributes e^0 = 1
// (also when both are +inf), so a bin holding +inf gets +inf and a NaN
// element makes its bin NaN.  An element equal to a +inf total gets the whole
// hs_bar (the limit of the softmax weight of a unique +inf); several +inf
// elements of one bin each get it.  Indices outside [0, m) are skipped.
#include "common.h"
#include "hpart.h"

namespace pvjp {

__device__ __forceinline__ float hl_exp(float x) { return expf(x); }
__device__ __forceinline__ double hl_exp(double x) { return exp(x); }
__device__ __forceinline__ float hl_log(float x) { return logf(x); }
__device__ __forceinline__ double hl_log(double x) { return log(x); }

// Elements per thread per step (their loads and bin gathers in flight
// together); the per-element streams go non-temporal so that they do not
// push the gathered bin lines out of L2.
constexpr int kHlU = 4;

template <class T>
__global__ __launch_bounds__(256) void hl_shift_kernel(const int32_t* __restrict__ inds, const T* __restrict__ x,
                                                       int64_t n, int64_t m, const T* __restrict__ hmax,
                                                       T* __restrict__ e) {
    const int64_t step = (int64_t)gridDim.x * blockDim.x * kHlU;
    for (int64_t base = (int64_t)blockIdx.x * blockDim.x * kHlU + threadIdx.x; base < n; base += step) {
        int32_t k[kHlU];
        T xi[kHlU], mx[kHlU];
#pragma unroll
        for (int u = 0; u < kHlU; ++u) {
            const int64_t i = base + (int64_t)u * blockDim.x;
            k[u] = i < n ? __builtin_nontemporal_load(inds + i) : -1;
            xi[u] = i < n ? __builtin_nontemporal_load(x + i) : T(0);
        }
#pragma unroll
        for (int u = 0; u < kHlU; ++u) mx[u] = (k[u] >= 0 && k[u] < m) ? hmax[k[u]] : -(T)INFINITY;
#pragma unroll
        for (int u = 0; u < kHlU; ++u) {
            const int64_t i = base + (int64_t)u * blockDim.x;
            if (i < n) {
                const bool live = xi[u] != -(T)INFINITY && mx[u] != -(T)INFINITY;
                const T v = xi[u] == mx[u] ? T(1) : hl_exp(xi[u] - mx[u]);
                __builtin_nontemporal_store(live ? v : T(0), e + i);
            }
        }
    }
}

template <class T>
__global__ __launch_bounds__(256) void hl_final_kernel(const T* __restrict__ hmax, const T* __restrict__ hsum,
                                                       int64_t m, T* __restrict__ hs) {
    for (int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; b < m; b += (int64_t)gridDim.x * blockDim.x)
        hs[b] = hsum[b] == T(0) ? -(T)INFINITY : hmax[b] + hl_log(hsum[b]);  // NaN sums stay NaN
}

template <class T, bool ACC>
__global__ __launch_bounds__(256) void hl_vjp_kernel(const int32_t* __restrict__ inds, const T* __restrict__ x,
                                                     int64_t n, int64_t m, const T* __restrict__ hs,
                                                     const T* __restrict__ hb, T* __restrict__ xb) {
    const int64_t step = (int64_t)gridDim.x * blockDim.x * kHlU;
    for (int64_t base = (int64_t)blockIdx.x * blockDim.x * kHlU + threadIdx.x; base < n; base += step) {
        int32_t k[kHlU];
        T xi[kHlU], h[kHlU], g[kHlU];
#pragma unroll
        for (int u = 0; u < kHlU; ++u) {
            const int64_t i = base + (int64_t)u * blockDim.x;
            k[u] = i < n ? __builtin_nontemporal_load(inds + i) : -1;
            xi[u] = i < n ? __builtin_nontemporal_load(x + i) : T(0);
        }
#pragma unroll
        for (int u = 0; u < kHlU; ++u) {
            const bool in = k[u] >= 0 && k[u] < m;
            h[u] = in ? hs[k[u]] : -(T)INFINITY;
            g[u] = in ? hb[k[u]] : T(0);
        }
#pragma unroll
        for (int u = 0; u < kHlU; ++u) {
            const int64_t i = base + (int64_t)u * blockDim.x;
            if (i < n) {
                const bool live = xi[u] != -(T)INFINITY && h[u] != -(T)INFINITY;
                const T v = live ? g[u] * (xi[u] == h[u] ? T(1) : hl_exp(xi[u] - h[u])) : T(0);
                if (ACC) xb[i] = xb[i] + v;
                else __builtin_nontemporal_store(v, xb + i);
            }
        }
    }
}

struct HlPlan {
    size_t winner, hmax, e, hsum, hist, hist_bytes, total;
};

static HlPlan hl_plan(pvjp_dtype dtype, int64_t n, int64_t m) {
    HlPlan p{};
    const size_t es = dsize(dtype);
    size_t o = 0;
    auto take = [&](size_t b) {
        const size_t at = o;
        o += align_up(b > 0 ? b : 1, 256);
        return at;
    };
    p.winner = take((size_t)m * 4);
    p.hmax = take((size_t)m * es);
    p.e = take((size_t)(n > 0 ? n : 1) * es);
    p.hsum = take((size_t)m * es);
    const size_t a = pvjp_hist_ws_bytes(PVJP_MAX, dtype, n, m), b = pvjp_hist_ws_bytes(PVJP_ADD, dtype, n, m);
    p.hist_bytes = align_up(a > b ? a : b, 256);
    p.hist = take(p.hist_bytes);
    p.total = o;
    return p;
}

template <class T>
static pvjp_status hl_primal(pvjp_dtype dtype, const int32_t* inds, const T* x, int64_t n, int64_t m, T* hs,
                             char* w, const HlPlan& p, hipStream_t st) {
    if constexpr (sizeof(T) == 4) {
        if (hist_lae_partition_ok(dtype, m)) {
            // one partition, the maximum and the scaled sum per work item
            hist_lae_partitioned(inds, (const float*)x, n, (int32_t)m, (float*)hs, w + p.hist, st);
            return PVJP_OK;
        }
    }
    T* hmax = (T*)(w + p.hmax);
    T* e = (T*)(w + p.e);
    T* hsum = (T*)(w + p.hsum);
    if (pvjp_status s = pvjp_hist(PVJP_MAX, dtype, inds, x, n, m, hmax, (int32_t*)(w + p.winner), nullptr, nullptr,
                                  nullptr, w + p.hist, p.hist_bytes, st))
        return s;
    if (n > 0)
        hipLaunchKernelGGL(hl_shift_kernel<T>, dim3(flat_grid(n, 256, 4)), dim3(256), 0, st, inds, x, n, m,
                           (const T*)hmax, e);
    if (pvjp_status s = pvjp_hist(PVJP_ADD, dtype, inds, e, n, m, hsum, nullptr, nullptr, nullptr, nullptr,
                                  w + p.hist, p.hist_bytes, st))
        return s;
    hipLaunchKernelGGL(hl_final_kernel<T>, dim3(flat_grid(m, 256, 4)), dim3(256), 0, st, (const T*)hmax,
                       (const T*)hsum, m, hs);
    return PVJP_OK;
}

}  // namespace pvjp

using namespace pvjp;

extern "C" size_t pvjp_hist_lae_ws_bytes(pvjp_dtype dtype, int64_t n, int64_t m) {
    if (!valid_dtype(dtype) || n < 0 || m < 1) return 0;
    return hl_plan(dtype, n, m).total;
}

extern "C" pvjp_status pvjp_hist_lae(pvjp_dtype dtype, const int32_t* inds, const void* x, int64_t n, int64_t m,
                                     void* hs, void* ws, size_t ws_bytes, void* stream) {
    clear_error();
    PVJP_REQUIRE(valid_dtype(dtype), "pvjp_hist_lae: unknown dtype %d", (int)dtype);
    PVJP_REQUIRE(n >= 0 && n < INT32_MAX && m >= 1 && m <= ((int64_t)1 << 30),
                 "pvjp_hist_lae: n = %lld, m = %lld out of range", (long long)n, (long long)m);
    PVJP_REQUIRE(hs != nullptr && (n == 0 || (inds != nullptr && x != nullptr)),
                 "pvjp_hist_lae: hs, inds and x must be non-NULL");
    PVJP_REQUIRE(ws != nullptr && aligned(ws, 256), "pvjp_hist_lae: ws must be non-NULL and 256-byte aligned");
    const HlPlan p = hl_plan(dtype, n, m);
    if (ws_bytes < p.total) {
        set_error("pvjp_hist_lae: workspace has %zu bytes, needs %zu", ws_bytes, p.total);
        return PVJP_ENOMEM;
    }
    char* w = reinterpret_cast<char*>(ws);
    hipStream_t st = as_stream(stream);
    const pvjp_status s = dtype == PVJP_F64
                              ? hl_primal<double>(dtype, inds, (const double*)x, n, m, (double*)hs, w, p, st)
                              : hl_primal<float>(dtype, inds, (const float*)x, n, m, (float*)hs, w, p, st);
    if (s != PVJP_OK) return s;
    PVJP_LAUNCHED("pvjp_hist_lae");
    return PVJP_OK;
}

extern "C" pvjp_status pvjp_hist_lae_vjp(pvjp_dtype dtype, const int32_t* inds, const void* x, int64_t n, int64_t m,
                                         const void* hs, const void* hs_bar, void* x_bar, int accumulate,
                                         void* stream) {
    clear_error();
    PVJP_REQUIRE(valid_dtype(dtype), "pvjp_hist_lae_vjp: unknown dtype %d", (int)dtype);
    PVJP_REQUIRE(n >= 0 && n < INT32_MAX && m >= 1 && m <= ((int64_t)1 << 30),
                 "pvjp_hist_lae_vjp: n = %lld, m = %lld out of range", (long long)n, (long long)m);
    if (n == 0) return PVJP_OK;
    PVJP_REQUIRE(inds != nullptr && x != nullptr && hs != nullptr && hs_bar != nullptr && x_bar != nullptr,
                 "pvjp_hist_lae_vjp: inds, x, hs, hs_bar and x_bar must be non-NULL");
    hipStream_t st = as_stream(stream);
    const dim3 g(flat_grid(n, 256, 4)), b(256);
    if (dtype == PVJP_F64) {
        if (accumulate)
            hipLaunchKernelGGL((hl_vjp_kernel<double, true>), g, b, 0, st, inds, (const double*)x, n, m,
                               (const double*)hs, (const double*)hs_bar, (double*)x_bar);
        else
            hipLaunchKernelGGL((hl_vjp_kernel<double, false>), g, b, 0, st, inds, (const double*)x, n, m,
                               (const double*)hs, (const double*)hs_bar, (double*)x_bar);
    } else {
        if (accumulate)
            hipLaunchKernelGGL((hl_vjp_kernel<float, true>), g, b, 0, st, inds, (const float*)x, n, m,
                               (const float*)hs, (const float*)hs_bar, (float*)x_bar);
        else
            hipLaunchKernelGGL((hl_vjp_kernel<float, false>), g, b, 0, st, inds, (const float*)x, n, m,
                               (const float*)hs, (const float*)hs_bar, (float*)x_bar);
    }
    PVJP_LAUNCHED("pvjp_hist_lae_vjp");
    return PVJP_OK;
}
