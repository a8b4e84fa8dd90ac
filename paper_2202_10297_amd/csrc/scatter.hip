// Scatter and its VJP (Sec. 5.3).
//
// Forward sweep: xs_saved = gather xs is; xs[is[j]] = vs[j] (in place).
// Return sweep, fused into one pass over the m updates:
//   vs_bar[j] += ys_bar[is[j]]       (the adjoint of the scatter is a gather),
//   ys_bar[is[j]] = 0                (the overwritten elements never were in xs),
//   ys[is[j]] = xs_saved[j]          (optional: restores xs in place).
// Work is proportional to m, never to n.
#include "common.h"

namespace pvjp {

template <class T>
__global__ __launch_bounds__(256) void scatter_kernel(T* __restrict__ xs, int64_t n, const int32_t* __restrict__ is,
                                                      const T* __restrict__ vs, int64_t m, T* __restrict__ saved) {
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < m; j += (int64_t)gridDim.x * blockDim.x) {
        const int64_t k = is[j];
        if (k >= 0 && k < n) {
            if (saved) saved[j] = xs[k];
            xs[k] = vs[j];
        } else if (saved) {
            saved[j] = T(0);
        }
    }
}

template <class T, bool ACC, bool RESTORE>
__global__ __launch_bounds__(256) void scatter_vjp_kernel(T* __restrict__ ybar, int64_t n,
                                                          const int32_t* __restrict__ is, int64_t m,
                                                          T* __restrict__ vbar, T* __restrict__ ys,
                                                          const T* __restrict__ saved) {
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < m; j += (int64_t)gridDim.x * blockDim.x) {
        const int64_t k = is[j];
        T g = T(0);
        if (k >= 0 && k < n) {
            g = ybar[k];
            ybar[k] = T(0);
            if (RESTORE) ys[k] = saved[j];
        }
        vbar[j] = ACC ? vbar[j] + g : g;
    }
}

template <class T>
static void launch_vjp(void* ybar, int64_t n, const int32_t* is, int64_t m, void* vbar, int acc, void* ys,
                       const void* saved, hipStream_t st) {
    const unsigned g = flat_grid(m, 256, 4);
    T* yb = (T*)ybar;
    T* vb = (T*)vbar;
    T* y = (T*)ys;
    const T* sv = (const T*)saved;
    if (acc) {
        if (ys)
            hipLaunchKernelGGL((scatter_vjp_kernel<T, true, true>), dim3(g), dim3(256), 0, st, yb, n, is, m, vb, y, sv);
        else
            hipLaunchKernelGGL((scatter_vjp_kernel<T, true, false>), dim3(g), dim3(256), 0, st, yb, n, is, m, vb, y, sv);
    } else {
        if (ys)
            hipLaunchKernelGGL((scatter_vjp_kernel<T, false, true>), dim3(g), dim3(256), 0, st, yb, n, is, m, vb, y, sv);
        else
            hipLaunchKernelGGL((scatter_vjp_kernel<T, false, false>), dim3(g), dim3(256), 0, st, yb, n, is, m, vb, y, sv);
    }
}

}  // namespace pvjp

using namespace pvjp;

extern "C" pvjp_status pvjp_scatter(pvjp_dtype dtype, void* xs, int64_t n, const int32_t* is, const void* vs,
                                    int64_t m, void* xs_saved, void* stream) {
    clear_error();
    PVJP_REQUIRE(valid_dtype(dtype), "pvjp_scatter: unknown dtype %d", (int)dtype);
    PVJP_REQUIRE(n >= 0 && m >= 0, "pvjp_scatter: negative size");
    if (m == 0) return PVJP_OK;
    PVJP_REQUIRE(is != nullptr && vs != nullptr, "pvjp_scatter: is and vs must be non-NULL");
    PVJP_REQUIRE(n == 0 || xs != nullptr, "pvjp_scatter: xs is NULL");
    const unsigned g = flat_grid(m, 256, 4);
    if (dtype == PVJP_F64)
        hipLaunchKernelGGL(scatter_kernel<double>, dim3(g), dim3(256), 0, as_stream(stream), (double*)xs, n, is,
                           (const double*)vs, m, (double*)xs_saved);
    else
        hipLaunchKernelGGL(scatter_kernel<float>, dim3(g), dim3(256), 0, as_stream(stream), (float*)xs, n, is,
                           (const float*)vs, m, (float*)xs_saved);
    PVJP_LAUNCHED("pvjp_scatter");
    return PVJP_OK;
}

extern "C" pvjp_status pvjp_scatter_vjp(pvjp_dtype dtype, void* ys_bar, int64_t n, const int32_t* is, int64_t m,
                                        void* vs_bar, int accumulate, void* ys, const void* xs_saved, void* stream) {
    clear_error();
    PVJP_REQUIRE(valid_dtype(dtype), "pvjp_scatter_vjp: unknown dtype %d", (int)dtype);
    PVJP_REQUIRE(n >= 0 && m >= 0, "pvjp_scatter_vjp: negative size");
    if (m == 0) return PVJP_OK;
    PVJP_REQUIRE(is != nullptr && vs_bar != nullptr, "pvjp_scatter_vjp: is and vs_bar must be non-NULL");
    PVJP_REQUIRE(n == 0 || ys_bar != nullptr, "pvjp_scatter_vjp: ys_bar is NULL");
    PVJP_REQUIRE(ys == nullptr || xs_saved != nullptr, "pvjp_scatter_vjp: restoring ys needs xs_saved");
    if (dtype == PVJP_F64)
        launch_vjp<double>(ys_bar, n, is, m, vs_bar, accumulate, ys, xs_saved, as_stream(stream));
    else
        launch_vjp<float>(ys_bar, n, is, m, vs_bar, accumulate, ys, xs_saved, as_stream(stream));
    PVJP_LAUNCHED("pvjp_scatter_vjp");
    return PVJP_OK;
}

// Forward mode: ys is a copy of xs with ys[is[j]] = vs[j], so its tangent is
// x_dot with the same assignment of v_dot: the primal scatter applied to the
// tangents, in place on ys_dot (which holds x_dot on entry).
extern "C" pvjp_status pvjp_scatter_jvp(pvjp_dtype dtype, void* ys_dot, int64_t n, const int32_t* is,
                                        const void* vs_dot, int64_t m, void* stream) {
    clear_error();
    const pvjp_status s = pvjp_scatter(dtype, ys_dot, n, is, vs_dot, m, nullptr, stream);
    if (s != PVJP_OK) {
        char inner[256];
        snprintf(inner, sizeof(inner), "%s", pvjp_last_error());
        set_error("pvjp_scatter_jvp: %s", inner);
    }
    return s;
}
