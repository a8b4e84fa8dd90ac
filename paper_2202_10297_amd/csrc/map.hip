// map and its VJP (Sec. 5.4): the return sweep maps the lambda's forward
// statements followed by its reverse statements over (x, y_bar).  Primal
// intermediates (sin, exp, tanh of x) are recomputed inside the lambda rather
// than read back from memory (Sec. 4.1: recomputing scalars is far cheaper
// than a global-memory tape).
#include "common.h"

namespace pvjp {

template <class T>
__device__ __forceinline__ T dsin(T x) { return sin(x); }
template <class T>
__device__ __forceinline__ T dcos(T x) { return cos(x); }
template <class T>
__device__ __forceinline__ T dexp(T x) { return exp(x); }
template <class T>
__device__ __forceinline__ T dlog(T x) { return log(x); }
template <class T>
__device__ __forceinline__ T dtanh(T x) { return tanh(x); }

template <class T, int FN>
__device__ __forceinline__ T fn_fwd(T x) {
    switch (FN) {
        case PVJP_FN_SQUARE: return x * x;
        case PVJP_FN_EXP: return dexp(x);
        case PVJP_FN_LOG: return dlog(x);
        case PVJP_FN_SIN: return dsin(x);
        default: return dtanh(x);
    }
}

// f'(x) * y_bar with the forward statements re-executed.
template <class T, int FN>
__device__ __forceinline__ T fn_vjp(T x, T yb) {
    switch (FN) {
        case PVJP_FN_SQUARE: return (x + x) * yb;
        case PVJP_FN_EXP: return dexp(x) * yb;
        case PVJP_FN_LOG: return yb / x;
        case PVJP_FN_SIN: return dcos(x) * yb;
        default: {
            const T t = dtanh(x);
            return (T(1) - t * t) * yb;
        }
    }
}

template <class T, int FN>
__global__ __launch_bounds__(256) void map_kernel(const T* __restrict__ x, int64_t n, T* __restrict__ y) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        y[i] = fn_fwd<T, FN>(x[i]);
}

template <class T, int FN, bool ACC>
__global__ __launch_bounds__(256) void map_vjp_kernel(const T* __restrict__ x, const T* __restrict__ yb, int64_t n,
                                                      T* __restrict__ xb) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const T c = fn_vjp<T, FN>(x[i], yb[i]);
        xb[i] = ACC ? xb[i] + c : c;
    }
}

// Fig. 1: v0 = sin(x0); v1 = x1*v0; v2 = x0*x1; (y0, y1) = (v1, v2).
template <class T>
__global__ __launch_bounds__(256) void fig1_kernel(const T* __restrict__ x0, const T* __restrict__ x1, int64_t n,
                                                   T* __restrict__ y0, T* __restrict__ y1) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const T a = x0[i], b = x1[i];
        y0[i] = b * dsin(a);
        y1[i] = a * b;
    }
}

// Fig. 1(c): adjoints in reverse statement order, v0 recomputed.
template <class T, bool ACC>
__global__ __launch_bounds__(256) void fig1_vjp_kernel(const T* __restrict__ x0, const T* __restrict__ x1,
                                                       const T* __restrict__ yb0, const T* __restrict__ yb1,
                                                       int64_t n, T* __restrict__ xb0, T* __restrict__ xb1) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const T a = x0[i], b = x1[i];
        const T v0 = dsin(a);
        const T v2b = yb1[i], v1b = yb0[i];
        T a_b = b * v2b;
        T b_b = a * v2b;
        b_b += v0 * v1b;
        const T v0b = b * v1b;
        a_b += dcos(a) * v0b;
        xb0[i] = ACC ? xb0[i] + a_b : a_b;
        xb1[i] = ACC ? xb1[i] + b_b : b_b;
    }
}

template <class T, int FN>
static void launch_map(const void* x, int64_t n, void* y, hipStream_t st) {
    hipLaunchKernelGGL((map_kernel<T, FN>), dim3(flat_grid(n, 256, 8)), dim3(256), 0, st, (const T*)x, n, (T*)y);
}

template <class T, int FN>
static void launch_map_vjp(const void* x, const void* yb, int64_t n, void* xb, int acc, hipStream_t st) {
    if (acc)
        hipLaunchKernelGGL((map_vjp_kernel<T, FN, true>), dim3(flat_grid(n, 256, 8)), dim3(256), 0, st, (const T*)x,
                           (const T*)yb, n, (T*)xb);
    else
        hipLaunchKernelGGL((map_vjp_kernel<T, FN, false>), dim3(flat_grid(n, 256, 8)), dim3(256), 0, st, (const T*)x,
                           (const T*)yb, n, (T*)xb);
}

template <class T>
static void dispatch_map(pvjp_fn fn, const void* x, int64_t n, void* y, hipStream_t st) {
    switch (fn) {
        case PVJP_FN_SQUARE: launch_map<T, PVJP_FN_SQUARE>(x, n, y, st); break;
        case PVJP_FN_EXP: launch_map<T, PVJP_FN_EXP>(x, n, y, st); break;
        case PVJP_FN_LOG: launch_map<T, PVJP_FN_LOG>(x, n, y, st); break;
        case PVJP_FN_SIN: launch_map<T, PVJP_FN_SIN>(x, n, y, st); break;
        default: launch_map<T, PVJP_FN_TANH>(x, n, y, st); break;
    }
}

template <class T>
static void dispatch_map_vjp(pvjp_fn fn, const void* x, const void* yb, int64_t n, void* xb, int acc, hipStream_t st) {
    switch (fn) {
        case PVJP_FN_SQUARE: launch_map_vjp<T, PVJP_FN_SQUARE>(x, yb, n, xb, acc, st); break;
        case PVJP_FN_EXP: launch_map_vjp<T, PVJP_FN_EXP>(x, yb, n, xb, acc, st); break;
        case PVJP_FN_LOG: launch_map_vjp<T, PVJP_FN_LOG>(x, yb, n, xb, acc, st); break;
        case PVJP_FN_SIN: launch_map_vjp<T, PVJP_FN_SIN>(x, yb, n, xb, acc, st); break;
        default: launch_map_vjp<T, PVJP_FN_TANH>(x, yb, n, xb, acc, st); break;
    }
}

static bool valid_fn(pvjp_fn f) { return f >= PVJP_FN_SQUARE && f <= PVJP_FN_TANH; }

}  // namespace pvjp

using namespace pvjp;

extern "C" pvjp_status pvjp_map(pvjp_fn fn, pvjp_dtype dtype, const void* x, int64_t n, void* y, void* stream) {
    clear_error();
    PVJP_REQUIRE(valid_fn(fn), "pvjp_map: unknown fn %d", (int)fn);
    PVJP_REQUIRE(valid_dtype(dtype), "pvjp_map: unknown dtype %d", (int)dtype);
    PVJP_REQUIRE(n >= 0, "pvjp_map: negative n");
    if (n == 0) return PVJP_OK;
    PVJP_REQUIRE(x && y, "pvjp_map: x and y must be non-NULL");
    if (dtype == PVJP_F64)
        dispatch_map<double>(fn, x, n, y, as_stream(stream));
    else
        dispatch_map<float>(fn, x, n, y, as_stream(stream));
    PVJP_LAUNCHED("pvjp_map");
    return PVJP_OK;
}

extern "C" pvjp_status pvjp_map_vjp(pvjp_fn fn, pvjp_dtype dtype, const void* x, const void* y_bar, int64_t n,
                                    void* x_bar, int accumulate, void* stream) {
    clear_error();
    PVJP_REQUIRE(valid_fn(fn), "pvjp_map_vjp: unknown fn %d", (int)fn);
    PVJP_REQUIRE(valid_dtype(dtype), "pvjp_map_vjp: unknown dtype %d", (int)dtype);
    PVJP_REQUIRE(n >= 0, "pvjp_map_vjp: negative n");
    if (n == 0) return PVJP_OK;
    PVJP_REQUIRE(x && y_bar && x_bar, "pvjp_map_vjp: x, y_bar and x_bar must be non-NULL");
    if (dtype == PVJP_F64)
        dispatch_map_vjp<double>(fn, x, y_bar, n, x_bar, accumulate, as_stream(stream));
    else
        dispatch_map_vjp<float>(fn, x, y_bar, n, x_bar, accumulate, as_stream(stream));
    PVJP_LAUNCHED("pvjp_map_vjp");
    return PVJP_OK;
}

extern "C" pvjp_status pvjp_fig1(pvjp_dtype dtype, const void* x0, const void* x1, int64_t n, void* y0, void* y1,
                                 void* stream) {
    clear_error();
    PVJP_REQUIRE(valid_dtype(dtype), "pvjp_fig1: unknown dtype %d", (int)dtype);
    PVJP_REQUIRE(n >= 0, "pvjp_fig1: negative n");
    if (n == 0) return PVJP_OK;
    PVJP_REQUIRE(x0 && x1 && y0 && y1, "pvjp_fig1: pointers must be non-NULL");
    const unsigned g = flat_grid(n, 256, 8);
    if (dtype == PVJP_F64)
        hipLaunchKernelGGL(fig1_kernel<double>, dim3(g), dim3(256), 0, as_stream(stream), (const double*)x0,
                           (const double*)x1, n, (double*)y0, (double*)y1);
    else
        hipLaunchKernelGGL(fig1_kernel<float>, dim3(g), dim3(256), 0, as_stream(stream), (const float*)x0,
                           (const float*)x1, n, (float*)y0, (float*)y1);
    PVJP_LAUNCHED("pvjp_fig1");
    return PVJP_OK;
}

template <class T>
static void launch_fig1_vjp(const void* x0, const void* x1, const void* b0, const void* b1, int64_t n, void* r0,
                            void* r1, int acc, hipStream_t st) {
    const unsigned g = flat_grid(n, 256, 8);
    if (acc)
        hipLaunchKernelGGL((fig1_vjp_kernel<T, true>), dim3(g), dim3(256), 0, st, (const T*)x0, (const T*)x1,
                           (const T*)b0, (const T*)b1, n, (T*)r0, (T*)r1);
    else
        hipLaunchKernelGGL((fig1_vjp_kernel<T, false>), dim3(g), dim3(256), 0, st, (const T*)x0, (const T*)x1,
                           (const T*)b0, (const T*)b1, n, (T*)r0, (T*)r1);
}

extern "C" pvjp_status pvjp_fig1_vjp(pvjp_dtype dtype, const void* x0, const void* x1, const void* y0_bar,
                                     const void* y1_bar, int64_t n, void* x0_bar, void* x1_bar, int accumulate,
                                     void* stream) {
    clear_error();
    PVJP_REQUIRE(valid_dtype(dtype), "pvjp_fig1_vjp: unknown dtype %d", (int)dtype);
    PVJP_REQUIRE(n >= 0, "pvjp_fig1_vjp: negative n");
    if (n == 0) return PVJP_OK;
    PVJP_REQUIRE(x0 && x1 && y0_bar && y1_bar && x0_bar && x1_bar, "pvjp_fig1_vjp: pointers must be non-NULL");
    if (dtype == PVJP_F64)
        launch_fig1_vjp<double>(x0, x1, y0_bar, y1_bar, n, x0_bar, x1_bar, accumulate, as_stream(stream));
    else
        launch_fig1_vjp<float>(x0, x1, y0_bar, y1_bar, n, x0_bar, x1_bar, accumulate, as_stream(stream));
    PVJP_LAUNCHED("pvjp_fig1_vjp");
    return PVJP_OK;
}

// Forward mode: y_dot_i = f'(x_i) x_dot_i.  The Jacobian of an elementwise
// unary map is diagonal, so this is the VJP kernel with x_dot in place of
// y_bar (and assignment, not accumulation).
extern "C" pvjp_status pvjp_map_jvp(pvjp_fn fn, pvjp_dtype dtype, const void* x, const void* x_dot, int64_t n,
                                    void* y_dot, void* stream) {
    clear_error();
    PVJP_REQUIRE(valid_fn(fn), "pvjp_map_jvp: unknown fn %d", (int)fn);
    PVJP_REQUIRE(valid_dtype(dtype), "pvjp_map_jvp: unknown dtype %d", (int)dtype);
    PVJP_REQUIRE(n >= 0, "pvjp_map_jvp: negative n");
    if (n == 0) return PVJP_OK;
    PVJP_REQUIRE(x != nullptr && x_dot != nullptr && y_dot != nullptr, "pvjp_map_jvp: NULL argument");
    if (dtype == PVJP_F64)
        dispatch_map_vjp<double>(fn, x, x_dot, n, y_dot, 0, as_stream(stream));
    else
        dispatch_map_vjp<float>(fn, x, x_dot, n, y_dot, 0, as_stream(stream));
    PVJP_LAUNCHED("pvjp_map_jvp");
    return PVJP_OK;
}
