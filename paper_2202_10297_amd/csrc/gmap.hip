// A map whose body reads a free array at computed indices (Sec. 5.4):
//   ys[i] = f(as[is[i]], vs[i]),  f = a (gather), a v, or (a - v)^2,
// and its return sweep, where the reads of the free array become an
// accumulator: as_bar[is[i]] += (df/da)(a_i, v_i) ys_bar[i], next to the
// per-element vs_bar[i] = (df/dv) ys_bar[i].  The accumulator is lowered
// (Sec. 6) to FP64 atomics in LDS bins when as fits a block's LDS (a bin
// per element of as, per block; the blocks' bins are then summed in a fixed
// order).  A larger as takes the reduce_by_index(+) path of this library on
// the partials, written once per element: its LDS bin caches and bucket
// partitioning keep hot indices off contended global atomics.  An index
// outside [0, n) reads 0 and updates nothing.
#include "common.h"
#include "prims.h"

namespace pvjp {

constexpr int kGmLdsBins = 16384;  // FP64 bins a block holds in LDS (128 KB)
constexpr int kGmLdsBlock = 1024;
constexpr int kGmLdsBlocks = 256;  // one per CU: the partials stay small
constexpr int kGmMergeWaves = 16;

template <int OP, class T>
__device__ inline T gm_f(T a, T v) {
    if (OP == 0) return a;
    if (OP == 1) return a * v;
    const T d = a - v;
    return d * d;
}

// The partials of one element's read (pa, into as_bar) and of vs (pv), in
// FP64 from the element's values.
template <int OP>
__device__ inline void gm_partials(double a, double v, double yb, double& pa, double& pv) {
    if (OP == 0) {
        pa = yb, pv = 0.0;
    } else if (OP == 1) {
        pa = v * yb, pv = a * yb;
    } else {
        const double d = 2.0 * (a - v) * yb;
        pa = d, pv = -d;
    }
}

constexpr int kGmU = 4;  // elements per thread per step, their loads in flight together

// The per-element arrays are streamed once: their loads and stores go
// non-temporal, so they do not push the gathered lines of as out of L2.
template <class T>
__device__ __forceinline__ T nt_ld(const T* p) {
    return __builtin_nontemporal_load(p);
}
template <class T>
__device__ __forceinline__ void nt_st(T* p, T v) {
    __builtin_nontemporal_store(v, p);
}

// Each step of a thread takes elements base + u 256 + t, u < kGmU (coalesced
// for every u): all index and value loads, then all gathers, then the stores.
template <int OP, class T>
__global__ __launch_bounds__(256) void gm_fwd_kernel(const T* __restrict__ as, int64_t n,
                                                     const int32_t* __restrict__ is, const T* __restrict__ vs,
                                                     int64_t m, T* __restrict__ ys) {
    const int64_t step = (int64_t)gridDim.x * blockDim.x * kGmU;
    for (int64_t base = (int64_t)blockIdx.x * blockDim.x * kGmU + threadIdx.x; base < m; base += step) {
        int64_t k[kGmU];
        T v[kGmU], a[kGmU];
#pragma unroll
        for (int u = 0; u < kGmU; ++u) {
            const int64_t i = base + (int64_t)u * blockDim.x;
            k[u] = i < m ? nt_ld(is + i) : -1;
            v[u] = (OP && i < m) ? nt_ld(vs + i) : T(0);
        }
#pragma unroll
        for (int u = 0; u < kGmU; ++u) a[u] = (k[u] >= 0 && k[u] < n) ? as[k[u]] : T(0);
#pragma unroll
        for (int u = 0; u < kGmU; ++u) {
            const int64_t i = base + (int64_t)u * blockDim.x;
            if (i < m) nt_st(ys + i, gm_f<OP, T>(a[u], v[u]));
        }
    }
}

// LDS plan: block b takes elements [b chunk, (b+1) chunk), adds each read's
// partial into its LDS bin, then writes its n bins to part[b][.].
template <int OP, class T>
__global__ __launch_bounds__(kGmLdsBlock) void gm_vjp_lds_kernel(const T* __restrict__ as, int n,
                                                                 const int32_t* __restrict__ is,
                                                                 const T* __restrict__ vs, const T* __restrict__ yb,
                                                                 int64_t m, int64_t chunk, T* __restrict__ vbar,
                                                                 int accumulate, double* __restrict__ part) {
    extern __shared__ double bins[];
    for (int k = threadIdx.x; k < n; k += blockDim.x) bins[k] = 0.0;
    __syncthreads();
    const int64_t i0 = (int64_t)blockIdx.x * chunk;
    const int64_t i1 = (i0 + chunk < m) ? i0 + chunk : m;
    for (int64_t base = i0 + threadIdx.x; base < i1; base += (int64_t)blockDim.x * kGmU) {
        int32_t k[kGmU];
        T v[kGmU], y[kGmU], a[kGmU];
#pragma unroll
        for (int u = 0; u < kGmU; ++u) {
            const int64_t i = base + (int64_t)u * blockDim.x;
            const bool in = i < i1;
            k[u] = in ? is[i] : -1;
            v[u] = (OP && in) ? vs[i] : T(0);
            y[u] = in ? yb[i] : T(0);
        }
#pragma unroll
        for (int u = 0; u < kGmU; ++u) a[u] = (k[u] >= 0 && k[u] < n) ? as[k[u]] : T(0);
#pragma unroll
        for (int u = 0; u < kGmU; ++u) {
            const int64_t i = base + (int64_t)u * blockDim.x;
            if (i < i1) {
                double pa, pv;
                gm_partials<OP>((double)a[u], (double)v[u], (double)y[u], pa, pv);
                if (OP) vbar[i] = accumulate ? vbar[i] + (T)pv : (T)pv;
                if (k[u] >= 0 && k[u] < n) atomicAdd(&bins[k[u]], pa);
            }
        }
    }
    __syncthreads();
    for (int k = threadIdx.x; k < n; k += blockDim.x) part[(int64_t)blockIdx.x * n + k] = bins[k];
}

// as_bar[k] (+)= sum_b part[b][k]: block x takes bins [64 x, 64 x + 64); wave
// w sums the partials b = w, w + 16, ... in order, and the 16 wave sums are
// added in wave order.
template <class T>
__global__ __launch_bounds__(kGmMergeWaves* kWave) void gm_merge_kernel(const double* __restrict__ part, int n,
                                                                        int G, T* __restrict__ abar,
                                                                        int accumulate) {
    __shared__ double sh[kGmMergeWaves][kWave];
    const int w = threadIdx.x / kWave, lane = threadIdx.x & (kWave - 1);
    const int k = blockIdx.x * kWave + lane;
    double s = 0.0;
    if (k < n)
        for (int b = w; b < G; b += kGmMergeWaves) s += part[(int64_t)b * n + k];
    sh[w][lane] = s;
    __syncthreads();
    if (w == 0 && k < n) {
        double t = 0.0;
        for (int q = 0; q < kGmMergeWaves; ++q) t += sh[q][lane];
        abar[k] = accumulate ? abar[k] + (T)t : (T)t;
    }
}

// Larger as: vs_bar and each element's partial c[i] (0 out of range), which
// the reduce_by_index(+) path then sums into the bins.
template <int OP, class T>
__global__ __launch_bounds__(256) void gm_contrib_kernel(const T* __restrict__ as, int64_t n,
                                                         const int32_t* __restrict__ is, const T* __restrict__ vs,
                                                         const T* __restrict__ yb, int64_t m, T* __restrict__ vbar,
                                                         int accumulate, T* __restrict__ c) {
    const int64_t step = (int64_t)gridDim.x * blockDim.x * kGmU;
    for (int64_t base = (int64_t)blockIdx.x * blockDim.x * kGmU + threadIdx.x; base < m; base += step) {
        int32_t k[kGmU];
        T v[kGmU], y[kGmU], a[kGmU];
#pragma unroll
        for (int u = 0; u < kGmU; ++u) {
            const int64_t i = base + (int64_t)u * blockDim.x;
            const bool in = i < m;
            k[u] = in ? nt_ld(is + i) : -1;
            v[u] = (OP && in) ? nt_ld(vs + i) : T(0);
            y[u] = in ? nt_ld(yb + i) : T(0);
        }
#pragma unroll
        for (int u = 0; u < kGmU; ++u) a[u] = (OP && k[u] >= 0 && k[u] < n) ? as[k[u]] : T(0);
#pragma unroll
        for (int u = 0; u < kGmU; ++u) {
            const int64_t i = base + (int64_t)u * blockDim.x;
            if (i < m) {
                double pa, pv;
                gm_partials<OP>((double)a[u], (double)v[u], (double)y[u], pa, pv);
                if (OP) {
                    if (accumulate) vbar[i] = vbar[i] + (T)pv;
                    else nt_st(vbar + i, (T)pv);
                }
                nt_st(c + i, (k[u] >= 0 && k[u] < n) ? (T)pa : T(0));
            }
        }
    }
}

template <class T>
__global__ __launch_bounds__(256) void gm_add_kernel(const T* __restrict__ h, int64_t n, T* __restrict__ abar) {
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x)
        abar[k] += h[k];
}

struct GmPlan {
    bool lds;
    int G;
    int64_t chunk;
    size_t c, hist, hist_bytes, tmp, total;  // larger as: partials, reduce_by_index workspace, sums
};

static GmPlan gm_plan(pvjp_dtype dtype, int64_t n, int64_t m) {
    GmPlan p{};
    p.lds = n <= kGmLdsBins;
    const int64_t m1 = m > 0 ? m : 1;
    if (p.lds) {
        int64_t g = ceil_div(m1, (int64_t)kGmLdsBlock * 8);
        p.G = (int)(g < kGmLdsBlocks ? g : kGmLdsBlocks);
        p.chunk = ceil_div(m1, p.G);
        p.total = align_up((size_t)p.G * (size_t)(n > 0 ? n : 1) * 8, 256);
    } else {
        const size_t es = dsize(dtype);
        p.c = 0;
        p.hist = align_up((size_t)m1 * es, 256);
        p.hist_bytes = align_up(pvjp_hist_ws_bytes(PVJP_ADD, dtype, m1, n), 256);
        p.tmp = p.hist + p.hist_bytes;
        p.total = p.tmp + align_up((size_t)n * es, 256);
    }
    return p;
}

template <int OP, class T>
static pvjp_status gm_launch_vjp(pvjp_dtype dtype, const void* as, int64_t n, const int32_t* is, const void* vs,
                                 int64_t m, const void* yb, void* abar, void* vbar, int acc, char* ws,
                                 const GmPlan& p, hipStream_t st) {
    const T* a = (const T*)as;
    const T* v = (const T*)vs;
    const T* y = (const T*)yb;
    T* ab = (T*)abar;
    T* vb = (T*)vbar;
    if (p.lds) {
        static const bool once = [] {  // allow the dynamic LDS beyond 64 KB, once per process
            if (hipFuncSetAttribute(reinterpret_cast<const void*>(&gm_vjp_lds_kernel<OP, T>),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, kGmLdsBins * 8) != hipSuccess)
                (void)hipGetLastError();
            return true;
        }();
        (void)once;
        double* w = (double*)ws;
        if (n > 0 || m > 0)
            hipLaunchKernelGGL((gm_vjp_lds_kernel<OP, T>), dim3((unsigned)p.G), dim3(kGmLdsBlock), (size_t)n * 8, st,
                               a, (int)n, is, v, y, m, p.chunk, vb, acc, w);
        if (n > 0)
            hipLaunchKernelGGL((gm_merge_kernel<T>), dim3((unsigned)ceil_div(n, kWave)), dim3(kGmMergeWaves * kWave),
                               0, st, (const double*)w, (int)n, p.G, ab, acc);
        return PVJP_OK;
    }
    T* c = (T*)(ws + p.c);
    T* sums = acc ? (T*)(ws + p.tmp) : ab;
    if (m > 0)
        hipLaunchKernelGGL((gm_contrib_kernel<OP, T>), dim3(flat_grid(m, 256, 4)), dim3(256), 0, st, a, n, is, v, y,
                           m, vb, acc, c);
    if (pvjp_status e = pvjp_hist(PVJP_ADD, dtype, is, c, m, n, sums, nullptr, nullptr, nullptr, nullptr,
                                  ws + p.hist, p.hist_bytes, st))
        return e;
    if (acc) hipLaunchKernelGGL((gm_add_kernel<T>), dim3(flat_grid(n, 256, 4)), dim3(256), 0, st, sums, n, ab);
    return PVJP_OK;
}

template <class T>
static void gm_launch_fwd(int op, const void* as, int64_t n, const int32_t* is, const void* vs, int64_t m, void* ys,
                          hipStream_t st) {
    const dim3 g(flat_grid(m, 256, 4)), b(256);
    const T* a = (const T*)as;
    const T* v = (const T*)vs;
    T* y = (T*)ys;
    if (op == PVJP_GMAP_GATHER) hipLaunchKernelGGL((gm_fwd_kernel<0, T>), g, b, 0, st, a, n, is, v, m, y);
    else if (op == PVJP_GMAP_MUL) hipLaunchKernelGGL((gm_fwd_kernel<1, T>), g, b, 0, st, a, n, is, v, m, y);
    else hipLaunchKernelGGL((gm_fwd_kernel<2, T>), g, b, 0, st, a, n, is, v, m, y);
}

static pvjp_status gm_check(const char* name, int op, pvjp_dtype dtype, const void* as, int64_t n, const int32_t* is,
                            const void* vs, int64_t m) {
    PVJP_REQUIRE(op >= PVJP_GMAP_GATHER && op <= PVJP_GMAP_SQDIFF, "%s: unknown op %d", name, op);
    PVJP_REQUIRE(valid_dtype(dtype), "%s: unknown dtype %d", name, (int)dtype);
    PVJP_REQUIRE(n >= 0 && n <= INT32_MAX && m >= 0, "%s: n = %lld, m = %lld out of range", name, (long long)n,
                 (long long)m);
    PVJP_REQUIRE(n == 0 || as != nullptr, "%s: as is NULL", name);
    PVJP_REQUIRE(m == 0 || (is != nullptr && (op == PVJP_GMAP_GATHER || vs != nullptr)), "%s: is or vs is NULL",
                 name);
    return PVJP_OK;
}

}  // namespace pvjp

using namespace pvjp;

extern "C" size_t pvjp_gather_map_ws_bytes(pvjp_dtype dtype, int64_t n, int64_t m) {
    if (n < 0 || m < 0 || !valid_dtype(dtype)) return 0;
    return gm_plan(dtype, n, m).total;
}

extern "C" pvjp_status pvjp_gather_map(int op, pvjp_dtype dtype, const void* as, int64_t n, const int32_t* is,
                                       const void* vs, int64_t m, void* ys, void* stream) {
    clear_error();
    if (pvjp_status e = gm_check("pvjp_gather_map", op, dtype, as, n, is, vs, m)) return e;
    PVJP_REQUIRE(m == 0 || ys != nullptr, "pvjp_gather_map: ys is NULL");
    if (m == 0) return PVJP_OK;
    hipStream_t st = as_stream(stream);
    if (dtype == PVJP_F32) gm_launch_fwd<float>(op, as, n, is, vs, m, ys, st);
    else gm_launch_fwd<double>(op, as, n, is, vs, m, ys, st);
    PVJP_LAUNCHED("pvjp_gather_map");
    return PVJP_OK;
}

extern "C" pvjp_status pvjp_gather_map_vjp(int op, pvjp_dtype dtype, const void* as, int64_t n, const int32_t* is,
                                           const void* vs, int64_t m, const void* ys_bar, void* as_bar, void* vs_bar,
                                           int accumulate, void* ws, size_t ws_bytes, void* stream) {
    clear_error();
    if (pvjp_status e = gm_check("pvjp_gather_map_vjp", op, dtype, as, n, is, vs, m)) return e;
    PVJP_REQUIRE(n == 0 || as_bar != nullptr, "pvjp_gather_map_vjp: as_bar is NULL");
    PVJP_REQUIRE(m == 0 || (ys_bar != nullptr && (op == PVJP_GMAP_GATHER || vs_bar != nullptr)),
                 "pvjp_gather_map_vjp: ys_bar or vs_bar is NULL");
    PVJP_REQUIRE(ws != nullptr && aligned(ws, 256), "pvjp_gather_map_vjp: ws must be non-NULL and 256-byte aligned");
    const GmPlan p = gm_plan(dtype, n, m);
    if (ws_bytes < p.total) {
        set_error("pvjp_gather_map_vjp: workspace has %zu bytes, needs %zu", ws_bytes, p.total);
        return PVJP_ENOMEM;
    }
    if (n == 0 && m == 0) return PVJP_OK;
    hipStream_t st = as_stream(stream);
    char* w = reinterpret_cast<char*>(ws);
    pvjp_status e;
    if (dtype == PVJP_F32) {
        if (op == PVJP_GMAP_GATHER) e = gm_launch_vjp<0, float>(dtype, as, n, is, vs, m, ys_bar, as_bar, vs_bar, accumulate, w, p, st);
        else if (op == PVJP_GMAP_MUL) e = gm_launch_vjp<1, float>(dtype, as, n, is, vs, m, ys_bar, as_bar, vs_bar, accumulate, w, p, st);
        else e = gm_launch_vjp<2, float>(dtype, as, n, is, vs, m, ys_bar, as_bar, vs_bar, accumulate, w, p, st);
    } else {
        if (op == PVJP_GMAP_GATHER) e = gm_launch_vjp<0, double>(dtype, as, n, is, vs, m, ys_bar, as_bar, vs_bar, accumulate, w, p, st);
        else if (op == PVJP_GMAP_MUL) e = gm_launch_vjp<1, double>(dtype, as, n, is, vs, m, ys_bar, as_bar, vs_bar, accumulate, w, p, st);
        else e = gm_launch_vjp<2, double>(dtype, as, n, is, vs, m, ys_bar, as_bar, vs_bar, accumulate, w, p, st);
    }
    if (e) return e;
    PVJP_LAUNCHED("pvjp_gather_map_vjp");
    return PVJP_OK;
}
