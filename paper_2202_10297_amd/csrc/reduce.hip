// reduce with the special operators of Sec. 5.1.1 and their VJPs.
//
// Forward sweeps compute the extended results the return sweeps need:
//   ADD: the sum (formed in FP64);
//   MUL: (p, z) = (product of the non-zero elements in FP64, zero count);
//   MIN/MAX: (y, i_y) with i_y the lowest index attaining the extreme.
// One launch: each block reduces a contiguous chunk, the last block to finish
// (a ticket in the workspace) combines the per-block partials in block order,
// so results are deterministic.
//
// Return sweeps are maps:
//   ADD: x_bar_i += y_bar;
//   MUL: z == 0: x_bar_i += p / x_i * y_bar; z == 1: only the zero element
//        gets p * y_bar; z >= 2: nothing;
//   MIN/MAX: only x_bar[i_y] += y_bar (the sparse adjoint of Sec. 5.1.1: with
//        accumulation a single element is touched).
#include "common.h"
#include "prims.h"

namespace pvjp {

constexpr int kRedBlock = 256;
constexpr int kRedMaxGrid = 1024;

struct RedPart {
    double v;
    int64_t i;
};

struct RedHdr {
    uint32_t done;
    uint32_t pad[63];
};

template <int OP>
__device__ __forceinline__ RedPart red_id() {
    if (OP == PVJP_ADD) return RedPart{0.0, 0};
    if (OP == PVJP_MUL) return RedPart{1.0, 0};
    if (OP == PVJP_MIN) return RedPart{__builtin_huge_val(), -1};
    return RedPart{-__builtin_huge_val(), -1};
}

template <int OP>
__device__ __forceinline__ RedPart red_comb(RedPart a, RedPart b) {
    if (OP == PVJP_ADD) return RedPart{a.v + b.v, 0};
    if (OP == PVJP_MUL) return RedPart{a.v * b.v, a.i + b.i};
    // MIN / MAX on (value, index): the better value wins, ties go to the
    // lower index; an index of -1 marks "no element yet".
    if (a.i < 0) return b;
    if (b.i < 0) return a;
    const bool b_better = (OP == PVJP_MAX) ? (b.v > a.v) : (b.v < a.v);
    const bool a_better = (OP == PVJP_MAX) ? (a.v > b.v) : (a.v < b.v);
    if (b_better) return b;
    if (a_better) return a;
    return (b.i < a.i) ? b : a;
}

template <class T, int OP>
__device__ __forceinline__ RedPart red_elem(T x, int64_t i) {
    if (OP == PVJP_ADD) return RedPart{(double)x, 0};
    if (OP == PVJP_MUL) return (x == T(0)) ? RedPart{1.0, 1} : RedPart{(double)x, 0};
    return RedPart{(double)x, i};
}

__device__ __forceinline__ RedPart red_shfl_down(RedPart v, int d) {
    return RedPart{__shfl_down(v.v, d, kWave), (int64_t)__shfl_down((long long)v.i, d, kWave)};
}

// Fixed-shape tree over the block: deterministic for a given input.
template <int OP>
__device__ __forceinline__ RedPart block_reduce(RedPart v, RedPart* sh) {
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
#pragma unroll
    for (int d = kWave / 2; d >= 1; d >>= 1) {
        RedPart o = red_shfl_down(v, d);
        v = red_comb<OP>(v, o);
    }
    __syncthreads();
    if (lane == 0) sh[wid] = v;
    __syncthreads();
    RedPart r = sh[0];
#pragma unroll
    for (int w = 1; w < kRedBlock / kWave; ++w) r = red_comb<OP>(r, sh[w]);
    return r;
}

// Four consecutive elements from 16-byte loads (FP32: one, FP64: two).
template <class T>
__device__ __forceinline__ void load4(const T* __restrict__ x, int64_t e, T (&v)[4]) {
    if (sizeof(T) == 4) {
        const float4 f = *reinterpret_cast<const float4*>(x + e);
        v[0] = (T)f.x, v[1] = (T)f.y, v[2] = (T)f.z, v[3] = (T)f.w;
    } else {
        const double2 a = *reinterpret_cast<const double2*>(x + e);
        const double2 b = *reinterpret_cast<const double2*>(x + e + 2);
        v[0] = (T)a.x, v[1] = (T)a.y, v[2] = (T)b.x, v[3] = (T)b.y;
    }
}

// VEC: the chunk starts 16-byte aligned; each thread keeps four partial
// results (one per position in a quad) and has kRedU quads in flight, so
// the loads are not serialised behind one accumulator chain.  The partials
// are combined in a fixed order; MIN/MAX ties still go to the lowest index
// whatever the order.
constexpr int kRedU = 4;

template <class T, int OP, bool VEC>
__global__ __launch_bounds__(kRedBlock) void reduce_kernel(const T* __restrict__ x, int64_t n,
                                                           int64_t chunk, RedHdr* hdr,
                                                           RedPart* parts, T* y, int64_t* arg,
                                                           T* p, int64_t* z) {
    __shared__ RedPart sh[kRedBlock / kWave];
    __shared__ int s_last;
    const int64_t lo = (int64_t)blockIdx.x * chunk;
    const int64_t hi = (lo + chunk < n) ? lo + chunk : n;
    RedPart acc = red_id<OP>();
    int64_t rest = lo;
    if (VEC) {
        RedPart a4[4] = {red_id<OP>(), red_id<OP>(), red_id<OP>(), red_id<OP>()};
        const int64_t q0 = lo >> 2, q1 = hi >> 2;  // whole quads of the chunk
        for (int64_t q = q0 + threadIdx.x; q < q1; q += (int64_t)kRedBlock * kRedU) {
            T v[kRedU][4];
#pragma unroll
            for (int u = 0; u < kRedU; ++u) {
                const int64_t qq = q + (int64_t)u * kRedBlock;
                if (qq < q1) load4<T>(x, 4 * qq, v[u]);
            }
#pragma unroll
            for (int u = 0; u < kRedU; ++u) {
                const int64_t qq = q + (int64_t)u * kRedBlock;
                if (qq < q1) {
#pragma unroll
                    for (int t = 0; t < 4; ++t) a4[t] = red_comb<OP>(a4[t], red_elem<T, OP>(v[u][t], 4 * qq + t));
                }
            }
        }
        acc = red_comb<OP>(red_comb<OP>(a4[0], a4[1]), red_comb<OP>(a4[2], a4[3]));
        rest = q1 << 2;
    }
    for (int64_t i = rest + threadIdx.x; i < hi; i += kRedBlock) acc = red_comb<OP>(acc, red_elem<T, OP>(x[i], i));
    acc = block_reduce<OP>(acc, sh);
    if (threadIdx.x == 0) {
        st_coherent(&parts[blockIdx.x], acc);
        uint32_t d = __hip_atomic_fetch_add(&hdr->done, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        s_last = (d == gridDim.x - 1);
    }
    __syncthreads();
    if (!s_last) return;
    RedPart r = red_id<OP>();
    for (int b = threadIdx.x; b < (int)gridDim.x; b += kRedBlock) r = red_comb<OP>(r, ld_coherent(&parts[b]));
    r = block_reduce<OP>(r, sh);
    if (threadIdx.x == 0) {
        if (OP == PVJP_ADD) {
            *y = (T)r.v;
        } else if (OP == PVJP_MUL) {
            *p = (T)r.v;
            *z = r.i;
            *y = (r.i == 0) ? (T)r.v : T(0);
        } else {
            *arg = r.i;
            *y = (r.i >= 0) ? x[r.i] : (T)r.v;  // the element itself: keeps the sign of a zero
        }
        __hip_atomic_store(&hdr->done, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

template <class T, int OP, bool ACC>
__global__ __launch_bounds__(256) void reduce_vjp_kernel(const T* __restrict__ x, int64_t n,
                                                         const int64_t* __restrict__ arg,
                                                         const T* __restrict__ p,
                                                         const int64_t* __restrict__ z,
                                                         const T* __restrict__ ybar,
                                                         T* __restrict__ xbar) {
    const T yb = *ybar;
    int64_t zz = 0, ia = -1;
    T pp = T(0);
    if (OP == PVJP_MUL) {
        zz = *z;
        pp = *p;
        if (ACC && zz >= 2) return;
    }
    if (OP == PVJP_MIN || OP == PVJP_MAX) ia = *arg;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        T c;
        if (OP == PVJP_ADD) {
            c = yb;
        } else if (OP == PVJP_MUL) {
            if (zz == 0) {
                c = pp / x[i] * yb;
            } else if (zz == 1) {
                c = (x[i] == T(0)) ? pp * yb : T(0);
            } else {
                c = T(0);
            }
        } else {
            c = (i == ia) ? yb : T(0);
        }
        xbar[i] = ACC ? xbar[i] + c : c;
    }
}

// Accumulating min/max adjoint: only the winner is touched.
template <class T>
__global__ void reduce_vjp_onehot_acc(const int64_t* __restrict__ arg, const T* __restrict__ ybar,
                                      T* __restrict__ xbar) {
    const int64_t i = *arg;
    if (i >= 0) xbar[i] += *ybar;
}

// ------------------------------------------------------------------ host
static int64_t red_grid(int64_t n) {
    int64_t g = ceil_div(n, (int64_t)kRedBlock * 16);
    if (g < 1) g = 1;
    if (g > kRedMaxGrid) g = kRedMaxGrid;
    return g;
}

template <class T, int OP>
static void launch_reduce(const void* x, int64_t n, void* y, int64_t* arg, void* p, int64_t* z,
                          void* ws, hipStream_t st) {
    const int64_t g = red_grid(n);
    // chunks are whole 4-element quads, so every chunk of an aligned input
    // starts aligned
    const int64_t chunk = ceil_div(ceil_div(n, g), (int64_t)4) * 4;
    const int64_t g2 = n > 0 ? ceil_div(n, chunk) : 1;
    auto* hdr = reinterpret_cast<RedHdr*>(ws);
    auto* parts = reinterpret_cast<RedPart*>(reinterpret_cast<char*>(ws) + sizeof(RedHdr));
    if (aligned(x, 16))
        hipLaunchKernelGGL((reduce_kernel<T, OP, true>), dim3((unsigned)g2), dim3(kRedBlock), 0, st, (const T*)x,
                           n, chunk, hdr, parts, (T*)y, arg, (T*)p, z);
    else
        hipLaunchKernelGGL((reduce_kernel<T, OP, false>), dim3((unsigned)g2), dim3(kRedBlock), 0, st, (const T*)x,
                           n, chunk, hdr, parts, (T*)y, arg, (T*)p, z);
}

template <class T, int OP>
static void launch_vjp(const void* x, int64_t n, const int64_t* arg, const void* p, const int64_t* z,
                       const void* ybar, void* xbar, int acc, hipStream_t st) {
    const unsigned g = flat_grid(n, 256, 8);
    if ((OP == PVJP_MIN || OP == PVJP_MAX) && acc) {
        hipLaunchKernelGGL(reduce_vjp_onehot_acc<T>, dim3(1), dim3(1), 0, st, arg, (const T*)ybar, (T*)xbar);
        return;
    }
    if (acc)
        hipLaunchKernelGGL((reduce_vjp_kernel<T, OP, true>), dim3(g), dim3(256), 0, st, (const T*)x, n, arg,
                           (const T*)p, z, (const T*)ybar, (T*)xbar);
    else
        hipLaunchKernelGGL((reduce_vjp_kernel<T, OP, false>), dim3(g), dim3(256), 0, st, (const T*)x, n, arg,
                           (const T*)p, z, (const T*)ybar, (T*)xbar);
}

// ------------------------------------------------------------ forward mode
// MIN/MAX: y_dot = x_dot[arg] (0 for an empty input).
template <class T>
__global__ void reduce_jvp_pick_kernel(const int64_t* arg, const T* __restrict__ xd, T* __restrict__ yd) {
    const int64_t a = *arg;
    *yd = a >= 0 ? xd[a] : T(0);
}

// MUL: with p the product of the non-zero elements and z the zero count,
// y = p if z == 0 else 0, so y_dot = p sum_i x_dot_i / x_i (z == 0),
// p x_dot_{i0} at the one zero i0 (z == 1), 0 (z >= 2).  One pass forms both
// sums in FP64 (s1 over non-zeros, s0 over zeros); the last block combines
// the block sums in a fixed order.
struct MulJvpPart {
    double s0, s1;
};

template <class T>
__global__ __launch_bounds__(kRedBlock) void reduce_mul_jvp_kernel(const T* __restrict__ x, const T* __restrict__ xd,
                                                                   int64_t n, int64_t chunk, RedHdr* hdr,
                                                                   MulJvpPart* parts, const T* p, const int64_t* z,
                                                                   T* yd) {
    __shared__ double sh0[kRedBlock], sh1[kRedBlock];
    __shared__ int s_last;
    const int64_t lo = (int64_t)blockIdx.x * chunk;
    const int64_t hi = (lo + chunk < n) ? lo + chunk : n;
    double a0 = 0.0, a1 = 0.0;
    for (int64_t i = lo + threadIdx.x; i < hi; i += kRedBlock) {
        const double v = (double)x[i], t = (double)xd[i];
        if (v == 0.0) a0 += t;
        else a1 += t / v;
    }
    sh0[threadIdx.x] = a0, sh1[threadIdx.x] = a1;
    __syncthreads();
    for (int d = kRedBlock / 2; d >= 1; d >>= 1) {
        if ((int)threadIdx.x < d) {
            sh0[threadIdx.x] += sh0[threadIdx.x + d];
            sh1[threadIdx.x] += sh1[threadIdx.x + d];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        __hip_atomic_store(&parts[blockIdx.x].s0, sh0[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(&parts[blockIdx.x].s1, sh1[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const uint32_t d = __hip_atomic_fetch_add(&hdr->done, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        s_last = (d == gridDim.x - 1);
    }
    __syncthreads();
    if (!s_last || threadIdx.x != 0) return;
    double s0 = 0.0, s1 = 0.0;
    for (unsigned b = 0; b < gridDim.x; ++b) {
        s0 += __hip_atomic_load(&parts[b].s0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        s1 += __hip_atomic_load(&parts[b].s1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    const int64_t zc = *z;
    const double pv = (double)*p;
    *yd = (T)(zc == 0 ? pv * s1 : (zc == 1 ? pv * s0 : 0.0));
    __hip_atomic_store(&hdr->done, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

static_assert(sizeof(MulJvpPart) <= sizeof(RedPart), "the MUL forward mode reuses the reduce partial slots");

template <class T>
static void launch_reduce_jvp(pvjp_op op, const void* x, const void* xd, int64_t n, const int64_t* arg,
                              const void* p, const int64_t* z, void* yd, void* ws, hipStream_t st) {
    if (op == PVJP_ADD) {
        launch_reduce<T, PVJP_ADD>(xd, n, yd, nullptr, nullptr, nullptr, ws, st);
    } else if (op == PVJP_MUL) {
        const int64_t g = red_grid(n);
        const int64_t chunk = n > 0 ? ceil_div(n, g) : 1;
        const int64_t g2 = n > 0 ? ceil_div(n, chunk) : 1;
        auto* hdr = reinterpret_cast<RedHdr*>(ws);
        auto* parts = reinterpret_cast<MulJvpPart*>(reinterpret_cast<char*>(ws) + sizeof(RedHdr));
        hipLaunchKernelGGL(reduce_mul_jvp_kernel<T>, dim3((unsigned)g2), dim3(kRedBlock), 0, st, (const T*)x,
                           (const T*)xd, n, chunk, hdr, parts, (const T*)p, z, (T*)yd);
    } else {
        hipLaunchKernelGGL(reduce_jvp_pick_kernel<T>, dim3(1), dim3(1), 0, st, arg, (const T*)xd, (T*)yd);
    }
}

template <class T>
static void dispatch_reduce(pvjp_op op, const void* x, int64_t n, void* y, int64_t* arg, void* p,
                            int64_t* z, void* ws, hipStream_t st) {
    switch (op) {
        case PVJP_ADD: launch_reduce<T, PVJP_ADD>(x, n, y, arg, p, z, ws, st); break;
        case PVJP_MUL: launch_reduce<T, PVJP_MUL>(x, n, y, arg, p, z, ws, st); break;
        case PVJP_MIN: launch_reduce<T, PVJP_MIN>(x, n, y, arg, p, z, ws, st); break;
        default: launch_reduce<T, PVJP_MAX>(x, n, y, arg, p, z, ws, st); break;
    }
}

template <class T>
static void dispatch_vjp(pvjp_op op, const void* x, int64_t n, const int64_t* arg, const void* p,
                         const int64_t* z, const void* ybar, void* xbar, int acc, hipStream_t st) {
    switch (op) {
        case PVJP_ADD: launch_vjp<T, PVJP_ADD>(x, n, arg, p, z, ybar, xbar, acc, st); break;
        case PVJP_MUL: launch_vjp<T, PVJP_MUL>(x, n, arg, p, z, ybar, xbar, acc, st); break;
        case PVJP_MIN: launch_vjp<T, PVJP_MIN>(x, n, arg, p, z, ybar, xbar, acc, st); break;
        default: launch_vjp<T, PVJP_MAX>(x, n, arg, p, z, ybar, xbar, acc, st); break;
    }
}

}  // namespace pvjp

using namespace pvjp;

extern "C" size_t pvjp_reduce_ws_bytes(pvjp_op op, pvjp_dtype dtype, int64_t n) {
    if (!valid_op(op) || !valid_dtype(dtype) || n < 0) return 0;
    return sizeof(RedHdr) + (size_t)red_grid(n) * sizeof(RedPart);
}

extern "C" pvjp_status pvjp_reduce(pvjp_op op, pvjp_dtype dtype, const void* x, int64_t n, void* y,
                                   int64_t* arg, void* p, int64_t* z, void* ws, size_t ws_bytes,
                                   void* stream) {
    clear_error();
    PVJP_REQUIRE(valid_op(op), "pvjp_reduce: unknown op %d", (int)op);
    PVJP_REQUIRE(valid_dtype(dtype), "pvjp_reduce: unknown dtype %d", (int)dtype);
    PVJP_REQUIRE(n >= 0, "pvjp_reduce: n = %lld is negative", (long long)n);
    PVJP_REQUIRE(y != nullptr && (n == 0 || x != nullptr), "pvjp_reduce: x and y must be non-NULL");
    PVJP_REQUIRE(!(op == PVJP_MIN || op == PVJP_MAX) || arg != nullptr,
                 "pvjp_reduce: MIN/MAX need the arg output");
    PVJP_REQUIRE(op != PVJP_MUL || (p != nullptr && z != nullptr), "pvjp_reduce: MUL needs the p and z outputs");
    PVJP_REQUIRE(ws != nullptr && aligned(ws, 256), "pvjp_reduce: ws must be non-NULL and 256-byte aligned");
    const size_t need = pvjp_reduce_ws_bytes(op, dtype, n);
    if (ws_bytes < need) {
        set_error("pvjp_reduce: workspace has %zu bytes, needs %zu", ws_bytes, need);
        return PVJP_ENOMEM;
    }
    if (dtype == PVJP_F64)
        dispatch_reduce<double>(op, x, n, y, arg, p, z, ws, as_stream(stream));
    else
        dispatch_reduce<float>(op, x, n, y, arg, p, z, ws, as_stream(stream));
    PVJP_LAUNCHED("pvjp_reduce");
    return PVJP_OK;
}

extern "C" pvjp_status pvjp_reduce_vjp(pvjp_op op, pvjp_dtype dtype, const void* x, int64_t n,
                                       const int64_t* arg, const void* p, const int64_t* z,
                                       const void* y_bar, void* x_bar, int accumulate, void* stream) {
    clear_error();
    PVJP_REQUIRE(valid_op(op), "pvjp_reduce_vjp: unknown op %d", (int)op);
    PVJP_REQUIRE(valid_dtype(dtype), "pvjp_reduce_vjp: unknown dtype %d", (int)dtype);
    PVJP_REQUIRE(n >= 0, "pvjp_reduce_vjp: n = %lld is negative", (long long)n);
    if (n == 0) return PVJP_OK;
    PVJP_REQUIRE(y_bar != nullptr && x_bar != nullptr, "pvjp_reduce_vjp: y_bar and x_bar must be non-NULL");
    PVJP_REQUIRE(op != PVJP_MUL || (x != nullptr && p != nullptr && z != nullptr),
                 "pvjp_reduce_vjp: MUL needs x, p and z");
    PVJP_REQUIRE(!(op == PVJP_MIN || op == PVJP_MAX) || arg != nullptr, "pvjp_reduce_vjp: MIN/MAX need arg");
    if (dtype == PVJP_F64)
        dispatch_vjp<double>(op, x, n, arg, p, z, y_bar, x_bar, accumulate, as_stream(stream));
    else
        dispatch_vjp<float>(op, x, n, arg, p, z, y_bar, x_bar, accumulate, as_stream(stream));
    PVJP_LAUNCHED("pvjp_reduce_vjp");
    return PVJP_OK;
}

extern "C" pvjp_status pvjp_reduce_jvp(pvjp_op op, pvjp_dtype dtype, const void* x, const void* x_dot, int64_t n,
                                       const int64_t* arg, const void* p, const int64_t* z, void* y_dot, void* ws,
                                       size_t ws_bytes, void* stream) {
    clear_error();
    PVJP_REQUIRE(valid_op(op), "pvjp_reduce_jvp: unknown op %d", (int)op);
    PVJP_REQUIRE(valid_dtype(dtype), "pvjp_reduce_jvp: unknown dtype %d", (int)dtype);
    PVJP_REQUIRE(n >= 0, "pvjp_reduce_jvp: n = %lld is negative", (long long)n);
    PVJP_REQUIRE(y_dot != nullptr && (n == 0 || x_dot != nullptr), "pvjp_reduce_jvp: x_dot and y_dot must be non-NULL");
    PVJP_REQUIRE(op != PVJP_MUL || ((n == 0 || x != nullptr) && p != nullptr && z != nullptr),
                 "pvjp_reduce_jvp: MUL needs x, p and z");
    PVJP_REQUIRE(!(op == PVJP_MIN || op == PVJP_MAX) || arg != nullptr, "pvjp_reduce_jvp: MIN/MAX need arg");
    if (op == PVJP_ADD || op == PVJP_MUL) {
        PVJP_REQUIRE(ws != nullptr && aligned(ws, 256), "pvjp_reduce_jvp: ws must be non-NULL and 256-byte aligned");
        const size_t need = pvjp_reduce_ws_bytes(op, dtype, n);
        if (ws_bytes < need) {
            set_error("pvjp_reduce_jvp: workspace has %zu bytes, needs %zu", ws_bytes, need);
            return PVJP_ENOMEM;
        }
    }
    if (dtype == PVJP_F64)
        launch_reduce_jvp<double>(op, x, x_dot, n, arg, p, z, y_dot, ws, as_stream(stream));
    else
        launch_reduce_jvp<float>(op, x, x_dot, n, arg, p, z, y_dot, ws, as_stream(stream));
    PVJP_LAUNCHED("pvjp_reduce_jvp");
    return PVJP_OK;
}
