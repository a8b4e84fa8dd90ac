// reduce with a general associative operator and its VJP by the general rule
// of Sec. 5.1.1.  With ls_i = x_0 (.) ... (.) x_{i-1} and
// rs_i = x_{i+1} (.) ... (.) x_{n-1} (an exclusive scan and an exclusive
// reversed scan), x_bar_i (+)= (d(ls_i (.) x_i (.) rs_i) / dx_i)^T y_bar with
// ls_i and rs_i held constant: the function f mapped over (ls, xs, rs).
//
// The rule as stated costs two whole-array scans plus a map (at least five
// global accesses per element).  Here the scans are split over fixed tiles:
//   1. tile aggregates (read x);
//   2. one block scans the aggregates forward and backward, giving every
//      tile the fold of all tiles before it and of all tiles after it (and
//      the primal result y);
//   3. per tile, the in-tile exclusive prefixes and suffixes are formed in
//      registers and LDS and f is applied at once (read x, write x_bar).
// x is read twice and x_bar written once; ls and rs never reach memory.
//
// Operators (an element has K components, each its own array):
//   log-add-exp   a (.) b = log(e^a + e^b), neutral -inf (K = 1);
//   linear recurrence (a1,b1) (.) (a2,b2) = (a2 a1, a2 b1 + b2) (K = 2);
//   2x2 matrix product, row-major components (K = 4).
#include <type_traits>

#include "common.h"
#include "prims.h"

namespace pvjp {

constexpr int kGrBlock = 256;
constexpr int kGrAggBlock = 1024;
constexpr size_t kGrSlot = 32;  // bytes per tile for an aggregate, prefix or suffix

template <class T, int K>
struct GS {
    T c[K];
};

template <class T, int K>
struct GShfl {
    using S = GS<T, K>;
    __device__ static __forceinline__ S up(S v, int d) {
        S r;
#pragma unroll
        for (int c = 0; c < K; ++c) r.c[c] = shfl_up1(v.c[c], d);
        return r;
    }
    __device__ static __forceinline__ S down(S v, int d) {
        S r;
#pragma unroll
        for (int c = 0; c < K; ++c) r.c[c] = shfl_down1(v.c[c], d);
        return r;
    }
    __device__ static __forceinline__ S idx(S v, int s) {
        S r;
#pragma unroll
        for (int c = 0; c < K; ++c) r.c[c] = shfl_idx1(v.c[c], s);
        return r;
    }
};

// comb(x, y) = x (.) y with x earlier in index order.  vjp(l, a, r, yb, out)
// is the function f: out = (d(l (.) a (.) r)/da)^T yb.
template <class T>
struct GLogAddExp : GShfl<T, 1> {
    static constexpr int K = 1;
    using Acc = T;
    using S = GS<T, 1>;
    __device__ static __forceinline__ S id() { return S{{-(T)INFINITY}}; }
    __device__ static __forceinline__ S comb(S x, S y) {
        const T a = x.c[0], b = y.c[0];
        if (b == -(T)INFINITY) return x;
        if (a == -(T)INFINITY) return y;
        const T m = a > b ? a : b;
        return S{{m + log1p(exp(-fabs(a - b)))}};
    }
    __device__ static __forceinline__ void vjp(S l, S a, S r, const T (&yb)[1], T (&out)[1]) {
        // d/da log(e^l + e^a + e^r) = e^(a - y); a -inf element receives 0
        if (a.c[0] == -(T)INFINITY) {
            out[0] = T(0);
            return;
        }
        const S y = comb(comb(l, a), r);
        out[0] = yb[0] * exp(a.c[0] - y.c[0]);
    }
};

template <class T>
struct GLinRec : GShfl<T, 2> {
    static constexpr int K = 2;
    using Acc = T;
    using S = GS<T, 2>;
    __device__ static __forceinline__ S id() { return S{{T(1), T(0)}}; }
    __device__ static __forceinline__ S comb(S x, S y) { return S{{y.c[0] * x.c[0], y.c[0] * x.c[1] + y.c[1]}}; }
    __device__ static __forceinline__ void vjp(S l, S, S r, const T (&yb)[2], T (&out)[2]) {
        // y = (r.a x.a l.a, r.a (x.a l.b + x.b) + r.b)
        out[0] = r.c[0] * (yb[0] * l.c[0] + yb[1] * l.c[1]);
        out[1] = r.c[0] * yb[1];
    }
};

template <class T>
struct GMat2 : GShfl<T, 4> {
    static constexpr int K = 4;
    using Acc = T;
    using S = GS<T, 4>;
    __device__ static __forceinline__ S id() { return S{{T(1), T(0), T(0), T(1)}}; }
    __device__ static __forceinline__ S comb(S x, S y) {
        return S{{x.c[0] * y.c[0] + x.c[1] * y.c[2], x.c[0] * y.c[1] + x.c[1] * y.c[3],
                  x.c[2] * y.c[0] + x.c[3] * y.c[2], x.c[2] * y.c[1] + x.c[3] * y.c[3]}};
    }
    __device__ static __forceinline__ void vjp(S l, S, S r, const T (&yb)[4], T (&out)[4]) {
        // y = l a r, so a_bar = l^T y_bar r^T; M = y_bar r^T first
        const T m00 = yb[0] * r.c[0] + yb[1] * r.c[1], m01 = yb[0] * r.c[2] + yb[1] * r.c[3];
        const T m10 = yb[2] * r.c[0] + yb[3] * r.c[1], m11 = yb[2] * r.c[2] + yb[3] * r.c[3];
        out[0] = l.c[0] * m00 + l.c[2] * m10;
        out[1] = l.c[0] * m01 + l.c[2] * m11;
        out[2] = l.c[1] * m00 + l.c[3] * m10;
        out[3] = l.c[1] * m01 + l.c[3] * m11;
    }
};

// The same operator with its operands exchanged: a scan in reversed index
// order with it folds x_{i+1} (.) x_{i+2} (.) ... (the reversed scan of the
// rule, whose operator is \x y -> y (.) x).
template <class Op>
struct Flip : Op {
    using S = typename Op::S;
    __device__ static __forceinline__ S comb(S x, S y) { return Op::comb(y, x); }
};

template <class T>
struct GPtrs {
    const T* p[4];
};
template <class T>
struct GOut {
    T* p[4];
};

// Items per thread: 32 bytes of every component (two 16-byte loads).
template <class T>
constexpr int gr_ipt() {
    return 32 / (int)sizeof(T);
}
template <class T>
constexpr int gr_tile() {
    return kGrBlock * gr_ipt<T>();
}

// A thread's IPT consecutive elements of one component; `cnt` of them exist.
template <class T, int IPT, bool VEC>
__device__ __forceinline__ void gr_load(const T* __restrict__ p, int cnt, T (&v)[IPT]) {
    if (VEC && cnt == IPT) {
        constexpr int NV = IPT * (int)sizeof(T) / 16;
        uint4 w[NV];
#pragma unroll
        for (int j = 0; j < NV; ++j) w[j] = reinterpret_cast<const uint4*>(p)[j];
        __builtin_memcpy(v, w, sizeof(w));
    } else {
#pragma unroll
        for (int k = 0; k < IPT; ++k) v[k] = (k < cnt) ? p[k] : T(0);
    }
}

template <class T, int IPT, bool VEC>
__device__ __forceinline__ void gr_store(T* __restrict__ p, int cnt, const T (&v)[IPT]) {
    if (VEC && cnt == IPT) {
        constexpr int NV = IPT * (int)sizeof(T) / 16;
        uint4 w[NV];
        __builtin_memcpy(w, v, sizeof(w));
#pragma unroll
        for (int j = 0; j < NV; ++j) reinterpret_cast<uint4*>(p)[j] = w[j];
    } else {
#pragma unroll
        for (int k = 0; k < IPT; ++k)
            if (k < cnt) p[k] = v[k];
    }
}

// Element k of a thread's run as an operator state (converted to the
// operator's arithmetic type).
template <class Op, class T, int IPT>
__device__ __forceinline__ typename Op::S gr_elem(const T (&v)[Op::K][IPT], int k) {
    typename Op::S s;
#pragma unroll
    for (int c = 0; c < Op::K; ++c) s.c[c] = (typename Op::Acc)v[c][k];
    return s;
}

// Pass 1: agg[t] = fold of tile t in index order.
template <class Op, class T, bool VEC>
__global__ __launch_bounds__(kGrBlock) void gred_tile_agg_kernel(GPtrs<T> x, int64_t n,
                                                                 typename Op::S* __restrict__ agg) {
    using S = typename Op::S;
    constexpr int IPT = gr_ipt<T>();
    __shared__ S wtot[kGrBlock / kWave];
    const int64_t base = (int64_t)blockIdx.x * gr_tile<T>() + (int64_t)threadIdx.x * IPT;
    const int64_t left = n - base;
    const int cnt = left <= 0 ? 0 : (left >= IPT ? IPT : (int)left);
    T v[Op::K][IPT];
#pragma unroll
    for (int c = 0; c < Op::K; ++c) gr_load<T, IPT, VEC>(x.p[c] + base, cnt, v[c]);
    S run = Op::id();
#pragma unroll
    for (int k = 0; k < IPT; ++k)
        if (k < cnt) run = Op::comb(run, gr_elem<Op, T, IPT>(v, k));
    S total;
    block_exclusive_scan<Op, kGrBlock, false>(run, total, wtot);
    if (threadIdx.x == 0) agg[blockIdx.x] = total;
}

// Pass 2 (one block): pre[t] = fold of tiles before t, suf[t] = fold of
// tiles after t (either may be NULL); y (nullable components) = fold of all.
// Thread j owns a contiguous run of tiles; runs are scanned across the block
// in both directions.
template <class Op, class T>
__global__ __launch_bounds__(kGrAggBlock) void gred_agg_scan_kernel(const typename Op::S* __restrict__ agg,
                                                                    int64_t nt, typename Op::S* __restrict__ pre,
                                                                    typename Op::S* __restrict__ suf, GOut<T> y) {
    using S = typename Op::S;
    constexpr int U = 8;
    __shared__ S wtot[kGrAggBlock / kWave];
    const int64_t per = (nt + kGrAggBlock - 1) / kGrAggBlock;
    const int64_t v0 = (int64_t)threadIdx.x * per < nt ? (int64_t)threadIdx.x * per : nt;
    const int64_t v1 = v0 + per < nt ? v0 + per : nt;
    S run = Op::id();
    for (int64_t v = v0; v < v1; v += U) {
        S a[U];
#pragma unroll
        for (int u = 0; u < U; ++u) a[u] = (v + u < v1) ? agg[v + u] : Op::id();
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (v + u < v1) run = Op::comb(run, a[u]);
    }
    S total;
    S ex = block_exclusive_scan<Op, kGrAggBlock, false>(run, total, wtot);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int c = 0; c < Op::K; ++c)
            if (y.p[c]) *y.p[c] = (T)total.c[c];
    }
    if (pre) {
        for (int64_t v = v0; v < v1; ++v) {
            pre[v] = ex;
            ex = Op::comb(ex, agg[v]);
        }
    }
    if (suf) {
        S total2;
        S sx = block_exclusive_scan<Flip<Op>, kGrAggBlock, true>(run, total2, wtot);
        for (int64_t v = v1 - 1; v >= v0; --v) {
            suf[v] = sx;
            sx = Op::comb(agg[v], sx);
        }
    }
}

// Pass 3: per tile, ls_i and rs_i from the tile's prefix/suffix, the block
// scans of the threads' runs and the in-thread folds; x_bar_i (+)= f.
template <class Op, class T, bool VEC, bool ACC>
__global__ __launch_bounds__(kGrBlock) void gred_vjp_kernel(GPtrs<T> x, int64_t n,
                                                            const typename Op::S* __restrict__ pre,
                                                            const typename Op::S* __restrict__ suf, GPtrs<T> ybar,
                                                            GOut<T> xbar) {
    using S = typename Op::S;
    constexpr int K = Op::K;
    constexpr int IPT = gr_ipt<T>();
    __shared__ S wtot[kGrBlock / kWave];
    const int64_t base = (int64_t)blockIdx.x * gr_tile<T>() + (int64_t)threadIdx.x * IPT;
    const int64_t left = n - base;
    const int cnt = left <= 0 ? 0 : (left >= IPT ? IPT : (int)left);
    T v[K][IPT];
#pragma unroll
    for (int c = 0; c < K; ++c) gr_load<T, IPT, VEC>(x.p[c] + base, cnt, v[c]);
    using A = typename Op::Acc;
    A yb[K];
#pragma unroll
    for (int c = 0; c < K; ++c) yb[c] = (A)*ybar.p[c];
    const S tpre = pre[blockIdx.x];
    const S tsuf = suf[blockIdx.x];
    S run = Op::id();
#pragma unroll
    for (int k = 0; k < IPT; ++k)
        if (k < cnt) run = Op::comb(run, gr_elem<Op, T, IPT>(v, k));
    S tot;
    const S tp = block_exclusive_scan<Op, kGrBlock, false>(run, tot, wtot);
    const S ts = block_exclusive_scan<Flip<Op>, kGrBlock, true>(run, tot, wtot);
    // in-thread suffixes: rs[k] = x_{k+1} (.) ... (.) x_{cnt-1} (.) R
    S rs[IPT];
    S s = Op::comb(ts, tsuf);
#pragma unroll
    for (int k = IPT - 1; k >= 0; --k) {
        rs[k] = s;
        if (k < cnt) s = Op::comb(gr_elem<Op, T, IPT>(v, k), s);
    }
    S l = Op::comb(tpre, tp);
    T out[K][IPT];
#pragma unroll
    for (int k = 0; k < IPT; ++k) {
        const S a = gr_elem<Op, T, IPT>(v, k);
        A o[K];
        Op::vjp(l, a, rs[k], yb, o);
#pragma unroll
        for (int c = 0; c < K; ++c) out[c][k] = (T)o[c];
        l = Op::comb(l, a);
    }
#pragma unroll
    for (int c = 0; c < K; ++c) {
        if (ACC) {
            T old[IPT];
            gr_load<T, IPT, VEC>(xbar.p[c] + base, cnt, old);
#pragma unroll
            for (int k = 0; k < IPT; ++k) out[c][k] += old[k];
        }
        gr_store<T, IPT, VEC>(xbar.p[c] + base, cnt, out[c]);
    }
}

// ------------------------------------------------------------------ host
static int gop_components(pvjp_gop op) {
    switch (op) {
        case PVJP_GOP_LOGADDEXP: return 1;
        case PVJP_GOP_LINREC: return 2;
        case PVJP_GOP_MAT2: return 4;
        default: return 0;
    }
}

template <class T>
static size_t gr_ws(int64_t n) {
    const int64_t nt = ceil_div(n, gr_tile<T>());
    return 3 * align_up((size_t)(nt > 0 ? nt : 1) * kGrSlot, 256);
}

template <class S>
static S* gr_slot(void* ws, int64_t n_tiles, int which) {
    return reinterpret_cast<S*>(reinterpret_cast<char*>(ws) +
                                (size_t)which * align_up((size_t)(n_tiles > 0 ? n_tiles : 1) * kGrSlot, 256));
}

template <class Op, class T>
static void launch_primal(const GPtrs<T>& x, int64_t n, const GOut<T>& y, void* ws, bool vec, hipStream_t st) {
    using S = typename Op::S;
    static_assert(sizeof(S) <= kGrSlot, "slot too small");
    const int64_t nt = ceil_div(n, gr_tile<T>());
    S* agg = gr_slot<S>(ws, nt, 0);
    if (nt > 0) {
        if (vec)
            hipLaunchKernelGGL((gred_tile_agg_kernel<Op, T, true>), dim3((unsigned)nt), dim3(kGrBlock), 0, st, x, n,
                               agg);
        else
            hipLaunchKernelGGL((gred_tile_agg_kernel<Op, T, false>), dim3((unsigned)nt), dim3(kGrBlock), 0, st, x, n,
                               agg);
    }
    hipLaunchKernelGGL((gred_agg_scan_kernel<Op, T>), dim3(1), dim3(kGrAggBlock), 0, st, (const S*)agg, nt,
                       (S*)nullptr, (S*)nullptr, y);
}

template <class Op, class T>
static void launch_vjp(const GPtrs<T>& x, int64_t n, const GPtrs<T>& yb, const GOut<T>& xb, int acc, void* ws,
                       bool vec, hipStream_t st) {
    using S = typename Op::S;
    const int64_t nt = ceil_div(n, gr_tile<T>());
    S* agg = gr_slot<S>(ws, nt, 0);
    S* pre = gr_slot<S>(ws, nt, 1);
    S* suf = gr_slot<S>(ws, nt, 2);
    const GOut<T> none{{nullptr, nullptr, nullptr, nullptr}};
    const dim3 g((unsigned)nt), b(kGrBlock);
    if (vec) {
        hipLaunchKernelGGL((gred_tile_agg_kernel<Op, T, true>), g, b, 0, st, x, n, agg);
    } else {
        hipLaunchKernelGGL((gred_tile_agg_kernel<Op, T, false>), g, b, 0, st, x, n, agg);
    }
    hipLaunchKernelGGL((gred_agg_scan_kernel<Op, T>), dim3(1), dim3(kGrAggBlock), 0, st, (const S*)agg, nt, pre,
                       suf, none);
    if (vec) {
        if (acc)
            hipLaunchKernelGGL((gred_vjp_kernel<Op, T, true, true>), g, b, 0, st, x, n, pre, suf, yb, xb);
        else
            hipLaunchKernelGGL((gred_vjp_kernel<Op, T, true, false>), g, b, 0, st, x, n, pre, suf, yb, xb);
    } else {
        if (acc)
            hipLaunchKernelGGL((gred_vjp_kernel<Op, T, false, true>), g, b, 0, st, x, n, pre, suf, yb, xb);
        else
            hipLaunchKernelGGL((gred_vjp_kernel<Op, T, false, false>), g, b, 0, st, x, n, pre, suf, yb, xb);
    }
}

// FP32 storage: the linear-recurrence and matrix folds run in FP64 (their
// rounding error grows with n otherwise: products of n factors); log-add-exp
// stays in FP32, where each step's error is relative to the running result.
template <template <class> class OpT, class T>
using GOpFor = OpT<typename std::conditional<std::is_same<T, float>::value &&
                                                 !std::is_same<OpT<float>, GLogAddExp<float>>::value,
                                             double, T>::type>;

template <template <class> class OpT, class T>
static void dispatch_primal(const void* const* x, int K, int64_t n, void* const* y, void* ws, hipStream_t st) {
    GPtrs<T> xp{};
    GOut<T> yp{};
    bool vec = true;
    for (int c = 0; c < K; ++c) {
        xp.p[c] = n > 0 ? (const T*)x[c] : nullptr;
        yp.p[c] = (T*)y[c];
        vec = vec && (n == 0 || aligned(x[c], 16));
    }
    launch_primal<GOpFor<OpT, T>, T>(xp, n, yp, ws, vec, st);
}

template <template <class> class OpT, class T>
static void dispatch_vjp(const void* const* x, int K, int64_t n, const void* const* yb, void* const* xb, int acc,
                         void* ws, hipStream_t st) {
    GPtrs<T> xp{}, yp{};
    GOut<T> xo{};
    bool vec = true;
    for (int c = 0; c < K; ++c) {
        xp.p[c] = (const T*)x[c];
        yp.p[c] = (const T*)yb[c];
        xo.p[c] = (T*)xb[c];
        vec = vec && aligned(x[c], 16) && aligned(xb[c], 16);
    }
    launch_vjp<GOpFor<OpT, T>, T>(xp, n, yp, xo, acc, ws, vec, st);
}

}  // namespace pvjp

using namespace pvjp;

extern "C" int pvjp_gop_components(pvjp_gop op) { return gop_components(op); }

extern "C" size_t pvjp_reduce_generic_ws_bytes(pvjp_gop op, pvjp_dtype dtype, int64_t n) {
    if (gop_components(op) == 0 || !valid_dtype(dtype) || n < 0) return 0;
    return dtype == PVJP_F64 ? gr_ws<double>(n) : gr_ws<float>(n);
}

static pvjp_status check_common(const char* name, pvjp_gop op, pvjp_dtype dtype, const void* const* x, int64_t n,
                                void* ws, size_t ws_bytes) {
    const int K = gop_components(op);
    PVJP_REQUIRE(K > 0, "%s: unknown operator %d", name, (int)op);
    PVJP_REQUIRE(valid_dtype(dtype), "%s: unknown dtype %d", name, (int)dtype);
    PVJP_REQUIRE(n >= 0, "%s: negative n", name);
    PVJP_REQUIRE(n < ((int64_t)1 << 40), "%s: n too large", name);
    PVJP_REQUIRE(ws != nullptr && aligned(ws, 256), "%s: workspace must be non-NULL and 256-byte aligned", name);
    if (ws_bytes < pvjp_reduce_generic_ws_bytes(op, dtype, n)) {
        set_error("%s: workspace of %zu bytes, need %zu", name, ws_bytes, pvjp_reduce_generic_ws_bytes(op, dtype, n));
        return PVJP_ENOMEM;
    }
    if (n > 0) {
        PVJP_REQUIRE(x != nullptr, "%s: x is NULL", name);
        for (int c = 0; c < K; ++c) {
            PVJP_REQUIRE(x[c] != nullptr, "%s: component %d of x is NULL", name, c);
            PVJP_REQUIRE(aligned(x[c], dsize(dtype)), "%s: component %d of x is misaligned", name, c);
        }
    }
    return PVJP_OK;
}

extern "C" pvjp_status pvjp_reduce_generic(pvjp_gop op, pvjp_dtype dtype, const void* const* x, int64_t n,
                                           void* const* y, void* ws, size_t ws_bytes, void* stream) {
    clear_error();
    const pvjp_status s = check_common("pvjp_reduce_generic", op, dtype, x, n, ws, ws_bytes);
    if (s != PVJP_OK) return s;
    const int K = gop_components(op);
    PVJP_REQUIRE(y != nullptr, "pvjp_reduce_generic: y is NULL");
    for (int c = 0; c < K; ++c) PVJP_REQUIRE(y[c] != nullptr, "pvjp_reduce_generic: component %d of y is NULL", c);
    const hipStream_t st = as_stream(stream);
    const void* none[4] = {nullptr, nullptr, nullptr, nullptr};
    const void* const* xx = n > 0 ? x : none;
    if (dtype == PVJP_F64) {
        if (op == PVJP_GOP_LOGADDEXP) dispatch_primal<GLogAddExp, double>(xx, K, n, y, ws, st);
        else if (op == PVJP_GOP_LINREC) dispatch_primal<GLinRec, double>(xx, K, n, y, ws, st);
        else dispatch_primal<GMat2, double>(xx, K, n, y, ws, st);
    } else {
        if (op == PVJP_GOP_LOGADDEXP) dispatch_primal<GLogAddExp, float>(xx, K, n, y, ws, st);
        else if (op == PVJP_GOP_LINREC) dispatch_primal<GLinRec, float>(xx, K, n, y, ws, st);
        else dispatch_primal<GMat2, float>(xx, K, n, y, ws, st);
    }
    PVJP_LAUNCHED("pvjp_reduce_generic");
    return PVJP_OK;
}

extern "C" pvjp_status pvjp_reduce_generic_vjp(pvjp_gop op, pvjp_dtype dtype, const void* const* x, int64_t n,
                                               const void* const* y_bar, void* const* x_bar, int accumulate,
                                               void* ws, size_t ws_bytes, void* stream) {
    clear_error();
    const pvjp_status s = check_common("pvjp_reduce_generic_vjp", op, dtype, x, n, ws, ws_bytes);
    if (s != PVJP_OK) return s;
    if (n == 0) return PVJP_OK;
    const int K = gop_components(op);
    PVJP_REQUIRE(y_bar != nullptr && x_bar != nullptr, "pvjp_reduce_generic_vjp: y_bar and x_bar must be non-NULL");
    for (int c = 0; c < K; ++c) {
        PVJP_REQUIRE(y_bar[c] != nullptr, "pvjp_reduce_generic_vjp: component %d of y_bar is NULL", c);
        PVJP_REQUIRE(x_bar[c] != nullptr, "pvjp_reduce_generic_vjp: component %d of x_bar is NULL", c);
        PVJP_REQUIRE(aligned(x_bar[c], dsize(dtype)), "pvjp_reduce_generic_vjp: component %d of x_bar is misaligned",
                     c);
    }
    const hipStream_t st = as_stream(stream);
    if (dtype == PVJP_F64) {
        if (op == PVJP_GOP_LOGADDEXP) dispatch_vjp<GLogAddExp, double>(x, K, n, y_bar, x_bar, accumulate, ws, st);
        else if (op == PVJP_GOP_LINREC) dispatch_vjp<GLinRec, double>(x, K, n, y_bar, x_bar, accumulate, ws, st);
        else dispatch_vjp<GMat2, double>(x, K, n, y_bar, x_bar, accumulate, ws, st);
    } else {
        if (op == PVJP_GOP_LOGADDEXP) dispatch_vjp<GLogAddExp, float>(x, K, n, y_bar, x_bar, accumulate, ws, st);
        else if (op == PVJP_GOP_LINREC) dispatch_vjp<GLinRec, float>(x, K, n, y_bar, x_bar, accumulate, ws, st);
        else dispatch_vjp<GMat2, float>(x, K, n, y_bar, x_bar, accumulate, ws, st);
    }
    PVJP_LAUNCHED("pvjp_reduce_generic_vjp");
    return PVJP_OK;
}
