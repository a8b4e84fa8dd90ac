// reduce with a general associative operator and its VJP by the general rule
// of Sec. 5.1.1.  With ls_i = x_0 (.) ... (.) x_{i-1} and
// rs_i = x_{i+1} (.) ... (.) x_{n-1} (an exclusive scan and an exclusive
// reversed scan), x_bar_i (+)= (d(ls_i (.) x_i (.) rs_i) / dx_i)^T y_bar with
// ls_i and rs_i held constant: the function f mapped over (ls, xs, rs).
//
// The rule as stated costs two whole-array scans plus a map (at least five
// global accesses per element).  Here the scans are split over fixed tiles
// in three levels (tiles, groups of 64 tiles, all groups):
//   1. one block per tile folds it (read x); one wave per group folds the
//      group's tile folds;
//   2. one block scans the group folds forward and backward (and gives the
//      primal result y); one wave per group then gives each tile the fold of
//      everything before it and of everything after it;
//   3. per tile, the in-tile exclusive prefixes and suffixes are formed in
//      registers and LDS and f is applied at once (read x, write x_bar).
// x is read twice and x_bar written once; ls and rs never reach memory.
//
// Operators (an element has K components, each its own array):
//   log-add-exp   a (.) b = log(e^a + e^b), neutral -inf (K = 1), carried
//                 as (max, scaled sum) pairs;
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

// An operator provides: K input components; a state S (its shuffles come
// from GShfl) with elem() turning an element's components into a state and
// value() turning a state back into K result components; the neutral id();
// comb(x, y) = x (.) y with x earlier in index order; and the function f,
// vjp(l, a, r, la, yb, out): out = (d(l (.) a (.) r)/da)^T yb, where la is
// l (.) a (already formed by the caller for the next prefix).

// log-add-exp.  The state is (m, s) standing for m + log(s), the neutral
// element (-inf, 0): combining costs one exp and no log, and exp(a - y)
// becomes exp(a - m_y) / s_y.  Each element is (x, 1), or the neutral
// element when x = -inf.
// exp and division for log-add-exp: in FP32 the hardware exp2 (about 1 ulp
// plus |x| * 2^-24 relative, x <= 0 here) and reciprocal; FP64 uses the
// library functions.
__device__ __forceinline__ float lae_exp(float x) { return __expf(x); }
__device__ __forceinline__ double lae_exp(double x) { return exp(x); }
__device__ __forceinline__ float lae_div(float a, float b) { return __fdividef(a, b); }
__device__ __forceinline__ double lae_div(double a, double b) { return a / b; }

template <class T>
struct GLogAddExp : GShfl<T, 2> {
    static constexpr int K = 1;
    using Acc = T;
    using S = GS<T, 2>;
    __device__ static __forceinline__ S id() { return S{{-(T)INFINITY, T(0)}}; }
    __device__ static __forceinline__ S elem(const T (&c)[1]) {
        return S{{c[0], c[0] == -(T)INFINITY ? T(0) : T(1)}};
    }
    __device__ static __forceinline__ void value(S v, T (&out)[1]) { out[0] = v.c[0] + log(v.c[1]); }
    __device__ static __forceinline__ S comb(S x, S y) {
        if (y.c[1] == T(0)) return x;
        if (x.c[1] == T(0)) return y;
        const T d = x.c[0] - y.c[0];
        const T e = lae_exp(-fabs(d));
        return d >= T(0) ? S{{x.c[0], x.c[1] + y.c[1] * e}} : S{{y.c[0], x.c[1] * e + y.c[1]}};
    }
    __device__ static __forceinline__ void vjp(S, S a, S r, S la, const T (&yb)[1], T (&out)[1]) {
        // d/da log(e^l + e^a + e^r) = e^(a - y); a -inf element receives 0
        if (a.c[1] == T(0)) {
            out[0] = T(0);
            return;
        }
        const S y = comb(la, r);
        out[0] = lae_div(yb[0] * lae_exp(a.c[0] - y.c[0]), y.c[1]);
    }
};

template <class T>
struct GLinRec : GShfl<T, 2> {
    static constexpr int K = 2;
    using Acc = T;
    using S = GS<T, 2>;
    __device__ static __forceinline__ S id() { return S{{T(1), T(0)}}; }
    __device__ static __forceinline__ S elem(const T (&c)[2]) { return S{{c[0], c[1]}}; }
    __device__ static __forceinline__ void value(S v, T (&out)[2]) { out[0] = v.c[0], out[1] = v.c[1]; }
    __device__ static __forceinline__ S comb(S x, S y) { return S{{y.c[0] * x.c[0], y.c[0] * x.c[1] + y.c[1]}}; }
    __device__ static __forceinline__ void vjp(S l, S, S r, S, const T (&yb)[2], T (&out)[2]) {
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
    __device__ static __forceinline__ S elem(const T (&c)[4]) { return S{{c[0], c[1], c[2], c[3]}}; }
    __device__ static __forceinline__ void value(S v, T (&out)[4]) {
        for (int c = 0; c < 4; ++c) out[c] = v.c[c];
    }
    __device__ static __forceinline__ S comb(S x, S y) {
        return S{{x.c[0] * y.c[0] + x.c[1] * y.c[2], x.c[0] * y.c[1] + x.c[1] * y.c[3],
                  x.c[2] * y.c[0] + x.c[3] * y.c[2], x.c[2] * y.c[1] + x.c[3] * y.c[3]}};
    }
    __device__ static __forceinline__ void vjp(S l, S, S r, S, const T (&yb)[4], T (&out)[4]) {
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

// Items per thread: 32 bytes of every component (two 16-byte loads), fewer
// where the operator state is large (at most 128 bytes of states per thread
// for the in-thread suffixes), so that occupancy stays up.
template <class Op, class T>
constexpr int gr_ipt() {
    return (32 / (int)sizeof(T)) < (128 / (int)sizeof(typename Op::S)) ? 32 / (int)sizeof(T)
                                                                        : 128 / (int)sizeof(typename Op::S);
}
template <class Op, class T>
constexpr int gr_tile() {
    return kGrBlock * gr_ipt<Op, T>();
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
    typename Op::Acc c[Op::K];
#pragma unroll
    for (int j = 0; j < Op::K; ++j) c[j] = (typename Op::Acc)v[j][k];
    return Op::elem(c);
}

template <int IPT>
__device__ __forceinline__ int gr_cnt(int64_t n, int64_t base) {
    const int64_t left = n - base;
    return left <= 0 ? 0 : (left >= IPT ? IPT : (int)left);
}

// Pass 1: agg[t] = fold of tile t in index order.
template <class Op, class T, bool VEC>
__global__ __launch_bounds__(kGrBlock) void gred_tile_agg_kernel(GPtrs<T> x, int64_t n,
                                                                 typename Op::S* __restrict__ agg) {
    using S = typename Op::S;
    constexpr int IPT = gr_ipt<Op, T>();
    __shared__ S wtot[kGrBlock / kWave];
    const int64_t base = (int64_t)blockIdx.x * gr_tile<Op, T>() + (int64_t)threadIdx.x * IPT;
    const int cnt = gr_cnt<IPT>(n, base);
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

// Tiles are taken in groups of kGrGroup; one wave handles a group, lane j
// its tile j.
constexpr int kGrGroup = kWave;

// Pass 1b: gagg[g] = fold of the tile folds of group g.
template <class Op>
__global__ __launch_bounds__(kGrBlock) void gred_group_fold_kernel(const typename Op::S* __restrict__ agg, int64_t nt,
                                                                   int64_t ng, typename Op::S* __restrict__ gagg) {
    using S = typename Op::S;
    const int64_t g = (int64_t)blockIdx.x * (kGrBlock / kWave) + threadIdx.x / kWave;
    if (g >= ng) return;  // whole waves leave together
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t t = g * kGrGroup + lane;
    const S own = t < nt ? agg[t] : Op::id();
    const S inc = Op::comb(wave_exclusive_scan<Op, false>(own), own);
    if (lane == kWave - 1) gagg[g] = inc;
}

// Pass 2 (one block): pre[g] = fold of the group folds before g, suf[g] =
// fold of those after g (either may be NULL); y (nullable components) =
// fold of all.  Thread j owns a contiguous run of the folds; runs are scanned
// across the block in both directions.
template <class Op, class T>
__global__ __launch_bounds__(kGrAggBlock) void gred_agg_scan_kernel(const typename Op::S* __restrict__ agg,
                                                                    int64_t nb, typename Op::S* __restrict__ pre,
                                                                    typename Op::S* __restrict__ suf, GOut<T> y) {
    using S = typename Op::S;
    __shared__ S wtot[kGrAggBlock / kWave];
    const int64_t per = (nb + kGrAggBlock - 1) / kGrAggBlock;
    const int64_t v0 = (int64_t)threadIdx.x * per < nb ? (int64_t)threadIdx.x * per : nb;
    const int64_t v1 = v0 + per < nb ? v0 + per : nb;
    S run = Op::id();
    for (int64_t v = v0; v < v1; ++v) run = Op::comb(run, agg[v]);
    S total;
    S ex = block_exclusive_scan<Op, kGrAggBlock, false>(run, total, wtot);
    if (threadIdx.x == 0) {
        typename Op::Acc yv[Op::K];
        Op::value(total, yv);
#pragma unroll
        for (int c = 0; c < Op::K; ++c)
            if (y.p[c]) *y.p[c] = (T)yv[c];
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

// Pass 2b: per tile t of group g, pre[t] = gpre[g] (.) the tiles of the
// group before t, suf[t] = the tiles of the group after t (.) gsuf[g].
template <class Op>
__global__ __launch_bounds__(kGrBlock) void gred_tile_prefix_kernel(const typename Op::S* __restrict__ agg,
                                                                    int64_t nt, int64_t ng,
                                                                    const typename Op::S* __restrict__ gpre,
                                                                    const typename Op::S* __restrict__ gsuf,
                                                                    typename Op::S* __restrict__ pre,
                                                                    typename Op::S* __restrict__ suf) {
    using S = typename Op::S;
    const int64_t g = (int64_t)blockIdx.x * (kGrBlock / kWave) + threadIdx.x / kWave;
    if (g >= ng) return;  // whole waves leave together
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t t = g * kGrGroup + lane;
    const S own = t < nt ? agg[t] : Op::id();
    const S exf = wave_exclusive_scan<Op, false>(own);
    const S exb = wave_exclusive_scan<Flip<Op>, true>(own);
    if (t < nt) {
        pre[t] = Op::comb(gpre[g], exf);
        suf[t] = Op::comb(exb, gsuf[g]);
    }
}

// Pass 3: per tile, ls_i and rs_i from the tile's prefix and suffix, the
// block scans of the threads' runs and the in-thread folds; then
// x_bar_i (+)= f(ls_i, x_i, rs_i).
template <class Op, class T, bool VEC, bool ACC>
__global__ __launch_bounds__(kGrBlock) void gred_vjp_kernel(GPtrs<T> x, int64_t n,
                                                            const typename Op::S* __restrict__ pre,
                                                            const typename Op::S* __restrict__ suf, GPtrs<T> ybar,
                                                            GOut<T> xbar) {
    using S = typename Op::S;
    using A = typename Op::Acc;
    constexpr int K = Op::K;
    constexpr int IPT = gr_ipt<Op, T>();
    __shared__ S wtot[kGrBlock / kWave];
    const int64_t base = (int64_t)blockIdx.x * gr_tile<Op, T>() + (int64_t)threadIdx.x * IPT;
    const int cnt = gr_cnt<IPT>(n, base);
    T v[K][IPT];
#pragma unroll
    for (int c = 0; c < K; ++c) gr_load<T, IPT, VEC>(x.p[c] + base, cnt, v[c]);
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
        const S la = Op::comb(l, a);
        A o[K];
        Op::vjp(l, a, rs[k], la, yb, o);
#pragma unroll
        for (int c = 0; c < K; ++c) out[c][k] = (T)o[c];
        l = la;
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

// Workspace: [tile folds | tile prefixes | tile suffixes] (nt each), then
// [group folds | group prefixes | group suffixes] (ng each), one 32-byte
// slot per state, every array 256-byte aligned.
struct GrPlan {
    int64_t nt, ng;
    size_t tiles, groups;  // bytes of one per-tile / per-group array
};

template <class Op, class T>
static GrPlan gr_plan(int64_t n) {
    GrPlan p;
    p.nt = ceil_div(n, gr_tile<Op, T>());
    p.ng = ceil_div(p.nt, kGrGroup);
    p.tiles = align_up((size_t)(p.nt > 0 ? p.nt : 1) * kGrSlot, 256);
    p.groups = align_up((size_t)(p.ng > 0 ? p.ng : 1) * kGrSlot, 256);
    return p;
}

template <class Op, class T>
static size_t gr_ws(int64_t n) {
    const GrPlan p = gr_plan<Op, T>(n);
    return 3 * p.tiles + 3 * p.groups;
}

template <class S>
static S* gr_array(void* ws, const GrPlan& p, int which) {
    const size_t off = which < 3 ? which * p.tiles : 3 * p.tiles + (which - 3) * p.groups;
    return reinterpret_cast<S*>(reinterpret_cast<char*>(ws) + off);
}

// tile folds (pass 1) and group folds (pass 1b)
template <class Op, class T>
static void launch_folds(const GPtrs<T>& x, int64_t n, const GrPlan& p, typename Op::S* agg,
                         typename Op::S* gagg, bool vec, hipStream_t st) {
    using S = typename Op::S;
    if (p.nt == 0) return;
    if (vec)
        hipLaunchKernelGGL((gred_tile_agg_kernel<Op, T, true>), dim3((unsigned)p.nt), dim3(kGrBlock), 0, st, x, n,
                           agg);
    else
        hipLaunchKernelGGL((gred_tile_agg_kernel<Op, T, false>), dim3((unsigned)p.nt), dim3(kGrBlock), 0, st, x, n,
                           agg);
    const unsigned gblocks = (unsigned)ceil_div(p.ng, kGrBlock / kWave);
    hipLaunchKernelGGL((gred_group_fold_kernel<Op>), dim3(gblocks), dim3(kGrBlock), 0, st, (const S*)agg, p.nt, p.ng,
                       gagg);
}

// The tile folds go to the caller's checkpoint when one is given (the VJP
// then starts from them instead of folding x again), else to the workspace.
template <class Op, class T>
static void launch_primal(const GPtrs<T>& x, int64_t n, const GOut<T>& y, void* ckpt, void* ws, bool vec,
                          hipStream_t st) {
    using S = typename Op::S;
    static_assert(sizeof(S) <= kGrSlot, "slot too small");
    const GrPlan p = gr_plan<Op, T>(n);
    S* gagg = gr_array<S>(ws, p, 3);
    S* agg = ckpt ? reinterpret_cast<S*>(ckpt) : gr_array<S>(ws, p, 0);
    launch_folds<Op, T>(x, n, p, agg, gagg, vec, st);
    hipLaunchKernelGGL((gred_agg_scan_kernel<Op, T>), dim3(1), dim3(kGrAggBlock), 0, st, (const S*)gagg, p.ng,
                       (S*)nullptr, (S*)nullptr, y);
}

template <class Op, class T>
static void launch_vjp(const GPtrs<T>& x, int64_t n, const void* ckpt, const GPtrs<T>& yb, const GOut<T>& xb, int acc,
                       void* ws, bool vec, hipStream_t st) {
    using S = typename Op::S;
    const GrPlan p = gr_plan<Op, T>(n);
    S* pre = gr_array<S>(ws, p, 1);
    S* suf = gr_array<S>(ws, p, 2);
    S* gagg = gr_array<S>(ws, p, 3);
    S* gpre = gr_array<S>(ws, p, 4);
    S* gsuf = gr_array<S>(ws, p, 5);
    const GOut<T> none{{nullptr, nullptr, nullptr, nullptr}};
    const unsigned gblocks = (unsigned)ceil_div(p.ng, kGrBlock / kWave);
    const S* agg;
    if (ckpt) {
        agg = reinterpret_cast<const S*>(ckpt);
        hipLaunchKernelGGL((gred_group_fold_kernel<Op>), dim3(gblocks), dim3(kGrBlock), 0, st, agg, p.nt, p.ng,
                           gagg);
    } else {
        S* a = gr_array<S>(ws, p, 0);
        launch_folds<Op, T>(x, n, p, a, gagg, vec, st);
        agg = a;
    }
    hipLaunchKernelGGL((gred_agg_scan_kernel<Op, T>), dim3(1), dim3(kGrAggBlock), 0, st, (const S*)gagg, p.ng, gpre,
                       gsuf, none);
    hipLaunchKernelGGL((gred_tile_prefix_kernel<Op>), dim3(gblocks), dim3(kGrBlock), 0, st, agg, p.nt, p.ng,
                       (const S*)gpre, (const S*)gsuf, pre, suf);
    const dim3 gt((unsigned)p.nt), b(kGrBlock);
    const S* cp = pre;
    const S* cs = suf;
    if (vec) {
        if (acc)
            hipLaunchKernelGGL((gred_vjp_kernel<Op, T, true, true>), gt, b, 0, st, x, n, cp, cs, yb, xb);
        else
            hipLaunchKernelGGL((gred_vjp_kernel<Op, T, true, false>), gt, b, 0, st, x, n, cp, cs, yb, xb);
    } else {
        if (acc)
            hipLaunchKernelGGL((gred_vjp_kernel<Op, T, false, true>), gt, b, 0, st, x, n, cp, cs, yb, xb);
        else
            hipLaunchKernelGGL((gred_vjp_kernel<Op, T, false, false>), gt, b, 0, st, x, n, cp, cs, yb, xb);
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
static void dispatch_primal(const void* const* x, int K, int64_t n, void* const* y, void* ckpt, void* ws,
                            hipStream_t st) {
    GPtrs<T> xp{};
    GOut<T> yp{};
    bool vec = true;
    for (int c = 0; c < K; ++c) {
        xp.p[c] = n > 0 ? (const T*)x[c] : nullptr;
        yp.p[c] = (T*)y[c];
        vec = vec && (n == 0 || aligned(x[c], 16));
    }
    launch_primal<GOpFor<OpT, T>, T>(xp, n, yp, ckpt, ws, vec, st);
}

template <template <class> class OpT, class T>
static void dispatch_vjp(const void* const* x, int K, int64_t n, const void* ckpt, const void* const* yb,
                         void* const* xb, int acc, void* ws, hipStream_t st) {
    GPtrs<T> xp{}, yp{};
    GOut<T> xo{};
    bool vec = true;
    for (int c = 0; c < K; ++c) {
        xp.p[c] = (const T*)x[c];
        yp.p[c] = (const T*)yb[c];
        xo.p[c] = (T*)xb[c];
        vec = vec && aligned(x[c], 16) && aligned(xb[c], 16);
    }
    launch_vjp<GOpFor<OpT, T>, T>(xp, n, ckpt, yp, xo, acc, ws, vec, st);
}

}  // namespace pvjp

using namespace pvjp;

extern "C" int pvjp_gop_components(pvjp_gop op) { return gop_components(op); }

extern "C" size_t pvjp_reduce_generic_ws_bytes(pvjp_gop op, pvjp_dtype dtype, int64_t n) {
    if (gop_components(op) == 0 || !valid_dtype(dtype) || n < 0) return 0;
    if (dtype == PVJP_F64) {
        if (op == PVJP_GOP_LOGADDEXP) return gr_ws<GOpFor<GLogAddExp, double>, double>(n);
        if (op == PVJP_GOP_LINREC) return gr_ws<GOpFor<GLinRec, double>, double>(n);
        return gr_ws<GOpFor<GMat2, double>, double>(n);
    }
    if (op == PVJP_GOP_LOGADDEXP) return gr_ws<GOpFor<GLogAddExp, float>, float>(n);
    if (op == PVJP_GOP_LINREC) return gr_ws<GOpFor<GLinRec, float>, float>(n);
    return gr_ws<GOpFor<GMat2, float>, float>(n);
}

extern "C" size_t pvjp_reduce_generic_ckpt_bytes(pvjp_gop op, pvjp_dtype dtype, int64_t n) {
    if (gop_components(op) == 0 || !valid_dtype(dtype) || n < 0) return 0;
    int64_t nt;
    if (dtype == PVJP_F64) {
        if (op == PVJP_GOP_LOGADDEXP) nt = gr_plan<GOpFor<GLogAddExp, double>, double>(n).nt;
        else if (op == PVJP_GOP_LINREC) nt = gr_plan<GOpFor<GLinRec, double>, double>(n).nt;
        else nt = gr_plan<GOpFor<GMat2, double>, double>(n).nt;
    } else {
        if (op == PVJP_GOP_LOGADDEXP) nt = gr_plan<GOpFor<GLogAddExp, float>, float>(n).nt;
        else if (op == PVJP_GOP_LINREC) nt = gr_plan<GOpFor<GLinRec, float>, float>(n).nt;
        else nt = gr_plan<GOpFor<GMat2, float>, float>(n).nt;
    }
    return (size_t)nt * kGrSlot;
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
                                           void* const* y, void* ckpt, void* ws, size_t ws_bytes, void* stream) {
    clear_error();
    const pvjp_status s = check_common("pvjp_reduce_generic", op, dtype, x, n, ws, ws_bytes);
    if (s != PVJP_OK) return s;
    PVJP_REQUIRE(ckpt == nullptr || aligned(ckpt, 16), "pvjp_reduce_generic: ckpt must be 16-byte aligned");
    const int K = gop_components(op);
    PVJP_REQUIRE(y != nullptr, "pvjp_reduce_generic: y is NULL");
    for (int c = 0; c < K; ++c) PVJP_REQUIRE(y[c] != nullptr, "pvjp_reduce_generic: component %d of y is NULL", c);
    const hipStream_t st = as_stream(stream);
    const void* none[4] = {nullptr, nullptr, nullptr, nullptr};
    const void* const* xx = n > 0 ? x : none;
    if (dtype == PVJP_F64) {
        if (op == PVJP_GOP_LOGADDEXP) dispatch_primal<GLogAddExp, double>(xx, K, n, y, ckpt, ws, st);
        else if (op == PVJP_GOP_LINREC) dispatch_primal<GLinRec, double>(xx, K, n, y, ckpt, ws, st);
        else dispatch_primal<GMat2, double>(xx, K, n, y, ckpt, ws, st);
    } else {
        if (op == PVJP_GOP_LOGADDEXP) dispatch_primal<GLogAddExp, float>(xx, K, n, y, ckpt, ws, st);
        else if (op == PVJP_GOP_LINREC) dispatch_primal<GLinRec, float>(xx, K, n, y, ckpt, ws, st);
        else dispatch_primal<GMat2, float>(xx, K, n, y, ckpt, ws, st);
    }
    PVJP_LAUNCHED("pvjp_reduce_generic");
    return PVJP_OK;
}

extern "C" pvjp_status pvjp_reduce_generic_vjp(pvjp_gop op, pvjp_dtype dtype, const void* const* x, int64_t n,
                                               const void* ckpt, const void* const* y_bar, void* const* x_bar,
                                               int accumulate, void* ws, size_t ws_bytes, void* stream) {
    clear_error();
    const pvjp_status s = check_common("pvjp_reduce_generic_vjp", op, dtype, x, n, ws, ws_bytes);
    if (s != PVJP_OK) return s;
    PVJP_REQUIRE(ckpt == nullptr || aligned(ckpt, 16), "pvjp_reduce_generic_vjp: ckpt must be 16-byte aligned");
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
        if (op == PVJP_GOP_LOGADDEXP) dispatch_vjp<GLogAddExp, double>(x, K, n, ckpt, y_bar, x_bar, accumulate, ws, st);
        else if (op == PVJP_GOP_LINREC) dispatch_vjp<GLinRec, double>(x, K, n, ckpt, y_bar, x_bar, accumulate, ws, st);
        else dispatch_vjp<GMat2, double>(x, K, n, ckpt, y_bar, x_bar, accumulate, ws, st);
    } else {
        if (op == PVJP_GOP_LOGADDEXP) dispatch_vjp<GLogAddExp, float>(x, K, n, ckpt, y_bar, x_bar, accumulate, ws, st);
        else if (op == PVJP_GOP_LINREC) dispatch_vjp<GLinRec, float>(x, K, n, ckpt, y_bar, x_bar, accumulate, ws, st);
        else dispatch_vjp<GMat2, float>(x, K, n, ckpt, y_bar, x_bar, accumulate, ws, st);
    }
    PVJP_LAUNCHED("pvjp_reduce_generic_vjp");
    return PVJP_OK;
}
