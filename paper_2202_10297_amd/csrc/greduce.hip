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
#include "gops.h"
#include "prims.h"

namespace pvjp {

constexpr int kGrBlock = 256;
constexpr int kGrAggBlock = 1024;
constexpr size_t kGrSlot = 32;  // bytes per tile for an aggregate, prefix or suffix
// Slot of a state: 32 bytes, 64 for the dual 2x2 matrix state in FP64.
template <class S>
constexpr size_t slot_of() {
    return sizeof(S) <= 32 ? 32 : 64;
}

// ------------------------------------------------------------ forward mode
// Dual numbers over an operator (forward mode, Sec. 3: each primal bundled
// with its tangent): an element is (x, x_dot), 2K components (the K primal
// ones, then the K tangents), and (x, xd) (.) (y, yd) = (x (.) y,
// d1(x, y) xd + d2(x, y) yd).  A reduce or scan with the dual operator
// gives the primal result and its tangent in one pass.

// log-add-exp: state (m, s, t) with value m + log s and tangent t / s (t is
// the tangent sum weighted like s: t = sum e^(x_j - m) x_dot_j).
template <class T>
struct GLaeDual : GShfl<T, 3> {
    static constexpr int K = 2;
    using Acc = T;
    using S = GS<T, 3>;
    __device__ static __forceinline__ S id() { return S{{-(T)INFINITY, T(0), T(0)}}; }
    __device__ static __forceinline__ S elem(const T (&c)[2]) {
        const bool ninf = c[0] == -(T)INFINITY;
        return S{{c[0], ninf ? T(0) : T(1), ninf ? T(0) : c[1]}};
    }
    __device__ static __forceinline__ void value(S v, T (&out)[2]) {
        out[0] = v.c[0] + log(v.c[1]);
        out[1] = v.c[1] == T(0) ? T(0) : v.c[2] / v.c[1];
    }
    __device__ static __forceinline__ S comb(S x, S y) {
        if (y.c[1] == T(0)) return x;
        if (x.c[1] == T(0)) return y;
        const T d = x.c[0] - y.c[0];
        const T e = lae_exp(-fabs(d));
        return d >= T(0) ? S{{x.c[0], x.c[1] + y.c[1] * e, x.c[2] + y.c[2] * e}}
                         : S{{y.c[0], x.c[1] * e + y.c[1], x.c[2] * e + y.c[2]}};
    }
};

// linear recurrence: (A, B, A_dot, B_dot); (later) o (earlier) by the
// product rule.
template <class T>
struct GLinRecDual : GShfl<T, 4> {
    static constexpr int K = 4;
    using Acc = T;
    using S = GS<T, 4>;
    __device__ static __forceinline__ S id() { return S{{T(1), T(0), T(0), T(0)}}; }
    __device__ static __forceinline__ S elem(const T (&c)[4]) { return S{{c[0], c[1], c[2], c[3]}}; }
    __device__ static __forceinline__ void value(S v, T (&out)[4]) {
        for (int c = 0; c < 4; ++c) out[c] = v.c[c];
    }
    __device__ static __forceinline__ S comb(S x, S y) {
        return S{{y.c[0] * x.c[0], y.c[0] * x.c[1] + y.c[1], y.c[2] * x.c[0] + y.c[0] * x.c[2],
                  y.c[2] * x.c[1] + y.c[0] * x.c[3] + y.c[3]}};
    }
};

// 2x2 matrix product: (X, X_dot) (.) (Y, Y_dot) = (X Y, X_dot Y + X Y_dot).
template <class T>
struct GMat2Dual : GShfl<T, 8> {
    static constexpr int K = 8;
    using Acc = T;
    using S = GS<T, 8>;
    __device__ static __forceinline__ S id() { return S{{T(1), T(0), T(0), T(1), T(0), T(0), T(0), T(0)}}; }
    __device__ static __forceinline__ S elem(const T (&c)[8]) {
        S s;
        for (int j = 0; j < 8; ++j) s.c[j] = c[j];
        return s;
    }
    __device__ static __forceinline__ void value(S v, T (&out)[8]) {
        for (int c = 0; c < 8; ++c) out[c] = v.c[c];
    }
    __device__ static __forceinline__ void mm(const T* a, const T* b, T* o, bool add) {
        const T r0 = a[0] * b[0] + a[1] * b[2], r1 = a[0] * b[1] + a[1] * b[3];
        const T r2 = a[2] * b[0] + a[3] * b[2], r3 = a[2] * b[1] + a[3] * b[3];
        if (add) o[0] += r0, o[1] += r1, o[2] += r2, o[3] += r3;
        else o[0] = r0, o[1] = r1, o[2] = r2, o[3] = r3;
    }
    __device__ static __forceinline__ S comb(S x, S y) {
        S r;
        mm(x.c, y.c, r.c, false);
        mm(x.c + 4, y.c, r.c + 4, false);
        mm(x.c, y.c + 4, r.c + 4, true);
        return r;
    }
};

// lin_o of Sec. 5.2 with a d-vector and a general d x d matrix: the affine
// map r -> v + c r; (v1,c1) then (v2,c2) gives (v2 + c2 v1, c2 c1), neutral
// (0, I).  The reversed scan of the VJP folds the elements (y_bar_i,
// J_left(i)^T) from the last index down.
template <class A, int D>
struct LinG {
    struct S {
        A v[D];
        A c[D][D];
    };
    __device__ static __forceinline__ S id() {
        S r;
#pragma unroll
        for (int i = 0; i < D; ++i) {
            r.v[i] = A(0);
#pragma unroll
            for (int j = 0; j < D; ++j) r.c[i][j] = i == j ? A(1) : A(0);
        }
        return r;
    }
    __device__ static __forceinline__ S comb(const S& x, const S& y) {
        S r;
#pragma unroll
        for (int i = 0; i < D; ++i) {
            A v = y.v[i];
#pragma unroll
            for (int j = 0; j < D; ++j) v += y.c[i][j] * x.v[j];
            r.v[i] = v;
#pragma unroll
            for (int k = 0; k < D; ++k) {
                A c = A(0);
#pragma unroll
                for (int j = 0; j < D; ++j) c += y.c[i][j] * x.c[j][k];
                r.c[i][k] = c;
            }
        }
        return r;
    }
    template <class F>
    __device__ static __forceinline__ S map(const S& v, F f) {
        S r;
#pragma unroll
        for (int i = 0; i < D; ++i) {
            r.v[i] = f(v.v[i]);
#pragma unroll
            for (int j = 0; j < D; ++j) r.c[i][j] = f(v.c[i][j]);
        }
        return r;
    }
    __device__ static __forceinline__ S up(S v, int d) {
        return map(v, [d](A a) { return shfl_up1(a, d); });
    }
    __device__ static __forceinline__ S down(S v, int d) {
        return map(v, [d](A a) { return shfl_down1(a, d); });
    }
    __device__ static __forceinline__ S idx(S v, int s) {
        return map(v, [s](A a) { return shfl_idx1(a, s); });
    }
};

// lin_o states of the scan VJP per operator.  The general form keeps J_left^T
// as a dense d x d matrix (LinG).  For the 2 x 2 matrix product J_left^T = I
// (x) X_next (the same 2 x 2 block on the diagonal twice), and lin_o
// compositions keep that form, (I (x) M2)(I (x) M1) = I (x) M2 M1, so the state
// is (v[4], M[2][2]): a 2 x 2 product per composition instead of a 4 x 4 one,
// with the same values (the dense form only adds exact zeros).
template <class A>
struct LinKron {
    struct S {
        A v[4];
        A m[2][2];
    };
    __device__ static __forceinline__ S id() { return S{{A(0), A(0), A(0), A(0)}, {{A(1), A(0)}, {A(0), A(1)}}}; }
    // x first, then y: (y.v + (I (x) y.m) x.v, y.m x.m)
    __device__ static __forceinline__ S comb(const S& x, const S& y) {
        S r;
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int a = 0; a < 2; ++a)
                r.v[2 * b + a] = y.v[2 * b + a] + y.m[a][0] * x.v[2 * b] + y.m[a][1] * x.v[2 * b + 1];
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int c = 0; c < 2; ++c) r.m[a][c] = y.m[a][0] * x.m[0][c] + y.m[a][1] * x.m[1][c];
        return r;
    }
    template <class F>
    __device__ static __forceinline__ S map(const S& v, F f) {
        S r;
#pragma unroll
        for (int i = 0; i < 4; ++i) r.v[i] = f(v.v[i]);
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int c = 0; c < 2; ++c) r.m[a][c] = f(v.m[a][c]);
        return r;
    }
    __device__ static __forceinline__ S up(S v, int d) {
        return map(v, [d](A a) { return shfl_up1(a, d); });
    }
    __device__ static __forceinline__ S down(S v, int d) {
        return map(v, [d](A a) { return shfl_down1(a, d); });
    }
    __device__ static __forceinline__ S idx(S v, int s) {
        return map(v, [s](A a) { return shfl_idx1(a, s); });
    }
};

// The lin_o element of position k, (y_bar_k, J_left(k)^T) with the next
// element nx (a zero matrix where nothing follows), and one step of the
// reversed recurrence r_k = y_bar_k + J_left(k)^T r_(k+1).
template <class Op>
struct LinOf {
    using A = typename Op::Acc;
    static constexpr int K = Op::K;
    using L = LinG<A, K>;
    __device__ static __forceinline__ typename L::S elem(const typename Op::S& y, const A (&nx)[K], bool has_next,
                                                         const A (&yb)[K]) {
        typename L::S e;
        if (has_next) {
            Op::jlT(y, nx, e.c);
        } else {
#pragma unroll
            for (int i = 0; i < K; ++i)
#pragma unroll
                for (int j = 0; j < K; ++j) e.c[i][j] = A(0);
        }
#pragma unroll
        for (int c = 0; c < K; ++c) e.v[c] = yb[c];
        return e;
    }
    __device__ static __forceinline__ void step(const typename Op::S& y, const A (&nx)[K], bool has_next,
                                                const A (&yb)[K], const A (&r)[K], A (&rn)[K]) {
        const typename L::S e = elem(y, nx, has_next, yb);
#pragma unroll
        for (int i = 0; i < K; ++i) {
            A v = e.v[i];
#pragma unroll
            for (int j = 0; j < K; ++j) v += e.c[i][j] * r[j];
            rn[i] = v;
        }
    }
};

template <class A0>
struct LinOf<GMat2<A0>> {
    using A = A0;
    static constexpr int K = 4;
    using L = LinKron<A>;
    __device__ static __forceinline__ typename L::S elem(const typename GMat2<A>::S&, const A (&nx)[4], bool has_next,
                                                         const A (&yb)[4]) {
        typename L::S e;
#pragma unroll
        for (int c = 0; c < 4; ++c) e.v[c] = yb[c];
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int c = 0; c < 2; ++c) e.m[a][c] = has_next ? nx[2 * a + c] : A(0);
        return e;
    }
    __device__ static __forceinline__ void step(const typename GMat2<A>::S&, const A (&nx)[4], bool has_next,
                                                const A (&yb)[4], const A (&r)[4], A (&rn)[4]) {
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int a = 0; a < 2; ++a)
                rn[2 * b + a] = has_next ? yb[2 * b + a] + nx[2 * a] * r[2 * b] + nx[2 * a + 1] * r[2 * b + 1]
                                         : yb[2 * b + a];
    }
};


template <class T>
struct GPtrs {
    const T* p[8];
};
template <class T>
struct GOut {
    T* p[8];
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
    constexpr bool WHOLE = (IPT * sizeof(T)) % 16 == 0;  // the run is whole 16-byte pieces
    if (VEC && WHOLE && cnt == IPT) {
        constexpr int NV = WHOLE ? IPT * (int)sizeof(T) / 16 : 1;
        uint4 w[NV];
#pragma unroll
        for (int j = 0; j < NV; ++j) w[j] = reinterpret_cast<const uint4*>(p)[j];
        __builtin_memcpy(v, w, sizeof(v));
    } else {
#pragma unroll
        for (int k = 0; k < IPT; ++k) v[k] = (k < cnt) ? p[k] : T(0);
    }
}

template <class T, int IPT, bool VEC>
__device__ __forceinline__ void gr_store(T* __restrict__ p, int cnt, const T (&v)[IPT]) {
    constexpr bool WHOLE = (IPT * sizeof(T)) % 16 == 0;
    if (VEC && WHOLE && cnt == IPT) {
        constexpr int NV = WHOLE ? IPT * (int)sizeof(T) / 16 : 1;
        uint4 w[NV];
        __builtin_memcpy(w, v, sizeof(v));
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

// blockIdx.y selects one of several independent arrays of n elements laid
// out back to back (a regular segmented scan); its tiles' states sit at
// blockIdx.y * gridDim.x.  A 1-D grid is segment 0.
template <class T, int K>
__device__ __forceinline__ void seg_shift(GPtrs<T>& x, int64_t n) {
#pragma unroll
    for (int c = 0; c < K; ++c) x.p[c] += (int64_t)blockIdx.y * n;
}
template <class T, int K>
__device__ __forceinline__ void seg_shift(GOut<T>& x, int64_t n) {
#pragma unroll
    for (int c = 0; c < K; ++c) x.p[c] += (int64_t)blockIdx.y * n;
}
__device__ __forceinline__ int64_t seg_tile() { return (int64_t)blockIdx.y * gridDim.x + blockIdx.x; }

// Pass 1: agg[t] = fold of tile t (kGrBlock * IPT elements) in index order.
template <class Op, class T, bool VEC, int IPT = gr_ipt<Op, T>()>
__global__ __launch_bounds__(kGrBlock) void gred_tile_agg_kernel(GPtrs<T> x, int64_t n,
                                                                 typename Op::S* __restrict__ agg) {
    using S = typename Op::S;
    __shared__ S wtot[kGrBlock / kWave];
    seg_shift<T, Op::K>(x, n);
    const int64_t base = (int64_t)blockIdx.x * (kGrBlock * IPT) + (int64_t)threadIdx.x * IPT;
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
    if (threadIdx.x == 0) agg[seg_tile()] = total;
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

// ====================================================================
// Inclusive scan with a general operator and its VJP (Sec. 5.2 with the
// Jacobian generalisation): y_i = x_0 (.) ... (.) x_i.  With
// J_left(i) = d(y_i (.) x_{i+1})/dy_i and J_right(i) = d(y_{i-1} (.) x_i)/dx_i
// the return sweep is the reversed scan r_i = y_bar_i + J_left(i)^T r_{i+1}
// (lin_o over (d-vector, d x d matrix)), then x_bar_i = J_right(i)^T r_i.
// Primal values are not read back: every VJP pass recomputes them per tile
// from the per-tile prefix checkpoint.
//
// Items per thread: at most 32 bytes of each input component and 64 bytes
// of inputs in the arithmetic type (the per-element states and Jacobians
// live in registers); 128 bytes for the 2 x 2 matrix product, whose lin_o
// state is small in its Kronecker form.
template <class Op>
constexpr int gs_arith_budget() {
    return Op::K == 4 ? 128 : 64;
}
template <class Op, class T>
constexpr int gs_ipt() {
    return (32 / (int)sizeof(T)) < (gs_arith_budget<Op>() / (Op::K * (int)sizeof(typename Op::Acc)))
               ? 32 / (int)sizeof(T)
               : gs_arith_budget<Op>() / (Op::K * (int)sizeof(typename Op::Acc));
}
template <class Op, class T>
constexpr int gs_tile() {
    return kGrBlock * gs_ipt<Op, T>();
}

// A thread's run of IPT elements starting at `base` (cnt of them exist):
// the elements in the arithmetic type, the element right after the run (xn,
// if it exists), the state before the run (sp: the tile prefix folded with
// the block scan of the runs) and the inclusive states ys[k].
template <class Op, class T, int IPT, bool VEC>
__device__ __forceinline__ void gs_run_states(const GPtrs<T>& x, int64_t n, int64_t base, int cnt,
                                              const typename Op::S& tpre, typename Op::S* wtot,
                                              typename Op::Acc (&xa)[Op::K][IPT], typename Op::Acc (&xn)[Op::K],
                                              typename Op::S (&ys)[IPT], typename Op::S& sp) {
    using S = typename Op::S;
    using A = typename Op::Acc;
    constexpr int K = Op::K;
    T v[K][IPT];
#pragma unroll
    for (int c = 0; c < K; ++c) gr_load<T, IPT, VEC>(x.p[c] + base, cnt, v[c]);
    const bool edge = base + IPT < n;
#pragma unroll
    for (int c = 0; c < K; ++c) {
        xn[c] = edge ? (A)x.p[c][base + IPT] : A(0);
#pragma unroll
        for (int k = 0; k < IPT; ++k) xa[c][k] = (A)v[c][k];
    }
    S run = Op::id();
#pragma unroll
    for (int k = 0; k < IPT; ++k) {
        A e[K];
#pragma unroll
        for (int c = 0; c < K; ++c) e[c] = xa[c][k];
        if (k < cnt) run = Op::comb(run, Op::elem(e));
    }
    S tot;
    const S tp = block_exclusive_scan<Op, kGrBlock, false>(run, tot, wtot);
    sp = Op::comb(tpre, tp);
    S st = sp;
#pragma unroll
    for (int k = 0; k < IPT; ++k) {
        A e[K];
#pragma unroll
        for (int c = 0; c < K; ++c) e[c] = xa[c][k];
        if (k < cnt) st = Op::comb(st, Op::elem(e));
        ys[k] = st;
    }
}

// The element after position k of a run (the run's next element past its end).
template <class Op, int IPT>
__device__ __forceinline__ void gs_next(const typename Op::Acc (&xa)[Op::K][IPT], const typename Op::Acc (&xn)[Op::K],
                                        int k, typename Op::Acc (&nx)[Op::K]) {
#pragma unroll
    for (int c = 0; c < Op::K; ++c) nx[c] = k + 1 < IPT ? xa[c][k + 1 < IPT ? k + 1 : 0] : xn[c];
}

// Fold of a run's lin_o elements in reversed index order.
template <class Op, class T, int IPT>
__device__ __forceinline__ typename LinOf<Op>::L::S gs_run_lin(
    const typename Op::S (&ys)[IPT], const typename Op::Acc (&xa)[Op::K][IPT], const typename Op::Acc (&xn)[Op::K],
    const T (&yb)[Op::K][IPT], int64_t n, int64_t base, int cnt) {
    using A = typename Op::Acc;
    using LG = typename LinOf<Op>::L;
    typename LG::S run = LG::id();
#pragma unroll
    for (int k = IPT - 1; k >= 0; --k) {
        if (k < cnt) {
            A nx[Op::K], ybk[Op::K];
            gs_next<Op, IPT>(xa, xn, k, nx);
#pragma unroll
            for (int c = 0; c < Op::K; ++c) ybk[c] = (A)yb[c][k];
            run = LG::comb(run, LinOf<Op>::elem(ys[k], nx, base + k + 1 < n, ybk));
        }
    }
    return run;
}

// Primal: y_i for every element of tile t from its prefix pre[t].
template <class Op, class T, int IPT, bool VEC>
__global__ __launch_bounds__(kGrBlock) void gscan_fwd_kernel(GPtrs<T> x, int64_t n,
                                                             const typename Op::S* __restrict__ pre, GOut<T> y) {
    using S = typename Op::S;
    using A = typename Op::Acc;
    constexpr int K = Op::K;
    __shared__ S wtot[kGrBlock / kWave];
    seg_shift<T, K>(x, n);
    seg_shift<T, K>(y, n);
    const int64_t base = (int64_t)blockIdx.x * (kGrBlock * IPT) + (int64_t)threadIdx.x * IPT;
    const int cnt = gr_cnt<IPT>(n, base);
    A xa[K][IPT], xn[K];
    S ys[IPT], sp;
    gs_run_states<Op, T, IPT, VEC>(x, n, base, cnt, pre[seg_tile()], wtot, xa, xn, ys, sp);
    T out[K][IPT];
#pragma unroll
    for (int k = 0; k < IPT; ++k) {
        A val[K];
        Op::value(ys[k], val);
#pragma unroll
        for (int c = 0; c < K; ++c) out[c][k] = (T)val[c];
    }
#pragma unroll
    for (int c = 0; c < K; ++c) gr_store<T, IPT, VEC>(y.p[c] + base, cnt, out[c]);
}

// VJP pass 1: the lin_o fold of every tile, in reversed index order.
template <class Op, class T, int IPT, bool VEC>
__global__ __launch_bounds__(kGrBlock) void gscan_vjp_agg_kernel(
    GPtrs<T> x, int64_t n, const typename Op::S* __restrict__ pre, GPtrs<T> ybar,
    typename LinOf<Op>::L::S* __restrict__ lagg) {
    using S = typename Op::S;
    using A = typename Op::Acc;
    using LG = typename LinOf<Op>::L;
    constexpr int K = Op::K;
    __shared__ S wtot[kGrBlock / kWave];
    __shared__ typename LG::S ltot[kGrBlock / kWave];
    seg_shift<T, K>(x, n);
    seg_shift<T, K>(ybar, n);
    const int64_t base = (int64_t)blockIdx.x * (kGrBlock * IPT) + (int64_t)threadIdx.x * IPT;
    const int cnt = gr_cnt<IPT>(n, base);
    T yb[K][IPT];
#pragma unroll
    for (int c = 0; c < K; ++c) gr_load<T, IPT, VEC>(ybar.p[c] + base, cnt, yb[c]);
    A xa[K][IPT], xn[K];
    S ys[IPT], sp;
    gs_run_states<Op, T, IPT, VEC>(x, n, base, cnt, pre[seg_tile()], wtot, xa, xn, ys, sp);
    const typename LG::S run = gs_run_lin<Op, T, IPT>(ys, xa, xn, yb, n, base, cnt);
    typename LG::S tot;
    block_exclusive_scan<LG, kGrBlock, true>(run, tot, ltot);
    if (threadIdx.x == 0) lagg[seg_tile()] = tot;
}

// VJP pass 3: lsuf[t] is the lin_o fold of every tile after t; with the
// reversed block scan of the runs it gives the adjoint r after each run,
// then r_k = y_bar_k + J_left(k)^T r_{k+1} walks the run down and
// x_bar_k (+)= J_right(k)^T r_k.
template <class Op, class T, int IPT, bool VEC, bool ACC>
__global__ __launch_bounds__(kGrBlock) void gscan_vjp_kernel(
    GPtrs<T> x, int64_t n, const typename Op::S* __restrict__ pre, GPtrs<T> ybar,
    const typename LinOf<Op>::L::S* __restrict__ lsuf, GOut<T> xbar) {
    using S = typename Op::S;
    using A = typename Op::Acc;
    using LG = typename LinOf<Op>::L;
    constexpr int K = Op::K;
    __shared__ S wtot[kGrBlock / kWave];
    __shared__ typename LG::S ltot[kGrBlock / kWave];
    seg_shift<T, K>(x, n);
    seg_shift<T, K>(ybar, n);
    seg_shift<T, K>(xbar, n);
    const int64_t base = (int64_t)blockIdx.x * (kGrBlock * IPT) + (int64_t)threadIdx.x * IPT;
    const int cnt = gr_cnt<IPT>(n, base);
    T yb[K][IPT];
#pragma unroll
    for (int c = 0; c < K; ++c) gr_load<T, IPT, VEC>(ybar.p[c] + base, cnt, yb[c]);
    A xa[K][IPT], xn[K];
    S ys[IPT], sp;
    gs_run_states<Op, T, IPT, VEC>(x, n, base, cnt, pre[seg_tile()], wtot, xa, xn, ys, sp);
    const typename LG::S run = gs_run_lin<Op, T, IPT>(ys, xa, xn, yb, n, base, cnt);
    typename LG::S tot;
    const typename LG::S ex = block_exclusive_scan<LG, kGrBlock, true>(run, tot, ltot);
    const typename LG::S after = LG::comb(lsuf[seg_tile()], ex);
    A r[K];
#pragma unroll
    for (int c = 0; c < K; ++c) r[c] = after.v[c];
    T out[K][IPT];
#pragma unroll
    for (int k = IPT - 1; k >= 0; --k) {
        A nx[K], ybk[K], rn[K];
        gs_next<Op, IPT>(xa, xn, k, nx);
#pragma unroll
        for (int c = 0; c < K; ++c) ybk[c] = (A)yb[c][k];
        LinOf<Op>::step(ys[k], nx, base + k + 1 < n, ybk, r, rn);
        A xk[K], o[K];
#pragma unroll
        for (int c = 0; c < K; ++c) {
            r[c] = k < cnt ? rn[c] : r[c];
            xk[c] = xa[c][k];
        }
        Op::jrT(k == 0 ? sp : ys[k > 0 ? k - 1 : 0], xk, ys[k], r, o);
#pragma unroll
        for (int c = 0; c < K; ++c) out[c][k] = (T)o[c];
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
    constexpr size_t slot = slot_of<typename Op::S>();
    p.tiles = align_up((size_t)(p.nt > 0 ? p.nt : 1) * slot, 256);
    p.groups = align_up((size_t)(p.ng > 0 ? p.ng : 1) * slot, 256);
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
    static_assert(sizeof(S) <= slot_of<S>(), "slot too small");
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
    const GOut<T> none{};
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

// The scans widen FP32 log-add-exp too: the reversed lin_o scan multiplies
// the coefficients c_k = s_k / (s_k + e^(x_(k+1) - m_k)) along whole suffixes,
// and an FP32 state rounds every c_k (about 1 late in the scan) by about
// 2^-24, errors that add up along the suffix (about n 2^-24 after n steps).
// With the state in FP64 and only the exponential in FP32, a coefficient's
// error is relative to the new element's share 1 - c_k, and the suffix
// products stay accurate.  The exponentials keep their FP32 cost.
template <class Op>
struct ScanWiden {
    using type = Op;
};
template <>
struct ScanWiden<GLogAddExpE<float, float>> {
    using type = GLogAddExpE<double, float>;
};
template <template <class> class OpT, class T>
using GScanOpFor = typename ScanWiden<GOpFor<OpT, T>>::type;

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

// ------------------------------------------------------------- scan host
constexpr size_t kLinSlot = 160;  // bytes per lin_o state (d = 4 in FP64: 4 + 16 values)

// Workspace: [tile folds | tile prefixes | group folds | group prefixes]
// of the operator's states (32-byte slots), then [tile lin_o folds | tile
// lin_o suffixes | group lin_o folds | group lin_o prefixes] (160-byte
// slots), every array 256-byte aligned.  The tile prefixes are the
// checkpoint when the caller keeps one.
struct GsPlan {
    int64_t nt, ng;  // tiles and groups of one segment
    int64_t B;       // segments (independent scans of n elements, back to back)
    size_t t32, g32, tl, gl;
};

template <class Op, class T>
static GsPlan gs_plan(int64_t n, int64_t B = 1) {
    GsPlan p;
    p.nt = ceil_div(n, gs_tile<Op, T>());
    p.ng = ceil_div(p.nt, kAggGroup);
    p.B = B;
    const size_t b = (size_t)(B > 0 ? B : 1);
    const size_t nt = b * (size_t)(p.nt > 0 ? p.nt : 1), ng = b * (size_t)(p.ng > 0 ? p.ng : 1);
    constexpr size_t slot = slot_of<typename Op::S>();
    p.t32 = align_up(nt * slot, 256);
    p.g32 = align_up(ng * slot, 256);
    p.tl = align_up(nt * kLinSlot, 256);
    p.gl = align_up(ng * kLinSlot, 256);
    return p;
}

template <class Op, class T>
static size_t gs_ws(int64_t n, int64_t B = 1) {
    const GsPlan p = gs_plan<Op, T>(n, B);
    return 2 * p.t32 + 2 * p.g32 + 2 * p.tl + 2 * p.gl;
}

static char* gs_at(void* ws, const GsPlan& p, int which) {
    const size_t offs[8] = {0,
                            p.t32,
                            2 * p.t32,
                            2 * p.t32 + p.g32,
                            2 * p.t32 + 2 * p.g32,
                            2 * p.t32 + 2 * p.g32 + p.tl,
                            2 * p.t32 + 2 * p.g32 + 2 * p.tl,
                            2 * p.t32 + 2 * p.g32 + 2 * p.tl + p.gl};
    return reinterpret_cast<char*>(ws) + offs[which];
}

// pre[t] = fold of every element before tile t (the forward reduce-then-scan
// up to the tile prefixes).
template <class Op, class T>
static void gs_prefixes(const GPtrs<T>& x, int64_t n, const GsPlan& p, typename Op::S* pre, void* ws, bool vec,
                        hipStream_t st) {
    using S = typename Op::S;
    constexpr int IPT = gs_ipt<Op, T>();
    if (p.nt == 0) return;
    S* agg = reinterpret_cast<S*>(gs_at(ws, p, 0));
    S* gagg = reinterpret_cast<S*>(gs_at(ws, p, 2));
    S* gpre = reinterpret_cast<S*>(gs_at(ws, p, 3));
    const unsigned B = (unsigned)p.B;
    if (vec)
        hipLaunchKernelGGL((gred_tile_agg_kernel<Op, T, true, IPT>), dim3((unsigned)p.nt, B), dim3(kGrBlock), 0, st,
                           x, n, agg);
    else
        hipLaunchKernelGGL((gred_tile_agg_kernel<Op, T, false, IPT>), dim3((unsigned)p.nt, B), dim3(kGrBlock), 0, st,
                           x, n, agg);
    const unsigned gb = (unsigned)ceil_div(p.ng, kGroupBlock / kWave);
    hipLaunchKernelGGL((group_fold_kernel<Op, false>), dim3(gb, B), dim3(kGroupBlock), 0, st, (const S*)agg, p.nt,
                       p.ng, gagg);
    hipLaunchKernelGGL((agg_scan_kernel<Op, false>), dim3(1, B), dim3(kAggBlock), 0, st, (const S*)gagg, p.ng, gpre);
    hipLaunchKernelGGL((group_prefix_kernel<Op, false>), dim3(gb, B), dim3(kGroupBlock), 0, st, (const S*)agg, p.nt,
                       p.ng, (const S*)gpre, pre);
}

template <class Op, class T>
static void launch_scan(const GPtrs<T>& x, int64_t n, const GOut<T>& y, void* ckpt, void* ws, bool vec,
                        hipStream_t st, int64_t B = 1) {
    using S = typename Op::S;
    constexpr int IPT = gs_ipt<Op, T>();
    const GsPlan p = gs_plan<Op, T>(n, B);
    if (p.nt == 0 || B == 0) return;
    S* pre = ckpt ? reinterpret_cast<S*>(ckpt) : reinterpret_cast<S*>(gs_at(ws, p, 1));
    gs_prefixes<Op, T>(x, n, p, pre, ws, vec, st);
    const dim3 gt((unsigned)p.nt, (unsigned)B);
    if (vec)
        hipLaunchKernelGGL((gscan_fwd_kernel<Op, T, IPT, true>), gt, dim3(kGrBlock), 0, st, x, n, (const S*)pre, y);
    else
        hipLaunchKernelGGL((gscan_fwd_kernel<Op, T, IPT, false>), gt, dim3(kGrBlock), 0, st, x, n, (const S*)pre, y);
}

template <class Op, class T>
static void launch_scan_vjp(const GPtrs<T>& x, int64_t n, const void* ckpt, const GPtrs<T>& yb, const GOut<T>& xb,
                            int acc, void* ws, bool vec, hipStream_t st, int64_t B = 1) {
    using S = typename Op::S;
    using LG = typename LinOf<Op>::L;
    using LS = typename LG::S;
    static_assert(sizeof(LS) <= kLinSlot, "lin_o slot too small");
    constexpr int IPT = gs_ipt<Op, T>();
    const GsPlan p = gs_plan<Op, T>(n, B);
    if (p.nt == 0 || B == 0) return;
    const S* pre = reinterpret_cast<const S*>(ckpt);
    if (!pre) {
        S* w = reinterpret_cast<S*>(gs_at(ws, p, 1));
        gs_prefixes<Op, T>(x, n, p, w, ws, vec, st);
        pre = w;
    }
    LS* lagg = reinterpret_cast<LS*>(gs_at(ws, p, 4));
    LS* lsuf = reinterpret_cast<LS*>(gs_at(ws, p, 5));
    LS* lgagg = reinterpret_cast<LS*>(gs_at(ws, p, 6));
    LS* lgpre = reinterpret_cast<LS*>(gs_at(ws, p, 7));
    const dim3 gt((unsigned)p.nt, (unsigned)B), b(kGrBlock);
    if (vec)
        hipLaunchKernelGGL((gscan_vjp_agg_kernel<Op, T, IPT, true>), gt, b, 0, st, x, n, pre, yb, lagg);
    else
        hipLaunchKernelGGL((gscan_vjp_agg_kernel<Op, T, IPT, false>), gt, b, 0, st, x, n, pre, yb, lagg);
    const unsigned gb = (unsigned)ceil_div(p.ng, kGroupBlock / kWave);
    hipLaunchKernelGGL((group_fold_kernel<LG, true>), dim3(gb, (unsigned)B), dim3(kGroupBlock), 0, st,
                       (const LS*)lagg, p.nt, p.ng, lgagg);
    hipLaunchKernelGGL((agg_scan_kernel<LG, true>), dim3(1, (unsigned)B), dim3(kAggBlock), 0, st, (const LS*)lgagg,
                       p.ng, lgpre);
    hipLaunchKernelGGL((group_prefix_kernel<LG, true>), dim3(gb, (unsigned)B), dim3(kGroupBlock), 0, st,
                       (const LS*)lagg, p.nt, p.ng, (const LS*)lgpre, lsuf);
    const LS* cs = lsuf;
    if (vec) {
        if (acc)
            hipLaunchKernelGGL((gscan_vjp_kernel<Op, T, IPT, true, true>), gt, b, 0, st, x, n, pre, yb, cs, xb);
        else
            hipLaunchKernelGGL((gscan_vjp_kernel<Op, T, IPT, true, false>), gt, b, 0, st, x, n, pre, yb, cs, xb);
    } else {
        if (acc)
            hipLaunchKernelGGL((gscan_vjp_kernel<Op, T, IPT, false, true>), gt, b, 0, st, x, n, pre, yb, cs, xb);
        else
            hipLaunchKernelGGL((gscan_vjp_kernel<Op, T, IPT, false, false>), gt, b, 0, st, x, n, pre, yb, cs, xb);
    }
}

// B > 1: B independent scans of n elements each, segment b at offset b n of
// every array; the 16-byte vector path needs every segment 16-byte aligned.
template <template <class> class OpT, class T>
static void dispatch_scan(const void* const* x, int K, int64_t n, void* const* y, void* ckpt, void* ws,
                          hipStream_t st, int64_t B = 1) {
    GPtrs<T> xp{};
    GOut<T> yp{};
    bool vec = B == 1 || ((size_t)n * sizeof(T)) % 16 == 0;
    for (int c = 0; c < K; ++c) {
        xp.p[c] = (const T*)x[c];
        yp.p[c] = (T*)y[c];
        vec = vec && aligned(x[c], 16) && aligned(y[c], 16);
    }
    launch_scan<GScanOpFor<OpT, T>, T>(xp, n, yp, ckpt, ws, vec, st, B);
}

template <template <class> class OpT, class T>
static void dispatch_scan_vjp(const void* const* x, int K, int64_t n, const void* ckpt, const void* const* yb,
                              void* const* xb, int acc, void* ws, hipStream_t st, int64_t B = 1) {
    GPtrs<T> xp{}, yp{};
    GOut<T> xo{};
    bool vec = B == 1 || ((size_t)n * sizeof(T)) % 16 == 0;
    for (int c = 0; c < K; ++c) {
        xp.p[c] = (const T*)x[c];
        yp.p[c] = (const T*)yb[c];
        xo.p[c] = (T*)xb[c];
        vec = vec && aligned(x[c], 16) && aligned(yb[c], 16) && aligned(xb[c], 16);
    }
    launch_scan_vjp<GScanOpFor<OpT, T>, T>(xp, n, ckpt, yp, xo, acc, ws, vec, st, B);
}

// Size queries by operator and dtype.
template <template <template <class> class, class> class Q>
static size_t gop_query(pvjp_gop op, pvjp_dtype dtype, int64_t n) {
    if (dtype == PVJP_F64) {
        if (op == PVJP_GOP_LOGADDEXP) return Q<GLogAddExp, double>::get(n);
        if (op == PVJP_GOP_LINREC) return Q<GLinRec, double>::get(n);
        return Q<GMat2, double>::get(n);
    }
    if (op == PVJP_GOP_LOGADDEXP) return Q<GLogAddExp, float>::get(n);
    if (op == PVJP_GOP_LINREC) return Q<GLinRec, float>::get(n);
    return Q<GMat2, float>::get(n);
}
// The same for B segments of n elements.
template <template <template <class> class, class> class Q>
static size_t gop_query_b(pvjp_gop op, pvjp_dtype dtype, int64_t n, int64_t B) {
    if (dtype == PVJP_F64) {
        if (op == PVJP_GOP_LOGADDEXP) return Q<GLogAddExp, double>::get(n, B);
        if (op == PVJP_GOP_LINREC) return Q<GLinRec, double>::get(n, B);
        return Q<GMat2, double>::get(n, B);
    }
    if (op == PVJP_GOP_LOGADDEXP) return Q<GLogAddExp, float>::get(n, B);
    if (op == PVJP_GOP_LINREC) return Q<GLinRec, float>::get(n, B);
    return Q<GMat2, float>::get(n, B);
}
template <template <class> class OpT, class T>
struct GsWsQ {
    static size_t get(int64_t n, int64_t B) { return gs_ws<GScanOpFor<OpT, T>, T>(n, B); }
};
template <template <class> class OpT, class T>
struct GsCkQ {
    static size_t get(int64_t n, int64_t B) {
        return (size_t)B * (size_t)gs_plan<GScanOpFor<OpT, T>, T>(n).nt * kGrSlot;
    }
};

// Forward mode: the dual operator of each operator and storage type (FP32
// linear-recurrence and matrix duals in FP64, as for the primal).
template <template <class> class DualT, class T>
using GDualFor = DualT<typename std::conditional<std::is_same<T, float>::value &&
                                                     !std::is_same<DualT<float>, GLaeDual<float>>::value,
                                                 double, T>::type>;

// [x components | x_dot components] -> [y | y_dot]
template <class T>
static void dual_ptrs(const void* const* x, const void* const* xd, int K, GPtrs<T>& xp, bool& vec) {
    for (int c = 0; c < K; ++c) {
        xp.p[c] = (const T*)x[c];
        xp.p[K + c] = (const T*)xd[c];
        vec = vec && aligned(x[c], 16) && aligned(xd[c], 16);
    }
}

template <template <class> class DualT, class T>
static void dispatch_reduce_jvp(const void* const* x, const void* const* xd, int K, int64_t n, void* const* y,
                                void* const* yd, void* ws, hipStream_t st) {
    GPtrs<T> xp{};
    GOut<T> yp{};
    bool vec = true;
    if (n > 0) dual_ptrs<T>(x, xd, K, xp, vec);
    for (int c = 0; c < K; ++c) {
        yp.p[c] = (T*)y[c];
        yp.p[K + c] = (T*)yd[c];
    }
    launch_primal<GDualFor<DualT, T>, T>(xp, n, yp, nullptr, ws, vec, st);
}

template <template <class> class DualT, class T>
static void dispatch_scan_jvp(const void* const* x, const void* const* xd, int K, int64_t n, void* const* y,
                              void* const* yd, void* ws, hipStream_t st) {
    GPtrs<T> xp{};
    GOut<T> yp{};
    bool vec = true;
    dual_ptrs<T>(x, xd, K, xp, vec);
    for (int c = 0; c < K; ++c) {
        yp.p[c] = (T*)y[c];
        yp.p[K + c] = (T*)yd[c];
        vec = vec && aligned(y[c], 16) && aligned(yd[c], 16);
    }
    launch_scan<GDualFor<DualT, T>, T>(xp, n, yp, nullptr, ws, vec, st);
}

template <template <class> class DualT, class T>
struct GrJvpWsQ {
    static size_t get(int64_t n) { return gr_ws<GDualFor<DualT, T>, T>(n); }
};
template <template <class> class DualT, class T>
struct GsJvpWsQ {
    static size_t get(int64_t n) { return gs_ws<GDualFor<DualT, T>, T>(n); }
};

template <template <template <class> class, class> class Q>
static size_t dual_query(pvjp_gop op, pvjp_dtype dtype, int64_t n) {
    if (dtype == PVJP_F64) {
        if (op == PVJP_GOP_LOGADDEXP) return Q<GLaeDual, double>::get(n);
        if (op == PVJP_GOP_LINREC) return Q<GLinRecDual, double>::get(n);
        return Q<GMat2Dual, double>::get(n);
    }
    if (op == PVJP_GOP_LOGADDEXP) return Q<GLaeDual, float>::get(n);
    if (op == PVJP_GOP_LINREC) return Q<GLinRecDual, float>::get(n);
    return Q<GMat2Dual, float>::get(n);
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
    const void* none[8] = {};
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

// ------------------------------------------------------------ scan entry points
constexpr int64_t kMaxSegments = 65535;  // segments ride on blockIdx.y

static size_t scan_ws_bytes(pvjp_gop op, pvjp_dtype dtype, int64_t B, int64_t n) {
    if (gop_components(op) == 0 || !valid_dtype(dtype) || n < 0 || B < 1 || B > kMaxSegments) return 0;
    return gop_query_b<GsWsQ>(op, dtype, n, B);
}

static size_t scan_ckpt_bytes(pvjp_gop op, pvjp_dtype dtype, int64_t B, int64_t n) {
    if (gop_components(op) == 0 || !valid_dtype(dtype) || n < 0 || B < 1 || B > kMaxSegments) return 0;
    return gop_query_b<GsCkQ>(op, dtype, n, B);
}

extern "C" size_t pvjp_scan_generic_ws_bytes(pvjp_gop op, pvjp_dtype dtype, int64_t n) {
    return scan_ws_bytes(op, dtype, 1, n);
}
extern "C" size_t pvjp_scan_generic_ckpt_bytes(pvjp_gop op, pvjp_dtype dtype, int64_t n) {
    return scan_ckpt_bytes(op, dtype, 1, n);
}
extern "C" size_t pvjp_scan_generic_batched_ws_bytes(pvjp_gop op, pvjp_dtype dtype, int64_t B, int64_t L) {
    return scan_ws_bytes(op, dtype, B, L);
}
extern "C" size_t pvjp_scan_generic_batched_ckpt_bytes(pvjp_gop op, pvjp_dtype dtype, int64_t B, int64_t L) {
    return scan_ckpt_bytes(op, dtype, B, L);
}

static pvjp_status check_scan(const char* name, pvjp_gop op, pvjp_dtype dtype, const void* const* x, int64_t B,
                              int64_t n, const void* ckpt, void* ws, size_t ws_bytes) {
    const int K = gop_components(op);
    PVJP_REQUIRE(K > 0, "%s: unknown operator %d", name, (int)op);
    PVJP_REQUIRE(valid_dtype(dtype), "%s: unknown dtype %d", name, (int)dtype);
    PVJP_REQUIRE(n >= 0, "%s: negative n", name);
    PVJP_REQUIRE(B >= 1 && B <= kMaxSegments, "%s: B = %lld segments out of range [1, %lld]", name, (long long)B,
                 (long long)kMaxSegments);
    PVJP_REQUIRE(n * B < ((int64_t)1 << 40), "%s: n too large", name);
    PVJP_REQUIRE(ws != nullptr && aligned(ws, 256), "%s: workspace must be non-NULL and 256-byte aligned", name);
    PVJP_REQUIRE(ckpt == nullptr || aligned(ckpt, 16), "%s: ckpt must be 16-byte aligned", name);
    const size_t need = scan_ws_bytes(op, dtype, B, n);
    if (ws_bytes < need) {
        set_error("%s: workspace of %zu bytes, need %zu", name, ws_bytes, need);
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

static pvjp_status scan_impl(const char* name, pvjp_gop op, pvjp_dtype dtype, const void* const* x, int64_t B,
                             int64_t n, void* const* y, void* ckpt, void* ws, size_t ws_bytes, void* stream) {
    clear_error();
    const pvjp_status s = check_scan(name, op, dtype, x, B, n, ckpt, ws, ws_bytes);
    if (s != PVJP_OK) return s;
    if (n == 0) return PVJP_OK;
    const int K = gop_components(op);
    PVJP_REQUIRE(y != nullptr, "%s: y is NULL", name);
    for (int c = 0; c < K; ++c) {
        PVJP_REQUIRE(y[c] != nullptr, "%s: component %d of y is NULL", name, c);
        PVJP_REQUIRE(aligned(y[c], dsize(dtype)), "%s: component %d of y is misaligned", name, c);
    }
    const hipStream_t st = as_stream(stream);
    if (dtype == PVJP_F64) {
        if (op == PVJP_GOP_LOGADDEXP) dispatch_scan<GLogAddExp, double>(x, K, n, y, ckpt, ws, st, B);
        else if (op == PVJP_GOP_LINREC) dispatch_scan<GLinRec, double>(x, K, n, y, ckpt, ws, st, B);
        else dispatch_scan<GMat2, double>(x, K, n, y, ckpt, ws, st, B);
    } else {
        if (op == PVJP_GOP_LOGADDEXP) dispatch_scan<GLogAddExp, float>(x, K, n, y, ckpt, ws, st, B);
        else if (op == PVJP_GOP_LINREC) dispatch_scan<GLinRec, float>(x, K, n, y, ckpt, ws, st, B);
        else dispatch_scan<GMat2, float>(x, K, n, y, ckpt, ws, st, B);
    }
    PVJP_LAUNCHED(name);
    return PVJP_OK;
}

static pvjp_status scan_vjp_impl(const char* name, pvjp_gop op, pvjp_dtype dtype, const void* const* x, int64_t B,
                                 int64_t n, const void* ckpt, const void* const* y_bar, void* const* x_bar,
                                 int accumulate, void* ws, size_t ws_bytes, void* stream) {
    clear_error();
    const pvjp_status s = check_scan(name, op, dtype, x, B, n, ckpt, ws, ws_bytes);
    if (s != PVJP_OK) return s;
    if (n == 0) return PVJP_OK;
    const int K = gop_components(op);
    PVJP_REQUIRE(y_bar != nullptr && x_bar != nullptr, "%s: y_bar and x_bar must be non-NULL", name);
    for (int c = 0; c < K; ++c) {
        PVJP_REQUIRE(y_bar[c] != nullptr, "%s: component %d of y_bar is NULL", name, c);
        PVJP_REQUIRE(x_bar[c] != nullptr, "%s: component %d of x_bar is NULL", name, c);
        PVJP_REQUIRE(aligned(y_bar[c], dsize(dtype)) && aligned(x_bar[c], dsize(dtype)),
                     "%s: component %d of y_bar or x_bar is misaligned", name, c);
    }
    const hipStream_t st = as_stream(stream);
    const int a = accumulate;
    if (dtype == PVJP_F64) {
        if (op == PVJP_GOP_LOGADDEXP) dispatch_scan_vjp<GLogAddExp, double>(x, K, n, ckpt, y_bar, x_bar, a, ws, st, B);
        else if (op == PVJP_GOP_LINREC) dispatch_scan_vjp<GLinRec, double>(x, K, n, ckpt, y_bar, x_bar, a, ws, st, B);
        else dispatch_scan_vjp<GMat2, double>(x, K, n, ckpt, y_bar, x_bar, a, ws, st, B);
    } else {
        if (op == PVJP_GOP_LOGADDEXP) dispatch_scan_vjp<GLogAddExp, float>(x, K, n, ckpt, y_bar, x_bar, a, ws, st, B);
        else if (op == PVJP_GOP_LINREC) dispatch_scan_vjp<GLinRec, float>(x, K, n, ckpt, y_bar, x_bar, a, ws, st, B);
        else dispatch_scan_vjp<GMat2, float>(x, K, n, ckpt, y_bar, x_bar, a, ws, st, B);
    }
    PVJP_LAUNCHED(name);
    return PVJP_OK;
}

extern "C" pvjp_status pvjp_scan_generic(pvjp_gop op, pvjp_dtype dtype, const void* const* x, int64_t n,
                                         void* const* y, void* ckpt, void* ws, size_t ws_bytes, void* stream) {
    return scan_impl("pvjp_scan_generic", op, dtype, x, 1, n, y, ckpt, ws, ws_bytes, stream);
}

extern "C" pvjp_status pvjp_scan_generic_vjp(pvjp_gop op, pvjp_dtype dtype, const void* const* x, int64_t n,
                                             const void* ckpt, const void* const* y_bar, void* const* x_bar,
                                             int accumulate, void* ws, size_t ws_bytes, void* stream) {
    return scan_vjp_impl("pvjp_scan_generic_vjp", op, dtype, x, 1, n, ckpt, y_bar, x_bar, accumulate, ws, ws_bytes,
                         stream);
}

extern "C" pvjp_status pvjp_scan_generic_batched(pvjp_gop op, pvjp_dtype dtype, const void* const* x, int64_t B,
                                                 int64_t L, void* const* y, void* ckpt, void* ws, size_t ws_bytes,
                                                 void* stream) {
    return scan_impl("pvjp_scan_generic_batched", op, dtype, x, B, L, y, ckpt, ws, ws_bytes, stream);
}

extern "C" pvjp_status pvjp_scan_generic_batched_vjp(pvjp_gop op, pvjp_dtype dtype, const void* const* x, int64_t B,
                                                     int64_t L, const void* ckpt, const void* const* y_bar,
                                                     void* const* x_bar, int accumulate, void* ws, size_t ws_bytes,
                                                     void* stream) {
    return scan_vjp_impl("pvjp_scan_generic_batched_vjp", op, dtype, x, B, L, ckpt, y_bar, x_bar, accumulate, ws,
                         ws_bytes, stream);
}

// ------------------------------------------------------- forward mode entries
extern "C" size_t pvjp_reduce_generic_jvp_ws_bytes(pvjp_gop op, pvjp_dtype dtype, int64_t n) {
    if (gop_components(op) == 0 || !valid_dtype(dtype) || n < 0) return 0;
    return dual_query<GrJvpWsQ>(op, dtype, n);
}

extern "C" size_t pvjp_scan_generic_jvp_ws_bytes(pvjp_gop op, pvjp_dtype dtype, int64_t n) {
    if (gop_components(op) == 0 || !valid_dtype(dtype) || n < 0) return 0;
    return dual_query<GsJvpWsQ>(op, dtype, n);
}

static pvjp_status check_jvp(const char* name, pvjp_gop op, pvjp_dtype dtype, const void* const* x,
                             const void* const* xd, int64_t n, void* const* y, void* const* yd, void* ws,
                             size_t ws_bytes, size_t need) {
    const int K = gop_components(op);
    PVJP_REQUIRE(K > 0, "%s: unknown operator %d", name, (int)op);
    PVJP_REQUIRE(valid_dtype(dtype), "%s: unknown dtype %d", name, (int)dtype);
    PVJP_REQUIRE(n >= 0 && n < ((int64_t)1 << 40), "%s: n out of range", name);
    PVJP_REQUIRE(ws != nullptr && aligned(ws, 256), "%s: workspace must be non-NULL and 256-byte aligned", name);
    if (ws_bytes < need) {
        set_error("%s: workspace of %zu bytes, need %zu", name, ws_bytes, need);
        return PVJP_ENOMEM;
    }
    PVJP_REQUIRE(y != nullptr && yd != nullptr, "%s: y and y_dot must be non-NULL", name);
    for (int c = 0; c < K; ++c) PVJP_REQUIRE(y[c] && yd[c], "%s: component %d of y or y_dot is NULL", name, c);
    if (n > 0) {
        PVJP_REQUIRE(x != nullptr && xd != nullptr, "%s: x and x_dot must be non-NULL", name);
        for (int c = 0; c < K; ++c) {
            PVJP_REQUIRE(x[c] && xd[c], "%s: component %d of x or x_dot is NULL", name, c);
            PVJP_REQUIRE(aligned(x[c], dsize(dtype)) && aligned(xd[c], dsize(dtype)),
                         "%s: component %d of x or x_dot is misaligned", name, c);
        }
    }
    return PVJP_OK;
}

extern "C" pvjp_status pvjp_reduce_generic_jvp(pvjp_gop op, pvjp_dtype dtype, const void* const* x,
                                               const void* const* x_dot, int64_t n, void* const* y,
                                               void* const* y_dot, void* ws, size_t ws_bytes, void* stream) {
    clear_error();
    const pvjp_status s = check_jvp("pvjp_reduce_generic_jvp", op, dtype, x, x_dot, n, y, y_dot, ws, ws_bytes,
                                    pvjp_reduce_generic_jvp_ws_bytes(op, dtype, n));
    if (s != PVJP_OK) return s;
    const int K = gop_components(op);
    const hipStream_t st = as_stream(stream);
    if (dtype == PVJP_F64) {
        if (op == PVJP_GOP_LOGADDEXP) dispatch_reduce_jvp<GLaeDual, double>(x, x_dot, K, n, y, y_dot, ws, st);
        else if (op == PVJP_GOP_LINREC) dispatch_reduce_jvp<GLinRecDual, double>(x, x_dot, K, n, y, y_dot, ws, st);
        else dispatch_reduce_jvp<GMat2Dual, double>(x, x_dot, K, n, y, y_dot, ws, st);
    } else {
        if (op == PVJP_GOP_LOGADDEXP) dispatch_reduce_jvp<GLaeDual, float>(x, x_dot, K, n, y, y_dot, ws, st);
        else if (op == PVJP_GOP_LINREC) dispatch_reduce_jvp<GLinRecDual, float>(x, x_dot, K, n, y, y_dot, ws, st);
        else dispatch_reduce_jvp<GMat2Dual, float>(x, x_dot, K, n, y, y_dot, ws, st);
    }
    PVJP_LAUNCHED("pvjp_reduce_generic_jvp");
    return PVJP_OK;
}

extern "C" pvjp_status pvjp_scan_generic_jvp(pvjp_gop op, pvjp_dtype dtype, const void* const* x,
                                             const void* const* x_dot, int64_t n, void* const* y, void* const* y_dot,
                                             void* ws, size_t ws_bytes, void* stream) {
    clear_error();
    const pvjp_status s = check_jvp("pvjp_scan_generic_jvp", op, dtype, x, x_dot, n, y, y_dot, ws, ws_bytes,
                                    pvjp_scan_generic_jvp_ws_bytes(op, dtype, n));
    if (s != PVJP_OK) return s;
    if (n == 0) return PVJP_OK;
    const int K = gop_components(op);
    for (int c = 0; c < K; ++c)
        PVJP_REQUIRE(aligned(y[c], dsize(dtype)) && aligned(y_dot[c], dsize(dtype)),
                     "pvjp_scan_generic_jvp: component %d of y or y_dot is misaligned", c);
    const hipStream_t st = as_stream(stream);
    if (dtype == PVJP_F64) {
        if (op == PVJP_GOP_LOGADDEXP) dispatch_scan_jvp<GLaeDual, double>(x, x_dot, K, n, y, y_dot, ws, st);
        else if (op == PVJP_GOP_LINREC) dispatch_scan_jvp<GLinRecDual, double>(x, x_dot, K, n, y, y_dot, ws, st);
        else dispatch_scan_jvp<GMat2Dual, double>(x, x_dot, K, n, y, y_dot, ws, st);
    } else {
        if (op == PVJP_GOP_LOGADDEXP) dispatch_scan_jvp<GLaeDual, float>(x, x_dot, K, n, y, y_dot, ws, st);
        else if (op == PVJP_GOP_LINREC) dispatch_scan_jvp<GLinRecDual, float>(x, x_dot, K, n, y, y_dot, ws, st);
        else dispatch_scan_jvp<GMat2Dual, float>(x, x_dot, K, n, y, y_dot, ws, st);
    }
    PVJP_LAUNCHED("pvjp_scan_generic_jvp");
    return PVJP_OK;
}
