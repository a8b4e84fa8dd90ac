// Inclusive scan of the first-order linear recurrence and its VJP (Sec. 5.2).
//
// Primal: single-pass decoupled-lookback scan with the operator
//   (a1,b1) (+) (a2,b2) = (a2*a1, a2*b1 + b2).
// It optionally writes a checkpoint (the exclusive prefix) every
// PVJP_LINREC_CKPT_INTERVAL elements; this is the only primal state the VJP
// keeps.
//
// VJP: the return sweep of Sec. 5.2 in one kernel per tile, tiles taken in
// reverse virtual order:
//   1. recompute the primal prefixes (A_{i-1}, B_{i-1}) of the tile from its
//      checkpoint (redundant execution of the forward sweep, Sec. 4.1);
//   2. map c_i = a_{i+1} (the left Jacobian of the operator is a_{i+1} * I),
//      d_i = y_bar_i;
//   3. reversed scan with lin_o over (c, d) -- tile aggregate, lookback over
//      the tiles to the right, local apply -- giving
//      r_bar_i = y_bar_i + a_{i+1} r_bar_{i+1};
//   4. map a_bar_i = A_{i-1} rA_bar_i + B_{i-1} rB_bar_i, b_bar_i = rB_bar_i
//      (the transposed right Jacobian [[A_{i-1}, 0], [B_{i-1}, 1]]).
#include <mutex>

#include "common.h"
#include "prims.h"

namespace pvjp {

constexpr int kCk = PVJP_LINREC_CKPT_INTERVAL;
constexpr int kScanBlock = 256;

template <class T>
struct ScanCfg;
template <>
struct ScanCfg<double> {
    static constexpr int IPT = 8;  // 2048-element tiles
};
template <>
struct ScanCfg<float> {
    static constexpr int IPT = 16;  // 4096-element tiles
};

template <class T>
constexpr int scan_tile() {
    return kScanBlock * ScanCfg<T>::IPT;
}

static_assert(scan_tile<double>() % kCk == 0 && scan_tile<float>() % kCk == 0,
              "scan tiles must be whole checkpoint intervals");

// GIVEN = false: single pass, the tile's exclusive prefix comes from the
// decoupled lookback (tiles taken in ticket order).  GIVEN = true: third
// pass of the reduce-then-scan form, the prefix is read from `pre`.
template <class T, bool GIVEN>
__global__ __launch_bounds__(kScanBlock) void linrec_fwd_kernel(
    const T* __restrict__ a, const T* __restrict__ b, int64_t n, T* __restrict__ A,
    T* __restrict__ B, T* __restrict__ ckpt, LookbackHdr* hdr,
    TileState<typename LinRec<T>::S>* states, int64_t ntiles, const typename LinRec<T>::S* __restrict__ pre) {
    using Op = LinRec<T>;
    using S = typename Op::S;
    constexpr int IPT = ScanCfg<T>::IPT;
    constexpr int TS = kScanBlock * IPT;
    __shared__ T lds[lds_elems<T, TS>()];
    __shared__ S wtot[kScanBlock / kWave];
    __shared__ uint32_t s_tag, s_ticket;
    __shared__ S s_prefix;

    if (GIVEN) {
        // right to left: the first tiles read are the last ones the
        // aggregate pass read, which the last-level cache may still hold
        if (threadIdx.x == 0) s_ticket = (uint32_t)(ntiles - 1 - blockIdx.x);
    } else if (threadIdx.x == 0) {
        s_ticket = lookback_draw(hdr, (uint32_t)(ntiles - 1), &s_tag);
        if (s_ticket >= ntiles) lookback_error(hdr, kErrTicket);
    }
    __syncthreads();
    const uint32_t tag = s_tag;
    if (s_ticket >= ntiles) return;  // the workspace was not in its rest state: do nothing
    const int64_t tile = s_ticket;
    const int64_t base = tile * TS;
    const int cnt = (int)((n - base) < TS ? (n - base) : TS);

    T ra[IPT], rb[IPT];
    {
        T sa[IPT], sb[IPT];  // both arrays in flight before the first transpose
        load_striped<T, kScanBlock, IPT>(a + base, cnt, sa, T(1));
        load_striped<T, kScanBlock, IPT>(b + base, cnt, sb, T(0));
        striped_to_blocked<T, kScanBlock, IPT>(sa, ra, lds);
        __syncthreads();
        striped_to_blocked<T, kScanBlock, IPT>(sb, rb, lds);
    }

    S agg = S{ra[0], rb[0]};
#pragma unroll
    for (int j = 1; j < IPT; ++j) agg = Op::comb(agg, S{ra[j], rb[j]});
    S total;
    S excl = block_exclusive_scan<Op, kScanBlock, false>(agg, total, wtot);

    if (GIVEN) {
        if (threadIdx.x == 0) s_prefix = pre[tile];
    } else if (threadIdx.x < kWave) {
        S prefix = Op::id();
        if (tile == 0) {
            if (threadIdx.x == 0) publish(&states[tile], total, kInc, tag);
        } else {
            if (threadIdx.x == 0) publish(&states[tile], total, kAgg, tag);
            prefix = lookback<Op>(states, states + ntiles, tile, total, tag, hdr);
            if (threadIdx.x == 0) publish(&states[tile], Op::comb(prefix, total), kInc, tag);
        }
        if (threadIdx.x == 0) s_prefix = prefix;
    }
    __syncthreads();

    S run = Op::comb(s_prefix, excl);
    const int first = (int)threadIdx.x * IPT;
    if (ckpt != nullptr && (first % kCk) == 0 && first < cnt) {
        const int64_t c = (base + first) / kCk;
        ckpt[2 * c] = run.a;
        ckpt[2 * c + 1] = run.b;
    }
#pragma unroll
    for (int j = 0; j < IPT; ++j) {
        run = Op::comb(run, S{ra[j], rb[j]});
        ra[j] = run.a;
        rb[j] = run.b;
    }
    if (A != nullptr) {
        store_blocked<T, kScanBlock, IPT, false>(A + base, cnt, ra, lds);
        store_blocked<T, kScanBlock, IPT, false>(B + base, cnt, rb, lds);
    }
}

// GIVEN as for the primal: the tile's suffix (in the reversed scan order)
// comes from the lookback, or from `pre` in the three-pass form.
template <class T, bool ACC, bool GIVEN>
__global__ __launch_bounds__(kScanBlock) void linrec_vjp_kernel(
    const T* __restrict__ a, const T* __restrict__ b, const T* __restrict__ ya,
    const T* __restrict__ yb, int64_t n, const T* __restrict__ ckpt, T* __restrict__ abar,
    T* __restrict__ bbar, LookbackHdr* hdr, TileState<typename LinO<T>::S>* states,
    int64_t ntiles, const typename LinO<T>::S* __restrict__ pre) {
    using P = LinRec<T>;
    using L = LinO<T>;
    using PS = typename P::S;
    using LS = typename L::S;
    constexpr int IPT = ScanCfg<T>::IPT;
    constexpr int TS = kScanBlock * IPT;
    __shared__ T lds[lds_elems<T, TS>()];
    __shared__ PS wtot_p[kScanBlock / kWave];
    __shared__ LS wtot_l[kScanBlock / kWave];
    __shared__ uint32_t s_tag, s_ticket;
    __shared__ LS s_suffix;

    if (GIVEN) {
        if (threadIdx.x == 0) s_ticket = blockIdx.x;
    } else if (threadIdx.x == 0) {
        s_ticket = lookback_draw(hdr, (uint32_t)(ntiles - 1), &s_tag);
        if (s_ticket >= ntiles) lookback_error(hdr, kErrTicket);
    }
    __syncthreads();
    const uint32_t tag = s_tag;
    if (s_ticket >= ntiles) return;  // the workspace was not in its rest state: do nothing
    const int64_t v = s_ticket;            // virtual index: scan order
    const int64_t tile = ntiles - 1 - v;  // tiles are taken right to left
    const int64_t base = tile * TS;
    const int cnt = (int)((n - base) < TS ? (n - base) : TS);
    const int first = (int)threadIdx.x * IPT;

    // --- loads (a with its one-element look-ahead for c_i = a_{i+1}); all
    //     four arrays are in flight before the first transpose
    T ra[IPT], rc[IPT], rb[IPT], rya[IPT], ryb[IPT];
    {
        T sa[IPT], sb[IPT], sya[IPT], syb[IPT];
        load_striped<T, kScanBlock, IPT>(a + base, cnt, sa, T(1));
        load_striped<T, kScanBlock, IPT>(b + base, cnt, sb, T(0));
        load_striped<T, kScanBlock, IPT>(ya + base, cnt, sya, T(0));
        load_striped<T, kScanBlock, IPT>(yb + base, cnt, syb, T(0));
        const T after = ((int)threadIdx.x == kScanBlock - 1 && base + TS < n) ? a[base + TS] : T(1);
        striped_to_blocked<T, kScanBlock, IPT>(sa, ra, lds);
        const T nxt = ((int)threadIdx.x < kScanBlock - 1) ? lds[lds_pad<T>(first + IPT)] : after;
#pragma unroll
        for (int j = 0; j < IPT - 1; ++j) rc[j] = ra[j + 1];
        rc[IPT - 1] = nxt;
        __syncthreads();
        striped_to_blocked<T, kScanBlock, IPT>(sb, rb, lds);
        __syncthreads();
        striped_to_blocked<T, kScanBlock, IPT>(sya, rya, lds);
        __syncthreads();
        striped_to_blocked<T, kScanBlock, IPT>(syb, ryb, lds);
    }

    // --- 1. recompute primal prefixes from the tile's checkpoint
    T pA[IPT], pB[IPT];
    {
        PS agg = PS{ra[0], rb[0]};
#pragma unroll
        for (int j = 1; j < IPT; ++j) agg = P::comb(agg, PS{ra[j], rb[j]});
        PS total;
        PS excl = block_exclusive_scan<P, kScanBlock, false>(agg, total, wtot_p);
        const int64_t c = base / kCk;
        PS run = P::comb(PS{ckpt[2 * c], ckpt[2 * c + 1]}, excl);
#pragma unroll
        for (int j = 0; j < IPT; ++j) {
            pA[j] = run.a;  // (A_{i-1}, B_{i-1})
            pB[j] = run.b;
            run = P::comb(run, PS{ra[j], rb[j]});
        }
    }

    // --- 2. map: lin_o elements (c_i, y_bar_i); the last element of the array
    //        has no successor, and padding elements are the neutral element.
    LS e[IPT];
#pragma unroll
    for (int j = 0; j < IPT; ++j) {
        const int64_t gi = base + first + j;
        T c = rc[j];
        if (gi == n - 1) c = T(0);
        e[j] = LS{c, rya[j], ryb[j]};
    }

    // --- 3. reversed scan (scan order = decreasing index)
    LS agg = L::id();
#pragma unroll
    for (int j = IPT - 1; j >= 0; --j) agg = L::comb(agg, e[j]);
    LS total;
    LS excl = block_exclusive_scan<L, kScanBlock, true>(agg, total, wtot_l);
    if (GIVEN) {
        if (threadIdx.x == 0) s_suffix = pre[tile];
    } else if (threadIdx.x < kWave) {
        LS suffix = L::id();
        if (v == 0) {
            if (threadIdx.x == 0) publish(&states[v], total, kInc, tag);
        } else {
            if (threadIdx.x == 0) publish(&states[v], total, kAgg, tag);
            suffix = lookback<L>(states, states + ntiles, v, total, tag, hdr);
            if (threadIdx.x == 0) publish(&states[v], L::comb(suffix, total), kInc, tag);
        }
        if (threadIdx.x == 0) s_suffix = suffix;
    }
    __syncthreads();

    // --- 4. map: input adjoints
    LS run = L::comb(s_suffix, excl);
#pragma unroll
    for (int j = IPT - 1; j >= 0; --j) {
        run = L::comb(run, e[j]);
        ra[j] = pA[j] * run.dA + pB[j] * run.dB;
        rb[j] = run.dB;
    }
    store_blocked<T, kScanBlock, IPT, ACC>(abar + base, cnt, ra, lds);
    store_blocked<T, kScanBlock, IPT, ACC>(bbar + base, cnt, rb, lds);
}

// ------------------------------------------------- reduce-then-scan form
// For long inputs the single pass is bound by its lookback: with the tens of
// MB in flight that saturate HBM, every device-scope round trip waits
// behind them, and each tile pays several such trips on its critical path.
// The three-pass form has none: (1) every tile writes its aggregate,
// (2) one block scans the aggregates, (3) every tile re-reads its input and
// applies its prefix.  It moves 16 (primal, FP64) or 24 (VJP) more bytes
// per element but streams at full rate.

// (1) primal tile aggregates
template <class T>
__global__ __launch_bounds__(kScanBlock) void linrec_tile_agg_kernel(const T* __restrict__ a, const T* __restrict__ b,
                                                                     int64_t n, typename LinRec<T>::S* __restrict__ agg) {
    using Op = LinRec<T>;
    using S = typename Op::S;
    constexpr int IPT = ScanCfg<T>::IPT;
    constexpr int TS = kScanBlock * IPT;
    __shared__ T lds[lds_elems<T, TS>()];
    __shared__ S wtot[kScanBlock / kWave];
    const int64_t tile = blockIdx.x;
    const int64_t base = tile * TS;
    const int cnt = (int)((n - base) < TS ? (n - base) : TS);
    T ra[IPT], rb[IPT];
    {
        T sa[IPT], sb[IPT];
        load_striped<T, kScanBlock, IPT>(a + base, cnt, sa, T(1));
        load_striped<T, kScanBlock, IPT>(b + base, cnt, sb, T(0));
        striped_to_blocked<T, kScanBlock, IPT>(sa, ra, lds);
        __syncthreads();
        striped_to_blocked<T, kScanBlock, IPT>(sb, rb, lds);
    }
    S v = S{ra[0], rb[0]};
#pragma unroll
    for (int j = 1; j < IPT; ++j) v = Op::comb(v, S{ra[j], rb[j]});
    S total;
    (void)block_exclusive_scan<Op, kScanBlock, false>(v, total, wtot);
    if (threadIdx.x == 0) agg[tile] = total;
}

// (1) adjoint tile aggregates: the lin_o elements (c_i, y_bar_i) of the tile,
// combined in decreasing index order.
template <class T>
__global__ __launch_bounds__(kScanBlock) void linrec_vjp_tile_agg_kernel(const T* __restrict__ a,
                                                                         const T* __restrict__ ya,
                                                                         const T* __restrict__ yb, int64_t n,
                                                                         typename LinO<T>::S* __restrict__ agg) {
    using L = LinO<T>;
    using LS = typename L::S;
    constexpr int IPT = ScanCfg<T>::IPT;
    constexpr int TS = kScanBlock * IPT;
    __shared__ T lds[lds_elems<T, TS>()];
    __shared__ LS wtot[kScanBlock / kWave];
    const int64_t tile = blockIdx.x;
    const int64_t base = tile * TS;
    const int cnt = (int)((n - base) < TS ? (n - base) : TS);
    const int first = (int)threadIdx.x * IPT;
    T ra[IPT], rc[IPT], rya[IPT], ryb[IPT];
    {
        T sa[IPT], sya[IPT], syb[IPT];
        load_striped<T, kScanBlock, IPT>(a + base, cnt, sa, T(1));
        load_striped<T, kScanBlock, IPT>(ya + base, cnt, sya, T(0));
        load_striped<T, kScanBlock, IPT>(yb + base, cnt, syb, T(0));
        const T after = ((int)threadIdx.x == kScanBlock - 1 && base + TS < n) ? a[base + TS] : T(1);
        striped_to_blocked<T, kScanBlock, IPT>(sa, ra, lds);
        const T nxt = ((int)threadIdx.x < kScanBlock - 1) ? lds[lds_pad<T>(first + IPT)] : after;
#pragma unroll
        for (int j = 0; j < IPT - 1; ++j) rc[j] = ra[j + 1];
        rc[IPT - 1] = nxt;
        __syncthreads();
        striped_to_blocked<T, kScanBlock, IPT>(sya, rya, lds);
        __syncthreads();
        striped_to_blocked<T, kScanBlock, IPT>(syb, ryb, lds);
    }
    LS v = L::id();
#pragma unroll
    for (int j = IPT - 1; j >= 0; --j) {
        const int64_t gi = base + first + j;
        const T c = (gi == n - 1) ? T(0) : rc[j];
        v = L::comb(v, LS{c, rya[j], ryb[j]});
    }
    LS total;
    (void)block_exclusive_scan<L, kScanBlock, true>(v, total, wtot);
    if (threadIdx.x == 0) agg[tile] = total;
}

// (2) the aggregates are scanned in scan order (increasing tile index, or
// decreasing for the VJP) by agg_scan_kernel / group_fold_kernel /
// group_prefix_kernel of prims.h.

// ------------------------------------------------------------------ host
// Inputs of more tiles than this take the three-pass form.
constexpr int64_t kThreePassTiles = 4096;
constexpr size_t kAggSlot = 32;  // bytes per tile for an aggregate or a prefix (either operator)

// [header | tile states | group states | tile aggregates | tile prefixes |
// group folds | group prefixes]: the three-pass form never touches the
// lookback states or the header.
static size_t group_bytes(int64_t ntiles) {
    return align_up((size_t)ceil_div(ntiles, kAggGroup) * kAggSlot, 256);
}

template <class S>
static size_t lookback_bytes(int64_t ntiles) {
    static_assert(sizeof(S) <= kAggSlot, "aggregate slot too small");
    return align_up(sizeof(LookbackHdr) + lookback_state_bytes<S>(ntiles), 256) +
           align_up((size_t)ntiles * kAggSlot * 2, 256) + 2 * group_bytes(ntiles);
}

template <class S>
static S* agg_array(void* ws, int64_t ntiles) {
    return reinterpret_cast<S*>(reinterpret_cast<char*>(ws) +
                                align_up(sizeof(LookbackHdr) + lookback_state_bytes<S>(ntiles), 256));
}

template <class S>
static S* pre_array(void* ws, int64_t ntiles) {
    return reinterpret_cast<S*>(reinterpret_cast<char*>(agg_array<S>(ws, ntiles)) + (size_t)ntiles * kAggSlot);
}

template <class S>
static S* group_array(void* ws, int64_t ntiles, int which) {
    return reinterpret_cast<S*>(reinterpret_cast<char*>(agg_array<S>(ws, ntiles)) +
                                align_up((size_t)ntiles * kAggSlot * 2, 256) + which * group_bytes(ntiles));
}

// (2a)-(2c): pre[t] = exclusive fold of the tile aggregates in scan order.
template <class Op, bool REV>
static void scan_aggregates(const typename Op::S* agg, int64_t nt, typename Op::S* pre, void* ws,
                            hipStream_t st) {
    using S = typename Op::S;
    const int64_t ng = ceil_div(nt, kAggGroup);
    S* gagg = group_array<S>(ws, nt, 0);
    S* gpre = group_array<S>(ws, nt, 1);
    const unsigned gb = (unsigned)ceil_div(ng, kGroupBlock / kWave);
    hipLaunchKernelGGL((group_fold_kernel<Op, REV>), dim3(gb), dim3(kGroupBlock), 0, st, agg, nt, ng, gagg);
    hipLaunchKernelGGL((agg_scan_kernel<Op, REV>), dim3(1), dim3(kAggBlock), 0, st, (const S*)gagg, ng, gpre);
    hipLaunchKernelGGL((group_prefix_kernel<Op, REV>), dim3(gb), dim3(kGroupBlock), 0, st, agg, nt, ng,
                       (const S*)gpre, pre);
}

template <class T>
static size_t fwd_ws(int64_t n) {
    return lookback_bytes<typename LinRec<T>::S>(ceil_div(n, scan_tile<T>()));
}

// Workspace layout of both entry points: [header | tile states | group
// states | aggregates | prefixes | ckpt].  The checkpoint-only pre-pass of the VJP and the VJP itself
// run one after the other on the same header and states (states are 128
// bytes for both operators and both use the same tile size), so every launch
// on a workspace takes its tag from the one epoch sequence.
template <class T>
static size_t vjp_ws(int64_t n) {
    const int64_t nt = ceil_div(n, scan_tile<T>());
    return align_up(lookback_bytes<typename LinO<T>::S>(nt), 256) +
           align_up((size_t)(2 * ceil_div(n, kCk)) * sizeof(T), 256);
}
static_assert(sizeof(TileState<LinRec<double>::S>) == sizeof(TileState<LinO<double>::S>) &&
                  sizeof(TileState<LinRec<float>::S>) == sizeof(TileState<LinO<float>::S>),
              "primal and adjoint tile states share one workspace region");

template <class T>
static pvjp_status launch_fwd(const void* a, const void* b, int64_t n, void* A, void* B,
                              void* ckpt, void* ws, hipStream_t st) {
    using S = typename LinRec<T>::S;
    const int64_t nt = ceil_div(n, scan_tile<T>());
    auto* hdr = reinterpret_cast<LookbackHdr*>(ws);
    auto* states = reinterpret_cast<TileState<S>*>(reinterpret_cast<char*>(ws) + sizeof(LookbackHdr));
    if (nt > kThreePassTiles) {
        S* agg = agg_array<S>(ws, nt);
        S* pre = pre_array<S>(ws, nt);
        hipLaunchKernelGGL(linrec_tile_agg_kernel<T>, dim3((unsigned)nt), dim3(kScanBlock), 0, st, (const T*)a,
                           (const T*)b, n, agg);
        scan_aggregates<LinRec<T>, false>(agg, nt, pre, ws, st);
        hipLaunchKernelGGL((linrec_fwd_kernel<T, true>), dim3((unsigned)nt), dim3(kScanBlock), 0, st,
                           (const T*)a, (const T*)b, n, (T*)A, (T*)B, (T*)ckpt, hdr, states, nt, (const S*)pre);
    } else {
        hipLaunchKernelGGL((linrec_fwd_kernel<T, false>), dim3((unsigned)nt), dim3(kScanBlock), 0, st,
                           (const T*)a, (const T*)b, n, (T*)A, (T*)B, (T*)ckpt, hdr, states, nt, (const S*)nullptr);
    }
    PVJP_LAUNCHED("pvjp_linrec_scan");
    return PVJP_OK;
}

template <class T>
static pvjp_status launch_vjp(const void* a, const void* b, const void* ya, const void* yb,
                              int64_t n, const void* ckpt, void* abar, void* bbar, int acc,
                              void* ws, hipStream_t st) {
    using LS = typename LinO<T>::S;
    const int64_t nt = ceil_div(n, scan_tile<T>());
    char* w = reinterpret_cast<char*>(ws);
    auto* hdr = reinterpret_cast<LookbackHdr*>(w);
    auto* states = reinterpret_cast<TileState<LS>*>(w + sizeof(LookbackHdr));
    if (ckpt == nullptr) {  // checkpoint-only primal pass into the workspace
        T* ck = reinterpret_cast<T*>(w + align_up(lookback_bytes<LS>(nt), 256));
        pvjp_status s = launch_fwd<T>(a, b, n, nullptr, nullptr, ck, ws, st);
        if (s != PVJP_OK) return s;
        ckpt = ck;
    }
    const LS* pre = nullptr;
    if (nt > kThreePassTiles) {
        LS* agg = agg_array<LS>(ws, nt);
        LS* p = pre_array<LS>(ws, nt);
        hipLaunchKernelGGL(linrec_vjp_tile_agg_kernel<T>, dim3((unsigned)nt), dim3(kScanBlock), 0, st, (const T*)a,
                           (const T*)ya, (const T*)yb, n, agg);
        scan_aggregates<LinO<T>, true>(agg, nt, p, ws, st);
        pre = p;
    }
    if (pre) {
        if (acc)
            hipLaunchKernelGGL((linrec_vjp_kernel<T, true, true>), dim3((unsigned)nt), dim3(kScanBlock), 0, st,
                               (const T*)a, (const T*)b, (const T*)ya, (const T*)yb, n, (const T*)ckpt,
                               (T*)abar, (T*)bbar, hdr, states, nt, pre);
        else
            hipLaunchKernelGGL((linrec_vjp_kernel<T, false, true>), dim3((unsigned)nt), dim3(kScanBlock), 0, st,
                               (const T*)a, (const T*)b, (const T*)ya, (const T*)yb, n, (const T*)ckpt,
                               (T*)abar, (T*)bbar, hdr, states, nt, pre);
    } else {
        if (acc)
            hipLaunchKernelGGL((linrec_vjp_kernel<T, true, false>), dim3((unsigned)nt), dim3(kScanBlock), 0, st,
                               (const T*)a, (const T*)b, (const T*)ya, (const T*)yb, n, (const T*)ckpt,
                               (T*)abar, (T*)bbar, hdr, states, nt, pre);
        else
            hipLaunchKernelGGL((linrec_vjp_kernel<T, false, false>), dim3((unsigned)nt), dim3(kScanBlock), 0, st,
                               (const T*)a, (const T*)b, (const T*)ya, (const T*)yb, n, (const T*)ckpt,
                               (T*)abar, (T*)bbar, hdr, states, nt, pre);
    }
    PVJP_LAUNCHED("pvjp_linrec_scan_vjp");
    return PVJP_OK;
}

// ------------------------------------------------- fixed-scratch variant
// The VJP entry point for callers that cannot allocate takes its workspace
// from this array instead of an argument.  Each GPU the library runs on
// holds its own copy until the process ends.  It starts zero-filled (as a
// workspace must), and every lookback launch leaves it ready for the next
// one, so it is never cleared again.  In host code `scratch` names a
// host-side stand-in, not device memory: the device address is looked up
// once per device with hipGetSymbolAddress and only that address is used.
constexpr size_t kNoAllocScratchBytes = (size_t)8 << 20;
static __device__ __align__(256) char scratch[kNoAllocScratchBytes];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch[kMaxDevices];

// Device address of `scratch` on the device that runs `st`.
static pvjp_status scratch_for(hipStream_t st, void** out) {
    int dev = 0;
    if (st != nullptr) {
        hipDevice_t d;
        if (hipStreamGetDevice(st, &d) != hipSuccess) {
            set_error("pvjp_linrec_scan_vjp_noalloc: cannot tell the stream's device");
            return PVJP_EDEVICE;
        }
        dev = (int)d;
    } else if (hipGetDevice(&dev) != hipSuccess) {
        set_error("pvjp_linrec_scan_vjp_noalloc: no current device");
        return PVJP_EDEVICE;
    }
    if (dev < 0 || dev >= kMaxDevices) {
        set_error("pvjp_linrec_scan_vjp_noalloc: device %d beyond the %d this library tracks", dev, kMaxDevices);
        return PVJP_EUNSUPPORTED;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch[dev] == nullptr) {
        int cur = 0;
        if (hipGetDevice(&cur) != hipSuccess || (cur != dev && hipSetDevice(dev) != hipSuccess)) {
            set_error("pvjp_linrec_scan_vjp_noalloc: cannot make device %d current", dev);
            return PVJP_EDEVICE;
        }
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (cur != dev) (void)hipSetDevice(cur);
        if (e != hipSuccess || p == nullptr) {
            set_error("pvjp_linrec_scan_vjp_noalloc: hipGetSymbolAddress failed on device %d: %s", dev,
                      hipGetErrorString(e));
            return PVJP_EDEVICE;
        }
        g_scratch[dev] = p;
    }
    *out = g_scratch[dev];
    return PVJP_OK;
}

}  // namespace pvjp

using namespace pvjp;

// Tile counts are carried in 32-bit tickets.
static constexpr int64_t kMaxScanN = (int64_t)1 << 40;

extern "C" int64_t pvjp_linrec_ckpt_len(int64_t n) { return n <= 0 ? 0 : ceil_div(n, kCk); }

extern "C" size_t pvjp_linrec_scan_ws_bytes(pvjp_dtype dtype, int64_t n) {
    if (n <= 0 || !valid_dtype(dtype)) return 0;
    return dtype == PVJP_F64 ? fwd_ws<double>(n) : fwd_ws<float>(n);
}

extern "C" size_t pvjp_linrec_scan_vjp_ws_bytes(pvjp_dtype dtype, int64_t n) {
    if (n <= 0 || !valid_dtype(dtype)) return 0;
    return dtype == PVJP_F64 ? vjp_ws<double>(n) : vjp_ws<float>(n);
}

extern "C" pvjp_status pvjp_linrec_scan(pvjp_dtype dtype, const void* a, const void* b, int64_t n,
                                        void* A, void* B, void* ckpt, void* ws, size_t ws_bytes,
                                        void* stream) {
    clear_error();
    PVJP_REQUIRE(valid_dtype(dtype), "pvjp_linrec_scan: unknown dtype %d", (int)dtype);
    PVJP_REQUIRE(n >= 0 && n <= kMaxScanN, "pvjp_linrec_scan: n = %lld out of range", (long long)n);
    if (n == 0) return PVJP_OK;
    PVJP_REQUIRE(a && b, "pvjp_linrec_scan: a and b must be non-NULL");
    PVJP_REQUIRE((A == nullptr) == (B == nullptr), "pvjp_linrec_scan: A and B must both be given or both NULL");
    PVJP_REQUIRE(A || ckpt, "pvjp_linrec_scan: nothing to compute (A, B and ckpt all NULL)");
    PVJP_REQUIRE(ws != nullptr, "pvjp_linrec_scan: ws is NULL");
    const size_t need = pvjp_linrec_scan_ws_bytes(dtype, n);
    if (ws_bytes < need) {
        set_error("pvjp_linrec_scan: workspace has %zu bytes, needs %zu", ws_bytes, need);
        return PVJP_ENOMEM;
    }
    PVJP_REQUIRE(aligned(ws, 256), "pvjp_linrec_scan: ws must be 256-byte aligned");
    return dtype == PVJP_F64 ? launch_fwd<double>(a, b, n, A, B, ckpt, ws, as_stream(stream))
                             : launch_fwd<float>(a, b, n, A, B, ckpt, ws, as_stream(stream));
}

extern "C" pvjp_status pvjp_linrec_scan_vjp(pvjp_dtype dtype, const void* a, const void* b,
                                            const void* yA_bar, const void* yB_bar, int64_t n,
                                            const void* ckpt, void* a_bar, void* b_bar,
                                            int accumulate, void* ws, size_t ws_bytes,
                                            void* stream) {
    clear_error();
    PVJP_REQUIRE(valid_dtype(dtype), "pvjp_linrec_scan_vjp: unknown dtype %d", (int)dtype);
    PVJP_REQUIRE(n >= 0 && n <= kMaxScanN, "pvjp_linrec_scan_vjp: n = %lld out of range", (long long)n);
    if (n == 0) return PVJP_OK;
    PVJP_REQUIRE(a && b && yA_bar && yB_bar && a_bar && b_bar,
                 "pvjp_linrec_scan_vjp: a, b, yA_bar, yB_bar, a_bar, b_bar must be non-NULL");
    PVJP_REQUIRE(ws != nullptr, "pvjp_linrec_scan_vjp: ws is NULL");
    const size_t need = pvjp_linrec_scan_vjp_ws_bytes(dtype, n);
    if (ws_bytes < need) {
        set_error("pvjp_linrec_scan_vjp: workspace has %zu bytes, needs %zu", ws_bytes, need);
        return PVJP_ENOMEM;
    }
    PVJP_REQUIRE(aligned(ws, 256), "pvjp_linrec_scan_vjp: ws must be 256-byte aligned");
    return dtype == PVJP_F64
               ? launch_vjp<double>(a, b, yA_bar, yB_bar, n, ckpt, a_bar, b_bar, accumulate, ws,
                                    as_stream(stream))
               : launch_vjp<float>(a, b, yA_bar, yB_bar, n, ckpt, a_bar, b_bar, accumulate, ws,
                                   as_stream(stream));
}

extern "C" size_t pvjp_linrec_scan_vjp_noalloc_max_bytes(void) { return kNoAllocScratchBytes; }

extern "C" pvjp_status pvjp_linrec_scan_vjp_noalloc(pvjp_dtype dtype, const void* a, const void* b,
                                                    const void* yA_bar, const void* yB_bar, int64_t n,
                                                    const void* ckpt, void* a_bar, void* b_bar, int accumulate,
                                                    void* stream) {
    clear_error();
    PVJP_REQUIRE(valid_dtype(dtype), "pvjp_linrec_scan_vjp_noalloc: unknown dtype %d", (int)dtype);
    PVJP_REQUIRE(n >= 0 && n <= kMaxScanN, "pvjp_linrec_scan_vjp_noalloc: n = %lld out of range", (long long)n);
    if (n == 0) return PVJP_OK;
    PVJP_REQUIRE(a && b && yA_bar && yB_bar && a_bar && b_bar,
                 "pvjp_linrec_scan_vjp_noalloc: a, b, yA_bar, yB_bar, a_bar, b_bar must be non-NULL");
    const size_t need = pvjp_linrec_scan_vjp_ws_bytes(dtype, n);
    if (need > kNoAllocScratchBytes) {
        set_error("pvjp_linrec_scan_vjp_noalloc: n = %lld needs %zu bytes of scratch, beyond the fixed %zu",
                  (long long)n, need, kNoAllocScratchBytes);
        return PVJP_ENOMEM;
    }
    hipStream_t st = as_stream(stream);
    void* ws = nullptr;
    if (pvjp_status s = scratch_for(st, &ws)) return s;
    const pvjp_status s =
        dtype == PVJP_F64 ? launch_vjp<double>(a, b, yA_bar, yB_bar, n, ckpt, a_bar, b_bar, accumulate, ws, st)
                          : launch_vjp<float>(a, b, yA_bar, yB_bar, n, ckpt, a_bar, b_bar, accumulate, ws, st);
    return s;
}
