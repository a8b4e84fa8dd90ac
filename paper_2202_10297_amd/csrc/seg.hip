// Segmented batches: many linear-recurrence scans (and their VJPs) and many
// sum-reduce VJPs of uneven lengths, stored back to back, processed as ONE
// segmented operation per launch (the segmented-scan idea of Sec. 5.2's
// vectorised-operator rule, generalised to irregular segments).
//
//  - Primal (seg_linrec_fwd): one decoupled-lookback scan over the whole
//    concatenation with the segmented operator (a flag restarts the
//    recurrence at each segment head), writing per-segment results and
//    checkpoints every PVJP_LINREC_CKPT_INTERVAL global elements.
//  - Return sweep (seg_batch_vjp): one persistent launch over a queue of
//    work items: first the scan's tile chains, longest first, then every
//    sum-reduce tile.  The lin_o reversed scan needs no flag: the last
//    element of each segment has no successor in its segment, so its c_i is
//    0, which cuts the carry exactly as the end of the array does.  So a
//    tile holding a segment end (a "cut tile") passes to its left a carry
//    that is its own aggregate, whatever lies to its right.  The tiles split
//    into chains: from just left of one cut tile down to the previous cut
//    tile included (the segment table fixes them when the batch is
//    prepared).  A chain's block first folds the cut tile at its right end
//    into its carry (one read of that tile's a and y_bar), then walks the
//    chain right to left, handing the carry from tile to tile in registers:
//    no tile ever waits on another block.  The
//    primal prefixes are recomputed from the checkpoint with the segmented
//    operator.  A sum-reduce tile writes x_bar_i = y_bar[segment of i]
//    (reduce(+)'s adjoint, Sec. 5.1.1).
//
// Segment heads of a tile come from an LDS bitmap built from the tile's first
// segment (a table written once by pvjp_seg_prepare) and the segment offsets.
#include <algorithm>
#include <utility>
#include <vector>

#include "common.h"
#include "prims.h"

namespace pvjp {

constexpr int kSegBlock = 256;
constexpr int kSegCk = PVJP_LINREC_CKPT_INTERVAL;
constexpr int64_t kSumGroup = 16;  // sum tiles per work item of the return sweep

constexpr size_t kSegState = 128;
static_assert(sizeof(TileState<SegLinRec<double>::S>) == kSegState && sizeof(TileState<LinO<double>::S>) == kSegState &&
                  sizeof(TileState<SegLinRec<float>::S>) == kSegState && sizeof(TileState<LinO<float>::S>) == kSegState,
              "tile states of both sweeps share one slot per tile");

// Workspace: [LookbackHdr | tile and group states (128 B each) |
//             tile_seg0 int32[ntiles+1] | offsets int64[nseg+1] |
//             chain count int32 | chains int32[3 * (ntiles + 1)] (right-end
//             tile, number of tiles, cut tile folded into the initial carry
//             or -1; longest first)]
struct SegLayout {
    size_t states, seg0, offs, nchain, chains, total;
    int64_t ntiles;
};

static SegLayout seg_layout(int64_t total, int64_t nseg, int ts) {
    SegLayout L{};
    L.ntiles = ceil_div(total > 0 ? total : 1, ts);
    L.states = sizeof(LookbackHdr);
    L.seg0 = L.states + align_up((size_t)(L.ntiles + lookback_groups(L.ntiles)) * kSegState, 256);
    L.offs = L.seg0 + align_up((size_t)(L.ntiles + 1) * 4, 256);
    L.nchain = L.offs + align_up((size_t)(nseg + 1) * 8, 256);
    L.chains = L.nchain + 256;
    L.total = L.chains + align_up((size_t)(L.ntiles + 1) * 12, 256);
    return L;
}


// Bitmap of segment heads over tile positions 0..TS (position TS is the first
// element of the next tile): bit j set iff base + j starts a segment (or is
// the end of the data).  Segments are non-empty, so a position holds at most
// one head.
template <int TS>
__device__ __forceinline__ void build_heads(uint32_t* bits, const int32_t* __restrict__ seg0,
                                            const int64_t* __restrict__ offs, int64_t nseg, int64_t tile,
                                            int64_t base) {
    constexpr int NW = (TS + 1 + 31) / 32;
    for (int w = threadIdx.x; w < NW; w += kSegBlock) bits[w] = 0u;
    __syncthreads();
    const int64_t s_lo = seg0[tile], s_hi = seg0[tile + 1] + 1;
    for (int64_t s = s_lo + threadIdx.x; s <= s_hi && s <= nseg; s += kSegBlock) {
        const int64_t j = offs[s] - base;
        if (j >= 0 && j <= TS) atomicOr(&bits[j >> 5], 1u << (j & 31));
    }
    __syncthreads();
}

__device__ __forceinline__ bool bit_at(const uint32_t* bits, int j) { return (bits[j >> 5] >> (j & 31)) & 1u; }

// ------------------------------------------------------------------ primal
template <class T, int IPT>
__global__ __launch_bounds__(kSegBlock) void seg_linrec_fwd_kernel(
    const T* __restrict__ a, const T* __restrict__ b, int64_t total, int64_t nseg, const int64_t* __restrict__ offs,
    const int32_t* __restrict__ seg0, T* __restrict__ A, T* __restrict__ B, T* __restrict__ ckpt, LookbackHdr* hdr,
    TileState<typename SegLinRec<T>::S>* states, int64_t ntiles) {
    using Op = SegLinRec<T>;
    using S = typename Op::S;
    constexpr int TS = kSegBlock * IPT;
    __shared__ T lds[lds_elems<T, TS>()];
    __shared__ S wtot[kSegBlock / kWave];
    __shared__ uint32_t bits[(TS + 1 + 31) / 32];
    __shared__ uint32_t s_tag, s_ticket;
    __shared__ S s_prefix;

    if (threadIdx.x == 0) {
        s_ticket = lookback_draw(hdr, (uint32_t)(ntiles - 1), &s_tag);
        if (s_ticket >= ntiles) lookback_error(hdr, kErrTicket);
    }
    __syncthreads();
    const uint32_t tag = s_tag;
    if (s_ticket >= ntiles) return;  // the workspace was not in its rest state: do nothing
    const int64_t tile = s_ticket;
    const int64_t base = tile * TS;
    const int cnt = (int)((total - base) < TS ? (total - base) : TS);
    const int first = (int)threadIdx.x * IPT;

    T ra[IPT], rb[IPT];
    {
        T sa[IPT], sb[IPT];  // both arrays in flight while the head bitmap is built
        load_striped<T, kSegBlock, IPT>(a + base, cnt, sa, T(1));
        load_striped<T, kSegBlock, IPT>(b + base, cnt, sb, T(0));
        build_heads<TS>(bits, seg0, offs, nseg, tile, base);
        striped_to_blocked<T, kSegBlock, IPT>(sa, ra, lds);
        __syncthreads();
        striped_to_blocked<T, kSegBlock, IPT>(sb, rb, lds);
    }

    S e[IPT];
#pragma unroll
    for (int j = 0; j < IPT; ++j) e[j] = S{ra[j], rb[j], (uint32_t)bit_at(bits, first + j), 0u};
    S agg = e[0];
#pragma unroll
    for (int j = 1; j < IPT; ++j) agg = Op::comb(agg, e[j]);
    S tot;
    S excl = block_exclusive_scan<Op, kSegBlock, false>(agg, tot, wtot);
    // A tile holding a segment head restarts the recurrence: its inclusive
    // state is its aggregate, published at once, and only the elements before
    // its first head take the prefix of the tiles to the left (none when the
    // tile starts with a head).
    if (threadIdx.x < kWave) {
        S prefix = Op::id();
        const bool early_inc = tile == 0 || tot.f != 0u;
        if (threadIdx.x == 0) publish(&states[tile], tot, early_inc ? kInc : kAgg, tag);
        if (tile > 0 && !bit_at(bits, 0)) {
            prefix = lookback<Op>(states, states + ntiles, tile, tot, tag, hdr);
            if (!early_inc && threadIdx.x == 0) publish(&states[tile], Op::comb(prefix, tot), kInc, tag);
        }
        if (threadIdx.x == 0) s_prefix = prefix;
    }
    __syncthreads();
    S run = Op::comb(s_prefix, excl);
    if (ckpt != nullptr && (first % kSegCk) == 0 && first < cnt) {
        const int64_t c = (base + first) / kSegCk;
        ckpt[2 * c] = run.a;
        ckpt[2 * c + 1] = run.b;
    }
#pragma unroll
    for (int j = 0; j < IPT; ++j) {
        run = Op::comb(run, e[j]);
        ra[j] = run.a;
        rb[j] = run.b;
    }
    if (A != nullptr) {
        store_blocked<T, kSegBlock, IPT, false>(A + base, cnt, ra, lds);
        store_blocked<T, kSegBlock, IPT, false>(B + base, cnt, rb, lds);
    }
}

// ----------------------------------------------------------- return sweep
// One scan tile of a chain: `carry` is the inclusive lin_o state of the tile
// to its right (the neutral element at the chain's right end); returns this
// tile's inclusive state (valid in every thread), the next tile's carry.
template <class T, int IPT, bool ACC>
__device__ __forceinline__ typename LinO<T>::S seg_scan_vjp_tile(const T* __restrict__ a, const T* __restrict__ b,
                                                                 const T* __restrict__ ya, const T* __restrict__ yb,
                                                                 int64_t total, const T* __restrict__ ckpt,
                                                                 T* __restrict__ abar, T* __restrict__ bbar,
                                                                 int64_t tile, typename LinO<T>::S carry, T* lds,
                                                                 const uint32_t* bits,
                                                                 typename SegLinRec<T>::S* wtot_p,
                                                                 typename LinO<T>::S* wtot_l) {
    using P = SegLinRec<T>;
    using L = LinO<T>;
    using PS = typename P::S;
    using LS = typename L::S;
    constexpr int TS = kSegBlock * IPT;
    const int64_t base = tile * TS;
    const int cnt = (int)((total - base) < TS ? (total - base) : TS);
    const int first = (int)threadIdx.x * IPT;

    // all four arrays in flight before the first transpose
    T ra[IPT], rc[IPT], rb[IPT], rya[IPT], ryb[IPT];
    {
        T sa[IPT], sb[IPT], sya[IPT], syb[IPT];
        load_striped<T, kSegBlock, IPT>(a + base, cnt, sa, T(1));
        load_striped<T, kSegBlock, IPT>(b + base, cnt, sb, T(0));
        load_striped<T, kSegBlock, IPT>(ya + base, cnt, sya, T(0));
        load_striped<T, kSegBlock, IPT>(yb + base, cnt, syb, T(0));
        const T after = ((int)threadIdx.x == kSegBlock - 1 && base + TS < total) ? a[base + TS] : T(1);
        striped_to_blocked<T, kSegBlock, IPT>(sa, ra, lds);
        const T nxt = ((int)threadIdx.x < kSegBlock - 1) ? lds[lds_pad<T>(first + IPT)] : after;
#pragma unroll
        for (int j = 0; j < IPT - 1; ++j) rc[j] = ra[j + 1];
        rc[IPT - 1] = nxt;
        __syncthreads();
        striped_to_blocked<T, kSegBlock, IPT>(sb, rb, lds);
        __syncthreads();
        striped_to_blocked<T, kSegBlock, IPT>(sya, rya, lds);
        __syncthreads();
        striped_to_blocked<T, kSegBlock, IPT>(syb, ryb, lds);
    }

    // 1. primal prefixes (A_{i-1}, B_{i-1}) within each segment
    T pA[IPT], pB[IPT];
    {
        PS pe[IPT];
#pragma unroll
        for (int j = 0; j < IPT; ++j) pe[j] = PS{ra[j], rb[j], (uint32_t)bit_at(bits, first + j), 0u};
        PS pagg = pe[0];
#pragma unroll
        for (int j = 1; j < IPT; ++j) pagg = P::comb(pagg, pe[j]);
        PS ptot;
        PS pexcl = block_exclusive_scan<P, kSegBlock, false>(pagg, ptot, wtot_p);
        const int64_t c = base / kSegCk;
        PS run = P::comb(PS{ckpt[2 * c], ckpt[2 * c + 1], 0u, 0u}, pexcl);
#pragma unroll
        for (int j = 0; j < IPT; ++j) {
            const bool head = pe[j].f != 0u;
            pA[j] = head ? T(1) : run.a;
            pB[j] = head ? T(0) : run.b;
            run = P::comb(run, pe[j]);
        }
    }
    // 2. lin_o elements: c_i = a_{i+1}, or 0 when i ends its segment
    LS e[IPT];
#pragma unroll
    for (int j = 0; j < IPT; ++j) {
        const bool last = bit_at(bits, first + j + 1);
        e[j] = LS{last ? T(0) : rc[j], rya[j], ryb[j]};
    }
    // 3. reversed scan inside the tile, after the carry from the right
    LS agg = L::id();
#pragma unroll
    for (int j = IPT - 1; j >= 0; --j) agg = L::comb(agg, e[j]);
    LS tot;
    LS excl = block_exclusive_scan<L, kSegBlock, true>(agg, tot, wtot_l);
    // 4. input adjoints
    LS run = L::comb(carry, excl);
#pragma unroll
    for (int j = IPT - 1; j >= 0; --j) {
        run = L::comb(run, e[j]);
        ra[j] = pA[j] * run.dA + pB[j] * run.dB;
        rb[j] = run.dB;
    }
    store_blocked<T, kSegBlock, IPT, ACC>(abar + base, cnt, ra, lds);
    store_blocked<T, kSegBlock, IPT, ACC>(bbar + base, cnt, rb, lds);
    return L::comb(carry, tot);
}

template <class T, int IPT, bool ACC>
__device__ __forceinline__ void seg_sum_vjp_tile(int64_t total, const int32_t* __restrict__ seg0,
                                                 const T* __restrict__ ybar, T* __restrict__ xbar, int64_t tile,
                                                 const uint32_t* bits, T* lds, IntSum::S* wtot_i) {
    constexpr int TS = kSegBlock * IPT;
    const int64_t base = tile * TS;
    const int cnt = (int)((total - base) < TS ? (total - base) : TS);
    const int first = (int)threadIdx.x * IPT;
    // The segment of tile position j is seg0[tile] plus the number of heads at
    // positions 1..j: a block exclusive scan of per-thread head counts, then a
    // walk over the thread's own items.
    int mine = 0;
#pragma unroll
    for (int j = 0; j < IPT; ++j) mine += (first + j > 0 && bit_at(bits, first + j)) ? 1 : 0;
    IntSum::S tot;
    int seg = seg0[tile] + block_exclusive_scan<IntSum, kSegBlock, false>(IntSum::S{mine}, tot, wtot_i).v;
    T out[IPT];
#pragma unroll
    for (int j = 0; j < IPT; ++j) {
        if (first + j > 0 && bit_at(bits, first + j)) ++seg;
        out[j] = (first + j < cnt) ? ybar[seg] : T(0);
    }
    store_blocked<T, kSegBlock, IPT, ACC>(xbar + base, cnt, out, lds);
}

// The lin_o aggregate of one tile (c_i = a_{i+1}, 0 at segment ends; d_i =
// y_bar_i), folded right to left; valid in every thread.
template <class T, int IPT>
__device__ __forceinline__ typename LinO<T>::S seg_tile_linagg(const T* __restrict__ a, const T* __restrict__ ya,
                                                               const T* __restrict__ yb, int64_t total, int64_t tile,
                                                               T* lds, const uint32_t* bits,
                                                               typename LinO<T>::S* wtot_l) {
    using L = LinO<T>;
    using LS = typename L::S;
    constexpr int TS = kSegBlock * IPT;
    const int64_t base = tile * TS;
    const int cnt = (int)((total - base) < TS ? (total - base) : TS);
    const int first = (int)threadIdx.x * IPT;
    T ra[IPT], rc[IPT], rya[IPT], ryb[IPT];
    {
        T sa[IPT], sya[IPT], syb[IPT];
        load_striped<T, kSegBlock, IPT>(a + base, cnt, sa, T(1));
        load_striped<T, kSegBlock, IPT>(ya + base, cnt, sya, T(0));
        load_striped<T, kSegBlock, IPT>(yb + base, cnt, syb, T(0));
        const T after = ((int)threadIdx.x == kSegBlock - 1 && base + TS < total) ? a[base + TS] : T(1);
        striped_to_blocked<T, kSegBlock, IPT>(sa, ra, lds);
        const T nxt = ((int)threadIdx.x < kSegBlock - 1) ? lds[lds_pad<T>(first + IPT)] : after;
#pragma unroll
        for (int j = 0; j < IPT - 1; ++j) rc[j] = ra[j + 1];
        rc[IPT - 1] = nxt;
        __syncthreads();
        striped_to_blocked<T, kSegBlock, IPT>(sya, rya, lds);
        __syncthreads();
        striped_to_blocked<T, kSegBlock, IPT>(syb, ryb, lds);
    }
    LS agg = L::id();
#pragma unroll
    for (int j = IPT - 1; j >= 0; --j) {
        const bool last = bit_at(bits, first + j + 1);
        agg = L::comb(agg, LS{last ? T(0) : rc[j], rya[j], ryb[j]});
    }
    LS tot;
    (void)block_exclusive_scan<L, kSegBlock, true>(agg, tot, wtot_l);
    return tot;
}

template <class T, int IPT, bool ACC>
__global__ __launch_bounds__(kSegBlock) void seg_batch_vjp_kernel(
    const T* __restrict__ a, const T* __restrict__ b, const T* __restrict__ ya, const T* __restrict__ yb,
    int64_t total, int64_t nseg, const int64_t* __restrict__ offs, const int32_t* __restrict__ seg0,
    const T* __restrict__ ckpt, T* __restrict__ abar, T* __restrict__ bbar, const T* __restrict__ sum_ybar,
    T* __restrict__ sum_xbar, LookbackHdr* hdr, const int32_t* __restrict__ nchain_p,
    const int32_t* __restrict__ chains, int64_t ntiles, int scan, int64_t nsum) {
    constexpr int TS = kSegBlock * IPT;
    __shared__ T lds[lds_elems<T, TS>()];
    __shared__ typename SegLinRec<T>::S wtot_p[kSegBlock / kWave];
    __shared__ typename LinO<T>::S wtot_l[kSegBlock / kWave];
    __shared__ IntSum::S wtot_i[kSegBlock / kWave];
    __shared__ uint32_t bits[(TS + 1 + 31) / 32];
    __shared__ uint32_t s_ticket;

    const int64_t nscan = scan ? (int64_t)*nchain_p : 0;
    // every block makes one final, empty draw: the launch's last ticket
    const uint32_t last = (uint32_t)(nscan + nsum + gridDim.x - 1);
    if (threadIdx.x == 0) {
        s_ticket = lookback_draw(hdr, last, nullptr);
        if (s_ticket > last) lookback_error(hdr, kErrTicket);
    }
    __syncthreads();
    if (s_ticket > last) return;  // the workspace was not in its rest state: do nothing
    // Queue: items [0, nscan) are the scan's tile chains (longest first),
    // items [nscan, nscan + nsum) runs of kSumGroup sum tiles.  No item waits
    // on another.
    while (true) {
        const int64_t item = s_ticket;
        if (item >= nscan + nsum) break;
        if (item < nscan) {
            const int64_t t1 = chains[3 * item], len = chains[3 * item + 1], cut = chains[3 * item + 2];
            typename LinO<T>::S carry = LinO<T>::id();
            if (cut >= 0) {  // the cut tile right of the chain: its aggregate is the carry
                build_heads<TS>(bits, seg0, offs, nseg, cut, cut * TS);
                carry = seg_tile_linagg<T, IPT>(a, ya, yb, total, cut, lds, bits, wtot_l);
                __syncthreads();
            }
            for (int64_t t = t1; t > t1 - len; --t) {
                build_heads<TS>(bits, seg0, offs, nseg, t, t * TS);
                carry = seg_scan_vjp_tile<T, IPT, ACC>(a, b, ya, yb, total, ckpt, abar, bbar, t, carry, lds, bits,
                                                       wtot_p, wtot_l);
                __syncthreads();
            }
        } else {
            // a sum item is a run of kSumGroup tiles: one ticket per run keeps
            // the queue's counter (one device-scope atomic per draw, serialised
            // on one address) off the critical path
            const int64_t t0 = (item - nscan) * kSumGroup;
            const int64_t t1 = (t0 + kSumGroup < ntiles) ? t0 + kSumGroup : ntiles;
            for (int64_t tile = t0; tile < t1; ++tile) {
                build_heads<TS>(bits, seg0, offs, nseg, tile, tile * TS);
                seg_sum_vjp_tile<T, IPT, ACC>(total, seg0, sum_ybar, sum_xbar, tile, bits, lds, wtot_i);
                __syncthreads();
            }
        }
        __syncthreads();
        if (threadIdx.x == 0) s_ticket = lookback_draw(hdr, last, nullptr);
        __syncthreads();
    }
}

// ------------------------------------------------------------------ host
static bool valid_tile(int ts) { return ts == 1024 || ts == 2048 || ts == 4096; }

template <class T, int IPT>
static void launch_fwd(const void* a, const void* b, int64_t total, int64_t nseg, void* A, void* B, void* ckpt,
                       char* ws, const SegLayout& L, hipStream_t st) {
    hipLaunchKernelGGL((seg_linrec_fwd_kernel<T, IPT>), dim3((unsigned)L.ntiles), dim3(kSegBlock), 0, st,
                       (const T*)a, (const T*)b, total, nseg, (const int64_t*)(ws + L.offs),
                       (const int32_t*)(ws + L.seg0), (T*)A, (T*)B, (T*)ckpt, (LookbackHdr*)ws,
                       (TileState<typename SegLinRec<T>::S>*)(ws + L.states), L.ntiles);
}

template <class T, int IPT, bool ACC>
static void launch_batch(const void* a, const void* b, const void* ya, const void* yb, int64_t total, int64_t nseg,
                         const void* ckpt, void* abar, void* bbar, const void* sy, void* sx, int grid, char* ws,
                         const SegLayout& L, hipStream_t st) {
    hipLaunchKernelGGL((seg_batch_vjp_kernel<T, IPT, ACC>), dim3((unsigned)grid), dim3(kSegBlock), 0, st, (const T*)a,
                       (const T*)b, (const T*)ya, (const T*)yb, total, nseg, (const int64_t*)(ws + L.offs),
                       (const int32_t*)(ws + L.seg0), (const T*)ckpt, (T*)abar, (T*)bbar, (const T*)sy, (T*)sx,
                       (LookbackHdr*)ws, (const int32_t*)(ws + L.nchain), (const int32_t*)(ws + L.chains), L.ntiles,
                       a ? 1 : 0, sy ? ceil_div(L.ntiles, kSumGroup) : 0);
}

template <class T, bool ACC>
static void dispatch_batch(int ts, const void* a, const void* b, const void* ya, const void* yb, int64_t total,
                           int64_t nseg, const void* ckpt, void* abar, void* bbar, const void* sy, void* sx, int grid,
                           char* ws, const SegLayout& L, hipStream_t st) {
    if (ts == 1024)
        launch_batch<T, 1024 / kSegBlock, ACC>(a, b, ya, yb, total, nseg, ckpt, abar, bbar, sy, sx, grid, ws, L, st);
    else if (ts == 2048)
        launch_batch<T, 2048 / kSegBlock, ACC>(a, b, ya, yb, total, nseg, ckpt, abar, bbar, sy, sx, grid, ws, L, st);
    else
        launch_batch<T, 4096 / kSegBlock, ACC>(a, b, ya, yb, total, nseg, ckpt, abar, bbar, sy, sx, grid, ws, L, st);
}

}  // namespace pvjp

using namespace pvjp;

extern "C" size_t pvjp_seg_ws_bytes(int64_t total, int64_t nseg, int tile_elems) {
    if (total < 1 || nseg < 1 || !valid_tile(tile_elems)) return 0;
    return seg_layout(total, nseg, tile_elems).total;
}

extern "C" pvjp_status pvjp_seg_prepare(const int64_t* host_offsets, int64_t nseg, int tile_elems, void* ws,
                                        size_t ws_bytes, void* stream) {
    clear_error();
    PVJP_REQUIRE(host_offsets != nullptr && nseg >= 1, "pvjp_seg_prepare: need host offsets of nseg >= 1 segments");
    PVJP_REQUIRE(valid_tile(tile_elems), "pvjp_seg_prepare: tile_elems must be 1024, 2048 or 4096");
    PVJP_REQUIRE(host_offsets[0] == 0, "pvjp_seg_prepare: offsets[0] must be 0");
    for (int64_t s = 0; s < nseg; ++s)
        PVJP_REQUIRE(host_offsets[s + 1] > host_offsets[s], "pvjp_seg_prepare: segment %lld is empty or offsets decrease",
                     (long long)s);
    const int64_t total = host_offsets[nseg];
    PVJP_REQUIRE(total <= ((int64_t)1 << 40), "pvjp_seg_prepare: total length out of range");
    PVJP_REQUIRE(ws != nullptr && aligned(ws, 256), "pvjp_seg_prepare: ws must be non-NULL and 256-byte aligned");
    const SegLayout L = seg_layout(total, nseg, tile_elems);
    if (ws_bytes < L.total) {
        set_error("pvjp_seg_prepare: workspace has %zu bytes, needs %zu", ws_bytes, L.total);
        return PVJP_ENOMEM;
    }
    std::vector<int32_t> seg0((size_t)L.ntiles + 1);
    int64_t s = 0;
    for (int64_t t = 0; t < L.ntiles; ++t) {
        const int64_t base = t * tile_elems;
        while (host_offsets[s + 1] <= base) ++s;
        seg0[(size_t)t] = (int32_t)s;
    }
    seg0[(size_t)L.ntiles] = (int32_t)nseg;
    // Tile chains of the return sweep.  A cut tile holds a segment end (the
    // last tile holds the end of the data); with the cut tiles c_0 < ... <
    // c_K, chain k covers tiles c_{k-1} .. c_k - 1 (0 .. c_0 - 1 for k = 0)
    // and starts from the carry of c_k's aggregate; a last chain holds c_K
    // alone with the neutral carry.  Longest first, so the queue's tail
    // holds short work.
    std::vector<char> cutv((size_t)L.ntiles, 0);
    for (int64_t s2 = 1; s2 <= nseg; ++s2) cutv[(size_t)((host_offsets[s2] - 1) / tile_elems)] = 1;
    struct Chain {
        int32_t len, right, cut;
    };
    std::vector<Chain> ch;
    {
        int64_t prev = -1;  // previous cut tile (-1: none)
        for (int64_t t = 0; t < L.ntiles; ++t) {
            if (!cutv[(size_t)t]) continue;
            const int64_t left = prev < 0 ? 0 : prev;
            if (t - 1 >= left) ch.push_back(Chain{(int32_t)(t - left), (int32_t)(t - 1), (int32_t)t});
            prev = t;
        }
        ch.push_back(Chain{1, (int32_t)(L.ntiles - 1), -1});  // the last tile is a cut tile
    }
    std::stable_sort(ch.begin(), ch.end(), [](const Chain& x, const Chain& y) { return x.len > y.len; });
    std::vector<int32_t> chains(3 * ch.size());
    for (size_t i = 0; i < ch.size(); ++i)
        chains[3 * i] = ch[i].right, chains[3 * i + 1] = ch[i].len, chains[3 * i + 2] = ch[i].cut;
    const int32_t nchain = (int32_t)ch.size();
    char* w = reinterpret_cast<char*>(ws);
    hipStream_t st = as_stream(stream);
    if (hipMemcpyAsync(w + L.seg0, seg0.data(), seg0.size() * 4, hipMemcpyHostToDevice, st) != hipSuccess ||
        hipMemcpyAsync(w + L.offs, host_offsets, (size_t)(nseg + 1) * 8, hipMemcpyHostToDevice, st) != hipSuccess ||
        hipMemcpyAsync(w + L.nchain, &nchain, 4, hipMemcpyHostToDevice, st) != hipSuccess ||
        hipMemcpyAsync(w + L.chains, chains.data(), chains.size() * 4, hipMemcpyHostToDevice, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess) {
        set_error("pvjp_seg_prepare: uploading the segment tables failed");
        return PVJP_EDEVICE;
    }
    return PVJP_OK;
}

extern "C" pvjp_status pvjp_seg_linrec_scan(pvjp_dtype dtype, const void* a, const void* b, int64_t total, int64_t nseg,
                                            int tile_elems, void* A, void* B, void* ckpt, void* ws, size_t ws_bytes,
                                            void* stream) {
    clear_error();
    PVJP_REQUIRE(valid_dtype(dtype), "pvjp_seg_linrec_scan: unknown dtype %d", (int)dtype);
    PVJP_REQUIRE(total >= 1 && nseg >= 1, "pvjp_seg_linrec_scan: total and nseg must be >= 1");
    PVJP_REQUIRE(valid_tile(tile_elems), "pvjp_seg_linrec_scan: tile_elems must be 1024, 2048 or 4096");
    PVJP_REQUIRE(a && b, "pvjp_seg_linrec_scan: a and b must be non-NULL");
    PVJP_REQUIRE((A == nullptr) == (B == nullptr) && (A || ckpt), "pvjp_seg_linrec_scan: need A and B, or ckpt");
    PVJP_REQUIRE(ws != nullptr && aligned(ws, 256), "pvjp_seg_linrec_scan: ws must be non-NULL and 256-byte aligned");
    const SegLayout L = seg_layout(total, nseg, tile_elems);
    if (ws_bytes < L.total) {
        set_error("pvjp_seg_linrec_scan: workspace has %zu bytes, needs %zu", ws_bytes, L.total);
        return PVJP_ENOMEM;
    }
    char* w = reinterpret_cast<char*>(ws);
    hipStream_t st = as_stream(stream);
    if (dtype == PVJP_F64) {
        if (tile_elems == 1024) launch_fwd<double, 4>(a, b, total, nseg, A, B, ckpt, w, L, st);
        else if (tile_elems == 2048) launch_fwd<double, 8>(a, b, total, nseg, A, B, ckpt, w, L, st);
        else launch_fwd<double, 16>(a, b, total, nseg, A, B, ckpt, w, L, st);
    } else {
        if (tile_elems == 1024) launch_fwd<float, 4>(a, b, total, nseg, A, B, ckpt, w, L, st);
        else if (tile_elems == 2048) launch_fwd<float, 8>(a, b, total, nseg, A, B, ckpt, w, L, st);
        else launch_fwd<float, 16>(a, b, total, nseg, A, B, ckpt, w, L, st);
    }
    PVJP_LAUNCHED("pvjp_seg_linrec_scan");
    return PVJP_OK;
}

extern "C" pvjp_status pvjp_seg_batch_vjp(pvjp_dtype dtype, const void* a, const void* b, const void* yA_bar,
                                          const void* yB_bar, int64_t total, int64_t nseg, int tile_elems,
                                          const void* ckpt, void* a_bar, void* b_bar, const void* sum_ybar,
                                          void* sum_xbar, int accumulate, int grid_blocks, void* ws, size_t ws_bytes,
                                          void* stream) {
    clear_error();
    PVJP_REQUIRE(valid_dtype(dtype), "pvjp_seg_batch_vjp: unknown dtype %d", (int)dtype);
    PVJP_REQUIRE(total >= 1 && nseg >= 1, "pvjp_seg_batch_vjp: total and nseg must be >= 1");
    PVJP_REQUIRE(valid_tile(tile_elems), "pvjp_seg_batch_vjp: tile_elems must be 1024, 2048 or 4096");
    const bool scan = a != nullptr;
    PVJP_REQUIRE(!scan || (b && yA_bar && yB_bar && ckpt && a_bar && b_bar),
                 "pvjp_seg_batch_vjp: the scan part needs b, yA_bar, yB_bar, ckpt, a_bar and b_bar");
    PVJP_REQUIRE((sum_ybar == nullptr) == (sum_xbar == nullptr), "pvjp_seg_batch_vjp: sum_ybar and sum_xbar go together");
    PVJP_REQUIRE(scan || sum_ybar, "pvjp_seg_batch_vjp: nothing to compute");
    PVJP_REQUIRE(grid_blocks >= 1 && grid_blocks <= 65536, "pvjp_seg_batch_vjp: grid_blocks out of range [1, 65536]");
    PVJP_REQUIRE(ws != nullptr && aligned(ws, 256), "pvjp_seg_batch_vjp: ws must be non-NULL and 256-byte aligned");
    const SegLayout L = seg_layout(total, nseg, tile_elems);
    if (ws_bytes < L.total) {
        set_error("pvjp_seg_batch_vjp: workspace has %zu bytes, needs %zu", ws_bytes, L.total);
        return PVJP_ENOMEM;
    }
    char* w = reinterpret_cast<char*>(ws);
    hipStream_t st = as_stream(stream);
    if (dtype == PVJP_F64) {
        if (accumulate)
            dispatch_batch<double, true>(tile_elems, a, b, yA_bar, yB_bar, total, nseg, ckpt, a_bar, b_bar, sum_ybar,
                                         sum_xbar, grid_blocks, w, L, st);
        else
            dispatch_batch<double, false>(tile_elems, a, b, yA_bar, yB_bar, total, nseg, ckpt, a_bar, b_bar, sum_ybar,
                                          sum_xbar, grid_blocks, w, L, st);
    } else {
        if (accumulate)
            dispatch_batch<float, true>(tile_elems, a, b, yA_bar, yB_bar, total, nseg, ckpt, a_bar, b_bar, sum_ybar,
                                        sum_xbar, grid_blocks, w, L, st);
        else
            dispatch_batch<float, false>(tile_elems, a, b, yA_bar, yB_bar, total, nseg, ckpt, a_bar, b_bar, sum_ybar,
                                         sum_xbar, grid_blocks, w, L, st);
    }
    PVJP_LAUNCHED("pvjp_seg_batch_vjp");
    return PVJP_OK;
}
