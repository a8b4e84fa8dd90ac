// Device primitives for gfx950 (CDNA4, wave64): shuffles of small structs,
// wave/block scans of an arbitrary associative operator in forward or reverse
// order, LDS transposes between striped (coalesced) and blocked (per-thread
// contiguous) layouts, and a single-pass decoupled lookback whose virtual
// tile order can run forward (a scan) or backward (the reversed scan of a
// VJP, Sec. 5.2).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pvjp {

constexpr int kWave = 64;

// ---------------------------------------------------------------- shuffles
template <class T>
__device__ __forceinline__ T shfl_up1(T v, int d) { return __shfl_up(v, d, kWave); }
template <class T>
__device__ __forceinline__ T shfl_down1(T v, int d) { return __shfl_down(v, d, kWave); }
template <class T>
__device__ __forceinline__ T shfl_idx1(T v, int s) { return __shfl(v, s, kWave); }

// ---------------------------------------------------------- scan operators
// An operator type provides a state S, the neutral element id(), the
// associative combination comb(earlier, later) in scan order, and lane
// shuffles of S.  "Earlier" means earlier in the direction the scan runs.

// First-order linear recurrence (A, B): (a1,b1) (+) (a2,b2) = (a2*a1, a2*b1+b2).
template <class T>
struct LinRec {
    struct S {
        T a, b;
    };
    __device__ static __forceinline__ S id() { return S{T(1), T(0)}; }
    __device__ static __forceinline__ S comb(S x, S y) { return S{y.a * x.a, y.a * x.b + y.b}; }
    __device__ static __forceinline__ S up(S v, int d) { return S{shfl_up1(v.a, d), shfl_up1(v.b, d)}; }
    __device__ static __forceinline__ S down(S v, int d) { return S{shfl_down1(v.a, d), shfl_down1(v.b, d)}; }
    __device__ static __forceinline__ S idx(S v, int s) { return S{shfl_idx1(v.a, s), shfl_idx1(v.b, s)}; }
};

// Composition of the affine maps r -> d + c*r with a vector d = (dA, dB) and a
// scalar-times-identity Jacobian c (lin_o of Sec. 5.2):
// lin_o((d1,c1),(d2,c2)) = (d2 + c2*d1, c2*c1), neutral (0, 1).
template <class T>
struct LinO {
    struct S {
        T c, dA, dB;
    };
    __device__ static __forceinline__ S id() { return S{T(1), T(0), T(0)}; }
    __device__ static __forceinline__ S comb(S x, S y) {
        return S{y.c * x.c, y.dA + y.c * x.dA, y.dB + y.c * x.dB};
    }
    __device__ static __forceinline__ S up(S v, int d) {
        return S{shfl_up1(v.c, d), shfl_up1(v.dA, d), shfl_up1(v.dB, d)};
    }
    __device__ static __forceinline__ S down(S v, int d) {
        return S{shfl_down1(v.c, d), shfl_down1(v.dA, d), shfl_down1(v.dB, d)};
    }
    __device__ static __forceinline__ S idx(S v, int s) {
        return S{shfl_idx1(v.c, s), shfl_idx1(v.dA, s), shfl_idx1(v.dB, s)};
    }
};

// The linear recurrence restarted at segment heads (the standard segmented
// form of an operator): a state carries a flag "contains a segment start";
// combining with a later flagged state discards the earlier one.
template <class T>
struct SegLinRec {
    struct S {
        T a, b;
        uint32_t f, pad;
    };
    __device__ static __forceinline__ S id() { return S{T(1), T(0), 0u, 0u}; }
    __device__ static __forceinline__ S comb(S x, S y) {
        return y.f ? y : S{y.a * x.a, y.a * x.b + y.b, x.f, 0u};
    }
    __device__ static __forceinline__ S up(S v, int d) {
        return S{shfl_up1(v.a, d), shfl_up1(v.b, d), (uint32_t)shfl_up1((int)v.f, d), 0u};
    }
    __device__ static __forceinline__ S down(S v, int d) {
        return S{shfl_down1(v.a, d), shfl_down1(v.b, d), (uint32_t)shfl_down1((int)v.f, d), 0u};
    }
    __device__ static __forceinline__ S idx(S v, int s) {
        return S{shfl_idx1(v.a, s), shfl_idx1(v.b, s), (uint32_t)shfl_idx1((int)v.f, s), 0u};
    }
};

// Integer sum (counts of segment heads).
struct IntSum {
    struct S {
        int v;
    };
    __device__ static __forceinline__ S id() { return S{0}; }
    __device__ static __forceinline__ S comb(S x, S y) { return S{x.v + y.v}; }
    __device__ static __forceinline__ S up(S v, int d) { return S{shfl_up1(v.v, d)}; }
    __device__ static __forceinline__ S down(S v, int d) { return S{shfl_down1(v.v, d)}; }
    __device__ static __forceinline__ S idx(S v, int s) { return S{shfl_idx1(v.v, s)}; }
};

// ------------------------------------------------------------- block scan
// Exclusive scan over the threads of a block in scan order.  With REV the
// scan order of threads is reversed (thread BLOCK-1 first).  `agg` is the
// thread's aggregate; returns the thread's exclusive prefix and writes the
// block total.  `wtot` is LDS scratch of BLOCK/64 states.
template <class Op, int BLOCK, bool REV>
__device__ __forceinline__ typename Op::S block_exclusive_scan(typename Op::S agg,
                                                               typename Op::S& total,
                                                               typename Op::S* wtot) {
    using S = typename Op::S;
    constexpr int NW = BLOCK / kWave;
    const int lane = threadIdx.x & (kWave - 1);
    const int wid = threadIdx.x / kWave;
    S v = agg;
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        S o = REV ? Op::down(v, d) : Op::up(v, d);
        bool ok = REV ? (lane + d < kWave) : (lane >= d);
        if (ok) v = Op::comb(o, v);
    }
    S ex = REV ? Op::down(v, 1) : Op::up(v, 1);
    if (REV ? (lane == kWave - 1) : (lane == 0)) ex = Op::id();
    if (lane == (REV ? 0 : kWave - 1)) wtot[wid] = v;
    __syncthreads();
    S wpre = Op::id();
    S tot = Op::id();
#pragma unroll
    for (int k = 0; k < NW; ++k) {
        const int w = REV ? NW - 1 - k : k;
        if (w == wid) wpre = tot;
        tot = Op::comb(tot, wtot[w]);
    }
    total = tot;
    __syncthreads();
    return Op::comb(wpre, ex);
}

// Exclusive scan over the lanes of one wave in scan order (REV: lane 63
// first); every lane holds one state.
template <class Op, bool REV>
__device__ __forceinline__ typename Op::S wave_exclusive_scan(typename Op::S v) {
    const int lane = threadIdx.x & (kWave - 1);
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        const typename Op::S o = REV ? Op::down(v, d) : Op::up(v, d);
        if (REV ? (lane + d < kWave) : (lane >= d)) v = Op::comb(o, v);
    }
    typename Op::S ex = REV ? Op::down(v, 1) : Op::up(v, 1);
    if (REV ? (lane == kWave - 1) : (lane == 0)) ex = Op::id();
    return ex;
}

// --------------------------------------------- scans of tile aggregates
// A reduce-then-scan over many tiles scans the tiles' aggregates in scan
// order (increasing tile index, or decreasing with REV).  One block walking
// tens of thousands of aggregates is slow (100-200 us at 32K), so tiles are
// taken in groups of 64, one wave per group: group_fold_kernel folds each
// group, agg_scan_kernel scans the group folds, group_prefix_kernel gives
// every tile its group's prefix folded with the group's tiles before it.
// blockIdx.y selects one of several independent scans laid out back to back
// (segment y's tiles at y nt, its groups at y ng); a 1-D grid is segment 0.
constexpr int kAggBlock = 1024;
constexpr int kAggGroup = kWave;
constexpr int kGroupBlock = 256;

// pre[i] = exclusive fold of agg in scan order.  Thread t folds a contiguous
// run of the scan order, the runs are scanned across the block, then each
// thread writes its run's prefixes.
template <class Op, bool REV>
__global__ __launch_bounds__(kAggBlock) void agg_scan_kernel(const typename Op::S* __restrict__ agg, int64_t cnt,
                                                             typename Op::S* __restrict__ pre) {
    using S = typename Op::S;
    __shared__ S wtot[kAggBlock / kWave];
    agg += (int64_t)blockIdx.y * cnt;
    pre += (int64_t)blockIdx.y * cnt;
    const int64_t per = (cnt + kAggBlock - 1) / kAggBlock;
    const int64_t v0 = (int64_t)threadIdx.x * per;
    const int64_t v1 = (v0 + per < cnt) ? v0 + per : cnt;
    auto at = [&](int64_t v) { return REV ? cnt - 1 - v : v; };
    S run = Op::id();
    for (int64_t v = v0; v < v1; ++v) run = Op::comb(run, agg[at(v)]);
    S total;
    S ex = block_exclusive_scan<Op, kAggBlock, false>(run, total, wtot);
    for (int64_t v = v0; v < v1; ++v) {
        pre[at(v)] = ex;
        ex = Op::comb(ex, agg[at(v)]);
    }
}

template <class Op, bool REV>
__global__ __launch_bounds__(kGroupBlock) void group_fold_kernel(const typename Op::S* __restrict__ agg, int64_t nt,
                                                                 int64_t ng, typename Op::S* __restrict__ gagg) {
    using S = typename Op::S;
    agg += (int64_t)blockIdx.y * nt;
    gagg += (int64_t)blockIdx.y * ng;
    const int64_t g = (int64_t)blockIdx.x * (kGroupBlock / kWave) + threadIdx.x / kWave;
    if (g >= ng) return;  // whole waves leave together
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t t = g * kAggGroup + lane;
    const S own = t < nt ? agg[t] : Op::id();
    const S inc = Op::comb(wave_exclusive_scan<Op, REV>(own), own);
    if (lane == (REV ? 0 : kWave - 1)) gagg[g] = inc;  // the last lane in scan order
}

template <class Op, bool REV>
__global__ __launch_bounds__(kGroupBlock) void group_prefix_kernel(const typename Op::S* __restrict__ agg, int64_t nt,
                                                                   int64_t ng, const typename Op::S* __restrict__ gpre,
                                                                   typename Op::S* __restrict__ pre) {
    using S = typename Op::S;
    agg += (int64_t)blockIdx.y * nt;
    gpre += (int64_t)blockIdx.y * ng;
    pre += (int64_t)blockIdx.y * nt;
    const int64_t g = (int64_t)blockIdx.x * (kGroupBlock / kWave) + threadIdx.x / kWave;
    if (g >= ng) return;
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t t = g * kAggGroup + lane;
    const S own = t < nt ? agg[t] : Op::id();
    const S ex = wave_exclusive_scan<Op, REV>(own);
    if (t < nt) pre[t] = Op::comb(gpre[g], ex);
}

// ------------------------------------------------------- LDS transposes
// Padded LDS index: one element of padding per 256 bytes keeps both the
// striped writes and the blocked reads free of bank conflicts for the
// items-per-thread counts used here.
template <class T>
__device__ __forceinline__ int lds_pad(int i) {
    return i + i / (256 / (int)sizeof(T));
}
template <class T, int TS>
constexpr int lds_elems() {
    return TS + TS / (256 / (int)sizeof(T)) + 1;
}

// Striped coalesced global load of a tile, returned in blocked order
// (thread t holds tile elements t*IPT .. t*IPT+IPT-1).  Elements at or past
// `cnt` read as `fill`.  Ends with the LDS buffer still holding the tile (a
// caller may read extra elements before the next barrier).
template <class T, int BLOCK, int IPT>
__device__ __forceinline__ void load_blocked(const T* __restrict__ src, int cnt, T (&items)[IPT],
                                             T* lds, T fill) {
#pragma unroll
    for (int k = 0; k < IPT; ++k) {
        const int i = k * BLOCK + (int)threadIdx.x;
        lds[lds_pad<T>(i)] = (i < cnt) ? src[i] : fill;
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < IPT; ++j) items[j] = lds[lds_pad<T>((int)threadIdx.x * IPT + j)];
}

// The two halves of load_blocked, so that a tile's several input arrays
// can all be in flight before the first is transposed: a striped coalesced
// load into registers (element k*BLOCK + t in slot k of thread t; `fill`
// past `cnt`), then the LDS transpose of those registers into blocked
// order.  The transpose ends with the LDS buffer holding the tile; the
// caller puts a barrier before reusing the buffer.
template <class T, int BLOCK, int IPT>
__device__ __forceinline__ void load_striped(const T* __restrict__ src, int cnt, T (&st)[IPT], T fill) {
#pragma unroll
    for (int k = 0; k < IPT; ++k) {
        const int i = k * BLOCK + (int)threadIdx.x;
        st[k] = (i < cnt) ? src[i] : fill;
    }
}

template <class T, int BLOCK, int IPT>
__device__ __forceinline__ void striped_to_blocked(const T (&st)[IPT], T (&items)[IPT], T* lds) {
#pragma unroll
    for (int k = 0; k < IPT; ++k) lds[lds_pad<T>(k * BLOCK + (int)threadIdx.x)] = st[k];
    __syncthreads();
#pragma unroll
    for (int j = 0; j < IPT; ++j) items[j] = lds[lds_pad<T>((int)threadIdx.x * IPT + j)];
}

// Blocked items written back through LDS as striped coalesced stores.  With
// ADD the existing destination value is added (x_bar += contribution).
template <class T, int BLOCK, int IPT, bool ADD>
__device__ __forceinline__ void store_blocked(T* __restrict__ dst, int cnt, const T (&items)[IPT],
                                              T* lds) {
    __syncthreads();
#pragma unroll
    for (int j = 0; j < IPT; ++j) lds[lds_pad<T>((int)threadIdx.x * IPT + j)] = items[j];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < IPT; ++k) {
        const int i = k * BLOCK + (int)threadIdx.x;
        if (i < cnt) {
            T v = lds[lds_pad<T>(i)];
            dst[i] = ADD ? dst[i] + v : v;
        }
    }
}

// ------------------------------------------------------ decoupled lookback
// Workspace header.  The whole workspace starts zeroed.  `seq` holds the
// launch epoch (high 32 bits) and the next tile ticket (low 32 bits), so one
// relaxed fetch-add gives a block both its launch tag (epoch + 1) and its
// ticket.  The block that draws the launch's last ticket stores the next
// epoch with a zero ticket: every other block of the launch has drawn by
// then, and the next launch on the workspace (stream-ordered after this one)
// starts from a clean counter.  No per-block completion counter is needed:
// on this chip every same-address device-scope atomic costs about 11 ns of
// serialised time, which at 2^15 tiles would exceed the scan itself.
//
// A tile's flag carries the launch tag in its upper 30 bits, which makes
// flags left by an earlier launch read as "not yet published".  Every
// lookback kernel that uses a workspace shares this one header at offset 0,
// so launches on a workspace draw their tags from one increasing sequence
// and a stale flag can never carry the current tag.  `error` is set (and
// stays set until cleared by the host) when a launch sees a ticket beyond
// its last or gives up waiting on a predecessor; either means the workspace
// was not in the state this protocol leaves it in.  `done` is the
// completion counter of the single-launch reductions (reduce, GMM), which
// reset it themselves.
struct alignas(256) LookbackHdr {
    uint64_t seq;
    uint32_t done;
    uint32_t error;
    uint32_t pad[60];
};

constexpr uint32_t kErrTicket = 1u;  // ticket outside the grid
constexpr uint32_t kErrSpin = 2u;    // a predecessor never published
// Bound on polls of one predecessor (each poll sleeps ~64 cycles plus a
// device-scope load): seconds, far beyond any legitimate wait, so a
// corrupted workspace ends the kernel with an error instead of hanging it.
constexpr uint32_t kMaxPolls = 1u << 20;
constexpr uint32_t kTagMod = (1u << 30) - 1u;  // tags are 1 .. 2^30 - 1

// A tile's published states.  Every 32-bit word of a state travels together
// with its launch tag and status in one 64-bit relaxed atomic, so a reader
// accepts a state only when every word carries the current tag: no fence and
// no ordering between words is needed.  (A release/acquire pair at device
// scope would write back and invalidate the whole L2 of an XCD at every
// publish and poll.)
template <class S>
struct alignas(128) TileState {
    static constexpr int W = (int)(sizeof(S) / 4);
    uint64_t agg[W];
    uint64_t inc[W];
};

constexpr uint32_t kAgg = 1u, kInc = 2u;

// Tiles are grouped by 64 consecutive virtual indices.  The last tile of a
// group publishes the group's aggregate (in the `agg` field of a group
// state) as soon as it has read its group-mates' aggregates, so a lookback
// crosses 64 tiles per state read once it leaves its own group.
constexpr int kGroupShift = 6;
constexpr int64_t kGroup = (int64_t)1 << kGroupShift;

inline int64_t lookback_groups(int64_t ntiles) { return (ntiles + kGroup - 1) >> kGroupShift; }

// Bytes of tile and group states for `ntiles` tiles.
template <class S>
inline size_t lookback_state_bytes(int64_t ntiles) {
    return (size_t)(ntiles + lookback_groups(ntiles)) * sizeof(TileState<S>);
}

template <class S>
__device__ __forceinline__ void publish(TileState<S>* st, const S& v, uint32_t status, uint32_t tag) {
    static_assert(sizeof(S) % 4 == 0, "state must be a whole number of words");
    const uint32_t* src = reinterpret_cast<const uint32_t*>(&v);
    uint64_t* dst = status == kInc ? st->inc : st->agg;
    const uint64_t hi = (uint64_t)((tag << 2) | status) << 32;
#pragma unroll
    for (int w = 0; w < TileState<S>::W; ++w)
        __hip_atomic_store(dst + w, hi | (uint64_t)src[w], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Coherent word-wise store/load of small records (reduction partials).
template <class S>
__device__ __forceinline__ void st_coherent(S* p, const S& v) {
    static_assert(sizeof(S) % 4 == 0, "record must be a whole number of words");
    const uint32_t* src = reinterpret_cast<const uint32_t*>(&v);
    uint32_t* dst = reinterpret_cast<uint32_t*>(p);
#pragma unroll
    for (int w = 0; w < (int)(sizeof(S) / 4); ++w)
        __hip_atomic_store(dst + w, src[w], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <class S>
__device__ __forceinline__ S ld_coherent(const S* p) {
    S v;
    uint32_t* dst = reinterpret_cast<uint32_t*>(&v);
    const uint32_t* src = reinterpret_cast<const uint32_t*>(p);
#pragma unroll
    for (int w = 0; w < (int)(sizeof(S) / 4); ++w)
        dst[w] = __hip_atomic_load(src + w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return v;
}

// Draws the next ticket of this launch; `last` is the value of the launch's
// final draw (grid size - 1 for one draw per block; items + grid - 1 for a
// persistent queue whose blocks each make one last, empty draw).  Called by
// one thread.  Tickets are handed out in the order blocks ask, so every tile
// a block waits on is held by a block that is already running: no deadlock.
__device__ __forceinline__ uint32_t lookback_draw(LookbackHdr* h, uint32_t last, uint32_t* tag) {
    const uint64_t old = __hip_atomic_fetch_add(&h->seq, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const uint32_t epoch = (uint32_t)(old >> 32);
    const uint32_t ticket = (uint32_t)old;
    if (tag) *tag = (epoch % kTagMod) + 1u;
    if (ticket == last)
        __hip_atomic_store(&h->seq, (uint64_t)((epoch + 1u) % kTagMod) << 32, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
    return ticket;
}

// Thread 0 records a workspace error (see LookbackHdr).
__device__ __forceinline__ void lookback_error(LookbackHdr* h, uint32_t bits) {
    __hip_atomic_fetch_or(&h->error, bits, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Tries to take a state in one round trip: every tagged word of the
// inclusive field (at `inc`) and of the aggregate field (at `agg`) is loaded
// before any is examined.  Returns kInc or kAgg when all words of that field
// carry the current tag, 0 when neither is complete.
template <class S>
__device__ __forceinline__ uint32_t try_state(const uint64_t* inc, const uint64_t* agg, uint64_t hinc,
                                              uint64_t hagg, S& v) {
    constexpr int W = TileState<S>::W;
    constexpr uint64_t mask = ~0xffffffffull;
    uint64_t wi[W], wa[W];
#pragma unroll
    for (int w = 0; w < W; ++w) wi[w] = __hip_atomic_load(inc + w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
#pragma unroll
    for (int w = 0; w < W; ++w) wa[w] = __hip_atomic_load(agg + w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    bool inc_ok = true, agg_ok = true;
#pragma unroll
    for (int w = 0; w < W; ++w) {
        inc_ok = inc_ok && (wi[w] & mask) == hinc;
        agg_ok = agg_ok && (wa[w] & mask) == hagg;
    }
    uint32_t* dst = reinterpret_cast<uint32_t*>(&v);
    if (inc_ok) {
#pragma unroll
        for (int w = 0; w < W; ++w) dst[w] = (uint32_t)wi[w];
        return kInc;
    }
    if (agg_ok) {
#pragma unroll
        for (int w = 0; w < W; ++w) dst[w] = (uint32_t)wa[w];
        return kAgg;
    }
    return 0u;
}

// Every active lane of the wave takes its state (one try_state each); while
// some are missing, ONE lane -- the lowest missing, i.e. the nearest
// predecessor still missing -- polls the first word of its two fields with
// a growing pause, then all missing lanes try again.  Hundreds of waiting
// waves polling every lane's state at full rate would take memory
// bandwidth from the tiles still streaming their data.  Bounded: after
// kMaxPolls polls the missing states are recorded in the header and read as
// inclusive neutral elements, so the kernel still terminates.
template <class Op>
__device__ __forceinline__ uint32_t wave_wait_states(bool active, const uint64_t* inc, const uint64_t* agg,
                                                     uint64_t hinc, uint64_t hagg, typename Op::S& v,
                                                     LookbackHdr* hdr) {
    constexpr uint64_t mask = ~0xffffffffull;
    const int lane = threadIdx.x & (kWave - 1);
    uint32_t st = active ? try_state(inc, agg, hinc, hagg, v) : 0u;
    uint32_t polls = 0;
    while (true) {
        const uint64_t pending = __ballot(active && st == 0u);
        if (!pending) return st;
        const int j = __ffsll((unsigned long long)pending) - 1;
        if (lane == j) {
            uint32_t pause = 1;
            while (true) {
                const uint64_t f0 = __hip_atomic_load(inc, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                const uint64_t f1 = __hip_atomic_load(agg, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if ((f0 & mask) == hinc || (f1 & mask) == hagg) break;
                if (++polls >= kMaxPolls) break;
                for (uint32_t i = 0; i < pause; ++i) __builtin_amdgcn_s_sleep(2);
                if (pause < 16) pause <<= 1;
            }
        }
        polls = __shfl(polls, j, kWave);
        if (polls >= kMaxPolls) {
            if (lane == 0) __hip_atomic_fetch_or(&hdr->error, kErrSpin, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (active && st == 0u) {
                v = Op::id();
                st = kInc;
            }
            return st;
        }
        if (active && st == 0u) st = try_state(inc, agg, hinc, hagg, v);
    }
}

// Ordered combination of one value per lane, lanes 0..k (lane 0 latest in
// scan order, higher lanes earlier); lanes above k hold the neutral element.
// Returns the combination, valid in lane 0 and broadcast.
template <class Op>
__device__ __forceinline__ typename Op::S lane_fold(typename Op::S mine, int k, int lane) {
    if (lane > k) mine = Op::id();
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        typename Op::S o = Op::down(mine, d);
        if (lane + d < kWave) mine = Op::comb(o, mine);
    }
    return Op::idx(mine, 0);
}

// Executed by all 64 lanes of one wave of the block holding virtual tile
// v > 0 (virtual order is scan order; tile 0 publishes its inclusive state
// without a lookback).  `own` is the tile's aggregate, already published.
// Returns the exclusive prefix of v:
//   1. the predecessors inside v's group of 64, nearest first, up to the
//      nearest inclusive state;
//   2. if none is inclusive, the earlier groups, 64 per round: a group
//      contributes the inclusive state of its last tile when published, else
//      the group aggregate.
// The last tile of a group that reaches step 2 publishes the group aggregate
// (its predecessors' aggregates and its own) before it looks further back.
template <class Op>
__device__ typename Op::S lookback(TileState<typename Op::S>* states, TileState<typename Op::S>* groups, int64_t v,
                                   const typename Op::S& own, uint32_t tag, LookbackHdr* hdr) {
    using S = typename Op::S;
    const int lane = threadIdx.x & (kWave - 1);
    const uint64_t hinc = (uint64_t)((tag << 2) | kInc) << 32;
    const uint64_t hagg = (uint64_t)((tag << 2) | kAgg) << 32;
    const int64_t g = v >> kGroupShift;
    const int64_t g0 = g << kGroupShift;

    // 1. inside the group
    {
        const int64_t p = v - 1 - lane;
        const bool act = p >= g0;
        const int64_t pc = act ? p : v - 1;  // a valid address for inactive lanes (not read)
        S val = Op::id();
        uint32_t st = wave_wait_states<Op>(act, states[pc].inc, states[pc].agg, hinc, hagg, val, hdr);
        if (!act) val = Op::id();
        const uint64_t incl = __ballot(st == kInc);
        const int k = incl ? __ffsll((unsigned long long)incl) - 1 : kWave - 1;
        S prefix = lane_fold<Op>(val, k, lane);
        if (incl) return prefix;
        if ((v & (kGroup - 1)) == kGroup - 1 && lane == 0) publish(&groups[g], Op::comb(prefix, own), kAgg, tag);
        // 2. earlier groups (g0 > 0 here: tile 0 is inclusive, so group 0
        //    always ends in step 1)
        int64_t h0 = g - 1;
        while (true) {
            const int64_t h = h0 - lane;
            const bool act = h >= 0;
            const int64_t hc = act ? h : 0;
            const int64_t last = (hc << kGroupShift) + kGroup - 1;
            S gv = Op::id();
            uint32_t gs = wave_wait_states<Op>(act, states[last].inc, groups[hc].agg, hinc, hagg, gv, hdr);
            if (!act) {  // before the first group: neutral, inclusive
                gv = Op::id();
                gs = kInc;
            }
            const uint64_t gincl = __ballot(gs == kInc);
            const int gk = gincl ? __ffsll((unsigned long long)gincl) - 1 : kWave - 1;
            prefix = Op::comb(lane_fold<Op>(gv, gk, lane), prefix);
            if (gincl) return prefix;
            h0 -= kWave;
        }
    }
}

}  // namespace pvjp
