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
// Workspace header.  The whole workspace starts zeroed; the last block of
// every launch resets `ticket` and `done` and advances `epoch`, so the next
// launch on the same workspace needs no clearing.  A tile's flag carries the
// launch tag (epoch + 1) in its upper 30 bits, which makes flags left by an
// earlier launch read as "not yet published".
//
// Every lookback kernel that uses a workspace shares this one header at
// offset 0, so launches on a workspace draw their tags from one increasing
// sequence and a stale flag can never carry the current tag.  `error` is set
// (and stays set until cleared by the host) when a launch sees a ticket
// outside its grid or gives up waiting on a predecessor; either means the
// workspace was not in the state this protocol leaves it in.
struct alignas(256) LookbackHdr {
    uint32_t ticket;
    uint32_t done;
    uint32_t epoch;
    uint32_t error;
    uint32_t pad[60];
};

constexpr uint32_t kErrTicket = 1u;  // ticket outside the grid
constexpr uint32_t kErrSpin = 2u;    // a predecessor never published
// Bound on polls of one predecessor flag (each poll sleeps ~64 cycles plus a
// device-scope load): seconds, far beyond any legitimate wait, so a corrupted
// workspace ends the kernel with an error instead of hanging it.
constexpr uint32_t kMaxPolls = 1u << 20;

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

// Reads a field whose first word already showed `hi`; spins (bounded) on any
// word not yet visible.  Returns false if a word never showed up.
template <class S>
__device__ __forceinline__ bool read_state(const uint64_t* f, uint64_t hi, S& v) {
    uint32_t* dst = reinterpret_cast<uint32_t*>(&v);
#pragma unroll
    for (int w = 0; w < TileState<S>::W; ++w) {
        uint64_t u;
        uint32_t polls = 0;
        while (((u = __hip_atomic_load(f + w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) & ~0xffffffffull) != hi) {
            if (++polls == (1u << 20)) return false;
            __builtin_amdgcn_s_sleep(1);
        }
        dst[w] = (uint32_t)u;
    }
    return true;
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

// Called by thread 0 at kernel start: fetches the launch tag and a dynamic
// tile ticket (tickets are handed out in the order blocks actually start, so
// every tile a block waits on is already resident: no deadlock).
__device__ __forceinline__ void lookback_begin(LookbackHdr* h, uint32_t& tag, uint32_t& ticket) {
    tag = __hip_atomic_load(&h->epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) + 1u;
    if (tag >= (1u << 30)) tag = 1u;  // flags hold 30 tag bits; 0 never matches
    ticket = __hip_atomic_fetch_add(&h->ticket, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Thread 0 records a workspace error (see LookbackHdr).
__device__ __forceinline__ void lookback_error(LookbackHdr* h, uint32_t bits) {
    __hip_atomic_fetch_or(&h->error, bits, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Called by every thread at kernel end.  The last block to finish resets the
// counters for the next launch on this workspace.
__device__ __forceinline__ void lookback_end(LookbackHdr* h, uint32_t tag) {
    __syncthreads();
    if (threadIdx.x == 0) {
        // Relaxed: the reset only has to be visible to the next launch, which
        // the kernel boundary orders.
        uint32_t d = __hip_atomic_fetch_add(&h->done, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (d == gridDim.x - 1) {
            __hip_atomic_store(&h->ticket, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&h->done, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&h->epoch, tag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

// Executed by all 64 lanes of one wave.  Returns the exclusive prefix (in
// scan order) of tile `tile`, combining the published states of its
// predecessors in scan order: tiles tile-1, tile-2, ... (forward) or tile+1,
// tile+2, ... (REV), 64 at a time, stopping at the nearest inclusive state.
// Positions before the first tile read as an inclusive neutral element.
template <class Op, bool REV>
__device__ typename Op::S lookback(TileState<typename Op::S>* states, int64_t tile, int64_t ntiles,
                                   uint32_t tag, LookbackHdr* hdr) {
    using S = typename Op::S;
    const int lane = threadIdx.x & (kWave - 1);
    S prefix = Op::id();
    int64_t base = tile;
    while (true) {
        const int64_t p = REV ? base + 1 + lane : base - 1 - lane;
        const bool virt = REV ? (p >= ntiles) : (p < 0);
        uint32_t status = kInc;
        S v = Op::id();
        if (!virt) {
            const uint64_t hinc = (uint64_t)((tag << 2) | kInc) << 32;
            const uint64_t hagg = (uint64_t)((tag << 2) | kAgg) << 32;
            const uint64_t mask = ~0xffffffffull;
            uint32_t polls = 0;
            status = 0;
            while (true) {
                if ((__hip_atomic_load(&states[p].inc[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & mask) == hinc) {
                    status = kInc;
                    break;
                }
                if ((__hip_atomic_load(&states[p].agg[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & mask) == hagg) {
                    status = kAgg;
                    break;
                }
                if (++polls == kMaxPolls) break;
                __builtin_amdgcn_s_sleep(1);
            }
            if (status == 0 || !read_state(status == kInc ? states[p].inc : states[p].agg,
                                           status == kInc ? hinc : hagg, v)) {
                // A predecessor never published: record it and end the wait
                // (results are invalid, but the kernel terminates).
                __hip_atomic_fetch_or(&hdr->error, kErrSpin, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                status = kInc;
                v = Op::id();
            }
        }
        const uint64_t incl = __ballot(status == kInc);
        const int k = incl ? __ffsll((unsigned long long)incl) - 1 : kWave;
        S mine = (lane <= k) ? v : Op::id();
        // Ordered reduction: lane 0 ends with v_k (+) ... (+) v_0, higher lanes
        // being earlier in scan order.
#pragma unroll
        for (int d = 1; d < kWave; d <<= 1) {
            S o = Op::down(mine, d);
            if (lane + d < kWave) mine = Op::comb(o, mine);
        }
        prefix = Op::comb(Op::idx(mine, 0), prefix);
        if (incl) break;
        base = REV ? base + kWave : base - kWave;
    }
    return prefix;
}

}  // namespace pvjp
