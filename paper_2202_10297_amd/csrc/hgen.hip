// reduce_by_index with a general associative operator (Sec. 5.1.2, with the
// general rule of Sec. 5.1.1 inside every bin) and its VJP.
//
// hs[b] = the fold, in index order, of the elements i with inds[i] = b (the
// neutral element for an empty bin; indices outside [0, m) are skipped).
// The operator need not commute, so each bin's elements must meet in index
// order:
//   1. a stable sort of the in-range elements by bin: passes of up to 8 bits
//      (9 for large records when that saves a pass; the bin's bits split evenly), low digit first, each a per-chunk digit
//      count, a digit-major scan of the counts and a stable scatter staged in
//      LDS (ranks among equal digits from wave ballots, so equal bins keep
//      their order; each digit's records leave as contiguous runs).  The sort
//      moves whole records -- bin, element index and the element's
//      components -- so x is read once, in index order, instead of gathered
//      at random into sorted order;
//   2. bin starts, by binary search of the sorted bins;
//   3. over the sorted elements, segmented exclusive scans: forward (the
//      fold of the bin's earlier elements, ls) and reversed (of its later
//      ones, rs), with the usual lifted operator that restarts at a flagged
//      element (a bin's first element forward, its last one reversed), over
//      fixed tiles: tile folds, the tiles' carries (a wave per 64 tiles, one
//      block over the groups, a wave per group again), then per tile the
//      in-tile scans with the tile's carry;
//   4. the primal writes each bin's fold at its last element; the VJP maps
//      f(ls, x, rs, hs_bar[bin]) (the reduce rule, y_bar = the bin's hs_bar)
//      over the sorted elements and writes it at the element's own index.
// Folds are formed in FP64 for FP32 and FP64 data alike.
#include <algorithm>

#include "common.h"
#include "gops.h"
#include "prims.h"

namespace pvjp {

// Row length of the per-chunk digit counts (a pass uses at most
// kHgPassDigits of a row's entries).
constexpr int kHgDigitBits = 12;
constexpr int kHgDigits = 1 << kHgDigitBits;
constexpr int64_t kHgChunk = 32768;  // elements per sort chunk (one block)
constexpr int kHgCountBlock = 256;
constexpr int kHgColChunk = 64;      // sort chunks per column-scan chunk
constexpr int kHgScanThreads = 1024;
constexpr int kHgBlock = 256;
constexpr int kHgIpt = 2;  // of 1, 2, 4, 8: 2 the fastest (adjacent lanes 32 bytes apart)
constexpr int kHgTile = kHgBlock * kHgIpt;
constexpr size_t kHgSlot = 64;       // bytes per tile for a lifted state
constexpr int64_t kHgMaxBins = (int64_t)1 << 24;  // three sort passes of 8 bits

// A sort record: word 0 the bin, word 1 the element index, from word 2 the
// element's K components (T each), padded to whole 16-byte vectors so that a
// record moves with full-width loads and stores.
template <int W>
struct alignas(16) HgRec {
    uint32_t w[W];
};
template <class T, int K>
constexpr int hg_words() {
    return (2 + K * (int)(sizeof(T) / 4) + 3) / 4 * 4;
}
template <class T, int W>
__device__ __forceinline__ T hg_comp(const HgRec<W>& r, int k) {
    return reinterpret_cast<const T*>(&r.w[2])[k];
}

// Up to four component arrays of one dtype.
template <class T>
struct HgIn {
    const T* p[4];
};
template <class T>
struct HgOut {
    T* p[4];
};

// ------------------------------------------------------------------ sort
// Digit counts of one chunk (any order: counting needs no stability).  The
// first pass reads the indices (out-of-range ones skipped), the second the
// first pass's output, whose length is on the device.
template <int W>
__global__ __launch_bounds__(kHgCountBlock) void hg_count_kernel(const int32_t* __restrict__ keys,
                                                                 const HgRec<W>* __restrict__ recs, int64_t n,
                                                                 const int32_t* __restrict__ nvalid, int32_t m,
                                                                 int shift, int dmask, int ndig,
                                                                 int32_t* __restrict__ cntb) {
    __shared__ int32_t cnt[kHgDigits];
    for (int d = threadIdx.x; d < ndig; d += kHgCountBlock) cnt[d] = 0;
    __syncthreads();
    const int64_t ne = nvalid ? (int64_t)*nvalid : n;
    const int64_t lo = (int64_t)blockIdx.x * kHgChunk;
    const int64_t hi = (lo + kHgChunk < ne) ? lo + kHgChunk : ne;
    for (int64_t i = lo + threadIdx.x; i < hi; i += kHgCountBlock) {
        const int32_t k = keys ? keys[i] : (int32_t)recs[i].w[0];
        if ((uint32_t)k < (uint32_t)m) atomicAdd(&cnt[(k >> shift) & dmask], 1);
    }
    __syncthreads();
    for (int d = threadIdx.x; d < ndig; d += kHgCountBlock) cntb[(int64_t)blockIdx.x * kHgDigits + d] = cnt[d];
}

// Per digit (a thread) and column chunk of kHgColChunk sort chunks (grid y):
// the count of each chunk is replaced by the sum of the earlier chunks'
// counts in the column chunk, whose total goes to ctot[c][d].
__global__ __launch_bounds__(kHgCountBlock) void hg_colscan_kernel(int32_t* __restrict__ cntb, int nblk, int ndig,
                                                                   int32_t* __restrict__ ctot) {
    const int d = blockIdx.x * kHgCountBlock + (int)threadIdx.x;
    const int c = blockIdx.y;
    if (d >= ndig) return;
    int v[kHgColChunk];
#pragma unroll
    for (int j = 0; j < kHgColChunk; ++j) {
        const int b = c * kHgColChunk + j;
        v[j] = b < nblk ? cntb[(int64_t)b * kHgDigits + d] : 0;
    }
    int run = 0;
#pragma unroll
    for (int j = 0; j < kHgColChunk; ++j) {
        const int b = c * kHgColChunk + j;
        if (b < nblk) cntb[(int64_t)b * kHgDigits + d] = run;
        run += v[j];
    }
    ctot[(int64_t)c * kHgDigits + d] = run;
}

// One block: ctot[c][d] becomes the start of (column chunk c, digit d) in the
// sorted output (the digit's start plus its earlier column chunks), and the
// number of sorted elements is written once.
__global__ __launch_bounds__(kHgScanThreads) void hg_digitscan_kernel(int32_t* __restrict__ ctot, int nchunks,
                                                                      int ndig, int32_t* __restrict__ nvalid) {
    __shared__ IntSum::S wtot[kHgScanThreads / kWave];
    constexpr int DPT = kHgDigits / kHgScanThreads;
    int tot[DPT], sum = 0;
#pragma unroll
    for (int u = 0; u < DPT; ++u) {
        const int d = DPT * (int)threadIdx.x + u;
        int run = 0;
        if (d < ndig) {
            for (int c = 0; c < nchunks; ++c) {
                int32_t* p = ctot + (int64_t)c * kHgDigits + d;
                const int v = *p;
                *p = run;
                run += v;
            }
        }
        tot[u] = run;
        sum += run;
    }
    IntSum::S all;
    int start = block_exclusive_scan<IntSum, kHgScanThreads, false>(IntSum::S{sum}, all, wtot).v;
#pragma unroll
    for (int u = 0; u < DPT; ++u) {
        const int d = DPT * (int)threadIdx.x + u;
        if (d < ndig)
            for (int c = 0; c < nchunks; ++c) ctot[(int64_t)c * kHgDigits + d] += start;
        start += tot[u];
    }
    if (threadIdx.x == 0 && nvalid) *nvalid = all.v;
}

// Stable scatter of one chunk, staged in LDS so that each digit's records
// leave as contiguous runs instead of one scattered store per record.  The
// chunk is taken in sub-chunks of kHgSub records in index order (long
// enough that a digit's run in it averages a whole line); wave w of the
// block owns records [w * 64 G, (w + 1) * 64 G) of a sub-chunk, as G =
// kHgSortGroups groups of 64 taken in order.  Ranks: within a group, the lanes of equal
// digit find each other with one ballot per digit bit (rank = earlier such
// lanes); a wave's running count per digit orders its groups; the counts
// of earlier waves order the waves; earlier sub-chunks and chunks come
// before through the digit's running position.  So equal digits keep their
// index order.  Records are placed in LDS at (the digit's start in the
// sub-chunk + rank), then thread t writes slots t, t + 256, ... to the
// digit's running position in the output.  The first pass builds each
// record from the indices and x (read in order), later passes move records.
constexpr int kHgSortThreads = 256;
constexpr int kHgSortWaves = kHgSortThreads / kWave;
constexpr int kHgSortGroups = 8;                               // groups of 64 per wave and sub-chunk
constexpr int kHgSub = kHgSortThreads * kHgSortGroups;         // 2048 records
constexpr int kHgPassBits = 8;                                 // bits per pass, one digit per thread
constexpr int kHgPassDigits = 1 << kHgPassBits;
static_assert(kHgPassDigits == kHgSortThreads, "a thread per digit in the sub-chunk scans");
static_assert(kHgChunk % kHgSub == 0, "chunks are whole sub-chunks");

// DPT: digits per thread in the per-digit steps (1: up to 256 digits, 2: up
// to 512); thread t owns digits [DPT t, DPT t + DPT).
template <class T, int K, int W, int DPT>
__global__ __launch_bounds__(kHgSortThreads) void hg_scatter_kernel(const int32_t* __restrict__ keys_in, HgIn<T> x,
                                                                    const HgRec<W>* __restrict__ recs_in, int64_t n,
                                                                    const int32_t* __restrict__ nvalid, int32_t m,
                                                                    int shift, int dmask, int ndig, int nbits,
                                                                    const int32_t* __restrict__ cntb,
                                                                    const int32_t* __restrict__ ctot,
                                                                    HgRec<W>* __restrict__ recs_out,
                                                                    int32_t* __restrict__ keys_out) {
    constexpr int ND = kHgPassDigits * DPT;
    __shared__ HgRec<W> stage[kHgSub];
    __shared__ int32_t wcnt[kHgSortWaves][ND];  // per wave: running count, then its offset
    __shared__ int32_t lstart[ND];              // the digit's first slot in the sub-chunk
    __shared__ int32_t gpos[ND];                // the digit's running output position
    __shared__ IntSum::S wtot[kHgSortWaves];
    const int tid = threadIdx.x;
    const int lane = tid & (kWave - 1);
    const int wave = tid / kWave;
    const int blk = blockIdx.x;
    const int c = blk / kHgColChunk;
#pragma unroll
    for (int u = 0; u < DPT; ++u) {
        const int d = DPT * tid + u;
        if (d < ndig) gpos[d] = ctot[(int64_t)c * kHgDigits + d] + cntb[(int64_t)blk * kHgDigits + d];
    }
    const int64_t ne = nvalid ? (int64_t)*nvalid : n;
    const int64_t lo = (int64_t)blk * kHgChunk;
    const int64_t hi = (lo + kHgChunk < ne) ? lo + kHgChunk : ne;
    const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (kWave - lane));
    for (int64_t s0 = lo; s0 < hi; s0 += kHgSub) {
        for (int w = 0; w < kHgSortWaves; ++w)
#pragma unroll
            for (int u = 0; u < DPT; ++u) wcnt[w][DPT * tid + u] = 0;
        HgRec<W> r[kHgSortGroups];
        bool valid[kHgSortGroups];
        int dg[kHgSortGroups];
#pragma unroll
        for (int g = 0; g < kHgSortGroups; ++g) {
            const int64_t i = s0 + wave * (kHgSortGroups * kWave) + g * kWave + lane;
            if (i < hi && keys_in) {
                r[g].w[0] = (uint32_t)keys_in[i];
                r[g].w[1] = (uint32_t)i;
#pragma unroll
                for (int w = 2; w < W; ++w) r[g].w[w] = 0u;
#pragma unroll
                for (int k = 0; k < K; ++k) reinterpret_cast<T*>(&r[g].w[2])[k] = x.p[k][i];
            } else if (i < hi) {
                r[g] = recs_in[i];
            } else {
                r[g].w[0] = 0xffffffffu;  // no element: outside every bin
            }
            valid[g] = (uint32_t)r[g].w[0] < (uint32_t)m;
            dg[g] = valid[g] ? ((int32_t)r[g].w[0] >> shift) & dmask : 0;
        }
        __syncthreads();  // counters cleared; the previous sub-chunk's slots read out
        // ranks within the wave, groups in order
        int rank[kHgSortGroups];
#pragma unroll
        for (int g = 0; g < kHgSortGroups; ++g) {
            const int d = dg[g];
            uint64_t peers = __ballot(valid[g]);
            for (int bit = 0; bit < nbits; ++bit) {
                const bool one = (d >> bit) & 1;
                const uint64_t b = __ballot(valid[g] && one);
                peers &= one ? b : ~b;
            }
            const int before = valid[g] ? wcnt[wave][d] : 0;
            rank[g] = before + __popcll(peers & below);
            // the highest lane of the group moves the wave's count on (lanes
            // of a wave run together: every lane has read it first)
            if (valid[g] && (peers >> lane) == 1ull) wcnt[wave][d] = before + __popcll(peers);
        }
        __syncthreads();
        // per digit (DPT a thread): the waves' offsets and the digit's total,
        // then the digits' starts in the sub-chunk
        int tot[DPT], sum = 0;
#pragma unroll
        for (int u = 0; u < DPT; ++u) {
            const int d = DPT * tid + u;
            tot[u] = 0;
            for (int w = 0; w < kHgSortWaves; ++w) {
                const int cw = wcnt[w][d];
                wcnt[w][d] = tot[u];
                tot[u] += cw;
            }
            sum += tot[u];
        }
        IntSum::S all;
        int st = block_exclusive_scan<IntSum, kHgSortThreads, false>(IntSum::S{sum}, all, wtot).v;
#pragma unroll
        for (int u = 0; u < DPT; ++u) {
            lstart[DPT * tid + u] = st;
            st += tot[u];
        }
        __syncthreads();
#pragma unroll
        for (int g = 0; g < kHgSortGroups; ++g)
            if (valid[g]) stage[lstart[dg[g]] + wcnt[wave][dg[g]] + rank[g]] = r[g];
        __syncthreads();
        for (int sl = tid; sl < all.v; sl += kHgSortThreads) {
            const HgRec<W> q = stage[sl];
            const int d = ((int32_t)q.w[0] >> shift) & dmask;
            const int64_t o = gpos[d] + (sl - lstart[d]);
            recs_out[o] = q;
            if (keys_out) keys_out[o] = (int32_t)q.w[0];  // what the next pass counts
        }
        __syncthreads();  // every slot placed before the positions move on
#pragma unroll
        for (int u = 0; u < DPT; ++u) gpos[DPT * tid + u] += tot[u];
    }
}

// off[b] = the first sorted position whose bin is b or later (b in [0, m]).
template <int W>
__global__ __launch_bounds__(256) void hg_off_kernel(const HgRec<W>* __restrict__ recs,
                                                     const int32_t* __restrict__ nvalid, int32_t m,
                                                     int32_t* __restrict__ off) {
    const int64_t b = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (b > m) return;
    int64_t lo = 0, hi = *nvalid;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if ((int64_t)recs[mid].w[0] < b) lo = mid + 1; else hi = mid;
    }
    off[b] = (int32_t)lo;
}

// --------------------------------------------------- segmented fold scans
// The lifted operator: a state remembers whether it holds a flagged element,
// and a later flagged state discards everything before it.
template <class Q>
struct SegOf {
    using QS = typename Q::S;
    struct S {
        QS v;
        uint32_t f, pad;
    };
    __device__ static __forceinline__ S id() { return S{Q::id(), 0u, 0u}; }
    __device__ static __forceinline__ S comb(S x, S y) { return y.f ? y : S{Q::comb(x.v, y.v), x.f, 0u}; }
    __device__ static __forceinline__ S up(S v, int d) {
        return S{Q::up(v.v, d), (uint32_t)shfl_up1((int)v.f, d), 0u};
    }
    __device__ static __forceinline__ S down(S v, int d) {
        return S{Q::down(v.v, d), (uint32_t)shfl_down1((int)v.f, d), 0u};
    }
};


// Sorted element p: its bin, its own index and its components (as FP64, from
// its record), plus whether it opens (first) and closes (last) its bin.
template <class Op, class T>
struct HgElem {
    int32_t key, src;
    bool first, last;
    typename Op::S a;
};

template <class Op, class T, int W>
__device__ __forceinline__ HgElem<Op, T> hg_elem(const HgRec<W>* __restrict__ recs, int64_t nv, int64_t p) {
    HgElem<Op, T> e;
    const HgRec<W> r = recs[p];
    e.key = (int32_t)r.w[0];
    e.src = (int32_t)r.w[1];
    e.first = p == 0 || (int32_t)recs[p - 1].w[0] != e.key;
    e.last = p + 1 == nv || (int32_t)recs[p + 1].w[0] != e.key;
    double c[Op::K];
#pragma unroll
    for (int k = 0; k < Op::K; ++k) c[k] = (double)hg_comp<T, W>(r, k);
    e.a = Op::elem(c);
    return e;
}

// Tile folds, forward (flag: the bin's first element) and reversed (flag:
// its last element, scanned with the operands exchanged).
template <class Op, class T, int W>
__global__ __launch_bounds__(kHgBlock) void hg_tile_fold_kernel(const HgRec<W>* __restrict__ recs,
                                                                const int32_t* __restrict__ nvalid, char* __restrict__ aggF,
                                                                char* __restrict__ aggR) {
    using F = SegOf<Op>;
    using R = SegOf<Flip<Op>>;
    __shared__ typename F::S wf[kHgBlock / kWave];
    __shared__ typename R::S wr[kHgBlock / kWave];
    const int64_t nv = *nvalid;
    const int64_t p0 = (int64_t)blockIdx.x * kHgTile + (int64_t)threadIdx.x * kHgIpt;
    typename F::S sf = F::id();
    typename R::S sr = R::id();
    typename R::S re[kHgIpt];
#pragma unroll
    for (int j = 0; j < kHgIpt; ++j) {
        re[j] = R::id();
        if (p0 + j < nv) {
            const HgElem<Op, T> e = hg_elem<Op, T, W>(recs, nv, p0 + j);
            sf = F::comb(sf, typename F::S{e.a, e.first ? 1u : 0u, 0u});
            re[j] = typename R::S{e.a, e.last ? 1u : 0u, 0u};
        }
    }
#pragma unroll
    for (int j = kHgIpt - 1; j >= 0; --j) sr = R::comb(sr, re[j]);
    typename F::S tf;
    typename R::S tr;
    block_exclusive_scan<F, kHgBlock, false>(sf, tf, wf);
    block_exclusive_scan<R, kHgBlock, true>(sr, tr, wr);
    if (threadIdx.x == 0) {
        *reinterpret_cast<typename F::S*>(aggF + (size_t)blockIdx.x * kHgSlot) = tf;
        *reinterpret_cast<typename R::S*>(aggR + (size_t)blockIdx.x * kHgSlot) = tr;
    }
}

// One block: each item's carry, the lifted fold of all items before it
// (forward) and after it (reversed), for an array of tile or group folds.
// Thread t owns a contiguous run of items.
template <class Op>
__global__ __launch_bounds__(kHgScanThreads) void hg_tile_scan_kernel(const char* __restrict__ aggF,
                                                                      const char* __restrict__ aggR, int64_t ntiles,
                                                                      char* __restrict__ carF, char* __restrict__ carR) {
    using F = SegOf<Op>;
    using R = SegOf<Flip<Op>>;
    __shared__ typename F::S wf[kHgScanThreads / kWave];
    __shared__ typename R::S wr[kHgScanThreads / kWave];
    const int64_t per = (ntiles + kHgScanThreads - 1) / kHgScanThreads;
    const int64_t t0 = (int64_t)threadIdx.x * per;
    const int64_t t1 = (t0 + per < ntiles) ? t0 + per : ntiles;
    auto getF = [&](int64_t t) { return *reinterpret_cast<const typename F::S*>(aggF + (size_t)t * kHgSlot); };
    auto getR = [&](int64_t t) { return *reinterpret_cast<const typename R::S*>(aggR + (size_t)t * kHgSlot); };
    typename F::S sf = F::id();
    typename R::S sr = R::id();
    for (int64_t t = t0; t < t1; ++t) sf = F::comb(sf, getF(t));
    for (int64_t t = t1 - 1; t >= t0; --t) sr = R::comb(sr, getR(t));
    typename F::S tf;
    typename R::S tr;
    sf = block_exclusive_scan<F, kHgScanThreads, false>(sf, tf, wf);
    sr = block_exclusive_scan<R, kHgScanThreads, true>(sr, tr, wr);
    for (int64_t t = t0; t < t1; ++t) {
        *reinterpret_cast<typename F::S*>(carF + (size_t)t * kHgSlot) = sf;
        sf = F::comb(sf, getF(t));
    }
    for (int64_t t = t1 - 1; t >= t0; --t) {
        *reinterpret_cast<typename R::S*>(carR + (size_t)t * kHgSlot) = sr;
        sr = R::comb(sr, getR(t));
    }
}

// Tile carries in three steps: a wave folds each group of 64 tiles, one
// block scans the group folds (hg_tile_scan_kernel over the groups), and a
// wave per group turns the group's carry into its tiles' carries.
constexpr int kHgGroup = kWave;

template <class Op>
__global__ __launch_bounds__(kHgGroup) void hg_group_fold_kernel(const char* __restrict__ aggF,
                                                                 const char* __restrict__ aggR, int64_t ntiles,
                                                                 char* __restrict__ gF, char* __restrict__ gR) {
    using F = SegOf<Op>;
    using R = SegOf<Flip<Op>>;
    __shared__ typename F::S wf[1];
    __shared__ typename R::S wr[1];
    const int64_t t = (int64_t)blockIdx.x * kHgGroup + threadIdx.x;
    const typename F::S af = t < ntiles ? *reinterpret_cast<const typename F::S*>(aggF + (size_t)t * kHgSlot) : F::id();
    const typename R::S ar = t < ntiles ? *reinterpret_cast<const typename R::S*>(aggR + (size_t)t * kHgSlot) : R::id();
    typename F::S tf;
    typename R::S tr;
    block_exclusive_scan<F, kHgGroup, false>(af, tf, wf);
    block_exclusive_scan<R, kHgGroup, true>(ar, tr, wr);
    if (threadIdx.x == 0) {
        *reinterpret_cast<typename F::S*>(gF + (size_t)blockIdx.x * kHgSlot) = tf;
        *reinterpret_cast<typename R::S*>(gR + (size_t)blockIdx.x * kHgSlot) = tr;
    }
}

template <class Op>
__global__ __launch_bounds__(kHgGroup) void hg_group_carry_kernel(const char* __restrict__ aggF,
                                                                  const char* __restrict__ aggR, int64_t ntiles,
                                                                  const char* __restrict__ gcF,
                                                                  const char* __restrict__ gcR,
                                                                  char* __restrict__ carF, char* __restrict__ carR) {
    using F = SegOf<Op>;
    using R = SegOf<Flip<Op>>;
    __shared__ typename F::S wf[1];
    __shared__ typename R::S wr[1];
    const int64_t t = (int64_t)blockIdx.x * kHgGroup + threadIdx.x;
    const typename F::S af = t < ntiles ? *reinterpret_cast<const typename F::S*>(aggF + (size_t)t * kHgSlot) : F::id();
    const typename R::S ar = t < ntiles ? *reinterpret_cast<const typename R::S*>(aggR + (size_t)t * kHgSlot) : R::id();
    typename F::S tf;
    typename R::S tr;
    const typename F::S xf = block_exclusive_scan<F, kHgGroup, false>(af, tf, wf);
    const typename R::S xr = block_exclusive_scan<R, kHgGroup, true>(ar, tr, wr);
    if (t < ntiles) {
        *reinterpret_cast<typename F::S*>(carF + (size_t)t * kHgSlot) =
            F::comb(*reinterpret_cast<const typename F::S*>(gcF + (size_t)blockIdx.x * kHgSlot), xf);
        *reinterpret_cast<typename R::S*>(carR + (size_t)t * kHgSlot) =
            R::comb(*reinterpret_cast<const typename R::S*>(gcR + (size_t)blockIdx.x * kHgSlot), xr);
    }
}

// Per tile: the forward scan with the tile's carry; the primal writes each
// bin's fold at its last element.  The VJP also runs the reversed scan and
// maps f over (ls, x, rs) with y_bar = hs_bar of the element's bin.
template <class Op, class T, int W, bool VJP, bool ACC>
__global__ __launch_bounds__(kHgBlock) void hg_apply_kernel(const HgRec<W>* __restrict__ recs,
                                                            HgRec<W>* __restrict__ urecs,
                                                            int32_t* __restrict__ ukeys,
                                                            const int32_t* __restrict__ nvalid,
                                                            const char* __restrict__ carF,
                                                            const char* __restrict__ carR, HgOut<T> hs,
                                                            HgIn<T> hs_bar, HgOut<T> x_bar) {
    using F = SegOf<Op>;
    using R = SegOf<Flip<Op>>;
    using QS = typename Op::S;
    __shared__ typename F::S wf[kHgBlock / kWave];
    __shared__ typename R::S wr[kHgBlock / kWave];
    const int64_t nv = *nvalid;
    const int64_t p0 = (int64_t)blockIdx.x * kHgTile + (int64_t)threadIdx.x * kHgIpt;
    HgElem<Op, T> e[kHgIpt];
    bool in[kHgIpt];
    typename F::S sf = F::id();
#pragma unroll
    for (int j = 0; j < kHgIpt; ++j) {
        in[j] = p0 + j < nv;
        if (in[j]) {
            e[j] = hg_elem<Op, T, W>(recs, nv, p0 + j);
            sf = F::comb(sf, typename F::S{e[j].a, e[j].first ? 1u : 0u, 0u});
        }
    }
    typename F::S tf;
    typename F::S xf = block_exclusive_scan<F, kHgBlock, false>(sf, tf, wf);
    xf = F::comb(*reinterpret_cast<const typename F::S*>(carF + (size_t)blockIdx.x * kHgSlot), xf);
    if (!VJP) {
#pragma unroll
        for (int j = 0; j < kHgIpt; ++j) {
            if (!in[j]) continue;
            xf = F::comb(xf, typename F::S{e[j].a, e[j].first ? 1u : 0u, 0u});
            if (e[j].last) {
                double out[Op::K];
                Op::value(xf.v, out);
#pragma unroll
                for (int k = 0; k < Op::K; ++k) hs.p[k][e[j].key] = (T)out[k];
            }
        }
        return;
    }
    QS ls[kHgIpt], la[kHgIpt];
#pragma unroll
    for (int j = 0; j < kHgIpt; ++j) {
        if (!in[j]) continue;
        ls[j] = e[j].first ? Op::id() : xf.v;
        la[j] = Op::comb(ls[j], e[j].a);
        xf = F::comb(xf, typename F::S{e[j].a, e[j].first ? 1u : 0u, 0u});
    }
    typename R::S sr = R::id();
#pragma unroll
    for (int j = kHgIpt - 1; j >= 0; --j)
        if (in[j]) sr = R::comb(sr, typename R::S{e[j].a, e[j].last ? 1u : 0u, 0u});
    typename R::S tr;
    typename R::S xr = block_exclusive_scan<R, kHgBlock, true>(sr, tr, wr);
    xr = R::comb(*reinterpret_cast<const typename R::S*>(carR + (size_t)blockIdx.x * kHgSlot), xr);
#pragma unroll
    for (int j = kHgIpt - 1; j >= 0; --j) {
        if (!in[j]) continue;
        const QS rs = e[j].last ? Op::id() : xr.v;
        double yb[Op::K], out[Op::K];
#pragma unroll
        for (int k = 0; k < Op::K; ++k) yb[k] = (double)hs_bar.p[k][e[j].key];
        Op::vjp(ls[j], e[j].a, rs, la[j], yb, out);
        if (urecs) {
            // (index, x_bar) records in sorted order, for the unsort
            HgRec<W> q;
            q.w[0] = (uint32_t)e[j].src;
#pragma unroll
            for (int w = 1; w < W; ++w) q.w[w] = 0u;
#pragma unroll
            for (int k = 0; k < Op::K; ++k) reinterpret_cast<T*>(&q.w[2])[k] = (T)out[k];
            urecs[p0 + j] = q;
            ukeys[p0 + j] = e[j].src;
        } else {
#pragma unroll
            for (int k = 0; k < Op::K; ++k) {
                T* dst = x_bar.p[k] + e[j].src;
                *dst = ACC ? (T)((double)*dst + out[k]) : (T)out[k];
            }
        }
        xr = R::comb(xr, typename R::S{e[j].a, e[j].last ? 1u : 0u, 0u});
    }
}

// Empty bins hold the neutral element.
template <class Op, class T>
__global__ __launch_bounds__(256) void hg_empty_kernel(const int32_t* __restrict__ off, int32_t m, HgOut<T> hs) {
    const int64_t b = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (b >= m || off[b] != off[b + 1]) return;
    double out[Op::K];
    Op::value(Op::id(), out);
#pragma unroll
    for (int k = 0; k < Op::K; ++k) hs.p[k][b] = (T)out[k];
}

// Without accumulation, every in-range element's x_bar is written by the
// apply (or the unsort); the elements whose index is outside [0, m) get 0
// here, read from the indices, instead of clearing whole arrays first.
template <class T>
__global__ __launch_bounds__(256) void hg_zero_oob_kernel(const int32_t* __restrict__ inds, int64_t n, int32_t m,
                                                          HgOut<T> x, int K) {
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
        if ((uint32_t)inds[i] >= (uint32_t)m)
            for (int k = 0; k < K; ++k) x.p[k][i] = T(0);
}

// The unsort's last step: records in increasing element index (in-range
// elements only), each component written at the element's index -- in
// order, with gaps where indices were out of range.
template <class T, int K, int W, bool ACC>
__global__ __launch_bounds__(256) void hg_unsort_write_kernel(const HgRec<W>* __restrict__ recs,
                                                              const int32_t* __restrict__ nvalid, HgOut<T> x_bar) {
    const int64_t nv = *nvalid;
    for (int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x; p < nv; p += (int64_t)gridDim.x * 256) {
        const HgRec<W> q = recs[p];
        const int64_t i = (int64_t)q.w[0];
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const T v = hg_comp<T, W>(q, k);
            x_bar.p[k][i] = ACC ? (T)((double)x_bar.p[k][i] + (double)v) : v;
        }
    }
}

// ------------------------------------------------------------------ host
static int hg_components(pvjp_gop op) {
    return op == PVJP_GOP_LOGADDEXP ? 1 : op == PVJP_GOP_LINREC ? 2 : op == PVJP_GOP_MAT2 ? 4 : 0;
}

struct HgLayout {
    int64_t nblk, nchunks, ntiles;
    int64_t ngroups;
    size_t cntb, ctot, nvalid, recA, recB, keyA, keyB, off, aggF, aggR, carF, carR, gF, gR, gcF, gcR, total;
};

static size_t hg_rec_bytes(int K, size_t tsize) {
    return (size_t)((2 + K * (int)(tsize / 4) + 3) / 4 * 4) * 4;
}

// rec_bytes: the size of one sort record (hg_rec_bytes).
static HgLayout hg_layout(int64_t n, int64_t m, size_t rec_bytes) {
    HgLayout L{};
    const int64_t nn = n > 0 ? n : 1;
    L.nblk = ceil_div(nn, kHgChunk);
    L.nchunks = ceil_div(L.nblk, kHgColChunk);
    L.ntiles = ceil_div(nn, kHgTile);
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t at = o;
        o += align_up(bytes, 256);
        return at;
    };
    L.cntb = take((size_t)L.nblk * kHgDigits * 4);
    L.ctot = take((size_t)L.nchunks * kHgDigits * 4);
    L.nvalid = take(4);
    L.recA = take((size_t)nn * rec_bytes);
    L.recB = take((size_t)nn * rec_bytes);
    L.keyA = take((size_t)nn * 4);
    L.keyB = take((size_t)nn * 4);
    L.off = take((size_t)(m + 1) * 4);
    L.aggF = take((size_t)L.ntiles * kHgSlot);
    L.aggR = take((size_t)L.ntiles * kHgSlot);
    L.carF = take((size_t)L.ntiles * kHgSlot);
    L.carR = take((size_t)L.ntiles * kHgSlot);
    L.ngroups = ceil_div(L.ntiles, kHgGroup);
    L.gF = take((size_t)L.ngroups * kHgSlot);
    L.gR = take((size_t)L.ngroups * kHgSlot);
    L.gcF = take((size_t)L.ngroups * kHgSlot);
    L.gcR = take((size_t)L.ngroups * kHgSlot);
    L.total = o;
    return L;
}

// Stable LSD passes of at most 8 bits, or 9 for records of 32 bytes or more
// when that saves a pass (the key's bits split evenly; at least one pass) over keys below m: from the indices and x (keys != NULL; the
// first pass also counts the in-range elements into *nvalid) or from the
// records rin, whose keys ckeys may hold compactly (nv on the device).
// Records ping-pong between bufA and bufB; for records of 32 bytes or more,
// each pass but the last also writes its output's keys compactly (keyA /
// keyB), which the next pass counts instead of reading whole records.
// Returns the sorted records.
template <class T, int K, int W>
static const HgRec<W>* hg_sort_passes(const int32_t* keys, const HgIn<T>& x, const HgRec<W>* rin,
                                      const int32_t* ckeys, int64_t n, const int32_t* nv_in, int64_t m,
                                      HgRec<W>* bufA, HgRec<W>* bufB, int32_t* keyA, int32_t* keyB, int32_t* cntb,
                                      int32_t* ctot, int32_t* nvalid, const HgLayout& L, hipStream_t st) {
    int bbits = 0;
    while (((int64_t)1 << bbits) < m) ++bbits;
    int passes = std::max(1, (bbits + kHgPassBits - 1) / kHgPassBits);
    // records of 32 bytes or more run whole lines with 512 digits too: take
    // 9-bit passes when that saves one (an unsort of 2^26 indices: 3, not 4)
    const int passes9 = std::max(1, (bbits + kHgPassBits) / (kHgPassBits + 1));
    if (W >= 8 && passes9 < passes) passes = passes9;
    const int bpp = std::max(1, (bbits + passes - 1) / passes);
    const int32_t* kcount = keys ? keys : ckeys;
    for (int pass = 0; pass < passes; ++pass) {
        const int shift = pass * bpp;
        const int dmask = (1 << bpp) - 1;
        const int ndig = (int)std::min<int64_t>((int64_t)1 << bpp, ceil_div(m, (int64_t)1 << shift));
        int nbits = 0;
        while ((1 << nbits) < ndig) ++nbits;
        HgRec<W>* rout = (pass & 1) ? bufB : bufA;
        // compact keys pay for their extra stores only when a record is at
        // least 32 bytes (a 16-byte one costs the count about as much to read)
        int32_t* kout = (W >= 8 && pass + 1 < passes) ? ((pass & 1) ? keyB : keyA) : nullptr;
        const int32_t* kin = pass == 0 ? keys : nullptr;
        const int32_t* nv = (pass == 0 && keys) ? nullptr : (keys ? nvalid : nv_in);
        hipLaunchKernelGGL(hg_count_kernel<W>, dim3((unsigned)L.nblk), dim3(kHgCountBlock), 0, st, kcount, rin, n,
                           nv, (int32_t)m, shift, dmask, ndig, cntb);
        hipLaunchKernelGGL(hg_colscan_kernel, dim3((unsigned)ceil_div(ndig, kHgCountBlock), (unsigned)L.nchunks),
                           dim3(kHgCountBlock), 0, st, cntb, (int)L.nblk, ndig, ctot);
        hipLaunchKernelGGL(hg_digitscan_kernel, dim3(1), dim3(kHgScanThreads), 0, st, ctot, (int)L.nchunks, ndig,
                           (pass == 0 && keys) ? nvalid : nullptr);
        if (ndig > kHgPassDigits)
            hipLaunchKernelGGL((hg_scatter_kernel<T, K, W, 2>), dim3((unsigned)L.nblk), dim3(kHgSortThreads), 0, st,
                               kin, x, rin, n, nv, (int32_t)m, shift, dmask, ndig, nbits, cntb, ctot, rout, kout);
        else
            hipLaunchKernelGGL((hg_scatter_kernel<T, K, W, 1>), dim3((unsigned)L.nblk), dim3(kHgSortThreads), 0, st,
                               kin, x, rin, n, nv, (int32_t)m, shift, dmask, ndig, nbits, cntb, ctot, rout, kout);
        rin = rout;
        kcount = kout;
    }
    return rin;
}

// The sort and the tile carries, shared by both entry points.  Returns the
// sorted records.
template <class Op, class T>
static const HgRec<hg_words<T, Op::K>()>* hg_prepare(const int32_t* inds, int64_t n, int32_t m, const HgIn<T>& x,
                                                     char* w, const HgLayout& L, hipStream_t st) {
    constexpr int W = hg_words<T, Op::K>();
    using Rec = HgRec<W>;
    int32_t* cntb = reinterpret_cast<int32_t*>(w + L.cntb);
    int32_t* ctot = reinterpret_cast<int32_t*>(w + L.ctot);
    int32_t* nvalid = reinterpret_cast<int32_t*>(w + L.nvalid);
    Rec* rA = reinterpret_cast<Rec*>(w + L.recA);
    Rec* rB = reinterpret_cast<Rec*>(w + L.recB);
    const Rec* rin = hg_sort_passes<T, Op::K, W>(inds, x, nullptr, nullptr, n, nullptr, m, rA, rB,
                                                 reinterpret_cast<int32_t*>(w + L.keyA),
                                                 reinterpret_cast<int32_t*>(w + L.keyB), cntb, ctot, nvalid, L, st);
    hipLaunchKernelGGL((hg_tile_fold_kernel<Op, T, W>), dim3((unsigned)L.ntiles), dim3(kHgBlock), 0, st, rin,
                       nvalid, w + L.aggF, w + L.aggR);
    hipLaunchKernelGGL(hg_group_fold_kernel<Op>, dim3((unsigned)L.ngroups), dim3(kHgGroup), 0, st, w + L.aggF,
                       w + L.aggR, L.ntiles, w + L.gF, w + L.gR);
    hipLaunchKernelGGL(hg_tile_scan_kernel<Op>, dim3(1), dim3(kHgScanThreads), 0, st, w + L.gF, w + L.gR,
                       L.ngroups, w + L.gcF, w + L.gcR);
    hipLaunchKernelGGL(hg_group_carry_kernel<Op>, dim3((unsigned)L.ngroups), dim3(kHgGroup), 0, st, w + L.aggF,
                       w + L.aggR, L.ntiles, w + L.gcF, w + L.gcR, w + L.carF, w + L.carR);
    return rin;
}

template <class Op, class T>
static void hg_primal(const int32_t* inds, int64_t n, int32_t m, const void* const* x, void* const* hs, char* w,
                      hipStream_t st) {
    constexpr int W = hg_words<T, Op::K>();
    const HgLayout L = hg_layout(n, m, hg_rec_bytes(Op::K, sizeof(T)));
    HgIn<T> xi{};
    HgOut<T> ho{};
    for (int k = 0; k < Op::K; ++k) {
        xi.p[k] = n > 0 ? (const T*)x[k] : nullptr;
        ho.p[k] = (T*)hs[k];
    }
    const HgRec<W>* recs = hg_prepare<Op, T>(inds, n, m, xi, w, L, st);
    int32_t* nvalid = reinterpret_cast<int32_t*>(w + L.nvalid);
    int32_t* off = reinterpret_cast<int32_t*>(w + L.off);
    hipLaunchKernelGGL(hg_off_kernel<W>, dim3((unsigned)ceil_div((int64_t)m + 1, 256)), dim3(256), 0, st, recs,
                       nvalid, m, off);
    hipLaunchKernelGGL((hg_apply_kernel<Op, T, W, false, false>), dim3((unsigned)L.ntiles), dim3(kHgBlock), 0, st,
                       recs, (HgRec<W>*)nullptr, (int32_t*)nullptr, nvalid, w + L.carF, w + L.carR, ho, HgIn<T>{},
                       HgOut<T>{});
    hipLaunchKernelGGL((hg_empty_kernel<Op, T>), dim3((unsigned)ceil_div(m, 256)), dim3(256), 0, st, off, m, ho);
}

template <class Op, class T>
static void hg_vjp(const int32_t* inds, int64_t n, int32_t m, const void* const* x, const void* const* hs_bar,
                   void* const* x_bar, bool acc, char* w, hipStream_t st) {
    constexpr int W = hg_words<T, Op::K>();
    const HgLayout L = hg_layout(n, m, hg_rec_bytes(Op::K, sizeof(T)));
    HgIn<T> xi{}, hb{};
    HgOut<T> xb{};
    for (int k = 0; k < Op::K; ++k) {
        xi.p[k] = (const T*)x[k];
        hb.p[k] = (const T*)hs_bar[k];
        xb.p[k] = (T*)x_bar[k];
    }
    if (!acc)  // elements outside [0, m) get a zero adjoint
        hipLaunchKernelGGL(hg_zero_oob_kernel<T>, dim3(flat_grid(n, 256, 4)), dim3(256), 0, st, inds, n, m, xb,
                           Op::K);
    const HgRec<W>* recs = hg_prepare<Op, T>(inds, n, m, xi, w, L, st);
    int32_t* nvalid = reinterpret_cast<int32_t*>(w + L.nvalid);
    // With four components, K scattered stores per element cost more than
    // writing (index, x_bar) records in sorted order and sorting them back by
    // index with the same staged passes; with fewer, the stores are cheaper.
    HgRec<W>* urecs = nullptr;
    HgRec<W>* rA = reinterpret_cast<HgRec<W>*>(w + L.recA);
    HgRec<W>* rB = reinterpret_cast<HgRec<W>*>(w + L.recB);
    if (Op::K >= 4) urecs = (recs == rA) ? rB : rA;
    int32_t* kA = reinterpret_cast<int32_t*>(w + L.keyA);
    int32_t* kB = reinterpret_cast<int32_t*>(w + L.keyB);
    int32_t* ukeys = urecs ? kB : nullptr;  // the unsort's first pass writes kA
    if (acc)
        hipLaunchKernelGGL((hg_apply_kernel<Op, T, W, true, true>), dim3((unsigned)L.ntiles), dim3(kHgBlock), 0, st,
                           recs, urecs, ukeys, nvalid, w + L.carF, w + L.carR, HgOut<T>{}, hb, xb);
    else
        hipLaunchKernelGGL((hg_apply_kernel<Op, T, W, true, false>), dim3((unsigned)L.ntiles), dim3(kHgBlock), 0, st,
                           recs, urecs, ukeys, nvalid, w + L.carF, w + L.carR, HgOut<T>{}, hb, xb);
    if (urecs) {
        // the sorted records' buffer is free now: the passes start there, so
        // that no pass reads and writes one buffer
        HgRec<W>* other = (urecs == rA) ? rB : rA;
        int32_t* cntb = reinterpret_cast<int32_t*>(w + L.cntb);
        int32_t* ctot = reinterpret_cast<int32_t*>(w + L.ctot);
        const HgRec<W>* out = hg_sort_passes<T, Op::K, W>(nullptr, HgIn<T>{}, urecs, ukeys, n, nvalid, n, other,
                                                          urecs, kA, kB, cntb, ctot, nvalid, L, st);
        if (acc)
            hipLaunchKernelGGL((hg_unsort_write_kernel<T, Op::K, W, true>), dim3(flat_grid(n, 256, 4)), dim3(256), 0,
                               st, out, nvalid, xb);
        else
            hipLaunchKernelGGL((hg_unsort_write_kernel<T, Op::K, W, false>), dim3(flat_grid(n, 256, 4)), dim3(256), 0,
                               st, out, nvalid, xb);
    }
}

static pvjp_status hg_check(const char* name, pvjp_gop op, pvjp_dtype dtype, const int32_t* inds,
                            const void* const* x, int64_t n, int64_t m, void* ws, size_t ws_bytes) {
    const int K = hg_components(op);
    PVJP_REQUIRE(K > 0, "%s: unknown operator %d", name, (int)op);
    PVJP_REQUIRE(valid_dtype(dtype), "%s: unknown dtype %d", name, (int)dtype);
    PVJP_REQUIRE(n >= 0 && n <= INT32_MAX, "%s: n = %lld out of range [0, 2^31)", name, (long long)n);
    PVJP_REQUIRE(m >= 1 && m <= kHgMaxBins, "%s: m = %lld out of range [1, 2^24]", name, (long long)m);
    PVJP_REQUIRE(ws != nullptr && aligned(ws, 256), "%s: workspace must be non-NULL and 256-byte aligned", name);
    const size_t need = pvjp_hist_generic_ws_bytes(op, dtype, n, m);
    if (ws_bytes < need) {
        set_error("%s: workspace of %zu bytes, need %zu", name, ws_bytes, need);
        return PVJP_ENOMEM;
    }
    if (n > 0) {
        PVJP_REQUIRE(inds != nullptr && x != nullptr, "%s: inds and x must be non-NULL", name);
        for (int c = 0; c < K; ++c) {
            PVJP_REQUIRE(x[c] != nullptr, "%s: component %d of x is NULL", name, c);
            PVJP_REQUIRE(aligned(x[c], dsize(dtype)), "%s: component %d of x is misaligned", name, c);
        }
    }
    return PVJP_OK;
}

}  // namespace pvjp

using namespace pvjp;

extern "C" size_t pvjp_hist_generic_ws_bytes(pvjp_gop op, pvjp_dtype dtype, int64_t n, int64_t m) {
    if (hg_components(op) == 0 || !valid_dtype(dtype) || n < 0 || m < 1 || m > kHgMaxBins) return 0;
    return hg_layout(n, m, hg_rec_bytes(hg_components(op), dsize(dtype))).total;
}

extern "C" pvjp_status pvjp_hist_generic(pvjp_gop op, pvjp_dtype dtype, const int32_t* inds, const void* const* x,
                                         int64_t n, int64_t m, void* const* hs, void* ws, size_t ws_bytes,
                                         void* stream) {
    clear_error();
    const pvjp_status s = hg_check("pvjp_hist_generic", op, dtype, inds, x, n, m, ws, ws_bytes);
    if (s != PVJP_OK) return s;
    const int K = hg_components(op);
    PVJP_REQUIRE(hs != nullptr, "pvjp_hist_generic: hs is NULL");
    for (int c = 0; c < K; ++c) PVJP_REQUIRE(hs[c] != nullptr, "pvjp_hist_generic: component %d of hs is NULL", c);
    const hipStream_t st = as_stream(stream);
    char* w = reinterpret_cast<char*>(ws);
    const int32_t mm = (int32_t)m;
    if (dtype == PVJP_F64) {
        if (op == PVJP_GOP_LOGADDEXP) hg_primal<GLogAddExp<double>, double>(inds, n, mm, x, hs, w, st);
        else if (op == PVJP_GOP_LINREC) hg_primal<GLinRec<double>, double>(inds, n, mm, x, hs, w, st);
        else hg_primal<GMat2<double>, double>(inds, n, mm, x, hs, w, st);
    } else {
        if (op == PVJP_GOP_LOGADDEXP) hg_primal<GLogAddExp<double>, float>(inds, n, mm, x, hs, w, st);
        else if (op == PVJP_GOP_LINREC) hg_primal<GLinRec<double>, float>(inds, n, mm, x, hs, w, st);
        else hg_primal<GMat2<double>, float>(inds, n, mm, x, hs, w, st);
    }
    PVJP_LAUNCHED("pvjp_hist_generic");
    return PVJP_OK;
}

extern "C" pvjp_status pvjp_hist_generic_vjp(pvjp_gop op, pvjp_dtype dtype, const int32_t* inds,
                                             const void* const* x, int64_t n, int64_t m, const void* const* hs_bar,
                                             void* const* x_bar, int accumulate, void* ws, size_t ws_bytes,
                                             void* stream) {
    clear_error();
    const pvjp_status s = hg_check("pvjp_hist_generic_vjp", op, dtype, inds, x, n, m, ws, ws_bytes);
    if (s != PVJP_OK) return s;
    if (n == 0) return PVJP_OK;
    const int K = hg_components(op);
    PVJP_REQUIRE(hs_bar != nullptr && x_bar != nullptr, "pvjp_hist_generic_vjp: hs_bar and x_bar must be non-NULL");
    for (int c = 0; c < K; ++c) {
        PVJP_REQUIRE(hs_bar[c] != nullptr, "pvjp_hist_generic_vjp: component %d of hs_bar is NULL", c);
        PVJP_REQUIRE(x_bar[c] != nullptr, "pvjp_hist_generic_vjp: component %d of x_bar is NULL", c);
        PVJP_REQUIRE(aligned(x_bar[c], dsize(dtype)), "pvjp_hist_generic_vjp: component %d of x_bar is misaligned",
                     c);
    }
    const hipStream_t st = as_stream(stream);
    char* w = reinterpret_cast<char*>(ws);
    const int32_t mm = (int32_t)m;
    const bool acc = accumulate != 0;
    if (dtype == PVJP_F64) {
        if (op == PVJP_GOP_LOGADDEXP) hg_vjp<GLogAddExp<double>, double>(inds, n, mm, x, hs_bar, x_bar, acc, w, st);
        else if (op == PVJP_GOP_LINREC) hg_vjp<GLinRec<double>, double>(inds, n, mm, x, hs_bar, x_bar, acc, w, st);
        else hg_vjp<GMat2<double>, double>(inds, n, mm, x, hs_bar, x_bar, acc, w, st);
    } else {
        if (op == PVJP_GOP_LOGADDEXP) hg_vjp<GLogAddExp<double>, float>(inds, n, mm, x, hs_bar, x_bar, acc, w, st);
        else if (op == PVJP_GOP_LINREC) hg_vjp<GLinRec<double>, float>(inds, n, mm, x, hs_bar, x_bar, acc, w, st);
        else hg_vjp<GMat2<double>, float>(inds, n, mm, x, hs_bar, x_bar, acc, w, st);
    }
    PVJP_LAUNCHED("pvjp_hist_generic_vjp");
    return PVJP_OK;
}
