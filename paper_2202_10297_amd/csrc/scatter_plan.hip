// Scatter and its VJP over a target-ordered plan (Sec. 5.3).
//
// The forward sweep of scatter may return more than the result: here it
// returns, besides the scattered array, the updates grouped by target
// window (an auxiliary result the return sweep reads instead of the random
// index array).  A window is 32 KiB of the target array (8192 FP32 or 4096
// FP64 elements), small enough to stage in LDS.  Random 4-byte accesses on
// this chip are limited by their request rate (one cache-line request per
// lane), not by bytes, so both sweeps are laid out to touch the target array
// only through whole windows:
//   forward  1. bucket the m updates by coarse digit k >> S1 (64 windows per
//               coarse bucket): count per chunk of 4096 updates, scan the
//               (digit, chunk) counts, scatter (k, j, v) records in runs;
//            2. within each coarse bucket, the same by fine digit
//               (k >> S0) & 63, which leaves the records grouped by window;
//            3. per window: load it into LDS, save each target's old value
//               (in record order, kept in the plan), write the new value,
//               store the window back;
//   return   per window: load ys_bar's window (and ys's, to restore) into
//            LDS; for each record take g = ys_bar[k], zero it, restore
//            ys[k] from the saved value and write vs_bar[j] (+)= g; store the
//            windows back.  Only vs_bar is written at random.
// Targets must be unique (the paper's assumption); repeated targets race.
// Targets outside [0, n) are dropped from the plan: they change nothing and
// their adjoint is 0.
#include <type_traits>

#include "common.h"
#include "prims.h"

namespace pvjp {

constexpr int kSpBlock = 512;
constexpr int kSpChunk = 4096;          // updates per chunk of a bucketing pass
constexpr int kSpPer = kSpChunk / kSpBlock;
constexpr int kSpFineBits = 6;          // fine digits per coarse bucket: 64
constexpr int kSpFine = 1 << kSpFineBits;
constexpr int kSpMaxCoarse = 4096;
constexpr int kSpWindowBytes = 32 * 1024;
constexpr int kSpScanTile = 4096;       // entries per tile of the count scans (1024 threads x 4)

template <class T>
constexpr int sp_s0() { return sizeof(T) == 4 ? 13 : 12; }  // log2 of window elements

// Blocks are dealt to the 8 accelerator dies in turn (block b to die b % 8),
// and each die has its own L2.  The bucketing passes give each die a
// contiguous range of chunks instead: the count or run that chunk c writes
// for a digit sits right before chunk c + 1's, so the lines the two share
// are completed in one L2 and leave it whole instead of as two partial
// writes from two dies.  Returns -1 for the few blocks past the last chunk.
constexpr int kSpXcds = 8;
__device__ __forceinline__ int sp_xcd_chunk(int nchunks) {
    const int per = (nchunks + kSpXcds - 1) / kSpXcds;
    const int slot = (int)(blockIdx.x / kSpXcds);
    const int c = (int)(blockIdx.x % kSpXcds) * per + slot;
    return (slot < per && c < nchunks) ? c : -1;
}
static unsigned sp_xcd_grid(int64_t nchunks) { return (unsigned)(ceil_div(nchunks, (int64_t)kSpXcds) * kSpXcds); }

// --------------------------------------------------------- bucketing pass 1
// cnt[d * nch + c] = number of valid updates of chunk c whose coarse digit is d.
__global__ __launch_bounds__(kSpBlock) void sp_count1_kernel(const int32_t* __restrict__ is, int64_t m, int64_t n,
                                                             int s1, int nc, int nch, int32_t* __restrict__ cnt) {
    extern __shared__ int32_t lc[];  // [nc]
    const int c = sp_xcd_chunk(nch);
    if (c < 0) return;
    for (int d = threadIdx.x; d < nc; d += kSpBlock) lc[d] = 0;
    __syncthreads();
    const int64_t j0 = (int64_t)c * kSpChunk;
    if (m > 0) {
        // all of the thread's loads first (clamped, not predicated, so that
        // they are in flight together), then the counts
        int32_t k[kSpPer];
#pragma unroll
        for (int u = 0; u < kSpPer; ++u) {
            const int64_t j = j0 + (int64_t)u * kSpBlock + threadIdx.x;
            k[u] = is[j < m ? j : m - 1];
        }
#pragma unroll
        for (int u = 0; u < kSpPer; ++u) {
            const int64_t j = j0 + (int64_t)u * kSpBlock + threadIdx.x;
            if (j < m && k[u] >= 0 && (int64_t)k[u] < n) atomicAdd(&lc[k[u] >> s1], 1);
        }
    }
    __syncthreads();
    for (int d = threadIdx.x; d < nc; d += kSpBlock) cnt[(int64_t)d * nch + c] = lc[d];
}

// ------------------------------------------------------ flat exclusive scan
// tsum[t] = sum of entries [t * 4096, (t + 1) * 4096) of a[0, N).
__global__ __launch_bounds__(1024) void sp_tile_sum_kernel(const int32_t* __restrict__ a, int64_t N,
                                                           int32_t* __restrict__ tsum) {
    __shared__ int32_t red[1024 / kWave];
    const int64_t i0 = (int64_t)blockIdx.x * kSpScanTile + 4 * threadIdx.x;
    int s = 0;
#pragma unroll
    for (int t = 0; t < 4; ++t) s += (i0 + t < N) ? a[i0 + t] : 0;
    for (int o = kWave / 2; o > 0; o >>= 1) s += __shfl_xor(s, o);
    if ((threadIdx.x & (kWave - 1)) == 0) red[threadIdx.x / kWave] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        int tot = 0;
        for (int w = 0; w < 1024 / kWave; ++w) tot += red[w];
        tsum[blockIdx.x] = tot;
    }
}

// In place: a[i] = sum of a[0, i).  Tile t adds the sums of tiles before it.
// The last tile writes the grand total to *total (when total != NULL).
__global__ __launch_bounds__(1024) void sp_tile_scan_kernel(int32_t* __restrict__ a, int64_t N,
                                                            const int32_t* __restrict__ tsum, int32_t* __restrict__ total) {
    __shared__ IntSum::S wtot[1024 / kWave];
    __shared__ int32_t red[1024 / kWave];
    __shared__ int32_t s_pre;
    int p = 0;
    for (int t = threadIdx.x; t < (int)blockIdx.x; t += 1024) p += tsum[t];
    for (int o = kWave / 2; o > 0; o >>= 1) p += __shfl_xor(p, o);
    if ((threadIdx.x & (kWave - 1)) == 0) red[threadIdx.x / kWave] = p;
    __syncthreads();
    if (threadIdx.x == 0) {
        int tot = 0;
        for (int w = 0; w < 1024 / kWave; ++w) tot += red[w];
        s_pre = tot;
    }
    __syncthreads();
    const int64_t i0 = (int64_t)blockIdx.x * kSpScanTile + 4 * threadIdx.x;
    int v[4], s = 0;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        v[t] = (i0 + t < N) ? a[i0 + t] : 0;
        s += v[t];
    }
    IntSum::S tot;
    int ex = block_exclusive_scan<IntSum, 1024, false>(IntSum::S{s}, tot, wtot).v + s_pre;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        if (i0 + t < N) a[i0 + t] = ex;
        ex += v[t];
    }
    if (total != nullptr && blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) *total = s_pre + tot.v;
}

// ------------------------------------------------ coarse bucket boundaries
// From pass 1's scanned counts: the start of every coarse bucket, the
// number of chunks pass 2 gives it and their exclusive prefix.  One block.
__global__ __launch_bounds__(1024) void sp_seg_kernel(const int32_t* __restrict__ off1, int nch, int nc,
                                                      const int32_t* __restrict__ total, int32_t* __restrict__ cstart,
                                                      int32_t* __restrict__ nch2, int32_t* __restrict__ chb2) {
    __shared__ IntSum::S wtot[1024 / kWave];
    constexpr int kPer = kSpMaxCoarse / 1024;
    const int tot = *total;
    int own[kPer], s = 0;
#pragma unroll
    for (int t = 0; t < kPer; ++t) {
        const int c = kPer * threadIdx.x + t;
        own[t] = 0;
        if (c < nc) {
            const int b = off1[(int64_t)c * nch];
            const int e = (c + 1 < nc) ? off1[(int64_t)(c + 1) * nch] : tot;
            cstart[c] = b;
            own[t] = (e - b + kSpChunk - 1) / kSpChunk;
            nch2[c] = own[t];
        }
        s += own[t];
    }
    IntSum::S all;
    int ex = block_exclusive_scan<IntSum, 1024, false>(IntSum::S{s}, all, wtot).v;
#pragma unroll
    for (int t = 0; t < kPer; ++t) {
        const int c = kPer * threadIdx.x + t;
        if (c < nc) chb2[c] = ex;
        ex += own[t];
    }
    if (threadIdx.x == 0) {
        cstart[nc] = tot;
        chb2[nc] = all.v;
    }
}

// --------------------------------------------- scatter of a chunk's records
// Shared by both passes: the chunk's records are ranked by digit in LDS,
// staged digit by digit, and each digit's run leaves as one contiguous
// write at lbase[d] (the scanned (digit, chunk) offset).
template <class T>
struct SpStage {
    int32_t* cnt;   // [nd] counts, then run starts in the stage
    int32_t* base;  // [nd] global position of the digit's run
    int32_t* sk;    // [kSpChunk]
    int32_t* sj;
    T* sv;
};

template <class T>
__device__ __forceinline__ SpStage<T> sp_stage_layout(char* smem, int nd) {
    SpStage<T> L;
    L.cnt = reinterpret_cast<int32_t*>(smem);
    L.base = L.cnt + nd;
    L.sk = L.base + nd;
    L.sj = L.sk + kSpChunk;
    L.sv = reinterpret_cast<T*>(L.sj + kSpChunk);  // 8-byte aligned: an even number of words precede it
    return L;
}

static size_t sp_stage_bytes(int nd, size_t tsize) {
    return (size_t)2 * nd * 4 + (size_t)2 * kSpChunk * 4 + (size_t)kSpChunk * tsize;
}

// k[u], j[u], v[u] with k[u] < 0 for "no record"; digit(k) < nd.
template <class T, class Digit>
__device__ __forceinline__ void sp_scatter_chunk(const SpStage<T>& L, int nd, const int32_t (&k)[kSpPer],
                                                 const int32_t (&j)[kSpPer], const T (&v)[kSpPer], Digit digit,
                                                 int32_t* __restrict__ ok, int32_t* __restrict__ oj,
                                                 T* __restrict__ ov, IntSum::S* wtot) {
    int rank[kSpPer];
#pragma unroll
    for (int u = 0; u < kSpPer; ++u) rank[u] = k[u] >= 0 ? atomicAdd(&L.cnt[digit(k[u])], 1) : -1;
    __syncthreads();
    // run starts: thread t owns digits [t * per, t * per + per)
    const int per = (nd + kSpBlock - 1) / kSpBlock;
    int s = 0;
    for (int q = 0; q < per; ++q) {
        const int d = per * (int)threadIdx.x + q;
        s += d < nd ? L.cnt[d] : 0;
    }
    IntSum::S tot;
    int ex = block_exclusive_scan<IntSum, kSpBlock, false>(IntSum::S{s}, tot, wtot).v;
    for (int q = 0; q < per; ++q) {
        const int d = per * (int)threadIdx.x + q;
        if (d < nd) {
            const int c = L.cnt[d];
            L.cnt[d] = ex;
            ex += c;
        }
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < kSpPer; ++u) {
        if (rank[u] < 0) continue;
        const int slot = L.cnt[digit(k[u])] + rank[u];
        L.sk[slot] = k[u];
        L.sj[slot] = j[u];
        L.sv[slot] = v[u];
    }
    __syncthreads();
    for (int sl = threadIdx.x; sl < tot.v; sl += kSpBlock) {
        const int32_t kk = L.sk[sl];
        const int d = digit(kk);
        const int pos = L.base[d] + (sl - L.cnt[d]);
        ok[pos] = kk;
        oj[pos] = L.sj[sl];
        ov[pos] = L.sv[sl];
    }
}

struct CoarseDigit {
    int s1;
    __device__ int operator()(int32_t k) const { return k >> s1; }
};
struct FineDigit {
    int s0;
    __device__ int operator()(int32_t k) const { return (k >> s0) & (kSpFine - 1); }
};

template <class T>
__global__ __launch_bounds__(kSpBlock) void sp_scatter1_kernel(const int32_t* __restrict__ is, const T* __restrict__ vs,
                                                               int64_t m, int64_t n, int s1, int nc, int nch,
                                                               const int32_t* __restrict__ off1,
                                                               int32_t* __restrict__ rk, int32_t* __restrict__ rj,
                                                               T* __restrict__ rv) {
    extern __shared__ __align__(16) char smem[];
    __shared__ IntSum::S wtot[kSpBlock / kWave];
    const SpStage<T> L = sp_stage_layout<T>(smem, nc);
    const int c = sp_xcd_chunk(nch);
    if (c < 0 || m <= 0) return;  // with no updates there is nothing to place
    for (int d = threadIdx.x; d < nc; d += kSpBlock) {
        L.cnt[d] = 0;
        L.base[d] = off1[(int64_t)d * nch + c];
    }
    __syncthreads();
    const int64_t j0 = (int64_t)c * kSpChunk;
    int32_t k[kSpPer], jj[kSpPer];
    T v[kSpPer];
    // loads clamped to the last update, then the ones past it or out of
    // range are marked "no record"
#pragma unroll
    for (int u = 0; u < kSpPer; ++u) {
        const int64_t j = j0 + (int64_t)u * kSpBlock + threadIdx.x;
        const int64_t jc = j < m ? j : m - 1;
        k[u] = is[jc];
        v[u] = vs[jc];
        jj[u] = (int32_t)j;
    }
#pragma unroll
    for (int u = 0; u < kSpPer; ++u) {
        const int64_t j = j0 + (int64_t)u * kSpBlock + threadIdx.x;
        if (j >= m || k[u] < 0 || (int64_t)k[u] >= n) k[u] = -1;
    }
    sp_scatter_chunk<T>(L, nc, k, jj, v, CoarseDigit{s1}, rk, rj, rv, wtot);
}

// --------------------------------------------------------- bucketing pass 2
// Chunk g of pass 2 belongs to the coarse bucket c with chb2[c] <= g <
// chb2[c + 1] (empty buckets own no chunk).
__device__ __forceinline__ int sp_owner(const int32_t* __restrict__ chb2, int nc, int g) {
    int lo = 0, hi = nc;  // invariant: chb2[lo] <= g < chb2[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (chb2[mid] <= g) lo = mid; else hi = mid;
    }
    return lo;
}

// cnt2 layout: [bucket][fine digit][chunk of the bucket], at chb2[c] * 64 +
// f * nch2[c] + i.  Blocks past the last chunk zero their 64 entries, so the
// whole array scans to valid offsets.
__global__ __launch_bounds__(kSpBlock) void sp_count2_kernel(const int32_t* __restrict__ rk, int s0, int nc,
                                                             int nch2max,
                                                             const int32_t* __restrict__ cstart,
                                                             const int32_t* __restrict__ nch2,
                                                             const int32_t* __restrict__ chb2,
                                                             int32_t* __restrict__ cnt2) {
    __shared__ int32_t lc[kSpFine];
    const int g = sp_xcd_chunk(nch2max);
    if (g < 0) return;
    const int nchunks = chb2[nc];
    if (g >= nchunks) {
        if (threadIdx.x < kSpFine) cnt2[(int64_t)g * kSpFine + threadIdx.x] = 0;
        return;
    }
    if (threadIdx.x < kSpFine) lc[threadIdx.x] = 0;
    __syncthreads();
    const int c = sp_owner(chb2, nc, g);
    const int i = g - chb2[c];
    const int64_t r0 = (int64_t)cstart[c] + (int64_t)i * kSpChunk;
    const int64_t r1 = (r0 + kSpChunk < (int64_t)cstart[c + 1]) ? r0 + kSpChunk : (int64_t)cstart[c + 1];
    // a chunk holds at least one record: loads clamped to its last one
    int32_t k[kSpPer];
#pragma unroll
    for (int u = 0; u < kSpPer; ++u) {
        const int64_t r = r0 + (int64_t)u * kSpBlock + threadIdx.x;
        k[u] = rk[r < r1 ? r : r1 - 1];
    }
#pragma unroll
    for (int u = 0; u < kSpPer; ++u) {
        const int64_t r = r0 + (int64_t)u * kSpBlock + threadIdx.x;
        if (r < r1) atomicAdd(&lc[(k[u] >> s0) & (kSpFine - 1)], 1);
    }
    __syncthreads();
    if (threadIdx.x < kSpFine)
        cnt2[(int64_t)chb2[c] * kSpFine + (int64_t)threadIdx.x * nch2[c] + i] = lc[threadIdx.x];
}

template <class T>
__global__ __launch_bounds__(kSpBlock) void sp_scatter2_kernel(const int32_t* __restrict__ rk1,
                                                               const int32_t* __restrict__ rj1,
                                                               const T* __restrict__ rv1, int s0, int nc,
                                                               int nch2max, const int32_t* __restrict__ cstart,
                                                               const int32_t* __restrict__ nch2,
                                                               const int32_t* __restrict__ chb2,
                                                               const int32_t* __restrict__ off2,
                                                               int32_t* __restrict__ rk, int32_t* __restrict__ rj,
                                                               T* __restrict__ rv) {
    extern __shared__ __align__(16) char smem[];
    __shared__ IntSum::S wtot[kSpBlock / kWave];
    const int g = sp_xcd_chunk(nch2max);
    if (g < 0 || g >= chb2[nc]) return;
    const int c = sp_owner(chb2, nc, g);
    const int i = g - chb2[c];
    const SpStage<T> L = sp_stage_layout<T>(smem, kSpFine);
    if (threadIdx.x < kSpFine) {
        L.cnt[threadIdx.x] = 0;
        L.base[threadIdx.x] = off2[(int64_t)chb2[c] * kSpFine + (int64_t)threadIdx.x * nch2[c] + i];
    }
    __syncthreads();
    const int64_t r0 = (int64_t)cstart[c] + (int64_t)i * kSpChunk;
    const int64_t r1 = (r0 + kSpChunk < (int64_t)cstart[c + 1]) ? r0 + kSpChunk : (int64_t)cstart[c + 1];
    int32_t k[kSpPer], jj[kSpPer];
    T v[kSpPer];
#pragma unroll
    for (int u = 0; u < kSpPer; ++u) {
        const int64_t r = r0 + (int64_t)u * kSpBlock + threadIdx.x;
        const int64_t rc = r < r1 ? r : r1 - 1;  // a chunk holds at least one record
        k[u] = rk1[rc];
        jj[u] = rj1[rc];
        v[u] = rv1[rc];
    }
#pragma unroll
    for (int u = 0; u < kSpPer; ++u)
        if (r0 + (int64_t)u * kSpBlock + threadIdx.x >= r1) k[u] = -1;
    sp_scatter_chunk<T>(L, kSpFine, k, jj, v, FineDigit{s0}, rk, rj, rv, wtot);
}

// wstart[w] = first record of window w = (c, f); wstart[nc * 64] = total.
__global__ __launch_bounds__(256) void sp_wstart_kernel(int nc, const int32_t* __restrict__ cstart,
                                                        const int32_t* __restrict__ nch2,
                                                        const int32_t* __restrict__ chb2,
                                                        const int32_t* __restrict__ off2, int32_t* __restrict__ wstart) {
    const int64_t nw = (int64_t)nc * kSpFine;
    for (int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; w <= nw; w += (int64_t)gridDim.x * blockDim.x) {
        if (w == nw) {
            wstart[w] = cstart[nc];
            continue;
        }
        const int c = (int)(w >> kSpFineBits), f = (int)(w & (kSpFine - 1));
        wstart[w] = nch2[c] > 0 ? off2[(int64_t)chb2[c] * kSpFine + (int64_t)f * nch2[c]] : cstart[c];
    }
}

// ------------------------------------------------------- window sweeps
// Copies of a window between device memory and LDS: 16-byte vectors when the
// window is whole and the array 16-byte aligned (vec != 0), else elements.
template <class T>
using Vec16 = typename std::conditional<sizeof(T) == 4, float4, double2>::type;

template <class T, int B>
__device__ __forceinline__ void sp_win_load(T* __restrict__ l, const T* __restrict__ g, int len, bool whole) {
    if (whole) {
        constexpr int E = 16 / sizeof(T);
        const Vec16<T>* gv = reinterpret_cast<const Vec16<T>*>(g);
        Vec16<T>* lv = reinterpret_cast<Vec16<T>*>(l);
        for (int i = threadIdx.x; i < len / E; i += B) lv[i] = gv[i];
    } else {
        for (int i = threadIdx.x; i < len; i += B) l[i] = g[i];
    }
}

template <class T, int B>
__device__ __forceinline__ void sp_win_store(T* __restrict__ g, const T* __restrict__ l, int len, bool whole) {
    if (whole) {
        constexpr int E = 16 / sizeof(T);
        Vec16<T>* gv = reinterpret_cast<Vec16<T>*>(g);
        const Vec16<T>* lv = reinterpret_cast<const Vec16<T>*>(l);
        for (int i = threadIdx.x; i < len / E; i += B) gv[i] = lv[i];
    } else {
        for (int i = threadIdx.x; i < len; i += B) g[i] = l[i];
    }
}
// The first kSpFwdHeld rounds of a window's records are loaded before the
// window itself, so both are in flight together (a window of uniformly
// spread targets holds about 2^s0 / 4 records: 4 rounds of 512).  The loads
// are clamped to the window's last record rather than predicated.
constexpr int kSpFwdBlock = 512;
constexpr int kSpFwdHeld = 4;

template <class T>
__global__ __launch_bounds__(kSpFwdBlock) void sp_apply_fwd_kernel(T* __restrict__ xs, int64_t n, int s0, int vec,
                                                                   const int32_t* __restrict__ wstart,
                                                                   const int32_t* __restrict__ rk,
                                                                   const T* __restrict__ rv, T* __restrict__ saved) {
    __shared__ __align__(16) T lx[kSpWindowBytes / sizeof(T)];
    const int w = blockIdx.x;
    const int r0 = wstart[w], r1 = wstart[w + 1];
    if (r0 >= r1) return;
    const int64_t x0 = (int64_t)w << s0;
    const int len = (int)((n - x0) < ((int64_t)1 << s0) ? (n - x0) : ((int64_t)1 << s0));
    const bool whole = vec && len == (1 << s0);
    int32_t hk[kSpFwdHeld];
    T hv[kSpFwdHeld];
#pragma unroll
    for (int t = 0; t < kSpFwdHeld; ++t) {
        const int r = r0 + t * kSpFwdBlock + (int)threadIdx.x;
        const int rc = r < r1 ? r : r1 - 1;
        hk[t] = rk[rc];
        hv[t] = rv[rc];
    }
    sp_win_load<T, kSpFwdBlock>(lx, xs + x0, len, whole);
    __syncthreads();
#pragma unroll
    for (int t = 0; t < kSpFwdHeld; ++t) {
        const int r = r0 + t * kSpFwdBlock + (int)threadIdx.x;
        if (r < r1) {
            const int kl = (int)(hk[t] - x0);
            saved[r] = lx[kl];
            lx[kl] = hv[t];
        }
    }
    for (int r = r0 + kSpFwdHeld * kSpFwdBlock + (int)threadIdx.x; r < r1; r += kSpFwdBlock) {
        const int kl = (int)(rk[r] - x0);
        saved[r] = lx[kl];
        lx[kl] = rv[r];
    }
    __syncthreads();
    sp_win_store<T, kSpFwdBlock>(xs + x0, lx, len, whole);
}

// The random writes of vs_bar are issued after the block's last barrier, so
// that they drain while the next window's loads run instead of holding the
// barrier: each thread keeps the (j, g) of its first kSpHeld rounds of
// records in registers (a window holds at most 2^s0 unique targets; rounds
// beyond kSpHeld, possible only with more than kSpHeld * 512 records, write
// at once).
constexpr int kSpVjpBlock = 512;
constexpr int kSpHeld = 8;

template <class T, bool ACC, bool RESTORE>
__global__ __launch_bounds__(kSpVjpBlock) void sp_apply_vjp_kernel(T* __restrict__ ybar, T* __restrict__ ys, int64_t n,
                                                                   int s0, int vec, const int32_t* __restrict__ wstart,
                                                                   const int32_t* __restrict__ rk,
                                                                   const int32_t* __restrict__ rj,
                                                                   const T* __restrict__ saved,
                                                                   T* __restrict__ vbar) {
    __shared__ __align__(16) T ly[kSpWindowBytes / sizeof(T)];
    __shared__ __align__(16) T lys[RESTORE ? kSpWindowBytes / sizeof(T) : 2];
    const int w = blockIdx.x;
    const int r0 = wstart[w], r1 = wstart[w + 1];
    if (r0 >= r1) return;
    const int64_t x0 = (int64_t)w << s0;
    const int len = (int)((n - x0) < ((int64_t)1 << s0) ? (n - x0) : ((int64_t)1 << s0));
    const bool whole = vec && len == (1 << s0);
    // the held rounds' records are loaded (clamped to the last record)
    // before the windows, so that all of them are in flight together
    int32_t hk[kSpHeld], hj[kSpHeld];
    T hs[kSpHeld], hg[kSpHeld];
#pragma unroll
    for (int t = 0; t < kSpHeld; ++t) {
        const int r = r0 + t * kSpVjpBlock + (int)threadIdx.x;
        const int rc = r < r1 ? r : r1 - 1;
        hk[t] = rk[rc];
        hj[t] = rj[rc];
        hs[t] = RESTORE ? saved[rc] : T(0);
    }
    sp_win_load<T, kSpVjpBlock>(ly, ybar + x0, len, whole);
    if (RESTORE) sp_win_load<T, kSpVjpBlock>(lys, ys + x0, len, whole);
    __syncthreads();
#pragma unroll
    for (int t = 0; t < kSpHeld; ++t) {
        const int r = r0 + t * kSpVjpBlock + (int)threadIdx.x;
        hg[t] = T(0);
        if (r < r1) {
            const int kl = (int)(hk[t] - x0);
            hg[t] = ly[kl];
            ly[kl] = T(0);
            if (RESTORE) lys[kl] = hs[t];
        } else {
            hj[t] = -1;
        }
    }
    for (int r = r0 + kSpHeld * kSpVjpBlock + (int)threadIdx.x; r < r1; r += kSpVjpBlock) {
        const int kl = (int)(rk[r] - x0);
        const int32_t j = rj[r];
        const T g = ly[kl];
        ly[kl] = T(0);
        if (RESTORE) lys[kl] = saved[r];
        vbar[j] = ACC ? vbar[j] + g : g;
    }
    __syncthreads();
    sp_win_store<T, kSpVjpBlock>(ybar + x0, ly, len, whole);
    if (RESTORE) sp_win_store<T, kSpVjpBlock>(ys + x0, lys, len, whole);
#pragma unroll
    for (int t = 0; t < kSpHeld; ++t)
        if (hj[t] >= 0) vbar[hj[t]] = ACC ? vbar[hj[t]] + hg[t] : hg[t];
}

// Without accumulate, updates whose target was out of range get adjoint 0;
// they are not in the plan, so vs_bar is cleared first when there are any.
template <class T>
__global__ __launch_bounds__(256) void sp_clear_kernel(T* __restrict__ x, int64_t m, const int32_t* __restrict__ valid) {
    if ((int64_t)*valid == m) return;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x)
        x[i] = T(0);
}

// ------------------------------------------------------------------ host
struct SpLayout {
    int s0, s1, nc, nch1, nch2max;
    int64_t n1, n2, nt1, nt2, nw;
    size_t cnt1, tsum1, total, cstart, nch2, chb2, cnt2, tsum2, wstart, rk1, rj1, rv1, rk, rj, rv, saved, bytes;
};

static SpLayout sp_layout(pvjp_dtype dtype, int64_t n, int64_t m) {
    SpLayout L{};
    const size_t ts = dsize(dtype);
    L.s0 = dtype == PVJP_F64 ? sp_s0<double>() : sp_s0<float>();
    L.s1 = L.s0 + kSpFineBits;
    L.nc = (int)ceil_div(n > 0 ? n : 1, (int64_t)1 << L.s1);
    L.nch1 = (int)ceil_div(m > 0 ? m : 1, kSpChunk);
    L.nch2max = L.nch1 + L.nc;
    L.n1 = (int64_t)L.nc * L.nch1;
    L.n2 = (int64_t)L.nch2max * kSpFine;
    L.nt1 = ceil_div(L.n1, kSpScanTile);
    L.nt2 = ceil_div(L.n2, kSpScanTile);
    L.nw = (int64_t)L.nc * kSpFine;
    const size_t mm = (size_t)(m > 0 ? m : 1);
    size_t o = 0;
    auto take = [&](size_t b) {
        const size_t at = o;
        o += align_up(b > 0 ? b : 1, 256);
        return at;
    };
    L.cnt1 = take((size_t)L.n1 * 4);
    L.tsum1 = take((size_t)L.nt1 * 4);
    L.total = take(16);
    L.cstart = take((size_t)(L.nc + 1) * 4);
    L.nch2 = take((size_t)L.nc * 4);
    L.chb2 = take((size_t)(L.nc + 1) * 4);
    L.cnt2 = take((size_t)L.n2 * 4);
    L.tsum2 = take((size_t)L.nt2 * 4);
    L.wstart = take((size_t)(L.nw + 1) * 4);
    L.rk1 = take(mm * 4);
    L.rj1 = take(mm * 4);
    L.rv1 = take(mm * ts);
    L.rk = take(mm * 4);
    L.rj = take(mm * 4);
    L.rv = take(mm * ts);
    L.saved = take(mm * ts);
    L.bytes = o;
    return L;
}

// The staging of a chunk can exceed the default 64 KiB of dynamic LDS (FP64
// records, many coarse digits): raise the limit of both scatter kernels once.
template <class T>
static void sp_allow_lds() {
    static const bool once = [] {
        constexpr int kMax = 160 * 1024 - 1024;  // the CU's LDS less the kernels' static share
        if (hipFuncSetAttribute(reinterpret_cast<const void*>(&sp_scatter1_kernel<T>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, kMax) != hipSuccess)
            (void)hipGetLastError();
        if (hipFuncSetAttribute(reinterpret_cast<const void*>(&sp_scatter2_kernel<T>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, kMax) != hipSuccess)
            (void)hipGetLastError();
        return true;
    }();
    (void)once;
}

template <class T>
static pvjp_status sp_forward(T* xs, int64_t n, const int32_t* is, const T* vs, int64_t m, char* p, const SpLayout& L,
                              hipStream_t st) {
    int32_t* cnt1 = (int32_t*)(p + L.cnt1);
    int32_t* tsum1 = (int32_t*)(p + L.tsum1);
    int32_t* total = (int32_t*)(p + L.total);
    int32_t* cstart = (int32_t*)(p + L.cstart);
    int32_t* nch2 = (int32_t*)(p + L.nch2);
    int32_t* chb2 = (int32_t*)(p + L.chb2);
    int32_t* cnt2 = (int32_t*)(p + L.cnt2);
    int32_t* tsum2 = (int32_t*)(p + L.tsum2);
    int32_t* wstart = (int32_t*)(p + L.wstart);
    int32_t* rk1 = (int32_t*)(p + L.rk1);
    int32_t* rj1 = (int32_t*)(p + L.rj1);
    T* rv1 = (T*)(p + L.rv1);
    int32_t* rk = (int32_t*)(p + L.rk);
    int32_t* rj = (int32_t*)(p + L.rj);
    T* rv = (T*)(p + L.rv);
    T* saved = (T*)(p + L.saved);
    sp_allow_lds<T>();
    // pass 1: coarse buckets
    hipLaunchKernelGGL(sp_count1_kernel, dim3(sp_xcd_grid(L.nch1)), dim3(kSpBlock), (size_t)L.nc * 4, st, is, m, n, L.s1, L.nc,
                       L.nch1, cnt1);
    hipLaunchKernelGGL(sp_tile_sum_kernel, dim3((unsigned)L.nt1), dim3(1024), 0, st, cnt1, L.n1, tsum1);
    hipLaunchKernelGGL(sp_tile_scan_kernel, dim3((unsigned)L.nt1), dim3(1024), 0, st, cnt1, L.n1, (const int32_t*)tsum1,
                       total);
    hipLaunchKernelGGL(sp_seg_kernel, dim3(1), dim3(1024), 0, st, (const int32_t*)cnt1, L.nch1, L.nc,
                       (const int32_t*)total, cstart, nch2, chb2);
    const size_t lds1 = sp_stage_bytes(L.nc, sizeof(T));
    hipLaunchKernelGGL(sp_scatter1_kernel<T>, dim3(sp_xcd_grid(L.nch1)), dim3(kSpBlock), lds1, st, is, vs, m, n, L.s1, L.nc, L.nch1,
                       (const int32_t*)cnt1, rk1, rj1, rv1);
    // pass 2: fine buckets inside each coarse bucket
    hipLaunchKernelGGL(sp_count2_kernel, dim3(sp_xcd_grid(L.nch2max)), dim3(kSpBlock), 0, st, (const int32_t*)rk1,
                       L.s0, L.nc, L.nch2max,
                       (const int32_t*)cstart, (const int32_t*)nch2, (const int32_t*)chb2, cnt2);
    hipLaunchKernelGGL(sp_tile_sum_kernel, dim3((unsigned)L.nt2), dim3(1024), 0, st, cnt2, L.n2, tsum2);
    hipLaunchKernelGGL(sp_tile_scan_kernel, dim3((unsigned)L.nt2), dim3(1024), 0, st, cnt2, L.n2, (const int32_t*)tsum2,
                       (int32_t*)nullptr);
    const size_t lds2 = sp_stage_bytes(kSpFine, sizeof(T));
    hipLaunchKernelGGL(sp_scatter2_kernel<T>, dim3(sp_xcd_grid(L.nch2max)), dim3(kSpBlock), lds2, st,
                       (const int32_t*)rk1, (const int32_t*)rj1, (const T*)rv1, L.s0, L.nc, L.nch2max,
                       (const int32_t*)cstart, (const int32_t*)nch2,
                       (const int32_t*)chb2, (const int32_t*)cnt2, rk, rj, rv);
    hipLaunchKernelGGL(sp_wstart_kernel, dim3(flat_grid(L.nw + 1, 256, 1)), dim3(256), 0, st, L.nc,
                       (const int32_t*)cstart, (const int32_t*)nch2, (const int32_t*)chb2, (const int32_t*)cnt2, wstart);
    // the window sweep
    const int vec = aligned(xs, 16) ? 1 : 0;
    hipLaunchKernelGGL(sp_apply_fwd_kernel<T>, dim3((unsigned)L.nw), dim3(kSpFwdBlock), 0, st, xs, n, L.s0, vec,
                       (const int32_t*)wstart, (const int32_t*)rk, (const T*)rv, saved);
    return PVJP_OK;
}

template <class T>
static void sp_vjp(T* ybar, int64_t n, int64_t m, T* vbar, int acc, T* ys, const char* p, const SpLayout& L,
                   hipStream_t st) {
    const int32_t* total = (const int32_t*)(p + L.total);
    const int32_t* wstart = (const int32_t*)(p + L.wstart);
    const int32_t* rk = (const int32_t*)(p + L.rk);
    const int32_t* rj = (const int32_t*)(p + L.rj);
    const T* saved = (const T*)(p + L.saved);
    if (!acc) hipLaunchKernelGGL(sp_clear_kernel<T>, dim3(flat_grid(m, 256, 8)), dim3(256), 0, st, vbar, m, total);
    const dim3 g((unsigned)L.nw), b(kSpVjpBlock);
    const int vec = aligned(ybar, 16) && (ys == nullptr || aligned(ys, 16)) ? 1 : 0;
    if (acc) {
        if (ys)
            hipLaunchKernelGGL((sp_apply_vjp_kernel<T, true, true>), g, b, 0, st, ybar, ys, n, L.s0, vec, wstart, rk, rj, saved, vbar);
        else
            hipLaunchKernelGGL((sp_apply_vjp_kernel<T, true, false>), g, b, 0, st, ybar, ys, n, L.s0, vec, wstart, rk, rj, saved, vbar);
    } else {
        if (ys)
            hipLaunchKernelGGL((sp_apply_vjp_kernel<T, false, true>), g, b, 0, st, ybar, ys, n, L.s0, vec, wstart, rk, rj, saved, vbar);
        else
            hipLaunchKernelGGL((sp_apply_vjp_kernel<T, false, false>), g, b, 0, st, ybar, ys, n, L.s0, vec, wstart, rk, rj, saved, vbar);
    }
}

static bool sp_sizes_ok(pvjp_dtype dtype, int64_t n, int64_t m) {
    if (n < 0 || m < 0 || n > INT32_MAX || m > INT32_MAX) return false;
    const int s1 = (dtype == PVJP_F64 ? sp_s0<double>() : sp_s0<float>()) + kSpFineBits;
    return ceil_div(n > 0 ? n : 1, (int64_t)1 << s1) <= kSpMaxCoarse;
}

}  // namespace pvjp

using namespace pvjp;

extern "C" size_t pvjp_scatter_plan_bytes(pvjp_dtype dtype, int64_t n, int64_t m) {
    if (!valid_dtype(dtype) || !sp_sizes_ok(dtype, n, m)) return 0;
    return sp_layout(dtype, n, m).bytes;
}

extern "C" pvjp_status pvjp_scatter_planned(pvjp_dtype dtype, void* xs, int64_t n, const int32_t* is, const void* vs,
                                            int64_t m, void* plan, size_t plan_bytes, void* stream) {
    clear_error();
    PVJP_REQUIRE(valid_dtype(dtype), "pvjp_scatter_planned: unknown dtype %d", (int)dtype);
    PVJP_REQUIRE(sp_sizes_ok(dtype, n, m), "pvjp_scatter_planned: n = %lld, m = %lld out of range", (long long)n,
                 (long long)m);
    PVJP_REQUIRE(plan != nullptr && aligned(plan, 256), "pvjp_scatter_planned: plan must be non-NULL and 256-byte aligned");
    const SpLayout L = sp_layout(dtype, n, m);
    if (plan_bytes < L.bytes) {
        set_error("pvjp_scatter_planned: plan has %zu bytes, needs %zu", plan_bytes, L.bytes);
        return PVJP_ENOMEM;
    }
    PVJP_REQUIRE(m == 0 || (is != nullptr && vs != nullptr), "pvjp_scatter_planned: is and vs must be non-NULL");
    PVJP_REQUIRE(n == 0 || xs != nullptr, "pvjp_scatter_planned: xs is NULL");
    hipStream_t st = as_stream(stream);
    char* p = reinterpret_cast<char*>(plan);
    if (dtype == PVJP_F64)
        sp_forward<double>((double*)xs, n, is, (const double*)vs, m, p, L, st);
    else
        sp_forward<float>((float*)xs, n, is, (const float*)vs, m, p, L, st);
    PVJP_LAUNCHED("pvjp_scatter_planned");
    return PVJP_OK;
}

extern "C" pvjp_status pvjp_scatter_planned_vjp(pvjp_dtype dtype, void* ys_bar, int64_t n, int64_t m, void* vs_bar,
                                                int accumulate, void* ys, const void* plan, size_t plan_bytes,
                                                void* stream) {
    clear_error();
    PVJP_REQUIRE(valid_dtype(dtype), "pvjp_scatter_planned_vjp: unknown dtype %d", (int)dtype);
    PVJP_REQUIRE(sp_sizes_ok(dtype, n, m), "pvjp_scatter_planned_vjp: n = %lld, m = %lld out of range",
                 (long long)n, (long long)m);
    PVJP_REQUIRE(plan != nullptr && aligned(plan, 256),
                 "pvjp_scatter_planned_vjp: plan must be non-NULL and 256-byte aligned");
    const SpLayout L = sp_layout(dtype, n, m);
    if (plan_bytes < L.bytes) {
        set_error("pvjp_scatter_planned_vjp: plan has %zu bytes, needs %zu", plan_bytes, L.bytes);
        return PVJP_ENOMEM;
    }
    if (m == 0) return PVJP_OK;
    PVJP_REQUIRE(vs_bar != nullptr, "pvjp_scatter_planned_vjp: vs_bar is NULL");
    PVJP_REQUIRE(n == 0 || ys_bar != nullptr, "pvjp_scatter_planned_vjp: ys_bar is NULL");
    hipStream_t st = as_stream(stream);
    const char* p = reinterpret_cast<const char*>(plan);
    if (dtype == PVJP_F64)
        sp_vjp<double>((double*)ys_bar, n, m, (double*)vs_bar, accumulate, (double*)ys, p, L, st);
    else
        sp_vjp<float>((float*)ys_bar, n, m, (float*)vs_bar, accumulate, (float*)ys, p, L, st);
    PVJP_LAUNCHED("pvjp_scatter_planned_vjp");
    return PVJP_OK;
}
