// reduce_by_index (histogram) with the special operators + * min max and
// their VJPs (Sec. 5.1.2).
//
// Forward sweep: the histogram with the extended operators of Sec. 5.1.1:
//   ADD: sums accumulated in FP64;
//   MIN/MAX: (value, lowest index) packed into one ordered 64-bit key
//            (FP32 values: key = order(v) << 32 | ~i, one atomic max per
//            element); FP64 values take a second pass that picks the lowest
//            index among the elements equal to the bin's extreme;
//   MUL: product of the non-zero values (FP64) and a zero count.
// Each block privatises a sub-histogram in LDS.  When all m bins fit, a bin
// is its own LDS slot; otherwise the LDS holds a direct-mapped cache of bins
// (slot = bin mod S) that bins claim on first touch, and an element whose
// slot belongs to another bin goes straight to a global atomic.  Hot bins
// (Zipf) are touched early and often, so they end up LDS-resident.  At the
// end each block merges its slots into the global FP64/u64 accumulators.
//
// Return sweep (the update formula of reduce with y_bar := hs_bar[inds[i]]):
//   ADD: vs_bar[i] += hs_bar[inds[i]]            (a gather);
//   MIN/MAX: vs_bar[winner[k]] += hs_bar[k]      (m writes; zero-fill first
//            when not accumulating);
//   MUL: per bin, the three zero-count cases of reduce(*).
#include <algorithm>

#include "common.h"
#include "prims.h"

namespace pvjp {

constexpr int kHistBlock = 256;
constexpr int kHistLds = 64 * 1024;   // dynamic LDS per block
constexpr int kCacheSlots = 4096;     // LDS cache slots when the bins do not fit
constexpr int32_t kEmptyTag = -1;

__device__ __forceinline__ int64_t ceil_div_dev(int64_t a, int64_t b) { return (a + b - 1) / b; }

__device__ __forceinline__ uint32_t ord32(float v) {
    const uint32_t b = __float_as_uint(v == 0.0f ? 0.0f : v);  // -0 and +0 tie
    return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}
__device__ __forceinline__ uint64_t ord64(double v) {
    const uint64_t b = (uint64_t)__double_as_longlong(v == 0.0 ? 0.0 : v);
    return (b >> 63) ? ~b : (b | (1ull << 63));
}

// Key of one element for the accumulator (u64 bits).
template <int OP>
__device__ __forceinline__ uint64_t elem_key(float v, int64_t i) {
    const uint32_t o = (OP == PVJP_MAX) ? ord32(v) : ~ord32(v);
    return ((uint64_t)o << 32) | (uint64_t)(~(uint32_t)i);
}
template <int OP>
__device__ __forceinline__ uint64_t elem_key(double v, int64_t) {
    return (OP == PVJP_MAX) ? ord64(v) : ~ord64(v);
}

template <int OP>
__device__ __forceinline__ uint64_t acc_identity() {
    if (OP == PVJP_MUL) return 0x3FF0000000000000ull;  // 1.0
    return 0ull;                                        // 0.0 for ADD; empty key
}

__device__ __forceinline__ void mul_f64_atomic(uint64_t* a, double v) {
    unsigned long long* p = reinterpret_cast<unsigned long long*>(a);
    unsigned long long old = *p, assumed;
    do {
        assumed = old;
        old = atomicCAS(p, assumed, (unsigned long long)__double_as_longlong(__longlong_as_double(assumed) * v));
    } while (assumed != old);
}

// One update of accumulator word `a` (LDS or global) and zero counter `zc`.
template <class T, int OP>
__device__ __forceinline__ void acc_update(uint64_t* a, int32_t* zc, T v, int64_t i) {
    if (OP == PVJP_ADD) {
        atomicAdd(reinterpret_cast<double*>(a), (double)v);
    } else if (OP == PVJP_MUL) {
        if (v == T(0))
            atomicAdd(zc, 1);
        else
            mul_f64_atomic(a, (double)v);
    } else {
        atomicMax(reinterpret_cast<unsigned long long*>(a), (unsigned long long)elem_key<OP>(v, i));
    }
}

// Merge of a whole slot into the global accumulator.
template <int OP>
__device__ __forceinline__ void acc_merge(uint64_t* g, int32_t* gz, uint64_t a, int32_t zc) {
    if (OP == PVJP_ADD) {
        atomicAdd(reinterpret_cast<double*>(g), __longlong_as_double((long long)a));
    } else if (OP == PVJP_MUL) {
        if (zc) atomicAdd(gz, zc);
        if (a != acc_identity<OP>()) mul_f64_atomic(g, __longlong_as_double((long long)a));
    } else {
        if (a) atomicMax(reinterpret_cast<unsigned long long*>(g), (unsigned long long)a);
    }
}

// One element's update: into its LDS slot when the block owns the bin (always
// in FULL mode), else straight into the global accumulator.
template <class T, int OP, bool CACHE, bool COUNTS>
__device__ __forceinline__ void hist_update(int32_t k, T v, int64_t i, int32_t m, int slots, uint64_t* sacc,
                                            int32_t* stag, int32_t* scnt, int32_t* szc, uint64_t* gacc, int32_t* gz,
                                            int32_t* gcount) {
    if ((uint32_t)k >= (uint32_t)m) return;
    int s;
    bool local;
    if (!CACHE) {
        s = k;
        local = true;
    } else {
        s = k & (slots - 1);
        // A slot's tag goes from empty to a bin once and never changes
        // again, so a plain read that sees a bin is final.
        int32_t t = stag[s];
        if (t == kEmptyTag) {
            t = atomicCAS(&stag[s], kEmptyTag, k);
            if (t == kEmptyTag) t = k;
        }
        local = (t == k);
    }
    if (local) {
        acc_update<T, OP>(&sacc[s], OP == PVJP_MUL ? &szc[s] : nullptr, v, i);
        if (COUNTS) atomicAdd(&scnt[s], 1);
    } else {
        acc_update<T, OP>(&gacc[k], OP == PVJP_MUL ? &gz[k] : nullptr, v, i);
        if (COUNTS) atomicAdd(&gcount[k], 1);
    }
}

// Four consecutive elements (one 16-byte load of indices).
template <class T>
struct Quad {
    int4 k;
    T v[4];
};

template <class T, bool VEC>
__device__ __forceinline__ Quad<T> load_quad(const int32_t* __restrict__ inds, const T* __restrict__ vs, int64_t e,
                                             int64_t hi) {
    Quad<T> q;
    if (VEC && e + 3 < hi) {
        q.k = *reinterpret_cast<const int4*>(inds + e);
        if (sizeof(T) == 4) {
            const float4 f = *reinterpret_cast<const float4*>(vs + e);
            q.v[0] = (T)f.x, q.v[1] = (T)f.y, q.v[2] = (T)f.z, q.v[3] = (T)f.w;
        } else {
            const double2 d0 = *reinterpret_cast<const double2*>(vs + e);
            const double2 d1 = *reinterpret_cast<const double2*>(vs + e + 2);
            q.v[0] = (T)d0.x, q.v[1] = (T)d0.y, q.v[2] = (T)d1.x, q.v[3] = (T)d1.y;
        }
    } else {
        int kk[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const bool ok = e + u < hi;
            kk[u] = ok ? inds[e + u] : -1;  // -1: out of range, skipped
            q.v[u] = ok ? vs[e + u] : T(0);
        }
        q.k = make_int4(kk[0], kk[1], kk[2], kk[3]);
    }
    return q;
}

constexpr int kHistBatch = 4;  // quads per thread per batch: 16 elements in flight

// Each block accumulates a contiguous chunk (a multiple of 4 * 256
// elements) into its LDS sub-histogram.  Loads are 16-byte vectors, four per
// thread per batch, and the next batch is loaded before the current batch's
// atomics are issued: the in-order memory counter then never makes a wave
// wait for its own atomics before it can use newly loaded data.
// FULL mode (!CACHE) writes the block's sub-histogram to `part` for a
// fixed-order merge; CACHE mode flushes its claimed slots with atomics.
template <class T, int OP, bool CACHE, bool COUNTS, bool VEC>
__global__ __launch_bounds__(kHistBlock) void hist_acc_kernel(
    const int32_t* __restrict__ inds, const T* __restrict__ vs, int64_t n, int32_t m, int64_t chunk, int slots,
    uint64_t* __restrict__ gacc, int32_t* __restrict__ gz, int32_t* __restrict__ gcount, uint64_t* __restrict__ pacc,
    int32_t* __restrict__ pz, int32_t* __restrict__ pcnt) {
    extern __shared__ uint64_t smem[];
    uint64_t* sacc = smem;                                       // [slots]
    int32_t* stag = reinterpret_cast<int32_t*>(sacc + slots);    // [slots] (CACHE)
    int32_t* scnt = stag + (CACHE ? slots : 0);                  // [slots] (COUNTS)
    int32_t* szc = scnt + (COUNTS ? slots : 0);                  // [slots] (MUL)

    for (int s = threadIdx.x; s < slots; s += kHistBlock) {
        sacc[s] = acc_identity<OP>();
        if (CACHE) stag[s] = kEmptyTag;
        if (COUNTS) scnt[s] = 0;
        if (OP == PVJP_MUL) szc[s] = 0;
    }
    __syncthreads();

    const int64_t lo = (int64_t)blockIdx.x * chunk;
    const int64_t hi = (lo + chunk < n) ? lo + chunk : n;
    constexpr int64_t kStride = 4 * kHistBlock * kHistBatch;  // elements per block batch
    Quad<T> cur[kHistBatch], nxt[kHistBatch];
#pragma unroll
    for (int u = 0; u < kHistBatch; ++u)
        cur[u] = load_quad<T, VEC>(inds, vs, lo + 4 * ((int64_t)u * kHistBlock + threadIdx.x), hi);
    for (int64_t base = lo; base < hi; base += kStride) {
        const int64_t nb = base + kStride;
        if (nb < hi) {
#pragma unroll
            for (int u = 0; u < kHistBatch; ++u)
                nxt[u] = load_quad<T, VEC>(inds, vs, nb + 4 * ((int64_t)u * kHistBlock + threadIdx.x), hi);
        }
#pragma unroll
        for (int u = 0; u < kHistBatch; ++u) {
            const int64_t e = base + 4 * ((int64_t)u * kHistBlock + threadIdx.x);
            hist_update<T, OP, CACHE, COUNTS>(cur[u].k.x, cur[u].v[0], e, m, slots, sacc, stag, scnt, szc, gacc, gz, gcount);
            hist_update<T, OP, CACHE, COUNTS>(cur[u].k.y, cur[u].v[1], e + 1, m, slots, sacc, stag, scnt, szc, gacc, gz, gcount);
            hist_update<T, OP, CACHE, COUNTS>(cur[u].k.z, cur[u].v[2], e + 2, m, slots, sacc, stag, scnt, szc, gacc, gz, gcount);
            hist_update<T, OP, CACHE, COUNTS>(cur[u].k.w, cur[u].v[3], e + 3, m, slots, sacc, stag, scnt, szc, gacc, gz, gcount);
        }
#pragma unroll
        for (int u = 0; u < kHistBatch; ++u) cur[u] = nxt[u];
    }
    __syncthreads();

    if (!CACHE) {
        const int64_t row = (int64_t)blockIdx.x * m;
        for (int s = threadIdx.x; s < m; s += kHistBlock) {
            pacc[row + s] = sacc[s];
            if (OP == PVJP_MUL) pz[row + s] = szc[s];
            if (COUNTS) pcnt[row + s] = scnt[s];
        }
        return;
    }
    for (int s = threadIdx.x; s < slots; s += kHistBlock) {
        const int32_t k = stag[s];
        if (k < 0 || k >= m) continue;
        acc_merge<OP>(&gacc[k], OP == PVJP_MUL ? &gz[k] : nullptr, sacc[s], OP == PVJP_MUL ? szc[s] : 0);
        if (COUNTS && scnt[s]) atomicAdd(&gcount[k], scnt[s]);
    }
}

// Fixed-order merge of the per-block sub-histograms (FULL mode), in two
// levels so that many waves share the work: level 1 folds slice j of the
// per-block partials (blocks j*per .. (j+1)*per-1) for 64 bins per wave;
// level 2 folds the slices in order.  Sums, products and maxima are formed in
// FP64/u64, in the same order on every run.
constexpr int kMergeSlices = 32;

template <int OP>
__device__ __forceinline__ void merge_fold(uint64_t& acc, int32_t& zz, int32_t& cc, uint64_t a, int32_t z, int32_t c) {
    if (OP == PVJP_ADD) acc = (uint64_t)__double_as_longlong(__longlong_as_double((long long)acc) +
                                                             __longlong_as_double((long long)a));
    if (OP == PVJP_MUL) acc = (uint64_t)__double_as_longlong(__longlong_as_double((long long)acc) *
                                                             __longlong_as_double((long long)a)), zz += z;
    if (OP == PVJP_MIN || OP == PVJP_MAX) acc = a > acc ? a : acc;
    cc += c;
}

template <int OP>
__global__ __launch_bounds__(256) void hist_merge1_kernel(const uint64_t* __restrict__ pacc,
                                                          const int32_t* __restrict__ pz,
                                                          const int32_t* __restrict__ pcnt, int64_t nblocks, int32_t m,
                                                          uint64_t* __restrict__ sacc, int32_t* __restrict__ sz,
                                                          int32_t* __restrict__ scnt) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y;
    if (k >= m) return;
    const int64_t per = ceil_div_dev(nblocks, kMergeSlices);
    const int64_t b0 = j * per, b1 = (b0 + per < nblocks) ? b0 + per : nblocks;
    uint64_t acc = acc_identity<OP>();
    int32_t zz = 0, cc = 0;
    for (int64_t b = b0; b < b1; ++b)
        merge_fold<OP>(acc, zz, cc, pacc[b * m + k], OP == PVJP_MUL ? pz[b * m + k] : 0, pcnt ? pcnt[b * m + k] : 0);
    sacc[(int64_t)j * m + k] = acc;
    if (OP == PVJP_MUL) sz[(int64_t)j * m + k] = zz;
    if (pcnt) scnt[(int64_t)j * m + k] = cc;
}

template <int OP>
__global__ __launch_bounds__(256) void hist_merge2_kernel(const uint64_t* __restrict__ sacc,
                                                          const int32_t* __restrict__ sz,
                                                          const int32_t* __restrict__ scnt, int32_t m,
                                                          uint64_t* __restrict__ gacc, int32_t* __restrict__ gz,
                                                          int32_t* __restrict__ gcount) {
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < m; k += (int64_t)gridDim.x * blockDim.x) {
        uint64_t acc = acc_identity<OP>();
        int32_t zz = 0, cc = 0;
        for (int j = 0; j < kMergeSlices; ++j)
            merge_fold<OP>(acc, zz, cc, sacc[(int64_t)j * m + k], OP == PVJP_MUL ? sz[(int64_t)j * m + k] : 0,
                           scnt ? scnt[(int64_t)j * m + k] : 0);
        gacc[k] = acc;
        if (OP == PVJP_MUL) gz[k] = zz;
        if (gcount) gcount[k] = cc;
    }
}

// FP64 min/max, second pass: the lowest index whose value equals the bin's
// extreme (found by the first pass as an ordered key without index).
template <int OP>
__global__ __launch_bounds__(256) void hist_f64_winner_kernel(const int32_t* __restrict__ inds,
                                                              const double* __restrict__ vs, int64_t n,
                                                              int32_t m, const uint64_t* __restrict__ gacc,
                                                              int32_t* __restrict__ winner) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t k = inds[i];
        if ((uint32_t)k >= (uint32_t)m) continue;
        if (elem_key<OP>(vs[i], i) == gacc[k]) atomicMin(&winner[k], (int32_t)i);
    }
}

template <int OP>
__global__ void hist_init_kernel(uint64_t* __restrict__ gacc, int32_t* __restrict__ gz,
                                 int32_t* __restrict__ gcount, int32_t* __restrict__ winner, int32_t m) {
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < m; k += (int64_t)gridDim.x * blockDim.x) {
        gacc[k] = acc_identity<OP>();
        if (gz) gz[k] = 0;
        if (gcount) gcount[k] = 0;
        if (winner) winner[k] = 0x7fffffff;
    }
}

template <class T, int OP>
__global__ void hist_final_kernel(const T* __restrict__ vs, const uint64_t* __restrict__ gacc,
                                  const int32_t* __restrict__ gz, int32_t m, T* __restrict__ hs,
                                  int32_t* __restrict__ winner, T* __restrict__ p, int32_t* __restrict__ z) {
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < m; k += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t a = gacc[k];
        if (OP == PVJP_ADD) {
            hs[k] = (T)__longlong_as_double((long long)a);
        } else if (OP == PVJP_MUL) {
            const double pr = __longlong_as_double((long long)a);
            const int32_t zz = gz[k];
            p[k] = (T)pr;
            z[k] = zz;
            hs[k] = zz == 0 ? (T)pr : T(0);
        } else {
            int32_t w;
            if (sizeof(T) == 4)
                w = a ? (int32_t)(~(uint32_t)(a & 0xffffffffull)) : -1;
            else
                w = (winner[k] == 0x7fffffff) ? -1 : winner[k];
            winner[k] = w;
            if (w < 0) {
                hs[k] = OP == PVJP_MAX ? -(T)__builtin_huge_val() : (T)__builtin_huge_val();
            } else if (sizeof(T) == 4) {
                // the key's upper half is the order-preserving code of the
                // winner's value; it reads back exactly except for a zero,
                // whose sign the code drops: that one is read from vs
                const uint32_t o = OP == PVJP_MAX ? (uint32_t)(a >> 32) : ~(uint32_t)(a >> 32);
                const uint32_t bits = (o & 0x80000000u) ? (o & 0x7fffffffu) : ~o;
                hs[k] = bits == 0u ? vs[w] : (T)__uint_as_float(bits);
            } else {
                hs[k] = vs[w];
            }
        }
    }
}

// ------------------------------------------------------------ VJP kernels
template <class T, bool ACC>
__global__ __launch_bounds__(256) void hist_vjp_add_kernel(const int32_t* __restrict__ inds, int64_t n,
                                                           int32_t m, const T* __restrict__ hsbar,
                                                           T* __restrict__ vsbar) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t k = inds[i];
        const T g = ((uint32_t)k < (uint32_t)m) ? hsbar[k] : T(0);
        vsbar[i] = ACC ? vsbar[i] + g : g;
    }
}

// Streaming accesses of the adjoint gathers (the indices read once, vs_bar
// written once) go non-temporal, so they do not push the gathered hs_bar
// lines out of L2.
typedef int pvjp_v4i __attribute__((ext_vector_type(4)));
typedef float pvjp_v4f __attribute__((ext_vector_type(4)));
__device__ __forceinline__ int4 nt_load_i4(const int4* p) {
    const pvjp_v4i v = __builtin_nontemporal_load(reinterpret_cast<const pvjp_v4i*>(p));
    return make_int4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ void nt_store_f4(float4* p, float4 o) {
    const pvjp_v4f v = {o.x, o.y, o.z, o.w};
    __builtin_nontemporal_store(v, reinterpret_cast<pvjp_v4f*>(p));
}

// 16-byte vector form of the gather: four indices per load, four adjoints
// per store (pointers 16-byte aligned; the last n % 4 elements are done by
// the first threads of block 0).
template <class T, bool ACC>
__global__ __launch_bounds__(256) void hist_vjp_add_vec_kernel(const int32_t* __restrict__ inds, int64_t n,
                                                               int32_t m, const T* __restrict__ hsbar,
                                                               T* __restrict__ vsbar) {
    const int64_t nq = n >> 2;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < nq; q += (int64_t)gridDim.x * blockDim.x) {
        const int4 k = nt_load_i4(reinterpret_cast<const int4*>(inds) + q);
        T g[4];
        g[0] = ((uint32_t)k.x < (uint32_t)m) ? hsbar[k.x] : T(0);
        g[1] = ((uint32_t)k.y < (uint32_t)m) ? hsbar[k.y] : T(0);
        g[2] = ((uint32_t)k.z < (uint32_t)m) ? hsbar[k.z] : T(0);
        g[3] = ((uint32_t)k.w < (uint32_t)m) ? hsbar[k.w] : T(0);
        if (sizeof(T) == 4) {
            float4* dst = reinterpret_cast<float4*>(vsbar) + q;
            float4 o = make_float4((float)g[0], (float)g[1], (float)g[2], (float)g[3]);
            if (ACC) {
                const float4 c = *dst;
                o.x += c.x, o.y += c.y, o.z += c.z, o.w += c.w;
                *dst = o;
            } else {
                nt_store_f4(dst, o);
            }
        } else {
            double2* dst = reinterpret_cast<double2*>(vsbar) + 2 * q;
            double2 o0 = make_double2((double)g[0], (double)g[1]), o1 = make_double2((double)g[2], (double)g[3]);
            if (ACC) {
                const double2 c0 = dst[0], c1 = dst[1];
                o0.x += c0.x, o0.y += c0.y, o1.x += c1.x, o1.y += c1.y;
            }
            dst[0] = o0;
            dst[1] = o1;
        }
    }
    if (blockIdx.x == 0 && threadIdx.x < (n & 3)) {
        const int64_t i = (nq << 2) + threadIdx.x;
        const int32_t k = inds[i];
        const T g = ((uint32_t)k < (uint32_t)m) ? hsbar[k] : T(0);
        vsbar[i] = ACC ? vsbar[i] + g : g;
    }
}

// Gather with the head of hs_bar staged in LDS.  A random 4-byte gather
// served by L2 brings a whole cache line into the CU for each lane, so once
// hs_bar outgrows the vector cache the gather is bound by the L2-to-CU fill
// rate, not by HBM.  One 1024-thread block per CU copies the first L bins (up
// to 160 KB) into LDS and serves them from there; bins at or beyond L come
// from global memory as before.  Each thread keeps kGatherU index quads in
// flight.
constexpr int kGatherBlock = 1024;
constexpr int kGatherLdsBytes = 160 * 1024;
constexpr int kGatherU = 4;
constexpr int32_t kGatherMinBins = 8192;  // below this hs_bar lives in the vector cache

template <class T>
__device__ __forceinline__ T gather_bin(const T* sh, int32_t L, const T* __restrict__ hsbar, int32_t m, int32_t k) {
    if ((uint32_t)k < (uint32_t)L) return sh[k];
    return ((uint32_t)k < (uint32_t)m) ? hsbar[k] : T(0);
}

template <class T, bool ACC>
__global__ __launch_bounds__(kGatherBlock) void hist_vjp_add_lds_kernel(const int32_t* __restrict__ inds, int64_t n,
                                                                        int32_t m, int32_t L,
                                                                        const T* __restrict__ hsbar,
                                                                        T* __restrict__ vsbar) {
    extern __shared__ uint64_t gather_smem[];
    T* sh = reinterpret_cast<T*>(gather_smem);
    for (int t = threadIdx.x; t < L; t += kGatherBlock) sh[t] = hsbar[t];
    __syncthreads();
    const int64_t nq = n >> 2;
    const int64_t step = (int64_t)gridDim.x * kGatherBlock;
    for (int64_t q0 = (int64_t)blockIdx.x * kGatherBlock + threadIdx.x; q0 < nq; q0 += step * kGatherU) {
        int4 k[kGatherU];
#pragma unroll
        for (int u = 0; u < kGatherU; ++u) {
            const int64_t q = q0 + u * step;
            k[u] = q < nq ? nt_load_i4(reinterpret_cast<const int4*>(inds) + q) : make_int4(-1, -1, -1, -1);
        }
#pragma unroll
        for (int u = 0; u < kGatherU; ++u) {
            const int64_t q = q0 + u * step;
            if (q >= nq) break;
            T g[4];
            g[0] = gather_bin<T>(sh, L, hsbar, m, k[u].x);
            g[1] = gather_bin<T>(sh, L, hsbar, m, k[u].y);
            g[2] = gather_bin<T>(sh, L, hsbar, m, k[u].z);
            g[3] = gather_bin<T>(sh, L, hsbar, m, k[u].w);
            if (sizeof(T) == 4) {
                float4* dst = reinterpret_cast<float4*>(vsbar) + q;
                float4 o = make_float4((float)g[0], (float)g[1], (float)g[2], (float)g[3]);
                if (ACC) {
                    const float4 c = *dst;
                    o.x += c.x, o.y += c.y, o.z += c.z, o.w += c.w;
                    *dst = o;
                } else {
                    nt_store_f4(dst, o);
                }
            } else {
                double2* dst = reinterpret_cast<double2*>(vsbar) + 2 * q;
                double2 o0 = make_double2((double)g[0], (double)g[1]), o1 = make_double2((double)g[2], (double)g[3]);
                if (ACC) {
                    const double2 c0 = dst[0], c1 = dst[1];
                    o0.x += c0.x, o0.y += c0.y, o1.x += c1.x, o1.y += c1.y;
                }
                dst[0] = o0;
                dst[1] = o1;
            }
        }
    }
    if (blockIdx.x == 0 && threadIdx.x < (n & 3)) {
        const int64_t i = (nq << 2) + threadIdx.x;
        const T g = gather_bin<T>(sh, L, hsbar, m, inds[i]);
        vsbar[i] = ACC ? vsbar[i] + g : g;
    }
}

// Lets the gather kernel take all of a CU's LDS dynamically (set once per
// instantiation; a failure here surfaces as a launch error).
template <class T, bool ACC>
static void allow_gather_lds() {
    static const bool once = [] {
        if (hipFuncSetAttribute(reinterpret_cast<const void*>(&hist_vjp_add_lds_kernel<T, ACC>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, kGatherLdsBytes) != hipSuccess)
            (void)hipGetLastError();
        return true;
    }();
    (void)once;
}

template <class T>
__global__ __launch_bounds__(256) void fill_zero_vec_kernel(T* __restrict__ x, int64_t n) {
    const int64_t nq = (int64_t)(n * sizeof(T)) >> 4;  // 16-byte words
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < nq; q += (int64_t)gridDim.x * blockDim.x)
        reinterpret_cast<int4*>(x)[q] = make_int4(0, 0, 0, 0);
    const int64_t done = (nq << 4) / (int64_t)sizeof(T);
    if (blockIdx.x == 0 && threadIdx.x < n - done) x[done + threadIdx.x] = T(0);
}

template <class T, bool ACC>
__global__ __launch_bounds__(256) void hist_vjp_mul_kernel(const int32_t* __restrict__ inds,
                                                           const T* __restrict__ vs, int64_t n, int32_t m,
                                                           const T* __restrict__ p, const int32_t* __restrict__ z,
                                                           const T* __restrict__ hsbar, T* __restrict__ vsbar) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t k = inds[i];
        T c = T(0);
        if ((uint32_t)k < (uint32_t)m) {
            const int32_t zz = z[k];
            const T v = vs[i];
            if (zz == 0)
                c = p[k] / v * hsbar[k];
            else if (zz == 1 && v == T(0))
                c = p[k] * hsbar[k];
        }
        vsbar[i] = ACC ? vsbar[i] + c : c;
    }
}

template <class T>
__global__ __launch_bounds__(256) void fill_zero_kernel(T* __restrict__ x, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        x[i] = T(0);
}

template <class T, bool ACC>
__global__ __launch_bounds__(256) void hist_vjp_winner_kernel(const int32_t* __restrict__ winner, int32_t m,
                                                              const T* __restrict__ hsbar, T* __restrict__ vsbar) {
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < m; k += (int64_t)gridDim.x * blockDim.x) {
        const int32_t w = winner[k];
        if (w >= 0) vsbar[w] = ACC ? vsbar[w] + hsbar[k] : hsbar[k];
    }
}

// ------------------------------------------------- bucket-partitioned path
// For FP32 values with + / min / max when the m bins do not fit one block's
// LDS (m up to 2^22), instead of one global atomic per element:
//   1. tile sort: one block per tile of kTile consecutive elements ranks
//      them by 4096-bin bucket in LDS, writes them back into the tile's own
//      slice of the record arrays in bucket order (fully contiguous,
//      coalesced stores whatever the bucket count) and records the tile's
//      bucket offsets;
//   2. per bucket, an exclusive scan of its run lengths over the tiles;
//      each bucket is split into work items of about kPartSeg records made
//      of whole runs;
//   3. one block per work item walks its runs and accumulates the bucket's
//      4096 bins in LDS, then writes them out as a partial;
//   4. merge the partials of each bin in work-item order.
// No pass over the input only to count it, and no record store depends on
// a global cursor.
constexpr int kPartShift = 12;
constexpr int kPartBins = 1 << kPartShift;
constexpr int kPartMaxBuckets = 1024;
constexpr int64_t kPartSeg = (int64_t)1 << 17;
constexpr int kPartScanThreads = 1024;
constexpr int kTileThreads = 512;
constexpr int kTileQuads = 4;                              // quads of elements per thread
constexpr int kTile = 4 * kTileThreads * kTileQuads;       // 8192 elements
constexpr int kTileBucketsPerThread = kPartMaxBuckets / kTileThreads;
static_assert(kTile <= 65536, "an element's position in its tile must fit 16 bits");
static_assert(kPartMaxBuckets % kTileThreads == 0, "tile threads own whole groups of buckets in the scan");
static_assert(kTile < kPartSeg, "a work item must hold any single run");

// Stores of the first cnt staged words of a tile, 16 bytes per lane.
__device__ __forceinline__ void tile_store_u32(uint32_t* __restrict__ dst, const uint32_t* stage, int cnt) {
    for (int i = 4 * (int)threadIdx.x; i < cnt; i += 4 * kTileThreads) {
        if (i + 3 < cnt)
            *reinterpret_cast<uint4*>(dst + i) = *reinterpret_cast<const uint4*>(stage + i);
        else
            for (int k = i; k < cnt; ++k) dst[k] = stage[k];
    }
}
__device__ __forceinline__ void tile_store_u16(uint16_t* __restrict__ dst, const uint16_t* stage, int cnt) {
    for (int i = 8 * (int)threadIdx.x; i < cnt; i += 8 * kTileThreads) {
        if (i + 7 < cnt)
            *reinterpret_cast<uint4*>(dst + i) = *reinterpret_cast<const uint4*>(stage + i);
        else
            for (int k = i; k < cnt; ++k) dst[k] = stage[k];
    }
}

// Tile sort.  Tile t owns records [t * kTile, t * kTile + valid) of every
// record array; toff[t][b] is the start of bucket b's run in the tile and
// toff[t][nb] the number of in-range elements.  Record of element e with bin
// k = b * 4096 + j: rval = the value's bits; for + rbin = j (2 bytes), for
// min/max rbin = j | (e - t * kTile) << 16 (4 bytes: the position in the
// tile gives back the element index for the lowest-index rule).
template <int OP, bool VEC>
__global__ __launch_bounds__(kTileThreads) void hpart_tile_kernel(const int32_t* __restrict__ inds,
                                                                const float* __restrict__ vs, int64_t n, int32_t m,
                                                                int nb, uint32_t* __restrict__ rval,
                                                                void* __restrict__ rbin, int32_t* __restrict__ toff) {
    constexpr bool KEYS = OP != PVJP_ADD;
    __shared__ int32_t bcnt[kPartMaxBuckets];  // counts, then run starts
    __shared__ __align__(16) uint32_t sval[kTile];
    __shared__ __align__(16) uint32_t sbin[KEYS ? kTile : kTile / 2];
    __shared__ IntSum::S wtot[kTileThreads / kWave];
    const int64_t base = (int64_t)blockIdx.x * kTile;
    const int64_t hi = (base + kTile < n) ? base + kTile : n;
    for (int b = threadIdx.x; b < nb; b += kTileThreads) bcnt[b] = 0;
    Quad<float> q[kTileQuads];
#pragma unroll
    for (int u = 0; u < kTileQuads; ++u)
        q[u] = load_quad<float, VEC>(inds, vs, base + 4 * ((int64_t)u * kTileThreads + threadIdx.x), hi);
    __syncthreads();
    int rank[4 * kTileQuads];
#pragma unroll
    for (int u = 0; u < kTileQuads; ++u) {
        const int32_t kk[4] = {q[u].k.x, q[u].k.y, q[u].k.z, q[u].k.w};
#pragma unroll
        for (int t = 0; t < 4; ++t)
            rank[4 * u + t] = ((uint32_t)kk[t] < (uint32_t)m) ? atomicAdd(&bcnt[kk[t] >> kPartShift], 1) : -1;
    }
    __syncthreads();
    // exclusive scan of the tile's bucket counts: each thread owns a few buckets
    int c[kTileBucketsPerThread], sum = 0;
#pragma unroll
    for (int i = 0; i < kTileBucketsPerThread; ++i) {
        const int b = kTileBucketsPerThread * (int)threadIdx.x + i;
        c[i] = b < nb ? bcnt[b] : 0;
        sum += c[i];
    }
    IntSum::S tot;
    int ex = block_exclusive_scan<IntSum, kTileThreads, false>(IntSum::S{sum}, tot, wtot).v;
    int32_t* to = toff + (int64_t)blockIdx.x * (nb + 1);
#pragma unroll
    for (int i = 0; i < kTileBucketsPerThread; ++i) {
        const int b = kTileBucketsPerThread * (int)threadIdx.x + i;
        if (b < nb) {
            bcnt[b] = ex;
            to[b] = ex;
        }
        ex += c[i];
    }
    if (threadIdx.x == 0) to[nb] = tot.v;
    __syncthreads();
    uint16_t* sbin16 = reinterpret_cast<uint16_t*>(sbin);
#pragma unroll
    for (int u = 0; u < kTileQuads; ++u) {
        const int32_t kk[4] = {q[u].k.x, q[u].k.y, q[u].k.z, q[u].k.w};
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            if (rank[4 * u + t] < 0) continue;
            const int slot = bcnt[kk[t] >> kPartShift] + rank[4 * u + t];
            const uint32_t j = (uint32_t)kk[t] & (kPartBins - 1);
            sval[slot] = __float_as_uint(q[u].v[t]);
            if (KEYS)
                sbin[slot] = j | ((uint32_t)(4 * (u * kTileThreads + (int)threadIdx.x) + t) << 16);
            else
                sbin16[slot] = (uint16_t)j;
        }
    }
    __syncthreads();
    tile_store_u32(rval + base, sval, tot.v);
    if (KEYS)
        tile_store_u32(reinterpret_cast<uint32_t*>(rbin) + base, sbin, tot.v);
    else
        tile_store_u16(reinterpret_cast<uint16_t*>(rbin) + base, sbin16, tot.v);
}

// Per chunk c of kColChunk tiles (grid y) and group of kColThreads buckets
// (grid x), a thread per bucket b walks the chunk's tiles: the bucket-major
// run descriptor D[b][t] = start of b's run in tile t | its length << 16,
// the run's start within the chunk's part of the bucket (Ploc), the chunk
// total ctot[b][c] and the chunk-local start of its last non-empty run
// clast[b][c] (-1: none).  Reads of a tile's offsets are coalesced across
// the threads; each thread writes its rows 16 bytes at a time.
constexpr int kColChunk = 32;
constexpr int kColThreads = 256;
__global__ __launch_bounds__(kColThreads) void hpart_colscan_kernel(const int32_t* __restrict__ toff, int ntiles,
                                                                    int nb, int nchunks, uint32_t* __restrict__ D,
                                                                    int32_t* __restrict__ Ploc,
                                                                    int32_t* __restrict__ ctot,
                                                                    int32_t* __restrict__ clast) {
    const int b = blockIdx.x * kColThreads + (int)threadIdx.x;
    const int c = blockIdx.y;
    if (b >= nb) return;
    const int t0 = c * kColChunk;
    const int nt = (ntiles - t0 < kColChunk) ? ntiles - t0 : kColChunk;
    uint32_t* Db = D + (int64_t)b * ntiles + t0;
    int32_t* Pb = Ploc + (int64_t)b * ntiles + t0;
    // rows of D and Ploc are 16-byte aligned when ntiles is a multiple of 4
    const bool vec = (ntiles & 3) == 0;
    // every offset of the chunk is loaded before any is used
    int s0[kColChunk], s1[kColChunk];
#pragma unroll
    for (int u = 0; u < kColChunk; ++u) {
        const int32_t* o = toff + (int64_t)(t0 + (u < nt ? u : 0)) * (nb + 1) + b;
        s0[u] = o[0];
        s1[u] = o[1];
    }
    int run = 0, last = -1;
#pragma unroll
    for (int q = 0; q < kColChunk; q += 4) {
        uint32_t d[4];
        int p[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int len = q + u < nt ? s1[q + u] - s0[q + u] : 0;
            d[u] = (uint32_t)s0[q + u] | ((uint32_t)len << 16);
            p[u] = run;
            if (len > 0) last = run;
            run += len;
        }
        if (q >= nt) continue;
        if (vec && q + 4 <= nt) {
            *reinterpret_cast<uint4*>(Db + q) = make_uint4(d[0], d[1], d[2], d[3]);
            *reinterpret_cast<int4*>(Pb + q) = make_int4(p[0], p[1], p[2], p[3]);
        } else {
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                if (q + u < nt) {
                    Db[q + u] = d[u];
                    Pb[q + u] = p[u];
                }
            }
        }
    }
    ctot[(int64_t)b * nchunks + c] = run;
    clast[(int64_t)b * nchunks + c] = last;
}

// Per bucket (one block each): chunk prefixes (ctot is overwritten with the
// exclusive prefix) and the bucket's work-item count -- item i takes the
// runs that start in [i * kPartSeg, (i + 1) * kPartSeg), so the count is one
// more than the last non-empty run's start over kPartSeg, none for an empty
// bucket.
constexpr int kBscanThreads = 256;
__global__ __launch_bounds__(kBscanThreads) void hpart_bscan_kernel(int32_t* __restrict__ ctot,
                                                                    const int32_t* __restrict__ clast,
                                                                    int nchunks, int32_t* __restrict__ bitems) {
    __shared__ IntSum::S wtot[kBscanThreads / kWave];
    __shared__ int lastp;
    const int b = blockIdx.x;
    int32_t* cb = ctot + (int64_t)b * nchunks;
    const int32_t* lb = clast + (int64_t)b * nchunks;
    if (threadIdx.x == 0) lastp = -1;
    int carry = 0;
    for (int c0 = 0; c0 < nchunks; c0 += kBscanThreads) {
        const int c = c0 + (int)threadIdx.x;
        const int tc = c < nchunks ? cb[c] : 0;
        const int lc = c < nchunks ? lb[c] : -1;
        IntSum::S tot;
        const int ex = block_exclusive_scan<IntSum, kBscanThreads, false>(IntSum::S{tc}, tot, wtot).v;
        if (c < nchunks) cb[c] = carry + ex;
        if (lc >= 0) atomicMax(&lastp, carry + ex + lc);
        carry += tot.v;
    }
    __syncthreads();
    if (threadIdx.x == 0) bitems[b] = lastp >= 0 ? (int)(lastp / kPartSeg) + 1 : 0;
}

// One block: work-item starts per bucket.
__global__ __launch_bounds__(kPartScanThreads) void hpart_scan_kernel(const int32_t* __restrict__ bitems, int nb,
                                                                      int32_t* __restrict__ istart) {
    __shared__ IntSum::S wtot[kPartScanThreads / kWave];
    const int b = threadIdx.x;
    const int items = b < nb ? bitems[b] : 0;
    IntSum::S itot;
    const int iex = block_exclusive_scan<IntSum, kPartScanThreads, false>(IntSum::S{items}, itot, wtot).v;
    if (b < nb) istart[b] = iex;
    if (b == 0) istart[nb] = itot.v;
}

// First tile of every work item: item i of bucket b takes the tiles whose run
// of b starts in [i * kPartSeg, (i + 1) * kPartSeg), i.e. from the first tile
// t with P[b][t] >= i * kPartSeg, where P[b][t] = Ploc + the chunk prefix is
// the start of b's run in tile t within the bucket.  Non-empty runs start at
// 0 and are shorter than kPartSeg, so up to the last non-empty run every
// such interval holds a run start, and exactly one thread finds the first
// tile of each item.
__global__ __launch_bounds__(256) void hpart_items_kernel(const int32_t* __restrict__ Ploc,
                                                          const int32_t* __restrict__ cpre, int ntiles, int nb,
                                                          int nchunks, const int32_t* __restrict__ istart,
                                                          int32_t* __restrict__ itile) {
    const int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (g >= (int64_t)nb * ntiles) return;
    const int b = (int)(g / ntiles), t = (int)(g % ntiles);
    auto P = [&](int tt) {
        return (int64_t)Ploc[(int64_t)b * ntiles + tt] + cpre[(int64_t)b * nchunks + tt / kColChunk];
    };
    const int items = istart[b + 1] - istart[b];
    int64_t i;
    if (t == 0) {
        i = 0;
    } else {
        i = P(t) / kPartSeg;
        if (i == 0 || i * kPartSeg <= P(t - 1)) return;
    }
    if (i < items) itile[istart[b] + i] = t;
}

// One block per work item accumulates its bucket's 4096 bins in LDS.  The
// accumulators are kept in kAccCopies interleaved copies (bin j, copy c at
// j * kAccCopies + c; lane l updates copy l % kAccCopies), so lanes of a
// wave that hit one hot bin -- Zipf-distributed indices put a large share
// of the records on a few bins -- update different words in different
// banks instead of serialising on one address.  The copies are folded in a
// fixed order at the end.
// Each wave takes a contiguous share of the item's tiles.  It loads the run
// descriptors of 64 tiles at a time (a lane each, one coalesced load) and
// reads kAccPar groups of up to kAccGroup consecutive runs side by side
// (when the share is short, its runs are split evenly between the groups,
// which keeps long runs of a hot bucket spread over all of a lane's
// loads).  Within such a group the runs form one flat
// sequence (lane l takes records l, l + 64, ...; a record finds its run by
// comparing its rank with the group's run prefix), so lanes stay full
// whatever the run lengths, and each lane has kAccPar * kAccSlots records
// in flight.
constexpr int kAccBlock = 1024;
constexpr int kAccCopies = 2;
constexpr int kXcds = 8;  // accelerator dies of an MI355X, each with its own L2
constexpr int kXcdMapBuckets = 128;
constexpr int kAccGroup = 8;
constexpr int kAccSlots = 4;  // records per lane and group in flight
constexpr int kAccPar = 2;    // groups read side by side

// Uniform run table of one group: run u holds records [pre[u], pre[u + 1])
// of the group's flat sequence, at record slot off[u] + r.
struct AccGroup {
    int pre[kAccGroup + 1];
    uint32_t off[kAccGroup];
};

// Runs first .. first + count - 1 of the lanes' descriptors (count <=
// kAccGroup); slots are counted from the start of the chunk's first tile.
__device__ __forceinline__ AccGroup acc_group(uint32_t dl, int first, int count) {
    AccGroup G;
    G.pre[0] = 0;
#pragma unroll
    for (int u = 0; u < kAccGroup; ++u) {
        uint32_t d = 0u;
        if (u < count) d = (uint32_t)__builtin_amdgcn_readlane((int)dl, first + u);
        const int len = (int)(d >> 16);
        G.off[u] = (uint32_t)(first + u) * (uint32_t)kTile + (d & 0xffffu) - (uint32_t)G.pre[u];
        G.pre[u + 1] = G.pre[u] + len;
    }
    return G;
}

// The empty asm keeps the chain as conditional moves from scalar registers
// (left alone, the compiler turns it into an indexed load from a private
// array in scratch memory).
__device__ __forceinline__ uint32_t acc_slot(const AccGroup& G, int r) {
    uint32_t o = G.off[0];
#pragma unroll
    for (int u = 1; u < kAccGroup; ++u) {
        o = (r >= G.pre[u]) ? G.off[u] : o;
        __asm__ volatile("" : "+v"(o));
    }
    return o + (uint32_t)r;
}

template <int OP, bool COUNTS>
__device__ __forceinline__ void acc_record(uint64_t* acc, int32_t* cnt, uint32_t copy, int64_t tile_base,
                                           uint32_t at, uint32_t v, uint32_t bn) {
    const uint32_t j = bn & (kPartBins - 1);
    if (OP != PVJP_ADD) {
        // the tile start plus the position in the tile: the element index
        const int64_t e = tile_base + (int64_t)(at & ~(uint32_t)(kTile - 1)) + (int64_t)(bn >> 16);
        // A key only ever grows, so a record whose key does not exceed the
        // word read now cannot win and skips the atomic.  A read of one word
        // by many lanes is a broadcast, while atomics on one word serialise:
        // on a hot bin almost every record stops here, and on a uniform one
        // the expected number of winners among k records is the k-th
        // harmonic number.
        const uint64_t key = elem_key<OP>(__uint_as_float(v), e);
        uint64_t* w = &acc[j * kAccCopies + copy];
        if (key > __hip_atomic_load(w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP))
            atomicMax(reinterpret_cast<unsigned long long*>(w), (unsigned long long)key);
    } else {
        atomicAdd(reinterpret_cast<double*>(&acc[j * kAccCopies + copy]), (double)__uint_as_float(v));
    }
    if (COUNTS) atomicAdd(&cnt[j], 1);
}

// The work item of this block (-1: none) with its bucket and tiles.  With
// many buckets (short runs): blocks go to the XCDs round-robin, so each XCD
// takes an equal contiguous range of the items (the grid is a multiple of
// kXcds and covers them) and items of adjacent buckets, whose runs share
// cache lines in every tile, meet in one L2.  With few buckets the runs span
// whole lines and items go in grid order.
struct PartItem {
    int item, b, ta, tb;
};

__device__ __forceinline__ PartItem part_item(int nb, int ntiles, const int32_t* __restrict__ istart,
                                              const int32_t* __restrict__ itile) {
    PartItem I{-1, 0, 0, 0};
    const int nitems = istart[nb];
    int item = (int)blockIdx.x;
    if (nb >= kXcdMapBuckets) {
        const int per = (nitems + kXcds - 1) / kXcds;
        if ((int)(blockIdx.x / kXcds) >= per) return I;
        item = (int)(blockIdx.x % kXcds) * per + (int)(blockIdx.x / kXcds);
    }
    if (item >= nitems) return I;
    int lo = 0, hi = nb;  // last bucket b with istart[b] <= item
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (istart[mid] <= item) lo = mid; else hi = mid;
    }
    I.item = item;
    I.b = lo;
    I.ta = itile[item];
    I.tb = (item + 1 < istart[lo + 1]) ? itile[item + 1] : ntiles;
    return I;
}

// Walks the item's records (see above) and hands each lane's records to
// fn(tile_base, ok, slot, value bits, bin word), the whole wave calling.
template <bool KEYS, class Fn>
__device__ __forceinline__ void part_walk(const uint32_t* __restrict__ rval, const void* __restrict__ rbin,
                                          const uint32_t* __restrict__ D, int ntiles, const PartItem& I, Fn fn) {
    constexpr int NW = kAccBlock / kWave;
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = __builtin_amdgcn_readfirstlane((int)threadIdx.x / kWave);
    const int span = (I.tb - I.ta + NW - 1) / NW;
    const int w0 = I.ta + wave * span;
    const int w1 = (w0 + span < I.tb) ? w0 + span : I.tb;
    const uint32_t* Db = D + (int64_t)I.b * ntiles;
    for (int c0 = w0; c0 < w1; c0 += kWave) {
        // lane l: the descriptor of tile c0 + l (an empty run past the share)
        const uint32_t dl = (c0 + lane < w1) ? Db[c0 + lane] : 0u;
        const int nc = (w1 - c0 < kWave) ? w1 - c0 : kWave;
        const int64_t tbase = (int64_t)c0 * kTile;
        const char* cv = reinterpret_cast<const char*>(rval + tbase);
        const char* cb = reinterpret_cast<const char*>(rbin) + tbase * (KEYS ? 4 : 2);
        // a pass reads kAccPar groups of kAccGroup consecutive runs side by
        // side; fewer runs than one pass takes are split evenly between them
        const bool split = nc < kAccPar * kAccGroup;
        const int ps = split ? (nc + kAccPar - 1) / kAccPar : kAccGroup;
        for (int g = 0; g < nc; g += kAccPar * ps) {
            AccGroup G[kAccPar];
            int R = 0;
#pragma unroll
            for (int p = 0; p < kAccPar; ++p) {
                const int first = g + p * ps;
                const int count = nc - first < ps ? nc - first : ps;
                G[p] = acc_group(dl, first, count);
                R = G[p].pre[kAccGroup] > R ? G[p].pre[kAccGroup] : R;
            }
            for (int r0 = 0; r0 < R; r0 += kAccSlots * kWave) {
                uint32_t at[kAccPar * kAccSlots], vv[kAccPar * kAccSlots], bb[kAccPar * kAccSlots];
                bool ok[kAccPar * kAccSlots];
#pragma unroll
                for (int s = 0; s < kAccPar * kAccSlots; ++s) {
                    const int p = s / kAccSlots;
                    const int r = r0 + (s % kAccSlots) * kWave + lane;
                    ok[s] = r < G[p].pre[kAccGroup];
                    // past the group's end a lane reads the chunk's first
                    // slot (always allocated) and drops it: the loads stay
                    // outside branches, so all of them are in flight at once
                    at[s] = ok[s] ? acc_slot(G[p], r) : 0u;
                    // a uniform base and a 32-bit byte offset per lane
                    vv[s] = *reinterpret_cast<const uint32_t*>(cv + (at[s] << 2));
                    bb[s] = KEYS ? *reinterpret_cast<const uint32_t*>(cb + (at[s] << 2))
                                 : (uint32_t)*reinterpret_cast<const uint16_t*>(cb + (at[s] << 1));
                }
#pragma unroll
                for (int s = 0; s < kAccPar * kAccSlots; ++s) fn(tbase, ok[s], at[s], vv[s], bb[s]);
            }
        }
    }
}

template <int OP, bool COUNTS>
__global__ __launch_bounds__(kAccBlock) void hpart_acc_kernel(const uint32_t* __restrict__ rval,
                                                              const void* __restrict__ rbin, int nb, int ntiles,
                                                              const uint32_t* __restrict__ D,
                                                              const int32_t* __restrict__ istart,
                                                              const int32_t* __restrict__ itile,
                                                              uint64_t* __restrict__ pacc,
                                                              int32_t* __restrict__ pcnt) {
    constexpr bool KEYS = OP != PVJP_ADD;
    __shared__ uint64_t acc[kPartBins * kAccCopies];
    __shared__ int32_t cnt[COUNTS ? kPartBins : 1];
    const PartItem I = part_item(nb, ntiles, istart, itile);
    if (I.item < 0) return;
    const int item = I.item;
    for (int j = threadIdx.x; j < kPartBins * kAccCopies; j += kAccBlock) acc[j] = acc_identity<OP>();
    if (COUNTS)
        for (int j = threadIdx.x; j < kPartBins; j += kAccBlock) cnt[j] = 0;
    __syncthreads();
    const uint32_t copy = threadIdx.x & (kAccCopies - 1);
    part_walk<KEYS>(rval, rbin, D, ntiles, I, [&](int64_t tbase, bool ok, uint32_t at, uint32_t v, uint32_t bn) {
        if (ok) acc_record<OP, COUNTS>(acc, cnt, copy, tbase, at, v, bn);
    });
    __syncthreads();
    for (int j = threadIdx.x; j < kPartBins; j += kAccBlock) {
        uint64_t v = acc[j * kAccCopies];
#pragma unroll
        for (int c = 1; c < kAccCopies; ++c) {
            const uint64_t w = acc[j * kAccCopies + c];
            if (OP == PVJP_ADD)
                v = (uint64_t)__double_as_longlong(__longlong_as_double((long long)v) + __longlong_as_double((long long)w));
            else
                v = w > v ? w : v;
        }
        pacc[(int64_t)item * kPartBins + j] = v;
        if (COUNTS) pcnt[(int64_t)item * kPartBins + j] = cnt[j];
    }
}
template <int OP>
__global__ __launch_bounds__(256) void hpart_merge_kernel(const uint64_t* __restrict__ pacc,
                                                          const int32_t* __restrict__ pcnt,
                                                          const int32_t* __restrict__ istart, int32_t m,
                                                          uint64_t* __restrict__ gacc, int32_t* __restrict__ gcount) {
    // A thread per bin; eight work items' partials in flight, folded in order.
    constexpr int U = 8;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < m; k += (int64_t)gridDim.x * blockDim.x) {
        const int b = (int)(k >> kPartShift), j = (int)(k & (kPartBins - 1));
        uint64_t acc = acc_identity<OP>();
        int32_t zz = 0, cc = 0;
        const int i1 = istart[b + 1];
        int it = istart[b];
        for (; it + U <= i1; it += U) {
            uint64_t v[U];
            int32_t c[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                v[u] = pacc[(int64_t)(it + u) * kPartBins + j];
                c[u] = pcnt ? pcnt[(int64_t)(it + u) * kPartBins + j] : 0;
            }
#pragma unroll
            for (int u = 0; u < U; ++u) merge_fold<OP>(acc, zz, cc, v[u], 0, c[u]);
        }
        for (; it < i1; ++it)
            merge_fold<OP>(acc, zz, cc, pacc[(int64_t)it * kPartBins + j], 0, pcnt ? pcnt[(int64_t)it * kPartBins + j] : 0);
        gacc[k] = acc;
        if (gcount) gcount[k] = cc;
    }
}

// log-add-exp over the partition (the operator of the log-add-exp
// reduce_by_index): per work item, each bin's largest element (ordered keys,
// one sweep over the item's records), then the sum of e^(x - that maximum)
// over the same records in FP64 (a second sweep); the partial of a bin is
// its (maximum key, sum).  -inf elements add nothing; an element equal to
// the maximum adds e^0 = 1, also when both are +inf.
__device__ __forceinline__ float unord32(uint32_t o) {
    return __uint_as_float((o & 0x80000000u) ? (o & 0x7fffffffu) : ~o);
}

__global__ __launch_bounds__(kAccBlock) void hpart_lae_acc_kernel(const uint32_t* __restrict__ rval,
                                                                  const void* __restrict__ rbin, int nb, int ntiles,
                                                                  const uint32_t* __restrict__ D,
                                                                  const int32_t* __restrict__ istart,
                                                                  const int32_t* __restrict__ itile,
                                                                  double* __restrict__ psum,
                                                                  uint32_t* __restrict__ pmax) {
    __shared__ uint32_t mx[kPartBins];
    __shared__ double sm[kPartBins * kAccCopies];
    const PartItem I = part_item(nb, ntiles, istart, itile);
    if (I.item < 0) return;
    for (int j = threadIdx.x; j < kPartBins; j += kAccBlock) mx[j] = 0u;
    for (int j = threadIdx.x; j < kPartBins * kAccCopies; j += kAccBlock) sm[j] = 0.0;
    __syncthreads();
    part_walk<false>(rval, rbin, D, ntiles, I, [&](int64_t, bool ok, uint32_t, uint32_t v, uint32_t bn) {
        if (ok) atomicMax(&mx[bn & (kPartBins - 1)], ord32(__uint_as_float(v)));
    });
    __syncthreads();
    const uint32_t copy = threadIdx.x & (kAccCopies - 1);
    part_walk<false>(rval, rbin, D, ntiles, I, [&](int64_t, bool ok, uint32_t, uint32_t v, uint32_t bn) {
        if (!ok) return;
        const uint32_t j = bn & (kPartBins - 1);
        const float x = __uint_as_float(v), m = unord32(mx[j]);
        if (x != -INFINITY && m != -INFINITY)
            atomicAdd(&sm[j * kAccCopies + copy], (double)(x == m ? 1.0f : expf(x - m)));
    });
    __syncthreads();
    for (int j = threadIdx.x; j < kPartBins; j += kAccBlock) {
        double v = sm[j * kAccCopies];
#pragma unroll
        for (int c = 1; c < kAccCopies; ++c) v += sm[j * kAccCopies + c];
        psum[(int64_t)I.item * kPartBins + j] = v;
        pmax[(int64_t)I.item * kPartBins + j] = mx[j];
    }
}

// A thread per bin folds its items' (maximum, sum) partials in item order:
// the largest maximum M over the items that hold a live element, then
// sum_i s_i e^(m_i - M) (1 where m_i = M), and hs = M + log(sum); -inf for a
// bin without live elements.  A NaN anywhere in the bin makes the sum NaN.
__global__ __launch_bounds__(256) void hpart_lae_merge_kernel(const double* __restrict__ psum,
                                                              const uint32_t* __restrict__ pmax,
                                                              const int32_t* __restrict__ istart, int32_t m,
                                                              float* __restrict__ hs) {
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < m; k += (int64_t)gridDim.x * blockDim.x) {
        const int b = (int)(k >> kPartShift), j = (int)(k & (kPartBins - 1));
        const int i0 = istart[b], i1 = istart[b + 1];
        uint32_t mk = 0u;
        bool any = false;
        for (int it = i0; it < i1; ++it) {
            const double sv = psum[(int64_t)it * kPartBins + j];
            if (sv != 0.0 || sv != sv) {
                const uint32_t key = pmax[(int64_t)it * kPartBins + j];
                mk = key > mk ? key : mk;
                any = true;
            }
        }
        if (!any) {
            hs[k] = -INFINITY;
            continue;
        }
        const double M = (double)unord32(mk);
        double S = 0.0;
        for (int it = i0; it < i1; ++it) {
            const double sv = psum[(int64_t)it * kPartBins + j];
            if (sv != 0.0 || sv != sv) {
                const uint32_t key = pmax[(int64_t)it * kPartBins + j];
                S += key == mk ? sv : sv * exp((double)unord32(key) - M);
            }
        }
        hs[k] = (float)(M + log(S));
    }
}

// ------------------------------------------------------------------ host
static size_t slot_bytes(int op, bool counts, bool cache) {
    return 8 + (counts ? 4 : 0) + (op == PVJP_MUL ? 4 : 0) + (cache ? 4 : 0);
}

constexpr int kCuCount = 256;         // MI355X compute units
constexpr int kLdsPerCu = 160 * 1024;  // LDS bytes per CU on gfx950
constexpr int64_t kMaxPartEntries = (int64_t)1 << 23;

struct HistPlan {
    bool cache;
    int slots;
    int64_t grid, chunk;
    size_t lds;
};

// FULL mode when the m bins fit one block's LDS; then as many resident blocks
// as LDS allows (up to 8 per CU), capped so the per-block partials stay
// bounded.  CACHE mode otherwise, 3 blocks per CU.
static HistPlan hist_plan(int op, int64_t n, int64_t m, bool counts) {
    HistPlan P{};
    const int full_slots = (int)(kHistLds / slot_bytes(op, counts, false));
    P.cache = m > full_slots;
    if (!P.cache) {
        P.slots = (int)m;
        P.lds = (size_t)m * slot_bytes(op, counts, false);
    } else {
        int slots = kCacheSlots;
        while ((size_t)slots * slot_bytes(op, counts, true) > (size_t)kHistLds) slots >>= 1;
        P.slots = slots;
        P.lds = (size_t)slots * slot_bytes(op, counts, true);
    }
    int64_t per_cu = kLdsPerCu / (int64_t)(P.lds > 0 ? P.lds : 1);
    if (per_cu > 8) per_cu = 8;
    // Whole bin tables: two blocks per CU, each thread with two batches of
    // 16 elements in flight, already cover HBM's latency, and every further
    // block adds m partials to the merge (at m = 2^10, 8 blocks per CU took
    // 0.20 / 0.14 ms for + / max, 4 took 0.19 / 0.124, 2 take 0.18 / 0.125,
    // 1 takes 0.21 / 0.19).
    if (!P.cache && per_cu > 2) per_cu = 2;
    if (per_cu < 1) per_cu = 1;
    int64_t g = kCuCount * per_cu;
    if (!P.cache && g * m > kMaxPartEntries) g = kMaxPartEntries / m > 0 ? kMaxPartEntries / m : 1;
    const int64_t quantum = 4 * kHistBlock;  // chunks are whole vector rows
    int64_t want = ceil_div(n > 0 ? n : 1, (int64_t)4 * kHistBlock * kHistBatch);
    if (g > want) g = want;
    if (g < 1) g = 1;
    P.chunk = ceil_div(ceil_div(n > 0 ? n : 1, g), quantum) * quantum;
    P.grid = ceil_div(n > 0 ? n : 1, P.chunk);
    return P;
}

// The bucket-partitioned path serves FP32 + / min / max when m does not fit
// one block's LDS and the buckets fit the scan block.
static bool use_partition(int op, bool f32, int64_t m, bool counts) {
    const int full_slots = (int)(kHistLds / slot_bytes(op, counts, false));
    return f32 && op != PVJP_MUL && m > full_slots && ceil_div(m, kPartBins) <= kPartMaxBuckets;
}

struct PartLayout {
    int nb, ntiles, nchunks;
    int64_t items_max;
    size_t toff, D, Ploc, ctot, clast, bitems, istart, itile, rval, rbin, pacc, pcnt, total;
};

static PartLayout part_layout(int64_t n, int64_t m) {
    PartLayout L{};
    L.nb = (int)ceil_div(m, kPartBins);
    L.ntiles = (int)ceil_div(n > 0 ? n : 1, kTile);
    L.nchunks = (int)ceil_div(L.ntiles, kColChunk);
    L.items_max = ceil_div(n > 0 ? n : 1, kPartSeg) + L.nb;
    const size_t slots = (size_t)L.ntiles * kTile;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t at = o;
        o += align_up(bytes, 256);
        return at;
    };
    L.toff = take((size_t)L.ntiles * (L.nb + 1) * 4);
    L.D = take((size_t)L.nb * L.ntiles * 4);
    L.Ploc = take((size_t)L.nb * L.ntiles * 4);
    L.ctot = take((size_t)L.nb * L.nchunks * 4);
    L.clast = take((size_t)L.nb * L.nchunks * 4);
    L.bitems = take((size_t)L.nb * 4);
    L.istart = take((size_t)(L.nb + 1) * 4);
    L.itile = take((size_t)L.items_max * 4);
    L.rval = take(slots * 4);
    L.rbin = take(slots * 4);  // 2 bytes per record for +, 4 for min/max
    L.pacc = take((size_t)L.items_max * kPartBins * 8);
    L.pcnt = take((size_t)L.items_max * kPartBins * 4);
    L.total = o;
    return L;
}

// Covers both plans (with and without counts): the FULL/CACHE choice and the
// grid depend on whether counts are requested.
static size_t hist_ws(int op, int64_t n, int64_t m, bool f32) {
    if (use_partition(op, f32, m, false) || use_partition(op, f32, m, true)) {
        // either plan may run: reserve the larger of the two layouts below
        const size_t part = part_layout(n, m).total;
        size_t other = 0;
        for (int counts = 0; counts < 2; ++counts) {
            const HistPlan P = hist_plan(op, n, m, counts != 0);
            if (!P.cache) other = std::max(other, align_up((size_t)(P.grid + kMergeSlices) * m * 16, 256));
        }
        return align_up((size_t)m * 8, 256) + std::max(part, other);
    }
    size_t part = 0;
    for (int counts = 0; counts < 2; ++counts) {
        const HistPlan P = hist_plan(op, n, m, counts != 0);
        if (!P.cache) {
            // per-block partials and the merge slices: acc 8 + zeros 4 + counts 4
            const size_t b = align_up((size_t)(P.grid + kMergeSlices) * m * 16, 256);
            if (b > part) part = b;
        }
    }
    return align_up((size_t)m * 8, 256) + (op == PVJP_MUL ? align_up((size_t)m * 4, 256) : 0) + part;
}

// The partition shared by the accumulators: the tile sort, the run
// descriptors and the work items.
template <int OP>
static void part_sort(const int32_t* inds, const float* vs, int64_t n, int32_t m, const PartLayout& L, char* base,
                      hipStream_t st) {
    int32_t* toff = reinterpret_cast<int32_t*>(base + L.toff);
    uint32_t* D = reinterpret_cast<uint32_t*>(base + L.D);
    int32_t* Ploc = reinterpret_cast<int32_t*>(base + L.Ploc);
    int32_t* ctot = reinterpret_cast<int32_t*>(base + L.ctot);
    int32_t* clast = reinterpret_cast<int32_t*>(base + L.clast);
    int32_t* bitems = reinterpret_cast<int32_t*>(base + L.bitems);
    int32_t* istart = reinterpret_cast<int32_t*>(base + L.istart);
    int32_t* itile = reinterpret_cast<int32_t*>(base + L.itile);
    uint32_t* rval = reinterpret_cast<uint32_t*>(base + L.rval);
    void* rbin = base + L.rbin;
    const bool vec = aligned(inds, 16) && aligned(vs, 16);
    // n == 0 still runs one (empty) tile, so every table is written
    if (vec)
        hipLaunchKernelGGL((hpart_tile_kernel<OP, true>), dim3(L.ntiles), dim3(kTileThreads), 0, st, inds, vs, n, m,
                           L.nb, rval, rbin, toff);
    else
        hipLaunchKernelGGL((hpart_tile_kernel<OP, false>), dim3(L.ntiles), dim3(kTileThreads), 0, st, inds, vs, n, m,
                           L.nb, rval, rbin, toff);
    hipLaunchKernelGGL(hpart_colscan_kernel, dim3((unsigned)ceil_div(L.nb, kColThreads), L.nchunks),
                       dim3(kColThreads), 0, st, toff, L.ntiles, L.nb, L.nchunks, D, Ploc, ctot, clast);
    hipLaunchKernelGGL(hpart_bscan_kernel, dim3(L.nb), dim3(kBscanThreads), 0, st, ctot, clast, L.nchunks, bitems);
    hipLaunchKernelGGL(hpart_scan_kernel, dim3(1), dim3(kPartScanThreads), 0, st, bitems, L.nb, istart);
    hipLaunchKernelGGL(hpart_items_kernel, dim3((unsigned)ceil_div((int64_t)L.nb * L.ntiles, 256)), dim3(256), 0, st,
                       Ploc, ctot, L.ntiles, L.nb, L.nchunks, istart, itile);
}

template <int OP>
static void run_partitioned(const int32_t* inds, const float* vs, int64_t n, int32_t m, int32_t* count, char* w,
                            size_t off, uint64_t* gacc, hipStream_t st) {
    const PartLayout L = part_layout(n, m);
    char* base = w + off;
    part_sort<OP>(inds, vs, n, m, L, base, st);
    const uint32_t* D = reinterpret_cast<const uint32_t*>(base + L.D);
    const int32_t* istart = reinterpret_cast<const int32_t*>(base + L.istart);
    const int32_t* itile = reinterpret_cast<const int32_t*>(base + L.itile);
    const uint32_t* rval = reinterpret_cast<const uint32_t*>(base + L.rval);
    const void* rbin = base + L.rbin;
    uint64_t* pacc = reinterpret_cast<uint64_t*>(base + L.pacc);
    int32_t* pcnt = reinterpret_cast<int32_t*>(base + L.pcnt);
    const unsigned agrid = (unsigned)(ceil_div(L.items_max, (int64_t)kXcds) * kXcds);
    if (count)
        hipLaunchKernelGGL((hpart_acc_kernel<OP, true>), dim3(agrid), dim3(kAccBlock), 0, st, rval, rbin, L.nb,
                           L.ntiles, D, istart, itile, pacc, pcnt);
    else
        hipLaunchKernelGGL((hpart_acc_kernel<OP, false>), dim3(agrid), dim3(kAccBlock), 0, st, rval, rbin, L.nb,
                           L.ntiles, D, istart, itile, pacc, pcnt);
    hipLaunchKernelGGL(hpart_merge_kernel<OP>, dim3(flat_grid(m, 256, 1)), dim3(256), 0, st, pacc,
                       count ? pcnt : nullptr, istart, m, gacc, count);
}

// The log-add-exp reduce_by_index on the partition (FP32, the bins beyond
// one block's LDS): one tile sort, two sweeps per work item, one merge.
bool hist_lae_partition_ok(pvjp_dtype dtype, int64_t m) {
    return dtype == PVJP_F32 && use_partition(PVJP_ADD, true, m, false);
}

void hist_lae_partitioned(const int32_t* inds, const float* x, int64_t n, int32_t m, float* hs, char* ws,
                          hipStream_t st) {
    const PartLayout L = part_layout(n, m);
    part_sort<PVJP_ADD>(inds, x, n, m, L, ws, st);
    double* psum = reinterpret_cast<double*>(ws + L.pacc);
    uint32_t* pmax = reinterpret_cast<uint32_t*>(ws + L.pcnt);
    const unsigned agrid = (unsigned)(ceil_div(L.items_max, (int64_t)kXcds) * kXcds);
    hipLaunchKernelGGL(hpart_lae_acc_kernel, dim3(agrid), dim3(kAccBlock), 0, st,
                       reinterpret_cast<const uint32_t*>(ws + L.rval), (const void*)(ws + L.rbin), L.nb, L.ntiles,
                       reinterpret_cast<const uint32_t*>(ws + L.D), reinterpret_cast<const int32_t*>(ws + L.istart),
                       reinterpret_cast<const int32_t*>(ws + L.itile), psum, pmax);
    hipLaunchKernelGGL(hpart_lae_merge_kernel, dim3(flat_grid(m, 256, 1)), dim3(256), 0, st, psum, pmax,
                       reinterpret_cast<const int32_t*>(ws + L.istart), m, hs);
}

template <class T, int OP, bool CACHE, bool COUNTS>
static void launch_acc(const int32_t* inds, const T* vs, int64_t n, int32_t m, const HistPlan& P, uint64_t* gacc,
                       int32_t* gz, int32_t* gcount, uint64_t* pacc, int32_t* pz, int32_t* pcnt, hipStream_t st) {
    const bool vec = aligned(inds, 16) && aligned(vs, 16);
    if (vec)
        hipLaunchKernelGGL((hist_acc_kernel<T, OP, CACHE, COUNTS, true>), dim3((unsigned)P.grid), dim3(kHistBlock),
                           P.lds, st, inds, vs, n, m, P.chunk, P.slots, gacc, gz, gcount, pacc, pz, pcnt);
    else
        hipLaunchKernelGGL((hist_acc_kernel<T, OP, CACHE, COUNTS, false>), dim3((unsigned)P.grid), dim3(kHistBlock),
                           P.lds, st, inds, vs, n, m, P.chunk, P.slots, gacc, gz, gcount, pacc, pz, pcnt);
}

template <class T, int OP>
static void run_hist(const int32_t* inds, const T* vs, int64_t n, int32_t m, T* hs, int32_t* winner, T* p,
                     int32_t* z, int32_t* count, void* ws, hipStream_t st) {
    char* w = reinterpret_cast<char*>(ws);
    uint64_t* gacc = reinterpret_cast<uint64_t*>(w);
    size_t off = align_up((size_t)m * 8, 256);
    int32_t* gz = nullptr;
    if (OP == PVJP_MUL) {
        gz = reinterpret_cast<int32_t*>(w + off);
        off += align_up((size_t)m * 4, 256);
    }
    const bool counts = count != nullptr;
    if constexpr (sizeof(T) == 4 && OP != PVJP_MUL) {
        if (use_partition(OP, true, m, counts)) {
            run_partitioned<OP>(inds, (const float*)vs, n, m, count, w, off, gacc, st);
            hipLaunchKernelGGL((hist_final_kernel<T, OP>), dim3(flat_grid(m, 256, 4)), dim3(256), 0, st, vs, gacc, gz,
                               m, hs, winner, p, z);
            return;
        }
    }
    const HistPlan P = hist_plan(OP, n, m, counts);
    uint64_t* pacc = reinterpret_cast<uint64_t*>(w + off);
    int32_t* pz = reinterpret_cast<int32_t*>(pacc + (size_t)P.grid * m);
    int32_t* pcnt = pz + (size_t)P.grid * m;
    uint64_t* macc = reinterpret_cast<uint64_t*>(pcnt + (size_t)P.grid * m);
    int32_t* mz = reinterpret_cast<int32_t*>(macc + (size_t)kMergeSlices * m);
    int32_t* mcnt = mz + (size_t)kMergeSlices * m;
    const bool f64minmax = sizeof(T) == 8 && (OP == PVJP_MIN || OP == PVJP_MAX);
    const unsigned gm = flat_grid(m, 256, 4);
    if (P.cache || f64minmax)
        hipLaunchKernelGGL(hist_init_kernel<OP>, dim3(gm), dim3(256), 0, st, gacc, gz, P.cache ? count : nullptr,
                           f64minmax ? winner : nullptr, m);
    if (P.cache) {
        if (counts)
            launch_acc<T, OP, true, true>(inds, vs, n, m, P, gacc, gz, count, nullptr, nullptr, nullptr, st);
        else
            launch_acc<T, OP, true, false>(inds, vs, n, m, P, gacc, gz, count, nullptr, nullptr, nullptr, st);
    } else {
        if (counts)
            launch_acc<T, OP, false, true>(inds, vs, n, m, P, gacc, gz, count, pacc, pz, pcnt, st);
        else
            launch_acc<T, OP, false, false>(inds, vs, n, m, P, gacc, gz, count, pacc, pz, pcnt, st);
        hipLaunchKernelGGL(hist_merge1_kernel<OP>, dim3((unsigned)ceil_div(m, 256), kMergeSlices), dim3(256), 0, st,
                           pacc, pz, counts ? pcnt : nullptr, P.grid, m, macc, mz, mcnt);
        hipLaunchKernelGGL(hist_merge2_kernel<OP>, dim3(gm), dim3(256), 0, st, macc, mz, counts ? mcnt : nullptr, m,
                           gacc, gz, count);
    }
    if (f64minmax)
        hipLaunchKernelGGL(hist_f64_winner_kernel<OP>, dim3(flat_grid(n, 256, 8)), dim3(256), 0, st, inds,
                           (const double*)vs, n, m, gacc, winner);
    hipLaunchKernelGGL((hist_final_kernel<T, OP>), dim3(gm), dim3(256), 0, st, vs, gacc, gz, m, hs, winner, p, z);
}

template <class T>
static void dispatch_hist(pvjp_op op, const int32_t* inds, const void* vs, int64_t n, int32_t m, void* hs,
                          int32_t* winner, void* p, int32_t* z, int32_t* count, void* ws, hipStream_t st) {
    const T* v = (const T*)vs;
    switch (op) {
        case PVJP_ADD: run_hist<T, PVJP_ADD>(inds, v, n, m, (T*)hs, winner, (T*)p, z, count, ws, st); break;
        case PVJP_MUL: run_hist<T, PVJP_MUL>(inds, v, n, m, (T*)hs, winner, (T*)p, z, count, ws, st); break;
        case PVJP_MIN: run_hist<T, PVJP_MIN>(inds, v, n, m, (T*)hs, winner, (T*)p, z, count, ws, st); break;
        default: run_hist<T, PVJP_MAX>(inds, v, n, m, (T*)hs, winner, (T*)p, z, count, ws, st); break;
    }
}

template <class T>
static void dispatch_vjp(pvjp_op op, const int32_t* inds, const void* vs, int64_t n, int32_t m,
                         const int32_t* winner, const void* p, const int32_t* z, const void* hsbar, void* vsbar,
                         int acc, hipStream_t st) {
    const unsigned gn = flat_grid(n, 256, 8), gm = flat_grid(m, 256, 4);
    const T* hb = (const T*)hsbar;
    T* vb = (T*)vsbar;
    const bool vec = aligned(inds, 16) && aligned(vsbar, 16);
    const unsigned gq = flat_grid(n, 256, 16);
    if (op == PVJP_ADD) {
        if (vec && m >= kGatherMinBins) {
            const int32_t L = (int32_t)std::min<int64_t>(m, kGatherLdsBytes / (int)sizeof(T));
            const size_t lds = (size_t)L * sizeof(T);
            const unsigned g = (unsigned)std::max<int64_t>(1, std::min<int64_t>(kCuCount, ceil_div(n, 4 * kGatherBlock)));
            if (acc) {
                allow_gather_lds<T, true>();
                hipLaunchKernelGGL((hist_vjp_add_lds_kernel<T, true>), dim3(g), dim3(kGatherBlock), lds, st, inds, n,
                                   m, L, hb, vb);
            } else {
                allow_gather_lds<T, false>();
                hipLaunchKernelGGL((hist_vjp_add_lds_kernel<T, false>), dim3(g), dim3(kGatherBlock), lds, st, inds, n,
                                   m, L, hb, vb);
            }
        } else if (vec && acc)
            hipLaunchKernelGGL((hist_vjp_add_vec_kernel<T, true>), dim3(gq), dim3(256), 0, st, inds, n, m, hb, vb);
        else if (vec)
            hipLaunchKernelGGL((hist_vjp_add_vec_kernel<T, false>), dim3(gq), dim3(256), 0, st, inds, n, m, hb, vb);
        else if (acc)
            hipLaunchKernelGGL((hist_vjp_add_kernel<T, true>), dim3(gn), dim3(256), 0, st, inds, n, m, hb, vb);
        else
            hipLaunchKernelGGL((hist_vjp_add_kernel<T, false>), dim3(gn), dim3(256), 0, st, inds, n, m, hb, vb);
    } else if (op == PVJP_MUL) {
        if (acc)
            hipLaunchKernelGGL((hist_vjp_mul_kernel<T, true>), dim3(gn), dim3(256), 0, st, inds, (const T*)vs, n, m,
                               (const T*)p, z, hb, vb);
        else
            hipLaunchKernelGGL((hist_vjp_mul_kernel<T, false>), dim3(gn), dim3(256), 0, st, inds, (const T*)vs, n, m,
                               (const T*)p, z, hb, vb);
    } else {
        if (acc) {
            hipLaunchKernelGGL((hist_vjp_winner_kernel<T, true>), dim3(gm), dim3(256), 0, st, winner, m, hb, vb);
        } else {
            if (aligned(vsbar, 16))
                hipLaunchKernelGGL(fill_zero_vec_kernel<T>, dim3(gq), dim3(256), 0, st, vb, n);
            else
                hipLaunchKernelGGL(fill_zero_kernel<T>, dim3(gn), dim3(256), 0, st, vb, n);
            hipLaunchKernelGGL((hist_vjp_winner_kernel<T, false>), dim3(gm), dim3(256), 0, st, winner, m, hb, vb);
        }
    }
}

// Forward mode of MIN/MAX: hs[k] is a copy of vs[winner[k]], so its
// tangent is vs_dot[winner[k]] (0 for an empty bin, whose value is the
// constant neutral element).
template <class T>
__global__ __launch_bounds__(256) void hist_jvp_winner_kernel(const int32_t* __restrict__ winner, int64_t m,
                                                              const T* __restrict__ vd, T* __restrict__ hd) {
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < m; k += (int64_t)gridDim.x * blockDim.x) {
        const int32_t w = winner[k];
        hd[k] = w >= 0 ? vd[w] : T(0);
    }
}

}  // namespace pvjp

using namespace pvjp;

static constexpr int64_t kMaxBins = (int64_t)1 << 30;

extern "C" size_t pvjp_hist_ws_bytes(pvjp_op op, pvjp_dtype dtype, int64_t n, int64_t m) {
    if (!valid_op(op) || !valid_dtype(dtype) || n < 0 || m < 1 || m > kMaxBins) return 0;
    return hist_ws(op, n, m, dtype == PVJP_F32);
}

extern "C" pvjp_status pvjp_hist_plan_info(pvjp_op op, pvjp_dtype dtype, int64_t n, int64_t m, int counts,
                                           int64_t* info) {
    clear_error();
    PVJP_REQUIRE(valid_op(op) && valid_dtype(dtype), "pvjp_hist_plan_info: unknown op or dtype");
    PVJP_REQUIRE(n >= 0 && n <= INT32_MAX && m >= 1 && m <= kMaxBins, "pvjp_hist_plan_info: n or m out of range");
    PVJP_REQUIRE(info != nullptr, "pvjp_hist_plan_info: info is NULL");
    info[1] = info[2] = info[3] = 0;
    if (use_partition(op, dtype == PVJP_F32, m, counts != 0)) {
        info[0] = PVJP_HIST_PATH_PARTITION;
        info[1] = kPartBins;
        info[2] = kPartSeg + kTile;  // runs start within kPartSeg records; a run is below kTile
        info[3] = ceil_div(m, kPartBins);
    } else {
        info[0] = hist_plan(op, n, m, counts != 0).cache ? PVJP_HIST_PATH_CACHE : PVJP_HIST_PATH_LDS;
    }
    return PVJP_OK;
}

extern "C" pvjp_status pvjp_hist(pvjp_op op, pvjp_dtype dtype, const int32_t* inds, const void* vs, int64_t n,
                                 int64_t m, void* hs, int32_t* winner, void* p, int32_t* z, int32_t* count,
                                 void* ws, size_t ws_bytes, void* stream) {
    clear_error();
    PVJP_REQUIRE(valid_op(op), "pvjp_hist: unknown op %d", (int)op);
    PVJP_REQUIRE(valid_dtype(dtype), "pvjp_hist: unknown dtype %d", (int)dtype);
    PVJP_REQUIRE(n >= 0 && n <= INT32_MAX, "pvjp_hist: n = %lld out of range [0, 2^31)", (long long)n);
    PVJP_REQUIRE(m >= 1 && m <= kMaxBins, "pvjp_hist: m = %lld out of range [1, 2^30]", (long long)m);
    PVJP_REQUIRE(hs != nullptr, "pvjp_hist: hs is NULL");
    PVJP_REQUIRE(n == 0 || (inds != nullptr && vs != nullptr), "pvjp_hist: inds and vs must be non-NULL");
    PVJP_REQUIRE(!(op == PVJP_MIN || op == PVJP_MAX) || winner != nullptr, "pvjp_hist: MIN/MAX need winner");
    PVJP_REQUIRE(op != PVJP_MUL || (p != nullptr && z != nullptr), "pvjp_hist: MUL needs p and z");
    PVJP_REQUIRE(ws != nullptr && aligned(ws, 256), "pvjp_hist: ws must be non-NULL and 256-byte aligned");
    const size_t need = pvjp_hist_ws_bytes(op, dtype, n, m);
    if (ws_bytes < need) {
        set_error("pvjp_hist: workspace has %zu bytes, needs %zu", ws_bytes, need);
        return PVJP_ENOMEM;
    }
    if (dtype == PVJP_F64)
        dispatch_hist<double>(op, inds, vs, n, (int32_t)m, hs, winner, p, z, count, ws, as_stream(stream));
    else
        dispatch_hist<float>(op, inds, vs, n, (int32_t)m, hs, winner, p, z, count, ws, as_stream(stream));
    PVJP_LAUNCHED("pvjp_hist");
    return PVJP_OK;
}

extern "C" pvjp_status pvjp_hist_vjp(pvjp_op op, pvjp_dtype dtype, const int32_t* inds, const void* vs, int64_t n,
                                     int64_t m, const int32_t* winner, const void* p, const int32_t* z,
                                     const void* hs_bar, void* vs_bar, int accumulate, void* stream) {
    clear_error();
    PVJP_REQUIRE(valid_op(op), "pvjp_hist_vjp: unknown op %d", (int)op);
    PVJP_REQUIRE(valid_dtype(dtype), "pvjp_hist_vjp: unknown dtype %d", (int)dtype);
    PVJP_REQUIRE(n >= 0 && n <= INT32_MAX, "pvjp_hist_vjp: n = %lld out of range [0, 2^31)", (long long)n);
    PVJP_REQUIRE(m >= 1 && m <= kMaxBins, "pvjp_hist_vjp: m = %lld out of range [1, 2^30]", (long long)m);
    if (n == 0) return PVJP_OK;
    PVJP_REQUIRE(hs_bar != nullptr && vs_bar != nullptr, "pvjp_hist_vjp: hs_bar and vs_bar must be non-NULL");
    PVJP_REQUIRE(op == PVJP_MIN || op == PVJP_MAX || inds != nullptr, "pvjp_hist_vjp: inds is NULL");
    PVJP_REQUIRE(!(op == PVJP_MIN || op == PVJP_MAX) || winner != nullptr, "pvjp_hist_vjp: MIN/MAX need winner");
    PVJP_REQUIRE(op != PVJP_MUL || (vs != nullptr && p != nullptr && z != nullptr),
                 "pvjp_hist_vjp: MUL needs vs, p and z");
    if (dtype == PVJP_F64)
        dispatch_vjp<double>(op, inds, vs, n, (int32_t)m, winner, p, z, hs_bar, vs_bar, accumulate,
                             as_stream(stream));
    else
        dispatch_vjp<float>(op, inds, vs, n, (int32_t)m, winner, p, z, hs_bar, vs_bar, accumulate,
                            as_stream(stream));
    PVJP_LAUNCHED("pvjp_hist_vjp");
    return PVJP_OK;
}

// Forward mode (Sec. 3): ADD is linear, so hs_dot = reduce_by_index(+) of
// vs_dot over the same bins; MIN/MAX take the winner's tangent.  MUL is not
// offered in forward mode.
extern "C" size_t pvjp_hist_jvp_ws_bytes(pvjp_op op, pvjp_dtype dtype, int64_t n, int64_t m) {
    if (op != PVJP_ADD) return 0;
    return pvjp_hist_ws_bytes(op, dtype, n, m);
}

extern "C" pvjp_status pvjp_hist_jvp(pvjp_op op, pvjp_dtype dtype, const int32_t* inds, const void* vs_dot,
                                     int64_t n, int64_t m, const int32_t* winner, void* hs_dot, void* ws,
                                     size_t ws_bytes, void* stream) {
    clear_error();
    PVJP_REQUIRE(valid_op(op), "pvjp_hist_jvp: unknown op %d", (int)op);
    if (op == PVJP_MUL) {
        set_error("pvjp_hist_jvp: reduce_by_index(*) has no forward mode here");
        return PVJP_EUNSUPPORTED;
    }
    PVJP_REQUIRE(valid_dtype(dtype), "pvjp_hist_jvp: unknown dtype %d", (int)dtype);
    PVJP_REQUIRE(m >= 1 && m <= kMaxBins, "pvjp_hist_jvp: m = %lld out of range [1, 2^30]", (long long)m);
    PVJP_REQUIRE(n >= 0 && n <= INT32_MAX, "pvjp_hist_jvp: n = %lld out of range [0, 2^31)", (long long)n);
    PVJP_REQUIRE(hs_dot != nullptr, "pvjp_hist_jvp: hs_dot is NULL");
    if (op == PVJP_ADD) {
        const pvjp_status s = pvjp_hist(op, dtype, inds, vs_dot, n, m, hs_dot, nullptr, nullptr, nullptr, nullptr, ws,
                                        ws_bytes, stream);
        if (s != PVJP_OK) {
            char inner[256];
            snprintf(inner, sizeof(inner), "%s", pvjp_last_error());
            set_error("pvjp_hist_jvp: %s", inner);
        }
        return s;
    }
    PVJP_REQUIRE(winner != nullptr, "pvjp_hist_jvp: MIN/MAX need the winners of pvjp_hist");
    PVJP_REQUIRE(n == 0 || vs_dot != nullptr, "pvjp_hist_jvp: vs_dot is NULL");
    const unsigned g = flat_grid(m, 256, 4);
    if (dtype == PVJP_F64)
        hipLaunchKernelGGL(hist_jvp_winner_kernel<double>, dim3(g), dim3(256), 0, as_stream(stream), winner, m,
                           (const double*)vs_dot, (double*)hs_dot);
    else
        hipLaunchKernelGGL(hist_jvp_winner_kernel<float>, dim3(g), dim3(256), 0, as_stream(stream), winner, m,
                           (const float*)vs_dot, (float*)hs_dot);
    PVJP_LAUNCHED("pvjp_hist_jvp");
    return PVJP_OK;
}
