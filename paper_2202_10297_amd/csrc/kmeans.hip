// Dense k-means (Sec. 7.4), the workload of the forward-over-reverse example:
//   f(C) = sum_i min_k |x_i - c_k|^2   (squared distance; X [N x D] and
//   C [K x D] row-major FP32).
// The objective's search keeps each point's nearest centre (the primal's
// auxiliary output).  With the assignments fixed the gradient is an
// accumulator of the points into their centres (Sec. 5.4 / 6):
//   C_bar_k = 2 f_bar (n_k c_k - S_k),  S_k = sum_{a_i = k} x_i,
// and the jvp of the vjp in direction C_dot (the Hessian-vector product,
// the Hessian being diagonal) is 2 f_bar n_k C_dot_k; C_dot = 1 gives the
// diagonal.  Both come from one accumulation pass, and the search is not
// repeated.
//
// Distances are formed in FP64 by the chain acc = fma(x_d - c_d, x_d - c_d,
// acc), d = 0..D-1, so every implementation of that chain (the oracle's
// included) decides the same nearest centre, ties going to the lowest k.
#include "common.h"
#include "prims.h"

namespace pvjp {

constexpr int kKmChunkD = 32;        // dimensions of X staged (and held in registers) at a time
constexpr int kKmMaxD = 1024;
constexpr size_t kKmSliceBytes = 64 * 1024;  // a slice's FP64 centres: 32 centres up to D = 256
constexpr int kKmPts = 256;          // points per distance block, one per lane
constexpr int kKmSumBlocks = 1024;   // fixed partition of the objective's sum
constexpr int kKmSmallK = 16;        // register accumulators in the gradient up to this K
constexpr int kKmChunkMax = 4096;

// Centres per slice: as many as kKmSliceBytes of FP64 holds (>= 4), at most 32.
static int km_cps(int D, int K) {
    int c = (int)(kKmSliceBytes / ((size_t)D * 8));
    c = c >= 32 ? 32 : (c >= 16 ? 16 : (c >= 8 ? 8 : 4));
    return K < c ? K : c;
}

// The centres in FP64, once per call, laid out per slice as [d][CPS]: Cw[(s D
// + d) CPS + k'] = c_{s cps + k'}[d], zero beyond the slice's centres.  A
// chunk of dimensions of one slice is then one contiguous block that the
// distance kernel reads at wave-uniform addresses, and the chains subtract
// FP64 values without a conversion.
__global__ __launch_bounds__(256) void km_widen_kernel(const float* __restrict__ C, int K, int D, int cps, int CPS,
                                                       int64_t n, double* __restrict__ Cw) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        const int kp = (int)(e % CPS);
        const int64_t sd = e / CPS;
        const int d = (int)(sd % D);
        const int64_t k = (sd / D) * cps + kp;
        Cw[e] = (kp < cps && k < K) ? (double)C[k * D + d] : 0.0;
    }
}

// Block (bx, s) takes points [bx 256, bx 256 + 256), one per lane, and centre
// slice s (centres [s cps, s cps + cps)).  X comes in 32-dimension chunks,
// copied into LDS with consecutive threads on consecutive addresses.  For each
// dimension d in order, a lane reads x[d] once and extends the CPS chains
// acc_k = fma(x[d] - c_k[d], x[d] - c_k[d], acc_k) (independent of each
// other, each in d order); the c_k[d] are wave-uniform reads of the widened
// centres (scalar loads, no LDS).  Every lane writes its nearest (distance,
// centre) of the slice.
template <int CPS>
__global__ __launch_bounds__(256) void km_dist_kernel(const float* __restrict__ X, int64_t N, int D,
                                                      const double* __restrict__ Cw, int K, int cps,
                                                      double* __restrict__ bd, int32_t* __restrict__ bk) {
    constexpr int kStride = kKmChunkD + 1;  // odd row stride: lanes hit distinct banks
    __shared__ float xs[kKmPts * kStride];
    const int s = blockIdx.y;
    const int k0 = s * cps;
    const int kc = (K - k0) < cps ? (K - k0) : cps;
    const int64_t p0 = (int64_t)blockIdx.x * kKmPts;
    const int np = (N - p0) < kKmPts ? (int)(N - p0) : kKmPts;
    const int t = threadIdx.x;
    const bool live = t < np;
    double acc[CPS];
#pragma unroll
    for (int k = 0; k < CPS; ++k) acc[k] = 0.0;
    for (int d0 = 0; d0 < D; d0 += kKmChunkD) {
        const int dn = (D - d0) < kKmChunkD ? (D - d0) : kKmChunkD;
        if (d0 > 0) __syncthreads();  // the previous chunk has been read
        const float* xb = X + p0 * D + d0;
        if (dn == kKmChunkD && np == kKmPts) {
            // thread t copies column t % 32 of rows t / 32 + 8 u, u < 32, kU
            // loads in flight (fewer where the chains need the registers);
            // each 32-lane group reads one contiguous 128-byte row piece
            constexpr int kU = CPS >= 16 ? 8 : kKmChunkD;
            const int j = t & (kKmChunkD - 1), r0 = t / kKmChunkD;
            const uint32_t lo = (uint32_t)(r0 * D + j);  // the lane's offset from a uniform row base
#pragma unroll
            for (int u0 = 0; u0 < kKmChunkD; u0 += kU) {
                float v[kU];
#pragma unroll
                for (int u = 0; u < kU; ++u) v[u] = (xb + (int64_t)(8 * (u0 + u)) * D)[lo];
#pragma unroll
                for (int u = 0; u < kU; ++u) xs[(r0 + 8 * (u0 + u)) * kStride + j] = v[u];
            }
        } else {
            for (int e = t; e < np * dn; e += kKmPts) {
                const int pt = e / dn, j = e - pt * dn;
                xs[pt * kStride + j] = xb[(int64_t)pt * D + j];
            }
        }
        __syncthreads();
        const double* cb = Cw + ((int64_t)s * D + d0) * CPS;
        const float* xr = xs + (live ? t : 0) * kStride;
#pragma unroll 2
        for (int j = 0; j < dn; ++j) {
            const double xj = (double)xr[j];
#pragma unroll
            for (int k = 0; k < CPS; ++k) {
                const double u = xj - cb[j * CPS + k];
                acc[k] = fma(u, u, acc[k]);
            }
        }
    }
    if (!live) return;  // after the last barrier
    double best = acc[0];
    int bkk = 0;
#pragma unroll
    for (int k = 1; k < CPS; ++k)
        if (k < kc && acc[k] < best) best = acc[k], bkk = k;
    bd[(int64_t)s * N + p0 + t] = best;
    bk[(int64_t)s * N + p0 + t] = k0 + bkk;
}

// Nearest centre over the slices in increasing order (strict <: ties keep
// the lower centre), and the block's share of the objective: block b takes
// points b 256 + t + r G 256 (G = gridDim.x, fixed by N), sums them per
// thread in r order and then over the block in a fixed tree.
__global__ __launch_bounds__(256) void km_combine_kernel(const double* __restrict__ bd, const int32_t* __restrict__ bk,
                                                         int64_t N, int nslice, int32_t* __restrict__ assign,
                                                         double* __restrict__ part) {
    __shared__ double sh[256];
    double acc = 0.0;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < N; p += (int64_t)gridDim.x * blockDim.x) {
        double best = bd[p];
        int32_t k = bk[p];
        for (int s = 1; s < nslice; ++s) {
            const double v = bd[(int64_t)s * N + p];
            if (v < best) best = v, k = bk[(int64_t)s * N + p];
        }
        assign[p] = k;
        acc += best;
    }
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int d = 128; d >= 1; d >>= 1) {
        if ((int)threadIdx.x < d) sh[threadIdx.x] += sh[threadIdx.x + d];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

// f = the sum of the G block shares in a fixed tree (G <= 1024).
__global__ __launch_bounds__(1024) void km_sum_kernel(const double* __restrict__ part, int G, double* f) {
    __shared__ double sh[1024];
    sh[threadIdx.x] = (int)threadIdx.x < G ? part[threadIdx.x] : 0.0;
    __syncthreads();
    for (int d = 512; d >= 1; d >>= 1) {
        if ((int)threadIdx.x < d) sh[threadIdx.x] += sh[threadIdx.x + d];
        __syncthreads();
    }
    if (threadIdx.x == 0) *f = sh[0];
}

// Accumulators of the gradient for K <= kKmSmallK and D <= 256: block c takes
// points [c chunk, (c+1) chunk); thread t is column d = t % D of point lane
// g = t / D (G = 256 / D lanes), adds x_j[d] of points j = g, g + G, ... into
// KM FP64 registers, the one of its centre selected (the others add 0, which
// leaves them unchanged), then the G lanes are summed per column in g order.
// All of X's reads are coalesced rows.  No atomics: the order is fixed.
template <int KM>
__global__ __launch_bounds__(256) void km_acc_small_kernel(const float* __restrict__ X, int64_t N, int D, int K,
                                                           int64_t chunk, const int32_t* __restrict__ assign,
                                                           double* __restrict__ spart, int32_t* __restrict__ npart) {
    __shared__ double rs[256];
    __shared__ int32_t rc[256];
    const int G = 256 / D;
    const int t = threadIdx.x, g = t / D, d = t - g * D;
    const bool act = g < G;
    const int64_t i0 = (int64_t)blockIdx.x * chunk;
    const int64_t i1 = (i0 + chunk < N) ? i0 + chunk : N;
    double acc[KM];
    int32_t cnt[KM];
#pragma unroll
    for (int k = 0; k < KM; ++k) acc[k] = 0.0, cnt[k] = 0;
    if (act) {
        constexpr int U = 8;  // points whose loads are in flight together
        int64_t j = i0 + g;
        for (; j + (U - 1) * (int64_t)G < i1; j += U * (int64_t)G) {
            int32_t a[U];
            float x[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                a[u] = assign[j + u * (int64_t)G];
                x[u] = X[(j + u * (int64_t)G) * D + d];
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
#pragma unroll
                for (int k = 0; k < KM; ++k) {
                    acc[k] += (a[u] == k) ? (double)x[u] : 0.0;
                    cnt[k] += (a[u] == k) ? 1 : 0;
                }
            }
        }
        for (; j < i1; j += G) {
            const int32_t a = assign[j];
            const double x = (double)X[j * D + d];
#pragma unroll
            for (int k = 0; k < KM; ++k) {
                acc[k] += (a == k) ? x : 0.0;
                cnt[k] += (a == k) ? 1 : 0;
            }
        }
    }
#pragma unroll
    for (int k = 0; k < KM; ++k) {
        if (k < K) {  // uniform: every thread meets the same barriers
            rs[t] = acc[k];
            rc[t] = cnt[k];
            __syncthreads();
            if (t < D) {
                double sum = 0.0;
                int32_t c = 0;
                for (int q = 0; q < G; ++q) sum += rs[q * D + t], c += rc[q * D + t];
                const int64_t o = (int64_t)blockIdx.x * K + k;
                spart[o * D + t] = sum;
                if (t == 0) npart[o] = c;
            }
            __syncthreads();
        }
    }
}

// Accumulators of the gradient for larger K: block (c, sl) takes points
// [c chunk, (c+1) chunk) and centres [sl cpb, sl cpb + cpb).  The block first
// lists, in point order, the chunk's points assigned to its centres (a stable
// compaction by ballots and a running offset); then thread (kk, d) adds x_i[d]
// of the listed points of centre sl cpb + kk in that order, in FP64 (thread
// (kk, 0) also counts them).  No atomics: the order is fixed.
__global__ __launch_bounds__(1024) void km_acc_kernel(const float* __restrict__ X, int64_t N, int D, int K, int cpb,
                                                      int64_t chunk, const int32_t* __restrict__ assign,
                                                      double* __restrict__ spart, int32_t* __restrict__ npart) {
    __shared__ int32_t lj[kKmChunkMax];  // listed point offsets within the chunk
    __shared__ int32_t lk[kKmChunkMax];  // and their centres
    __shared__ int32_t wtot[1024 / kWave];
    const int64_t i0 = (int64_t)blockIdx.x * chunk;
    const int64_t i1 = (i0 + chunk < N) ? i0 + chunk : N;
    const int cnt = (int)(i1 - i0);
    const int klo = blockIdx.y * cpb;
    const int khi = (klo + cpb < K) ? klo + cpb : K;
    const int w = threadIdx.x / kWave, lane = threadIdx.x & (kWave - 1);
    const int nw = (int)((blockDim.x + kWave - 1) / kWave);
    int m = 0;  // listed so far (the same in every thread)
    for (int j0 = 0; j0 < cnt; j0 += blockDim.x) {
        const int j = j0 + (int)threadIdx.x;
        const int32_t a = j < cnt ? assign[i0 + j] : -1;
        const bool f = a >= klo && a < khi;
        const uint64_t bal = __ballot(f);
        const int rank = __popcll(bal & ((1ull << lane) - 1ull));
        if (lane == 0) wtot[w] = __popcll(bal);
        __syncthreads();
        int base = m, tot = 0;
        for (int q = 0; q < nw; ++q) {
            if (q < w) base += wtot[q];
            tot += wtot[q];
        }
        if (f) lj[base + rank] = j, lk[base + rank] = a;
        m += tot;
        __syncthreads();  // wtot is rewritten next round; the list is read below
    }
    const int kk = threadIdx.x / D, d = threadIdx.x % D;
    const int k = klo + kk;
    if (kk >= cpb || k >= K) return;  // after the last barrier
    double s = 0.0;
    int32_t c = 0;
    const float* xc = X + i0 * D + d;
    for (int q = 0; q < m; ++q) {
        if (lk[q] == k) {
            s += (double)xc[(int64_t)lj[q] * D];
            ++c;
        }
    }
    const int64_t o = ((int64_t)blockIdx.x * K + k);
    spart[o * D + d] = s;
    if (d == 0) npart[o] = c;
}

// C_bar = 2 f_bar (n c - S) and, with C_dot, hvp = 2 f_bar n C_dot, from the
// chunk partials summed in chunk order.  WAVE: one wave per element, lane l
// takes the partials l, l + 64, ... and a fixed shuffle tree combines the
// lanes (many chunks); otherwise one thread per element (few chunks).
template <bool WAVE>
__global__ __launch_bounds__(256) void km_finish_kernel(int D, int K, int nchunk, const float* __restrict__ C,
                                                        double f_bar, const double* __restrict__ spart,
                                                        const int32_t* __restrict__ npart, float* __restrict__ cbar,
                                                        const float* __restrict__ cdot, float* __restrict__ hvp,
                                                        int accumulate) {
    const int64_t KD = (int64_t)K * D;
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t e = WAVE ? (int64_t)blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave
                           : (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= KD) return;  // whole waves leave together when WAVE
    const int64_t k = e / D;
    double S = 0.0;
    int64_t n = 0;
    if (WAVE) {
        for (int c = lane; c < nchunk; c += kWave) {
            S += spart[(int64_t)c * KD + e];
            n += npart[(int64_t)c * K + k];
        }
#pragma unroll
        for (int o = kWave / 2; o >= 1; o >>= 1) {
            S += __shfl_down(S, o, kWave);
            n += __shfl_down(n, o, kWave);
        }
        if (lane != 0) return;
    } else {
        for (int c = 0; c < nchunk; ++c) {
            S += spart[(int64_t)c * KD + e];
            n += npart[(int64_t)c * K + k];
        }
    }
    const double g = 2.0 * f_bar * ((double)n * (double)C[e] - S);
    cbar[e] = accumulate ? cbar[e] + (float)g : (float)g;
    if (hvp) {
        const double h = 2.0 * f_bar * (double)n * (double)cdot[e];
        hvp[e] = accumulate ? hvp[e] + (float)h : (float)h;
    }
}

// ------------------------------------------------------------------ host
struct KmPlan {
    int cps, cpsT, nslice, sum_blocks;  // centres per slice, and the kernel's width for them
    bool small;  // register accumulators in the gradient
    int cpb, nslices_acc;
    int64_t chunk, nchunk;
    size_t cd, bd, bk, part, spart, npart, total;
};

static KmPlan km_plan(int64_t N, int D, int K) {
    KmPlan p{};
    p.cps = km_cps(D, K);
    p.cpsT = p.cps <= 4 ? 4 : (p.cps <= 8 ? 8 : (p.cps <= 16 ? 16 : 32));
    p.nslice = (int)ceil_div(K, p.cps);
    {
        const int64_t b = ceil_div(N > 0 ? N : 1, 256);
        p.sum_blocks = (int)(b < kKmSumBlocks ? b : kKmSumBlocks);
    }
    const int64_t n1 = N > 0 ? N : 1;
    p.small = K <= kKmSmallK && D <= 256;
    if (p.small) {
        p.cpb = K;
        p.nslices_acc = 1;
        p.chunk = ceil_div(n1, 1024);  // about 1024 blocks
        if (p.chunk < 64) p.chunk = 64;
    } else {
        p.cpb = 1024 / D;
        if (p.cpb > K) p.cpb = K;
        if (p.cpb < 1) p.cpb = 1;
        p.nslices_acc = (int)ceil_div(K, p.cpb);
        int64_t want = ceil_div(1024, p.nslices_acc);  // enough blocks to fill the chip
        if (want < 1) want = 1;
        p.chunk = ceil_div(n1, want);
        if (p.chunk < 64) p.chunk = 64;
        if (p.chunk > kKmChunkMax) p.chunk = kKmChunkMax;
    }
    p.nchunk = ceil_div(n1, p.chunk);
    size_t o = 0;
    auto take = [&](size_t b) {
        const size_t at = o;
        o += align_up(b > 0 ? b : 1, 256);
        return at;
    };
    p.cd = take((size_t)p.nslice * D * p.cpsT * 8);
    p.bd = take((size_t)p.nslice * n1 * 8);
    p.bk = take((size_t)p.nslice * n1 * 4);
    p.part = take((size_t)kKmSumBlocks * 8);
    p.spart = take((size_t)p.nchunk * K * D * 8);
    p.npart = take((size_t)p.nchunk * K * 4);
    p.total = o;
    return p;
}

template <int CPS>
static void launch_dist(const float* X, int64_t N, int D, int K, const KmPlan& p, char* ws, hipStream_t st) {
    const dim3 grid((unsigned)ceil_div(N, kKmPts), (unsigned)p.nslice);
    hipLaunchKernelGGL((km_dist_kernel<CPS>), grid, dim3(kKmPts), 0, st, X, N, D, (const double*)(ws + p.cd), K,
                       p.cps, (double*)(ws + p.bd), (int32_t*)(ws + p.bk));
}

template <int KM>
static void launch_acc_small(const float* X, int64_t N, int D, int K, const int32_t* assign, const KmPlan& p, char* ws,
                             hipStream_t st) {
    hipLaunchKernelGGL((km_acc_small_kernel<KM>), dim3((unsigned)p.nchunk), dim3(256), 0, st, X, N, D, K, p.chunk,
                       assign, (double*)(ws + p.spart), (int32_t*)(ws + p.npart));
}

static pvjp_status km_check(const char* name, const float* X, int64_t N, int D, const float* C, int K, void* ws,
                            size_t ws_bytes) {
    PVJP_REQUIRE(N >= 0 && N <= INT32_MAX, "%s: N = %lld out of range [0, 2^31)", name, (long long)N);
    PVJP_REQUIRE(D >= 1 && D <= kKmMaxD, "%s: D = %d out of range [1, %d]", name, D, kKmMaxD);
    PVJP_REQUIRE(K >= 1 && K <= (1 << 20), "%s: K = %d out of range [1, 2^20]", name, K);
    PVJP_REQUIRE(C != nullptr && (N == 0 || X != nullptr), "%s: X and C must be non-NULL", name);
    PVJP_REQUIRE(ws != nullptr && aligned(ws, 256), "%s: ws must be non-NULL and 256-byte aligned", name);
    const size_t need = km_plan(N, D, K).total;
    if (ws_bytes < need) {
        set_error("%s: workspace has %zu bytes, needs %zu", name, ws_bytes, need);
        return PVJP_ENOMEM;
    }
    return PVJP_OK;
}

}  // namespace pvjp

using namespace pvjp;

extern "C" size_t pvjp_kmeans_ws_bytes(int64_t N, int D, int K) {
    if (N < 0 || D < 1 || D > kKmMaxD || K < 1) return 0;
    return km_plan(N, D, K).total;
}

extern "C" pvjp_status pvjp_kmeans_objective(const float* X, int64_t N, int D, const float* C, int K, int32_t* assign,
                                             double* f, void* ws, size_t ws_bytes, void* stream) {
    clear_error();
    if (pvjp_status e = km_check("pvjp_kmeans_objective", X, N, D, C, K, ws, ws_bytes)) return e;
    PVJP_REQUIRE(f != nullptr && (N == 0 || assign != nullptr), "pvjp_kmeans_objective: assign and f are required");
    const KmPlan p = km_plan(N, D, K);
    char* w = reinterpret_cast<char*>(ws);
    hipStream_t st = as_stream(stream);
    if (N > 0) {
        const int64_t nw = (int64_t)p.nslice * D * p.cpsT;
        hipLaunchKernelGGL(km_widen_kernel, dim3(flat_grid(nw, 256, 4)), dim3(256), 0, st, C, K, D, p.cps, p.cpsT, nw,
                           (double*)(w + p.cd));
        if (p.cpsT == 4) launch_dist<4>(X, N, D, K, p, w, st);
        else if (p.cpsT == 8) launch_dist<8>(X, N, D, K, p, w, st);
        else if (p.cpsT == 16) launch_dist<16>(X, N, D, K, p, w, st);
        else launch_dist<32>(X, N, D, K, p, w, st);
        hipLaunchKernelGGL(km_combine_kernel, dim3((unsigned)p.sum_blocks), dim3(256), 0, st,
                           (const double*)(w + p.bd), (const int32_t*)(w + p.bk), N, p.nslice, assign,
                           (double*)(w + p.part));
    }
    hipLaunchKernelGGL(km_sum_kernel, dim3(1), dim3(1024), 0, st, (const double*)(w + p.part),
                       N > 0 ? p.sum_blocks : 0, f);
    PVJP_LAUNCHED("pvjp_kmeans_objective");
    return PVJP_OK;
}

extern "C" pvjp_status pvjp_kmeans_vjp(const float* X, int64_t N, int D, const float* C, int K, const int32_t* assign,
                                       double f_bar, float* C_bar, const float* C_dot, float* hvp, int accumulate,
                                       void* ws, size_t ws_bytes, void* stream) {
    clear_error();
    if (pvjp_status e = km_check("pvjp_kmeans_vjp", X, N, D, C, K, ws, ws_bytes)) return e;
    PVJP_REQUIRE(C_bar != nullptr, "pvjp_kmeans_vjp: C_bar is NULL");
    PVJP_REQUIRE(N == 0 || assign != nullptr, "pvjp_kmeans_vjp: assign (from pvjp_kmeans_objective) is NULL");
    PVJP_REQUIRE((C_dot == nullptr) == (hvp == nullptr), "pvjp_kmeans_vjp: C_dot and hvp go together");
    const KmPlan p = km_plan(N, D, K);
    char* w = reinterpret_cast<char*>(ws);
    hipStream_t st = as_stream(stream);
    if (N > 0) {
        if (p.small) {
            if (K <= 4) launch_acc_small<4>(X, N, D, K, assign, p, w, st);
            else if (K <= 8) launch_acc_small<8>(X, N, D, K, assign, p, w, st);
            else launch_acc_small<16>(X, N, D, K, assign, p, w, st);
        } else {
            const dim3 grid((unsigned)p.nchunk, (unsigned)p.nslices_acc);
            hipLaunchKernelGGL(km_acc_kernel, grid, dim3((unsigned)(p.cpb * D)), 0, st, X, N, D, K, p.cpb, p.chunk,
                               assign, (double*)(w + p.spart), (int32_t*)(w + p.npart));
        }
    }
    const int nchunk = N > 0 ? (int)p.nchunk : 0;
    const int64_t KD = (int64_t)K * D;
    if (nchunk > kWave)
        hipLaunchKernelGGL((km_finish_kernel<true>), dim3((unsigned)ceil_div(KD, 256 / kWave)), dim3(256), 0, st, D, K,
                           nchunk, C, f_bar, (const double*)(w + p.spart), (const int32_t*)(w + p.npart), C_bar, C_dot,
                           hvp, accumulate);
    else
        hipLaunchKernelGGL((km_finish_kernel<false>), dim3((unsigned)ceil_div(KD, 256)), dim3(256), 0, st, D, K,
                           nchunk, C, f_bar, (const double*)(w + p.spart), (const int32_t*)(w + p.npart), C_bar, C_dot,
                           hvp, accumulate);
    PVJP_LAUNCHED("pvjp_kmeans_vjp");
    return PVJP_OK;
}
