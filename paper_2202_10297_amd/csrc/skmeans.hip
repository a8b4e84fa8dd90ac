// Sparse k-means (Sec. 7.5): the dense cost with the squared distance, for
// points stored in CSR (rowptr [N+1] int64, col [nnz] int32, val [nnz] FP32)
// and dense centres C [K x D] FP32.
//
// The distance of row i to centre k is one FP64 chain over the row's stored
// entries only: acc = |c_k|^2, then for each stored (j, x) of the row in CSR
// order acc = fma(x, x - 2 c_kj, acc), since |x - c|^2 = |c|^2 + sum over
// stored x of x (x - 2 c).  |c_k|^2 is summed in blocks of 1024 dimensions,
// each an fma chain in d order, the block sums added in block order.  This
// equals the plain sum of (x_d - c_d)^2 over every dimension up to FP64
// rounding, so the nearest centre agrees with it wherever the two best
// distances are further apart than that rounding.  Ties go to the lowest k.
//
// At fixed assignments the gradient is 2 f_bar (n_k c_k - S_k), S_k the sum
// of the rows assigned to k: a histogram-like accumulator of every stored
// entry into bin (a_i, j), which runs on the reduce_by_index(+) path of this
// library.  The jvp of the VJP is 2 f_bar n_k C_dot_k.
#include "common.h"
#include "prims.h"

namespace pvjp {

constexpr int kSkMaxK = 64;          // one lane per centre
constexpr int kSkNormBlock = 1024;   // dimensions per |c|^2 chain
constexpr int kSkSumBlocks = 1024;   // fixed partition of the objective's sum
constexpr int kSkU = 8;              // stored entries whose loads are in flight together

// Cw[d K + k] = c_k[d] (FP32; widened exactly to FP64 where used): a row's
// entry j reads centre values j K .. j K + K - 1, contiguous across the lanes,
// and the table is half the size of an FP64 one, so more of it stays in L2.
__global__ __launch_bounds__(256) void skm_widen_kernel(const float* __restrict__ C, int K, int64_t D,
                                                        float* __restrict__ Cw) {
    const int64_t n = (int64_t)K * D;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t d = e / K;
        const int k = (int)(e - d * K);
        Cw[e] = C[(int64_t)k * D + d];
    }
}

// cpart[k nblk + b]: the chain over dimensions [1024 b, 1024 b + 1024) of c_k.
__global__ __launch_bounds__(256) void skm_cnorm_part_kernel(const float* __restrict__ C, int K, int64_t D, int nblk,
                                                             double* __restrict__ cpart) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)K * nblk) return;
    const int k = (int)(t / nblk), b = (int)(t - (int64_t)k * nblk);
    const int64_t d0 = (int64_t)b * kSkNormBlock;
    const int64_t d1 = (d0 + kSkNormBlock < D) ? d0 + kSkNormBlock : D;
    const float* c = C + (int64_t)k * D;
    double s = 0.0;
    int64_t d = d0;
    for (; d + 32 <= d1; d += 32) {  // 32 loads in flight ahead of the chain
        float v[32];
#pragma unroll
        for (int u = 0; u < 32; ++u) v[u] = c[d + u];
#pragma unroll
        for (int u = 0; u < 32; ++u) s = fma((double)v[u], (double)v[u], s);
    }
    for (; d < d1; ++d) {
        const double v = (double)c[d];
        s = fma(v, v, s);
    }
    cpart[t] = s;
}

__global__ __launch_bounds__(64) void skm_cnorm_kernel(const double* __restrict__ cpart, int K, int nblk,
                                                       double* __restrict__ cn) {
    const int k = threadIdx.x;
    if (k >= K) return;
    double tot = 0.0;
    for (int b = 0; b < nblk; ++b) tot += cpart[(int64_t)k * nblk + b];
    cn[k] = tot;
}

// Rows are packed R = 64 / Kp to a wave (Kp: K rounded up to a power of two),
// lane group g of Kp lanes takes its own row, lane k < K of the group the
// chain of centre k over the row's stored entries (groups advance together,
// so R rows' gathers are in flight); then the nearest centre by a butterfly
// inside the group (offsets below Kp) that keeps the lower k on ties.
// Entries outside [0, nnz) or columns outside [0, D) are skipped (malformed
// input does not leave the arrays).
__global__ __launch_bounds__(256) void skm_dist_kernel(const int64_t* __restrict__ rowptr,
                                                       const int32_t* __restrict__ col, const float* __restrict__ val,
                                                       int64_t N, int64_t D, int64_t nnz, int K, int Kp,
                                                       const float* __restrict__ Cw, const double* __restrict__ cn,
                                                       int32_t* __restrict__ assign, double* __restrict__ dmin) {
    const int lane = threadIdx.x & (kWave - 1);
    const int R = kWave / Kp;
    const int grp = lane / Kp, k = lane - grp * Kp;
    const int64_t w0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const int64_t nw = (int64_t)gridDim.x * blockDim.x / kWave;
    const bool on = k < K;
    const double base = on ? cn[k] : 0.0;
    for (int64_t r0 = w0 * R; r0 < N; r0 += nw * R) {
        const int64_t i = r0 + grp;
        int64_t e0 = 0, e1 = 0;
        if (i < N) {
            e0 = rowptr[i], e1 = rowptr[i + 1];
            e0 = e0 < 0 ? 0 : (e0 > nnz ? nnz : e0);
            e1 = e1 < e0 ? e0 : (e1 > nnz ? nnz : e1);
        }
        double acc = base;
        int64_t e = e0;
        for (; e + kSkU <= e1; e += kSkU) {
            int32_t j[kSkU];
            double x[kSkU], c[kSkU];
#pragma unroll
            for (int u = 0; u < kSkU; ++u) j[u] = col[e + u], x[u] = (double)val[e + u];
#pragma unroll
            for (int u = 0; u < kSkU; ++u) {
                const bool ok = on && j[u] >= 0 && j[u] < D;
                c[u] = ok ? (double)Cw[(int64_t)j[u] * K + k] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < kSkU; ++u)
                if (j[u] >= 0 && j[u] < D) acc = fma(x[u], x[u] - 2.0 * c[u], acc);
        }
        for (; e < e1; ++e) {
            const int32_t j = col[e];
            if (j >= 0 && j < D) {
                const double x = (double)val[e];
                const double c = on ? (double)Cw[(int64_t)j * K + k] : 0.0;
                acc = fma(x, x - 2.0 * c, acc);
            }
        }
        double bd = on ? acc : (double)INFINITY;
        int bk = on ? k : kWave;
        for (int off = Kp / 2; off >= 1; off >>= 1) {
            const double od = __shfl_xor(bd, off, kWave);
            const int okk = __shfl_xor(bk, off, kWave);
            if (od < bd || (od == bd && okk < bk)) bd = od, bk = okk;
        }
        if (k == 0 && i < N) {
            assign[i] = bk;
            dmin[i] = bd;
        }
    }
}

// The objective in a fixed order: block b sums points b 256 + t + r G 256
// per thread in r order, then over the block in a fixed tree; one block adds
// the G block sums.
__global__ __launch_bounds__(256) void skm_part_kernel(const double* __restrict__ dmin, int64_t N,
                                                       double* __restrict__ part) {
    __shared__ double sh[256];
    double acc = 0.0;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < N; p += (int64_t)gridDim.x * blockDim.x)
        acc += dmin[p];
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int d = 128; d >= 1; d >>= 1) {
        if ((int)threadIdx.x < d) sh[threadIdx.x] += sh[threadIdx.x + d];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

__global__ __launch_bounds__(1024) void skm_sum_kernel(const double* __restrict__ part, int G, double* f) {
    __shared__ double sh[1024];
    sh[threadIdx.x] = (int)threadIdx.x < G ? part[threadIdx.x] : 0.0;
    __syncthreads();
    for (int d = 512; d >= 1; d >>= 1) {
        if ((int)threadIdx.x < d) sh[threadIdx.x] += sh[threadIdx.x + d];
        __syncthreads();
    }
    if (threadIdx.x == 0) *f = sh[0];
}

// bins[e] = a_i D + j for every stored entry (j, x) of row i (-1 for a
// column outside [0, D): the reduce_by_index path skips it).
__global__ __launch_bounds__(256) void skm_bins_kernel(const int64_t* __restrict__ rowptr,
                                                       const int32_t* __restrict__ col, int64_t N, int64_t D,
                                                       int64_t nnz, const int32_t* __restrict__ assign,
                                                       int32_t* __restrict__ bins) {
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t w0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const int64_t nw = (int64_t)gridDim.x * blockDim.x / kWave;
    for (int64_t i = w0; i < N; i += nw) {
        int64_t e0 = rowptr[i], e1 = rowptr[i + 1];
        e0 = e0 < 0 ? 0 : (e0 > nnz ? nnz : e0);
        e1 = e1 < e0 ? e0 : (e1 > nnz ? nnz : e1);
        const int64_t a = assign[i];
        for (int64_t e = e0 + lane; e < e1; e += kWave) {
            const int32_t j = col[e];
            bins[e] = (j >= 0 && j < D) ? (int32_t)(a * D + j) : -1;
        }
    }
}

// Entries no row covers (outside every [rowptr[i], rowptr[i+1])) must not be
// counted: they start as -1.
__global__ __launch_bounds__(256) void skm_fill_kernel(int32_t* __restrict__ bins, int64_t nnz) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nnz; e += (int64_t)gridDim.x * blockDim.x)
        bins[e] = -1;
}

// n_k: LDS counters per block, then exact integer atomics into cnt (zeroed
// by the first kernel of the call).
__global__ __launch_bounds__(256) void skm_count_kernel(const int32_t* __restrict__ assign, int64_t N, int K,
                                                        int32_t* __restrict__ cnt) {
    __shared__ int32_t h[kSkMaxK];
    if ((int)threadIdx.x < K) h[threadIdx.x] = 0;
    __syncthreads();
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t a = assign[i];
        if (a >= 0 && a < K) atomicAdd(&h[a], 1);
    }
    __syncthreads();
    if ((int)threadIdx.x < K && h[threadIdx.x]) atomicAdd(&cnt[threadIdx.x], h[threadIdx.x]);
}

__global__ __launch_bounds__(64) void skm_zero_cnt_kernel(int32_t* __restrict__ cnt, int K) {
    if ((int)threadIdx.x < K) cnt[threadIdx.x] = 0;
}

// C_bar = 2 f_bar (n_k c - S) and, with C_dot, hvp = 2 f_bar n_k C_dot.
__global__ __launch_bounds__(256) void skm_finish_kernel(int64_t D, int K, const float* __restrict__ C, double f_bar,
                                                         const float* __restrict__ S, const int32_t* __restrict__ cnt,
                                                         float* __restrict__ cbar, const float* __restrict__ cdot,
                                                         float* __restrict__ hvp, int accumulate) {
    const int64_t KD = (int64_t)K * D;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < KD; e += (int64_t)gridDim.x * blockDim.x) {
        const double n = (double)cnt[e / D];
        const double g = 2.0 * f_bar * (n * (double)C[e] - (double)S[e]);
        cbar[e] = accumulate ? cbar[e] + (float)g : (float)g;
        if (hvp) {
            const double h = 2.0 * f_bar * n * (double)cdot[e];
            hvp[e] = accumulate ? hvp[e] + (float)h : (float)h;
        }
    }
}

struct SkPlan {
    int nblk, G;
    size_t cw, cpart, cn, dmin, part, bins, S, cnt, hist, hist_bytes, total;
};

static SkPlan skm_plan(int64_t N, int64_t D, int K, int64_t nnz) {
    SkPlan p{};
    p.nblk = (int)ceil_div(D, kSkNormBlock);
    const int64_t g = ceil_div(N > 0 ? N : 1, 256);
    p.G = (int)(g < kSkSumBlocks ? g : kSkSumBlocks);
    size_t o = 0;
    auto take = [&](size_t b) {
        const size_t at = o;
        o += align_up(b > 0 ? b : 1, 256);
        return at;
    };
    p.cw = take((size_t)K * D * 4);
    p.cpart = take((size_t)K * p.nblk * 8);
    p.cn = take((size_t)K * 8);
    p.dmin = take((size_t)(N > 0 ? N : 1) * 8);
    p.part = take((size_t)kSkSumBlocks * 8);
    p.bins = take((size_t)(nnz > 0 ? nnz : 1) * 4);
    p.S = take((size_t)K * D * 4);
    p.cnt = take((size_t)kSkMaxK * 4);
    p.hist_bytes = align_up(pvjp_hist_ws_bytes(PVJP_ADD, PVJP_F32, nnz > 0 ? nnz : 1, (int64_t)K * D), 256);
    p.hist = take(p.hist_bytes);
    p.total = o;
    return p;
}

static pvjp_status skm_check(const char* name, const int64_t* rowptr, const int32_t* col, const float* val,
                             int64_t N, int64_t D, int64_t nnz, const float* C, int K, void* ws, size_t ws_bytes) {
    PVJP_REQUIRE(N >= 0 && N < INT32_MAX, "%s: N = %lld out of range", name, (long long)N);
    PVJP_REQUIRE(D >= 1 && nnz >= 0 && nnz < INT32_MAX, "%s: D = %lld, nnz = %lld out of range", name, (long long)D,
                 (long long)nnz);
    PVJP_REQUIRE(K >= 1 && K <= kSkMaxK, "%s: K = %d out of range [1, %d]", name, K, kSkMaxK);
    PVJP_REQUIRE((int64_t)K * D < INT32_MAX && (int64_t)K * D <= ((int64_t)1 << 30),
                 "%s: K D = %lld bins exceed the accumulator's range", name, (long long)K * D);
    PVJP_REQUIRE(C != nullptr && rowptr != nullptr, "%s: C and rowptr must be non-NULL", name);
    PVJP_REQUIRE(nnz == 0 || (col != nullptr && val != nullptr), "%s: col and val must be non-NULL", name);
    PVJP_REQUIRE(ws != nullptr && aligned(ws, 256), "%s: ws must be non-NULL and 256-byte aligned", name);
    const size_t need = skm_plan(N, D, K, nnz).total;
    if (ws_bytes < need) {
        set_error("%s: workspace has %zu bytes, needs %zu", name, ws_bytes, need);
        return PVJP_ENOMEM;
    }
    return PVJP_OK;
}

}  // namespace pvjp

using namespace pvjp;

extern "C" size_t pvjp_sparse_kmeans_ws_bytes(int64_t N, int64_t D, int K, int64_t nnz) {
    if (N < 0 || D < 1 || K < 1 || K > kSkMaxK || nnz < 0) return 0;
    return skm_plan(N, D, K, nnz).total;
}

extern "C" pvjp_status pvjp_sparse_kmeans_objective(const int64_t* rowptr, const int32_t* col, const float* val,
                                                    int64_t N, int64_t D, int64_t nnz, const float* C, int K,
                                                    int32_t* assign, double* f, void* ws, size_t ws_bytes,
                                                    void* stream) {
    clear_error();
    if (pvjp_status e = skm_check("pvjp_sparse_kmeans_objective", rowptr, col, val, N, D, nnz, C, K, ws, ws_bytes))
        return e;
    PVJP_REQUIRE(f != nullptr && (N == 0 || assign != nullptr),
                 "pvjp_sparse_kmeans_objective: assign and f are required");
    const SkPlan p = skm_plan(N, D, K, nnz);
    char* w = reinterpret_cast<char*>(ws);
    hipStream_t st = as_stream(stream);
    if (N > 0) {
        const int64_t KD = (int64_t)K * D;
        hipLaunchKernelGGL(skm_widen_kernel, dim3(flat_grid(KD, 256, 4)), dim3(256), 0, st, C, K, D,
                           (float*)(w + p.cw));
        hipLaunchKernelGGL(skm_cnorm_part_kernel, dim3((unsigned)ceil_div((int64_t)K * p.nblk, 256)), dim3(256), 0, st,
                           C, K, D, p.nblk, (double*)(w + p.cpart));
        hipLaunchKernelGGL(skm_cnorm_kernel, dim3(1), dim3(64), 0, st, (const double*)(w + p.cpart), K, p.nblk,
                           (double*)(w + p.cn));
        int Kp = 1;
        while (Kp < K) Kp <<= 1;
        const int64_t rw = ceil_div(N, (int64_t)(kWave / Kp));  // waves that cover every row once
        const int64_t waves = rw < 65536 ? rw : 65536;
        hipLaunchKernelGGL(skm_dist_kernel, dim3((unsigned)ceil_div(waves, 4)), dim3(256), 0, st, rowptr, col, val, N,
                           D, nnz, K, Kp, (const float*)(w + p.cw), (const double*)(w + p.cn), assign,
                           (double*)(w + p.dmin));
        hipLaunchKernelGGL(skm_part_kernel, dim3((unsigned)p.G), dim3(256), 0, st, (const double*)(w + p.dmin), N,
                           (double*)(w + p.part));
    }
    hipLaunchKernelGGL(skm_sum_kernel, dim3(1), dim3(1024), 0, st, (const double*)(w + p.part), N > 0 ? p.G : 0, f);
    PVJP_LAUNCHED("pvjp_sparse_kmeans_objective");
    return PVJP_OK;
}

extern "C" pvjp_status pvjp_sparse_kmeans_vjp(const int64_t* rowptr, const int32_t* col, const float* val, int64_t N,
                                              int64_t D, int64_t nnz, const float* C, int K, const int32_t* assign,
                                              double f_bar, float* C_bar, const float* C_dot, float* hvp,
                                              int accumulate, void* ws, size_t ws_bytes, void* stream) {
    clear_error();
    if (pvjp_status e = skm_check("pvjp_sparse_kmeans_vjp", rowptr, col, val, N, D, nnz, C, K, ws, ws_bytes))
        return e;
    PVJP_REQUIRE(C_bar != nullptr, "pvjp_sparse_kmeans_vjp: C_bar is NULL");
    PVJP_REQUIRE(N == 0 || assign != nullptr, "pvjp_sparse_kmeans_vjp: assign (from the objective) is NULL");
    PVJP_REQUIRE((C_dot == nullptr) == (hvp == nullptr), "pvjp_sparse_kmeans_vjp: C_dot and hvp go together");
    const SkPlan p = skm_plan(N, D, K, nnz);
    char* w = reinterpret_cast<char*>(ws);
    hipStream_t st = as_stream(stream);
    const int64_t KD = (int64_t)K * D;
    int32_t* cnt = (int32_t*)(w + p.cnt);
    float* S = (float*)(w + p.S);
    int32_t* bins = (int32_t*)(w + p.bins);
    hipLaunchKernelGGL(skm_zero_cnt_kernel, dim3(1), dim3(64), 0, st, cnt, K);
    if (N > 0) hipLaunchKernelGGL(skm_count_kernel, dim3(flat_grid(N, 256, 8)), dim3(256), 0, st, assign, N, K, cnt);
    if (nnz > 0) {
        hipLaunchKernelGGL(skm_fill_kernel, dim3(flat_grid(nnz, 256, 4)), dim3(256), 0, st, bins, nnz);
        const int64_t waves = N < 65536 ? N : 65536;
        if (N > 0)
            hipLaunchKernelGGL(skm_bins_kernel, dim3((unsigned)ceil_div(waves, 4)), dim3(256), 0, st, rowptr, col, N, D,
                               nnz, assign, bins);
    }
    if (pvjp_status e = pvjp_hist(PVJP_ADD, PVJP_F32, bins, val, nnz, KD, S, nullptr, nullptr, nullptr, nullptr,
                                  w + p.hist, p.hist_bytes, st))
        return e;
    hipLaunchKernelGGL(skm_finish_kernel, dim3(flat_grid(KD, 256, 4)), dim3(256), 0, st, D, K, C, f_bar,
                       (const float*)S, (const int32_t*)cnt, C_bar, C_dot, hvp, accumulate);
    PVJP_LAUNCHED("pvjp_sparse_kmeans_vjp");
    return PVJP_OK;
}
