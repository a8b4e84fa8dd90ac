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

constexpr int kKmCps = 32;     // centres per slice (one wave's accumulators)
constexpr int kKmChunkD = 32;  // dimensions held in registers at a time
constexpr int kKmMaxD = 1024;
constexpr size_t kKmLds = 160 * 1024;

// Waves per block so that the block's centre slices fit the LDS.
static int km_waves(int D, int cps) {
    int w = (int)(kKmLds / ((size_t)cps * D * 4));
    return w < 1 ? 1 : (w > 4 ? 4 : w);
}

// Wave w of block (bx, by) takes 64 points from bx * 64 and centre slice
// s = by * waves + w (centres [s cps, s cps + cps)), staged in LDS.  Every
// lane keeps its point's distances to the slice's centres as FP64 chains
// over d and writes its nearest (distance, centre) of the slice.
template <int CPS>
__global__ __launch_bounds__(256) void km_dist_kernel(const float* __restrict__ X, int64_t N, int D,
                                                      const float* __restrict__ C, int K, int nslice,
                                                      double* __restrict__ bd, int32_t* __restrict__ bk) {
    extern __shared__ float cs[];
    const int w = threadIdx.x / kWave, lane = threadIdx.x & (kWave - 1);
    const int nw = blockDim.x / kWave;
    const int s = blockIdx.y * nw + w;
    const int k0 = s * CPS;
    const int kc = (s < nslice) ? ((K - k0) < CPS ? (K - k0) : CPS) : 0;
    float* mine = cs + (size_t)w * CPS * D;
    for (int e = lane; e < kc * D; e += kWave) mine[e] = C[(int64_t)k0 * D + e];
    __syncthreads();
    if (kc == 0) return;  // whole waves leave together; no barrier follows
    const int64_t p = (int64_t)blockIdx.x * kWave + lane;
    const bool live = p < N;
    const float* xr = X + (live ? p : 0) * D;
    double acc[CPS];
#pragma unroll
    for (int k = 0; k < CPS; ++k) acc[k] = 0.0;
    for (int d0 = 0; d0 < D; d0 += kKmChunkD) {
        const int dn = (D - d0) < kKmChunkD ? (D - d0) : kKmChunkD;
        double xv[kKmChunkD];
#pragma unroll
        for (int j = 0; j < kKmChunkD; ++j) xv[j] = (j < dn && live) ? (double)xr[d0 + j] : 0.0;
#pragma unroll
        for (int k = 0; k < CPS; ++k) {
            if (k < kc) {
                const float* cr = mine + k * D + d0;
                double a = acc[k];
#pragma unroll
                for (int j = 0; j < kKmChunkD; ++j) {
                    if (j < dn) {
                        const double t = xv[j] - (double)cr[j];
                        a = fma(t, t, a);
                    }
                }
                acc[k] = a;
            }
        }
    }
    if (!live) return;
    double best = acc[0];
    int bkk = 0;
#pragma unroll
    for (int k = 1; k < CPS; ++k)
        if (k < kc && acc[k] < best) best = acc[k], bkk = k;
    bd[(int64_t)s * N + p] = best;
    bk[(int64_t)s * N + p] = k0 + bkk;
}

// Nearest centre over the slices in increasing order (strict <: ties keep
// the lower centre).
__global__ __launch_bounds__(256) void km_combine_kernel(const double* __restrict__ bd, const int32_t* __restrict__ bk,
                                                         int64_t N, int nslice, int32_t* __restrict__ assign,
                                                         double* __restrict__ dmin) {
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < N; p += (int64_t)gridDim.x * blockDim.x) {
        double best = bd[p];
        int32_t k = bk[p];
        for (int s = 1; s < nslice; ++s) {
            const double v = bd[(int64_t)s * N + p];
            if (v < best) best = v, k = bk[(int64_t)s * N + p];
        }
        assign[p] = k;
        dmin[p] = best;
    }
}

// f = sum_i dmin_i in a fixed order: thread t sums a contiguous run, then a
// fixed tree over the block.
__global__ __launch_bounds__(1024) void km_sum_kernel(const double* __restrict__ v, int64_t N, double* f) {
    __shared__ double sh[1024];
    const int64_t per = (N + 1023) / 1024;
    const int64_t a = (int64_t)threadIdx.x * per;
    const int64_t b = (a + per < N) ? a + per : N;
    double s = 0.0;
    for (int64_t i = a; i < b; ++i) s += v[i];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int d = 512; d >= 1; d >>= 1) {
        if ((int)threadIdx.x < d) sh[threadIdx.x] += sh[threadIdx.x + d];
        __syncthreads();
    }
    if (threadIdx.x == 0) *f = sh[0];
}

// Accumulators of the gradient: block (c, sl) takes points [c chunk, (c+1)
// chunk) and centres [sl cpb, sl cpb + cpb); thread (kk, d) adds x_i[d] of
// every point of the chunk assigned to centre sl cpb + kk, in point order,
// in FP64 (thread (kk, 0) also counts them).  No atomics: the order is fixed.
// The chunk's assignments are staged in LDS first.
constexpr int kKmChunkMax = 4096;

__global__ __launch_bounds__(1024) void km_acc_kernel(const float* __restrict__ X, int64_t N, int D, int K, int cpb,
                                                      int64_t chunk, const int32_t* __restrict__ assign,
                                                      double* __restrict__ spart, int32_t* __restrict__ npart) {
    __shared__ int32_t sa[kKmChunkMax];
    const int64_t i0 = (int64_t)blockIdx.x * chunk;
    const int64_t i1 = (i0 + chunk < N) ? i0 + chunk : N;
    const int cnt = (int)(i1 - i0);
    for (int j = threadIdx.x; j < cnt; j += blockDim.x) sa[j] = assign[i0 + j];
    __syncthreads();
    const int kk = threadIdx.x / D, d = threadIdx.x % D;
    const int k = blockIdx.y * cpb + kk;
    if (kk >= cpb || k >= K) return;  // after the only barrier
    double s = 0.0;
    int32_t c = 0;
    const float* xc = X + i0 * D + d;
    for (int j = 0; j < cnt; ++j) {
        if (sa[j] == k) {
            s += (double)xc[(int64_t)j * D];
            ++c;
        }
    }
    const int64_t o = ((int64_t)blockIdx.x * K + k);
    spart[o * D + d] = s;
    if (d == 0) npart[o] = c;
}

// C_bar = 2 f_bar (n c - S) and, with C_dot, hvp = 2 f_bar n C_dot.  One
// wave per element: lane l sums the chunk partials l, l + 64, ... in order,
// then a fixed shuffle tree combines the lanes.
__global__ __launch_bounds__(256) void km_finish_kernel(int D, int K, int nchunk, const float* __restrict__ C,
                                                        double f_bar, const double* __restrict__ spart,
                                                        const int32_t* __restrict__ npart, float* __restrict__ cbar,
                                                        const float* __restrict__ cdot, float* __restrict__ hvp,
                                                        int accumulate) {
    const int64_t KD = (int64_t)K * D;
    const int64_t e = (int64_t)blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
    if (e >= KD) return;  // whole waves leave together
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t k = e / D;
    double S = 0.0;
    int64_t n = 0;
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
    const double g = 2.0 * f_bar * ((double)n * (double)C[e] - S);
    cbar[e] = accumulate ? cbar[e] + (float)g : (float)g;
    if (hvp) {
        const double h = 2.0 * f_bar * (double)n * (double)cdot[e];
        hvp[e] = accumulate ? hvp[e] + (float)h : (float)h;
    }
}

// ------------------------------------------------------------------ host
struct KmPlan {
    int cps, nslice, waves;
    int cpb, nslices_acc;
    int64_t chunk, nchunk;
    size_t bd, bk, dmin, spart, npart, total;
};

static KmPlan km_plan(int64_t N, int D, int K) {
    KmPlan p{};
    p.cps = K < kKmCps ? K : kKmCps;
    p.nslice = (int)ceil_div(K, p.cps);
    p.waves = km_waves(D, p.cps);
    if (p.waves > p.nslice) p.waves = p.nslice;
    p.cpb = 1024 / D;
    if (p.cpb > K) p.cpb = K;
    if (p.cpb < 1) p.cpb = 1;
    p.nslices_acc = (int)ceil_div(K, p.cpb);
    int64_t want = ceil_div(1024, p.nslices_acc);  // enough blocks to fill the chip
    if (want < 1) want = 1;
    const int64_t n1 = N > 0 ? N : 1;
    p.chunk = ceil_div(n1, want);
    if (p.chunk < 64) p.chunk = 64;
    if (p.chunk > kKmChunkMax) p.chunk = kKmChunkMax;
    p.nchunk = ceil_div(n1, p.chunk);
    size_t o = 0;
    auto take = [&](size_t b) {
        const size_t at = o;
        o += align_up(b > 0 ? b : 1, 256);
        return at;
    };
    p.bd = take((size_t)p.nslice * n1 * 8);
    p.bk = take((size_t)p.nslice * n1 * 4);
    p.dmin = take((size_t)n1 * 8);
    p.spart = take((size_t)p.nchunk * K * D * 8);
    p.npart = take((size_t)p.nchunk * K * 4);
    p.total = o;
    return p;
}

template <int CPS>
static hipError_t launch_dist(const float* X, int64_t N, int D, const float* C, int K, const KmPlan& p, char* ws,
                              hipStream_t st) {
    const size_t lds = (size_t)p.waves * CPS * D * 4;
    static const bool once = [] {  // allow the dynamic LDS beyond 64 KB, once per process
        if (hipFuncSetAttribute(reinterpret_cast<const void*>(&km_dist_kernel<CPS>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)kKmLds) != hipSuccess)
            (void)hipGetLastError();
        return true;
    }();
    (void)once;
    const dim3 grid((unsigned)ceil_div(N, kWave), (unsigned)ceil_div(p.nslice, p.waves));
    hipLaunchKernelGGL((km_dist_kernel<CPS>), grid, dim3(p.waves * kWave), lds, st, X, N, D, C, K, p.nslice,
                       (double*)(ws + p.bd), (int32_t*)(ws + p.bk));
    return hipGetLastError();
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
        hipError_t e = hipSuccess;
        if (p.cps <= 4) e = launch_dist<4>(X, N, D, C, K, p, w, st);
        else if (p.cps <= 8) e = launch_dist<8>(X, N, D, C, K, p, w, st);
        else if (p.cps <= 16) e = launch_dist<16>(X, N, D, C, K, p, w, st);
        else e = launch_dist<32>(X, N, D, C, K, p, w, st);
        if (e != hipSuccess) {
            set_error("pvjp_kmeans_objective: launch failed: %s", hipGetErrorString(e));
            return PVJP_EDEVICE;
        }
        hipLaunchKernelGGL(km_combine_kernel, dim3(flat_grid(N, 256, 4)), dim3(256), 0, st,
                           (const double*)(w + p.bd), (const int32_t*)(w + p.bk), N, p.nslice, assign,
                           (double*)(w + p.dmin));
    }
    hipLaunchKernelGGL(km_sum_kernel, dim3(1), dim3(1024), 0, st, (const double*)(w + p.dmin), N, f);
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
        const dim3 grid((unsigned)p.nchunk, (unsigned)p.nslices_acc);
        hipLaunchKernelGGL(km_acc_kernel, grid, dim3((unsigned)(p.cpb * D)), 0, st, X, N, D, K, p.cpb, p.chunk, assign,
                           (double*)(w + p.spart), (int32_t*)(w + p.npart));
    }
    const int nchunk = N > 0 ? (int)p.nchunk : 0;
    hipLaunchKernelGGL(km_finish_kernel, dim3((unsigned)ceil_div((int64_t)K * D, 256 / kWave)), dim3(256), 0, st, D,
                       K, nchunk, C, f_bar, (const double*)(w + p.spart), (const int32_t*)(w + p.npart), C_bar, C_dot,
                       hvp, accumulate);
    PVJP_LAUNCHED("pvjp_kmeans_vjp");
    return PVJP_OK;
}
