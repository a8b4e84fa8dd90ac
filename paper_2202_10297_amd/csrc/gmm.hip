// Gaussian-mixture log-likelihood and its full reverse-mode gradient (the
// workload of Sec. 7.6; accumulators turned into reductions and contractions
// as in Sec. 6.1).
//
// Objective (precision-Cholesky parametrisation; the paper leaves the
// definition to its benchmark suite, this is the textbook mixture):
//   Q_k = diag(exp q_k) + L_k (L_k strictly lower, row-major packed in l_k),
//   z_ik = Q_k (x_i - mu_k) = Q_k x_i - c_k with c_k = Q_k mu_k,
//   s_ik = alpha_k + sum_d q_kd - |z_ik|^2 / 2,
//   loglik = sum_i LSE_k s_ik - N LSE(alpha) - N D/2 log(2 pi).
//
// Forward sweep (gmm_fwd): per 32-point tile a wave forms Z^T = Q_k X^T with
// FP32 MFMA 32x32x2 (only the lower-triangular 32x32 blocks of Q_k), squares
// and sums z in FP64, and keeps an online FP64 log-sum-exp over k.  LSE_i is
// the per-point checkpoint of the reverse sweep.
//
// Return sweep: with w_ik = ell_bar * exp(s_ik - LSE_i) (s_ik recomputed,
// Sec. 4.1), the parameter adjoints are
//   G_k = sum_i w_ik z_ik y_ik^T = Q_k S_k with S_k = sum_i w_ik y_ik y_ik^T
//         (y = x - mu_k; S_k is an MFMA contraction over points of the
//         weighted and plain Y tiles, the product with Q_k is FP64),
//   v_k = sum_i w_ik z_ik = Q_k sum_i w_ik y_ik, W_k = sum_i w_ik,
//   alpha_bar_k = W_k - N ell_bar softmax(alpha)_k,
//   mu_bar_k = Q_k^T v_k,
//   q_bar_kd = W_k - exp(q_kd) G_k[d][d],
//   l_bar_k[r,c] = -G_k[r][c]  (r > c).
// Per (component, point chunk) blocks write FP32 partials of S_k and u_k
// (accumulated in the MFMA registers over at most 4096 points per wave); a
// per-component kernel sums them in FP64 in a fixed order, forms G_k and v_k
// and applies the parameter maps.
#include <math.h>

#include "common.h"
#include "prims.h"

namespace pvjp {

typedef float f32x16 __attribute__((ext_vector_type(16)));

__device__ __forceinline__ f32x16 mfma32(float a, float b, f32x16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
}

// Result layout of a 32x32 MFMA: lane l, item t holds row drow(t, l) and
// column l % 32.
__device__ __forceinline__ int drow(int t, int lane) { return 8 * (t >> 2) + 4 * (lane >> 5) + (t & 3); }

// Operand layout of a 32x32x2 MFMA step: lane l supplies A[l % 32][l / 32] and
// B[l / 32][l % 32]; the contraction index of step s, half h, is c = 2s + h.
template <int D>
struct Gm {
    static constexpr int RT = D / 32;                    // 32-row tiles of Q_k
    static constexpr int S = D / 2;                      // steps over a full row
    static constexpr int NF = 16 * RT * (RT + 1) / 2;    // A fragments in the lower triangle
    static constexpr int NGT = RT * (RT + 1) / 2;        // lower-triangular 32x32 blocks of G_k
};

// Fragment index of row tile rt, step s (rt's row needs steps s < 16 (rt+1)).
__host__ __device__ constexpr int fidx(int rt, int s) { return 8 * rt * (rt + 1) + s; }

// X tile of 32 points in LDS, row-major [p][c] with an XOR swizzle that keeps
// both the point-major and the column-major fragment reads conflict-free.
template <int D>
__device__ __forceinline__ int xs_at(int p, int c) {
    return p * D + (c ^ (D == 64 ? 2 * p : 2 * (p >> 1)));
}
// Weighted-Z tile [r][p] (32 points per row), swizzled the same way.
__device__ __forceinline__ int zs_at(int r, int p) { return r * 32 + (p ^ (2 * ((r >> 1) & 15))); }

constexpr double kLog2Pi = 1.8378770664093454835606594728112;

// -------------------------------------------------------------------- prep
template <int D>
__global__ __launch_bounds__(256) void gmm_prep_kernel(const float* __restrict__ alpha, const float* __restrict__ mu,
                                                       const float* __restrict__ q, const float* __restrict__ l,
                                                       int K, float* __restrict__ Qf, float* __restrict__ cvec,
                                                       double* __restrict__ bias, double* __restrict__ lse_alpha) {
    using C = Gm<D>;
    const int k = blockIdx.x;
    const int64_t tri = (int64_t)D * (D - 1) / 2;
    __shared__ float Q[D][D + 1];
    for (int e = threadIdx.x; e < D * D; e += blockDim.x) {
        const int r = e / D, c = e % D;
        float v = 0.f;
        if (r == c)
            v = (float)exp((double)q[(int64_t)k * D + r]);
        else if (r > c)
            v = l[(int64_t)k * tri + r * (r - 1) / 2 + c];
        Q[r][c] = v;
    }
    __syncthreads();
    for (int r = threadIdx.x; r < D; r += blockDim.x) {
        double acc = 0.0;
        for (int c = 0; c <= r; ++c) acc += (double)Q[r][c] * (double)mu[(int64_t)k * D + c];
        cvec[(int64_t)k * D + r] = (float)acc;
    }
    for (int e = threadIdx.x; e < C::NF * 64; e += blockDim.x) {
        const int f = e / 64, lane = e % 64;
        const int rt = (f < 16) ? 0 : 1;
        const int s = f - fidx(rt, 0);
        Qf[((int64_t)k * C::NF + f) * 64 + lane] = Q[32 * rt + (lane & 31)][2 * s + (lane >> 5)];
    }
    if (threadIdx.x == 0) {
        double b = (double)alpha[k];
        for (int d = 0; d < D; ++d) b += (double)q[(int64_t)k * D + d];
        bias[k] = b;
        if (k == 0) {
            double mx = -INFINITY;
            for (int j = 0; j < K; ++j) mx = fmax(mx, (double)alpha[j]);
            double s = 0.0;
            for (int j = 0; j < K; ++j) s += exp((double)alpha[j] - mx);
            *lse_alpha = mx + log(s);
        }
    }
}

// The wave's share of a 32-point X tile in registers (loaded ahead of use)
// and its store into the LDS tile.
template <int D>
struct XRegs {
    float4 v[(32 * D) / 256];
};

template <int D>
__device__ __forceinline__ void load_x(const float* __restrict__ X, int64_t N, int64_t p0, XRegs<D>& r) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int q = 0; q < (32 * D) / 256; ++q) {
        const int e = 4 * (lane + 64 * q);  // 4 consecutive floats of one point
        const int64_t p = p0 + e / D;
        r.v[q] = make_float4(0.f, 0.f, 0.f, 0.f);
        if (p < N) r.v[q] = *reinterpret_cast<const float4*>(X + p * D + e % D);
    }
}

template <int D>
__device__ __forceinline__ void store_x(const XRegs<D>& r, float* xs) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int q = 0; q < (32 * D) / 256; ++q) {
        const int e = 4 * (lane + 64 * q);
        const int pt = e / D, c = e % D;
        xs[xs_at<D>(pt, c)] = r.v[q].x;
        xs[xs_at<D>(pt, c + 1)] = r.v[q].y;
        xs[xs_at<D>(pt, c + 2)] = r.v[q].z;
        xs[xs_at<D>(pt, c + 3)] = r.v[q].w;
    }
}

template <int D>
__device__ __forceinline__ void stage_x(const float* __restrict__ X, int64_t N, int64_t p0, float* xs) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int q = 0; q < (32 * D) / 256; ++q) {
        const int e = 4 * (lane + 64 * q);  // 4 consecutive floats of one point
        const int pt = e / D, c = e % D;
        const int64_t p = p0 + pt;
        float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
        if (p < N) v = *reinterpret_cast<const float4*>(X + p * D + c);
        xs[xs_at<D>(pt, c)] = v.x;
        xs[xs_at<D>(pt, c + 1)] = v.y;
        xs[xs_at<D>(pt, c + 2)] = v.z;
        xs[xs_at<D>(pt, c + 3)] = v.w;
    }
}

// z = Q_k x - c_k for the wave's 32 points (column j = lane % 32) as MFMA
// accumulators, with Q_k's fragments (qs[f * 64 + lane]), c_k (cs[r]) and
// the X tile (xs, the wave's 32 points) read from LDS; the row tiles' MFMA
// chains are interleaved.  Each accumulator sees the operands in step order
// s = 0, 1, ..., the same as the forward sweep's chains, so z and |z|^2 are
// bit-identical to the forward's.  Returns sum_r z_r^2 in FP64 for the
// lane's point.
template <int D>
__device__ __forceinline__ double tile_znorm_lds(const float* qs, const float* cs, const float* xs,
                                                 f32x16 (&acc)[Gm<D>::RT]) {
    using C = Gm<D>;
    const int lane = threadIdx.x & 63;
    const int j = lane & 31, h = lane >> 5;
#pragma unroll
    for (int rt = 0; rt < C::RT; ++rt)
#pragma unroll
        for (int t = 0; t < 16; ++t) acc[rt][t] = 0.f;
#pragma unroll 8
    for (int s = 0; s < C::S; ++s) {
        const float bx = xs[xs_at<D>(j, 2 * s + h)];
#pragma unroll
        for (int rt = 0; rt < C::RT; ++rt)
            if (s < 16 * (rt + 1)) acc[rt] = mfma32(qs[fidx(rt, s) * 64 + lane], bx, acc[rt]);
    }
    double nrm = 0.0;
#pragma unroll
    for (int rt = 0; rt < C::RT; ++rt) {
#pragma unroll
        for (int t = 0; t < 16; ++t) {
            const float z = acc[rt][t] - cs[32 * rt + drow(t, lane)];
            acc[rt][t] = z;
            nrm = fma((double)z, (double)z, nrm);
        }
    }
    return nrm + __shfl_xor(nrm, 32, kWave);
}

template <int D>
__device__ __forceinline__ void load_component(const float* __restrict__ Qf, const float* __restrict__ cvec, int k,
                                               float (&qa)[Gm<D>::NF], float (&cl)[Gm<D>::RT][16]) {
    using C = Gm<D>;
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int f = 0; f < C::NF; ++f) qa[f] = Qf[((int64_t)k * C::NF + f) * 64 + lane];
#pragma unroll
    for (int rt = 0; rt < C::RT; ++rt)
#pragma unroll
        for (int t = 0; t < 16; ++t) cl[rt][t] = cvec[(int64_t)k * D + 32 * rt + drow(t, lane)];
}

// LDS written by a wave and read back by other lanes of the same wave: a
// wave-scope fence around a wave barrier (no other wave takes part).
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

struct GmmHdr {
    uint32_t done;
    uint32_t pad[63];
};

// ------------------------------------------------------------------ forward
// The block's four waves share each batch of CPB components: Q_k's fragments
// and c_k are staged in LDS once per block, and each wave interleaves the
// independent MFMA chains of the batch (CPB components x the row tiles of
// each), so the matrix unit has several chains to alternate between.  Every
// chain sees the same operands in the same order as tile_znorm_lds, so z, |z|^2
// and s_ik are bit-identical to the per-component form, and the online LSE
// takes the components in index order.
template <int D>
struct GmFwd {
    static constexpr int CPB = D == 64 ? 2 : 4;                // components per batch
    static constexpr int QF = Gm<D>::NF * 64;                  // fragment floats per component
    static constexpr int STAGE = CPB * (QF + D);               // floats staged per batch
    static constexpr int PER = (STAGE + 255) / 256;            // per thread (the last round partly empty)
    static constexpr int XS = 4 * 32 * D;                      // the X tiles, staged first
    static constexpr int LDS = XS > PER * 256 ? XS : PER * 256;
};

template <int D>
__device__ __forceinline__ void fwd_fetch(const float* __restrict__ Qf, const float* __restrict__ cvec, int k0, int K,
                                          float (&r)[GmFwd<D>::PER]) {
    using F = GmFwd<D>;
#pragma unroll
    for (int u = 0; u < F::PER; ++u) {
        const int e = u * 256 + (int)threadIdx.x;  // staged float index
        const int c = e < F::CPB * F::QF ? e / F::QF : (e - F::CPB * F::QF) / D;
        const int k = k0 + c;
        float v = 0.f;
        if (e < F::STAGE && k < K) {
            if (e < F::CPB * F::QF)
                v = Qf[(int64_t)k * F::QF + (e - c * F::QF)];
            else
                v = cvec[(int64_t)k * D + (e - F::CPB * F::QF - c * D)];
        }
        r[u] = v;
    }
}

template <int D>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) void gmm_fwd_kernel(const float* __restrict__ X, int64_t N, int K,
                                                      const float* __restrict__ Qf, const float* __restrict__ cvec,
                                                      const double* __restrict__ bias,
                                                      const double* __restrict__ lse_alpha, double* __restrict__ lse,
                                                      double* __restrict__ sck, double* parts, GmmHdr* hdr,
                                                      double* loglik) {
    using C = Gm<D>;
    using F = GmFwd<D>;
    __shared__ float sm[F::LDS];
    __shared__ double red[4];
    __shared__ int s_last;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t p0 = ((int64_t)blockIdx.x * 4 + w) * 32;
    float* Xs = sm + w * 32 * D;
    stage_x<D>(X, N, p0, Xs);
    __syncthreads();
    float bx[C::S];
#pragma unroll
    for (int s = 0; s < C::S; ++s) bx[s] = Xs[xs_at<D>(lane & 31, 2 * s + (lane >> 5))];
    const int64_t p = p0 + (lane & 31);
    const float* qs = sm;                       // [CPB][QF] during the batches
    const float* cs = sm + F::CPB * F::QF;      // [CPB][D]

    double m = -INFINITY, ssum = 0.0;
    const bool own = (lane < 32) && (p < N);
    for (int k0 = 0; k0 < K; k0 += F::CPB) {
        {
            float nxt[F::PER];
            fwd_fetch<D>(Qf, cvec, k0, K, nxt);
            __syncthreads();  // every wave is done with the previous batch (or with X)
#pragma unroll
            for (int u = 0; u < F::PER; ++u) sm[u * 256 + threadIdx.x] = nxt[u];
            __syncthreads();
        }
        f32x16 acc[F::CPB][C::RT];
#pragma unroll
        for (int c = 0; c < F::CPB; ++c)
#pragma unroll
            for (int rt = 0; rt < C::RT; ++rt)
#pragma unroll
                for (int t = 0; t < 16; ++t) acc[c][rt][t] = 0.f;
#pragma unroll 4
        for (int s = 0; s < C::S; ++s)
#pragma unroll
            for (int rt = 0; rt < C::RT; ++rt)
#pragma unroll
                for (int c = 0; c < F::CPB; ++c)
                    if (s < 16 * (rt + 1)) acc[c][rt] = mfma32(qs[c * F::QF + fidx(rt, s) * 64 + lane], bx[s], acc[c][rt]);
#pragma unroll
        for (int c = 0; c < F::CPB; ++c) {
            const int k = k0 + c;
            if (k >= K) break;
            double nrm = 0.0;
#pragma unroll
            for (int rt = 0; rt < C::RT; ++rt) {
#pragma unroll
                for (int t = 0; t < 16; ++t) {
                    const float z = acc[c][rt][t] - cs[c * D + 32 * rt + drow(t, lane)];
                    nrm = fma((double)z, (double)z, nrm);
                }
            }
            nrm += __shfl_xor(nrm, 32, kWave);
            const double sv = bias[k] - 0.5 * nrm;
            if (sck && own) sck[(int64_t)k * N + p] = sv;  // component-major: 32 points per wave in a row
            if (sv > m) {
                ssum = ssum * exp(m - sv) + 1.0;
                m = sv;
            } else {
                ssum += exp(sv - m);
            }
        }
    }
    const double l_i = m + log(ssum);
    const bool valid = (lane < 32) && (p < N);
    if (valid && lse) lse[p] = l_i;

    double v = valid ? l_i : 0.0;
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, kWave);
    if (lane == 0) red[w] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        st_coherent(&parts[blockIdx.x], (red[0] + red[1]) + (red[2] + red[3]));
        const uint32_t d = __hip_atomic_fetch_add(&hdr->done, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        s_last = (d == gridDim.x - 1);
    }
    __syncthreads();
    if (!s_last) return;
    // Last block: fixed-order sum of the block partials.
    double acc = 0.0;
    for (int b = threadIdx.x; b < (int)gridDim.x; b += 256) acc += ld_coherent(&parts[b]);
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) acc += __shfl_xor(acc, d, kWave);
    __syncthreads();
    if (lane == 0) red[w] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        const double tot = (red[0] + red[1]) + (red[2] + red[3]);
        *loglik = tot - (double)N * (*lse_alpha) - 0.5 * (double)N * D * kLog2Pi;
        __hip_atomic_store(&hdr->done, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// ----------------------------------------------------------------- backward
// The contraction runs over y = x - mu_k on both sides: S_k = sum_i w_ik
// y_ik y_ik^T and u_k = sum_i w_ik y_ik, from the X tile in LDS and each
// point's weight (no weighted-z tile); gmm_param_kernel then forms
// G_k = Q_k S_k and v_k = Q_k u_k in FP64 (z_ik = Q_k y_ik).  The weight
// needs s_ik: recomputed from |z_ik|^2 (one MFMA pass over Q_k), or, with
// FROM_S, read from the forward's s_ik checkpoint (sck, K x N), which halves
// the MFMA work.
template <int D, bool FROM_S>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void gmm_bwd_kernel(const float* __restrict__ X, int64_t N, int K, int64_t chunk,
                                                      int nch, const float* __restrict__ Qf,
                                                      const float* __restrict__ cvec, const float* __restrict__ mu,
                                                      const double* __restrict__ bias, const double* __restrict__ lse,
                                                      const double* __restrict__ sck,
                                                      double ell_bar, float* __restrict__ gpart,
                                                      float* __restrict__ vpart, double* __restrict__ wpart) {
    using C = Gm<D>;
    // X tiles of the four waves, and room for the scratch of the cross-wave
    // reduction at the end.  Q_k's MFMA fragments live in LDS too, read at
    // each step: held in registers they would leave room for only one wave
    // per SIMD.
    __shared__ __align__(16) float smem[2 * 4 * 32 * D];
    __shared__ float qs[C::NF * 64];
    __shared__ float cs[D];
    float* const Xw = smem + (threadIdx.x >> 6) * 32 * D;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int k = blockIdx.x % K;
    const int ch = blockIdx.x / K;
    const int h = lane >> 5, j = lane & 31;

    if (!FROM_S)
        for (int e = threadIdx.x; e < C::NF * 64; e += 256) qs[e] = Qf[(int64_t)k * C::NF * 64 + e];
    // cs: c_k for the recomputing form, mu_k for the checkpointed one
    if (threadIdx.x < D) cs[threadIdx.x] = FROM_S ? mu[(int64_t)k * D + threadIdx.x] : cvec[(int64_t)k * D + threadIdx.x];
    float mub[C::RT];
#pragma unroll
    for (int ct = 0; ct < C::RT; ++ct) mub[ct] = mu[(int64_t)k * D + 32 * ct + j];
    const double bk = bias[k];

    f32x16 gacc[C::NGT];
#pragma unroll
    for (int g = 0; g < C::NGT; ++g)
#pragma unroll
        for (int t = 0; t < 16; ++t) gacc[g][t] = 0.f;
    float urow[C::RT];
#pragma unroll
    for (int t = 0; t < C::RT; ++t) urow[t] = 0.f;
    double wsum = 0.0;

    const int64_t cbeg = (int64_t)ch * chunk;
    const int iters = (int)(chunk / 128);
    __syncthreads();  // qs and cs
    // Every tile below is private to its wave (Xw), so the waves only
    // synchronise with themselves and drift apart freely: one wave's MFMA
    // phase overlaps another's loads and FP64 work.
    // The next tile's X values (and its point's LSE and s_ik) are loaded
    // while this tile computes.
    XRegs<D> xr;
    double lse_n = 0.0, s_n = 0.0;
    {
        const int64_t p0 = cbeg + (int64_t)w * 32;
        load_x<D>(X, N, p0, xr);
        if (p0 + j < N) {
            lse_n = lse[p0 + j];
            if (FROM_S) s_n = sck[(int64_t)k * N + p0 + j];
        }
    }
    for (int it = 0; it < iters; ++it) {
        const int64_t p0 = cbeg + (int64_t)(it * 4 + w) * 32;
        wave_lds_sync();
        store_x<D>(xr, Xw);
        wave_lds_sync();
        const double lse_p = lse_n, s_p = s_n;
        if (it + 1 < iters) {
            const int64_t pn = p0 + 4 * 32;
            load_x<D>(X, N, pn, xr);
            if (pn + j < N) {
                lse_n = lse[pn + j];
                if (FROM_S) s_n = sck[(int64_t)k * N + pn + j];
            }
        }
        const int64_t p = p0 + j;
        double wd = 0.0;
        if (FROM_S) {
            if (p < N) wd = ell_bar * exp(s_p - lse_p);
        } else {
            // s_ik from |z|^2: z is recomputed for its norm only (the MFMA
            // phases run at raised wave priority, so that the other wave on
            // the SIMD issues its loads and FP64 work in their gaps)
            f32x16 z[C::RT];
            __builtin_amdgcn_s_setprio(1);
            const double nrm = tile_znorm_lds<D>(qs, cs, Xw, z);
            __builtin_amdgcn_s_setprio(0);
            if (p < N) wd = ell_bar * exp((bk - 0.5 * nrm) - lse_p);
        }
        const float wf = (float)wd;  // lane (j, h): the weight of point j
        if (h == 0) wsum += wd;
        // S_k += (w Y)^T Y over this tile's 32 points, lower-triangular
        // blocks: step s contracts point 2s + h, whose weight comes from lane
        // 2s + h; u_k = sum w y accumulates from the same products.  Each step
        // loads one operand per row tile and feeds the blocks' independent
        // accumulators in turn.
        __builtin_amdgcn_s_setprio(1);
#pragma unroll 8
        for (int s = 0; s < 16; ++s) {
            const int pt = 2 * s + h;
            const float wp = __shfl(wf, pt, kWave);
            float za[C::RT], yb[C::RT];
#pragma unroll
            for (int t = 0; t < C::RT; ++t) {
                yb[t] = Xw[xs_at<D>(pt, 32 * t + j)] - mub[t];
                za[t] = wp * yb[t];
                urow[t] += za[t];
            }
            int g = 0;
#pragma unroll
            for (int rt = 0; rt < C::RT; ++rt)
#pragma unroll
                for (int ct = 0; ct <= rt; ++ct) {
                    gacc[g] = mfma32(za[rt], yb[ct], gacc[g]);
                    ++g;
                }
        }
        __builtin_amdgcn_s_setprio(0);
    }

    // u: the two half-waves hold the halves of each row sum; lane r < D takes
    // row r's (rows 32 t + j live in lane j's urow[t]).
#pragma unroll
    for (int t = 0; t < C::RT; ++t) urow[t] += __shfl_xor(urow[t], 32, kWave);
    const float uhi = __shfl(urow[C::RT - 1], lane & 31, kWave);
    float vrow = lane < 32 ? urow[0] : uhi;
#pragma unroll
    for (int d = 16; d >= 1; d >>= 1) wsum += __shfl_xor(wsum, d, kWave);

    // Combine the four waves through LDS (reusing the tiles) in a fixed order.
    __syncthreads();
    float* red = smem;
    constexpr int kRedFloats = 3 * Gm<D>::NGT * 1024 + 3 * D;
    static_assert(kRedFloats + 8 <= 2 * 4 * 32 * D, "reduction scratch");
    double* wred = reinterpret_cast<double*>(smem + ((kRedFloats + 1) & ~1));
    if (w > 0) {
#pragma unroll
        for (int g = 0; g < C::NGT; ++g)
#pragma unroll
            for (int t = 0; t < 16; ++t) red[((w - 1) * C::NGT * 16 + g * 16 + t) * 64 + lane] = gacc[g][t];
        if (lane < D) red[3 * C::NGT * 1024 + (w - 1) * D + lane] = vrow;
    }
    if (lane == 0) wred[w] = wsum;
    __syncthreads();
    if (w == 0) {
        const int64_t rec = (int64_t)k * nch + ch;
#pragma unroll
        for (int g = 0; g < C::NGT; ++g)
#pragma unroll
            for (int t = 0; t < 16; ++t) {
                float s = gacc[g][t];
                for (int o = 0; o < 3; ++o) s += red[(o * C::NGT * 16 + g * 16 + t) * 64 + lane];
                gpart[(rec * C::NGT * 16 + g * 16 + t) * 64 + lane] = s;
            }
        if (lane < D) {
            float s = vrow;
            for (int o = 0; o < 3; ++o) s += red[3 * C::NGT * 1024 + o * D + lane];
            vpart[rec * D + lane] = s;
        }
        if (lane == 0) wpart[rec] = (wred[0] + wred[1]) + (wred[2] + wred[3]);
    }
}

// ------------------------------------------------------ reduce + parameters
template <int D>
__global__ __launch_bounds__(256) void gmm_param_kernel(int64_t N, int K, int nch, const float* __restrict__ alpha,
                                                        const float* __restrict__ q, const float* __restrict__ l,
                                                        const double* __restrict__ lse_alpha, double ell_bar,
                                                        const float* __restrict__ gpart,
                                                        const float* __restrict__ vpart,
                                                        const double* __restrict__ wpart, float* __restrict__ abar,
                                                        float* __restrict__ mbar, float* __restrict__ qbar,
                                                        float* __restrict__ lbar, int accumulate) {
    using C = Gm<D>;
    const int k = blockIdx.x;
    const int64_t tri = (int64_t)D * (D - 1) / 2;
    __shared__ double G[D][D + 1];
    __shared__ double v[D];
    __shared__ double Wk;
    __shared__ float Q[D][D + 1];
    // G (lower-triangular 32x32 blocks) summed over chunks in FP64, chunk order.
    for (int e = threadIdx.x; e < C::NGT * 1024; e += blockDim.x) {
        const int g = e / 1024, t = (e / 64) % 16, lane = e % 64;
        int rt = 0, ct = 0;
        if (g == 1) rt = 1;
        if (g == 2) rt = 1, ct = 1;
        double s = 0.0;
        for (int c = 0; c < nch; ++c) s += (double)gpart[(((int64_t)k * nch + c) * C::NGT * 16 + g * 16 + t) * 64 + lane];
        G[32 * rt + drow(t, lane)][32 * ct + (lane & 31)] = s;
    }
    for (int r = threadIdx.x; r < D; r += blockDim.x) {
        double s = 0.0;
        for (int c = 0; c < nch; ++c) s += (double)vpart[((int64_t)k * nch + c) * D + r];
        v[r] = s;
    }
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int c = 0; c < nch; ++c) s += wpart[(int64_t)k * nch + c];
        Wk = s;
    }
    for (int e = threadIdx.x; e < D * D; e += blockDim.x) {
        const int r = e / D, c = e % D;
        float x = 0.f;
        if (r == c)
            x = (float)exp((double)q[(int64_t)k * D + r]);
        else if (r > c)
            x = l[(int64_t)k * tri + r * (r - 1) / 2 + c];
        Q[r][c] = x;
    }
    __syncthreads();
    {
        // The partials hold S_k (lower 32x32 blocks, symmetric) and u_k:
        // mirror S, then G_k = Q_k S_k row by row from the bottom (row r of G
        // needs rows <= r of S, which are still unchanged) and v_k = Q_k u_k.
        for (int e = threadIdx.x; e < D * D; e += blockDim.x) {
            const int r = e / D, c = e % D;
            if (c > r) G[r][c] = G[c][r];
        }
        __syncthreads();
        for (int r = D - 1; r >= 0; --r) {
            double gr = 0.0;
            const int c = threadIdx.x;
            if (c < D)
                for (int j2 = 0; j2 <= r; ++j2) gr += (double)Q[r][j2] * G[j2][c];
            double vr = 0.0;
            if (threadIdx.x == 0)
                for (int j2 = 0; j2 <= r; ++j2) vr += (double)Q[r][j2] * v[j2];
            __syncthreads();
            if (c < D) G[r][c] = gr;
            if (threadIdx.x == 0) v[r] = vr;
            __syncthreads();
        }
    }
    const double W = Wk;
    if (threadIdx.x == 0) {
        const double a = W - (double)N * ell_bar * exp((double)alpha[k] - *lse_alpha);
        abar[k] = accumulate ? abar[k] + (float)a : (float)a;
    }
    for (int c = threadIdx.x; c < D; c += blockDim.x) {
        double s = 0.0;  // (Q_k^T v_k)_c = sum_{r >= c} Q[r][c] v[r]
        for (int r = c; r < D; ++r) s += (double)Q[r][c] * v[r];
        const int64_t o = (int64_t)k * D + c;
        mbar[o] = accumulate ? mbar[o] + (float)s : (float)s;
        const double qd = W - (double)Q[c][c] * G[c][c];
        qbar[o] = accumulate ? qbar[o] + (float)qd : (float)qd;
    }
    for (int e = threadIdx.x; e < tri; e += blockDim.x) {
        // packed strictly-lower index e -> (r, c), r > c, e = r(r-1)/2 + c
        int r = (int)((1.0 + sqrt(1.0 + 8.0 * (double)e)) / 2.0);
        while (r * (r - 1) / 2 > e) --r;
        while ((r + 1) * r / 2 <= e) ++r;
        const int c = e - r * (r - 1) / 2;
        const int64_t o = (int64_t)k * tri + e;
        const float g = (float)(-G[r][c]);
        lbar[o] = accumulate ? lbar[o] + g : g;
    }
}

// ------------------------------------------------------------------ host
struct GmmLayout {
    size_t Qf, cvec, bias, scal, fparts, lse, gpart, vpart, wpart, total;
    int64_t nch, chunk;
    unsigned fgrid;
};

static GmmLayout gmm_layout(int64_t N, int D, int K) {
    GmmLayout L{};
    const int RT = D / 32;
    const int NF = 16 * RT * (RT + 1) / 2, NGT = RT * (RT + 1) / 2;
    int64_t target = 4096 / K;
    if (target < 1) target = 1;
    int64_t chunk = ceil_div(ceil_div(N > 0 ? N : 1, target), 128) * 128;
    if (chunk > 16384) chunk = 16384;
    if (chunk < 128) chunk = 128;
    L.chunk = chunk;
    L.nch = ceil_div(N > 0 ? N : 1, chunk);
    L.fgrid = (unsigned)ceil_div(N > 0 ? N : 1, 128);
    size_t o = 0;
    auto take = [&](size_t bytes) {
        size_t at = o;
        o += align_up(bytes, 256);
        return at;
    };
    L.scal = take(sizeof(GmmHdr) + 256);  // header, lse_alpha, loglik scratch
    L.Qf = take((size_t)K * NF * 64 * 4);
    L.cvec = take((size_t)K * D * 4);
    L.bias = take((size_t)K * 8);
    L.fparts = take((size_t)L.fgrid * 8);
    L.lse = take((size_t)(N > 0 ? N : 1) * 8);
    L.gpart = take((size_t)K * L.nch * NGT * 1024 * 4);
    L.vpart = take((size_t)K * L.nch * D * 4);
    L.wpart = take((size_t)K * L.nch * 8);
    L.total = o;
    return L;
}

template <int D>
static void launch_prep(const float* alpha, const float* mu, const float* q, const float* l, int K, char* ws,
                        const GmmLayout& L, hipStream_t st) {
    double* scal = reinterpret_cast<double*>(ws + L.scal + sizeof(GmmHdr));
    hipLaunchKernelGGL(gmm_prep_kernel<D>, dim3(K), dim3(256), 0, st, alpha, mu, q, l, K, (float*)(ws + L.Qf),
                       (float*)(ws + L.cvec), (double*)(ws + L.bias), scal);
}

template <int D>
static void launch_fwd(const float* X, int64_t N, int K, char* ws, const GmmLayout& L, double* lse, double* sck,
                       double* loglik, hipStream_t st) {
    double* scal = reinterpret_cast<double*>(ws + L.scal + sizeof(GmmHdr));
    hipLaunchKernelGGL(gmm_fwd_kernel<D>, dim3(L.fgrid), dim3(256), 0, st, X, N, K, (const float*)(ws + L.Qf),
                       (const float*)(ws + L.cvec), (const double*)(ws + L.bias), (const double*)scal, lse, sck,
                       (double*)(ws + L.fparts), (GmmHdr*)(ws + L.scal), loglik);
}

template <int D, bool FROM_S>
static void launch_bwd_t(const float* X, int64_t N, int K, const float* alpha, const float* mu, const float* q,
                         const float* l, double ell_bar, const double* lse, const double* sck, float* ab, float* mb,
                         float* qb, float* lb, int acc, char* ws, const GmmLayout& L, hipStream_t st) {
    double* scal = reinterpret_cast<double*>(ws + L.scal + sizeof(GmmHdr));
    hipLaunchKernelGGL((gmm_bwd_kernel<D, FROM_S>), dim3((unsigned)(K * L.nch)), dim3(256), 0, st, X, N, K, L.chunk,
                       (int)L.nch, (const float*)(ws + L.Qf), (const float*)(ws + L.cvec), mu,
                       (const double*)(ws + L.bias), lse, sck, ell_bar, (float*)(ws + L.gpart),
                       (float*)(ws + L.vpart), (double*)(ws + L.wpart));
    hipLaunchKernelGGL((gmm_param_kernel<D>), dim3(K), dim3(256), 0, st, N, K, (int)L.nch, alpha, q, l,
                       (const double*)scal, ell_bar, (const float*)(ws + L.gpart), (const float*)(ws + L.vpart),
                       (const double*)(ws + L.wpart), ab, mb, qb, lb, acc);
}

template <int D>
static void launch_bwd(const float* X, int64_t N, int K, const float* alpha, const float* mu, const float* q,
                       const float* l, double ell_bar, const double* lse, const double* sck, float* ab, float* mb,
                       float* qb, float* lb, int acc, char* ws, const GmmLayout& L, hipStream_t st) {
    if (sck)
        launch_bwd_t<D, true>(X, N, K, alpha, mu, q, l, ell_bar, lse, sck, ab, mb, qb, lb, acc, ws, L, st);
    else
        launch_bwd_t<D, false>(X, N, K, alpha, mu, q, l, ell_bar, lse, sck, ab, mb, qb, lb, acc, ws, L, st);
}

static pvjp_status gmm_args(int64_t N, int D, int K, const void* X, const void* alpha, const void* mu,
                            const void* q, const void* l, const char* name) {
    if (D != 32 && D != 64) {
        set_error("%s: D = %d unsupported (the MFMA path is built for D = 32 and D = 64)", name, D);
        return PVJP_EUNSUPPORTED;
    }
    PVJP_REQUIRE(N >= 0 && N <= ((int64_t)1 << 40), "%s: N = %lld out of range", name, (long long)N);
    PVJP_REQUIRE(K >= 1 && K <= 65535, "%s: K = %d out of range [1, 65535]", name, K);
    PVJP_REQUIRE(alpha && mu && q && l && (N == 0 || X), "%s: X, alpha, mu, q and l must be non-NULL", name);
    PVJP_REQUIRE(aligned(X, 16), "%s: X must be 16-byte aligned", name);
    return PVJP_OK;
}

}  // namespace pvjp

using namespace pvjp;

extern "C" size_t pvjp_gmm_ws_bytes(int64_t N, int D, int K) {
    if (N < 0 || (D != 32 && D != 64) || K < 1) return 0;
    return gmm_layout(N, D, K).total;
}

extern "C" pvjp_status pvjp_gmm_objective(const float* X, int64_t N, int D, int K, const float* alpha,
                                          const float* mu, const float* q, const float* l, double* loglik,
                                          double* lse, double* s, void* ws, size_t ws_bytes, void* stream) {
    clear_error();
    if (pvjp_status e = gmm_args(N, D, K, X, alpha, mu, q, l, "pvjp_gmm_objective")) return e;
    PVJP_REQUIRE(loglik != nullptr, "pvjp_gmm_objective: loglik is NULL");
    PVJP_REQUIRE(ws != nullptr && aligned(ws, 256), "pvjp_gmm_objective: ws must be non-NULL and 256-byte aligned");
    const GmmLayout L = gmm_layout(N, D, K);
    if (ws_bytes < L.total) {
        set_error("pvjp_gmm_objective: workspace has %zu bytes, needs %zu", ws_bytes, L.total);
        return PVJP_ENOMEM;
    }
    char* w = reinterpret_cast<char*>(ws);
    hipStream_t st = as_stream(stream);
    if (D == 64) {
        launch_prep<64>(alpha, mu, q, l, K, w, L, st);
        launch_fwd<64>(X, N, K, w, L, lse, s, loglik, st);
    } else {
        launch_prep<32>(alpha, mu, q, l, K, w, L, st);
        launch_fwd<32>(X, N, K, w, L, lse, s, loglik, st);
    }
    PVJP_LAUNCHED("pvjp_gmm_objective");
    return PVJP_OK;
}

extern "C" pvjp_status pvjp_gmm_vjp(const float* X, int64_t N, int D, int K, const float* alpha, const float* mu,
                                    const float* q, const float* l, double ell_bar, const double* lse,
                                    const double* s, float* alpha_bar, float* mu_bar, float* q_bar, float* l_bar,
                                    int accumulate, void* ws, size_t ws_bytes, void* stream) {
    clear_error();
    if (pvjp_status e = gmm_args(N, D, K, X, alpha, mu, q, l, "pvjp_gmm_vjp")) return e;
    PVJP_REQUIRE(s == nullptr || lse != nullptr, "pvjp_gmm_vjp: the s checkpoint needs lse as well");
    PVJP_REQUIRE(alpha_bar && mu_bar && q_bar && l_bar, "pvjp_gmm_vjp: the four adjoint outputs must be non-NULL");
    PVJP_REQUIRE(ws != nullptr && aligned(ws, 256), "pvjp_gmm_vjp: ws must be non-NULL and 256-byte aligned");
    const GmmLayout L = gmm_layout(N, D, K);
    if (ws_bytes < L.total) {
        set_error("pvjp_gmm_vjp: workspace has %zu bytes, needs %zu", ws_bytes, L.total);
        return PVJP_ENOMEM;
    }
    char* w = reinterpret_cast<char*>(ws);
    hipStream_t st = as_stream(stream);
    double* ll_scratch = reinterpret_cast<double*>(w + L.scal + sizeof(GmmHdr)) + 1;
    if (D == 64) {
        launch_prep<64>(alpha, mu, q, l, K, w, L, st);
        if (lse == nullptr) {
            launch_fwd<64>(X, N, K, w, L, (double*)(w + L.lse), nullptr, ll_scratch, st);
            lse = (const double*)(w + L.lse);
        }
        launch_bwd<64>(X, N, K, alpha, mu, q, l, ell_bar, lse, s, alpha_bar, mu_bar, q_bar, l_bar, accumulate, w, L,
                       st);
    } else {
        launch_prep<32>(alpha, mu, q, l, K, w, L, st);
        if (lse == nullptr) {
            launch_fwd<32>(X, N, K, w, L, (double*)(w + L.lse), nullptr, ll_scratch, st);
            lse = (const double*)(w + L.lse);
        }
        launch_bwd<32>(X, N, K, alpha, mu, q, l, ell_bar, lse, s, alpha_bar, mu_bar, q_bar, l_bar, accumulate, w, L,
                       st);
    }
    PVJP_LAUNCHED("pvjp_gmm_vjp");
    return PVJP_OK;
}
