// The general operators of the reduce and scan rules (Sec. 5.1.1, 5.2) as
// device structs: log-add-exp, the first-order linear recurrence and the 2x2
// matrix product, plus the operand-exchanged form used by reversed scans.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>

#include "prims.h"

namespace pvjp {

template <class T, int K>
struct GS {
    T c[K];
};

template <class T, int K>
struct GShfl {
    using S = GS<T, K>;
    __device__ static __forceinline__ S up(S v, int d) {
        S r;
#pragma unroll
        for (int c = 0; c < K; ++c) r.c[c] = shfl_up1(v.c[c], d);
        return r;
    }
    __device__ static __forceinline__ S down(S v, int d) {
        S r;
#pragma unroll
        for (int c = 0; c < K; ++c) r.c[c] = shfl_down1(v.c[c], d);
        return r;
    }
    __device__ static __forceinline__ S idx(S v, int s) {
        S r;
#pragma unroll
        for (int c = 0; c < K; ++c) r.c[c] = shfl_idx1(v.c[c], s);
        return r;
    }
};

// An operator provides: K input components; a state S (its shuffles come
// from GShfl) with elem() turning an element's components into a state and
// value() turning a state back into K result components; the neutral id();
// comb(x, y) = x (.) y with x earlier in index order; and the function f,
// vjp(l, a, r, la, yb, out): out = (d(l (.) a (.) r)/da)^T yb, where la is
// l (.) a (already formed by the caller for the next prefix).

// log-add-exp.  The state is (m, s) standing for m + log(s), the neutral
// element (-inf, 0): combining costs one exp and no log, and exp(a - y)
// becomes exp(a - m_y) / s_y.  Each element is (x, 1), or the neutral
// element when x = -inf.
// exp and division for log-add-exp: in FP32 the hardware exp2 (about 1 ulp
// plus |x| * 2^-24 relative, x <= 0 here) and reciprocal; FP64 uses the
// library functions.
__device__ __forceinline__ float lae_exp(float x) { return __expf(x); }
__device__ __forceinline__ double lae_exp(double x) { return exp(x); }
__device__ __forceinline__ float lae_div(float a, float b) { return __fdividef(a, b); }
__device__ __forceinline__ double lae_div(double a, double b) { return a / b; }
__device__ __forceinline__ float lae_log(float x) { return logf(x); }
__device__ __forceinline__ double lae_log(double x) { return log(x); }

// Log-add-exp with the state (m, s) in T and the exponentials evaluated in E
// (E = T, or FP32 with an FP64 state: see the scans' widening below).
template <class T, class E = T>
struct GLogAddExpE : GShfl<T, 2> {
    static constexpr int K = 1;
    using Acc = T;
    using S = GS<T, 2>;
    __device__ static __forceinline__ T ex(T a) { return (T)lae_exp((E)a); }
    // The output's logarithm in E: nothing downstream accumulates it.
    __device__ static __forceinline__ S id() { return S{{-(T)INFINITY, T(0)}}; }
    __device__ static __forceinline__ S elem(const T (&c)[1]) {
        return S{{c[0], c[0] == -(T)INFINITY ? T(0) : T(1)}};
    }
    __device__ static __forceinline__ void value(S v, T (&out)[1]) { out[0] = v.c[0] + (T)lae_log((E)v.c[1]); }
    __device__ static __forceinline__ S comb(S x, S y) {
        if (y.c[1] == T(0)) return x;
        if (x.c[1] == T(0)) return y;
        const T d = x.c[0] - y.c[0];
        const T e = ex(-fabs(d));
        return d >= T(0) ? S{{x.c[0], x.c[1] + y.c[1] * e}} : S{{y.c[0], x.c[1] * e + y.c[1]}};
    }
    __device__ static __forceinline__ void vjp(S, S a, S r, S la, const T (&yb)[1], T (&out)[1]) {
        // d/da log(e^l + e^a + e^r) = e^(a - y); a -inf element receives 0
        if (a.c[1] == T(0)) {
            out[0] = T(0);
            return;
        }
        const S y = comb(la, r);
        out[0] = lae_div(yb[0] * ex(a.c[0] - y.c[0]), y.c[1]);
    }
    // Scan Jacobians (value y = m + log s).  cT = d(y (.) xn)/dy = e^y / (e^y +
    // e^xn) = s / (s + e^(xn - m)), 0 where y = -inf.
    __device__ static __forceinline__ void jlT(const S& y, const T (&xn)[1], T (&cT)[1][1]) {
        cT[0][0] = y.c[1] == T(0) ? T(0) : lae_div(y.c[1], y.c[1] + ex(xn[0] - y.c[0]));
    }
    // out = (d(yp (.) x)/dx)^T r = r e^(x - y) with y = yp (.) x; 0 where x = -inf.
    __device__ static __forceinline__ void jrT(const S&, const T (&x)[1], const S& y, const T (&r)[1], T (&out)[1]) {
        out[0] = x[0] == -(T)INFINITY ? T(0) : r[0] * lae_div(ex(x[0] - y.c[0]), y.c[1]);
    }
};
template <class T>
using GLogAddExp = GLogAddExpE<T, T>;

template <class T>
struct GLinRec : GShfl<T, 2> {
    static constexpr int K = 2;
    using Acc = T;
    using S = GS<T, 2>;
    __device__ static __forceinline__ S id() { return S{{T(1), T(0)}}; }
    __device__ static __forceinline__ S elem(const T (&c)[2]) { return S{{c[0], c[1]}}; }
    __device__ static __forceinline__ void value(S v, T (&out)[2]) { out[0] = v.c[0], out[1] = v.c[1]; }
    __device__ static __forceinline__ S comb(S x, S y) { return S{{y.c[0] * x.c[0], y.c[0] * x.c[1] + y.c[1]}}; }
    __device__ static __forceinline__ void vjp(S l, S, S r, S, const T (&yb)[2], T (&out)[2]) {
        // y = (r.a x.a l.a, r.a (x.a l.b + x.b) + r.b)
        out[0] = r.c[0] * (yb[0] * l.c[0] + yb[1] * l.c[1]);
        out[1] = r.c[0] * yb[1];
    }
    // Scan Jacobians: d(y (.) xn)/dy = a' I; d(yp (.) x)/dx = [[A, 0], [B, 1]].
    __device__ static __forceinline__ void jlT(const S&, const T (&xn)[2], T (&cT)[2][2]) {
        cT[0][0] = xn[0], cT[0][1] = T(0), cT[1][0] = T(0), cT[1][1] = xn[0];
    }
    __device__ static __forceinline__ void jrT(const S& yp, const T (&)[2], const S&, const T (&r)[2], T (&out)[2]) {
        out[0] = yp.c[0] * r[0] + yp.c[1] * r[1];
        out[1] = r[1];
    }
};

template <class T>
struct GMat2 : GShfl<T, 4> {
    static constexpr int K = 4;
    using Acc = T;
    using S = GS<T, 4>;
    __device__ static __forceinline__ S id() { return S{{T(1), T(0), T(0), T(1)}}; }
    __device__ static __forceinline__ S elem(const T (&c)[4]) { return S{{c[0], c[1], c[2], c[3]}}; }
    __device__ static __forceinline__ void value(S v, T (&out)[4]) {
        for (int c = 0; c < 4; ++c) out[c] = v.c[c];
    }
    __device__ static __forceinline__ S comb(S x, S y) {
        return S{{x.c[0] * y.c[0] + x.c[1] * y.c[2], x.c[0] * y.c[1] + x.c[1] * y.c[3],
                  x.c[2] * y.c[0] + x.c[3] * y.c[2], x.c[2] * y.c[1] + x.c[3] * y.c[3]}};
    }
    __device__ static __forceinline__ void vjp(S l, S, S r, S, const T (&yb)[4], T (&out)[4]) {
        // y = l a r, so a_bar = l^T y_bar r^T; M = y_bar r^T first
        const T m00 = yb[0] * r.c[0] + yb[1] * r.c[1], m01 = yb[0] * r.c[2] + yb[1] * r.c[3];
        const T m10 = yb[2] * r.c[0] + yb[3] * r.c[1], m11 = yb[2] * r.c[2] + yb[3] * r.c[3];
        out[0] = l.c[0] * m00 + l.c[2] * m10;
        out[1] = l.c[0] * m01 + l.c[2] * m11;
        out[2] = l.c[1] * m00 + l.c[3] * m10;
        out[3] = l.c[1] * m01 + l.c[3] * m11;
    }
    // Scan Jacobians on row-major 4-vectors.  Y' = Y X: dY'[r][c]/dY[r][k] =
    // X[k][c], so cT[2r+k][2r+c] = X[k][c] (zero across rows); and
    // (dY'/dX)^T R = Yp^T R.
    __device__ static __forceinline__ void jlT(const S&, const T (&xn)[4], T (&cT)[4][4]) {
#pragma unroll
        for (int p = 0; p < 4; ++p)
#pragma unroll
            for (int q = 0; q < 4; ++q) cT[p][q] = (p >> 1) == (q >> 1) ? xn[2 * (p & 1) + (q & 1)] : T(0);
    }
    __device__ static __forceinline__ void jrT(const S& yp, const T (&)[4], const S&, const T (&r)[4], T (&out)[4]) {
#pragma unroll
        for (int k = 0; k < 2; ++k)
#pragma unroll
            for (int c = 0; c < 2; ++c) out[2 * k + c] = yp.c[k] * r[c] + yp.c[2 + k] * r[2 + c];
    }
};

// The same operator with its operands exchanged: a scan in reversed index
// order with it folds x_{i+1} (.) x_{i+2} (.) ... (the reversed scan of the
// rule, whose operator is \x y -> y (.) x).
template <class Op>
struct Flip : Op {
    using S = typename Op::S;
    __device__ static __forceinline__ S comb(S x, S y) { return Op::comb(y, x); }
};

}  // namespace pvjp
