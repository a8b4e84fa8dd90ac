/*
 * CPU oracle for the reverse-mode rules of bulk-parallel operators.
 *
 * TEST INFRASTRUCTURE ONLY. Nothing in the product path may include, link or
 * call this code; it exists so that the GPU library can be checked against a
 * plain, slow, obviously correct implementation that shares no code with it.
 *
 * Method. Every function evaluates its operator by the sequential semantics
 * the paper states for it (reduce: Sec. 5.1; reduce_by_index: Sec. 5.1.2;
 * inclusive scan: Sec. 5.2; scatter: Sec. 5.3; map: Sec. 5.4) in FP64 while
 * recording each elementary step on an explicit tape (a Wengert list of
 * records holding the local partial derivatives).  A VJP seeds the output
 * adjoints and sweeps the tape in reverse, applying the core rewrite rule
 * a_bar += (df/da) * v_bar of Sec. 2.0.2 (eq. rewrite-adj), summing over all
 * uses of a variable.  The oracle deliberately does NOT implement the
 * paper's per-operator rewrite rules (two scans for reduce, the three-case
 * product rule, the lin_o reversed scan, the gather form of the scatter
 * adjoint): those are what the GPU kernels implement, so agreement between the
 * two is independent evidence.
 *
 * All arrays are host arrays owned by the caller; all floating-point data is
 * double (FP32 inputs are upcast exactly by the caller).  Return value: 0 on
 * success, -1 on bad arguments, -2 on allocation failure.
 */
#ifndef PVJP_ORACLE_H
#define PVJP_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_ADD = 0, ORC_MUL = 1, ORC_MIN = 2, ORC_MAX = 3 };
enum { ORC_FN_SQUARE = 0, ORC_FN_EXP = 1, ORC_FN_LOG = 2, ORC_FN_SIN = 3, ORC_FN_TANH = 4 };

/* Linear-recurrence inclusive scan (Sec. 5.2 with the operator
 * (a1,b1) (+) (a2,b2) = (a2*a1, a2*b1 + b2)). */
int orc_linrec_scan(int64_t n, const double* a, const double* b, double* A, double* B);
int orc_linrec_scan_vjp(int64_t n, const double* a, const double* b,
                        const double* yA_bar, const double* yB_bar,
                        double* a_bar, double* b_bar);

/* reduce (Sec. 5.1, 5.1.1).  Primal outputs: y; for MIN/MAX the lowest index
 * attaining y (-1 if n == 0); for MUL the product of the non-zero elements p
 * and the zero count z. */
int orc_reduce(int op, int64_t n, const double* x, double* y, int64_t* arg,
               double* p, int64_t* z);
int orc_reduce_vjp(int op, int64_t n, const double* x, double y_bar, double* x_bar);

/* reduce_by_index (Sec. 5.1.2): hs[k] = (+) over {i : inds[i] == k} of vs[i].
 * Indices outside [0, m) are ignored.  Outputs (any may be NULL): hs[m];
 * winner[m] (MIN/MAX: lowest index attaining hs[k], -1 if empty); p[m] and
 * z[m] (MUL: product of non-zeros, zero count); count[m]. */
int orc_hist(int op, int64_t n, int64_t m, const int32_t* inds, const double* vs,
             double* hs, int64_t* winner, double* p, int64_t* z, int64_t* count);
int orc_hist_vjp(int op, int64_t n, int64_t m, const int32_t* inds, const double* vs,
                 const double* hs_bar, double* vs_bar);

/* scatter (Sec. 5.3): ys = xs with ys[is[j]] = vs[j]; xs_saved[j] = xs[is[j]].
 * Indices outside [0, n) are ignored (xs_saved[j] = 0 for them). */
int orc_scatter(int64_t n, const double* xs, int64_t m, const int32_t* is,
                const double* vs, double* ys, double* xs_saved);
int orc_scatter_vjp(int64_t n, int64_t m, const int32_t* is, const double* ys_bar,
                    double* xs_bar, double* vs_bar);

/* map (Sec. 5.4) of a unary elementwise function. */
int orc_map(int fn, int64_t n, const double* x, double* y);
int orc_map_vjp(int fn, int64_t n, const double* x, const double* y_bar, double* x_bar);

/* map of the two-input, two-output program of Fig. 1:
 * P(x0, x1) = (x1 * sin(x0), x0 * x1), applied elementwise. */
int orc_fig1(int64_t n, const double* x0, const double* x1, double* y0, double* y1);
int orc_fig1_vjp(int64_t n, const double* x0, const double* x1,
                 const double* y0_bar, const double* y1_bar,
                 double* x0_bar, double* x1_bar);

/* Gaussian-mixture log-likelihood with a precision-Cholesky parametrisation:
 *   Q_k = diag(exp(q_k)) + L_k,  L_k strictly lower, entry (r,c), r > c, at
 *         l[k*D(D-1)/2 + r(r-1)/2 + c];
 *   s_ik = alpha_k + sum_d q_kd - 0.5 * || Q_k (x_i - mu_k) ||^2;
 *   loglik = sum_i LSE_k(s_ik) - N * LSE(alpha) - (N*D/2) * log(2*pi).
 * X is row-major N x D, mu and q are K x D.  lse (nullable) receives the
 * per-point LSE_k(s_ik). */
int orc_gmm_objective(int64_t N, int D, int K, const double* X, const double* alpha,
                      const double* mu, const double* q, const double* l,
                      double* loglik, double* lse);
int orc_gmm_vjp(int64_t N, int D, int K, const double* X, const double* alpha,
                const double* mu, const double* q, const double* l, double ell_bar,
                double* alpha_bar, double* mu_bar, double* q_bar, double* l_bar);

/* reduce with a general associative operator (Sec. 5.1.1, general rule):
 * y = x_0 (.) x_1 (.) ... (.) x_{n-1}, a left fold from the neutral element.
 * An element has K components, each a separate array (x[c][i]):
 *   LOGADDEXP (K=1): a (.) b = log(exp(a) + exp(b)), neutral -inf.  Inputs
 *       are finite or -inf; a -inf element contributes nothing and receives
 *       a zero adjoint.
 *   LINREC (K=2, components a, b): (a1,b1) (.) (a2,b2) = (a2*a1, a2*b1 + b2),
 *       neutral (1, 0).
 *   MAT2 (K=4, row-major m00, m01, m10, m11): the 2x2 matrix product
 *       y = x_0 x_1 ... x_{n-1}, neutral the identity.
 * y, y_bar: K values.  x_bar: K arrays of n, overwritten.  The VJP records
 * the fold's elementary steps on the tape and sweeps it in reverse.
 * orc_reduce_generic_vjp_at gives the adjoints of the elements idx[0..cnt)
 * only (out[j*K + c]), in O(n) time and O(cnt) memory: the left fold before
 * and the right fold after each sampled element are plain FP64 folds, and
 * only the three-operand fold l (.) x_i (.) r is recorded and swept. */
enum { ORC_GOP_LOGADDEXP = 0, ORC_GOP_LINREC = 1, ORC_GOP_MAT2 = 2 };
int orc_gop_components(int op);
int orc_reduce_generic(int op, int64_t n, const double* const* x, double* y);
int orc_reduce_generic_vjp(int op, int64_t n, const double* const* x, const double* y_bar,
                           double* const* x_bar);
int orc_reduce_generic_vjp_at(int op, int64_t n, const double* const* x, const double* y_bar,
                              int64_t cnt, const int64_t* idx, double* out);

/* Inclusive scan with the same general operators (Sec. 5.2 and its Jacobian
 * generalisation): y_i = x_0 (.) ... (.) x_i, K output components per
 * element (LOGADDEXP: the running log-sum-exp).  y[c], y_bar[c], x_bar[c]:
 * K arrays of n.  The VJP records the fold on the tape, seeds every y_i with
 * y_bar_i and sweeps in reverse. */
int orc_scan_generic(int op, int64_t n, const double* const* x, double* const* y);
/* The same started from the state init (K values; NULL: neutral). */
int orc_scan_generic_from(int op, int64_t n, const double* init, const double* const* x, double* const* y);
int orc_scan_generic_vjp(int op, int64_t n, const double* const* x, const double* const* y_bar,
                         double* const* x_bar);
/* The same with the fold started from the constant state init (K values;
 * NULL: the neutral element): y_i = init (.) x_0 (.) ... (.) x_i.  With init
 * the fold of the elements before a window, this gives the exact adjoints of
 * the window's elements for the window's output adjoints. */
int orc_scan_generic_vjp_from(int op, int64_t n, const double* init, const double* const* x,
                              const double* const* y_bar, double* const* x_bar);

/* Forward mode (Sec. 3): Jacobian-vector products by a forward sweep over
 * the same tape records (tan[out] = sum of partial * tan[in] in record
 * order).  Outputs: the tangents of the primal outputs (for hist: hs_dot[m],
 * 0 for an empty bin; for the general operators: K values or K arrays). */
int orc_reduce_jvp(int op, int64_t n, const double* x, const double* x_dot, double* y_dot);
int orc_hist_jvp(int op, int64_t n, int64_t m, const int32_t* inds, const double* vs,
                 const double* vs_dot, double* hs_dot);
int orc_scatter_jvp(int64_t n, const double* xs_dot, int64_t m, const int32_t* is, const double* vs_dot,
                    double* ys_dot);
int orc_map_jvp(int fn, int64_t n, const double* x, const double* x_dot, double* y_dot);
int orc_reduce_generic_jvp(int op, int64_t n, const double* const* x, const double* const* x_dot,
                           double* y_dot);
int orc_scan_generic_jvp(int op, int64_t n, const double* const* x, const double* const* x_dot,
                         double* const* y_dot);
/* The same with the fold started from the constant state init (tangent 0). */
int orc_scan_generic_jvp_from(int op, int64_t n, const double* init, const double* const* x,
                              const double* const* x_dot, double* const* y_dot);

/* Dense k-means (Sec. 7.4) with the squared distance: f(C) = sum_i
 * min_k |x_i - c_k|^2; X [N x D], C [K x D] row-major.  Distances are the
 * FP64 chain acc = fma(x_d - c_d, x_d - c_d, acc), d = 0..D-1; ties go to the
 * lowest k.  assign (nullable) [N].  The VJP tapes each point's term
 * separately (f is a sum of per-point terms); the jvp of the VJP in
 * direction C_dot (the Hessian-vector product) is the unit-step central
 * difference of the gradient at fixed assignments, exact for a quadratic. */
int orc_kmeans_objective(int64_t N, int D, int K, const double* X, const double* C, int32_t* assign,
                         double* f);
int orc_kmeans_vjp(int64_t N, int D, int K, const double* X, const double* C, double f_bar, double* C_bar);
int orc_kmeans_hvp(int64_t N, int D, int K, const double* X, const double* C, double f_bar,
                   const double* C_dot, double* out);

/* A map whose body reads a free array at computed indices (Sec. 5.4):
 * ys[i] = f(as[is[i]], vs[i]) with op 0: f = a (vs unused, may be NULL),
 * 1: a v, 2: (a - v)^2.  An index outside [0, n) reads 0.  The VJP returns
 * as_bar (every read's partial accumulated into its element) and vs_bar (not
 * written for op 0). */
int orc_gather_map(int op, int64_t n, const double* as, int64_t m, const int32_t* is, const double* vs,
                   double* ys);
int orc_gather_map_vjp(int op, int64_t n, const double* as, int64_t m, const int32_t* is, const double* vs,
                       const double* ys_bar, double* as_bar, double* vs_bar);

/* Sparse k-means (Sec. 7.5): CSR points (rowptr [N+1] int64, col [nnz] int32,
 * val [nnz]), dense centres C [K x D].  The distance of a row to a centre is
 * the plain squared distance of the densified row, summed over d = 0..D-1 in
 * order; ties to the lowest k.  The VJP is 2 f_bar (n_k c_k - S_k) at fixed
 * assignments, the jvp of the VJP 2 f_bar n_k C_dot_k.  orc_skm_dist gives
 * every distance, dist [N x K]. */
int orc_skm_dist(int64_t N, int64_t D, int K, const int64_t* rowptr, const int32_t* col, const double* val,
                 const double* C, double* dist);
int orc_skm_objective(int64_t N, int64_t D, int K, const int64_t* rowptr, const int32_t* col, const double* val,
                      const double* C, int32_t* assign, double* f);
int orc_skm_vjp(int64_t N, int64_t D, int K, const int64_t* rowptr, const int32_t* col, const double* val,
                const double* C, double f_bar, double* C_bar);
int orc_skm_hvp(int64_t N, int64_t D, int K, const int64_t* rowptr, const int32_t* col, const double* val,
                const double* C, double f_bar, const double* C_dot, double* out);

/* reduce_by_index with a general operator (Sec. 5.1.2 with the general rule
 * of Sec. 5.1.1 per bin): hs[c][b] = the index-order fold of the elements of
 * bin b (the neutral element if none); inds outside [0, m) skipped (their
 * adjoint 0).  K component arrays for x, hs, hs_bar, x_bar. */
int orc_hist_generic(int op, int64_t n, int64_t m, const int32_t* inds, const double* const* x,
                     double* const* hs);
int orc_hist_generic_vjp(int op, int64_t n, int64_t m, const int32_t* inds, const double* const* x,
                         const double* const* hs_bar, double* const* x_bar);

#ifdef __cplusplus
}
#endif
#endif
