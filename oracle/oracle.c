/*
 * CPU oracle: sequential FP64 semantics + explicit tape + reverse sweep.
 *
 * TEST INFRASTRUCTURE ONLY (see oracle.h).  Plain C99, libm only, single
 * thread.  It is meant to be slow and easy to check by eye, not fast.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* 2*pi to double precision. */
static const double TWO_PI = 6.283185307179586476925286766559;

/* ------------------------------------------------------------------------ */
/* The tape.                                                                  */
/*                                                                            */
/* A variable is a slot holding a value and an adjoint.  Every elementary     */
/* step v = f(a, b) appends one record {v, a, b, df/da, df/db} with the local */
/* partial derivatives evaluated at the forward point (Sec. 2.0.2).  The      */
/* reverse sweep visits the records newest-first and applies                  */
/* adj[a] += df/da * adj[v], adj[b] += df/db * adj[v]; a variable used many   */
/* times therefore receives the sum of all its contributions.                 */
/* ------------------------------------------------------------------------ */

typedef struct {
    int64_t out, in0, in1; /* in1 == -1 for unary steps */
    double w0, w1;         /* partials of out w.r.t. in0 and in1 */
} rec_t;

typedef struct {
    double* val;
    double* adj;
    int64_t nv, capv;
    rec_t* rec;
    int64_t nr, capr;
    int oom;
} tape_t;

static int tape_init(tape_t* t, int64_t capv, int64_t capr) {
    memset(t, 0, sizeof(*t));
    if (capv < 16) capv = 16;
    if (capr < 16) capr = 16;
    t->val = (double*)malloc((size_t)capv * sizeof(double));
    t->rec = (rec_t*)malloc((size_t)capr * sizeof(rec_t));
    t->capv = capv;
    t->capr = capr;
    if (!t->val || !t->rec) {
        free(t->val);
        free(t->rec);
        t->val = NULL;
        t->rec = NULL;
        return -2;
    }
    return 0;
}

static void tape_free(tape_t* t) {
    free(t->val);
    free(t->adj);
    free(t->rec);
    memset(t, 0, sizeof(*t));
}

static void tape_clear(tape_t* t) {
    t->nv = 0;
    t->nr = 0;
}

static int64_t new_slot(tape_t* t, double v) {
    if (t->nv == t->capv) {
        int64_t c = t->capv * 2;
        double* p = (double*)realloc(t->val, (size_t)c * sizeof(double));
        if (!p) {
            t->oom = 1;
            return 0;
        }
        t->val = p;
        t->capv = c;
    }
    t->val[t->nv] = v;
    return t->nv++;
}

static void push_rec(tape_t* t, int64_t out, int64_t a, double wa, int64_t b, double wb) {
    if (t->nr == t->capr) {
        int64_t c = t->capr * 2;
        rec_t* p = (rec_t*)realloc(t->rec, (size_t)c * sizeof(rec_t));
        if (!p) {
            t->oom = 1;
            return;
        }
        t->rec = p;
        t->capr = c;
    }
    rec_t* r = &t->rec[t->nr++];
    r->out = out;
    r->in0 = a;
    r->in1 = b;
    r->w0 = wa;
    r->w1 = wb;
}

#define V(s) (t->val[(s)])

/* An independent variable (or a constant whose adjoint is simply ignored). */
static int64_t leaf(tape_t* t, double v) { return new_slot(t, v); }

static int64_t emit1(tape_t* t, double v, int64_t a, double wa) {
    int64_t s = new_slot(t, v);
    push_rec(t, s, a, wa, -1, 0.0);
    return s;
}

static int64_t emit2(tape_t* t, double v, int64_t a, double wa, int64_t b, double wb) {
    int64_t s = new_slot(t, v);
    push_rec(t, s, a, wa, b, wb);
    return s;
}

/* Elementary steps with their textbook partial derivatives. */
static int64_t t_add(tape_t* t, int64_t a, int64_t b) { return emit2(t, V(a) + V(b), a, 1.0, b, 1.0); }
static int64_t t_sub(tape_t* t, int64_t a, int64_t b) { return emit2(t, V(a) - V(b), a, 1.0, b, -1.0); }
static int64_t t_mul(tape_t* t, int64_t a, int64_t b) {
    double va = V(a), vb = V(b);
    return emit2(t, va * vb, a, vb, b, va);
}
static int64_t t_scale(tape_t* t, int64_t a, double c) { return emit1(t, c * V(a), a, c); }
static int64_t t_exp(tape_t* t, int64_t a) {
    double e = exp(V(a));
    return emit1(t, e, a, e);
}
static int64_t t_log(tape_t* t, int64_t a) {
    double va = V(a);
    return emit1(t, log(va), a, 1.0 / va);
}
static int64_t t_sin(tape_t* t, int64_t a) {
    double va = V(a);
    return emit1(t, sin(va), a, cos(va));
}
static int64_t t_tanh(tape_t* t, int64_t a) {
    double y = tanh(V(a));
    return emit1(t, y, a, 1.0 - y * y);
}
/* A selection: the result is a copy of whichever operand was chosen, so the
 * whole adjoint flows to that operand (min/max, Sec. 5.1.1). */
static int64_t t_pick(tape_t* t, int64_t a, int64_t b, int take_b) {
    return take_b ? emit1(t, V(b), b, 1.0) : emit1(t, V(a), a, 1.0);
}

static int tape_reverse(tape_t* t) {
    free(t->adj);
    t->adj = (double*)calloc((size_t)(t->nv > 0 ? t->nv : 1), sizeof(double));
    return t->adj ? 0 : -2;
}

/* Seeds must be placed after tape_reverse() allocated adj and before sweep(). */
static void sweep(tape_t* t) {
    for (int64_t r = t->nr - 1; r >= 0; --r) {
        const rec_t* q = &t->rec[r];
        double g = t->adj[q->out];
        if (g == 0.0) continue; /* exact: contributions would be +-0 */
        t->adj[q->in0] += q->w0 * g;
        if (q->in1 >= 0) t->adj[q->in1] += q->w1 * g;
    }
}

/* ------------------------------------------------------------------------ */
/* Linear-recurrence inclusive scan (Sec. 5.2).                               */
/* rs[0] = as[0]; rs[i] = rs[i-1] (+) as[i], with                             */
/* (A, B) (+) (a, b) = (a*A, a*B + b).                                        */
/* ------------------------------------------------------------------------ */

int orc_linrec_scan(int64_t n, const double* a, const double* b, double* A, double* B) {
    if (n < 0 || (n > 0 && (!a || !b || !A || !B))) return -1;
    for (int64_t i = 0; i < n; ++i) {
        if (i == 0) {
            A[0] = a[0];
            B[0] = b[0];
        } else {
            A[i] = a[i] * A[i - 1];
            B[i] = a[i] * B[i - 1] + b[i];
        }
    }
    return 0;
}

int orc_linrec_scan_vjp(int64_t n, const double* a, const double* b,
                        const double* yA_bar, const double* yB_bar,
                        double* a_bar, double* b_bar) {
    if (n < 0 || (n > 0 && (!a || !b || !yA_bar || !yB_bar || !a_bar || !b_bar))) return -1;
    if (n == 0) return 0;
    tape_t T, *t = &T;
    if (tape_init(t, 5 * n + 16, 3 * n + 16)) return -2;
    int64_t* sa = (int64_t*)malloc((size_t)n * sizeof(int64_t));
    int64_t* sb = (int64_t*)malloc((size_t)n * sizeof(int64_t));
    int64_t* sA = (int64_t*)malloc((size_t)n * sizeof(int64_t));
    int64_t* sB = (int64_t*)malloc((size_t)n * sizeof(int64_t));
    int rc = 0;
    if (!sa || !sb || !sA || !sB) {
        rc = -2;
        goto done;
    }
    for (int64_t i = 0; i < n; ++i) {
        sa[i] = leaf(t, a[i]);
        sb[i] = leaf(t, b[i]);
    }
    for (int64_t i = 0; i < n; ++i) {
        if (i == 0) { /* rs[0] = as[0]: the same variables */
            sA[0] = sa[0];
            sB[0] = sb[0];
        } else {
            sA[i] = t_mul(t, sa[i], sA[i - 1]);
            sB[i] = t_add(t, t_mul(t, sa[i], sB[i - 1]), sb[i]);
        }
    }
    if (t->oom || tape_reverse(t)) {
        rc = -2;
        goto done;
    }
    for (int64_t i = 0; i < n; ++i) { /* += : A[0] aliases a[0] */
        t->adj[sA[i]] += yA_bar[i];
        t->adj[sB[i]] += yB_bar[i];
    }
    sweep(t);
    for (int64_t i = 0; i < n; ++i) {
        a_bar[i] = t->adj[sa[i]];
        b_bar[i] = t->adj[sb[i]];
    }
done:
    free(sa);
    free(sb);
    free(sA);
    free(sB);
    tape_free(t);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* reduce (Sec. 5.1): y = e; for i: y = y (+) x[i].                           */
/* For min/max the first element of the array always replaces the neutral    */
/* element and a later element replaces y only when strictly better, so the   */
/* adjoint goes to the lowest index attaining the extreme (Sec. 5.1.1).       */
/* ------------------------------------------------------------------------ */

static double neutral(int op) {
    switch (op) {
        case ORC_ADD: return 0.0;
        case ORC_MUL: return 1.0;
        case ORC_MIN: return INFINITY;
        default: return -INFINITY;
    }
}

static int better(int op, double v, double cur) { return op == ORC_MAX ? (v > cur) : (v < cur); }

int orc_reduce(int op, int64_t n, const double* x, double* y, int64_t* arg,
               double* p, int64_t* z) {
    if (op < ORC_ADD || op > ORC_MAX || n < 0 || (n > 0 && !x) || !y) return -1;
    double acc = neutral(op);
    int64_t best = -1;
    double prod_nz = 1.0;
    int64_t zeros = 0;
    for (int64_t i = 0; i < n; ++i) {
        switch (op) {
            case ORC_ADD: acc = acc + x[i]; break;
            case ORC_MUL:
                acc = acc * x[i];
                if (x[i] == 0.0)
                    zeros++;
                else
                    prod_nz *= x[i];
                break;
            default:
                if (best < 0 || better(op, x[i], acc)) {
                    acc = x[i];
                    best = i;
                }
        }
    }
    *y = acc;
    if (arg) *arg = best;
    if (p) *p = prod_nz;
    if (z) *z = zeros;
    return 0;
}

int orc_reduce_vjp(int op, int64_t n, const double* x, double y_bar, double* x_bar) {
    if (op < ORC_ADD || op > ORC_MAX || n < 0 || (n > 0 && (!x || !x_bar))) return -1;
    if (n == 0) return 0;
    tape_t T, *t = &T;
    if (tape_init(t, 2 * n + 16, n + 16)) return -2;
    int64_t* sx = (int64_t*)malloc((size_t)n * sizeof(int64_t));
    if (!sx) {
        tape_free(t);
        return -2;
    }
    for (int64_t i = 0; i < n; ++i) sx[i] = leaf(t, x[i]);
    int64_t y = leaf(t, neutral(op)); /* the neutral element: a constant */
    int first = 1;
    for (int64_t i = 0; i < n; ++i) {
        switch (op) {
            case ORC_ADD: y = t_add(t, y, sx[i]); break;
            case ORC_MUL: y = t_mul(t, y, sx[i]); break;
            default: y = t_pick(t, y, sx[i], first || better(op, x[i], V(y)));
        }
        first = 0;
    }
    int rc = (t->oom || tape_reverse(t)) ? -2 : 0;
    if (!rc) {
        t->adj[y] += y_bar;
        sweep(t);
        for (int64_t i = 0; i < n; ++i) x_bar[i] = t->adj[sx[i]];
    }
    free(sx);
    tape_free(t);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* reduce_by_index (Sec. 5.1.2):                                               */
/* hs = replicate m e; for i in 0..n-1: hs[inds[i]] (+)= vs[i].               */
/* The first element of a bin replaces the neutral element exactly (e (+) v   */
/* == v for all four operators), so a bin's variable is that element's.       */
/* ------------------------------------------------------------------------ */

int orc_hist(int op, int64_t n, int64_t m, const int32_t* inds, const double* vs,
             double* hs, int64_t* winner, double* p, int64_t* z, int64_t* count) {
    if (op < ORC_ADD || op > ORC_MAX || n < 0 || m < 0 || (n > 0 && (!inds || !vs))) return -1;
    for (int64_t k = 0; k < m; ++k) {
        if (hs) hs[k] = neutral(op);
        if (winner) winner[k] = -1;
        if (p) p[k] = 1.0;
        if (z) z[k] = 0;
        if (count) count[k] = 0;
    }
    int64_t* cnt = (int64_t*)calloc((size_t)(m > 0 ? m : 1), sizeof(int64_t));
    double* h = (double*)malloc((size_t)(m > 0 ? m : 1) * sizeof(double));
    if (!cnt || !h) {
        free(cnt);
        free(h);
        return -2;
    }
    for (int64_t k = 0; k < m; ++k) h[k] = neutral(op);
    for (int64_t i = 0; i < n; ++i) {
        int64_t k = inds[i];
        if (k < 0 || k >= m) continue;
        double v = vs[i];
        switch (op) {
            case ORC_ADD: h[k] = h[k] + v; break;
            case ORC_MUL:
                h[k] = h[k] * v;
                if (v == 0.0) {
                    if (z) z[k]++;
                } else if (p) {
                    p[k] *= v;
                }
                break;
            default:
                if (cnt[k] == 0 || better(op, v, h[k])) {
                    h[k] = v;
                    if (winner) winner[k] = i;
                }
        }
        cnt[k]++;
    }
    for (int64_t k = 0; k < m; ++k) {
        if (hs) hs[k] = h[k];
        if (count) count[k] = cnt[k];
    }
    free(cnt);
    free(h);
    return 0;
}

int orc_hist_vjp(int op, int64_t n, int64_t m, const int32_t* inds, const double* vs,
                 const double* hs_bar, double* vs_bar) {
    if (op < ORC_ADD || op > ORC_MAX || n < 0 || m < 0 ||
        (n > 0 && (!inds || !vs || !vs_bar)) || (m > 0 && !hs_bar))
        return -1;
    if (n == 0) return 0;
    tape_t T, *t = &T;
    if (tape_init(t, 2 * n + 16, n + 16)) return -2;
    int64_t* sv = (int64_t*)malloc((size_t)n * sizeof(int64_t));
    int64_t* sh = (int64_t*)malloc((size_t)(m > 0 ? m : 1) * sizeof(int64_t));
    if (!sv || !sh) {
        free(sv);
        free(sh);
        tape_free(t);
        return -2;
    }
    for (int64_t i = 0; i < n; ++i) sv[i] = leaf(t, vs[i]);
    for (int64_t k = 0; k < m; ++k) sh[k] = -1; /* empty bin: still the constant e */
    for (int64_t i = 0; i < n; ++i) {
        int64_t k = inds[i];
        if (k < 0 || k >= m) continue;
        if (sh[k] < 0) {
            sh[k] = sv[i];
            continue;
        }
        switch (op) {
            case ORC_ADD: sh[k] = t_add(t, sh[k], sv[i]); break;
            case ORC_MUL: sh[k] = t_mul(t, sh[k], sv[i]); break;
            default: sh[k] = t_pick(t, sh[k], sv[i], better(op, vs[i], V(sh[k])));
        }
    }
    int rc = (t->oom || tape_reverse(t)) ? -2 : 0;
    if (!rc) {
        for (int64_t k = 0; k < m; ++k)
            if (sh[k] >= 0) t->adj[sh[k]] += hs_bar[k];
        sweep(t);
        for (int64_t i = 0; i < n; ++i) vs_bar[i] = t->adj[sv[i]];
    }
    free(sv);
    free(sh);
    tape_free(t);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* scatter (Sec. 5.3): ys = xs; for j: ys[is[j]] = vs[j].                     */
/* An assignment makes ys[k] the very variable vs[j]; the tape needs no       */
/* records, only the map from output positions to variables.                  */
/* ------------------------------------------------------------------------ */

int orc_scatter(int64_t n, const double* xs, int64_t m, const int32_t* is,
                const double* vs, double* ys, double* xs_saved) {
    if (n < 0 || m < 0 || (n > 0 && (!xs || !ys)) || (m > 0 && (!is || !vs))) return -1;
    for (int64_t k = 0; k < n; ++k) ys[k] = xs[k];
    for (int64_t j = 0; j < m; ++j) {
        int64_t k = is[j];
        int ok = (k >= 0 && k < n);
        if (xs_saved) xs_saved[j] = ok ? xs[k] : 0.0;
        if (ok) ys[k] = vs[j];
    }
    return 0;
}

int orc_scatter_vjp(int64_t n, int64_t m, const int32_t* is, const double* ys_bar,
                    double* xs_bar, double* vs_bar) {
    if (n < 0 || m < 0 || (n > 0 && (!ys_bar || !xs_bar)) || (m > 0 && (!is || !vs_bar))) return -1;
    tape_t T, *t = &T;
    if (tape_init(t, n + m + 16, 16)) return -2;
    int64_t* out = (int64_t*)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
    if (!out) {
        tape_free(t);
        return -2;
    }
    int64_t x0 = t->nv;
    for (int64_t k = 0; k < n; ++k) out[k] = leaf(t, 0.0); /* xs variables */
    int64_t v0 = t->nv;
    for (int64_t j = 0; j < m; ++j) leaf(t, 0.0); /* vs variables */
    for (int64_t j = 0; j < m; ++j) {
        int64_t k = is[j];
        if (k >= 0 && k < n) out[k] = v0 + j;
    }
    int rc = (t->oom || tape_reverse(t)) ? -2 : 0;
    if (!rc) {
        for (int64_t k = 0; k < n; ++k) t->adj[out[k]] += ys_bar[k];
        sweep(t);
        for (int64_t k = 0; k < n; ++k) xs_bar[k] = t->adj[x0 + k];
        for (int64_t j = 0; j < m; ++j) vs_bar[j] = t->adj[v0 + j];
    }
    free(out);
    tape_free(t);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* map (Sec. 5.4).  Each element is an independent small program.           */
/* ------------------------------------------------------------------------ */

static int64_t apply_fn(tape_t* t, int fn, int64_t x) {
    switch (fn) {
        case ORC_FN_SQUARE: return t_mul(t, x, x);
        case ORC_FN_EXP: return t_exp(t, x);
        case ORC_FN_LOG: return t_log(t, x);
        case ORC_FN_SIN: return t_sin(t, x);
        default: return t_tanh(t, x);
    }
}

int orc_map(int fn, int64_t n, const double* x, double* y) {
    if (fn < ORC_FN_SQUARE || fn > ORC_FN_TANH || n < 0 || (n > 0 && (!x || !y))) return -1;
    tape_t T, *t = &T;
    if (tape_init(t, 16, 16)) return -2;
    for (int64_t i = 0; i < n; ++i) {
        tape_clear(t);
        y[i] = V(apply_fn(t, fn, leaf(t, x[i])));
    }
    tape_free(t);
    return 0;
}

int orc_map_vjp(int fn, int64_t n, const double* x, const double* y_bar, double* x_bar) {
    if (fn < ORC_FN_SQUARE || fn > ORC_FN_TANH || n < 0 || (n > 0 && (!x || !y_bar || !x_bar)))
        return -1;
    tape_t T, *t = &T;
    if (tape_init(t, 16, 16)) return -2;
    for (int64_t i = 0; i < n; ++i) {
        tape_clear(t);
        int64_t xs = leaf(t, x[i]);
        int64_t ys = apply_fn(t, fn, xs);
        if (tape_reverse(t)) {
            tape_free(t);
            return -2;
        }
        t->adj[ys] += y_bar[i];
        sweep(t);
        x_bar[i] = t->adj[xs];
    }
    tape_free(t);
    return 0;
}

/* Fig. 1(a): v0 = sin(x0); v1 = x1 * v0; v2 = x0 * x1; (y0, y1) = (v1, v2). */
static void fig1_program(tape_t* t, int64_t x0, int64_t x1, int64_t* y0, int64_t* y1) {
    int64_t v0 = t_sin(t, x0);
    int64_t v1 = t_mul(t, x1, v0);
    int64_t v2 = t_mul(t, x0, x1);
    *y0 = v1;
    *y1 = v2;
}

int orc_fig1(int64_t n, const double* x0, const double* x1, double* y0, double* y1) {
    if (n < 0 || (n > 0 && (!x0 || !x1 || !y0 || !y1))) return -1;
    tape_t T, *t = &T;
    if (tape_init(t, 16, 16)) return -2;
    for (int64_t i = 0; i < n; ++i) {
        tape_clear(t);
        int64_t a = leaf(t, x0[i]), b = leaf(t, x1[i]), r0, r1;
        fig1_program(t, a, b, &r0, &r1);
        y0[i] = V(r0);
        y1[i] = V(r1);
    }
    tape_free(t);
    return 0;
}

int orc_fig1_vjp(int64_t n, const double* x0, const double* x1,
                 const double* y0_bar, const double* y1_bar,
                 double* x0_bar, double* x1_bar) {
    if (n < 0 || (n > 0 && (!x0 || !x1 || !y0_bar || !y1_bar || !x0_bar || !x1_bar))) return -1;
    tape_t T, *t = &T;
    if (tape_init(t, 16, 16)) return -2;
    for (int64_t i = 0; i < n; ++i) {
        tape_clear(t);
        int64_t a = leaf(t, x0[i]), b = leaf(t, x1[i]), r0, r1;
        fig1_program(t, a, b, &r0, &r1);
        if (tape_reverse(t)) {
            tape_free(t);
            return -2;
        }
        t->adj[r0] += y0_bar[i];
        t->adj[r1] += y1_bar[i];
        sweep(t);
        x0_bar[i] = t->adj[a];
        x1_bar[i] = t->adj[b];
    }
    tape_free(t);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Gaussian mixture (the objective is stated in oracle.h).                    */
/* ------------------------------------------------------------------------ */

/* log-sum-exp of the variables s[0..K-1]: mx + log(sum_k exp(s_k - mx)).
 * The shift mx = max_k s_k enters as a constant: the derivative of LSE does
 * not depend on the shift. */
static int64_t t_lse(tape_t* t, const int64_t* s, int K) {
    double mx = -INFINITY;
    for (int k = 0; k < K; ++k)
        if (V(s[k]) > mx) mx = V(s[k]);
    int64_t c = leaf(t, mx);
    int64_t acc = -1;
    for (int k = 0; k < K; ++k) {
        int64_t e = t_exp(t, t_sub(t, s[k], c));
        acc = (acc < 0) ? e : t_add(t, acc, e);
    }
    return t_add(t, t_log(t, acc), c);
}

typedef struct {
    int64_t *alpha, *mu, *q, *l; /* parameter variables */
} gmm_slots;

/* Records the point term LSE_k(s_ik) of point x (length D); returns its slot. */
static int64_t gmm_point(tape_t* t, int D, int K, const double* x, const gmm_slots* P,
                         int64_t* s /* K scratch */) {
    const int64_t tri = (int64_t)D * (D - 1) / 2;
    int64_t* y = (int64_t*)malloc((size_t)D * sizeof(int64_t));
    int64_t* ed = (int64_t*)malloc((size_t)D * sizeof(int64_t));
    if (!y || !ed) {
        free(y);
        free(ed);
        t->oom = 1;
        return 0;
    }
    for (int k = 0; k < K; ++k) {
        for (int d = 0; d < D; ++d) {
            y[d] = t_sub(t, leaf(t, x[d]), P->mu[(int64_t)k * D + d]); /* y = x - mu_k */
            ed[d] = t_exp(t, P->q[(int64_t)k * D + d]);                /* diag of Q_k */
        }
        int64_t sq = -1;
        for (int r = 0; r < D; ++r) { /* z_r = exp(q_kr) y_r + sum_{c<r} L_rc y_c */
            int64_t z = t_mul(t, ed[r], y[r]);
            for (int c = 0; c < r; ++c)
                z = t_add(t, z, t_mul(t, P->l[(int64_t)k * tri + (int64_t)r * (r - 1) / 2 + c], y[c]));
            int64_t z2 = t_mul(t, z, z);
            sq = (sq < 0) ? z2 : t_add(t, sq, z2);
        }
        int64_t sumq = P->q[(int64_t)k * D];
        for (int d = 1; d < D; ++d) sumq = t_add(t, sumq, P->q[(int64_t)k * D + d]);
        s[k] = t_sub(t, t_add(t, P->alpha[k], sumq), t_scale(t, sq, 0.5));
    }
    free(y);
    free(ed);
    return t_lse(t, s, K);
}

static int gmm_make_leaves(tape_t* t, int D, int K, const double* alpha, const double* mu,
                           const double* q, const double* l, gmm_slots* P) {
    const int64_t tri = (int64_t)D * (D - 1) / 2;
    P->alpha = (int64_t*)malloc((size_t)K * sizeof(int64_t));
    P->mu = (int64_t*)malloc((size_t)K * D * sizeof(int64_t));
    P->q = (int64_t*)malloc((size_t)K * D * sizeof(int64_t));
    P->l = (int64_t*)malloc((size_t)(K * tri > 0 ? K * tri : 1) * sizeof(int64_t));
    if (!P->alpha || !P->mu || !P->q || !P->l) return -2;
    for (int k = 0; k < K; ++k) P->alpha[k] = leaf(t, alpha[k]);
    for (int64_t j = 0; j < (int64_t)K * D; ++j) P->mu[j] = leaf(t, mu[j]);
    for (int64_t j = 0; j < (int64_t)K * D; ++j) P->q[j] = leaf(t, q[j]);
    for (int64_t j = 0; j < (int64_t)K * tri; ++j) P->l[j] = leaf(t, l[j]);
    return t->oom ? -2 : 0;
}

static void gmm_free_leaves(gmm_slots* P) {
    free(P->alpha);
    free(P->mu);
    free(P->q);
    free(P->l);
}

static int gmm_args_ok(int64_t N, int D, int K, const double* X, const double* alpha,
                       const double* mu, const double* q, const double* l) {
    if (N < 0 || D < 1 || K < 1) return 0;
    if (!alpha || !mu || !q || (D > 1 && !l) || (N > 0 && !X)) return 0;
    return 1;
}

int orc_gmm_objective(int64_t N, int D, int K, const double* X, const double* alpha,
                      const double* mu, const double* q, const double* l,
                      double* loglik, double* lse) {
    if (!gmm_args_ok(N, D, K, X, alpha, mu, q, l) || !loglik) return -1;
    tape_t T, *t = &T;
    if (tape_init(t, 1 << 16, 1 << 16)) return -2;
    int64_t* s = (int64_t*)malloc((size_t)K * sizeof(int64_t));
    gmm_slots P = {0, 0, 0, 0};
    int rc = s ? 0 : -2;
    double total = 0.0;
    for (int64_t i = 0; i < N && !rc; ++i) {
        tape_clear(t);
        if ((rc = gmm_make_leaves(t, D, K, alpha, mu, q, l, &P))) break;
        int64_t r = gmm_point(t, D, K, X + i * D, &P, s);
        gmm_free_leaves(&P);
        if (t->oom) {
            rc = -2;
            break;
        }
        if (lse) lse[i] = V(r);
        total += V(r);
    }
    if (!rc) {
        tape_clear(t);
        if (!(rc = gmm_make_leaves(t, D, K, alpha, mu, q, l, &P))) {
            double la = V(t_lse(t, P.alpha, K));
            *loglik = total - (double)N * la - 0.5 * (double)N * D * log(TWO_PI);
        }
        gmm_free_leaves(&P);
    }
    free(s);
    tape_free(t);
    return rc;
}

int orc_gmm_vjp(int64_t N, int D, int K, const double* X, const double* alpha,
                const double* mu, const double* q, const double* l, double ell_bar,
                double* alpha_bar, double* mu_bar, double* q_bar, double* l_bar) {
    if (!gmm_args_ok(N, D, K, X, alpha, mu, q, l) || !alpha_bar || !mu_bar || !q_bar ||
        (D > 1 && !l_bar))
        return -1;
    const int64_t tri = (int64_t)D * (D - 1) / 2;
    memset(alpha_bar, 0, (size_t)K * sizeof(double));
    memset(mu_bar, 0, (size_t)K * D * sizeof(double));
    memset(q_bar, 0, (size_t)K * D * sizeof(double));
    if (tri > 0) memset(l_bar, 0, (size_t)(K * tri) * sizeof(double));
    tape_t T, *t = &T;
    if (tape_init(t, 1 << 16, 1 << 16)) return -2;
    int64_t* s = (int64_t*)malloc((size_t)K * sizeof(int64_t));
    gmm_slots P = {0, 0, 0, 0};
    int rc = s ? 0 : -2;
    /* One tape per point term (each point's LSE is its own small program), plus
     * one for the -N * LSE(alpha) term.  Parameter adjoints are summed. */
    for (int64_t i = 0; i <= N && !rc; ++i) {
        tape_clear(t);
        if ((rc = gmm_make_leaves(t, D, K, alpha, mu, q, l, &P))) break;
        int64_t r;
        double seed;
        if (i < N) {
            r = gmm_point(t, D, K, X + i * D, &P, s);
            seed = ell_bar;
        } else {
            r = t_lse(t, P.alpha, K);
            seed = -(double)N * ell_bar;
        }
        if (t->oom || tape_reverse(t)) {
            rc = -2;
            gmm_free_leaves(&P);
            break;
        }
        t->adj[r] += seed;
        sweep(t);
        for (int k = 0; k < K; ++k) alpha_bar[k] += t->adj[P.alpha[k]];
        for (int64_t j = 0; j < (int64_t)K * D; ++j) {
            mu_bar[j] += t->adj[P.mu[j]];
            q_bar[j] += t->adj[P.q[j]];
        }
        for (int64_t j = 0; j < (int64_t)K * tri; ++j) l_bar[j] += t->adj[P.l[j]];
        gmm_free_leaves(&P);
    }
    free(s);
    tape_free(t);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* reduce with a general associative operator (Sec. 5.1.1): the left fold     */
/* acc = e; acc = acc (.) x_i for i = 0..n-1.  Each operator step is written  */
/* out of elementary steps; the VJP records them on the tape.                 */
/* ------------------------------------------------------------------------ */

int orc_gop_components(int op) {
    switch (op) {
        case ORC_GOP_LOGADDEXP: return 1;
        case ORC_GOP_LINREC: return 2;
        case ORC_GOP_MAT2: return 4;
        default: return 0;
    }
}

static void gop_neutral(int op, double* e) {
    switch (op) {
        case ORC_GOP_LOGADDEXP: e[0] = -INFINITY; break;
        case ORC_GOP_LINREC: e[0] = 1.0, e[1] = 0.0; break;
        default: e[0] = 1.0, e[1] = 0.0, e[2] = 0.0, e[3] = 1.0;
    }
}

/* out = l (.) r on plain values (out may alias l or r). */
static void gop_comb(int op, const double* l, const double* r, double* out) {
    double o[4];
    switch (op) {
        case ORC_GOP_LOGADDEXP:
            /* over the extended reals: -inf is the neutral element, NaN
             * propagates, and e^(+inf) = +inf absorbs the other term */
            if (r[0] == -INFINITY) o[0] = l[0];
            else if (l[0] == -INFINITY) o[0] = r[0];
            else if (isnan(l[0]) || isnan(r[0])) o[0] = l[0] + r[0];
            else if (l[0] == INFINITY || r[0] == INFINITY) o[0] = INFINITY;
            else {
                double m = l[0] > r[0] ? l[0] : r[0];
                o[0] = m + log(exp(l[0] - m) + exp(r[0] - m));
            }
            break;
        case ORC_GOP_LINREC:
            o[0] = r[0] * l[0];
            o[1] = r[0] * l[1] + r[1];
            break;
        default:
            o[0] = l[0] * r[0] + l[1] * r[2];
            o[1] = l[0] * r[1] + l[1] * r[3];
            o[2] = l[2] * r[0] + l[3] * r[2];
            o[3] = l[2] * r[1] + l[3] * r[3];
    }
    for (int c = 0; c < orc_gop_components(op); ++c) out[c] = o[c];
}

/* Records out = l (.) r on the tape (slot arrays of K entries). */
static void gop_step(tape_t* t, int op, const int64_t* l, const int64_t* r, int64_t* out) {
    int64_t o[4];
    switch (op) {
        case ORC_GOP_LOGADDEXP:
            if (V(r[0]) == -INFINITY) o[0] = l[0]; /* r contributes nothing */
            else if (V(l[0]) == -INFINITY) o[0] = r[0];
            else if (!isnan(V(l[0])) && !isnan(V(r[0])) && (V(l[0]) == INFINITY || V(r[0]) == INFINITY))
                o[0] = t_pick(t, l[0], r[0], V(l[0]) != INFINITY); /* the +inf operand absorbs the other */
            else {
                /* the shift m is a constant: d/da log(e^(a-m) + e^(b-m)) + m
                 * does not depend on it */
                int64_t m = leaf(t, V(l[0]) > V(r[0]) ? V(l[0]) : V(r[0]));
                int64_t s = t_add(t, t_exp(t, t_sub(t, l[0], m)), t_exp(t, t_sub(t, r[0], m)));
                o[0] = t_add(t, t_log(t, s), m);
            }
            break;
        case ORC_GOP_LINREC:
            o[0] = t_mul(t, r[0], l[0]);
            o[1] = t_add(t, t_mul(t, r[0], l[1]), r[1]);
            break;
        default:
            o[0] = t_add(t, t_mul(t, l[0], r[0]), t_mul(t, l[1], r[2]));
            o[1] = t_add(t, t_mul(t, l[0], r[1]), t_mul(t, l[1], r[3]));
            o[2] = t_add(t, t_mul(t, l[2], r[0]), t_mul(t, l[3], r[2]));
            o[3] = t_add(t, t_mul(t, l[2], r[1]), t_mul(t, l[3], r[3]));
    }
    for (int c = 0; c < orc_gop_components(op); ++c) out[c] = o[c];
}

static int gop_args_ok(int op, int64_t n, const double* const* x) {
    int K = orc_gop_components(op);
    if (K == 0 || n < 0) return 0;
    if (n > 0) {
        if (!x) return 0;
        for (int c = 0; c < K; ++c)
            if (!x[c]) return 0;
    }
    return 1;
}

int orc_reduce_generic(int op, int64_t n, const double* const* x, double* y) {
    if (!gop_args_ok(op, n, x) || !y) return -1;
    int K = orc_gop_components(op);
    double acc[4], xi[4];
    gop_neutral(op, acc);
    for (int64_t i = 0; i < n; ++i) {
        for (int c = 0; c < K; ++c) xi[c] = x[c][i];
        gop_comb(op, acc, xi, acc);
    }
    for (int c = 0; c < K; ++c) y[c] = acc[c];
    return 0;
}

int orc_reduce_generic_vjp(int op, int64_t n, const double* const* x, const double* y_bar,
                           double* const* x_bar) {
    if (!gop_args_ok(op, n, x) || !y_bar) return -1;
    int K = orc_gop_components(op);
    if (n == 0) return 0;
    for (int c = 0; c < K; ++c)
        if (!x_bar || !x_bar[c]) return -1;
    tape_t T, *t = &T;
    if (tape_init(t, (int64_t)(K * 4 + 4) * n + 16, (int64_t)(K * 3 + 4) * n + 16)) return -2;
    int64_t* sx = (int64_t*)malloc((size_t)n * K * sizeof(int64_t));
    if (!sx) {
        tape_free(t);
        return -2;
    }
    double e[4];
    gop_neutral(op, e);
    int64_t acc[4];
    for (int c = 0; c < K; ++c) acc[c] = leaf(t, e[c]); /* constants */
    for (int64_t i = 0; i < n; ++i) {
        for (int c = 0; c < K; ++c) sx[i * K + c] = leaf(t, x[c][i]);
        gop_step(t, op, acc, &sx[i * K], acc);
    }
    int rc = (t->oom || tape_reverse(t)) ? -2 : 0;
    if (!rc) {
        for (int c = 0; c < K; ++c) t->adj[acc[c]] += y_bar[c];
        sweep(t);
        for (int64_t i = 0; i < n; ++i)
            for (int c = 0; c < K; ++c) x_bar[c][i] = t->adj[sx[i * K + c]];
    }
    free(sx);
    tape_free(t);
    return rc;
}

static int cmp_i64(const void* a, const void* b) {
    int64_t x = *(const int64_t*)a, y = *(const int64_t*)b;
    return (x > y) - (x < y);
}

int orc_reduce_generic_vjp_at(int op, int64_t n, const double* const* x, const double* y_bar,
                              int64_t cnt, const int64_t* idx, double* out) {
    if (!gop_args_ok(op, n, x) || !y_bar || cnt < 0 || (cnt > 0 && (!idx || !out))) return -1;
    int K = orc_gop_components(op);
    for (int64_t j = 0; j < cnt; ++j)
        if (idx[j] < 0 || idx[j] >= n) return -1;
    if (cnt == 0) return 0;
    /* samples in index order; L[j], R[j]: folds before and after sample j */
    int64_t* ord = (int64_t*)malloc((size_t)cnt * sizeof(int64_t));
    double* L = (double*)malloc((size_t)cnt * K * sizeof(double));
    double* R = (double*)malloc((size_t)cnt * K * sizeof(double));
    if (!ord || !L || !R) {
        free(ord), free(L), free(R);
        return -2;
    }
    for (int64_t j = 0; j < cnt; ++j) ord[j] = idx[j];
    qsort(ord, (size_t)cnt, sizeof(int64_t), cmp_i64);
    double acc[4], xi[4];
    gop_neutral(op, acc);
    int64_t j = 0;
    for (int64_t i = 0; i < n && j < cnt; ++i) {
        while (j < cnt && ord[j] == i) {
            for (int c = 0; c < K; ++c) L[j * K + c] = acc[c];
            ++j;
        }
        for (int c = 0; c < K; ++c) xi[c] = x[c][i];
        gop_comb(op, acc, xi, acc);
    }
    /* right folds: r = x_{i+1} (.) r, walking down from the end */
    gop_neutral(op, acc);
    j = cnt - 1;
    for (int64_t i = n - 1; i >= 0 && j >= 0; --i) {
        while (j >= 0 && ord[j] == i) {
            for (int c = 0; c < K; ++c) R[j * K + c] = acc[c];
            --j;
        }
        for (int c = 0; c < K; ++c) xi[c] = x[c][i];
        gop_comb(op, xi, acc, acc);
    }
    int rc = 0;
    tape_t T, *t = &T;
    if (tape_init(t, 64, 64)) rc = -2;
    for (int64_t s = 0; s < cnt && !rc; ++s) {
        /* position of idx[s] among the sorted samples */
        int64_t lo = 0, hi = cnt - 1;
        while (lo < hi) {
            int64_t mid = (lo + hi) / 2;
            if (ord[mid] < idx[s]) lo = mid + 1;
            else hi = mid;
        }
        tape_clear(t);
        int64_t sl[4], sa[4], sr[4], acc_s[4];
        for (int c = 0; c < K; ++c) {
            sl[c] = leaf(t, L[lo * K + c]);
            sa[c] = leaf(t, x[c][idx[s]]);
            sr[c] = leaf(t, R[lo * K + c]);
        }
        gop_step(t, op, sl, sa, acc_s);
        gop_step(t, op, acc_s, sr, acc_s);
        if (t->oom || tape_reverse(t)) {
            rc = -2;
            break;
        }
        for (int c = 0; c < K; ++c) t->adj[acc_s[c]] += y_bar[c];
        sweep(t);
        for (int c = 0; c < K; ++c) out[s * K + c] = t->adj[sa[c]];
    }
    tape_free(t);
    free(ord), free(L), free(R);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Inclusive scan with a general operator: y_i = acc after folding x_i.       */
/* ------------------------------------------------------------------------ */

int orc_scan_generic(int op, int64_t n, const double* const* x, double* const* y) {
    return orc_scan_generic_from(op, n, NULL, x, y);
}

int orc_scan_generic_from(int op, int64_t n, const double* init, const double* const* x, double* const* y) {
    if (!gop_args_ok(op, n, x)) return -1;
    int K = orc_gop_components(op);
    if (n > 0) {
        if (!y) return -1;
        for (int c = 0; c < K; ++c)
            if (!y[c]) return -1;
    }
    double acc[4], xi[4];
    gop_neutral(op, acc);
    if (init)
        for (int c = 0; c < K; ++c) acc[c] = init[c];
    for (int64_t i = 0; i < n; ++i) {
        for (int c = 0; c < K; ++c) xi[c] = x[c][i];
        gop_comb(op, acc, xi, acc);
        for (int c = 0; c < K; ++c) y[c][i] = acc[c];
    }
    return 0;
}

int orc_scan_generic_vjp(int op, int64_t n, const double* const* x, const double* const* y_bar,
                         double* const* x_bar) {
    return orc_scan_generic_vjp_from(op, n, NULL, x, y_bar, x_bar);
}

int orc_scan_generic_vjp_from(int op, int64_t n, const double* init, const double* const* x,
                              const double* const* y_bar, double* const* x_bar) {
    if (!gop_args_ok(op, n, x)) return -1;
    int K = orc_gop_components(op);
    if (n == 0) return 0;
    if (!y_bar || !x_bar) return -1;
    for (int c = 0; c < K; ++c)
        if (!y_bar[c] || !x_bar[c]) return -1;
    tape_t T, *t = &T;
    if (tape_init(t, (int64_t)(K * 4 + 4) * n + 16, (int64_t)(K * 3 + 4) * n + 16)) return -2;
    int64_t* sx = (int64_t*)malloc((size_t)n * K * sizeof(int64_t));
    int64_t* sy = (int64_t*)malloc((size_t)n * K * sizeof(int64_t));
    if (!sx || !sy) {
        free(sx), free(sy);
        tape_free(t);
        return -2;
    }
    double e[4];
    gop_neutral(op, e);
    if (init)
        for (int c = 0; c < K; ++c) e[c] = init[c];
    int64_t acc[4];
    for (int c = 0; c < K; ++c) acc[c] = leaf(t, e[c]); /* constants */
    for (int64_t i = 0; i < n; ++i) {
        for (int c = 0; c < K; ++c) sx[i * K + c] = leaf(t, x[c][i]);
        gop_step(t, op, acc, &sx[i * K], acc);
        for (int c = 0; c < K; ++c) sy[i * K + c] = acc[c]; /* the slot holding y_i */
    }
    int rc = (t->oom || tape_reverse(t)) ? -2 : 0;
    if (!rc) {
        /* y_i and y_{i-1} may share a slot (a -inf log-add-exp element leaves
         * the fold unchanged): their seeds then add up, as they must */
        for (int64_t i = 0; i < n; ++i)
            for (int c = 0; c < K; ++c) t->adj[sy[i * K + c]] += y_bar[c][i];
        sweep(t);
        for (int64_t i = 0; i < n; ++i)
            for (int c = 0; c < K; ++c) x_bar[c][i] = t->adj[sx[i * K + c]];
    }
    free(sx), free(sy);
    tape_free(t);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Forward mode (Sec. 3, the tangent rewrite rule): the primal is recorded on */
/* the tape exactly as for the VJP, then one sweep in record order applies    */
/* tan[out] = d out/d in0 * tan[in0] + d out/d in1 * tan[in1], starting from   */
/* the seeded leaves.                                                          */
/* ------------------------------------------------------------------------ */

static double* tan_alloc(tape_t* t) { return (double*)calloc((size_t)(t->nv > 0 ? t->nv : 1), sizeof(double)); }

static void tan_sweep(const tape_t* t, double* tan) {
    for (int64_t r = 0; r < t->nr; ++r) {
        const rec_t* q = &t->rec[r];
        double v = q->w0 * tan[q->in0];
        if (q->in1 >= 0) v += q->w1 * tan[q->in1];
        tan[q->out] = v;
    }
}

int orc_reduce_jvp(int op, int64_t n, const double* x, const double* x_dot, double* y_dot) {
    if (op < ORC_ADD || op > ORC_MAX || n < 0 || (n > 0 && (!x || !x_dot)) || !y_dot) return -1;
    tape_t T, *t = &T;
    if (tape_init(t, 2 * n + 16, n + 16)) return -2;
    int64_t* sx = (int64_t*)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
    if (!sx) {
        tape_free(t);
        return -2;
    }
    for (int64_t i = 0; i < n; ++i) sx[i] = leaf(t, x[i]);
    int64_t y = leaf(t, neutral(op));
    int first = 1;
    for (int64_t i = 0; i < n; ++i) {
        switch (op) {
            case ORC_ADD: y = t_add(t, y, sx[i]); break;
            case ORC_MUL: y = t_mul(t, y, sx[i]); break;
            default: y = t_pick(t, y, sx[i], first || better(op, x[i], V(y)));
        }
        first = 0;
    }
    double* tan = t->oom ? NULL : tan_alloc(t);
    int rc = tan ? 0 : -2;
    if (!rc) {
        for (int64_t i = 0; i < n; ++i) tan[sx[i]] = x_dot[i];
        tan_sweep(t, tan);
        *y_dot = tan[y];
    }
    free(tan);
    free(sx);
    tape_free(t);
    return rc;
}

int orc_hist_jvp(int op, int64_t n, int64_t m, const int32_t* inds, const double* vs,
                 const double* vs_dot, double* hs_dot) {
    if (op < ORC_ADD || op > ORC_MAX || n < 0 || m < 0 || (n > 0 && (!inds || !vs || !vs_dot)) ||
        (m > 0 && !hs_dot))
        return -1;
    tape_t T, *t = &T;
    if (tape_init(t, 2 * n + 16, n + 16)) return -2;
    int64_t* sv = (int64_t*)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
    int64_t* sh = (int64_t*)malloc((size_t)(m > 0 ? m : 1) * sizeof(int64_t));
    if (!sv || !sh) {
        free(sv), free(sh);
        tape_free(t);
        return -2;
    }
    for (int64_t i = 0; i < n; ++i) sv[i] = leaf(t, vs[i]);
    for (int64_t k = 0; k < m; ++k) sh[k] = -1;
    for (int64_t i = 0; i < n; ++i) {
        int64_t k = inds[i];
        if (k < 0 || k >= m) continue;
        if (sh[k] < 0) {
            sh[k] = sv[i];
            continue;
        }
        switch (op) {
            case ORC_ADD: sh[k] = t_add(t, sh[k], sv[i]); break;
            case ORC_MUL: sh[k] = t_mul(t, sh[k], sv[i]); break;
            default: sh[k] = t_pick(t, sh[k], sv[i], better(op, vs[i], V(sh[k])));
        }
    }
    double* tan = t->oom ? NULL : tan_alloc(t);
    int rc = tan ? 0 : -2;
    if (!rc) {
        for (int64_t i = 0; i < n; ++i) tan[sv[i]] = vs_dot[i];
        tan_sweep(t, tan);
        for (int64_t k = 0; k < m; ++k) hs_dot[k] = sh[k] >= 0 ? tan[sh[k]] : 0.0; /* empty: the constant e */
    }
    free(tan);
    free(sv), free(sh);
    tape_free(t);
    return rc;
}

int orc_scatter_jvp(int64_t n, const double* xs_dot, int64_t m, const int32_t* is, const double* vs_dot,
                    double* ys_dot) {
    if (n < 0 || m < 0 || (n > 0 && (!xs_dot || !ys_dot)) || (m > 0 && (!is || !vs_dot))) return -1;
    /* ys[k] is a copy of xs[k] or of the last vs[j] with is[j] == k: its
     * tangent is that variable's tangent */
    for (int64_t k = 0; k < n; ++k) ys_dot[k] = xs_dot[k];
    for (int64_t j = 0; j < m; ++j) {
        int64_t k = is[j];
        if (k >= 0 && k < n) ys_dot[k] = vs_dot[j];
    }
    return 0;
}

int orc_map_jvp(int fn, int64_t n, const double* x, const double* x_dot, double* y_dot) {
    if (fn < ORC_FN_SQUARE || fn > ORC_FN_TANH || n < 0 || (n > 0 && (!x || !x_dot || !y_dot))) return -1;
    tape_t T, *t = &T;
    if (tape_init(t, 16, 16)) return -2;
    double tan[16];
    for (int64_t i = 0; i < n; ++i) {
        tape_clear(t);
        int64_t xs = leaf(t, x[i]);
        int64_t ys = apply_fn(t, fn, xs);
        for (int64_t s = 0; s < t->nv && s < 16; ++s) tan[s] = 0.0;
        tan[xs] = x_dot[i];
        tan_sweep(t, tan);
        y_dot[i] = tan[ys];
    }
    tape_free(t);
    return 0;
}

int orc_reduce_generic_jvp(int op, int64_t n, const double* const* x, const double* const* x_dot,
                           double* y_dot) {
    if (!gop_args_ok(op, n, x) || !gop_args_ok(op, n, x_dot) || !y_dot) return -1;
    int K = orc_gop_components(op);
    tape_t T, *t = &T;
    if (tape_init(t, (int64_t)(K * 4 + 4) * n + 16, (int64_t)(K * 3 + 4) * n + 16)) return -2;
    int64_t* sx = (int64_t*)malloc((size_t)(n > 0 ? n : 1) * K * sizeof(int64_t));
    if (!sx) {
        tape_free(t);
        return -2;
    }
    double e[4];
    gop_neutral(op, e);
    int64_t acc[4];
    for (int c = 0; c < K; ++c) acc[c] = leaf(t, e[c]);
    for (int64_t i = 0; i < n; ++i) {
        for (int c = 0; c < K; ++c) sx[i * K + c] = leaf(t, x[c][i]);
        gop_step(t, op, acc, &sx[i * K], acc);
    }
    double* tan = t->oom ? NULL : tan_alloc(t);
    int rc = tan ? 0 : -2;
    if (!rc) {
        for (int64_t i = 0; i < n; ++i)
            for (int c = 0; c < K; ++c) tan[sx[i * K + c]] = x_dot[c][i];
        tan_sweep(t, tan);
        for (int c = 0; c < K; ++c) y_dot[c] = tan[acc[c]];
    }
    free(tan);
    free(sx);
    tape_free(t);
    return rc;
}

int orc_scan_generic_jvp(int op, int64_t n, const double* const* x, const double* const* x_dot,
                         double* const* y_dot) {
    return orc_scan_generic_jvp_from(op, n, NULL, x, x_dot, y_dot);
}

int orc_scan_generic_jvp_from(int op, int64_t n, const double* init, const double* const* x,
                              const double* const* x_dot, double* const* y_dot) {
    if (!gop_args_ok(op, n, x) || !gop_args_ok(op, n, x_dot)) return -1;
    int K = orc_gop_components(op);
    if (n == 0) return 0;
    if (!y_dot) return -1;
    for (int c = 0; c < K; ++c)
        if (!y_dot[c]) return -1;
    tape_t T, *t = &T;
    if (tape_init(t, (int64_t)(K * 4 + 4) * n + 16, (int64_t)(K * 3 + 4) * n + 16)) return -2;
    int64_t* sx = (int64_t*)malloc((size_t)n * K * sizeof(int64_t));
    int64_t* sy = (int64_t*)malloc((size_t)n * K * sizeof(int64_t));
    if (!sx || !sy) {
        free(sx), free(sy);
        tape_free(t);
        return -2;
    }
    double e[4];
    gop_neutral(op, e);
    if (init)
        for (int c = 0; c < K; ++c) e[c] = init[c];
    int64_t acc[4];
    for (int c = 0; c < K; ++c) acc[c] = leaf(t, e[c]);
    for (int64_t i = 0; i < n; ++i) {
        for (int c = 0; c < K; ++c) sx[i * K + c] = leaf(t, x[c][i]);
        gop_step(t, op, acc, &sx[i * K], acc);
        for (int c = 0; c < K; ++c) sy[i * K + c] = acc[c];
    }
    double* tan = t->oom ? NULL : tan_alloc(t);
    int rc = tan ? 0 : -2;
    if (!rc) {
        for (int64_t i = 0; i < n; ++i)
            for (int c = 0; c < K; ++c) tan[sx[i * K + c]] = x_dot[c][i];
        tan_sweep(t, tan);
        for (int64_t i = 0; i < n; ++i)
            for (int c = 0; c < K; ++c) y_dot[c][i] = tan[sy[i * K + c]];
    }
    free(tan);
    free(sx), free(sy);
    tape_free(t);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Dense k-means (Sec. 7.4): f(C) = sum_i min_k |x_i - c_k|^2 (squared        */
/* distance: the reading under which the Hessian is diagonal).  X is N x D,   */
/* C is K x D, row-major.  The distance is the fused chain                    */
/* acc = fma(x_d - c_d, x_d - c_d, acc) over d = 0..D-1 in FP64, so that the  */
/* assignment (lowest k among equal distances) is decided on exactly the     */
/* values any implementation of the same chain computes.                     */
/* ------------------------------------------------------------------------ */

static double km_dist(int D, const double* x, const double* c) {
    double acc = 0.0;
    for (int d = 0; d < D; ++d) {
        double t = x[d] - c[d];
        acc = fma(t, t, acc);
    }
    return acc;
}

static void km_assign(int64_t N, int D, int K, const double* X, const double* C, int32_t* a, double* dmin) {
    for (int64_t i = 0; i < N; ++i) {
        int best = 0;
        double bd = km_dist(D, X + i * D, C);
        for (int k = 1; k < K; ++k) {
            double dk = km_dist(D, X + i * D, C + (int64_t)k * D);
            if (dk < bd) bd = dk, best = k;
        }
        a[i] = best;
        if (dmin) dmin[i] = bd;
    }
}

int orc_kmeans_objective(int64_t N, int D, int K, const double* X, const double* C, int32_t* assign,
                         double* f) {
    if (N < 0 || D < 1 || K < 1 || (N > 0 && !X) || !C || !f) return -1;
    int32_t* a = assign ? assign : (int32_t*)malloc((size_t)(N > 0 ? N : 1) * sizeof(int32_t));
    double* dm = (double*)malloc((size_t)(N > 0 ? N : 1) * sizeof(double));
    if (!a || !dm) {
        if (!assign) free(a);
        free(dm);
        return -2;
    }
    km_assign(N, D, K, X, C, a, dm);
    double s = 0.0;
    for (int64_t i = 0; i < N; ++i) s += dm[i];
    *f = s;
    if (!assign) free(a);
    free(dm);
    return 0;
}

/* Gradient for fixed assignments a: f is a sum of independent per-point
 * terms |x_i - c_{a_i}|^2, so each term is recorded on a small tape of its
 * own, swept, and its adjoint added to the centre's (the adjoint of a sum
 * reaches every term unchanged). */
static int km_grad_fixed(int64_t N, int D, int K, const double* X, const double* C, const int32_t* a,
                         double f_bar, double* C_bar) {
    for (int64_t e = 0; e < (int64_t)K * D; ++e) C_bar[e] = 0.0;
    tape_t T, *t = &T;
    if (tape_init(t, 4 * D + 16, 4 * D + 16)) return -2;
    int64_t* sc = (int64_t*)malloc((size_t)D * sizeof(int64_t));
    if (!sc) {
        tape_free(t);
        return -2;
    }
    for (int64_t i = 0; i < N; ++i) {
        const double* c = C + (int64_t)a[i] * D;
        tape_clear(t);
        int64_t acc = -1;
        for (int d = 0; d < D; ++d) {
            sc[d] = leaf(t, c[d]);
            int64_t xd = leaf(t, X[i * D + d]); /* a constant */
            int64_t df = t_sub(t, xd, sc[d]);
            int64_t sq = t_mul(t, df, df);
            acc = (acc < 0) ? sq : t_add(t, acc, sq);
        }
        if (t->oom || tape_reverse(t)) {
            free(sc);
            tape_free(t);
            return -2;
        }
        t->adj[acc] += f_bar;
        sweep(t);
        for (int d = 0; d < D; ++d) C_bar[(int64_t)a[i] * D + d] += t->adj[sc[d]];
    }
    free(sc);
    tape_free(t);
    return 0;
}

int orc_kmeans_vjp(int64_t N, int D, int K, const double* X, const double* C, double f_bar, double* C_bar) {
    if (N < 0 || D < 1 || K < 1 || (N > 0 && !X) || !C || !C_bar) return -1;
    int32_t* a = (int32_t*)malloc((size_t)(N > 0 ? N : 1) * sizeof(int32_t));
    if (!a) return -2;
    km_assign(N, D, K, X, C, a, NULL);
    int rc = km_grad_fixed(N, D, K, X, C, a, f_bar, C_bar);
    free(a);
    return rc;
}

/* jvp of the vjp in direction C_dot (Sec. 7.4): the assignments are locally
 * constant, so the gradient is an affine function of C and its directional
 * derivative is its central difference with a unit step, exact up to
 * rounding: (g(C + C_dot) - g(C - C_dot)) / 2 with the assignment of C. */
int orc_kmeans_hvp(int64_t N, int D, int K, const double* X, const double* C, double f_bar,
                   const double* C_dot, double* out) {
    if (N < 0 || D < 1 || K < 1 || (N > 0 && !X) || !C || !C_dot || !out) return -1;
    const int64_t KD = (int64_t)K * D;
    int32_t* a = (int32_t*)malloc((size_t)(N > 0 ? N : 1) * sizeof(int32_t));
    double* cp = (double*)malloc((size_t)KD * sizeof(double));
    double* cm = (double*)malloc((size_t)KD * sizeof(double));
    double* gp = (double*)malloc((size_t)KD * sizeof(double));
    double* gm = (double*)malloc((size_t)KD * sizeof(double));
    int rc = (a && cp && cm && gp && gm) ? 0 : -2;
    if (!rc) {
        km_assign(N, D, K, X, C, a, NULL);
        for (int64_t e = 0; e < KD; ++e) cp[e] = C[e] + C_dot[e], cm[e] = C[e] - C_dot[e];
        rc = km_grad_fixed(N, D, K, X, cp, a, f_bar, gp);
        if (!rc) rc = km_grad_fixed(N, D, K, X, cm, a, f_bar, gm);
        if (!rc)
            for (int64_t e = 0; e < KD; ++e) out[e] = 0.5 * (gp[e] - gm[e]);
    }
    free(a), free(cp), free(cm), free(gp), free(gm);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* A map whose body reads a free array at computed indices (Sec. 5.4):       */
/*   ys[i] = f(as[is[i]], vs[i]),  f = a (gather), a v, or (a - v)^2.        */
/* On the tape each as[k] is one leaf variable and every read of it is an    */
/* edge from that leaf, so the reverse sweep adds each read's partial into   */
/* the leaf's adjoint: the accumulator's list of (index, value) updates,     */
/* applied in reverse record order.  An index outside [0, n) reads the       */
/* constant 0 (a leaf of its own that the result ignores).                   */
static int64_t gm_body(tape_t* t, int op, int64_t a, int64_t v) {
    if (op == 0) return emit1(t, V(a), a, 1.0);
    if (op == 1) return t_mul(t, a, v);
    int64_t d = t_sub(t, a, v);
    return t_mul(t, d, d);
}

static int gm_check(int op, int64_t n, const double* as, int64_t m, const int32_t* is, const double* vs) {
    if (op < 0 || op > 2 || n < 0 || m < 0) return -1;
    if ((n > 0 && !as) || (m > 0 && !is) || (m > 0 && op != 0 && !vs)) return -1;
    return 0;
}

int orc_gather_map(int op, int64_t n, const double* as, int64_t m, const int32_t* is, const double* vs,
                   double* ys) {
    if (gm_check(op, n, as, m, is, vs) || (m > 0 && !ys)) return -1;
    tape_t T, *t = &T;
    if (tape_init(t, n + 4 * m + 16, 3 * m + 16)) return -2;
    int64_t a0 = t->nv;
    for (int64_t k = 0; k < n; ++k) leaf(t, as[k]);
    for (int64_t i = 0; i < m; ++i) {
        const int64_t k = is[i];
        const int64_t a = (k >= 0 && k < n) ? a0 + k : leaf(t, 0.0);
        const int64_t v = leaf(t, op ? vs[i] : 0.0);
        ys[i] = V(gm_body(t, op, a, v));
    }
    int rc = t->oom ? -2 : 0;
    tape_free(t);
    return rc;
}

int orc_gather_map_vjp(int op, int64_t n, const double* as, int64_t m, const int32_t* is, const double* vs,
                       const double* ys_bar, double* as_bar, double* vs_bar) {
    if (gm_check(op, n, as, m, is, vs) || (n > 0 && !as_bar) || (m > 0 && (!ys_bar || (op && !vs_bar))))
        return -1;
    tape_t T, *t = &T;
    if (tape_init(t, n + 4 * m + 16, 3 * m + 16)) return -2;
    int64_t* y = (int64_t*)malloc((size_t)(m > 0 ? m : 1) * sizeof(int64_t));
    int64_t* vv = (int64_t*)malloc((size_t)(m > 0 ? m : 1) * sizeof(int64_t));
    if (!y || !vv) {
        free(y), free(vv), tape_free(t);
        return -2;
    }
    int64_t a0 = t->nv;
    for (int64_t k = 0; k < n; ++k) leaf(t, as[k]);
    for (int64_t i = 0; i < m; ++i) {
        const int64_t k = is[i];
        const int64_t a = (k >= 0 && k < n) ? a0 + k : leaf(t, 0.0);
        vv[i] = leaf(t, op ? vs[i] : 0.0);
        y[i] = gm_body(t, op, a, vv[i]);
    }
    int rc = (t->oom || tape_reverse(t)) ? -2 : 0;
    if (!rc) {
        for (int64_t i = 0; i < m; ++i) t->adj[y[i]] += ys_bar[i];
        sweep(t);
        for (int64_t k = 0; k < n; ++k) as_bar[k] = t->adj[a0 + k];
        if (op)
            for (int64_t i = 0; i < m; ++i) vs_bar[i] = t->adj[vv[i]];
    }
    free(y), free(vv);
    tape_free(t);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Sparse k-means (Sec. 7.5): points in CSR (rowptr [N+1], col [nnz], val    */
/* [nnz]), dense centres C [K x D].  The cost is the dense one with the      */
/* squared distance, taken by its definition: row i is densified (zero       */
/* where nothing is stored) and its distance to centre k is the plain sum    */
/* over d = 0..D-1 of (x_d - c_kd)^2, in d order.  Ties go to the lowest k.  */
/* The gradient at fixed assignments is the closed form                      */
/* 2 f_bar (n_k c_k - S_k), S_k the sum of the rows assigned to k, and the   */
/* jvp of the VJP is 2 f_bar n_k C_dot_k.                                    */
static int skm_check(int64_t N, int64_t D, int K, const int64_t* rowptr, const int32_t* col, const double* val,
                     const double* C) {
    if (N < 0 || D < 1 || K < 1 || !rowptr || !C) return -1;
    if (rowptr[0] != 0) return -1;
    for (int64_t i = 0; i < N; ++i)
        if (rowptr[i + 1] < rowptr[i]) return -1;
    const int64_t nnz = rowptr[N];
    if (nnz > 0 && (!col || !val)) return -1;
    for (int64_t e = 0; e < nnz; ++e)
        if (col[e] < 0 || col[e] >= D) return -1;
    return 0;
}

/* dist [N x K] (nullable): every row's distance to every centre. */
static int skm_assign(int64_t N, int64_t D, int K, const int64_t* rowptr, const int32_t* col, const double* val,
                      const double* C, int32_t* a, double* dmin, double* dist) {
    double* x = (double*)calloc((size_t)D, sizeof(double));
    if (!x) return -2;
    for (int64_t i = 0; i < N; ++i) {
        for (int64_t e = rowptr[i]; e < rowptr[i + 1]; ++e) x[col[e]] = val[e];
        int best = 0;
        double bd = 0.0;
        for (int k = 0; k < K; ++k) {
            const double* c = C + (int64_t)k * D;
            double acc = 0.0;
            for (int64_t d = 0; d < D; ++d) {
                const double t = x[d] - c[d];
                acc += t * t;
            }
            if (dist) dist[i * K + k] = acc;
            if (k == 0 || acc < bd) bd = acc, best = k;
        }
        if (a) a[i] = best;
        if (dmin) dmin[i] = bd;
        for (int64_t e = rowptr[i]; e < rowptr[i + 1]; ++e) x[col[e]] = 0.0;
    }
    free(x);
    return 0;
}

int orc_skm_dist(int64_t N, int64_t D, int K, const int64_t* rowptr, const int32_t* col, const double* val,
                 const double* C, double* dist) {
    if (skm_check(N, D, K, rowptr, col, val, C) || !dist) return -1;
    return skm_assign(N, D, K, rowptr, col, val, C, NULL, NULL, dist);
}

int orc_skm_objective(int64_t N, int64_t D, int K, const int64_t* rowptr, const int32_t* col, const double* val,
                      const double* C, int32_t* assign, double* f) {
    if (skm_check(N, D, K, rowptr, col, val, C) || !f) return -1;
    int32_t* a = assign ? assign : (int32_t*)malloc((size_t)(N > 0 ? N : 1) * sizeof(int32_t));
    double* dm = (double*)malloc((size_t)(N > 0 ? N : 1) * sizeof(double));
    int rc = (a && dm) ? skm_assign(N, D, K, rowptr, col, val, C, a, dm, NULL) : -2;
    if (!rc) {
        double s = 0.0;
        for (int64_t i = 0; i < N; ++i) s += dm[i];
        *f = s;
    }
    if (!assign) free(a);
    free(dm);
    return rc;
}

static int skm_grad(int64_t N, int64_t D, int K, const int64_t* rowptr, const int32_t* col, const double* val,
                    const double* C, double f_bar, const double* C_dot, double* out) {
    if (skm_check(N, D, K, rowptr, col, val, C) || !out) return -1;
    int32_t* a = (int32_t*)malloc((size_t)(N > 0 ? N : 1) * sizeof(int32_t));
    int64_t* n = (int64_t*)calloc((size_t)K, sizeof(int64_t));
    if (!a || !n) {
        free(a), free(n);
        return -2;
    }
    int rc = skm_assign(N, D, K, rowptr, col, val, C, a, NULL, NULL);
    if (!rc) {
        for (int64_t i = 0; i < N; ++i) ++n[a[i]];
        for (int k = 0; k < K; ++k)
            for (int64_t d = 0; d < D; ++d) {
                const int64_t e = (int64_t)k * D + d;
                out[e] = C_dot ? 2.0 * f_bar * (double)n[k] * C_dot[e] : 2.0 * f_bar * (double)n[k] * C[e];
            }
        if (!C_dot)
            for (int64_t i = 0; i < N; ++i)
                for (int64_t e = rowptr[i]; e < rowptr[i + 1]; ++e)
                    out[(int64_t)a[i] * D + col[e]] -= 2.0 * f_bar * val[e];
    }
    free(a), free(n);
    return rc;
}

int orc_skm_vjp(int64_t N, int64_t D, int K, const int64_t* rowptr, const int32_t* col, const double* val,
                const double* C, double f_bar, double* C_bar) {
    return skm_grad(N, D, K, rowptr, col, val, C, f_bar, NULL, C_bar);
}

int orc_skm_hvp(int64_t N, int64_t D, int K, const int64_t* rowptr, const int32_t* col, const double* val,
                const double* C, double f_bar, const double* C_dot, double* out) {
    if (!C_dot) return -1;
    return skm_grad(N, D, K, rowptr, col, val, C, f_bar, C_dot, out);
}

/* ------------------------------------------------------------------------ */
/* reduce_by_index with a general operator (Sec. 5.1.2, with the general     */
/* rule of Sec. 5.1.1 inside each bin): hs[b] = the fold, in index order, of */
/* the elements i with inds[i] = b (the neutral element for an empty bin;    */
/* indices outside [0, m) are skipped).  Each bin's elements are gathered in */
/* index order and handed to the generic reduce and its VJP; elements out of */
/* range get adjoint 0.  x, hs, hs_bar, x_bar: K component arrays.           */
static int hg_order(int64_t n, int64_t m, const int32_t* inds, int64_t** off_out, int64_t** perm_out) {
    int64_t* off = (int64_t*)calloc((size_t)(m + 1), sizeof(int64_t));
    int64_t* perm = (int64_t*)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
    int64_t* cur = (int64_t*)malloc((size_t)(m > 0 ? m : 1) * sizeof(int64_t));
    if (!off || !perm || !cur) {
        free(off), free(perm), free(cur);
        return -2;
    }
    for (int64_t i = 0; i < n; ++i)
        if (inds[i] >= 0 && inds[i] < m) ++off[inds[i] + 1];
    for (int64_t b = 0; b < m; ++b) off[b + 1] += off[b];
    for (int64_t b = 0; b < m; ++b) cur[b] = off[b];
    for (int64_t i = 0; i < n; ++i)  /* in index order: stable */
        if (inds[i] >= 0 && inds[i] < m) perm[cur[inds[i]]++] = i;
    free(cur);
    *off_out = off, *perm_out = perm;
    return 0;
}

int orc_hist_generic(int op, int64_t n, int64_t m, const int32_t* inds, const double* const* x,
                     double* const* hs) {
    const int K = orc_gop_components(op);
    if (K == 0 || n < 0 || m < 1 || (n > 0 && (!inds || !x)) || !hs) return -1;
    int64_t *off, *perm;
    if (hg_order(n, m, inds, &off, &perm)) return -2;
    double* sub[4] = {0, 0, 0, 0};
    int rc = 0;
    for (int c = 0; c < K && !rc; ++c)
        if (!(sub[c] = (double*)malloc((size_t)(n > 0 ? n : 1) * sizeof(double)))) rc = -2;
    for (int64_t b = 0; b < m && !rc; ++b) {
        const int64_t cnt = off[b + 1] - off[b];
        for (int64_t r = 0; r < cnt; ++r)
            for (int c = 0; c < K; ++c) sub[c][r] = x[c][perm[off[b] + r]];
        double y[4];
        rc = orc_reduce_generic(op, cnt, (const double* const*)sub, y);
        for (int c = 0; c < K; ++c) hs[c][b] = y[c];
    }
    for (int c = 0; c < K; ++c) free(sub[c]);
    free(off), free(perm);
    return rc;
}

int orc_hist_generic_vjp(int op, int64_t n, int64_t m, const int32_t* inds, const double* const* x,
                         const double* const* hs_bar, double* const* x_bar) {
    const int K = orc_gop_components(op);
    if (K == 0 || n < 0 || m < 1 || (n > 0 && (!inds || !x || !x_bar)) || !hs_bar) return -1;
    int64_t *off, *perm;
    if (hg_order(n, m, inds, &off, &perm)) return -2;
    double* sub[4] = {0, 0, 0, 0};
    double* gs[4] = {0, 0, 0, 0};
    int rc = 0;
    for (int c = 0; c < K && !rc; ++c) {
        sub[c] = (double*)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
        gs[c] = (double*)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
        if (!sub[c] || !gs[c]) rc = -2;
    }
    for (int c = 0; c < K && !rc; ++c)
        for (int64_t i = 0; i < n; ++i) x_bar[c][i] = 0.0;
    for (int64_t b = 0; b < m && !rc; ++b) {
        const int64_t cnt = off[b + 1] - off[b];
        if (cnt == 0) continue;
        for (int64_t r = 0; r < cnt; ++r)
            for (int c = 0; c < K; ++c) sub[c][r] = x[c][perm[off[b] + r]];
        double yb[4];
        for (int c = 0; c < K; ++c) yb[c] = hs_bar[c][b];
        rc = orc_reduce_generic_vjp(op, cnt, (const double* const*)sub, yb, gs);
        for (int64_t r = 0; r < cnt && !rc; ++r)
            for (int c = 0; c < K; ++c) x_bar[c][perm[off[b] + r]] = gs[c][r];
    }
    for (int c = 0; c < K; ++c) free(sub[c]), free(gs[c]);
    free(off), free(perm);
    return rc;
}
