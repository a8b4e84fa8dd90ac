"""CPU oracle for the reverse-mode rules (test infrastructure only).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product library never does: it
shares no code with the oracle, and neither imports the other.

The arithmetic lives in ``oracle.c`` (plain C, FP64, explicit tape, reverse
sweep).  This module only converts numpy arrays (every floating-point input is
upcast to float64, which is exact for float32) and calls it through ctypes.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")

ADD, MUL, MIN, MAX = 0, 1, 2, 3
OPS = {"add": ADD, "mul": MUL, "min": MIN, "max": MAX}
FN_SQUARE, FN_EXP, FN_LOG, FN_SIN, FN_TANH = 0, 1, 2, 3, 4
FNS = {"square": FN_SQUARE, "exp": FN_EXP, "log": FN_LOG, "sin": FN_SIN, "tanh": FN_TANH}
GOP_LOGADDEXP, GOP_LINREC, GOP_MAT2 = 0, 1, 2
GOPS = {"logaddexp": GOP_LOGADDEXP, "linrec": GOP_LINREC, "mat2": GOP_MAT2}

_lib = None

_P = ctypes.c_void_p
_I = ctypes.c_int
_L = ctypes.c_int64
_D = ctypes.c_double

_SIGS = {
    "orc_linrec_scan": [_L, _P, _P, _P, _P],
    "orc_linrec_scan_vjp": [_L, _P, _P, _P, _P, _P, _P],
    "orc_reduce": [_I, _L, _P, _P, _P, _P, _P],
    "orc_reduce_vjp": [_I, _L, _P, _D, _P],
    "orc_hist": [_I, _L, _L, _P, _P, _P, _P, _P, _P, _P],
    "orc_hist_vjp": [_I, _L, _L, _P, _P, _P, _P],
    "orc_scatter": [_L, _P, _L, _P, _P, _P, _P],
    "orc_scatter_vjp": [_L, _L, _P, _P, _P, _P],
    "orc_map": [_I, _L, _P, _P],
    "orc_map_vjp": [_I, _L, _P, _P, _P],
    "orc_fig1": [_L, _P, _P, _P, _P],
    "orc_fig1_vjp": [_L, _P, _P, _P, _P, _P, _P],
    "orc_gmm_objective": [_L, _I, _I, _P, _P, _P, _P, _P, _P, _P],
    "orc_gmm_vjp": [_L, _I, _I, _P, _P, _P, _P, _P, _D, _P, _P, _P, _P],
    "orc_gop_components": [_I],
    "orc_reduce_generic": [_I, _L, _P, _P],
    "orc_reduce_generic_vjp": [_I, _L, _P, _P, _P],
    "orc_reduce_generic_vjp_at": [_I, _L, _P, _P, _L, _P, _P],
    "orc_scan_generic": [_I, _L, _P, _P],
    "orc_scan_generic_from": [_I, _L, _P, _P, _P],
    "orc_scan_generic_vjp": [_I, _L, _P, _P, _P],
    "orc_scan_generic_vjp_from": [_I, _L, _P, _P, _P, _P],
    "orc_reduce_jvp": [_I, _L, _P, _P, _P],
    "orc_hist_jvp": [_I, _L, _L, _P, _P, _P, _P],
    "orc_scatter_jvp": [_L, _P, _L, _P, _P, _P],
    "orc_map_jvp": [_I, _L, _P, _P, _P],
    "orc_reduce_generic_jvp": [_I, _L, _P, _P, _P],
    "orc_scan_generic_jvp": [_I, _L, _P, _P, _P],
    "orc_scan_generic_jvp_from": [_I, _L, _P, _P, _P, _P],
    "orc_kmeans_objective": [_L, _I, _I, _P, _P, _P, _P],
    "orc_kmeans_vjp": [_L, _I, _I, _P, _P, _D, _P],
    "orc_kmeans_hvp": [_L, _I, _I, _P, _P, _D, _P, _P],
    "orc_gather_map": [_I, _L, _P, _L, _P, _P, _P],
    "orc_skm_objective": [_L, _L, _I, _P, _P, _P, _P, _P, _P],
    "orc_skm_dist": [_L, _L, _I, _P, _P, _P, _P, _P],
    "orc_hist_generic": [_I, _L, _L, _P, _P, _P],
    "orc_hist_generic_vjp": [_I, _L, _L, _P, _P, _P, _P],
    "orc_skm_vjp": [_L, _L, _I, _P, _P, _P, _P, _D, _P],
    "orc_skm_hvp": [_L, _L, _I, _P, _P, _P, _P, _D, _P, _P],
    "orc_gather_map_vjp": [_I, _L, _P, _L, _P, _P, _P, _P, _P],
}


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc (plain C, no fast-math)."""
    from . import _build as _b

    return _b.build(force=force)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = ctypes.CDLL(LIB_PATH)
        for name, argt in _SIGS.items():
            f = getattr(L, name)
            f.argtypes = argt
            f.restype = ctypes.c_int
        _lib = L
    return _lib


def _f64(x):
    return np.ascontiguousarray(np.asarray(x, dtype=np.float64))


def _i32(x):
    return np.ascontiguousarray(np.asarray(x, dtype=np.int32))


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _check(rc, name):
    if rc != 0:
        raise RuntimeError(f"oracle {name} failed with status {rc}")


# ---------------------------------------------------------------- linrec scan
def linrec_scan(a, b):
    a, b = _f64(a), _f64(b)
    n = a.size
    A, B = np.empty(n), np.empty(n)
    _check(lib().orc_linrec_scan(n, _p(a), _p(b), _p(A), _p(B)), "linrec_scan")
    return A, B


def linrec_scan_vjp(a, b, yA_bar, yB_bar):
    a, b, ya, yb = _f64(a), _f64(b), _f64(yA_bar), _f64(yB_bar)
    n = a.size
    ab, bb = np.empty(n), np.empty(n)
    _check(lib().orc_linrec_scan_vjp(n, _p(a), _p(b), _p(ya), _p(yb), _p(ab), _p(bb)),
           "linrec_scan_vjp")
    return ab, bb


# --------------------------------------------------------------------- reduce
def reduce(op, x):
    """Returns (y, arg, p, z): arg is the lowest index of the extreme for
    min/max (-1 for n == 0); p, z the non-zero product and zero count."""
    op = OPS.get(op, op)
    x = _f64(x)
    y, p = ctypes.c_double(), ctypes.c_double()
    arg, z = ctypes.c_int64(), ctypes.c_int64()
    _check(lib().orc_reduce(op, x.size, _p(x), ctypes.byref(y), ctypes.byref(arg),
                            ctypes.byref(p), ctypes.byref(z)), "reduce")
    return y.value, arg.value, p.value, z.value


def reduce_vjp(op, x, y_bar):
    op = OPS.get(op, op)
    x = _f64(x)
    xb = np.empty(x.size)
    _check(lib().orc_reduce_vjp(op, x.size, _p(x), float(y_bar), _p(xb)), "reduce_vjp")
    return xb


# ------------------------------------------------------------ reduce_by_index
def hist(op, inds, vs, m):
    """Returns dict with hs, winner, p, z, count (all length m)."""
    op = OPS.get(op, op)
    inds, vs = _i32(inds), _f64(vs)
    out = {
        "hs": np.empty(m),
        "winner": np.empty(m, dtype=np.int64),
        "p": np.empty(m),
        "z": np.empty(m, dtype=np.int64),
        "count": np.empty(m, dtype=np.int64),
    }
    _check(lib().orc_hist(op, vs.size, m, _p(inds), _p(vs), _p(out["hs"]), _p(out["winner"]),
                          _p(out["p"]), _p(out["z"]), _p(out["count"])), "hist")
    return out


def hist_vjp(op, inds, vs, hs_bar):
    op = OPS.get(op, op)
    inds, vs, hb = _i32(inds), _f64(vs), _f64(hs_bar)
    vb = np.empty(vs.size)
    _check(lib().orc_hist_vjp(op, vs.size, hb.size, _p(inds), _p(vs), _p(hb), _p(vb)),
           "hist_vjp")
    return vb


# -------------------------------------------------------------------- scatter
def scatter(xs, is_, vs):
    xs, is_, vs = _f64(xs), _i32(is_), _f64(vs)
    ys, saved = np.empty(xs.size), np.empty(is_.size)
    _check(lib().orc_scatter(xs.size, _p(xs), is_.size, _p(is_), _p(vs), _p(ys), _p(saved)),
           "scatter")
    return ys, saved


def scatter_vjp(is_, ys_bar):
    is_, yb = _i32(is_), _f64(ys_bar)
    xb, vb = np.empty(yb.size), np.empty(is_.size)
    _check(lib().orc_scatter_vjp(yb.size, is_.size, _p(is_), _p(yb), _p(xb), _p(vb)),
           "scatter_vjp")
    return xb, vb


# ------------------------------------------------------------------------ map
def map_(fn, x):
    fn = FNS.get(fn, fn)
    x = _f64(x)
    y = np.empty(x.size)
    _check(lib().orc_map(fn, x.size, _p(x), _p(y)), "map")
    return y


def map_vjp(fn, x, y_bar):
    fn = FNS.get(fn, fn)
    x, yb = _f64(x), _f64(y_bar)
    xb = np.empty(x.size)
    _check(lib().orc_map_vjp(fn, x.size, _p(x), _p(yb), _p(xb)), "map_vjp")
    return xb


def fig1(x0, x1):
    x0, x1 = _f64(x0), _f64(x1)
    y0, y1 = np.empty(x0.size), np.empty(x0.size)
    _check(lib().orc_fig1(x0.size, _p(x0), _p(x1), _p(y0), _p(y1)), "fig1")
    return y0, y1


def fig1_vjp(x0, x1, y0_bar, y1_bar):
    x0, x1, b0, b1 = _f64(x0), _f64(x1), _f64(y0_bar), _f64(y1_bar)
    r0, r1 = np.empty(x0.size), np.empty(x0.size)
    _check(lib().orc_fig1_vjp(x0.size, _p(x0), _p(x1), _p(b0), _p(b1), _p(r0), _p(r1)),
           "fig1_vjp")
    return r0, r1


# ------------------------------------------------------------------------ GMM
def _gmm_args(X, alpha, mu, q, l):
    X, alpha, mu, q, l = _f64(X), _f64(alpha), _f64(mu), _f64(q), _f64(l)
    N, D = X.shape if X.ndim == 2 else (0, mu.shape[-1])
    K = alpha.size
    return X, alpha, mu, q, l, N, D, K


def gmm_objective(X, alpha, mu, q, l):
    """Returns (loglik, lse[N])."""
    X, alpha, mu, q, l, N, D, K = _gmm_args(X, alpha, mu, q, l)
    ll = ctypes.c_double()
    lse = np.empty(N)
    _check(lib().orc_gmm_objective(N, D, K, _p(X), _p(alpha), _p(mu), _p(q), _p(l),
                                   ctypes.byref(ll), _p(lse)), "gmm_objective")
    return ll.value, lse


def gmm_vjp(X, alpha, mu, q, l, ell_bar=1.0):
    """Returns (alpha_bar, mu_bar, q_bar, l_bar) shaped like the parameters."""
    X, alpha, mu, q, l, N, D, K = _gmm_args(X, alpha, mu, q, l)
    ab, mb, qb, lb = (np.zeros_like(alpha), np.zeros_like(mu), np.zeros_like(q),
                      np.zeros_like(l))
    _check(lib().orc_gmm_vjp(N, D, K, _p(X), _p(alpha), _p(mu), _p(q), _p(l), float(ell_bar),
                             _p(ab), _p(mb), _p(qb), _p(lb)), "gmm_vjp")
    return ab, mb, qb, lb


# ------------------------------------------------------ generic-operator reduce
def _gop(op):
    return GOPS.get(op, op)


def _components(op, xs):
    K = lib().orc_gop_components(_gop(op))
    if K == 0 or len(xs) != K:
        raise ValueError(f"operator {op} takes {K} component arrays, got {len(xs)}")
    xs = [_f64(x) for x in xs]
    n = xs[0].size
    if any(x.size != n for x in xs):
        raise ValueError("component arrays differ in length")
    ptrs = (ctypes.c_void_p * K)(*[x.ctypes.data for x in xs])
    return xs, ptrs, n, K


def reduce_generic(op, xs):
    """y = xs_0 (.) ... (.) xs_{n-1}; xs is a list of K component arrays.
    Returns K floats."""
    xs, ptrs, n, K = _components(op, xs)
    y = np.empty(K)
    _check(lib().orc_reduce_generic(_gop(op), n, ptrs, _p(y)), "reduce_generic")
    return y


def reduce_generic_vjp(op, xs, y_bar):
    """Adjoints of every element: a list of K arrays."""
    xs, ptrs, n, K = _components(op, xs)
    yb = _f64(y_bar).reshape(K)
    out = [np.empty(n) for _ in range(K)]
    optr = (ctypes.c_void_p * K)(*[o.ctypes.data for o in out])
    _check(lib().orc_reduce_generic_vjp(_gop(op), n, ptrs, _p(yb), optr), "reduce_generic_vjp")
    return out


def reduce_generic_vjp_at(op, xs, y_bar, idx):
    """Adjoints of the elements idx only: array [len(idx), K]."""
    xs, ptrs, n, K = _components(op, xs)
    yb = _f64(y_bar).reshape(K)
    idx = np.ascontiguousarray(np.asarray(idx, dtype=np.int64))
    out = np.empty((idx.size, K))
    _check(lib().orc_reduce_generic_vjp_at(_gop(op), n, ptrs, _p(yb), idx.size, _p(idx), _p(out)),
           "reduce_generic_vjp_at")
    return out


def _arrays(K, n):
    out = [np.empty(n) for _ in range(K)]
    return out, (ctypes.c_void_p * K)(*[o.ctypes.data for o in out])


def scan_generic(op, xs, init=None):
    """Inclusive scan y_i = init (.) xs_0 (.) ... (.) xs_i (init None: the
    neutral element): a list of K arrays."""
    xs, ptrs, n, K = _components(op, xs)
    ys, yptr = _arrays(K, n)
    ini = None if init is None else _f64(init).reshape(K)
    _check(lib().orc_scan_generic_from(_gop(op), n, _p(ini), ptrs, yptr), "scan_generic")
    return ys


def scan_generic_vjp(op, xs, y_bar, init=None):
    """Adjoints of every input element given the adjoints of every output
    (y_bar: list of K arrays).  init: the state the fold starts from (K
    values; None: the neutral element)."""
    xs, ptrs, n, K = _components(op, xs)
    yb = [_f64(y) for y in y_bar]
    if len(yb) != K or any(y.size != n for y in yb):
        raise ValueError("y_bar must be K arrays of n")
    ybp = (ctypes.c_void_p * K)(*[y.ctypes.data for y in yb])
    out, optr = _arrays(K, n)
    ini = None if init is None else _f64(init).reshape(K)
    _check(lib().orc_scan_generic_vjp_from(_gop(op), n, _p(ini), ptrs, ybp, optr), "scan_generic_vjp")
    return out


# ------------------------------------------------------------ forward mode
def reduce_jvp(op, x, x_dot):
    op = OPS.get(op, op)
    x, xd = _f64(x), _f64(x_dot)
    yd = ctypes.c_double()
    _check(lib().orc_reduce_jvp(op, x.size, _p(x), _p(xd), ctypes.byref(yd)), "reduce_jvp")
    return yd.value


def hist_jvp(op, inds, vs, vs_dot, m):
    op = OPS.get(op, op)
    inds, vs, vd = _i32(inds), _f64(vs), _f64(vs_dot)
    out = np.empty(m)
    _check(lib().orc_hist_jvp(op, vs.size, m, _p(inds), _p(vs), _p(vd), _p(out)), "hist_jvp")
    return out


def scatter_jvp(xs_dot, is_, vs_dot):
    xd, is_, vd = _f64(xs_dot), _i32(is_), _f64(vs_dot)
    out = np.empty(xd.size)
    _check(lib().orc_scatter_jvp(xd.size, _p(xd), is_.size, _p(is_), _p(vd), _p(out)), "scatter_jvp")
    return out


def map_jvp(fn, x, x_dot):
    fn = FNS.get(fn, fn)
    x, xd = _f64(x), _f64(x_dot)
    out = np.empty(x.size)
    _check(lib().orc_map_jvp(fn, x.size, _p(x), _p(xd), _p(out)), "map_jvp")
    return out


def reduce_generic_jvp(op, xs, xs_dot):
    xs, ptrs, n, K = _components(op, xs)
    xd, dptrs, n2, _ = _components(op, xs_dot)
    out = np.empty(K)
    _check(lib().orc_reduce_generic_jvp(_gop(op), n, ptrs, dptrs, _p(out)), "reduce_generic_jvp")
    return out


def scan_generic_jvp(op, xs, xs_dot, init=None):
    """Tangents of every output; init: the (constant) state the fold starts
    from, None for the neutral element."""
    xs, ptrs, n, K = _components(op, xs)
    xd, dptrs, n2, _ = _components(op, xs_dot)
    out, optr = _arrays(K, n)
    ini = None if init is None else _f64(init).reshape(K)
    _check(lib().orc_scan_generic_jvp_from(_gop(op), n, _p(ini), ptrs, dptrs, optr), "scan_generic_jvp")
    return out


# ------------------------------------------------------------------ k-means
def kmeans_objective(X, C):
    """(f, assign [N] int32)."""
    X, C = _f64(X), _f64(C)
    N, D = X.shape
    K = C.shape[0]
    a = np.empty(N, dtype=np.int32)
    f = ctypes.c_double()
    _check(lib().orc_kmeans_objective(N, D, K, _p(X), _p(C), _p(a), ctypes.byref(f)), "kmeans_objective")
    return f.value, a


def kmeans_vjp(X, C, f_bar=1.0):
    X, C = _f64(X), _f64(C)
    N, D = X.shape
    out = np.empty_like(C)
    _check(lib().orc_kmeans_vjp(N, D, C.shape[0], _p(X), _p(C), float(f_bar), _p(out)), "kmeans_vjp")
    return out


def kmeans_hvp(X, C, C_dot, f_bar=1.0):
    X, C, Cd = _f64(X), _f64(C), _f64(C_dot)
    N, D = X.shape
    out = np.empty_like(C)
    _check(lib().orc_kmeans_hvp(N, D, C.shape[0], _p(X), _p(C), float(f_bar), _p(Cd), _p(out)), "kmeans_hvp")
    return out


# ------------------------------------------------------------- gather map
GMAP = {"gather": 0, "mul": 1, "sqdiff": 2}


def gather_map(op, as_, is_, vs=None):
    """ys[i] = f(as[is[i]], vs[i]) (Sec. 5.4: a map reading a free array)."""
    o = GMAP[op]
    as_, is_ = _f64(as_), _i32(is_)
    vs = _f64(vs) if vs is not None else np.zeros(is_.size)
    ys = np.empty(is_.size)
    _check(lib().orc_gather_map(o, as_.size, _p(as_), is_.size, _p(is_), _p(vs), _p(ys)), "gather_map")
    return ys


def gather_map_vjp(op, as_, is_, vs, ys_bar):
    """(as_bar, vs_bar or None): the read's adjoints accumulated into as_bar."""
    o = GMAP[op]
    as_, is_, yb = _f64(as_), _i32(is_), _f64(ys_bar)
    vs = _f64(vs) if vs is not None else np.zeros(is_.size)
    ab, vb = np.empty(as_.size), np.empty(is_.size)
    _check(lib().orc_gather_map_vjp(o, as_.size, _p(as_), is_.size, _p(is_), _p(vs), _p(yb), _p(ab), _p(vb)),
           "gather_map_vjp")
    return ab, (vb if o else None)


def scan_generic_rows(op, xs):
    """Each row of the [B, L] component arrays scanned on its own (a regular
    segmented scan): the single-scan oracle applied row by row."""
    xs = [np.atleast_2d(_f64(x)) for x in xs]
    out = [np.empty_like(x) for x in xs]
    for b in range(xs[0].shape[0]):
        ys = scan_generic(op, [x[b] for x in xs])
        for o, y in zip(out, ys):
            o[b] = y
    return out


def scan_generic_rows_vjp(op, xs, ys_bar):
    """The VJP of scan_generic_rows, row by row."""
    xs = [np.atleast_2d(_f64(x)) for x in xs]
    yb = [np.atleast_2d(_f64(y)) for y in ys_bar]
    out = [np.empty_like(x) for x in xs]
    for b in range(xs[0].shape[0]):
        g = scan_generic_vjp(op, [x[b] for x in xs], [y[b] for y in yb])
        for o, v in zip(out, g):
            o[b] = v
    return out


# ---------------------------------------------------------- sparse k-means
def _i64(x):
    return np.ascontiguousarray(np.asarray(x, dtype=np.int64))


def sparse_kmeans_objective(rowptr, col, val, D, C):
    """(f, assign) for CSR points and dense centres C [K, D] (Sec. 7.5)."""
    rp, cl, v, C = _i64(rowptr), _i32(col), _f64(val), _f64(C)
    N = rp.size - 1
    a = np.empty(N, dtype=np.int32)
    f = np.zeros(1)
    _check(lib().orc_skm_objective(N, D, C.shape[0], _p(rp), _p(cl), _p(v), _p(C), _p(a), _p(f)),
           "sparse_kmeans_objective")
    return float(f[0]), a


def sparse_kmeans_distances(rowptr, col, val, D, C):
    """[N, K]: every row's squared distance to every centre."""
    rp, cl, v, C = _i64(rowptr), _i32(col), _f64(val), _f64(C)
    N = rp.size - 1
    out = np.empty((N, C.shape[0]))
    _check(lib().orc_skm_dist(N, D, C.shape[0], _p(rp), _p(cl), _p(v), _p(C), _p(out)), "sparse_kmeans_distances")
    return out


def sparse_kmeans_vjp(rowptr, col, val, D, C, f_bar=1.0):
    rp, cl, v, C = _i64(rowptr), _i32(col), _f64(val), _f64(C)
    out = np.empty_like(C)
    _check(lib().orc_skm_vjp(rp.size - 1, D, C.shape[0], _p(rp), _p(cl), _p(v), _p(C), float(f_bar), _p(out)),
           "sparse_kmeans_vjp")
    return out


def sparse_kmeans_hvp(rowptr, col, val, D, C, C_dot, f_bar=1.0):
    rp, cl, v, C, Cd = _i64(rowptr), _i32(col), _f64(val), _f64(C), _f64(C_dot)
    out = np.empty_like(C)
    _check(lib().orc_skm_hvp(rp.size - 1, D, C.shape[0], _p(rp), _p(cl), _p(v), _p(C), float(f_bar), _p(Cd),
                             _p(out)), "sparse_kmeans_hvp")
    return out


# ------------------------------------------- reduce_by_index, general operator
def hist_generic(op, inds, xs, m):
    """hs: K arrays [m], the index-order fold of each bin (Sec. 5.1.2)."""
    xs, ptrs, n, K = _components(op, xs)
    inds = _i32(inds)
    hs = [np.empty(m) for _ in range(K)]
    hp = (ctypes.c_void_p * K)(*[h.ctypes.data for h in hs])
    _check(lib().orc_hist_generic(_gop(op), n, m, _p(inds), ptrs, hp), "hist_generic")
    return hs


def hist_generic_vjp(op, inds, xs, hs_bar):
    """x_bar: K arrays [n], the general rule applied within each bin."""
    xs, ptrs, n, K = _components(op, xs)
    inds = _i32(inds)
    hb = [_f64(h) for h in hs_bar]
    m = hb[0].size
    hbp = (ctypes.c_void_p * K)(*[h.ctypes.data for h in hb])
    out = [np.empty(n) for _ in range(K)]
    op_ = (ctypes.c_void_p * K)(*[o.ctypes.data for o in out])
    _check(lib().orc_hist_generic_vjp(_gop(op), n, m, _p(inds), ptrs, hbp, op_), "hist_generic_vjp")
    return out
