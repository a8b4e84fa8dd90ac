"""Seeded synthetic inputs shaped like the paper's workloads.

This module holds no arithmetic of the method: it only draws random inputs
(numpy ``Generator(PCG64(seed))``, draws in the order listed in each
function).  Both the GPU tests and the CPU oracle tests take their inputs from
here, so the two sides see identical data.

Shapes and distributions follow the operator workloads the library is
measured on:

* linear-recurrence scan: a ~ U[0.5, 1), b ~ N(0, 1), output adjoints
  (yA_bar, yB_bar) i.i.d. N(0, 1);
* reduce_by_index: values ~ N(0, 1) float32, bin indices uniform or Zipf(s)
  on the finite support {1..m} (inverse CDF of pmf ~ k^-s), ranks mapped to
  bins through a seeded permutation so that hot bins are scattered;
* scatter: 2^24-style unique target indices drawn without replacement;
* Gaussian mixture: X ~ N(0,1), alpha ~ N(0,1), mu ~ N(0,1), q and l ~
  N(0, 0.1) (standard deviation 0.1);
* segmented batches: lengths floor(exp(U[ln lo, ln hi]));
* k-means: K well-separated blobs (centres ~ N(0, 9), points = centre +
  N(0, 1)), initial centres = K distinct points drawn without replacement;
* reduce with a general operator: log-add-exp values ~ N(0, 1); linear-
  recurrence pairs as for the scan; 2x2 matrices that are rotations, each
  composed with the reflection diag(1, -1) with probability 1/2, so that
  products of any length stay orthogonal (no overflow or underflow) while
  the factors do not commute.
"""
from __future__ import annotations

import numpy as np


def rng(seed: int = 0) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def _dt(dtype):
    return np.dtype({"f32": np.float32, "f64": np.float64}.get(dtype, dtype))


def linrec(n: int, dtype="f64", seed: int = 0):
    """(a, b, yA_bar, yB_bar) for the first-order linear recurrence scan."""
    g = rng(seed)
    dt = _dt(dtype)
    a = g.uniform(0.5, 1.0, n).astype(dt)
    b = g.standard_normal(n).astype(dt)
    ya = g.standard_normal(n).astype(dt)
    yb = g.standard_normal(n).astype(dt)
    return a, b, ya, yb


def zipf_indices(n: int, m: int, s: float, g: np.random.Generator) -> np.ndarray:
    """n bin indices in [0, m): Zipf(s) ranks on {1..m} by inverse CDF, then a
    seeded permutation maps rank -> bin."""
    k = np.arange(1, m + 1, dtype=np.float64)
    cdf = np.cumsum(k ** (-s))
    cdf /= cdf[-1]
    out = np.empty(n, dtype=np.int32)
    step = 1 << 22
    for lo in range(0, n, step):
        u = g.random(min(step, n - lo))
        r = np.searchsorted(cdf, u, side="right")
        np.minimum(r, m - 1, out=r)
        out[lo:lo + r.size] = r
    perm = g.permutation(m).astype(np.int32)
    return perm[out]


def hist(n: int, m: int, dist: str = "uniform", dtype="f32", seed: int = 0, s: float = 1.1):
    """(inds, vs, hs_bar) for reduce_by_index."""
    g = rng(seed)
    dt = _dt(dtype)
    vs = g.standard_normal(n, dtype=np.float32 if dt == np.float32 else np.float64).astype(dt)
    if dist == "uniform":
        inds = g.integers(0, m, n, dtype=np.int32)
    elif dist == "zipf":
        inds = zipf_indices(n, m, s, g)
    else:
        raise ValueError(dist)
    hs_bar = g.standard_normal(m).astype(dt)
    return inds, vs, hs_bar


def gather_map(m: int, n: int, dist: str = "uniform", dtype="f32", seed: int = 0):
    """(as_, is_, vs, ys_bar) for a map reading the free array as_ [n] at
    indices is_ [m] (uniform, or Zipf(1.1) over n as for the histograms)."""
    is_, vs, _ = hist(m, n, dist, dtype, seed)
    g = rng(seed + 1)
    dt = _dt(dtype)
    as_ = g.standard_normal(n).astype(dt)
    ys_bar = g.standard_normal(m).astype(dt)
    return as_, is_, vs, ys_bar


def sparse_kmeans(N: int, D: int, K: int, nnz_mean: float = 50.0, dtype="f32", seed: int = 0):
    """(rowptr [N+1] int64, col [nnz] int32, val [nnz], C [K, D]) for sparse
    k-means: bag-of-words-like rows whose lengths are drawn log-normal around
    nnz_mean (capped at D), columns Zipf(1.1) over D with repeats in a row
    dropped (so a row keeps its distinct draws, sorted), counts 1..4 as
    values; initial centres = K distinct rows, densified."""
    g = rng(seed)
    dt = _dt(dtype)
    lens = np.minimum(np.maximum(np.round(g.lognormal(np.log(nnz_mean), 0.6, N)), 0), D).astype(np.int64)
    rows = np.repeat(np.arange(N, dtype=np.int64), lens)
    cols = zipf_indices(int(lens.sum()), D, 1.1, g).astype(np.int64)
    keys = np.unique(rows * D + cols)
    rowptr = np.zeros(N + 1, dtype=np.int64)
    rowptr[1:] = np.cumsum(np.bincount(keys // D, minlength=N))
    col = (keys % D).astype(np.int32)
    val = g.integers(1, 5, col.size).astype(dt)
    pick = g.choice(N, size=min(K, N), replace=False) if N else np.zeros(0, dtype=np.int64)
    C = np.zeros((K, D), dtype=dt)
    for r, i in enumerate(pick):
        C[r, col[rowptr[i]:rowptr[i + 1]]] = val[rowptr[i]:rowptr[i + 1]]
    return rowptr, col, val, C


def tie_values(n: int, dtype="f32", seed: int = 0):
    """Values quantised to multiples of 2^-4 in [-4, 4]: many exact ties."""
    g = rng(seed)
    return (g.integers(-64, 65, n) / 16.0).astype(_dt(dtype))


def product_values(n: int, zeros: int, dtype="f32", seed: int = 0):
    """Values in +-U[0.5, 2) with `zeros` elements set to zero (half of them
    negative zero) at seeded positions."""
    g = rng(seed)
    v = g.uniform(0.5, 2.0, n) * np.where(g.random(n) < 0.5, -1.0, 1.0)
    if zeros:
        pos = g.choice(n, size=min(zeros, n), replace=False)
        v[pos] = 0.0
        v[pos[::2]] = -0.0
    return v.astype(_dt(dtype))


def scatter(n: int, m: int, dtype="f32", seed: int = 0):
    """(xs, is, vs, ys_bar): m unique targets in [0, n) in random order."""
    g = rng(seed)
    dt = _dt(dtype)
    xs = g.standard_normal(n).astype(dt)
    if m * 4 >= n:
        is_ = g.permutation(n)[:m].astype(np.int32)
    else:
        is_ = g.choice(n, size=m, replace=False).astype(np.int32)
    vs = g.standard_normal(m).astype(dt)
    ys_bar = g.standard_normal(n).astype(dt)
    return xs, is_, vs, ys_bar


def gmm(N: int, D: int, K: int, seed: int = 0, dtype="f32"):
    """(X, alpha, mu, q, l) with l the K x D(D-1)/2 strictly-lower entries."""
    g = rng(seed)
    dt = _dt(dtype)
    X = g.standard_normal((N, D)).astype(dt)
    alpha = g.standard_normal(K).astype(dt)
    mu = g.standard_normal((K, D)).astype(dt)
    q = (0.1 * g.standard_normal((K, D))).astype(dt)
    l = (0.1 * g.standard_normal((K, D * (D - 1) // 2))).astype(dt)
    return X, alpha, mu, q, l


def segment_lengths(nseg: int, lo: int, hi: int, seed: int = 0) -> np.ndarray:
    g = rng(seed)
    return np.floor(np.exp(g.uniform(np.log(lo), np.log(hi), nseg))).astype(np.int64)


def gop(op: str, n: int, dtype="f64", seed: int = 0, general: bool = False):
    """(components, y_bar) for a reduce with a general operator.  components
    is a list of K arrays of length n; y_bar has K entries ~ N(0, 1).  With
    `general`, mat2 factors are dense N(0, 1/2) matrices instead (short
    inputs only: their products grow or shrink geometrically)."""
    g = rng(seed)
    dt = _dt(dtype)
    if op == "logaddexp":
        xs = [g.standard_normal(n).astype(dt)]
        yb = g.standard_normal(1).astype(dt)
    elif op == "linrec":
        xs = [g.uniform(0.5, 1.0, n).astype(dt), g.standard_normal(n).astype(dt)]
        yb = g.standard_normal(2).astype(dt)
    elif op == "mat2":
        if general:
            m = g.standard_normal((4, n)) * np.sqrt(0.5)
        else:
            th = g.uniform(-np.pi, np.pi, n)
            f = np.where(g.random(n) < 0.5, -1.0, 1.0)
            c, s_ = np.cos(th), np.sin(th)
            # [[c, -s], [s, c]] @ diag(1, f)
            m = np.stack([c, -s_ * f, s_, c * f])
        xs = [m[k].astype(dt) for k in range(4)]
        yb = g.standard_normal(4).astype(dt)
    else:
        raise ValueError(f"unknown operator {op}")
    return xs, yb


def gop_scan(op: str, n: int, dtype="f64", seed: int = 0, general: bool = False):
    """(components, y_bar) for an inclusive scan with a general operator:
    the components as in gop(); y_bar is a list of K arrays ~ N(0, 1), one
    output adjoint per element and component."""
    xs, _ = gop(op, n, dtype, seed, general)
    g = rng(seed + 7777)
    dt = _dt(dtype)
    return xs, [g.standard_normal(n).astype(dt) for _ in xs]


def kmeans(N: int, D: int, K: int, dtype="f32", seed: int = 0):
    """(X [N, D], C [K, D]) for k-means: points around K random blob centres,
    initial centres = K distinct points."""
    g = rng(seed)
    dt = _dt(dtype)
    centres = g.standard_normal((K, D)) * 3.0
    lab = g.integers(0, K, N)
    X = (centres[lab] + g.standard_normal((N, D))).astype(dt)
    pick = g.choice(N, size=K, replace=False) if N >= K else np.arange(N)
    C = X[pick].copy()
    return X, C


def hist_generic(op: str, n: int, m: int, dist: str = "uniform", dtype="f64", seed: int = 0):
    """(inds, components, hs_bar) for reduce_by_index with a general operator:
    indices as for hist() (uniform or Zipf(1.1) over m), components as for
    gop(), hs_bar a list of K arrays [m] ~ N(0, 1)."""
    inds, _, _ = hist(n, m, dist, "f32", seed=seed)
    xs, _ = gop(op, n, dtype, seed=seed + 1)
    g = rng(seed + 2)
    dt = _dt(dtype)
    return inds, xs, [g.standard_normal(m).astype(dt) for _ in xs]
