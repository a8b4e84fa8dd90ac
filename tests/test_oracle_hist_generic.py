"""Pins for the oracle's reduce_by_index with a general operator (Sec. 5.1.2
with the general rule of Sec. 5.1.1 inside each bin): every bin's fold in
index order and the per-bin adjoints.

Checked against scipy's logsumexp per bin and the softmax closed form of its
adjoint, numpy's chained 2 x 2 products per bin (order matters: the operator
does not commute), the linear recurrence's closed form per bin, central
differences of those numpy primals, the neutral element for empty bins and
zero adjoints for indices out of range.
"""
import numpy as np
import pytest
from scipy.special import logsumexp

from _util import rel_l2
from paper_2202_10297_amd import workloads


def bins_of(inds, m):
    return [np.nonzero(inds == b)[0] for b in range(m)]


def np_fold(op, xs, idx):
    if op == "logaddexp":
        return [logsumexp(xs[0][idx]) if idx.size else -np.inf]
    if op == "linrec":
        A, B = 1.0, 0.0
        for i in idx:
            A, B = xs[0][i] * A, xs[0][i] * B + xs[1][i]
        return [A, B]
    M = np.eye(2)
    for i in idx:
        M = M @ np.array([[xs[0][i], xs[1][i]], [xs[2][i], xs[3][i]]])
    return list(M.reshape(4))


def inputs(op, n, m, seed):
    xs, _ = workloads.gop(op, n, "f64", seed=seed, general=(op == "mat2"))
    inds = workloads.rng(seed + 1).integers(-1, m + 1, n).astype(np.int32)  # some out of range
    return xs, inds


@pytest.mark.parametrize("op", ["logaddexp", "linrec", "mat2"])
@pytest.mark.parametrize("n,m", [(1, 1), (40, 5), (300, 17)])
def test_primal_per_bin(orc, op, n, m):
    xs, inds = inputs(op, n, m, seed=n + m)
    hs = orc.hist_generic(op, inds, xs, m)
    for b, idx in enumerate(bins_of(inds, m)):
        ref = np_fold(op, xs, idx)
        got = [h[b] for h in hs]
        if op == "logaddexp" and not idx.size:
            assert got[0] == -np.inf
        else:
            assert rel_l2(got, ref) <= 1e-13


def test_logaddexp_adjoint_is_the_softmax(orc):
    xs, inds = inputs("logaddexp", 500, 7, seed=3)
    hb = workloads.rng(4).standard_normal(7)
    xb = orc.hist_generic_vjp("logaddexp", inds, xs, [hb])[0]
    ref = np.zeros(500)
    for b, idx in enumerate(bins_of(inds, 7)):
        if idx.size:
            ref[idx] = hb[b] * np.exp(xs[0][idx] - logsumexp(xs[0][idx]))
    assert rel_l2(xb, ref) <= 1e-14
    out = (inds < 0) | (inds >= 7)
    assert np.all(xb[out] == 0)


@pytest.mark.parametrize("op", ["logaddexp", "linrec", "mat2"])
def test_adjoint_finite_differences(orc, op):
    n, m = 30, 4
    xs, inds = inputs(op, n, m, seed=9)
    K = len(xs)
    hb = [workloads.rng(10 + c).standard_normal(m) for c in range(K)]
    xb = orc.hist_generic_vjp(op, inds, xs, hb)

    def f(ys):
        tot = 0.0
        for b, idx in enumerate(bins_of(inds, m)):
            if idx.size:
                tot += float(np.dot([h[b] for h in hb], np_fold(op, ys, idx)))
        return tot

    h = 1e-6
    for c in range(K):
        fd = np.empty(n)
        for i in range(n):
            p = [x.copy() for x in xs]
            q = [x.copy() for x in xs]
            p[c][i] += h
            q[c][i] -= h
            fd[i] = (f(p) - f(q)) / (2 * h)
        assert rel_l2(xb[c], fd) <= 1e-7


def test_logaddexp_non_finite_bins(orc):
    # over the extended reals: -inf is neutral, NaN propagates, +inf absorbs;
    # numpy's logaddexp is an independent implementation of the same operator
    x = np.array([0.5, np.inf, -1.0, np.nan, 2.0, -np.inf, np.inf, np.inf, -np.inf, 3.0])
    inds = np.array([0, 0, 0, 1, 1, 2, 3, 3, 4, 5], dtype=np.int32)
    got = orc.hist_generic("logaddexp", inds, [x], 7)[0]
    for b in range(7):
        sel = x[inds == b]
        ref = np.logaddexp.reduce(sel) if sel.size else -np.inf
        assert (np.isnan(got[b]) and np.isnan(ref)) or got[b] == ref, (b, got[b], ref)
    assert np.isposinf(got[0]) and np.isnan(got[1]) and np.isneginf(got[2]) and np.isposinf(got[3])
