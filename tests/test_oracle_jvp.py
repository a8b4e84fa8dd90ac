"""Pins for the oracle's forward mode (Sec. 3): Jacobian-vector products from a
forward sweep over the same tape records the VJPs sweep backwards.

Each is checked against something other than itself: the dot-product
identity <y_bar, J x_dot> = <J^T y_bar, x_dot> with the separately pinned
VJPs, central finite differences of independently written numpy primals,
and closed forms (the tangent of a sum is the sum of the tangents, of a
maximum the tangent of the winner, of a scatter the scattered tangents).
"""
import numpy as np
import pytest
from scipy.special import logsumexp

from _util import rel_l2
from paper_2202_10297_amd import workloads


def _g(seed):
    return workloads.rng(seed)


@pytest.mark.parametrize("op", ["add", "mul", "min", "max"])
def test_reduce_jvp_dot_product(orc, op):
    g = _g(1)
    x = workloads.product_values(60, 0, "f64", seed=3) if op == "mul" else g.standard_normal(60)
    xd, yb = g.standard_normal(60), 0.7
    yd = orc.reduce_jvp(op, x, xd)
    xb = orc.reduce_vjp(op, x, yb)
    assert abs(yb * yd - np.dot(xb, xd)) <= 1e-13 * max(1.0, abs(yb * yd))


def test_reduce_jvp_closed_forms(orc):
    g = _g(2)
    x, xd = g.standard_normal(100), g.standard_normal(100)
    assert abs(orc.reduce_jvp("add", x, xd) - np.sum(xd)) <= 1e-13
    assert orc.reduce_jvp("max", x, xd) == xd[np.argmax(x)]
    assert orc.reduce_jvp("min", x, xd) == xd[np.argmin(x)]
    p = workloads.product_values(20, 0, "f64", seed=4)
    h = 1e-6
    fd = (np.prod(p + h * xd[:20]) - np.prod(p - h * xd[:20])) / (2 * h)
    assert abs(orc.reduce_jvp("mul", p, xd[:20]) - fd) <= 1e-7 * max(1.0, abs(fd))
    # one zero: only that element's tangent survives, times the other factors
    p[5] = 0.0
    assert abs(orc.reduce_jvp("mul", p, xd[:20]) - xd[5] * np.prod(np.delete(p, 5))) <= 1e-12


@pytest.mark.parametrize("op", ["add", "mul", "min", "max"])
def test_hist_jvp_dot_product(orc, op):
    n, m = 400, 13
    inds, vs, _ = workloads.hist(n, m, "zipf", "f64", seed=5)
    if op == "mul":
        vs = workloads.product_values(n, 0, "f64", seed=6)
    g = _g(7)
    vd, hb = g.standard_normal(n), g.standard_normal(m)
    hd = orc.hist_jvp(op, inds, vs, vd, m)
    vb = orc.hist_vjp(op, inds, vs, hb)
    assert abs(np.dot(hb, hd) - np.dot(vb, vd)) <= 1e-12 * max(1.0, np.abs(hb * hd).sum())


def test_hist_jvp_closed_forms(orc):
    n, m = 500, 17
    inds, vs, _ = workloads.hist(n, m, "uniform", "f64", seed=8)
    vd = _g(9).standard_normal(n)
    assert rel_l2(orc.hist_jvp("add", inds, vs, vd, m), np.bincount(inds, weights=vd, minlength=m)) <= 1e-14
    w = orc.hist("max", inds, vs, m)["winner"]
    ref = np.where(w >= 0, vd[np.maximum(w, 0)], 0.0)
    assert np.array_equal(orc.hist_jvp("max", inds, vs, vd, m), ref)


def test_scatter_jvp_is_the_scattered_tangents(orc):
    n, m = 300, 90
    xs, is_, vs, _ = workloads.scatter(n, m, "f64", seed=10)
    g = _g(11)
    xd, vd = g.standard_normal(n), g.standard_normal(m)
    ref = xd.copy()
    ref[is_] = vd
    assert np.array_equal(orc.scatter_jvp(xd, is_, vd), ref)


@pytest.mark.parametrize("fn", ["square", "exp", "log", "sin", "tanh"])
def test_map_jvp_finite_differences(orc, fn):
    g = _g(12)
    x = g.uniform(0.5, 2.0, 50)
    xd = g.standard_normal(50)
    f = {"square": np.square, "exp": np.exp, "log": np.log, "sin": np.sin, "tanh": np.tanh}[fn]
    h = 1e-6
    fd = (f(x + h * xd) - f(x - h * xd)) / (2 * h)
    assert rel_l2(orc.map_jvp(fn, x, xd), fd) <= 1e-8


@pytest.mark.parametrize("op", ["logaddexp", "linrec", "mat2"])
def test_generic_jvp_dot_products(orc, op):
    n = 40
    xs, yb = workloads.gop(op, n, seed=13, general=(op == "mat2"))
    g = _g(14)
    xd = [g.standard_normal(n) for _ in xs]
    yd = orc.reduce_generic_jvp(op, xs, xd)
    xb = orc.reduce_generic_vjp(op, xs, yb)
    lhs, rhs = float(np.dot(yb, yd)), sum(float(np.dot(a, b)) for a, b in zip(xb, xd))
    assert abs(lhs - rhs) <= 1e-12 * max(1.0, abs(lhs))
    _, ybs = workloads.gop_scan(op, n, seed=15, general=(op == "mat2"))
    yds = orc.scan_generic_jvp(op, xs, xd)
    xbs = orc.scan_generic_vjp(op, xs, ybs)
    lhs = sum(float(np.dot(a, b)) for a, b in zip(ybs, yds))
    rhs = sum(float(np.dot(a, b)) for a, b in zip(xbs, xd))
    assert abs(lhs - rhs) <= 1e-12 * max(1.0, abs(lhs))


def test_generic_jvp_finite_differences(orc):
    g = _g(16)
    x = g.standard_normal(30)
    xd = g.standard_normal(30)
    h = 1e-6
    fd = (logsumexp(x + h * xd) - logsumexp(x - h * xd)) / (2 * h)
    assert abs(orc.reduce_generic_jvp("logaddexp", [x], [xd])[0] - fd) <= 1e-8
    fds = (np.logaddexp.accumulate(x + h * xd) - np.logaddexp.accumulate(x - h * xd)) / (2 * h)
    assert rel_l2(orc.scan_generic_jvp("logaddexp", [x], [xd]), [fds]) <= 1e-8
    # the tangent of a log-sum-exp prefix with all tangents 1 is 1
    assert np.allclose(orc.scan_generic_jvp("logaddexp", [x], [np.ones(30)])[0], 1.0, rtol=1e-14)


@pytest.mark.parametrize("op", ["logaddexp", "linrec", "mat2"])
def test_scan_jvp_window_from_a_prefix_state(orc, op):
    # with tangents zero before a window, the window's output tangents come
    # from the fold started at the state of everything before it
    n, w = 300, 100
    xs, _ = workloads.gop_scan(op, n, seed=41)
    g = _g(42)
    xd = [np.concatenate([np.zeros(n - w), g.standard_normal(w)]) for _ in xs]
    full = orc.scan_generic_jvp(op, xs, xd)
    init = orc.reduce_generic(op, [x[:n - w] for x in xs])
    win = orc.scan_generic_jvp(op, [x[n - w:] for x in xs], [t[n - w:] for t in xd], init=init)
    assert rel_l2(win, [f[n - w:] for f in full]) <= 1e-13
