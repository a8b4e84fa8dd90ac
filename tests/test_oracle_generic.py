"""Pins for the oracle's reduce (Sec. 5.1.1, general rule) and inclusive scan
(Sec. 5.2, Jacobian generalisation) with a general associative operator, and
their VJPs.

The oracle folds x_0 (.) ... (.) x_{n-1} on a tape; these pins check it
against things other than itself: library routines (logsumexp, softmax,
chained matrix products), closed forms, central finite differences of
independently written primal functions, an invariant of multilinear maps and
the oracle's separately pinned scan VJP.
"""
import functools

import numpy as np
import pytest
from scipy.special import logsumexp, softmax

from _util import fd_grad, rel_l2
from paper_2202_10297_amd import workloads


def _mats(xs):
    return [np.array([[xs[0][i], xs[1][i]], [xs[2][i], xs[3][i]]]) for i in range(xs[0].size)]


def _matprod(xs):
    return functools.reduce(np.matmul, _mats(xs), np.eye(2))


def _linrec_closed(a, b):
    # yA = prod a_k; yB = sum_j b_j prod_{k>j} a_k
    tail = np.concatenate([np.cumprod(a[::-1])[::-1][1:], [1.0]])
    return np.prod(a), np.sum(b * tail)


@pytest.mark.parametrize("n", [1, 7, 1000])
def test_logaddexp_primal_is_logsumexp(orc, n):
    (x,), _ = workloads.gop("logaddexp", n, seed=n)
    if n > 2:
        x[1] = -np.inf
    y = orc.reduce_generic("logaddexp", [x])
    assert abs(y[0] - logsumexp(x)) <= 1e-14 * abs(logsumexp(x)) + 1e-15


@pytest.mark.parametrize("n", [1, 7, 1000])
def test_logaddexp_vjp_is_softmax(orc, n):
    (x,), yb = workloads.gop("logaddexp", n, seed=n + 1)
    if n > 2:
        x[n // 2] = -np.inf
    (xb,) = orc.reduce_generic_vjp("logaddexp", [x], yb)
    ref = yb[0] * softmax(x)
    assert rel_l2(xb, ref) <= 1e-13
    if n > 2:
        assert xb[n // 2] == 0.0


def test_logaddexp_degenerate(orc):
    assert orc.reduce_generic("logaddexp", [np.zeros(0)])[0] == -np.inf
    x = np.full(5, -np.inf)
    assert orc.reduce_generic("logaddexp", [x])[0] == -np.inf
    (xb,) = orc.reduce_generic_vjp("logaddexp", [x], [1.0])
    assert np.array_equal(xb, np.zeros(5))


@pytest.mark.parametrize("n", [1, 2, 50, 300])
def test_linrec_primal_closed_form(orc, n):
    (a, b), _ = workloads.gop("linrec", n, seed=n)
    y = orc.reduce_generic("linrec", [a, b])
    yA, yB = _linrec_closed(a, b)
    assert abs(y[0] - yA) <= 1e-14 * abs(yA)
    assert abs(y[1] - yB) <= 1e-13 * max(1.0, np.abs(b).sum())


def test_linrec_vjp_finite_differences(orc):
    (a, b), yb = workloads.gop("linrec", 6, seed=11)
    ab, bb = orc.reduce_generic_vjp("linrec", [a, b], yb)

    def L(a_, b_):
        yA, yB = _linrec_closed(a_, b_)
        return yb[0] * yA + yb[1] * yB

    ga, gb = fd_grad(L, [a, b])
    assert rel_l2([ab, bb], [ga, gb]) <= 1e-8


def test_linrec_vjp_is_scan_vjp_seeded_at_the_end(orc):
    # The reduce is the last element of the inclusive scan, so its adjoint is
    # the scan adjoint with the output adjoint seeded at the last position
    # only (scan oracle: pinned separately).
    n = 300
    (a, b), yb = workloads.gop("linrec", n, seed=5)
    ya, ybb = np.zeros(n), np.zeros(n)
    ya[-1], ybb[-1] = yb
    ref = orc.linrec_scan_vjp(a, b, ya, ybb)
    got = orc.reduce_generic_vjp("linrec", [a, b], yb)
    assert rel_l2(got, list(ref)) <= 1e-14


@pytest.mark.parametrize("general", [False, True])
def test_mat2_primal_is_matrix_chain(orc, general):
    xs, _ = workloads.gop("mat2", 40, seed=2, general=general)
    y = orc.reduce_generic("mat2", xs)
    ref = _matprod(xs)
    assert rel_l2(y, ref.reshape(-1)) <= 1e-14


def test_mat2_rotations_stay_orthogonal(orc):
    xs, _ = workloads.gop("mat2", 4096, seed=9)
    Y = np.asarray(orc.reduce_generic("mat2", xs)).reshape(2, 2)
    assert np.allclose(Y @ Y.T, np.eye(2), atol=1e-12)


def test_mat2_vjp_finite_differences(orc):
    xs, yb = workloads.gop("mat2", 5, seed=4, general=True)
    got = orc.reduce_generic_vjp("mat2", xs, yb)

    def L(*comp):
        return float(np.sum(_matprod(list(comp)).reshape(-1) * yb))

    ref = fd_grad(L, xs)
    assert rel_l2(got, ref) <= 1e-8


@pytest.mark.parametrize("general", [False, True])
def test_mat2_vjp_multilinear_identity(orc, general):
    # Y is linear in each factor, so sum_i <A_bar_i, A_i> = n <Y_bar, Y>.
    n = 12 if general else 64
    xs, yb = workloads.gop("mat2", n, seed=8, general=general)
    got = orc.reduce_generic_vjp("mat2", xs, yb)
    lhs = sum(float(np.dot(g, x)) for g, x in zip(got, xs))
    rhs = n * float(np.dot(yb, _matprod(xs).reshape(-1)))
    assert abs(lhs - rhs) <= 1e-12 * max(1.0, abs(rhs))


def test_single_element_adjoint_is_the_output_adjoint(orc):
    # With n == 1 the fold is e (.) x_0 == x_0, so x_bar == y_bar.
    for op, K in (("logaddexp", 1), ("linrec", 2), ("mat2", 4)):
        xs, yb = workloads.gop(op, 1, seed=3)
        got = orc.reduce_generic_vjp(op, xs, yb)
        assert np.allclose([g[0] for g in got], yb, rtol=1e-15, atol=0), op


def test_empty_gives_the_neutral_element(orc):
    assert list(orc.reduce_generic("linrec", [np.zeros(0)] * 2)) == [1.0, 0.0]
    assert list(orc.reduce_generic("mat2", [np.zeros(0)] * 4)) == [1.0, 0.0, 0.0, 1.0]


@pytest.mark.parametrize("op", ["logaddexp", "linrec", "mat2"])
def test_sampled_adjoints_match_the_full_sweep(orc, op):
    n = 777
    xs, yb = workloads.gop(op, n, seed=21)
    full = orc.reduce_generic_vjp(op, xs, yb)
    idx = np.array([0, n - 1, 5, 5, 400, 123, 776, 1])
    got = orc.reduce_generic_vjp_at(op, xs, yb, idx)
    ref = np.stack([f[idx] for f in full], axis=1)
    assert rel_l2(got, ref) <= 1e-13


# ------------------------------------------------- inclusive scan, general operator
def _matscan(xs):
    out, acc = [], np.eye(2)
    for m in _mats(xs):
        acc = acc @ m
        out.append(acc.reshape(-1))
    return np.array(out).T  # K x n


@pytest.mark.parametrize("n", [1, 9, 500])
def test_scan_logaddexp_is_logaddexp_accumulate(orc, n):
    (x,), _ = workloads.gop_scan("logaddexp", n, seed=n)
    if n > 3:
        x[2] = -np.inf
    (y,) = orc.scan_generic("logaddexp", [x])
    assert rel_l2(y, np.logaddexp.accumulate(x)) <= 1e-14


def test_scan_logaddexp_vjp_closed_form(orc):
    # y_i = log sum_{j<=i} e^{x_j}, so x_bar_j = sum_{i>=j} y_bar_i e^{x_j - y_i}
    n = 200
    (x,), (yb,) = workloads.gop_scan("logaddexp", n, seed=3)
    x[7] = -np.inf
    y = np.logaddexp.accumulate(x)
    ref = np.array([np.sum(yb[j:] * np.exp(x[j] - y[j:])) for j in range(n)])
    (got,) = orc.scan_generic_vjp("logaddexp", [x], [yb])
    assert rel_l2(got, ref) <= 1e-13
    assert got[7] == 0.0


def test_scan_logaddexp_vjp_finite_differences(orc):
    (x,), (yb,) = workloads.gop_scan("logaddexp", 6, seed=4)
    (got,) = orc.scan_generic_vjp("logaddexp", [x], [yb])
    (ref,) = fd_grad(lambda x_: float(np.dot(yb, np.logaddexp.accumulate(x_))), [x])
    assert rel_l2(got, ref) <= 1e-8


def test_scan_linrec_matches_the_pinned_scan(orc):
    n = 300
    (a, b), (ya, yb) = workloads.gop_scan("linrec", n, seed=6)
    A, B = orc.scan_generic("linrec", [a, b])
    RA, RB = orc.linrec_scan(a, b)
    assert rel_l2([A, B], [RA, RB]) <= 1e-15
    got = orc.scan_generic_vjp("linrec", [a, b], [ya, yb])
    assert rel_l2(got, list(orc.linrec_scan_vjp(a, b, ya, yb))) <= 1e-14


@pytest.mark.parametrize("general", [False, True])
def test_scan_mat2_is_cumulative_matrix_product(orc, general):
    xs, _ = workloads.gop_scan("mat2", 30, seed=2, general=general)
    ys = orc.scan_generic("mat2", xs)
    assert rel_l2(ys, list(_matscan(xs))) <= 1e-14


def test_scan_mat2_vjp_finite_differences(orc):
    xs, ybs = workloads.gop_scan("mat2", 5, seed=12, general=True)
    got = orc.scan_generic_vjp("mat2", xs, ybs)

    def L(*comp):
        return float(np.sum(_matscan(list(comp)) * np.array(ybs)))

    assert rel_l2(got, fd_grad(L, xs)) <= 1e-8


@pytest.mark.parametrize("general", [False, True])
def test_scan_mat2_vjp_multilinear_identity(orc, general):
    # Y_i is linear in each of X_0..X_i, so sum_j <X_bar_j, X_j> = sum_i (i+1) <Y_bar_i, Y_i>
    n = 10 if general else 80
    xs, ybs = workloads.gop_scan("mat2", n, seed=15, general=general)
    got = orc.scan_generic_vjp("mat2", xs, ybs)
    lhs = sum(float(np.dot(g, x)) for g, x in zip(got, xs))
    Y = _matscan(xs)
    rhs = float(np.sum((np.arange(n) + 1) * np.sum(np.array(ybs) * Y, axis=0)))
    assert abs(lhs - rhs) <= 1e-12 * max(1.0, abs(rhs))


def test_scan_single_element(orc):
    for op in ("logaddexp", "linrec", "mat2"):
        xs, ybs = workloads.gop_scan(op, 1, seed=1)
        got = orc.scan_generic_vjp(op, xs, ybs)
        assert np.allclose([g[0] for g in got], [y[0] for y in ybs], rtol=1e-15, atol=0), op


@pytest.mark.parametrize("op", ["logaddexp", "linrec", "mat2"])
def test_scan_window_from_a_prefix_state(orc, op):
    # The adjoints of the last w elements for the last w output adjoints do
    # not depend on the earlier adjoints: a fold started from the state of
    # the first n - w elements reproduces them.
    n, w = 400, 150
    xs, ybs = workloads.gop_scan(op, n, seed=31)
    ybw = [np.concatenate([np.zeros(n - w), y[n - w:]]) for y in ybs]
    full = orc.scan_generic_vjp(op, xs, ybw)
    init = orc.reduce_generic(op, [x[:n - w] for x in xs])
    tail = orc.scan_generic_vjp(op, [x[n - w:] for x in xs], [y[n - w:] for y in ybs], init=init)
    assert rel_l2(tail, [f[n - w:] for f in full]) <= 1e-13
