"""Pins for the oracle's map over a free array (Sec. 5.4): ys[i] =
f(as[is[i]], vs[i]) and its VJP, whose reads of as become accumulator
updates of as_bar.

Checked against numpy's primal, the closed form of the accumulated adjoint
(`np.add.at` of each read's partial), and the Jacobian of the replicated
formulation (as passed to every element as a bound variable, Sec. 5.4's naive
rewrite) by central differences on small inputs, where every read's
contribution is summed explicitly.
"""
import numpy as np
import pytest

from _util import rel_l2
from paper_2202_10297_amd import workloads

FNS = {
    "gather": (lambda a, v: a, lambda a, v: np.ones_like(a), None),
    "mul": (lambda a, v: a * v, lambda a, v: v, lambda a, v: a),
    "sqdiff": (lambda a, v: (a - v) ** 2, lambda a, v: 2 * (a - v), lambda a, v: -2 * (a - v)),
}


def np_reads(as_, is_):
    ok = (is_ >= 0) & (is_ < as_.size)
    return np.where(ok, as_[np.where(ok, is_, 0)], 0.0), ok


@pytest.mark.parametrize("op", list(FNS))
@pytest.mark.parametrize("m,n,dist", [(1, 1, "uniform"), (500, 7, "zipf"), (3000, 400, "uniform")])
def test_primal_and_closed_form_adjoint(orc, op, m, n, dist):
    as_, is_, vs, yb = workloads.gather_map(m, n, dist, "f64", seed=m + n)
    is_ = is_.copy()
    if m > 3:
        is_[[0, m // 2]] = [-1, n]  # out of range: reads 0, no update
    f, da, dv = FNS[op]
    a, ok = np_reads(as_, is_)
    assert rel_l2(orc.gather_map(op, as_, is_, vs), f(a, vs)) <= 1e-15
    ab, vb = orc.gather_map_vjp(op, as_, is_, vs, yb)
    ref = np.zeros(n)
    np.add.at(ref, is_[ok], (da(a, vs) * yb)[ok])
    assert rel_l2(ab, ref) <= 1e-14
    if dv is None:
        assert vb is None
    else:
        assert rel_l2(vb, dv(a, vs) * yb) <= 1e-15


@pytest.mark.parametrize("op", list(FNS))
def test_adjoint_is_the_replicated_jacobian(orc, op):
    # as as a bound variable of every element: J[i, k] = d ys[i] / d as[k] by
    # central differences, and as_bar = J^T ys_bar sums every read explicitly
    m, n = 40, 6
    as_, is_, vs, yb = workloads.gather_map(m, n, "zipf", "f64", seed=9)
    f = FNS[op][0]
    h = 1e-6
    J = np.zeros((m, n))
    for k in range(n):
        e = np.zeros(n)
        e[k] = h
        J[:, k] = (f((as_ + e)[is_], vs) - f((as_ - e)[is_], vs)) / (2 * h)
    ab, vb = orc.gather_map_vjp(op, as_, is_, vs, yb)
    assert rel_l2(ab, J.T @ yb) <= 1e-8
    if vb is not None:
        dv = (f(as_[is_], vs + h) - f(as_[is_], vs - h)) / (2 * h)
        assert rel_l2(vb, dv * yb) <= 1e-8


def test_empty_and_all_out_of_range(orc):
    ab, vb = orc.gather_map_vjp("mul", np.ones(3), np.array([], dtype=np.int32), np.array([]), np.array([]))
    assert np.all(ab == 0) and vb.size == 0
    ys = orc.gather_map("sqdiff", np.zeros(0), np.array([0, 1]), np.array([2.0, -3.0]))
    assert np.array_equal(ys, [4.0, 9.0])
    ab, vb = orc.gather_map_vjp("sqdiff", np.zeros(0), np.array([0, 1]), np.array([2.0, -3.0]), np.ones(2))
    assert ab.size == 0 and np.array_equal(vb, [4.0, -6.0])
