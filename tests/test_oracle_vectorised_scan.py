"""Pins for the vectorised-operator rule of Sec. 5.2: a scan whose operator
is applied componentwise to vectors of w elements (xs stored [n x w]) equals
transpose, a scan of every row, transpose.  The left side is computed
independently with numpy (log-add-exp accumulate along the vector axis, the
closed form of the linear recurrence, chained 2 x 2 matrix products per
component); the right side is the oracle's single scan applied to each row
of the transposed arrays.  The VJP per row is checked against central
differences of the numpy vectorised primal.
"""
import numpy as np
import pytest

from _util import rel_l2
from paper_2202_10297_amd import workloads


def vectorised_numpy(op, xs):
    """Columns of [n x w] scanned along axis 0, with numpy only."""
    if op == "logaddexp":
        return [np.logaddexp.accumulate(xs[0], axis=0)]
    if op == "linrec":
        a, b = xs
        A = np.cumprod(a, axis=0)
        B = np.empty_like(b)
        acc = np.zeros(b.shape[1])
        for i in range(b.shape[0]):
            acc = acc * a[i] + b[i]
            B[i] = acc
        return [A, B]
    m = np.stack(xs, axis=-1).reshape(xs[0].shape + (2, 2))  # [n, w, 2, 2] row-major 2x2
    out = np.empty_like(m)
    acc = np.broadcast_to(np.eye(2), m.shape[1:]).copy()
    for i in range(m.shape[0]):
        acc = acc @ m[i]
        out[i] = acc
    flat = out.reshape(xs[0].shape + (4,))
    return [flat[..., c] for c in range(4)]


def vec_inputs(op, n, w, seed):
    xs, _ = workloads.gop_scan(op, n * w, "f64", seed=seed)
    return [x.reshape(n, w) for x in xs]


@pytest.mark.parametrize("op", ["logaddexp", "linrec", "mat2"])
@pytest.mark.parametrize("n,w", [(1, 1), (7, 3), (40, 16)])
def test_rule_transpose_scan_transpose(orc, op, n, w):
    xs = vec_inputs(op, n, w, seed=n * w)
    lhs = vectorised_numpy(op, xs)
    rows = orc.scan_generic_rows(op, [x.T for x in xs])
    assert rel_l2([r.T for r in rows], lhs) <= 1e-13


@pytest.mark.parametrize("op", ["logaddexp", "linrec", "mat2"])
def test_rule_vjp_finite_differences(orc, op):
    n, w = 9, 3
    xs = vec_inputs(op, n, w, seed=5)
    g = workloads.rng(6)
    yb = [g.standard_normal((n, w)) for _ in xs]
    rows = orc.scan_generic_rows_vjp(op, [x.T for x in xs], [y.T for y in yb])
    h = 1e-6
    for c in range(len(xs)):
        fd = np.empty((n, w))
        for i in range(n):
            for j in range(w):
                p = [x.copy() for x in xs]
                q = [x.copy() for x in xs]
                p[c][i, j] += h
                q[c][i, j] -= h
                fp = sum(float((y * o).sum()) for y, o in zip(yb, vectorised_numpy(op, p)))
                fq = sum(float((y * o).sum()) for y, o in zip(yb, vectorised_numpy(op, q)))
                fd[i, j] = (fp - fq) / (2 * h)
        assert rel_l2(rows[c].T, fd) <= 1e-7
