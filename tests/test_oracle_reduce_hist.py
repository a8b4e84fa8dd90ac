"""Pins for the oracle's reduce and reduce_by_index (Sec. 5.1, 5.1.1, 5.1.2).

Closed forms: the adjoint of a sum is all-ones; the adjoint of a product is
prod/x_i with the one-zero and several-zero cases spelled out; min/max send the
adjoint to the first extreme (numpy's argmax/argmin return the first
occurrence).  Histograms are checked against numpy's bincount and ufunc.at,
and small cases against brute-force Jacobians.
"""
import math

import numpy as np
import pytest

from _util import fd_grad, fd_jacobian, rel_l2
from paper_2202_10297_amd import workloads


# ---------------------------------------------------------------- reduce
def test_sum_closed_form(orc):
    x = workloads.rng(1).standard_normal(1000)
    y, _, _, _ = orc.reduce("add", x)
    assert abs(y - math.fsum(x)) < 1e-12
    assert np.array_equal(orc.reduce_vjp("add", x, 2.5), np.full(1000, 2.5))


def test_prod_no_zero_closed_form(orc):
    x = workloads.product_values(40, 0, "f64", seed=2)
    y, _, p, z = orc.reduce("mul", x)
    assert z == 0 and np.isclose(p, np.prod(x), rtol=1e-14) and np.isclose(y, p, rtol=1e-14)
    xb = orc.reduce_vjp("mul", x, -1.5)
    assert rel_l2(xb, np.prod(x) / x * -1.5) < 1e-14


@pytest.mark.parametrize("nz", [1, 2, 3])
def test_prod_zero_cases_every_position(orc, nz):
    n = 6
    base = workloads.product_values(n, 0, "f64", seed=9)
    import itertools

    for pos in itertools.combinations(range(n), nz):
        x = base.copy()
        x[list(pos)] = 0.0
        y, _, p, z = orc.reduce("mul", x)
        assert z == nz and y == 0.0
        assert np.isclose(p, np.prod(np.delete(x, pos)), rtol=1e-14)
        xb = orc.reduce_vjp("mul", x, 2.0)
        ref = np.zeros(n)
        if nz == 1:
            ref[pos[0]] = 2.0 * np.prod(np.delete(x, pos))
        assert np.allclose(xb, ref, rtol=1e-14, atol=0)


def test_prod_negative_zero_counts_as_zero(orc):
    x = np.array([1.5, -0.0, 2.0])
    _, _, p, z = orc.reduce("mul", x)
    assert z == 1 and p == 3.0
    assert np.array_equal(orc.reduce_vjp("mul", x, 1.0), [0.0, 3.0, 0.0])


@pytest.mark.parametrize("op", ["add", "mul"])
def test_reduce_fd(orc, op):
    x = workloads.product_values(8, 0, "f64", seed=4)
    g = fd_grad(lambda v: orc.reduce(op, v)[0] * 0.75, [x])[0]
    assert np.allclose(orc.reduce_vjp(op, x, 0.75), g, rtol=1e-7, atol=1e-9)


@pytest.mark.parametrize("op", ["min", "max"])
def test_minmax_first_index(orc, op):
    for seed in range(5):
        x = workloads.tie_values(300, "f64", seed=seed)
        y, arg, _, _ = orc.reduce(op, x)
        ref = np.argmax(x) if op == "max" else np.argmin(x)  # first occurrence
        assert arg == ref and y == x[ref]
        xb = orc.reduce_vjp(op, x, 3.0)
        exp = np.zeros(300)
        exp[ref] = 3.0
        assert np.array_equal(xb, exp)


def test_minmax_signed_zero_tie(orc):
    x = np.array([-1.0, -0.0, 0.0, -2.0])
    y, arg, _, _ = orc.reduce("max", x)
    assert arg == 1 and math.copysign(1.0, y) == -1.0
    x = np.array([0.0, -0.0])
    assert orc.reduce("min", x)[1] == 0


def test_reduce_empty(orc):
    assert orc.reduce("add", [])[0] == 0.0
    assert orc.reduce("mul", [])[0] == 1.0
    y, arg, _, _ = orc.reduce("max", [])
    assert y == -math.inf and arg == -1
    y, arg, _, _ = orc.reduce("min", [])
    assert y == math.inf and arg == -1


def test_max_all_neutral(orc):
    # An element equal to the neutral element still wins when it is first.
    y, arg, _, _ = orc.reduce("max", [-math.inf, -math.inf])
    assert arg == 0 and np.array_equal(orc.reduce_vjp("max", [-math.inf, -math.inf], 1.0), [1.0, 0.0])


# ------------------------------------------------------- reduce_by_index
@pytest.mark.parametrize("dist", ["uniform", "zipf"])
def test_hist_counts_and_sums(orc, dist):
    n, m = 20000, 64
    inds, vs, hb = workloads.hist(n, m, dist, "f64", seed=7)
    out = orc.hist("add", inds, vs, m)
    assert np.array_equal(out["count"], np.bincount(inds, minlength=m))
    ref = np.zeros(m)
    np.add.at(ref, inds, vs)
    assert rel_l2(out["hs"], ref) < 1e-13
    vb = orc.hist_vjp("add", inds, vs, hb)
    assert np.array_equal(vb, hb[inds])  # the gather, exactly


def test_hist_out_of_range_ignored(orc):
    inds = np.array([0, 5, -1, 1, 2, 1], dtype=np.int32)
    vs = np.array([1.0, 2.0, 3.0, 4.0, 5.0, 6.0])
    out = orc.hist("add", inds, vs, 3)
    assert np.array_equal(out["hs"], [1.0, 10.0, 5.0])
    assert np.array_equal(out["count"], [1, 2, 1])
    vb = orc.hist_vjp("add", inds, vs, [1.0, 2.0, 3.0])
    assert np.array_equal(vb, [1.0, 0.0, 0.0, 2.0, 3.0, 2.0])


@pytest.mark.parametrize("op", ["min", "max"])
def test_hist_minmax_winners(orc, op):
    n, m = 5000, 37
    g = workloads.rng(13)
    inds = g.integers(0, m + 3, n).astype(np.int32)  # some bins empty-ish, some out of range
    vs = workloads.tie_values(n, "f64", seed=14)
    hb = g.standard_normal(m)
    out = orc.hist(op, inds, vs, m)
    ref = np.full(m, -np.inf if op == "max" else np.inf)
    ok = inds < m
    (np.maximum if op == "max" else np.minimum).at(ref, inds[ok], vs[ok])
    assert np.array_equal(out["hs"], ref)
    for k in range(m):
        sel = np.nonzero((inds == k))[0]
        if sel.size == 0:
            assert out["winner"][k] == -1
        else:
            assert out["winner"][k] == sel[np.nonzero(vs[sel] == ref[k])[0][0]]
    vb = orc.hist_vjp(op, inds, vs, hb)
    exp = np.zeros(n)
    w = out["winner"]
    exp[w[w >= 0]] = hb[w >= 0]
    assert np.array_equal(vb, exp)


def test_hist_mul(orc):
    n, m = 400, 5
    g = workloads.rng(17)
    inds = g.integers(0, m, n).astype(np.int32)
    vs = workloads.product_values(n, 3, "f64", seed=18)
    hb = g.standard_normal(m)
    out = orc.hist("mul", inds, vs, m)
    ref = np.ones(m)
    np.multiply.at(ref, inds, vs)
    assert np.allclose(out["hs"], ref, rtol=1e-13, atol=0)
    vb = orc.hist_vjp("mul", inds, vs, hb)
    for k in range(m):
        sel = np.nonzero(inds == k)[0]
        zs = sel[vs[sel] == 0]
        assert out["z"][k] == zs.size
        pnz = np.prod(vs[sel][vs[sel] != 0])
        assert np.isclose(out["p"][k], pnz, rtol=1e-13)
        if zs.size == 0:
            assert np.allclose(vb[sel], pnz / vs[sel] * hb[k], rtol=1e-12)
        elif zs.size == 1:
            exp = np.zeros(sel.size)
            exp[sel == zs[0]] = pnz * hb[k]
            assert np.allclose(vb[sel], exp, rtol=1e-12, atol=0)
        else:
            assert np.all(vb[sel] == 0)


@pytest.mark.parametrize("op", ["add", "mul"])
@pytest.mark.parametrize("m", [1, 2, 3])
def test_hist_bruteforce_jacobian(orc, op, m):
    n = 8
    g = workloads.rng(100 + m)
    inds = g.integers(0, m, n).astype(np.int32)
    vs = workloads.product_values(n, 0, "f64", seed=200 + m)
    J = fd_jacobian(lambda v: orc.hist(op, inds, v, m)["hs"], vs)
    Jv = np.stack([orc.hist_vjp(op, inds, vs, np.eye(m)[r]) for r in range(m)])
    assert np.allclose(Jv, J, rtol=1e-7, atol=1e-8)
