"""Pins for the oracle's scatter (Sec. 5.3), map (Sec. 5.4) and the Fig. 1
worked example (Sec. 2.0.2)."""
import os

import numpy as np
import pytest

from _util import fd_grad, fd_jacobian
from paper_2202_10297_amd import workloads

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# --------------------------------------------------------------- scatter
def test_scatter_primal_matches_numpy(orc):
    xs, is_, vs, _ = workloads.scatter(4096, 1024, "f64", seed=1)
    ys, saved = orc.scatter(xs, is_, vs)
    ref = xs.copy()
    ref[is_] = vs
    assert np.array_equal(ys, ref)
    assert np.array_equal(saved, xs[is_])


def test_scatter_vjp_invariants(orc):
    n, m = 4096, 1024
    _, is_, _, yb = workloads.scatter(n, m, "f64", seed=2)
    yb = np.round(yb * 8)  # integer-valued: every sum below is exact
    xb, vb = orc.scatter_vjp(is_, yb)
    assert np.array_equal(vb, yb[is_])  # gather
    assert np.all(xb[is_] == 0)
    back = xb.copy()
    back[is_] = vb  # x_bar + scatter(0, is, v_bar) == y_bar
    assert np.array_equal(back, yb)
    assert xb.sum() + vb.sum() == yb.sum()


def test_scatter_bruteforce(orc):
    n = 8
    is_ = np.array([5, 1, 6], dtype=np.int32)
    xs = workloads.rng(3).standard_normal(n)
    vs = workloads.rng(4).standard_normal(3)
    J = fd_jacobian(lambda x: orc.scatter(x[:n], is_, x[n:])[0], np.concatenate([xs, vs]))
    Jv = np.stack([np.concatenate(orc.scatter_vjp(is_, np.eye(n)[r])) for r in range(n)])
    assert np.allclose(Jv, J, atol=1e-9)


def test_scatter_out_of_range(orc):
    xs = np.arange(4.0)
    ys, saved = orc.scatter(xs, [7, 2, -1], [10.0, 20.0, 30.0])
    assert np.array_equal(ys, [0.0, 1.0, 20.0, 3.0]) and np.array_equal(saved, [0.0, 2.0, 0.0])
    xb, vb = orc.scatter_vjp([7, 2, -1], [1.0, 2.0, 3.0, 4.0])
    assert np.array_equal(xb, [1.0, 2.0, 0.0, 4.0]) and np.array_equal(vb, [0.0, 3.0, 0.0])


# ------------------------------------------------------------------- map
TEXTBOOK = {
    "square": lambda x: 2 * x,
    "exp": np.exp,
    "log": lambda x: 1 / x,
    "sin": np.cos,
    "tanh": lambda x: 1 - np.tanh(x) ** 2,
}
PRIMAL = {"square": np.square, "exp": np.exp, "log": np.log, "sin": np.sin, "tanh": np.tanh}


@pytest.mark.parametrize("fn", sorted(TEXTBOOK))
def test_map_textbook_derivatives(orc, fn):
    g = workloads.rng(5)
    x = g.uniform(0.2, 3.0, 500)
    yb = g.standard_normal(500)
    assert np.allclose(orc.map_(fn, x), PRIMAL[fn](x), rtol=1e-15)
    # 1 - tanh^2 cancels near |x| ~ 3, so allow a few hundred ulps
    assert np.allclose(orc.map_vjp(fn, x, yb), TEXTBOOK[fn](x) * yb, rtol=1e-12, atol=0)
    # and against finite differences of the primal
    fdg = fd_grad(lambda v: float(np.dot(orc.map_(fn, v), yb[:6])), [x[:6]])[0]
    assert np.allclose(orc.map_vjp(fn, x[:6], yb[:6]), fdg, rtol=1e-7)


# ----------------------------------------------------------------- Fig. 1
def test_fig1_adjoint_program(orc):
    # Fig. 1(c): x0_bar = x1*y1_bar + cos(x0)*(x1*y0_bar); x1_bar = x0*y1_bar + sin(x0)*y0_bar.
    g = workloads.rng(6)
    x0, x1, b0, b1 = (g.standard_normal(300) for _ in range(4))
    r0, r1 = orc.fig1_vjp(x0, x1, b0, b1)
    assert np.allclose(r0, x1 * b1 + np.cos(x0) * x1 * b0, rtol=1e-14, atol=1e-15)
    assert np.allclose(r1, x0 * b1 + np.sin(x0) * b0, rtol=1e-14, atol=1e-15)
    y0, y1 = orc.fig1(x0, x1)
    assert np.allclose(y0, x1 * np.sin(x0)) and np.allclose(y1, x0 * x1)


def test_fig1_golden(orc):
    rows = np.loadtxt(os.path.join(GOLDEN, "fig1_adjoint.txt"), comments="#")
    for x0, x1, b0, b1, e0, e1 in rows:
        r0, r1 = orc.fig1_vjp([x0], [x1], [b0], [b1])
        assert abs(r0[0] - e0) <= 1e-15 * max(1, abs(e0)) and abs(r1[0] - e1) <= 1e-15 * max(1, abs(e1))


def test_fig1_jacobian_fd(orc):
    x = np.array([0.7, -1.3])
    J = fd_jacobian(lambda v: np.concatenate(orc.fig1(v[:1], v[1:])), x)
    Jv = np.stack([np.concatenate(orc.fig1_vjp([0.7], [-1.3], *np.eye(2)[r][:, None])) for r in range(2)])
    assert np.allclose(Jv, J, rtol=1e-8)
