"""GPU parity of reduce_by_index with the log-add-exp operator (Sec. 5.1.2
with the general rule of Sec. 5.1.1 per bin) against the oracle's
general-operator reduce_by_index, on the same seeded inputs: FP64 relative
L2 1e-12, FP32 2e-5; -inf elements, empty bins, indices out of range, bin
counts from one to 2^20 (every reduce_by_index plan), uniform and Zipf(1.1).
"""
import numpy as np
import pytest

from _util import TOL_F32, TOL_F64, rel_l2
from paper_2202_10297_amd import workloads

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


@pytest.fixture(scope="module")
def ops():
    from paper_2202_10297_amd import capi, ops as o

    capi.lib()
    return o


CASES = [(1, 1, "uniform"), (1000, 7, "zipf"), (300001, 1024, "uniform"), (300001, 1 << 16, "zipf"),
         (1 << 21, 1 << 20, "uniform")]


@pytest.mark.parametrize("dtype", ["f32", "f64"])
@pytest.mark.parametrize("n,m,dist", CASES)
def test_hist_lae(ops, orc, dtype, n, m, dist):
    inds, x, hb = workloads.hist(n, m, dist, dtype, seed=n % 977 + m)
    inds = inds.copy()
    x = x.copy()
    if n > 10:
        inds[[0, n // 2]] = [-1, m]  # skipped
        x[[1, n // 3]] = -np.inf     # adjoint 0
    hs = ops.hist_lae(dev(inds), dev(x), m)
    ref = orc.hist_generic("logaddexp", inds, [x], m)[0]
    got = host(hs).astype(np.float64)
    fin = np.isfinite(ref)
    assert np.array_equal(np.isneginf(got), np.isneginf(ref))
    assert rel_l2(got[fin], ref[fin]) <= (1e-13 if dtype == "f64" else 1e-6)
    xb = host(ops.hist_lae_vjp(dev(inds), dev(x), hs, dev(hb)))
    rxb = orc.hist_generic_vjp("logaddexp", inds, [x], [hb])[0]
    assert rel_l2(xb, rxb) <= (TOL_F64 if dtype == "f64" else TOL_F32)
    if n > 10:
        assert xb[0] == 0 and xb[1] == 0


def test_hist_lae_accumulate_and_one_bin_is_the_generic_reduce(ops, orc):
    n = 50001
    x = workloads.rng(2).standard_normal(n)
    inds = np.zeros(n, dtype=np.int32)
    hs = ops.hist_lae(dev(inds), dev(x), 1)
    assert abs(host(hs)[0] - orc.reduce_generic("logaddexp", [x])[0]) <= 1e-12 * abs(host(hs)[0])
    base = np.full(n, 0.5)
    xb = host(ops.hist_lae_vjp(dev(inds), dev(x), hs, dev(np.array([2.0])), x_bar=dev(base), accumulate=True))
    assert rel_l2(xb - 0.5, orc.reduce_generic_vjp("logaddexp", [x], [2.0])[0]) <= TOL_F64


def test_autograd(orc):
    from paper_2202_10297_amd import autograd

    inds, x, hb = workloads.hist(20001, 300, "zipf", "f64", seed=31)
    t = dev(x).requires_grad_()
    hs = autograd.reduce_by_index_logaddexp(t, dev(inds), 300)
    (hs * dev(hb)).sum().backward()
    assert rel_l2(host(t.grad), orc.hist_generic_vjp("logaddexp", inds, [x], [hb])[0]) <= TOL_F64
