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


@pytest.mark.parametrize("dtype", ["f32", "f64"])
@pytest.mark.parametrize("m", [7, 1 << 16])
def test_hist_lae_non_finite_bins(ops, orc, dtype, m):
    # Over the extended reals: -inf is neutral, NaN propagates, +inf absorbs.
    # Bin 0 one +inf among finite values, bin 1 a NaN, bin 2 only -inf,
    # bin 3 two +inf, bin 4 empty; the rest of the bins ordinary.
    n = 60000
    inds, x, hb = workloads.hist(n, m, "uniform", dtype, seed=m)
    inds, x = inds.copy(), x.copy()
    inds[inds <= 4] = 5
    head = [(0, 0.5), (0, np.inf), (0, -1.0), (1, np.nan), (1, 2.0), (2, -np.inf), (3, np.inf), (3, 1.0),
            (3, np.inf)]
    for j, (b, v) in enumerate(head):
        inds[97 * j + 3], x[97 * j + 3] = b, v
    hs = ops.hist_lae(dev(inds), dev(x), m)
    ref = orc.hist_generic("logaddexp", inds, [x], m)[0]
    got = host(hs).astype(np.float64)
    assert np.array_equal(np.isnan(got), np.isnan(ref))
    inf = np.isinf(ref)
    assert np.array_equal(got[inf], ref[inf])
    fin = np.isfinite(ref)
    assert rel_l2(got[fin], ref[fin]) <= (1e-13 if dtype == "f64" else 1e-6)
    assert np.isposinf(got[0]) and np.isnan(got[1]) and np.isneginf(got[2]) and np.isposinf(got[3])
    assert np.isneginf(got[4])
    xb = host(ops.hist_lae_vjp(dev(inds), dev(x), hs, dev(hb))).astype(np.float64)
    rxb = orc.hist_generic_vjp("logaddexp", inds, [x], [hb])[0]
    # The one reading that differs: several +inf elements of one bin each get
    # hs_bar here; the oracle's index-order fold gives it to the first one.
    tie = (inds == 3) & np.isposinf(x)
    assert np.array_equal(xb[tie], np.full(2, hb[3]))
    keep = ~tie
    assert np.array_equal(np.isnan(xb[keep]), np.isnan(rxb[keep]))
    ok = keep & ~np.isnan(rxb)
    assert rel_l2(xb[ok], rxb[ok]) <= (TOL_F64 if dtype == "f64" else TOL_F32)
    assert xb[3 + 97] == hb[0]  # the single +inf of bin 0 takes the whole adjoint


def test_hist_lae_bench_shape_sampled_bins(ops, orc):
    # n = 2^26 FP32, Zipf(1.1), m = 2^16: the hot bins' buckets are split
    # into many work items of the partitioned MAX and + passes.  The three
    # fullest bins and a few others against the oracle's reduce of the bin's
    # own elements.
    n, m = 1 << 26, 1 << 16
    inds, x, hb = workloads.hist(n, m, "zipf", "f32", seed=0)
    dinds, dx = dev(inds), dev(x)
    hs = ops.hist_lae(dinds, dx, m)
    xb = host(ops.hist_lae_vjp(dinds, dx, hs, dev(hb)))
    got = host(hs)
    cnt = np.bincount(inds, minlength=m)
    hot = [int(b) for b in np.argsort(cnt)[-3:]]
    for b in hot + [0, 17, 4095, 4096, 40000, m - 1]:
        sel = np.nonzero(inds == b)[0]
        ref = orc.reduce_generic("logaddexp", [x[sel]])[0] if sel.size else -np.inf
        if sel.size == 0:
            assert np.isneginf(got[b])
            continue
        assert abs(got[b] - ref) <= 1e-6 * max(1.0, abs(ref)), b
        rxb = orc.reduce_generic_vjp("logaddexp", [x[sel]], [float(hb[b])])[0]
        assert rel_l2(xb[sel], rxb) <= TOL_F32, b
