"""GPU parity of reduce_by_index with a general operator (Sec. 5.1.2 with
the general rule of Sec. 5.1.1 inside each bin; the operators need not
commute) and its VJP, through the C ABI, against the oracle on the same
seeded inputs.

Bars: FP64 relative L2 1e-12 per component; FP32 inputs 2e-5 against the
FP64 oracle on the same FP32 values, rounded to FP32; empty log-add-exp bins -inf exactly;
adjoints of out-of-range indices exactly 0.  Cases: one bin (every element
in it, across every tile), few bins (one sort pass of at most 8 bits),
m = 257, 2^10 and 2^16 (two passes), 2^17 + 3 and 2^20 (three), the largest
m = 2^24 (three full passes), Zipf(1.1) indices, indices out of range on both sides,
n = 0 and 1, more sort chunks than a column-scan chunk holds (n = 2.5M),
accumulation, and bitwise repeatability.
"""
import numpy as np
import pytest

from _util import TOL_F32, TOL_F64, rel_l2
from paper_2202_10297_amd import workloads

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

OPS = ["linrec", "mat2", "logaddexp"]


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


def check(got, ref, bar):
    # the reference rounded to the output's dtype (an FP32 output cannot hold
    # the FP64 oracle's value below FP32's range: long linear-recurrence
    # products underflow)
    ref = np.asarray(ref, dtype=np.float64)
    if got.dtype == np.float32:
        ref = ref.astype(np.float32).astype(np.float64)
    got = np.asarray(got, dtype=np.float64)
    fin = np.isfinite(ref)
    assert np.array_equal(np.isfinite(got), fin)
    assert np.array_equal(got[~fin], ref[~fin])
    if fin.any():
        assert rel_l2(got[fin], ref[fin]) <= bar


def run_case(ops, orc, op, n, m, dtype, dist="uniform", seed=0, oob=True):
    inds, xs, hb = workloads.hist_generic(op, n, m, dist, dtype, seed=seed)
    if oob and n > 4:
        inds[::97] = -1
        inds[5::89] = m
    bar = TOL_F64 if dtype == "f64" else TOL_F32
    dx = [dev(x) for x in xs]
    di = dev(inds)
    hs = ops.hist_generic(op, di, dx, m)
    ref = orc.hist_generic(op, inds, [x.astype(np.float64) for x in xs], m)
    for g, r in zip(hs, ref):
        check(host(g), r, bar)
    xb = ops.hist_generic_vjp(op, di, dx, [dev(h) for h in hb])
    rvb = orc.hist_generic_vjp(op, inds, [x.astype(np.float64) for x in xs], [h.astype(np.float64) for h in hb])
    out = (inds < 0) | (inds >= m)
    for g, r in zip(xb, rvb):
        g = host(g)
        assert np.all(g[out] == 0)
        check(g, r, bar)
    return di, dx, hb, hs, xb


CASES = [(0, 5), (1, 1), (1000, 1), (5003, 7), (20011, 257), (300007, 1 << 10), (300007, 1 << 16),
         (100003, (1 << 17) + 3), (200003, 1 << 20)]


@pytest.mark.parametrize("op", OPS)
@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("n,m", CASES)
def test_parity(ops, orc, op, dtype, n, m):
    run_case(ops, orc, op, n, m, dtype, seed=n + m)


@pytest.mark.parametrize("op", OPS)
def test_zipf(ops, orc, op):
    run_case(ops, orc, op, 300007, 4096 + 3, "f64", dist="zipf", seed=11)


@pytest.mark.parametrize("op", ["linrec", "mat2"])
def test_largest_bin_count(ops, orc, op):
    # m = 2^24: three sort passes of 8 bits each
    run_case(ops, orc, op, 60013, 1 << 24, "f32", seed=24)


def test_many_sort_chunks(ops, orc):
    # 77 sort chunks of 32768 elements: more than one column-scan chunk of 64
    run_case(ops, orc, "linrec", 77 * 32768 - 5, 1 << 16, "f32", seed=5)


@pytest.mark.parametrize("op", ["linrec", "mat2"])
def test_accumulate_and_repeat(ops, orc, op):
    n, m = 100003, 1 << 12
    di, dx, hb, hs, xb = run_case(ops, orc, op, n, m, "f64", seed=3)
    again = ops.hist_generic(op, di, dx, m)
    for a, b in zip(hs, again):
        assert np.array_equal(host(a), host(b))
    base = [np.full(n, 0.5) for _ in dx]
    acc = ops.hist_generic_vjp(op, di, dx, [dev(h) for h in hb], x_bar=[dev(b) for b in base], accumulate=True)
    for a, g, b in zip(acc, xb, base):
        np.testing.assert_allclose(host(a), host(g) + b, rtol=1e-14, atol=1e-14)


def test_full_size_sampled(ops, orc):
    # the benchmark's shape (n = 2^26 FP32, m = 2^16, uniform): 64 sampled
    # bins against the oracle on exactly those bins' elements, in index
    # order (a bin's fold and adjoints depend on nothing else)
    n, m, op = 1 << 26, 1 << 16, "linrec"
    inds, xs, hb = workloads.hist_generic(op, n, m, "uniform", "f32", seed=0)
    di = dev(inds)
    dx = [dev(x) for x in xs]
    hs = [host(h) for h in ops.hist_generic(op, di, dx, m)]
    xb = [host(g) for g in ops.hist_generic_vjp(op, di, dx, [dev(h) for h in hb])]
    bins = np.random.default_rng(1).choice(m, 64, replace=False)
    sel = np.nonzero(np.isin(inds, bins))[0]
    remap = np.full(m, -1, np.int64)
    remap[bins] = np.arange(64)
    sub_inds = remap[inds[sel]].astype(np.int32)
    sub_x = [x[sel].astype(np.float64) for x in xs]
    ref = orc.hist_generic(op, sub_inds, sub_x, 64)
    for g, r in zip(hs, ref):
        check(g[bins], r, TOL_F32)
    rvb = orc.hist_generic_vjp(op, sub_inds, sub_x, [h[bins].astype(np.float64) for h in hb])
    for g, r in zip(xb, rvb):
        check(g[sel], r, TOL_F32)
