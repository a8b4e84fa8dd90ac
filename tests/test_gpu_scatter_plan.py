"""GPU parity of the target-ordered scatter (Sec. 5.3, the forward sweep
returning its updates grouped by target window) against the oracle, bit for
bit: the scattered array, the return sweep's vs_bar and xs_bar, and the
restored array.  Sizes from one update to the full 2^24 targets into 2^26,
windows cut by the array's end, windows full of updates, out-of-range
targets, accumulate, FP32 and FP64; at full size against the oracle on sampled targets and against the
unplanned kernels everywhere.
"""
import numpy as np
import pytest

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


CASES = [(1, 1), (10, 3), (8192, 8192), (8193, 2000), (100003, 25000), (1 << 20, 1 << 18), (3000001, 700001)]


@pytest.mark.parametrize("dtype", ["f32", "f64"])
@pytest.mark.parametrize("n,m", CASES)
def test_scatter_planned(ops, orc, dtype, n, m):
    xs, is_, vs, yb = workloads.scatter(n, m, dtype, seed=n + m)
    x = dev(xs)
    plan = ops.scatter_planned_(x, dev(is_), dev(vs))
    rys, _ = orc.scatter(xs, is_, vs)
    assert np.array_equal(host(x), rys)
    ybar = dev(yb)
    vbar = ops.scatter_planned_vjp_(ybar, m, plan, ys=x)
    rxb, rvb = orc.scatter_vjp(is_, yb)
    assert np.array_equal(host(ybar), rxb) and np.array_equal(host(vbar), rvb)
    assert np.array_equal(host(x), xs)  # restored


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_scatter_planned_dense_windows(ops, orc, dtype):
    # Every target of [0, 2^18) and of the array's last 40000 elements, in
    # random order: whole windows full of updates (more records per window
    # than either sweep holds in registers), one coarse bucket split into
    # many chunks of the second bucketing pass, most buckets empty.
    n = 1 << 20
    xs, _, _, yb = workloads.scatter(n, 1, dtype, seed=21)
    g = workloads.rng(22)
    is_ = g.permutation(np.concatenate([np.arange(1 << 18), np.arange(n - 40000, n)])).astype(np.int32)
    m = is_.size
    vs = g.standard_normal(m).astype(xs.dtype)
    x = dev(xs)
    plan = ops.scatter_planned_(x, dev(is_), dev(vs))
    rys, _ = orc.scatter(xs, is_, vs)
    assert np.array_equal(host(x), rys)
    ybar = dev(yb)
    vbar = ops.scatter_planned_vjp_(ybar, m, plan, ys=x)
    rxb, rvb = orc.scatter_vjp(is_, yb)
    assert np.array_equal(host(ybar), rxb) and np.array_equal(host(vbar), rvb)
    assert np.array_equal(host(x), xs)


def test_scatter_planned_out_of_range_and_accumulate(ops, orc):
    n = 20000
    g = workloads.rng(4)
    is_ = g.permutation(n)[:3000].astype(np.int32)
    is_[[0, 7, 2999]] = [-3, n, n + 5000]
    xs, vs, yb = g.standard_normal(n), g.standard_normal(3000), g.standard_normal(n)
    x = dev(xs)
    plan = ops.scatter_planned_(x, dev(is_), dev(vs))
    rys, _ = orc.scatter(xs, is_, vs)
    assert np.array_equal(host(x), rys)
    # without accumulate the dropped targets' adjoints are 0 (vs_bar starts as garbage)
    vb = dev(np.full(3000, 7.0))
    ybar = dev(yb)
    ops.scatter_planned_vjp_(ybar, 3000, plan, vs_bar=vb, ys=x)
    rxb, rvb = orc.scatter_vjp(is_, yb)
    assert np.array_equal(host(ybar), rxb) and np.array_equal(host(vb), rvb)
    assert np.array_equal(host(x), xs)
    # accumulate, no restore
    base = np.arange(3000, dtype=np.float64)
    vb2 = dev(base)
    ybar2 = dev(yb)
    ops.scatter_planned_vjp_(ybar2, 3000, plan, vs_bar=vb2, accumulate=True)
    assert np.array_equal(host(ybar2), rxb) and np.array_equal(host(vb2), base + rvb)


def test_scatter_planned_empty(ops):
    x = dev(np.ones(100, dtype=np.float32))
    plan = ops.scatter_planned_(x, dev(np.zeros(0, dtype=np.int32)), dev(np.zeros(0, dtype=np.float32)))
    ops.scatter_planned_vjp_(dev(np.ones(100, dtype=np.float32)), 0, plan)
    assert np.all(host(x) == 1)


def test_scatter_planned_full_size(ops, orc):
    # the bench shape: 2^24 unique targets into 2^26 FP32
    n, m = 1 << 26, 1 << 24
    xs, is_, vs, yb = workloads.scatter(n, m, "f32", seed=7)
    dis, dvs = dev(is_), dev(vs)
    x1, x2 = dev(xs), dev(xs)
    saved = ops.scatter_(x1, dis, dvs)
    plan = ops.scatter_planned_(x2, dis, dvs)
    assert torch.equal(x1, x2)
    y1, y2 = dev(yb), dev(yb)
    v1 = ops.scatter_vjp_(y1, dis, ys=x1, xs_saved=saved)
    v2 = ops.scatter_planned_vjp_(y2, m, plan, ys=x2)
    assert torch.equal(y1, y2) and torch.equal(v1, v2) and torch.equal(x1, x2)
    # sampled against the oracle: the adjoint of a scatter is a gather
    j = workloads.rng(1).integers(0, m, 4096)
    sel = np.unique(j)
    _, rvb = orc.scatter_vjp(is_[sel], yb)
    assert np.array_equal(host(v2)[sel], rvb.astype(np.float32))
    assert np.array_equal(host(x2), xs)
