"""GPU parity of a map reading a free array (Sec. 5.4) and its return sweep,
whose reads become an accumulator (lowered to FP64 LDS bins when the array
has at most 16384 elements, else to FP64 global atomics), through the C ABI
against the oracle on the same seeded inputs.

Bars: primal FP64 bit-exact (same operations), FP32 relative L2 1e-6;
adjoints FP64 relative L2 1e-12, FP32 2e-5.  Sizes span both accumulator
plans and their boundary; indices uniform or Zipf(1.1) (hot bins), with
out-of-range entries.  At 2^26 elements the accumulator is checked per
sampled bin against the oracle run on exactly the elements that read it,
and the element adjoints on sampled elements.
"""
import numpy as np
import pytest

from _util import TOL_F32, TOL_F64, rel_l2
from paper_2202_10297_amd import workloads

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

OPS = ["gather", "mul", "sqdiff"]


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def tol(dtype):
    return TOL_F64 if dtype == "f64" else TOL_F32


@pytest.fixture(scope="module")
def ops():
    from paper_2202_10297_amd import capi, ops as o

    capi.lib()
    return o


def inputs(m, n, dist, dtype, seed):
    as_, is_, vs, yb = workloads.gather_map(m, n, dist, dtype, seed)
    if m > 10:
        is_ = is_.copy()
        is_[[1, m // 3, m - 1]] = [-5, n, 2**31 - 1]
    return as_, is_, vs, yb


CASES = [(1, 1, "uniform"), (1000, 7, "zipf"), (100003, 4096, "zipf"), (100003, 16384, "uniform"),
         (100003, 16385, "uniform"), (300001, 1 << 20, "zipf")]


@pytest.mark.parametrize("op", OPS)
@pytest.mark.parametrize("dtype", ["f32", "f64"])
@pytest.mark.parametrize("m,n,dist", CASES)
def test_gather_map_and_vjp(ops, orc, op, dtype, m, n, dist):
    as_, is_, vs, yb = inputs(m, n, dist, dtype, seed=m + n)
    v = None if op == "gather" else vs
    ys = host(ops.gather_map(op, dev(as_), dev(is_), dev(v) if v is not None else None))
    ref = orc.gather_map(op, as_, is_, v)
    if dtype == "f64":
        assert np.array_equal(ys, ref)
    else:
        assert rel_l2(ys, ref) <= 1e-6
    ab, vb = ops.gather_map_vjp(op, dev(as_), dev(is_), dev(v) if v is not None else None, dev(yb))
    rab, rvb = orc.gather_map_vjp(op, as_, is_, v, yb)
    assert rel_l2(host(ab), rab) <= tol(dtype)
    if op != "gather":
        assert rel_l2(host(vb), rvb) <= tol(dtype)


@pytest.mark.parametrize("n", [300, 1 << 18])
def test_accumulate(ops, orc, n):
    m = 50001
    as_, is_, vs, yb = inputs(m, n, "zipf", "f32", seed=3)
    base_a = np.full(n, 0.5, dtype=np.float32)
    base_v = np.full(m, -0.25, dtype=np.float32)
    ab, vb = ops.gather_map_vjp("sqdiff", dev(as_), dev(is_), dev(vs), dev(yb), as_bar=dev(base_a),
                                vs_bar=dev(base_v), accumulate=True)
    rab, rvb = orc.gather_map_vjp("sqdiff", as_, is_, vs, yb)
    assert rel_l2(host(ab) - 0.5, rab) <= 2 * TOL_F32
    assert rel_l2(host(vb) + 0.25, rvb) <= 2 * TOL_F32


def test_empty_and_all_out_of_range(ops, orc):
    # m = 0: as_bar is all zeros (every k < n written)
    as_ = dev(np.ones(5, dtype=np.float32))
    e_i = torch.empty(0, dtype=torch.int32, device="cuda")
    e_v = torch.empty(0, dtype=torch.float32, device="cuda")
    ab = torch.full((5,), 7.0, device="cuda")
    ops.gather_map_vjp("mul", as_, e_i, e_v, e_v, as_bar=ab, vs_bar=e_v)
    assert np.all(host(ab) == 0)
    # n = 0: every read is out of range and reads 0
    vs = np.array([2.0, -3.0], dtype=np.float64)
    none = torch.empty(0, dtype=torch.float64, device="cuda")
    is_ = dev(np.array([0, 1], dtype=np.int32))
    ys = ops.gather_map("sqdiff", none, is_, dev(vs))
    assert np.array_equal(host(ys), orc.gather_map("sqdiff", np.zeros(0), [0, 1], vs))
    _, vb = ops.gather_map_vjp("sqdiff", none, is_, dev(vs), dev(np.ones(2)))
    assert np.array_equal(host(vb), orc.gather_map_vjp("sqdiff", np.zeros(0), [0, 1], vs, np.ones(2))[1])


def test_refusals(ops):
    from paper_2202_10297_amd import capi

    x = dev(np.ones(4, dtype=np.float32))
    i = dev(np.zeros(4, dtype=np.int32))
    with pytest.raises(capi.PvjpError):
        ops.gather_map("mul", x, i, None)  # vs required for mul
    with pytest.raises(KeyError):
        ops.gather_map("div", x, i, x)


@pytest.mark.parametrize("n,dist", [(1 << 12, "zipf"), (1 << 20, "zipf"), (1 << 20, "uniform")])
def test_benchmark_size_sampled(ops, orc, n, dist):
    m = 1 << 26
    as_, is_, vs, yb = workloads.gather_map(m, n, dist, "f32", seed=0)
    ab, vb = ops.gather_map_vjp("mul", dev(as_), dev(is_), dev(vs), dev(yb))
    ab, vb = host(ab), host(vb)
    g = workloads.rng(5)
    # per sampled bin (the hottest included): the oracle on the elements
    # that read it, with the bin as a one-element free array
    hot = int(np.bincount(is_[: 1 << 20], minlength=n).argmax())
    for k in [hot, *g.integers(0, n, 4).tolist()]:
        sel = np.nonzero(is_ == k)[0]
        rab, _ = orc.gather_map_vjp("mul", as_[k:k + 1], np.zeros(sel.size, dtype=np.int32), vs[sel], yb[sel])
        assert abs(ab[k] - rab[0]) <= TOL_F32 * max(1.0, np.abs(vs[sel] * yb[sel]).sum())
    # sampled element adjoints
    s = g.integers(0, m, 4096)
    _, rvb = orc.gather_map_vjp("mul", as_, is_[s], vs[s], yb[s])
    assert rel_l2(vb[s], rvb) <= TOL_F32
    # any size: the accumulated total is the sum of every read's partial
    tot = np.dot(vs.astype(np.float64), yb.astype(np.float64))
    assert abs(ab.astype(np.float64).sum() - tot) <= 1e-5 * np.abs(vs * yb).sum()


def test_autograd(orc):
    from paper_2202_10297_amd import autograd

    as_, is_, vs, yb = inputs(20001, 300, "zipf", "f64", seed=12)
    a, v = dev(as_).requires_grad_(), dev(vs).requires_grad_()
    ys = autograd.gather_map(a, dev(is_), v, op="sqdiff")
    (ys * dev(yb)).sum().backward()
    rab, rvb = orc.gather_map_vjp("sqdiff", as_, is_, vs, yb)
    assert rel_l2(host(a.grad), rab) <= TOL_F64
    assert rel_l2(host(v.grad), rvb) <= TOL_F64
