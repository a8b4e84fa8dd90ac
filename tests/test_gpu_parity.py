"""GPU parity: every operator's primal and VJP through the C ABI against the
oracle, on the same seeded inputs.

Bars: indices, counts, winners, gathers and broadcasts bit-exact; FP64
gradients within relative L2 1e-12; FP32 within 2e-5 (against the FP64
oracle on the same FP32 inputs).  Sizes span several tiles, ragged tails and
the edge cases (empty, single element, exact tile multiples).
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


def tol(dtype):
    return TOL_F64 if dtype == "f64" else TOL_F32


@pytest.fixture(scope="module")
def ops():
    from paper_2202_10297_amd import capi, ops as o

    capi.lib()  # loud failure if the native library is missing
    return o


# ------------------------------------------------------------ linrec scan
SCAN_SIZES = {"f64": [1, 2, 63, 64, 65, 1023, 1024, 2047, 2048, 2049, 4103, 65536, 100003],
              "f32": [1, 3, 4095, 4096, 4097, 12289, 65536, 300001]}


@pytest.mark.parametrize("dtype,n", [(d, n) for d in SCAN_SIZES for n in SCAN_SIZES[d]])
def test_linrec_scan_and_vjp(ops, orc, dtype, n):
    a, b, ya, yb = workloads.linrec(n, dtype, seed=n)
    A, B, ck = ops.linrec_scan(dev(a), dev(b))
    RA, RB = orc.linrec_scan(a, b)
    assert rel_l2([host(A), host(B)], [RA, RB]) <= tol(dtype)
    ra, rb = orc.linrec_scan_vjp(a, b, ya, yb)
    ab, bb = ops.linrec_scan_vjp(dev(a), dev(b), dev(ya), dev(yb), ckpt=ck)
    assert rel_l2([host(ab), host(bb)], [ra, rb]) <= tol(dtype)
    # without a checkpoint: the VJP recomputes it in a pre-pass
    ab2, bb2 = ops.linrec_scan_vjp(dev(a), dev(b), dev(ya), dev(yb), ckpt=None)
    assert rel_l2([host(ab2), host(bb2)], [ra, rb]) <= tol(dtype)


# Past 4096 tiles the scan takes the reduce-then-scan form (tile aggregates,
# one-block scan of the aggregates, scan with given prefixes); the ragged
# last tile and the checkpoint pre-pass are covered too.
@pytest.mark.parametrize("dtype,n", [("f64", 4097 * 2048 + 123), ("f32", 4097 * 4096 + 5)])
def test_linrec_three_pass_form(ops, orc, dtype, n):
    a, b, ya, yb = workloads.linrec(n, dtype, seed=7)
    A, B, ck = ops.linrec_scan(dev(a), dev(b))
    RA, RB = orc.linrec_scan(a, b)
    assert rel_l2([host(A), host(B)], [RA, RB]) <= tol(dtype)
    RCK = np.stack([np.concatenate([[1.0], RA[1023:-1:1024]]), np.concatenate([[0.0], RB[1023:-1:1024]])], 1)
    assert rel_l2(host(ck).reshape(-1, 2), RCK) <= tol(dtype)
    ra, rb = orc.linrec_scan_vjp(a, b, ya, yb)
    ab, bb = ops.linrec_scan_vjp(dev(a), dev(b), dev(ya), dev(yb), ckpt=ck)
    assert rel_l2([host(ab), host(bb)], [ra, rb]) <= tol(dtype)
    ab2, bb2 = ops.linrec_scan_vjp(dev(a), dev(b), dev(ya), dev(yb), ckpt=None)
    assert rel_l2([host(ab2), host(bb2)], [ra, rb]) <= tol(dtype)


def test_linrec_checkpoint_values(ops, orc):
    n = 5000
    a, b, _, _ = workloads.linrec(n, "f64", seed=1)
    _, _, ck = ops.linrec_scan(dev(a), dev(b))
    ck = host(ck).reshape(-1, 2)
    RA, RB = orc.linrec_scan(a, b)
    assert ck.shape[0] == (n + 1023) // 1024
    assert ck[0, 0] == 1.0 and ck[0, 1] == 0.0
    for c in range(1, ck.shape[0]):
        assert rel_l2(ck[c], [RA[c * 1024 - 1], RB[c * 1024 - 1]]) <= 1e-13


def test_linrec_accumulate(ops, orc):
    n = 9001
    a, b, ya, yb = workloads.linrec(n, "f64", seed=4)
    base_a = workloads.rng(5).standard_normal(n)
    base_b = workloads.rng(6).standard_normal(n)
    _, _, ck = ops.linrec_scan(dev(a), dev(b))
    ab, bb = dev(base_a), dev(base_b)
    ops.linrec_scan_vjp(dev(a), dev(b), dev(ya), dev(yb), ckpt=ck, a_bar=ab, b_bar=bb, accumulate=True)
    ra, rb = orc.linrec_scan_vjp(a, b, ya, yb)
    assert rel_l2([host(ab), host(bb)], [ra + base_a, rb + base_b]) <= 1e-12


def test_linrec_workspace_reuse_many_launches(ops, orc):
    # The lookback state resets itself at the end of every launch: repeated
    # launches of different sizes on one workspace stay correct.
    for rep, n in enumerate([70000, 3000, 70000, 1, 140000, 2048] * 3):
        a, b, ya, yb = workloads.linrec(n, "f64", seed=rep)
        A, B, ck = ops.linrec_scan(dev(a), dev(b))
        ab, bb = ops.linrec_scan_vjp(dev(a), dev(b), dev(ya), dev(yb), ckpt=ck)
        RA, RB = orc.linrec_scan(a, b)
        ra, rb = orc.linrec_scan_vjp(a, b, ya, yb)
        assert rel_l2([host(A), host(B)], [RA, RB]) <= 1e-12
        assert rel_l2([host(ab), host(bb)], [ra, rb]) <= 1e-12


def test_linrec_mixed_dtype_sizes_share_workspace(ops, orc):
    # Regression: a workspace cached from an FP64 VJP of 100003 elements was
    # reused by an FP32 VJP of one element whose checkpoint pre-pass used to
    # take its header from a different offset (an old tile-state word), and
    # hung.  All lookback kernels now share the header at offset 0.
    from paper_2202_10297_amd import capi

    for dtype, n in [("f64", 100003), ("f32", 1), ("f64", 5), ("f32", 300001), ("f64", 2049), ("f32", 4097)]:
        a, b, ya, yb = workloads.linrec(n, dtype, seed=n)
        ab, bb = ops.linrec_scan_vjp(dev(a), dev(b), dev(ya), dev(yb), ckpt=None)
        ra, rb = orc.linrec_scan_vjp(a, b, ya, yb)
        assert rel_l2([host(ab), host(bb)], [ra, rb]) <= tol(dtype)
    for key, buf in ops.WS._bufs.items():
        if "linrec" in key[2]:
            assert capi.lib().pvjp_ws_check(buf.data_ptr(), 0, None) == capi.PVJP_OK, capi.last_error()


def test_linrec_a_equal_one(ops):
    # a == 1: B is a prefix sum, b_bar the suffix sum of yB_bar.
    n = 50000
    g = workloads.rng(8)
    b, ya, yb = g.standard_normal(n), g.standard_normal(n), g.standard_normal(n)
    a = np.ones(n)
    A, B, ck = ops.linrec_scan(dev(a), dev(b))
    assert np.array_equal(host(A), a)
    assert rel_l2(host(B), np.cumsum(b)) <= 1e-12
    _, bb = ops.linrec_scan_vjp(dev(a), dev(b), dev(ya), dev(yb), ckpt=ck)
    assert rel_l2(host(bb), np.cumsum(yb[::-1])[::-1]) <= 1e-12


# ----------------------------------------------------------------- reduce
RED_SIZES = [0, 1, 255, 256, 257, 65539, 1000003]


@pytest.mark.parametrize("dtype", ["f32", "f64"])
@pytest.mark.parametrize("n", RED_SIZES)
def test_reduce_add(ops, orc, dtype, n):
    x = workloads.rng(n).standard_normal(n).astype(np.float32 if dtype == "f32" else np.float64)
    y, aux = ops.reduce("add", dev(x))
    ry = orc.reduce("add", x)[0]
    got = host(y)[0]
    assert abs(got - ry) <= (1e-12 if dtype == "f64" else 1e-6) * max(1.0, np.abs(x).sum())
    yb = np.array([1.75], dtype=x.dtype)
    xb = host(ops.reduce_vjp("add", dev(x), aux, dev(yb)))
    assert np.array_equal(xb, orc.reduce_vjp("add", x, yb[0]).astype(x.dtype))


# 700 factors of magnitude about e^(+-1) leave the FP32 range: FP64 only
MUL_CASES = [(d, n, z) for d in ("f32", "f64")
             for n, z in [(1, 0), (1, 1), (150, 0), (150, 1), (150, 2), (150, 3), (700, 0)] if d == "f64" or n <= 200]


@pytest.mark.parametrize("dtype,n,zeros", MUL_CASES)
def test_reduce_mul(ops, orc, dtype, n, zeros):
    x = workloads.product_values(n, zeros, dtype, seed=n + zeros)
    y, aux = ops.reduce("mul", dev(x))
    ry, _, rp, rz = orc.reduce("mul", x)
    assert int(host(aux["z"])[0]) == rz
    t = 1e-13 if dtype == "f64" else 3e-7
    assert abs(host(aux["p"])[0] - rp) <= t * abs(rp)
    assert abs(host(y)[0] - ry) <= t * abs(ry)
    yb = np.array([-0.625], dtype=x.dtype)
    xb = host(ops.reduce_vjp("mul", dev(x), aux, dev(yb)))
    ref = orc.reduce_vjp("mul", x, yb[0])
    assert rel_l2(xb, ref) <= (1e-12 if dtype == "f64" else TOL_F32)
    if zeros >= 1:
        assert np.array_equal(xb != 0, ref != 0)


@pytest.mark.parametrize("dtype", ["f32", "f64"])
@pytest.mark.parametrize("offset", [0, 1, 3])
def test_reduce_vector_and_unaligned(ops, orc, dtype, offset):
    # Many blocks of whole quads plus a ragged tail; offset > 0 passes a view
    # that is not 16-byte aligned (the scalar path).
    n = 1000003
    g = workloads.rng(offset + 7)
    dt = np.float32 if dtype == "f32" else np.float64
    base = g.uniform(0.995, 1.005, n + offset).astype(dt) * np.where(g.random(n + offset) < 0.5, -1, 1).astype(dt)
    base[offset + 12345] = 0
    base[offset + n - 2] = 0
    x = base[offset:]
    xd = dev(base)[offset:]
    y, aux = ops.reduce("mul", xd)
    ry, _, rp, rz = orc.reduce("mul", x)
    assert int(host(aux["z"])[0]) == rz == 2
    # A product of n factors rounds n times: about sqrt(n) units of the last
    # place; dropping or repeating one factor moves it by ~2.5e-3.
    ulp = 2.0 ** -53 if dtype == "f64" else 2.0 ** -24
    assert abs(host(aux["p"])[0] - rp) <= 3 * np.sqrt(n) * ulp * abs(rp)
    assert host(y)[0] == 0
    for op in ("min", "max"):
        xt = workloads.tie_values(n + offset, dtype, seed=offset)[offset:]
        xtd = dev(workloads.tie_values(n + offset, dtype, seed=offset))[offset:]
        y, aux = ops.reduce(op, xtd)
        ry, rarg, _, _ = orc.reduce(op, xt)
        assert int(host(aux["arg"])[0]) == rarg and host(y)[0] == ry
    xs = g.standard_normal(n).astype(dt)
    xsd = dev(np.concatenate([np.zeros(offset, dt), xs]))[offset:]
    y, _ = ops.reduce("add", xsd)
    assert abs(host(y)[0] - orc.reduce("add", xs)[0]) <= (1e-12 if dtype == "f64" else 1e-6) * np.abs(xs).sum()


@pytest.mark.parametrize("dtype", ["f32", "f64"])
@pytest.mark.parametrize("op", ["min", "max"])
@pytest.mark.parametrize("n", [0, 1, 300, 65537, 1000003])
def test_reduce_minmax(ops, orc, dtype, op, n):
    x = workloads.tie_values(n, dtype, seed=n)
    if n > 2:
        x[n // 3] = -0.0
    y, aux = ops.reduce(op, dev(x))
    ry, rarg, _, _ = orc.reduce(op, x)
    assert int(host(aux["arg"])[0]) == rarg
    got = host(y)[0]
    assert (got == ry) and (np.signbit(got) == np.signbit(ry))
    if n == 0:
        return
    yb = np.array([2.5], dtype=x.dtype)
    xb = host(ops.reduce_vjp(op, dev(x), aux, dev(yb)))
    assert np.array_equal(xb, orc.reduce_vjp(op, x, yb[0]))
    base = np.full(n, 0.5, dtype=x.dtype)
    xb2 = dev(base)
    ops.reduce_vjp(op, dev(x), aux, dev(yb), x_bar=xb2, accumulate=True)
    exp = base.copy()
    exp[rarg] += yb[0]
    assert np.array_equal(host(xb2), exp)


def test_reduce_signed_zero_tie(ops):
    x = np.array([-1.0, -0.0, 0.0, -2.0], dtype=np.float32)
    y, aux = ops.reduce("max", dev(x))
    assert int(host(aux["arg"])[0]) == 1 and np.signbit(host(y)[0])


# ------------------------------------------------------- reduce_by_index
HIST_CASES = [(0, 7), (1, 1), (1000, 1), (1000, 7), (65536 + 17, 1024), (200003, 5000), (200003, 9000),
              (300007, 1 << 16), (300007, 1 << 20)]


@pytest.mark.parametrize("dtype", ["f32", "f64"])
@pytest.mark.parametrize("dist", ["uniform", "zipf"])
@pytest.mark.parametrize("n,m", HIST_CASES)
def test_hist_add(ops, orc, dtype, dist, n, m):
    inds, vs, hb = workloads.hist(n, m, dist, dtype, seed=n + m)
    hs, aux = ops.hist("add", dev(inds), dev(vs), m, counts=True)
    ref = orc.hist("add", inds, vs, m)
    assert np.array_equal(host(aux["count"]), ref["count"])
    assert rel_l2(host(hs), ref["hs"]) <= tol(dtype)
    vb = host(ops.hist_vjp("add", dev(inds), None, m, aux, dev(hb)))
    assert np.array_equal(vb, orc.hist_vjp("add", inds, vs, hb).astype(vb.dtype))  # a gather: exact


@pytest.mark.parametrize("dtype", ["f32", "f64"])
@pytest.mark.parametrize("op", ["min", "max"])
@pytest.mark.parametrize("dist", ["uniform", "zipf"])
@pytest.mark.parametrize("n,m", HIST_CASES)
def test_hist_minmax(ops, orc, dtype, op, dist, n, m):
    inds, _, hb = workloads.hist(n, m, dist, dtype, seed=n + m + 1)
    vs = workloads.tie_values(n, dtype, seed=n + 2)  # many ties
    if n > 10:
        vs[::7] = -0.0
    hs, aux = ops.hist(op, dev(inds), dev(vs), m)
    ref = orc.hist(op, inds, vs, m)
    assert np.array_equal(host(aux["winner"]), ref["winner"])
    got = host(hs)
    assert np.array_equal(got, ref["hs"]) and np.array_equal(np.signbit(got), np.signbit(ref["hs"]))
    vb = host(ops.hist_vjp(op, dev(inds), None, m, aux, dev(hb)))
    assert np.array_equal(vb, orc.hist_vjp(op, inds, vs, hb).astype(vb.dtype))


@pytest.mark.parametrize("dtype", ["f32", "f64"])
@pytest.mark.parametrize("n,m", [(1, 1), (5000, 3), (20000, 64), (20000, 9000), (50000, 1 << 16)])
def test_hist_mul(ops, orc, dtype, n, m):
    g = workloads.rng(n + m)
    inds = g.integers(0, m, n).astype(np.int32)
    vs = workloads.product_values(n, max(1, n // 500), dtype, seed=n)
    # keep per-bin products in range: bins of ~n/m elements of magnitude ~1
    vs = np.where(np.abs(vs) > 0, np.sign(vs) * np.abs(vs) ** (1.0 / max(1.0, n / m / 20)), vs).astype(vs.dtype)
    hb = g.standard_normal(m).astype(vs.dtype)
    hs, aux = ops.hist("mul", dev(inds), dev(vs), m)
    ref = orc.hist("mul", inds, vs, m)
    assert np.array_equal(host(aux["z"]), ref["z"])
    assert rel_l2(host(aux["p"]), ref["p"]) <= tol(dtype)
    assert rel_l2(host(hs), ref["hs"]) <= tol(dtype)
    vb = host(ops.hist_vjp("mul", dev(inds), dev(vs), m, aux, dev(hb)))
    assert rel_l2(vb, orc.hist_vjp("mul", inds, vs, hb)) <= tol(dtype)


@pytest.mark.parametrize("dtype", ["f32", "f64"])
@pytest.mark.parametrize("m", [8192, 20480, 20481, 40960, 40961, 1 << 17])
@pytest.mark.parametrize("accumulate", [False, True])
def test_hist_add_vjp_gather_paths(ops, orc, dtype, m, accumulate):
    # Bins below and beyond the LDS-staged head, out-of-range indices, and a
    # length that is not a multiple of 4 (the tail is done separately).
    n = 262147
    g = workloads.rng(m + accumulate)
    inds = g.integers(-5, m + 5, n).astype(np.int32)
    inds[::3] = g.integers(0, 64, inds[::3].size)  # a hot head
    vs = g.standard_normal(n).astype(np.float32 if dtype == "f32" else np.float64)
    hb = g.standard_normal(m).astype(vs.dtype)
    base = g.standard_normal(n).astype(vs.dtype)
    aux = {}
    vb = dev(base) if accumulate else None
    out = ops.hist_vjp("add", dev(inds), None, m, aux, dev(hb), vs_bar=vb, accumulate=accumulate)
    got = host(out)
    ref = orc.hist_vjp("add", inds, vs, hb).astype(vs.dtype)
    assert np.array_equal(got, base + ref if accumulate else ref)


def test_hist_out_of_range_and_accumulate(ops, orc):
    n, m = 100000, 300
    g = workloads.rng(3)
    inds = g.integers(-20, m + 20, n).astype(np.int32)
    vs = g.standard_normal(n).astype(np.float32)
    hb = g.standard_normal(m).astype(np.float32)
    for op in ["add", "max"]:
        hs, aux = ops.hist(op, dev(inds), dev(vs), m, counts=True)
        ref = orc.hist(op, inds, vs, m)
        assert np.array_equal(host(aux["count"]), ref["count"])
        base = g.standard_normal(n).astype(np.float32)
        vb = dev(base)
        ops.hist_vjp(op, dev(inds), None, m, aux, dev(hb), vs_bar=vb, accumulate=True)
        exp = base + orc.hist_vjp(op, inds, vs, hb).astype(np.float32)
        assert np.array_equal(host(vb), exp)


# ----------------------------------------------------------------- scatter
@pytest.mark.parametrize("dtype", ["f32", "f64"])
@pytest.mark.parametrize("n,m", [(1, 1), (100, 0), (4096, 1024), (1 << 20, 1 << 18), (1000003, 777)])
def test_scatter(ops, orc, dtype, n, m):
    xs, is_, vs, yb = workloads.scatter(n, m, dtype, seed=n + m)
    x = dev(xs)
    saved = ops.scatter_(x, dev(is_), dev(vs))
    rys, rsaved = orc.scatter(xs, is_, vs)
    assert np.array_equal(host(x), rys)
    assert np.array_equal(host(saved), rsaved)
    ybar = dev(yb)
    vbar = ops.scatter_vjp_(ybar, dev(is_), ys=x, xs_saved=saved)
    rxb, rvb = orc.scatter_vjp(is_, yb)
    assert np.array_equal(host(ybar), rxb) and np.array_equal(host(vbar), rvb)
    assert np.array_equal(host(x), xs)  # restored


def test_scatter_out_of_range_accumulate(ops, orc):
    n = 1000
    is_ = np.array([5, -3, 999, 1000, 17], dtype=np.int32)
    xs = workloads.rng(1).standard_normal(n)
    vs = workloads.rng(2).standard_normal(5)
    yb = workloads.rng(3).standard_normal(n)
    x = dev(xs)
    saved = ops.scatter_(x, dev(is_), dev(vs))
    rys, rs = orc.scatter(xs, is_, vs)
    assert np.array_equal(host(x), rys) and np.array_equal(host(saved), rs)
    base = np.arange(5, dtype=np.float64)
    vbar = dev(base)
    ybar = dev(yb)
    ops.scatter_vjp_(ybar, dev(is_), vs_bar=vbar, accumulate=True)
    rxb, rvb = orc.scatter_vjp(is_, yb)
    assert np.array_equal(host(ybar), rxb) and np.array_equal(host(vbar), base + rvb)


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_scatter_unaligned_indices(ops, orc, dtype):
    # An index view one element into its buffer takes the scalar-load path.
    n, m = 50000, 4099
    xs, is_, vs, yb = workloads.scatter(n, m + 1, dtype, seed=11)
    dis = dev(is_)[1:]
    is_, vs = is_[1:], vs[1:]
    x = dev(xs)
    saved = ops.scatter_(x, dis, dev(vs))
    rys, rsaved = orc.scatter(xs, is_, vs)
    assert np.array_equal(host(x), rys) and np.array_equal(host(saved), rsaved)
    ybar = dev(yb)
    vbar = ops.scatter_vjp_(ybar, dis, ys=x, xs_saved=saved)
    rxb, rvb = orc.scatter_vjp(is_, yb)
    assert np.array_equal(host(ybar), rxb) and np.array_equal(host(vbar), rvb)
    assert np.array_equal(host(x), xs)


# --------------------------------------------------------------------- map
@pytest.mark.parametrize("dtype", ["f32", "f64"])
@pytest.mark.parametrize("fn", ["square", "exp", "log", "sin", "tanh"])
def test_map(ops, orc, dtype, fn):
    n = 100003
    g = workloads.rng(11)
    dt = np.float32 if dtype == "f32" else np.float64
    x = g.uniform(0.1, 3.0, n).astype(dt)
    yb = g.standard_normal(n).astype(dt)
    assert rel_l2(host(ops.map_(fn, dev(x))), orc.map_(fn, x)) <= tol(dtype)
    assert rel_l2(host(ops.map_vjp(fn, dev(x), dev(yb))), orc.map_vjp(fn, x, yb)) <= tol(dtype)


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_fig1(ops, orc, dtype):
    n = 65541
    g = workloads.rng(12)
    dt = np.float32 if dtype == "f32" else np.float64
    x0, x1, b0, b1 = (g.standard_normal(n).astype(dt) for _ in range(4))
    y0, y1 = ops.fig1(dev(x0), dev(x1))
    r0, r1 = orc.fig1(x0, x1)
    assert rel_l2([host(y0), host(y1)], [r0, r1]) <= tol(dtype)
    a0, a1 = ops.fig1_vjp(dev(x0), dev(x1), dev(b0), dev(b1))
    s0, s1 = orc.fig1_vjp(x0, x1, b0, b1)
    assert rel_l2([host(a0), host(a1)], [s0, s1]) <= tol(dtype)
