"""GPU parity of the regular segmented scan with a general operator (Sec.
5.2's vectorised-operator rule: B independent scans of L elements in one
launch sequence) and its VJP, through the C ABI, against the oracle's
row-by-row scan on the same seeded inputs.

Every row must also be bit-identical to the single-scan entry point run on
that row alone (same tiles, same groups, same arithmetic).  Bars otherwise as
for the single scan: FP64 relative L2 1e-12 (outputs 1e-13), FP32 2e-5
(outputs 1e-6).  Shapes span one tile, ragged tails, rows longer than 64
tiles (grouped aggregates), many short rows up to the largest B = 65535,
and rows that are not 16-byte aligned (element path).
"""
import numpy as np
import pytest

from _util import TOL_F32, TOL_F64, rel_l2
from paper_2202_10297_amd import workloads

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

OPS = ["logaddexp", "linrec", "mat2"]


def tile(op, dtype):
    if op == "logaddexp":
        return 2048 if dtype == "f32" else 1024
    return 1024  # linear recurrence and 2x2 product: 256 threads x 4 items


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


def rows(op, B, L, dtype, seed):
    xs, ybs = workloads.gop_scan(op, B * L, dtype, seed=seed)
    xs = [x.reshape(B, L) for x in xs]
    if op == "logaddexp" and L > 3:
        xs[0][:, 0] = -np.inf  # every row starts with the neutral element
        xs[0][B // 2, L // 2] = -np.inf
    return xs, [y.reshape(B, L) for y in ybs]


def close(got, ref, bound):
    got = [np.asarray(g, dtype=np.float64) for g in got]
    for g, r in zip(got, ref):
        assert np.array_equal(np.isneginf(g), np.isneginf(r))
    fin = lambda arrs: [np.where(np.isneginf(r), 0.0, a) for a, r in zip(arrs, ref)]
    return rel_l2(fin(got), fin(ref)) <= bound


def shapes(op, dtype):
    t = tile(op, dtype)
    return [(1, 1), (3, 5), (7, t - 1), (5, t + 1), (4, 3 * t + 5), (2, 64 * t + 7), (300, 100)]


CASES = [(op, d, B, L) for op in OPS for d in ("f32", "f64") for B, L in shapes(op, d)]


@pytest.mark.parametrize("op,dtype,B,L", CASES)
def test_batched_scan_and_vjp(ops, orc, op, dtype, B, L):
    xs, ybs = rows(op, B, L, dtype, seed=B * 7 + L)
    dx = [dev(x) for x in xs]
    ys, ck = ops.scan_generic_batched(op, dx)
    xb = ops.scan_generic_batched_vjp(op, dx, [dev(y) for y in ybs], ckpt=ck)
    ys, xb = [host(y) for y in ys], [host(g) for g in xb]
    # each row equals the single scan of that row, bit for bit
    for b in sorted({0, B // 2, B - 1}):
        ys1, ck1 = ops.scan_generic(op, [dev(x[b]) for x in xs])
        xb1 = ops.scan_generic_vjp(op, [dev(x[b]) for x in xs], [dev(y[b]) for y in ybs], ckpt=ck1)
        assert all(np.array_equal(host(a), r[b]) for a, r in zip(ys1, ys))
        assert all(np.array_equal(host(a), r[b]) for a, r in zip(xb1, xb))
    assert close(ys, orc.scan_generic_rows(op, xs), 1e-13 if dtype == "f64" else 1e-6)
    assert rel_l2(xb, orc.scan_generic_rows_vjp(op, xs, ybs)) <= tol(dtype)


@pytest.mark.parametrize("op", OPS)
def test_without_checkpoint_and_accumulate(ops, orc, op):
    B, L = 6, 2 * tile(op, "f64") + 33
    xs, ybs = rows(op, B, L, "f64", seed=4)
    dx, dyb = [dev(x) for x in xs], [dev(y) for y in ybs]
    ys, ck = ops.scan_generic_batched(op, dx)
    a = [host(g) for g in ops.scan_generic_batched_vjp(op, dx, dyb, ckpt=ck)]
    b = [host(g) for g in ops.scan_generic_batched_vjp(op, dx, dyb)]  # prefixes recomputed
    assert all(np.array_equal(u, v) for u, v in zip(a, b))
    base = [dev(np.full((B, L), -0.5)) for _ in xs]
    c = ops.scan_generic_batched_vjp(op, dx, dyb, x_bar=base, accumulate=True, ckpt=ck)
    assert rel_l2([host(g) + 0.5 for g in c], orc.scan_generic_rows_vjp(op, xs, ybs)) <= 2 * TOL_F64


def test_most_rows_and_unaligned(ops, orc):
    # B = 65535 rows of 3 (the grid's second dimension at its limit; rows of
    # 12 bytes take the element path)
    B, L = 65535, 3
    xs, ybs = rows("linrec", B, L, "f32", seed=8)
    dx = [dev(x) for x in xs]
    ys, ck = ops.scan_generic_batched("linrec", dx)
    xb = ops.scan_generic_batched_vjp("linrec", dx, [dev(y) for y in ybs], ckpt=ck)
    ys, xb = [host(y) for y in ys], [host(g) for g in xb]
    pick = np.array([0, 1, 777, 40000, B - 1])
    sub = [x[pick] for x in xs]
    assert rel_l2([y[pick] for y in ys], orc.scan_generic_rows("linrec", sub)) <= 1e-6
    assert rel_l2([g[pick] for g in xb], orc.scan_generic_rows_vjp("linrec", sub, [y[pick] for y in ybs])) <= TOL_F32
    from paper_2202_10297_amd import capi

    with pytest.raises(capi.PvjpError):
        ops.scan_generic_batched("linrec", [dev(np.zeros((65536, 1), np.float32))] * 2)


def test_vectorised_operator_rule(ops):
    # a log-add-exp scan over vectors of w = 24 components, [n x w], is the
    # batched scan of the transposed [w x n] arrays
    n, w = 5000, 24
    x = workloads.rng(9).standard_normal((n, w))
    ys, _ = ops.scan_generic_batched("logaddexp", [dev(x).t().contiguous()])
    got = host(ys[0].t().contiguous())
    assert rel_l2(got, np.logaddexp.accumulate(x, axis=0)) <= 1e-12


@pytest.mark.parametrize("op,dtype", [("logaddexp", "f32"), ("linrec", "f64"), ("mat2", "f32")])
def test_benchmark_size_sampled_rows(ops, orc, op, dtype):
    B, L = 1024, 65536
    xs, ybs = rows(op, B, L, dtype, seed=0)
    dx = [dev(x) for x in xs]
    ys, ck = ops.scan_generic_batched(op, dx)
    xb = ops.scan_generic_batched_vjp(op, dx, [dev(y) for y in ybs], ckpt=ck)
    for b in (0, 517, B - 1):
        assert close([host(y[b]) for y in ys], orc.scan_generic(op, [x[b] for x in xs]),
                     1e-12 if dtype == "f64" else 1e-5)
        assert rel_l2([host(g[b]) for g in xb], orc.scan_generic_vjp(op, [x[b] for x in xs], [y[b] for y in ybs])) \
            <= tol(dtype)


def test_autograd(orc):
    from paper_2202_10297_amd import autograd

    xs, ybs = rows("mat2", 5, 3001, "f64", seed=13)
    t = [dev(x).requires_grad_() for x in xs]
    ys = autograd.scan_generic_batched("mat2", *t)
    sum((y * dev(g)).sum() for y, g in zip(ys, ybs)).backward()
    assert rel_l2([host(x.grad) for x in t], orc.scan_generic_rows_vjp("mat2", xs, ybs)) <= TOL_F64
