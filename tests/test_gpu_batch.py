"""GPU parity of the segmented batch (one persistent launch for many scan VJPs
and sum-reduce VJPs) against the oracle run segment by segment, against one
launch per instance, and across HIP-graph replays."""
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
def batch():
    from paper_2202_10297_amd import batch as b, capi

    capi.lib()
    return b


def seg_inputs(lengths, dtype, seed):
    total = int(np.sum(lengths))
    a, b, ya, yb = workloads.linrec(total, dtype, seed=seed)
    sy = workloads.rng(seed + 1).standard_normal(len(lengths)).astype(a.dtype)
    return a, b, ya, yb, sy


LENGTHS = [[1], [5000], [1, 2, 3], [1023, 1, 1024, 1025, 4096, 4097, 7], [64] * 100 + [3000] * 5,
           list(workloads.segment_lengths(60, 64, 20000, seed=3))]


@pytest.mark.parametrize("dtype", ["f32", "f64"])
@pytest.mark.parametrize("tile", [1024, 2048, 4096])
@pytest.mark.parametrize("case", range(len(LENGTHS)))
def test_seg_scan_and_batch_vjp(batch, orc, dtype, tile, case):
    lengths = np.array(LENGTHS[case], dtype=np.int64)
    a, b, ya, yb, sy = seg_inputs(lengths, dtype, seed=case + tile)
    plan = batch.SegPlan(lengths, torch.float32 if dtype == "f32" else torch.float64, tile=tile, grid=97)
    A, B, ck = plan.scan(dev(a), dev(b))
    ab, bb, sx = plan.vjp(dev(a), dev(b), dev(ya), dev(yb), ck, sum_ybar=dev(sy))
    A, B, ab, bb, sx = host(A), host(B), host(ab), host(bb), host(sx)
    off = plan.offsets
    refs = [[], [], [], []]
    for s in range(len(lengths)):
        sl = slice(off[s], off[s + 1])
        RA, RB = orc.linrec_scan(a[sl], b[sl])
        ra, rb = orc.linrec_scan_vjp(a[sl], b[sl], ya[sl], yb[sl])
        for lst, v in zip(refs, (RA, RB, ra, rb)):
            lst.append(v)
    R = [np.concatenate(x) for x in refs]
    assert rel_l2([A, B], R[:2]) <= tol(dtype)
    assert rel_l2([ab, bb], R[2:]) <= tol(dtype)
    assert np.array_equal(sx, np.repeat(sy, lengths))  # broadcast: exact


def test_seg_parts_alone_and_accumulate(batch, orc):
    lengths = np.array([700, 5, 9000, 64], dtype=np.int64)
    a, b, ya, yb, sy = seg_inputs(lengths, "f32", seed=9)
    plan = batch.SegPlan(lengths, torch.float32, tile=2048, grid=33)
    _, _, ck = plan.scan(dev(a), dev(b), outputs=False)
    # sum part only
    _, _, sx = plan.vjp(sum_ybar=dev(sy))
    assert np.array_equal(host(sx), np.repeat(sy, lengths))
    # scan part only, accumulating
    base = workloads.rng(4).standard_normal(a.size).astype(np.float32)
    ab, bb = dev(base), dev(base)
    plan.vjp(dev(a), dev(b), dev(ya), dev(yb), ck, a_bar=ab, b_bar=bb, accumulate=True)
    ra = np.concatenate([orc.linrec_scan_vjp(a[s:e], b[s:e], ya[s:e], yb[s:e])[0]
                         for s, e in zip(plan.offsets[:-1], plan.offsets[1:])])
    assert rel_l2(host(ab), base + ra) <= TOL_F32


def test_batch_matches_per_instance_launches(batch):
    from paper_2202_10297_amd import ops

    lengths = workloads.segment_lengths(40, 64, 50000, seed=5)
    a, b, ya, yb, sy = seg_inputs(lengths, "f32", seed=6)
    plan = batch.SegPlan(lengths, torch.float32)
    _, _, ck = plan.scan(dev(a), dev(b), outputs=False)
    ab, bb, _ = plan.vjp(dev(a), dev(b), dev(ya), dev(yb), ck)
    ab, bb = host(ab), host(bb)
    for s, e in zip(plan.offsets[:-1], plan.offsets[1:]):
        _, _, c1 = ops.linrec_scan(dev(a[s:e]), dev(b[s:e]))
        x, y = ops.linrec_scan_vjp(dev(a[s:e]), dev(b[s:e]), dev(ya[s:e]), dev(yb[s:e]), ckpt=c1)
        assert rel_l2([ab[s:e], bb[s:e]], [host(x), host(y)]) <= TOL_F32


def test_graph_replay(batch):
    lengths = workloads.segment_lengths(64, 64, 100000, seed=7)
    a, b, ya, yb, sy = seg_inputs(lengths, "f32", seed=8)
    plan = batch.SegPlan(lengths, torch.float32)
    da, db, dya, dyb, dsy = dev(a), dev(b), dev(ya), dev(yb), dev(sy)
    _, _, ck = plan.scan(da, db, outputs=False)
    eager = [host(t) for t in plan.vjp(da, db, dya, dyb, ck, sum_ybar=dsy)]
    outs = dict(a_bar=torch.empty_like(da), b_bar=torch.empty_like(db), sum_xbar=torch.empty_like(da))
    plan.capture(a=da, b=db, yA_bar=dya, yB_bar=dyb, ckpt=ck, sum_ybar=dsy, **outs)
    for rep in range(4):
        for t in outs.values():
            t.fill_(float("nan"))  # eager work between replays
        plan.replay()
        torch.cuda.synchronize()
        got = [host(outs["a_bar"]), host(outs["b_bar"]), host(outs["sum_xbar"])]
        assert rel_l2(got[:2], eager[:2]) <= TOL_F32, rep
        assert np.array_equal(got[2], eager[2]), rep


def test_batch_full_size_sampled(batch, orc):
    # 4096 segments, lengths log-uniform in [64, 2^20] (about 4.4e8 elements),
    # FP32: oracle on a sample of segments (incl. the shortest and longest),
    # the sum adjoint checked everywhere.
    lengths = workloads.segment_lengths(4096, 64, 1 << 20, seed=0)
    total = int(lengths.sum())
    g = workloads.rng(0)
    a = g.uniform(0.5, 1.0, total).astype(np.float32)
    b = g.standard_normal(total, dtype=np.float32)
    ya = g.standard_normal(total, dtype=np.float32)
    yb = g.standard_normal(total, dtype=np.float32)
    sy = g.standard_normal(4096).astype(np.float32)
    plan = batch.SegPlan(lengths, torch.float32)
    da, db = dev(a), dev(b)
    _, _, ck = plan.scan(da, db, outputs=False)
    ab, bb, sx = plan.vjp(da, db, dev(ya), dev(yb), ck, sum_ybar=dev(sy))
    torch.cuda.synchronize()
    pick = set(np.random.default_rng(1).choice(4096, 12, replace=False)) | {int(np.argmin(lengths)),
                                                                           int(np.argmax(lengths))}
    for s in sorted(pick):
        lo, hi = int(plan.offsets[s]), int(plan.offsets[s + 1])
        ra, rb = orc.linrec_scan_vjp(a[lo:hi], b[lo:hi], ya[lo:hi], yb[lo:hi])
        assert rel_l2([ab[lo:hi].cpu().numpy(), bb[lo:hi].cpu().numpy()], [ra, rb]) <= TOL_F32, s
    sxh = sx.cpu().numpy()
    assert np.array_equal(sxh, np.repeat(sy, lengths))
