"""Element-wise parity of reduce_by_index (Sec. 5.1.2) at n = 2^24 FP32
against the oracle, on the paths that the full-size calls take: bins
m in {2^10, 2^16, 2^20}, indices uniform and Zipf(1.1), operators + and max,
primal and VJP.  Winners, counts and the max/+ adjoints are compared bit for
bit (a winner is an index, the adjoints are copies of hs_bar), the + bin sums
within the FP32 bar (relative L2 2e-5).  Where the plan is the partitioned one,
the test checks on the host that at least one bucket holds more records than
one work item takes, so the merge of a bucket's items is exercised.
"""
import ctypes

import numpy as np
import pytest

from _util import TOL_F32, rel_l2
from paper_2202_10297_amd import workloads

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

N = 1 << 24


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


def plan(op, n, m, counts):
    from paper_2202_10297_amd import capi

    info = (ctypes.c_int64 * 4)()
    capi.call("pvjp_hist_plan_info", {"add": capi.ADD, "max": capi.MAX}[op], capi.F32, n, m, int(counts),
              ctypes.cast(info, ctypes.c_void_p))
    return list(info)


def split_buckets(inds, m, info):
    """Number of buckets whose records span more than one work item."""
    bins_per_bucket, per_item = info[1], info[2]
    per_bucket = np.bincount(inds[(inds >= 0) & (inds < m)] // bins_per_bucket)
    return int((per_bucket > per_item).sum())


@pytest.mark.parametrize("dist", ["uniform", "zipf"])
@pytest.mark.parametrize("m", [1 << 10, 1 << 16, 1 << 20])
def test_hist_add_large(ops, orc, m, dist):
    from paper_2202_10297_amd import capi

    inds, vs, hb = workloads.hist(N, m, dist, "f32", seed=m + (dist == "zipf"))
    info = plan("add", N, m, True)
    if info[0] == capi.HIST_PATH_PARTITION and not (m == 1 << 20 and dist == "uniform"):
        assert split_buckets(inds, m, info) >= 1
    di = dev(inds)
    hs, aux = ops.hist("add", di, dev(vs), m, counts=True)
    ref = orc.hist("add", inds, vs, m)
    assert np.array_equal(host(aux["count"]), ref["count"])
    assert rel_l2(host(hs), ref["hs"]) <= TOL_F32
    hs2, _ = ops.hist("add", di, dev(vs), m)  # the plan without counts
    assert rel_l2(host(hs2), ref["hs"]) <= TOL_F32
    vb = host(ops.hist_vjp("add", di, None, m, aux, dev(hb)))
    assert np.array_equal(vb, orc.hist_vjp("add", inds, vs, hb).astype(np.float32))


@pytest.mark.parametrize("dist", ["uniform", "zipf"])
@pytest.mark.parametrize("m", [1 << 10, 1 << 16, 1 << 20])
def test_hist_max_large(ops, orc, m, dist):
    from paper_2202_10297_amd import capi

    inds, vs, hb = workloads.hist(N, m, dist, "f32", seed=m + 2 + (dist == "zipf"))
    # coarse values: ties inside a bin are common, so the lowest-index rule
    # decides many winners
    vs = (np.round(vs * 8) / 8).astype(np.float32)
    vs[::13] = -0.0
    info = plan("max", N, m, False)
    if info[0] == capi.HIST_PATH_PARTITION and not (m == 1 << 20 and dist == "uniform"):
        assert split_buckets(inds, m, info) >= 1
    di = dev(inds)
    hs, aux = ops.hist("max", di, dev(vs), m)
    ref = orc.hist("max", inds, vs, m)
    assert np.array_equal(host(aux["winner"]), ref["winner"])
    got = host(hs)
    assert np.array_equal(got, ref["hs"]) and np.array_equal(np.signbit(got), np.signbit(ref["hs"]))
    vb = host(ops.hist_vjp("max", di, None, m, aux, dev(hb)))
    assert np.array_equal(vb, orc.hist_vjp("max", inds, vs, hb).astype(np.float32))


def test_plan_info_names_the_paths(ops):
    from paper_2202_10297_amd import capi

    assert plan("add", N, 1 << 10, False)[0] == capi.HIST_PATH_LDS
    for m in (1 << 16, 1 << 20):
        for op in ("add", "max"):
            info = plan(op, N, m, False)
            assert info[0] in (capi.HIST_PATH_CACHE, capi.HIST_PATH_PARTITION)
