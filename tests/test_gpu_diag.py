"""Checked mode through the C ABI: the device counters of out-of-range
indices (reduce_by_index, Sec. 5.1.2), repeated scatter targets (Sec. 5.3
assumes unique ones), NaN and infinite values, each fed inputs with a known
number of such entries; and the workspace check after a lookback scan.
"""
import numpy as np
import pytest

from paper_2202_10297_amd import workloads

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


@pytest.fixture(scope="module")
def capi():
    from paper_2202_10297_amd import capi as c

    c.lib()
    return c


def counters():
    return torch.zeros(4, dtype=torch.int64, device="cuda")


def read(c):
    torch.cuda.synchronize()
    return c.cpu().numpy().tolist()


@pytest.mark.parametrize("n,m", [(1, 1), (1000, 7), (1 << 20, 1 << 16), (3000001, 5)])
def test_out_of_range_indices(capi, n, m):
    g = workloads.rng(n)
    inds = g.integers(0, m, n).astype(np.int32)
    bad = g.choice(n, size=min(n, 37), replace=False)
    inds[bad[::2]] = -1 - g.integers(0, 1000, bad[::2].size)
    inds[bad[1::2]] = m + g.integers(0, 1000, bad[1::2].size)
    c = counters()
    capi.call("pvjp_diag_indices", dev(inds).data_ptr(), n, m, c.data_ptr(), None)
    assert read(c) == [bad.size, 0, 0, 0]
    capi.call("pvjp_diag_indices", dev(inds).data_ptr(), n, m, c.data_ptr(), None)  # counts add up
    assert read(c)[0] == 2 * bad.size


@pytest.mark.parametrize("n,m", [(10, 10), (1 << 20, 1 << 18), (1 << 26, 1 << 24)])
def test_repeated_scatter_targets(capi, n, m):
    g = workloads.rng(m)
    is_ = g.permutation(n)[:m].astype(np.int32)
    # 3 targets repeated: one twice more, two once more; 2 out of range
    is_[m // 2] = is_[0]
    is_[m // 2 + 1] = is_[0]
    is_[m - 1] = is_[1]
    is_[m - 2] = is_[2]
    is_[3 % m] = n
    is_[4 % m] = -5
    want_dup = len({m // 2, m // 2 + 1, m - 1, m - 2} - {3 % m, 4 % m}) if m > 8 else None
    nb = capi.lib().pvjp_diag_scatter_ws_bytes(n)
    ws = torch.full((nb,), 0xAB, dtype=torch.uint8, device="cuda")  # the call clears its bitmap itself
    c = counters()
    capi.call("pvjp_diag_scatter", dev(is_).data_ptr(), m, n, c.data_ptr(), ws.data_ptr(), nb, None)
    got = read(c)
    if want_dup is not None:
        assert got == [2, want_dup, 0, 0]
    # brute force on the host
    ok = is_[(is_ >= 0) & (is_ < n)]
    assert got[0] == m - ok.size and got[1] == ok.size - np.unique(ok).size


def test_unique_targets_count_nothing(capi):
    n, m = 1 << 22, 1 << 20
    is_ = workloads.rng(3).permutation(n)[:m].astype(np.int32)
    nb = capi.lib().pvjp_diag_scatter_ws_bytes(n)
    ws = torch.empty(nb, dtype=torch.uint8, device="cuda")
    c = counters()
    capi.call("pvjp_diag_scatter", dev(is_).data_ptr(), m, n, c.data_ptr(), ws.data_ptr(), nb, None)
    assert read(c) == [0, 0, 0, 0]


@pytest.mark.parametrize("dtype", ["f32", "f64"])
@pytest.mark.parametrize("n", [1, 999, 1 << 20])
def test_nonfinite_values(capi, dtype, n):
    x = workloads.rng(n).standard_normal(n).astype(np.float32 if dtype == "f32" else np.float64)
    pos = workloads.rng(n + 1).permutation(n)
    k = min(n, 11)
    x[pos[:k][0::3]] = np.nan
    x[pos[:k][1::3]] = np.inf
    x[pos[:k][2::3]] = -np.inf
    c = counters()
    capi.call("pvjp_diag_nonfinite", 0 if dtype == "f32" else 1, dev(x).data_ptr(), n, c.data_ptr(), None)
    assert read(c) == [0, 0, int(np.isnan(x).sum()), int(np.isinf(x).sum())]


def test_refusals(capi):
    c = counters()
    assert capi.lib().pvjp_diag_indices(None, 5, 3, c.data_ptr(), None) == capi.PVJP_EINVAL
    assert capi.lib().pvjp_diag_nonfinite(7, c.data_ptr(), 1, c.data_ptr(), None) == capi.PVJP_EINVAL
    is_ = dev(np.arange(100, dtype=np.int32))
    small = torch.empty(4, dtype=torch.uint8, device="cuda")
    assert capi.lib().pvjp_diag_scatter(is_.data_ptr(), 100, 1 << 20, c.data_ptr(), small.data_ptr(), 4,
                                        None) == capi.PVJP_ENOMEM


def test_checked_mode_in_ops(capi):
    from paper_2202_10297_amd import ops

    ops.set_checked(True)
    try:
        ops.diag(reset=True)
        n, m = 100000, 1000
        inds, vs, hb = workloads.hist(n, m, "uniform", "f32", seed=4)
        inds = inds.copy()
        vs = vs.copy()
        inds[[5, 6, 7]] = [-1, m, m + 10]
        vs[9] = np.nan
        hs, aux = ops.hist("add", dev(inds), dev(vs), m)
        d = ops.diag(reset=True)
        assert d == {"oob": 3, "dup": 0, "nan": 1, "inf": 0}
        xs = dev(np.zeros(5000, dtype=np.float32))
        is_ = np.arange(0, 5000, 7, dtype=np.int32)
        is_[10] = is_[11]
        ops.scatter_(xs, dev(is_), dev(np.ones(is_.size, dtype=np.float32)))
        assert ops.diag(reset=True) == {"oob": 0, "dup": 1, "nan": 0, "inf": 0}
        # a lookback scan on a clean workspace passes the check
        a, b, ya, yb = workloads.linrec(300001, "f32", seed=1)
        ops.linrec_scan(dev(a), dev(b))
        assert ops.diag()["nan"] == 0
    finally:
        ops.set_checked(False)
