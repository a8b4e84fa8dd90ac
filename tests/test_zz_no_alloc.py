"""The linear-recurrence scan VJP entry point that allocates nothing
(pvjp_linrec_scan_vjp_noalloc, its workspace a fixed array in the library)
against the entry point that takes a workspace, through the C ABI: two calls
in a row, the second smaller, each checked against the oracle to the FP64 /
FP32 bar and against the workspace entry point's result; sizes beyond the
fixed scratch are refused with a clear error.
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
def capi():
    from paper_2202_10297_amd import capi as c

    c.lib()
    return c


def noalloc(capi, dtype, a, b, ya, yb, ckpt=None, out=None, accumulate=False):
    ab = out[0] if out else torch.empty_like(a)
    bb = out[1] if out else torch.empty_like(b)
    capi.call("pvjp_linrec_scan_vjp_noalloc", 0 if dtype == "f32" else 1, a.data_ptr(), b.data_ptr(),
              ya.data_ptr(), yb.data_ptr(), a.numel(), ckpt.data_ptr() if ckpt is not None else None,
              ab.data_ptr(), bb.data_ptr(), int(accumulate), torch.cuda.current_stream().cuda_stream)
    return ab, bb


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("sizes", [(65536, 10007), (5_000_001, 65536), (1 << 22, 1)])
def test_noalloc_matches_workspace_entry(capi, orc, dtype, sizes):
    from paper_2202_10297_amd import ops

    tol = TOL_F64 if dtype == "f64" else TOL_F32
    for call, n in enumerate(sizes):
        a, b, ya, yb = workloads.linrec(n, dtype, seed=n + call)
        da, db, dya, dyb = dev(a), dev(b), dev(ya), dev(yb)
        _, _, ck = ops.linrec_scan(da, db)
        ref_ab, ref_bb = ops.linrec_scan_vjp(da, db, dya, dyb, ckpt=None)
        for ckpt in (None, ck):
            ab, bb = noalloc(capi, dtype, da, db, dya, dyb, ckpt=ckpt)
            got = [host(ab), host(bb)]
            # the same kernels on the same inputs: the same bits
            assert np.array_equal(got[0], host(ref_ab)) and np.array_equal(got[1], host(ref_bb))
            if n <= 65536:
                ra, rb = orc.linrec_scan_vjp(a, b, ya, yb)
                assert rel_l2(got, [ra, rb]) <= tol


def test_noalloc_accumulate_and_refusal(capi):
    from paper_2202_10297_amd import ops

    n = 300001
    a, b, ya, yb = workloads.linrec(n, "f64", seed=5)
    da, db, dya, dyb = dev(a), dev(b), dev(ya), dev(yb)
    ref_ab, ref_bb = ops.linrec_scan_vjp(da, db, dya, dyb)
    base = dev(np.full(n, 0.5)), dev(np.full(n, -1.0))
    noalloc(capi, "f64", da, db, dya, dyb, out=base, accumulate=True)
    assert np.array_equal(host(base[0]), host(ref_ab) + 0.5)
    assert np.array_equal(host(base[1]), host(ref_bb) - 1.0)
    cap = capi.lib().pvjp_linrec_scan_vjp_noalloc_max_bytes()
    big = 1 << 28  # FP64: about 28 MiB of workspace, beyond the fixed scratch
    assert capi.lib().pvjp_linrec_scan_vjp_ws_bytes(1, big) > cap
    st = capi.lib().pvjp_linrec_scan_vjp_noalloc(1, da.data_ptr(), db.data_ptr(), dya.data_ptr(), dyb.data_ptr(),
                                                 big, None, base[0].data_ptr(), base[1].data_ptr(), 0, None)
    assert st == capi.PVJP_ENOMEM and "fixed" in capi.last_error()
