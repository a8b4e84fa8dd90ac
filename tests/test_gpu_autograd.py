"""torch.autograd.Function wrappers: gradcheck in FP64 at small sizes (finite
differences of the GPU primal against the GPU VJP), and the GMM wrapper
against the oracle."""
import numpy as np
import pytest

from _util import TOL_F32, rel_l2
from paper_2202_10297_amd import workloads

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ag():
    from paper_2202_10297_amd import autograd, capi

    capi.lib()
    return autograd


def d64(x, grad=True):
    return torch.tensor(np.asarray(x, dtype=np.float64), device="cuda", requires_grad=grad)


def test_gradcheck_linrec(ag):
    a, b, _, _ = workloads.linrec(37, "f64", seed=1)
    assert torch.autograd.gradcheck(lambda x, y: ag.linrec_scan(x, y), (d64(a), d64(b)), eps=1e-6, atol=1e-7)


@pytest.mark.parametrize("op", ["add", "mul", "min", "max"])
def test_gradcheck_reduce(ag, op):
    x = workloads.product_values(11, 0, "f64", seed=2)  # distinct, non-zero: differentiable point
    assert torch.autograd.gradcheck(lambda v: ag.reduce(v, op), (d64(x),), eps=1e-6, atol=1e-7)


@pytest.mark.parametrize("op", ["add", "mul", "max"])
def test_gradcheck_reduce_by_index(ag, op):
    g = workloads.rng(3)
    inds = torch.tensor(g.integers(0, 4, 19).astype(np.int32), device="cuda")
    v = workloads.product_values(19, 0, "f64", seed=4)
    assert torch.autograd.gradcheck(lambda x: ag.reduce_by_index(x, inds, 4, op), (d64(v),), eps=1e-6, atol=1e-7)


def test_gradcheck_scatter(ag):
    xs = workloads.rng(5).standard_normal(12)
    vs = workloads.rng(6).standard_normal(4)
    is_ = torch.tensor([7, 0, 11, 3], dtype=torch.int32, device="cuda")
    assert torch.autograd.gradcheck(lambda x, v: ag.scatter(x, is_, v), (d64(xs), d64(vs)), eps=1e-6, atol=1e-7)


@pytest.mark.parametrize("fn", ["square", "exp", "log", "sin", "tanh"])
def test_gradcheck_map(ag, fn):
    x = workloads.rng(7).uniform(0.3, 2.0, 9)
    assert torch.autograd.gradcheck(lambda v: ag.map(v, fn), (d64(x),), eps=1e-6, atol=1e-7)


def test_composed_program(ag):
    # A small program built from the operators: loss = sum(max-hist(exp(scan_B)))
    a, b, _, _ = workloads.linrec(300, "f64", seed=8)
    inds = torch.tensor(workloads.rng(9).integers(0, 7, 300).astype(np.int32), device="cuda")

    def prog(x, y):
        _, B = ag.linrec_scan(x, y)
        return ag.reduce(ag.reduce_by_index(ag.map(B, "exp"), inds, 7, "max"), "add")

    assert torch.autograd.gradcheck(prog, (d64(a), d64(b)), eps=1e-6, atol=1e-6)


def test_gmm_autograd_matches_oracle(ag, orc):
    X, alpha, mu, q, l = workloads.gmm(300, 32, 6, seed=10)
    P = [torch.tensor(t, device="cuda", requires_grad=(i > 0)) for i, t in enumerate((X, alpha, mu, q, l))]
    ll = ag.gmm_loglik(*P)
    (2.0 * ll).backward()
    ref = orc.gmm_vjp(X, alpha, mu, q, l, 2.0)
    for t, r in zip(P[1:], ref):
        assert rel_l2(t.grad.cpu().numpy(), r) <= TOL_F32
