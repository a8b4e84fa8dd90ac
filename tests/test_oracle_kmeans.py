"""Pins for the oracle's dense k-means (Sec. 7.4): objective, gradient (VJP)
and the jvp of the VJP (Hessian-vector product), against numpy's all-pairs
distances, the closed-form gradient 2 f_bar (n_k c_k - S_k) (S_k the sum of
the points assigned to k), the closed-form Hessian-vector product
2 f_bar n_k C_dot_k, and central differences of a numpy objective.
"""
import numpy as np
import pytest

from _util import fd_grad, rel_l2
from paper_2202_10297_amd import workloads


def np_objective(X, C):
    d = ((X[:, None, :] - C[None, :, :]) ** 2).sum(-1)
    return d.min(axis=1).sum(), d.argmin(axis=1)


def closed_grad(X, C, a, f_bar):
    K, D = C.shape
    n = np.bincount(a, minlength=K).astype(np.float64)
    S = np.zeros((K, D))
    np.add.at(S, a, X)
    return 2 * f_bar * (n[:, None] * C - S), n


@pytest.mark.parametrize("N,D,K", [(1, 3, 1), (50, 2, 3), (500, 35, 5), (300, 16, 40)])
def test_objective_matches_numpy(orc, N, D, K):
    X, C = workloads.kmeans(N, D, K, "f64", seed=N + D + K)
    f, a = orc.kmeans_objective(X, C)
    rf, ra = np_objective(X, C)
    assert abs(f - rf) <= 1e-12 * max(1.0, rf)
    assert np.array_equal(a, ra)


@pytest.mark.parametrize("N,D,K", [(50, 2, 3), (500, 35, 5), (300, 16, 40)])
def test_gradient_closed_form(orc, N, D, K):
    X, C = workloads.kmeans(N, D, K, "f64", seed=N)
    g = orc.kmeans_vjp(X, C, 0.75)
    _, a = np_objective(X, C)
    ref, _ = closed_grad(X, C, a, 0.75)
    assert rel_l2(g, ref) <= 1e-13


def test_gradient_finite_differences(orc):
    X, C = workloads.kmeans(60, 3, 4, "f64", seed=2)
    g = orc.kmeans_vjp(X, C, 1.0)
    (ref,) = fd_grad(lambda c: np_objective(X, c)[0], [C], h_rel=1e-7)
    assert rel_l2(g, ref) <= 1e-7


@pytest.mark.parametrize("N,D,K", [(500, 35, 5), (300, 16, 40)])
def test_hvp_closed_form(orc, N, D, K):
    X, C = workloads.kmeans(N, D, K, "f64", seed=N + 1)
    Cd = workloads.rng(3).standard_normal(C.shape)
    h = orc.kmeans_hvp(X, C, Cd, 0.5)
    _, a = np_objective(X, C)
    _, n = closed_grad(X, C, a, 0.5)
    assert rel_l2(h, 2 * 0.5 * n[:, None] * Cd) <= 1e-13
    # with C_dot = 1 it is the Hessian's diagonal, and the Newton step
    # C - g / diag(H) is the mean of each cluster (Lloyd's update)
    diag = orc.kmeans_hvp(X, C, np.ones_like(C), 1.0)
    g = orc.kmeans_vjp(X, C, 1.0)
    nz = n > 0
    S = np.zeros_like(C)
    np.add.at(S, a, X)
    assert rel_l2((C - g / np.where(diag == 0, 1, diag))[nz], (S / np.maximum(n, 1)[:, None])[nz]) <= 1e-13


def test_empty_cluster_has_zero_gradient(orc):
    X, C = workloads.kmeans(40, 2, 3, "f64", seed=4)
    C[2] = 1e6  # nobody is closest to it
    g = orc.kmeans_vjp(X, C, 1.0)
    h = orc.kmeans_hvp(X, C, np.ones_like(C), 1.0)
    assert np.all(g[2] == 0) and np.all(h[2] == 0)


def test_ties_go_to_the_lowest_centre(orc):
    X = np.array([[0.0, 0.0], [1.0, 0.0]])
    # the origin is at distance 2 from all three; (1, 0) at 1 from the first two
    C = np.array([[1.0, 1.0], [1.0, -1.0], [-1.0, 1.0]])
    _, a = orc.kmeans_objective(X, C)
    assert a[0] == 0 and a[1] == 0
