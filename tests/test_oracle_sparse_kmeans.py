"""Pins for the oracle's sparse k-means (Sec. 7.5): CSR points, dense centres,
squared distance of the densified row.  Checked against numpy on the densified points (all-pairs
distances, argmin, the closed-form gradient), against the separately pinned
dense-k-means oracle (a taped gradient) on the same densified points, against
central differences of the numpy objective, and the Hessian-vector product
against 2 f_bar n_k C_dot_k.
"""
import numpy as np
import pytest

from _util import fd_grad, rel_l2
from paper_2202_10297_amd import workloads


def dense(rowptr, col, val, D):
    N = rowptr.size - 1
    X = np.zeros((N, D))
    for i in range(N):
        X[i, col[rowptr[i]:rowptr[i + 1]]] = val[rowptr[i]:rowptr[i + 1]]
    return X


def np_objective(X, C):
    d = ((X[:, None, :] - C[None, :, :]) ** 2).sum(-1)
    return d.min(axis=1).sum(), d.argmin(axis=1), d


@pytest.mark.parametrize("N,D,K,L", [(1, 3, 1, 2), (60, 40, 3, 6), (300, 700, 5, 25), (200, 2500, 8, 40)])
def test_objective_matches_dense_numpy(orc, N, D, K, L):
    rp, cl, v, C = workloads.sparse_kmeans(N, D, K, L, "f64", seed=N + D)
    C = C + workloads.rng(3).standard_normal(C.shape) * 0.1  # break exact ties between centres
    f, a = orc.sparse_kmeans_objective(rp, cl, v, D, C)
    X = dense(rp, cl, v, D)
    rf, ra, dist = np_objective(X, C)
    assert abs(f - rf) <= 1e-12 * max(1.0, rf)
    # every distance, against numpy's (pairwise-summed) squared distances,
    # and the objective is the sum of each row's smallest one
    od = orc.sparse_kmeans_distances(rp, cl, v, D, C)
    assert np.allclose(od, dist, rtol=1e-13, atol=0)
    assert f == od.min(axis=1).sum() or abs(f - od.min(axis=1).sum()) <= 1e-13 * f
    assert np.array_equal(a, od.argmin(axis=1))
    # the same nearest centre wherever the two best distances are not within rounding
    srt = np.sort(dist, axis=1)
    clear = (srt[:, 1] - srt[:, 0]) > 1e-9 * np.maximum(1.0, srt[:, 0]) if K > 1 else np.ones(N, bool)
    assert np.array_equal(a[clear], ra[clear])


@pytest.mark.parametrize("N,D,K,L", [(60, 40, 3, 6), (300, 700, 5, 25)])
def test_gradient_against_dense_oracle_and_numpy(orc, N, D, K, L):
    rp, cl, v, C = workloads.sparse_kmeans(N, D, K, L, "f64", seed=N)
    C = C + workloads.rng(4).standard_normal(C.shape) * 0.1
    g = orc.sparse_kmeans_vjp(rp, cl, v, D, C, 0.75)
    X = dense(rp, cl, v, D)
    assert rel_l2(g, orc.kmeans_vjp(X, C, 0.75)) <= 1e-12  # the taped dense oracle
    _, a, _ = np_objective(X, C)
    n = np.bincount(a, minlength=K).astype(float)
    S = np.zeros_like(C)
    np.add.at(S, a, X)
    assert rel_l2(g, 2 * 0.75 * (n[:, None] * C - S)) <= 1e-13


def test_gradient_finite_differences(orc):
    D = 12
    rp, cl, v, C = workloads.sparse_kmeans(40, D, 3, 5, "f64", seed=7)
    C = C + workloads.rng(8).standard_normal(C.shape) * 0.3
    X = dense(rp, cl, v, D)
    (ref,) = fd_grad(lambda c: np_objective(X, c)[0], [C], h_rel=1e-7)
    assert rel_l2(orc.sparse_kmeans_vjp(rp, cl, v, D, C), ref) <= 1e-7


def test_hvp_and_empty_rows_and_clusters(orc):
    D, K = 50, 4
    rp, cl, v, C = workloads.sparse_kmeans(80, D, K, 4, "f64", seed=9)
    # an empty row (distance |c_k|^2) and a centre far from everything
    rp = np.concatenate([[0], rp[1:], [rp[-1]]])
    C = C + 0.05
    C[3] = 1e3
    Cd = workloads.rng(10).standard_normal(C.shape)
    f, a = orc.sparse_kmeans_objective(rp, cl, v, D, C)
    assert a[-1] == int(np.argmin((C ** 2).sum(1)))
    n = np.bincount(a, minlength=K).astype(float)
    assert n[3] == 0
    assert rel_l2(orc.sparse_kmeans_hvp(rp, cl, v, D, C, Cd, 0.5), 2 * 0.5 * n[:, None] * Cd) <= 1e-14
    g = orc.sparse_kmeans_vjp(rp, cl, v, D, C)
    assert np.all(g[3] == 0)
