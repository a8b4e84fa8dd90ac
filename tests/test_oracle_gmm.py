"""Pins for the oracle's Gaussian-mixture objective and gradient.

The paper measures a GMM log-likelihood (Sec. 7.6) without stating it; the
objective used here is the textbook mixture with a precision-Cholesky
parametrisation (stated in oracle.h).  Pins: the K = 1, L = 0, q = 0 closed
form; central finite differences over every parameter; sum(alpha_bar) == 0;
permutation equivariance; and the per-point log-sum-exp against scipy.
"""
import math

import numpy as np
import pytest
from scipy.special import logsumexp

from _util import fd_grad, rel_l2
from paper_2202_10297_amd import workloads


def test_k1_closed_form(orc):
    N, D = 50, 4
    X, _, mu, _, _ = workloads.gmm(N, D, 1, seed=1, dtype="f64")
    alpha = np.array([0.37])
    q = np.zeros((1, D))
    l = np.zeros((1, D * (D - 1) // 2))
    Y = X - mu[0]
    ll, _ = orc.gmm_objective(X, alpha, mu, q, l)
    assert abs(ll - (-0.5 * np.sum(Y * Y) - 0.5 * N * D * math.log(2 * math.pi))) < 1e-10
    ab, mb, qb, lb = orc.gmm_vjp(X, alpha, mu, q, l)
    assert abs(ab[0]) < 1e-12
    assert np.allclose(mb[0], Y.sum(0), rtol=1e-12)
    assert np.allclose(qb[0], N - (Y * Y).sum(0), rtol=1e-12)
    # l_bar_rc = -sum_i y_ir y_ic  (z = y when L = 0, q = 0)
    ref = [-(Y[:, r] * Y[:, c]).sum() for r in range(D) for c in range(r)]
    assert np.allclose(lb[0], ref, rtol=1e-12)


@pytest.mark.parametrize("N,D,K", [(1, 1, 1), (5, 2, 3), (8, 3, 2)])
def test_fd_every_parameter(orc, N, D, K):
    X, alpha, mu, q, l = workloads.gmm(N, D, K, seed=N + D + K, dtype="f64")
    f = lambda a, m, qq, ll: orc.gmm_objective(X, a, m, qq, ll)[0]
    grads = orc.gmm_vjp(X, alpha, mu, q, l)
    fds = fd_grad(f, [alpha, mu, q, l])
    for g, r in zip(grads, fds):
        if r.size:
            assert np.allclose(g, r, rtol=1e-6, atol=1e-7)


def test_alpha_bar_sums_to_zero(orc):
    X, alpha, mu, q, l = workloads.gmm(200, 6, 7, seed=3, dtype="f64")
    ab, _, _, _ = orc.gmm_vjp(X, alpha, mu, q, l)
    assert abs(ab.sum()) <= 1e-9 * 200


def test_permutation_equivariance(orc):
    X, alpha, mu, q, l = workloads.gmm(40, 5, 6, seed=4, dtype="f64")
    perm = np.array([3, 0, 5, 1, 4, 2])
    g1 = orc.gmm_vjp(X, alpha, mu, q, l)
    g2 = orc.gmm_vjp(X, alpha[perm], mu[perm], q[perm], l[perm])
    for a, b in zip(g1, g2):
        assert rel_l2(b, a[perm]) < 1e-13
    assert abs(orc.gmm_objective(X, alpha, mu, q, l)[0] -
               orc.gmm_objective(X, alpha[perm], mu[perm], q[perm], l[perm])[0]) < 1e-9


def test_lse_against_scipy(orc):
    N, D, K = 30, 4, 5
    X, alpha, mu, q, l = workloads.gmm(N, D, K, seed=5, dtype="f64")
    ll, lse = orc.gmm_objective(X, alpha, mu, q, l)
    # Build Q_k explicitly and evaluate s_ik with numpy matrix products.
    S = np.empty((N, K))
    for k in range(K):
        Q = np.diag(np.exp(q[k]))
        r, c = np.tril_indices(D, -1)
        Q[r, c] = l[k][r * (r - 1) // 2 + c]
        Z = (X - mu[k]) @ Q.T
        S[:, k] = alpha[k] + q[k].sum() - 0.5 * (Z * Z).sum(1)
    assert np.allclose(lse, logsumexp(S, axis=1), rtol=1e-13)
    ref = logsumexp(S, axis=1).sum() - N * logsumexp(alpha) - 0.5 * N * D * math.log(2 * math.pi)
    assert abs(ll - ref) < 1e-10 * abs(ref)


def test_large_shift_is_stable(orc):
    # A huge common offset in alpha must not overflow: LSE uses the max shift.
    X, alpha, mu, q, l = workloads.gmm(10, 3, 4, seed=6, dtype="f64")
    ll1, _ = orc.gmm_objective(X, alpha, mu, q, l)
    ll2, _ = orc.gmm_objective(X, alpha + 800.0, mu, q, l)
    assert np.isfinite(ll2) and abs(ll1 - ll2) < 1e-9 * abs(ll1)
