"""Shared helpers for the tests: error measures and finite differences.

Nothing here implements a rule of the method; finite differences only call a
primal function and difference its outputs.
"""
from __future__ import annotations

import numpy as np

TOL_F64 = 1e-12  # relative L2 bound for FP64 gradients
TOL_F32 = 2e-5  # relative L2 bound for FP32 gradients (vs the FP64 oracle)


def rel_l2(got, ref) -> float:
    """||got - ref||_2 / max(||ref||_2, 1e-300) over all components."""
    got = np.concatenate([np.ravel(np.asarray(g, dtype=np.float64)) for g in _seq(got)])
    ref = np.concatenate([np.ravel(np.asarray(r, dtype=np.float64)) for r in _seq(ref)])
    return float(np.linalg.norm(got - ref) / max(np.linalg.norm(ref), 1e-300))


def _seq(x):
    return x if isinstance(x, (list, tuple)) else [x]


def fd_grad(f, xs, h_rel=1e-6):
    """Central finite differences of the scalar function f(*xs) w.r.t. every
    component of every array in xs; h = h_rel * max(1, |x|)."""
    xs = [np.array(x, dtype=np.float64) for x in xs]
    grads = []
    for a in range(len(xs)):
        g = np.zeros_like(xs[a])
        flat = xs[a].reshape(-1)
        gf = g.reshape(-1)
        for j in range(flat.size):
            h = h_rel * max(1.0, abs(flat[j]))
            old = flat[j]
            flat[j] = old + h
            fp = f(*xs)
            flat[j] = old - h
            fm = f(*xs)
            flat[j] = old
            gf[j] = (fp - fm) / (2 * h)
        grads.append(g)
    return grads


def fd_jacobian(F, x, h_rel=1e-6):
    """Jacobian of the vector function F at x by central differences (columns)."""
    x = np.array(x, dtype=np.float64)
    y0 = np.asarray(F(x))
    J = np.zeros((y0.size, x.size))
    for j in range(x.size):
        h = h_rel * max(1.0, abs(x[j]))
        xp, xm = x.copy(), x.copy()
        xp[j] += h
        xm[j] -= h
        J[:, j] = (np.asarray(F(xp)) - np.asarray(F(xm))) / (2 * h)
    return J
