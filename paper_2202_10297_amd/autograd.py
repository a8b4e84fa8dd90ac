"""torch.autograd.Function wrappers: each operator's primal and VJP kernels as
one differentiable op (and, for map, reduce and the general-operator reduce
and scan, the JVP kernels for torch's forward-mode AD).

Forward saves only the inputs and the small auxiliary results the return
sweep needs (scan checkpoints, argmax indices, zero counts and non-zero
products, histogram winners, scatter's overwritten values, per-point LSE);
never a tape of intermediates.  Backward calls the library's VJP kernel.
"""
from __future__ import annotations

import torch

from . import ops


class LinRecScan(torch.autograd.Function):
    """(A, B) = inclusive scan of (a, b) under (a1,b1)(+)(a2,b2) = (a2 a1, a2 b1 + b2)."""

    @staticmethod
    def forward(ctx, a, b):
        a, b = a.contiguous(), b.contiguous()
        A, B, ck = ops.linrec_scan(a, b)
        ctx.save_for_backward(a, b, ck)
        return A, B

    @staticmethod
    def backward(ctx, gA, gB):
        a, b, ck = ctx.saved_tensors
        gA = torch.zeros_like(a) if gA is None else gA.contiguous()
        gB = torch.zeros_like(b) if gB is None else gB.contiguous()
        ab, bb = ops.linrec_scan_vjp(a, b, gA, gB, ckpt=ck)
        return ab, bb


class Reduce(torch.autograd.Function):
    """y = reduce(op) x for op in add, mul, min, max (Sec. 5.1.1 adjoints)."""

    @staticmethod
    def forward(ctx, x, op):
        x = x.contiguous()
        y, aux = ops.reduce(op, x)
        ctx.op = op
        ctx.aux_keys = tuple(aux)
        ctx.save_for_backward(x, *aux.values())
        ctx.save_for_forward(x, *aux.values())
        return y.reshape(())

    @staticmethod
    def backward(ctx, gy):
        x, *vals = ctx.saved_tensors
        aux = dict(zip(ctx.aux_keys, vals))
        xb = ops.reduce_vjp(ctx.op, x, aux, gy.reshape(1).contiguous())
        return xb, None

    @staticmethod
    def jvp(ctx, xd, _op):
        x, *vals = ctx.saved_tensors
        aux = dict(zip(ctx.aux_keys, vals))
        return ops.reduce_jvp(ctx.op, x, aux, xd.contiguous()).reshape(())


class ReduceGeneric(torch.autograd.Function):
    """y = x_0 (.) ... (.) x_{n-1} for a general operator (Sec. 5.1.1); the
    inputs are the K component tensors, the outputs K scalars.  Saved: the
    inputs and the per-tile checkpoint (32 bytes per tile of 1024-2048
    elements); the backward recomputes the prefix and suffix folds from it."""

    @staticmethod
    def forward(ctx, op, *xs):
        xs = [x.contiguous() for x in xs]
        ys, ck = ops.reduce_generic(op, xs, ckpt=True)
        ctx.op = op
        ctx.save_for_backward(ck, *xs)
        ctx.save_for_forward(ck, *xs)  # the same list, whichever sweep reads it
        return tuple(y.reshape(()) for y in ys)

    @staticmethod
    def jvp(ctx, _op, *xds):
        xs = ctx.saved_tensors[1:]
        xds = [torch.zeros_like(x) if t is None else t.contiguous() for t, x in zip(xds, xs)]
        _, yds = ops.reduce_generic_jvp(ctx.op, xs, xds)
        return tuple(y.reshape(()) for y in yds)

    @staticmethod
    def backward(ctx, *gys):
        ck, *xs = ctx.saved_tensors
        yb = [torch.zeros(1, dtype=xs[0].dtype, device=xs[0].device) if g is None else g.reshape(1).contiguous()
              for g in gys]
        return (None, *ops.reduce_generic_vjp(ctx.op, xs, yb, ckpt=ck))


class ScanGeneric(torch.autograd.Function):
    """Inclusive scan with a general operator (Sec. 5.2): K component tensors
    in, K out.  Saved: the inputs and the per-tile prefix checkpoint; the
    backward recomputes the primal per tile."""

    @staticmethod
    def forward(ctx, op, *xs):
        xs = [x.contiguous() for x in xs]
        ys, ck = ops.scan_generic(op, xs, ckpt=True)
        ctx.op = op
        ctx.save_for_backward(ck, *xs)
        ctx.save_for_forward(ck, *xs)  # the same list, whichever sweep reads it
        return tuple(ys)

    @staticmethod
    def jvp(ctx, _op, *xds):
        xs = ctx.saved_tensors[1:]
        xds = [torch.zeros_like(x) if t is None else t.contiguous() for t, x in zip(xds, xs)]
        _, yds = ops.scan_generic_jvp(ctx.op, xs, xds)
        return tuple(yds)

    @staticmethod
    def backward(ctx, *gys):
        ck, *xs = ctx.saved_tensors
        yb = [torch.zeros_like(x) if g is None else g.contiguous() for g, x in zip(gys, xs)]
        return (None, *ops.scan_generic_vjp(ctx.op, xs, yb, ckpt=ck))


class ReduceByIndex(torch.autograd.Function):
    """hs = reduce_by_index(op) over bins inds[i] of vs[i], m bins."""

    @staticmethod
    def forward(ctx, vs, inds, m, op):
        vs, inds = vs.contiguous(), inds.contiguous()
        hs, aux = ops.hist(op, inds, vs, m)
        ctx.op, ctx.m = op, m
        ctx.aux_keys = tuple(aux)
        ctx.save_for_backward(vs, inds, *aux.values())
        return hs

    @staticmethod
    def backward(ctx, ghs):
        vs, inds, *vals = ctx.saved_tensors
        aux = dict(zip(ctx.aux_keys, vals))
        vb = ops.hist_vjp(ctx.op, inds, vs if ctx.op == "mul" else None, ctx.m, aux, ghs.contiguous(),
                          n=vs.numel())
        return vb, None, None, None


class Scatter(torch.autograd.Function):
    """ys = scatter(xs, is, vs) out of place (xs is copied first, so autograd
    sees a pure function); is must hold no duplicates."""

    @staticmethod
    def forward(ctx, xs, is_, vs):
        ys = xs.contiguous().clone()
        ops.scatter_(ys, is_.contiguous(), vs.contiguous(), save=False)
        ctx.save_for_backward(is_)
        return ys

    @staticmethod
    def backward(ctx, gys):
        (is_,) = ctx.saved_tensors
        xb = gys.contiguous().clone()
        vb = ops.scatter_vjp_(xb, is_)
        return xb, None, vb


class Map(torch.autograd.Function):
    """y = f(x) elementwise, f in square, exp, log, sin, tanh."""

    @staticmethod
    def forward(ctx, x, fn):
        x = x.contiguous()
        ctx.fn = fn
        ctx.save_for_backward(x)
        ctx.save_for_forward(x)
        return ops.map_(fn, x)

    @staticmethod
    def backward(ctx, gy):
        (x,) = ctx.saved_tensors
        return ops.map_vjp(ctx.fn, x, gy.contiguous()), None

    @staticmethod
    def jvp(ctx, xd, _fn):
        (x,) = ctx.saved_tensors
        return ops.map_jvp(ctx.fn, x, xd.contiguous())


class GMMLogLik(torch.autograd.Function):
    """Gaussian-mixture log-likelihood (FP32 parameters, FP64 result)."""

    @staticmethod
    def forward(ctx, X, alpha, mu, q, l):
        args = [t.contiguous() for t in (X, alpha, mu, q, l)]
        ll, lse = ops.gmm_objective(*args)
        ctx.save_for_backward(*args, lse)
        return ll.reshape(())

    @staticmethod
    def backward(ctx, g):
        X, alpha, mu, q, l, lse = ctx.saved_tensors
        ab, mb, qb, lb = ops.gmm_vjp(X, alpha, mu, q, l, lse=lse, ell_bar=float(g))
        return None, ab, mb, qb, lb


class ScanGenericBatched(torch.autograd.Function):
    """Regular segmented scan (Sec. 5.2's vectorised-operator rule): every row
    of the K [B, L] component tensors scanned on its own.  Saved: the inputs
    and the per-tile prefix checkpoint of every row."""

    @staticmethod
    def forward(ctx, op, *xs):
        xs = [x.contiguous() for x in xs]
        ys, ck = ops.scan_generic_batched(op, xs, ckpt=True)
        ctx.op = op
        ctx.save_for_backward(ck, *xs)
        return tuple(ys)

    @staticmethod
    def backward(ctx, *gys):
        ck, *xs = ctx.saved_tensors
        yb = [torch.zeros_like(x) if g is None else g.contiguous() for g, x in zip(gys, xs)]
        return (None, *ops.scan_generic_batched_vjp(ctx.op, xs, yb, ckpt=ck))


class GatherMap(torch.autograd.Function):
    """ys[i] = f(as_[is_[i]], vs[i]) (Sec. 5.4, a map reading a free array);
    the backward accumulates the reads' adjoints into as_ (no grad for is_)."""

    @staticmethod
    def forward(ctx, as_, is_, vs, op):
        as_, is_ = as_.contiguous(), is_.contiguous()
        vs = vs.contiguous() if vs is not None else None
        ctx.op = op
        ctx.save_for_backward(as_, is_, vs)
        return ops.gather_map(op, as_, is_, vs)

    @staticmethod
    def backward(ctx, gys):
        as_, is_, vs = ctx.saved_tensors
        ab, vb = ops.gather_map_vjp(ctx.op, as_, is_, vs, gys.contiguous())
        return ab, None, vb, None


class KMeansObjective(torch.autograd.Function):
    """f(C) = sum_i min_k |x_i - c_k|^2 (Sec. 7.4) for fixed points X.  Saved:
    the assignments (the search is not repeated in the backward).  The jvp of
    the VJP (Hessian-vector product) is ops.kmeans_vjp with C_dot."""

    @staticmethod
    def forward(ctx, X, C):
        X, C = X.contiguous(), C.contiguous()
        f, assign = ops.kmeans_objective(X, C)
        ctx.save_for_backward(X, C, assign)
        return f[0]

    @staticmethod
    def backward(ctx, gf):
        X, C, assign = ctx.saved_tensors
        cb, _ = ops.kmeans_vjp(X, C, assign, f_bar=float(gf))
        return None, cb


class SparseKMeansObjective(torch.autograd.Function):
    """f(C) = sum_i min_k |x_i - c_k|^2 (Sec. 7.5) for fixed CSR points.
    Saved: the assignments (the search is not repeated in the backward)."""

    @staticmethod
    def forward(ctx, rowptr, col, val, D, C):
        C = C.contiguous()
        f, assign = ops.sparse_kmeans_objective(rowptr, col, val, D, C)
        ctx.D = D
        ctx.save_for_backward(rowptr, col, val, C, assign)
        return f[0]

    @staticmethod
    def backward(ctx, gf):
        rowptr, col, val, C, assign = ctx.saved_tensors
        cb, _ = ops.sparse_kmeans_vjp(rowptr, col, val, ctx.D, C, assign, f_bar=float(gf))
        return None, None, None, None, cb


class ReduceByIndexLogAddExp(torch.autograd.Function):
    """hs[b] = log sum over bin b of e^(x_i) (reduce_by_index with the
    log-add-exp operator).  Saved: x, the indices and hs."""

    @staticmethod
    def forward(ctx, x, inds, m):
        x, inds = x.contiguous(), inds.contiguous()
        hs = ops.hist_lae(inds, x, m)
        ctx.save_for_backward(x, inds, hs)
        return hs

    @staticmethod
    def backward(ctx, ghs):
        x, inds, hs = ctx.saved_tensors
        return ops.hist_lae_vjp(inds, x, hs, ghs.contiguous()), None, None


def linrec_scan(a, b):
    return LinRecScan.apply(a, b)


def reduce(x, op="add"):
    return Reduce.apply(x, op)


def reduce_generic(op, *xs):
    return ReduceGeneric.apply(op, *xs)


def scan_generic(op, *xs):
    return ScanGeneric.apply(op, *xs)


def reduce_by_index(vs, inds, m, op="add"):
    return ReduceByIndex.apply(vs, inds, m, op)


def scatter(xs, is_, vs):
    return Scatter.apply(xs, is_, vs)


def map(x, fn):  # noqa: A001 - the operator's name
    return Map.apply(x, fn)


def gmm_loglik(X, alpha, mu, q, l):
    return GMMLogLik.apply(X, alpha, mu, q, l)


def scan_generic_batched(op, *xs):
    return ScanGenericBatched.apply(op, *xs)


def gather_map(as_, is_, vs=None, op="mul"):
    return GatherMap.apply(as_, is_, vs, op)


def kmeans_objective(X, C):
    return KMeansObjective.apply(X, C)


def sparse_kmeans_objective(rowptr, col, val, D, C):
    return SparseKMeansObjective.apply(rowptr, col, val, D, C)


def reduce_by_index_logaddexp(x, inds, m):
    return ReduceByIndexLogAddExp.apply(x, inds, m)
