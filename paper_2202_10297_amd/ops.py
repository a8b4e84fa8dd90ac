"""Torch-tensor front end of libpvjp.so.

Torch provides device memory and the current HIP stream; every step of every
operator runs in the library's kernels (called through ``capi``).  Outputs and
workspaces are allocated here with torch, then raw pointers are passed on.
"""
from __future__ import annotations

import torch

from . import capi

_DT = {torch.float32: capi.F32, torch.float64: capi.F64}
_OPS = {"add": capi.ADD, "mul": capi.MUL, "min": capi.MIN, "max": capi.MAX}
_GOPS = {"logaddexp": capi.GOP_LOGADDEXP, "linrec": capi.GOP_LINREC, "mat2": capi.GOP_MAT2}
_FNS = {"square": capi.FN_SQUARE, "exp": capi.FN_EXP, "log": capi.FN_LOG, "sin": capi.FN_SIN,
        "tanh": capi.FN_TANH}


def _dt(t: torch.Tensor) -> int:
    try:
        return _DT[t.dtype]
    except KeyError:
        raise TypeError(f"unsupported dtype {t.dtype}; expected float32 or float64") from None


def _op(op) -> int:
    return _OPS[op] if isinstance(op, str) else int(op)


def _fn(fn) -> int:
    return _FNS[fn] if isinstance(fn, str) else int(fn)


def _ptr(t):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("pvjp operates on device tensors only")
    if not t.is_contiguous():
        raise ValueError("pvjp expects contiguous tensors")
    return t.data_ptr() or None


def _stream(device=None):
    return torch.cuda.current_stream(device).cuda_stream


class Workspaces:
    """Zero-initialised device workspaces, cached per (device, stream, key).

    The library leaves a workspace ready for reuse after every call; calls on
    one stream are ordered, so one workspace per stream and purpose is safe."""

    def __init__(self):
        self._bufs = {}

    def get(self, key, nbytes: int, device) -> torch.Tensor:
        dev = torch.device(device)
        k = (dev.index, _stream(dev), key)
        buf = self._bufs.get(k)
        if buf is None or buf.numel() < nbytes:
            buf = torch.zeros(max(nbytes, 256) + 256, dtype=torch.uint8, device=dev)
            off = (-buf.data_ptr()) % 256
            buf = buf[off:off + max(nbytes, 256)]
            self._bufs[k] = buf
        return buf

    def clear(self):
        self._bufs.clear()


WS = Workspaces()


# ------------------------------------------------------------ checked mode
class _Checked:
    """Checked mode.  When on, the operators below first run the library's
    diagnostic kernels on their inputs: indices outside the bin or target
    range, repeated scatter targets, NaN and infinite values are added to a
    per-device int64 counter block (read with ``diag``).  After a lookback
    scan, the workspace's error word is read back (a stream synchronisation)
    and a recorded error raises ``capi.PvjpError``.  Off by default: the
    checks cost a pass over the inputs and, for the scans, a host wait."""

    def __init__(self):
        self.on = False
        self.counters = {}

    def block(self, device) -> torch.Tensor:
        dev = torch.device(device)
        c = self.counters.get(dev.index)
        if c is None:
            c = self.counters[dev.index] = torch.zeros(capi.DIAG_N, dtype=torch.int64, device=dev)
        return c


CHECKED = _Checked()


def set_checked(on: bool = True) -> None:
    CHECKED.on = bool(on)


def diag(device=None, reset: bool = False) -> dict:
    """Counts collected in checked mode on `device` (default: the current
    one): {"oob", "dup", "nan", "inf"}; reset=True clears them."""
    dev = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
    c = CHECKED.block(dev)
    v = c.cpu().tolist()
    if reset:
        c.zero_()
    return {"oob": v[capi.DIAG_OOB], "dup": v[capi.DIAG_DUP], "nan": v[capi.DIAG_NAN], "inf": v[capi.DIAG_INF]}


def _check_indices(inds, m):
    if CHECKED.on and inds.numel():
        capi.call("pvjp_diag_indices", _ptr(inds), inds.numel(), int(m), _ptr(CHECKED.block(inds.device)),
                  _stream(inds.device))


def _check_values(*xs):
    if not CHECKED.on:
        return
    for x in xs:
        if x is not None and x.numel() and x.dtype in _DT:
            capi.call("pvjp_diag_nonfinite", _dt(x), _ptr(x), x.numel(), _ptr(CHECKED.block(x.device)),
                      _stream(x.device))


def _check_targets(is_, n):
    if CHECKED.on and is_.numel():
        nb = capi.lib().pvjp_diag_scatter_ws_bytes(int(n))
        ws = WS.get("diag_scatter", nb, is_.device)
        capi.call("pvjp_diag_scatter", _ptr(is_), is_.numel(), int(n), _ptr(CHECKED.block(is_.device)), _ptr(ws),
                  ws.numel(), _stream(is_.device))


def check_workspace(ws) -> None:
    """Raises capi.PvjpError if a lookback launch recorded an error in `ws`
    (and clears it); synchronises the stream."""
    capi.call("pvjp_ws_check", _ptr(ws), 1, _stream(ws.device))


def _after_lookback(ws):
    # not while a graph is being captured: the check waits on the stream
    if CHECKED.on and not torch.cuda.is_current_stream_capturing():
        check_workspace(ws)


# ------------------------------------------------------------ linrec scan
def linrec_scan(a: torch.Tensor, b: torch.Tensor, ckpt: bool = True):
    """Inclusive scan of (a, b) under (a1,b1)(+)(a2,b2) = (a2 a1, a2 b1 + b2).
    Returns (A, B, ckpt or None)."""
    n = a.numel()
    dt = _dt(a)
    A, B = torch.empty_like(a), torch.empty_like(b)
    ck = torch.empty(2 * capi.lib().pvjp_linrec_ckpt_len(n), dtype=a.dtype, device=a.device) if ckpt else None
    nb = capi.lib().pvjp_linrec_scan_ws_bytes(dt, n)
    ws = WS.get("linrec_fwd", nb, a.device)
    _check_values(a, b)
    capi.call("pvjp_linrec_scan", dt, _ptr(a), _ptr(b), n, _ptr(A), _ptr(B), _ptr(ck), _ptr(ws), ws.numel(),
              _stream(a.device))
    _after_lookback(ws)
    return A, B, ck


def linrec_scan_vjp(a, b, yA_bar, yB_bar, ckpt=None, a_bar=None, b_bar=None, accumulate=False):
    n = a.numel()
    dt = _dt(a)
    if a_bar is None:
        a_bar = torch.zeros_like(a) if accumulate else torch.empty_like(a)
    if b_bar is None:
        b_bar = torch.zeros_like(b) if accumulate else torch.empty_like(b)
    nb = capi.lib().pvjp_linrec_scan_vjp_ws_bytes(dt, n)
    ws = WS.get("linrec_vjp", nb, a.device)
    _check_values(a, b, yA_bar, yB_bar)
    capi.call("pvjp_linrec_scan_vjp", dt, _ptr(a), _ptr(b), _ptr(yA_bar), _ptr(yB_bar), n, _ptr(ckpt),
              _ptr(a_bar), _ptr(b_bar), int(accumulate), _ptr(ws), ws.numel(), _stream(a.device))
    _after_lookback(ws)
    return a_bar, b_bar


# ----------------------------------------------------------------- reduce
def reduce(op, x: torch.Tensor):
    """Returns (y, aux) with aux = {"arg"} for min/max, {"p", "z"} for mul."""
    o, dt, n = _op(op), _dt(x), x.numel()
    dev = x.device
    y = torch.empty(1, dtype=x.dtype, device=dev)
    aux = {}
    arg = p = z = None
    if o in (capi.MIN, capi.MAX):
        arg = aux["arg"] = torch.empty(1, dtype=torch.int64, device=dev)
    if o == capi.MUL:
        p = aux["p"] = torch.empty(1, dtype=x.dtype, device=dev)
        z = aux["z"] = torch.empty(1, dtype=torch.int64, device=dev)
    nb = capi.lib().pvjp_reduce_ws_bytes(o, dt, n)
    ws = WS.get("reduce", nb, dev)
    capi.call("pvjp_reduce", o, dt, _ptr(x), n, _ptr(y), _ptr(arg), _ptr(p), _ptr(z), _ptr(ws), ws.numel(),
              _stream(dev))
    return y, aux


def reduce_vjp(op, x, aux, y_bar, x_bar=None, accumulate=False):
    o, dt, n = _op(op), _dt(x), x.numel()
    if x_bar is None:
        x_bar = torch.zeros_like(x) if accumulate else torch.empty_like(x)
    capi.call("pvjp_reduce_vjp", o, dt, _ptr(x), n, _ptr(aux.get("arg")), _ptr(aux.get("p")), _ptr(aux.get("z")),
              _ptr(y_bar), _ptr(x_bar), int(accumulate), _stream(x.device))
    return x_bar


# ------------------------------------------------ reduce, general operator
def _gop(op) -> int:
    return _GOPS[op] if isinstance(op, str) else int(op)


def _components(op, xs):
    K = capi.lib().pvjp_gop_components(_gop(op))
    xs = list(xs)
    if K == 0 or len(xs) != K:
        raise ValueError(f"operator {op} takes {K} component tensors, got {len(xs)}")
    n = xs[0].numel()
    if any(x.numel() != n or x.dtype != xs[0].dtype or x.device != xs[0].device for x in xs):
        raise ValueError("component tensors differ in length, dtype or device")
    return xs, n, K


def reduce_generic(op, xs, ckpt: bool = False):
    """y = xs_0 (.) ... (.) xs_{n-1} for an operator of Sec. 5.1.1's general
    rule; xs is the list of K component tensors.  Returns (ys, ckpt): K
    one-element tensors and, if asked for, the per-tile checkpoint (the tile
    folds, a uint8 tensor) that lets the VJP read x once."""
    xs, n, K = _components(op, xs)
    dt, dev = _dt(xs[0]), xs[0].device
    ys = [torch.empty(1, dtype=xs[0].dtype, device=dev) for _ in range(K)]
    ck = None
    if ckpt:
        ck = torch.empty(max(capi.lib().pvjp_reduce_generic_ckpt_bytes(_gop(op), dt, n), 16), dtype=torch.uint8,
                         device=dev)
    nb = capi.lib().pvjp_reduce_generic_ws_bytes(_gop(op), dt, n)
    ws = WS.get("reduce_generic", nb, dev)
    capi.call("pvjp_reduce_generic", _gop(op), dt, capi.ptr_array([_ptr(x) for x in xs]), n,
              capi.ptr_array([_ptr(y) for y in ys]), _ptr(ck), _ptr(ws), ws.numel(), _stream(dev))
    return ys, ck


def reduce_generic_vjp(op, xs, y_bar, x_bar=None, accumulate=False, ckpt=None):
    """x_bar (+)= the adjoint of every element (list of K tensors); y_bar is
    a list of K one-element device tensors; ckpt is the checkpoint from
    reduce_generic on the same xs (or None: the tile folds are recomputed)."""
    xs, n, K = _components(op, xs)
    dt, dev = _dt(xs[0]), xs[0].device
    if x_bar is None:
        x_bar = [torch.zeros_like(x) if accumulate else torch.empty_like(x) for x in xs]
    if len(y_bar) != K or len(x_bar) != K:
        raise ValueError(f"operator {op} takes {K} components")
    nb = capi.lib().pvjp_reduce_generic_ws_bytes(_gop(op), dt, n)
    ws = WS.get("reduce_generic", nb, dev)
    capi.call("pvjp_reduce_generic_vjp", _gop(op), dt, capi.ptr_array([_ptr(x) for x in xs]), n, _ptr(ckpt),
              capi.ptr_array([_ptr(y) for y in y_bar]), capi.ptr_array([_ptr(x) for x in x_bar]),
              int(accumulate), _ptr(ws), ws.numel(), _stream(dev))
    return x_bar


def scan_generic(op, xs, ckpt: bool = True):
    """Inclusive scan y_i = xs_0 (.) ... (.) xs_i with a general operator
    (Sec. 5.2); xs is the list of K component tensors.  Returns (ys, ckpt):
    K tensors and the per-tile checkpoint (uint8 tensor) if asked for."""
    xs, n, K = _components(op, xs)
    dt, dev = _dt(xs[0]), xs[0].device
    ys = [torch.empty_like(x) for x in xs]
    ck = None
    if ckpt:
        ck = torch.empty(max(capi.lib().pvjp_scan_generic_ckpt_bytes(_gop(op), dt, n), 16), dtype=torch.uint8,
                         device=dev)
    nb = capi.lib().pvjp_scan_generic_ws_bytes(_gop(op), dt, n)
    ws = WS.get("scan_generic", nb, dev)
    capi.call("pvjp_scan_generic", _gop(op), dt, capi.ptr_array([_ptr(x) for x in xs]), n,
              capi.ptr_array([_ptr(y) for y in ys]), _ptr(ck), _ptr(ws), ws.numel(), _stream(dev))
    return ys, ck


def scan_generic_vjp(op, xs, y_bar, x_bar=None, accumulate=False, ckpt=None):
    """x_bar (+)= the adjoints of the inputs given the adjoints y_bar of every
    output (lists of K tensors); ckpt from scan_generic on the same xs, or
    None (the tile prefixes are recomputed)."""
    xs, n, K = _components(op, xs)
    dt, dev = _dt(xs[0]), xs[0].device
    if x_bar is None:
        x_bar = [torch.zeros_like(x) if accumulate else torch.empty_like(x) for x in xs]
    if len(y_bar) != K or len(x_bar) != K:
        raise ValueError(f"operator {op} takes {K} components")
    nb = capi.lib().pvjp_scan_generic_ws_bytes(_gop(op), dt, n)
    ws = WS.get("scan_generic", nb, dev)
    capi.call("pvjp_scan_generic_vjp", _gop(op), dt, capi.ptr_array([_ptr(x) for x in xs]), n, _ptr(ckpt),
              capi.ptr_array([_ptr(y) for y in y_bar]), capi.ptr_array([_ptr(x) for x in x_bar]),
              int(accumulate), _ptr(ws), ws.numel(), _stream(dev))
    return x_bar


# ---------------------------------------------------------- reduce_by_index
def hist(op, inds: torch.Tensor, vs: torch.Tensor, m: int, counts: bool = False):
    """Returns (hs, aux): aux has "winner" (min/max), "p" and "z" (mul),
    "count" (if counts)."""
    o, dt, n = _op(op), _dt(vs), vs.numel()
    dev = vs.device
    if inds.dtype != torch.int32:
        raise TypeError("inds must be int32")
    hs = torch.empty(m, dtype=vs.dtype, device=dev)
    aux = {}
    winner = p = z = count = None
    if o in (capi.MIN, capi.MAX):
        winner = aux["winner"] = torch.empty(m, dtype=torch.int32, device=dev)
    if o == capi.MUL:
        p = aux["p"] = torch.empty(m, dtype=vs.dtype, device=dev)
        z = aux["z"] = torch.empty(m, dtype=torch.int32, device=dev)
    if counts:
        count = aux["count"] = torch.empty(m, dtype=torch.int32, device=dev)
    _check_indices(inds, m)
    _check_values(vs)
    nb = capi.lib().pvjp_hist_ws_bytes(o, dt, n, m)
    ws = WS.get("hist", nb, dev)
    capi.call("pvjp_hist", o, dt, _ptr(inds), _ptr(vs), n, m, _ptr(hs), _ptr(winner), _ptr(p), _ptr(z),
              _ptr(count), _ptr(ws), ws.numel(), _stream(dev))
    return hs, aux


def hist_vjp(op, inds, vs, m, aux, hs_bar, vs_bar=None, accumulate=False, n=None):
    o = _op(op)
    dt = _dt(hs_bar)
    n = inds.numel() if n is None else n
    if vs_bar is None:
        shape = (n,)
        vs_bar = (torch.zeros if accumulate else torch.empty)(shape, dtype=hs_bar.dtype, device=hs_bar.device)
    if o == capi.ADD or o == capi.MUL:
        _check_indices(inds, m)
    _check_values(hs_bar)
    capi.call("pvjp_hist_vjp", o, dt, _ptr(inds), _ptr(vs), n, m, _ptr(aux.get("winner")), _ptr(aux.get("p")),
              _ptr(aux.get("z")), _ptr(hs_bar), _ptr(vs_bar), int(accumulate), _stream(hs_bar.device))
    return vs_bar


# ----------------------------------------------------------------- scatter
def scatter_(xs: torch.Tensor, is_: torch.Tensor, vs: torch.Tensor, save: bool = True):
    """In place on xs; returns xs_saved (or None)."""
    dt = _dt(xs)
    saved = torch.empty(is_.numel(), dtype=xs.dtype, device=xs.device) if save else None
    _check_targets(is_, xs.numel())
    _check_values(vs)
    capi.call("pvjp_scatter", dt, _ptr(xs), xs.numel(), _ptr(is_), _ptr(vs), is_.numel(), _ptr(saved),
              _stream(xs.device))
    return saved


def scatter_vjp_(ys_bar, is_, vs_bar=None, accumulate=False, ys=None, xs_saved=None):
    """In place on ys_bar (which becomes xs_bar); optionally restores ys."""
    dt = _dt(ys_bar)
    if vs_bar is None:
        vs_bar = (torch.zeros if accumulate else torch.empty)(is_.numel(), dtype=ys_bar.dtype, device=ys_bar.device)
    _check_targets(is_, ys_bar.numel())
    _check_values(ys_bar)
    capi.call("pvjp_scatter_vjp", dt, _ptr(ys_bar), ys_bar.numel(), _ptr(is_), is_.numel(), _ptr(vs_bar),
              int(accumulate), _ptr(ys), _ptr(xs_saved), _stream(ys_bar.device))
    return vs_bar


def scatter_plan_bytes(dtype, n: int, m: int) -> int:
    return capi.lib().pvjp_scatter_plan_bytes(_DT[dtype], int(n), int(m))


def scatter_planned_(xs: torch.Tensor, is_: torch.Tensor, vs: torch.Tensor, plan=None):
    """In place on xs; returns the plan (the forward sweep's target-ordered
    auxiliary result, holding the overwritten values) for
    scatter_planned_vjp_."""
    if is_.dtype != torch.int32:
        raise TypeError("is_ must be int32")
    if vs.dtype != xs.dtype or vs.numel() != is_.numel():
        raise ValueError("vs must have the dtype of xs and one value per target")
    n, m = xs.numel(), is_.numel()
    nb = scatter_plan_bytes(xs.dtype, n, m)
    if nb == 0:
        raise ValueError(f"scatter plan: n = {n}, m = {m} out of range")
    if plan is None or plan.numel() < nb:
        buf = torch.empty(nb + 256, dtype=torch.uint8, device=xs.device)
        off = (-buf.data_ptr()) % 256
        plan = buf[off:off + nb]
    _check_targets(is_, n)
    _check_values(vs)
    capi.call("pvjp_scatter_planned", _dt(xs), _ptr(xs), n, _ptr(is_), _ptr(vs), m, _ptr(plan), plan.numel(),
              _stream(xs.device))
    return plan


def scatter_planned_vjp_(ys_bar, m: int, plan, vs_bar=None, accumulate=False, ys=None):
    """In place on ys_bar (which becomes xs_bar); restores ys if given."""
    n = ys_bar.numel()
    if vs_bar is None:
        vs_bar = (torch.zeros if accumulate else torch.empty)(m, dtype=ys_bar.dtype, device=ys_bar.device)
    if ys is not None and (ys.dtype != ys_bar.dtype or ys.numel() != n):
        raise ValueError("ys must have the dtype and size of ys_bar")
    capi.call("pvjp_scatter_planned_vjp", _dt(ys_bar), _ptr(ys_bar), n, int(m), _ptr(vs_bar), int(accumulate),
              _ptr(ys), _ptr(plan), plan.numel(), _stream(ys_bar.device))
    return vs_bar


# --------------------------------------------------------------------- map
def map_(fn, x):
    y = torch.empty_like(x)
    capi.call("pvjp_map", _fn(fn), _dt(x), _ptr(x), x.numel(), _ptr(y), _stream(x.device))
    return y


def map_vjp(fn, x, y_bar, x_bar=None, accumulate=False):
    if x_bar is None:
        x_bar = torch.zeros_like(x) if accumulate else torch.empty_like(x)
    capi.call("pvjp_map_vjp", _fn(fn), _dt(x), _ptr(x), _ptr(y_bar), x.numel(), _ptr(x_bar), int(accumulate),
              _stream(x.device))
    return x_bar


def fig1(x0, x1):
    y0, y1 = torch.empty_like(x0), torch.empty_like(x0)
    capi.call("pvjp_fig1", _dt(x0), _ptr(x0), _ptr(x1), x0.numel(), _ptr(y0), _ptr(y1), _stream(x0.device))
    return y0, y1


def fig1_vjp(x0, x1, y0_bar, y1_bar, accumulate=False, x0_bar=None, x1_bar=None):
    if x0_bar is None:
        x0_bar = torch.zeros_like(x0) if accumulate else torch.empty_like(x0)
    if x1_bar is None:
        x1_bar = torch.zeros_like(x1) if accumulate else torch.empty_like(x1)
    capi.call("pvjp_fig1_vjp", _dt(x0), _ptr(x0), _ptr(x1), _ptr(y0_bar), _ptr(y1_bar), x0.numel(), _ptr(x0_bar),
              _ptr(x1_bar), int(accumulate), _stream(x0.device))
    return x0_bar, x1_bar


# --------------------------------------------------------------------- GMM
def gmm_objective(X, alpha, mu, q, l, want_lse=True, s_out=None):
    """Returns (loglik [1] float64 device tensor, lse [N] float64 or None).
    s_out (float64 [K, N], optional) receives every s_ik."""
    N, D = X.shape
    K = alpha.numel()
    dev = X.device
    ll = torch.empty(1, dtype=torch.float64, device=dev)
    lse = torch.empty(N, dtype=torch.float64, device=dev) if want_lse else None
    nb = capi.lib().pvjp_gmm_ws_bytes(N, D, K)
    ws = WS.get("gmm", nb, dev)
    capi.call("pvjp_gmm_objective", _ptr(X), N, D, K, _ptr(alpha), _ptr(mu), _ptr(q), _ptr(l), _ptr(ll), _ptr(lse),
              _ptr(s_out), _ptr(ws), ws.numel(), _stream(dev))
    return ll, lse


def gmm_objective_ckpt(X, alpha, mu, q, l):
    """The objective with both checkpoints: (loglik, lse [N], s [K, N])."""
    N = X.shape[0]
    s = torch.empty((alpha.numel(), N), dtype=torch.float64, device=X.device)
    ll, lse = gmm_objective(X, alpha, mu, q, l, want_lse=True, s_out=s)
    return ll, lse, s


def gmm_vjp(X, alpha, mu, q, l, lse=None, ell_bar=1.0, out=None, accumulate=False, s=None):
    """Returns (alpha_bar, mu_bar, q_bar, l_bar) (float32, device).  With the
    s checkpoint of gmm_objective_ckpt (and its lse) the contraction is
    S_k = sum w y y^T instead of recomputing z."""
    N, D = X.shape
    K = alpha.numel()
    dev = X.device
    if out is None:
        mk = torch.zeros_like if accumulate else torch.empty_like
        out = (mk(alpha), mk(mu), mk(q), mk(l))
    ab, mb, qb, lb = out
    nb = capi.lib().pvjp_gmm_ws_bytes(N, D, K)
    ws = WS.get("gmm", nb, dev)
    capi.call("pvjp_gmm_vjp", _ptr(X), N, D, K, _ptr(alpha), _ptr(mu), _ptr(q), _ptr(l), float(ell_bar), _ptr(lse),
              _ptr(s), _ptr(ab), _ptr(mb), _ptr(qb), _ptr(lb), int(accumulate), _ptr(ws), ws.numel(), _stream(dev))
    return ab, mb, qb, lb


# ------------------------------------------------------------ forward mode
def map_jvp(fn, x, x_dot):
    """y_dot = f'(x) x_dot."""
    y_dot = torch.empty_like(x)
    capi.call("pvjp_map_jvp", _fn(fn), _dt(x), _ptr(x), _ptr(x_dot), x.numel(), _ptr(y_dot), _stream(x.device))
    return y_dot


def reduce_jvp(op, x, aux, x_dot):
    """Tangent of reduce(op) x (aux from reduce() on the same x)."""
    o, dt, n = _op(op), _dt(x), x.numel()
    yd = torch.empty(1, dtype=x.dtype, device=x.device)
    nb = capi.lib().pvjp_reduce_ws_bytes(o, dt, n)
    ws = WS.get("reduce", nb, x.device)
    capi.call("pvjp_reduce_jvp", o, dt, _ptr(x), _ptr(x_dot), n, _ptr(aux.get("arg")), _ptr(aux.get("p")),
              _ptr(aux.get("z")), _ptr(yd), _ptr(ws), ws.numel(), _stream(x.device))
    return yd


def hist_jvp(op, inds, vs_dot, m, aux=None):
    """Tangent of reduce_by_index(op) (aux with "winner" for min/max)."""
    o, dt, n = _op(op), _dt(vs_dot), vs_dot.numel()
    hd = torch.empty(m, dtype=vs_dot.dtype, device=vs_dot.device)
    nb = capi.lib().pvjp_hist_jvp_ws_bytes(o, dt, n, m)
    ws = WS.get("hist", nb, vs_dot.device) if nb else None
    capi.call("pvjp_hist_jvp", o, dt, _ptr(inds), _ptr(vs_dot), n, m, _ptr((aux or {}).get("winner")), _ptr(hd),
              _ptr(ws), ws.numel() if ws is not None else 0, _stream(vs_dot.device))
    return hd


def scatter_jvp_(ys_dot, is_, vs_dot):
    """In place on ys_dot (x_dot on entry)."""
    capi.call("pvjp_scatter_jvp", _dt(ys_dot), _ptr(ys_dot), ys_dot.numel(), _ptr(is_), _ptr(vs_dot), is_.numel(),
              _stream(ys_dot.device))
    return ys_dot


def reduce_generic_jvp(op, xs, xs_dot):
    """(ys, ys_dot): K one-element tensors each."""
    xs, n, K = _components(op, xs)
    xd, _, _ = _components(op, xs_dot)
    dt, dev = _dt(xs[0]), xs[0].device
    ys = [torch.empty(1, dtype=xs[0].dtype, device=dev) for _ in range(K)]
    yds = [torch.empty(1, dtype=xs[0].dtype, device=dev) for _ in range(K)]
    nb = capi.lib().pvjp_reduce_generic_jvp_ws_bytes(_gop(op), dt, n)
    ws = WS.get("reduce_generic_jvp", nb, dev)
    capi.call("pvjp_reduce_generic_jvp", _gop(op), dt, capi.ptr_array([_ptr(x) for x in xs]),
              capi.ptr_array([_ptr(x) for x in xd]), n, capi.ptr_array([_ptr(y) for y in ys]),
              capi.ptr_array([_ptr(y) for y in yds]), _ptr(ws), ws.numel(), _stream(dev))
    return ys, yds


def scan_generic_jvp(op, xs, xs_dot):
    """(ys, ys_dot): K tensors of n each."""
    xs, n, K = _components(op, xs)
    xd, _, _ = _components(op, xs_dot)
    dt, dev = _dt(xs[0]), xs[0].device
    ys = [torch.empty_like(x) for x in xs]
    yds = [torch.empty_like(x) for x in xs]
    nb = capi.lib().pvjp_scan_generic_jvp_ws_bytes(_gop(op), dt, n)
    ws = WS.get("scan_generic_jvp", nb, dev)
    capi.call("pvjp_scan_generic_jvp", _gop(op), dt, capi.ptr_array([_ptr(x) for x in xs]),
              capi.ptr_array([_ptr(x) for x in xd]), n, capi.ptr_array([_ptr(y) for y in ys]),
              capi.ptr_array([_ptr(y) for y in yds]), _ptr(ws), ws.numel(), _stream(dev))
    return ys, yds


# ------------------------------------------------------------------ k-means
def kmeans_objective(X, C):
    """(f [1] float64, assign [N] int32) for f = sum_i min_k |x_i - c_k|^2."""
    N, D = X.shape
    K = C.shape[0]
    dev = X.device
    f = torch.empty(1, dtype=torch.float64, device=dev)
    a = torch.empty(N, dtype=torch.int32, device=dev)
    nb = capi.lib().pvjp_kmeans_ws_bytes(N, D, K)
    ws = WS.get("kmeans", nb, dev)
    capi.call("pvjp_kmeans_objective", _ptr(X), N, D, _ptr(C), K, _ptr(a), _ptr(f), _ptr(ws), ws.numel(),
              _stream(dev))
    return f, a


def kmeans_vjp(X, C, assign, f_bar=1.0, C_dot=None, out=None, accumulate=False):
    """C_bar, and with C_dot also the jvp of the VJP (Hessian-vector
    product): returns (C_bar, hvp or None)."""
    N, D = X.shape
    K = C.shape[0]
    dev = X.device
    mk = torch.zeros_like if accumulate else torch.empty_like
    cb, hv = out if out is not None else (mk(C), mk(C) if C_dot is not None else None)
    nb = capi.lib().pvjp_kmeans_ws_bytes(N, D, K)
    ws = WS.get("kmeans", nb, dev)
    capi.call("pvjp_kmeans_vjp", _ptr(X), N, D, _ptr(C), K, _ptr(assign), float(f_bar), _ptr(cb), _ptr(C_dot),
              _ptr(hv), int(accumulate), _ptr(ws), ws.numel(), _stream(dev))
    return cb, hv


def gather_map(op, as_, is_, vs=None, out=None):
    """ys[i] = f(as_[is_[i]], vs[i]) (a map reading the free array as_):
    op "gather" (f = a), "mul" (a v) or "sqdiff" ((a - v)^2)."""
    o = capi.GMAP[op]
    if is_.dtype != torch.int32:
        raise TypeError("is_ must be int32")
    m = is_.numel()
    ys = out if out is not None else torch.empty(m, dtype=as_.dtype, device=as_.device)
    _check_indices(is_, as_.numel())
    _check_values(as_, vs)
    capi.call("pvjp_gather_map", o, _dt(as_), _ptr(as_), as_.numel(), _ptr(is_), _ptr(vs), m, _ptr(ys),
              _stream(as_.device))
    return ys


def gather_map_vjp(op, as_, is_, vs, ys_bar, as_bar=None, vs_bar=None, accumulate=False):
    """(as_bar, vs_bar or None): each read's partial accumulated into as_bar."""
    o = capi.GMAP[op]
    n, m = as_.numel(), is_.numel()
    dev = as_.device
    mk = torch.zeros if accumulate else torch.empty
    ab = as_bar if as_bar is not None else mk(n, dtype=as_.dtype, device=dev)
    vb = vs_bar if (vs_bar is not None or o == 0) else mk(m, dtype=as_.dtype, device=dev)
    _check_indices(is_, n)
    _check_values(ys_bar)
    nb = capi.lib().pvjp_gather_map_ws_bytes(_dt(as_), n, m)
    ws = WS.get("gather_map", nb, dev)
    capi.call("pvjp_gather_map_vjp", o, _dt(as_), _ptr(as_), n, _ptr(is_), _ptr(vs), m, _ptr(ys_bar), _ptr(ab),
              _ptr(vb), int(accumulate), _ptr(ws), ws.numel(), _stream(dev))
    return ab, vb


def _rows(op, xs):
    xs, _, K = _components(op, xs)
    if xs[0].dim() != 2:
        raise ValueError("batched scans take [B, L] component tensors")
    B, L = xs[0].shape
    if any(tuple(x.shape) != (B, L) for x in xs):
        raise ValueError("component tensors differ in shape")
    return xs, B, L, K


def scan_generic_batched(op, xs, ckpt: bool = True):
    """Each row of the [B, L] component tensors scanned independently with a
    general operator (the regular segmented scan that a vectorised operator
    becomes).  Returns (ys, ckpt) like scan_generic."""
    xs, B, L, K = _rows(op, xs)
    dt, dev = _dt(xs[0]), xs[0].device
    ys = [torch.empty_like(x) for x in xs]
    ck = None
    if ckpt:
        ck = torch.empty(max(capi.lib().pvjp_scan_generic_batched_ckpt_bytes(_gop(op), dt, B, L), 16),
                         dtype=torch.uint8, device=dev)
    nb = capi.lib().pvjp_scan_generic_batched_ws_bytes(_gop(op), dt, B, L)
    ws = WS.get("scan_generic", nb, dev)
    capi.call("pvjp_scan_generic_batched", _gop(op), dt, capi.ptr_array([_ptr(x) for x in xs]), B, L,
              capi.ptr_array([_ptr(y) for y in ys]), _ptr(ck), _ptr(ws), ws.numel(), _stream(dev))
    return ys, ck


def scan_generic_batched_vjp(op, xs, y_bar, x_bar=None, accumulate=False, ckpt=None):
    """The VJP of scan_generic_batched, row by row (lists of K [B, L] tensors)."""
    xs, B, L, K = _rows(op, xs)
    dt, dev = _dt(xs[0]), xs[0].device
    if x_bar is None:
        x_bar = [torch.zeros_like(x) if accumulate else torch.empty_like(x) for x in xs]
    if len(y_bar) != K or len(x_bar) != K:
        raise ValueError(f"operator {op} takes {K} components")
    nb = capi.lib().pvjp_scan_generic_batched_ws_bytes(_gop(op), dt, B, L)
    ws = WS.get("scan_generic", nb, dev)
    capi.call("pvjp_scan_generic_batched_vjp", _gop(op), dt, capi.ptr_array([_ptr(x) for x in xs]), B, L,
              _ptr(ckpt), capi.ptr_array([_ptr(y) for y in y_bar]), capi.ptr_array([_ptr(x) for x in x_bar]),
              int(accumulate), _ptr(ws), ws.numel(), _stream(dev))
    return x_bar


def sparse_kmeans_objective(rowptr, col, val, D, C):
    """(f [1] float64, assign [N] int32) for CSR points (rowptr int64, col
    int32, val float32) and dense centres C [K, D] float32."""
    N, K, nnz = rowptr.numel() - 1, C.shape[0], col.numel()
    dev = C.device
    f = torch.empty(1, dtype=torch.float64, device=dev)
    a = torch.empty(N, dtype=torch.int32, device=dev)
    nb = capi.lib().pvjp_sparse_kmeans_ws_bytes(N, D, K, nnz)
    ws = WS.get("sparse_kmeans", nb, dev)
    capi.call("pvjp_sparse_kmeans_objective", _ptr(rowptr), _ptr(col), _ptr(val), N, D, nnz, _ptr(C), K, _ptr(a),
              _ptr(f), _ptr(ws), ws.numel(), _stream(dev))
    return f, a


def sparse_kmeans_vjp(rowptr, col, val, D, C, assign, f_bar=1.0, C_dot=None, out=None, accumulate=False):
    """(C_bar, hvp or None) at the objective's assignments."""
    N, K, nnz = rowptr.numel() - 1, C.shape[0], col.numel()
    dev = C.device
    mk = torch.zeros_like if accumulate else torch.empty_like
    cb, hv = out if out is not None else (mk(C), mk(C) if C_dot is not None else None)
    nb = capi.lib().pvjp_sparse_kmeans_ws_bytes(N, D, K, nnz)
    ws = WS.get("sparse_kmeans", nb, dev)
    capi.call("pvjp_sparse_kmeans_vjp", _ptr(rowptr), _ptr(col), _ptr(val), N, D, nnz, _ptr(C), K, _ptr(assign),
              float(f_bar), _ptr(cb), _ptr(C_dot), _ptr(hv), int(accumulate), _ptr(ws), ws.numel(), _stream(dev))
    return cb, hv


def hist_lae(inds, x, m):
    """hs [m]: log sum exp of each bin's elements (reduce_by_index with the
    log-add-exp operator)."""
    if inds.dtype != torch.int32:
        raise TypeError("inds must be int32")
    dt, dev, n = _dt(x), x.device, x.numel()
    hs = torch.empty(m, dtype=x.dtype, device=dev)
    _check_indices(inds, m)
    _check_values(x)
    nb = capi.lib().pvjp_hist_lae_ws_bytes(dt, n, m)
    ws = WS.get("hist_lae", nb, dev)
    capi.call("pvjp_hist_lae", dt, _ptr(inds), _ptr(x), n, m, _ptr(hs), _ptr(ws), ws.numel(), _stream(dev))
    return hs


def hist_lae_vjp(inds, x, hs, hs_bar, x_bar=None, accumulate=False):
    """x_bar (+)= hs_bar[b] e^(x - hs[b]) per element of bin b."""
    if inds.dtype != torch.int32:
        raise TypeError("inds must be int32")
    if inds.numel() != x.numel():
        raise ValueError("inds and x must have the same number of elements")
    if hs.dtype != x.dtype or hs_bar.dtype != x.dtype:
        raise TypeError("hs and hs_bar must have the dtype of x")
    if hs_bar.numel() != hs.numel():
        raise ValueError("hs_bar must have one element per bin")
    if x_bar is not None and (x_bar.dtype != x.dtype or x_bar.numel() != x.numel()):
        raise ValueError("x_bar must have the dtype and size of x")
    if x_bar is None:
        x_bar = (torch.zeros_like if accumulate else torch.empty_like)(x)
    capi.call("pvjp_hist_lae_vjp", _dt(x), _ptr(inds), _ptr(x), x.numel(), hs.numel(), _ptr(hs), _ptr(hs_bar),
              _ptr(x_bar), int(accumulate), _stream(x.device))
    return x_bar


# ------------------------------------------- reduce_by_index, general operator
def hist_generic(op, inds, xs, m):
    """hs: K tensors [m], each bin's fold in index order with an operator of
    Sec. 5.1.1's general rule (it need not commute); the neutral element for
    an empty bin."""
    if inds.dtype != torch.int32:
        raise TypeError("inds must be int32")
    xs, n, K = _components(op, xs)
    if inds.numel() != n:
        raise ValueError("inds and the components must have the same number of elements")
    dt, dev = _dt(xs[0]), xs[0].device
    _check_indices(inds, m)
    _check_values(*xs)
    hs = [torch.empty(m, dtype=xs[0].dtype, device=dev) for _ in range(K)]
    nb = capi.lib().pvjp_hist_generic_ws_bytes(_gop(op), dt, n, m)
    ws = WS.get("hist_generic", nb, dev)
    capi.call("pvjp_hist_generic", _gop(op), dt, _ptr(inds), capi.ptr_array([_ptr(x) for x in xs]), n, m,
              capi.ptr_array([_ptr(h) for h in hs]), _ptr(ws), ws.numel(), _stream(dev))
    return hs


def hist_generic_vjp(op, inds, xs, hs_bar, x_bar=None, accumulate=False):
    """x_bar (+)= the general rule inside each bin with y_bar = the bin's
    hs_bar (K tensors [m]); 0 for an element whose index is out of range."""
    if inds.dtype != torch.int32:
        raise TypeError("inds must be int32")
    xs, n, K = _components(op, xs)
    if inds.numel() != n:
        raise ValueError("inds and the components must have the same number of elements")
    hs_bar = list(hs_bar)
    if len(hs_bar) != K:
        raise ValueError(f"operator {op} takes {K} components")
    m = hs_bar[0].numel()
    if any(h.numel() != m or h.dtype != xs[0].dtype for h in hs_bar):
        raise ValueError("hs_bar components must have m elements of the dtype of x")
    if x_bar is None:
        x_bar = [(torch.zeros_like if accumulate else torch.empty_like)(x) for x in xs]
    if len(x_bar) != K or any(b.numel() != n or b.dtype != xs[0].dtype for b in x_bar):
        raise ValueError("x_bar must hold K tensors of the size and dtype of x")
    dt, dev = _dt(xs[0]), xs[0].device
    nb = capi.lib().pvjp_hist_generic_ws_bytes(_gop(op), dt, n, m)
    ws = WS.get("hist_generic", nb, dev)
    capi.call("pvjp_hist_generic_vjp", _gop(op), dt, _ptr(inds), capi.ptr_array([_ptr(x) for x in xs]), n, m,
              capi.ptr_array([_ptr(h) for h in hs_bar]), capi.ptr_array([_ptr(b) for b in x_bar]), int(accumulate),
              _ptr(ws), ws.numel(), _stream(dev))
    return x_bar
