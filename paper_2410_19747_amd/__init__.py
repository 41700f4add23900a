"""Python binding of libttm: tensor-train multiplication on an MI355X (gfx950).

Argument marshalling only.  Every step of the product runs in the HIP
kernels of ``libttm.so``; PyTorch provides device memory and the stream.
The functions mirror the C entry points of ``include/ttm.h``:

    multiply(A, B, chi_out, tol, **options)       -> ttm_multiply_ex
    multiply_static(A, B, chi_out, tol, ...)      -> ttm_multiply_static (no workspace)
    conventional(A, B, chi_out, tol, **options)   -> conventional_multiply_ex
    query(A, B, chi_out, **options)               -> ttm_query
    multiply_batch(pairs, chi_out, tol, ...)      -> ttm_multiply_batch
    tune_batch_streams(pairs, chi_out, tol)       -> products in flight, by timing
    inner_grad(W, A, B)                           -> ttm_inner_grad
    multiply_vjp(A, B, chi_out, tol, Cbar)        -> ttm_multiply_vjp (reverse mode)
    ttm_inner_loss(W, A, B, chi_out, tol)         -> torch.autograd.Function over
                                                     ttm_multiply_ex + ttm_inner_grad

A tensor train is a list of float64 CUDA tensors, core i of shape
[r_i, d_i, r_{i+1}] (r_0 = r_N = 1), or a ``PackedTT``.
"""
from __future__ import annotations

import ctypes
import os

from ._abi import (  # noqa: F401
    TTM_OK, TTM_EINVAL, TTM_ESHAPE, TTM_EWORKSPACE, TTM_ECAPACITY, TTM_ENOCONV, TTM_ENONFINITE,
    TTM_EHIP, TTM_EFORCED, TTM_EUNSUPPORTED, TTM_SVD_JACOBI, TTM_SVD_RANDOMIZED, SVD_MODES, TtmTT, TtmTTOut,
    TtmOptions, TtmStats, load_library, library_path,
)

__all__ = [
    "TTMError", "PackedTT", "pack", "multiply", "multiply_static", "multiply_vjp", "multiply_batch", "tune_batch_streams", "inner_grad",
    "ttm_inner_loss",
    "conventional", "query", "conventional_query",
    "Workspace", "lib",
]


class TTMError(RuntimeError):
    def __init__(self, code, where):
        self.code = code
        msg = lib().ttm_strerror(code).decode()
        detail = (lib().ttm_last_error() or b"").decode()
        super().__init__("%s failed: %s (code %d)%s" % (where, msg, code, (": " + detail) if detail else ""))


_LIB = None


def lib():
    """The loaded libttm.so; raises if it has not been built."""
    global _LIB
    if _LIB is None:
        _LIB = load_library()
    return _LIB


class PackedTT:
    """A TT packed into one contiguous float64 device buffer plus host arrays."""

    def __init__(self, data, phys, bonds, offsets):
        import torch

        self.data = data
        self.phys = list(int(p) for p in phys)
        self.bonds = list(int(b) for b in bonds)
        self.offsets = list(int(o) for o in offsets)
        n = len(self.phys)
        if len(self.bonds) != n + 1 or len(self.offsets) != n:
            raise ValueError("a PackedTT of %d sites needs %d bonds and %d offsets" % (n, n + 1, n))
        # The library takes raw device pointers: every core must lie inside data.
        for i in range(n):
            size = self.bonds[i] * self.phys[i] * self.bonds[i + 1]
            if min(self.bonds[i], self.phys[i], self.bonds[i + 1]) < 1 or self.offsets[i] < 0 \
                    or self.offsets[i] + size > data.numel():
                raise ValueError("core %d (offset %d, shape %d x %d x %d) lies outside the %d-element buffer"
                                 % (i, self.offsets[i], self.bonds[i], self.phys[i], self.bonds[i + 1],
                                    data.numel()))
        if data.dtype != torch.float64 or not data.is_contiguous() or data.device.type != "cuda":
            raise ValueError("a PackedTT holds a contiguous float64 GPU tensor (got %s %s on %s)"
                             % ("contiguous" if data.is_contiguous() else "strided", data.dtype, data.device))
        self._phys = (ctypes.c_int32 * n)(*self.phys)
        self._bonds = (ctypes.c_int32 * (n + 1))(*self.bonds)
        self._offsets = (ctypes.c_int64 * n)(*self.offsets)
        self.view = TtmTT(n, ctypes.cast(self._phys, ctypes.POINTER(ctypes.c_int32)),
                          ctypes.cast(self._bonds, ctypes.POINTER(ctypes.c_int32)),
                          ctypes.cast(self._offsets, ctypes.POINTER(ctypes.c_int64)),
                          ctypes.c_void_p(data.data_ptr()), 0)

    @property
    def n_sites(self):
        return len(self.phys)

    def cores(self):
        out = []
        for i, p in enumerate(self.phys):
            rl, rr = self.bonds[i], self.bonds[i + 1]
            o = self.offsets[i]
            out.append(self.data[o:o + rl * p * rr].view(rl, p, rr))
        return out


def pack(cores, device=None):
    """Pack a list of cores (NumPy arrays or tensors) into a PackedTT on the GPU."""
    import numpy as np
    import torch

    if isinstance(cores, PackedTT):
        return cores
    if device is None:
        device = torch.device("cuda", torch.cuda.current_device())
    flat = []
    phys, bonds, offsets = [], [int(cores[0].shape[0])], []
    pos = 0
    for c in cores:
        t = torch.as_tensor(np.asarray(c) if not isinstance(c, torch.Tensor) else c)
        t = t.to(dtype=torch.float64)
        assert t.dim() == 3
        phys.append(int(t.shape[1]))
        bonds.append(int(t.shape[2]))
        offsets.append(pos)
        pos += t.numel()
        flat.append(t.reshape(-1).cpu())
    data = torch.cat(flat).to(device).contiguous()
    return PackedTT(data, phys, bonds, offsets)


class Workspace:
    """A reusable device workspace (grows on demand)."""

    def __init__(self, device=None):
        self.buf = None
        self.device = device

    def get(self, nbytes):
        import torch

        if self.buf is None or self.buf.numel() < nbytes:
            dev = torch.device(self.device) if self.device is not None else \
                torch.device("cuda", torch.cuda.current_device())
            if dev.type != "cuda":
                raise ValueError("a Workspace lives in GPU memory (got %s)" % dev)
            self.buf = torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=dev)
        return self.buf


def _same_device(what, tensor, device):
    """The library is given raw pointers: every buffer of one call must be
    GPU memory on the inputs' device."""
    if tensor.device != device:
        raise ValueError("%s is on %s, the inputs on %s" % (what, tensor.device, device))


_DEFAULT_WS = {}


def _options(chi_mid=None, final_round=True, max_sweeps=10, svd_max_sweeps=40, seed=12345,
             forced_ranks=None, trace_cap=0, profile=False, contract_precision="f64", move_factor="second",
             gauge="moving", svd_mode="jacobi", rsvd_power=None, rsvd_tol=None):
    from ._abi import PRECISIONS, SVD_MODES
    o = TtmOptions()
    lib().ttm_default_options(ctypes.byref(o))
    o.svd_mode = SVD_MODES[svd_mode] if isinstance(svd_mode, str) else int(svd_mode)
    if rsvd_power is not None:
        o.rsvd_power = int(rsvd_power)
    if rsvd_tol is not None:
        o.rsvd_tol = float(rsvd_tol)
    o.move_factor = {"second": 0, "smaller": 1}[move_factor] if isinstance(move_factor, str) else int(move_factor)
    o.gauge = {"moving": 0, "right": 1}[gauge] if isinstance(gauge, str) else int(gauge)
    o.contract_precision = (PRECISIONS[contract_precision] if isinstance(contract_precision, str)
                            else int(contract_precision))
    o.chi_mid = -1 if chi_mid is None else int(chi_mid)
    o.final_round = 1 if final_round else 0
    o.max_sweeps = int(max_sweeps)
    o.svd_max_sweeps = int(svd_max_sweeps)
    o.seed = int(seed)
    o.profile = 1 if profile else 0
    keep = []
    if forced_ranks is not None:
        arr = (ctypes.c_int32 * max(1, len(forced_ranks)))(*[int(r) for r in forced_ranks])
        keep.append(arr)
        o.forced_ranks = ctypes.cast(arr, ctypes.POINTER(ctypes.c_int32))
        o.n_forced = len(forced_ranks)
    if trace_cap:
        ra = (ctypes.c_int32 * trace_cap)()
        da = (ctypes.c_double * trace_cap)()
        keep += [ra, da]
        o.trace_cap = trace_cap
        o.rank_trace = ctypes.cast(ra, ctypes.POINTER(ctypes.c_int32))
        o.discard_trace = ctypes.cast(da, ctypes.POINTER(ctypes.c_double))
    return o, keep


def _stream_handle(stream):
    import torch

    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _query(fn, A, B, chi_out, o):
    ws = ctypes.c_size_t(0)
    cap = ctypes.c_int64(0)
    rc = fn(ctypes.byref(A.view), ctypes.byref(B.view), int(chi_out), ctypes.byref(o),
            ctypes.byref(ws), ctypes.byref(cap))
    if rc != TTM_OK:
        raise TTMError(rc, fn.__name__)
    return ws.value, cap.value


def query(A, B, chi_out, **opts):
    A, B = pack(A), pack(B)
    o, _keep = _options(**opts)
    return _query(lib().ttm_query, A, B, chi_out, o)


def conventional_query(A, B, chi_out, **opts):
    A, B = pack(A), pack(B)
    o, _keep = _options(**opts)
    return _query(lib().conventional_query, A, B, chi_out, o)


def _run(kind, A, B, chi_out, tol, workspace=None, out=None, stream=None, **opts):
    import torch

    A, B = pack(A), pack(B)
    _same_device("B", B.data, A.data.device)
    trace_cap = opts.pop("trace_cap", None)
    if trace_cap is None:
        trace_cap = 4 * A.n_sites * A.n_sites + 16
    o, keep = _options(trace_cap=trace_cap, **opts)
    L = lib()
    qfn = L.conventional_query if kind == "conv" else L.ttm_query
    mfn = {"ttm": L.ttm_multiply_ex, "conv": L.conventional_multiply_ex, "static": L.ttm_multiply_static}[kind]
    ws_bytes, cap = _query(qfn, A, B, chi_out, o)
    wbuf = None
    if kind != "static":
        if workspace is None:
            dev = A.data.device
            workspace = _DEFAULT_WS.setdefault(str(dev), Workspace(dev))
        wbuf = workspace.get(ws_bytes)
        _same_device("the workspace", wbuf, A.data.device)
    if out is not None:
        if out.dtype != torch.float64 or not out.is_contiguous():
            raise ValueError("out must be a contiguous float64 tensor (got %s)" % out.dtype)
        _same_device("out", out, A.data.device)
    if out is None or out.numel() < cap:
        out = torch.empty(max(cap, 1), dtype=torch.float64, device=A.data.device)
    n = A.n_sites
    bonds = (ctypes.c_int32 * (n + 1))()
    offs = (ctypes.c_int64 * n)()
    cout = TtmTTOut(ctypes.cast(bonds, ctypes.POINTER(ctypes.c_int32)),
                    ctypes.cast(offs, ctypes.POINTER(ctypes.c_int64)),
                    ctypes.c_void_p(out.data_ptr()), out.numel())
    st = TtmStats()
    if kind == "static":
        rc = mfn(ctypes.byref(A.view), ctypes.byref(B.view), int(chi_out), float(tol), ctypes.byref(cout),
                 _stream_handle(stream), ctypes.byref(o), ctypes.byref(st))
    else:
        rc = mfn(ctypes.byref(A.view), ctypes.byref(B.view), int(chi_out), float(tol), ctypes.byref(cout),
                 ctypes.c_void_p(wbuf.data_ptr()), ctypes.c_size_t(wbuf.numel()), _stream_handle(stream),
                 ctypes.byref(o), ctypes.byref(st))
    if rc != TTM_OK:
        raise TTMError(rc, mfn.__name__)
    res = PackedTT(out, [A.phys[i] for i in range(n)], list(bonds), list(offs))
    stats = _stats_dict(st, o)
    del keep
    return res, stats


def _stats_dict(st, o):
    from ._abi import KERNEL_CLASSES
    stats = {f: getattr(st, f) for f, _ in TtmStats._fields_ if f not in ("kernel_ms", "kernel_launches")}
    stats["kernel_ms"] = dict(zip(KERNEL_CLASSES, list(st.kernel_ms)))
    stats["kernel_launches"] = dict(zip(KERNEL_CLASSES, list(st.kernel_launches)))
    nt = min(st.n_trace, o.trace_cap)
    if o.trace_cap:
        stats["ranks"] = [o.rank_trace[i] for i in range(nt)]
        stats["discards"] = [o.discard_trace[i] for i in range(nt)]
    return stats


def multiply(A, B, chi_out, tol, **opts):
    """C = A * B elementwise by TTM.  Returns (PackedTT, stats dict).

    Options: chi_mid, final_round, svd_max_sweeps, forced_ranks, trace_cap,
    profile, contract_precision ("f64", "f32", "bf16" or "bf16x3"),
    move_factor ("second" or "smaller"), gauge ("moving" or "right"),
    svd_mode ("jacobi" or "randomized": the reduced-accuracy range-finder SVD
    of the capped swaps), rsvd_power (its subspace iterations, default 10) and
    rsvd_tol (its acceptance bound, default 2e-8)."""
    return _run("ttm", A, B, chi_out, tol, **opts)


def multiply_static(A, B, chi_out, tol, **opts):
    """As multiply, through ttm_multiply_static: the library's static device
    workspace (TTM_STATIC_WS_BYTES per device) instead of a caller buffer,
    for code that must not allocate device memory.  Calls overlapping on one
    device race on that workspace."""
    if "workspace" in opts:
        raise ValueError("multiply_static takes no workspace")
    return _run("static", A, B, chi_out, tol, **opts)


def conventional(A, B, chi_out, tol, **opts):
    """C ~ A * B by the variational baseline.  Returns (PackedTT, stats dict)."""
    return _run("conv", A, B, chi_out, tol, **opts)


def multiply_batch(pairs, chi_out, tol, streams=4, workspaces=None, options=None, raise_errors=True,
                   stream=None, **opts):
    """Products C_k = A_k * B_k for every (A_k, B_k) in ``pairs`` by one call of
    ttm_multiply_batch.  ``chi_out`` and ``tol`` are a value for all or a list.
    ``streams`` is the number of products in flight, each on a stream the
    library creates; they start after the work on ``stream`` (default: the
    current torch stream).
    ``workspaces`` (a list of Workspace, one per product) is created when not
    given; ``options`` (a list of dicts, one per product) overrides the shared
    keyword options per product.  Returns a list of (PackedTT, stats dict).
    A failed product raises TTMError with the lowest-index failure's code,
    naming every failed product; with ``raise_errors=False`` the call returns
    (results, codes) instead, a failed product's result being None."""
    import torch

    n = len(pairs)
    if n == 0:
        return [] if raise_errors else ([], [])
    packed = [(pack(a), pack(b)) for a, b in pairs]
    chis = [int(chi_out)] * n if isinstance(chi_out, int) else [int(c) for c in chi_out]
    tols = [float(tol)] * n if isinstance(tol, (int, float)) else [float(t) for t in tol]
    assert len(chis) == n and len(tols) == n
    dev = packed[0][0].data.device
    for k, (A, B) in enumerate(packed):
        _same_device("A of product %d" % k, A.data, dev)
        _same_device("B of product %d" % k, B.data, dev)
    trace_cap = opts.pop("trace_cap", None)
    L = lib()
    opt_arr = (TtmOptions * n)()
    keep, outs, wbufs, bonds, offs = [], [], [], [], []
    if workspaces is None:
        workspaces = [Workspace(dev) for _ in range(n)]
    assert len(workspaces) == n and int(streams) >= 1
    if options is None:
        options = [{}] * n
    assert len(options) == n
    couts = (TtmTTOut * n)()
    for k, (A, B) in enumerate(packed):
        tc = trace_cap if trace_cap is not None else 4 * A.n_sites * A.n_sites + 16
        o, kp = _options(trace_cap=tc, **dict(opts, **options[k]))
        keep.append(kp)
        opt_arr[k] = o
        ws_bytes, cap = _query(L.ttm_query, A, B, chis[k], o)
        wbufs.append(workspaces[k].get(ws_bytes))
        _same_device("the workspace of product %d" % k, wbufs[k], dev)
        outs.append(torch.empty(max(cap, 1), dtype=torch.float64, device=dev))
        nb = A.n_sites
        bonds.append((ctypes.c_int32 * (nb + 1))())
        offs.append((ctypes.c_int64 * nb)())
        couts[k] = TtmTTOut(ctypes.cast(bonds[k], ctypes.POINTER(ctypes.c_int32)),
                            ctypes.cast(offs[k], ctypes.POINTER(ctypes.c_int64)),
                            ctypes.c_void_p(outs[k].data_ptr()), outs[k].numel())
    a_arr = (TtmTT * n)(*[A.view for A, _ in packed])
    b_arr = (TtmTT * n)(*[B.view for _, B in packed])
    chi_arr = (ctypes.c_int32 * n)(*chis)
    tol_arr = (ctypes.c_double * n)(*tols)
    ws_arr = (ctypes.c_void_p * n)(*[w.data_ptr() for w in wbufs])
    wsb_arr = (ctypes.c_size_t * n)(*[w.numel() for w in wbufs])
    stats_arr = (TtmStats * n)()
    status = (ctypes.c_int32 * n)()
    rc = L.ttm_multiply_batch(n, a_arr, b_arr, chi_arr, tol_arr, couts, ws_arr, wsb_arr, opt_arr, stats_arr,
                              int(streams), _stream_handle(stream), status)
    codes = [int(status[k]) for k in range(n)]
    if rc != TTM_OK and (raise_errors or all(c == TTM_OK for c in codes)):
        bad = [k for k in range(n) if codes[k] != TTM_OK]
        raise TTMError(rc, "ttm_multiply_batch (products %s)" % bad)
    res = []
    for k, (A, _) in enumerate(packed):
        if codes[k] != TTM_OK:
            res.append(None)
            continue
        c = PackedTT(outs[k], list(A.phys), list(bonds[k]), list(offs[k]))
        res.append((c, _stats_dict(stats_arr[k], opt_arr[k])))
    del keep
    return res if raise_errors else (res, codes)


def inner_grad(W, A, B, contract_precision="f64", grads=True, workspace=None, stream=None, env_stride=1):
    """L = <W, A*B> and, with ``grads``, dL/dA and dL/dB as PackedTTs laid
    out like A and B, by one call of ttm_inner_grad_ex.  ``env_stride``: 1
    keeps every right environment, s >= 2 keeps every s-th and recomputes
    the others one segment at a time, 0 picks s = ceil(sqrt(N)).  Returns
    (L, dA, dB) (dA, dB None without ``grads``)."""
    import torch
    from ._abi import PRECISIONS

    W, A, B = pack(W), pack(A), pack(B)
    _same_device("W", W.data, A.data.device)
    _same_device("B", B.data, A.data.device)
    L = lib()
    need = ctypes.c_size_t(0)
    rc = L.ttm_inner_grad_query_ex(ctypes.byref(W.view), ctypes.byref(A.view), ctypes.byref(B.view),
                                   int(env_stride), ctypes.byref(need))
    if rc != TTM_OK:
        raise TTMError(rc, "ttm_inner_grad_query_ex")
    if workspace is None:
        dev = A.data.device
        workspace = _DEFAULT_WS.setdefault(str(dev), Workspace(dev))
    wbuf = workspace.get(need.value)
    _same_device("the workspace", wbuf, A.data.device)
    dA = torch.empty_like(A.data) if grads else None
    dB = torch.empty_like(B.data) if grads else None
    value = ctypes.c_double(0.0)
    prec = PRECISIONS[contract_precision] if isinstance(contract_precision, str) else int(contract_precision)
    rc = L.ttm_inner_grad_ex(ctypes.byref(W.view), ctypes.byref(A.view), ctypes.byref(B.view), prec,
                             ctypes.byref(value), ctypes.c_void_p(dA.data_ptr() if grads else None),
                             ctypes.c_void_p(dB.data_ptr() if grads else None), int(env_stride),
                             ctypes.c_void_p(wbuf.data_ptr()), ctypes.c_size_t(wbuf.numel()),
                             _stream_handle(stream))
    if rc != TTM_OK:
        raise TTMError(rc, "ttm_inner_grad_ex")
    if not grads:
        return value.value, None, None
    return (value.value, PackedTT(dA, A.phys, A.bonds, A.offsets), PackedTT(dB, B.phys, B.bonds, B.offsets))


def multiply_vjp(A, B, chi_out, tol, Cbar, workspace=None, stream=None, **opts):
    """Reverse mode of the TTM product through ttm_multiply_vjp: for the
    cotangent ``Cbar`` of the output cores (a PackedTT with C's bonds, e.g.
    dL/dC), returns (C, dA, dB, stats) with dA, dB the cotangents of A's and
    B's cores (PackedTTs laid out like A and B).  The product C is recomputed
    with every step recorded; ranks are those of that product."""
    import torch

    A, B, Cbar = pack(A), pack(B), pack(Cbar)
    _same_device("B", B.data, A.data.device)
    _same_device("Cbar", Cbar.data, A.data.device)
    trace_cap = opts.pop("trace_cap", None)
    if trace_cap is None:
        trace_cap = 4 * A.n_sites * A.n_sites + 16
    o, keep = _options(trace_cap=trace_cap, **opts)
    L = lib()
    need = ctypes.c_size_t(0)
    cap = ctypes.c_int64(0)
    rc = L.ttm_vjp_query(ctypes.byref(A.view), ctypes.byref(B.view), int(chi_out), ctypes.byref(o),
                         ctypes.byref(need), ctypes.byref(cap))
    if rc != TTM_OK:
        raise TTMError(rc, "ttm_vjp_query")
    if workspace is None:
        dev = A.data.device
        workspace = _DEFAULT_WS.setdefault(str(dev), Workspace(dev))
    wbuf = workspace.get(need.value)
    _same_device("the workspace", wbuf, A.data.device)
    out = torch.empty(max(cap.value, 1), dtype=torch.float64, device=A.data.device)
    n = A.n_sites
    bonds = (ctypes.c_int32 * (n + 1))()
    offs = (ctypes.c_int64 * n)()
    cout = TtmTTOut(ctypes.cast(bonds, ctypes.POINTER(ctypes.c_int32)),
                    ctypes.cast(offs, ctypes.POINTER(ctypes.c_int64)),
                    ctypes.c_void_p(out.data_ptr()), out.numel())
    dA = torch.zeros_like(A.data)
    dB = torch.zeros_like(B.data)
    st = TtmStats()
    rc = L.ttm_multiply_vjp(ctypes.byref(A.view), ctypes.byref(B.view), int(chi_out), float(tol), ctypes.byref(o),
                            ctypes.byref(Cbar.view), ctypes.byref(cout), ctypes.c_void_p(dA.data_ptr()),
                            ctypes.c_void_p(dB.data_ptr()), ctypes.c_void_p(wbuf.data_ptr()),
                            ctypes.c_size_t(wbuf.numel()), _stream_handle(stream), ctypes.byref(st))
    if rc != TTM_OK:
        raise TTMError(rc, "ttm_multiply_vjp")
    C = PackedTT(out, list(A.phys), list(bonds), list(offs))
    stats = _stats_dict(st, o)
    del keep
    return (C, PackedTT(dA, A.phys, A.bonds, A.offsets), PackedTT(dB, B.phys, B.bonds, B.offsets), stats)


def _ones_like_train(T):
    """The all-ones train (every bond 1) with T's physical dimensions."""
    import torch

    offs, pos = [], 0
    for p in T.phys:
        offs.append(pos)
        pos += p
    data = torch.ones(pos, dtype=torch.float64, device=T.data.device)
    return PackedTT(data, T.phys, [1] * (len(T.phys) + 1), offs)


def _make_inner_loss_function():
    import torch

    class TTMInnerLoss(torch.autograd.Function):
        """loss = <W, TTM(A, B)> with W fixed.  Forward: the TTM product
        (ttm_multiply_ex), then <W, C> (ttm_inner_grad against the all-ones
        train).  Backward: dL/dC = the gradient of <W, C> with respect to C's
        cores (ttm_inner_grad_ex, environments recomputed from W and C, with
        checkpoints every ceil(sqrt(N)) sites and the others rebuilt one
        segment at a time), then
        the reverse mode of the product (ttm_multiply_vjp), which recomputes
        the product with every step recorded and undoes the steps, truncated
        SVDs included.  Only the inputs and C are kept from the forward pass."""

        @staticmethod
        def forward(ctx, a_data, b_data, A, B, W, chi_out, tol, prec, opts):
            C, st = multiply(A, B, chi_out, tol, contract_precision=prec, **opts)
            value, _, _ = inner_grad(W, C, _ones_like_train(C), contract_precision=prec, grads=False)
            ctx.trains = (A, B, W, C, chi_out, tol, prec, opts)
            return torch.tensor(value, dtype=torch.float64, device=a_data.device)

        @staticmethod
        def backward(ctx, g):
            A, B, W, C, chi_out, tol, prec, opts = ctx.trains
            _, dC, _ = inner_grad(W, C, _ones_like_train(C), env_stride=0)
            _, dA, dB, _ = multiply_vjp(A, B, chi_out, tol, dC, contract_precision=prec, **opts)
            return g * dA.data, g * dB.data, None, None, None, None, None, None, None

    return TTMInnerLoss


_INNER_LOSS = None


def ttm_inner_loss(W, A, B, chi_out, tol, contract_precision="f64", **opts):
    """0-d tensor <W, TTM(A, B)> whose backward gives dL/dA.data and
    dL/dB.data (PackedTT data tensors with requires_grad): the environments
    of ttm_inner_grad for dL/dC, then the reverse mode of the truncated
    product (ttm_multiply_vjp).  W is a constant train.  Only the full swap
    SVD (svd_mode "jacobi") is differentiated; other modes raise TTMError
    (TTM_EUNSUPPORTED)."""
    global _INNER_LOSS
    mode = opts.get("svd_mode", "jacobi")
    if (SVD_MODES[mode] if isinstance(mode, str) else int(mode)) != TTM_SVD_JACOBI:
        # refused before the forward product: the reverse mode differentiates
        # the full SVD's truncation only
        raise TTMError(TTM_EUNSUPPORTED, "ttm_inner_loss (svd_mode %r; only the full SVD is differentiated)" % (mode,))
    if _INNER_LOSS is None:
        _INNER_LOSS = _make_inner_loss_function()
    W, A, B = pack(W), pack(A), pack(B)
    return _INNER_LOSS.apply(A.data, B.data, A, B, W, int(chi_out), float(tol), contract_precision, opts)


def tune_batch_streams(pairs, chi_out, tol, candidates=(1, 2, 4), repeats=1, **opts):
    """Products in flight for ttm_multiply_batch, chosen by measurement: each
    candidate stream count runs the whole batch `repeats` times and the
    fastest wins.  For a batch that recurs (the nine advective products of
    every time step) the tuning cost is paid once.  Returns (best, {streams:
    seconds per batch}); every candidate's results are discarded."""
    import time

    import torch

    packed = [(pack(a), pack(b)) for a, b in pairs]
    wss = [Workspace(packed[0][0].data.device) for _ in packed]
    times = {}
    for k in candidates:
        k = int(k)
        if k < 1:
            continue
        multiply_batch(packed, chi_out, tol, streams=k, workspaces=wss, **opts)   # warm-up
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(max(1, int(repeats))):
            multiply_batch(packed, chi_out, tol, streams=k, workspaces=wss, **opts)
        torch.cuda.synchronize()
        times[k] = (time.perf_counter() - t) / max(1, int(repeats))
    best = min(times, key=times.get)
    return best, times
