"""Host-side checks of the C ABI (no GPU needed).

The library loads, exports every function include/ttm.h declares, sizes
workspaces from shapes alone, and rejects bad arguments with the documented
codes before touching the GPU.
"""
import ctypes
import os
import re

import pytest

from paper_2410_19747_amd import _abi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def L():
    return _abi.load_library()


def _declared_functions(header="ttm.h"):
    text = open(os.path.join(ROOT, "include", header)).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*([a-z_0-9]+)\s*\(", text, flags=re.M)
    return sorted(set(names))


def test_header_symbols_exported(L):
    names = _declared_functions()
    assert "ttm_multiply" in names and "conventional_multiply" in names
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(_abi.PROTOTYPES)
    tnames = _declared_functions("ttm_testing.h")
    for n in tnames:
        assert hasattr(L, n), n
    assert set(tnames) == set(_abi.TESTING_PROTOTYPES)
    assert sorted(os.listdir(os.path.join(ROOT, "include"))) == ["ttm.h", "ttm_testing.h"]


def test_version_and_strerror(L):
    assert b"gfx950" in L.ttm_version()
    for code in range(0, -10, -1):
        assert L.ttm_strerror(code) not in (None, b"unknown error")
    assert L.ttm_strerror(-99) == b"unknown error"


class _TT:
    def __init__(self, phys, bonds, data_ptr=0x1000):
        n = len(phys)
        self.p = (ctypes.c_int32 * n)(*phys)
        self.b = (ctypes.c_int32 * (n + 1))(*bonds)
        offs, pos = [], 0
        for i in range(n):
            offs.append(pos)
            pos += bonds[i] * phys[i] * bonds[i + 1]
        self.o = (ctypes.c_int64 * n)(*offs)
        self.view = _abi.TtmTT(n, ctypes.cast(self.p, _abi.I32P), ctypes.cast(self.b, _abi.I32P),
                               ctypes.cast(self.o, _abi.I64P), ctypes.c_void_p(data_ptr), 0)


def _query(L, A, B, chi, opt=None):
    ws = ctypes.c_size_t(0)
    cap = ctypes.c_int64(0)
    rc = L.ttm_query(ctypes.byref(A.view), ctypes.byref(B.view), chi,
                     ctypes.byref(opt) if opt is not None else None, ctypes.byref(ws), ctypes.byref(cap))
    return rc, ws.value, cap.value


def test_query_sizes_config_shapes(L):
    b10 = [1, 2, 4, 8, 8, 8, 8, 8, 4, 2, 1]
    A = _TT([2] * 10, b10)
    rc, ws, cap = _query(L, A, A, 8)
    assert rc == 0 and ws > 0
    assert cap == sum(b10[i] * 2 * b10[i + 1] for i in range(10))
    b8 = [1, 8, 64, 128, 128, 128, 64, 8, 1]
    A = _TT([8] * 8, b8)
    rc, ws, cap = _query(L, A, A, 128)
    assert rc == 0
    assert cap == sum(b8[i] * 8 * b8[i + 1] for i in range(8))
    assert ws < 512 * 1024 * 1024   # O(d^2 chi^2) workspace, far below the chi^3 environments


def test_query_capacity_follows_chi_out(L):
    b = [1, 2, 4, 8, 8, 8, 8, 8, 4, 2, 1]
    A = _TT([2] * 10, b)
    import ttm_inputs as I
    for chi in (1, 3, 8, 64):
        rc, ws, cap = _query(L, A, A, chi)
        sb = I.structural_bonds([2] * 10, chi)
        assert rc == 0 and cap == sum(sb[i] * 2 * sb[i + 1] for i in range(10))


def test_validation_codes(L):
    good = _TT([2] * 4, [1, 2, 4, 2, 1])
    rc, _, _ = _query(L, good, good, 0)
    assert rc == _abi.TTM_EINVAL                       # chi_out < 1
    other = _TT([2] * 5, [1, 2, 4, 4, 2, 1])
    assert _query(L, good, other, 4)[0] == _abi.TTM_ESHAPE   # N differs
    d3 = _TT([2, 3, 2, 2], [1, 2, 4, 2, 1])
    assert _query(L, good, d3, 4)[0] == _abi.TTM_ESHAPE      # d differs
    bad_end = _TT([2] * 4, [2, 2, 4, 2, 1])
    assert _query(L, bad_end, bad_end, 4)[0] == _abi.TTM_ESHAPE
    neg = _TT([2] * 4, [1, 2, 0, 2, 1])
    assert _query(L, neg, neg, 4)[0] == _abi.TTM_EINVAL
    null = _TT([2] * 4, [1, 2, 4, 2, 1], data_ptr=0)
    assert _query(L, null, null, 4)[0] == _abi.TTM_EINVAL
    f32 = _TT([2] * 4, [1, 2, 4, 2, 1])
    f32.view.dtype = 1
    assert _query(L, f32, f32, 4)[0] == _abi.TTM_EUNSUPPORTED
    o = _abi.TtmOptions()
    L.ttm_default_options(ctypes.byref(o))
    o.chi_mid = -5
    assert _query(L, good, good, 4, o)[0] == _abi.TTM_EINVAL
    L.ttm_default_options(ctypes.byref(o))
    arr = (ctypes.c_int32 * 2)(3, 0)
    o.forced_ranks = ctypes.cast(arr, _abi.I32P)
    o.n_forced = 2
    assert _query(L, good, good, 4, o)[0] == _abi.TTM_EFORCED
    L.ttm_default_options(ctypes.byref(o))
    o.trace_cap = 4      # arrays missing
    assert _query(L, good, good, 4, o)[0] == _abi.TTM_EINVAL
    L.ttm_default_options(ctypes.byref(o))
    assert o.contract_precision == _abi.TTM_PREC_F64
    for bad in (-1, 4):
        o.contract_precision = bad
        assert _query(L, good, good, 4, o)[0] == _abi.TTM_EINVAL
    for ok in (_abi.TTM_PREC_F32, _abi.TTM_PREC_BF16, _abi.TTM_PREC_BF16X3):
        o.contract_precision = ok
        assert _query(L, good, good, 4, o)[0] == _abi.TTM_OK


def test_multiply_rejects_before_gpu_work(L):
    """Argument errors come back before any HIP call (this host has no GPU)."""
    A = _TT([2] * 4, [1, 2, 4, 2, 1])
    bonds = (ctypes.c_int32 * 5)()
    offs = (ctypes.c_int64 * 4)()
    out = _abi.TtmTTOut(ctypes.cast(bonds, _abi.I32P), ctypes.cast(offs, _abi.I64P),
                        ctypes.c_void_p(0x2000), 1 << 20)
    args = (ctypes.byref(A.view), ctypes.byref(A.view), 4)
    # negative / NaN tolerance
    assert L.ttm_multiply(*args, -1.0, ctypes.byref(out), ctypes.c_void_p(0x3000), 1 << 30, None) == _abi.TTM_EINVAL
    assert L.ttm_multiply(*args, float("nan"), ctypes.byref(out), ctypes.c_void_p(0x3000), 1 << 30, None) == _abi.TTM_EINVAL
    # workspace too small / missing
    assert L.ttm_multiply(*args, 1e-12, ctypes.byref(out), ctypes.c_void_p(0x3000), 16, None) == _abi.TTM_EWORKSPACE
    assert L.ttm_multiply(*args, 1e-12, ctypes.byref(out), None, 1 << 30, None) == _abi.TTM_EWORKSPACE
    # output capacity too small
    small = _abi.TtmTTOut(ctypes.cast(bonds, _abi.I32P), ctypes.cast(offs, _abi.I64P),
                          ctypes.c_void_p(0x2000), 3)
    assert L.ttm_multiply(*args, 1e-12, ctypes.byref(small), ctypes.c_void_p(0x3000), 1 << 30, None) == _abi.TTM_ECAPACITY
    # null output
    assert L.ttm_multiply(*args, 1e-12, None, ctypes.c_void_p(0x3000), 1 << 30, None) == _abi.TTM_EINVAL


def test_conventional_query_sizes(L):
    import ttm_inputs as I
    b8 = [1, 8, 64, 64, 64, 64, 64, 8, 1]
    A = _TT([8] * 8, b8)
    ws = ctypes.c_size_t(0)
    cap = ctypes.c_int64(0)
    rc = L.conventional_query(ctypes.byref(A.view), ctypes.byref(A.view), 64, None, ctypes.byref(ws),
                              ctypes.byref(cap))
    assert rc == 0
    sb = I.structural_bonds([8] * 8, 64)
    assert cap.value == sum(sb[i] * 8 * sb[i + 1] for i in range(8))
    # chi^3 environments: at least 2 (N+1) of them at chi_C chi_A chi_B doubles
    assert ws.value >= 64 ** 3 * 8
    bad = _TT([8] * 8, b8, data_ptr=0)
    assert L.conventional_query(ctypes.byref(bad.view), ctypes.byref(A.view), 64, None, ctypes.byref(ws),
                                ctypes.byref(cap)) == _abi.TTM_EINVAL


def test_batch_rejects_before_gpu_work(L):
    """ttm_multiply_batch checks every product, and that no two products share
    workspace or output memory, before any HIP call."""
    A = _TT([2] * 4, [1, 2, 4, 2, 1])
    n = 3
    rc, need, cap = _query(L, A, A, 4)
    assert rc == 0
    bonds = [(ctypes.c_int32 * 5)() for _ in range(n)]
    offs = [(ctypes.c_int64 * 4)() for _ in range(n)]

    def outs(caps, bases=(0x10000000, 0x20000000, 0x30000000)):
        arr = (_abi.TtmTTOut * n)()
        for k in range(n):
            arr[k] = _abi.TtmTTOut(ctypes.cast(bonds[k], _abi.I32P), ctypes.cast(offs[k], _abi.I64P),
                                   ctypes.c_void_p(bases[k]), caps[k])
        return arr

    As = (_abi.TtmTT * n)(*([A.view] * n))
    chis = (ctypes.c_int32 * n)(4, 4, 4)
    tols = (ctypes.c_double * n)(1e-12, 1e-12, 1e-12)
    status = (ctypes.c_int32 * n)()

    def call(ws_ptrs, ws_sizes, out_arr, tol_arr=tols, chi_arr=chis, count=n, n_streams=2):
        wp = (ctypes.c_void_p * n)(*ws_ptrs)
        wb = (ctypes.c_size_t * n)(*ws_sizes)
        return L.ttm_multiply_batch(count, As, As, chi_arr, tol_arr, out_arr, wp, wb, None, None, n_streams,
                                    None, status)

    base = [0x40000000, 0x50000000, 0x60000000]
    assert call(base, [need] * n, outs([cap] * n), count=0) == _abi.TTM_OK
    assert call(base, [need] * n, outs([cap] * n), count=-1) == _abi.TTM_EINVAL
    assert call(base, [need] * n, outs([cap] * n), n_streams=0) == _abi.TTM_EINVAL
    assert call(base, [need] * n, outs([cap] * n), n_streams=5) == _abi.TTM_EINVAL
    assert L.ttm_multiply_batch(n, As, As, chis, tols, None, None, None, None, None, 2, None,
                                status) == _abi.TTM_EINVAL
    # one product's workspace too small, one product's output too small
    assert call(base, [need, need - 8, need], outs([cap] * n)) == _abi.TTM_EWORKSPACE
    assert call(base, [need] * n, outs([cap, cap, cap - 1])) == _abi.TTM_ECAPACITY
    # one bad tolerance, one bad chi_out
    bad_tol = (ctypes.c_double * n)(1e-12, float("nan"), 1e-12)
    assert call(base, [need] * n, outs([cap] * n), tol_arr=bad_tol) == _abi.TTM_EINVAL
    bad_chi = (ctypes.c_int32 * n)(4, 4, 0)
    assert call(base, [need] * n, outs([cap] * n), chi_arr=bad_chi) == _abi.TTM_EINVAL
    # overlapping workspaces, overlapping outputs, a workspace over another product's output
    assert call([base[0], base[0] + 8, base[2]], [need] * n, outs([cap] * n)) == _abi.TTM_EINVAL
    assert call(base, [need] * n, outs([cap] * n, (0x10000000, 0x10000000 + 8, 0x30000000))) == _abi.TTM_EINVAL
    assert call([0x10000000 + 8, base[1], base[2]], [need] * n,
                outs([cap] * n, (0x70000000, 0x10000000, 0x30000000))) == _abi.TTM_EINVAL


def test_inner_grad_rejects_before_gpu_work(L):
    """ttm_inner_grad sizes its workspace from shapes and rejects bad
    arguments before any HIP call."""
    W = _TT([2, 3, 2], [1, 2, 2, 1])
    A = _TT([2, 3, 2], [1, 2, 3, 1])
    B = _TT([2, 3, 2], [1, 2, 1, 1])
    ws = ctypes.c_size_t(0)
    assert L.ttm_inner_grad_query(ctypes.byref(W.view), ctypes.byref(A.view), ctypes.byref(B.view),
                                  ctypes.byref(ws)) == 0
    # right environments (bonds 1,2x2x2,2x3x1,1) + two left ones + three scratch tensors, 32-aligned
    assert ws.value >= 8 * (1 + 8 + 6 + 1)
    Bad = _TT([2, 2, 2], [1, 2, 1, 1])
    assert L.ttm_inner_grad_query(ctypes.byref(W.view), ctypes.byref(A.view), ctypes.byref(Bad.view),
                                  ctypes.byref(ws)) == _abi.TTM_ESHAPE
    v = ctypes.c_double(0.0)
    args = (ctypes.byref(W.view), ctypes.byref(A.view), ctypes.byref(B.view))
    assert L.ttm_inner_grad(*args, 0, None, None, None, ctypes.c_void_p(0x1000), 1 << 20, None) == _abi.TTM_EINVAL
    assert L.ttm_inner_grad(*args, 7, ctypes.byref(v), None, None, ctypes.c_void_p(0x1000), 1 << 20,
                            None) == _abi.TTM_EINVAL
    assert L.ttm_inner_grad(*args, 0, ctypes.byref(v), None, None, None, 1 << 20, None) == _abi.TTM_EWORKSPACE
    assert L.ttm_inner_grad(*args, 0, ctypes.byref(v), None, None, ctypes.c_void_p(0x1000), 16,
                            None) == _abi.TTM_EWORKSPACE


def test_oversized_shapes_rejected_by_every_query(L):
    """Shapes whose QR or SVD unfoldings exceed 2^30 on a side, or whose
    buffers exceed 2^36 doubles, are rejected by the size queries with
    TTM_EINVAL; the sizes are formed in 64 bits and checked before use."""
    ws = ctypes.c_size_t(0)
    cap = ctypes.c_int64(0)
    big = 1 << 16
    # The swap of the product merges a 2^16 bond with a 2^16 dimension: 2^32 rows.
    A = _TT([big, big], [1, big, 1])
    B = _TT([big, big], [1, 1, 1])
    assert _query(L, A, B, 1 << 20)[0] == _abi.TTM_EINVAL
    # Conventional: the initial guess's unfolding d * chi is 2^32 long.
    R1 = _TT([big, big], [1, 1, 1])
    assert L.conventional_query(ctypes.byref(R1.view), ctypes.byref(R1.view), big, None, ctypes.byref(ws),
                                ctypes.byref(cap)) == _abi.TTM_EINVAL
    # Conventional: environments of chi_C * chi_A * chi_B = 2^16 * 2^20 * 2^20 doubles.
    Wide = _TT([2] * 44, [1] + [1 << 20] * 43 + [1])
    assert L.conventional_query(ctypes.byref(Wide.view), ctypes.byref(Wide.view), big, None, ctypes.byref(ws),
                                ctypes.byref(cap)) == _abi.TTM_EINVAL
    # Gradient: environments of 2^60 doubles, then GEMM extents of 2^31.
    G = _TT([big, big], [1, 1 << 20, 1])
    assert L.ttm_inner_grad_query(ctypes.byref(G.view), ctypes.byref(G.view), ctypes.byref(G.view),
                                  ctypes.byref(ws)) == _abi.TTM_EINVAL
    H = _TT([big, big], [1, 1 << 15, 1])
    One = _TT([big, big], [1, 1, 1])
    assert L.ttm_inner_grad_query(ctypes.byref(One.view), ctypes.byref(One.view), ctypes.byref(H.view),
                                  ctypes.byref(ws)) == _abi.TTM_EINVAL
    # The largest shapes the bond-dimension sweep uses still size normally.
    b10 = [1, 8, 64, 512, 1024, 1024, 1024, 512, 64, 8, 1]
    S = _TT([8] * 10, b10)
    rc, need, _ = _query(L, S, S, 1024)
    assert rc == 0 and need >= 8192 * 8192 * 8
    assert L.ttm_inner_grad_query(ctypes.byref(S.view), ctypes.byref(S.view), ctypes.byref(S.view),
                                  ctypes.byref(ws)) == 0


def test_svd_size_limit_rejected_by_query(L):
    """A schedule whose truncated SVD would keep more than 8192 rows
    orthonormal (the SVD kernels' limit) is rejected by ttm_query with
    TTM_EUNSUPPORTED before any GPU work, rather than failing partway."""
    b8 = [1, 8, 64, 128, 128, 128, 64, 8, 1]
    S = _TT([8] * 8, b8)
    assert _query(L, S, S, 128)[0] == _abi.TTM_OK
    uncapped = _abi.TtmOptions()
    L.ttm_default_options(ctypes.byref(uncapped))
    uncapped.chi_mid = 0
    assert _query(L, S, S, 128, uncapped)[0] == _abi.TTM_EUNSUPPORTED
    wide = _abi.TtmOptions()
    L.ttm_default_options(ctypes.byref(wide))
    wide.chi_mid = 2048  # swap matrices of (2048 * 8) rows
    assert _query(L, S, S, 128, wide)[0] == _abi.TTM_EUNSUPPORTED
    # d = 16 at bond 1024: swap matrices of 16384 rows
    D = _TT([16] * 6, [1, 16, 256, 1024, 256, 16, 1])
    assert _query(L, D, D, 1024)[0] == _abi.TTM_EUNSUPPORTED
    # exactly at the limit: 1024 * 8 = 8192 rows is accepted
    b10 = [1, 8, 64, 512, 1024, 1024, 1024, 512, 64, 8, 1]
    T = _TT([8] * 10, b10)
    assert _query(L, T, T, 1024)[0] == _abi.TTM_OK
    assert b"SVD" in L.ttm_strerror(_abi.TTM_EUNSUPPORTED)


def test_static_workspace_entry_rejects_before_gpu_work(L):
    """ttm_multiply_static checks its arguments, the profile option and the
    product's workspace against the static array's size before any HIP
    call, and says why in ttm_last_error."""
    bonds = (ctypes.c_int32 * 9)()
    offs = (ctypes.c_int64 * 8)()
    out = _abi.TtmTTOut(ctypes.cast(bonds, _abi.I32P), ctypes.cast(offs, _abi.I64P), ctypes.c_void_p(0x2000),
                        1 << 30)
    big = _TT([8] * 8, [1, 8, 64, 128, 128, 128, 64, 8, 1])
    rc, need, _ = _query(L, big, big, 128)
    assert rc == 0 and need > _abi.TTM_STATIC_WS_BYTES
    assert L.ttm_multiply_static(ctypes.byref(big.view), ctypes.byref(big.view), 128, 1e-14, ctypes.byref(out),
                                 None, None, None) == _abi.TTM_EWORKSPACE
    msg = L.ttm_last_error().decode()
    assert str(need) in msg and str(_abi.TTM_STATIC_WS_BYTES) in msg
    small = _TT([8] * 8, [1, 8, 64, 64, 64, 64, 64, 8, 1])
    rc, need, _ = _query(L, small, small, 64)
    assert rc == 0 and need <= _abi.TTM_STATIC_WS_BYTES
    o = _abi.TtmOptions()
    L.ttm_default_options(ctypes.byref(o))
    o.profile = 1
    assert L.ttm_multiply_static(ctypes.byref(small.view), ctypes.byref(small.view), 64, 1e-14,
                                 ctypes.byref(out), None, ctypes.byref(o), None) == _abi.TTM_EINVAL
    assert L.ttm_multiply_static(ctypes.byref(small.view), ctypes.byref(small.view), 64, float("nan"),
                                 ctypes.byref(out), None, None, None) == _abi.TTM_EINVAL
    assert L.ttm_multiply_static(ctypes.byref(small.view), ctypes.byref(small.view), 0, 1e-14,
                                 ctypes.byref(out), None, None, None) == _abi.TTM_EINVAL
    assert L.ttm_multiply_static(None, ctypes.byref(small.view), 64, 1e-14, ctypes.byref(out), None, None,
                                 None) == _abi.TTM_EINVAL
    assert L.ttm_multiply_static(ctypes.byref(small.view), ctypes.byref(small.view), 64, 1e-14, None, None, None,
                                 None) == _abi.TTM_EINVAL
    tight = _abi.TtmTTOut(ctypes.cast(bonds, _abi.I32P), ctypes.cast(offs, _abi.I64P), ctypes.c_void_p(0x2000), 8)
    assert L.ttm_multiply_static(ctypes.byref(small.view), ctypes.byref(small.view), 64, 1e-14, ctypes.byref(tight),
                                 None, None, None) == _abi.TTM_ECAPACITY


def test_last_error_is_cleared_by_each_call(L):
    """ttm_last_error describes the last failure of a compute call on this
    thread and is emptied when the next call starts."""
    big = _TT([8] * 8, [1, 8, 64, 128, 128, 128, 64, 8, 1])
    bonds = (ctypes.c_int32 * 9)()
    offs = (ctypes.c_int64 * 8)()
    out = _abi.TtmTTOut(ctypes.cast(bonds, _abi.I32P), ctypes.cast(offs, _abi.I64P), ctypes.c_void_p(0x2000),
                        1 << 30)
    assert L.ttm_multiply_static(ctypes.byref(big.view), ctypes.byref(big.view), 128, 1e-14, ctypes.byref(out),
                                 None, None, None) == _abi.TTM_EWORKSPACE
    assert L.ttm_last_error() != b""
    # an argument error of the next call leaves no stale text behind
    assert L.ttm_multiply_ex(ctypes.byref(big.view), ctypes.byref(big.view), 0, 1e-14, ctypes.byref(out),
                             None, 0, None, None, None) == _abi.TTM_EINVAL
    assert L.ttm_last_error() == b""


def test_vjp_rejects_before_gpu_work(L):
    """ttm_vjp_query sizes the reverse mode from shapes (more than the
    product's own workspace: the record of the steps comes on top), refuses
    the centre-right gauge, and ttm_multiply_vjp rejects bad arguments before
    any HIP call."""
    A = _TT([2] * 4, [1, 2, 4, 2, 1])
    o = _abi.TtmOptions()
    L.ttm_default_options(ctypes.byref(o))
    need, cap = ctypes.c_size_t(0), ctypes.c_int64(0)
    assert L.ttm_vjp_query(ctypes.byref(A.view), ctypes.byref(A.view), 4, ctypes.byref(o), ctypes.byref(need),
                           ctypes.byref(cap)) == 0
    rc, fwd, fcap = _query(L, A, A, 4, o)
    assert rc == 0 and cap.value == fcap
    assert need.value > fwd
    right = _abi.TtmOptions()
    L.ttm_default_options(ctypes.byref(right))
    right.gauge = _abi.TTM_GAUGE_RIGHT
    assert L.ttm_vjp_query(ctypes.byref(A.view), ctypes.byref(A.view), 4, ctypes.byref(right),
                           ctypes.byref(need), ctypes.byref(cap)) == _abi.TTM_EUNSUPPORTED
    assert L.ttm_vjp_query(ctypes.byref(A.view), ctypes.byref(A.view), 0, ctypes.byref(o), ctypes.byref(need),
                           ctypes.byref(cap)) == _abi.TTM_EINVAL
    bonds = (ctypes.c_int32 * 5)()
    offs = (ctypes.c_int64 * 4)()
    out = _abi.TtmTTOut(ctypes.cast(bonds, _abi.I32P), ctypes.cast(offs, _abi.I64P), ctypes.c_void_p(0x2000),
                        1 << 20)
    dA, dB, ws = ctypes.c_void_p(0x4000), ctypes.c_void_p(0x5000), ctypes.c_void_p(0x3000)
    pre = (ctypes.byref(A.view), ctypes.byref(A.view), 4)

    def call(tol=1e-12, opt=o, cbar=A, C=out, ws=ws, nbytes=1 << 30, da=dA):
        return L.ttm_multiply_vjp(*pre, tol, ctypes.byref(opt), ctypes.byref(cbar.view) if cbar else None,
                                  ctypes.byref(C) if C else None, da, dB, ws, nbytes, None, None)

    assert call(tol=float("nan")) == _abi.TTM_EINVAL
    assert call(tol=-1.0) == _abi.TTM_EINVAL
    prof = _abi.TtmOptions()
    L.ttm_default_options(ctypes.byref(prof))
    prof.profile = 1
    assert call(opt=prof) == _abi.TTM_EINVAL
    assert call(opt=right) == _abi.TTM_EUNSUPPORTED
    assert call(ws=None) == _abi.TTM_EWORKSPACE
    assert call(nbytes=need.value - 8) == _abi.TTM_EWORKSPACE
    assert call(C=None) == _abi.TTM_EINVAL
    small = _abi.TtmTTOut(ctypes.cast(bonds, _abi.I32P), ctypes.cast(offs, _abi.I64P), ctypes.c_void_p(0x2000), 3)
    assert call(C=small) == _abi.TTM_ECAPACITY
    assert call(cbar=None) == _abi.TTM_EINVAL
    assert call(da=None) == _abi.TTM_EINVAL
    three = _TT([2] * 3, [1, 2, 2, 1])
    assert call(cbar=three) == _abi.TTM_ESHAPE


def test_inner_grad_checkpoint_sizes(L):
    """ttm_inner_grad_query_ex: stride 1 is the plain query; checkpoints need
    less workspace as N grows; a negative stride is rejected."""
    n = 16
    W = _TT([2] * n, [1] + [4] * (n - 1) + [1])
    A = _TT([2] * n, [1] + [8] * (n - 1) + [1])
    plain, s1, s0, s4 = (ctypes.c_size_t(0) for _ in range(4))
    args = (ctypes.byref(W.view), ctypes.byref(A.view), ctypes.byref(A.view))
    assert L.ttm_inner_grad_query(*args, ctypes.byref(plain)) == 0
    assert L.ttm_inner_grad_query_ex(*args, 1, ctypes.byref(s1)) == 0
    assert L.ttm_inner_grad_query_ex(*args, 0, ctypes.byref(s0)) == 0
    assert L.ttm_inner_grad_query_ex(*args, 4, ctypes.byref(s4)) == 0
    assert s1.value == plain.value
    env = 4 * 8 * 8 * 8  # one environment slot, in bytes
    # 17 environments stored against 4 checkpoints + 3 segment buffers (stride 4 = ceil(sqrt(16)))
    assert plain.value - s0.value >= (17 - 7) * env - 64 * 8 * 17
    assert s4.value == s0.value
    assert L.ttm_inner_grad_query_ex(*args, -1, ctypes.byref(s0)) == _abi.TTM_EINVAL
    v = ctypes.c_double(0.0)
    assert L.ttm_inner_grad_ex(*args, 0, ctypes.byref(v), None, None, -2, ctypes.c_void_p(0x1000), 1 << 20,
                               None) == _abi.TTM_EINVAL


def test_randomized_svd_options(L):
    """svd_mode and rsvd_power are checked on the host; the randomized mode
    asks for at least the full SVD's workspace (the full SVD stays its
    fallback) and is refused by the reverse mode, which differentiates the
    full SVD's truncation only."""
    A = _TT([8] * 8, [1, 8, 64, 128, 128, 128, 64, 8, 1])
    o = _abi.TtmOptions()
    L.ttm_default_options(ctypes.byref(o))
    assert o.svd_mode == _abi.TTM_SVD_JACOBI and o.rsvd_power == 10 and o.rsvd_tol == 2e-8
    rc, ws_full, cap_full = _query(L, A, A, 128, o)
    assert rc == 0
    o.svd_mode = _abi.TTM_SVD_RANDOMIZED
    rc, ws_r, cap_r = _query(L, A, A, 128, o)
    assert rc == 0 and ws_r >= ws_full and cap_r == cap_full
    for mode, power in ((2, 10), (-1, 10), (1, -1), (1, 65)):
        o.svd_mode, o.rsvd_power = mode, power
        assert _query(L, A, A, 128, o)[0] == _abi.TTM_EINVAL
    o.svd_mode, o.rsvd_power = _abi.TTM_SVD_RANDOMIZED, 0
    assert _query(L, A, A, 128, o)[0] == 0
    for tol in (0.0, -1e-8, 1.5, float("nan")):
        o.rsvd_tol = tol
        assert _query(L, A, A, 128, o)[0] == _abi.TTM_EINVAL
    o.rsvd_tol = 1e-14
    assert _query(L, A, A, 128, o)[0] == 0
    need, cap = ctypes.c_size_t(0), ctypes.c_int64(0)
    assert L.ttm_vjp_query(ctypes.byref(A.view), ctypes.byref(A.view), 128, ctypes.byref(o), ctypes.byref(need),
                           ctypes.byref(cap)) == _abi.TTM_EUNSUPPORTED
