"""Reads of uninitialised memory, provoked: every entry point run on a
workspace and an output buffer filled with NaN bit patterns (0xFF bytes, so
doubles are NaN and ints -1) must give bitwise the result it gives on
zero-filled buffers.  A read of a workspace or output byte before the call
writes it would turn into a NaN, a wrong index or a different rounding."""
import sys

import numpy as np
import pytest

import oracle as O
import ttm_inputs as I

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _buffers(torch, T, nbytes, cap, fill):
    ws = T.Workspace(torch.device("cuda", 0))
    buf = ws.get(nbytes)
    buf.fill_(fill)
    out = torch.empty(max(cap, 1), dtype=torch.float64, device="cuda")
    out.view(torch.uint8).fill_(fill)
    return ws, out


def _packed(C):
    n = sum(C.bonds[i] * C.phys[i] * C.bonds[i + 1] for i in range(C.n_sites))
    return C.bonds, C.data[:n].clone()


@pytest.mark.parametrize("case", ["r10", "turbulence256_chi64"])
def test_ttm_on_poisoned_workspace(case):
    import torch
    import paper_2410_19747_amd as T
    assert torch.cuda.is_available()
    _say("case: TTM on a NaN-filled workspace and output, %s" % case)
    if case == "r10":
        A, B, chi = I.random_tt(10, 2, 8, 1), I.random_tt(10, 2, 8, 2), 8
    else:
        A = I.turbulence_qtt(256, 101, 64)
        B, chi = A, 64
    nbytes, cap = T.query(A, B, chi)
    res = {}
    for fill in (0, 255):
        ws, out = _buffers(torch, T, nbytes, cap, fill)
        C, st = T.multiply(A, B, chi, 1e-14, workspace=ws, out=out)
        torch.cuda.synchronize()
        res[fill] = (_packed(C), st["ranks"])
    (b0, d0), r0 = res[0]
    (b1, d1), r1 = res[255]
    assert r0 == r1 and b0 == b1
    assert bool(torch.isfinite(d1).all())
    assert torch.equal(d0, d1)
    if case == "r10":
        ref = O.ttm(A, B, chi, 1e-14)
        host = [c.detach().cpu().numpy() for c in C.cores()]
        assert O.rel_frob(host, ref.cores) <= 1e-12


def test_conventional_on_poisoned_workspace():
    import torch
    import paper_2410_19747_amd as T
    _say("case: conventional on a NaN-filled workspace and output")
    A, B = I.random_tt(10, 2, 8, 1), I.random_tt(10, 2, 8, 2)
    nbytes, cap = T.conventional_query(A, B, 8)
    res = {}
    for fill in (0, 255):
        ws, out = _buffers(torch, T, nbytes, cap, fill)
        C, st = T.conventional(A, B, 8, 1e-13, max_sweeps=6, workspace=ws, out=out)
        torch.cuda.synchronize()
        res[fill] = _packed(C)
    assert res[0][0] == res[255][0]
    assert torch.equal(res[0][1], res[255][1])


def test_inner_grad_on_poisoned_workspace():
    import torch
    import paper_2410_19747_amd as T
    _say("case: ttm_inner_grad on a NaN-filled workspace")
    d = [3, 2, 4, 2, 3]
    W, A, B = I.random_tt(5, d, 6, 41), I.random_tt(5, d, 5, 42), I.random_tt(5, d, 7, 43)
    res = {}
    for fill in (0, 255):
        ws = T.Workspace(torch.device("cuda", 0))
        ws.get(1 << 24).fill_(fill)
        v, dA, dB = T.inner_grad(W, A, B, workspace=ws)
        torch.cuda.synchronize()
        res[fill] = (v, dA.data.clone(), dB.data.clone())
    assert res[0][0] == res[255][0]
    assert torch.equal(res[0][1], res[255][1]) and torch.equal(res[0][2], res[255][2])
    vo, _, _ = O.inner3_grad(W, A, B)
    assert abs(res[255][0] - vo) <= 1e-12 * abs(vo)


def test_batch_on_poisoned_workspaces():
    import torch
    import paper_2410_19747_amd as T
    _say("case: ttm_multiply_batch on NaN-filled workspaces")
    pairs = [(I.random_tt(8, 2, 6, 50 + k), I.random_tt(8, 2, 5, 60 + k)) for k in range(3)]
    res = {}
    for fill in (0, 255):
        wss = []
        for A, B in pairs:
            ws = T.Workspace(torch.device("cuda", 0))
            ws.get(T.query(A, B, 6)[0]).fill_(fill)
            wss.append(ws)
        out = T.multiply_batch(pairs, 6, 1e-14, streams=2, workspaces=wss)
        torch.cuda.synchronize()
        res[fill] = [_packed(C) for C, _ in out]
    for (b0, d0), (b1, d1) in zip(res[0], res[255]):
        assert b0 == b1 and torch.equal(d0, d1)
