"""GPU tests of ttm_multiply_batch: many products in one call, through the C ABI.

Each product of a batch must be the product ttm_multiply_ex gives for the
same arguments (bit for bit: the kernels of one product do not depend on
what runs beside them), and so match the oracle at the FP64 bound.  The
workload is the one that motivates the method (Sec. I): the nine products
u_j * d_j u_i of a synthetic turbulence velocity field at uneven bonds.
"""
import sys

import numpy as np
import pytest

import oracle as O
import ttm_inputs as I

pytestmark = pytest.mark.gpu

TOL = 1e-12


def _torch():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _host(packed):
    return [c.detach().cpu().numpy() for c in packed.cores()]


def _random_pairs():
    """Nine pairs of 8-site trains with d = 2, 3 or 4 and uneven bonds."""
    pairs, chis = [], []
    for k in range(9):
        d = (2, 3, 4)[k % 3]
        chi = (2, 16, 4, 8, 16, 2, 8, 4, 16)[k]
        pairs.append((I.random_tt(8, d, chi, 500 + 2 * k), I.random_tt(8, d, chi, 501 + 2 * k)))
        chis.append(chi)
    return pairs, chis


def test_gpu_batch_equals_single_products():
    import paper_2410_19747_amd as T
    _torch()
    _say("case: batch of 9 random products, uneven bonds, vs single calls")
    pairs, chis = _random_pairs()
    single = [T.multiply(A, B, c, 1e-14) for (A, B), c in zip(pairs, chis)]
    for streams in (4, 1, 3, 2):
        _say("  streams=%d" % streams)
        batch = T.multiply_batch(pairs, chis, 1e-14, streams=streams)
        for k, ((Cb, sb), (Cs, ss)) in enumerate(zip(batch, single)):
            assert Cb.bonds == Cs.bonds, k
            assert sb["ranks"] == ss["ranks"], k
            for x, y in zip(_host(Cb), _host(Cs)):
                assert np.array_equal(x, y), (k, float(np.abs(x - y).max()))
    # and one of them against the oracle
    (A, B), c = pairs[1], chis[1]
    o = O.ttm(A, B, c, 1e-14)
    assert single[1][1]["ranks"] == o.ranks
    assert O.rel_frob(_host(single[1][0]), o.cores) <= TOL


def test_gpu_batch_advective_products_vs_oracle():
    """The nine advective products of a 64^3 field (6 sites, d = 8) at
    uneven bonds, FP64, against the oracle; then with FP32 contractions
    against the same oracle products at the mixed-precision bound."""
    import paper_2410_19747_amd as T
    torch = _torch()
    chis = (32, 8, 16, 24, 8, 32, 16, 24, 8)
    _say("case: advective products 64^3, chis %s" % (chis,))
    prods = I.advective_qtts_device(64, 11, chis=chis, device=torch.device("cuda", 0))
    torch.cuda.empty_cache()
    pairs = [(A, B) for A, B, _ in prods]
    res = T.multiply_batch(pairs, list(chis), 1e-14)
    ref, kappa = [], []
    for k, ((A, B, chi), (C, st)) in enumerate(zip(prods, res)):
        o, kap = _oracle_with_conditioning(A, B, chi)
        ref.append(o)
        kappa.append(kap)
        err = O.rel_frob(_host(C), o.cores)
        _say("  product %d chi=%d rel err %.3e, truncation condition %.1f" % (k, chi, err, kap))
        assert st["ranks"] == o.ranks, k
        assert err <= TOL, k
    res32 = T.multiply_batch(pairs, list(chis), 1e-14, contract_precision="f32")
    errs = [O.rel_frob(_host(C), o.cores) for (C, _), o in zip(res32, ref)]
    for k, (err, kap) in enumerate(zip(errs, kappa)):
        _say("  FP32 contractions: product %d rel err %.3e (condition %.1f)" % (k, err, kap))
    for k, (err, kap) in enumerate(zip(errs, kappa)):
        # FP32 contractions perturb each merged pair by ~1e-7 of its norm; a
        # truncation moves by that times its condition
        # sigma_{r+1} / (sigma_r - sigma_{r+1}).  Well-conditioned products
        # meet the mixed-precision bar of 1e-6.
        assert err <= 1e-6 * max(1.0, kap / 10.0), (k, err, kap)


def _oracle_with_conditioning(A, B, chi):
    """The oracle's product and the largest condition
    sigma_{r+1} / (sigma_r - sigma_{r+1}) over its truncating cuts (0 when
    nothing is truncated): how much a small perturbation of the merged pairs
    can move the truncated result."""
    mod = sys.modules["oracle.ttm"]
    rule = mod.rank_rule
    worst = [0.0]

    def recording(s, eps, cap):
        r, disc = rule(s, eps, cap)
        if r < len(s) and s[r - 1] > 0:
            worst[0] = max(worst[0], float(s[r]) / max(float(s[r - 1] - s[r]), 1e-300))
        return r, disc

    mod.rank_rule = recording
    try:
        o = O.ttm(A, B, chi, 1e-14)
    finally:
        mod.rank_rule = rule
    return o, worst[0]


def test_gpu_batch_advective_products_256_uneven_bonds_vs_oracle():
    """The nine advective products of a 256^3 field (8 sites, d = 8) at the
    uneven bonds 32, 64 and 128 of the batched workload, in one
    ttm_multiply_batch call on 4 streams, FP64, against the oracle: ranks
    equal and <= 1e-12 for every product."""
    import paper_2410_19747_amd as T
    torch = _torch()
    chis = (128, 32, 64, 64, 32, 128, 64, 128, 32)
    _say("case: advective products 256^3, chis %s" % (chis,))
    prods = I.advective_qtts_device(256, 21, chis=chis, device=torch.device("cuda", 0))
    torch.cuda.empty_cache()
    pairs = [(A, B) for A, B, _ in prods]
    res = T.multiply_batch(pairs, list(chis), 1e-14, streams=4)
    for k, ((A, B, chi), (C, st)) in enumerate(zip(prods, res)):
        o = O.ttm(A, B, chi, 1e-14)
        err = O.rel_frob(_host(C), o.cores)
        _say("  product %d chi=%d rel err %.3e" % (k, chi, err))
        assert st["ranks"] == o.ranks, k
        assert err <= TOL, (k, err)


def test_gpu_batch_failure_is_per_product():
    """A product that fails (here: an SVD sweep limit of 1) reports its own
    code; the other products of the batch still finish correctly."""
    import paper_2410_19747_amd as T
    _torch()
    _say("case: batch with one failing product")
    pairs = [(I.random_tt(8, 8, 64, 1), I.random_tt(8, 8, 64, 2)),
             (I.random_tt(6, 2, 4, 3), I.random_tt(6, 2, 4, 4)),
             (I.random_tt(6, 3, 4, 5), I.random_tt(6, 3, 4, 6))]
    options = [{"svd_max_sweeps": 1}, {"chi_mid": 0}, {"chi_mid": 0}]
    res, codes = T.multiply_batch(pairs, [64, 16, 16], 1e-28, options=options, raise_errors=False)
    assert codes[0] == T.TTM_ENOCONV and codes[1:] == [T.TTM_OK, T.TTM_OK]
    assert res[0] is None
    for (A, B), (C, _) in zip(pairs[1:], res[1:]):
        assert O.rel_frob(_host(C), O.brute_force(A, B)) <= TOL
    with pytest.raises(T.TTMError) as ei:
        T.multiply_batch(pairs, [64, 16, 16], 1e-28, options=options)
    assert ei.value.code == T.TTM_ENOCONV


def test_gpu_batch_mixed_shapes_and_precisions():
    """Products of different lengths and physical dimensions in one batch,
    per-product options (uncapped swaps, FP32 contractions): each equals the
    single call with the same options, bit for bit."""
    import paper_2410_19747_amd as T
    _torch()
    _say("case: batch of mixed shapes and options")
    pairs = [(I.random_tt(4, 3, 4, 900), I.random_tt(4, 3, 4, 901)),
             (I.random_tt(7, 2, 8, 902), I.random_tt(7, 2, 8, 903)),
             (I.random_tt(5, [2, 5, 3, 5, 2], 6, 904), I.random_tt(5, [2, 5, 3, 5, 2], 6, 905)),
             (I.random_tt(1, 6, 1, 906), I.random_tt(1, 6, 1, 907))]
    chis = [16, 8, 12, 1]
    options = [{"chi_mid": 0}, {"contract_precision": "f32"}, {"contract_precision": "bf16x3"}, {}]
    single = [T.multiply(A, B, c, 1e-14, **o) for (A, B), c, o in zip(pairs, chis, options)]
    batch = T.multiply_batch(pairs, chis, 1e-14, streams=3, options=options)
    for k, ((Cb, sb), (Cs, ss)) in enumerate(zip(batch, single)):
        assert Cb.bonds == Cs.bonds and sb["ranks"] == ss["ranks"], k
        for x, y in zip(_host(Cb), _host(Cs)):
            assert np.array_equal(x, y), k
    # the exact one against brute force
    (A, B) = pairs[0]
    assert O.rel_frob(_host(batch[0][0]), O.brute_force(A, B)) <= TOL


def test_gpu_batch_stream_tuner():
    """The stream-count tuner times each candidate and returns one of them;
    the batch run with its choice still equals the single calls."""
    import paper_2410_19747_amd as T
    _torch()
    _say("case: batch stream tuner")
    pairs, chis = _random_pairs()
    best, times = T.tune_batch_streams(pairs, chis, 1e-14, candidates=(1, 2, 4))
    assert best in (1, 2, 4) and set(times) == {1, 2, 4}
    assert all(t > 0 for t in times.values())
    batch = T.multiply_batch(pairs, chis, 1e-14, streams=best)
    for (A, B), c, (Cb, _) in zip(pairs, chis, batch):
        Cs, _ = T.multiply(A, B, c, 1e-14)
        for x, y in zip(_host(Cb), _host(Cs)):
            assert np.array_equal(x, y)


def test_gpu_batch_profiled_calls_repeat():
    """Per-kernel timing inside a batch: each worker thread's events are
    released when the call's threads end, so profiled batches can repeat;
    every product reports kernel times and equals the unprofiled one."""
    import paper_2410_19747_amd as T
    _torch()
    _say("case: repeated profiled batches")
    pairs, chis = _random_pairs()
    plain = T.multiply_batch(pairs, chis, 1e-14, streams=4)
    for rep in range(12):
        res = T.multiply_batch(pairs, chis, 1e-14, streams=4, profile=True)
        for (Cp, sp), (Cq, _) in zip(res, plain):
            assert sum(sp["kernel_ms"].values()) > 0.0, rep
            for x, y in zip(_host(Cp), _host(Cq)):
                assert np.array_equal(x, y), rep


def test_gpu_batch_tall_panels_concurrently():
    """Two chi = 512 products of the 1024^3 field side by side (4096-row
    swap matrices: their QR panels run as cooperative multi-workgroup
    launches, their trailing updates through the per-column-block
    reduction), in one batch on two streams: bit for bit the single calls."""
    import paper_2410_19747_amd as T
    torch = _torch()
    _say("case: batch of two chi=512 products on two streams")
    q = I.turbulence_qtt_device(1024, 101, [512], torch.device("cuda", 0))[512]
    torch.cuda.empty_cache()
    A = T.pack(q)
    pairs = [(A, A), (A, A)]
    single = T.multiply(A, A, 512, 1e-14)
    batch = T.multiply_batch(pairs, [512, 512], 1e-14, streams=2)
    for Cb, sb in batch:
        assert sb["ranks"] == single[1]["ranks"]
        assert Cb.bonds == single[0].bonds
        for x, y in zip(Cb.cores(), single[0].cores()):
            assert torch.equal(x, y)


def test_gpu_batch_randomized_svd_equals_single():
    """Products in the reduced-accuracy mode (svd_mode="randomized") in one
    batch beside a full-SVD product: each equals its single call bit for bit
    (the test matrices come from the product's own counter stream), and the
    randomized ones are within 1e-6 of the oracle."""
    import paper_2410_19747_amd as T
    _torch()
    _say("case: batch with randomized swap SVDs")
    ux = I.turbulence_qtt(256, 101, 64)
    uy = I.turbulence_qtt(256, 102, 64)
    pairs = [(ux, uy), (uy, uy), (ux, ux)]
    chis = [64, 64, 64]
    options = [{"svd_mode": "randomized"}, {}, {"svd_mode": "randomized", "contract_precision": "f32"}]
    single = [T.multiply(A, B, c, 1e-14, **o) for (A, B), c, o in zip(pairs, chis, options)]
    batch = T.multiply_batch(pairs, chis, 1e-14, streams=2, options=options)
    for k, ((Cb, sb), (Cs, ss)) in enumerate(zip(batch, single)):
        assert Cb.bonds == Cs.bonds and sb["ranks"] == ss["ranks"], k
        assert sb["n_rsvd"] == ss["n_rsvd"], k
        for x, y in zip(_host(Cb), _host(Cs)):
            assert np.array_equal(x, y), k
    assert batch[0][1]["n_rsvd"] > 0 and batch[1][1]["n_rsvd"] == 0
    o = O.ttm(ux, uy, 64, 1e-14)
    e = O.rel_frob(_host(batch[0][0]), o.cores)
    _say("  randomized product in the batch: relative error vs oracle %.3e" % e)
    assert e <= 1e-6
