"""Benchmark: FP64 TT products per second on one MI355X.

Workload: the square u_x * u_x of one component of a synthetic 3D
random-phase turbulence field on a 256^3 grid (E(k) ~ k^-5/3, seeded),
compressed to a QTT of 8 sites with d = 8 (interleaved x, y, z bits) at bond
dimension chi, product truncated to chi_out = chi_mid = chi with eps = 1e-14.
A step is one whole TTM product (canonicalisation, all contractions, swaps
with truncated SVD, gauge moves and the final rounding) on inputs already
resident in device memory.

Prints one JSON line with the throughput, the roofline of the dominant
kernel (the Jacobi block-pair solve kernel of the swap SVDs, timed with HIP events on
the library's stream during the timed steps), and the CPU oracle's rate on a
bounded sample of the same workload.

``--sweep`` instead measures the bond-dimension sweep on the 10-site shapes
(a 1024^3 field, d = 8, chi in --sweep-chis): one JSON line per chi with the
product rate, the algorithmic flop rate against the FP64 MFMA peak, and the
relative error of sampled entries against the exact product A(x) B(x).

``--batched`` measures the nine advective products u_j * d_j u_i of a
synthetic velocity field (1024^3, 10 sites, d = 8) at uneven bonds, one
after another and in single ttm_multiply_batch calls (FP64 and FP32
contractions): one JSON line per run.

``--adjoint`` measures the gradient of <W, A*B> with respect to the cores
of A and B (ttm_inner_grad) on the 1024^3 chi = 128 QTTs, then the reverse
mode through the truncated product (ttm_multiply_vjp) against the product.

``--binary-sites`` runs the bench product with the field encoded as the
paper's binary QTT (d = 2 sites) beside the d = 8 encoding.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

FP64_MFMA_PEAK_TFLOPS = 78.6   # MI355X dense FP64 matrix peak (published)
# FP64 vector peak from the unit counts: 256 CUs x 4 SIMDs x 16 FP64 lanes x
# 2 flops (FMA) x 2.4 GHz.
FP64_VALU_PEAK_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12
HBM_PEAK_GBS = 8000.0


def _log(msg):
    print(msg, file=sys.stderr, flush=True)


def _measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed counter profile,
    or None when the kernel source changed after the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "jacobi_solve_traffic_turbulence256_chi128.json")
    try:
        prof = json.load(open(path))
        src = open(os.path.join(ROOT, "paper_2410_19747_amd", "csrc", "kernels_svd.hip"), "rb").read()
    except OSError:
        return None
    if prof.get("kernel") != kernel or prof.get("kernel_source_sha256") != hashlib.sha256(src).hexdigest():
        return None
    return float(prof["traffic_bytes_per_dispatch"])


def _cpu_threads():
    try:
        from threadpoolctl import threadpool_info
        n = [i.get("num_threads", 0) for i in threadpool_info() if i.get("user_api") == "blas"]
        if n:
            return int(max(n))
    except Exception:
        pass
    return os.cpu_count() or 1


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--chi", type=int, default=128)
    ap.add_argument("--eps", type=float, default=1e-14)
    ap.add_argument("--grid", type=int, default=256)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-profile", action="store_true", help="no per-kernel event timing")
    ap.add_argument("--no-conventional", action="store_true", help="skip timing the conventional product")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run one 256 MiB device-to-device copy first (reference for HBM counters)")
    ap.add_argument("--sweep", action="store_true", help="bond-dimension sweep on the 10-site shapes")
    ap.add_argument("--sweep-chis", default="64,128,256,512,1024")
    ap.add_argument("--sweep-grid", type=int, default=1024)
    ap.add_argument("--qtt-cache", default="",
                    help="directory for the sweep's QTTs: loaded when present, else generated and saved there")
    ap.add_argument("--generate-only", action="store_true",
                    help="with --sweep and --qtt-cache: generate and save the QTTs, then stop")
    ap.add_argument("--svd-size", type=int, default=0,
                    help="time one N x N truncated SVD (cap N/8, columns scaled by 1/j) through the test hook")
    ap.add_argument("--sweep-precisions", default="f64",
                    help="contraction arithmetic per sweep point, e.g. f64,f32,bf16x3,bf16 (f64 first)")
    ap.add_argument("--batched", action="store_true",
                    help="the nine advective products u_j * d_j u_i at uneven bonds, serial and batched")
    ap.add_argument("--batch-grid", type=int, default=1024)
    ap.add_argument("--batch-chis", default="", help="nine bonds (comma list); default: the fixed uneven set")
    ap.add_argument("--batch-streams", default="4",
                    help="products in flight (streams) for the batched runs, comma list")
    ap.add_argument("--batch-precisions", default="f64,f32",
                    help="contraction arithmetic of the batched runs (f64 first)")
    ap.add_argument("--binary-sites", action="store_true",
                    help="the bench field as a binary QTT (3 log2 n sites, d = 2) beside the d = 8 one")
    ap.add_argument("--mfma-peak", action="store_true",
                    help="measure the FP64 matrix-core rate that the roofline quotes as its peak")
    ap.add_argument("--adjoint", action="store_true",
                    help="gradient of <W, A*B> (1024^3 turbulence QTTs at chi 128, W random at chi 32)")
    ap.add_argument("--upper-chis", default="256,1024",
                    help="bond dimensions of the 10-site 1024^3 points added to the default line")
    ap.add_argument("--upper-precisions", default="f32,rsvd,rsvd+f32,rsvd-fp64",
                    help="reduced-accuracy modes timed at each added point: contraction precisions, "
                         "rsvd (randomized swap SVDs) and rsvd+<precision>")
    ap.add_argument("--no-upper", action="store_true", help="skip the 10-site points of the default line")
    ap.add_argument("--no-rsvd", action="store_true",
                    help="skip the randomized-swap-SVD products of the default line")
    ap.add_argument("--svd-mode", default="jacobi", choices=["jacobi", "randomized"],
                    help="swap SVD of the timed products (randomized: the reduced-accuracy mode; the line's "
                         "value is then that mode's, for profiling runs)")
    ap.add_argument("--no-exact", action="store_true",
                    help="skip the comparison with the dense exact product and the Eckart-Young floor")
    ap.add_argument("--chi-mid-sweep", action="store_true",
                    help="accuracy and time of chi_mid in {chi, 2 chi, 4 chi} against the exact product")
    ap.add_argument("--chi-mid-chis", default="64,128")
    ap.add_argument("--variants", action="store_true",
                    help="schedule variants: the moving factor and where a swap leaves the gauge centre")
    args = ap.parse_args()

    if args.gpus != 1:
        print("bench.py measures one GPU only: a single TT product is a dependent chain of "
              "swaps and is not sharded across GPUs (independent products would be given to "
              "separate GPUs).  Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import ttm_inputs as I
    import paper_2410_19747_amd as T

    assert torch.cuda.is_available(), "needs a GPU"
    torch.cuda.set_device(0)
    dev = torch.device("cuda", 0)
    if args.svd_size:
        return svd_size(args, dev)
    if args.sweep:
        return sweep(args, dev)
    if args.batched:
        return batched(args, dev)
    if args.adjoint:
        return adjoint(args, dev)
    if args.binary_sites:
        return binary_sites(args, dev)
    if args.mfma_peak:
        return mfma_peak(args, dev)
    if args.chi_mid_sweep:
        return chi_mid_sweep(args, dev)
    if args.variants:
        return variants(args, dev)

    if args.calibrate_copy:
        # A plain copy kernel of known size: 256 MiB read, 256 MiB written.
        src = torch.ones(32 << 20, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    _log("generating inputs: %d^3 turbulence, chi=%d" % (args.grid, args.chi))
    t0 = time.time()
    ux = I.turbulence_qtt(args.grid, 101, args.chi)
    _log("  done in %.1f s, bonds %s" % (time.time() - t0, [c.shape[0] for c in ux] + [1]))
    A = T.pack(ux, dev)
    B = T.pack(ux, dev)
    ws = T.Workspace(dev)
    ws_bytes, cap = T.query(A, B, args.chi)
    out = torch.empty(cap, dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream()
    prof = not args.no_profile

    mode = {"svd_mode": args.svd_mode}
    for _ in range(args.warmup):
        T.multiply(A, B, args.chi, args.eps, workspace=ws, out=out, stream=stream, profile=prof, **mode)
    torch.cuda.synchronize()

    # Timed region: K whole products, no instrumentation.
    stats = []
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for _ in range(args.steps):
        C, st = T.multiply(A, B, args.chi, args.eps, workspace=ws, out=out, stream=stream, **mode)
        stats.append(st)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    value = args.steps / elapsed
    ms_per_step = 1e3 * elapsed / args.steps
    _log("  timed: %.1f ms per product, %d Jacobi sweeps, max bond %d"
         % (ms_per_step, stats[-1]["sweeps"], stats[-1]["max_bond"]))

    st = stats[-1]
    model_flops = st["model_flops"]
    svd_flops = st["svd_model_flops"]

    roofline = None
    kernel_share = None
    if prof:
        # The same K products again, every kernel launch bracketed by HIP events
        # recorded on the library's stream (the events cost ~15% wall time, so
        # this pass does not set `value`).
        pstats = []
        torch.cuda.synchronize()
        tp = time.perf_counter()
        for _ in range(args.steps):
            _, s_ = T.multiply(A, B, args.chi, args.eps, workspace=ws, out=out, stream=stream,
                               profile=True, **mode)
            pstats.append(s_)
        torch.cuda.synchronize()
        tp = time.perf_counter() - tp
        rot_ms = sum(s["kernel_ms"]["jacobi_solve"] for s in pstats)
        rot_n = sum(s["kernel_launches"]["jacobi_solve"] for s in pstats)
        tot_ms = sum(sum(s["kernel_ms"].values()) for s in pstats)
        # Algorithmic SVD flops of the product, attributed to the launches of
        # its dominant kernel (one launch = one round of one Jacobi sweep of
        # one SVD: every block pair's Gram diagonalised, V rotated).
        flops_per_launch = sum(s["svd_model_flops"] for s in pstats) / rot_n
        own_per_launch = sum(s["jacobi_solve_flops"] for s in pstats) / rot_n
        avg_launch_s = rot_ms / rot_n / 1e3
        achieved = flops_per_launch / avg_launch_s / 1e12
        # The solve kernel's arithmetic is FP64 vector ALU work (plane
        # rotations of the pair Gram in LDS), so its bound is the ALU peak.
        roofline = {
            "bound": "alu",
            "kernel": "jacobi_solve_kernel",
            "achieved": achieved,
            "peak": FP64_VALU_PEAK_TFLOPS,
            "unit": "TFLOP/s",
            "frac": achieved / FP64_VALU_PEAK_TFLOPS,
            "traffic": _measured_traffic("jacobi_solve_kernel"),
            "launches_per_step": rot_n / args.steps,
            "avg_launch_us": avg_launch_s * 1e6,
            "algorithmic_flops_per_launch": flops_per_launch,
            "profiled_ms_per_step": 1e3 * tp / args.steps,
            # Context for the accounting above, which credits the product's
            # SVD model flops to the solve launches: the solve kernel's own
            # arithmetic (it diagonalises small pair Grams in LDS: latency
            # bound), and the whole product's model flops against the FP64
            # matrix-core peak.
            "kernel_own_flops_per_launch": own_per_launch,
            "kernel_own_frac": own_per_launch / avg_launch_s / 1e12 / FP64_VALU_PEAK_TFLOPS,
            "product_algorithmic_tflops": model_flops / (ms_per_step / 1e3) / 1e12,
            "product_mfma_frac": model_flops / (ms_per_step / 1e3) / 1e12 / FP64_MFMA_PEAK_TFLOPS,
        }
        if roofline["traffic"] is not None:
            roofline["traffic_gbs"] = roofline["traffic"] / avg_launch_s / 1e9
        kernel_share = {k: sum(s["kernel_ms"][k] for s in pstats) / tot_ms for k in st["kernel_ms"]}

    # The conventional chi^4 variational product of the same inputs, for comparison:
    # time per call, sweeps, and its distance from the TTM result.
    conv = None
    if not args.no_conventional:
        cws = T.Workspace(dev)
        _, ccap = T.conventional_query(A, B, args.chi)
        cout = torch.empty(ccap, dtype=torch.float64, device=dev)
        T.conventional(A, B, args.chi, 1e-12, max_sweeps=10, workspace=cws, out=cout, stream=stream)
        torch.cuda.synchronize()
        tc = time.perf_counter()
        for _ in range(args.steps):
            Cc, stc = T.conventional(A, B, args.chi, 1e-12, max_sweeps=10, workspace=cws, out=cout,
                                     stream=stream)
        torch.cuda.synchronize()
        tc = (time.perf_counter() - tc) / args.steps
        conv = {"ms_per_product": 1e3 * tc, "products_per_s": 1.0 / tc, "sweeps": stc["sweeps"],
                "tol": 1e-12, "max_sweeps": 10, "model_flops": stc["model_flops"]}
        _log("  conventional: %.1f ms per product, %d sweeps" % (1e3 * tc, stc["sweeps"]))

    cores = [c.detach().cpu().numpy() for c in C.cores()]
    # The reduced-accuracy mode on the same workload: the swap SVDs by the
    # randomized range finder (svd_mode="randomized"), with FP64 and with
    # FP32 contractions, K products each after one warm-up.
    rsvd = {}
    rsvd_cores = {}
    if not args.no_rsvd and args.svd_mode == "jacobi":
        for mode in ("rsvd", "rsvd+f32", "rsvd-fp64"):
            kw = _mode_options(mode)
            rout = torch.empty(cap, dtype=torch.float64, device=dev)
            T.multiply(A, B, args.chi, args.eps, workspace=ws, out=rout, stream=stream, **kw)
            torch.cuda.synchronize()
            tr = time.perf_counter()
            for _ in range(args.steps):
                Cr, sr = T.multiply(A, B, args.chi, args.eps, workspace=ws, out=rout, stream=stream, **kw)
            torch.cuda.synchronize()
            tr = (time.perf_counter() - tr) / args.steps
            rsvd_cores[mode] = [c.detach().cpu().numpy() for c in Cr.cores()]
            rsvd[mode] = {"ms_per_product": 1e3 * tr, "products_per_s": 1.0 / tr,
                          "speedup_vs_f64": (ms_per_step / 1e3) / tr, "randomized_svds": sr["n_rsvd"],
                          "randomized_fallbacks": sr["n_rsvd_fallback"], "jacobi_sweeps": sr["sweeps"],
                          "ranks_equal_f64": sr["ranks"] == st["ranks"],
                          "effective_fp64_mfma_frac": model_flops / tr / 1e12 / FP64_MFMA_PEAK_TFLOPS}
            _log("  %s: %.1f ms per product (%.2fx over FP64), %d randomized SVDs"
                 % (mode, 1e3 * tr, rsvd[mode]["speedup_vs_f64"], sr["n_rsvd"]))
    accuracy = None
    if not args.no_exact:
        _log("accuracy against the dense exact product (%d entries) and the Eckart-Young floor" % args.grid ** 3)
        conv_cores = [c.detach().cpu().numpy() for c in Cc.cores()] if conv is not None else None
        accuracy = accuracy_vs_exact(ux, ux, cores, conv_cores, args.chi)
        _log("  rel err vs exact: TTM %.4f, conventional %s, Eckart-Young floor %.4f"
             % (accuracy["ttm"], "-" if accuracy["conventional"] is None else "%.4f" % accuracy["conventional"],
                accuracy["eckart_young_floor"]))

    rel_err = None
    cpu = None
    if not args.no_cpu:
        import oracle as O
        from threadpoolctl import threadpool_limits
        _log("CPU oracle on the same product (one product as the sample), all BLAS threads")
        t0 = time.perf_counter()
        ref = O.ttm(ux, ux, args.chi, args.eps)
        dt = time.perf_counter() - t0
        rel_err = O.rel_frob(cores, ref.cores)
        if conv is not None:
            conv["rel_diff_vs_ttm"] = O.rel_frob([c.detach().cpu().numpy() for c in Cc.cores()], cores)
        for mode, rc_ in rsvd_cores.items():
            rsvd[mode]["rel_err_vs_oracle"] = O.rel_frob(rc_, ref.cores)
            _log("  %s: rel. Frobenius error vs the FP64 oracle %.2e" % (mode, rsvd[mode]["rel_err_vs_oracle"]))
        _log("  oracle %.2f s, GPU vs oracle rel. Frobenius error %.2e, ranks equal: %s"
             % (dt, rel_err, st["ranks"] == ref.ranks))
        _log("CPU oracle, one BLAS thread (the paper's timings are from one core)")
        with threadpool_limits(limits=1, user_api="blas"):
            t1 = time.perf_counter()
            O.ttm(ux, ux, args.chi, args.eps)
            dt1 = time.perf_counter() - t1
        _log("  oracle on one thread %.2f s" % dt1)
        cpu = {"value": 1.0 / dt, "unit": "TT products/s", "cores": _cpu_threads(), "kind": "oracle",
               "sample": "one full product (%d^3 u_x*u_x, chi=%d, eps=%g), %.1f s" % (args.grid, args.chi,
                                                                                       args.eps, dt),
               "one_thread": {"value": 1.0 / dt1, "unit": "TT products/s", "cores": 1,
                              "sample": "the same product on one BLAS thread, %.1f s" % dt1}}

    upper = None
    if not args.no_upper:
        upper = upper_points(args, dev)

    line = {
        "metric": "TT products/s + MFMA util vs \u03c7 (64\u20131024); mixed vs FP64 TTM at rel err 1e-6",
        "value": value,
        "unit": "TT products/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "3D turbulence QTT u_x*u_x, %d^3 grid, N=8 sites, d=8" % args.grid,
                   "chi": args.chi, "chi_out": args.chi, "chi_mid": args.chi, "eps": args.eps,
                   "svd_mode": args.svd_mode, "parallelism": "single GPU"},
        "model_flops_per_step": model_flops,
        "svd_model_flops_per_step": svd_flops,
        "algorithmic_tflops": model_flops / (ms_per_step / 1e3) / 1e12,
        "fp64_mfma_frac": model_flops / (ms_per_step / 1e3) / 1e12 / FP64_MFMA_PEAK_TFLOPS,
        "jacobi_sweeps_per_step": st["sweeps"],
        "max_bond": st["max_bond"],
        "rel_err_vs_oracle": rel_err,
        "rel_err_vs_exact": accuracy,
        "kernel_time_share": kernel_share,
        "conventional": conv,
        "randomized_svd": rsvd or None,
        "bond_dimension_points": upper,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


def accuracy_vs_exact(A, B, ttm_cores, conv_cores, chi):
    """Relative Frobenius errors against the dense exact product A(x) B(x)
    of the TTM result and the conventional fit, and the Eckart-Young floor
    at bond chi: any TT with every bond <= chi is at least
    sqrt(max_k sum_{i > chi} sigma_i(k)^2) / ||A*B|| from the exact product,
    sigma(k) the singular values of the unfolding at cut k (computed from
    the Gram matrix of the unfolding's shorter side).  Host-side harness."""
    import numpy as np

    import oracle as O

    exact = (O.dense(A) * O.dense(B)).reshape(-1)
    nrm = float(np.linalg.norm(exact))
    out = {"ttm": float(np.linalg.norm(O.dense(ttm_cores).reshape(-1) - exact) / nrm),
           "conventional": (float(np.linalg.norm(O.dense(conv_cores).reshape(-1) - exact) / nrm)
                            if conv_cores is not None else None)}
    phys = [c.shape[1] for c in A]
    worst = 0.0
    m = 1
    for k in range(len(phys) - 1):
        m *= phys[k]
        M = exact.reshape(m, -1)
        G = M @ M.T if M.shape[0] <= M.shape[1] else M.T @ M
        ev = np.linalg.eigvalsh(G)[::-1]
        worst = max(worst, float(np.sum(np.clip(ev[chi:], 0.0, None))))
    out["eckart_young_floor"] = float(np.sqrt(worst) / nrm)
    out["ttm_over_floor"] = out["ttm"] / out["eckart_young_floor"] if out["eckart_young_floor"] > 0 else None
    if out["conventional"] is not None and out["eckart_young_floor"] > 0:
        out["conventional_over_floor"] = out["conventional"] / out["eckart_young_floor"]
    return out


def upper_points(args, dev):
    """The metric's upper bond dimensions on the 10-site shapes (a 1024^3
    field, d = 8): one measure_point per chi in --upper-chis, FP64 and the
    reduced contraction precisions of --upper-precisions.  Returns a list."""
    import torch

    import ttm_inputs as I

    chis = [int(c) for c in args.upper_chis.split(",") if c]
    if not chis:
        return None
    _log("10-site points: generating 1024^3 turbulence QTTs on the device for chi %s" % chis)
    t0 = time.time()
    qtts = I.turbulence_qtt_device(1024, 101, chis, dev)
    torch.cuda.empty_cache()
    _log("  done in %.1f s" % (time.time() - t0))
    g = torch.Generator(device="cpu")
    g.manual_seed(7)
    idx = torch.randint(0, 8, (4096, 10), generator=g).to(dev)
    pts = []
    for chi in chis:
        pt = measure_point(qtts[chi], chi, args.eps, idx, dev,
                           [q for q in args.upper_precisions.split(",") if q and q != "f64"])
        pt["workload"] = "3D turbulence QTT u_x*u_x, 1024^3 grid, N=10 sites, d=8"
        pts.append(pt)
        torch.cuda.empty_cache()
    return pts


def variants(args, dev):
    """Schedule variants on the bench grid.  (1) Where a swap leaves the
    gauge centre: u_x * u_x at chi --chi with the default (singular values
    into the moving carriage) and with the stated reading (into the right
    carriage, then an LQ move).  (2) Which factor moves: u_y (bond 32) times
    u_x (bond --chi), chi_out = --chi, moving u_x (the second factor) or the
    smaller u_y.  Time per product, QR count, largest bond, relative
    difference between the two variants and error against the dense exact
    product.  One JSON line per run."""
    import torch

    import oracle as O
    import ttm_inputs as I
    import paper_2410_19747_amd as T

    chi = args.chi
    ux = I.turbulence_qtt(args.grid, 101, chi)
    uy = I.turbulence_qtt(args.grid, 102, 32)

    def timed(A, B, **kw):
        ws = T.Workspace(dev)
        T.multiply(A, B, chi, args.eps, workspace=ws, **kw)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(args.steps):
            C, st = T.multiply(A, B, chi, args.eps, workspace=ws, **kw)
        torch.cuda.synchronize()
        return C, st, (time.perf_counter() - t) / args.steps

    exact_xx = (O.dense(ux) * O.dense(ux)).reshape(-1)
    exact_yx = (O.dense(uy) * O.dense(ux)).reshape(-1)
    runs = [("gauge", "moving", (ux, ux), {}), ("gauge", "right", (ux, ux), {"gauge": "right"}),
            ("move_factor", "second", (uy, ux), {}), ("move_factor", "smaller", (uy, ux), {"move_factor": "smaller"})]
    first = {}
    for kind, name, (a, b), kw in runs:
        C, st, dt = timed(T.pack(a, dev), T.pack(b, dev), **kw)
        cores = [c.detach().cpu().numpy() for c in C.cores()]
        exact = exact_xx if kind == "gauge" else exact_yx
        err = float(((O.dense(cores).reshape(-1) - exact) ** 2).sum() ** 0.5 / (exact ** 2).sum() ** 0.5)
        diff = None
        if kind in first:
            diff = O.rel_frob(cores, first[kind])
        else:
            first[kind] = cores
        line = {"variant": kind, "setting": name, "workload": "3D turbulence QTTs, %d^3 grid, N=8 sites, d=8, %s"
                % (args.grid, "u_x*u_x at chi %d" % chi if kind == "gauge" else "u_y (chi 32) * u_x (chi %d)" % chi),
                "chi_out": chi, "eps": args.eps, "ms_per_product": 1e3 * dt, "n_qr": st["n_qr"],
                "n_swap": st["n_swap"], "max_bond": st["max_bond"], "jacobi_sweeps": st["sweeps"],
                "model_flops": st["model_flops"], "rel_err_vs_exact": err, "rel_diff_vs_default": diff}
        print(json.dumps(line), flush=True)
        _log("  %s=%s: %.1f ms, %d QRs, max bond %d, rel err vs exact %.4f%s"
             % (kind, name, 1e3 * dt, st["n_qr"], st["max_bond"], err,
                "" if diff is None else ", rel diff vs default %.2e" % diff))
    return None


def chi_mid_sweep(args, dev):
    """The trade-off of the swap cap (the analogue of the bond growth of
    Sec. II.B and Fig. 3C/D): the bench field squared at each chi of
    --chi-mid-chis with chi_mid in {chi, 2 chi, 4 chi} and the final sweep
    capping at chi: time per product, largest bond, error against the dense
    exact product, beside the conventional fit and the Eckart-Young floor.
    One JSON line per (chi, chi_mid)."""
    import torch

    import ttm_inputs as I
    import paper_2410_19747_amd as T

    for chi in [int(c) for c in args.chi_mid_chis.split(",") if c]:
        ux = I.turbulence_qtt(args.grid, 101, chi)
        A = T.pack(ux, dev)
        Cc, _ = T.conventional(A, A, chi, 1e-12, max_sweeps=10)
        conv_cores = [c.detach().cpu().numpy() for c in Cc.cores()]
        floor = None
        for mult in (1, 2, 4):
            cm = mult * chi
            ws = T.Workspace(dev)
            T.multiply(A, A, chi, args.eps, chi_mid=cm, workspace=ws)
            torch.cuda.synchronize()
            t = time.perf_counter()
            C, st = T.multiply(A, A, chi, args.eps, chi_mid=cm, workspace=ws)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t
            acc = accuracy_vs_exact(ux, ux, [c.detach().cpu().numpy() for c in C.cores()],
                                    conv_cores if floor is None else None, chi)
            if floor is None:
                floor = acc
            line = {"chi_mid_sweep": True, "workload": "3D turbulence QTT u_x*u_x, %d^3 grid, N=8 sites, d=8"
                    % args.grid, "chi": chi, "chi_mid": cm, "eps": args.eps, "ms_per_product": 1e3 * dt,
                    "max_bond": st["max_bond"], "jacobi_sweeps": st["sweeps"], "model_flops": st["model_flops"],
                    "rel_err_vs_exact": acc["ttm"], "conventional_rel_err_vs_exact": floor["conventional"],
                    "eckart_young_floor": floor["eckart_young_floor"]}
            print(json.dumps(line), flush=True)
            _log("  chi=%d chi_mid=%d: %.1f ms, max bond %d, rel err vs exact %.4f (conventional %.4f, floor %.4f)"
                 % (chi, cm, 1e3 * dt, st["max_bond"], acc["ttm"], floor["conventional"],
                    floor["eckart_young_floor"]))
    return None


def _tt_entries(cores, idx):
    """Entries T(x) = prod_i core_i[:, x_i, :] of a TT at the multi-indices
    idx (S x N), by S vector-matrix chains grouped by physical value."""
    import torch

    S = idx.shape[0]
    v = torch.ones(S, 1, dtype=torch.float64, device=idx.device)
    for i, c in enumerate(cores):
        nv = torch.zeros(S, c.shape[2], dtype=torch.float64, device=idx.device)
        for e in range(c.shape[1]):
            sel = (idx[:, i] == e).nonzero().squeeze(1)
            if sel.numel():
                nv[sel] = v[sel] @ c[:, e, :].contiguous()
        v = nv
    return v[:, 0]


def _sweep_qtts(args, chis, dev):
    """The sweep's QTTs (seed 101) for each chi: from --qtt-cache when saved
    there, else generated on the device (and saved when a cache is given).
    Loading them lets a counter run profile the product without the input
    generator's own GPU libraries in the process."""
    import numpy as np

    import ttm_inputs as I

    out, missing = {}, []
    for chi in chis:
        path = os.path.join(args.qtt_cache, "turbulence%d_s101_chi%d.npz" % (args.sweep_grid, chi))
        if args.qtt_cache and os.path.exists(path):
            z = np.load(path)
            out[chi] = [z["arr_%d" % i] for i in range(len(z.files))]
        else:
            missing.append(chi)
    if missing:
        out.update(I.turbulence_qtt_device(args.sweep_grid, 101, missing, dev))
        if args.qtt_cache:
            os.makedirs(args.qtt_cache, exist_ok=True)
            for chi in missing:
                np.savez(os.path.join(args.qtt_cache, "turbulence%d_s101_chi%d.npz" % (args.sweep_grid, chi)),
                         *out[chi])
    return out


def svd_size(args, dev):
    """One N x N truncated SVD, the size of a swap matrix at chi = N / 8 and
    d = 8 (Gaussian columns scaled by 1/j, cap N / 8, eps 1e-14), through the
    library's SVD test hook: time and Jacobi sweeps.  One JSON line."""
    import ctypes

    import numpy as np
    import torch

    from paper_2410_19747_amd import _abi

    L = _abi.load_library()
    n = args.svd_size
    rng = np.random.default_rng(3)
    M = rng.standard_normal((n, n)) * (np.arange(1, n + 1) ** -1.0)[None, :]
    dM = torch.tensor(M.T.copy().ravel(), device=dev)
    del M
    dl = torch.zeros(n * n, dtype=torch.float64, device=dev)
    dr = torch.zeros(n * n, dtype=torch.float64, device=dev)
    ds = torch.zeros(n, dtype=torch.float64, device=dev)
    nb = L.ttm_test_svd_ws_bytes_bw(n, n, 0)
    ws = torch.zeros(nb // 8 + 1, dtype=torch.float64, device=dev)
    rank, sw = ctypes.c_int(0), ctypes.c_int(0)
    _log("svd %d x %d, workspace %.1f GiB" % (n, n, nb / 2 ** 30))
    torch.cuda.synchronize()
    t = time.perf_counter()
    rc = L.ttm_test_svd_bw(ctypes.c_void_p(dM.data_ptr()), n, n, 1e-14, n // 8, 0, 1, 0,
                           ctypes.c_void_p(dl.data_ptr()), ctypes.c_void_p(dr.data_ptr()),
                           ctypes.c_void_p(ds.data_ptr()), ctypes.byref(rank), ctypes.byref(sw), 0,
                           ctypes.c_void_p(ws.data_ptr()), ws.numel() * 8, None)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t
    if rc != 0:
        raise RuntimeError("ttm_test_svd returned %d" % rc)
    print(json.dumps({"svd_size": n, "cap": n // 8, "rank": rank.value, "jacobi_sweeps": sw.value,
                      "seconds": dt}), flush=True)
    return None


def sweep(args, dev):
    import numpy as np
    import torch

    import ttm_inputs as I
    import paper_2410_19747_amd as T

    chis = [int(c) for c in args.sweep_chis.split(",") if c]
    _log("generating %d^3 turbulence QTTs on the device for chi %s" % (args.sweep_grid, chis))
    t0 = time.time()
    qtts = _sweep_qtts(args, chis, dev)
    if args.generate_only:
        return None
    torch.cuda.empty_cache()
    _log("  done in %.1f s" % (time.time() - t0))
    n_sites = len(next(iter(qtts.values())))
    g = torch.Generator(device="cpu")
    g.manual_seed(7)
    idx = torch.randint(0, 8, (4096, n_sites), generator=g).to(dev)
    for chi in chis:
        line = measure_point(qtts[chi], chi, args.eps, idx, dev,
                             [q for q in args.sweep_precisions.split(",") if q and q != "f64"],
                             profile=not args.no_profile, base={"svd_mode": args.svd_mode})
        line["svd_mode"] = args.svd_mode
        line = dict({"sweep": True, "workload": "3D turbulence QTT u_x*u_x, %d^3 grid, N=%d sites, d=8"
                     % (args.sweep_grid, n_sites)}, **line)
        print(json.dumps(line), flush=True)
        torch.cuda.empty_cache()


def _mode_options(mode):
    """Options of a reduced-accuracy mode name: a contraction precision
    ("f32", "bf16", "bf16x3"), "rsvd" (the randomized swap SVD, FP64
    contractions), "rsvd+<precision>", or "rsvd-fp64" (the randomized swap
    SVD with 20 iterations and an acceptance bound of 1e-14)."""
    if mode == "rsvd-fp64":
        # the randomized swap SVD tuned to FP64 parity: 20 iterations, acceptance bound 1e-14
        return {"svd_mode": "randomized", "rsvd_power": 20, "rsvd_tol": 1e-14}
    if mode.startswith("rsvd"):
        kw = {"svd_mode": "randomized"}
        if "+" in mode:
            kw["contract_precision"] = mode.split("+", 1)[1]
        return kw
    return {"contract_precision": mode}


def measure_point(cores, chi, eps, idx, dev, precisions, profile=False, steps=None, base=None):
    """One point of the bond-dimension sweep: u * u for the QTT ``cores`` at
    chi_out = chi_mid = chi.  FP64 products per second (after one warm-up
    product below chi 512), the algorithmic flop rate and its fraction of
    the FP64 MFMA peak, Jacobi sweeps, the relative error of the sampled
    entries ``idx`` against the exact square A(x)^2, and for each reduced
    contraction precision its time and the relative difference of the
    sampled entries from the FP64 product's.  Returns a dict."""
    import torch

    import paper_2410_19747_amd as T

    A = T.pack(cores, dev)
    ws = T.Workspace(dev)
    _, cap = T.query(A, A, chi)
    out = torch.empty(cap, dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream()
    if steps is None:
        steps = 2 if chi <= 256 else 1
    base = base or {}
    if chi <= 256:
        T.multiply(A, A, chi, eps, workspace=ws, out=out, stream=stream, **base)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(steps):
        C, st = T.multiply(A, A, chi, eps, workspace=ws, out=out, stream=stream, **base)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t) / steps
    share = None
    if profile:
        _, sp = T.multiply(A, A, chi, eps, workspace=ws, out=out, stream=stream, profile=True, **base)
        tot = sum(sp["kernel_ms"].values())
        share = {k: v / tot for k, v in sp["kernel_ms"].items()} if tot > 0 else None
    exact = _tt_entries(A.cores(), idx) ** 2
    got = _tt_entries(C.cores(), idx)
    rel = float(torch.linalg.norm(got - exact) / torch.linalg.norm(exact))
    # Mixed-precision contractions at the same point: time and the relative
    # difference of the sampled entries from the FP64 product's.
    mixed = {}
    for prec in precisions:
        kw = _mode_options(prec)
        if kw.get("svd_mode") == "randomized" and chi <= 256:
            # one warm-up, as for the FP64 timing
            T.multiply(A, A, chi, eps, workspace=ws, out=torch.empty_like(out), stream=stream, **kw)
        torch.cuda.synchronize()
        tm = time.perf_counter()
        Cm, stm = T.multiply(A, A, chi, eps, workspace=ws, out=torch.empty_like(out), stream=stream, **kw)
        torch.cuda.synchronize()
        tm = time.perf_counter() - tm
        gm = _tt_entries(Cm.cores(), idx)
        mixed[prec] = {"ms_per_product": 1e3 * tm, "speedup_vs_f64": dt / tm,
                       "sampled_rel_diff_vs_f64": float(torch.linalg.norm(gm - got) / torch.linalg.norm(got)),
                       "jacobi_sweeps": stm["sweeps"], "max_bond": stm["max_bond"],
                       "randomized_svds": stm["n_rsvd"], "randomized_fallbacks": stm["n_rsvd_fallback"],
                       # the FP64 schedule's algorithmic flops over this mode's time: the rate at
                       # which it delivers the same product, against the FP64 matrix peak
                       "effective_fp64_mfma_frac": st["model_flops"] / tm / 1e12 / FP64_MFMA_PEAK_TFLOPS}
        _log("    %s: %.1f ms (%.2fx), sampled rel diff vs FP64 %.2e"
             % (prec, 1e3 * tm, dt / tm, mixed[prec]["sampled_rel_diff_vs_f64"]))
        del Cm
    line = {
        "chi": chi, "eps": eps, "chi_out": chi, "chi_mid": chi,
        "products_per_s": 1.0 / dt, "ms_per_product": 1e3 * dt, "steps": steps,
        "model_flops": st["model_flops"], "svd_model_flops": st["svd_model_flops"],
        "algorithmic_tflops": st["model_flops"] / dt / 1e12,
        "fp64_mfma_frac": st["model_flops"] / dt / 1e12 / FP64_MFMA_PEAK_TFLOPS,
        "jacobi_sweeps": st["sweeps"], "jacobi_max_sweeps": st["jacobi_max_sweeps"],
        "max_bond": st["max_bond"], "n_svd": st["n_svd"],
        "sampled_rel_err_vs_exact": rel, "sampled_points": int(idx.shape[0]),
        "error_bound_abs": st["error_bound"], "kernel_time_share": share,
        "mixed_precision": mixed or None,
        "workspace_bytes": st["peak_ws_bytes"],
    }
    _log("  chi=%d: %.1f ms per product, %.3f TFLOP/s algorithmic, %d sweeps, sampled rel err %.2e"
         % (chi, 1e3 * dt, line["algorithmic_tflops"], st["sweeps"], rel))
    del A, C, out, ws
    return line


def batched(args, dev):
    """Nine products u_j * d_j u_i (i, j in x, y, z) of a synthetic velocity
    field, operands compressed at the uneven bonds ADVECTIVE_CHIS, chi_out =
    chi_mid = the product's bond: one after another (FP64), then in one
    ttm_multiply_batch call per worker count and contraction precision.
    Prints one JSON line per run."""
    import torch

    import ttm_inputs as I
    import paper_2410_19747_amd as T

    chis = [int(c) for c in args.batch_chis.split(",") if c] or list(I.ADVECTIVE_CHIS)
    assert len(chis) == 9
    _log("generating the advective operands on a %d^3 grid, chis %s" % (args.batch_grid, chis))
    t0 = time.time()
    prods = I.advective_qtts_device(args.batch_grid, 201, chis=chis, device=dev)
    torch.cuda.empty_cache()
    _log("  done in %.1f s" % (time.time() - t0))
    n_sites = len(prods[0][0])
    pairs = [(T.pack(A, dev), T.pack(B, dev)) for A, B, _ in prods]
    g = torch.Generator(device="cpu")
    g.manual_seed(7)
    idx = torch.randint(0, 8, (4096, n_sites), generator=g).to(dev)
    exact = [_tt_entries(A.cores(), idx) * _tt_entries(B.cores(), idx) for A, B in pairs]
    workload = ("9 advective products u_j*d_j u_i, 3D turbulence QTTs, %d^3 grid, N=%d sites, d=8, chi %s"
                % (args.batch_grid, n_sites, chis))
    wss = [T.Workspace(dev) for _ in pairs]

    def sampled(results):
        out = []
        for (C, _), ex in zip(results, exact):
            got = _tt_entries(C.cores(), idx)
            out.append(float(torch.linalg.norm(got - ex) / torch.linalg.norm(ex)))
        return out

    # Serial FP64: one ttm_multiply after another on one stream.
    torch.cuda.synchronize()
    t = time.perf_counter()
    serial = []
    per = []
    for (A, B), chi, w in zip(pairs, chis, wss):
        tp = time.perf_counter()
        serial.append(T.multiply(A, B, chi, args.eps, workspace=w))
        per.append(1e3 * (time.perf_counter() - tp))
    torch.cuda.synchronize()
    t_serial = time.perf_counter() - t
    ref = [_tt_entries(C.cores(), idx) for C, _ in serial]
    line = {"batched": False, "workload": workload, "precision": "f64", "products": len(pairs),
            "ms_per_batch": 1e3 * t_serial, "products_per_s": len(pairs) / t_serial,
            "ms_per_product": per, "sampled_rel_err_vs_exact": sampled(serial),
            "model_flops": sum(st["model_flops"] for _, st in serial)}
    print(json.dumps(line), flush=True)
    _log("  serial f64: %.1f ms for %d products (%s)" % (1e3 * t_serial, len(pairs),
                                                           ", ".join("%.0f" % x for x in per)))
    for prec in [q for q in args.batch_precisions.split(",") if q]:
        for nstreams in [int(x) for x in args.batch_streams.split(",") if x]:
            torch.cuda.synchronize()
            t = time.perf_counter()
            res = T.multiply_batch([(A, B) for A, B in pairs], chis, args.eps, streams=nstreams,
                                   workspaces=wss, contract_precision=prec)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t
            same = None
            diffs = []
            for (C, _), r in zip(res, ref):
                got = _tt_entries(C.cores(), idx)
                diffs.append(float(torch.linalg.norm(got - r) / torch.linalg.norm(r)))
            if prec == "f64":
                same = all(
                    torch.equal(C.data[:sum(C.bonds[i] * C.phys[i] * C.bonds[i + 1] for i in range(C.n_sites))],
                                Cs.data[:sum(Cs.bonds[i] * Cs.phys[i] * Cs.bonds[i + 1] for i in range(Cs.n_sites))])
                    for (C, _), (Cs, _) in zip(res, serial))
            line = {"batched": True, "workload": workload, "precision": prec, "streams": nstreams,
                    "products": len(pairs), "ms_per_batch": 1e3 * dt, "products_per_s": len(pairs) / dt,
                    "speedup_vs_serial_f64": t_serial / dt, "identical_to_serial": same,
                    "sampled_rel_diff_vs_serial_f64": diffs, "sampled_rel_err_vs_exact": sampled(res),
                    "jacobi_sweeps": [st["sweeps"] for _, st in res]}
            print(json.dumps(line), flush=True)
            _log("  batched %s, %d streams: %.1f ms (x%.2f vs serial f64), max sampled diff vs f64 %.2e"
                 % (prec, nstreams, 1e3 * dt, t_serial / dt, max(diffs)))
            del res
    return None


def _inner_grad_flops(W, A, B):
    """Algorithmic flops of one ttm_inner_grad call with gradients: the
    right sweep's three contractions per site (sites 1..N-1) and the left
    sweep's six (two for the environment, four for the gradients)."""
    f = 0.0
    n = len(A)
    for k in range(n):
        rw, d, rw2 = W[k].shape
        ra, _, ra2 = A[k].shape
        rb, _, rb2 = B[k].shape
        if k >= 1:
            f += 2.0 * (rw * d * ra2 * rb2 * rw2 + ra * rw * rb2 * ra2 * d + rw * ra * d * rb2 * rb)
        f += 2.0 * (ra * rb * d * rw2 * rw + rb * rw2 * ra2 * ra * d + rb * d * rb2 * rw2 * ra2
                    + rb * rw2 * ra2 * rb2 * d + ra * ra2 * rb * rw2 * d + rw2 * ra2 * rb2 * rb * d)
    return f


def adjoint(args, dev):
    """Gradient of <W, A*B> with respect to the cores of A and B (A, B: the
    1024^3 turbulence QTTs u_x, u_y at chi = 128, 10 sites, d = 8; W a random
    train at chi = 32), FP64 and FP32 contractions, against the oracle's
    gradient, which is also timed on the host.  One JSON line per precision."""
    import numpy as np
    import torch

    import ttm_inputs as I
    import paper_2410_19747_amd as T

    _log("generating 1024^3 turbulence QTTs at chi 128 on the device")
    qa = I.turbulence_qtt_device(1024, 101, [128], dev)[128]
    qb = I.turbulence_qtt_device(1024, 102, [128], dev)[128]
    torch.cuda.empty_cache()
    W = I.random_tt(10, 8, 32, 77)
    A, B, Wp = T.pack(qa, dev), T.pack(qb, dev), T.pack(W, dev)
    flops = _inner_grad_flops(W, qa, qb)
    ref = None
    cpu = None
    if not args.no_cpu:
        import oracle as O
        t = time.perf_counter()
        ref = O.inner3_grad(W, qa, qb)
        cpu = time.perf_counter() - t
    for prec, stride in (("f64", 1), ("f32", 1), ("f64", 0)):
        ws = T.Workspace(dev)
        for _ in range(max(args.warmup, 1)):
            T.inner_grad(Wp, A, B, contract_precision=prec, workspace=ws, env_stride=stride)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(args.steps):
            v, dA, dB = T.inner_grad(Wp, A, B, contract_precision=prec, workspace=ws, env_stride=stride)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t) / args.steps
        err = None
        if ref is not None:
            gA = [c.detach().cpu().numpy() for c in dA.cores()]
            gB = [c.detach().cpu().numpy() for c in dB.cores()]
            num = sum(np.sum((x - y) ** 2) for x, y in zip(gA + gB, ref[1] + ref[2]))
            den = sum(np.sum(y ** 2) for y in ref[1] + ref[2])
            err = float(np.sqrt(num / den))
        line = {"adjoint": True, "workload": "grad of <W, A*B>: 1024^3 turbulence QTTs u_x, u_y at chi 128 "
                "(N=10, d=8), W random at chi 32", "precision": prec, "ms_per_gradient": 1e3 * dt,
                "gradients_per_s": 1.0 / dt, "algorithmic_flops": flops,
                "algorithmic_tflops": flops / dt / 1e12,
                "fp64_mfma_frac": flops / dt / 1e12 / FP64_MFMA_PEAK_TFLOPS,
                "rel_err_vs_oracle_gradient": err, "value": v,
                "env_stride": stride, "workspace_mib": ws.get(0).numel() / 2 ** 20,
                "cpu_oracle_s": cpu, "cpu_cores": _cpu_threads() if cpu is not None else None}
        print(json.dumps(line), flush=True)
        _log("  %s, env stride %d: %.2f ms per gradient, %.2f TFLOP/s algorithmic, rel err vs oracle %s"
             % (prec, stride, 1e3 * dt, flops / dt / 1e12, "%.2e" % err if err is not None else "-"))
    _reverse_mode(args, dev, A, B, Wp)
    return None


def _reverse_mode(args, dev, A, B, Wp):
    """Reverse mode through the truncated product: the gradient of
    <W, TTM(A, B)> at chi = 128, eps = 1e-14 (dL/dC by ttm_inner_grad, then
    ttm_multiply_vjp, which re-runs the product with every step recorded),
    timed against the product alone.  One JSON line."""
    import torch

    import paper_2410_19747_amd as T

    chi, tol = 128, 1e-14
    ws, wsv = T.Workspace(dev), T.Workspace(dev)
    C, st = T.multiply(A, B, chi, tol, workspace=ws)
    _, dC, _ = T.inner_grad(Wp, C, T._ones_like_train(C), workspace=ws)
    for _ in range(max(args.warmup, 1)):
        T.multiply(A, B, chi, tol, workspace=ws)
        T.multiply_vjp(A, B, chi, tol, dC, workspace=wsv)
    torch.cuda.synchronize()
    steps = max(1, min(args.steps, 5))
    t = time.perf_counter()
    for _ in range(steps):
        T.multiply(A, B, chi, tol, workspace=ws)
    torch.cuda.synchronize()
    t_fwd = (time.perf_counter() - t) / steps
    t = time.perf_counter()
    for _ in range(steps):
        _, dA, dB, stv = T.multiply_vjp(A, B, chi, tol, dC, workspace=wsv)
    torch.cuda.synchronize()
    t_vjp = (time.perf_counter() - t) / steps
    line = {"reverse_mode": True, "workload": "grad of <W, TTM(A, B)>: 1024^3 turbulence QTTs u_x, u_y at chi 128 "
            "(N=10, d=8), product at chi 128, eps 1e-14, W random at chi 32",
            "ms_product": 1e3 * t_fwd, "ms_vjp": 1e3 * t_vjp, "vjp_over_product": t_vjp / t_fwd,
            "workspace_gib": wsv.get(0).numel() / 2 ** 30, "ranks_equal": stv["ranks"] == st["ranks"],
            "grad_norm": float(torch.sqrt((dA.data ** 2).sum() + (dB.data ** 2).sum()))}
    print(json.dumps(line), flush=True)
    _log("  reverse mode: product %.1f ms, product + reverse pass %.1f ms" % (1e3 * t_fwd, 1e3 * t_vjp))


def binary_sites(args, dev):
    """The bench field (grid --grid, seed 101) squared at chi = --chi in two
    encodings: sites of d = 8 (bits x_s, y_s, z_s together) and the paper's
    binary sites (each split in three, d = 2).  Time per product, swap and
    sweep counts, sampled error against the exact square of each input, and
    for the binary one the relative error against the oracle.  One JSON
    line per encoding."""
    import numpy as np
    import torch

    import ttm_inputs as I
    import paper_2410_19747_amd as T

    n, chi = args.grid, args.chi
    L = int(round(np.log2(n)))
    _log("generating the %d^3 field as d = 8 and binary QTTs at chi %d" % (n, chi))
    enc = {8: I.turbulence_qtt_device(n, 101, [chi], dev)[chi], 2: I.turbulence_qtt_binary_device(n, 101, chi, dev)}
    torch.cuda.empty_cache()
    g = torch.Generator(device="cpu")
    g.manual_seed(7)
    eta = torch.randint(0, 8, (4096, L), generator=g)
    bits = torch.stack([(eta >> 2) & 1, (eta >> 1) & 1, eta & 1], dim=2).reshape(4096, 3 * L)
    idx = {8: eta.to(dev), 2: bits.to(dev)}
    for d in (8, 2):
        q = enc[d]
        A = T.pack(q, dev)
        ws = T.Workspace(dev)
        T.multiply(A, A, chi, args.eps, workspace=ws)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(args.steps):
            C, st = T.multiply(A, A, chi, args.eps, workspace=ws)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t) / args.steps
        exact = _tt_entries(A.cores(), idx[d]) ** 2
        got = _tt_entries(C.cores(), idx[d])
        rel = float(torch.linalg.norm(got - exact) / torch.linalg.norm(exact))
        oracle_err = None
        oracle_s = None
        if d == 2 and not args.no_cpu:
            import oracle as O
            t0 = time.perf_counter()
            o = O.ttm(q, q, chi, args.eps)
            oracle_s = time.perf_counter() - t0
            oracle_err = float(O.rel_frob([c.detach().cpu().numpy() for c in C.cores()], o.cores))
        line = {"binary_sites": d == 2, "workload": "3D turbulence QTT u_x*u_x, %d^3 grid, N=%d sites, d=%d"
                % (n, len(q), d), "chi": chi, "eps": args.eps, "ms_per_product": 1e3 * dt,
                "products_per_s": 1.0 / dt, "n_swap": st["n_swap"], "n_svd": st["n_svd"],
                "jacobi_sweeps": st["sweeps"], "max_bond": st["max_bond"], "model_flops": st["model_flops"],
                "sampled_rel_err_vs_exact": rel, "rel_err_vs_oracle": oracle_err, "cpu_oracle_s": oracle_s}
        print(json.dumps(line), flush=True)
        _log("  d=%d (%d sites): %.1f ms per product, %d swaps, %d sweeps, sampled rel err %.3e%s"
             % (d, len(q), 1e3 * dt, st["n_swap"], st["sweeps"], rel,
                "" if oracle_err is None else ", vs oracle %.2e (oracle %.1f s)" % (oracle_err, oracle_s)))
    return None


def mfma_peak(args, dev):
    """FP64 matrix-core rate measured on this device (eight independent
    v_mfma_f64_16x16x4f64 chains per wave, 4096 workgroups of four waves),
    beside the published peak that the roofline divides by."""
    import ctypes

    import torch

    import paper_2410_19747_amd as T

    L = T.lib()
    blocks, iters = 4096, 10000
    out = torch.empty(blocks * 256, dtype=torch.float64, device=dev)
    sec, fl = ctypes.c_double(0.0), ctypes.c_double(0.0)
    best = 0.0
    for _ in range(3):
        rc = L.ttm_test_mfma_f64_rate(blocks, iters, ctypes.c_void_p(out.data_ptr()), ctypes.byref(sec),
                                      ctypes.byref(fl), None)
        assert rc == 0, rc
        best = max(best, fl.value / sec.value / 1e12)
    assert bool(torch.isfinite(out).all())
    line = {"mfma_f64_measured_tflops": best, "mfma_f64_published_tflops": FP64_MFMA_PEAK_TFLOPS,
            "ratio": best / FP64_MFMA_PEAK_TFLOPS, "workgroups": blocks, "mfma_per_wave": 8 * iters}
    print(json.dumps(line), flush=True)
    _log("  FP64 MFMA measured %.1f TFLOP/s (published %.1f)" % (best, FP64_MFMA_PEAK_TFLOPS))
    return None


if __name__ == "__main__":
    main()
