"""Benchmark of the fast GFT on one MI355X.

Default workload (the headline line): 8x8 4-neighbour grid, 2^20 AR(1) signals, FP32.
One step = forward GFT (y = U^T x) + inverse GFT (x' = U y) of the whole batch, inputs
resident in HBM; ``value`` counts the values both transforms produce (2 * S * n) per
second.  Also reported: the dominant (forward) kernel's achieved HBM bandwidth against the
8 TB/s peak (HIP events on the launch stream), the dense-GFT GEMM (torch.matmul, FP32 and
BF16) on the same GPU and basis, a plain device copy of the same bytes, and the FP64
oracle timed on host cores on a bounded sample (with the GPU's relative error there).

Other workloads (``--workload``): ``skeleton`` (25-joint skeleton, 16384 x 3 x 300
signals, BF16 leaf blocks), ``mixed`` (the ~150-graph uneven batch, one persistent launch
per direction), ``grid64`` (64x64 grid, 12 stages, 65536 signals) and ``wpath1024``
(weighted symmetric path, n = 1024, 65536 signals); the last two run the large-signal
engine (stage/permutation passes + grouped MFMA GEMM) and are reported against the MFMA
roofline of their precision.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload grid8x8]
"""
from __future__ import annotations

import argparse
import ctypes
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# block precision -> the library's precision number (GFT_FP32 .. GFT_SPLIT_BF16)
PREC_ID = {"fp32": 0, "bf16": 1, "fp16": 2, "split_bf16": 3}
MFMA_PEAK_TFLOPS = {"fp32": 157.3, "bf16": 2500.0, "fp16": 2500.0,
                    "split_bf16": 2500.0 / 3.0}   # split: three BF16 products per product
METRIC = "GFT coeffs/sec, fast vs dense GFT on 1 GPU at stated rel. err; % HBM roofline"

# HBM bytes per forward launch of the 8x8-grid workload from rocprofv3 FETCH_SIZE /
# WRITE_SIZE, scaled by the same counters on a 256 MiB device copy
# (profiles/gft_grid8x8_hbm_traffic.md).  Valid only for the kernel source it was measured
# on: reported as null once that file changes.
PROFILED_TRAFFIC = {"sources": ["paper_1907_07875_amd/csrc/gft_butterfly.hip",
                                "paper_1907_07875_amd/csrc/butterfly_core.hpp",
                                "paper_1907_07875_amd/csrc/device_program.hpp"],
                    "sha256_16": "fc5dea449a1a5f30",
                    "bytes_per_launch": 2.0 * 131161.1 * 1024 + 262149.2 * 1024}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="grid8x8",
                    choices=["grid8x8", "skeleton", "mixed", "grid64", "wpath1024"])
    ap.add_argument("--signals", type=int, default=None, help="override the signal count")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-dense", action="store_true")
    ap.add_argument("--engine", default="auto", choices=["auto", "generic", "butterfly", "large", "product"],
                    help="grid64: large runs the 12-stage plan's dense leaf blocks on the large engine; "
                         "product plans the grid with gft_plan_product from two 64-node paths")
    ap.add_argument("--precision", default=None, choices=["fp32", "bf16", "fp16", "split_bf16"])
    ap.add_argument("--io", default="fp32", choices=["fp32", "bf16"],
                    help="storage type of signals and coefficients (single-graph workloads)")
    ap.add_argument("--profile-copy", action="store_true",
                    help="only run a plain device copy of the input size (counter calibration)")
    return ap.parse_args()


def _threads():
    try:
        from threadpoolctl import threadpool_info
        return max([d.get("num_threads", 1) for d in threadpool_info()] + [1])
    except Exception:
        return os.cpu_count() or 1


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except Exception:
        pass
    return "unknown"


def _oracle_apply_rate(bases, seconds):
    """Values per second of the oracle's forward + inverse (FP64 GEMMs) over `seconds`."""
    from oracle import gft_oracle as O
    t0 = time.perf_counter()
    reps, values = 0, 0.0
    while True:
        for lam, U, Xd in bases:
            C = O.forward(Xd, U)
            O.inverse(C, U)
            values += 2.0 * Xd.size
        reps += 1
        if time.perf_counter() - t0 > seconds:
            break
    dt = time.perf_counter() - t0
    return values / dt, reps, dt


def cpu_baseline(samples, desc, seconds=8.0):
    """FP64 oracle on the host on a bounded sample: Laplacian + eigh once per graph (timed
    apart), then forward + inverse repeatedly for `seconds` with every BLAS thread and again
    with one thread; beside it the GPU's errors on the sample against the oracle, its basis
    aligned per eigenvalue cluster: batch Frobenius relative error, the largest per-signal
    relative error, and the paper's delta and epsilon (Sec. VI-B) of the basis the GPU
    applies (forward of the unit vectors).

    samples: list of (graph, X_sample [s, n] float32, Y_gpu_sample [s, n], plan_basis,
    gpu_basis [n, n]).
    """
    import numpy as np
    from oracle import gft_oracle as O
    t0 = time.perf_counter()
    bases = []
    for g, X, _, _, _ in samples:
        lam, U = O.gft(O.laplacian_of(g))
        bases.append((lam, U, X.astype(np.float64)))
    eigh_s = time.perf_counter() - t0
    rate_all, reps_all, dt_all = _oracle_apply_rate(bases, seconds)
    one = {"value": None, "cores": 1}
    try:
        from threadpoolctl import threadpool_limits
        with threadpool_limits(limits=1):
            rate_one, reps_one, dt_one = _oracle_apply_rate(bases, seconds)
        one = {"value": rate_one, "unit": "coeffs/s", "cores": 1,
               "sample": f"{reps_one} x (forward + inverse), {dt_one:.1f} s"}
    except ImportError:
        pass
    num = den = 0.0
    min_sv, max_row, delta, eps = 1.0, 0.0, 0.0, 0.0
    for (g, X, Yg, Ub, Ug), (lam, U, Xd) in zip(samples, bases):
        Ua, sv = O.align(U, Ub, lam)
        min_sv = min(min_sv, sv)
        ref = O.forward(Xd, Ua)
        num += float(np.sum((Yg - ref) ** 2))
        den += float(np.sum(ref ** 2))
        max_row = max(max_row, O.max_row_relative_error(Yg, ref))
        delta = max(delta, O.delta_metric(Ug, Ua))
        eps = max(eps, O.epsilon_metric(Ug, Ua, Xd))
    return {
        "value": rate_all, "unit": "coeffs/s", "cores": int(_threads()), "kind": "oracle",
        "sample": f"{desc}; Laplacian + eigh once per graph ({eigh_s:.2f} s), then {reps_all} x "
                  f"(forward + inverse) FP64 NumPy/LAPACK, {dt_all:.1f} s",
        "eigh_s": eigh_s,
        "one_core": one,
        "gpu_forward_rel_err_vs_oracle": (num / den) ** 0.5 if den > 0 else 0.0,
        "gpu_forward_max_signal_rel_err": max_row,
        "gpu_basis_delta": delta,
        "gpu_epsilon": eps,
        "error_note": "oracle basis aligned per eigenvalue cluster (sign, or rotation inside a "
                      "repeated eigenspace); delta and epsilon of Sec. VI-B on the basis the GPU "
                      "applies; worst graph where the sample has several",
        "plan_basis_min_singular_value": min_sv,
        "cpu_model": _cpu_model(), "os_cpu_count": os.cpu_count(),
    }


def avg_ms(torch, stream, fn, reps):
    """Average duration of `reps` back-to-back launches, by HIP events on `stream`."""
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for i in range(reps):
        fn(i)
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def run_steps(torch, stream, fwd, inv, steps, warmup):
    """Warm up, then time `steps` steps of forward + inverse (wall clock, synchronised on
    both sides) with HIP events around every forward launch."""
    import numpy as np
    for i in range(warmup):
        fwd(i)
        inv(i)
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        evs[i][0].record(stream)
        fwd(i)
        evs[i][1].record(stream)
        inv(i)
    torch.cuda.synchronize()
    ms_step = (time.perf_counter() - t0) * 1e3 / steps
    fwd_ms = float(np.mean([a.elapsed_time(b) for a, b in evs]))
    return ms_step, fwd_ms


def _c(ptr):
    return ctypes.c_void_p(ptr)


def bench_single(args, graph, X_host, precision, workload_cfg, sample_rows, sample_desc,
                 kernel_names=None, flops_per_signal=None, make_plan=None):
    """Shared body of the single-graph workloads (make_plan: builds the plan instead of
    planning `graph`, which then only serves the oracle)."""
    import torch

    import paper_1907_07875_amd as G

    dev = torch.device("cuda:0")
    S, n = X_host.shape
    io16 = getattr(args, "io", "fp32") == "bf16"
    esz = 2 if io16 else 4
    xa = torch.from_numpy(X_host).to(dev)
    if io16:
        xa = xa.to(torch.bfloat16)
    xb = torch.roll(xa, shifts=1, dims=0).contiguous()   # second buffer: defeats the 256 MB cache
    if args.profile_copy:
        out = torch.empty_like(xa)
        for _ in range(max(1, args.steps)):
            out.copy_(xa)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_per_launch": 2 * xa.numel() * esz}))
        return

    plan = make_plan() if make_plan else G.Plan.from_graph(graph, engine=args.engine, precision=precision,
                                                           in_dtype=args.io, out_dtype=args.io)
    plan.prepare()
    if (plan.in_dtype, plan.out_dtype) != (args.io, args.io):
        # the buffers below hold args.io values: a plan with other storage would read and
        # write past them
        raise SystemExit(f"plan storage {plan.in_dtype}/{plan.out_dtype} differs from --io {args.io}")
    eng = plan.engine()
    tiles = plan.tiles()
    launch = plan.tuning()
    stream = torch.cuda.current_stream()
    ya, yb, xr = torch.empty_like(xa), torch.empty_like(xa), torch.empty_like(xa)
    bufs = [(xa, ya), (xb, yb)]
    # the timed loops call the C ABI directly with pre-marshalled arguments, so that host
    # overhead between the timing events and the launches stays at a few microseconds
    lib, h, sp = G.load_library(), plan.handle, _c(int(stream.cuda_stream))
    P = {id(t): _c(t.data_ptr()) for t in (xa, xb, ya, yb, xr)}

    def fwd(i):
        x, y = bufs[i & 1]
        st = lib.gft_forward(h, P[id(x)], P[id(y)], S, sp)
        if st:
            G._check(st)

    def inv(i):
        st = lib.gft_inverse(h, P[id(bufs[i & 1][1])], P[id(xr)], S, sp)
        if st:
            G._check(st)

    ms_step, fwd_ms = run_steps(torch, stream, fwd, inv, args.steps, args.warmup)
    inv_ms = avg_ms(torch, stream, inv, args.steps)
    # copies of the same bytes: the library's streaming copy (non-temporal 16-byte loads and
    # stores, the HBM reference) and the runtime's device copy
    G.gft_stream_copy(bufs[0][0], bufs[0][1], stream=stream)
    scopy_ms = avg_ms(torch, stream, lambda i: G.gft_stream_copy(bufs[i & 1][0], bufs[i & 1][1], stream=stream),
                      args.steps)
    copy_ms = avg_ms(torch, stream, lambda i: bufs[i & 1][1].copy_(bufs[i & 1][0]), args.steps)
    bytes_per_launch = 2.0 * S * n * esz
    achieved = bytes_per_launch / (fwd_ms * 1e-3) / 1e9
    scopy_gbs = bytes_per_launch / (scopy_ms * 1e-3) / 1e9
    copy_gbs = bytes_per_launch / (copy_ms * 1e-3) / 1e9
    kname = (kernel_names or {}).get(eng, f"{eng} engine kernel")
    if callable(kname):
        kname = kname(launch)

    traffic = None
    try:
        src = b"".join(open(os.path.join(ROOT, f), "rb").read() for f in PROFILED_TRAFFIC["sources"])
        if (args.workload == "grid8x8" and eng == "butterfly" and S == 1 << 20 and not io16
                and hashlib.sha256(src).hexdigest()[:16] == PROFILED_TRAFFIC["sha256_16"]):
            traffic = PROFILED_TRAFFIC["bytes_per_launch"]
    except OSError:
        pass

    roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
            "traffic_unit": "HBM bytes per launch (rocprofv3, copy-calibrated)",
            "kernel": kname + " (forward)", "engine": eng, "signals_per_tile": list(tiles), "launch": launch,
            "algorithmic_bytes_per_launch": bytes_per_launch, "avg_launch_ms": fwd_ms}
    if flops_per_signal is not None:
        # the binding roofline: MFMA when the leaf products' arithmetic intensity (flop per
        # algorithmic byte) is above the ridge point of their precision, else HBM
        tflops = flops_per_signal * S / (fwd_ms * 1e-3) / 1e12
        peak = MFMA_PEAK_TFLOPS[precision]
        intensity = flops_per_signal / (bytes_per_launch / S)
        ridge = peak * 1e12 / (HBM_PEAK_GBS * 1e9)
        roof.update({"intensity_flop_per_byte": intensity, "ridge_flop_per_byte": ridge,
                     "algorithmic_flops_per_launch": flops_per_signal * S,
                     "mfma_TFLOP_per_s": tflops, "mfma_peak": peak, "mfma_frac": tflops / peak})
        if intensity >= ridge:
            roof.update({"bound": "mfma", "achieved": tflops, "peak": peak, "unit": "TFLOP/s",
                         "frac": tflops / peak, "hbm_GB_per_s": achieved,
                         "hbm_frac": achieved / HBM_PEAK_GBS})
    result = {
        "metric": METRIC,
        "value": 2.0 * S * n / (ms_step * 1e-3), "unit": "coeffs/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": ("f32" if precision == "fp32" else f"f32 haar, {precision} blocks, f32 acc") +
                 (", bf16 storage" if io16 else ""),
        "data": "synthetic",
        "config": dict(workload_cfg, signals=S, n=n, values_per_step=2 * S * n, precision=precision,
                       storage=args.io),
        "roofline": roof,
        "forward_coeffs_per_s": S * n / (fwd_ms * 1e-3),
        "inverse_values_per_s": S * n / (inv_ms * 1e-3), "inverse_avg_launch_ms": inv_ms,
        "copy_reference": {"kernel": "gft_stream_copy (non-temporal 16-byte streaming copy)",
                           "GB_per_s": scopy_gbs, "avg_launch_ms": scopy_ms,
                           "frac_of_peak": scopy_gbs / HBM_PEAK_GBS,
                           "forward_frac_of_copy": achieved / scopy_gbs,
                           "runtime_copy": {"GB_per_s": copy_gbs, "avg_launch_ms": copy_ms,
                                            "forward_frac_of_copy": achieved / copy_gbs}},
    }

    if not args.no_dense:
        # dense GFT as one GEMM on the same GPU, same basis (rows of U = forward(e_i))
        torch.backends.cuda.matmul.allow_tf32 = False
        Ud = torch.from_numpy(plan.basis()).float().to(dev)   # y = x @ Ud, the plan's basis
        dense = {}
        for dt_name, dt in (("fp32", torch.float32), ("bf16", torch.bfloat16)):
            U1 = Ud.to(dt).contiguous()
            U2 = Ud.t().contiguous().to(dt)
            if io16 and dt_name == "fp32":
                continue   # with BF16 storage the comparable dense GEMM is the BF16 one
            xs = [b[0].to(dt) for b in bufs]
            ys = [torch.empty_like(xs[0]) for _ in range(2)]
            xo = torch.empty_like(xs[0])

            def dfwd(i):
                torch.matmul(xs[i & 1], U1, out=ys[i & 1])

            def dinv(i):
                torch.matmul(ys[i & 1], U2, out=xo)

            d_step, d_fwd = run_steps(torch, stream, dfwd, dinv, args.steps, 3)
            dense[dt_name] = {"value": 2.0 * S * n / (d_step * 1e-3), "unit": "coeffs/s",
                              "ms_per_step": d_step, "forward_avg_launch_ms": d_fwd,
                              "impl": f"torch.matmul {dt_name} (hipBLASLt/rocBLAS)" +
                                      (", no TF32" if dt_name == "fp32" else "")}
            del xs, ys, xo
        result["dense_gemm"] = dense
        for k, v in dense.items():
            result[f"speedup_vs_dense_{k}"] = result["value"] / v["value"]

    if not args.no_cpu_baseline:
        # the timed launch's own output: rows of ya, the forward of buffer xa
        fwd(0)
        torch.cuda.synchronize()
        Yg = ya[:sample_rows].double().cpu().numpy()
        Xs = xa[:sample_rows].float().cpu().numpy()          # the values the GPU consumed
        Ug = G.gft_forward(plan, torch.eye(n, device=dev, dtype=xa.dtype)).double().cpu().numpy()
        result["cpu_baseline"] = cpu_baseline([(graph, Xs, Yg, plan.basis(), Ug)], sample_desc)
    print(json.dumps(result), flush=True)


def bench_grid(args):
    import workloads as wl
    S = args.signals or (1 << 20)
    X = wl.ar1_field(S, 8, 8, 0.95, wl.rng_for(2))
    bench_single(args, wl.config2_graph(), X, args.precision or "fp32",
                 {"workload": "grid8x8_ar1_fwd_inv", "graph": "8x8 4-neighbour grid, unit weights",
                  "stages": "LR then UD (2 x 32 Haar units), 4 leaf blocks of 16", "rho": 0.95},
                 1 << 16, "65536 signals of the same AR(1) workload (first rows of the batch)",
                 kernel_names={"butterfly": "gft_butterfly_f32<2,16,0>", "generic": "gft_apply<4,fp32>"})


def bench_skeleton(args):
    import workloads as wl
    seqs = (args.signals // 900) if args.signals else 16384
    X = wl.skeleton_walks_chunked(seqs).reshape(-1, 25)
    bench_single(args, wl.config3_graph(), X, args.precision or "bf16",
                 {"workload": "skeleton25_walks_fwd_inv",
                  "graph": "25-node skeleton: 5-node spine, 4 limbs of 5, unit weights",
                  "stages": "left/right limb swap (10 Haar units), leaf blocks 15 + 5 + 5",
                  "shape": f"[{seqs}, 3, 300, 25]"},
                 8 * 900, "first 8 sequences (7200 signals) of the same skeleton workload",
                 kernel_names={"butterfly": "gft_butterfly_f32<1,16,0> (one-stage layout)",
                               "generic": f"gft_apply<8,{args.precision or 'bf16'}>"})


def _large_workload(args, graph, S, name, desc):
    import paper_1907_07875_amd as G
    import workloads as wl
    X = wl.gaussian(S, graph.n, wl.rng_for(5, 7))
    precision = args.precision or "fp32"
    engine = args.engine if args.engine in ("large", "product", "generic") else "auto"
    plan = G.Plan.from_graph(graph, engine=engine, precision=precision, in_dtype=args.io, out_dtype=args.io)
    plan.prepare()
    st = plan.info()
    eng = plan.engine()
    tuning = plan.tuning()
    if eng == "product" and tuning["variant"] == 0:
        # separable engine, dense factors: two factor GFTs as dense products, 2 n (na + nb)
        import math
        na = int(round(math.sqrt(graph.n)))
        flops = 2.0 * graph.n * (na + graph.n // na)
    elif eng == "product":
        # staged factors: the Kronecker leaves' block products b_a b_b (b_a + b_b) summed,
        # plus the Haar units' add/sub
        flops = 2.0 * (st["separable_mults"] - st["num_z_scalings"]) + 2.0 * st["num_units"]
    else:
        # per signal: 2 flops per block multiply-add, plus the Haar units' add/sub
        flops = 2.0 * (st["mults"] - st["num_z_scalings"]) + 2.0 * st["num_units"]
    bench_single(args, graph, X, precision,
                 {"workload": name, "graph": desc, "stages": st["num_stages"],
                  "leaf_blocks": st["num_blocks"], "max_block": st["max_block"],
                  "kron_leaves": st["num_kron_leaves"], "separable_mults": st["separable_mults"],
                  "launch": tuning,
                  "dense_flops_per_signal": 2.0 * graph.n * graph.n, "fast_flops_per_signal": flops},
                 256, "first 256 signals of the same workload",
                 kernel_names={"large": lambda launch: {
                                   0: "large engine, three passes: permute_stages + block_gemm + permute_stages",
                                   1: "large engine: permute_stages + block_gemm writing the output order",
                                   2: f"gft_onepass<{PREC_ID[precision]}> (large engine, one-pass form)"}
                               .get(launch.get("variant"), "large engine"),
                               "product": "gft_product<64,64> (separable Kronecker leaves)"},
                 flops_per_signal=flops, make_plan=lambda: plan)


def bench_grid64(args):
    import workloads as wl
    if args.engine == "product":
        return bench_grid64_product(args)   # the explicit product plan (gft_plan_product)
    _large_workload(args, wl.config5a_graph(), args.signals or 65536, "grid64x64_fwd_inv",
                    "64x64 grid, LR/UD reversals recursed on the + branch (12 stages)")


def bench_grid64_product(args):
    """The same 64x64 grid planned as the Cartesian product path64 x path64 (each axis with
    its 6 halving reversal stages): separable factor GFTs, y = U_a^T X U_b per signal."""
    import paper_1907_07875_amd as G
    import workloads as wl
    precision = args.precision or "fp32"
    if precision == "fp16" or args.io != "fp32":
        sys.exit("product plans run FP32, BF16 or split BF16 products on FP32 storage")
    S = args.signals or 65536
    axis = wl.path_recursive(64)
    graph = wl.cartesian_product(axis, axis, name="grid64x64")
    X = wl.gaussian(S, graph.n, wl.rng_for(5, 7))
    bench_single(args, graph, X, precision,
                 {"workload": "grid64x64_product_fwd_inv",
                  "graph": "64x64 grid as path64 x path64, halving reversal stages per axis (6 + 6)",
                  "factor_gfts": f"two dense 64x64 factor GFTs per signal (separable), {precision} products",
                  "dense_flops_per_signal": 2.0 * graph.n * graph.n,
                  "fast_flops_per_signal": 2.0 * graph.n * (64 + 64)},
                 256, "first 256 signals of the same workload",
                 kernel_names={"product": "gft_product<64,64,0>"},
                 flops_per_signal=2.0 * graph.n * (64 + 64),
                 make_plan=lambda: G.Plan.from_product(axis, axis, precision=precision, in_dtype=args.io,
                                                       out_dtype=args.io))


def bench_wpath(args):
    import workloads as wl
    _large_workload(args, wl.config5b_graph(), args.signals or 65536, "wpath1024_fwd_inv",
                    "weighted symmetric path, n = 1024, mirrored weights and self-loops")


def bench_mixed(args):
    import numpy as np
    import torch

    import paper_1907_07875_amd as G
    import workloads as wl

    dev = torch.device("cuda:0")
    precision = args.precision or "fp32"
    graphs = wl.config4_graphs(wl.rng_for(4))
    counts = wl.config4_signal_counts(len(graphs), wl.rng_for(4, 1))
    rng = wl.rng_for(4, 2)
    xs = [wl.gaussian(int(s), g.n, rng) for g, s in zip(graphs, counts)]
    flat = np.concatenate([x.reshape(-1) for x in xs])
    off = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    E = flat.size
    plan = G.gft_plan_batch(graphs, precision=precision)
    plan.prepare()
    launch = plan.tuning()
    xa = torch.from_numpy(flat).to(dev)
    xb = torch.roll(xa, shifts=1).contiguous()
    ya, yb, xr = torch.empty_like(xa), torch.empty_like(xa), torch.empty_like(xa)
    offs = torch.from_numpy(off).to(dev)
    stream = torch.cuda.current_stream()
    lib, h, sp = G.load_library(), plan.handle, _c(int(stream.cuda_stream))
    bufs = [(xa, ya), (xb, yb)]
    P = {id(t): _c(t.data_ptr()) for t in (xa, xb, ya, yb, xr, offs)}

    def fwd(i):
        x, y = bufs[i & 1]
        st = lib.gft_forward_batch(h, P[id(x)], P[id(y)], P[id(offs)], E, sp)
        if st:
            G._check(st)

    def inv(i):
        st = lib.gft_inverse_batch(h, P[id(bufs[i & 1][1])], P[id(xr)], P[id(offs)], E, sp)
        if st:
            G._check(st)

    ms_step, fwd_ms = run_steps(torch, stream, fwd, inv, args.steps, args.warmup)
    bytes_per_launch = 2.0 * E * 4
    achieved = bytes_per_launch / (fwd_ms * 1e-3) / 1e9
    result = {
        "metric": METRIC, "value": 2.0 * E / (ms_step * 1e-3), "unit": "coeffs/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32" if precision == "fp32" else f"f32 io, {precision} blocks",
        "data": "synthetic",
        "config": {"workload": "mixed_batch_fwd_inv", "graphs": len(graphs),
                   "families": "paths 4..64, cycles 8..64, grids 4x4..16x16, bipartite 16..128",
                   "signals": int(counts.sum()), "elements": int(E), "precision": precision},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": f"gft_apply_batch<{precision}> (forward)", "launch": launch,
                     "algorithmic_bytes_per_launch": bytes_per_launch, "avg_launch_ms": fwd_ms},
    }
    if not args.no_dense:
        # the same batch as one dense GEMM launch per graph (FP32, same bases)
        torch.backends.cuda.matmul.allow_tf32 = False
        Us = [G.gft_forward(G.Plan.from_graph(g), torch.eye(g.n, device=dev)) for g in graphs]
        pos = np.concatenate([[0], np.cumsum(counts * np.array([g.n for g in graphs]))])
        views = [(xa[pos[i]:pos[i + 1]].view(-1, g.n), ya[pos[i]:pos[i + 1]].view(-1, g.n))
                 for i, g in enumerate(graphs)]

        def dfwd(i):
            for (xv, yv), U in zip(views, Us):
                if xv.shape[0]:
                    torch.matmul(xv, U, out=yv)

        d_step, _ = run_steps(torch, stream, dfwd, dfwd, args.steps, 2)
        result["dense_gemm"] = {"value": 2.0 * E / (d_step * 1e-3), "unit": "coeffs/s",
                                "ms_per_step": d_step,
                                "impl": f"torch.matmul FP32, one launch per graph ({len(graphs)} per direction)"}
    if not args.no_cpu_baseline:
        # the timed batch launch's own output (forward of buffer xa into ya), sliced per graph;
        # each graph's applied basis from a batch launch on the unit vectors
        fwd(0)
        torch.cuda.synchronize()
        pos = np.concatenate([[0], np.cumsum(counts * np.array([g.n for g in graphs]))])
        samples = []
        for i in (0, 60, 118, 125, 140):
            g = graphs[i]
            s = min(int(counts[i]), 4096)
            Xs = xs[i][:s]
            Yg = ya[pos[i]:pos[i] + s * g.n].view(s, g.n).double().cpu().numpy()
            ecounts = np.zeros(len(graphs), dtype=np.int64)
            ecounts[i] = g.n
            eoff = torch.from_numpy(np.concatenate([[0], np.cumsum(ecounts)]).astype(np.int64)).to(dev)
            Ug = G.gft_forward_batch(plan, torch.eye(g.n, device=dev).reshape(-1), eoff)
            samples.append((g, Xs, Yg, plan.basis(i), Ug.view(g.n, g.n).double().cpu().numpy()))
        result["cpu_baseline"] = cpu_baseline(
            samples, "5 graphs of the batch (path, cycle, grid, 2 bipartite), up to 4096 signals "
                     "each, GPU values from the timed batch launch")
    print(json.dumps(result), flush=True)


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU: every signal is "
                          "independent, so N GPUs would each run this same kernel on 1/N of the "
                          "batch with no exchange; runs on more than one GPU are not supported"}))
        sys.exit(2)
    {"grid8x8": bench_grid, "skeleton": bench_skeleton, "mixed": bench_mixed,
     "grid64": bench_grid64, "wpath1024": bench_wpath}[args.workload](args)


if __name__ == "__main__":
    main()
