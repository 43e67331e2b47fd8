"""Headline benchmark: effective GFLOPS (2MNK / wall-clock) of FP32 Winograd
on MFMA leaves vs the plain MFMA SGEMM, square n = 19456, operands in pinned
host memory so that the wall-clock includes the host<->device transfers (the
paper measures GFLOPS as 2N^3 over wall-clock with transfers included,
Section 4).

One step = one synchronous fastmm_gemm call: stage A, B in, pre-additions,
grouped leaf products, post-additions, C out.  Inputs are seeded synthetic
(uniform on the 2^-23 grid of [-1, 1)).  Prints one JSON line.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--n N] [--depth D]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "effective GFLOPS (2MNK/wall-clock) n=19456 FP32 Winograd vs plain MFMA SGEMM"
PEAK_FP32_TFLOPS = 157.3   # MI355X dense FP32 matrix peak
PEAK_HBM_GBS = 8000.0
# HBM bytes per leaf launch (pipelined depth-3 call: 14 launches of 49 leaves
# of 1280 or 1152 x 2432 x 2432) from the FETCH_SIZE and WRITE_SIZE counter
# runs, each scaled by its reading for a 1 GiB calibration copy (fetch x2.000,
# write x1.000); see profiles/leaf_gemm_n19456_d3_pinned_hbm_traffic.md.
# Valid for leaf_gemm_kernel<128,128,16,2,2> in that configuration only.
TRAFFIC_BYTES_PER_LAUNCH = 2669524.3 * 1024 * 2.000 + 576963.6 * 1024 * 1.000


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def time_calls(fn, steps, warmup):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    times = []
    t0 = time.perf_counter()
    for _ in range(steps):
        a = time.perf_counter()
        fn()
        times.append(time.perf_counter() - a)
    torch.cuda.synchronize()
    return time.perf_counter() - t0, times


def batched_context(fastmm, torch):
    """256 independent products with M, N, K log-uniform in [256, 6144]
    (multiples of 64), device-resident, uniform[-1, 1) inputs: one
    fastmm_gemm_batched call (each problem's plan from the default rule;
    replayed from its HIP graph after the first call) against the same
    products issued one fastmm_gemm call at a time, and against the batched
    plain product (depth 0)."""
    import synthgen
    shapes = synthgen.shapes_loguniform(3001, 256, lo=256, hi=6144)
    g = torch.Generator(device="cuda")
    g.manual_seed(5001)
    As, Bs, Cs = [], [], []
    for m, n, k in shapes.tolist():
        As.append(torch.rand((m, k), device="cuda", generator=g) * 2 - 1)
        Bs.append(torch.rand((k, n), device="cuda", generator=g) * 2 - 1)
        Cs.append(torch.empty((m, n), device="cuda"))
    flops = float(sum(2.0 * m * n * k for m, n, k in shapes.tolist()))
    fastmm.set_plan_mode(fastmm.PLAN_DEFAULT)

    def timed(fn, reps):
        fn()
        torch.cuda.synchronize()
        best = 1e30
        for _ in range(reps):
            t = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            best = min(best, time.perf_counter() - t)
        return best

    t_b = timed(lambda: fastmm.gemm_batched(As, Bs, Cs), 3)
    st = fastmm.get_stats()
    t_plain = timed(lambda: fastmm.gemm_batched(As, Bs, Cs, depth=[0] * len(As)), 3)

    def singles():
        for (m, n, k), A, B, C in zip(shapes.tolist(), As, Bs, Cs):
            fastmm.gemm(m, n, k, A, B, C, depth=-1)
    t_s = timed(singles, 1)
    return {"problems": len(As), "flops": flops, "ms": 1e3 * t_b, "TFLOPS": flops / t_b / 1e12,
            "graph_replayed": st["graph_replayed"], "launches": st["launches"],
            "plain_batched_ms": 1e3 * t_plain, "plain_batched_TFLOPS": flops / t_plain / 1e12,
            "single_calls_ms": 1e3 * t_s, "single_calls_TFLOPS": flops / t_s / 1e12}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=19456)
    ap.add_argument("--depth", type=int, default=-1, help="-1: pick the best of 2, 3, 4")
    ap.add_argument("--leaf", type=int, default=1024)
    ap.add_argument("--tile", type=int, default=0)
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-device-context", action="store_true")
    ap.add_argument("--no-shards", action="store_true",
                    help="skip one GPU's share of the sharded product")
    ap.add_argument("--no-batched", action="store_true",
                    help="skip the 256-problem batched context (uneven shapes)")
    ap.add_argument("--resident", action="store_true",
                    help="operands in device memory (no transfers): profiling the device path")
    ap.add_argument("--traffic-probe", action="store_true",
                    help="first run one plain 1 GiB device copy (calibrates HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; the sharded "
                                   "multi-GPU path is a design note, not built"}))
        sys.exit(2)

    import numpy as np
    import torch

    import synthgen
    from paper_1205_2927_amd import fastmm

    fastmm.load()
    if args.traffic_probe:
        src = torch.empty(1 << 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        torch.cuda.empty_cache()
    n = args.n
    M = N = K = n
    log(f"bench: n={n} allocating pinned host operands")
    A = torch.empty((M, K), dtype=torch.float32, pin_memory=True)
    B = torch.empty((K, N), dtype=torch.float32, pin_memory=True)
    C = torch.empty((M, N), dtype=torch.float32, pin_memory=True)
    synthgen.build() if synthgen._load() is None else None
    synthgen.fill_uniform_pm1(1001 + 3, M, K, A.data_ptr())
    synthgen.fill_uniform_pm1(2001 + 3, K, N, B.data_ptr())
    flops = 2.0 * M * N * K
    if args.resident:
        # Device-path profiling: the same inputs, resident in HBM.
        A, B = A.to("cuda"), B.to("cuda")
        C = torch.empty((M, N), dtype=torch.float32, device="cuda")

    fastmm.set_profiling(True)

    def run(depth, tile=args.tile, leaf=args.leaf):
        return lambda: fastmm.gemm(M, N, K, A, B, C, depth=depth, leaf=leaf, tile=tile)

    # Plain MFMA SGEMM (depth 0), same staging path.
    plain = None
    if not args.no_plain:
        log("bench: plain SGEMM (depth 0)")
        tot, ts = time_calls(run(0), args.steps, args.warmup)
        st = fastmm.get_stats()
        plain = {"ms_per_step": 1e3 * tot / args.steps, "value": flops / (tot / args.steps) / 1e9,
                 "leaf_ms": st["leaf_ms"], "h2d_span_ms": st["h2d_ms"],
                 "leaf_tflops": st["leaf_flops"] / (st["leaf_ms"] * 1e-3) / 1e12}
        log(f"  plain: {plain}")

    depths = [args.depth] if args.depth >= 0 else [2, 3, 4]
    probe = {}
    if len(depths) > 1:
        for d in depths:
            tot, ts = time_calls(run(d), 2, 1)
            probe[d] = min(ts)
            log(f"  probe depth {d}: {1e3 * probe[d]:.1f} ms")
        best = min(probe, key=probe.get)
    else:
        best = depths[0]
    log(f"bench: Winograd depth {best}, {args.steps} timed steps")
    leaf_ms, h2d_ms = [], []

    def step():
        fastmm.gemm(M, N, K, A, B, C, depth=best, leaf=args.leaf, tile=args.tile)
        s = fastmm.get_stats()
        leaf_ms.append(s["leaf_ms"])
        h2d_ms.append(s["h2d_ms"])

    for _ in range(args.warmup):
        step()
    leaf_ms.clear()
    h2d_ms.clear()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    st = fastmm.get_stats()
    ms_per_step = 1e3 * elapsed / args.steps
    value = flops / (elapsed / args.steps) / 1e9

    # Parity of the last result: sampled rows + Freivalds against the oracle
    # (the oracle is the checker; the timed path never touches it).
    from oracle import checks
    An = A.cpu().numpy()
    Bn = B.cpu().numpy()
    Cn = C.cpu().numpy()
    rows = synthgen.row_sample(7004, M, 8)
    parity = {"sampled_rows_rel": checks.sampled_rows_rel(Cn, An, Bn, rows),
              "freivalds_rel": checks.freivalds_rel(Cn, An, Bn, synthgen.signs_pm1(7005, N)),
              "rows": int(rows.size), "tolerance": 1e-4}
    log(f"bench: parity {parity}")

    # One GPU's share of the column-panel sharding (the paper's two-device
    # split, eqs. (3)-(4), generalised): 1 x 8 panels (19456 x 19456 x 2432)
    # and a 2 x 4 grid (9728 x 19456 x 4864), staged from the same pinned
    # host operands (strided views), as many levels as the leaf cutoff allows.
    shards = None
    if n == 19456 and not args.resident and not args.no_shards:
        shards = {}
        for name, (sm, sn) in {"panel_1x8": (M, N // 8), "grid_2x4": (M // 2, N // 4)}.items():
            fn = lambda: fastmm.gemm(sm, sn, K, A[:sm], B[:, :sn], C[:sm, :sn], depth=16,
                                     leaf=args.leaf)
            tot, ts = time_calls(fn, 3, 1)
            sst = fastmm.get_stats()
            shards[name] = {"M": sm, "N": sn, "K": K, "depth": sst["depth"], "ms": 1e3 * min(ts),
                            "effective_GFLOPS": 2.0 * sm * sn * K / min(ts) / 1e9}
        log(f"bench: shard shapes {shards}")

    # Dominant kernel: the grouped leaf GEMM.  Its launches are timed with
    # HIP events recorded by the library on the stream it launches them on.
    n_launch = max(1, st["leaf_launches"])
    leaf_sum = float(np.mean(leaf_ms))          # ms per step, all leaf launches
    avg_launch = leaf_sum / n_launch
    flops_launch = st["leaf_flops"] / n_launch
    leaf_tflops = flops_launch / (avg_launch * 1e-3) / 1e12
    roofline = {"bound": "mfma", "kernel": "leaf_gemm_kernel<128,128,16,2,2> (grouped leaves)",
                "achieved": leaf_tflops, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                "frac": leaf_tflops / PEAK_FP32_TFLOPS,
                "traffic": TRAFFIC_BYTES_PER_LAUNCH if (best == 3 and n == 19456 and args.tile == 0
                                                        and args.leaf == 1024) else None,
                "flops_per_launch": flops_launch, "avg_launch_ms": avg_launch,
                "launches_per_step": n_launch}

    # Context: the same product with device-resident operands (level-wise
    # path, no transfers), with the addition kernels timed separately.
    dev_ctx = None
    if not args.no_device_context and not args.resident:
        dA = A.to("cuda")
        dB = B.to("cuda")
        dC = torch.empty((M, N), dtype=torch.float32, device="cuda")
        fastmm.gemm(M, N, K, dA, dB, dC, depth=best, leaf=args.leaf, tile=args.tile)
        ts = []
        for _ in range(2):
            torch.cuda.synchronize()
            t = time.perf_counter()
            fastmm.gemm(M, N, K, dA, dB, dC, depth=best, leaf=args.leaf, tile=args.tile)
            ts.append(time.perf_counter() - t)
        sd = fastmm.get_stats()
        add_ms = sd["preadd_ms"] + sd["postadd_ms"]
        dev_ctx = {"ms": 1e3 * min(ts), "effective_GFLOPS": flops / min(ts) / 1e9,
                   "leaf_ms": sd["leaf_ms"],
                   "leaf_TFLOPs": sd["leaf_flops"] / (sd["leaf_ms"] * 1e-3) / 1e12,
                   "preadd_ms": sd["preadd_ms"], "postadd_ms": sd["postadd_ms"],
                   "add_bytes": sd["add_bytes"],
                   "add_GBps": sd["add_bytes"] / (add_ms * 1e-3) / 1e9 if add_ms > 0 else None,
                   "add_frac_of_hbm_peak": (sd["add_bytes"] / (add_ms * 1e-3) / 1e9 / PEAK_HBM_GBS)
                   if add_ms > 0 else None}
        # The paper's own algorithm: the classic eight-product recursion of
        # Table 1 with its recursion point (leaves below 6016, i.e. leaf
        # cutoff 3008), MFMA leaves, same operands.
        fastmm.rmul(M, N, K, dA, dB, dC, depth=8, leaf=3008)
        torch.cuda.synchronize()
        t = time.perf_counter()
        fastmm.rmul(M, N, K, dA, dB, dC, depth=8, leaf=3008)
        torch.cuda.synchronize()
        t = time.perf_counter() - t
        dev_ctx["classic_recursion"] = {"ms": 1e3 * t, "effective_GFLOPS": flops / t / 1e9,
                                        "depth": fastmm.get_stats()["depth"], "leaf": 3008}
        del dA, dB, dC
        torch.cuda.empty_cache()
        log(f"bench: device-resident context {dev_ctx}")
    batched = None
    if not args.no_batched and not args.resident:
        batched = batched_context(fastmm, torch)
        log(f"bench: batched context {batched}")
    phases = {"h2d_span_ms": float(np.mean(h2d_ms)), "leaf_ms": leaf_sum,
              "add_bytes": st["add_bytes"], "transfer_bytes": st["transfer_bytes"]}

    cpu = None
    if not args.no_cpu:
        from oracle import classic
        threads = classic.num_threads()
        rows_c = synthgen.row_sample(7006, M, 32)
        t = time.perf_counter()
        classic.gemm_rows(An, Bn, rows_c)
        per_row = (time.perf_counter() - t) / rows_c.size
        R = int(max(4, min(4096, args.cpu_seconds / max(per_row, 1e-6))))
        rows_c = synthgen.row_sample(7007, M, R)
        t = time.perf_counter()
        classic.gemm_rows(An, Bn, rows_c)
        dt = time.perf_counter() - t
        cpu = {"value": 2.0 * rows_c.size * N * K / dt / 1e9, "unit": "GFLOPS", "cores": threads,
               "kind": "oracle",
               "sample": f"{rows_c.size} seeded rows of C (FP64-accumulated triple loop, "
                         f"OpenMP over rows), {dt:.1f} s"}
        log(f"bench: cpu {cpu}")

    out = {
        "metric": METRIC, "value": value, "unit": "GFLOPS", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"FP32 Winograd-Strassen C=A*B, square n={n}, "
                               + ("device-resident operands" if args.resident else
                                  "pinned host in/out (transfers timed)")
                               + f", depth {st['depth']}, leaf {args.leaf}",
                   "M": M, "N": N, "K": K, "depth": st["depth"], "leaf": args.leaf,
                   "tile": args.tile, "parallelism": "single GPU"},
        "roofline": roofline, "cpu_baseline": cpu,
        "plain_sgemm": plain,
        "speedup_vs_plain": (plain["ms_per_step"] / ms_per_step) if plain else None,
        "depth_probe_ms": {str(k): 1e3 * v for k, v in probe.items()},
        "phases": phases, "device_resident": dev_ctx, "batched": batched, "shards": shards, "parity": parity,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
