"""Headline benchmark: effective GFLOPS (2MNK / wall-clock) of FP32 Winograd
on MFMA leaves vs the plain MFMA SGEMM, square n = 19456.

One step = one synchronous fastmm_gemm call with A, B and C in pinned host
memory: the wall-clock includes the host->device transfers of A and B, the
recursion (pre-additions, grouped leaf products, post-additions) and the
device->host transfer of C, as the paper measures GFLOPS (2N^3 over
wall-clock with transfers included, Section 4).  The plain SGEMM (depth 0)
runs on the same path as the comparator.  The same product with the operands
already resident in HBM is reported beside it (`hbm_resident`).  Inputs are
seeded synthetic (uniform on the 2^-23 grid of [-1, 1)).  Prints one JSON
line.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--n N] [--depth D]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "effective GFLOPS (2MNK/wall-clock) n=19456 FP32 Winograd vs plain MFMA SGEMM"
PEAK_FP32_TFLOPS = 157.3   # MI355X dense FP32 matrix peak
PEAK_16BIT_TFLOPS = 2500.0  # MI355X dense BF16 / FP16 matrix peak
# --tile 8 / 9 time a split-precision form instead of the FP32 leaf: three
# 16-bit products per FP32 product, so its FP32-equivalent ceiling is a third
# of the 16-bit peak; its leaf phase is a pack pass (and for FP16 a scale
# pass) plus the leaf kernel.
SPLIT_FORMS = {8: ("bf16x3", "leaf_pack_kernel<0> + leaf_packed_kernel<0,256,256,4,4>"),
               9: ("fp16x3", "leaf_scale_kernel + leaf_pack_kernel<1> + leaf_packed_kernel<1,256,256,4,4>")}
PEAK_HBM_GBS = 8000.0
# HBM bytes per leaf launch from the FETCH_SIZE and WRITE_SIZE counter runs,
# each scaled by its reading for a 1 GiB calibration copy (fetch x2.000,
# write x1.000).  HBM-resident depth-3 call: one grouped launch of 343 leaves
# of 2432 x 2432 x 2432 (profiles/leaf_gemm_n19456_d3_device_hbm_traffic.md).
# Pinned-host depth-3 call: 56 launches of 49 leaves of (640 | 512) x 2432
# x (1280 | 1152), mean per launch
# (profiles/leaf_gemm_n19456_d3_pinned_hbm_traffic.md).  Valid for
# leaf_gemm_kernel<128,128,16,2,2> in those configurations only.
TRAFFIC_DEVICE_BYTES_PER_LAUNCH = 37626398.4 * 1024 * 2.000 + 7924672.0 * 1024 * 1.000
TRAFFIC_PINNED_BYTES_PER_LAUNCH = 674390.6 * 1024 * 2.000 + 142322.4 * 1024 * 1.000


def cpu_model():
    """The host CPU's model name (the oracle's cores are reported with it)."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


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


def batched_context(fastmm, torch, with_planner=True):
    """The 256-problem batched workload: M, N, K log-uniform in [256, 6144]
    (multiples of 64, shape seed 3001), seeded uniform[-1, 1) operands,
    device-resident, one fastmm_gemm_batched call (replayed from its HIP
    graph after the first).  Timed with the plans of each planner mode --
    DEFAULT (fixed rule), MODEL (the cost model, trained first on the
    exhaustive timings of 160 shapes of seed 4001) and EXHAUSTIVE (every
    candidate of every shape timed) -- against the batched plain product
    (depth 0) and the same products as 256 single fastmm_gemm calls; the
    timed calls of the modes and the plain product alternate.  The result of
    each mode is checked against the oracle (2 sampled rows and Freivalds'
    check per problem)."""
    import synthgen
    from oracle import checks
    shapes = [tuple(int(v) for v in x) for x in synthgen.shapes_loguniform(3001, 256, lo=256, hi=6144)]
    hA, hB, As, Bs, Cs = [], [], [], [], []
    for i, (m, n, k) in enumerate(shapes):
        sa, sb = synthgen.batch_seeds(5, i)
        hA.append(synthgen.uniform_pm1(sa, m, k))
        hB.append(synthgen.uniform_pm1(sb, k, n))
        As.append(torch.from_numpy(hA[-1]).to("cuda"))
        Bs.append(torch.from_numpy(hB[-1]).to("cuda"))
        Cs.append(torch.empty((m, n), device="cuda"))
    flops = float(sum(2.0 * m * n * k for m, n, k in shapes))
    # No per-phase timing events here: they cost about 4 us each per call,
    # which the 256 single calls would otherwise pay.
    fastmm.set_profiling(False)

    def timed(fn, reps):
        fn()
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            t = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t)
        return float(np.median(ts)), min(ts)

    def parity():
        worst = 0.0
        for i, (m, n, k) in enumerate(shapes):
            C = Cs[i].cpu().numpy()
            rows = synthgen.row_sample(7100 + i, m, 2)
            worst = max(worst, checks.sampled_rows_rel(C, hA[i], hB[i], rows),
                        checks.freivalds_rel(C, hA[i], hB[i], synthgen.signs_pm1(7400 + i, n)))
        return worst

    out = {"problems": len(shapes), "flops": flops, "modes": {}}
    modes = [("default", fastmm.PLAN_DEFAULT)]
    if with_planner:
        log("bench: batched: timing the planner's training shapes, training the cost model")
        t = time.perf_counter()
        for (M, N, K) in synthgen.shapes_loguniform(4001, 160):
            fastmm.plan(int(M), int(N), int(K), fastmm.PLAN_EXHAUSTIVE)
        loss = fastmm.planner_train(epochs=400, batch=64, lr=3e-3, seed=4001)
        out["model_training"] = {"shapes": 160, "records": fastmm.planner_records(),
                                 "loss": loss, "seconds": time.perf_counter() - t}
        modes += [("model", fastmm.PLAN_MODEL), ("exhaustive", fastmm.PLAN_EXHAUSTIVE)]
    # Each mode's first call plans (EXHAUSTIVE times every candidate) and
    # captures its graph; its result is checked against the oracle.  The
    # timed calls then go round the modes and the batched plain product in
    # turn, eleven rounds, so that the clock's drift over the run weighs on
    # all of them alike.
    # The calls go through fastmm.Batch, which builds the argument arrays
    # once (a serving loop's binding): building them for 256 problems costs
    # about a millisecond of Python per call.
    run = fastmm.Batch(As, Bs, Cs)
    plain_fn = fastmm.Batch(As, Bs, Cs, depth=[0] * len(As))
    for name, code in modes:
        fastmm.set_plan_mode(code)
        t = time.perf_counter()
        run()
        first = time.perf_counter() - t
        run()
        torch.cuda.synchronize()
        st = fastmm.get_stats()
        out["modes"][name] = {"first_call_s": first, "max_depth": st["depth"], "leaves": st["leaves"],
                              "leaf_launches": st["leaf_launches"], "launches": st["launches"],
                              "graph_replayed": st["graph_replayed"], "parity_worst_rel": parity()}
    fastmm.set_plan_mode(fastmm.PLAN_DEFAULT)
    plain_fn()
    plain_fn()
    torch.cuda.synchronize()
    out["plain_batched"] = {"parity_worst_rel": parity()}
    ts = {name: [] for name, _ in modes}
    ts["plain"] = []
    for _ in range(11):
        for name, code in modes + [("plain", None)]:
            if code is not None:
                fastmm.set_plan_mode(code)
            torch.cuda.synchronize()
            t = time.perf_counter()
            (plain_fn if code is None else run)()
            torch.cuda.synchronize()
            ts[name].append(time.perf_counter() - t)
    fastmm.set_plan_mode(fastmm.PLAN_DEFAULT)
    for name, _ in modes:
        med = float(np.median(ts[name]))
        out["modes"][name].update({"ms": 1e3 * med, "ms_min": 1e3 * min(ts[name]),
                                   "TFLOPS": flops / med / 1e12})
    med = float(np.median(ts["plain"]))
    out["plain_batched"].update({"ms": 1e3 * med, "TFLOPS": flops / med / 1e12})
    if with_planner:
        out["model_regret_vs_exhaustive"] = out["modes"]["model"]["ms"] / out["modes"]["exhaustive"]["ms"] - 1
        out["model_gain_vs_default"] = out["modes"]["default"]["ms"] / out["modes"]["model"]["ms"]

    def singles():
        for (m, n, k), A, B, C in zip(shapes, As, Bs, Cs):
            fastmm.gemm(m, n, k, A, B, C, depth=-1)
    med, best = timed(singles, 1)
    out["single_calls"] = {"ms": 1e3 * med, "TFLOPS": flops / med / 1e12}
    out["tolerance"] = 1e-4
    fastmm.set_profiling(True)
    return out


def hbm_probe(torch):
    """Practical HBM ceilings on this device, from the vendor's own kernels
    (torch's copy, fill, sum and add on 1 GiB float32 buffers), each the
    best of 10 launches timed with events on torch's stream: the roofs the
    addition kernels (streams of reads and writes) are compared with."""
    n = 1 << 28
    a = torch.ones(n, device="cuda")
    b = torch.ones(n, device="cuda")
    c = torch.empty(n, device="cuda")
    cases = {"copy (1 read + 1 write)": (lambda: c.copy_(a), 8.0 * n),
             "fill (1 write)": (lambda: c.fill_(1.0), 4.0 * n),
             "sum (1 read)": (lambda: a.sum(), 4.0 * n),
             "add (2 reads + 1 write)": (lambda: torch.add(a, b, out=c), 12.0 * n)}
    for name, (fn, nbytes) in cases.items():
        fn()
        torch.cuda.synchronize()
        best = 1e30
        for _ in range(10):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            e1.synchronize()
            best = min(best, e0.elapsed_time(e1))
        print(json.dumps({"hbm_probe": name, "ms": best, "GBps": nbytes / (best * 1e-3) / 1e9,
                          "frac_of_peak": nbytes / (best * 1e-3) / 1e9 / PEAK_HBM_GBS}), flush=True)


def sweep(fastmm, torch, sizes):
    """Dense n-sweep, device-resident, one JSON line per n: the plain MFMA
    SGEMM, Winograd at the planner's default depth, and the paper's classic
    eight-product recursion with its stop rule (recurse while the half is at
    least 3008), the comparison behind the paper's saw-tooth curve of the
    classic recursion (Section 4)."""
    for n in sizes:
        A = torch.empty((n, n), device="cuda").uniform_(-1, 1)
        B = torch.empty((n, n), device="cuda").uniform_(-1, 1)
        C = torch.empty((n, n), device="cuda")
        flops = 2.0 * n ** 3
        row = {"sweep_n": n}
        for name, fn in (("plain", lambda: fastmm.gemm(n, n, n, A, B, C, depth=0)),
                         ("winograd", lambda: fastmm.gemm(n, n, n, A, B, C, depth=-1)),
                         ("classic", lambda: fastmm.rmul(n, n, n, A, B, C, depth=16, leaf=3008))):
            tot, ts = time_calls(fn, 3, 1)
            row[name + "_ms"] = 1e3 * min(ts)
            row[name + "_GFLOPS"] = flops / min(ts) / 1e9
            row[name + "_depth"] = fastmm.get_stats()["depth"]
        print(json.dumps(row), flush=True)
        del A, B, C


def sweep_pinned(fastmm, torch, sizes):
    """n-sweep of the paper's own measurement: A, B, C in pinned host
    memory, the transfers inside the wall-clock (Section 4), one JSON line
    per n: the plain MFMA SGEMM (depth 0) and Winograd at the fixed rule's
    depth, both through the pipelined host path, and the depth an automatic
    call with host operands takes.  The whole of each buffer is used a few
    times first (the first device-to-host copies into freshly pinned memory
    run at about half rate for a while); then the two are timed alternately,
    the median of 5 calls each."""
    nmax = max(sizes)
    buf = [torch.empty(nmax * nmax, dtype=torch.float32, pin_memory=True) for _ in range(3)]
    buf[0].uniform_(-1, 1)
    buf[1].uniform_(-1, 1)
    A, B, C = (x.view(nmax, nmax) for x in buf)
    for _ in range(8):
        for d in (0, 3):
            fastmm.gemm(nmax, nmax, nmax, A, B, C, depth=d, leaf=1)
    for n in sizes:
        A, B, C = (x[:n * n].view(n, n) for x in buf)
        flops = 2.0 * n ** 3
        row = {"sweep_pinned_n": n}
        pl = fastmm.plan(n, n, n, fastmm.PLAN_DEFAULT)
        runs = {"plain": (0, 1), "winograd": (pl.depth, pl.leaf)}
        ts = {k: [] for k in runs}
        for k, (d, lf) in runs.items():
            fastmm.gemm(n, n, n, A, B, C, depth=d, leaf=lf)
        for _ in range(5):
            for k, (d, lf) in runs.items():
                torch.cuda.synchronize()
                t = time.perf_counter()
                fastmm.gemm(n, n, n, A, B, C, depth=d, leaf=lf)
                ts[k].append(time.perf_counter() - t)
                row[k + "_depth"] = fastmm.get_stats()["depth"]
        for k in runs:
            t = float(np.median(ts[k]))
            row[k + "_ms"] = 1e3 * t
            row[k + "_GFLOPS"] = flops / t / 1e9
        row["speedup"] = row["plain_ms"] / row["winograd_ms"]
        fastmm.gemm(n, n, n, A, B, C, depth=fastmm.AUTO)
        row["auto_depth"] = fastmm.get_stats()["depth"]
        print(json.dumps(row), flush=True)


def precision_config(fastmm, torch):
    """The precision forms' own workload: n = 8192 and 16384, depth 2,
    inputs uniform[-1, 1] and log-uniform magnitudes 2^-8..2^8 with random
    signs; the FP32 leaf, split-BF16 and scaled split-FP16 leaves on the same
    operands (in HBM), each timed (best of 3) and checked against the oracle
    on sampled rows.  One JSON line per (n, distribution, leaf form)."""
    import synthgen
    from oracle import checks
    fastmm.set_profiling(True)  # leaf-phase times from the library's HIP events
    for n in (8192, 16384):
        for dist in ("uniform", "loguniform"):
            hA = torch.empty((n, n), dtype=torch.float32, pin_memory=True)
            hB = torch.empty((n, n), dtype=torch.float32, pin_memory=True)
            fill = synthgen.fill_uniform_pm1 if dist == "uniform" else synthgen.fill_loguniform
            fill(1001 + 4, n, n, hA.data_ptr())
            fill(2001 + 4, n, n, hB.data_ptr())
            A, B = hA.to("cuda"), hB.to("cuda")
            C = torch.empty((n, n), device="cuda")
            rows = synthgen.row_sample(7008, n, 8)
            for name, tile in (("fp32", 0), ("bf16x3", 8), ("fp16x3", 9)):
                fn = lambda: fastmm.gemm(n, n, n, A, B, C, depth=2, leaf=1, tile=tile)
                tot, ts = time_calls(fn, 3, 1)
                st = fastmm.get_stats()
                err = checks.sampled_rows_rel(C.cpu().numpy(), hA.numpy(), hB.numpy(), rows)
                leaf_tf = st["leaf_flops"] / (st["leaf_ms"] * 1e-3) / 1e12
                peak = PEAK_FP32_TFLOPS if tile == 0 else PEAK_16BIT_TFLOPS / 3
                print(json.dumps({"precision_n": n, "dist": dist, "leaf_form": name, "depth": 2,
                                  "ms": 1e3 * min(ts), "effective_GFLOPS": 2.0 * n ** 3 / min(ts) / 1e9,
                                  "leaf_TFLOPs_fp32_equivalent": leaf_tf,
                                  "leaf_frac_of_roofline": leaf_tf / peak,
                                  "sampled_rows_rel": err}), flush=True)
            del A, B, C, hA, hB


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
    ap.add_argument("--operands", choices=["pinned", "device"], default="pinned",
                    help="where A, B, C live in the timed loop: pinned host memory (transfers "
                         "timed, the headline) or HBM")
    ap.add_argument("--no-device-context", action="store_true",
                    help="skip the HBM-resident, classic-recursion and precision-form context")
    ap.add_argument("--no-shards", action="store_true",
                    help="skip one GPU's share of the sharded product")
    ap.add_argument("--no-rect", action="store_true",
                    help="skip the rectangular 19456 x 16384 x 12288 context block")
    ap.add_argument("--no-batched", action="store_true",
                    help="skip the 256-problem batched context (uneven shapes)")
    ap.add_argument("--no-planner", action="store_true",
                    help="batched context with the fixed rule only (no cost-model training)")
    ap.add_argument("--traffic-probe", action="store_true",
                    help="first run one plain 1 GiB device copy (calibrates HBM counters)")
    ap.add_argument("--precision-config", action="store_true",
                    help="instead of the headline: the precision forms at n = 8192 and 16384, "
                         "depth 2, uniform and log-uniform inputs, one JSON line each")
    ap.add_argument("--hbm-probe", action="store_true",
                    help="instead of the headline: practical HBM ceilings (torch copy, fill, sum, add "
                         "on 1 GiB), one JSON line each")
    ap.add_argument("--sweep", action="store_true",
                    help="instead of the headline: n-sweep of plain, Winograd and the classic "
                         "recursion, one JSON line per n")
    ap.add_argument("--sweep-pinned", action="store_true",
                    help="instead of the headline: n-sweep of plain and Winograd with A, B, C in "
                         "pinned host memory (transfers timed), one JSON line per n")
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
    if args.hbm_probe:
        hbm_probe(torch)
        return
    if args.precision_config:
        precision_config(fastmm, torch)
        return
    if args.sweep:
        sizes = sorted(set(range(2048, 19457, 512)) | {6004, 6015, 6016, 10004, 12031, 12032, 14004})
        sweep(fastmm, torch, sizes)
        return
    if args.sweep_pinned:
        sweep_pinned(fastmm, torch, list(range(2048, 19457, 1024)))
        return
    if args.traffic_probe:
        src = torch.empty(1 << 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        torch.cuda.empty_cache()
    n = args.n
    M = N = K = n
    on_device = args.operands == "device"
    log(f"bench: n={n} generating operands (pinned host)")
    hA = torch.empty((M, K), dtype=torch.float32, pin_memory=True)
    hB = torch.empty((K, N), dtype=torch.float32, pin_memory=True)
    hC = torch.empty((M, N), dtype=torch.float32, pin_memory=True)
    synthgen.build() if synthgen._load() is None else None
    synthgen.fill_uniform_pm1(1001 + 3, M, K, hA.data_ptr())
    synthgen.fill_uniform_pm1(2001 + 3, K, N, hB.data_ptr())
    flops = 2.0 * M * N * K
    dA = dB = dC = None
    if on_device or not args.no_device_context:
        dA, dB = hA.to("cuda"), hB.to("cuda")
        dC = torch.empty((M, N), dtype=torch.float32, device="cuda")
    A, B, C = (dA, dB, dC) if on_device else (hA, hB, hC)
    torch.cuda.synchronize()

    fastmm.set_profiling(True)

    def run(depth, a=A, b=B, c=C):
        return lambda: fastmm.gemm(M, N, K, a, b, c, depth=depth, leaf=args.leaf, tile=args.tile)

    def stats_ms(ts):
        q = np.percentile(np.asarray(ts) * 1e3, [25, 50, 75])
        return {"median": float(q[1]), "min": 1e3 * min(ts), "iqr": float(q[2] - q[0])}

    # Plain MFMA SGEMM (depth 0) on the same operands and path.
    plain = None
    if not args.no_plain:
        log("bench: plain SGEMM (depth 0)")
        tot, ts = time_calls(run(0), args.steps, args.warmup)
        st = fastmm.get_stats()
        plain = {"ms_per_step": 1e3 * tot / args.steps, "value": flops / (tot / args.steps) / 1e9,
                 "ms": stats_ms(ts), "leaf_ms": st["leaf_ms"],
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
    leaf_ms, leaf_launches, step_s = [], [], []

    def step():
        t = time.perf_counter()
        fastmm.gemm(M, N, K, A, B, C, depth=best, leaf=args.leaf, tile=args.tile)
        step_s.append(time.perf_counter() - t)
        s_ = fastmm.get_stats()
        leaf_ms.append(s_["leaf_ms"])
        leaf_launches.append(s_["leaf_launches"])

    for _ in range(args.warmup):
        step()
    leaf_ms.clear()
    leaf_launches.clear()
    step_s.clear()
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
    An = hA.numpy()
    Bn = hB.numpy()
    Cn = C.cpu().numpy() if on_device else hC.numpy()
    rows = synthgen.row_sample(7004, M, 8)
    parity = {"sampled_rows_rel": checks.sampled_rows_rel(Cn, An, Bn, rows),
              "freivalds_rel": checks.freivalds_rel(Cn, An, Bn, synthgen.signs_pm1(7005, N)),
              "rows": int(rows.size), "tolerance": 1e-4}
    log(f"bench: parity {parity}")

    # Dominant kernel: the grouped leaf GEMM.  Its launches are timed with
    # HIP events recorded by the library on the stream it launches each on;
    # the library reports the union of the launches' intervals (with host
    # operands consecutive launches overlap on two compute streams, so the
    # union, not the sum, is the time the leaf work took), and a launch's
    # duration is that union over the launches.
    def leaf_roofline(leaf_list, launch_list, stats, traffic, kernel):
        n_launch = max(1, int(np.mean(launch_list)))
        leaf_sum = float(np.mean(leaf_list))          # ms per step, union of all leaf launches
        avg_launch = leaf_sum / n_launch
        flops_launch = stats["leaf_flops"] / n_launch
        tf = flops_launch / (avg_launch * 1e-3) / 1e12
        peak = PEAK_16BIT_TFLOPS / 3 if split else PEAK_FP32_TFLOPS
        return {"bound": "mfma", "kernel": kernel, "achieved": tf, "peak": peak, "unit": "TFLOP/s",
                "frac": tf / peak, "traffic": traffic, "flops_per_launch": flops_launch,
                "avg_launch_ms": avg_launch, "launches_per_step": n_launch,
                "launch_ms_is": "union of the step's leaf launch intervals / launches"}, leaf_sum

    split = SPLIT_FORMS.get(args.tile)
    if split and st["depth"] >= 1:  # the scale and pack passes run fused with the last pre-additions
        kernel = f"leaf_packed_kernel<{args.tile - 8},256,256,4,4>"
    else:
        kernel = split[1] if split else "leaf_gemm_kernel<128,128,16,2,2> (grouped leaves)"
    std_cfg = best == 3 and n == 19456 and args.tile == 0 and args.leaf == 1024
    traffic = (TRAFFIC_DEVICE_BYTES_PER_LAUNCH if on_device else TRAFFIC_PINNED_BYTES_PER_LAUNCH) \
        if std_cfg else None
    roofline, leaf_sum = leaf_roofline(leaf_ms, leaf_launches, st, traffic, kernel)
    phases = {"leaf_ms": leaf_sum, "preadd_ms": st["preadd_ms"], "postadd_ms": st["postadd_ms"],
              "h2d_span_ms": st["h2d_ms"], "call_span_ms": st["total_ms"],
              "add_bytes": st["add_bytes"], "transfer_bytes": st["transfer_bytes"]}
    add_ms = st["preadd_ms"] + st["postadd_ms"]
    if add_ms > 0:
        phases["add_GBps"] = st["add_bytes"] / (add_ms * 1e-3) / 1e9
        phases["add_frac_of_hbm_peak"] = phases["add_GBps"] / PEAK_HBM_GBS

    # Context: the same product with A, B, C already resident in HBM (no
    # transfers in the wall-clock), best depth of 2-4, and the plain SGEMM.
    hbm = None
    if not on_device and not args.no_device_context:
        log("bench: HBM-resident context")
        hp = {}
        for d in (2, 3, 4):
            tot, ts = time_calls(run(d, dA, dB, dC), 2, 1)
            hp[d] = min(ts)
        hb = min(hp, key=hp.get)
        lm, ll, hs = [], [], []
        fn = run(hb, dA, dB, dC)
        for _ in range(2):
            fn()
        torch.cuda.synchronize()
        for _ in range(max(5, min(args.steps, 10))):
            t = time.perf_counter()
            fn()
            hs.append(time.perf_counter() - t)
            s_ = fastmm.get_stats()
            lm.append(s_["leaf_ms"])
            ll.append(s_["leaf_launches"])
        sh = fastmm.get_stats()
        hroof, hleaf = leaf_roofline(lm, ll, sh, TRAFFIC_DEVICE_BYTES_PER_LAUNCH
                                     if hb == 3 and n == 19456 and args.tile == 0 and args.leaf == 1024
                                     else None, kernel)
        hbm = {"depth": hb, "ms": stats_ms(hs), "effective_GFLOPS": flops / float(np.median(hs)) / 1e9,
               "depth_probe_ms": {str(k): 1e3 * v for k, v in hp.items()}, "roofline": hroof,
               "preadd_ms": sh["preadd_ms"], "postadd_ms": sh["postadd_ms"], "add_bytes": sh["add_bytes"]}
        if sh["preadd_ms"] + sh["postadd_ms"] > 0:
            hbm["add_GBps"] = sh["add_bytes"] / ((sh["preadd_ms"] + sh["postadd_ms"]) * 1e-3) / 1e9
        if not args.no_plain:
            tot, ts = time_calls(run(0, dA, dB, dC), max(3, min(args.steps, 5)), 1)
            hbm["plain_ms"] = stats_ms(ts)
            hbm["speedup_vs_plain"] = hbm["plain_ms"]["median"] / hbm["ms"]["median"]
        log(f"bench: HBM-resident {hbm}")

    # Context: the paper's own algorithm, the classic eight-product recursion
    # of Table 1 at its recursion point (leaves below 6016, i.e. leaf cutoff
    # 3008), MFMA leaves, operands in HBM.
    classic = None
    if dA is not None and not args.no_device_context:
        fastmm.rmul(M, N, K, dA, dB, dC, depth=8, leaf=3008)
        torch.cuda.synchronize()
        t = time.perf_counter()
        fastmm.rmul(M, N, K, dA, dB, dC, depth=8, leaf=3008)
        torch.cuda.synchronize()
        t = time.perf_counter() - t
        classic = {"ms": 1e3 * t, "effective_GFLOPS": flops / t / 1e9,
                   "depth": fastmm.get_stats()["depth"], "leaf": 3008, "operands": "HBM"}
        log(f"bench: classic recursion {classic}")

    # Context: torch.matmul in FP32 (hipBLASLt, TF32 off) on the same
    # operands in HBM -- the vendor library's plain product.
    torch_mm = None
    if dA is not None and not args.no_device_context:
        prev = torch.backends.cuda.matmul.allow_tf32
        torch.backends.cuda.matmul.allow_tf32 = False

        def mm():
            torch.matmul(dA, dB, out=dC)
            torch.cuda.synchronize()

        tot, ts = time_calls(mm, 3, 1)
        torch.backends.cuda.matmul.allow_tf32 = prev
        torch_mm = {"ms": stats_ms(ts), "effective_GFLOPS": flops / min(ts) / 1e9,
                    "library": "hipBLASLt via torch.matmul", "tf32": False}
        log(f"bench: torch.matmul FP32 {torch_mm}")

    # Context: the split-precision leaf forms (never the FP32 headline): split
    # BF16 (tile 8) and scaled split FP16 (tile 9) leaves, plain and at depth
    # 2 (their workload's depth), operands in HBM; sampled-row error against
    # the oracle.  Leaf times include the forms' pack (and FP16 scale) passes.
    precision = None
    if dA is not None and not args.no_device_context:
        precision = {}
        rows_p = synthgen.row_sample(7008, M, 4)
        for name, tile in (("bf16x3", 8), ("fp16x3", 9)):
            for d in (0, 2):
                fn = lambda: fastmm.gemm(M, N, K, dA, dB, dC, depth=d, leaf=args.leaf, tile=tile)
                tot, ts = time_calls(fn, 3, 1)
                sp = fastmm.get_stats()
                Cp = dC.cpu().numpy()
                precision[f"{name}_depth{sp['depth']}"] = {
                    "ms": 1e3 * min(ts), "effective_GFLOPS": flops / min(ts) / 1e9,
                    "leaf_ms": sp["leaf_ms"],
                    "leaf_TFLOPs_fp32_equivalent": sp["leaf_flops"] / (sp["leaf_ms"] * 1e-3) / 1e12,
                    "leaf_frac_of_16bit_roofline":
                        sp["leaf_flops"] / (sp["leaf_ms"] * 1e-3) / 1e12 / (PEAK_16BIT_TFLOPS / 3),
                    "sampled_rows_rel": checks.sampled_rows_rel(Cp, An, Bn, rows_p)}
                del Cp
        log(f"bench: precision forms {precision}")

    # One GPU's share of the column-panel sharding (the paper's two-device
    # split, eqs. (3)-(4), generalised): 1 x 8 panels (19456 x 19456 x 2432)
    # and a 2 x 4 grid (9728 x 19456 x 4864), staged from the pinned host
    # operands (strided views), as many levels as the leaf cutoff allows.
    shards = None
    if n == 19456 and not args.no_shards and not on_device:
        shards = {}
        for name, (sm, sn) in {"panel_1x8": (M, N // 8), "grid_2x4": (M // 2, N // 4)}.items():
            fn = lambda: fastmm.gemm(sm, sn, K, hA[:sm], hB[:, :sn], hC[:sm, :sn], depth=16,
                                     leaf=args.leaf)
            tot, ts = time_calls(fn, 3, 1)
            sst = fastmm.get_stats()
            shards[name] = {"M": sm, "N": sn, "K": K, "depth": sst["depth"], "ms": 1e3 * min(ts),
                            "effective_GFLOPS": 2.0 * sm * sn * K / min(ts) / 1e9}
        log(f"bench: shard shapes {shards}")

    # The paper-scale rectangular product, M = 19456, K = 16384, N = 12288,
    # with operands in pinned host memory (transfers timed) at depths 2-4 and
    # plain, and the same shape with operands in HBM; strided views of the
    # square operands.
    rect = None
    if n == 19456 and not args.no_rect and dA is not None and not on_device:
        rm, rk, rn = 19456, 16384, 12288
        rect = {"M": rm, "N": rn, "K": rk, "pinned_ms": {}, "device_ms": {}}
        rf = 2.0 * rm * rn * rk
        for where, (a, b, c) in (("pinned_ms", (hA[:, :rk], hB[:rk, :rn], hC[:, :rn])),
                                 ("device_ms", (dA[:, :rk], dB[:rk, :rn], dC[:, :rn]))):
            for d in (0, 2, 3, 4):
                fn = lambda: fastmm.gemm(rm, rn, rk, a, b, c, depth=d, leaf=1)
                tot, ts = time_calls(fn, 2, 1)
                assert fastmm.get_stats()["depth"] == d
                rect[where][str(d)] = 1e3 * min(ts)
        for where in ("pinned", "device"):
            t = rect[where + "_ms"]
            bd = min(("2", "3", "4"), key=lambda k: t[k])
            rect[where + "_best"] = {"depth": int(bd), "effective_GFLOPS": rf / (t[bd] * 1e-3) / 1e9,
                                     "speedup_vs_plain": t["0"] / t[bd]}
        log(f"bench: rectangular {rect}")

    batched = None
    if not args.no_batched and not on_device:
        del dA, dB, dC
        dA = dB = dC = None
        torch.cuda.empty_cache()
        batched = batched_context(fastmm, torch, with_planner=not args.no_planner)
        log(f"bench: batched context {batched}")

    cpu = None
    if not args.no_cpu:
        from oracle import classic as oracle_classic
        threads = oracle_classic.num_threads()
        rows_c = synthgen.row_sample(7006, M, 32)
        t = time.perf_counter()
        oracle_classic.gemm_rows(An, Bn, rows_c)
        per_row = (time.perf_counter() - t) / rows_c.size
        R = int(max(4, min(4096, args.cpu_seconds / max(per_row, 1e-6))))
        rows_c = synthgen.row_sample(7007, M, R)
        t = time.perf_counter()
        oracle_classic.gemm_rows(An, Bn, rows_c)
        dt = time.perf_counter() - t
        cpu = {"value": 2.0 * rows_c.size * N * K / dt / 1e9, "unit": "GFLOPS", "cores": threads,
               "cpu_model": cpu_model(), "kind": "oracle",
               "sample": f"{rows_c.size} seeded rows of C (FP64-accumulated triple loop, "
                         f"OpenMP over rows), {dt:.1f} s"}
        log(f"bench: cpu {cpu}")

    where = ("operands resident in HBM" if on_device
             else "pinned host in/out (H2D and D2H transfers inside the wall-clock)")
    out = {
        "metric": METRIC, "value": value, "unit": "GFLOPS", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
        "ms": stats_ms(step_s),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": split[0] if split else "f32",
        "data": "synthetic",
        "config": {"workload": f"FP32 Winograd-Strassen C=A*B, square n={n}, {where}, "
                               + (f"{split[0]} leaves, " if split else "") +
                               f"depth {st['depth']}, leaf {args.leaf}",
                   "M": M, "N": N, "K": K, "depth": st["depth"], "leaf": args.leaf,
                   "tile": args.tile, "operands": args.operands, "parallelism": "single GPU"},
        "roofline": roofline, "cpu_baseline": cpu,
        "plain_sgemm": plain,
        "speedup_vs_plain": (plain["ms_per_step"] / ms_per_step) if plain else None,
        "depth_probe_ms": {str(k): 1e3 * v for k, v in probe.items()},
        "phases": phases, "hbm_resident": hbm, "classic_recursion": classic, "torch_matmul_fp32": torch_mm,
        "precision_forms": precision, "batched": batched, "shards": shards, "rectangular": rect,
        "parity": parity,
    }
    print(json.dumps(out), flush=True)
    # Release the library's streams, workspace and staging while the runtime
    # is fully up, rather than leaving them to process teardown.
    torch.cuda.synchronize()
    fastmm.finalize()


if __name__ == "__main__":
    main()
