"""Benchmark: GEMM TFLOP/s through the selected variant vs the plain FP32 variant, and the
selector's regret against exhaustive timing, on one MI355X.

Phases (all on cuda:0, synthetic seeded inputs, no files read):
  1. time-and-record: every variant (the four default built-ins, the optional
     MX fp6 variant unless --no-fp6, and the host CPU variant up to --host-max)
     on the square sweep N in {128, ..., 8192}
     (normal(0,1) operands, 3 warm-up + 20 timed reps, median) -> history;
  2. timed region: `--steps` steps after `--warmup` steps; one step is one
     cmp_gemm per tolerance class {1e-5, 1e-3, 1e-2} at M = N = K = `--size`
     with the history nearest-neighbour selector, operands resident in HBM;
     per-kernel HIP-event timing is on during this region;
  3. selector experiment (skipped with --no-selector): 2000 training and 500
     held-out shapes with M, N, K log-uniform in [64, 8192], the four default
     variants timed (the network has one output per default variant),
     network trained on the GPU from the training table, regret of each selector
     on the held-out rows of the measured table;
  4. CPU baseline: the FP64 CPU oracle on a bounded row panel of the same product.
Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import synth  # noqa: E402

PEAK = {  # MI355X published dense peaks (TFLOP/s) and HBM bandwidth (GB/s)
    "bf16": 2516.6, "fp8": 5033.2, "fp6": 10066.3, "fp32_vector": 157.3, "fp64_vector": 78.6,
    "hbm_gbs": 8000.0,
}
BOUNDS = [1e-5, 1e-5, 1e-3, 1e-2]


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_roofline(name: str, M: int, N: int, K: int):
    """(bound, algorithmic work per launch, peak, unit) of a built-in kernel at M x N x K."""
    Kp64 = -(-K // 64) * 64
    Kp128 = -(-K // 128) * 128
    if name == "gemm_f32_simt":
        return "alu", 2.0 * M * N * K, PEAK["fp32_vector"], "TFLOP/s"
    if name == "gemm_bf16_tn":
        return "mfma", 2.0 * M * N * K, PEAK["bf16"], "TFLOP/s"
    if name == "gemm_bf16x3_tn":
        return "mfma", 3 * 2.0 * M * N * K, PEAK["bf16"], "TFLOP/s"
    if name == "gemm_fp8r_tn":
        return "mfma", 4 * 2.0 * M * N * K, PEAK["fp8"], "TFLOP/s"
    if name == "gemm_fp6x3_tn":
        return "mfma", 3 * 2.0 * M * N * K, PEAK["fp6"], "TFLOP/s"
    # pre-pass kernels: bytes read + written (HBM-bound)
    if name == "split_bf16_ab":       # both operands in one launch
        return "hbm", 4.0 * (M * K + K * N) + 2.0 * (M + N) * Kp64, PEAK["hbm_gbs"], "GB/s"
    if name == "split_bf16_hilo_ab":
        return "hbm", 4.0 * (M * K + K * N) + 4.0 * (M + N) * Kp64, PEAK["hbm_gbs"], "GB/s"
    if name == "quant_fp8_ab":
        return "hbm", 4.0 * (M * K + K * N) + 2.0 * (M + N) * Kp128, PEAK["hbm_gbs"], "GB/s"
    # MX fp6 images: 3/4 byte per K value and level, plus 4 scale bytes per 64 K values
    if name == "quant_mx6_ab":
        return "hbm", 4.0 * (M * K + K * N) + 1.5625 * (M + N) * Kp64, PEAK["hbm_gbs"], "GB/s"
    return None


KERNEL_SOURCES = {  # kernel name -> source file (relative to the repo root)
    "gemm_f32_simt": "paper_2311_03543_amd/csrc/gemm_f32_simt.hip",
    "gemm_bf16_tn": "paper_2311_03543_amd/csrc/gemm_mfma.hip",
    "gemm_bf16x3_tn": "paper_2311_03543_amd/csrc/gemm_mfma.hip",
    "gemm_fp8r_tn": "paper_2311_03543_amd/csrc/gemm_mfma.hip",
    "gemm_fp6x3_tn": "paper_2311_03543_amd/csrc/gemm_mfma.hip",
}


def measured_traffic(name: str, n: int):
    """HBM bytes per launch of kernel `name` at M = N = K = n from the committed counter summary
    (FETCH_SIZE and WRITE_SIZE per dispatch, each scaled by the factor a plain copy of known size
    gives), or None when there is none or the kernel source changed since it was taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"hbm_traffic_n{n}.json")
    src = KERNEL_SOURCES.get(name)
    if not src or not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f).get("kernels", {}).get(name)
    if not rec:
        return None
    with open(os.path.join(ROOT, src), "rb") as f:
        digest = hashlib.sha256(f.read()).hexdigest()
    if rec.get("source_sha256") != digest:
        return None
    return rec.get("hbm_bytes_per_launch")


def regret(T, choices, tols):
    """Aggregate sum T[s, choice] / sum T[s, best admissible] - 1, plus mean and p95 per shape."""
    best = []
    for s in range(T.shape[0]):
        adm = [v for v in range(4) if BOUNDS[v] <= tols[s]]
        best.append(min(adm, key=lambda v: (T[s, v], BOUNDS[v], v)))
    sel = np.array([T[s, c] for s, c in enumerate(choices)])
    opt = np.array([T[s, b] for s, b in enumerate(best)])
    per = sel / opt - 1.0
    return dict(aggregate_pct=100.0 * float(sel.sum() / opt.sum() - 1.0),
                mean_pct=100.0 * float(per.mean()), p95_pct=100.0 * float(np.percentile(per, 95)))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--size", type=int, default=8192)
    ap.add_argument("--reps", type=int, default=20, help="timed reps per variant and shape")
    ap.add_argument("--no-selector", action="store_true")
    ap.add_argument("--no-grouped", action="store_true")
    ap.add_argument("--no-stream", action="store_true")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run a plain 256 MiB device copy (reference kernel for HBM byte counters)")
    ap.add_argument("--stream-requests", type=int, default=10000)
    ap.add_argument("--grouped-problems", type=int, default=1024)
    ap.add_argument("--train-shapes", type=int, default=2000)
    ap.add_argument("--heldout-shapes", type=int, default=500)
    ap.add_argument("--mlp-steps", type=int, default=5000)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-vendor", action="store_true",
                    help="skip the vendor-library reference (torch.mm, i.e. hipBLASLt, at the same size)")
    ap.add_argument("--clock-seconds", type=float, default=8.0,
                    help="sustained bf16 run while sampling board power and GFX clocks (0 = skip)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-fp6", action="store_true", help="leave the optional MX fp6 variant unregistered")
    ap.add_argument("--host-max", type=int, default=1024,
                    help="time the host CPU variant on sweep sizes up to this N (0: leave it unregistered)")
    ap.add_argument("--sweep", type=str, default="",
                    help="comma-separated square sizes to time and record (default: 128..--size)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus > 1 or world > 1:
        print(f"bench.py runs on one GPU only: --gpus {args.gpus} is not supported by this "
              "single-GPU build (a GEMM shards by row panels of C with no exchange, one process per GPU)",
              file=sys.stderr, flush=True)
        sys.exit(2)

    import torch
    import paper_2311_03543_amd as pa

    cx = pa.Compar(0)
    dev = cx.device()
    log(f"device {dev}")
    n = args.size
    # the four default built-ins plus the optional MX fp6 variant: every one is timed,
    # recorded, and open to selection
    names = list(pa.BUILTIN_VARIANTS)
    if not args.no_fp6:
        assert cx.register_builtin("fp6x3") == len(names)
        names.append("fp6x3")
    # the host CPU variant: timed (and so selectable) up to --host-max only
    if args.host_max > 0:
        assert cx.register_builtin("host_f32") == len(names)
        names.append("host_f32")

    # ---- 1. time and record: square sweep -----------------------------------------
    sweep = {}
    if args.sweep:
        sizes = sorted({int(v) for v in args.sweep.split(",")} | {n})
    else:
        sizes = [s for s in synth.square_sweep_sizes() if s <= n] or [n]
        if n not in sizes:
            sizes.append(n)
    big = {}
    for s in sizes:
        A, B = synth.gemm_operands(s, s, s, seed=synth.square_sweep_seed(s))
        dA, dB = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
        dC = torch.zeros((s, s), dtype=torch.float32, device="cuda")
        row = {}
        for vid, name in enumerate(names):
            if name == "host_f32" and s > args.host_max:
                continue
            med, mn, mean = cx.time_variant(vid, dA, dB, dC, warmup=3, reps=args.reps)
            cx.history_add(s, s, s, vid, args.reps, med, mn, mean)
            row[name] = dict(median_ms=med, min_ms=mn, mean_ms=mean, tflops=2.0 * s ** 3 / (med * 1e-3) / 1e12)
        sweep[s] = row
        log(f"sweep N={s}: " + ", ".join(f"{k} {v['tflops']:.1f} TF" for k, v in row.items()))
        if s == n:
            big = dict(A=A, B=B, dA=dA, dB=dB, dC=dC)
        else:
            del dA, dB, dC

    # ---- 2. timed region ----------------------------------------------------------
    dA, dB, dC = big["dA"], big["dB"], big["dC"]
    cx.selector_set(pa.CMP_SEL_NN)
    tols = list(synth.TOL_CLASSES)
    for _ in range(args.warmup):
        for tol in tols:
            cx.gemm(dA, dB, dC, tol=tol)
    torch.cuda.synchronize()
    cx.kernel_stats(reset=True)
    cx.kernel_timing(True)
    chosen = {}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        for tol in tols:
            chosen[tol] = cx.gemm(dA, dB, dC, tol=tol)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    cx.kernel_timing(False)
    kstats = cx.kernel_stats(reset=True)
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    flops_step = len(tols) * 2.0 * n ** 3
    value = flops_step / (ms_per_step * 1e-3) / 1e12
    log(f"timed: {ms_per_step:.3f} ms/step, {value:.1f} TFLOP/s; chosen "
        + ", ".join(f"{t:g}->{names[v]}" for t, v in chosen.items()))

    kernels = {}
    for name, (cnt, tot) in kstats.items():
        kernels[name] = dict(launches=cnt, avg_ms=tot / cnt, share=tot / (ms_per_step * args.steps))
    dominant = max(kstats, key=lambda k: kstats[k][1])
    bound, work, peak, unit = kernel_roofline(dominant, n, n, n)
    avg_s = kernels[dominant]["avg_ms"] * 1e-3
    achieved = work / avg_s / (1e12 if unit == "TFLOP/s" else 1e9)
    roofline = dict(kernel=dominant, bound=bound, achieved=achieved, peak=peak, unit=unit,
                    frac=achieved / peak, traffic=measured_traffic(dominant, n))
    for name, k in kernels.items():
        r = kernel_roofline(name, n, n, n)
        if r:
            kb, kw, kp, ku = r
            ach = kw / (k["avg_ms"] * 1e-3) / (1e12 if ku == "TFLOP/s" else 1e9)
            k.update(achieved=ach, unit=ku, frac=ach / kp)
    log("kernels: " + ", ".join(f"{k} {v['avg_ms']:.3f} ms ({v.get('frac', 0):.1%})" for k, v in kernels.items()))

    fp32_tflops = sweep[n]["f32_simt"]["tflops"]
    per_tol = {f"{t:g}": dict(variant=names[v], median_ms=sweep[n][names[v]]["median_ms"],
                              tflops=sweep[n][names[v]]["tflops"]) for t, v in chosen.items()}
    del big
    torch.cuda.empty_cache()

    if args.copy_probe:
        # a plain copy of known size: its FETCH_SIZE / WRITE_SIZE calibrate the HBM counters
        src = torch.empty(64 << 20, dtype=torch.float32, device="cuda").normal_()
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    # ---- 2a. context: the vendor GEMM library at the same size -----------------------
    vendor = None
    if not args.no_vendor:
        vendor = vendor_reference(torch, n)

    # ---- 2b. sustained load: board power and GFX clocks --------------------------------
    clock = None
    if args.clock_seconds > 0:
        clock = sustained_clock(cx, pa, torch, n, args.clock_seconds)

    # ---- 3. selector experiment -----------------------------------------------------
    selector = None
    if not args.no_selector:
        selector = selector_experiment(cx, pa, torch, args)

    # ---- 3b. batched uneven GEMMs: one grouped launch vs separate launches -----------
    grouped = None
    if not args.no_grouped:
        grouped = grouped_experiment(cx, pa, torch, args)

    # ---- 3c. request stream: per-request tolerance, Zipf shapes ---------------------
    stream_res = None
    if not args.no_stream:
        stream_res = stream_experiment(pa, torch, args)

    # ---- 4. CPU baseline: the oracle on a bounded row panel ----------------------------
    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(n, args.cpu_seconds)

    out = {
        "metric": "GEMM TFLOP/s via selected variant vs plain FP32; selector regret % vs oracle",
        "value": value,
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"square GEMM M=N=K={n}, FP32 in/out, normal(0,1) operands, one cmp_gemm "
                               f"per tolerance class {{1e-5,1e-3,1e-2}} per step, history nearest-neighbour "
                               f"selection", "M": n, "N": n, "K": n, "tolerances": tols},
        "per_tolerance": per_tol,
        "fp32_simt_tflops": fp32_tflops,
        "speedup_vs_fp32": value / fp32_tflops,
        "selector": selector,
        "grouped": grouped,
        "stream": stream_res,
        "roofline": roofline,
        "sustained_clock": clock,
        "vendor_reference": vendor,
        "kernels": kernels,
        "sweep_tflops": {str(s): {k: round(v["tflops"], 2) for k, v in row.items()} for s, row in sweep.items()},
        "cpu_baseline": cpu,
        "device": dev,
    }
    cx.close()
    print(json.dumps(out), flush=True)


def vendor_reference(torch, n):
    """Context only: torch.mm (hipBLASLt) on contiguous n x n operands in bf16 (bf16 output) and
    in fp32, median of 20 timed calls after 3 warm-ups; and a plain 512 MiB device copy (the HBM
    rate a read-and-write kernel reaches)."""
    res = {}
    g = torch.Generator(device="cuda").manual_seed(12)
    for name, dt in (("bf16", torch.bfloat16), ("f32", torch.float32)):
        A = torch.randn((n, n), device="cuda", generator=g).to(dt).contiguous()
        B = torch.randn((n, n), device="cuda", generator=g).to(dt).contiguous()
        for _ in range(3):
            torch.mm(A, B)
        torch.cuda.synchronize()
        ts = []
        for _ in range(20):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            torch.mm(A, B)
            e1.record()
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1))
        med = float(np.median(ts))
        res[f"torch_mm_{name}"] = dict(median_ms=med, tflops=2.0 * n ** 3 / (med * 1e-3) / 1e12)
        del A, B
    # a plain device copy (read + write of 512 MiB): the HBM rate the pre-pass kernels compare with
    src = torch.empty(128 << 20, dtype=torch.float32, device="cuda").normal_()
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    ts = []
    for _ in range(20):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        dst.copy_(src)
        e1.record()
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1))
    med = float(np.median(ts))
    copy = dict(median_ms=med, bytes=2.0 * src.numel() * 4, gbs=2.0 * src.numel() * 4 / (med * 1e-3) / 1e9)
    del src, dst
    torch.cuda.empty_cache()
    log("vendor reference: " + ", ".join(f"{k} {v['median_ms']:.3f} ms {v['tflops']:.0f} TF" for k, v in res.items())
        + f", device copy {copy['gbs']:.0f} GB/s")
    res["torch_copy_512MiB"] = copy
    return res


def sustained_clock(cx, pa, torch, n, seconds):
    """Run the bf16 variant back to back at n^3 for `seconds` while a thread samples the board's
    socket power and per-XCD GFX clocks with amd-smi (a child process, about once a second).
    Samples from the first 1.5 s (clock ramp) are dropped.  The published MFMA peaks assume
    2.4 GHz; `clock_adjusted_bf16_peak` rescales the bf16 peak to the measured mean clock."""
    import re
    import shutil
    import subprocess
    import threading
    smi = shutil.which("amd-smi") or "/opt/rocm/bin/amd-smi"
    if not os.path.exists(smi):
        return None
    vid = pa.BUILTIN_VARIANTS.index("bf16")
    g = torch.Generator(device="cuda").manual_seed(11)
    A = torch.randn((n, n), device="cuda", generator=g)
    B = torch.randn((n, n), device="cuda", generator=g)
    C = torch.zeros((n, n), device="cuda")
    samples = []
    stop = threading.Event()

    def sampler():
        while not stop.is_set():
            try:
                out = subprocess.run([smi, "metric", "-g", "0", "--clock", "--power"], capture_output=True,
                                     text=True, timeout=10).stdout
            except Exception:
                return
            clks = [int(x) for x in re.findall(r"GFX_\d+:\s*\n\s*CLK:\s*(\d+) MHz", out)]
            pw = re.search(r"SOCKET_POWER:\s*([\d.]+) W", out)
            if clks:
                samples.append((time.perf_counter(), clks, float(pw.group(1)) if pw else None))
            stop.wait(0.5)

    cx.gemm_variant(vid, A, B, C)
    torch.cuda.synchronize()
    th = threading.Thread(target=sampler, daemon=True)
    t0 = time.perf_counter()
    th.start()
    launches = 0
    while time.perf_counter() - t0 < seconds:
        for _ in range(10):
            cx.gemm_variant(vid, A, B, C)
        torch.cuda.synchronize()
        launches += 10
    dt = time.perf_counter() - t0
    stop.set()
    th.join(timeout=15)
    steady = [s for s in samples if s[0] - t0 > 1.5]
    tflops = launches * 2.0 * n ** 3 / dt / 1e12
    if not steady:
        return dict(variant="bf16", seconds=dt, launches=launches, tflops=tflops, samples=0)
    clk = np.array([c for _, cs, _ in steady for c in cs], dtype=np.float64)
    pw = [p for _, _, p in steady if p is not None]
    mean_mhz = float(clk.mean())
    adj = PEAK["bf16"] * mean_mhz / 2400.0
    log(f"sustained bf16: {tflops:.0f} TFLOP/s over {dt:.1f} s, GFX clock {mean_mhz:.0f} MHz "
        f"[{clk.min():.0f}, {clk.max():.0f}], socket power {np.mean(pw) if pw else float('nan'):.0f} W")
    return dict(variant="bf16", seconds=dt, launches=launches, tflops=tflops, samples=len(steady),
                gfx_mhz_mean=mean_mhz, gfx_mhz_min=float(clk.min()), gfx_mhz_max=float(clk.max()),
                socket_power_w_mean=float(np.mean(pw)) if pw else None,
                socket_power_w_max=float(np.max(pw)) if pw else None,
                clock_adjusted_bf16_peak=adj, frac_of_published_peak=tflops / PEAK["bf16"],
                frac_of_clock_adjusted_peak=tflops / adj)


def selector_experiment(cx, pa, torch, args):
    ntr, nho = args.train_shapes, args.heldout_shapes
    train = synth.log_uniform_shapes(ntr, 64, 8192, 2)
    held = synth.log_uniform_shapes(nho, 64, 8192, 3, avoid={tuple(r) for r in train})
    tol_tr = synth.tol_classes(ntr, 12)
    tol_ho = synth.tol_classes(nho, 13)
    # operands: the largest shape's A and B; each shape uses a tight prefix
    need_a = int(max((s[0] * s[2] for s in np.vstack([train, held]))))
    need_b = int(max((s[2] * s[1] for s in np.vstack([train, held]))))
    need_c = int(max((s[0] * s[1] for s in np.vstack([train, held]))))
    g = torch.Generator(device="cuda").manual_seed(4)
    dA = torch.randn(need_a, device="cuda", generator=g)
    dB = torch.randn(need_b, device="cuda", generator=g)
    dC = torch.zeros(need_c, device="cuda")
    sel = pa.Compar(0)
    t0 = time.perf_counter()
    shapes = np.vstack([train, held])
    chunk = 100
    for i in range(0, len(shapes), chunk):
        sel.calibrate([tuple(map(int, s)) for s in shapes[i:i + chunk]], dA, dB, dC, warmup=2, reps=args.reps)
        log(f"selector: timed {min(i + chunk, len(shapes))}/{len(shapes)} shapes ({time.perf_counter() - t0:.1f} s)")
    rows = sel.history()
    T = {}
    for (M, N, K, vid, reps, med, mn, mean) in rows:
        T.setdefault((M, N, K), [0.0] * 4)[vid] = med
    Ttr = np.array([T[tuple(map(int, s))] for s in train])
    Tho = np.array([T[tuple(map(int, s))] for s in held])
    # training history only
    sel.history_clear()
    for s, trow in zip(train, Ttr):
        for v in range(4):
            sel.history_add(int(s[0]), int(s[1]), int(s[2]), v, args.reps, float(trow[v]))
    q = [(int(m), int(nn), int(k), float(t)) for (m, nn, k), t in zip(held, tol_ho)]
    res = {}
    for kind, label in [(pa.CMP_SEL_NN, "nn"), (pa.CMP_SEL_STATIC, "static")]:
        sel.selector_set(kind)
        res[label] = regret(Tho, sel.select_batch(q), tol_ho)
    t1 = time.perf_counter()
    loss = sel.mlp_fit_history(steps=args.mlp_steps, lr=1e-3, seed=0)
    t2 = time.perf_counter()
    sel.selector_set(pa.CMP_SEL_MLP)
    t3 = time.perf_counter()
    mlp_choice = sel.select_batch(q)
    t4 = time.perf_counter()
    res["mlp"] = regret(Tho, mlp_choice, tol_ho)
    res["always_fp32"] = regret(Tho, [0] * len(q), tol_ho)
    # per-call decision cost: the 500 held-out contexts through cmp_select_batch, first
    # uncached (network inference or nearest-neighbour search), then from the decision cache
    # (the path every repeated call takes), averaged over 200 passes
    decision_us = {}
    for kind, label in [(pa.CMP_SEL_MLP, "mlp"), (pa.CMP_SEL_NN, "nn")]:
        sel.selector_set(kind)                  # switching the selector clears the cache
        ta = time.perf_counter()
        sel.select_batch(q)
        tb = time.perf_counter()
        for _ in range(200):
            sel.select_batch(q)
        tc = time.perf_counter()
        decision_us[f"{label}_uncached"] = (tb - ta) * 1e6 / len(q)
        decision_us[f"{label}_cached"] = (tc - tb) * 1e6 / (200 * len(q))
    # the best variant differs across shapes: how often each is the held-out optimum
    best_counts = {}
    for s in range(len(held)):
        adm = [v for v in range(4) if BOUNDS[v] <= tol_ho[s]]
        b = min(adm, key=lambda v: (Tho[s, v], BOUNDS[v], v))
        best_counts[pa.BUILTIN_VARIANTS[b]] = best_counts.get(pa.BUILTIN_VARIANTS[b], 0) + 1
    sel.close()
    log(f"selector regret: " + ", ".join(f"{k} {v['aggregate_pct']:.2f}%" for k, v in res.items()))
    return dict(train_shapes=ntr, heldout_shapes=nho, reps=args.reps, mlp_steps=args.mlp_steps,
                mlp_final_loss=loss, mlp_train_s=t2 - t1, mlp_select_500_ms=(t4 - t3) * 1e3,
                calibration_s=t1 - t0, regret=res, heldout_best_counts=best_counts,
                decision_us_per_call=decision_us,
                regret_pct=res["mlp"]["aggregate_pct"])


def grouped_experiment(cx, pa, torch, args):
    """1024 problems, M, N, K log-uniform in [32, 1024] (seed 4), normal(0,1) FP32 operands.
    The separate launches run f32_simt per problem; the grouped plan's autotuner picks among the
    FP32 SIMT tiles and the bf16x3 MFMA configuration (both in the 1e-5 class)."""
    count = args.grouped_problems
    shapes = synth.log_uniform_shapes(count, 32, 1024, 4)
    g = torch.Generator(device="cuda").manual_seed(5)
    probs = []
    for (M, N, K) in shapes:
        A = torch.randn((int(M), int(K)), device="cuda", generator=g)
        B = torch.randn((int(K), int(N)), device="cuda", generator=g)
        probs.append((A, B, torch.zeros((int(M), int(N)), device="cuda")))
    flops = float(sum(2.0 * int(M) * int(N) * int(K) for M, N, K in shapes))
    reps = 10

    def timed(fn):
        for _ in range(2):
            fn()
        torch.cuda.synchronize()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
        for a, b in ev:
            a.record()
            fn()
            b.record()
        torch.cuda.synchronize()
        ts = sorted(a.elapsed_time(b) for a, b in ev)
        return ts[len(ts) // 2]

    def separate():
        for A, B, C in probs:
            cx.gemm_variant(0, A, B, C)
    t_sep = timed(separate)
    # the same 1024 launches captured once in a graph
    graph = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        separate()
    torch.cuda.current_stream().wait_stream(s)
    with torch.cuda.graph(graph):
        separate()
    t_sep_graph = timed(graph.replay)
    t0 = time.perf_counter()
    plan = cx.grouped_plan(probs, config=-1, reps=5)
    t_tune = time.perf_counter() - t0
    info = plan.info()
    t_grp = timed(plan.launch)
    t_grp_graph = timed(plan.graph_launch)
    plan.destroy()
    cfgs = pa.grouped_configs()
    arith = [("f32_simt", "bf16x3")[pa.grouped_config_variant(i)] for i in range(len(cfgs))]
    res = dict(problems=count, gflop=flops / 1e9,
               separate_ms=t_sep, separate_graph_ms=t_sep_graph,
               grouped_ms=t_grp, grouped_graph_ms=t_grp_graph,
               grouped_tflops=flops / (t_grp_graph * 1e-3) / 1e12,
               separate_tflops=flops / (t_sep * 1e-3) / 1e12,
               speedup_vs_separate=t_sep / t_grp_graph,
               autotune_s=t_tune, tile=cfgs[info["config"]], arithmetic=arith[info["config"]],
               tiles=info["tiles"], grid=info["grid"],
               autotune_ms={f"{c[0]}x{c[1]}x{c[2]} {a}": ms for c, a, ms in zip(cfgs, arith, info["config_ms"])})
    log(f"grouped: separate {t_sep:.2f} ms, separate+graph {t_sep_graph:.2f} ms, grouped {t_grp:.2f} ms, "
        f"grouped+graph {t_grp_graph:.2f} ms, tile {res['tile']} {res['arithmetic']}")
    del probs
    torch.cuda.empty_cache()
    return res


def stream_experiment(pa, torch, args):
    """10000 requests over 50 shapes (M, N, K log-uniform in [64, 4096]), Zipf(1.1) ranks,
    tolerance per request, 20% ill-conditioned operands served in verify mode; each request
    completes before the next is submitted."""
    from paper_2311_03543_amd import stream as st
    req = st.make_stream(nshapes=50, nreq=args.stream_requests, lo=64, hi=4096, s=1.1, ill_frac=0.2, seed=5)
    pool = st.build_pool(req["shapes"], seed=9, device_gen=True)
    cx = pa.Compar(0)
    shapes = [tuple(map(int, s)) for s in req["shapes"]]
    need = max(max(m * k, k * n, m * n) for m, n, k in shapes)
    A = torch.randn(need, device="cuda")
    B = torch.randn(need, device="cuda")
    C = torch.zeros(need, device="cuda")
    cx.calibrate(shapes, A, B, C, warmup=2, reps=args.reps)
    del A, B, C
    cx.selector_set(pa.CMP_SEL_NN)
    # warm the workspace and the decision cache on every (shape, tolerance) pair
    for sh in range(len(shapes)):
        for t in synth.TOL_CLASSES:
            a, b = pool[sh]["well"][0]
            cx.gemm(a, b, pool[sh]["C"], tol=t)
    torch.cuda.synchronize()
    # served by the library's executor (cmp_gemm_stream), then once more one cmp_gemm per
    # request from Python, for the host overhead of the binding
    t0 = time.perf_counter()
    lat, chosen, fallbacks = st.run_stream_native(cx, req, pool, verify_ill=True)
    wall = time.perf_counter() - t0
    t0 = time.perf_counter()
    lat_py, _, _ = st.run_stream(cx, req, pool, verify_ill=True)
    wall_py = time.perf_counter() - t0
    cx.close()
    flops = sum(2.0 * shapes[r - 1][0] * shapes[r - 1][1] * shapes[r - 1][2] for r in req["ranks"])
    mix = {pa.BUILTIN_VARIANTS[v]: int((chosen == v).sum()) for v in range(4)}
    ill = req["ill"]
    res = dict(requests=len(lat), executor="cmp_gemm_stream", wall_s=wall, req_per_s=len(lat) / wall,
               tflops=flops / wall / 1e12,
               p50_us=float(np.percentile(lat, 50)), p99_us=float(np.percentile(lat, 99)),
               p50_us_well=float(np.percentile(lat[~ill], 50)), p99_us_well=float(np.percentile(lat[~ill], 99)),
               p50_us_ill_verify=float(np.percentile(lat[ill], 50)),
               p99_us_ill_verify=float(np.percentile(lat[ill], 99)),
               variant_mix=mix, verify_fallbacks=int(fallbacks),
               per_call_python=dict(req_per_s=len(lat_py) / wall_py, p50_us=float(np.percentile(lat_py, 50)),
                                    p99_us=float(np.percentile(lat_py, 99))))
    log(f"stream: {res['req_per_s']:.0f} req/s, p50 {res['p50_us']:.0f} us, p99 {res['p99_us']:.0f} us, "
        f"mix {mix}, fallbacks {fallbacks}; one cmp_gemm per request from Python "
        f"{res['per_call_python']['req_per_s']:.0f} req/s, p50 {res['per_call_python']['p50_us']:.0f} us")
    del pool
    torch.cuda.empty_cache()
    return res


def cpu_baseline(n, seconds):
    """The FP64 oracle (cpu_baseline leg) on rows [0, r) of the n^3 product, r sized for ~`seconds`."""
    import oracle
    A, B = synth.gemm_operands(n, n, n, seed=synth.square_sweep_seed(n))
    probe = 16
    t0 = time.perf_counter()
    oracle.gemm(A[:probe], B)
    dt = time.perf_counter() - t0
    rows = int(max(probe, min(n, probe * seconds / max(dt, 1e-6))))
    rows = max(probe, (rows // 32) * 32)
    t0 = time.perf_counter()
    oracle.gemm(A[:rows], B)
    dt = time.perf_counter() - t0
    flops = 2.0 * rows * n * n
    log(f"cpu baseline: {rows} rows of {n}^3 in {dt:.1f} s = {flops / dt / 1e9:.1f} GFLOP/s")
    return dict(value=flops / dt / 1e12, unit="TFLOP/s", cores=oracle.threads(), kind="oracle",
                sample=f"FP64 oracle (blocked triple loop) on rows 0..{rows} of the {n}x{n}x{n} product "
                       f"({flops / 1e9:.0f} GFLOP, {dt:.1f} s)", seconds=dt)


if __name__ == "__main__":
    main()
