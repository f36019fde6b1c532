"""Benchmark of the streaming taches convolution on one MI355X.

Workload (one step): one mono 48 kHz stream of 480 000 samples (10 s) of
seeded Gaussian noise, two seeded decaying-noise impulse responses of
L = 65 536 taps swapped every 4 800 samples (99 swaps, at the next block
boundary), block size B = 256.  A step stages both IRs into the stream's IR
slots, processes the 1 875 blocks with their IR schedule in one
taches_process_blocks call (device-resident input and output), then drains
the temporal overflow (L - 1 samples) with a NULL-input call.

value: direct-convolution-equivalent multiply-accumulates of the step
(sum over input samples of the active L = 480 000 * 65 536) per second.

Also reported: per-block latency of the host-synchronous streaming call
(taches_process, one block per call), the roofline of the dominant kernel
(timed with HIP events that the library records on its launch stream right
around the kernel launch, taches_set_timing), and the CPU oracle on a
bounded sample of the same workload.
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

FP32_PEAK_TFLOPS = 157.3        # MI355X published FP32 vector peak
HBM_PEAK_GBS = 8000.0

# HBM traffic of the main kernel per launch, from two rocprofv3 --pmc runs of
# this benchmark (FETCH_SIZE, then WRITE_SIZE, KiB per dispatch), each scaled
# by what the same counter reads for a plain device copy of 1 GiB (FETCH_SIZE
# reads half the bytes copied, WRITE_SIZE all of them).  Valid only for the
# kernel source the counters were taken on (SHA-256 of k_gather.hip followed
# by taches_internal.h); reported as null once that source has changed.
TRAFFIC_COUNTERS = {
    "kernel": "k_gather<16,4,float>",
    "source_sha256": "7d81db9338a09f9b097027d78f32ed5ce33f059a64ff532897edebacc14977dd",
    "fetch_kib": 9986.6, "fetch_scale": 2.0,
    "write_kib": 4006.0, "write_scale": 1.0,
}


def measured_traffic_bytes(kernel: str):
    import hashlib
    c = TRAFFIC_COUNTERS
    if kernel != c["kernel"]:
        return None
    src = os.path.join(ROOT, "paper_2401_01607_amd", "csrc")
    h = hashlib.sha256()
    for f in ("k_gather.hip", "taches_internal.h"):
        with open(os.path.join(src, f), "rb") as fh:
            h.update(fh.read())
    if h.hexdigest() != c["source_sha256"]:
        return None
    return round(1024 * (c["fetch_kib"] * c["fetch_scale"] + c["write_kib"] * c["write_scale"]))


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=20)
    p.add_argument("--warmup", type=int, default=3)
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--cpu-seconds", type=float, default=12.0, help="target oracle sample duration")
    p.add_argument("--latency-blocks", type=int, default=400)
    p.add_argument("--tile", type=str, default="", help="force gather tile 'R,W'")
    p.add_argument("--calibrate-copy", type=int, default=0, metavar="MB",
                   help="only run a plain device copy of MB megabytes (HBM counter calibration)")
    p.add_argument("--no-extras", action="store_true",
                   help="skip the multichannel, batched and latency comparisons")
    p.add_argument("--only", type=str, default="", help="run one extra section only (c1, c3, c4, c5, f2, f4; f3 runs only when named)")
    p.add_argument("--device-warmup-s", type=float, default=1.5,
                   help="seconds of untimed steps before the warm-up steps (device clock ramp)")
    return p.parse_args()


def calibrate_copy(mb: int) -> None:
    """A plain device-to-device copy of known size, for scaling the HBM byte
    counters (FETCH_SIZE, WRITE_SIZE) of a profiler run."""
    import torch
    n = mb * (1 << 20) // 4
    a = torch.ones(n, device="cuda:0")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_each_way": n * 4, "copies": 3}), flush=True)


def main():
    args = parse()
    if args.calibrate_copy:
        calibrate_copy(args.calibrate_copy)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU only; --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import torch
    from paper_2401_01607_amd import taches as T
    from paper_2401_01607_amd import workloads as W

    torch.cuda.set_device(0)
    dev = torch.device("cuda:0")
    spec = W.config2()
    B, L = spec.block, spec.max_ir_len
    nb = spec.n_blocks()                       # 1875
    nb_drain = -(-(L - 1) // B)                # 256
    macs = spec.direct_macs()                  # 480 000 * 65 536
    xp = np.zeros(nb * B, np.float32)
    xp[: spec.n_samples] = spec.x[0]
    x_dev = torch.from_numpy(xp).to(dev)[None]
    y_dev = torch.empty_like(x_dev)
    yt_dev = torch.empty((1, nb_drain * B), dtype=torch.float32, device=dev)
    irs_dev = [torch.from_numpy(h).to(dev) for h in spec.irs]
    sched = np.full(nb, -1, np.int32)
    for b, k in spec.schedule:
        sched[b] = k

    s = T.Stream(B, L, max_blocks_per_call=max(nb, nb_drain), ir_slots=2)
    tune = None
    if args.tile:
        r, w = (int(v) for v in args.tile.split(","))
        s.set_tile(r, w)
    stream = torch.cuda.current_stream()

    main_tile = []

    def step(i):
        s.load_ir_slot(0, irs_dev[0])                # a1: IR staging (device copies)
        s.load_ir_slot(1, irs_dev[1])
        s.set_timing(True)                           # HIP events around the kernel launch
        s.process_blocks(x_dev, y_dev, nb, sched)    # a2-a4: all blocks, IR schedule
        s.set_timing(False)
        if not main_tile:
            mi = s.info()
            main_tile.extend([mi.tile_r, mi.tile_w])
        s.process_blocks(None, yt_dev, nb_drain)     # temporal overflow

    if not args.tile:
        # empirical tile choice on this call shape (untimed; every tile gives
        # the same bits).  It runs first: the tuner synchronizes after every
        # candidate, and the idle gaps let the device clock fall again.
        from paper_2401_01607_amd import autotune
        best, tried = autotune.tune_stream(B, L, 1, nb, T.TACHES_PREC_FP32, cache=None, warm_s=1.0)
        s.set_tile(*best)
        tune = {"tile": list(best), "ms_by_tile": {k: round(v, 4) for k, v in sorted(tried.items(), key=lambda kv: kv[1])[:6]}}
    # bring the device out of its idle clock state: run whole steps for
    # --device-warmup-s seconds before the W warm-up steps (the kernel's clock
    # ramps up over its first ~second of work; the timed region is unchanged)
    t_warm = time.perf_counter()
    while time.perf_counter() - t_warm < args.device_warmup_s:
        for _ in range(20):
            step(0)
        torch.cuda.synchronize()
    for i in range(args.warmup):
        step(i)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.warmup, args.warmup + args.steps):
        step(i)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    info = s.info()
    k_ms = s.call_times(args.steps)               # the timed steps' main calls
    assert len(k_ms) == args.steps
    k_avg_s = float(np.mean(k_ms)) / 1e3
    assert info.live == 0, "the drain must leave an empty tail"

    gmacs = macs / dt / 1e9
    flops = 2.0 * macs
    fma_ceiling = T.taches_fp32_fma_ceiling(0)
    achieved_tflops = flops / k_avg_s / 1e12

    # ---- per-block latency, host-synchronous streaming call ----------------
    lat = []
    sl = T.Stream(B, L)
    sl.set_ir(spec.irs[0])
    y_blk = np.zeros(B, np.float32)
    for b in range(min(args.latency_blocks, nb)):
        xb = np.ascontiguousarray(xp[b * B:(b + 1) * B])
        t1 = time.perf_counter()
        rc = T.taches_process(sl.h, xb, y_blk)
        lat.append(time.perf_counter() - t1)
        assert rc == 0
    lat_us = np.array(lat[10:]) * 1e6
    sl.close()

    # ---- per-block device time, asynchronous calls -------------------------
    sa = T.Stream(B, L)
    sa.set_ir(irs_dev[0])
    xb_dev = x_dev[0, : 64 * B].reshape(64, B)
    yb_dev = torch.empty_like(xb_dev)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for b in range(8):
        sa.process_async(xb_dev[b], yb_dev[b])
    e0.record(stream)
    for b in range(64):
        sa.process_async(xb_dev[b], yb_dev[b])
    e1.record(stream)
    torch.cuda.synchronize()
    per_block_async_us = e0.elapsed_time(e1) / 64 * 1e3
    sa.close()

    out = {
        "metric": "GMAC/s direct-conv equiv + p99 block latency; split-BF16/batched vs plain FP32",
        "value": round(gmacs, 2),
        "unit": "GMAC/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(dt * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "1 mono stream, 480000 Gaussian samples (10 s @ 48 kHz), two decaying-noise IRs "
                        "L=65536 swapped every 4800 samples (99 swaps), block 256, plus L-1 drain",
            "block_size": B, "ir_len": L, "samples": spec.n_samples, "ir_swaps": len(spec.schedule) - 1,
            "direct_macs": macs, "tile": main_tile, "tail": "fp64" if info.tail_fp64 else "fp32",
            "tile_autotune": tune,
        },
        "roofline": {
            "bound": "alu",
            "kernel": f"k_gather<{main_tile[0]},{main_tile[1]},float>",
            "achieved": round(achieved_tflops, 3),
            "peak": FP32_PEAK_TFLOPS,
            "unit": "TFLOP/s",
            "frac": round(achieved_tflops / FP32_PEAK_TFLOPS, 4),
            "traffic": measured_traffic_bytes(f"k_gather<{main_tile[0]},{main_tile[1]},float>"),
            "kernel_ms": round(k_avg_s * 1e3, 4),
            "flops_per_launch": flops,
            # the unpacked-FMA issue ceiling measured on this device (the
            # library is built without packed FP32, which the peak counts)
            "fma_ceiling_tflops": round(fma_ceiling, 1),
            "frac_of_fma_ceiling": round(achieved_tflops / fma_ceiling, 4) if fma_ceiling > 0 else None,
        },
        "block_latency_us": {
            "mode": "host-synchronous taches_process, host buffers, B=256, L=65536",
            "p50": round(float(np.percentile(lat_us, 50)), 2),
            "p99": round(float(np.percentile(lat_us, 99)), 2),
            "max": round(float(np.max(lat_us)), 2),
            "deadline_us": round(B / 48_000 * 1e6, 1),
            "async_device_us_per_block": round(per_block_async_us, 2),
        },
    }

    if not args.no_extras:
        out["extras"] = extras(args)

    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(spec, args.cpu_seconds)

    print(json.dumps(out), flush=True)
    s.close()


def _timed(fn, reps=3, warm=1):
    """Median wall time of fn() (synchronized) over reps runs."""
    import torch
    for _ in range(warm):
        fn()
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        t0 = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t0)
    return float(np.median(ts))


def extra_c1_latency():
    """Plain taches, 1 mono stream, L = 1024, B = 64: host-synchronous
    per-block latency (taches_process with host buffers)."""
    from paper_2401_01607_amd import taches as T
    from paper_2401_01607_amd import workloads as W
    spec = W.config1()
    B = spec.block
    s = T.Stream(B, spec.max_ir_len)
    s.set_ir(spec.irs[0])
    y = np.zeros(B, np.float32)
    lat = []
    for b in range(spec.n_blocks()):
        xb = np.ascontiguousarray(spec.x[0, b * B:(b + 1) * B])
        if xb.size < B:
            xb = np.pad(xb, (0, B - xb.size))
        t0 = time.perf_counter()
        assert T.taches_process(s.h, xb, y) == 0
        lat.append(time.perf_counter() - t0)
    s.close()
    us = np.array(lat[20:]) * 1e6
    return {"workload": "1 mono stream, 48000 uniform samples, L=1024, B=64, one taches_process per block",
            "p50_us": round(float(np.percentile(us, 50)), 2), "p99_us": round(float(np.percentile(us, 99)), 2),
            "max_us": round(float(us.max()), 2), "deadline_us": round(B / 48_000 * 1e6, 1),
            "gmacs": round(spec.direct_macs() / float(np.sum(lat)) / 1e9, 3)}


def extra_c3_split_vs_fp32():
    """64 channels x 240 000 samples sharing one IR of 2^18 taps, B = 512:
    split-BF16 Toeplitz MFMA (FP64 tail) vs the FP32 gather (FP64 tail),
    whole signal in one call each, device-resident."""
    import torch
    from paper_2401_01607_amd import taches as T
    from paper_2401_01607_amd import workloads as W
    spec = W.config3()
    B, L, C = spec.block, spec.max_ir_len, spec.channels
    nb = spec.n_blocks()
    macs = spec.direct_macs()
    xp = np.zeros((C, nb * B), np.float32)
    xp[:, :spec.n_samples] = spec.x
    xd = torch.from_numpy(xp).cuda()
    res = {"workload": "64 channels x 240000 Gaussian samples, one decaying-noise IR L=262144, B=512, "
                       "469 blocks in one call", "direct_macs": macs}
    outs = {}
    for name, prec in (("split_bf16", T.TACHES_PREC_SPLIT_BF16), ("fp32", T.TACHES_PREC_FP32)):
        s = T.Stream(B, L, channels=C, max_blocks_per_call=nb, precision=prec)
        s.set_ir(spec.irs[0])
        yd = torch.empty_like(xd)

        def run():
            # each run starts from an empty tail: drain is not part of it
            s.process_blocks(xd, yd, nb)
        run()
        torch.cuda.synchronize()
        # reopen so every timed run starts from the same empty tail
        s.close()
        s = T.Stream(B, L, channels=C, max_blocks_per_call=nb, precision=prec)
        s.set_ir(spec.irs[0])
        st = torch.cuda.current_stream()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(st)
        s.process_blocks(xd, yd, nb)
        e1.record(st)
        torch.cuda.synchronize()
        sec = e0.elapsed_time(e1) / 1e3
        info = s.info()
        res[name] = {"ms": round(sec * 1e3, 3), "gmacs": round(macs / sec / 1e9, 1),
                     "tail": "fp64" if info.tail_fp64 else "fp32"}
        if name == "split_bf16":
            # MFMA work: three BF16 products per direct MAC (plus Toeplitz padding)
            res[name]["mfma_tflops_bf16"] = round(3 * 2 * macs / sec / 1e12, 1)
            res[name]["frac_of_bf16_dense_peak"] = round(3 * 2 * macs / sec / 2.5e15, 4)
        else:
            res[name]["tflops"] = round(2 * macs / sec / 1e12, 2)
            res[name]["tile"] = [info.tile_r, info.tile_w]
        outs[name] = yd.clone()
        s.close()
    d = (outs["split_bf16"].double() - outs["fp32"].double()).abs().max().item()
    rms = outs["fp32"].double().pow(2).mean().sqrt().item()
    res["speedup_split_over_fp32"] = round(res["fp32"]["ms"] / res["split_bf16"]["ms"], 2)
    res["max_abs_split_minus_fp32_over_rms"] = float(f"{d / rms:.3e}")
    return res


def extra_c4_batched_vs_plain():
    """512 independent mono streams of 96 000 samples, L log-uniform in
    [256, 131072], B in {32..512}: every stream's whole input in one pool
    step (one persistent launch replayed from a hipGraph) vs one
    taches_process_blocks launch per stream."""
    import torch
    from paper_2401_01607_amd import taches as T
    from paper_2401_01607_amd import workloads as W
    Ls, Bs = W.config4_draws()
    n = 96_000
    nbs = [-(-n // B) for B in Bs]
    macs = sum(n * L for L in Ls)
    xs, ys = [], []
    for i, (L, B) in enumerate(zip(Ls, Bs)):
        xp = np.zeros(nbs[i] * B, np.float32)
        xp[:n] = W.signal_gauss(n, 410_000 + i)
        xs.append(torch.from_numpy(xp).cuda()[None])
        ys.append(torch.empty_like(xs[-1]))
    irs = [W.impulse_response(L, 420_000 + i) for i, L in enumerate(Ls)]

    def open_streams():
        ss = []
        for i, (L, B) in enumerate(zip(Ls, Bs)):
            s = T.Stream(B, L, max_blocks_per_call=nbs[i])
            s.set_ir(irs[i])
            ss.append(s)
        return ss

    res = {"workload": "512 mono streams x 96000 Gaussian samples, L log-uniform [256, 131072], "
                       "B from {32..512}, whole input per stream", "direct_macs": macs}
    # plain: one launch per stream
    ss = open_streams()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s, x, y, nb in zip(ss, xs, ys, nbs):
        s.process_blocks(x, y, nb)
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t0
    alone = [ys[i].clone() for i in range(0, 512, 64)]
    for s in ss:
        s.close()
    # batched: one pool step per repetition, replayed from the pool's graph;
    # the per-lane tile is first tuned on the same step (untimed)
    timings, dev_ms = [], []
    pool = T.Pool(512, 1 << 40, use_graph=True)

    def one_step():
        st = open_streams()
        for s in st:
            pool.attach(s)
        pool.step(st, xs, ys, nbs)
        for s in st:
            pool.detach(s)
            s.close()
    from paper_2401_01607_amd import autotune
    tuned_r, tuned_ms = autotune.tune_pool(pool, one_step)
    for rep in range(4):
        ss = open_streams()
        for s in ss:
            pool.attach(s)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        pool.step(ss, xs, ys, nbs)
        torch.cuda.synchronize()
        timings.append(time.perf_counter() - t0)
        info = pool.info()
        dev_ms.append(info.last_device_ms)
        for s in ss:
            pool.detach(s)
            s.close()
    pool.close()
    timings = timings[1:]  # the first step also captures the graph
    t_batch = float(np.median(timings))
    t_dev = float(np.median(dev_ms[1:])) / 1e3
    same = all(torch.equal(a, ys[i * 64]) for i, a in enumerate(alone))
    res["plain"] = {"ms": round(t_plain * 1e3, 2), "gmacs": round(macs / t_plain / 1e9, 1)}
    res["batched"] = {"ms": round(t_batch * 1e3, 2), "gmacs": round(macs / t_batch / 1e9, 1),
                      "tflops": round(2 * macs / t_batch / 1e12, 2),
                      "frac_of_fp32_peak": round(2 * macs / t_batch / 1e12 / FP32_PEAK_TFLOPS, 4),
                      "tile_r": info.last_r, "items": info.last_items, "workgroups": info.last_workgroups,
                      "plan_ms": round(info.last_plan_ms, 2), "imbalance": round(info.last_imbalance, 4),
                      "graph_replays": int(info.graph_replays),
                      "device_ms": round(t_dev * 1e3, 2),
                      "device_tflops": round(2 * macs / t_dev / 1e12, 2),
                      "device_frac_of_fp32_peak": round(2 * macs / t_dev / 1e12 / FP32_PEAK_TFLOPS, 4)}
    res["batched"]["tile_autotune"] = {"r": tuned_r, "device_ms_by_r": {str(k): round(v, 3) for k, v in tuned_ms.items()}}
    res["speedup_batched_over_plain"] = round(t_plain / t_batch, 2)
    res["batched_equals_alone_bitwise"] = bool(same)
    return res


def extra_c5_serving(duration_s=30.0, warmup_s=10.0):
    """Poisson arrivals (200 / s) of mono/stereo streams lasting 10-60 s, IRs
    log-uniform in [512, 262144] taps, IR swaps at 0.5 / s, B in {32..512},
    up to 4096 streams admitted by HBM budget, real-time paced at 48 kHz,
    continuous batching through one pool (graph replays)."""
    from paper_2401_01607_amd import workloads as W
    from paper_2401_01607_amd.serving import GpuExecutor, Scheduler
    reqs = W.config5_requests(horizon_s=duration_s)
    ex = GpuExecutor(max_streams=4096, hbm_budget_bytes=64 << 30, use_graph=True)
    sch = Scheduler(reqs, ex, warmup_s=warmup_s)
    st = sch.run_realtime(duration_s)
    info = ex.pool.info()
    st["gpu_busy_fraction"] = round(ex.device_s / st["wall_s"], 3)
    ex.close()
    st.update({"workload": "Poisson 200 streams/s, 10-60 s, mono/stereo, L log-U[512, 262144], swaps 0.5/s, "
                           "B from {32..512}, <= 4096 streams, 64 GiB budget, FP32, real-time 48 kHz",
               "run_s": duration_s, "warmup_s": warmup_s, "last_step_items": info.last_items,
               "last_plan_ms": round(info.last_plan_ms, 2), "graph_replays": int(info.graph_replays)})
    # FP32 against split-BF16 at a reduced load (20 streams/s): split-BF16
    # streams run their Toeplitz MFMA kernel one launch per stream inside
    # each step, and a mono or stereo stream fills only 1-2 of its 32
    # padded channel columns, so the full load is served in FP32
    st["precision_at_20_per_s"] = {}
    from paper_2401_01607_amd import taches as T
    for name, prec in (("fp32", T.TACHES_PREC_FP32), ("split_bf16", T.TACHES_PREC_SPLIT_BF16)):
        r2 = W.config5_requests(horizon_s=10.0, rate_hz=20.0, seed=502)
        ex2 = GpuExecutor(max_streams=4096, hbm_budget_bytes=64 << 30, use_graph=True, precision=prec)
        s2 = Scheduler(r2, ex2, warmup_s=3.0).run_realtime(10.0)
        ex2.close()
        st["precision_at_20_per_s"][name] = {
            k: s2[k] for k in ("admitted", "latency_ms_p50", "latency_ms_p99", "latency_ms_max",
                               "deadline_misses", "deadline_miss_fraction", "gmacs", "step_busy_fraction") if k in s2}
    return st


def extra_f4_zero_bypass():
    """The main step's stream with every other 4 800-sample period silent
    (exact zeros): chunks of zeros skip their multiply-adds (exact-zero
    bypass).  Same call as the main step, timed with HIP events."""
    import torch
    from paper_2401_01607_amd import taches as T
    from paper_2401_01607_amd import workloads as W
    spec = W.config2()
    B, L = spec.block, spec.max_ir_len
    nb = spec.n_blocks()
    sched = np.full(nb, -1, np.int32)
    for b, k in spec.schedule:
        sched[b] = k
    full = np.zeros(nb * B, np.float32)
    full[:spec.n_samples] = spec.x[0]
    quiet = full.copy()
    for p0 in range(4800, quiet.size, 9600):
        quiet[p0:p0 + 4800] = 0
    zero_blocks = int(sum(not quiet[b * B:(b + 1) * B].any() for b in range(nb)))
    irs = [torch.from_numpy(h).cuda() for h in spec.irs]
    res = {"workload": "main-step stream, every other 4800-sample period silent",
           "silent_blocks": zero_blocks, "blocks": nb}
    for name, xp in (("full", full), ("half_silent", quiet)):
        x = torch.from_numpy(xp).cuda()[None]
        y = torch.empty_like(x)
        s = T.Stream(B, L, max_blocks_per_call=nb, ir_slots=2)
        for k in range(2):
            s.load_ir_slot(k, irs[k])
        ts = []
        for rep in range(8):
            s.reset()
            for k in range(2):
                s.load_ir_slot(k, irs[k])
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            s.process_blocks(x, y, nb, sched)
            e1.record()
            torch.cuda.synchronize()
            if rep >= 2:
                ts.append(e0.elapsed_time(e1))
        s.close()
        res[name + "_ms"] = round(float(np.median(ts)), 4)
    res["speedup"] = round(res["full_ms"] / res["half_silent_ms"], 2)
    return res


def extra_f3_capacity():
    """Real-time capacity on one GPU, the counterpart of the paper's
    real-time limit filter length (Section 5.1, Figs. 7-13; Table 2).
    A: one mono stream, host-synchronous taches_process per block (host
    buffers, PCIe round trip included): per-block time against the block
    period B/fs for growing L; the longest real-time L is extrapolated
    linearly from the longest L measured.  B: pools of N identical mono
    streams advancing one block each per step (one batched launch, graph
    replay): step time against the block period; the real-time stream count
    is extrapolated linearly from the largest N."""
    import torch
    from paper_2401_01607_amd import taches as T
    from paper_2401_01607_amd import workloads as W
    fs = float(W.FS)
    out = {"single_stream": [], "pool": []}
    for B in (256, 8192):
        for L in (1 << 16, 1 << 18, 1 << 20, 1 << 22):
            s = T.Stream(B, L)
            s.set_ir(W.impulse_response(L, 700 + L % 97))
            x = W.signal_gauss(B, 701)[None]
            y = np.zeros_like(x)
            ts = []
            for k in range(25):
                t0 = time.perf_counter()
                assert T.taches_process(s.h, x, y) == 0
                ts.append(time.perf_counter() - t0)
            s.close()
            t = float(np.median(ts[5:]))
            out["single_stream"].append({"B": B, "L": L, "ms_per_block": round(t * 1e3, 4),
                                         "period_ms": round(B / fs * 1e3, 3), "real_time": t < B / fs,
                                         "gmacs": round(B * L / t / 1e9, 1)})
        last = out["single_stream"][-1]
        out["single_stream_max_L_estimate_B%d" % B] = int(last["L"] * (B / fs) / (last["ms_per_block"] / 1e3))
    for L, B in ((4096, 256), (65536, 256), (262144, 1024)):
        h = torch.from_numpy(W.impulse_response(L, 702)).cuda()
        xbank = torch.from_numpy(W.signal_gauss(B * 8192, 703)).cuda()
        for N in (256, 1024, 4096):
            pool = T.Pool(N, 1 << 42, use_graph=True)
            ss = []
            for i in range(N):
                st = T.Stream(B, L)
                st.set_ir(h)
                assert pool.attach(st) == T.TACHES_OK
                ss.append(st)
            sp = np.array([st.h for st in ss], np.uint64)
            xp = np.array([xbank.data_ptr() + 4 * B * (i % 8192) for i in range(N)], np.uint64)
            ybuf = torch.empty(N * B, device="cuda")
            yp = np.array([ybuf.data_ptr() + 4 * B * i for i in range(N)], np.uint64)
            nbs = np.ones(N, np.int32)
            ts, dev = [], []
            for k in range(13):
                t0 = time.perf_counter()
                pool.step_strided(sp, xp, None, yp, None, nbs)
                pool.synchronize()
                if k >= 3:
                    ts.append(time.perf_counter() - t0)
                    dev.append(pool.info().last_device_ms)
            for st in ss:
                pool.detach(st)
                st.close()
            pool.close()
            t = float(np.median(ts))
            out["pool"].append({"L": L, "B": B, "streams": N, "step_ms": round(t * 1e3, 3),
                                "device_ms": round(float(np.median(dev)), 3), "period_ms": round(B / fs * 1e3, 3),
                                "real_time": t < B / fs, "gmacs": round(N * B * L / t / 1e9, 1)})
        last = out["pool"][-1]
        out["pool_max_streams_estimate_L%d_B%d" % (L, B)] = int(last["streams"] * (B / fs) /
                                                                 (last["step_ms"] / 1e3))
    return out


def extra_f2_offline():
    """Off-line whole-signal convolution (taches_convolve, one call over all
    blocks and the temporal overflow): the main step's signal with IR_A
    (no swaps), and a short input (0.1 s) with a long IR (2^22 taps) with
    and without exchanging the roles of input and IR."""
    import torch
    from paper_2401_01607_amd import taches as T
    from paper_2401_01607_amd import workloads as W
    res = {}
    cases = (("signal_10s_ir_65536", W.signal_gauss(480_000, 201), W.impulse_response(65_536, 202), (False,)),
             ("signal_0.1s_ir_4M", W.signal_gauss(4_800, 205), W.impulse_response(1 << 22, 206), (False, True)))
    for name, x, h, swaps in cases:
        xd = torch.from_numpy(x).cuda()
        hd = torch.from_numpy(h).cuda()
        yd = torch.empty(x.size + h.size - 1, device="cuda")
        for swap in swaps:
            ts = []
            for rep in range(4):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                assert T.taches_convolve(xd, hd, yd, role_swap=swap) == T.TACHES_OK
                ts.append(time.perf_counter() - t0)
            t = float(np.median(ts[1:]))
            res[name + ("_roles_exchanged" if swap else "")] = {
                "ms": round(t * 1e3, 3), "gmacs": round(x.size * h.size / t / 1e9, 1)}
    return res


def extras(args):
    out = {}
    sections = {"c1": extra_c1_latency, "c3": extra_c3_split_vs_fp32, "c4": extra_c4_batched_vs_plain,
                "c5": extra_c5_serving, "f2": extra_f2_offline, "f4": extra_f4_zero_bypass}
    if args.only == "f3":
        sections = {"f3": extra_f3_capacity}     # on request only: about a minute
    for name, fn in sections.items():
        if args.only and args.only != name:
            continue
        t0 = time.perf_counter()
        out[name] = fn()
        out[name]["section_s"] = round(time.perf_counter() - t0, 1)
    return out


def cpu_baseline(spec, target_s):
    """The FP64 oracle (paper's buffer loop, one thread: one stream) on the
    first blocks of the same workload, sized to about ``target_s`` seconds."""
    from oracle import oracle as O
    B = spec.block
    probe = 8
    t0 = time.perf_counter()
    O.run_channel(spec.x[0][: probe * B], spec.irs, spec.schedule, B, spec.max_ir_len, n_blocks=probe)
    per_block = (time.perf_counter() - t0) / probe
    nblk = int(max(probe, min(spec.n_blocks(), target_s / max(per_block, 1e-9))))
    t0 = time.perf_counter()
    O.run_channel(spec.x[0][: nblk * B], spec.irs, spec.schedule, B, spec.max_ir_len, n_blocks=nblk)
    el = time.perf_counter() - t0
    # direct MACs of the sample: every input sample scatters the active L taps
    macs = nblk * B * spec.max_ir_len
    return {"value": round(macs / el / 1e9, 4), "unit": "GMAC/s", "cores": 1, "kind": "oracle",
            "sample": f"first {nblk} blocks ({nblk * B} samples, {el:.1f} s) of the same stream, "
                      "FP64 buffer-form oracle, single thread"}


if __name__ == "__main__":
    main()
