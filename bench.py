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
(timed with HIP events on the launch stream), and the CPU oracle on a
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
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1",
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
    if args.tile:
        r, w = (int(v) for v in args.tile.split(","))
        s.set_tile(r, w)
    stream = torch.cuda.current_stream()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(args.warmup + args.steps)]

    main_tile = []

    def step(i):
        s.load_ir_slot(0, irs_dev[0])                # a1: IR staging (device copies)
        s.load_ir_slot(1, irs_dev[1])
        ev[i][0].record(stream)
        s.process_blocks(x_dev, y_dev, nb, sched)    # a2-a4: all blocks, IR schedule
        ev[i][1].record(stream)
        if not main_tile:
            mi = s.info()
            main_tile.extend([mi.tile_r, mi.tile_w])
        s.process_blocks(None, yt_dev, nb_drain)     # temporal overflow

    for i in range(args.warmup):
        step(i)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.warmup, args.warmup + args.steps):
        step(i)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    info = s.info()
    k_ms = [ev[i][0].elapsed_time(ev[i][1]) for i in range(args.warmup, args.warmup + args.steps)]
    k_avg_s = float(np.mean(k_ms)) / 1e3
    assert info.live == 0, "the drain must leave an empty tail"

    gmacs = macs / dt / 1e9
    flops = 2.0 * macs
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
        },
        "roofline": {
            "bound": "alu",
            "kernel": f"k_gather<{main_tile[0]},{main_tile[1]},float>",
            "achieved": round(achieved_tflops, 3),
            "peak": FP32_PEAK_TFLOPS,
            "unit": "TFLOP/s",
            "frac": round(achieved_tflops / FP32_PEAK_TFLOPS, 4),
            "traffic": None,
            "kernel_ms": round(k_avg_s * 1e3, 4),
            "flops_per_launch": flops,
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

    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(spec, args.cpu_seconds)

    print(json.dumps(out), flush=True)
    s.close()


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
