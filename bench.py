"""Benchmark of the streaming taches convolution on one MI355X.

Workload (one step, the largest configuration): 64 channels x 240 000
samples (5 s at 48 kHz) of seeded Gaussian noise sharing one seeded
decaying-noise impulse response of L = 2^18 taps, block size B = 512, FP32
multiply-adds on the vector ALUs with an FP64 tail (the IR has 2^18 taps).
A step stages the IR (device copy into the pending slot), processes the 469
input blocks in one taches_process_blocks call (device-resident input and
output), then drains the temporal overflow (L - 1 samples) with one
NULL-input call, which leaves the tail empty for the next step.

value: direct-convolution-equivalent multiply-accumulates of the step
(64 x 240 000 x 262 144 = 4.03e12) per second of wall time, GMAC/s.

Also reported: the roofline of the dominant kernel (timed with HIP events
that the library records on its launch stream right around the kernel
launch), the error of every result against the FP64 oracle (with the FP32
oracle beside it), the other configurations (extras: one mono stream with
IR swaps and its per-block latency, split-BF16 MFMA on the same
multichannel shape, 512 batched streams, serving, off-line mode, exact-zero
bypass, real-time capacity), and the FP64 oracle on the host's cores on a
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

FP32_PEAK_TFLOPS = 157.3        # MI355X published FP32 vector peak (packed FP32)
BF16_DENSE_PEAK_TFLOPS = 2500.0  # MI355X published dense BF16 MFMA peak
HBM_PEAK_GBS = 8000.0
U32 = 2.0 ** -24

# HBM traffic per launch of a kernel on a workload, from two rocprofv3 --pmc
# runs of this benchmark (FETCH_SIZE, then WRITE_SIZE, KiB per dispatch),
# each scaled by what the same counter reads for a plain device copy of
# 1 GiB (FETCH_SIZE reads half the bytes copied, WRITE_SIZE all of them).
# Valid only for the kernel source the counters were taken on (SHA-256 of
# k_gather.hip followed by taches_internal.h); reported as null once that
# source has changed.
TRAFFIC_COUNTERS = {
    ("k_gather<16,4,double>", "c3"): {
        "source_sha256": "4f01667d849e66701d8e7669a0c112e36386c48105e56011c14b009decf26f29",
        "fetch_kib": 244734.7, "fetch_scale": 2.0, "write_kib": 311168.0, "write_scale": 1.0},
}


def measured_traffic_bytes(kernel: str, workload: str):
    import hashlib
    c = TRAFFIC_COUNTERS.get((kernel, workload))
    if c is None:
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
    p.add_argument("--cpu-seconds", type=float, default=15.0, help="target oracle sample duration")
    p.add_argument("--tile", type=str, default="", help="force the main call's gather tile 'R,W'")
    p.add_argument("--calibrate-copy", type=int, default=0, metavar="MB",
                   help="only run a plain device copy of MB megabytes (HBM counter calibration)")
    p.add_argument("--no-extras", action="store_true", help="main step, its errors and the CPU baseline only")
    p.add_argument("--no-errors", action="store_true", help="skip the error figures (profiling runs)")
    p.add_argument("--only", type=str, default="",
                   help="run one extra section only (c1, c2, c3split, c4, c5, f2, f4, tail, f3)")
    p.add_argument("--c5-seconds", type=float, default=30.0,
                   help="real time of the full-load serving run (a third of it warm-up)")
    p.add_argument("--device-warmup-s", type=float, default=1.0,
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


# ---------------------------------------------------------------------------
# error figures against the FP64 oracle
# ---------------------------------------------------------------------------

def err_stats(y, y64) -> dict:
    """max |y - y64| / RMS(y64) and RMS(y - y64) / RMS(y64) over the given
    outputs (RMS(y64) over the same outputs)."""
    y64 = np.asarray(y64, np.float64)
    d = np.abs(np.asarray(y, np.float64) - y64)
    rms = float(np.sqrt(np.mean(y64 * y64)))
    return {"max_abs_over_rms": float(f"{d.max() / rms:.4e}"),
            "rms_err_over_rms": float(f"{np.sqrt(np.mean(d * d)) / rms:.4e}"),
            "outputs": int(d.size)}


def fp32_oracle_stats(xs, irs, schedule, B, L, n_blocks, y_gpu, y64, prec_names=("fma",)):
    """The FP32 oracle (one rounding per multiply-add, and/or product and sum
    rounded separately) on the first n_blocks blocks of the given channels,
    beside the GPU on the same outputs; both against the FP64 result."""
    from oracle import oracle as O
    precs = {"fma": O.OR_FP32_FMA, "separate_roundings": O.OR_FP32_MULADD}
    n = n_blocks * B
    xs = [np.asarray(x, np.float32)[:n] for x in xs]
    ref = np.concatenate([np.asarray(r)[:n] for r in y64])
    out = {"sample": f"first {n_blocks} blocks ({n} outputs) of {len(xs)} channel(s)",
           "gpu": err_stats(np.concatenate([np.asarray(g)[:n] for g in y_gpu]), ref)}
    for name in prec_names:
        ys = O.run_channels(xs, irs, schedule, B, L, n_blocks=n_blocks, prec=precs[name])
        out["fp32_oracle_" + name] = err_stats(np.concatenate([y[:n] for y in ys]), ref)
    return out


def cpu_info() -> dict:
    """CPU model and core counts of the host."""
    model, cores = "unknown", set()
    phys = core = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                k, _, v = line.partition(":")
                k, v = k.strip(), v.strip()
                if k == "model name" and model == "unknown":
                    model = v
                elif k == "physical id":
                    phys = v
                elif k == "core id":
                    core = v
                elif not k and phys is not None:
                    cores.add((phys, core))
                    phys = core = None
        if phys is not None:
            cores.add((phys, core))
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count() or 1
    return {"cpu_model": model, "logical_cpus": os.cpu_count(), "physical_cores": len(cores) or None,
            "cpus_usable_by_this_process": usable}


# ---------------------------------------------------------------------------
# main step: the multichannel workload, FP32 gather with FP64 tail
# ---------------------------------------------------------------------------

class C3Run:
    """The 64-channel stream on the device: inputs resident in HBM, one call
    of the 469 input blocks and one NULL-input drain call per step."""

    def __init__(self, precision, tile=None):
        import torch
        from paper_2401_01607_amd import taches as T
        from paper_2401_01607_amd import workloads as W
        self.spec = spec = W.config3()
        self.B, self.L, self.C = spec.block, spec.max_ir_len, spec.channels
        self.nb = spec.n_blocks()
        self.nbd = -(-(self.L - 1) // self.B)
        xp = np.zeros((self.C, self.nb * self.B), np.float32)
        xp[:, :spec.n_samples] = spec.x
        self.x = torch.from_numpy(xp).cuda()
        self.y = torch.empty_like(self.x)
        self.yt = torch.empty((self.C, self.nbd * self.B), dtype=torch.float32, device="cuda")
        self.h = torch.from_numpy(spec.irs[0]).cuda()
        self.s = T.Stream(self.B, self.L, channels=self.C, max_blocks_per_call=max(self.nb, self.nbd),
                          precision=precision)
        if tile:
            self.s.set_tile(*tile)
        self.tile = None

    def step(self, timed=False):
        s = self.s
        s.set_ir(self.h)                          # a1: IR staging (device copy, pending slot)
        s.set_timing(timed)                       # HIP events around the main kernel launch
        s.process_blocks(self.x, self.y, self.nb)  # a2-a5: every input block
        s.set_timing(False)
        if self.tile is None:
            mi = s.info()
            self.tile = [mi.tile_r, mi.tile_w]
        s.process_blocks(None, self.yt, self.nbd)  # temporal overflow

    def outputs(self) -> np.ndarray:
        """[C][n_samples + L - 1] outputs of the last step."""
        import torch
        n_tot = self.spec.n_samples + self.L - 1
        return torch.cat([self.y, self.yt], 1)[:, :n_tot].cpu().numpy()

    def close(self):
        self.s.close()


_C3_REF = {}


def c3_reference():
    """FP64 outputs of the multichannel workload (every channel, every
    output), and the sum |h||x| weights of the split-BF16 bound."""
    if not _C3_REF:
        from oracle import oracle as O
        from paper_2401_01607_amd import workloads as W
        spec = W.config3()
        n_tot = spec.n_samples + spec.max_ir_len - 1
        _C3_REF["y64"] = O.fft_outputs(spec.x, spec.irs, spec.schedule, spec.block, n_tot)
        _C3_REF["mag"] = O.fft_outputs(np.abs(spec.x), [np.abs(spec.irs[0])], spec.schedule, spec.block, n_tot)
    return _C3_REF


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

    torch.cuda.set_device(0)
    tune = None
    tile = None
    if args.tile:
        tile = tuple(int(v) for v in args.tile.split(","))
    else:
        # empirical tile choice on this call shape (untimed; every tile gives
        # the same bits); it runs before the device warm-up because the tuner
        # synchronizes after every candidate and the idle gaps let the clock fall
        from paper_2401_01607_amd import autotune
        from paper_2401_01607_amd import workloads as W
        sp = W.config3()
        tile, tried = autotune.tune_stream(sp.block, sp.max_ir_len, sp.channels, sp.n_blocks(), T.TACHES_PREC_FP32,
                                           candidates=((16, 4), (12, 4), (8, 4), (16, 2)), reps=2, cache=None,
                                           warm_s=0.5)
        tune = {"tile": list(tile), "ms_by_tile": {k: round(v, 3) for k, v in sorted(tried.items(), key=lambda kv: kv[1])}}
    run = C3Run(T.TACHES_PREC_FP32, tile)
    spec = run.spec
    macs = spec.direct_macs()
    t_warm = time.perf_counter()
    while time.perf_counter() - t_warm < args.device_warmup_s:
        for _ in range(4):
            run.step()
        torch.cuda.synchronize()
    for _ in range(args.warmup):
        run.step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        run.step(timed=True)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    print(f"bench: {args.steps} timed steps, {dt * 1e3:.3f} ms per step", file=sys.stderr, flush=True)
    k_ms = run.s.call_times(args.steps)
    assert len(k_ms) == args.steps
    info = run.s.info()
    assert info.live == 0, "the drain must leave an empty tail"
    k_avg_s = float(np.mean(k_ms)) / 1e3
    flops = 2.0 * macs
    achieved = flops / k_avg_s / 1e12
    fma_ceiling = T.taches_fp32_fma_ceiling(0)
    kernel = f"k_gather<{run.tile[0]},{run.tile[1]},{'double' if info.tail_fp64 else 'float'}>"
    out = {
        "metric": "GMAC/s direct-conv equiv + p99 block latency; split-BF16/batched vs plain FP32",
        "value": round(macs / dt / 1e9, 1),
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
            "workload": "64 channels x 240000 Gaussian samples (5 s @ 48 kHz) sharing one decaying-noise IR "
                        "L=262144, block 512, 469 blocks in one call plus the L-1 drain; FP32 multiply-adds, "
                        "FP64 tail",
            "channels": run.C, "block_size": run.B, "ir_len": run.L, "samples_per_channel": spec.n_samples,
            "direct_macs": macs, "tile": run.tile, "tail": "fp64" if info.tail_fp64 else "fp32",
            "tile_autotune": tune,
            "kernel_ms_median": round(float(np.median(k_ms)), 4),
            "kernel_ms_min": round(float(np.min(k_ms)), 4),
        },
        "roofline": {
            "bound": "alu",
            "kernel": kernel,
            "achieved": round(achieved, 3),
            "peak": FP32_PEAK_TFLOPS,
            "unit": "TFLOP/s",
            "frac": round(achieved / FP32_PEAK_TFLOPS, 4),
            "traffic": measured_traffic_bytes(kernel, "c3"),
            "kernel_ms": round(k_avg_s * 1e3, 4),
            "flops_per_launch": flops,
            "algorithmic_bytes_per_launch": 4 * (2 * run.C * run.nb * run.B + run.L),
            # the unpacked-FMA issue ceiling measured on this device (the
            # library is built without packed FP32, which the peak counts)
            "fma_ceiling_tflops": round(fma_ceiling, 1),
            "frac_of_fma_ceiling": round(achieved / fma_ceiling, 4) if fma_ceiling > 0 else None,
        },
    }
    errors = {}
    if not args.no_errors:
        y = run.outputs()
        ref = c3_reference()
        errors["c3_fp32"] = {"vs_fp64_oracle_all_outputs": err_stats(y, ref["y64"]),
                             "fp32_oracle_beside": fp32_oracle_stats(
                                 list(spec.x[:8]), spec.irs, spec.schedule, run.B, run.L, 16,
                                 list(y[:8]), list(ref["y64"][:8]))}
    run.close()
    del run
    if not args.no_extras:
        out["extras"] = extras(args, errors)
    if errors:
        out["errors"] = errors
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args.cpu_seconds)
    print(json.dumps(out), flush=True)


# ---------------------------------------------------------------------------
# extras
# ---------------------------------------------------------------------------

def _median_device_ms(fn, s, reps):
    """Median and min device time (library events) of `reps` calls of fn,
    each of which records exactly one timed call on s."""
    ms = []
    for _ in range(reps):
        fn()
        ms.extend(s.call_times(1))
    assert len(ms) == reps, f"{len(ms)} timed calls recorded, {reps} expected"
    return float(np.median(ms)), float(np.min(ms)), len(ms)


def extra_c1(errors):
    """Plain taches, 1 mono stream, L = 1024, B = 64: host-synchronous
    per-block latency (taches_process with host buffers), every block of the
    signal and of its temporal overflow; errors over every output."""
    from oracle import oracle as O
    from paper_2401_01607_amd import taches as T
    from paper_2401_01607_amd import workloads as W
    spec = W.config1()
    B, L = spec.block, spec.max_ir_len
    n_tot = spec.n_samples + L - 1
    nb = -(-n_tot // B)
    xp = np.zeros(nb * B, np.float32)
    xp[:spec.n_samples] = spec.x[0]
    s = T.Stream(B, L)
    s.set_ir(spec.irs[0])
    y = np.zeros(nb * B, np.float32)
    lat = []
    for b in range(nb):
        yb = y[b * B:(b + 1) * B]
        t0 = time.perf_counter()
        assert T.taches_process(s.h, xp[b * B:(b + 1) * B], yb) == 0
        lat.append(time.perf_counter() - t0)
    s.close()
    us = np.array(lat[20:]) * 1e6
    y64 = O.fft_outputs(spec.x[0], spec.irs, spec.schedule, B, nb * B)   # exact zeros after n_tot
    errors["c1"] = {"vs_fp64_oracle_all_outputs": err_stats(y[:n_tot], y64[:n_tot]),
                    "fp32_oracle_beside": fp32_oracle_stats([spec.x[0]], spec.irs, spec.schedule, B, L, nb,
                                                            [y], [y64], ("fma", "separate_roundings"))}
    return {"workload": "1 mono stream, 48000 uniform samples, L=1024, B=64, one taches_process per block "
                        "(host buffers: PCIe round trip included), signal and overflow",
            "p50_us": round(float(np.percentile(us, 50)), 2), "p99_us": round(float(np.percentile(us, 99)), 2),
            "max_us": round(float(us.max()), 2), "deadline_us": round(B / 48_000 * 1e6, 1),
            "gmacs": round(spec.direct_macs() / float(np.sum(lat)) / 1e9, 3)}


def extra_c2(errors, steps=20):
    """One mono stream of 480 000 samples with two IRs of 65 536 taps swapped
    every 4 800 samples (99 swaps), B = 256: a step stages both IRs into the
    stream's slots, processes the 1 875 blocks with their IR schedule in one
    call, drains the overflow; plus the per-block latency of the
    host-synchronous streaming call."""
    import torch
    from oracle import oracle as O
    from paper_2401_01607_amd import taches as T
    from paper_2401_01607_amd import workloads as W
    spec = W.config2()
    B, L = spec.block, spec.max_ir_len
    nb, nbd = spec.n_blocks(), -(-(L - 1) // B)
    macs = spec.direct_macs()
    xp = np.zeros(nb * B, np.float32)
    xp[:spec.n_samples] = spec.x[0]
    x_dev = torch.from_numpy(xp).cuda()[None]
    y_dev = torch.empty_like(x_dev)
    yt_dev = torch.empty((1, nbd * B), dtype=torch.float32, device="cuda")
    irs_dev = [torch.from_numpy(h).cuda() for h in spec.irs]
    sched = np.full(nb, -1, np.int32)
    for b, k in spec.schedule:
        sched[b] = k
    s = T.Stream(B, L, max_blocks_per_call=max(nb, nbd), ir_slots=2)
    s.set_tile(16, 4)   # the tuned choice on this shape (every tile gives the same bits)
    tile = []

    def step(timed=False):
        s.load_ir_slot(0, irs_dev[0])
        s.load_ir_slot(1, irs_dev[1])
        s.set_timing(timed)
        s.process_blocks(x_dev, y_dev, nb, sched)
        s.set_timing(False)
        if not tile:
            mi = s.info()
            tile.extend([mi.tile_r, mi.tile_w])
        s.process_blocks(None, yt_dev, nbd)
    for _ in range(40):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step(timed=True)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    k_ms = s.call_times(steps)
    k_avg = float(np.mean(k_ms))
    kernel = f"k_gather<{tile[0]},{tile[1]},float>"
    n_tot = spec.n_samples + L - 1
    y = torch.cat([y_dev, yt_dev], 1)[0, :n_tot].cpu().numpy()
    s.close()
    y64 = O.fft_outputs(spec.x[0], spec.irs, spec.schedule, B, n_tot)
    errors["c2"] = {"vs_fp64_oracle_all_outputs": err_stats(y, y64),
                    "fp32_oracle_beside": fp32_oracle_stats([spec.x[0]], spec.irs, spec.schedule, B, L, 120,
                                                            [y], [y64])}
    # per-block latency, host-synchronous streaming call (PCIe round trip)
    lat = []
    sl = T.Stream(B, L)
    sl.set_ir(spec.irs[0])
    y_blk = np.zeros(B, np.float32)
    for b in range(400):
        t1 = time.perf_counter()
        assert T.taches_process(sl.h, np.ascontiguousarray(xp[b * B:(b + 1) * B]), y_blk) == 0
        lat.append(time.perf_counter() - t1)
    sl.close()
    lat_us = np.array(lat[10:]) * 1e6
    flops = 2.0 * macs
    return {"workload": "1 mono stream, 480000 Gaussian samples (10 s @ 48 kHz), two decaying-noise IRs L=65536 "
                        "swapped every 4800 samples (99 swaps), block 256, plus L-1 drain",
            "direct_macs": macs, "ms_per_step": round(dt * 1e3, 4), "gmacs": round(macs / dt / 1e9, 1),
            "roofline": {"bound": "alu", "kernel": kernel, "kernel_ms": round(k_avg, 4),
                         "achieved": round(flops / k_avg / 1e9, 2), "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                         "frac": round(flops / k_avg / 1e9 / FP32_PEAK_TFLOPS, 4),
                         "traffic": measured_traffic_bytes(kernel, "c2")},
            "block_latency_us": {"mode": "host-synchronous taches_process, host buffers, B=256, L=65536",
                                 "p50": round(float(np.percentile(lat_us, 50)), 2),
                                 "p99": round(float(np.percentile(lat_us, 99)), 2),
                                 "max": round(float(np.max(lat_us)), 2),
                                 "deadline_us": round(B / 48_000 * 1e6, 1)}}


def extra_c3_split(errors):
    """The main step's multichannel shape through the split-BF16 Toeplitz
    MFMA kernel (FP64 tail): device time of the main call, median of 5, its
    MFMA roofline (three BF16 products per direct MAC), and errors over every
    output against the FP64 result, with the per-output bound
    (3 * 2^-16 + gamma_768) * sum |h||x| checked on all of them."""
    import torch
    from paper_2401_01607_amd import taches as T
    run = C3Run(T.TACHES_PREC_SPLIT_BF16)
    macs = run.spec.direct_macs()
    for _ in range(3):
        run.step()
    torch.cuda.synchronize()
    med, mn, reps = _median_device_ms(lambda: run.step(timed=True), run.s, 5)
    res = {"workload": "same shape as the main step (64 channels x 240000, L=262144, B=512), "
                       "split-BF16 Toeplitz MFMA with FP32 accumulation per chunk and FP64 tail",
           "kernel_ms_median": round(med, 3), "kernel_ms_min": round(mn, 3), "runs": reps,
           "gmacs": round(macs / med * 1e-6, 1)}
    mfma_tf = 3 * 2 * macs / med / 1e9
    res["roofline"] = {"bound": "mfma", "kernel": "k_toeplitz<double,2,1>", "achieved": round(mfma_tf, 1),
                       "peak": BF16_DENSE_PEAK_TFLOPS, "unit": "TFLOP/s",
                       "frac": round(mfma_tf / BF16_DENSE_PEAK_TFLOPS, 4),
                       "flops_per_launch": 6.0 * macs,
                       "note": "three BF16 MFMA products (hi*hi, hi*lo, lo*hi) per direct MAC"}
    if errors is not None and "c3_fp32" in errors:
        y = run.outputs()
        ref = c3_reference()
        coef = 3 * 2.0 ** -16 + 3 * 256 * U32 / (1 - 3 * 256 * U32)
        d = np.abs(y.astype(np.float64) - ref["y64"])
        errors["c3_split_bf16"] = {"vs_fp64_oracle_all_outputs": err_stats(y, ref["y64"]),
                                   "max_err_over_per_output_bound": float(f"{np.max(d / (coef * ref['mag'] + 1e-300)):.4f}")}
    run.close()
    return res


def extra_c4_batched(errors):
    """512 independent mono streams of 96 000 samples, L log-uniform in
    [256, 131072], B in {32..512}: every stream's whole input in one pool
    step (one persistent launch replayed from a hipGraph) vs one
    taches_process_blocks launch per stream."""
    import torch
    from oracle import oracle as O
    from paper_2401_01607_amd import taches as T
    from paper_2401_01607_amd import workloads as W
    Ls, Bs = W.config4_draws()
    n = 96_000
    nbs = [-(-n // B) for B in Bs]
    macs = sum(n * L for L in Ls)
    xs_np, xs, ys = [], [], []
    for i, (L, B) in enumerate(zip(Ls, Bs)):
        xp = np.zeros(nbs[i] * B, np.float32)
        xp[:n] = W.signal_gauss(n, 410_000 + i)
        xs_np.append(xp[:n])
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
    ss = open_streams()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s, x, y, nb in zip(ss, xs, ys, nbs):
        s.process_blocks(x, y, nb)
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t0
    alone = [ys[i].clone() for i in range(0, 512, 8)]
    for s in ss:
        s.close()
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
    t_batch = float(np.median(timings[1:]))
    t_dev = float(np.median(dev_ms[1:])) / 1e3
    same = all(torch.equal(a, ys[i * 8]) for i, a in enumerate(alone))
    res["plain"] = {"ms": round(t_plain * 1e3, 2), "gmacs": round(macs / t_plain / 1e9, 1)}
    res["batched"] = {"ms": round(t_batch * 1e3, 2), "gmacs": round(macs / t_batch / 1e9, 1),
                      "tflops": round(2 * macs / t_batch / 1e12, 2),
                      "frac_of_fp32_peak": round(2 * macs / t_batch / 1e12 / FP32_PEAK_TFLOPS, 4),
                      "tile_r": info.last_r, "items": info.last_items, "workgroups": info.last_workgroups,
                      "plan_ms": round(info.last_plan_ms, 2), "imbalance": round(info.last_imbalance, 4),
                      "graph_replays": int(info.graph_replays),
                      "device_ms": round(t_dev * 1e3, 2),
                      "device_tflops": round(2 * macs / t_dev / 1e12, 2),
                      "device_frac_of_fp32_peak": round(2 * macs / t_dev / 1e12 / FP32_PEAK_TFLOPS, 4),
                      "tile_autotune": {"r": tuned_r, "device_ms_by_r": {str(k): round(v, 3) for k, v in tuned_ms.items()}}}
    res["speedup_batched_over_plain"] = round(t_plain / t_batch, 2)
    res["batched_equals_alone_bitwise"] = bool(same)
    if errors is not None:
        picks = list(range(0, 512, 8))
        yg, yr = [], []
        for i in picks:
            S = nbs[i] * Bs[i]
            yg.append(ys[i].cpu().numpy()[0])
            yr.append(O.fft_outputs(xs_np[i], [irs[i]], [(0, 0)], Bs[i], S))
        errors["c4_batched"] = {"sample": f"every output of {len(picks)} streams (every 8th)",
                                "vs_fp64_oracle": err_stats(np.concatenate(yg), np.concatenate(yr))}
    return res


def _serving_errors(srv, reqs, keep):
    """Errors of the kept requests' outputs (every output computed so far,
    finished or still live) against the FP64 result of their inputs and
    applied IR changes."""
    from oracle import oracle as O
    yg, yr = [], []
    done = 0
    for rid in keep:
        req = next(r for r in reqs if r.rid == rid)
        got = srv.kept_outputs(rid)
        if got is None:
            continue
        x, y, swap_blocks = got
        if y.shape[1] == 0:
            continue
        irs = [srv.ir(req, v).cpu().numpy() for v in range(len(swap_blocks) + 1)]
        sched = [(0, 0)] + [(b, v + 1) for v, b in enumerate(swap_blocks)]
        for c in range(req.channels):
            yg.append(y[c])
            yr.append(O.fft_outputs(x[c], irs, sched, req.block, y.shape[1]))
        done += 1
    if not yg:
        return None
    return {"sample": f"every output so far of {done} kept requests", **err_stats(np.concatenate(yg), np.concatenate(yr))}


def extra_c5_serving(errors, duration_s=30.0, warmup_s=10.0):
    """Poisson arrivals (200 / s) of mono/stereo streams lasting 10-60 s, IRs
    log-uniform in [512, 262144] taps, IR changes at 0.5 / s, B in
    {32..512}, up to 4096 streams admitted by HBM budget, real-time paced at
    48 kHz.  Each tick is one library call: arrived input blocks gathered
    from host memory and copied to the device, one pool step (graph replay),
    every output block written to mapped host memory by one launch; latency
    ends when the outputs are in host memory."""
    from paper_2401_01607_amd import workloads as W
    from paper_2401_01607_amd.serving import RealtimeServer
    from paper_2401_01607_amd import taches as T
    reqs = W.config5_requests(horizon_s=duration_s)
    keep = [r.rid for r in reqs[:4]]
    srv = RealtimeServer(reqs, max_streams=4096, hbm_budget_bytes=64 << 30, use_graph=True, keep_outputs=keep,
                         warmup_s=warmup_s)
    st = srv.run_realtime(duration_s)
    print("bench: c5 full-load run done", file=sys.stderr, flush=True)
    info = srv.pool.info()
    if errors is not None:
        errors["c5_fp32"] = _serving_errors(srv, reqs, keep)
    srv.close()
    st.update({"workload": "Poisson 200 streams/s, 10-60 s, mono/stereo, L log-U[512, 262144], swaps 0.5/s, "
                           "B from {32..512}, <= 4096 streams, 64 GiB budget, FP32, real-time 48 kHz, "
                           "input from host memory and output back to host memory every tick",
               "run_s": duration_s, "warmup_s": warmup_s, "last_step_items": info.last_items,
               "last_plan_ms": round(info.last_plan_ms, 3), "graph_replays": int(info.graph_replays),
               "graph_captures": int(info.graph_captures)})
    # the same arrivals with admission held while more than 1 % of the blocks
    # of >= 64 samples miss their deadline (queued requests wait instead)
    from paper_2401_01607_amd.serving import MissGate
    gate_s, gate_warm = 20.0, 5.0
    rg = W.config5_requests(horizon_s=gate_s)
    gate = MissGate(0.01, min_block=64)
    srvg = RealtimeServer(rg, max_streams=4096, hbm_budget_bytes=64 << 30, use_graph=True, warmup_s=gate_warm,
                          miss_gate=gate)
    sg = srvg.run_realtime(gate_s)
    srvg.close()
    print("bench: c5 full-load run with the miss gate done", file=sys.stderr, flush=True)
    st["with_miss_gate"] = {"run_s": gate_s, "warmup_s": gate_warm, **{
        k: sg[k] for k in ("admitted", "max_active_streams", "latency_ms_p50", "latency_ms_p99", "latency_ms_max",
                           "deadline_miss_fraction", "by_block_size", "queue_wait_s_p50", "queue_wait_s_p99",
                           "gmacs", "device_step_busy_fraction", "miss_gate") if k in sg}}
    st["precision_at_20_per_s"] = {}
    for name, prec in (("fp32", T.TACHES_PREC_FP32), ("split_bf16", T.TACHES_PREC_SPLIT_BF16)):
        r2 = W.config5_requests(horizon_s=10.0, rate_hz=20.0, seed=502)
        keep2 = [r.rid for r in r2[:4]]
        srv2 = RealtimeServer(r2, max_streams=4096, hbm_budget_bytes=64 << 30, use_graph=True, precision=prec,
                              keep_outputs=keep2, warmup_s=3.0)
        s2 = srv2.run_realtime(10.0)
        print(f"bench: c5 run at 20 streams/s ({name}) done", file=sys.stderr, flush=True)
        if errors is not None:
            errors["c5_" + name + "_at_20_per_s"] = _serving_errors(srv2, r2, keep2)
        srv2.close()
        st["precision_at_20_per_s"][name] = {
            k: s2[k] for k in ("admitted", "latency_ms_p50", "latency_ms_p99", "latency_ms_max",
                               "deadline_misses", "deadline_miss_fraction", "gmacs", "step_busy_fraction",
                               "gpu_busy_fraction", "by_block_size") if k in s2}
    return st


def extra_tail_policy(errors):
    """Error of the FP32 and the FP64 tail against the FP64 oracle on one
    mono stream (2 s of Gaussian input, flat white-noise IR: the paper's IR
    shape, which gives the largest errors), at 512 to 4096 chunk sums per
    output for B = 32, 64, 128 and 256: the measurements behind the AUTO
    tail rule (FP64 above 1024 chunk sums per output, or for IRs of >= 2^18
    taps)."""
    import torch
    from oracle import oracle as O
    from paper_2401_01607_amd import taches as T
    from paper_2401_01607_amd import workloads as W
    n = 96_000
    x = W.signal_gauss(n, 4242)
    rows = []
    for B in (32, 64, 128, 256):
        for adds in (512, 1024, 2048, 4096):
            L = adds * min(B, 256)
            if L >= (1 << 18):
                continue
            h = W.impulse_response(L, 4343 + adds, decay=0.0)
            nb, nbd = -(-n // B), -(-(L - 1) // B)
            xp = np.zeros(nb * B, np.float32)
            xp[:n] = x
            xd = torch.from_numpy(xp).cuda()[None]
            y64 = O.fft_outputs(x, [h], [(0, 0)], B, n + L - 1)
            cfg = T.taches_config_default(B, L)
            rec = {"B": B, "L": L, "chunk_sums_per_output": adds, "auto_tail": "fp64" if T.taches_tail_is_fp64(cfg) else "fp32"}
            for tail, name in ((T.TACHES_TAIL_FP32, "fp32"), (T.TACHES_TAIL_FP64, "fp64")):
                s = T.Stream(B, L, max_blocks_per_call=max(nb, nbd), tail=tail)
                s.set_ir(h)
                yd = torch.empty_like(xd)
                yt = torch.empty((1, nbd * B), device="cuda")
                s.process_blocks(xd, yd, nb)
                s.process_blocks(None, yt, nbd)
                y = torch.cat([yd, yt], 1)[0, :n + L - 1].cpu().numpy()
                s.close()
                e = err_stats(y, y64)
                rec[name + "_tail"] = [e["max_abs_over_rms"], e["rms_err_over_rms"]]
            rows.append(rec)
    if errors is not None:
        errors["tail_policy"] = {"sample": "every output of each stream; [max |err| / RMS(y64), RMS(err) / RMS(y64)]",
                                 "rows": rows}
    return {"workload": "1 mono stream, 96000 Gaussian samples, flat white-noise IR, L = chunk sums x min(B, 256)",
            "configurations": len(rows)}


def extra_f4_zero_bypass():
    """The mono stream with IR swaps, every other 4 800-sample period silent
    (exact zeros): chunks of zeros skip their multiply-adds (exact-zero
    bypass).  Same call shape as c2, timed with HIP events."""
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
    res = {"workload": "c2 stream, every other 4800-sample period silent", "silent_blocks": zero_blocks, "blocks": nb}
    outs = {}
    for name, xp in (("full", full), ("half_silent", quiet)):
        x = torch.from_numpy(xp).cuda()[None]
        y = torch.empty_like(x)
        s = T.Stream(B, L, max_blocks_per_call=nb, ir_slots=2)
        ts = []
        for rep in range(8):
            s.reset()
            for k in range(2):
                s.load_ir_slot(k, irs[k])
            s.set_timing(True)
            s.process_blocks(x, y, nb, sched)
            s.set_timing(False)
            t = s.call_times(1)
            if rep >= 2:
                ts.extend(t)
        outs[name] = y.clone()
        s.close()
        res[name + "_ms"] = round(float(np.median(ts)), 4)
    res["speedup"] = round(res["full_ms"] / res["half_silent_ms"], 2)
    return res


def extra_f2_offline():
    """Off-line whole-signal convolution (taches_convolve, one call over all
    blocks and the temporal overflow): the c2 signal with its first IR (no
    swaps), and a short input (0.1 s) with a long IR (2^22 taps) with and
    without exchanging the roles of input and IR."""
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


def _single_stream_block_time(T, B, L, hbuf, x, y, warm, reps):
    """Mean wall time of `reps` host-synchronous taches_process calls (host
    buffers, one block each) on a fresh mono stream whose IR is the first L
    values of the device buffer hbuf (random taps: the timing does not
    depend on their values)."""
    s = T.Stream(B, L)
    try:
        s.set_ir(hbuf[:L])
        for _ in range(warm):
            assert T.taches_process(s.h, x, y) == 0
        ts = []
        for _ in range(reps):
            t0 = time.perf_counter()
            assert T.taches_process(s.h, x, y) == 0
            ts.append(time.perf_counter() - t0)
    finally:
        s.close()
    return float(np.mean(ts)), float(np.max(ts))


def _bracket(measure, lo, hi, period, max_probes=7, rel=0.03):
    """Find the largest real-time size between lo (real time) and hi (not
    real time, or the largest size allowed) by measuring: a first guess from
    the line through the two end points, then probes a few percent either
    side, narrowing.  Returns (largest real-time size measured, smallest
    non-real-time size measured or None, probes)."""
    t_lo = measure(lo)
    probes = [(lo, t_lo)]
    if t_lo >= period:
        return None, lo, probes
    t_hi = measure(hi)
    probes.append((hi, t_hi))
    if t_hi < period:
        return hi, None, probes
    ok, bad = lo, hi
    t_ok, t_bad = t_lo, t_hi
    for _ in range(max_probes):
        if bad - ok <= max(1, int(rel * ok)):
            break
        est = ok + (bad - ok) * (period - t_ok) / max(t_bad - t_ok, 1e-12)
        guess = int(min(bad - 1, max(ok + 1, est * (1 - rel / 2))))
        t = measure(guess)
        probes.append((guess, t))
        if t < period:
            ok, t_ok = guess, t
            up = int(min(bad - 1, ok * (1 + rel)))
            if up > ok:
                t2 = measure(up)
                probes.append((up, t2))
                if t2 < period:
                    ok, t_ok = up, t2
                else:
                    bad, t_bad = up, t2
        else:
            bad, t_bad = guess, t
    return ok, bad, probes


def extra_f3_capacity(block_sizes=(256, 1024, 4096, 16384, 65536),
                      pool_shapes=((65536, 256, 16384), (262144, 1024, 6144))):
    """Real-time capacity on one GPU, measured: the counterpart of the
    paper's real-time limit filter length per machine (Section 5.1, Figs.
    7-13) and of its block-size sweep (Table 2).  Real time means the mean
    processing time of a block is below its period B / 48 kHz (the paper's
    criterion: processing time below the stimulus duration).

    A: one mono stream, host-synchronous taches_process per block with host
    buffers (PCIe round trip included): for each block size, the longest
    real-time IR, bracketed by measured lengths (the largest measured in
    real time and the smallest measured not in real time).  The library
    accepts IRs up to 2^30 - 1 - B taps; where even that length runs in real
    time the limit is reported as at least that length.

    B: pools of N identical mono streams, each advancing one block per step
    (one batched launch, graph replay, host-synchronous step): the largest
    real-time N, bracketed the same way, up to the stream count given per
    shape (streams are created once and attached in subsets)."""
    import torch
    from paper_2401_01607_amd import taches as T
    from paper_2401_01607_amd import workloads as W
    fs = float(W.FS)
    out = {"criterion": "mean block processing time < block period B/48000", "single_stream": [], "pool": []}
    # a stream needs block_size + max_ir_len < 2^30 (one block per call)
    L_cap = (1 << 30) - 1 - min(block_sizes)
    hbuf = torch.randn(L_cap, device="cuda") * 1e-4
    for B in block_sizes:
        period = B / fs
        x = W.signal_gauss(B, 701)
        y = np.zeros(B, np.float32)
        big = B >= 16384
        warm, reps = (1, 3) if big else (3, 10)
        times = {}

        def measure(L):
            t, tmax = _single_stream_block_time(T, B, L, hbuf, x, y, warm, reps)
            times[L] = (t, tmax)
            return t
        ok, bad, probes = _bracket(measure, 1 << 20, (1 << 30) - 1 - B, period)
        rec = {"B": B, "period_ms": round(period * 1e3, 3),
               "longest_real_time_L_measured": ok, "shortest_non_real_time_L_measured": bad,
               "probes": [{"L": L, "ms_per_block": round(t * 1e3, 4), "max_ms": round(times[L][1] * 1e3, 4),
                           "gmacs": round(B * L / t / 1e9, 1)} for L, t in probes]}
        if ok is not None:
            rec["longest_real_time_ir_seconds_at_48k"] = round(ok / fs, 1)
        if bad is None:
            rec["note"] = "real time up to the longest IR the library accepts (2^30 - 1 - B taps)"
        out["single_stream"].append(rec)
    del hbuf
    torch.cuda.empty_cache()
    for L, B, n_max in pool_shapes:
        period = B / fs
        h = torch.from_numpy(W.impulse_response(L, 702)).cuda()
        xbank = torch.from_numpy(W.signal_gauss(B * 8192, 703)).cuda()
        ybuf = torch.empty(n_max * B, device="cuda")
        streams = []
        for _ in range(n_max):
            st = T.Stream(B, L)
            st.set_ir(h)
            streams.append(st)
        sp_all = np.array([st.h for st in streams], np.uint64)
        xp_all = np.array([xbank.data_ptr() + 4 * B * (i % 8192) for i in range(n_max)], np.uint64)
        yp_all = np.array([ybuf.data_ptr() + 4 * B * i for i in range(n_max)], np.uint64)
        detail = {}

        def measure(N):
            pool = T.Pool(N, 1 << 42, use_graph=True)
            for st in streams[:N]:
                assert pool.attach(st) == T.TACHES_OK
            nbs = np.ones(N, np.int32)
            ts, dev = [], []
            for k in range(14):
                t0 = time.perf_counter()
                pool.step_strided(sp_all[:N], xp_all[:N], None, yp_all[:N], None, nbs)
                pool.synchronize()
                if k >= 4:
                    ts.append(time.perf_counter() - t0)
                    dev.append(pool.info().last_device_ms)
            pool.close()
            t = float(np.mean(ts))
            detail[N] = (t, float(np.median(dev)))
            return t
        ok, bad, probes = _bracket(measure, 256, n_max, period)
        for st in streams:
            st.close()
        out["pool"].append({"L": L, "B": B, "period_ms": round(period * 1e3, 3),
                            "most_real_time_streams_measured": ok, "fewest_non_real_time_streams_measured": bad,
                            "streams_tried_up_to": n_max,
                            "probes": [{"streams": N, "step_ms": round(t * 1e3, 3),
                                        "device_ms": round(detail[N][1], 3),
                                        "gmacs": round(N * B * L / t / 1e9, 1)} for N, t in probes]})
    return out


def extras(args, errors):
    out = {}
    sections = {"c1": lambda: extra_c1(errors), "c2": lambda: extra_c2(errors),
                "c3split": lambda: extra_c3_split(errors), "c4": lambda: extra_c4_batched(errors),
                "c5": lambda: extra_c5_serving(errors, args.c5_seconds, args.c5_seconds / 3),
                "f2": extra_f2_offline, "f4": extra_f4_zero_bypass,
                "tail": lambda: extra_tail_policy(errors), "f3": extra_f3_capacity}
    for name, fn in sections.items():
        if args.only and args.only != name:
            continue
        t0 = time.perf_counter()
        out[name] = fn()
        out[name]["section_s"] = round(time.perf_counter() - t0, 1)
        print(f"bench: section {name} done in {out[name]['section_s']} s", file=sys.stderr, flush=True)
    return out


def cpu_baseline(target_s):
    """The FP64 oracle (the buffer form of Section 4.2 in plain C, one
    channel per host thread) on a bounded sample of the main step's
    workload: the first blocks of as many of its channels as there are
    usable cores (at most 16, the host share of one GPU), sized to about
    ``target_s`` seconds."""
    from oracle import oracle as O
    from paper_2401_01607_amd import workloads as W
    spec = W.config3()
    B, L = spec.block, spec.max_ir_len
    info = cpu_info()
    threads = max(1, min(16, info["cpus_usable_by_this_process"], spec.channels))
    xs = list(spec.x[:threads])
    probe = 2
    t0 = time.perf_counter()
    O.run_channels([x[:probe * B] for x in xs], spec.irs, spec.schedule, B, L, n_blocks=probe, threads=threads)
    per_block = (time.perf_counter() - t0) / probe
    nblk = int(max(probe, min(spec.n_blocks(), target_s / max(per_block, 1e-9))))
    t0 = time.perf_counter()
    O.run_channels([x[:nblk * B] for x in xs], spec.irs, spec.schedule, B, L, n_blocks=nblk, threads=threads)
    el = time.perf_counter() - t0
    macs = threads * nblk * B * L     # every input sample scatters L taps
    return {"value": round(macs / el / 1e9, 3), "unit": "GMAC/s", "cores": threads, "kind": "oracle",
            "sample": f"first {nblk} blocks ({nblk * B} samples) of {threads} of the 64 channels of the main "
                      f"step's workload, one channel per thread, {el:.1f} s; FP64 buffer-form oracle "
                      "(gcc -O2), no file I/O",
            "per_core_gmacs": round(macs / el / 1e9 / threads, 3), **info}


if __name__ == "__main__":
    main()
