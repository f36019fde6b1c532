"""Empirical tile autotuner for the gather kernels.

The library chooses a gather tile for every call from a cost model (R
outputs per lane, W waves per tile, launch order; ``taches_set_tile`` can
force one) and, for a batched pool step, one per-lane tile R from the number
of work items (``taches_pool_set_tile`` can force one).  The autotuner
measures instead of modelling: it times candidate tiles on the real call
shape or on the real pool step, with the library's device timing (HIP
events recorded on the launch stream around the kernel launches), and keeps
the fastest.  Every tile gives the same bits (a fixed summation order, see
``csrc/k_gather.hip``), so a tuned choice changes only the speed.

Choices are cached in a JSON file keyed by the device name and the call
shape, with the IR length and the block count of a call bucketed to powers
of two; ``TuneCache(None)`` keeps them in memory only.
"""
from __future__ import annotations

import json
import os
import statistics
import time

DEFAULT_CACHE = os.environ.get("TACHES_TUNE_CACHE",
                               os.path.join(os.path.expanduser("~"), ".cache", "taches", "tune.json"))

STREAM_CANDIDATES = tuple((r, w) for r in (16, 14, 12, 8, 4) for w in (4, 2, 1))
POOL_CANDIDATES = (16, 12, 8, 4)


def _pow2(v: int) -> int:
    return 1 << max(0, int(v - 1).bit_length())


class TuneCache:
    """Tuned choices by key; persisted as JSON when a path is given."""

    def __init__(self, path: str | None = DEFAULT_CACHE):
        self.path = path
        self.data: dict = {}
        if path and os.path.exists(path):
            try:
                with open(path) as f:
                    self.data = json.load(f)
            except (OSError, ValueError):
                self.data = {}

    def get(self, key: str):
        return self.data.get(key)

    def put(self, key: str, value) -> None:
        self.data[key] = value
        if not self.path:
            return
        try:
            os.makedirs(os.path.dirname(self.path) or ".", exist_ok=True)
            tmp = self.path + ".tmp"
            with open(tmp, "w") as f:
                json.dump(self.data, f, indent=1, sort_keys=True)
            os.replace(tmp, self.path)
        except OSError:
            pass          # a read-only cache location only loses persistence


def _device_tag() -> str:
    import torch
    return torch.cuda.get_device_name(torch.cuda.current_device()).replace(" ", "_")


def stream_key(block: int, ir_len: int, channels: int, n_blocks: int, precision: int) -> str:
    return f"stream/{_device_tag()}/B{block}/L{_pow2(ir_len)}/C{channels}/n{_pow2(n_blocks)}/p{precision}"


def tune_stream(block: int, ir_len: int, channels: int = 1, n_blocks: int = 1, precision: int = 0,
                candidates=STREAM_CANDIDATES, reps: int = 3, cache: TuneCache | None = None, seed: int = 77,
                warm_s: float = 0.3):
    """Time every candidate (R, W) on a scratch stream of this shape: one
    call of n_blocks blocks of seeded noise through an IR of ir_len
    decaying-noise taps, from an empty tail.  The device first runs such
    calls for `warm_s` seconds (its clock ramps up under load); then the
    candidates are timed in `reps` interleaved rounds, so that a drifting
    clock affects them alike, and each keeps its median.  Returns
    ((R, W), {"R,W": ms}); the split-BF16 path has no gather tile and
    returns (None, {})."""
    import numpy as np
    import torch
    from . import taches as T
    from . import workloads as W
    if precision == T.TACHES_PREC_SPLIT_BF16:
        return None, {}
    key = stream_key(block, ir_len, channels, n_blocks, precision)
    if cache is not None:
        hit = cache.get(key)
        if hit:
            return tuple(hit["tile"]), hit["ms"]
    rng = np.random.default_rng(seed)
    x = torch.from_numpy((rng.standard_normal((channels, n_blocks * block)) * 0.25).astype(np.float32)).cuda()
    y = torch.empty_like(x)
    h = torch.from_numpy(W.impulse_response(ir_len, seed + 1)).cuda()
    s = T.Stream(block, ir_len, channels=channels, max_blocks_per_call=n_blocks, precision=precision)
    samples = {f"{r},{w}": [] for r, w in candidates}

    def call(tile):
        s.set_tile(*tile)
        s.reset()
        s.set_ir(h)
        s.process_blocks(x, y, n_blocks)
    try:
        t0 = time.perf_counter()
        while True:                               # warm the device, and every candidate once
            for tile in candidates:
                call(tile)
            torch.cuda.synchronize()
            if time.perf_counter() - t0 >= warm_s:
                break
        for _ in range(reps):
            for r, w in candidates:
                s.set_timing(True)
                call((r, w))
                s.set_timing(False)
                samples[f"{r},{w}"].extend(s.call_times(1))
    finally:
        s.close()
    times = {k: float(statistics.median(v)) for k, v in samples.items()}
    best = min(times, key=times.get)
    tile = tuple(int(v) for v in best.split(","))
    if cache is not None:
        cache.put(key, {"tile": list(tile), "ms": times})
    return tile, times


def tune_pool(pool, run_step, candidates=POOL_CANDIDATES, cache: TuneCache | None = None, key: str | None = None):
    """Time each candidate per-lane tile R on a pool step: `run_step()` runs
    one step on a fresh state (the same step every time); each candidate is
    run twice and the device time of the second launch is kept (the first
    also captures the pool's graph).  Leaves the fastest R set on the pool
    and returns (R, {R: ms})."""
    if cache is not None and key is not None:
        hit = cache.get(key)
        if hit:
            pool.set_tile(int(hit["r"]))
            return int(hit["r"]), {int(k): v for k, v in hit["ms"].items()}
    times = {}
    for r in candidates:
        pool.set_tile(r)
        run_step()
        run_step()
        pool.synchronize()
        times[r] = float(pool.info().last_device_ms)
    best = min(times, key=times.get)
    pool.set_tile(best)
    if cache is not None and key is not None:
        cache.put(key, {"r": best, "ms": {str(k): v for k, v in times.items()}})
    return best, times
