"""Serving: continuous batching of real-time audio streams on one GPU.

Requests (audio streams with their own block size, channel count and
impulse-response length) arrive over time.  A request is admitted when a
stream slot is free and its device bytes fit the HBM budget; until then it
waits in a FIFO queue.  An admitted stream delivers one block of B samples
every B / fs seconds (real-time pacing).  Each scheduler tick gathers every
block that has arrived, over all admitted streams, into one batched step
(one persistent launch through the library's pool), so requests that arrive
while others are running join the next step.  IR changes requested during
a stream apply to its next block (Abstract; Section 6).  When a stream's
input ends, its temporal overflow (L - 1 samples, Section 4.1) is drained
with zero-input blocks, then the stream retires and frees its slot and bytes.

Per block the scheduler records latency = time its output is ready minus
time its last input sample arrived; the deadline is one block period.

The Scheduler holds all the policy and is independent of the device: the
executor it drives is GpuExecutor here (library pool) or a stub in tests.
"""
from __future__ import annotations

import math
import time
from collections import deque
from dataclasses import dataclass, field

import numpy as np

from . import workloads as W


class AdmissionRefused(Exception):
    """The executor has no free slot or not enough HBM budget right now."""


@dataclass
class Active:
    req: W.ServingRequest
    handle: object
    start_s: float              # admission time: the stream's first sample time
    n_in: int                   # input blocks
    n_drain: int                # zero-input blocks for the temporal overflow
    next_block: int = 0
    ir_version: int = 0
    swap_blocks: list = field(default_factory=list)  # block index of each applied swap

    @property
    def n_total(self) -> int:
        return self.n_in + self.n_drain

    def block_ready_s(self, k: int, fs: float) -> float:
        """Time the last sample of block k has arrived (drain blocks: at the
        end of the input)."""
        k_in = min(k, self.n_in - 1)
        return self.start_s + (k_in + 1) * self.req.block / fs

    def block_start_s(self, k: int, fs: float) -> float:
        return self.start_s + k * self.req.block / fs


@dataclass
class Stats:
    latencies_s: list = field(default_factory=list)    # per block (after warm-up)
    deadlines_s: list = field(default_factory=list)
    queue_waits_s: list = field(default_factory=list)
    admitted: int = 0
    completed: int = 0
    steps: int = 0
    blocks: int = 0
    macs: int = 0                                       # direct-equivalent MACs of input blocks
    busy_s: float = 0.0
    max_active: int = 0
    refused_attempts: int = 0
    max_range: int = 0                                  # most blocks of one stream in one step

    def summary(self, wall_s: float) -> dict:
        lat = np.array(self.latencies_s) * 1e3
        dl = np.array(self.deadlines_s) * 1e3
        out = {
            "admitted": self.admitted, "completed": self.completed, "steps": self.steps, "blocks": self.blocks,
            "max_active_streams": self.max_active, "wall_s": round(wall_s, 2),
            "gmacs": round(self.macs / wall_s / 1e9, 2) if wall_s > 0 else 0.0,
            "step_busy_fraction": round(self.busy_s / wall_s, 3) if wall_s > 0 else 0.0,
            "max_blocks_in_a_range": self.max_range,
        }
        if lat.size:
            out.update({"latency_ms_p50": round(float(np.percentile(lat, 50)), 3),
                        "latency_ms_p99": round(float(np.percentile(lat, 99)), 3),
                        "latency_ms_max": round(float(lat.max()), 3),
                        "deadline_misses": int(np.sum(lat > dl)),
                        "deadline_miss_fraction": round(float(np.mean(lat > dl)), 5)})
        if self.queue_waits_s:
            q = np.array(self.queue_waits_s)
            out.update({"queue_wait_s_p50": round(float(np.percentile(q, 50)), 3),
                        "queue_wait_s_p99": round(float(np.percentile(q, 99)), 3)})
        return out


class Scheduler:
    """Admission, pacing, IR swaps, batching and retirement."""

    def __init__(self, requests, executor, fs: float = W.FS, max_blocks_per_step=None,
                 warmup_s: float = 0.0, step_cost_s=None, min_tick_s: float = 0.0):
        self.pending = deque(sorted(requests, key=lambda r: r.arrival_s))
        self.queue: deque = deque()
        self.active: dict = {}
        self.ex = executor
        self.fs = fs
        # blocks of one stream per step: the executor's limit unless given
        self.max_blocks_per_step = max_blocks_per_step or getattr(executor, "max_blocks_per_step", 1)
        self.warmup_s = warmup_s
        self.stats = Stats()
        self.history: dict = {}   # rid -> Active after retirement (swap blocks etc.)
        # simulated clock: a step takes step_cost_s; None = measured wall time
        self.step_cost_s = step_cost_s
        # a step starts at least min_tick_s after the previous one started, so
        # that blocks arriving meanwhile are batched (trades latency for
        # fewer, larger steps)
        self.min_tick_s = min_tick_s
        self._last_step_s = -1e30

    # -- one tick --------------------------------------------------------
    def tick(self, now: float) -> bool:
        """Advance to time `now`; returns True if a step was run."""
        if now < self._last_step_s + self.min_tick_s:
            return False
        while self.pending and self.pending[0].arrival_s <= now:
            self.queue.append(self.pending.popleft())
        while self.queue:
            req = self.queue[0]
            try:
                handle = self.ex.admit(req)
            except AdmissionRefused:
                self.stats.refused_attempts += 1
                break
            self.queue.popleft()
            n_in = max(1, math.ceil(req.n_samples() / req.block))
            n_drain = math.ceil((req.ir_len - 1) / req.block)
            self.active[req.rid] = Active(req, handle, now, n_in, n_drain)
            self.stats.admitted += 1
            if req.arrival_s >= self.warmup_s:
                self.stats.queue_waits_s.append(now - req.arrival_s)
        self.stats.max_active = max(self.stats.max_active, len(self.active))
        batch = []
        for a in self.active.values():
            if a.next_block >= a.n_total or a.block_ready_s(a.next_block, self.fs) > now:
                continue
            # IR swaps due by the start of this block apply to it
            t_block = a.block_start_s(a.next_block, self.fs) - a.start_s
            while a.ir_version < len(a.req.swap_times_s) and a.req.swap_times_s[a.ir_version] <= t_block \
                    and a.next_block < a.n_in:
                a.ir_version += 1
                self.ex.set_ir(a.handle, a.req, a.ir_version)
                a.swap_blocks.append(a.next_block)
            # catch up on every block that has arrived, in one range that
            # stops before the next due swap (it applies to the block that
            # starts the next range) and at the end of the input (drain
            # blocks have no input)
            k0 = a.next_block
            stop = a.n_in if k0 < a.n_in else a.n_total
            next_swap = a.req.swap_times_s[a.ir_version] \
                if k0 < a.n_in and a.ir_version < len(a.req.swap_times_s) else math.inf
            n = 1
            while n < self.max_blocks_per_step and k0 + n < stop \
                    and a.block_ready_s(k0 + n, self.fs) <= now \
                    and not (next_swap <= a.block_start_s(k0 + n, self.fs) - a.start_s):
                n += 1
            batch.append((a, k0, n))
        if not batch:
            return False
        self._last_step_s = now
        t0 = time.perf_counter()
        self.ex.step([(a.handle, a.req, k0, n) for a, k0, n in batch])   # outputs ready on return
        elapsed = time.perf_counter() - t0
        self.stats.busy_s += elapsed
        done_s = now + (elapsed if self.step_cost_s is None else self.step_cost_s)
        self.stats.steps += 1
        for a, k0, n in batch:
            for k in range(k0, k0 + n):
                if a.block_ready_s(k, self.fs) >= self.warmup_s:
                    self.stats.latencies_s.append(done_s - a.block_ready_s(k, self.fs))
                    self.stats.deadlines_s.append(a.req.block / self.fs)
                if k < a.n_in:
                    self.stats.macs += a.req.block * a.req.ir_len * a.req.channels
            self.stats.blocks += n
            self.stats.max_range = max(self.stats.max_range, n)
            a.next_block += n
        for rid in [rid for rid, a in self.active.items() if a.next_block >= a.n_total]:
            a = self.active.pop(rid)
            self.ex.retire(a.handle, a.req)
            self.history[rid] = a
            self.stats.completed += 1
        return True

    # -- drivers -----------------------------------------------------------
    def run_realtime(self, duration_s: float, clock=time.perf_counter, sleep=time.sleep) -> dict:
        t0 = clock()
        while True:
            now = clock() - t0
            if now >= duration_s:
                break
            if not self.tick(now):
                nxt = self._next_event_s(now)
                if nxt is not None and nxt > now:
                    sleep(min(nxt - now, 0.0005))
        return self.stats.summary(clock() - t0)

    def run_simulated(self, duration_s: float) -> dict:
        """Event-driven clock: jump to the next arrival or block; each step
        takes `step_cost_s` of simulated time (0 if unset)."""
        if self.step_cost_s is None:
            self.step_cost_s = 0.0
        now = 0.0
        while now < duration_s:
            if self.tick(now):
                now += self.step_cost_s
                continue
            nxt = self._next_event_s(now)
            if nxt is None:
                break
            now = max(nxt, now + 1e-9)
        return self.stats.summary(duration_s)

    def _next_event_s(self, now):
        cands = []
        if self.pending:
            cands.append(self.pending[0].arrival_s)
        for a in self.active.values():
            if a.next_block < a.n_total:
                cands.append(a.block_ready_s(a.next_block, self.fs))
        if not cands:
            return None
        # nothing can run before the minimum tick interval has passed
        return max(min(cands), self._last_step_s + self.min_tick_s)


class GpuExecutor:
    """Runs the scheduler's steps on the library's pool.

    Input audio comes from one seeded two-channel noise bank in HBM, planar
    [2][70 s]: request r reads channels [0, C) from a seeded sample offset
    on, its duration rounded up to whole blocks.  A step over blocks
    k0 .. k0+n-1 of a stream passes the bank slice that starts at block k0,
    with the bank's channel stride, so no input is copied; drain blocks have
    no input.  IRs are built on the device from a seeded noise bank: tap n of
    version v of request r is irbank[(r.seed + v) mod NB][n] *
    exp(-6.91 n / L), normalised to unit L2 norm.  Outputs of the requests
    listed in keep_outputs go to a [C][n_total*B] buffer per request, the
    others to a scratch buffer reused by every step.  Retired streams are
    reset and reused for later requests with the same (B, channels,
    IR-length class); idle ones count against the HBM budget and are closed
    when a new stream needs their bytes."""

    BANK_SECONDS = 70.0
    DEFAULT_MAX_BLOCKS = 64

    def __init__(self, max_streams: int, hbm_budget_bytes: int, precision: int = 0, use_graph: bool = True,
                 ir_bank: int = 16, max_ir_len: int = 262_144, seed: int = 9, keep_outputs=(),
                 max_blocks_per_step: int = DEFAULT_MAX_BLOCKS):
        import torch
        from . import taches as T
        self.T, self.torch = T, torch
        self.pool = T.Pool(max_streams, hbm_budget_bytes, use_graph=use_graph)
        self.precision = precision
        self.max_blocks_per_step = max_blocks_per_step
        n = int(self.BANK_SECONDS * W.FS)
        noise = np.stack([W.signal_gauss(n, seed * 100 + c) for c in range(2)])
        self.bank = torch.from_numpy(noise).cuda()
        self.bank_len = n
        self.bank_addr = self.bank.data_ptr()
        self.irbank = torch.from_numpy(np.stack([W.impulse_response(max_ir_len, seed * 1000 + k, decay=0.0)
                                                 for k in range(ir_bank)])).cuda()
        self.max_ir_len = max_ir_len
        self.free: dict = {}
        self.live: dict = {}
        self.keep = set(keep_outputs)
        self.kept: dict = {}
        self.slots_used = 0
        self.max_streams = max_streams
        self.budget = hbm_budget_bytes
        self.idle_bytes = 0          # recycled streams not attached (counted against the budget)
        self.scratch = torch.empty(1 << 20, device="cuda")

    @staticmethod
    def ir_class(L: int) -> int:
        return 1 << max(0, (L - 1).bit_length())

    def ir(self, req, version: int):
        torch = self.torch
        L = req.ir_len
        base = self.irbank[(req.seed + version) % self.irbank.shape[0], :L]
        env = torch.exp(-W.DECAY * torch.arange(L, device="cuda", dtype=torch.float64) / L)
        v = base.double() * env
        return (v / torch.linalg.vector_norm(v)).float().contiguous()

    @staticmethod
    def n_input_blocks(req) -> int:
        return max(1, math.ceil(req.n_samples() / req.block))

    def input_offset(self, req) -> int:
        span = self.n_input_blocks(req) * req.block
        return ((req.seed * 7919) % ((self.bank_len - span) // 64 + 1)) * 64

    def input_signal(self, req):
        """[C][n_in * B] input of a request (a view of the bank)."""
        off = self.input_offset(req)
        return self.bank[:req.channels, off:off + self.n_input_blocks(req) * req.block]

    def admit(self, req):
        T = self.T
        key = (req.block, req.channels, min(self.ir_class(req.ir_len), self.max_ir_len))
        if self.slots_used >= self.max_streams:
            raise AdmissionRefused("slots")
        lst = self.free.get(key)
        if lst:
            s = lst.pop()
            self.idle_bytes -= s.info().device_bytes
        else:
            cfg = T.taches_config_default(req.block, key[2])
            cfg.channels = req.channels
            cfg.max_blocks_per_call = self.max_blocks_per_step
            cfg.precision = self.precision
            need = T.taches_bytes_for(cfg)
            used = self.pool.info().used_bytes
            # close idle recycled streams (largest first) until the new one fits
            while used + self.idle_bytes + need > self.budget and self.idle_bytes > 0:
                k_big = max((k for k in self.free if self.free[k]), key=lambda k: k[2])
                victim = self.free[k_big].pop()
                self.idle_bytes -= victim.info().device_bytes
                victim.close()
            if used + self.idle_bytes + need > self.budget:
                raise AdmissionRefused("budget")
            s = T.Stream(req.block, key[2], channels=req.channels, max_blocks_per_call=self.max_blocks_per_step,
                         precision=self.precision)
        rc = self.pool.attach(s)
        if rc != T.TACHES_OK:
            self.free.setdefault(key, []).append(s)
            self.idle_bytes += s.info().device_bytes
            raise AdmissionRefused(T.STATUS_NAMES.get(rc, rc))
        s.set_ir(self.ir(req, 0))
        n_in = self.n_input_blocks(req)
        n_total = n_in + math.ceil((req.ir_len - 1) / req.block)
        y = None
        if req.rid in self.keep:
            y = self.torch.empty((req.channels, n_total * req.block), device="cuda")
        x_addr = self.bank_addr + 4 * self.input_offset(req)
        self.live[req.rid] = (s, x_addr, n_in, y, key)
        self.slots_used += 1
        return req.rid

    def set_ir(self, handle, req, version: int):
        self.live[handle][0].set_ir(self.ir(req, version))

    def step(self, batch) -> None:
        n = len(batch)
        sp = np.empty(n, np.uint64)
        xp = np.zeros(n, np.uint64)
        yp = np.empty(n, np.uint64)
        ycs = np.zeros(n, np.int64)
        nbs = np.empty(n, np.int32)
        scratch_n = sum(req.channels * req.block * nb for h, req, k0, nb in batch if self.live[h][3] is None)
        if scratch_n > self.scratch.numel():
            self.scratch = self.torch.empty(scratch_n, device="cuda")
        sa = self.scratch.data_ptr()
        pos = 0
        for i, (handle, req, k0, nb) in enumerate(batch):
            s, x_addr, n_in, y, _ = self.live[handle]
            B = req.block
            sp[i] = s.h
            if k0 < n_in:
                xp[i] = x_addr + 4 * k0 * B
            if y is not None:
                yp[i] = y.data_ptr() + 4 * k0 * B
                ycs[i] = y.shape[1]
            else:
                yp[i] = sa + 4 * pos
                pos += req.channels * B * nb
            nbs[i] = nb
        self.pool.step_strided(sp, xp, np.full(n, self.bank_len, np.int64), yp, ycs, nbs)
        self.pool.synchronize()

    def retire(self, handle, req):
        s, x_addr, n_in, y, key = self.live.pop(handle)
        if y is not None:
            C, B = req.channels, req.block
            xin = self.input_signal(req).cpu().numpy()
            self.kept[handle] = (xin.reshape(C, n_in, B).transpose(1, 0, 2).copy(),
                                 y.cpu().numpy().reshape(C, -1, B).transpose(1, 0, 2).copy())
        self.pool.detach(s)
        s.reset()
        self.free.setdefault(key, []).append(s)
        self.idle_bytes += s.info().device_bytes
        self.slots_used -= 1

    def close(self):
        for s, *_ in self.live.values():
            self.pool.detach(s)
            s.close()
        self.live.clear()
        for lst in self.free.values():
            for s in lst:
                s.close()
        self.free.clear()
        self.pool.close()
