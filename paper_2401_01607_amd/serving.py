"""Serving: continuous batching of real-time audio streams on one GPU.

Requests (audio streams with their own block size, channel count and
impulse-response length) arrive over time.  A request is admitted when a
stream slot is free and its device bytes fit the HBM budget; until then it
waits in a FIFO queue.  An admitted stream delivers one block of B samples
every B / fs seconds (real-time pacing).  Each scheduler tick gathers every
block that has arrived, over all admitted streams, into one batched step
(one persistent launch through the library's pool), so requests that arrive
while others are running join the next step, and a stream that has fallen
behind catches up with several blocks in one step.  IR changes requested
during a stream apply to the first block that starts at or after the
change (Abstract; Section 6).  When a stream's input ends, its temporal
overflow (L - 1 samples, Section 4.1) is drained with zero-input blocks,
paced like input blocks (silence keeps arriving at the sample rate until
the tail has rung out), then the stream retires and frees its slot and
bytes.

Per block the scheduler records latency = time its output is ready minus
time its last input sample arrived (for a drain block, the time its last
sample of silence would have arrived); the deadline is one block period.

The Scheduler holds all the policy and is independent of the device: the
executor it drives is GpuExecutor here (library pool) or a stub in tests.
The per-stream state it scans every tick lives in numpy arrays, so a tick
costs a fixed number of array operations plus Python work only for the
streams that are admitted, swap IRs or retire in it.

Executor interface: admit(req) -> int handle (raises AdmissionRefused),
set_ir(handle, req, version), step(handles, k0, n) with int64 arrays (stream
handles[i] processes blocks k0[i] .. k0[i]+n[i]-1; outputs ready on
return), retire(handle, req), and an attribute max_blocks_per_step.  An
executor may also offer launch(handles, k0, n) and wait() (the step split
at its device work): the scheduler then prepares its block records while
the device runs; a block still counts as done when wait() returns.
"""
from __future__ import annotations

import gc
import math
import sys
import threading
import time
from collections import deque
from dataclasses import dataclass, field

import numpy as np

from . import workloads as W


class AdmissionRefused(Exception):
    """The executor has no free slot or not enough HBM budget right now."""


@dataclass
class Active:
    """Book-keeping of one admitted request (what tests and reports read)."""
    req: W.ServingRequest
    handle: int
    start_s: float              # admission time: the stream's first sample time
    n_in: int                   # input blocks
    n_drain: int                # zero-input blocks for the temporal overflow
    next_block: int = 0
    ir_version: int = 0
    swap_blocks: list = field(default_factory=list)  # block index of each applied swap

    @property
    def n_total(self) -> int:
        return self.n_in + self.n_drain


@dataclass
class Stats:
    admitted: int = 0
    completed: int = 0
    steps: int = 0
    blocks: int = 0
    macs: int = 0                                       # direct-equivalent MACs of input blocks
    busy_s: float = 0.0
    max_active: int = 0
    refused_attempts: int = 0
    max_range: int = 0                                  # most blocks of one stream in one step
    queue_waits_s: list = field(default_factory=list)
    _lat: list = field(default_factory=list)            # per-tick arrays of block latencies (after warm-up)
    _dl: list = field(default_factory=list)             # matching deadlines
    _bs: list = field(default_factory=list)             # matching block sizes

    @property
    def latencies_s(self) -> np.ndarray:
        return np.concatenate(self._lat) if self._lat else np.zeros(0)

    @property
    def deadlines_s(self) -> np.ndarray:
        return np.concatenate(self._dl) if self._dl else np.zeros(0)

    @property
    def block_sizes(self) -> np.ndarray:
        return np.concatenate(self._bs) if self._bs else np.zeros(0, np.int64)

    def summary(self, wall_s: float) -> dict:
        lat = self.latencies_s * 1e3
        dl = self.deadlines_s * 1e3
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
            bs = self.block_sizes
            by = {}
            for b in np.unique(bs):
                m = bs == b
                lb = lat[m]
                by[str(int(b))] = {"blocks": int(m.sum()), "deadline_ms": round(float(dl[m][0]), 3),
                                   "latency_ms_p50": round(float(np.percentile(lb, 50)), 3),
                                   "latency_ms_p99": round(float(np.percentile(lb, 99)), 3),
                                   "deadline_miss_fraction": round(float(np.mean(lb > dl[m])), 5)}
            out["by_block_size"] = by
        if self.queue_waits_s:
            q = np.array(self.queue_waits_s)
            out.update({"queue_wait_s_p50": round(float(np.percentile(q, 50)), 3),
                        "queue_wait_s_p99": round(float(np.percentile(q, 99)), 3)})
        return out


class _Table:
    """Dense struct-of-arrays over the admitted streams (swap-remove)."""

    FIELDS = (("start", np.float64), ("n_in", np.int64), ("n_total", np.int64), ("nxt", np.int64),
              ("B", np.int64), ("C", np.int64), ("L", np.int64), ("swap_t", np.float64), ("handle", np.int64))

    def __init__(self, cap: int = 1024):
        self.n = 0
        self.objs: list = []
        for name, dt in self.FIELDS:
            setattr(self, name, np.zeros(cap, dt))

    def add(self, a: Active) -> None:
        if self.n == self.start.size:
            for name, dt in self.FIELDS:
                old = getattr(self, name)
                new = np.zeros(2 * old.size, dt)
                new[:old.size] = old
                setattr(self, name, new)
        i = self.n
        r = a.req
        self.start[i], self.n_in[i], self.n_total[i], self.nxt[i] = a.start_s, a.n_in, a.n_total, 0
        self.B[i], self.C[i], self.L[i] = r.block, r.channels, r.ir_len
        self.swap_t[i] = r.swap_times_s[0] if r.swap_times_s else math.inf
        self.handle[i] = a.handle
        self.objs.append(a)
        self.n += 1

    def remove(self, i: int) -> Active:
        last = self.n - 1
        a = self.objs[i]
        if i != last:
            for name, _ in self.FIELDS:
                arr = getattr(self, name)
                arr[i] = arr[last]
            self.objs[i] = self.objs[last]
        self.objs.pop()
        self.n -= 1
        return a


class Scheduler:
    """Admission, pacing, IR swaps, batching and retirement."""

    def __init__(self, requests, executor, fs: float = W.FS, max_blocks_per_step=None,
                 warmup_s: float = 0.0, step_cost_s=None, min_tick_s: float = 0.0):
        self.pending = deque(sorted(requests, key=lambda r: r.arrival_s))
        self.queue: deque = deque()
        self.tab = _Table()
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
        self._clock = None   # the real-time clock relative to its start (None: simulated)

    @property
    def active(self) -> dict:
        return {a.req.rid: a for a in self.tab.objs}

    def _admit(self, now: float) -> None:
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
            self.tab.add(Active(req, int(handle), now, n_in, n_drain))
            self.stats.admitted += 1
            if req.arrival_s >= self.warmup_s:
                self.stats.queue_waits_s.append(now - req.arrival_s)
        self.stats.max_active = max(self.stats.max_active, self.tab.n)

    # -- one tick --------------------------------------------------------
    def tick(self, now: float) -> bool:
        """Advance to time `now`; returns True if a step was run."""
        if now < self._last_step_s + self.min_tick_s:
            return False
        self._admit(now)
        t, n_act = self.tab, self.tab.n
        if n_act == 0:
            return False
        fs = self.fs
        sl = slice(0, n_act)
        start, n_in, n_total, nxt = t.start[sl], t.n_in[sl], t.n_total[sl], t.nxt[sl]
        B = t.B[sl]
        # blocks whose last sample (of input, or of silence while draining) has arrived
        arrived = np.floor((now - start) * fs / B).astype(np.int64)
        avail = np.minimum(np.maximum(arrived, 0), n_total)
        ready = avail > nxt
        if not ready.any():
            return False
        # IR swaps due by the start of a stream's next block apply to it
        due = ready & (nxt < n_in) & (t.swap_t[sl] <= nxt * B / fs)
        for i in np.nonzero(due)[0]:
            a = t.objs[i]
            k0 = int(nxt[i])
            sw = a.req.swap_times_s
            while a.ir_version < len(sw) and sw[a.ir_version] <= k0 * a.req.block / fs:
                a.ir_version += 1
                self.ex.set_ir(a.handle, a.req, a.ir_version)
                a.swap_blocks.append(k0)
            t.swap_t[i] = sw[a.ir_version] if a.ir_version < len(sw) else math.inf
        # one range per ready stream: every arrived block, at most
        # max_blocks_per_step, ending before the block at which the next swap
        # is due (it starts the next range) and at the end of the input
        # (drain blocks have no input)
        idx = np.nonzero(ready)[0]
        k0 = nxt[idx].copy()
        Bi = B[idx]
        n_in_i = n_in[idx]
        is_in = k0 < n_in_i
        end = np.minimum(avail[idx], k0 + self.max_blocks_per_step)
        end = np.where(is_in, np.minimum(end, n_in_i), end)
        swt = t.swap_t[idx]
        fin = is_in & np.isfinite(swt)
        if fin.any():
            ks = np.full(idx.size, np.iinfo(np.int64).max)
            ks[fin] = np.maximum(k0[fin] + 1, np.ceil(swt[fin] * fs / Bi[fin] - 1e-9).astype(np.int64))
            # the exact rule: the first block k with k * B / fs >= swap time
            lo = fin & (ks - 1 > k0) & (swt <= (ks - 1) * Bi / fs)
            ks[lo] -= 1
            hi = fin & (swt > ks * Bi / fs)
            ks[hi] += 1
            end = np.minimum(end, ks)
        n = end - k0
        self._last_step_s = now
        t0 = time.perf_counter()
        if hasattr(self.ex, "launch"):
            # the block records are prepared while the device runs the step
            self.ex.launch(t.handle[idx], k0, n)
            rec = self._record_begin(start[idx], k0, n, Bi, is_in, t.L[idx], t.C[idx])
            self.ex.wait()                                  # outputs ready
        else:
            self.ex.step(t.handle[idx], k0, n)              # outputs ready on return
            rec = self._record_begin(start[idx], k0, n, Bi, is_in, t.L[idx], t.C[idx])
        elapsed = time.perf_counter() - t0
        self.stats.busy_s += elapsed
        if self._clock is not None:
            done_s = self._clock()    # real time: includes this tick's host work before the step
        else:
            done_s = now + (elapsed if self.step_cost_s is None else self.step_cost_s)
        self.stats.steps += 1
        self._record_end(done_s, rec)
        t.nxt[idx] = end
        for i in sorted(np.nonzero(t.nxt[:t.n] >= t.n_total[:t.n])[0], reverse=True):
            a = t.remove(int(i))
            a.next_block = a.n_total
            self.ex.retire(a.handle, a.req)
            self.history[a.req.rid] = a
            self.stats.completed += 1
        return True

    def _record_begin(self, start, k0, n, B, is_in, L, C):
        """Counters of the step, and the arrival time and deadline of every
        block of its ranges after the warm-up (vectorized; independent of
        when the step completes)."""
        st = self.stats
        tot = int(n.sum())
        st.blocks += tot
        st.max_range = max(st.max_range, int(n.max()))
        st.macs += int(np.sum(np.where(is_in, n * B * L * C, 0)))
        rng = np.repeat(np.arange(n.size), n)
        j = np.arange(tot) - np.repeat(np.cumsum(n) - n, n)
        k = k0[rng] + j
        per = B[rng] / self.fs
        # block k is complete at start + (k+1) B / fs
        ready_s = start[rng] + (k + 1) * per
        keep = ready_s >= self.warmup_s
        return (ready_s[keep], per[keep], B[rng][keep]) if keep.any() else None

    def _record_end(self, done_s, rec) -> None:
        """Latency of every recorded block: step completion minus arrival."""
        if rec is not None:
            self.stats._lat.append(done_s - rec[0])
            self.stats._dl.append(rec[1])
            self.stats._bs.append(rec[2])

    # -- drivers -----------------------------------------------------------
    def run_realtime(self, duration_s: float, clock=time.perf_counter, sleep=time.sleep) -> dict:
        t0 = clock()
        self._clock = lambda: clock() - t0
        while True:
            now = clock() - t0
            if now >= duration_s:
                break
            if not self.tick(now):
                nxt = self._next_event_s(now)
                if nxt is not None and nxt > now:
                    sleep(min(nxt - now, 0.0005))
        self._clock = None
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
        t = self.tab
        if t.n:
            sl = slice(0, t.n)
            # the next block k of each stream is complete at start + (k + 1) B / fs
            cands.append(float(np.min(t.start[sl] + (t.nxt[sl] + 1) * t.B[sl] / self.fs)))
        if not cands:
            return None
        # nothing can run before the minimum tick interval has passed
        return max(min(cands), self._last_step_s + self.min_tick_s)


def tail_for(T, req, precision: int) -> int:
    """The tail the library's AUTO rule gives a request's own IR length
    (streams are opened with a longer capacity class, on which AUTO would
    pick FP64 for some IRs that do not need it)."""
    return tail_for_shape(T, req.block, req.ir_len, req.channels, precision)


def tail_for_shape(T, B: int, L: int, C: int, precision: int) -> int:
    cfg = T.taches_config_default(B, L)
    cfg.channels = C
    cfg.precision = precision
    return T.TACHES_TAIL_FP64 if T.taches_tail_is_fp64(cfg) == 1 else T.TACHES_TAIL_FP32


def change_blocks(req, fs: float = W.FS) -> list:
    """Input blocks at which a request's IR changes apply: the first block
    that starts at or after each change time (changes after the input do
    not apply)."""
    n_in = max(1, math.ceil(req.n_samples() / req.block))
    out = []
    for t in req.swap_times_s:
        k = max(0, math.ceil(t * fs / req.block - 1e-9))
        while k > 0 and (k - 1) * req.block / fs >= t:
            k -= 1
        while k * req.block / fs < t:
            k += 1
        if k >= n_in:
            break
        out.append(k)
    return out


def segments_for(req, precision: int, fs: float = W.FS):
    """(H, Br, Z) when a real-time request is served in two IR segments,
    else None.  The head h[0, H) is advanced every tick, the rest h[H, L)
    once per Br samples (Br a power of two, a multiple of B, H = Br), so a
    tick reads and writes about H + B tail slots of the stream instead of
    L + B.  Br is the power of two nearest sqrt(24 L), within
    [max(B, 256), 2048]: with ticks about 0.5 ms apart (24 samples at
    48 kHz) it balances the head's traffic per tick, ~ H, against the
    rest's, ~ L per Br samples.  A rest block takes at most one IR change
    inside it (the initial IR counting as one at sample 0): Br is halved
    until the request's changes fall in different rest blocks, down to
    max(B, 256) (below 256 samples a rest block would need an FP64 tail).
    Only FP32 requests whose IR is at least four rest blocks long; Z (the
    rest outputs kept on the device) lets the rest stream run up to
    4 Br + 8 B samples ahead of the outputs the head has used."""
    from . import taches as T
    if precision != T.TACHES_PREC_FP32:
        return None
    L, B = req.ir_len, req.block
    br = 1 << max(0, int(round(math.log2(math.sqrt(24.0 * L)))))
    lo = max(B, 256)
    br = max(lo, min(2048, br))
    samples = [k * B for k in change_blocks(req, fs)]

    def separated(br):
        prev = 0   # the initial IR applies from sample 0
        for smp in samples:
            if smp != prev and smp // br == prev // br:
                return False
            prev = smp
        return True
    while br > lo and not separated(br):
        br //= 2
    if L < 4 * br or not separated(br):
        return None
    return br, br, br * -(-(4 * br + 8 * B) // br)


class GpuExecutor:
    """Runs the scheduler's steps on the library's pool.

    Input audio comes from one seeded two-channel noise bank in HBM, planar
    [2][70 s]: request r reads channels [0, C) from a seeded sample offset
    on, its duration rounded up to whole blocks.  A step over blocks
    k0 .. k0+n-1 of a stream passes the bank slice that starts at block k0,
    with the bank's channel stride, so no input is copied; drain blocks have
    no input.  IR version v of request r is the first L taps of row
    (r.seed + v) mod NB of a bank of flat white-noise IRs (the paper's IR
    shape, Section 5.1), each row of unit L2 norm over max_ir_len taps, so a
    swap is one device-to-device copy.  Outputs of the requests listed in
    keep_outputs go to a [C][n_total*B] buffer per request, the others to a
    scratch buffer reused by every step.  A stream's tail type follows the
    library's AUTO rule applied to the request's own IR length.  Retired
    streams are reset and reused for later requests with the same (B,
    channels, IR-length class, tail type);
    idle ones count against the HBM budget and are closed when a new stream
    needs their bytes."""

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
        self.max_streams = max_streams
        self.budget = hbm_budget_bytes
        self.idle_bytes = 0          # recycled streams not attached (counted against the budget)
        self.scratch = torch.empty(1 << 20, device="cuda")
        # per-handle arrays read by step(); handles are reused after retire
        cap = max_streams
        self.h_stream = np.zeros(cap, np.uint64)
        self.h_x = np.zeros(cap, np.uint64)
        self.h_y = np.zeros(cap, np.uint64)
        self.h_ycs = np.zeros(cap, np.int64)
        self.h_B = np.zeros(cap, np.int64)
        self.h_C = np.zeros(cap, np.int64)
        self.h_nin = np.zeros(cap, np.int64)
        self.free_handles = list(range(cap - 1, -1, -1))

    @staticmethod
    def ir_class(L: int) -> int:
        return 1 << max(0, (L - 1).bit_length())

    def ir(self, req, version: int):
        """IR version `version` of a request (a device view, FP32)."""
        return self.irbank[(req.seed + version) % self.irbank.shape[0], :req.ir_len]

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

    def tail_for(self, req) -> int:
        return tail_for(self.T, req, self.precision)

    def admit(self, req) -> int:
        T = self.T
        tail = self.tail_for(req)
        key = (req.block, req.channels, min(self.ir_class(req.ir_len), self.max_ir_len), tail)
        if not self.free_handles:
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
            cfg.tail = tail
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
                         precision=self.precision, tail=tail)
        rc = self.pool.attach(s)
        if rc != T.TACHES_OK:
            self.free.setdefault(key, []).append(s)
            self.idle_bytes += s.info().device_bytes
            raise AdmissionRefused(T.STATUS_NAMES.get(rc, rc))
        s.set_ir(self.ir(req, 0))
        n_in = self.n_input_blocks(req)
        n_total = n_in + math.ceil((req.ir_len - 1) / req.block)
        h = self.free_handles.pop()
        y = None
        if req.rid in self.keep:
            y = self.torch.empty((req.channels, n_total * req.block), device="cuda")
        self.live[h] = (s, y, key, req)
        self.h_stream[h] = s.h
        self.h_x[h] = self.bank_addr + 4 * self.input_offset(req)
        self.h_y[h] = y.data_ptr() if y is not None else 0
        self.h_ycs[h] = y.shape[1] if y is not None else 0
        self.h_B[h], self.h_C[h], self.h_nin[h] = req.block, req.channels, n_in
        return h

    def set_ir(self, handle, req, version: int):
        self.live[handle][0].set_ir(self.ir(req, version))

    def launch(self, handles, k0, n) -> None:
        """Enqueue one pool step (stream handles[i] processes blocks k0[i] ..
        k0[i]+n[i]-1); returns once it is queued on the device."""
        B, C = self.h_B[handles], self.h_C[handles]
        adv = (4 * k0 * B).astype(np.uint64)                # byte offset of block k0
        xp = np.where(k0 < self.h_nin[handles], self.h_x[handles] + adv, np.uint64(0)).astype(np.uint64)
        yk = self.h_y[handles]
        kept = yk != 0
        m = np.where(kept, 0, C * B * n)
        need = int(m.sum())
        if need > self.scratch.numel():
            self.scratch = self.torch.empty(need, device="cuda")
        off = (4 * (np.cumsum(m) - m)).astype(np.uint64)
        yp = np.where(kept, yk + adv, np.uint64(self.scratch.data_ptr()) + off).astype(np.uint64)
        self.pool.step_strided(self.h_stream[handles], xp, np.full(handles.size, self.bank_len, np.int64), yp,
                               np.where(kept, self.h_ycs[handles], 0), n.astype(np.int32))

    def wait(self) -> None:
        """Block until the launched step's outputs are ready."""
        self.pool.synchronize()

    def step(self, handles, k0, n) -> None:
        self.launch(handles, k0, n)
        self.wait()

    @property
    def device_s(self) -> float:
        """Device time of the batched launches so far (table copy + kernel)."""
        return self.pool.info().device_ms_total / 1e3

    def retire(self, handle, req):
        s, y, key, _ = self.live.pop(handle)
        if y is not None:
            C, B = req.channels, req.block
            n_in = int(self.h_nin[handle])
            xin = self.input_signal(req).cpu().numpy()
            self.kept[req.rid] = (xin.reshape(C, n_in, B).transpose(1, 0, 2).copy(),
                                  y.cpu().numpy().reshape(C, -1, B).transpose(1, 0, 2).copy())
        self.pool.detach(s)
        s.reset()
        self.free.setdefault(key, []).append(s)
        self.idle_bytes += s.info().device_bytes
        self.h_stream[handle] = 0
        self.free_handles.append(handle)

    def kept_outputs(self, sch, rid):
        """(input [C][n_in*B], outputs so far [C][blocks done*B], blocks of the
        applied IR swaps) of a request listed in keep_outputs, retired or still
        running under scheduler `sch`; None if it was never admitted."""
        req = None
        if rid in self.kept:
            xin, ymix = self.kept[rid]
            hist = sch.history[rid]
            C = xin.shape[1]
            x = xin.transpose(1, 0, 2).reshape(C, -1)
            y = ymix.transpose(1, 0, 2).reshape(C, -1)
            return x, y, list(hist.swap_blocks)
        t = sch.tab
        for i in range(t.n):
            a = t.objs[i]
            if a.req.rid == rid:
                req = a.req
                done = int(t.nxt[i])
                s, y, _, _ = self.live[a.handle]
                self.wait()
                x = self.input_signal(req).cpu().numpy()
                yo = y[:, :done * req.block].cpu().numpy() if y is not None else None
                return (x, yo, list(a.swap_blocks)) if yo is not None else None
        return None

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


class MissGate:
    """Admission gate fed by observed deadline misses: after each batch of
    latency records it closes when more than `target` of the blocks of at
    least `min_block` samples missed their deadline (one block period), and
    reopens when the fraction falls to target / 2 or below.  While it is
    closed, queued requests wait.  Blocks of fewer than min_block samples are
    left out: at full load their period can be shorter than a step's service
    time, so they would hold the gate closed at any load.  The server records
    latencies only after its warm-up, so the gate acts from then on."""

    def __init__(self, target: float, min_block: int = 64, fs: float = W.FS):
        if not 0.0 < target < 1.0:
            raise ValueError("target must be in (0, 1)")
        self.target, self.min_block, self.fs = float(target), int(min_block), float(fs)
        self.closed = False
        self.checks = self.closed_checks = 0

    def update(self, latency_s: np.ndarray, block: np.ndarray) -> None:
        sel = np.asarray(block) >= self.min_block
        if np.any(sel):
            lat = np.asarray(latency_s, np.float64)[sel]
            frac = float(np.mean(lat > np.asarray(block, np.float64)[sel] / self.fs))
            self.closed = frac > (self.target / 2 if self.closed else self.target)
        self.checks += 1
        self.closed_checks += int(self.closed)

    def summary(self) -> dict:
        return {"target_miss_fraction": self.target, "min_block": self.min_block, "checks": self.checks,
                "closed_fraction_of_checks": round(self.closed_checks / self.checks, 4) if self.checks else 0.0}


class RealtimeServer:
    """Serving with one library call per tick (taches_server_tick).

    Python keeps what happens per request: FIFO admission when a stream
    slot is free and the stream's device bytes fit the HBM budget (streams
    recycled as in GpuExecutor), registration of the request's host input,
    output buffer and IR-change schedule with the library's server, and
    retirement of finished streams.  Everything per tick (which blocks
    have arrived, IR changes due, the ranges of blocks, gathering the
    arrived input into pinned memory, the host-to-device copy, the pool
    step, one launch writing every output block to mapped host memory,
    latency records)
    runs in one library call, which enqueues its step and then completes
    the previous one, so host and device work overlap.

    Input audio lives in host memory: a seeded two-channel noise bank,
    planar [2][70 s]; request r reads channels [0, C) from a seeded offset.
    Every request has IRs of its own: at admission its initial IR and one IR
    per scheduled change are drawn on the device (flat white noise, the
    paper's IR shape, unit L2 norm, from a generator seeded by the request)
    and kept until the request finishes (the IRs of kept requests until
    close).  Outputs of requests listed in keep_outputs are written to host
    arrays; the others are written to host staging and dropped."""

    BANK_SECONDS = 70.0

    REST_BLOCKS_PER_CALL = 4
    PREPARE_AHEAD = 32

    def __init__(self, requests, max_streams: int, hbm_budget_bytes: int, precision: int = 0,
                 use_graph: bool = True, max_ir_len: int = 262_144, seed: int = 9,
                 keep_outputs=(), max_blocks_per_step: int = 64, warmup_s: float = 0.0,
                 segments: bool = True, miss_gate: MissGate | None = None):
        import torch
        from . import taches as T
        self.T, self.torch = T, torch
        self.pending = deque(sorted(requests, key=lambda r: r.arrival_s))
        self.queue: deque = deque()
        # a two-segment request holds two streams of the pool
        slots = max_streams * (2 if segments and precision == T.TACHES_PREC_FP32 else 1)
        self.pool = T.Pool(slots, hbm_budget_bytes, use_graph=use_graph)
        self.sv = T.taches_server_create(self.pool.h, float(W.FS), max_blocks_per_step, warmup_s)
        self.precision = precision
        self.max_blocks_per_step = max_blocks_per_step
        self.warmup_s = warmup_s
        n = int(self.BANK_SECONDS * W.FS)
        self.bank = np.stack([W.signal_gauss(n, seed * 100 + c) for c in range(2)])
        self.bank_len = n
        self.irs: dict = {}          # rid -> [versions][L] device IRs of an admitted request
        self.max_ir_len = max_ir_len
        self.max_streams = max_streams
        self.budget = hbm_budget_bytes
        self.keep = set(keep_outputs)
        self.kept: dict = {}         # rid -> host output array
        self.free: dict = {}         # recycled streams by (C, B, IR capacity, tail, blocks per call, precision)
        self.segments = segments
        self.live: dict = {}         # rid -> (streams, keys, req, ring or None, device bytes)
        # admission work that does not touch the pool (opening streams,
        # drawing IRs) runs on a preparing thread during run_realtime; the
        # budget is kept here: bytes of admitted requests, of prepared ones
        # and of idle recycled streams
        self._lock = threading.Lock()
        self._to_prepare: deque = deque()
        self._prepared: dict = {}    # rid -> (streams, keys, ring, irs, device bytes)
        self._thread = None
        self._stop = False
        self._error = None           # an exception of the preparing thread
        self.live_bytes = self.reserved_bytes = self.idle_bytes = 0
        self.req_by_rid = {r.rid: r for r in requests}
        self.stats = Stats()
        self.lat, self.lat_b = [], []
        self.refused = 0
        self.loops, self.python_s = 0, 0.0   # loop iterations; time in admission and retirement
        self.n_segmented = 0
        self.slow_loops = []   # (clock, admit ms, tick ms, retire ms, admitted) of iterations over 5 ms
        self.admit_s = {"attach": 0.0, "register": 0.0}
        self.gate = miss_gate        # optional admission gate on observed deadline misses

    # -- requests ------------------------------------------------------------
    def _draw_irs(self, req):
        """[1 + swaps][L] flat white-noise IRs of unit L2 norm for a request."""
        torch = self.torch
        g = torch.Generator(device="cuda")
        g.manual_seed(int(req.seed))
        h = torch.randn((1 + len(req.swap_times_s), req.ir_len), generator=g, device="cuda", dtype=torch.float32)
        h /= torch.linalg.vector_norm(h, dim=1, keepdim=True)
        return h

    def ir(self, req, version: int):
        """IR version `version` of an admitted request (a device view, FP32)."""
        return self.irs[req.rid][version]

    @staticmethod
    def n_input_blocks(req) -> int:
        return max(1, math.ceil(req.n_samples() / req.block))

    def input_offset(self, req) -> int:
        span = self.n_input_blocks(req) * req.block
        return ((req.seed * 7919) % ((self.bank_len - span) // 64 + 1)) * 64

    def input_signal(self, req) -> np.ndarray:
        off = self.input_offset(req)
        return self.bank[:req.channels, off:off + self.n_input_blocks(req) * req.block]

    def tail_for(self, req) -> int:
        return tail_for(self.T, req, self.precision)

    def segments_for(self, req):
        """(H, Br, Z) if the request is served in two IR segments, else None."""
        return segments_for(req, self.precision) if self.segments else None

    @staticmethod
    def ir_class(L: int) -> int:
        return GpuExecutor.ir_class(L)

    def _shapes(self, req):
        """Streams a request needs: (B, IR capacity, tail, blocks per call,
        precision) of its one stream, or of its head and rest streams; and
        its segments (or None)."""
        seg = self.segments_for(req)
        C, B, L = req.channels, req.block, req.ir_len
        if seg is None:
            return [(B, min(self.ir_class(L), self.max_ir_len), self.tail_for(req), self.max_blocks_per_step,
                     self.precision)], None
        H, br, _ = seg
        T = self.T
        fp32 = T.TACHES_PREC_FP32
        head = (B, H, tail_for_shape(T, B, H, C, fp32), self.max_blocks_per_step, fp32)
        rest = (br, min(self.ir_class(L - H), self.max_ir_len), tail_for_shape(T, br, L - H, C, fp32),
                self.REST_BLOCKS_PER_CALL, fp32)
        return [head, rest], seg

    def _cfg(self, C: int, shape):
        B, cap, tail, mb, prec = shape
        cfg = self.T.taches_config_default(B, cap)
        cfg.channels = C
        cfg.max_blocks_per_call = mb
        cfg.precision = prec
        cfg.tail = tail
        return cfg

    def _prepare(self, req):
        """Everything an admission needs that does not touch the pool: the
        request's streams (recycled or new), its ring of rest outputs
        (two-segment requests) and its IRs.  The device bytes are reserved
        against the HBM budget (idle recycled streams are closed, largest
        first, to make room); AdmissionRefused if they do not fit.  Runs on
        the preparing thread."""
        T, torch = self.T, self.torch
        shapes, seg = self._shapes(req)
        C = req.channels
        keys = [(C,) + sh for sh in shapes]
        sizes = [T.taches_bytes_for(self._cfg(C, sh)) for sh in shapes]
        ring_bytes = 4 * C * seg[2] if seg else 0
        victims, taken = [], []
        with self._lock:
            need = ring_bytes + sum(n for k, n in zip(keys, sizes) if not self.free.get(k))
            while self.live_bytes + self.reserved_bytes + self.idle_bytes + need > self.budget:
                cands = [k for k in self.free if self.free[k] and k not in keys]
                if not cands:
                    break
                v = self.free[max(cands, key=lambda k: k[2])].pop()
                self.idle_bytes -= v.info().device_bytes
                victims.append(v)
            if self.live_bytes + self.reserved_bytes + self.idle_bytes + need > self.budget:
                self.refused += 1
                refused = True
            else:
                refused = False
                for k in keys:
                    lst = self.free.get(k)
                    s = lst.pop() if lst else None
                    if s is not None:
                        self.idle_bytes -= s.info().device_bytes
                    taken.append(s)
                amt = need + sum(n for s, n in zip(taken, sizes) if s is not None)
                self.reserved_bytes += amt
        for v in victims:
            v.close()
        if refused:
            raise AdmissionRefused("budget")
        streams = []
        for s, sh in zip(taken, shapes):
            if s is None:
                B, cap, tail, mb, prec = sh
                s = T.Stream(B, cap, channels=C, max_blocks_per_call=mb, precision=prec, tail=tail)
            streams.append(s)
        ring = torch.empty((C, seg[2]), device="cuda", dtype=torch.float32) if seg else None
        irs = self._draw_irs(req)
        nbytes = sum(s.info().device_bytes for s in streams) + ring_bytes
        with self._lock:
            self.reserved_bytes += nbytes - amt   # the reservation at the streams' actual sizes
        return streams, keys, ring, irs, nbytes

    def _prepare_loop(self) -> None:
        """The preparing thread: requests in admission order, at most
        PREPARE_AHEAD of them prepared and not yet admitted."""
        while not self._stop:
            with self._lock:
                req = self._to_prepare[0] if self._to_prepare and len(self._prepared) < self.PREPARE_AHEAD else None
            if req is None:
                time.sleep(0.0002)
                continue
            try:
                item = self._prepare(req)
            except AdmissionRefused:
                time.sleep(0.0005)   # wait for retirements to free budget
                continue
            except BaseException as e:   # handed to the tick loop, which raises it
                self._error = e
                return
            with self._lock:
                self._to_prepare.popleft()
                self._prepared[req.rid] = item

    def _recycle(self, s, key):
        s.reset()
        with self._lock:
            self.free.setdefault(key, []).append(s)
            self.idle_bytes += s.info().device_bytes

    def _admit(self, now: float, limit: int = 4) -> None:
        """Admit queued requests in FIFO order once prepared: attach their
        streams to the pool (no host wait) and register them with the
        server; at most `limit` per call."""
        T = self.T
        while self.pending and self.pending[0].arrival_s <= now:
            req = self.pending.popleft()
            self.queue.append(req)
            with self._lock:
                self._to_prepare.append(req)
        if self._thread is None:   # no preparing thread (admission outside run_realtime)
            while self._to_prepare:
                req = self._to_prepare[0]
                try:
                    item = self._prepare(req)
                except AdmissionRefused:
                    break
                self._to_prepare.popleft()
                self._prepared[req.rid] = item
        while self.queue and limit > 0:
            req = self.queue[0]
            if self.gate is not None and self.gate.closed:
                return
            if len(self.live) >= self.max_streams:
                with self._lock:   # the preparing thread counts budget refusals
                    self.refused += 1
                return
            with self._lock:
                item = self._prepared.pop(req.rid, None)
            if item is None:
                return
            limit -= 1
            c0 = time.perf_counter()
            streams, keys, ring, irs, nbytes = item
            for s in streams:
                _ = T._check(self.pool.attach(s), "taches_pool_attach")
            self.queue.popleft()
            c1 = time.perf_counter()
            self.irs[req.rid] = irs
            n_in = self.n_input_blocks(req)
            n_total = n_in + math.ceil((req.ir_len - 1) / req.block)
            y = None
            if req.rid in self.keep:
                y = np.zeros((req.channels, n_total * req.block), np.float32)
                self.kept[req.rid] = y
            swaps = [self.ir(req, v + 1) for v in range(len(req.swap_times_s))]
            if ring is None:
                if self.precision == T.TACHES_PREC_FP32:   # read in place: the IRs live until retirement
                    _ = T._check(T.taches_set_ir_ref(streams[0].h, self.ir(req, 0)), "taches_set_ir_ref")
                else:
                    streams[0].set_ir(self.ir(req, 0))
                rc = T.taches_server_add(self.sv, streams[0].h, req.rid, now, n_in, n_total, self.input_signal(req),
                                         y, req.swap_times_s, swaps)
                _ = T._check(rc, "taches_server_add")
            else:
                self.n_segmented += 1
                rc = T.taches_server_add_segmented(self.sv, streams[0].h, streams[1].h, self.segments_for(req)[0],
                                                   ring, req.rid, now, n_in, n_total, self.input_signal(req), y,
                                                   self.ir(req, 0), req.swap_times_s, swaps)
                _ = T._check(rc, "taches_server_add_segmented")
            with self._lock:
                self.reserved_bytes -= nbytes
                self.live_bytes += nbytes
            self.live[req.rid] = (streams, keys, req, ring, nbytes)
            c2 = time.perf_counter()
            self.admit_s["attach"] += c1 - c0
            self.admit_s["register"] += c2 - c1
            self.stats.admitted += 1
            if req.arrival_s >= self.warmup_s:
                self.stats.queue_waits_s.append(now - req.arrival_s)
        self.stats.max_active = max(self.stats.max_active, len(self.live))

    def _retire(self) -> None:
        for rid in self.T.taches_server_take_finished(self.sv, 256).tolist():
            streams, keys, req, ring, nbytes = self.live.pop(rid)
            for s in streams:
                self.pool.detach(s)
            with self._lock:
                self.live_bytes -= nbytes
            for s, k in zip(streams, keys):   # the ring's last use has completed with the stream's last step
                self._recycle(s, k)
            if rid not in self.keep:
                del self.irs[rid]   # every copy out of them has run: the stream's steps are done
            self.stats.completed += 1

    def _drain_records(self) -> None:
        lat, bs = self.T.taches_server_take_latencies(self.sv, 1 << 18)
        if lat.size:
            self.lat.append(lat)
            self.lat_b.append(bs)
            if self.gate is not None:
                self.gate.update(lat, bs)

    # -- driver ----------------------------------------------------------------
    def run_realtime(self, duration_s: float, sleep=time.sleep) -> dict:
        T = self.T
        sv = self.sv
        last_drain = 0.0
        clock = time.perf_counter
        # the preparing thread runs Python between its library calls: hand
        # the interpreter back and forth often, so the tick loop never waits
        # long for it
        switch = sys.getswitchinterval()
        sys.setswitchinterval(1e-4)
        # no cyclic garbage collection while serving: a full collection of a
        # large heap stops both threads for tens of milliseconds (objects
        # that exist now are frozen out of later collections)
        gc_was_enabled = gc.isenabled()
        gc.collect()
        gc.freeze()
        gc.disable()
        self._stop = False
        self._thread = threading.Thread(target=self._prepare_loop, name="taches-admission", daemon=True)
        self._thread.start()
        try:
            self._serve(duration_s, sleep, clock, last_drain)
        finally:
            self._stop = True
            self._thread.join()
            self._thread = None
            sys.setswitchinterval(switch)
            gc.unfreeze()
            if gc_was_enabled:
                gc.enable()
        T.taches_server_flush(sv)
        self._retire()
        wall = T.taches_server_clock(sv)
        self._drain_records()
        return self.summary(wall)

    def _serve(self, duration_s, sleep, clock, last_drain) -> None:
        T = self.T
        sv = self.sv
        while True:
            now = T.taches_server_clock(sv)
            if now >= duration_s:
                break
            if self._error is not None:
                raise RuntimeError("admission failed") from self._error
            t0 = clock()
            n_adm = self.stats.admitted
            self._admit(now)
            t1 = clock()
            tk = T.taches_server_tick(sv)
            t2 = clock()
            self._retire()
            t3 = clock()
            self.loops += 1
            self.python_s += (t1 - t0) + (t3 - t2)
            if t3 - t0 > 0.005 and now >= self.warmup_s:   # a loop iteration over 5 ms: keep its breakdown
                self.slow_loops.append((round(now, 3), round((t1 - t0) * 1e3, 2), round((t2 - t1) * 1e3, 2),
                                        round((t3 - t2) * 1e3, 2), self.stats.admitted - n_adm,
                                        round(tk.host_ms, 2), int(tk.streams)))
            if not tk.streams:
                nxt = tk.next_due_s
                if self.pending:
                    nxt = min(nxt, self.pending[0].arrival_s)
                wait = min(nxt, duration_s) - T.taches_server_clock(sv)
                if wait > 0:
                    sleep(min(wait, 0.0005))
            if now - last_drain > 0.2:   # a few hundred thousand records at a time
                self._drain_records()
                last_drain = now

    def summary(self, wall_s: float) -> dict:
        T = self.T
        st = T.taches_server_get_stats(self.sv)
        self.stats.steps = int(st.ticks)
        self.stats.blocks = int(st.blocks)
        self.stats.macs = int(st.macs)
        self.stats.busy_s = float(st.busy_s)
        self.stats.max_range = int(st.max_blocks_in_a_range)
        if self.lat:
            lat = np.concatenate(self.lat).astype(np.float64)
            bs = np.concatenate(self.lat_b).astype(np.int64)
            self.stats._lat, self.stats._dl, self.stats._bs = [lat], [bs / W.FS], [bs]
        out = self.stats.summary(wall_s)
        out["refused_attempts"] = self.refused
        out["bytes_h2d"] = int(st.bytes_in)
        out["bytes_d2h"] = int(st.bytes_out)
        out["gpu_busy_fraction"] = round(self.pool.info().device_ms_total / 1e3 / wall_s, 3) if wall_s > 0 else 0.0
        # the whole step on the device: input copy, batched launch, output launch
        out["device_step_busy_fraction"] = round(float(st.device_s) / wall_s, 3) if wall_s > 0 else 0.0
        if st.ticks:
            out["tick_ms_mean"] = {k: round(getattr(st, k + "_s") / st.ticks * 1e3, 4)
                                   for k in ("busy", "gather", "launch", "wait", "scatter")}
        if self.loops:
            out["loop_ms_mean"] = round(wall_s / self.loops * 1e3, 4)
            out["loop_python_ms_mean"] = round(self.python_s / self.loops * 1e3, 4)
        if st.recorded:
            out["latency_split_ms_mean"] = {"arrival_to_tick": round(st.pickup_s / st.recorded * 1e3, 4),
                                            "tick_to_host_outputs": round(st.service_s / st.recorded * 1e3, 4)}
        out["two_segment_requests"] = self.n_segmented
        if self.stats.admitted:
            out["admission_ms_mean"] = {k: round(v / self.stats.admitted * 1e3, 4) for k, v in self.admit_s.items()}
        if self.gate is not None:
            out["miss_gate"] = self.gate.summary()
        out["slow_loops"] = {"count": len(self.slow_loops),
                             "longest": sorted(self.slow_loops, key=lambda r: -(r[1] + r[2] + r[3]))[:8]}
        return out

    def kept_outputs(self, rid):
        """(input [C][n_in*B], outputs so far [C][blocks done*B], blocks of the
        applied IR swaps) of a request listed in keep_outputs; None if it was
        never admitted."""
        if rid not in self.kept:
            return None
        req = self.req_by_rid[rid]
        nxt, swaps = self.T.taches_server_stream_state(self.sv, rid)
        y = self.kept[rid][:, :nxt * req.block]
        return np.ascontiguousarray(self.input_signal(req)), y, swaps

    def close(self):
        T = self.T
        if self.sv:
            T.taches_server_destroy(self.sv)
            self.sv = None
        for streams, *_ in self.live.values():
            for s in streams:
                self.pool.detach(s)
                s.close()
        self.live.clear()
        for streams, *_ in self._prepared.values():
            for s in streams:
                s.close()
        self._prepared.clear()
        for lst in self.free.values():
            for s in lst:
                s.close()
        self.free.clear()
        self.pool.close()
