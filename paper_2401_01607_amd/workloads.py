"""Seeded synthetic inputs shaped like the paper's audio workloads.

This module is the only code shared between the CPU oracle and the HIP path.
It holds no convolution arithmetic: it only draws signals, impulse responses
and schedules.  The paper measured music stimuli and white-noise impulse
responses made in a sound editor (Section 5.1); neither is available, so the
signals here are seeded noise of the same length and sample rate and the
impulse responses are seeded decaying noise, as described below.

All draws use ``numpy.random.default_rng(seed)`` (PCG64).  The float32 arrays
returned are canonical: every consumer (oracle, kernels, benchmark) reads the
same bytes.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

FS = 48_000  # sample rate of every synthetic workload (Hz)

# Amplitude decay constant: exp(-6.91 n / L) is -60 dB (x 1/1000) at n = L.
DECAY = 6.91


def impulse_response(L: int, seed: int, decay: float = DECAY) -> np.ndarray:
    """Decaying-noise reverb IR of ``L`` taps, unit L2 norm, float32.

    ``v[n] = N(0,1) * exp(-decay * n / L)``, normalised in float64, then cast.
    ``decay=0`` gives the flat white-noise IR the paper used (Section 5.1).
    """
    if L < 1:
        raise ValueError("L must be >= 1")
    rng = np.random.default_rng(seed)
    n = np.arange(L, dtype=np.float64)
    v = rng.standard_normal(L) * np.exp(-decay * n / L)
    nrm = float(np.sqrt(np.sum(v * v)))
    if nrm > 0:
        v = v / nrm
    return v.astype(np.float32)


def signal_uniform(n: int, seed: int) -> np.ndarray:
    """``n`` float32 samples uniform in [-1, 1), drawn directly as float32."""
    rng = np.random.default_rng(seed)
    return (rng.random(n, dtype=np.float32) * np.float32(2.0) - np.float32(1.0)).astype(np.float32)


def signal_gauss(n: int, seed: int, sigma: float = 0.25) -> np.ndarray:
    """``n`` float32 samples of Gaussian noise with standard deviation ``sigma``."""
    rng = np.random.default_rng(seed)
    return (rng.standard_normal(n) * sigma).astype(np.float32)


def signal_int(n: int, seed: int, amp: int = 127) -> np.ndarray:
    """Integer-valued float32 samples in [-amp, amp].

    With ``|x|, |h| <= 127`` and ``L * 127**2 < 2**24`` every partial sum is an
    exact integer in float32, float64 and bfloat16-hi (lo = 0), so any correct
    summation order gives bit-identical results.
    """
    rng = np.random.default_rng(seed)
    return rng.integers(-amp, amp + 1, size=n).astype(np.float32)


def log_uniform_int(rng: np.random.Generator, a: int, b: int, size=None):
    """``round(exp(U(ln a, ln b)))`` clipped to [a, b]."""
    u = rng.uniform(math.log(a), math.log(b), size=size)
    return np.clip(np.round(np.exp(u)), a, b).astype(np.int64)


# ---------------------------------------------------------------------------
# Concrete workloads.  Sizes follow the five benchmark configurations; seeds
# are fixed so that every run sees the same bytes.
# ---------------------------------------------------------------------------

@dataclass
class StreamSpec:
    """One mono or multichannel stream: input, IR schedule, block size."""
    x: np.ndarray                 # [C, N] float32 planar
    block: int                    # B
    irs: list                     # list of float32 IR arrays
    schedule: list                # list of (block_index, ir_index): set_ir before that block
    max_ir_len: int
    name: str = ""
    extra: dict = field(default_factory=dict)

    @property
    def channels(self) -> int:
        return int(self.x.shape[0])

    @property
    def n_samples(self) -> int:
        return int(self.x.shape[1])

    def n_blocks(self) -> int:
        return -(-self.n_samples // self.block)

    def ir_of_block(self) -> np.ndarray:
        """Index of the IR active for each block (last schedule entry at or before it)."""
        nb = self.n_blocks()
        out = np.full(nb, -1, dtype=np.int64)
        sched = sorted(self.schedule)
        j = -1
        cur = -1
        for b in range(nb):
            while j + 1 < len(sched) and sched[j + 1][0] <= b:
                j += 1
                cur = sched[j][1]
            out[b] = cur
        return out

    def direct_macs(self) -> int:
        """Direct-equivalent MACs: sum over input samples of the active IR length."""
        ib = self.ir_of_block()
        lens = np.array([len(h) for h in self.irs], dtype=np.int64)
        per_block = lens[ib] * self.block
        # the last block may be short: count only real samples
        tail = self.n_blocks() * self.block - self.n_samples
        total = int(per_block.sum()) - int(lens[ib[-1]]) * tail
        return total * self.channels


def config1(n: int = 48_000) -> StreamSpec:
    """Plain taches, 1 mono stream, uniform input, L = 1024, B = 64."""
    x = signal_uniform(n, 101)[None, :]
    h = impulse_response(1024, 102)
    return StreamSpec(x=x, block=64, irs=[h], schedule=[(0, 0)], max_ir_len=1024, name="c1")


def swap_blocks(n_samples: int, block: int, period: int) -> list:
    """Blocks before which an IR swap is issued: the first block starting at or
    after ``period * k`` for k = 1, 2, ... while that sample is inside the input."""
    out = []
    k = 1
    while period * k < n_samples:
        out.append(-(-(period * k) // block))
        k += 1
    return out


def config2(n: int = 480_000, L: int = 65_536, block: int = 256, period: int = 4_800) -> StreamSpec:
    """Plain taches, 1 mono stream, Gaussian input, two IRs swapped every
    ``period`` samples (at the next block boundary), alternating A, B, A, ..."""
    x = signal_gauss(n, 201)[None, :]
    ha = impulse_response(L, 202)
    hb = impulse_response(L, 203)
    sched = [(0, 0)]
    for i, b in enumerate(swap_blocks(n, block, period)):
        sched.append((b, (i + 1) % 2))
    return StreamSpec(x=x, block=block, irs=[ha, hb], schedule=sched, max_ir_len=L, name="c2")


def config3(channels: int = 64, n: int = 240_000, L: int = 262_144, block: int = 512) -> StreamSpec:
    """Multichannel stream: ``channels`` Gaussian channels sharing one IR."""
    x = np.stack([signal_gauss(n, 301_000 + c) for c in range(channels)])
    h = impulse_response(L, 302)
    return StreamSpec(x=x, block=block, irs=[h], schedule=[(0, 0)], max_ir_len=L, name="c3")


BLOCK_CHOICES = (32, 64, 128, 256, 512)


def config4_draws(n_streams: int = 512, lmin: int = 256, lmax: int = 131_072, seed: int = 401):
    """Per-stream (L, B) draws of the batched workload."""
    rng = np.random.default_rng(seed)
    Ls = log_uniform_int(rng, lmin, lmax, size=n_streams)
    Bs = rng.choice(np.array(BLOCK_CHOICES), size=n_streams)
    return [int(v) for v in Ls], [int(v) for v in Bs]


def config4(n_streams: int = 512, n: int = 96_000, lmin: int = 256, lmax: int = 131_072) -> list:
    """Batched workload: independent mono streams with log-uniform IR lengths
    and block sizes drawn from {32, ..., 512}."""
    Ls, Bs = config4_draws(n_streams, lmin, lmax)
    out = []
    for s in range(n_streams):
        x = signal_gauss(n, 410_000 + s)[None, :]
        h = impulse_response(Ls[s], 420_000 + s)
        out.append(StreamSpec(x=x, block=Bs[s], irs=[h], schedule=[(0, 0)], max_ir_len=Ls[s],
                              name=f"c4s{s}"))
    return out


@dataclass
class ServingRequest:
    """One serving request: arrival time, stream shape, IR-swap times."""
    rid: int
    arrival_s: float
    duration_s: float
    channels: int
    block: int
    ir_len: int
    seed: int
    swap_times_s: list

    def n_samples(self) -> int:
        return int(round(self.duration_s * FS))

    def signal(self) -> np.ndarray:
        n = self.n_samples()
        return np.stack([signal_gauss(n, self.seed * 8 + c) for c in range(self.channels)])

    def ir(self, version: int) -> np.ndarray:
        """IR number ``version`` of this request (0 = initial, k = after swap k)."""
        return impulse_response(self.ir_len, self.seed * 1000 + 7 + version)


def config5_requests(horizon_s: float, rate_hz: float = 200.0, seed: int = 501,
                     dur=(10.0, 60.0), lrange=(512, 262_144), swap_rate_hz: float = 0.5,
                     stereo_p: float = 0.5) -> list:
    """Poisson arrivals of mono/stereo streams with IR swaps (Poisson, mean one
    per ``1/swap_rate_hz`` seconds) at the same IR length."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    rid = 0
    while True:
        t += float(rng.exponential(1.0 / rate_hz))
        if t >= horizon_s:
            break
        d = float(rng.uniform(*dur))
        ch = 2 if rng.random() < stereo_p else 1
        B = int(rng.choice(np.array(BLOCK_CHOICES)))
        L = int(log_uniform_int(rng, lrange[0], lrange[1]))
        swaps = []
        ts = 0.0
        while swap_rate_hz > 0:
            ts += float(rng.exponential(1.0 / swap_rate_hz))
            if ts >= d:
                break
            swaps.append(ts)
        out.append(ServingRequest(rid=rid, arrival_s=t, duration_s=d, channels=ch, block=B,
                                  ir_len=L, seed=int(rng.integers(1, 2**31 - 1)), swap_times_s=swaps))
        rid += 1
    return out
