"""CPU oracle for the streaming taches convolution.  TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this module.  It shares no code with the HIP path; the only common
module is the seeded input generator (``paper_2401_01607_amd.workloads``),
which holds none of the method's arithmetic.

Four forms of the same computation:

* ``OracleStream`` (O1 FP64, O2 FP32 with fused or separate roundings): the
  buffer form of Section 4.2 (a circular residue that receives every
  sample's tache, emits and clears one slot per sample), in C
  (``taches_oracle.c``).
* ``tache_sum`` (O3): Eq. (4) written as a sum of taches into a whole output
  array (Section 3.2), no residue.  numpy, FP64.  Small inputs only.
* ``brute_force`` (O4): Eq. (4) evaluated one output at a time, with exact
  Python integers / fractions.  Tiny inputs only.
* ``sampled_outputs``: Eq. (4) for chosen output indices in FP64 with numpy
  dot products (a library primitive), for full-size parity at sampled points.

Block-IR semantics everywhere: the IR used for the tache of input sample m is
the one active for the block that holds m (the last one set before that
block); taches keep the IR that produced them.  A schedule entry
(block, ir, offset) sets the IR from sample ``offset`` of that block on
(sample-accurate swap); (block, ir) means offset 0.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from concurrent.futures import ThreadPoolExecutor
from fractions import Fraction

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")
SRC_PATH = os.path.join(HERE, "taches_oracle.c")

OR_FP64, OR_FP32_FMA, OR_FP32_MULADD = 0, 1, 2
OR_OK, OR_EINVAL, OR_ENOIR, OR_ENOMEM = 0, -1, -2, -3

BUILD_CMD = ["gcc", "-O2", "-fPIC", "-shared", "-ffp-contract=off", "-std=c99",
             "-o", LIB_PATH, SRC_PATH, "-lm"]


def build() -> None:
    """Compile the C oracle (a checker, built beside the product)."""
    subprocess.run(BUILD_CMD, check=True)


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, i64 = ctypes.c_void_p, ctypes.c_int, ctypes.c_long
        L.or_open.restype = vp
        L.or_open.argtypes = [i32, i32, i32, i32]
        L.or_close.restype = None
        L.or_close.argtypes = [vp]
        L.or_set_ir.restype = i32
        L.or_set_ir.argtypes = [vp, vp, i32]
        L.or_set_ir_at.restype = i32
        L.or_set_ir_at.argtypes = [vp, vp, i32, i32]
        L.or_process.restype = i32
        L.or_process.argtypes = [vp, vp, vp]
        L.or_get_residue.restype = i32
        L.or_get_residue.argtypes = [vp, i32, vp]
        L.or_run_channel.restype = i32
        L.or_run_channel.argtypes = [i32, i32, i32, vp, i64, i32, vp, vp, vp, vp, vp]
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data)


class OracleStream:
    """Block-by-block oracle stream (O1 / O2).  Mirrors the library's calls:
    open(B, Lmax, C), set_ir(h), process(x[C][B]) -> y[C][B] (float64)."""

    def __init__(self, block: int, max_ir_len: int, channels: int = 1, prec: int = OR_FP64):
        self.B, self.Lmax, self.C, self.prec = block, max_ir_len, channels, prec
        self._h = lib().or_open(block, max_ir_len, channels, prec)
        if not self._h:
            raise ValueError("or_open failed")

    def set_ir(self, h: np.ndarray, offset: int = 0) -> int:
        """Queue h; it applies from sample ``offset`` of the next block."""
        h = np.ascontiguousarray(h, dtype=np.float32)
        return lib().or_set_ir_at(self._h, _ptr(h), int(h.size), int(offset))

    def process(self, x: np.ndarray):
        x = np.ascontiguousarray(np.asarray(x, dtype=np.float32).reshape(self.C, self.B))
        y = np.zeros((self.C, self.B), dtype=np.float64)
        rc = lib().or_process(self._h, _ptr(x), _ptr(y))
        return rc, y

    def residue(self, c: int = 0) -> np.ndarray:
        out = np.zeros(self.Lmax, dtype=np.float64)
        lib().or_get_residue(self._h, c, _ptr(out))
        return out

    def close(self):
        if self._h:
            lib().or_close(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _entry(e):
    """Schedule entry -> (block, ir, offset)."""
    return (int(e[0]), int(e[1]), int(e[2]) if len(e) > 2 else 0)


def _schedule_arrays(n_blocks: int, schedule):
    """ir_of_block[b] = IR index set before block b (-1 = no change) and the
    sample of block b it takes over at."""
    a = np.full(n_blocks, -1, dtype=np.int32)
    off = np.zeros(n_blocks, dtype=np.int32)
    for e in schedule:
        b, k, o = _entry(e)
        if 0 <= b < n_blocks:
            a[b], off[b] = k, o
    return a, off


def ir_of_sample(n_samples: int, schedule, block: int) -> np.ndarray:
    """Index of the IR whose tache input sample m gets (-1 = none yet): the
    schedule entry with the latest start b*B + offset at or before m."""
    starts = sorted((b * block + o, k) for b, k, o in map(_entry, schedule))
    out = np.full(n_samples, -1, dtype=np.int64)
    for pos, k in starts:
        if pos < n_samples:
            out[pos:] = k
    return out


def run_channel(x: np.ndarray, irs, schedule, block: int, max_ir_len: int,
                n_blocks: int | None = None, prec: int = OR_FP64) -> np.ndarray:
    """Whole-signal oracle for one channel: ``n_blocks`` blocks (default: enough
    for the input plus its temporal overflow), zero input beyond ``x``."""
    x = np.ascontiguousarray(x, dtype=np.float32).ravel()
    Lmax_used = max(len(h) for h in irs)
    if n_blocks is None:
        n_blocks = -(-(x.size + Lmax_used - 1) // block)
    irs32 = [np.ascontiguousarray(h, dtype=np.float32) for h in irs]
    ptrs = (ctypes.c_void_p * len(irs32))(*[h.ctypes.data for h in irs32])
    lens = np.array([h.size for h in irs32], dtype=np.int32)
    sched, offs = _schedule_arrays(n_blocks, schedule)
    y = np.zeros(n_blocks * block, dtype=np.float64)
    rc = lib().or_run_channel(block, max_ir_len, prec, _ptr(x), x.size, n_blocks,
                              ctypes.cast(ptrs, ctypes.c_void_p), _ptr(lens), _ptr(sched), _ptr(offs), _ptr(y))
    if rc != OR_OK:
        raise RuntimeError(f"oracle rc={rc}")
    return y


def run_channels(xs, irs, schedule, block: int, max_ir_len: int, n_blocks=None,
                 prec: int = OR_FP64, threads: int | None = None):
    """Run independent channels/streams on host threads (the C calls release
    the GIL).  ``xs``: list of 1-D signals sharing (irs, schedule)."""
    threads = threads or min(len(xs), os.cpu_count() or 1)
    with ThreadPoolExecutor(max_workers=threads) as ex:
        futs = [ex.submit(run_channel, x, irs, schedule, block, max_ir_len, n_blocks, prec) for x in xs]
        return [f.result() for f in futs]


# ---------------------------------------------------------------------------
# O3: the sum of taches written into the output array, FP64, small inputs.
# ---------------------------------------------------------------------------

def tache_sum(e: np.ndarray, h_of_sample) -> np.ndarray:
    """Eq. (4) as a sum of taches (Section 3.2): input sample n adds its
    tache e(n) * h to the output samples n .. n + len(h) - 1.

    ``h_of_sample(n)`` returns the IR for input sample n (the IR active when
    n is consumed).  The output has Ne + Nh - 1 samples (Nh = longest IR),
    the input length plus the temporal overflow (Section 4.1).  Each output
    receives its products in input order, as in the residue of the buffer
    form, so in FP64 the two agree bit for bit.
    """
    e = np.asarray(e, dtype=np.float32)
    Ne = e.size
    hs = [np.asarray(h_of_sample(n), dtype=np.float32).astype(np.float64) for n in range(Ne)]
    Nh = max(h.size for h in hs)
    s = np.zeros(Ne + Nh - 1, dtype=np.float64)
    for n in range(Ne):
        h = hs[n]
        s[n:n + h.size] += np.float64(e[n]) * h
    return s


# ---------------------------------------------------------------------------
# O4: brute force of Eq. (4), exact arithmetic, tiny inputs.
# ---------------------------------------------------------------------------

def _exact(v):
    f = float(v)
    return int(f) if f.is_integer() else Fraction(f)


def brute_force(x: np.ndarray, irs, schedule, block: int, n_out: int):
    """y[n] = sum over m <= n of x[m] * h_(IR of sample m)[n - m], exactly.

    ``schedule``: list of (block, ir_index[, offset]) entries, as for the
    streaming calls.  Returns a list of exact numbers (int or Fraction)."""
    x = [_exact(v) for v in np.asarray(x, dtype=np.float32)]
    irs_e = [[_exact(v) for v in np.asarray(h, dtype=np.float32)] for h in irs]
    act = ir_of_sample(len(x), schedule, block)
    y = []
    for n in range(n_out):
        acc = 0
        for m in range(0, min(n, len(x) - 1) + 1):
            k = int(act[m])
            if k < 0:
                continue
            h = irs_e[k]
            j = n - m
            if j < len(h):
                acc += x[m] * h[j]
        y.append(acc)
    return y


# ---------------------------------------------------------------------------
# Sampled outputs of Eq. (4) in FP64 for full-size parity.
# ---------------------------------------------------------------------------

def _ir_runs(n_samples: int, schedule, block: int):
    """Maximal runs [a, b) of input samples whose taches use the same IR k
    (k >= 0), in input order."""
    act = ir_of_sample(n_samples, schedule, block)
    runs = []
    a = 0
    while a < n_samples:
        b = a + 1
        while b < n_samples and act[b] == act[a]:
            b += 1
        if act[a] >= 0:
            runs.append((a, b, int(act[a])))
        a = b
    return runs


def sampled_outputs(x: np.ndarray, irs, schedule, block: int, idx) -> np.ndarray:
    """FP64 values of y[n] (Eq. 4) for the output indices ``idx``: for each
    run of input samples that share an IR, the dot product of the input
    window x[m] with the IR taps h[n - m] (a library primitive)."""
    x = np.asarray(x, dtype=np.float32).astype(np.float64)
    irs64 = [np.asarray(h, dtype=np.float32).astype(np.float64) for h in irs]
    runs = _ir_runs(x.size, schedule, block)
    out = np.zeros(len(idx), dtype=np.float64)
    for t, n in enumerate(idx):
        n = int(n)
        acc = 0.0
        for a, b, k in runs:
            h = irs64[k]
            lo = max(a, n - h.size + 1)          # taps h[n - m] exist for m > n - L
            hi = min(b - 1, n)                   # causal: m <= n
            if hi < lo:
                continue
            # m = lo .. hi pairs with h[n - lo] .. h[n - hi]
            acc += float(np.dot(x[lo:hi + 1], h[n - hi:n - lo + 1][::-1]))
        out[t] = acc
    return out


def fft_outputs(x: np.ndarray, irs, schedule, block: int, n_out: int) -> np.ndarray:
    """All outputs y[0 .. n_out) of Eq. (4) in FP64 via the convolution
    theorem (numpy's FFT as a library primitive): y is the sum over IR runs
    of conv(x restricted to the run, h of the run).  Its error is a few
    units of 2^-53 times sqrt(n) * ||x|| * ||h|| per output (far below any
    FP32 tolerance); used for statistics over whole outputs (the RMS that
    tolerances are stated against, error figures over every output).
    ``x``: one signal [N], or channels sharing the schedule [C, N] (then the
    result is [C, n_out])."""
    x = np.asarray(x, dtype=np.float32)
    one = x.ndim == 1
    xs = np.atleast_2d(x)
    y = np.zeros((xs.shape[0], n_out), dtype=np.float64)
    for a, b, k in _ir_runs(xs.shape[1], schedule, block):
        h = np.asarray(irs[k], dtype=np.float32).astype(np.float64)
        m = (b - a) + h.size - 1
        nfft = 1 << (m - 1).bit_length()
        hf = np.fft.rfft(h, nfft)
        e = min(n_out, a + m)
        for c0 in range(0, xs.shape[0], 8):          # 8 channels at a time bounds the memory
            seg = xs[c0:c0 + 8, a:b].astype(np.float64)
            c = np.fft.irfft(np.fft.rfft(seg, nfft, axis=1) * hf, nfft, axis=1)
            if a < n_out:
                y[c0:c0 + 8, a:e] += c[:, : e - a]
    return y[0] if one else y


def abs_bound_weights(x: np.ndarray, irs, schedule, block: int, max_ir_len: int, n_blocks=None):
    """sum_k |h_k| |x_{n-k}| per output (the magnitude the rounding bounds
    scale with): the same oracle run on absolute values."""
    return run_channel(np.abs(np.asarray(x, dtype=np.float32)), [np.abs(np.asarray(h, np.float32)) for h in irs],
                       schedule, block, max_ir_len, n_blocks, OR_FP64)
