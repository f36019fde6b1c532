"""Thin Python binding of libtaches (ctypes).  Argument marshalling only:
every step of the convolution runs in the library's HIP kernels.  PyTorch
supplies device memory (tensor.data_ptr()) and streams
(torch.cuda.current_stream().cuda_stream).

The functions keep the C names (taches_open, taches_set_ir, ...); ``Stream``
wraps a handle for convenience.  Importing this module fails loudly if the
library has not been built: there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch  # loads the HIP runtime first, so the library shares it

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libtaches.so")

TACHES_OK, TACHES_EINVAL, TACHES_ENOIR, TACHES_ENOMEM, TACHES_EDEVICE, TACHES_EBUSY = 0, -1, -2, -3, -4, -5
TACHES_PREC_FP32, TACHES_PREC_SPLIT_BF16 = 0, 1
TACHES_TAIL_AUTO, TACHES_TAIL_FP32, TACHES_TAIL_FP64 = 0, 1, 2

STATUS_NAMES = {0: "TACHES_OK", -1: "TACHES_EINVAL", -2: "TACHES_ENOIR", -3: "TACHES_ENOMEM",
                -4: "TACHES_EDEVICE", -5: "TACHES_EBUSY"}

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                      "(or python -m paper_2401_01607_amd.build)")

lib = ctypes.CDLL(LIB_PATH)


class taches_config(ctypes.Structure):
    _fields_ = [("block_size", ctypes.c_int32), ("max_ir_len", ctypes.c_int32),
                ("channels", ctypes.c_int32), ("max_blocks_per_call", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("tail", ctypes.c_int32),
                ("ir_slots", ctypes.c_int32), ("device", ctypes.c_int32)]


class taches_info(ctypes.Structure):
    _fields_ = [("block_size", ctypes.c_int32), ("max_ir_len", ctypes.c_int32),
                ("channels", ctypes.c_int32), ("max_blocks_per_call", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("tail_fp64", ctypes.c_int32),
                ("ring_slots", ctypes.c_int32), ("head", ctypes.c_int32), ("live", ctypes.c_int32),
                ("active_len", ctypes.c_int32), ("blocks_done", ctypes.c_int64),
                ("device_bytes", ctypes.c_int64), ("tile_r", ctypes.c_int32), ("tile_w", ctypes.c_int32)]


class taches_pool_info(ctypes.Structure):
    _fields_ = [("attached", ctypes.c_int32), ("max_streams", ctypes.c_int32),
                ("budget_bytes", ctypes.c_int64), ("used_bytes", ctypes.c_int64),
                ("last_items", ctypes.c_int32), ("last_workgroups", ctypes.c_int32),
                ("last_r", ctypes.c_int32), ("pad_", ctypes.c_int32), ("graph_replays", ctypes.c_int64),
                ("last_plan_ms", ctypes.c_double), ("last_imbalance", ctypes.c_double),
                ("last_device_ms", ctypes.c_double), ("device_ms_total", ctypes.c_double),
                ("graph_captures", ctypes.c_int64)]


class taches_server_tick_info(ctypes.Structure):
    _fields_ = [("streams", ctypes.c_int32), ("pad_", ctypes.c_int32), ("blocks", ctypes.c_int64),
                ("now_s", ctypes.c_double), ("done_s", ctypes.c_double), ("host_ms", ctypes.c_double),
                ("step_ms", ctypes.c_double), ("next_due_s", ctypes.c_double)]


class taches_server_stats(ctypes.Structure):
    _fields_ = [("ticks", ctypes.c_int64), ("blocks", ctypes.c_int64), ("macs", ctypes.c_int64),
                ("max_blocks_in_a_range", ctypes.c_int64), ("bytes_in", ctypes.c_int64),
                ("bytes_out", ctypes.c_int64), ("busy_s", ctypes.c_double), ("gather_s", ctypes.c_double),
                ("launch_s", ctypes.c_double), ("wait_s", ctypes.c_double), ("scatter_s", ctypes.c_double),
                ("streams", ctypes.c_int32), ("pad_", ctypes.c_int32), ("recorded", ctypes.c_int64),
                ("pickup_s", ctypes.c_double), ("service_s", ctypes.c_double), ("device_s", ctypes.c_double)]


_vp, _i32, _i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
_P = ctypes.POINTER
_SIGS = {
    "taches_config_default": (None, [_P(taches_config), _i32, _i32]),
    "taches_open": (_vp, [_i32, _i32]),
    "taches_open_ex": (_vp, [_P(taches_config)]),
    "taches_close": (ctypes.c_int, [_vp]),
    "taches_last_error": (ctypes.c_char_p, []),
    "taches_set_hip_stream": (ctypes.c_int, [_vp, _vp]),
    "taches_synchronize": (ctypes.c_int, [_vp]),
    "taches_set_ir": (ctypes.c_int, [_vp, _vp, _i32]),
    "taches_set_ir_device": (ctypes.c_int, [_vp, _vp, _i32]),
    "taches_set_ir_at": (ctypes.c_int, [_vp, _vp, _i32, _i32, _i32]),
    "taches_load_ir_slot": (ctypes.c_int, [_vp, _i32, _vp, _i32, _i32]),
    "taches_process": (ctypes.c_int, [_vp, _vp, _vp]),
    "taches_process_async": (ctypes.c_int, [_vp, _vp, _vp]),
    "taches_process_blocks": (ctypes.c_int, [_vp, _vp, _vp, _i32, _vp]),
    "taches_process_blocks_at": (ctypes.c_int, [_vp, _vp, _vp, _i32, _vp, _vp]),
    "taches_get_info": (ctypes.c_int, [_vp, _P(taches_info)]),
    "taches_bytes_for": (_i64, [_P(taches_config)]),
    "taches_tail_is_fp64": (ctypes.c_int, [_P(taches_config)]),
    "taches_read_tail": (ctypes.c_int, [_vp, _i32, _vp, _i32]),
    "taches_set_tile": (ctypes.c_int, [_vp, _i32, _i32]),
    "taches_set_timing": (ctypes.c_int, [_vp, _i32]),
    "taches_call_times": (ctypes.c_int, [_vp, _vp, _i32]),
    "taches_reset": (ctypes.c_int, [_vp]),
    "taches_pool_create": (_vp, [_i32, _i64, _i32]),
    "taches_pool_destroy": (ctypes.c_int, [_vp]),
    "taches_pool_attach": (ctypes.c_int, [_vp, _vp]),
    "taches_pool_detach": (ctypes.c_int, [_vp, _vp]),
    "taches_pool_step": (ctypes.c_int, [_vp, _i32, _vp, _vp, _vp, _vp]),
    "taches_pool_step_strided": (ctypes.c_int, [_vp, _i32, _vp, _vp, _vp, _vp, _vp, _vp]),
    "taches_pool_set_hip_stream": (ctypes.c_int, [_vp, _vp]),
    "taches_pool_set_copy_stream": (ctypes.c_int, [_vp, _vp]),
    "taches_pool_set_tile": (ctypes.c_int, [_vp, _i32]),
    "taches_pool_use_graph": (ctypes.c_int, [_vp, _i32]),
    "taches_pool_synchronize": (ctypes.c_int, [_vp]),
    "taches_pool_get_info": (ctypes.c_int, [_vp, _P(taches_pool_info)]),
    "taches_fp32_fma_ceiling": (ctypes.c_int, [_i32, _P(ctypes.c_double)]),
    "taches_convolve": (ctypes.c_int, [_vp, _i64, _i32, _vp, _i32, _vp, _i32, _i32, _i32, _vp]),
    "taches_convolve_noalloc": (ctypes.c_int, [_vp, _i64, _i32, _vp, _i32, _vp, _i32, _i32, _vp]),
    "taches_set_ir_ref": (ctypes.c_int, [_vp, _vp, _i32, _i32]),
    "taches_server_create": (_vp, [_vp, ctypes.c_double, _i32, ctypes.c_double]),
    "taches_server_destroy": (ctypes.c_int, [_vp]),
    "taches_server_clock": (ctypes.c_double, [_vp]),
    "taches_server_add": (ctypes.c_int, [_vp, _vp, _i64, ctypes.c_double, _i64, _i64, _vp, _i64, _vp, _i64, _i32,
                                         _vp, _vp, _vp]),
    "taches_server_add_segmented": (ctypes.c_int, [_vp, _vp, _vp, _i32, _vp, _i32, _i64, ctypes.c_double, _i64,
                                                   _i64, _vp, _i64, _vp, _i64, _vp, _i32, _i32, _vp, _vp, _vp]),
    "taches_server_tick": (ctypes.c_int, [_vp, _P(taches_server_tick_info)]),
    "taches_server_flush": (ctypes.c_int, [_vp]),
    "taches_server_take_finished": (ctypes.c_int, [_vp, _vp, _i32]),
    "taches_server_take_latencies": (ctypes.c_int, [_vp, _vp, _vp, _i32]),
    "taches_server_stream_state": (ctypes.c_int, [_vp, _i64, _P(_i64), _vp, _i32]),
    "taches_server_get_stats": (ctypes.c_int, [_vp, _P(taches_server_stats)]),
}
for _name, (_res, _args) in _SIGS.items():
    _f = getattr(lib, _name)
    _f.restype = _res
    _f.argtypes = _args


class TachesError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        msg = lib.taches_last_error().decode(errors="replace")
        super().__init__(f"{where}: {STATUS_NAMES.get(status, status)}: {msg}")


def _check(rc: int, where: str) -> int:
    if rc != TACHES_OK:
        raise TachesError(rc, where)
    return rc


def _host_ptr(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data)


def _dev_ptr(t):
    if t is None:
        return None
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()):
        raise TypeError("expected a contiguous float32 CUDA tensor")
    return ctypes.c_void_p(t.data_ptr())


# ---- same-name wrappers -----------------------------------------------------

def taches_config_default(block_size: int, max_ir_len: int) -> taches_config:
    c = taches_config()
    lib.taches_config_default(ctypes.byref(c), block_size, max_ir_len)
    return c


def taches_open(block_size: int, max_ir_len: int):
    h = lib.taches_open(block_size, max_ir_len)
    if not h:
        raise TachesError(TACHES_EINVAL, "taches_open")
    return h


def taches_open_ex(cfg: taches_config):
    h = lib.taches_open_ex(ctypes.byref(cfg))
    if not h:
        raise TachesError(TACHES_EINVAL, "taches_open_ex")
    return h


def taches_close(s) -> int:
    return lib.taches_close(s)


def taches_set_ir(s, h: np.ndarray) -> int:
    h = np.ascontiguousarray(h, dtype=np.float32)
    return lib.taches_set_ir(s, _host_ptr(h), int(h.size))


def taches_set_ir_device(s, h_dev) -> int:
    return lib.taches_set_ir_device(s, _dev_ptr(h_dev), int(h_dev.numel()))


def taches_set_ir_ref(s, h_dev, offset: int = 0) -> int:
    """h_dev: a contiguous float32 CUDA tensor the stream reads in place
    (kept alive and unchanged by the caller until replaced and done)."""
    return lib.taches_set_ir_ref(s, _dev_ptr(h_dev), int(h_dev.numel()), int(offset))


def taches_set_ir_at(s, h, offset: int) -> int:
    """h: host array or CUDA tensor; it takes over at sample ``offset`` of
    the next processed block."""
    if isinstance(h, torch.Tensor):
        return lib.taches_set_ir_at(s, _dev_ptr(h), int(h.numel()), int(offset), 1)
    h = np.ascontiguousarray(h, dtype=np.float32)
    return lib.taches_set_ir_at(s, _host_ptr(h), int(h.size), int(offset), 0)


def taches_load_ir_slot(s, slot: int, h) -> int:
    if isinstance(h, torch.Tensor):
        return lib.taches_load_ir_slot(s, slot, _dev_ptr(h), int(h.numel()), 1)
    h = np.ascontiguousarray(h, dtype=np.float32)
    return lib.taches_load_ir_slot(s, slot, _host_ptr(h), int(h.size), 0)


def taches_process(s, x: np.ndarray, y: np.ndarray) -> int:
    return lib.taches_process(s, _host_ptr(x), _host_ptr(y))


def taches_process_async(s, x_dev, y_dev) -> int:
    return lib.taches_process_async(s, _dev_ptr(x_dev), _dev_ptr(y_dev))


def taches_process_blocks(s, x_dev, y_dev, n_blocks: int, ir_slot_of_block=None) -> int:
    sched = None
    if ir_slot_of_block is not None:
        sched = np.ascontiguousarray(ir_slot_of_block, dtype=np.int32)
        if sched.size != n_blocks:
            raise ValueError("ir_slot_of_block must have n_blocks entries")
    return lib.taches_process_blocks(s, _dev_ptr(x_dev), _dev_ptr(y_dev), n_blocks,
                                     None if sched is None else _host_ptr(sched))


def taches_process_blocks_at(s, x_dev, y_dev, n_blocks: int, ir_slot_of_block, offset_of_block=None) -> int:
    sched = np.ascontiguousarray(ir_slot_of_block, dtype=np.int32)
    if sched.size != n_blocks:
        raise ValueError("ir_slot_of_block must have n_blocks entries")
    offs = None
    if offset_of_block is not None:
        offs = np.ascontiguousarray(offset_of_block, dtype=np.int32)
        if offs.size != n_blocks:
            raise ValueError("offset_of_block must have n_blocks entries")
    return lib.taches_process_blocks_at(s, _dev_ptr(x_dev), _dev_ptr(y_dev), n_blocks, _host_ptr(sched),
                                        None if offs is None else _host_ptr(offs))


def taches_get_info(s) -> taches_info:
    info = taches_info()
    _check(lib.taches_get_info(s, ctypes.byref(info)), "taches_get_info")
    return info


def taches_bytes_for(cfg: taches_config) -> int:
    return int(lib.taches_bytes_for(ctypes.byref(cfg)))


def taches_tail_is_fp64(cfg: taches_config) -> int:
    return int(lib.taches_tail_is_fp64(ctypes.byref(cfg)))


def taches_read_tail(s, channel: int, n: int) -> np.ndarray:
    out = np.zeros(n, dtype=np.float64)
    _check(lib.taches_read_tail(s, channel, _host_ptr(out), n), "taches_read_tail")
    return out


def taches_set_tile(s, r: int, w: int) -> int:
    return lib.taches_set_tile(s, r, w)


def taches_set_timing(s, on: bool) -> int:
    return lib.taches_set_timing(s, 1 if on else 0)


def taches_call_times(s, n: int) -> np.ndarray:
    out = np.zeros(max(n, 0), dtype=np.float64)
    m = lib.taches_call_times(s, _host_ptr(out) if n > 0 else None, n)
    if m < 0:
        _check(m, "taches_call_times")
    return out[:m]


def taches_reset(s) -> int:
    return lib.taches_reset(s)


def taches_set_hip_stream(s, stream: int) -> int:
    """stream: a hipStream_t value (torch.cuda.Stream.cuda_stream); 0 is HIP's null stream."""
    return lib.taches_set_hip_stream(s, ctypes.c_void_p(stream) if stream else None)


def taches_synchronize(s) -> int:
    return lib.taches_synchronize(s)


def taches_last_error() -> str:
    return lib.taches_last_error().decode(errors="replace")


def taches_pool_create(max_streams: int, hbm_budget_bytes: int, device: int = 0):
    h = lib.taches_pool_create(max_streams, hbm_budget_bytes, device)
    if not h:
        raise TachesError(TACHES_EINVAL, "taches_pool_create")
    return h


def taches_pool_destroy(p) -> int:
    return lib.taches_pool_destroy(p)


def taches_pool_attach(p, s) -> int:
    return lib.taches_pool_attach(p, s)


def taches_pool_detach(p, s) -> int:
    return lib.taches_pool_detach(p, s)


def taches_pool_step(p, streams, xs, ys, n_blocks) -> int:
    """streams: handles; xs: CUDA tensors or None (zero input); ys: CUDA tensors."""
    n = len(streams)
    sarr = (ctypes.c_void_p * n)(*streams)
    xarr = None
    if xs is not None:
        xarr = (ctypes.c_void_p * n)(*[None if x is None else _dev_ptr(x).value for x in xs])
    yarr = (ctypes.c_void_p * n)(*[_dev_ptr(y).value for y in ys])
    nb = (ctypes.c_int32 * n)(*n_blocks)
    return lib.taches_pool_step(p, n, sarr, xarr, yarr, nb)


def taches_pool_step_strided(p, streams, x_ptrs, x_cstride, y_ptrs, y_cstride, n_blocks) -> int:
    """Raw-address form for large steps: numpy arrays of length n holding
    stream handles and device addresses (uint64, 0 = NULL input), channel
    strides in floats (int64, or None = packed) and block counts (int32)."""
    n = len(n_blocks)

    def arr(a, dt):
        if a is None:
            return None, None
        a = np.ascontiguousarray(a, dtype=dt)
        if a.shape != (n,):
            raise ValueError("per-stream arrays must have one entry per stream")
        return a, ctypes.c_void_p(a.ctypes.data)
    keep = [arr(streams, np.uint64), arr(x_ptrs, np.uint64), arr(x_cstride, np.int64), arr(y_ptrs, np.uint64),
            arr(y_cstride, np.int64), arr(n_blocks, np.int32)]
    if keep[0][0] is None or keep[3][0] is None:
        raise ValueError("streams and y_ptrs are required")
    return lib.taches_pool_step_strided(p, n, *[k[1] for k in keep])


def taches_convolve(x_dev, h_dev, y_dev, precision: int = TACHES_PREC_FP32, role_swap: bool = False,
                    device: int = 0, hip_stream=None) -> int:
    """Off-line convolution: x_dev [C][nx] (or [nx]), h_dev [nh], y_dev
    [C][nx + nh - 1] CUDA tensors; runs on torch's current stream unless a
    HIP stream handle is given."""
    C = 1 if x_dev.dim() == 1 else int(x_dev.shape[0])
    nx = int(x_dev.shape[-1])
    nh = int(h_dev.numel())
    if tuple(y_dev.shape[-1:]) != (nx + nh - 1,) or (x_dev.dim() > 1 and int(y_dev.shape[0]) != C):
        raise ValueError("y must be [C][nx + nh - 1]")
    if hip_stream is None:
        hip_stream = torch.cuda.current_stream(device).cuda_stream
    return lib.taches_convolve(_dev_ptr(x_dev), nx, C, _dev_ptr(h_dev), nh, _dev_ptr(y_dev), precision,
                               1 if role_swap else 0, device, ctypes.c_void_p(hip_stream) if hip_stream else None)


def taches_convolve_noalloc(x_dev, h_dev, y_dev, role_swap: bool = False, device: int = 0, hip_stream=None) -> int:
    """taches_convolve (FP32) without allocation: same tensors as
    taches_convolve; the work is only enqueued (synchronize the stream
    before reading y_dev)."""
    C = 1 if x_dev.dim() == 1 else int(x_dev.shape[0])
    nx = int(x_dev.shape[-1])
    nh = int(h_dev.numel())
    if tuple(y_dev.shape[-1:]) != (nx + nh - 1,) or (x_dev.dim() > 1 and int(y_dev.shape[0]) != C):
        raise ValueError("y must be [C][nx + nh - 1]")
    if hip_stream is None:
        hip_stream = torch.cuda.current_stream(device).cuda_stream
    return lib.taches_convolve_noalloc(_dev_ptr(x_dev), nx, C, _dev_ptr(h_dev), nh, _dev_ptr(y_dev),
                                       1 if role_swap else 0, device,
                                       ctypes.c_void_p(hip_stream) if hip_stream else None)


def taches_fp32_fma_ceiling(device: int = 0) -> float:
    """TFLOP/s of unpacked FP32 FMA chains on the device (see the header)."""
    v = ctypes.c_double()
    _check(lib.taches_fp32_fma_ceiling(device, ctypes.byref(v)), "taches_fp32_fma_ceiling")
    return v.value


def taches_pool_set_hip_stream(p, stream: int) -> int:
    return lib.taches_pool_set_hip_stream(p, ctypes.c_void_p(stream) if stream else None)


def taches_pool_set_copy_stream(p, stream: int) -> int:
    return lib.taches_pool_set_copy_stream(p, ctypes.c_void_p(stream) if stream else None)


def taches_pool_set_tile(p, r: int) -> int:
    return lib.taches_pool_set_tile(p, r)


def taches_pool_use_graph(p, on: bool) -> int:
    return lib.taches_pool_use_graph(p, 1 if on else 0)


def taches_pool_synchronize(p) -> int:
    return lib.taches_pool_synchronize(p)


def taches_pool_get_info(p) -> taches_pool_info:
    info = taches_pool_info()
    _check(lib.taches_pool_get_info(p, ctypes.byref(info)), "taches_pool_get_info")
    return info


# ---- convenience wrappers -----------------------------------------------------

class Stream:
    """One taches stream (a handle).  Raises TachesError on any failure."""

    def __init__(self, block_size: int, max_ir_len: int, channels: int = 1, max_blocks_per_call: int = 1,
                 precision: int = TACHES_PREC_FP32, tail: int = TACHES_TAIL_AUTO, ir_slots: int = 2,
                 device: int = 0, torch_stream: bool = True):
        cfg = taches_config_default(block_size, max_ir_len)
        cfg.channels = channels
        cfg.max_blocks_per_call = max_blocks_per_call
        cfg.precision = precision
        cfg.tail = tail
        cfg.ir_slots = ir_slots
        cfg.device = device
        self.cfg = cfg
        self.h = taches_open_ex(cfg)
        if torch_stream:
            _check(taches_set_hip_stream(self.h, torch.cuda.current_stream(device).cuda_stream),
                   "taches_set_hip_stream")

    @property
    def B(self) -> int:
        return self.cfg.block_size

    @property
    def C(self) -> int:
        return self.cfg.channels

    def set_ir(self, h, offset: int = 0) -> None:
        """Queue h for the next block, taking over at sample ``offset`` of it."""
        if offset:
            _check(taches_set_ir_at(self.h, h, offset), "taches_set_ir_at")
        elif isinstance(h, torch.Tensor):
            _check(taches_set_ir_device(self.h, h), "taches_set_ir_device")
        else:
            _check(taches_set_ir(self.h, h), "taches_set_ir")

    def load_ir_slot(self, slot: int, h) -> None:
        _check(taches_load_ir_slot(self.h, slot, h), "taches_load_ir_slot")

    def process(self, x: np.ndarray) -> np.ndarray:
        x = np.ascontiguousarray(x, dtype=np.float32).reshape(self.C, self.B)
        y = np.zeros_like(x)
        _check(taches_process(self.h, x, y), "taches_process")
        return y

    def process_async(self, x_dev, y_dev) -> None:
        _check(taches_process_async(self.h, x_dev, y_dev), "taches_process_async")

    def process_blocks(self, x_dev, y_dev, n_blocks: int, ir_slot_of_block=None, offset_of_block=None) -> None:
        if offset_of_block is not None:
            _check(taches_process_blocks_at(self.h, x_dev, y_dev, n_blocks, ir_slot_of_block, offset_of_block),
                   "taches_process_blocks_at")
        else:
            _check(taches_process_blocks(self.h, x_dev, y_dev, n_blocks, ir_slot_of_block), "taches_process_blocks")

    def info(self) -> taches_info:
        return taches_get_info(self.h)

    def read_tail(self, channel: int = 0, n: int | None = None) -> np.ndarray:
        if n is None:
            n = self.info().ring_slots
        return taches_read_tail(self.h, channel, n)

    def set_tile(self, r: int, w: int) -> None:
        _check(taches_set_tile(self.h, r, w), "taches_set_tile")

    def set_timing(self, on: bool) -> None:
        """Record HIP events around each call's kernel launches (see call_times)."""
        _check(taches_set_timing(self.h, on), "taches_set_timing")

    def call_times(self, n: int) -> np.ndarray:
        """Device times (ms) of the last n timed calls, oldest first; clears the record."""
        return taches_call_times(self.h, n)

    def synchronize(self) -> None:
        _check(taches_synchronize(self.h), "taches_synchronize")

    def reset(self) -> None:
        _check(taches_reset(self.h), "taches_reset")

    def close(self) -> None:
        if self.h:
            _check(taches_close(self.h), "taches_close")
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            if self.h:
                lib.taches_close(self.h)
                self.h = None
        except Exception:
            pass


# ---- serving tick ------------------------------------------------------------

def taches_server_create(pool, fs: float, max_blocks_per_step: int, warmup_s: float = 0.0):
    h = lib.taches_server_create(pool, fs, max_blocks_per_step, warmup_s)
    if not h:
        raise TachesError(TACHES_EINVAL, "taches_server_create")
    return h


def taches_server_destroy(sv) -> int:
    return lib.taches_server_destroy(sv)


def taches_server_clock(sv) -> float:
    return float(lib.taches_server_clock(sv))


def _server_buffers(x_host, y_host, swap_times_s, swap_irs):
    x_host = np.atleast_2d(x_host)
    if x_host.dtype != np.float32 or x_host.strides[1] != 4 or x_host.strides[0] % 4:
        raise TypeError("x_host must be a float32 array with contiguous rows")
    x_cs = x_host.shape[1] if x_host.shape[0] == 1 else x_host.strides[0] // 4
    y_ptr, y_cs = None, 0
    if y_host is not None:
        y_host = np.atleast_2d(y_host)
        if y_host.dtype != np.float32 or not y_host.flags.c_contiguous:
            raise TypeError("y_host must be a C-contiguous float32 array")
        y_ptr, y_cs = _host_ptr(y_host), y_host.shape[1]
    n = len(swap_times_s)
    if len(swap_irs) != n:
        raise ValueError("one IR per swap time")
    t = np.ascontiguousarray(swap_times_s, np.float64)
    hp = np.array([ir.data_ptr() for ir in swap_irs], np.uint64)
    hl = np.array([ir.numel() for ir in swap_irs], np.int32)
    swaps = (n, _host_ptr(t) if n else None, _host_ptr(hp) if n else None, _host_ptr(hl) if n else None)
    # the arrays behind the pointers stay referenced by the returned tuple
    return (_host_ptr(x_host), x_cs, y_ptr, y_cs) + swaps, (x_host, y_host, t, hp, hl)


def taches_server_add(sv, stream, tag: int, start_s: float, n_in_blocks: int, n_total_blocks: int,
                      x_host: np.ndarray, y_host, swap_times_s=(), swap_irs=()) -> int:
    """x_host: [C][x_cstride] float32 host array (kept alive by the caller);
    y_host: [C][y_cstride] float32 host array or None; swap_irs: device
    tensors (kept alive by the caller until applied)."""
    args, _keep = _server_buffers(x_host, y_host, swap_times_s, swap_irs)
    return lib.taches_server_add(sv, stream, tag, start_s, n_in_blocks, n_total_blocks, *args)


def taches_server_add_segmented(sv, head, rest, head_len: int, z_ring, tag: int, start_s: float, n_in_blocks: int,
                                n_total_blocks: int, x_host: np.ndarray, y_host, ir, swap_times_s=(),
                                swap_irs=()) -> int:
    """As taches_server_add for a stream served in two IR segments: head
    and rest stream handles, z_ring a [C][Z] float32 device tensor, ir the
    initial device IR (all IRs kept alive by the caller until applied)."""
    if z_ring.dtype != torch.float32 or not z_ring.is_cuda or not z_ring.is_contiguous() or z_ring.dim() != 2:
        raise TypeError("z_ring must be a contiguous [C][Z] float32 device tensor")
    args, _keep = _server_buffers(x_host, y_host, swap_times_s, swap_irs)
    x_ptr, x_cs, y_ptr, y_cs, n, t, hp, hl = args
    return lib.taches_server_add_segmented(sv, head, rest, head_len, z_ring.data_ptr(), z_ring.shape[1], tag, start_s,
                                           n_in_blocks, n_total_blocks, x_ptr, x_cs, y_ptr, y_cs, ir.data_ptr(),
                                           ir.numel(), n, t, hp, hl)


def taches_server_tick(sv) -> taches_server_tick_info:
    out = taches_server_tick_info()
    _check(lib.taches_server_tick(sv, ctypes.byref(out)), "taches_server_tick")
    return out


def taches_server_flush(sv) -> None:
    _check(lib.taches_server_flush(sv), "taches_server_flush")


def taches_server_take_finished(sv, cap: int = 4096) -> np.ndarray:
    buf = np.zeros(cap, np.int64)
    n = lib.taches_server_take_finished(sv, _host_ptr(buf), cap)
    _check(min(n, 0), "taches_server_take_finished")
    return buf[:n]


def taches_server_take_latencies(sv, cap: int = 1 << 20):
    """(latencies in seconds, block sizes) recorded since the last call."""
    lat, bs = [], []
    while True:
        a = np.zeros(cap, np.float32)
        b = np.zeros(cap, np.int32)
        n = lib.taches_server_take_latencies(sv, _host_ptr(a), _host_ptr(b), cap)
        _check(min(n, 0), "taches_server_take_latencies")
        lat.append(a[:n])
        bs.append(b[:n])
        if n < cap:
            return np.concatenate(lat), np.concatenate(bs)


def taches_server_stream_state(sv, tag: int, cap: int = 4096):
    """(next block, blocks at which the IR changes took effect)."""
    nxt = ctypes.c_int64()
    buf = np.zeros(cap, np.int64)
    n = lib.taches_server_stream_state(sv, tag, ctypes.byref(nxt), _host_ptr(buf), cap)
    _check(min(n, 0), "taches_server_stream_state")
    return int(nxt.value), buf[:min(n, cap)].tolist()


def taches_server_get_stats(sv) -> taches_server_stats:
    out = taches_server_stats()
    _check(lib.taches_server_get_stats(sv, ctypes.byref(out)), "taches_server_get_stats")
    return out


class Pool:
    """A pool of attached streams advanced by one batched launch per step."""

    def __init__(self, max_streams: int, hbm_budget_bytes: int, device: int = 0, torch_stream: bool = True,
                 use_graph: bool = False, tile_r: int = 0):
        self.h = taches_pool_create(max_streams, hbm_budget_bytes, device)
        if torch_stream:
            _check(taches_pool_set_hip_stream(self.h, torch.cuda.current_stream(device).cuda_stream),
                   "taches_pool_set_hip_stream")
        _check(taches_pool_use_graph(self.h, use_graph), "taches_pool_use_graph")
        _check(taches_pool_set_tile(self.h, tile_r), "taches_pool_set_tile")
        self.members = set()

    def attach(self, stream: "Stream") -> int:
        rc = taches_pool_attach(self.h, stream.h)
        if rc == TACHES_OK:
            self.members.add(stream)
        return rc

    def detach(self, stream: "Stream") -> None:
        _check(taches_pool_detach(self.h, stream.h), "taches_pool_detach")
        self.members.discard(stream)

    def step(self, streams, xs, ys, n_blocks) -> None:
        _check(taches_pool_step(self.h, [s.h for s in streams], xs, ys, n_blocks), "taches_pool_step")

    def step_strided(self, stream_ptrs, x_ptrs, x_cstride, y_ptrs, y_cstride, n_blocks) -> None:
        """Step with raw addresses (see taches_pool_step_strided)."""
        _check(taches_pool_step_strided(self.h, stream_ptrs, x_ptrs, x_cstride, y_ptrs, y_cstride, n_blocks),
               "taches_pool_step_strided")

    def set_tile(self, r: int) -> None:
        _check(taches_pool_set_tile(self.h, r), "taches_pool_set_tile")

    def use_graph(self, on: bool) -> None:
        _check(taches_pool_use_graph(self.h, on), "taches_pool_use_graph")

    def synchronize(self) -> None:
        _check(taches_pool_synchronize(self.h), "taches_pool_synchronize")

    def info(self) -> taches_pool_info:
        return taches_pool_get_info(self.h)

    def close(self) -> None:
        if self.h:
            for s in list(self.members):
                self.detach(s)
            _check(taches_pool_destroy(self.h), "taches_pool_destroy")
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
