"""Helpers for the GPU tests: run a stream spec through the HIP library
(per-block and multi-block) and through the oracle, and compare."""
from __future__ import annotations

import numpy as np


def binding():
    from paper_2401_01607_amd import taches as T
    return T


def pad_signal(x: np.ndarray, n_blocks: int, B: int) -> np.ndarray:
    """[C, N] -> [C, n_blocks*B] zero-padded float32."""
    x = np.atleast_2d(np.asarray(x, dtype=np.float32))
    out = np.zeros((x.shape[0], n_blocks * B), dtype=np.float32)
    n = min(x.shape[1], n_blocks * B)
    out[:, :n] = x[:, :n]
    return out


def gpu_per_block(x, irs, schedule, B, Lmax, n_blocks, tail=0, tile=None, host_io=False, precision=0):
    """One taches_process_async (or taches_process) call per block; IR swaps
    through taches_set_ir before the scheduled block."""
    import torch
    T = binding()
    xp = pad_signal(x, n_blocks, B)
    C = xp.shape[0]
    s = T.Stream(B, Lmax, channels=C, tail=tail, precision=precision)
    if tile:
        s.set_tile(*tile)
    sched = {e[0]: (e[1], e[2] if len(e) > 2 else 0) for e in schedule}
    if host_io:
        ys = []
        for b in range(n_blocks):
            if b in sched:
                s.set_ir(irs[sched[b][0]], sched[b][1])
            ys.append(s.process(xp[:, b * B:(b + 1) * B]))
        y = np.concatenate(ys, axis=1)
    else:
        xb = torch.from_numpy(np.ascontiguousarray(xp.reshape(C, n_blocks, B).transpose(1, 0, 2))).cuda()
        yb = torch.empty_like(xb)
        for b in range(n_blocks):
            if b in sched:
                s.set_ir(irs[sched[b][0]], sched[b][1])
            s.process_async(xb[b], yb[b])
        s.synchronize()
        y = yb.cpu().numpy().transpose(1, 0, 2).reshape(C, n_blocks * B)
    info = s.info()
    s.close()
    return y, info


def gpu_multi_block(x, irs, schedule, B, Lmax, n_blocks, tail=0, tile=None, calls=1, drain_x_null=0,
                    precision=0):
    """All blocks in ``calls`` taches_process_blocks calls with an IR-slot
    schedule; then ``drain_x_null`` blocks with x = NULL."""
    import torch
    T = binding()
    xp = pad_signal(x, n_blocks, B)
    C = xp.shape[0]
    per = -(-n_blocks // calls)
    s = T.Stream(B, Lmax, channels=C, max_blocks_per_call=max(per, drain_x_null, 1), tail=tail,
                 ir_slots=max(2, len(irs)), precision=precision)
    if tile:
        s.set_tile(*tile)
    for k, h in enumerate(irs):
        s.load_ir_slot(k, h)
    sched = np.full(n_blocks, -1, dtype=np.int32)
    offs = np.zeros(n_blocks, dtype=np.int32)
    for e in schedule:
        if e[0] < n_blocks:
            sched[e[0]] = e[1]
            offs[e[0]] = e[2] if len(e) > 2 else 0
    use_offs = bool(np.any(offs))
    outs = []
    for c0 in range(0, n_blocks, per):
        nb = min(per, n_blocks - c0)
        xd = torch.from_numpy(np.ascontiguousarray(xp[:, c0 * B:(c0 + nb) * B])).cuda()
        yd = torch.empty_like(xd)
        s.process_blocks(xd, yd, nb, sched[c0:c0 + nb], offs[c0:c0 + nb] if use_offs else None)
        outs.append(yd)
    if drain_x_null:
        yd = torch.empty((C, drain_x_null * B), dtype=torch.float32, device="cuda")
        s.process_blocks(None, yd, drain_x_null)
        outs.append(yd)
    s.synchronize()
    y = torch.cat([o.cpu() for o in outs], dim=1).numpy()
    info = s.info()
    s.close()
    return y, info


def oracle_run(x, irs, schedule, B, Lmax, n_blocks):
    from oracle import oracle as O
    xp = np.atleast_2d(np.asarray(x, dtype=np.float32))
    return np.stack(O.run_channels(list(xp), irs, schedule, B, Lmax, n_blocks=n_blocks))


def oracle_abs_run(x, irs, schedule, B, Lmax, n_blocks):
    """sum_k |h_k| |x_{n-k}| per output: the oracle on absolute values."""
    xa = np.abs(np.atleast_2d(np.asarray(x, dtype=np.float32)))
    return oracle_run(xa, [np.abs(np.asarray(h, np.float32)) for h in irs], schedule, B, Lmax, n_blocks)


def rel_err(y, y64):
    """max |y - y64| / RMS(y64) over all outputs."""
    y = np.asarray(y, np.float64)
    rms = float(np.sqrt(np.mean(np.square(y64))))
    return float(np.max(np.abs(y - y64))) / rms if rms > 0 else float(np.max(np.abs(y - y64)))


def rms_y64(x, irs, schedule, B, n_out):
    """RMS over every output (all channels, n_out samples each) of the FP64
    result of Eq. (4): the normaliser of the stated tolerances.  Computed
    with the oracle's FFT helper (FP64; its error is far below the
    tolerances)."""
    from oracle import oracle as O
    y = O.fft_outputs(np.atleast_2d(np.asarray(x, dtype=np.float32)), irs, schedule, B, n_out)
    return float(np.sqrt(np.mean(np.square(y))))
