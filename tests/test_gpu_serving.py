"""Serving on the GPU: a short real-time run with continuous batching; each
kept stream's output in the mix equals the same stream processed alone bit
for bit, and the FP64 oracle within 1e-5 * RMS."""
import math

import numpy as np
import pytest

from paper_2401_01607_amd import workloads as W
from tests.gpu_harness import binding, oracle_run, rel_err, rms_y64

pytestmark = pytest.mark.gpu


def _replay_alone(ex, req, hist, x_in, precision=0):
    """The same request on its own stream: same input blocks, same IR
    versions applied at the same blocks."""
    import torch
    T = binding()
    B, C = req.block, req.channels
    s = T.Stream(B, ex.ir_class(req.ir_len), channels=C, max_blocks_per_call=1, precision=precision,
                 tail=ex.tail_for(req))
    s.set_ir(ex.ir(req, 0))
    swaps = dict((b, v + 1) for v, b in enumerate(hist.swap_blocks))
    outs = []
    for k in range(hist.n_total):
        if k in swaps:
            s.set_ir(ex.ir(req, swaps[k]))
        y = torch.empty((C, B), device="cuda")
        if k < hist.n_in:
            s.process_async(torch.from_numpy(np.ascontiguousarray(x_in[k])).cuda(), y)
        else:
            s.process_blocks(None, y, 1)
        outs.append(y)
    s.synchronize()
    out = torch.stack(outs).cpu().numpy()
    s.close()
    return out


def test_mix_equals_alone_and_oracle():
    from paper_2401_01607_amd.serving import GpuExecutor, Scheduler
    reqs = W.config5_requests(horizon_s=1.2, rate_hz=40.0, seed=77, dur=(0.2, 0.5), lrange=(256, 8192),
                              swap_rate_hz=6.0)
    keep = [r.rid for r in reqs[::4]]
    ex = GpuExecutor(max_streams=16, hbm_budget_bytes=1 << 34, keep_outputs=keep, ir_bank=8,
                     max_ir_len=8192)
    sch = Scheduler(reqs, ex, min_tick_s=0.005)   # ticks 5 ms apart: multi-block catch-up ranges
    st = sch.run_realtime(1.2 + 0.5 + 8192 / 48000 + 1.5)
    assert st["completed"] == st["admitted"] == len(reqs)
    assert st["max_blocks_in_a_range"] > 1
    assert st["steps"] > 0 and "latency_ms_p99" in st
    assert any(len(sch.history[rid].swap_blocks) > 0 for rid in keep)
    checked = 0
    for rid in keep:
        req = next(r for r in reqs if r.rid == rid)
        hist = sch.history[rid]
        x_in, y_mix = ex.kept[rid]
        y_alone = _replay_alone(ex, req, hist, x_in)
        assert np.array_equal(y_mix, y_alone)
        if checked < 2:
            irs = [ex.ir(req, v).cpu().numpy() for v in range(len(hist.swap_blocks) + 1)]
            sched = [(0, 0)] + [(b, v + 1) for v, b in enumerate(hist.swap_blocks)]
            x_planar = x_in.transpose(1, 0, 2).reshape(req.channels, -1)
            ref = oracle_run(x_planar, irs, sched, req.block, req.ir_len, hist.n_total)
            y_planar = y_mix.transpose(1, 0, 2).reshape(req.channels, -1)
            for c in range(req.channels):
                assert rel_err(y_planar[c], ref[c]) <= 1e-5
            checked += 1
    ex.close()


def test_small_budget_queues_requests():
    from paper_2401_01607_amd.serving import GpuExecutor, Scheduler
    T = binding()
    reqs = W.config5_requests(horizon_s=0.3, rate_hz=30.0, seed=78, dur=(0.2, 0.3), lrange=(4096, 4096),
                              swap_rate_hz=0.0)

    def nbytes(B, C):
        cfg = T.taches_config_default(B, 4096)
        cfg.channels = C
        cfg.max_blocks_per_call = GpuExecutor.DEFAULT_MAX_BLOCKS
        return T.taches_bytes_for(cfg)
    per_max = max(nbytes(r.block, r.channels) for r in reqs)
    per_min = min(nbytes(r.block, r.channels) for r in reqs)
    budget = int(2.2 * per_max)
    ex = GpuExecutor(max_streams=64, hbm_budget_bytes=budget, ir_bank=4, max_ir_len=4096)
    sch = Scheduler(reqs, ex)
    st = sch.run_realtime(4.0)
    assert st["max_active_streams"] <= budget // per_min
    assert st["completed"] == len(reqs)
    assert sch.stats.refused_attempts > 0
    ex.close()


def test_split_bf16_mix_equals_alone_and_within_bound():
    """Serving with split-BF16 streams (each runs its Toeplitz MFMA kernel on
    the pool's stream inside the batched step): each kept stream equals the
    same stream processed alone bit for bit, and the FP64 oracle within the
    split-BF16 bound (max |err| <= 1e-4 * RMS)."""
    from paper_2401_01607_amd.serving import GpuExecutor, Scheduler
    T = binding()
    reqs = W.config5_requests(horizon_s=0.8, rate_hz=30.0, seed=79, dur=(0.2, 0.4), lrange=(256, 4096),
                              swap_rate_hz=5.0)
    keep = [r.rid for r in reqs[::3]]
    ex = GpuExecutor(max_streams=16, hbm_budget_bytes=1 << 34, keep_outputs=keep, ir_bank=8,
                     max_ir_len=4096, precision=T.TACHES_PREC_SPLIT_BF16)
    sch = Scheduler(reqs, ex, min_tick_s=0.005)
    st = sch.run_realtime(0.8 + 0.4 + 4096 / 48000 + 1.5)
    assert st["completed"] == st["admitted"] == len(reqs)
    assert any(len(sch.history[rid].swap_blocks) > 0 for rid in keep)
    for i, rid in enumerate(keep):
        req = next(r for r in reqs if r.rid == rid)
        hist = sch.history[rid]
        x_in, y_mix = ex.kept[rid]
        y_alone = _replay_alone(ex, req, hist, x_in, precision=T.TACHES_PREC_SPLIT_BF16)
        assert np.array_equal(y_mix, y_alone)
        if i < 2:
            irs = [ex.ir(req, v).cpu().numpy() for v in range(len(hist.swap_blocks) + 1)]
            sched = [(0, 0)] + [(b, v + 1) for v, b in enumerate(hist.swap_blocks)]
            x_planar = x_in.transpose(1, 0, 2).reshape(req.channels, -1)
            ref = oracle_run(x_planar, irs, sched, req.block, req.ir_len, hist.n_total)
            y_planar = y_mix.transpose(1, 0, 2).reshape(req.channels, -1)
            err = np.abs(y_planar.astype(np.float64) - ref)
            assert err.max() <= 1e-4 * np.sqrt(np.mean(ref ** 2))
    ex.close()


def test_config5_full_load_sampled_parity():
    """The serving workload at full size (Poisson 200 streams/s of 10-60 s,
    L log-uniform in [512, 262 144], mono/stereo, B in {32..512}, IR swaps
    at 0.5/s, 4096 slots, 64 GiB) driven on a simulated clock (2 ms per
    step) through the real executor until about 3 700 streams are active;
    short early requests are kept and, after retiring, checked on sampled
    outputs (both sides of every applied swap) against Eq. (4) in FP64."""
    from oracle import oracle as O
    from paper_2401_01607_amd.serving import GpuExecutor, Scheduler
    horizon = 20.0
    reqs = W.config5_requests(horizon_s=horizon)
    done_by = [r for r in reqs if r.arrival_s < 3.0 and r.arrival_s + r.duration_s + r.ir_len / W.FS < horizon - 2.0]
    keep = [r.rid for r in sorted(done_by, key=lambda r: -r.ir_len)[:2]] + [r.rid for r in done_by[:2]]
    ex = GpuExecutor(max_streams=4096, hbm_budget_bytes=64 << 30, use_graph=True, keep_outputs=keep)
    sch = Scheduler(reqs, ex, step_cost_s=0.002)
    st = sch.run_simulated(horizon)
    assert st["max_active_streams"] >= 3000
    rng = np.random.default_rng(505)
    checked = 0
    for rid in dict.fromkeys(keep):
        req = next(r for r in reqs if r.rid == rid)
        hist = sch.history[rid]
        x_in, y_mix = ex.kept[rid]
        irs = [ex.ir(req, v).cpu().numpy() for v in range(len(hist.swap_blocks) + 1)]
        sched = [(0, 0)] + [(b, v + 1) for v, b in enumerate(hist.swap_blocks)]
        x = x_in.transpose(1, 0, 2).reshape(req.channels, -1)
        y = y_mix.transpose(1, 0, 2).reshape(req.channels, -1).astype(np.float64)
        S = y.shape[1]
        idx = set(rng.integers(0, S, 40).tolist()) | {0, x.shape[1] - 1, x.shape[1], S - 1}
        for b in hist.swap_blocks:
            idx.update([b * req.block - 1, b * req.block])
        idx = np.array(sorted(j for j in idx if 0 <= j < S))
        for c in range(req.channels):
            ref = O.sampled_outputs(x[c], irs, sched, req.block, idx)
            rms = rms_y64(x[c], irs, sched, req.block, S)
            assert np.max(np.abs(y[c][idx] - ref)) <= 1e-5 * rms, f"request {rid} channel {c}"
        checked += 1
    assert checked >= 3
    ex.close()


# ---- serving with one library call per tick (taches_server_tick) ----------

def _swap_rule_blocks(req):
    """Blocks at which a request's IR changes apply: the first block that
    starts at or after each change time, within the input blocks."""
    n_in = max(1, math.ceil(req.n_samples() / req.block))
    out = []
    for t in req.swap_times_s:
        k = 0 if t <= 0 else math.ceil(t * 48000 / req.block - 1e-9)
        while k > 0 and (k - 1) * req.block / 48000 >= t:
            k -= 1
        while k * req.block / 48000 < t:
            k += 1
        if k < n_in:
            out.append(k)
    return out


def _replay_segmented(srv, req, swaps, x, n_in, n_total):
    """A two-segment request on its own: its head and rest streams (the
    server's configurations) run block by block, the head's IR changes at
    its blocks, the rest's at the same input samples inside its blocks;
    y = head + rest shifted by H, added in FP32."""
    import torch
    T = binding()
    shapes, (H, br, _) = srv._shapes(req)
    C, B = req.channels, req.block
    head, rest = [T.Stream(b, cap, channels=C, max_blocks_per_call=1, precision=prec, tail=tail)
                  for b, cap, tail, _, prec in shapes]
    irs = [srv.ir(req, v) for v in range(len(swaps) + 1)]
    head.set_ir(irs[0][:H])
    rest.set_ir(irs[0][H:])
    at_block = {b: v + 1 for v, b in enumerate(swaps)}      # the last change of a block wins
    yh = []
    for k in range(n_total):
        if k in at_block:
            head.set_ir(irs[at_block[k]][:H])
        y = torch.empty((C, B), device="cuda")
        if k < n_in:
            head.process_async(torch.from_numpy(np.ascontiguousarray(x[:, k * B:(k + 1) * B])).cuda(), y)
        else:
            head.process_blocks(None, y, 1)
        yh.append(y)
    r_in = -(-n_in * B // br)
    r_total = max(r_in, -(-(n_total * B - H) // br))
    xr = np.zeros((C, r_in * br), np.float32)
    xr[:, :n_in * B] = x[:, :n_in * B]
    at_rest = {}
    for v, b in enumerate(swaps):
        at_rest[b * B // br] = (v + 1, b * B % br)
    yr = []
    for j in range(r_total):
        if j in at_rest:
            v, off = at_rest[j]
            rest.set_ir(irs[v][H:], offset=off)
        y = torch.empty((C, br), device="cuda")
        if j < r_in:
            rest.process_async(torch.from_numpy(np.ascontiguousarray(xr[:, j * br:(j + 1) * br])).cuda(), y)
        else:
            rest.process_blocks(None, y, 1)
        yr.append(y)
    head.synchronize()
    rest.synchronize()
    out = torch.cat(yh, dim=1).cpu().numpy()
    z = torch.cat(yr, dim=1).cpu().numpy()
    head.close()
    rest.close()
    out[:, H:] += z[:, :out.shape[1] - H]      # float32 + float32, rounded to float32
    return out


def _server_check(precision, seed, tol_max):
    from paper_2401_01607_amd.serving import RealtimeServer
    T = binding()
    reqs = W.config5_requests(horizon_s=1.0, rate_hz=40.0, seed=seed, dur=(0.2, 0.5), lrange=(256, 8192),
                              swap_rate_hz=6.0)
    keep = [r.rid for r in reqs[::3]]
    srv = RealtimeServer(reqs, max_streams=16, hbm_budget_bytes=1 << 34, keep_outputs=keep,
                         max_ir_len=8192, precision=precision)
    st = srv.run_realtime(1.0 + 0.5 + 8192 / 48000 + 1.5)
    assert st["completed"] == st["admitted"] == len(reqs)
    assert st["steps"] > 0 and "latency_ms_p99" in st and st["bytes_h2d"] > 0 and st["bytes_d2h"] > 0
    n_swapped, kinds, seg_swapped_checked = 0, set(), 0
    for i, rid in enumerate(keep):
        req = next(r for r in reqs if r.rid == rid)
        x, y_mix, swaps = srv.kept_outputs(rid)
        assert swaps == _swap_rule_blocks(req)
        n_swapped += len(swaps)
        n_in = max(1, math.ceil(req.n_samples() / req.block))
        n_total = n_in + math.ceil((req.ir_len - 1) / req.block)
        assert y_mix.shape == (req.channels, n_total * req.block)
        B, C = req.block, req.channels
        segmented = srv.segments_for(req) is not None
        kinds.add(segmented)
        if segmented:
            y_alone = _replay_segmented(srv, req, swaps, x, n_in, n_total)
        else:
            x_in = x.reshape(C, n_in, B).transpose(1, 0, 2)

            class Hist:
                pass
            hist = Hist()
            hist.n_in, hist.n_total, hist.swap_blocks = n_in, n_total, swaps
            y_alone = _replay_alone(srv, req, hist, x_in, precision=precision).transpose(1, 0, 2).reshape(C, -1)
        assert np.array_equal(y_mix, y_alone), f"request {rid} (two segments: {segmented})"
        if i < 2 or (segmented and swaps and seg_swapped_checked < 2):
            seg_swapped_checked += bool(segmented and swaps)
            irs = [srv.ir(req, v).cpu().numpy() for v in range(len(swaps) + 1)]
            sched = [(0, 0)] + [(b, v + 1) for v, b in enumerate(swaps)]
            ref = oracle_run(x, irs, sched, B, req.ir_len, n_total)
            for c in range(C):
                assert rel_err(y_mix[c], ref[c]) <= tol_max
    assert n_swapped > 0
    if precision == 0:
        assert kinds == {False, True}   # both one-stream and two-segment requests were served
    srv.close()


def test_server_tick_mix_equals_alone_and_oracle():
    """One library call per tick (input gathered from host memory and copied
    in, outputs copied back): each kept stream equals the same stream run
    alone bit for bit and the FP64 oracle within 1e-5 * RMS, and its IR
    changes apply at the first block starting at or after each change."""
    _server_check(0, 177, 1e-5)


def test_server_tick_split_bf16():
    T = binding()
    _server_check(T.TACHES_PREC_SPLIT_BF16, 179, 1e-4)


def test_server_tick_small_budget_queues():
    from paper_2401_01607_amd.serving import GpuExecutor, RealtimeServer
    T = binding()
    reqs = W.config5_requests(horizon_s=0.3, rate_hz=30.0, seed=78, dur=(0.2, 0.3), lrange=(4096, 4096),
                              swap_rate_hz=0.0)

    def nbytes(B, C):
        cfg = T.taches_config_default(B, 4096)
        cfg.channels = C
        cfg.max_blocks_per_call = 64
        return T.taches_bytes_for(cfg)
    per_max = max(nbytes(r.block, r.channels) for r in reqs)
    per_min = min(nbytes(r.block, r.channels) for r in reqs)
    budget = int(2.2 * per_max)
    srv = RealtimeServer(reqs, max_streams=64, hbm_budget_bytes=budget, max_ir_len=4096)
    st = srv.run_realtime(4.0)
    assert st["max_active_streams"] <= budget // per_min
    assert st["completed"] == len(reqs)
    assert st["refused_attempts"] > 0
    srv.close()


def test_server_add_segmented_rejects_bad_shapes():
    """taches_server_add_segmented refuses (EINVAL, nothing registered)
    segments that break its rules: Br not a multiple of B, H < Br, a ring
    shorter than 2 Br or not a multiple of Br, a split-BF16 stream, an IR no longer than H, and two
    IR changes inside one rest block (the initial IR counting as one)."""
    import torch
    T = binding()
    pool = T.Pool(8, 1 << 30)
    sv = T.taches_server_create(pool.h, 48000.0, 4, 0.0)
    C, B, L = 1, 64, 8192
    h = torch.randn(L, device="cuda")
    x = np.zeros((C, 40 * B), np.float32)

    def stream(b, cap, prec=0):
        s = T.Stream(b, cap, channels=C, max_blocks_per_call=4, precision=prec)
        assert pool.attach(s) == T.TACHES_OK
        return s
    head, rest = stream(B, 1024), stream(512, 8192)
    ring = torch.empty((C, 4096), device="cuda")

    def add(hd, rs, H, z, ir=h, swaps=(), tag=1):
        irs = [ir for _ in swaps]
        return T.taches_server_add_segmented(sv, hd.h, rs.h, H, z, tag, 0.0, 40, 40 + L // B, x, None, ir,
                                             list(swaps), irs)
    assert add(head, rest, 256, ring) == T.TACHES_EINVAL                     # H < Br
    odd = stream(96, 8192)
    assert add(head, odd, 1024, ring) == T.TACHES_EINVAL                     # Br not a multiple of B
    assert add(head, rest, 1024, torch.empty((C, 512), device="cuda")) == T.TACHES_EINVAL   # ring < 2 Br
    assert add(head, rest, 1024, torch.empty((C, 4000), device="cuda")) == T.TACHES_EINVAL  # not a multiple of Br
    assert add(head, rest, 1024, ring, ir=h[:1024]) == T.TACHES_EINVAL       # IR not longer than H
    split = stream(512, 8192, prec=T.TACHES_PREC_SPLIT_BF16)
    assert add(head, split, 1024, ring) == T.TACHES_EINVAL                   # rest segment not FP32
    assert add(head, rest, 1024, ring, swaps=[128 / 48000]) == T.TACHES_EINVAL           # inside rest block 0
    assert add(head, rest, 1024, ring, swaps=[640 / 48000, 900 / 48000]) == T.TACHES_EINVAL  # two in block 1
    assert T.taches_server_get_stats(sv).streams == 0
    assert add(head, rest, 1024, ring, swaps=[512 / 48000, 1100 / 48000]) == T.TACHES_OK
    assert T.taches_server_get_stats(sv).streams == 1
    T.taches_server_destroy(sv)
    for s in (head, rest, odd, split):
        pool.detach(s)
        s.close()
    pool.close()


def test_server_tick_full_load_sampled_parity():
    """The serving workload at full rate through the library tick, as the
    benchmark runs it (Poisson 200 streams/s of 10-60 s, L log-uniform in
    [512, 262 144], mono/stereo, B in {32..512}, IR changes at 0.5/s, real
    time, long IRs in two segments): 14 s of real time, about 2 800
    requests admitted.  Kept requests that finish in the run (the longest
    IRs among the early ones, and the first ones) are checked on sampled
    outputs, both sides of every applied IR change, against Eq. (4) in FP64."""
    from oracle import oracle as O
    from paper_2401_01607_amd.serving import RealtimeServer
    horizon = 14.0
    reqs = W.config5_requests(horizon_s=horizon)
    done_by = [r for r in reqs if r.arrival_s < 2.0 and r.arrival_s + r.duration_s + r.ir_len / W.FS < horizon - 1.5]
    keep = list(dict.fromkeys([r.rid for r in sorted(done_by, key=lambda r: -r.ir_len)[:3]] +
                              [r.rid for r in done_by[:2]]))
    srv = RealtimeServer(reqs, max_streams=4096, hbm_budget_bytes=64 << 30, keep_outputs=keep)
    st = srv.run_realtime(horizon)
    assert st["admitted"] >= 2000 and st["completed"] >= len(keep)
    rng = np.random.default_rng(606)
    checked = segmented = 0
    for rid in keep:
        req = next(r for r in reqs if r.rid == rid)
        got = srv.kept_outputs(rid)
        assert got is not None, f"request {rid} not admitted"
        x, y, swaps = got
        n_in = max(1, math.ceil(req.n_samples() / req.block))
        n_total = n_in + math.ceil((req.ir_len - 1) / req.block)
        assert y.shape[1] == n_total * req.block, f"request {rid} did not finish"
        assert swaps == _swap_rule_blocks(req)
        irs = [srv.ir(req, v).cpu().numpy() for v in range(len(swaps) + 1)]
        sched = [(0, 0)] + [(b, v + 1) for v, b in enumerate(swaps)]
        S = y.shape[1]
        idx = set(rng.integers(0, S, 60).tolist()) | {0, x.shape[1] - 1, x.shape[1], S - 1}
        for b in swaps:
            idx.update([b * req.block - 1, b * req.block])
        seg = srv.segments_for(req)
        if seg is not None:   # both sides of where the rest segment starts to count, and of its blocks
            H, br, _ = seg
            idx.update([H - 1, H, H + br - 1, H + br])
            segmented += 1
        idx = np.array(sorted(j for j in idx if 0 <= j < S))
        for c in range(req.channels):
            ref = O.sampled_outputs(x[c], irs, sched, req.block, idx)
            rms = rms_y64(x[c], irs, sched, req.block, S)
            assert np.max(np.abs(y[c][idx].astype(np.float64) - ref)) <= 1e-5 * rms, f"request {rid} channel {c}"
        checked += 1
    assert checked == len(keep) and segmented >= 2
    srv.close()


def test_server_admission_failure_is_raised():
    """An error on the preparing thread (forced from the host) stops the
    run with an exception instead of leaving requests unadmitted."""
    from paper_2401_01607_amd.serving import RealtimeServer
    reqs = W.config5_requests(horizon_s=0.2, rate_hz=20.0, seed=80, dur=(0.2, 0.3), lrange=(512, 2048))
    srv = RealtimeServer(reqs, max_streams=8, hbm_budget_bytes=1 << 30)

    def fail(req):
        raise MemoryError("forced")
    srv._prepare = fail
    with pytest.raises(RuntimeError, match="admission failed"):
        srv.run_realtime(2.0)
    srv.close()
