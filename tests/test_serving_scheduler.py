"""Serving policy on the CPU: the scheduler driven on a simulated clock by a
stub executor that runs each stream through the oracle."""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2401_01607_amd import workloads as W
from paper_2401_01607_amd.serving import AdmissionRefused, MissGate, Scheduler


class OracleExecutor:
    """Slots and a byte budget like the pool; outputs from the FP64 oracle."""

    def __init__(self, max_streams, budget, max_blocks_per_step=1):
        self.max_streams, self.budget = max_streams, budget
        self.max_blocks_per_step = max_blocks_per_step
        self.live, self.used, self.out, self.steps = {}, 0, {}, []
        self.active_counts = []
        self.max_range = 0

    @staticmethod
    def bytes_for(req):
        return req.channels * (req.ir_len + req.block) * 4 + 2 * req.ir_len * 4

    @staticmethod
    def ir(req, v):
        return W.impulse_response(req.ir_len, req.seed * 1000 + 7 + v)

    @staticmethod
    def signal(req):
        n_in = max(1, math.ceil(req.n_samples() / req.block))
        x = np.zeros((req.channels, n_in * req.block), np.float32)
        rng = np.random.default_rng(req.seed)
        x[:, :req.n_samples()] = rng.standard_normal((req.channels, req.n_samples())).astype(np.float32)
        return x

    def admit(self, req):
        b = self.bytes_for(req)
        if len(self.live) >= self.max_streams or self.used + b > self.budget:
            raise AdmissionRefused("full")
        s = O.OracleStream(req.block, req.ir_len, req.channels)
        s.set_ir(self.ir(req, 0))
        self.live[req.rid] = (s, self.signal(req), [], req)
        self.used += b
        return req.rid

    def set_ir(self, h, req, v):
        self.live[h][0].set_ir(self.ir(req, v))

    def step(self, handles, k0s, ns):
        self.steps.append(len(handles))
        self.active_counts.append(len(self.live))
        assert len(set(handles.tolist())) == len(handles)
        for h, k0, n in zip(handles.tolist(), k0s.tolist(), ns.tolist()):
            assert 1 <= n <= self.max_blocks_per_step
            self.max_range = max(self.max_range, n)
            s, x, ys, req = self.live[h]
            assert len(ys) == k0, "ranges of a stream are consecutive"
            for k in range(k0, k0 + n):
                xb = x[:, k * req.block:(k + 1) * req.block]
                if xb.shape[1] < req.block:
                    xb = np.zeros((req.channels, req.block), np.float32)
                ys.append(s.process(xb)[1])

    def retire(self, h, req):
        s, x, ys, _ = self.live.pop(h)
        self.out[h] = (x, np.concatenate(ys, axis=1))
        self.used -= self.bytes_for(req)


def _reqs(n, rate, dur=(0.02, 0.08), L=(32, 600), seed=5, swap_rate=30.0):
    return W.config5_requests(horizon_s=n / rate, rate_hz=rate, seed=seed, dur=dur, lrange=L, swap_rate_hz=swap_rate)


@pytest.mark.parametrize("max_blocks,step_cost", [(1, 1e-4), (16, 4e-3)])
def test_every_request_completes_with_its_exact_output(max_blocks, step_cost):
    """Also with multi-block catch-up ranges: a range never runs past a due
    IR swap or the end of the input, so swaps still land on the first block
    starting at or after their time."""
    reqs = _reqs(30, 200.0)
    ex = OracleExecutor(max_streams=8, budget=1 << 30, max_blocks_per_step=max_blocks)
    sch = Scheduler(reqs, ex, step_cost_s=step_cost)
    st = sch.run_simulated(10.0)
    assert st["admitted"] == st["completed"] == len(reqs)
    assert (ex.max_range > 1) == (max_blocks > 1)
    for r in reqs:
        x, y = ex.out[r.rid]
        a = sch.history[r.rid]
        # swaps apply at the first block starting at or after their time
        want = [math.ceil(t * W.FS / r.block - 1e-9) for t in r.swap_times_s]
        want = [b for b in want if b < a.n_in]
        assert a.swap_blocks == want
        sched = [(0, 0)] + [(b, v + 1) for v, b in enumerate(a.swap_blocks)]
        irs = [ex.ir(r, v) for v in range(len(a.swap_blocks) + 1)]
        n_blocks = a.n_in + a.n_drain
        for c in range(r.channels):
            ref = O.run_channel(x[c], irs, sched, r.block, r.ir_len, n_blocks=n_blocks)
            assert np.array_equal(y[c], ref)
        # the drain covers the temporal overflow: nothing is left after it
        assert n_blocks * r.block >= r.n_samples() + r.ir_len - 1


def test_slot_limit_and_fifo_admission():
    reqs = _reqs(40, 2000.0, dur=(0.05, 0.1))
    ex = OracleExecutor(max_streams=3, budget=1 << 30)
    sch = Scheduler(reqs, ex, step_cost_s=1e-4)
    st = sch.run_simulated(10.0)
    assert max(ex.active_counts) <= 3
    assert st["completed"] == len(reqs)
    assert st["queue_wait_s_p99"] > 0
    order = sorted(sch.history.values(), key=lambda a: a.start_s)
    assert [a.req.rid for a in order] == sorted(a.req.rid for a in order)  # FIFO


def test_hbm_budget_limits_admission():
    reqs = _reqs(20, 2000.0, L=(4000, 4000))
    per = OracleExecutor.bytes_for(reqs[0])
    ex = OracleExecutor(max_streams=100, budget=int(2.5 * per) + 10_000)
    sch = Scheduler(reqs, ex, step_cost_s=1e-4)
    sch.run_simulated(10.0)
    assert max(ex.active_counts) <= 2
    assert sch.stats.refused_attempts > 0
    assert sch.stats.completed == len(reqs)


def test_latency_is_step_completion_minus_block_arrival():
    reqs = _reqs(5, 50.0)
    ex = OracleExecutor(max_streams=10, budget=1 << 30)
    sch = Scheduler(reqs, ex, step_cost_s=2e-3)
    st = sch.run_simulated(10.0)
    lat = np.array(sch.stats.latencies_s)
    assert np.all(lat >= 2e-3 - 1e-12)
    assert st["latency_ms_p50"] >= 2.0
    assert st["blocks"] == sum(a.n_in + a.n_drain for a in sch.history.values())


def test_continuous_batching_joins_streams_in_one_step():
    """Blocks that arrive while a step runs, from streams admitted at
    different times, join the next step."""
    reqs = _reqs(12, 400.0, dur=(0.2, 0.3))
    ex = OracleExecutor(max_streams=16, budget=1 << 30)
    sch = Scheduler(reqs, ex, step_cost_s=2e-3)
    sch.run_simulated(10.0)
    assert max(ex.steps) >= 4
    ex2 = OracleExecutor(max_streams=16, budget=1 << 30)
    sch2 = Scheduler(reqs, ex2, step_cost_s=0.0, min_tick_s=5e-3)
    sch2.run_simulated(10.0)
    assert max(ex2.steps) >= 4 and len(ex2.steps) < len(ex.steps) * 3


class SplitOracleExecutor(OracleExecutor):
    """The same executor offering the step split into launch and wait."""

    def __init__(self, *a, **k):
        super().__init__(*a, **k)
        self.calls, self._queued = [], None

    def launch(self, handles, k0s, ns):
        assert self._queued is None, "one step at a time"
        self.calls.append("launch")
        self._queued = (handles.copy(), k0s.copy(), ns.copy())

    def wait(self):
        assert self._queued is not None
        self.calls.append("wait")
        self.step(*self._queued)
        self._queued = None


def test_split_launch_and_wait_give_the_same_records():
    """An executor with launch/wait: the scheduler prepares the block records
    between the two calls, and the run (outputs, latencies, deadlines,
    counters) equals the run through step() on the same simulated clock."""
    reqs = _reqs(30, 200.0)
    runs = []
    for cls in (OracleExecutor, SplitOracleExecutor):
        ex = cls(max_streams=8, budget=1 << 30, max_blocks_per_step=16)
        sch = Scheduler(reqs, ex, step_cost_s=4e-3, warmup_s=0.02)
        st = sch.run_simulated(10.0)
        runs.append((ex, sch, st))
    (ex_a, sch_a, st_a), (ex_b, sch_b, st_b) = runs
    assert ex_b.calls and ex_b.calls == ["launch", "wait"] * (len(ex_b.calls) // 2)
    busy = "step_busy_fraction"          # measured host time, not simulated
    assert {k: v for k, v in st_a.items() if k != busy} == {k: v for k, v in st_b.items() if k != busy}
    assert np.array_equal(sch_a.stats.latencies_s, sch_b.stats.latencies_s)
    assert np.array_equal(sch_a.stats.deadlines_s, sch_b.stats.deadlines_s)
    assert sch_a.stats.latencies_s.size > 0
    for r in reqs:
        assert np.array_equal(ex_a.out[r.rid][1], ex_b.out[r.rid][1])


# ---- two-segment serving: the decomposition the server applies -------------

def _seg_request(L, B, swaps, dur_s=0.05, C=1, seed=3):
    return W.ServingRequest(rid=0, arrival_s=0.0, duration_s=dur_s, channels=C, block=B, ir_len=L,
                           seed=seed, swap_times_s=list(swaps))


def test_change_blocks_rule():
    from paper_2401_01607_amd.serving import change_blocks
    fs = W.FS
    req = _seg_request(4096, 64, [0.0, 64 / fs, 64.5 / fs, 0.02, 1.0])
    n_in = math.ceil(req.n_samples() / 64)
    # a change at t applies to the first block starting at or after t; none after the input
    assert change_blocks(req) == [0, 1, 2, math.ceil(0.02 * fs / 64)]
    assert all(k < n_in for k in change_blocks(req))


def test_segments_rule():
    from paper_2401_01607_amd import taches as T
    from paper_2401_01607_amd.serving import segments_for
    fp32, split = T.TACHES_PREC_FP32, T.TACHES_PREC_SPLIT_BF16
    assert segments_for(_seg_request(512, 32, []), fp32) is None          # shorter than four rest blocks
    assert segments_for(_seg_request(65536, 32, []), split) is None       # split-BF16 streams stay whole
    for L, B in [(2048, 32), (41_940, 64), (262_144, 512), (8192, 512)]:
        H, br, Z = segments_for(_seg_request(L, B, []), fp32)
        assert br & (br - 1) == 0 and br % B == 0 and max(B, 256) <= br <= 2048 and H == br
        assert L >= 4 * br and Z % br == 0 and Z >= 4 * br + 8 * B
    # two changes inside one rest block: served whole
    H, br, _ = segments_for(_seg_request(65536, 32, []), fp32)
    assert segments_for(_seg_request(65536, 32, [br / W.FS + 32 / W.FS, br / W.FS + 96 / W.FS]), fp32) is None
    assert segments_for(_seg_request(65536, 32, [br / W.FS, 2 * br / W.FS + 32 / W.FS]), fp32) is not None
    # a change inside the first rest block, where the initial IR starts: served whole
    assert segments_for(_seg_request(65536, 32, [64 / W.FS]), fp32) is None
    assert segments_for(_seg_request(65536, 32, [0.0]), fp32) is not None


@pytest.mark.parametrize("L,B,swaps", [
    (3000, 32, []),
    (9000, 64, [0.013, 0.031]),
    (20000, 128, [0.0, 0.013, 0.031]),
])
def test_two_segments_equal_the_whole_ir(L, B, swaps):
    """y = head + rest shifted by H, with the head's IR changes at its blocks
    and the rest's at the same input samples (inside its longer blocks),
    equals the whole IR's taches exactly on integer inputs (Eq. (1) is
    linear in h; the oracle runs all three)."""
    from paper_2401_01607_amd import taches as T
    from paper_2401_01607_amd.serving import change_blocks, segments_for
    req = _seg_request(L, B, swaps, dur_s=0.045)
    H, br, _ = segments_for(req, T.TACHES_PREC_FP32)
    n_in = math.ceil(req.n_samples() / B)
    n_total = n_in + math.ceil((L - 1) / B)
    ks = change_blocks(req)
    rng = np.random.default_rng(L)
    irs = [rng.integers(-8, 9, L).astype(np.float32) for _ in range(len(ks) + 1)]
    x = rng.integers(-8, 9, n_in * B).astype(np.float32)
    whole = O.run_channel(x, irs, [(0, 0)] + [(k, v + 1) for v, k in enumerate(ks)], B, L, n_total)
    head = O.run_channel(x, [h[:H] for h in irs], [(0, 0)] + [(k, v + 1) for v, k in enumerate(ks)], B, H, n_total)
    r_in = -(-n_in * B // br)
    r_total = max(r_in, -(-(n_total * B - H) // br))
    xr = np.zeros(r_in * br, np.float32)
    xr[:x.size] = x
    rest_sched = [(0, 0)] + [(k * B // br, v + 1, k * B % br) for v, k in enumerate(ks)]
    z = O.run_channel(xr, [h[H:] for h in irs], rest_sched, br, L - H, r_total)
    y = head.copy()
    y[H:] += z[:y.size - H]
    assert np.array_equal(y, whole)


def test_miss_gate_closes_above_target_and_reopens_at_half():
    """The admission gate: closes when more than the target fraction of the
    blocks of at least min_block samples missed one block period, reopens at
    half the target or below; shorter blocks do not count."""
    g = MissGate(0.02, min_block=64)
    dl = 64 / W.FS

    def batch(n, late, b=64):
        lat = np.full(n, 0.5 * dl)
        lat[:late] = 1.5 * dl
        return lat, np.full(n, b, np.int32)

    g.update(*batch(100, 2))             # 2 % = target: stays open
    assert not g.closed
    g.update(*batch(100, 3))             # 3 % > 2 %: closes
    assert g.closed
    g.update(*batch(200, 3))             # 1.5 % > 1 %: stays closed
    assert g.closed
    g.update(*batch(200, 2))             # 1 % = half the target: reopens
    assert not g.closed
    g.update(*batch(50, 50, b=32))       # only short blocks, all late: no change
    assert not g.closed
    lat = np.full(10, dl)                # exactly one period is not a miss
    g.update(lat, np.full(10, 64, np.int32))
    assert not g.closed
    s = g.summary()
    assert s["checks"] == 6 and s["closed_fraction_of_checks"] == round(2 / 6, 4)
    with pytest.raises(ValueError):
        MissGate(0.0)
