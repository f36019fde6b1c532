"""Parity of the FP32 gather path (K1, and K1d with the FP64 tail) with the
CPU oracle, through the C-ABI.  Tolerance for float inputs:
max |y_gpu - y_fp64_oracle| <= 1e-5 * RMS(y_fp64_oracle); integer-valued
inputs (every partial sum exact) must match bit for bit."""
import numpy as np
import pytest

from paper_2401_01607_amd import workloads as W
from tests.gpu_harness import gpu_multi_block, gpu_per_block, oracle_run, rel_err, rms_y64

pytestmark = pytest.mark.gpu

TOL = 1e-5

INT_CASES = [
    # B, L1, L2, n, swap blocks
    (1, 1, 1, 20, [5]),
    (2, 3, 5, 50, [3, 10]),
    (3, 7, 2, 40, [4]),
    (5, 16, 16, 100, []),
    (8, 100, 37, 500, [10, 20, 30]),
    (64, 10, 10, 300, [1]),          # B > L
    (64, 1000, 500, 5000, [7, 40]),
    (300, 700, 1200, 4000, [3, 5]),  # B not a power of two, two chunks per block
    (513, 2000, 64, 6000, [2]),      # three chunks per block
]


def _int_case(B, L1, L2, n, swaps, seed=1):
    amp = 31 if max(L1, L2) > 1000 else 100
    x = W.signal_int(n, seed, amp)
    irs = [W.signal_int(L1, seed + 1, amp), W.signal_int(L2, seed + 2, amp)]
    sched = [(0, 0)] + [(b, (i + 1) % 2) for i, b in enumerate(swaps)]
    Lmax = max(L1, L2)
    n_blocks = -(-(n + Lmax) // B) + 1
    return x, irs, sched, Lmax, n_blocks


@pytest.mark.parametrize("case", INT_CASES, ids=[f"B{c[0]}_L{c[1]}-{c[2]}" for c in INT_CASES])
def test_integer_inputs_bitwise(case):
    x, irs, sched, Lmax, nb = _int_case(*case)
    B = case[0]
    ref = oracle_run(x, irs, sched, B, Lmax, nb)
    y1, _ = gpu_per_block(x, irs, sched, B, Lmax, nb)
    assert np.array_equal(y1, ref)
    y2, _ = gpu_multi_block(x, irs, sched, B, Lmax, nb)
    assert np.array_equal(y2, ref)
    y3, _ = gpu_multi_block(x, irs, sched, B, Lmax, nb, tail=2)  # FP64 tail
    assert np.array_equal(y3, ref)


def test_host_blocking_path_bitwise():
    x, irs, sched, Lmax, nb = _int_case(*INT_CASES[6])
    ref = oracle_run(x, irs, sched, 64, Lmax, nb)
    y, _ = gpu_per_block(x, irs, sched, 64, Lmax, nb, host_io=True)
    assert np.array_equal(y, ref)


def test_config1_parity_and_modes_agree():
    """Plain taches, 48 000 uniform samples, L = 1024, B = 64 (plus drain)."""
    spec = W.config1()
    B, L = spec.block, spec.max_ir_len
    nb = -(-(spec.n_samples + L - 1) // B)
    ref = oracle_run(spec.x, spec.irs, spec.schedule, B, L, nb)
    y1, i1 = gpu_per_block(spec.x, spec.irs, spec.schedule, B, L, nb)
    assert rel_err(y1, ref) <= TOL
    y2, _ = gpu_multi_block(spec.x, spec.irs, spec.schedule, B, L, nb)
    assert np.array_equal(y1, y2), "per-block and multi-block calls must agree bit for bit"
    y3, _ = gpu_multi_block(spec.x, spec.irs, spec.schedule, B, L, nb, calls=7)
    assert np.array_equal(y1, y3)
    assert i1.tail_fp64 == 0


@pytest.mark.parametrize("tile", [(r, w) for r in (4, 8, 12, 14, 16) for w in (1, 2, 4)])
def test_every_tile_shape_gives_the_same_bits(tile):
    spec = W.config2(n=20_000, L=5000, block=256, period=4800)
    nb = -(-(spec.n_samples + 4999) // 256)
    base, _ = gpu_multi_block(spec.x, spec.irs, spec.schedule, 256, 5000, nb, tile=(16, 1))
    y, info = gpu_multi_block(spec.x, spec.irs, spec.schedule, 256, 5000, nb, tile=tile)
    assert (info.tile_r, info.tile_w) == tile
    assert np.array_equal(y, base)


def test_config2_reduced_parity_with_swaps():
    """Config-2 shape (L = 65 536, B = 256, IR swapped every 4800 samples)
    on the first second of input, plus the full temporal overflow."""
    spec = W.config2(n=48_000)
    B, L = 256, 65_536
    nb = -(-(spec.n_samples + L - 1) // B)
    ref = oracle_run(spec.x, spec.irs, spec.schedule, B, L, nb)
    y, info = gpu_multi_block(spec.x, spec.irs, spec.schedule, B, L, nb)
    assert rel_err(y, ref) <= TOL
    yb, _ = gpu_per_block(spec.x, spec.irs, spec.schedule, B, L, nb)
    assert np.array_equal(y, yb)
    # the FP64 tail is at least as accurate
    y64, _ = gpu_multi_block(spec.x, spec.irs, spec.schedule, B, L, nb, tail=2)
    assert rel_err(y64, ref) <= rel_err(y, ref) + 1e-9


def test_swap_one_block_off_differs():
    spec = W.config2(n=12_000, L=2000, block=256, period=4800)
    nb = -(-(12_000 + 1999) // 256)
    y, _ = gpu_multi_block(spec.x, spec.irs, spec.schedule, 256, 2000, nb)
    shifted = [(b + 1 if b > 0 else 0, k) for b, k in spec.schedule]
    ref_shift = oracle_run(spec.x, spec.irs, shifted, 256, 2000, nb)
    assert rel_err(y, ref_shift) > 1e-2


def test_impulse_returns_h_exactly():
    h = W.impulse_response(3000, 5)
    for d in (0, 255, 256, 3 * 256 + 3):
        x = np.zeros(d + 1, np.float32)
        x[d] = 1.0
        nb = -(-(d + 3000) // 256) + 1
        y, _ = gpu_multi_block(x, [h], [(0, 0)], 256, 3000, nb)
        want = np.zeros(nb * 256, np.float32)
        want[d:d + 3000] = h
        assert np.array_equal(y[0], want)


def test_drain_with_null_input_and_exact_zero_after_overflow():
    x = W.signal_int(1000, 9, 50)
    h = W.signal_int(700, 10, 50)
    B = 128
    nb_in = -(-1000 // B)
    nb_drain = -(-699 // B) + 2
    ref = oracle_run(x, [h], [(0, 0)], B, 700, nb_in + nb_drain)
    import torch
    from tests.gpu_harness import binding
    T = binding()
    s = T.Stream(B, 700, max_blocks_per_call=nb_drain)
    s.set_ir(h)
    xp = np.zeros(nb_in * B, np.float32)
    xp[:1000] = x
    xd = torch.from_numpy(xp).cuda()[None]
    y1 = torch.empty_like(xd)
    s.process_blocks(xd, y1, nb_in)
    y2 = torch.empty((1, nb_drain * B), device="cuda")
    s.process_blocks(None, y2, nb_drain)
    y = torch.cat([y1, y2], 1).cpu().numpy()[0]
    assert np.array_equal(y, ref[0])
    assert not np.any(y[1000 + 699:])
    assert s.info().live == 0


def test_tail_state_matches_oracle_residue():
    """After a few blocks the device tail equals the oracle's residue in
    output order (Section 4.2's r, read from the current index on)."""
    from oracle import oracle as O
    from tests.gpu_harness import binding
    T = binding()
    B, L = 64, 500
    x = W.signal_int(5 * B, 3, 100)
    h = W.signal_int(L, 4, 100)
    o = O.OracleStream(B, L, 1)
    o.set_ir(h)
    s = T.Stream(B, L)
    s.set_ir(h)
    for b in range(5):
        o.process(x[b * B:(b + 1) * B])
        s.process(x[b * B:(b + 1) * B])
    assert np.array_equal(s.read_tail(0, L), o.residue(0))


def test_multichannel_fp32_matches_per_channel_oracle():
    C, B, L, n = 5, 128, 3000, 6000
    x = np.stack([W.signal_gauss(n, 100 + c) for c in range(C)])
    h = W.impulse_response(L, 99)
    nb = -(-(n + L - 1) // B)
    ref = oracle_run(x, [h], [(0, 0)], B, L, nb)
    y, _ = gpu_multi_block(x, [h], [(0, 0)], B, L, nb)
    for c in range(C):
        assert rel_err(y[c], ref[c]) <= TOL
    yb, _ = gpu_per_block(x, [h], [(0, 0)], B, L, nb)
    assert np.array_equal(y, yb)


def test_flat_white_noise_ir_parity():
    """The paper's IRs are flat white noise (Section 5.1), the worst case."""
    x = W.signal_gauss(20_000, 21)
    h = W.impulse_response(16_384, 22, decay=0.0)
    nb = -(-(20_000 + 16_383) // 256)
    ref = oracle_run(x, [h], [(0, 0)], 256, 16_384, nb)
    y, _ = gpu_multi_block(x, [h], [(0, 0)], 256, 16_384, nb)
    assert rel_err(y, ref) <= TOL


def test_long_ir_auto_picks_fp64_tail():
    from tests.gpu_harness import binding
    T = binding()
    s = T.Stream(512, 1 << 18)
    assert s.info().tail_fp64 == 1
    s.close()
    s = T.Stream(32, 32_768)
    assert s.info().tail_fp64 == 0
    s.close()
    s = T.Stream(32, 32_769)
    assert s.info().tail_fp64 == 1
    s.close()


@pytest.mark.parametrize("B,L", [(32, 32_768), (64, 65_536), (128, 131_072)])
def test_fp32_tail_at_the_auto_limit_meets_the_tolerance(B, L):
    """The longest IRs that AUTO leaves on an FP32 tail (1024 chunk sums per
    output), with a flat white-noise IR (the paper's IR shape, which gives
    the largest errors): every output within 1e-5 * RMS of the FP64 result."""
    from oracle import oracle as O
    n = 96_000
    x = W.signal_gauss(n, 151)
    h = W.impulse_response(L, 152, decay=0.0)
    nb = -(-(n + L - 1) // B)
    y, info = gpu_multi_block(x, [h], [(0, 0)], B, L, nb)
    assert info.tail_fp64 == 0
    n_out = n + L - 1
    y64 = O.fft_outputs(x, [h], [(0, 0)], B, n_out)
    assert rel_err(y[0][:n_out], y64) <= TOL


def test_longest_ir_4m_taps_streaming_sampled_parity():
    """A stream with a 4 194 304-tap IR (FP64 tail chosen automatically):
    40 blocks of 256 in one call, then the whole temporal overflow (16 384
    zero blocks) in one NULL-input call; sampled outputs against Eq. (4) in
    FP64, and the tail empty afterwards."""
    import torch
    from oracle import oracle as O
    from tests.gpu_harness import binding
    T = binding()
    B, L, nb = 256, 1 << 22, 40
    nbd = -(-(L - 1) // B)
    s = T.Stream(B, L, max_blocks_per_call=nbd)
    assert s.info().tail_fp64 == 1
    x = W.signal_gauss(nb * B, 141)
    h = W.impulse_response(L, 142)
    s.set_ir(h)
    xd = torch.from_numpy(x).cuda()[None]
    yd = torch.empty_like(xd)
    yt = torch.empty((1, nbd * B), device="cuda")
    s.process_blocks(xd, yd, nb)
    s.process_blocks(None, yt, nbd)
    s.synchronize()
    assert s.info().live == 0
    y = torch.cat([yd, yt], 1).cpu().numpy()[0].astype(np.float64)
    n_out = nb * B + L - 1
    rng = np.random.default_rng(143)
    idx = set(rng.integers(0, n_out, 300).tolist()) | {0, nb * B - 1, nb * B, L - 1, L, n_out - 1}
    idx = np.array(sorted(idx))
    ref = O.sampled_outputs(x, [h], [(0, 0)], B, idx)
    rms = rms_y64(x, [h], [(0, 0)], B, n_out)
    assert np.max(np.abs(y[idx] - ref)) <= 1e-5 * rms
    assert not np.any(y[n_out:])
    s.close()


def test_config2_full_size_sampled_parity():
    """Full config-2 size in the benchmark's launch configuration (one
    1875-block call with the IR schedule, then a NULL-input drain), checked
    on sampled outputs against Eq. (4) in FP64 (numpy dot products)."""
    import torch
    from oracle import oracle as O
    from tests.gpu_harness import binding
    T = binding()
    spec = W.config2()
    B, L = spec.block, spec.max_ir_len
    nb, nbd = spec.n_blocks(), -(-(L - 1) // B)
    xp = np.zeros((1, nb * B), np.float32)
    xp[0, :spec.n_samples] = spec.x[0]
    s = T.Stream(B, L, max_blocks_per_call=nb, ir_slots=2)
    for k, h in enumerate(spec.irs):
        s.load_ir_slot(k, torch.from_numpy(h).cuda())
    sched = np.full(nb, -1, np.int32)
    for b, k in spec.schedule:
        sched[b] = k
    xd = torch.from_numpy(xp).cuda()
    yd = torch.empty_like(xd)
    yt = torch.empty((1, nbd * B), device="cuda")
    s.process_blocks(xd, yd, nb, sched)
    s.process_blocks(None, yt, nbd)
    y = torch.cat([yd, yt], 1).cpu().numpy()[0].astype(np.float64)
    rng = np.random.default_rng(7)
    idx = set(rng.integers(0, spec.n_samples + L - 1, 600).tolist())
    for b, _ in spec.schedule:          # both sides of every swap boundary
        idx.update([b * B - 1, b * B, b * B + 1])
    idx.update([0, 1, spec.n_samples - 1, spec.n_samples, spec.n_samples + L - 2])
    idx = np.array(sorted(i for i in idx if 0 <= i < spec.n_samples + L - 1))
    ref = O.sampled_outputs(spec.x[0], spec.irs, spec.schedule, B, idx)
    rms = rms_y64(spec.x[0], spec.irs, spec.schedule, B, spec.n_samples + L - 1)
    assert np.max(np.abs(y[idx] - ref)) <= 1e-5 * rms
    assert not np.any(y[spec.n_samples + L - 1:])
    s.close()


@pytest.mark.parametrize("B", (32, 64, 128))
@pytest.mark.parametrize("r", (4, 8, 12, 16))
def test_short_blocks_staged_together_bitwise(B, r):
    """One-wave tiles stage runs of up to 256/B short blocks that share an
    IR as one unit; swaps inside a call (including runs of a single block)
    split the runs.  Integer inputs: exact against the oracle.  Float
    inputs: one-wave tiles equal two-wave tiles (one chunk per wave, no
    grouping) and per-block calls bit for bit."""
    swaps = [3, 4, 11, 20, 21, 22, 40]
    sched = [(0, 0)] + [(b, (i + 1) % 2) for i, b in enumerate(swaps)]
    L1, L2 = 700, 1900
    n = 60 * B
    nb = -(-(n + L2) // B) + 1
    xi = W.signal_int(n, 71, 31)
    irs_i = [W.signal_int(L1, 72, 31), W.signal_int(L2, 73, 31)]
    ref = oracle_run(xi, irs_i, sched, B, L2, nb)
    yi, info = gpu_multi_block(xi, irs_i, sched, B, L2, nb, tile=(r, 1))
    assert (info.tile_r, info.tile_w) == (r, 1)
    assert np.array_equal(yi, ref)
    x = W.signal_gauss(n, 74)
    irs = [W.impulse_response(L1, 75), W.impulse_response(L2, 76)]
    y1, _ = gpu_multi_block(x, irs, sched, B, L2, nb, tile=(r, 1))
    y2, _ = gpu_multi_block(x, irs, sched, B, L2, nb, tile=(r, 2))
    yb, _ = gpu_per_block(x, irs, sched, B, L2, nb, tile=(r, 1))
    assert np.array_equal(y1, y2)
    assert np.array_equal(y1, yb)
    assert rel_err(y1, oracle_run(x, irs, sched, B, L2, nb)) <= TOL


def _silence(x, B, seed):
    """Zero about 40 % of the blocks, plus one run of several blocks."""
    x = x.copy()
    nb = -(-x.size // B)
    rng = np.random.default_rng(seed)
    for b in np.nonzero(rng.random(nb) < 0.4)[0]:
        x[b * B:(b + 1) * B] = 0
    x[3 * B:min(x.size, 9 * B + B // 2)] = 0
    return x


@pytest.mark.parametrize("B", (32, 64, 256, 300))
@pytest.mark.parametrize("tile", [(16, 1), (16, 4), (4, 1), (12, 2), (14, 4)])
def test_zero_blocks_are_bypassed_exactly(B, tile):
    """Chunks whose samples are all zero skip their multiply-adds and their
    addition to the tail (exact-zero bypass); outputs stay exact."""
    L1, L2 = 900, 2100
    n = 40 * B
    nb = -(-(n + L2) // B) + 1
    sched = [(0, 0), (7, 1), (20, 0), (21, 1)]
    xi = _silence(W.signal_int(n, 81, 31), B, 82)
    irs_i = [W.signal_int(L1, 83, 31), W.signal_int(L2, 84, 31)]
    ref = oracle_run(xi, irs_i, sched, B, L2, nb)
    yi, _ = gpu_multi_block(xi, irs_i, sched, B, L2, nb, tile=tile)
    assert np.array_equal(yi, ref)
    yb, _ = gpu_per_block(xi, irs_i, sched, B, L2, nb, tile=tile)
    assert np.array_equal(yb, ref)
    x = _silence(W.signal_gauss(n, 85), B, 86)
    irs = [W.impulse_response(L1, 87), W.impulse_response(L2, 88)]
    y, _ = gpu_multi_block(x, irs, sched, B, L2, nb, tile=tile)
    assert rel_err(y, oracle_run(x, irs, sched, B, L2, nb)) <= TOL
    y4, _ = gpu_multi_block(x, irs, sched, B, L2, nb, tile=(tile[0], 4))
    assert np.array_equal(y, y4)


def test_all_zero_input_gives_exact_zeros_and_keeps_the_tail():
    """A silent block after a sound one: the tail keeps ringing exactly as
    the oracle says, and an all-zero stream outputs exact zeros."""
    B, L = 64, 3000
    x = np.zeros(30 * B, np.float32)
    nb = -(-(x.size + L) // B)
    y, _ = gpu_multi_block(x, [W.impulse_response(L, 89)], [(0, 0)], B, L, nb)
    assert not np.any(y)
    x[5 * B + 7] = 1.0
    h = W.impulse_response(L, 90)
    y, _ = gpu_per_block(x, [h], [(0, 0)], B, L, nb)
    d = 5 * B + 7
    assert np.array_equal(y[0, d:d + L], h) and not np.any(y[0, :d]) and not np.any(y[0, d + L:])


SAMPLE_SWAP_CASES = [
    # B, L1, L2, swaps as (block, offset)
    (64, 500, 1300, [(3, 1), (5, 63), (6, 0), (9, 17)]),
    (300, 700, 1200, [(2, 150), (3, 299), (5, 1)]),      # two chunks per block, cut anywhere
    (513, 2000, 64, [(1, 256), (2, 257), (4, 5)]),       # three chunks per block
    (32, 100, 2500, [(4, 16), (5, 16), (7, 31)]),        # short blocks (grouped staging off)
]


@pytest.mark.parametrize("case", SAMPLE_SWAP_CASES, ids=[f"B{c[0]}" for c in SAMPLE_SWAP_CASES])
@pytest.mark.parametrize("tile", [None, (16, 1), (16, 4), (4, 2), (14, 4)])
def test_sample_accurate_swap_bitwise(case, tile):
    """An IR taking over at sample o of a block: integer inputs match the
    oracle exactly, per-block calls (taches_set_ir_at) and multi-block calls
    (taches_process_blocks_at) alike."""
    B, L1, L2, swaps = case
    sched = [(0, 0)] + [(b, (i + 1) % 2, o) for i, (b, o) in enumerate(swaps)]
    Lmax = max(L1, L2)
    n = 12 * B
    nb = -(-(n + Lmax) // B) + 1
    x = W.signal_int(n, 93, 31)
    irs = [W.signal_int(L1, 94, 31), W.signal_int(L2, 95, 31)]
    ref = oracle_run(x, irs, sched, B, Lmax, nb)
    y1, _ = gpu_per_block(x, irs, sched, B, Lmax, nb, tile=tile)
    assert np.array_equal(y1, ref)
    y2, _ = gpu_multi_block(x, irs, sched, B, Lmax, nb, tile=tile)
    assert np.array_equal(y2, ref)
    y3, _ = gpu_multi_block(x, irs, sched, B, Lmax, nb, tile=tile, calls=3)
    assert np.array_equal(y3, ref)


def test_sample_accurate_swap_float_modes_agree():
    """Float inputs: per-block and multi-block calls give the same bits and
    stay within the tolerance of the FP64 oracle; moving the swap by one
    sample changes the output."""
    B, L = 256, 6000
    x = W.signal_gauss(30 * B, 96)
    irs = [W.impulse_response(L, 97), W.impulse_response(L, 98)]
    sched = [(0, 0), (4, 1, 100), (9, 0, 255), (15, 1, 1)]
    nb = -(-(x.size + L) // B)
    ref = oracle_run(x, irs, sched, B, L, nb)
    y1, _ = gpu_per_block(x, irs, sched, B, L, nb)
    y2, _ = gpu_multi_block(x, irs, sched, B, L, nb)
    assert np.array_equal(y1, y2)
    assert rel_err(y1, ref) <= TOL
    moved = [(0, 0), (4, 1, 101), (9, 0, 255), (15, 1, 1)]
    assert rel_err(y1, oracle_run(x, irs, moved, B, L, nb)) > 1e-3


def test_sample_accurate_swap_errors():
    from tests.gpu_harness import binding
    T = binding()
    s = T.Stream(64, 128)
    h = W.impulse_response(100, 99)
    with pytest.raises(T.TachesError):
        s.set_ir(h, 64)
    with pytest.raises(T.TachesError):
        s.set_ir(h, -1)
    s.set_ir(h, 5)                      # no IR before sample 5 of the first block
    with pytest.raises(T.TachesError) as e:
        s.process(np.ones(64, np.float32))
    assert e.value.status == T.TACHES_ENOIR
    s.set_ir(h)
    s.process(np.ones(64, np.float32))
    s.close()
    sp = T.Stream(64, 128, precision=1)
    with pytest.raises(T.TachesError):
        sp.set_ir(h, 3)
    sp.close()


@pytest.mark.parametrize("tail", ["fp32", "fp64"])
def test_reset_stream_equals_fresh_stream(tail):
    """A stream reset after use (no device clear: the tail counts as empty)
    gives the same bits as a freshly opened one on a new input and IR, and
    its tail reads back as zeros right after the reset."""
    import torch
    from tests.gpu_harness import binding
    T = binding()
    tail = T.TACHES_TAIL_FP32 if tail == "fp32" else T.TACHES_TAIL_FP64
    B, L, C, nb = 64, 3000, 2, 40
    x1 = np.stack([W.signal_gauss(nb * B, 900 + c) for c in range(C)])
    x2 = np.stack([W.signal_gauss(nb * B, 910 + c) for c in range(C)])
    h1, h2 = W.impulse_response(L, 920), W.impulse_response(L - 700, 921)

    def run(s, x, h):
        s.set_ir(h)
        y = torch.empty((C, nb * B), device="cuda")
        s.process_blocks(torch.from_numpy(x).cuda(), y, nb)
        s.synchronize()
        return y.cpu().numpy()
    used = T.Stream(B, L, channels=C, max_blocks_per_call=nb, tail=tail)
    run(used, x1, h1)
    assert np.any(used.read_tail(0, L) != 0)
    used.reset()
    assert not np.any(used.read_tail(0, L))
    assert not np.any(used.read_tail(C - 1, L))
    fresh = T.Stream(B, L, channels=C, max_blocks_per_call=nb, tail=tail)
    assert np.array_equal(run(used, x2, h2), run(fresh, x2, h2))
    for c in range(C):
        assert np.array_equal(used.read_tail(c, L), fresh.read_tail(c, L))
    used.close()
    fresh.close()


def test_ir_read_in_place_equals_copied_ir():
    """taches_set_ir_ref (the stream reads the caller's device IR without a
    copy) gives the same bits as taches_set_ir / taches_set_ir_at, for swaps
    at block starts and inside blocks, block by block and through a pool;
    refused on a split-BF16 stream."""
    import torch
    from tests.gpu_harness import binding
    T = binding()
    B, L, C, nb = 128, 2500, 2, 30
    x = np.stack([W.signal_gauss(nb * B, 930 + c) for c in range(C)])
    hs = [torch.from_numpy(W.impulse_response(L - 300 * v, 940 + v)).cuda() for v in range(3)]
    swaps = {0: (0, 0), 7: (1, 0), 12: (2, 37), 20: (0, 101)}   # block -> (IR, offset)

    def run(ref, pool=None):
        s = T.Stream(B, L, channels=C)
        if pool is not None:
            assert pool.attach(s) == T.TACHES_OK
        ys = []
        for k in range(nb):
            if k in swaps:
                v, off = swaps[k]
                if ref:
                    assert T.taches_set_ir_ref(s.h, hs[v], off) == T.TACHES_OK
                else:
                    s.set_ir(hs[v], offset=off)
            xb = torch.from_numpy(np.ascontiguousarray(x[:, k * B:(k + 1) * B])).cuda()
            y = torch.empty((C, B), device="cuda")
            if pool is None:
                s.process_async(xb, y)
            else:
                pool.step([s], [xb], [y], [1])
            ys.append(y)
        torch.cuda.synchronize()
        out = torch.cat(ys, dim=1).cpu().numpy()
        if pool is not None:
            pool.detach(s)
        s.close()
        return out
    base = run(False)
    assert np.array_equal(run(True), base)
    pool = T.Pool(4, 1 << 30, use_graph=True)
    assert np.array_equal(run(True, pool), base)
    pool.close()
    sp = T.Stream(B, L, channels=C, precision=T.TACHES_PREC_SPLIT_BF16)
    assert T.taches_set_ir_ref(sp.h, hs[0], 0) == T.TACHES_EINVAL
    sp.close()
