"""Parity of the split-BF16 Toeplitz MFMA path (channels sharing one IR)
with the FP64 oracle.

Bound (per output n): |y - y64| <= (3 * 2^-16 + gamma_K) * sum_k |h_k| |x_{n-k}|
with gamma_K = K u / (1 - K u), u = 2^-24, K = 3 * 256 (the products of one
chunk accumulated in FP32): 2^-16 covers each value's hi+lo representation
and the dropped lo*lo product.  Statistical targets over a run:
max |err| <= 1e-4 * RMS(y64) and RMS(err) <= 1e-5 * RMS(y64)."""
import numpy as np
import pytest

from paper_2401_01607_amd import workloads as W
from tests.gpu_harness import gpu_multi_block, oracle_run, rel_err

pytestmark = pytest.mark.gpu

SPLIT = 1
U = 2.0**-24
GAMMA = (3 * 256 * U) / (1 - 3 * 256 * U)
BOUND_COEF = 3 * 2.0**-16 + GAMMA


def split_run(x, irs, sched, B, Lmax, nb, calls=1, tail=0, drain=0):
    return gpu_multi_block(x, irs, sched, B, Lmax, nb, calls=calls, tail=tail, drain_x_null=drain,
                           precision=SPLIT)


def per_block_split(x, irs, sched, B, Lmax, nb):
    from tests.gpu_harness import gpu_per_block
    return gpu_per_block(x, irs, sched, B, Lmax, nb, precision=SPLIT)


def check_bound(y, x, irs, sched, B, Lmax, nb):
    from tests.gpu_harness import oracle_abs_run
    ref = oracle_run(x, irs, sched, B, Lmax, nb)
    mag = oracle_abs_run(x, irs, sched, B, Lmax, nb)
    err = np.abs(np.asarray(y, np.float64) - ref)
    assert np.all(err <= BOUND_COEF * mag + 1e-30)
    rms = np.sqrt(np.mean(ref**2))
    assert err.max() <= 1e-4 * rms
    assert np.sqrt(np.mean(err**2)) <= 1e-5 * rms
    return ref, err.max() / rms


@pytest.mark.parametrize("C,B,L1,L2,n,swaps", [
    (1, 64, 100, 100, 700, []),
    (3, 5, 40, 17, 200, [7, 20]),
    (33, 512, 1000, 300, 3000, [2]),
    (64, 256, 700, 700, 2000, [3, 5]),
])
def test_integer_inputs_bitwise(C, B, L1, L2, n, swaps):
    amp = 20
    x = np.stack([W.signal_int(n, 10 + c, amp) for c in range(C)])
    irs = [W.signal_int(L1, 5, amp), W.signal_int(L2, 6, amp)]
    sched = [(0, 0)] + [(b, (i + 1) % 2) for i, b in enumerate(swaps)]
    Lmax = max(L1, L2)
    nb = -(-(n + Lmax) // B) + 1
    ref = oracle_run(x, irs, sched, B, Lmax, nb)
    y, info = split_run(x, irs, sched, B, Lmax, nb)
    assert info.precision == SPLIT
    assert np.array_equal(y, ref)
    yb, _ = per_block_split(x, irs, sched, B, Lmax, nb)
    assert np.array_equal(yb, ref)


def test_impulse_is_hi_plus_lo():
    L, B = 2000, 512
    h = W.impulse_response(L, 3)
    x = np.zeros((2, 700), np.float32)
    x[0, 0] = 1.0
    x[1, 600] = 1.0
    nb = -(-(700 + L) // B) + 1
    y, _ = split_run(x, [h], [(0, 0)], B, L, nb)
    for c, d in ((0, 0), (1, 600)):
        got = y[c, d:d + L].astype(np.float64)
        assert np.all(np.abs(got - h) <= 2.0**-16 * np.abs(h) + 1e-45)
        assert not np.any(y[c, :d]) and not np.any(y[c, d + L:])


@pytest.mark.parametrize("C", [1, 5, 32, 33, 64])
def test_gaussian_within_split_bound(C):
    B, L, n = 512, 4096, 6000
    x = np.stack([W.signal_gauss(n, 200 + c) for c in range(C)])
    h = W.impulse_response(L, 201)
    nb = -(-(n + L - 1) // B)
    y, _ = split_run(x, [h], [(0, 0)], B, L, nb)
    check_bound(y, x, [h], [(0, 0)], B, L, nb)


def test_modes_agree_bitwise_and_swaps():
    C, B, L, n = 8, 256, 3000, 8000
    x = np.stack([W.signal_gauss(n, 300 + c) for c in range(C)])
    ha, hb = W.impulse_response(L, 301), W.impulse_response(L, 302)
    sched = [(0, 0), (5, 1), (11, 0), (20, 1)]
    nb = -(-(n + L - 1) // B)
    y1, _ = split_run(x, [ha, hb], sched, B, L, nb)
    y2, _ = split_run(x, [ha, hb], sched, B, L, nb, calls=5)
    y3, _ = per_block_split(x, [ha, hb], sched, B, L, nb)
    assert np.array_equal(y1, y2) and np.array_equal(y1, y3)
    check_bound(y1, x, [ha, hb], sched, B, L, nb)


def test_fp32_tail_split_stream():
    C, B, L, n = 4, 128, 2000, 4000
    x = np.stack([W.signal_gauss(n, 400 + c) for c in range(C)])
    h = W.impulse_response(L, 401)
    nb = -(-(n + L - 1) // B)
    y, info = split_run(x, [h], [(0, 0)], B, L, nb, tail=1)
    assert info.tail_fp64 == 0
    check_bound(y, x, [h], [(0, 0)], B, L, nb)


def test_tail_state_split_layout():
    """read_tail on the [slot][channel] layout returns the oracle residue."""
    from oracle import oracle as O
    from tests.gpu_harness import binding
    T = binding()
    C, B, L = 3, 32, 300
    x = np.stack([W.signal_int(4 * B, 50 + c, 20) for c in range(C)])
    h = W.signal_int(L, 60, 20)
    o = O.OracleStream(B, L, C)
    o.set_ir(h)
    s = T.Stream(B, L, channels=C, precision=SPLIT)
    s.set_ir(h)
    for b in range(4):
        xb = x[:, b * B:(b + 1) * B]
        o.process(xb)
        s.process(xb)
    for c in range(C):
        assert np.array_equal(s.read_tail(c, L), o.residue(c))
