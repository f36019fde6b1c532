"""Pins for the CPU oracle, checked against what the paper and mathematics fix.

Every pin is written as a function of an implementation
``impl(x, irs, schedule, B, Lmax, n_out) -> float64[n_out]`` so that the same
pins run on the buffer-form oracle in its three precisions (O1 FP64, O2 FP32
with one rounding per multiply-accumulate, O2m FP32 with the product and the
sum rounded separately; C), on the tache-sum oracle (O3) and on deliberately
broken variants of a shift-register formulation (Section 4.1), which must
each fail at least one pin.
"""
import os

import numpy as np
import pytest

from oracle import oracle as O
from paper_2401_01607_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------------------
# implementations under test
# ---------------------------------------------------------------------------

def impl_o1(x, irs, schedule, B, Lmax, n_out, prec=O.OR_FP64):
    nb = -(-n_out // B)
    return O.run_channel(x, irs, schedule, B, Lmax, n_blocks=nb, prec=prec)[:n_out]


def impl_o2(x, irs, schedule, B, Lmax, n_out):
    return impl_o1(x, irs, schedule, B, Lmax, n_out, prec=O.OR_FP32_FMA)


def impl_o2m(x, irs, schedule, B, Lmax, n_out):
    return impl_o1(x, irs, schedule, B, Lmax, n_out, prec=O.OR_FP32_MULADD)


def _active_of_sample(schedule, B, n, ignore_offsets=False):
    """IR index of each input sample 0 .. n-1 (None before the first IR): a
    schedule entry (block, ir[, offset]) applies from sample block*B + offset
    on; a later entry overrides."""
    act = [None] * n
    for e in sorted(schedule, key=lambda e: e[0] * B + (0 if ignore_offsets or len(e) < 3 else e[2])):
        start = e[0] * B + (0 if ignore_offsets or len(e) < 3 else e[2])
        for m in range(max(start, 0), n):
            act[m] = e[1]
    return act


def impl_o3(x, irs, schedule, B, Lmax, n_out):
    xx = np.zeros(n_out, dtype=np.float32)
    xx[: min(len(x), n_out)] = np.asarray(x, np.float32)[:n_out]
    act = _active_of_sample(schedule, B, n_out)
    zero = np.zeros(1, np.float32)

    def h_of(n):
        k = act[n]
        return zero if k is None else irs[k]
    return O.tache_sum(xx, h_of)[:n_out]


# Broken variants of a shift-register formulation (a residue that receives
# e(n) * h, emits its first element and shifts left, Section 4.1): each is a
# plausible coding mistake.
def _vector_mutant(kind):
    def impl(x, irs, schedule, B, Lmax, n_out):
        xx = np.zeros(n_out, dtype=np.float32)
        xx[: min(len(x), n_out)] = np.asarray(x, np.float32)[:n_out]
        act = _active_of_sample(schedule, B, n_out, ignore_offsets=(kind == "offset_ignored"))
        if kind == "swap_late":          # IR taken from the previous block
            act = [act[max(m - B, 0)] for m in range(n_out)]
        if kind == "swap_early":         # IR taken from the next block
            act = [act[min(m + B, n_out - 1)] for m in range(n_out)]
        if kind == "offset_late":        # a swap takes over one sample late
            act = [act[max(m - 1, 0)] for m in range(n_out)]
        Nh = max(len(h) for h in irs)
        r = np.zeros(Nh + 1, np.float64)
        s = []
        for n in range(n_out):
            k = act[n]
            h = np.zeros(1) if k is None else np.asarray(irs[k], np.float64)
            if kind == "drop_last_tap":
                h = h[:-1]
            if kind == "sign":
                r[: h.size] -= np.float64(xx[n]) * h
            elif kind == "rotated":      # literal index of the printed listing
                hr = np.roll(h, 1)
                r[: hr.size] += np.float64(xx[n]) * hr
            elif kind == "reversed_ir":  # operand read backwards
                r[: h.size] += np.float64(xx[n]) * h[::-1]
            else:
                r[: h.size] += np.float64(xx[n]) * h
            if kind == "emit_after_shift":
                r = np.concatenate([r[1:], [0.0]])
                s.append(r[0])
            elif kind == "shift_right":
                s.append(r[0])
                r = np.concatenate([[0.0], r[:-1]])
            else:
                s.append(r[0])
                r = np.concatenate([r[1:], [0.0]])
        return np.array(s)
    return impl


MUTANTS = ["swap_late", "swap_early", "drop_last_tap", "sign", "rotated", "reversed_ir",
           "emit_after_shift", "shift_right", "offset_late", "offset_ignored"]


# ---------------------------------------------------------------------------
# pins: each returns True when the implementation satisfies it
# ---------------------------------------------------------------------------

def _read_golden(name):
    out = {}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            k, v = line.split(":", 1)
            out[k.strip()] = v.split()
    return out


def pin_golden_fig5(impl):
    """Hand-derived worked example of the Fig. 4-6 shape, every block size."""
    g = _read_golden("fig5_taches_6x3.txt")
    x = np.array(g["x"], np.float32)
    h = np.array(g["h"], np.float32)
    y = np.array(g["y"], np.float64)
    return all(np.array_equal(impl(x, [h], [(0, 0)], B, 3, 8), y) for B in (1, 2, 3, 4, 6, 8))


def pin_golden_swap(impl):
    """Hand-derived IR swap at the next block."""
    g = _read_golden("ir_swap_next_block.txt")
    B = int(g["block"][0])
    x = np.array(g["x"], np.float32)
    hA = np.array(g["h_A"], np.float32)
    hB = np.array(g["h_B"], np.float32)
    y = np.array(g["y"], np.float64)
    return np.array_equal(impl(x, [hA, hB], [(0, 0), (1, 1)], B, 2, len(y)), y)


def _int_case(seed, n, L1, L2, B, swaps):
    x = W.signal_int(n, seed)
    h1 = W.signal_int(L1, seed + 1)
    h2 = W.signal_int(L2, seed + 2)
    sched = [(0, 0)] + [(b, (i + 1) % 2) for i, b in enumerate(swaps)]
    return x, [h1, h2], sched


def pin_brute_force(impl):
    """Exact equality with Eq. (4) summed with Python integers, with swaps,
    B > L, L = 1, B = 1 and IRs of different lengths."""
    cases = [(11, 37, 5, 9, 4, [3, 5]), (12, 20, 1, 1, 1, [7]), (13, 25, 3, 3, 8, [1]),
             (14, 30, 7, 2, 3, [2, 4, 6]), (15, 16, 16, 4, 5, [])]
    for seed, n, L1, L2, B, swaps in cases:
        x, irs, sched = _int_case(seed, n, L1, L2, B, swaps)
        Lmax = max(L1, L2)
        n_out = n + Lmax + B
        ref = np.array([float(v) for v in O.brute_force(x, irs, sched, B, n_out)])
        if not np.array_equal(impl(x, irs, sched, B, Lmax, n_out), ref):
            return False
    return True


def pin_impulse(impl):
    """An impulse at d returns h exactly at d .. d+L-1 and zero elsewhere."""
    L, B = 13, 5
    h = W.impulse_response(L, 7)
    for d in (0, B - 1, B, 3 * B + 3):
        x = np.zeros(d + 1, np.float32)
        x[d] = 1.0
        n_out = d + L + 2 * B
        y = impl(x, [h], [(0, 0)], B, L, n_out)
        want = np.zeros(n_out)
        want[d:d + L] = h.astype(np.float64)
        if not np.array_equal(y, want):
            return False
    return True


def pin_overflow(impl):
    """Output is Ne + L - 1 long: exactly zero after that (Section 4.1), and
    the overflow samples equal numpy.convolve's tail."""
    x = W.signal_int(23, 3)
    h = W.signal_int(6, 4)
    n_out = 23 + 6 - 1 + 9
    y = impl(x, [h], [(0, 0)], 4, 6, n_out)
    full = np.convolve(x.astype(np.float64), h.astype(np.float64))
    return np.array_equal(y[:28], full) and not np.any(y[28:])


def pin_swap_decomposition(impl):
    """y = conv(x*1[m<s], h_old) + conv(x*1[m>=s], h_new) for a swap before
    block s/B, exactly (integers); moving the swap by one block changes y."""
    B, n = 4, 24
    x = W.signal_int(n, 21)
    ha, hb = W.signal_int(5, 22), W.signal_int(5, 23)
    s_blk = 3
    s = s_blk * B
    n_out = n + 5 - 1
    y = impl(x, [ha, hb], [(0, 0), (s_blk, 1)], B, 5, n_out)
    x1 = x.astype(np.float64).copy()
    x1[s:] = 0
    x2 = x.astype(np.float64) - x1
    want = np.convolve(x1, ha.astype(np.float64)) + np.convolve(x2, hb.astype(np.float64))
    if not np.array_equal(y, want):
        return False
    for other in (s_blk - 1, s_blk + 1):
        if np.array_equal(impl(x, [ha, hb], [(0, 0), (other, 1)], B, 5, n_out), want):
            return False
    return True


def pin_linearity_shift(impl):
    """Linearity and time-shift invariance (LTI, Section 3.2), exact with
    integers: y(a*x1 + b*x2) = a*y(x1) + b*y(x2); y(x delayed by d) = y
    delayed by d for any d without swaps."""
    B, L, n = 3, 7, 20
    h = W.signal_int(L, 31)
    x1, x2 = W.signal_int(n, 32, amp=10), W.signal_int(n, 33, amp=10)
    n_out = n + L + 8
    y1 = impl(x1, [h], [(0, 0)], B, L, n_out)
    y2 = impl(x2, [h], [(0, 0)], B, L, n_out)
    y12 = impl((3 * x1 - 2 * x2).astype(np.float32), [h], [(0, 0)], B, L, n_out)
    if not np.array_equal(y12, 3 * y1 - 2 * y2):
        return False
    for d in (1, 2, 5):
        xd = np.concatenate([np.zeros(d, np.float32), x1])
        yd = impl(xd, [h], [(0, 0)], B, L, n_out)
        if not (np.array_equal(yd[d:], y1[: n_out - d]) and not np.any(yd[:d])):
            return False
    return True


def pin_commutativity(impl):
    """Exchanging the roles of input and IR gives the same output (Section
    3.2, Fig. 6), exactly with integers."""
    x = W.signal_int(6, 41)
    h = W.signal_int(3, 42)
    a = impl(x, [h], [(0, 0)], 2, 3, 8)
    b = impl(h, [x], [(0, 0)], 2, 6, 8)
    return np.array_equal(a, b)


def pin_sample_swap_decomposition(impl):
    """Sample-accurate swap (Section 6: the IR may change even sample by
    sample): an IR set to take over at sample o of block b gives
    y = conv(x*1[m<p], h_old) + conv(x*1[m>=p], h_new), p = b*B + o, exactly;
    moving the swap by one sample changes y."""
    B, n = 5, 30
    x = W.signal_int(n, 24)
    ha, hb = W.signal_int(6, 25), W.signal_int(4, 26)
    n_out = n + 6 - 1

    def conv(v, h):
        out = np.zeros(n_out)
        c = np.convolve(v, h.astype(np.float64))
        out[: c.size] = c
        return out
    for blk, o in ((2, 0), (2, 1), (2, 3), (3, B - 1), (1, 2)):
        p = blk * B + o
        x1 = x.astype(np.float64).copy()
        x1[p:] = 0
        x2 = x.astype(np.float64) - x1
        want = conv(x1, ha) + conv(x2, hb)
        if not np.array_equal(impl(x, [ha, hb], [(0, 0), (blk, 1, o)], B, 6, n_out), want):
            return False
        for q in (p - 1, p + 1):
            if np.array_equal(impl(x, [ha, hb], [(0, 0), (q // B, 1, q % B)], B, 6, n_out), want):
                return False
    return True


def pin_brute_force_sample_swaps(impl):
    """Exact equality with Eq. (4) (integers) under schedules whose swaps
    take over inside blocks, including several swaps and unequal lengths."""
    cases = [(17, 40, 6, 3, 4, [(2, 1), (5, 3), (7, 0)]), (18, 33, 2, 5, 7, [(1, 6), (3, 2)]),
             (19, 21, 4, 4, 1, [(3, 0), (9, 0)]), (20, 26, 9, 1, 5, [(1, 4), (2, 4), (4, 1)])]
    for seed, n, L1, L2, B, swaps in cases:
        x = W.signal_int(n, seed)
        irs = [W.signal_int(L1, seed + 1), W.signal_int(L2, seed + 2)]
        sched = [(0, 0)] + [(b, (i + 1) % 2, o) for i, (b, o) in enumerate(swaps)]
        Lmax = max(L1, L2)
        n_out = n + Lmax + B
        ref = np.array([float(v) for v in O.brute_force(x, irs, sched, B, n_out)])
        if not np.array_equal(impl(x, irs, sched, B, Lmax, n_out), ref):
            return False
    return True


PINS = [pin_golden_fig5, pin_golden_swap, pin_brute_force, pin_impulse, pin_overflow,
        pin_swap_decomposition, pin_linearity_shift, pin_commutativity, pin_sample_swap_decomposition,
        pin_brute_force_sample_swaps]


@pytest.mark.parametrize("pin", PINS, ids=lambda p: p.__name__)
@pytest.mark.parametrize("impl", [impl_o1, impl_o2, impl_o2m, impl_o3],
                         ids=["O1_fp64", "O2_fp32_fma", "O2m_fp32_muladd", "O3_tache_sum"])
def test_pin_holds(impl, pin):
    assert pin(impl)


@pytest.mark.parametrize("kind", MUTANTS)
def test_mutant_is_caught(kind):
    impl = _vector_mutant(kind)
    failed = [p.__name__ for p in PINS if not p(impl)]
    assert failed, f"no pin catches mutant {kind}"


def test_unmutated_variant_passes():
    impl = _vector_mutant("none")
    assert all(p(impl) for p in PINS)


# ---------------------------------------------------------------------------
# further pins on float inputs
# ---------------------------------------------------------------------------

def test_o1_matches_numpy_convolve():
    """Without swaps the method is the direct convolution (Eq. 1), the
    library routine numpy.convolve, up to FP64 rounding order."""
    x = W.signal_uniform(3000, 5)
    h = W.impulse_response(257, 6)
    y = impl_o1(x, [h], [(0, 0)], 64, 257, 3000 + 256)
    ref = np.convolve(x.astype(np.float64), h.astype(np.float64))
    mag = O.abs_bound_weights(x, [h], [(0, 0)], 64, 257)[: ref.size]
    assert np.all(np.abs(y - ref) <= 2 * 257 * 2.0**-53 * mag + 1e-300)


def test_tache_sum_bitwise_equals_buffer_form():
    """The residue of the buffer form (Section 4.2) and the whole-array sum
    of taches (Section 3.2) add each output's products in input order, so in
    FP64 they agree bit for bit."""
    x = W.signal_gauss(500, 8)
    ha, hb = W.impulse_response(40, 9), W.impulse_response(25, 10)
    sched = [(0, 0), (7, 1), (20, 0)]
    a = impl_o1(x, [ha, hb], sched, 16, 40, 560)
    b = impl_o3(x, [ha, hb], sched, 16, 40, 560)
    assert np.array_equal(a, b)


def test_block_size_invariance_bitwise():
    """Without swaps the block size changes only timing, not the output
    (Section 5.2, Table 2): each slot receives its taches in input order
    whatever B is, so FP64 results are bit-identical."""
    x = W.signal_gauss(2000, 11)
    h = W.impulse_response(300, 12)
    ys = [impl_o1(x, [h], [(0, 0)], B, 300, 2400) for B in (1, 7, 64, 256, 2400)]
    for y in ys[1:]:
        assert np.array_equal(y, ys[0])


def test_zero_block_generates_no_tache():
    """A zero input adds nothing (Section 3.2): after a zero block the
    residue equals the previous residue advanced by B, bit for bit."""
    B, L = 8, 50
    s = O.OracleStream(B, L, 1)
    s.set_ir(W.impulse_response(L, 13))
    s.process(W.signal_gauss(B, 14))
    before = s.residue()
    rc, y = s.process(np.zeros(B, np.float32))
    after = s.residue()
    assert rc == 0
    assert np.array_equal(y[0], before[:B])
    assert np.array_equal(after[: L - B], before[B:])
    assert not np.any(after[L - B:])


def test_process_before_ir_is_enoir():
    s = O.OracleStream(4, 8, 1)
    rc, _ = s.process(np.ones(4, np.float32))
    assert rc == O.OR_ENOIR
    assert s.set_ir(np.ones(9, np.float32)) == O.OR_EINVAL
    assert s.set_ir(np.ones(8, np.float32)) == 0


def test_last_set_ir_wins():
    B = 4
    x = W.signal_int(12, 51)
    h1, h2 = W.signal_int(3, 52), W.signal_int(3, 53)
    s = O.OracleStream(B, 3, 1)
    s.set_ir(h1)
    s.set_ir(h2)
    ys = [s.process(x[i:i + B])[1][0] for i in range(0, 12, B)]
    y = np.concatenate(ys)
    assert np.array_equal(y, np.convolve(x.astype(np.float64), h2.astype(np.float64))[:12])


def test_multichannel_equals_single_channels():
    B, L, C = 16, 33, 3
    h = W.impulse_response(L, 61)
    xs = [W.signal_gauss(64, 62 + c) for c in range(C)]
    s = O.OracleStream(B, L, C)
    s.set_ir(h)
    ys = []
    for b in range(4):
        ys.append(s.process(np.stack([xc[b * B:(b + 1) * B] for xc in xs]))[1])
    y = np.concatenate(ys, axis=1)
    for c in range(C):
        assert np.array_equal(y[c], impl_o1(xs[c], [h], [(0, 0)], B, L, 64))


def test_printed_listing_literal_index_rotates_ir():
    """Reading of the buffer listing's index (Section 4.2): taken literally,
    h(1) lands one slot after the emitted one and an impulse returns the IR
    rotated by one, [h(Nh), h(1), ...].  The oracle's corrected index returns h."""
    h = np.array([1.0, 2.0, 3.0, 4.0])
    Nh = 4
    r = [0.0] * (Nh + 1)            # 1-based residue
    r_index = 1
    out = []
    for e0 in [1.0, 0.0, 0.0, 0.0]:
        for i in range(r_index + 1, Nh + 1):
            r[i] += e0 * h[i - r_index - 1]
        for i in range(1, r_index + 1):
            r[i] += e0 * h[Nh - r_index + i - 1]
        out.append(r[r_index])
        r[r_index] = 0.0
        r_index = r_index + 1 if r_index < Nh else 1
    assert out == [4.0, 1.0, 2.0, 3.0]
    y = impl_o1(np.array([1, 0, 0, 0], np.float32), [h.astype(np.float32)], [(0, 0)], 1, 4, 4)
    assert y.tolist() == [1.0, 2.0, 3.0, 4.0]


def test_fp32_oracle_within_rounding_bound():
    """O2 rounds once per multiply-accumulate (Section 5.5's per-MAC
    requantization).  A chain of k fused MACs is within gamma_k * sum|x h|
    of the exact sum (gamma_k = k u / (1 - k u), u = 2^-24); O1 is exact up
    to 2^-53 relative, far below."""
    x = W.signal_gauss(4000, 71)
    h = W.impulse_response(2048, 72)
    n_out = 4000 + 2047
    y64 = impl_o1(x, [h], [(0, 0)], 128, 2048, n_out)
    y32 = impl_o2(x, [h], [(0, 0)], 128, 2048, n_out)
    mag = O.abs_bound_weights(x, [h], [(0, 0)], 128, 2048)[:n_out]
    u = 2.0**-24
    gam = 2048 * u / (1 - 2048 * u)
    assert np.all(np.abs(y32 - y64) <= gam * mag * (1 + 1e-9) + 1e-30)
    assert np.any(y32 != y64)  # it really is a different precision


def test_fp32_separate_roundings_within_bound():
    """O2m rounds every product to FP32 and then every sum (two roundings per
    multiply-accumulate, the form of Section 5.3's requantization count with
    the product requantized before the accumulation).  An output that sums k
    products is within gamma_k * sum|x h| of the exact sum (the product of
    the first term and the k - 1 additions that follow it are k roundings;
    gamma_k = k u / (1 - k u), u = 2^-24).  It differs from the fused form."""
    x = W.signal_gauss(4000, 73)
    h = W.impulse_response(2048, 74)
    n_out = 4000 + 2047
    y64 = impl_o1(x, [h], [(0, 0)], 128, 2048, n_out)
    y32m = impl_o2m(x, [h], [(0, 0)], 128, 2048, n_out)
    y32f = impl_o2(x, [h], [(0, 0)], 128, 2048, n_out)
    mag = O.abs_bound_weights(x, [h], [(0, 0)], 128, 2048)[:n_out]
    u = 2.0**-24
    gam = 2048 * u / (1 - 2048 * u)
    assert np.all(np.abs(y32m - y64) <= gam * mag * (1 + 1e-9) + 1e-30)
    assert np.any(y32m != y64)
    assert np.any(y32m != y32f)


def test_precision_modes_on_a_hand_derived_rounding_case():
    """Two samples, two taps: output 1 = x0*h1 + x1*h0 with x0*h1 =
    -(1 + 2^-11) (exact) and x1*h0 = (1 + 2^-12)^2 = 1 + 2^-11 + 2^-24.  The
    exact sum is 2^-24.  FP64 holds every step exactly; one fused rounding
    of -(1 + 2^-11) + (1 + 2^-11 + 2^-24) is exact too; but the product
    rounded to FP32 first is a tie between 1 + 2^-11 and 1 + 2^-11 + 2^-23,
    which rounds to the even 1 + 2^-11, and the sum is then 0.  Output 0 =
    x0*h0 = -(1 + 2^-11)(1 + 2^-12) = -(1 + 2^-12 + 2^-11 + 2^-23) fits in 24
    bits: exact in every mode."""
    a = 1.0 + 2.0**-12
    x = np.array([-(1.0 + 2.0**-11), a], np.float32)
    h = np.array([a, 1.0], np.float32)
    y0 = -(1.0 + 2.0**-12 + 2.0**-11 + 2.0**-23)
    want = {O.OR_FP64: [y0, 2.0**-24, 1.0 + 2.0**-12],
            O.OR_FP32_FMA: [y0, 2.0**-24, 1.0 + 2.0**-12],
            O.OR_FP32_MULADD: [y0, 0.0, 1.0 + 2.0**-12]}
    for prec, w in want.items():
        y = impl_o1(x, [h], [(0, 0)], 1, 2, 3, prec=prec)
        assert y.tolist() == w, (prec, y.tolist())


def test_sampled_outputs_match_full_oracle():
    spec = W.config2(n=6000, L=3000, block=256, period=1000)
    y = impl_o1(spec.x[0], spec.irs, spec.schedule, 256, 3000, 6000 + 2999)
    idx = np.array([0, 1, 255, 256, 999, 1000, 1024, 2999, 3000, 5999, 6000, 8998])
    s = O.sampled_outputs(spec.x[0], spec.irs, spec.schedule, 256, idx)
    mag = O.abs_bound_weights(spec.x[0], spec.irs, spec.schedule, 256, 3000)
    assert np.all(np.abs(s - y[idx]) <= 1e-12 * mag[idx] + 1e-300)


def test_sampled_and_fft_outputs_on_integer_swap_cases():
    """The two whole-signal helpers used for full-size checks against Eq. (4)
    summed in Python integers: sampled_outputs (FP64 dot products per IR
    run) is exact on integers; fft_outputs (FP64 FFT per IR run) rounds to
    the exact integers, with a swap inside a block too."""
    cases = [(11, 37, 5, 9, 4, [(3, 0), (5, 0)]), (17, 40, 6, 3, 4, [(2, 1), (5, 3), (7, 0)]),
             (15, 16, 16, 4, 5, [])]
    for seed, n, L1, L2, B, swaps in cases:
        x = W.signal_int(n, seed)
        irs = [W.signal_int(L1, seed + 1), W.signal_int(L2, seed + 2)]
        sched = [(0, 0)] + [(b, (i + 1) % 2, o) for i, (b, o) in enumerate(swaps)]
        n_out = n + max(L1, L2) + B
        ref = np.array([float(v) for v in O.brute_force(x, irs, sched, B, n_out)])
        idx = np.arange(n_out)
        assert np.array_equal(O.sampled_outputs(x, irs, sched, B, idx), ref)
        f = O.fft_outputs(x, irs, sched, B, n_out)
        assert np.array_equal(np.rint(f), ref)
        assert np.max(np.abs(f - ref)) < 1e-9


def test_fft_outputs_match_buffer_oracle_on_floats():
    """fft_outputs agrees with O1 to FP64 rounding (1e-12 of the output RMS)
    on a stream with swaps, and with numpy.convolve without swaps."""
    spec = W.config2(n=6000, L=3000, block=256, period=1000)
    n_out = 6000 + 2999
    y = impl_o1(spec.x[0], spec.irs, spec.schedule, 256, 3000, n_out)
    f = O.fft_outputs(spec.x[0], spec.irs, spec.schedule, 256, n_out)
    rms = np.sqrt(np.mean(y ** 2))
    assert np.max(np.abs(f - y)) <= 1e-12 * rms
    x = W.signal_gauss(5000, 91)
    h = W.impulse_response(777, 92)
    c = np.convolve(x.astype(np.float64), h.astype(np.float64))
    assert np.max(np.abs(O.fft_outputs(x, [h], [(0, 0)], 64, c.size) - c)) <= 1e-12 * np.sqrt(np.mean(c ** 2))


def test_sample_swap_per_block_calls_equal_schedule_run():
    """set_ir(h, offset) between two blocks equals the scheduled whole-signal
    run bit for bit; a swap at offset 0 equals the block swap."""
    B, L = 16, 40
    x = W.signal_gauss(10 * B, 27)
    ha, hb = W.impulse_response(L, 28), W.impulse_response(30, 29)
    sched = [(0, 0), (3, 1, 5), (6, 0, 15), (8, 1, 0)]
    ref = impl_o1(x, [ha, hb], sched, B, L, 10 * B)
    s = O.OracleStream(B, L, 1)
    ys = []
    for b in range(10):
        for e in sched:
            if e[0] == b:
                s.set_ir([ha, hb][e[1]], e[2] if len(e) > 2 else 0)
        ys.append(s.process(x[b * B:(b + 1) * B])[1][0])
    assert np.array_equal(np.concatenate(ys), ref)
    assert np.array_equal(impl_o1(x, [ha, hb], [(0, 0), (3, 1, 0)], B, L, 10 * B),
                          impl_o1(x, [ha, hb], [(0, 0), (3, 1)], B, L, 10 * B))


def test_swap_inside_the_first_block_without_an_ir_is_enoir():
    s = O.OracleStream(8, 8, 1)
    assert s.set_ir(np.ones(4, np.float32), 3) == 0
    rc, _ = s.process(np.ones(8, np.float32))
    assert rc == O.OR_ENOIR
    assert s.set_ir(np.ones(4, np.float32), 8) == O.OR_EINVAL
    assert s.set_ir(np.ones(4, np.float32), -1) == O.OR_EINVAL
