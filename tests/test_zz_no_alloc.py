"""The off-line convolution without allocation (taches_convolve_noalloc),
called through the C-ABI: its output equals taches_convolve's (FP32) bit
for bit and stays within 1e-5 * RMS of the FP64 result, over calls in a row
on one stream whose later inputs are smaller (the shared work memory keeps
the previous call's contents), in both roles, with an FP64 tail, and with
several channels; sizes beyond its work memory are refused on the host."""
import numpy as np
import pytest

from paper_2401_01607_amd import workloads as W
from tests.gpu_harness import binding, rel_err

pytestmark = pytest.mark.gpu


def _tensors(x, h):
    import torch
    xd = torch.from_numpy(np.ascontiguousarray(x, np.float32)).cuda()
    hd = torch.from_numpy(np.ascontiguousarray(h, np.float32)).cuda()
    shape = (xd.shape[0], xd.shape[-1] + hd.numel() - 1) if xd.dim() > 1 else (xd.numel() + hd.numel() - 1,)
    return xd, hd, shape


def _both(x, h, swap=False):
    """(taches_convolve, taches_convolve_noalloc) outputs on the same inputs;
    the no-allocation call writes into a buffer filled with NaN first."""
    import torch
    T = binding()
    xd, hd, shape = _tensors(x, h)
    y_ref = torch.full(shape, float("nan"), device="cuda")
    assert T.taches_convolve(xd, hd, y_ref, role_swap=swap) == T.TACHES_OK, T.lib.taches_last_error()
    y = torch.full(shape, float("nan"), device="cuda")
    print(f"noalloc: x {tuple(xd.shape)} h {hd.numel()} swap={swap}", flush=True)
    assert T.taches_convolve_noalloc(xd, hd, y, role_swap=swap) == T.TACHES_OK, T.lib.taches_last_error()
    torch.cuda.synchronize()
    return y_ref.cpu().numpy(), y.cpu().numpy()


def _fp64(x, h):
    return np.convolve(np.asarray(x, np.float64), np.asarray(h, np.float64))


def test_calls_in_a_row_second_smaller_equal_the_allocating_call():
    cases = [
        (np.stack([W.signal_gauss(30_001, 901 + c) for c in range(2)]), W.impulse_response(4097, 903)),
        (W.signal_gauss(1000, 904), W.impulse_response(300, 905)),
        (W.signal_gauss(7, 906), W.impulse_response(5, 907)),
    ]
    for x, h in cases:
        y_ref, y = _both(x, h)
        assert np.array_equal(y, y_ref)
        for c, xc in enumerate(np.atleast_2d(x)):
            yc = np.atleast_2d(y)[c]
            assert rel_err(yc, _fp64(xc, h)) <= 1e-5


@pytest.mark.parametrize("swap", [False, True])
def test_roles_and_fp64_tail(swap):
    # IR of 2^18 taps: FP64 tail; with the roles exchanged the 5 000-sample
    # input becomes the IR (FP32 tail)
    x = W.signal_gauss(5000, 911)
    h = W.impulse_response(1 << 18, 912)
    y_ref, y = _both(x, h, swap)
    assert np.array_equal(y, y_ref)
    assert rel_err(y, _fp64(x, h)) <= 1e-5
    # then a smaller call on the same work memory
    x2, h2 = W.signal_gauss(3000, 913), W.impulse_response(1000, 914)
    y_ref2, y2 = _both(x2, h2, swap)
    assert np.array_equal(y2, y_ref2)
    assert rel_err(y2, _fp64(x2, h2)) <= 1e-5


def test_integer_inputs_exact():
    x = W.signal_int(4000, 921, 31)
    h = W.signal_int(999, 922, 31)
    y_ref, y = _both(x, h)
    assert np.array_equal(y, _fp64(x, h)) and np.array_equal(y, y_ref)


def test_too_large_and_bad_arguments_are_refused():
    import torch
    T = binding()
    # 2^24 input samples need 64 MiB for the padded input alone
    x = torch.zeros(1 << 24, device="cuda")
    h = torch.zeros(16, device="cuda")
    y = torch.zeros((1 << 24) + 15, device="cuda")
    assert T.taches_convolve_noalloc(x, h, y) == T.TACHES_EINVAL
    assert "limit" in T.lib.taches_last_error().decode()
    xs = torch.zeros(10, device="cuda")
    ys = torch.zeros(25, device="cuda")
    assert T.lib.taches_convolve_noalloc(None, 10, 1, T._dev_ptr(h), 16, T._dev_ptr(ys), 0, 0, None) == T.TACHES_EINVAL
    assert T.lib.taches_convolve_noalloc(T._dev_ptr(xs), 0, 1, T._dev_ptr(h), 16, T._dev_ptr(ys), 0, 0, None) == T.TACHES_EINVAL
    assert T.lib.taches_convolve_noalloc(T._dev_ptr(xs), 10, 1, T._dev_ptr(h), 16, T._dev_ptr(ys), 0, 64, None) == T.TACHES_EINVAL
    # a valid call still works after the refusals
    x2, h2 = W.signal_gauss(600, 931), W.impulse_response(77, 932)
    y_ref, y2 = _both(x2, h2)
    assert np.array_equal(y2, y_ref)
