"""Off-line whole-signal convolution (taches_convolve): the same kernels over
all blocks plus the temporal overflow in one call, optionally with the roles
of input and IR exchanged (Section 3.2, Fig. 6).  Integer inputs must equal
numpy.convolve exactly under both roles; float inputs stay within
1e-5 * RMS of the FP64 result."""
import numpy as np
import pytest

from paper_2401_01607_amd import workloads as W
from tests.gpu_harness import binding, rel_err, rms_y64

pytestmark = pytest.mark.gpu


def _conv(x, h, **kw):
    import torch
    T = binding()
    xd = torch.from_numpy(np.ascontiguousarray(x, np.float32)).cuda()
    hd = torch.from_numpy(np.ascontiguousarray(h, np.float32)).cuda()
    shape = (xd.shape[0], xd.shape[-1] + hd.numel() - 1) if xd.dim() > 1 else (xd.numel() + hd.numel() - 1,)
    yd = torch.full(shape, float("nan"), device="cuda")
    rc = T.taches_convolve(xd, hd, yd, **kw)
    assert rc == T.TACHES_OK, T.lib.taches_last_error()
    torch.cuda.synchronize()
    return yd.cpu().numpy()


@pytest.mark.parametrize("nx,nh", [(5000, 700), (300, 4000), (1, 1), (257, 1), (1, 513), (4096, 4096)])
@pytest.mark.parametrize("swap", [False, True])
def test_integer_convolution_is_exact(nx, nh, swap):
    x = W.signal_int(nx, 111, 31)
    h = W.signal_int(nh, 112, 31)
    y = _conv(x, h, role_swap=swap)
    assert np.array_equal(y, np.convolve(x.astype(np.float64), h.astype(np.float64)))


def test_float_parity_and_roles_agree():
    x = W.signal_gauss(3000, 113)
    h = W.impulse_response(50_000, 114)
    ref = np.convolve(x.astype(np.float64), h.astype(np.float64))
    y0 = _conv(x, h)
    y1 = _conv(x, h, role_swap=True)
    assert rel_err(y0, ref) <= 1e-5
    assert rel_err(y1, ref) <= 1e-5


def test_multichannel_fp32_and_split():
    C = 5
    x = np.stack([W.signal_gauss(20_000, 115 + c) for c in range(C)])
    h = W.impulse_response(9000, 120)
    y = _conv(x, h)
    ys = _conv(x, h, precision=1)
    for c in range(C):
        ref = np.convolve(x[c].astype(np.float64), h.astype(np.float64))
        assert rel_err(y[c], ref) <= 1e-5
        err = np.abs(ys[c].astype(np.float64) - ref)
        rms = np.sqrt(np.mean(ref ** 2))
        assert err.max() <= 1e-4 * rms and np.sqrt(np.mean(err ** 2)) <= 1e-5 * rms


def test_errors():
    import torch
    T = binding()
    x = torch.zeros(10, device="cuda")
    h = torch.zeros(4, device="cuda")
    y = torch.zeros(13, device="cuda")
    assert T.lib.taches_convolve(None, 10, 1, T._dev_ptr(h), 4, T._dev_ptr(y), 0, 0, 0, None) == T.TACHES_EINVAL
    assert T.lib.taches_convolve(T._dev_ptr(x), 0, 1, T._dev_ptr(h), 4, T._dev_ptr(y), 0, 0, 0, None) == T.TACHES_EINVAL
    assert T.lib.taches_convolve(T._dev_ptr(x), 10, 1, T._dev_ptr(h), 4, T._dev_ptr(y), 7, 0, 0, None) == T.TACHES_EINVAL


@pytest.mark.parametrize("swap", [False, True])
def test_longest_ir_4m_taps_sampled_parity(swap):
    """The off-line capacity shape: 0.1 s of input (4 800 samples) through a
    4 194 304-tap IR, in both roles; sampled outputs (the ramp, the flat part
    and the end) against Eq. (1) in FP64."""
    from oracle import oracle as O
    x = W.signal_gauss(4800, 131)
    h = W.impulse_response(1 << 22, 132)
    y = _conv(x, h, role_swap=swap).astype(np.float64)
    n_out = x.size + h.size - 1
    assert y.shape == (n_out,) and np.all(np.isfinite(y))
    rng = np.random.default_rng(133)
    idx = set(rng.integers(0, n_out, 300).tolist()) | {0, 1, 4799, 4800, h.size - 1, h.size, n_out - 1}
    idx = np.array(sorted(idx))
    ref = O.sampled_outputs(x, [h], [(0, 0)], 4800, idx)
    rms = rms_y64(x, [h], [(0, 0)], 4800, n_out)
    assert np.max(np.abs(y[idx] - ref)) <= 1e-5 * rms
