"""Error behaviour of the C-ABI (status codes, outputs untouched on error)."""
import numpy as np
import pytest

from paper_2401_01607_amd import workloads as W
from tests.gpu_harness import binding

pytestmark = pytest.mark.gpu


def test_process_before_ir_is_enoir_and_y_untouched():
    T = binding()
    s = T.taches_open(64, 128)
    x = np.ones(64, np.float32)
    y = np.full(64, 7.0, np.float32)
    assert T.taches_process(s, x, y) == T.TACHES_ENOIR
    assert np.all(y == 7.0)
    assert "impulse response" in T.taches_last_error()
    assert T.taches_close(s) == T.TACHES_OK


def test_bad_sizes_and_nulls():
    T = binding()
    s = T.taches_open(64, 128)
    assert T.taches_set_ir(s, np.ones(129, np.float32)) == T.TACHES_EINVAL
    assert T.taches_set_ir(s, np.ones(0, np.float32)) == T.TACHES_EINVAL
    assert T.lib.taches_set_ir(s, None, 10) == T.TACHES_EINVAL
    assert T.lib.taches_process(s, None, None) == T.TACHES_EINVAL
    assert T.taches_set_ir(s, np.ones(128, np.float32)) == T.TACHES_OK
    assert T.taches_set_tile(s, 5, 1) == T.TACHES_EINVAL
    assert T.lib.taches_load_ir_slot(s, 2, None, 4, 0) == T.TACHES_EINVAL
    assert T.taches_load_ir_slot(s, 9, np.ones(4, np.float32)) == T.TACHES_EINVAL
    assert T.taches_close(s) == T.TACHES_OK
    assert T.lib.taches_close(None) == T.TACHES_OK
    assert T.lib.taches_open(0, 10) is None
    assert T.lib.taches_open(10, 0) is None


def test_process_blocks_limits_and_empty_slot():
    import torch
    T = binding()
    s = T.Stream(32, 64, max_blocks_per_call=4)
    xd = torch.zeros((1, 5 * 32), device="cuda")
    yd = torch.full((1, 5 * 32), 3.0, device="cuda")
    s.load_ir_slot(0, W.impulse_response(64, 1))
    with pytest.raises(T.TachesError) as e:
        s.process_blocks(xd, yd, 5)
    assert e.value.status == T.TACHES_EINVAL
    with pytest.raises(T.TachesError) as e:
        s.process_blocks(xd[:, :128].contiguous(), yd[:, :128].contiguous(), 4, [1, -1, -1, -1])
    assert e.value.status == T.TACHES_ENOIR
    s.process_blocks(xd[:, :128].contiguous(), yd[:, :128].contiguous(), 4, [0, -1, -1, -1])
    s.synchronize()
    assert torch.all(yd[:, 128:] == 3.0)
    s.close()


def test_info_and_device_bytes():
    T = binding()
    cfg = T.taches_config_default(256, 65536)
    s = T.taches_open_ex(cfg)
    info = T.taches_get_info(s)
    assert info.ring_slots >= 65535 + 256
    assert info.device_bytes == T.taches_bytes_for(cfg)
    assert info.active_len == 0 and info.live == 0
    T.taches_set_ir(s, np.ones(1000, np.float32))
    y = np.zeros(256, np.float32)
    assert T.taches_process(s, np.ones(256, np.float32), y) == 0
    info = T.taches_get_info(s)
    assert info.active_len == 1000 and info.live == 999 and info.blocks_done == 1
    assert T.taches_close(s) == 0


def test_close_reopen_many_times():
    T = binding()
    for i in range(20):
        s = T.Stream(64, 2048)
        s.set_ir(np.ones(2048, np.float32))
        s.process(np.ones(64, np.float32))
        s.close()


def test_fp32_fma_ceiling_is_positive_and_below_the_packed_peak():
    from paper_2401_01607_amd import taches as T
    v = T.taches_fp32_fma_ceiling(0)
    assert 1.0 < v < 2 * 157.3


def test_call_times_record_only_timed_calls():
    """taches_set_timing / taches_call_times: only calls made while timing is
    on are recorded, oldest first; reading clears the record; the device time
    of a long call exceeds that of a one-block call."""
    import torch
    from paper_2401_01607_amd import taches as T
    B, L = 256, 4096
    s = T.Stream(B, L, max_blocks_per_call=64)
    s.set_ir(torch.ones(L, device="cuda"))
    x = torch.ones((1, 64 * B), device="cuda")
    y = torch.empty_like(x)
    s.process_blocks(x, y, 64)                   # not timed
    assert len(s.call_times(8)) == 0
    s.set_timing(True)
    s.process_blocks(x[:, :B], y[:, :B], 1)
    s.process_blocks(x, y, 64)
    s.set_timing(False)
    s.process_blocks(x, y, 64)                   # not timed
    t = s.call_times(8)
    assert len(t) == 2 and t[0] > 0 and t[1] > t[0]
    assert len(s.call_times(8)) == 0
    s.set_timing(True)
    for _ in range(3):
        s.process_blocks(x, y, 64)
    t = s.call_times(2)                          # the last two of three
    assert len(t) == 2 and all(v > 0 for v in t)
    s.close()
