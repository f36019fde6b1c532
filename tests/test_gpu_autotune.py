"""Empirical tile autotuner on the GPU: it times real calls, returns one of
its candidates, caches the choice, and the tuned tile gives the same bits."""
import numpy as np
import pytest

from paper_2401_01607_amd import autotune as A
from paper_2401_01607_amd import workloads as W
from tests.gpu_harness import binding

pytestmark = pytest.mark.gpu


def test_tune_stream_picks_a_timed_candidate_and_caches_it():
    T = binding()
    cache = A.TuneCache(None)
    cands = [(16, 4), (8, 1), (12, 2)]
    tile, ms = A.tune_stream(256, 4096, 1, 24, T.TACHES_PREC_FP32, candidates=cands, reps=2, cache=cache)
    assert tile in cands
    assert set(ms) == {"16,4", "8,1", "12,2"} and all(v > 0 for v in ms.values())
    assert ms[f"{tile[0]},{tile[1]}"] == min(ms.values())
    again, ms2 = A.tune_stream(256, 4096, 1, 24, T.TACHES_PREC_FP32, candidates=cands, cache=cache)
    assert again == tile and ms2 == ms


def test_tune_pool_sets_the_fastest_tile_and_bits_do_not_change():
    import torch
    T = binding()
    B, L, n, N = 128, 3000, 40 * 128, 24
    xs = [torch.from_numpy(W.signal_gauss(n, 500 + i)).cuda()[None] for i in range(N)]
    ys = [torch.empty_like(x) for x in xs]
    h = W.impulse_response(L, 499)
    pool = T.Pool(N, 1 << 33, use_graph=True)
    outs = []

    def one_step():
        ss = [T.Stream(B, L, max_blocks_per_call=n // B) for _ in range(N)]
        for s in ss:
            s.set_ir(h)
            pool.attach(s)
        pool.step(ss, xs, ys, [n // B] * N)
        pool.synchronize()
        outs.append(torch.stack([y.clone() for y in ys]))
        for s in ss:
            pool.detach(s)
            s.close()
    r, ms = A.tune_pool(pool, one_step, candidates=(16, 8))
    assert r in (16, 8) and ms[r] == min(ms.values())
    assert pool.info().last_r == 8 and set(ms) == {16, 8}
    one_step()
    assert pool.info().last_r == r
    assert all(torch.equal(o, outs[0]) for o in outs)
    pool.close()
