"""Pools: many streams advanced by one batched launch (optionally a hipGraph
replay).  Every stream's output must equal, bit for bit, the same stream
processed alone; float results must match the FP64 oracle within
1e-5 * RMS."""
import numpy as np
import pytest

from paper_2401_01607_amd import workloads as W
from tests.gpu_harness import binding, oracle_run, rel_err, rms_y64

pytestmark = pytest.mark.gpu

GB = 1 << 30


def _streams(n, seed, n_samples, lmin=64, lmax=4096, blocks=(32, 64, 128, 256, 512)):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        L = int(W.log_uniform_int(rng, lmin, lmax))
        B = int(rng.choice(np.array(blocks)))
        x = W.signal_gauss(n_samples, seed * 1000 + i)
        h = W.impulse_response(L, seed * 1000 + 500 + i)
        out.append((x, h, B, L))
    return out


def _alone(x, h, B, L, nb):
    import torch
    T = binding()
    s = T.Stream(B, L, max_blocks_per_call=nb)
    s.set_ir(h)
    xp = np.zeros(nb * B, np.float32)
    xp[: min(x.size, nb * B)] = x[: nb * B]
    xd = torch.from_numpy(xp).cuda()[None]
    yd = torch.empty_like(xd)
    s.process_blocks(xd, yd, nb)
    s.synchronize()
    y = yd.cpu().numpy()[0]
    s.close()
    return y


def _pool_run(specs, steps, use_graph=False, tile=0, between=None, copy_stream=None):
    """Run every stream through `steps` pool steps; specs: (x, h, B, L);
    steps: list of per-step block counts (same for every stream);
    copy_stream: a torch stream for the work-table copies, or None."""
    import torch
    T = binding()
    total = sum(steps)
    pool = T.Pool(len(specs), 64 * GB, use_graph=use_graph, tile_r=tile)
    if copy_stream is not None:
        assert T.taches_pool_set_copy_stream(pool.h, copy_stream.cuda_stream) == T.TACHES_OK
    ss, xs = [], []
    for x, h, B, L in specs:
        s = T.Stream(B, L, max_blocks_per_call=max(steps))
        s.set_ir(h)
        assert pool.attach(s) == T.TACHES_OK
        ss.append(s)
        xp = np.zeros(total * B, np.float32)
        xp[: min(x.size, total * B)] = x[: total * B]
        xs.append(torch.from_numpy(xp).cuda())
    ys = [torch.empty_like(x) for x in xs]
    done = 0
    for k, nbk in enumerate(steps):
        xin = [x[done * s.B:(done + nbk) * s.B][None] for x, s in zip(xs, ss)]
        yout = [torch.empty((1, nbk * s.B), device="cuda") for s in ss]
        pool.step(ss, xin, yout, [nbk] * len(ss))
        for y, yo, s in zip(ys, yout, ss):
            y[done * s.B:(done + nbk) * s.B] = yo[0]
        done += nbk
        if between is not None:
            between(k)
    pool.synchronize()
    info = pool.info()
    res = [y.cpu().numpy() for y in ys]
    if copy_stream is not None:
        assert T.taches_pool_set_copy_stream(pool.h, 0) == T.TACHES_OK
    pool.close()
    for s in ss:
        s.close()
    return res, info


def test_batched_equals_alone_bitwise_and_oracle():
    specs = _streams(24, 7, 6000)
    nb_of = [-(-(6000 + L - 1) // B) for _, _, B, L in specs]
    nb = max(nb_of)
    # one step covering the whole input of every stream (blocks beyond a
    # stream's input are zero input)
    ys, info = _pool_run(specs, [nb])
    assert info.last_items > 0 and info.last_workgroups > 0
    for (x, h, B, L), y in zip(specs, ys):
        alone = _alone(x, h, B, L, nb)
        assert np.array_equal(y, alone)
        ref = oracle_run(x, [h], [(0, 0)], B, L, nb)[0]
        assert rel_err(y, ref) <= 1e-5


@pytest.mark.parametrize("tile", [4, 8, 12, 16])
def test_every_pool_tile_gives_the_same_bits(tile):
    specs = _streams(10, 11, 3000, lmax=2000)
    base, _ = _pool_run(specs, [4, 7, 5], tile=16)
    ys, info = _pool_run(specs, [4, 7, 5], tile=tile)
    assert info.last_r == tile
    for a, b in zip(base, ys):
        assert np.array_equal(a, b)


def test_graph_replays_equal_eager_steps():
    """Many small steps (one block per stream per step) replayed from a
    captured graph, with eager torch work and synchronisations between
    replays; every step's outputs must equal the eager pool's."""
    import torch
    specs = _streams(16, 13, 2048, lmax=1500, blocks=(32, 64))
    steps = [1] * 24
    scratch = torch.zeros(1 << 20, device="cuda")

    def eager_work(k):
        scratch.add_(1.0)
        if k % 5 == 0:
            torch.cuda.synchronize()

    eager, _ = _pool_run(specs, steps)
    graphed, info = _pool_run(specs, steps, use_graph=True, between=eager_work)
    assert info.graph_replays >= len(steps) - 1
    assert info.graph_captures <= 2   # steps of one shape replay one captured graph
    for a, b in zip(eager, graphed):
        assert np.array_equal(a, b)
    assert float(scratch[0]) == len(steps)


@pytest.mark.parametrize("use_graph", [False, True])
def test_table_copy_stream_equals_default(use_graph):
    """Work tables copied on a stream of their own (the pool's stream waits
    for each copy; the two device tables are used in turn) give the same
    bits as copies on the pool's stream, step after step, with eager work
    and synchronisations between steps."""
    import torch
    specs = _streams(12, 17, 3000, lmax=2500, blocks=(32, 64, 128))
    steps = [1, 3, 1, 2, 1, 1, 4, 1, 2, 1]
    scratch = torch.zeros(1 << 20, device="cuda")

    def eager_work(k):
        scratch.add_(1.0)
        if k % 3 == 0:
            torch.cuda.synchronize()

    base, _ = _pool_run(specs, steps, use_graph=use_graph)
    cs = torch.cuda.Stream()
    sep, info = _pool_run(specs, steps, use_graph=use_graph, between=eager_work, copy_stream=cs)
    for a, b in zip(base, sep):
        assert np.array_equal(a, b)
    if use_graph:
        assert info.graph_replays >= len(steps) - 4


def test_admission_budget_and_slots():
    T = binding()
    s1, s2, s3 = T.Stream(64, 4096), T.Stream(64, 4096), T.Stream(64, 4096)
    b = s1.info().device_bytes
    pool = T.Pool(2, 2 * b + b // 2)
    assert pool.attach(s1) == T.TACHES_OK
    assert pool.attach(s1) == T.TACHES_EBUSY          # already attached
    assert pool.attach(s2) == T.TACHES_OK
    assert pool.attach(s3) == T.TACHES_EBUSY          # no free slot
    pool.detach(s2)
    big = T.Stream(64, 1 << 16)
    assert pool.attach(big) == T.TACHES_ENOMEM        # over the byte budget
    assert pool.info().used_bytes == b
    # an attached stream can only advance through the pool
    import torch
    x = torch.zeros((1, 64), device="cuda")
    with pytest.raises(T.TachesError) as e:
        s1.process_async(x, torch.empty_like(x))
    assert e.value.status == T.TACHES_EBUSY
    assert T.taches_close(s1.h) == T.TACHES_EBUSY
    assert T.taches_pool_destroy(pool.h) == T.TACHES_EBUSY
    pool.close()
    for s in (s1, s2, s3, big):
        s.close()


def test_ir_swap_between_steps_on_attached_stream():
    import torch
    T = binding()
    B, L = 64, 700
    x = W.signal_int(40 * B, 3, 30)
    ha, hb = W.signal_int(L, 4, 30), W.signal_int(L, 5, 30)
    s = T.Stream(B, L, max_blocks_per_call=10)
    s.set_ir(ha)
    pool = T.Pool(4, 8 * GB)
    pool.attach(s)
    outs = []
    for k in range(4):
        if k == 2:
            s.set_ir(hb)   # takes effect at the next step (block 20)
        xd = torch.from_numpy(x[k * 10 * B:(k + 1) * 10 * B]).cuda()[None]
        yd = torch.empty_like(xd)
        pool.step([s], [xd], [yd], [10])
        outs.append(yd)
    pool.synchronize()
    y = torch.cat(outs, 1).cpu().numpy()[0]
    ref = oracle_run(x, [ha, hb], [(0, 0), (20, 1)], B, L, 40)[0]
    assert np.array_equal(y, ref)
    pool.close()
    s.close()


def test_mixed_split_and_fp32_streams_in_one_step():
    import torch
    T = binding()
    B, L, n = 128, 1500, 4000
    nb = -(-(n + L - 1) // B)
    xs = np.stack([W.signal_gauss(n, 60 + c) for c in range(3)])
    h = W.impulse_response(L, 61)
    sf = T.Stream(B, L, max_blocks_per_call=nb)
    sp = T.Stream(B, L, channels=3, max_blocks_per_call=nb, precision=T.TACHES_PREC_SPLIT_BF16)
    sf.set_ir(h)
    sp.set_ir(h)
    pool = T.Pool(4, 8 * GB)
    pool.attach(sf)
    pool.attach(sp)
    xpad = np.zeros((3, nb * B), np.float32)
    xpad[:, :n] = xs
    xf = torch.from_numpy(xpad[:1].copy()).cuda()
    xsplit = torch.from_numpy(xpad).cuda()
    yf, ysp = torch.empty_like(xf), torch.empty_like(xsplit)
    pool.step([sf, sp], [xf, xsplit], [yf, ysp], [nb, nb])
    pool.synchronize()
    ref = oracle_run(xs, [h], [(0, 0)], B, L, nb)
    assert rel_err(yf.cpu().numpy()[0], ref[0]) <= 1e-5
    err = np.abs(ysp.cpu().numpy().astype(np.float64) - ref)
    assert err.max() <= 1e-4 * np.sqrt(np.mean(ref**2))
    pool.close()
    sf.close()
    sp.close()


def test_split_streams_batched_equal_alone_bitwise():
    """Split-BF16 streams of every kernel class in one pool step (one
    split-input and one Toeplitz launch per class: FP32 or FP64 tail, 32 or
    64 padded channels), with FP32 streams beside them, over uneven steps:
    each equals the same stream run alone bit for bit, and stays within the
    split-BF16 bound of the FP64 oracle."""
    import torch
    from tests.test_gpu_split import check_bound
    T = binding()
    SPLIT = T.TACHES_PREC_SPLIT_BF16
    shapes = [(1, 64, 700, 1), (2, 128, 1500, 2), (40, 256, 900, 1), (3, 32, 400, 2), (33, 512, 1200, 2),
              (1, 256, 2000, 0)]   # (channels, B, L, tail: 0 auto, 1 FP32, 2 FP64); the last is FP32 precision
    steps = [3, 1, 4, 2]
    nbs = sum(steps)

    def make(i, C, B, L, tail):
        prec = SPLIT if i < len(shapes) - 1 else T.TACHES_PREC_FP32
        s = T.Stream(B, L, channels=C, max_blocks_per_call=max(steps), precision=prec, tail=tail)
        s.set_ir(W.impulse_response(L, 610 + i))
        return s
    xs = [np.stack([W.signal_gauss(nbs * B, 620 + 10 * i + c) for c in range(C)]) for i, (C, B, L, _) in enumerate(shapes)]
    # alone
    alone = []
    for i, (C, B, L, tail) in enumerate(shapes):
        s = make(i, C, B, L, tail)
        outs, k0 = [], 0
        for n in steps:
            xd = torch.from_numpy(np.ascontiguousarray(xs[i][:, k0 * B:(k0 + n) * B])).cuda()
            yd = torch.empty_like(xd)
            s.process_blocks(xd, yd, n)
            outs.append(yd)
            k0 += n
        s.synchronize()
        alone.append(torch.cat(outs, 1).cpu().numpy())
        s.close()
    # batched
    ss = [make(i, *sh) for i, sh in enumerate(shapes)]
    pool = T.Pool(len(ss), 64 * GB, use_graph=True)
    for s in ss:
        assert pool.attach(s) == T.TACHES_OK
    outs = [[] for _ in ss]
    k0 = 0
    for n in steps:
        xd = [torch.from_numpy(np.ascontiguousarray(xs[i][:, k0 * sh[1]:(k0 + n) * sh[1]])).cuda()
              for i, sh in enumerate(shapes)]
        yd = [torch.empty_like(x) for x in xd]
        pool.step(ss, xd, yd, [n] * len(ss))
        for i in range(len(ss)):
            outs[i].append(yd[i])
        k0 += n
    pool.synchronize()
    for i in range(len(ss)):
        y = torch.cat(outs[i], 1).cpu().numpy()
        assert np.array_equal(y, alone[i]), f"stream {i} {shapes[i]}"
    for i in (0, 2, 4):
        C, B, L, _ = shapes[i]
        check_bound(alone[i], xs[i], [W.impulse_response(L, 610 + i)], [(0, 0)], B, L, nbs)
    pool.close()
    for s in ss:
        s.close()


def test_failed_step_with_a_split_stream_advances_nothing():
    """A step that lists a split-BF16 stream before a stream whose call is
    invalid fails as a whole: no stream advances (blocks done unchanged) and
    later steps give the same outputs as if the failed step never happened."""
    import torch
    T = binding()
    B, L, n = 128, 900, 2048
    nb = n // B
    xs = np.stack([W.signal_gauss(n, 80 + c) for c in range(2)])
    h = W.impulse_response(L, 82)

    def run(with_failure):
        sp = T.Stream(B, L, channels=2, max_blocks_per_call=nb, precision=T.TACHES_PREC_SPLIT_BF16)
        sf = T.Stream(B, L, max_blocks_per_call=4)
        sp.set_ir(h)
        sf.set_ir(h)
        pool = T.Pool(4, 8 * GB)
        pool.attach(sp)
        pool.attach(sf)
        xsp = torch.from_numpy(np.ascontiguousarray(xs)).cuda()
        xf = torch.from_numpy(np.ascontiguousarray(xs[:1, :4 * B])).cuda()
        ysp, yf = torch.empty_like(xsp), torch.empty_like(xf)
        if with_failure:
            rc = T.taches_pool_step(pool.h, [sp.h, sf.h], [xsp, xf], [ysp, yf], [nb, 5])  # 5 > 4 blocks
            assert rc == T.TACHES_EINVAL
            pool.synchronize()
            assert sp.info().blocks_done == 0 and sf.info().blocks_done == 0
        pool.step([sp, sf], [xsp, xf], [ysp, yf], [nb, 4])
        pool.synchronize()
        out = (ysp.cpu().numpy(), yf.cpu().numpy(), sp.info().blocks_done, sf.info().blocks_done)
        pool.close()
        sp.close()
        sf.close()
        return out
    a, b = run(False), run(True)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    assert a[2:] == b[2:] == (nb, 4)


def test_config4_reduced_parity():
    """Batched-workload shape (log-uniform L, B in {32..512}) on 48 streams
    of 12 000 samples with L up to 16 384, one launch, vs the oracle."""
    rng = np.random.default_rng(401)
    specs = []
    for i in range(48):
        L = int(W.log_uniform_int(rng, 256, 16384))
        B = int(rng.choice(np.array(W.BLOCK_CHOICES)))
        specs.append((W.signal_gauss(12_000, 410_000 + i), W.impulse_response(L, 420_000 + i), B, L))
    nb = max(-(-12_000 // B) for _, _, B, _ in specs)
    ys, info = _pool_run(specs, [nb])
    assert info.last_imbalance < 1.5
    for (x, h, B, L), y in list(zip(specs, ys))[::6]:
        ref = oracle_run(x, [h], [(0, 0)], B, L, nb)[0]
        assert rel_err(y, ref) <= 1e-5


def test_strided_multiblock_steps_from_planar_buffers():
    """Mono and stereo streams read blocks k .. k+n-1 straight out of one
    planar [2][N] buffer (channel stride N) and write slices of planar
    [C][total] outputs through taches_pool_step_strided, with a different
    block count per stream and step (drain steps with no input included);
    each equals the stream processed alone, bit for bit."""
    import torch
    T = binding()
    N = 200_000
    bank = torch.from_numpy(np.stack([W.signal_gauss(N, 61), W.signal_gauss(N, 62)])).cuda()
    shapes = [(1, 32, 300), (2, 64, 2500), (2, 256, 9000), (1, 512, 700), (2, 32, 5000), (1, 128, 64)]
    steps = 9
    counts = [[1 + (i * 3 + k) % 5 for k in range(steps)] for i in range(len(shapes))]
    pool = T.Pool(len(shapes), 64 * GB, use_graph=True)
    ss, offs, ys, irs, n_in = [], [], [], [], []
    for i, (C, B, L) in enumerate(shapes):
        s = T.Stream(B, L, channels=C, max_blocks_per_call=5)
        h = W.impulse_response(L, 6000 + i)
        s.set_ir(h)
        assert pool.attach(s) == T.TACHES_OK
        ss.append(s)
        irs.append(h)
        offs.append(1000 * i + 64 * (i % 3))
        total = sum(counts[i])
        n_in.append(total - 2)                     # the last two blocks drain with no input
        ys.append(torch.full((C, total * B), float("nan"), device="cuda"))
    done = [0] * len(ss)
    for k in range(steps):
        sp, xp, xcs, yp, ycs, nbs = [], [], [], [], [], []
        for i, s in enumerate(ss):
            B, nk = s.B, counts[i][k]
            # a range never mixes input and drain blocks
            if done[i] < n_in[i]:
                nk = min(nk, n_in[i] - done[i])
            sp.append(s.h)
            xp.append(bank.data_ptr() + 4 * (offs[i] + done[i] * B) if done[i] < n_in[i] else 0)
            xcs.append(N)
            yp.append(ys[i].data_ptr() + 4 * done[i] * B)
            ycs.append(ys[i].shape[1])
            nbs.append(nk)
            counts[i][k] = nk
        pool.step_strided(np.array(sp, np.uint64), np.array(xp, np.uint64), np.array(xcs), np.array(yp, np.uint64),
                          np.array(ycs), np.array(nbs, np.int32))
        for i in range(len(ss)):
            done[i] += counts[i][k]
    pool.synchronize()
    for i, (C, B, L) in enumerate(shapes):
        nb = done[i]
        x = np.zeros((C, nb * B), np.float32)
        x[:, :n_in[i] * B] = bank[:C, offs[i]:offs[i] + n_in[i] * B].cpu().numpy()
        s = T.Stream(B, L, channels=C, max_blocks_per_call=nb)
        s.set_ir(irs[i])
        xd = torch.from_numpy(x).cuda()
        yd = torch.empty_like(xd)
        s.process_blocks(xd, yd, nb)
        s.synchronize()
        got = ys[i][:, :nb * B].cpu().numpy()
        assert np.array_equal(got, yd.cpu().numpy()), f"stream {i}"
        if i < 2:
            ref = oracle_run(x, [irs[i]], [(0, 0)], B, L, nb)
            for c in range(C):
                assert rel_err(got[c], ref[c]) <= 1e-5
        s.close()
    pool.close()
    for s in ss:
        s.close()


def test_strided_step_rejects_short_channel_stride():
    import torch
    T = binding()
    pool = T.Pool(1, 64 * GB)
    s = T.Stream(64, 256, channels=2, max_blocks_per_call=4)
    s.set_ir(W.impulse_response(256, 3))
    assert pool.attach(s) == T.TACHES_OK
    y = torch.empty((2, 4 * 64), device="cuda")
    with pytest.raises(T.TachesError):
        pool.step_strided(np.array([s.h], np.uint64), np.zeros(1, np.uint64), None, np.array([y.data_ptr()], np.uint64),
                          np.array([100], np.int64), np.array([4], np.int32))
    pool.step_strided(np.array([s.h], np.uint64), np.zeros(1, np.uint64), None, np.array([y.data_ptr()], np.uint64),
                      np.array([256], np.int64), np.array([4], np.int32))
    pool.synchronize()
    assert s.info().blocks_done == 4
    pool.close()
    s.close()


def test_many_tiles_are_merged_into_range_items_exactly():
    """1024 streams x L = 270336 advancing one block per step: about
    2.7 x 10^5 output tiles per step, more than 32 per resident workgroup
    at any occupancy up to 32 one-wave workgroups per CU, merged into items
    of consecutive tiles; sampled streams equal their solo runs bit for bit."""
    import torch
    T = binding()
    N, B, L, steps = 1024, 64, 270336, 3
    h = torch.from_numpy(W.impulse_response(L, 91)).cuda()
    xbank = torch.from_numpy(W.signal_gauss(N * steps * B, 92)).cuda()
    pool = T.Pool(N, 64 * GB, use_graph=True, tile_r=16)
    ss = []
    for i in range(N):
        s = T.Stream(B, L)
        s.set_ir(h)
        assert pool.attach(s) == T.TACHES_OK
        ss.append(s)
    ys = torch.empty((steps, N, B), device="cuda")
    sp = np.array([s.h for s in ss], np.uint64)
    for k in range(steps):
        xp = np.array([xbank.data_ptr() + 4 * B * (i * steps + k) for i in range(N)], np.uint64)
        yp = np.array([ys[k, i].data_ptr() for i in range(N)], np.uint64)
        pool.step_strided(sp, xp, None, yp, None, np.ones(N, np.int32))
    pool.synchronize()
    info = pool.info()
    tiles = N * -(-(B + L - 1) // (64 * info.last_r))
    assert tiles > 32 * info.last_workgroups   # the merge condition holds
    assert 0 < info.last_items <= tiles // 3
    for i in range(0, N, 67):
        s = T.Stream(B, L)
        s.set_ir(h)
        y = torch.empty((steps, B), device="cuda")
        for k in range(steps):
            s.process_async(xbank[B * (i * steps + k):B * (i * steps + k + 1)], y[k])
        s.synchronize()
        assert torch.equal(y, ys[:, i]), f"stream {i}"
        s.close()
    for s in ss:
        pool.detach(s)
        s.close()
    pool.close()


def test_config4_full_size_sampled_parity():
    """Full batched-workload size in the benchmark's launch configuration:
    512 streams of 96 000 samples (L log-uniform in [256, 131 072], B in
    {32..512}), every stream's whole input in one pool step replayed from
    the pool's graph; sampled outputs of 15 streams (the longest IR among
    them) against Eq. (4) in FP64."""
    import torch
    from oracle import oracle as O
    T = binding()
    Ls, Bs = W.config4_draws()
    n = 96_000
    nbs = [-(-n // int(B)) for B in Bs]
    pool = T.Pool(len(Ls), 64 * GB, use_graph=True)
    ss, xs, ys, irs = [], [], [], []
    for i, (L, B) in enumerate(zip(Ls, Bs)):
        L, B = int(L), int(B)
        xp = np.zeros(nbs[i] * B, np.float32)
        xp[:n] = W.signal_gauss(n, 410_000 + i)
        irs.append(W.impulse_response(L, 420_000 + i))
        s = T.Stream(B, L, max_blocks_per_call=nbs[i])
        s.set_ir(irs[-1])
        assert pool.attach(s) == T.TACHES_OK
        ss.append(s)
        xs.append(torch.from_numpy(xp).cuda()[None])
        ys.append(torch.empty_like(xs[-1]))
    pool.step(ss, xs, ys, nbs)
    pool.synchronize()
    picks = sorted(set(list(range(0, len(Ls), 37)) + [int(np.argmax(Ls))]))
    rng = np.random.default_rng(404)
    for i in picks:
        B, S = int(Bs[i]), nbs[i] * int(Bs[i])
        y = ys[i].cpu().numpy()[0].astype(np.float64)
        idx = set(rng.integers(0, S, 40).tolist()) | {0, 1, n - 1, n, S - 1}
        idx = np.array(sorted(j for j in idx if 0 <= j < S))
        xi = xs[i].cpu().numpy()[0]
        ref = O.sampled_outputs(xi, [irs[i]], [(0, 0)], B, idx)
        rms = rms_y64(xi, [irs[i]], [(0, 0)], B, S)
        assert np.max(np.abs(y[idx] - ref)) <= 1e-5 * rms, f"stream {i} (L={int(Ls[i])}, B={B})"
    for s in ss:
        pool.detach(s)
        s.close()
    pool.close()


def test_heavy_and_light_streams_in_one_step_exactly():
    """256 light streams (one block of 64 per step) and 2 heavy ones (40
    blocks of 512 per step), L = 16 384, R = 16: every tile is one item
    (too few tiles to merge), many per workgroup, with tiles of very
    different work (dealt out largest first); the heavy streams and sampled
    light ones equal their solo runs bit for bit."""
    import torch
    T = binding()
    n_light, L, steps = 256, 16384, 2
    specs = [(64, 1, 700 + i) for i in range(n_light)] + [(512, 40, 900), (512, 40, 901)]
    h = torch.from_numpy(W.impulse_response(L, 95)).cuda()
    pool = T.Pool(len(specs), 64 * GB, use_graph=True, tile_r=16)
    ss, xs, ys = [], [], []
    for B, nb, seed in specs:
        s = T.Stream(B, L, max_blocks_per_call=nb)
        s.set_ir(h)
        assert pool.attach(s) == T.TACHES_OK
        ss.append(s)
        xs.append(torch.from_numpy(W.signal_gauss(steps * nb * B, seed)).cuda())
        ys.append(torch.empty(steps * nb * B, device="cuda"))
    sp = np.array([s.h for s in ss], np.uint64)
    nbs = np.array([nb for _, nb, _ in specs], np.int32)
    for k in range(steps):
        xp = np.array([x.data_ptr() + 4 * k * nb * B for x, (B, nb, _) in zip(xs, specs)], np.uint64)
        yp = np.array([y.data_ptr() + 4 * k * nb * B for y, (B, nb, _) in zip(ys, specs)], np.uint64)
        pool.step_strided(sp, xp, None, yp, None, nbs)
    pool.synchronize()
    info = pool.info()
    assert info.last_r == 16
    assert info.last_items == n_light * -(-(64 + L - 1) // 1024) + 2 * -(-(40 * 512 + L - 1) // 1024)
    assert info.last_items >= 8 * info.last_workgroups
    hn = h.cpu().numpy()
    for i in list(range(0, n_light, 37)) + [n_light, n_light + 1]:
        B, nb, _ = specs[i]
        y = _alone(xs[i].cpu().numpy(), hn, B, L, steps * nb)
        assert np.array_equal(ys[i].cpu().numpy(), y), f"stream {i}"
    for s in ss:
        pool.detach(s)
        s.close()
    pool.close()


def test_sample_accurate_swap_on_attached_stream():
    """taches_set_ir_at on a stream attached to a pool applies at its next
    step, from the given sample: equals the oracle exactly (integers)."""
    import torch
    T = binding()
    B, L, nb = 128, 900, 12
    x = W.signal_int(nb * B, 101, 31)
    ha, hb = W.signal_int(L, 102, 31), W.signal_int(400, 103, 31)
    pool = T.Pool(2, 64 * GB, use_graph=True)
    s = T.Stream(B, L, max_blocks_per_call=4)
    s.set_ir(ha)
    assert pool.attach(s) == T.TACHES_OK
    xd = torch.from_numpy(x).cuda()
    ys = []
    for k, n in enumerate((4, 3, 4, 1)):
        if k == 2:
            s.set_ir(hb, 77)            # takes over at sample 77 of the first block of step 2
        y = torch.empty(n * B, device="cuda")
        done = sum((4, 3, 4, 1)[:k])
        pool.step([s], [xd[done * B:(done + n) * B][None]], [y[None]], [n])
        ys.append(y)
    pool.synchronize()
    got = torch.cat(ys).cpu().numpy()
    ref = oracle_run(x, [ha, hb], [(0, 0), (7, 1, 77)], B, L, nb)[0]
    assert np.array_equal(got, ref)
    pool.detach(s)
    s.close()
    pool.close()


def test_detach_does_not_wait_and_keeps_order():
    """A stream detached right after a step was queued (no synchronisation)
    continues on its own HIP stream after that step: a call made right
    after the detach gives the same bits as the two calls made alone.  The
    pool's running device time covers its completed launches."""
    import torch
    T = binding()
    B, L = 128, 3000
    nb1, nb2 = 12, 40
    h = W.impulse_response(L, 171)
    x = W.signal_gauss((nb1 + nb2) * B, 172)
    xd = torch.from_numpy(x).cuda()
    ref = T.Stream(B, L, max_blocks_per_call=nb2)
    ref.set_ir(h)
    y_ref = torch.empty(((nb1 + nb2) * B,), device="cuda")
    ref.process_blocks(xd[None, :nb1 * B], y_ref[None, :nb1 * B], nb1)
    ref.process_blocks(xd[None, nb1 * B:], y_ref[None, nb1 * B:], nb2)
    ref.synchronize()
    s = T.Stream(B, L, max_blocks_per_call=nb2, torch_stream=False)   # its own HIP stream
    s.set_ir(h)
    pool = T.Pool(4, 8 * GB, use_graph=True)
    assert pool.attach(s) == T.TACHES_OK
    y = torch.empty_like(y_ref)
    pool.step([s], [xd[None, :nb1 * B]], [y[None, :nb1 * B]], [nb1])
    pool.detach(s)                                   # the step may still be queued
    s.process_blocks(xd[None, nb1 * B:], y[None, nb1 * B:], nb2)
    s.synchronize()
    pool.synchronize()
    assert torch.equal(y, y_ref)
    info = pool.info()
    assert info.device_ms_total > 0 and info.device_ms_total >= info.last_device_ms > 0
    pool.close()
    s.close()
    ref.close()
