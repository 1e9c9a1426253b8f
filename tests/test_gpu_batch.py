"""GPU parity of the persistent batched path against the CPU oracle.

A batch must produce, bit for bit, what the oracle produces for each request
on its own: plain requests continue their streams (and advance them),
substream requests draw substreams (sec. 4.1) of one stream and leave it
unchanged.  Work decompositions (segment length, lane/wave threshold, static
or dynamic schedule), the graph launch, the direct launch and the
per-request reference schedule must all agree.
"""
import sys

import numpy as np
import pytest

import oracle
from paper_1412_8266_amd import workloads as wl

pytestmark = pytest.mark.gpu

SEED = 0xBA7C4


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def mg():
    import torch
    import paper_1412_8266_amd as m
    assert torch.cuda.is_available()
    return m


def host(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy()


def make_plain(mg, rng, n_req, max_k, max_n, budget):
    """Contiguous plain requests; returns rows, tensors, specs."""
    import torch
    rows, outs, specs = [], [], []
    first = 0
    total = 0
    while len(rows) < n_req:
        k = int(wl.log_uniform_int(rng, max_k, 1)[0])
        n = int(wl.log_uniform_int(rng, max_n, 1)[0])
        if total + k * n > budget:
            continue
        dt = int(rng.integers(0, 3))
        if rng.random() < 0.1:
            k, n = (0, n) if rng.random() < 0.5 else (k, 0)  # empty requests are skipped
        t = torch.empty((k, n), dtype=mg.torch_dtype(dt), device="cuda")
        rows.append((first, k, n, 0, t.data_ptr() if t.numel() else 0, dt, 0))
        outs.append(t)
        specs.append((first, k, n, dt))
        first += k
        total += k * n
    return rows, outs, specs, first


def check_plain(base, specs, outs, states_before):
    """Each request against the oracle from the given start states."""
    for (first, k, n, dt), t in zip(specs, outs):
        if k == 0 or n == 0:
            continue
        want, _ = oracle.fill(states_before[first:first + k], n, dt)
        got = host(t)
        assert np.array_equal(got.view(np.uint8), want.view(np.uint8)), (first, k, n, dt)


CONFIGS = {
    "default": dict(),
    "small-seg": dict(segment_bytes=16 * 1024),
    "static": dict(schedule=2, waves_per_cu=4),
    "all-rows": dict(wave_min_bytes=1 << 40),
    "all-waves": dict(wave_min_bytes=4, segment_bytes=32 * 1024),
}


@pytest.mark.parametrize("name", list(CONFIGS))
@pytest.mark.parametrize("engine", [0, 1], ids=["int", "f64"])
def test_plain_batch_matches_oracle(mg, name, engine):
    say("batch", name, engine)
    old = mg.mrg_config_get("engine")
    mg.mrg_config_set("engine", engine)
    try:
        rng = np.random.default_rng(SEED + len(name))
        rows, outs, specs, nstreams = make_plain(mg, rng, 40, 150, 60000, 6_000_000)
        base = oracle.seed_from_master(SEED)
        ss = mg.StreamSet(nstreams, seed=[int(x) for x in base])
        st0 = oracle.streams(base, 0, nstreams)
        b = mg.Batch(ss, rows, mg.batch_config(**CONFIGS[name]))
        info = b.info()
        assert info["requests"] == sum(1 for s in specs if s[1] and s[2])
        b.run()
        check_plain(base, specs, outs, st0)
        # end states advanced by n for every stream of every request
        st1 = st0.copy()
        for first, k, n, dt in specs:
            if k and n:
                st1[first:first + k] = oracle.jump_many(st0[first:first + k], n)
        assert np.array_equal(ss.get_states(), st1)
        # a second run continues the streams
        b.run()
        check_plain(base, specs, outs, st1)
        b.close()
        ss.close()
    finally:
        mg.mrg_config_set("engine", old)


# (streams, values per stream, dtype): row requests whose items carry several
# 64-stream blocks (short rows: up to 16 blocks, about 128 KiB of output per
# item) with a partial last item and a partial last block, next to requests of
# one block or less and rows long enough for one block per item.
ROW_BLOCK_SHAPES = [(1100, 20, 0), (1100, 33, 1), (1025, 7, 2), (1, 20, 0), (63, 33, 0),
                    (64, 100, 1), (65, 100, 0), (700, 1000, 0), (130, 700, 2), (2500, 3, 1)]


@pytest.mark.parametrize("engine", [0, 1], ids=["int", "f64"])
def test_row_items_in_blocks(mg, engine):
    import torch
    say("row blocks", engine)
    old = mg.mrg_config_get("engine")
    mg.mrg_config_set("engine", engine)
    try:
        rows, outs, specs, first = [], [], [], 0
        for k, n, dt in ROW_BLOCK_SHAPES:
            t = torch.empty((k, n), dtype=mg.torch_dtype(dt), device="cuda")
            rows.append((first, k, n, 0, t.data_ptr(), dt, 0))
            outs.append(t)
            specs.append((first, k, n, dt))
            first += k
        base = oracle.seed_from_master(SEED + 7)
        ss = mg.StreamSet(first, seed=[int(x) for x in base])
        st0 = oracle.streams(base, 0, first)
        # every request a row request; a few resident waves, so that waves
        # take several items each
        b = mg.Batch(ss, rows, mg.batch_config(wave_min_bytes=1 << 40, waves_per_cu=1))
        b.run()
        check_plain(base, specs, outs, st0)
        st1 = st0.copy()
        for f, k, n, dt in specs:
            st1[f:f + k] = oracle.jump_many(st0[f:f + k], n)
        assert np.array_equal(ss.get_states(), st1)
        # the per-request launches agree
        b.run_per_request()
        check_plain(base, specs, outs, st1)
        b.close()
        ss.close()
    finally:
        mg.mrg_config_set("engine", old)


def test_substream_requests(mg):
    import torch
    say("substreams")
    rng = np.random.default_rng(SEED + 7)
    base = oracle.seed_from_master(SEED + 7)
    ss = mg.StreamSet(12, seed=[int(x) for x in base])
    st0 = ss.get_states()
    rows, outs, specs = [], [], []
    for i in range(30):
        s = int(rng.integers(0, 12))
        k = int(wl.log_uniform_int(rng, 100, 1)[0])
        n = int(wl.log_uniform_int(rng, 20000, 1)[0])
        if k * n > 400_000:
            n = max(1, 400_000 // k)
        sub0 = int(rng.integers(0, 1 << 40))
        dt = int(rng.integers(0, 3))
        t = torch.empty((k, n), dtype=mg.torch_dtype(dt), device="cuda")
        rows.append((s, k, n, sub0, t.data_ptr(), dt, mg.REQ_SUBSTREAMS))
        outs.append(t)
        specs.append((s, k, n, sub0, dt))
    b = mg.Batch(ss, rows, mg.batch_config(segment_bytes=16 * 1024))
    for rep in range(2):
        b.run()
        for (s, k, n, sub0, dt), t in zip(specs, outs):
            starts = np.stack([oracle.jump(st0[s], (sub0 + j) << 76) for j in range(k)])
            want, _ = oracle.fill(starts, n, dt)
            assert np.array_equal(host(t).view(np.uint8), want.view(np.uint8)), (s, k, n, sub0)
        assert np.array_equal(ss.get_states(), st0)  # unchanged
    b.close()
    ss.close()


@pytest.mark.parametrize("engine", [0, 1], ids=["int", "f64"])
def test_mixed_plain_and_substream_groups(mg, engine):
    """Plain and substream requests of all three dtypes, rows and waves,
    in one batch: one persistent kernel per (dtype, kind) group."""
    import torch
    say("mixed groups", engine)
    old = mg.mrg_config_get("engine")
    mg.mrg_config_set("engine", engine)
    try:
        rng = np.random.default_rng(SEED + 11)
        rows, outs, specs, nplain = make_plain(mg, rng, 30, 120, 50000, 4_000_000)
        subs = []
        for i in range(12):
            s = nplain + int(rng.integers(0, 4))
            k = int(wl.log_uniform_int(rng, 80, 1)[0])
            n = int(wl.log_uniform_int(rng, 30000, 1)[0])
            if k * n > 300_000:
                n = max(1, 300_000 // k)
            sub0 = int(rng.integers(0, 1 << 30))
            dt = i % 3
            t = torch.empty((k, n), dtype=mg.torch_dtype(dt), device="cuda")
            rows.append((s, k, n, sub0, t.data_ptr(), dt, mg.REQ_SUBSTREAMS))
            outs.append(t)
            subs.append((s, k, n, sub0, dt))
        order = rng.permutation(len(rows))
        base = oracle.seed_from_master(SEED + 11)
        ss = mg.StreamSet(nplain + 4, seed=[int(x) for x in base])
        st0 = oracle.streams(base, 0, nplain + 4)
        b = mg.Batch(ss, [rows[i] for i in order], mg.batch_config(segment_bytes=32 * 1024))
        b.run()
        check_plain(base, specs, outs[:len(specs)], st0)
        for (s, k, n, sub0, dt), t in zip(subs, outs[len(specs):]):
            starts = np.stack([oracle.jump(st0[s], (sub0 + j) << 76) for j in range(k)])
            want, _ = oracle.fill(starts, n, dt)
            assert np.array_equal(host(t).view(np.uint8), want.view(np.uint8)), (s, k, n, sub0)
        st1 = st0.copy()
        for first, k, n, dt in specs:
            if k and n:
                st1[first:first + k] = oracle.jump_many(st0[first:first + k], n)
        assert np.array_equal(ss.get_states(), st1)
        b.close()
        ss.close()
    finally:
        mg.mrg_config_set("engine", old)


def test_graph_direct_and_per_request_agree(mg):
    import torch
    say("graph vs direct vs per-request")
    rng = np.random.default_rng(SEED + 3)
    sets, batches, outsets = [], [], []
    for mode in range(3):
        rng = np.random.default_rng(SEED + 3)
        rows, outs, specs, nstreams = make_plain(mg, rng, 50, 300, 40000, 8_000_000)
        ss = mg.StreamSet(nstreams, master_seed=SEED + 3)
        sets.append(ss)
        batches.append(mg.Batch(ss, rows, mg.batch_config(segment_bytes=64 * 1024)))
        outsets.append(outs)
    for rep in range(3):
        batches[0].run()
        junk = torch.randn(1 << 20, device="cuda").sum()  # eager work between replays
        batches[1].run_direct()
        batches[2].run_per_request()
        torch.cuda.synchronize()
        del junk
        for t0, t1, t2 in zip(*outsets):
            a, b_, c = host(t0), host(t1), host(t2)
            assert np.array_equal(a.view(np.uint8), b_.view(np.uint8))
            assert np.array_equal(a.view(np.uint8), c.view(np.uint8))
        s0 = sets[0].get_states()
        assert np.array_equal(s0, sets[1].get_states())
        assert np.array_equal(s0, sets[2].get_states())
    for b in batches:
        b.close()
    for s in sets:
        s.close()


def test_request_completion_times(mg):
    import torch
    say("request completion stamps")
    rng = np.random.default_rng(SEED + 9)
    rows, outs, specs, nstreams = make_plain(mg, rng, 60, 200, 40000, 6_000_000)
    ss = mg.StreamSet(nstreams, master_seed=SEED + 9)
    b = mg.Batch(ss, rows, mg.batch_config(segment_bytes=32 * 1024))
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for rep in range(2):
        e0.record()
        b.run()
        e1.record()
        torch.cuda.synchronize()
        total = e0.elapsed_time(e1)
        t = b.request_times()
        assert t.shape == (len(rows),)
        for (first, k, n, dt), ti in zip(specs, t):
            if k and n:
                assert 0 < ti <= total + 0.05, (ti, total)
            else:
                assert ti == 0
    b.close()
    ss.close()


def test_autotune_restores_states_and_keeps_results(mg):
    say("autotune")
    rng = np.random.default_rng(SEED + 5)
    rows, outs, specs, nstreams = make_plain(mg, rng, 40, 200, 50000, 6_000_000)
    base = oracle.seed_from_master(SEED + 5)
    ss = mg.StreamSet(nstreams, seed=[int(x) for x in base])
    st0 = oracle.streams(base, 0, nstreams)
    b = mg.Batch(ss, rows)
    cands = [mg.batch_config(segment_bytes=s, waves_per_cu=w, schedule=sc)
             for s, w, sc in [(64 << 10, 8, 1), (256 << 10, 16, 1), (1 << 20, 16, 2)]]
    best, ms = b.autotune(cands, reps=1)
    assert 0 <= best < 3 and all(x > 0 for x in ms)
    assert np.array_equal(ss.get_states(), st0)
    assert b.info()["segment_bytes"] == cands[best].segment_bytes
    b.run()
    check_plain(base, specs, outs, st0)
    b.close()
    ss.close()


def test_c4_full_mix_in_waves(mg):
    """The whole 10,000-request mix at full size (1.76 TiB of output), run in
    waves of consecutive requests whose outputs fit in device memory, each
    wave one batch (one graph launch).  Against the oracle: the first and the
    last 64 values of every stream (the tail reached by an oracle jump),
    twenty requests drawn at random in full, and the end state of every
    stream."""
    import torch
    W = 64
    req = wl.c4_requests()
    nb = req.bytes()
    R = len(req)
    S = int(req.n_streams.sum())
    starts = oracle.streams_adjacent(oracle.seed_from_master(wl.MASTER_SEED), 0, S)
    rng = np.random.default_rng(45)
    full = set(rng.choice(np.flatnonzero(nb <= (64 << 20)), 20, replace=False).tolist())
    ends = np.zeros((S, 6), dtype=np.uint32)
    ss = mg.StreamSet(S, master_seed=wl.MASTER_SEED)

    def padded(x):
        return (int(x) + 255) // 256 * 256

    cap = min(int(torch.cuda.mem_get_info()[0] * 0.7), 200 << 30)
    i = wave = 0
    while i < R:
        j, tot = i, 0
        while j < R and tot + padded(nb[j]) <= cap:
            tot += padded(nb[j])
            j += 1
        assert j > i, "request %d alone exceeds the wave budget" % i
        say("C4 wave %d: requests %d..%d, %.1f GB" % (wave, i, j - 1, tot / 1e9))
        buf = torch.empty(tot, dtype=torch.uint8, device="cuda")
        rows, offs, off = [], [], 0
        for r in range(i, j):
            rows.append((int(req.first_stream[r]), int(req.n_streams[r]), int(req.length[r]), 0,
                         buf.data_ptr() + off, int(req.dtype[r]), 0))
            offs.append(off)
            off += padded(nb[r])
        b = mg.Batch(ss, rows)
        b.run()
        torch.cuda.synchronize()
        for r, off in zip(range(i, j), offs):
            first, k, n, dt = (int(req.first_stream[r]), int(req.n_streams[r]),
                               int(req.length[r]), int(req.dtype[r]))
            es = 8 if dt == 2 else 4
            t = buf[off:off + k * n * es].view(mg.torch_dtype(dt)).view(k, n)
            st = starts[first:first + k]
            h = min(W, n)
            want, end = oracle.fill(st, h, dt)
            got = t[:, :h].cpu().numpy()
            assert np.array_equal(got.view(np.uint8), want.view(np.uint8)), ("head", r)
            if n > h:
                want, end = oracle.fill(oracle.jump_uniform(st, n - W), W, dt)
                got = t[:, n - W:].cpu().numpy()
                assert np.array_equal(got.view(np.uint8), want.view(np.uint8)), ("tail", r)
            ends[first:first + k] = end
            if r in full:
                want, _ = oracle.fill(st, n, dt)
                assert np.array_equal(t.cpu().numpy().view(np.uint8), want.view(np.uint8)), r
        b.close()
        del buf, t
        torch.cuda.empty_cache()
        i, wave = j, wave + 1
    assert np.array_equal(ss.get_states(), ends)
    ss.close()


def test_batch_validation(mg):
    import torch
    ss = mg.StreamSet(100, master_seed=1)
    t = torch.empty((10, 10), dtype=torch.uint32, device="cuda")
    with pytest.raises(mg.MRGError):  # overlapping streams
        mg.Batch(ss, [(0, 10, 10, 0, t.data_ptr(), 0, 0), (5, 10, 10, 0, t.data_ptr(), 0, 0)])
    with pytest.raises(mg.MRGError):  # outside the set
        mg.Batch(ss, [(95, 10, 10, 0, t.data_ptr(), 0, 0)])
    with pytest.raises(mg.MRGError):  # bad dtype
        mg.Batch(ss, [(0, 10, 10, 0, t.data_ptr(), 7, 0)])
    u = torch.empty((10, 10), dtype=torch.uint32, device="cuda")
    with pytest.raises(mg.MRGError):  # substreams of a stream that a plain request advances
        mg.Batch(ss, [(0, 10, 10, 0, t.data_ptr(), 0, 0),
                      (3, 10, 10, 0, u.data_ptr(), 0, mg.REQ_SUBSTREAMS)])
    b = mg.Batch(ss, [(0, 10, 10, 0, t.data_ptr(), 0, 0),  # next to it is fine
                      (10, 10, 10, 0, u.data_ptr(), 0, mg.REQ_SUBSTREAMS)])
    b.close()
    b = mg.Batch(ss, [])  # empty batch runs as a no-op
    b.run()
    b.close()
    ss.close()
