"""GPU parity: the HIP library against the CPU oracle, bit for bit.

Every output of every dtype must equal the oracle's (tolerance 0: the
generator is an exact integer recurrence and both conversions are defined
by a single rounding or none).  Small cases span several LDS tiles and
ragged tails; the headline workload (2^20 streams x 4096) is checked in
full, slice by slice, against the oracle run on several threads.
"""
import os
import sys

import numpy as np
import pytest

import oracle
from paper_1412_8266_amd import workloads as wl

pytestmark = pytest.mark.gpu

# (engine, stream-major strategy): integer / binary64 arithmetic, lane per
# stream / wave per stream
# (engine, strategy, lanes per stream of the wave-per-stream fill)
CONFIGS = [(1, 0, 0), (0, 1, 64), (1, 1, 64), (0, 2, 64), (1, 2, 64), (1, 2, 32), (0, 2, 16),
           (1, 2, 16), (1, 2, 8)]
CONFIG_IDS = ["default", "int-lane", "f64-lane", "int-wave", "f64-wave", "f64-wave32",
              "int-wave16", "f64-wave16", "f64-wave8"]


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def mg():
    import torch
    import paper_1412_8266_amd as m
    assert torch.cuda.is_available()
    return m


@pytest.fixture(params=CONFIGS, ids=CONFIG_IDS)
def engine(request, mg):
    keys = ("engine", "strategy", "coop_lanes")
    old = [mg.mrg_config_get(k) for k in keys]
    for k, v in zip(keys, request.param):
        mg.mrg_config_set(k, v)
    yield request.param
    for k, v in zip(keys, old):
        mg.mrg_config_set(k, v)


def host(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy()


def oracle_fill(base, first, count, n, dtype, layout=oracle.STREAM_MAJOR):
    st = oracle.streams(np.asarray(base, dtype=np.uint32), first, count)
    return oracle.fill(st, n, dtype, layout)


def test_c1_seed_12345_u32_then_f64(mg, engine):
    say("C1 engine", engine)
    ss = mg.StreamSet(wl.C1_STREAMS, seed=wl.C1_SEED)
    got = host(ss.fill(wl.C1_N, mg.U32))
    want, st = oracle_fill(wl.C1_SEED, 0, wl.C1_STREAMS, wl.C1_N, oracle.U32)
    assert np.array_equal(got, want)
    assert np.array_equal(ss.get_states(), st)
    ss.close()
    ss = mg.StreamSet(wl.C1_STREAMS, seed=wl.C1_SEED)
    got = host(ss.fill(wl.C1_N, mg.F64))
    wantd, _ = oracle_fill(wl.C1_SEED, 0, wl.C1_STREAMS, wl.C1_N, oracle.F64)
    assert np.array_equal(got.view(np.uint64), wantd.view(np.uint64))
    # the first output of stream 0 is the worked example's
    assert int(want[0, 0]) == 545508589
    ss.close()


@pytest.mark.parametrize("dtype", [0, 1, 2], ids=["u32", "f32", "f64"])
@pytest.mark.parametrize("layout", [0, 1], ids=["sm", "il"])
def test_ragged_shapes(mg, engine, dtype, layout):
    base = oracle.seed_from_master(99)
    for first, count, n in [(0, 1, 1), (3, 5, 33), (0, 63, 31), (1, 64, 32), (0, 65, 64),
                            (7, 130, 100), (0, 129, 257), (2, 3, 0), (0, 200, 3),
                            (1, 3, 2048), (0, 2, 4096), (2, 3, 4097), (0, 4, 9000),
                            (0, 70, 1100)]:
        say("ragged", engine, dtype, layout, first, count, n)
        ss = mg.StreamSet(first + count + 2, seed=[int(x) for x in base])
        out = ss.fill(n, dtype, layout, first=first, count=count)
        got = host(out)
        want, st = oracle_fill(base, first, count, n, dtype, layout)
        assert got.shape == want.shape
        assert np.array_equal(got.view(np.uint8), want.view(np.uint8)), (first, count, n)
        assert np.array_equal(ss.get_states(first, count), st)
        # untouched streams keep their start states
        assert np.array_equal(ss.get_states(0, first), oracle.streams(base, 0, first))
        ss.close()


def test_unaligned_row_and_pointer(mg, engine):
    import torch
    base = oracle.seed_from_master(7)
    say("unaligned", engine)
    for n, off in [(37, 1), (40, 1), (64, 3), (2050, 1), (4096, 2), (4097, 7), (9000, 5),
                   (8192, 31)]:
        ss = mg.StreamSet(70, seed=[int(x) for x in base])
        buf = torch.zeros(70 * n + 40, dtype=torch.uint32, device="cuda")
        ss.fill_ptr(n, mg.U32, mg.STREAM_MAJOR, buf.data_ptr() + 4 * off)
        h = host(buf)
        got = h[off:off + 70 * n].reshape(70, n)
        want, _ = oracle_fill(base, 0, 70, n, oracle.U32)
        assert np.array_equal(got, want), (n, off)
        # nothing written outside the rows
        assert not h[:off].any() and not h[off + 70 * n:].any(), (n, off)
        ss.close()
    for n, off in [(1000, 1), (2049, 3), (5000, 5)]:  # f64 rows off the 128-byte lines
        ss = mg.StreamSet(33, seed=[int(x) for x in base])
        buf = torch.zeros(33 * n + 24, dtype=torch.float64, device="cuda")
        ss.fill_ptr(n, mg.F64, mg.STREAM_MAJOR, buf.data_ptr() + 8 * off)
        h = host(buf)
        want, _ = oracle_fill(base, 0, 33, n, oracle.F64)
        assert np.array_equal(h[off:off + 33 * n].reshape(33, n).view(np.uint64),
                              want.view(np.uint64)), (n, off)
        assert not h[:off].any() and not h[off + 33 * n:].any(), (n, off)
        ss.close()


def test_chained_fills_equal_one_fill(mg, engine):
    base = oracle.seed_from_master(11)
    say("chained", engine)
    ss = mg.StreamSet(77, seed=[int(x) for x in base])
    ns = (5, 32, 1, 100, 64, 4096, 2049)
    parts = [host(ss.fill(n, mg.U32)) for n in ns]
    got = np.concatenate(parts, axis=1)
    want, st = oracle_fill(base, 0, 77, sum(ns), oracle.U32)
    assert np.array_equal(got, want)
    assert np.array_equal(ss.get_states(), st)
    ss.close()


def test_dtypes_share_one_sequence(mg, engine):
    say("dtypes", engine)
    u = mg.StreamSet(100, master_seed=5)
    f = mg.StreamSet(100, master_seed=5)
    d = mg.StreamSet(100, master_seed=5)
    zu = host(u.fill(300, mg.U32)).astype(np.int64)
    zf = host(f.fill(300, mg.F32))
    zd = host(d.fill(300, mg.F64))
    assert np.array_equal(zf, ((2 * ((zu - 1) >> 9) + 1) * 2.0**-24).astype(np.float32))
    assert np.array_equal(zd, zu.astype(np.float64) * 2.328306549295727688e-10)
    for s in (u, f, d):
        s.close()


def test_jump_per_stream_exponents(mg):
    import torch
    base = oracle.seed_from_master(21)
    for bits in (17, 64, 100, 192):
        say("jump bits", bits)
        S = 333
        ss = mg.StreamSet(S + 4, seed=[int(x) for x in base])
        w = wl.random_exponents(S, bits, seed=bits)
        ss.jump(torch.from_numpy(w.view(np.int64)).cuda(), first=2, count=S)
        got = ss.get_states(2, S)
        want = oracle.jump_many_words(oracle.streams(base, 2, S), w)
        assert np.array_equal(got, want)
        ss.close()


def test_jump_uniform_and_substreams(mg):
    base = oracle.seed_from_master(22)
    ss = mg.StreamSet(50, seed=[int(x) for x in base])
    say("jump uniform")
    e = (1 << 150) + 12345
    ss.jump_uniform(e, first=5, count=40)
    want = oracle.jump_many(oracle.streams(base, 5, 40), e)
    assert np.array_equal(ss.get_states(5, 40), want)
    ss.jump_substreams(3, first=5, count=40)
    want = oracle.jump_many(want, 3 << 76)
    assert np.array_equal(ss.get_states(5, 40), want)
    ss.close()


def test_jump_zero_and_small_equal_stepping(mg):
    import torch
    base = oracle.seed_from_master(23)
    say("jump small")
    S = 64
    ss = mg.StreamSet(S, seed=[int(x) for x in base])
    e = np.arange(S, dtype=np.uint64)
    w = np.zeros((S, 3), dtype=np.uint64)
    w[:, 0] = e
    ss.jump(torch.from_numpy(w.view(np.int64)).cuda())
    got = ss.get_states()
    st = oracle.streams(base, 0, S)
    for i in range(S):
        assert np.array_equal(got[i], oracle.skip(st[i], i))
    ss.close()


def test_streamset_first_stream_offset(mg):
    say("first_stream offset")
    base = oracle.seed_from_master(24)
    for first in (1, 1000, 2**40 + 7, 2**64 - 10):
        ss = mg.StreamSet(10, seed=[int(x) for x in base], first_stream=first)
        assert np.array_equal(ss.get_states(), oracle.streams(base, first, 10))
        ss.close()


def test_state_roundtrip_and_validation(mg):
    say("states")
    ss = mg.StreamSet(10, master_seed=1)
    st = ss.get_states()
    st2 = st.copy()
    st2[3] = [1, 2, 3, 4, 5, 6]
    ss.set_states(st2)
    assert np.array_equal(ss.get_states(), st2)
    bad = st2.copy()
    bad[0] = [0, 0, 0, 1, 1, 1]
    with pytest.raises(mg.MRGError):
        ss.set_states(bad)
    assert np.array_equal(ss.get_states(), st2)
    with pytest.raises(mg.MRGError):
        ss.fill(4, first=8, count=5)
    ss.close()


_C3_CACHE = {}


def c3_expected():
    """Oracle: stream starts, jump by the offsets, then by one substream, then
    1024 outputs (computed once per session)."""
    if "want" not in _C3_CACHE:
        base = oracle.seed_from_master(wl.MASTER_SEED)
        S, n = wl.C3_STREAMS, wl.C3_N
        off = wl.c3_offsets(S)
        st = oracle.streams(base, 0, S)
        st = oracle.jump_many_words(st, np.stack([off, np.zeros_like(off), np.zeros_like(off)], 1))
        st = oracle.jump_many(st, 1 << 76)
        _C3_CACHE["want"] = oracle.fill(st, n, oracle.U32)
    return _C3_CACHE["want"]


def test_c3_full(mg, engine):
    """2^16 streams, random 64-bit offsets plus one substream, 1024 outputs."""
    import torch
    say("C3 engine", engine)
    S, n = wl.C3_STREAMS, wl.C3_N
    ss = mg.StreamSet(S, master_seed=wl.MASTER_SEED)
    off = wl.c3_offsets(S)
    ss.jump(torch.from_numpy(wl.c3_exponents(off).view(np.int64)).cuda())
    got = host(ss.fill(n, mg.U32))
    want, st2 = c3_expected()
    assert np.array_equal(got, want)
    assert np.array_equal(ss.get_states(), st2)
    ss.close()


@pytest.mark.parametrize("dtype", [0, 1, 2], ids=["u32", "f32", "f64"])
def test_negative_component2_words(mg, engine, dtype):
    """Streams steered so that one output each draws the component-2 residue
    m2 - 1 or m2 - 2, where the binary64 reduction's biased quotient is one
    too big and the word comes out negative: the wave-per-stream writer's
    checked draws must draw that piece again.  Positions fall in row heads,
    first and last pieces, chunk and member boundaries and row tails, for
    aligned and unaligned rows (aligned rows of whole chunks go through the
    whole-chunk writer), inside guard words."""
    import torch
    from tests import crafted
    rng = np.random.default_rng(77)
    es = 8 if dtype == 2 else 4
    for n, off in [(4096, 0), (4096, 5), (5000, 3), (2048, 0), (9000, 1), (300, 1), (8192, 0)]:
        pos = {0, 1, 2, 31, 32, 33, 63, 64, 127, 128, 255, 256, 257, 511, 512, 1023, 1024,
               n - 33, n - 32, n - 2, n - 1} | set(int(x) for x in rng.integers(0, n, 12))
        positions = sorted(k for k in pos if 0 <= k < n)
        starts = crafted.hits(positions, [oracle.M2 - 1, oracle.M2 - 2], seed=n + dtype)
        S = len(starts)
        say("negative words", engine, dtype, n, off, S)
        ss = mg.StreamSet(S, master_seed=1)
        ss.set_states(starts)
        guard = 32  # 128 or 256 bytes: off = 0 leaves the rows on lines
        buf = torch.zeros(S * n + off + 2 * guard, dtype=mg.torch_dtype(dtype), device="cuda")
        ss.fill_ptr(n, dtype, mg.STREAM_MAJOR, buf.data_ptr() + (guard + off) * es)
        h = host(buf)
        want, st = oracle.fill(starts, n, dtype)
        got = h[guard + off:guard + off + S * n]
        assert np.array_equal(got.view(np.uint8), want.reshape(-1).view(np.uint8)), (n, off)
        assert not h[:guard + off].view(np.uint8).any() and not h[guard + off + S * n:].view(np.uint8).any()
        assert np.array_equal(ss.get_states(), st), (n, off)
        ss.close()


def test_negative_component2_words_batch_and_deal(mg):
    """The same steered streams through the other users of the wave writer:
    the persistent batch's stream segments and the in-order leapfrog deal."""
    import torch
    from tests import crafted
    n = 40000  # 160 KiB per stream: several batch segments
    positions = [0, 33, 4095, 4096, 16383, 16384, 20000, 32768, 39999]
    starts = crafted.hits(positions, [oracle.M2 - 1, oracle.M2 - 2], seed=3)
    S = len(starts)
    ss = mg.StreamSet(S, master_seed=2)
    ss.set_states(starts)
    out = torch.zeros((S, n), dtype=torch.uint32, device="cuda")
    b = mg.Batch(ss, [(0, 4, n, 0, out.data_ptr(), mg.U32, 0),
                      (4, S - 4, n, 0, out[4].data_ptr(), mg.U32, 0)],
                 mg.batch_config(segment_bytes=64 << 10))
    b.run()
    want, st = oracle.fill(starts, n, oracle.U32)
    assert np.array_equal(host(out), want)
    assert np.array_equal(ss.get_states(), st)
    b.close()
    ss.close()
    # one stream dealt in order: P * K outputs of it, blocks of 16-256 KiB
    k = 300001
    start = crafted.hits([k], [oracle.M2 - 1], seed=4)[0]
    ss = mg.StreamSet(1, master_seed=3)
    ss.set_states(start[None, :])
    P, K = 1000, 700
    got = host(ss.fill_leapfrog(0, P, K, mg.U32, mg.INTERLEAVED))
    want, st = oracle.fill(start[None, :], P * K, oracle.U32)
    assert np.array_equal(got.reshape(-1), want[0])
    assert np.array_equal(ss.get_states(), st)
    ss.close()


def oracle_threaded(st, n, dtype, layout=oracle.STREAM_MAJOR):
    """oracle.fill over the rows of st, split across up to 16 threads (the C
    oracle runs outside the interpreter lock); same result as one call."""
    from concurrent.futures import ThreadPoolExecutor
    threads = max(1, min(16, os.cpu_count() or 1))
    parts = [ix for ix in np.array_split(np.arange(len(st)), threads) if len(ix)]
    with ThreadPoolExecutor(len(parts)) as ex:
        res = list(ex.map(lambda ix: oracle.fill(st[ix[0]:ix[-1] + 1], n, dtype, layout), parts))
    axis = 0 if layout == oracle.STREAM_MAJOR else 1
    return np.concatenate([r[0] for r in res], axis=axis), np.concatenate([r[1] for r in res])


@pytest.mark.parametrize("dtype,layout", [(0, 0), (1, 0), (0, 1)], ids=["u32-sm", "f32-sm", "u32-il"])
def test_c2_full(mg, dtype, layout):
    """The benchmark's workload in full: 2^20 streams from the master seed,
    4096 outputs each (16 GiB), every output and every end state against the
    oracle, copied back and recomputed in slices of 2^15 streams."""
    import torch
    S, n = wl.C2_STREAMS, wl.C2_N
    say("C2 full", dtype, layout)
    base = oracle.seed_from_master(wl.MASTER_SEED)
    st0 = oracle.streams_adjacent(base, 0, S)
    ss = mg.StreamSet(S, master_seed=wl.MASTER_SEED)
    assert np.array_equal(ss.get_states(), st0)
    out = ss.fill(n, dtype, layout)
    torch.cuda.synchronize()
    ends = []
    ch = 1 << 15
    for c0 in range(0, S, ch):
        part = out[c0:c0 + ch] if layout == 0 else out[:, c0:c0 + ch].contiguous()
        got = host(part)
        want, st = oracle_threaded(st0[c0:c0 + ch], n, dtype, layout)
        assert np.array_equal(got.view(np.uint32), want.view(np.uint32)), c0
        ends.append(st)
        del part, got, want
    assert np.array_equal(ss.get_states(), np.concatenate(ends))
    del out
    ss.close()


# whole and partial super-chunks of 512 stream groups (16 lanes per stream
# below 64 KiB rows, 4 streams per group; one stream per group from 64 KiB)
PLACEMENT_SHAPES = [(3000, 4096, 0), (4100, 4096, 0), (2052, 2048, 0), (1100, 20000, 0),
                    (600, 4100, 2), (2049, 3000, 1)]
PLACEMENT_KNOBS = [(1, 0, 0), (1, 1, 0), (1, 0, 1), (1, 0, 3), (1, 1, 2), (0, 0, 0), (0, 1, 3)]


@pytest.mark.parametrize("knobs", PLACEMENT_KNOBS,
                         ids=["chunked", "ranges", "persist1", "persist3", "ranges-persist2",
                              "int-chunked", "int-ranges-persist3"])
def test_wave_writer_placements(mg, knobs):
    """The wave-per-stream writer's group placements (chunked XCD order with
    its tail of groups past the last whole super-chunk, one range per XCD,
    persistent workgroups looping over groups: settings that promise no
    effect on results) against the oracle, every output and end state."""
    keys = ("engine", "coop_order", "coop_wgs_per_cu")
    old = [mg.mrg_config_get(k) for k in keys]
    base = oracle.seed_from_master(31)
    try:
        for k, v in zip(keys, knobs):
            mg.mrg_config_set(k, v)
        for count, n, dtype in PLACEMENT_SHAPES:
            say("placement", knobs, count, n, dtype)
            ss = mg.StreamSet(count + 5, seed=[int(x) for x in base])
            got = host(ss.fill(n, dtype, first=5, count=count))
            want, st = oracle_threaded(oracle.streams(base, 5, count), n, dtype)
            assert np.array_equal(got.view(np.uint8), want.view(np.uint8)), (count, n, dtype)
            assert np.array_equal(ss.get_states(5, count), st), (count, n, dtype)
            ss.close()
    finally:
        for k, v in zip(keys, old):
            mg.mrg_config_set(k, v)


def test_random_fill_sweep(mg):
    """Seeded random fills against the oracle: row counts and lengths across
    the lane-per-stream / wave-per-stream boundary and several chunks,
    output pointers off their 128-byte lines by any number of elements,
    8/16/32/64 lanes per stream or automatic, both engines, every dtype,
    both layouts, and a second fill continuing from the first.  Guard words
    around the output must stay untouched."""
    import torch
    rng = np.random.default_rng(1412)
    keys = ("engine", "strategy", "coop_lanes")
    old = [mg.mrg_config_get(k) for k in keys]
    base = oracle.seed_from_master(2012)
    try:
        for case in range(200):
            engine = int(rng.integers(2))
            lanes = int(rng.choice([0, 8, 16, 32, 64]))
            strategy = int(rng.choice([0, 0, 1, 2]))
            dt = int(rng.integers(3))
            layout = int(rng.integers(2)) if case % 3 == 0 else 0
            count = int(rng.integers(1, 200))
            n = int(np.exp(rng.uniform(0, np.log(12000))))
            first = int(rng.integers(0, 50))
            es = 8 if dt == 2 else 4
            off = int(rng.integers(0, 128 // es))
            for k, v in zip(keys, (engine, strategy, lanes)):
                mg.mrg_config_set(k, v)
            say("sweep", case, dict(engine=engine, lanes=lanes, strategy=strategy, dt=dt,
                                    layout=layout, count=count, n=n, first=first, off=off))
            ss = mg.StreamSet(first + count + 3, seed=[int(x) for x in base])
            st = oracle.streams(base, first, count)
            tdt = mg.torch_dtype(dt)
            guard = 16
            buf = torch.zeros(count * n + off + 2 * guard, dtype=tdt, device="cuda")
            for rep in range(2):
                buf.zero_()
                view = buf[guard + off:guard + off + count * n]
                ss.fill_ptr(n, dt, layout, view.data_ptr(), first=first, count=count)
                h = host(buf)
                want, st = oracle.fill(st, n, dt, layout)
                got = h[guard + off:guard + off + count * n]
                assert np.array_equal(got.view(np.uint8), want.reshape(-1).view(np.uint8)), \
                    (case, rep)
                assert not h[:guard + off].view(np.uint8).any(), (case, rep, "before")
                assert not h[guard + off + count * n:].view(np.uint8).any(), (case, rep, "after")
            assert np.array_equal(ss.get_states(first, count), st), case
            ss.close()
    finally:
        for k, v in zip(keys, old):
            mg.mrg_config_set(k, v)


# (count, n, dtype, lanes per stream): rows on 128-byte lines and whole
# chunks only, so every full group takes the whole-chunk writer; counts that
# leave a partial last group (general writer), one and several chunks per row
WHOLE_SHAPES = [(1001, 4096, 0, 16), (7, 12288, 0, 16), (66, 8192, 1, 32), (130, 4096, 2, 16),
                (9, 16384, 0, 8), (3, 65536, 0, 64), (64, 2048, 1, 16), (255, 6144, 0, 32)]


@pytest.mark.parametrize("engine_id", [1, 0], ids=["f64", "int"])
def test_whole_chunk_writer(mg, engine_id):
    """The wave-per-stream fill's whole-chunk writer (rows starting on lines,
    row lengths a multiple of the chunk) against the oracle, with stream
    ranges that start inside the set and end in a partial group, twice in a
    row, every output and end state, inside guard words."""
    import torch
    keys = ("engine", "strategy", "coop_lanes")
    old = [mg.mrg_config_get(k) for k in keys]
    base = oracle.seed_from_master(4096)
    try:
        for count, n, dt, lanes in WHOLE_SHAPES:
            for k, v in zip(keys, (engine_id, 2, lanes)):
                mg.mrg_config_set(k, v)
            say("whole-chunk writer", engine_id, count, n, dt, lanes)
            first = 3
            ss = mg.StreamSet(first + count + 2, seed=[int(x) for x in base])
            st = oracle.streams(base, first, count)
            guard = 1024  # a line-aligned view inside the buffer
            buf = torch.zeros(count * n + 2 * guard, dtype=mg.torch_dtype(dt), device="cuda")
            assert buf.data_ptr() % 128 == 0
            for rep in range(2):
                buf.zero_()
                view = buf[guard:guard + count * n]
                ss.fill_ptr(n, dt, 0, view.data_ptr(), first=first, count=count)
                h = host(buf)
                want, st = oracle_threaded(st, n, dt)
                got = h[guard:guard + count * n]
                assert np.array_equal(got.view(np.uint8), want.reshape(-1).view(np.uint8)), \
                    (count, n, dt, lanes, rep)
                assert not h[:guard].view(np.uint8).any(), (count, n, dt, lanes, "before")
                assert not h[guard + count * n:].view(np.uint8).any(), (count, n, dt, lanes, "after")
            assert np.array_equal(ss.get_states(first, count), st), (count, n, dt, lanes)
            ss.close()
    finally:
        for k, v in zip(keys, old):
            mg.mrg_config_set(k, v)


def test_lane_writer_rows_off_lines(mg):
    """The lane-per-stream writer for rows off their 128-byte lines (each
    line shared by two rows written once, from both rows' lanes): row lengths
    from one line up, offsets across a line, waves of 1 to 64 rows and
    partial last waves, every dtype, both engines, twice in a row, inside
    guard words (the bytes around the output belong to nobody).  Rows of
    4 mod 8 dwords (the wider LDS pitch) run both on 16-byte boundaries
    (16-byte staging) and off them."""
    import torch
    keys = ("engine", "strategy")
    old = [mg.mrg_config_get(k) for k in keys]
    base = oracle.seed_from_master(128)
    rng = np.random.default_rng(128)
    try:
        for engine_id in (1, 0):
            for dt in (0, 1, 2):
                es = 8 if dt == 2 else 4
                lens = [128 // es, 128 // es + 1, 256 // es - 1, 256 // es, 256 // es + 1,
                        1000, 1001, 333]
                # (n, element offset or None for a random one): rows of 4 mod 8
                # dwords, 16-byte aligned (offset 0) and not (offset 1)
                cases = [(n, None) for n in lens] + [(m * 4 // es, o) for m in (44, 1500)
                                                     for o in (0, 1)]
                for n, off in cases:
                    count = int(rng.choice([1, 2, 63, 64, 65, 130]))
                    if off is None:
                        off = int(rng.integers(0, 128 // es))
                    for k, v in zip(keys, (engine_id, 1)):
                        mg.mrg_config_set(k, v)
                    say("rows off lines", engine_id, dt, n, count, off)
                    ss = mg.StreamSet(count, seed=[int(x) for x in base])
                    st = oracle.streams(base, 0, count)
                    guard = 64
                    buf = torch.zeros(count * n + off + 2 * guard, dtype=mg.torch_dtype(dt),
                                      device="cuda")
                    for rep in range(2):
                        buf.zero_()
                        view = buf[guard + off:guard + off + count * n]
                        ss.fill_ptr(n, dt, 0, view.data_ptr())
                        h = host(buf)
                        want, st = oracle.fill(st, n, dt)
                        got = h[guard + off:guard + off + count * n]
                        assert np.array_equal(got.view(np.uint8), want.reshape(-1).view(np.uint8)), \
                            (engine_id, dt, n, count, off, rep)
                        assert not h[:guard + off].view(np.uint8).any()
                        assert not h[guard + off + count * n:].view(np.uint8).any()
                    assert np.array_equal(ss.get_states(), st)
                    ss.close()
    finally:
        for k, v in zip(keys, old):
            mg.mrg_config_set(k, v)


@pytest.mark.parametrize("gen", ["mrg32k3a", "philox"])
def test_degenerate_calls_change_nothing(mg, gen):
    """Empty ranges, zero-length fills, zero jumps and empty deals write
    nothing and move no state; a zero jump of the whole set is the identity."""
    import torch
    with mg.StreamSet(70, master_seed=5, generator=gen) as ss:
        st = np.asarray(ss.get_states(), dtype=np.uint32).copy()
        guard = torch.full((256,), 0x5A5A5A5A, dtype=torch.int32, device="cuda")
        assert ss.fill(7, mg.U32, first=10, count=0).numel() == 0
        assert ss.fill(0, mg.F64, mg.INTERLEAVED).numel() == 0
        ss.fill_ptr(0, mg.U32, mg.STREAM_MAJOR, guard.data_ptr())
        ss.fill_ptr(0, mg.F64, mg.INTERLEAVED, guard.data_ptr(), first=3, count=5)
        ss.fill_ptr(9, mg.F32, mg.STREAM_MAJOR, guard.data_ptr(), first=69, count=0)
        ss.jump_uniform(0)
        ss.jump_uniform(12345, first=20, count=0)
        ss.jump(torch.zeros(3 * 70, dtype=torch.int64, device="cuda"))
        if gen == "mrg32k3a":
            ss.jump_substreams(0)
            assert ss.fill_leapfrog(4, 0, 9).numel() == 0
            assert ss.fill_leapfrog(4, 5, 0, mg.F64, mg.INTERLEAVED).numel() == 0
        torch.cuda.synchronize()
        assert np.all(guard.cpu().numpy().view(np.uint32) == 0x5A5A5A5A)
        assert np.array_equal(np.asarray(ss.get_states(), dtype=np.uint32), st)
        # and the set still continues its streams: one value each equals the oracle
        one = host(ss.fill(1, mg.U32))
        if gen == "mrg32k3a":
            want, _ = oracle.fill(st, 1, oracle.U32)
        else:
            want, _ = oracle.philox_fill(st, 1, oracle.U32)
        assert np.array_equal(one, want)
