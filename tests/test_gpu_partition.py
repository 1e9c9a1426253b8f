"""GPU parity of the other two partitions of one sequence in sec. 2.3, random
spacing and the leapfrog deal, against the CPU oracle, bit for bit.

Random spacing: every state of the set equals the oracle's expansion of its
SplitMix64 draw, and fills from those states equal the oracle's.  Leapfrog:
small deals are compared in full (both layouts, every dtype, both engines,
ragged player and card counts, an output pointer off its 128-byte line) and
the end state of the dealt stream is checked; large deals are compared on
sampled cards that the oracle computes one by one with a jump.
"""
import sys

import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu

MASTER = 0x0123456789ABCDEF


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def mg():
    import torch
    import paper_1412_8266_amd as m
    assert torch.cuda.is_available()
    return m


@pytest.fixture(params=[1, 0], ids=["f64-engine", "int-engine"])
def engine(request, mg):
    old = mg.mrg_config_get("engine")
    mg.mrg_config_set("engine", request.param)
    yield request.param
    mg.mrg_config_set("engine", old)


def host(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy()


def states_of(ss):
    return np.asarray(ss.get_states(), dtype=np.uint32).reshape(-1, 6)


# --------------------------------------------------------------------------
# random spacing
# --------------------------------------------------------------------------
@pytest.mark.parametrize("first,count", [(0, 1), (0, 1000), (2**40 + 7, 333), (2**64 - 5, 5)])
def test_random_spacing_states(mg, first, count):
    say("random spacing", first, count)
    with mg.StreamSet(count, master_seed=MASTER, first_stream=first, spacing="random") as ss:
        got = states_of(ss)
        assert np.array_equal(got, oracle.random_spacing_states(MASTER, first, count))
        assert list(ss.base_state) == [0] * 6


def test_random_spacing_fill(mg, engine):
    say("random spacing fill, engine", engine)
    with mg.StreamSet(300, master_seed=7, spacing="random") as ss:
        st = oracle.random_spacing_states(7, 0, 300)
        out = host(ss.fill(1500, mg.U32))
        want, end = oracle.fill(st, 1500, oracle.U32)
        assert np.array_equal(out, want)
        assert np.array_equal(states_of(ss), end)


# --------------------------------------------------------------------------
# leapfrog
# --------------------------------------------------------------------------
DEALS = [(1, 1), (1, 5000), (5000, 1), (64, 64), (100, 77), (3, 7000), (1000, 1000),
         (257, 130), (70000, 3), (1000, 5), (4097, 63), (10000, 2), (777, 32), (123457, 17),
         (65, 33)]


@pytest.mark.parametrize("players,per_player", DEALS, ids=["%dx%d" % d for d in DEALS])
@pytest.mark.parametrize("layout", [0, 1], ids=["player-rows", "in-order"])
def test_leapfrog_small(mg, engine, players, per_player, layout):
    say("leapfrog", players, per_player, "layout", layout, "engine", engine)
    with mg.StreamSet(5, master_seed=MASTER) as ss:
        before = states_of(ss)
        for dtype in (mg.U32, mg.F32, mg.F64):
            st = states_of(ss)
            out = host(ss.fill_leapfrog(3, players, per_player, dtype, layout))
            want, end = oracle.leapfrog(st[3], players, per_player, dtype, layout)
            assert out.shape == want.shape
            assert np.array_equal(out, want), (dtype, layout)
            after = states_of(ss)
            assert np.array_equal(after[3], end)
            # the other streams are untouched
            assert np.array_equal(np.delete(after, 3, 0), np.delete(before, 3, 0))


@pytest.mark.parametrize("layout", [0, 1], ids=["player-rows", "in-order"])
def test_leapfrog_unaligned_output(mg, layout):
    import torch
    players, per_player = 333, 129
    say("leapfrog unaligned", layout)
    with mg.StreamSet(2, master_seed=11) as ss:
        st = states_of(ss)
        buf = torch.full((players * per_player + 64,), 0xDEADBEEF, dtype=torch.uint32, device="cuda")
        view = buf[1:1 + players * per_player]
        ss.fill_leapfrog(1, players, per_player, mg.U32, layout, out=view)
        b = host(buf)
        want, end = oracle.leapfrog(st[1], players, per_player, oracle.U32, layout)
        assert np.array_equal(b[1:1 + players * per_player], want.reshape(-1))
        assert b[0] == 0xDEADBEEF and np.all(b[1 + players * per_player:] == 0xDEADBEEF)
        assert np.array_equal(states_of(ss)[1], end)


def test_leapfrog_zero_is_noop_and_validation(mg):
    with mg.StreamSet(2, master_seed=1) as ss:
        st = states_of(ss)
        ss.fill_leapfrog(0, 0, 10)
        ss.fill_leapfrog(0, 10, 0)
        assert np.array_equal(states_of(ss), st)
        with pytest.raises(mg._abi.MRGError):
            ss.fill_leapfrog(2, 4, 4)  # stream outside the set
        with pytest.raises(mg._abi.MRGError):
            mg._abi.mrg_fill_leapfrog(ss.handle, 0, 2**40, 2**40, mg.U32, 0, 1 << 20)


def card(state, players, t, k, dtype):
    """Card k of player t, computed alone: jump t + k*players, then one step."""
    s = oracle.jump(state, t + k * players)
    z = oracle.step(s)
    if dtype == oracle.U32:
        return z
    return oracle.to_f32(z) if dtype == oracle.F32 else oracle.to_f64(z)


@pytest.mark.parametrize("players,per_player,layout,dtype",
                         [(1 << 14, 1 << 14, 0, 0), (1 << 10, 1 << 18, 1, 0),
                          (12345, 6789, 0, 1), (1 << 20, 100, 1, 2), (1 << 24, 5, 0, 0),
                          ((1 << 22) + 3, 48, 0, 2)],
                         ids=["rows-2^28-u32", "in-order-2^28-u32", "rows-ragged-f32",
                              "in-order-f64", "rows-5-cards-u32", "rows-48-cards-f64"])
def test_leapfrog_large_sampled(mg, players, per_player, layout, dtype):
    say("leapfrog large", players, per_player, layout, dtype)
    rng = np.random.default_rng(17)
    with mg.StreamSet(1, master_seed=MASTER) as ss:
        st = states_of(ss)[0]
        out = host(ss.fill_leapfrog(0, players, per_player, dtype, layout))
        rows = out if layout == 0 else out.T  # [player, card] view
        picks = [(0, 0), (players - 1, per_player - 1), (players - 1, 0), (0, per_player - 1)]
        picks += [(int(rng.integers(players)), int(rng.integers(per_player))) for _ in range(150)]
        for t, k in picks:
            assert rows[t, k] == card(st, players, t, k, dtype), (t, k)
        # the first and last thousand outputs of the stream, in order:
        # output i is card i // players of player i % players
        n = players * per_player
        head, _ = oracle.fill(st, 1000, dtype)
        i = np.arange(1000)
        assert np.array_equal(rows[i % players, i // players], head[0])
        tail, end = oracle.fill(oracle.jump(st, n - 1000), 1000, dtype)
        i = np.arange(n - 1000, n)
        assert np.array_equal(rows[i % players, i // players], tail[0])
        assert np.array_equal(states_of(ss)[0], end[0])
        if dtype != 0:
            assert np.all(out > 0) and np.all(out < 1)


def test_random_spacing_set_with_jumps_batches_and_leapfrog(mg):
    """A random-spacing set is an ordinary stream set: substream jumps, a
    batch over it and a leapfrog deal of one of its streams all match the
    oracle run on the expanded states."""
    import torch
    say("random spacing: jumps, batch, leapfrog")
    master, S = 0xC0FFEE, 200
    with mg.StreamSet(S, master_seed=master, spacing="random") as ss:
        st = oracle.random_spacing_states(master, 0, S)
        ss.jump_substreams(3)
        st = oracle.jump_many(st, 3 * 2**76)
        assert np.array_equal(states_of(ss), st)
        # a batch of three plain requests
        specs = [(0, 50, 5000, 0), (50, 100, 300, 2), (150, 50, 4097, 1)]
        outs, rows = [], []
        for first, k, n, dt in specs:
            t = torch.empty((k, n), dtype=mg.torch_dtype(dt), device="cuda")
            outs.append(t)
            rows.append((first, k, n, 0, t.data_ptr(), dt, 0))
        b = mg.Batch(ss, rows)
        b.run()
        for (first, k, n, dt), t in zip(specs, outs):
            want, end = oracle.fill(st[first:first + k], n, dt)
            assert np.array_equal(host(t).view(np.uint8), want.view(np.uint8)), (first, k, n)
            st[first:first + k] = end
        b.close()
        assert np.array_equal(states_of(ss), st)
        # leapfrog of stream 7
        cards = host(ss.fill_leapfrog(7, 33, 70, mg.U32, mg.STREAM_MAJOR))
        want, end = oracle.leapfrog(st[7], 33, 70, oracle.U32, oracle.STREAM_MAJOR)
        assert np.array_equal(cards, want)
        assert np.array_equal(states_of(ss)[7], end)


def test_random_leapfrog_sweep(mg):
    """Seeded random deals against the oracle: players and cards from 1 to
    thousands (fewer and more than 64 cards), both layouts, every dtype, both
    engines, output pointers off their lines, guard words untouched, and two
    deals in a row continuing the stream."""
    import torch
    rng = np.random.default_rng(2003)
    old = mg.mrg_config_get("engine")
    try:
        for case in range(80):
            engine = int(rng.integers(2))
            mg.mrg_config_set("engine", engine)
            players = int(np.exp(rng.uniform(0, np.log(5000))))
            per_player = int(np.exp(rng.uniform(0, np.log(3000))))
            if players * per_player > 3_000_000:
                per_player = max(1, 3_000_000 // players)
            dt = int(rng.integers(3))
            layout = int(rng.integers(2))
            es = 8 if dt == 2 else 4
            off = int(rng.integers(0, 128 // es))
            say("leapfrog sweep", case, players, per_player, dt, layout, off, engine)
            with mg.StreamSet(4, master_seed=case) as ss:
                st = states_of(ss)[2]
                guard = 16
                size = players * per_player
                buf = torch.zeros(size + off + 2 * guard, dtype=mg.torch_dtype(dt), device="cuda")
                for rep in range(2):
                    buf.zero_()
                    view = buf[guard + off:guard + off + size]
                    ss.fill_leapfrog(2, players, per_player, dt, layout, out=view)
                    h = host(buf)
                    want, st = oracle.leapfrog(st, players, per_player, dt, layout)
                    assert np.array_equal(h[guard + off:guard + off + size].view(np.uint8),
                                          want.reshape(-1).view(np.uint8)), (case, rep)
                    assert not h[:guard + off].view(np.uint8).any(), (case, rep)
                    assert not h[guard + off + size:].view(np.uint8).any(), (case, rep)
                assert np.array_equal(states_of(ss)[2], st), case
    finally:
        mg.mrg_config_set("engine", old)
