"""GPU parity of the Philox4x32-10 stream sets (the counter-based second
generator) against the CPU oracle, bit for bit: stream creation, fills in
both layouts and every dtype over ragged shapes and positions that are not
multiples of 4, unaligned output, jumps (per stream, uniform, across 2^32 and
2^64), state round trips, and what Philox sets refuse.  The oracle's round
multipliers are parity unpinned (no closed form, no known-answer file), so
these tests check that the library computes the oracle's function.
"""
import sys

import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu

KEY = 0x0123456789ABCDEF


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


def states_of(ss):
    return np.asarray(ss.get_states(), dtype=np.uint32).reshape(-1, 6)


@pytest.mark.parametrize("first,count", [(0, 1), (0, 777), (2**40 + 3, 100), (2**64 - 4, 4)])
def test_philox_streams(mg, first, count):
    with mg.StreamSet(count, master_seed=KEY, first_stream=first, generator="philox") as ss:
        assert np.array_equal(states_of(ss), oracle.philox_streams(KEY, first, count))
        assert list(ss.base_state) == [0] * 6


SHAPES = [(1, 1), (3, 5), (64, 4096), (100, 1000), (257, 33), (5, 100003), (1000, 4)]


@pytest.mark.parametrize("count,n", SHAPES, ids=["%dx%d" % s for s in SHAPES])
@pytest.mark.parametrize("layout", [0, 1], ids=["stream-major", "interleaved"])
def test_philox_fill(mg, count, n, layout):
    say("philox fill", count, n, layout)
    with mg.StreamSet(count, master_seed=KEY, generator="philox") as ss:
        st = states_of(ss)
        for dtype, first_n in ((mg.U32, 3), (mg.F32, 1), (mg.F64, 2)):
            # a short fill first, so later fills start at positions % 4 != 0
            a = host(ss.fill(first_n, dtype, layout))
            wa, st = oracle.philox_fill(st, first_n, dtype, layout)
            assert np.array_equal(a, wa)
            out = host(ss.fill(n, dtype, layout))
            want, st = oracle.philox_fill(st, n, dtype, layout)
            assert np.array_equal(out, want), dtype
            assert np.array_equal(states_of(ss), st)


def test_philox_unaligned_output_and_subrange(mg):
    import torch
    count, n = 70, 515
    with mg.StreamSet(100, master_seed=KEY, generator="philox") as ss:
        st = states_of(ss)
        buf = torch.full((count * n + 8,), 0xDEADBEEF, dtype=torch.uint32, device="cuda")
        ss.fill(n, mg.U32, mg.STREAM_MAJOR, out=buf[1:1 + count * n], first=20, count=count)
        b = host(buf)
        want, end = oracle.philox_fill(st[20:90], n, oracle.U32)
        assert np.array_equal(b[1:1 + count * n], want.reshape(-1))
        assert b[0] == 0xDEADBEEF and np.all(b[1 + count * n:] == 0xDEADBEEF)
        got = states_of(ss)
        assert np.array_equal(got[20:90], end)
        assert np.array_equal(got[:20], st[:20]) and np.array_equal(got[90:], st[90:])


def test_philox_jumps(mg):
    import torch
    with mg.StreamSet(6, master_seed=KEY, generator="philox") as ss:
        st = states_of(ss)
        ss.jump_uniform(2**32 + 5)
        st = oracle.philox_jump(st, 2**32 + 5)
        assert np.array_equal(states_of(ss), st)
        exps = [0, 1, 3, 2**40 + 1, 2**64 - 7, 2**70 + 2]  # e mod 2^64 moves the position
        words = np.array([[e & (2**64 - 1), (e >> 64) & (2**64 - 1), 0] for e in exps],
                         dtype=np.uint64)
        ss.jump(torch.from_numpy(words.reshape(-1).view(np.int64)).cuda())
        st = oracle.philox_jump(st, [e % 2**64 for e in exps])
        assert np.array_equal(states_of(ss), st)
        # a fill across position 2^64 wraps the block counter
        out = host(ss.fill(21, mg.U32))
        want, st = oracle.philox_fill(st, 21, oracle.U32)
        assert np.array_equal(out, want)
        assert np.array_equal(states_of(ss), st)


def test_philox_state_roundtrip_and_refusals(mg):
    with mg.StreamSet(4, master_seed=KEY, generator="philox") as ss:
        anything = np.array([[0, 0, 0, 0, 0, 0], [2**32 - 1] * 6, [5, 6, 7, 8, 9, 10],
                             [3, 0, 1, 0, 2, 0]], dtype=np.uint32)
        ss.set_states(anything)
        assert np.array_equal(states_of(ss), anything)
        out = host(ss.fill(9, mg.U32))
        want, _ = oracle.philox_fill(anything, 9, oracle.U32)
        assert np.array_equal(out, want)
        with pytest.raises(mg.MRGError):
            ss.jump_substreams(1)
        with pytest.raises(mg.MRGError):
            ss.fill_leapfrog(0, 4, 4)
        import torch
        buf = torch.empty(16, dtype=torch.uint32, device="cuda")
        with pytest.raises(mg.MRGError):
            mg.Batch(ss, [(0, 1, 16, 0, buf.data_ptr(), mg.U32, 0)])


def test_philox_large_sampled(mg):
    """2^20 streams x 1024 uint32 (4 GiB), sampled rows against the oracle."""
    S, n = 1 << 20, 1024
    rng = np.random.default_rng(5)
    with mg.StreamSet(S, master_seed=KEY, generator="philox") as ss:
        st = states_of(ss)
        out = host(ss.fill(n, mg.U32))
        rows = [0, S - 1] + [int(x) for x in rng.integers(0, S, 40)]
        want, _ = oracle.philox_fill(st[rows], n, oracle.U32)
        assert np.array_equal(out[rows], want)


def test_philox_random_sweep(mg):
    """Seeded random Philox fills against the oracle: arbitrary positions
    (near the 2^64 wrap too), ids and keys, row lengths from 1 to tens of
    thousands, both layouts, every dtype, sub-ranges, output pointers off
    their 16-byte and line boundaries, guard words untouched."""
    import torch
    rng = np.random.default_rng(1011)
    for case in range(60):
        total = int(np.exp(rng.uniform(0, np.log(3000))))
        first = int(rng.integers(0, total))
        count = int(rng.integers(1, total - first + 1))
        n = int(np.exp(rng.uniform(0, np.log(40000))))
        if count * n > 2_000_000:
            n = max(1, 2_000_000 // count)
        dt = int(rng.integers(3))
        layout = int(rng.integers(2))
        es = 8 if dt == 2 else 4
        off = int(rng.integers(0, 128 // es))
        say("philox sweep", case, total, first, count, n, dt, layout, off)
        st = rng.integers(0, 2**32, size=(total, 6), dtype=np.uint64).astype(np.uint32)
        if case % 3 == 0:
            st[:, 1] = 0xFFFFFFFF  # positions within 2^32 of the wrap
        with mg.StreamSet(total, master_seed=case, generator="philox") as ss:
            ss.set_states(st)
            guard = 16
            size = count * n
            buf = torch.zeros(size + off + 2 * guard, dtype=mg.torch_dtype(dt), device="cuda")
            view = buf[guard + off:guard + off + size]
            ss.fill(n, dt, layout, out=view, first=first, count=count)
            h = host(buf)
            want, end = oracle.philox_fill(st[first:first + count], n, dt, layout)
            assert np.array_equal(h[guard + off:guard + off + size].view(np.uint8),
                                  want.reshape(-1).view(np.uint8)), case
            assert not h[:guard + off].view(np.uint8).any(), case
            assert not h[guard + off + size:].view(np.uint8).any(), case
            got = states_of(ss)
            assert np.array_equal(got[first:first + count], end), case
            assert np.array_equal(got[:first], st[:first]), case
            assert np.array_equal(got[first + count:], st[first + count:]), case
