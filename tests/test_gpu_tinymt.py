"""GPU parity of the TinyMT32 stream sets (the sec. 4.2 hybrid: a parameter
set shared by a group of streams, sub-streams 2^64 apart by sequence
splitting) against the CPU oracle, bit for bit: the device parameter search
(every candidate's linear complexity, characteristic polynomial and accept
decision; the accepted sets in order), stream placement over ragged ranges,
fills in both layouts and every dtype over ragged shapes, chained fills,
sub-ranges and unaligned output with guard words, jumps (per stream and
uniform, exponents up to 2^192), state round trips, what TinyMT sets refuse,
and the 2^20 x 4096 workload sampled.  TinyMT's exact output is parity
unpinned (no known-answer file); these tests check that the library computes
the oracle's function.
"""
import sys
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu

MASTER = 0x5EED0123456789AB


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


_SETS = {}


def oracle_sets(master, count):
    """Parameter sets 0 .. count-1 of the oracle's search: candidates tested
    in parallel threads (each call is the oracle's own test), accepted ones
    taken in candidate order."""
    key = master
    have = _SETS.get(key, (np.zeros((0, 3), np.uint32), np.zeros(0, np.uint64), 0))
    P, C, c_next = have
    if len(P) >= count:
        return P[:count], C[:count]
    P, C = list(P), list(C)
    with ThreadPoolExecutor(16) as ex:
        while len(P) < count:
            batch = range(c_next, c_next + 4096)
            cands = [oracle.tmt_candidate(master, c) for c in batch]
            oks = list(ex.map(oracle.tmt_params_ok, cands))
            for c, p, ok in zip(batch, cands, oks):
                if ok:
                    P.append(p)
                    C.append(c)
            c_next += 4096
    P = np.array(P, dtype=np.uint32).reshape(-1, 3)
    C = np.array(C, dtype=np.uint64)
    _SETS[key] = (P, C, c_next)
    return P[:count], C[:count]


def test_candidate_flags_and_polynomials(mg):
    c0, n = 1000, 768
    flags, phi = mg.tinymt_test_candidates(MASTER, c0, n, with_phi=True)
    f = host(flags).view(np.uint32)
    ph = host(phi).view(np.uint32)
    kept = 0
    for i in range(n):
        p = oracle.tmt_candidate(MASTER, c0 + i)
        L, w = oracle.tmt_charpoly(p)
        ok = oracle.tmt_params_ok(p)
        assert f[i] & 0xFFFF == L, i
        assert (f[i] >> 16) == ok, i
        got = sum(int(x) << (32 * k) for k, x in enumerate(ph[i]))
        assert got == (w if L == 127 else 0), i
        kept += ok
    assert kept > 0


@pytest.mark.parametrize("master,count", [(MASTER, 12), (7, 1), (2**64 - 1, 40)])
def test_search_matches_oracle(mg, master, count):
    P, C = mg.tinymt_search(master, count)
    wP, wC = oracle.tmt_search(master, count)
    assert np.array_equal(P, wP)
    assert np.array_equal(C, wC)


STREAMS = [(64, 0, 256), (7, 3, 50), (1000, 2500, 1000), (1 << 20, 0, 300), (1, 5, 9),
           (256, 2**33 - 40, 100)]


@pytest.mark.parametrize("per,first,count", STREAMS, ids=["%d/%d/%d" % s for s in STREAMS])
def test_streams_match_oracle(mg, per, first, count):
    say("tinymt streams", per, first, count)
    q0, ql = first // per, (first + count - 1) // per
    if ql < 64:
        P, _ = oracle.tmt_search(MASTER, ql + 1)
        with mg.StreamSet(count, master_seed=MASTER, first_stream=first, generator="tinymt",
                          per_param=per) as ss:
            assert np.array_equal(states_of(ss), oracle.tmt_streams(MASTER, per, first, count, P))
            assert ss.tinymt_info[:3] == (per, q0, ql - q0 + 1)
    # parameter sets given by the caller (a parameter file), starting below
    # q0; three accepted sets repeated over the range
    P3, _ = oracle.tmt_search(MASTER, 3)
    pf = max(q0 - 1, 0)
    k = ql - pf + 1
    given = np.concatenate([P3] * (k // 3 + 1))[:k]
    with mg.StreamSet(count, master_seed=MASTER, first_stream=first, generator="tinymt",
                      per_param=per, params=given, params_first=pf) as ss:
        want = oracle.tmt_streams(MASTER, per, first, count, given, pf)
        assert np.array_equal(states_of(ss), want)


SHAPES = [(1, 1), (3, 5), (64, 4096), (100, 1000), (257, 33), (5, 100003), (1000, 4), (130, 64)]


@pytest.mark.parametrize("count,n", SHAPES, ids=["%dx%d" % s for s in SHAPES])
@pytest.mark.parametrize("layout", [0, 1], ids=["stream-major", "interleaved"])
def test_fill_matches_oracle(mg, count, n, layout):
    say("tinymt fill", count, n, layout)
    per = 64
    P, _ = oracle.tmt_search(MASTER, (count - 1) // per + 1)
    with mg.StreamSet(count, master_seed=MASTER, generator="tinymt", per_param=per) as ss:
        st = states_of(ss)
        for dtype, first_n in ((mg.U32, 3), (mg.F32, 1), (mg.F64, 2)):
            a = host(ss.fill(first_n, dtype, layout))
            wa, st = oracle.tmt_fill(st, first_n, dtype, layout, P)
            assert np.array_equal(a, wa)
            out = host(ss.fill(n, dtype, layout))
            want, st = oracle.tmt_fill(st, n, dtype, layout, P)
            assert np.array_equal(out.view(np.uint8), want.view(np.uint8)), dtype
            assert np.array_equal(states_of(ss), st)


@pytest.mark.parametrize("tile", [128, 256])
def test_fill_tiles_subrange_unaligned_with_guards(mg, tile):
    import torch
    per, count, n = 32, 70, 515
    P, _ = oracle.tmt_search(MASTER, 4)
    mg.mrg_config_set("tile_bytes", tile)
    try:
        with mg.StreamSet(128, master_seed=MASTER, generator="tinymt", per_param=per) as ss:
            st = states_of(ss)
            for dtype, es in ((mg.U32, 4), (mg.F64, 8)):
                tdt = torch.uint32 if es == 4 else torch.float64
                buf = torch.full((count * n + 8,), 7, dtype=tdt, device="cuda")
                guard = host(buf).copy()
                ss.fill(n, dtype, mg.STREAM_MAJOR, out=buf[1:1 + count * n], first=20, count=count)
                b = host(buf)
                want, end = oracle.tmt_fill(st[20:90], n, dtype, 0, P)
                assert np.array_equal(b[1:1 + count * n].view(np.uint8), want.reshape(-1).view(np.uint8))
                assert b[0] == guard[0] and np.array_equal(b[1 + count * n:], guard[1 + count * n:])
                st[20:90] = end
                assert np.array_equal(states_of(ss), st)
    finally:
        mg.mrg_config_set("tile_bytes", 0)


def test_chained_fills_equal_one_fill(mg):
    per, count = 16, 40
    P, _ = oracle.tmt_search(MASTER, 3)
    with mg.StreamSet(count, master_seed=MASTER, generator="tinymt", per_param=per) as a, \
            mg.StreamSet(count, master_seed=MASTER, generator="tinymt", per_param=per) as b:
        whole = host(a.fill(3000, mg.U32))
        parts = [host(b.fill(k, mg.U32)) for k in (1, 999, 31, 1969)]
        assert np.array_equal(whole, np.concatenate(parts, axis=1))
        assert np.array_equal(states_of(a), states_of(b))


def test_jumps_match_oracle(mg):
    import torch
    rng = np.random.default_rng(11)
    per, count = 50, 120
    P, _ = oracle.tmt_search(MASTER, 3)
    exps = [0, 1, 2, 127, 1 << 64, (1 << 127) - 1, 1 << 127, (1 << 128) - 1]
    exps += [int(rng.integers(0, 2**63)) << 65 | int(rng.integers(0, 2**63)) for _ in range(count - len(exps))]
    big = [(1 << 191) | 12345, (1 << 150) + 7]  # past 2^128: the oracle's at e mod (2^127 - 1)
    exps[-len(big):] = big
    words = np.array([[e & (2**64 - 1), (e >> 64) & (2**64 - 1), e >> 128] for e in exps],
                     dtype=np.uint64)
    with mg.StreamSet(count, master_seed=MASTER, generator="tinymt", per_param=per) as ss:
        st = states_of(ss)
        ss.jump(torch.from_numpy(words.view(np.int64)).cuda())
        got = states_of(ss)
        for i, e in enumerate(exps):
            p = P[st[i, 4]]
            er = e if e < 1 << 128 else e % ((1 << 127) - 1)
            assert np.array_equal(got[i, :4], oracle.tmt_jump(st[i, :4], p, er)), (i, e)
            assert got[i, 4] == st[i, 4] and got[i, 5] == 0
        # a uniform jump over a sub-range
        ss.jump_uniform(10**30 + 17, first=30, count=60)
        got2 = states_of(ss)
        for i in range(count):
            want = oracle.tmt_jump(got[i, :4], P[got[i, 4]], 10**30 + 17) if 30 <= i < 90 else got[i, :4]
            assert np.array_equal(got2[i, :4], want), i
        # the fill after a jump continues from the jumped state
        out = host(ss.fill(77, mg.U32))
        want, _ = oracle.tmt_fill(got2, 77, oracle.U32, 0, P)
        assert np.array_equal(out, want)


def test_state_round_trip_and_checks(mg):
    per, count = 10, 25
    with mg.StreamSet(count, master_seed=MASTER, generator="tinymt", per_param=per) as ss:
        st = states_of(ss)
        ss.fill(100, mg.U32)
        ss.set_states(st)
        assert np.array_equal(states_of(ss), st)
        bad = st.copy()
        bad[3, 4] += 1  # another stream's parameter set
        with pytest.raises(mg.MRGError):
            ss.set_states(bad)
        bad = st.copy()
        bad[4, :4] = [0x80000000, 0, 0, 0]  # zero 127-bit state
        with pytest.raises(mg.MRGError):
            ss.set_states(bad)
        assert np.array_equal(states_of(ss), st)


def test_refusals(mg):
    import torch
    with mg.StreamSet(64, master_seed=MASTER, generator="tinymt", per_param=64) as ss:
        with pytest.raises(mg.MRGError):
            ss.jump_substreams(1)
        out = torch.empty(64, dtype=torch.uint32, device="cuda")
        with pytest.raises(mg.MRGError):
            ss.fill_leapfrog(0, 8, 8, mg.U32, out=out)
        with pytest.raises(mg.MRGError):
            mg.Batch(ss, [(0, 1, 64, 0, out.data_ptr(), mg.U32, 0)])
    with pytest.raises(mg.MRGError):  # sets that do not cover the streams
        P, _ = oracle.tmt_search(MASTER, 2)
        mg.StreamSet(100, master_seed=MASTER, generator="tinymt", per_param=10, params=P)
    with pytest.raises(mg.MRGError):  # a parameter set without full period
        rej = next(oracle.tmt_candidate(MASTER, c) for c in range(1000)
                   if not oracle.tmt_params_ok(oracle.tmt_candidate(MASTER, c)))
        mg.StreamSet(8, master_seed=MASTER, generator="tinymt", per_param=8, params=[rej])
    with pytest.raises(mg.MRGError):
        mg.StreamSet(8, master_seed=MASTER, generator="tinymt", per_param=0)


def test_full_workload_sampled(mg):
    """2^20 streams x 4096 uint32, 256 streams per parameter set (4096 sets
    from the device search): the search in full against the oracle's, then
    sampled rows in both layouts and the advanced states."""
    import torch
    S, n, per = 1 << 20, 4096, 256
    P, _ = oracle_sets(MASTER, S // per)
    say("tinymt full workload: oracle sets ready")
    with mg.StreamSet(S, master_seed=MASTER, generator="tinymt", per_param=per) as ss:
        gP, _ = mg.tinymt_search(MASTER, S // per)
        assert np.array_equal(gP, P)
        rng = np.random.default_rng(12)
        rows = np.unique(np.concatenate([[0, 1, 255, 256, S - 1], rng.integers(0, S, 600)]))
        st = np.concatenate([oracle.tmt_streams(MASTER, per, int(g), 1, P) for g in rows])
        assert np.array_equal(states_of(ss)[rows], st)
        out = ss.fill(n, mg.U32)
        torch.cuda.synchronize()
        idx = torch.from_numpy(rows.astype(np.int64)).cuda()
        got = host(out.index_select(0, idx))
        want, st2 = oracle.tmt_fill(st, n, oracle.U32, 0, P)
        assert np.array_equal(got, want)
        del out
        out = ss.fill(n, mg.U32, mg.INTERLEAVED)
        got = host(out.index_select(1, idx)).T
        want, st3 = oracle.tmt_fill(st2, n, oracle.U32, 0, P)
        assert np.array_equal(got, want)
        assert np.array_equal(states_of(ss)[rows], st3)
