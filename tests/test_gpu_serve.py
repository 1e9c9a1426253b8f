"""GPU tests of the serving engine (continuous batching).

Each finished request must equal, bit for bit, (a) the CPU oracle for its
client's substreams and (b) the same request generated alone through the
batch kernel; substream cursors advance in admission order; admission never
exceeds the arena; outputs held in the arena block admission until released.
"""
import sys
import time

import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu

SEED = 0x5E12E


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def mg():
    import torch
    import paper_1412_8266_amd as m
    from paper_1412_8266_amd import serve  # noqa: F401
    assert torch.cuda.is_available()
    return m


def wait_all(srv, n, timeout=120.0):
    got = []
    t_end = time.time() + timeout
    while sum(len(g) for g in got) < n:
        got.append(srv.poll())
        assert time.time() < t_end, "requests did not finish"
        time.sleep(0.002)
    return np.concatenate(got)


def expected(base, first_stream, rec):
    c, k, n = int(rec["client"]), int(rec["n_streams"]), int(rec["n_per_stream"])
    s0 = oracle.stream_start(base, first_stream + c)
    sub0 = int(rec["substream0"])
    starts = np.stack([oracle.jump(s0, (sub0 + j) << 76) for j in range(k)])
    return oracle.fill(starts, n, int(rec["dtype"]))[0]


@pytest.mark.parametrize("big", [0, 64 << 10], ids=["one-class", "two-classes"])
def test_mix_equals_oracle_and_alone(mg, big):
    import torch
    from paper_1412_8266_amd.serve import Server
    say("serve mix", big)
    base = oracle.seed_from_master(SEED)
    first = 1000
    rng = np.random.default_rng(SEED)
    srv = Server(64, SEED, 256 << 20, first_stream=first, max_inflight=3, max_batch=16,
                 big_request_bytes=big)
    subs = []
    for i in range(150):
        c = int(rng.integers(0, 64))
        k = int(rng.integers(1, 40))
        n = int(rng.integers(1, 6000))
        dt = int(rng.integers(0, 3))
        subs.append(srv.submit(c, k, n, dt))
    recs = wait_all(srv, len(subs))
    assert sorted(int(t) for t in recs["ticket"]) == sorted(subs)
    # cursors: each client's requests take consecutive, disjoint runs of
    # substreams (in admission order, which size classes may reorder)
    for c in np.unique(recs["client"]):
        r = np.sort(recs[recs["client"] == c], order="substream0")
        assert int(r["substream0"][0]) == 0
        assert np.array_equal(r["substream0"][1:], np.cumsum(r["n_streams"])[:-1])
    if big:
        nb = recs["n_streams"] * recs["n_per_stream"] * np.where(recs["dtype"] == 2, 8, 4)
        assert (nb >= big).any() and (nb < big).any()  # both classes ran
    # a client set for running single requests alone through the batch kernel
    ss = mg.StreamSet(64, seed=[int(x) for x in base], first_stream=first)
    for rec in recs[:: max(1, len(recs) // 40)]:
        got = srv.output(rec)
        want = expected(base, first, rec)
        assert np.array_equal(got.view(np.uint8), want.view(np.uint8)), rec
        k, n, dt = int(rec["n_streams"]), int(rec["n_per_stream"]), int(rec["dtype"])
        t = torch.empty((k, n), dtype=mg.torch_dtype(dt), device="cuda")
        b = mg.Batch(ss, [(int(rec["client"]), k, n, int(rec["substream0"]), t.data_ptr(), dt,
                           mg.REQ_SUBSTREAMS)])
        b.run()
        alone = t.cpu().numpy()
        assert np.array_equal(alone.view(np.uint8), got.view(np.uint8))
        b.close()
    for rec in recs:
        srv.release(int(rec["ticket"]))
    assert srv.stats()["arena_used"] == 0
    srv.close()
    ss.close()


def test_admission_respects_arena(mg):
    from paper_1412_8266_amd.serve import Server
    say("serve admission")
    arena = 48 << 20
    srv = Server(16, SEED + 1, arena, max_inflight=4, max_batch=8, auto_release=True)
    rng = np.random.default_rng(SEED + 1)
    total = 0
    n_req = 120
    for i in range(n_req):
        k = int(rng.integers(1, 64))
        n = int(rng.integers(1000, 60000))
        total += k * n * 4
        srv.submit(int(rng.integers(0, 16)), k, n, 0)
    peak = 0
    got = 0
    t_end = time.time() + 120
    while got < n_req:
        st = srv.stats()
        peak = max(peak, st["arena_used"])
        assert st["arena_used"] <= arena
        got += len(srv.poll())
        assert time.time() < t_end
    assert total > 4 * arena  # the queue really had to wait for memory
    assert peak <= arena
    srv.drain(30)
    srv.close()


def test_held_outputs_block_until_released(mg):
    from paper_1412_8266_amd.serve import Server
    say("serve held outputs")
    srv = Server(4, SEED + 2, 32 << 20, max_inflight=2)
    t1 = srv.submit(0, 10, 500_000, 0)  # 20 MB
    t2 = srv.submit(1, 10, 500_000, 0)  # 20 MB: cannot fit while t1 is held
    r = wait_all(srv, 1)
    assert int(r["ticket"][0]) == t1
    with pytest.raises(mg.MRGError):
        srv.drain(0.5)
    assert srv.stats()["pending"] == 1
    srv.release(t1)
    r2 = wait_all(srv, 1)
    assert int(r2["ticket"][0]) == t2
    srv.release(t2)
    srv.close()


def test_trace_replay_and_errors(mg):
    from paper_1412_8266_amd.serve import Server
    say("serve trace")
    srv = Server(100, SEED + 3, 128 << 20, auto_release=True)
    rng = np.random.default_rng(SEED + 3)
    n = 400
    t = np.sort(rng.random(n) * 0.2)
    wall = srv.run_trace(t, rng.integers(0, 100, n), rng.integers(1, 20, n),
                         rng.integers(1, 3000, n), rng.integers(0, 3, n))
    recs = srv.poll()
    assert len(recs) == n and wall >= 0.2
    assert np.all(recs["latency_s"] > 0) and np.all(recs["queue_s"] >= 0)
    with pytest.raises(mg.MRGError):
        srv.submit(100, 1, 1, 0)  # client out of range
    with pytest.raises(mg.MRGError):
        srv.submit(0, 1 << 20, 1 << 20, 0)  # larger than the arena
    srv.close()


def test_c5_shaped_trace_sampled(mg):
    """The first 0.2 s of the C5 arrivals (50,000 clients, sizes as C4, 64 GiB
    arena) submitted at once, outputs held until the poll loop releases them.
    Every request finishes; sampled requests (first and last substream) equal
    the oracle; the arena drains to zero."""
    from paper_1412_8266_amd import workloads as wl
    from paper_1412_8266_amd.serve import Server
    say("serve C5-shaped")
    arr = wl.c5_arrivals()
    keep = arr.t < 0.2
    k, n, dt = arr.req.n_streams[keep], arr.req.length[keep], arr.req.dtype[keep]
    client = arr.client[keep]
    base = oracle.seed_from_master(wl.MASTER_SEED)
    srv = Server(wl.C5_CLIENTS, wl.MASTER_SEED, wl.C5_ARENA_BYTES)
    tickets = [srv.submit(int(c), int(a), int(b), int(d)) for c, a, b, d in zip(client, k, n, dt)]
    sample = set(tickets[::40])
    kept, done = [], 0
    t_end = time.time() + 120
    while done < len(tickets):
        for rec in srv.poll():
            done += 1
            nbytes = int(rec["n_streams"]) * int(rec["n_per_stream"]) * (8 if rec["dtype"] == 2 else 4)
            if int(rec["ticket"]) in sample and int(rec["n_per_stream"]) <= (1 << 18) \
                    and nbytes <= (64 << 20):
                kept.append((rec.copy(), srv.output(rec)))
            srv.release(int(rec["ticket"]))
        assert time.time() < t_end, "requests did not finish"
        time.sleep(0.001)
    assert srv.stats()["arena_used"] == 0
    assert len(kept) >= 20
    for rec, got in kept:
        c, kk, nn, d = int(rec["client"]), int(rec["n_streams"]), int(rec["n_per_stream"]), \
            int(rec["dtype"])
        s0 = oracle.stream_start(base, c)
        for j in sorted({0, kk - 1}):
            st = oracle.jump(s0, (int(rec["substream0"]) + j) << 76)[None, :]
            want = oracle.fill(st, nn, d)[0][0]
            assert np.array_equal(got[j].view(np.uint8), want.view(np.uint8)), (rec, j)
    srv.close()
