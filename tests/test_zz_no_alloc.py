"""The batch entry point that allocates nothing, against the one that does.

mrg_batch_run_noalloc plans and runs a batch out of a fixed device array.  Its
outputs and end states must equal, bit for bit, those of mrg_batch_create +
mrg_batch_run on an identical stream set, over two calls in a row (the second
smaller, so it runs over what the first left in the array), and equal the
oracle's; a batch too large for the array is refused before anything runs.
Everything goes through the C ABI (ctypes).
"""
import sys

import numpy as np
import pytest

import oracle
from paper_1412_8266_amd import workloads as wl

pytestmark = pytest.mark.gpu

SEED = 0x0A110C
S = 4096


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def mg():
    import torch
    import paper_1412_8266_amd as m
    assert torch.cuda.is_available()
    return m


def requests(rng, n_plain, max_k, max_n, sub_stream):
    """Plain requests on contiguous streams [0, ...) (below sub_stream) and
    two substream requests on stream sub_stream, which no plain request
    advances.  Returns specs (first, count, n, substream0, dtype, flags)."""
    specs, first = [], 0
    while len(specs) < n_plain:
        k = int(wl.log_uniform_int(rng, max_k, 1)[0])
        n = int(wl.log_uniform_int(rng, max_n, 1)[0])
        if first + k + 5 > sub_stream:
            break
        specs.append((first, k, n, 0, int(rng.integers(0, 3)), 0))
        first += k
    specs.append((first, 5, 40000, 0, 0, 0))  # streams of several 64 KiB segments
    specs.append((first + 5, 0, 5, 0, 0, 0))  # empty requests are skipped
    for sub0, k, n, dt in ((7, 40, 700, 1), (1 << 40, 3, 9000, 2)):
        specs.append((sub_stream, k, n, sub0, dt, 1))
    return specs


def outputs(mg, specs):
    import torch
    outs = [torch.empty((k, n), dtype=mg.torch_dtype(dt), device="cuda")
            for (_, k, n, _, dt, _) in specs]
    rows = [(f, k, n, s0, t.data_ptr() if t.numel() else 0, dt, fl)
            for (f, k, n, s0, dt, fl), t in zip(specs, outs)]
    return outs, rows


def host(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy()


def expected(specs, states):
    """Oracle outputs of every request from the given start states, and the
    end states (plain requests advance their streams)."""
    want, end = [], states.copy()
    for (f, k, n, s0, dt, fl) in specs:
        if k == 0 or n == 0:
            want.append(None)
            continue
        if fl:
            starts = np.stack([oracle.jump(states[f], (s0 + j) << 76) for j in range(k)])
            out, _ = oracle.fill(starts, n, dt)
        else:
            out, end[f:f + k] = oracle.fill(states[f:f + k], n, dt)
        want.append(out)
    return want, end


@pytest.mark.parametrize("cfg", [dict(segment_bytes=16 * 1024),
                                 dict(segment_bytes=16 * 1024, schedule=2, waves_per_cu=4),
                                 dict()], ids=["small-seg", "static", "default"])
def test_noalloc_equals_batch_run_twice(mg, cfg):
    import torch
    abi = mg._abi
    stream = torch.cuda.current_stream().cuda_stream
    rng = np.random.default_rng(SEED)
    a = mg.StreamSet(S, master_seed=wl.MASTER_SEED)   # mrg_batch_create + mrg_batch_run
    b = mg.StreamSet(S, master_seed=wl.MASTER_SEED)   # mrg_batch_run_noalloc
    c = mg.batch_config(**cfg)
    # the second call is the smaller one: fewer requests, shorter streams
    for call, (n_plain, max_k, max_n) in enumerate(((40, 200, 20000), (6, 30, 5000))):
        specs = requests(rng, n_plain, max_k, max_n, S - 1)
        before = a.get_states()
        assert np.array_equal(before, b.get_states())
        outs_a, rows_a = outputs(mg, specs)
        outs_b, rows_b = outputs(mg, specs)
        arr_a, arr_b = abi.make_requests(rows_a), abi.make_requests(rows_b)
        say("call %d (%s): %d requests, %d samples" % (
            call, cfg, len(specs), sum(k * n for (_, k, n, _, _, _) in specs)))
        h = abi.mrg_batch_create(a.handle, arr_a, len(rows_a), c)
        info = abi.mrg_batch_info(h)
        abi.mrg_batch_run(h, stream)
        abi.mrg_batch_run_noalloc(b.handle, arr_b, len(rows_b), c, stream)
        torch.cuda.synchronize()
        abi.mrg_batch_destroy(h)
        if cfg.get("segment_bytes"):
            assert info["scratch_states"] > 0  # multi-segment streams staged in the array
        for spec, ta, tb in zip(specs, outs_a, outs_b):
            assert np.array_equal(host(ta).view(np.uint8), host(tb).view(np.uint8)), spec
        assert np.array_equal(a.get_states(), b.get_states())
        want, end = expected(specs, before)
        for spec, tb, w in zip(specs, outs_b, want):
            if w is not None:
                assert np.array_equal(host(tb).view(np.uint8), w.view(np.uint8)), spec
        assert np.array_equal(b.get_states(), end)
    a.close()
    b.close()


def test_noalloc_refuses_batches_beyond_the_array(mg):
    import torch
    abi = mg._abi
    stream = torch.cuda.current_stream().cuda_stream
    # 210,000 one-value requests: 16.8 MB of request descriptors, beyond the
    # 16 MiB array
    k = 210_000
    ss = mg.StreamSet(k, master_seed=wl.MASTER_SEED)
    before = ss.get_states(0, 1000)
    out = torch.empty(k, dtype=torch.uint32, device="cuda")
    base = out.data_ptr()
    arr = abi.make_requests([(i, 1, 1, 0, base + 4 * i, 0, 0) for i in range(k)])
    with pytest.raises(abi.MRGError) as e:
        abi.mrg_batch_run_noalloc(ss.handle, arr, k, None, stream)
    assert e.value.status == -4  # MRG_ERANGE
    assert "scratch" in str(e.value)
    torch.cuda.synchronize()
    assert np.array_equal(ss.get_states(0, 1000), before)
    del out
    ss.close()
    # and a small batch on the same device still runs afterwards
    ss = mg.StreamSet(8, master_seed=wl.MASTER_SEED)
    st = ss.get_states()
    t = torch.empty((8, 100), dtype=torch.uint32, device="cuda")
    abi.mrg_batch_run_noalloc(ss.handle, abi.make_requests([(0, 8, 100, 0, t.data_ptr(), 0, 0)]),
                              1, None, stream)
    want, end = oracle.fill(st, 100, oracle.U32)
    assert np.array_equal(host(t), want)
    assert np.array_equal(ss.get_states(), end)
    ss.close()


def test_noalloc_validation_matches_batch_create(mg):
    import torch
    abi = mg._abi
    stream = torch.cuda.current_stream().cuda_stream
    ss = mg.StreamSet(16, master_seed=wl.MASTER_SEED)
    t = torch.empty((8, 10), dtype=torch.uint32, device="cuda")
    cpu = torch.empty((8, 10), dtype=torch.uint32)
    bad = [
        [(0, 8, 10, 0, t.data_ptr(), 7, 0)],                       # unknown dtype
        [(10, 8, 10, 0, t.data_ptr(), 0, 0)],                      # streams past the set
        [(0, 8, 10, 0, cpu.data_ptr(), 0, 0)],                     # host output
        [(0, 8, 10, 0, t.data_ptr(), 0, 0), (4, 4, 1, 0, t.data_ptr(), 0, 0)],  # overlap
    ]
    before = ss.get_states()
    for rows in bad:
        arr = abi.make_requests(rows)
        with pytest.raises(abi.MRGError) as e1:
            abi.mrg_batch_create(ss.handle, arr, len(rows), None)
        with pytest.raises(abi.MRGError) as e2:
            abi.mrg_batch_run_noalloc(ss.handle, arr, len(rows), None, stream)
        assert e1.value.status == e2.value.status
    torch.cuda.synchronize()
    assert np.array_equal(ss.get_states(), before)
    # no requests, or only empty ones: nothing to do
    abi.mrg_batch_run_noalloc(ss.handle, None, 0, None, stream)
    abi.mrg_batch_run_noalloc(ss.handle, abi.make_requests([(0, 0, 10, 0, 0, 0, 0)]), 1, None,
                              stream)
    assert np.array_equal(ss.get_states(), before)
    ss.close()
