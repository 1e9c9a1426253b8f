"""The public device headers at run time: user kernels written against
include/mrg32k3a_device.h and include/philox_device.h alone (built without
the library's compile flags, as a user would build them) draw from the streams
of library-created sets, and every draw equals the oracle's: MRG32k3a
substreams and jumps under both engines, uint32/binary32/binary64 draws in
one sequence; Philox draws across a jump and a stored position."""
import ctypes
import os
import sys

import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu

LIB = os.path.join(os.path.dirname(os.path.abspath(__file__)), "device_api", "libuser_kernels.so")
P, u64 = ctypes.c_void_p, ctypes.c_uint64


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def user():
    import torch
    assert torch.cuda.is_available()
    if not os.path.exists(LIB):
        pytest.fail("user-kernel library not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(LIB)
    lib.user_mrg_draws.argtypes = [P, u64, u64, P, u64, u64, ctypes.c_int, P, P, P]
    lib.user_philox_draws.argtypes = [P, u64, ctypes.c_int, u64, P, P, P]
    return lib


@pytest.fixture(scope="module")
def mg():
    import paper_1412_8266_amd as m
    return m


@pytest.mark.parametrize("engine", [1, 0], ids=["f64-engine", "int-engine"])
@pytest.mark.parametrize("e", [0, 1000, 2**63 + 12345])
def test_mrg_stream_substream_jump_draws(user, mg, engine, e):
    import torch
    count, base = 300, 5
    with mg.StreamSet(8, master_seed=0xC0FFEE) as ss:
        st = np.asarray(ss.get_states(), dtype=np.uint32).reshape(-1, 6)[base]
        u = torch.zeros(count, dtype=torch.int32, device="cuda")
        f = torch.zeros(count, dtype=torch.float32, device="cuda")
        d = torch.zeros(count, dtype=torch.float64, device="cuda")
        say("device api mrg", engine, e)
        rc = user.user_mrg_draws(ss.states_ptr, 8, base, ss.tables_ptr, e, count,
                                 engine, u.data_ptr(), f.data_ptr(), d.data_ptr())
        assert rc == 0
        torch.cuda.synchronize()
        # thread i: i * 2^76 + e values past the base stream's state
        i = np.arange(count, dtype=np.uint64)
        words = np.stack([np.full(count, e, dtype=np.uint64), i << np.uint64(12),
                          i >> np.uint64(52)], 1)
        starts = oracle.jump_many_words(np.repeat(st[None], count, 0), words)
        zu, _ = oracle.fill(starts, 3, oracle.U32)
        zf, _ = oracle.fill(starts, 3, oracle.F32)
        zd, _ = oracle.fill(starts, 3, oracle.F64)
        assert np.array_equal(u.cpu().numpy().view(np.uint32), zu[:, 0])
        assert np.array_equal(f.cpu().numpy().view(np.uint32), zf[:, 1].view(np.uint32))
        assert np.array_equal(d.cpu().numpy().view(np.uint64), zd[:, 2].view(np.uint64))
        # the user kernel wrote no state back
        assert np.array_equal(np.asarray(ss.get_states(), dtype=np.uint32).reshape(-1, 6)[base], st)


@pytest.mark.parametrize("k", [1, 3, 9])
def test_philox_stream_draws_jump_and_store(user, mg, k):
    import torch
    S, e = 777, 2**40 + 3
    with mg.StreamSet(S, master_seed=0xBEEF, generator="philox") as ss:
        st = np.asarray(ss.get_states(), dtype=np.uint32).reshape(-1, 6)
        if k == 9:  # arbitrary positions, some near the 2^64 wrap
            rng = np.random.default_rng(9)
            st[:, 0] = rng.integers(0, 2**32, S, dtype=np.uint64).astype(np.uint32)
            st[:, 1] = np.where(np.arange(S) % 2 == 0, 0xFFFFFFFF, 7).astype(np.uint32)
            ss.set_states(st)
        u = torch.zeros(S * k, dtype=torch.int32, device="cuda")
        f = torch.zeros(S, dtype=torch.float32, device="cuda")
        d = torch.zeros(S, dtype=torch.float64, device="cuda")
        say("device api philox", k)
        rc = user.user_philox_draws(ss.states_ptr, S, k, e, u.data_ptr(), f.data_ptr(),
                                    d.data_ptr())
        assert rc == 0
        torch.cuda.synchronize()
        want_u, mid = oracle.philox_fill(st, k, oracle.U32)
        assert np.array_equal(u.cpu().numpy().view(np.uint32).reshape(S, k), want_u)
        mid = oracle.philox_jump(mid, e)
        want_f, mid2 = oracle.philox_fill(mid, 1, oracle.F32)
        want_d, end = oracle.philox_fill(mid2, 1, oracle.F64)
        assert np.array_equal(f.cpu().numpy().view(np.uint32), want_f[:, 0].view(np.uint32))
        assert np.array_equal(d.cpu().numpy().view(np.uint64), want_d[:, 0].view(np.uint64))
        assert np.array_equal(np.asarray(ss.get_states(), dtype=np.uint32).reshape(-1, 6), end)
