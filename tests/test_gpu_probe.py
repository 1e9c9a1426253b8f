"""The store-only bandwidth probes write exactly the bytes they are given, in
the documented geometry (they time the fills' store patterns in bench.py)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mg():
    import torch
    import paper_1412_8266_amd as m
    assert torch.cuda.is_available()
    return m


def test_stream_probe_covers_every_word(mg):
    import torch
    buf = torch.zeros(4 * 1000 + 4, dtype=torch.int32, device="cuda")
    mg.write_probe(buf[:4000], 0)
    torch.cuda.synchronize()
    h = buf.cpu().numpy().view(np.uint32)
    i = np.arange(1000, dtype=np.uint64)
    tag = ((i % 256) * np.uint64(0x9E3779B9)) & np.uint64(0xFFFFFFFF)
    want = np.stack([tag, i & np.uint64(0xFFFFFFFF), tag ^ np.uint64(1), i >> np.uint64(32)], 1)
    assert np.array_equal(h[:4000].reshape(1000, 4), want.astype(np.uint32))
    assert not h[4000:].any()


@pytest.mark.parametrize("pattern", [1, 3], ids=["two-lines", "single-lines"])
def test_pieces_probe_geometry(mg, pattern):
    import torch
    groups = 3
    buf = torch.zeros(groups * 65536 // 4 + 32, dtype=torch.int32, device="cuda")
    mg.write_probe(buf[:groups * 65536 // 4], pattern)
    torch.cuda.synchronize()
    h = buf.cpu().numpy().view(np.uint32)
    # word offset of (group, row t, member g, piece h, 16-byte column q)
    v = h[:groups * 65536 // 4].reshape(groups, 4, 16, 8, 8, 4)
    gr, t, g, fl, q = np.meshgrid(np.arange(groups), np.arange(4), np.arange(16), np.arange(8),
                                  np.arange(8), indexing="ij")
    assert np.array_equal(v[..., 0], gr)
    assert np.array_equal(v[..., 1], fl)
    assert np.array_equal(v[..., 2], 16 * t + g)
    assert np.array_equal(v[..., 3], q)
    assert not h[groups * 65536 // 4:].any()


def test_runs_probe_geometry(mg):
    import torch
    groups = 3
    buf = torch.zeros(groups * 65536 // 4 + 32, dtype=torch.int32, device="cuda")
    mg.write_probe(buf[:groups * 65536 // 4], 2)
    torch.cuda.synchronize()
    h = buf.cpu().numpy().view(np.uint32)
    # word offset of (group, member segment, line p, 16-byte column c): lane 8p + c
    v = h[:groups * 65536 // 4].reshape(groups, 64, 8, 8, 4)
    gr, _, p, c = np.meshgrid(np.arange(groups), np.arange(64), np.arange(8), np.arange(8),
                              indexing="ij")
    assert np.array_equal(v[..., 0], gr)
    assert np.array_equal(v[..., 1], 8 * p + c)
    assert np.all(v[..., 2] == 0x5A5A) and np.all(v[..., 3] == 0xA5A5)
    assert not h[groups * 65536 // 4:].any()
