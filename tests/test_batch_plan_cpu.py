"""CPU checks of the batch planner (mrg_batch_plan_groups): how requests are
cut into work items and grouped into launches, computed on the host alone.
The GPU tests check what the launches write; these check the plan itself."""
import numpy as np
import pytest

import paper_1412_8266_amd as mg
from paper_1412_8266_amd import workloads as wl

NONE = 2**64 - 1
CHUNK_BYTES = 64 * 1024  # values per wave_fill chunk: 64 lanes x 1 KiB of output


def es(dt):
    return 8 if dt == 2 else 4


def expected_items(k, n, dt, seg_bytes=256 << 10, wave_min=16 << 10):
    """Work items of one request under the documented decomposition."""
    e = es(dt)
    if n * e < wave_min:  # row items: blocks of 64 streams, about 128 KiB per item
        spi = max(1, min(16, (128 << 10) // (64 * n * e)))
        return -(-(-(-k // 64)) // spi)
    chunk = CHUNK_BYTES // e
    seg = max(chunk, seg_bytes // e // chunk * chunk)
    segs = -(-n // seg)
    if segs == 1:
        spi = max(1, min(seg // n, 1 << 20))
        return -(-k // spi)
    return k * segs


def test_small_plan_is_as_documented():
    rows = [(0, 100, 50, 0, 0, mg.U32, 0),        # rows of 200 B: row items
            (100, 10, 5000, 0, 0, mg.F64, 0),     # 40,000 B: wave items, streams packed
            (110, 3000, 2, 0, 0, mg.F32, 0),      # rows of 8 B: row items, 16 blocks each
            (3110, 1, 1 << 20, 0, 0, mg.U32, 0),  # one long stream: 16 segments
            (3111, 0, 5, 0, 0, mg.U32, 0)]        # empty
    groups, pos, items = mg.batch_plan_groups(rows)
    assert items == [expected_items(k, n, dt) for _, k, n, _, _, dt, _ in rows[:4]] + [0]
    assert items == [1, 2, 3, 16, 0]
    # wave groups least output first; the first also holds every row request
    assert [(g["dtype"], g["rows"]) for g in groups] == [(mg.F64, True), (mg.U32, False)]
    assert groups[0]["requests"] == 3 and groups[0]["row_items"] == 4 and groups[0]["items"] == 6
    assert groups[1]["requests"] == 1 and groups[1]["items"] == 16 and groups[1]["row_items"] == 0
    # row requests first, the larger items first, then the group's wave request
    assert pos == [0, 2, 1, 3, NONE]


def test_rows_only_and_waves_only():
    rows = [(0, 70, 10, 0, 0, mg.U32, 0), (70, 5, 10, 0, 0, mg.F64, 0)]
    groups, pos, items = mg.batch_plan_groups(rows)
    assert len(groups) == 1 and groups[0]["rows"] and groups[0]["row_items"] == sum(items)
    rows = [(0, 3, 1 << 16, 0, 0, mg.F32, 0), (3, 3, 1 << 15, 0, 0, mg.U32, 0)]
    groups, pos, items = mg.batch_plan_groups(rows)
    assert [g["rows"] for g in groups] == [False, False]
    assert [g["dtype"] for g in groups] == [mg.U32, mg.F32]  # 384 KiB before 768 KiB


@pytest.mark.parametrize("cfg", [None, dict(wave_min_bytes=64 << 10, segment_bytes=1 << 20),
                                 dict(wave_min_bytes=4 << 10, segment_bytes=64 << 10)])
def test_c4_mix_plan(cfg):
    req = wl.c4_requests()
    rows = [(int(req.first_stream[i]), int(req.n_streams[i]), int(req.length[i]), 0, 0,
             int(req.dtype[i]), 0) for i in range(len(req))]
    kw = cfg or {}
    groups, pos, items = mg.batch_plan_groups(rows, mg.batch_config(**kw) if cfg else None)
    wave_min = kw.get("wave_min_bytes", 16 << 10)
    seg_bytes = kw.get("segment_bytes", 256 << 10)
    k, n, dt = req.n_streams, req.length, req.dtype
    e = np.where(dt == 2, 8, 4)
    assert items == [expected_items(int(k[i]), int(n[i]), int(dt[i]), seg_bytes, wave_min)
                     for i in range(len(req))]
    is_row = n * e < wave_min
    # one group per dtype with wave items, least output first, the first led by the rows
    assert groups[0]["rows"] and not any(g["rows"] for g in groups[1:])
    assert groups[0]["row_items"] == sum(it for it, r in zip(items, is_row) if r)
    assert len(groups) == len(set(dt[~is_row].tolist()))
    wave_bytes = [g["bytes"] - (groups[0]["bytes"] - sum(int(b) for b, r in
                  zip(k * n * e, is_row) if r) if g is groups[0] else 0) for g in groups]
    assert wave_bytes == sorted(wave_bytes)
    assert sum(g["items"] for g in groups) == sum(items)
    assert sum(g["bytes"] for g in groups) == int((k * n * e).sum())
    # the positions are a permutation; rows come first, largest item first
    assert sorted(pos) == list(range(len(req)))
    order = np.argsort(pos)
    nrow = int(is_row.sum())
    assert is_row[order[:nrow]].all() and not is_row[order[nrow:]].any()
    spi = np.clip((128 << 10) // (64 * n * e), 1, 16)
    item_bytes = np.minimum(k, 64 * spi) * n * e
    ib = item_bytes[order[:nrow]]
    assert (ib[:-1] >= ib[1:]).all()
    # the wave requests of one group keep their input order
    for d in set(dt[~is_row].tolist()):
        p = [pos[i] for i in range(len(req)) if not is_row[i] and dt[i] == d]
        assert p == sorted(p)


def test_plan_rejects_bad_dtype_and_flags():
    with pytest.raises(mg.MRGError):
        mg.batch_plan_groups([(0, 1, 1, 0, 0, 7, 0)])
    with pytest.raises(mg.MRGError):
        mg.batch_plan_groups([(0, 1, 1, 0, 0, 0, 8)])
    groups, pos, items = mg.batch_plan_groups([])
    assert groups == [] and pos == [] and items == []
