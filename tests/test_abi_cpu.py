"""CPU checks of the C-ABI library: it loads without a GPU, exports every
function the header declares, and its host-only helpers and argument
validation behave as documented (no kernel is launched here)."""
import ctypes
import os
import random
import re

import numpy as np
import pytest

import oracle
from paper_1412_8266_amd import _abi
from paper_1412_8266_amd import workloads as wl

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mrg32k3a_gpu.h")


def header_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(mrg_[a-z0-9_]+)\s*\(", text)
    return sorted(set(names))


def test_header_declares_entry_points():
    names = header_functions()
    for n in ("mrg_streamset_create", "mrg_jump", "mrg_fill", "mrg_streamset_destroy"):
        assert n in names


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(_abi.LIB_PATH)
    missing = [n for n in header_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_seed_from_master_matches_oracle():
    for seed in (0, 1, wl.MASTER_SEED, 2**64 - 1, 0xDEADBEEFCAFEBABE):
        assert _abi.mrg_seed_from_master(seed) == [int(x) for x in oracle.seed_from_master(seed)]


def test_jump_matrix_matches_oracle():
    rng = random.Random(5)
    exps = [0, 1, 2, 3, 1000, 1 << 76, 1 << 127, (1 << 192) - 1] + \
           [rng.randrange(0, 1 << 192) for _ in range(20)]
    for comp in (0, 1):
        for e in exps:
            assert _abi.mrg_jump_matrix(comp, e) == oracle.matpow(comp, e).tolist(), (comp, e)


def test_state_check():
    assert _abi.mrg_state_check([1, 2, 3, 4, 5, 6]) == _abi.MRG_OK
    assert _abi.mrg_state_check([0, 0, 0, 4, 5, 6]) == _abi.MRG_EINVAL
    assert _abi.mrg_state_check([1, 2, 3, 0, 0, 0]) == _abi.MRG_EINVAL
    assert _abi.mrg_state_check([oracle.M1, 2, 3, 4, 5, 6]) == _abi.MRG_EINVAL
    assert _abi.mrg_state_check([1, 2, 3, 4, 5, oracle.M2]) == _abi.MRG_EINVAL
    assert _abi.mrg_state_check([oracle.M1 - 1, 2, 3, 4, 5, oracle.M2 - 1]) == _abi.MRG_OK


def test_config_roundtrip_and_rejects():
    old = _abi.mrg_config_get("engine")
    try:
        _abi.mrg_config_set("engine", 0)
        assert _abi.mrg_config_get("engine") == 0
        _abi.mrg_config_set("engine", 1)
        assert _abi.mrg_config_get("engine") == 1
        with pytest.raises(_abi.MRGError):
            _abi.mrg_config_set("engine", 7)
        with pytest.raises(_abi.MRGError):
            _abi.mrg_config_set("no_such_key", 1)
        with pytest.raises(_abi.MRGError):
            _abi.mrg_config_set("tile_bytes", 100)
        lanes = _abi.mrg_config_get("coop_lanes")
        assert lanes == 0  # automatic by row length
        for v in (64, 32, 16, 8, 0):
            _abi.mrg_config_set("coop_lanes", v)
            assert _abi.mrg_config_get("coop_lanes") == v
        with pytest.raises(_abi.MRGError):
            _abi.mrg_config_set("coop_lanes", 12)
    finally:
        _abi.mrg_config_set("engine", old)


def test_validation_returns_before_any_device_work():
    lib = _abi.lib
    h = ctypes.c_void_p()
    bad_seed = (ctypes.c_uint32 * 6)(0, 0, 0, 1, 1, 1)
    assert lib.mrg_streamset_create(ctypes.byref(h), 4, 0, bad_seed, None) == _abi.MRG_EINVAL
    good = (ctypes.c_uint32 * 6)(*([12345] * 6))
    assert lib.mrg_streamset_create(None, 4, 0, good, None) == _abi.MRG_EINVAL
    assert lib.mrg_streamset_create(ctypes.byref(h), 0, 0, good, None) == _abi.MRG_ERANGE
    assert lib.mrg_streamset_create(ctypes.byref(h), 2, 2**64 - 1, good, None) == _abi.MRG_ERANGE
    assert lib.mrg_fill(None, 0, 1, 1, 0, 0, None, None) == _abi.MRG_EINVAL
    assert lib.mrg_jump(None, 0, 1, None, None) == _abi.MRG_EINVAL
    # random-spacing and Philox sets: sizes are checked before the device
    assert lib.mrg_streamset_create_random(None, 4, 0, 1, None) == _abi.MRG_EINVAL
    assert lib.mrg_streamset_create_random(ctypes.byref(h), 0, 0, 1, None) == _abi.MRG_ERANGE
    assert lib.mrg_streamset_create_philox(None, 4, 0, 1, None) == _abi.MRG_EINVAL
    assert lib.mrg_streamset_create_philox(ctypes.byref(h), 2, 2**64 - 1, 1, None) == _abi.MRG_ERANGE
    assert lib.mrg_streamset_create_philox(ctypes.byref(h), 2**36 + 1, 0, 1, None) == _abi.MRG_ERANGE
    assert lib.mrg_fill_leapfrog(None, 0, 4, 4, 0, 0, None, None) == _abi.MRG_EINVAL
    assert "null" in _abi.mrg_last_error()
    assert lib.mrg_streamset_destroy(None) == _abi.MRG_OK
    # store probe: pattern, size unit and alignment are checked first
    assert lib.mrg_write_probe(None, 16, 0, None) == _abi.MRG_EINVAL
    assert lib.mrg_write_probe(4096, 16, 3, None) == _abi.MRG_EINVAL
    assert lib.mrg_write_probe(4096, 16, -1, None) == _abi.MRG_EINVAL
    assert lib.mrg_write_probe(4096, 65536 + 16, 2, None) == _abi.MRG_EINVAL
    assert lib.mrg_write_probe(4096, 24, 0, None) == _abi.MRG_EINVAL
    assert lib.mrg_write_probe(4096, 65536 + 16, 1, None) == _abi.MRG_EINVAL
    assert lib.mrg_write_probe(4096 + 16, 65536, 1, None) == _abi.MRG_EINVAL
    assert lib.mrg_write_probe(4096, 0, 0, None) == _abi.MRG_OK
    for s in (0, -1, -2, -3, -4, -5, -6):
        assert _abi.mrg_status_string(s).startswith("MRG_")


def test_create_without_gpu_reports_no_device():
    try:
        import torch
        if torch.cuda.is_available():
            pytest.skip("a GPU is present")
    except Exception:
        pass
    lib = _abi.lib
    h = ctypes.c_void_p()
    good = (ctypes.c_uint32 * 6)(*([12345] * 6))
    assert lib.mrg_streamset_create(ctypes.byref(h), 4, 0, good, None) == _abi.MRG_ENODEV
    assert lib.mrg_write_probe(4096, 16, 0, None) == _abi.MRG_ENODEV


def test_workload_generators_are_deterministic_and_in_range():
    off = wl.c3_offsets(1000)
    assert off.dtype == np.uint64 and np.array_equal(off, wl.c3_offsets(1000))
    e = wl.c3_exponents(off)
    assert wl.words_to_int(e[0]) == int(off[0]) + (1 << 76)
    r = wl.c4_requests(2000)
    assert r.n_streams.min() >= 1 and r.n_streams.max() <= 4096
    assert r.length.min() >= 1 and r.length.max() <= 1 << 20
    assert set(np.unique(r.dtype)) <= {0, 1, 2}
    assert np.array_equal(r.first_stream[1:], np.cumsum(r.n_streams)[:-1])
    a = wl.c5_arrivals(rate=1000.0, duration=2.0)
    assert np.all(np.diff(a.t) > 0) and a.t[-1] < 2.0
    assert 1500 < len(a.t) < 2500
