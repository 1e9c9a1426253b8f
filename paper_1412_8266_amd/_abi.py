"""ctypes binding of ``libmrg32k3a_gpu.so`` (declared in include/mrg32k3a_gpu.h).

Argument marshalling only: every function here forwards to the C entry point
of the same name.  Device pointers and HIP streams are passed as integers
(``tensor.data_ptr()``, ``torch.cuda.Stream.cuda_stream``).  There is no CPU
path: if the library is not built, importing this module raises.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmrg32k3a_gpu.so")

MRG_OK, MRG_EINVAL, MRG_ENOMEM, MRG_EHIP, MRG_ERANGE, MRG_ENODEV, MRG_EBUSY = 0, -1, -2, -3, -4, -5, -6
MRG_U32, MRG_F32, MRG_F64 = 0, 1, 2
MRG_STREAM_MAJOR, MRG_INTERLEAVED = 0, 1


class MRGError(RuntimeError):
    def __init__(self, status: int, func: str, detail: str):
        super().__init__("%s failed with %d: %s" % (func, status, detail))
        self.status = status


def _load() -> ctypes.CDLL:
    # PyTorch ships its own HIP runtime.  Importing it first makes the
    # library's libamdhip64.so.7 / libhsa-runtime64.so.1 resolve to the copies
    # already in the process, so that the library and torch share one runtime
    # (two runtimes in one process cannot both open the device).
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            "libmrg32k3a_gpu.so is not built (expected at %s); build it with "
            "`python paper_1412_8266_amd/build.py`" % LIB_PATH)
    return ctypes.CDLL(LIB_PATH)


lib = _load()

_P = ctypes.c_void_p
_U64 = ctypes.c_uint64
_I32 = ctypes.c_int32
_I64 = ctypes.c_int64
_PU32 = ctypes.POINTER(ctypes.c_uint32)
_PU64 = ctypes.POINTER(ctypes.c_uint64)

_SIGS = {
    "mrg_streamset_create": [ctypes.POINTER(_P), _U64, _U64, _PU32, _P],
    "mrg_streamset_create_seed64": [ctypes.POINTER(_P), _U64, _U64, _U64, _P],
    "mrg_streamset_create_random": [ctypes.POINTER(_P), _U64, _U64, _U64, _P],
    "mrg_streamset_create_philox": [ctypes.POINTER(_P), _U64, _U64, _U64, _P],
    "mrg_streamset_create_tinymt": [ctypes.POINTER(_P), _U64, _U64, _U64, _U64, _PU32, _U64, _U64,
                                    _P],
    "mrg_streamset_tinymt_info": [_P, _PU64, _PU64, _PU64, ctypes.POINTER(_P)],
    "mrg_tinymt_test_candidates": [_U64, _U64, _U64, _P, _P, _P],
    "mrg_tinymt_search": [_U64, _U64, _PU32, _PU64, _P],
    "mrg_streamset_destroy": [_P],
    "mrg_streamset_info": [_P, _PU64, _PU64, _PU32],
    "mrg_streamset_states_ptr": [_P, ctypes.POINTER(_P)],
    "mrg_streamset_tables_ptr": [_P, ctypes.POINTER(_P)],
    "mrg_jump": [_P, _U64, _U64, _P, _P],
    "mrg_jump_uniform": [_P, _U64, _U64, _PU64, _P],
    "mrg_jump_substreams": [_P, _U64, _U64, _U64, _P],
    "mrg_fill": [_P, _U64, _U64, _U64, _I32, _I32, _P, _P],
    "mrg_fill_leapfrog": [_P, _U64, _U64, _U64, _I32, _I32, _P, _P],
    "mrg_get_states": [_P, _U64, _U64, _PU32, _P],
    "mrg_set_states": [_P, _U64, _U64, _PU32, _P],
    "mrg_seed_from_master": [_U64, _PU32],
    "mrg_jump_matrix": [_I32, _PU64, _PU32],
    "mrg_state_check": [_PU32],
    "mrg_config_set": [ctypes.c_char_p, _I64],
    "mrg_config_get": [ctypes.c_char_p, ctypes.POINTER(_I64)],
}
MRG_REQ_SUBSTREAMS = 1
MRG_SCHEDULE_DYNAMIC, MRG_SCHEDULE_STATIC = 1, 2


class mrg_request(ctypes.Structure):
    _fields_ = [("first", ctypes.c_uint64), ("count", ctypes.c_uint64),
                ("n_per_stream", ctypes.c_uint64), ("substream0", ctypes.c_uint64),
                ("d_out", ctypes.c_void_p), ("dtype", ctypes.c_int32), ("flags", ctypes.c_uint32)]


class mrg_batch_config(ctypes.Structure):
    _fields_ = [("segment_bytes", ctypes.c_uint64), ("wave_min_bytes", ctypes.c_uint64),
                ("waves_per_cu", ctypes.c_uint32), ("schedule", ctypes.c_uint32)]


class mrg_batch_info_t(ctypes.Structure):
    _fields_ = [("requests", ctypes.c_uint64), ("items", ctypes.c_uint64),
                ("samples", ctypes.c_uint64), ("bytes", ctypes.c_uint64),
                ("scratch_states", ctypes.c_uint64), ("grid", ctypes.c_uint32),
                ("pad", ctypes.c_uint32), ("config", mrg_batch_config)]


class mrg_plan_group(ctypes.Structure):
    _fields_ = [("dtype", ctypes.c_int32), ("rows", ctypes.c_int32), ("requests", ctypes.c_uint64),
                ("items", ctypes.c_uint64), ("row_items", ctypes.c_uint64),
                ("bytes", ctypes.c_uint64)]


_SIGS.update({
    "mrg_batch_plan_groups": [ctypes.POINTER(mrg_request), _U64, ctypes.POINTER(mrg_batch_config),
                              ctypes.POINTER(mrg_plan_group), ctypes.POINTER(ctypes.c_uint32),
                              ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(ctypes.c_uint64)],
    "mrg_batch_create": [ctypes.POINTER(_P), _P, ctypes.POINTER(mrg_request), _U64,
                         ctypes.POINTER(mrg_batch_config)],
    "mrg_batch_run": [_P, _P],
    "mrg_batch_run_direct": [_P, _P],
    "mrg_batch_run_per_request": [_P, _P],
    "mrg_batch_info": [_P, ctypes.POINTER(mrg_batch_info_t)],
    "mrg_batch_request_times": [_P, _P, ctypes.POINTER(ctypes.c_double)],
    "mrg_batch_autotune": [_P, ctypes.POINTER(mrg_batch_config), ctypes.c_uint32, ctypes.c_uint32,
                           _P, ctypes.POINTER(ctypes.c_uint32), ctypes.POINTER(ctypes.c_float)],
    "mrg_batch_destroy": [_P],
    "mrg_batch_run_noalloc": [_P, ctypes.POINTER(mrg_request), _U64,
                              ctypes.POINTER(mrg_batch_config), _P],
})

class mrg_server_config(ctypes.Structure):
    _fields_ = [("n_clients", ctypes.c_uint64), ("first_stream", ctypes.c_uint64),
                ("master_seed", ctypes.c_uint64), ("arena_bytes", ctypes.c_uint64),
                ("max_inflight", ctypes.c_uint32), ("max_batch", ctypes.c_uint32),
                ("waves_per_cu", ctypes.c_uint32), ("auto_release", ctypes.c_uint32),
                ("pad", ctypes.c_uint32), ("big_request_bytes", ctypes.c_uint64)]


class mrg_server_result(ctypes.Structure):
    _fields_ = [("ticket", ctypes.c_uint64), ("client", ctypes.c_uint64),
                ("n_streams", ctypes.c_uint64), ("n_per_stream", ctypes.c_uint64),
                ("substream0", ctypes.c_uint64), ("d_out", ctypes.c_void_p),
                ("dtype", ctypes.c_int32), ("pad", ctypes.c_int32),
                ("latency_s", ctypes.c_double), ("queue_s", ctypes.c_double),
                ("t_submit", ctypes.c_double)]


class mrg_server_stats_t(ctypes.Structure):
    _fields_ = [(f, ctypes.c_uint64) for f in ("pending", "inflight", "completed", "ticks",
                                               "samples", "bytes", "arena_used", "arena_bytes")]


class mrg_arrival(ctypes.Structure):
    _fields_ = [("t", ctypes.c_double), ("client", ctypes.c_uint64),
                ("n_streams", ctypes.c_uint64), ("n_per_stream", ctypes.c_uint64),
                ("dtype", ctypes.c_int32), ("pad", ctypes.c_int32)]


_SIGS.update({
    "mrg_server_create": [ctypes.POINTER(_P), ctypes.POINTER(mrg_server_config)],
    "mrg_server_submit": [_P, _U64, _U64, _U64, _I32, ctypes.POINTER(_U64)],
    "mrg_server_poll": [_P, ctypes.POINTER(mrg_server_result), _U64, ctypes.POINTER(_U64)],
    "mrg_server_release": [_P, _U64],
    "mrg_server_copy_output": [_P, _U64, _P, _U64],
    "mrg_server_stats": [_P, ctypes.POINTER(mrg_server_stats_t)],
    "mrg_server_drain": [_P, ctypes.c_double],
    "mrg_server_run_trace": [_P, ctypes.POINTER(mrg_arrival), _U64, ctypes.c_double,
                             ctypes.POINTER(ctypes.c_double)],
    "mrg_server_client_state": [_P, _U64, _PU32, ctypes.POINTER(_U64)],
    "mrg_server_destroy": [_P],
    "mrg_write_probe": [_P, _U64, _I32, _P],
})

for _name, _args in _SIGS.items():
    _f = getattr(lib, _name)
    _f.argtypes = _args
    _f.restype = _I32
lib.mrg_status_string.argtypes = [_I32]
lib.mrg_status_string.restype = ctypes.c_char_p
lib.mrg_last_error.argtypes = []
lib.mrg_last_error.restype = ctypes.c_char_p
lib.mrg_version.argtypes = []
lib.mrg_version.restype = _I32


def check(status: int, func: str) -> None:
    if status != MRG_OK:
        raise MRGError(status, func, lib.mrg_last_error().decode(errors="replace"))


def _call(name, *args):
    check(getattr(lib, name)(*args), name)


def _u32(words, n):
    arr = (ctypes.c_uint32 * n)(*[int(w) for w in words])
    return arr


def _u64x3(e: int):
    if not (0 <= int(e) < 1 << 192):
        raise ValueError("exponent must be in [0, 2^192)")
    e = int(e)
    return (ctypes.c_uint64 * 3)(*[(e >> (64 * i)) & ((1 << 64) - 1) for i in range(3)])


# ---- same-named wrappers ------------------------------------------------------
def mrg_streamset_create(n_streams: int, first_stream: int, seed6, stream: int = 0) -> int:
    h = _P()
    _call("mrg_streamset_create", ctypes.byref(h), n_streams, first_stream, _u32(seed6, 6), stream)
    return h.value


def mrg_streamset_create_seed64(n_streams: int, first_stream: int, master_seed: int,
                                stream: int = 0) -> int:
    h = _P()
    _call("mrg_streamset_create_seed64", ctypes.byref(h), n_streams, first_stream,
          master_seed & ((1 << 64) - 1), stream)
    return h.value


def mrg_streamset_create_random(n_streams: int, first_stream: int, master_seed: int,
                                stream: int = 0) -> int:
    h = _P()
    _call("mrg_streamset_create_random", ctypes.byref(h), n_streams, first_stream,
          master_seed & ((1 << 64) - 1), stream)
    return h.value


def mrg_streamset_create_philox(n_streams: int, first_stream: int, key: int,
                                stream: int = 0) -> int:
    h = _P()
    _call("mrg_streamset_create_philox", ctypes.byref(h), n_streams, first_stream,
          key & ((1 << 64) - 1), stream)
    return h.value


def mrg_streamset_create_tinymt(n_streams: int, first_stream: int, per_param: int,
                                master_seed: int, params=None, params_first: int = 0,
                                stream: int = 0) -> int:
    """params: None (the library searches the sets) or a [k, 3] array of
    parameter sets params_first .. params_first + k - 1."""
    h = _P()
    if params is None:
        arr, k = None, 0
    else:
        flat = [int(w) for row in params for w in row]
        k = len(flat) // 3
        arr = _u32(flat, len(flat))
    _call("mrg_streamset_create_tinymt", ctypes.byref(h), n_streams, first_stream, per_param,
          master_seed & ((1 << 64) - 1), arr, params_first, k, stream)
    return h.value


def mrg_streamset_tinymt_info(ss: int):
    """(per_param, q0, n_sets, device address of the parameter records)."""
    per, q0, n = _U64(), _U64(), _U64()
    rec = _P()
    _call("mrg_streamset_tinymt_info", ss, ctypes.byref(per), ctypes.byref(q0), ctypes.byref(n),
          ctypes.byref(rec))
    return per.value, q0.value, n.value, int(rec.value or 0)


def mrg_tinymt_test_candidates(master_seed: int, c0: int, n: int, d_flags: int, d_phi: int = 0,
                               stream: int = 0) -> None:
    _call("mrg_tinymt_test_candidates", master_seed & ((1 << 64) - 1), c0, n, d_flags,
          d_phi or None, stream)


def mrg_tinymt_search(master_seed: int, count: int, stream: int = 0):
    """([count][3] parameter sets, [count] candidate numbers) as lists."""
    params = (ctypes.c_uint32 * max(3 * count, 1))()
    cand = (ctypes.c_uint64 * max(count, 1))()
    _call("mrg_tinymt_search", master_seed & ((1 << 64) - 1), count, params, cand, stream)
    return ([list(params[3 * i:3 * i + 3]) for i in range(count)], list(cand[:count]))


def mrg_streamset_destroy(ss: int) -> None:
    _call("mrg_streamset_destroy", ss)


def mrg_streamset_info(ss: int):
    n, first = _U64(), _U64()
    seed = (ctypes.c_uint32 * 6)()
    _call("mrg_streamset_info", ss, ctypes.byref(n), ctypes.byref(first), seed)
    return n.value, first.value, list(seed)


def mrg_streamset_tables_ptr(ss: int) -> int:
    p = _P()
    _call("mrg_streamset_tables_ptr", ss, ctypes.byref(p))
    return int(p.value or 0)


def mrg_streamset_states_ptr(ss: int) -> int:
    p = _P()
    _call("mrg_streamset_states_ptr", ss, ctypes.byref(p))
    return p.value


def mrg_jump(ss: int, first: int, count: int, d_exp: int, stream: int = 0) -> None:
    _call("mrg_jump", ss, first, count, d_exp, stream)


def mrg_jump_uniform(ss: int, first: int, count: int, e: int, stream: int = 0) -> None:
    _call("mrg_jump_uniform", ss, first, count, _u64x3(e), stream)


def mrg_jump_substreams(ss: int, first: int, count: int, k: int, stream: int = 0) -> None:
    _call("mrg_jump_substreams", ss, first, count, k, stream)


def mrg_fill(ss: int, first: int, count: int, n_per_stream: int, dtype: int, layout: int,
             d_out: int, stream: int = 0) -> None:
    _call("mrg_fill", ss, first, count, n_per_stream, dtype, layout, d_out, stream)


def mrg_fill_leapfrog(ss: int, s: int, players: int, per_player: int, dtype: int, layout: int,
                      d_out: int, stream: int = 0) -> None:
    _call("mrg_fill_leapfrog", ss, s, players, per_player, dtype, layout, d_out, stream)


def mrg_get_states(ss: int, first: int, count: int, stream: int = 0):
    """[count * 6] uint32 numpy array of the states, stream after stream."""
    import numpy as np
    buf = np.empty(6 * count, dtype=np.uint32)
    _call("mrg_get_states", ss, first, count, buf.ctypes.data_as(_PU32), stream)
    return buf


def mrg_set_states(ss: int, first: int, count: int, words, stream: int = 0) -> None:
    import numpy as np
    buf = np.ascontiguousarray(np.asarray(words, dtype=np.uint32).reshape(-1))
    if buf.size < 6 * count:
        raise ValueError("need 6 words per stream")
    _call("mrg_set_states", ss, first, count, buf.ctypes.data_as(_PU32), stream)


def mrg_seed_from_master(master_seed: int):
    out = (ctypes.c_uint32 * 6)()
    _call("mrg_seed_from_master", master_seed & ((1 << 64) - 1), out)
    return list(out)


def mrg_jump_matrix(component: int, e: int):
    out = (ctypes.c_uint32 * 9)()
    _call("mrg_jump_matrix", component, _u64x3(e), out)
    return [list(out[0:3]), list(out[3:6]), list(out[6:9])]


def mrg_state_check(state6) -> int:
    return int(lib.mrg_state_check(_u32(state6, 6)))


def mrg_config_set(key: str, value: int) -> None:
    _call("mrg_config_set", key.encode(), value)


def mrg_config_get(key: str) -> int:
    v = _I64()
    _call("mrg_config_get", key.encode(), ctypes.byref(v))
    return v.value


def mrg_status_string(status: int) -> str:
    return lib.mrg_status_string(status).decode()


def mrg_last_error() -> str:
    return lib.mrg_last_error().decode(errors="replace")


def mrg_version() -> int:
    return int(lib.mrg_version())


def mrg_write_probe(d_out: int, nbytes: int, pattern: int, stream: int = 0) -> None:
    _call("mrg_write_probe", d_out, nbytes, pattern, stream)


def make_requests(rows) -> "ctypes.Array":
    """rows: iterable of (first, count, n_per_stream, substream0, d_out, dtype, flags)."""
    rows = list(rows)
    arr = (mrg_request * max(len(rows), 1))()
    for i, r in enumerate(rows):
        arr[i] = mrg_request(*[int(v) for v in r])
    return arr


def make_config(segment_bytes=0, wave_min_bytes=0, waves_per_cu=0, schedule=0):
    return mrg_batch_config(segment_bytes, wave_min_bytes, waves_per_cu, schedule)


def mrg_batch_create(ss: int, reqs, n_reqs: int, cfg=None) -> int:
    h = _P()
    _call("mrg_batch_create", ctypes.byref(h), ss, reqs, n_reqs,
          ctypes.byref(cfg) if cfg is not None else None)
    return h.value


def mrg_batch_run(b: int, stream: int = 0) -> None:
    _call("mrg_batch_run", b, stream)


def mrg_batch_run_direct(b: int, stream: int = 0) -> None:
    _call("mrg_batch_run_direct", b, stream)


def mrg_batch_run_per_request(b: int, stream: int = 0) -> None:
    _call("mrg_batch_run_per_request", b, stream)


def mrg_batch_info(b: int) -> dict:
    info = mrg_batch_info_t()
    _call("mrg_batch_info", b, ctypes.byref(info))
    c = info.config
    return {"requests": info.requests, "items": info.items, "samples": info.samples,
            "bytes": info.bytes, "scratch_states": info.scratch_states, "grid": info.grid,
            "segment_bytes": c.segment_bytes, "wave_min_bytes": c.wave_min_bytes,
            "waves_per_cu": c.waves_per_cu, "schedule": c.schedule}


def mrg_batch_plan_groups(reqs, n_reqs: int, cfg=None):
    """Host-only plan: (groups in launch order as dicts, pos, items) per input request."""
    groups = (mrg_plan_group * 3)()
    ng = ctypes.c_uint32()
    pos = (ctypes.c_uint64 * max(n_reqs, 1))()
    items = (ctypes.c_uint64 * max(n_reqs, 1))()
    _call("mrg_batch_plan_groups", reqs, n_reqs, ctypes.byref(cfg) if cfg is not None else None,
          groups, ctypes.byref(ng), pos, items)
    out = [{"dtype": g.dtype, "rows": bool(g.rows), "requests": g.requests, "items": g.items,
            "row_items": g.row_items, "bytes": g.bytes} for g in groups[:ng.value]]
    return out, [pos[i] for i in range(n_reqs)], [items[i] for i in range(n_reqs)]


def mrg_batch_request_times(b: int, n_reqs: int, stream: int = 0):
    arr = (ctypes.c_double * max(n_reqs, 1))()
    _call("mrg_batch_request_times", b, stream, arr)
    return [arr[i] for i in range(n_reqs)]


def mrg_batch_autotune(b: int, configs, reps: int = 1, stream: int = 0):
    n = len(configs)
    arr = (mrg_batch_config * n)(*configs)
    best = ctypes.c_uint32()
    ms = (ctypes.c_float * n)()
    _call("mrg_batch_autotune", b, arr, n, reps, stream, ctypes.byref(best), ms)
    return best.value, list(ms)


def mrg_batch_destroy(b: int) -> None:
    _call("mrg_batch_destroy", b)


def mrg_batch_run_noalloc(ss: int, reqs, n_reqs: int, cfg=None, stream: int = 0) -> None:
    _call("mrg_batch_run_noalloc", ss, reqs, n_reqs,
          ctypes.byref(cfg) if cfg is not None else None, stream)


def mrg_server_create(n_clients, first_stream, master_seed, arena_bytes, max_inflight=0,
                      max_batch=0, waves_per_cu=0, auto_release=0, big_request_bytes=0) -> int:
    cfg = mrg_server_config(n_clients, first_stream, master_seed & ((1 << 64) - 1), arena_bytes,
                            max_inflight, max_batch, waves_per_cu, auto_release, 0,
                            big_request_bytes)
    h = _P()
    _call("mrg_server_create", ctypes.byref(h), ctypes.byref(cfg))
    return h.value


def mrg_server_submit(s: int, client: int, n_streams: int, n_per_stream: int, dtype: int) -> int:
    t = _U64()
    _call("mrg_server_submit", s, client, n_streams, n_per_stream, dtype, ctypes.byref(t))
    return t.value


def mrg_server_poll(s: int, max_out: int = 4096):
    buf = (mrg_server_result * max(max_out, 1))()
    n = _U64()
    _call("mrg_server_poll", s, buf, max_out, ctypes.byref(n))
    return buf, n.value


def mrg_server_release(s: int, ticket: int) -> None:
    _call("mrg_server_release", s, ticket)


def mrg_server_copy_output(s: int, ticket: int, h_dst: int, nbytes: int) -> None:
    _call("mrg_server_copy_output", s, ticket, h_dst, nbytes)


def mrg_server_stats(s: int) -> dict:
    st = mrg_server_stats_t()
    _call("mrg_server_stats", s, ctypes.byref(st))
    return {f: getattr(st, f) for f, _ in mrg_server_stats_t._fields_}


def mrg_server_drain(s: int, timeout_s: float) -> None:
    _call("mrg_server_drain", s, timeout_s)


def mrg_server_run_trace(s: int, arrivals, n: int, time_scale: float = 1.0) -> float:
    wall = ctypes.c_double()
    _call("mrg_server_run_trace", s, arrivals, n, time_scale, ctypes.byref(wall))
    return wall.value


def mrg_server_client_state(s: int, client: int):
    out = (ctypes.c_uint32 * 6)()
    nxt = _U64()
    _call("mrg_server_client_state", s, client, out, ctypes.byref(nxt))
    return list(out), nxt.value


def mrg_server_destroy(s: int) -> None:
    _call("mrg_server_destroy", s)
