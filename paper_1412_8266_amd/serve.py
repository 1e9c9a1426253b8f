"""Serving front end: a thin wrapper of the native continuous-batching
engine (mrg_server_* in the C ABI).  The scheduler, admission, arena and
device launches all run in the library; this module marshals arguments and
turns finished-request records into numpy arrays."""
from __future__ import annotations

import ctypes

import numpy as np

from . import _abi

RESULT_DTYPE = np.dtype([
    ("ticket", np.uint64), ("client", np.uint64), ("n_streams", np.uint64),
    ("n_per_stream", np.uint64), ("substream0", np.uint64), ("d_out", np.uint64),
    ("dtype", np.int32), ("pad", np.int32), ("latency_s", np.float64), ("queue_s", np.float64),
    ("t_submit", np.float64)])
assert RESULT_DTYPE.itemsize == ctypes.sizeof(_abi.mrg_server_result)


class Server:
    """Clients 0 .. n_clients-1 own global streams first_stream + c of the
    generator seeded by master_seed; requests get each client's next
    substreams.  Outputs live in a device arena of arena_bytes."""

    def __init__(self, n_clients: int, master_seed: int, arena_bytes: int, first_stream: int = 0,
                 max_inflight: int = 0, max_batch: int = 0, waves_per_cu: int = 0,
                 auto_release: bool = False, big_request_bytes: int = 0):
        self._h = _abi.mrg_server_create(n_clients, first_stream, master_seed, arena_bytes,
                                         max_inflight, max_batch, waves_per_cu,
                                         1 if auto_release else 0, big_request_bytes)
        self.auto_release = auto_release

    def submit(self, client: int, n_streams: int, n_per_stream: int, dtype: int) -> int:
        return _abi.mrg_server_submit(self._h, client, n_streams, n_per_stream, dtype)

    def poll(self, max_out: int = 65536) -> np.ndarray:
        """Finished requests as a structured array (oldest first)."""
        out = []
        while True:
            buf, n = _abi.mrg_server_poll(self._h, max_out)
            if n:
                out.append(np.frombuffer(buf, dtype=RESULT_DTYPE, count=n).copy())
            if n < max_out:
                break
        if not out:
            return np.zeros(0, dtype=RESULT_DTYPE)
        return np.concatenate(out)

    def release(self, ticket: int) -> None:
        _abi.mrg_server_release(self._h, ticket)

    def output(self, rec) -> np.ndarray:
        """Host copy of a finished, held request's [k, n] output."""
        dt = {0: np.uint32, 1: np.float32, 2: np.float64}[int(rec["dtype"])]
        out = np.empty((int(rec["n_streams"]), int(rec["n_per_stream"])), dtype=dt)
        _abi.mrg_server_copy_output(self._h, int(rec["ticket"]), out.ctypes.data, out.nbytes)
        return out

    def stats(self) -> dict:
        return _abi.mrg_server_stats(self._h)

    def drain(self, timeout_s: float = 60.0) -> None:
        _abi.mrg_server_drain(self._h, timeout_s)

    def run_trace(self, t, client, n_streams, n_per_stream, dtype, time_scale: float = 1.0) -> float:
        n = len(t)
        arr = (_abi.mrg_arrival * max(n, 1))()
        view = np.frombuffer(arr, dtype=np.dtype([("t", np.float64), ("client", np.uint64),
                                                  ("n_streams", np.uint64),
                                                  ("n_per_stream", np.uint64),
                                                  ("dtype", np.int32), ("pad", np.int32)]),
                             count=n)
        view["t"] = t
        view["client"] = client
        view["n_streams"] = n_streams
        view["n_per_stream"] = n_per_stream
        view["dtype"] = dtype
        return _abi.mrg_server_run_trace(self._h, arr, n, time_scale)

    def client_state(self, client: int):
        return _abi.mrg_server_client_state(self._h, client)

    def close(self) -> None:
        if getattr(self, "_h", None):
            _abi.mrg_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
