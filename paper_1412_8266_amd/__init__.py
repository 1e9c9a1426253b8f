"""MI355X-native MRG32k3a stream library (HIP kernels for gfx950).

Bulk uniform random generation from many independent, reproducible streams
of MRG32k3a placed by jump ahead (Passerat-Palmbach & Hill, HPCS 2012:
sec. 4.1 streams of 2^127 and substreams of 2^76; sec. 2.3 sequence
splitting; sec. 5 host initialisation and per-thread ``next()``).

Every step runs in the HIP library ``libmrg32k3a_gpu.so``; this package only
marshals arguments.  PyTorch provides device memory and HIP streams.
"""
from __future__ import annotations

from typing import Optional

import numpy as np

from . import _abi
from ._abi import (MRGError, MRG_F32, MRG_F64, MRG_INTERLEAVED, MRG_STREAM_MAJOR, MRG_U32,
                   mrg_config_get, mrg_config_set, mrg_jump_matrix, mrg_seed_from_master,
                   mrg_state_check, mrg_version)

U32, F32, F64 = MRG_U32, MRG_F32, MRG_F64
STREAM_MAJOR, INTERLEAVED = MRG_STREAM_MAJOR, MRG_INTERLEAVED
M1 = 4294967087
M2 = 4294944443

_ESIZE = {U32: 4, F32: 4, F64: 8}


def _torch():
    import torch
    return torch


def torch_dtype(dtype: int):
    torch = _torch()
    return {U32: torch.uint32, F32: torch.float32, F64: torch.float64}[dtype]


def check_tensor(t, device: int, elems: int, esize: int, what: str = "output") -> None:
    """Raise ValueError unless ``t`` is a contiguous tensor in the memory of GPU
    ``device`` holding at least ``elems`` elements of ``esize`` bytes: the
    kernels store through its address, so a host tensor must never reach
    them (the C entry points check the pointer again)."""
    if not getattr(t, "is_cuda", False):
        raise ValueError("%s tensor must be on the GPU, not %s" % (what, getattr(t, "device", type(t))))
    if t.device.index != device:
        raise ValueError("%s tensor is on cuda:%s, the stream set on cuda:%d" % (what, t.device.index, device))
    if t.numel() < elems or t.element_size() != esize:
        raise ValueError("%s tensor too small or of the wrong element size" % what)
    if not t.is_contiguous():
        raise ValueError("%s tensor must be contiguous" % what)


def _stream_handle(stream) -> int:
    torch = _torch()
    if stream is None:
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


class StreamSet:
    """``n_streams`` consecutive MRG32k3a streams resident on the current GPU.

    Global stream g starts at A^(g * 2^127) * base; the stream set holds
    streams [first_stream, first_stream + n_streams).  The base state is
    ``seed`` (6 words) or is expanded from ``master_seed`` (64 bits).  With
    ``spacing="random"`` (and a master seed) stream g instead starts at its
    own random state, expanded from SplitMix64 output g of the master seed
    (random spacing, sec. 2.3).  With ``generator="philox"`` the streams are
    Philox4x32-10 streams under the key ``master_seed`` (stream g: counter
    words 2-3 = g).  With ``generator="tinymt"`` they are TinyMT32 streams in
    the hybrid of sec. 4.2: ``per_param`` consecutive streams share a
    parameter set (``params``: a [k, 3] array of sets ``params_first`` ..,
    else the library's search under ``master_seed``) and stream g starts
    (g % per_param) * 2^64 outputs past its set's base status.
    """

    def __init__(self, n_streams: int, seed=None, master_seed: Optional[int] = None,
                 first_stream: int = 0, stream=None, spacing: str = "jump",
                 generator: str = "mrg32k3a", per_param: int = 256, params=None,
                 params_first: int = 0):
        if (seed is None) == (master_seed is None):
            raise ValueError("give exactly one of seed (6 words) or master_seed")
        if spacing not in ("jump", "random"):
            raise ValueError("spacing must be 'jump' or 'random'")
        if generator not in ("mrg32k3a", "philox", "tinymt"):
            raise ValueError("generator must be 'mrg32k3a', 'philox' or 'tinymt'")
        if (spacing == "random" or generator != "mrg32k3a") and master_seed is None:
            raise ValueError("random spacing, Philox and TinyMT take a master_seed")
        if generator != "mrg32k3a" and spacing != "jump":
            raise ValueError("Philox and TinyMT streams are placed by their own scheme")
        h = _stream_handle(stream)
        self.generator = generator
        if generator == "tinymt":
            self._h = _abi.mrg_streamset_create_tinymt(n_streams, first_stream, per_param,
                                                       master_seed, params, params_first, h)
        elif generator == "philox":
            self._h = _abi.mrg_streamset_create_philox(n_streams, first_stream, master_seed, h)
        elif seed is not None:
            self._h = _abi.mrg_streamset_create(n_streams, first_stream, seed, h)
        elif spacing == "random":
            self._h = _abi.mrg_streamset_create_random(n_streams, first_stream, master_seed, h)
        else:
            self._h = _abi.mrg_streamset_create_seed64(n_streams, first_stream, master_seed, h)
        self.n_streams = int(n_streams)
        self.first_stream = int(first_stream)
        self.device = _torch().cuda.current_device()  # the set's states live here

    # -- lifetime -----------------------------------------------------------
    def close(self) -> None:
        if getattr(self, "_h", None):
            _abi.mrg_streamset_destroy(self._h)
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

    @property
    def handle(self) -> int:
        return self._h

    @property
    def base_state(self):
        return _abi.mrg_streamset_info(self._h)[2]

    @property
    def states_ptr(self) -> int:
        """Device address of the six state planes ([6][n] uint32), for user
        kernels built on mrg::Stream (include/mrg32k3a_device.h)."""
        return _abi.mrg_streamset_states_ptr(self._h)

    @property
    def tinymt_info(self):
        """(per_param, q0, n_sets, records address) of a TinyMT set, for user
        kernels built on mrg::TinyMTStream (include/tinymt_device.h)."""
        return _abi.mrg_streamset_tinymt_info(self._h)

    @property
    def tables_ptr(self) -> int:
        """Device address of the windowed jump tables, for mrg::Stream::jump."""
        return _abi.mrg_streamset_tables_ptr(self._h)

    def _range(self, first, count):
        if count is None:
            count = self.n_streams - first
        return int(first), int(count)

    # -- generation -----------------------------------------------------------
    def fill(self, n: int, dtype: int = U32, layout: int = STREAM_MAJOR, out=None,
             first: int = 0, count: Optional[int] = None, stream=None):
        """n outputs of each stream in [first, first+count); advances them by n.
        Returns a [count, n] (stream-major) or [n, count] (interleaved) tensor."""
        torch = _torch()
        first, count = self._range(first, count)
        shape = (count, n) if layout == STREAM_MAJOR else (n, count)
        if out is None:
            out = torch.empty(shape, dtype=torch_dtype(dtype), device="cuda:%d" % self.device)
        else:
            check_tensor(out, self.device, count * n, _ESIZE[dtype])
        _abi.mrg_fill(self._h, first, count, n, dtype, layout,
                      out.data_ptr() if out.numel() else 0, _stream_handle(stream))
        return out

    def fill_ptr(self, n: int, dtype: int, layout: int, d_out: int, first: int = 0,
                 count: Optional[int] = None, stream=None) -> None:
        first, count = self._range(first, count)
        _abi.mrg_fill(self._h, first, count, n, dtype, layout, d_out, _stream_handle(stream))

    def fill_leapfrog(self, s: int, players: int, per_player: int, dtype: int = U32,
                      layout: int = STREAM_MAJOR, out=None, stream=None):
        """Leapfrog (sec. 2.3): stream s dealt to ``players`` players, card k of
        player t being output t + k*players; advances stream s by
        players*per_player.  Returns a [players, per_player] (STREAM_MAJOR) or
        [per_player, players] (INTERLEAVED: the stream in order) tensor."""
        torch = _torch()
        shape = (players, per_player) if layout == STREAM_MAJOR else (per_player, players)
        if out is None:
            out = torch.empty(shape, dtype=torch_dtype(dtype), device="cuda:%d" % self.device)
        else:
            check_tensor(out, self.device, players * per_player, _ESIZE[dtype])
        _abi.mrg_fill_leapfrog(self._h, s, players, per_player, dtype, layout,
                               out.data_ptr() if out.numel() else 0, _stream_handle(stream))
        return out

    # -- jumps ------------------------------------------------------------------
    def jump(self, exps, first: int = 0, count: Optional[int] = None, stream=None) -> None:
        """Jump stream first+i by exps[i]; ``exps`` is a device uint64 tensor
        [count, 3] (little-endian words of each exponent)."""
        first, count = self._range(first, count)
        check_tensor(exps, self.device, 3 * count, 8, "exponent")
        _abi.mrg_jump(self._h, first, count, exps.data_ptr(), _stream_handle(stream))

    def jump_uniform(self, e: int, first: int = 0, count: Optional[int] = None,
                     stream=None) -> None:
        first, count = self._range(first, count)
        _abi.mrg_jump_uniform(self._h, first, count, e, _stream_handle(stream))

    def jump_substreams(self, k: int, first: int = 0, count: Optional[int] = None,
                        stream=None) -> None:
        first, count = self._range(first, count)
        _abi.mrg_jump_substreams(self._h, first, count, k, _stream_handle(stream))

    # -- states -----------------------------------------------------------------
    def get_states(self, first: int = 0, count: Optional[int] = None, stream=None) -> np.ndarray:
        first, count = self._range(first, count)
        w = _abi.mrg_get_states(self._h, first, count, _stream_handle(stream))
        return w.reshape(count, 6)

    def set_states(self, states, first: int = 0, stream=None) -> None:
        st = np.asarray(states, dtype=np.uint32).reshape(-1, 6)
        _abi.mrg_set_states(self._h, first, st.shape[0], st.reshape(-1), _stream_handle(stream))


__all__ = [
    "StreamSet", "MRGError", "U32", "F32", "F64", "STREAM_MAJOR", "INTERLEAVED", "M1", "M2",
    "mrg_seed_from_master", "mrg_jump_matrix", "mrg_state_check", "mrg_config_set",
    "mrg_config_get", "mrg_version", "torch_dtype", "write_probe", "check_tensor",
    "tinymt_search", "tinymt_test_candidates",
]


def tinymt_search(master_seed: int, count: int, stream=None):
    """Parameter sets 0 .. count-1 of the TinyMT32 search under master_seed:
    ([count, 3] uint32 array, [count] candidate numbers)."""
    p, c = _abi.mrg_tinymt_search(master_seed, count, _stream_handle(stream))
    return (np.array(p, dtype=np.uint32).reshape(-1, 3), np.array(c, dtype=np.uint64))


def tinymt_test_candidates(master_seed: int, c0: int, n: int, with_phi: bool = False,
                           stream=None):
    """Device test of candidates c0 .. c0+n-1: (flags tensor [n] int32 holding
    L | accepted << 16, characteristic polynomials [n, 4] or None)."""
    torch = _torch()
    dev = "cuda:%d" % torch.cuda.current_device()
    flags = torch.empty(max(n, 1), dtype=torch.int32, device=dev)
    phi = torch.empty((max(n, 1), 4), dtype=torch.int32, device=dev) if with_phi else None
    _abi.mrg_tinymt_test_candidates(master_seed, c0, n, flags.data_ptr(),
                                    phi.data_ptr() if phi is not None else 0,
                                    _stream_handle(stream))
    return flags[:n], (phi[:n] if phi is not None else None)


def write_probe(out, pattern: int = 0, stream=None) -> None:
    """Store-only bandwidth probe over the whole of `out` (a CUDA tensor):
    pattern 0 streaming 16-byte stores in one pass, 1 the wave-per-stream
    fill's geometry (runs of two 128-byte lines per member), 2 the same with
    runs of 8 lines per store instruction, 3 single lines per member
    (mrg_write_probe in the C ABI)."""
    _abi.mrg_write_probe(out.data_ptr(), out.numel() * out.element_size(), pattern,
                         _stream_handle(stream))


# ---------------------------------------------------------------------------
# batched generation
# ---------------------------------------------------------------------------
from ._abi import MRG_REQ_SUBSTREAMS, MRG_SCHEDULE_DYNAMIC, MRG_SCHEDULE_STATIC  # noqa: E402

REQ_SUBSTREAMS = MRG_REQ_SUBSTREAMS
SCHEDULE_DYNAMIC, SCHEDULE_STATIC = MRG_SCHEDULE_DYNAMIC, MRG_SCHEDULE_STATIC


def batch_config(segment_bytes=0, wave_min_bytes=0, waves_per_cu=0, schedule=0):
    return _abi.make_config(segment_bytes, wave_min_bytes, waves_per_cu, schedule)


def batch_plan_groups(requests, config=None):
    """The launch groups a Batch of these request rows would run, planned on
    the host alone (no device, d_out not read): (groups in launch order,
    each request's index in the grouped order, each request's work items)."""
    rows = list(requests)
    return _abi.mrg_batch_plan_groups(_abi.make_requests(rows), len(rows), config)


class Batch:
    """Many fill requests over one StreamSet run as one hipGraph of
    persistent launches (batch_plan_groups shows the grouping).

    ``requests`` rows are (first, count, n_per_stream, substream0, d_out,
    dtype, flags); d_out is a device pointer (int) to a [count, n] array.
    The outputs and the stream set must outlive the batch.
    """

    def __init__(self, streamset: StreamSet, requests, config=None):
        rows = list(requests)
        self._arr = _abi.make_requests(rows)
        self.n_requests = len(rows)
        self.streamset = streamset
        self._h = _abi.mrg_batch_create(streamset.handle, self._arr, len(rows), config)

    def run(self, stream=None) -> None:
        _abi.mrg_batch_run(self._h, _stream_handle(stream))

    def run_direct(self, stream=None) -> None:
        _abi.mrg_batch_run_direct(self._h, _stream_handle(stream))

    def request_times(self, stream=None) -> np.ndarray:
        """Milliseconds from the start of the last run to each request's end
        (input order; 0 for empty requests)."""
        return np.asarray(_abi.mrg_batch_request_times(self._h, self.n_requests,
                                                       _stream_handle(stream)))

    def run_per_request(self, stream=None) -> None:
        _abi.mrg_batch_run_per_request(self._h, _stream_handle(stream))

    def info(self) -> dict:
        return _abi.mrg_batch_info(self._h)

    def autotune(self, configs, reps: int = 1, stream=None):
        return _abi.mrg_batch_autotune(self._h, configs, reps, _stream_handle(stream))

    def close(self) -> None:
        if getattr(self, "_h", None):
            _abi.mrg_batch_destroy(self._h)
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


__all__ += ["Batch", "batch_config", "batch_plan_groups", "REQ_SUBSTREAMS", "SCHEDULE_DYNAMIC",
            "SCHEDULE_STATIC"]
