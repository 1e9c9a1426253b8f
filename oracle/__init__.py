"""MRG32k3a CPU oracle -- test infrastructure only.

Only ``tests/``, the smoke check in ``__graft_entry__`` and the CPU-baseline
leg of ``bench.py`` may import this package.  The GPU library never imports,
links or calls it, and it imports nothing from the GPU library.

Two independent CPU implementations live here:

* ``mrg32k3a_oracle.c`` -- plain C99, single thread, 64-bit ``%`` (the bulk
  oracle), loaded with ctypes through the wrappers below;
* ``ref.py`` -- pure-Python big-integer arithmetic for tiny cases and for the
  closed-form pins (matrix powers with ~100-bit exponents).

Both follow sec. 4.1 (MRG32k3a: 6-integer state, streams of 2^127 and
substreams of 2^76) and sec. 2.3 (sequence splitting by jump ahead, random
spacing) of Passerat-Palmbach & Hill, HPCS 2012, with the generator's
constants from L'Ecuyer 1999, which that section cites.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mrg32k3a_oracle.c")
_LIB = os.path.join(_HERE, "libmrg32k3a_oracle.so")

U32, F32, F64 = 0, 1, 2
STREAM_MAJOR, INTERLEAVED = 0, 1
M1 = 4294967087
M2 = 4294944443

_DTYPES = {U32: np.uint32, F32: np.float32, F64: np.float64}
_lock = threading.Lock()
_lib = None


def build(force: bool = False) -> str:
    """Compile the C oracle into ``oracle/libmrg32k3a_oracle.so``."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call([
            "gcc", "-O2", "-std=c99", "-ffp-contract=off", "-fno-fast-math",
            "-fPIC", "-shared", "-o", tmp, _SRC,
        ])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        build()
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        u64 = ctypes.c_uint64
        lib.orc_step.argtypes = [P]
        lib.orc_step.restype = ctypes.c_uint32
        lib.orc_to_f64.argtypes = [ctypes.c_uint32]
        lib.orc_to_f64.restype = ctypes.c_double
        lib.orc_to_f32.argtypes = [ctypes.c_uint32]
        lib.orc_to_f32.restype = ctypes.c_float
        lib.orc_fill.argtypes = [P, u64, u64, ctypes.c_int, ctypes.c_int, P]
        lib.orc_fill.restype = None
        lib.orc_skip.argtypes = [P, u64]
        lib.orc_skip.restype = None
        lib.orc_companion.argtypes = [ctypes.c_int, P]
        lib.orc_matpow.argtypes = [ctypes.c_int, P, P]
        lib.orc_matvec.argtypes = [ctypes.c_int, P, P]
        lib.orc_jump.argtypes = [P, P]
        lib.orc_jump_many.argtypes = [P, u64, P, ctypes.c_int]
        lib.orc_stream_start.argtypes = [P, u64, P]
        lib.orc_streams.argtypes = [P, u64, u64, P]
        lib.orc_streams_adjacent.argtypes = [P, u64, u64, P]
        lib.orc_jump_uniform.argtypes = [P, u64, P]
        lib.orc_splitmix64_next.argtypes = [P]
        lib.orc_splitmix64_next.restype = u64
        lib.orc_seed_from_master.argtypes = [u64, P]
        lib.orc_splitmix64_at.argtypes = [u64, u64]
        lib.orc_splitmix64_at.restype = u64
        lib.orc_random_spacing.argtypes = [u64, u64, u64, P]
        lib.orc_random_spacing.restype = None
        lib.orc_philox_constants.argtypes = [P]
        lib.orc_philox4x32_10.argtypes = [P, P, P]
        lib.orc_philox_next.argtypes = [P]
        lib.orc_philox_next.restype = ctypes.c_uint32
        lib.orc_philox_to_f32.argtypes = [ctypes.c_uint32]
        lib.orc_philox_to_f32.restype = ctypes.c_float
        lib.orc_philox_to_f64.argtypes = [ctypes.c_uint32]
        lib.orc_philox_to_f64.restype = ctypes.c_double
        lib.orc_philox_fill.argtypes = [P, u64, u64, ctypes.c_int, ctypes.c_int, P]
        lib.orc_philox_fill.restype = None
        lib.orc_philox_streams.argtypes = [u64, u64, u64, P]
        lib.orc_philox_streams.restype = None
        lib.orc_state_valid.argtypes = [P]
        lib.orc_state_valid.restype = ctypes.c_int
        _lib = lib
        return lib


def _ptr(a: np.ndarray) -> int:
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data


def _exp_words(e: int) -> np.ndarray:
    """A non-negative exponent below 2^192 as 3 little-endian uint64 words."""
    if not (0 <= e < 1 << 192):
        raise ValueError("exponent out of [0, 2^192)")
    return np.array([(e >> (64 * i)) & ((1 << 64) - 1) for i in range(3)], dtype=np.uint64)


def _state(s) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(s, dtype=np.uint32).reshape(-1))


# --------------------------------------------------------------------------
# Public oracle functions.  States are [6] or [S, 6] uint32 arrays in the
# order (x1[n-3], x1[n-2], x1[n-1], x2[n-3], x2[n-2], x2[n-1]).
# --------------------------------------------------------------------------
def step(state: np.ndarray) -> int:
    """Advance ``state`` (a writable [6] uint32 array) in place; return z'."""
    assert state.dtype == np.uint32 and state.shape == (6,) and state.flags["C_CONTIGUOUS"]
    return int(_load().orc_step(_ptr(state)))


def to_f64(z: int) -> float:
    return float(_load().orc_to_f64(int(z)))


def to_f32(z: int) -> float:
    return float(np.float32(_load().orc_to_f32(int(z))))


def fill(states, n: int, dtype: int = U32, layout: int = STREAM_MAJOR):
    """Return (out, advanced_states).  ``out`` is [S, n] (stream-major) or
    [n, S] (interleaved) of the dtype; states are not modified in place."""
    st = np.array(states, dtype=np.uint32, copy=True).reshape(-1, 6)
    st = np.ascontiguousarray(st)
    S = st.shape[0]
    shape = (S, n) if layout == STREAM_MAJOR else (n, S)
    out = np.empty(shape, dtype=_DTYPES[dtype])
    _load().orc_fill(_ptr(st), S, n, dtype, layout, _ptr(out) if out.size else None)
    return out, st


def skip(state, k: int) -> np.ndarray:
    """State advanced by k single steps (brute force)."""
    st = _state(state).copy()
    _load().orc_skip(_ptr(st), int(k))
    return st


def companion(comp: int) -> np.ndarray:
    A = np.zeros(9, dtype=np.uint32)
    _load().orc_companion(comp, _ptr(A))
    return A.reshape(3, 3)


def matpow(comp: int, e: int) -> np.ndarray:
    """A_comp^e mod m_comp for 0 <= e < 2^192 (C oracle)."""
    R = np.zeros(9, dtype=np.uint32)
    w = _exp_words(e)
    _load().orc_matpow(comp, _ptr(w), _ptr(R))
    return R.reshape(3, 3)


def jump(state, e: int) -> np.ndarray:
    st = _state(state).copy()
    w = _exp_words(e)
    _load().orc_jump(_ptr(st), _ptr(w))
    return st


def jump_many(states, exps) -> np.ndarray:
    """Jump each of S states by its own exponent (python ints < 2^192) or,
    when ``exps`` is a single int, all by that one."""
    st = np.array(states, dtype=np.uint32, copy=True).reshape(-1, 6)
    st = np.ascontiguousarray(st)
    if isinstance(exps, (int, np.integer)):
        w = _exp_words(int(exps))
        _load().orc_jump_many(_ptr(st), st.shape[0], _ptr(w), 0)
    else:
        w = np.ascontiguousarray(np.stack([_exp_words(int(e)) for e in exps]).reshape(-1))
        assert w.size == 3 * st.shape[0]
        _load().orc_jump_many(_ptr(st), st.shape[0], _ptr(w), 1)
    return st


def jump_many_words(states, words: np.ndarray) -> np.ndarray:
    """As ``jump_many`` with exponents given as a [S, 3] uint64 array."""
    st = np.array(states, dtype=np.uint32, copy=True).reshape(-1, 6)
    st = np.ascontiguousarray(st)
    w = np.ascontiguousarray(np.asarray(words, dtype=np.uint64).reshape(-1))
    assert w.size == 3 * st.shape[0]
    _load().orc_jump_many(_ptr(st), st.shape[0], _ptr(w), 1)
    return st


def stream_start(base, g: int) -> np.ndarray:
    out = np.zeros(6, dtype=np.uint32)
    _load().orc_stream_start(_ptr(_state(base)), int(g), _ptr(out))
    return out


def streams(base, first: int, count: int) -> np.ndarray:
    out = np.zeros((count, 6), dtype=np.uint32)
    if count:
        _load().orc_streams(_ptr(_state(base)), int(first), int(count), _ptr(out))
    return out


def streams_adjacent(base, first: int, count: int) -> np.ndarray:
    """As ``streams``, each start after the first computed from the previous
    one (one product by A^(2^127)): for millions of streams."""
    out = np.zeros((count, 6), dtype=np.uint32)
    if count:
        _load().orc_streams_adjacent(_ptr(_state(base)), int(first), int(count), _ptr(out))
    return out


def jump_uniform(states, e: int) -> np.ndarray:
    """Every state jumped by the one exponent e (A^e formed once)."""
    st = np.ascontiguousarray(np.array(states, dtype=np.uint32, copy=True).reshape(-1, 6))
    w = _exp_words(int(e))
    _load().orc_jump_uniform(_ptr(st), st.shape[0], _ptr(w))
    return st


def splitmix64(seed: int, count: int) -> list:
    x = np.array([seed], dtype=np.uint64)
    lib = _load()
    return [int(lib.orc_splitmix64_next(_ptr(x))) for _ in range(count)]


def seed_from_master(master: int) -> np.ndarray:
    out = np.zeros(6, dtype=np.uint32)
    _load().orc_seed_from_master(int(master), _ptr(out))
    return out


def splitmix64_at(seed: int, k: int) -> int:
    """Output number k of SplitMix64 seeded with ``seed``."""
    return int(_load().orc_splitmix64_at(int(seed), int(k)))


def random_spacing_states(master: int, first: int, count: int) -> np.ndarray:
    """Random spacing (sec. 2.3): [count, 6] start states of streams
    first .. first+count-1, stream g started from the state expanded from
    SplitMix64 output g of ``master`` (as ``seed_from_master`` expands a
    seed)."""
    out = np.zeros((count, 6), dtype=np.uint32)
    if count:
        _load().orc_random_spacing(int(master), int(first), int(count), _ptr(out))
    return out


def leapfrog(state, players: int, per_player: int, dtype: int = U32,
             layout: int = STREAM_MAJOR):
    """Leapfrog (sec. 2.3): the outputs of one stream dealt to ``players``
    players like cards, ``per_player`` each: card k of player t is output
    t + k * players of the stream.  Returns (out, advanced_state): out is
    [players, per_player] (STREAM_MAJOR: each player's cards in a row) or
    [per_player, players] (INTERLEAVED: the stream's outputs in order)."""
    seq, end = fill(_state(state), players * per_player, dtype, STREAM_MAJOR)
    dealt = seq.reshape(per_player, players)  # row k: card k of every player
    if layout == STREAM_MAJOR:
        dealt = np.ascontiguousarray(dealt.T)
    return dealt, end.reshape(6)


# --------------------------------------------------------------------------
# Philox4x32-10 streams.  A state is (position lo, hi, stream id lo, hi,
# key lo, hi); output number `position` is word position % 4 of the block
# whose counter is (position // 4, stream id).
# --------------------------------------------------------------------------
def philox_constants() -> list:
    """[M0, M1, W0, W1]: the two round multipliers and the two Weyl key
    increments."""
    out = np.zeros(4, dtype=np.uint32)
    _load().orc_philox_constants(_ptr(out))
    return [int(v) for v in out]


def philox4x32_10(ctr, key) -> list:
    c = np.ascontiguousarray(np.asarray(ctr, dtype=np.uint32).reshape(4))
    k = np.ascontiguousarray(np.asarray(key, dtype=np.uint32).reshape(2))
    out = np.zeros(4, dtype=np.uint32)
    _load().orc_philox4x32_10(_ptr(c), _ptr(k), _ptr(out))
    return [int(v) for v in out]


def philox_streams(key: int, first: int, count: int) -> np.ndarray:
    out = np.zeros((count, 6), dtype=np.uint32)
    if count:
        _load().orc_philox_streams(int(key), int(first), int(count), _ptr(out))
    return out


def philox_to_f32(w: int) -> float:
    return float(np.float32(_load().orc_philox_to_f32(int(w))))


def philox_to_f64(w: int) -> float:
    return float(_load().orc_philox_to_f64(int(w)))


def philox_fill(states, n: int, dtype: int = U32, layout: int = STREAM_MAJOR):
    """As ``fill`` for Philox stream states."""
    st = np.ascontiguousarray(np.array(states, dtype=np.uint32, copy=True).reshape(-1, 6))
    S = st.shape[0]
    shape = (S, n) if layout == STREAM_MAJOR else (n, S)
    out = np.empty(shape, dtype=_DTYPES[dtype])
    _load().orc_philox_fill(_ptr(st), S, n, dtype, layout, _ptr(out) if out.size else None)
    return out, st


def philox_jump(states, e) -> np.ndarray:
    """Philox states moved e outputs ahead (e an int, or one per state); the
    position wraps at 2^64."""
    st = np.array(states, dtype=np.uint32, copy=True).reshape(-1, 6)
    es = [int(e)] * st.shape[0] if isinstance(e, (int, np.integer)) else [int(x) for x in e]
    for i, x in enumerate(es):
        pos = (int(st[i, 0]) | int(st[i, 1]) << 32) + x
        pos &= (1 << 64) - 1
        st[i, 0], st[i, 1] = pos & 0xFFFFFFFF, pos >> 32
    return st


def state_valid(state) -> bool:
    return bool(_load().orc_state_valid(_ptr(_state(state))))
