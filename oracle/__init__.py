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
_SRCS = [_SRC, os.path.join(_HERE, "tinymt_oracle.c")]
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
    stale = not os.path.exists(_LIB) or any(
        os.path.getmtime(_LIB) < os.path.getmtime(src) for src in _SRCS)
    if force or stale:
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call([
            "gcc", "-O2", "-std=c99", "-ffp-contract=off", "-fno-fast-math",
            "-fPIC", "-shared", "-o", tmp, *_SRCS,
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
        lib.orc_tmt_next.argtypes = [P, P]
        lib.orc_tmt_next.restype = None
        lib.orc_tmt_temper.argtypes = [P, P]
        lib.orc_tmt_temper.restype = ctypes.c_uint32
        lib.orc_tmt_draw.argtypes = [P, P]
        lib.orc_tmt_draw.restype = ctypes.c_uint32
        lib.orc_tmt_init.argtypes = [ctypes.c_uint32, P, P]
        lib.orc_tmt_init.restype = None
        lib.orc_gf2_irreducible_prime_degree.argtypes = [P]
        lib.orc_gf2_irreducible_prime_degree.restype = ctypes.c_int
        lib.orc_gf2_berlekamp_massey.argtypes = [P, ctypes.c_int, P]
        lib.orc_gf2_berlekamp_massey.restype = ctypes.c_int
        lib.orc_tmt_charpoly.argtypes = [P, P]
        lib.orc_tmt_charpoly.restype = ctypes.c_int
        lib.orc_tmt_params_ok.argtypes = [P]
        lib.orc_tmt_params_ok.restype = ctypes.c_int
        lib.orc_tmt_jump.argtypes = [P, P, P, P]
        lib.orc_tmt_jump.restype = None
        lib.orc_tmt_skip.argtypes = [P, P, u64]
        lib.orc_tmt_skip.restype = None
        lib.orc_tmt_candidate.argtypes = [u64, u64, P]
        lib.orc_tmt_candidate.restype = None
        lib.orc_tmt_search.argtypes = [u64, u64, P, P]
        lib.orc_tmt_search.restype = None
        lib.orc_tmt_streams.argtypes = [u64, u64, u64, u64, P, u64, P]
        lib.orc_tmt_streams.restype = None
        lib.orc_tmt_to_f32.argtypes = [ctypes.c_uint32]
        lib.orc_tmt_to_f32.restype = ctypes.c_float
        lib.orc_tmt_to_f64.argtypes = [ctypes.c_uint32]
        lib.orc_tmt_to_f64.restype = ctypes.c_double
        lib.orc_tmt_fill.argtypes = [P, u64, u64, ctypes.c_int, ctypes.c_int, P, u64, P]
        lib.orc_tmt_fill.restype = None
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


# --------------------------------------------------------------------------
# TinyMT32 (sec. 4.2): states [4] uint32 (s0..s3) for the generator
# functions; stream-set states [S, 6] = (s0, s1, s2, s3, parameter set, 0).
# Parameter sets are [3] uint32 (mat1, mat2, tmat).  Polynomials over GF(2)
# are Python ints (bit i = coefficient of x^i).
# --------------------------------------------------------------------------
def _u32a(a, n) -> np.ndarray:
    out = np.ascontiguousarray(np.asarray(a, dtype=np.uint32).reshape(-1))
    assert out.size == n
    return out


def _poly_words(f: int) -> np.ndarray:
    return np.array([(f >> (64 * i)) & ((1 << 64) - 1) for i in range(4)], dtype=np.uint64)


def _words_poly(w: np.ndarray) -> int:
    return sum(int(x) << (64 * i) for i, x in enumerate(w))


def tmt_next(state, params) -> np.ndarray:
    s = _u32a(state, 4).copy()
    _load().orc_tmt_next(_ptr(s), _ptr(_u32a(params, 3)))
    return s


def tmt_temper(state, params) -> int:
    return int(_load().orc_tmt_temper(_ptr(_u32a(state, 4)), _ptr(_u32a(params, 3))))


def tmt_init(seed: int, params) -> np.ndarray:
    s = np.zeros(4, dtype=np.uint32)
    _load().orc_tmt_init(int(seed) & 0xFFFFFFFF, _ptr(_u32a(params, 3)), _ptr(s))
    return s


def tmt_outputs(state, params, n: int):
    """(n uint32 outputs, state after them) from a [4] state."""
    s = _u32a(state, 4).copy()
    p = _u32a(params, 3)
    lib = _load()
    out = np.array([lib.orc_tmt_draw(_ptr(s), _ptr(p)) for _ in range(n)], dtype=np.uint32)
    return out, s


def gf2_irreducible_prime_degree(f: int) -> bool:
    return bool(_load().orc_gf2_irreducible_prime_degree(_ptr(_poly_words(f))))


def gf2_berlekamp_massey(bits):
    """(L, C) for a sequence of 0/1 values (at most 255 of them); C as an int."""
    a = np.ascontiguousarray(np.asarray(bits, dtype=np.uint8))
    w = np.zeros(4, dtype=np.uint64)
    L = _load().orc_gf2_berlekamp_massey(_ptr(a), int(a.size), _ptr(w))
    return int(L), _words_poly(w)


def tmt_charpoly(params):
    """(degree, phi) of the parameter set's transition."""
    w = np.zeros(4, dtype=np.uint64)
    L = _load().orc_tmt_charpoly(_ptr(_u32a(params, 3)), _ptr(w))
    return int(L), _words_poly(w)


def tmt_params_ok(params) -> bool:
    return bool(_load().orc_tmt_params_ok(_ptr(_u32a(params, 3))))


def tmt_jump(state, params, e: int) -> np.ndarray:
    """T^e state for 0 <= e < 2^128."""
    assert 0 <= e < 1 << 128
    s = _u32a(state, 4).copy()
    p = _u32a(params, 3)
    _, phi = tmt_charpoly(p)
    ew = np.array([e & ((1 << 64) - 1), e >> 64], dtype=np.uint64)
    _load().orc_tmt_jump(_ptr(s), _ptr(p), _ptr(_poly_words(phi)), _ptr(ew))
    return s


def tmt_skip(state, params, k: int) -> np.ndarray:
    s = _u32a(state, 4).copy()
    _load().orc_tmt_skip(_ptr(s), _ptr(_u32a(params, 3)), int(k))
    return s


def tmt_candidate(master: int, c: int) -> np.ndarray:
    p = np.zeros(3, dtype=np.uint32)
    _load().orc_tmt_candidate(int(master), int(c), _ptr(p))
    return p


def tmt_search(master: int, count: int):
    """([count, 3] parameter sets, [count] candidate numbers) of master's search."""
    out = np.zeros((max(count, 1), 3), dtype=np.uint32)
    cand = np.zeros(max(count, 1), dtype=np.uint64)
    if count:
        _load().orc_tmt_search(int(master), int(count), _ptr(out), _ptr(cand))
    return out[:count], cand[:count]


def tmt_streams(master: int, per_param: int, first: int, count: int, params, q0: int = 0):
    """[count, 6] start states of streams first .. first+count-1 of a TinyMT
    stream set (params: sets q0, q0 + 1, ... of master's search)."""
    pr = np.ascontiguousarray(np.asarray(params, dtype=np.uint32).reshape(-1))
    out = np.zeros((max(count, 1), 6), dtype=np.uint32)
    if count:
        _load().orc_tmt_streams(int(master), int(per_param), int(first), int(count), _ptr(pr),
                                int(q0), _ptr(out))
    return out[:count]


def tmt_fill(states, n: int, dtype: int, layout: int, params, q0: int = 0):
    """(out, advanced states) as ``fill`` for TinyMT stream-set states."""
    st = np.ascontiguousarray(np.array(states, dtype=np.uint32, copy=True).reshape(-1, 6))
    S = st.shape[0]
    pr = np.ascontiguousarray(np.asarray(params, dtype=np.uint32).reshape(-1))
    shape = (S, n) if layout == STREAM_MAJOR else (n, S)
    out = np.empty(shape, dtype=_DTYPES[dtype])
    _load().orc_tmt_fill(_ptr(st), S, n, dtype, layout, _ptr(pr), int(q0),
                         _ptr(out) if out.size else None)
    return out, st
