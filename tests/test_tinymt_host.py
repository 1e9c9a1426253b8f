"""The library's TinyMT32 arithmetic (include/tinymt_arith.hpp), compiled for
the host with g++, against the CPU oracle: draws, the published seeding, the
parameter search's decisions and characteristic polynomials, the jump tables
and jumps, and the stream placement of the sec. 4.2 hybrid (parameter sets
shared by groups of streams, sub-streams 2^64 apart).  Runs on the CPU and
validates the arithmetic before any GPU run."""
import ctypes
import os
import random
import subprocess

import numpy as np
import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "host_arith", "tinymt_shim.cpp")
INC = os.path.join(ROOT, "include")
P = ctypes.c_void_p


@pytest.fixture(scope="module")
def shim(tmp_path_factory):
    out = str(tmp_path_factory.mktemp("tshim") / "tinymt_shim.so")
    subprocess.check_call(["g++", "-O2", "-std=c++17", "-fPIC", "-shared", "-I", INC, SRC,
                           "-o", out])
    lib = ctypes.CDLL(out)
    lib.tshim_draw.argtypes = [P, P, ctypes.c_uint64, P]
    lib.tshim_seed.argtypes = [ctypes.c_uint32, P, P]
    lib.tshim_candidate.argtypes = [ctypes.c_uint64, ctypes.c_uint64, P]
    lib.tshim_charpoly.argtypes = [P, P]
    lib.tshim_charpoly.restype = ctypes.c_int
    lib.tshim_irreducible.argtypes = [P]
    lib.tshim_irreducible.restype = ctypes.c_int
    lib.tshim_params_ok.argtypes = [P]
    lib.tshim_params_ok.restype = ctypes.c_int
    lib.tshim_mulmod.argtypes = [P, P, P, P]
    lib.tshim_pow_table.argtypes = [P, P]
    lib.tshim_jump.argtypes = [P, P, P, P, P]
    lib.tshim_to_f32.argtypes = [ctypes.c_uint32]
    lib.tshim_to_f32.restype = ctypes.c_float
    lib.tshim_to_f64.argtypes = [ctypes.c_uint32]
    lib.tshim_to_f64.restype = ctypes.c_double
    return lib


def _p(a):
    return a.ctypes.data


def u32(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.uint32))


def poly_u32(f: int) -> np.ndarray:
    return np.array([(f >> (32 * i)) & 0xFFFFFFFF for i in range(4)], dtype=np.uint32)


def u32_poly(w) -> int:
    return sum(int(x) << (32 * i) for i, x in enumerate(w))


def params(master, count):
    return oracle.tmt_search(master, count)


def test_draws_and_seeding_match_oracle(shim):
    rng = random.Random(1)
    P_, _ = params(21, 3)
    for p in P_:
        p = u32(p)
        for seed in [0, 1, 12345, 0xFFFFFFFF, rng.getrandbits(32)]:
            s = np.zeros(4, dtype=np.uint32)
            shim.tshim_seed(seed, _p(p), _p(s))
            assert np.array_equal(s, oracle.tmt_init(seed, p)), seed
            want, wst = oracle.tmt_outputs(s, p, 300)
            got = np.zeros(300, dtype=np.uint32)
            shim.tshim_draw(_p(s), _p(p), 300, _p(got))
            assert np.array_equal(got, want)
            assert np.array_equal(s, wst)


def test_conversions_match_oracle(shim):
    rng = random.Random(2)
    for w in [0, 1, 511, 512, 0x7FFFFFFF, 0x80000000, 0xFFFFFFFE, 0xFFFFFFFF] + \
            [rng.getrandbits(32) for _ in range(2000)]:
        assert shim.tshim_to_f32(w) == oracle._load().orc_tmt_to_f32(w)
        assert shim.tshim_to_f64(w) == oracle._load().orc_tmt_to_f64(w)


def test_candidates_and_search_decisions_match_oracle(shim):
    """Every candidate's linear complexity, characteristic polynomial and
    accept decision over a run of 400 candidates (a few accepted)."""
    master = 0x1234
    kept = 0
    for c in range(400):
        p = np.zeros(3, dtype=np.uint32)
        shim.tshim_candidate(master, c, _p(p))
        assert np.array_equal(p, oracle.tmt_candidate(master, c))
        phi = np.zeros(4, dtype=np.uint32)
        L = shim.tshim_charpoly(_p(p), _p(phi))
        Lw, phiw = oracle.tmt_charpoly(p)
        assert L == Lw, c
        if L == 127:  # the only degree kept (phi is written for it alone)
            assert u32_poly(phi) == phiw, c
        else:
            assert u32_poly(phi) == 0, c
        ok = shim.tshim_params_ok(_p(p))
        assert ok == oracle.tmt_params_ok(p), c
        kept += ok
    assert kept >= 1


def test_irreducibility_matches_oracle_on_built_polynomials(shim):
    rng = random.Random(3)
    cases = [(1 << 127) | 3, (1 << 127) | 1, (1 << 127) | (1 << 63) | 1]
    for _ in range(40):
        cases.append((1 << 127) | rng.getrandbits(127) | 1)
    for _ in range(10):  # (x^2 + x + 1) * g: reducible without a root
        g = (1 << 125) | rng.getrandbits(125) | 1
        cases.append(g ^ (g << 1) ^ (g << 2))
    for f in cases:
        pf = poly_u32(f)
        assert shim.tshim_irreducible(_p(pf)) == oracle.gf2_irreducible_prime_degree(f), hex(f)


def clmul_mod(a, b, f):
    r = 0
    while b:
        if b & 1:
            r ^= a
        b >>= 1
        a <<= 1
    d = f.bit_length() - 1
    while r and r.bit_length() - 1 >= d:
        r ^= f << (r.bit_length() - 1 - d)
    return r


def test_mulmod_and_pow_table(shim):
    rng = random.Random(4)
    P_, _ = params(5, 2)
    for p in P_:
        _, phi = oracle.tmt_charpoly(p)
        for _ in range(30):
            a, b = rng.getrandbits(127), rng.getrandbits(127)
            r = np.zeros(4, dtype=np.uint32)
            pa, pb, pf = poly_u32(a), poly_u32(b), poly_u32(phi)  # kept alive over the call
            shim.tshim_mulmod(_p(pa), _p(pb), _p(pf), _p(r))
            assert u32_poly(r) == clmul_mod(a, b, phi)
        pw = np.zeros(192 * 4, dtype=np.uint32)
        pf = poly_u32(phi)
        shim.tshim_pow_table(_p(pf), _p(pw))
        t = 2
        for i in range(192):
            assert u32_poly(pw[4 * i:4 * i + 4]) == t, i
            t = clmul_mod(t, t, phi)


def test_jumps_match_oracle(shim):
    rng = random.Random(5)
    P_, _ = params(8, 2)
    for p in P_:
        p = u32(p)
        _, phi = oracle.tmt_charpoly(p)
        phw = poly_u32(phi)
        pw = np.zeros(192 * 4, dtype=np.uint32)
        shim.tshim_pow_table(_p(phw), _p(pw))
        s0 = oracle.tmt_init(rng.getrandbits(32), p)
        exps = [0, 1, 2, 3, 127, 128, 1 << 64, (1 << 64) * 5, (1 << 127) - 1, (1 << 127),
                (1 << 128) - 1] + [rng.getrandbits(128) for _ in range(10)]
        for e in exps:
            s = s0.copy()
            ew = np.array([e & (2**64 - 1), e >> 64, 0], dtype=np.uint64)
            shim.tshim_jump(_p(s), _p(p), _p(phw), _p(pw), _p(ew))
            assert np.array_equal(s, oracle.tmt_jump(s0, p, e)), e
        # exponents past 2^128 agree with the oracle's at e mod (2^127 - 1)
        # (the period), whenever that is at least 1
        for _ in range(6):
            e = rng.getrandbits(191) | 1 << 150
            er = e % ((1 << 127) - 1)
            s = s0.copy()
            ew = np.array([e & (2**64 - 1), (e >> 64) & (2**64 - 1), e >> 128], dtype=np.uint64)
            shim.tshim_jump(_p(s), _p(p), _p(phw), _p(pw), _p(ew))
            assert er >= 1 and np.array_equal(s, oracle.tmt_jump(s0, p, er)), e


def test_stream_starts_match_oracle(shim):
    """Start of stream g: set q = g // per, seeded from SplitMix64 output q,
    jumped (g % per) * 2^64."""
    master, per = 0xABCDEF, 7
    P_, _ = params(master, 3)
    want = oracle.tmt_streams(master, per, 3, 17, P_)
    for i in range(17):
        g = 3 + i
        q, j = g // per, g % per
        p = u32(P_[q])
        s = np.zeros(4, dtype=np.uint32)
        shim.tshim_seed(oracle.splitmix64_at(master, q) & 0xFFFFFFFF, _p(p), _p(s))
        _, phi = oracle.tmt_charpoly(p)
        pf = poly_u32(phi)
        pw = np.zeros(192 * 4, dtype=np.uint32)
        shim.tshim_pow_table(_p(pf), _p(pw))
        ew = np.array([0, j, 0], dtype=np.uint64)
        shim.tshim_jump(_p(s), _p(p), _p(pf), _p(pw), _p(ew))
        assert np.array_equal(s, want[i, :4]), g
        assert want[i, 4] == q and want[i, 5] == 0
