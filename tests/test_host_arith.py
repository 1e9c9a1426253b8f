"""The library's device arithmetic (include/mrg_arith.hpp), compiled for the host
with g++, against the CPU oracle.  Both formulations (32-bit integer with
lazy residues, binary64 with centred residues) are stepped from random and
boundary states and compared output by output; the combination and
canonicalisation helpers are checked exhaustively around their boundaries.
This runs on the CPU and validates the arithmetic before any GPU run."""
import ctypes
import os
import random
import subprocess

import numpy as np
import pytest

import oracle
from oracle import ref

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "host_arith", "arith_shim.cpp")
INC = os.path.join(ROOT, "include")
M1, M2 = oracle.M1, oracle.M2


@pytest.fixture(scope="module")
def shim(tmp_path_factory):
    out = str(tmp_path_factory.mktemp("shim") / "arith_shim.so")
    subprocess.check_call(["g++", "-O2", "-std=c++17", "-ffp-contract=off", "-fPIC", "-shared",
                           "-I", INC, SRC, "-o", out])
    lib = ctypes.CDLL(out)
    P = ctypes.c_void_p
    lib.shim_run_int.argtypes = [P, ctypes.c_uint64, P]
    lib.shim_run_f64.argtypes = [P, ctypes.c_uint64, P, P, P]
    lib.shim_combine.argtypes = [ctypes.c_uint32, ctypes.c_uint32]
    lib.shim_combine.restype = ctypes.c_uint32
    lib.shim_combinef.argtypes = [ctypes.c_double, ctypes.c_double]
    lib.shim_combinef.restype = ctypes.c_double
    lib.shim_combinef_nn.argtypes = [ctypes.c_double, ctypes.c_double]
    lib.shim_combinef_nn.restype = ctypes.c_double
    lib.shim_hi_word.argtypes = [ctypes.c_double]
    lib.shim_hi_word.restype = ctypes.c_uint32
    lib.shim_run_f64_checked.argtypes = [P, ctypes.c_uint64, ctypes.c_uint64, P]
    lib.shim_run_f64_checked.restype = ctypes.c_uint64
    for n in ("shim_next1f", "shim_next2f"):
        getattr(lib, n).argtypes = [ctypes.c_double, ctypes.c_double]
        getattr(lib, n).restype = ctypes.c_double
    for n in ("shim_canon1", "shim_canon2"):
        getattr(lib, n).argtypes = [ctypes.c_uint32]
        getattr(lib, n).restype = ctypes.c_uint32
    lib.shim_canonf.argtypes = [ctypes.c_double, ctypes.c_int]
    lib.shim_canonf.restype = ctypes.c_uint32
    lib.shim_to_f32.argtypes = [ctypes.c_uint32]
    lib.shim_to_f32.restype = ctypes.c_float
    lib.shim_to_f64.argtypes = [ctypes.c_uint32]
    lib.shim_to_f64.restype = ctypes.c_double
    lib.shim_to_f32f.argtypes = [ctypes.c_double]
    lib.shim_to_f32f.restype = ctypes.c_float
    lib.shim_dot3.argtypes = [ctypes.c_int, P, P]
    lib.shim_dot3.restype = ctypes.c_uint32
    return lib


def _states():
    rng = random.Random(7)
    edge1 = [0, 1, 2, M1 - 2, M1 - 1, (M1 - 1) // 2, (M1 + 1) // 2]
    edge2 = [0, 1, 2, M2 - 2, M2 - 1, (M2 - 1) // 2, (M2 + 1) // 2]
    out = []
    for _ in range(150):
        a = [rng.choice(edge1) if rng.random() < 0.5 else rng.randrange(M1) for _ in range(3)]
        b = [rng.choice(edge2) if rng.random() < 0.5 else rng.randrange(M2) for _ in range(3)]
        if not any(a):
            a[0] = 1
        if not any(b):
            b[0] = 1
        out.append(np.array(a + b, dtype=np.uint32))
    return out


def _p(a):
    return a.ctypes.data


def test_integer_formulation_matches_oracle(shim):
    n = 400
    for s in _states():
        want, st = oracle.fill(s[None, :], n, oracle.U32)
        w = s.copy()
        got = np.empty(n, dtype=np.uint32)
        shim.shim_run_int(_p(w), n, _p(got))
        assert np.array_equal(got, want[0])
        canon = [shim.shim_canon1(int(x)) for x in w[:3]] + [shim.shim_canon2(int(x)) for x in w[3:]]
        assert canon == [int(x) for x in st[0]]


def test_integer_formulation_accepts_lazy_words(shim):
    # words in [m, 2^32) are representatives of x - m: same outputs
    rng = random.Random(8)
    for _ in range(100):
        a = [rng.randrange(0, 208) for _ in range(3)]
        b = [rng.randrange(0, 22852) for _ in range(3)]
        a[0] |= 1
        b[0] |= 1
        canon = np.array(a + b, dtype=np.uint32)
        lazy = np.array([x + M1 for x in a] + [x + M2 for x in b], dtype=np.uint32)
        want, _ = oracle.fill(canon[None, :], 50, oracle.U32)
        got = np.empty(50, dtype=np.uint32)
        shim.shim_run_int(_p(lazy), 50, _p(got))
        assert np.array_equal(got, want[0])


def test_binary64_formulation_matches_oracle(shim):
    n = 400
    for s in _states():
        want, st = oracle.fill(s[None, :], n, oracle.U32)
        wf, _ = oracle.fill(s[None, :], n, oracle.F32)
        wd, _ = oracle.fill(s[None, :], n, oracle.F64)
        w = s.copy()
        got = np.empty(n, dtype=np.uint32)
        gf = np.empty(n, dtype=np.float32)
        gd = np.empty(n, dtype=np.float64)
        shim.shim_run_f64(_p(w), n, _p(got), _p(gf), _p(gd))
        assert np.array_equal(got, want[0])
        assert np.array_equal(gf.view(np.uint32), wf[0].view(np.uint32))
        assert np.array_equal(gd.view(np.uint64), wd[0].view(np.uint64))
        assert np.array_equal(w, st[0])


def test_combine_boundaries(shim):
    xs1 = [0, 1, 2, 208, 209, 210, 22643, 22644, 22645, 22852, 22853, M2 - 1, M2, M2 + 1,
           M1 - 1, M1, M1 + 1, 2**32 - 2, 2**32 - 1, 2**31, 12345]
    for x1 in xs1:
        for x2 in xs1:
            c1, c2 = x1 % M1, x2 % M2
            z = (c1 - c2) % M1 or M1
            assert shim.shim_combine(x1, x2) == z, (x1, x2)


def test_combinef_boundaries(shim):
    # near-canonical representatives: r1 in [-5, m1), r2 in [-5, m2)
    r1s = [-5, -4, -1, 0, 1, 2, 22643, 22644, 22645, M2 - 1, M2, M1 - 2, M1 - 1, 2**31, 12345]
    r2s = [-5, -1, 0, 1, 22644, M2 - 2, M2 - 1, 2**31, 12345]
    for r1 in r1s:
        for r2 in r2s:
            z = ((r1 % M1) - (r2 % M2)) % M1 or M1
            assert shim.shim_combinef(float(r1), float(r2)) == float(z), (r1, r2)
    # equal residues give m1
    assert shim.shim_combinef(0.0, 0.0) == float(M1)
    assert shim.shim_combinef(float(M2 - 1), -1.0) == float(M1)
    for r in (-5, -1, 0, 1, M1 - 1):
        assert shim.shim_canonf(float(r), 0) == r % M1
    for r in (-5, -1, 0, 1, M2 - 1):
        assert shim.shim_canonf(float(r), 1) == r % M2


def test_checked_combination(shim):
    """The three-operation combination equals the exact one whenever the
    component-2 word is non-negative, and the sign bit of its high word
    flags every negative one (the case it gets wrong)."""
    rng = random.Random(13)
    r1s = ([-5, -4, -1, 0, 1, 2, 22643, 22644, 22645, M2 - 1, M2, M1 - 2, M1 - 1, 2**31]
           + [rng.randrange(-5, M1) for _ in range(300)])
    r2s = ([-5, -4, -3, -2, -1, 0, 1, 2, 22644, M2 - 2, M2 - 1, 2**31]
           + [rng.randrange(-5, M2) for _ in range(300)])
    for r1 in r1s:
        for r2 in r2s:
            flagged = shim.shim_hi_word(float(r2)) >> 31
            assert flagged == (r2 < 0), (r1, r2)
            if r2 >= 0:
                assert shim.shim_combinef_nn(float(r1), float(r2)) == \
                    shim.shim_combinef(float(r1), float(r2)), (r1, r2)


def test_checked_draws_redraw_exactly_where_needed(shim):
    """Streams steered so that output k draws the component-2 residue m2 - 1
    or m2 - 2 (where the binary64 reduction's biased quotient is one too big,
    so the word comes out negative): the checked run flags those blocks,
    draws them again and matches the oracle; untouched streams never redraw."""
    from tests import crafted
    n, block = 300, 32
    positions = [0, 1, 2, 31, 32, 33, 95, 150, 255, 299]
    starts = crafted.hits(positions, [M2 - 1, M2 - 2], seed=5)
    for k, s in zip(positions, starts):
        # the kernel arithmetic itself: the word drawn at output k is negative
        w = s.copy()
        got = np.empty(n, dtype=np.uint32)
        if k:
            gf, gd = np.empty(k, np.float32), np.empty(k, np.float64)
            shim.shim_run_f64(_p(w), k, _p(got), _p(gf), _p(gd))
        assert shim.shim_next2f(float(w[3]), float(w[5])) < 0, k
        want, st = oracle.fill(s[None, :], n, oracle.U32)
        w = s.copy()
        redrawn = shim.shim_run_f64_checked(_p(w), n, block, _p(got))
        assert redrawn >= 1, k
        assert np.array_equal(got, want[0]), k
        assert np.array_equal(w, st[0]), k
    for s in _states()[:20]:
        want, _ = oracle.fill(s[None, :], n, oracle.U32)
        w = s.copy()
        got = np.empty(n, dtype=np.uint32)
        shim.shim_run_f64_checked(_p(w), n, block, _p(got))
        assert np.array_equal(got, want[0])


def test_binary64_reduction_at_quotient_boundaries(shim):
    """next1f/next2f on inputs whose product-sum has residue 0, 1, 2 or m-1 ..
    m-6 (where a rounded quotient can be off by one), at the largest and
    smallest product-sums the input range allows: the result must be an
    exact representative in [-5, m)."""
    rng = random.Random(12)
    for comp, m, a, b, f in ((0, M1, 1403580, 810728, shim.shim_next1f),
                             (1, M2, 527612, 1370589, shim.shim_next2f)):
        ainv = pow(a, -1, m)
        olds = [-5, -1, 0, 1, m - 1, m - 2, (m - 1) // 2] + [rng.randrange(m) for _ in range(40)]
        targets = [0, 1, 2, 3, m - 1, m - 2, m - 3, m - 4, m - 5, m - 6, m - 7]
        for s0 in olds:
            for tgt in targets:
                # a*s1 - b*s0 = tgt (mod m); also try s1 shifted to its extremes
                s1 = (tgt + b * s0) * ainv % m
                for s1r in {s1, s1 - m if s1 <= 5 else s1}:
                    r = f(float(s0), float(s1r))
                    assert r == int(r) and -5 <= r < m, (comp, s0, s1r, r)
                    assert int(r) % m == (a * s1r - b * s0) % m, (comp, s0, s1r, r)


def test_conversions_match_oracle(shim):
    rng = random.Random(9)
    zs = [1, 2, 511, 512, 513, M1 - 1, M1] + [rng.randrange(1, M1 + 1) for _ in range(5000)]
    for z in zs:
        assert shim.shim_to_f64(z) == oracle.to_f64(z)
        f = oracle.to_f32(z)
        assert shim.shim_to_f32(z) == f
        assert shim.shim_to_f32f(float(z)) == f


def test_dot3_matches_bigint(shim):
    rng = random.Random(10)
    for comp, m in ((0, M1), (1, M2)):
        for _ in range(2000):
            mm = np.array([rng.choice([0, 1, m - 1, 2**32 - 1, rng.randrange(2**32)]) for _ in range(3)],
                          dtype=np.uint32)
            x = np.array([rng.choice([0, 1, m - 1, 2**32 - 1, rng.randrange(2**32)]) for _ in range(3)],
                         dtype=np.uint32)
            want = sum(int(a) * int(b) for a, b in zip(mm, x)) % m
            assert shim.shim_dot3(comp, _p(mm), _p(x)) == want
