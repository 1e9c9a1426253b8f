"""Pins of the CPU oracle against what the mathematics and the paper fix.

Nothing here compares the oracle with a retyped copy of itself.  The pins are:

* number theory: the moduli are prime and each component's companion matrix
  has multiplicative order exactly m^3 - 1 (full period, sec. 4.1's "period of
  about 2^191"), checked with primes found by this file's own Miller-Rabin;
  planted lag, sign and digit mistakes fail it (about one cubic in six is
  primitive, so it cannot fix a multiplier alone: the worked example does);
* linear algebra: one step equals one companion-matrix product, and a jump by
  e equals e brute-force steps;
* the worked example in ``golden/worked_example_seed12345.txt`` (hand
  arithmetic from the published definition);
* stream and substream spacing of sec. 4.1: 2^64 streams of 2^127 numbers,
  substreams of 2^76 (2^51 substreams per stream);
* the floating-point conversions, evaluated in exact rational arithmetic;
* the SplitMix64 known-answer value used by the master-seed expansion, and
  its random access (output k) against the sequential generator;
* the two partitions of one sequence in sec. 2.3 beside sequence splitting:
  random spacing (each stream from its own expanded SplitMix64 draw) and the
  leapfrog deal (every card checked against the big-integer jump of
  ``oracle/ref.py``);
* Philox4x32-10: the Weyl key increments derived from sqrt(5) and sqrt(3),
  and the round wiring, key schedule and round count through an inverse
  written here from the round structure.  The two round multipliers have no
  closed form and no known-answer file is available: parity unpinned.
"""
import math
import os
import random
from fractions import Fraction

import numpy as np
import pytest

import oracle
from oracle import ref

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
M1, M2 = ref.M1, ref.M2


# --------------------------------------------------------------------------
# number theory helpers written here, independent of the oracle
# --------------------------------------------------------------------------
def is_prime(n: int) -> bool:
    """Deterministic Miller-Rabin for n < 3.3e24 (first 13 prime bases)."""
    if n < 2:
        return False
    small = [2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37, 41]
    for p in small:
        if n % p == 0:
            return n == p
    d, r = n - 1, 0
    while d % 2 == 0:
        d //= 2
        r += 1
    for a in small:
        x = pow(a, d, n)
        if x in (1, n - 1):
            continue
        for _ in range(r - 1):
            x = x * x % n
            if x == n - 1:
                break
        else:
            return False
    return True


def prime_factors(n: int) -> list:
    """Factor m^3 - 1 = (m - 1)(m^2 + m + 1) by trial division of m - 1 and a
    primality test of the big cofactor."""
    out = []
    d = 2
    while d * d <= n and d < 1 << 20:
        while n % d == 0:
            out.append(d)
            n //= d
        d += 1
    if n > 1:
        # remaining cofactor must itself be a product of primes we can test
        if is_prime(n):
            out.append(n)
        else:
            # split with Pollard rho (deterministic seed)
            stack = [n]
            while stack:
                v = stack.pop()
                if is_prime(v):
                    out.append(v)
                    continue
                f = _rho(v)
                stack += [f, v // f]
    return sorted(set(out))


def _rho(n: int) -> int:
    for c in range(1, 100):
        x = y = 2
        d = 1
        while d == 1:
            x = (x * x + c) % n
            y = (y * y + c) % n
            y = (y * y + c) % n
            d = math.gcd(abs(x - y), n)
        if d != n:
            return d
    raise AssertionError("rho failed")


I3 = np.eye(3, dtype=np.uint32)


# --------------------------------------------------------------------------
# constants: full period of each component (sec. 4.1)
# --------------------------------------------------------------------------
def test_moduli_are_prime():
    assert is_prime(M1) and is_prime(M2)
    assert M1 == 2**32 - 209 and M2 == 2**32 - 22853


@pytest.mark.parametrize("comp", [0, 1])
def test_component_has_full_period(comp):
    m = (M1, M2)[comp]
    order = m**3 - 1
    qs = prime_factors(order)
    prod = 1
    for q in qs:
        e = 0
        t = order
        while t % q == 0:
            t //= q
            e += 1
        prod *= q**e
    assert prod == order
    # C oracle and big-integer reference must both give A^(m^3-1) = I
    assert np.array_equal(oracle.matpow(comp, order), I3)
    assert ref.matpow(comp, order) == ref.identity()
    for q in qs:
        assert not np.array_equal(oracle.matpow(comp, order // q), I3), q
        assert ref.matpow(comp, order // q) != ref.identity(), q


def test_period_is_about_2_pow_191():
    # the combined period is lcm(m1^3-1, m2^3-1); sec. 4.1 quotes 2^191
    rho = (M1**3 - 1) * (M2**3 - 1) // math.gcd(M1**3 - 1, M2**3 - 1)
    assert rho == (M1**3 - 1) * (M2**3 - 1) // 2
    assert 190.99 < math.log2(rho) < 191.0


def _full_period_holds(matrix, m):
    """Order test of an arbitrary 3x3 matrix, used on planted mistakes."""
    def mp(M, e):
        R = ref.identity()
        B = [row[:] for row in M]
        while e:
            if e & 1:
                R = ref.matmul(R, B, m)
            B = ref.matmul(B, B, m)
            e >>= 1
        return R
    order = m**3 - 1
    if mp(matrix, order) != ref.identity():
        return False
    return all(mp(matrix, order // q) != ref.identity() for q in prime_factors(order))


def test_planted_mistakes_fail_the_period_pin():
    # About one cubic in six over F_m is primitive, so the order test alone
    # does not fix a multiplier exactly (a12 +- 1 happen to be primitive too;
    # the worked example below pins the exact values).  It does catch lag,
    # sign and most digit mistakes:
    good1, good2 = ref.companion(0), ref.companion(1)
    assert _full_period_holds(good1, M1) and _full_period_holds(good2, M2)
    bad = [row[:] for row in good1]          # a12 on x[n-1] instead of x[n-2]
    bad[2][1], bad[2][2] = 0, good1[2][1]
    assert not _full_period_holds(bad, M1)
    bad = [row[:] for row in good1]          # sign of the a13 term flipped
    bad[2][0] = 810728
    assert not _full_period_holds(bad, M1)
    bad = [row[:] for row in good1]          # a13 off by one
    bad[2][0] = M1 - 810729
    assert not _full_period_holds(bad, M1)
    bad = [row[:] for row in good2]          # a21 off by one
    bad[2][2] += 1
    assert not _full_period_holds(bad, M2)
    bad = [row[:] for row in good2]          # a21 on x[n-2] instead of x[n-1]
    bad[2][1], bad[2][2] = good2[2][2], 0
    assert not _full_period_holds(bad, M2)
    bad = [row[:] for row in good2]          # sign of the a23 term flipped
    bad[2][0] = 1370589
    assert not _full_period_holds(bad, M2)


# --------------------------------------------------------------------------
# step = companion matrix product; jump = brute force
# --------------------------------------------------------------------------
def _random_state(rng):
    return np.array([rng.randrange(1, M1) for _ in range(3)]
                    + [rng.randrange(1, M2) for _ in range(3)], dtype=np.uint32)


def test_step_equals_companion_product():
    rng = random.Random(11)
    A1 = oracle.companion(0).astype(object)
    A2 = oracle.companion(1).astype(object)
    for _ in range(200):
        s = _random_state(rng)
        v1 = [int(x) for x in s[:3]]
        v2 = [int(x) for x in s[3:]]
        want = [int(sum(A1[i, k] * v1[k] for k in range(3)) % M1) for i in range(3)] + \
               [int(sum(A2[i, k] * v2[k] for k in range(3)) % M2) for i in range(3)]
        t = s.copy()
        oracle.step(t)
        assert [int(x) for x in t] == want


def test_jump_equals_bruteforce_small_offsets():
    rng = random.Random(12)
    s = _random_state(rng)
    cur = s.copy()
    for e in range(0, 1001):
        assert np.array_equal(oracle.jump(s, e), cur), e
        oracle.step(cur)
    for _ in range(20):
        e = rng.randrange(0, 1 << 17)
        assert np.array_equal(oracle.jump(s, e), oracle.skip(s, e)), e


def test_jump_composes():
    rng = random.Random(13)
    s = _random_state(rng)
    for _ in range(10):
        a = rng.randrange(0, 1 << 100)
        b = rng.randrange(0, 1 << 90)
        assert np.array_equal(oracle.jump(oracle.jump(s, a), b), oracle.jump(s, a + b))
    # python big-integer reference agrees on large exponents
    for _ in range(5):
        e = rng.randrange(0, 1 << 191)
        assert [int(x) for x in oracle.jump(s, e)] == ref.jump([int(x) for x in s], e)


# --------------------------------------------------------------------------
# worked example (hand arithmetic)
# --------------------------------------------------------------------------
def _golden_rows():
    recs, outs = [], []
    with open(os.path.join(GOLDEN, "worked_example_seed12345.txt")) as f:
        for line in f:
            t = line.split()
            if not t or t[0].startswith("#"):
                continue
            if t[0] == "rec":
                recs.append(tuple(int(v) for v in t[1:]))
            elif t[0] == "out":
                outs.append((int(t[1]), int(t[2]), t[3], int(t[4])))
    return recs, outs


def test_golden_arithmetic_is_consistent():
    recs, _ = _golden_rows()
    for k, comp, a, sa, b, sb, v, q, r in recs:
        m = M1 if comp == 1 else M2
        assert a * sa - b * sb == v
        assert q * m + r == v and 0 <= r < m


def test_worked_example_seed_12345():
    recs, outs = _golden_rows()
    s = np.full(6, 12345, dtype=np.uint32)
    for k, z, u_str, f_num in outs:
        got = oracle.step(s)
        x1 = [r for r in recs if r[0] == k and r[1] == 1][0][-1]
        x2 = [r for r in recs if r[0] == k and r[1] == 2][0][-1]
        assert int(s[2]) == x1 and int(s[5]) == x2
        assert got == z
        assert oracle.to_f64(z) == float(u_str)
        assert Fraction(oracle.to_f32(z)) == Fraction(f_num, 2**24)
    # big-integer reference agrees
    assert ref.outputs([12345] * 6, 3) == [o[1] for o in outs]


# --------------------------------------------------------------------------
# streams / substreams (sec. 4.1)
# --------------------------------------------------------------------------
def test_substreams_tile_a_stream():
    # 2^51 substreams of 2^76 make one stream of 2^127
    for comp in (0, 1):
        sub = oracle.matpow(comp, 1 << 76).astype(np.uint64)
        m = (M1, M2)[comp]
        R = np.eye(3, dtype=object)
        B = sub.astype(object)
        e = 1 << 51
        while e:
            if e & 1:
                R = (R.dot(B)) % m
            B = (B.dot(B)) % m
            e >>= 1
        assert np.array_equal(R.astype(np.uint32), oracle.matpow(comp, 1 << 127))


def test_stream_starts_three_ways():
    base = np.full(6, 12345, dtype=np.uint32)
    # 1) via the bits of g; 2) by repeated jumps of 2^127
    cur = base.copy()
    for g in range(0, 40):
        assert np.array_equal(oracle.stream_start(base, g), cur), g
        cur = oracle.jump(cur, 1 << 127)
    # 3) stream 0 is the seed itself; stream g+1 = substream 2^51 of stream g
    for g in (0, 1, 5, 12345, 2**20 - 1, 2**40 + 3):
        a = oracle.stream_start(base, g)
        b = oracle.jump(a, (1 << 51) << 76)
        assert np.array_equal(b, oracle.stream_start(base, g + 1))
    assert np.array_equal(oracle.stream_start(base, 0), base)
    st = oracle.streams(base, 7, 5)
    for i in range(5):
        assert np.array_equal(st[i], oracle.stream_start(base, 7 + i))


def test_stream_2_pow_64_nearly_wraps():
    # 2^64 streams of 2^127 exceed the period by a hair: A^(2^191) != I but
    # A^(period) = I for the combined generator.
    rho = (M1**3 - 1) * (M2**3 - 1) // 2
    assert rho < 1 << 191
    s = np.full(6, 12345, dtype=np.uint32)
    assert np.array_equal(oracle.jump(s, rho), s)
    assert not np.array_equal(oracle.jump(s, (1 << 191) - 1), s)


# --------------------------------------------------------------------------
# conversions (exact rational arithmetic)
# --------------------------------------------------------------------------
def _z_samples():
    rng = random.Random(21)
    zs = [1, 2, 3, 511, 512, 513, 1023, 1024, 1025, M1 - 1, M1, M1 - 511, M1 - 512,
          2**31, 2**31 + 1, 2**32 - 2**9 - 209]
    zs += [rng.randrange(1, M1 + 1) for _ in range(3000)]
    return zs


def test_norm_is_nearest_double_to_inverse():
    assert ref.NORM == 2.328306549295727688e-10
    q = Fraction(1, M1 + 1)
    n = Fraction(ref.NORM)
    ulp = Fraction(2) ** (math.frexp(ref.NORM)[1] - 53)
    assert abs(n - q) <= ulp / 2


def test_f64_conversion_exact_rounding():
    for z in _z_samples():
        u = oracle.to_f64(z)
        assert u == ref.to_f64(z)
        assert 0.0 < u < 1.0
        # within one ulp of the real quotient z / (m1 + 1)
        exact = Fraction(z, M1 + 1)
        assert abs(Fraction(u) - exact) <= Fraction(2) ** (math.frexp(u)[1] - 52)


def test_f32_conversion_buckets():
    prev = None
    for z in sorted(set(_z_samples())):
        f = oracle.to_f32(z)
        fr = Fraction(f)
        num = fr * 2**24
        assert num.denominator == 1 and num.numerator % 2 == 1
        assert 0 < fr < 1
        # bucket containment: (z-1)/2^32 lies in [num-1, num+1) / 2^24
        x = Fraction(z - 1, 2**32)
        assert Fraction(num.numerator - 1, 2**24) <= x < Fraction(num.numerator + 1, 2**24)
        assert fr == ref.to_f32_exact(z)
        if prev is not None:
            assert f >= prev
        prev = f
    assert oracle.to_f32(1) == 2.0**-24
    assert oracle.to_f32(M1) == (2 * ((M1 - 1) >> 9) + 1) / 2**24 < 1.0


# --------------------------------------------------------------------------
# master-seed expansion (random spacing, sec. 2.3)
# --------------------------------------------------------------------------
def test_splitmix64_known_answer():
    # first output of SplitMix64 for seed 0 in its public-domain reference
    # implementation
    assert oracle.splitmix64(0, 1)[0] == 0xE220A8397B1DCDAF


def test_seed_from_master_is_valid_and_defined():
    for seed in (0, 1, 0x0123456789ABCDEF, 2**64 - 1):
        s = oracle.seed_from_master(seed)
        assert oracle.state_valid(s)
        w = oracle.splitmix64(seed, 6)
        want = [w[i] % M1 for i in range(3)] + [w[i] % M2 for i in range(3, 6)]
        assert [int(x) for x in s] == want


def test_adjacent_stream_starts_and_uniform_jump():
    base = oracle.seed_from_master(0x0123456789ABCDEF)
    for first in (0, 5, 2**40 - 3):
        assert np.array_equal(oracle.streams_adjacent(base, first, 40),
                              oracle.streams(base, first, 40))
    st = oracle.streams(base, 0, 30)
    for e in (0, 1, 999, 2**76 + 12345, 2**190 + 7):
        assert np.array_equal(oracle.jump_uniform(st, e), oracle.jump_many(st, e))
    # and against stepping, for a small exponent
    assert np.array_equal(oracle.jump_uniform(st[:3], 57)[2], oracle.skip(st[2], 57))


def test_splitmix64_random_access_matches_sequential():
    for seed in (0, 1, 0x0123456789ABCDEF, 2**64 - 1):
        seq = oracle.splitmix64(seed, 1500)
        for k in list(range(40)) + [777, 1499]:
            assert oracle.splitmix64_at(seed, k) == seq[k]
    assert oracle.splitmix64_at(0, 0) == 0xE220A8397B1DCDAF


# --------------------------------------------------------------------------
# random spacing and leapfrog (sec. 2.3)
# --------------------------------------------------------------------------
def test_random_spacing_states_are_expanded_draws():
    master = 0x0123456789ABCDEF
    seq = oracle.splitmix64(master, 64)
    st = oracle.random_spacing_states(master, 0, 64)
    assert st.shape == (64, 6)
    for g in range(64):
        assert np.array_equal(st[g], oracle.seed_from_master(seq[g]))
        assert oracle.state_valid(st[g])
    assert len({tuple(r) for r in st.tolist()}) == 64
    # a window of the set is the same streams
    assert np.array_equal(oracle.random_spacing_states(master, 17, 9), st[17:26])
    far = oracle.random_spacing_states(master, 2**40 + 3, 2)
    assert np.array_equal(far[1], oracle.seed_from_master(oracle.splitmix64_at(master, 2**40 + 4)))


@pytest.mark.parametrize("players,per_player", [(1, 9), (7, 1), (5, 6), (64, 3), (3, 70)])
def test_leapfrog_cards_are_every_pth_output(players, per_player):
    seed = oracle.seed_from_master(99)
    pm, end = oracle.leapfrog(seed, players, per_player, oracle.U32, oracle.STREAM_MAJOR)
    il, end2 = oracle.leapfrog(seed, players, per_player, oracle.U32, oracle.INTERLEAVED)
    assert pm.shape == (players, per_player) and il.shape == (per_player, players)
    assert np.array_equal(pm, il.T) and np.array_equal(end, end2)
    for t in range(players):
        for k in range(per_player):
            # card k of player t: one step from the state t + k*players
            # steps on, computed with big-integer matrix powers
            assert int(pm[t, k]) == ref.outputs(ref.jump(seed, t + k * players), 1)[0]
    assert [int(v) for v in end] == ref.jump(seed, players * per_player)


def test_leapfrog_floats_follow_the_integers():
    seed = oracle.seed_from_master(5)
    u, _ = oracle.leapfrog(seed, 11, 4, oracle.U32)
    f, _ = oracle.leapfrog(seed, 11, 4, oracle.F32)
    d, _ = oracle.leapfrog(seed, 11, 4, oracle.F64, oracle.INTERLEAVED)
    assert np.array_equal(f, np.vectorize(oracle.to_f32)(u).astype(np.float32))
    assert np.array_equal(d, np.vectorize(oracle.to_f64)(u.T))


# --------------------------------------------------------------------------
# Philox4x32-10 (the counter-based second generator)
# --------------------------------------------------------------------------
def test_philox_weyl_increments_are_golden_ratio_and_sqrt3():
    M0, M1, W0, W1 = oracle.philox_constants()
    # floor(2^32 (sqrt(5) - 1) / 2) and floor(2^32 (sqrt(3) - 1)), exactly
    assert W0 == (math.isqrt(5 << 64) - (1 << 32)) // 2
    assert W1 == math.isqrt(3 << 64) - (1 << 32)
    # the multipliers must be odd for each round to be a bijection; their
    # values (found by search in Salmon et al.) have no closed form here
    assert M0 % 2 == 1 and M1 % 2 == 1


def philox_inverse(out, key, rounds=10):
    """Undo Philox4x32 rounds, written from the round structure: the low
    halves of the two products are the new words 3 and 1, so the old words 0
    and 2 come back by multiplying with the multipliers' inverses mod 2^32;
    the high halves then unmask the old words 3 and 1."""
    M0, M1, W0, W1 = oracle.philox_constants()
    inv0, inv1 = pow(M0, -1, 1 << 32), pow(M1, -1, 1 << 32)
    n0, n1, n2, n3 = [int(v) for v in out]
    for r in reversed(range(rounds)):
        k0 = (key[0] + r * W0) & 0xFFFFFFFF
        k1 = (key[1] + r * W1) & 0xFFFFFFFF
        c0 = (n3 * inv0) & 0xFFFFFFFF
        c2 = (n1 * inv1) & 0xFFFFFFFF
        c3 = n2 ^ ((M0 * c0) >> 32) ^ k1
        c1 = n0 ^ ((M1 * c2) >> 32) ^ k0
        n0, n1, n2, n3 = c0, c1, c2, c3
    return [n0, n1, n2, n3]


def test_philox_rounds_are_undone_by_the_inverse():
    rng = random.Random(1412)
    for _ in range(300):
        ctr = [rng.getrandbits(32) for _ in range(4)]
        key = [rng.getrandbits(32) for _ in range(2)]
        out = oracle.philox4x32_10(ctr, key)
        assert philox_inverse(out, key) == ctr
        assert philox_inverse(out, key, rounds=9) != ctr


def test_philox_streams_fill_and_jump():
    key = 0x0123456789ABCDEF
    st = oracle.philox_streams(key, 2**40, 3)
    assert [int(v) for v in st[1]] == [0, 0, (2**40 + 1) & 0xFFFFFFFF, (2**40 + 1) >> 32,
                                       key & 0xFFFFFFFF, key >> 32]
    out, end = oracle.philox_fill(st, 11, oracle.U32)
    for s in range(3):
        words = []
        for b in range(3):
            words += oracle.philox4x32_10([b, 0, int(st[s, 2]), int(st[s, 3])],
                                          [int(st[s, 4]), int(st[s, 5])])
        assert [int(v) for v in out[s]] == words[:11]
        assert int(end[s, 0]) == 11 and int(end[s, 1]) == 0
    # a jump equals drawing: positions 5.. of a longer fill
    j = oracle.philox_jump(st, 5)
    tail, _ = oracle.philox_fill(j, 6, oracle.U32)
    assert np.array_equal(tail, out[:, 5:])
    # the position carries into its high word, and wraps at 2^64
    hi = oracle.philox_jump(st, 2**32 + 7)
    assert [int(hi[0, 0]), int(hi[0, 1])] == [7, 1]
    wrap = oracle.philox_jump(oracle.philox_jump(st, 2**64 - 1), 1)
    assert np.array_equal(wrap, st)


def test_philox_conversions_are_exact_and_open():
    for w in (0, 1, 255, 256, 2**31, 2**32 - 1, 123456789):
        f = oracle.philox_to_f32(w)
        d = oracle.philox_to_f64(w)
        assert Fraction(f) * 2**24 == 2 * (w >> 9) + 1 and 0 < f < 1
        assert Fraction(d) * 2**33 == 2 * w + 1 and 0 < d < 1
    st = oracle.philox_streams(9, 0, 2)
    u, _ = oracle.philox_fill(st, 40, oracle.U32)
    f, _ = oracle.philox_fill(st, 40, oracle.F32)
    d, _ = oracle.philox_fill(st, 40, oracle.F64, oracle.INTERLEAVED)
    assert np.array_equal(f, np.vectorize(oracle.philox_to_f32)(u).astype(np.float32))
    assert np.array_equal(d, np.vectorize(oracle.philox_to_f64)(u.T))


# --------------------------------------------------------------------------
# fill: layouts, chaining, state ranges
# --------------------------------------------------------------------------
def test_fill_layouts_and_chaining():
    base = oracle.seed_from_master(0x0123456789ABCDEF)
    st = oracle.streams(base, 0, 5)
    a, st_a = oracle.fill(st, 37, oracle.U32, oracle.STREAM_MAJOR)
    b, st_b = oracle.fill(st, 37, oracle.U32, oracle.INTERLEAVED)
    assert np.array_equal(a, b.T) and np.array_equal(st_a, st_b)
    c1, mid = oracle.fill(st, 20, oracle.U32)
    c2, end = oracle.fill(mid, 17, oracle.U32)
    assert np.array_equal(np.concatenate([c1, c2], axis=1), a)
    assert np.array_equal(end, st_a)
    # advanced state = jump by n
    for i in range(5):
        assert np.array_equal(st_a[i], oracle.jump(st[i], 37))
    # dtypes derive from the same integers
    f, _ = oracle.fill(st, 37, oracle.F32)
    d, _ = oracle.fill(st, 37, oracle.F64)
    for i in range(5):
        for k in range(37):
            assert f[i, k] == np.float32(oracle.to_f32(int(a[i, k])))
            assert d[i, k] == oracle.to_f64(int(a[i, k]))
    assert a.min() >= 1 and a.max() <= M1
    for row in st_a:
        assert oracle.state_valid(row)


def test_c_oracle_matches_bigint_reference():
    base = [12345] * 6
    st = oracle.streams(np.array(base, dtype=np.uint32), 0, 3)
    out, _ = oracle.fill(st, 300, oracle.U32)
    for i in range(3):
        assert [int(v) for v in out[i]] == ref.outputs([int(v) for v in st[i]], 300)
