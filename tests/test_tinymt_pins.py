"""Pins of the TinyMT32 oracle (sec. 4.2 hybrid: parameter sets shared by a
group of streams, sub-streams by sequence splitting) against facts fixed by
the mathematics rather than by the oracle itself: the Berlekamp-Massey
routine recovers linear recurrences built here, the irreducibility test
finds exactly as many irreducible polynomials of each prime degree as
Gauss's formula counts and rejects products, the transition is linear over
GF(2), accepted parameter sets have period exactly 2^127 - 1, and jumps
equal brute-force stepping.  The transition, tempering and seeding
themselves are parity unpinned (no known-answer output available)."""
import random

import numpy as np
import pytest

import oracle

MASK = 0x7FFFFFFF


def lfsr_bits(taps, init, n):
    """a_k = sum of a_{k-t} over t in taps (mod 2), from the first len(init) bits."""
    a = list(init)
    while len(a) < n:
        k = len(a)
        a.append(sum(a[k - t] for t in taps) & 1)
    return a


def test_berlekamp_massey_recovers_built_recurrences():
    # x^7 + x + 1 (primitive): a_k = a_{k-6} + a_{k-7}
    bits = lfsr_bits([6, 7], [1, 0, 0, 0, 0, 0, 0], 60)
    L, C = oracle.gf2_berlekamp_massey(bits)
    assert L == 7
    assert C == 1 | (1 << 6) | (1 << 7)  # C(x) = 1 + x^6 + x^7, the reciprocal
    # a product (x^3 + x + 1)(x^4 + x + 1) = x^7 + x^5 + x^3 + x^2 + 1
    # (multiplied out by hand: the two x^4 and the two x terms cancel), so
    # a_k = a_{k-2} + a_{k-4} + a_{k-5} + a_{k-7}
    bits = lfsr_bits([2, 4, 5, 7], [1, 1, 0, 1, 0, 0, 1], 60)
    L, C = oracle.gf2_berlekamp_massey(bits)
    assert L == 7
    assert C == 1 | 1 << 2 | 1 << 4 | 1 << 5 | 1 << 7
    # started inside the x^3 + x + 1 part (its own sequence, period 7), the
    # minimal recurrence is that factor alone: a_k = a_{k-2} + a_{k-3}
    small = lfsr_bits([2, 3], [1, 0, 0], 60)
    assert all(small[k] == small[k - 2] ^ small[k - 4] ^ small[k - 5] ^ small[k - 7]
               for k in range(7, 60))
    assert oracle.gf2_berlekamp_massey(small) == (3, 1 | 1 << 2 | 1 << 3)
    # a sequence of period 3 that a degree-2 recurrence (x^2 + x + 1) makes
    L, C = oracle.gf2_berlekamp_massey([0, 1, 1] * 20)
    assert (L, C) == (2, 0b111)
    # the all-zero sequence has linear complexity 0
    assert oracle.gf2_berlekamp_massey([0] * 30)[0] == 0


def trial_division_irreducible(f, n):
    """Irreducible over GF(2) when no polynomial of degree 1..n//2 divides f."""
    def pmod(a, b):
        db = b.bit_length() - 1
        while a and a.bit_length() - 1 >= db:
            a ^= b << (a.bit_length() - 1 - db)
        return a
    for d in range(1, n // 2 + 1):
        for g in range(1 << d, 1 << (d + 1)):
            if pmod(f, g) == 0:
                return False
    return True


@pytest.mark.parametrize("n", [3, 5, 7, 11, 13])
def test_irreducibility_test_counts_match_gauss(n):
    """For a prime degree n there are (2^n - 2) / n irreducible polynomials."""
    count = 0
    rng = random.Random(n)
    checked = 0
    for f in range(1 << n, 1 << (n + 1)):
        ok = oracle.gf2_irreducible_prime_degree(f)
        count += ok
        if n <= 11 and rng.random() < 0.1:
            assert ok == trial_division_irreducible(f, n), f
            checked += 1
    assert count == ((1 << n) - 2) // n
    assert n > 11 or checked > 0


def test_irreducibility_test_at_degree_127():
    # x^127 + x + 1 is a primitive trinomial of the Mersenne exponent 127
    assert oracle.gf2_irreducible_prime_degree((1 << 127) | 2 | 1)
    # x^127 + 1 has the root 1; (x^2 + x + 1) times a degree-125 polynomial
    # has no root in GF(2) but is reducible
    assert not oracle.gf2_irreducible_prime_degree((1 << 127) | 1)
    rng = random.Random(5)
    for _ in range(20):
        g = (1 << 125) | rng.getrandbits(125) | 1
        f = 0
        for i in range(3):  # carry-less (x^2 + x + 1) * g
            f ^= g << i
        assert f.bit_length() - 1 == 127
        assert not oracle.gf2_irreducible_prime_degree(f)


def rand_state(rng):
    return np.array([rng.getrandbits(32) for _ in range(4)], dtype=np.uint32)


def params(count=4, master=0x5EED):
    return oracle.tmt_search(master, count)[0]


def test_transition_is_linear_over_gf2():
    rng = random.Random(1)
    for p in params():
        for _ in range(50):
            a, b = rand_state(rng), rand_state(rng)
            ta, tb, tab = oracle.tmt_next(a, p), oracle.tmt_next(b, p), oracle.tmt_next(a ^ b, p)
            assert np.array_equal(tab, ta ^ tb)
        # the bit outside the 127-bit state (bit 31 of s0) changes nothing
        s = rand_state(rng)
        t = s.copy()
        t[0] ^= 0x80000000
        assert np.array_equal(oracle.tmt_next(s, p), oracle.tmt_next(t, p))


def horner(phi, s, p):
    acc = np.zeros(4, dtype=np.uint32)
    for i in range(phi.bit_length() - 1, -1, -1):
        acc = oracle.tmt_next(acc, p)
        if (phi >> i) & 1:
            acc = acc ^ s
    return acc


def test_characteristic_polynomial_annihilates_the_state():
    rng = random.Random(2)
    for p in params():
        deg, phi = oracle.tmt_charpoly(p)
        assert deg == 127 and phi.bit_length() - 1 == 127
        assert oracle.gf2_irreducible_prime_degree(phi)
        for _ in range(5):
            v = horner(phi, rand_state(rng), p)
            v[0] &= MASK
            assert not v.any()


def test_accepted_parameter_sets_have_period_2p127_minus_1():
    """2^127 - 1 is prime, so T^(2^127 - 1) = I on the 127-bit state and
    T != I make the period exactly 2^127 - 1."""
    rng = random.Random(3)
    for p in params():
        s = rand_state(rng)
        t = oracle.tmt_jump(s, p, (1 << 127) - 1)
        assert np.array_equal(t[1:], s[1:]) and (t[0] & MASK) == (s[0] & MASK)
        assert np.array_equal(oracle.tmt_jump(s, p, 1 << 127), oracle.tmt_next(s, p))
        assert not np.array_equal(oracle.tmt_next(s, p), s)


def test_jumps_equal_stepping():
    rng = random.Random(4)
    p = params(1)[0]
    s = oracle.tmt_init(12345, p)
    for e in list(range(0, 40)) + [127, 128, 255, 256, 1000] + [rng.randrange(1 << 17) for _ in range(5)]:
        assert np.array_equal(oracle.tmt_jump(s, p, e), oracle.tmt_skip(s, p, e)), e
    for _ in range(5):
        a, b = rng.getrandbits(100), rng.getrandbits(100)
        assert np.array_equal(oracle.tmt_jump(oracle.tmt_jump(s, p, a), p, b),
                              oracle.tmt_jump(s, p, a + b))


def test_search_keeps_exactly_the_accepted_candidates_in_order():
    master = 77
    P, cand = oracle.tmt_search(master, 5)
    want = [c for c in range(int(cand[-1]) + 1) if oracle.tmt_params_ok(oracle.tmt_candidate(master, c))]
    assert want == [int(c) for c in cand]
    for i, c in enumerate(cand):
        assert np.array_equal(P[i], oracle.tmt_candidate(master, int(c)))
    # and a rejected candidate really is reducible or of lower degree
    rej = next(c for c in range(100) if c not in want)
    deg, phi = oracle.tmt_charpoly(oracle.tmt_candidate(master, rej))
    assert deg < 127 or not oracle.gf2_irreducible_prime_degree(phi)


def test_streams_are_chunks_of_2p64_of_each_parameter_set():
    master, per = 9, 5
    P, _ = oracle.tmt_search(master, 3)
    st = oracle.tmt_streams(master, per, 0, 3 * per, P)
    for q in range(3):
        base = oracle.tmt_init(oracle.splitmix64_at(master, q) & 0xFFFFFFFF, P[q])
        assert np.array_equal(st[q * per, :4], base)
        for j in range(per):
            assert st[q * per + j, 4] == q
            if j + 1 < per:
                nxt = oracle.tmt_jump(st[q * per + j, :4], P[q], 1 << 64)
                assert np.array_equal(nxt, st[q * per + j + 1, :4])
    # a window of the set equals the same rows of the whole set
    w = oracle.tmt_streams(master, per, 4, 7, P[0:], 0)
    assert np.array_equal(w, st[4:11])


def test_fill_layouts_and_conversions():
    master, per = 11, 4
    P, _ = oracle.tmt_search(master, 2)
    st = oracle.tmt_streams(master, per, 0, 8, P)
    n = 37
    u, end = oracle.tmt_fill(st, n, oracle.U32, oracle.STREAM_MAJOR, P)
    for i in range(8):
        want, s_end = oracle.tmt_outputs(st[i, :4], P[st[i, 4]], n)
        assert np.array_equal(u[i], want)
        assert np.array_equal(end[i, :4], s_end) and end[i, 4] == st[i, 4]
    ui, _ = oracle.tmt_fill(st, n, oracle.U32, oracle.INTERLEAVED, P)
    assert np.array_equal(ui, u.T)
    f, _ = oracle.tmt_fill(st, n, oracle.F32, oracle.STREAM_MAJOR, P)
    d, _ = oracle.tmt_fill(st, n, oracle.F64, oracle.STREAM_MAJOR, P)
    w = u.astype(np.int64)
    assert np.array_equal(f, ((2 * (w >> 9) + 1) * 2.0**-24).astype(np.float32))
    assert np.array_equal(d, (2 * w + 1) * 2.0**-33)
    assert (f > 0).all() and (f < 1).all() and (d > 0).all() and (d < 1).all()
