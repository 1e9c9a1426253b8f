"""Pure-Python MRG32k3a reference -- test infrastructure only.

A second CPU implementation, independent of ``mrg32k3a_oracle.c``: Python's
unbounded integers and ``%`` (always non-negative for a positive modulus), for
tiny cases and for matrix powers with exponents of any size.  Follows sec. 4.1
(MRG32k3a) and sec. 2.3 (sequence splitting by jump ahead) of
Passerat-Palmbach & Hill, HPCS 2012; constants from L'Ecuyer 1999, which
sec. 4.1 cites.  Conversions to floating point are evaluated in exact rational
arithmetic (``fractions``) and then rounded once, so they do not depend on the
host's floating-point unit.
"""
from __future__ import annotations

from fractions import Fraction

M1 = 2**32 - 209
M2 = 2**32 - 22853
A12, A13N = 1403580, 810728
A21, A23N = 527612, 1370589
MODULI = (M1, M2)


def step(s: list) -> int:
    """Advance the 6-word state list in place (oldest word first in each
    triple); return the combined output z' in [1, m1]."""
    p1 = (A12 * s[1] - A13N * s[0]) % M1
    p2 = (A21 * s[5] - A23N * s[3]) % M2
    s[0], s[1], s[2] = s[1], s[2], p1
    s[3], s[4], s[5] = s[4], s[5], p2
    z = (p1 - p2) % M1
    return z if z else M1


def outputs(seed, n: int) -> list:
    s = list(int(v) for v in seed)
    return [step(s) for _ in range(n)]


def companion(comp: int) -> list:
    """Companion matrix of component ``comp`` acting on the column vector
    (x[n-3], x[n-2], x[n-1])."""
    if comp == 0:
        last = [(-A13N) % M1, A12, 0]
    else:
        last = [(-A23N) % M2, 0, A21]
    return [[0, 1, 0], [0, 0, 1], last]


def matmul(X, Y, m):
    return [[sum(X[i][k] * Y[k][j] for k in range(3)) % m for j in range(3)] for i in range(3)]


def identity():
    return [[1, 0, 0], [0, 1, 0], [0, 0, 1]]


def matpow(comp: int, e: int):
    m = MODULI[comp]
    R, B = identity(), companion(comp)
    while e:
        if e & 1:
            R = matmul(R, B, m)
        B = matmul(B, B, m)
        e >>= 1
    return R


def matvec(M, v, m):
    return [sum(M[i][k] * v[k] for k in range(3)) % m for i in range(3)]


def jump(seed, e: int) -> list:
    s = [int(v) for v in seed]
    return matvec(matpow(0, e), s[:3], M1) + matvec(matpow(1, e), s[3:], M2)


# ---- conversions, exact rational arithmetic then one rounding -------------
def _round_to_double(q: Fraction) -> float:
    """Round a positive rational to the nearest IEEE double (ties to even)."""
    assert q > 0
    # exponent e with 2^e <= q < 2^(e+1)
    e = q.numerator.bit_length() - q.denominator.bit_length()
    if Fraction(2) ** e > q:
        e -= 1
    scale = Fraction(2) ** (52 - e)          # 53-bit significand
    t = q * scale
    i = t.numerator // t.denominator
    r = t - i
    if r > Fraction(1, 2) or (r == Fraction(1, 2) and i % 2 == 1):
        i += 1
    return float(Fraction(i) / scale)


NORM = _round_to_double(Fraction(1, M1 + 1))


def to_f64(z: int) -> float:
    """(double) z times NORM, rounded once to nearest-even."""
    return _round_to_double(Fraction(z) * Fraction(NORM))


def to_f32_exact(z: int) -> Fraction:
    """FP32 output as an exact rational: (2*((z-1) >> 9) + 1) / 2^24."""
    k = (z - 1) >> 9
    return Fraction(2 * k + 1, 2**24)
