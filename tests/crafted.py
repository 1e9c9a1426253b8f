"""Test inputs that steer MRG32k3a to chosen words at chosen outputs.

A state is written down at the moment output k is drawn, with its
component-2 lags chosen so that the new component-2 word takes a given value
(a21 * x2[n-1] - a23n * x2[n-3] = target mod m2, solved for x2[n-3]); the
oracle's jump by the combined period minus k then moves it back to the
stream's start.  The period (m1^3 - 1)(m2^3 - 1) / 2 is the lcm of the two
components' orders, which the oracle pins prove exact, so jumping by it is
the identity on both components.  Inputs only: expected values still come
from the oracle's fill.
"""
import numpy as np

import oracle

M1, M2 = oracle.M1, oracle.M2
A21, A23N = 527612, 1370589
PERIOD = (M1**3 - 1) * (M2**3 - 1) // 2


def state_hitting(k: int, x2_target: int, rng) -> np.ndarray:
    """A valid start state whose output number k (0-based) is drawn with the
    new component-2 word equal to x2_target (in [0, m2))."""
    a = [int(rng.integers(1, M1)) for _ in range(3)]
    b1, b2 = int(rng.integers(0, M2)), int(rng.integers(1, M2))
    b0 = (A21 * b2 - x2_target) * pow(A23N, -1, M2) % M2
    at_k = np.array(a + [b0, b1, b2], dtype=np.uint32)
    start = oracle.jump(at_k, PERIOD - k) if k else at_k
    assert np.array_equal(oracle.jump(start, k), at_k)
    return start


def hits(positions, targets, seed: int) -> np.ndarray:
    """[len(positions), 6] start states, stream i hitting targets[i % len] at
    positions[i]."""
    rng = np.random.default_rng(seed)
    return np.stack([state_hitting(int(k), int(targets[i % len(targets)]), rng)
                     for i, k in enumerate(positions)])
