"""SplitMix64 counter-based generator (oracle, test-only).

Published by Steele, Lea and Flood, "Fast splittable pseudorandom number
generators" (OOPSLA 2014).  Used for the Arnoldi start vector, which must be
the same on every implementation: value(seed, i) mixes the 64-bit word
seed XOR i with the SplitMix64 finaliser, and the top 53 bits give a double
in [0, 1), mapped to [-1, 1).
"""
import numpy as np

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(x):
    x = np.asarray(x, dtype=np.uint64)
    with np.errstate(over='ignore'):
        z = x + _GOLDEN
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        return z ^ (z >> np.uint64(31))


def uniform_pm1(seed, index):
    """U(-1, 1) sample number `index` of stream `seed`."""
    z = splitmix64(np.uint64(seed) ^ np.asarray(index, dtype=np.uint64))
    u = (z >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)
    return 2.0 * u - 1.0
