"""SplitMix64 (Steele, Lea, Flood, "Fast splittable pseudorandom number
generators", OOPSLA 2014; the 64-bit finaliser constants of Vigna's public-domain
reference), used as a counter-based generator: the value for index i is the first
output of a SplitMix64 stream seeded with i.  Test infrastructure only.
"""
import numpy as np

_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(i):
    z = np.asarray(i, dtype=np.uint64) + _GAMMA
    z = (z ^ (z >> np.uint64(30))) * _M1
    z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def unit(i):
    """Uniform double in [0, 1): top 53 bits of splitmix64(i) times 2^-53."""
    with np.errstate(over="ignore"):
        z = splitmix64(i)
    return (z >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)
