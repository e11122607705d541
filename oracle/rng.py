"""Counter-based SplitMix64 stream (oracle side).

SplitMix64 (Steele, Lea & Flood, OOPSLA 2014; the reference C code by
S. Vigna): the i-th output of the stream started at ``seed`` is
``mix(seed + (i + 1) * 0x9E3779B97F4A7C15)`` with the finaliser

    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9
    z = (z ^ (z >> 27)) * 0x94D049BB133111EB
    z =  z ^ (z >> 31)

(all arithmetic mod 2^64).  A uniform double in [0, 1) is ``(z >> 11) * 2^-53``.
Used for the power iteration's start vectors (Algorithm 4 asks for a random
vector of unit norm); uniform entries in [-1, 1) are exact in any language, so
both sides start from bit-identical vectors.
"""
import numpy as np

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(seed, n):
    with np.errstate(over="ignore"):
        z = np.uint64(seed) + (np.arange(1, n + 1, dtype=np.uint64) * _GOLDEN)
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def uniform_pm1(seed, n):
    """n doubles uniform in [-1, 1): 2 * ((z >> 11) * 2^-53) - 1."""
    z = splitmix64(seed, n)
    u = (z >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)
    return 2.0 * u - 1.0


def normal(seed, n):
    """n standard normals by the Box-Muller transform of consecutive pairs:
    u1 = 1 - U(2k), u2 = U(2k+1); x_2k = R cos(2 pi u2), x_2k+1 = R sin(2 pi u2),
    R = sqrt(-2 log u1)."""
    m = (n + 1) // 2
    z = splitmix64(seed, 2 * m)
    u = (z >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)
    u1 = 1.0 - u[0::2]
    u2 = u[1::2]
    R = np.sqrt(-2.0 * np.log(u1))
    out = np.empty(2 * m)
    out[0::2] = R * np.cos(2.0 * np.pi * u2)
    out[1::2] = R * np.sin(2.0 * np.pi * u2)
    return out[:n]
