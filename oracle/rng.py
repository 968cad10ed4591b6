"""Counter-based random field for on-the-fly disorder (oracle; test
infrastructure).

Sec. 3.3 generates the disorder inside the kernel instead of streaming it
from memory.  The value has to be the same in every matrix-vector product
and independent of the order in which sites are visited, so it is a pure
function of (seed, index): SplitMix64 (Steele, Lea, Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014), whose n-th output is the
mixing function applied to seed + n * gamma with gamma = 0x9E3779B97F4A7C15.

    u_i = (output number i + 1) >> 11, times 2^-53     in [0, 1)
    V_i = W * (u_i - 1/2)                              in [-W/2, W/2)

with i the site index (field per site) or the orbital row (field per orbital).
"""

from __future__ import annotations

import numpy as np

GAMMA = np.uint64(0x9E3779B97F4A7C15)
M1 = np.uint64(0xBF58476D1CE4E5B9)
M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(seed: int, first: int, count: int) -> np.ndarray:
    """Outputs number first + 1 .. first + count of the stream seeded with
    `seed` (uint64 array; arithmetic modulo 2^64)."""
    n = np.arange(first + 1, first + 1 + count, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed) + n * GAMMA
        z = (z ^ (z >> np.uint64(30))) * M1
        z = (z ^ (z >> np.uint64(27))) * M2
    return z ^ (z >> np.uint64(31))


def uniform(seed: int, n: int) -> np.ndarray:
    """u_i for i = 0 .. n-1: the top 53 bits of each output scaled to [0, 1)."""
    return (splitmix64(seed, 0, n) >> np.uint64(11)).astype(np.float64) * 2.0 ** -53


def field(seed: int, W: float, n: int) -> np.ndarray:
    """The on-the-fly disorder V_i = W (u_i - 1/2), i = 0 .. n-1."""
    return W * (uniform(seed, n) - 0.5)
