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

Start blocks for the stochastic trace of KPM (Sec. 4.2) come from the same
generator (Sec. 3.4 fills vectors from a function of the site, the orbital,
the column and a random seed): element (r, c) of an n_b-column block takes
index i = r * n_b + c, with r the global row, and z_i = output number i + 1,

    random phase   exp(i phi),  phi = 2 pi u_i,   u_i = (z_i >> 11) 2^-53
    Z4 phase       i^k,         k = z_i >> 62     (1, i, -1, -i)

so any part of a block is the same values whoever generates it.
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


PHASE, Z4 = 0, 1


def splitmix64_at(seed: int, idx) -> np.ndarray:
    """Output number i + 1 of the stream seeded with `seed`, for each index i
    of the array idx (the counter form: no other output is computed)."""
    n = np.asarray(idx, dtype=np.uint64) + np.uint64(1)
    with np.errstate(over="ignore"):
        z = np.uint64(seed) + n * GAMMA
        z = (z ^ (z >> np.uint64(30))) * M1
        z = (z ^ (z >> np.uint64(27))) * M2
    return z ^ (z >> np.uint64(31))


def phase_values(z: np.ndarray, kind: int) -> np.ndarray:
    """Unit-modulus complex128 values of generator outputs z (kinds above)."""
    if kind == PHASE:
        u = (z >> np.uint64(11)).astype(np.float64) * 2.0 ** -53
        phi = (2.0 * np.pi) * u
        return np.cos(phi) + 1j * np.sin(phi)
    if kind == Z4:
        k = (z >> np.uint64(62)).astype(np.int64)
        return np.array([complex(1.0, 0.0), complex(0.0, 1.0), complex(-1.0, 0.0), complex(0.0, -1.0)])[k]
    raise ValueError(f"unknown kind {kind}")


def random_block(seed: int, rows: int, nb: int, kind: int, row0: int = 0) -> np.ndarray:
    """Rows row0 .. row0 + rows - 1 of the n_b-column start block [rows, nb]."""
    z = splitmix64(seed, row0 * nb, rows * nb)
    return phase_values(z, kind).reshape(rows, nb)


def random_block_at(seed: int, nb: int, kind: int, rows, cols) -> np.ndarray:
    """Entries (rows[j], cols[j]) of the same block (sampled check)."""
    idx = np.asarray(rows, dtype=np.uint64) * np.uint64(nb) + np.asarray(cols, dtype=np.uint64)
    return phase_values(splitmix64_at(seed, idx), kind)
