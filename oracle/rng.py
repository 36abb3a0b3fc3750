"""Counter-based standard normal generator (oracle; test infrastructure only).

The H^2 construction draws a Gaussian sketch of large proxy matrices (see
oracle/h2.py).  Those random numbers cannot be passed in as an input (one
matrix of up to 16384 x 8192 entries, per run), so the oracle and the library
each implement the same published generator:

* SplitMix64 (Steele, Lea and Flood, "Fast splittable pseudorandom number
  generators", OOPSLA 2014), in the form of Vigna's reference code: the state
  is advanced by the golden-gamma 0x9E3779B97F4A7C15 and mixed by two
  xor-shift-multiply rounds;
* two 53-bit uniforms from two hashed counters, turned into one standard
  normal by the Box-Muller formula (Box and Muller, 1958).

Entry (t, j) of the sketch uses the counter (t << 24) | j; this module holds
none of the method's arithmetic.
"""
from __future__ import annotations

import numpy as np

GOLDEN = np.uint64(0x9E3779B97F4A7C15)
M1 = np.uint64(0xBF58476D1CE4E5B9)
M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(x) -> np.ndarray:
    """The SplitMix64 output for state x (before its increment); uint64 arrays."""
    x = np.asarray(x, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = x + GOLDEN
        z = (z ^ (z >> np.uint64(30))) * M1
        z = (z ^ (z >> np.uint64(27))) * M2
    return z ^ (z >> np.uint64(31))


def normal(seed: int, ctr) -> np.ndarray:
    """Standard normal for each counter value (uint64 array) under `seed`."""
    seed = np.uint64(seed)
    c = np.asarray(ctr, dtype=np.uint64)
    with np.errstate(over="ignore"):
        h1 = splitmix64(seed ^ splitmix64(np.uint64(2) * c))
        h2 = splitmix64(seed ^ splitmix64(np.uint64(2) * c + np.uint64(1)))
    u1 = ((h1 >> np.uint64(11)).astype(np.float64) + 1.0) * (1.0 / 9007199254740993.0)  # (0, 1]
    u2 = (h2 >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)        # [0, 1)
    return np.sqrt(-2.0 * np.log(u1)) * np.cos(6.283185307179586 * u2)


_cache: dict[int, np.ndarray] = {}


def sketch(rows: int, cols: int, seed: int) -> np.ndarray:
    """rows x cols matrix with entry (t, j) = normal(seed, (t << 24) | j).

    Entries depend only on (t, j), so the largest block drawn so far is kept
    and smaller requests are its leading blocks (read-only view)."""
    big = _cache.get(seed)
    if big is None or big.shape[0] < rows or big.shape[1] < cols:
        r = max(rows, big.shape[0] if big is not None else 0)
        c = max(cols, big.shape[1] if big is not None else 0)
        t = np.arange(r, dtype=np.uint64)[:, None]
        j = np.arange(c, dtype=np.uint64)[None, :]
        big = normal(seed, (t << np.uint64(24)) | j)
        big.setflags(write=False)
        _cache[seed] = big
    return big[:rows, :cols]
