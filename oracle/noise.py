"""Volume noise sources eta_r (Section 2: random sources; Section 2.3: the
paper draws them on the host with RANLUX; Section 2.4 plans GPU generation).

Reading (the paper does not fix the noise or the generator):

* Z2 noise is real, +-1; Z4 noise takes the values {1, i, -1, -i}.  Both have
  E[eta eta^dag] = 1, which the one-end-trick estimators need.
* One draw per (site, spin, colour).  The generator is SplitMix64 (Steele, Lea
  & Flood, OOPSLA 2014) used as a counter-based generator: output i of the
  stream seeded with ``seed`` is ``mix(seed + (i + 1) * 0x9E3779B97F4A7C15)``,
  with counter ``i = (r * V + site) * 12 + 3 * spin + colour`` and ``site`` the
  lexicographic index (x fastest).  Source r is therefore a pure function of
  (seed, r).
* Z2 takes bit 0 (0 -> +1, 1 -> -1); Z4 takes bits 0-1 (0 -> 1, 1 -> i,
  2 -> -1, 3 -> -i).
"""
from __future__ import annotations

import numpy as np

Z2, Z4 = 0, 1

_M64 = (1 << 64) - 1


def splitmix64_scalar(seed: int, i: int) -> int:
    """Output i of SplitMix64 seeded with ``seed``, in Python integers."""
    z = (seed + (i + 1) * 0x9E3779B97F4A7C15) & _M64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _M64
    return z ^ (z >> 31)


def splitmix64_array(seed: int, counters: np.ndarray) -> np.ndarray:
    """Vectorised ``splitmix64_scalar`` over a uint64 array of counters."""
    c = counters.astype(np.uint64)
    with np.errstate(over="ignore"):
        z = (c + np.uint64(1)) * np.uint64(0x9E3779B97F4A7C15) + np.uint64(seed & _M64)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
    return z ^ (z >> np.uint64(31))


def source(dims, seed: int, r: int, kind: int) -> np.ndarray:
    """Noise source number r, complex128 [T, Z, Y, X, 4, 3]."""
    X, Y, Z, T = dims
    V = X * Y * Z * T
    site = np.arange(V, dtype=np.uint64)[:, None]
    comp = np.arange(12, dtype=np.uint64)[None, :]
    ctr = (np.uint64(r) * np.uint64(V) + site) * np.uint64(12) + comp
    w = splitmix64_array(seed, ctr)
    if kind == Z2:
        bit = (w & np.uint64(1)).astype(np.int64)
        eta = (1 - 2 * bit).astype(complex)
    elif kind == Z4:
        table = np.array([1, 1j, -1, -1j], dtype=complex)
        eta = table[(w & np.uint64(3)).astype(np.int64)]
    else:
        raise ValueError("noise kind must be Z2 (0) or Z4 (1)")
    return eta.reshape(T, Z, Y, X, 4, 3)
