"""Pins of the oracle's counter RNG and Z2 / Z4 volume sources (CPU only)."""
import os

import numpy as np
import pytest

from oracle import noise

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "splitmix64.txt")


def _golden():
    rows = []
    for line in open(GOLDEN):
        line = line.split("#")[0].strip()
        if line:
            s, i, v = line.split()
            rows.append((int(s), int(i), int(v)))
    return rows


def test_splitmix64_published_outputs():
    rows = _golden()
    assert len(rows) == 6
    for seed, i, v in rows:
        assert noise.splitmix64_scalar(seed, i) == v
        assert int(noise.splitmix64_array(seed, np.array([i], dtype=np.uint64))[0]) == v


def test_splitmix64_vector_matches_scalar_large_seed_and_counter():
    seed = 0xFEDCBA9876543210
    ctr = np.array([0, 1, 2**32 + 5, 2**40 + 12345, 2**63 - 1], dtype=np.uint64)
    vec = noise.splitmix64_array(seed, ctr)
    for c, v in zip(ctr, vec):
        assert noise.splitmix64_scalar(seed, int(c)) == int(v)


def test_source_counter_map():
    """Component (site, spin, colour) of source r uses counter (r V + site) 12 + 3 spin + colour."""
    dims = (4, 2, 2, 6)
    X, Y, Z, T = dims
    V = X * Y * Z * T
    seed, r = 6750, 3
    eta = noise.source(dims, seed, r, noise.Z4)
    table = [1, 1j, -1, -1j]
    for (t, z, y, x, s, c) in [(0, 0, 0, 0, 0, 0), (5, 1, 1, 3, 3, 2), (2, 0, 1, 1, 1, 0)]:
        site = x + X * (y + Y * (z + Z * t))
        w = noise.splitmix64_scalar(seed, (r * V + site) * 12 + 3 * s + c)
        assert eta[t, z, y, x, s, c] == table[w & 3]
    eta2 = noise.source(dims, seed, r, noise.Z2)
    site = 1 + X * (1 + Y * (0 + Z * 4))
    w = noise.splitmix64_scalar(seed, (r * V + site) * 12 + 7)
    assert eta2[4, 0, 1, 1, 2, 1] == (1 if (w & 1) == 0 else -1)


def test_noise_statistics():
    dims = (8, 8, 8, 8)
    n = 8 ** 4 * 12
    for kind, vals in ((noise.Z2, [1, -1]), (noise.Z4, [1, 1j, -1, -1j])):
        eta = noise.source(dims, 6750, 0, kind).ravel()
        assert set(np.unique(np.round(eta, 12))) <= set(vals)
        for v in vals:                      # each value with its share, within 5 sigma
            frac = np.mean(np.isclose(eta, v))
            p = 1 / len(vals)
            assert abs(frac - p) < 5 * np.sqrt(p * (1 - p) / n)
        # E[eta_i eta_j^*] = delta_ij: neighbouring components and two sources uncorrelated
        assert abs(np.mean(eta[1:] * eta[:-1].conj())) < 5 / np.sqrt(n)
        other = noise.source(dims, 6750, 1, kind).ravel()
        assert abs(np.mean(eta * other.conj())) < 5 / np.sqrt(n)
        assert np.allclose(np.abs(eta), 1)
