"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module only *generates inputs*: gauge fields, gauge transformations and
generic random spinor fields.  It contains none of the method's arithmetic
(no Dirac operator, no solver, no noise of the estimator, no contraction), so
the oracle and the HIP path can both consume what it produces without
sharing any part of the computation under test.

The paper's production ensembles (32^3 x 64 twisted-mass configurations,
Section 2.1.1) are not available; the synthetic stand-in is a field of random
SU(3) links ``U = exp(i eps H)`` with ``H = sum_a h_a lambda_a / 2`` and
``h_a ~ N(0, 1)`` (``lambda_a`` the Gell-Mann matrices).  The Gaussians come
from a SplitMix64 counter stream (Steele, Lea & Flood, OOPSLA 2014) through
the Box-Muller transform, so a link is a pure function of (seed, site, mu).

Layout of every gauge array handed out here: ``[t][z][y][x][mu][3][3]``
complex128 with x fastest and ``mu = 0..3`` for x, y, z, t.
"""
from __future__ import annotations

import numpy as np

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_MIX1 = np.uint64(0xBF58476D1CE4E5B9)
_MIX2 = np.uint64(0x94D049BB133111EB)


def splitmix64(seed: int, counter) -> np.ndarray:
    """Output number ``counter`` (0-based) of the SplitMix64 stream seeded with ``seed``.

    SplitMix64 advances its 64-bit state by the golden-ratio increment and
    returns a bijective mix of the new state, so output i of the stream is
    ``mix(seed + (i + 1) * golden)``: random access by counter.
    """
    c = np.asarray(counter, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed) + (c + np.uint64(1)) * _GOLDEN
        z = (z ^ (z >> np.uint64(30))) * _MIX1
        z = (z ^ (z >> np.uint64(27))) * _MIX2
        z = z ^ (z >> np.uint64(31))
    return z


def _uniform_open(w: np.ndarray) -> np.ndarray:
    """Map 64-bit words to doubles in (0, 1) using their top 53 bits."""
    return ((w >> np.uint64(11)).astype(np.float64) + 0.5) * (1.0 / 9007199254740992.0)


def gell_mann() -> np.ndarray:
    """The eight Gell-Mann matrices, shape [8, 3, 3]."""
    l = np.zeros((8, 3, 3), dtype=np.complex128)
    l[0][0, 1] = l[0][1, 0] = 1
    l[1][0, 1], l[1][1, 0] = -1j, 1j
    l[2][0, 0], l[2][1, 1] = 1, -1
    l[3][0, 2] = l[3][2, 0] = 1
    l[4][0, 2], l[4][2, 0] = -1j, 1j
    l[5][1, 2] = l[5][2, 1] = 1
    l[6][1, 2], l[6][2, 1] = -1j, 1j
    l[7][0, 0] = l[7][1, 1] = 1 / np.sqrt(3)
    l[7][2, 2] = -2 / np.sqrt(3)
    return l


def _expi_hermitian(h: np.ndarray, eps: float) -> np.ndarray:
    """exp(i eps h) for a stack of Hermitian 3x3 matrices, via eigendecomposition."""
    w, v = np.linalg.eigh(h)
    ph = np.exp(1j * eps * w)
    return np.einsum("...ij,...j,...kj->...ik", v, ph, v.conj())


def random_gauge(dims, seed: int, eps: float, chunk: int = 1 << 18) -> np.ndarray:
    """Random SU(3) gauge field ``U = exp(i eps H)`` on an X x Y x Z x T lattice.

    ``dims = (X, Y, Z, T)``.  Link ``l = 4 * site + mu`` (site lexicographic,
    x fastest) draws SplitMix64 outputs ``8 l .. 8 l + 7``; Box-Muller turns
    them into the eight Gaussian coefficients ``h_a``.
    Returns complex128 ``[T, Z, Y, X, 4, 3, 3]``.
    """
    X, Y, Z, T = (int(d) for d in dims)
    nlink = X * Y * Z * T * 4
    lam = gell_mann() / 2
    out = np.empty((nlink, 3, 3), dtype=np.complex128)
    for a0 in range(0, nlink, chunk):
        n = min(chunk, nlink - a0)
        ctr = (np.arange(a0, a0 + n, dtype=np.uint64)[:, None] * np.uint64(8)
               + np.arange(8, dtype=np.uint64)[None, :])
        u = _uniform_open(splitmix64(seed, ctr))
        rad = np.sqrt(-2.0 * np.log(u[:, 0::2]))
        ang = 2.0 * np.pi * u[:, 1::2]
        g = np.empty((n, 8))
        g[:, 0::2] = rad * np.cos(ang)
        g[:, 1::2] = rad * np.sin(ang)
        h = np.einsum("na,aij->nij", g, lam)
        out[a0:a0 + n] = _expi_hermitian(h, eps)
    return out.reshape(T, Z, Y, X, 4, 3, 3)


def unit_gauge(dims) -> np.ndarray:
    """The free field U = 1, layout [T, Z, Y, X, 4, 3, 3]."""
    X, Y, Z, T = dims
    u = np.zeros((T, Z, Y, X, 4, 3, 3), dtype=np.complex128)
    u[..., 0, 0] = u[..., 1, 1] = u[..., 2, 2] = 1
    return u


def random_su3_field(dims, seed: int, eps: float = 1.0) -> np.ndarray:
    """One random SU(3) matrix per site (a gauge transformation), [T, Z, Y, X, 3, 3]."""
    X, Y, Z, T = dims
    u = random_gauge((X, Y, Z, T), seed, eps)[..., 0, :, :]
    return u


def random_spinor(dims, seed: int, nrhs: int | None = None) -> np.ndarray:
    """Complex Gaussian spinor field(s), [T, Z, Y, X, 4, 3] (or [nrhs, ...]).

    Uses numpy's PCG64 generator: these are generic test vectors, not the
    estimator's noise.
    """
    X, Y, Z, T = dims
    shape = (T, Z, Y, X, 4, 3) if nrhs is None else (nrhs, T, Z, Y, X, 4, 3)
    rng = np.random.default_rng(seed)
    return (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) / np.sqrt(2)


# Workloads: the paper measures on 32^3 x 64 twisted-mass ensembles that are
# not available; these synthetic lattices stand in for them.
WORKLOADS = {
    "plain_4x4x4x4": dict(dims=(4, 4, 4, 4), eps=0.3, kappa=0.16, mu=0.01,
                          gauge_seed=1401, source_seed=6750),
    "tsm_16x16x16x32": dict(dims=(16, 16, 16, 32), eps=0.2, kappa=0.1615, mu=0.004,
                            gauge_seed=1402, source_seed=6751),
    "batched_24x24x24x48": dict(dims=(24, 24, 24, 48), eps=0.2, kappa=0.1615, mu=0.004,
                                gauge_seed=1403, source_seed=6752),
    # the volume of the paper's ensembles (largest size the tests run)
    "paper_32x32x32x64": dict(dims=(32, 32, 32, 64), eps=0.2, kappa=0.1615, mu=0.004,
                              gauge_seed=1404, source_seed=6753),
}
