"""Helpers for the GPU parity tests: device buffers through torch, lattice setup."""
from __future__ import annotations

import numpy as np

import paper_1401_6750_amd as dl
import synth


def torch():
    import torch as t
    return t


def dev(a: np.ndarray):
    """Host complex128 array -> contiguous device tensor."""
    t = torch()
    return t.from_numpy(np.ascontiguousarray(a)).to("cuda")


def host(x) -> np.ndarray:
    return x.detach().cpu().numpy()


def zeros_dev(shape, dtype="complex128"):
    t = torch()
    return t.zeros(shape, dtype=getattr(t, dtype), device="cuda")


class Lattice:
    """A library lattice with its gauge field; keeps the host copy for the oracle."""

    def __init__(self, ctx, dims, U, kappa, mu, bc=-1):
        self.ctx, self.dims, self.U, self.kappa, self.mu, self.bc = ctx, tuple(dims), U, kappa, mu, bc
        self.h = dl.dl_lattice_create(ctx, dims, bc)
        dl.dl_gauge_set(self.h, np.ascontiguousarray(U), 0)
        dl.dl_set_params(self.h, kappa, mu)
        X, Y, Z, T = dims
        self.V = X * Y * Z * T
        self.field_shape = (T, Z, Y, X, 4, 3)

    def close(self):
        dl.dl_lattice_destroy(self.h)


def make_lattice(ctx, dims, seed, eps, kappa, mu, bc=-1):
    return Lattice(ctx, dims, synth.random_gauge(dims, seed, eps), kappa, mu, bc)


def rel(a, b):
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))


def elementwise_check(got, want, rtol, atol, nblock):
    """Element-wise parity of loop arrays, without asserting.

    Every element must satisfy |got - want| <= rtol |want| + atol m, where m is the
    largest |want| of its block: one index of the leading ``nblock`` axes (flavour,
    op, Gamma for a [2][nops][16][T][Np] array) over the remaining ones (time slice,
    momentum).  A small wrong entry inside a block cannot hide behind the block's
    norm.  Returns (worst |got - want| / m, list of the first bad indices, count).
    """
    got = np.asarray(got)
    want = np.asarray(want)
    assert got.shape == want.shape, (got.shape, want.shape)
    axes = tuple(range(nblock, want.ndim))
    m = np.abs(want).max(axis=axes, keepdims=True)
    d = np.abs(got - want)
    bound = rtol * np.abs(want) + atol * m
    worst = float((d / np.where(m > 0, m, 1.0)).max()) if d.size else 0.0
    bad = d > bound
    idx = [tuple(int(i) for i in ix) for ix in np.argwhere(bad)[:4]]
    return worst, idx, int(bad.sum())


def elementwise(got, want, rtol, atol, nblock):
    """elementwise_check() that raises on any element out of bounds; returns the worst
    |got - want| / m, for the log."""
    worst, idx, nbad = elementwise_check(got, want, rtol, atol, nblock)
    if nbad:
        raise AssertionError(f"{nbad} of {np.asarray(want).size} elements out of bounds (rtol {rtol}, atol {atol}); "
                             f"first {idx}; worst |d|/m {worst:.3e}")
    return worst
