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
