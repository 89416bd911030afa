"""Time dilution of the noise sources (FP64).

Test infrastructure: a plain CPU reference, used only by the tests and the
benchmark's CPU baseline; it shares no code with the HIP library.

The paper also works with time-diluted sources and has kernels that contract
either a whole vector or a single time slice, returning loops indexed by time
slice (Section 2.2); the dilution scheme itself is not spelled out.  Reading:

* D components per noise vector: component c (0 <= c < D) keeps eta on the
  time slices t with t mod D == c and is zero elsewhere; D = T gives one time
  slice per component.  The components sum to eta and have disjoint supports,
  so E[sum_c eta_c eta_c^dag] = 1 still holds and every estimator stays
  unbiased, while the noise products that couple different components -- the
  cross terms between those time slices -- drop out.
* Every component is solved on its own, s_c = M^-1 eta_c; the loop of one noise
  vector is the sum of its components' loops.  The one-end-trick structures
  contract each s_c over the whole lattice ("whole vector"); the estimators
  that pair s with eta itself (the hopping parameter expansion) are non-zero
  only next to the component's own time slices ("single time slice").
"""
from __future__ import annotations

import numpy as np

from . import hpe, loops


def slice_mask(T, D, c):
    """Boolean [T]: the time slices of component c."""
    return (np.arange(T) % D) == c


def split(eta, D):
    """The D components of a full-lattice field [..., T, Z, Y, X, 4, 3]."""
    T = eta.shape[-6]
    out = []
    for c in range(D):
        m = slice_mask(T, D, c).astype(float).reshape((T, 1, 1, 1, 1, 1))
        out.append(eta * m)
    return out


def one_end_site_loops(U, sols, kappa, bc_t, deriv=True):
    """One noise vector's one-end-trick loops from its component solutions:
    sum_c of the whole-vector contractions, [2, nops, 16, T, Z, Y, X]."""
    return sum(loops.source_site_loops(U, s, kappa, bc_t, deriv) for s in sols)


def hpe_site_loops(U, etas, sols, kappa, mu, bc_t, n, deriv=True):
    """One noise vector's no-tau_3 loops with the hopping parameter expansion of
    order n (exact part excluded): sum_c over the components' (eta_c, s_c)."""
    return sum(hpe.hpe_site_loops(U, e, s, kappa, mu, bc_t, n, deriv) for e, s in zip(etas, sols))
