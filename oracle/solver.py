"""Solvers for M s = eta (Section 2, eq. (1)), FP64.

The paper inverts with QUDA's twisted-mass CG and states only the target
residuals of the two TSM tiers (Section 2.1: rho ~ 1e-2 for the many
low-precision solves, rho ~ 1e-8 for the few corrections).  Reading:

* The solve is CG on the normal equations of the even-odd (Schur complement)
  system, ``Mhat^dag Mhat s_o = Mhat^dag bhat`` (CGNR), followed by the
  even-site reconstruction.  ``pAp`` is evaluated as ``||Mhat p||^2``.
* rho is the solver's own relative residual: stop at the first iteration with
  ``||r|| <= rho ||Mhat^dag bhat||`` where r is the iterated residual of the
  normal system.  The true residual ``||eta - M s|| / ||eta||`` is reported
  alongside.

``cgnr_eo`` spells out the iteration exactly as the GPU path runs it, so an
FP64 GPU solve takes the same number of iterations and agrees to rounding.
"""
from __future__ import annotations

import numpy as np

from . import dirac


def vdot(a, b):
    """<a, b> = sum conj(a) b over all sites and components."""
    return np.vdot(a.ravel(), b.ravel())


def cgnr_eo(U, eta, kappa, mu, bc_t, dims, tol, maxiter=10000, C=None):
    """Even-odd CGNR solve of M(mu) s = eta.

    Returns (s, info) with s the full-lattice solution and info a dict holding
    the iteration count, the final iterated relative residual and whether it
    converged.  C: optional clover term (oracle/clover.py).
    """
    bhat = dirac.schur_rhs(U, eta, kappa, mu, bc_t, dims, C)
    c = dirac.Mhat_dag(U, bhat, kappa, mu, bc_t, dims, C)
    x = np.zeros_like(c)
    r = c.copy()
    p = r.copy()
    rr = vdot(r, r).real
    cc = rr
    it = 0
    converged = rr <= tol * tol * cc
    while not converged and it < maxiter:
        t = dirac.Mhat(U, p, kappa, mu, bc_t, dims, C)
        pap = vdot(t, t).real
        alpha = rr / pap
        x = x + alpha * p
        r = r - alpha * dirac.Mhat_dag(U, t, kappa, mu, bc_t, dims, C)
        rr_new = vdot(r, r).real
        it += 1
        if rr_new <= tol * tol * cc:
            converged = True
            rr = rr_new
            break
        beta = rr_new / rr
        p = r + beta * p
        rr = rr_new
    s = dirac.reconstruct_even(U, eta, x, kappa, mu, bc_t, dims, C)
    info = dict(iters=it, rel_resid=float(np.sqrt(rr / cc)) if cc > 0 else 0.0,
                converged=bool(converged))
    return s, info


def true_residual(U, eta, s, kappa, mu, bc_t, C=None):
    """||eta - M s|| / ||eta||, evaluated with the full-lattice operator."""
    r = eta - dirac.apply_M(U, s, kappa, mu, bc_t, C)
    return float(np.linalg.norm(r.ravel()) / np.linalg.norm(eta.ravel()))


def dense_solve(U, eta, kappa, mu, bc_t, dims, C=None):
    """Exact solve by dense LU (tiny lattices only)."""
    m = dirac.dense_M(U, kappa, mu, bc_t, dims, C)
    shape = eta.shape
    return np.linalg.solve(m, eta.reshape(-1)).reshape(shape)
