"""Gradients of the one-end-trick loops with respect to the sources and mu (FP64).

The paper computes loops but no gradients; this is the derivative of the same
estimator, used by the backward pass of the loop function.  Convention (PyTorch's for
complex tensors): the gradient of a real loss F with respect to a complex z is
dF/dRe z + i dF/dIm z (= 2 dF/dz^*).  With upstream gradient g of the loops L,
F = Re sum_k conj(g_k) L_k to first order, and:

* every per-source loop is a quadratic form c s^dag B_k s with s = M^-1 eta, so
  grad_eta = M^-dag (B + B^dag) s with B = sum_k conj(g_k) c_k B_k;
* dF/dmu = Re sum_k conj(g_k) dL_k/dmu = (1/mu) Re sum_r s_r^dag B_tau3 s_r
           - sum_r Re[(P s_r)^dag z_r],  P = dM/dmu = 2 i kappa gamma_5,
  z_r = M^-dag (B + B^dag) s_r (only the tau_3 prefactor depends on mu).

B is assembled from per-site spin matrices
  Omega_{f,op}(x) = (pf_f / N) sum_n [sum_p conj(g[f,op,n,t,p]) e^{-ip.x}] Gamma_n
as  B = gamma_5 Q_tau3 + M_0^dag Q_1,
  Q_f = Omega_{f,0} + 1/2 sum_nu (Omega_{f,nu} D_nu + D_nu Omega_{f,nu}),
using D_nu^dag = -D_nu.  ``loss`` and finite differences of it pin this.
"""
from __future__ import annotations

import numpy as np

from . import dirac, loops, solver


def omega_fields(g, kappa, mu, nsrc, p2max, dims):
    """Per-site spin matrices Omega_{f,op}(x): [2, nops, T, Z, Y, X, 4, 4]."""
    X, Y, Z, T = dims
    moms = loops.momenta(p2max, dims)
    z, y, x = np.meshgrid(np.arange(Z), np.arange(Y), np.arange(X), indexing="ij")
    phase = np.exp(-2j * np.pi * (moms[:, 0, None, None, None] * x / X + moms[:, 1, None, None, None] * y / Y
                                  + moms[:, 2, None, None, None] * z / Z))      # [Np, Z, Y, X]
    pf = loops.prefactors(kappa, mu) / nsrc
    a = np.einsum("fontp,pzyx->fontzyx", np.conj(g), phase) * pf[:, None, None, None, None, None, None]
    return np.einsum("fontzyx,nab->fotzyxab", a, dirac.GAMMA_BASIS)


def _site_mat(om, u):
    """(Omega u)(x) for per-site spin matrices om [..., 4, 4] and spinors u [..., 4, 3]."""
    return np.einsum("...ab,...bc->...ac", om, u)


def apply_Q(U, om_f, u, bc_t, adjoint=False):
    """Q u (or Q^dag u) for one flavour's Omega fields om_f [nops, T, Z, Y, X, 4, 4]."""
    if adjoint:
        om_f = np.conj(np.swapaxes(om_f, -1, -2))
    out = _site_mat(om_f[0], u)
    for nu in range(om_f.shape[0] - 1):
        w = om_f[1 + nu]
        a = _site_mat(w, loops.covariant_derivative(U, u, nu, bc_t))
        b = loops.covariant_derivative(U, _site_mat(w, u), nu, bc_t)
        out = out + (-0.5 if adjoint else 0.5) * (a + b)
    return out


def apply_B_plus_Bdag(U, om, s, kappa, bc_t):
    """(B + B^dag) s for the Omega fields of both flavours."""
    g5 = dirac.GAMMA5
    m0s = dirac.apply_M0(U, s, kappa, bc_t)
    v = dirac.spin_mul(g5, apply_Q(U, om[0], s, bc_t))
    v = v + apply_Q(U, om[0], dirac.spin_mul(g5, s), bc_t, adjoint=True)
    q1 = apply_Q(U, om[1], s, bc_t)
    v = v + q1 - kappa * dirac.hop(U, q1, bc_t, dagger=True)       # M_0^dag Q_1 s
    v = v + apply_Q(U, om[1], m0s, bc_t, adjoint=True)
    return v


def solve_dagger(U, v, kappa, mu, bc_t, dims, tol):
    """z = M(mu)^-dag v via M^dag = gamma_5 M(-mu) gamma_5."""
    g5 = dirac.GAMMA5
    zp, _ = solver.cgnr_eo(U, dirac.spin_mul(g5, v), kappa, -mu, bc_t, dims, tol)
    return dirac.spin_mul(g5, zp)


def vjp(U, etas, g, kappa, mu, bc_t, dims, p2max, tol=1e-12, sols=None):
    """(grad_eta per source [nsrc, ...], dF/dmu) for upstream gradient g."""
    nsrc = len(etas)
    om = omega_fields(g, kappa, mu, nsrc, p2max, dims)
    g5 = dirac.GAMMA5
    grads = []
    dmu = 0.0
    for r, eta in enumerate(etas):
        s = sols[r] if sols is not None else solver.cgnr_eo(U, eta, kappa, mu, bc_t, dims, tol)[0]
        z = solve_dagger(U, apply_B_plus_Bdag(U, om, s, kappa, bc_t), kappa, mu, bc_t, dims, tol)
        grads.append(z)
        bt3s = dirac.spin_mul(g5, apply_Q(U, om[0], s, bc_t))
        dmu += np.real(np.vdot(s, bt3s)) / mu
        dmu -= 2.0 * kappa * np.imag(np.vdot(dirac.spin_mul(g5, s), z))
    return np.array(grads), float(dmu)


def loss(U, etas, g, kappa, mu, bc_t, dims, p2max, solve):
    """F = Re sum_k conj(g_k) L_k for the plain estimator over `etas`.

    `solve(eta, mu)` returns M(mu)^-1 eta (dense or CG)."""
    per = [loops.source_loops(U, solve(eta, mu), kappa, bc_t, p2max, dims, deriv=g.shape[1] > 1)
           for eta in etas]
    L = loops.estimate(np.array(per), kappa, mu)
    return float(np.real(np.vdot(g, L)))
