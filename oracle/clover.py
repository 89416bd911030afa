"""Clover (Sheikholeslami-Wohlert) term of the twisted-mass operator, FP64.

Test infrastructure: plain, slow reference code; the library never calls it.

Section 2.4 expects the package to work for Wilson and clover fermions as well,
without printing either operator.  Reading taken here: the standard O(a)
improved Wilson operator, in kappa normalisation,

    M(mu) = 1 + C - kappa H + 2 i kappa mu gamma_5,
    C(x)  = i kappa c_sw sum_{mu < nu} sigma_{mu nu} Fhat_{mu nu}(x),
    sigma_{mu nu} = (i / 2) [gamma_mu, gamma_nu],
    Fhat_{mu nu}(x) = (Q_{mu nu}(x) - Q_{mu nu}(x)^dag) / 8,

with Q_{mu nu}(x) the sum of the four plaquettes of the (mu, nu) plane that start
and end at x, each walked in the same sense as U_mu(x) U_nu(x + mu) U_mu(x + nu)^dag
U_nu(x)^dag.  The links close the plaquettes periodically in every direction; the
time-boundary factor belongs to the fermion hops only.  C is hermitian and
commutes with gamma_5, so in the chiral basis it is two 6 x 6 blocks per site
(spins 0, 1 and spins 2, 3).  C does not depend on mu, hence
M(mu)^dag = gamma_5 M(-mu) gamma_5 still holds and the one-end-trick identities
keep their form with M_0 = 1 + C - kappa H.

Layout: C is [..., T, Z, Y, X, 4, 3, 4, 3] (row spin, row colour, column spin,
column colour).
"""
from __future__ import annotations

import numpy as np

from . import dirac

# lattice axis of direction mu in a [T, Z, Y, X, 3, 3] link-component array
LINK_AXIS = {0: -3, 1: -4, 2: -5, 3: -6}


def sigma(mu, nu):
    """sigma_{mu nu} = (i/2) [gamma_mu, gamma_nu]."""
    g = dirac.GAMMA
    return 0.5j * (g[mu] @ g[nu] - g[nu] @ g[mu])


def _at(a, d, step):
    """a(x + step * d) for a link-component array a[T, Z, Y, X, 3, 3]."""
    return np.roll(a, -step, axis=LINK_AXIS[d])


def _mm(*ms):
    out = ms[0]
    for m in ms[1:]:
        out = np.einsum("...ab,...bc->...ac", out, m)
    return out


def _dag(a):
    return np.swapaxes(a.conj(), -1, -2)


def clover_leaves(U, mu, nu):
    """Q_{mu nu}(x): the four plaquettes of the (mu, nu) plane at x, [T, Z, Y, X, 3, 3]."""
    um, un = U[..., mu, :, :], U[..., nu, :, :]
    p1 = _mm(um, _at(un, mu, 1), _dag(_at(um, nu, 1)), _dag(un))
    # x -> x + nu -> x + nu - mu -> x - mu -> x
    p2 = _mm(un, _dag(_at(_at(um, nu, 1), mu, -1)), _dag(_at(un, mu, -1)), _at(um, mu, -1))
    # x -> x - mu -> x - mu - nu -> x - nu -> x
    p3 = _mm(_dag(_at(um, mu, -1)), _dag(_at(_at(un, mu, -1), nu, -1)), _at(_at(um, mu, -1), nu, -1),
             _at(un, nu, -1))
    # x -> x - nu -> x - nu + mu -> x + mu -> x
    p4 = _mm(_dag(_at(un, nu, -1)), _at(um, nu, -1), _at(_at(un, nu, -1), mu, 1), _dag(um))
    return p1 + p2 + p3 + p4


def field_strength(U, mu, nu):
    """Fhat_{mu nu}(x) = (Q - Q^dag) / 8 (anti-hermitian), [T, Z, Y, X, 3, 3]."""
    q = clover_leaves(U, mu, nu)
    return (q - _dag(q)) / 8.0


def clover_term(U, kappa, csw):
    """C(x) = i kappa c_sw sum_{mu<nu} sigma_{mu nu} (x) Fhat_{mu nu}(x); [T, Z, Y, X, 4, 3, 4, 3]."""
    shape = U.shape[:-3] + (4, 3, 4, 3)
    c = np.zeros(shape, dtype=complex)
    for mu in range(4):
        for nu in range(mu + 1, 4):
            f = field_strength(U, mu, nu)
            c += np.einsum("sr,...ab->...sarb", sigma(mu, nu), f)
    return 1j * kappa * csw * c


def apply_C(C, psi):
    """(C psi)(x) = sum C(x)[s, a, r, b] psi(x)[r, b]."""
    return np.einsum("...sarb,...rb->...sa", C, psi)


def site_matrix(C, kappa, mu):
    """A(x) = 1 + C(x) + 2 i kappa mu gamma_5 as [..., 12, 12] (index 3 spin + colour)."""
    n = C.shape[:-4]
    a = C.reshape(n + (12, 12)).copy()
    g5 = np.repeat(np.real(np.diag(dirac.GAMMA5)), 3)
    a += np.diag(1.0 + 2j * kappa * mu * g5)
    return a


def apply_site_inverse(C, kappa, mu, psi):
    """A(x)^-1 psi(x), A = 1 + C + 2 i kappa mu gamma_5, by a linear solve per site."""
    a = site_matrix(C, kappa, mu)
    shape = psi.shape
    v = psi.reshape(shape[:-2] + (12,))
    a = np.broadcast_to(a, v.shape[:-1] + (12, 12))
    return np.linalg.solve(a, v[..., None])[..., 0].reshape(shape)
