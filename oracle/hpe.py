"""Hopping parameter expansion (HPE) of the loops without tau_3 (FP64).

Test infrastructure: a plain CPU reference, used only by the tests and the
benchmark's CPU baseline; it shares no code with the HIP library.

The paper lists the HPE (Section 2.3, the interfaces) among the variance
reduction methods it combines with the TSM, without printing a formula.  The
reading used here:

Expansion.  With A = 1 + 2 i kappa mu gamma_5 (site-diagonal), B = A^-1 and the
kappa-normalised operator M = A - kappa H, the inverse is the geometric series

    M^-1 = sum_{k<n} T_k + R_n,   T_k = (kappa B H)^k B,   R_n = (kappa B H)^n M^-1 .

T_k couples only sites at most k hops apart.  The near-diagonal elements of
M^-1, which dominate the noise of a volume-source estimate, begin at order
kappa^0 in M^-1 but at order kappa^n in R_n, so the low orders are added
exactly and only R_n is estimated: with s = M^-1 eta and E[eta eta^dag] = 1,
R_n ~ phi eta^dag for phi = (kappa B H)^n s.

Flavour sum.  M_d = M(-mu) = gamma_5 M_u^dag gamma_5 and, term by term,
T_k^d = gamma_5 (T_k^u)^dag gamma_5, hence R_n^d = gamma_5 (R_n^u)^dag gamma_5,
estimated from the same sample by (gamma_5 eta)(gamma_5 phi)^dag.  The
per-source loop of the no-tau_3 structure is

    1/2 [ l(xi = eta, phi) + l(xi = gamma_5 phi, phi = gamma_5 eta) ]

with l the insertions of ``loops.site_loops`` (local and one-derivative), an
estimate of 1/2 tr Gamma (R_n^u + R_n^d) that takes the prefactor 4 kappa of
the generalised one-end trick; the exact part 1/2 tr Gamma (T^u + T^d) of the
subtracted orders is added per site.

Orders.  Local insertions subtract the orders k < n (n = 1..4), one-derivative
insertions the orders k < min(n, 3).  For those orders every subtracted
element -- closed paths of length <= 3 for the diagonal, open paths of length
<= 2 between neighbours -- retraces its own links, so it does not depend on the
gauge field, provided every lattice extent is at least 4 (no path of these
lengths winds around the lattice).  The exact part is then a constant per
site, computed here by summing the free-field spin factors of all hopping
paths.
"""
from __future__ import annotations

import itertools

import numpy as np

from . import dirac, loops

MAX_ORDER = 4


def deriv_order(n):
    """Order used by the one-derivative insertions for HPE order n."""
    return min(n, 3)


def hpe_fields(U, s, kappa, mu, bc_t, n):
    """[s, X s, X^2 s, ..., X^n s] with X = kappa A(mu)^-1 H."""
    binv = 1.0 / dirac.twist_diag(kappa, mu)
    out = [s]
    for _ in range(n):
        out.append(kappa * dirac.apply_spin_diag(binv, dirac.hop(U, out[-1], bc_t)))
    return out


def hpe_site_loops(U, eta, s, kappa, mu, bc_t, n, deriv=True):
    """Per-source no-tau_3 loops with HPE of order n (n = 0: the plain volume-source
    estimator of the flavour sum), without prefactor and exact part:
    [nops, 16, T, Z, Y, X]."""
    f = hpe_fields(U, s, kappa, mu, bc_t, n)
    g5 = dirac.GAMMA5

    def both_flavours(phi, use_deriv):
        u = loops.site_loops(U, eta, phi, bc_t, use_deriv)
        d = loops.site_loops(U, dirac.spin_mul(g5, phi), dirac.spin_mul(g5, eta), bc_t, use_deriv)
        return 0.5 * (u + d)

    local = both_flavours(f[n], False)
    if not deriv:
        return local
    der = both_flavours(f[deriv_order(n)], True)[1:]
    return np.concatenate([local, der])


def hpe_source_loops(U, eta, s, kappa, mu, bc_t, n, p2max, dims, deriv=True):
    """Projected per-source no-tau_3 HPE loops: [nops, 16, T, Np]."""
    moms = loops.momenta(p2max, dims)
    return loops.project(hpe_site_loops(U, eta, s, kappa, mu, bc_t, n, deriv), moms, dims)


# ---------------------------------------------------------------------------
# exact low orders
# ---------------------------------------------------------------------------

def _free_path_sum(kappa, mu, k, disp):
    """Spin matrix of T_k(x, x + disp) on the free field: the sum over all paths of
    k hops from x to x + disp of kappa^k B S_1 B S_2 ... B S_k B, where a hop from z
    to z + nu carries (1 - gamma_nu) and a hop to z - nu carries (1 + gamma_nu)."""
    one = np.eye(4, dtype=complex)
    B = np.diag(1.0 / dirac.twist_diag(kappa, mu))
    steps = [(nu, sgn) for nu in range(4) for sgn in (+1, -1)]
    tot = np.zeros((4, 4), dtype=complex)
    for path in itertools.product(steps, repeat=k):
        d = [0, 0, 0, 0]
        m = B.copy()
        for nu, sgn in path:
            d[nu] += sgn
            m = m @ (kappa * (one - sgn * dirac.GAMMA[nu])) @ B
        if tuple(d) == tuple(disp):
            tot += m
    return tot


def hpe_exact(kappa, mu, n, deriv=True):
    """Exact part per site, 1/2 sum_{k<n'} tr Gamma (T_k^u + T_k^d), for each insertion
    (n' = n local, min(n, 3) derivative), colour trace included: [nops, 16].

    The derivative insertion is the trace form of ``loops.site_loops``:
    1/4 {tr[Gamma U T(x+nu, x)] - tr[Gamma U^dag T(x-nu, x)] - tr[Gamma T(x, x+nu) U^dag]
         + tr[Gamma T(x, x-nu) U]}, in which every link product is the identity here.
    """
    G = dirac.GAMMA_BASIS
    zero = (0, 0, 0, 0)
    out = [np.zeros(16, dtype=complex)]
    for flav_mu in (mu, -mu):
        for k in range(n):
            t = _free_path_sum(kappa, flav_mu, k, zero)
            out[0] += 0.5 * 3 * np.einsum("nab,ba->n", G, t)
    if deriv:
        for nu in range(4):
            e = np.zeros(4, dtype=int)
            e[nu] = 1
            acc = np.zeros(16, dtype=complex)
            for flav_mu in (mu, -mu):
                for k in range(deriv_order(n)):
                    fwd = _free_path_sum(kappa, flav_mu, k, tuple(e))     # T(y, y + nu)
                    bwd = _free_path_sum(kappa, flav_mu, k, tuple(-e))    # T(y, y - nu)
                    # T(x+nu, x) = bwd, T(x-nu, x) = fwd, T(x, x+nu) = fwd, T(x, x-nu) = bwd
                    m = 0.25 * (bwd - fwd - fwd + bwd)
                    acc += 0.5 * 3 * np.einsum("nab,ba->n", G, m)
            out.append(acc)
    return np.stack(out)


def hpe_exact_projected(kappa, mu, n, p2max, dims, deriv=True):
    """The exact part projected to momenta: X Y Z times the per-site constant at n = 0,
    zero elsewhere: [nops, 16, T, Np]."""
    X, Y, Z, T = dims
    moms = loops.momenta(p2max, dims)
    ex = hpe_exact(kappa, mu, n, deriv)
    out = np.zeros(ex.shape + (T, len(moms)), dtype=complex)
    zero = np.where((moms == 0).all(axis=1))[0]
    if len(zero):
        out[..., zero[0]] = (X * Y * Z) * ex[..., None]
    return out
