"""One-end-trick fermion loops, momentum projection and the TSM estimator (FP64).

Section 2.1.1 computes all ultra-local and one-derivative insertions, with and
without tau_3 (160 in total), per time slice, at momenta up to a p^2 cut;
Section 2.2 builds every ultra-local Gamma from the colour-traced 4x4 Dirac
outer product of the two contracted vectors; Section 2.3 Fourier transforms
the per-site data and cuts in p^2.  The formulas are not printed, so the
readings below are used.

One-end trick (reading).  With s = M(mu)^-1 eta (kappa-normalised, u flavour)
and noise with E[eta eta^dag] = 1, E[s xi^dag] = M^-1 M^-dag X^dag for
xi = X s.  Two operator identities, which hold because M(mu) is
gamma_5-hermitian (M(mu)^dag = gamma_5 M(-mu) gamma_5), give both flavour
structures from the single u solve:

* with tau_3 (u - d):  M_u^-1 - M_d^-1 = -2 i (2 kappa mu) M_u^-1 M_u^-dag gamma_5
  -> xi = gamma_5 s, prefactor -2 i mu (2 kappa)^2 in physical normalisation;
* without tau_3 (u + d): M_u^-1 + M_d^-1 = 2 M_u^-1 M_u^-dag M_0^dag
  -> xi = M_0 s = (1 - kappa H) s, prefactor 4 kappa.

The per-source loop is ``xi^dag Gamma phi`` with phi = s; the estimator
averages over sources and multiplies by the prefactor.  Loops are traces of
the physically normalised propagators in the twisted basis; the fermion-loop
sign (-1) is not included.

Insertions.  Local: ``l_n(x) = xi(x)^dag Gamma_n phi(x)``.  One-derivative
(reading: the symmetric left-right covariant derivative)
``l_{n,nu}(x) = 1/2 [xi^dag Gamma_n (D_nu phi) - (D_nu xi)^dag Gamma_n phi](x)``
with ``(D_nu psi)(x) = 1/2 [U_nu(x) psi(x+nu) - U_nu(x-nu)^dag psi(x-nu)]``,
the time-boundary factor included.

Projection (reading): ``L(t, n) = sum_xvec exp(-2 pi i n.x / L) l(xvec, t)``
for integer vectors n with |n|^2 <= cut (the paper's "p^2"), components in
(-L/2, L/2], ordered by |n|^2 then (n_x, n_y, n_z) ascending.

Output index: ``[flavour][op][Gamma][t][momentum]`` with flavour 0 = tau_3,
1 = no tau_3, op 0 = local, 1..4 = derivative in x, y, z, t.
"""
from __future__ import annotations

import numpy as np

from . import dirac

TAU3, NOTAU3 = 0, 1


def prefactors(kappa, mu):
    """Physical-normalisation prefactors (tau_3, no tau_3)."""
    return np.array([-2j * mu * (2 * kappa) ** 2, 4 * kappa])


def xi_fields(U, s, kappa, bc_t, C=None):
    """The left vectors of the two flavour structures: gamma_5 s and M_0 s = (1 - kappa H) s
    (M_0 = 1 + C - kappa H with a clover term C)."""
    return dirac.spin_mul(dirac.GAMMA5, s), dirac.apply_M0(U, s, kappa, bc_t, C)


def outer_product(xi, phi):
    """Colour-traced Dirac outer product C_ab(x) = sum_c conj(xi_ac(x)) phi_bc(x)."""
    return np.einsum("...ac,...bc->...ab", xi.conj(), phi)


def insert_gammas(c):
    """l_n = sum_ab (Gamma_n)_ab C_ab = xi^dag Gamma_n phi; returns [16, ...]."""
    return np.einsum("nab,...ab->n...", dirac.GAMMA_BASIS, c)


def covariant_derivative(U, psi, nu, bc_t):
    """(D_nu psi)(x) = 1/2 [U_nu(x) psi(x+nu) - U_nu(x-nu)^dag psi(x-nu)]."""
    ax = dirac.SPINOR_AXIS[nu]
    fwd = dirac.color_mul(U[..., nu, :, :], dirac.shift_forward(psi, nu, bc_t, ax))
    bwd = dirac.shift_backward(dirac.color_mul_dag(U[..., nu, :, :], psi), nu, bc_t, ax)
    return 0.5 * (fwd - bwd)


def site_loops(U, xi, phi, bc_t, deriv=True):
    """Per-site insertions of one (xi, phi) pair: [nops, 16, T, Z, Y, X]."""
    ops = [insert_gammas(outer_product(xi, phi))]
    if deriv:
        for nu in range(4):
            a = outer_product(xi, covariant_derivative(U, phi, nu, bc_t))
            b = outer_product(covariant_derivative(U, xi, nu, bc_t), phi)
            ops.append(0.5 * (insert_gammas(a) - insert_gammas(b)))
    return np.stack(ops)


def source_site_loops(U, s, kappa, bc_t, deriv=True, C=None):
    """Both flavour structures for one solution s: [2, nops, 16, T, Z, Y, X]."""
    xi_t3, xi_1 = xi_fields(U, s, kappa, bc_t, C)
    return np.stack([site_loops(U, xi_t3, s, bc_t, deriv),
                     site_loops(U, xi_1, s, bc_t, deriv)])


def momenta(p2max, dims):
    """Integer momentum vectors with |n|^2 <= p2max, in output order; [Np, 3]."""
    X, Y, Z, _ = dims
    rng = [range(-(L // 2) + 1, L // 2 + 1) for L in (X, Y, Z)]
    vecs = [(nx, ny, nz) for nx in rng[0] for ny in rng[1] for nz in rng[2]
            if nx * nx + ny * ny + nz * nz <= p2max]
    vecs.sort(key=lambda n: (n[0] ** 2 + n[1] ** 2 + n[2] ** 2, n[0], n[1], n[2]))
    return np.array(vecs, dtype=np.int64).reshape(-1, 3)


def project(site_vals, moms, dims):
    """Fourier sum over space: [..., T, Z, Y, X] -> [..., T, Np]."""
    X, Y, Z, _ = dims
    px = np.exp(-2j * np.pi * np.outer(moms[:, 0], np.arange(X)) / X)
    py = np.exp(-2j * np.pi * np.outer(moms[:, 1], np.arange(Y)) / Y)
    pz = np.exp(-2j * np.pi * np.outer(moms[:, 2], np.arange(Z)) / Z)
    return np.einsum("...tzyx,px,py,pz->...tp", site_vals, px, py, pz)


def source_loops(U, s, kappa, bc_t, p2max, dims, deriv=True, C=None):
    """Projected per-source loops, without prefactor: [2, nops, 16, T, Np]."""
    moms = momenta(p2max, dims)
    return project(source_site_loops(U, s, kappa, bc_t, deriv, C), moms, dims)


def apply_prefactors(sums, kappa, mu):
    """Multiply flavour axis 0 of a [2, ...] array by the one-end-trick prefactors."""
    pf = prefactors(kappa, mu)
    return sums * pf.reshape((2,) + (1,) * (sums.ndim - 1))


def estimate(per_source, kappa, mu):
    """Plain stochastic estimator: prefactor x mean over sources (axis 0)."""
    return apply_prefactors(np.mean(per_source, axis=0), kappa, mu)


def tsm_combine(sum_lp, n_lp, sum_hp, sum_lpc, n_hp, kappa, mu):
    """Truncated solver method (Section 2.1; Bali, Collins & Schaefer's estimator).

    ``L = S_LP / N_LP + (S_HP - S_LPc) / N_HP`` with S_LP the sum over the many
    low-precision solves, S_HP the sum over the few high-precision solves and
    S_LPc the low-precision solves of the same N_HP sources (same LP map).
    Either tier may be empty; with no LP tier this is the plain estimator.
    """
    tot = 0.0
    if n_lp > 0:
        tot = tot + sum_lp / n_lp
    if n_hp > 0:
        tot = tot + (sum_hp - sum_lpc) / n_hp
    return apply_prefactors(np.asarray(tot), kappa, mu)


# ---------------------------------------------------------------------------
# exact loops from dense propagators (tiny lattices)
# ---------------------------------------------------------------------------

def exact_site_loops(U, kappa, mu, bc_t, dims, deriv=True, C=None):
    """Exact per-site loops tr[Gamma (D_u^-1 -+ D_d^-1)] from dense inverses.

    D^-1 = 2 kappa M^-1 (physical normalisation).  The derivative insertion is
    the trace form of ``site_loops``' definition:
    1/4 { tr[(Gamma x U_nu(x)) G(x+nu, x)] - tr[(Gamma x U_nu(x-nu)^dag) G(x-nu, x)]
          - tr[(Gamma x U_nu(x)^dag) G(x, x+nu)] + tr[(Gamma x U_nu(x-nu)) G(x, x-nu)] }.
    Returns [2, nops, 16, T, Z, Y, X].
    """
    X, Y, Z, T = dims
    V = X * Y * Z * T
    gu = 2 * kappa * np.linalg.inv(dirac.dense_M(U, kappa, mu, bc_t, dims, C))
    gd = 2 * kappa * np.linalg.inv(dirac.dense_M(U, kappa, -mu, bc_t, dims, C))
    out = []
    coords = [(t, z, y, x) for t in range(T) for z in range(Z) for y in range(Y)
              for x in range(X)]
    lex = {c: i for i, c in enumerate(coords)}
    ext = {0: X, 1: Y, 2: Z, 3: T}

    def neighbour(c, nu, step):
        t, z, y, x = c
        v = [x, y, z, t]
        v[nu] += step
        sign = 1.0
        if nu == 3 and not (0 <= v[3] < T):
            sign = bc_t
        v[nu] %= ext[nu]
        return lex[(v[3], v[2], v[1], v[0])], sign

    for g in (gu - gd, gu + gd):
        G = g.reshape(V, 4, 3, V, 4, 3)
        loc = np.zeros((16, V), dtype=complex)
        for i in range(V):
            blk = G[i, :, :, i, :, :]                   # [beta, b, alpha, a]
            loc[:, i] = np.einsum("nab,bcac->n", dirac.GAMMA_BASIS, blk)
        ops = [loc]
        if deriv:
            for nu in range(4):
                d = np.zeros((16, V), dtype=complex)
                for i, c in enumerate(coords):
                    jp, sp = neighbour(c, nu, +1)
                    jm, sm = neighbour(c, nu, -1)
                    u_here = U[c][nu]
                    u_back = U[coords[jm]][nu]
                    # tr[(Gamma x W) G(y, x)] = sum Gamma_ab W_ij G[y, b, j, x, a, i]
                    t1 = np.einsum("nab,ij,bjai->n", dirac.GAMMA_BASIS, u_here, G[jp, :, :, i, :, :])
                    t2 = np.einsum("nab,ij,bjai->n", dirac.GAMMA_BASIS, u_back.conj().T, G[jm, :, :, i, :, :])
                    t3 = np.einsum("nab,ij,bjai->n", dirac.GAMMA_BASIS, u_here.conj().T, G[i, :, :, jp, :, :])
                    t4 = np.einsum("nab,ij,bjai->n", dirac.GAMMA_BASIS, u_back, G[i, :, :, jm, :, :])
                    d[:, i] = 0.25 * (sp * t1 - sm * t2 - sp * t3 + sm * t4)
                ops.append(d)
        out.append(np.stack(ops))
    return np.stack(out).reshape(2, -1, 16, T, Z, Y, X)
