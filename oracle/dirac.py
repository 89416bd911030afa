"""Gamma matrices, lattice geometry and the twisted-mass Wilson operator (FP64).

Conventions (the paper names the twisted-mass operator, Section 2.1.1, but
prints neither its form nor a gamma basis; these are the readings taken):

* Fields are full-lattice numpy arrays.  Spinor: ``[..., T, Z, Y, X, 4, 3]``
  (spin, colour); gauge: ``[T, Z, Y, X, 4, 3, 3]`` with ``mu = 0..3`` for
  x, y, z, t.  Leading axes (``...``) are batch axes.
* Euclidean chiral basis: ``gamma_k = [[0, -i sigma_k], [i sigma_k, 0]]``
  (k = 1, 2, 3), ``gamma_4 = [[0, 1], [1, 0]]``, ``gamma_5 = g1 g2 g3 g4 =
  diag(1, 1, -1, -1)``.
* Hopping term ``(H psi)(x) = sum_mu (1 - gamma_mu) U_mu(x) psi(x + mu)
  + (1 + gamma_mu) U_mu(x - mu)^dag psi(x - mu)``; periodic in space, a hop
  that crosses the time boundary picks up ``bc_t`` (-1: antiperiodic).
* kappa-normalised twisted-mass operator of the u flavour
  ``M(mu) = 1 - kappa H + 2 i kappa mu gamma_5``; the d flavour is ``M(-mu)``.
  In physical normalisation ``M / (2 kappa) = D_W + i mu gamma_5``.
* Even-odd split by the parity ``(x + y + z + t) mod 2``; even-odd fields are
  full arrays that vanish on the other parity.
"""
from __future__ import annotations

import numpy as np

# lattice axis of direction mu in a [..., T, Z, Y, X, 4, 3] spinor
SPINOR_AXIS = {0: -3, 1: -4, 2: -5, 3: -6}


def gamma_matrices():
    """Return (gamma_1..gamma_4 as [4, 4, 4], gamma_5) in the chiral basis."""
    s = [np.array([[0, 1], [1, 0]], dtype=complex),
         np.array([[0, -1j], [1j, 0]], dtype=complex),
         np.array([[1, 0], [0, -1]], dtype=complex)]
    z = np.zeros((2, 2), dtype=complex)
    one = np.eye(2, dtype=complex)
    g = [np.block([[z, -1j * sk], [1j * sk, z]]) for sk in s]
    g.append(np.block([[z, one], [one, z]]))
    g = np.array(g)
    g5 = g[0] @ g[1] @ g[2] @ g[3]
    return g, g5


GAMMA, GAMMA5 = gamma_matrices()


def gamma_basis():
    """The 16 insertions ``Gamma_n = g1^n0 g2^n1 g3^n2 g4^n3`` (n0 = lowest bit).

    Section 2.2 only says any Gamma can be rebuilt from the 4x4 outer product;
    this bit-indexed ordering of the Clifford basis is the reading used for the
    output index.  ``Gamma_15 = gamma_5``.
    """
    out = np.zeros((16, 4, 4), dtype=complex)
    for n in range(16):
        m = np.eye(4, dtype=complex)
        for k in range(4):
            if (n >> k) & 1:
                m = m @ GAMMA[k]
        out[n] = m
    return out


GAMMA_BASIS = gamma_basis()


def lattice_shape(dims):
    X, Y, Z, T = dims
    return (T, Z, Y, X)


def parity(dims) -> np.ndarray:
    """Site parity (x + y + z + t) mod 2 as an int array [T, Z, Y, X]."""
    X, Y, Z, T = dims
    t, z, y, x = np.meshgrid(np.arange(T), np.arange(Z), np.arange(Y), np.arange(X),
                             indexing="ij")
    return (x + y + z + t) % 2


def shift_forward(f, mu, bc_t, lat_axis):
    """f(x + mu): roll by one site, boundary factor on hops across t = T-1 -> 0."""
    g = np.roll(f, -1, axis=lat_axis)
    if mu == 3 and bc_t != 1:
        idx = [slice(None)] * g.ndim
        idx[lat_axis] = -1
        g[tuple(idx)] *= bc_t
    return g


def shift_backward(f, mu, bc_t, lat_axis):
    """f(x - mu): roll by one site, boundary factor on hops across t = 0 -> T-1."""
    g = np.roll(f, 1, axis=lat_axis)
    if mu == 3 and bc_t != 1:
        idx = [slice(None)] * g.ndim
        idx[lat_axis] = 0
        g[tuple(idx)] *= bc_t
    return g


def color_mul(u, psi):
    """(U psi)_a = sum_b U_ab psi_b per site and spin; u [..., 3, 3], psi [..., 4, 3]."""
    return np.einsum("...ab,...sb->...sa", u, psi)


def color_mul_dag(u, psi):
    """(U^dag psi)_a = sum_b conj(U_ba) psi_b."""
    return np.einsum("...ba,...sb->...sa", u.conj(), psi)


def spin_mul(g, psi):
    """(G psi)_s = sum_r G_sr psi_r for a 4x4 spin matrix."""
    return np.einsum("sr,...rc->...sc", g, psi)


def hop(U, psi, bc_t, dagger=False):
    """Wilson hopping term H psi (or its adjoint H^dag psi).

    The adjoint swaps the spin projectors: forward hops carry (1 + gamma_mu),
    backward hops (1 - gamma_mu).
    """
    one = np.eye(4, dtype=complex)
    out = np.zeros_like(psi, dtype=complex)
    for mu in range(4):
        ax = SPINOR_AXIS[mu]
        pf = one + GAMMA[mu] if dagger else one - GAMMA[mu]
        pb = one - GAMMA[mu] if dagger else one + GAMMA[mu]
        fwd = color_mul(U[..., mu, :, :], shift_forward(psi, mu, bc_t, ax))
        bwd = shift_backward(color_mul_dag(U[..., mu, :, :], psi), mu, bc_t, ax)
        out += spin_mul(pf, fwd) + spin_mul(pb, bwd)
    return out


def twist_diag(kappa, mu):
    """Per-spin diagonal of A = 1 + 2 i kappa mu gamma_5 (gamma_5 is diagonal here)."""
    return 1.0 + 2j * kappa * mu * np.real(np.diag(GAMMA5))


def apply_spin_diag(d, psi):
    return psi * d[:, None]


def _clover(C, psi):
    """C psi for a clover term C [..., 4, 3, 4, 3] (oracle/clover.py), 0 without one."""
    if C is None:
        return 0.0
    return np.einsum("...sarb,...rb->...sa", C, psi)


def apply_M(U, psi, kappa, mu, bc_t, C=None):
    """M(mu) psi = psi - kappa H psi + 2 i kappa mu gamma_5 psi (+ C psi with a clover term)."""
    return psi - kappa * hop(U, psi, bc_t) + 2j * kappa * mu * spin_mul(GAMMA5, psi) + _clover(C, psi)


def apply_Mdag(U, psi, kappa, mu, bc_t, C=None):
    """M(mu)^dag psi = psi - kappa H^dag psi - 2 i kappa mu gamma_5 psi (+ C psi, C hermitian)."""
    return (psi - kappa * hop(U, psi, bc_t, dagger=True) - 2j * kappa * mu * spin_mul(GAMMA5, psi)
            + _clover(C, psi))


def apply_M0(U, psi, kappa, bc_t, C=None):
    """The mu-independent part M_0 = 1 - kappa H (= 2 kappa D_W), plus C with a clover term."""
    return psi - kappa * hop(U, psi, bc_t) + _clover(C, psi)


def apply_A_inv(psi, kappa, mu, C=None):
    """A^-1 psi with the site-diagonal part A = 1 + 2 i kappa mu gamma_5 (+ C): per spin,
    or by a 12 x 12 linear solve per site with a clover term."""
    if C is None:
        return apply_spin_diag(1.0 / twist_diag(kappa, mu), psi)
    from . import clover
    return clover.apply_site_inverse(C, kappa, mu, psi)


def hop_at_sites(U, psi, bc_t, sites):
    """(H psi)(x) at a list of sites (t, z, y, x), one site at a time.

    A second, site-by-site spelling of ``hop`` used to check outputs of very
    large lattices where the whole-field version is too slow.
    Returns [len(sites), 4, 3].
    """
    T, Z, Y, X = psi.shape[-6:-2]
    ext = {0: X, 1: Y, 2: Z, 3: T}
    one = np.eye(4, dtype=complex)
    out = np.zeros((len(sites), 4, 3), dtype=complex)
    for i, (t, z, y, x) in enumerate(sites):
        acc = np.zeros((4, 3), dtype=complex)
        for mu in range(4):
            c = [x, y, z, t]
            fw, bw = list(c), list(c)
            fw[mu] += 1
            bw[mu] -= 1
            sf = bc_t if (mu == 3 and fw[3] == T) else 1.0
            sb = bc_t if (mu == 3 and bw[3] < 0) else 1.0
            fw[mu] %= ext[mu]
            bw[mu] %= ext[mu]
            pf = psi[fw[3], fw[2], fw[1], fw[0]]
            pb = psi[bw[3], bw[2], bw[1], bw[0]]
            uf = U[t, z, y, x, mu]
            ub = U[bw[3], bw[2], bw[1], bw[0], mu]
            acc += sf * (one - GAMMA[mu]) @ (pf @ uf.T)
            acc += sb * (one + GAMMA[mu]) @ (pb @ ub.conj())
        out[i] = acc
    return out


# ---------------------------------------------------------------------------
# even-odd (Schur complement on odd sites)
# ---------------------------------------------------------------------------

def parity_mask(dims, p):
    """[T, Z, Y, X, 1, 1] mask selecting parity p."""
    return (parity(dims) == p).astype(float)[..., None, None]


def project(psi, mask):
    return psi * mask


def Mhat(U, psi_o, kappa, mu, bc_t, dims, C=None):
    """Schur complement on odd sites: 1 - kappa^2 A_o^-1 H_oe A_e^-1 H_eo.

    With M = [[A_e, -kappa H_eo], [-kappa H_oe, A_o]] (even block first), the
    odd-site equation after eliminating the even sites is
    A_o^-1 (A_o - kappa^2 H_oe A_e^-1 H_eo) s_o = A_o^-1 (eta_o + kappa H_oe A_e^-1 eta_e).
    """
    me, mo = parity_mask(dims, 0), parity_mask(dims, 1)
    u = apply_A_inv(me * hop(U, mo * psi_o, bc_t), kappa, mu, C)
    w = apply_A_inv(mo * hop(U, me * u, bc_t), kappa, mu, C)
    return mo * psi_o - kappa ** 2 * w


def Mhat_dag(U, psi_o, kappa, mu, bc_t, dims, C=None):
    """Adjoint of ``Mhat``: 1 - kappa^2 H_eo^dag A_e^-dag H_oe^dag A_o^-dag.

    (H_eo)^dag = P_o H^dag P_e and (H_oe)^dag = P_e H^dag P_o, with P_p the
    parity projectors; A^-dag = (1 - 2 i kappa mu gamma_5)^-1 = A(-mu)^-1 (also with a
    hermitian clover term).
    """
    me, mo = parity_mask(dims, 0), parity_mask(dims, 1)
    v = apply_A_inv(mo * psi_o, kappa, -mu, C)
    u = apply_A_inv(me * hop(U, v, bc_t, dagger=True), kappa, -mu, C)
    w = mo * hop(U, me * u, bc_t, dagger=True)
    return mo * psi_o - kappa ** 2 * w


def schur_rhs(U, eta, kappa, mu, bc_t, dims, C=None):
    """bhat = A_o^-1 (eta_o + kappa H_oe A_e^-1 eta_e), an odd-site field."""
    me, mo = parity_mask(dims, 0), parity_mask(dims, 1)
    ue = apply_A_inv(me * eta, kappa, mu, C)
    return apply_A_inv(mo * eta + kappa * mo * hop(U, ue, bc_t), kappa, mu, C)


def reconstruct_even(U, eta, s_o, kappa, mu, bc_t, dims, C=None):
    """Full solution from the odd half: s_e = A_e^-1 (eta_e + kappa H_eo s_o)."""
    me, mo = parity_mask(dims, 0), parity_mask(dims, 1)
    s_e = apply_A_inv(me * eta + kappa * me * hop(U, mo * s_o, bc_t), kappa, mu, C)
    return s_e + mo * s_o


# ---------------------------------------------------------------------------
# dense matrices (tiny lattices only)
# ---------------------------------------------------------------------------

def dense(op, dims, batch=64):
    """Dense matrix of a linear map on full-lattice spinors, index (site, spin, colour)."""
    X, Y, Z, T = dims
    n = X * Y * Z * T * 12
    mat = np.empty((n, n), dtype=complex)
    for c0 in range(0, n, batch):
        nb = min(batch, n - c0)
        e = np.zeros((nb, n), dtype=complex)
        e[np.arange(nb), c0 + np.arange(nb)] = 1
        cols = op(e.reshape((nb, T, Z, Y, X, 4, 3)))
        mat[:, c0:c0 + nb] = cols.reshape(nb, n).T
    return mat


def dense_M(U, kappa, mu, bc_t, dims, C=None):
    return dense(lambda p: apply_M(U, p, kappa, mu, bc_t, C), dims)
