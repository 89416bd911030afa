"""Pins of the oracle's clover term (oracle/clover.py), CPU only.

The clover variant of the operator is a reading of Section 2.4 (Wilson and clover
fermions); these tests fix it against things other than its own code: a closed form
on a constant abelian field, algebraic properties (hermiticity, chirality, traceless
spin structure, gauge covariance, gamma_5-hermiticity of M), dense solves and the
exact traces the one-end trick must reproduce.
"""
import numpy as np
import pytest

import synth
from oracle import clover, dirac, loops, solver


def rel(a, b):
    return np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300)


def flux_gauge(dims, n, mu, nu):
    """Constant abelian field in the (mu, nu) plane ('t Hooft flux): every plaquette
    U_mu(x) U_nu(x + mu) U_mu(x + nu)^dag U_nu(x)^dag equals diag(e^{iB}, e^{-iB}, 1),
    B = 2 pi n / (L_mu L_nu); every other link is 1."""
    X, Y, Z, T = dims
    L = (X, Y, Z, T)
    B = 2 * np.pi * n / (L[mu] * L[nu])
    U = np.zeros((T, Z, Y, X, 4, 3, 3), dtype=complex)
    U[...] = np.eye(3)

    def emb(phi):
        return np.diag([np.exp(1j * phi), np.exp(-1j * phi), 1.0])

    for t in range(T):
        for z in range(Z):
            for y in range(Y):
                for x in range(X):
                    c = (x, y, z, t)
                    U[t, z, y, x, nu] = emb(B * c[mu])
                    if c[mu] == L[mu] - 1:
                        U[t, z, y, x, mu] = emb(-B * L[mu] * c[nu])
    return U, B


S1 = np.array([[0, 1], [1, 0]], dtype=complex)
S2 = np.array([[0, -1j], [1j, 0]])
S3 = np.array([[1, 0], [0, -1]], dtype=complex)
Z2 = np.zeros((2, 2))
# sigma_{mu nu} = (i/2)[gamma_mu, gamma_nu] in the chiral basis, worked out by hand from
# gamma_k gamma_l = diag(s_k s_l, s_k s_l) and gamma_k gamma_4 = diag(-i s_k, i s_k)
SIGMA_BY_HAND = {(0, 1): -np.block([[S3, Z2], [Z2, S3]]), (0, 2): np.block([[S2, Z2], [Z2, S2]]),
                 (1, 2): -np.block([[S1, Z2], [Z2, S1]]), (0, 3): np.block([[S1, Z2], [Z2, -S1]]),
                 (1, 3): np.block([[S2, Z2], [Z2, -S2]]), (2, 3): np.block([[S3, Z2], [Z2, -S3]])}


@pytest.mark.parametrize("plane", sorted(SIGMA_BY_HAND))
def test_plaquette_orientation_and_flux_closed_form(plane):
    """On the flux field of one plane Fhat = i sin(B) diag(1, -1, 0) at every site and the
    other planes vanish, so C = i kappa c_sw sigma_{mu nu} (x) i sin(B) diag(1, -1, 0)."""
    mu, nu = plane
    dims = (4, 6, 2, 4)
    U, B = flux_gauge(dims, 1, mu, nu)
    p = clover.clover_leaves(U, mu, nu)
    want_leaf = 4 * np.diag([np.exp(1j * B), np.exp(-1j * B), 1.0])
    assert np.abs(p - want_leaf).max() < 1e-13
    f = clover.field_strength(U, mu, nu)
    assert np.abs(f - 1j * np.sin(B) * np.diag([1.0, -1.0, 0.0])).max() < 1e-13
    for other in SIGMA_BY_HAND:
        if other != plane:
            assert np.abs(clover.field_strength(U, *other)).max() < 1e-13
    assert np.abs(clover.sigma(mu, nu) - SIGMA_BY_HAND[plane]).max() < 1e-15
    kappa, csw = 0.13, 1.7
    C = clover.clover_term(U, kappa, csw)
    want = -kappa * csw * np.sin(B) * np.einsum("sr,ab->sarb", SIGMA_BY_HAND[plane], np.diag([1.0, -1, 0]))
    assert np.abs(C - want).max() < 1e-13


def test_clover_term_hermitian_chiral_traceless():
    dims = (4, 2, 2, 4)
    U = synth.random_gauge(dims, 71, 0.5)
    C = clover.clover_term(U, 0.14, 1.3)
    m = C.reshape(C.shape[:-4] + (12, 12))
    assert np.abs(m - np.swapaxes(m.conj(), -1, -2)).max() < 1e-14
    g5 = np.kron(np.diag(dirac.GAMMA5), np.ones(3))
    assert np.abs(m * g5[:, None] - m * g5[None, :]).max() < 1e-14      # commutes with gamma_5
    assert np.abs(np.einsum("...sasb->...ab", C)).max() < 1e-14          # spin-traceless
    assert np.abs(np.einsum("...sasa->...", C)).max() < 1e-14
    assert np.abs(C).max() > 0.01
    # no field strength, no clover term
    assert np.abs(clover.clover_term(synth.unit_gauge(dims), 0.14, 1.3)).max() == 0


def test_clover_term_gauge_covariant():
    dims = (2, 4, 2, 4)
    U = synth.random_gauge(dims, 72, 0.4)
    om = synth.random_su3_field(dims, 73)
    Ug = U.copy()
    for mu in range(4):
        om_fwd = np.roll(om, -1, axis=3 - mu)    # Omega(x + mu); om is [T, Z, Y, X, 3, 3]
        Ug[..., mu, :, :] = om @ U[..., mu, :, :] @ np.swapaxes(om_fwd.conj(), -1, -2)
    C = clover.clover_term(U, 0.12, 1.1)
    Cg = clover.clover_term(Ug, 0.12, 1.1)
    want = np.einsum("...ij,...sjrk,...lk->...sirl", om, C, om.conj())
    assert rel(Cg, want) < 1e-13


def test_clover_operator_gamma5_hermiticity_and_dense_solve():
    """M(mu)^dag = gamma_5 M(-mu) gamma_5 with the clover term (dense); even-odd CGNR with
    the site matrices A = 1 + C + 2 i kappa mu gamma_5 reproduces the dense solve."""
    dims = (2, 2, 2, 4)
    U = synth.random_gauge(dims, 74, 0.6)
    kappa, mu, csw, bc = 0.15, 0.05, 1.5, -1
    C = clover.clover_term(U, kappa, csw)
    m = dirac.dense_M(U, kappa, mu, bc, dims, C)
    mm = dirac.dense_M(U, kappa, -mu, bc, dims, C)
    g5 = np.kron(np.eye(32), np.kron(dirac.GAMMA5, np.eye(3)))
    assert np.abs(m.conj().T - g5 @ mm @ g5).max() < 1e-14
    assert np.abs(m - dirac.dense_M(U, kappa, mu, bc, dims)).max() > 1e-3       # the term is there
    eta = synth.random_spinor(dims, 75)
    exact = np.linalg.solve(m, eta.reshape(-1)).reshape(eta.shape)
    s, info = solver.cgnr_eo(U, eta, kappa, mu, bc, dims, 1e-13, C=C)
    assert info["converged"] and rel(s, exact) < 1e-11
    assert solver.true_residual(U, eta, s, kappa, mu, bc, C) < 1e-12
    # Mhat_dag is the adjoint of Mhat with the site matrices
    mo = dirac.parity_mask(dims, 1)
    a, b = mo * synth.random_spinor(dims, 76), mo * synth.random_spinor(dims, 77)
    lhs = np.vdot(a, dirac.Mhat(U, b, kappa, mu, bc, dims, C))
    rhs = np.vdot(dirac.Mhat_dag(U, a, kappa, mu, bc, dims, C), b)
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)


def test_clover_one_end_trick_complete_basis_equals_exact():
    """Unit-vector sources with the clover term (xi = M_0 s, M_0 = 1 + C - kappa H) give the
    exact tr Gamma (D_u^-1 -+ D_d^-1) from dense inverses, local and derivative."""
    dims = (2, 2, 2, 4)
    U = synth.random_gauge(dims, 78, 0.5)
    kappa, mu, csw, bc = 0.14, 0.07, 1.4, -1
    C = clover.clover_term(U, kappa, csw)
    X, Y, Z, T = dims
    n = X * Y * Z * T * 12
    minv = np.linalg.inv(dirac.dense_M(U, kappa, mu, bc, dims, C))
    cols = minv.T.reshape((n, T, Z, Y, X, 4, 3))
    xi_t3, xi_1 = loops.xi_fields(U, cols, kappa, bc, C)
    est = np.stack([loops.site_loops(U, xi_t3, cols, bc), loops.site_loops(U, xi_1, cols, bc)]).sum(axis=3)
    est = loops.apply_prefactors(est, kappa, mu)
    exact = loops.exact_site_loops(U, kappa, mu, bc, dims, C=C)
    assert np.abs(est - exact).max() < 1e-12 * np.abs(exact).max()
    # and the clover term changes the loops (no-tau_3 scalar)
    plain = loops.exact_site_loops(U, kappa, mu, bc, dims, deriv=False)
    assert np.abs(plain[1, 0, 0] - exact[1, 0, 0]).max() > 1e-3 * np.abs(exact[1, 0, 0]).max()
