"""Pins of the oracle's one-end-trick loops, projection and TSM (CPU only)."""
import numpy as np
import pytest

import synth
from oracle import dirac, loops, noise, solver


def rel(a, b):
    return np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300)


def _complete_basis_loops(U, kappa, mu, bc, dims, deriv=True, batch=256):
    """sum_k over unit-vector sources e_k of the per-source site loops (exact solves)."""
    X, Y, Z, T = dims
    n = X * Y * Z * T * 12
    minv = np.linalg.inv(dirac.dense_M(U, kappa, mu, bc, dims))
    tot = 0
    for c0 in range(0, n, batch):
        cols = minv[:, c0:c0 + batch].T.reshape((-1, T, Z, Y, X, 4, 3))
        xi_t3, xi_1 = loops.xi_fields(U, cols, kappa, bc)
        a = loops.site_loops(U, xi_t3, cols, bc, deriv)        # [nops, 16, B, T, Z, Y, X]
        b = loops.site_loops(U, xi_1, cols, bc, deriv)
        tot = tot + np.stack([a, b]).sum(axis=3)
    return loops.apply_prefactors(tot, kappa, mu)


def test_one_end_trick_complete_basis_equals_exact():
    """Unit-vector sources make the estimator exact: both flavour structures,
    local and derivative insertions, prefactors included."""
    dims = (4, 2, 4, 2)
    U = synth.random_gauge(dims, 61, 0.4)
    kappa, mu, bc = 0.15, 0.06, -1
    est = _complete_basis_loops(U, kappa, mu, bc, dims)
    exact = loops.exact_site_loops(U, kappa, mu, bc, dims)
    assert est.shape == exact.shape == (2, 5, 16, 2, 4, 2, 4)
    assert np.abs(est - exact).max() < 1e-13 * np.abs(exact).max()


def _free_sums(dims, kappa, mu, bc):
    X, Y, Z, T = dims
    shift = 0.5 if bc == -1 else 0.0
    ps = [2 * np.pi * np.arange(L) / L for L in (X, Y, Z)] + [2 * np.pi * (np.arange(T) + shift) / T]
    P = np.meshgrid(*ps, indexing="ij")
    a = 1 - 2 * kappa * sum(np.cos(p) for p in P)
    b = [2 * kappa * np.sin(p) for p in P]
    c = 2 * kappa * mu
    D = a ** 2 + sum(bb ** 2 for bb in b) + c ** 2
    V = X * Y * Z * T
    return P, a, D, V, c


def test_free_field_closed_forms():
    """U = 1: tr D^-1(x,x) and the derivative loop have closed forms in momentum space.

    M(p)^-1 = (a - i sum gamma_mu b_mu - i c gamma_5) / D, a = 1 - 2 kappa sum cos p,
    b_mu = 2 kappa sin p_mu, c = 2 kappa mu, D = a^2 + b^2 + c^2.
    """
    dims = (4, 4, 2, 4)
    kappa, mu, bc = 0.12, 0.2, -1
    U = synth.unit_gauge(dims)
    ex = loops.exact_site_loops(U, kappa, mu, bc, dims)
    P, a, D, V, c = _free_sums(dims, kappa, mu, bc)
    pref = 2 * kappa / V
    want_t3_g5 = pref * np.sum(-24j * c / D)            # tr g5 (D_u^-1 - D_d^-1)
    want_1_id = pref * np.sum(24 * a / D)               # tr (D_u^-1 + D_d^-1)
    assert np.allclose(ex[0, 0, 15], want_t3_g5, atol=1e-13)
    assert np.allclose(ex[1, 0, 0], want_1_id, atol=1e-13)
    # everything else local vanishes (odd in p or traceless)
    mask = np.ones((2, 16), bool)
    mask[0, 15] = mask[1, 0] = False
    assert np.abs(ex[:, 0][mask]).max() < 1e-13
    # derivative insertion Gamma = gamma_nu (bit nu) along nu, no tau3:
    for nu in range(4):
        want = pref * np.sum(2 * 12 * 2 * kappa * np.sin(P[nu]) ** 2 / D)
        assert np.allclose(ex[1, 1 + nu, 1 << nu], want, atol=1e-13)
        # the tau3 combination of the same insertion cancels
        assert np.abs(ex[0, 1 + nu, 1 << nu]).max() < 1e-13


def test_gauge_invariance_of_source_loops():
    """Transform U and the source together (eta -> Omega eta): per-source loops are invariant."""
    dims = (4, 4, 4, 4)
    U = synth.random_gauge(dims, 71, 0.3)
    om = synth.random_su3_field(dims, 72)
    Ug = np.empty_like(U)
    for m in range(4):
        om_fwd = np.roll(om, -1, axis=3 - m)
        Ug[..., m, :, :] = om @ U[..., m, :, :] @ np.swapaxes(om_fwd.conj(), -1, -2)
    kappa, mu, bc = 0.16, 0.01, -1
    eta = noise.source(dims, 5, 0, noise.Z4)
    s, _ = solver.cgnr_eo(U, eta, kappa, mu, bc, dims, tol=1e-13)
    sg, _ = solver.cgnr_eo(Ug, dirac.color_mul(om, eta), kappa, mu, bc, dims, tol=1e-13)
    la = loops.source_loops(U, s, kappa, bc, 3, dims)
    lb = loops.source_loops(Ug, sg, kappa, bc, 3, dims)
    assert rel(lb, la) < 1e-10


def test_projection_against_fft_and_translation_phase():
    dims = (4, 6, 8, 4)
    X, Y, Z, T = dims
    rng = np.random.default_rng(1)
    f = rng.standard_normal((3, T, Z, Y, X)) + 1j * rng.standard_normal((3, T, Z, Y, X))
    moms = loops.momenta(5, dims)
    got = loops.project(f, moms, dims)
    ff = np.fft.fftn(f, axes=(-3, -2, -1))            # [.., T, kz, ky, kx], e^{-2 pi i k x / L}
    for i, (nx, ny, nz) in enumerate(moms):
        assert np.allclose(got[..., i], ff[..., nz % Z, ny % Y, nx % X], atol=1e-12)
    # n = 0 is the plain spatial sum
    assert moms[0].tolist() == [0, 0, 0]
    assert np.allclose(got[..., 0], f.sum(axis=(-3, -2, -1)))
    # f'(x) = f(x + a)  =>  L'(n) = exp(+2 pi i n.a / L) L(n)
    a = (1, 2, 3)
    fs = np.roll(f, shift=(-a[2], -a[1], -a[0]), axis=(-3, -2, -1))
    gs = loops.project(fs, moms, dims)
    ph = np.exp(2j * np.pi * (moms[:, 0] * a[0] / X + moms[:, 1] * a[1] / Y + moms[:, 2] * a[2] / Z))
    assert np.allclose(gs, got * ph, atol=1e-12)


def test_translated_configuration_gives_phase_on_loops():
    """Shift U and eta by a spatial vector a: per-source loops pick up exp(+2 pi i n.a/L)."""
    dims = (4, 4, 4, 4)
    U = synth.random_gauge(dims, 81, 0.3)
    eta = noise.source(dims, 9, 2, noise.Z2)
    kappa, mu, bc = 0.16, 0.02, -1
    a = (1, 3, 2)          # x, y, z shift
    sh = (-a[2], -a[1], -a[0])
    Us = np.roll(U, shift=sh, axis=(1, 2, 3))
    etas = np.roll(eta, shift=sh, axis=(1, 2, 3))
    s, _ = solver.cgnr_eo(U, eta, kappa, mu, bc, dims, tol=1e-13)
    ss, _ = solver.cgnr_eo(Us, etas, kappa, mu, bc, dims, tol=1e-13)
    moms = loops.momenta(3, dims)
    la = loops.source_loops(U, s, kappa, bc, 3, dims)
    lb = loops.source_loops(Us, ss, kappa, bc, 3, dims)
    ph = np.exp(2j * np.pi * (moms[:, 0] * a[0] + moms[:, 1] * a[1] + moms[:, 2] * a[2]) / 4)
    assert rel(lb, la * ph) < 1e-10


def test_momentum_list_counts_and_order():
    big = (16, 16, 16, 32)
    assert [len(loops.momenta(c, big)) for c in (0, 1, 2, 3, 4, 9)] == [1, 7, 19, 27, 33, 123]
    m = loops.momenta(9, big)
    n2 = (m ** 2).sum(axis=1)
    keys = list(zip(n2, m[:, 0], m[:, 1], m[:, 2]))
    assert keys == sorted(keys)
    # brute force over the whole box
    cnt = sum(1 for x in range(-7, 9) for y in range(-7, 9) for z in range(-7, 9)
              if x * x + y * y + z * z <= 9)
    assert cnt == 123
    # a 4^3 box cannot hold both +2 and -2: components live in (-L/2, L/2]
    small = loops.momenta(4, (4, 4, 4, 4))
    assert len(small) == 30 and [-2, 0, 0] not in small.tolist()
    assert len(loops.momenta(3, (4, 4, 4, 4))) == 27


def test_insertion_count_is_160():
    dims = (2, 2, 2, 4)
    U = synth.random_gauge(dims, 3, 0.3)
    s = synth.random_spinor(dims, 3)
    l = loops.source_loops(U, s, 0.15, -1, 0, dims)
    assert l.shape[:3] == (2, 5, 16) and np.prod(l.shape[:3]) == 160


def test_tsm_identity():
    """If the correction uses the same sources as the LP tier, TSM equals the HP estimator."""
    rng = np.random.default_rng(2)
    hp = rng.standard_normal((7, 2, 3)) + 1j * rng.standard_normal((7, 2, 3))
    lp = hp + 0.01 * rng.standard_normal((7, 2, 3))
    got = loops.tsm_combine(lp.sum(0), 7, hp.sum(0), lp.sum(0), 7, 0.15, 0.01)
    want = loops.estimate(hp, 0.15, 0.01)
    assert np.allclose(got, want, rtol=1e-14, atol=1e-15)
    # no LP tier: plain estimator
    got2 = loops.tsm_combine(0, 0, hp.sum(0), 0, 7, 0.15, 0.01)
    assert np.allclose(got2, want)


@pytest.mark.slow
def test_tsm_is_unbiased():
    """Truncated LP solves (rho = 1e-2) + HP corrections: mean within 4 sigma of the exact trace."""
    dims = (2, 2, 2, 4)
    kappa, mu, bc = 0.16, 0.05, -1
    U = synth.random_gauge(dims, 91, 0.3)
    exact = loops.exact_site_loops(U, kappa, mu, bc, dims, deriv=False).sum(axis=(-4, -3, -2, -1))
    n_lp, n_hp = 600, 60
    per_lp, per_diff = [], []
    for r in range(n_lp + n_hp):
        eta = noise.source(dims, 7, r, noise.Z2)
        s_lp, _ = solver.cgnr_eo(U, eta, kappa, mu, bc, dims, tol=1e-2)
        l_lp = loops.source_loops(U, s_lp, kappa, bc, 0, dims, deriv=False)[..., 0].sum(-1)
        if r < n_lp:
            per_lp.append(l_lp)
        else:
            s_hp, _ = solver.cgnr_eo(U, eta, kappa, mu, bc, dims, tol=1e-10)
            l_hp = loops.source_loops(U, s_hp, kappa, bc, 0, dims, deriv=False)[..., 0].sum(-1)
            per_diff.append(l_hp - l_lp)
    per_lp, per_diff = np.array(per_lp), np.array(per_diff)
    est = loops.tsm_combine(per_lp.sum(0), n_lp, per_diff.sum(0), 0, n_hp, kappa, mu)
    pf = loops.prefactors(kappa, mu).reshape(2, 1, 1)
    var = (np.var(per_lp, axis=0, ddof=1) / n_lp + np.var(per_diff, axis=0, ddof=1) / n_hp)
    sigma = np.abs(pf) * np.sqrt(var)
    # compare only components with a non-negligible spread
    ok = sigma > 1e-12
    z = np.abs(est - exact)[ok] / sigma[ok]
    assert z.max() < 4.5, z.max()
    # the LP-only estimate is biased by much more than the TSM one for some component
    lp_only = loops.estimate(per_lp, kappa, mu)
    assert np.abs(lp_only - exact).max() > np.abs(est - exact).max()


def test_derivative_insertion_link_centred_form():
    """E(x) = F(x) + F(x - nu) with the per-link F(x) = 1/4 [xi(x)^dag Gamma T_phi(x)
    - T_xi(x)^dag Gamma phi(x)], T_psi(x) = U_nu(x) psi(x + nu): the form in which the
    GPU accumulates the one-derivative insertions before projecting (the backward half of
    D at x + nu repeats the forward half at x).  Random fields, antiperiodic in t."""
    dims = (4, 2, 4, 6)
    X, Y, Z, T = dims
    U = synth.random_gauge(dims, 77, 0.5)
    rng = np.random.default_rng(5)
    shape = (T, Z, Y, X, 4, 3)
    xi = rng.normal(size=shape) + 1j * rng.normal(size=shape)
    phi = rng.normal(size=shape) + 1j * rng.normal(size=shape)
    bc = -1
    site = loops.site_loops(U, xi, phi, bc, deriv=True)            # [5, 16, T, Z, Y, X]
    for nu in range(4):
        ax = dirac.SPINOR_AXIS[nu]
        t_phi = dirac.color_mul(U[..., nu, :, :], dirac.shift_forward(phi, nu, bc, ax))
        t_xi = dirac.color_mul(U[..., nu, :, :], dirac.shift_forward(xi, nu, bc, ax))
        f = 0.25 * (loops.insert_gammas(loops.outer_product(xi, t_phi))
                    - loops.insert_gammas(loops.outer_product(t_xi, phi)))   # [16, T, Z, Y, X]
        lat_axis = 1 + (3 - nu)                                     # axes of f: n, t, z, y, x
        f_back = np.roll(f, 1, axis=lat_axis)                       # F(x - nu), no extra sign
        assert rel(f + f_back, site[1 + nu]) < 1e-13, nu
