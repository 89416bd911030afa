"""Pins of the oracle's hopping parameter expansion (CPU only).

* the exact low orders (free-field path sums) equal the truncated series built
  from the oracle's hopping term on a random gauge field, at sites whose hops
  cross the antiperiodic time boundary;
* a complete basis of unit-vector sources makes the HPE estimator plus its exact
  part equal the exact no-tau_3 loops from dense inverses, for every order,
  local and one-derivative insertions;
* the expansion lowers the source-to-source variance of the estimator.
"""
import numpy as np
import pytest
import scipy.linalg

import synth
from oracle import dirac, hpe, loops, noise, solver

DIMS = (4, 4, 4, 4)
KAPPA, MU, BC = 0.15, 0.06, -1


def neighbours(dims, site):
    """[(nu, +1 site, sign), (nu, -1 site, sign)] of site (t, z, y, x); sign = boundary factor."""
    X, Y, Z, T = dims
    ext = [X, Y, Z, T]
    out = []
    for nu in range(4):
        for step in (+1, -1):
            v = [site[3], site[2], site[1], site[0]]
            v[nu] += step
            sign = BC if (nu == 3 and not 0 <= v[3] < T) else 1.0
            v[nu] %= ext[nu]
            out.append((nu, step, (v[3], v[2], v[1], v[0]), sign))
    return out


def unit_fields(dims, site):
    """The 12 unit spinors at one site: [12, T, Z, Y, X, 4, 3]."""
    X, Y, Z, T = dims
    e = np.zeros((12, T, Z, Y, X, 4, 3), dtype=complex)
    for k in range(12):
        e[(k,) + tuple(site) + (k // 3, k % 3)] = 1
    return e


def block(cols, row_site):
    """12x12 block G(row_site, col_site) from the 12 columns of col_site."""
    return cols[(slice(None),) + tuple(row_site)].reshape(12, 12).T


def trace_loops(U, dims, G, site):
    """Per-site loops from a matrix given by G(row_site, col_site) -> 12x12, in the
    trace form of the insertions: [5, 16]."""
    Gm = dirac.GAMMA_BASIS
    out = np.zeros((5, 16), dtype=complex)
    g = G(site, site).reshape(4, 3, 4, 3)
    out[0] = np.einsum("nab,bcac->n", Gm, g)
    nb = neighbours(dims, site)
    for nu in range(4):
        (_, _, sp, bp), (_, _, sm, bm) = nb[2 * nu], nb[2 * nu + 1]
        u_here = U[tuple(site)][nu]
        u_back = U[tuple(sm)][nu]

        def tr(W, blk):
            return np.einsum("nab,ij,bjai->n", Gm, W, blk.reshape(4, 3, 4, 3))

        t1 = tr(u_here, G(sp, site))
        t2 = tr(u_back.conj().T, G(sm, site))
        t3 = tr(u_here.conj().T, G(site, sp))
        t4 = tr(u_back, G(site, sm))
        out[1 + nu] = 0.25 * (bp * t1 - bm * t2 - bp * t3 + bm * t4)
    return out


SITES = [(0, 1, 2, 3), (3, 0, 3, 0), (2, 2, 1, 1)]   # (t, z, y, x); t = 0 and T-1 cross the boundary


def test_exact_low_orders_equal_truncated_series():
    U = synth.random_gauge(DIMS, 71, 0.5)
    per_flavour = {}
    for mu_f in (MU, -MU):
        binv = 1.0 / dirac.twist_diag(KAPPA, mu_f)
        for site in SITES:
            cols = {}
            for s in [site] + [nb[2] for nb in neighbours(DIMS, site)]:
                v = dirac.apply_spin_diag(binv, unit_fields(DIMS, s))
                terms = [v]
                for _ in range(3):
                    terms.append(KAPPA * dirac.apply_spin_diag(binv, dirac.hop(U, terms[-1], BC)))
                cols[s] = np.cumsum(np.stack(terms), axis=0)      # [k] = sum_{j<=k} T_j
            for n in range(1, hpe.MAX_ORDER + 1):
                nd = hpe.deriv_order(n)
                loc = trace_loops(U, DIMS, lambda r, c: block(cols[c][n - 1], r), site)[0]
                der = trace_loops(U, DIMS, lambda r, c: block(cols[c][nd - 1], r), site)[1:]
                per_flavour[(mu_f, site, n)] = np.concatenate([loc[None], der])
    for site in SITES:
        for n in range(1, hpe.MAX_ORDER + 1):
            want = 0.5 * (per_flavour[(MU, site, n)] + per_flavour[(-MU, site, n)])
            got = hpe.hpe_exact(KAPPA, MU, n)
            assert np.abs(got - want).max() < 1e-14 * np.abs(want).max(), (site, n)


def test_exact_orders_are_nonzero_where_expected():
    """k = 0 gives the identity insertion, k = 2 adds the gamma_5 term, derivative
    insertions start at order 1 with the gamma_nu term (and vanish for n = 1)."""
    e1, e2, e3 = (hpe.hpe_exact(KAPPA, MU, n) for n in (1, 2, 3))
    assert np.allclose(e1[1:], 0) and np.allclose(e1[0], e2[0])
    assert abs(e1[0, 0]) > 1 and np.allclose(e1[0, 1:], 0)
    assert abs(e3[0, 15] - e2[0, 15]) > 1e-4 or abs(e3[0, 0] - e2[0, 0]) > 1e-4
    for nu in range(4):
        assert abs(e2[1 + nu, 1 << nu]) > 0.1       # Gamma_n = gamma_nu


@pytest.mark.parametrize("n", [0, 1, 2, 3, 4])
def test_complete_basis_equals_exact(n, _dense_case):
    U, lu, exact = _dense_case
    for site in SITES:
        tot = 0
        for s in [site] + [nb[2] for nb in neighbours(DIMS, site)]:
            e = unit_fields(DIMS, s)
            sol = scipy.linalg.lu_solve(lu, e.reshape(12, -1).T).T.reshape(e.shape)
            vals = hpe.hpe_site_loops(U, e, sol, KAPPA, MU, BC, n)      # [5, 16, 12, T, Z, Y, X]
            tot = tot + vals[(slice(None), slice(None), slice(None)) + tuple(site)].sum(axis=2)
        est = 4 * KAPPA * (tot + hpe.hpe_exact(KAPPA, MU, n))
        want = exact[(1, slice(None), slice(None)) + tuple(site)]
        assert np.abs(est - want).max() < 1e-12 * np.abs(want).max(), (site, n)


@pytest.fixture(scope="module")
def _dense_case():
    U = synth.random_gauge(DIMS, 72, 0.5)
    lu = scipy.linalg.lu_factor(dirac.dense_M(U, KAPPA, MU, BC, DIMS))
    exact = loops.exact_site_loops(U, KAPPA, MU, BC, DIMS)
    return U, lu, exact


def test_projected_exact_part():
    p = hpe.hpe_exact_projected(KAPPA, MU, 4, 3, DIMS)
    ex = hpe.hpe_exact(KAPPA, MU, 4)
    assert p.shape == (5, 16, 4, 27)
    assert np.allclose(p[..., 0], 64 * ex[..., None]) and np.allclose(p[..., 1:], 0)


def test_expansion_lowers_the_variance():
    """Per-site variance over Z4 sources of the local and derivative no-tau_3 loops:
    the plain volume-source estimator (order 0) against orders 2 and 4, and the
    generalised one-end trick for reference."""
    dims = (4, 4, 4, 8)
    kappa, mu = 0.13, 0.05
    U = synth.random_gauge(dims, 73, 0.3)
    nsrc = 12
    vals = {n: [] for n in (0, 2, 4)}
    gen = []
    for r in range(nsrc):
        eta = noise.source(dims, 5, r, noise.Z4)
        s = solver.cgnr_eo(U, eta, kappa, mu, BC, dims, 1e-12)[0]
        for n in vals:
            vals[n].append(hpe.hpe_site_loops(U, eta, s, kappa, mu, BC, n))
        gen.append(loops.source_site_loops(U, s, kappa, BC)[loops.NOTAU3])
    var = {n: np.var(np.stack(v), axis=0) for n, v in vals.items()}     # [5, 16, sites]
    var["gen"] = np.var(np.stack(gen), axis=0)
    loc = {n: v[0].sum() for n, v in var.items()}
    der = {n: v[1:].sum() for n, v in var.items()}
    # measured: local 56e3 -> 23e3 -> 15e3 (one-end 133e3), derivative 67e3 -> 16e3 -> 12e3
    assert loc[2] < 0.6 * loc[0] and loc[4] < 0.8 * loc[2] and loc[4] < 0.25 * loc["gen"], loc
    assert der[2] < 0.5 * der[0] and der[4] < 0.8 * der[2] and der[4] < 0.25 * der["gen"], der
