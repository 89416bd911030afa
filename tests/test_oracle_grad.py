"""Pins of the oracle's adjoint-solve gradients by central finite differences (CPU only)."""
import numpy as np
import pytest

import synth
from oracle import dirac, grad, loops


@pytest.mark.parametrize("p2max,nops", [(1, 5), (0, 1)])
def test_vjp_matches_finite_differences(p2max, nops):
    dims = (4, 2, 2, 4)
    X, Y, Z, T = dims
    kappa, mu, bc = 0.15, 0.07, -1
    U = synth.random_gauge(dims, 17, 0.4)
    etas = synth.random_spinor(dims, 5, nrhs=2)
    np_ = len(loops.momenta(p2max, dims))
    rng = np.random.default_rng(3)
    g = rng.standard_normal((2, nops, 16, T, np_)) + 1j * rng.standard_normal((2, nops, 16, T, np_))
    dense = {}

    def solve(eta, m):
        if m not in dense:
            dense[m] = np.linalg.inv(dirac.dense_M(U, kappa, m, bc, dims))
        return (dense[m] @ eta.reshape(-1)).reshape(eta.shape)

    gr, dmu = grad.vjp(U, etas, g, kappa, mu, bc, dims, p2max, tol=1e-13,
                       sols=[solve(e, mu) for e in etas])
    h = 1e-5
    for (r, idx) in [(0, (0, 0, 0, 0, 0, 0)), (1, (3, 1, 0, 2, 3, 1)), (0, (2, 0, 1, 3, 2, 2))]:
        e_p, e_m = etas.copy(), etas.copy()
        e_p[r][idx] += h
        e_m[r][idx] -= h
        d_re = (grad.loss(U, e_p, g, kappa, mu, bc, dims, p2max, solve)
                - grad.loss(U, e_m, g, kappa, mu, bc, dims, p2max, solve)) / (2 * h)
        e_p, e_m = etas.copy(), etas.copy()
        e_p[r][idx] += 1j * h
        e_m[r][idx] -= 1j * h
        d_im = (grad.loss(U, e_p, g, kappa, mu, bc, dims, p2max, solve)
                - grad.loss(U, e_m, g, kappa, mu, bc, dims, p2max, solve)) / (2 * h)
        want = d_re + 1j * d_im                    # dF/dRe eta + i dF/dIm eta
        got = gr[r][idx]
        assert abs(got - want) < 1e-6 * max(abs(want), 1e-3), (r, idx, got, want)
    fp = grad.loss(U, etas, g, kappa, mu + h, bc, dims, p2max, solve)
    fm = grad.loss(U, etas, g, kappa, mu - h, bc, dims, p2max, solve)
    want_mu = (fp - fm) / (2 * h)
    assert abs(dmu - want_mu) < 1e-6 * abs(want_mu), (dmu, want_mu)
