"""GPU parity of the backward pass (adjoint solves) against the oracle and
against central finite differences of the GPU forward pass."""
import ctypes
import sys

import numpy as np
import pytest

import paper_1401_6750_amd as dl
import synth
from oracle import grad, loops, noise
from tests.gpu_util import dev, host, make_lattice, rel, torch, zeros_dev

pytestmark = pytest.mark.gpu


def log(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def ctx():
    t = torch()
    assert t.cuda.is_available()
    c = dl.dl_create(0, t.cuda.current_stream().cuda_stream)
    yield c
    dl.dl_destroy(c)


def _backward(ctx, lat, etas_dev, g, p2max, ops, tier, tol, sol=None):
    acc = dl.dl_accum_create(lat.h, ops)
    job = dl.make_job(lat.h, noise=dl.DL_NOISE_USER, tier=tier, nsrc=etas_dev.shape[0], tol=tol, maxiter=5000,
                      src_in=etas_dev, sol_out=sol, accum=acc)
    ge = zeros_dev(etas_dev.shape)
    gmu = ctypes.c_double()
    gh = np.ascontiguousarray(g)
    rc = dl.lib().dl_loops_backward(ctx, ctypes.byref(job), p2max, gh.ctypes.data, ge.data_ptr(),
                                    ctypes.addressof(gmu))
    assert rc == 0, dl.dl_last_error()
    torch().cuda.synchronize()
    dl.dl_accum_destroy(acc)
    return host(ge), gmu.value


@pytest.mark.parametrize("ops,p2max", [(dl.DL_OPS_LOCAL | dl.DL_OPS_DERIV, 1), (dl.DL_OPS_LOCAL, 2)])
def test_backward_matches_oracle(ctx, ops, p2max):
    dims = (4, 4, 4, 4)
    lat = make_lattice(ctx, dims, 77, 0.3, 0.16, 0.02)
    etas = synth.random_spinor(dims, 7, nrhs=3)
    nops = 5 if ops & dl.DL_OPS_DERIV else 1
    np_ = len(loops.momenta(p2max, dims))
    rng = np.random.default_rng(11)
    g = rng.standard_normal((2, nops, 16, dims[3], np_)) + 1j * rng.standard_normal((2, nops, 16, dims[3], np_))
    ge, gmu = _backward(ctx, lat, dev(etas), g, p2max, ops, dl.DL_TIER_FP64, 1e-12)
    want, dmu = grad.vjp(lat.U, etas, g, lat.kappa, lat.mu, lat.bc, dims, p2max, tol=1e-12)
    log("backward vs oracle: grad_eta rel", rel(ge, want), "dmu", gmu, dmu)
    assert rel(ge, want) < 1e-9
    assert abs(gmu - dmu) < 1e-9 * abs(dmu)
    # with checkpointed solutions from a forward solve
    sol = zeros_dev(etas.shape)
    job = dl.make_job(lat.h, noise=dl.DL_NOISE_USER, tier=dl.DL_TIER_FP64, nsrc=3, tol=1e-12, maxiter=5000,
                      src_in=dev(etas), sol_out=sol)
    dl.dl_solve_batch(ctx, job)
    ge2, gmu2 = _backward(ctx, lat, dev(etas), g, p2max, ops, dl.DL_TIER_FP64, 1e-12, sol=sol)
    assert rel(ge2, ge) < 1e-10 and abs(gmu2 - gmu) < 1e-10 * abs(gmu)
    # the FP32 tier (adjoint solves with FP64 reliable updates)
    ge3, gmu3 = _backward(ctx, lat, dev(etas), g, p2max, ops, dl.DL_TIER_HP_FP32, 1e-9, sol=sol)
    log("HP tier: grad_eta rel", rel(ge3, want), "dmu rel", abs(gmu3 - dmu) / abs(dmu))
    assert rel(ge3, want) < 1e-6 and abs(gmu3 - dmu) < 1e-6 * abs(dmu)
    lat.close()


def test_autograd_function_against_finite_differences(ctx):
    """DiscLoops: mu.grad against central differences in mu (h = 1e-5, FP64) and
    eta.grad against a directional central difference, both of the GPU forward."""
    t = torch()
    dims = (4, 4, 4, 8)
    lat = make_lattice(ctx, dims, 1405, 0.2, 0.1615, 0.004)
    nsrc, p2max, ops = 4, 1, dl.DL_OPS_LOCAL | dl.DL_OPS_DERIV
    etas = np.stack([noise.source(dims, 6755, r, noise.Z2) for r in range(nsrc)])
    np_ = len(loops.momenta(p2max, dims))
    rng = np.random.default_rng(5)
    gw = dev(rng.standard_normal((2, 5, 16, dims[3], np_)) + 1j * rng.standard_normal((2, 5, 16, dims[3], np_)))
    F_of = lambda L: (L * gw.conj()).real.sum()
    eta = dev(etas).requires_grad_(True)
    mu = t.tensor(lat.mu, dtype=t.float64, requires_grad=True)
    args = (ctx, lat.h, lat.kappa, p2max, ops, dl.DL_TIER_FP64, 1e-12)
    F = F_of(dl.DiscLoops.apply(eta, mu, *args))
    F.backward()
    h = 1e-5
    with t.no_grad():
        fp = F_of(dl.DiscLoops.apply(dev(etas), t.tensor(lat.mu + h, dtype=t.float64), *args)).item()
        fm = F_of(dl.DiscLoops.apply(dev(etas), t.tensor(lat.mu - h, dtype=t.float64), *args)).item()
        fd_mu = (fp - fm) / (2 * h)
        d = dev(synth.random_spinor(dims, 9, nrhs=nsrc))
        fp = F_of(dl.DiscLoops.apply(dev(etas) + h * d, t.tensor(lat.mu, dtype=t.float64), *args)).item()
        fm = F_of(dl.DiscLoops.apply(dev(etas) - h * d, t.tensor(lat.mu, dtype=t.float64), *args)).item()
        fd_eta = (fp - fm) / (2 * h)
    dir_grad = float((eta.grad.conj() * d).real.sum())
    log("mu.grad", mu.grad.item(), "fd", fd_mu, "| eta dir", dir_grad, "fd", fd_eta)
    assert abs(mu.grad.item() - fd_mu) < 1e-6 * abs(fd_mu)
    assert abs(dir_grad - fd_eta) < 1e-6 * abs(fd_eta)
    lat.close()


def test_autograd_double_backward_and_local_only(ctx):
    """retain_graph: a second backward through the same graph gives the same gradients (the
    forward frees its accumulator at once; the backward needs only the insertion set), also
    for a local-only insertion set, whose gradient has one op."""
    t = torch()
    dims = (4, 4, 4, 4)
    lat = make_lattice(ctx, dims, 1408, 0.3, 0.16, 0.02)
    for ops in (dl.DL_OPS_LOCAL | dl.DL_OPS_DERIV, dl.DL_OPS_LOCAL):
        nops = 5 if ops & dl.DL_OPS_DERIV else 1
        etas = np.stack([noise.source(dims, 6756, r, noise.Z2) for r in range(2)])
        np_ = len(loops.momenta(1, dims))
        rng = np.random.default_rng(6)
        gw = dev(rng.standard_normal((2, nops, 16, dims[3], np_)) + 1j * rng.standard_normal((2, nops, 16, dims[3], np_)))
        eta = dev(etas).requires_grad_(True)
        mu = t.tensor(lat.mu, dtype=t.float64, requires_grad=True)
        L = dl.DiscLoops.apply(eta, mu, ctx, lat.h, lat.kappa, 1, ops, dl.DL_TIER_FP64, 1e-12)
        assert L.shape == (2, nops, 16, dims[3], np_)
        F = (L * gw.conj()).real.sum()
        g1 = t.autograd.grad(F, (eta, mu), retain_graph=True)
        g2 = t.autograd.grad(F, (eta, mu))
        assert t.equal(g1[0], g2[0]) and t.equal(g1[1], g2[1])
        want, dmu = grad.vjp(lat.U, etas, host(gw), lat.kappa, lat.mu, lat.bc, dims, 1, tol=1e-12)
        assert rel(host(g1[0]), want) < 1e-9 and abs(g1[1].item() - dmu) < 1e-9 * abs(dmu)
    lat.close()
