"""GPU parity of time-diluted sources against the FP64 oracle, through the C ABI.

FP64 solves of every component match the oracle's solves of the masked sources
(1e-10); one-end-trick loops (whole-vector contractions of every component) and
the hopping parameter expansion (single-time-slice contractions) match the
oracle's sums over components (1e-10), for D = 2, 3 and T, including the
component whose link-centred time derivative wraps around the lattice.
"""
import sys

import numpy as np
import pytest

import paper_1401_6750_amd as dl
from oracle import dilution, hpe, loops, noise, solver
from tests.gpu_util import dev, elementwise, host, make_lattice, rel, torch, zeros_dev

pytestmark = pytest.mark.gpu

DIMS = (6, 4, 6, 6)        # Vh = 432 (ragged tile tail), T = 6
KAPPA, MU = 0.15, 0.02


def log(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def ctx():
    t = torch()
    assert t.cuda.is_available(), "GPU tests need a GPU"
    c = dl.dl_create(0, t.cuda.current_stream().cuda_stream)
    yield c
    dl.dl_destroy(c)


@pytest.fixture(scope="module")
def lat(ctx):
    la = make_lattice(ctx, DIMS, 1409, 0.3, KAPPA, MU)
    yield la
    la.close()


def oracle_vector_sums(la, seed, rs, D, p2, n_hpe=0, kind=noise.Z4, tol=1e-11):
    """Sum over noise vectors of the loops dl_loops_sets reports (components summed)."""
    pf = loops.prefactors(la.kappa, la.mu)
    moms = loops.momenta(p2, la.dims)
    tot = 0
    for r in rs:
        etas = dilution.split(noise.source(la.dims, seed, r, kind), D)
        sols = [solver.cgnr_eo(la.U, e, la.kappa, la.mu, la.bc, la.dims, tol)[0] for e in etas]
        per = dilution.one_end_site_loops(la.U, sols, la.kappa, la.bc)
        if n_hpe:
            h = dilution.hpe_site_loops(la.U, etas, sols, la.kappa, la.mu, la.bc, n_hpe)
            per = np.stack([per[loops.TAU3], h])
        site = loops.project(per, moms, la.dims)
        if n_hpe:
            site[1] = site[1] + hpe.hpe_exact_projected(la.kappa, la.mu, n_hpe, p2, la.dims)
        tot = tot + pf.reshape(2, 1, 1, 1, 1) * site
    return tot


def test_fp64_diluted_solutions_match_oracle(ctx, lat):
    seed, nsrc, D = 41, 2, 3
    sol = zeros_dev((nsrc * D,) + lat.field_shape)
    rc, stats = dl.dl_solve_batch(ctx, dl.make_job(lat.h, noise=dl.DL_NOISE_Z2, tier=dl.DL_TIER_FP64, seed=seed,
                                                   first_src=5, nsrc=nsrc, tol=1e-10, maxiter=1000, tdil=D,
                                                   rhs_block=4, report_true_resid=1, sol_out=sol))
    assert rc == dl.DL_OK and len(stats) == nsrc * D
    got = host(sol)
    for c in range(D):
        for k in range(nsrc):
            eta = dilution.split(noise.source(lat.dims, seed, 5 + k, noise.Z2), D)[c]
            s, info = solver.cgnr_eo(lat.U, eta, lat.kappa, lat.mu, lat.bc, lat.dims, 1e-10)
            e = c * nsrc + k                     # component-major
            assert stats[e].iters == info["iters"], (c, k)
            assert rel(got[e], s) < 1e-10, (c, k)
            assert 0 <= stats[e].true_resid < 1e-8


@pytest.mark.parametrize("D", [2, 3, 6])
def test_fp64_diluted_one_end_loops_match_oracle(ctx, lat, D):
    log("diluted one-end D", D)
    seed, nsrc, p2 = 42, 2, 2
    acc = dl.dl_accum_create(lat.h, dl.DL_OPS_LOCAL | dl.DL_OPS_DERIV)
    rc, _ = dl.dl_solve_batch(ctx, dl.make_job(lat.h, noise=dl.DL_NOISE_Z4, tier=dl.DL_TIER_FP64, seed=seed,
                                               nsrc=nsrc, tol=1e-11, maxiter=1000, tdil=D, accum=acc,
                                               accum_set=dl.DL_SET_LP))
    assert rc == dl.DL_OK
    assert dl.dl_accum_counts(acc) == [nsrc, 0, 0]
    npm = len(loops.momenta(p2, lat.dims))
    sets = np.zeros((3, 2, 5, 16, lat.dims[3], npm), dtype=np.complex128)
    dl.dl_loops_sets(ctx, acc, p2, sets, 0)
    want = oracle_vector_sums(lat, seed, range(nsrc), D, p2)
    log("  worst |d|/max|block|", elementwise(sets[dl.DL_SET_LP], want, 1e-10, 1e-10, 3))
    dl.dl_accum_destroy(acc)


@pytest.mark.parametrize("D,block", [(3, 1), (3, 3), (6, 5)])
def test_fp64_diluted_hpe_loops_match_oracle(ctx, lat, D, block):
    """Slots of one component (block 1) and slots that span components (3, 5)."""
    log("diluted hpe D", D, "block", block)
    seed, nsrc, p2, n = 43, 2, 2, 4
    acc = dl.dl_accum_create(lat.h, dl.DL_OPS_LOCAL | dl.DL_OPS_DERIV | dl.DL_OPS_HPE(n))
    rc, _ = dl.dl_solve_batch(ctx, dl.make_job(lat.h, noise=dl.DL_NOISE_Z4, tier=dl.DL_TIER_FP64, seed=seed,
                                               nsrc=nsrc, tol=1e-11, maxiter=1000, tdil=D, rhs_block=block,
                                               accum=acc, accum_set=dl.DL_SET_HP))
    assert dl.dl_accum_counts(acc) == [0, nsrc, 0]
    assert rc == dl.DL_OK
    npm = len(loops.momenta(p2, lat.dims))
    sets = np.zeros((3, 2, 5, 16, lat.dims[3], npm), dtype=np.complex128)
    dl.dl_loops_sets(ctx, acc, p2, sets, 0)
    want = oracle_vector_sums(lat, seed, range(nsrc), D, p2, n_hpe=n)
    log("  worst |d|/max|block|", elementwise(sets[dl.DL_SET_HP], want, 1e-10, 1e-10, 3))
    dl.dl_accum_destroy(acc)


def test_user_sources_are_diluted_like_generated_ones(ctx, lat):
    seed, nsrc, D, p2 = 44, 3, 2, 1
    src = dev(np.stack([noise.source(lat.dims, seed, r, noise.Z4) for r in range(nsrc)]))
    npm = len(loops.momenta(p2, lat.dims))
    outs = []
    for kw in (dict(noise=dl.DL_NOISE_Z4, seed=seed), dict(noise=dl.DL_NOISE_USER, src_in=src)):
        acc = dl.dl_accum_create(lat.h, dl.DL_OPS_LOCAL | dl.DL_OPS_HPE(2))
        dl.dl_solve_batch(ctx, dl.make_job(lat.h, tier=dl.DL_TIER_FP64, nsrc=nsrc, tol=1e-10, maxiter=1000,
                                           tdil=D, accum=acc, accum_set=dl.DL_SET_LP, **kw))
        out = np.zeros((3, 2, 1, 16, lat.dims[3], npm), dtype=np.complex128)
        dl.dl_loops_sets(ctx, acc, p2, out, 0)
        outs.append(out)
        dl.dl_accum_destroy(acc)
    assert np.array_equal(outs[0], outs[1])


def test_diluted_lp_maps_and_hp_guesses(ctx, lat):
    """bf16 LP maps of diluted sources are bit-identical across slot shapes, and HP solves
    started from the diluted LPC solutions converge to the oracle's solutions."""
    seed, nsrc, D, p2 = 45, 4, 3, 2
    npm = len(loops.momenta(p2, lat.dims))
    outs = []
    for block in (1, 4, 5):
        acc = dl.dl_accum_create(lat.h, dl.DL_OPS_LOCAL | dl.DL_OPS_DERIV | dl.DL_OPS_HPE(4))
        dl.dl_solve_batch(ctx, dl.make_job(lat.h, noise=dl.DL_NOISE_Z4, tier=dl.DL_TIER_LP_BF16, seed=seed,
                                           nsrc=nsrc, tol=1e-2, maxiter=500, rhs_block=block, tdil=D, accum=acc,
                                           accum_set=dl.DL_SET_LP))
        out = np.zeros((3, 2, 5, 16, lat.dims[3], npm), dtype=np.complex128)
        dl.dl_loops_sets(ctx, acc, p2, out, 0)
        outs.append(out)
        dl.dl_accum_destroy(acc)
    assert np.array_equal(outs[0], outs[1]) and np.array_equal(outs[0], outs[2])
    sol = zeros_dev((nsrc * D,) + lat.field_shape)
    jobs = [dl.make_job(lat.h, noise=dl.DL_NOISE_Z4, tier=dl.DL_TIER_HP_FP32, seed=seed, nsrc=nsrc, tol=1e-8,
                        maxiter=2000, tdil=D, sol_out=sol, guess_from=2, rhs_block=5),
            dl.make_job(lat.h, noise=dl.DL_NOISE_Z4, tier=dl.DL_TIER_LP_BF16, seed=seed, nsrc=nsrc, tol=1e-2,
                        maxiter=500, tdil=D, rhs_block=3)]
    rc, stats = dl.dl_solve_batch(ctx, jobs)
    assert rc == dl.DL_OK and len(stats) == 2 * nsrc * D
    got = host(sol)
    for c in range(D):
        for k in range(nsrc):
            eta = dilution.split(noise.source(lat.dims, seed, k, noise.Z4), D)[c]
            s, _ = solver.cgnr_eo(lat.U, eta, lat.kappa, lat.mu, lat.bc, lat.dims, 1e-12)
            assert rel(got[c * nsrc + k], s) < 1e-6, (c, k)


def test_dilution_argument_errors(ctx, lat):
    with pytest.raises(dl.DiscloopError) as e:
        dl.dl_solve_batch(ctx, dl.make_job(lat.h, nsrc=1, tol=1e-6, tdil=7))
    assert e.value.code == dl.DL_EINVAL
    with pytest.raises(dl.DiscloopError):
        dl.dl_solve_batch(ctx, [dl.make_job(lat.h, tier=dl.DL_TIER_HP_FP32, nsrc=1, tol=1e-6, tdil=2,
                                            guess_from=2),
                                dl.make_job(lat.h, tier=dl.DL_TIER_LP_BF16, nsrc=1, tol=1e-2, tdil=3)])
    g = np.zeros((2, 5, 16, lat.dims[3], 1), dtype=np.complex128)
    with pytest.raises(dl.DiscloopError):
        dl.dl_loops_backward(ctx, dl.make_job(lat.h, nsrc=1, tol=1e-6, tdil=2), 0, g, None, None)
