"""GPU parity of the hopping parameter expansion (loops without tau_3) against the
FP64 oracle, through the C ABI.

FP64 solves: every order 1..4, local and derivative insertions, per-set sums and the
normalised estimate to 1e-10 relative, on a lattice with a ragged tile tail.  The
storage-precision tiers are compared with the oracle evaluated on the solutions the
GPU returned (so only the expansion's arithmetic differs): the HP tier (FP64 contraction of
its FP64 solution) to 1e-10, bf16 and fp16 to a few units of their 2^-8 / 2^-11 storage
rounding; the bf16 maps are bit-identical across slot shapes.  Loops are compared element
by element against max|block| (gpu_util.elementwise).
"""
import sys

import numpy as np
import pytest

import paper_1401_6750_amd as dl
from oracle import hpe, loops, noise, solver
from tests.gpu_util import elementwise, host, make_lattice, rel, torch, zeros_dev

pytestmark = pytest.mark.gpu

DIMS = (6, 4, 6, 6)        # Vh = 432: six full 64-site tiles and a ragged one
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
    la = make_lattice(ctx, DIMS, 1407, 0.3, KAPPA, MU)
    yield la
    la.close()


def oracle_sums(la, seed, rs, n, p2, kind=noise.Z4, sols=None, tol=1e-11):
    """Sum over sources of the loops dl_loops_sets reports for an HPE(n) accumulator."""
    pf = loops.prefactors(la.kappa, la.mu)
    tot = 0
    for i, r in enumerate(rs):
        eta = noise.source(la.dims, seed, r, kind)
        if sols is None:
            s = solver.cgnr_eo(la.U, eta, la.kappa, la.mu, la.bc, la.dims, tol)[0]
        else:
            s = sols[i]
        t3 = loops.source_loops(la.U, s, la.kappa, la.bc, p2, la.dims)[loops.TAU3]
        h = hpe.hpe_source_loops(la.U, eta, s, la.kappa, la.mu, la.bc, n, p2, la.dims)
        h = h + hpe.hpe_exact_projected(la.kappa, la.mu, n, p2, la.dims)
        tot = tot + np.stack([pf[0] * t3, pf[1] * h])
    return tot


@pytest.mark.parametrize("n", [1, 2, 3, 4])
def test_fp64_hpe_loops_match_oracle(ctx, lat, n):
    log("hpe fp64 order", n)
    seed, nsrc, p2 = 31, 4, 3
    acc = dl.dl_accum_create(lat.h, dl.DL_OPS_LOCAL | dl.DL_OPS_DERIV | dl.DL_OPS_HPE(n))
    job = dl.make_job(lat.h, noise=dl.DL_NOISE_Z4, tier=dl.DL_TIER_FP64, seed=seed, nsrc=nsrc, tol=1e-11,
                      maxiter=1000, rhs_block=3, accum=acc, accum_set=dl.DL_SET_LP)
    rc, _ = dl.dl_solve_batch(ctx, job)
    assert rc == dl.DL_OK
    npm = len(loops.momenta(p2, lat.dims))
    sets = np.zeros((3, 2, 5, 16, lat.dims[3], npm), dtype=np.complex128)
    dl.dl_loops_sets(ctx, acc, p2, sets, 0)
    want = oracle_sums(lat, seed, range(nsrc), n, p2)
    log("  worst |d|/max|block|", elementwise(sets[dl.DL_SET_LP], want, 1e-10, 1e-10, 3))
    # the remainder on its own (exact part taken out) still agrees
    ex = 4 * lat.kappa * nsrc * hpe.hpe_exact_projected(lat.kappa, lat.mu, n, p2, lat.dims)
    elementwise(sets[dl.DL_SET_LP, 1] - ex, want[1] - ex, 1e-9, 1e-9, 2)
    assert np.abs(sets[dl.DL_SET_HP]).max() == 0 and np.abs(sets[dl.DL_SET_LPC]).max() == 0
    est = np.zeros((2, 5, 16, lat.dims[3], npm), dtype=np.complex128)
    dl.dl_loops(ctx, acc, p2, est, 0)
    elementwise(est, want / nsrc, 1e-10, 1e-10, 3)
    dl.dl_accum_destroy(acc)


def test_local_only_hpe_accumulator(ctx, lat):
    seed, nsrc, p2, n = 32, 2, 2, 4
    acc = dl.dl_accum_create(lat.h, dl.DL_OPS_LOCAL | dl.DL_OPS_HPE(n))
    dl.dl_solve_batch(ctx, dl.make_job(lat.h, noise=dl.DL_NOISE_Z2, tier=dl.DL_TIER_FP64, seed=seed, nsrc=nsrc,
                                       tol=1e-11, maxiter=1000, accum=acc, accum_set=dl.DL_SET_HP))
    npm = len(loops.momenta(p2, lat.dims))
    est = np.zeros((2, 1, 16, lat.dims[3], npm), dtype=np.complex128)
    dl.dl_loops(ctx, acc, p2, est, 0)
    want = oracle_sums(lat, seed, range(nsrc), n, p2, kind=noise.Z2)[:, :1] / nsrc
    elementwise(est, want, 1e-10, 1e-10, 3)
    dl.dl_accum_destroy(acc)


@pytest.mark.parametrize("tier,tol", [(dl.DL_TIER_HP_FP32, 1e-10), (dl.DL_TIER_LP_BF16, 2e-2),
                                      (dl.DL_TIER_LP_FP16, 4e-3)])
def test_storage_precision_hpe_against_oracle_on_gpu_solutions(ctx, lat, tier, tol):
    seed, nsrc, p2, n = 33, 4, 3, 4
    log("hpe tier", tier)
    acc = dl.dl_accum_create(lat.h, dl.DL_OPS_LOCAL | dl.DL_OPS_DERIV | dl.DL_OPS_HPE(n))
    sol = zeros_dev((nsrc,) + lat.field_shape)
    rho = 1e-8 if tier == dl.DL_TIER_HP_FP32 else 1e-2
    rc, _ = dl.dl_solve_batch(ctx, dl.make_job(lat.h, noise=dl.DL_NOISE_Z4, tier=tier, seed=seed, nsrc=nsrc,
                                               tol=rho, maxiter=2000, sol_out=sol, accum=acc,
                                               accum_set=dl.DL_SET_LP))
    assert rc == dl.DL_OK
    torch().cuda.synchronize()
    npm = len(loops.momenta(p2, lat.dims))
    sets = np.zeros((3, 2, 5, 16, lat.dims[3], npm), dtype=np.complex128)
    dl.dl_loops_sets(ctx, acc, p2, sets, 0)
    want = oracle_sums(lat, seed, range(nsrc), n, p2, sols=host(sol))
    ex = 4 * lat.kappa * nsrc * hpe.hpe_exact_projected(lat.kappa, lat.mu, n, p2, lat.dims)
    for f in range(2):
        for op in range(5):
            e = elementwise(sets[dl.DL_SET_LP, f, op] - (ex[op] if f else 0), want[f, op] - (ex[op] if f else 0),
                            tol if tier == dl.DL_TIER_HP_FP32 else 0.0, tol, 1)
            log("  flavour", f, "op", op, "worst |d|/max|block|", e)
    dl.dl_accum_destroy(acc)


def test_bf16_hpe_maps_bit_identical_across_slot_shapes(ctx, lat):
    seed, nsrc, p2 = 34, 10, 2
    npm = len(loops.momenta(p2, lat.dims))
    outs = []
    for block in (1, 4, 10):
        acc = dl.dl_accum_create(lat.h, dl.DL_OPS_LOCAL | dl.DL_OPS_DERIV | dl.DL_OPS_HPE(4))
        dl.dl_solve_batch(ctx, dl.make_job(lat.h, noise=dl.DL_NOISE_Z4, tier=dl.DL_TIER_LP_BF16, seed=seed,
                                           nsrc=nsrc, tol=1e-2, maxiter=500, rhs_block=block, accum=acc,
                                           accum_set=dl.DL_SET_LP))
        sets = np.zeros((3, 2, 5, 16, lat.dims[3], npm), dtype=np.complex128)
        dl.dl_loops_sets(ctx, acc, p2, sets, 0)
        outs.append(sets)
        dl.dl_accum_destroy(acc)
    assert np.array_equal(outs[0], outs[1]) and np.array_equal(outs[0], outs[2])


def test_tsm_with_hpe_and_mixed_accumulators(ctx, lat):
    """A TSM step with an HPE accumulator next to a one-end-trick accumulator in the
    same call: the tau_3 loops agree between the two, and the HPE estimate matches
    the oracle's TSM combination (LP / LPC at FP64 with rho = 1e-2)."""
    seed, p2, n = 35, 2, 4
    n_lp, n_hp = 6, 2
    a_h = dl.dl_accum_create(lat.h, dl.DL_OPS_LOCAL | dl.DL_OPS_DERIV | dl.DL_OPS_HPE(n))
    a_p = dl.dl_accum_create(lat.h, dl.DL_OPS_LOCAL | dl.DL_OPS_DERIV)
    jobs = []
    for acc in (a_h, a_p):
        jobs += [
            dl.make_job(lat.h, noise=dl.DL_NOISE_Z4, tier=dl.DL_TIER_FP64, seed=seed, first_src=0, nsrc=n_lp,
                        tol=1e-2, maxiter=300, accum=acc, accum_set=dl.DL_SET_LP),
            dl.make_job(lat.h, noise=dl.DL_NOISE_Z4, tier=dl.DL_TIER_FP64, seed=seed, first_src=n_lp, nsrc=n_hp,
                        tol=1e-11, maxiter=1000, accum=acc, accum_set=dl.DL_SET_HP),
            dl.make_job(lat.h, noise=dl.DL_NOISE_Z4, tier=dl.DL_TIER_FP64, seed=seed, first_src=n_lp, nsrc=n_hp,
                        tol=1e-2, maxiter=300, accum=acc, accum_set=dl.DL_SET_LPC),
        ]
    rc, _ = dl.dl_solve_batch(ctx, jobs)
    assert rc == dl.DL_OK
    npm = len(loops.momenta(p2, lat.dims))
    est_h = np.zeros((2, 5, 16, lat.dims[3], npm), dtype=np.complex128)
    est_p = np.zeros_like(est_h)
    dl.dl_loops(ctx, a_h, p2, est_h, 0)
    dl.dl_loops(ctx, a_p, p2, est_p, 0)
    elementwise(est_h[0], est_p[0], 1e-12, 1e-12, 2)
    s_lp = oracle_sums(lat, seed, range(n_lp), n, p2, tol=1e-2)
    s_hp = oracle_sums(lat, seed, range(n_lp, n_lp + n_hp), n, p2, tol=1e-11)
    s_lpc = oracle_sums(lat, seed, range(n_lp, n_lp + n_hp), n, p2, tol=1e-2)
    want = s_lp / n_lp + (s_hp - s_lpc) / n_hp
    elementwise(est_h, want, 1e-9, 1e-9, 3)
    dl.dl_accum_destroy(a_h)
    dl.dl_accum_destroy(a_p)


def test_hpe_argument_errors(ctx, lat):
    with pytest.raises(dl.DiscloopError) as e:
        dl.dl_accum_create(lat.h, dl.DL_OPS_LOCAL | dl.DL_OPS_HPE(5))
    assert e.value.code == dl.DL_EINVAL
    small = make_lattice(ctx, (4, 4, 4, 2), 3, 0.2, 0.15, 0.02)
    with pytest.raises(dl.DiscloopError):
        dl.dl_accum_create(small.h, dl.DL_OPS_LOCAL | dl.DL_OPS_HPE(1))
    small.close()
    a2 = dl.dl_accum_create(lat.h, dl.DL_OPS_LOCAL | dl.DL_OPS_HPE(2))
    a4 = dl.dl_accum_create(lat.h, dl.DL_OPS_LOCAL | dl.DL_OPS_HPE(4))
    with pytest.raises(dl.DiscloopError):
        dl.dl_solve_batch(ctx, [dl.make_job(lat.h, nsrc=1, tol=1e-6, accum=a2),
                                dl.make_job(lat.h, nsrc=1, tol=1e-6, accum=a4)])
    job = dl.make_job(lat.h, nsrc=1, tol=1e-6, accum=a4)
    g = np.zeros((2, 1, 16, lat.dims[3], 1), dtype=np.complex128)
    with pytest.raises(dl.DiscloopError):
        dl.dl_loops_backward(ctx, job, 0, g, None, None)
    dl.dl_accum_destroy(a2)
    dl.dl_accum_destroy(a4)
