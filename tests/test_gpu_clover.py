"""GPU parity of the clover variant of the operator (Section 2.4: Wilson and clover
fermions) against the FP64 oracle (oracle/clover.py), through the C ABI.

Tolerances as for the plain operator: FP64 operators 1e-13 relative, FP64 solves
and loops 1e-10 (element-wise, per (flavour, op, Gamma) block), storage-precision
operators a few units of their storage roundoff.  Also: a clover lattice and a plain
one in one batch give the same bits as alone, c_sw = 0 restores the plain operator,
the free field has no clover term, and the pieces not built for clover lattices
(expansion, gradients) are refused.
"""
import sys

import numpy as np
import pytest

import paper_1401_6750_amd as dl
import synth
from oracle import clover, dirac, loops, noise, solver
from tests.gpu_util import dev, elementwise, host, make_lattice, rel, torch, zeros_dev

pytestmark = pytest.mark.gpu

CSW = 1.6


def log(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def ctx():
    t = torch()
    assert t.cuda.is_available(), "GPU tests need a GPU"
    c = dl.dl_create(0, t.cuda.current_stream().cuda_stream)
    yield c
    dl.dl_destroy(c)


def clover_lattice(ctx, dims, seed, eps, kappa, mu, bc=-1, csw=CSW):
    la = make_lattice(ctx, dims, seed, eps, kappa, mu, bc)
    dl.dl_set_clover(la.h, csw)
    la.C = clover.clover_term(la.U, kappa, csw)
    return la


def oracle_op(la, op, psi):
    U, k, mu, bc, dims, C = la.U, la.kappa, la.mu, la.bc, la.dims, la.C
    mo = dirac.parity_mask(dims, 1)
    if op == dl.DL_OP_M:
        return dirac.apply_M(U, psi, k, mu, bc, C)
    if op == dl.DL_OP_MDAG:
        return dirac.apply_Mdag(U, psi, k, mu, bc, C)
    if op == dl.DL_OP_HOP:
        return dirac.hop(U, psi, bc)
    if op == dl.DL_OP_MHAT:
        return dirac.Mhat(U, mo * psi, k, mu, bc, dims, C)
    if op == dl.DL_OP_MHAT_DAG:
        return dirac.Mhat_dag(U, mo * psi, k, mu, bc, dims, C)
    raise ValueError(op)


OPS = [dl.DL_OP_M, dl.DL_OP_MDAG, dl.DL_OP_MHAT, dl.DL_OP_MHAT_DAG, dl.DL_OP_HOP]


def apply(la, op, tier, psi):
    out = zeros_dev(psi.shape)
    dl.dl_apply_op(la.h, op, tier, dev(psi), out, psi.shape[0])
    torch().cuda.synchronize()
    return host(out)


@pytest.mark.parametrize("dims", [(6, 4, 6, 6), (4, 4, 4, 4), (2, 4, 2, 4)])
@pytest.mark.parametrize("bc", [-1, 1])
def test_clover_operators_fp64(ctx, dims, bc):
    log("clover ops fp64", dims, bc)
    la = clover_lattice(ctx, dims, 81, 0.4, 0.14, 0.03, bc)
    psi = synth.random_spinor(dims, 5, nrhs=3)
    for op in OPS:
        e = rel(apply(la, op, dl.DL_TIER_FP64, psi), oracle_op(la, op, psi))
        log("  op", op, "rel", e)
        assert e < 1e-13, (op, e)
    # the term is really there: M differs from the plain operator's
    plain = dirac.apply_M(la.U, psi, la.kappa, la.mu, bc)
    assert rel(apply(la, dl.DL_OP_M, dl.DL_TIER_FP64, psi), plain) > 1e-3
    la.close()


@pytest.mark.parametrize("tier,tol", [(dl.DL_TIER_HP_FP32, 5e-7), (dl.DL_TIER_LP_FP16, 2e-3),
                                      (dl.DL_TIER_LP_BF16, 1.6e-2)])
def test_clover_operators_storage_precision(ctx, tier, tol):
    dims = (6, 4, 6, 6)
    la = clover_lattice(ctx, dims, 82, 0.3, 0.15, 0.02)
    psi = synth.random_spinor(dims, 6, nrhs=2)
    for op in OPS:
        e = rel(apply(la, op, tier, psi), oracle_op(la, op, psi))
        log("  clover op", tier, op, "rel", e)
        assert e < tol, (op, e)
    la.close()


def test_clover_fp64_solves_and_loops(ctx):
    """FP64 solves take the oracle's iteration counts and agree to 1e-10; all 160 loop
    insertions at p^2 <= 3 match the oracle's (with xi = (1 + C - kappa H) s) to 1e-10."""
    dims = (4, 4, 4, 4)
    la = clover_lattice(ctx, dims, 83, 0.3, 0.15, 0.01)
    seed, n, p2 = 91, 6, 3
    sol = zeros_dev((n,) + la.field_shape)
    acc = dl.dl_accum_create(la.h, dl.DL_OPS_LOCAL | dl.DL_OPS_DERIV)
    rc, st = dl.dl_solve_batch(ctx, dl.make_job(la.h, noise=dl.DL_NOISE_Z2, tier=dl.DL_TIER_FP64, seed=seed, nsrc=n,
                                                tol=1e-10, maxiter=500, rhs_block=4, report_true_resid=1,
                                                sol_out=sol, accum=acc, accum_set=dl.DL_SET_HP))
    assert rc == dl.DL_OK
    got = host(sol)
    per = []
    for r in range(n):
        eta = noise.source(dims, seed, r, noise.Z2)
        s, info = solver.cgnr_eo(la.U, eta, la.kappa, la.mu, la.bc, dims, 1e-10, C=la.C)
        assert st[r].iters == info["iters"], (r, st[r].iters, info["iters"])
        assert rel(got[r], s) < 1e-10
        assert solver.true_residual(la.U, eta, got[r], la.kappa, la.mu, la.bc, la.C) < 1e-8
        per.append(loops.source_loops(la.U, s, la.kappa, la.bc, p2, dims, C=la.C))
    out = np.zeros((2, 5, 16, dims[3], len(loops.momenta(p2, dims))), dtype=np.complex128)
    dl.dl_loops(ctx, acc, p2, out, 0)
    want = loops.estimate(np.array(per), la.kappa, la.mu)
    log("clover fp64 loops worst |d|/max|block|", elementwise(out, want, 1e-10, 1e-10, 3))
    # the no-tau_3 loops use the clover xi: differ from those with the plain xi
    plain_xi = loops.estimate(np.array([loops.source_loops(la.U, host(sol)[r], la.kappa, la.bc, p2, dims)
                                        for r in range(n)]), la.kappa, la.mu)
    assert np.abs(plain_xi[1] - want[1]).max() > 1e-3 * np.abs(want[1]).max()
    dl.dl_accum_destroy(acc)
    la.close()


def test_clover_tsm_tiers(ctx):
    """bf16 LP, FP32 + reliable-update HP (started from the LPC solutions) and LPC on a clover
    lattice: the HP solutions' true residuals (oracle operator with C) meet the target, the
    HP set's loops match the oracle's loops of the returned solutions, and the LP map is the
    same for every slot size."""
    dims = (6, 4, 6, 6)
    la = clover_lattice(ctx, dims, 84, 0.2, 0.1615, 0.004)
    seed, n_lp, n_hp, p2 = 92, 8, 4, 2
    hp_sol = zeros_dev((n_hp,) + la.field_shape)
    acc = dl.dl_accum_create(la.h, dl.DL_OPS_LOCAL | dl.DL_OPS_DERIV)
    jobs = [dl.make_job(la.h, noise=dl.DL_NOISE_Z4, tier=dl.DL_TIER_LP_BF16, seed=seed, nsrc=n_lp, tol=1e-2,
                        maxiter=500, accum=acc, accum_set=dl.DL_SET_LP),
            dl.make_job(la.h, noise=dl.DL_NOISE_Z4, tier=dl.DL_TIER_HP_FP32, seed=seed, first_src=n_lp, nsrc=n_hp,
                        tol=1e-8, maxiter=2000, sol_out=hp_sol, accum=acc, accum_set=dl.DL_SET_HP, guess_from=3),
            dl.make_job(la.h, noise=dl.DL_NOISE_Z4, tier=dl.DL_TIER_LP_BF16, seed=seed, first_src=n_lp, nsrc=n_hp,
                        tol=1e-2, maxiter=500, accum=acc, accum_set=dl.DL_SET_LPC)]
    rc, st = dl.dl_solve_batch(ctx, jobs)
    assert rc == dl.DL_OK
    sets = np.zeros((3, 2, 5, 16, dims[3], len(loops.momenta(p2, dims))), dtype=np.complex128)
    dl.dl_loops_sets(ctx, acc, p2, sets, 0)
    got = host(hp_sol)
    per = []
    for r in range(n_hp):
        eta = noise.source(dims, seed, n_lp + r, noise.Z4)
        tr = solver.true_residual(la.U, eta, got[r], la.kappa, la.mu, la.bc, la.C)
        log(f"clover hp {r}: iters {st[n_lp + r].iters} true resid {tr:.2e}")
        assert tr < 2e-7
        per.append(loops.source_loops(la.U, got[r], la.kappa, la.bc, p2, dims, C=la.C))
    want_hp = loops.apply_prefactors(np.sum(per, axis=0), la.kappa, la.mu)
    log("clover hp-set loops worst |d|/max|block|", elementwise(sets[1], want_hp, 1e-9, 1e-9, 3))
    # LP map independent of the slot size
    outs = []
    for blk in (8, 3, 1):
        sol = zeros_dev((n_lp,) + la.field_shape)
        dl.dl_solve_batch(ctx, dl.make_job(la.h, noise=dl.DL_NOISE_Z4, tier=dl.DL_TIER_LP_BF16, seed=seed,
                                           nsrc=n_lp, tol=1e-2, maxiter=500, rhs_block=blk, sol_out=sol))
        outs.append(host(sol))
    assert np.array_equal(outs[0], outs[1]) and np.array_equal(outs[0], outs[2])
    dl.dl_accum_destroy(acc)
    la.close()


def _solve(ctx, jobs_of, lats, tier, tol):
    sols = [zeros_dev((4,) + la.field_shape) for la in lats]
    jobs = [dl.make_job(la.h, noise=dl.DL_NOISE_Z4, tier=tier, seed=93, nsrc=4, tol=tol, maxiter=2000, sol_out=s)
            for la, s in zip(lats, sols)]
    rc, st = dl.dl_solve_batch(ctx, jobs)
    assert rc == dl.DL_OK
    return [host(s) for s in sols], [x.iters for x in st]


@pytest.mark.parametrize("tier,tol", [(dl.DL_TIER_LP_BF16, 1e-2), (dl.DL_TIER_HP_FP32, 1e-8), (dl.DL_TIER_FP64, 1e-9)])
def test_mixed_clover_and_plain_batch(ctx, tier, tol):
    """A clover lattice and a plain one in one call give the same bits as each alone."""
    a = clover_lattice(ctx, (4, 4, 4, 4), 85, 0.3, 0.15, 0.02)
    b = make_lattice(ctx, (6, 4, 4, 4), 86, 0.3, 0.15, 0.02)
    both, it_both = _solve(ctx, None, [a, b], tier, tol)
    sa, ia = _solve(ctx, None, [a], tier, tol)
    sb, ib = _solve(ctx, None, [b], tier, tol)
    assert np.array_equal(both[0], sa[0]) and np.array_equal(both[1], sb[0])
    assert it_both == ia + ib
    a.close()
    b.close()


def test_clover_off_free_field_and_refusals(ctx):
    dims = (4, 4, 4, 4)
    psi = synth.random_spinor(dims, 7, nrhs=2)
    # c_sw = 0 restores the plain operator bit for bit
    la = clover_lattice(ctx, dims, 87, 0.3, 0.15, 0.02)
    ref = make_lattice(ctx, dims, 87, 0.3, 0.15, 0.02)
    with_c = apply(la, dl.DL_OP_MHAT, dl.DL_TIER_FP64, psi)
    dl.dl_set_clover(la.h, 0.0)
    for op in OPS:
        assert np.array_equal(apply(la, op, dl.DL_TIER_FP64, psi), apply(ref, op, dl.DL_TIER_FP64, psi))
    assert rel(with_c, apply(ref, dl.DL_OP_MHAT, dl.DL_TIER_FP64, psi)) > 1e-3
    # setting it again (after kappa / mu changed) rebuilds the site matrices
    dl.dl_set_params(la.h, 0.13, 0.05)
    dl.dl_set_clover(la.h, 1.1)
    la.kappa, la.mu, la.C = 0.13, 0.05, clover.clover_term(la.U, 0.13, 1.1)
    assert rel(apply(la, dl.DL_OP_MHAT, dl.DL_TIER_FP64, psi), oracle_op(la, dl.DL_OP_MHAT, psi)) < 1e-13
    # free field: no field strength, the clover operator is the plain one
    fr = clover_lattice(ctx, dims, 88, 0.3, 0.15, 0.02)
    fr.U = synth.unit_gauge(dims)
    dl.dl_gauge_set(fr.h, np.ascontiguousarray(fr.U), 0)
    fp = make_lattice(ctx, dims, 88, 0.3, 0.15, 0.02)
    dl.dl_gauge_set(fp.h, np.ascontiguousarray(fr.U), 0)
    assert rel(apply(fr, dl.DL_OP_M, dl.DL_TIER_FP64, psi), apply(fp, dl.DL_OP_M, dl.DL_TIER_FP64, psi)) < 1e-15
    # not built for clover lattices: the expansion and the gradients
    acc = dl.dl_accum_create(la.h, dl.DL_OPS_LOCAL | dl.DL_OPS_HPE(2))
    with pytest.raises(dl.DiscloopError) as e:
        dl.dl_solve_batch(ctx, dl.make_job(la.h, nsrc=1, tol=1e-8, accum=acc))
    assert e.value.code == dl.DL_EINVAL
    dl.dl_accum_destroy(acc)
    g = np.zeros((2, 5, 16, dims[3], 1), dtype=np.complex128)
    with pytest.raises(dl.DiscloopError):
        dl.dl_loops_backward(ctx, dl.make_job(la.h, nsrc=1, tol=1e-8), 0, g, None, np.zeros(1))
    with pytest.raises(dl.DiscloopError):
        dl.dl_set_clover(la.h, float("nan"))
    for x in (la, ref, fr, fp):
        x.close()
