"""GPU parity of the HIP path against the FP64 oracle, through the C ABI.

Tolerances: integer work (noise) is bit-exact.  FP64 operators agree to
1e-13 relative (rounding order only); FP64 solves and loops to 1e-10 relative
(the FP64 solve requirement); the storage-precision operators to a few units
of their storage roundoff u (fp32 2^-24, fp16 2^-11, bf16 2^-8):
5e-7, 2e-3 and 1.6e-2 relative L2.
"""
import sys

import os

import numpy as np
import pytest

import paper_1401_6750_amd as dl
import synth
from oracle import dirac, loops, noise, solver
from tests.gpu_util import dev, host, make_lattice, rel, torch, zeros_dev

pytestmark = pytest.mark.gpu


def log(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def ctx():
    t = torch()
    assert t.cuda.is_available(), "GPU tests need a GPU"
    c = dl.dl_create(0, t.cuda.current_stream().cuda_stream)
    yield c
    dl.dl_destroy(c)


# ---------------------------------------------------------------------------
# noise: bit-exact
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("dims", [(4, 4, 4, 4), (6, 2, 4, 6), (2, 2, 2, 2)])
@pytest.mark.parametrize("kind", [dl.DL_NOISE_Z2, dl.DL_NOISE_Z4])
def test_noise_bit_exact(ctx, dims, kind):
    log("noise", dims, kind)
    lat = make_lattice(ctx, dims, 1, 0.2, 0.15, 0.01)
    for seed, r in [(6750, 0), (6750, 1), (6751, 7), (2**63 + 5, 12345)]:
        out = zeros_dev(lat.field_shape)
        dl.dl_fill_noise(lat.h, kind, seed, r, out)
        torch().cuda.synchronize()
        want = noise.source(dims, seed, r, kind)
        assert np.array_equal(host(out), want), (seed, r)
    lat.close()


# ---------------------------------------------------------------------------
# operators
# ---------------------------------------------------------------------------
def oracle_op(lat, op, psi):
    U, k, mu, bc, dims = lat.U, lat.kappa, lat.mu, lat.bc, lat.dims
    mo, me = dirac.parity_mask(dims, 1), dirac.parity_mask(dims, 0)
    if op == dl.DL_OP_M:
        return dirac.apply_M(U, psi, k, mu, bc)
    if op == dl.DL_OP_MDAG:
        return dirac.apply_Mdag(U, psi, k, mu, bc)
    if op == dl.DL_OP_HOP:
        return dirac.hop(U, psi, bc)
    if op == dl.DL_OP_MHAT:
        return dirac.Mhat(U, mo * psi, k, mu, bc, dims)
    if op == dl.DL_OP_MHAT_DAG:
        return dirac.Mhat_dag(U, mo * psi, k, mu, bc, dims)
    raise ValueError(op)


OPS = [dl.DL_OP_M, dl.DL_OP_MDAG, dl.DL_OP_MHAT, dl.DL_OP_MHAT_DAG, dl.DL_OP_HOP]


@pytest.mark.parametrize("dims", [(4, 4, 4, 4), (6, 6, 6, 6), (2, 4, 6, 8), (8, 2, 2, 4), (2, 2, 2, 2)])
@pytest.mark.parametrize("bc", [-1, 1])
def test_operators_fp64(ctx, dims, bc):
    log("ops fp64", dims, bc)
    lat = make_lattice(ctx, dims, 11, 0.4, 0.15, 0.03, bc)
    psi = synth.random_spinor(dims, 5, nrhs=3)
    for op in OPS:
        out = zeros_dev(psi.shape)
        dl.dl_apply_op(lat.h, op, dl.DL_TIER_FP64, dev(psi), out, 3)
        torch().cuda.synchronize()
        assert rel(host(out), oracle_op(lat, op, psi)) < 1e-13, op
    lat.close()


@pytest.mark.parametrize("tier,tol", [(dl.DL_TIER_HP_FP32, 5e-7), (dl.DL_TIER_LP_FP16, 2e-3),
                                      (dl.DL_TIER_LP_BF16, 1.6e-2)])
def test_operators_storage_precision(ctx, tier, tol):
    dims = (6, 4, 4, 8)
    log("ops", tier)
    lat = make_lattice(ctx, dims, 12, 0.3, 0.16, 0.02)
    psi = synth.random_spinor(dims, 6, nrhs=2)
    for op in OPS:
        out = zeros_dev(psi.shape)
        dl.dl_apply_op(lat.h, op, tier, dev(psi), out, 2)
        torch().cuda.synchronize()
        e = rel(host(out), oracle_op(lat, op, psi))
        log("  op", op, "rel err", e)
        assert e < tol, (op, e)
    lat.close()


# ---------------------------------------------------------------------------
# FP64 solves and loops: the plain method on 4^4 (eps 0.3, kappa 0.16, mu 0.01,
# 16 Z2 sources, CG to 1e-10, local insertions at p^2 <= 3)
# ---------------------------------------------------------------------------
PLAIN = synth.WORKLOADS["plain_4x4x4x4"]


def _oracle_solutions(lat, seed, rs, tol, kind=noise.Z2):
    out = []
    for r in rs:
        eta = noise.source(lat.dims, seed, r, kind)
        s, info = solver.cgnr_eo(lat.U, eta, lat.kappa, lat.mu, lat.bc, lat.dims, tol)
        out.append((s, info))
    return out


@pytest.fixture(scope="module")
def plain(ctx):
    w = PLAIN
    lat = make_lattice(ctx, w["dims"], w["gauge_seed"], w["eps"], w["kappa"], w["mu"])
    ref = _oracle_solutions(lat, w["source_seed"], range(16), 1e-10)
    yield lat, ref
    lat.close()


@pytest.mark.parametrize("block", [16, 5, 1])
def test_fp64_solves_match_oracle(ctx, plain, block):
    lat, ref = plain
    log("fp64 solves block", block)
    sol = zeros_dev((16,) + lat.field_shape)
    job = dl.make_job(lat.h, noise=dl.DL_NOISE_Z2, tier=dl.DL_TIER_FP64, seed=PLAIN["source_seed"], nsrc=16,
                      tol=1e-10, maxiter=500, rhs_block=block, report_true_resid=1, sol_out=sol)
    rc, stats = dl.dl_solve_batch(ctx, job)
    assert rc == dl.DL_OK
    got = host(sol)
    for r in range(16):
        s, info = ref[r]
        assert stats[r].status == dl.DL_SRC_CONVERGED
        assert stats[r].iters == info["iters"], (r, stats[r].iters, info["iters"])
        assert rel(got[r], s) < 1e-10
        assert abs(stats[r].rel_resid - info["rel_resid"]) < 1e-6 * info["rel_resid"] + 1e-14
        assert 0 <= stats[r].true_resid < 1e-8


def test_fp64_loops_match_oracle(ctx, plain):
    lat, ref = plain
    log("fp64 loops")
    acc = dl.dl_accum_create(lat.h, dl.DL_OPS_LOCAL | dl.DL_OPS_DERIV)
    job = dl.make_job(lat.h, noise=dl.DL_NOISE_Z2, tier=dl.DL_TIER_FP64, seed=PLAIN["source_seed"], nsrc=16,
                      tol=1e-10, maxiter=500, accum=acc, accum_set=dl.DL_SET_HP)
    dl.dl_solve_batch(ctx, job)
    for p2 in (3, 0):
        np_ = len(loops.momenta(p2, lat.dims))
        out = np.zeros((2, 5, 16, lat.dims[3], np_), dtype=np.complex128)
        assert dl.dl_loops(ctx, acc, p2, out, 0) == np_
        per = np.array([loops.source_loops(lat.U, s, lat.kappa, lat.bc, p2, lat.dims) for s, _ in ref])
        want = loops.estimate(per, lat.kappa, lat.mu)
        assert rel(out, want) < 1e-10, rel(out, want)
        # each flavour / operator block on its own scale
        for f in range(2):
            for op in range(5):
                assert rel(out[f, op], want[f, op]) < 1e-9, (f, op)
    assert dl.dl_accum_counts(acc) == [0, 16, 0]
    dl.dl_accum_destroy(acc)


def test_local_only_accumulator(ctx, plain):
    lat, ref = plain
    acc = dl.dl_accum_create(lat.h, dl.DL_OPS_LOCAL)
    job = dl.make_job(lat.h, noise=dl.DL_NOISE_Z2, tier=dl.DL_TIER_FP64, seed=PLAIN["source_seed"], nsrc=16,
                      tol=1e-10, maxiter=500, accum=acc, accum_set=dl.DL_SET_HP)
    dl.dl_solve_batch(ctx, job)
    np_ = len(loops.momenta(3, lat.dims))
    out = np.zeros((2, 1, 16, lat.dims[3], np_), dtype=np.complex128)
    dl.dl_loops(ctx, acc, 3, out, 0)
    per = np.array([loops.source_loops(lat.U, s, lat.kappa, lat.bc, 3, lat.dims, deriv=False) for s, _ in ref])
    assert rel(out, loops.estimate(per, lat.kappa, lat.mu)) < 1e-10
    dl.dl_accum_destroy(acc)


def test_tsm_combination_matches_oracle(ctx, plain):
    """All three TSM sets at FP64 (LP at rho = 1e-2): the combination matches the oracle's."""
    lat, _ = plain
    seed = 99
    acc = dl.dl_accum_create(lat.h, dl.DL_OPS_LOCAL | dl.DL_OPS_DERIV)
    n_lp, n_hp = 12, 4
    jobs = [
        dl.make_job(lat.h, noise=dl.DL_NOISE_Z4, tier=dl.DL_TIER_FP64, seed=seed, first_src=0, nsrc=n_lp, tol=1e-2,
                    maxiter=200, accum=acc, accum_set=dl.DL_SET_LP),
        dl.make_job(lat.h, noise=dl.DL_NOISE_Z4, tier=dl.DL_TIER_FP64, seed=seed, first_src=n_lp, nsrc=n_hp,
                    tol=1e-10, maxiter=500, accum=acc, accum_set=dl.DL_SET_HP),
        dl.make_job(lat.h, noise=dl.DL_NOISE_Z4, tier=dl.DL_TIER_FP64, seed=seed, first_src=n_lp, nsrc=n_hp,
                    tol=1e-2, maxiter=200, accum=acc, accum_set=dl.DL_SET_LPC),
    ]
    dl.dl_solve_batch(ctx, jobs)
    np_ = len(loops.momenta(3, lat.dims))
    out = np.zeros((2, 5, 16, lat.dims[3], np_), dtype=np.complex128)
    dl.dl_loops(ctx, acc, 3, out, 0)

    def sl(r, tol):
        eta = noise.source(lat.dims, seed, r, noise.Z4)
        s, _ = solver.cgnr_eo(lat.U, eta, lat.kappa, lat.mu, lat.bc, lat.dims, tol)
        return loops.source_loops(lat.U, s, lat.kappa, lat.bc, 3, lat.dims)

    s_lp = sum(sl(r, 1e-2) for r in range(n_lp))
    s_hp = sum(sl(r, 1e-10) for r in range(n_lp, n_lp + n_hp))
    s_lpc = sum(sl(r, 1e-2) for r in range(n_lp, n_lp + n_hp))
    want = loops.tsm_combine(s_lp, n_lp, s_hp, s_lpc, n_hp, lat.kappa, lat.mu)
    assert rel(out, want) < 1e-9
    dl.dl_accum_destroy(acc)


def test_loop_sets_and_base2_storage(ctx, plain, tmp_path):
    """dl_loops_sets: the per-set sums recombine to dl_loops and match the oracle's summed
    loops; base-2 storage (Fig. 2) rebuilds the estimate of any count from level files and
    resumes a missing level with identical bits."""
    from paper_1401_6750_amd import base2
    lat, _ = plain
    seed, p2 = 99, 3
    acc = dl.dl_accum_create(lat.h, dl.DL_OPS_LOCAL | dl.DL_OPS_DERIV)
    jobs = [
        dl.make_job(lat.h, noise=dl.DL_NOISE_Z4, tier=dl.DL_TIER_FP64, seed=seed, first_src=0, nsrc=6, tol=1e-2,
                    maxiter=200, accum=acc, accum_set=dl.DL_SET_LP),
        dl.make_job(lat.h, noise=dl.DL_NOISE_Z4, tier=dl.DL_TIER_FP64, seed=seed, first_src=6, nsrc=3,
                    tol=1e-10, maxiter=500, accum=acc, accum_set=dl.DL_SET_HP),
        dl.make_job(lat.h, noise=dl.DL_NOISE_Z4, tier=dl.DL_TIER_FP64, seed=seed, first_src=6, nsrc=3,
                    tol=1e-2, maxiter=200, accum=acc, accum_set=dl.DL_SET_LPC),
    ]
    dl.dl_solve_batch(ctx, jobs)
    npm = len(loops.momenta(p2, lat.dims))
    T = lat.dims[3]
    est = np.zeros((2, 5, 16, T, npm), dtype=np.complex128)
    sets = np.zeros((3, 2, 5, 16, T, npm), dtype=np.complex128)
    dl.dl_loops(ctx, acc, p2, est, 0)
    dl.dl_loops_sets(ctx, acc, p2, sets, 0)
    assert rel(sets[0] / 6 + (sets[1] - sets[2]) / 3, est) < 1e-12
    want_hp = loops.apply_prefactors(sum(
        loops.source_loops(lat.U, solver.cgnr_eo(lat.U, noise.source(lat.dims, seed, r, noise.Z4), lat.kappa,
                                                 lat.mu, lat.bc, lat.dims, 1e-10)[0], lat.kappa, lat.bc, p2, lat.dims)
        for r in range(6, 9)), lat.kappa, lat.mu)
    assert rel(sets[1], want_hp) < 1e-9
    dl.dl_accum_destroy(acc)

    # base-2 storage of a Z2 stream: 3 levels = 7 sources; n = 5 uses levels 0 and 2
    meta = {"dims": list(lat.dims), "seed": 5, "tier": "fp64", "tol": 1e-10, "p2max": p2}
    st = base2.Base2Store(str(tmp_path / "b2"), meta)
    kw = dict(tier=dl.DL_TIER_FP64, noise=dl.DL_NOISE_Z2, seed=5, tol=1e-10, maxiter=500, p2max=p2,
              ops=dl.DL_OPS_LOCAL | dl.DL_OPS_DERIV)
    assert base2.solve_base2(ctx, lat.h, lat.dims, st, 3, **kw) == [0, 1, 2]
    srcs = [0, 3, 4, 5, 6]
    per = [loops.source_loops(lat.U, solver.cgnr_eo(lat.U, noise.source(lat.dims, 5, r, noise.Z2), lat.kappa,
                                                    lat.mu, lat.bc, lat.dims, 1e-10)[0], lat.kappa, lat.bc, p2,
                              lat.dims) for r in srcs]
    assert rel(st.estimate(5), loops.estimate(np.stack(per), lat.kappa, lat.mu)) < 1e-9
    lvl1 = st.load(1)
    os.remove(os.path.join(st.dir, "level01.npy"))
    assert st.resume_level() == 1
    assert base2.solve_base2(ctx, lat.h, lat.dims, base2.Base2Store(st.dir, meta), 3, **kw) == [1]
    assert np.array_equal(st.load(1), lvl1)


# ---------------------------------------------------------------------------
# precision tiers: errors against the FP64 oracle at the LP / HP targets
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("tier,tol", [(dl.DL_TIER_LP_BF16, 1e-2), (dl.DL_TIER_LP_FP16, 1e-2),
                                      (dl.DL_TIER_HP_FP32, 1e-8)])
def test_tier_error_against_exact(ctx, tier, tol):
    dims = (8, 8, 8, 8)
    lat = make_lattice(ctx, dims, 1405, 0.2, 0.1615, 0.004)
    n = 4
    sol = zeros_dev((n,) + lat.field_shape)
    job = dl.make_job(lat.h, noise=dl.DL_NOISE_Z2, tier=tier, seed=3, nsrc=n, tol=tol, maxiter=2000,
                      report_true_resid=1, sol_out=sol)
    rc, stats = dl.dl_solve_batch(ctx, job)
    assert rc == dl.DL_OK
    got = host(sol)
    for r in range(n):
        eta = noise.source(dims, 3, r, noise.Z2)
        exact, _ = solver.cgnr_eo(lat.U, eta, lat.kappa, lat.mu, lat.bc, dims, 1e-13)
        err = rel(got[r], exact)
        tr = solver.true_residual(lat.U, eta, got[r], lat.kappa, lat.mu, lat.bc)
        log(f"tier {tier} rho {tol}: iters {stats[r].iters} rel_resid {stats[r].rel_resid:.3e} "
            f"true {stats[r].true_resid:.3e} (oracle {tr:.3e}) err vs exact {err:.3e} RU {stats[r].reliable_updates}")
        assert stats[r].status == dl.DL_SRC_CONVERGED
        assert abs(stats[r].true_resid - tr) < 1e-3 * tr + 1e-12
        if tier == dl.DL_TIER_HP_FP32:
            assert stats[r].reliable_updates >= 1
            assert tr < 20 * tol and err < 100 * tol
        else:
            assert tr < 6 * tol and err < 20 * tol
    lat.close()


# ---------------------------------------------------------------------------
# batching: block size, uneven lattices and repeat runs give identical results
# ---------------------------------------------------------------------------
def _solve(ctx, lat, tier, nsrc, block, seed=5, first=0):
    sol = zeros_dev((nsrc,) + lat.field_shape)
    job = dl.make_job(lat.h, noise=dl.DL_NOISE_Z4, tier=tier, seed=seed, first_src=first, nsrc=nsrc, tol=1e-2,
                      maxiter=200, rhs_block=block, sol_out=sol)
    rc, stats = dl.dl_solve_batch(ctx, job)
    return host(sol), [s.iters for s in stats]


@pytest.mark.parametrize("lp_sol", [False, True])
def test_hp_started_from_lp_solutions(ctx, lp_sol):
    """HP solves started from the LP solutions of the same sources (guess_from) reach the same
    accuracy against the exact solution in fewer iterations; the LP solutions come from the
    caller's sol_out when given, else from a library buffer."""
    dims = (8, 8, 8, 8)
    lat = make_lattice(ctx, dims, 1405, 0.2, 0.1615, 0.004)
    n, tol = 4, 1e-8
    sol0 = zeros_dev((n,) + lat.field_shape)
    base = dl.make_job(lat.h, noise=dl.DL_NOISE_Z2, tier=dl.DL_TIER_HP_FP32, seed=3, nsrc=n, tol=tol, maxiter=2000,
                       report_true_resid=1, sol_out=sol0)
    _, st0 = dl.dl_solve_batch(ctx, base)
    sol = zeros_dev((n,) + lat.field_shape)
    lp_out = zeros_dev((n,) + lat.field_shape) if lp_sol else None
    jobs = [dl.make_job(lat.h, noise=dl.DL_NOISE_Z2, tier=dl.DL_TIER_LP_BF16, seed=3, nsrc=n, tol=1e-2,
                        maxiter=500, sol_out=lp_out),
            dl.make_job(lat.h, noise=dl.DL_NOISE_Z2, tier=dl.DL_TIER_HP_FP32, seed=3, nsrc=n, tol=tol, maxiter=2000,
                        report_true_resid=1, sol_out=sol, guess_from=1)]
    rc, st = dl.dl_solve_batch(ctx, jobs)
    assert rc == dl.DL_OK
    got = host(sol)
    for r in range(n):
        hs = st[n + r]
        eta = noise.source(dims, 3, r, noise.Z2)
        exact, _ = solver.cgnr_eo(lat.U, eta, lat.kappa, lat.mu, lat.bc, dims, 1e-13)
        err = rel(got[r], exact)
        tr = solver.true_residual(lat.U, eta, got[r], lat.kappa, lat.mu, lat.bc)
        log(f"guess: iters {hs.iters} (from zero {st0[r].iters}) RU {hs.reliable_updates} true {tr:.3e} err {err:.3e}")
        assert hs.status == dl.DL_SRC_CONVERGED
        assert tr < 20 * tol and err < 100 * tol
        assert hs.iters < st0[r].iters
    # invalid pairings are rejected before any work
    bad = [dict(guess_from=2), dict(guess_from=5), dict(seed=4, guess_from=1)]
    for kw in bad:
        lp = dl.make_job(lat.h, noise=dl.DL_NOISE_Z2, tier=dl.DL_TIER_LP_BF16, seed=3, nsrc=n, tol=1e-2)
        args = dict(noise=dl.DL_NOISE_Z2, tier=dl.DL_TIER_HP_FP32, seed=3, nsrc=n, tol=tol)
        args.update(kw)
        with pytest.raises(dl.DiscloopError):
            dl.dl_solve_batch(ctx, [lp, dl.make_job(lat.h, **args)])


@pytest.mark.parametrize("tier", [dl.DL_TIER_LP_BF16, dl.DL_TIER_LP_FP16])
def test_lp_map_is_independent_of_blocking(ctx, tier):
    lat = make_lattice(ctx, (6, 6, 6, 8), 21, 0.2, 0.1615, 0.004)
    a, ia = _solve(ctx, lat, tier, 10, 10)
    b, ib = _solve(ctx, lat, tier, 10, 1)
    c, ic = _solve(ctx, lat, tier, 10, 4)
    d, idd = _solve(ctx, lat, tier, 10, 10)
    e, ie = _solve(ctx, lat, tier, 3, 3, first=7)      # sources 7..9 alone
    assert ia == ib == ic == idd
    assert np.array_equal(a, b) and np.array_equal(a, c) and np.array_equal(a, d)
    assert np.array_equal(a[7:], e) and ia[7:] == ie
    lat.close()


def test_tile_order_and_tuned_shape_do_not_change_results(tmp_path):
    """The slot shape the autotuner hands the solver (rhs per slot, tile-order time block) changes
    only the order of the work: LP solutions and iteration counts are bit-identical for every
    shape (reductions are ordered by physical tile).  8^4 has whole tiles per time slice, so the
    time-blocked order is really used; the shape is forced through the tuning cache file."""
    import json, os
    t = torch()
    U = None
    ref = None
    for blk, tb in [(4, 1), (4, 2), (4, 4), (2, 8), (8, 3), (16, 1)]:
        cache = tmp_path / f"tune_{blk}_{tb}.json"
        cache.write_text(json.dumps({"8x8x8x8:bf16:16": blk, "8x8x8x8:bf16:16:t": tb}))
        old = os.environ.get("DL_TUNE_CACHE")
        os.environ["DL_TUNE_CACHE"] = str(cache)
        try:
            c = dl.dl_create(0, t.cuda.current_stream().cuda_stream)
            lat = make_lattice(c, (8, 8, 8, 8), 41, 0.2, 0.1615, 0.004)
            assert dl.dl_autotune(c, lat.h, dl.DL_TIER_LP_BF16, 10) == (min(blk, 10), tb)
            got = _solve(c, lat, dl.DL_TIER_LP_BF16, 10, 0)
            lat.close()
            dl.dl_destroy(c)
        finally:
            if old is None:
                del os.environ["DL_TUNE_CACHE"]
            else:
                os.environ["DL_TUNE_CACHE"] = old
        if ref is None:
            ref = got
        assert np.array_equal(got[0], ref[0]) and got[1] == ref[1], (blk, tb)


def test_graph_replay_equals_plain_launches(ctx):
    """CG iterations replayed from a HIP graph give the same bits as plain launches,
    and repeated graph runs with host work in between stay identical."""
    lat = make_lattice(ctx, (6, 6, 6, 8), 25, 0.2, 0.1615, 0.004)
    runs = []
    for use_graph in (1, 0, 1, 1):
        dl.dl_set_option(ctx, "use_graph", use_graph)
        a, ia = _solve(ctx, lat, dl.DL_TIER_LP_BF16, 6, 3)
        b, ib = _solve(ctx, lat, dl.DL_TIER_FP64, 2, 2)
        runs.append((a, ia, b, ib))
        _ = np.linalg.norm(a)          # host work between replays
    dl.dl_set_option(ctx, "use_graph", 1)
    for a, ia, b, ib in runs[1:]:
        assert np.array_equal(a, runs[0][0]) and ia == runs[0][1]
        assert np.array_equal(b, runs[0][2]) and ib == runs[0][3]
    lat.close()


def test_uneven_batch_equals_separate_runs(ctx):
    la = make_lattice(ctx, (4, 4, 4, 4), 31, 0.1, 0.1615, 0.004)
    lb = make_lattice(ctx, (8, 6, 4, 6), 32, 0.3, 0.1615, 0.004)
    lc = make_lattice(ctx, (6, 6, 6, 8), 33, 0.2, 0.1615, 0.004)
    lats, ns = [la, lb, lc], [9, 3, 5]
    sols = [zeros_dev((n,) + l.field_shape) for l, n in zip(lats, ns)]
    accs = [dl.dl_accum_create(l.h, dl.DL_OPS_LOCAL | dl.DL_OPS_DERIV) for l in lats]
    jobs = [dl.make_job(l.h, noise=dl.DL_NOISE_Z4, tier=dl.DL_TIER_LP_FP16, seed=7, nsrc=n, tol=1e-2, maxiter=200,
                        rhs_block=4, sol_out=s, accum=a, accum_set=dl.DL_SET_LP)
            for l, n, s, a in zip(lats, ns, sols, accs)]
    dl.dl_solve_batch(ctx, jobs)
    for l, n, s, a in zip(lats, ns, sols, accs):
        alone = zeros_dev((n,) + l.field_shape)
        acc2 = dl.dl_accum_create(l.h, dl.DL_OPS_LOCAL | dl.DL_OPS_DERIV)
        job = dl.make_job(l.h, noise=dl.DL_NOISE_Z4, tier=dl.DL_TIER_LP_FP16, seed=7, nsrc=n, tol=1e-2, maxiter=200,
                          rhs_block=4, sol_out=alone, accum=acc2, accum_set=dl.DL_SET_LP)
        dl.dl_solve_batch(ctx, job)
        assert np.array_equal(host(s), host(alone))
        np_ = len(loops.momenta(2, l.dims))
        o1 = np.zeros((2, 5, 16, l.dims[3], np_), dtype=np.complex128)
        o2 = np.zeros_like(o1)
        dl.dl_loops(ctx, a, 2, o1, 0)
        dl.dl_loops(ctx, acc2, 2, o2, 0)
        assert np.array_equal(o1, o2)
        dl.dl_accum_destroy(acc2)
    for a in accs:
        dl.dl_accum_destroy(a)
    for l in lats:
        l.close()


# ---------------------------------------------------------------------------
# full-size lattices: sampled sites against the oracle's per-site operator
# ---------------------------------------------------------------------------
def _boundary_sites(dims, rng, n):
    X, Y, Z, T = dims
    pick = [(0, 0, 0, 0), (T - 1, Z - 1, Y - 1, X - 1), (0, Z - 1, 0, X - 1), (T - 1, 0, Y - 1, 0)]
    for _ in range(n):
        pick.append((int(rng.integers(T)), int(rng.integers(Z)), int(rng.integers(Y)), int(rng.integers(X))))
    return pick


@pytest.mark.parametrize("name", ["tsm_16x16x16x32", "batched_24x24x24x48", "paper_32x32x32x64"])
def test_full_size_hop_sampled(ctx, name):
    w = synth.WORKLOADS[name]
    dims = w["dims"]
    log("full size hop", name)
    lat = make_lattice(ctx, dims, w["gauge_seed"], w["eps"], w["kappa"], w["mu"])
    psi = synth.random_spinor(dims, 8, nrhs=2)
    sites = _boundary_sites(dims, np.random.default_rng(0), 120)
    for tier, tol in [(dl.DL_TIER_FP64, 1e-13), (dl.DL_TIER_HP_FP32, 5e-7), (dl.DL_TIER_LP_BF16, 1.6e-2)]:
        out = zeros_dev(psi.shape)
        dl.dl_apply_op(lat.h, dl.DL_OP_HOP, tier, dev(psi), out, 2)
        got = host(out)
        for r in range(2):
            want = dirac.hop_at_sites(lat.U, psi[r], lat.bc, sites)
            g = np.array([got[r][s] for s in sites])
            assert rel(g, want) < tol, (tier, r, rel(g, want))
    lat.close()


def test_full_size_loops_from_gpu_solutions(ctx):
    """24^3 x 48, the bench's LP tier (bf16) and contraction kernels with two slots
    merged into one contraction launch (as the bench's slots are): the per-set loop sums at p = 0 equal the
    oracle's loops of the solutions the GPU returned.  Local tau_3 structure (s only,
    exact bf16 values, FP32 block sums): 1e-5; derivative insertions transport with
    the tier's bf16 links, and the structure without tau_3 reads xi = (1 - kappa H) s
    stored in bf16 (2^-9 rounding per element): 1.6e-2 and 2e-2."""
    w = synth.WORKLOADS["batched_24x24x24x48"]
    log("full size loops 24^3x48")
    lat = make_lattice(ctx, w["dims"], w["gauge_seed"], w["eps"], w["kappa"], w["mu"])
    nsrc, p2 = 2, 0                        # the oracle takes ~40 s per source here
    acc = dl.dl_accum_create(lat.h, dl.DL_OPS_LOCAL | dl.DL_OPS_DERIV)
    sol = zeros_dev((nsrc,) + lat.field_shape)
    rc, _ = dl.dl_solve_batch(ctx, dl.make_job(lat.h, noise=dl.DL_NOISE_Z4, tier=dl.DL_TIER_LP_BF16,
                                               seed=w["source_seed"], nsrc=nsrc, tol=1e-2, maxiter=500, rhs_block=1,
                                               sol_out=sol, accum=acc, accum_set=dl.DL_SET_LP))
    assert rc == dl.DL_OK
    sets = np.zeros((3, 2, 5, 16, lat.dims[3], 1), dtype=np.complex128)
    dl.dl_loops_sets(ctx, acc, p2, sets, 0)
    dl.dl_accum_destroy(acc)
    sols = host(sol)
    del sol
    want = 0
    for r in range(nsrc):
        want = want + loops.apply_prefactors(loops.source_loops(lat.U, sols[r], lat.kappa, lat.bc, p2, lat.dims),
                                             lat.kappa, lat.mu)
    for f in range(2):
        for op in range(5):
            tol = 2e-2 if f else (1e-5 if op == 0 else 1.6e-2)
            e = rel(sets[dl.DL_SET_LP, f, op], want[f, op])
            log("  flavour", f, "op", op, "rel err", e)
            assert e < tol, (f, op, e)
    lat.close()


def test_largest_size_tiers_true_residual(ctx):
    """32^3 x 64 (the volume of the paper's ensembles): bf16 LP and FP32 + reliable-update
    HP solves; the oracle's FP64 operator recomputes each returned solution's true
    residual, which must agree with the library's report and meet the tier's target."""
    w = synth.WORKLOADS["paper_32x32x32x64"]
    log("largest size tiers 32^3x64")
    lat = make_lattice(ctx, w["dims"], w["gauge_seed"], w["eps"], w["kappa"], w["mu"])
    for tier, tol in ((dl.DL_TIER_LP_BF16, 1e-2), (dl.DL_TIER_HP_FP32, 1e-8)):
        sol = zeros_dev((1,) + lat.field_shape)
        rc, stats = dl.dl_solve_batch(ctx, dl.make_job(lat.h, noise=dl.DL_NOISE_Z4, tier=tier, seed=w["source_seed"],
                                                       nsrc=1, tol=tol, maxiter=2000, report_true_resid=1,
                                                       sol_out=sol))
        assert rc == dl.DL_OK
        eta = noise.source(w["dims"], w["source_seed"], 0, noise.Z4)
        tr = solver.true_residual(lat.U, eta, host(sol)[0], lat.kappa, lat.mu, lat.bc)
        log("  tier", tier, "iters", stats[0].iters, "true resid", tr, "reported", stats[0].true_resid)
        assert abs(stats[0].true_resid - tr) < 1e-6 * tr + 1e-12
        # rho bounds the iterated normal-equation residual; the true one is looser
        assert tr < (5 if tier == dl.DL_TIER_LP_BF16 else 10) * tol, tr   # measured 1.03e-2, 8.8e-9
        del sol
    lat.close()


def test_full_size_fp64_solve_true_residual(ctx):
    """16^3 x 32 FP64 solve: the oracle's own operator confirms the residual."""
    w = synth.WORKLOADS["tsm_16x16x16x32"]
    lat = make_lattice(ctx, w["dims"], w["gauge_seed"], w["eps"], w["kappa"], w["mu"])
    sol = zeros_dev((1,) + lat.field_shape)
    job = dl.make_job(lat.h, noise=dl.DL_NOISE_Z2, tier=dl.DL_TIER_FP64, seed=w["source_seed"], nsrc=1, tol=1e-10,
                      maxiter=1000, report_true_resid=1, sol_out=sol)
    rc, stats = dl.dl_solve_batch(ctx, job)
    assert rc == dl.DL_OK
    eta = noise.source(w["dims"], w["source_seed"], 0, noise.Z2)
    tr = solver.true_residual(lat.U, eta, host(sol)[0], lat.kappa, lat.mu, lat.bc)
    log("16^3x32 fp64 iters", stats[0].iters, "true resid", tr)
    assert tr < 1e-9 and abs(stats[0].true_resid - tr) < 1e-3 * tr
    lat.close()


# ---------------------------------------------------------------------------
# edge cases and failure handling (conditions forced from the host)
# ---------------------------------------------------------------------------
def test_edge_cases(ctx):
    lat = make_lattice(ctx, (4, 4, 4, 4), 41, 0.3, 0.16, 0.01)
    # empty job
    rc, stats = dl.dl_solve_batch(ctx, dl.make_job(lat.h, nsrc=0))
    assert rc == dl.DL_OK and stats == []
    # zero source: converged at iteration 0, zero solution
    src = zeros_dev((1,) + lat.field_shape)
    sol = zeros_dev((1,) + lat.field_shape) + 1
    rc, stats = dl.dl_solve_batch(ctx, dl.make_job(lat.h, noise=dl.DL_NOISE_USER, src_in=src, sol_out=sol, nsrc=1))
    assert rc == dl.DL_OK and stats[0].iters == 0 and stats[0].status == dl.DL_SRC_CONVERGED
    assert np.abs(host(sol)).max() == 0
    # iteration cap
    rc, stats = dl.dl_solve_batch(ctx, dl.make_job(lat.h, nsrc=2, tol=1e-30, maxiter=1))
    assert rc == dl.DL_NOT_CONVERGED
    assert all(s.status == dl.DL_SRC_MAXITER and s.iters == 1 for s in stats)
    # NaN in a caller source: breakdown flagged, other sources unaffected
    bad = dev(np.stack([noise.source(lat.dims, 1, 0, noise.Z2), noise.source(lat.dims, 1, 1, noise.Z2)]))
    bad[1, 0, 0, 0, 0, 0, 0] = float("nan")
    rc, stats = dl.dl_solve_batch(ctx, dl.make_job(lat.h, noise=dl.DL_NOISE_USER, src_in=bad, nsrc=2, tol=1e-8))
    assert rc == dl.DL_NOT_CONVERGED
    assert stats[0].status == dl.DL_SRC_CONVERGED and stats[1].status == dl.DL_SRC_BREAKDOWN
    # invalid arguments
    with pytest.raises(dl.DiscloopError) as e:
        dl.dl_lattice_create(ctx, (4, 4, 3, 4))
    assert e.value.code == dl.DL_EINVAL
    with pytest.raises(dl.DiscloopError):
        dl.dl_set_params(lat.h, 0.16, float("nan"))
    with pytest.raises(dl.DiscloopError):
        dl.dl_solve_batch(ctx, dl.make_job(lat.h, nsrc=1, tol=-1))
    # LPC set must mirror the HP set
    acc = dl.dl_accum_create(lat.h, dl.DL_OPS_LOCAL)
    dl.dl_solve_batch(ctx, [dl.make_job(lat.h, nsrc=2, tol=1e-8, accum=acc, accum_set=dl.DL_SET_HP),
                            dl.make_job(lat.h, nsrc=1, tol=1e-2, accum=acc, accum_set=dl.DL_SET_LPC)])
    out = np.zeros((2, 1, 16, 4, 27), dtype=np.complex128)
    with pytest.raises(dl.DiscloopError):
        dl.dl_loops(ctx, acc, 3, out, 0)
    dl.dl_accum_reset(acc)
    assert dl.dl_accum_counts(acc) == [0, 0, 0]
    dl.dl_accum_destroy(acc)
    lat.close()
