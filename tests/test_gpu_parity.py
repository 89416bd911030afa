"""GPU parity of the HIP path against the FP64 oracle, through the C ABI.

Tolerances: integer work (noise) is bit-exact.  FP64 operators agree to
1e-13 relative (rounding order only); FP64 solves and loops to 1e-10 relative
(the FP64 solve requirement); the storage-precision operators to a few units
of their storage roundoff u (fp32 2^-24, fp16 2^-11, bf16 2^-8):
5e-7, 2e-3 and 1.6e-2 relative L2.  Loops are compared element by element
(gpu_util.elementwise: every (flavour, op, Gamma, t, p) entry within
rtol |want| + atol max|block|), with bounds a few times the measured error.
"""
import sys

import os

import numpy as np
import pytest

import paper_1401_6750_amd as dl
import synth
from oracle import dirac, loops, noise, solver
from tests.gpu_util import Lattice, dev, elementwise, elementwise_check, host, make_lattice, rel, torch, zeros_dev

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


@pytest.mark.parametrize("dims,seed,eps", [((4, 4, 4, 4), 1401, 0.3), ((6, 2, 4, 8), 21, 0.2)])
def test_gauge_random_loads_the_synthetic_field(ctx, dims, seed, eps):
    """dl_gauge_random builds the same links on the library side as the Python synthetic
    generator: every operator equals the oracle's on synth.random_gauge to 1e-13."""
    lat = make_lattice(ctx, dims, seed, eps, 0.15, 0.03)
    dl.dl_gauge_random(lat.h, seed, eps)
    psi = synth.random_spinor(dims, 4, nrhs=2)
    for op in OPS:
        out = zeros_dev(psi.shape)
        dl.dl_apply_op(lat.h, op, dl.DL_TIER_FP64, dev(psi), out, 2)
        torch().cuda.synchronize()
        assert rel(host(out), oracle_op(lat, op, psi)) < 1e-13, op
    lat.close()


@pytest.mark.parametrize("tier,tol", [(dl.DL_TIER_HP_FP32, 5e-7), (dl.DL_TIER_LP_FP16, 2e-3),
                                      (dl.DL_TIER_LP_BF16, 1.6e-2)])
@pytest.mark.parametrize("dims", [(6, 4, 4, 8), (4, 4, 4, 4), (6, 6, 6, 6), (2, 4, 6, 8), (8, 2, 2, 4), (2, 2, 2, 2)])
@pytest.mark.parametrize("bc", [-1, 1])
def test_operators_storage_precision(ctx, tier, tol, dims, bc):
    log("ops", tier, dims, bc)
    lat = make_lattice(ctx, dims, 12, 0.3, 0.16, 0.02, bc)
    psi = synth.random_spinor(dims, 6, nrhs=2)
    for op in OPS:
        out = zeros_dev(psi.shape)
        dl.dl_apply_op(lat.h, op, tier, dev(psi), out, 2)
        torch().cuda.synchronize()
        e = rel(host(out), oracle_op(lat, op, psi))
        log("  op", op, "rel err", e)
        assert e < tol, (op, e)
    lat.close()


def test_two_row_links_follow_the_upload_check(ctx):
    """Which hops rebuild row 2 of the links: the upload check sets it per
    storage class (1e-6 for the 16-bit hops, 1e-7 for the FP32 ones).  Row 2
    of every link is moved by d off the SU(3) identity; a hop that rebuilds it
    never reads it, so its result is bit-identical to the unperturbed field's,
    and a hop that reads it sees the change."""
    dims = (6, 4, 4, 8)
    U = synth.random_gauge(dims, 41, 0.3)
    psi = synth.random_spinor(dims, 9, nrhs=2)

    def hop(Uf, tier):
        lat = Lattice(ctx, dims, Uf, 0.16, 0.02, -1)
        out = zeros_dev(psi.shape)
        dl.dl_apply_op(lat.h, dl.DL_OP_HOP, tier, dev(psi), out, 2)
        torch().cuda.synchronize()
        got = host(out)
        want = oracle_op(lat, dl.DL_OP_HOP, psi)
        lat.close()
        return got, want

    def moved(d):
        V = U.copy()
        V[..., 2, :] += d * (1 + 1j)
        return V

    b16, _ = hop(U, dl.DL_TIER_LP_BF16)
    b32, _ = hop(U, dl.DL_TIER_HP_FP32)
    for d, rebuilt16, rebuilt32 in ((3e-8, True, True), (3e-7, True, False), (1e-3, False, False)):
        g16, w16 = hop(moved(d), dl.DL_TIER_LP_BF16)
        g32, w32 = hop(moved(d), dl.DL_TIER_HP_FP32)
        log("row 2 moved by", d, "bf16 rel", rel(g16, w16), "fp32 rel", rel(g32, w32))
        assert np.array_equal(g16, b16) == rebuilt16, d
        assert np.array_equal(g32, b32) == rebuilt32, d
        assert rel(g16, w16) < 1.6e-2 and rel(g32, w32) < (5e-7 if not rebuilt32 else 5e-7 + 4 * d)


@pytest.mark.parametrize("tier,tol", [(dl.DL_TIER_LP_FP16, 2e-3), (dl.DL_TIER_LP_BF16, 1.6e-2)])
def test_operators_16bit_links_not_special_unitary(ctx, tier, tol):
    """Links in U(3) but not SU(3) (a random phase per link, so row 2 is not
    conj(row 0 x row 1)): the 16-bit hop must read all nine stored entries
    instead of rebuilding row 2.  A rebuilt row would be off by the phase,
    an O(1) error; the bound is that of SU(3) links."""
    dims = (6, 4, 4, 8)
    U = synth.random_gauge(dims, 31, 0.3)
    rng = np.random.default_rng(5)
    U = U * np.exp(1j * rng.uniform(-np.pi, np.pi, U.shape[:-2]))[..., None, None]
    lat = Lattice(ctx, dims, U, 0.16, 0.02, -1)
    psi = synth.random_spinor(dims, 8, nrhs=2)
    for op in OPS:
        out = zeros_dev(psi.shape)
        dl.dl_apply_op(lat.h, op, tier, dev(psi), out, 2)
        torch().cuda.synchronize()
        e = rel(host(out), oracle_op(lat, op, psi))
        log("  U(3) op", op, "rel err", e)
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
        log("  p2", p2, "worst element error / block max", elementwise(out, want, 1e-10, 1e-10, 3))
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
    elementwise(out, loops.estimate(per, lat.kappa, lat.mu), 1e-10, 1e-10, 3)
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
    log("tsm combination worst element error / block max", elementwise(out, want, 1e-9, 1e-9, 3))
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
    elementwise(sets[0] / 6 + (sets[1] - sets[2]) / 3, est, 1e-12, 1e-12, 3)
    want_hp = loops.apply_prefactors(sum(
        loops.source_loops(lat.U, solver.cgnr_eo(lat.U, noise.source(lat.dims, seed, r, noise.Z4), lat.kappa,
                                                 lat.mu, lat.bc, lat.dims, 1e-10)[0], lat.kappa, lat.bc, p2, lat.dims)
        for r in range(6, 9)), lat.kappa, lat.mu)
    elementwise(sets[1], want_hp, 1e-9, 1e-9, 3)
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
    elementwise(st.estimate(5), loops.estimate(np.stack(per), lat.kappa, lat.mu), 1e-9, 1e-9, 3)
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
            assert tr < 20 * tol and err < 1e-7          # measured err 1.5e-8
        else:
            assert tr < 6 * tol and err < 5e-2           # measured err 1.7e-2
    lat.close()


def _loop_sets(ctx, acc, p2, dims, nops=5):
    npm = len(loops.momenta(p2, dims))
    sets = np.zeros((3, 2, nops, 16, dims[3], npm), dtype=np.complex128)
    dl.dl_loops_sets(ctx, acc, p2, sets, 0)
    return sets


def _oracle_set(lat, sols, p2, deriv=True):
    """Prefactored sum over the given solutions of the oracle's per-source loops."""
    tot = 0
    for s in sols:
        tot = tot + loops.source_loops(lat.U, s, lat.kappa, lat.bc, p2, lat.dims, deriv=deriv)
    return loops.apply_prefactors(tot, lat.kappa, lat.mu)


@pytest.mark.parametrize("block", [5, 2])
def test_hp_tier_loops_match_oracle_on_gpu_solutions(ctx, block):
    """The high-precision tier (FP32 + FP64 reliable updates, the TSM correction tier of
    Section 2.1) contracts its FP64 solution with FP64 products and per-source FP64 sums:
    its loop set equals the oracle's loops of the solutions it returned, both flavour
    structures (xi = gamma_5 s and xi = (1 - kappa H) s), local and derivative, element by
    element to 1e-10."""
    dims = (6, 4, 6, 6)
    lat = make_lattice(ctx, dims, 1406, 0.3, 0.15, 0.02)
    nsrc, p2 = 5, 3
    acc = dl.dl_accum_create(lat.h, dl.DL_OPS_LOCAL | dl.DL_OPS_DERIV)
    sol = zeros_dev((nsrc,) + lat.field_shape)
    rc, stats = dl.dl_solve_batch(ctx, dl.make_job(lat.h, noise=dl.DL_NOISE_Z4, tier=dl.DL_TIER_HP_FP32, seed=17,
                                                   nsrc=nsrc, tol=1e-8, maxiter=2000, rhs_block=block,
                                                   sol_out=sol, accum=acc, accum_set=dl.DL_SET_HP))
    assert rc == dl.DL_OK
    sets = _loop_sets(ctx, acc, p2, dims)
    dl.dl_accum_destroy(acc)
    want = _oracle_set(lat, host(sol), p2)
    w = elementwise(sets[dl.DL_SET_HP], want, 1e-10, 1e-10, 3)
    log(f"HP tier loops vs oracle on the GPU's solutions (block {block}): worst |d|/max|block| {w:.2e}")
    assert np.abs(sets[dl.DL_SET_LP]).max() == 0 and np.abs(sets[dl.DL_SET_LPC]).max() == 0
    lat.close()


def test_tier_loop_error_against_exact(ctx):
    """Each tier's loops against the FP64 oracle's loops of the exact solutions of the same
    sources, at the LP (1e-2) and HP (1e-8) target residuals: the error the truncated solver
    method corrects (LP) and the one it leaves (HP).  The bounds are a few times the
    measured worst |d| / max|block| per tier."""
    dims = (8, 8, 8, 8)
    lat = make_lattice(ctx, dims, 1405, 0.2, 0.1615, 0.004)
    nsrc, p2, seed = 4, 1, 3
    exact = [solver.cgnr_eo(lat.U, noise.source(dims, seed, r, noise.Z2), lat.kappa, lat.mu, lat.bc, dims,
                            1e-13)[0] for r in range(nsrc)]
    want = _oracle_set(lat, exact, p2)
    bounds = {dl.DL_TIER_LP_BF16: (1e-2, 0.3), dl.DL_TIER_LP_FP16: (1e-2, 0.3), dl.DL_TIER_HP_FP32: (1e-8, 1e-6),
              dl.DL_TIER_FP64: (1e-8, 1e-6)}
    for tier, (rho, bound) in bounds.items():
        acc = dl.dl_accum_create(lat.h, dl.DL_OPS_LOCAL | dl.DL_OPS_DERIV)
        rc, _ = dl.dl_solve_batch(ctx, dl.make_job(lat.h, noise=dl.DL_NOISE_Z2, tier=tier, seed=seed, nsrc=nsrc,
                                                   tol=rho, maxiter=2000, accum=acc, accum_set=dl.DL_SET_HP))
        assert rc == dl.DL_OK
        got = _loop_sets(ctx, acc, p2, dims)[dl.DL_SET_HP]
        dl.dl_accum_destroy(acc)
        worst = {}
        for f in range(2):
            for op in range(5):
                worst[(f, op)] = elementwise(got[f, op], want[f, op], 0.0, bound, 1)
        log(f"tier {tier} rho {rho}: loop error vs exact-solve loops (worst |d|/max|block|, "
            f"(flavour, op)): " + ", ".join(f"{k}: {v:.2e}" for k, v in worst.items()))
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
        # the LDS-staged hop keys its own shapes (":blk"); write both
        cache.write_text(json.dumps({"8x8x8x8:bf16:16": blk, "8x8x8x8:bf16:16:t": tb,
                                     "8x8x8x8:bf16:16:blk": blk, "8x8x8x8:bf16:16:blk:t": tb}))
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


def test_contraction_tile_order_does_not_change_loops():
    """The derivative contraction's time-blocked tile order (option contract_tblk) only reorders
    work over sites whose accumulators are independent: the loops are bit-identical for 1, 2, 3
    and 8 slices per block (8^4 has whole tiles per time slice, so the blocked order is used;
    3 leaves a partial block at the end)."""
    t = torch()
    ref = None
    for tb in (1, 2, 3, 8):
        c = dl.dl_create(0, t.cuda.current_stream().cuda_stream)
        dl.dl_set_option(c, "contract_tblk", tb)
        lat = make_lattice(c, (8, 8, 8, 8), 43, 0.2, 0.1615, 0.004)
        acc = dl.dl_accum_create(lat.h, dl.DL_OPS_LOCAL | dl.DL_OPS_DERIV)
        rc, _ = dl.dl_solve_batch(c, dl.make_job(lat.h, noise=dl.DL_NOISE_Z4, tier=dl.DL_TIER_LP_BF16, seed=7,
                                                 nsrc=12, tol=1e-2, maxiter=200, rhs_block=4, accum=acc,
                                                 accum_set=dl.DL_SET_HP))
        assert rc == dl.DL_OK
        out = np.zeros((2, 5, 16, 8, 7), dtype=np.complex128)
        assert dl.dl_loops(c, acc, 1, out, 0) == 7
        dl.dl_accum_destroy(acc)
        lat.close()
        dl.dl_destroy(c)
        if ref is None:
            ref = out
        assert np.array_equal(out, ref), tb
    assert np.abs(ref).max() > 0
    c = dl.dl_create(0, t.cuda.current_stream().cuda_stream)
    try:
        with pytest.raises(dl.DiscloopError):
            dl.dl_set_option(c, "contract_tblk", 0)
    finally:
        dl.dl_destroy(c)


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


@pytest.mark.parametrize("dims", [(6, 6, 6, 6), (8, 8, 8, 8), (12, 4, 8, 6), (16, 8, 4, 4)])
def test_block_hop_option(dims):
    """The LDS-staged 16-bit hop (option block_hop) does the tile kernel's per-site arithmetic:
    every 16-bit operator gives the same bits.  Its low-precision solves sum the norms per
    (block, slice), so their iterates are its own: the LP map is the same for every slot size,
    and the solutions meet the tier's accuracy against the oracle."""
    t = torch()
    lat_args = (dims, 27, 0.3, 0.16, 0.02)
    psi = synth.random_spinor(dims, 8, nrhs=3)
    outs = {}
    for opt in (0, 1):
        c = dl.dl_create(0, t.cuda.current_stream().cuda_stream)
        dl.dl_set_option(c, "block_hop", opt)
        lat = make_lattice(c, *lat_args)
        for tier in (dl.DL_TIER_LP_BF16, dl.DL_TIER_LP_FP16):
            for op in OPS:
                out = zeros_dev(psi.shape)
                dl.dl_apply_op(lat.h, op, tier, dev(psi), out, 3)
                t.cuda.synchronize()
                outs[(opt, tier, op)] = host(out)
        if opt == 1:
            sols = []
            for blk in (6, 4, 1):
                sol = zeros_dev((6,) + lat.field_shape)
                rc, st = dl.dl_solve_batch(c, dl.make_job(lat.h, noise=dl.DL_NOISE_Z4, tier=dl.DL_TIER_LP_BF16,
                                                          seed=17, nsrc=6, tol=1e-2, maxiter=500, rhs_block=blk,
                                                          sol_out=sol))
                assert rc == dl.DL_OK
                sols.append((host(sol), [x.iters for x in st]))
            assert all(np.array_equal(sols[0][0], x[0]) and sols[0][1] == x[1] for x in sols[1:])
            for r in range(6):
                eta = noise.source(dims, 17, r, noise.Z4)
                tr = solver.true_residual(lat.U, eta, sols[0][0][r], lat.kappa, lat.mu, lat.bc)
                log(f"block hop {dims} LP source {r}: iters {sols[0][1][r]} true residual {tr:.3e}")
                assert tr < 5e-2
        lat.close()
        dl.dl_destroy(c)
    for (opt, tier, op), v in outs.items():
        if opt == 1:
            assert np.array_equal(v, outs[(0, tier, op)]), (tier, op)


def test_hp_graph_equals_host_driven(ctx):
    """The high-precision tier replayed from a graph (reliable-update decisions on the
    device) gives the same bits as the host-driven loop: solutions, iteration and
    reliable-update counts, residuals, status and loops; with and without LP starting
    guesses, at a tolerance that forces restarts from the true residual, and at an
    iteration cap."""
    lat = make_lattice(ctx, (8, 8, 8, 8), 26, 0.2, 0.1615, 0.004)
    n = 6
    cases = [dict(tol=1e-8, maxiter=2000, guess=True), dict(tol=1e-10, maxiter=2000, guess=False),
             dict(tol=1e-8, maxiter=6, guess=False)]
    for cs in cases:
        runs = []
        for use_graph in (1, 0):
            dl.dl_set_option(ctx, "use_graph", use_graph)
            sol = zeros_dev((n,) + lat.field_shape)
            acc = dl.dl_accum_create(lat.h, dl.DL_OPS_LOCAL | dl.DL_OPS_DERIV)
            hp = dl.make_job(lat.h, noise=dl.DL_NOISE_Z4, tier=dl.DL_TIER_HP_FP32, seed=8, nsrc=n, tol=cs["tol"],
                             maxiter=cs["maxiter"], rhs_block=4, sol_out=sol, accum=acc, accum_set=dl.DL_SET_HP,
                             guess_from=2 if cs["guess"] else 0)
            jobs = [hp]
            if cs["guess"]:
                jobs = [hp, dl.make_job(lat.h, noise=dl.DL_NOISE_Z4, tier=dl.DL_TIER_LP_BF16, seed=8, nsrc=n,
                                        tol=1e-2, maxiter=500)]
            rc, st = dl.dl_solve_batch(ctx, jobs)
            out = np.zeros((2, 5, 16, 8, 1), dtype=np.complex128)
            dl.dl_loops(ctx, acc, 0, out, 0)
            dl.dl_accum_destroy(acc)
            runs.append((rc, host(sol), [(x.iters, x.status, x.reliable_updates, x.rel_resid) for x in st[:n]], out))
        dl.dl_set_option(ctx, "use_graph", 1)
        (rg, sg, tg, lg), (rp, sp, tp, lp) = runs
        log(f"hp graph vs host {cs}: rc {rg} stats {tg}")
        assert rg == rp and tg == tp
        assert np.array_equal(sg, sp) and np.array_equal(lg, lp)
        if cs["maxiter"] == 6:
            assert rg == dl.DL_NOT_CONVERGED and all(t[1] == dl.DL_SRC_MAXITER for t in tg)
        else:
            assert rg == dl.DL_OK and all(t[1] == dl.DL_SRC_CONVERGED for t in tg)
            assert all(t[2] >= 1 for t in tg)
    lat.close()


# fp16 loops against the oracle on the same solutions, per (flavour, derivative?)
UNEVEN_FP16_TOL = {(0, False): 1e-5, (0, True): 2e-3, (1, False): 2e-3, (1, True): 2e-3}


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
        # and both equal the oracle's loops of the fp16 solutions the batch returned: the
        # contraction rounds (1 - kappa H) s and the transported vectors to fp16 (2^-11)
        want = loops.estimate(np.array([loops.source_loops(l.U, x, l.kappa, l.bc, 2, l.dims)
                                        for x in host(s)]), l.kappa, l.mu)
        w = [elementwise(o1[f, op], want[f, op], 0.0, UNEVEN_FP16_TOL[(f, op > 0)], 1)
             for f in range(2) for op in range(5)]
        log(f"uneven batch {l.dims}: fp16 loops vs oracle on the batch's solutions, worst |d|/max|block| "
            f"per (flavour, op) {['%.1e' % x for x in w]}")
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


# Element-wise bounds of the 16-bit LP tier's loops against the oracle on the same
# solutions, per (flavour, derivative?): (atol, nblock) for gpu_util.elementwise.  The
# tau_3 local block multiplies stored bf16 values exactly (FP32 sums of 64 sources),
# checked per Gamma block.  The derivative insertions transport with the tier's bf16
# links and round the transported vector to bf16; the structure without tau_3 reads
# xi = (1 - kappa H) s built with bf16 links and stored in bf16.  Those rounding errors
# enter all 16 Gamma of one (flavour, op) with one absolute scale, that of the fields,
# so for the structure without tau_3, whose gamma_5-like blocks are a few hundred
# times smaller than its scalar block, the scale is the (flavour, op) maximum over
# Gamma, t and p (nblock 2 on [2][5][16][T][Np]).  Bounds are about 3x the measured
# worst |d| / m.
FULL_BF16_TOL = {(0, False): (2e-7, 3), (0, True): (8e-3, 3), (1, False): (1e-3, 2), (1, True): (1e-3, 2)}


@pytest.mark.timeout(900)
def test_full_size_loops_all_sets_from_gpu_solutions(ctx):
    """24^3 x 48 at p^2 <= 4, the benchmark's configuration in miniature: bf16 LP solves
    (two one-rhs slots merged into one contraction launch), an FP32 + reliable-update HP
    solve started from its LPC solution, and that LPC solve.  Each set's projected sum
    equals the oracle's loops of the solutions the GPU returned, element by element
    (the HP set, contracted in FP64, to 1e-10)."""
    from concurrent.futures import ThreadPoolExecutor
    w = synth.WORKLOADS["batched_24x24x24x48"]
    log("full size loops 24^3x48, p^2 <= 4, LP / HP / LPC sets")
    lat = make_lattice(ctx, w["dims"], w["gauge_seed"], w["eps"], w["kappa"], w["mu"])
    p2, seed = 4, w["source_seed"]
    acc = dl.dl_accum_create(lat.h, dl.DL_OPS_LOCAL | dl.DL_OPS_DERIV)
    s_lp = zeros_dev((2,) + lat.field_shape)
    s_lpc = zeros_dev((1,) + lat.field_shape)
    s_hp = zeros_dev((1,) + lat.field_shape)
    jobs = [dl.make_job(lat.h, noise=dl.DL_NOISE_Z4, tier=dl.DL_TIER_LP_BF16, seed=seed, first_src=0, nsrc=2,
                        tol=1e-2, maxiter=500, rhs_block=1, sol_out=s_lp, accum=acc, accum_set=dl.DL_SET_LP),
            dl.make_job(lat.h, noise=dl.DL_NOISE_Z4, tier=dl.DL_TIER_LP_BF16, seed=seed, first_src=2, nsrc=1,
                        tol=1e-2, maxiter=500, sol_out=s_lpc, accum=acc, accum_set=dl.DL_SET_LPC),
            dl.make_job(lat.h, noise=dl.DL_NOISE_Z4, tier=dl.DL_TIER_HP_FP32, seed=seed, first_src=2, nsrc=1,
                        tol=1e-8, maxiter=2000, sol_out=s_hp, accum=acc, accum_set=dl.DL_SET_HP, guess_from=2)]
    rc, _ = dl.dl_solve_batch(ctx, jobs)
    assert rc == dl.DL_OK
    sets = _loop_sets(ctx, acc, p2, lat.dims)
    dl.dl_accum_destroy(acc)
    sols = [host(s_lp)[0], host(s_lp)[1], host(s_lpc)[0], host(s_hp)[0]]
    del s_lp, s_lpc, s_hp
    log("  oracle loops of 4 solutions (threads)")
    with ThreadPoolExecutor(4) as ex:
        per = list(ex.map(lambda x: loops.source_loops(lat.U, x, lat.kappa, lat.bc, p2, lat.dims), sols))
    pre = lambda x: loops.apply_prefactors(x, lat.kappa, lat.mu)
    want = {dl.DL_SET_LP: pre(per[0] + per[1]), dl.DL_SET_LPC: pre(per[2]), dl.DL_SET_HP: pre(per[3])}
    failed = []
    for k, name in ((dl.DL_SET_LP, "LP"), (dl.DL_SET_LPC, "LPC")):
        for f in range(2):
            for op in range(5):
                atol, nb = FULL_BF16_TOL[(f, op > 0)]
                # blocks of nblock leading axes of [2][5][16][T][Np]
                e, idx, nbad = elementwise_check(sets[k][f:f + 1, op:op + 1], want[k][f:f + 1, op:op + 1], 0.0,
                                                 atol, nb)
                log(f"  {name} flavour {f} op {op}: worst |d|/m {e:.2e} (blocks of {nb} axes, bound {atol:g})")
                if nbad:
                    failed.append((name, f, op, e, idx))
    assert not failed, failed
    e = elementwise(sets[dl.DL_SET_HP], want[dl.DL_SET_HP], 1e-10, 1e-10, 3)
    log(f"  HP (FP64 contraction): worst |d|/max|block| {e:.2e}")
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
    # more than 2^28 sites per parity (the kernels' 32-bit row offsets): refused
    # before anything is allocated
    with pytest.raises(dl.DiscloopError) as e:
        dl.dl_lattice_create(ctx, (512, 512, 512, 4))
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
    # LP and HP sets without the LPC set: S_LP/N_LP + S_HP/N_HP is no estimator
    dl.dl_solve_batch(ctx, [dl.make_job(lat.h, nsrc=2, tol=1e-2, accum=acc, accum_set=dl.DL_SET_LP),
                            dl.make_job(lat.h, first_src=2, nsrc=1, tol=1e-8, accum=acc, accum_set=dl.DL_SET_HP)])
    with pytest.raises(dl.DiscloopError) as e:
        dl.dl_loops(ctx, acc, 3, out, 0)
    assert "LPC" in str(e.value)
    dl.dl_solve_batch(ctx, dl.make_job(lat.h, first_src=2, nsrc=1, tol=1e-2, accum=acc, accum_set=dl.DL_SET_LPC))
    dl.dl_loops(ctx, acc, 3, out, 0)
    dl.dl_accum_destroy(acc)
    lat.close()
