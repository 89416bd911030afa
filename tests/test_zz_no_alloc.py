"""dl_loops_noalloc: the projection with no device allocation, against dl_loops.

Both entry points run the same kernels in the same order on the same
accumulators, so their outputs must agree bit for bit.  Two calls in a row on
the same GPU (the second one smaller) check that nothing of the first call's
scratch contents leaks into the second.  A projection larger than the scratch
array is refused on the host, before any GPU work.
"""
import sys

import numpy as np
import pytest

import paper_1401_6750_amd as dl
from oracle import loops
from tests.gpu_util import host, make_lattice, torch, zeros_dev

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


def _tsm_accum(ctx, lat, ops, seed):
    """An accumulator with all three TSM sets filled (bf16 LP, FP32 HP, bf16 LPC)."""
    acc = dl.dl_accum_create(lat.h, ops)
    n_lp, n_hp = 6, 2
    jobs = [
        dl.make_job(lat.h, noise=dl.DL_NOISE_Z4, tier=dl.DL_TIER_LP_BF16, seed=seed, first_src=0, nsrc=n_lp,
                    tol=1e-2, maxiter=200, accum=acc, accum_set=dl.DL_SET_LP),
        dl.make_job(lat.h, noise=dl.DL_NOISE_Z4, tier=dl.DL_TIER_LP_BF16, seed=seed, first_src=n_lp, nsrc=n_hp,
                    tol=1e-2, maxiter=200, accum=acc, accum_set=dl.DL_SET_LPC),
        dl.make_job(lat.h, noise=dl.DL_NOISE_Z4, tier=dl.DL_TIER_HP_FP32, seed=seed, first_src=n_lp, nsrc=n_hp,
                    tol=1e-8, maxiter=500, accum=acc, accum_set=dl.DL_SET_HP),
    ]
    dl.dl_solve_batch(ctx, jobs)
    return acc


def _both(ctx, lat, acc, p2max, nops):
    np_ = len(loops.momenta(p2max, lat.dims))
    shape = (2, nops, 16, lat.dims[3], np_)
    ref = zeros_dev(shape)
    got = zeros_dev(shape).fill_(complex(float("nan"), float("nan")))
    assert dl.dl_loops(ctx, acc, p2max, ref, 1) == np_
    assert dl.dl_loops_noalloc(ctx, acc, p2max, got) == np_
    torch().cuda.synchronize()
    return host(got), host(ref)


def test_noalloc_equals_dl_loops_two_calls(ctx):
    """Large call (derivatives, p^2 <= 4, 8x6x6x8), then a smaller one (local, p^2 <= 1,
    4^4), then an expansion accumulator: each bit-identical to dl_loops."""
    cases = [((8, 6, 6, 8), dl.DL_OPS_LOCAL | dl.DL_OPS_DERIV, 4, 5),
             ((4, 4, 4, 4), dl.DL_OPS_LOCAL, 1, 1),
             ((4, 4, 4, 4), dl.DL_OPS_LOCAL | dl.DL_OPS_DERIV | dl.DL_OPS_HPE(2), 3, 5)]
    for i, (dims, ops, p2, nops) in enumerate(cases):
        log(f"no-alloc case {i}: dims {dims} ops {ops} p2max {p2}")
        lat = make_lattice(ctx, dims, 1401 + i, 0.2, 0.1615, 0.004)
        acc = _tsm_accum(ctx, lat, ops, 6750 + i)
        got, ref = _both(ctx, lat, acc, p2, nops)
        assert np.isfinite(ref).all()
        assert np.array_equal(got, ref), np.abs(got - ref).max()
        assert np.abs(ref).max() > 0
        dl.dl_accum_destroy(acc)
        lat.close()


def test_noalloc_refuses_oversized_projection(ctx):
    """24^3 x 48 with derivatives at p^2 <= 9 needs about 128 MB of scratch: DL_EINVAL,
    the output left untouched; the same accumulator at p^2 <= 4 fits."""
    dims = (24, 24, 24, 48)
    lat = dl.dl_lattice_create(ctx, dims, -1)
    dl.dl_set_params(lat, 0.1615, 0.004)
    acc = dl.dl_accum_create(lat, dl.DL_OPS_LOCAL | dl.DL_OPS_DERIV)
    np9 = len(loops.momenta(9, dims))
    out = zeros_dev((2, 5, 16, dims[3], np9))
    with pytest.raises(dl.DiscloopError) as e:
        dl.dl_loops_noalloc(ctx, acc, 9, out)
    assert e.value.code == dl.DL_EINVAL and "scratch" in str(e.value)
    torch().cuda.synchronize()
    assert float(out.abs().max()) == 0.0
    # an empty accumulator projects to zeros through the fill kernel
    np4 = len(loops.momenta(4, dims))
    out4 = zeros_dev((2, 5, 16, dims[3], np4)).fill_(1.0)
    assert dl.dl_loops_noalloc(ctx, acc, 4, out4) == np4
    torch().cuda.synchronize()
    assert float(out4.abs().max()) == 0.0
    dl.dl_accum_destroy(acc)
    dl.dl_lattice_destroy(lat)
