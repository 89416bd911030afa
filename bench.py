#!/usr/bin/env python3
"""Benchmark of the truncated-solver-method fermion-loop pipeline on one MI355X.

One step = the whole hot path on one synthetic gauge field: N_LP
low-precision Z4 solves (bf16 storage, FP32 arithmetic, rho = 1e-2), N_HP
high-precision solves (FP32 with FP64 reliable updates, rho = 1e-8), the
low-precision solves of the same N_HP sources, one-end-trick contractions of
all 160 local and one-derivative insertions accumulated in FP64 on the GPU,
and the momentum projection (p^2 <= 4) with the TSM combination.  Inputs are
resident on the GPU before timing starts; the loops stay in device memory.

Prints one JSON line: the metric, the roofline of the dominant hopping kernel,
the same-accuracy comparison with the plain FP64 path and the oracle baseline
timed on the host cores.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "TSM LP solves/s + dslash HBM GB/s at rho=1e-2/1e-8 vs plain FP64 GPU path"
HBM_PEAK_GBS = 8000.0
COUNTERS = os.path.join(ROOT, "profiles", "dslash_bf16_24x24x24x48_counters.json")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_1401_6750_amd", "csrc", f) for f in ("dslash.hip", "common.h")]

WORKLOADS = {
    # lattice name -> TSM sizes
    "batched_24x24x24x48": dict(n_lp=1000, n_hp=50, p2max=4, noise="Z4"),
    "tsm_16x16x16x32": dict(n_lp=200, n_hp=10, p2max=4, noise="Z2"),
    # not TSM steps of one lattice: see bench_uneven / bench_grad / bench_sweep
    "uneven": None,
    "uneven_small": None,
    "grad_16x16x16x32": None,
    "dslash_sweep": None,
    "tsm_error_16x16x16x32": None,
}

# serving-shaped mix of lattices: (dims, eps, LP sources); kappa 0.1615, mu 0.004
UNEVEN = [((8, 8, 8, 8), 0.1, 64), ((8, 8, 8, 8), 0.3, 4), ((16, 16, 16, 32), 0.2, 32),
          ((16, 16, 16, 32), 0.1, 8), ((24, 24, 24, 48), 0.3, 16), ((24, 24, 24, 48), 0.2, 4)]
# many small lattices, where one call per lattice is launch-bound
UNEVEN_SMALL = [((8, 8, 8, 8), round(0.1 + 0.05 * (i % 4), 2), 8 + 8 * (i % 3)) for i in range(8)] + \
               [((12, 12, 12, 12), 0.2, 16), ((12, 12, 12, 24), 0.2, 8), ((16, 16, 16, 16), 0.2, 8),
                ((8, 8, 8, 16), 0.3, 24)]


def _setup_lattice(dl, torch, synth, ctx, dims, seed, eps, kappa, mu):
    import numpy as np
    U = synth.random_gauge(dims, seed, eps)
    lat = dl.dl_lattice_create(ctx, dims, -1)
    dl.dl_gauge_set(lat, torch.from_numpy(np.ascontiguousarray(U)).to("cuda"), 1)
    dl.dl_set_params(lat, kappa, mu)
    return lat, U


def copy_gbs(torch, gib: int = 4, reps: int = 5) -> float:
    """Achieved bandwidth of a plain device-to-device copy (read + write bytes / time)."""
    x = torch.empty(gib << 28, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    y.copy_(x)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        y.copy_(x)
    e1.record()
    e1.synchronize()
    ms = e0.elapsed_time(e1)
    del x, y
    return 2.0 * (gib << 30) * reps / (ms * 1e-3) / 1e9


def bench_sweep(a) -> int:
    """Hopping-kernel bandwidth per storage precision and number of right-hand
    sides on the 24^3x48 lattice: each configuration solves nsrc sources (LP
    tiers and FP64 to rho = 1e-2, HP to 1e-8) with the kernel profiled; GB/s =
    algorithmic bytes of the u_e = A^-1 H_eo p_o launches / their HIP-event
    time.  One JSON line per configuration, then the plain-copy bandwidth."""
    import torch

    import paper_1401_6750_amd as dl
    import synth

    w = synth.WORKLOADS["batched_24x24x24x48"]
    ctx = dl.dl_create(0, torch.cuda.current_stream().cuda_stream)
    dl.dl_set_option(ctx, "inflight_mb", a.inflight_mb)
    lat, _ = _setup_lattice(dl, torch, synth, ctx, w["dims"], w["gauge_seed"], w["eps"], w["kappa"], w["mu"])
    tiers = [("bf16", dl.DL_TIER_LP_BF16, 1e-2, [1, 8, 64, 512]), ("fp16", dl.DL_TIER_LP_FP16, 1e-2, [1, 8, 64, 512]),
             ("fp32", dl.DL_TIER_HP_FP32, 1e-8, [1, 8, 64]), ("fp64", dl.DL_TIER_FP64, 1e-2, [1, 8, 64])]
    for name, tier, tol, ns in tiers:
        for n in ns:
            job = dl.make_job(lat, noise=dl.DL_NOISE_Z4, tier=tier, seed=w["source_seed"], nsrc=n, tol=tol,
                              maxiter=2000)
            dl.dl_solve_batch(ctx, job)               # tuning and warm-up
            dl.dl_profile_read(ctx, tier)
            dl.dl_set_option(ctx, "profile", 1)
            dl.dl_solve_batch(ctx, job)
            torch.cuda.synchronize()
            dl.dl_set_option(ctx, "profile", 0)
            launches, kms, kbytes, krhs = dl.dl_profile_read(ctx, tier)
            blk = dl.dl_autotune(ctx, lat, tier, n)
            print(json.dumps({"sweep": "dslash", "precision": name, "nsrc": n, "rhs_block": list(blk),
                              "launches": int(launches), "avg_launch_us": round(kms * 1e3 / max(launches, 1), 1),
                              "gbs": round(kbytes / (kms * 1e-3) / 1e9, 1) if kms > 0 else 0.0,
                              "frac": round(kbytes / (kms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4) if kms > 0 else 0.0}),
                  flush=True)
    print(json.dumps({"sweep": "copy", "gbs": round(copy_gbs(torch), 1)}), flush=True)
    dl.dl_lattice_destroy(lat)
    dl.dl_destroy(ctx)
    return 0


def bench_uneven(a, table=UNEVEN, name="uneven") -> int:
    """Uneven batch: lattices of different sizes (six from 8^4 to 24^3x48, or twelve
    small ones) solved in one dl_solve_batch call (shared launches) against one
    call per lattice.  Per lattice: FP16 LP sources at rho = 1e-2, n/8 HP sources
    (FP32 + FP64 reliable updates) at 1e-8 and their LPC solves, all with local +
    derivative contractions."""
    import numpy as np
    import torch

    import paper_1401_6750_amd as dl
    import synth

    ctx = dl.dl_create(0, torch.cuda.current_stream().cuda_stream)
    dl.dl_set_option(ctx, "inflight_mb", a.inflight_mb)
    lats, accs = [], []
    for i, (dims, eps, n) in enumerate(table):
        lat, _ = _setup_lattice(dl, torch, synth, ctx, dims, 1410 + i, eps, 0.1615, 0.004)
        lats.append(lat)
        accs.append(dl.dl_accum_create(lat, dl.DL_OPS_LOCAL | dl.DL_OPS_DERIV))

    def jobs(i):
        lat, acc, n = lats[i], accs[i], table[i][2]
        nh = max(1, n // 8)
        return [dl.make_job(lat, noise=dl.DL_NOISE_Z2, tier=dl.DL_TIER_LP_FP16, seed=6760 + i, nsrc=n, tol=1e-2,
                            maxiter=500, accum=acc, accum_set=dl.DL_SET_LP),
                dl.make_job(lat, noise=dl.DL_NOISE_Z2, tier=dl.DL_TIER_HP_FP32, seed=6760 + i, first_src=n,
                            nsrc=nh, tol=1e-8, maxiter=2000, accum=acc, accum_set=dl.DL_SET_HP),
                dl.make_job(lat, noise=dl.DL_NOISE_Z2, tier=dl.DL_TIER_LP_FP16, seed=6760 + i, first_src=n,
                            nsrc=nh, tol=1e-2, maxiter=500, accum=acc, accum_set=dl.DL_SET_LPC)]

    def together():
        for acc in accs:
            dl.dl_accum_reset(acc)
        dl.dl_solve_batch(ctx, [j for i in range(len(table)) for j in jobs(i)])

    def separate():
        for i, acc in enumerate(accs):
            dl.dl_accum_reset(acc)
            dl.dl_solve_batch(ctx, jobs(i))

    def timed(fn):
        for _ in range(a.warmup):
            fn()
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(a.steps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t) / a.steps

    t_tog, t_sep = timed(together), timed(separate)
    n_lp = sum(n for _, _, n in table)
    res = {"metric": "uneven batch LP solves/s (one call for all lattices)", "value": round(n_lp / t_tog, 2),
           "unit": "LP solves/s", "ms_per_step": round(t_tog * 1e3, 2), "ms_per_step_separate_calls":
           round(t_sep * 1e3, 2), "batched_vs_separate": round(t_sep / t_tog, 3), "steps": a.steps,
           "config": {"workload": name, "lattices": [f"{'x'.join(map(str, d))} eps={e} n_lp={n}"
                                                     for d, e, n in table]}}
    print(json.dumps(res), flush=True)
    return 0


def bench_grad(a) -> int:
    """Differentiation workload: 16^3x32, 64 Z2 sources; forward (HP tier solve,
    contractions, projection) and backward (adjoint solves) through the
    autograd function; checks d/dmu against central differences (FP64, h=1e-5)."""
    import numpy as np
    import torch

    import paper_1401_6750_amd as dl
    import synth
    w = synth.WORKLOADS["tsm_16x16x16x32"]
    dims = w["dims"]
    ctx = dl.dl_create(0, torch.cuda.current_stream().cuda_stream)
    lat, _ = _setup_lattice(dl, torch, synth, ctx, dims, w["gauge_seed"], w["eps"], w["kappa"], w["mu"])
    nsrc, p2 = 64, 4
    vol = dims[0] * dims[1] * dims[2] * dims[3]
    eta0 = torch.zeros((nsrc, dims[3], dims[2], dims[1], dims[0], 4, 3), dtype=torch.complex128, device="cuda")
    for r in range(nsrc):   # the library's own Z2 generator (the sources the forward pass would draw)
        dl.dl_fill_noise(lat, dl.DL_NOISE_Z2, w["source_seed"], r, eta0[r])
    assert eta0.numel() == nsrc * vol * 12
    np_ = len(dl.dl_momenta(dims, p2))
    rng = np.random.default_rng(0)
    gw = torch.from_numpy(rng.standard_normal((2, 5, 16, dims[3], np_))
                          + 1j * rng.standard_normal((2, 5, 16, dims[3], np_))).to("cuda")
    ops = dl.DL_OPS_LOCAL | dl.DL_OPS_DERIV

    def run(tier, tol, mu_val, grad=True):
        eta = eta0.clone().requires_grad_(grad)
        mu = torch.tensor(mu_val, dtype=torch.float64, requires_grad=grad)
        L = dl.DiscLoops.apply(eta, mu, ctx, lat, w["kappa"], p2, ops, tier, tol)
        F = (L * gw.conj()).real.sum()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        if grad:
            F.backward()
            torch.cuda.synchronize()
        return F.item(), (mu.grad.item() if grad else None), t1

    run(dl.DL_TIER_HP_FP32, 1e-8, w["mu"])             # warm-up (autotuner, allocations)
    t0 = time.perf_counter()
    F, dmu, t1 = run(dl.DL_TIER_HP_FP32, 1e-8, w["mu"])
    t2 = time.perf_counter()
    h = 1e-5
    fp = run(dl.DL_TIER_FP64, 1e-12, w["mu"] + h, grad=False)[0]
    fm = run(dl.DL_TIER_FP64, 1e-12, w["mu"] - h, grad=False)[0]
    fd = (fp - fm) / (2 * h)
    _, dmu64, _ = run(dl.DL_TIER_FP64, 1e-12, w["mu"])
    res = {"metric": "loop gradient (adjoint) cost", "forward_ms": round((t1 - t0) * 1e3, 2),
           "backward_ms": round((t2 - t1) * 1e3, 2), "backward_over_forward": round((t2 - t1) / (t1 - t0), 3),
           "dF_dmu_hp": dmu, "dF_dmu_fp64": dmu64, "dF_dmu_central_difference_fp64": fd,
           "rel_err_fp64_vs_fd": abs(dmu64 - fd) / abs(fd), "rel_err_hp_vs_fd": abs(dmu - fd) / abs(fd),
           "config": {"workload": "grad_16x16x16x32", "nsrc": nsrc, "p2max": p2, "forward_tier": "fp32+RU",
                      "tol": 1e-8}}
    print(json.dumps(res), flush=True)
    return 0


def bench_error(a) -> int:
    print(json.dumps(equal_error_record()), flush=True)
    return 0


def equal_error_record() -> dict:
    """Same final accuracy: the truncated solver method against plain FP64 solves at
    equal standard error of one loop, on 16^3x32 (Z2 sources).

    The observable is the tau_3 loop with Gamma_15 = gamma_5 at p = 0 summed over t.
    TSM: 200 LP (bf16, rho 1e-2) + 10 HP (fp32 + RU, rho 1e-8, started from the LPC
    solutions) + the 10 LPC solves; its standard error is the jackknife error of 10
    bins (20 LP + 1 HP + 1 LPC each, every bin a complete TSM estimate).  Plain: FP64
    solves to rho 1e-8; the per-source variance from 10 bins of 4 sources gives the
    number of plain sources N_eq with the TSM's error, timed single-rhs (the
    comparator path) and batched."""
    import numpy as np
    import torch

    import paper_1401_6750_amd as dl
    import synth
    w = synth.WORKLOADS["tsm_16x16x16x32"]
    dims = w["dims"]
    ctx = dl.dl_create(0, torch.cuda.current_stream().cuda_stream)
    lat, _ = _setup_lattice(dl, torch, synth, ctx, dims, w["gauge_seed"], w["eps"], w["kappa"], w["mu"])
    seed, nb, n_lp, n_hp, p2 = w["source_seed"], 10, 200, 10, 0
    ops = dl.DL_OPS_LOCAL
    Z2 = dl.DL_NOISE_Z2

    def tsm_jobs(acc, lp0, nlp, hp0, nhp):
        return [dl.make_job(lat, noise=Z2, tier=dl.DL_TIER_LP_BF16, seed=seed, first_src=lp0, nsrc=nlp, tol=1e-2,
                            maxiter=500, accum=acc, accum_set=dl.DL_SET_LP),
                dl.make_job(lat, noise=Z2, tier=dl.DL_TIER_HP_FP32, seed=seed, first_src=hp0, nsrc=nhp, tol=1e-8,
                            maxiter=2000, accum=acc, accum_set=dl.DL_SET_HP, guess_from=3),
                dl.make_job(lat, noise=Z2, tier=dl.DL_TIER_LP_BF16, seed=seed, first_src=hp0, nsrc=nhp, tol=1e-2,
                            maxiter=500, accum=acc, accum_set=dl.DL_SET_LPC)]

    def observable(acc):
        out = np.zeros((2, 1, 16, dims[3], 1), dtype=np.complex128)
        dl.dl_loops(ctx, acc, p2, out, 0)
        return out[0, 0, 15, :, 0].sum()

    def timed(fn, reps=2):
        fn()
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t) / reps

    # TSM: the production step (one accumulator), timed
    acc = dl.dl_accum_create(lat, ops)

    def tsm_step():
        dl.dl_accum_reset(acc)
        dl.dl_solve_batch(ctx, tsm_jobs(acc, 0, n_lp, n_lp, n_hp))
        return observable(acc)

    t_tsm = timed(tsm_step)
    est_tsm = tsm_step()
    # TSM errors from bins
    accs = [dl.dl_accum_create(lat, ops) for _ in range(nb)]
    jobs = []
    for b in range(nb):
        jobs += tsm_jobs(accs[b], b * (n_lp // nb), n_lp // nb, n_lp + b * (n_hp // nb), n_hp // nb)
    for j, q in enumerate(jobs):
        if q.guess_from:
            q.guess_from = j + 2          # the LPC job right after it
    rc, _ = dl.dl_solve_batch(ctx, jobs)
    assert rc == dl.DL_OK
    bins_tsm = np.array([observable(x) for x in accs])
    for x in accs:
        dl.dl_accum_destroy(x)
    err_tsm = float(np.sqrt(np.mean(np.abs(bins_tsm - bins_tsm.mean()) ** 2) / (nb - 1)))
    # plain FP64: per-source variance from bins of 4
    per_bin = 4
    accs = [dl.dl_accum_create(lat, ops) for _ in range(nb)]
    rc, _ = dl.dl_solve_batch(ctx, [dl.make_job(lat, noise=Z2, tier=dl.DL_TIER_FP64, seed=seed,
                                                first_src=10_000 + b * per_bin, nsrc=per_bin, tol=1e-8,
                                                maxiter=2000, accum=accs[b], accum_set=dl.DL_SET_HP)
                                    for b in range(nb)])
    assert rc == dl.DL_OK
    bins_plain = np.array([observable(x) for x in accs])
    for x in accs:
        dl.dl_accum_destroy(x)
    var_plain = per_bin * float(np.sum(np.abs(bins_plain - bins_plain.mean()) ** 2) / (nb - 1))
    n_eq = var_plain / err_tsm ** 2
    # plain FP64 time per source: single-rhs without graph (the comparator), and batched
    acc1 = dl.dl_accum_create(lat, ops)

    def plain(n, single):
        dl.dl_accum_reset(acc1)
        if single:
            dl.dl_set_option(ctx, "inflight_rhs", 1)
            dl.dl_set_option(ctx, "use_graph", 0)
        dl.dl_solve_batch(ctx, dl.make_job(lat, noise=Z2, tier=dl.DL_TIER_FP64, seed=seed, first_src=20_000,
                                           nsrc=n, tol=1e-8, maxiter=2000, rhs_block=1 if single else 0,
                                           accum=acc1, accum_set=dl.DL_SET_HP))
        observable(acc1)
        dl.dl_set_option(ctx, "inflight_rhs", 1024)
        dl.dl_set_option(ctx, "use_graph", 1)

    t_single = timed(lambda: plain(4, True), reps=1) / 4
    t_batch = timed(lambda: plain(64, False), reps=1) / 64
    res = {"metric": "TSM time to equal standard error vs plain FP64 (tau_3 gamma_5 loop, p=0)",
           "value": round(n_eq * t_single / t_tsm, 2), "unit": "x (plain FP64 single-rhs time / TSM time)",
           "higher_is_better": True, "tsm_ms": round(t_tsm * 1e3, 2), "tsm_estimate": [est_tsm.real, est_tsm.imag],
           "tsm_error": err_tsm, "plain_per_source_sigma": var_plain ** 0.5, "plain_sources_for_equal_error":
           round(n_eq, 1), "plain_fp64_single_rhs_ms_per_source": round(t_single * 1e3, 2),
           "plain_fp64_batched_ms_per_source": round(t_batch * 1e3, 2),
           "vs_plain_fp64_batched": round(n_eq * t_batch / t_tsm, 2),
           "config": {"workload": "tsm_error_16x16x16x32", "n_lp": n_lp, "n_hp": n_hp, "bins": nb,
                      "plain_bins": [nb, per_bin], "noise": "Z2", "insertions": "local", "p2max": p2}}
    dl.dl_accum_destroy(acc)
    dl.dl_accum_destroy(acc1)
    dl.dl_lattice_destroy(lat)
    dl.dl_destroy(ctx)
    return res


# ---- CPU baseline: the FP64 oracle on the host cores -----------------------
# Stages of the oracle's per-source pipeline, each timed in a worker process of
# its own; every host core the run may use holds one worker, so each stage is
# timed under full load.
ORACLE_STAGES = ("solve0", "solve1", "loops")


def _oracle_stage(task):
    """One timed stage of the oracle's per-source work (runs in a spawned worker).
    solve0 / solve1: the even-odd CGNR solve to rho = 1e-2 stopped after zero / one
    iterations (Schur right-hand side, its M^dag, the iterations, the even-site
    reconstruction); loops: the 160 site loops of one source and their projection."""
    kind, upath, dims, kappa, mu, seed, src, z4, p2 = task
    for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
        os.environ[k] = "1"
    import numpy as np

    from oracle import loops, noise as onoise, solver
    U = np.load(upath, mmap_mode="r")
    eta = onoise.source(tuple(dims), seed, src, onoise.Z4 if z4 else onoise.Z2)
    t = time.perf_counter()
    if kind == "solve0":
        solver.cgnr_eo(U, eta, kappa, mu, -1, tuple(dims), 1e-2, maxiter=0)
    elif kind == "solve1":
        solver.cgnr_eo(U, eta, kappa, mu, -1, tuple(dims), 1e-2, maxiter=1)
    else:
        # the cost of the loops does not depend on the values: the source stands in
        # for the solution
        loops.source_loops(U, eta, kappa, -1, p2, tuple(dims))
    return kind, time.perf_counter() - t


def oracle_stage_times(U, dims, kappa, mu, seed, z4, p2, workers):
    """Time the oracle stages in `workers` spawned processes at once (stage k of
    worker k mod 3).  Call before the GPU is initialised.  Returns (mean seconds
    per stage, workers, wall seconds)."""
    import multiprocessing as mp
    import tempfile

    import numpy as np
    fd, upath = tempfile.mkstemp(suffix=".npy")
    os.close(fd)
    try:
        np.save(upath, np.ascontiguousarray(U))
        tasks = [(ORACLE_STAGES[k % 3], upath, list(dims), kappa, mu, seed, k, z4, p2) for k in range(workers)]
        t = time.perf_counter()
        with mp.get_context("spawn").Pool(workers) as pool:
            res = pool.map(_oracle_stage, tasks, chunksize=1)
        wall = time.perf_counter() - t
    finally:
        os.remove(upath)
    times = {k: [dt for kk, dt in res if kk == k] for k in ORACLE_STAGES}
    return {k: sum(v) / len(v) for k, v in times.items()}, workers, wall


def host_cores() -> int:
    """Cores this process may run on, at most 16 (the host share of one GPU)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def kernel_hash() -> str:
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        h.update(open(p, "rb").read())
    return h.hexdigest()[:16]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="batched_24x24x24x48", choices=sorted(WORKLOADS))
    ap.add_argument("--rhs-block", type=int, default=0)
    ap.add_argument("--inflight-mb", type=float, default=65536.0)
    ap.add_argument("--contract-tblk", type=int, default=0,
                    help="time slices per block of the derivative contraction's tile order (0: the library's)")
    ap.add_argument("--inflight-rhs", type=int, default=0,
                    help="most right-hand sides per solve batch (0: the library's default)")
    ap.add_argument("--hpe", type=int, default=0,
                    help="hopping parameter expansion order (1..4) for the loops without tau_3; 0: off")
    ap.add_argument("--tdil", type=int, default=0,
                    help="time dilution: D components per noise vector (the noise-vector counts are "
                         "divided by D so the number of solves stays the same); 0: off")
    ap.add_argument("--p2max", type=int, default=-1,
                    help="momentum cut |n|^2 <= p2max of the projection (default: the workload's; "
                         "a cut >= 3 (L/2)^2 keeps every momentum)")
    ap.add_argument("--csw", type=float, default=0.0,
                    help="clover coefficient c_sw of the operator (0: the plain twisted-mass operator)")
    ap.add_argument("--block-hop", action="store_true",
                    help="16-bit hops through the LDS-staged kernel (option block_hop) instead of the tile kernel")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-comparator", action="store_true")
    ap.add_argument("--profile-only", action="store_true",
                    help="run only the profiled LP pass (for rocprofv3 counter runs)")
    a = ap.parse_args()
    if a.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: the library runs on one GPU only; the per-GPU share of a multi-GPU run is the "
              "N=1 workload (sources shard across GPUs with one final reduction of the projected loops)",
              file=sys.stderr)
        return 2

    import numpy as np
    import torch

    import paper_1401_6750_amd as dl
    import synth

    if a.workload not in ("batched_24x24x24x48", "tsm_16x16x16x32"):
        assert torch.cuda.is_available(), "bench.py needs a GPU"
    if a.workload == "uneven":
        return bench_uneven(a)
    if a.workload == "uneven_small":
        return bench_uneven(a, UNEVEN_SMALL, "uneven_small")
    if a.workload == "grad_16x16x16x32":
        return bench_grad(a)
    if a.workload == "dslash_sweep":
        return bench_sweep(a)
    if a.workload == "tsm_error_16x16x16x32":
        return bench_error(a)
    w = synth.WORKLOADS[a.workload]
    tw = WORKLOADS[a.workload]
    dims, kappa, mu = w["dims"], w["kappa"], w["mu"]
    X, Y, Z, T = dims
    noise_kind = dl.DL_NOISE_Z4 if tw["noise"] == "Z4" else dl.DL_NOISE_Z2
    n_lp, n_hp, p2 = tw["n_lp"], tw["n_hp"], tw["p2max"]
    if a.p2max >= 0:
        p2 = a.p2max
    ncomp = max(a.tdil, 1)
    v_lp, v_hp = n_lp // ncomp, n_hp // ncomp      # noise vectors; n_lp, n_hp stay the solve counts
    n_lp, n_hp = v_lp * ncomp, v_hp * ncomp

    log(f"setup: {a.workload} gauge field")
    U = synth.random_gauge(dims, w["gauge_seed"], w["eps"])
    seed = w["source_seed"]
    # the oracle's stages run first, in processes spawned before this process
    # touches the GPU
    stages = None
    if not (a.no_cpu_baseline or a.profile_only):
        nwk = max(3, host_cores())
        log(f"cpu baseline: oracle stages in {nwk} processes")
        stages, nwk, wall = oracle_stage_times(U, dims, kappa, mu, seed, noise_kind == dl.DL_NOISE_Z4, p2, nwk)
        log(f"cpu baseline: {wall:.1f} s wall, stage seconds " +
            ", ".join(f"{k} {v:.2f}" for k, v in stages.items()))
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    U_dev = torch.from_numpy(np.ascontiguousarray(U)).to("cuda")
    stream = torch.cuda.current_stream()
    ctx = dl.dl_create(0, stream.cuda_stream)
    dl.dl_set_option(ctx, "inflight_mb", a.inflight_mb)
    if a.inflight_rhs:
        dl.dl_set_option(ctx, "inflight_rhs", a.inflight_rhs)
    if a.contract_tblk:
        dl.dl_set_option(ctx, "contract_tblk", a.contract_tblk)
    if a.block_hop:
        dl.dl_set_option(ctx, "block_hop", 1)
    lat = dl.dl_lattice_create(ctx, dims, -1)
    dl.dl_gauge_set(lat, U_dev, 1)
    dl.dl_set_params(lat, kappa, mu)
    if a.csw:
        dl.dl_set_clover(lat, a.csw)
    acc = dl.dl_accum_create(lat, dl.DL_OPS_LOCAL | dl.DL_OPS_DERIV | dl.DL_OPS_HPE(a.hpe))
    blocks = {"bf16": list(dl.dl_autotune(ctx, lat, dl.DL_TIER_LP_BF16, n_lp)),
              "fp32": list(dl.dl_autotune(ctx, lat, dl.DL_TIER_HP_FP32, n_hp))}
    if a.rhs_block:
        blocks = {k: [a.rhs_block, 4] for k in blocks}
    log(f"rhs blocks: {blocks}")
    nmom = len(dl.dl_momenta(dims, p2))
    out = torch.zeros((2, 5, 16, T, nmom), dtype=torch.complex128, device="cuda")

    def jobs():
        return [
            dl.make_job(lat, noise=noise_kind, tier=dl.DL_TIER_LP_BF16, seed=seed, first_src=0, nsrc=v_lp,
                        tol=1e-2, maxiter=500, rhs_block=a.rhs_block, accum=acc, accum_set=dl.DL_SET_LP,
                        tdil=a.tdil),
            # HP correction solves start from the LPC solutions of the same sources (job 2)
            dl.make_job(lat, noise=noise_kind, tier=dl.DL_TIER_HP_FP32, seed=seed, first_src=v_lp, nsrc=v_hp,
                        tol=1e-8, maxiter=2000, rhs_block=a.rhs_block, accum=acc, accum_set=dl.DL_SET_HP,
                        guess_from=3, tdil=a.tdil),
            dl.make_job(lat, noise=noise_kind, tier=dl.DL_TIER_LP_BF16, seed=seed, first_src=v_lp, nsrc=v_hp,
                        tol=1e-2, maxiter=500, rhs_block=a.rhs_block, accum=acc, accum_set=dl.DL_SET_LPC,
                        tdil=a.tdil),
        ]

    def step():
        dl.dl_accum_reset(acc)
        rc, st = dl.dl_solve_batch(ctx, jobs())
        dl.dl_loops(ctx, acc, p2, out, 1)
        return rc, st

    if a.profile_only:
        dl.dl_set_option(ctx, "profile", 1)
        step()
        torch.cuda.synchronize()
        pr = dl.dl_profile_read(ctx, dl.DL_TIER_LP_BF16)
        log(f"profile: launches {pr[0]:.0f}, kernel ms {pr[1]:.3f}, alg bytes {pr[2]:.0f}, rhs {pr[3]:.0f}")
        # calibration kernel of known traffic for the HBM byte counters:
        # reads 1 GiB and writes 1 GiB (torch's elementwise multiply)
        x = torch.ones(2 ** 28, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        torch.mul(x, 2.0, out=y)
        torch.cuda.synchronize()
        log("calibration: elementwise multiply, 1073741824 bytes read, 1073741824 bytes written")
        return 0

    for i in range(a.warmup):
        log(f"warmup step {i}")
        rc, st = step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    marks = []
    for i in range(a.steps):
        rc, st = step()          # the solves synchronise; only the projection may still run
        marks.append(time.perf_counter())
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms = (t1 - t0) * 1e3 / a.steps
    per = [round((b - a_) * 1e3, 1) for a_, b in zip([t0] + marks[:-1], marks)]
    log(f"timed {a.steps} steps: {ms:.1f} ms/step (each: {per})")
    assert rc == dl.DL_OK, f"solve status {rc}"
    # projection + Gamma rebuild + TSM combination alone (part of every step above)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(3):
        dl.dl_loops(ctx, acc, p2, out, 1)
    torch.cuda.synchronize()
    loops_ms = (time.perf_counter() - t) * 1e3 / 3
    it_lp = [s.iters for s in st[:n_lp]]
    it_hp = [s.iters for s in st[n_lp:n_lp + n_hp]]
    ru_hp = [s.reliable_updates for s in st[n_lp:n_lp + n_hp]]

    # ---- roofline of the hopping kernel, timed live with HIP events -----------
    dl.dl_set_option(ctx, "profile", 1)
    step()
    torch.cuda.synchronize()
    dl.dl_set_option(ctx, "profile", 0)
    launches, kms, kbytes, krhs = dl.dl_profile_read(ctx, dl.DL_TIER_LP_BF16)
    achieved = kbytes / (kms * 1e-3) / 1e9 if kms > 0 else 0.0
    traffic = None
    if os.path.exists(COUNTERS):
        c = json.load(open(COUNTERS))
        if c.get("kernel_hash") == kernel_hash() and c.get("workload") == a.workload:
            traffic = c.get("hbm_bytes_per_launch")
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "kernel": "k_dslash<bf16s, 0> (u_e = A^-1 H_eo p_o, LP tier)",
                "launches": int(launches), "avg_launch_us": round(kms * 1e3 / max(launches, 1), 2),
                "alg_bytes_per_launch": round(kbytes / max(launches, 1)),
                "avg_active_rhs": round(krhs / max(launches, 1), 1),
                "copy_gbs": round(copy_gbs(torch), 1)}

    # ---- per-tier breakdown and the plain FP64 comparator (untimed in value) --
    extra = {}
    if not a.no_comparator:
        def timed(job_list, reps=1):
            torch.cuda.synchronize()
            t = time.perf_counter()
            for _ in range(reps):
                dl.dl_solve_batch(ctx, job_list)
            torch.cuda.synchronize()
            return (time.perf_counter() - t) / reps

        t_lp = timed([dl.make_job(lat, noise=noise_kind, tier=dl.DL_TIER_LP_BF16, seed=seed, nsrc=n_lp, tol=1e-2,
                                  maxiter=500, rhs_block=a.rhs_block)])
        t_hp = timed([dl.make_job(lat, noise=noise_kind, tier=dl.DL_TIER_HP_FP32, seed=seed, first_src=n_lp,
                                  nsrc=n_hp, tol=1e-8, maxiter=2000, rhs_block=a.rhs_block)])
        n_cmp = 4
        dl.dl_set_option(ctx, "inflight_rhs", 1)
        dl.dl_set_option(ctx, "use_graph", 0)
        t_64 = timed([dl.make_job(lat, noise=noise_kind, tier=dl.DL_TIER_FP64, seed=seed, first_src=n_lp, nsrc=n_cmp,
                                  tol=1e-8, maxiter=2000, rhs_block=1)])
        dl.dl_set_option(ctx, "inflight_rhs", 1024)
        dl.dl_set_option(ctx, "use_graph", 1)
        extra = {
            "lp_solves_per_s_solve_only": round(n_lp / t_lp, 2),
            "hp_solves_per_s": round(n_hp / t_hp, 2),
            "fp64_plain_single_rhs_solves_per_s_rho1e-8": round(n_cmp / t_64, 3),
            # solve rates at different final accuracies (LP rho 1e-2 against FP64
            # rho 1e-8); the same-accuracy comparison is equal_error_16x16x16x32
            "lp_rho1e-2_over_fp64_single_rhs_rho1e-8_solve_rate": round((n_lp / t_lp) / (n_cmp / t_64), 1),
            "hp_over_fp64_single_rhs_solve_rate_both_rho1e-8": round((n_hp / t_hp) / (n_cmp / t_64), 2),
        }
        log("equal-error comparison on 16^3x32")
        rec = equal_error_record()
        extra["equal_error_16x16x16x32"] = {
            "metric": rec["metric"], "value": rec["value"], "unit": rec["unit"],
            "vs_plain_fp64_batched": rec["vs_plain_fp64_batched"], "tsm_ms": rec["tsm_ms"],
            "tsm_error": rec["tsm_error"], "plain_per_source_sigma": rec["plain_per_source_sigma"],
            "plain_sources_for_equal_error": rec["plain_sources_for_equal_error"],
            "plain_fp64_single_rhs_ms_per_source": rec["plain_fp64_single_rhs_ms_per_source"],
            "plain_fp64_batched_ms_per_source": rec["plain_fp64_batched_ms_per_source"],
            "config": rec["config"]}

    # ---- CPU baseline: the FP64 oracle, stages timed on every host core --------
    cpu = None
    if stages is not None:
        mean_lp, mean_hp = float(np.mean(it_lp)), float(np.mean(it_hp))
        t_it = max(stages["solve1"] - stages["solve0"], 0.0)
        t_src_lp = stages["solve0"] + mean_lp * t_it + stages["loops"]
        t_src_hp = stages["solve0"] + mean_hp * t_it + stages["loops"]
        step_one = (n_lp + n_hp) * t_src_lp + n_hp * t_src_hp     # LP and LPC sources, HP sources
        per_proc = n_lp / step_one
        cpu = {"value": round(per_proc * nwk, 6), "unit": "LP solves/s", "cores": nwk, "kind": "oracle",
               "sample": f"the FP64 oracle's per-source stages on the {a.workload} workload, timed in {nwk} "
                         f"concurrent processes (one per host core): even-odd CGNR to rho 1e-2 stopped after "
                         f"0 and 1 iterations ({stages['solve0']:.1f} s, {stages['solve1']:.1f} s: Schur "
                         f"right-hand side, iterations, reconstruction) and one source's 160 site loops with "
                         f"the p^2 <= {p2} projection ({stages['loops']:.1f} s); a source costs solve0 + "
                         f"iterations x (solve1 - solve0) + loops with this run's GPU iteration counts "
                         f"(LP {mean_lp:.1f}, HP {mean_hp:.1f}); a step is {n_lp + n_hp} LP-tier and {n_hp} HP "
                         f"sources; value = cores x the rate of one process under full load",
               "per_process_value": round(per_proc, 6),
               "stage_s": {k: round(v, 3) for k, v in stages.items()}}

    res = {
        "metric": METRIC, "value": round(n_lp / (ms * 1e-3), 2), "unit": "LP solves/s",
        "n_gpus": 1, "steps": a.steps, "warmup": a.warmup, "ms_per_step": round(ms, 2),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": a.workload, "lattice": "x".join(map(str, dims)), "n_lp": n_lp, "n_hp": n_hp,
                   "n_lpc": n_hp, "lp_storage": "bf16", "hp": "fp32+fp64 reliable updates",
                   "noise": tw["noise"], "p2max": p2, "insertions": 160, "rhs_block": blocks,
                   "hpe_order": a.hpe, "tdil": a.tdil, "csw": a.csw},
        "iters_lp_mean": round(float(np.mean(it_lp)), 2), "iters_hp_mean": round(float(np.mean(it_hp)), 2),
        "reliable_updates_hp_mean": round(float(np.mean(ru_hp)), 2),
        "momenta": nmom, "projection_ms": round(loops_ms, 2),
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    res.update(extra)
    print(json.dumps(res), flush=True)
    dl.dl_accum_destroy(acc)
    dl.dl_lattice_destroy(lat)
    dl.dl_destroy(ctx)
    return 0


if __name__ == "__main__":
    sys.exit(main())
