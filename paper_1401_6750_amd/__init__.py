"""Python binding of libdiscloop, the gfx950 stochastic fermion-loop library.

Argument marshalling only: every function here calls the C entry point of the
same name in ``libdiscloop.so`` (declared in ``include/discloop.h``) and
raises ``DiscloopError`` on a negative status.  Pointer arguments accept torch
tensors (their ``data_ptr()``), numpy arrays (host memory), plain integers or
``None``.  There is no fallback: if the shared library is missing the import
of any function fails loudly.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdiscloop.so")

# constants mirrored from include/discloop.h
DL_OK, DL_NOT_CONVERGED = 0, 1
DL_EINVAL, DL_ENOMEM, DL_EHIP, DL_ESTATE, DL_EBREAKDOWN = -1, -2, -3, -4, -5
DL_NOISE_Z2, DL_NOISE_Z4, DL_NOISE_USER = 0, 1, 2
DL_TIER_FP64, DL_TIER_LP_BF16, DL_TIER_LP_FP16, DL_TIER_HP_FP32 = 0, 1, 2, 3
DL_SET_LP, DL_SET_HP, DL_SET_LPC = 0, 1, 2
DL_OPS_LOCAL, DL_OPS_DERIV = 1, 2


def DL_OPS_HPE(n: int) -> int:
    """Hopping parameter expansion of order n (1..4) for the loops without tau_3."""
    return n << 4


def DL_OPS_HPE_ORDER(ops: int) -> int:
    return (ops >> 4) & 7


DL_SRC_CONVERGED, DL_SRC_MAXITER, DL_SRC_BREAKDOWN = 0, 1, 2
DL_OP_M, DL_OP_MDAG, DL_OP_MHAT, DL_OP_MHAT_DAG, DL_OP_HOP = 0, 1, 2, 3, 4


class DiscloopError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"[{code}] {msg}")
        self.code = code


class dl_job(ctypes.Structure):
    _fields_ = [
        ("lat", ctypes.c_void_p),
        ("noise", ctypes.c_int),
        ("tier", ctypes.c_int),
        ("seed", ctypes.c_uint64),
        ("first_src", ctypes.c_int64),
        ("nsrc", ctypes.c_int),
        ("maxiter", ctypes.c_int),
        ("tol", ctypes.c_double),
        ("rhs_block", ctypes.c_int),
        ("report_true_resid", ctypes.c_int),
        ("src_in", ctypes.c_void_p),
        ("sol_out", ctypes.c_void_p),
        ("accum", ctypes.c_void_p),
        ("accum_set", ctypes.c_int),
        ("guess_from", ctypes.c_int),
        ("tdil", ctypes.c_int),
        ("grad_ops", ctypes.c_int),
    ]


class dl_src_stats(ctypes.Structure):
    _fields_ = [
        ("iters", ctypes.c_int),
        ("status", ctypes.c_int),
        ("rel_resid", ctypes.c_double),
        ("true_resid", ctypes.c_double),
        ("reliable_updates", ctypes.c_int),
        ("pad", ctypes.c_int),
    ]


_lib = None

_P = ctypes.c_void_p
_I = ctypes.c_int
_D = ctypes.c_double
_SIGS = {
    "dl_create": ([ctypes.POINTER(_P), _I, _P], _I),
    "dl_destroy": ([_P], _I),
    "dl_last_error": ([], ctypes.c_char_p),
    "dl_version": ([], ctypes.c_char_p),
    "dl_lattice_create": ([_P, ctypes.POINTER(_I), _I, ctypes.POINTER(_P)], _I),
    "dl_lattice_destroy": ([_P], _I),
    "dl_gauge_set": ([_P, _P, _I], _I),
    "dl_set_params": ([_P, _D, _D], _I),
    "dl_set_clover": ([_P, _D], _I),
    "dl_gauge_random": ([_P, ctypes.c_uint64, _D], _I),
    "dl_gauge_random_host": ([ctypes.POINTER(_I), ctypes.c_uint64, _D, _P], _I),
    "dl_solve_batch": ([_P, ctypes.POINTER(dl_job), _I, ctypes.POINTER(dl_src_stats)], _I),
    "dl_accum_create": ([_P, _I, ctypes.POINTER(_P)], _I),
    "dl_accum_reset": ([_P], _I),
    "dl_accum_destroy": ([_P], _I),
    "dl_accum_counts": ([_P, ctypes.POINTER(ctypes.c_int64)], _I),
    "dl_momenta": ([ctypes.POINTER(_I), _I, ctypes.POINTER(_I), _I, ctypes.POINTER(_I)], _I),
    "dl_loops": ([_P, _P, _I, _P, _I, ctypes.POINTER(_I)], _I),
    "dl_loops_sets": ([_P, _P, _I, _P, _I, ctypes.POINTER(_I)], _I),
    "dl_loops_noalloc": ([_P, _P, _I, _P, ctypes.POINTER(_I)], _I),
    "dl_loops_backward": ([_P, ctypes.POINTER(dl_job), _I, _P, _P, _P], _I),
    "dl_set_option": ([_P, ctypes.c_char_p, _D], _I),
    "dl_profile_read": ([_P, _I, ctypes.POINTER(_D)], _I),
    "dl_autotune": ([_P, _P, _I, _I, ctypes.POINTER(_I), ctypes.POINTER(_I)], _I),
    "dl_apply_op": ([_P, _I, _I, _P, _P, _I], _I),
    "dl_fill_noise": ([_P, _I, ctypes.c_uint64, ctypes.c_int64, _P], _I),
}


def lib():
    """The loaded shared library (raises if it was not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1401_6750_amd.build`")
        l = ctypes.CDLL(LIB_PATH)
        for name, (args, res) in _SIGS.items():
            fn = getattr(l, name)
            fn.argtypes = args
            fn.restype = res
        _lib = l
    return _lib


def _ptr(x):
    """Raw address of a torch tensor, numpy array, int or None."""
    if x is None:
        return None
    if isinstance(x, int):
        return x
    if hasattr(x, "data_ptr"):
        return x.data_ptr()
    if hasattr(x, "ctypes"):
        return x.ctypes.data
    raise TypeError(f"cannot take the address of {type(x)}")


def _check(rc: int) -> int:
    if rc < 0:
        raise DiscloopError(rc, lib().dl_last_error().decode())
    return rc


def dl_last_error() -> str:
    return lib().dl_last_error().decode()


def dl_version() -> str:
    return lib().dl_version().decode()


def dl_create(device: int = 0, hip_stream=None):
    """Context on `device`; hip_stream is a raw stream handle (int) or None."""
    h = _P()
    _check(lib().dl_create(ctypes.byref(h), device, hip_stream))
    return h


def dl_destroy(ctx) -> None:
    _check(lib().dl_destroy(ctx))


def dl_lattice_create(ctx, dims, t_bc: int = -1):
    d = (_I * 4)(*dims)
    h = _P()
    _check(lib().dl_lattice_create(ctx, d, t_bc, ctypes.byref(h)))
    return h


def dl_lattice_destroy(lat) -> None:
    _check(lib().dl_lattice_destroy(lat))


def dl_gauge_set(lat, links, on_device: int) -> None:
    _check(lib().dl_gauge_set(lat, _ptr(links), on_device))


def dl_gauge_random(lat, seed: int, eps: float) -> None:
    _check(lib().dl_gauge_random(lat, seed, eps))


def dl_gauge_random_host(dims, seed: int, eps: float, links) -> None:
    """Fill host complex128 links [T, Z, Y, X, 4, 3, 3] with the synthetic field."""
    d = (_I * 4)(*dims)
    _check(lib().dl_gauge_random_host(d, seed, eps, _ptr(links)))


def dl_set_params(lat, kappa: float, mu: float) -> None:
    _check(lib().dl_set_params(lat, kappa, mu))


def dl_set_clover(lat, csw: float) -> None:
    """Clover coefficient c_sw of the lattice's operator (0: no clover term)."""
    _check(lib().dl_set_clover(lat, csw))


def dl_accum_create(lat, ops: int):
    h = _P()
    _check(lib().dl_accum_create(lat, ops, ctypes.byref(h)))
    return h


def dl_accum_reset(acc) -> None:
    _check(lib().dl_accum_reset(acc))


def dl_accum_destroy(acc) -> None:
    _check(lib().dl_accum_destroy(acc))


def dl_accum_counts(acc):
    c = (ctypes.c_int64 * 3)()
    _check(lib().dl_accum_counts(acc, c))
    return list(c)


def dl_momenta(dims, p2max: int):
    """List of integer momenta [(nx, ny, nz), ...] in output order."""
    d = (_I * 4)(*dims)
    n = _I()
    _check(lib().dl_momenta(d, p2max, None, 0, ctypes.byref(n)))
    buf = (_I * (3 * max(n.value, 1)))()
    _check(lib().dl_momenta(d, p2max, buf, n.value, ctypes.byref(n)))
    return [tuple(buf[3 * i:3 * i + 3]) for i in range(n.value)]


def make_job(lat, *, noise=DL_NOISE_Z2, tier=DL_TIER_FP64, seed=0, first_src=0, nsrc=1, maxiter=1000,
             tol=1e-10, rhs_block=0, report_true_resid=0, src_in=None, sol_out=None, accum=None,
             accum_set=DL_SET_HP, guess_from=0, tdil=0, grad_ops=0) -> dl_job:
    """One job; guess_from = j + 1 starts an HP job from the solutions of job j of the same call;
    tdil = D >= 2 dilutes every noise vector into D time-slice components; grad_ops names the
    insertion set for dl_loops_backward when accum is None."""
    return dl_job(lat, noise, tier, seed, first_src, nsrc, maxiter, tol, rhs_block, report_true_resid,
                  _ptr(src_in), _ptr(sol_out), accum, accum_set, guess_from, tdil, grad_ops)


def dl_solve_batch(ctx, jobs):
    """Run jobs (a dl_job or a list of them); returns (status, [dl_src_stats ...])."""
    if isinstance(jobs, dl_job):
        jobs = [jobs]
    arr = (dl_job * len(jobs))(*jobs)
    n = sum(j.nsrc * max(j.tdil, 1) for j in jobs)
    stats = (dl_src_stats * max(n, 1))()
    rc = _check(lib().dl_solve_batch(ctx, arr, len(jobs), stats))
    return rc, list(stats)[:n]


def dl_loops(ctx, acc, p2max: int, out, out_on_device: int) -> int:
    n = _I()
    _check(lib().dl_loops(ctx, acc, p2max, _ptr(out), out_on_device, ctypes.byref(n)))
    return n.value


def dl_loops_sets(ctx, acc, p2max: int, out, out_on_device: int) -> int:
    """Per-set loop sums [3][2][nops][16][T][Np] (LP, HP, LPC), not divided by the counts."""
    n = _I()
    _check(lib().dl_loops_sets(ctx, acc, p2max, _ptr(out), out_on_device, ctypes.byref(n)))
    return n.value


def dl_loops_noalloc(ctx, acc, p2max: int, out) -> int:
    """dl_loops into device memory `out`, using the library's static device scratch (no allocation)."""
    n = _I()
    _check(lib().dl_loops_noalloc(ctx, acc, p2max, _ptr(out), ctypes.byref(n)))
    return n.value


def dl_loops_backward(ctx, job: dl_job, p2max: int, grad_loops, grad_eta, grad_mu) -> None:
    _check(lib().dl_loops_backward(ctx, ctypes.byref(job), p2max, _ptr(grad_loops), _ptr(grad_eta),
                                   _ptr(grad_mu)))


def dl_set_option(ctx, name: str, value: float) -> None:
    _check(lib().dl_set_option(ctx, name.encode(), float(value)))


def dl_profile_read(ctx, tier: int):
    """(launches, total_ms, total_bytes, total_active_rhs) of the hopping kernel; resets them."""
    out = (_D * 4)()
    _check(lib().dl_profile_read(ctx, tier, out))
    return tuple(out)


def dl_autotune(ctx, lat, tier: int, nsrc: int = 128):
    """(rhs block, tile-order time block) the solver uses for a job of nsrc sources (tunes on first use)."""
    blk, tb = _I(0), _I(0)
    _check(lib().dl_autotune(ctx, lat, tier, nsrc, ctypes.byref(blk), ctypes.byref(tb)))
    return blk.value, tb.value


def dl_apply_op(lat, op: int, tier: int, inp, out, nrhs: int) -> None:
    _check(lib().dl_apply_op(lat, op, tier, _ptr(inp), _ptr(out), nrhs))


def dl_fill_noise(lat, noise: int, seed: int, src: int, out) -> None:
    _check(lib().dl_fill_noise(lat, noise, seed, src, _ptr(out)))


def _make_disc_loops():
    import torch

    class DiscLoops(torch.autograd.Function):
        """Loops of caller sources as a differentiable function of (eta, mu).

        forward(eta, mu, ctx, lat, kappa, p2max, ops, tier, tol) -> loops
          eta: complex128 CUDA tensor [nsrc, T, Z, Y, X, 4, 3]; mu: real 0-d tensor.
          Returns the plain estimator over the sources, complex128 CUDA
          [2, nops, 16, T, Np] (dl_loops layout).  The solutions are kept for
          the backward pass (checkpoint), which calls dl_loops_backward.
        """

        @staticmethod
        def forward(fctx, eta, mu, dlctx, lat, kappa, p2max, ops, tier, tol):
            mu_v = float(mu)
            dl_set_params(lat, kappa, mu_v)
            eta = eta.contiguous()
            nsrc = eta.shape[0]
            acc = dl_accum_create(lat, ops)
            try:
                sol = torch.empty_like(eta)
                job = make_job(lat, noise=DL_NOISE_USER, tier=tier, nsrc=nsrc, tol=tol, maxiter=10000,
                               src_in=eta, sol_out=sol, accum=acc, accum_set=DL_SET_HP)
                dl_solve_batch(dlctx, job)
                T = eta.shape[1]
                nops = 5 if ops & DL_OPS_DERIV else 1
                np_ = len(dl_momenta((eta.shape[4], eta.shape[3], eta.shape[2], T), p2max))
                out = torch.empty((2, nops, 16, T, np_), dtype=torch.complex128, device=eta.device)
                dl_loops(dlctx, acc, p2max, out, 1)
                torch.cuda.current_stream().synchronize()
            finally:
                # the backward pass needs only the insertion set (grad_ops), not the sums
                dl_accum_destroy(acc)
            fctx.save_for_backward(eta, sol)
            fctx.meta = (dlctx, lat, kappa, mu_v, p2max, ops, tier, tol)
            return out

        @staticmethod
        def backward(fctx, gout):
            eta, sol = fctx.saved_tensors
            dlctx, lat, kappa, mu_v, p2max, ops, tier, tol = fctx.meta
            dl_set_params(lat, kappa, mu_v)
            g_host = gout.detach().to("cpu", torch.complex128).contiguous().numpy()
            grad_eta = torch.empty_like(eta)
            gmu = ctypes.c_double()
            job = make_job(lat, noise=DL_NOISE_USER, tier=tier, nsrc=eta.shape[0], tol=tol, maxiter=10000,
                           src_in=eta, sol_out=sol, grad_ops=ops & (DL_OPS_LOCAL | DL_OPS_DERIV))
            _check(lib().dl_loops_backward(dlctx, ctypes.byref(job), p2max, g_host.ctypes.data,
                                           grad_eta.data_ptr(), ctypes.addressof(gmu)))
            torch.cuda.current_stream().synchronize()
            grad_mu = torch.tensor(gmu.value, dtype=torch.float64)
            return grad_eta, grad_mu, None, None, None, None, None, None, None

    return DiscLoops


def __getattr__(name):
    if name == "DiscLoops":
        cls = _make_disc_loops()
        globals()["DiscLoops"] = cls
        return cls
    raise AttributeError(name)
