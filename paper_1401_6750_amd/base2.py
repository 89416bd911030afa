"""Base-2 storage of loop partial sums (Section 2.1.1, Fig. 2).

The sources of one stream are grouped in blocks of 1, 2, 4, ... sources: level k
holds the summed loops of sources [2^k - 1, 2^(k+1) - 1) of the stream.  Any
count n < 2^K is the sum of the levels of the binary digits of n (13 = 1 + 4 + 8
uses levels 0, 2 and 3), so K files stand in for n per-source files and the
estimate for any n can be rebuilt from them; the sources are independent and
identically distributed, so which n sources enter does not matter.  A run that
stopped resumes at the first missing level.

Level files hold the per-set sums of ``dl_loops_sets`` (complex128
[2][nops][16][T][Np], prefactors applied, not divided by the count) as ``.npy``
files written atomically; ``meta.json`` identifies the source stream and is
checked when a store is reopened.
"""
from __future__ import annotations

import json
import os

import numpy as np


def levels_for(n: int) -> list[int]:
    """Levels whose blocks add up to n sources: the set bits of n."""
    if n < 0:
        raise ValueError("n must be >= 0")
    return [k for k in range(n.bit_length()) if (n >> k) & 1]


def level_sources(k: int) -> tuple[int, int]:
    """Source range [begin, end) of level k within the stream."""
    if k < 0:
        raise ValueError("level must be >= 0")
    return (1 << k) - 1, (1 << (k + 1)) - 1


class Base2Store:
    """A directory of level files for one source stream."""

    def __init__(self, directory: str, meta: dict):
        os.makedirs(directory, exist_ok=True)
        self.dir = directory
        path = os.path.join(directory, "meta.json")
        meta = json.loads(json.dumps(meta, sort_keys=True))   # plain JSON types
        if os.path.exists(path):
            with open(path) as f:
                old = json.load(f)
            if old != meta:
                raise ValueError(f"{directory} holds a different source stream: {old} != {meta}")
        else:
            tmp = path + ".tmp"
            with open(tmp, "w") as f:
                json.dump(meta, f, indent=1, sort_keys=True)
            os.replace(tmp, path)
        self.meta = meta

    def _file(self, k: int) -> str:
        return os.path.join(self.dir, f"level{k:02d}.npy")

    def has(self, k: int) -> bool:
        return os.path.exists(self._file(k))

    def levels(self) -> list[int]:
        out = []
        for name in os.listdir(self.dir):
            if name.startswith("level") and name.endswith(".npy"):
                out.append(int(name[5:-4]))
        return sorted(out)

    def save(self, k: int, sums) -> None:
        tmp = self._file(k) + ".tmp.npy"
        np.save(tmp, np.asarray(sums), allow_pickle=False)
        os.replace(tmp, self._file(k))

    def load(self, k: int) -> np.ndarray:
        return np.load(self._file(k), allow_pickle=False)

    def resume_level(self) -> int:
        """First level not stored yet."""
        k = 0
        while self.has(k):
            k += 1
        return k

    def total(self, n: int) -> np.ndarray:
        """Summed loops of n sources, from the levels of n's binary digits."""
        ls = levels_for(n)
        missing = [k for k in ls if not self.has(k)]
        if not ls:
            raise ValueError("n must be >= 1")
        if missing:
            raise KeyError(f"levels {missing} are not stored")
        out = self.load(ls[0]).copy()
        for k in ls[1:]:
            out += self.load(k)
        return out

    def estimate(self, n: int) -> np.ndarray:
        """Loop estimate (mean over sources) from n sources."""
        return self.total(n) / n


def solve_base2(ctx, lat, dims, store: Base2Store, nlevels: int, *, tier: int, noise: int, seed: int, tol: float,
                maxiter: int, p2max: int, ops: int, first_src: int = 0, rhs_block: int = 0) -> list[int]:
    """Solve and contract the stream level by level, storing each level's loop sums.

    Levels already in the store are skipped (resume).  Returns the levels computed by this
    call.  A level whose solves did not all converge is not stored (RuntimeError)."""
    from . import (DL_OK, DL_OPS_DERIV, DL_SET_LP, dl_accum_create, dl_accum_destroy, dl_accum_reset,
                   dl_loops_sets, dl_momenta, dl_solve_batch, make_job)

    nops = 5 if ops & DL_OPS_DERIV else 1
    npm = len(dl_momenta(dims, p2max))
    acc = dl_accum_create(lat, ops)
    done = []
    try:
        for k in range(nlevels):
            if store.has(k):
                continue
            b, e = level_sources(k)
            dl_accum_reset(acc)
            job = make_job(lat, noise=noise, tier=tier, seed=seed, first_src=first_src + b, nsrc=e - b, tol=tol,
                           maxiter=maxiter, rhs_block=rhs_block, accum=acc, accum_set=DL_SET_LP)
            rc, stats = dl_solve_batch(ctx, job)
            if rc != DL_OK:
                bad = [i for i, s in enumerate(stats) if s.status != 0]
                raise RuntimeError(f"level {k}: sources {[first_src + b + i for i in bad]} did not converge")
            out = np.zeros((3, 2, nops, 16, dims[3], npm), dtype=np.complex128)
            dl_loops_sets(ctx, acc, p2max, out, 0)
            store.save(k, out[DL_SET_LP])
            done.append(k)
    finally:
        dl_accum_destroy(acc)
    return done
