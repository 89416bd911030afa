"""The C-ABI library: it loads, exports every declared symbol, and its host-only
logic and argument checks work without a GPU."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

import paper_1401_6750_amd as dl
from oracle import loops

HEADER = os.path.join(os.path.dirname(os.path.dirname(__file__)), "include", "discloop.h")


def declared_functions():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(dl_[a-z_]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    lib = dl.lib()
    names = declared_functions()
    assert len(names) >= 15
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(dl._SIGS)


@pytest.mark.parametrize("dims,cut", [((16, 16, 16, 32), 4), ((24, 24, 24, 48), 4), ((4, 4, 4, 4), 3),
                                      ((4, 4, 4, 4), 4), ((8, 6, 4, 2), 9), ((2, 2, 2, 2), 9),
                                      ((32, 32, 32, 64), 9)])
def test_momentum_list_matches_oracle(dims, cut):
    got = np.array(dl.dl_momenta(dims, cut)).reshape(-1, 3)
    want = loops.momenta(cut, dims)
    assert np.array_equal(got, want)


def test_argument_errors_without_gpu():
    lib = dl.lib()
    assert lib.dl_set_params(None, 0.1, 0.01) == dl.DL_EINVAL
    assert "NULL" in dl.dl_last_error()
    h = ctypes.c_void_p()
    dims = (ctypes.c_int * 4)(4, 4, 4, 4)
    assert lib.dl_lattice_create(None, dims, -1, ctypes.byref(h)) == dl.DL_EINVAL
    n = ctypes.c_int()
    assert lib.dl_momenta(dims, -1, None, 0, ctypes.byref(n)) == dl.DL_EINVAL
    assert lib.dl_solve_batch(None, None, 0, None) == dl.DL_EINVAL
    assert lib.dl_loops(None, None, 0, None, 0, None) == dl.DL_EINVAL
    assert lib.dl_apply_op(None, 0, 0, None, None, 1) == dl.DL_EINVAL
    assert lib.dl_fill_noise(None, 0, 0, 0, None) == dl.DL_EINVAL
    assert lib.dl_accum_counts(None, None) == dl.DL_EINVAL
    # destroying NULL handles is a no-op
    assert lib.dl_destroy(None) == 0
    assert lib.dl_lattice_destroy(None) == 0
    assert lib.dl_accum_destroy(None) == 0
    with pytest.raises(dl.DiscloopError) as e:
        dl.dl_set_params(None, 0.1, 0.0)
    assert e.value.code == dl.DL_EINVAL


def test_struct_layouts_match_header(tmp_path):
    """Sizes and field offsets of the binding's structs equal what a C compiler makes of
    the header."""
    structs = {"dl_job": dl.dl_job, "dl_src_stats": dl.dl_src_stats}
    lines = ['#include <stddef.h>', '#include <stdio.h>', f'#include "{HEADER}"', "int main(void) {"]
    for name, cls in structs.items():
        lines.append(f'  printf("{name} size %zu\\n", sizeof({name}));')
        for f, _ in cls._fields_:
            lines.append(f'  printf("{name} {f} %zu\\n", offsetof({name}, {f}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-o", str(exe), str(src)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l.strip()}
    for name, cls in structs.items():
        assert got[(name, "size")] == ctypes.sizeof(cls), name
        for f, _ in cls._fields_:
            assert got[(name, f)] == getattr(cls, f).offset, (name, f)


def test_binding_refuses_to_run_without_library(monkeypatch, tmp_path):
    monkeypatch.setattr(dl, "_lib", None)
    monkeypatch.setattr(dl, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(ImportError):
        dl.lib()


@pytest.mark.parametrize("dims,seed,eps", [((4, 4, 4, 4), 1401, 0.3), ((6, 2, 4, 8), 7, 0.2),
                                           ((16, 16, 16, 32), 1402, 0.2), ((2, 2, 2, 2), 2**63 + 11, 1.0)])
def test_gauge_random_host_matches_synthetic_generator(dims, seed, eps):
    """dl_gauge_random_host (the library's own link generator, host code) reproduces the
    seeded synthetic ensemble the tests and benchmark build in Python: same counter stream,
    Box-Muller pairs and Gell-Mann generator; the exponentials agree to rounding."""
    import synth
    X, Y, Z, T = dims
    got = np.zeros((T, Z, Y, X, 4, 3, 3), dtype=np.complex128)
    dl.dl_gauge_random_host(dims, seed, eps, got)
    want = synth.random_gauge(dims, seed, eps)
    assert np.abs(got - want).max() < 1e-13
    u = got.reshape(-1, 3, 3)[:500]
    assert np.abs(np.einsum("nab,ncb->nac", u, u.conj()) - np.eye(3)).max() < 1e-13
    assert np.abs(np.linalg.det(u) - 1).max() < 1e-13


def test_gauge_random_host_argument_errors():
    lib = dl.lib()
    dims = (ctypes.c_int * 4)(4, 4, 4, 4)
    assert lib.dl_gauge_random_host(dims, 1, 0.2, None) == dl.DL_EINVAL
    assert lib.dl_gauge_random(None, 1, 0.2) == dl.DL_EINVAL
    buf = np.zeros(4 ** 4 * 4 * 18)
    assert lib.dl_gauge_random_host(dims, 1, float("nan"), buf.ctypes.data) == dl.DL_EINVAL
