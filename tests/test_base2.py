"""Base-2 storage of loop partial sums (CPU): level bookkeeping, the paper's worked
example, estimates rebuilt from level files, resume and stream checks."""
import json
import os

import numpy as np
import pytest

from paper_1401_6750_amd import base2

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "base2_fig2.txt")


def test_worked_example_of_fig2():
    """13 sources = files of weights 1, 4 and 8 (Fig. 2)."""
    rows = [l.split() for l in open(GOLDEN) if l.strip() and not l.startswith("#")]
    for row in rows:
        n, mask = int(row[0]), [int(x) for x in row[1:]]
        assert [1 << k for k, m in enumerate(mask) if m] == [1 << k for k in base2.levels_for(n)]
        assert sum(w * m for w, m in zip((1, 2, 4, 8), mask)) == n


def test_levels_partition_the_stream():
    for K in range(1, 12):
        covered = []
        for k in range(K):
            b, e = base2.level_sources(k)
            assert e - b == 1 << k
            covered += list(range(b, e))
        assert covered == list(range((1 << K) - 1))
    for n in range(1, 300):
        assert sum(1 << k for k in base2.levels_for(n)) == n
    with pytest.raises(ValueError):
        base2.levels_for(-1)


def test_estimates_rebuilt_from_levels(tmp_path):
    """Every n < 2^K gives the mean over exactly the sources of its levels' blocks."""
    rng = np.random.default_rng(3)
    K = 5
    per_source = rng.normal(size=((1 << K) - 1, 2, 3, 4)) + 1j * rng.normal(size=((1 << K) - 1, 2, 3, 4))
    st = base2.Base2Store(str(tmp_path / "s"), {"seed": 1, "tier": "bf16"})
    for k in range(K):
        b, e = base2.level_sources(k)
        st.save(k, per_source[b:e].sum(axis=0))
    assert st.levels() == list(range(K)) and st.resume_level() == K
    for n in range(1, 1 << K):
        idx = [r for k in base2.levels_for(n) for r in range(*base2.level_sources(k))]
        assert len(idx) == n
        np.testing.assert_allclose(st.estimate(n), per_source[idx].mean(axis=0), rtol=1e-13, atol=1e-13)


def test_resume_and_stream_identity(tmp_path):
    d = str(tmp_path / "s")
    st = base2.Base2Store(d, {"seed": 7, "dims": [4, 4, 4, 4]})
    for k in (0, 1, 3):
        st.save(k, np.full((2,), k, dtype=np.complex128))
    assert st.resume_level() == 2
    with pytest.raises(KeyError):
        st.total(4)                      # level 2 missing
    assert np.array_equal(st.total(9), np.full((2,), 3, dtype=np.complex128))   # levels 0 and 3
    again = base2.Base2Store(d, {"dims": [4, 4, 4, 4], "seed": 7})
    assert again.levels() == [0, 1, 3]
    with pytest.raises(ValueError):
        base2.Base2Store(d, {"seed": 8, "dims": [4, 4, 4, 4]})
    assert json.load(open(os.path.join(d, "meta.json"))) == {"dims": [4, 4, 4, 4], "seed": 7}
    assert not [f for f in os.listdir(d) if "tmp" in f]
