"""Consistency of the stored expected values (CPU only).

* The paper's printed S-ADI tables: each printed order is log2 of the ratio of the two
  printed errors it is computed from, up to the rounding of the printed digits, so a
  transcription slip in either shows here.
* The oracle's stored 1000-step runs (tests/golden/make_long_runs.py): one file per
  configured grid and order, with the sample nodes the generator defines and finite values;
  and the second runs at another embedding size, close to the first but not identical.
"""
import importlib.util
import math
import os

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


def test_printed_orders_match_printed_errors(golden):
    tables = golden["s_adi_tables"]
    count = 0
    for name, t in tables.items():
        if name.startswith("_"):
            continue
        assert len(t["steps"]) == 4
        for row in t["rows"]:
            e, o = row["error"], row["order"]
            assert len(e) == 4 and o[0] is None
            for k in range(1, 4):
                # errors carry five significant digits: their ratio is known to ~1e-4 in log2
                assert abs(math.log2(e[k - 1] / e[k]) - o[k]) <= 1.5e-4, (name, row["alpha"], k)
                count += 1
            # the steps halve from one row to the next (second-order convergence tables)
            assert all(abs(t["steps"][k] / t["steps"][k + 1] - 2.0) < 1e-12 for k in range(3))
    assert count == 36


def _generator():
    spec = importlib.util.spec_from_file_location("make_long_runs", os.path.join(HERE, "golden", "make_long_runs.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


@pytest.mark.parametrize("n,alpha,embed", [(1023, 1.2, None), (1023, 1.5, None), (1023, 1.8, None),
                                           (2047, 1.2, None), (2047, 1.5, None), (2047, 1.8, None),
                                           (4095, 1.2, None), (4095, 1.5, None), (4095, 1.8, None),
                                           (2047, 1.8, 4096), (4095, 1.5, 8192), (4095, 1.8, 8192)])
def test_stored_long_runs(n, alpha, embed):
    gen = _generator()
    path = gen.path_for(n, alpha, embed)
    assert os.path.exists(path), "stored oracle run missing (tests/golden/make_long_runs.py)"
    with np.load(path, allow_pickle=False) as z:
        meta, idx = z["meta"], z["idx"]
        prev, cur, fmax, fl2 = z["prev"], z["cur"], z["full_max"], z["full_l2"]
    assert int(meta[0]) == n and meta[1] == alpha and meta[2] == 1e-3 and int(meta[3]) == 1000
    assert np.array_equal(idx, gen.sample_indices(n))
    assert prev.shape == cur.shape == idx.shape
    assert np.all(np.isfinite(prev)) and np.all(np.isfinite(cur))
    # the sample holds the centre lines, so it reaches the whole grid's maximum closely
    assert np.abs(cur).max() <= fmax[1] and np.abs(prev).max() <= fmax[0]
    assert np.abs(cur).max() >= 0.5 * fmax[1]
    assert fl2[1] > 0 and not np.array_equal(prev, cur)
    if embed is not None:
        # the second embedding changes only the rounding: the two oracle runs agree closely
        # but not bit for bit
        with np.load(gen.path_for(n, alpha), allow_pickle=False) as z:
            base = z["cur"]
        d = np.abs(base - cur).max() / fmax[1]
        assert 0.0 < d < 1e-8
