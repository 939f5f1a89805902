"""Host checks of the profile summaries the benchmark reads (no GPU)."""
import json
import os

import pytest

from paper_2312_06206_amd import profiling as P

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_kernel_keys_match_the_step_kernels():
    m = 4096
    names = {
        "void sadi::cols_gs_fwd_kernel<4096, 1>(double const*, int, ...)": "cols_gs_fwd",
        "void sadi::cols_conv_kernel<4096>(HIP_vector_type<double, 2u>*, int, ...)": "cols_conv",
        "void sadi::rows_rhs_gs_kernel<4096, 0, 1, 1>(HIP_vector_type<double, 2u> const*, ...)": "rows_rhs_gs",
        "void sadi::rows_fwd_kernel<4096, 0, 0>(double const*, double*, ...)": "rows_fwd",
        # not step kernels of a run
        "void sadi::rows_rhs_gs_kernel<4096, 1, 1, 0>(...)": None,
        "void sadi::rows_rhs_gs_kernel<4096, 0, 1, 0>(...)": None,
        "void sadi::cols_gs_fwd_kernel<4096, 0>(...)": None,
        "void sadi::cols_gs_kernel<4096, 2, 0>(...)": None,
        "void sadi::cols_conv_kernel<1024>(...)": None,
        "void sadi::cols_conv_batched<4096>(...)": None,
    }
    for name, key in names.items():
        assert P.kernel_key(name, m) == key, name


def test_committed_profiles_cover_every_step_kernel():
    steps = ("cols_conv", "rows_rhs_gs", "cols_gs_fwd")
    current = True
    for fname in ("hbm_counters_N4095.json", "valu_counters_N4095.json"):
        with open(os.path.join(ROOT, "profiles", fname)) as f:
            rec = json.load(f)
        assert "rocprofv3" in rec["command"]
        for k in steps:
            assert k in rec["kernels"], (fname, k)
        current = current and rec["source_hash"] == P.source_hash()
    with open(os.path.join(ROOT, "profiles", "kernel_trace_sadi_fp64_N4095.md")) as f:
        trace = f.read()
    for k in steps:
        assert f"| {k} |" in trace, k
    if not current:
        pytest.skip("kernel sources changed since the counters were taken (the bench reports traffic null)")
    for k in steps:
        assert P.traffic_for(k) > 0
        v = P.valu_for(k)
        assert v["SQ_INSTS_VALU"] > 0 and v["fp64_flops"] > 0
