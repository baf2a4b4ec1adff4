"""The byte model that bench.py prices the kernels against (CPU only)."""

import math

import bench


def test_whole_step_model_at_2560():
    # 722.3 MB per slice for forward + adjoint at 2560^2, 1024 angles, 2560 bins
    # (349.9 MB forward, 372.4 MB adjoint)
    assert abs(bench.model_bytes_per_slice(2560, 2560, 1024) / 1e6 - 722.3) < 0.05


def test_stage_bytes_add_up_to_the_model():
    # the per-stage accounting covers the whole-step model once, plus the
    # spreading's point list
    for n, nd, na in ((2560, 2560, 1024), (1280, 1280, 256), (512, 640, 97)):
        sb = bench.stage_bytes(n, nd, na, 0)
        assert math.isclose(sum(sb.values()), bench.model_bytes_per_slice(n, nd, na), rel_tol=1e-12)
        assert bench.stage_bytes(n, nd, na, 1000)["spread"] == sb["spread"] + 4000


def test_traffic_summary_is_tied_to_launch_size():
    # a summary taken with another number of slices per launch is never used
    assert bench.measured_traffic("fwd_cols", 2560, 1024, 3.0) is None
    assert bench.measured_traffic("fwd_cols", 1280, 256, 8.0) is None
