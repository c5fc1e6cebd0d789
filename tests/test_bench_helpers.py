"""Host-side pieces of the benchmark that compute something: the exact DCT
used as the comparison in the quality sweep is the orthonormal DCT-II."""
import numpy as np

import bench


def test_dct_reference_is_orthonormal_dct2():
    C = bench.dct2_matrix()
    assert np.allclose(C @ C.T, np.eye(8), atol=1e-14)
    assert np.allclose(C[0], 1 / np.sqrt(8))
    assert np.isclose(C[1, 0], np.cos(np.pi / 16) / 2)
    assert np.isclose(C[4, 1], -np.sqrt(2) / 4)  # cos(3*4*pi/16) * 1/2
    # DC of a constant block is 8x the value; a ramp has no even-order AC
    x = np.arange(8, dtype=float)
    y = C @ x
    assert np.allclose(y[2::2], 0, atol=1e-12)


def test_launch_shape_parsing():
    """--tune / --fused-tune accept 3 to 5 fields; missing ones are 0."""
    assert bench.parse_tune("4,1,2") == dict(waves_per_group=4, groups_per_cu=1, tile_waves=2,
                                             xcd_remap=0, pixel_cache=0)
    assert bench.parse_tune("2,4096,1,1") == dict(waves_per_group=2, groups_per_cu=4096, tile_waves=1,
                                                  xcd_remap=1, pixel_cache=0)
    assert bench.parse_tune("8,1,1,0,1") == dict(waves_per_group=8, groups_per_cu=1, tile_waves=1,
                                                 xcd_remap=0, pixel_cache=1)
    for bad in ("4,1", "1,2,3,4,5,6"):
        try:
            bench.parse_tune(bad)
        except SystemExit:
            continue
        raise AssertionError(bad)


def test_config_numbers_name_known_legs():
    """--config N runs the headline step and workload N's leg (2: the step
    alone); other numbers, or --config with --legs, are refused before any
    GPU work."""
    import subprocess
    import sys
    assert sorted(bench.CONFIG_LEGS) == [1, 2, 3, 4, 5]
    assert bench.CONFIG_LEGS[2] == ""
    for legs in bench.CONFIG_LEGS.values():
        assert legs in ("", "latency_512", "batched", "video", "serving")
    for args in (["--config", "6"], ["--config", "3", "--legs", "video"], ["--config", "1", "--no-extras"]):
        r = subprocess.run([sys.executable, bench.__file__] + args, capture_output=True, text=True, timeout=60)
        assert r.returncode == 2 and "--config" in r.stderr
