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
