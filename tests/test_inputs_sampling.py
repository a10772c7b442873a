"""The shared counter-based point sampler (nnm_inputs.sampling) against the
published definition of splitmix64."""

import numpy as np

from nnm_inputs.sampling import box_points, splitmix64_at


def test_splitmix64_reference_outputs():
    # first three outputs of splitmix64 from state 0 (Vigna's reference generator)
    got = splitmix64_at(0, np.arange(3, dtype=np.uint64))
    assert [int(v) for v in got] == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]


def test_box_points_layout_and_range():
    x, t = box_points(5, 1000, -1.5, 1.5)
    assert x.dtype == np.float32 and x.shape == (1000, 3) and t.shape == (1000,)
    assert x.min() >= -1.5 and x.max() < 1.5 and t.min() >= 0.0 and t.max() < 1.0
    # point i uses stream positions 4 i .. 4 i + 3: a window of the sequence is a slice of it
    x2, t2 = box_points(5, 10, -1.5, 1.5, first=37)
    assert np.array_equal(x2, x[37:47]) and np.array_equal(t2, t[37:47])
    # coordinate c of point i is the top 24 bits of output 4 i + c, mapped affinely
    u = (splitmix64_at(5, np.array([4 * 3 + 1], np.uint64)) >> np.uint64(40)).astype(np.float64) / 2 ** 24
    assert x[3, 1] == np.float32(-1.5 + 3.0 * u[0])
