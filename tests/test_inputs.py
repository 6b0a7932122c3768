"""The seeded input generator follows the published SplitMix64 definition."""
import numpy as np

from paper_2403_06218_amd import inputs


def test_splitmix64_reference_outputs():
    """First three outputs of SplitMix64 seeded with 0 (Vigna's splitmix64.c)."""
    with np.errstate(over="ignore"):
        got = [int(inputs._mix(np.uint64(k) * inputs.GAMMA)) for k in (1, 2, 3)]
    assert got == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]


def test_stream_layout_and_ranges():
    A = inputs.uniform_matrix(37, 11, seed=5)
    assert A.flags["F_CONTIGUOUS"] and A.shape == (37, 11)
    assert A.min() >= -1.0 and A.max() < 1.0
    np.testing.assert_array_equal(inputs.uniform_rows(37, 11, 5, [0, 36, 7]), A[[0, 36, 7]])
    np.testing.assert_array_equal(inputs.uniform_cols(37, 11, 5, [10, 2]), A[:, [10, 2]])
    B = inputs.uniform_matrix(37, 11, seed=5, lo=-0.5, hi=0.5)
    np.testing.assert_array_equal(B, A / 2)   # both affine maps are exact
    assert not np.array_equal(A, inputs.uniform_matrix(37, 11, seed=6))


def test_uniform_moments():
    u = inputs.uniform01(3, np.arange(200000, dtype=np.uint64))
    assert abs(u.mean() - 0.5) < 5e-3 and abs(u.var() - 1 / 12) < 2e-3


def test_diag_dominant_and_batch_sizes():
    A = inputs.diag_dominant(50, seed=1)
    off = np.abs(A).sum(axis=1) - np.abs(np.diag(A))
    assert np.all(np.diag(A) > off)
    n = inputs.batch_sizes(10000, 8, 256, seed=0)
    assert n.min() == 8 and n.max() == 256 and abs(n.mean() - 132) < 2
