"""Host-side arithmetic of the benchmark: the algorithmic byte counts that the
roofline fractions are priced on.

touched_rows is checked against the oracle's tap indices (eqs. 1-4 with
clamp-to-edge): the number of distinct clamped source indices over every
output index, for growing, shrinking, identity and strongly shrinking axes.
"""

import numpy as np
import pytest

import bench
from oracle import ref_resize as ref

AXES = [(1, 1), (1, 7), (7, 1), (2, 3), (64, 128), (512, 1024), (1024, 512),
        (1000, 333), (2048, 256), (2048, 300), (97, 24), (96, 24), (300, 75),
        (300, 74), (64, 16), (63, 16), (5, 7), (1024, 1024)]


@pytest.mark.parametrize("n_in,n_out", AXES)
@pytest.mark.parametrize("filt", [ref.BILINEAR, ref.BICUBIC])
def test_touched_rows_is_union_of_clamped_taps(n_in, n_out, filt):
    idx, _, _, _ = ref.axis_taps(n_in, n_out, filt)
    taps = 4 if filt == ref.BICUBIC else 2
    assert bench.touched_rows(n_in, n_out, taps) == len(np.unique(idx))


def test_touched_rows_every_row_unless_shrinking_past_the_reach():
    # Windows of K taps at spacing n_in / n_out leave no gap while the spacing
    # is at most K, so every source row is read.
    for n_in, n_out in [(2048, 1024), (2048, 4096), (999, 500)]:
        assert bench.touched_rows(n_in, n_out, 2) == n_in
        assert bench.touched_rows(n_in, n_out, 4) == n_in
    # x0.25 bilinear: two of every four rows.
    assert bench.touched_rows(2048, 512, 2) == 1024


def test_batch_alg_bytes_counts_touched_pixels_and_outputs():
    class Job:
        def __init__(self, in_h, in_w, out_h, out_w, channels, filt):
            self.in_h, self.in_w, self.out_h, self.out_w = in_h, in_w, out_h, out_w
            self.channels, self.filter = channels, filt

    jobs = [Job(512, 512, 1024, 1024, 4, 0), Job(2048, 1024, 512, 256, 1, 0),
            Job(300, 200, 75, 50, 3, 1)]
    want = (512 * 512 * 4 + 1024 * 1024 * 4
            + 1024 * 512 * 1 + 512 * 256 * 1
            + 300 * 200 * 3 + 75 * 50 * 3)
    assert bench.batch_alg_bytes(jobs) == want
