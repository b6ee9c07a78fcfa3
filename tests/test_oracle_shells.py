"""Pins of the |k|-shell binning (oracle.shells).

Bins are equal-width in |k| on (0, sqrt(3) k_Ny]; a mode with |k| exactly on
an edge belongs to the upper bin, the corner mode to the last bin.  The pin
enumerates every full-grid mode and places it with exact rational arithmetic
on (|k| / dk)^2 = 4 n_bins^2 q / (3 N^2), independently of the thresholds.
"""
import math
from fractions import Fraction

import numpy as np
import pytest

from oracle import shells


def brute_force_counts(n, n_bins):
    counts = np.zeros(n_bins, dtype=np.int64)
    m = [i if i <= n // 2 else i - n for i in range(n)]
    for mx in m:
        for my in m:
            for mz in m:
                q = mx * mx + my * my + mz * mz
                if q == 0:
                    continue
                x = Fraction(4 * n_bins * n_bins * q, 3 * n * n)   # (|k|/dk)^2
                b = math.isqrt(x.numerator // x.denominator)      # floor(|k|/dk)
                counts[min(b, n_bins - 1)] += 1
    return counts


@pytest.mark.parametrize("n,n_bins", [(8, 4), (8, 6), (12, 5), (16, 8), (16, 16), (24, 7)])
def test_mode_counts_brute_force(n, n_bins):
    got = shells.mode_counts(n, n_bins)
    assert np.array_equal(got, brute_force_counts(n, n_bins))
    assert got.sum() == n ** 3 - 1


@pytest.mark.parametrize("n,n_bins", [(32, 16), (64, 16), (128, 32), (256, 64), (48, 16), (96, 16)])
def test_total_and_edge_ties(n, n_bins):
    counts = shells.mode_counts(n, n_bins)
    assert counts.sum() == n ** 3 - 1
    q_edges = shells.thresholds(n, n_bins)
    # the threshold of bin b is the least q whose |k| reaches b * dk
    for b in range(1, n_bins):
        qb = int(q_edges[b])
        assert 4 * n_bins ** 2 * qb >= 3 * b * b * n * n
        assert 4 * n_bins ** 2 * (qb - 1) < 3 * b * b * n * n
    # a q exactly on an edge goes to the upper bin
    if (3 * n * n) % (4 * n_bins ** 2) == 0:
        step = 3 * n * n // (4 * n_bins ** 2)
        qs = np.array([step * b * b for b in range(1, n_bins)])
        assert np.array_equal(shells.bin_of_q(qs, n, n_bins), np.arange(1, n_bins))
    # the corner mode is in the last bin
    assert shells.bin_of_q(np.array([3 * (n // 2) ** 2]), n, n_bins)[0] == n_bins - 1
    assert shells.bin_of_q(np.array([0]), n, n_bins)[0] == -1


def test_half_grid_weights_cover_full_grid():
    n = 8
    w = shells.half_grid_weight(n)
    assert w.sum() * n * n == n ** 3
