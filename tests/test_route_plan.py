"""CPU checks of the routed table-gradient scatter's invariants (the layout the kernels rely on).

The training kernel sends each corner x-pair (the corners at dx = 0 and 1 of
one (dy, dz)) of every (sample, level) to the 2^k-entry partition of its first
entry; the pair's second entry must lie in the same partition, except on dense
levels where the first entry is a partition's last (those pairs bypass the
routing).  Summing the records per partition must give the plain scatter.
"""
import numpy as np
import pytest

from oracle import hashgrid


def route(pos, res, T, k, dense):
    idx, w = hashgrid.corners(pos, res, T)
    M = (1 << k) - 1
    e0 = idx[:, 0::2]          # corners 0, 2, 4, 6: dx = 0
    e1 = idx[:, 1::2]          # corners 1, 3, 5, 7: dx = 1
    straddle = dense & ((e0 & M) == M)
    return idx, w, e0, e1, straddle


@pytest.mark.parametrize("growth,T,levels", [(1.447, 1 << 19, 16), (1.447, 1 << 20, 16), (1.5, 1 << 14, 8),
                                             (1.5, 1 << 14, 10)])
def test_pairs_share_a_partition(growth, T, levels):
    rng = np.random.default_rng(0)
    pos = rng.uniform(0, 1, size=(20000, 3)).astype(np.float32)
    pos[:4] = [[1, 1, 1], [0, 0, 0], [1, 0, 1], [0.999999, 0.5, 0.25]]
    k = 12
    for r in hashgrid.level_resolutions(16, growth, levels):
        dense = hashgrid.level_is_dense(r, T)
        if not dense and T > (1 << k):
            assert r < (1 << k)         # the plan's condition for hashed levels
        idx, w, e0, e1, straddle = route(pos, r, T, k, dense)
        same = (e0 >> k) == (e1 >> k)
        assert np.all(same | straddle)
        if not dense:
            assert not straddle.any()
        else:
            assert np.all(e1 == e0 + 1)
        entries = (r + 1) ** 3 if dense else T
        assert e0.max() < entries and e1.max() < entries


def test_routed_sum_equals_plain_scatter():
    rng = np.random.default_rng(1)
    pos = rng.uniform(0, 1, size=(5000, 3)).astype(np.float32)
    T, k, F = 1 << 14, 12, 2
    for r in (16, 24, 36, 81, 273):
        dense = hashgrid.level_is_dense(r, T)
        entries = (r + 1) ** 3 if dense else T
        d = rng.normal(size=(5000, F))
        idx, w, e0, e1, straddle = route(pos, r, T, k, dense)
        plain = np.zeros((entries, F))
        np.add.at(plain, idx.reshape(-1), (w[:, :, None] * d[:, None, :]).reshape(-1, F))
        routed = np.zeros((entries, F))
        M = (1 << k) - 1
        v0 = w[:, 0::2, None] * d[:, None, :]
        v1 = w[:, 1::2, None] * d[:, None, :]
        keep = ~straddle
        bucket = e0 >> k
        for b in np.unique(bucket[keep]):
            sel = keep & (bucket == b)
            part = np.zeros((1 << k, F))
            np.add.at(part, e0[sel] & M, v0[sel])
            np.add.at(part, e1[sel] & M, v1[sel])
            lo = b << k
            hi = min(entries, lo + (1 << k))
            routed[lo:hi] += part[:hi - lo]
        np.add.at(routed, e0[straddle], v0[straddle])
        np.add.at(routed, e1[straddle], v1[straddle])
        assert np.allclose(routed, plain, atol=1e-12)
