"""CPU check of the per-lane indexing of the two kernels that load the limb
constants per lane with a 64-bit division in the index (the naive radix-2
stage of the design ladder and its separate reduction launch): the index
computation of every lane of every workgroup of their launch grids, restated
here in numpy, stays inside the data, twiddle and constant arrays, and every
(polynomial, coefficient pair) is visited exactly once per stage.  Shapes:
the GPU tests' and the ladder benchmark's [1024][8][2^15]."""
import numpy as np
import pytest


def naive_stage_indices(units, limbs, logn, s, gid):
    """k_naive_stage: one butterfly per lane; returns (valid, word j, word j+gap, twiddle, constant)."""
    lh = logn - 1
    unit = gid >> np.uint64(lh)
    valid = unit < units
    i = (gid & np.uint64((1 << lh) - 1)).astype(np.uint64)
    limb = unit % np.uint64(limbs)
    lt = lh - s
    grp = i >> np.uint64(lt)
    j = (grp << np.uint64(lt + 1)) | (i & np.uint64((1 << lt) - 1))
    base = unit << np.uint64(logn)
    tw = (limb << np.uint64(logn + 1)) + np.uint64(1 << s) + grp
    return valid, base + j, base + j + np.uint64(1 << lt), tw, limb


@pytest.mark.parametrize("batch,limbs,logn", [(2, 3, 6), (2, 3, 12), (2, 3, 15), (2, 3, 17), (1024, 8, 15)])
def test_naive_stage_lanes_in_bounds(batch, limbs, logn):
    """Every lane of the grid for the test shapes (and every word visited
    once per stage); for the benchmark shape, every lane of the first and last
    4096 workgroups and a lane of every 1009th in between."""
    units = batch * limbs
    words = units << logn
    grid = ((units << (logn - 1)) + 255) // 256
    total = grid * 256
    full = words <= (1 << 22)
    if full:
        gids = [np.arange(0, total, dtype=np.uint64)]
    else:
        gids = [np.arange(0, 4096 * 256, dtype=np.uint64), np.arange(total - 4096 * 256, total, dtype=np.uint64),
                np.arange(0, total, 1009 * 256 + 17, dtype=np.uint64)]
    for s in range(logn):
        seen = np.zeros(words, dtype=np.uint8) if full else None
        for gid in gids:
            valid, a, b, tw, limb = naive_stage_indices(units, limbs, logn, s, gid)
            a, b, tw, limb = a[valid], b[valid], tw[valid], limb[valid]
            assert a.size == 0 or (int(b.max()) < words and int(tw.max()) < limbs * 2 * (1 << logn)
                                   and int(limb.max()) < limbs)
            assert np.all((tw & np.uint64((2 << logn) - 1)) < np.uint64(1 << logn))   # forward table half
            if seen is not None:
                np.add.at(seen, a.astype(np.int64), 1)
                np.add.at(seen, b.astype(np.int64), 1)
        if seen is not None:
            assert np.all(seen == 1), (s, int(seen.min()), int(seen.max()))     # each word once per stage


@pytest.mark.parametrize("batch,limbs,logn", [(2, 3, 6), (2, 3, 17), (1024, 8, 15)])
def test_reduce_launch_lanes_in_bounds(batch, limbs, logn):
    words = (batch * limbs) << logn
    grid = (words + 255) // 256
    gid = np.arange(0, grid * 256, 997, dtype=np.uint64)        # a sampled lane of every few workgroups
    gid = np.concatenate([gid, np.arange(grid * 256 - 512, grid * 256, dtype=np.uint64)])
    valid = gid < np.uint64(words)
    limb = (gid[valid] >> np.uint64(logn)) % np.uint64(limbs)
    assert int(limb.max()) < limbs and int(gid[valid].max()) == words - 1
