"""CPU check of the per-lane indexing of the two kernels that load the limb
constants per lane with a 64-bit division in the index (the naive radix-2
stage of the design ladder and its separate reduction launch): the index
computation of every lane of every workgroup of their launch grids, restated
here in numpy, stays inside the data, twiddle and constant arrays, and every
(polynomial, coefficient pair) is visited exactly once per stage.  Shapes:
the GPU tests' and the ladder benchmark's [1024][8][2^15].  Also the map of
the direct-to-LDS first load of inverse blocks (which global pair each lane
fetches, where each lane reads its words back)."""
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


def dma_swz(pair):
    """The pair permutation of the direct-to-LDS load (an XOR within groups of eight pairs)."""
    return pair ^ ((pair >> 3) & 7)


@pytest.mark.parametrize("b,e", [(10, 4), (10, 3), (11, 4), (12, 4), (12, 3), (13, 4), (14, 4)])
def test_direct_lds_load_map(b, e):
    """The first load of an inverse block (load_global_m0_fresh): restated over
    every lane of a workgroup of 2^(b-e) lanes.  Every direct-to-LDS
    instruction fills its wave's 1 KB window with 64 pairs fetched from the
    block (all in bounds, each LDS pair written once); each lane then reads
    back exactly its 2^e consecutive words; and the eight pairs an 8-lane
    group reads at one step lie in eight different 16-byte bank groups."""
    lanes = 1 << (b - e)
    assert lanes % 64 == 0
    wave_words = 64 << e
    lds_src = np.full(1 << (b - 1), -1, dtype=np.int64)      # global pair held by each LDS pair
    for wave in range(lanes // 64):
        for i in range(wave_words // 128):
            win = wave * wave_words + 128 * i
            pair = win // 2 + np.arange(64)
            src = dma_swz(pair)
            assert src.min() >= 0 and src.max() < (1 << (b - 1))
            assert (lds_src[pair] == -1).all()                     # each LDS pair written once
            lds_src[pair] = src
    assert (lds_src >= 0).all() and len(np.unique(lds_src)) == lds_src.size
    tid = np.arange(lanes)
    for j in range(1 << (e - 1)):
        want = (tid << (e - 1)) + j                                # the lane's j-th pair of consecutive words
        slot = dma_swz(want)
        assert (lds_src[slot] == want).all()
        for g in range(0, lanes, 8):                               # one 8-lane group per 128-byte LDS access
            assert len(set((slot[g:g + 8] % 8).tolist())) == 8
