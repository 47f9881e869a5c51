"""Expected compact-path lists from the oracle's stencils (test helper).

The frame path stores each level's work list in ranking-tile order: tiles of
tile_words x tile_rows stencil words (32 texels each), row-major over the
level; inside a tile, texels in row-major order.  This is a fixed
permutation of the oracle's row-major list (Sec. 4.1 stencil texels), so the
expected list, stencil words and per-word ranks follow from the oracle's
stencil alone."""
import numpy as np


def tile_order(stencil, tile_words=16, tile_rows=32):
    """(list, stencil words, ranks) the compact path must produce for a level
    stencil u8 [H_i][W_i] (W_i divisible by 32)."""
    Hi, Wi = stencil.shape
    wpr = Wi // 32
    tiles_x = -(-wpr // tile_words)
    ys, xs = np.nonzero(stencil)
    tile = (ys // tile_rows) * tiles_x + (xs // 32) // tile_words
    key = tile.astype(np.int64) * (Hi * Wi) + ys.astype(np.int64) * Wi + xs
    order = np.argsort(key, kind="stable")
    lst = (ys.astype(np.int64) * Wi + xs)[order]
    keys = key[order]
    wy, ww = np.divmod(np.arange(Hi * wpr), wpr)
    wtile = (wy // tile_rows) * tiles_x + ww // tile_words
    wkey = wtile.astype(np.int64) * (Hi * Wi) + wy.astype(np.int64) * Wi + ww * 32
    ranks = np.searchsorted(keys, wkey).astype(np.uint32).reshape(Hi, wpr)
    bits = np.packbits(stencil.astype(bool).reshape(Hi, wpr, 32), axis=-1, bitorder="little")
    words = bits.reshape(Hi, wpr, 4).copy().view("<u4").reshape(Hi, wpr)
    return lst, words, ranks


def check_frame_lists(got, pyramid, tile_words=16, tile_rows=32):
    """got: FrameRunner.lists(); pyramid: the oracle's.  Bit-exact lists,
    stencil words and ranks for every list level; also checks that sorting
    the list gives the oracle's row-major list."""
    L = pyramid.levels[-1]
    levels = [i for i in pyramid.levels if i != L]
    assert sorted(got) == levels, (sorted(got), levels)
    for i in levels:
        lst, words, ranks = got[i]
        e_lst, e_words, e_ranks = tile_order(pyramid.stencil[i], tile_words, tile_rows)
        assert len(lst) == len(pyramid.worklist[i]), f"count level {i}"
        assert np.array_equal(words, e_words), f"stencil words level {i}"
        assert np.array_equal(lst, e_lst), f"list level {i}"
        assert np.array_equal(np.sort(lst), pyramid.worklist[i].astype(np.int64)), f"list set level {i}"
        assert np.array_equal(ranks, e_ranks), f"ranks level {i}"
