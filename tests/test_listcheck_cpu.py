"""The test helper that turns an oracle stencil into the compact path's
expected tile-order lists, stencil words and ranks, against a brute-force
walk over the tiles (so the GPU list tests rest on a checked expectation)."""
import numpy as np
import pytest

from listcheck import tile_order


@pytest.mark.parametrize("Hi,Wi,tw,tr", [(70, 96, 2, 8), (33, 64, 1, 4), (40, 128, 3, 5), (64, 512, 16, 32)])
def test_tile_order_brute_force(Hi, Wi, tw, tr):
    rng = np.random.default_rng(Hi * Wi)
    st = (rng.random((Hi, Wi)) < 0.3).astype(np.uint8)
    lst, words, ranks = tile_order(st, tw, tr)
    wpr = Wi // 32
    tx, ty = -(-wpr // tw), -(-Hi // tr)
    exp, er = [], np.zeros((Hi, wpr), np.uint32)
    for T in range(tx * ty):
        by, bx = divmod(T, tx)
        for y in range(by * tr, min(Hi, by * tr + tr)):
            for w in range(bx * tw, min(wpr, bx * tw + tw)):
                er[y, w] = len(exp)
                exp += [y * Wi + w * 32 + b for b in range(32) if st[y, w * 32 + b]]
    assert np.array_equal(lst, np.array(exp))
    assert np.array_equal(ranks, er)
    for y in range(Hi):
        for w in range(wpr):
            assert words[y, w] == sum(int(st[y, w * 32 + b]) << b for b in range(32))
