"""Host check of the tile passes' division-free quotients (small_quot in
csrc/sph_tiles.hpp): for 0 <= c < 2^10 and 1 <= d <= 144, truncating the
FP32 product (c + 1/2) * fl(1/d) gives floor(c / d) exactly, also with the
reciprocal one ulp off either way (the hardware reciprocal's error).  The
union-cell and target-cell coordinates of every tile rest on it."""
import numpy as np


def test_small_quot_exact_over_its_range():
    c = np.arange(1024, dtype=np.int64)
    cf = c.astype(np.float32) + np.float32(0.5)
    for d in range(1, 145):
        inv = np.float32(1.0) / np.float32(d)
        for invd in (inv, np.nextafter(inv, np.float32(0.0)), np.nextafter(inv, np.float32(1.0))):
            q = (cf * np.float32(invd)).astype(np.int64)
            assert np.array_equal(q, c // d), d


def test_union_coords_roundtrip():
    # (x, y, z) from c by two small quotients, for every union box shape
    for uw in range(1, 13):
        for uh in range(1, 13):
            wh = uw * uh
            c = np.arange(min(1024, wh * 12), dtype=np.int64)
            z = ((c.astype(np.float32) + np.float32(0.5)) * (np.float32(1.0) / np.float32(wh))).astype(np.int64)
            r = c - z * wh
            y = ((r.astype(np.float32) + np.float32(0.5)) * (np.float32(1.0) / np.float32(uw))).astype(np.int64)
            x = r - y * uw
            assert np.array_equal(x + uw * (y + uh * z), c)
            assert (x >= 0).all() and (x < uw).all() and (y >= 0).all() and (y < uh).all()
