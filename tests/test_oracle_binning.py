"""Pins of the integer binning reference: a hand-built example and invariants."""
import numpy as np

from oracle import binning, core
from paper_2603_18707_amd import scenes


def test_hand_built_example():
    # 3 splats on a 3x2 tile grid
    rect = np.array([[0, 0, 1, 0],     # tiles 0, 1
                     [1, 0, 2, 1],     # tiles 1, 2, 4, 5
                     [0, 0, -1, -1]],  # culled
                    np.int32)
    depth = np.array([2.0, 1.0, 0.5], np.float32)
    keys, vals, ranges = binning.bin_and_sort(rect, depth, 3, 2)
    b = lambda d: int(np.float32(d).view(np.uint32))
    exp = [(0 << 32 | b(2.0), 0), (1 << 32 | b(1.0), 1), (1 << 32 | b(2.0), 0), (2 << 32 | b(1.0), 1),
           (4 << 32 | b(1.0), 1), (5 << 32 | b(1.0), 1)]
    assert [(int(k), int(v)) for k, v in zip(keys, vals)] == exp
    assert ranges.tolist() == [[0, 1], [1, 3], [3, 4], [0, 0], [4, 5], [5, 6]]


def test_equal_keys_keep_index_order():
    rect = np.array([[0, 0, 0, 0]] * 4, np.int32)
    depth = np.array([1.0, 1.0, 0.5, 1.0], np.float32)
    _, vals, _ = binning.bin_and_sort(rect, depth, 1, 1)
    assert vals.tolist() == [2, 0, 1, 3]


def test_invariants_and_fast_path():
    sc, cam = scenes.workload_tiny()
    p = core.project(sc, cam, core.Cfg(kind=core.KERNEL_EXP, radius_mode=core.RADIUS_SIGMA3))
    gx, gy = 8, 8
    keys, vals, ranges = binning.bin_and_sort(p["rect"], p["depth32"], gx, gy)
    assert keys.shape[0] == int(p["tiles"].sum())
    assert np.all(keys[1:] >= keys[:-1])
    nz = ranges[ranges[:, 1] > ranges[:, 0]]
    assert nz[0, 0] == 0 and nz[-1, 1] == keys.shape[0] and np.all(nz[1:, 0] == nz[:-1, 1])
    k2, v2, r2 = binning.bin_and_sort_fast(p["rect"], p["depth32"], gx, gy)
    assert np.array_equal(keys, k2) and np.array_equal(vals, v2) and np.array_equal(ranges, r2)
    # each tile's copies are exactly the splats whose rectangle contains it
    for t in range(gx * gy):
        tx, ty = t % gx, t // gx
        r = p["rect"]
        inside = np.nonzero((r[:, 0] <= tx) & (tx <= r[:, 2]) & (r[:, 1] <= ty) & (ty <= r[:, 3]))[0]
        got = vals[ranges[t, 0]:ranges[t, 1]]
        assert sorted(got.tolist()) == inside.tolist()


def test_tile_histogram_and_tile_list_match_the_full_binning():
    """The per-tile helpers used at frame sizes too large to bin whole agree
    with the full loop binning (ties in depth included)."""
    sc, cam = scenes.workload_tiny()
    sc.scales *= 2.0
    p = core.project(sc, cam, core.Cfg(kind=core.KERNEL_EXP, radius_mode=core.RADIUS_SIGMA3))
    depth = p["depth32"].copy()
    depth[1::7] = depth[0]  # equal depths must fall back to index order
    gx, gy = 8, 8
    keys, vals, ranges = binning.bin_and_sort(p["rect"], depth, gx, gy)
    hist = binning.tile_histogram(p["rect"], gx, gy)
    assert np.array_equal(hist, (ranges[:, 1].astype(np.int64) - ranges[:, 0]))
    assert hist.sum() == keys.shape[0]
    for t in range(gx * gy):
        kb, v = binning.tile_list(p["rect"], depth, t % gx, t // gx)
        lo, hi = ranges[t]
        assert np.array_equal(v, vals[lo:hi])
        assert np.array_equal(kb.astype(np.uint64), keys[lo:hi] & np.uint64(0xFFFFFFFF))


def test_tile_histogram_edges():
    rect = np.array([[0, 0, 2, 1], [2, 1, 2, 1], [1, 0, 0, 0], [0, 0, -1, -1]], np.int32)
    h = binning.tile_histogram(rect, 3, 2).reshape(2, 3)
    assert h.tolist() == [[1, 1, 1], [1, 1, 2]]
