"""gs_bin_sort alone on the GPU, through the C ABI, against the oracle's
binning (oracle.binning), bit for bit: keys, values, tile ranges and the key
count, on seeded synthetic rectangles and depths (scenes.binning_inputs) with
depth ties, culled splats and splats spanning up to the whole grid. Grid
shapes cover one, two and four tile-digit passes and per-tile lists longer
than one LDS chunk; capacities cover the exact fit, one short (overflow) and
zero.
"""
import numpy as np
import pytest
import torch

from oracle import binning
from paper_2603_18707_amd import _lib as L
from paper_2603_18707_amd import scenes

pytestmark = pytest.mark.gpu


def _run(depth, rect, tiles, gw, gh, capacity, with_order=True):
    dev = torch.device("cuda", 0)
    n = depth.shape[0]
    d = torch.from_numpy(depth).to(dev)
    r = torch.from_numpy(rect).to(dev)
    t = torch.from_numpy(tiles.view(np.int32)).to(dev)
    ntiles = gw * gh
    ws_bytes = L.gs_bin_sort_workspace(n, capacity, ntiles)
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device=dev)
    keys = torch.full((max(capacity, 1),), -1, dtype=torch.int64, device=dev)
    vals = torch.full((max(capacity, 1),), -1, dtype=torch.int32, device=dev)
    ranges = torch.full((ntiles, 2), -1, dtype=torch.int32, device=dev)
    order = torch.full((ntiles,), -1, dtype=torch.int32, device=dev) if with_order else None
    num_keys = torch.full((1,), -1, dtype=torch.int64, device=dev)
    overflow = torch.full((1,), -1, dtype=torch.int32, device=dev)
    L.gs_bin_sort(n, d, r, t, gw, gh, capacity, ws, ws_bytes, keys, vals, ranges, order, num_keys, overflow)
    torch.cuda.synchronize()
    K = int(num_keys.item())
    kk = min(K, capacity)
    return dict(K=K, overflow=int(overflow.item()), keys=keys.cpu().numpy()[:kk].view(np.uint64),
                vals=vals.cpu().numpy()[:kk].view(np.uint32), ranges=ranges.cpu().numpy().view(np.uint32),
                order=order.cpu().numpy().view(np.uint32) if with_order else None)


CASES = [  # n, grid_w, grid_h, seed, share of big splats
    (0, 4, 4, 1, 0.0),
    (1, 1, 1, 2, 0.0),
    (5000, 120, 68, 3, 0.003),
    (300_000, 120, 68, 4, 0.003),     # ~150 depth partitions, ~1500 key partitions
    (20_000, 200, 1, 5, 0.003),       # 8 tile bits: the emitted copies go straight to the last pass
    (20_000, 300, 1, 6, 0.003),       # 9 tile bits: two 5-bit passes
    (3000, 8192, 2100, 7, 0.0),       # 25 tile bits: four 7-bit passes
    (20_000, 4, 4, 11, 0.0),          # lists up to ~6k: longer than a workgroup sorts in LDS
    (60_000, 3, 2, 12, 0.0),          # lists up to ~29k: many chunks per depth pass
    (4_300_000, 160, 90, 14, 0.0),    # over 4096 emission partitions: their sums scanned once
]


@pytest.mark.parametrize("n,gw,gh,seed,big", CASES)
def test_bin_sort_matches_oracle(n, gw, gh, seed, big):
    depth, rect, tiles = scenes.binning_inputs(n, gw, gh, seed, big=big)
    keys, vals, ranges = binning.bin_and_sort_fast(rect, depth, gw, gh)
    K = keys.shape[0]
    print(f"[gpu] bin_sort n={n} grid={gw}x{gh} K={K}", flush=True)
    g = _run(depth, rect, tiles, gw, gh, K + 17)
    assert g["overflow"] == 0 and g["K"] == K
    assert np.array_equal(g["keys"], keys)
    assert np.array_equal(g["vals"], vals)
    assert np.array_equal(g["ranges"], ranges)
    _check_order(g["order"], ranges)


def _check_order(order, ranges):
    """Every tile once, lists non-increasing in length up to the documented
    bucket width (16 log-spaced buckets per doubling, longer than 2^16 merged)."""
    ntiles = ranges.shape[0]
    assert np.array_equal(np.sort(order), np.arange(ntiles, dtype=np.uint32))
    lens = ranges[:, 1].astype(np.float64) - ranges[:, 0]
    lo = np.minimum(np.log2(lens[order] + 1.0) * 16.0, 255.999)
    run_min = np.minimum.accumulate(lo)
    assert np.all(lo[1:] < run_min[:-1] + 1.0 + 1e-4)


def test_bin_sort_capacity_edges():
    gw, gh = 120, 68
    depth, rect, tiles = scenes.binning_inputs(40_000, gw, gh, 8)
    keys, vals, ranges = binning.bin_and_sort_fast(rect, depth, gw, gh)
    K = keys.shape[0]
    g = _run(depth, rect, tiles, gw, gh, K)  # exact fit
    assert g["overflow"] == 0 and g["K"] == K
    assert np.array_equal(g["keys"], keys) and np.array_equal(g["vals"], vals)
    _check_order(g["order"], ranges)
    for cap in (K - 1, 0):
        g = _run(depth, rect, tiles, gw, gh, cap)
        assert g["overflow"] == 1 and g["K"] == K
        assert np.all(g["ranges"] == 0)


def test_bin_sort_all_culled_and_repeatable():
    gw, gh = 64, 40
    depth, rect, tiles = scenes.binning_inputs(10_000, gw, gh, 9, culled=1.0)
    g = _run(depth, rect, tiles, gw, gh, 128)
    assert g["K"] == 0 and g["overflow"] == 0 and np.all(g["ranges"] == 0)
    depth, rect, tiles = scenes.binning_inputs(70_000, gw, gh, 10)
    a = _run(depth, rect, tiles, gw, gh, 1 << 20)
    b = _run(depth, rect, tiles, gw, gh, 1 << 20)
    for k in ("keys", "vals", "ranges"):  # tile_order's order inside a length bucket is unspecified
        assert np.array_equal(a[k], b[k]), k


def test_bin_sort_without_tile_order():
    """tile_order = NULL: the same keys, values and ranges (lists of every
    length, including ones sorted in chunks)."""
    gw, gh = 3, 2
    depth, rect, tiles = scenes.binning_inputs(60_000, gw, gh, 12)
    keys, vals, ranges = binning.bin_and_sort_fast(rect, depth, gw, gh)
    g = _run(depth, rect, tiles, gw, gh, keys.shape[0], with_order=False)
    assert g["overflow"] == 0 and g["K"] == keys.shape[0]
    assert np.array_equal(g["keys"], keys) and np.array_equal(g["vals"], vals)
    assert np.array_equal(g["ranges"], ranges)


@pytest.mark.parametrize("n,gw,gh,seed,big", [(20_000, 4, 4, 11, 0.0), (300_000, 120, 68, 4, 0.003),
                                              (60_000, 3, 2, 12, 0.0), (5000, 120, 68, 3, 0.003),
                                              (20_000, 200, 1, 5, 0.003)])
def test_depth_first_and_per_tile_sorts_agree(n, gw, gh, seed, big):
    """Both routes to the sorted keys, forced by the capacity (a capacity of
    2048 copies per tile or more sorts the splats by depth before emitting
    their copies; a smaller one sorts each tile's list, and from 512 copies
    per tile the tile passes take larger partitions), give the oracle's
    keys, values and ranges."""
    depth, rect, tiles = scenes.binning_inputs(n, gw, gh, seed, big=big)
    keys, vals, ranges = binning.bin_and_sort_fast(rect, depth, gw, gh)
    K = keys.shape[0]
    T = gw * gh
    small, mid, large = K, max(K, 512 * T), max(K, 2048 * T)
    caps = [c for c in (small, mid) if c < 2048 * T] + [large]
    longest = int((ranges[:, 1] - ranges[:, 0]).max())
    print(f"[gpu] bin_sort routes n={n} grid={gw}x{gh} K={K} longest list {longest} capacities {caps}", flush=True)
    outs = []
    for cap in dict.fromkeys(caps):
        g = _run(depth, rect, tiles, gw, gh, cap)
        assert g["overflow"] == 0 and g["K"] == K
        assert np.array_equal(g["keys"], keys) and np.array_equal(g["vals"], vals)
        assert np.array_equal(g["ranges"], ranges)
        _check_order(g["order"], ranges)
        outs.append(g)


def test_hot_tiles_on_the_per_tile_route():
    """A few very long lists beside short ones, at an average below the
    depth-first route's threshold: lists sorted in LDS up to 2048 copies and
    in 2048-copy chunks beyond, with both partition sizes of the tile passes
    (capacities below and above 512 copies per tile), ties included, give
    the oracle's keys, values and ranges."""
    gw, gh, n = 16, 1, 8000
    rng = np.random.default_rng(8)
    tx = rng.integers(0, gw, size=n)
    tx[:5200] = 0                      # a hot tile: 5200+ copies
    tx[5200:6700] = 1                  # 1500+ copies: a workgroup's sort in LDS
    rect = np.stack([tx, np.zeros(n, np.int64), tx, np.zeros(n, np.int64)], 1).astype(np.int32)
    depth = rng.choice(np.linspace(1.0, 50.0, 3000), size=n).astype(np.float32)  # many ties
    tiles = np.ones(n, np.uint32)
    keys, vals, ranges = binning.bin_and_sort_fast(rect, depth, gw, gh)
    K = keys.shape[0]
    for cap in (K, 512 * gw * gh + 7):
        assert cap < 2048 * gw * gh  # the per-tile route
        print(f"[gpu] bin_sort hot tiles K={K} capacity {cap}", flush=True)
        g = _run(depth, rect, tiles, gw, gh, cap)
        assert g["overflow"] == 0 and g["K"] == K
        assert np.array_equal(g["keys"], keys) and np.array_equal(g["vals"], vals)
        assert np.array_equal(g["ranges"], ranges)


def test_splats_with_millions_of_tiles():
    """A splat whose rectangle holds more than 2^22 tiles: the emission's copy
    index within a splat leaves the range where a float quotient by the
    rectangle's width is exact to within one, and takes the integer division."""
    gw, gh = 4096, 1100
    rect = np.array([[0, 0, gw - 1, gh - 1], [17, 3, 3016, 1099], [5, 7, 9, 8], [0, 0, -1, -1],
                     [4095, 1099, 4095, 1099]], np.int32)
    depth = np.array([3.0, 2.0, 3.0, 1.0, 0.5], np.float32)
    w = np.maximum(rect[:, 2] - rect[:, 0] + 1, 0)
    h = np.maximum(rect[:, 3] - rect[:, 1] + 1, 0)
    tiles = (w * h).astype(np.uint32)
    keys, vals, ranges = binning.bin_and_sort_fast(rect, depth, gw, gh)
    K = keys.shape[0]
    assert tiles.max() > (1 << 22)
    print(f"[gpu] bin_sort millions of tiles K={K}", flush=True)
    g = _run(depth, rect, tiles, gw, gh, K)
    assert g["overflow"] == 0 and g["K"] == K
    assert np.array_equal(g["keys"], keys) and np.array_equal(g["vals"], vals)
    assert np.array_equal(g["ranges"], ranges)
