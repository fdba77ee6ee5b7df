"""gs_bin_sort_noalloc (the binning with its workspace in the library's static
device array, for callers that cannot allocate) through the C ABI: its
outputs equal gs_bin_sort's, bit for bit, on consecutive calls that share the
array, a large input then smaller ones (the array keeps the previous call's
contents), on both sorting routes and on an overflowing capacity; and the
oracle's binning for the same inputs."""
import numpy as np
import pytest
import torch

from oracle import binning
from paper_2603_18707_amd import _lib as L
from paper_2603_18707_amd import scenes
from tests.test_gpu_binsort import _check_order

pytestmark = pytest.mark.gpu


def _outputs(n, gw, gh, capacity, dev):
    ntiles = gw * gh
    return dict(keys=torch.full((max(capacity, 1),), -1, dtype=torch.int64, device=dev),
                vals=torch.full((max(capacity, 1),), -1, dtype=torch.int32, device=dev),
                ranges=torch.full((ntiles, 2), -1, dtype=torch.int32, device=dev),
                order=torch.full((ntiles,), -1, dtype=torch.int32, device=dev),
                num_keys=torch.full((1,), -1, dtype=torch.int64, device=dev),
                overflow=torch.full((1,), -1, dtype=torch.int32, device=dev))


def _host(o, capacity):
    K = int(o["num_keys"].item())
    kk = min(K, capacity)
    return dict(K=K, overflow=int(o["overflow"].item()), keys=o["keys"].cpu().numpy()[:kk].view(np.uint64),
                vals=o["vals"].cpu().numpy()[:kk].view(np.uint32), ranges=o["ranges"].cpu().numpy().view(np.uint32),
                order=o["order"].cpu().numpy().view(np.uint32))


# n, grid, seed, big-splat share, capacity offset from K: in call order, the
# largest first, then smaller inputs on both routes (lists of ~6k copies take
# the depth-first route), an overflowing capacity, and an empty frame
SEQUENCE = [(300_000, 120, 68, 4, 0.003, 17), (5000, 120, 68, 3, 0.003, 0), (20_000, 4, 4, 11, 0.0, 5),
            (5000, 120, 68, 8, 0.003, -1), (0, 4, 4, 1, 0.0, 3)]


def test_noalloc_bin_sort_matches_the_workspace_entry_point():
    dev = torch.device("cuda", 0)
    for n, gw, gh, seed, big, extra in SEQUENCE:
        depth, rect, tiles = scenes.binning_inputs(n, gw, gh, seed, big=big)
        keys, vals, ranges = binning.bin_and_sort_fast(rect, depth, gw, gh)
        K = keys.shape[0]
        cap = max(K + extra, 0)
        print(f"[gpu] bin_sort_noalloc n={n} grid={gw}x{gh} K={K} capacity={cap}", flush=True)
        d = torch.from_numpy(depth).to(dev)
        r = torch.from_numpy(rect).to(dev)
        t = torch.from_numpy(tiles.view(np.int32)).to(dev)
        ws_bytes = L.gs_bin_sort_workspace(n, cap, gw * gh)
        assert ws_bytes <= L.GS_NOALLOC_SCRATCH_BYTES
        ws = torch.empty(ws_bytes, dtype=torch.uint8, device=dev)
        a, b = _outputs(n, gw, gh, cap, dev), _outputs(n, gw, gh, cap, dev)
        L.gs_bin_sort(n, d, r, t, gw, gh, cap, ws, ws_bytes, a["keys"], a["vals"], a["ranges"], a["order"],
                      a["num_keys"], a["overflow"])
        L.gs_bin_sort_noalloc(n, d, r, t, gw, gh, cap, b["keys"], b["vals"], b["ranges"], b["order"],
                              b["num_keys"], b["overflow"])
        torch.cuda.synchronize()
        ha, hb = _host(a, cap), _host(b, cap)
        assert ha["K"] == hb["K"] == K and ha["overflow"] == hb["overflow"] == int(K > cap)
        # on overflow only the count, the flag and the (empty) ranges are defined
        for f in ("keys", "vals", "ranges") if K <= cap else ("ranges",):
            assert np.array_equal(ha[f], hb[f]), (n, f, int((ha[f] != hb[f]).sum()))
        if K > cap:
            assert not hb["ranges"].any()
        else:
            assert np.array_equal(hb["keys"], keys) and np.array_equal(hb["vals"], vals)
            assert np.array_equal(hb["ranges"], ranges)
            # the tile order is one of several valid ones (tiles within a
            # length bucket in any order): checked for validity
            _check_order(ha["order"], ranges)
            _check_order(hb["order"], ranges)


def test_noalloc_rejects_what_exceeds_its_scratch():
    with pytest.raises(L.GsError) as e:
        L.gs_bin_sort_noalloc(1_000_000, None, None, None, 120, 68, 20_000_000, None, None, None, None, None, None)
    assert e.value.status == L.GS_ECAPACITY
