"""Pins of the tile-binning oracle.

* The vectorised emission + stable sort equals the definition written out
  directly: for every tile, every Gaussian whose square covers one of the
  tile's pixels, in (depth, index) order (pure-Python loops, tiny inputs).
* The rect equals brute-force pixel membership |u - mx| <= rx, |v - my| <= ry on inputs where
  the binary32 bounds are exact.
"""
import numpy as np

from oracle import binning


def _direct_lists(mx, my, rx, ry, depth, W, H, B):
    tx_n, ty_n = (W + B - 1) // B, (H + B - 1) // B
    lists = []
    for ty in range(ty_n):
        for tx in range(tx_n):
            members = []
            for i in range(len(mx)):
                if rx[i] <= 0 or ry[i] <= 0:
                    continue
                hit = False
                for v in range(ty * B, min((ty + 1) * B, H)):
                    if abs(v - float(my[i])) > ry[i]:
                        continue
                    for u in range(tx * B, min((tx + 1) * B, W)):
                        if abs(u - float(mx[i])) <= rx[i]:
                            hit = True
                            break
                    if hit:
                        break
                if hit:
                    members.append((float(depth[i]), i))
            lists.append([i for _, i in sorted(members)])
    return lists


def test_binning_matches_direct_definition():
    rng = np.random.default_rng(0)
    W, H, B = 37, 29, 8
    n = 60
    # binary32 bounds are exact: means on a 1/1024 grid, small radii
    mx = (np.round(rng.uniform(-6, W + 6, n) * 1024) / 1024).astype(np.float32)
    my = (np.round(rng.uniform(-6, H + 6, n) * 1024) / 1024).astype(np.float32)
    rx = rng.integers(0, 9, n).astype(np.int32)
    ry = rng.integers(1, 9, n).astype(np.int32)
    depth = rng.uniform(1, 3, n).astype(np.float32)
    depth[5] = depth[9] = depth[13]  # ties resolve by index
    out = binning.bin_and_sort(mx, my, rx, ry, depth, W, H, B)
    ref = _direct_lists(mx, my, rx, ry, depth, W, H, B)
    for t, members in enumerate(ref):
        s, e = out["ranges"][t]
        got = out["values"][s:e].tolist()
        assert got == members, (t, got, members)
        assert all((out["keys"][s:e] >> np.uint64(32)) == t)
    assert out["tiles_touched"].sum() == len(out["values"])
    assert sum(len(m) for m in ref) == len(out["values"])


def test_rect_matches_pixel_membership():
    rng = np.random.default_rng(1)
    W, H, B = 64, 48, 16
    n = 200
    mx = (np.round(rng.uniform(-20, W + 20, n) * 256) / 256).astype(np.float32)
    my = (np.round(rng.uniform(-20, H + 20, n) * 256) / 256).astype(np.float32)
    rx = rng.integers(0, 30, n).astype(np.int32)
    ry = rng.integers(0, 30, n).astype(np.int32)
    tx0, ty0, tx1, ty1, count = binning.tile_rects(mx, my, rx, ry, W, H, B)
    for i in range(n):
        us = [u for u in range(W) if abs(u - float(mx[i])) <= rx[i]]
        vs = [v for v in range(H) if abs(v - float(my[i])) <= ry[i]]
        if rx[i] <= 0 or ry[i] <= 0 or not us or not vs:
            assert count[i] == 0
            continue
        assert (tx0[i], tx1[i], ty0[i], ty1[i]) == (us[0] // B, us[-1] // B, vs[0] // B, vs[-1] // B)
        assert count[i] == (tx1[i] - tx0[i] + 1) * (ty1[i] - ty0[i] + 1)


def test_empty_input():
    out = binning.bin_and_sort(np.zeros(0, np.float32), np.zeros(0, np.float32), np.zeros(0, np.int32),
                               np.zeros(0, np.int32), np.zeros(0, np.float32), 16, 16, 16)
    assert len(out["values"]) == 0 and (out["ranges"] == 0).all()
