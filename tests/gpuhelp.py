"""Helpers of the GPU parity tests: upload reference-projected records to the
device in the library's layouts and read results back."""
from __future__ import annotations

import numpy as np
import pytest
import torch


def device():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def gsmi():
    from paper_2605_13794_amd import gsmi as G
    G.lib()  # raises if the library is missing: no fallback
    return G


def f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def tiles_touched(pr, width, height):
    """Tile counts of the integer rectangle rule (numpy, vectorised)."""
    TX = -(-width // 16)
    TY = -(-height // 16)
    r = pr.radius.astype(np.int64)
    xi = np.floor(pr.mean2d[0]).astype(np.int64)
    yi = np.floor(pr.mean2d[1]).astype(np.int64)
    x0 = np.clip((xi - r) // 16, 0, TX)
    x1 = np.clip((xi + r) // 16 + 1, 0, TX)
    y0 = np.clip((yi - r) // 16, 0, TY)
    y1 = np.clip((yi + r) // 16 + 1, 0, TY)
    return np.where(r > 0, (x1 - x0) * (y1 - y0), 0)


def upload_projection(pr, width, height, dev, centre=True):
    """Packed render records (12 floats per Gaussian) built from a reference
    projection rounded to float32, with depth, radius and tile counts, and,
    with centre, the component-major screen centres (the binning then reads
    those instead of the records)."""
    from paper_2605_13794_amd.raster import ProjBuffers
    n = pr.n
    rec = np.zeros((n, 12), dtype=np.float32)
    rec[:, 0:2] = f32(pr.mean2d).T
    rec[:, 2] = f32(pr.conic[0])
    rec[:, 3] = f32(pr.conic[1])
    rec[:, 4] = f32(pr.conic[2])
    rec[:, 5] = f32(pr.opacity)
    rec[:, 6:9] = f32(pr.rgb).T
    rec[:, 9] = pr.depth
    pb = ProjBuffers(n, dev, centre=centre)
    pb.rec.copy_(torch.from_numpy(rec.reshape(-1)))
    if centre:
        pb.mean2d.copy_(torch.from_numpy(np.ascontiguousarray(f32(pr.mean2d))))
    pb.depth.copy_(torch.from_numpy(f32(pr.depth)))
    pb.radius.copy_(torch.from_numpy(pr.radius.astype(np.int32)))
    pb.tiles.copy_(torch.from_numpy(tiles_touched(pr, width, height).astype(np.int32)))
    pb.clamp.zero_()
    return pb


def to_np(t):
    return t.detach().cpu().numpy()


def u32(t):
    return to_np(t).view(np.uint32)


def tie_pixel_mask(pr, keys, vals, depth64, width, height, rel=4e-7):
    """[H][W] mask, False at pixels whose colour depends on the order of two
    Gaussians whose float64 depths lie within `rel` of each other (a float32
    depth computed by another rounding may order them either way).  A swap
    of two consecutive list entries changes a pixel only where both are
    composited, i.e. both have alpha >= 1/255 there."""
    m = np.ones((height, width), dtype=bool)
    keys = np.asarray(keys, dtype=np.uint64)
    if keys.size < 2:
        return m
    tiles = (keys >> np.uint64(32)).astype(np.int64)
    vals = np.asarray(vals, dtype=np.int64)
    z = np.asarray(depth64, dtype=np.float64)[vals]
    same = tiles[1:] == tiles[:-1]
    close = np.abs(z[1:] - z[:-1]) <= rel * np.maximum(np.abs(z[1:]), np.abs(z[:-1]))
    TX = -(-width // 16)
    for k in np.nonzero(same & close)[0]:
        t = int(tiles[k + 1])
        ty, tx = divmod(t, TX)
        ys = np.arange(ty * 16, min(height, ty * 16 + 16))
        xs = np.arange(tx * 16, min(width, tx * 16 + 16))
        X, Y = np.meshgrid(xs + 0.5, ys + 0.5)
        both = np.ones_like(X, dtype=bool)
        for j in (vals[k], vals[k + 1]):
            dx = pr.mean2d[0, j] - X
            dy = pr.mean2d[1, j] - Y
            a, b, c = pr.conic[:, j]
            al = np.minimum(0.99, pr.opacity[j] * np.exp(-0.5 * (a * dx * dx + c * dy * dy) - b * dx * dy))
            both &= al >= (1.0 / 255.0) * (1.0 - 1e-3)
        m[np.ix_(ys, xs)] &= ~both
    return m


def ambiguous_tiles(keys, vals, depth64, width, rel=1e-6):
    """Tiles whose depth order could differ between two float32 roundings of
    the same depths: two consecutive entries of the tile's sorted list whose
    float64 depths lie within `rel` of each other."""
    keys = np.asarray(keys, dtype=np.uint64)
    if keys.size < 2:
        return set()
    tiles = (keys >> np.uint64(32)).astype(np.int64)
    z = np.asarray(depth64, dtype=np.float64)[np.asarray(vals, dtype=np.int64)]
    same = tiles[1:] == tiles[:-1]
    close = np.abs(z[1:] - z[:-1]) <= rel * np.maximum(np.abs(z[1:]), np.abs(z[:-1]))
    return set(tiles[1:][same & close].tolist())


def tile_mask(tiles, width, height):
    """Boolean [H][W] mask, True outside the given tiles."""
    m = np.ones((height, width), dtype=bool)
    TX = -(-width // 16)
    for t in tiles:
        ty, tx = divmod(int(t), TX)
        m[ty * 16:(ty + 1) * 16, tx * 16:(tx + 1) * 16] = False
    return m


def assert_same_ranges(got, ref):
    """Tile ranges agree: every tile has the same list length, and non-empty
    tiles the same start (an empty tile's start is not unique)."""
    got = np.asarray(got).reshape(2, -1).astype(np.int64)
    ref = np.asarray(ref).reshape(2, -1).astype(np.int64)
    np.testing.assert_array_equal(got[1] - got[0], ref[1] - ref[0])
    ne = ref[1] > ref[0]
    np.testing.assert_array_equal(got[0][ne], ref[0][ne])


def comparable_pixels(ref, rad_gpu, width, height, margin=1e-3):
    """[H][W] mask of the pixels where an end-to-end comparison (float32
    projection against the float64 one) is meaningful: every threshold test
    of the pixel clears its threshold by `margin` (relative), no Gaussian of
    the pixel's tile has a different integer radius on the two sides, and the
    pixel's colour does not depend on the order of two near-equal depths.
    `ref` is the reference's forward_backward result for the same entries
    that the device projected; rad_gpu the device radii of those entries."""
    pr = ref["projected"]
    bad = set(np.nonzero(np.asarray(rad_gpu)[:pr.n] != pr.radius)[0].tolist())
    tiles = set()
    if bad:
        for key, val in zip(ref["keys"].tolist(), ref["vals"].tolist()):
            if val in bad:
                tiles.add(key >> 32)
    ties = tie_pixel_mask(pr, ref["keys"], ref["vals"], ref["out"]["depth"].detach().numpy(), width, height)
    return (ref["margin"] >= margin) & tile_mask(tiles, width, height) & ties, len(bad)


def rel_inf(g, ref):
    """max|g - ref| / max|ref| (per tensor)."""
    return float(np.abs(g - ref).max() / max(np.abs(ref).max(), 1e-30))
