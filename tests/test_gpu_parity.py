"""GPU parity of the HIP path against the float64 reference, through the C ABI.

Tolerances (float32 device arithmetic against a float64 reference):
  keys, sorted values, tile ranges, pair counts: bit-exact when both sides are
      fed the same float32 projected record;
  images: max-abs 1e-4 on pixels whose threshold decisions are not within a
      1e-5 relative margin (the reference reports that margin per pixel);
  screen-space and parameter gradients: per tensor
      max|g - g_ref| <= 1e-3 max|g_ref|.
"""
from __future__ import annotations

import math

import numpy as np
import pytest
import torch

from paper_2605_13794_amd import scenes as S
from tests.gpuhelp import (assert_same_ranges, device, gsmi, tie_pixel_mask, tile_mask, to_np, u32,
                           upload_projection)

pytestmark = pytest.mark.gpu


def make_case(name):
    if name == "cfg1":  # the small configuration: 4,096 Gaussians, 128x128
        return S.cube_scene(4096, seed=0), S.cube_camera(128, 128, 128.0)
    if name == "ragged":  # partial edge tiles on both axes
        return S.cube_scene(2000, seed=3, log_scale_mu=-2.6), S.cube_camera(100, 75, 90.0)
    if name == "city":  # aerial city subset: many tiles, several sort partitions
        sc = S.city_scene(1 << 20, seed=2)
        idx = np.nonzero((np.abs(sc.mean[0]) < 120) & (sc.mean[1] > -60) & (sc.mean[1] < 200))[0][:60000]
        return sc.subset(idx), S.aerial_camera(480, 270)
    raise KeyError(name)


CASES = ["cfg1", "ragged", "city"]


def _frame(cams, n, dev, **kw):
    from paper_2605_13794_amd.raster import Frame
    return Frame(cams, n, dev, **kw)


def _ref_sorted(oracle, sc, cam):
    _, out, pr = oracle.project(sc.arrays(), cam)
    prf = pr.rounded_f32()
    K, keys, vals, ranges = oracle.bin_sort(prf, cam.width, cam.height)
    return out, pr, prf, K, keys, vals, ranges


def _gpu_lists(prf, cam, vals, ranges, dev):
    pb = upload_projection(prf, cam.width, cam.height, dev)
    v = torch.from_numpy(np.asarray(vals, dtype=np.uint32).view(np.int32).copy()).to(dev)
    if v.numel() == 0:
        v = torch.zeros(1, dtype=torch.int32, device=dev)
    r = torch.from_numpy(np.asarray(ranges, dtype=np.uint32).reshape(-1).view(np.int32).copy()).to(dev)
    return pb, v, r


# ---------------------------------------------------------------------------
# Projection
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("case", CASES)
def test_project_matches_reference(oracle, case):
    dev = device()
    gsmi()
    from paper_2605_13794_amd.raster import DeviceScene
    sc, cam = make_case(case)
    ds = DeviceScene(sc, dev)
    fr = _frame([cam], sc.n, dev, soa=True)
    fr.project(ds.struct())
    torch.cuda.synchronize()
    _, out, pr = oracle.project(sc.arrays(), cam)
    p = fr.proj[0]
    rad_g, rad_o = to_np(p.radius), pr.radius
    lam = out["lam"].numpy()
    e = 3.0 * np.sqrt(np.maximum(lam, 0))
    amb = (np.abs(e - np.round(e)) < 1e-4 * np.maximum(e, 1)) | \
          (np.abs(out["mean2d"].detach().numpy().T - np.round(out["mean2d"].detach().numpy().T)) < 1e-3).any(0) | \
          (np.abs(out["depth"].detach().numpy() - cam.znear) < 1e-5)
    assert amb.mean() < 0.01
    ok = ~amb
    np.testing.assert_array_equal(rad_g[ok], rad_o[ok])
    tt_o = out["tiles_touched"].numpy()
    np.testing.assert_array_equal(to_np(p.tiles)[ok], tt_o[ok])
    vis = ok & (rad_o > 0)
    assert vis.sum() > 0.2 * sc.n or case == "city"
    scale = max(cam.width, cam.height)
    np.testing.assert_allclose(to_np(p.mean2d)[:, vis], pr.mean2d[:, vis], rtol=0, atol=2e-7 * scale * 4)
    np.testing.assert_allclose(to_np(p.depth)[vis], pr.depth[vis], rtol=1e-6)
    # conic relative to its own magnitude sqrt(a c)
    cg, co = to_np(p.conic)[:, vis], pr.conic[:, vis]
    mag = np.sqrt(co[0] * co[2])
    assert (np.abs(cg - co) / mag).max() < 1e-4
    np.testing.assert_allclose(to_np(p.opacity)[vis], pr.opacity[vis], rtol=1e-6, atol=1e-7)
    np.testing.assert_allclose(to_np(p.rgb)[:, vis], pr.rgb[:, vis], atol=2e-6)
    # clamp bits where the raw colour is not within 1e-5 of 0
    cb_o = out["clamp_bits"].numpy()
    bits_o = (cb_o * np.array([1, 2, 4])).sum(1)
    raw_far = (np.abs(pr.rgb) > 1e-5).all(0) | (cb_o.any(1) == False)  # noqa: E712
    sel = vis & raw_far
    np.testing.assert_array_equal(to_np(p.clamp)[sel], bits_o[sel])
    # render records agree with the component-major copies
    rec = to_np(p.rec).reshape(-1, 12)
    np.testing.assert_array_equal(rec[vis, 0], to_np(p.mean2d)[0, vis])
    np.testing.assert_array_equal(rec[vis, 8], to_np(p.rgb)[2, vis])


# ---------------------------------------------------------------------------
# Binning and sort: bit-exact on identical projected inputs
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("case", CASES)
def test_bin_sort_bitexact(oracle, case):
    dev = device()
    G = gsmi()
    sc, cam = make_case(case)
    _, pr, prf, K, keys, vals, ranges = _ref_sorted(oracle, sc, cam)
    fr = _frame([cam], sc.n, dev, capacity=K + 777)
    # rectangles from the records, then from the component-major centres
    for centre in (False, True):
        fr.proj[0] = upload_projection(prf, cam.width, cam.height, dev, centre=centre)
        Kg = fr.bin_sort()
        torch.cuda.synchronize()
        assert Kg == K
        np.testing.assert_array_equal(to_np(fr.keys[:K]).view(np.uint64), keys)
        np.testing.assert_array_equal(u32(fr.vals[:K]), vals)
        assert_same_ranges(u32(fr.ranges), ranges)
    # deterministic: a second run gives the same bits
    k1, v1 = fr.keys[:K].clone(), fr.vals[:K].clone()
    fr.bin_sort()
    torch.cuda.synchronize()
    assert torch.equal(k1, fr.keys[:K]) and torch.equal(v1, fr.vals[:K])


def test_bin_sort_large_many_passes(oracle):
    """>100k pairs over 8,160 tiles (1080p): 6 radix passes, many partitions."""
    dev = device()
    sc = S.city_scene(1 << 20, seed=2)
    idx = np.nonzero((np.abs(sc.mean[0]) < 250) & (sc.mean[1] > -80) & (sc.mean[1] < 300))[0][:200000]
    sc = sc.subset(idx)
    cam = S.aerial_camera(1920, 1080)
    _, pr, prf, K, keys, vals, ranges = _ref_sorted(oracle, sc, cam)
    assert K > 100000
    fr = _frame([cam], sc.n, dev, capacity=K)
    fr.proj[0] = upload_projection(prf, cam.width, cam.height, dev)
    assert fr.bin_sort() == K
    torch.cuda.synchronize()
    np.testing.assert_array_equal(to_np(fr.keys[:K]).view(np.uint64), keys)
    np.testing.assert_array_equal(u32(fr.vals[:K]), vals)
    assert_same_ranges(u32(fr.ranges), ranges)


def test_bin_sort_large_persistent_grid(oracle):
    """2.5M Gaussians, one orbit view: over 3M pairs, long tile lists (the
    full-key radix path) and more 3,840-key partitions than workgroups, so
    each workgroup claims partitions in a loop."""
    dev = device()
    sc = S.city_scene(2500000, seed=5)
    cam = S.orbit_cameras(64, 500.0, 300.0, 1920, 1080)[0]
    _, pr, prf, K, keys, vals, ranges = _ref_sorted(oracle, sc, cam)
    assert K > 768 * 3840
    fr = _frame([cam], sc.n, dev, capacity=K)
    fr.proj[0] = upload_projection(prf, cam.width, cam.height, dev)
    assert fr.bin_sort() == K
    torch.cuda.synchronize()
    np.testing.assert_array_equal(to_np(fr.keys[:K]).view(np.uint64), keys)
    np.testing.assert_array_equal(u32(fr.vals[:K]), vals)
    assert_same_ranges(u32(fr.ranges), ranges)


def test_bin_sort_partition_loop(oracle):
    """More than 2,048 partitions of 3,840 keys in a pass (7.9M pairs), so
    every workgroup of the counts and the scatter loops over partitions: a
    synthetic projection of 2.5M entries over a 1080p view (centres uniform
    over the image and a margin, radii 2-14 px, 10 % culled, depths from 400
    values so that equal keys occur), ~9M pairs on the depth-first path,
    bit-exact against the reference's sort of the same records."""
    dev = device()
    rng = np.random.default_rng(77)
    n, W, H = 2_500_000, 1920, 1080
    mean2d = np.stack([rng.uniform(-40.0, W + 40.0, n), rng.uniform(-40.0, H + 40.0, n)])
    mean2d = mean2d.astype(np.float32).astype(np.float64)
    radius = rng.integers(2, 15, n).astype(np.int32)
    radius[rng.random(n) < 0.1] = 0
    depth = (rng.integers(0, 400, n) * 0.75 + 10.0).astype(np.float32)
    conic = np.tile(np.array([[1.0], [0.0], [1.0]]), (1, n))
    prf = oracle.Projected(mean2d, depth, conic, np.full(n, 0.5), np.full((3, n), 0.5), radius)
    K, keys, vals, ranges = oracle.bin_sort(prf, W, H)
    print(f"[partition loop] K={K}", flush=True)
    assert K > 2048 * 3840
    cam = S.aerial_camera(W, H)
    fr = _frame([cam], n, dev, capacity=K)
    fr.proj[0] = upload_projection(prf, W, H, dev)
    assert fr.bin_sort() == K
    torch.cuda.synchronize()
    np.testing.assert_array_equal(to_np(fr.keys[:K]).view(np.uint64), keys)
    np.testing.assert_array_equal(u32(fr.vals[:K]), vals)
    assert_same_ranges(u32(fr.ranges), ranges)


@pytest.mark.parametrize("path", ["per_tile", "depth_first"])
def test_bin_sort_equal_depths(oracle, path):
    """Every Gaussian at one depth: the order inside a tile is the index
    order.  On the depth-first path (forced by the capacity) each of the four
    depth passes sees a single digit, so each is a copy, the last one
    gathering the records and their pair counts."""
    dev = device()
    sc = S.city_scene(1 << 20, seed=2)
    idx = np.nonzero((np.abs(sc.mean[0]) < 200) & (sc.mean[1] > -60) & (sc.mean[1] < 200))[0][:60000]
    sc = sc.subset(idx)
    cam = S.aerial_camera(1920, 1080)
    _, _, pr = oracle.project(sc.arrays(), cam)
    prf = pr.rounded_f32()
    prf = type(prf)(prf.mean2d, np.full_like(prf.depth, 211.25), prf.conic, prf.opacity, prf.rgb, prf.radius)
    K, keys, vals, ranges = oracle.bin_sort(prf, cam.width, cam.height)
    assert K > 20000
    cap = K if path == "per_tile" else 256 * gsmi().gs_num_tiles(cam.width, cam.height) + 1
    fr = _frame([cam], sc.n, dev, capacity=cap)
    fr.proj[0] = upload_projection(prf, cam.width, cam.height, dev)
    assert fr.bin_sort() == K
    torch.cuda.synchronize()
    np.testing.assert_array_equal(to_np(fr.keys[:K]).view(np.uint64), keys)
    np.testing.assert_array_equal(u32(fr.vals[:K]), vals)
    assert_same_ranges(u32(fr.ranges), ranges)


def test_bin_sort_single_tile_long_segment(oracle):
    """A 16x16 image is one tile holding every pair: the full-key radix path
    with no tile bits."""
    dev = device()
    sc = S.cube_scene(6000, seed=11)
    cam = S.cube_camera(16, 16, f=16.0)
    _, pr, prf, K, keys, vals, ranges = _ref_sorted(oracle, sc, cam)
    assert K > 2048
    fr = _frame([cam], sc.n, dev, capacity=K)
    fr.proj[0] = upload_projection(prf, cam.width, cam.height, dev)
    assert fr.bin_sort() == K
    torch.cuda.synchronize()
    np.testing.assert_array_equal(to_np(fr.keys[:K]).view(np.uint64), keys)
    np.testing.assert_array_equal(u32(fr.vals[:K]), vals)
    assert_same_ranges(u32(fr.ranges), ranges)


def test_bin_sort_segment_paths(oracle):
    """6,000 Gaussians seen small in a 256x256 image: ~57 pairs per tile on
    average (so the per-tile path), with tiles of up to 512 pairs (register
    network), 512-2,048 (LDS network) and over 2,048 (global radix) in one
    sort."""
    dev = device()
    sc = S.cube_scene(6000, seed=12)
    cam = S.cube_camera(256, 256, f=64.0)
    _, pr, prf, K, keys, vals, ranges = _ref_sorted(oracle, sc, cam)
    lens = ranges[1].astype(np.int64) - ranges[0].astype(np.int64)
    assert lens.max() > 2048 and ((lens > 512) & (lens <= 2048)).any() and (lens <= 512).any()
    fr = _frame([cam], sc.n, dev, capacity=K)
    fr.proj[0] = upload_projection(prf, cam.width, cam.height, dev)
    assert fr.bin_sort() == K
    torch.cuda.synchronize()
    np.testing.assert_array_equal(to_np(fr.keys[:K]).view(np.uint64), keys)
    np.testing.assert_array_equal(u32(fr.vals[:K]), vals)
    assert_same_ranges(u32(fr.ranges), ranges)


@pytest.mark.parametrize("path", ["depth_first", "per_tile"])
@pytest.mark.parametrize("layout", ["one_tile_pass", "wide_tile_ids"])
def test_bin_sort_layouts(oracle, layout, path):
    """Both binning paths (depth-first forced by a pair capacity above 256
    per tile, per-tile by the smallest capacity) in the two layouts of their
    tile passes: a 256-tile image (one tile pass over 16-bit tile ids that
    writes the full pairs), and three 4K views in one batch, whose 97,200
    global tile ids need 17 bits (three passes over the full 64-bit keys).
    Bit-exact against the reference, camera by camera, with each camera's
    list after the previous ones."""
    dev = device()
    G = gsmi()
    if layout == "one_tile_pass":
        sc = S.cube_scene(6000, seed=12)
        cams = [S.cube_camera(256, 256, f=64.0)]
    else:
        sc = S.city_scene(1 << 20, seed=2)
        idx = np.nonzero((np.abs(sc.mean[0]) < 150) & (sc.mean[1] > -60) & (sc.mean[1] < 220))[0][:40000]
        sc = sc.subset(idx)
        cams = [S.aerial_camera(3840, 2160, h) for h in (0.0, 120.0, 240.0)]
    refs = [_ref_sorted(oracle, sc, cam) for cam in cams]
    tiles = [G.gs_num_tiles(c.width, c.height) for c in cams]
    assert (sum(tiles) > 65536) == (layout == "wide_tile_ids")
    K = sum(r[3] for r in refs)
    print(f"[{path} {layout}] tiles={sum(tiles)} K={K}", flush=True)
    fr = _frame(cams, sc.n, dev, capacity=256 * sum(tiles) + 1 if path == "depth_first" else K)
    for c, (cam, r) in enumerate(zip(cams, refs)):
        # the one-pass case takes the rectangles' centres from the records
        fr.proj[c] = upload_projection(r[2], cam.width, cam.height, dev, centre=layout != "one_tile_pass")
    assert fr.bin_sort() == K
    torch.cuda.synchronize()
    toff = np.concatenate([[0], np.cumsum(tiles)[:-1]]).astype(np.uint64)
    koff = np.concatenate([[0], np.cumsum([r[3] for r in refs])[:-1]]).astype(np.int64)
    keys = np.concatenate([r[4].astype(np.uint64) + (t << np.uint64(32)) for r, t in zip(refs, toff)])
    vals = np.concatenate([r[5] for r in refs])
    ranges = np.concatenate([np.asarray(r[6]).reshape(2, -1).astype(np.int64) + o for r, o in zip(refs, koff)],
                            axis=1)
    np.testing.assert_array_equal(to_np(fr.keys[:K]).view(np.uint64), keys)
    np.testing.assert_array_equal(u32(fr.vals[:K]), vals)
    assert_same_ranges(u32(fr.ranges), ranges)


def test_bin_sort_empty_and_overflow(oracle):
    dev = device()
    G = gsmi()
    sc, cam = make_case("cfg1")
    _, pr, prf, K, keys, vals, ranges = _ref_sorted(oracle, sc, cam)
    # capacity below K: the count is reported, nothing is sorted, ranges empty
    fr = _frame([cam], sc.n, dev, capacity=K // 3)
    fr.proj[0] = upload_projection(prf, cam.width, cam.height, dev)
    assert fr.bin_sort(check=False) is None
    torch.cuda.synchronize()
    assert int(fr.n_pairs.item()) == K
    rg = u32(fr.ranges).reshape(2, -1)
    assert (rg[0] == rg[1]).all()
    # the depth-first path (a capacity above 256 pairs per tile) overflows the
    # same way, and a later call that fits sorts in full
    tiles = ((cam.width + 15) // 16) * ((cam.height + 15) // 16)
    cap = 256 * tiles + 100
    assert cap < K
    fr3 = _frame([cam], sc.n, dev, capacity=cap)
    fr3.proj[0] = upload_projection(prf, cam.width, cam.height, dev)
    assert fr3.bin_sort(check=False) is None
    torch.cuda.synchronize()
    assert int(fr3.n_pairs.item()) == K
    rg = u32(fr3.ranges).reshape(2, -1)
    assert (rg[0] == rg[1]).all()
    fr4 = _frame([cam], sc.n, dev, capacity=K + 1)
    fr4.proj[0] = upload_projection(prf, cam.width, cam.height, dev)
    assert fr4.bin_sort() == K
    np.testing.assert_array_equal(to_np(fr4.keys[:K]).view(np.uint64), keys)
    np.testing.assert_array_equal(u32(fr4.vals[:K]), vals)
    assert_same_ranges(u32(fr4.ranges), ranges)
    # nothing visible: K = 0
    behind = S.cube_scene(300, seed=5)
    behind.mean[2] -= 10.0
    _, _, prb = oracle.project(behind.arrays(), cam)
    assert (prb.radius == 0).all()
    fr2 = _frame([cam], behind.n, dev, capacity=100)
    fr2.proj[0] = upload_projection(prb.rounded_f32(), cam.width, cam.height, dev)
    assert fr2.bin_sort() == 0
    rg = u32(fr2.ranges).reshape(2, -1)
    assert (rg[0] == rg[1]).all()


# ---------------------------------------------------------------------------
# Compositing, forward and backward, on identical projected inputs
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("case", CASES)
def test_render_fwd_matches_reference(oracle, case):
    dev = device()
    G = gsmi()
    sc, cam = make_case(case)
    _, pr, prf, K, keys, vals, ranges = _ref_sorted(oracle, sc, cam)
    bg = (0.1, 0.2, 0.3)
    ref = oracle.render_fwd(prf, vals, ranges, cam.width, cam.height, bg)
    pb, v, r = _gpu_lists(prf, cam, vals, ranges, dev)
    H, W = cam.height, cam.width
    img = torch.empty(3, H, W, device=dev)
    T = torch.empty(H, W, device=dev)
    last = torch.empty(H, W, dtype=torch.int32, device=dev)
    G.gs_render_fwd([pb.struct()], G.camera_array([cam]), v, r, bg, [img], [T], [last])
    torch.cuda.synchronize()
    ok = ref["margin"] >= 1e-5
    assert (~ok).mean() < 2e-3
    assert np.abs(to_np(img) - ref["rgb"])[:, ok].max() <= 1e-4
    assert np.abs(to_np(T) - ref["T"])[ok].max() <= 1e-4
    np.testing.assert_array_equal(u32(last)[ok], ref["last"][ok])
    # bit-deterministic
    img2 = torch.empty_like(img)
    G.gs_render_fwd([pb.struct()], G.camera_array([cam]), v, r, bg, [img2], [T], [last])
    torch.cuda.synchronize()
    assert torch.equal(img, img2)


def _rel_inf(g, ref):
    return np.abs(g - ref).max() / max(np.abs(ref).max(), 1e-30)


@pytest.mark.parametrize("case", CASES)
def test_render_bwd_matches_reference(oracle, case):
    dev = device()
    G = gsmi()
    from paper_2605_13794_amd.raster import DeviceScene
    sc, cam = make_case(case)
    _, pr, prf, K, keys, vals, ranges = _ref_sorted(oracle, sc, cam)
    bg = (0.0, 0.0, 0.0)
    H, W = cam.height, cam.width
    ref = oracle.render_fwd(prf, vals, ranges, W, H, bg)
    target = S.target_image(W, H, seed=1)
    _, g = oracle.l1_loss(ref["rgb"], target)
    g[:, ref["margin"] < 1e-5] = 0.0
    d2 = oracle.render_bwd(prf, vals, ranges, W, H, g, bg)
    pb, v, r = _gpu_lists(prf, cam, vals, ranges, dev)
    img = torch.empty(3, H, W, device=dev)
    T = torch.empty(H, W, device=dev)
    last = torch.empty(H, W, dtype=torch.int32, device=dev)
    cams = G.camera_array([cam])
    G.gs_render_fwd([pb.struct()], cams, v, r, bg, [img], [T], [last])
    ds = DeviceScene(sc, dev)
    grads = [torch.zeros_like(p) for p in ds.params()]
    g2 = torch.empty(9, sc.n, device=dev)
    gt = torch.from_numpy(g.astype(np.float32)).to(dev)
    ws = torch.empty(G.gs_workspace_size(G.GS_OP_RENDER_BWD, sc.n, 0, 0, 1), dtype=torch.uint8, device=dev)
    G.gs_render_bwd(ds.struct(), None, sc.n, None, [pb.struct()], cams, v, r, bg, [T], [last], [gt],
                    G.grads(*grads), g2, ws)
    torch.cuda.synchronize()
    got = to_np(g2)
    # the stored-chain backward gives the same partials
    chain = torch.empty(max(K, 1) * 256, device=dev)
    G.gs_render_fwd([pb.struct()], cams, v, r, bg, [img], [T], [last], chain=chain)
    g3 = torch.empty(9, sc.n, device=dev)
    G.gs_render_bwd(ds.struct(), None, sc.n, None, [pb.struct()], cams, v, r, bg, [T], [last], [gt],
                    G.grads(*grads), g3, ws, chain=chain)
    # the forward's per-pair flags (composited by some pixel of the tile) let
    # the backward skip the other pairs without changing the partials
    live = torch.full((max(K, 1),), 7, dtype=torch.uint8, device=dev)
    G.gs_render_fwd([pb.struct()], cams, v, r, bg, [img], [T], [last], live=live)
    g4 = torch.empty(9, sc.n, device=dev)
    G.gs_render_bwd(ds.struct(), None, sc.n, None, [pb.struct()], cams, v, r, bg, [T], [last], [gt],
                    G.grads(*grads), g4, ws, live=live)
    torch.cuda.synchronize()
    got = to_np(g2)
    rows = {"mean2d": (0, 2), "conic": (2, 5), "opacity": (5, 6), "rgb": (6, 9)}
    got3 = to_np(g3)
    got4 = to_np(g4)
    for name, (a, b) in rows.items():
        refv = d2[name].reshape(b - a, -1)
        assert _rel_inf(got[a:b], refv) <= 1e-3, (name, _rel_inf(got[a:b], refv))
        assert _rel_inf(got3[a:b], refv) <= 1e-3, ("stored chain", name, _rel_inf(got3[a:b], refv))
        assert _rel_inf(got4[a:b], refv) <= 1e-3, ("live flags", name, _rel_inf(got4[a:b], refv))
        # same contributions, only the order of the atomic adds may differ
        scale = max(float(np.abs(got[a:b]).max()), 1e-30)
        assert float(np.abs(got4[a:b] - got[a:b]).max()) <= 1e-5 * scale, ("live flags vs all pairs", name)
    # flags are 0 or 1 below each tile's largest `last`, and the pair at every
    # pixel's last composited position is live
    lv = to_np(live).astype(np.int64)
    lastn = ref["last"].astype(np.int64)
    TXn, TYn = (W + 15) // 16, (H + 15) // 16
    rr = np.asarray(ranges, dtype=np.int64).reshape(2, -1)
    py, px = np.nonzero(lastn)
    tile = (py // 16) * TXn + px // 16
    assert np.all(lv[rr[0, tile] + lastn[py, px] - 1] == 1)
    pad = np.zeros((TYn * 16, TXn * 16), dtype=np.int64)
    pad[:H, :W] = lastn
    lmax = pad.reshape(TYn, 16, TXn, 16).max(axis=(1, 3)).reshape(-1)
    below = np.concatenate([lv[rr[0, t]:rr[0, t] + lmax[t]] for t in range(rr.shape[1])] + [np.zeros(0, np.int64)])
    assert np.all((below == 0) | (below == 1))


# ---------------------------------------------------------------------------
# End to end from the parameters
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("case", CASES)
def test_end_to_end_forward_backward(oracle, case):
    """GPU projection + sort + compositing + backward against the float64
    pipeline.  The same upstream gradient (the reference's L1 gradient, zero
    on pixels whose decisions sit within a 1e-3 margin or whose tiles hold a
    Gaussian with an ambiguous radius/rectangle) is fed to both backward
    passes."""
    dev = device()
    G = gsmi()
    from paper_2605_13794_amd.raster import DeviceScene
    sc, cam = make_case(case)
    H, W = cam.height, cam.width
    ds = DeviceScene(sc, dev)
    fr = _frame([cam], sc.n, dev)
    out, K = fr.forward(ds.struct())
    torch.cuda.synchronize()
    ref = oracle.forward_backward(sc.arrays(), cam)
    pr = ref["projected"]
    # Integer decisions taken from floats on both sides: tiles covered by a
    # Gaussian whose radius/rectangle differs, and tiles whose depth order
    # holds a near tie (float64 depths within 1e-6), are excluded.
    rad_g = to_np(fr.proj[0].radius)
    bad = np.nonzero(rad_g != pr.radius)[0]
    tiles = set()
    badset = set(bad.tolist())
    for key, val in zip(ref["keys"].tolist(), ref["vals"].tolist()):
        if val in badset:
            tiles.add(key >> 32)
    ties = tie_pixel_mask(pr, ref["keys"], ref["vals"], ref["out"]["depth"].detach().numpy(), W, H)
    mask = (ref["margin"] >= 1e-3) & tile_mask(tiles, W, H) & ties
    assert bad.size <= 3 and mask.mean() > 0.95, (bad.size, ties.mean(), mask.mean())
    diff = np.abs(to_np(out.rgb[0]) - ref["rgb"])[:, mask]
    assert diff.max() <= 1e-4, (diff.max(), ties.mean())
    target = S.target_image(W, H, seed=1)
    _, g = oracle.l1_loss(ref["rgb"], target)
    g[:, ~mask] = 0.0
    refb = oracle.forward_backward(sc.arrays(), cam, grad_img=g)
    grads = [torch.zeros_like(p) for p in ds.params()]
    fr.backward(ds.struct(), G.grads(*grads), grad_rgb=[torch.from_numpy(g.astype(np.float32)).to(dev)])
    torch.cuda.synchronize()
    for name, t in zip(("mean", "log_scale", "quat", "opacity_logit", "sh"), grads):
        e = _rel_inf(to_np(t), refb["grads"][name])
        assert e <= 1e-3, (name, e)


# ---------------------------------------------------------------------------
# Loss, optimizer, batched cameras
# ---------------------------------------------------------------------------
def test_l1_loss_matches_reference(oracle):
    dev = device()
    G = gsmi()
    rng = np.random.default_rng(0)
    for shape in [(3, 128, 128), (3, 37, 53), (3, 1080, 1920)]:
        a = rng.random(shape).astype(np.float32)
        b = rng.random(shape).astype(np.float32)
        b.reshape(-1)[::97] = a.reshape(-1)[::97]  # exact ties: sign 0
        L, g = oracle.l1_loss(a, b)
        at, bt = torch.from_numpy(a).to(dev), torch.from_numpy(b).to(dev)
        loss = torch.zeros(1, device=dev)
        grad = torch.empty_like(at)
        ws = torch.empty(G.gs_workspace_size(G.GS_OP_L1_LOSS), dtype=torch.uint8, device=dev)
        G.gs_l1_loss(at, bt, at.numel(), loss, grad, ws)
        torch.cuda.synchronize()
        assert abs(loss.item() - L) <= 1e-6 * max(L, 1)
        np.testing.assert_allclose(to_np(grad), g, rtol=1e-6, atol=0)
        # the same values at addresses one float past a 16-byte boundary
        # (the kernel's one-value-per-load path)
        n = at.numel()
        ab = torch.empty(n + 1, device=dev)
        bb = torch.empty(n + 1, device=dev)
        gb = torch.full((n + 2,), 7.0, device=dev)
        ab[1:] = at.reshape(-1)
        bb[1:] = bt.reshape(-1)
        loss.zero_()
        G.gs_l1_loss(ab[1:], bb[1:], n, loss, gb[1:n + 1], ws)
        torch.cuda.synchronize()
        assert abs(loss.item() - L) <= 1e-6 * max(L, 1)
        gh = to_np(gb)
        np.testing.assert_allclose(gh[1:n + 1].reshape(shape), g, rtol=1e-6, atol=0)
        assert gh[0] == 7.0 and gh[n + 1] == 7.0          # nothing written outside


def test_adam_matches_reference(oracle):
    dev = device()
    G = gsmi()
    rng = np.random.default_rng(1)
    sizes = [12288, 4096, 7, 1 << 16, 1001]
    lrs = [1e-3, 2e-2, 5e-2, 3e-4, 1e-2]
    # the last group sits one float past a 16-byte boundary (the kernel's
    # one-value-per-load path)
    offs = [0, 0, 0, 0, 1]

    def on_dev(x, off):
        buf = torch.zeros(x.size + off, device=dev)
        buf[off:] = torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).to(dev)
        return buf[off:]
    p0 = [rng.standard_normal(n).astype(np.float32) for n in sizes]
    ps = [on_dev(x, o) for x, o in zip(p0, offs)]
    ms = [on_dev(np.zeros(n), o) for n, o in zip(sizes, offs)]
    vs = [on_dev(np.zeros(n), o) for n, o in zip(sizes, offs)]
    ref = [(x.astype(np.float64), np.zeros(n), np.zeros(n)) for x, n in zip(p0, sizes)]
    for step in range(1, 5):
        gs = [rng.standard_normal(n).astype(np.float32) for n in sizes]
        G.gs_adam_step(ps, [on_dev(g, o) for g, o in zip(gs, offs)], ms, vs, lrs, 0.9, 0.999, 1e-15, step)
        ref = [oracle.adam_step(p, g, m, v, lr, step) for (p, m, v), g, lr in zip(ref, gs, lrs)]
    torch.cuda.synchronize()
    for t, (p, _, _) in zip(ps, ref):
        np.testing.assert_allclose(to_np(t), p, rtol=2e-6, atol=1e-6)


def test_adam_past_4gb_offsets(oracle):
    """One group of 2^30 + 2^28 + 3 floats (5.4 GB per array): byte offsets
    past 4 GB and a ragged tail.  Windows at the start, middle and end hold
    random values; the rest starts at p = 0.25, g = -0.5.  Two steps with the
    gradients cleared after each read, compared with the reference on the
    windows and at a point of the uniform region."""
    dev = device()
    G = gsmi()
    n = (1 << 30) + (1 << 28) + 3
    print(f"[adam past 4 GB] n={n}", flush=True)
    p = torch.full((n,), 0.25, device=dev)
    g = torch.full((n,), -0.5, device=dev)
    m = torch.zeros(n, device=dev)
    v = torch.zeros(n, device=dev)
    rng = np.random.default_rng(9)
    wins = [(0, 4096), (n // 2 - 2048, n // 2 + 2048), (n - 4099, n)]
    ref = {}
    for a, b in wins:
        x = rng.standard_normal(b - a).astype(np.float32)
        p[a:b] = torch.from_numpy(x).to(dev)
        ref[(a, b)] = (x.astype(np.float64), np.zeros(b - a), np.zeros(b - a))
    probe = n // 4
    ref_u = (np.array([0.25]), np.zeros(1), np.zeros(1))
    for step, g_u in ((1, -0.5), (2, 0.0)):
        gw = {}
        for a, b in wins:
            gw[(a, b)] = rng.standard_normal(b - a).astype(np.float32)
            g[a:b] = torch.from_numpy(gw[(a, b)]).to(dev)
        G.gs_adam_step([p], [g], [m], [v], [1e-2], 0.9, 0.999, 1e-15, step, clear_grads=True)
        for w in wins:
            ref[w] = oracle.adam_step(ref[w][0], gw[w], ref[w][1], ref[w][2], 1e-2, step)
        ref_u = oracle.adam_step(ref_u[0], np.array([g_u]), ref_u[1], ref_u[2], 1e-2, step)
    torch.cuda.synchronize()
    for (a, b), (pr, mr, vr) in ref.items():
        np.testing.assert_allclose(to_np(p[a:b]), pr, rtol=2e-6, atol=1e-6)
        np.testing.assert_allclose(to_np(m[a:b]), mr, rtol=2e-6, atol=1e-7)
        assert (to_np(g[a:b]) == 0).all()
    np.testing.assert_allclose(to_np(p[probe:probe + 1]), ref_u[0], rtol=2e-6, atol=1e-6)
    assert float(g[probe].item()) == 0.0


@pytest.mark.parametrize("n_cams", [3, 8])
def test_batched_cameras_match_single(oracle, n_cams):
    """Cameras of different resolutions in one project/sort/render batch (up
    to the eight cameras a launch takes) give bit-identical images to separate
    single-camera runs."""
    dev = device()
    G = gsmi()
    from paper_2605_13794_amd.raster import DeviceScene
    sc = S.city_scene(1 << 18, seed=7)
    cams = [S.aerial_camera(640, 360, 0.0), S.aerial_camera(320, 200, 90.0), S.aerial_camera(480, 272, 200.0)]
    if n_cams == 8:
        cams += [S.aerial_camera(w, h, a) for w, h, a in
                 [(100, 75, 30.0), (1920, 1080, 130.0), (33, 17, 250.0), (256, 256, 300.0), (720, 405, 45.0)]]
    assert len(cams) == n_cams <= G.GS_MAX_CAMS
    ds = DeviceScene(sc, dev)
    fb = _frame(cams, sc.n, dev)
    out, K = fb.forward(ds.struct())
    torch.cuda.synchronize()
    Ks = 0
    for c, cam in enumerate(cams):
        f1 = _frame([cam], sc.n, dev)
        o1, k1 = f1.forward(ds.struct())
        torch.cuda.synchronize()
        Ks += k1
        assert torch.equal(o1.rgb[0], out.rgb[c])
        assert torch.equal(o1.last[0], out.last[c])
    assert Ks == K
