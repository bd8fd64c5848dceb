"""Render server on the GPU: every image is bit-identical whether rendered
alone or inside a continuous batch that overlaps other batches on other
streams (the forward uses no atomics and no order-dependent reduction)."""
from __future__ import annotations

import math

import numpy as np
import pytest
import torch

from paper_2605_13794_amd import scenes as S
from tests.gpuhelp import device, gsmi

pytestmark = pytest.mark.gpu


def test_served_images_equal_alone_and_in_the_mix():
    dev = device()
    gsmi()
    from paper_2605_13794_amd.raster import DeviceScene, Frame
    from paper_2605_13794_amd.serve import GpuExecutor, Request, Scheduler, serve
    sc = S.city_scene(300_000, seed=6)
    ds = DeviceScene(sc, dev)
    rng = np.random.default_rng(0)
    res = [(320, 180), (640, 360), (960, 540), (1280, 720)]
    reqs = []
    for i in range(16):
        w, h = res[int(rng.integers(0, 4))]
        xy = rng.uniform(-300, 300, 2)
        cam = S.yaw_pitch_camera((xy[0], xy[1], rng.uniform(80, 400)), rng.uniform(0, 2 * math.pi),
                                 math.radians(rng.uniform(30, 90)), w, h)
        reqs.append(Request(rid=i, arrival=0.0, cam=cam))   # a burst: batches of up to 4 on 3 streams
    ex = GpuExecutor(ds, n_slots=3, max_batch=4, device=dev)
    sch = Scheduler(n_slots=3, max_batch=4, memory_budget=1 << 30, pairs_per_px=0.5)
    done, images = serve(reqs, ex, sch, keep_images=True)
    torch.cuda.synchronize()
    assert len(done) == 16
    assert sch.n_batches <= 8
    assert max(r.batch for r in done) == sch.n_batches
    for r in done:
        fr = Frame([r.cam], sc.n, dev)
        out, K = fr.forward(ds.struct())
        torch.cuda.synchronize()
        assert torch.equal(out.rgb[0], images[r.rid]), r.rid


def test_served_4k_images_match_reference(oracle):
    """Requests of every served resolution, 3840x2160 among them, in one burst
    over three streams: each served image is bit-identical to the same view
    rendered alone, and that single-view 4K render matches the float64
    reference (max-abs 2e-4 end to end at 3840 px, on the comparable pixels)."""
    dev = device()
    gsmi()
    from paper_2605_13794_amd.raster import DeviceScene, Frame
    from paper_2605_13794_amd.serve import GpuExecutor, Request, Scheduler, serve
    from tests.gpuhelp import comparable_pixels, to_np
    sc = S.city_scene(150_000, seed=7)
    ds = DeviceScene(sc, dev)
    rng = np.random.default_rng(1)
    res = [(3840, 2160), (640, 360), (1920, 1080), (3840, 2160), (1280, 720), (3840, 2160)]
    reqs = []
    for i, (w, h) in enumerate(res * 2):
        xy = rng.uniform(-250, 250, 2)
        cam = S.yaw_pitch_camera((xy[0], xy[1], rng.uniform(120, 300)), rng.uniform(0, 2 * math.pi),
                                 math.radians(rng.uniform(40, 80)), w, h)
        reqs.append(Request(rid=i, arrival=0.0, cam=cam))
    ex = GpuExecutor(ds, n_slots=3, max_batch=4, device=dev)
    sch = Scheduler(n_slots=3, max_batch=4, memory_budget=4 << 30, pairs_per_px=0.5)
    done, images = serve(reqs, ex, sch, keep_images=True)
    torch.cuda.synchronize()
    assert len(done) == len(reqs)
    singles = {}
    for r in done:
        fr = Frame([r.cam], sc.n, dev)
        out, K = fr.forward(ds.struct())
        torch.cuda.synchronize()
        assert torch.equal(out.rgb[0], images[r.rid]), r.rid
        singles[r.rid] = (fr, out)
    # the first 4K view against the reference
    r = next(r for r in reqs if r.cam.width == 3840)
    fr, out = singles[r.rid]
    ref = oracle.forward_backward(sc.arrays(), r.cam)
    mask, n_bad = comparable_pixels(ref, to_np(fr.proj[0].radius), r.cam.width, r.cam.height)
    assert n_bad <= 3 and mask.mean() > 0.95, (n_bad, mask.mean())
    diff = np.abs(to_np(out.rgb[0]) - ref["rgb"])[:, mask]
    # float32 screen coordinates between 2,048 and 4,096 px are 2.4e-4 px apart
    # (twice the spacing of a 1080p view), so the end-to-end drift doubles
    assert diff.max() <= 2e-4, diff.max()
