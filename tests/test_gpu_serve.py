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
