"""Captured HIP graphs of the hot path: every replay, interleaved with eager
work and synchronisations, matches the eager result."""
from __future__ import annotations

import numpy as np
import pytest
import torch

from paper_2605_13794_amd import scenes as S
from tests.gpuhelp import device, gsmi, to_np

pytestmark = pytest.mark.gpu


def _capture(fn):
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        fn()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        fn()
    torch.cuda.synchronize()
    return g


def test_forward_graph_replays_match_eager():
    dev = device()
    gsmi()
    from paper_2605_13794_amd.raster import DeviceScene, Frame
    sc = S.city_scene(200_000, seed=9)
    cam = S.aerial_camera(640, 360)
    ds = DeviceScene(sc, dev)
    fr = Frame([cam], sc.n, dev)
    fr.forward(ds.struct(), check=True)
    torch.cuda.synchronize()
    ref = fr.rgb[0].clone()
    ref_last = fr.last[0].clone()
    g = _capture(lambda: fr.forward(ds.struct(), check=False))
    other = Frame([S.aerial_camera(320, 180, 90.0)], sc.n, dev)
    for k in range(4):
        fr.rgb[0].zero_()
        other.forward(ds.struct(), check=True)   # eager work between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(fr.rgb[0], ref), k
        assert torch.equal(fr.last[0], ref_last), k


def test_training_step_graph_replays_match_eager():
    """Gated training step (gate, projection, sort, forward, L1, backward,
    Adam with the device step counter) replayed 3 times against 3 eager steps
    from the same start (the backward's float atomics allow rounding-level
    differences)."""
    dev = device()
    G = gsmi()
    from paper_2605_13794_amd.raster import Adam, DEFAULT_LRS, DeviceScene, Frame
    sc = S.city_scene(200_000, seed=9)
    cam = S.aerial_camera(640, 360)
    target = torch.from_numpy(S.target_image(640, 360, seed=2)).to(dev)
    keep = torch.from_numpy((np.arange(sc.n) % 4 != 0).astype(np.uint8)).to(dev)

    def make():
        ds = DeviceScene(sc, dev)
        fr = Frame([cam], sc.n, dev)
        grads = [torch.zeros_like(p) for p in ds.params()]
        opt = Adam(ds.params(), DEFAULT_LRS)
        bits = torch.zeros((sc.n + 31) // 32, dtype=torch.int32, device=dev)
        import oracle
        bits.copy_(torch.from_numpy(oracle.pack_bits(keep.cpu().numpy().astype(bool)).view(np.int32)))
        active = torch.empty(sc.n, dtype=torch.int32, device=dev)
        n_act = torch.zeros(1, dtype=torch.int64, device=dev)
        ws = torch.empty(G.gs_workspace_size(G.GS_OP_LOD_MASK, sc.n), dtype=torch.uint8, device=dev)
        lodp = G.lod_params(G.GS_LOD_RADIUS, radius_min_px=0.5)

        def step(check=False):
            G.gs_lod_mask(ds.struct(), G.camera(cam), lodp, bits, active, n_act, ws)
            fr.forward(ds.struct(), active, sc.n, n_act, check=check)
            fr.l1_loss([target])
            fr.backward(ds.struct(), G.grads(*grads))
            opt.step(grads, clear_grads=True)
        return ds, fr, step

    ds_e, fr_e, step_e = make()
    ds_g, fr_g, step_g = make()
    step_e(check=True)
    step_g(check=True)   # sizes buffers; both runs now at step 1
    torch.cuda.synchronize()
    for _ in range(3):
        step_e()
    g = _capture(step_g)
    torch.cuda.synchronize()
    # _capture ran step_g once eagerly on a side stream (step 2) and recorded it
    # without executing: two more replays give 4 steps in total, like the eager run.
    for k in range(2):
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
    for a, b in zip(ds_e.params(), ds_g.params()):
        np.testing.assert_allclose(to_np(b), to_np(a), rtol=1e-4, atol=1e-6)
