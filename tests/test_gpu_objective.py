"""GPU parity of the paper's objective (Eqs. 4-5) against the float64
reference: L1 + SSIM photometric loss with its gradient, and the scale
regulariser over the visible set."""
from __future__ import annotations

import numpy as np
import pytest
import torch

from paper_2605_13794_amd import scenes as S
from tests.gpuhelp import device, gsmi, to_np

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("shape", [(3, 37, 53), (3, 128, 128), (3, 540, 960)])
def test_photo_loss_matches_reference(oracle, shape):
    dev = device()
    G = gsmi()
    rng = np.random.default_rng(shape[1])
    x = rng.random(shape).astype(np.float32)
    y = np.clip(x + 0.2 * rng.standard_normal(shape), 0, 1).astype(np.float32)
    y.reshape(-1)[::101] = x.reshape(-1)[::101]
    L, g = oracle.photo_loss(x.astype(np.float64), y.astype(np.float64), 0.2)
    H, W = shape[1], shape[2]
    xt, yt = torch.from_numpy(x).to(dev), torch.from_numpy(y).to(dev)
    loss = torch.zeros(1, device=dev)
    grad = torch.empty_like(xt)
    ws = torch.empty(G.gs_workspace_size(G.GS_OP_PHOTO_LOSS, W * 65536 + H), dtype=torch.uint8, device=dev)
    G.gs_photo_loss(xt, yt, W, H, 0.2, 1.0, loss, grad, ws)
    torch.cuda.synchronize()
    assert abs(loss.item() - L) <= 1e-5 * abs(L)
    gg = to_np(grad)
    assert np.abs(gg - g).max() <= 1e-3 * np.abs(g).max()
    # scale applies to both
    G.gs_photo_loss(xt, yt, W, H, 0.2, 0.25, loss, grad, ws)
    torch.cuda.synchronize()
    assert abs(loss.item() - 0.25 * L) <= 1e-5 * abs(L)
    np.testing.assert_allclose(to_np(grad), 0.25 * gg, rtol=1e-6, atol=0)


def test_scale_reg_matches_reference(oracle):
    dev = device()
    G = gsmi()
    from paper_2605_13794_amd.raster import DeviceScene
    sc = S.city_scene(50_000, seed=4)
    rng = np.random.default_rng(0)
    active = np.sort(rng.choice(sc.n, 30_000, replace=False)).astype(np.int32)
    radius = np.where(rng.random(30_000) < 0.6, 3, 0).astype(np.int32)
    vis = np.zeros(sc.n, dtype=bool)
    vis[active[radius > 0]] = True
    L, g = oracle.scale_reg(sc.log_scale, vis, beta=10.0)
    ds = DeviceScene(sc, dev)
    loss = torch.zeros(1, device=dev)
    grad = torch.zeros(3, sc.n, device=dev)
    ws = torch.empty(G.gs_workspace_size(G.GS_OP_SCALE_REG), dtype=torch.uint8, device=dev)
    n_in_dev = torch.tensor([30_000], dtype=torch.int64, device=dev)
    G.gs_scale_reg(ds.struct(), torch.from_numpy(active).to(dev), 30_000, n_in_dev,
                   torch.from_numpy(radius).to(dev), 10.0, loss, grad, ws)
    torch.cuda.synchronize()
    assert abs(loss.item() - L) <= 1e-5 * L
    np.testing.assert_allclose(to_np(grad), g, rtol=1e-5, atol=1e-12)
