"""GPU parity of whole training paths that the benchmark runs, end to end from
the parameters, against the float64 reference, through the C ABI:

  - the gated path: gs_lod_mask -> gs_project over the device-resident active
    list and count -> gs_bin_sort -> gs_render_fwd -> gs_l1_loss ->
    gs_render_bwd with the same list and count, whose gradients land at the
    Gaussians the list names (Sec. 3.3, Eq. 3: the backward runs over the
    active set only);
  - inputs of more than 2,097,152 entries, where projection and backward
    switch to their large-chunk list-building kernels;
  - a batch of four cameras in one projection / sort / compositing / backward
    (the multi-view training batch).

Tolerances as in the other parity tests: images max-abs 1e-4 end to end on
pixels whose decisions are not near a threshold, gradients per tensor
max|g - g_ref| <= 1e-3 max|g_ref|, active lists bit-exact, and gradients
exactly zero at every Gaussian outside the active list.
"""
from __future__ import annotations

import math

import numpy as np
import pytest
import torch

from paper_2605_13794_amd import scenes as S
from tests.gpuhelp import comparable_pixels, device, gsmi, rel_inf, to_np

pytestmark = pytest.mark.gpu

NAMES = ("mean", "log_scale", "quat", "opacity_logit", "sh")
SMALL_LIST_INPUT = 2 << 20   # entries above which the large-chunk kernels run


def _frame(cams, n, dev, **kw):
    from paper_2605_13794_amd.raster import Frame
    return Frame(cams, n, dev, **kw)


def _gate_and_keep(oracle, sc, cam, mode, rng, keep_frac=0.7):
    """Reference gate of one view and a random keep mask (dropping visible
    Gaussians too).  Gaussians whose gate value lies within a relative 1e-4
    of the gate's threshold are removed from the keep mask as well, so that
    the float32 gate and the float64 one decide every listed Gaussian alike.
    Returns (lod params, gate, keep mask, reference active list)."""
    G = gsmi()
    pos = cam.position
    if mode == "radius":
        rmin = 0.5
        gate, r = oracle.lod_gate_radius(sc.mean, sc.log_scale, pos, cam.fx, rmin)
        near = np.abs(r - rmin) <= 1e-4 * rmin
        params = G.lod_params(G.GS_LOD_RADIUS, fallback_ratio=0.95, radius_min_px=rmin, radius_sigma_k=1.0)
    else:
        d = np.linalg.norm(sc.mean.astype(np.float64) - pos[:, None], axis=0)
        d0, l_max = float(np.median(d)), 7
        gate = oracle.lod_gate_level(sc.mean, sc.lod, pos, d0, l_max)
        x = np.log2(d0 / d) + 0.5
        near = np.abs(x - np.round(x)) <= 1e-4
        params = G.lod_params(G.GS_LOD_LEVEL, d0=d0, f=2.0, l_max=l_max, fallback_ratio=0.95)
    keep = (rng.random(sc.n) < keep_frac) & ~near
    act = oracle.active_set(gate, oracle.pack_bits(keep), 0.95)
    # the gate acts (no fall-back) and removes Gaussians the camera sees
    assert 0.2 < gate.mean() < 0.95, gate.mean()
    return params, gate, keep, act


def _device_gate(ds, cam, params, keep, dev):
    import oracle as O
    G = gsmi()
    n = ds.n
    kb = torch.from_numpy(O.pack_bits(keep).view(np.int32).copy()).to(dev)
    active = torch.full((n,), -7, dtype=torch.int32, device=dev)
    n_act = torch.zeros(1, dtype=torch.int64, device=dev)
    ws = torch.empty(G.gs_workspace_size(G.GS_OP_LOD_MASK, n), dtype=torch.uint8, device=dev)
    G.gs_lod_mask(ds.struct(), G.camera(cam), params, kb, active, n_act, ws)
    return active, n_act


def _check_images(fr, refs, cams, tol=1e-4):
    """Returns per camera the comparable-pixel mask after checking the image
    there."""
    masks = []
    for c, (cam, ref) in enumerate(zip(cams, refs)):
        mask, nbad = comparable_pixels(ref, to_np(fr.proj[c].radius), cam.width, cam.height)
        assert nbad <= 3 and mask.mean() > 0.95, (c, nbad, mask.mean())
        diff = np.abs(to_np(fr.rgb[c]) - ref["rgb"])[:, mask]
        assert diff.max() <= tol, (c, diff.max())
        masks.append(mask)
    return masks


def _masked_l1_grad(oracle, ref, target, mask):
    _, g = oracle.l1_loss(ref["rgb"], target)
    g[:, ~mask] = 0.0
    return g


def _scatter(act, grads_sub, n):
    out = {}
    for k, g in grads_sub.items():
        full = np.zeros(g.shape[:-1] + (n,), dtype=np.float64)
        full[..., act] = g
        out[k] = full
    return out


def _gated_path(oracle, sc, cam, mode, seed):
    dev = device()
    G = gsmi()
    from paper_2605_13794_amd.raster import DeviceScene
    rng = np.random.default_rng(seed)
    params, gate, keep, act = _gate_and_keep(oracle, sc, cam, mode, rng)
    ds = DeviceScene(sc, dev)
    print(f"[gated path] mode={mode} n={sc.n} active={act.size} {cam.width}x{cam.height}", flush=True)
    active, n_act = _device_gate(ds, cam, params, keep, dev)
    fr = _frame([cam], sc.n, dev)
    out, K = fr.forward(ds.struct(), active, sc.n, n_act)
    target = torch.from_numpy(S.target_image(cam.width, cam.height, seed=seed)).to(dev)
    fr.l1_loss([target])
    torch.cuda.synchronize()
    # the device active list is the reference's, in ascending order
    na = int(n_act.item())
    assert na == act.size
    np.testing.assert_array_equal(to_np(active)[:na], act)
    sub = sc.subset(act)
    ref = oracle.forward_backward(sub.arrays(), cam)
    # entries past the device count are projected as culled
    assert not to_np(fr.proj[0].radius)[na:].any()
    (mask,) = _check_images(fr, [ref], [cam])
    loss_ref, _ = oracle.l1_loss(ref["rgb"], S.target_image(cam.width, cam.height, seed=seed))
    assert abs(float(fr.loss[0].item()) - loss_ref) <= 1e-3
    g = _masked_l1_grad(oracle, ref, S.target_image(cam.width, cam.height, seed=seed), mask)
    refb = oracle.forward_backward(sub.arrays(), cam, grad_img=g)
    grads = [torch.zeros_like(p) for p in ds.params()]
    fr.backward(ds.struct(), G.grads(*grads), grad_rgb=[torch.from_numpy(g.astype(np.float32)).to(dev)])
    torch.cuda.synchronize()
    full = _scatter(act, refb["grads"], sc.n)
    outside = np.ones(sc.n, dtype=bool)
    outside[act] = False
    for name, t in zip(NAMES, grads):
        got = to_np(t)
        e = rel_inf(got, full[name])
        assert e <= 1e-3, (name, e)
        assert not got[..., outside].any(), name      # nothing outside the active set
    return K


@pytest.mark.parametrize("mode", ["radius", "level"])
def test_gated_training_path_matches_reference(oracle, mode):
    """400k city Gaussians, one 640x360 aerial view: the gate (radius or
    level mode) and a keep mask that drops visible Gaussians."""
    sc = S.city_scene(400_000, seed=21).spatially_ordered()
    cam = S.aerial_camera(640, 360, heading_deg=20.0)
    K = _gated_path(oracle, sc, cam, mode, seed=31)
    assert K > 10_000


def test_large_input_plain_matches_reference(oracle):
    """2.3M Gaussians projected and differentiated without a list: the
    projection's cull and the backward's visible-entry list run their
    large-chunk kernels."""
    dev = device()
    G = gsmi()
    from paper_2605_13794_amd.raster import DeviceScene
    n = 2_300_000
    assert n > SMALL_LIST_INPUT
    sc = S.city_scene(n, seed=8)
    cam = S.aerial_camera(320, 180)
    print(f"[large plain] n={n}", flush=True)
    ds = DeviceScene(sc, dev)
    fr = _frame([cam], n, dev, capacity=1 << 20)
    out, K = fr.forward(ds.struct())
    torch.cuda.synchronize()
    ref = oracle.forward_backward(sc.arrays(), cam)
    assert K == ref["K"] or abs(K - ref["K"]) <= 64
    (mask,) = _check_images(fr, [ref], [cam])
    g = _masked_l1_grad(oracle, ref, S.target_image(cam.width, cam.height, seed=3), mask)
    refb = oracle.forward_backward(sc.arrays(), cam, grad_img=g)
    grads = [torch.zeros_like(p) for p in ds.params()]
    fr.backward(ds.struct(), G.grads(*grads), grad_rgb=[torch.from_numpy(g.astype(np.float32)).to(dev)])
    torch.cuda.synchronize()
    for name, t in zip(NAMES, grads):
        e = rel_inf(to_np(t), refb["grads"][name])
        assert e <= 1e-3, (name, e)


def test_projection_past_4gb_offsets(oracle):
    """24 x 2^20 + 5 Gaussians, so the [16][3][n] coefficient array (4.8 GB)
    has rows past 4 GB: an 8,192-Gaussian scene repeated along the index and
    projected in one call (the single-pass kernel of large inputs); entries
    at the start, middle and end are compared with the reference's
    projection of the base scene, with the tolerances of the projection
    parity test."""
    dev = device()
    G = gsmi()
    from paper_2605_13794_amd.raster import ProjBuffers
    base = S.cube_scene(8192, seed=7)
    cam = S.cube_camera(128, 128, 128.0)
    n, nb = 24 * (1 << 20) + 5, base.n
    print(f"[projection past 4 GB] n={n}", flush=True)
    idx = torch.arange(n, device=dev) % nb
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)  # noqa: E731
    mean = t(base.mean)[:, idx].contiguous()
    log_scale = t(base.log_scale)[:, idx].contiguous()
    quat = t(base.quat)[:, idx].contiguous()
    opac = t(base.opacity_logit)[idx].contiguous()
    sh = t(base.sh)[:, :, idx].contiguous()
    del idx
    assert sh.numel() * 4 > (1 << 32)
    pb = ProjBuffers(n, dev, soa=True)
    ws = torch.empty(G.gs_workspace_size(G.GS_OP_PROJECT, n), dtype=torch.uint8, device=dev)
    G.gs_project(G.scene(mean, log_scale, quat, opac, sh), None, n, None, G.camera_array([cam]), [pb.struct()], ws)
    torch.cuda.synchronize()
    _, out, pr = oracle.project(base.arrays(), cam)
    lam = out["lam"].numpy()
    e = 3.0 * np.sqrt(np.maximum(lam, 0))
    m2 = out["mean2d"].detach().numpy().T
    amb = (np.abs(e - np.round(e)) < 1e-4 * np.maximum(e, 1)) | (np.abs(m2 - np.round(m2)) < 1e-3).any(0) | \
          (np.abs(out["depth"].detach().numpy() - cam.znear) < 1e-5)
    ok = ~amb
    vis = ok & (pr.radius > 0)
    scale = max(cam.width, cam.height)
    for j0 in (0, (n // 2) // nb * nb, (n - 5) // nb * nb - nb):
        sl = slice(j0, j0 + nb)
        np.testing.assert_array_equal(to_np(pb.radius[sl])[ok], pr.radius[ok])
        np.testing.assert_allclose(to_np(pb.mean2d[:, sl])[:, vis], pr.mean2d[:, vis], rtol=0, atol=2e-7 * scale * 4)
        np.testing.assert_allclose(to_np(pb.depth[sl])[vis], pr.depth[vis], rtol=1e-6)
        np.testing.assert_allclose(to_np(pb.rgb[:, sl])[:, vis], pr.rgb[:, vis], atol=2e-6)
    # the last five entries repeat base Gaussians 0..4 bit for bit
    tail = slice(n - 5, n)
    np.testing.assert_array_equal(to_np(pb.rgb[:, tail]), to_np(pb.rgb[:, 0:5]))
    np.testing.assert_array_equal(to_np(pb.radius[tail]), to_np(pb.radius[0:5]))


def test_large_input_gated_matches_reference(oracle):
    """The gated path over a 2.3M-Gaussian shard (list of 2.3M entries of
    capacity, device count below it)."""
    sc = S.city_scene(2_300_000, seed=9).spatially_ordered()
    cam = S.aerial_camera(320, 180, heading_deg=-35.0)
    _gated_path(oracle, sc, cam, "radius", seed=41)


@pytest.mark.parametrize("headings", [(0.0, 90.0, 180.0, 270.0), tuple(45.0 * k for k in range(8))],
                         ids=["four_views", "eight_views"])
def test_four_camera_batch_backward_matches_reference(oracle, headings):
    """Four views (the aerial pose at headings 0, 90, 180, 270 degrees), and
    the eight a launch takes (every 45 degrees), in one batch: images per
    camera and parameter gradients summed over the views against the
    reference run per camera."""
    dev = device()
    G = gsmi()
    from paper_2605_13794_amd.raster import DeviceScene
    sc = S.city_scene(300_000, seed=23).spatially_ordered()
    cams = [S.aerial_camera(320, 180, h) for h in headings]
    ds = DeviceScene(sc, dev)
    fr = _frame(cams, sc.n, dev)
    out, K = fr.forward(ds.struct())
    torch.cuda.synchronize()
    refs = [oracle.forward_backward(sc.arrays(), cam) for cam in cams]
    assert K == sum(r["K"] for r in refs) or abs(K - sum(r["K"] for r in refs)) <= 64
    masks = _check_images(fr, refs, cams)
    total = {k: 0.0 for k in NAMES}
    gs = []
    for c, (cam, ref, mask) in enumerate(zip(cams, refs, masks)):
        g = _masked_l1_grad(oracle, ref, S.target_image(cam.width, cam.height, seed=50 + c), mask)
        gs.append(torch.from_numpy(g.astype(np.float32)).to(dev))
        rb = oracle.forward_backward(sc.arrays(), cam, grad_img=g)
        for k in NAMES:
            total[k] = total[k] + rb["grads"][k]
    grads = [torch.zeros_like(p) for p in ds.params()]
    fr.backward(ds.struct(), G.grads(*grads), grad_rgb=gs)
    torch.cuda.synchronize()
    for name, t in zip(NAMES, grads):
        e = rel_inf(to_np(t), total[name])
        assert e <= 1e-3, (name, e)


def test_l1_loss_autograd_function(oracle):
    """L1LossFn: the loss and the gradient scaled by the upstream derivative
    (read on the device) against the reference; gs_l1_loss with only one of
    its two outputs."""
    dev = device()
    G = gsmi()
    from paper_2605_13794_amd.raster import l1_loss
    rng = np.random.default_rng(5)
    a = rng.random((2, 3, 37, 53)).astype(np.float32)
    b = rng.random((2, 3, 37, 53)).astype(np.float32)
    b.reshape(-1)[::31] = a.reshape(-1)[::31]          # exact ties: sign 0
    L, g = oracle.l1_loss(a, b)
    x = torch.from_numpy(a).to(dev).requires_grad_(True)
    y = torch.from_numpy(b).to(dev)
    loss = l1_loss(x, y)
    (loss * 2.5).backward()
    torch.cuda.synchronize()
    assert abs(float(loss.item()) - L) <= 1e-6 * max(L, 1)
    np.testing.assert_allclose(to_np(x.grad), 2.5 * g, rtol=1e-6, atol=0)
    # loss only, and gradient only
    ws = torch.empty(G.gs_workspace_size(G.GS_OP_L1_LOSS), dtype=torch.uint8, device=dev)
    lo = torch.zeros(1, device=dev)
    G.gs_l1_loss(x.detach(), y, x.numel(), lo, None, ws)
    gr = torch.full_like(y, 9.0)
    G.gs_l1_loss(x.detach(), y, x.numel(), None, gr, None)
    torch.cuda.synchronize()
    assert abs(float(lo.item()) - L) <= 1e-6 * max(L, 1)
    np.testing.assert_allclose(to_np(gr), g, rtol=1e-6, atol=0)
    with pytest.raises(G.GsmiError):
        G.gs_l1_loss(x.detach(), y, x.numel(), None, None, ws)


def test_rasterize_stale_frame_raises(oracle):
    """A second forward through a frame before the first graph's backward
    makes that backward raise (the frame holds only its latest lists)."""
    device()
    gsmi()
    from paper_2605_13794_amd.raster import DeviceScene, Frame, rasterize
    sc = S.cube_scene(256, seed=2)
    ds = DeviceScene(sc, "cuda:0", requires_grad=True)
    fr = Frame([S.cube_camera(32, 32, 32.0)], sc.n, "cuda:0")
    first = rasterize(fr, ds)
    second = rasterize(fr, ds)
    with pytest.raises(RuntimeError, match="another forward"):
        first.sum().backward()
    second.sum().backward()     # the latest forward still differentiates
    torch.cuda.synchronize()
    assert ds.mean.grad is not None and torch.isfinite(ds.mean.grad).all()


def test_backward_overwrite_mode():
    """gs_grads.overwrite = 1 stores the reached Gaussians' gradients: equal
    to accumulating into zeros (up to the last bits of the blend's float
    atomics, which differ between two backward calls), and Gaussians the view
    does not reach keep whatever their arrays held."""
    from paper_2605_13794_amd.raster import DeviceScene
    dev = device()
    G = gsmi()
    sc = S.city_scene(200_000, seed=31)
    cam = S.aerial_camera(480, 270, 20.0)
    ds = DeviceScene(sc, dev)
    fr = _frame([cam], sc.n, dev)
    fr.forward(ds.struct())
    tgt = torch.from_numpy(S.target_image(480, 270, seed=3)).to(dev)
    fr.l1_loss([tgt])
    acc = [torch.zeros_like(p) for p in ds.params()]
    fr.backward(ds.struct(), G.grads(*acc))
    over = [torch.full_like(p, 7.0) for p in ds.params()]
    fr.backward(ds.struct(), G.grads(*over, overwrite=True))
    torch.cuda.synchronize()
    reached = (fr.proj[0].radius[:sc.n] > 0)
    assert 0 < int(reached.sum()) < sc.n
    for a, o in zip(acc, over):
        a2, o2 = a.reshape(-1, sc.n), o.reshape(-1, sc.n)
        ar, orr = a2[:, reached], o2[:, reached]
        assert float((ar - orr).abs().max()) <= 1e-5 * float(ar.abs().max())
        assert bool((o2[:, ~reached] == 7.0).all())
