"""GPU parity of the importance sweep, the view-level gate, the score mask
and the autograd wrapper against the float64 reference, through the C ABI.

Decisions taken from floats (top-mass membership, gate predicates) are
compared exactly except for elements whose reference value sits within a
stated relative band of the threshold, which may go either way in float32.
"""
from __future__ import annotations

import math

import numpy as np
import pytest
import torch

from paper_2605_13794_amd import scenes as S
from tests.gpuhelp import device, gsmi, to_np, u32, upload_projection
from tests.test_gpu_parity import make_case

pytestmark = pytest.mark.gpu


def _lists(prf, cam, dev, oracle):
    K, keys, vals, ranges = oracle.bin_sort(prf, cam.width, cam.height)
    v = torch.from_numpy(np.asarray(vals, dtype=np.uint32).view(np.int32).copy()).to(dev)
    if v.numel() == 0:
        v = torch.zeros(1, dtype=torch.int32, device=dev)
    r = torch.from_numpy(np.asarray(ranges, dtype=np.uint32).reshape(-1).view(np.int32).copy()).to(dev)
    return K, keys, vals, ranges, v, r


def _affected(vals, ranges, margin, width):
    """Gaussians listed in a tile that holds a pixel with a near-threshold
    decision (their counts may differ by that pixel)."""
    TX = -(-width // 16)
    bad_t = set()
    for (y, x) in zip(*np.nonzero(margin < 1e-5)):
        bad_t.add((y // 16) * TX + x // 16)
    out = set()
    for t in bad_t:
        out.update(np.asarray(vals[ranges[0, t]:ranges[1, t]]).tolist())
    return np.array(sorted(out), dtype=np.int64)


@pytest.mark.parametrize("case", ["cfg1", "city"])
def test_importance_matches_reference(oracle, case):
    dev = device()
    G = gsmi()
    sc, cam0 = make_case(case)
    cams = [cam0]
    if case == "cfg1":
        cams.append(S.look_at((1.5, -1.0, -3.5), (0, 0, 0), 128, 128, up=(0, -1, 0)))
    else:
        cams.append(S.aerial_camera(480, 270, 30.0))
    n = sc.n
    st = oracle.ImportanceState(n, len(cams))
    score = torch.zeros(n, device=dev)
    c_rad = torch.zeros(n, dtype=torch.int32, device=dev)
    c_vis = torch.zeros(n, dtype=torch.int32, device=dev)
    cull = torch.zeros(len(cams), (n + 31) // 32, dtype=torch.int32, device=dev)
    w = torch.empty(n, device=dev)
    a = torch.empty(n, dtype=torch.int32, device=dev)
    ws = torch.empty(G.gs_workspace_size(G.GS_OP_IMPORTANCE, n), dtype=torch.uint8, device=dev)
    ambiguous = np.zeros(n, dtype=bool)
    for v_i, cam in enumerate(cams):
        _, out, pr = oracle.project(sc.arrays(), cam)
        prf = pr.rounded_f32()
        K, keys, vals, ranges, vt, rt = _lists(prf, cam, dev, oracle)
        w_ref, a_ref = oracle.importance_blend(prf, vals, ranges, cam.width, cam.height)
        fwd = oracle.render_fwd(prf, vals, ranges, cam.width, cam.height)
        oracle.importance_fold(st, v_i, w_ref, a_ref, prf.radius)
        pb = upload_projection(prf, cam.width, cam.height, dev)
        G.gs_importance(pb.struct(), G.camera(cam), n, vt, rt, 0.99, 1e-6, w, a, score, c_rad, c_vis, cull[v_i], ws)
        torch.cuda.synchronize()
        aff = _affected(vals, ranges, fwd["margin"], cam.width)
        ok = np.ones(n, dtype=bool)
        ok[aff] = False
        wg = to_np(w)
        assert np.abs(wg - w_ref).max() <= 1e-4 * max(w_ref.max(), 1e-12)
        np.testing.assert_array_equal(u32(a)[ok], a_ref[ok])
        # membership band around the cut of this view
        idx = np.nonzero(w_ref > 0)[0]
        order = idx[np.lexsort((idx, -w_ref[idx]))]
        cs = np.cumsum(w_ref[order])
        W = cs[-1]
        before = cs - w_ref[order]
        tau = w_ref[order][int(np.searchsorted(cs, 0.99 * W))]
        band = np.zeros(n, dtype=bool)
        band[order[np.abs(before - 0.99 * W) <= 1e-5 * W]] = True
        band |= np.abs(w_ref - tau) <= 1e-4 * tau
        ambiguous |= band | ~ok
        cvis_g = ~oracle.unpack_bits(u32(cull[v_i]), n)
        cvis_r = oracle.top_mass(w_ref)
        diff = cvis_g != cvis_r
        assert not (diff & ~band & ok).any(), np.nonzero(diff & ~band & ok)[0][:10]
        assert band.sum() < 0.01 * n + 5
    amb = ambiguous
    np.testing.assert_array_equal(u32(c_rad), st.c_rad.astype(np.uint32))
    np.testing.assert_array_equal(u32(c_vis)[~amb], st.c_vis[~amb].astype(np.uint32))
    sg = to_np(score)
    assert np.abs(sg - st.score)[~amb].max() <= 1e-4 * max(st.score.max(), 1e-12)


@pytest.mark.parametrize("case", ["cfg1", "city"])
def test_importance_footprint_count_matches_reference(oracle, case):
    """The footprint reading of a (GS_COUNT_FOOTPRINT): every pixel of the
    Gaussian's tiles inside its 1/255 footprint, occluded or not.  w is as in
    the composited reading; counts agree except for a few Gaussians with a
    pixel on the 1/255 boundary (float32 against float64), by at most 2."""
    dev = device()
    G = gsmi()
    sc, cam = make_case(case)
    n = sc.n
    _, out, pr = oracle.project(sc.arrays(), cam)
    prf = pr.rounded_f32()
    K, keys, vals, ranges, vt, rt = _lists(prf, cam, dev, oracle)
    w_ref, a_ref = oracle.importance_blend(prf, vals, ranges, cam.width, cam.height, footprint=True)
    _, a_comp = oracle.importance_blend(prf, vals, ranges, cam.width, cam.height)
    assert (a_ref >= a_comp).all() and (a_ref > a_comp).any()
    pb = upload_projection(prf, cam.width, cam.height, dev)
    w = torch.empty(n, device=dev)
    a = torch.empty(n, dtype=torch.int32, device=dev)
    score = torch.zeros(n, device=dev)
    c_rad = torch.zeros(n, dtype=torch.int32, device=dev)
    c_vis = torch.zeros(n, dtype=torch.int32, device=dev)
    cull = torch.zeros((n + 31) // 32, dtype=torch.int32, device=dev)
    ws = torch.empty(G.gs_workspace_size(G.GS_OP_IMPORTANCE, n), dtype=torch.uint8, device=dev)
    G.gs_importance(pb.struct(), G.camera(cam), n, vt, rt, 0.99, 1e-6, w, a, score, c_rad, c_vis, cull, ws,
                    count_mode=G.GS_COUNT_FOOTPRINT)
    torch.cuda.synchronize()
    assert np.abs(to_np(w) - w_ref).max() <= 1e-4 * max(w_ref.max(), 1e-12)
    d = u32(a).astype(np.int64) - a_ref
    assert np.abs(d).max() <= 2
    assert (d != 0).sum() <= max(5, n // 1000), (d != 0).sum()


def test_score_keep_bits_bitexact(oracle):
    dev = device()
    G = gsmi()
    rng = np.random.default_rng(3)
    for n in [1, 1000, 4096 + 37, 1 << 20]:
        s = rng.exponential(1.0, n).astype(np.float32)
        s[rng.random(n) < 0.3] = 0.0                      # never-seen Gaussians
        s[rng.random(n) < 0.05] = np.float32(0.5)          # ties away from zero
        st = torch.from_numpy(s).to(dev)
        ws = torch.empty(G.gs_workspace_size(G.GS_OP_SCORE_KEEP, n), dtype=torch.uint8, device=dev)
        for frac in [0.0, 0.4, 0.31, 1.0]:
            n_drop = oracle.drop_count(n, frac)
            keep = torch.zeros((n + 31) // 32, dtype=torch.int32, device=dev)
            G.gs_score_keep_bits(st, n, n_drop, keep, ws)
            torch.cuda.synchronize()
            ref = oracle.pack_bits(oracle.score_keep(s.astype(np.float64), n_drop))
            np.testing.assert_array_equal(u32(keep), ref)


def _gate_case(n=200000):
    sc = S.city_scene(n, seed=12)
    cam = S.aerial_camera(1920, 1080, 20.0)
    return sc, cam


@pytest.mark.parametrize("mode,with_keep,n", [(m, k, 200000) for m in ("radius", "level", "none")
                                              for k in (False, True)] + [("radius", True, 2600000)])
def test_lod_mask_matches_reference(oracle, mode, with_keep, n):
    """2.6M Gaussians take the larger per-workgroup chunk of the gate."""
    dev = device()
    G = gsmi()
    from paper_2605_13794_amd.raster import DeviceScene
    sc, cam = _gate_case(n)
    n = sc.n
    ds = DeviceScene(sc, dev)
    campos = cam.position.astype(np.float32).astype(np.float64)
    rng = np.random.default_rng(0)
    keepm = rng.random(n) < 0.7
    bits = oracle.pack_bits(keepm) if with_keep else None
    fb = float(np.float32(0.95))
    mean64 = sc.mean.astype(np.float64)
    if mode == "radius":
        gate, r = oracle.lod_gate_radius(mean64, sc.log_scale, campos, cam.fx, 2.0)
        amb = np.abs(r - 2.0) <= 1e-5 * 2.0
        params = G.lod_params(G.GS_LOD_RADIUS, fallback_ratio=fb, radius_min_px=2.0, radius_sigma_k=1.0)
    elif mode == "level":
        d = np.linalg.norm(mean64 - campos[:, None], axis=0)
        d0 = float(np.median(d))
        gate = oracle.lod_gate_level(mean64, sc.lod, campos, d0=d0, l_max=3)
        x = np.log2(d0 / d) + 0.5
        amb = np.abs(x - np.round(x)) <= 1e-5
        params = G.lod_params(G.GS_LOD_LEVEL, d0=d0, f=2.0, l_max=3, fallback_ratio=fb)
    else:
        gate = np.ones(n, dtype=bool)
        amb = np.zeros(n, dtype=bool)
        params = G.lod_params(G.GS_LOD_NONE, fallback_ratio=fb)
    ratio = gate.sum() / n
    assert abs(ratio - 0.95) > 1e-3 or mode == "none"
    ref = oracle.active_set(gate, bits, fallback_ratio=fb)
    active = torch.empty(n, dtype=torch.int32, device=dev)
    n_act = torch.zeros(1, dtype=torch.int64, device=dev)
    ws = torch.empty(G.gs_workspace_size(G.GS_OP_LOD_MASK, n), dtype=torch.uint8, device=dev)
    kb = torch.from_numpy(bits.view(np.int32).copy()).to(dev) if bits is not None else None
    G.gs_lod_mask(ds.struct(), G.camera(cam), params, kb, active, n_act, ws)
    torch.cuda.synchronize()
    m = int(n_act.item())
    got = to_np(active[:m]).astype(np.int64)
    assert (np.diff(got) > 0).all()
    sym = np.setxor1d(got, ref)
    assert amb[sym].all(), sym[~amb[sym]][:10]
    assert sym.size <= max(5, 1e-4 * n)


def test_lod_mask_several_rounds_per_workgroup(oracle):
    """Above 2,048 x 8,192 Gaussians every compaction workgroup takes its
    words in several rounds of 256: random means and log-scales, radius gate
    with keep bits, then the same input with a fallback that the gate trips."""
    dev = device()
    G = gsmi()
    n = 2048 * 8192 + 12345
    rng = np.random.default_rng(21)
    mean = np.empty((3, n), dtype=np.float32)
    mean[:2] = rng.uniform(-500.0, 500.0, (2, n))
    mean[2] = rng.uniform(0.0, 80.0, n)
    log_scale = rng.normal(np.log(0.3), 0.7, (3, n)).astype(np.float32)
    keepm = rng.random(n) < 0.7
    bits = oracle.pack_bits(keepm)
    cam = S.aerial_camera(1920, 1080, 20.0)
    campos = cam.position.astype(np.float32).astype(np.float64)
    gate, r = oracle.lod_gate_radius(mean.astype(np.float64), log_scale, campos, cam.fx, 2.0)
    amb = np.abs(r - 2.0) <= 1e-5 * 2.0
    assert 0.2 < gate.mean() < 0.8
    mean_t, ls_t = torch.from_numpy(mean).to(dev), torch.from_numpy(log_scale).to(dev)
    scene = G.scene(mean_t, ls_t, None, None, None)
    kb = torch.from_numpy(bits.view(np.int32).copy()).to(dev)
    active = torch.empty(n, dtype=torch.int32, device=dev)
    n_act = torch.zeros(1, dtype=torch.int64, device=dev)
    ws = torch.empty(G.gs_workspace_size(G.GS_OP_LOD_MASK, n), dtype=torch.uint8, device=dev)
    for fb in (0.95, 0.1):
        ref = oracle.active_set(gate, bits, fallback_ratio=fb)
        params = G.lod_params(G.GS_LOD_RADIUS, fallback_ratio=fb, radius_min_px=2.0, radius_sigma_k=1.0)
        G.gs_lod_mask(scene, G.camera(cam), params, kb, active, n_act, ws)
        torch.cuda.synchronize()
        m = int(n_act.item())
        got = to_np(active[:m]).astype(np.int64)
        assert (np.diff(got) > 0).all()
        sym = np.setxor1d(got, ref)
        assert amb[sym].all(), sym[~amb[sym]][:10]
        assert sym.size <= max(5, 1e-4 * n)
        if fb < 0.5:
            np.testing.assert_array_equal(got, np.nonzero(keepm)[0])


@pytest.mark.parametrize("n", [1, 31, 33, 511, 513, 2049])
def test_lod_mask_small_sizes(oracle, n):
    """Ragged sizes around the 32-Gaussian words and the 512-Gaussian chunks of
    the gate: level gate with keep bits against the reference."""
    dev = device()
    G = gsmi()
    rng = np.random.default_rng(100 + n)
    mean = rng.uniform(-50.0, 50.0, (3, n)).astype(np.float32)
    lod = rng.integers(0, 8, n).astype(np.uint8)
    keepm = rng.random(n) < 0.7
    bits = oracle.pack_bits(keepm)
    cam = S.aerial_camera(1920, 1080, 20.0)
    campos = cam.position.astype(np.float32).astype(np.float64)
    d = np.linalg.norm(mean.astype(np.float64) - campos[:, None], axis=0)
    d0 = float(np.median(d))
    gate = oracle.lod_gate_level(mean.astype(np.float64), lod, campos, d0=d0, l_max=3)
    x = np.log2(d0 / d) + 0.5
    amb = np.abs(x - np.round(x)) <= 1e-5
    mean_t = torch.from_numpy(mean).to(dev)
    lod_t = torch.from_numpy(lod).to(dev)
    scene = G.scene(mean_t, None, None, None, None, lod=lod_t)
    kb = torch.from_numpy(bits.view(np.int32).copy()).to(dev)
    active = torch.empty(n, dtype=torch.int32, device=dev)
    n_act = torch.zeros(1, dtype=torch.int64, device=dev)
    ws = torch.empty(G.gs_workspace_size(G.GS_OP_LOD_MASK, n), dtype=torch.uint8, device=dev)
    for fb in (1.5, 0.0):  # never falls back; always falls back (keep bits alone)
        ref = oracle.active_set(gate, bits, fallback_ratio=fb)
        params = G.lod_params(G.GS_LOD_LEVEL, d0=d0, f=2.0, l_max=3, fallback_ratio=fb)
        G.gs_lod_mask(scene, G.camera(cam), params, kb, active, n_act, ws)
        torch.cuda.synchronize()
        m = int(n_act.item())
        got = to_np(active[:m]).astype(np.int64)
        assert (np.diff(got) > 0).all()
        sym = np.setxor1d(got, ref)
        assert amb[sym].all(), sym[~amb[sym]][:10]


def test_lod_mask_fallback_and_empty(oracle):
    dev = device()
    G = gsmi()
    from paper_2605_13794_amd.raster import DeviceScene
    sc, cam = _gate_case()
    n = sc.n
    ds = DeviceScene(sc, dev)
    active = torch.empty(n, dtype=torch.int32, device=dev)
    n_act = torch.zeros(1, dtype=torch.int64, device=dev)
    ws = torch.empty(G.gs_workspace_size(G.GS_OP_LOD_MASK, n), dtype=torch.uint8, device=dev)
    keepm = np.arange(n) % 5 != 0
    kb = torch.from_numpy(oracle.pack_bits(keepm).view(np.int32).copy()).to(dev)
    # a gate that keeps nearly everything falls back to the keep bits alone
    p = G.lod_params(G.GS_LOD_RADIUS, fallback_ratio=0.5, radius_min_px=1e-3)
    G.gs_lod_mask(ds.struct(), G.camera(cam), p, kb, active, n_act, ws)
    torch.cuda.synchronize()
    m = int(n_act.item())
    np.testing.assert_array_equal(to_np(active[:m]), np.nonzero(keepm)[0])
    # nothing kept
    zero = torch.zeros_like(kb)
    G.gs_lod_mask(ds.struct(), G.camera(cam), G.lod_params(G.GS_LOD_NONE), zero, active, n_act, ws)
    torch.cuda.synchronize()
    assert int(n_act.item()) == 0


def test_gated_projection_uses_active_list(oracle):
    """gs_project over an active list (device count, no host sync) equals the
    projection of the compacted scene."""
    dev = device()
    G = gsmi()
    from paper_2605_13794_amd.raster import DeviceScene, Frame
    sc, cam = make_case("city")
    n = sc.n
    ds = DeviceScene(sc, dev)
    keepm = np.arange(n) % 3 != 1
    kb = torch.from_numpy(oracle.pack_bits(keepm).view(np.int32).copy()).to(dev)
    active = torch.empty(n, dtype=torch.int32, device=dev)
    n_act = torch.zeros(1, dtype=torch.int64, device=dev)
    ws = torch.empty(G.gs_workspace_size(G.GS_OP_LOD_MASK, n), dtype=torch.uint8, device=dev)
    G.gs_lod_mask(ds.struct(), G.camera(cam), G.lod_params(G.GS_LOD_NONE), kb, active, n_act, ws)
    fr = Frame([cam], n, dev)
    out, K = fr.forward(ds.struct(), active=active, n_in=n, n_in_dev=n_act)
    torch.cuda.synchronize()
    sub = sc.subset(np.nonzero(keepm)[0])
    ds2 = DeviceScene(sub, dev)
    fr2 = Frame([cam], sub.n, dev)
    out2, K2 = fr2.forward(ds2.struct())
    torch.cuda.synchronize()
    assert K == K2
    assert torch.equal(out.rgb[0], out2.rgb[0])


def test_rasterize_autograd_function(oracle):
    """RasterizeFn: torch autograd through the HIP backward, two cameras, L1
    written in torch on the returned images; gradients against the float64
    pipeline summed over both views."""
    dev = device()
    gsmi()
    from paper_2605_13794_amd.raster import DeviceScene, Frame, rasterize
    sc = S.cube_scene(512, seed=4)
    cams = [S.cube_camera(64, 64, 64.0), S.look_at((1.0, -0.5, -3.8), (0, 0, 0), 64, 64, up=(0, -1, 0))]
    ds = DeviceScene(sc, dev, requires_grad=True)
    fr = Frame(cams, sc.n, dev)
    imgs = rasterize(fr, ds)
    tg = [S.target_image(64, 64, seed=10 + c) for c in range(2)]
    # upstream gradient: the reference L1 gradient masked where decisions are near a threshold
    refs = [oracle.forward_backward(sc.arrays(), c) for c in cams]
    gs = []
    for r, t in zip(refs, tg):
        _, g = oracle.l1_loss(r["rgb"], t)
        g[:, r["margin"] < 1e-3] = 0.0
        gs.append(g)
    gt = torch.from_numpy(np.stack(gs).astype(np.float32)).to(dev)
    (imgs * gt).sum().backward()
    torch.cuda.synchronize()
    tot = None
    for c, g in zip(cams, gs):
        rb = oracle.forward_backward(sc.arrays(), c, grad_img=g)["grads"]
        tot = rb if tot is None else {k: tot[k] + rb[k] for k in tot}
    for name, p in zip(("mean", "log_scale", "quat", "opacity_logit", "sh"), ds.params()):
        g = to_np(p.grad)
        e = np.abs(g - tot[name]).max() / np.abs(tot[name]).max()
        assert e <= 1e-3, (name, e)
