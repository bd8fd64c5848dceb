"""Pins of the CPU reference against closed forms, invariants, library routines
and brute force (no GPU needed).  Each test names what it pins."""
from __future__ import annotations

import math

import numpy as np
import pytest
import torch

from paper_2605_13794_amd import scenes as S
from tests import bruteforce as BF


def _one_gaussian(mu, log_scale, quat=(1.0, 0.0, 0.0, 0.0), logit=0.0, dc=(0.0, 0.0, 0.0)):
    sh = np.zeros((16, 3, 1), dtype=np.float32)
    sh[0, :, 0] = dc
    return dict(mean=np.array(mu, dtype=np.float64).reshape(3, 1),
                log_scale=np.array(log_scale, dtype=np.float64).reshape(3, 1),
                quat=np.array(quat, dtype=np.float64).reshape(4, 1),
                opacity_logit=np.array([logit], dtype=np.float64), sh=sh)


def _tiny_scene(n=40, seed=11, log_mu=-2.3):
    sc = S.cube_scene(n, seed=seed, log_scale_mu=log_mu, log_scale_sigma=0.4)
    return sc.arrays()


# --------------------------------------------------------------------------
# Spherical harmonics
# --------------------------------------------------------------------------
def test_sh_y00_constant(oracle):
    d = torch.nn.functional.normalize(torch.randn(50, 3, dtype=torch.float64), dim=1)
    Y = oracle.sh_basis(d)
    assert torch.allclose(Y[:, 0], torch.full((50,), 1.0 / (2.0 * math.sqrt(math.pi)),
                                              dtype=torch.float64), atol=1e-15)


def test_sh_matches_scipy_complex_harmonics(oracle):
    """Real SH = sqrt(2) Re/Im of scipy's complex Y_l^m (Condon-Shortley phase
    included in both)."""
    sp = pytest.importorskip("scipy.special")
    rng = np.random.default_rng(3)
    v = rng.standard_normal((64, 3))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    theta = np.arccos(np.clip(v[:, 2], -1, 1))
    phi = np.arctan2(v[:, 1], v[:, 0])
    Y = oracle.sh_basis(torch.from_numpy(v)).numpy()
    for l in range(4):
        for m in range(-l, l + 1):
            c = sp.sph_harm_y(l, abs(m), theta, phi)
            ref = c.real if m == 0 else math.sqrt(2.0) * (c.real if m > 0 else c.imag)
            np.testing.assert_allclose(Y[:, l * l + l + m], ref, atol=1e-12)


def test_sh_orthonormal_by_quadrature(oracle):
    """Gauss-Legendre in cos(theta) x uniform phi integrates products of
    degree <= 6 exactly: int Y_a Y_b dOmega = delta_ab."""
    xg, wg = np.polynomial.legendre.leggauss(12)
    nphi = 24
    phi = (np.arange(nphi) + 0.5) * 2 * math.pi / nphi
    Z, P = np.meshgrid(xg, phi, indexing="ij")
    Wt = np.repeat(wg[:, None], nphi, axis=1) * (2 * math.pi / nphi)
    s = np.sqrt(1 - Z * Z)
    d = np.stack([s * np.cos(P), s * np.sin(P), Z], axis=-1).reshape(-1, 3)
    Y = oracle.sh_basis(torch.from_numpy(d)).numpy()
    G = (Y * Wt.reshape(-1, 1)).T @ Y
    np.testing.assert_allclose(G, np.eye(16), atol=1e-12)


# --------------------------------------------------------------------------
# Projection
# --------------------------------------------------------------------------
def test_rotation_orthonormal(oracle):
    q = torch.nn.functional.normalize(torch.randn(100, 4, dtype=torch.float64), dim=1)
    R = oracle.quat_to_rotmat(q)
    I = torch.eye(3, dtype=torch.float64).expand(100, 3, 3)
    assert torch.allclose(R @ R.transpose(1, 2), I, atol=1e-13)
    assert torch.allclose(torch.linalg.det(R), torch.ones(100, dtype=torch.float64), atol=1e-13)


@pytest.mark.parametrize("z0,s", [(0.0, 0.25), (1.0, 0.1), (-2.0, 0.05)])
def test_isotropic_on_axis_closed_form(oracle, z0, s):
    """Centre on the optical axis, isotropic scale s at depth z:
    Sigma2D = ((f s / z)^2 + 0.3) I, conic = I / that, r = ceil(3 sqrt(that))."""
    cam = S.cube_camera(128, 128, 128.0)
    p = _one_gaussian((0.0, 0.0, z0), [math.log(s)] * 3)
    _, out, pr = oracle.project(p, cam)
    z = z0 + 4.0
    v = (128.0 * s / z) ** 2 + 0.3
    assert pr.mean2d[:, 0].tolist() == pytest.approx([64.0, 64.0], abs=1e-12)
    assert pr.conic[:, 0] == pytest.approx([1.0 / v, 0.0, 1.0 / v], rel=1e-12, abs=1e-15)
    assert int(pr.radius[0]) == math.ceil(3.0 * math.sqrt(v))
    assert float(pr.depth[0]) == pytest.approx(z, rel=1e-7)


def test_axis_aligned_anisotropic(oracle):
    """Identity rotation, scales (sx, sy, sz) facing the camera: eigenvalues
    (f sx / z)^2 + 0.3 and (f sy / z)^2 + 0.3, no cross term."""
    cam = S.cube_camera(128, 128, 100.0)
    sx, sy, sz = 0.3, 0.08, 0.5
    p = _one_gaussian((0.0, 0.0, 1.0), [math.log(sx), math.log(sy), math.log(sz)])
    _, out, pr = oracle.project(p, cam)
    a = (100.0 * sx / 5.0) ** 2 + 0.3
    c = (100.0 * sy / 5.0) ** 2 + 0.3
    assert pr.conic[:, 0] == pytest.approx([1.0 / a, 0.0, 1.0 / c], rel=1e-12, abs=1e-15)


def test_screen_covariance_matches_numeric_jacobian(oracle):
    """Off-axis Gaussians: Sigma2D - 0.3 I equals J_num Sigma J_num^T with J_num
    the central-difference Jacobian of the world-to-pixel map at the centre
    (pins the composition of the camera rotation and the EWA Jacobian)."""
    cam = S.aerial_camera(320, 180)
    rng = np.random.default_rng(5)
    n = 20
    mu = np.stack([rng.uniform(-20, 20, n), rng.uniform(-20, 20, n), rng.uniform(0, 10, n)])
    ls = rng.normal(-0.5, 0.3, (3, n))
    q = rng.standard_normal((4, n))
    p = dict(mean=mu, log_scale=ls, quat=q, opacity_logit=np.zeros(n),
             sh=np.zeros((16, 3, n)))
    _, out, pr = oracle.project(p, cam)

    def pix(x):
        c = cam.R @ x + cam.t
        return np.array([cam.fx * c[0] / c[2] + cam.cx, cam.fy * c[1] / c[2] + cam.cy])

    for i in range(n):
        if not bool(out["visible"][i]):
            continue
        c = cam.R @ mu[:, i] + cam.t
        if abs(c[0] / c[2]) > 1.3 * cam.width / 2 / cam.fx or abs(c[1] / c[2]) > 1.3 * cam.height / 2 / cam.fy:
            continue
        J = np.zeros((2, 3))
        for k in range(3):
            e = np.zeros(3)
            e[k] = 1e-4
            J[:, k] = (pix(mu[:, i] + e) - pix(mu[:, i] - e)) / 2e-4
        qn = q[:, i] / np.linalg.norm(q[:, i])
        w, x, y, z = qn
        R = np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                      [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                      [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])
        Sg = R @ np.diag(np.exp(2 * ls[:, i])) @ R.T
        S2 = J @ Sg @ J.T + 0.3 * np.eye(2)
        inv = np.linalg.inv(S2)
        np.testing.assert_allclose(pr.conic[:, i], [inv[0, 0], inv[0, 1], inv[1, 1]], rtol=1e-6)
        np.testing.assert_allclose(pr.mean2d[:, i], pix(mu[:, i]), rtol=1e-12)


def test_behind_camera_culled(oracle):
    cam = S.cube_camera()
    p = _one_gaussian((0.0, 0.0, -4.1), [math.log(0.1)] * 3)
    _, out, pr = oracle.project(p, cam)
    assert int(pr.radius[0]) == 0 and int(out["tiles_touched"][0]) == 0


def test_dc_colour_view_independent(oracle):
    """Only the degree-0 coefficient set: colour = Y00 * c + 0.5 for every view."""
    dc = (0.3, -0.2, -3.0)
    p = _one_gaussian((0.2, -0.1, 0.3), [math.log(0.1)] * 3, dc=dc)
    y00 = 1.0 / (2.0 * math.sqrt(math.pi))
    for cam in (S.cube_camera(), S.look_at((3.0, 2.0, -5.0), (0, 0, 0), 64, 64, up=(0, 1, 0))):
        _, out, pr = oracle.project(p, cam)
        expect = [max(0.0, y00 * c + 0.5) for c in dc]
        np.testing.assert_allclose(pr.rgb[:, 0], expect, atol=1e-12)
        assert out["clamp_bits"][0].tolist() == [False, False, True]


def test_golden_single_gaussian(oracle):
    """Hand-derived single-Gaussian case, tests/golden/single_gaussian.txt."""
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "single_gaussian.txt")
    g = {}
    for line in open(path):
        line = line.split("#", 1)[0].strip()
        if line:
            k, v = line.split("=")
            g[k.strip()] = [float(x) for x in v.split()]
    cam = S.cube_camera(128, 128, 128.0)
    p = _one_gaussian((0.0, 0.0, 0.0), [math.log(0.25)] * 3, logit=0.0, dc=(1.0, 0.0, -0.5))
    r = oracle.forward_backward(p, cam)
    pr = r["projected"]
    assert pr.conic[:, 0] == pytest.approx(g["conic"], rel=1e-12, abs=1e-15)
    assert int(pr.radius[0]) == int(g["radius"][0])
    assert r["K"] == int(g["pairs"][0])
    assert pr.rgb[:, 0] == pytest.approx(g["rgb"], rel=1e-12)
    assert r["rgb"][:, 64, 64] == pytest.approx(g["pixel_64_64"], rel=1e-12)
    assert r["T"][64, 64] == pytest.approx(g["T_64_64"][0], rel=1e-12)
    assert r["rgb"][:, 64, 100] == pytest.approx(g["pixel_64_100"], rel=1e-10)


def _golden(name):
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", name)
    g = {}
    for line in open(path):
        line = line.split("#", 1)[0].strip()
        if line:
            k, v = line.split("=")
            g[k.strip()] = [float(x) for x in v.split()]
    return g


def test_golden_tile_rect_edge(oracle):
    """Hand-derived support-rule case, tests/golden/tile_rect_edge.txt: the
    pixel just across the edge of the Gaussian's tile rectangle keeps the
    background although its alpha passes 1/255."""
    g = _golden("tile_rect_edge.txt")
    cam = S.camera_from_rt(128, 128, 128.0, 128.0, np.eye(3), np.array([0.0, 0.0, 4.0]), cx=70.5, cy=64.0)
    p = _one_gaussian((0.0, 0.0, 0.0), [math.log(0.25)] * 3, logit=math.log(9.0))
    p["sh"] = np.zeros((16, 3, 1), dtype=np.float64)
    p["sh"][0, :, 0] = (0.8, 0.2, -0.3)
    r = oracle.forward_backward(p, cam)
    pr = r["projected"]
    assert pr.mean2d[:, 0] == pytest.approx([70.5, 64.0], abs=1e-12)
    assert int(pr.radius[0]) == int(g["radius"][0])
    assert r["K"] == int(g["pairs"][0])
    assert pr.rgb[:, 0] == pytest.approx(g["rgb"], rel=1e-12)
    assert r["rgb"][:, 64, 95] == pytest.approx(g["pixel_64_95"], rel=1e-9)
    assert r["T"][64, 95] == pytest.approx(g["T_64_95"][0], rel=1e-12)
    assert g["alpha_64_96"][0] > 1.0 / 255.0
    assert r["rgb"][:, 64, 96].tolist() == g["pixel_64_96"]
    assert r["T"][64, 96] == g["T_64_96"][0]
    assert int(r["last"][64, 96]) == 0


# --------------------------------------------------------------------------
# Binning
# --------------------------------------------------------------------------
@pytest.mark.parametrize("w,h", [(48, 40), (33, 17), (16, 16)])
def test_binning_matches_python_sorted(oracle, w, h):
    cam = S.cube_camera(w, h, float(w))
    _, out, pr = oracle.project(_tiny_scene(60, seed=w + h), cam)
    K, keys, vals, ranges = oracle.bin_sort(pr, w, h)
    emitted, ordered = BF.pairs(pr, w, h)
    assert K == len(emitted)
    # the projection's per-Gaussian tile counts agree with the emitted pairs
    assert int(out["tiles_touched"].sum()) == K
    assert keys.tolist() == [k for k, _ in ordered]
    assert vals.tolist() == [v for _, v in ordered]
    nt = oracle.n_tiles(w, h)
    for t in range(nt):
        idx = [k for k, (key, _) in enumerate(ordered) if key >> 32 == t]
        if idx:
            assert (ranges[0, t], ranges[1, t]) == (idx[0], idx[-1] + 1)
        else:
            assert ranges[0, t] == ranges[1, t]


def test_binning_covers_radius_box(oracle):
    """Every pixel whose sample point is within r of the mean along x and y
    falls in an emitted tile of that Gaussian."""
    w, h = 70, 45
    cam = S.cube_camera(w, h, 70.0)
    _, _, pr = oracle.project(_tiny_scene(50, seed=9), cam)
    K, keys, vals, ranges = oracle.bin_sort(pr, w, h)
    TX = -(-w // 16)
    tiles = {}
    for key, v in zip(keys.tolist(), vals.tolist()):
        tiles.setdefault(v, set()).add(key >> 32)
    for i in range(pr.n):
        r = int(pr.radius[i])
        if r <= 0:
            continue
        for v in range(h):
            for u in range(w):
                if abs(u + 0.5 - pr.mean2d[0, i]) <= r and abs(v + 0.5 - pr.mean2d[1, i]) <= r:
                    assert (v // 16) * TX + u // 16 in tiles[i]


# --------------------------------------------------------------------------
# Compositing
# --------------------------------------------------------------------------
def test_single_gaussian_closed_form(oracle):
    """One Gaussian: C(p) = alpha(p) c with alpha = min(0.99, o exp(power)) where
    alpha >= 1/255 and the pixel's tile is covered, else 0; T = 1 - alpha."""
    cam = S.cube_camera(64, 64, 64.0)
    p = _one_gaussian((0.1, -0.05, 0.0), [math.log(0.3), math.log(0.15), math.log(0.2)],
                      quat=(0.9, 0.2, 0.1, 0.3), logit=3.0, dc=(0.5, 0.1, -0.4))
    r = oracle.forward_backward(p, cam)
    pr = r["projected"]
    x0, x1, y0, y1 = BF.rect(pr.mean2d[0, 0], pr.mean2d[1, 0], int(pr.radius[0]), 64, 64)
    ca, cb, cc = pr.conic[:, 0]
    o = pr.opacity[0]
    for v in range(64):
        for u in range(64):
            dx = pr.mean2d[0, 0] - (u + 0.5)
            dy = pr.mean2d[1, 0] - (v + 0.5)
            al = min(0.99, o * math.exp(-0.5 * (ca * dx * dx + cc * dy * dy) - cb * dx * dy))
            inside = x0 <= u // 16 < x1 and y0 <= v // 16 < y1
            if not inside or al < 1 / 255:
                al = 0.0
            np.testing.assert_allclose(r["rgb"][:, v, u], al * pr.rgb[:, 0], rtol=1e-13, atol=1e-15)
            assert r["T"][v, u] == pytest.approx(1 - al, rel=1e-13)
    assert (r["rgb"][:, :, :] > 0).any() and (r["T"] > 0.0099).all()


def test_partition_of_unity(oracle):
    """sum_i alpha_i T_i + T_final = 1: white Gaussians on a white background
    give an all-ones image; T is monotone and never below 1e-4."""
    cam = S.cube_camera(48, 40, 48.0)
    _, _, pr = oracle.project(_tiny_scene(120, seed=2, log_mu=-2.0), cam)
    pr.rgb[:] = 1.0
    K, keys, vals, ranges = oracle.bin_sort(pr, 48, 40)
    f = oracle.render_fwd(pr, vals, ranges, 48, 40, bg=(1.0, 1.0, 1.0))
    np.testing.assert_allclose(f["rgb"], 1.0, atol=1e-13)
    assert f["T"].min() >= 1e-4
    assert (f["stop"] < np.diff(ranges, axis=0).max() + 1).all()


def test_opaque_stack_stops_at_transmittance_floor(oracle):
    """Five wide, nearly opaque Gaussians on the optical axis at distinct
    depths: alpha clamps to 0.99 at the centre pixel, so T falls 1 -> 0.01 ->
    1e-4 and the third would take it to 1e-6 < 1e-4, so the pixel stops before
    compositing it: C = 0.99 c_0 + 0.99 * 0.01 c_1 + T bg, T_final = 0.01^2."""
    cam = S.cube_camera(128, 128, 128.0)
    n = 5
    dcs = [(1.0, 0.0, -1.0), (-1.0, 1.0, 0.0), (0.0, -1.0, 1.0), (0.5, 0.5, 0.5), (-0.5, 0.0, 0.5)]
    sh = np.zeros((16, 3, n))
    for i, dc in enumerate(dcs):
        sh[0, :, i] = dc
    p = dict(mean=np.stack([np.zeros(n), np.zeros(n), 0.2 * np.arange(n)]), log_scale=np.full((3, n), math.log(0.8)),
             quat=np.tile(np.array([[1.0], [0.0], [0.0], [0.0]]), (1, n)), opacity_logit=np.full(n, 10.0), sh=sh)
    bg = (0.2, 0.4, 0.6)
    r = oracle.forward_backward(p, cam, bg=bg)
    pr = r["projected"]
    g = pr.opacity * np.exp(-0.5 * (pr.conic[0] * 0.25 + pr.conic[2] * 0.25) - pr.conic[1] * 0.25)
    assert (g > 0.99).all()                      # every alpha at pixel (64, 64) clamps
    a = 0.99
    T1 = 1.0 * (1.0 - a)
    T2 = T1 * (1.0 - a)
    assert r["T"][64, 64] == pytest.approx(T2, rel=1e-12)
    expect = a * pr.rgb[:, 0] + a * T1 * pr.rgb[:, 1] + T2 * np.array(bg)
    np.testing.assert_allclose(r["rgb"][:, 64, 64], expect, rtol=1e-12)


def test_matches_bruteforce_depth_order(oracle):
    """Tile lists + sorted keys give the same image as sorting every pixel's
    candidates by depth with Python's sorted()."""
    w, h = 40, 36
    cam = S.cube_camera(w, h, 40.0)
    _, _, pr = oracle.project(_tiny_scene(50, seed=4), cam)
    K, keys, vals, ranges = oracle.bin_sort(pr, w, h)
    f = oracle.render_fwd(pr, vals, ranges, w, h, bg=(0.1, 0.2, 0.3))
    img, T, wimp, aimp = BF.render(pr, w, h, bg=(0.1, 0.2, 0.3))
    np.testing.assert_allclose(f["rgb"], img, atol=1e-13)
    np.testing.assert_allclose(f["T"], T, atol=1e-15)
    w2, a2 = oracle.importance_blend(pr, vals, ranges, w, h)
    np.testing.assert_allclose(w2, wimp, atol=1e-13)
    np.testing.assert_array_equal(a2, aimp)


def test_permutation_invariance(oracle):
    w, h = 48, 32
    cam = S.cube_camera(w, h, 48.0)
    p = _tiny_scene(80, seed=8)
    r1 = oracle.forward_backward(p, cam)
    perm = np.random.default_rng(0).permutation(80)
    p2 = {k: (v[..., perm] if k != "lod" else v) for k, v in p.items()}
    r2 = oracle.forward_backward(p2, cam)
    assert len(set(r1["projected"].depth.tolist())) == 80
    np.testing.assert_allclose(r1["rgb"], r2["rgb"], atol=1e-13)


def test_integral_of_wide_gaussian(oracle):
    """sum_p alpha(p) for a wide Gaussian of small opacity equals
    o * 2 pi sqrt(det Sigma2D) * (1 - exp(-R^2/2)) with R^2/2 = ln(255 o), the
    mass inside the 1/255 cut (pixel sum vs integral, loose tolerance)."""
    cam = S.cube_camera(256, 256, 256.0)
    logit = math.log(0.2 / 0.8)
    p = _one_gaussian((0.0, 0.0, 0.0), [math.log(0.2), math.log(0.12), math.log(0.1)],
                      quat=(0.8, 0.0, 0.3, 0.5), logit=logit, dc=(1 / 0.28209479177387814 * 0.5, 0, 0))
    r = oracle.forward_backward(p, cam)
    pr = r["projected"]
    det_inv = pr.conic[0, 0] * pr.conic[2, 0] - pr.conic[1, 0] ** 2
    o = 0.2
    expect = o * 2 * math.pi / math.sqrt(det_inv) * (1 - 1 / (255 * o))
    assert r["rgb"][0].sum() == pytest.approx(expect, rel=2e-3)


# --------------------------------------------------------------------------
# Gradients (central finite differences of the float64 pipeline)
# --------------------------------------------------------------------------
def _clamped_evaluations(pr, w, h):
    """(Gaussian, pixel) pairs inside the Gaussian's tile rectangle where
    o G exceeds 0.99 (alpha clamped), counted by brute force."""
    u = np.arange(w) + 0.5
    v = np.arange(h) + 0.5
    count = 0
    for i in np.nonzero(pr.radius > 0)[0]:
        x0, x1, y0, y1 = BF.rect(pr.mean2d[0, i], pr.mean2d[1, i], int(pr.radius[i]), w, h)
        dx = pr.mean2d[0, i] - u[None, 16 * x0:16 * x1]
        dy = pr.mean2d[1, i] - v[16 * y0:16 * y1, None]
        a, b, c = pr.conic[:, i]
        power = -0.5 * (a * dx * dx + c * dy * dy) - b * dx * dy
        count += int((pr.opacity[i] * np.exp(np.minimum(power, 0.0)) > 0.99).sum())
    return count


def _signature(oracle, p, cam, target, bg):
    r = oracle.forward_backward(p, cam, bg=bg)
    sig = (r["sig"].tobytes(), r["projected"].radius.tobytes(),
           r["out"]["rect"].numpy().tobytes(), r["out"]["clamp_bits"].numpy().tobytes())
    return oracle.l1_loss(r["rgb"], target)[0], sig


@pytest.mark.parametrize("bg,logit_shift,log_mu", [((0.0, 0.0, 0.0), 0.0, -1.8), ((0.3, 0.6, 0.9), 0.0, -1.8),
                                                    ((0.3, 0.6, 0.9), 7.0, -0.6)])
def test_gradients_match_finite_differences(oracle, bg, logit_shift, log_mu):
    """Every parameter group against central differences of the loss, on a
    black and on a coloured background (the background enters dC/dalpha), and
    with opacities high enough that alpha = min(0.99, o G) clamps on many
    pixels (zero derivative there)."""
    w, h = 32, 32
    cam = S.cube_camera(w, h, 32.0)
    sc = S.cube_scene(24, seed=4, log_scale_mu=log_mu, log_scale_sigma=0.3)
    p = {k: v.astype(np.float64) for k, v in sc.arrays().items() if k != "lod"}
    p["opacity_logit"] = p["opacity_logit"] + logit_shift
    target = S.target_image(w, h, seed=4)
    r = oracle.forward_backward(p, cam, target=target, bg=bg)
    if logit_shift > 0:
        pr = r["projected"]
        assert _clamped_evaluations(pr, w, h) > 20
    grads = r["grads"]
    vis = np.nonzero(r["projected"].radius > 0)[0]
    rng = np.random.default_rng(1)
    checked = 0
    for name, arr in p.items():
        for _ in range(14):
            i = int(rng.choice(vis))
            comp = tuple(int(rng.integers(0, s)) for s in arr.shape[:-1])
            idx = comp + (i,)
            x = arr[idx]
            hstep = 1e-6 * max(1.0, abs(x))
            pp = {k: v.copy() for k, v in p.items()}
            pm = {k: v.copy() for k, v in p.items()}
            pp[name][idx] = x + hstep
            pm[name][idx] = x - hstep
            lp, sp = _signature(oracle, pp, cam, target, bg)
            lm, sm = _signature(oracle, pm, cam, target, bg)
            if sp != sm:
                continue
            fd = (lp - lm) / (2 * hstep)
            an = grads[name][idx]
            scale = np.abs(grads[name]).max()
            assert abs(fd - an) <= 1e-6 * scale + 1e-9, (name, idx, fd, an)
            checked += 1
    assert checked >= 50


# --------------------------------------------------------------------------
# Importance aggregation
# --------------------------------------------------------------------------
def test_importance_sum_identity(oracle):
    """sum_i w_{i,v} = sum_p (1 - T_final(p))."""
    w_, h_ = 64, 48
    cam = S.cube_camera(w_, h_, 64.0)
    _, _, pr = oracle.project(_tiny_scene(300, seed=3), cam)
    K, keys, vals, ranges = oracle.bin_sort(pr, w_, h_)
    f = oracle.render_fwd(pr, vals, ranges, w_, h_)
    w, a = oracle.importance_blend(pr, vals, ranges, w_, h_)
    assert w.sum() == pytest.approx((1 - f["T"]).sum(), rel=1e-12)
    assert (a[pr.radius == 0] == 0).all()


def _footprint_brute(pr, i, width, height):
    """Pixels of Gaussian i's tile rectangle (the tiles it is listed in, inside
    the image) whose kernel value passes the 1/255 test, counted pixel by
    pixel from the definition: what the footprint reading of a_{i,v} counts,
    and what the composited count is when nothing else is drawn."""
    if pr.radius[i] <= 0:
        return 0
    TX, TY = -(-width // 16), -(-height // 16)
    r = int(pr.radius[i])
    xi, yi = math.floor(pr.mean2d[0, i]), math.floor(pr.mean2d[1, i])
    tx0, tx1 = min(max((xi - r) // 16, 0), TX), min(max((xi + r) // 16 + 1, 0), TX)
    ty0, ty1 = min(max((yi - r) // 16, 0), TY), min(max((yi + r) // 16 + 1, 0), TY)
    a, b, c = pr.conic[0, i], pr.conic[1, i], pr.conic[2, i]
    count = 0
    for v in range(ty0 * 16, min(ty1 * 16, height)):
        for u in range(tx0 * 16, min(tx1 * 16, width)):
            dx, dy = pr.mean2d[0, i] - (u + 0.5), pr.mean2d[1, i] - (v + 0.5)
            power = -0.5 * (a * dx * dx + c * dy * dy) - b * dx * dy
            if power > 0:
                continue
            if min(0.99, pr.opacity[i] * math.exp(power)) >= 1.0 / 255.0:
                count += 1
    return count


def test_importance_footprint_count_ignores_occlusion(oracle):
    """Footprint reading of a_{i,v}: the count of every Gaussian equals its
    count when drawn alone (occluders and stopped pixels do not change it),
    computed pixel by pixel; the composited count is never larger, and is
    smaller where an opaque stack stops pixels early."""
    w_, h_ = 48, 40
    cam = S.cube_camera(w_, h_, 48.0)
    scn = _tiny_scene(120, seed=5, log_mu=-1.8)
    scn["opacity_logit"] = scn["opacity_logit"] + 4.0        # nearly opaque: pixels stop
    _, _, pr = oracle.project(scn, cam)
    K, keys, vals, ranges = oracle.bin_sort(pr, w_, h_)
    w_c, a_c = oracle.importance_blend(pr, vals, ranges, w_, h_)
    w_f, a_f = oracle.importance_blend(pr, vals, ranges, w_, h_, footprint=True)
    want = np.array([_footprint_brute(pr, i, w_, h_) for i in range(pr.n)])
    np.testing.assert_array_equal(a_f, want)
    np.testing.assert_array_equal(w_f, w_c)                  # w is the same either way
    assert (a_c <= a_f).all() and (a_c < a_f).any()


def test_top_mass_hand_cases(oracle):
    # W = 100, 0.99 W = 99: prefix 50, 30, 10, 9.5 reaches 99.5 (crossing included)
    w = np.array([10.0, 0.5, 30.0, 9.5, 50.0, 0.0])
    assert oracle.top_mass(w).tolist() == [True, False, True, True, True, False]
    # ties broken by ascending index
    w = np.array([1.0, 1.0, 1.0, 1.0])
    assert oracle.top_mass(w, 0.5).tolist() == [True, True, False, False]
    assert not oracle.top_mass(np.zeros(5)).any()


def test_top_mass_minimal_prefix_bruteforce(oracle):
    rng = np.random.default_rng(7)
    for _ in range(50):
        n = int(rng.integers(1, 30))
        w = rng.exponential(1.0, n) * (rng.random(n) < 0.8)
        sel = oracle.top_mass(w, 0.9)
        if w.sum() == 0:
            assert not sel.any()
            continue
        assert w[sel].sum() >= 0.9 * w.sum() - 1e-12
        # minimal: every selected weight >= every unselected one, and dropping
        # the smallest selected falls below the target
        if (~sel).any():
            assert w[sel].min() >= w[~sel].max()
        assert w[sel].sum() - w[sel].min() < 0.9 * w.sum()


def test_importance_fold_and_phi(oracle):
    st = oracle.ImportanceState(5, 2)
    w = np.array([4.0, 0.0, 1.0, 0.01, 2.0])
    a = np.array([2, 0, 1, 1, 4])
    radius = np.array([3, 2, 0, 5, 4])
    oracle.importance_fold(st, 0, w, a, radius, frac=0.99)
    np.testing.assert_allclose(st.score, [4 / (2 + 1e-6), 0, 1 / (1 + 1e-6), 0.01 / (1 + 1e-6),
                                          2 / (4 + 1e-6)])
    assert st.c_rad.tolist() == [1, 1, 0, 1, 1]
    assert st.c_vis.tolist() == [1, 0, 1, 0, 1]   # 4+2+1 = 7 >= 0.99 * 7.01
    assert oracle.unpack_bits(st.cull[0], 5).tolist() == [False, True, False, True, False]
    np.testing.assert_allclose(st.phi(), [1 / (1 + 1e-6), 0, 1 / 1e-6, 0, 1 / (1 + 1e-6)])


# --------------------------------------------------------------------------
# View-level gate, active set, score mask
# --------------------------------------------------------------------------
def test_lod_level_equation_values(oracle):
    """Eq. 1 with d0 = 100, f = 2: d = 100 -> 0, 50 -> 1, 25 -> 2, 200 -> 0 (clamped),
    100/2^1.5 -> round-half-up 2; L_max = 2 caps d = 10 at 2."""
    d = np.array([100.0, 50.0, 25.0, 200.0, 100 / 2 ** 1.5, 10.0])
    mean = np.stack([d, np.zeros(6), np.zeros(6)])
    for lvl, expect in [(0, [1, 1, 1, 1, 1, 1]), (1, [0, 1, 1, 0, 1, 1]), (2, [0, 0, 1, 0, 1, 1]),
                        (3, [0, 0, 0, 0, 0, 0])]:
        keep = oracle.lod_gate_level(mean, np.full(6, lvl), np.zeros(3), d0=100.0, l_max=2)
        assert keep.astype(int).tolist() == expect


def test_lod_radius_gate_boundary_values(oracle):
    """Radius gate r = k fx max_j s_j / d at hand-chosen values: fx = 50 and
    s = 1 (log-scale 0) at d = 100 (a 60-80-0 offset) give r = 0.5 px
    exactly, kept; d one part in 1e9 farther gives r below 0.5, dropped; the
    largest of the three axes decides (the third axis here); k = 3 triples
    r; a Gaussian at the camera centre has infinite r and is kept."""
    cam_pos = np.array([10.0, -20.0, 5.0])
    off = np.array([[60.0, 80.0, 0.0], [60.0 * (1 + 1e-9), 80.0 * (1 + 1e-9), 0.0], [0.0, 0.0, 100.0],
                    [0.0, 0.0, 0.0], [0.0, 0.0, 300.0], [0.0, 0.0, 301.0]])
    mean = (cam_pos[None, :] + off).T
    log_scale = np.array([[0.0, -1.0, -2.0], [0.0, 0.0, 0.0], [-3.0, -2.0, 0.0], [-5.0, -5.0, -5.0],
                          [0.0, -1.0, -1.0], [0.0, -1.0, -1.0]]).T
    keep, r = oracle.lod_gate_radius(mean, log_scale, cam_pos, fx=50.0, r_min=0.5)
    assert r[0] == 0.5 and r[2] == 0.5
    assert r[1] < 0.5
    assert keep.tolist() == [True, False, True, True, False, False]
    keep3, r3 = oracle.lod_gate_radius(mean, log_scale, cam_pos, fx=50.0, r_min=0.5, k_sigma=3.0)
    assert r3[4] == 0.5 and r3[5] < 0.5
    assert keep3.tolist() == [True, True, True, True, True, False]


def test_gates_bruteforce_and_compaction(oracle):
    sc = S.city_scene(3000, seed=12)
    cam_pos = np.array([10.0, -200.0, 150.0])
    keep_r, r = oracle.lod_gate_radius(sc.mean, sc.log_scale, cam_pos, fx=1662.8, r_min=0.5)
    for i in range(0, 3000, 37):
        d = math.dist(sc.mean[:, i].astype(float), cam_pos)
        rr = 1662.8 * math.exp(float(sc.log_scale[:, i].astype(float).max())) / d
        assert keep_r[i] == (rr >= 0.5)
    keep_l = oracle.lod_gate_level(sc.mean, sc.lod, cam_pos, d0=300.0, l_max=7)
    for i in range(0, 3000, 41):
        d = math.dist(sc.mean[:, i].astype(float), cam_pos)
        L = min(7, max(0, math.floor(math.log2(300.0 / d) + 0.5)))
        assert keep_l[i] == (sc.lod[i] <= L)
    bits = oracle.pack_bits(np.arange(3000) % 3 != 0)
    act = oracle.active_set(keep_r, bits, fallback_ratio=2.0)   # ratio > 1: never skip
    assert 0 < keep_r.sum() < 3000
    np.testing.assert_array_equal(act, np.nonzero(keep_r & (np.arange(3000) % 3 != 0))[0])
    # fallback: a gate keeping >= the ratio is skipped
    act2 = oracle.active_set(np.ones(3000, dtype=bool) & (np.arange(3000) != 5), None, 0.95)
    assert act2.size == 3000


def test_bits_roundtrip(oracle):
    m = np.random.default_rng(0).random(77) < 0.5
    assert (oracle.unpack_bits(oracle.pack_bits(m), 77) == m).all()
    assert oracle.pack_bits(np.array([1, 0, 0, 0, 0, 1], dtype=bool)).tolist() == [33]


def test_score_keep_ties_and_count(oracle):
    s = np.array([0.5, 0.0, 0.2, 0.0, 0.2, 0.9, 0.1])
    n_drop = oracle.drop_count(7, 0.4)
    assert n_drop == 3                      # ceil(2.8)
    assert oracle.score_keep(s, n_drop).tolist() == [True, False, True, False, True, True, False]
    # the tie at 0.2 is broken by index: index 2 goes before index 4
    assert oracle.score_keep(s, 4).tolist() == [True, False, False, False, True, True, False]


# --------------------------------------------------------------------------
# Loss and optimizer
# --------------------------------------------------------------------------
def test_l1_loss_closed_form(oracle):
    img = np.array([[[0.5, 1.0]], [[0.0, 0.25]], [[1.0, 1.0]]])
    tgt = np.array([[[0.25, 1.0]], [[0.5, 0.0]], [[0.0, 1.0]]])
    L, g = oracle.l1_loss(img, tgt)
    assert L == pytest.approx((0.25 + 0 + 0.5 + 0.25 + 1.0 + 0) / 6)
    np.testing.assert_array_equal(g * 6, [[[1, 0]], [[-1, 1]], [[1, 0]]])


def test_adam_first_step_and_torch(oracle):
    rng = np.random.default_rng(2)
    p0 = rng.standard_normal(20)
    g = rng.standard_normal(20)
    p1, m, v = oracle.adam_step(p0, g, np.zeros(20), np.zeros(20), lr=0.01, step=1, eps=0.0)
    np.testing.assert_allclose(p1, p0 - 0.01 * np.sign(g), atol=1e-15)
    # several steps against torch.optim.Adam in float64
    x = torch.tensor(p0, dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([x], lr=0.003, betas=(0.9, 0.999), eps=1e-15)
    p, m, v = p0.copy(), np.zeros(20), np.zeros(20)
    for step in range(1, 6):
        gs = rng.standard_normal(20)
        x.grad = torch.tensor(gs)
        opt.step()
        p, m, v = oracle.adam_step(p, gs, m, v, lr=0.003, step=step)
    np.testing.assert_allclose(p, x.detach().numpy(), rtol=1e-13, atol=1e-15)
