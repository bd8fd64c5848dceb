"""CPU reference of the rasterizer hot path, in float64 (test infrastructure).

This package is the checker, not the product: only `tests/`, the smoke check
and the CPU-baseline leg of the benchmark import it.  It shares no code with the
HIP path.

Parts and the passages they follow:
  project.py   per-Gaussian projection + SH colour (Appendix A, Eq. `gaussian`);
               derivatives by torch autograd in float64.
  raster.c     tile binning, front-to-back compositing (Appendix A, Eq.
               `alpha_compositing`), its backward with the stored float64
               transmittance chain, and the colour-less instrumented blend of
               the importance sweep (Sec. 3.2, Fig. 3).
  levels.py    LOD labels from multi-resolution voxelisation, the L_max(t)
               schedule, the clone/split level inheritance and the spawn
               gate's rank veto (Sec. 3.3; Sec. 3.2 and Appendix E).
  this file    loss, importance aggregation (s_i, c^rad, c^vis, Cull; Sec. 3.2),
               the view-level LOD gate and active set (Sec. 3.3, Eqs. 1-3),
               the score mask, Adam, and the end-to-end pipeline.

Readings where the paper is silent are documented at each function.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np
import torch

from . import project as _proj
from .project import TILE, sh_basis, quat_to_rotmat  # noqa: F401

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libgso.so")
_lib = None

ALPHA_MIN = 1.0 / 255.0
ALPHA_MAX = 0.99
T_MIN = 1e-4


def build(force: bool = False) -> str:
    """Compile raster.c with gcc (IEEE float64, no FMA contraction)."""
    src = os.path.join(_HERE, "raster.c")
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(src):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
                               "-fno-fast-math", src, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        L = ctypes.CDLL(_LIB_PATH)
        P = ctypes.c_void_p
        i64, i32 = ctypes.c_int64, ctypes.c_int32
        L.gso_bin_sort.restype = i64
        L.gso_bin_sort.argtypes = [i64, P, P, P, i32, i32, P, P, i64, P]
        L.gso_render_fwd.restype = None
        L.gso_render_fwd.argtypes = [i32, i32, i64, P, P, P, P, P, P, P, P, P, P, P, P, P]
        L.gso_render_bwd.restype = None
        L.gso_render_bwd.argtypes = [i32, i32, i64, P, P, P, P, P, P, P, P, P, P, P, P]
        L.gso_importance_blend.restype = None
        L.gso_importance_blend.argtypes = [i32, i32, i64, P, P, P, P, P, P, P, i32]
        L.gso_num_threads.restype = ctypes.c_int
        L.gso_num_threads.argtypes = []
        _lib = L
    return _lib


def _p(a: np.ndarray):
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.c_void_p)


def num_threads() -> int:
    """Threads the compiled compositing loops use (OpenMP)."""
    return int(lib().gso_num_threads())


def n_tiles(width: int, height: int) -> int:
    return ((width + TILE - 1) // TILE) * ((height + TILE - 1) // TILE)


# --------------------------------------------------------------------------
# Projected record in the layouts the C part takes
# --------------------------------------------------------------------------
class Projected:
    """Component-major float64 copies of a projection (plus float32 depth)."""

    def __init__(self, mean2d, depth, conic, opacity, rgb, radius):
        self.mean2d = np.ascontiguousarray(mean2d, dtype=np.float64)      # [2][n]
        self.depth = np.ascontiguousarray(depth, dtype=np.float32)        # [n]
        self.conic = np.ascontiguousarray(conic, dtype=np.float64)        # [3][n]
        self.opacity = np.ascontiguousarray(opacity, dtype=np.float64)    # [n]
        self.rgb = np.ascontiguousarray(rgb, dtype=np.float64)            # [3][n]
        self.radius = np.ascontiguousarray(radius, dtype=np.int32)        # [n]

    @property
    def n(self):
        return self.depth.shape[0]

    @staticmethod
    def from_projection(out) -> "Projected":
        d = lambda t: t.detach().cpu().numpy()  # noqa: E731
        vis = d(out["visible"])
        z = lambda a: np.where(vis, a, 0.0)  # noqa: E731
        return Projected(mean2d=z(d(out["mean2d"]).T), depth=z(d(out["depth"])).astype(np.float32),
                         conic=z(d(out["conic"]).T), opacity=z(d(out["opacity"])),
                         rgb=z(d(out["rgb"]).T), radius=d(out["radius"]))

    def rounded_f32(self) -> "Projected":
        """The same record rounded to float32 (what a float32 device holds)."""
        f = lambda a: a.astype(np.float32).astype(np.float64)  # noqa: E731
        return Projected(f(self.mean2d), self.depth, f(self.conic), f(self.opacity), f(self.rgb),
                         self.radius)


def project(scene_arrays: dict, cam, requires_grad: bool = False):
    """Projection (see project.py).  Returns (leaves, torch outputs, Projected)."""
    leaves, out = _proj.project(scene_arrays, cam, requires_grad=requires_grad)
    return leaves, out, Projected.from_projection(out)


# --------------------------------------------------------------------------
# Binning and compositing (C)
# --------------------------------------------------------------------------
def bin_sort(pr: Projected, width: int, height: int, capacity: int | None = None):
    """Keys (tile<<32 | float32 depth bits), values (Gaussian index) sorted
    stably by key, and per-tile [start, end) ranges ([2][n_tiles])."""
    nt = n_tiles(width, height)
    ranges = np.zeros(2 * nt, dtype=np.uint32)
    K = lib().gso_bin_sort(pr.n, _p(pr.mean2d), _p(pr.radius), _p(pr.depth), width, height,
                           None, None, 0, _p(ranges))
    cap = K if capacity is None else capacity
    keys = np.zeros(max(cap, 1), dtype=np.uint64)
    vals = np.zeros(max(cap, 1), dtype=np.uint32)
    K2 = lib().gso_bin_sort(pr.n, _p(pr.mean2d), _p(pr.radius), _p(pr.depth), width, height,
                            _p(keys), _p(vals), cap, _p(ranges))
    assert K2 == K
    return int(K), keys[:K], vals[:K], ranges.reshape(2, nt)


def render_fwd(pr: Projected, vals, ranges, width, height, bg=(0.0, 0.0, 0.0)):
    """Returns dict(rgb [3][H][W], T [H][W], last [H][W] uint32,
    stop [H][W] int64 (1-based position where the pixel stopped, or the list
    length), margin [H][W] (smallest relative gap of a threshold test),
    sig [H][W] (hash of the discrete decisions taken))."""
    npx = width * height
    rgb = np.zeros(3 * npx)
    T = np.zeros(npx)
    last = np.zeros(npx, dtype=np.uint32)
    stop = np.zeros(npx, dtype=np.int64)
    margin = np.zeros(npx)
    sig = np.zeros(npx, dtype=np.uint64)
    bgv = np.ascontiguousarray(bg, dtype=np.float64)
    vals = np.ascontiguousarray(vals, dtype=np.uint32)
    ranges = np.ascontiguousarray(ranges, dtype=np.uint32).reshape(-1)
    if vals.size == 0:
        vals = np.zeros(1, dtype=np.uint32)
    lib().gso_render_fwd(width, height, pr.n, _p(pr.mean2d), _p(pr.conic), _p(pr.opacity),
                         _p(pr.rgb), _p(vals), _p(ranges), _p(bgv), _p(rgb), _p(T), _p(last),
                         _p(stop), _p(margin), _p(sig))
    return dict(rgb=rgb.reshape(3, height, width), T=T.reshape(height, width),
                last=last.reshape(height, width), stop=stop.reshape(height, width),
                margin=margin.reshape(height, width), sig=sig.reshape(height, width))


def render_bwd(pr: Projected, vals, ranges, width, height, grad_img, bg=(0.0, 0.0, 0.0)):
    """Gradients of sum(grad_img * C) with respect to mean2d [2][n],
    conic [3][n], opacity [n] and rgb [3][n]."""
    n = pr.n
    d_mean2d = np.zeros(2 * n)
    d_conic = np.zeros(3 * n)
    d_opacity = np.zeros(n)
    d_rgb = np.zeros(3 * n)
    g = np.ascontiguousarray(grad_img, dtype=np.float64).reshape(-1)
    bgv = np.ascontiguousarray(bg, dtype=np.float64)
    vals = np.ascontiguousarray(vals, dtype=np.uint32)
    ranges = np.ascontiguousarray(ranges, dtype=np.uint32).reshape(-1)
    if vals.size == 0:
        vals = np.zeros(1, dtype=np.uint32)
    lib().gso_render_bwd(width, height, n, _p(pr.mean2d), _p(pr.conic), _p(pr.opacity),
                         _p(pr.rgb), _p(vals), _p(ranges), _p(bgv), _p(g), _p(d_mean2d),
                         _p(d_conic), _p(d_opacity), _p(d_rgb))
    return dict(mean2d=d_mean2d.reshape(2, n), conic=d_conic.reshape(3, n), opacity=d_opacity,
                rgb=d_rgb.reshape(3, n))


def l1_loss(img, target):
    """L = mean |C - target| over 3*H*W values; dL/dC = sign(C - target)/(3HW)
    with sign(0) = 0 (Eq. 4 with lambda = 0, B = 1)."""
    diff = np.asarray(img, dtype=np.float64) - np.asarray(target, dtype=np.float64)
    m = diff.size
    return float(np.abs(diff).sum() / m), np.sign(diff) / m


# --------------------------------------------------------------------------
# End-to-end forward + backward
# --------------------------------------------------------------------------
def forward_backward(scene_arrays: dict, cam, target=None, bg=(0.0, 0.0, 0.0),
                     projected_override: Projected | None = None, grad_img=None):
    """Project, bin, composite; with a target also the L1 loss and the
    gradients of every parameter (mean, log_scale, quat, opacity_logit, sh).

    `projected_override` (tests only) replaces the projected record fed to
    binning and compositing, e.g. by its float32 rounding.  `grad_img`
    (tests only) replaces dL/dC, so that two implementations can be compared
    on the same upstream gradient."""
    want = target is not None or grad_img is not None
    leaves, out, pr = project(scene_arrays, cam, requires_grad=want)
    prx = projected_override if projected_override is not None else pr
    W, H = cam.width, cam.height
    K, keys, vals, ranges = bin_sort(prx, W, H)
    fwd = render_fwd(prx, vals, ranges, W, H, bg)
    res = dict(projected=pr, out=out, K=K, keys=keys, vals=vals, ranges=ranges, **fwd)
    if not want:
        return res
    if grad_img is not None:
        loss, g = float("nan"), np.asarray(grad_img, dtype=np.float64)
    else:
        loss, g = l1_loss(fwd["rgb"], target)
    d2 = render_bwd(prx, vals, ranges, W, H, g, bg)
    vis = out["visible"]
    grads_out = [torch.from_numpy(d2["mean2d"].T.copy()), torch.from_numpy(d2["conic"].T.copy()),
                 torch.from_numpy(d2["opacity"].copy()), torch.from_numpy(d2["rgb"].T.copy())]
    outs = [out["mean2d"], out["conic"], out["opacity"], out["rgb"]]
    m = vis.to(torch.float64)
    outs = [o * (m[:, None] if o.dim() == 2 else m) for o in outs]
    gr = torch.autograd.grad(outs, [leaves[k] for k in ("mean", "log_scale", "quat",
                                                          "opacity_logit", "sh")],
                             grads_out, allow_unused=True)
    names = ("mean", "log_scale", "quat", "opacity_logit", "sh")
    res.update(loss=loss, grad_img=g, grads2d=d2,
               grads={k: (torch.zeros_like(leaves[k]) if v is None else v).numpy()
                      for k, v in zip(names, gr)})
    return res


# --------------------------------------------------------------------------
# Importance sweep (Sec. 3.2, Fig. 3)
# --------------------------------------------------------------------------
def importance_blend(pr: Projected, vals, ranges, width, height, footprint: bool = False):
    """Per-view w_{i,v} = sum_p alpha_p T_p and a_{i,v} = number of pixels at
    which g_i is composited (reading: the pixels that the instrumented blend
    actually visits and composites).  footprint=True takes the other reading
    of "pixels it touches": a_{i,v} counts every pixel of g_i's tiles inside
    its footprint (kernel value passing the 1/255 test), occluded or not."""
    w = np.zeros(pr.n)
    a = np.zeros(pr.n, dtype=np.int64)
    vals = np.ascontiguousarray(vals, dtype=np.uint32)
    ranges = np.ascontiguousarray(ranges, dtype=np.uint32).reshape(-1)
    if vals.size == 0:
        vals = np.zeros(1, dtype=np.uint32)
    lib().gso_importance_blend(width, height, pr.n, _p(pr.mean2d), _p(pr.conic), _p(pr.opacity),
                               _p(vals), _p(ranges), _p(w), _p(a), 1 if footprint else 0)
    return w, a


def top_mass(w: np.ndarray, frac: float = 0.99) -> np.ndarray:
    """c^vis of one view: the Gaussians of the shortest prefix of the order
    (w descending, index ascending) whose summed w reaches frac * sum(w),
    the crossing element included.  w = 0 is never selected."""
    w = np.asarray(w, dtype=np.float64)
    sel = np.zeros(w.shape[0], dtype=bool)
    idx = np.nonzero(w > 0)[0]
    if idx.size == 0:
        return sel
    order = idx[np.lexsort((idx, -w[idx]))]
    cs = np.cumsum(w[order])
    target = frac * cs[-1]
    m = int(np.searchsorted(cs, target, side="left")) + 1
    m = min(m, order.size)
    sel[order[:m]] = True
    return sel


def pack_bits(mask: np.ndarray) -> np.ndarray:
    """Bit i of word i // 32 (least significant first), uint32 words."""
    mask = np.asarray(mask, dtype=bool)
    n = mask.shape[0]
    words = (n + 31) // 32
    padded = np.zeros(words * 32, dtype=np.uint64)
    padded[:n] = mask
    sh = np.arange(32, dtype=np.uint64)
    return (padded.reshape(words, 32) << sh).sum(axis=1).astype(np.uint32)


def unpack_bits(words: np.ndarray, n: int) -> np.ndarray:
    words = np.asarray(words, dtype=np.uint32).astype(np.uint64)
    bits = (words[:, None] >> np.arange(32, dtype=np.uint64)) & 1
    return bits.reshape(-1)[:n].astype(bool)


class ImportanceState:
    """Aggregates of one sweep: s_i, c^rad_i, c^vis_i and the view-major Cull
    bitmap [V][ceil(N/32)]."""

    def __init__(self, n: int, n_views: int):
        self.n = n
        self.score = np.zeros(n)
        self.c_rad = np.zeros(n, dtype=np.int64)
        self.c_vis = np.zeros(n, dtype=np.int64)
        self.cull = np.zeros((n_views, (n + 31) // 32), dtype=np.uint32)

    def phi(self, eps: float = 1e-6):
        return self.c_vis / (self.c_rad + eps)


def importance_fold(state: ImportanceState, view: int, w, a, radius, frac=0.99, eps=1e-6):
    """Folds one view: c^rad = [radius > 0], c^vis = top-mass membership,
    Cull = 1 - c^vis, s_i += w/(a + eps) where a > 0 (eps reading: 1e-6)."""
    crad = np.asarray(radius) > 0
    cvis = top_mass(w, frac)
    a = np.asarray(a)
    pos = a > 0
    state.score[pos] += np.asarray(w)[pos] / (a[pos] + eps)
    state.c_rad += crad
    state.c_vis += cvis
    state.cull[view] = pack_bits(~cvis)
    return crad, cvis


def importance_view(scene_arrays, cam, state: ImportanceState, view: int, frac=0.99, eps=1e-6,
                    projected_override: Projected | None = None, footprint: bool = False):
    _, _, pr = project(scene_arrays, cam)
    prx = projected_override if projected_override is not None else pr
    K, keys, vals, ranges = bin_sort(prx, cam.width, cam.height)
    w, a = importance_blend(prx, vals, ranges, cam.width, cam.height, footprint)
    crad, cvis = importance_fold(state, view, w, a, prx.radius, frac, eps)
    return dict(w=w, a=a, c_rad=crad, c_vis=cvis, K=K)


# --------------------------------------------------------------------------
# View-level filtering (Sec. 3.3, Eqs. 1-3) and the score mask
# --------------------------------------------------------------------------
def lod_gate_level(mean, lod, cam_pos, d0: float, l_max: int, f: float = 2.0):
    """Eq. 1-2: L_v(d) = clamp(round(log_f(d0/d)), 0, L_max); keep l_i <= L_v.
    Readings: round half up, floor(x + 0.5); d < 1e-6 gives L_max."""
    mean = np.asarray(mean, dtype=np.float64)
    d = np.linalg.norm(mean - np.asarray(cam_pos, dtype=np.float64)[:, None], axis=0)
    with np.errstate(divide="ignore"):
        lv = np.floor(np.log(d0 / np.maximum(d, 1e-300)) / math.log(f) + 0.5)
    lv = np.where(d < 1e-6, l_max, np.clip(lv, 0, l_max))
    return np.asarray(lod, dtype=np.int64) <= lv


def lod_gate_radius(mean, log_scale, cam_pos, fx: float, r_min: float, k_sigma: float = 1.0):
    """Projected-radius gate: r = k * fx * max_j s_ij / |mu_i - c_v|; keep r >= r_min
    (reading of "drop if projected radius < 0.5 px")."""
    mean = np.asarray(mean, dtype=np.float64)
    d = np.linalg.norm(mean - np.asarray(cam_pos, dtype=np.float64)[:, None], axis=0)
    smax = np.exp(np.asarray(log_scale, dtype=np.float64).max(axis=0))
    with np.errstate(divide="ignore"):
        r = k_sigma * fx * smax / d
    return r >= r_min, r


def active_set(gate: np.ndarray, keep_bits: np.ndarray | None, fallback_ratio: float = 0.95):
    """Eq. 3: indices (ascending) of gate AND keep.  If the gate keeps at least
    fallback_ratio of the shard it is skipped (reading of "close to one")."""
    gate = np.asarray(gate, dtype=bool)
    n = gate.shape[0]
    if n > 0 and gate.sum() / n >= fallback_ratio:
        gate = np.ones(n, dtype=bool)
    keep = np.ones(n, dtype=bool) if keep_bits is None else unpack_bits(keep_bits, n)
    return np.nonzero(gate & keep)[0].astype(np.int32)


def drop_count(n: int, drop_frac: float) -> int:
    """ceil(drop_frac * n), the number of Gaussians "drop the bottom x%" removes
    (the rank rule of the spawn gate, Sec. 3.2 and Appendix E, rounds up)."""
    return min(n, max(0, int(math.ceil(drop_frac * n))))


def score_keep(score, n_drop: int):
    """Keep mask that drops the n_drop lowest scores, ordered by
    (score ascending, index ascending); never-seen Gaussians score 0."""
    score = np.asarray(score, dtype=np.float64)
    n = score.shape[0]
    order = np.lexsort((np.arange(n), score))
    keep = np.ones(n, dtype=bool)
    keep[order[:n_drop]] = False
    return keep


# --------------------------------------------------------------------------
# Adam (the optimizer the paper's per-rank optimizer state implies)
# --------------------------------------------------------------------------
def adam_step(p, g, m, v, lr, step, b1=0.9, b2=0.999, eps=1e-15):
    """Kingma & Ba (2015), Algorithm 1, with bias correction.  Returns new
    (p, m, v) as float64."""
    p = np.asarray(p, dtype=np.float64)
    g = np.asarray(g, dtype=np.float64)
    m = b1 * np.asarray(m, dtype=np.float64) + (1 - b1) * g
    v = b2 * np.asarray(v, dtype=np.float64) + (1 - b2) * g * g
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


# --------------------------------------------------------------------------
# Scheduled simplification passes (Sec. 3.2 "Scheduled simplification")
# --------------------------------------------------------------------------
def mass_keep(score, frac: float = 0.99):
    """Second pass: the deterministic cumulative-mass cut keeps the smallest
    prefix of (score descending, index ascending) whose summed score reaches
    frac of the total (the crossing element included)."""
    return top_mass(score, frac)


def race_times(score, u):
    """Exponential-race form of weighted sampling without replacement
    (Efraimidis & Spirakis 2006): e_i = -ln(u_i) / s_i, +inf where s_i = 0.
    Keeping the k smallest e_i (equivalently the k largest u_i^(1/s_i)) draws
    k items without replacement with probabilities proportional to s."""
    s = np.asarray(score, dtype=np.float64)
    u = np.asarray(u, dtype=np.float64)
    with np.errstate(divide="ignore"):
        return np.where(s > 0, -np.log(u) / np.where(s > 0, s, 1.0), np.inf)


def sample_keep(score, u, n_keep: int):
    """First pass: stochastic importance-weighted sampling without replacement
    of n_keep Gaussians, with the uniforms u in (0, 1] given; the kept set is
    the n_keep smallest race times, ties by index."""
    e = race_times(score, u)
    n = e.shape[0]
    order = np.lexsort((np.arange(n), e))
    keep = np.zeros(n, dtype=bool)
    keep[order[:n_keep]] = True
    return keep


def compact(arrays, keep):
    """Component-major arrays [..., N] restricted to the kept Gaussians, in
    ascending index order."""
    keep = np.asarray(keep, dtype=bool)
    return [np.ascontiguousarray(np.asarray(a)[..., keep]) for a in arrays]


# --------------------------------------------------------------------------
# The paper's objective (Sec. 3.4, Eqs. 4-5)
# --------------------------------------------------------------------------
SSIM_SIZE = 11
SSIM_SIGMA = 1.5
SSIM_C1 = 0.01 ** 2
SSIM_C2 = 0.03 ** 2


def ssim_window(size: int = SSIM_SIZE, sigma: float = SSIM_SIGMA) -> np.ndarray:
    """Normalised 1-D Gaussian window (the 2-D window is its outer product)."""
    x = np.arange(size, dtype=np.float64) - (size - 1) / 2.0
    g = np.exp(-x * x / (2.0 * sigma * sigma))
    return g / g.sum()


def ssim_map(img, tgt):
    """Per-pixel SSIM (Wang et al. 2004) of two [3][H][W] images with an 11x11
    Gaussian window (sigma 1.5), constants (0.01)^2 and (0.03)^2 for a unit
    dynamic range, local statistics by zero-padded 'same' convolution (the
    paper does not state its SSIM settings; these are the customary ones).
    Differentiable float64 torch expression."""
    x = torch.as_tensor(img, dtype=torch.float64)
    y = torch.as_tensor(tgt, dtype=torch.float64)
    g = torch.from_numpy(ssim_window())
    w = torch.outer(g, g)[None, None].repeat(3, 1, 1, 1)
    conv = lambda t: torch.nn.functional.conv2d(t[None], w, padding=SSIM_SIZE // 2, groups=3)[0]  # noqa: E731
    mx, my = conv(x), conv(y)
    sxx = conv(x * x) - mx * mx
    syy = conv(y * y) - my * my
    sxy = conv(x * y) - mx * my
    return ((2 * mx * my + SSIM_C1) * (2 * sxy + SSIM_C2)) / ((mx * mx + my * my + SSIM_C1) * (sxx + syy + SSIM_C2))


def photo_loss(img, tgt, lam: float = 0.2):
    """Eq. 4 for one view: (1 - lambda) mean|C - I| + lambda (1 - mean SSIM).
    Returns (loss, dL/dC) with the gradient from autograd (sign(0) = 0 in the
    L1 part, as torch's abs)."""
    x = torch.as_tensor(np.asarray(img, dtype=np.float64)).clone().requires_grad_(True)
    y = torch.as_tensor(np.asarray(tgt, dtype=np.float64))
    L = (1 - lam) * (x - y).abs().mean() + lam * (1 - ssim_map(x, y).mean())
    (g,) = torch.autograd.grad(L, x)
    return float(L.item()), g.numpy()


def scale_reg(log_scale, visible, beta: float = 10.0):
    """Eq. 5 regulariser: beta * mean over the visible set of the smallest
    scale axis, and its gradient with respect to the log-scales (the
    derivative flows to the arg-min axis only; first axis wins ties)."""
    ls = np.asarray(log_scale, dtype=np.float64)
    vis = np.asarray(visible, dtype=bool)
    nv = int(vis.sum())
    grad = np.zeros_like(ls)
    if nv == 0:
        return 0.0, grad
    j = np.argmin(ls, axis=0)
    smin = np.exp(ls[j, np.arange(ls.shape[1])])
    L = beta * smin[vis].sum() / nv
    cols = np.nonzero(vis)[0]
    grad[j[cols], cols] = beta * smin[cols] / nv
    return float(L), grad
