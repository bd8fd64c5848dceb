"""ctypes binding of libgsmi.so: one Python function per C entry point, with
the same name, doing argument marshalling only (torch tensors supply device
pointers and the HIP stream).  Every step of the work runs in the library's
HIP kernels; there is no fallback path, and loading fails loudly when the
library has not been built.
"""
from __future__ import annotations

import ctypes
import math
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgsmi.so")

GS_OK = 0
GS_ERR_INVALID_ARG = -1
GS_ERR_CAPACITY = -2
GS_ERR_WORKSPACE = -3
GS_ERR_HIP = -4

GS_LOD_NONE, GS_LOD_LEVEL, GS_LOD_RADIUS = 0, 1, 2
GS_COUNT_COMPOSITED, GS_COUNT_FOOTPRINT = 0, 1
(GS_OP_LOD_MASK, GS_OP_BIN_SORT, GS_OP_RENDER_BWD, GS_OP_IMPORTANCE, GS_OP_SCORE_KEEP, GS_OP_L1_LOSS,
 GS_OP_SIMPLIFY, GS_OP_PHOTO_LOSS, GS_OP_SCALE_REG, GS_OP_PROJECT, GS_OP_VOXEL_LEVELS, GS_OP_SPAWN_GATE) = range(12)
GS_MAX_CAMS = 8
GS_MAX_PAIRS = 1 << 30
REC_FLOATS = 12

EXPORTED = ("gs_workspace_size", "gs_last_error", "gs_num_tiles", "gs_lod_mask", "gs_project", "gs_bin_sort",
            "gs_render_fwd", "gs_render_bwd", "gs_importance", "gs_score_keep_bits", "gs_l1_loss",
            "gs_adam_step", "gs_profile_kernel", "gs_mass_keep_bits", "gs_sample_keep_bits", "gs_compact",
            "gs_photo_loss", "gs_scale_reg", "gs_lod_mask_noalloc", "gs_voxel_levels", "gs_spawn_gate",
            "gs_spawn_stub_score", "gs_lod_level_ceiling")

c_int, c_i32, c_i64, c_f, c_p, c_sz = (ctypes.c_int, ctypes.c_int32, ctypes.c_int64, ctypes.c_float,
                                       ctypes.c_void_p, ctypes.c_size_t)


class GsCamera(ctypes.Structure):
    _fields_ = [("width", c_i32), ("height", c_i32), ("fx", c_f), ("fy", c_f), ("cx", c_f), ("cy", c_f),
                ("R", c_f * 9), ("t", c_f * 3), ("znear", c_f)]


class GsScene(ctypes.Structure):
    _fields_ = [("n", c_i64), ("mean", c_p), ("log_scale", c_p), ("quat", c_p), ("opacity_logit", c_p),
                ("sh", c_p), ("lod", c_p)]


class GsProjected(ctypes.Structure):
    _fields_ = [("rec", c_p), ("depth", c_p), ("radius", c_p), ("tiles_touched", c_p), ("clamp_bits", c_p),
                ("mean2d", c_p), ("conic", c_p), ("opacity", c_p), ("rgb", c_p)]


class GsGrads(ctypes.Structure):
    _fields_ = [("mean", c_p), ("log_scale", c_p), ("quat", c_p), ("opacity_logit", c_p), ("sh", c_p),
                ("overwrite", c_i32)]


class GsLodParams(ctypes.Structure):
    _fields_ = [("mode", c_i32), ("d0", c_f), ("f", c_f), ("l_max", c_i32), ("fallback_ratio", c_f),
                ("radius_min_px", c_f), ("radius_sigma_k", c_f)]


_lib = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2605_13794_amd.build` "
                               "(there is no fallback implementation)")
        L = ctypes.CDLL(LIB_PATH)
        P = c_p
        L.gs_workspace_size.restype = c_sz
        L.gs_workspace_size.argtypes = [c_int, c_i64, c_i64, c_i64, c_int]
        L.gs_last_error.restype = ctypes.c_char_p
        L.gs_last_error.argtypes = []
        L.gs_num_tiles.restype = c_i64
        L.gs_num_tiles.argtypes = [c_i32, c_i32]
        L.gs_lod_mask.argtypes = [P, P, P, P, P, P, P, c_sz, P]
        L.gs_lod_mask_noalloc.argtypes = [P, P, P, P, P, P, P]
        L.gs_voxel_levels.argtypes = [P, c_i64, P, c_f, c_i32, P, P, c_sz, P]
        L.gs_spawn_gate.argtypes = [P, P, P, c_i64, P, P, c_i64, ctypes.c_double, c_i32, P, P, P, P, P, c_sz, P]
        L.gs_spawn_stub_score.argtypes = [P, P, c_i64, P, P]
        L.gs_lod_level_ceiling.argtypes = [c_i64, c_i64, c_i64, c_i32]
        L.gs_lod_level_ceiling.restype = c_i32
        L.gs_project.argtypes = [P, P, c_i64, P, P, c_int, P, P, c_sz, P]
        L.gs_bin_sort.argtypes = [P, P, c_int, c_i64, P, P, c_i64, P, P, P, c_sz, P]
        L.gs_render_fwd.argtypes = [P, P, c_int, P, P, P, P, P, P, P, P, P]
        L.gs_render_bwd.argtypes = [P, P, c_i64, P, P, P, c_int, P, P, P, P, P, P, P, P, P, P, P, c_sz, P]
        L.gs_importance.argtypes = [P, P, c_i64, P, P, c_f, c_f, c_i32, P, P, P, P, P, P, P, c_sz, P]
        L.gs_score_keep_bits.argtypes = [P, c_i64, c_i64, P, P, c_sz, P]
        L.gs_l1_loss.argtypes = [P, P, c_i64, P, P, P, P, c_sz, P]
        L.gs_adam_step.argtypes = [P, P, P, P, P, c_int, P, c_f, c_f, c_f, c_int, P, c_int, P]
        L.gs_profile_kernel.argtypes = [ctypes.c_char_p, P, P]
        L.gs_mass_keep_bits.argtypes = [P, c_i64, c_f, P, P, P, c_sz, P]
        L.gs_sample_keep_bits.argtypes = [P, P, c_i64, c_i64, P, P, c_sz, P]
        L.gs_compact.argtypes = [P, P, P, P, c_int, c_i64, c_i64, P, P, c_sz, P]
        L.gs_photo_loss.argtypes = [P, P, c_i32, c_i32, c_f, c_f, P, P, P, c_sz, P]
        L.gs_scale_reg.argtypes = [P, P, c_i64, P, P, c_f, P, P, P, c_sz, P]
        for name in EXPORTED:
            if name not in ("gs_workspace_size", "gs_last_error", "gs_num_tiles", "gs_lod_level_ceiling"):
                getattr(L, name).restype = c_int
        _lib = L
    return _lib


class GsmiError(RuntimeError):
    def __init__(self, code, fn, msg):
        super().__init__(f"{fn} failed ({code}): {msg}")
        self.code = code


def _check(rc: int, fn: str):
    if rc != GS_OK:
        raise GsmiError(rc, fn, lib().gs_last_error().decode(errors="replace"))


def ptr(t) -> int | None:
    """Device pointer of a tensor (None for None)."""
    if t is None:
        return None
    assert isinstance(t, torch.Tensor)
    return t.data_ptr()


def stream_handle(stream=None) -> int | None:
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


def _ref(x):
    return ctypes.byref(x) if x is not None else None


def camera(cam) -> GsCamera:
    """gs_camera from an object with width, height, fx, fy, cx, cy, R, t, znear."""
    c = GsCamera()
    c.width, c.height = int(cam.width), int(cam.height)
    c.fx, c.fy, c.cx, c.cy = float(cam.fx), float(cam.fy), float(cam.cx), float(cam.cy)
    R = [float(v) for v in __import__("numpy").asarray(cam.R, dtype="float64").reshape(-1)]
    t = [float(v) for v in __import__("numpy").asarray(cam.t, dtype="float64").reshape(-1)]
    c.R[:] = R
    c.t[:] = t
    c.znear = float(getattr(cam, "znear", 0.2))
    return c


def camera_array(cams):
    arr = (GsCamera * len(cams))()
    for i, c in enumerate(cams):
        arr[i] = camera(c)
    return arr


def scene(mean, log_scale, quat, opacity_logit, sh, lod=None) -> GsScene:
    s = GsScene()
    s.n = int(mean.shape[-1])
    s.mean, s.log_scale, s.quat = ptr(mean), ptr(log_scale), ptr(quat)
    s.opacity_logit, s.sh, s.lod = ptr(opacity_logit), ptr(sh), ptr(lod)
    return s


def projected(rec, depth, radius, tiles_touched, clamp_bits, mean2d=None, conic=None, opacity=None,
              rgb=None) -> GsProjected:
    p = GsProjected()
    p.rec, p.depth, p.radius, p.tiles_touched, p.clamp_bits = (ptr(rec), ptr(depth), ptr(radius),
                                                               ptr(tiles_touched), ptr(clamp_bits))
    p.mean2d, p.conic, p.opacity, p.rgb = ptr(mean2d), ptr(conic), ptr(opacity), ptr(rgb)
    return p


def grads(mean, log_scale, quat, opacity_logit, sh, overwrite: bool = False) -> GsGrads:
    g = GsGrads()
    g.mean, g.log_scale, g.quat, g.opacity_logit, g.sh = (ptr(mean), ptr(log_scale), ptr(quat),
                                                          ptr(opacity_logit), ptr(sh))
    g.overwrite = 1 if overwrite else 0
    return g


def lod_params(mode=GS_LOD_NONE, d0=1.0, f=2.0, l_max=0, fallback_ratio=0.95, radius_min_px=0.5,
               radius_sigma_k=1.0) -> GsLodParams:
    p = GsLodParams()
    p.mode, p.d0, p.f, p.l_max = int(mode), float(d0), float(f), int(l_max)
    p.fallback_ratio, p.radius_min_px, p.radius_sigma_k = float(fallback_ratio), float(radius_min_px), float(
        radius_sigma_k)
    return p


def _ptr_array(tensors, ctype=c_p):
    arr = (ctype * len(tensors))()
    for i, t in enumerate(tensors):
        arr[i] = ptr(t)
    return arr


# ---------------------------------------------------------------------------
# Entry points (same names as the C ABI)
# ---------------------------------------------------------------------------
def gs_workspace_size(op, n=0, n_pairs=0, n_tiles=0, n_cams=1) -> int:
    return int(lib().gs_workspace_size(op, n, n_pairs, n_tiles, n_cams))


def gs_num_tiles(width, height) -> int:
    return int(lib().gs_num_tiles(width, height))


def gs_last_error() -> str:
    return lib().gs_last_error().decode(errors="replace")


def gs_lod_mask(scn: GsScene, cam: GsCamera, params: GsLodParams, keep_bits, active_idx, n_active_dev, ws,
                stream=None):
    _check(lib().gs_lod_mask(ctypes.byref(scn), ctypes.byref(cam), ctypes.byref(params), ptr(keep_bits),
                             ptr(active_idx), ptr(n_active_dev), ptr(ws), ws.numel() if ws is not None else 0,
                             stream_handle(stream)), "gs_lod_mask")


def gs_lod_mask_noalloc(scn: GsScene, cam: GsCamera, params: GsLodParams, keep_bits, active_idx, n_active_dev,
                        stream=None):
    _check(lib().gs_lod_mask_noalloc(ctypes.byref(scn), ctypes.byref(cam), ctypes.byref(params), ptr(keep_bits),
                                     ptr(active_idx), ptr(n_active_dev), stream_handle(stream)),
           "gs_lod_mask_noalloc")


def gs_project(scn: GsScene, active_idx, n_in, n_in_dev, cams, outs, ws, stream=None):
    outs_arr = (GsProjected * len(outs))(*outs)
    _check(lib().gs_project(ctypes.byref(scn), ptr(active_idx), int(n_in), ptr(n_in_dev), cams, len(cams),
                            outs_arr, ptr(ws), ws.numel(), stream_handle(stream)), "gs_project")


def gs_bin_sort(projs, cams, n_in, keys, vals, capacity, tile_ranges, n_pairs_dev, ws, stream=None):
    parr = (GsProjected * len(projs))(*projs)
    _check(lib().gs_bin_sort(parr, cams, len(cams), int(n_in), ptr(keys), ptr(vals), int(capacity),
                             ptr(tile_ranges), ptr(n_pairs_dev), ptr(ws), ws.numel(), stream_handle(stream)),
           "gs_bin_sort")


def gs_render_fwd(projs, cams, vals, tile_ranges, bg, out_rgb, out_T, out_last, chain=None, live=None,
                  stream=None):
    parr = (GsProjected * len(projs))(*projs)
    bgv = (c_f * 3)(*[float(x) for x in bg])
    _check(lib().gs_render_fwd(parr, cams, len(cams), ptr(vals), ptr(tile_ranges), bgv, _ptr_array(out_rgb),
                               _ptr_array(out_T), _ptr_array(out_last), ptr(chain), ptr(live),
                               stream_handle(stream)), "gs_render_fwd")


def gs_render_bwd(scn: GsScene, active_idx, n_in, n_in_dev, projs, cams, vals, tile_ranges, bg, out_T, out_last,
                  grad_rgb, grd: GsGrads, grads2d, ws, chain=None, live=None, stream=None):
    parr = (GsProjected * len(projs))(*projs)
    bgv = (c_f * 3)(*[float(x) for x in bg])
    _check(lib().gs_render_bwd(ctypes.byref(scn), ptr(active_idx), int(n_in), ptr(n_in_dev), parr, cams, len(cams),
                               ptr(vals), ptr(tile_ranges), bgv, _ptr_array(out_T), _ptr_array(out_last),
                               _ptr_array(grad_rgb), ptr(chain), ptr(live), ctypes.byref(grd), ptr(grads2d), ptr(ws),
                               ws.numel(),
                               stream_handle(stream)), "gs_render_bwd")


def gs_importance(proj: GsProjected, cam: GsCamera, n, vals, tile_ranges, mass_frac, eps, w, a, score, c_rad, c_vis,
                  cull_row, ws, stream=None, count_mode=0):
    _check(lib().gs_importance(ctypes.byref(proj), ctypes.byref(cam), int(n), ptr(vals), ptr(tile_ranges),
                               float(mass_frac), float(eps), int(count_mode), ptr(w), ptr(a), ptr(score), ptr(c_rad),
                               ptr(c_vis), ptr(cull_row), ptr(ws), ws.numel(), stream_handle(stream)),
           "gs_importance")


def gs_score_keep_bits(score, n, n_drop, keep_bits, ws, stream=None):
    _check(lib().gs_score_keep_bits(ptr(score), int(n), int(n_drop), ptr(keep_bits), ptr(ws), ws.numel(),
                                    stream_handle(stream)), "gs_score_keep_bits")


def gs_voxel_levels(mean, n, origin, delta0, n_levels, lod, ws, stream=None):
    o = (c_f * 3)(*[float(v) for v in origin])
    _check(lib().gs_voxel_levels(ptr(mean), int(n), o, float(delta0), int(n_levels), ptr(lod), ptr(ws), ws.numel(),
                                 stream_handle(stream)), "gs_voxel_levels")


def gs_spawn_gate(lod, clone_parent, p_clone, n_clone, split_parent, p_split, n_split, rho, n_levels,
                  child_parent, child_lod, child_split, ws, stream=None) -> int:
    """Returns the number of instantiated candidates (known on the host)."""
    out = c_i64(-1)
    _check(lib().gs_spawn_gate(ptr(lod), ptr(clone_parent), ptr(p_clone), int(n_clone), ptr(split_parent),
                               ptr(p_split), int(n_split), float(rho), int(n_levels), ptr(child_parent),
                               ptr(child_lod), ptr(child_split), ctypes.byref(out), ptr(ws), ws.numel(),
                               stream_handle(stream)), "gs_spawn_gate")
    return int(out.value)


def gs_lod_level_ceiling(t, t0, t1, n_levels) -> int:
    return int(lib().gs_lod_level_ceiling(int(t), int(t0), int(t1), int(n_levels)))


def gs_spawn_stub_score(scn: GsScene, parent, n, p, stream=None):
    _check(lib().gs_spawn_stub_score(ctypes.byref(scn), ptr(parent), int(n), ptr(p), stream_handle(stream)),
           "gs_spawn_stub_score")


def gs_mass_keep_bits(score, n, mass_frac, keep_bits, n_keep_dev, ws, stream=None):
    _check(lib().gs_mass_keep_bits(ptr(score), int(n), float(mass_frac), ptr(keep_bits), ptr(n_keep_dev), ptr(ws),
                                   ws.numel(), stream_handle(stream)), "gs_mass_keep_bits")


def gs_sample_keep_bits(score, uniforms, n, n_keep, keep_bits, ws, stream=None):
    _check(lib().gs_sample_keep_bits(ptr(score), ptr(uniforms), int(n), int(n_keep), ptr(keep_bits), ptr(ws),
                                     ws.numel(), stream_handle(stream)), "gs_sample_keep_bits")


def gs_compact(src, dst, n, n_keep, keep_bits, ws, stream=None):
    """src/dst: lists of contiguous tensors [..., n] / [..., n_keep] (float32
    or uint8); every leading dimension counts as rows (e.g. [16][3][n] SH is
    48 rows)."""
    k = len(src)
    rows = (ctypes.c_int32 * k)(*[math.prod(int(x) for x in t.shape[:-1]) for t in src])
    eb = (ctypes.c_int32 * k)(*[int(t.element_size()) for t in src])
    _check(lib().gs_compact(_ptr_array(src), _ptr_array(dst), rows, eb, k, int(n), int(n_keep), ptr(keep_bits),
                            ptr(ws), ws.numel(), stream_handle(stream)), "gs_compact")


def gs_photo_loss(rgb, target, width, height, lam, scale, loss_dev, grad, ws, stream=None):
    _check(lib().gs_photo_loss(ptr(rgb), ptr(target), int(width), int(height), float(lam), float(scale),
                               ptr(loss_dev), ptr(grad), ptr(ws), ws.numel(), stream_handle(stream)), "gs_photo_loss")


def gs_scale_reg(scn: GsScene, active_idx, n_in, n_in_dev, radius, beta, loss_dev, grad_log_scale, ws, stream=None):
    _check(lib().gs_scale_reg(ctypes.byref(scn), ptr(active_idx), int(n_in), ptr(n_in_dev), ptr(radius), float(beta),
                              ptr(loss_dev), ptr(grad_log_scale), ptr(ws), ws.numel(), stream_handle(stream)),
           "gs_scale_reg")


def gs_l1_loss(rgb, target, n_vals, loss_dev, grad, ws, stream=None, grad_scale=None):
    _check(lib().gs_l1_loss(ptr(rgb), ptr(target), int(n_vals), ptr(loss_dev), ptr(grad), ptr(grad_scale), ptr(ws),
                            ws.numel() if ws is not None else 0, stream_handle(stream)), "gs_l1_loss")


def gs_adam_step(params, grads_, m, v, lrs, b1, b2, eps, step, clear_grads=False, step_dev=None, stream=None):
    n = len(params)
    counts = (c_i64 * n)(*[int(p.numel()) for p in params])
    lr = (c_f * n)(*[float(x) for x in lrs])
    _check(lib().gs_adam_step(_ptr_array(params), _ptr_array(grads_), _ptr_array(m), _ptr_array(v), counts, n, lr,
                              float(b1), float(b2), float(eps), int(step), ptr(step_dev), int(bool(clear_grads)),
                              stream_handle(stream)), "gs_adam_step")


def gs_profile_kernel(name, start=None, stop=None):
    """Times the launches of kernel `name` with HIP events (see HipEvent)."""
    _check(lib().gs_profile_kernel(name.encode() if name else None, start, stop), "gs_profile_kernel")


class HipEvent:
    """A raw HIP event (handle usable by gs_profile_kernel)."""
    _hip = None

    @classmethod
    def hip(cls):
        if cls._hip is None:
            torch.cuda.init()
            h = None
            for name in ("libamdhip64.so", "libamdhip64.so.7", "libamdhip64.so.6"):
                try:
                    h = ctypes.CDLL(name)
                    break
                except OSError:
                    continue
            if h is None:
                raise RuntimeError("libamdhip64 not found")
            h.hipEventCreate.argtypes = [ctypes.POINTER(c_p)]
            h.hipEventElapsedTime.argtypes = [ctypes.POINTER(ctypes.c_float), c_p, c_p]
            h.hipEventSynchronize.argtypes = [c_p]
            h.hipEventDestroy.argtypes = [c_p]
            cls._hip = h
        return cls._hip

    def __init__(self):
        self.handle = c_p()
        if self.hip().hipEventCreate(ctypes.byref(self.handle)) != 0:
            raise RuntimeError("hipEventCreate failed")

    def elapsed_ms(self, end: "HipEvent") -> float:
        h = self.hip()
        h.hipEventSynchronize(end.handle)
        ms = ctypes.c_float()
        if h.hipEventElapsedTime(ctypes.byref(ms), self.handle, end.handle) != 0:
            raise RuntimeError("hipEventElapsedTime failed")
        return float(ms.value)

    def __del__(self):
        try:
            if self.handle:
                self.hip().hipEventDestroy(self.handle)
        except Exception:
            pass
