"""Device buffers and the forward/backward pipeline of the rasterizer over the
C ABI, plus the torch.autograd.Function that exposes it to training code.

PyTorch only allocates device memory and provides the stream; every step
(gate, projection, binning, sort, compositing, loss, backward, Adam) is a
library call.
"""
from __future__ import annotations

import dataclasses

import numpy as np
import torch

from . import gsmi as G
from . import scenes as S

F32, I32, U8 = torch.float32, torch.int32, torch.uint8


class Workspace:
    """Grow-only device scratch buffer (256-byte aligned)."""

    def __init__(self, device):
        self.device = device
        self.buf = torch.empty(0, dtype=U8, device=device)

    def get(self, nbytes: int) -> torch.Tensor:
        nbytes = max(int(nbytes), 256)
        if self.buf.numel() < nbytes:
            self.buf = torch.empty(nbytes + 4096, dtype=U8, device=self.device)
            if self.buf.data_ptr() % 256:
                raise RuntimeError("workspace allocation is not 256-byte aligned")
        return self.buf


class DeviceScene:
    """Scene parameters resident in device memory (SoA, float32)."""

    def __init__(self, scene: S.Scene, device="cuda", requires_grad=False):
        t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(device)  # noqa: E731
        self.mean = t(scene.mean)
        self.log_scale = t(scene.log_scale)
        self.quat = t(scene.quat)
        self.opacity_logit = t(scene.opacity_logit)
        self.sh = t(scene.sh)
        self.lod = t(scene.lod)
        self.n = scene.n
        if requires_grad:
            for p in self.params():
                p.requires_grad_(True)

    def params(self):
        return [self.mean, self.log_scale, self.quat, self.opacity_logit, self.sh]

    def struct(self, params=None) -> G.GsScene:
        p = params if params is not None else self.params()
        return G.scene(*[x.detach() for x in p], lod=self.lod)


class ProjBuffers:
    """Per-camera outputs of gs_project for up to n entries."""

    def __init__(self, n: int, device, soa: bool = False, centre: bool = True):
        """soa: all component-major copies; centre: the [2][n] mean2d copy
        only, which the binning reads instead of the 48-byte records."""
        n = max(int(n), 1)
        self.n = n
        self.rec = torch.empty(n * G.REC_FLOATS, dtype=F32, device=device)
        self.depth = torch.empty(n, dtype=F32, device=device)
        self.radius = torch.empty(n, dtype=I32, device=device)
        self.tiles = torch.empty(n, dtype=I32, device=device)
        self.clamp = torch.empty(n, dtype=U8, device=device)
        self.soa = soa
        self.mean2d = torch.empty(2, n, dtype=F32, device=device) if (soa or centre) else None
        if soa:
            self.conic = torch.empty(3, n, dtype=F32, device=device)
            self.opacity = torch.empty(n, dtype=F32, device=device)
            self.rgb = torch.empty(3, n, dtype=F32, device=device)

    def struct(self) -> G.GsProjected:
        if self.soa:
            return G.projected(self.rec, self.depth, self.radius, self.tiles, self.clamp, self.mean2d, self.conic,
                               self.opacity, self.rgb)
        return G.projected(self.rec, self.depth, self.radius, self.tiles, self.clamp, self.mean2d)


@dataclasses.dataclass
class FrameOutputs:
    rgb: list
    T: list
    last: list


class Frame:
    """All buffers of one rasterization pass over a batch of cameras."""

    def __init__(self, cams, n_max: int, device="cuda", capacity: int | None = None, soa: bool = False,
                 store_chain: bool = False):
        assert 1 <= len(cams) <= G.GS_MAX_CAMS
        self.store_chain = store_chain
        self.chain = None
        self.device = torch.device(device)
        self.cams = list(cams)
        self.cam_arr = G.camera_array(self.cams)
        self.n_max = int(n_max)
        self.proj = [ProjBuffers(n_max, self.device, soa) for _ in cams]
        self.total_tiles = sum(G.gs_num_tiles(c.width, c.height) for c in cams)
        self.ranges = torch.empty(2 * self.total_tiles, dtype=I32, device=self.device)
        self.n_pairs = torch.zeros(1, dtype=torch.int64, device=self.device)
        self.capacity = 0
        self.keys = self.vals = self.live = None
        self.ws_sort = Workspace(self.device)
        self.ws_proj = Workspace(self.device)
        self.ws_bwd = Workspace(self.device)
        self.ws_loss = Workspace(self.device)
        self.rgb = [torch.empty(3, c.height, c.width, dtype=F32, device=self.device) for c in cams]
        self.T = [torch.empty(c.height, c.width, dtype=F32, device=self.device) for c in cams]
        self.last = [torch.empty(c.height, c.width, dtype=I32, device=self.device) for c in cams]
        self.grad_rgb = [torch.empty_like(x) for x in self.rgb]
        self.loss = torch.zeros(len(cams), dtype=F32, device=self.device)
        self.ensure_capacity(capacity if capacity is not None else max(1024, 4 * self.n_max * len(cams)))
        self.n_in = self.n_max
        self.active = None
        self.n_in_dev = None
        # incremented by every forward: the buffers a backward reads (lists,
        # final transmittance, `last`, projections) belong to one forward
        self.generation = 0

    def ensure_capacity(self, cap: int):
        cap = int(min(max(cap, 1), G.GS_MAX_PAIRS - 1))
        if cap <= self.capacity:
            return
        self.set_capacity(cap)

    def set_capacity(self, cap: int):
        """Pair buffers of exactly `cap` entries (the sort picks its partition
        size from the capacity, so an oversized buffer costs time)."""
        cap = int(min(max(cap, 1), G.GS_MAX_PAIRS - 1))
        self.capacity = cap
        self.keys = torch.empty(cap, dtype=torch.int64, device=self.device)
        self.vals = torch.empty(cap, dtype=I32, device=self.device)
        # per pair: composited by some pixel of its tile (written by the
        # forward, lets the backward skip the others)
        self.live = torch.empty(cap, dtype=torch.uint8, device=self.device)
        self.chain = None

    def proj_structs(self):
        return [p.struct() for p in self.proj]

    # -- forward -----------------------------------------------------------
    def project(self, scn: G.GsScene, active=None, n_in=None, n_in_dev=None, stream=None):
        self.n_in = self.n_max if n_in is None else int(n_in)
        self.active, self.n_in_dev = active, n_in_dev
        ws = self.ws_proj.get(G.gs_workspace_size(G.GS_OP_PROJECT, self.n_in))
        G.gs_project(scn, active, self.n_in, n_in_dev, self.cam_arr, self.proj_structs(), ws, stream)

    def bin_sort(self, check: bool = True, stream=None):
        ws = self.ws_sort.get(G.gs_workspace_size(G.GS_OP_BIN_SORT, self.n_in, self.capacity, self.total_tiles,
                                                  len(self.cams)))
        G.gs_bin_sort(self.proj_structs(), self.cam_arr, self.n_in, self.keys, self.vals, self.capacity,
                      self.ranges, self.n_pairs, ws, stream)
        if check:
            K = int(self.n_pairs.item())
            if K > self.capacity:
                self.ensure_capacity(int(K * 1.25) + 1024)
                return self.bin_sort(check=True, stream=stream)
            return K
        return None

    def render_fwd(self, bg=(0.0, 0.0, 0.0), stream=None, out_rgb=None):
        """Composites every camera; out_rgb (optional) replaces the frame's
        own image buffers (one [3][H][W] tensor per camera)."""
        self.generation += 1
        if out_rgb is not None:
            self.rgb = list(out_rgb)
        self.bg = tuple(float(x) for x in bg)
        chain = None
        if self.store_chain:
            need = 256 * self.capacity
            if self.chain is None or self.chain.numel() < need:
                self.chain = torch.empty(need, dtype=F32, device=self.device)
            chain = self.chain
        G.gs_render_fwd(self.proj_structs(), self.cam_arr, self.vals, self.ranges, self.bg, self.rgb, self.T,
                        self.last, chain=chain, live=self.live, stream=stream)
        return FrameOutputs(self.rgb, self.T, self.last)

    def forward(self, scn, active=None, n_in=None, n_in_dev=None, bg=(0.0, 0.0, 0.0), check=True, stream=None,
                out_rgb=None):
        self.project(scn, active, n_in, n_in_dev, stream)
        K = self.bin_sort(check=check, stream=stream)
        out = self.render_fwd(bg, stream, out_rgb=out_rgb)
        return out, K

    # -- loss and backward ----------------------------------------------------
    def l1_loss(self, targets, stream=None):
        for c, (img, tgt) in enumerate(zip(self.rgb, targets)):
            ws = self.ws_loss.get(G.gs_workspace_size(G.GS_OP_L1_LOSS))
            G.gs_l1_loss(img, tgt, img.numel(), self.loss[c:c + 1], self.grad_rgb[c], ws, stream)
        return self.loss

    def backward(self, scn, grd: G.GsGrads, grad_rgb=None, grads2d=None, stream=None):
        g = grad_rgb if grad_rgb is not None else self.grad_rgb
        ws = self.ws_bwd.get(G.gs_workspace_size(G.GS_OP_RENDER_BWD, self.n_in, 0, 0, len(self.cams)))
        G.gs_render_bwd(scn, self.active, self.n_in, self.n_in_dev, self.proj_structs(), self.cam_arr, self.vals,
                        self.ranges, self.bg, self.T, self.last, g, grd, grads2d, ws,
                        chain=self.chain if self.store_chain else None, live=self.live, stream=stream)


class RasterizeFn(torch.autograd.Function):
    """Differentiable rasterization of a batch of cameras.

    forward(frame, scene, mean, log_scale, quat, opacity_logit, sh) -> images
    [B, 3, H, W] (all cameras of the frame must share one resolution),
    composited straight into a new tensor.  The backward calls gs_render_bwd,
    which recomputes every pixel's transmittance chain from the final T
    instead of storing it (or reads the chain when the frame stores it).

    A frame holds the buffers of its latest forward only: a second forward
    through the same frame before this graph's backward makes the backward
    raise instead of differentiating the wrong frame.
    """

    @staticmethod
    def forward(ctx, frame: Frame, dscene: DeviceScene, mean, log_scale, quat, opacity_logit, sh, active=None,
                n_in_dev=None):
        params = [mean, log_scale, quat, opacity_logit, sh]
        scn = G.scene(*[p.detach() for p in params], lod=dscene.lod)
        n_in = None if active is None else int(active.numel())
        h, w = frame.cams[0].height, frame.cams[0].width
        if any((c.height, c.width) != (h, w) for c in frame.cams):
            raise ValueError("RasterizeFn: every camera of the frame must share one resolution")
        images = torch.empty(len(frame.cams), 3, h, w, dtype=F32, device=frame.device)
        frame.forward(scn, active, n_in, n_in_dev, out_rgb=list(images.unbind(0)))
        ctx.frame, ctx.scn, ctx.params = frame, scn, [p.detach() for p in params]
        ctx.generation = frame.generation
        return images

    @staticmethod
    def backward(ctx, grad_out):
        frame = ctx.frame
        if frame.generation != ctx.generation:
            raise RuntimeError("RasterizeFn.backward: the frame ran another forward after this one; its lists and "
                               "transmittance no longer belong to this graph (use one frame per graph)")
        gr = [torch.zeros_like(p) for p in ctx.params]
        grad_out = grad_out.contiguous()
        frame.backward(ctx.scn, G.grads(*gr, overwrite=True), grad_rgb=list(grad_out.unbind(0)))
        return (None, None, *gr, None, None)


def rasterize(frame: Frame, dscene: DeviceScene, active=None, n_in_dev=None):
    return RasterizeFn.apply(frame, dscene, *dscene.params(), active, n_in_dev)


class L1LossFn(torch.autograd.Function):
    """L = mean |C - target| over all values of C (any shape, float32,
    contiguous) through gs_l1_loss; the backward writes
    dL/dC = g * sign(C - target) / numel with the upstream derivative g read
    on the device (no host synchronisation, no tensor arithmetic)."""

    @staticmethod
    def forward(ctx, img, target):
        img_c, tgt_c = img.detach().contiguous(), target.detach().contiguous()
        if img_c.shape != tgt_c.shape or img_c.dtype != F32 or tgt_c.dtype != F32:
            raise ValueError("l1_loss: image and target must be float32 tensors of one shape")
        loss = torch.empty((), dtype=F32, device=img_c.device)
        ws = torch.empty(G.gs_workspace_size(G.GS_OP_L1_LOSS), dtype=U8, device=img_c.device)
        G.gs_l1_loss(img_c, tgt_c, img_c.numel(), loss, None, ws)
        ctx.save_for_backward(img_c, tgt_c)
        return loss

    @staticmethod
    def backward(ctx, grad_loss):
        img_c, tgt_c = ctx.saved_tensors
        grad = torch.empty_like(img_c)
        G.gs_l1_loss(img_c, tgt_c, img_c.numel(), None, grad, None, grad_scale=grad_loss.detach().contiguous())
        return grad, None


def l1_loss(img, target):
    return L1LossFn.apply(img, target)


class Adam:
    """Adam over the scene's parameter tensors through gs_adam_step.  The
    step counter lives on the device, so a captured graph replays successive
    steps."""

    def __init__(self, params, lrs, b1=0.9, b2=0.999, eps=1e-15):
        self.params = list(params)
        self.lrs = list(lrs)
        self.m = [torch.zeros_like(p) for p in self.params]
        self.v = [torch.zeros_like(p) for p in self.params]
        self.b1, self.b2, self.eps = b1, b2, eps
        self.t_dev = torch.zeros(1, dtype=torch.int32, device=self.params[0].device)

    def step(self, grads, clear_grads=False, stream=None):
        G.gs_adam_step([p.detach() for p in self.params], grads, self.m, self.v, self.lrs, self.b1, self.b2,
                       self.eps, 0, clear_grads, self.t_dev, stream)


DEFAULT_LRS = (1.6e-4, 5e-3, 1e-3, 5e-2, 2.5e-3)  # mean, log_scale, quat, opacity_logit, sh
