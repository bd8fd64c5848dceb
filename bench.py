#!/usr/bin/env python3
"""Throughput of the rasterizer hot path on one MI355X.

Workload (default): the 1M-Gaussian synthetic aerial city, one 1920x1080 view
from 150 m altitude pitched 45 degrees down, L1 loss against a uniform-random
target, FP32.  One step runs every stage of the hot path once, in this order:

  importance refresh of the view: gs_project (whole shard) -> gs_bin_sort ->
      gs_importance (instrumented blend, top-99% mass, Cull row, score fold)
  gated training iteration: gs_lod_mask (0.5 px projected-radius gate AND the
      score mask that drops the 40% lowest-scored Gaussians) -> gs_project
      (active list, device count) -> gs_bin_sort -> gs_render_fwd ->
      gs_l1_loss -> gs_render_bwd (blend + projection backward) -> gs_adam_step

The score mask comes from an importance sweep over 8 views run before the
timed region.  The plain (ungated) and gated training iterations are also
timed on their own and reported beside the step rate, with the PSNR of the
gated image against the plain one.

Prints one JSON line.  `value` is steps/s with all inputs resident in HBM.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "fwd+bwd iterations/s and Mpix/s at 1080p, gated vs plain; serving p50/p99 latency"
PEAK_HBM_GBS = 8000.0
# VALU lane-operation issue rate without packed FP32: 256 CUs x 4 SIMDs x 16
# lanes x 2.4 GHz (an FMA counts as one operation).
PEAK_ALU_GOPS = 256 * 4 * 16 * 2.4
# Algorithmic operations of the backward blend (an FMA counts as one): every
# list position below a pixel's `last` re-evaluates alpha (13 ops: offsets,
# quadratic form, exp, opacity product, clamp, threshold test); each
# composited (pixel, Gaussian) pair then costs 37 more (transmittance
# recovery, dL/dalpha over 3 channels and the background term, the running
# colour behind, colour, opacity, mean and conic partials).
ALPHA_OPS = 13.0
BWD_COMPOSITED_OPS = 37.0
# Algorithmic bytes of Adam per parameter float: parameter, gradient and both
# moments read, parameter and moments written (4 B each).
ADAM_BYTES_PER_FLOAT = 28


def parse():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--n", type=int, default=1 << 20, help="Gaussians in the shard")
    ap.add_argument("--width", type=int, default=1920)
    ap.add_argument("--height", type=int, default=1080)
    ap.add_argument("--drop", type=float, default=0.4, help="score-mask drop fraction")
    ap.add_argument("--rmin", type=float, default=0.5, help="projected-radius gate, px")
    ap.add_argument("--kernel", default="adam", help="kernel of the roofline entry: adam (the step's largest "
                                                    "kernel, HBM-bound), render_bwd (ALU-bound), or any kernel "
                                                    "for its time only")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--quick", action="store_true", help="skip the plain/gated side measurements")
    ap.add_argument("--graph", action="store_true", help="capture the step in a HIP graph and replay it")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device-to-device copy 5 times (counter calibration)")
    ap.add_argument("--serve-seconds", type=float, default=60.0,
                    help="measured seconds of the serving trace (0 disables serving)")
    ap.add_argument("--serve-warmup", type=float, default=5.0)
    ap.add_argument("--serve-n", type=int, default=8 << 20, help="Gaussians of the served scene")
    ap.add_argument("--layout", default="morton", choices=["morton", "generated"],
                    help="memory order of the Gaussians: Morton order of the means, or the generator's order")
    ap.add_argument("--config", default="cfg2", choices=["cfg2", "cfg3", "cfg4", "serve"],
                    help="cfg2: 1M city, one 1080p view (default line); cfg3: 8M city, 64-view importance "
                         "sweep and gated vs ungated views; cfg4: 5M city, batch of 4 1080p views with Adam; "
                         "serve: the serving traces alone over the resident 8M city")
    return ap.parse_args()


# Committed HBM traffic per launch (profiler counters) and the sources each
# figure was taken from.
TRAFFIC = {
    "render_bwd": ("render_bwd_1M_city_1080p_traffic.md",
                   ("paper_2605_13794_amd/csrc/render.hip", "paper_2605_13794_amd/csrc/common.h")),
    "adam": ("adam_1M_city_1080p_traffic.md",
             ("paper_2605_13794_amd/csrc/misc.hip", "paper_2605_13794_amd/csrc/common.h")),
}


def recorded_traffic(kernel, args):
    """HBM bytes per launch of `kernel` from the committed profiler counters
    (read + write, copy-calibrated), or None when they do not apply: another
    kernel or workload, or kernel sources changed since the counters were
    taken (their sha256 is recorded with them)."""
    import hashlib
    if kernel not in TRAFFIC or args.config != "cfg2" or args.layout != "morton" or args.n != 1 << 20 or \
            (args.width, args.height) != (1920, 1080) or args.rmin != 0.5 or args.drop != 0.4:
        return None
    fname, sources = TRAFFIC[kernel]
    root = os.path.dirname(os.path.abspath(__file__))
    try:
        text = open(os.path.join(root, "profiles", fname)).read()
    except OSError:
        return None
    fields = dict(line.split(": ", 1) for line in text.splitlines() if ": " in line and not line.startswith("|"))
    h = hashlib.sha256()
    for f in sources:
        h.update(open(os.path.join(root, f), "rb").read())
    if fields.get("kernel") != kernel or fields.get("source_sha256") != h.hexdigest():
        return None
    return int(fields["fetch_bytes_per_launch"]) + int(fields["write_bytes_per_launch"])


def layout(scene, args):
    """Memory order of the shard: Morton order of the means (default), or the
    generator's random order."""
    return scene.spatially_ordered() if args.layout == "morton" else scene


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


class Bench:
    def __init__(self, args):
        import numpy as np
        import torch

        from paper_2605_13794_amd import gsmi as G
        from paper_2605_13794_amd import scenes as S
        from paper_2605_13794_amd.raster import Adam, DEFAULT_LRS, DeviceScene, Frame, Workspace

        self.np, self.torch, self.G, self.S = np, torch, G, S
        G.lib()
        self.dev = torch.device("cuda:0")
        dev = self.dev
        self.args = args
        t0 = time.time()
        self.scene = layout(S.city_scene(args.n, seed=2), args)
        self.cam = S.aerial_camera(args.width, args.height)
        log(f"scene {self.scene.n} Gaussians generated in {time.time() - t0:.1f}s")
        self.ds = DeviceScene(self.scene, dev)
        self.n = self.scene.n
        n = self.n
        self.camc = G.camera(self.cam)
        self.target = torch.from_numpy(S.target_image(args.width, args.height, seed=1)).to(dev)
        self.fr_all = Frame([self.cam], n, dev)        # whole shard (importance, plain)
        self.fr = Frame([self.cam], n, dev)            # gated active set
        self.grads = [torch.zeros_like(p) for p in self.ds.params()]
        # Adam clears the gradients it reads, so the backward stores the
        # reached Gaussians' gradients instead of adding to zeros
        self.grads_s = G.grads(*self.grads, overwrite=True)
        self.adam = Adam(self.ds.params(), DEFAULT_LRS)
        # importance state
        self.w = torch.empty(n, device=dev)
        self.a = torch.empty(n, dtype=torch.int32, device=dev)
        self.score = torch.zeros(n, device=dev)
        self.c_rad = torch.zeros(n, dtype=torch.int32, device=dev)
        self.c_vis = torch.zeros(n, dtype=torch.int32, device=dev)
        self.sweep_views = 8
        self.cull = torch.zeros(self.sweep_views + 1, (n + 31) // 32, dtype=torch.int32, device=dev)
        self.keep = torch.zeros((n + 31) // 32, dtype=torch.int32, device=dev)
        self.ws_imp = Workspace(dev).get(G.gs_workspace_size(G.GS_OP_IMPORTANCE, n))
        self.ws_keep = Workspace(dev).get(G.gs_workspace_size(G.GS_OP_SCORE_KEEP, n))
        self.ws_lod = Workspace(dev).get(G.gs_workspace_size(G.GS_OP_LOD_MASK, n))
        self.active = torch.empty(n, dtype=torch.int32, device=dev)
        self.n_act = torch.zeros(1, dtype=torch.int64, device=dev)
        self.lodp = G.lod_params(G.GS_LOD_RADIUS, fallback_ratio=0.95, radius_min_px=args.rmin, radius_sigma_k=1.0)
        # second stream (default priority) for the importance refresh
        self.s_imp = torch.cuda.Stream(device=dev)
        self.ev_proj = torch.cuda.Event()

    # -- pieces ---------------------------------------------------------------
    def importance_view(self, fr, camc, view_row):
        G = self.G
        fr.project(self.ds.struct())
        fr.bin_sort(check=False)
        G.gs_importance(fr.proj[0].struct(), camc, self.n, fr.vals, fr.ranges, 0.99, 1e-6, self.w, self.a,
                        self.score, self.c_rad, self.c_vis, self.cull[view_row], self.ws_imp)

    def sweep(self):
        """Importance sweep over 8 views around the training view, then the
        score mask (outside the timed region)."""
        from paper_2605_13794_amd.raster import Frame
        S, G = self.S, self.G
        self.score.zero_()
        self.c_rad.zero_()
        self.c_vis.zero_()
        for v in range(self.sweep_views):
            cam = S.aerial_camera(self.args.width, self.args.height, heading_deg=45.0 * v)
            fr = Frame([cam], self.n, self.dev)
            fr.project(self.ds.struct())
            fr.bin_sort(check=True)
            G.gs_importance(fr.proj[0].struct(), G.camera(cam), self.n, fr.vals, fr.ranges, 0.99, 1e-6, self.w,
                            self.a, self.score, self.c_rad, self.c_vis, self.cull[v], self.ws_imp)
        n_drop = int(math.ceil(self.args.drop * self.n))
        G.gs_score_keep_bits(self.score, self.n, n_drop, self.keep, self.ws_keep)
        self.torch.cuda.synchronize()

    def gate(self):
        self.G.gs_lod_mask(self.ds.struct(), self.camc, self.lodp, self.keep, self.active, self.n_act, self.ws_lod)

    def train_iter(self, gated: bool, before_adam=None):
        fr = self.fr if gated else self.fr_all
        scn = self.ds.struct()
        if gated:
            self.gate()
            fr.project(scn, self.active, self.n, self.n_act)
        else:
            fr.project(scn)
        fr.bin_sort(check=False)
        fr.render_fwd()
        fr.l1_loss([self.target])
        fr.backward(scn, self.grads_s)
        if before_adam is not None:
            before_adam()
        self.adam.step(self.grads, clear_grads=True)

    def step(self):
        """One step: the view's importance refresh runs on its own stream
        beside the gated training iteration.  The refresh reads the parameters
        only in its projection, so Adam waits for that projection (an event),
        and the next step's refresh waits for Adam; the step ends when both
        streams are done."""
        torch, G = self.torch, self.G
        main = torch.cuda.current_stream()
        side = self.s_imp
        side.wait_stream(main)
        with torch.cuda.stream(side):
            fr = self.fr_all
            fr.project(self.ds.struct())
            self.ev_proj.record(side)
            fr.bin_sort(check=False)
            G.gs_importance(fr.proj[0].struct(), self.camc, self.n, fr.vals, fr.ranges, 0.99, 1e-6, self.w, self.a,
                            self.score, self.c_rad, self.c_vis, self.cull[self.sweep_views], self.ws_imp)
        self.train_iter(gated=True, before_adam=lambda: main.wait_event(self.ev_proj))
        main.wait_stream(side)

    # -- setup ---------------------------------------------------------------
    def size_buffers(self):
        """One checked pass per frame sizes the pair buffers (twice the pairs: the
        optimizer grows the footprints while the timed steps run)."""
        scn = self.ds.struct()
        self.fr_all.project(scn)
        K_all = self.fr_all.bin_sort(check=True)
        self.fr_all.set_capacity(int(K_all * 2) + 4096)
        self.gate()
        self.fr.project(scn, self.active, self.n, self.n_act)
        K = self.fr.bin_sort(check=True)
        self.fr.set_capacity(int(K * 2) + 4096)
        self.torch.cuda.synchronize()
        return K_all, K

    def check_capacity(self):
        for fr in (self.fr, self.fr_all):
            k = int(fr.n_pairs.item())
            if k < 0 or k > fr.capacity:
                raise RuntimeError(f"pair buffer overflow during timing: K={k} capacity={fr.capacity}")

    def graphed(self, fn):
        """Captures fn (no host synchronisation inside) into a HIP graph;
        returns its replay."""
        torch = self.torch
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
        self._graphs = getattr(self, "_graphs", []) + [g]
        return g.replay

    def timed(self, fn, steps, warmup):
        torch = self.torch
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / steps

    def kernel_time(self, name, fn, reps, after_each=None):
        """Average duration of kernel `name` over `reps` calls of fn, from HIP
        events recorded around the kernel itself on its own stream.  With
        after_each, the launch durations are returned one per call, and
        after_each() runs after each call (outside the kernel's events) to
        record the work that launch did."""
        G = self.G
        evs = [(G.HipEvent(), G.HipEvent()) for _ in range(reps)]
        work = []
        for e0, e1 in evs:
            G.gs_profile_kernel(name, e0.handle, e1.handle)
            fn()
            if after_each is not None:
                G.gs_profile_kernel(None)
                self.torch.cuda.synchronize()
                work.append(after_each())
        G.gs_profile_kernel(None)
        self.torch.cuda.synchronize()
        ms = [e0.elapsed_ms(e1) for e0, e1 in evs]
        if after_each is not None:
            return ms, work
        return sum(ms) / reps

    def psnr_gated_vs_plain(self):
        torch = self.torch
        scn = self.ds.struct()
        self.fr_all.forward(scn, check=False)
        self.gate()
        self.fr.forward(scn, self.active, self.n, self.n_act, check=False)
        torch.cuda.synchronize()
        mse = float(((self.fr.rgb[0] - self.fr_all.rgb[0]) ** 2).mean().item())
        return psnr_db(mse)


def psnr_db(mse):
    """PSNR in dB of an image pair with mean squared error `mse` on [0, 1]
    colours; None for identical images (infinite PSNR, which strict JSON
    cannot carry)."""
    return 10.0 * math.log10(1.0 / mse) if mse > 0 else None


def finite(x):
    """`x` with every non-finite float replaced by None, so that the printed
    line is strict JSON."""
    if isinstance(x, dict):
        return {k: finite(v) for k, v in x.items()}
    if isinstance(x, (list, tuple)):
        return [finite(v) for v in x]
    if isinstance(x, float) and not math.isfinite(x):
        return None
    return x


def hbm_fractions(ds, cam, n, capacity, dev, reps=5):
    """Algorithmic HBM bytes per second of the ungated projection, of the
    whole binning call (scan, emission, sort, ranges) and of the projection
    backward on one view, timed with events on their stream, against 8 TB/s.
    Bytes: projection 12 N (means, read to cull) + 224 N_vis (the rest) + 49 N
    (outputs); binning 8 N (scan) + 20 N_vis + 12 K (emission) + K (8 + 24 d)
    (d = 8-bit passes of a full-key radix sort over the 32 depth and the tile
    bits) + 8 K + 8 tiles (ranges); projection backward 557 N_vis; gate and
    active-set compaction 24 N + N/8 + 4 N_active; compaction of parameters
    and Adam moments 708 N (read: at a 60 % keep density every 128-byte line
    of a row holds kept columns) + 708 N_keep (written) + N/8."""
    import torch

    from paper_2605_13794_amd import gsmi as G
    from paper_2605_13794_amd.raster import Frame
    f = Frame([cam], n, dev, capacity=int(capacity * 1.2) + 4096)
    f.project(ds.struct())
    f.bin_sort(check=False)
    torch.cuda.synchronize()
    e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    t_proj = t_sort = 0.0
    for _ in range(reps):
        e[0].record()
        f.project(ds.struct())
        e[1].record()
        f.bin_sort(check=False)
        e[2].record()
        torch.cuda.synchronize()
        t_proj += e[0].elapsed_time(e[1]) / reps
        t_sort += e[1].elapsed_time(e[2]) / reps
    n_vis = int((f.proj[0].radius[:n] > 0).sum().item())
    K = int(f.n_pairs.item())
    tiles = f.total_tiles
    d = (32 + max(1, (tiles - 1).bit_length()) + 7) // 8
    b_proj = 12 * n + 224 * n_vis + 49 * n
    b_sort = 8 * n + 20 * n_vis + 12 * K + K * (8 + 24 * d) + 8 * K + 8 * tiles
    # projection backward: parameters (236), projection (49) and screen-space
    # partials (36) read, parameter gradients (236) written per visible entry
    # (stored, not added: the gradients start at zero); its two kernels timed
    # on their own launches
    grads = [torch.zeros_like(p) for p in ds.params()]
    gs = G.grads(*grads, overwrite=True)
    f.render_fwd()
    g_img = [torch.full_like(f.rgb[0], 1e-7)]
    t_pbwd = 0.0
    for kname in ("project_bwd", "project_bwd_sh"):
        evs = [(G.HipEvent(), G.HipEvent()) for _ in range(reps)]
        for e0, e1 in evs:
            G.gs_profile_kernel(kname, e0.handle, e1.handle)
            f.backward(ds.struct(), gs, grad_rgb=g_img)
        G.gs_profile_kernel(None)
        torch.cuda.synchronize()
        t_pbwd += sum(e0.elapsed_ms(e1) for e0, e1 in evs) / reps
    b_pbwd = (236 + 49 + 36 + 236) * n_vis
    # the active set and the compaction after a simplification pass, with one
    # seeded keep mask (60 % of the shard): the gate (radius mode, 0.5 px) and
    # its compaction read the means and log-scales (24 B) and the keep bits,
    # and write the active indices (4 B each); gs_compact reads every line of
    # the parameters and both Adam moments (708 B per Gaussian), writes the
    # kept columns (708 B each) and reads the keep bits
    import numpy as np
    rng = np.random.default_rng(11)
    keep_np = rng.random(n) < 0.6
    # bit i % 32 of word i / 32
    words = np.packbits(np.pad(keep_np, (0, (-n) % 32)).reshape(-1, 32), axis=1, bitorder="little")
    keep_w = torch.from_numpy(np.ascontiguousarray(words).view("<u4").view(np.int32).reshape(-1).copy()).to(dev)
    n_keep = int(keep_np.sum())
    active = torch.empty(n, dtype=torch.int32, device=dev)
    n_act = torch.zeros(1, dtype=torch.int64, device=dev)
    ws_lod = torch.empty(G.gs_workspace_size(G.GS_OP_LOD_MASK, n), dtype=torch.uint8, device=dev)
    lodp = G.lod_params(G.GS_LOD_RADIUS, fallback_ratio=0.95, radius_min_px=0.5, radius_sigma_k=1.0)
    camc = G.camera(cam)
    G.gs_lod_mask(ds.struct(), camc, lodp, keep_w, active, n_act, ws_lod)
    for _ in range(2):
        e[0].record()
        for _ in range(reps):
            G.gs_lod_mask(ds.struct(), camc, lodp, keep_w, active, n_act, ws_lod)
        e[1].record()
        torch.cuda.synchronize()
    t_gate = e[0].elapsed_time(e[1]) / reps
    n_active = int(n_act.item())
    b_gate = 24 * n + (n + 7) // 8 + 4 * n_active
    params = [p.detach() for p in ds.params()]
    src = params + [torch.zeros_like(p) for p in params] + [torch.zeros_like(p) for p in params]
    dst = [torch.empty(*(p.shape[:-1] + (n_keep,)), dtype=p.dtype, device=dev) for p in src]
    ws_c = torch.empty(G.gs_workspace_size(G.GS_OP_SIMPLIFY, n), dtype=torch.uint8, device=dev)
    G.gs_compact(src, dst, n, n_keep, keep_w, ws_c)
    torch.cuda.synchronize()
    e[0].record()
    for _ in range(reps):
        G.gs_compact(src, dst, n, n_keep, keep_w, ws_c)
    e[1].record()
    torch.cuda.synchronize()
    t_comp = e[0].elapsed_time(e[1]) / reps
    per_g = sum(int(t.element_size()) * (t.numel() // n) for t in src)
    b_comp = per_g * (n + n_keep) + (n + 7) // 8
    del src, dst
    res = {}
    for name, b, t in (("project", b_proj, t_proj), ("bin_sort", b_sort, t_sort), ("project_bwd", b_pbwd, t_pbwd),
                       ("lod_mask", b_gate, t_gate), ("compact", b_comp, t_comp)):
        gbs = b / (t * 1e-3) / 1e9
        res[name] = {"ms": t, "bytes": b, "GB_per_s": gbs, "frac": gbs / PEAK_HBM_GBS}
    res["n"], res["n_visible"], res["pairs"] = n, n_vis, K
    res["n_active"], res["n_keep"] = n_active, n_keep
    res["sort_path"] = "per-tile depth sort" if f.capacity <= 256 * tiles else "depth-first"
    return res


LOD_LEVELS = 8


def voxel_lod(ds, mean_host, cams, dev):
    """LOD labels of the resident scene by multi-resolution voxelisation
    (gs_voxel_levels), replacing the generator's labels.  d0 is the median
    over the views of the camera's distance to the centroid of the means; the
    level-0 cube edge is d0 / fx, so a level-l cube spans about one pixel at
    distance d0 / 2^l and the level gate keeps one Gaussian per cube of about
    a pixel or more.  Returns (d0, seconds of the labelling call, counts per
    level)."""
    import numpy as np
    import torch

    from paper_2605_13794_amd import gsmi as G
    from paper_2605_13794_amd.raster import Workspace
    centre = mean_host.astype(np.float64).mean(axis=1)
    d0 = float(np.median([np.linalg.norm(c.position - centre) for c in cams]))
    origin = mean_host.min(axis=1).astype(np.float32)
    delta0 = d0 / cams[0].fx
    n = ds.n
    lod = torch.empty(n, dtype=torch.uint8, device=dev)
    ws = Workspace(dev).get(G.gs_workspace_size(G.GS_OP_VOXEL_LEVELS, n))
    G.gs_voxel_levels(ds.mean, n, origin, delta0, LOD_LEVELS, lod, ws)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    G.gs_voxel_levels(ds.mean, n, origin, delta0, LOD_LEVELS, lod, ws)
    torch.cuda.synchronize()
    sec = time.perf_counter() - t0
    ds.lod = lod
    counts = torch.bincount(lod.to(torch.int64), minlength=LOD_LEVELS).tolist()
    return d0, delta0, sec, counts


def active_set_leg(ds, mean_host, args, sample_views=tuple(range(0, 64, 8)), reps=5, drop_sweep=False):
    """Active-set reduction on one GPU's shard (Sec. 3.2-3.3): importance over
    64 orbit views, the score mask (drop the lowest 40% by score), then per
    view the projected-radius gate (0.5 px) or the level gate (Eqs. 1-2, labels
    by voxelisation), each AND the mask (Eq. 3); forward+backward (L1) of the
    plain and gated views timed side by side, PSNR of each gated image against
    the plain one."""
    import numpy as np
    import torch

    from paper_2605_13794_amd import gsmi as G
    from paper_2605_13794_amd import scenes as S
    from paper_2605_13794_amd.raster import Frame, Workspace
    dev = torch.device("cuda:0")
    n = ds.n
    W, H = args.width, args.height
    cams = S.orbit_cameras(64, 500.0, 300.0, W, H)
    d0, delta0, lod_sec, lod_counts = voxel_lod(ds, mean_host, cams, dev)
    fr = Frame([cams[0]], n, dev)
    w = torch.empty(n, device=dev)
    a = torch.empty(n, dtype=torch.int32, device=dev)
    score = torch.zeros(n, device=dev)
    c_rad = torch.zeros(n, dtype=torch.int32, device=dev)
    c_vis = torch.zeros(n, dtype=torch.int32, device=dev)
    cull = torch.zeros(64, (n + 31) // 32, dtype=torch.int32, device=dev)
    ws_imp = Workspace(dev).get(G.gs_workspace_size(G.GS_OP_IMPORTANCE, n))
    fr.project(ds.struct())
    K0 = fr.bin_sort(check=True)
    fr.ensure_capacity(int(K0 * 1.5) + 4096)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    Ks = []
    for v, cam in enumerate(cams):
        fr.cams, fr.cam_arr = [cam], G.camera_array([cam])
        fr.project(ds.struct())
        fr.bin_sort(check=False)
        G.gs_importance(fr.proj[0].struct(), G.camera(cam), n, fr.vals, fr.ranges, 0.99, 1e-6, w, a, score, c_rad,
                        c_vis, cull[v], ws_imp)
        Ks.append(fr.n_pairs.clone())
    torch.cuda.synchronize()
    sweep_ms = 1e3 * (time.perf_counter() - t0) / 64
    Kmax = max(int(k.item()) for k in Ks)
    if Kmax > fr.capacity:
        raise RuntimeError("pair capacity exceeded during the importance sweep")
    keep = torch.zeros((n + 31) // 32, dtype=torch.int32, device=dev)
    ws_keep = Workspace(dev).get(G.gs_workspace_size(G.GS_OP_SCORE_KEEP, n))
    G.gs_score_keep_bits(score, n, int(math.ceil(0.4 * n)), keep, ws_keep)
    active = torch.empty(n, dtype=torch.int32, device=dev)
    n_act = torch.zeros(1, dtype=torch.int64, device=dev)
    ws_lod = Workspace(dev).get(G.gs_workspace_size(G.GS_OP_LOD_MASK, n))
    modes = {
        "mask": (G.lod_params(G.GS_LOD_NONE, fallback_ratio=0.95), keep),
        "radius+mask": (G.lod_params(G.GS_LOD_RADIUS, fallback_ratio=0.95, radius_min_px=0.5), keep),
        "level+mask": (G.lod_params(G.GS_LOD_LEVEL, d0=d0, f=2.0, l_max=LOD_LEVELS - 1, fallback_ratio=0.95), keep),
        "level": (G.lod_params(G.GS_LOD_LEVEL, d0=d0, f=2.0, l_max=LOD_LEVELS - 1, fallback_ratio=0.95), None),
    }
    fractions = {}
    for name, (prm, kb) in modes.items():
        got = []
        for cam in cams:
            G.gs_lod_mask(ds.struct(), G.camera(cam), prm, kb, active, n_act, ws_lod)
            got.append(n_act.clone())
        f = [int(x.item()) / n for x in got]
        fractions[name] = {"mean": float(np.mean(f)), "min": float(np.min(f)), "max": float(np.max(f))}
    grads = [torch.zeros_like(p) for p in ds.params()]
    gs = G.grads(*grads, overwrite=True)
    target = torch.from_numpy(S.target_image(W, H, seed=1)).to(dev)
    f = Frame([cams[0]], n, dev, capacity=int(Kmax * 1.2) + 4096)

    def timed_fb(fn):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        return 1e3 * (time.perf_counter() - t0) / reps

    rows = []
    for v in sample_views:
        cam = cams[v]
        f.cams, f.cam_arr = [cam], G.camera_array([cam])
        camc = G.camera(cam)

        def fb_plain():
            f.forward(ds.struct(), check=False)
            f.l1_loss([target])
            f.backward(ds.struct(), gs)

        row = {"view": v, "plain_fwd_bwd_ms": timed_fb(fb_plain), "plain_pairs": int(f.n_pairs.item())}
        plain_img = f.rgb[0].clone()
        for name, (prm, kb) in modes.items():
            def fb_gated(prm=prm, kb=kb):
                G.gs_lod_mask(ds.struct(), camc, prm, kb, active, n_act, ws_lod)
                f.forward(ds.struct(), active, n, n_act, check=False)
                f.l1_loss([target])
                f.backward(ds.struct(), gs)
            ms = timed_fb(fb_gated)
            mse = float(((f.rgb[0] - plain_img) ** 2).mean().item())
            row[name] = {"fwd_bwd_ms": ms, "speedup": row["plain_fwd_bwd_ms"] / ms, "psnr_db": psnr_db(mse),
                         "active_fraction": int(n_act.item()) / n, "pairs": int(f.n_pairs.item())}
        rows.append(row)
    px = W * H
    summary = {}
    plain_ms = float(np.mean([r["plain_fwd_bwd_ms"] for r in rows]))
    summary["plain"] = {"fwd_bwd_ms": plain_ms, "it_per_s": 1e3 / plain_ms, "mpix_per_s": px / 1e3 / plain_ms}
    for name in modes:
        ms = float(np.mean([r[name]["fwd_bwd_ms"] for r in rows]))
        ps = [r[name]["psnr_db"] for r in rows]
        summary[name] = {"fwd_bwd_ms": ms, "it_per_s": 1e3 / ms, "mpix_per_s": px / 1e3 / ms,
                         "speedup": plain_ms / ms,
                         "psnr_db_min": None if any(p is None for p in ps) else float(np.min(ps)),
                         "psnr_db_mean": None if any(p is None for p in ps) else float(np.mean(ps)),
                         "active_fraction_64_views": fractions[name]}
    hbm = hbm_fractions(ds, cams[0], n, Kmax, dev)
    out = {"workload": f"aerial city {n} Gaussians, 64 orbit views {W}x{H} (radius 500 m, altitude 300 m): "
                       f"importance sweep, score mask (drop 40%), radius gate 0.5 px or level gate (Eqs. 1-2), "
                       f"fwd+bwd L1 on views {list(sample_views)}",
           "importance_ms_per_view": sweep_ms, "pairs_max": Kmax,
           "lod": {"levels": LOD_LEVELS, "d0_m": d0, "delta0_m": delta0, "labelling_ms": 1e3 * lod_sec,
                   "gaussians_per_level": lod_counts},
           "summary": summary, "views": rows, "hbm_fraction": hbm}
    if drop_sweep:
        out["drop_radius_sweep"] = drop_radius_sweep(ds, cams, score, f, target, gs, active, n_act, ws_lod, dev)
    return out


def drop_radius_sweep(ds, cams, score, f, target, gs, active, n_act, ws_lod, dev, views=(0, 32)):
    """Speed at equal image error: drop share x radius threshold on two views."""
    import torch

    from paper_2605_13794_amd import gsmi as G
    from paper_2605_13794_amd.raster import Workspace
    n = ds.n
    sweep = []
    ws_keep = Workspace(dev).get(G.gs_workspace_size(G.GS_OP_SCORE_KEEP, n))
    keep2 = torch.zeros((n + 31) // 32, dtype=torch.int32, device=dev)
    plain_img, plain_ms = {}, {}

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(5):
            fn()
        torch.cuda.synchronize()
        return 1e3 * (time.perf_counter() - t0) / 5

    for v in views:
        f.cams, f.cam_arr = [cams[v]], G.camera_array([cams[v]])

        def fb_plain():
            f.forward(ds.struct(), check=False)
            f.l1_loss([target])
            f.backward(ds.struct(), gs)
        plain_ms[v] = timed(fb_plain)
        plain_img[v] = f.rgb[0].clone()
    for drop in (0.0, 0.2, 0.4, 0.6):
        G.gs_score_keep_bits(score, n, int(math.ceil(drop * n)), keep2, ws_keep)
        for rmin in (0.0, 0.5, 1.0):
            p2 = G.lod_params(G.GS_LOD_RADIUS, fallback_ratio=0.95, radius_min_px=rmin)
            for v in views:
                cam = cams[v]
                f.cams, f.cam_arr = [cam], G.camera_array([cam])

                def fb_gated():
                    G.gs_lod_mask(ds.struct(), G.camera(cam), p2, keep2, active, n_act, ws_lod)
                    f.forward(ds.struct(), active, n, n_act, check=False)
                    f.l1_loss([target])
                    f.backward(ds.struct(), gs)
                ms = timed(fb_gated)
                mse = float(((f.rgb[0] - plain_img[v]) ** 2).mean().item())
                sweep.append({"drop": drop, "radius_min_px": rmin, "view": v,
                              "active_fraction": int(n_act.item()) / n, "fwd_bwd_ms": ms,
                              "speedup": plain_ms[v] / ms, "psnr_db": psnr_db(mse)})
    return sweep


def run_cfg3(args):
    """8M city on its own: the active-set leg of the default line plus the
    drop x radius sweep; with --quick only the HBM fractions of projection,
    binning and projection backward on the first orbit view (the command the
    committed 8M kernel profiles come from)."""
    import torch

    from paper_2605_13794_amd import scenes as S
    from paper_2605_13794_amd.raster import DeviceScene, Frame
    n = args.n if args.n != (1 << 20) else (8 << 20)
    sc = layout(S.city_scene(n, seed=5), args)
    ds = DeviceScene(sc, "cuda:0")
    mean_host = sc.mean
    del sc
    if args.quick:
        dev = torch.device("cuda:0")
        cam = S.orbit_cameras(64, 500.0, 300.0, args.width, args.height)[0]
        f = Frame([cam], n, dev)
        f.project(ds.struct())
        K = f.bin_sort(check=True)
        del f
        hbm = hbm_fractions(ds, cam, n, K, dev, reps=max(5, args.steps))
        out = {"metric": METRIC, "config": {"workload": f"aerial city {n} Gaussians, orbit view 0 "
                                                        f"{args.width}x{args.height}, ungated"},
               "hbm_fraction": hbm}
        print(json.dumps(finite(out), allow_nan=False), flush=True)
        return
    res = active_set_leg(ds, mean_host, args, drop_sweep=True)
    torch.cuda.synchronize()
    out = {"metric": METRIC, "config": {"workload": res.pop("workload")}, **res}
    print(json.dumps(finite(out), allow_nan=False), flush=True)


def batch4_leg(args, n=5 << 20, steps=10, warmup=3):
    """5M city, a batch of 4 1080p views (the aerial pose at headings 0, 90,
    180, 270 degrees) through RasterizeFn, the L1 autograd function (both
    through the library) and Adam; once with the transmittance recomputed
    from the final T in the backward, once with the forward storing the
    chain; peak device memory of each."""
    import torch

    from paper_2605_13794_amd import gsmi as G
    from paper_2605_13794_amd import scenes as S
    from paper_2605_13794_amd.raster import Adam, DEFAULT_LRS, DeviceScene, Frame, l1_loss, rasterize
    t0 = time.time()
    sc = layout(S.city_scene(n, seed=3), args)
    ds = DeviceScene(sc, "cuda:0", requires_grad=True)
    del sc
    log(f"5M scene ready in {time.time() - t0:.1f}s")
    dev = torch.device("cuda:0")
    cams = [S.aerial_camera(args.width, args.height, h) for h in (0.0, 90.0, 180.0, 270.0)]
    targets = torch.stack([torch.from_numpy(S.target_image(args.width, args.height, seed=10 + k)) for k in
                           range(4)]).to(dev)
    res = {}
    for mode, store in (("recompute", False), ("stored_chain", True)):
        fr = Frame(cams, n, dev, store_chain=store)
        fr.forward(G.scene(*[p.detach() for p in ds.params()], lod=ds.lod), check=True)
        fr.ensure_capacity(int(int(fr.n_pairs.item()) * 1.25) + 4096)
        opt = Adam(ds.params(), DEFAULT_LRS)

        def step():
            imgs = rasterize(fr, ds)
            loss = l1_loss(imgs, targets)
            loss.backward()
            opt.step([p.grad for p in ds.params()], clear_grads=True)

        for _ in range(warmup):
            step()
        torch.cuda.synchronize()
        torch.cuda.reset_peak_memory_stats()
        t0 = time.perf_counter()
        for _ in range(steps):
            step()
        torch.cuda.synchronize()
        sec = (time.perf_counter() - t0) / steps
        res[mode] = {"it_per_s": 1 / sec, "ms_per_step": 1e3 * sec,
                     "mpix_per_s": 4 * args.width * args.height / 1e6 / sec,
                     "peak_allocated_gib": torch.cuda.max_memory_allocated() / 2**30,
                     "pairs": int(fr.n_pairs.item()), "steps": steps}
        del fr, opt
        for p in ds.params():
            p.grad = None
        torch.cuda.empty_cache()
    return {"workload": f"aerial city {n} Gaussians, batch of 4 {args.width}x{args.height} views, RasterizeFn + "
                        f"L1 + Adam", **res}


def run_cfg4(args):
    import torch
    n = args.n if args.n != (1 << 20) else (5 << 20)
    res = batch4_leg(args, n=n, steps=args.steps, warmup=args.warmup)
    torch.cuda.synchronize()
    out = {"metric": METRIC, "value": res["recompute"]["it_per_s"], "unit": "it/s", "dtype": "f32",
           "data": "synthetic", "config": {"workload": res.pop("workload")}, **res}
    print(json.dumps(finite(out), allow_nan=False), flush=True)


def host_cpu():
    """CPU model and logical CPU count of the host."""
    model = platform.processor() or "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count()
    return model, os.cpu_count(), avail


def cpu_baseline(scene, cam, sweep_cams, min_seconds=15.0):
    """The float64 reference (test infrastructure) timed on the host: its
    compiled compositing loops on all OpenMP threads (OMP_NUM_THREADS, else
    every available CPU) and its float64 projection on as many torch threads.
    As on the GPU, the score mask comes from an untimed importance sweep over
    the same 8 views; then whole steps of the workload run until min_seconds
    have passed."""
    import numpy as np
    import torch

    import oracle
    model, n_cpu, n_avail = host_cpu()
    threads = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or n_avail
    os.environ.setdefault("OMP_NUM_THREADS", str(threads))
    torch.set_num_threads(threads)
    oracle.build()
    omp = oracle.num_threads()
    S = __import__("paper_2605_13794_amd.scenes", fromlist=["x"])
    tgt = S.target_image(cam.width, cam.height, seed=1)
    arrays = scene.arrays()
    t0 = time.perf_counter()
    st = oracle.ImportanceState(scene.n, len(sweep_cams) + 1)
    for v, c in enumerate(sweep_cams):
        oracle.importance_view(arrays, c, st, v)
    keep = oracle.score_keep(st.score, oracle.drop_count(scene.n, 0.4))
    keep_bits = oracle.pack_bits(keep)
    sweep_s = time.perf_counter() - t0
    log(f"reference sweep of {len(sweep_cams)} views on {omp} threads: {sweep_s:.1f}s")

    def one_step():
        # importance refresh of the training view
        info = oracle.importance_view(arrays, cam, st, len(sweep_cams))
        gate, _ = oracle.lod_gate_radius(scene.mean, scene.log_scale, cam.position, cam.fx, 0.5)
        act = oracle.active_set(gate, keep_bits, 0.95)
        sub = scene.subset(act)
        r = oracle.forward_backward(sub.arrays(), cam, target=tgt)
        lrs = (1.6e-4, 5e-3, 1e-3, 5e-2, 2.5e-3)
        for (k, g), lr in zip(r["grads"].items(), lrs):
            p = sub.arrays()[k]
            oracle.adam_step(p, g, np.zeros_like(g), np.zeros_like(g), lr, 1)
        return r, info

    t0 = time.perf_counter()
    steps = 0
    while True:
        r, info = one_step()
        steps += 1
        if time.perf_counter() - t0 >= min_seconds:
            break
    dt = time.perf_counter() - t0
    return dict(value=steps / dt, unit="it/s", cores=omp, kind="oracle",
                sample=f"{steps} full steps ({scene.n} Gaussians, {cam.width}x{cam.height}: importance refresh, "
                       f"gate with the score mask of an untimed 8-view reference sweep ({sweep_s:.1f} s), "
                       f"projection, sort, compositing, L1, backward, Adam) in {dt:.1f} s on {omp} threads",
                seconds=dt, threads_compositing=omp, threads_torch=torch.get_num_threads(), nproc=n_cpu,
                cpus_available=n_avail, cpu_model=model, pairs=int(r["K"]), imp_pairs=int(info["K"]))


def serving(args, ds):
    """Continuous-batching server over the resident city: Poisson arrivals at
    200 requests/s, resolutions uniform over {640x360, 1280x720, 1920x1080,
    3840x2160}, random aerial poses.  Latency runs from arrival to the
    completion of the request's batch on the device clock (its completion
    event).  A second, saturating trace (6,000 requests offered at 4,000/s)
    measures the served capacity."""
    import torch

    from paper_2605_13794_amd import scenes as S
    from paper_2605_13794_amd.serve import GpuExecutor, Request, Scheduler, percentile, serve
    pool = 16 << 30

    def run(rate, seconds, warmup, seed):
        total = warmup + seconds
        n_req = int(total * rate * 1.2) + 16
        trace = [(t, cam) for t, cam in S.serving_requests(n_req, rate_hz=rate, seed=seed) if t < total]
        reqs = [Request(rid=i, arrival=t, cam=cam) for i, (t, cam) in enumerate(trace)]
        ex = GpuExecutor(ds, n_slots=3, max_batch=8)
        sch = Scheduler(n_slots=3, max_batch=8, memory_budget=pool, pairs_per_px=2.0)
        serve([Request(rid=-1, arrival=0.0, cam=trace[0][1])], ex, sch)
        torch.cuda.synchronize()
        done, _ = serve(reqs, ex, sch)
        meas = [r for r in done if r.arrival >= warmup]
        lat = [1e3 * r.latency for r in meas]
        seen = [1e3 * (r.t_seen - r.arrival) for r in meas]
        mpix = sum(r.pixels for r in meas) / 1e6
        span = max(r.t_done for r in meas) - min(r.arrival for r in meas)
        by_res = {}
        for r in meas:
            by_res.setdefault(f"{r.cam.width}x{r.cam.height}", []).append(1e3 * r.latency)
        out = {"requests": len(meas), "offered_req_per_s": rate, "measured_s": seconds,
               "p50_ms": percentile(lat, 50), "p99_ms": percentile(lat, 99), "mean_ms": sum(lat) / len(lat),
               "p50_p99_ms_by_resolution": {k: [percentile(v, 50), percentile(v, 99)] for k, v in
                                            sorted(by_res.items())},
               "p99_ms_host_observed": percentile(seen, 99), "mpix_per_s": mpix / span,
               "served_req_per_s": len(meas) / span, "batches": sch.n_batches,
               "retries": sum(r.retries for r in done)}
        del ex
        torch.cuda.empty_cache()
        return out

    res = run(200.0, args.serve_seconds, args.serve_warmup, 6)
    res.update({"memory_pool_gib": pool / 2**30, "gaussians": ds.n, "slots": 3, "max_batch": 8,
                "latency_clock": "device completion event"})
    sat = run(4000.0, 1.5, 0.0, 7)
    res["saturation"] = {k: sat[k] for k in ("requests", "offered_req_per_s", "mpix_per_s", "served_req_per_s",
                                            "p50_ms", "p99_ms", "batches")}
    return res


def run_serve(args):
    import torch

    from paper_2605_13794_amd import scenes as S
    from paper_2605_13794_amd.raster import DeviceScene
    sc = layout(S.city_scene(args.serve_n, seed=5), args)
    ds = DeviceScene(sc, "cuda:0")
    del sc
    res = serving(args, ds)
    torch.cuda.synchronize()
    print(json.dumps(finite({"metric": METRIC, "config": {"workload": f"serving over aerial city {ds.n} "
                                                                     f"Gaussians"}, "serving": res}),
                     allow_nan=False), flush=True)


def copy_calibration():
    """A plain copy of 1 GiB (reads 1 GiB, writes 1 GiB), five times, for
    scaling the HBM byte counters of the profiler."""
    import torch
    src = torch.empty(1 << 28, dtype=torch.float32, device="cuda:0").fill_(1.0)
    dst = torch.empty_like(src)
    for _ in range(5):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": src.numel() * 4, "reps": 5}), flush=True)


def roofline(b, name, reps, args):
    """Roofline entry of kernel `name`: its average launch duration over `reps`
    steps (HIP events around its own launches) against its algorithmic work
    per launch."""
    torch = b.torch
    if name == "adam":
        kms = b.kernel_time(name, b.step, reps)
        floats = sum(int(p.numel()) for p in b.ds.params())
        nbytes = ADAM_BYTES_PER_FLOAT * floats
        achieved = nbytes / (kms * 1e-3) / 1e9
        return dict(bound="hbm", achieved=achieved, peak=PEAK_HBM_GBS, unit="GB/s", frac=achieved / PEAK_HBM_GBS,
                    traffic=recorded_traffic(name, args), kernel=name, ms=kms, bytes_per_launch=nbytes,
                    floats=floats, bytes_per_float=ADAM_BYTES_PER_FLOAT)
    if name == "render_bwd":
        # algorithmic work of each timed launch, read right after its step from
        # the gated frame's lists and forward outputs (which that backward used)
        G = b.G
        a2 = torch.empty(b.n, dtype=torch.int32, device=b.dev)
        w2, s2 = torch.empty(b.n, device=b.dev), torch.zeros(b.n, device=b.dev)
        c2 = torch.zeros(b.n, dtype=torch.int32, device=b.dev)
        cull2 = torch.zeros((b.n + 31) // 32, dtype=torch.int32, device=b.dev)

        def work():
            last_sum = int(b.fr.last[0].to(torch.int64).sum().item())
            G.gs_importance(b.fr.proj[0].struct(), b.camc, b.n, b.fr.vals, b.fr.ranges, 0.99, 1e-6, w2, a2, s2, c2,
                            c2.clone(), cull2, b.ws_imp)
            composited = int(a2.to(torch.int64).sum().item())
            return last_sum, composited, int(b.fr.n_pairs.item())

        ms, counts = b.kernel_time(name, b.step, reps, after_each=work)
        ops = [ALPHA_OPS * ls + BWD_COMPOSITED_OPS * cp for ls, cp, _ in counts]
        achieved = sum(ops) / (sum(ms) * 1e-3) / 1e12
        return dict(bound="alu", achieved=achieved, peak=PEAK_ALU_GOPS / 1e3, unit="TOP/s",
                    frac=achieved / (PEAK_ALU_GOPS / 1e3), traffic=recorded_traffic(name, args), kernel=name,
                    ms=sum(ms) / reps, launches=reps, positions=sum(c[0] for c in counts) // reps,
                    composited=sum(c[1] for c in counts) // reps,
                    pairs_min_max=[min(c[2] for c in counts), max(c[2] for c in counts)],
                    ops_per_position=ALPHA_OPS, ops_per_composited=BWD_COMPOSITED_OPS,
                    counted="per timed launch, from that launch's own lists and forward outputs")
    kms = b.kernel_time(name, b.step, reps)
    return dict(bound="hbm", achieved=None, peak=PEAK_HBM_GBS, unit="GB/s", frac=None, traffic=None,
                kernel=name, ms=kms)


def main():
    args = parse()
    if args.copy_calibration:
        return copy_calibration()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (the library has no multi-GPU path); got --gpus {args.gpus}",
              file=sys.stderr)
        sys.exit(2)
    if args.config == "cfg3":
        return run_cfg3(args)
    if args.config == "cfg4":
        return run_cfg4(args)
    if args.config == "serve":
        return run_serve(args)
    b = Bench(args)
    torch = b.torch
    b.sweep()
    K_all, K = b.size_buffers()
    log(f"pairs: whole shard {K_all}, gated {K}")
    step_fn = b.graphed(b.step) if args.graph else b.step
    sec = b.timed(step_fn, args.steps, args.warmup)
    b.check_capacity()
    act_frac = int(b.n_act.item()) / b.n
    log(f"active fraction {act_frac:.3f}")
    log(f"step {sec * 1e3:.3f} ms")
    px = args.width * args.height
    extras = {}
    if not args.quick:
        g_ms = 1e3 * b.timed(lambda: b.train_iter(True), args.steps, 2)
        p_ms = 1e3 * b.timed(lambda: b.train_iter(False), args.steps, 2)
        extras["train_iteration"] = {
            "what": "one fwd+bwd training iteration on the 1080p view (gate, projection, sort, compositing, L1, "
                    "backward, Adam), without the importance refresh",
            "gated": {"ms": g_ms, "it_per_s": 1e3 / g_ms, "mpix_per_s": px / 1e3 / g_ms},
            "plain": {"ms": p_ms, "it_per_s": 1e3 / p_ms, "mpix_per_s": px / 1e3 / p_ms}}
        extras["importance_view_ms"] = 1e3 * b.timed(
            lambda: b.importance_view(b.fr_all, b.camc, b.sweep_views), args.steps, 2)
        b.check_capacity()
        extras["psnr_gated_vs_plain_db"] = b.psnr_gated_vs_plain()
    # roofline entries: live HIP-event timing inside the same process
    reps = max(5, min(args.steps, 20))
    roof = roofline(b, args.kernel, reps, args)
    roof_blend = roofline(b, "render_bwd", reps, args) if args.kernel != "render_bwd" else None
    pairs = int(b.fr.n_pairs.item())
    out = {
        "metric": METRIC,
        "value": 1.0 / sec,
        "unit": "it/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": sec * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "launch": "hip graph replay" if args.graph else "eager",
        "step": "one pass of the whole hot path on the view: its importance refresh (projection, sort, importance "
                "blend, top-99% mass, fold) on a second stream beside the gated training iteration (gate with "
                "the score mask, projection, sort, compositing, L1, backward, Adam)",
        "config": {"workload": f"aerial city {b.n} Gaussians, one {args.width}x{args.height} view per step: "
                               f"importance refresh + gated (r>={args.rmin}px, drop {args.drop:.0%} by score) "
                               f"fwd+bwd L1 + Adam",
                   "gaussians": b.n, "width": args.width, "height": args.height, "views_per_step": 1,
                   "layout": args.layout},
        "mpix_per_s": px / 1e6 / sec,
        "active_fraction": act_frac,
        "pairs_gated": pairs,
        "pairs_plain": int(b.fr_all.n_pairs.item()),
        "roofline": roof,
    }
    if roof_blend is not None:
        out["roofline_blend"] = roof_blend
    out.update(extras)
    del b
    torch.cuda.empty_cache()
    ds8 = None
    if not args.quick or args.serve_seconds > 0:
        from paper_2605_13794_amd import scenes as S
        from paper_2605_13794_amd.raster import DeviceScene
        t0 = time.time()
        sc8 = layout(S.city_scene(args.serve_n, seed=5), args)
        ds8 = DeviceScene(sc8, "cuda:0")
        mean8 = sc8.mean
        del sc8
        log(f"8M scene ready in {time.time() - t0:.1f}s")
    if not args.quick:
        log("active-set leg (64-view importance sweep, gates, gated vs plain) ...")
        out["active_set_8M"] = active_set_leg(ds8, mean8, args)
        torch.cuda.empty_cache()
        log("batch of four views on 5M (recompute vs stored chain) ...")
        out["batch4_5M"] = batch4_leg(args)
        torch.cuda.empty_cache()
    if args.serve_seconds > 0:
        log("serving trace ...")
        out["serving"] = serving(args, ds8)
    del ds8
    torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        log("timing the CPU reference ...")
        from paper_2605_13794_amd import scenes as S
        out["cpu_baseline"] = cpu_baseline(layout(S.city_scene(args.n, seed=2), args),
                                           S.aerial_camera(args.width, args.height),
                                           [S.aerial_camera(args.width, args.height, heading_deg=45.0 * v)
                                            for v in range(8)])
    print(json.dumps(finite(out), allow_nan=False), flush=True)


if __name__ == "__main__":
    main()
