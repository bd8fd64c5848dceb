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
# Algorithmic operations per Gaussian-pixel evaluation (see the design notes):
OPS_PER_EVAL = {"render_fwd": 16.0, "render_bwd": 47.0, "importance_blend": 14.0}


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
    ap.add_argument("--kernel", default="render_bwd", help="kernel timed for the roofline entry")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--quick", action="store_true", help="skip the plain/gated side measurements")
    return ap.parse_args()


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
        self.scene = S.city_scene(args.n, seed=2)
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
        self.grads_s = G.grads(*self.grads)
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

    def train_iter(self, gated: bool):
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
        self.adam.step(self.grads, clear_grads=True)

    def step(self):
        self.importance_view(self.fr_all, self.camc, self.sweep_views)
        self.train_iter(gated=True)

    # -- setup ---------------------------------------------------------------
    def size_buffers(self):
        """One checked pass per frame sizes the pair buffers (25% headroom)."""
        scn = self.ds.struct()
        self.fr_all.project(scn)
        K_all = self.fr_all.bin_sort(check=True)
        self.fr_all.ensure_capacity(int(K_all * 1.25) + 4096)
        self.gate()
        self.fr.project(scn, self.active, self.n, self.n_act)
        K = self.fr.bin_sort(check=True)
        self.fr.ensure_capacity(int(K * 1.25) + 4096)
        self.torch.cuda.synchronize()
        return K_all, K

    def check_capacity(self):
        for fr in (self.fr, self.fr_all):
            k = int(fr.n_pairs.item())
            if k < 0 or k > fr.capacity:
                raise RuntimeError(f"pair buffer overflow during timing: K={k} capacity={fr.capacity}")

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

    def kernel_time(self, name, fn, reps):
        """Average duration of kernel `name` over `reps` calls of fn, from HIP
        events recorded around the kernel itself on its own stream."""
        G = self.G
        evs = [(G.HipEvent(), G.HipEvent()) for _ in range(reps)]
        for e0, e1 in evs:
            G.gs_profile_kernel(name, e0.handle, e1.handle)
            fn()
        G.gs_profile_kernel(None)
        self.torch.cuda.synchronize()
        return sum(e0.elapsed_ms(e1) for e0, e1 in evs) / reps

    def psnr_gated_vs_plain(self):
        torch = self.torch
        scn = self.ds.struct()
        self.fr_all.forward(scn, check=False)
        self.gate()
        self.fr.forward(scn, self.active, self.n, self.n_act, check=False)
        torch.cuda.synchronize()
        mse = float(((self.fr.rgb[0] - self.fr_all.rgb[0]) ** 2).mean().item())
        return 10.0 * math.log10(1.0 / mse) if mse > 0 else float("inf")


def cpu_baseline(scene, cam):
    """The float64 reference (test infrastructure) timed on the host for one
    full step of the same workload, single-threaded."""
    import numpy as np
    import torch

    import oracle
    torch.set_num_threads(1)
    oracle.build()
    S = __import__("paper_2605_13794_amd.scenes", fromlist=["x"])
    tgt = S.target_image(cam.width, cam.height, seed=1)
    arrays = scene.arrays()
    t0 = time.perf_counter()
    # importance refresh of the view
    st = oracle.ImportanceState(scene.n, 1)
    info = oracle.importance_view(arrays, cam, st, 0)
    # gate + score mask (the sweep's score is replaced by this view's)
    keep = oracle.score_keep(st.score, oracle.drop_count(scene.n, 0.4))
    gate, _ = oracle.lod_gate_radius(scene.mean, scene.log_scale, cam.position, cam.fx, 0.5)
    act = oracle.active_set(gate, oracle.pack_bits(keep), 0.95)
    sub = scene.subset(act)
    r = oracle.forward_backward(sub.arrays(), cam, target=tgt)
    lrs = (1.6e-4, 5e-3, 1e-3, 5e-2, 2.5e-3)
    for (k, g), lr in zip(r["grads"].items(), lrs):
        p = sub.arrays()[k]
        oracle.adam_step(p, g, np.zeros_like(g), np.zeros_like(g), lr, 1)
    dt = time.perf_counter() - t0
    return dict(value=1.0 / dt, unit="it/s", cores=1, kind="oracle",
                sample=f"one full step ({scene.n} Gaussians, {cam.width}x{cam.height}: importance refresh, "
                       f"gate, projection, sort, compositing, L1, backward, Adam) in {dt:.1f} s on one "
                       f"{platform.processor() or 'host'} core", seconds=dt, pairs=int(r["K"]),
                imp_pairs=int(info["K"]))


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (this build has no multi-GPU path); got --gpus {args.gpus}",
              file=sys.stderr)
        sys.exit(2)
    b = Bench(args)
    torch = b.torch
    K_all, K = b.size_buffers()
    log(f"pairs: whole shard {K_all}, gated {K}")
    b.sweep()
    act_frac = int(b.n_act.item()) / b.n
    log(f"sweep done; active fraction {act_frac:.3f}")
    sec = b.timed(b.step, args.steps, args.warmup)
    b.check_capacity()
    log(f"step {sec * 1e3:.3f} ms")
    extras = {}
    if not args.quick:
        extras["gated_train_ms"] = 1e3 * b.timed(lambda: b.train_iter(True), args.steps, 2)
        extras["plain_train_ms"] = 1e3 * b.timed(lambda: b.train_iter(False), args.steps, 2)
        extras["importance_view_ms"] = 1e3 * b.timed(
            lambda: b.importance_view(b.fr_all, b.camc, b.sweep_views), args.steps, 2)
        b.check_capacity()
        extras["psnr_gated_vs_plain_db"] = b.psnr_gated_vs_plain()
    # dominant kernel: live HIP-event timing inside the same process
    name = args.kernel
    reps = max(5, min(args.steps, 20))
    kms = b.kernel_time(name, b.step, reps)
    # algorithmic work of one launch of that kernel on the gated frame
    last_sum = int(b.fr.last[0].to(torch.int64).sum().item())
    pairs = int(b.fr.n_pairs.item())
    if name in OPS_PER_EVAL:
        evals = last_sum
        achieved = evals * OPS_PER_EVAL[name] / (kms * 1e-3) / 1e12
        roof = dict(bound="alu", achieved=achieved, peak=PEAK_ALU_GOPS / 1e3, unit="TOP/s",
                    frac=achieved / (PEAK_ALU_GOPS / 1e3), traffic=None, kernel=name, ms=kms,
                    evals=evals, ops_per_eval=OPS_PER_EVAL[name])
    else:
        roof = dict(bound="hbm", achieved=None, peak=PEAK_HBM_GBS, unit="GB/s", frac=None, traffic=None,
                    kernel=name, ms=kms)
    px = args.width * args.height
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
        "config": {"workload": f"aerial city {b.n} Gaussians, one {args.width}x{args.height} view per step: "
                               f"importance refresh + gated (r>={args.rmin}px, drop {args.drop:.0%} by score) "
                               f"fwd+bwd L1 + Adam",
                   "gaussians": b.n, "width": args.width, "height": args.height, "views_per_step": 1},
        "mpix_per_s": px / 1e6 / sec,
        "active_fraction": act_frac,
        "pairs_gated": pairs,
        "pairs_plain": int(b.fr_all.n_pairs.item()),
        "roofline": roof,
    }
    out.update(extras)
    if "gated_train_ms" in extras:
        out["gated_train_it_per_s"] = 1e3 / extras["gated_train_ms"]
        out["plain_train_it_per_s"] = 1e3 / extras["plain_train_ms"]
    if not args.no_cpu_baseline:
        log("timing the CPU reference on one step ...")
        out["cpu_baseline"] = cpu_baseline(b.scene, b.cam)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
