"""Continuous-batching render server over a scene resident in HBM.

Requests (novel views of mixed resolutions) arrive over time.  A scheduler
admits queued requests into batches as execution slots and memory free up:
each request is charged its tile-buffer memory (pair keys and values, tile
ranges and image buffers, from a running estimate of pairs per pixel), and a
batch starts only if the charge fits the memory pool.  A batch is one
projection of the scene into all its cameras (the scene is read once), one
sort over the concatenated tile space and one compositing launch over every
tile of every camera.  Several slots, each with its own HIP stream and
buffers, keep batches in flight concurrently, so requests that arrive while
others run overlap with them on the device.

The scheduler (`Scheduler`) is plain Python and runs without a GPU; the
executor (`GpuExecutor`) drives the C ABI.
"""
from __future__ import annotations

import collections
import dataclasses
import math
import time

PAIR_BYTES = 24          # u64 key + u32 value, plus the sort's ping-pong copy
PIXEL_BYTES = 20         # rgb (12) + final T (4) + last (4)


@dataclasses.dataclass
class Request:
    rid: int
    arrival: float
    cam: object
    t_start: float | None = None
    t_done: float | None = None
    t_seen: float | None = None
    pairs: int | None = None
    batch: int | None = None
    retries: int = 0

    @property
    def pixels(self) -> int:
        return int(self.cam.width) * int(self.cam.height)

    @property
    def latency(self) -> float | None:
        return None if self.t_done is None else self.t_done - self.arrival


class Scheduler:
    """Admission by tile-buffer memory and batching into free slots.

    memory_budget: bytes of the pool that pair buffers and images draw from.
    pairs_per_px: initial estimate of (Gaussian, tile) pairs per pixel, updated
    from completed batches (exponential average, kept an upper-biased margin).
    """

    def __init__(self, n_slots: int, max_batch: int, memory_budget: int, pairs_per_px: float = 2.0,
                 margin: float = 1.3):
        self.n_slots = n_slots
        self.max_batch = max_batch
        self.budget = int(memory_budget)
        self.ppx = float(pairs_per_px)
        self.margin = margin
        self.queue: collections.deque[Request] = collections.deque()
        self.in_use = 0
        self.free_slots = list(range(n_slots))
        self.running: dict[int, tuple[list[Request], int]] = {}
        self.n_batches = 0
        self.max_in_use = 0

    def charge(self, req: Request) -> int:
        return int(math.ceil(req.pixels * (self.ppx * self.margin * PAIR_BYTES + PIXEL_BYTES)))

    def capacity_for(self, reqs) -> int:
        return int(math.ceil(sum(r.pixels for r in reqs) * self.ppx * self.margin)) + 4096

    def submit(self, req: Request):
        self.queue.append(req)

    def next_batch(self):
        """Pops the next batch (FIFO) that fits the free memory, or None."""
        if not self.free_slots or not self.queue:
            return None
        batch, cost = [], 0
        while self.queue and len(batch) < self.max_batch:
            c = self.charge(self.queue[0])
            if self.in_use + cost + c > self.budget:
                # a request larger than the whole pool still runs alone
                if not batch and self.in_use == 0:
                    batch.append(self.queue.popleft())
                    cost += c
                break
            batch.append(self.queue.popleft())
            cost += c
        if not batch:
            return None
        slot = self.free_slots.pop(0)
        self.in_use += cost
        self.max_in_use = max(self.max_in_use, self.in_use)
        self.running[slot] = (batch, cost)
        self.n_batches += 1
        return slot, batch

    def finish(self, slot: int, pairs_total: int | None = None):
        batch, cost = self.running.pop(slot)
        self.in_use -= cost
        self.free_slots.append(slot)
        self.free_slots.sort()
        if pairs_total is not None and pairs_total > 0:
            px = sum(r.pixels for r in batch)
            self.ppx = max(0.7 * self.ppx + 0.3 * pairs_total / px, pairs_total / px)
        return batch

    def retry(self, slot: int, pairs_total: int):
        """The batch's pairs overflowed its capacity: release it and put its
        requests back at the head of the queue with a raised estimate."""
        batch, cost = self.running.pop(slot)
        self.in_use -= cost
        self.free_slots.append(slot)
        self.free_slots.sort()
        px = sum(r.pixels for r in batch)
        self.ppx = max(self.ppx, pairs_total / px * 1.05)
        for r in reversed(batch):
            r.retries += 1
            self.queue.appendleft(r)


class GpuExecutor:
    """Slots with their own stream and buffers; a batch is three library
    calls (gs_project, gs_bin_sort, gs_render_fwd) plus a completion event."""

    def __init__(self, dscene, n_slots: int, max_batch: int, device="cuda", bg=(0.0, 0.0, 0.0)):
        import torch

        from . import gsmi as G
        from .raster import ProjBuffers, Workspace
        self.torch, self.G = torch, G
        self.ds = dscene
        self.dev = torch.device(device)
        self.bg = bg
        self.n = dscene.n
        self.max_batch = max_batch
        self.slots = []
        for _ in range(n_slots):
            s = dict(stream=torch.cuda.Stream(device=self.dev),
                     proj=[ProjBuffers(self.n, self.dev) for _ in range(max_batch)],
                     ws=Workspace(self.dev), wsp=Workspace(self.dev), keys=None, vals=None, cap=0,
                     n_pairs=torch.zeros(1, dtype=torch.int64, device=self.dev),
                     ranges=None, event=None, batch=None, out=None)
            self.slots.append(s)

    def _ensure(self, s, cap, tiles):
        torch = self.torch
        if cap > s["cap"]:
            s["cap"] = int(cap)
            s["keys"] = torch.empty(s["cap"], dtype=torch.int64, device=self.dev)
            s["vals"] = torch.empty(s["cap"], dtype=torch.int32, device=self.dev)
        if s["ranges"] is None or s["ranges"].numel() < 2 * tiles:
            s["ranges"] = torch.empty(2 * tiles, dtype=torch.int32, device=self.dev)

    def launch(self, slot: int, batch, capacity: int):
        torch, G = self.torch, self.G
        s = self.slots[slot]
        cams = [r.cam for r in batch]
        tiles = sum(G.gs_num_tiles(c.width, c.height) for c in cams)
        self._ensure(s, min(capacity, G.GS_MAX_PAIRS - 1), tiles)
        carr = G.camera_array(cams)
        projs = [p.struct() for p in s["proj"][:len(cams)]]
        stream = s["stream"]
        with torch.cuda.stream(stream):
            out = [(torch.empty(3, c.height, c.width, device=self.dev),
                    torch.empty(c.height, c.width, device=self.dev),
                    torch.empty(c.height, c.width, dtype=torch.int32, device=self.dev)) for c in cams]
            wsp = s["wsp"].get(G.gs_workspace_size(G.GS_OP_PROJECT, self.n))
            G.gs_project(self.ds.struct(), None, self.n, None, carr, projs, wsp, stream)
            ws = s["ws"].get(G.gs_workspace_size(G.GS_OP_BIN_SORT, self.n, s["cap"], tiles, len(cams)))
            G.gs_bin_sort(projs, carr, self.n, s["keys"], s["vals"], s["cap"], s["ranges"], s["n_pairs"], ws,
                          stream)
            G.gs_render_fwd(projs, carr, s["vals"], s["ranges"], self.bg, [o[0] for o in out], [o[1] for o in out],
                            [o[2] for o in out], stream=stream)
            ev = torch.cuda.Event(enable_timing=True)
            ev.record(stream)
        s["event"], s["batch"], s["out"] = ev, batch, out

    def start_clock(self):
        """Records the reference event of device time stamps (after every
        earlier launch) and waits for it; returns nothing."""
        torch = self.torch
        self.ref = torch.cuda.Event(enable_timing=True)
        self.ref.record(torch.cuda.current_stream())
        self.ref.synchronize()

    def device_time(self, slot: int) -> float:
        """Seconds from the reference event to the completion event of the
        slot's batch, on the device clock."""
        return self.ref.elapsed_time(self.slots[slot]["event"]) / 1e3

    def done(self, slot: int) -> bool:
        ev = self.slots[slot]["event"]
        return ev is not None and ev.query()

    def pairs(self, slot: int) -> int:
        return int(self.slots[slot]["n_pairs"].item())

    def capacity(self, slot: int) -> int:
        return self.slots[slot]["cap"]

    def images(self, slot: int):
        return self.slots[slot]["out"]

    def copy_images(self, slot: int):
        """Copies of the slot's finished images, made on the slot's own stream
        (so they are ordered before the slot's next batch, which may reuse
        the memory of these outputs); the current stream then waits for them."""
        torch = self.torch
        s = self.slots[slot]
        with torch.cuda.stream(s["stream"]):
            copies = [o[0].clone() for o in s["out"]]
        cur = torch.cuda.current_stream()
        cur.wait_stream(s["stream"])
        for c in copies:
            c.record_stream(cur)
        return copies


def serve(requests, executor, scheduler: Scheduler, clock=time.perf_counter, keep_images=False, idle_sleep=0.0,
          max_retries: int = 8):
    """Runs the arrival trace (request.arrival in seconds from the start)
    through the scheduler and executor; returns the completed requests (with
    t_done set) and, if asked, their images keyed by request id.  A request
    whose batch still overflows its pair buffer after max_retries re-queues
    (pairs beyond the largest buffer the executor can give) raises
    RuntimeError.

    If the executor keeps device time stamps (start_clock / device_time),
    t_done is the completion of the request's batch on the device clock,
    mapped to the trace's clock at the moment the reference event completed;
    t_seen is when the host observed it."""
    pending = sorted(requests, key=lambda r: r.arrival)
    pi = 0
    done = []
    images = {}
    device_clock = hasattr(executor, "start_clock")
    if device_clock:
        executor.start_clock()
    t0 = clock()
    while len(done) < len(pending):
        now = clock() - t0
        while pi < len(pending) and pending[pi].arrival <= now:
            scheduler.submit(pending[pi])
            pi += 1
        # completions
        for slot in list(scheduler.running.keys()):
            if executor.done(slot):
                K = executor.pairs(slot)
                if K > executor.capacity(slot):
                    batch = scheduler.running[slot][0]
                    if max(r.retries for r in batch) >= max_retries:
                        raise RuntimeError(f"serve: a batch of {len(batch)} requests needs {K} pairs, more than "
                                           f"its buffer of {executor.capacity(slot)}, after {max_retries} retries")
                    scheduler.retry(slot, K)
                    continue
                t = clock() - t0
                t_dev = executor.device_time(slot) if device_clock else t
                batch = scheduler.finish(slot, K)
                imgs = executor.copy_images(slot) if keep_images else None
                for k, r in enumerate(batch):
                    r.t_done = t_dev
                    r.t_seen = t
                    r.pairs = K
                    done.append(r)
                    if keep_images:
                        images[r.rid] = imgs[k]
        # admissions
        while True:
            nb = scheduler.next_batch()
            if nb is None:
                break
            slot, batch = nb
            now = clock() - t0
            for r in batch:
                r.t_start = now
                r.batch = scheduler.n_batches
            executor.launch(slot, batch, scheduler.capacity_for(batch))
        if idle_sleep:
            time.sleep(idle_sleep)
    return done, images


def percentile(xs, q):
    xs = sorted(xs)
    if not xs:
        return float("nan")
    k = (len(xs) - 1) * q / 100.0
    f = math.floor(k)
    c = min(f + 1, len(xs) - 1)
    return xs[f] + (xs[c] - xs[f]) * (k - f)
