"""Serving form: one resident cell of Gaussians, view requests admitted by
the sort-buffer bytes they need, and continuous batching into batched
launches (the paper's view bucketing and overlapped pipeline, Sec. 4.4,
on one GPU).

Every request is one camera.  The server keeps up to `inflight` batches on
the GPU at once, each on its own stream with its own buffers, so that a
batch formed from requests that arrived while another ran overlaps it on
the device (continuous batching); a batch takes up to `max_batch` queued
requests in arrival order while their estimated sort buffers (instance
values + sort workspace) fit into the batch's arena of `arena_bytes`.  A
batch runs one preprocess launch for all its views, one asynchronous sort
per view into its arena slice (the sorts of a batch on side streams of its
own), one render launch over all (view, tile) work items and a composition
per view (K = 1: background under the residual transmittance); a batch of
one request takes the per-view calls, which give the same image.
Completion is seen on the host by polling the batch's event.  The instance
estimate is learned from completed requests; a request whose instances
overflow its estimate is re-queued at the front with the exact count.

With plain=True the loop serves one request at a time on one stream with
the per-view calls (sx_preprocess, sx_sort, sx_render_partial,
sx_composite): the baseline the batched form is measured against.

Buffers are torch tensors (device memory, pinned host memory, streams);
every step runs in libsplaxel's kernels.
"""
from __future__ import annotations

import collections
import math
import time
from dataclasses import dataclass, field
from typing import Dict, List, Optional, Sequence

import numpy as np
import torch

from . import binding as B
from .pipeline import GaussianParams, run_on_streams

_ALIGN = 256
_MAX_CAPACITY = (1 << 31) - 1  # largest instance capacity the sort accepts


def _align(n: int) -> int:
    return (n + _ALIGN - 1) // _ALIGN * _ALIGN


@dataclass
class Done:
    rid: int
    arrival_s: float
    done_s: float
    width: int
    height: int
    instances: int
    batch: int

    @property
    def latency_s(self) -> float:
        return self.done_s - self.arrival_s


class _Slot:
    """Per-view buffers of one batch position, sized for the largest view."""

    def __init__(self, n: int, max_px: int, max_tiles: int, device):
        self.rec = torch.empty((max(n, 1), 12), dtype=torch.float32, device=device)
        self.rect = torch.empty((max(n, 1), 4), dtype=torch.int16, device=device)
        self.n_tiles = torch.empty((max(n, 1),), dtype=torch.int32, device=device)
        self.block_sums = torch.empty((B.sx_preprocess_blocks(n) * 2,), dtype=torch.int32,
                                      device=device)
        self.c_proj = B.projected(self.rec, self.rect, self.n_tiles, self.block_sums)
        self.ranges = torch.empty(((max_tiles + 1) * 2,), dtype=torch.int32, device=device)
        self.partial = torch.empty((max_px * 4,), dtype=torch.float32, device=device)
        self.last = torch.empty((max_px,), dtype=torch.int32, device=device)
        self.out = torch.empty((max_px * 4,), dtype=torch.float32, device=device)


@dataclass
class _Item:
    rid: int
    arrival_s: float
    cam: object
    need: int = 0  # exact instance count once known (after an overflow)


@dataclass
class _Batch:
    index: int
    items: List[_Item]
    caps: List[int]
    event: object
    counts: torch.Tensor  # pinned [V, 4] uint64 as int64
    slots: List[_Slot]
    pixels: List[int]
    slot: int  # the in-flight slot (stream and buffers) it runs on


def slot_bytes(n: int, max_px: int, max_tiles: int) -> int:
    """Device bytes of one view slot (_Slot): the projection's per-Gaussian
    record, tile rectangle and tile count (60 B per Gaussian, indexed by
    Gaussian), its block sums, the tile ranges and three per-pixel buffers
    of the largest view."""
    return (60 * max(n, 1) + 8 * B.sx_preprocess_blocks(n) + 8 * (max_tiles + 1)
            + 36 * max_px)


def batch_width(max_batch: int, inflight: int, per_slot: int, budget: int) -> int:
    """Views per batch such that inflight x width slots fit `budget` bytes
    (at least 1, at most max_batch)."""
    fit = budget // max(per_slot * inflight, 1)
    return int(max(1, min(max_batch, fit)))


class Server:
    def __init__(self, params: GaussianParams, settings, max_width=3840, max_height=2160,
                 max_batch=16, inflight=2, arena_bytes=24 << 30, plain=False,
                 safety=1.15, slot_budget=None, device="cuda"):
        """slot_budget: device bytes the view slots of all in-flight batches
        may take (default: half the memory free once the arenas are set
        aside).  A slot holds the projection of the whole scene for one view,
        so on a large scene the budget, not max_batch, bounds the views per
        batch."""
        if not 1 <= max_batch <= B.SX_MAX_VIEWS:
            raise ValueError(f"max_batch must be in 1..{B.SX_MAX_VIEWS}")
        self.params = params
        self.settings = settings
        self.plain = plain
        if plain:
            inflight = 1
        # every in-flight batch has its own stream, side streams for its
        # sorts and workspaces, so batch k + 1 runs while batch k is on the
        # GPU (all streams at the default priority)
        self.streams = [torch.cuda.Stream(device=device) for _ in range(inflight)]
        self.side = (None if plain else
                     [[torch.cuda.Stream(device=device) for _ in range(4)]
                      for _ in range(inflight)])
        self.max_batch = 1 if plain else max_batch
        self.inflight = inflight
        self.arena_bytes = int(arena_bytes)
        self.safety = safety
        self.device = device
        self.n = params.n
        self.c_g = params.struct()
        self.c_par = B.params(settings, params.sh_degree, 0)
        self.max_w, self.max_h = max_width, max_height
        tx = (max_width + settings.tile_w - 1) // settings.tile_w
        ty = (max_height + settings.tile_h - 1) // settings.tile_h
        self.max_tiles = tx * ty
        per_slot = slot_bytes(self.n, max_width * max_height, self.max_tiles)
        if slot_budget is None:
            free, _ = torch.cuda.mem_get_info(device)
            slot_budget = max(0, free - inflight * self.arena_bytes) // 2
        self.slot_budget = int(slot_budget)
        self.max_batch = batch_width(self.max_batch, inflight, per_slot, self.slot_budget)
        self.slots = [[_Slot(self.n, max_width * max_height, self.max_tiles, device)
                       for _ in range(self.max_batch)] for _ in range(inflight)]
        self.arenas = [torch.empty((self.arena_bytes,), dtype=torch.uint8, device=device)
                       for _ in range(inflight)]
        self.counts = [torch.zeros((self.max_batch, 4), dtype=torch.int64, pin_memory=True)
                       for _ in range(inflight)]
        mw = B.sx_multi_workspace_size([B.camera(_dummy_cam(max_width, max_height))] *
                                       self.max_batch, self.c_par)
        self.multi_ws = [torch.empty((mw,), dtype=torch.uint8, device=device)
                         for _ in range(inflight)]
        self.box = [_Box()]
        self.ratio = None  # instances per pixel, learned
        self.recent = collections.deque(maxlen=64)
        self.overflows = 0
        self.images: Optional[Dict[int, torch.Tensor]] = None

    # ------------------------------------------------------------ estimate
    def calibrate(self, cam) -> None:
        """One synchronous sort of a representative view seeds the estimate of
        instances per pixel."""
        from .pipeline import CellView
        v = CellView(self.params, cam, self.settings)
        v.preprocess()
        vis, inst = v.sort(sync=True)
        self.ratio = inst / float(cam.width * cam.height)
        self.recent.append(self.ratio)

    def _estimate(self, it: _Item) -> int:
        px = it.cam.width * it.cam.height
        if it.need:
            return it.need
        r = max(self.recent) if self.recent else (self.ratio or 64.0)
        return min(int(math.ceil(r * px * self.safety)) + 4096, _MAX_CAPACITY)

    def _bytes(self, it: _Item, cap: int) -> int:
        tx, ty = _tile_grid(it.cam, self.settings)
        return _align(4 * cap) + _align(B.sx_sort_workspace_size(self.n, cap, tx, ty))

    # -------------------------------------------------------------- batches
    def _form(self, queue: collections.deque):
        items, caps, used = [], [], 0
        while queue and len(items) < self.max_batch:
            it = queue[0]
            if it.cam.width > self.max_w or it.cam.height > self.max_h:
                raise ValueError(f"request {it.rid}: view larger than the server's maximum")
            cap = self._estimate(it)
            nb = self._bytes(it, cap)
            if nb > self.arena_bytes:
                raise RuntimeError(f"request {it.rid} needs {nb} sort bytes > arena "
                                   f"{self.arena_bytes}")
            if used + nb > self.arena_bytes:
                break
            queue.popleft()
            items.append(it)
            caps.append(cap)
            used += nb
        return items, caps

    def _launch(self, k: int, index: int, items: List[_Item], caps: List[int]) -> _Batch:
        """Enqueue a batch on in-flight slot k's stream."""
        with torch.cuda.stream(self.streams[k]):
            return self._launch_on(k, index, items, caps)

    def _launch_on(self, k: int, index: int, items: List[_Item], caps: List[int]) -> _Batch:
        # one request alone takes the per-view calls (the same results as
        # the batched launches, bit for bit, with less overhead)
        single = self.plain or len(items) == 1
        slots = self.slots[k][:len(items)]
        arena = self.arenas[k]
        counts = self.counts[k]
        cams = [B.camera(it.cam) for it in items]
        projs = [s.c_proj for s in slots]
        if single:
            B.sx_preprocess(self.c_g, cams[0], self.c_par, projs[0])
        else:
            B.sx_preprocess_multi(self.c_g, cams, self.c_par, projs)
        off = 0
        views = []
        pixels = []
        bufs = []
        for it, cap in zip(items, caps):
            tx, ty = _tile_grid(it.cam, self.settings)
            wsb = B.sx_sort_workspace_size(self.n, cap, tx, ty)
            vals = arena[off:off + 4 * cap].view(torch.int32)
            off += _align(4 * cap)
            ws = arena[off:off + wsb]
            off += _align(wsb)
            bufs.append((vals, ws, tx * ty))

        def sort_job(j):
            vals, ws, tiles = bufs[j]
            s = slots[j]
            B.sx_sort(s.c_proj, self.n, cams[j], self.c_par, caps[j], None, vals,
                      s.ranges[:2 * (tiles + 1)], ws, sync_counts=False)
            counts[j].copy_(ws[:32].view(torch.int64), non_blocking=True)

        # the requests' sorts are independent: batched, they overlap on the
        # side streams (joined before the render)
        run_on_streams(None if single else self.side[k],
                       [lambda j=j: sort_job(j) for j in range(len(items))])
        for j, (it, cam, s, cap) in enumerate(zip(items, cams, slots, caps)):
            vals, ws, tiles = bufs[j]
            ranges = s.ranges[:2 * (tiles + 1)]
            px = it.cam.width * it.cam.height
            pixels.append(px)
            if single:
                B.sx_render_partial(s.c_proj, vals, ranges, cam, self.c_par, None,
                                    s.partial[:4 * px], None, s.last[:px], None)
            else:
                v = B.SxView()
                v.cam = cam
                v.proj = s.c_proj
                v.vals = B.ptr(vals)
                v.tile_ranges = B.ptr(ranges)
                v.sort_ws = B.ptr(ws)
                v.capacity = cap
                v.partial = B.ptr(s.partial)
                v.last = B.ptr(s.last)
                views.append(v)
        if not single:
            B.sx_render_multi(views, self.c_par, self.multi_ws[k])
        for it, cam, s, px in zip(items, cams, slots, pixels):
            B.sx_composite([s.partial[:4 * px]], self.box, cam, self.c_par, s.out[:4 * px], None)
        ev = torch.cuda.Event()
        ev.record()
        return _Batch(index, items, caps, ev, counts, slots, pixels, k)

    def _finish(self, b: _Batch, now: float, queue: collections.deque, done: List[Done]):
        requeue = []
        for j, (it, cap) in enumerate(zip(b.items, b.caps)):
            vis, inst, over, err = (int(x) for x in b.counts[j, :4])
            if err:
                raise RuntimeError(f"request {it.rid}: the sort's error word is set; its "
                                   "instance list must not be used")
            if over or inst > cap:
                if inst > _MAX_CAPACITY:
                    raise RuntimeError(f"request {it.rid}: {inst} instances exceed the sort's "
                                       f"limit of {_MAX_CAPACITY}")
                self.overflows += 1
                it.need = min(inst + 1024, _MAX_CAPACITY)
                requeue.append(it)
                continue
            self.recent.append(inst / float(b.pixels[j]))
            done.append(Done(it.rid, it.arrival_s, now, it.cam.width, it.cam.height, inst,
                             b.index))
            if self.images is not None:
                px = b.pixels[j]
                self.images[it.rid] = b.slots[j].out[:4 * px].view(
                    it.cam.height, it.cam.width, 4).clone()
        if self.images is not None:
            # the next batch on this slot's stream rewrites the images just
            # copied on the caller's stream: it waits for the copies
            self.streams[b.slot].wait_stream(torch.cuda.current_stream())
        for it in reversed(requeue):
            queue.appendleft(it)

    # ---------------------------------------------------------------- serve
    def serve(self, requests: Sequence, open_loop=True, keep_images=False,
              time_limit_s: float = 600.0) -> List[Done]:
        """Serve `requests` (objects with .arrival_s, .camera, .rid).  Open
        loop: a request joins the queue at its arrival time; closed loop:
        every request is queued at time zero.  Returns completions in the
        order they were seen."""
        self.images = {} if keep_images else None
        reqs = sorted(requests, key=lambda r: r.arrival_s)
        pending = collections.deque(
            _Item(r.rid, r.arrival_s if open_loop else 0.0, r.camera) for r in reqs)
        queue: collections.deque = collections.deque()
        running: List[Optional[_Batch]] = [None] * self.inflight
        done: List[Done] = []
        n_batches = 0
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        while len(done) < len(reqs):
            now = time.perf_counter() - t0
            if now > time_limit_s:
                raise TimeoutError(f"served {len(done)} of {len(reqs)} in {time_limit_s} s")
            while pending and pending[0].arrival_s <= now:
                queue.append(pending.popleft())
            progressed = False
            for k in range(self.inflight):
                b = running[k]
                if b is not None and b.event.query():
                    self._finish(b, time.perf_counter() - t0, queue, done)
                    running[k] = None
                    progressed = True
            for k in range(self.inflight):
                if running[k] is None and queue:
                    items, caps = self._form(queue)
                    if items:
                        running[k] = self._launch(k, n_batches, items, caps)
                        n_batches += 1
                        progressed = True
            if not progressed:
                if not queue and pending and all(r is None for r in running):
                    wait = pending[0].arrival_s - (time.perf_counter() - t0)
                    if wait > 2e-4:
                        time.sleep(wait - 1e-4)
                else:
                    time.sleep(0)
        self.n_batches = n_batches
        return done


def summarize(done: Sequence[Done], wall_s: Optional[float] = None) -> dict:
    lat = np.array([d.latency_s for d in done]) * 1e3
    t_end = max(d.done_s for d in done)
    t_begin = min(d.arrival_s for d in done)
    span = wall_s if wall_s is not None else (t_end - t_begin)
    return {"requests": len(done), "p50_ms": float(np.percentile(lat, 50)),
            "p99_ms": float(np.percentile(lat, 99)), "mean_ms": float(lat.mean()),
            "frames_per_s": len(done) / span if span > 0 else float("inf"),
            "batches": len({d.batch for d in done})}


class _Box:
    lo = (-1e30,) * 3
    hi = (1e30,) * 3


def _tile_grid(cam, settings):
    return ((cam.width + settings.tile_w - 1) // settings.tile_w,
            (cam.height + settings.tile_h - 1) // settings.tile_h)


@dataclass
class _DummyCam:
    width: int
    height: int
    R: tuple = (1, 0, 0, 0, 1, 0, 0, 0, 1)
    t: tuple = (0, 0, 0)
    fx: float = 1.0
    fy: float = 1.0
    cx: float = 0.0
    cy: float = 0.0
    znear: float = 0.2


def _dummy_cam(w, h):
    return _DummyCam(w, h)
