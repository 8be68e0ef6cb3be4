"""Batched multi-view training step and its autotuner.

A training step over V views of one cell (paper Sec. 4.4 batches views;
on one GPU the views of a batch share the device): every view is rendered,
compared with its target image (L1), back-propagated, and the views'
parameter gradients are summed before one Adam update.

Batched form: the views are cut into groups of `batch`; each group runs one
preprocess launch for all its views, a sort per view, one render launch and
one render-backward launch over the group's (view, tile) work items, and
the views' parameter gradients summed in view order.  Plain form: the
per-view calls one view after another.  Both forms give bit-identical
images, and the same screen-space and parameter gradients: the render
backward has no atomics and the views' gradients are added in view order.

Per-instance buffers (instance values, sort workspace, backward rows) are
the bulk of the memory; groups run one after another on one stream, so all
groups share one arena sized for the largest group.  Capacities come from a
counting pass at set-up plus a margin; `check()` verifies that no view
overflowed.
"""
from __future__ import annotations

import itertools
import time
from dataclasses import dataclass
from typing import List, Optional, Sequence

import torch

from . import binding as B
from .pipeline import BatchedViews, CellView, GaussianParams, run_on_streams

_ALIGN = 256


def _align(n: int) -> int:
    return (n + _ALIGN - 1) // _ALIGN * _ALIGN


def count_instances(view: CellView) -> tuple:
    """(visible, instances) of a view: preprocess plus a counting sort call
    into a zero capacity (nothing is emitted)."""
    view.preprocess()
    try:
        B.sx_sort(view.c_proj, view.params.n, view.c_cam, view.c_par, 0, None, view.vals,
                  view.ranges, view.ws, sync_counts=True)
        return (0, 0)
    except B.SplaxelError as e:
        if e.code != B.SX_ECAPACITY:
            raise
    c = B.sx_sort_counts(view.ws, view.params.n)
    return (c[0], c[1])


class MultiViewStep:
    def __init__(self, params: GaussianParams, grads: GaussianParams, cams: Sequence, targets,
                 settings, batch: int = 16, plain: bool = False, margin: float = 1.1,
                 device="cuda"):
        self.params, self.grads = params, grads
        self.settings = settings
        self.plain = plain
        self.batch = 1 if plain else int(batch)
        self.views = [CellView(params, c, settings, capacity=0, device=device) for c in cams]
        self.targets = list(targets)
        self.counts = [count_instances(v) for v in self.views]
        self.margin = margin
        self.caps = [int(inst * margin) + 4096 for _, inst in self.counts]
        self.groups = [list(range(i, min(i + self.batch, len(cams))))
                       for i in range(0, len(cams), self.batch)]
        self._build_arena(device)
        self.box = [_Box()]
        self.batches = [BatchedViews.from_views([self.views[i] for i in g]) for g in self.groups]
        # the batched form overlaps the views' independent sorts and losses
        self.side = None if plain else [torch.cuda.Stream(device=device) for _ in range(4)]
        self.adam_m = [torch.zeros_like(t) for t in params.tensors()]
        self.adam_v = [torch.zeros_like(t) for t in params.tensors()]
        self.t = 0
        self.blends = None
        self.regrown = 0  # arena rebuilds after views came near their capacity

    def _build_arena(self, device):
        """One arena for the per-instance buffers of the largest group; the
        groups run one after another and reuse it."""
        need = 0
        layout = {}
        for g in self.groups:
            off = 0
            for i in g:
                v, cap = self.views[i], self.caps[i]
                parts = (4 * cap, v.sort_bytes(cap), v.backward_bytes(cap))
                layout[i] = (off, parts)
                off += sum(_align(p) for p in parts)
            need = max(need, off)
        self.arena_bytes = need
        self.arena = torch.empty((max(need, 1),), dtype=torch.uint8, device=device)
        for i, (off, (nv, ns, nb)) in layout.items():
            a = self.arena
            vals = a[off:off + nv].view(torch.int32)
            off += _align(nv)
            ws = a[off:off + ns]
            off += _align(ns)
            bw = a[off:off + nb]
            self.views[i].bind_instance_buffers(self.caps[i], vals, ws, bw)
        for v in self.views:
            v.ensure_backward_buffers()
            if getattr(v, "out", None) is None:
                v.out = torch.empty_like(v.partial)

    def _watch_counts(self):
        """The previous step's instance counts, posted by its asynchronous
        sorts (their copies are normally complete by the time the host
        enqueues the next step).  A view that overflowed raises: that step
        rendered a truncated list.  Views that came within 5% of their
        capacity (the Gaussians move and grow during training) get larger
        buffers before this step."""
        grow = []
        for i, v in enumerate(self.views):
            vis, inst, over = v.poll_counts()
            self.counts[i] = (vis, inst)
            if over:
                raise RuntimeError(f"view {i}: {inst} instances overflowed its capacity "
                                   "in the previous step")
            if inst * 1.05 > self.caps[i]:
                grow.append(i)
        if grow:
            torch.cuda.synchronize()  # the old arena may still be in use on side streams
            for i in grow:
                self.caps[i] = int(self.counts[i][1] * self.margin) + 4096
            self.arena = None
            self._build_arena(self.views[0].device)
            self.regrown += 1

    @property
    def n_views(self):
        return len(self.views)

    def _loss_and_grad(self, v: CellView, target):
        # composition, L1 and composition backward in one pass (bit-identical
        # to sx_composite, sx_l1_loss and sx_composite_backward)
        B.sx_composite_l1([v.partial], self.box, v.c_cam, v.c_par, target, v.out, None, None,
                          [v.dpartial])

    def run(self, lr: float = 1e-4, count_blends: bool = False, check: bool = False):
        """One step; with check, synchronises after each group and raises if
        any view's instances overflowed its capacity.  Without, the counts
        of this step are read at the start of the next one."""
        if self.t > 0 and not check:
            self._watch_counts()
        blends = 0
        if self.plain:
            for t in self.grads.tensors():
                B.sx_fill_u32(t, 0)
            for i, v in enumerate(self.views):
                v.preprocess()
                v.sort(sync=False)
                v.render(None, want_nblend=count_blends)
                self._loss_and_grad(v, self.targets[i])
                v.render_backward(v.dpartial)
                v.preprocess_backward(self.grads, accumulate=True)
                if check:
                    self._check([i])
                if count_blends:
                    blends += int(v.nblend.sum().item())
        else:
            for g, bv in zip(self.groups, self.batches):
                bv.preprocess()
                bv.sort(sync=False, streams=self.side)
                bv.render(want_nblend=count_blends)
                run_on_streams(self.side, [lambda i=i: self._loss_and_grad(self.views[i],
                                                                           self.targets[i])
                                           for i in g])
                bv.render_backward()
                # the first group overwrites the gradients, later ones add
                bv.preprocess_backward(self.grads, accumulate=g is not self.groups[0])
                if check:
                    self._check(g)
                if count_blends:
                    blends += sum(int(self.views[i].nblend.sum().item()) for i in g)
        self.t += 1
        for p, gr, m, vv in zip(self.params.tensors(), self.grads.tensors(), self.adam_m,
                                self.adam_v):
            B.sx_adam(p, gr, m, vv, self.t, lr)
        if count_blends:
            self.blends = blends
        return blends

    def _check(self, group):
        for i in group:
            vis, inst, over = self.views[i].poll_counts()
            if over or inst > self.caps[i]:
                raise RuntimeError(f"view {i}: {inst} instances overflow capacity {self.caps[i]}")


class _Box:
    lo = (-1e30,) * 3
    hi = (1e30,) * 3


@dataclass
class TuneResult:
    tile: str
    batch: int
    ms: float


def time_step(step: MultiViewStep, reps: int = 3, warmup: int = 1, lr: float = 1e-7) -> float:
    for _ in range(warmup):
        step.run(lr)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        step.run(lr)
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def autotune(params: GaussianParams, grads: GaussianParams, cams, targets, make_settings,
             tiles=("16x16", "32x8", "16x32"), batches=(2, 4, 8, 16),
             mem_budget: Optional[int] = None, reps: int = 2, log=None) -> List[TuneResult]:
    """Time one batched step per (tile shape, batch size) that fits the
    memory budget (bytes of free device memory if None) and return the
    results sorted fastest first.  The parameters are restored after each
    trial, so tuning leaves no trace in the model."""
    saved = [t.clone() for t in params.tensors()]
    out = []
    for tile, b in itertools.product(tiles, batches):
        tw, th = (int(x) for x in tile.split("x"))
        st = make_settings(tw, th)
        try:
            step = MultiViewStep(params, grads, cams, targets, st, batch=b)
        except torch.cuda.OutOfMemoryError:
            if log:
                log(f"autotune: tile {tile} batch {b}: out of memory")
            torch.cuda.empty_cache()
            continue
        budget = mem_budget if mem_budget is not None else torch.cuda.mem_get_info()[0]
        if step.arena_bytes > budget:
            del step
            continue
        ms = time_step(step, reps=reps)
        out.append(TuneResult(tile, b, ms))
        if log:
            log(f"autotune: tile {tile} batch {b}: {ms:.2f} ms/step")
        del step
        for t, s in zip(params.tensors(), saved):
            t.copy_(s)
        torch.cuda.empty_cache()
    out.sort(key=lambda r: r.ms)
    return out


# ------------------------------------------------------------------ K > 1 --
def bucket_views(participants: Sequence[set]) -> List[List[int]]:
    """Conflict-free view bucketing (Sec. 4.4, view consolidation): the
    views in order, each put into the first bucket whose cells are disjoint
    from its participant cells (that bucket then holds those cells too), or
    into a new bucket when every existing one conflicts.  Views in a bucket
    never touch the same cell."""
    buckets: List[List[int]] = []
    used: List[set] = []
    for v, parts in enumerate(participants):
        for b, u in zip(buckets, used):
            if not (u & parts):
                b.append(v)
                u |= parts
                break
        else:
            buckets.append([v])
            used.append(set(parts))
    return buckets


def item_struct(v: CellView, mask, n: int, backward: bool) -> B.SxView:
    """One (view, cell) work item of a batched launch."""
    s = B.SxView()
    s.cam = v.c_cam
    s.proj = v.c_proj
    s.vals = B.ptr(v.vals)
    s.tile_ranges = B.ptr(v.ranges)
    s.sort_ws = B.ptr(v.ws)
    s.capacity = v.capacity
    s.mask = B.ptr(mask)
    s.partial = B.ptr(v.partial)
    s.depth = None
    s.last = B.ptr(v.last)
    s.nblend = B.ptr(v.nblend)
    s.n = n
    if backward:
        v.ensure_backward_buffers()
        s.dpartial = B.ptr(v.dpartial)
        s.g2d = B.ptr(v.g2d)
        s.bwd_ws = B.ptr(v.bwd_ws)
    return s


class BucketedCells:
    """K = 8-style training over V views of a scene split into K cells,
    scheduled by conflict-free view bucketing (Sec. 4.4).  A view's
    participants are the cells whose geometric visibility map is non-empty
    (sx_mask_counts of sx_visibility); views are bucketed so that the views
    of a bucket share no cell.  Per bucket: every (view, participant cell)
    item is projected and sorted (the sorts on side streams), one render
    launch covers all items' tiles, each view is composed with its L1 loss
    and composition backward (sx_composite_l1; a cell outside the view's
    participants holds the identity partial, rendered once with an empty
    mask), and one render-backward launch covers all items.  Finally every
    cell's parameter gradient sums its items over the views in view order
    (sx_preprocess_backward_multi).  Masks start from the geometric maps and
    are cleared by saturation, as in Frame.train_l1; the results equal the
    per-view frames' bit for bit."""

    def __init__(self, cells: Sequence[GaussianParams], boxes, cams, settings, margin=1.1,
                 streams: int = 4, device="cuda"):
        from .pipeline import Frame
        self.cells = list(cells)
        self.K = len(self.cells)
        self.frames = [Frame(self.cells, boxes, c, settings, device=device) for c in cams]
        self.c_par = self.frames[0].c_par
        counts = torch.empty((self.K,), dtype=torch.int32, device=device)
        self.participants = []
        for f in self.frames:
            f.init_masks(geometric=True)
            B.sx_mask_counts(f.masks, counts)
            self.participants.append({m for m, c in enumerate(counts.tolist()) if c > 0})
        self.buckets = bucket_views(self.participants)
        # size every item's buffers from one synchronous pass; cells outside a
        # view render the identity once (their masks are empty and stay so)
        for f in self.frames:
            f.forward(use_masks=True, sync=True)
            for v in f.views:
                v._alloc_sort(int(v.counts[1] * margin) + 4096)
                v.ensure_backward_buffers()
        self.margin = margin
        self.side = [torch.cuda.Stream(device=device) for _ in range(streams)] if streams else None
        need = 1
        for b in self.buckets:
            cams_b = [self.frames[vi].c_cam for vi, _ in self.items(b)]
            if cams_b:
                need = max(need, B.sx_multi_workspace_size(cams_b, self.c_par))
        self.ws = torch.empty((need,), dtype=torch.uint8, device=device)
        self.t = 0
        self.regrown = 0

    def items(self, views: Sequence[int]):
        return [(vi, m) for vi in views for m in sorted(self.participants[vi])]

    def _watch_counts(self):
        """The previous step's posted instance counts: an overflow raises;
        items within 5% of their capacity get larger buffers."""
        grow = []
        for f in self.frames:
            for m, v in enumerate(f.views):
                if v._counts_ev is None:
                    continue
                vis, inst, over = v.poll_counts()
                if over:
                    raise RuntimeError(f"cell {m}: {inst} instances overflowed its capacity")
                if inst * 1.05 > v.capacity:
                    grow.append((v, inst))
        if grow:
            torch.cuda.synchronize()
            for v, inst in grow:
                v._alloc_sort(int(inst * self.margin) + 4096)
                v.ensure_backward_buffers()
            self.regrown += 1

    def step(self, targets, grads: Sequence[GaussianParams], count_blends=False):
        """Forward, L1 against targets[view], backward of every view; the
        cells' gradients are overwritten with the sums.  Returns the blend
        count when asked (one read-back per item)."""
        if self.t > 0:
            self._watch_counts()
        blends = 0
        for b in self.buckets:
            items = self.items(b)
            jobs = []
            for vi, m in items:
                v = self.frames[vi].views[m]
                jobs.append(lambda v=v: (v.preprocess(), v.sort(sync=False)))
            run_on_streams(self.side, jobs)
            # the renders read a copy of the masks the compositions update
            for vi in b:
                f = self.frames[vi]
                if f._masks_fwd is None:
                    f._masks_fwd = torch.empty_like(f.masks)
                f._masks_fwd.copy_(f.masks)
            fwd = [item_struct(self.frames[vi].views[m], self.frames[vi]._masks_fwd[m],
                               self.cells[m].n, False) for vi, m in items]
            if fwd:
                B.sx_render_multi(fwd, self.c_par, self.ws)
            for vi in b:
                f = self.frames[vi]
                B.sx_composite_l1([v.partial for v in f.views], f.boxes, f.c_cam, f.c_par,
                                  targets[vi], f.out, f.masks, None,
                                  [v.dpartial for v in f.views])
            bwd = [item_struct(self.frames[vi].views[m], self.frames[vi]._masks_fwd[m],
                               self.cells[m].n, True) for vi, m in items]
            if bwd:
                B.sx_render_backward_multi(bwd, 0, self.c_par, self.ws)
            if count_blends:
                blends += sum(int(self.frames[vi].views[m].nblend.sum().item())
                              for vi, m in items)
        for m in range(self.K):
            its = [(vi, m) for vi in range(len(self.frames)) if m in self.participants[vi]]
            g = grads[m]
            if not its:
                for t in g.tensors():
                    B.sx_fill_u32(t, 0)
                continue
            for k in range(0, len(its), B.SX_MAX_VIEWS):
                chunk = its[k:k + B.SX_MAX_VIEWS]
                st = [item_struct(self.frames[vi].views[mm], self.frames[vi]._masks_fwd[mm],
                                  self.cells[mm].n, True) for vi, mm in chunk]
                B.sx_preprocess_backward_multi(self.cells[m].struct(), st, self.c_par,
                                               g.grad_struct(),
                                               B.SX_BWD_ACCUMULATE if k else 0)
        self.t += 1
        return blends
