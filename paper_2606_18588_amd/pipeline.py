"""One view over K cells on one GPU: per cell preprocess -> sort -> partial
render (Eq. 1-4), then composition (Eq. 5) and the backward (Eq. 6-7).

The paper gives every GPU one convex cell and exchanges partial pixels
between GPUs; here the K cells' partial buffers stay resident in HBM and the
composition reads them directly.  Buffers are torch tensors (device memory
and streams only); every step runs in libsplaxel's HIP kernels.
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import List, Optional, Sequence

import numpy as np
import torch

from . import binding as B


@dataclass
class GaussianParams:
    """One cell's Gaussian parameters on the GPU (FP32, SoA)."""

    means: torch.Tensor
    log_scales: torch.Tensor
    quats: torch.Tensor
    opacity_logits: torch.Tensor
    sh: torch.Tensor

    @classmethod
    def from_arrays(cls, means, log_scales, quats, opacity_logits, sh,
                    device="cuda") -> "GaussianParams":
        def t(a):
            return torch.as_tensor(np.ascontiguousarray(a, np.float32)).to(device)
        return cls(t(means), t(log_scales), t(quats), t(opacity_logits), t(sh))

    @classmethod
    def from_scene(cls, scene, device="cuda") -> "GaussianParams":
        return cls.from_arrays(scene.means, scene.log_scales, scene.quats,
                               scene.opacity_logits, scene.sh, device)

    @property
    def n(self) -> int:
        return int(self.means.shape[0])

    @property
    def sh_degree(self) -> int:
        return int(round(math.sqrt(self.sh.shape[1]))) - 1

    def tensors(self) -> List[torch.Tensor]:
        return [self.means, self.log_scales, self.quats, self.opacity_logits, self.sh]

    def zeros_like(self) -> "GaussianParams":
        return GaussianParams(*[torch.zeros_like(t) for t in self.tensors()])

    def struct(self) -> B.SxGaussians:
        return B.gaussians(*self.tensors())

    def grad_struct(self) -> B.SxGrads:
        return B.grads(*self.tensors())


def spatial_order(means: np.ndarray, bits: int = 10) -> np.ndarray:
    """Permutation that stores Gaussians in Morton (Z-curve) order of their
    means, quantised to 2^bits cells per axis over the bounding box.  The
    Gaussians one view sees then occupy few contiguous index ranges, so the
    projection and its backward read and write whole cache lines instead of
    one short row per line.  Rendering is unchanged (up to the index order of
    exactly equal depths)."""
    m = np.asarray(means, np.float64)
    lo, hi = m.min(0), m.max(0)
    q = ((m - lo) / np.maximum(hi - lo, 1e-30) * ((1 << bits) - 1)).astype(np.uint64)

    def spread(x):  # insert two zero bits between the low 10 bits
        x = (x | (x << np.uint64(16))) & np.uint64(0x030000FF)
        x = (x | (x << np.uint64(8))) & np.uint64(0x0300F00F)
        x = (x | (x << np.uint64(4))) & np.uint64(0x030C30C3)
        return (x | (x << np.uint64(2))) & np.uint64(0x09249249)
    code = spread(q[:, 0]) | (spread(q[:, 1]) << np.uint64(1)) | (spread(q[:, 2]) << np.uint64(2))
    return np.argsort(code, kind="stable")


_COUNT_STREAMS = {}


def _count_stream(device) -> torch.cuda.Stream:
    """A side stream per device for the copies of sort count words to the
    host, so that they overlap the render instead of following the sort on
    the caller's stream."""
    s = _COUNT_STREAMS.get(device)
    if s is None:
        s = _COUNT_STREAMS[device] = torch.cuda.Stream(device=device)
    return s


REPARTITION_THRESHOLD = 0.2  # the paper's trigger on N_max / mean(N) - 1


def imbalance(cells: Sequence["GaussianParams"]) -> float:
    """Load imbalance N_max / mean(N) - 1 of the cells' Gaussian counts."""
    return B.sx_imbalance([c.n for c in cells])


def repartition(cells: Sequence["GaussianParams"], K: int = None, states=None):
    """New KD-tree cells over all Gaussians of `cells` (the partition
    strategy of the paper's appendix), with every Gaussian's parameter rows
    (and the rows of `states`: per cell a list of tensors laid out like its
    parameter arrays, e.g. Adam moments) moved to its new cell on the
    device, keeping the Gaussians' relative order.  The means go to the host
    for the KD split (12 bytes per Gaussian); nothing else leaves the GPU.
    Returns (new cells, boxes as synth-style (lo, hi) tuples, new states)."""
    K = len(cells) if K is None else int(K)
    dev = cells[0].means.device
    means = torch.cat([c.means for c in cells]).cpu().numpy()
    boxes, cell_of = B.sx_kd_partition(means, K)
    dst_index, counts = B.sx_repartition_plan(cell_of, K)
    d_cell = torch.as_tensor(cell_of).to(dev)
    d_index = torch.as_tensor(dst_index).to(dev)
    src_counts = [c.n for c in cells]

    def move(src):  # src: one tensor per old cell, rows of equal width
        width = int(src[0][0].numel()) if src[0].shape[0] else int(np.prod(src[0].shape[1:]))
        out = [torch.empty((max(int(n), 1),) + tuple(src[0].shape[1:]), dtype=src[0].dtype,
                           device=dev) for n in counts]
        B.sx_move_rows(width, src, src_counts, out, d_cell, d_index)
        return [o[:int(n)] for o, n in zip(out, counts)]
    arrays = [move([getattr(c, name) for c in cells])
              for name in ("means", "log_scales", "quats", "opacity_logits", "sh")]
    new_cells = [GaussianParams(*[arrays[a][k] for a in range(5)]) for k in range(K)]
    new_states = None
    if states is not None:
        moved = [move([st[j] for st in states]) for j in range(len(states[0]))]
        new_states = [[moved[j][k] for j in range(len(moved))] for k in range(K)]
    return new_cells, boxes, new_states


def tiles_of(cam, settings):
    tx = (cam.width + settings.tile_w - 1) // settings.tile_w
    ty = (cam.height + settings.tile_h - 1) // settings.tile_h
    return tx, ty


class CellView:
    """Buffers and steps for one (cell, view) pair."""

    def __init__(self, params: GaussianParams, cam, settings, capacity=None,
                 keep_keys=False, flags=0, device="cuda"):
        self.params = params
        self.cam = cam
        self.settings = settings
        self.flags = flags
        self.device = device
        n = params.n
        self.tiles_x, self.tiles_y = tiles_of(cam, settings)
        self.tiles = self.tiles_x * self.tiles_y
        self.H, self.W = cam.height, cam.width
        self.c_cam = B.camera(cam)
        self.c_par = B.params(settings, params.sh_degree, flags)
        self.c_g = params.struct()
        self.rec = torch.empty((max(n, 1), 12), dtype=torch.float32, device=device)
        self.rect = torch.empty((max(n, 1), 4), dtype=torch.int16, device=device)
        self.n_tiles = torch.empty((max(n, 1),), dtype=torch.int32, device=device)
        self.block_sums = torch.empty((B.sx_preprocess_blocks(n) * 2,), dtype=torch.int32,
                                      device=device)
        self.c_proj = B.projected(self.rec, self.rect, self.n_tiles, self.block_sums)
        # per tile [start, end), plus the one spare range the sort may write
        self.ranges = torch.empty((self.tiles + 1, 2), dtype=torch.int32, device=device)
        self.keep_keys = keep_keys
        self.counts = None
        # pinned copy of the sort workspace's count words {visible,
        # instances, overflow, error}, posted after every asynchronous sort
        self._h_counts = None
        self._counts_ev = None
        self._alloc_sort(capacity if capacity is not None else max(1024, 4 * n))
        hw = self.H * self.W
        self.partial = torch.empty((self.H, self.W, 4), dtype=torch.float32, device=device)
        self.last = torch.empty((self.H, self.W), dtype=torch.int32, device=device)
        self.nblend = torch.empty((self.H, self.W), dtype=torch.int32, device=device)
        self.depth = None
        self.g2d = None
        self.dpartial = None
        self.mask = None
        self._hw = hw
        self.xf = None  # cross-boundary filter bits, when the filter is on

    def set_cross_filter(self, boxes=None, cell: int = 0, omega=None):
        """Remove this cell's cross-boundary Gaussians from the rays where
        both cells are visible (omega: the view's K geometric maps from
        sx_visibility, kept alive by the caller); omega None turns it off.
        The bits are recomputed by every preprocess."""
        if omega is None:
            self.xf = None
            B.set_cross_filter(self.c_proj, None, None, 0, 0)
            return
        self.xf = torch.empty((max(self.params.n, 1),), dtype=torch.int32, device=self.device)
        self._xf_boxes, self._xf_cell, self._omega = list(boxes), int(cell), omega
        B.set_cross_filter(self.c_proj, self.xf, omega, cell, len(self._xf_boxes))

    def _wait_count_copy(self):
        # a posted copy of the count words may still read the workspace
        if self._counts_ev is not None:
            self._counts_ev.synchronize()

    def _alloc_sort(self, capacity: int):
        self._wait_count_copy()
        self.capacity = int(capacity)
        self.vals = torch.empty((max(self.capacity, 1),), dtype=torch.int32, device=self.device)
        self.keys = (torch.empty((max(self.capacity, 1),), dtype=torch.int64, device=self.device)
                     if self.keep_keys else None)
        self.ws = torch.empty((self.sort_bytes(self.capacity),), dtype=torch.uint8,
                              device=self.device)
        self.bwd_ws = None

    def sort_bytes(self, capacity: int) -> int:
        return B.sx_sort_workspace_size(self.params.n, capacity, self.tiles_x, self.tiles_y)

    def backward_bytes(self, capacity: int) -> int:
        return B.sx_backward_workspace_size(capacity, self.tiles)

    def bind_instance_buffers(self, capacity: int, vals, ws, bwd_ws=None):
        """Use caller-owned per-instance buffers (e.g. slices of an arena
        shared by views that are not in flight together)."""
        if ws.numel() < self.sort_bytes(capacity) or vals.numel() < max(capacity, 1):
            raise ValueError("instance buffers too small for the capacity")
        if bwd_ws is not None and bwd_ws.numel() < self.backward_bytes(capacity):
            raise ValueError("backward workspace too small for the capacity")
        self._wait_count_copy()
        self.capacity = int(capacity)
        self.vals, self.ws, self.bwd_ws = vals, ws, bwd_ws
        self.keys = None

    # ---------------------------------------------------------------- steps
    def preprocess(self):
        B.sx_preprocess(self.c_g, self.c_cam, self.c_par, self.c_proj)
        if self.xf is not None:
            B.sx_cross_filter(self.c_g, self.c_proj, self._xf_boxes, self._xf_cell, self.c_cam,
                              self.xf)

    def sort(self, sync=True):
        """With sync, reads the instance count back once and grows the
        buffers when they are too small; without, sorts asynchronously into
        the current capacity and posts an asynchronous copy of the count
        words (read them with poll_counts once the stream got that far)."""
        if self._counts_ev is not None:
            # the previous sort's count copy reads the words this sort clears
            torch.cuda.current_stream().wait_event(self._counts_ev)
        if not sync:
            B.sx_sort(self.c_proj, self.params.n, self.c_cam, self.c_par, self.capacity,
                      self.keys, self.vals, self.ranges, self.ws, sync_counts=False)
            self.post_counts()
            return None
        try:
            self.counts = B.sx_sort(self.c_proj, self.params.n, self.c_cam, self.c_par,
                                    self.capacity, self.keys, self.vals, self.ranges, self.ws,
                                    sync_counts=True)
        except B.SplaxelError as e:
            if e.code != B.SX_ECAPACITY:
                raise
            need = B.sx_sort_counts(self.ws, self.params.n)[1]
            self._alloc_sort(int(need * 1.25) + 1024)
            self.counts = B.sx_sort(self.c_proj, self.params.n, self.c_cam, self.c_par,
                                    self.capacity, self.keys, self.vals, self.ranges, self.ws,
                                    sync_counts=True)
        return self.counts

    def post_counts(self):
        """Enqueue a copy of the last sort's count words into pinned host
        memory, on a side stream after the current stream's sort."""
        if self._h_counts is None:
            self._h_counts = torch.zeros((4,), dtype=torch.int64, pin_memory=True)
            self._counts_ev = torch.cuda.Event()
        main = torch.cuda.current_stream()
        side = _count_stream(main.device)
        ready = torch.cuda.Event()
        ready.record(main)
        side.wait_event(ready)
        with torch.cuda.stream(side):
            self._h_counts.copy_(self.ws[:32].view(torch.int64), non_blocking=True)
            self._counts_ev.record(side)

    def poll_counts(self):
        """(visible, instances, overflow) of the last asynchronous sort; waits
        for its count copy.  The fourth count word (reserved for a sort that
        could not complete; the current sort always leaves it 0) raises when
        set."""
        if self._counts_ev is None:
            raise RuntimeError("no asynchronous sort posted its counts")
        self._counts_ev.synchronize()
        vis, inst, over, err = (int(x) for x in self._h_counts.tolist())
        if err:
            raise RuntimeError("sx_sort: the error count word is set; the instance list of "
                               "this view must not be used")
        return vis, inst, over

    def render(self, mask=None, want_depth=False, want_nblend=True):
        self.mask = mask
        if want_depth and self.depth is None:
            self.depth = torch.empty((self.H, self.W), dtype=torch.float32, device=self.device)
        B.sx_render_partial(self.c_proj, self.vals, self.ranges, self.c_cam, self.c_par, mask,
                            self.partial, self.depth if want_depth else None, self.last,
                            self.nblend if want_nblend else None)
        return self.partial

    def ensure_backward_buffers(self):
        if self.g2d is None:
            self.g2d = torch.empty((max(self.params.n, 1), 12), dtype=torch.float32,
                                   device=self.device)
            self.dpartial = torch.empty((self.H, self.W, 4), dtype=torch.float32,
                                        device=self.device)
        if self.bwd_ws is None:
            self.bwd_ws = torch.empty((self.backward_bytes(self.capacity),), dtype=torch.uint8,
                                      device=self.device)

    def render_backward(self, dpartial, ddepth=None, walk_events=None):
        """With walk_events (a list), the three stages are called one by one
        and a (start, end) pair of timing events around the reverse walk is
        appended to it."""
        self.ensure_backward_buffers()
        if walk_events is None:
            B.sx_render_backward(self.c_proj, self.vals, self.ranges, self.ws, self.params.n,
                                 self.capacity, self.bwd_ws, self.c_cam, self.c_par, self.mask,
                                 self.partial, self.last, dpartial, ddepth, self.g2d)
            return self.g2d
        ev = (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
        for stage in (B.SX_RB_PREPARE, B.SX_RB_WALK, B.SX_RB_REDUCE):
            if stage == B.SX_RB_WALK:
                ev[0].record()
            B.sx_render_backward_stages(self.c_proj, self.vals, self.ranges, self.ws,
                                        self.params.n, self.capacity, self.bwd_ws, self.c_cam,
                                        self.c_par, self.mask, self.partial, self.last,
                                        dpartial, ddepth, self.g2d, stage)
            if stage == B.SX_RB_WALK:
                ev[1].record()
        walk_events.append(ev)
        return self.g2d

    def preprocess_backward(self, grads: GaussianParams, accumulate=False):
        B.sx_preprocess_backward(self.c_g, self.c_cam, self.c_par, self.c_proj, self.ws,
                                 self.capacity, self.g2d, grads.grad_struct(),
                                 B.SX_BWD_ACCUMULATE if accumulate else 0)

    def state(self, grads: GaussianParams) -> B.SxCellState:
        """C struct for sx_backward; keeps the referenced structs alive."""
        self.ensure_backward_buffers()
        self._gs = grads.grad_struct()
        s = B.SxCellState()
        s.g = ctypes_pointer(self.c_g)
        s.proj = ctypes_pointer(self.c_proj)
        s.vals = B.ptr(self.vals)
        s.ranges = B.ptr(self.ranges)
        s.sort_ws = B.ptr(self.ws)
        s.capacity = self.capacity
        s.bwd_ws = B.ptr(self.bwd_ws)
        s.partial = B.ptr(self.partial)
        s.last = B.ptr(self.last)
        s.mask = B.ptr(self.mask) if self.mask is not None else None
        s.grads = ctypes_pointer(self._gs)
        s.g2d_ws = B.ptr(self.g2d)
        s.dpartial_ws = B.ptr(self.dpartial)
        return s


def run_on_streams(streams, jobs):
    """Run independent jobs (callables enqueueing device work) round-robin on
    `streams` after the current stream's earlier work; the current stream
    then waits for all of them (no streams: on the current stream).
    Returns the jobs' results."""
    if not streams:
        return [job() for job in jobs]
    main = torch.cuda.current_stream()
    ready = torch.cuda.Event()
    ready.record(main)
    for st in streams:
        st.wait_event(ready)
    out = []
    for k, job in enumerate(jobs):
        with torch.cuda.stream(streams[k % len(streams)]):
            out.append(job())
    for st in streams:
        done = torch.cuda.Event()
        done.record(st)
        main.wait_event(done)
    return out


def ctypes_pointer(obj):
    import ctypes
    return ctypes.pointer(obj)


class Frame:
    """One view of a scene split into K cells: forward and backward."""

    def __init__(self, cells: Sequence[GaussianParams], boxes, cam, settings,
                 flags=0, capacities=None, keep_keys=False, device="cuda",
                 cross_filter=False, streams=1):
        self.cross_filter = cross_filter
        # asynchronous forwards spread the cells' independent preprocess,
        # sort and render chains over this many streams (default priority)
        self.side = ([torch.cuda.Stream(device=device) for _ in range(streams)]
                     if streams > 1 else None)
        self.cells = list(cells)
        self.boxes = list(boxes)
        assert len(self.cells) == len(self.boxes)
        self.cam = cam
        self.settings = settings
        self.flags = flags
        sh_deg = self.cells[0].sh_degree
        self.views = [CellView(c, cam, settings,
                               None if capacities is None else capacities[k],
                               keep_keys, flags, device)
                      for k, c in enumerate(self.cells)]
        self.c_cam = B.camera(cam)
        self.c_par = B.params(settings, sh_deg, flags)
        self.out = torch.empty((cam.height, cam.width, 4), dtype=torch.float32, device=device)
        self.masks = None
        # the masks a forward rendered with (the composition may clear bits
        # of self.masks; the backward of that forward needs the old ones)
        self._masks_fwd = None
        self.omega = None   # geometric maps (re-evaluation, cross-boundary filter)
        self.budget = None  # [K, H*W] stale consumption of pruned pairs
        # a list to time every cell's reverse walk in (see CellView.render_backward)
        self.walk_events = None
        if cross_filter:
            self._set_omega(self._visibility())

    @property
    def K(self):
        return len(self.cells)

    def init_masks(self, geometric=False, reeval=False):
        """Every (cell, pixel) pair active, or with geometric, only the pairs
        where the cell's box is visible (sx_visibility); the composition
        then clears the pairs behind saturated prefixes.  With reeval the
        masks become the view's saturation state: pruned pairs keep their
        transmittance consumption and come back when the transmittance in
        front of them recovers (sx_composite_reeval)."""
        if geometric:
            vis = self.omega if self.omega is not None else self._visibility()
            self.masks = vis.clone()
            if reeval:
                self._set_omega(vis)
        else:
            self.masks = torch.empty_like(self._visibility_buffer())
            B.sx_fill_u32(self.masks, 0xFFFFFFFF)
        self.budget = (torch.zeros((self.K, self.cam.width * self.cam.height),
                                   dtype=torch.float32, device=self.out.device)
                       if reeval else None)
        return self.masks

    def _visibility_buffer(self):
        words = (self.cam.width * self.cam.height + 31) // 32
        return torch.empty((self.K, words), dtype=torch.int32, device=self.out.device)

    def _visibility(self):
        vis = self._visibility_buffer()
        B.sx_visibility(self.boxes, self.c_cam, vis)
        return vis

    def _set_omega(self, vis):
        self.omega = vis
        if self.cross_filter:
            for k, v in enumerate(self.views):
                v.set_cross_filter(self.boxes, k, vis)

    def forward(self, use_masks=False, update_masks=False, sync=True):
        """Render every cell (optionally restricted to the active mask bits
        from the previous render of this view) and compose them; with
        update_masks the composition clears the bits of saturated pairs, or,
        after init_masks(reeval=True), re-evaluates the view's state."""
        if update_masks and self.budget is not None and not use_masks:
            raise ValueError("re-evaluation needs the renders restricted to the masks")
        self._render_cells(use_masks, sync, update_masks)
        parts = [v.partial for v in self.views]
        if update_masks and self.budget is not None:
            B.sx_composite_reeval(parts, self.boxes, self.c_cam, self.c_par, self.out,
                                  self.masks, self.omega, self.budget)
        else:
            B.sx_composite(parts, self.boxes, self.c_cam, self.c_par, self.out,
                           self.masks if update_masks else None)
        if sync:
            self._raise_on_overflow(self.check_counts())
        return self.out

    def check_counts(self):
        """Reads every cell's posted sort counts (waiting for them) and
        returns the indices of the cells whose instances overflowed their
        capacity; raises if a sort's error word is set."""
        bad = []
        for k, v in enumerate(self.views):
            vis, inst, over = v.poll_counts()
            v.counts = (vis, inst)
            if over or inst > v.capacity:
                bad.append(k)
        return bad

    def _raise_on_overflow(self, bad):
        if bad:
            raise RuntimeError(f"cells {bad}: instances overflow the sort capacity")

    def forward_checked(self, use_masks=False, update_masks=False, headroom=1.25):
        """Asynchronous forward followed by one host synchronisation: the
        cells' count words are read back together, and cells whose
        instances overflowed are regrown (with `headroom`) and the view is
        rendered again, starting from the same masks and budgets."""
        saved = None
        if update_masks and self.masks is not None:
            saved = (self.masks.clone(), None if self.budget is None else self.budget.clone())
        for attempt in range(2):
            out = self.forward(use_masks, update_masks, sync=False)
            bad = self.check_counts()
            if not bad:
                return out
            for k in bad:
                v = self.views[k]
                v._alloc_sort(int(v.counts[1] * headroom) + 1024)
            if saved is not None:
                self.masks.copy_(saved[0])
                if saved[1] is not None:
                    self.budget.copy_(saved[1])
        self._raise_on_overflow(bad)

    def _render_cells(self, use_masks, sync, update_masks=False):
        side = self.side if (self.side is not None and not sync) else None
        main = torch.cuda.current_stream()
        masks = self.masks if use_masks else None
        if masks is not None and update_masks:
            # render from a copy: the composition is about to clear bits of
            # self.masks, and this forward's backward needs the bits it used
            if self._masks_fwd is None or self._masks_fwd.shape != masks.shape:
                self._masks_fwd = torch.empty_like(masks)
            self._masks_fwd.copy_(masks)
            masks = self._masks_fwd
        if side is not None:
            ready = torch.cuda.Event()
            ready.record(main)
            for s in side:
                s.wait_event(ready)
        for k, v in enumerate(self.views):
            m = masks[k] if masks is not None else None
            with torch.cuda.stream(side[k % len(side)] if side is not None else main):
                v.preprocess()
                v.sort(sync=sync)
                if sync:
                    v.post_counts()
                v.render(m)
        if side is not None:
            for s in side:
                done = torch.cuda.Event()
                done.record(s)
                main.wait_event(done)

    def train_l1(self, target, grads: Sequence[GaussianParams], accumulate=False,
                 use_masks=False, update_masks=False, sync=True, loss_sum=None):
        """One training pass of the view against an L1 target: every cell
        rendered, composed with the L1 loss and its composition backward in
        one pass (sx_composite_l1; the saturation masks follow the clearing
        rule), then every cell's backward.  The same results as forward,
        sx_l1_loss and backward; re-evaluating frames use those instead."""
        if self.budget is not None:
            raise ValueError("re-evaluating frames compose with forward()")
        self._render_cells(use_masks, sync, update_masks)
        for v in self.views:
            v.ensure_backward_buffers()
        B.sx_composite_l1([v.partial for v in self.views], self.boxes, self.c_cam, self.c_par,
                          target, self.out, self.masks if update_masks else None, loss_sum,
                          [v.dpartial for v in self.views])
        self._cells_backward(grads, accumulate)
        if sync:
            self._raise_on_overflow(self.check_counts())
        return self.out

    def backward(self, dout, grads: Sequence[GaussianParams], accumulate=False):
        if self.side is None:
            states = [v.state(g) for v, g in zip(self.views, grads)]
            B.sx_backward(states, self.boxes, self.c_cam, self.c_par, dout,
                          B.SX_BWD_ACCUMULATE if accumulate else 0)
            return
        # the same calls as sx_backward, with the cells' render and
        # projection backwards on the side streams (cell k always on stream
        # k mod n, so its gradient accumulations keep their order)
        for v in self.views:
            v.ensure_backward_buffers()
        B.sx_composite_backward([v.partial for v in self.views], self.boxes, self.c_cam,
                                self.c_par, dout, [v.dpartial for v in self.views])
        self._cells_backward(grads, accumulate)

    def _cells_backward(self, grads, accumulate):
        """Every cell's render and projection backward from its dpartial."""
        if self.side is None:
            for v, g in zip(self.views, grads):
                v.render_backward(v.dpartial, walk_events=self.walk_events)
                v.preprocess_backward(g, accumulate)
            return
        main = torch.cuda.current_stream()
        ready = torch.cuda.Event()
        ready.record(main)
        for s in self.side:
            s.wait_event(ready)
        for k, (v, g) in enumerate(zip(self.views, grads)):
            with torch.cuda.stream(self.side[k % len(self.side)]):
                v.render_backward(v.dpartial)
                v.preprocess_backward(g, accumulate)
        for s in self.side:
            done = torch.cuda.Event()
            done.record(s)
            main.wait_event(done)


class BatchedViews:
    """V views of one cell stepped together: one preprocess launch for all
    views, a sort per view, one render launch and one render-backward launch
    over all (view, tile) items, and the views' parameter gradients summed
    by the preprocess backward."""

    def __init__(self, params: GaussianParams, cams: Sequence, settings, capacities=None,
                 flags=0, device="cuda"):
        if not 1 <= len(cams) <= B.SX_MAX_VIEWS:
            raise ValueError(f"1..{B.SX_MAX_VIEWS} views per batch")
        self.params = params
        self.cams = list(cams)
        self.settings = settings
        self.views = [CellView(params, c, settings,
                               None if capacities is None else capacities[v], flags=flags,
                               device=device)
                      for v, c in enumerate(self.cams)]
        self.c_par = self.views[0].c_par
        self.c_cams = [v.c_cam for v in self.views]
        nb = B.sx_multi_workspace_size(self.c_cams, self.c_par)
        self.ws = torch.empty((nb,), dtype=torch.uint8, device=device)
        self.masks = [None] * len(self.views)

    @classmethod
    def from_views(cls, views: Sequence[CellView]) -> "BatchedViews":
        """Batch existing views of one cell (their buffers are used as is)."""
        if not 1 <= len(views) <= B.SX_MAX_VIEWS:
            raise ValueError(f"1..{B.SX_MAX_VIEWS} views per batch")
        self = cls.__new__(cls)
        self.params = views[0].params
        self.cams = [v.cam for v in views]
        self.settings = views[0].settings
        self.views = list(views)
        self.c_par = self.views[0].c_par
        self.c_cams = [v.c_cam for v in self.views]
        nb = B.sx_multi_workspace_size(self.c_cams, self.c_par)
        self.ws = torch.empty((nb,), dtype=torch.uint8, device=views[0].device)
        self.masks = [None] * len(self.views)
        return self

    @property
    def V(self):
        return len(self.views)

    def preprocess(self):
        B.sx_preprocess_multi(self.views[0].c_g, self.c_cams, self.c_par,
                              [v.c_proj for v in self.views])

    def sort(self, sync=True, streams=None):
        """Per-view sorts; asynchronous ones may be spread over `streams`
        (the views' sorts are independent; the caller's stream waits for
        all of them)."""
        if sync or not streams:
            return [v.sort(sync=sync) for v in self.views]
        return run_on_streams(streams, [lambda v=v: v.sort(sync=False) for v in self.views])

    def _structs(self, backward=False, want_nblend=True):
        out = []
        for v, m in zip(self.views, self.masks):
            s = B.SxView()
            s.cam = v.c_cam
            s.proj = v.c_proj
            s.vals = B.ptr(v.vals)
            s.tile_ranges = B.ptr(v.ranges)
            s.sort_ws = B.ptr(v.ws)
            s.capacity = v.capacity
            s.mask = B.ptr(m)
            s.partial = B.ptr(v.partial)
            s.depth = None
            s.last = B.ptr(v.last)
            s.nblend = B.ptr(v.nblend) if want_nblend else None
            if backward:
                v.ensure_backward_buffers()
                s.dpartial = B.ptr(v.dpartial)
                s.g2d = B.ptr(v.g2d)
                s.bwd_ws = B.ptr(v.bwd_ws)
            out.append(s)
        return out

    def render(self, masks=None, want_nblend=True):
        self.masks = list(masks) if masks is not None else [None] * self.V
        for v, m in zip(self.views, self.masks):
            v.mask = m
        B.sx_render_multi(self._structs(want_nblend=want_nblend), self.c_par, self.ws)
        return [v.partial for v in self.views]

    def render_backward(self):
        """Each view's upstream gradient must already be in view.dpartial."""
        B.sx_render_backward_multi(self._structs(backward=True), self.params.n, self.c_par,
                                   self.ws)

    def preprocess_backward(self, grads: GaussianParams, accumulate=False):
        """Sum of the views' parameter gradients in view order: written
        into grads (zero where no view sees a Gaussian), or added to them
        with accumulate."""
        self._gs = grads.grad_struct()
        B.sx_preprocess_backward_multi(self.views[0].c_g, self._structs(backward=True),
                                       self.c_par, self._gs,
                                       B.SX_BWD_ACCUMULATE if accumulate else 0)
