"""ctypes binding of libsplaxel.so (the C ABI in include/splaxel.h).

Argument marshalling only: every function here has the name of the C entry
point it calls, takes torch tensors that live on the GPU and passes their
device pointers and the current HIP stream.  There is no fallback: if the
HIP library is missing or a call fails, an exception is raised.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np
import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libsplaxel.so")

SX_OK = 0
SX_EINVAL = -1
SX_ECAPACITY = -2
SX_EDEVICE = -3
SX_FLAG_SAME_FRAME_CULL = 1
SX_BWD_ACCUMULATE = 1
SX_RB_PREPARE, SX_RB_WALK, SX_RB_REDUCE, SX_RB_ALL = 1, 2, 4, 7

c_f = ctypes.c_float
c_i32 = ctypes.c_int32
c_i64 = ctypes.c_int64
c_p = ctypes.c_void_p


class SxCamera(ctypes.Structure):
    _fields_ = [("R", c_f * 9), ("t", c_f * 3), ("fx", c_f), ("fy", c_f),
                ("cx", c_f), ("cy", c_f), ("width", c_i32), ("height", c_i32),
                ("znear", c_f)]


class SxParams(ctypes.Structure):
    _fields_ = [("tile_w", c_i32), ("tile_h", c_i32), ("sh_degree", c_i32),
                ("flags", c_i32), ("alpha_min", c_f), ("alpha_max", c_f),
                ("t_min", c_f), ("eps2d", c_f), ("bg", c_f * 3), ("fov_guard", c_f)]


class SxGaussians(ctypes.Structure):
    _fields_ = [("n", c_i64), ("means", c_p), ("log_scales", c_p),
                ("quats", c_p), ("opacity_logits", c_p), ("sh", c_p)]


class SxProjected(ctypes.Structure):
    _fields_ = [("rec", c_p), ("rect", c_p), ("n_tiles", c_p),
                ("block_sums", c_p), ("xf", c_p), ("omega", c_p),
                ("cell", ctypes.c_int32), ("n_cells", ctypes.c_int32)]


class SxCell(ctypes.Structure):
    _fields_ = [("lo", c_f * 3), ("hi", c_f * 3)]


class SxGrads(ctypes.Structure):
    _fields_ = [("means", c_p), ("log_scales", c_p), ("quats", c_p),
                ("opacity_logits", c_p), ("sh", c_p)]


class SxCellState(ctypes.Structure):
    _fields_ = [("g", ctypes.POINTER(SxGaussians)),
                ("proj", ctypes.POINTER(SxProjected)), ("vals", c_p),
                ("ranges", c_p), ("sort_ws", c_p), ("capacity", c_i64),
                ("partial", c_p), ("last", c_p),
                ("mask", c_p), ("grads", ctypes.POINTER(SxGrads)),
                ("g2d_ws", c_p), ("dpartial_ws", c_p), ("bwd_ws", c_p)]


class SxView(ctypes.Structure):
    _fields_ = [("cam", SxCamera), ("proj", SxProjected), ("vals", c_p),
                ("tile_ranges", c_p), ("sort_ws", c_p), ("capacity", c_i64),
                ("mask", c_p), ("partial", c_p), ("depth", c_p), ("last", c_p),
                ("nblend", c_p), ("dpartial", c_p), ("g2d", c_p), ("bwd_ws", c_p),
                ("n", c_i64)]


SX_MAX_VIEWS = 16

EXPORTS = (
    "sx_last_error_string", "sx_version", "sx_preprocess_blocks",
    "sx_preprocess", "sx_sort_workspace_size", "sx_sort", "sx_sort_counts",
    "sx_backward_workspace_size",
    "sx_render_partial", "sx_composite", "sx_l1_loss", "sx_backward",
    "sx_composite_backward", "sx_render_backward", "sx_preprocess_backward",
    "sx_adam", "sx_fill_u32", "sx_preprocess_multi", "sx_multi_workspace_size",
    "sx_render_multi", "sx_render_backward_multi", "sx_preprocess_backward_multi",
    "sx_render_backward_stages", "sx_visibility", "sx_kd_partition",
    "sx_composite_reeval", "sx_cross_filter", "sx_composite_l1",
    "sx_render_backward_noalloc", "sx_imbalance", "sx_repartition_plan", "sx_move_rows",
    "sx_mask_counts",
)
SX_NOALLOC_SCRATCH_BYTES = 64 << 20  # the static scratch of sx_render_backward_noalloc

_lib = None


class SplaxelError(RuntimeError):
    def __init__(self, fn: str, code: int, msg: str):
        super().__init__(f"{fn} failed ({code}): {msg}")
        self.code = code


def lib() -> ctypes.CDLL:
    """Load libsplaxel.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing: build it with "
                "`python -m paper_2606_18588_amd.build` (no CPU fallback "
                "exists)")
        L = ctypes.CDLL(LIB_PATH)
        L.sx_last_error_string.restype = ctypes.c_char_p
        L.sx_version.restype = ctypes.c_char_p
        L.sx_preprocess_blocks.restype = c_i64
        L.sx_preprocess_blocks.argtypes = [c_i64]
        for name in EXPORTS[3:]:
            getattr(L, name).restype = c_i32
        _lib = L
    return _lib


def _check(fn: str, code: int) -> int:
    if code != SX_OK:
        raise SplaxelError(fn, code, lib().sx_last_error_string().decode())
    return code


def ptr(t: Optional[torch.Tensor]):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("tensor must be on the GPU")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


def stream_handle(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


# --------------------------------------------------------------------------
# struct builders


def camera(cam) -> SxCamera:
    """Any object with R (3x3), t (3), fx, fy, cx, cy, width, height, znear."""
    c = SxCamera()
    R = [float(v) for v in np.asarray(cam.R, np.float32).reshape(9)]
    t = [float(v) for v in np.asarray(cam.t, np.float32).reshape(3)]
    for i in range(9):
        c.R[i] = R[i]
    for i in range(3):
        c.t[i] = t[i]
    c.fx, c.fy, c.cx, c.cy = float(cam.fx), float(cam.fy), float(cam.cx), float(cam.cy)
    c.width, c.height = int(cam.width), int(cam.height)
    c.znear = float(cam.znear)
    return c


def params(settings, sh_degree: int, flags: int = 0) -> SxParams:
    p = SxParams()
    p.tile_w, p.tile_h = int(settings.tile_w), int(settings.tile_h)
    p.sh_degree = int(sh_degree)
    p.flags = int(flags)
    p.alpha_min, p.alpha_max = float(settings.alpha_min), float(settings.alpha_max)
    p.t_min, p.eps2d = float(settings.t_min), float(settings.eps2d)
    for i in range(3):
        p.bg[i] = float(settings.bg[i])
    p.fov_guard = float(settings.fov_guard)
    return p


def gaussians(means, log_scales, quats, opacity_logits, sh) -> SxGaussians:
    g = SxGaussians()
    g.n = int(means.shape[0])
    g.means, g.log_scales, g.quats = ptr(means), ptr(log_scales), ptr(quats)
    g.opacity_logits, g.sh = ptr(opacity_logits), ptr(sh)
    return g


def projected(rec, rect, n_tiles, block_sums) -> SxProjected:
    p = SxProjected()
    p.rec, p.rect, p.n_tiles, p.block_sums = ptr(rec), ptr(rect), ptr(n_tiles), ptr(block_sums)
    return p


def grads(means, log_scales, quats, opacity_logits, sh) -> SxGrads:
    g = SxGrads()
    g.means, g.log_scales, g.quats = ptr(means), ptr(log_scales), ptr(quats)
    g.opacity_logits, g.sh = ptr(opacity_logits), ptr(sh)
    return g


def cells_array(cells: Sequence) -> ctypes.Array:
    arr = (SxCell * len(cells))()
    for k, c in enumerate(cells):
        for j in range(3):
            arr[k].lo[j] = float(c.lo[j])
            arr[k].hi[j] = float(c.hi[j])
    return arr


def ptr_array(ts: Sequence[torch.Tensor]):
    arr = (c_p * len(ts))()
    for k, t in enumerate(ts):
        arr[k] = ptr(t).value
    return arr


# --------------------------------------------------------------------------
# entry points (same names as the C ABI)


def sx_version() -> str:
    return lib().sx_version().decode()


def sx_preprocess_blocks(n: int) -> int:
    return int(lib().sx_preprocess_blocks(c_i64(n)))


def sx_preprocess(g: SxGaussians, cam: SxCamera, p: SxParams,
                  out: SxProjected, stream=None) -> None:
    _check("sx_preprocess", lib().sx_preprocess(
        ctypes.byref(g), ctypes.byref(cam), ctypes.byref(p), ctypes.byref(out),
        stream_handle(stream)))


def sx_sort_workspace_size(n: int, capacity: int, tiles_x: int, tiles_y: int) -> int:
    b = ctypes.c_size_t(0)
    _check("sx_sort_workspace_size", lib().sx_sort_workspace_size(
        c_i64(n), c_i64(capacity), c_i32(tiles_x), c_i32(tiles_y), ctypes.byref(b)))
    return int(b.value)


def sx_sort(proj: SxProjected, n: int, cam: SxCamera, p: SxParams,
            capacity: int, keys: Optional[torch.Tensor], vals: torch.Tensor,
            ranges: torch.Tensor, ws: torch.Tensor, sync_counts: bool = False,
            stream=None):
    """Returns (visible, instances) when sync_counts, else None."""
    hc = (ctypes.c_uint64 * 2)() if sync_counts else None
    code = lib().sx_sort(
        ctypes.byref(proj), c_i64(n), ctypes.byref(cam), ctypes.byref(p),
        c_i64(capacity), ptr(keys), ptr(vals), ptr(ranges), ptr(ws),
        ctypes.c_size_t(ws.numel() * ws.element_size()),
        hc if hc is not None else None, stream_handle(stream))
    _check("sx_sort", code)
    return (int(hc[0]), int(hc[1])) if hc is not None else None


def sx_sort_counts(ws: torch.Tensor, n: int, stream=None):
    out = (ctypes.c_uint64 * 4)()
    _check("sx_sort_counts", lib().sx_sort_counts(ptr(ws), c_i64(n), out,
                                                  stream_handle(stream)))
    return tuple(int(v) for v in out)


def sx_render_partial(proj: SxProjected, vals, ranges, cam: SxCamera,
                      p: SxParams, mask, partial, depth, last, nblend,
                      stream=None) -> None:
    _check("sx_render_partial", lib().sx_render_partial(
        ctypes.byref(proj), ptr(vals), ptr(ranges), ctypes.byref(cam),
        ctypes.byref(p), ptr(mask), ptr(partial), ptr(depth), ptr(last),
        ptr(nblend), stream_handle(stream)))


def sx_composite(partials: Sequence[torch.Tensor], cells, cam: SxCamera,
                 p: SxParams, out, masks, stream=None) -> None:
    _check("sx_composite", lib().sx_composite(
        c_i32(len(partials)), ptr_array(partials), cells_array(cells),
        ctypes.byref(cam), ctypes.byref(p), ptr(out), ptr(masks),
        stream_handle(stream)))


def sx_composite_reeval(partials: Sequence[torch.Tensor], cells, cam: SxCamera,
                        p: SxParams, out, masks, omega, budget, stream=None) -> None:
    _check("sx_composite_reeval", lib().sx_composite_reeval(
        c_i32(len(partials)), ptr_array(partials), cells_array(cells),
        ctypes.byref(cam), ctypes.byref(p), ptr(out), ptr(masks), ptr(omega),
        ptr(budget), stream_handle(stream)))


def sx_cross_filter(g: "SxGaussians", proj: SxProjected, cells, cell: int, cam: SxCamera,
                    xf, stream=None) -> None:
    _check("sx_cross_filter", lib().sx_cross_filter(
        ctypes.byref(g), ctypes.byref(proj), c_i32(len(cells)), cells_array(cells),
        c_i32(cell), ctypes.byref(cam), ptr(xf), stream_handle(stream)))


def set_cross_filter(proj: SxProjected, xf, omega, cell: int, n_cells: int) -> None:
    """Turn the per-ray cross-boundary filter of a projection on (xf None:
    off) for the render and backward calls that take it."""
    proj.xf = None if xf is None else ptr(xf)
    proj.omega = None if xf is None else ptr(omega)
    proj.cell = int(cell) if xf is not None else 0
    proj.n_cells = int(n_cells) if xf is not None else 0


def sx_composite_l1(partials: Sequence[torch.Tensor], cells, cam: SxCamera, p: SxParams,
                    target, out, masks, loss_sum, dpartials, stream=None) -> None:
    _check("sx_composite_l1", lib().sx_composite_l1(
        c_i32(len(partials)), ptr_array(partials), cells_array(cells), ctypes.byref(cam),
        ctypes.byref(p), ptr(target), ptr(out), ptr(masks), ptr(loss_sum),
        ptr_array(dpartials), stream_handle(stream)))


def sx_l1_loss(out, target, width: int, height: int, dout, loss_sum,
               stream=None) -> None:
    _check("sx_l1_loss", lib().sx_l1_loss(
        ptr(out), ptr(target), c_i32(width), c_i32(height), ptr(dout),
        ptr(loss_sum), stream_handle(stream)))


def sx_composite_backward(partials, cells, cam: SxCamera, p: SxParams, dout,
                          dpartials, stream=None) -> None:
    _check("sx_composite_backward", lib().sx_composite_backward(
        c_i32(len(partials)), ptr_array(partials), cells_array(cells),
        ctypes.byref(cam), ctypes.byref(p), None, ptr(dout),
        ptr_array(dpartials), stream_handle(stream)))


def sx_backward_workspace_size(capacity: int, tiles_total: int) -> int:
    b = ctypes.c_size_t(0)
    _check("sx_backward_workspace_size", lib().sx_backward_workspace_size(
        c_i64(capacity), c_i64(tiles_total), ctypes.byref(b)))
    return int(b.value)


def sx_render_backward(proj: SxProjected, vals, ranges, sort_ws, n: int,
                       capacity: int, bwd_ws, cam: SxCamera, p: SxParams,
                       mask, partial, last, dpartial, ddepth, g2d,
                       stream=None) -> None:
    _check("sx_render_backward", lib().sx_render_backward(
        ctypes.byref(proj), ptr(vals), ptr(ranges), ptr(sort_ws), c_i64(n),
        c_i64(capacity), ptr(bwd_ws), ctypes.byref(cam), ctypes.byref(p),
        ptr(mask), ptr(partial), ptr(last), ptr(dpartial), ptr(ddepth),
        ptr(g2d), stream_handle(stream)))


def sx_render_backward_noalloc(proj: SxProjected, vals, ranges, sort_ws, n: int,
                               capacity: int, cam: SxCamera, p: SxParams, mask, partial,
                               last, dpartial, ddepth, g2d, stream=None) -> None:
    """sx_render_backward with its scratch in the library's static device
    array (for callers that cannot allocate; calls on one device must not
    overlap)."""
    _check("sx_render_backward_noalloc", lib().sx_render_backward_noalloc(
        ctypes.byref(proj), ptr(vals), ptr(ranges), ptr(sort_ws), c_i64(n),
        c_i64(capacity), ctypes.byref(cam), ctypes.byref(p), ptr(mask), ptr(partial),
        ptr(last), ptr(dpartial), ptr(ddepth), ptr(g2d), stream_handle(stream)))


def sx_render_backward_stages(proj: SxProjected, vals, ranges, sort_ws, n: int,
                              capacity: int, bwd_ws, cam: SxCamera, p: SxParams,
                              mask, partial, last, dpartial, ddepth, g2d, stages: int,
                              stream=None) -> None:
    _check("sx_render_backward_stages", lib().sx_render_backward_stages(
        ctypes.byref(proj), ptr(vals), ptr(ranges), ptr(sort_ws), c_i64(n),
        c_i64(capacity), ptr(bwd_ws), ctypes.byref(cam), ctypes.byref(p),
        ptr(mask), ptr(partial), ptr(last), ptr(dpartial), ptr(ddepth),
        ptr(g2d), c_i32(stages), stream_handle(stream)))


def sx_preprocess_backward(g: SxGaussians, cam: SxCamera, p: SxParams,
                           proj: SxProjected, sort_ws, capacity: int, g2d,
                           gr: SxGrads, flags: int = 0, stream=None) -> None:
    _check("sx_preprocess_backward", lib().sx_preprocess_backward(
        ctypes.byref(g), ctypes.byref(cam), ctypes.byref(p), ctypes.byref(proj),
        ptr(sort_ws), c_i64(capacity), ptr(g2d), ctypes.byref(gr), c_i32(flags),
        stream_handle(stream)))


def sx_backward(states: Sequence[SxCellState], cells, cam: SxCamera,
                p: SxParams, dout, flags: int = 0, stream=None) -> None:
    arr = (SxCellState * len(states))(*states)
    _check("sx_backward", lib().sx_backward(
        c_i32(len(states)), arr, cells_array(cells), ctypes.byref(cam),
        ctypes.byref(p), ptr(dout), c_i32(flags), stream_handle(stream)))


def sx_kd_partition(means, K: int):
    """KD-tree cells of host means [n,3] (float32): returns (boxes as
    (lo, hi) tuples, cell_of int32 [n])."""
    import numpy as np
    m = np.ascontiguousarray(np.asarray(means, np.float32).reshape(-1, 3))
    n = m.shape[0]
    cells = (SxCell * K)()
    cell_of = np.zeros(n, np.int32)
    _check("sx_kd_partition", lib().sx_kd_partition(
        c_i64(n), m.ctypes.data_as(ctypes.c_void_p), c_i32(K), cells,
        cell_of.ctypes.data_as(ctypes.c_void_p)))
    boxes = [(tuple(c.lo), tuple(c.hi)) for c in cells]
    return boxes, cell_of


def sx_imbalance(counts) -> float:
    """N_max / mean(N) - 1 of the cells' Gaussian counts."""
    import numpy as np
    c = np.ascontiguousarray(np.asarray(counts, np.int64))
    r = ctypes.c_double()
    _check("sx_imbalance", lib().sx_imbalance(c_i32(len(c)), c.ctypes.data_as(ctypes.c_void_p),
                                              ctypes.byref(r)))
    return float(r.value)


def sx_repartition_plan(cell_of, K: int):
    """(dst_index int32 [n], counts int64 [K]) for the new cell of every
    Gaussian (host arrays)."""
    import numpy as np
    co = np.ascontiguousarray(np.asarray(cell_of, np.int32))
    dst = np.zeros(len(co), np.int32)
    counts = np.zeros(K, np.int64)
    _check("sx_repartition_plan", lib().sx_repartition_plan(
        c_i64(len(co)), co.ctypes.data_as(ctypes.c_void_p), c_i32(K),
        dst.ctypes.data_as(ctypes.c_void_p), counts.ctypes.data_as(ctypes.c_void_p)))
    return dst, counts


def sx_move_rows(row_floats: int, src: Sequence[torch.Tensor], src_counts,
                 dst: Sequence[torch.Tensor], dst_cell: torch.Tensor, dst_index: torch.Tensor,
                 stream=None) -> None:
    sc = (ctypes.c_int64 * len(src))(*[int(c) for c in src_counts])
    _check("sx_move_rows", lib().sx_move_rows(
        c_i32(row_floats), c_i32(len(src)), sc, ptr_array(src), c_i32(len(dst)),
        ptr_array(dst), ptr(dst_cell), ptr(dst_index), stream_handle(stream)))


def sx_mask_counts(masks: torch.Tensor, counts: torch.Tensor, stream=None) -> None:
    """counts[m] = set bits of row m of masks [K, words]."""
    K, words = masks.shape
    _check("sx_mask_counts", lib().sx_mask_counts(c_i32(K), ptr(masks), c_i64(words),
                                                  ptr(counts), stream_handle(stream)))


def sx_visibility(cells, cam: SxCamera, masks, stream=None) -> None:
    arr = cells_array(cells)
    _check("sx_visibility", lib().sx_visibility(c_i32(len(cells)), arr, ctypes.byref(cam),
                                                ptr(masks), stream_handle(stream)))


def sx_adam(param, grad, m, v, step: int, lr: float, beta1: float = 0.9,
            beta2: float = 0.999, eps: float = 1e-8, stream=None) -> None:
    _check("sx_adam", lib().sx_adam(
        c_i64(param.numel()), ptr(param), ptr(grad), ptr(m), ptr(v),
        c_i32(step), c_f(lr), c_f(beta1), c_f(beta2), c_f(eps),
        stream_handle(stream)))


def sx_fill_u32(t: torch.Tensor, value: int, stream=None) -> None:
    _check("sx_fill_u32", lib().sx_fill_u32(
        ptr(t), c_i64(t.numel() * t.element_size() // 4),
        ctypes.c_uint32(value & 0xFFFFFFFF), stream_handle(stream)))


def sx_preprocess_multi(g: SxGaussians, cams: Sequence[SxCamera], p: SxParams,
                        outs: Sequence[SxProjected], stream=None) -> None:
    ca = (SxCamera * len(cams))(*cams)
    oa = (SxProjected * len(outs))(*outs)
    _check("sx_preprocess_multi", lib().sx_preprocess_multi(
        ctypes.byref(g), c_i32(len(cams)), ca, ctypes.byref(p), oa,
        stream_handle(stream)))


def sx_multi_workspace_size(cams: Sequence[SxCamera], p: SxParams) -> int:
    ca = (SxCamera * len(cams))(*cams)
    b = ctypes.c_size_t(0)
    _check("sx_multi_workspace_size", lib().sx_multi_workspace_size(
        c_i32(len(cams)), ca, ctypes.byref(p), ctypes.byref(b)))
    return int(b.value)


def sx_render_multi(views: Sequence[SxView], p: SxParams, ws: torch.Tensor,
                    stream=None) -> None:
    va = (SxView * len(views))(*views)
    _check("sx_render_multi", lib().sx_render_multi(
        c_i32(len(views)), va, ctypes.byref(p), ptr(ws),
        ctypes.c_size_t(ws.numel() * ws.element_size()), stream_handle(stream)))


def sx_preprocess_backward_multi(g: SxGaussians, views: Sequence[SxView], p: SxParams,
                                 gr: SxGrads, flags: int = 0, stream=None) -> None:
    va = (SxView * len(views))(*views)
    _check("sx_preprocess_backward_multi", lib().sx_preprocess_backward_multi(
        ctypes.byref(g), c_i32(len(views)), va, ctypes.byref(p), ctypes.byref(gr),
        c_i32(flags), stream_handle(stream)))


def sx_render_backward_multi(views: Sequence[SxView], n: int, p: SxParams,
                             ws: torch.Tensor, stream=None) -> None:
    va = (SxView * len(views))(*views)
    _check("sx_render_backward_multi", lib().sx_render_backward_multi(
        c_i32(len(views)), va, c_i64(n), ctypes.byref(p), ptr(ws),
        ctypes.c_size_t(ws.numel() * ws.element_size()), stream_handle(stream)))
