"""FP64 CPU oracle for the pixel-level splatting path.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by ``__graft_entry__``'s
smoke check and by the CPU-baseline leg of ``bench.py``.  The product library
never imports, links or calls anything in this directory.

The heavy lifting is in ``splat_oracle.cpp`` (double precision, OpenMP over
pixels/Gaussians); this module marshals numpy arrays through ctypes and adds
the pieces that are plain enough to state in numpy (L1 loss, Adam).

Paper anchors (the paper's own numbering of equations):
  * Eq. 1  alpha_i = o_i exp(-1/2 d^T (Sigma2D)^-1 d)
  * Eq. 2  C_p = sum_i c_i alpha_i T_i,  T_i = prod_{j<i} (1 - alpha_j)
  * Eq. 3-4 per-cell partial colour C^m, transmittance T^m, depth D^m
  * Eq. 5  C_p = sum_m C^m prod_{k<m} T^k   (cells in ray order)
  * Eq. 6-7 gradients of C_p with respect to alpha_i and c_i through Eq. 5
  * saturation redundancy: cells behind prod T^k < eps are inactive for the
    next render of the same view.
  * geometric visibility of the cell boxes (redundancy reduction, spatial
    part); KD-tree partition (appendix, partition strategy).
  * speculative re-evaluation of pruned pairs with stale transmittance
    budgets (appendix, saturation stability during training).
  * per-ray cross-boundary filter (appendix, cross-boundary Gaussians).
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass
from typing import List, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "splat_oracle.cpp")
_LIB = os.path.join(_HERE, "libsplat_oracle.so")

FLAG_ALPHA_BAND = 1
FLAG_TERMINATE = 2
FLAG_DEPTH_ROUND = 4
FLAG_ORDER = 8
FLAG_CLAMP = 16
FLAG_VISIBILITY = 32
FLAG_SATURATION = 64
FLAG_CROSS = 128


def build(force: bool = False) -> str:
    """Compile the oracle with g++ (no fast-math, no FP contraction)."""
    if force or not os.path.exists(_LIB) or (
            os.path.getmtime(_LIB) < os.path.getmtime(_SRC)):
        cmd = ["g++", "-O2", "-std=c++17", "-fopenmp", "-ffp-contract=off",
               "-fno-fast-math", "-shared", "-fPIC", _SRC, "-o", _LIB + ".tmp"]
        subprocess.check_call(cmd)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class _Cam(ctypes.Structure):
    _fields_ = [("R", ctypes.c_double * 9), ("t", ctypes.c_double * 3),
                ("fx", ctypes.c_double), ("fy", ctypes.c_double),
                ("cx", ctypes.c_double), ("cy", ctypes.c_double),
                ("znear", ctypes.c_double), ("width", ctypes.c_int32),
                ("height", ctypes.c_int32)]


class _Params(ctypes.Structure):
    _fields_ = [("tile_w", ctypes.c_int32), ("tile_h", ctypes.c_int32),
                ("sh_degree", ctypes.c_int32),
                ("same_frame_cull", ctypes.c_int32),
                ("alpha_min", ctypes.c_double), ("alpha_max", ctypes.c_double),
                ("t_min", ctypes.c_double), ("eps2d", ctypes.c_double),
                ("bg", ctypes.c_double * 3), ("delta_q", ctypes.c_double),
                ("fov_guard", ctypes.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        _lib = ctypes.CDLL(_LIB)
        _lib.or_sort_keys.restype = ctypes.c_int64
    return _lib


def _p(a: Optional[np.ndarray]):
    if a is None:
        return None
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.c_void_p)


def _cam(cam) -> _Cam:
    c = _Cam()
    R = np.asarray(cam.R, np.float64).reshape(9)
    t = np.asarray(cam.t, np.float64).reshape(3)
    for i in range(9):
        c.R[i] = float(np.float32(R[i]))
    for i in range(3):
        c.t[i] = float(np.float32(t[i]))
    c.fx, c.fy = float(np.float32(cam.fx)), float(np.float32(cam.fy))
    c.cx, c.cy = float(np.float32(cam.cx)), float(np.float32(cam.cy))
    c.znear = float(np.float32(cam.znear))
    c.width, c.height = int(cam.width), int(cam.height)
    return c


def _params(settings, sh_degree: int, same_frame_cull: bool = False,
            delta_q: float = 0.0) -> _Params:
    p = _Params()
    p.tile_w, p.tile_h = int(settings.tile_w), int(settings.tile_h)
    p.sh_degree = int(sh_degree)
    p.same_frame_cull = int(bool(same_frame_cull))
    # the FP32 path receives these as float32; the oracle uses the same values
    p.alpha_min = float(np.float32(settings.alpha_min))
    p.alpha_max = float(np.float32(settings.alpha_max))
    p.t_min = float(np.float32(settings.t_min))
    p.eps2d = float(np.float32(settings.eps2d))
    for i in range(3):
        p.bg[i] = float(np.float32(settings.bg[i]))
    p.delta_q = float(delta_q)
    p.fov_guard = float(np.float32(settings.fov_guard))
    return p


def _scene64(scene):
    return [np.ascontiguousarray(np.asarray(a, np.float64))
            for a in (scene.means, scene.log_scales, scene.quats,
                      scene.opacity_logits, scene.sh)]


def _sh_degree(scene) -> int:
    k = scene.sh.shape[1]
    d = int(round(k ** 0.5)) - 1
    assert (d + 1) ** 2 == k
    return d


# --------------------------------------------------------------------------
def preprocess(scene, cam, settings) -> dict:
    """Per-Gaussian projection (double).  Keys: valid, depth, tcam, mean2d,
    cov2d, conic, opacity, rgb, rgb_pos, tau, pix_rect, tile_rect, n_tiles."""
    n = scene.n
    s = _scene64(scene)
    out = dict(valid=np.zeros(n, np.uint8), depth=np.zeros(n),
               tcam=np.zeros((n, 3)), mean2d=np.zeros((n, 2)),
               cov2d=np.zeros((n, 3)), conic=np.zeros((n, 3)),
               opacity=np.zeros(n), rgb=np.zeros((n, 3)),
               rgb_pos=np.zeros((n, 3), np.uint8), tau=np.zeros(n),
               pix_rect=np.zeros((n, 4), np.int32),
               tile_rect=np.zeros((n, 4), np.int32),
               n_tiles=np.zeros(n, np.int64))
    c, p = _cam(cam), _params(settings, _sh_degree(scene))
    lib().or_preprocess(
        ctypes.c_int64(n), *[_p(a) for a in s], ctypes.byref(c),
        ctypes.byref(p), *[_p(out[k]) for k in (
            "valid", "depth", "tcam", "mean2d", "cov2d", "conic", "opacity",
            "rgb", "rgb_pos", "tau", "pix_rect", "tile_rect", "n_tiles")])
    return out


def sh_eval(degree: int, dirs: np.ndarray):
    """Real SH basis values [n,(D+1)^2] and gradients [n,(D+1)^2,3]."""
    dirs = np.ascontiguousarray(np.asarray(dirs, np.float64).reshape(-1, 3))
    n = dirs.shape[0]
    nc = (degree + 1) ** 2
    Y = np.zeros((n, nc))
    G = np.zeros((n, nc, 3))
    lib().or_sh_eval(ctypes.c_int(degree), ctypes.c_int64(n), _p(dirs), _p(Y),
                     _p(G))
    return Y, G


def sort_keys(scene, cam, settings):
    """Sorted instance keys (tile<<32 | float32 depth bits), values (Gaussian
    index) and per-tile [start, end) ranges."""
    s = _scene64(scene)
    c, p = _cam(cam), _params(settings, _sh_degree(scene))
    n_inst = lib().or_sort_keys(ctypes.c_int64(scene.n), *[_p(a) for a in s],
                                ctypes.byref(c), ctypes.byref(p), None, None,
                                None)
    tiles = (((cam.width + settings.tile_w - 1) // settings.tile_w) *
             ((cam.height + settings.tile_h - 1) // settings.tile_h))
    keys = np.zeros(n_inst, np.uint64)
    vals = np.zeros(n_inst, np.uint32)
    ranges = np.zeros((tiles, 2), np.uint32)
    lib().or_sort_keys(ctypes.c_int64(scene.n), *[_p(a) for a in s],
                       ctypes.byref(c), ctypes.byref(p), _p(keys), _p(vals),
                       _p(ranges))
    return keys, vals, ranges


def _xfilter_args(xfilter):
    if xfilter is None:
        return None, None, None
    return (np.ascontiguousarray(xfilter["xf"], np.uint32),
            np.ascontiguousarray(xfilter["amb"], np.uint32),
            np.ascontiguousarray(xfilter["pixbits"], np.uint32).reshape(-1))


def render(scene, cam, settings, mode: str = "binned",
           mask: Optional[np.ndarray] = None, delta_q: float = 0.0,
           xfilter: Optional[dict] = None) -> dict:
    """Partial render of one cell (Eq. 3-4).  Returns C [H,W,3], T [H,W],
    D [H,W], nblend [H,W] (blended pairs) and flags [H,W].  ``xfilter``
    (xf, amb from cross_filter; pixbits from pixel_bits) removes
    cross-boundary Gaussians from the rays it selects."""
    H, W = cam.height, cam.width
    s = _scene64(scene)
    c = _cam(cam)
    p = _params(settings, _sh_degree(scene), delta_q=delta_q)
    out = dict(C=np.zeros((H, W, 3)), T=np.zeros((H, W)), D=np.zeros((H, W)),
               nblend=np.zeros((H, W), np.int32),
               flags=np.zeros((H, W), np.uint8))
    m = None if mask is None else np.ascontiguousarray(mask.astype(np.uint8))
    xf, xa, pb = _xfilter_args(xfilter)
    lib().or_render(ctypes.c_int64(scene.n), *[_p(a) for a in s],
                    ctypes.byref(c), ctypes.byref(p),
                    ctypes.c_int(0 if mode == "brute" else 1), _p(m),
                    _p(out["C"]), _p(out["T"]), _p(out["D"]),
                    _p(out["nblend"]), _p(out["flags"]), _p(xf), _p(xa), _p(pb))
    return out


def cross_filter(scene, cam, settings, cells, cell: int) -> dict:
    """Cross-boundary filter bits of the Gaussians of cell ``cell`` for one
    view (appendix, implementation details: cross-boundary Gaussians): bit s
    of xf[i] when Gaussian i is visible, its 3-sigma support box meets box s
    and its depth lies in the overlap of the camera-z ranges of the two
    boxes; amb[i] marks decisions within rounding reach."""
    K = len(cells)
    lo, hi = _cells_lohi(cells)
    s = _scene64(scene)
    out = dict(xf=np.zeros(scene.n, np.uint32), amb=np.zeros(scene.n, np.uint32))
    lib().or_cross_filter(ctypes.c_int64(scene.n), *[_p(a) for a in s],
                          ctypes.byref(_cam(cam)),
                          ctypes.byref(_params(settings, _sh_degree(scene))),
                          ctypes.c_int(K), _p(lo), _p(hi), ctypes.c_int(cell),
                          _p(out["xf"]), _p(out["amb"]))
    return out


def pixel_bits(vis: np.ndarray, cell: int) -> np.ndarray:
    """Per pixel, the cells whose box its ray meets (bit s = vis[s]), zero
    where the ray misses cell ``cell``'s own box: the pixel region of the
    cross-boundary filter, where both visibility maps cover the pixel."""
    K = vis.shape[0]
    bits = np.zeros(vis.shape[1:], np.uint32)
    for s in range(K):
        bits |= vis[s].astype(np.uint32) << np.uint32(s)
    return np.where(vis[cell] != 0, bits, np.uint32(0)).astype(np.uint32)


def _cells_lohi(cells):
    # the FP32 path receives the box bounds as float32; the oracle uses the
    # same values
    lo = np.ascontiguousarray(np.array([c.lo for c in cells], np.float32).astype(np.float64))
    hi = np.ascontiguousarray(np.array([c.hi for c in cells], np.float32).astype(np.float64))
    return lo, hi


def kd_partition(means, K: int):
    """Partition strategy of the paper's robustness study: recursive binary
    splits of the Gaussians by their means, each along the axis on which the
    node's means have the largest extent (first axis on ties), at the value
    of rank floor(n * K_left / K) among the node's means on that axis
    (K_left = floor(K / 2) cells go left: the median for K a power of two);
    means below it go left.  Cells numbered depth first, left first; an
    empty node keeps its box in its first cell and gives the others empty
    boxes.  Returns (boxes [(lo, hi)], cell_of int32 [n])."""
    m = np.asarray(means, np.float32).reshape(-1, 3)
    cell_of = np.zeros(len(m), np.int32)
    boxes = [None] * K

    def node(idx, k, lo, hi, first):
        if k == 1 or len(idx) == 0:
            for c in range(k):
                boxes[first + c] = (tuple(lo), tuple(hi) if c == 0 else tuple(lo))
            cell_of[idx] = first
            return
        pts = m[idx]
        ext = pts.max(0) - pts.min(0)  # float32, as the means are
        ax = int(np.argmax(ext))
        kl = k // 2
        s = np.sort(pts[:, ax])[len(idx) * kl // k]
        go_left = pts[:, ax] < s
        lo_r, hi_l = list(lo), list(hi)
        hi_l[ax] = float(s)
        lo_r[ax] = float(s)
        node(idx[go_left], kl, lo, hi_l, first)
        node(idx[~go_left], k - kl, lo_r, hi, first + kl)

    node(np.arange(len(m)), K, [-math.inf] * 3, [math.inf] * 3, 0)
    return boxes, cell_of


def repartition(cell_arrays: Sequence[np.ndarray], cell_of, K: int) -> List[np.ndarray]:
    """The redistribution of a repartition (appendix, implementation
    details: all-to-all redistribution after new boundaries): the old
    cells' rows laid end to end, row g belongs to new cell cell_of[g], and
    each new cell keeps the rows in their old order."""
    rows = np.concatenate([np.asarray(a) for a in cell_arrays])
    cell_of = np.asarray(cell_of)
    return [rows[cell_of == k] for k in range(K)]


def imbalance(cell_of, K: int) -> float:
    """N_max / mean(N) - 1 over the K cells' Gaussian counts."""
    counts = np.bincount(np.asarray(cell_of), minlength=K)
    return float(counts.max() / counts.mean() - 1.0)


def visibility(cells, cam) -> dict:
    """Geometric visibility of each cell box (redundancy reduction section,
    spatial part): vis [K,H,W] uint8, 1 where the pixel's centre ray meets
    the part of the box inside the view frustum; flags [H,W] mark decisions
    within rounding reach of flipping."""
    K = len(cells)
    lo, hi = _cells_lohi(cells)
    H, W = cam.height, cam.width
    out = dict(vis=np.zeros((K, H, W), np.uint8), flags=np.zeros((H, W), np.uint8))
    lib().or_visibility(ctypes.c_int(K), _p(lo), _p(hi), ctypes.byref(_cam(cam)),
                        _p(out["vis"]), _p(out["flags"]))
    return out


def composite(Cparts: np.ndarray, Tparts: np.ndarray, cells, cam, settings,
              same_frame_cull: bool = False) -> dict:
    """Eq. 5 over K partial buffers Cparts [K,H,W,3], Tparts [K,H,W].
    Returns rgb [H,W,3], T [H,W], order [H,W,K], mask [K,H,W] (1 = cell
    still active for the next render of this view), flags [H,W]."""
    K = len(cells)
    H, W = cam.height, cam.width
    Cp = np.ascontiguousarray(np.asarray(Cparts, np.float64))
    Tp = np.ascontiguousarray(np.asarray(Tparts, np.float64))
    lo, hi = _cells_lohi(cells)
    out = dict(rgb=np.zeros((H, W, 3)), T=np.zeros((H, W)),
               order=np.zeros((H, W, K), np.int32),
               mask=np.zeros((K, H, W), np.uint8),
               flags=np.zeros((H, W), np.uint8))
    lib().or_composite(ctypes.c_int(K), _p(Cp), _p(Tp), _p(lo), _p(hi),
                       ctypes.byref(_cam(cam)),
                       ctypes.byref(_params(settings, 0, same_frame_cull)),
                       _p(out["rgb"]), _p(out["T"]), _p(out["order"]),
                       _p(out["mask"]), _p(out["flags"]))
    return out


def composite_reeval(Cparts: np.ndarray, Tparts: np.ndarray, cells, cam, settings,
                     mask_in: np.ndarray, budget: np.ndarray,
                     omega: Optional[np.ndarray] = None,
                     same_frame_cull: bool = False) -> dict:
    """Eq. 5 with the saturation state carried between renders of a view and
    its speculative re-evaluation (appendix, saturation stability during
    training).  mask_in [K,H,W] (1 = cell rendered at the pixel), omega
    [K,H,W] (1 = the pixel's ray meets the cell's box; None = every box),
    budget [K,H,W] the stale transmittance consumption of pruned pairs
    (updated in place for the pairs pruned now).  Returns rgb, T, mask (the
    state for the next render), flips [H,W] (re-activated cells per pixel)
    and flags."""
    K = len(cells)
    H, W = cam.height, cam.width
    Cp = np.ascontiguousarray(np.asarray(Cparts, np.float64))
    Tp = np.ascontiguousarray(np.asarray(Tparts, np.float64))
    lo, hi = _cells_lohi(cells)
    mi = np.ascontiguousarray(mask_in.astype(np.uint8))
    om = None if omega is None else np.ascontiguousarray(omega.astype(np.uint8))
    assert budget.dtype == np.float64 and budget.flags.c_contiguous
    assert budget.shape == (K, H, W) and mi.shape == (K, H, W)
    out = dict(rgb=np.zeros((H, W, 3)), T=np.zeros((H, W)),
               mask=np.zeros((K, H, W), np.uint8), flips=np.zeros((H, W), np.int32),
               flags=np.zeros((H, W), np.uint8))
    lib().or_composite_reeval(ctypes.c_int(K), _p(Cp), _p(Tp), _p(lo), _p(hi),
                              ctypes.byref(_cam(cam)),
                              ctypes.byref(_params(settings, 0, same_frame_cull)),
                              _p(mi), _p(om), _p(budget), _p(out["rgb"]), _p(out["T"]),
                              _p(out["mask"]), _p(out["flips"]), _p(out["flags"]))
    return out


def composite_backward(Cparts, Tparts, order, cam, settings, drgb,
                       dT=None, active=None, same_frame_cull=False):
    K = Cparts.shape[0]
    H, W = cam.height, cam.width
    Cp = np.ascontiguousarray(np.asarray(Cparts, np.float64))
    Tp = np.ascontiguousarray(np.asarray(Tparts, np.float64))
    dC = np.zeros((K, H, W, 3))
    dTo = np.zeros((K, H, W))
    g = np.ascontiguousarray(np.asarray(drgb, np.float64))
    gT = None if dT is None else np.ascontiguousarray(np.asarray(dT, np.float64))
    act = None if active is None else np.ascontiguousarray(active.astype(np.uint8))
    lib().or_composite_backward(
        ctypes.c_int(K), _p(Cp), _p(Tp), _p(np.ascontiguousarray(order)),
        _p(act), ctypes.byref(_cam(cam)),
        ctypes.byref(_params(settings, 0, same_frame_cull)), _p(g), _p(gT),
        _p(dC), _p(dTo))
    return dC, dTo


def render_backward(scene, cam, settings, dC=None, dT=None, dD=None,
                    mask=None, xfilter=None) -> dict:
    """Gradients of one cell's partial render with respect to the screen
    quantities (g2d [n,10]: mean2d x/y, conic a/b/c, opacity, rgb, depth) and
    the raw parameters (means, log_scales, quats, opacity_logits, sh).  Also
    g2d_scale [n,10]: a first-order scale of the rounding error of an FP32
    evaluation of each screen-space entry, in units of the FP32 unit
    roundoff (for test tolerances; it enters no gradient): per pixel term,
    the sizes of the quantities it is formed from before they cancel, times
    the ulps its inputs carry (the pairs the walk spans, the rounding of
    alpha from FP32 screen position, conic and opacity)."""
    n = scene.n
    nc = scene.sh.shape[1]
    s = _scene64(scene)
    out = dict(g2d=np.zeros((n, 10)), means=np.zeros((n, 3)),
               log_scales=np.zeros((n, 3)), quats=np.zeros((n, 4)),
               opacity_logits=np.zeros(n), sh=np.zeros((n, nc, 3)),
               g2d_scale=np.zeros((n, 10)))

    def arr(a):
        return None if a is None else np.ascontiguousarray(np.asarray(a, np.float64))
    m = None if mask is None else np.ascontiguousarray(mask.astype(np.uint8))
    xf, _, pb = _xfilter_args(xfilter)
    lib().or_render_backward(
        ctypes.c_int64(n), *[_p(a) for a in s], ctypes.byref(_cam(cam)),
        ctypes.byref(_params(settings, _sh_degree(scene))), _p(m),
        _p(arr(dC)), _p(arr(dT)), _p(arr(dD)), _p(out["g2d"]),
        _p(out["means"]), _p(out["log_scales"]), _p(out["quats"]),
        _p(out["opacity_logits"]), _p(out["sh"]), _p(xf), _p(pb), _p(out["g2d_scale"]))
    return out


def preprocess_backward(scene, cam, settings, g2d) -> dict:
    """The projection backward alone: screen-space gradients g2d [n,10] of
    one view (as render_backward returns them) chained to the raw
    parameters (means, log_scales, quats, opacity_logits, sh)."""
    n = scene.n
    nc = scene.sh.shape[1]
    s = _scene64(scene)
    out = dict(means=np.zeros((n, 3)), log_scales=np.zeros((n, 3)), quats=np.zeros((n, 4)),
               opacity_logits=np.zeros(n), sh=np.zeros((n, nc, 3)))
    g = np.ascontiguousarray(np.asarray(g2d, np.float64)[:, :10])
    lib().or_preprocess_backward(
        ctypes.c_int64(n), *[_p(a) for a in s], ctypes.byref(_cam(cam)),
        ctypes.byref(_params(settings, _sh_degree(scene))), _p(g),
        _p(out["means"]), _p(out["log_scales"]), _p(out["quats"]),
        _p(out["opacity_logits"]), _p(out["sh"]))
    return out


# --------------------------------------------------------------------------
# whole-frame drivers over K cells


@dataclass
class Frame:
    parts: List[dict]  # per-cell render outputs
    comp: dict         # composite outputs
    Cparts: np.ndarray
    Tparts: np.ndarray


def cross_filters(cell_scenes: Sequence, cells, cam, settings) -> List[dict]:
    """The cross-boundary filter of every cell's render for one view, with
    the pixel regions taken from the geometric visibility maps."""
    vis = visibility(cells, cam)["vis"]
    out = []
    for k, sc in enumerate(cell_scenes):
        f = cross_filter(sc, cam, settings, cells, k)
        f["pixbits"] = pixel_bits(vis, k)
        out.append(f)
    return out


def forward(cell_scenes: Sequence, cells, cam, settings,
            masks: Optional[np.ndarray] = None, same_frame_cull=False,
            delta_q: float = 0.0, xfilters: Optional[List[dict]] = None) -> Frame:
    """Render every cell (Eq. 3-4) and compose them (Eq. 5).  ``masks``
    [K,H,W] (1 = active) restricts each cell's render; ``xfilters`` (from
    cross_filters) removes cross-boundary Gaussians per ray."""
    parts = [render(sc, cam, settings, "binned",
                    None if masks is None else masks[k], delta_q,
                    None if xfilters is None else xfilters[k])
             for k, sc in enumerate(cell_scenes)]
    Cp = np.stack([p["C"] for p in parts])
    Tp = np.stack([p["T"] for p in parts])
    comp = composite(Cp, Tp, cells, cam, settings, same_frame_cull)
    return Frame(parts, comp, Cp, Tp)


def backward(cell_scenes, cells, cam, settings, frame: Frame, drgb, dT=None,
             masks=None, same_frame_cull=False, xfilters=None) -> List[dict]:
    """Gradients for every cell's Gaussians through the composition (Eq. 6-7)
    and each cell's local render."""
    dC, dTp = composite_backward(frame.Cparts, frame.Tparts,
                                 frame.comp["order"], cam, settings, drgb, dT,
                                 frame.comp["mask"], same_frame_cull)
    return [render_backward(sc, cam, settings, dC[k], dTp[k], None,
                            None if masks is None else masks[k],
                            None if xfilters is None else xfilters[k])
            for k, sc in enumerate(cell_scenes)]


def l1_loss(rgb: np.ndarray, target: np.ndarray):
    """Mean absolute error over H*W*3 and its gradient sign(C - target)/(3HW)
    with sign(0) = 0 (the RGB term of the paper's training loss)."""
    d = np.asarray(rgb, np.float64) - np.asarray(target, np.float64)
    n = d.size
    return float(np.abs(d).sum() / n), np.sign(d) / n


def adam_step(param, grad, m, v, step: int, lr: float, beta1: float = 0.9,
              beta2: float = 0.999, eps: float = 1e-8):
    """Textbook Adam (Kingma & Ba, Algorithm 1) with bias correction; updates
    the arrays in place and returns them."""
    m *= beta1
    m += (1 - beta1) * grad
    v *= beta2
    v += (1 - beta2) * grad * grad
    mhat = m / (1 - beta1 ** step)
    vhat = v / (1 - beta2 ** step)
    param -= lr * mhat / (np.sqrt(vhat) + eps)
    return param, m, v


def num_threads() -> int:
    return int(lib().or_num_threads())


def set_threads(n: int) -> None:
    lib().or_set_threads(ctypes.c_int(n))
