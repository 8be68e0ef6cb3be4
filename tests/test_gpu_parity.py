"""GPU parity of every hot-path step against the FP64 oracle, through the
C ABI (ctypes binding), at the tiny workload (5k Gaussians, 128x128, 16x16
tiles: 64 tiles with a ragged tail of sizes per tile) and on edge cases.

Tolerances: integer/byte/index work bit-exact (tile counts, footprints,
sort keys, values, ranges, masks); pixels max-abs 1e-4 on pixels the oracle
does not flag as ambiguous (a pair within rounding reach of alpha_min, a
transmittance within reach of t_min, an ambiguous float32 depth rounding or
composite order), flagged pixels within the jump bound; gradients per
element within 1e-3 relative, each entry's magnitude floored at 1e-3 of
the largest entry of its parameter family.
"""
import math

import numpy as np
import pytest

import oracle
import synth
from gpu_helpers import (assert_ranges, assert_same, big_box, compare_image,
                         check_grad, expand_lists, grid_cells_xy, jump_bound,
                         need_gpu, rec_fields)

pytestmark = pytest.mark.gpu
ST = synth.RenderSettings()


@pytest.fixture(scope="module")
def torch_gpu():
    need_gpu()
    import torch
    return torch


def _cell_view(torch, scene, cam, st=ST, keep_keys=True):
    from paper_2606_18588_amd.pipeline import CellView, GaussianParams
    p = GaussianParams.from_scene(scene)
    v = CellView(p, cam, st, keep_keys=keep_keys)
    return p, v


def test_library_version(torch_gpu):
    from paper_2606_18588_amd import binding as B
    print("case: version", B.sx_version(), flush=True)
    assert "gfx950" in B.sx_version()


# -------------------------------------------------------------------- a1 --
def test_preprocess_matches_oracle(torch_gpu):
    print("case: preprocess tiny seed 0", flush=True)
    torch = torch_gpu
    scene, cam = synth.tiny_scene(), synth.tiny_camera()
    _, v = _cell_view(torch, scene, cam)
    v.preprocess()
    torch.cuda.synchronize()
    ref = oracle.preprocess(scene, cam, ST)
    nt = v.n_tiles.cpu().numpy().astype(np.int64)
    assert_same(nt, ref["n_tiles"], "tiles touched")
    vis = ref["valid"] == 1
    rect = v.rect.cpu().numpy().astype(np.int64)[vis]
    tr = ref["tile_rect"][vis]
    assert_same(rect[:, :2], tr[:, :2], "rect lo")
    assert_same(rect[:, 2:], tr[:, 2:] + 1, "rect hi")
    f = rec_fields(v.rec)
    assert_same(f["depth"][vis], ref["depth"][vis].astype(np.float32), "depth")
    mc = ref["mean2d"][vis] - np.array([cam.cx, cam.cy])
    assert np.abs(f["mean2d_c"][vis] - mc).max() <= 1e-6 * (1 + np.abs(mc).max())
    np.testing.assert_allclose(f["conic"][vis], ref["conic"][vis], rtol=2e-6, atol=1e-9)
    np.testing.assert_allclose(f["opacity"][vis], ref["opacity"][vis], rtol=2e-7)
    np.testing.assert_allclose(f["rgb"][vis], ref["rgb"][vis], atol=2e-7)


def test_preprocess_sh3_colour(torch_gpu):
    """SH degree 3 evaluation (polynomial basis in the kernel, Legendre
    construction in the oracle) on a ground scene seen from the aerial
    camera."""
    print("case: preprocess sh3 ground 20k", flush=True)
    torch = torch_gpu
    scene = synth.make_ground_scene(21, 20000, half_extent=60.0)
    cam = synth.aerial_camera((0.0, -60.0, 40.0), 0.0, math.radians(30), 320, 180)
    _, v = _cell_view(torch, scene, cam)
    v.preprocess()
    torch.cuda.synchronize()
    ref = oracle.preprocess(scene, cam, ST)
    vis = ref["valid"] == 1
    assert vis.sum() > 1000
    assert_same(v.n_tiles.cpu().numpy().astype(np.int64), ref["n_tiles"], "tiles touched")
    f = rec_fields(v.rec)
    np.testing.assert_allclose(f["rgb"][vis], ref["rgb"][vis], atol=1e-6)
    np.testing.assert_allclose(f["conic"][vis], ref["conic"][vis], rtol=5e-6, atol=1e-9)


def test_preprocess_frustum_cull(torch_gpu):
    """Frustum cull by the mean with the guard off, at the literal field of
    view and at the default guard: tile counts bit-exact against the oracle
    on a scene spread far beyond the view, with large footprints."""
    print("case: preprocess frustum cull guards", flush=True)
    torch = torch_gpu
    scene = synth.make_cube_scene(17, 20000, log_scale=(-1.5, 0.5))
    scene.means *= np.float32(3.0)
    cam = synth.tiny_camera(120, 90)
    kept = []
    for guard in (0.0, 1.0, 1.3):
        st = synth.RenderSettings(fov_guard=guard)
        _, v = _cell_view(torch, scene, cam, st)
        v.preprocess()
        torch.cuda.synchronize()
        ref = oracle.preprocess(scene, cam, st)
        assert_same(v.n_tiles.cpu().numpy().astype(np.int64), ref["n_tiles"], f"guard {guard}")
        kept.append(int((ref["valid"] == 1).sum()))
    assert kept[0] > kept[2] > kept[1] > 0, kept


# ------------------------------------------------------------------ a2-a4 --
@pytest.mark.parametrize("tile", [(16, 16), (32, 8), (8, 8)])
def test_sort_keys_vals_ranges_bit_exact(torch_gpu, tile):
    print(f"case: sort tiny tile={tile}", flush=True)
    torch = torch_gpu
    st = synth.RenderSettings(tile_w=tile[0], tile_h=tile[1])
    scene, cam = synth.tiny_scene(), synth.tiny_camera()
    _, v = _cell_view(torch, scene, cam, st)
    v.preprocess()
    counts = v.sort(sync=True)
    torch.cuda.synchronize()
    keys, vals, ranges = oracle.sort_keys(scene, cam, st)
    ref_vis = int(oracle.preprocess(scene, cam, st)["valid"].sum())
    assert counts[0] == ref_vis
    _check_lists(v, counts, keys, vals, ranges)


def _check_lists(v, counts, keys, vals, ranges):
    """Instance count, keys, values and tile ranges equal the oracle's
    sorted instances bit for bit."""
    assert counts[1] == len(keys)
    n = len(keys)
    assert_same(v.keys[:n].cpu().numpy().view(np.uint64), keys, "keys")
    assert_same(v.vals[:n].cpu().numpy().view(np.uint32), vals, "vals")
    assert_ranges(v.ranges.cpu().numpy().view(np.uint32)[:-1], ranges)


def test_sort_ragged_and_capacity(torch_gpu):
    """Non-multiple image size (ragged tile tail), a capacity that is too
    small (SX_ECAPACITY, then a retry with grown buffers), and more than
    12k instances."""
    print("case: sort ragged 100x70 capacity", flush=True)
    torch = torch_gpu
    from paper_2606_18588_amd import binding as B
    from paper_2606_18588_amd.pipeline import CellView, GaussianParams
    scene = synth.make_cube_scene(5, 30000, log_scale=(-3.3, 0.5))
    cam = synth.tiny_camera(100, 70)
    p = GaussianParams.from_scene(scene)
    v = CellView(p, cam, ST, capacity=1000, keep_keys=True)
    v.preprocess()
    with pytest.raises(B.SplaxelError) as ei:
        B.sx_sort(v.c_proj, p.n, v.c_cam, v.c_par, v.capacity, v.keys, v.vals, v.ranges, v.ws,
                  sync_counts=True)
    assert ei.value.code == B.SX_ECAPACITY
    counts = v.sort(sync=True)
    keys, vals, ranges = oracle.sort_keys(scene, cam, ST)
    assert len(keys) > 3 * 4096
    _check_lists(v, counts, keys, vals, ranges)
    c4 = B.sx_sort_counts(v.ws, p.n)
    assert c4[2] == 0 and c4[3] == 0


def test_sort_large_grid(torch_gpu):
    """A large tile grid (2048x1152 with 8x8 tiles: 36864 tiles, more than
    the binning's LDS counters hold, so it counts and reserves slots with a
    device atomic per instance): keys, values and ranges are still
    bit-exact."""
    print("case: sort large grid 2048x1152 8x8", flush=True)
    torch = torch_gpu
    st = synth.RenderSettings(tile_w=8, tile_h=8)
    scene = synth.make_cube_scene(8, 20000, log_scale=(-3.0, 0.6))
    cam = synth.tiny_camera(2048, 1152)
    _, v = _cell_view(torch, scene, cam, st)
    v.preprocess()
    counts = v.sort(sync=True)
    keys, vals, ranges = oracle.sort_keys(scene, cam, st)
    assert len(keys) > 4 * 4096
    _check_lists(v, counts, keys, vals, ranges)


def test_sort_long_tile_lists_bit_exact(torch_gpu):
    """Tile lists of 839 to 10130 entries (30k large Gaussians in a 128x96
    view): the per-tile sort's bitonic network (up to 2048 entries) and its
    merge of sorted 2048-entry chunks through LDS windows (one to three
    merge passes) give the oracle's keys, values and ranges bit for bit."""
    print("case: sort long tile lists 128x96", flush=True)
    torch = torch_gpu
    scene = synth.make_cube_scene(17, 30000, log_scale=(-2.3, 0.5))
    cam = synth.tiny_camera(128, 96)
    _, v = _cell_view(torch, scene, cam)
    v.preprocess()
    counts = v.sort(sync=True)
    keys, vals, ranges = oracle.sort_keys(scene, cam, ST)
    lens = ranges[:, 1].astype(np.int64) - ranges[:, 0]
    assert lens.max() > 8192 and ((lens > 256) & (lens <= 2048)).any()
    _check_lists(v, counts, keys, vals, ranges)


def test_sort_async_overflow_flag(torch_gpu):
    """Without the synchronous count check an overflow writes no instance
    (every tile range is empty), stays in bounds and raises the overflow
    flag."""
    print("case: sort async overflow", flush=True)
    torch = torch_gpu
    from paper_2606_18588_amd import binding as B
    from paper_2606_18588_amd.pipeline import CellView, GaussianParams
    scene = synth.tiny_scene()
    cam = synth.tiny_camera()
    p = GaussianParams.from_scene(scene)
    v = CellView(p, cam, ST, capacity=2000)
    v.preprocess()
    v.sort(sync=False)
    c4 = B.sx_sort_counts(v.ws, p.n)
    assert c4[1] > 2000 and c4[2] == 1 and c4[3] == 0
    r = v.ranges.cpu().numpy().view(np.uint32)[:-1]  # the tiles' rows (the last is spare)
    assert not r.any()


# -------------------------------------------------------------------- a5 --
def _render(torch, scene, cam, st=ST, mask=None):
    _, v = _cell_view(torch, scene, cam, st, keep_keys=False)
    v.preprocess()
    v.sort(sync=True)
    v.render(mask, want_depth=True)
    torch.cuda.synchronize()
    return v


def test_render_matches_oracle(torch_gpu):
    print("case: render tiny", flush=True)
    torch = torch_gpu
    scene, cam = synth.tiny_scene(), synth.tiny_camera()
    v = _render(torch, scene, cam)
    ref = oracle.render(scene, cam, ST)
    part = v.partial.cpu().numpy()
    cmax = float(oracle.preprocess(scene, cam, ST)["rgb"].max())
    e, nf = compare_image(part[..., :3], ref["C"], ref["flags"], 1e-4, jump_bound(ST, cmax))
    compare_image(part[..., 3], ref["T"], ref["flags"], 1e-4, 1.0)
    compare_image(v.depth.cpu().numpy(), ref["D"], ref["flags"], 1e-3 * 4.0, None)
    fl = ref["flags"] != 0
    nb = v.nblend.cpu().numpy()
    assert_same(nb[~fl], ref["nblend"][~fl], "blended pairs per pixel")
    print(f"render tiny: max-abs {e:.3g}, flagged {nf}", flush=True)


@pytest.mark.parametrize("tile", [(32, 8), (8, 32), (32, 16), (16, 32), (8, 8)])
def test_render_tile_shape_bit_identical(torch_gpu, tile):
    """Tiling invariance: every supported tile shape gives bit-identical
    pixels (the per-pixel list and arithmetic do not depend on tiling)."""
    print(f"case: render tile {tile}", flush=True)
    torch = torch_gpu
    scene, cam = synth.tiny_scene(), synth.tiny_camera()
    a = _render(torch, scene, cam).partial.cpu().numpy()
    st = synth.RenderSettings(tile_w=tile[0], tile_h=tile[1])
    b = _render(torch, scene, cam, st).partial.cpu().numpy()
    assert_same(a, b, "partials across tile shapes")


def test_render_constant_colour_invariant(torch_gpu):
    """C = c0 (1 - T) for constant colour (telescoping of Eq. 2)."""
    print("case: render constant colour", flush=True)
    torch = torch_gpu
    scene = synth.tiny_scene()
    scene.sh[:] = np.float32((0.6 - 0.5) * 2.0 * math.sqrt(math.pi))
    v = _render(torch, scene, synth.tiny_camera())
    part = v.partial.cpu().numpy().astype(np.float64)
    c0 = float(rec_fields(v.rec)["rgb"][v.n_tiles.cpu().numpy() > 0][0, 0])
    assert np.abs(part[..., 0] - c0 * (1 - part[..., 3])).max() < 2e-6


def test_render_single_gaussian_closed_form(torch_gpu):
    """A Gaussian on a pixel centre: alpha there equals its opacity."""
    print("case: render single gaussian", flush=True)
    torch = torch_gpu
    sc = synth.Scene(np.zeros((1, 3), np.float32), np.full((1, 3), -3.0, np.float32),
                     np.array([[1, 0, 0, 0]], np.float32), np.array([0.3], np.float32),
                     (np.array([[[0.2, 0.4, 0.6]]]) - 0.5).astype(np.float32) * np.float32(2 * math.sqrt(math.pi)))
    cam = synth.camera_from_rows(np.eye(3), (0, 0, -3), 64, 64, 50.0, cx=32.5, cy=32.5)
    v = _render(torch, sc, cam)
    part = v.partial.cpu().numpy()
    o = 1 / (1 + math.exp(-float(np.float32(0.3))))
    col = sc.sh[0, 0].astype(np.float64) / (2 * math.sqrt(math.pi)) + 0.5
    assert np.abs(part[32, 32, :3] - col * o).max() < 1e-6
    assert abs(part[32, 32, 3] - (1 - o)) < 1e-6


def test_render_empty_and_all_culled(torch_gpu):
    """n = 0 and a camera facing away: identity partials (C=0, T=1)."""
    print("case: render empty", flush=True)
    torch = torch_gpu
    cam = synth.tiny_camera(48, 40)
    empty = synth.tiny_scene(n=1).subset(np.zeros(0, np.int64))
    v = _render(torch, empty, cam)
    p = v.partial.cpu().numpy()
    assert np.all(p[..., :3] == 0) and np.all(p[..., 3] == 1)
    away = synth.tiny_scene()
    away.means[:, 2] = -10.0
    v = _render(torch, away, cam)
    p = v.partial.cpu().numpy()
    assert np.all(p[..., :3] == 0) and np.all(p[..., 3] == 1)
    assert int(v.counts[0]) == 0


def test_render_mask(torch_gpu):
    """Masked pixels output the identity; unmasked pixels are unchanged."""
    print("case: render mask", flush=True)
    torch = torch_gpu
    from paper_2606_18588_amd import binding as B
    scene, cam = synth.tiny_scene(), synth.tiny_camera()
    full = _render(torch, scene, cam).partial.cpu().numpy()
    rng = np.random.default_rng(0)
    bits = rng.integers(0, 2, size=cam.width * cam.height).astype(np.uint8)
    words = np.packbits(bits, bitorder="little").view(np.uint32).astype(np.int64)
    mask = torch.as_tensor(words.astype(np.uint32).view(np.int32)).cuda()
    m = _render(torch, scene, cam, mask=mask).partial.cpu().numpy()
    on = bits.reshape(cam.height, cam.width) == 1
    assert_same(m[on], full[on], "unmasked pixels")
    assert np.all(m[~on][:, :3] == 0) and np.all(m[~on][:, 3] == 1)


# -------------------------------------------------------------------- a6 --
def _frame(torch, scenes, boxes, cam, st=ST, flags=0):
    from paper_2606_18588_amd.pipeline import Frame, GaussianParams
    params = [GaussianParams.from_scene(s) for s in scenes]
    return Frame(params, boxes, cam, st, flags=flags), params


def test_composite_k8_grid_matches_oracle(torch_gpu):
    """Eq. 5 over a 4x2 grid of prisms (cells ordered per pixel by ray entry)
    against the oracle's composition of its own partials."""
    print("case: composite k8 grid tiny", flush=True)
    torch = torch_gpu
    scene = synth.make_cube_scene(3, 8000, log_scale=(-3.6, 0.5))
    cam = synth.camera_from_rows(
        np.array([[1, 0, 0], [0, 0.9950, -0.0998], [0, 0.0998, 0.9950]]), (0.13, 0.21, -3.0),
        96, 80, 70.0)
    xe, ye = [-1.0, -0.5, 0.0, 0.5, 1.0], [-1.0, 0.0, 1.0]
    part = synth.grid_partition(scene, xe, ye)
    boxes = grid_cells_xy(xe, ye)
    part.cells = boxes
    scenes = part.cell_scenes(scene)
    fr, _ = _frame(torch, scenes, boxes, cam)
    fr.init_masks()
    out = fr.forward(update_masks=True).cpu().numpy()
    torch.cuda.synchronize()
    ref = oracle.forward(scenes, boxes, cam, ST)
    fl = ref.comp["flags"].copy()
    for p in ref.parts:
        fl |= p["flags"]
    cmax = max(float(oracle.preprocess(s, cam, ST)["rgb"].max()) for s in scenes)
    e, nf = compare_image(out[..., :3], ref.comp["rgb"], fl, 1e-4, 8 * jump_bound(ST, cmax))
    compare_image(out[..., 3], ref.comp["T"], fl, 1e-4, 1.0)
    masks = fr.masks.cpu().numpy().view(np.uint32)
    bits = np.unpackbits(masks.view(np.uint8), bitorder="little").reshape(8, -1)[:, :cam.width * cam.height]
    refm = ref.comp["mask"].reshape(8, -1)
    okpix = (fl.reshape(-1) == 0)
    assert_same(bits[:, okpix], refm[:, okpix], "saturation masks")
    print(f"composite k8: max-abs {e:.3g} flagged {nf} inactive pairs {(refm == 0).sum()}", flush=True)


def test_visibility_maps_bit_exact(torch_gpu):
    """Geometric visibility maps (redundancy reduction, spatial part) equal
    the oracle's bit for bit: the 4x2 ground grid from an aerial camera at a
    ragged size, and boxes of the cube scene (one behind the camera, one
    holding it, one half-infinite) from a rotated camera."""
    print("case: visibility maps", flush=True)
    torch = torch_gpu
    from paper_2606_18588_amd import binding as B
    xe, ye = synth.GRID_X, synth.GRID_Y
    grid = [synth.Cell((xe[i], ye[j], -math.inf), (xe[i + 1], ye[j + 1], math.inf))
            for j in range(2) for i in range(4)]
    boxes = [synth.Cell((-0.6, -0.3, -0.4), (0.5, 0.7, 0.2)),
             synth.Cell((3.0, -5.0, 1.0), (9.0, 5.0, 9.0)),
             synth.Cell((2.0, -2.0, 0.0), (3.0, -1.0, 2.0)),
             synth.Cell((0.3, -math.inf, -math.inf), (math.inf, math.inf, 0.25))]
    cases = [(grid, synth.aerial_camera((10.0, 20.0, 150.0), 0.7, math.radians(45.0), 333, 217)),
             (boxes, synth.look_at_camera((2.5, -1.7, 1.3), (0.1, 0.2, -0.1), 150, 101,
                                          hfov_deg=60.0))]
    for cells, cam in cases:
        K, H, W = len(cells), cam.height, cam.width
        words = (H * W + 31) // 32
        m = torch.zeros((K, words), dtype=torch.int32, device="cuda")
        B.sx_visibility(cells, B.camera(cam), m)
        torch.cuda.synchronize()
        bits = np.unpackbits(m.cpu().numpy().view(np.uint8), bitorder="little").reshape(K, -1)[:, :H * W]
        ref = oracle.visibility(cells, cam)
        assert not ref["flags"].any()
        assert_same(bits, ref["vis"].reshape(K, -1), "visibility bits")
        print(f"visibility {K} cells {W}x{H}: visible pairs {int(bits.sum())} of {bits.size}",
              flush=True)


def test_composite_with_visibility_matches_oracle(torch_gpu):
    """A K = 8 frame whose masks start from the geometric visibility maps:
    each cell renders only where its box is visible, and the composition
    and its saturation masks match the oracle given the same maps."""
    print("case: composite k8 with visibility", flush=True)
    torch = torch_gpu
    scene = synth.make_cube_scene(3, 8000, log_scale=(-3.6, 0.5))
    cam = synth.camera_from_rows(
        np.array([[1, 0, 0], [0, 0.9950, -0.0998], [0, 0.0998, 0.9950]]), (0.13, 0.21, -3.0),
        96, 80, 70.0)
    xe, ye = [-1.0, -0.5, 0.0, 0.5, 1.0], [-1.0, 0.0, 1.0]
    part = synth.grid_partition(scene, xe, ye)
    boxes = grid_cells_xy(xe, ye)
    part.cells = boxes
    scenes = part.cell_scenes(scene)
    fr, _ = _frame(torch, scenes, boxes, cam)
    fr.init_masks(geometric=True)
    out = fr.forward(use_masks=True, update_masks=True).cpu().numpy()
    torch.cuda.synchronize()
    vis = oracle.visibility(boxes, cam)
    assert not vis["flags"].any()
    assert 0 < vis["vis"].sum() < vis["vis"].size
    ref = oracle.forward(scenes, boxes, cam, ST, masks=vis["vis"])
    fl = ref.comp["flags"].copy()
    for p in ref.parts:
        fl |= p["flags"]
    cmax = max(float(oracle.preprocess(s, cam, ST)["rgb"].max()) for s in scenes)
    e, nf = compare_image(out[..., :3], ref.comp["rgb"], fl, 1e-4, 8 * jump_bound(ST, cmax))
    compare_image(out[..., 3], ref.comp["T"], fl, 1e-4, 1.0)
    masks = fr.masks.cpu().numpy().view(np.uint32)
    bits = np.unpackbits(masks.view(np.uint8), bitorder="little").reshape(8, -1)[:, :cam.width * cam.height]
    refm = (ref.comp["mask"] & vis["vis"]).reshape(8, -1)
    okpix = fl.reshape(-1) == 0
    assert_same(bits[:, okpix], refm[:, okpix], "visibility and saturation masks")
    print(f"composite k8 + visibility: max-abs {e:.3g} flagged {nf} "
          f"invisible pairs {(vis['vis'] == 0).sum()}", flush=True)


@pytest.mark.parametrize("geometric,same_frame", [(True, False), (False, False), (True, True)])
def test_composite_reeval_three_renders_match_oracle(torch_gpu, geometric, same_frame):
    """Saturation carried across three renders of one view with speculative
    re-evaluation: KD cells starting from their geometric maps; render 1
    prunes pairs behind saturated prefixes and keeps their budgets; the
    opacities are then lowered, and render 2 re-activates the pairs the
    fresh residual covers; render 3 renders them.  Image, masks and budgets
    match the oracle run on its own state at every render (pixels flagged
    at any render excluded from then on)."""
    print("case: composite re-evaluation, three renders", flush=True)
    torch = torch_gpu
    from paper_2606_18588_amd import binding as B
    scene = synth.make_cube_scene(4, 9000, log_scale=(-3.2, 0.4), logit_sigma=2.0)
    cam = synth.look_at_camera((2.4, -2.9, 1.6), (0.0, 0.1, 0.0), 112, 84, hfov_deg=55.0)
    boxes_t, cell_of = B.sx_kd_partition(scene.means, 8)
    boxes = [synth.Cell(lo, hi) for lo, hi in boxes_t]
    scenes = [scene.subset(np.nonzero(cell_of == k)[0]) for k in range(8)]
    K, H, W = 8, cam.height, cam.width
    from paper_2606_18588_amd import binding as Bf
    fr, params = _frame(torch, scenes, boxes, cam,
                        flags=Bf.SX_FLAG_SAME_FRAME_CULL if same_frame else 0)
    fr.init_masks(geometric=geometric, reeval=True)
    vis = oracle.visibility(boxes, cam)
    assert not vis["flags"].any()
    # without the geometric maps every box counts as met by every ray
    om = vis["vis"] if geometric else np.ones((K, H, W), np.uint8)
    state, budget = om.copy(), np.zeros((K, H, W))
    faded = [s.subset(np.arange(s.n)) for s in scenes]
    for s in faded:
        s.opacity_logits = s.opacity_logits - 0.7
    bad = np.zeros((H, W), bool)
    stats = []
    for r, scs in enumerate((scenes, faded, faded)):
        if r == 1:
            for prm in params:
                prm.opacity_logits -= 0.7
        out = fr.forward(use_masks=True, update_masks=True).cpu().numpy()
        torch.cuda.synchronize()
        ref = oracle.forward(scs, boxes, cam, ST, masks=state)
        rr = oracle.composite_reeval(ref.Cparts, ref.Tparts, boxes, cam, ST, state, budget,
                                     omega=om if geometric else None,
                                     same_frame_cull=same_frame)
        for p in ref.parts:
            bad |= p["flags"] != 0
        bad |= rr["flags"] != 0
        fl = bad.astype(np.uint8)
        cmax = max(float(oracle.preprocess(s, cam, ST)["rgb"].max()) for s in scs)
        e, nf = compare_image(out[..., :3], rr["rgb"], fl, 1e-4, 8 * jump_bound(ST, cmax))
        compare_image(out[..., 3], rr["T"], fl, 1e-4, 1.0)
        bits = np.unpackbits(fr.masks.cpu().numpy().view(np.uint8),
                             bitorder="little").reshape(K, -1)[:, :H * W]
        ok = ~bad.reshape(-1)
        assert_same(bits[:, ok], rr["mask"].reshape(K, -1)[:, ok], f"masks after render {r + 1}")
        got_b = fr.budget.cpu().numpy().reshape(K, -1)[:, ok]
        np.testing.assert_allclose(got_b, budget.reshape(K, -1)[:, ok], rtol=1e-3, atol=1e-10)
        pruned = int(((rr["mask"] == 0) & (om == 1)).sum())
        stats.append((pruned, int(rr["flips"].sum())))
        print(f"render {r + 1}: max-abs {e:.3g}, flagged {int(bad.sum())}, pruned {pruned}, "
              f"re-activated {stats[-1][1]}", flush=True)
        state = rr["mask"]
    assert stats[0][0] > 1000 and stats[0][1] == 0
    assert stats[1][1] > 500 and stats[1][0] > 1000


@pytest.mark.parametrize("cells_kind,tile", [("grid", (16, 16)), ("kd", (16, 16)),
                                             ("grid", (32, 8))])
def test_cross_boundary_filter_matches_oracle(torch_gpu, cells_kind, tile):
    """Per-ray cross-boundary filtering on K = 8 cells: the filter bits of
    every Gaussian bit-exact where the oracle's decision is not within
    rounding reach, and the filtered renders, composition, masks and
    gradients against the oracle run with its own bits."""
    print(f"case: cross-boundary filter k8 {cells_kind} tile {tile}", flush=True)
    st = synth.RenderSettings(tile_w=tile[0], tile_h=tile[1])
    torch = torch_gpu
    from paper_2606_18588_amd import binding as B
    scene = synth.make_cube_scene(6, 9000, log_scale=(-3.0, 0.5))
    if cells_kind == "grid":
        cam = synth.camera_from_rows(
            np.array([[1, 0, 0], [0, 0.9950, -0.0998], [0, 0.0998, 0.9950]]), (0.13, 0.21, -3.0),
            96, 80, 70.0)
        xe, ye = [-1.0, -0.5, 0.0, 0.5, 1.0], [-1.0, 0.0, 1.0]
        part = synth.grid_partition(scene, xe, ye)
        boxes = grid_cells_xy(xe, ye)
        scenes = part.cell_scenes(scene)
    else:
        cam = synth.look_at_camera((2.4, -2.9, 1.6), (0.0, 0.1, 0.0), 112, 84, hfov_deg=55.0)
        boxes_t, cell_of = B.sx_kd_partition(scene.means, 8)
        boxes = [synth.Cell(lo, hi) for lo, hi in boxes_t]
        scenes = [scene.subset(np.nonzero(cell_of == k)[0]) for k in range(8)]
    K, H, W = 8, cam.height, cam.width
    from paper_2606_18588_amd.pipeline import Frame, GaussianParams
    params = [GaussianParams.from_scene(c) for c in scenes]
    fr = Frame(params, boxes, cam, st, cross_filter=True)
    fr.init_masks()
    out = fr.forward(update_masks=True).cpu().numpy()
    torch.cuda.synchronize()
    vis = oracle.visibility(boxes, cam)
    assert not vis["flags"].any()
    xfs = oracle.cross_filters(scenes, boxes, cam, st)
    nfilt = 0
    for k in range(K):
        got = fr.views[k].xf.cpu().numpy().view(np.uint32)[:scenes[k].n]
        ok = xfs[k]["amb"] == 0
        assert_same(got[ok], xfs[k]["xf"][ok], f"filter bits of cell {k}")
        nfilt += int((xfs[k]["xf"] != 0).sum())
    assert nfilt > 100
    ref = oracle.forward(scenes, boxes, cam, st, xfilters=xfs)
    fl = ref.comp["flags"].copy()
    for p in ref.parts:
        fl |= p["flags"]
    cmax = max(float(oracle.preprocess(c, cam, ST)["rgb"].max()) for c in scenes)
    e, nf = compare_image(out[..., :3], ref.comp["rgb"], fl, 1e-4, K * jump_bound(ST, cmax))
    compare_image(out[..., 3], ref.comp["T"], fl, 1e-4, 1.0)
    unf = oracle.forward(scenes, boxes, cam, ST)
    changed = np.abs(unf.comp["rgb"] - ref.comp["rgb"]).max(-1) > 1e-3
    assert changed.sum() > 50  # the filter changes the image
    ok = fl == 0
    for k in range(K):
        assert_same(fr.views[k].nblend.cpu().numpy()[ok], ref.parts[k]["nblend"][ok],
                    f"blended pairs of cell {k}")
    bits = np.unpackbits(fr.masks.cpu().numpy().view(np.uint8), bitorder="little").reshape(K, -1)[:, :H * W]
    assert_same(bits[:, ok.reshape(-1)], ref.comp["mask"].reshape(K, -1)[:, ok.reshape(-1)],
                "saturation masks")
    print(f"cross filter {cells_kind}: {nfilt} filtered Gaussians, {int(changed.sum())} pixels "
          f"changed, max-abs {e:.3g}, flagged {nf}", flush=True)
    # backward: upstream gradient on unflagged pixels
    rng = np.random.default_rng(31)
    d = (rng.normal(size=(H, W, 4)) * ok[..., None]).astype(np.float32)
    grads = [p.zeros_like() for p in params]
    fr.backward(torch.as_tensor(d).cuda(), grads)
    torch.cuda.synchronize()
    gref = oracle.backward(scenes, boxes, cam, st, ref, d[..., :3].astype(np.float64),
                           d[..., 3].astype(np.float64), xfilters=xfs)
    for k in range(K):
        v = fr.views[k].n_tiles.cpu().numpy() > 0
        if not v.any():
            continue
        for name in ("means", "log_scales", "quats", "opacity_logits", "sh"):
            got = getattr(grads[k], name).cpu().numpy()[v]
            check_grad(got, gref[k][name][v], f"filtered cell {k} {name}")


def test_cross_boundary_filter_degenerate_cases(torch_gpu):
    """One cell (no other box to span): every filter bit is zero and the
    filtered render equals the unfiltered one bit for bit; an empty cell
    renders the identity with the filter on; the batched renders refuse a
    projection that asks for the filter."""
    print("case: cross-boundary filter k1 / empty / batched", flush=True)
    torch = torch_gpu
    from paper_2606_18588_amd import binding as B
    from paper_2606_18588_amd.pipeline import Frame, GaussianParams
    scene, cam = synth.tiny_scene(), synth.tiny_camera(100, 70)
    box = [big_box()]
    plain = Frame([GaussianParams.from_scene(scene)], box, cam, ST)
    filt = Frame([GaussianParams.from_scene(scene)], box, cam, ST, cross_filter=True)
    a = plain.forward().cpu().numpy()
    b = filt.forward().cpu().numpy()
    torch.cuda.synchronize()
    assert not filt.views[0].xf.cpu().numpy()[:scene.n].any()
    assert np.array_equal(a, b)
    empty = Frame([GaussianParams.from_scene(scene.subset(np.array([], np.int64)))], box, cam, ST,
                  cross_filter=True)
    out = empty.forward().cpu().numpy()
    assert np.all(out[..., :3] == 0) and np.all(out[..., 3] == 1)
    from paper_2606_18588_amd.pipeline import BatchedViews
    bv = BatchedViews(GaussianParams.from_scene(scene), [cam, cam], ST)
    bv.preprocess()
    bv.sort()
    B.set_cross_filter(bv.views[0].c_proj, filt.views[0].xf, filt.omega, 0, 1)
    with pytest.raises(B.SplaxelError) as ei:
        bv.render()
    assert ei.value.code == B.SX_EINVAL
    B.set_cross_filter(bv.views[0].c_proj, None, None, 0, 0)
    bv.render()
    torch.cuda.synchronize()


def test_frame_forward_on_side_streams_bit_identical(torch_gpu):
    """The cells' forward and backward chains spread over four streams give
    the same image, masks and gradients bit for bit as one stream."""
    print("case: frame forward on side streams", flush=True)
    torch = torch_gpu
    from paper_2606_18588_amd.pipeline import Frame, GaussianParams
    scene = synth.make_cube_scene(3, 8000, log_scale=(-3.6, 0.5))
    cam = synth.camera_from_rows(
        np.array([[1, 0, 0], [0, 0.9950, -0.0998], [0, 0.0998, 0.9950]]), (0.13, 0.21, -3.0),
        96, 80, 70.0)
    xe, ye = [-1.0, -0.5, 0.0, 0.5, 1.0], [-1.0, 0.0, 1.0]
    part = synth.grid_partition(scene, xe, ye)
    boxes = grid_cells_xy(xe, ye)
    scenes = part.cell_scenes(scene)
    outs = []
    dout = torch.as_tensor(np.random.default_rng(3).normal(
        size=(cam.height, cam.width, 4)).astype(np.float32)).cuda()
    for streams in (1, 4):
        params = [GaussianParams.from_scene(c) for c in scenes]
        fr = Frame(params, boxes, cam, ST, streams=streams)
        fr.init_masks(geometric=True)
        fr.forward(use_masks=True, sync=True)  # sizes the buffers
        fr.init_masks(geometric=True)
        out = fr.forward(use_masks=True, update_masks=True, sync=False)
        grads = [p.zeros_like() for p in params]
        fr.backward(dout, grads)
        fr.backward(dout, grads, accumulate=True)
        torch.cuda.synchronize()
        outs.append((out.cpu().numpy(), fr.masks.cpu().numpy(),
                     [t.cpu().numpy() for g in grads for t in g.tensors()]))
    assert np.array_equal(outs[0][0], outs[1][0])
    assert np.array_equal(outs[0][1], outs[1][1])
    for a, b in zip(outs[0][2], outs[1][2]):
        assert np.array_equal(a, b)
    # the fused training pass against forward, L1 and backward
    from paper_2606_18588_amd import binding as Bb
    target = torch.as_tensor(np.random.default_rng(4).uniform(
        size=(cam.height, cam.width, 3)).astype(np.float32)).cuda()
    res = []
    for fused in (False, True):
        params = [GaussianParams.from_scene(c) for c in scenes]
        fr = Frame(params, boxes, cam, ST, streams=4)
        fr.init_masks(geometric=True)
        fr.forward(use_masks=True, sync=True)
        fr.init_masks(geometric=True)
        grads = [p.zeros_like() for p in params]
        if fused:
            out = fr.train_l1(target, grads, use_masks=True, update_masks=True, sync=False)
        else:
            out = fr.forward(use_masks=True, update_masks=True, sync=False)
            dl = torch.empty_like(out)
            Bb.sx_l1_loss(out, target, cam.width, cam.height, dl, None)
            fr.backward(dl, grads)
        torch.cuda.synchronize()
        res.append([out.cpu().numpy(), fr.masks.cpu().numpy()] +
                   [t.cpu().numpy() for g in grads for t in g.tensors()])
    for a, b in zip(*res):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("K", [1, 8])
def test_composite_l1_fused_equals_three_calls(torch_gpu, K):
    """sx_composite_l1 gives bit for bit the image, masks, loss and partial
    gradients of sx_composite, sx_l1_loss and sx_composite_backward."""
    print(f"case: fused composite + L1 + backward K={K}", flush=True)
    torch = torch_gpu
    from paper_2606_18588_amd import binding as B
    scene = synth.make_cube_scene(3, 8000, log_scale=(-3.6, 0.5))
    cam = synth.camera_from_rows(
        np.array([[1, 0, 0], [0, 0.9950, -0.0998], [0, 0.0998, 0.9950]]), (0.13, 0.21, -3.0),
        97, 81, 70.0)
    if K == 1:
        boxes, scenes = [big_box()], [scene]
    else:
        xe, ye = [-1.0, -0.5, 0.0, 0.5, 1.0], [-1.0, 0.0, 1.0]
        boxes = grid_cells_xy(xe, ye)
        scenes = synth.grid_partition(scene, xe, ye).cell_scenes(scene)
    fr, _ = _frame(torch, scenes, boxes, cam)
    fr.forward()
    H, W = cam.height, cam.width
    target = torch.as_tensor(np.random.default_rng(2).uniform(
        size=(H, W, 3)).astype(np.float32)).cuda()
    parts = [v.partial for v in fr.views]
    words = (H * W + 31) // 32
    res = []
    for fused in (False, True):
        out = torch.empty((H, W, 4), dtype=torch.float32, device="cuda")
        masks = torch.full((K, words), -1, dtype=torch.int32, device="cuda")
        loss = torch.zeros(1, dtype=torch.float32, device="cuda")
        dparts = [torch.empty((H, W, 4), dtype=torch.float32, device="cuda") for _ in range(K)]
        if fused:
            B.sx_composite_l1(parts, boxes, fr.c_cam, fr.c_par, target, out, masks, loss, dparts)
        else:
            dout = torch.empty_like(out)
            B.sx_composite(parts, boxes, fr.c_cam, fr.c_par, out, masks)
            B.sx_l1_loss(out, target, W, H, dout, loss)
            B.sx_composite_backward(parts, boxes, fr.c_cam, fr.c_par, dout, dparts)
        torch.cuda.synchronize()
        res.append([out.cpu().numpy(), masks.cpu().numpy()] + [d.cpu().numpy() for d in dparts])
        res[-1].append(float(loss.item()))
    for a, b in zip(res[0][:-1], res[1][:-1]):
        assert np.array_equal(a, b)
    # the loss sum is an atomic sum of per-wavefront partials: order may differ
    assert abs(res[0][-1] - res[1][-1]) <= 1e-6 * abs(res[0][-1])


def test_composite_kd_cells_matches_oracle(torch_gpu):
    """K = 8 cells from the KD-tree partitioner (boxes bounded on some axes,
    unbounded at the scene's outside): the composition by ray entry order
    and its saturation masks match the oracle's on the same cells."""
    print("case: composite k8 kd-tree cells", flush=True)
    torch = torch_gpu
    from paper_2606_18588_amd import binding as B
    scene = synth.make_cube_scene(4, 9000, log_scale=(-3.6, 0.5))
    cam = synth.look_at_camera((2.4, -2.9, 1.6), (0.0, 0.1, 0.0), 112, 84, hfov_deg=55.0)
    boxes_t, cell_of = B.sx_kd_partition(scene.means, 8)
    ref_boxes, ref_cell = oracle.kd_partition(scene.means, 8)
    assert np.array_equal(cell_of, ref_cell)
    boxes = [synth.Cell(lo, hi) for lo, hi in boxes_t]
    scenes = [scene.subset(np.nonzero(cell_of == k)[0]) for k in range(8)]
    fr, _ = _frame(torch, scenes, boxes, cam)
    fr.init_masks()
    out = fr.forward(update_masks=True).cpu().numpy()
    torch.cuda.synchronize()
    ref = oracle.forward(scenes, boxes, cam, ST)
    fl = ref.comp["flags"].copy()
    for p in ref.parts:
        fl |= p["flags"]
    cmax = max(float(oracle.preprocess(s, cam, ST)["rgb"].max()) for s in scenes)
    e, nf = compare_image(out[..., :3], ref.comp["rgb"], fl, 1e-4, 8 * jump_bound(ST, cmax))
    compare_image(out[..., 3], ref.comp["T"], fl, 1e-4, 1.0)
    masks = fr.masks.cpu().numpy().view(np.uint32)
    bits = np.unpackbits(masks.view(np.uint8), bitorder="little").reshape(8, -1)[:, :cam.width * cam.height]
    okpix = fl.reshape(-1) == 0
    assert_same(bits[:, okpix], ref.comp["mask"].reshape(8, -1)[:, okpix], "saturation masks")
    print(f"composite kd cells: max-abs {e:.3g} flagged {nf}", flush=True)


def test_slab_composite_equals_single_pass(torch_gpu):
    """The paper's Eq. 5 = Eq. 2 claim on the GPU: with t_min = 0, the
    composition of depth-separated slab partials equals the single-pass
    render up to FP32 reassociation."""
    print("case: slab composite", flush=True)
    torch = torch_gpu
    st0 = synth.RenderSettings(t_min=0.0)
    scene, cam = synth.tiny_scene(), synth.tiny_camera()
    edges = synth.quantile_edges(scene.means[:, 2], 8)
    part = synth.axis_slab_partition(scene, 2, edges)
    fr, _ = _frame(torch, part.cell_scenes(scene), part.cells, cam, st0)
    out = fr.forward().cpu().numpy()
    single = _render(torch, scene, cam, st0).partial.cpu().numpy()
    assert np.abs(out[..., :3] - single[..., :3]).max() <= 1e-5
    assert np.abs(out[..., 3] - single[..., 3]).max() <= 1e-5


def test_saturation_culling_next_render(torch_gpu):
    """Temporal saturation masks: the next render with the masks skips the
    saturated (cell, pixel) pairs; the image changes by at most t_min * max c
    and matches the same-frame-culled composition."""
    print("case: saturation masks", flush=True)
    torch = torch_gpu
    from paper_2606_18588_amd import binding as B
    scene = synth.make_cube_scene(11, 6000, log_scale=(-3.2, 0.4), logit_sigma=2.0)
    cam = synth.tiny_camera(64, 64)
    edges = synth.quantile_edges(scene.means[:, 2], 4)
    part = synth.axis_slab_partition(scene, 2, edges)
    scenes = part.cell_scenes(scene)
    fr, _ = _frame(torch, scenes, part.cells, cam)
    fr.init_masks()
    first = fr.forward(update_masks=True).cpu().numpy()
    second = fr.forward(use_masks=True).cpu().numpy()
    frc, _ = _frame(torch, scenes, part.cells, cam, flags=B.SX_FLAG_SAME_FRAME_CULL)
    culled = frc.forward().cpu().numpy()
    ref = oracle.forward(scenes, part.cells, cam, ST)
    assert (ref.comp["mask"] == 0).sum() > 0
    assert np.abs(second - culled).max() <= 1e-6
    assert np.abs(second[..., :3] - first[..., :3]).max() <= ST.t_min * 2.0 + 1e-6


# -------------------------------------------------------------- a7 - a9 --
def _fd_scene(seed0, cam, cells_fn):
    for seed in range(seed0, seed0 + 40):
        sc = synth.fd_scene(seed)
        part = cells_fn(sc)
        fr = oracle.forward(part.cell_scenes(sc), part.cells, cam, ST, delta_q=1e-3)
        fl = np.bitwise_or.reduce([p["flags"] for p in fr.parts])
        if not np.any(fl) and not np.any(fr.comp["flags"]):
            return sc, part
    raise AssertionError("no flag-free scene")


@pytest.mark.parametrize("K", [1, 2, 4])
def test_backward_matches_oracle_and_fd(torch_gpu, K):
    """Kernel gradients (FP32, through sx_backward) against the oracle's
    analytic FP64 gradients, and the oracle against central differences, on
    flag-free 64-Gaussian scenes split into K depth slabs."""
    print(f"case: backward fd scene K={K}", flush=True)
    torch = torch_gpu
    cam = synth.fd_camera()

    def cells(s):
        return synth.axis_slab_partition(s, 2, np.linspace(-0.7, 0.7, K + 1))
    sc, part = _fd_scene(300 + 50 * K, cam, cells)
    scenes = part.cell_scenes(sc)
    fr, params = _frame(torch, scenes, part.cells, cam)
    out = fr.forward()
    rng = np.random.default_rng(K)
    w = rng.normal(size=(cam.height, cam.width, 4)).astype(np.float32)
    dout = torch.as_tensor(w).cuda()
    grads = [p.zeros_like() for p in params]
    fr.backward(dout, grads)
    torch.cuda.synchronize()
    ref = oracle.forward(scenes, part.cells, cam, ST)
    np.testing.assert_allclose(out.cpu().numpy()[..., :3], ref.comp["rgb"], atol=1e-5)
    gref = oracle.backward(scenes, part.cells, cam, ST, ref, w[..., :3].astype(np.float64),
                           w[..., 3].astype(np.float64))
    for k in range(K):
        for name in ("means", "log_scales", "quats", "opacity_logits", "sh"):
            got = getattr(grads[k], name).cpu().numpy().astype(np.float64)
            check_grad(got, gref[k][name], f"K={K} cell {k} {name}")


def test_backward_screen_space_matches_oracle(torch_gpu):
    """Per-Gaussian screen-space gradients (mean2d, conic, opacity, colour)
    of the render backward against the oracle on the tiny workload, excluding
    Gaussians that touch a flagged pixel."""
    print("case: backward screen-space tiny", flush=True)
    torch = torch_gpu
    scene, cam = synth.tiny_scene(), synth.tiny_camera()
    fr, params = _frame(torch, [scene], [big_box()], cam)
    out = fr.forward()
    target = torch.as_tensor(synth.random_image(101, cam.width, cam.height)).cuda()
    from paper_2606_18588_amd import binding as B
    dout = torch.empty_like(out)
    B.sx_l1_loss(out, target, cam.width, cam.height, dout, None)
    grads = [params[0].zeros_like()]
    fr.backward(dout, grads)
    torch.cuda.synchronize()
    d = dout.cpu().numpy()
    ref = oracle.forward([scene], [big_box()], cam, ST)
    rb = oracle.render_backward(scene, cam, ST, d[..., :3].astype(np.float64), None, None)
    g2d = fr.views[0].g2d.cpu().numpy()[:, :10]
    pr = oracle.preprocess(scene, cam, ST)
    fl = ref.parts[0]["flags"] != 0
    bad = np.zeros(scene.n, bool)
    ys, xs = np.nonzero(fl)
    for y, x in zip(ys, xs):
        pr_r = pr["pix_rect"]
        bad |= (pr_r[:, 0] <= x) & (x <= pr_r[:, 2]) & (pr_r[:, 1] <= y) & (y <= pr_r[:, 3])
    ok = (pr["valid"] == 1) & ~bad
    for c in range(9):
        check_grad(g2d[ok, c], rb["g2d"][ok, c], f"tiny g2d[{c}]")
    for name in ("means", "opacity_logits", "sh"):
        got = getattr(grads[0], name).cpu().numpy()[ok]
        check_grad(got, rb[name][ok], f"tiny {name}")


def test_backward_walks_every_tile_poisoned_rows(torch_gpu):
    """Every tile is walked and every instance row written: the backward
    workspace is filled with NaN bytes first, on a view where the cube
    covers the centre of a wide image, so that 2,000 of its 2,048
    tiles are empty and the walk's tile order places them in runs (the
    order's shortest-list bucket, filled a wavefront at a time).  The
    screen-space gradients must be finite and match the oracle."""
    print("case: backward with poisoned rows, 1024x512, mostly empty tiles", flush=True)
    torch = torch_gpu
    scene = synth.tiny_scene()
    f = (128 / 2.0) / math.tan(math.radians(30.0))
    cam = synth.camera_from_rows(np.eye(3), (0.0, 0.0, -3.0), 1024, 512, f)
    fr, params = _frame(torch, [scene], [big_box()], cam)
    out = fr.forward()
    target = torch.as_tensor(synth.random_image(103, cam.width, cam.height)).cuda()
    from paper_2606_18588_amd import binding as B
    dout = torch.empty_like(out)
    B.sx_l1_loss(out, target, cam.width, cam.height, dout, None)
    v = fr.views[0]
    v.ensure_backward_buffers()
    v.bwd_ws.fill_(255)
    grads = [params[0].zeros_like()]
    fr.backward(dout, grads)
    torch.cuda.synchronize()
    pr = oracle.preprocess(scene, cam, ST)
    vis = pr["valid"] == 1
    g2d = v.g2d.cpu().numpy()[:, :10]
    assert np.isfinite(g2d[vis]).all()
    d = dout.cpu().numpy()
    ref = oracle.forward([scene], [big_box()], cam, ST)
    rb = oracle.render_backward(scene, cam, ST, d[..., :3].astype(np.float64), None, None)
    fl = ref.parts[0]["flags"] != 0
    bad = np.zeros(scene.n, bool)
    for y, x in zip(*np.nonzero(fl)):
        pr_r = pr["pix_rect"]
        bad |= (pr_r[:, 0] <= x) & (x <= pr_r[:, 2]) & (pr_r[:, 1] <= y) & (y <= pr_r[:, 3])
    ok = vis & ~bad
    print(f"visible {int(vis.sum())}, compared {int(ok.sum())}", flush=True)
    for c in range(9):
        check_grad(g2d[ok, c], rb["g2d"][ok, c], f"wide g2d[{c}]")


# ------------------------------------------------------------------- a10 --
def test_adam_matches_oracle(torch_gpu):
    print("case: adam", flush=True)
    torch = torch_gpu
    from paper_2606_18588_amd import binding as B
    rng = np.random.default_rng(0)
    for n in (1, 3, 1027, 100003):
        p = rng.normal(size=n).astype(np.float32)
        m = np.zeros(n)
        v = np.zeros(n)
        pt = torch.as_tensor(p.copy()).cuda()
        mt = torch.zeros(n, device="cuda")
        vt = torch.zeros(n, device="cuda")
        pr = p.astype(np.float64)
        for step in range(1, 4):
            g = rng.normal(size=n).astype(np.float32)
            B.sx_adam(pt, torch.as_tensor(g).cuda(), mt, vt, step, 1e-2)
            oracle.adam_step(pr, g.astype(np.float64), m, v, step, 1e-2)
        np.testing.assert_allclose(pt.cpu().numpy(), pr, atol=1e-5)


def test_l1_matches_oracle(torch_gpu):
    print("case: l1", flush=True)
    torch = torch_gpu
    from paper_2606_18588_amd import binding as B
    rng = np.random.default_rng(1)
    H, W = 37, 53
    out = rng.uniform(size=(H, W, 4)).astype(np.float32)
    tgt = rng.uniform(size=(H, W, 3)).astype(np.float32)
    ot = torch.as_tensor(out).cuda()
    dt = torch.empty_like(ot)
    ls = torch.zeros(1, device="cuda")
    B.sx_l1_loss(ot, torch.as_tensor(tgt).cuda(), W, H, dt, ls)
    L, g = oracle.l1_loss(out[..., :3], tgt)
    assert abs(float(ls.item()) - L) < 1e-5
    np.testing.assert_allclose(dt.cpu().numpy()[..., :3], g, rtol=1e-6)
    assert np.all(dt.cpu().numpy()[..., 3] == 0)


def test_invalid_arguments_rejected(torch_gpu):
    print("case: invalid args", flush=True)
    torch = torch_gpu
    from paper_2606_18588_amd import binding as B
    scene, cam = synth.tiny_scene(n=10), synth.tiny_camera()
    _, v = _cell_view(torch, scene, cam)
    bad = B.params(synth.RenderSettings(tile_w=12), 0)
    with pytest.raises(B.SplaxelError) as ei:
        B.sx_preprocess(v.c_g, v.c_cam, bad, v.c_proj)
    assert ei.value.code == B.SX_EINVAL
    bad = B.params(ST, 4)
    with pytest.raises(B.SplaxelError):
        B.sx_preprocess(v.c_g, v.c_cam, bad, v.c_proj)


# ------------------------------------------------- screen list (merged walk)
@pytest.mark.skip(reason="the screen-list path is switched off: the run that introduced it "
                         "ended in a GPU memory fault whose cause is not yet shown")
@pytest.mark.parametrize("n_near", [32, 400])
def test_screen_list_sort_render_backward(torch_gpu, n_near):
    """Gaussians whose footprint covers the whole view are kept once in the
    screen list and merged into every tile's walk by (depth, index).  With
    32 near-camera Gaussians (9 cover the view) and with 400 (screen list
    and walks longer than one 64-entry batch): the expanded lists equal the
    oracle's sorted instances, pixels match the oracle, pixels are equal
    across tile shapes, and screen-space gradients match the oracle."""
    print(f"case: screen list tiny n_near={n_near}", flush=True)
    torch = torch_gpu
    from paper_2606_18588_amd import binding as B
    scene, cam = synth.screen_scene(n_near=n_near), synth.tiny_camera()
    _, v = _cell_view(torch, scene, cam)
    v.preprocess()
    counts = v.sort(sync=True)
    torch.cuda.synchronize()
    r = v.ranges.cpu().numpy().view(np.uint32)
    n_screen = int(r[-1][1])
    assert n_screen >= (9 if n_near == 32 else 65), n_screen
    keys, vals, ranges = oracle.sort_keys(scene, cam, ST)
    _check_lists(v, counts, keys, vals, ranges)
    # forward
    v.render(None, want_depth=True)
    torch.cuda.synchronize()
    ref = oracle.render(scene, cam, ST)
    part = v.partial.cpu().numpy()
    cmax = float(oracle.preprocess(scene, cam, ST)["rgb"].max())
    compare_image(part[..., :3], ref["C"], ref["flags"], 1e-4, jump_bound(ST, cmax))
    compare_image(part[..., 3], ref["T"], ref["flags"], 1e-4, 1.0)
    fl = ref["flags"] != 0
    assert_same(v.nblend.cpu().numpy()[~fl], ref["nblend"][~fl], "blended pairs per pixel")
    if n_near == 400:
        assert int(v.last.max().item()) > 64  # walks span several merge batches
    for tile in ((32, 8), (8, 8)):
        st2 = synth.RenderSettings(tile_w=tile[0], tile_h=tile[1])
        assert_same(_render(torch, scene, cam, st2).partial.cpu().numpy(), part,
                    f"partials across tile shapes {tile}")
    # backward (screen-space gradients of the render)
    fr, params = _frame(torch, [scene], [big_box()], cam)
    out = fr.forward()
    target = torch.as_tensor(synth.random_image(101, cam.width, cam.height)).cuda()
    dout = torch.empty_like(out)
    B.sx_l1_loss(out, target, cam.width, cam.height, dout, None)
    grads = [params[0].zeros_like()]
    fr.backward(dout, grads)
    torch.cuda.synchronize()
    d = dout.cpu().numpy()
    rb = oracle.render_backward(scene, cam, ST, d[..., :3].astype(np.float64), None, None)
    g2d = fr.views[0].g2d.cpu().numpy()[:, :10]
    pr = oracle.preprocess(scene, cam, ST)
    bad = np.zeros(scene.n, bool)
    for y, x in zip(*np.nonzero(fl)):
        pr_r = pr["pix_rect"]
        bad |= (pr_r[:, 0] <= x) & (x <= pr_r[:, 2]) & (pr_r[:, 1] <= y) & (y <= pr_r[:, 3])
    ok = (pr["valid"] == 1) & ~bad
    assert ok[-n_near:].any()
    for c in range(9):
        check_grad(g2d[ok, c], rb["g2d"][ok, c], f"screen list g2d[{c}]")
