"""CPU-only checks of the C ABI: the library loads, exports every entry point
include/splaxel.h declares, answers size queries, and rejects invalid
arguments on the host (SX_EINVAL) before anything reaches a device.  No
compute call is made (there is no GPU here)."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "splaxel.h")


@pytest.fixture(scope="module")
def L():
    from paper_2606_18588_amd import binding as B
    if not os.path.exists(B.LIB_PATH):
        from paper_2606_18588_amd import build
        build.build(verbose=False)
    return B.lib()


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sx_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_hot_path_calls():
    names = declared_symbols()
    for n in ("sx_preprocess", "sx_sort", "sx_render_partial", "sx_composite", "sx_backward"):
        assert n in names


def test_every_declared_symbol_is_exported(L):
    out = subprocess.run(["nm", "-D", "--defined-only", L._name], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r"\b(sx_[a-z0-9_]+)\b", out))
    missing = [n for n in declared_symbols() if n not in exported]
    assert not missing, missing
    for n in declared_symbols():
        getattr(L, n)


def test_library_is_built_for_gfx950(L):
    out = subprocess.run(["strings", L._name], capture_output=True, text=True).stdout
    assert "gfx950" in out


def test_version(L):
    from paper_2606_18588_amd import binding as B
    assert "gfx950" in B.sx_version()


def test_size_queries(L):
    from paper_2606_18588_amd import binding as B
    assert B.sx_preprocess_blocks(0) == 1
    assert B.sx_preprocess_blocks(257) == 2
    a = B.sx_sort_workspace_size(1000, 5000, 8, 8)
    b = B.sx_sort_workspace_size(1000, 50000, 8, 8)
    assert 0 < a < b
    # per instance: 16 bytes of per-tile (depth, index) lists and their
    # merge buffer, whatever the grid (each buffer rounded to 256 bytes)
    c = B.sx_sort_workspace_size(1000, 50000, 241, 136)
    d = B.sx_sort_workspace_size(1000, 60000, 241, 136)
    assert abs((d - c) - 16 * 10000) <= 512
    assert abs((b - a) - 16 * 45000) <= 512
    # one 40-byte gradient row per instance and a word per tile
    c = B.sx_backward_workspace_size(5000, 64)
    assert 5000 * 40 <= c <= 5000 * 40 + 64 * 4 + 512
    with pytest.raises(B.SplaxelError) as e:
        B.sx_sort_workspace_size(-1, 10, 2, 2)
    assert e.value.code == B.SX_EINVAL
    with pytest.raises(B.SplaxelError):
        B.sx_sort_workspace_size(10, 1 << 31, 2, 2)


def _cam(B):
    import synth
    return B.camera(synth.tiny_camera())


def test_invalid_arguments_are_rejected_on_host(L):
    from paper_2606_18588_amd import binding as B
    import synth
    cam = _cam(B)
    good = B.params(synth.RenderSettings(), 0)
    g = B.SxGaussians()
    g.n = 10  # null arrays with n > 0
    out = B.SxProjected()
    assert L.sx_preprocess(ctypes.byref(g), ctypes.byref(cam), ctypes.byref(good),
                           ctypes.byref(out), None) == B.SX_EINVAL
    assert b"null" in L.sx_last_error_string()
    g.n = 0
    bad_tile = B.params(synth.RenderSettings(tile_w=12), 0)
    assert L.sx_preprocess(ctypes.byref(g), ctypes.byref(cam), ctypes.byref(bad_tile),
                           ctypes.byref(out), None) == B.SX_EINVAL
    bad_sh = B.params(synth.RenderSettings(), 4)
    assert L.sx_preprocess(ctypes.byref(g), ctypes.byref(cam), ctypes.byref(bad_sh),
                           ctypes.byref(out), None) == B.SX_EINVAL
    bad_alpha = B.params(synth.RenderSettings(alpha_min=0.5, alpha_max=0.4), 0)
    assert L.sx_preprocess(ctypes.byref(g), ctypes.byref(cam), ctypes.byref(bad_alpha),
                           ctypes.byref(out), None) == B.SX_EINVAL
    bad_cam = B.camera(synth.tiny_camera())
    bad_cam.width = 0
    assert L.sx_preprocess(ctypes.byref(g), ctypes.byref(bad_cam), ctypes.byref(good),
                           ctypes.byref(out), None) == B.SX_EINVAL
    # composite: K out of range, empty box
    parts = (ctypes.c_void_p * 1)(1)
    cells = (B.SxCell * 1)()
    assert L.sx_composite(ctypes.c_int32(0), parts, cells, ctypes.byref(cam),
                          ctypes.byref(good), ctypes.c_void_p(1), None, None) == B.SX_EINVAL
    assert L.sx_composite(ctypes.c_int32(17), parts, cells, ctypes.byref(cam),
                          ctypes.byref(good), ctypes.c_void_p(1), None, None) == B.SX_EINVAL
    cells[0].lo[0], cells[0].hi[0] = 1.0, 0.0
    assert L.sx_composite(ctypes.c_int32(1), parts, cells, ctypes.byref(cam),
                          ctypes.byref(good), ctypes.c_void_p(1), None, None) == B.SX_EINVAL
    # sort: undersized workspace, misaligned block sums
    proj = B.SxProjected()
    proj.rec = proj.rect = proj.n_tiles = proj.block_sums = ctypes.c_void_p(256)
    assert L.sx_sort(ctypes.byref(proj), ctypes.c_int64(10), ctypes.byref(cam),
                     ctypes.byref(good), ctypes.c_int64(100), None, ctypes.c_void_p(256),
                     ctypes.c_void_p(256), ctypes.c_void_p(256), ctypes.c_size_t(16), None,
                     None) == B.SX_EINVAL
    assert b"workspace" in L.sx_last_error_string()
    proj.block_sums = ctypes.c_void_p(260)
    assert L.sx_sort(ctypes.byref(proj), ctypes.c_int64(10), ctypes.byref(cam),
                     ctypes.byref(good), ctypes.c_int64(100), None, ctypes.c_void_p(256),
                     ctypes.c_void_p(256), ctypes.c_void_p(256), ctypes.c_size_t(1 << 30), None,
                     None) == B.SX_EINVAL
    assert b"aligned" in L.sx_last_error_string()
    # adam: step must be >= 1
    assert L.sx_adam(ctypes.c_int64(4), ctypes.c_void_p(1), ctypes.c_void_p(1),
                     ctypes.c_void_p(1), ctypes.c_void_p(1), ctypes.c_int32(0),
                     ctypes.c_float(1e-3), ctypes.c_float(0.9), ctypes.c_float(0.999),
                     ctypes.c_float(1e-8), None) == B.SX_EINVAL
    # backward: K out of range
    assert L.sx_backward(ctypes.c_int32(0), None, None, ctypes.byref(cam), ctypes.byref(good),
                         None, ctypes.c_int32(0), None) == B.SX_EINVAL
    # re-evaluating composition: masks and budget are required
    cells[0].lo[0], cells[0].hi[0] = 0.0, 1.0
    assert L.sx_composite_reeval(ctypes.c_int32(1), parts, cells, ctypes.byref(cam),
                                 ctypes.byref(good), ctypes.c_void_p(1), None, None,
                                 ctypes.c_void_p(1), None) == B.SX_EINVAL
    assert L.sx_composite_reeval(ctypes.c_int32(1), parts, cells, ctypes.byref(cam),
                                 ctypes.byref(good), ctypes.c_void_p(1), ctypes.c_void_p(1),
                                 None, None, None) == B.SX_EINVAL
    # cross-boundary filter: cell outside 0..K-1, K out of range, inverted box
    g.n = 10
    g.means = g.log_scales = g.quats = ctypes.c_void_p(1)
    cells2 = (B.SxCell * 2)()
    for c in cells2:
        c.hi[0] = c.hi[1] = c.hi[2] = 1.0
    for K, cell in ((2, 2), (2, -1), (0, 0), (17, 0)):
        assert L.sx_cross_filter(ctypes.byref(g), ctypes.byref(proj), ctypes.c_int32(K), cells2,
                                 ctypes.c_int32(cell), ctypes.byref(cam), ctypes.c_void_p(1),
                                 None) == B.SX_EINVAL, (K, cell)
    cells2[1].lo[2] = 2.0
    assert L.sx_cross_filter(ctypes.byref(g), ctypes.byref(proj), ctypes.c_int32(2), cells2,
                             ctypes.c_int32(0), ctypes.byref(cam), ctypes.c_void_p(1),
                             None) == B.SX_EINVAL
    # a projection that asks for the filter must bring the maps and a valid cell
    proj.xf = ctypes.c_void_p(1)
    proj.n_cells, proj.cell = 2, 0
    assert L.sx_render_partial(ctypes.byref(proj), ctypes.c_void_p(1), ctypes.c_void_p(1),
                               ctypes.byref(cam), ctypes.byref(good), None, ctypes.c_void_p(1),
                               None, ctypes.c_void_p(1), None, None) == B.SX_EINVAL
    proj.omega = ctypes.c_void_p(1)
    proj.cell = 2
    assert L.sx_render_partial(ctypes.byref(proj), ctypes.c_void_p(1), ctypes.c_void_p(1),
                               ctypes.byref(cam), ctypes.byref(good), None, ctypes.c_void_p(1),
                               None, ctypes.c_void_p(1), None, None) == B.SX_EINVAL
    assert b"cross-boundary" in L.sx_last_error_string()


def test_missing_library_fails_loudly(monkeypatch):
    from paper_2606_18588_amd import binding as B
    monkeypatch.setattr(B, "_lib", None)
    monkeypatch.setattr(B, "LIB_PATH", os.path.join(ROOT, "does_not_exist.so"))
    with pytest.raises(RuntimeError, match="no CPU fallback"):
        B.lib()


def test_product_path_never_touches_the_oracle():
    pkg = os.path.join(ROOT, "paper_2606_18588_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                src = open(os.path.join(dirpath, f)).read()
                assert not re.search(r"^\s*(import|from)\s+oracle\b", src, re.M), f
                assert "splat_oracle" not in src, f


def test_kd_partition_matches_oracle(L):
    """The library's KD-tree partitioner (host code) gives the oracle's cells
    and boxes exactly, for several K, and rejects bad arguments."""
    import numpy as np
    import oracle
    import synth
    from paper_2606_18588_amd import binding as B
    sc = synth.make_ground_scene(11, 60000)
    for K in (1, 2, 5, 8, 16):
        b_ref, c_ref = oracle.kd_partition(sc.means, K)
        b, c = B.sx_kd_partition(sc.means, K)
        assert np.array_equal(c, c_ref), K
        for (lo, hi), (lo_r, hi_r) in zip(b, b_ref):
            assert np.array_equal(np.float32(lo), np.float32(lo_r))
            assert np.array_equal(np.float32(hi), np.float32(hi_r))
    with pytest.raises(B.SplaxelError):
        B.sx_kd_partition(sc.means, 17)
    bad = sc.means.copy()
    bad[5, 1] = np.nan
    with pytest.raises(B.SplaxelError):
        B.sx_kd_partition(bad, 4)


def test_noalloc_backward_rejects_capacity_beyond_its_scratch(L):
    """The allocation-free render backward refuses, on the host, a capacity
    whose gradient rows do not fit its static scratch array."""
    from paper_2606_18588_amd import binding as B
    import synth
    cam = B.camera(synth.tiny_camera(128, 128))
    par = B.params(synth.RenderSettings(), 0, 0)
    rows = B.SX_NOALLOC_SCRATCH_BYTES // 40
    code = L.sx_render_backward_noalloc(None, None, None, None, ctypes.c_int64(10),
                                        ctypes.c_int64(rows + 1), ctypes.byref(cam),
                                        ctypes.byref(par), None, None, None, None, None, None,
                                        None)
    assert code == B.SX_EINVAL
    assert b"scratch" in L.sx_last_error_string()


def test_imbalance_and_repartition_plan_match_the_oracle(L):
    """Host parts of a repartition: the imbalance ratio against the
    oracle's, and the plan (each Gaussian's row in its new cell) against
    the oracle's redistribution of the global row indices."""
    import numpy as np
    import oracle
    from paper_2606_18588_amd import binding as B
    rng = np.random.default_rng(4)
    cell_of = rng.integers(0, 5, size=1000).astype(np.int32)
    counts = np.bincount(cell_of, minlength=5)
    assert abs(B.sx_imbalance(counts) - oracle.imbalance(cell_of, 5)) < 1e-12
    dst, cnt = B.sx_repartition_plan(cell_of, 5)
    assert np.array_equal(cnt, counts)
    moved = oracle.repartition([np.arange(1000)], cell_of, 5)
    for k in range(5):
        rows = np.nonzero(cell_of == k)[0]
        assert np.array_equal(moved[k], rows)
        assert np.array_equal(dst[rows], np.arange(len(rows)))
    with pytest.raises(B.SplaxelError):
        B.sx_repartition_plan(np.array([0, 5], np.int32), 5)
    with pytest.raises(B.SplaxelError):
        B.sx_imbalance([0, 0])


def test_bucket_views_greedy_first_fit():
    """Sec. 4.4's scheduler: each view joins the first bucket with no cell in
    common, else opens a new one."""
    from paper_2606_18588_amd.batched import bucket_views
    parts = [{0, 1}, {2}, {1, 3}, {0}, {3}, set(), {2, 4}]
    assert bucket_views(parts) == [[0, 1, 4, 5], [2, 3, 6]]
    assert bucket_views([{0}, {0}, {0}]) == [[0], [1], [2]]


def test_server_batch_width_from_memory_budget():
    """The serving loop's view slots hold a whole-scene projection each, so
    the batch width comes from the slot memory budget: 60 bytes per Gaussian
    plus the largest view's pixel buffers per slot, inflight x width slots
    within the budget, never below one view or above max_batch."""
    from paper_2606_18588_amd import binding as B
    from paper_2606_18588_amd.serve import batch_width, slot_bytes
    n, px, tiles = 30_000_000, 3840 * 2160, 240 * 135
    per = slot_bytes(n, px, tiles)
    assert per == 60 * n + 8 * B.sx_preprocess_blocks(n) + 8 * (tiles + 1) + 36 * px
    assert batch_width(16, 2, per, 32 * per) == 16          # fits: unchanged
    assert batch_width(16, 2, per, 14 * per + per // 2) == 7  # 2 x 7 slots fit, 2 x 8 do not
    assert batch_width(16, 2, per, per) == 1                  # at least one view
    # a 120M-Gaussian scene: 7.5 GB per slot, 106 GB of budget -> 7 views per batch
    big = slot_bytes(120_000_000, px, tiles)
    assert batch_width(16, 2, big, 106 << 30) == (106 << 30) // (2 * big)
