"""Parity of the usage forms at the sizes their benchmarks run:

- batched training views: the 15M-Gaussian scene (Morton order), two of the
  16 uneven views in one batched preprocess / render / render-backward
  launch with the autotuned 16x32 tiles; sampled tiles of both views against
  the oracle, and the batched backward (upstream gradient on sampled pixels
  of the first view) against the oracle's gradients;
- serving: the 30M-Gaussian scene, a 3840x2160 request served in a batch
  with a small one; sampled tiles of the 4K image against the oracle.
"""
import math

import numpy as np
import pytest

import oracle
import synth
from gpu_helpers import (check_grad, check_grad_scaled, compare_image, jump_bound, param_scales,
                         need_gpu, rec_fields)

pytestmark = pytest.mark.gpu


def _sample_mask(cam, st, seed, count):
    tx = (cam.width + st.tile_w - 1) // st.tile_w
    ty = (cam.height + st.tile_h - 1) // st.tile_h
    rng = np.random.default_rng(seed)
    tiles = set(int(x) for x in rng.choice(tx * ty, size=count, replace=False))
    tiles |= {tx - 1, ty * tx - 1}  # ragged right column and bottom row
    m = np.zeros((cam.height, cam.width), np.uint8)
    for t in tiles:
        x0, y0 = (t % tx) * st.tile_w, (t // tx) * st.tile_h
        m[y0:y0 + st.tile_h, x0:x0 + st.tile_w] = 1
    return m


def test_fullsize_batched_views(torch_gpu_fs):
    torch = torch_gpu_fs
    from paper_2606_18588_amd.pipeline import BatchedViews, GaussianParams, spatial_order
    print("case: full-size batched views, 15M Gaussians, 2 uneven views, 16x32 tiles",
          flush=True)
    st = synth.RenderSettings(tile_w=16, tile_h=32)
    scene = synth.g15_scene()
    scene = scene.subset(spatial_order(scene.means))
    cams = synth.g15_cameras()[:2]
    params = GaussianParams.from_scene(scene)
    bv = BatchedViews(params, cams, st)
    bv.preprocess()
    bv.sort(sync=True)
    bv.render()
    torch.cuda.synchronize()
    masks = [_sample_mask(c, st, 40 + k, 20) for k, c in enumerate(cams)]
    for k, (v, c, m) in enumerate(zip(bv.views, cams, masks)):
        ref = oracle.render(scene, c, st, mask=m)
        on = m == 1
        part = v.partial.cpu().numpy()
        cmax = float(rec_fields(v.rec)["rgb"][v.n_tiles.cpu().numpy() > 0].max())
        e, nf = compare_image(part[on][:, :3], ref["C"][on], ref["flags"][on], 1e-4,
                              jump_bound(st, cmax), max_flagged=0.05)
        compare_image(part[on][:, 3], ref["T"][on], ref["flags"][on], 1e-4, 1.0)
        print(f"batched view {k} {c.width}x{c.height}: max-abs {e:.3g} flagged {nf}", flush=True)
        if k == 0:
            ok0 = on & (ref["flags"] == 0)
    # backward of both views in one launch; only view 0 carries a gradient
    rng = np.random.default_rng(29)
    for k, v in enumerate(bv.views):
        v.ensure_backward_buffers()
        d = rng.normal(size=(v.H, v.W, 4)) * (ok0[..., None] if k == 0 else 0.0)
        v.dpartial.copy_(torch.as_tensor(d.astype(np.float32)).cuda())
    d0 = bv.views[0].dpartial.cpu().numpy()
    grads = params.zeros_like()
    bv.render_backward()
    bv.preprocess_backward(grads)
    torch.cuda.synchronize()
    rb = oracle.render_backward(scene, cams[0], st, d0[..., :3].astype(np.float64),
                                d0[..., 3].astype(np.float64), None, mask=masks[0])
    vis = bv.views[0].n_tiles.cpu().numpy() > 0
    assert (np.abs(rb["g2d"]).max(1) > 0).sum() > 100
    g2d = bv.views[0].g2d.cpu().numpy()[:, :10]
    for c in range(9):
        check_grad_scaled(g2d[vis, c], rb["g2d"][vis, c], rb["g2d_scale"][vis, c],
                          f"15M batched g2d[{c}]")
    pb = oracle.preprocess_backward(scene, cams[0], st, bv.views[0].g2d.cpu().numpy())
    ps = param_scales(scene, cams[0], st, rb["g2d_scale"], vis)
    for name in ("means", "log_scales", "quats", "opacity_logits", "sh"):
        got = getattr(grads, name).cpu().numpy()[vis]
        check_grad(got, pb[name][vis], f"15M batched {name} (chain of the kernel's g2d)",
                   tol=1e-5, floor=1e-4)
        check_grad_scaled(got, rb[name][vis], ps[name], f"15M batched {name}")


def test_fullsize_served_4k_request(torch_gpu_fs):
    torch = torch_gpu_fs
    from paper_2606_18588_amd.pipeline import GaussianParams, spatial_order
    from paper_2606_18588_amd.serve import Server
    print("case: full-size serving, 30M Gaussians, 3840x2160 request in a batch", flush=True)
    st = synth.RenderSettings()
    scene = synth.g30_scene()
    scene = scene.subset(spatial_order(scene.means))
    params = GaussianParams.from_scene(scene)
    big = synth.aerial_camera((120.0, -340.0, 150.0), 1.1, math.radians(45.0), 3840, 2160)
    small = synth.aerial_camera((-400.0, 250.0, 150.0), 4.0, math.radians(45.0), 640, 360)
    reqs = [synth.Request(0.0, big, 0), synth.Request(0.0, small, 1)]
    srv = Server(params, st, arena_bytes=24 << 30)
    srv.calibrate(big)
    done = srv.serve(reqs, open_loop=False, keep_images=True)
    torch.cuda.synchronize()
    assert sorted(d.rid for d in done) == [0, 1]
    img = srv.images[0].cpu().numpy()
    m = _sample_mask(big, st, 7, 24)
    ref = oracle.render(scene, big, st, mask=m)
    on = m == 1
    e, nf = compare_image(img[on][:, :3], ref["C"][on], ref["flags"][on], 1e-4,
                          jump_bound(st, 1.5), max_flagged=0.05)
    compare_image(img[on][:, 3], ref["T"][on], ref["flags"][on], 1e-4, 1.0)
    print(f"served 4K: max-abs {e:.3g} flagged {nf}", flush=True)
