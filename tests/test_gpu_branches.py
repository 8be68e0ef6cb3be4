"""GPU parity of the backward's less travelled branches (Eq. 6-7) against
the FP64 oracle, on flag-free 64-Gaussian finite-difference scenes (the
oracle's analytic gradients on these scenes are pinned by central
differences in the CPU suite):

- the depth gradient: a loss with the partial depth D through
  sx_render_backward (ddepth given, the reverse walk with its depth terms)
  and the projection backward (the camera z of the mean);
- a background behind the last cell (B_{K+1} = bg) through sx_backward;
- the same-frame saturation cull (SX_FLAG_SAME_FRAME_CULL) through
  sx_composite and sx_backward;
- alpha clamped at alpha_max, which passes no gradient to the opacity or
  the conic.

Gradients are compared per element, relative to each entry's own magnitude
floored at 1e-3 of the largest entry of its family, at 1e-3.
"""
import dataclasses
import math

import numpy as np
import pytest

import oracle
import synth
from gpu_helpers import grad_err, need_gpu

pytestmark = pytest.mark.gpu
ST = synth.RenderSettings()
NAMES = ("means", "log_scales", "quats", "opacity_logits", "sh")
ALL = synth.Cell((-math.inf,) * 3, (math.inf,) * 3)


@pytest.fixture(scope="module")
def torch_gpu():
    need_gpu()
    import torch
    return torch


def _flag_free(scenes_fn, cells, cam, st, seeds, accept=lambda fr: True, **kw):
    """First seed whose (FP32) cell scenes render with no flagged pixel."""
    for seed in seeds:
        scenes = [s.astype(np.float32) for s in scenes_fn(seed)]
        fr = oracle.forward(scenes, cells, cam, st, delta_q=1e-3, **kw)
        fl = np.bitwise_or.reduce([p["flags"] for p in fr.parts]) | fr.comp["flags"]
        if not fl.any() and accept(fr):
            return scenes
    raise AssertionError("no flag-free scene")


def _check_grads(got_list, ref_list, tol=1e-3, names=NAMES):
    worst = {}
    for k, (got, ref) in enumerate(zip(got_list, ref_list)):
        for name in names:
            g = getattr(got, name).cpu().numpy().astype(np.float64)
            e = grad_err(g, ref[name])
            worst[(k, name)] = e
            assert e <= tol, (k, name, e)
    print("per-element gradient errors:",
          {f"{k}:{n}": float(f"{e:.3g}") for (k, n), e in worst.items()}, flush=True)


def _weights(seed, cam):
    rng = np.random.default_rng(seed)
    return (rng.normal(size=(cam.height, cam.width, 3)).astype(np.float32),
            rng.normal(size=(cam.height, cam.width)).astype(np.float32),
            rng.normal(size=(cam.height, cam.width)).astype(np.float32))


def test_render_backward_depth_gradient_matches_oracle(torch_gpu):
    """L = sum wC.C + wT.T + wD.D over one cell: the partial depth's
    gradient enters the reverse walk (k_render_bwd with its depth terms) and
    reaches the means through the camera z in the projection backward."""
    print("case: depth gradient through sx_render_backward (fd scene)", flush=True)
    torch = torch_gpu
    from paper_2606_18588_amd.pipeline import CellView, GaussianParams
    cam = synth.fd_camera()
    sc = _flag_free(lambda s: [synth.fd_scene(s)], [ALL], cam, ST, range(400, 440))[0]
    wc, wt, wd = _weights(11, cam)
    params = GaussianParams.from_scene(sc)
    v = CellView(params, cam, ST)
    v.preprocess()
    v.sort(sync=True)
    v.render(None, want_depth=True)
    dpart = torch.as_tensor(np.concatenate([wc, wt[..., None]], -1)).cuda()
    dd = torch.as_tensor(wd).cuda()
    grads = params.zeros_like()
    v.render_backward(dpart, dd)
    v.preprocess_backward(grads)
    torch.cuda.synchronize()
    ref = oracle.render(sc, cam, ST)
    np.testing.assert_allclose(v.depth.cpu().numpy(), ref["D"], rtol=1e-5, atol=1e-5)
    rb = oracle.render_backward(sc, cam, ST, wc.astype(np.float64), wt.astype(np.float64),
                                wd.astype(np.float64))
    vis = v.n_tiles.cpu().numpy() > 0
    g2d = v.g2d.cpu().numpy()[:, :10]
    assert np.abs(rb["g2d"][vis, 9]).max() > 0
    for c in range(10):
        e = grad_err(g2d[vis, c], rb["g2d"][vis, c])
        assert e <= 1e-3, ("g2d", c, e)
    _check_grads([grads], [rb])


def _frame_grads(torch, scenes, cells, cam, st, flags, wr, wt):
    from paper_2606_18588_amd.pipeline import Frame, GaussianParams
    params = [GaussianParams.from_scene(s) for s in scenes]
    fr = Frame(params, cells, cam, st, flags=flags)
    out = fr.forward()
    dout = torch.as_tensor(np.concatenate([wr, wt[..., None]], -1)).cuda()
    grads = [p.zeros_like() for p in params]
    fr.backward(dout, grads)
    torch.cuda.synchronize()
    return out.cpu().numpy(), grads


def test_backward_background_matches_oracle(torch_gpu):
    """bg = (0.3, 0.6, 0.9) behind two depth slabs: the transmittance
    gradient of each cell sees the background in the colour behind it."""
    print("case: background term through sx_backward (K=2 slabs)", flush=True)
    torch = torch_gpu
    st = dataclasses.replace(ST, bg=(0.3, 0.6, 0.9))
    cam = synth.fd_camera()
    part_of = lambda s: synth.axis_slab_partition(s, 2, [-10.0, 0.0, 10.0])
    cells = part_of(synth.fd_scene(0)).cells

    def scenes_of(seed):
        s = synth.fd_scene(seed)
        return part_of(s).cell_scenes(s)
    scenes = _flag_free(scenes_of, cells, cam, st, range(500, 540))
    wr, wt, _ = _weights(12, cam)
    out, grads = _frame_grads(torch, scenes, cells, cam, st, 0, wr, wt)
    fr = oracle.forward(scenes, cells, cam, st)
    np.testing.assert_allclose(out[..., :3], fr.comp["rgb"], atol=1e-5)
    np.testing.assert_allclose(out[..., 3], fr.comp["T"], atol=1e-5)
    ref = oracle.backward(scenes, cells, cam, st, fr, wr.astype(np.float64),
                          wt.astype(np.float64))
    _check_grads(grads, ref)


def test_backward_same_frame_cull_matches_oracle(torch_gpu):
    """SX_FLAG_SAME_FRAME_CULL with t_min = 0.05: the back slab is the
    identity behind a saturated prefix, in the composition and in the
    backward (it gets no gradient there)."""
    print("case: same-frame saturation cull through sx_backward (K=2 slabs)", flush=True)
    torch = torch_gpu
    from paper_2606_18588_amd import binding as B
    st = dataclasses.replace(ST, t_min=0.05)
    cam = synth.fd_camera()
    cells = synth.same_frame_fd_scenes(0)[1]

    def culls(fr):
        return int((fr.comp["mask"][1] == 0).sum()) >= 20
    scenes = _flag_free(lambda s: synth.same_frame_fd_scenes(s)[0], cells, cam, st,
                        range(700, 760), accept=culls, same_frame_cull=True)
    wr, wt, _ = _weights(14, cam)
    out, grads = _frame_grads(torch, scenes, cells, cam, st, B.SX_FLAG_SAME_FRAME_CULL,
                              wr, wt)
    fr = oracle.forward(scenes, cells, cam, st, same_frame_cull=True)
    fr0 = oracle.forward(scenes, cells, cam, st)
    assert np.abs(fr0.comp["rgb"] - fr.comp["rgb"]).max() > 1e-4  # the cull changes pixels
    np.testing.assert_allclose(out[..., :3], fr.comp["rgb"], atol=1e-5)
    np.testing.assert_allclose(out[..., 3], fr.comp["T"], atol=1e-5)
    ref = oracle.backward(scenes, cells, cam, st, fr, wr.astype(np.float64),
                          wt.astype(np.float64), same_frame_cull=True)
    _check_grads(grads, ref)


def test_backward_clamped_alpha_matches_oracle(torch_gpu):
    """A nearly opaque Gaussian in front whose alpha is clamped at 0.99 at
    several pixel centres: those pairs pass gradient to its colour and
    through the transmittance chain but none to its opacity or conic."""
    print("case: clamped alpha through sx_backward (K=1)", flush=True)
    torch = torch_gpu
    cam = synth.fd_camera()
    scenes = _flag_free(lambda s: [synth.clamp_fd_scene(s)], [ALL], cam, ST, range(600, 640))
    sc = scenes[0]
    pr = oracle.preprocess(sc, cam, ST)
    ys, xs = np.mgrid[0:cam.height, 0:cam.width] + 0.5
    dx, dy = xs - pr["mean2d"][0, 0], ys - pr["mean2d"][0, 1]
    a, b, c = pr["conic"][0]
    G = np.exp(-0.5 * (a * dx * dx + 2 * b * dx * dy + c * dy * dy))
    assert int((pr["opacity"][0] * G > ST.alpha_max).sum()) >= 3
    wr, wt, _ = _weights(13, cam)
    out, grads = _frame_grads(torch, [sc], [ALL], cam, ST, 0, wr, wt)
    fr = oracle.forward([sc], [ALL], cam, ST)
    np.testing.assert_allclose(out[..., :3], fr.comp["rgb"], atol=1e-5)
    ref = oracle.backward([sc], [ALL], cam, ST, fr, wr.astype(np.float64),
                          wt.astype(np.float64))
    _check_grads(grads, ref)


def test_backward_after_mask_update_matches_oracle(torch_gpu):
    """Two training passes of one view with temporal saturation masks
    (t_min = 0.05, two opaque slabs): each pass renders with the masks left
    by the previous composition, and its composition clears more bits.  The
    backward of each pass must be the gradient of that pass's forward, i.e.
    use the masks the render used, not the ones its composition wrote."""
    print("case: backward after a mask update (K=2 slabs, two passes)", flush=True)
    torch = torch_gpu
    from paper_2606_18588_amd.pipeline import Frame, GaussianParams
    st = dataclasses.replace(ST, t_min=0.05)
    cam = synth.fd_camera()
    cells = synth.same_frame_fd_scenes(0)[1]

    def culls(fr):
        return int((fr.comp["mask"][1] == 0).sum()) >= 20
    scenes = _flag_free(lambda s: synth.same_frame_fd_scenes(s)[0], cells, cam, st,
                        range(700, 760), accept=culls)
    params = [GaussianParams.from_scene(s) for s in scenes]
    fr = Frame(params, cells, cam, st)
    fr.init_masks()
    K, H, W = len(cells), cam.height, cam.width
    masks = np.ones((K, H, W), np.uint8)
    for step in range(2):
        wr, wt, _ = _weights(30 + step, cam)
        out = fr.forward(use_masks=True, update_masks=True).cpu().numpy()
        dout = torch.as_tensor(np.concatenate([wr, wt[..., None]], -1)).cuda()
        grads = [p.zeros_like() for p in params]
        fr.backward(dout, grads)
        torch.cuda.synchronize()
        ref = oracle.forward(scenes, cells, cam, st, masks=masks)
        np.testing.assert_allclose(out[..., :3], ref.comp["rgb"], atol=1e-5)
        got_m = np.unpackbits(fr.masks.cpu().numpy().view(np.uint8),
                              bitorder="little").reshape(K, -1)[:, :H * W].reshape(K, H, W)
        np.testing.assert_array_equal(got_m, ref.comp["mask"])
        gref = oracle.backward(scenes, cells, cam, st, ref, wr.astype(np.float64),
                               wt.astype(np.float64), masks=masks)
        _check_grads(grads, gref)
        if step == 0:
            assert (ref.comp["mask"] == 0).sum() >= 20  # the second pass renders fewer pairs
        masks = ref.comp["mask"].astype(np.uint8)
