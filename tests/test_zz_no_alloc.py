"""The allocation-free render backward (sx_render_backward_noalloc, for
callers that cannot allocate device memory) against sx_render_backward with
a caller workspace: the same kernels, so the screen-space gradients must be
bit-identical, on two calls in a row through the C ABI, the second on a
smaller view and scene than the first (the static scratch keeps the first
call's rows, which the second must not read)."""
import numpy as np
import pytest

import synth
from gpu_helpers import assert_same, need_gpu

pytestmark = pytest.mark.gpu
ST = synth.RenderSettings()


def test_noalloc_render_backward_matches_workspace_form():
    need_gpu()
    import torch
    from paper_2606_18588_amd import binding as B
    from paper_2606_18588_amd.pipeline import CellView, GaussianParams
    cases = [(synth.tiny_scene(seed=0, n=5000), synth.tiny_camera(128, 128), True),
             (synth.tiny_scene(seed=2, n=1500), synth.tiny_camera(72, 56), False)]
    rng = np.random.default_rng(3)
    for k, (scene, cam, with_depth) in enumerate(cases):
        print(f"case: noalloc render backward, call {k}: {scene.n} Gaussians, "
              f"{cam.width}x{cam.height}, depth gradient {with_depth}", flush=True)
        params = GaussianParams.from_scene(scene)
        v = CellView(params, cam, ST)
        v.preprocess()
        counts = v.sort(sync=True)
        v.render(None, want_depth=with_depth)
        v.ensure_backward_buffers()
        need = B.sx_backward_workspace_size(v.capacity, v.tiles)
        assert need <= B.SX_NOALLOC_SCRATCH_BYTES
        d = rng.normal(size=(cam.height, cam.width, 4)).astype(np.float32)
        v.dpartial.copy_(torch.as_tensor(d).cuda())
        dd = (torch.as_tensor(rng.normal(size=(cam.height, cam.width)).astype(np.float32)).cuda()
              if with_depth else None)
        g_ref = torch.full_like(v.g2d, float("nan"))
        g_new = torch.full_like(v.g2d, float("nan"))
        B.sx_render_backward(v.c_proj, v.vals, v.ranges, v.ws, params.n, v.capacity, v.bwd_ws,
                             v.c_cam, v.c_par, None, v.partial, v.last, v.dpartial, dd, g_ref)
        B.sx_render_backward_noalloc(v.c_proj, v.vals, v.ranges, v.ws, params.n, v.capacity,
                                     v.c_cam, v.c_par, None, v.partial, v.last, v.dpartial, dd,
                                     g_new)
        torch.cuda.synchronize()
        vis = v.n_tiles.cpu().numpy() > 0
        a, b = g_new.cpu().numpy(), g_ref.cpu().numpy()
        assert counts[0] > 0 and np.abs(b[vis][:, :10]).max() > 0
        assert_same(a[vis].view(np.uint32), b[vis].view(np.uint32), f"g2d call {k}")
        assert np.isnan(a[~vis]).all()  # rows of culled Gaussians untouched
