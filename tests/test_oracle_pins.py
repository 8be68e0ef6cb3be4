"""Pins of the FP64 oracle against facts fixed by the paper and by
mathematics (closed forms, invariants, library routines, brute force), so
that the oracle is trusted before any kernel is compared with it.

Each test names the passage it pins: the paper's Eq. 1 (alpha), Eq. 2
(blending), Eq. 3-4 (partials), Eq. 5 and the claim that it equals Eq. 2
(composition), Eq. 6-7 (gradients), the saturation rule of the redundancy
reduction section, and the projection step of the background section.
"""
import math

import numpy as np
import pytest

import synth

ST = synth.RenderSettings()


def _sigmoid(x):
    return 1.0 / (1.0 + math.exp(-x))


def _one(mean, log_scale, quat, logit, rgb):
    """A Scene holding the given Gaussians (SH degree 0 colour = rgb)."""
    mean = np.atleast_2d(np.asarray(mean, np.float64))
    n = mean.shape[0]
    rgb = np.broadcast_to(np.asarray(rgb, np.float64), (n, 3))
    sh = ((rgb - 0.5) * 2.0 * math.sqrt(math.pi))[:, None, :]
    return synth.Scene(
        mean.astype(np.float32),
        np.broadcast_to(np.asarray(log_scale, np.float64), (n, 3)).astype(np.float32).copy(),
        np.broadcast_to(np.asarray(quat, np.float64), (n, 4)).astype(np.float32).copy(),
        np.broadcast_to(np.asarray(logit, np.float64), (n,)).astype(np.float32).copy(),
        sh.astype(np.float32))


def _col(sc, i=0):
    """Colour that degree-0 SH coefficients stored in FP32 evaluate to:
    k0 / (2 sqrt(pi)) + 0.5 (the DC real harmonic is 1/(2 sqrt(pi)))."""
    return sc.sh[i, 0].astype(np.float64) / (2.0 * math.sqrt(math.pi)) + 0.5


def _axis_cam(size=64, f=50.0, centre=32.5):
    # camera at (0,0,-3) looking +z; the optical axis hits pixel `centre`
    return synth.camera_from_rows(np.eye(3), (0.0, 0.0, -3.0), size, size, f,
                                  cx=centre, cy=centre)


# ----------------------------------------------------------------- Eq. 1-2
def test_single_gaussian_centre_alpha_equals_opacity(orc):
    """A Gaussian projected exactly onto a pixel centre has alpha = o there
    (Eq. 1 with d = 0), so C = c min(o, 0.99) and T = 1 - min(o, 0.99)."""
    cam = _axis_cam()
    for logit in (-1.3, 0.5, 6.0):
        rgb = (0.25, 0.5, 0.75)
        sc = _one([0, 0, 0], (-3.0, -3.2, -2.9), (1, 0, 0, 0), logit, rgb)
        r = orc.render(sc, cam, ST)
        o = _sigmoid(float(np.float32(logit)))
        a = min(o, float(np.float32(0.99)))
        c = r["C"][32, 32]
        np.testing.assert_allclose(c, _col(sc) * a, rtol=0, atol=1e-15)
        np.testing.assert_allclose(c, np.array(rgb) * a, rtol=0, atol=1e-7)
        assert abs(r["T"][32, 32] - (1 - a)) < 1e-12
        assert r["nblend"][32, 32] == 1


def test_on_axis_ewa_closed_form(orc):
    """Projection step: on the optical axis with R = I, J W Sigma W^T J^T is
    diag((f s_x / z)^2, (f s_y / z)^2); alpha off-centre follows Eq. 1."""
    cam = _axis_cam()
    ls = np.array([-3.0, -2.6, -2.2], np.float32)
    sc = _one([0, 0, 0.5], ls, (1, 0, 0, 0), 0.7, (0.3, 0.3, 0.3))
    pr = orc.preprocess(sc, cam, ST)
    z = 3.5
    s = np.exp(ls.astype(np.float64))
    eps = float(np.float32(ST.eps2d))
    vx, vy = (50.0 * s[0] / z) ** 2 + eps, (50.0 * s[1] / z) ** 2 + eps
    np.testing.assert_allclose(pr["cov2d"][0], [vx, 0.0, vy], rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(pr["conic"][0], [1 / vx, 0.0, 1 / vy], rtol=1e-12)
    assert pr["depth"][0] == z
    r = orc.render(sc, cam, ST)
    o = _sigmoid(float(np.float32(0.7)))
    for (px, py) in [(33, 32), (34, 33), (31, 30)]:
        dx, dy = px + 0.5 - 32.5, py + 0.5 - 32.5
        a = o * math.exp(-0.5 * (dx * dx / vx + dy * dy / vy))
        if a < 1 / 255:
            continue
        assert abs(r["C"][py, px, 0] - _col(sc)[0] * a) < 1e-15


def test_frustum_cull_by_mean(orc):
    """Projection step: Gaussians whose mean lies outside the camera's field
    of view are discarded by their mean.  With an off-centre principal point
    (cx=20 of 64, cy=30 of 48, f=50, z=3) the pixel offset of a mean is
    50 x / 3; the field of view widened by the guard g spans
    [-g cx, g (W - cx)] x [-g cy, g (H - cy)].  Every Gaussian below has a
    footprint that reaches the image, so only the mean test decides."""
    cam = synth.camera_from_rows(np.eye(3), (0, 0, -3), 64, 48, 50.0, cx=20.0, cy=30.0)
    pts = [(-1.50, 0.0, True), (-1.62, 0.0, False),   # left:   -25 | -27 vs -26
           (3.30, 0.0, True), (3.60, 0.0, False),     # right:   55 |  60 vs 57.2
           (0.0, -2.20, True), (0.0, -2.50, False),   # top:  -36.7 | -41.7 vs -39
           (0.0, 1.30, True), (0.0, 1.50, False),     # bottom: 21.7 | 25 vs 23.4
           (0.6, 0.6, True)]                          # (10, 10): inside for g >= 1
    sc = _one([(x, y, 0.0) for x, y, _ in pts], (0.0, 0.0, 0.0), (1, 0, 0, 0), 4.0,
              (0.5, 0.5, 0.5))
    want = np.array([k for _, _, k in pts])
    pr = orc.preprocess(sc, cam, ST)  # guard 1.3
    assert_equal = np.testing.assert_array_equal
    assert_equal(pr["valid"] == 1, want)
    assert np.all(pr["n_tiles"][want] > 0)
    off = synth.RenderSettings(fov_guard=0.0)  # the lateral test switched off
    pr0 = orc.preprocess(sc, cam, off)
    assert np.all(pr0["valid"] == 1)  # every footprint reaches the image
    one = synth.RenderSettings(fov_guard=1.0)  # the literal field of view
    pr1 = orc.preprocess(sc, cam, one)
    assert_equal(pr1["valid"] == 1, [False] * 8 + [True])
    # a culled Gaussian contributes nothing: the image equals the render of
    # the kept ones alone
    full = orc.render(sc, cam, ST)
    kept = orc.render(sc.subset(np.nonzero(want)[0]), cam, ST)
    assert np.array_equal(full["C"], kept["C"]) and np.array_equal(full["T"], kept["T"])


def test_geometric_visibility(orc):
    """Redundancy reduction, spatial part: a cell box is visible at the
    pixels whose centre ray meets the part of the box inside the frustum.
    Axis camera at (0,0,-3), f = 61, principal point (32, 32): the box
    [-0.5,0.5] x [-0.25,0.25] x [0,1] spans ray depths 3..4, so a ray
    (u, v, 1) meets it iff |u| <= 0.5/3 and |v| <= 0.25/3, i.e. pixel
    columns 22..41 and rows 27..36.  A box behind the camera or between it
    and the near plane is invisible; a box holding the camera is visible
    everywhere; and the projection of a convex set is convex (each row and
    column of the map is one run)."""
    cam = synth.camera_from_rows(np.eye(3), (0, 0, -3), 64, 64, 61.0, cx=32.0, cy=32.0)
    inf = math.inf
    boxes = [synth.Cell((-0.5, -0.25, 0.0), (0.5, 0.25, 1.0)),   # in front
             synth.Cell((-1.0, -1.0, -9.0), (1.0, 1.0, -4.0)),   # behind
             synth.Cell((-1.0, -1.0, -2.95), (1.0, 1.0, -2.9)),  # before the near plane
             synth.Cell((-1.0, -1.0, -4.0), (1.0, 1.0, -2.0)),   # holds the camera
             synth.Cell((0.2, -inf, -inf), (inf, inf, inf))]     # half-space x >= 0.2
    r = orc.visibility(boxes, cam)
    assert not r["flags"].any()
    want = np.zeros((64, 64), np.uint8)
    want[27:37, 22:42] = 1
    np.testing.assert_array_equal(r["vis"][0], want)
    assert not r["vis"][1].any() and not r["vis"][2].any()
    assert r["vis"][3].all()
    # x >= 0.2: from x = 0 a ray with u > 0 reaches it, u <= 0 never does
    cols = (np.arange(64) + 0.5 - 32.0) > 0
    np.testing.assert_array_equal(r["vis"][4], np.broadcast_to(cols, (64, 64)).astype(np.uint8))
    # convexity on a rotated, off-axis view of a box
    cam2 = synth.look_at_camera((2.5, -1.7, 1.3), (0.1, 0.2, -0.1), 96, 72, hfov_deg=60.0)
    v = orc.visibility([synth.Cell((-0.6, -0.3, -0.4), (0.5, 0.7, 0.2))], cam2)["vis"][0]
    assert 100 < v.sum() < v.size
    for line in list(v) + list(v.T):
        idx = np.nonzero(line)[0]
        if len(idx):
            assert idx[-1] - idx[0] + 1 == len(idx)


def test_kd_partition(orc):
    """Partition strategy: 8 means on the x axis at 0..7 split at the
    median 4 (K = 2), then at 2 and 6 (K = 4), numbered depth first; on a
    ground scene the counts are balanced, every mean lies in its half-open
    box, and the boxes tile space (each probe point is in exactly one)."""
    pts = np.zeros((8, 3), np.float32)
    pts[:, 0] = np.arange(8)
    boxes, cell = orc.kd_partition(pts, 2)
    np.testing.assert_array_equal(cell, [0, 0, 0, 0, 1, 1, 1, 1])
    assert boxes[0][1][0] == 4.0 and boxes[1][0][0] == 4.0 and boxes[0][0][0] == -math.inf
    boxes, cell = orc.kd_partition(pts[::-1], 4)
    np.testing.assert_array_equal(cell, [3, 3, 2, 2, 1, 1, 0, 0])
    assert [b[1][0] for b in boxes[:3]] == [2.0, 4.0, 6.0]
    sc = synth.make_ground_scene(3, 40000)
    for K in (3, 8, 16):
        boxes, cell = orc.kd_partition(sc.means, K)
        cnt = np.bincount(cell, minlength=K)
        assert cnt.max() - cnt.min() <= 2, cnt
        assert orc.imbalance(cell, K) < 1e-3
        lo = np.array([b[0] for b in boxes])
        hi = np.array([b[1] for b in boxes])
        m = sc.means.astype(np.float64)
        assert np.all((lo[cell] <= m) & (m < hi[cell]))
        probe = np.random.default_rng(K).uniform(-600, 600, size=(5000, 3))
        inside = ((lo[None] <= probe[:, None]) & (probe[:, None] < hi[None])).all(-1)
        np.testing.assert_array_equal(inside.sum(1), 1)


def test_rotation_matches_library(orc):
    """Sigma = R S S^T R^T with R from the unit quaternion (w,x,y,z): checked
    against scipy's rotation for a Gaussian on the optical axis, where the
    projected covariance is (f/z)^2 times the upper-left 2x2 block."""
    from scipy.spatial.transform import Rotation
    cam = _axis_cam()
    rng = np.random.default_rng(3)
    for _ in range(5):
        q = rng.normal(size=4).astype(np.float32)
        ls = rng.normal(-2.5, 0.4, size=3).astype(np.float32)
        sc = _one([0, 0, 0], ls, q * np.float32(1.7), 0.0, (0.5, 0.5, 0.5))
        pr = orc.preprocess(sc, cam, ST)
        q64 = sc.quats[0].astype(np.float64)
        Rm = Rotation.from_quat([q64[1], q64[2], q64[3], q64[0]]).as_matrix()
        Sig = Rm @ np.diag(np.exp(2 * ls.astype(np.float64))) @ Rm.T
        k = (50.0 / 3.0) ** 2
        eps = float(np.float32(ST.eps2d))
        np.testing.assert_allclose(
            pr["cov2d"][0], [k * Sig[0, 0] + eps, k * Sig[0, 1], k * Sig[1, 1] + eps],
            rtol=1e-10)


def test_ewa_matches_numerical_jacobian(orc):
    """Off-axis: Sigma2D equals Jn (W Sigma W^T) Jn^T + eps I where Jn is a
    central-difference Jacobian of the pinhole projection (x,y,z) ->
    (fx x/z + cx, fy y/z + cy) at the camera-space mean."""
    cam = synth.g2_camera(320, 180)
    rng = np.random.default_rng(5)
    for _ in range(5):
        mu = np.array([rng.uniform(-30, 30), rng.uniform(120, 200), rng.uniform(0, 20)])
        ls = rng.normal(0.0, 0.5, 3).astype(np.float32)
        q = rng.normal(size=4).astype(np.float32)
        sc = _one(mu, ls, q, 2.0, (0.5, 0.5, 0.5))
        pr = orc.preprocess(sc, cam, ST)
        assert pr["valid"][0]
        R = cam.R.astype(np.float64)
        t = R @ sc.means[0].astype(np.float64) + cam.t.astype(np.float64)

        fx, fy = float(np.float32(cam.fx)), float(np.float32(cam.fy))
        cx, cy = float(np.float32(cam.cx)), float(np.float32(cam.cy))

        def proj(v):
            return np.array([fx * v[0] / v[2] + cx, fy * v[1] / v[2] + cy])
        Jn = np.zeros((2, 3))
        for k in range(3):
            h = 1e-4 * max(1.0, abs(t[k]))
            e = np.zeros(3)
            e[k] = h
            Jn[:, k] = (proj(t + e) - proj(t - e)) / (2 * h)
        qd = q.astype(np.float64) / np.linalg.norm(q.astype(np.float64))
        w, x, y, z = qd
        Rq = np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                       [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                       [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])
        Sig = Rq @ np.diag(np.exp(2 * ls.astype(np.float64))) @ Rq.T
        S2 = Jn @ (R @ Sig @ R.T) @ Jn.T
        eps = float(np.float32(ST.eps2d))
        np.testing.assert_allclose(pr["cov2d"][0],
                                   [S2[0, 0] + eps, S2[0, 1], S2[1, 1] + eps], rtol=2e-6)
        np.testing.assert_allclose(pr["mean2d"][0], proj(t), rtol=1e-13)


def test_two_gaussians_worked_example(orc):
    """Eq. 2 on two coincident on-axis Gaussians: the nearer one is blended
    first whatever its index: C = c1 a1 + c2 a2 (1 - a1), T = (1-a1)(1-a2)."""
    cam = _axis_cam()
    far = ([0, 0, 1.0], -1.0, (0.9, 0.1, 0.2))
    near = ([0, 0, -0.5], 0.4, (0.1, 0.8, 0.3))
    sc = _one([far[0], near[0]], (-3.0, -3.0, -3.0), (1, 0, 0, 0),
              np.array([far[1], near[1]]), np.array([far[2], near[2]]))
    r = orc.render(sc, cam, ST)
    a1 = _sigmoid(float(np.float32(near[1])))
    a2 = _sigmoid(float(np.float32(far[1])))
    c1, c2 = _col(sc, 1), _col(sc, 0)
    np.testing.assert_allclose(r["C"][32, 32], c1 * a1 + c2 * a2 * (1 - a1), atol=1e-15)
    assert abs(r["T"][32, 32] - (1 - a1) * (1 - a2)) < 1e-12
    assert abs(r["D"][32, 32] - (2.5 * a1 + 4.0 * a2 * (1 - a1))) < 1e-12


def test_termination_blend_then_stop(orc):
    """Transmittance stop: the walk ends right after the blend that takes T
    below t_min (1e-4); later Gaussians get no weight."""
    cam = _axis_cam()
    a = 0.95
    logit = math.log(a / (1 - a))
    zs = [[0, 0, -1.0 + 0.3 * k] for k in range(6)]
    cols = np.array([[0.1 * (k + 1)] * 3 for k in range(6)])
    sc = _one(zs, (-3.0, -3.0, -3.0), (1, 0, 0, 0), logit, cols)
    r = orc.render(sc, cam, ST)
    o = _sigmoid(float(np.float32(logit)))
    T, C, n = 1.0, 0.0, 0
    for k in range(6):
        C += _col(sc, k)[0] * o * T
        T *= 1 - o
        n += 1
        if T < float(np.float32(ST.t_min)):
            break
    assert n == 4 and r["nblend"][32, 32] == 4
    assert abs(r["C"][32, 32, 0] - C) < 1e-12 and abs(r["T"][32, 32] - T) < 1e-15


def test_alpha_skip_threshold(orc):
    """A pair with alpha < 1/255 is skipped (no blend, no transmittance)."""
    cam = _axis_cam()
    logit = math.log(0.003 / 0.997)  # o < alpha_min: culled entirely
    sc = _one([0, 0, 0], (-3.0, -3.0, -3.0), (1, 0, 0, 0), logit, (1, 1, 1))
    r = orc.render(sc, cam, ST)
    assert r["nblend"].sum() == 0 and np.all(r["T"] == 1.0)


def test_transmittance_is_product_and_constant_colour(orc):
    """Telescoping of Eq. 2: with every colour equal to c0, C = c0 (1 - T)
    exactly, for every pixel of the tiny workload."""
    sc = synth.tiny_scene()
    c0 = 0.37
    sc.sh[:] = np.float32((c0 - 0.5) * 2.0 * math.sqrt(math.pi))
    r = orc.render(sc, synth.tiny_camera(), ST)
    pr = orc.preprocess(sc, synth.tiny_camera(), ST)
    cval = pr["rgb"][pr["valid"] == 1]
    assert np.ptp(cval) < 1e-15
    np.testing.assert_allclose(r["C"], cval[0][None, None, :] * (1 - r["T"])[..., None], atol=1e-13)


def test_brute_equals_binned(orc):
    """Exact-extent bins drop only pairs with alpha < alpha_min: binned and
    brute-force renders agree bit for bit."""
    sc = synth.tiny_scene()
    cam = synth.tiny_camera()
    a = orc.render(sc, cam, ST, "brute")
    b = orc.render(sc, cam, ST, "binned")
    for k in ("C", "T", "D", "nblend"):
        assert np.array_equal(a[k], b[k]), k


def test_keys_sorted_complete_and_ranges(orc):
    """Sort step: keys are sorted by (tile, float32 depth, index); every pair
    with alpha >= alpha_min (checked by brute force over pixels) appears in
    its tile's list; ranges partition the instance list."""
    sc = synth.make_cube_scene(7, 300, log_scale=(-3.0, 0.5))
    cam = synth.tiny_camera(64, 48)
    keys, vals, ranges = orc.sort_keys(sc, cam, ST)
    pr = orc.preprocess(sc, cam, ST)
    order = np.lexsort((vals, keys))
    assert np.array_equal(order, np.arange(len(keys)))
    tiles = (keys >> np.uint64(32)).astype(np.int64)
    tx = (cam.width + 15) // 16
    assert ranges[0, 0] == 0 and ranges[-1, 1] == len(keys)
    assert np.array_equal(ranges[1:, 0], ranges[:-1, 1])
    for t in range(len(ranges)):
        assert np.all(tiles[ranges[t, 0]:ranges[t, 1]] == t)
    zbits = (keys & np.uint64(0xFFFFFFFF)).astype(np.uint32)
    assert np.array_equal(zbits, pr["depth"][vals].astype(np.float32).view(np.uint32))
    members = {(int(t), int(v)) for t, v in zip(tiles, vals)}
    ys, xs = np.mgrid[0:cam.height, 0:cam.width]
    for g in np.nonzero(pr["valid"])[0]:
        dx = xs + 0.5 - pr["mean2d"][g, 0]
        dy = ys + 0.5 - pr["mean2d"][g, 1]
        a, b, c = pr["conic"][g]
        alpha = pr["opacity"][g] * np.exp(-0.5 * (a * dx * dx + 2 * b * dx * dy + c * dy * dy))
        hit = np.nonzero(alpha >= ST.alpha_min * (1 + 1e-9))
        for y, x in zip(*hit):
            assert ((y // 16) * tx + x // 16, g) in members


# ------------------------------------------------------------------ SH ----
def _unit_dirs(n, seed=0):
    d = np.random.default_rng(seed).normal(size=(n, 3))
    return d / np.linalg.norm(d, axis=1, keepdims=True)


def test_sh_y00_and_addition_theorem(orc):
    d = _unit_dirs(200)
    Y, _ = orc.sh_eval(3, d)
    assert np.allclose(Y[:, 0], 1 / (2 * math.sqrt(math.pi)), atol=1e-15)
    for l in range(4):
        s = (Y[:, l * l:(l + 1) * (l + 1)] ** 2).sum(1)
        np.testing.assert_allclose(s, (2 * l + 1) / (4 * math.pi), rtol=1e-12)


def test_sh_orthonormal_by_quadrature(orc):
    """Gauss-Legendre in cos(theta) times the trapezoid rule in phi integrates
    products of degree <= 6 exactly."""
    xg, wg = np.polynomial.legendre.leggauss(8)
    nphi = 16
    phi = 2 * math.pi * np.arange(nphi) / nphi
    ct, ph = np.meshgrid(xg, phi, indexing="ij")
    st = np.sqrt(1 - ct ** 2)
    d = np.stack([st * np.cos(ph), st * np.sin(ph), ct], -1).reshape(-1, 3)
    w = (wg[:, None] * np.full(nphi, 2 * math.pi / nphi)[None, :]).reshape(-1)
    Y, _ = orc.sh_eval(3, d)
    G = (Y * w[:, None]).T @ Y
    np.testing.assert_allclose(G, np.eye(16), atol=1e-12)


def test_sh_matches_scipy_convention(orc):
    """Real basis from scipy's complex harmonics (Condon-Shortley phase):
    Y_l0 = Re Y_l^0, Y_lm = sqrt2 Re Y_l^m, Y_l,-m = sqrt2 Im Y_l^m."""
    import scipy.special as sp
    d = _unit_dirs(50, 1)
    theta = np.arccos(np.clip(d[:, 2], -1, 1))
    phi = np.arctan2(d[:, 1], d[:, 0])
    Y, _ = orc.sh_eval(3, d)
    for l in range(4):
        for m in range(0, l + 1):
            if hasattr(sp, "sph_harm_y"):
                c = sp.sph_harm_y(l, m, theta, phi)
            else:
                c = sp.sph_harm(m, l, phi, theta)
            if m == 0:
                np.testing.assert_allclose(Y[:, l * l + l], c.real, atol=1e-12)
            else:
                np.testing.assert_allclose(Y[:, l * l + l + m], math.sqrt(2) * c.real, atol=1e-12)
                np.testing.assert_allclose(Y[:, l * l + l - m], math.sqrt(2) * c.imag, atol=1e-12)


def test_sh_gradient_tangential_part(orc):
    """The tangential gradient of each basis function matches a central
    difference along the sphere (the radial part is irrelevant because the
    direction is normalised)."""
    d = _unit_dirs(20, 2)
    _, G = orc.sh_eval(3, d)
    h = 1e-6
    for k in range(3):
        e = np.zeros(3)
        e[k] = h
        dp = d + e
        dm = d - e
        dp /= np.linalg.norm(dp, axis=1, keepdims=True)
        dm /= np.linalg.norm(dm, axis=1, keepdims=True)
        Yp, _ = orc.sh_eval(3, dp)
        Ym, _ = orc.sh_eval(3, dm)
        fd = (Yp - Ym) / (2 * h)
        proj = G - (G * d[:, None, :]).sum(-1, keepdims=True) * d[:, None, :]
        np.testing.assert_allclose(proj[:, :, k], fd, atol=1e-7)


# ---------------------------------------------------------- composition ---
def _zslab_cells(edges):
    return [synth.Cell((-math.inf, -math.inf, float(edges[i])),
                       (math.inf, math.inf, float(edges[i + 1])))
            for i in range(len(edges) - 1)]


def test_composite_associative_identity_k1(orc):
    """over((C1,T1),(C2,T2)) = (C1 + T1 C2, T1 T2) is associative, (0,1) is
    its identity, and a single cell composes to C + T bg (Eq. 5)."""
    cam = synth.tiny_camera(16, 16)
    rng = np.random.default_rng(9)
    K = 3
    Tp = rng.uniform(0.0, 1.0, size=(K, 16, 16))
    Cp = rng.uniform(0, 1, size=(K, 16, 16, 3)) * (1 - Tp[..., None])
    cells = _zslab_cells([-2.0, -1.0, 0.0, 1.0])
    st0 = synth.RenderSettings(t_min=0.0)
    full = orc.composite(Cp, Tp, cells, cam, st0)
    ab = orc.composite(Cp[:2], Tp[:2], cells[:2], cam, st0)
    left = orc.composite(np.stack([ab["rgb"], Cp[2]]), np.stack([ab["T"], Tp[2]]),
                         [cells[0], cells[2]], cam, st0)
    bc = orc.composite(Cp[1:], Tp[1:], cells[1:], cam, st0)
    right = orc.composite(np.stack([Cp[0], bc["rgb"]]), np.stack([Tp[0], bc["T"]]),
                          [cells[0], cells[1]], cam, st0)
    for o in (left, right):
        np.testing.assert_allclose(o["rgb"], full["rgb"], atol=1e-14)
        np.testing.assert_allclose(o["T"], full["T"], atol=1e-15)
    Cid = Cp.copy()
    Tid = Tp.copy()
    Cid[1] = 0.0
    Tid[1] = 1.0
    ident = orc.composite(Cid, Tid, cells, cam, st0)
    two = orc.composite(Cp[[0, 2]], Tp[[0, 2]], [cells[0], cells[2]], cam, st0)
    np.testing.assert_allclose(ident["rgb"], two["rgb"], atol=1e-15)
    bg = synth.RenderSettings(t_min=0.0, bg=(0.2, 0.4, 0.6))
    one = orc.composite(Cp[:1], Tp[:1], cells[:1], cam, bg)
    np.testing.assert_allclose(one["rgb"], Cp[0] + Tp[0][..., None] * np.array(bg.bg, np.float32),
                               atol=1e-15)
    assert np.all(full["order"] == np.arange(K))


def test_eq5_equals_eq2_on_depth_separated_slabs(orc):
    """The paper's claim that Eq. 5 equals Eq. 2: with no early stop, the
    composite of depth-separated slab partials equals the single-pass render
    (to rounding)."""
    sc = synth.tiny_scene()
    cam = synth.tiny_camera()
    st0 = synth.RenderSettings(t_min=0.0)
    edges = synth.quantile_edges(sc.means[:, 2], 4)
    part = synth.axis_slab_partition(sc, 2, edges)
    cells = part.cells
    fr = orc.forward(part.cell_scenes(sc), cells, cam, st0)
    single = orc.render(sc, cam, st0)
    np.testing.assert_allclose(fr.comp["rgb"], single["C"], atol=1e-12)
    np.testing.assert_allclose(fr.comp["T"], single["T"], atol=1e-12)
    assert np.all(fr.comp["order"] == np.arange(4))


def test_saturation_culling_bound(orc):
    """Saturation redundancy: a cell behind prod T < eps is marked inactive;
    skipping it changes a pixel by at most eps * max colour."""
    sc = synth.make_cube_scene(11, 6000, log_scale=(-3.2, 0.4), logit_sigma=2.0)
    cam = synth.tiny_camera(64, 64)
    edges = synth.quantile_edges(sc.means[:, 2], 4)
    part = synth.axis_slab_partition(sc, 2, edges)
    scenes = part.cell_scenes(sc)
    full = orc.forward(scenes, part.cells, cam, ST)
    culled = orc.forward(scenes, part.cells, cam, ST, same_frame_cull=True)
    inactive = full.comp["mask"] == 0
    assert inactive.sum() > 0
    cmax = max(orc.preprocess(s, cam, ST)["rgb"].max() for s in scenes)
    assert np.abs(culled.comp["rgb"] - full.comp["rgb"]).max() <= ST.t_min * cmax + 1e-15
    # the next render of the view with the masks: inactive pairs produce the
    # identity partial, and composing gives the same-frame-culled image
    nxt = orc.forward(scenes, part.cells, cam, ST, masks=full.comp["mask"])
    np.testing.assert_allclose(nxt.comp["rgb"], culled.comp["rgb"], atol=1e-15)
    assert np.all(nxt.Tparts[inactive] == 1.0)


def test_reeval_hand_cases(orc):
    """Speculative re-evaluation of pruned pairs (appendix, saturation
    stability): three cells in entry order on every ray, the first rendered,
    the other two pruned with stale budgets; each case's outcome worked out
    by hand from the rule (residual R = P - S must reach t_min and cover the
    budget; the first failure ends the scan)."""
    cam = synth.tiny_camera(1, 1)
    cells = _zslab_cells([-2.0, -1.0, 0.0, 1.0])
    t = 1e-4
    st = synth.RenderSettings(t_min=np.float32(t))
    t = float(np.float32(t))  # the oracle compares against t_min as float32
    # (T of cell 0, budgets of cells 1 and 2) -> expected masks, flips
    cases = [
        (0.5, 3e-5, 5e-5, (1, 1, 1), 2),      # R = 0.5 covers both
        (1.5e-4, 3e-5, 5e-5, (1, 1, 1), 2),   # 1.5e-4 -> 1.2e-4 >= t_min
        (1.2e-4, 3e-5, 5e-5, (1, 1, 0), 1),   # 1.2e-4 -> 0.9e-4 < t_min: stop
        (1.5e-4, 2e-4, 1e-5, (1, 0, 0), 0),   # budget 2e-4 not covered: stop
        (0.9e-4, 1e-5, 1e-5, (1, 0, 0), 0),   # residual below t_min already
    ]
    for T0, b1, b2, want, nf in cases:
        Cp = np.zeros((3, 1, 1, 3))
        Cp[0] = 0.25
        Tp = np.ones((3, 1, 1))
        Tp[0] = T0
        mask_in = np.array([1, 0, 0], np.uint8).reshape(3, 1, 1)
        budget = np.array([0.0, b1, b2]).reshape(3, 1, 1)
        out = orc.composite_reeval(Cp, Tp, cells, cam, st, mask_in, budget)
        assert tuple(out["mask"].reshape(-1)) == want, (T0, b1, b2)
        assert out["flips"][0, 0] == nf
        assert out["rgb"][0, 0, 0] == 0.25 and out["T"][0, 0] == T0
        np.testing.assert_array_equal(budget.reshape(-1), [0.0, b1, b2])  # nothing pruned now
    # pruning now: cell 0 leaves 5e-5, so cell 1 (rendered, T = 0.3) is
    # pruned with budget 5e-5 * (1 - 0.3); cell 2 (pruned, budget 1e-6) is
    # tested with R = 5e-5 * 0.3 and stays pruned; cell 0 stays active
    Tp = np.array([5e-5, 0.3, 1.0]).reshape(3, 1, 1)
    Cp = np.zeros((3, 1, 1, 3))
    budget = np.array([0.0, 0.0, 1e-6]).reshape(3, 1, 1)
    out = orc.composite_reeval(Cp, Tp, cells, cam, st,
                               np.array([1, 1, 0], np.uint8).reshape(3, 1, 1), budget)
    assert tuple(out["mask"].reshape(-1)) == (1, 0, 0)
    assert budget[1, 0, 0] == 5e-5 * (1 - 0.3) and budget[2, 0, 0] == 1e-6
    assert out["T"][0, 0] == 5e-5 * 0.3
    # a box the ray misses (omega 0) is never re-activated
    out = orc.composite_reeval(np.zeros((3, 1, 1, 3)), np.ones((3, 1, 1)), cells, cam, st,
                               np.array([1, 0, 0], np.uint8).reshape(3, 1, 1),
                               np.zeros((3, 1, 1)),
                               omega=np.array([1, 0, 1], np.uint8).reshape(3, 1, 1))
    assert tuple(out["mask"].reshape(-1)) == (1, 0, 1)


def test_reeval_reduces_to_composite_and_is_stable(orc):
    """With every pair rendered the re-evaluating composition is Eq. 5 with
    the saturation test (the same image and masks); rendering the view again
    from its own masks and budgets, with the scene unchanged, re-activates
    nothing (the residual is the transmittance that pruned the pairs) and
    gives the same image.  Lowering the opacity of the front cell's
    Gaussians then re-activates pairs behind it, and only where the fresh
    residual reaches t_min."""
    sc = synth.make_cube_scene(11, 6000, log_scale=(-3.2, 0.4), logit_sigma=2.0)
    cam = synth.tiny_camera(64, 64)
    edges = synth.quantile_edges(sc.means[:, 2], 4)
    part = synth.axis_slab_partition(sc, 2, edges)
    scenes = part.cell_scenes(sc)
    K = len(scenes)
    fr = orc.forward(scenes, part.cells, cam, ST)
    ones = np.ones((K, cam.height, cam.width), np.uint8)
    budget = np.zeros((K, cam.height, cam.width))
    r1 = orc.composite_reeval(fr.Cparts, fr.Tparts, part.cells, cam, ST, ones, budget)
    np.testing.assert_array_equal(r1["rgb"], fr.comp["rgb"])
    np.testing.assert_array_equal(r1["T"], fr.comp["T"])
    np.testing.assert_array_equal(r1["mask"], fr.comp["mask"])
    pruned = r1["mask"] == 0
    assert pruned.sum() > 100 and np.all(r1["flips"] == 0)
    # a budget is P_j (1 - T_j) with P_j < t_min (zero where the cell is
    # transparent on the ray)
    assert np.all(budget[pruned] >= 0) and np.all(budget[pruned] < ST.t_min)
    assert (budget[pruned] > 0).mean() > 0.5
    assert np.all(budget[~pruned] == 0)
    # the same view again, from its own state
    f2 = orc.forward(scenes, part.cells, cam, ST, masks=r1["mask"])
    b2 = budget.copy()
    r2 = orc.composite_reeval(f2.Cparts, f2.Tparts, part.cells, cam, ST, r1["mask"], b2)
    assert np.all(r2["flips"] == 0)
    np.testing.assert_array_equal(r2["mask"], r1["mask"])
    np.testing.assert_array_equal(b2, budget)
    assert np.abs(r2["rgb"] - r1["rgb"]).max() <= ST.t_min
    # fade the front cell (order 0 on every ray of this camera)
    assert np.all(fr.comp["order"][..., 0] == 0)
    faded = [s for s in scenes]
    faded[0] = scenes[0].subset(np.arange(scenes[0].n))
    faded[0].opacity_logits = faded[0].opacity_logits - 6.0
    f3 = orc.forward(faded, part.cells, cam, ST, masks=r1["mask"])
    b3 = budget.copy()
    r3 = orc.composite_reeval(f3.Cparts, f3.Tparts, part.cells, cam, ST, r1["mask"], b3)
    flipped = (r3["mask"] == 1) & pruned
    assert flipped.sum() > 0 and flipped.sum() == r3["flips"].sum()
    # a pixel re-activates its first pruned cell iff the fresh residual
    # after its rendered cells reaches t_min (budgets are below t_min)
    for py, px in zip(*np.nonzero(pruned.any(0))):
        first = next(int(m) for m in fr.comp["order"][py, px] if pruned[m, py, px])
        R = r3["T"][py, px]
        if abs(R - ST.t_min) > 1e-3 * ST.t_min:
            assert bool(r3["mask"][first, py, px]) == (R >= np.float32(ST.t_min))


def _scene_of(means, scales, opac=0.8):
    n = len(means)
    sh = np.zeros((n, 1, 3), np.float32)
    sh[:, 0, :] = 1.0
    return synth.Scene(np.asarray(means, np.float32),
                       np.log(np.asarray(scales, np.float32))[:, None].repeat(3, 1),
                       np.tile(np.array([1, 0, 0, 0], np.float32), (n, 1)),
                       np.full(n, math.log(opac / (1 - opac)), np.float32), sh)


def test_cross_filter_hand_cases(orc):
    """Cross-boundary filter bits (appendix, cross-boundary Gaussians) worked
    out by hand: two cells split at x = 0, camera looking +z from z = -3
    (camera depth = world z + 3).  An isotropic Gaussian spans the other
    cell when its mean lies within 3 sigma of the plane; with boxes
    unbounded in z every depth is in the overlapped interval, with boxes
    z in [-1, 1] and [0.5, 3] (depths [2, 4] and [3.5, 6]) only depths in
    [3.5, 4] are."""
    cam = synth.camera_from_rows(np.eye(3), (-0.5, 0.0, -3.0), 48, 32, 40.0)
    inf = math.inf
    open_cells = [synth.Cell((-inf, -inf, -inf), (0.0, inf, inf)),
                  synth.Cell((0.0, -inf, -inf), (inf, inf, inf))]
    # cell 0: A spans (0.3 > 0.1), B does not (0.15 < 0.6); cell 1: C spans
    sc0 = _scene_of([(-0.1, 0.0, 0.0), (-0.6, 0.2, 0.0)], [0.1, 0.05])
    sc1 = _scene_of([(0.05, -0.2, 0.5)], [0.05])
    st = synth.RenderSettings(fov_guard=0.0)
    f0 = orc.cross_filter(sc0, cam, st, open_cells, 0)
    f1 = orc.cross_filter(sc1, cam, st, open_cells, 1)
    assert list(f0["xf"]) == [0b10, 0] and list(f1["xf"]) == [0b01]
    assert not f0["amb"].any() and not f1["amb"].any()
    boxed = [synth.Cell((-inf, -inf, -1.0), (0.0, inf, 1.0)),
             synth.Cell((0.0, -inf, 0.5), (inf, inf, 3.0))]
    # depths 3 (out), 3.8 (in), 4.5 (out: beyond cell 0's range)
    sc = _scene_of([(-0.1, 0.0, 0.0), (-0.1, 0.0, 0.8), (-0.1, 0.0, 1.5)], [0.1, 0.1, 0.1])
    f = orc.cross_filter(sc, cam, st, boxed, 0)
    assert list(f["xf"]) == [0, 0b10, 0]
    # a culled Gaussian (behind the camera) carries no bits
    f = orc.cross_filter(_scene_of([(-0.1, 0.0, -5.0)], [0.1]), cam, st, open_cells, 0)
    assert list(f["xf"]) == [0]
    # anisotropic support: scales (0.3, 0.01, 0.01) reach 0.9 along the long
    # axis and 0.03 across it; along x the Gaussian at x = -0.1 spans the
    # plane, turned 90 degrees about z (long axis along y) it does not, and
    # turned 45 degrees its x half-extent is 3 sqrt((0.09 + 1e-4) / 2) = 0.637
    sc = _scene_of([(-0.1, 0.0, 0.0)] * 3, [1.0] * 3)
    sc.log_scales = np.log(np.array([[0.3, 0.01, 0.01]] * 3, np.float32))
    c45, s45 = math.cos(math.pi / 8), math.sin(math.pi / 8)
    sc.quats = np.array([[1, 0, 0, 0], [math.sqrt(0.5), 0, 0, math.sqrt(0.5)],
                         [c45, 0, 0, s45]], np.float32)
    f = orc.cross_filter(sc, cam, st, open_cells, 0)
    assert list(f["xf"]) == [0b10, 0, 0b10]
    sc.means = np.array([[-0.62, 0.0, 0.0], [-0.62, 0.0, 0.0], [-0.65, 0.0, 0.0]], np.float32)
    sc.quats = np.array([[c45, 0, 0, s45]] * 3, np.float32)
    f = orc.cross_filter(sc, cam, st, open_cells, 0)
    assert list(f["xf"]) == [0b10, 0b10, 0]  # 0.637 > 0.62 and < 0.65


def test_cross_filter_render_drops_exactly_the_pair(orc):
    """The pixel region of the filter is where both cells' visibility maps
    cover the pixel: from a camera at x = -0.5, the rays that reach x >= 0
    are those heading to +x (pixel centre right of cx).  There the filtered
    render of cell 0 equals the render without the spanning Gaussian; on
    the other pixels it equals the unfiltered render (bit for bit)."""
    cam = synth.camera_from_rows(np.eye(3), (-0.5, 0.0, -3.0), 48, 32, 40.0)
    inf = math.inf
    cells = [synth.Cell((-inf, -inf, -inf), (0.0, inf, inf)),
             synth.Cell((0.0, -inf, -inf), (inf, inf, inf))]
    sc0 = _scene_of([(-0.1, 0.0, 0.0), (-0.6, 0.2, 0.0), (-0.4, -0.1, 0.3)],
                    [0.1, 0.05, 0.08])
    st = synth.RenderSettings(fov_guard=0.0)
    vis = orc.visibility(cells, cam)
    assert not vis["flags"].any()
    pb = orc.pixel_bits(vis["vis"], 0)
    px = np.arange(cam.width) + 0.5
    right = np.broadcast_to(px > cam.cx, (cam.height, cam.width))
    assert np.array_equal(pb, np.where(right, 3, 1).astype(np.uint32))
    f = orc.cross_filter(sc0, cam, st, cells, 0)
    assert list(f["xf"]) == [0b10, 0, 0]
    f["pixbits"] = pb
    filt = orc.render(sc0, cam, st, xfilter=f)
    plain = orc.render(sc0, cam, st)
    without = orc.render(sc0.subset(np.array([1, 2])), cam, st)
    assert not filt["flags"].any()
    for key in ("C", "T", "D"):
        np.testing.assert_array_equal(filt[key][right], without[key][right])
        np.testing.assert_array_equal(filt[key][~right], plain[key][~right])
    assert (plain["nblend"] - filt["nblend"])[right].sum() > 20


def test_backward_with_cross_filter_matches_finite_differences(orc):
    """Eq. 6-7 through two cells split at x = 0 with the cross-boundary
    filter on (held fixed, as the gradient treats it): Gaussians near the
    plane are removed from the rays where both cells are visible, and the
    gradients of the remaining pairs match central differences."""
    cam = synth.camera_from_rows(np.eye(3), (-0.3, 0.0, -3.0), 64, 64,
                                 32.0 / math.tan(math.radians(30.0)))
    inf = math.inf
    cells = [synth.Cell((-inf, -inf, -inf), (0.0, inf, inf)),
             synth.Cell((0.0, -inf, -inf), (inf, inf, inf))]
    for seed in range(300, 340):
        sc = synth.fd_scene(seed).astype(np.float64)
        left = np.nonzero(sc.means[:, 0] < 0)[0]
        right = np.nonzero(sc.means[:, 0] >= 0)[0]
        scenes = [sc.subset(left), sc.subset(right)]
        xfs = orc.cross_filters(scenes, cells, cam, ST)
        fr = orc.forward(scenes, cells, cam, ST, delta_q=1e-3, xfilters=xfs)
        fl = np.bitwise_or.reduce([p["flags"] for p in fr.parts]) | fr.comp["flags"]
        if not fl.any() and sum(int((x["xf"] != 0).sum()) for x in xfs) >= 4:
            break
    else:
        raise AssertionError("no flag-free scene with cross-boundary Gaussians")
    rng = np.random.default_rng(5)
    wr = rng.normal(size=(cam.height, cam.width, 3))
    wt = rng.normal(size=(cam.height, cam.width))
    fr = orc.forward(scenes, cells, cam, ST, xfilters=xfs)
    grads = orc.backward(scenes, cells, cam, ST, fr, wr, wt, xfilters=xfs)
    unf = orc.forward(scenes, cells, cam, ST)
    assert np.abs(unf.comp["rgb"] - fr.comp["rgb"]).max() > 1e-3  # the filter acts

    def loss():
        f = orc.forward(scenes, cells, cam, ST, xfilters=xfs)
        return float((f.comp["rgb"] * wr).sum() + (f.comp["T"] * wt).sum())

    for k, cs in enumerate(scenes):
        for name in ("means", "opacity_logits", "sh"):
            flat = getattr(cs, name).reshape(-1)
            g = grads[k][name].reshape(-1)
            idx = np.sort(rng.choice(flat.size, min(flat.size, 40), replace=False))
            fd = np.zeros(len(idx))
            for j, i in enumerate(idx):
                h = 1e-6 * max(1.0, abs(flat[i]))
                old = flat[i]
                flat[i] = old + h
                lp = loss()
                flat[i] = old - h
                lm = loss()
                flat[i] = old
                fd[j] = (lp - lm) / (2 * h)
            scale = max(np.abs(fd).max(), 1e-12)
            err = np.abs(g[idx] - fd) / np.maximum(np.abs(fd), 1e-3 * scale)
            assert err.max() <= 1e-3, (k, name, err.max())


# ------------------------------------------------------------ Eq. 6-7 -----
def _flag_free_fd_scene(orc, seed0, cam, cells_fn):
    for seed in range(seed0, seed0 + 40):
        sc = synth.fd_scene(seed).astype(np.float64)
        part = cells_fn(sc)
        fr = orc.forward(part.cell_scenes(sc), part.cells, cam, ST, delta_q=1e-3)
        fl = np.bitwise_or.reduce([p["flags"] for p in fr.parts])
        if not np.any(fl) and not np.any(fr.comp["flags"]):
            return sc, part
    raise AssertionError("no flag-free FD scene")


def _fd_check(orc, sc, part, cam, seed):
    rng = np.random.default_rng(seed)
    H, W = cam.height, cam.width
    wr = rng.normal(size=(H, W, 3))
    wt = rng.normal(size=(H, W))
    scenes = part.cell_scenes(sc)
    fr = orc.forward(scenes, part.cells, cam, ST)
    grads = orc.backward(scenes, part.cells, cam, ST, fr, wr, wt)

    def loss(scs):
        f = orc.forward(scs, part.cells, cam, ST)
        return float((f.comp["rgb"] * wr).sum() + (f.comp["T"] * wt).sum())

    names = ("means", "log_scales", "quats", "opacity_logits", "sh")
    for k, cs in enumerate(scenes):
        for name in names:
            arr = getattr(cs, name)
            g = grads[k][name]
            flat = arr.reshape(-1)
            gflat = g.reshape(-1)
            idx = np.arange(flat.size)
            if flat.size > 120:
                idx = np.sort(rng.choice(flat.size, 120, replace=False))
            fd = np.zeros(len(idx))
            for j, i in enumerate(idx):
                h = 1e-6 * max(1.0, abs(flat[i]))
                old = flat[i]
                flat[i] = old + h
                lp = loss(scenes)
                flat[i] = old - h
                lm = loss(scenes)
                flat[i] = old
                fd[j] = (lp - lm) / (2 * h)
            ga = gflat[idx]
            scale = max(np.abs(fd).max(), 1e-12)
            err = np.abs(ga - fd) / np.maximum(np.abs(fd), 1e-3 * scale)
            assert err.max() <= 1e-3, (k, name, err.max())


def test_backward_matches_finite_differences_k1(orc):
    """Eq. 6-7 with one cell, every parameter family, FP64 central
    differences on a 64-Gaussian scene (seed re-drawn if any pair sits within
    reach of a discrete threshold)."""
    cam = synth.fd_camera()

    def one_cell(s):
        return synth.axis_slab_partition(s, 2, [-10.0, 10.0])
    sc, part = _flag_free_fd_scene(orc, 100, cam, one_cell)
    _fd_check(orc, sc, part, cam, 1)


def test_backward_matches_finite_differences_k2(orc):
    """Eq. 6-7 through a two-cell composition (depth-separated slabs): the
    transmittance gradient term of Eq. 6 reaches the front cell."""
    cam = synth.fd_camera()

    def two_cells(s):
        return synth.axis_slab_partition(s, 2, [-10.0, 0.0, 10.0])
    sc, part = _flag_free_fd_scene(orc, 200, cam, two_cells)
    _fd_check(orc, sc, part, cam, 2)


def _fd_grads(loss, scenes, grads, rng, names=("means", "log_scales", "quats",
                                                 "opacity_logits", "sh"),
              per_array=120, only=None):
    """Central differences of loss() at sampled entries of each cell's
    parameter arrays, compared with the analytic gradients per element
    (relative, floored at 1e-3 of the largest difference quotient).
    `only` maps a cell to the Gaussian indices whose entries are sampled."""
    for k, cs in enumerate(scenes):
        for name in names:
            arr = getattr(cs, name)
            flat = arr.reshape(-1)
            gflat = grads[k][name].reshape(-1)
            per = flat.size // max(cs.n, 1)
            pool = np.arange(flat.size)
            if only is not None and k in only:
                pool = (np.asarray(only[k])[:, None] * per + np.arange(per)).reshape(-1)
            idx = pool if pool.size <= per_array else np.sort(rng.choice(pool, per_array,
                                                                          replace=False))
            fd = np.zeros(len(idx))
            for j, i in enumerate(idx):
                h = 1e-6 * max(1.0, abs(flat[i]))
                old = flat[i]
                flat[i] = old + h
                lp = loss()
                flat[i] = old - h
                lm = loss()
                flat[i] = old
                fd[j] = (lp - lm) / (2 * h)
            scale = max(np.abs(fd).max(), 1e-12)
            err = np.abs(gflat[idx] - fd) / np.maximum(np.abs(fd), 1e-3 * scale)
            assert err.max() <= 1e-3, (k, name, err.max())


def _flag_free(orc, scenes_fn, cells, cam, st, seeds, accept=lambda fr: True, **kw):
    """The first seed whose scenes render with no flagged pixel (no pair
    within rounding or difference-step reach of a discrete threshold) and
    that `accept` takes."""
    for seed in seeds:
        scenes = scenes_fn(seed)
        fr = orc.forward(scenes, cells, cam, st, delta_q=1e-3, **kw)
        fl = np.bitwise_or.reduce([p["flags"] for p in fr.parts]) | fr.comp["flags"]
        if not fl.any() and accept(fr):
            return scenes, fr
    raise AssertionError("no flag-free scene")


def test_depth_gradient_matches_finite_differences(orc):
    """Eq. 6-7 with the partial depth D = sum z_i alpha_i T_i in the loss
    (reading 1 of the garbled D^m): the depth terms of the reverse walk
    (dalpha gets g_D (z_i - RD), the depth itself gets alpha_i T_i g_D,
    which reaches the means through the camera z) against central
    differences of L = sum wC.C + wT.T + wD.D on one cell."""
    cam = synth.fd_camera()
    cell = [synth.Cell((-math.inf,) * 3, (math.inf,) * 3)]
    scenes, _ = _flag_free(orc, lambda s: [synth.fd_scene(s).astype(np.float64)], cell, cam,
                           ST, range(400, 440))
    sc = scenes[0]
    rng = np.random.default_rng(11)
    wc = rng.normal(size=(cam.height, cam.width, 3))
    wt = rng.normal(size=(cam.height, cam.width))
    wd = rng.normal(size=(cam.height, cam.width))
    g = orc.render_backward(sc, cam, ST, wc, wt, wd)
    g0 = orc.render_backward(sc, cam, ST, wc, wt, None)
    # the depth term changes the mean and opacity gradients substantially
    for name in ("means", "opacity_logits"):
        assert np.abs(g[name] - g0[name]).max() > 0.05 * np.abs(g[name]).max(), name
    assert np.abs(g["g2d"][:, 9]).max() > 0 and not g0["g2d"][:, 9].any()

    def loss():
        r = orc.render(sc, cam, ST)
        return float((r["C"] * wc).sum() + (r["T"] * wt).sum() + (r["D"] * wd).sum())
    _fd_grads(loss, [sc], [g], rng)


def test_background_term_matches_finite_differences(orc):
    """Eq. 6-7 with a background behind the last cell (B_{K+1} = bg): the
    transmittance gradient of every cell gets P_j G.B_{j+1} with the
    background in B, through two depth-separated cells."""
    import dataclasses
    st = dataclasses.replace(ST, bg=(0.3, 0.6, 0.9))
    cam = synth.fd_camera()
    part_of = lambda s: synth.axis_slab_partition(s, 2, [-10.0, 0.0, 10.0])
    cells = part_of(synth.fd_scene(0)).cells

    def scenes_of(seed):
        s = synth.fd_scene(seed).astype(np.float64)
        return part_of(s).cell_scenes(s)
    scenes, _ = _flag_free(orc, scenes_of, cells, cam, st, range(500, 540))
    rng = np.random.default_rng(12)
    wr = rng.normal(size=(cam.height, cam.width, 3))
    wt = rng.normal(size=(cam.height, cam.width))
    fr = orc.forward(scenes, cells, cam, st)
    grads = orc.backward(scenes, cells, cam, st, fr, wr, wt)
    # against bg = 0 the gradients differ (the background term is exercised)
    fr0 = orc.forward(scenes, cells, cam, ST)
    g0 = orc.backward(scenes, cells, cam, ST, fr0, wr, wt)
    assert np.abs(grads[0]["opacity_logits"] - g0[0]["opacity_logits"]).max() > \
        0.05 * np.abs(grads[0]["opacity_logits"]).max()

    def loss():
        f = orc.forward(scenes, cells, cam, st)
        return float((f.comp["rgb"] * wr).sum() + (f.comp["T"] * wt).sum())
    _fd_grads(loss, scenes, grads, rng, per_array=60)


def test_clamped_alpha_matches_finite_differences(orc):
    """Eq. 1 with the clamp alpha = min(alpha_max, o G): where it is clamped
    alpha does not depend on the opacity or the conic, so those pairs pass
    no gradient to them (only colour and the transmittance chain see them).
    Central differences of every parameter of the clamped Gaussian and a
    sample of the others."""
    cam = synth.fd_camera()
    cell = [synth.Cell((-math.inf,) * 3, (math.inf,) * 3)]
    scenes, _ = _flag_free(orc, lambda s: [synth.clamp_fd_scene(s)], cell, cam, ST, range(600, 640))
    sc = scenes[0]
    pr = orc.preprocess(sc, cam, ST)
    # pixel centres where Gaussian 0 is clamped (it is first on every ray)
    ys, xs = np.mgrid[0:cam.height, 0:cam.width] + 0.5
    dx, dy = xs - pr["mean2d"][0, 0], ys - pr["mean2d"][0, 1]
    a, b, c = pr["conic"][0]
    G = np.exp(-0.5 * (a * dx * dx + 2 * b * dx * dy + c * dy * dy))
    n_clamped = int((pr["opacity"][0] * G > ST.alpha_max).sum())
    assert n_clamped >= 3, n_clamped
    rng = np.random.default_rng(13)
    wc = rng.normal(size=(cam.height, cam.width, 3))
    wt = rng.normal(size=(cam.height, cam.width))
    g = orc.render_backward(sc, cam, ST, wc, wt, None)

    def loss():
        r = orc.render(sc, cam, ST)
        return float((r["C"] * wc).sum() + (r["T"] * wt).sum())
    _fd_grads(loss, [sc], [g], rng, only={0: [0]})
    _fd_grads(loss, [sc], [g], rng, names=("means", "opacity_logits"), per_array=40)


def test_same_frame_cull_matches_finite_differences(orc):
    """The saturation rule applied in the same frame: a cell behind a prefix
    with P_j < t_min is treated as the identity in Eq. 5 and gets no
    gradient (its dC, dT are zero and the cells in front of it see B and U
    without it).  t_min = 0.05 here so that two opaque slabs saturate;
    central differences through two cells with the culling on."""
    import dataclasses
    st = dataclasses.replace(ST, t_min=0.05)
    cam = synth.fd_camera()
    cells = synth.same_frame_fd_scenes(0)[1]

    def culls(fr):
        return int((fr.comp["mask"][1] == 0).sum()) >= 20
    scenes, fr = _flag_free(orc, lambda s: synth.same_frame_fd_scenes(s)[0], cells, cam, st,
                            range(700, 760), accept=culls, same_frame_cull=True)
    rng = np.random.default_rng(14)
    wr = rng.normal(size=(cam.height, cam.width, 3))
    wt = rng.normal(size=(cam.height, cam.width))
    fr = orc.forward(scenes, cells, cam, st, same_frame_cull=True)
    grads = orc.backward(scenes, cells, cam, st, fr, wr, wt, same_frame_cull=True)
    # culling changes the image and the back cell's gradients
    fr0 = orc.forward(scenes, cells, cam, st)
    assert np.abs(fr0.comp["rgb"] - fr.comp["rgb"]).max() > 1e-4
    g0 = orc.backward(scenes, cells, cam, st, fr0, wr, wt)
    assert np.abs(g0[1]["means"] - grads[1]["means"]).max() > 0

    def loss():
        f = orc.forward(scenes, cells, cam, st, same_frame_cull=True)
        return float((f.comp["rgb"] * wr).sum() + (f.comp["T"] * wt).sum())
    _fd_grads(loss, scenes, grads, rng, per_array=60)


def test_projection_backward_alone_and_error_scale(orc):
    """The projection backward on its own (the chain from screen-space to
    parameter gradients) reproduces the parameter gradients of the full
    render backward from its screen-space gradients (the same chain; the
    full chain is pinned by the central differences above), and is linear
    in them.  The rounding-error scale that tolerances use bounds each
    entry's magnitude from above by at least its 16-fold (every term is
    counted with its pre-cancellation magnitude, times at least the pixel's
    blended pairs + 16) and is zero exactly where a Gaussian has no blended
    pair."""
    cam = synth.fd_camera()
    sc = synth.fd_scene(3).astype(np.float64)
    rng = np.random.default_rng(5)
    wc = rng.normal(size=(cam.height, cam.width, 3))
    wt = rng.normal(size=(cam.height, cam.width))
    wd = rng.normal(size=(cam.height, cam.width))
    rb = orc.render_backward(sc, cam, ST, wc, wt, wd)
    pb = orc.preprocess_backward(sc, cam, ST, rb["g2d"])
    for name in ("means", "log_scales", "quats", "opacity_logits", "sh"):
        np.testing.assert_allclose(pb[name], rb[name], rtol=1e-12, atol=1e-14 *
                                   max(1.0, np.abs(rb[name]).max()), err_msg=name)
    pb2 = orc.preprocess_backward(sc, cam, ST, 2.0 * rb["g2d"])
    np.testing.assert_allclose(pb2["means"], 2.0 * pb["means"], rtol=1e-12, atol=1e-14)
    sc_ = rb["g2d_scale"]
    assert np.all(sc_ >= 16.0 * np.abs(rb["g2d"]) * (1.0 - 1e-12))
    r = orc.render(sc, cam, ST)
    blended = np.zeros(sc.n, bool)
    pr = orc.preprocess(sc, cam, ST)
    blended[pr["valid"] == 1] = np.abs(rb["g2d"][pr["valid"] == 1]).max(1) > 0
    assert np.array_equal(sc_.max(1) > 0, blended)
    assert r["nblend"].sum() > 0


def test_repartition_redistribution_by_brute_force(orc):
    """The oracle's redistribution equals a row-by-row placement: every old
    row appended, in order, to the list of its new cell; rows are neither
    lost nor duplicated."""
    rng = np.random.default_rng(8)
    cells = [rng.normal(size=(n, 3)) for n in (5, 0, 9, 4)]
    cell_of = rng.integers(0, 3, size=18)
    got = orc.repartition(cells, cell_of, 3)
    lists = [[], [], []]
    g = 0
    for a in cells:
        for row in a:
            lists[cell_of[g]].append(row)
            g += 1
    for k in range(3):
        ref = np.array(lists[k]).reshape(-1, 3)
        assert np.array_equal(got[k], ref), k
    assert sum(len(x) for x in got) == 18


def test_imbalance_ratio_closed_form(orc):
    """N_max / mean(N) - 1: zero for equal counts; 3 of 4 Gaussians in one
    of two cells: 3 / 2 - 1 = 0.5."""
    assert orc.imbalance([0, 1, 0, 1], 2) == 0.0
    assert orc.imbalance([0, 0, 0, 1], 2) == 0.5
    assert abs(orc.imbalance([0] * 6 + [1] * 2 + [2] * 2, 3) - (6 / (10 / 3) - 1)) < 1e-15


# ------------------------------------------------------------- harness ----
def test_l1_and_adam_match_torch(orc):
    import torch
    rng = np.random.default_rng(4)
    x = rng.normal(size=(8, 6, 3))
    tgt = rng.normal(size=(8, 6, 3))
    tgt[0, 0, 0] = x[0, 0, 0]
    L, g = orc.l1_loss(x, tgt)
    xt = torch.tensor(x, requires_grad=True)
    lt = torch.nn.functional.l1_loss(xt, torch.tensor(tgt))
    lt.backward()
    assert abs(L - lt.item()) < 1e-14
    np.testing.assert_allclose(g, xt.grad.numpy(), atol=1e-17)
    p = rng.normal(size=50)
    pt = torch.tensor(p.copy(), requires_grad=True)
    opt = torch.optim.Adam([pt], lr=1e-2, betas=(0.9, 0.999), eps=1e-8)
    m = np.zeros(50)
    v = np.zeros(50)
    for step in range(1, 6):
        gr = rng.normal(size=50)
        pt.grad = torch.tensor(gr)
        opt.step()
        orc.adam_step(p, gr, m, v, step, 1e-2)
    np.testing.assert_allclose(p, pt.detach().numpy(), rtol=1e-12, atol=1e-14)
