"""Shared helpers for the GPU parity tests (kernel path vs FP64 oracle)."""
import math

import numpy as np
import pytest

import synth

INF = 1e30


def need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2606_18588_amd import binding
    binding.lib()


def big_box():
    return synth.Cell((-INF, -INF, -INF), (INF, INF, INF))


def rec_fields(rec):
    """Split the [n,12] float record into named numpy arrays."""
    r = rec.detach().cpu().numpy()
    return dict(mean2d_c=r[:, 0:2], conic=r[:, 2:5], opacity=r[:, 5], rgb=r[:, 6:9],
                depth=r[:, 9])


def jump_bound(settings, cmax):
    """Largest change a single pair crossing a threshold within rounding can
    make to a pixel: alpha_min * max|c - R| plus the termination bound."""
    return settings.alpha_min * 2.0 * cmax + settings.t_min * cmax + 1e-4


def compare_image(got, ref, flags, tol=1e-4, bound=None, max_flagged=None):
    """max-abs on unflagged pixels <= tol; flagged pixels within `bound`;
    with max_flagged, the fraction of flagged pixels at most that.
    Returns (max unflagged error, number flagged)."""
    err = np.abs(got - ref)
    if err.ndim == 3:
        err = err.max(-1)
    fl = flags != 0
    if max_flagged is not None:
        frac = float(fl.mean()) if fl.size else 0.0
        print(f"flagged {int(fl.sum())} of {fl.size} pixels ({frac:.2%}; bound "
              f"{max_flagged:.2%})", flush=True)
        assert frac <= max_flagged, f"flagged fraction {frac} > {max_flagged}"
    e_un = float(err[~fl].max()) if (~fl).any() else 0.0
    assert e_un <= tol, f"unflagged max-abs {e_un} > {tol}"
    if bound is not None and fl.any():
        e_fl = float(err[fl].max())
        assert e_fl <= bound, f"flagged max-abs {e_fl} > jump bound {bound}"
    return e_un, int(fl.sum())


def grid_cells_xy(xe, ye):
    return [synth.Cell((float(xe[i]), float(ye[j]), -INF), (float(xe[i + 1]), float(ye[j + 1]), INF))
            for j in range(len(ye) - 1) for i in range(len(xe) - 1)]


def grad_err(got, ref, floor=1e-3):
    """Per-element relative error |got - ref| / max(|ref|, floor * max|ref|):
    every element is held to its own magnitude, down to `floor` of the
    largest entry of its family (below that, rounding of the sums that form
    the entry dominates in either precision)."""
    got = np.asarray(got, np.float64)
    ref = np.asarray(ref, np.float64)
    if ref.size == 0:
        return 0.0
    scale = max(float(np.abs(ref).max()), 1e-30)
    return float((np.abs(got - ref) / np.maximum(np.abs(ref), floor * scale)).max())


def assert_same(got, ref, what):
    """Bit-exact comparison with a short message."""
    got = np.asarray(got)
    ref = np.asarray(ref)
    assert got.shape == ref.shape, f"{what}: shape {got.shape} != {ref.shape}"
    bad = np.nonzero(got != ref)
    if len(bad[0]):
        i = tuple(b[0] for b in bad)
        raise AssertionError(f"{what}: {len(bad[0])} mismatches, first at {i}: "
                             f"{got[i]} != {ref[i]}")


def assert_ranges(got, ref):
    """Tile ranges: non-empty ranges equal; empty ones have start == end."""
    got = np.asarray(got).astype(np.int64)
    ref = np.asarray(ref).astype(np.int64)
    ne = ref[:, 1] > ref[:, 0]
    assert_same(got[ne], ref[ne], "non-empty tile ranges")
    assert_same(got[~ne, 0], got[~ne, 1], "empty tile ranges")


def expand_lists(keys, vals, ranges):
    """The kernel's sort output as full per-tile lists: every tile's own
    list merged by (depth bits, index) with the screen list (the range at
    index `tiles`).  Returns (keys, vals, ranges) in the layout of the
    oracle's sorted instance list."""
    keys = np.asarray(keys).astype(np.uint64)
    vals = np.asarray(vals).astype(np.uint64)
    ranges = np.asarray(ranges).astype(np.int64)
    tiles = len(ranges) - 1
    s0, s1 = ranges[tiles]
    sd, sv = keys[s0:s1] & np.uint64(0xFFFFFFFF), vals[s0:s1]
    ok, ov, orng = [], [], np.zeros((tiles, 2), np.int64)
    pos = 0
    for t in range(tiles):
        a, b = ranges[t]
        d = np.concatenate([sd, keys[a:b] & np.uint64(0xFFFFFFFF)])
        v = np.concatenate([sv, vals[a:b]])
        order = np.lexsort((v, d))
        ok.append((np.uint64(t) << np.uint64(32)) | d[order])
        ov.append(v[order])
        orng[t] = (pos, pos + len(d))
        pos += len(d)
    cat = lambda xs: np.concatenate(xs) if xs else np.zeros(0, np.uint64)
    return cat(ok), cat(ov).astype(np.uint32), orng


U32 = 2.0 ** -24  # unit roundoff of FP32


def check_grad_scaled(got, ref, scale, what, tol=1e-3, kappa=1.0):
    """Per element |got - ref| <= tol |ref| + kappa u32 scale, with `scale`
    the oracle's rounding-error scale of each entry (the magnitudes of the
    terms before they cancel, times the blended pairs a term's walk spans
    plus 16).  Prints the smallest kappa that would pass."""
    got = np.asarray(got, np.float64)
    ref = np.asarray(ref, np.float64)
    scale = np.asarray(scale, np.float64)
    excess = np.maximum(np.abs(got - ref) - tol * np.abs(ref), 0.0)
    need = float((excess / np.maximum(U32 * scale, 1e-300)).max()) if ref.size else 0.0
    bad = excess > kappa * U32 * scale
    w = int((excess / np.maximum(U32 * scale, 1e-300)).argmax()) if ref.size else 0
    print(f"grad {what}: kappa needed {need:.3g} (bound {kappa:g}); {int(bad.sum())} of "
          f"{ref.size} entries outside" + (f"; worst got {got.flat[w]:.6g} ref {ref.flat[w]:.6g} "
                                           f"scale*u {U32 * scale.flat[w]:.3g}" if ref.size else ""),
          flush=True)
    assert not bad.any(), (what, need)
    return need


PARAM_NAMES = ("means", "log_scales", "quats", "opacity_logits", "sh")


def param_scales(scene, cam, settings, g2d_scale, vis):
    """FP32 error scale of each raw-parameter gradient of the visible
    Gaussians (rows of `vis`), propagated from the screen-space scale.  The
    projection backward is linear in g2d: column c moves the parameter
    gradients by J_c g2d[c], so an error within u g2d_scale[c] in every
    column moves them by at most u sum_c |J_c| g2d_scale[c].  Each column's
    chain |J_c| g2d_scale[c] is the oracle's projection backward of that
    column alone (one Gaussian's chain does not involve another's)."""
    import oracle
    idx = np.nonzero(vis)[0]
    sub = scene.subset(idx)
    out = {}
    for c in range(10):
        g = np.zeros((idx.size, 10))
        g[:, c] = np.asarray(g2d_scale, np.float64)[idx, c]
        pb = oracle.preprocess_backward(sub, cam, settings, g)
        for name in PARAM_NAMES:
            out[name] = out.get(name, 0.0) + np.abs(pb[name])
    return out


def check_grad(got, ref, what, tol=1e-3, floor=1e-3):
    """Assert grad_err(got, ref, floor) <= tol; prints the error, the worst
    element's magnitude relative to the family's largest and how many
    elements exceed 1e-3 relative."""
    e = grad_err(got, ref, floor)
    g = np.asarray(got, np.float64).reshape(-1)
    r = np.asarray(ref, np.float64).reshape(-1)
    if r.size:
        scale = max(float(np.abs(r).max()), 1e-30)
        rel = np.abs(g - r) / np.maximum(np.abs(r), floor * scale)
        w = int(rel.argmax())
        print(f"grad {what}: per-element rel {e:.3g} (floor {floor:g} of max); worst at "
              f"|ref|/max {abs(r[w]) / scale:.3g}, abs err/max {abs(g[w] - r[w]) / scale:.3g}; "
              f"{int((rel > 1e-3).sum())} of {r.size} above 1e-3", flush=True)
    assert e <= tol, (what, e)
    return e
