"""Helpers of the GPU parity tests: run the HIP path through the C ABI and
compare it with the FP64 oracle on the same seeded scene."""
import numpy as np
import pytest

# parity bar (forward): features of unit-variance inputs and alpha
TOL_FEAT = 2e-4
TOL_ALPHA = 1e-5


def torch_cuda():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def gpu_render(scene, rast=None, bg=None, lists=True):
    """Render `scene` on cuda:0; returns numpy arrays and the rasterizer."""
    torch = torch_cuda()
    from paper_2405_14866_amd.rasterize import GaussianSoA, Rasterizer
    print(f"[gpu] render {scene.name} n={scene.n} c={scene.c} "
          f"{scene.cam.width}x{scene.cam.height}", flush=True)
    g = GaussianSoA.from_scene(scene)
    if rast is None:
        rast = Rasterizer(0, max_n=max(1, scene.n), max_w=scene.cam.width, max_h=scene.cam.height)
    bgt = None if bg is None else torch.as_tensor(bg, dtype=torch.float32, device="cuda")
    feat, alpha = rast.forward(g, scene.cam, bgt)
    T, last = rast.pixel_state(scene.cam)
    out = dict(feat=feat.cpu().numpy(), alpha=alpha.cpu().numpy(), T=T.cpu().numpy(),
               last=last.cpu().numpy(), n_keys=rast.n_keys)
    if lists:
        ts, so = rast.tile_lists(scene.cam)
        out["tile_start"] = ts.cpu().numpy().astype(np.int64)
        out["sorted"] = so.cpu().numpy()
    torch.cuda.synchronize()
    return out, rast, g


def compare_lists(gpu, ora):
    start, lst = ora.tile_lists()
    np.testing.assert_array_equal(gpu["tile_start"], start)
    np.testing.assert_array_equal(gpu["sorted"], lst)


def compare_forward(gpu, ora, ref=None, bg=None, tol_feat=TOL_FEAT, tol_alpha=TOL_ALPHA,
                    check_last=True):
    """Element-wise forward parity.  Pixels with a near-threshold decision
    (flagged by the oracle) must match one of the oracle's branch variants.
    Returns a small report dict."""
    ref = ora.render(bg=bg) if ref is None else ref
    F, A = gpu["feat"].astype(np.float64), gpu["alpha"].astype(np.float64)
    dF = np.abs(F - ref["feat"]).max(0)
    dA = np.abs(A - ref["alpha"])
    flagged = ref["nflags"] > 0
    ok = (dF <= tol_feat) & (dA <= tol_alpha)
    bad = ~ok & ~flagged
    assert not bad.any(), (
        f"{bad.sum()} unflagged pixels off: max dF {dF[~flagged].max():.3g} "
        f"max dA {dA[~flagged].max():.3g} at {np.argwhere(bad)[:5].tolist()}")
    # last contributor is an index: exact where no decision was near a threshold
    if check_last:
        np.testing.assert_array_equal(gpu["last"][~flagged], ref["last"][~flagged])
    excluded = 0
    for (y, x) in np.argwhere(flagged & ~ok):
        var = ora.pixel_variants(int(x), int(y), bg=bg)
        if var is None:
            excluded += 1
            continue
        want = np.concatenate([F[:, y, x], [A[y, x]]])
        d = np.abs(var - want[None])
        hit = (d[:, :-1].max(1) <= tol_feat) & (d[:, -1] <= tol_alpha)
        assert hit.any(), f"flagged pixel {(x, y)} matches no branch variant: {d.max(1)}"
    assert excluded <= max(2, flagged.size // 100000), excluded
    return dict(max_dF=float(dF[~flagged].max()) if (~flagged).any() else 0.0,
                max_dA=float(dA[~flagged].max()) if (~flagged).any() else 0.0,
                flagged=int(flagged.sum()), excluded=excluded)


# ---------------------------------------------------------------- gradients
GROUPS = ("mean", "log_scale", "quat", "opacity_logit", "feat")


def walked_by(ora, pixels):
    """Gaussians that the walks of `pixels` ((y, x) pairs) evaluate."""
    out = set()
    for (y, x) in pixels:
        out.update(ora.pixel_walk(int(x), int(y)).tolist())
    return np.array(sorted(out), dtype=np.int64)


def gpu_branches(gpu, ora, ref, bg=None, tol_feat=TOL_FEAT, t_rel=1e-3, t_abs=2.0 ** -23):
    """The branch the GPU took at each pixel with near-threshold decisions:
    the oracle variant whose features match the GPU's to tol_feat and whose
    final transmittance matches to t_rel (relative) + t_abs.  Inverting a
    decision multiplies T by (1 - alpha) with alpha >= 1/255 or divides it
    by that, so variants are at least 0.39 % apart in T; two variants that
    still both match (or a pixel with more than two flags) leave the branch
    undetermined.  gpu: dict with feat [C, H, W] and T [H, W].  Returns
    (mask [H, W] uint8 for Oracle.backward, undetermined (y, x) pixels)."""
    mask = np.zeros(ref["nflags"].shape, np.uint8)
    undetermined = []
    F = np.asarray(gpu["feat"], np.float64)
    T = np.asarray(gpu["T"], np.float64)
    for (y, x) in np.argwhere(ref["nflags"] > 0):
        var = ora.pixel_variants(int(x), int(y), bg=bg)
        if var is None:
            undetermined.append((y, x))
            continue
        tv = 1.0 - var[:, -1]
        ok = (np.abs(var[:, :-1] - F[:, y, x][None]).max(1) <= tol_feat) & \
             (np.abs(tv - T[y, x]) <= t_rel * tv + t_abs)
        hit = np.flatnonzero(ok)
        if len(hit) == 1:
            mask[y, x] = hit[0]
        else:
            undetermined.append((y, x))
    return mask, undetermined


def compare_backward(got, gpu, ora, d_feat, d_alpha=None, bg=None, ref_fwd=None, rel=1e-4):
    """Gradient parity against the oracle's FP64 backward taken under the
    branch the GPU took at every near-threshold decision (gpu_branches).
    Gaussians walked by a pixel whose branch is undetermined are held to the
    loose bar only.  Returns (worst normalised error per group, number of
    undetermined pixels, number of Gaussians on the loose bar)."""
    bg64 = None if bg is None else np.asarray(bg, np.float64)
    ref_fwd = ora.render(bg=bg64) if ref_fwd is None else ref_fwd
    mask, undet = gpu_branches(gpu, ora, ref_fwd, bg=bg64)
    ref = ora.backward(np.asarray(d_feat, np.float64),
                       None if d_alpha is None else np.asarray(d_alpha, np.float64),
                       bg=bg64, flip_mask=mask)
    loose = walked_by(ora, undet)
    worst = compare_grads(got, ref, loose, rel=rel)
    compare_grads_loose(got, ref, loose)
    return worst, len(undet), len(loose)


def _per_gaussian(k, arr):
    """A gradient group as [n, m], one row per Gaussian ([3, n] / [4, n] have
    the Gaussian index last, [n] and [n, c] first)."""
    a = np.asarray(arr, np.float64)
    if a.ndim == 1:
        return a[:, None]
    return a.T if k != "feat" else a


def _errors(a, b, rms):
    """|g - g*| / (max_j |g*_j| + rms), the maximum taken over the
    components j of the same Gaussian's group: a normwise relative error per
    Gaussian.  Every component of a group is one linear map of the same
    FP32-accumulated screen-space gradients, so a component that is small by
    cancellation carries the absolute rounding of the whole vector."""
    scale = np.abs(b).max(axis=1, keepdims=True)
    return np.abs(a - b) / (scale + rms)


def _rms_floor(ref):
    return 1e-9 * max(np.sqrt(np.mean(np.asarray(ref[k], np.float64) ** 2)) for k in GROUPS)


def compare_grads(gpu, ref, skip, rel=1e-4):
    """|g - g*| <= rel (max |g*| over the Gaussian's group + rms(g*)) per
    parameter group, Gaussians in `skip` excluded.  A group whose true
    gradient vanishes identically (the quaternion of an isotropic Gaussian:
    Sigma3D = s^2 I does not depend on the rotation) has only rounding noise
    on both sides, so its rms is floored at 1e-9 of the largest group rms.
    Returns the worst normalised error per group."""
    worst = {}
    floor = _rms_floor(ref)
    for k in GROUPS:
        a = _per_gaussian(k, gpu[k]).copy()
        b = _per_gaussian(k, ref[k]).copy()
        a[skip] = b[skip] = 0
        rms = max(np.sqrt(np.mean(b ** 2)), floor) + 1e-30
        err = _errors(a, b, rms)
        worst[k] = float(err.max())
        assert worst[k] <= rel, (k, worst[k], np.unravel_index(err.argmax(), err.shape))
    return worst


def compare_grads_loose(gpu, ref, only, rel=2e-2):
    """The Gaussians a near-threshold pixel walks over, against a looser bar:
    a decision that flips at alpha = 1/255 or T = 1e-4 changes that pixel's
    transmittance by well under 1 %, and the Gaussian's gradient sums many
    pixels."""
    floor = _rms_floor(ref)
    for k in GROUPS:
        # same rms and floor as compare_grads
        rms = max(np.sqrt(np.mean(np.asarray(ref[k], np.float64) ** 2)), floor) + 1e-30
        a = _per_gaussian(k, gpu[k])[only]
        b = _per_gaussian(k, ref[k])[only]
        err = _errors(a, b, rms)
        assert err.size == 0 or err.max() <= rel, (k, float(err.max()))
